"""Pseudopotential term of E_L (Sec. 2.1, basis choice: valence calculations
with energy-consistent pseudopotentials; the semilocal form) through the C
ABI on the GPU against the oracle (oracle/ecp.py, which re-evaluates every
moved configuration from scratch): vbqmc_evaluate on one-electron s, p and d
systems (closed-form pinned in the oracle's tests) and on the F2 valence
system; VMC walks (single-electron and all-electron moves) step by step,
positions and acceptances draw for draw and E_L of every step; a DMC
trajectory with the term in E_L (locality approximation) against the C++
oracle's (native_ecp); the entry points that do not take pseudopotentials
refuse them."""

import numpy as np
import pytest

import systems as S
from oracle import ecp as ECP

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2207_14715_amd as vb
    vb.load_library()
    return vb


def _scale(ev):
    return np.maximum(1.0, np.abs(ev["kin"]) + np.abs(ev["eloc"] - ev["kin"]))


def _walkers(sysd, W, seed):
    """Start positions with electrons inside and outside r_cut of the centres."""
    return S.initial_walkers(sysd, W, seed=seed, sigma=1.2)


@pytest.mark.parametrize("l,lam", [(0, [1.0]), (1, [0.3, -0.5, 0.8]), (2, [0.2, -0.7, 0.4, 0.5, -0.3])])
def test_evaluate_one_electron(lib, oracle_mod, l, lam):
    import torch
    sysd = S.ecp_one_centre(l, lam, 0.7)
    o = oracle_mod.Oracle(sysd)
    R = _walkers(sysd, 64, 20 + l) * 1.5
    print(f"[ecp evaluate] one electron l={l} W={len(R)}", flush=True)
    ctx = lib.Context(sysd)
    out = ctx.evaluate(torch.from_numpy(R).cuda(), want=("eloc",))
    el = out["eloc"].cpu().numpy()
    torch.cuda.synchronize()
    ref = ECP.evaluate(o, sysd, R)
    err = np.abs(el - ref["eloc"]) / _scale(ref)
    assert err.max() < 1e-10, err.max()


def test_evaluate_f2_valence(lib, oracle_mod):
    import torch
    sysd = S.f2_valence_ecp()
    o = oracle_mod.Oracle(sysd)
    R = _walkers(sysd, 12, 31)
    print(f"[ecp evaluate] f2 valence W={len(R)}", flush=True)
    ctx = lib.Context(sysd)
    out = ctx.evaluate(torch.from_numpy(R).cuda())
    el = out["eloc"].cpu().numpy()
    la = out["logabs"].cpu().numpy()
    torch.cuda.synchronize()
    ref = ECP.evaluate(o, sysd, R)
    np.testing.assert_allclose(la, ref["logabs"], rtol=0, atol=1e-10 * np.abs(ref["logabs"]).max())
    part = ECP.ecp_energy(o, sysd, R)
    assert np.all(np.abs(part) > 1e-3)  # the term is really there
    err = np.abs(el - ref["eloc"]) / _scale(ref)
    assert err.max() < 1e-10, err.max()
    # removing the pseudopotentials gives back the plain E_L with the valence charges
    ctx.set_ecp(None)
    el0 = ctx.evaluate(torch.from_numpy(R).cuda(), want=("eloc",))["eloc"].cpu().numpy()
    torch.cuda.synchronize()
    base = o.evaluate(R)
    assert np.max(np.abs(el0 - base["eloc"]) / _scale(base)) < 1e-10


@pytest.mark.parametrize("all_electron,steps", [(False, 3), (True, 2)])
def test_vmc_walk_step_by_step(lib, oracle_mod, all_electron, steps):
    import torch
    sysd = S.f2_valence_ecp()
    o = oracle_mod.Oracle(sysd)
    W, seed, step0, step_size = 6, 77, 5, 0.4
    R = _walkers(sysd, W, 41)
    ctx = lib.Context(sysd)
    print(f"[ecp vmc] f2 valence W={W} all_electron={all_electron} steps={steps} "
          f"step_kernel={ctx.info['step_kernel']}", flush=True)
    state = ctx.walkers_init(torch.from_numpy(R).cuda())
    acc = ctx.new_vmc_acc(W)
    e_sum = np.zeros(W)
    n_acc = np.zeros(W)
    for k in range(steps):
        ref = o.vmc(R, 1, seed, step0 + k, step_size, all_electron)
        ctx.vmc_advance(state, 1, seed, step0 + k, step_size, all_electron, acc=acc)
        Rg = ctx.positions(state).cpu().numpy()
        el = acc["e_last"].cpu().numpy()
        na = acc["n_accept"].cpu().numpy()
        torch.cuda.synchronize()
        R = ref["R"]
        n_acc += ref["n_acc"]
        assert np.all(np.abs(Rg - R) <= 1e-9 * (1 + np.abs(R))), f"step {k}: walkers diverged"
        np.testing.assert_array_equal(na, n_acc)
        fin = ECP.evaluate(o, sysd, R)
        worst = np.max(np.abs(el - fin["eloc"]) / _scale(fin))
        assert worst < 1e-10, f"step {k}: e_last scaled error {worst:.2e}"
        e_sum += fin["eloc"]
    es = acc["e_sum"].cpu().numpy()
    torch.cuda.synchronize()
    assert np.max(np.abs(es - e_sum) / np.maximum(1.0, np.abs(e_sum))) < 1e-10


def test_entry_points_without_pseudopotentials_refuse(lib):
    import torch
    sysd = S.f2_valence_ecp()
    ctx = lib.Context(sysd)
    R = torch.from_numpy(_walkers(sysd, 4, 3)).cuda()
    state = ctx.walkers_init(R)
    with pytest.raises(lib.VBQMCError):
        ctx.vmc_sweep(state, 1, 0, 0.3, torch.zeros(4, dtype=torch.float64, device="cuda"))
    with pytest.raises(lib.VBQMCError):
        ctx.param_grad(R)
    bad = [dict(sysd["ecp"][0], center=5)]
    with pytest.raises(lib.VBQMCError):
        ctx.set_ecp(bad)
    bad = [dict(sysd["ecp"][0], local=[[1.0, 2.5, 1.0]])]
    with pytest.raises(lib.VBQMCError):
        ctx.set_ecp(bad)
    with pytest.raises(lib.VBQMCError):
        ctx.set_ecp([sysd["ecp"][0], sysd["ecp"][0]])
    with pytest.raises(lib.VBQMCError):
        lib.Context(sysd, precision="fp32")
    torch.cuda.synchronize()


def test_dmc_trajectory_with_pseudopotentials(lib, oracle_mod):
    """Fixed-node DMC on the F2 valence system: E_L with the projected term
    drives the weights (the locality approximation).  Populations, weights,
    acceptances, positions and every surviving walker's E_L against the C++
    oracle with the same term."""
    import torch
    from tests.test_gpu_walks import _check_dmc
    sysd = S.f2_valence_ecp()
    o = oracle_mod.Oracle(sysd, native_ecp=True)
    W, steps, tau, seed, step0 = 8, 3, 0.01, 77, 3
    R0 = _walkers(sysd, W, 8)
    e0 = o.evaluate(R0)["eloc"]
    et = float(np.mean(e0))
    ref = o.dmc(R0, e0, steps, seed, step0, tau, et, W, capacity=4 * W)
    ctx = lib.Context(sysd)
    print(f"[ecp dmc] f2 valence W={W} steps={steps}", flush=True)
    st0 = ctx.new_state(4 * W)
    st1 = ctx.new_state(4 * W)
    ctx.walkers_init(torch.from_numpy(R0).cuda(), st0)
    out = ctx.dmc_advance([st0, st1], W, steps, seed, step0, tau, et, W)
    R = ctx.positions(st0, out["W"]).cpu().numpy()
    e_rec = ctx.record_eloc(st0, out["W"]).cpu().numpy()
    torch.cuda.synchronize()
    _check_dmc(ref, out, R, e_rec, o)
