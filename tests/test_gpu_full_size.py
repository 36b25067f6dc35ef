"""Parity at the workloads' full sizes, in the launch configurations that
bench.py times: the oracle cannot follow 32768 walkers, so these tests check
sampled outputs one by one (each sampled walker's E_L against the oracle's at
the walker's final configuration, its parameter derivatives against the
oracle's dual numbers) and properties that hold at any size (population band,
finite records, acceptance counts within the move count).

E_L is compared at 1e-10 scaled by |T_L| + |V| for configurations with
kappa_ref <= 1e3 in both spins and kappa_D <= 1e4, and within
1e-10 + 1e-13 kappa_ref kappa_D otherwise (the conditioning bound of the
reference-determinant scheme)."""

import numpy as np
import pytest

import systems as S
from tests.test_gpu_walks import _eloc_scale, _kappa_ref

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2207_14715_amd as vb
    vb.load_library()
    return vb


def _sample(W, k=16, seed=0):
    """k walker indices spread over [0, W), the first and the last included
    (the last sits in a partly filled workgroup when W is not a multiple of 4)."""
    rng = np.random.default_rng(seed)
    idx = np.unique(np.concatenate([[0, W - 1], rng.choice(W, k - 2, replace=False)]))
    return idx


def _check_eloc(oracle_mod, sysd, R, e_gpu, label):
    o = oracle_mod.Oracle(sysd)
    ref = o.evaluate(R)
    ku, kdn, kd = _kappa_ref(o, sysd, R)
    kr = np.maximum(ku, kdn)
    err = np.abs(e_gpu - ref["eloc"]) / _eloc_scale(ref)
    well = (kr <= 1e3) & (kd <= 1e4)
    print(f"[{label}] {len(R)} sampled walkers, {int((~well).sum())} poorly conditioned, worst scaled E_L error "
          f"{err.max():.2e}", flush=True)
    if well.any():
        assert err[well].max() <= 1e-10, float(err[well].max())
    assert np.all(err <= 1e-10 + 1e-13 * kr * kd), float((err / (1e-10 + 1e-13 * kr * kd)).max())


def test_dmc_64_electrons_32768_walkers(lib, oracle_mod):
    """The headline configuration: 32768 target walkers, capacity 3x, the
    walker-resident kernel, walkers from the 3-step FP64 VMC burn-in; two DMC
    steps, then 16 surviving walkers' record E_L against the oracle."""
    import torch
    sysd = S.dmc_molecule()
    W = 32768
    ctx = lib.Context(sysd)
    assert ctx.info["dmc_kernel"] == 3
    st = [ctx.new_state(3 * W), ctx.new_state(3 * W)]
    print(f"[full dmc] {sysd['name']} W={W}", flush=True)
    ctx.walkers_init(torch.from_numpy(S.initial_walkers(sysd, W, seed=13)).cuda(), st[0])
    ctx.vmc_advance(st[0], 3, 17, 0, 0.3, False, None, W)
    et = float(ctx.record_eloc(st[0], W).median().item())
    out = ctx.dmc_advance(st, W, 2, 2022, 0, 0.005, et, W)
    Wn = out["W"]
    pop = out["pop"].cpu().numpy()
    assert np.all(np.abs(pop / W - 1.0) <= 0.10), pop
    assert abs(Wn / W - 1.0) <= 0.10
    acc, prop = out["n_accept"].cpu().numpy(), out["n_prop"].cpu().numpy()
    assert np.all(acc <= prop) and np.all(acc > 0.5 * prop)
    R = ctx.positions(st[0], Wn).cpu().numpy()
    e = ctx.record_eloc(st[0], Wn).cpu().numpy()
    torch.cuda.synchronize()
    assert np.all(np.isfinite(R))
    idx = _sample(Wn)
    _check_eloc(oracle_mod, sysd, R[idx], e[idx], "full dmc")


def test_vmc_40_electrons_16384_walkers(lib, oracle_mod):
    """The 40-electron VMC line: 16384 walkers on the walker-resident kernel,
    one call of 3 steps; sampled walkers' last E_L against the oracle."""
    import torch
    sysd = S.precision_molecule()
    W = 16384
    ctx = lib.Context(sysd)
    assert ctx.info["step_kernel"] == 3
    print(f"[full vmc] {sysd['name']} W={W}", flush=True)
    st = ctx.walkers_init(torch.from_numpy(S.initial_walkers(sysd, W, seed=5)).cuda())
    acc = ctx.vmc_advance(st, 3, 20220728, 0, 0.3)
    R = ctx.positions(st).cpu().numpy()
    e = acc["e_last"].cpu().numpy()
    na = acc["n_accept"].cpu().numpy()
    torch.cuda.synchronize()
    assert np.all(na <= 3 * ctx.N) and na.mean() > 0.3 * 3 * ctx.N
    idx = _sample(W)
    _check_eloc(oracle_mod, sysd, R[idx], e[idx], "full vmc 40e")


def test_vmc_f2_4096_walkers_row_kernel(lib, oracle_mod):
    """The F2 VMC line: 4096 walkers, one row-kernel launch of 100 steps;
    sampled walkers' last E_L against the oracle."""
    import torch
    sysd = S.f2_shaped()
    W = 4096
    ctx = lib.Context(sysd)
    assert ctx.info["step_kernel"] == 2
    print(f"[full vmc] {sysd['name']} W={W}", flush=True)
    st = ctx.walkers_init(torch.from_numpy(S.initial_walkers(sysd, W, seed=5)).cuda())
    acc = ctx.vmc_advance(st, 100, 20220728, 0, 0.3)
    R = ctx.positions(st).cpu().numpy()
    e = acc["e_last"].cpu().numpy()
    torch.cuda.synchronize()
    idx = _sample(W)
    _check_eloc(oracle_mod, sysd, R[idx], e[idx], "full vmc f2")


def test_adjoint_30_electrons_8192_walkers(lib, oracle_mod):
    """The adjoint line: 8192 walkers in one call; four sampled walkers'
    derivatives of 60 sampled parameters (structure, orbital and Jastrow
    ones) against the oracle's dual numbers."""
    import torch
    sysd = S.adjoint_molecule()
    W = 8192
    ctx = lib.Context(sysd)
    R = S.initial_walkers(sysd, W, seed=3)
    print(f"[full adjoint] {sysd['name']} W={W} P={ctx.n_params}", flush=True)
    dl, de = ctx.param_grad(torch.from_numpy(R).cuda())
    dl, de = dl.cpu().numpy(), de.cpu().numpy()
    torch.cuda.synchronize()
    o = oracle_mod.Oracle(sysd)
    cs, ls, js = o.param_slices()
    rng = np.random.default_rng(4)
    lam_nz = np.flatnonzero(np.asarray(sysd["lam"]).reshape(-1) != 0) + ls.start
    pidx = np.concatenate([np.arange(cs.start, cs.stop), rng.choice(lam_nz, 30, replace=False),
                           rng.choice(np.arange(js.start, js.stop), 18, replace=False)])
    widx = np.array([0, 1777, 5000, W - 1])
    rl, re = o.param_deriv(R[widx], pidx)
    for name, gpu, ref in (("d lnPsi/dp", dl[np.ix_(widx, pidx)], rl), ("d E_L/dp", de[np.ix_(widx, pidx)], re)):
        err = np.max(np.abs(gpu - ref) / np.maximum(1.0, np.abs(ref).max(axis=1, keepdims=True)))
        assert err < 1e-8, f"{name}: scaled error {err:.2e}"
