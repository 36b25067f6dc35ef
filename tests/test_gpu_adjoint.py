"""The hand-written adjoint (vbqmc_param_grad) against the oracle's
forward-mode dual numbers, against central finite differences of the GPU
evaluation (h = 1e-5), against the Euler identities of the structure
coefficients, and through the torch.autograd.Function wrapper."""

import json

import numpy as np
import pytest

import systems as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2207_14715_amd as vb
    vb.load_library()
    return vb


def _scaled_err(gpu, ref):
    scale = np.maximum(1.0, np.abs(ref).max(axis=1, keepdims=True))
    return np.max(np.abs(gpu - ref) / scale)


def _compare(lib, oracle_mod, sysd, W, idx=None, tol=1e-8, seed=3):
    import torch
    o = oracle_mod.Oracle(sysd)
    R = S.initial_walkers(sysd, W, seed=seed)
    ctx = lib.Context(sysd)
    print(f"[adjoint] {sysd['name']} W={W} n_params={ctx.n_params} lds={ctx.info['lds_bytes']}", flush=True)
    dl, de = ctx.param_grad(torch.from_numpy(R).cuda())
    dl, de = dl.cpu().numpy(), de.cpu().numpy()
    assert dl.shape == (W, o.n_params)
    if idx is None:
        idx = np.arange(o.n_params)
    rl, re = o.param_deriv(R, idx)
    el = _scaled_err(dl[:, idx], rl)
    ee = _scaled_err(de[:, idx], re)
    assert el < tol, f"d lnPsi/dp scaled error {el:.2e}"
    assert ee < tol, f"d E_L/dp scaled error {ee:.2e}"
    return ctx, o, R, dl, de


@pytest.mark.parametrize("seed,npairs,nunp", [(401, 1, 0), (402, 2, 1), (403, 1, 2)])
def test_small_systems_all_parameters(lib, oracle_mod, seed, npairs, nunp):
    sysd = S.small_random_system(seed, n_inactive=2, n_active=5, n_pairs=npairs, n_unpaired=nunp,
                                 n_structures=4, kappa=0.8, poly=True)
    _compare(lib, oracle_mod, sysd, 6)


def test_h2_all_parameters(lib, oracle_mod):
    _compare(lib, oracle_mod, S.h2_heitler_london(), 8)


def test_slater_d_shells_all_parameters(lib, oracle_mod):
    # Slater s, p, d shells on the second F2 atom (the five basis channels of
    # a Slater d function feed both orbital-coefficient contractions)
    sysd = S.f2_shaped()
    rng = np.random.default_rng(78)
    shells = []
    for sh in sysd["shells"]:
        sh = dict(sh)
        if sh["center"] == 1:
            n = len(sh["exps"])
            sh["kind"] = "sto"
            sh["exps"] = sorted(rng.uniform(0.6, 4.0, size=n).tolist(), reverse=True)
            sh["coefs"] = rng.uniform(0.2, 1.0, size=n).tolist()
        shells.append(sh)
    _compare(lib, oracle_mod, dict(sysd, shells=shells, name="f2_slater_spd"), 4)


def test_f2_bovb_all_parameters(lib, oracle_mod):
    # the breathing orbitals' coefficients are parameters of their own
    _compare(lib, oracle_mod, S.f2_bovb(), 4)


def test_adjoint_molecule_sampled_parameters(lib, oracle_mod):
    sysd = S.adjoint_molecule()
    o = oracle_mod.Oracle(sysd)
    cs, ls, js = o.param_slices()
    rng = np.random.default_rng(0)
    lam_nz = np.flatnonzero(np.asarray(sysd["lam"]).reshape(-1) != 0) + ls.start
    lam_z = np.flatnonzero(np.asarray(sysd["lam"]).reshape(-1) == 0) + ls.start
    idx = np.concatenate([np.arange(cs.start, cs.stop), rng.choice(lam_nz, 60, replace=False),
                          rng.choice(lam_z, 20, replace=False), np.arange(js.start, js.stop)])
    ctx, o, R, dl, de = _compare(lib, oracle_mod, sysd, 2, idx)
    # Euler identities in the structure coefficients
    c = o.c
    np.testing.assert_allclose(dl[:, cs] @ c, 1.0, rtol=1e-10)
    assert np.all(np.abs(de[:, cs] @ c) <= 1e-8 * np.abs(de[:, cs]).max())


def test_adjoint_matches_gpu_central_differences(lib, oracle_mod):
    """Central differences (h = 1e-5, fourth-order five-point stencil, so the
    truncation error stays below 1e-6 relative even where E_L is steep) of the
    GPU evaluation, parameters set through vbqmc_set_params; 1e-6 relative
    with a floor of 1e-3 max|g|."""
    import torch
    sysd = S.small_random_system(411, n_inactive=2, n_active=5, n_pairs=2, n_unpaired=0, n_structures=4)
    ctx = lib.Context(sysd)
    R = torch.from_numpy(S.initial_walkers(sysd, 4, seed=2)).cuda()
    dl, de = ctx.param_grad(R)
    dl, de = dl.cpu().numpy(), de.cpu().numpy()
    p0 = ctx.get_params()
    h = 1e-5
    rng = np.random.default_rng(1)
    for j in rng.choice(ctx.n_params, 40, replace=False):
        out = []
        for k in (2, 1, -1, -2):
            p = p0.copy()
            p[j] += k * h
            ctx.set_params(p)
            ev = ctx.evaluate(R, want=("eloc",))
            out.append((ev["logabs"].cpu().numpy(), ev["eloc"].cpu().numpy()))
        fl = (-out[0][0] + 8 * out[1][0] - 8 * out[2][0] + out[3][0]) / (12 * h)
        fe = (-out[0][1] + 8 * out[1][1] - 8 * out[2][1] + out[3][1]) / (12 * h)
        for g, f, full in ((dl[:, j], fl, dl), (de[:, j], fe, de)):
            floor = 1e-3 * np.abs(full).max(axis=1)
            assert np.all(np.abs(g - f) <= 1e-6 * np.maximum(np.abs(f), floor) + 1e-9), (j, g, f)
    ctx.set_params(p0)


def test_autograd_function_contracts_upstream_gradients(lib, oracle_mod):
    import torch
    sysd = S.small_random_system(421, n_inactive=1, n_active=4, n_pairs=1, n_unpaired=1, n_structures=3)
    ctx = lib.Context(sysd)
    W = 16
    R = torch.from_numpy(S.initial_walkers(sysd, W, seed=4)).cuda()
    p = torch.tensor(ctx.get_params(), dtype=torch.float64, requires_grad=True)
    lp, el = lib.jvb_apply(p, R, ctx)
    a = torch.linspace(0.5, 1.5, W, dtype=torch.float64, device="cuda")
    b = torch.linspace(-1.0, 1.0, W, dtype=torch.float64, device="cuda")
    loss = (a * lp).sum() + (b * el).sum()
    (gp,) = torch.autograd.grad(loss, p)
    dl, de = ctx.param_grad(R)
    ref = (a[:, None] * dl + b[:, None] * de).sum(0).cpu()
    np.testing.assert_allclose(gp.numpy(), ref.numpy(), rtol=1e-12, atol=1e-12)


def test_autograd_backward_uses_its_own_parameters(lib, oracle_mod):
    # two graphs at different parameter points: the backward of the first,
    # run after the second forward, must give the gradient at the first
    # point, and leave the context at the parameters it held
    import torch
    sysd = S.small_random_system(421, n_inactive=1, n_active=4, n_pairs=1, n_unpaired=1, n_structures=3)
    ctx = lib.Context(sysd)
    W = 16
    R = torch.from_numpy(S.initial_walkers(sysd, W, seed=4)).cuda()
    p0 = ctx.get_params()
    p2v = p0.copy()
    p2v[: ctx.n_struct] *= np.linspace(0.7, 1.3, ctx.n_struct)
    p2v[ctx.n_struct:ctx.n_struct + 20] += 0.05
    p1 = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    p2 = torch.tensor(p2v, dtype=torch.float64, requires_grad=True)
    lp1, el1 = lib.jvb_apply(p1, R, ctx)
    lp2, el2 = lib.jvb_apply(p2, R, ctx)
    (g1,) = torch.autograd.grad(lp1.sum() + el1.sum(), p1)
    np.testing.assert_array_equal(ctx.get_params(), p2v)
    ctx.set_params(p0)
    dl, de = ctx.param_grad(R)
    ref = (dl + de).sum(0).cpu()
    np.testing.assert_allclose(g1.numpy(), ref.numpy(), rtol=1e-12, atol=1e-12)
    ctx.set_params(p2v)
    dl2, de2 = ctx.param_grad(R)
    assert not np.allclose((dl2 + de2).sum(0).cpu().numpy(), ref.numpy(), rtol=1e-6)
