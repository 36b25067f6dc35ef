"""Orbital-rotation parameters (Sec. 2.2, Eq. PsiJVBp) through the C ABI on the
GPU: the context's determinant occupancy gives the oracle's pair list, the
derivatives with respect to the rotation parameters (vbqmc_rotation_grad on
vbqmc_param_grad outputs) match the oracle's, and a rotated parameter vector
set on the context evaluates like the oracle's rotated wave function."""

import numpy as np
import pytest

import systems as S
from oracle import rotations as ROT
from tests.test_oracle_rotations import SYSTEMS

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2207_14715_amd as vb
    vb.load_library()
    return vb


def _rows(occ):
    return sorted({o.tobytes() for o in occ})


@pytest.mark.parametrize("name", ["h2_virtual", "f2", "f2_bovb", "small", "adjoint"])
def test_context_occupancy_gives_the_oracle_pairs(lib, oracle_mod, name):
    sysd = SYSTEMS[name]()
    o = oracle_mod.Oracle(sysd)
    ctx = lib.Context(sysd)
    occ = ctx.det_occupancy()
    ref = ROT.occupancy(o)
    assert _rows(occ) == _rows(ref)
    cls = lib.orbital_classes(np.asarray(sysd["lam"]))
    for lc in (None, cls):
        np.testing.assert_array_equal(lib.rotation_pairs(occ, lc), ROT.pairs(ref, lc))


@pytest.mark.parametrize("name,W", [("h2_virtual", 16), ("f2", 6), ("small", 6), ("adjoint", 2)])
def test_rotation_derivatives_match_oracle(lib, oracle_mod, name, W):
    """Every kept pair (both kinds) of the system, d lnPsi / d kappa and
    d E_L / d kappa per walker, scaled by the largest reference of the
    walker as in the adjoint tests."""
    import torch
    sysd = SYSTEMS[name]()
    o = oracle_mod.Oracle(sysd)
    prs = ROT.pairs(ROT.occupancy(o))
    if name == "adjoint":
        prs = prs[np.random.default_rng(2).choice(len(prs), 40, replace=False)]
    R = S.initial_walkers(sysd, W, seed=31)
    ctx = lib.Context(sysd)
    print(f"[rotation grad] {name} W={W} pairs={len(prs)}", flush=True)
    dl, de = ctx.param_grad(torch.from_numpy(R).cuda())
    kl, ke = ctx.rotation_grad(dl, de, prs)
    kl, ke = kl.cpu().numpy(), ke.cpu().numpy()
    torch.cuda.synchronize()
    rl, re = ROT.kappa_deriv(o, R, prs)
    for label, gpu, ref in (("d lnPsi/dkappa", kl, rl), ("d E_L/dkappa", ke, re)):
        err = np.max(np.abs(gpu - ref) / np.maximum(1.0, np.abs(ref).max(axis=1, keepdims=True)))
        assert err < 1e-8, f"{label}: scaled error {err:.2e}"


def test_out_of_range_pairs_give_nan_columns(lib):
    import torch
    sysd = S.f2_shaped()
    ctx = lib.Context(sysd)
    R = torch.from_numpy(S.initial_walkers(sysd, 3, seed=1)).cuda()
    dl, de = ctx.param_grad(R)
    prs = np.array([[8, 0, 1], [99, 0, 1], [8, -1, 0], [9, 8, 2]], np.int32)
    kl, ke = ctx.rotation_grad(dl, de, prs)
    kl, ke = kl.cpu().numpy(), ke.cpu().numpy()
    torch.cuda.synchronize()
    assert np.all(np.isfinite(kl[:, 0])) and np.all(np.isfinite(ke[:, 0]))
    assert np.all(np.isnan(kl[:, 1:])) and np.all(np.isnan(ke[:, 1:]))


def test_rotated_parameters_evaluate_like_the_oracle(lib, oracle_mod):
    """F2: theta for every kept pair, lambda' = exp(K)^T lambda on the host
    (vbqmc_rotate_orbitals), set on the context with the other parameters
    unchanged; evaluation against the oracle of the system built with
    scipy's rotated orbitals."""
    import torch
    from tests._helpers import compare_evaluate
    sysd = S.f2_shaped()
    ctx = lib.Context(sysd)
    o = oracle_mod.Oracle(sysd)
    prs = ROT.pairs(ROT.occupancy(o))
    theta = 0.05 * np.random.default_rng(4).normal(size=len(prs))
    p = ctx.get_params()
    cs, ls, _ = o.param_slices()
    lam = p[ls].reshape(o.n_orb, o.M)
    p[ls] = lib.rotate_orbitals(lam, prs, theta).reshape(-1)
    ctx.set_params(p)
    rot = dict(sysd, lam=ROT.rotate(sysd["lam"], prs, theta).tolist())
    R = S.initial_walkers(sysd, 32, seed=8)
    out = ctx.evaluate(torch.from_numpy(R).cuda())
    torch.cuda.synchronize()
    compare_evaluate(out, oracle_mod.Oracle(rot).evaluate(R), 1e-10)
