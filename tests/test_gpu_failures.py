"""Failure handling and resumption, forced from the host with inputs the library checks:
a configuration with a non-finite coordinate, two same-spin electrons at one
point (Psi = 0) and two opposite-spin electrons at one point (a non-finite
E_L).  Evaluation reports such walkers (sign 0, a rounding-level |Psi| or a
non-finite E_L) without
disturbing the others; VMC keeps a flagged walker out of the sums; DMC
stops with ENONFINITE.  (No coordinate becomes an index anywhere in the
kernels: a non-finite value can only make values non-finite, and the
kernels turn those into flags.)"""

import numpy as np
import pytest

import systems as S
from tests._helpers import compare_evaluate

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2207_14715_amd as vb
    vb.load_library()
    return vb


def _bad_batch(sysd, W, seed=5):
    """W configurations; walker 1 has a NaN coordinate, walker 2 has electrons
    0 and 1 (same spin) at one point, walker 3 has electrons 0 and n_up
    (opposite spins) at one point."""
    R = S.initial_walkers(sysd, W, seed=seed)
    R[1, 0, 1] = np.nan
    R[2, 1] = R[2, 0]
    R[3, sysd["n_up"]] = R[3, 0]
    return R


def test_evaluate_reports_bad_configurations(lib, oracle_mod):
    import torch
    sysd = S.f2_shaped()
    W = 16
    R = _bad_batch(sysd, W)
    ctx = lib.Context(sysd)
    out = ctx.evaluate(torch.from_numpy(R).cuda())
    torch.cuda.synchronize()
    sign = out["sign"].cpu().numpy()
    eloc = out["eloc"].cpu().numpy()
    la = out["logabs"].cpu().numpy()
    assert sign[1] == 0 and not np.isfinite(eloc[1])
    # identical rows: Psi = 0 exactly; the library's inversion scales rows by
    # a reciprocal pivot, so it may leave a rounding-level determinant
    # instead (|Psi| below 1e-11 of the other walkers') rather than sign 0
    assert sign[2] == 0 or la[2] < np.min(la[np.r_[0, 4:W]]) - 25.0, (sign[2], la[2])
    assert not np.isfinite(eloc[3])
    good = np.r_[0, 4:W]
    ref = oracle_mod.Oracle(sysd).evaluate(R[good])
    compare_evaluate({k: v[good] for k, v in out.items()}, ref, 1e-10)


@pytest.mark.parametrize("kernel", ["rows", "wres", 32])
def test_vmc_keeps_flagged_walkers_out_of_the_sums(lib, kernel):
    import torch
    sysd = S.f2_shaped()
    W = 16
    kw = {"rows": {"step_kernel": 2}, "wres": {"step_kernel": 3}, 32: {"walker_lanes": 32, "step_kernel": 1}}[kernel]
    ctx = lib.Context(sysd, **kw)
    st = ctx.walkers_init(torch.from_numpy(_bad_batch(sysd, W)).cuda())
    acc = ctx.vmc_advance(st, 3, 7, 0, 0.3)
    torch.cuda.synchronize()
    es, el = acc["e_sum"].cpu().numpy(), acc["e_last"].cpu().numpy()
    # walker 1 (NaN) is flagged at init and stays out; the others move
    # away from their coincidences (walker 3's first move separates its two
    # electrons)
    assert es[1] == 0.0 and not np.isfinite(el[1]), (es[1], el[1])
    assert np.all(np.isfinite(es[np.r_[0, 3:W]])) and np.all(np.isfinite(el[np.r_[0, 3:W]]))


@pytest.mark.parametrize("kern", [1, 2, 3])
def test_dmc_stops_on_a_non_finite_walker(lib, kern):
    import torch
    sysd = S.f2_shaped()
    W = 16
    ctx = lib.Context(sysd, dmc_kernel=kern)
    st0, st1 = ctx.new_state(4 * W), ctx.new_state(4 * W)
    ctx.walkers_init(torch.from_numpy(_bad_batch(sysd, W)).cuda(), st0)
    with pytest.raises(lib.VBQMCError) as ei:
        ctx.dmc_advance([st0, st1], W, 2, 3, 0, 0.002, -200.0, W)
    assert ei.value.code == -6
    torch.cuda.synchronize()


@pytest.mark.parametrize("kernel", [2, 3])
def test_vmc_resumes_from_positions(lib, kernel):
    """Checkpoint = the walker positions (vbqmc_walkers_positions); there is
    no random-number state, the Philox counters come from (seed, walker,
    step).  Six steps in one call equal three steps, a checkpoint, a fresh
    vbqmc_walkers_init from the saved positions (fresh inverses) and three
    more steps, to rounding: same acceptances, same positions and energies
    (row kernel and walker-resident kernel)."""
    import torch
    sysd = S.f2_shaped()
    W, seed = 61, 99
    R0 = torch.from_numpy(S.initial_walkers(sysd, W, seed=2)).cuda()
    ctx = lib.Context(sysd, step_kernel=kernel)
    st_a = ctx.walkers_init(R0)
    a = ctx.vmc_advance(st_a, 6, seed, 0, 0.3)
    st = ctx.walkers_init(R0)
    b = ctx.vmc_advance(st, 3, seed, 0, 0.3)
    saved = ctx.positions(st).cpu().numpy()          # the checkpoint
    st2 = ctx.walkers_init(torch.from_numpy(saved).cuda())
    ctx.vmc_advance(st2, 3, seed, 3, 0.3, False, b)
    Ra, Rb = ctx.positions(st_a).cpu().numpy(), ctx.positions(st2).cpu().numpy()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(a["n_accept"].cpu().numpy(), b["n_accept"].cpu().numpy())
    np.testing.assert_allclose(Rb, Ra, rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(b["e_sum"].cpu().numpy(), a["e_sum"].cpu().numpy(), rtol=1e-9, atol=1e-9)
