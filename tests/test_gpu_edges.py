"""Edge cases and error paths of the C ABI on the GPU: empty batches,
determinism of the counter-based walks, DMC population overflow, invalid
systems, and a DMC trajectory of a larger multi-determinant molecule."""

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


def test_empty_batches_are_no_ops(lib):
    import torch
    ctx = lib.Context(S.h2_heitler_london())
    R = torch.zeros(0, 2, 3, dtype=torch.float64, device="cuda")
    out = ctx.evaluate(R)
    assert out["logabs"].numel() == 0
    st = ctx.new_state(0)
    ctx.vmc_advance(st, 5, 1, 0, 0.5, W=0)


def test_vmc_is_bitwise_deterministic(lib):
    import torch
    sysd = S.f2_shaped()
    ctx = lib.Context(sysd)
    R0 = torch.from_numpy(S.initial_walkers(sysd, 256, seed=1)).cuda()
    outs = []
    for _ in range(2):
        st = ctx.walkers_init(R0)
        acc = ctx.vmc_advance(st, 6, 31, 0, 0.3)
        outs.append((ctx.positions(st).cpu().numpy(), acc["e_sum"].cpu().numpy()))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])


def test_dmc_population_overflow_is_reported(lib):
    import torch
    sysd = S.hydrogen_gaussian(0.3)
    ctx = lib.Context(sysd)
    W = 64
    R0 = torch.from_numpy(np.random.default_rng(0).normal(size=(W, 1, 3))).cuda()
    st0, st1 = ctx.new_state(W), ctx.new_state(W)
    ctx.walkers_init(R0, st0)
    # a trial energy far above E_L makes every weight large: the population
    # grows beyond the capacity of W records in the first step
    with pytest.raises(lib.VBQMCError) as ei:
        ctx.dmc_advance([st0, st1], W, 3, 1, 0, 0.05, 50.0, W)
    assert ei.value.code == -7


def test_invalid_system_rejected(lib):
    sysd = S.h2_heitler_london()
    bad = dict(sysd)
    bad["n_up"] = 2  # terms hold one up electron
    with pytest.raises(lib.VBQMCError):
        lib.Context(bad)


@pytest.mark.parametrize("kern", [1, 2])
def test_dmc_multideterminant_molecule_trajectory(lib, oracle_mod, kern):
    """DMC with the 10-nucleus, 64-determinant molecule against the oracle for
    a few steps, with one workgroup per walker (two waves) and with the
    electron-major launches."""
    import torch
    sysd = S.precision_molecule()
    W = 16
    o = oracle_mod.Oracle(sysd)
    R0 = S.initial_walkers(sysd, W, seed=12)
    e0 = o.evaluate(R0)["eloc"]
    et = float(np.median(e0))
    ref = o.dmc(R0, e0, 3, 5, 0, 0.002, et, W, capacity=4 * W)
    ctx = lib.Context(sysd, dmc_kernel=kern)
    print(f"[dmc molecule] dmc_kernel={ctx.info['dmc_kernel']}", flush=True)
    st0, st1 = ctx.new_state(4 * W), ctx.new_state(4 * W)
    ctx.walkers_init(torch.from_numpy(R0).cuda(), st0)
    out = ctx.dmc_advance([st0, st1], W, 3, 5, 0, 0.002, et, W)
    assert ref["rc"] == 0
    np.testing.assert_array_equal(out["pop"].cpu().numpy(), ref["pop"])
    np.testing.assert_array_equal(out["n_accept"].cpu().numpy(), ref["acc"])
    np.testing.assert_allclose(out["wsum"].cpu().numpy(), ref["wsum"], rtol=1e-8)
    R = ctx.positions(st0, out["W"]).cpu().numpy()
    np.testing.assert_allclose(R, ref["R"], rtol=1e-8, atol=1e-8)


@pytest.mark.parametrize("kern", [1, 2, 3])
def test_dmc_is_bitwise_deterministic(lib, kern):
    """Counter-based draws and fixed-order reductions: two DMC runs from the
    same walkers and seed give the same records and logs bit for bit."""
    import torch
    sysd = S.f2_shaped()
    ctx = lib.Context(sysd, dmc_kernel=kern)
    W = 96
    R0 = torch.from_numpy(S.initial_walkers(sysd, W, seed=4)).cuda()
    outs = []
    for _ in range(2):
        st = [ctx.new_state(4 * W), ctx.new_state(4 * W)]
        ctx.walkers_init(R0, st[0])
        out = ctx.dmc_advance(st, W, 4, 8, 0, 0.002, -200.0, W)
        outs.append((ctx.positions(st[0], out["W"]).cpu().numpy(), ctx.record_eloc(st[0], out["W"]).cpu().numpy(),
                     {k: v.cpu().numpy() for k, v in out.items() if hasattr(v, "cpu")}))
    torch.cuda.synchronize()
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1], equal_nan=True)
    for k in outs[0][2]:
        assert np.array_equal(outs[0][2][k], outs[1][2][k], equal_nan=True), k
