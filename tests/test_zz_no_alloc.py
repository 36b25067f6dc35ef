"""vbqmc_dmc_advance_noalloc (the DMC entry point that allocates nothing)
against vbqmc_dmc_advance with a caller workspace: two calls in a row on the
same records' inputs, the second with fewer walkers, must give the same
walks, logs and trial energies bit for bit; a capacity whose workspace
exceeds the fixed scratch is refused before any work."""

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


def _log(n, dev="cuda"):
    import torch
    return {k: torch.zeros(n, dtype=torch.float64, device=dev)
            for k in ("pop", "wsum", "wesum", "wcsum", "etrial", "n_accept", "n_prop")}


@pytest.mark.parametrize("kern", [1, 2, 3])
def test_noalloc_matches_workspace_entry_point(lib, oracle_mod, kern):
    import torch
    sysd = S.small_random_system(311, n_inactive=2, n_active=5, n_pairs=2, n_unpaired=1, n_structures=4)
    ctx = lib.Context(sysd, dmc_kernel=kern)
    o = oracle_mod.Oracle(sysd)
    cases = []
    for W, steps, seed in ((64, 4, 77), (40, 3, 91)):  # the second call is smaller
        R0 = S.initial_walkers(sysd, W, seed=seed)
        cases.append((W, steps, seed, R0, float(np.mean(o.evaluate(R0)["eloc"]))))

    def run(case, noalloc):
        W, steps, seed, R0, et = case
        print(f"[noalloc] W={W} steps={steps} dmc_kernel={kern} noalloc={noalloc}", flush=True)
        st = [ctx.new_state(4 * W), ctx.new_state(4 * W)]
        ctx.walkers_init(torch.from_numpy(R0).cuda(), st[0])
        lg = _log(steps)
        if noalloc:
            res = ctx.dmc_advance_noalloc(st, W, steps, seed, 5, 0.005, et, W, lg)
        else:
            res = ctx.dmc_advance(st, W, steps, seed, 5, 0.005, et, W, log=lg)
        torch.cuda.synchronize()
        return res, ctx.positions(st[0], res["W"]).cpu().numpy(), ctx.record_eloc(st[0], res["W"]).cpu().numpy()

    ref = [run(c, False) for c in cases]
    got = [run(c, True) for c in cases]  # two no-alloc calls in a row, the second smaller
    for (a, Ra, ea), (b, Rb, eb) in zip(ref, got):
        assert a["W"] == b["W"] and a["e_trial"] == b["e_trial"]
        for k in ("pop", "wsum", "wesum", "wcsum", "etrial", "n_accept", "n_prop"):
            assert torch.equal(a[k], b[k]), k
        np.testing.assert_array_equal(Ra, Rb)
        np.testing.assert_array_equal(ea, eb)


def test_noalloc_refuses_capacity_beyond_scratch(lib):
    import torch
    sysd = S.hydrogen_gaussian(0.4)
    ctx = lib.Context(sysd, dmc_kernel=2)
    nb = ctx.dmc_workspace(16, 1).numel() * 8
    per = (ctx.dmc_workspace(32, 1).numel() * 8 - nb) / 16
    cap = int((32 << 20) / per) + 64
    st = [ctx.new_state(cap), ctx.new_state(cap)]
    with pytest.raises(lib.VBQMCError) as ei:
        ctx.dmc_advance_noalloc(st, 8, 1, 1, 0, 0.01, -0.5, 8, _log(1))
    assert ei.value.code == -3
