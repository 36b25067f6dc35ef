"""The three-body Jastrow f_een (Sec. 2.1) on the GPU against the oracle:
evaluation (ln|Psi|, gradient, E_L) of systems with f_een, single-electron
VMC and DMC walks on the walker-resident kernel, all-electron VMC on the
one-workgroup-per-walker kernel (S_IJ sums included), the parameter
derivatives and linear-method sums, and the calls that refuse f_een."""

import numpy as np
import pytest

import systems as S
from tests._helpers import compare_evaluate
from tests.test_gpu_walks import _check_dmc, _check_vmc, _dmc_pair, _vmc_pair

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2207_14715_amd as vb
    vb.load_library()
    return vb


def _small_een():
    # (the system of the plain evaluate parity test with seed 102)
    return S.with_een(S.small_random_system(102, n_inactive=2, n_active=5, n_pairs=2, n_unpaired=1,
                                            n_structures=4), scale=0.2)


@pytest.mark.parametrize("name", ["h2", "small", "f2", "adjoint"])
def test_evaluate(lib, oracle_mod, name):
    import torch
    sysd = {"h2": lambda: S.with_een(S.h2_heitler_london(), scale=0.3), "small": _small_een,
            "f2": lambda: S.with_een(S.f2_shaped()), "adjoint": lambda: S.with_een(S.adjoint_molecule())}[name]()
    W = {"h2": 200, "small": 64, "f2": 96, "adjoint": 8}[name]
    o = oracle_mod.Oracle(sysd)
    R = S.initial_walkers(sysd, W, seed=102, sigma=0.5)
    ref = o.evaluate(R)
    ctx = lib.Context(sysd)
    assert ctx.n_params == o.n_params
    print(f"[een evaluate] {sysd['name']} W={W} N={ctx.N}", flush=True)
    out = ctx.evaluate(torch.from_numpy(R).cuda())
    torch.cuda.synchronize()
    compare_evaluate(out, ref, 1e-10)


def test_vmc_all_electron_h2(lib, oracle_mod):
    ref, acc, R, _ = _vmc_pair(lib, oracle_mod, S.with_een(S.h2_heitler_london(), scale=0.3), 128, 20, 0.5, True)
    _check_vmc(ref, acc, R, 20, oracle_obj=ref["oracle"])


@pytest.mark.parametrize("name", ["small", "f2"])
def test_vmc_walker_resident(lib, oracle_mod, name):
    # 12 sweeps pass the 32-update refresh on F2 (Newton-Schulz from the
    # running inverse); 61 / 45 walkers leave a partly filled workgroup
    # (with S_IJ sums on the small system)
    sysd = _small_een() if name == "small" else S.with_een(S.f2_shaped())
    W, steps = (45, 10) if name == "small" else (61, 12)
    ref, acc, R, ctx = _vmc_pair(lib, oracle_mod, sysd, W, steps, 0.3, False, sij=name == "small")
    assert ctx.info["step_kernel"] == 3
    _check_vmc(ref, acc, R, steps, oracle_obj=ref["oracle"])
    if name == "small":
        np.testing.assert_allclose(acc["sij_sum"].cpu().numpy(), ref["sij_sum"], rtol=1e-8, atol=1e-8)


def test_vmc_walker_resident_40_electrons(lib, oracle_mod):
    sysd = S.with_een(S.precision_molecule(), scale=0.02)
    ref, acc, R, ctx = _vmc_pair(lib, oracle_mod, sysd, 12, 4, 0.3, False)
    assert ctx.info["step_kernel"] == 3
    _check_vmc(ref, acc, R, 4, oracle_obj=ref["oracle"])


@pytest.mark.parametrize("name", ["small", "f2"])
def test_dmc_walker_resident(lib, oracle_mod, name):
    sysd = _small_een() if name == "small" else S.with_een(S.f2_shaped())
    W, steps, tau = (64, 5, 0.005) if name == "small" else (45, 3, 0.002)
    ref, out, R = _dmc_pair(lib, oracle_mod, sysd, W, steps, tau, dmc_kernel=3, et_median=True)
    _check_dmc(ref, out, R, ref["e_rec"], ref["oracle"])


def test_paths_without_f_een_refuse_it(lib):
    import torch
    sysd = S.with_een(S.f2_shaped())
    for kw in ({"step_kernel": 1}, {"step_kernel": 2}, {"dmc_kernel": 1}, {"dmc_kernel": 2}):
        with pytest.raises(lib.VBQMCError):
            lib.Context(sysd, **kw)
    ctx = lib.Context(sysd)
    W = 8
    st = ctx.walkers_init(torch.from_numpy(S.initial_walkers(sysd, W, seed=1)).cuda())
    acc = ctx.new_vmc_acc(W)
    with pytest.raises(lib.VBQMCError):
        ctx.vmc_sweep(st, 1, 0, 0.3, acc["n_accept"])
    with pytest.raises(lib.VBQMCError):
        ctx.vmc_measure(st, acc)
    torch.cuda.synchronize()


@pytest.mark.parametrize("name", ["small", "f2"])
def test_parameter_derivatives_all_parameters(lib, oracle_mod, name):
    """vbqmc_param_grad with f_een: every parameter (the 23 f_een
    coefficients per nucleus close the vector) against the oracle's dual
    numbers; the f_een gradient also enters every other dE_L/dp."""
    from tests.test_gpu_adjoint import _compare
    sysd = _small_een() if name == "small" else S.with_een(S.f2_shaped())
    ctx, o, R, dl, de = _compare(lib, oracle_mod, sysd, 6 if name == "small" else 4)
    assert ctx.n_params == o.n_params == o.param_slices()[2].stop


def test_parameter_derivatives_30_electrons(lib, oracle_mod):
    """The 6-nucleus, 30-electron molecule with f_een: structure coefficients,
    sampled orbital coefficients and every Jastrow parameter (138 f_een)."""
    from tests.test_gpu_adjoint import _compare
    sysd = S.with_een(S.adjoint_molecule(), scale=0.02)
    o = oracle_mod.Oracle(sysd)
    cs, ls, js = o.param_slices()
    rng = np.random.default_rng(1)
    lam_nz = np.flatnonzero(np.asarray(sysd["lam"]).reshape(-1) != 0) + ls.start
    idx = np.concatenate([np.arange(cs.start, cs.stop), rng.choice(lam_nz, 30, replace=False),
                          np.arange(js.start, js.stop)])
    _compare(lib, oracle_mod, sysd, 2, idx)


def test_linear_method_sums_cover_the_een_parameters(lib):
    """The linear-method accumulator of a system with f_een spans all its
    parameters: it equals the weighted products of its own inputs."""
    import torch
    sysd = _small_een()
    ctx = lib.Context(sysd)
    P = ctx.n_params
    W = 21
    R = torch.from_numpy(S.initial_walkers(sysd, W, seed=21)).cuda()
    dl, de = ctx.param_grad(R)
    el = ctx.evaluate(R, want=("eloc",))["eloc"]
    acc = ctx.new_lm_acc()
    ctx.lm_accumulate(dl, de, el, acc)
    torch.cuda.synchronize()
    O, D, E = dl.cpu().numpy(), de.cpu().numpy(), el.cpu().numpy()
    X = np.hstack([np.ones((W, 1)), O])
    Y = np.hstack([(E * E)[:, None], D])
    a = acc.cpu().numpy().reshape(3, P + 1, P + 1)
    for k, ref in enumerate([X.T @ X, (X * E[:, None]).T @ X, X.T @ Y]):
        assert np.max(np.abs(a[k] - ref)) <= 1e-12 * np.abs(ref).max(), k
