"""The linear-method sample sums on the GPU (vbqmc_lm_accumulate, FP64 MFMA
over walkers) and the estimators and step formed from them, against the
oracle (oracle/linear_method.py on the oracle's own derivatives and local
energies at the same seeded configurations), plus the strong zero-variance
step driven end to end by GPU derivatives."""

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


def _gpu_sums(ctx, R, w, splits):
    """param_grad + E_L on the GPU, accumulated in several calls."""
    import torch
    acc = ctx.new_lm_acc()
    Rt = torch.from_numpy(R).cuda()
    wt = None if w is None else torch.from_numpy(w).cuda()
    a = 0
    for b in splits:
        dl, de = ctx.param_grad(Rt[a:b].contiguous())
        el = ctx.evaluate(Rt[a:b].contiguous(), want=("eloc",))["eloc"]
        ctx.lm_accumulate(dl, de, el, acc, None if wt is None else wt[a:b].contiguous())
        a = b
    torch.cuda.synchronize()
    return acc


def _scaled(a, b):
    return np.max(np.abs(a - b)) / max(1.0, np.abs(b).max())


@pytest.mark.parametrize("seed,weighted", [(411, False), (412, True)])
def test_accumulated_estimators_match_oracle(lib, oracle_mod, seed, weighted):
    from oracle import linear_method as lm
    sysd = S.small_random_system(seed, n_inactive=2, n_active=5, n_pairs=2, n_unpaired=1, n_structures=4,
                                 kappa=0.8, poly=True)
    o = oracle_mod.Oracle(sysd)
    ctx = lib.Context(sysd)
    W = 70  # two calls, 48 + 22 walkers: ragged sample tails, several 64-wide blocks of P + 1
    R = S.initial_walkers(sysd, W, seed=seed)
    rng = np.random.default_rng(seed)
    w = rng.uniform(0.3, 1.7, W) if weighted else None
    print(f"[lm] {sysd['name']} W={W} P={ctx.n_params} weighted={weighted}", flush=True)
    acc = _gpu_sums(ctx, R, w, [48, W])
    got = lib.lm_estimators(acc, ctx.n_params)
    O, D = o.param_deriv(R)
    E = o.evaluate(R)["eloc"]
    ref = lm.estimators(O, E, D, w)
    assert abs(got["e0"] - ref["e0"]) <= 1e-10 * max(1.0, abs(ref["e0"]))
    for k in ("g_l", "g_r", "h_bar", "s_bar"):
        err = _scaled(got[k], ref[k])
        assert err < 1e-8, f"{k}: scaled error {err:.2e}"


def test_accumulate_large_parameter_set_is_the_weighted_product(lib):
    """The 6-nucleus / 30-electron / 1836-parameter system (29 x 29 blocks of
    64 per matrix, ragged edge): the accumulator equals the weighted products
    of its own inputs (kernel arithmetic at full size; the inputs' parity is
    the adjoint tests')."""
    import torch
    sysd = S.adjoint_molecule()
    ctx = lib.Context(sysd)
    P = ctx.n_params
    W = 37
    R = torch.from_numpy(S.initial_walkers(sysd, W, seed=21)).cuda()
    dl, de = ctx.param_grad(R)
    el = ctx.evaluate(R, want=("eloc",))["eloc"]
    w = torch.from_numpy(np.random.default_rng(3).uniform(0.5, 1.5, W)).cuda()
    print(f"[lm] adjoint molecule W={W} P={P}", flush=True)
    acc = ctx.new_lm_acc()
    ctx.lm_accumulate(dl, de, el, acc, w)
    torch.cuda.synchronize()
    O, D, E, wn = dl.cpu().numpy(), de.cpu().numpy(), el.cpu().numpy(), w.cpu().numpy()
    X = np.hstack([np.ones((W, 1)), O])
    Y = np.hstack([(E * E)[:, None], D])
    a = acc.cpu().numpy().reshape(3, P + 1, P + 1)
    for k, ref in enumerate([(X * wn[:, None]).T @ X, (X * (wn * E)[:, None]).T @ X, (X * wn[:, None]).T @ Y]):
        err = np.max(np.abs(a[k] - ref)) / np.abs(ref).max()
        assert err < 1e-13, f"matrix {k}: {err:.2e}"


def test_zero_variance_step_from_gpu_derivatives(lib):
    """Hydrogen in 0.3 e^-r + 0.5 e^-2r + 0.4 e^-3r, the e^-2r, e^-3r
    coefficients varied: the step from any sample reaches the exact 1s."""
    import torch
    sysd = S.hydrogen_sto_mix(coefs=(0.3, 0.5, 0.4))
    ctx = lib.Context(sysd)
    rng = np.random.default_rng(9)
    W = 64
    R = rng.normal(size=(W, 1, 3)) * 1.3
    acc = _gpu_sums(ctx, R, None, [W])
    est = lib.lm_estimators(acc, ctx.n_params)
    sel = np.array([2, 3])  # [c | lambda_00, lambda_01, lambda_02 | Jastrow]
    dp, e_lin = lib.lm_solve(est["e0"], est["g_l"][sel], est["g_r"][sel], est["h_bar"][np.ix_(sel, sel)],
                             est["s_bar"][np.ix_(sel, sel)])
    assert abs(e_lin + 0.5) < 1e-9, e_lin
    a = acc.cpu().numpy().reshape(3, ctx.n_params + 1, ctx.n_params + 1)
    mO = a[0, 0, 1 + sel] / a[0, 0, 0]
    c = (1.0 - dp @ mO) * np.array([0.3, 0.5, 0.4])
    c[1:] += dp
    assert np.max(np.abs(c[1:])) < 1e-9 * abs(c[0]), c
    assert est["var"] > 1e-3  # the sample's E_L is far from constant
    torch.cuda.synchronize()
