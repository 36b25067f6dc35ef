"""Pins of the linear-method oracle (oracle/linear_method.py) and the
library's host-side estimator formation and step (vbqmc_lm_estimators,
vbqmc_lm_solve) against it.

* Strong zero-variance principle (the property the paper states for the
  non-symmetric estimators of Sec. 2.3.1): a hydrogen electron in
  c1 e^-r + c2 e^-2r + c3 e^-3r with c2, c3 varied; the derivatives span the
  exact 1s, so ANY sample (here random points with random weights, not even
  drawn from rho_0) gives E_lin = -1/2 and a linear wave function with no
  e^-2r, e^-3r component.
* The estimators are covariances: invariant when a constant is added to any
  Psi_i / Psi_0 column (a dropped or misplaced mean term breaks this).
* Sbar is symmetric positive semi-definite.
"""

import ctypes

import numpy as np
import pytest

import systems as S


def _hydrogen_samples(oracle_mod, M, seed):
    sysd = S.hydrogen_sto_mix(coefs=(0.3, 0.5, 0.4))
    o = oracle_mod.Oracle(sysd)
    rng = np.random.default_rng(seed)
    R = rng.normal(size=(M, 1, 3)) * 1.3
    _, ls, _ = o.param_slices()
    idx = np.array([ls.start + 1, ls.start + 2])  # the e^-2r and e^-3r coefficients
    O, D = o.param_deriv(R, idx)
    E = o.evaluate(R)["eloc"]
    return sysd, O, E, D, rng


def _linear_coefficients(sysd, O, w, dp):
    """Orbital coefficients of Psi_0 + sum_j dp_j Psibar_j (Eq. Psiblin with
    Eq. semiorthog): (1 - sum_j dp_j <O_j>) c0 + dp on the varied ones."""
    mO = (w @ O) / w.sum()
    c = (1.0 - dp @ mO) * np.asarray(sysd["lam"][0], np.float64)
    c[1:] += dp
    return c


@pytest.mark.parametrize("weighted", [False, True])
def test_zero_variance_hydrogen(oracle_mod, weighted):
    from oracle import linear_method as lm
    sysd, O, E, D, rng = _hydrogen_samples(oracle_mod, 40, 5)
    w = rng.uniform(0.2, 2.0, len(E)) if weighted else np.ones(len(E))
    # the sample itself is far from the ground state: E_L spreads widely
    assert np.ptp(E) > 0.3
    est = lm.estimators(O, E, D, w)
    dp, e_lin = lm.solve(est["e0"], est["g_l"], est["g_r"], est["h_bar"], est["s_bar"])
    assert abs(e_lin + 0.5) < 1e-10, e_lin
    c = _linear_coefficients(sysd, O, w, dp)
    assert np.max(np.abs(c[1:])) < 1e-10 * abs(c[0]), c


def test_estimators_are_covariances():
    from oracle import linear_method as lm
    rng = np.random.default_rng(11)
    M, P = 50, 6
    O = rng.normal(size=(M, P))
    E = rng.normal(size=M) - 3.0
    D = rng.normal(size=(M, P))
    w = rng.uniform(0.5, 1.5, M)
    a = lm.estimators(O, E, D, w)
    b = lm.estimators(O + rng.normal(size=P) * 5.0, E, D, w)
    for k in ("g_l", "g_r", "h_bar", "s_bar"):
        np.testing.assert_allclose(b[k], a[k], rtol=1e-11, atol=1e-11 * np.abs(a[k]).max())
    assert b["e0"] == a["e0"]
    np.testing.assert_allclose(a["s_bar"], a["s_bar"].T, rtol=0, atol=1e-14)
    assert np.linalg.eigvalsh(a["s_bar"]).min() > -1e-12
    # E_L,j enters g_R (and Hbar) only: zero D gives g_L = g_R
    z = lm.estimators(O, E, np.zeros_like(D), w)
    np.testing.assert_allclose(z["g_r"], z["g_l"], rtol=1e-14, atol=1e-14)


def _accumulator(O, E, D, w):
    """The library's accumulator layout built from sample arrays (augmented
    rows X = [1 | O], Y = [E^2 | D])."""
    M, P = O.shape
    X = np.hstack([np.ones((M, 1)), O])
    Y = np.hstack([(E * E)[:, None], D])
    return np.concatenate([((X * w[:, None]).T @ X).ravel(), ((X * (w * E)[:, None]).T @ X).ravel(),
                           ((X * w[:, None]).T @ Y).ravel()])


def _lib_or_skip():
    import paper_2207_14715_amd as vb
    try:
        vb.load_library()
    except RuntimeError as e:
        pytest.skip(str(e))
    return vb


def test_library_estimators_match_oracle():
    from oracle import linear_method as lm
    vb = _lib_or_skip()
    rng = np.random.default_rng(12)
    M, P = 40, 7
    O = rng.normal(size=(M, P))
    E = rng.normal(size=M) - 2.0
    D = rng.normal(size=(M, P))
    w = rng.uniform(0.5, 1.5, M)
    got = vb.lm_estimators(_accumulator(O, E, D, w), P)
    ref = lm.estimators(O, E, D, w)
    assert abs(got["e0"] - ref["e0"]) < 1e-13
    for k in ("g_l", "g_r", "h_bar", "s_bar"):
        np.testing.assert_allclose(got[k], ref[k], rtol=1e-11, atol=1e-12 * np.abs(ref[k]).max())
    var = (w @ (E * E)) / w.sum() - ((w @ E) / w.sum()) ** 2
    assert abs(got["var"] - var) < 1e-12


@pytest.mark.parametrize("weighted", [False, True])
def test_library_step_zero_variance(oracle_mod, weighted):
    vb = _lib_or_skip()
    sysd, O, E, D, rng = _hydrogen_samples(oracle_mod, 40, 6)
    w = rng.uniform(0.2, 2.0, len(E)) if weighted else np.ones(len(E))
    est = vb.lm_estimators(_accumulator(O, E, D, w), O.shape[1])
    dp, e_lin = vb.lm_solve(est["e0"], est["g_l"], est["g_r"], est["h_bar"], est["s_bar"])
    assert abs(e_lin + 0.5) < 1e-10, e_lin
    c = _linear_coefficients(sysd, O, w, dp)
    assert np.max(np.abs(c[1:])) < 1e-10 * abs(c[0]), c


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_library_step_matches_oracle_eigenproblem(seed):
    """A random pencil whose other eigenvalues lie about 1 Ha above E0: the
    library's root next to E0 is the oracle's least-change eigenvector."""
    from oracle import linear_method as lm
    vb = _lib_or_skip()
    rng = np.random.default_rng(seed)
    n, e0 = 9, -7.3
    A = rng.normal(size=(n, n))
    s_bar = A @ A.T / n + 0.5 * np.eye(n)
    h_bar = (e0 + 1.0) * s_bar + 0.05 * rng.normal(size=(n, n))
    g_l = 0.1 * rng.normal(size=n)
    g_r = g_l + 0.01 * rng.normal(size=n)
    for a_diag in (0.0, 0.2):
        dp, el = vb.lm_solve(e0, g_l, g_r, h_bar, s_bar, a_diag)
        rdp, rel = lm.solve(e0, g_l, g_r, h_bar, s_bar, a_diag)
        assert abs(el - rel) < 1e-11 * abs(rel)
        np.testing.assert_allclose(dp, rdp, rtol=1e-9, atol=1e-12)
        assert el < e0


def test_library_step_rejects_bad_arguments():
    vb = _lib_or_skip()
    lib = vb.load_library()
    z = np.zeros(4)
    pd = ctypes.POINTER(ctypes.c_double)
    rc = lib.vbqmc_lm_solve(0, 0.0, z.ctypes.data_as(pd), z.ctypes.data_as(pd), z.ctypes.data_as(pd),
                            z.ctypes.data_as(pd), 0.0, z.ctypes.data_as(pd), z.ctypes.data_as(pd))
    assert rc == -1
    n = ctypes.c_int64()
    assert lib.vbqmc_lm_acc_doubles(0, ctypes.byref(n)) == -1
    assert lib.vbqmc_lm_acc_doubles(5, ctypes.byref(n)) == 0 and n.value == 3 * 36
    # an exactly singular pencil (a zero parameter) is reported, not solved
    with pytest.raises(vb.VBQMCError):
        vb.lm_solve(-1.0, np.zeros(2), np.zeros(2), np.zeros((2, 2)), np.zeros((2, 2)))
