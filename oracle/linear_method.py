"""Oracle of the linear optimisation method -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU baseline
may use it; the library never does.  Plain numpy in FP64, written from the
paper: the sampled estimators of Sec. 2.3.1 (Eqs. Hi0, H0j, Hij, Sij) term by
term from per-sample arrays, and the step of Sec. 2.2 (Eqs. Psiblin,
geneigeq, geneigeqM) as the full (P+1)-dimensional generalised eigenproblem
solved by a library routine (scipy.linalg.eig), with the eigenvector chosen
that changes the wave function least.

Inputs per sample k (a configuration drawn from rho_0, or any configuration
with a weight): O[k][i] = Psi_i / Psi_0 = d ln|Psi| / dp_i, E[k] = E_L and
D[k][j] = E_L,j = d E_L / dp_j (the oracle's own derivatives,
``Oracle.param_deriv``, and local energies, ``Oracle.evaluate``).

Pins (tests/test_oracle_linear_method.py): the strong zero-variance property
that the paper states for these non-symmetric estimators (a wave function
whose derivatives span the exact ground state gives the exact energy and
parameters from any sample), the invariance of every estimator under a
constant shift of O (they are covariances), and symmetry of Sbar.
"""

import numpy as np


def estimators(O, E, D, w=None):
    """E0, g_L, g_R, Hbar, Sbar as averages over the samples (weights w, or
    unit weights)."""
    O = np.asarray(O, np.float64)
    D = np.asarray(D, np.float64)
    E = np.asarray(E, np.float64)
    M = O.shape[0]
    w = np.ones(M) if w is None else np.asarray(w, np.float64)
    sw = w.sum()

    def avg(x):  # weighted average over the sample axis
        return np.tensordot(w, x, axes=(0, 0)) / sw

    mO = avg(O)                      # <Psi_i / Psi_0>
    mE = avg(E)                      # <E_L>
    mOE = avg(O * E[:, None])        # <(Psi_i / Psi_0) E_L>
    mD = avg(D)                      # <E_L,j>
    OO = (O * w[:, None]).T @ O / sw                # <O_i O_j>
    OOE = (O * (w * E)[:, None]).T @ O / sw         # <O_i O_j E_L>
    OD = (O * w[:, None]).T @ D / sw                # <O_i E_L,j>
    g_l = 2.0 * (mOE - mO * mE)                               # Eq. Hi0
    g_r = 2.0 * (mOE - mO * mE + mD)                          # Eq. H0j
    h_bar = (OOE - np.outer(mO, mOE) - np.outer(mOE, mO)      # Eq. Hij
             + np.outer(mO, mO) * mE + OD - np.outer(mO, mD))
    s_bar = OO - np.outer(mO, mO)                             # Eq. Sij
    return {"e0": mE, "g_l": g_l, "g_r": g_r, "h_bar": h_bar, "s_bar": s_bar}


def solve(e0, g_l, g_r, h_bar, s_bar, a_diag=0.0):
    """(dp, E_lin): the generalised eigenproblem
    [[E0, g_R^T / 2], [g_L / 2, Hbar + a_diag I]] v = E [[1, 0], [0, Sbar]] v
    (Eq. geneigeqM) in full; among the real eigenpairs with v_0 != 0 the one
    with the largest |v_0|^2 / |v^T B v| (the smallest change of the current
    wave function), scaled to v_0 = 1."""
    import scipy.linalg
    n = len(g_l)
    A = np.zeros((n + 1, n + 1))
    A[0, 0] = e0
    A[0, 1:] = 0.5 * np.asarray(g_r)
    A[1:, 0] = 0.5 * np.asarray(g_l)
    A[1:, 1:] = np.asarray(h_bar) + a_diag * np.eye(n)
    B = np.zeros((n + 1, n + 1))
    B[0, 0] = 1.0
    B[1:, 1:] = s_bar
    vals, vecs = scipy.linalg.eig(A, B)
    best, pick = -1.0, None
    for k in range(n + 1):
        lam, v = vals[k], vecs[:, k]
        if not np.isfinite(lam) or abs(lam.imag) > 1e-9 * max(1.0, abs(lam.real)) or abs(v[0]) == 0:
            continue
        v = (v / v[0]).real
        score = 1.0 / abs(v @ B @ v)
        if score > best:
            best, pick = score, (v[1:].copy(), float(lam.real))
    if pick is None:
        raise ValueError("no admissible eigenvector")
    return pick
