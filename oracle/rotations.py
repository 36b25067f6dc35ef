"""Oracle of the orbital-rotation parameters -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU baseline
may use it; the library never does.  Plain numpy / scipy in FP64, written
from Sec. 2.2 (Eq. PsiJVBp and the passage on orbital classes that follows):

* the orbitals fall into three classes by their occupation in the
  determinants of the wave function: inactive (doubly occupied in all of
  them), active (occupied in some), virtual (in none);
* the excitations l -> k kept are inactive -> active, inactive -> virtual,
  active -> virtual and active -> active, the last only where the
  excitation acts on the wave function; where the reverse excitation does
  not act the pair carries the condition kappa_lk = -kappa_kl (one
  parameter), where both act kappa_kl and kappa_lk are independent;
* orbitals of different localization classes (expanded on different sets of
  basis functions) do not mix;
* redundant parameters are found from the samples (here: a parameter whose
  centred derivative column lies in the span of the kept earlier ones, by
  least squares).

The determinants come from the oracle's own HLSP expansion
(``Oracle.dets()``); a determinant with a repeated orbital in one spin is
identically zero and is left out.  The rotation itself is exp(kappa) acting
on the orbitals, phi'_l = sum_k exp(K)[k][l] phi_k (scipy's expm); to first
order orbital l gains kappa_kl phi_k, so d/d kappa_kl at kappa = 0 is
sum_mu lambda[k][mu] d/d lambda[l][mu], formed here from the oracle's dual
numbers (``Oracle.param_deriv``).

Pins (tests/test_oracle_rotations.py): hand-enumerated pair lists of the H2,
H2-with-a-virtual and F2-shaped systems; the pair list against the
brute-force test "the derivative along E_kl vanishes at every sampled
configuration" over all ordered orbital pairs; the derivative formula
against fourth-order finite differences of ln|Psi| and E_L of the rotated
wave function; the redundancy rule against the exact linear relations of the
H2 Heitler-London function (one structure coefficient and one of the two
active-active parameters are redundant).
"""

import numpy as np

INACTIVE, ACTIVE, VIRTUAL = 0, 1, 2


def occupancy(oracle_obj):
    """[n_dets][2][n_orb] occupation of each nonvanishing determinant."""
    _, up, dn = oracle_obj.dets()
    rows = []
    for u, d in zip(up, dn):
        if len(set(u.tolist())) < len(u) or len(set(d.tolist())) < len(d):
            continue  # a repeated orbital: the determinant is zero
        o = np.zeros((2, oracle_obj.n_orb), np.uint8)
        o[0, u] = 1
        o[1, d] = 1
        rows.append(o)
    return np.array(rows, np.uint8)


def orbital_kinds(occ):
    """INACTIVE / ACTIVE / VIRTUAL per orbital."""
    both = occ.all(axis=(0, 1))
    none = ~occ.any(axis=(0, 1))
    return np.where(both, INACTIVE, np.where(none, VIRTUAL, ACTIVE))


def acts(occ, k, l):
    """Does the excitation l -> k act on some determinant (l present and k
    absent in one of its spins)?"""
    return bool(np.any(occ[:, :, l].astype(bool) & ~occ[:, :, k].astype(bool)))


def pairs(occ, loc_class=None):
    """(k, l, kind) of the kept excitations l -> k, ordered by l then k; kind 1
    for a pair with kappa_lk = -kappa_kl, 0 for an independent parameter."""
    kinds = orbital_kinds(occ)
    n = occ.shape[2]
    allowed = {(INACTIVE, ACTIVE), (INACTIVE, VIRTUAL), (ACTIVE, VIRTUAL), (ACTIVE, ACTIVE)}
    out = []
    for l in range(n):
        for k in range(n):
            if k == l or (kinds[l], kinds[k]) not in allowed:
                continue
            if loc_class is not None and loc_class[k] != loc_class[l]:
                continue
            if kinds[l] == ACTIVE and kinds[k] == ACTIVE:
                if not acts(occ, k, l):
                    continue
                kind = 0 if acts(occ, l, k) else 1
            else:
                kind = 1  # the reverse excitation lands in an inactive orbital or leaves a virtual one
            out.append((k, l, kind))
    return np.array(out, np.int32).reshape(-1, 3)


def classes_from_support(lam):
    """Orbitals with the same set of nonzero coefficients share a class
    (numbered by the first orbital of the class)."""
    lam = np.asarray(lam)
    pat = lam != 0
    cls = np.arange(lam.shape[0])
    for p in range(lam.shape[0]):
        for q in range(p):
            if np.array_equal(pat[p], pat[q]):
                cls[p] = cls[q]
                break
    return cls


def generator(n_orb, prs, theta):
    K = np.zeros((n_orb, n_orb))
    for (k, l, kind), t in zip(prs, theta):
        K[k, l] += t
        if kind == 1:
            K[l, k] -= t
    return K


def rotate(lam, prs, theta):
    """lambda' with phi'_l = sum_k exp(K)[k][l] phi_k."""
    import scipy.linalg
    lam = np.asarray(lam, np.float64)
    E = scipy.linalg.expm(generator(lam.shape[0], prs, theta))
    return E.T @ lam


def kappa_deriv(oracle_obj, R, prs):
    """d ln|Psi| / d kappa and d E_L / d kappa [W][n_pairs] from the oracle's
    derivatives with respect to the orbital coefficients."""
    _, ls, _ = oracle_obj.param_slices()
    M = oracle_obj.M
    lam = oracle_obj.lam
    dl, de = oracle_obj.param_deriv(R, np.arange(ls.start, ls.stop))
    W = dl.shape[0]
    dl = dl.reshape(W, oracle_obj.n_orb, M)
    de = de.reshape(W, oracle_obj.n_orb, M)
    ol = np.zeros((W, len(prs)))
    oe = np.zeros((W, len(prs)))
    for q, (k, l, kind) in enumerate(prs):
        ol[:, q] = dl[:, l, :] @ lam[k]
        oe[:, q] = de[:, l, :] @ lam[k]
        if kind == 1:
            ol[:, q] -= dl[:, k, :] @ lam[l]
            oe[:, q] -= de[:, k, :] @ lam[l]
    return ol, oe


def kappa_fd(oracle_cls, system, R, pair, h=1e-3):
    """Fourth-order central differences of ln|Psi| and E_L along one rotation
    parameter (the wave function rebuilt with the rotated orbitals)."""
    vals = {}
    for m in (-2, -1, 1, 2):
        sysd = dict(system)
        sysd["lam"] = rotate(system["lam"], [pair], [m * h]).tolist()
        ev = oracle_cls(sysd).evaluate(R)
        vals[m] = (ev["logabs"], ev["eloc"])
    d = [(8.0 * (vals[1][i] - vals[-1][i]) - (vals[2][i] - vals[-2][i])) / (12.0 * h) for i in (0, 1)]
    return d[0], d[1]


def redundant_keep(O, w=None, tol=1e-8):
    """Keep mask over the columns of the per-sample derivatives O [W][n],
    taken in order: a column is kept when its weighted, centred residual
    after least squares on the kept earlier columns has more than tol of its
    own centred sum of squares."""
    O = np.asarray(O, np.float64)
    W = O.shape[0]
    w = np.ones(W) if w is None else np.asarray(w, np.float64)
    sw = np.sqrt(w / w.sum())
    X = (O - (w @ O) / w.sum()) * sw[:, None]
    keep = np.zeros(O.shape[1], bool)
    for i in range(O.shape[1]):
        x = X[:, i]
        tot = x @ x
        if not tot > 0:
            continue
        B = X[:, keep]
        if B.shape[1]:
            coef, *_ = np.linalg.lstsq(B, x, rcond=None)
            r = x - B @ coef
        else:
            r = x
        keep[i] = (r @ r) > tol * tot
    return keep
