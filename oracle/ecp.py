"""Oracle of the pseudopotential part of the local energy -- TEST
INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU baseline
may use it; the library never does.  Plain numpy in FP64.

The paper runs its valence calculations with energy-consistent
pseudopotentials (Sec. 2.1, basis choice; the applications of Sec. 3) and
describes neither their form nor how their nonlocal part enters E_L = H Psi /
Psi.  This oracle takes the usual semilocal form of such potentials: per
pseudo-nucleus a with effective (valence) charge Z_a, which is the charge the
system lists for it,

    V_a = -Z_a / r + V_loc,a(r) + sum_{l < L_a} V_l,a(r) sum_m |l m><l m|,
    V(r) = sum_k c_k r^(n_k - 2) exp(-alpha_k r^2)   (each radial part),

and the projector of channel l acting on Psi for electron i at distance r
from a as the angular integral

    (2l + 1) / (4 pi) * int dOmega' P_l(cos theta') Psi(.., r_i', ..) / Psi(R),

r_i' on the sphere of radius r about a, theta' the angle between r_i - a and
r_i' - a, taken by the 12-point rule on the vertices of the icosahedron
(equal weights, exact for spherical harmonics up to degree 5), in a fixed
orientation.  The nonlocal part of a centre is applied only for r < r_cut of
that centre; the local part everywhere.  The -Z_a / r term is the ordinary
electron-nucleus attraction with the listed charge, already in the oracle's
E_L.

Every ratio Psi(R') / Psi(R) is a fresh evaluation of the moved
configuration (``Oracle.evaluate``), not an update formula.

Pins (tests/test_oracle_ecp.py): the rule's integrals of every monomial up
to degree 5 against their closed forms; the Legendre polynomials'
normalisation and orthogonality against Gauss-Legendre quadrature; E_L of
one electron in an s, p or d Gaussian (any orientation) at the centre in
closed form (kinetic + local + the matching channel, the others vanishing);
the cutoff; a two-electron product of an s and a p orbital (each electron
its own channel).
"""

import numpy as np


def ico_points():
    """The 12 unit vectors to the vertices of an icosahedron."""
    g = (1.0 + np.sqrt(5.0)) / 2.0
    v = []
    for s1 in (-1.0, 1.0):
        for s2 in (-1.0, 1.0):
            v += [(0.0, s1, s2 * g), (s1, s2 * g, 0.0), (s2 * g, 0.0, s1)]
    return np.array(v) / np.sqrt(1.0 + g * g)


def legendre(l, x):
    """P_l(x) for l = 0..3."""
    x = np.asarray(x, np.float64)
    if l == 0:
        return np.ones_like(x)
    if l == 1:
        return x
    if l == 2:
        return 0.5 * (3.0 * x * x - 1.0)
    if l == 3:
        return 0.5 * (5.0 * x ** 3 - 3.0 * x)
    raise ValueError("channels up to l = 3")


def radial(terms, r):
    """sum_k c_k r^(n_k - 2) exp(-alpha_k r^2) at distances r."""
    r = np.asarray(r, np.float64)
    out = np.zeros_like(r)
    for c, n, a in terms:
        out = out + c * r ** (int(n) - 2) * np.exp(-a * r * r)
    return out


def ecp_energy(oracle_obj, system, R):
    """The pseudopotential energy per configuration [W]: the local radial
    parts plus the projected nonlocal channels (the -Z/r part excluded)."""
    ecp = system.get("ecp") or []
    N = oracle_obj.N
    R = np.asarray(R, np.float64).reshape(-1, N, 3)
    W = R.shape[0]
    pos = np.asarray(system["nuclei"]["pos"], np.float64).reshape(-1, 3)
    u = ico_points()
    out = np.zeros(W)
    base = oracle_obj.evaluate(R, level=0)
    for w in range(W):
        moved, weights = [], []
        for cen in ecp:
            a = pos[cen["center"]]
            for i in range(N):
                d = R[w, i] - a
                r = np.sqrt(d @ d)
                out[w] += radial(cen["local"], r)
                if not r < cen["r_cut"] or not cen["channels"]:
                    continue
                cth = u @ (d / r)
                wq = np.zeros(len(u))
                for l, terms in enumerate(cen["channels"]):
                    wq += radial(terms, r) * (2 * l + 1) / len(u) * legendre(l, cth)
                for q in range(len(u)):
                    Rq = R[w].copy()
                    Rq[i] = a + r * u[q]
                    moved.append(Rq)
                    weights.append(wq[q])
        if moved:
            ev = oracle_obj.evaluate(np.array(moved), level=0)
            ratio = ev["sign"] * base["sign"][w] * np.exp(ev["logabs"] - base["logabs"][w])
            out[w] += float(np.dot(weights, ratio))
    return out


def evaluate(oracle_obj, system, R):
    """Oracle.evaluate with the pseudopotential energy added to E_L."""
    ev = oracle_obj.evaluate(R)
    ev["eloc"] = ev["eloc"] + ecp_energy(oracle_obj, system, R)
    return ev
