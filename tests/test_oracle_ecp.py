"""Pseudopotential term of the local energy (Sec. 2.1, basis choice: the
valence calculations with energy-consistent pseudopotentials): the oracle
(oracle/ecp.py) pinned to closed forms.  The angular rule against the exact
sphere integrals of monomials, the Legendre polynomials against
Gauss-Legendre quadrature, and E_L of one electron in an s, p or d Gaussian
at the pseudo-nucleus, where the projectors act exactly: the channel of the
orbital's l contributes V_l(r), every other channel nothing."""

import math

import numpy as np
import pytest

import systems as S
from oracle import ecp as ECP


def _sphere_mean(a, b, c):
    """(1/4pi) int x^a y^b z^c dOmega."""
    if a % 2 or b % 2 or c % 2:
        return 0.0
    df = lambda k: math.prod(range(k, 0, -2)) if k > 0 else 1  # noqa: E731
    return df(a - 1) * df(b - 1) * df(c - 1) / df(a + b + c + 1)


def test_rule_integrates_monomials_to_degree_five():
    u = ECP.ico_points()
    np.testing.assert_allclose(np.linalg.norm(u, axis=1), 1.0, rtol=0, atol=1e-15)
    for a in range(6):
        for b in range(6 - a):
            for c in range(6 - a - b):
                got = np.mean(u[:, 0] ** a * u[:, 1] ** b * u[:, 2] ** c)
                assert abs(got - _sphere_mean(a, b, c)) < 1e-15, (a, b, c)
    # and not beyond: x^6 is off
    assert abs(np.mean(u[:, 0] ** 6) - _sphere_mean(6, 0, 0)) > 1e-3


def test_legendre_normalisation_and_orthogonality():
    x, w = np.polynomial.legendre.leggauss(16)
    for l in range(4):
        assert ECP.legendre(l, np.array(1.0)) == 1.0
        for k in range(4):
            got = np.sum(w * ECP.legendre(l, x) * ECP.legendre(k, x))
            assert abs(got - (2.0 / (2 * l + 1) if k == l else 0.0)) < 1e-14


def _closed_form(sysd, R, l, alpha):
    """E_L of one electron in r^l Y_l exp(-alpha r^2) at the centre:
    (2l + 3) alpha - 2 alpha^2 r^2 - Z/r + V_loc(r) + V_l(r)."""
    r = np.linalg.norm(R[:, 0, :], axis=1)
    cen = sysd["ecp"][0]
    z = sysd["nuclei"]["Z"][0]
    e = (2 * l + 3) * alpha - 2 * alpha ** 2 * r ** 2 - z / r + ECP.radial(cen["local"], r)
    near = r < cen["r_cut"]
    return e + np.where(near, ECP.radial(cen["channels"][l], r), 0.0)


@pytest.mark.parametrize("native", [False, True])
@pytest.mark.parametrize("l,lam", [(0, [1.0]), (1, [0.0, 0.0, 1.0]), (1, [0.3, -0.5, 0.8]),
                                   (2, [1.0, 0.0, 0.0, 0.0, 0.0]), (2, [0.2, -0.7, 0.4, 0.5, -0.3])])
def test_one_electron_channels_in_closed_form(oracle_mod, l, lam, native):
    """Both implementations of the oracle: numpy (oracle.ecp) and the C++
    oracle's own (native_ecp, used by its VMC and DMC loops)."""
    alpha = 0.7
    sysd = S.ecp_one_centre(l, lam, alpha)
    rng = np.random.default_rng(10 + l)
    d = rng.normal(size=(40, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    R = (d * rng.uniform(0.05, 3.5, size=(40, 1)))[:, None, :]  # both sides of r_cut = 2.5
    if native:
        got = oracle_mod.Oracle(sysd, native_ecp=True).evaluate(R)["eloc"]
    else:
        got = ECP.evaluate(oracle_mod.Oracle(sysd), sysd, R)["eloc"]
    want = _closed_form(sysd, R, l, alpha)
    err = np.abs(got - want) / np.maximum(1.0, np.abs(want))
    assert err.max() < 1e-10, err.max()


def test_two_electron_product_takes_each_electrons_channel(oracle_mod):
    """A singlet pair of an s and a p orbital at the centre, no Jastrow:
    Psi = phi_p(r1) phi_s(r2) + phi_s(r1) phi_p(r2), so the nonlocal part is
    [(V_1(r1) + V_0(r2)) t1 + (V_0(r1) + V_1(r2)) t2] / Psi, each electron
    projected on its own factor of each term."""
    sysd = S.ecp_one_centre(0, [1.0], 0.7)
    sysd["shells"] = [{"center": 0, "kind": "gto", "l": 0, "exps": [0.7], "coefs": [1.0]},
                      {"center": 0, "kind": "gto", "l": 1, "exps": [0.4], "coefs": [1.0]}]
    sysd["lam"] = [[1.0, 0.0, 0.0, 0.0], [0.0, 0.6, 0.0, -0.8]]
    sysd["n_up"], sysd["n_dn"] = 1, 1
    sysd["structures"] = [{"c": 1.0, "terms": [{"inactive": [], "pairs": [[1, 0]], "unpaired": []}]}]
    sysd["nuclei"]["Z"] = [2.0]
    o = oracle_mod.Oracle(sysd)
    rng = np.random.default_rng(3)
    R = rng.normal(size=(25, 2, 3))
    got = ECP.ecp_energy(o, sysd, R)
    cen = sysd["ecp"][0]
    r = np.linalg.norm(R, axis=2)
    want = ECP.radial(cen["local"], r[:, 0]) + ECP.radial(cen["local"], r[:, 1])
    # the singlet pair puts the p orbital on the up electron in one term and
    # on the down electron in the other; each factor is pure l = 0 or l = 1
    # about the centre, so each electron's projector acts term by term
    p = lambda x: 0.6 * x[..., 0] - 0.8 * x[..., 2]  # noqa: E731
    s = lambda x: np.ones(x.shape[:-1])  # noqa: E731
    g = lambda x, a: np.exp(-a * np.sum(x * x, axis=-1))  # noqa: E731
    psi = lambda X: p(X[:, 0]) * g(X[:, 0], 0.4) * g(X[:, 1], 0.7) + g(X[:, 0], 0.7) * p(X[:, 1]) * g(X[:, 1], 0.4)  # noqa: E731
    V0 = [ECP.radial(cen["channels"][0], r[:, i]) * (r[:, i] < cen["r_cut"]) for i in range(2)]
    V1 = [ECP.radial(cen["channels"][1], r[:, i]) * (r[:, i] < cen["r_cut"]) for i in range(2)]
    t1 = p(R[:, 0]) * g(R[:, 0], 0.4) * g(R[:, 1], 0.7)
    t2 = g(R[:, 0], 0.7) * p(R[:, 1]) * g(R[:, 1], 0.4)
    want = want + ((V1[0] + V0[1]) * t1 + (V0[0] + V1[1]) * t2) / psi(R)
    err = np.abs(got - want) / np.maximum(1.0, np.abs(want))
    assert err.max() < 1e-10, err.max()


def test_f2_valence_system_is_consistent(oracle_mod):
    """The F2 valence system: finite E_L, and the nonlocal part vanishes once
    every electron is beyond r_cut of both centres."""
    sysd = S.f2_valence_ecp()
    o = oracle_mod.Oracle(sysd)
    R = S.initial_walkers(sysd, 3, seed=5)
    ev = ECP.evaluate(o, sysd, R)
    assert np.all(np.isfinite(ev["eloc"]))
    far = sysd.copy()
    far["ecp"] = [dict(c, channels=[]) for c in sysd["ecp"]]
    Rf = R + np.array([0.0, 9.0, 0.0])
    np.testing.assert_allclose(ECP.ecp_energy(o, sysd, Rf), ECP.ecp_energy(o, far, Rf), rtol=0, atol=1e-15)


def test_native_term_matches_numpy_on_f2_valence(oracle_mod):
    """The C++ oracle's term (native_ecp) against oracle.ecp on the
    many-electron system, where no closed form exists."""
    sysd = S.f2_valence_ecp()
    R = S.initial_walkers(sysd, 4, seed=6, sigma=1.2)
    a = oracle_mod.Oracle(sysd, native_ecp=True).evaluate(R)["eloc"]
    b = ECP.evaluate(oracle_mod.Oracle(sysd), sysd, R)["eloc"]
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-12)
