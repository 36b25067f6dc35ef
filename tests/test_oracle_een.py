"""Pins of the oracle's three-body Jastrow term f_een (Sec. 2.1).

* The term list: every (k, l, m) the paper's rule admits (p = k + l + 2m from
  2 to 5, k < p, l up to p - k, or p - k - 2 when k = 0), enumerated here
  independently and in the order p, k, l: 23 terms.
* Values: for two electrons and one nucleus each coefficient alone changes
  ln|Psi| by c Rbar_12^k (Rbar_1^l + Rbar_2^l) (Rbar_1 Rbar_2)^m with
  Rbar(r) = 1 / (1 + kappa r), written out here in numpy.
* Structure of the sums: the f_een of three electrons is the sum of the f_een
  of its three pairs, each with both nuclei.
* Derivatives: the gradient and kinetic energy of a system with f_een against
  finite differences of ln|Psi|, and the derivatives with respect to the f_een
  coefficients against central differences of ln|Psi| and E_L.
"""

import json

import numpy as np
import pytest

import systems as S


def _terms_by_rule():
    out = []
    for p in range(2, 6):
        for k in range(p):
            lmax = p - k if k > 0 else p - k - 2
            for l in range(lmax + 1):
                if (p - k - l) % 2 == 0:
                    out.append((k, l, (p - k - l) // 2))
    return out


def test_term_list(oracle_mod):
    t = oracle_mod.een_terms()
    assert t == _terms_by_rule()
    assert len(t) == 23 == S.N_EEN_TERMS
    # every term has k > 0 or m > 0: none survives one electron far away
    assert all(k > 0 or m > 0 for k, l, m in t)
    assert len(set(t)) == 23


def _helium_een(coefs, kappa=0.8):
    jas = {"kappa": kappa,
           "ee": {"a_anti": 0.0, "a_par": 0.0, "b_anti": 0.0, "b_par": 0.0, "poly": [0.0] * 4},
           "en": [{"a1": 0.0, "a2": 0.0, "poly": [0.0] * 4}],
           "een": [list(coefs)]}
    return S.helium_gaussian(0.7, jastrow=jas)


def test_single_term_values(oracle_mod):
    R = np.array([[[0.3, -0.4, 0.9], [-1.1, 0.5, 0.2]], [[0.05, 0.1, -0.2], [2.5, 1.0, -0.7]]])
    kappa = 0.8
    base = oracle_mod.Oracle(_helium_een([0.0] * 23, kappa)).evaluate(R)["logabs"]
    rb = lambda r: 1.0 / (1.0 + kappa * r)  # noqa: E731
    for t, (k, l, m) in enumerate(_terms_by_rule()):
        c = np.zeros(23)
        c[t] = 0.37
        got = oracle_mod.Oracle(_helium_een(c, kappa)).evaluate(R)["logabs"] - base
        for w in range(len(R)):
            a = rb(np.linalg.norm(R[w, 0] - R[w, 1]))
            b, d = rb(np.linalg.norm(R[w, 0])), rb(np.linalg.norm(R[w, 1]))
            ref = 0.37 * a ** k * (b ** l + d ** l) * (b * d) ** m
            assert got[w] == pytest.approx(ref, rel=1e-12, abs=1e-15), (t, w)


def test_sum_over_pairs_and_nuclei(oracle_mod):
    """Three electrons (2 up, 1 down) near two nuclei of different elements:
    f_een is the sum of the f_een of the three electron pairs, each taken
    alone with both nuclei (the ln|Psi| difference with and without f_een;
    the coefficients do not depend on spin)."""
    rng = np.random.default_rng(3)
    een = [rng.normal(size=23).tolist(), rng.normal(size=23).tolist()]
    zero_en = {"a1": 0.0, "a2": 0.0, "poly": [0.0] * 4}
    jas = {"kappa": 0.8, "ee": {"a_anti": 0.0, "a_par": 0.0, "b_anti": 0.0, "b_par": 0.0, "poly": [0.0] * 4},
           "en": [zero_en, zero_en]}
    shells = [{"center": 0, "kind": "gto", "l": 0, "exps": [0.5], "coefs": [1.0]},
              {"center": 1, "kind": "gto", "l": 0, "exps": [0.6], "coefs": [1.0]}]

    def u_een(n_up, n_dn, term, R):
        out = []
        for j in (dict(jas, een=een), jas):
            s = {"name": "two_centre", "seed": 0,
                 "nuclei": {"Z": [1.0, 2.0], "pos": [[0, 0, -0.7], [0, 0, 0.7]]},
                 "n_up": n_up, "n_dn": n_dn, "shells": shells, "lam": [[1.0, 0.0], [0.0, 1.0]],
                 "structures": [{"c": 1.0, "terms": [term]}], "jastrow": j}
            out.append(oracle_mod.Oracle(s).evaluate(R, level=0)["logabs"])
        return out[0] - out[1]

    R = np.array([[[0.2, 0.1, -0.5], [1.1, -0.6, 0.9], [-0.3, 0.4, 0.6]]])
    u3 = u_een(2, 1, {"inactive": [0], "pairs": [], "unpaired": [1]}, R)
    u01 = u_een(2, 0, {"inactive": [], "pairs": [], "unpaired": [0, 1]}, R[:, [0, 1]])
    u02 = u_een(1, 1, {"inactive": [0], "pairs": [], "unpaired": []}, R[:, [0, 2]])
    u12 = u_een(1, 1, {"inactive": [0], "pairs": [], "unpaired": []}, R[:, [1, 2]])
    assert min(abs(u01[0]), abs(u02[0]), abs(u12[0])) > 1e-3
    assert u3[0] == pytest.approx(u01[0] + u02[0] + u12[0], rel=1e-12)


def _fd_check(o, R, h=1e-4):
    ev = o.evaluate(R)
    N = o.N
    g = np.zeros((N, 3))
    lap = 0.0
    l0 = ev["logabs"][0]
    for i in range(N):
        for x in range(3):
            pts = []
            for k in (-2, -1, 1, 2):
                Rk = R[0].copy()
                Rk[i, x] += k * h
                pts.append(Rk)
            lv = o.evaluate(np.array(pts), level=0)["logabs"]
            gi = (lv[0] - 8 * lv[1] + 8 * lv[2] - lv[3]) / (12 * h)
            li = (-lv[0] + 16 * lv[1] - 30 * l0 + 16 * lv[2] - lv[3]) / (12 * h * h)
            g[i, x] = gi
            lap += li + gi * gi
    return ev, g, -0.5 * lap


@pytest.mark.parametrize("name", ["small", "h2"])
def test_gradient_and_kinetic_energy_match_finite_differences(oracle_mod, name):
    # (soft basis sets: fourth-order differences at h = 1e-4 are accurate to
    # about 1e-6 there, unlike on the F2 basis with exponents up to 1e4)
    sysd = S.with_een(S.small_random_system(31, n_inactive=1, n_active=4, n_pairs=2, n_unpaired=1), scale=0.3) \
        if name == "small" else S.with_een(S.h2_heitler_london(), scale=0.3)
    o = oracle_mod.Oracle(sysd)
    R = S.initial_walkers(sysd, 2, seed=4)
    for w in range(2):
        ev, g, kin = _fd_check(o, R[w:w + 1])
        np.testing.assert_allclose(ev["grad"][0], g, rtol=1e-6, atol=1e-6 * np.abs(g).max())
        assert ev["kin"][0] == pytest.approx(kin, rel=2e-5, abs=2e-5 * max(1.0, abs(kin)))


def test_een_parameter_derivatives_match_central_differences(oracle_mod):
    sysd = S.with_een(S.small_random_system(62, n_inactive=1, n_active=3, n_pairs=1, n_unpaired=0,
                                            n_structures=3), scale=0.3)
    o = oracle_mod.Oracle(sysd)
    R = S.initial_walkers(sysd, 2, seed=9)
    _, _, js = o.param_slices()
    e0 = js.start + 6 + 6 * o.n_nuc
    assert js.stop - e0 == 23 * o.n_nuc
    idx = np.arange(e0, js.stop)
    dl, de = o.param_deriv(R, idx)
    h = 1e-5
    for q, k in enumerate(idx):
        a, t = divmod(k - e0, 23)

        def shifted(delta):
            s = json.loads(json.dumps(sysd))
            s["jastrow"]["een"][a][t] += delta
            return oracle_mod.Oracle(s).evaluate(R)

        p, m = shifted(h), shifted(-h)
        np.testing.assert_allclose(dl[:, q], (p["logabs"] - m["logabs"]) / (2 * h), rtol=1e-6, atol=1e-8)
        np.testing.assert_allclose(de[:, q], (p["eloc"] - m["eloc"]) / (2 * h), rtol=1e-5,
                                   atol=1e-5 * max(1.0, np.abs(de).max()))
