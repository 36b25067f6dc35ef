"""Pins of the CPU oracle to facts outside itself.

Each test checks the oracle against something the paper or the mathematics
fixes: closed-form local energies, finite differences, Leibniz determinants,
a brute-force spin-orbital antisymmetriser for Eq. (PhiI), invariances,
weight identities (Sec. 2.4), Euler homogeneity of the parameter
derivatives, and the published Philox known-answer vectors.
"""

import itertools
import json
import math
import os

import numpy as np
import pytest

import systems as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
CLOSED = json.load(open(os.path.join(GOLDEN, "closed_forms.json")))


# ---------------------------------------------------------------------------
# Philox
# ---------------------------------------------------------------------------

def test_philox_known_answers(oracle_mod):
    for line in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(x, 16) for x in line.split()]
        out = oracle_mod.philox4x32_10(v[0:4], v[4:6])
        assert out.tolist() == v[6:10]


def test_uniforms_are_uniform(oracle_mod):
    u = np.array([oracle_mod.uniforms(12345, w, 3, 7, 0) for w in range(20000)]).reshape(-1)
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 5 * math.sqrt(1 / 12 / u.size)
    assert abs(u.var() - 1 / 12) < 0.01
    h, _ = np.histogram(u, bins=20, range=(0, 1))
    chi2 = ((h - u.size / 20) ** 2 / (u.size / 20)).sum()
    assert chi2 < 60  # 19 dof


# ---------------------------------------------------------------------------
# basis functions against finite differences
# ---------------------------------------------------------------------------

def _fd_ao(o, r, h=1e-3):
    """4th-order central differences of the AO values."""
    g = np.zeros((3, o.M))
    lap = np.zeros(o.M)
    v0 = o.ao(r)[0]
    for x in range(3):
        e = np.zeros(3)
        e[x] = h
        vp1, vm1 = o.ao(r + e)[0], o.ao(r - e)[0]
        vp2, vm2 = o.ao(r + 2 * e)[0], o.ao(r - 2 * e)[0]
        g[x] = (-vp2 + 8 * vp1 - 8 * vm1 + vm2) / (12 * h)
        lap += (-vp2 + 16 * vp1 - 30 * v0 + 16 * vm1 - vm2) / (12 * h * h)
    return g, lap


@pytest.mark.parametrize("seed", [1, 2])
def test_ao_derivatives_match_finite_differences(oracle_mod, seed):
    sysd = S.small_random_system(seed, n_nuc=2)
    sysd["shells"].append({"center": 0, "kind": "sto", "l": 1, "exps": [0.9, 2.1], "coefs": [1.0, -0.3]})
    sysd["shells"].append({"center": 1, "kind": "sto", "l": 0, "exps": [1.3], "coefs": [0.7]})
    sysd["lam"] = np.zeros((len(sysd["lam"]), S.n_basis(sysd))).tolist()
    o = oracle_mod.Oracle(sysd)
    rng = np.random.default_rng(seed)
    for _ in range(4):
        r = rng.normal(size=3)
        a = o.ao(r)
        g, lap = _fd_ao(o, r)
        scale = np.abs(a).max(axis=0) + 1e-3
        np.testing.assert_array_less(np.abs(a[1:4] - g) / scale, 1e-7)
        np.testing.assert_array_less(np.abs(a[4] - lap) / scale, 1e-5)


def test_d_shell_polynomials_are_harmonic(oracle_mod):
    """For Gaussian shells the Laplacian equals P (2(2l+3) g' + 4 r^2 g'') because the
    angular set is harmonic (lap P = 0) and homogeneous of degree l."""
    sysd = S.small_random_system(5, n_nuc=1)
    o = oracle_mod.Oracle(sysd)
    r = np.array([0.3, -0.4, 0.55])
    a = o.ao(r)
    mu = 0
    A = np.asarray(sysd["nuclei"]["pos"][0])
    d = r - A
    r2 = d @ d
    for sh in sysd["shells"]:
        l = sh["l"]
        ex, cf = np.asarray(sh["exps"]), np.asarray(sh["coefs"])
        e = cf * np.exp(-ex * r2)
        g, g1, g2 = e.sum(), (-ex * e).sum(), (ex * ex * e).sum()
        nf = {0: 1, 1: 3, 2: 5}[l]
        for m in range(nf):
            P = a[0, mu + m] / g
            assert a[4, mu + m] == pytest.approx(P * (2 * (2 * l + 3) * g1 + 4 * r2 * g2), rel=1e-12, abs=1e-14)
        mu += nf


# ---------------------------------------------------------------------------
# closed-form local energies
# ---------------------------------------------------------------------------

def test_hydrogen_exact_orbital_zero_variance(oracle_mod):
    """H with exp(-r): H psi = -1/2 psi at every point, so E_L == -0.5 and Var(E_L) = 0."""
    o = oracle_mod.Oracle(S.hydrogen_sto_1s(1.0))
    R = np.random.default_rng(3).normal(scale=1.5, size=(200, 1, 3))
    e = o.evaluate(R)["eloc"]
    np.testing.assert_allclose(e, CLOSED["hydrogen_1s_sto_zeta1_eloc"], rtol=0, atol=1e-13)
    assert e.var() < 1e-26


def test_hydrogen_2p_exact(oracle_mod):
    """H with z exp(-r/2) is the 2p_z eigenfunction: E_L == -1/8."""
    o = oracle_mod.Oracle(S.hydrogen_sto_2p(0.5))
    R = np.random.default_rng(4).normal(scale=3.0, size=(100, 1, 3))
    np.testing.assert_allclose(o.evaluate(R)["eloc"], CLOSED["hydrogen_2p_sto_zeta_half_eloc"], atol=1e-12)


def test_hydrogen_gaussian_local_energy(oracle_mod):
    """psi = exp(-a r^2): -1/2 lap psi / psi = 3a - 2 a^2 r^2, so E_L = 3a - 2a^2 r^2 - 1/r."""
    a = 0.37
    o = oracle_mod.Oracle(S.hydrogen_gaussian(a))
    R = np.random.default_rng(5).normal(size=(50, 1, 3))
    r = np.linalg.norm(R[:, 0], axis=1)
    np.testing.assert_allclose(o.evaluate(R)["eloc"], 3 * a - 2 * a * a * r * r - 1 / r, rtol=1e-12)


def test_helium_product_forms(oracle_mod):
    """He, both electrons in one orbital: E_L sums the one-electron parts plus 1/r12."""
    rng = np.random.default_rng(6)
    R = rng.normal(size=(50, 2, 3))
    r1, r2 = np.linalg.norm(R[:, 0], axis=1), np.linalg.norm(R[:, 1], axis=1)
    r12 = np.linalg.norm(R[:, 0] - R[:, 1], axis=1)
    a = 0.8
    o = oracle_mod.Oracle(S.helium_gaussian(a))
    ref = (3 * a - 2 * a * a * r1 ** 2 - 2 / r1) + (3 * a - 2 * a * a * r2 ** 2 - 2 / r2) + 1 / r12
    np.testing.assert_allclose(o.evaluate(R)["eloc"], ref, rtol=1e-12)
    z = 1.6875
    o = oracle_mod.Oracle(S.helium_sto(z))
    ref = -z * z + (z - 2) / r1 + (z - 2) / r2 + 1 / r12
    np.testing.assert_allclose(o.evaluate(R)["eloc"], ref, rtol=1e-12)


def test_multicentre_potential(oracle_mod):
    """One Gaussian on nucleus A among three nuclei (no Jastrow).  The kinetic
    part is that of the one-centre Gaussian about A, so
    E_L = sum_i (3a - 2a^2 r_iA^2) - sum_i sum_alpha Z_alpha / r_i,alpha
          + sum_{i<j} 1/r_ij + sum_{alpha<beta} Z_alpha Z_beta / R_alpha,beta.
    Three unequal charges at unequal separations make a dropped, doubled or
    misassigned nucleus-nucleus pair, or an electron-nucleus term taken from
    the wrong centre, change the value."""
    a = 0.45
    Z = [3.0, 1.0, 2.0]
    pos = np.array([[0.2, -0.1, 0.3], [1.7, 0.4, -0.6], [-0.9, 2.1, 1.1]])
    Vnn = sum(Z[p] * Z[q] / np.linalg.norm(pos[p] - pos[q]) for p in range(3) for q in range(p + 1, 3))
    rng = np.random.default_rng(21)
    for n_up, n_dn in ((1, 0), (1, 1)):
        o = oracle_mod.Oracle(S.gaussian_multicentre(a, Z, pos, n_up, n_dn))
        R = pos[0] + rng.normal(scale=0.9, size=(60, n_up + n_dn, 3))
        ref = np.full(len(R), Vnn)
        for i in range(n_up + n_dn):
            rA2 = ((R[:, i] - pos[0]) ** 2).sum(1)
            ref += 3 * a - 2 * a * a * rA2
            for al in range(3):
                ref -= Z[al] / np.linalg.norm(R[:, i] - pos[al], axis=1)
        if n_dn:
            ref += 1 / np.linalg.norm(R[:, 0] - R[:, 1], axis=1)
        np.testing.assert_allclose(o.evaluate(R)["eloc"], ref, rtol=1e-12)


def test_jastrow_only_hydrogen(oracle_mod):
    """Constant orbital (Gaussian exponent 0) and e-n Pade A = -1, B = 0 with kappa = 0
    give Psi = exp(-r), the exact ground state: E_L == -0.5."""
    jas = {"kappa": 0.0, "ee": {"a_anti": 0.5, "a_par": 0.25, "b_anti": 1.0, "b_par": 1.0, "poly": [0, 0, 0, 0]},
           "en": [{"a1": -1.0, "a2": 0.0, "poly": [0, 0, 0, 0]}]}
    o = oracle_mod.Oracle(S.hydrogen_gaussian(0.0, jastrow=jas))
    R = np.random.default_rng(7).normal(scale=2.0, size=(100, 1, 3))
    np.testing.assert_allclose(o.evaluate(R)["eloc"], -0.5, atol=1e-13)


def test_two_electron_jastrow_formula(oracle_mod):
    """Psi = phi(r1) phi(r2) exp(u(r12)) with phi = exp(-a r^2) and u = A r / (1 + B r):
    E_L = sum_i (3a - 2a^2 r_i^2) - [u'' + 2u'/r + u'^2] - u' r12_hat . (grad ln phi(r1) - grad ln phi(r2)) + V."""
    a, A, B = 0.6, 0.5, 0.8
    jas = {"kappa": 0.0, "ee": {"a_anti": A, "a_par": 0.25, "b_anti": B, "b_par": B, "poly": [0, 0, 0, 0]},
           "en": [{"a1": 0.0, "a2": 0.0, "poly": [0, 0, 0, 0]}]}
    o = oracle_mod.Oracle(S.helium_gaussian(a, jastrow=jas))
    rng = np.random.default_rng(8)
    R = rng.normal(size=(40, 2, 3))
    r1v, r2v = R[:, 0], R[:, 1]
    d = r1v - r2v
    r = np.linalg.norm(d, axis=1)
    u1 = A / (1 + B * r) ** 2
    u2 = -2 * A * B / (1 + B * r) ** 3
    gl1, gl2 = -2 * a * r1v, -2 * a * r2v
    kin_orb = (3 * a - 2 * a * a * (r1v ** 2).sum(1)) + (3 * a - 2 * a * a * (r2v ** 2).sum(1))
    cross = u1 * ((d / r[:, None]) * (gl1 - gl2)).sum(1)
    V = -2 / np.linalg.norm(r1v, axis=1) - 2 / np.linalg.norm(r2v, axis=1) + 1 / r
    ref = kin_orb - (u2 + 2 * u1 / r + u1 ** 2) - cross + V
    np.testing.assert_allclose(o.evaluate(R)["eloc"], ref, rtol=1e-11)


def test_electron_electron_cusp(oracle_mod):
    """Antiparallel A = 1/2 cancels the 1/r12 divergence: r12 * E_L -> 0 as r12 -> 0."""
    jas = {"kappa": 0.0, "ee": {"a_anti": 0.5, "a_par": 0.25, "b_anti": 1.0, "b_par": 1.0, "poly": [0, 0, 0, 0]},
           "en": [{"a1": 0.0, "a2": 0.0, "poly": [0, 0, 0, 0]}]}
    o = oracle_mod.Oracle(S.helium_gaussian(0.7, jastrow=jas))
    base = np.array([0.4, -0.2, 0.3])
    vals = []
    for eps in (1e-3, 1e-5, 1e-7):
        R = np.array([[base, base + eps * np.array([0.6, 0.0, 0.8])]])
        vals.append(eps * o.evaluate(R)["eloc"][0])
    assert abs(vals[-1]) < 1e-5 and abs(vals[-1]) < abs(vals[0]) + 1e-12


# ---------------------------------------------------------------------------
# determinants
# ---------------------------------------------------------------------------

def _leibniz(A):
    n = A.shape[0]
    tot = 0.0
    for perm in itertools.permutations(range(n)):
        inv = sum(1 for i in range(n) for j in range(i + 1, n) if perm[i] > perm[j])
        tot += (-1) ** inv * np.prod([A[i, perm[i]] for i in range(n)])
    return tot


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_lu_determinant_matches_leibniz(oracle_mod, n):
    rng = np.random.default_rng(n)
    for _ in range(20):
        A = rng.normal(size=(n, n))
        la, sg, inv = oracle_mod.lu(A)
        det = _leibniz(A)
        assert sg * math.exp(la) == pytest.approx(det, rel=1e-13, abs=1e-15)
        np.testing.assert_allclose(inv, np.linalg.inv(A), rtol=1e-10, atol=1e-12)


def test_singular_determinant_detected(oracle_mod):
    A = np.array([[1.0, 2.0, 1.0], [3.0, 1.0, 3.0], [0.5, 0.2, 0.5]])  # equal columns 0 and 2
    la, sg, inv = oracle_mod.lu(A)
    assert la == -np.inf and sg == 0


def test_identical_orbitals_give_zero_structure(oracle_mod):
    """A structure whose up determinant holds one orbital twice contributes nothing."""
    sysd = S.small_random_system(11, n_active=3, n_pairs=1)
    base = oracle_mod.Oracle(sysd)
    bad = json.loads(json.dumps(sysd))
    bad["structures"].append({"c": 0.7, "terms": [{"inactive": [1], "pairs": [[1, 2]], "unpaired": []}]})
    o = oracle_mod.Oracle(bad)
    R = S.initial_walkers(sysd, 5, seed=2)
    a, b = base.evaluate(R), o.evaluate(R)
    np.testing.assert_allclose(a["logabs"], b["logabs"], rtol=1e-13)
    np.testing.assert_allclose(a["eloc"], b["eloc"], rtol=1e-11)
    np.testing.assert_allclose(b["ratio"][:, -1], 0.0, atol=0)


def test_antisymmetry_under_same_spin_swaps(oracle_mod):
    sysd = S.small_random_system(12, n_inactive=1, n_active=4, n_pairs=2, n_unpaired=1)
    o = oracle_mod.Oracle(sysd)
    R = S.initial_walkers(sysd, 6, seed=3)
    a = o.evaluate(R)
    for (i, j) in [(0, 1), (1, 3), (4, 6)]:  # up-up, up-up, down-down
        R2 = R.copy()
        R2[:, [i, j]] = R2[:, [j, i]]
        b = o.evaluate(R2)
        np.testing.assert_array_equal(b["sign"], -a["sign"])
        np.testing.assert_allclose(b["logabs"], a["logabs"], rtol=1e-12)
        np.testing.assert_allclose(b["eloc"], a["eloc"], rtol=1e-10)
        g = a["grad"].copy()
        g[:, [i, j]] = g[:, [j, i]]
        np.testing.assert_allclose(b["grad"], g, rtol=1e-10, atol=1e-12)


# ---------------------------------------------------------------------------
# Eq. (PhiI) against a brute-force spin-orbital antisymmetriser
# ---------------------------------------------------------------------------

def _brute_structure_values(sysd, o, R):
    """Expand each HLSP term literally into strings of spin-orbital creation operators
    (a pair (i,j) gives a+_{i up} a+_{j dn} - a+_{i dn} a+_{j up}; a self-pair gives both
    terms), and evaluate each string as the N x N spin-orbital Slater determinant at
    electrons with fixed spins (up for the first n_up).  Each term is divided by
    2^{number of self-pairs}: structures are unnormalised."""
    lam = np.asarray(sysd["lam"])
    N, nup = o.N, o.n_up
    phi = np.array([lam @ o.ao(R[i])[0] for i in range(N)])  # [electron][orbital]
    spins = [0] * nup + [1] * (N - nup)
    vals = []
    for st in sysd["structures"]:
        tot = 0.0
        for t in st["terms"]:
            base = []
            for p in t["inactive"]:
                base += [(p, 0), (p, 1)]
            strings = [(1.0, base)]
            for (i, j) in t["pairs"]:
                new = []
                for coef, sstr in strings:
                    new.append((coef, sstr + [(i, 0), (j, 1)]))
                    new.append((-coef, sstr + [(i, 1), (j, 0)]))
                strings = new
            strings = [(cf, s + [(q, 0) for q in t["unpaired"]]) for cf, s in strings]
            nself = sum(1 for (i, j) in t["pairs"] if i == j)
            for coef, sstr in strings:
                A = np.array([[phi[e, orb] if sp == spins[e] else 0.0 for (orb, sp) in sstr] for e in range(N)])
                tot += coef * np.linalg.det(A) / 2 ** nself
        vals.append(tot)
    return np.array(vals)


def _zero_jastrow(sysd):
    s = json.loads(json.dumps(sysd))
    for e in s["jastrow"]["en"]:
        e["a1"] = 0.0
        e["poly"] = [0, 0, 0, 0]
    s["jastrow"]["ee"]["a_anti"] = 0.0
    s["jastrow"]["ee"]["a_par"] = 0.0
    s["jastrow"]["ee"]["poly"] = [0, 0, 0, 0]
    return s


@pytest.mark.parametrize("seed,npairs,nunp", [(21, 1, 0), (22, 2, 1), (23, 2, 0)])
def test_hlsp_expansion_matches_antisymmetriser(oracle_mod, seed, npairs, nunp):
    sysd = _zero_jastrow(S.small_random_system(seed, n_inactive=1, n_active=5, n_pairs=npairs,
                                               n_unpaired=nunp, n_structures=4))
    o = oracle_mod.Oracle(sysd)
    R = S.initial_walkers(sysd, 4, seed=seed)
    ev = o.evaluate(R)
    ratios = []
    for w in range(R.shape[0]):
        brute = _brute_structure_values(sysd, o, R[w])
        D = ev["sign"][w] * math.exp(ev["logabs"][w])
        mine = ev["ratio"][w] * D
        ratios.append(brute / mine)
    ratios = np.array(ratios)
    # one constant for every structure and configuration (the operator-reordering sign)
    np.testing.assert_allclose(ratios, ratios[0, 0], rtol=1e-9)
    assert abs(abs(ratios[0, 0]) - 1.0) < 1e-9


def test_heitler_london_h2_formula(oracle_mod):
    """H2 system: Psi = e^U [0.9 (a1 b2 + b1 a2) + 0.3 (a1 a2 + b1 b2)], symmetric under r1 <-> r2."""
    sysd = _zero_jastrow(S.h2_heitler_london())
    o = oracle_mod.Oracle(sysd)
    lam = np.asarray(sysd["lam"])
    R = S.initial_walkers(sysd, 10, seed=1)
    ev = o.evaluate(R)
    for w in range(10):
        a1, b1 = lam @ o.ao(R[w, 0])[0]
        a2, b2 = lam @ o.ao(R[w, 1])[0]
        ref = 0.9 * (a1 * b2 + b1 * a2) + 0.3 * (a1 * a2 + b1 * b2)
        assert ev["sign"][w] * math.exp(ev["logabs"][w]) == pytest.approx(ref, rel=1e-12)
    ev2 = o.evaluate(R[:, ::-1])
    np.testing.assert_allclose(ev2["logabs"], ev["logabs"], rtol=1e-13)
    np.testing.assert_array_equal(ev2["sign"], ev["sign"])


# ---------------------------------------------------------------------------
# finite differences of ln Psi: gradient and kinetic energy
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["small", "h2"])
def test_gradient_and_laplacian_match_finite_differences(oracle_mod, name):
    sysd = S.small_random_system(31, n_inactive=1, n_active=4, n_pairs=2, n_unpaired=1) if name == "small" \
        else S.h2_heitler_london()
    o = oracle_mod.Oracle(sysd)
    R = S.initial_walkers(sysd, 3, seed=4)
    h = 1e-4
    for w in range(3):
        ev = o.evaluate(R[w:w + 1])
        N = o.N
        g = np.zeros((N, 3))
        lap = 0.0
        l0 = ev["logabs"][0]
        for i in range(N):
            for x in range(3):
                pts = []
                for k in (-2, -1, 1, 2):
                    Rk = R[w].copy()
                    Rk[i, x] += k * h
                    pts.append(Rk)
                lv = o.evaluate(np.array(pts), level=0)["logabs"]
                gi = (lv[0] - 8 * lv[1] + 8 * lv[2] - lv[3]) / (12 * h)
                li = (-lv[0] + 16 * lv[1] - 30 * l0 + 16 * lv[2] - lv[3]) / (12 * h * h)
                g[i, x] = gi
                lap += li + gi * gi
        np.testing.assert_allclose(ev["grad"][0], g, rtol=1e-6, atol=1e-6 * np.abs(g).max())
        kin_fd = -0.5 * lap
        assert ev["kin"][0] == pytest.approx(kin_fd, rel=2e-5, abs=2e-5)


# ---------------------------------------------------------------------------
# invariances
# ---------------------------------------------------------------------------

def test_translation_invariance(oracle_mod):
    sysd = S.small_random_system(41, n_inactive=1, n_active=3, n_pairs=1, n_unpaired=1)
    o = oracle_mod.Oracle(sysd)
    R = S.initial_walkers(sysd, 5, seed=5)
    shift = np.array([0.7, -1.3, 2.1])
    moved = json.loads(json.dumps(sysd))
    moved["nuclei"]["pos"] = (np.asarray(sysd["nuclei"]["pos"]) + shift).tolist()
    o2 = oracle_mod.Oracle(moved)
    a, b = o.evaluate(R), o2.evaluate(R + shift)
    np.testing.assert_allclose(b["logabs"], a["logabs"], rtol=1e-10)
    np.testing.assert_allclose(b["eloc"], a["eloc"], rtol=1e-9)
    np.testing.assert_allclose(b["grad"], a["grad"], rtol=1e-9, atol=1e-10)


def test_bovb_without_breathing_is_the_shared_orbital_function(oracle_mod):
    # Eq. PsiJBOVB with every structure's own active orbitals equal to the
    # shared ones is the VBSCF wave function of the same structures (a
    # mistake in the per-structure orbital bookkeeping breaks this); with
    # breathing the functions differ
    R = S.initial_walkers(S.f2_shaped(), 24, seed=31)
    a = oracle_mod.Oracle(S.f2_shaped()).evaluate(R)
    b = oracle_mod.Oracle(S.f2_bovb(breathing=0.0)).evaluate(R)
    np.testing.assert_allclose(b["logabs"], a["logabs"], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(b["eloc"], a["eloc"], rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(b["grad"], a["grad"], rtol=1e-10, atol=1e-11)
    np.testing.assert_allclose(b["ratio"], a["ratio"], rtol=1e-10, atol=1e-12)
    c = oracle_mod.Oracle(S.f2_bovb()).evaluate(R)
    assert np.max(np.abs(c["logabs"] - a["logabs"])) > 1e-3


def test_coefficient_scaling_invariance(oracle_mod):
    sysd = S.small_random_system(42)
    o = oracle_mod.Oracle(sysd)
    sc = json.loads(json.dumps(sysd))
    for st in sc["structures"]:
        st["c"] *= 3.5
    o2 = oracle_mod.Oracle(sc)
    R = S.initial_walkers(sysd, 5, seed=6)
    a, b = o.evaluate(R), o2.evaluate(R)
    np.testing.assert_allclose(b["logabs"] - a["logabs"], math.log(3.5), rtol=1e-12)
    np.testing.assert_allclose(b["eloc"], a["eloc"], rtol=1e-12)
    np.testing.assert_allclose(b["grad"], a["grad"], rtol=1e-12, atol=1e-14)


# ---------------------------------------------------------------------------
# structure weights (Sec. 2.4)
# ---------------------------------------------------------------------------

def test_weights_sum_to_one(oracle_mod):
    sysd = S.small_random_system(51, n_structures=4)
    o = oracle_mod.Oracle(sysd)
    R = S.initial_walkers(sysd, 50, seed=7)
    ev = o.evaluate(R)
    r = ev["ratio"]
    c = o.c
    # per configuration sum_I c_I r_I = 1, hence sum_IJ c_I c_J r_I r_J = 1
    np.testing.assert_allclose(r @ c, 1.0, rtol=1e-12)
    Smat = np.einsum("wi,wj->ij", r, r) / len(r)
    assert c @ Smat @ c == pytest.approx(1.0, rel=1e-12)
    assert oracle_mod.weights_chirgwin_coulson(Smat, c).sum() == pytest.approx(1.0, rel=1e-12)
    assert oracle_mod.weights_lowdin(Smat, c).sum() == pytest.approx(1.0, rel=1e-12)
    np.testing.assert_allclose(oracle_mod.weights_chirgwin_coulson([[2.0]], [0.3]), [1.0])
    np.testing.assert_allclose(oracle_mod.weights_lowdin([[2.0]], [0.3]), [1.0])


def test_lowdin_orthonormal_limit(oracle_mod):
    """For orthonormal structures (S = I) both weights reduce to c_I^2 / sum c^2."""
    c = np.array([0.3, -0.5, 0.8])
    ref = c * c / (c * c).sum()
    np.testing.assert_allclose(oracle_mod.weights_chirgwin_coulson(np.eye(3), c), ref, rtol=1e-14)
    np.testing.assert_allclose(oracle_mod.weights_lowdin(np.eye(3), c), ref, rtol=1e-14)


# ---------------------------------------------------------------------------
# parameter derivatives (Sec. 2.2)
# ---------------------------------------------------------------------------

def test_parameter_derivatives_identities(oracle_mod):
    sysd = S.small_random_system(61, n_inactive=2, n_active=4, n_pairs=1, n_unpaired=1, n_structures=4)
    o = oracle_mod.Oracle(sysd)
    R = S.initial_walkers(sysd, 3, seed=8)
    dl, de = o.param_deriv(R)
    cs, ls, js = o.param_slices()
    ev = o.evaluate(R)
    # d lnPsi / d c_I = r_I; Euler: sum_I c_I d lnPsi/dc_I = 1, sum_I c_I dE_L/dc_I = 0
    np.testing.assert_allclose(dl[:, cs], ev["ratio"], rtol=1e-12)
    np.testing.assert_allclose(dl[:, cs] @ o.c, 1.0, rtol=1e-12)
    np.testing.assert_allclose(de[:, cs] @ o.c, 0.0, atol=1e-9 * np.abs(de[:, cs]).max())
    # inactive orbital p (doubly occupied in every determinant): homogeneous of degree 2
    lam = o.lam
    dlam_l = dl[:, ls].reshape(-1, o.n_orb, o.M)
    dlam_e = de[:, ls].reshape(-1, o.n_orb, o.M)
    for p in range(2):
        np.testing.assert_allclose((dlam_l[:, p] * lam[p]).sum(1), 2.0, rtol=1e-11)
        np.testing.assert_allclose((dlam_e[:, p] * lam[p]).sum(1), 0.0, atol=1e-8 * np.abs(dlam_e).max())
    # linear Jastrow coefficient b3 multiplies sum_{i<j} R(r_ij)^2
    kappa = sysd["jastrow"]["kappa"]
    for w in range(3):
        Rw = R[w]
        tot = 0.0
        for i in range(o.N):
            for j in range(i + 1, o.N):
                r = np.linalg.norm(Rw[i] - Rw[j])
                tot += (r / (1 + kappa * r)) ** 2
        assert dl[w, js][2] == pytest.approx(tot, rel=1e-12)


def test_parameter_derivatives_match_central_differences(oracle_mod):
    sysd = S.small_random_system(62, n_inactive=1, n_active=3, n_pairs=1, n_unpaired=0, n_structures=3)
    o = oracle_mod.Oracle(sysd)
    R = S.initial_walkers(sysd, 2, seed=9)
    dl, de = o.param_deriv(R)
    h = 1e-5
    cs, ls, js = o.param_slices()

    def with_param(k, delta):
        s = json.loads(json.dumps(sysd))
        if k < cs.stop:
            s["structures"][k]["c"] += delta
        elif k < ls.stop:
            q = k - ls.start
            s["lam"][q // o.M][q % o.M] += delta
        else:
            q = k - js.start
            ee = s["jastrow"]["ee"]
            if q == 0:
                ee["b_anti"] += delta
            elif q == 1:
                ee["b_par"] += delta
            elif q < 6:
                ee["poly"][q - 2] += delta
            else:
                a, m = divmod(q - 6, 6)
                en = s["jastrow"]["en"][a]
                if m == 0:
                    en["a1"] += delta
                elif m == 1:
                    en["a2"] += delta
                else:
                    en["poly"][m - 2] += delta
        return oracle_mod.Oracle(s).evaluate(R)

    rng = np.random.default_rng(0)
    ks = list(range(cs.stop)) + rng.choice(np.arange(ls.start, ls.stop), 12, replace=False).tolist() + \
        list(range(js.start, js.stop))
    for k in ks:
        p, m = with_param(k, h), with_param(k, -h)
        fl = (p["logabs"] - m["logabs"]) / (2 * h)
        fe = (p["eloc"] - m["eloc"]) / (2 * h)
        np.testing.assert_allclose(dl[:, k], fl, rtol=1e-6, atol=1e-6 * max(1.0, np.abs(dl).max()))
        np.testing.assert_allclose(de[:, k], fe, rtol=1e-6, atol=1e-5 * max(1.0, np.abs(de).max()))
