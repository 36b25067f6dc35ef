"""Orbital-rotation parameters (Sec. 2.2, Eq. PsiJVBp and the orbital classes
that follow it): the oracle (oracle/rotations.py) pinned to hand-enumerated
pair lists, to brute-force derivatives and to finite differences of the
rotated wave function, and the library's host-only entry points
(vbqmc_rotation_pairs, vbqmc_orbital_classes, vbqmc_rotate_orbitals,
vbqmc_lm_redundant) against it.  No GPU: the library is loaded for its host
functions only."""

import numpy as np
import pytest

import systems as S
from oracle import rotations as ROT


def _lib():
    import paper_2207_14715_amd as vb
    try:
        vb.load_library()
    except (OSError, RuntimeError) as e:
        pytest.skip(f"library not loadable here: {e}")
    return vb


def _h2_virtual():
    """H2 Heitler-London plus a third orbital that no structure occupies."""
    sysd = S.h2_heitler_london()
    lam = np.asarray(sysd["lam"])
    extra = np.zeros((1, lam.shape[1]))
    extra[0, 1] = 0.7
    extra[0, 4] = -0.4
    return dict(sysd, name="h2_virtual", lam=np.vstack([lam, extra]).tolist())


def _small(seed):
    return S.small_random_system(seed, n_inactive=2, n_active=5, n_pairs=2, n_unpaired=1, n_structures=4)


SYSTEMS = {"h2": S.h2_heitler_london, "h2_virtual": _h2_virtual, "f2": S.f2_shaped, "f2_bovb": S.f2_bovb,
           "small": lambda: _small(102), "small2": lambda: _small(7), "adjoint": S.adjoint_molecule}


# ---------------------------------------------------------------------------
# pins of the oracle
# ---------------------------------------------------------------------------

def test_hand_enumerated_pairs(oracle_mod):
    """The rules applied by hand.  H2: orbitals a, b active, both directions
    act (two independent parameters).  H2 + virtual c: a, b -> c with
    kappa_lk = -kappa_kl.  F2: 8 inactive orbitals -> the two active sigma
    orbitals (kind 1), the two active ones to each other (kind 0); with the
    localization classes of the basis blocks (orbitals 0-3, 8 on atom A,
    4-7, 9 on B) only inactive -> active on the same atom remain."""
    occ = ROT.occupancy(oracle_mod.Oracle(S.h2_heitler_london()))
    np.testing.assert_array_equal(ROT.pairs(occ), [[1, 0, 0], [0, 1, 0]])
    occ = ROT.occupancy(oracle_mod.Oracle(_h2_virtual()))
    np.testing.assert_array_equal(ROT.orbital_kinds(occ), [ROT.ACTIVE, ROT.ACTIVE, ROT.VIRTUAL])
    np.testing.assert_array_equal(ROT.pairs(occ), [[1, 0, 0], [2, 0, 1], [0, 1, 0], [2, 1, 1]])
    f2 = S.f2_shaped()
    occ = ROT.occupancy(oracle_mod.Oracle(f2))
    kinds = ROT.orbital_kinds(occ)
    np.testing.assert_array_equal(kinds, [ROT.INACTIVE] * 8 + [ROT.ACTIVE] * 2)
    want = [[k, l, 1] for l in range(8) for k in (8, 9)] + [[9, 8, 0], [8, 9, 0]]
    np.testing.assert_array_equal(ROT.pairs(occ), want)
    cls = ROT.classes_from_support(f2["lam"])
    np.testing.assert_array_equal(cls, [0, 0, 0, 0, 4, 4, 4, 4, 0, 4])
    want = [[8, l, 1] for l in range(4)] + [[9, l, 1] for l in range(4, 8)]
    np.testing.assert_array_equal(ROT.pairs(occ, cls), want)


@pytest.mark.parametrize("name", ["h2_virtual", "f2", "small"])
def test_pairs_are_the_excitations_with_a_derivative(oracle_mod, name):
    """Brute force over every ordered orbital pair: the derivative of ln|Psi|
    along E_kl (orbital l gains phi_k), from the oracle's dual numbers, is
    nonzero at some sampled configuration exactly for the listed directions
    (both directions of a kind-0 pair, the listed direction of a kind-1
    pair)."""
    sysd = SYSTEMS[name]()
    o = oracle_mod.Oracle(sysd)
    R = S.initial_walkers(sysd, 6, seed=41)
    n = o.n_orb
    every = np.array([[k, l, 0] for l in range(n) for k in range(n) if k != l], np.int32)
    dl, _ = ROT.kappa_deriv(o, R, every)
    scale = np.abs(dl).max()
    acting = {(int(k), int(l)) for (k, l, _), col in zip(every, dl.T) if np.abs(col).max() > 1e-9 * scale}
    listed = ROT.pairs(ROT.occupancy(o))
    want = {(int(k), int(l)) for k, l, _ in listed}
    assert acting == want, (sorted(acting - want), sorted(want - acting))
    for k, l, kind in listed:
        assert ((int(l), int(k)) in acting) == (kind == 0)


@pytest.mark.parametrize("name,pair", [("f2", (8, 0, 1)), ("f2", (9, 8, 0)), ("h2_virtual", (2, 1, 1)),
                                       ("small", None)])
def test_derivative_matches_the_rotated_wave_function(oracle_mod, name, pair):
    """d/d kappa from the linear map of the orbital-coefficient duals against
    fourth-order central differences of ln|Psi| and E_L of the wave function
    rebuilt with exp(kappa)-rotated orbitals (scipy's expm)."""
    sysd = SYSTEMS[name]()
    o = oracle_mod.Oracle(sysd)
    if pair is None:
        pair = tuple(ROT.pairs(ROT.occupancy(o))[-1])
    R = S.initial_walkers(sysd, 4, seed=3)
    dl, de = ROT.kappa_deriv(o, R, [pair])
    fl, fe = ROT.kappa_fd(oracle_mod.Oracle, sysd, R, pair, h=1e-3)
    ev = o.evaluate(R)
    np.testing.assert_allclose(dl[:, 0], fl, rtol=0, atol=1e-7 * max(1.0, np.abs(fl).max()))
    tol = 1e-6 * np.maximum(1.0, np.abs(ev["eloc"]))
    assert np.all(np.abs(de[:, 0] - fe) <= tol), (de[:, 0], fe)


def test_redundancy_of_the_heitler_london_function(oracle_mod):
    """H2 with covalent (a, b) and ionic aa + bb structures: E_ab Psi + E_ba Psi
    = 2 c_cov Phi_ion + 2 c_ion Phi_cov, and sum_I c_I d lnPsi / d c_I = 1, so
    in the order [c_cov, c_ion, kappa(b <- a), kappa(a <- b)] the second
    coefficient and the second rotation are redundant."""
    sysd = S.h2_heitler_london()
    o = oracle_mod.Oracle(sysd)
    R = S.initial_walkers(sysd, 300, seed=9, sigma=1.0)
    prs = ROT.pairs(ROT.occupancy(o))
    cs, _, _ = o.param_slices()
    oc, _ = o.param_deriv(R, np.arange(cs.start, cs.stop))
    ok, _ = ROT.kappa_deriv(o, R, prs)
    c = np.asarray([s["c"] for s in sysd["structures"]])
    # the two linear relations themselves, at every configuration
    np.testing.assert_allclose(oc @ c, 1.0, rtol=0, atol=1e-12)
    np.testing.assert_allclose(ok[:, 0] + ok[:, 1], 2 * c[0] * oc[:, 1] + 2 * c[1] * oc[:, 0], rtol=0,
                               atol=1e-10 * np.abs(ok).max())
    O = np.hstack([oc, ok])
    want = [True, False, True, False]
    np.testing.assert_array_equal(ROT.redundant_keep(O), want)
    vb = _lib()
    s_bar = np.cov(O, rowvar=False, bias=True)
    np.testing.assert_array_equal(vb.lm_redundant(s_bar), want)


# ---------------------------------------------------------------------------
# the library's host functions against the oracle
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name", sorted(SYSTEMS))
def test_library_pairs_and_classes_match_oracle(oracle_mod, name):
    vb = _lib()
    sysd = SYSTEMS[name]()
    o = oracle_mod.Oracle(sysd)
    occ = ROT.occupancy(o)
    cls = ROT.classes_from_support(sysd["lam"])
    np.testing.assert_array_equal(vb.orbital_classes(np.asarray(sysd["lam"])), cls)
    for lc in (None, cls):
        got = vb.rotation_pairs(occ, lc)
        want = ROT.pairs(occ, lc)
        np.testing.assert_array_equal(got, want)


def test_library_rotation_matches_expm():
    """vbqmc_rotate_orbitals against scipy's expm, for generators from small
    to large norm (several squarings) and both pair kinds."""
    vb = _lib()
    rng = np.random.default_rng(5)
    lam = rng.normal(size=(7, 11))
    prs = np.array([[k, l, int(rng.integers(0, 2))] for l in range(7) for k in range(7) if k != l], np.int32)
    for scale in (1e-6, 0.05, 0.7, 3.0):
        theta = scale * rng.normal(size=len(prs))
        got = vb.rotate_orbitals(lam, prs, theta)
        want = ROT.rotate(lam, prs, theta)
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-12 * max(1.0, np.abs(want).max()))
    # theta = 0 is the identity
    np.testing.assert_array_equal(vb.rotate_orbitals(lam, prs, np.zeros(len(prs))), lam)


def test_library_redundancy_matches_oracle(oracle_mod):
    """F2: the three structure coefficients and all 18 rotations, in that
    order; the library's Cholesky rule and the oracle's least squares keep
    the same parameters.  By the algebra, one coefficient goes by the
    normalisation (sum_I c_I d lnPsi / d c_I = 1) and both active-active
    rotations lie in the span of the structures (with its own coefficient
    for each ionic structure, E_98 Psi = 2 c_cov Phi_99 + c_88 Phi_cov and
    E_89 Psi = 2 c_cov Phi_88 + c_99 Phi_cov)."""
    vb = _lib()
    sysd = S.f2_shaped()
    o = oracle_mod.Oracle(sysd)
    R = S.initial_walkers(sysd, 200, seed=12, sigma=0.8)
    prs = ROT.pairs(ROT.occupancy(o))
    cs, _, _ = o.param_slices()
    oc, _ = o.param_deriv(R, np.arange(cs.start, cs.stop))
    ok, _ = ROT.kappa_deriv(o, R, prs)
    O = np.hstack([oc, ok])
    want = ROT.redundant_keep(O)
    got = vb.lm_redundant(np.cov(O, rowvar=False, bias=True))
    np.testing.assert_array_equal(got, want)
    np.testing.assert_array_equal(np.flatnonzero(~want), [2, len(want) - 2, len(want) - 1])


def test_library_rejects_bad_arguments():
    vb = _lib()
    with pytest.raises(vb.VBQMCError):
        vb.rotate_orbitals(np.eye(3), [[0, 0, 1]], [0.1])       # diagonal pair
    with pytest.raises(vb.VBQMCError):
        vb.rotate_orbitals(np.eye(3), [[0, 5, 1]], [0.1])       # orbital out of range
    with pytest.raises(vb.VBQMCError):
        vb.rotate_orbitals(np.eye(3), [[0, 1, 1]], [np.nan])
    with pytest.raises(vb.VBQMCError):
        vb.lm_redundant(np.eye(2), tol=-1.0)
