"""Seeded generators for the synthetic JVB systems (inputs only, no method arithmetic)."""

import numpy as np

_L_NFUNC = {0: 1, 1: 3, 2: 5}


def n_basis(system):
    return sum(_L_NFUNC[s["l"]] for s in system["shells"])


def n_electrons(system):
    return system["n_up"] + system["n_dn"]


# --------------------------------------------------------------------------
# building blocks
# --------------------------------------------------------------------------

def _gto_shells(rng, center, spec, kmin, kmax, lo, hi):
    """Contracted Gaussian shells on one atom.

    spec: list of (l, count).  Per shell K ~ U{kmin..kmax} primitives with
    exponents log-uniform in [lo, hi] (sorted, tight first) and coefficients
    U(0.1, 1) times the s-type primitive scale (2a/pi)^(3/4) (4a)^(l/2), so
    that tight and diffuse primitives contribute values of similar size.
    """
    shells = []
    for l, count in spec:
        for _ in range(count):
            k = int(rng.integers(kmin, kmax + 1))
            exps = np.sort(np.exp(rng.uniform(np.log(lo), np.log(hi), size=k)))[::-1]
            raw = rng.uniform(0.1, 1.0, size=k)
            scale = (2.0 * exps / np.pi) ** 0.75 * (4.0 * exps) ** (0.5 * l)
            shells.append({"center": center, "kind": "gto", "l": l,
                           "exps": exps.tolist(), "coefs": (raw * scale).tolist()})
    return shells


def _atom_blocks(shells, n_nuc):
    """Basis-function index ranges per atom (shells are grouped by atom)."""
    blocks = [[] for _ in range(n_nuc)]
    mu = 0
    for s in shells:
        nf = _L_NFUNC[s["l"]]
        blocks[s["center"]].extend(range(mu, mu + nf))
        mu += nf
    return blocks


def _pade_jastrow(n_nuc, a_anti=0.5, a_par=0.25, b_ee=1.0, a_en=-0.2, b_en=1.5, kappa=0.0):
    return {
        "kappa": kappa,
        "ee": {"a_anti": a_anti, "a_par": a_par, "b_anti": b_ee, "b_par": b_ee,
               "poly": [0.0, 0.0, 0.0, 0.0]},
        "en": [{"a1": a_en, "a2": b_en, "poly": [0.0, 0.0, 0.0, 0.0]} for _ in range(n_nuc)],
    }


def _zero_jastrow(n_nuc):
    return _pade_jastrow(n_nuc, 0.0, 0.0, 0.0, 0.0, 0.0)


def _place_nuclei(rng, n, side, min_sep):
    while True:
        pos = rng.uniform(-side / 2, side / 2, size=(n, 3))
        d = np.linalg.norm(pos[:, None, :] - pos[None, :, :], axis=-1)
        d[np.arange(n), np.arange(n)] = np.inf
        if d.min() >= min_sep:
            return pos


def _charges(rng, n, choices, total):
    while True:
        z = rng.choice(choices, size=n)
        if int(z.sum()) == total:
            return z


def _normalised_normal(rng, n):
    c = rng.normal(size=n)
    return c / np.linalg.norm(c)


def _two_unit_structures(rng, inactive, pool, n_two_pair, n_pair_self, n_self_self):
    """Structures made of the inactive set plus two singlet-paired units drawn
    from the active pool: two distinct pairs, a pair plus a self-pair, or two
    self-pairs.  Duplicates are redrawn."""
    seen = set()
    out = []

    def add(kind, count):
        made = 0
        while made < count:
            if kind == "pp":
                a, b, c, d = rng.choice(pool, size=4, replace=False)
                pairs = [[int(a), int(b)], [int(c), int(d)]]
            elif kind == "ps":
                a, b, c = rng.choice(pool, size=3, replace=False)
                pairs = [[int(a), int(b)], [int(c), int(c)]]
            else:
                a, c = rng.choice(pool, size=2, replace=False)
                pairs = [[int(a), int(a)], [int(c), int(c)]]
            key = tuple(sorted(tuple(sorted(p)) for p in pairs))
            if key in seen:
                continue
            seen.add(key)
            out.append({"terms": [{"inactive": list(inactive), "pairs": pairs, "unpaired": []}]})
            made += 1

    add("pp", n_two_pair)
    add("ps", n_pair_self)
    add("ss", n_self_self)
    return out


# --------------------------------------------------------------------------
# the five workload systems
# --------------------------------------------------------------------------

def h2_heitler_london(seed=1000):
    """H2-like Heitler-London JVB: protons at z = -0.7, +0.7; 1 up + 1 down electron.

    Basis: 3 contracted s Gaussians per atom, 3 primitives each, exponents
    log-uniform in [0.1, 20], coefficients U(0.1, 1).  Orbitals a (atom A) and
    b (atom B), coefficients U(0.1, 1) on their own atom.  Structures: covalent
    pair (a, b) with c = 0.9 and the ionic sum of the self-pairs (a, a) + (b, b)
    with c = 0.3.  Pade Jastrow: e-e A = 0.5 (anti) / 0.25 (parallel), B = 1;
    e-n A = -0.2, B = 1.5.
    """
    rng = np.random.default_rng(seed)
    pos = np.array([[0.0, 0.0, -0.7], [0.0, 0.0, 0.7]])
    shells = []
    for a in range(2):
        for _ in range(3):
            exps = np.sort(np.exp(rng.uniform(np.log(0.1), np.log(20.0), size=3)))[::-1]
            coefs = rng.uniform(0.1, 1.0, size=3)
            shells.append({"center": a, "kind": "gto", "l": 0,
                           "exps": exps.tolist(), "coefs": coefs.tolist()})
    lam = np.zeros((2, 6))
    lam[0, 0:3] = rng.uniform(0.1, 1.0, size=3)
    lam[1, 3:6] = rng.uniform(0.1, 1.0, size=3)
    structures = [
        {"c": 0.9, "terms": [{"inactive": [], "pairs": [[0, 1]], "unpaired": []}]},
        {"c": 0.3, "terms": [{"inactive": [], "pairs": [[0, 0]], "unpaired": []},
                             {"inactive": [], "pairs": [[1, 1]], "unpaired": []}]},
    ]
    return {"name": "h2_heitler_london", "seed": seed,
            "nuclei": {"Z": [1.0, 1.0], "pos": pos.tolist()},
            "n_up": 1, "n_dn": 1, "shells": shells, "lam": lam.tolist(),
            "structures": structures, "jastrow": _pade_jastrow(2)}


def f2_shaped(seed=1001):
    """F2-shaped diatomic: Z = 9 at z = -1.33, +1.33; 9 up + 9 down electrons.

    Basis per atom 3s2p1d (14 functions), 3-8 primitives per shell, exponents
    log-uniform in [0.05, 1e4].  Orbitals: 8 inactive (4 per atom) and the two
    active sigma orbitals, each N(0,1)/sqrt(14) on its own atom's block.
    Structures: covalent (sA, sB) and the two ionic self-pairs, c ~ N(0,1)
    normalised.  Pade Jastrow as the H2 system with per-nucleus e-n terms.
    """
    rng = np.random.default_rng(seed)
    pos = np.array([[0.0, 0.0, -1.33], [0.0, 0.0, 1.33]])
    shells = []
    for a in range(2):
        shells += _gto_shells(rng, a, [(0, 3), (1, 2), (2, 1)], 3, 8, 0.05, 1e4)
    blocks = _atom_blocks(shells, 2)
    M = 28
    lam = np.zeros((10, M))
    owner = [0, 0, 0, 0, 1, 1, 1, 1, 0, 1]
    for p, a in enumerate(owner):
        lam[p, blocks[a]] = rng.normal(size=len(blocks[a])) / np.sqrt(len(blocks[a]))
    c = _normalised_normal(rng, 3)
    inact = list(range(8))
    structures = [
        {"c": float(c[0]), "terms": [{"inactive": inact, "pairs": [[8, 9]], "unpaired": []}]},
        {"c": float(c[1]), "terms": [{"inactive": inact, "pairs": [[8, 8]], "unpaired": []}]},
        {"c": float(c[2]), "terms": [{"inactive": inact, "pairs": [[9, 9]], "unpaired": []}]},
    ]
    return {"name": "f2_shaped", "seed": seed,
            "nuclei": {"Z": [9.0, 9.0], "pos": pos.tolist()},
            "n_up": 9, "n_dn": 9, "shells": shells, "lam": lam.tolist(),
            "structures": structures, "jastrow": _pade_jastrow(2)}


def f2_bovb(seed=1001, breathing=0.3):
    """BOVB form (Eq. PsiJBOVB) of the F2-shaped system: every structure has
    its own active orbitals, the 8 inactive ones are shared.  Covalent
    (sA, sB) = orbitals 8, 9 as in f2_shaped; the ionic structures pair sA'
    (orbital 10) and sB' (orbital 11) with themselves.  The breathing orbitals
    are sA, sB plus N(0, breathing^2)/sqrt(14) on their own atom's block
    (breathing = 0 gives back the f2_shaped wave function)."""
    base = f2_shaped(seed)
    rng = np.random.default_rng(seed + 500)
    lam = np.array(base["lam"])
    blocks = _atom_blocks(base["shells"], 2)
    extra = []
    for p, a in ((8, 0), (9, 1)):
        row = lam[p].copy()
        row[blocks[a]] += breathing * rng.normal(size=len(blocks[a])) / np.sqrt(len(blocks[a]))
        extra.append(row)
    lam = np.vstack([lam, np.array(extra)])
    st = base["structures"]
    inact = list(range(8))
    structures = [
        st[0],
        {"c": st[1]["c"], "terms": [{"inactive": inact, "pairs": [[10, 10]], "unpaired": []}]},
        {"c": st[2]["c"], "terms": [{"inactive": inact, "pairs": [[11, 11]], "unpaired": []}]},
    ]
    return {**base, "name": "f2_bovb", "lam": lam.tolist(), "structures": structures}


# terms of the f_een expansion per nucleus (Sec. 2.1: p = 2..5 with the
# paper's l_max and integer-m rules)
N_EEN_TERMS = 23


def synthetic_ecp(center, z_eff, scale=1.0, r_cut=2.5):
    """A pseudopotential record of the energy-consistent shape (no tabulated
    potential is used): local part Z/r e^(-a r^2) + Z a r e^(-b r^2) + g e^(-d r^2)
    (cancelling the -Z/r singularity at the nucleus) and s and p channels of
    one and two Gaussian terms; the numbers are made up at the magnitude of
    first-row valence potentials, times scale."""
    return {"center": int(center), "r_cut": float(r_cut),
            "local": [[z_eff * scale, 1, 12.0], [z_eff * 12.0 * scale, 3, 10.0], [-20.0 * scale, 2, 9.0]],
            "channels": [[[60.0 * scale, 2, 15.0], [-4.0 * scale, 2, 3.0]], [[-10.0 * scale, 2, 8.0]]]}


def ecp_one_centre(l, lam, alpha=0.7, z_eff=1.0, jastrow=None, r_cut=2.5):
    """One electron in a Gaussian shell of angular momentum l (combination lam
    of its functions) at a pseudo-nucleus of charge z_eff carrying s, p and d
    channels with different radial parts."""
    sysd = _one_centre(z_eff, 1, 0, {"center": 0, "kind": "gto", "l": l, "exps": [alpha], "coefs": [1.0]},
                       [list(map(float, lam))],
                       [{"c": 1.0, "terms": [{"inactive": [], "pairs": [], "unpaired": [0]}]}], jastrow)
    sysd["name"] = f"ecp_one_centre_l{l}"
    sysd["ecp"] = [{"center": 0, "r_cut": float(r_cut), "local": [[z_eff, 1, 5.0], [-2.0, 2, 1.5]],
                    "channels": [[[3.0, 2, 1.1]], [[-1.7, 2, 0.8], [0.6, 3, 2.0]], [[0.9, 2, 0.5]]]}]
    return sysd


def f2_valence_ecp(seed=1005):
    """F2-shaped diatomic with the 1s cores replaced by pseudopotentials:
    Z = 7 at z = -1.33, +1.33; 7 up + 7 down electrons.  Basis per atom
    3s2p1d, 2-5 primitives per shell, exponents log-uniform in [0.08, 30]
    (valence range).  Orbitals: 6 inactive (3 per atom) and the two active
    sigma orbitals, N(0,1)/sqrt(14) on their own atom's block; covalent and
    two ionic structures, c ~ N(0,1) normalised; Pade Jastrow; per atom the
    synthetic_ecp record (r_cut 2.5 bohr)."""
    rng = np.random.default_rng(seed)
    pos = np.array([[0.0, 0.0, -1.33], [0.0, 0.0, 1.33]])
    shells = []
    for a in range(2):
        shells += _gto_shells(rng, a, [(0, 3), (1, 2), (2, 1)], 2, 5, 0.08, 30.0)
    blocks = _atom_blocks(shells, 2)
    lam = np.zeros((8, 28))
    owner = [0, 0, 0, 1, 1, 1, 0, 1]
    for p, a in enumerate(owner):
        lam[p, blocks[a]] = rng.normal(size=len(blocks[a])) / np.sqrt(len(blocks[a]))
    c = _normalised_normal(rng, 3)
    inact = list(range(6))
    structures = [
        {"c": float(c[0]), "terms": [{"inactive": inact, "pairs": [[6, 7]], "unpaired": []}]},
        {"c": float(c[1]), "terms": [{"inactive": inact, "pairs": [[6, 6]], "unpaired": []}]},
        {"c": float(c[2]), "terms": [{"inactive": inact, "pairs": [[7, 7]], "unpaired": []}]},
    ]
    return {"name": "f2_valence_ecp", "seed": seed,
            "nuclei": {"Z": [7.0, 7.0], "pos": pos.tolist()},
            "n_up": 7, "n_dn": 7, "shells": shells, "lam": lam.tolist(),
            "structures": structures, "jastrow": _pade_jastrow(2),
            "ecp": [synthetic_ecp(0, 7.0), synthetic_ecp(1, 7.0)]}


def with_een(system, seed=2207, scale=0.05, kappa=0.8):
    """The system with an f_een three-body Jastrow: per chemical element
    N_EEN_TERMS coefficients ~ N(0, scale^2), shared by the nuclei of that
    element (Sec. 2.1), in the term order of the library's f_een
    coefficients; kappa set to the paper's 0.8 where it was 0."""
    rng = np.random.default_rng(seed)
    Z = system["nuclei"]["Z"]
    per_z = {z: (scale * rng.normal(size=N_EEN_TERMS)).tolist() for z in sorted(set(Z))}
    jas = dict(system["jastrow"])
    if jas["kappa"] == 0.0:
        jas["kappa"] = kappa
    jas["een"] = [list(per_z[z]) for z in Z]
    return {**system, "name": system["name"] + "_een", "jastrow": jas}


def _molecule(seed, name, n_nuc, zchoices, ztotal, side, shell_spec, n_inactive,
              n_active_per_atom, active_atoms, struct_counts, jastrow_kind,
              delocal_sigma=0.1, active_perturb=0.0, max_exponent=1e4):
    rng = np.random.default_rng(seed)
    pos = _place_nuclei(rng, n_nuc, side, 2.0)
    Z = _charges(rng, n_nuc, zchoices, ztotal).astype(float)
    shells = []
    for a in range(n_nuc):
        shells += _gto_shells(rng, a, shell_spec, 3, 8, 0.05, max_exponent)
    blocks = _atom_blocks(shells, n_nuc)
    M = sum(_L_NFUNC[s["l"]] for s in shells)
    n_act = n_active_per_atom * len(active_atoms)
    n_orb = n_inactive + n_act
    lam = np.zeros((n_orb, M))
    order = np.argsort(-Z, kind="stable")
    for p in range(n_inactive):
        a = int(order[p % n_nuc])
        lam[p, blocks[a]] = rng.normal(size=len(blocks[a])) / np.sqrt(len(blocks[a]))
        lam[p, :] += rng.normal(scale=delocal_sigma, size=M)
    p = n_inactive
    for a in active_atoms:
        for _ in range(n_active_per_atom):
            blk = blocks[a]
            lam[p, blk] = rng.normal(size=len(blk)) / np.sqrt(len(blk))
            if active_perturb > 0:
                lam[p, blk] += rng.normal(scale=active_perturb, size=len(blk))
            p += 1
    pool = list(range(n_inactive, n_orb))
    structures = _two_unit_structures(rng, range(n_inactive), pool, *struct_counts)
    c = _normalised_normal(rng, len(structures))
    for s, ci in zip(structures, c):
        s["c"] = float(ci)
    if jastrow_kind == "pade":
        jas = _pade_jastrow(n_nuc)
    else:
        # kappa = 0.8 scaled variables; the Pade parts equal A r / (1 + B r)
        # with B = kappa + b; polynomial coefficients are small draws.
        kappa = 0.8
        jas = {"kappa": kappa,
               "ee": {"a_anti": 0.5, "a_par": 0.25, "b_anti": 1.0 - kappa, "b_par": 1.0 - kappa,
                      "poly": rng.normal(scale=0.01, size=4).tolist()},
               "en": [{"a1": -0.2, "a2": 1.5 - kappa,
                       "poly": [float(rng.normal(scale=0.01)), 0.0, 0.0, 0.0]}
                      for _ in range(n_nuc)]}
    n = ztotal // 2
    return {"name": name, "seed": seed, "nuclei": {"Z": Z.tolist(), "pos": pos.tolist()},
            "n_up": n, "n_dn": ztotal - n, "shells": shells, "lam": lam.tolist(),
            "structures": structures, "jastrow": jas}


def precision_molecule(seed=1002, max_exponent=1e4):
    """10 nuclei (Z in {1,6,7,8}, sum 40) in a 12-bohr box, 4s2p1d per atom
    (150 functions), 18 delocalised inactive orbitals + 8 active on 8 distinct
    atoms, 20 structures (14 two-pair, 2 pair+self, 4 self+self) = 64 dets.
    max_exponent caps the Gaussian exponents (log-uniform from 0.05); every
    other draw is the same for any cap."""
    rng = np.random.default_rng(seed + 7)
    act_atoms = sorted(rng.choice(10, size=8, replace=False).tolist())
    name = "precision_molecule" if max_exponent == 1e4 else f"precision_molecule_amax{max_exponent:g}"
    return _molecule(seed, name, 10, [1, 6, 7, 8], 40, 12.0,
                     [(0, 4), (1, 2), (2, 1)], 18, 1, act_atoms, (14, 2, 4), "pade",
                     max_exponent=max_exponent)


def adjoint_molecule(seed=1003):
    """6 nuclei (Z in {1,6,7,8}, sum 30), 4s2p2d per atom (120 functions),
    13 dense inactive orbitals + 12 active (2 per atom), 12 structures
    (9 two-pair, 1 pair+self, 2 self+self) = 40 dets, kappa = 0.8 Jastrow with
    polynomial terms."""
    side = 12.0 * (6 / 10) ** (1 / 3)
    return _molecule(seed, "adjoint_molecule", 6, [1, 6, 7, 8], 30, side,
                     [(0, 4), (1, 2), (2, 2)], 13, 2, list(range(6)), (9, 1, 2), "scaled",
                     delocal_sigma=0.1, active_perturb=0.1)


def dmc_molecule(seed=1004):
    """16 nuclei (Z in {1,6,8}, sum 64), 4s2p1d per atom (240 functions),
    30 inactive + 16 active (one per atom), 32 two-pair structures = 128 dets."""
    side = 12.0 * (16 / 10) ** (1 / 3)
    return _molecule(seed, "dmc_molecule", 16, [1, 6, 8], 64, side,
                     [(0, 4), (1, 2), (2, 1)], 30, 1, list(range(16)), (32, 0, 0), "pade")


# --------------------------------------------------------------------------
# closed-form systems (pins)
# --------------------------------------------------------------------------

def _one_centre(Z, n_up, n_dn, shell, lam, structures, jastrow=None):
    return {"name": "one_centre", "seed": 0,
            "nuclei": {"Z": [float(Z)], "pos": [[0.0, 0.0, 0.0]]},
            "n_up": n_up, "n_dn": n_dn, "shells": [shell], "lam": lam,
            "structures": structures, "jastrow": jastrow or _zero_jastrow(1)}


def hydrogen_sto_1s(zeta=1.0):
    """Hydrogen atom, one spin-up electron in exp(-zeta r)."""
    return _one_centre(1, 1, 0, {"center": 0, "kind": "sto", "l": 0, "exps": [zeta], "coefs": [1.0]},
                       [[1.0]], [{"c": 1.0, "terms": [{"inactive": [], "pairs": [], "unpaired": [0]}]}])


def hydrogen_sto_mix(zetas=(1.0, 2.0, 3.0), coefs=(0.7, 0.2, 0.1)):
    """Hydrogen atom, one spin-up electron in sum_k coefs[k] exp(-zetas[k] r)
    (one Slater s shell per exponent, a single orbital, no Jastrow); the
    zeta = 1 function alone is the exact ground state."""
    shells = [{"center": 0, "kind": "sto", "l": 0, "exps": [float(z)], "coefs": [1.0]} for z in zetas]
    return {"name": "hydrogen_sto_mix", "seed": 0,
            "nuclei": {"Z": [1.0], "pos": [[0.0, 0.0, 0.0]]},
            "n_up": 1, "n_dn": 0, "shells": shells, "lam": [[float(c) for c in coefs]],
            "structures": [{"c": 1.0, "terms": [{"inactive": [], "pairs": [], "unpaired": [0]}]}],
            "jastrow": _zero_jastrow(1)}


def hydrogen_sto_2p(zeta=0.5):
    """Hydrogen atom, one electron in z exp(-zeta r)."""
    return _one_centre(1, 1, 0, {"center": 0, "kind": "sto", "l": 1, "exps": [zeta], "coefs": [1.0]},
                       [[0.0, 0.0, 1.0]],
                       [{"c": 1.0, "terms": [{"inactive": [], "pairs": [], "unpaired": [0]}]}])


def hydrogen_gaussian(alpha, jastrow=None):
    """Hydrogen atom, one electron in exp(-alpha r^2)."""
    return _one_centre(1, 1, 0, {"center": 0, "kind": "gto", "l": 0, "exps": [alpha], "coefs": [1.0]},
                       [[1.0]], [{"c": 1.0, "terms": [{"inactive": [], "pairs": [], "unpaired": [0]}]}],
                       jastrow)


def helium_gaussian(alpha, jastrow=None):
    """Helium atom, both electrons in exp(-alpha r^2) (one doubly occupied orbital)."""
    return _one_centre(2, 1, 1, {"center": 0, "kind": "gto", "l": 0, "exps": [alpha], "coefs": [1.0]},
                       [[1.0]], [{"c": 1.0, "terms": [{"inactive": [0], "pairs": [], "unpaired": []}]}],
                       jastrow)


def helium_sto(zeta):
    """Helium atom, both electrons in exp(-zeta r)."""
    return _one_centre(2, 1, 1, {"center": 0, "kind": "sto", "l": 0, "exps": [zeta], "coefs": [1.0]},
                       [[1.0]], [{"c": 1.0, "terms": [{"inactive": [0], "pairs": [], "unpaired": []}]}])


def gaussian_multicentre(alpha, Z, pos, n_up=1, n_dn=0):
    """Electrons in one Gaussian exp(-alpha r^2) centred on the first of
    several nuclei (charges Z, positions pos), no Jastrow: one electron
    (n_up = 1) or two in a doubly occupied orbital (n_up = n_dn = 1)."""
    n_nuc = len(Z)
    occ = {"inactive": [0], "pairs": [], "unpaired": []} if n_dn else {"inactive": [], "pairs": [], "unpaired": [0]}
    return {"name": "gaussian_multicentre", "seed": 0,
            "nuclei": {"Z": [float(z) for z in Z], "pos": [[float(c) for c in p] for p in pos]},
            "n_up": n_up, "n_dn": n_dn,
            "shells": [{"center": 0, "kind": "gto", "l": 0, "exps": [alpha], "coefs": [1.0]}],
            "lam": [[1.0]], "structures": [{"c": 1.0, "terms": [occ]}], "jastrow": _zero_jastrow(n_nuc)}


def small_random_system(seed, n_nuc=2, n_inactive=1, n_active=3, n_pairs=1, n_unpaired=0,
                        n_structures=3, lmax=2, kappa=0.8, poly=True):
    """Small random JVB system for parity and pin tests.

    Every structure holds the same inactive orbitals, `n_pairs` singlet pairs
    (self-pairs allowed) and `n_unpaired` unpaired up orbitals drawn from the
    active set; one structure may be the unit sum of two HLSP terms.
    """
    rng = np.random.default_rng(seed)
    pos = _place_nuclei(rng, n_nuc, 4.0, 1.2)
    Z = rng.integers(1, 4, size=n_nuc).astype(float)
    spec = [(0, 2), (1, 1)] + ([(2, 1)] if lmax >= 2 else [])
    shells = []
    for a in range(n_nuc):
        shells += _gto_shells(rng, a, spec, 1, 3, 0.2, 8.0)
    M = sum(_L_NFUNC[s["l"]] for s in shells)
    n_orb = n_inactive + n_active
    lam = rng.normal(size=(n_orb, M)) / np.sqrt(M)
    inact = list(range(n_inactive))
    act = list(range(n_inactive, n_orb))
    structures = []
    seen = set()
    tries = 0
    while len(structures) < n_structures and tries < 1000:
        tries += 1
        pairs, used = [], set()
        for _ in range(n_pairs):
            free = [o for o in act if o not in used]
            if len(free) < 2 or rng.uniform() < 0.3:
                i = int(rng.choice(free))
                pairs.append([i, i])
                used.add(i)
            else:
                i, j = (int(x) for x in rng.choice(free, size=2, replace=False))
                pairs.append([i, j])
                used.update((i, j))
        free = [o for o in act if o not in used]
        if len(free) < n_unpaired:
            continue
        unp = [int(x) for x in rng.choice(free, size=n_unpaired, replace=False)]
        key = (tuple(tuple(sorted(p)) for p in pairs), tuple(sorted(unp)))
        if key in seen:
            continue
        seen.add(key)
        structures.append({"terms": [{"inactive": inact, "pairs": pairs, "unpaired": unp}]})
    if len(structures) >= 2:
        structures[-2]["terms"] = structures[-2]["terms"] + structures[-1]["terms"]
        structures = structures[:-1]
    c = _normalised_normal(rng, len(structures))
    for s, ci in zip(structures, c):
        s["c"] = float(ci)
    n_dn = n_inactive + n_pairs
    n_up = n_dn + n_unpaired
    jas = {"kappa": kappa,
           "ee": {"a_anti": 0.5, "a_par": 0.25, "b_anti": float(rng.uniform(0.3, 1.2)),
                  "b_par": float(rng.uniform(0.3, 1.2)),
                  "poly": (rng.normal(scale=0.05, size=4) if poly else np.zeros(4)).tolist()},
           "en": [{"a1": float(rng.uniform(-0.5, 0.0)), "a2": float(rng.uniform(0.5, 1.5)),
                   "poly": (rng.normal(scale=0.05, size=4) if poly else np.zeros(4)).tolist()}
                  for _ in range(n_nuc)]}
    return {"name": f"small_random_{seed}", "seed": seed,
            "nuclei": {"Z": Z.tolist(), "pos": pos.tolist()},
            "n_up": n_up, "n_dn": n_dn, "shells": shells, "lam": lam.tolist(),
            "structures": structures, "jastrow": jas}


# --------------------------------------------------------------------------
# walkers
# --------------------------------------------------------------------------

def initial_walkers(system, n_walkers, seed=7, sigma=0.5):
    """Start positions [W, N, 3]: electrons are spread over the nuclei in
    proportion to Z (a shuffled list per walker) and displaced by N(0, sigma^2)."""
    rng = np.random.default_rng(seed)
    Z = np.asarray(system["nuclei"]["Z"])
    pos = np.asarray(system["nuclei"]["pos"], dtype=float)
    N = n_electrons(system)
    weights = np.maximum(np.rint(Z).astype(int), 1)
    owners = np.repeat(np.arange(len(Z)), weights)
    while len(owners) < N:
        owners = np.concatenate([owners, owners])
    R = np.empty((n_walkers, N, 3))
    for w in range(n_walkers):
        own = rng.permutation(owners)[:N]
        R[w] = pos[own] + rng.normal(scale=sigma, size=(N, 3))
    return R


def named_config(name):
    table = {
        "h2": h2_heitler_london,
        "f2": f2_shaped,
        "precision": precision_molecule,
        "adjoint": adjoint_molecule,
        "dmc": dmc_molecule,
    }
    return table[name]()


