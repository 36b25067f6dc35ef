"""Seeded synthetic inputs for the JVB hot path.

This module only draws numbers: nuclei, basis shells, orbital coefficients,
VB-structure specifications in the paper's HLSP notation, Jastrow parameters
and walker start positions.  It holds none of the method's arithmetic (no
orbital, determinant, Jastrow or energy evaluation, no determinant expansion
of the structures).  Both the CPU oracle and the GPU library read the dicts
built here, each with its own code.

A system is a plain dict:

    nuclei      : {"Z": [..], "pos": [[x, y, z], ..]}            (bohr)
    n_up, n_dn  : spin-up electrons are 0..n_up-1, spin-down the rest
    shells      : list of {"center", "kind" ("gto"|"sto"), "l", "exps", "coefs"}
                  kind "gto": radial sum_k c_k exp(-a_k r^2)
                  kind "sto": radial sum_k c_k exp(-a_k r)
                  angular: l=0 -> 1; l=1 -> x, y, z;
                  l=2 -> xy, yz, zx, x^2-y^2, 3z^2-r^2 (unnormalised harmonic set)
    lam         : orbital coefficients, n_orb x M (row p = orbital p)
    structures  : list of {"c": c_I, "terms": [{"inactive": [...],
                  "pairs": [[i, j], ...], "unpaired": [...]}, ...]}
                  (a structure is the unit-weight sum of its HLSP terms)
    jastrow     : {"kappa", "ee": {"a_anti", "a_par", "b_anti", "b_par",
                  "poly": [b3, b4, b5, b6]},
                  "en": [{"a1", "a2", "poly": [a3, a4, a5, a6]} per nucleus],
                  optional "een": [[c_1 .. c_23] per nucleus] (f_een terms)}
    ecp         : optional list of pseudopotentials, one per pseudo-nucleus:
                  {"center", "r_cut", "local": [[c, n, alpha], ..],
                  "channels": [[[c, n, alpha], ..] for l = 0, 1, ..]}, each
                  radial part sum_k c r^(n-2) exp(-alpha r^2); the nucleus's
                  "Z" is then its effective (valence) charge

Each generator's docstring gives its recipe (seed, distributions, shapes).
"""

from .generate import (  # noqa: F401
    h2_heitler_london,
    f2_shaped,
    f2_bovb,
    f2_valence_ecp,
    synthetic_ecp,
    ecp_one_centre,
    with_een,
    N_EEN_TERMS,
    precision_molecule,
    adjoint_molecule,
    dmc_molecule,
    hydrogen_sto_1s,
    hydrogen_sto_2p,
    hydrogen_sto_mix,
    hydrogen_gaussian,
    helium_gaussian,
    helium_sto,
    gaussian_multicentre,
    small_random_system,
    initial_walkers,
    named_config,
    n_electrons,
    n_basis,
)
