"""One step of VB-VMC wave-function optimisation in the paper's
parametrisation (Sec. 2.2, Eq. PsiJVBp: structure coefficients and orbital
rotations; the linear method of Eqs. Psiblin, geneigeq with the estimators
of Eqs. Hi0, H0j, Hij, Sij), every sample-side step on the GPU through the C
ABI: VMC samples, the adjoint's parameter derivatives, the rotation
derivatives, the sample sums over the assembled parameter set; then on the
host the estimators, the redundancy filter, the step and the exp(kappa)
orbital update.  H2 (Heitler-London) starts from a structure ratio far too
ionic and from orbitals rotated away from their atoms.  Energies at new
parameters are estimated by correlated sampling on the same configurations
(weights |Psi_new / Psi_old|^2), whose derivative at the old parameters is,
configuration set by configuration set, (g_L + g_R) / 2 of the estimators
(Eqs. Hi0, H0j): a tiny step along the linear method's direction must change
that energy by (g_L + g_R) / 2 . dp to first order (this ties together the
adjoint's derivatives, the rotation derivatives, the sums, the exp(kappa)
update and vbqmc_set_params), and the full step must lower it."""

import numpy as np
import pytest

import systems as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2207_14715_amd as vb
    vb.load_library()
    return vb


def test_one_linear_method_step_in_rotation_space(lib):
    import torch
    sysd = S.h2_heitler_london()
    ctx0 = lib.Context(sysd)
    pairs = lib.rotation_pairs(ctx0.det_occupancy())
    np.testing.assert_array_equal(pairs, [[1, 0, 0], [0, 1, 0]])
    # start: ionic / covalent = 2 instead of 1/3, orbitals mixed with each other
    lam0 = lib.rotate_orbitals(np.asarray(sysd["lam"]), pairs, np.array([0.3, 0.2]))
    structs = [dict(st) for st in sysd["structures"]]
    structs[0]["c"], structs[1]["c"] = 0.4, 0.8
    start = dict(sysd, lam=lam0.tolist(), structures=structs)
    ctx = lib.Context(start)
    nc = ctx.n_struct
    W = 16384
    R0 = torch.from_numpy(S.initial_walkers(start, W, seed=77, sigma=1.0)).cuda()

    # samples: four blocks of W configurations from one VMC walk
    P = nc + len(pairs)
    acc = torch.zeros(3 * (P + 1) ** 2, dtype=torch.float64, device="cuda")
    st = ctx.walkers_init(R0)
    ctx.vmc_advance(st, 100, 7, 0, 0.5)
    blocks = []
    for b in range(4):
        ctx.vmc_advance(st, 10, 7, 100 + 10 * b, 0.5)
        R = ctx.positions(st).clone()
        dl, de = ctx.param_grad(R)
        kl, ke = ctx.rotation_grad(dl, de, pairs)
        ev = ctx.evaluate(R, want=("eloc",))
        O = torch.cat([dl[:, :nc], kl], dim=1).contiguous()
        D = torch.cat([de[:, :nc], ke], dim=1).contiguous()
        lib.lm_accumulate_cols(O, D, ev["eloc"], acc)
        blocks.append((R, ev["logabs"].clone(), ev["eloc"].clone()))
    est = lib.lm_estimators(acc, P)
    # [c_cov, c_ion, kappa(b <- a), kappa(a <- b)]: the normalisation and the
    # relation E_ab Psi + E_ba Psi = 2 c_cov Phi_ion + 2 c_ion Phi_cov
    keep = lib.lm_redundant(est["s_bar"])
    np.testing.assert_array_equal(keep, [True, False, True, False])
    idx = np.flatnonzero(keep)
    dp, e_lin = lib.lm_solve(est["e0"], est["g_l"][idx], est["g_r"][idx], est["h_bar"][np.ix_(idx, idx)],
                             est["s_bar"][np.ix_(idx, idx)], a_diag=1e-3)
    step = np.zeros(P)
    step[idx] = dp
    assert e_lin < est["e0"]

    def reweighted_energy(dp_full):
        """Correlated-sampling energy after c += dc and the exp(kappa) update."""
        p = p0.copy()
        p[:nc] += dp_full[:nc]
        p[nc:nc + lam0.size] = lib.rotate_orbitals(lam0, pairs, dp_full[nc:]).reshape(-1)
        ctx.set_params(p)
        num = den = 0.0
        for R, la_old, _ in blocks:
            ev = ctx.evaluate(R, want=("eloc",))
            w = torch.exp(2.0 * (ev["logabs"] - la_old))
            num += float((w * ev["eloc"]).sum())
            den += float(w.sum())
        torch.cuda.synchronize()
        return num / den

    p0 = ctx.get_params()
    e_old = sum(float(b[2].sum()) for b in blocks) / sum(b[0].shape[0] for b in blocks)
    assert abs(e_old - est["e0"]) < 1e-12 * max(1.0, abs(e_old))
    slope = 0.5 * (est["g_l"] + est["g_r"])
    h = 1e-4 / np.abs(step).max()
    d_small = (reweighted_energy(h * step) - reweighted_energy(-h * step)) / 2.0
    e_new = reweighted_energy(step)
    print(f"[lm rotation step] E0 {est['e0']:.6f} E_lin {e_lin:.6f} step {step}; correlated sampling: "
          f"central difference {d_small:.4e} vs slope.dp {h * slope @ step:.4e}; full step {e_old:.6f} -> "
          f"{e_new:.6f}", flush=True)
    np.testing.assert_allclose(d_small, h * slope @ step, rtol=1e-5)
    assert h * slope @ step < 0.0
    assert e_new < e_old
