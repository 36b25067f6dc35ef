"""GPU evaluate() parity with the CPU oracle: ln|Psi|, sign, grad ln|Psi|, E_L and
structure ratios per fixed configuration, to 1e-10 relative (scaled as in the
helpers), at sizes that span several electron tiles and ragged tails."""

import numpy as np
import pytest

import systems as S
from tests._helpers import compare_evaluate

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2207_14715_amd as vb
    vb.load_library()
    return vb


def _run(lib, oracle_mod, sysd, W, seed, tol=1e-10, scale=0.5):
    import torch
    o = oracle_mod.Oracle(sysd)
    R = S.initial_walkers(sysd, W, seed=seed, sigma=scale)
    ref = o.evaluate(R)
    ctx = lib.Context(sysd)
    print(f"[evaluate] {sysd['name']} W={W} N={ctx.N} M={ctx.info['n_basis']} nt={ctx.info['block_threads']} "
          f"lds={ctx.info['lds_bytes']}", flush=True)
    out = ctx.evaluate(torch.from_numpy(R).cuda())
    torch.cuda.synchronize()
    compare_evaluate(out, ref, tol)
    return ctx, out, ref


def test_hydrogen_exact_orbital(lib, oracle_mod):
    import torch
    sysd = S.hydrogen_sto_1s(1.0)
    ctx = lib.Context(sysd)
    R = torch.from_numpy(np.random.default_rng(0).normal(scale=1.5, size=(256, 1, 3))).cuda()
    out = ctx.evaluate(R)
    e = out["eloc"].cpu().numpy()
    assert np.allclose(e, -0.5, atol=1e-12, rtol=0)


def test_h2_heitler_london(lib, oracle_mod):
    _run(lib, oracle_mod, S.h2_heitler_london(), 300, 1)


@pytest.mark.parametrize("seed,npairs,nunp,nact", [(101, 1, 0, 3), (102, 2, 1, 5), (103, 2, 0, 6), (104, 1, 2, 5)])
def test_small_random(lib, oracle_mod, seed, npairs, nunp, nact):
    sysd = S.small_random_system(seed, n_inactive=2, n_active=nact, n_pairs=npairs, n_unpaired=nunp,
                                 n_structures=4)
    _run(lib, oracle_mod, sysd, 64, seed)


def test_f2_shaped(lib, oracle_mod):
    _run(lib, oracle_mod, S.f2_shaped(), 128, 2)


def test_f2_bovb(lib, oracle_mod):
    # per-structure active orbitals (Eq. PsiJBOVB): 12 orbitals, 3 table orbitals per spin
    _run(lib, oracle_mod, S.f2_bovb(), 96, 7)


@pytest.mark.parametrize("name", ["precision", "adjoint", "dmc"])
def test_workload_systems(lib, oracle_mod, name):
    _run(lib, oracle_mod, S.named_config(name), 8, 3)
