"""The C-ABI library builds, loads and exports every entry point that
include/vbqmc.h declares (no GPU needed: no compute call is made)."""

import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "vbqmc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vbqmc_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for want in ("vbqmc_create", "vbqmc_evaluate", "vbqmc_vmc_advance", "vbqmc_dmc_advance", "vbqmc_param_grad"):
        assert want in names


def test_library_exports_every_declared_symbol():
    import paper_2207_14715_amd as vb
    if not os.path.exists(vb.LIB_PATH):
        from paper_2207_14715_amd import build
        build.build()
    lib = ctypes.CDLL(vb.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(vb.EXPORTS) == _declared()


def test_host_weight_helpers_match_definitions():
    """Chirgwin-Coulson and Loewdin weights of the library (host code) on a
    random positive-definite S: sum to 1, and Loewdin equals the definition
    with the symmetric square root from numpy's eigh."""
    import numpy as np
    import paper_2207_14715_amd as vb
    rng = np.random.default_rng(0)
    A = rng.normal(size=(5, 5))
    Smat = A @ A.T + 5 * np.eye(5)
    c = rng.normal(size=5)
    w = vb.weights_chirgwin_coulson(Smat, c)
    assert abs(w.sum() - 1) < 1e-13
    np.testing.assert_allclose(w, c * (Smat @ c) / (c @ Smat @ c), rtol=1e-12)
    ev, U = np.linalg.eigh(Smat)
    cb = (U * np.sqrt(ev)) @ U.T @ c
    np.testing.assert_allclose(vb.weights_lowdin(Smat, c), cb ** 2 / (cb @ cb), rtol=1e-10)


def _struct_fields(name):
    """(type, field) pairs of a typedef struct of the header, in order."""
    src = open(os.path.join(ROOT, "include", "vbqmc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    body = re.search(r"typedef struct \{([^{}]*)\}\s*" + name + r"\s*;", src).group(1)
    out = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        m = re.match(r"(int32_t|int64_t|double)\s+(.*)", decl)
        assert m, decl
        for f in m.group(2).split(","):
            out.append((m.group(1), f.strip()))
    return out


def test_binding_structs_match_the_header():
    """The ctypes mirrors of vbqmc_options and vbqmc_info_t list the header's
    fields in the header's order with the same integer widths."""
    import ctypes as ct
    import paper_2207_14715_amd as vb
    width = {"int32_t": ct.c_int32, "int64_t": ct.c_int64, "double": ct.c_double}
    for cname, pycls in (("vbqmc_options", vb._Options), ("vbqmc_info_t", vb._Info)):
        want = [(f, width[t]) for t, f in _struct_fields(cname)]
        assert [(f, t) for f, t in pycls._fields_] == want, cname
