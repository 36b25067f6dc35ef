"""Shared helpers for the GPU parity tests (no method arithmetic here)."""

import numpy as np


def rel_tol_check(name, gpu, ref, scale, tol):
    """max |gpu - ref| / max(1, scale) <= tol, elementwise; returns the worst ratio."""
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.maximum(1.0, np.asarray(scale, dtype=np.float64))
    err = np.abs(gpu - ref) / scale
    worst = float(np.nanmax(err)) if err.size else 0.0
    assert np.all(np.isfinite(gpu)), f"{name}: non-finite GPU values"
    assert worst <= tol, f"{name}: worst scaled error {worst:.3e} > {tol:.1e}"
    return worst


def compare_evaluate(out_gpu, ref, tol=1e-10):
    """Parity of ln|Psi|, sign, grad ln|Psi|, E_L and structure ratios.

    E_L is a difference of large kinetic and potential terms, so its error is
    scaled by |T_L| + |V| (both from the oracle)."""
    la = out_gpu["logabs"].cpu().numpy()
    sg = out_gpu["sign"].cpu().numpy()
    assert np.array_equal(sg, ref["sign"]), "sign mismatch"
    rel_tol_check("logabs", la, ref["logabs"], np.abs(ref["logabs"]), tol)
    if out_gpu.get("grad") is not None:
        g = out_gpu["grad"].cpu().numpy()
        gs = np.abs(ref["grad"]).reshape(len(g), -1).max(axis=1)[:, None, None]
        rel_tol_check("grad", g, ref["grad"], gs, tol)
    if out_gpu.get("eloc") is not None:
        e = out_gpu["eloc"].cpu().numpy()
        V = ref["eloc"] - ref["kin"]
        rel_tol_check("eloc", e, ref["eloc"], np.abs(ref["kin"]) + np.abs(V), tol)
    if out_gpu.get("ratio") is not None:
        r = out_gpu["ratio"].cpu().numpy()
        rs = np.abs(ref["ratio"]).max(axis=1)[:, None]
        rel_tol_check("ratio", r, ref["ratio"], rs, tol)
