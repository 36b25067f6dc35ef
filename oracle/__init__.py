"""Plain FP64 CPU oracle for the JVB hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product (``paper_2207_14715_amd``)
never does, and shares no code with it: the oracle has its own HLSP
expansion, basis functions, LU determinants, Jastrow, local energy, Philox
and VMC/DMC loops (``vbqmc_oracle.cpp``), evaluated from scratch for every
configuration.  Structure weights (Chirgwin-Coulson and Loewdin, Sec. 2.4)
are finalised here in numpy.

Parity pins: the closed forms, finite differences, Leibniz determinants,
brute-force antisymmetriser and Philox known-answer checks under
``tests/test_oracle_*.py``.  Parity unpinned: multi-electron VMC/DMC means of
the workload systems (only oracle-versus-GPU agreement is checked there).
"""

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vbqmc_oracle.cpp")
_LIB = os.path.join(_HERE, "_vbqmc_oracle.so")

_L_NFUNC = {0: 1, 1: 3, 2: 5}


def build(force=True):
    """Compile the oracle with g++ (OpenMP, no FMA contraction, no fast-math)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp"
    cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-shared", "-fPIC", "-o", tmp, _SRC]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.orc_create.restype = P
        lib.orc_destroy.argtypes = [P]
        lib.orc_num_dets.argtypes = [P]
        lib.orc_num_params.argtypes = [P]
        lib.orc_evaluate.restype = ctypes.c_int
        lib.orc_vmc.restype = ctypes.c_int
        lib.orc_dmc.restype = ctypes.c_int
        lib.orc_lu.restype = ctypes.c_int
        lib.orc_conditioning.restype = ctypes.c_int
        _lib = lib
    return _lib


def een_terms():
    """The f_een terms (k, l, m) in the oracle's order (Sec. 2.1)."""
    klm = np.zeros((64, 3), dtype=np.int32)
    n = int(_load().orc_een_terms(_ip(klm)))
    return [tuple(int(x) for x in r) for r in klm[:n]]


def een_term_count():
    return len(een_terms())


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _up(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def max_threads():
    return int(_load().orc_max_threads())


class Oracle:
    """The oracle for one system dict (see ``systems``)."""

    def __init__(self, system, native_ecp=False):
        """native_ecp: include the system's pseudopotentials (its "ecp" list)
        in E_L of evaluate, vmc and dmc, computed in the C++ oracle (ratios by
        fresh evaluation, as oracle.ecp does in numpy); off by default, so
        that oracle.ecp can add the term itself."""
        lib = _load()
        self.system = system
        nuc = system["nuclei"]
        self.Z = np.ascontiguousarray(nuc["Z"], dtype=np.float64)
        self.pos = np.ascontiguousarray(nuc["pos"], dtype=np.float64).reshape(-1)
        self.n_nuc = len(self.Z)
        self.n_up, self.n_dn = int(system["n_up"]), int(system["n_dn"])
        self.N = self.n_up + self.n_dn
        sh = system["shells"]
        self._sh = [np.ascontiguousarray([s["center"] for s in sh], dtype=np.int32),
                    np.ascontiguousarray([0 if s["kind"] == "gto" else 1 for s in sh], dtype=np.int32),
                    np.ascontiguousarray([s["l"] for s in sh], dtype=np.int32),
                    np.ascontiguousarray([len(s["exps"]) for s in sh], dtype=np.int32)]
        self._pexp = np.ascontiguousarray(np.concatenate([s["exps"] for s in sh]), dtype=np.float64)
        self._pcoef = np.ascontiguousarray(np.concatenate([s["coefs"] for s in sh]), dtype=np.float64)
        self.M = sum(_L_NFUNC[s["l"]] for s in sh)
        self.lam = np.ascontiguousarray(system["lam"], dtype=np.float64)
        self.n_orb = self.lam.shape[0]
        st = system["structures"]
        self.n_struct = len(st)
        self.c = np.ascontiguousarray([s["c"] for s in st], dtype=np.float64)
        tstruct, tcounts, torbs = [], [], []
        for I, s in enumerate(st):
            for t in s["terms"]:
                tstruct.append(I)
                tcounts += [len(t["inactive"]), len(t["pairs"]), len(t["unpaired"])]
                torbs += list(t["inactive"]) + [o for p in t["pairs"] for o in p] + list(t["unpaired"])
        self._tstruct = np.ascontiguousarray(tstruct, dtype=np.int32)
        self._tcounts = np.ascontiguousarray(tcounts, dtype=np.int32)
        self._torbs = np.ascontiguousarray(torbs if torbs else [0], dtype=np.int32)
        jas = system["jastrow"]
        ee = jas["ee"]
        self._ee = np.ascontiguousarray([ee["a_anti"], ee["a_par"], ee["b_anti"], ee["b_par"]] + list(ee["poly"]),
                                        dtype=np.float64)
        self._en = np.ascontiguousarray([[e["a1"], e["a2"]] + list(e["poly"]) for e in jas["en"]],
                                        dtype=np.float64).reshape(-1)
        self.kappa = float(jas["kappa"])
        # f_een coefficients (Sec. 2.1), per nucleus in the oracle's term
        # order, or none
        self.n_een = een_term_count() if jas.get("een") is not None else 0
        self._een = (np.ascontiguousarray(jas["een"], dtype=np.float64).reshape(-1) if self.n_een else None)
        if self.n_een:
            assert self._een.size == self.n_een * self.n_nuc, "een: one row of coefficients per nucleus"
        self._h = lib.orc_create(
            ctypes.c_int(self.n_nuc), _dp(self.Z), _dp(self.pos), ctypes.c_int(self.n_up), ctypes.c_int(self.n_dn),
            ctypes.c_int(len(sh)), _ip(self._sh[0]), _ip(self._sh[1]), _ip(self._sh[2]), _ip(self._sh[3]),
            _dp(self._pexp), _dp(self._pcoef), ctypes.c_int(self.n_orb), _dp(self.lam),
            ctypes.c_int(self.n_struct), _dp(self.c), ctypes.c_int(len(tstruct)), _ip(self._tstruct),
            _ip(self._tcounts), _ip(self._torbs), ctypes.c_double(self.kappa), _dp(self._ee), _dp(self._en),
            _dp(self._een) if self.n_een else None)
        self._lib = lib
        if native_ecp and system.get("ecp"):
            ecp = system["ecp"]
            cen = np.ascontiguousarray([e["center"] for e in ecp], np.int32)
            nch = np.ascontiguousarray([len(e["channels"]) for e in ecp], np.int32)
            rc = np.ascontiguousarray([e["r_cut"] for e in ecp], np.float64)
            parts = [p for e in ecp for p in [e["local"]] + list(e["channels"])]
            nt = np.ascontiguousarray([len(p) for p in parts], np.int32)
            terms = np.ascontiguousarray([t for p in parts for t in p] or [[0.0] * 3], np.float64).reshape(-1)
            lib.orc_set_ecp(ctypes.c_void_p(self._h), ctypes.c_int(len(ecp)), _ip(cen), _ip(nch), _dp(rc), _ip(nt),
                            _dp(terms))
        self.n_dets = int(lib.orc_num_dets(ctypes.c_void_p(self._h)))
        self.n_params = int(lib.orc_num_params(ctypes.c_void_p(self._h)))
        self.n_jastrow = 6 + 6 * self.n_nuc + self.n_een * self.n_nuc

    def __del__(self):
        if getattr(self, "_h", None):
            self._lib.orc_destroy(ctypes.c_void_p(self._h))
            self._h = None

    # ------------------------------------------------------------------
    def param_slices(self):
        """Parameter layout: [c | lambda (row-major) | Jastrow]."""
        a = self.n_struct
        b = a + self.n_orb * self.M
        return slice(0, a), slice(a, b), slice(b, b + self.n_jastrow)

    def dets(self):
        k = self.n_dets
        s = np.zeros(k, np.int32)
        up = np.zeros(max(1, k * self.n_up), np.int32)
        dn = np.zeros(max(1, k * self.n_dn), np.int32)
        self._lib.orc_dets(ctypes.c_void_p(self._h), _ip(s), _ip(up), _ip(dn))
        return s, up[:k * self.n_up].reshape(k, self.n_up), dn[:k * self.n_dn].reshape(k, self.n_dn)

    def ao(self, r):
        r = np.ascontiguousarray(r, dtype=np.float64)
        out = np.zeros(5 * self.M)
        self._lib.orc_ao(ctypes.c_void_p(self._h), _dp(r), _dp(out))
        return out.reshape(5, self.M)

    def evaluate(self, R, level=2):
        R = np.ascontiguousarray(R, dtype=np.float64).reshape(-1, self.N, 3)
        W = R.shape[0]
        out = {"logabs": np.zeros(W), "sign": np.zeros(W, np.int32), "grad": np.zeros((W, self.N, 3)),
               "eloc": np.zeros(W), "ratio": np.zeros((W, self.n_struct)), "kin": np.zeros(W)}
        bad = self._lib.orc_evaluate(ctypes.c_void_p(self._h), ctypes.c_int(W), _dp(R), ctypes.c_int(level),
                                     _dp(out["logabs"]), _ip(out["sign"]), _dp(out["grad"]), _dp(out["eloc"]),
                                     _dp(out["ratio"]), _dp(out["kin"]))
        out["bad"] = int(bad)
        return out

    def conditioning(self, R):
        """kappa_D = sum_k |c d Delta_up Delta_dn| / |D| per configuration (the
        cancellation of the determinant sum) and ln|Delta^sigma_k| of every
        determinant product k per spin ([W][n_dets] each, in the order of
        ``dets()``)."""
        R = np.ascontiguousarray(R, dtype=np.float64).reshape(-1, self.N, 3)
        W = R.shape[0]
        kd = np.zeros(W)
        lup = np.zeros((W, self.n_dets))
        ldn = np.zeros((W, self.n_dets))
        self._lib.orc_conditioning(ctypes.c_void_p(self._h), ctypes.c_int(W), _dp(R), _dp(kd), _dp(lup), _dp(ldn))
        return kd, lup, ldn

    def param_deriv(self, R, idx=None):
        """Per-configuration d lnPsi / dp and d E_L / dp for the listed parameters."""
        R = np.ascontiguousarray(R, dtype=np.float64).reshape(-1, self.N, 3)
        W = R.shape[0]
        idx = np.arange(self.n_params) if idx is None else np.asarray(idx)
        idx = np.ascontiguousarray(idx, dtype=np.int32)
        dl = np.zeros((W, len(idx)))
        de = np.zeros((W, len(idx)))
        self._lib.orc_param_deriv(ctypes.c_void_p(self._h), ctypes.c_int(W), _dp(R), ctypes.c_int(len(idx)),
                                  _ip(idx), _dp(dl), _dp(de))
        return dl, de

    def vmc(self, R, n_steps, seed, step0=0, step_size=0.3, all_electron=False, want_sij=False):
        R = np.array(R, dtype=np.float64).reshape(-1, self.N, 3)
        W = R.shape[0]
        out = {"e_sum": np.zeros(W), "e2_sum": np.zeros(W), "n_acc": np.zeros(W), "e_last": np.zeros(W)}
        sij = np.zeros((W, self.n_struct, self.n_struct)) if want_sij else None
        bad = self._lib.orc_vmc(ctypes.c_void_p(self._h), ctypes.c_int(W), _dp(R), ctypes.c_int(n_steps),
                                ctypes.c_uint64(seed), ctypes.c_uint32(step0), ctypes.c_double(step_size),
                                ctypes.c_int(0 if all_electron else 1), _dp(out["e_sum"]), _dp(out["e2_sum"]),
                                _dp(out["n_acc"]), _dp(out["e_last"]), _dp(sij) if want_sij else None)
        out["R"] = R
        out["sij_sum"] = sij
        out["bad"] = int(bad)
        return out

    def dmc(self, R, eloc, n_steps, seed, step0, tau, e_trial, w_target, capacity=None):
        R0 = np.asarray(R, dtype=np.float64).reshape(-1, self.N, 3)
        W = R0.shape[0]
        cap = capacity or max(4 * W, 16)
        Rb = np.zeros((cap, self.N, 3))
        Rb[:W] = R0
        Eb = np.zeros(cap)
        Eb[:W] = eloc
        Wio = ctypes.c_int(W)
        et = ctypes.c_double(e_trial)
        hist = {k: np.zeros(n_steps) for k in ("pop", "wsum", "wesum", "wcsum", "etrial", "acc", "prop", "dr2_acc",
                                                "dr2_prop")}
        rc = self._lib.orc_dmc(ctypes.c_void_p(self._h), ctypes.byref(Wio), ctypes.c_int(cap), _dp(Rb), _dp(Eb),
                               ctypes.c_int(n_steps), ctypes.c_uint64(seed), ctypes.c_uint32(step0),
                               ctypes.c_double(tau), ctypes.byref(et), ctypes.c_int(w_target),
                               _dp(hist["pop"]), _dp(hist["wsum"]), _dp(hist["wesum"]), _dp(hist["wcsum"]),
                               _dp(hist["etrial"]),
                               _dp(hist["acc"]), _dp(hist["prop"]), _dp(hist["dr2_acc"]), _dp(hist["dr2_prop"]))
        Wn = Wio.value
        return {"rc": int(rc), "R": Rb[:Wn].copy(), "eloc": Eb[:Wn].copy(), "W": Wn, "e_trial": et.value, **hist}


def lu(A):
    """(ln|det A|, sign, A^-1) from the oracle's partial-pivot LU."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    la = ctypes.c_double()
    sg = ctypes.c_int()
    inv = np.zeros((n, n))
    rc = _load().orc_lu(ctypes.c_int(n), _dp(A), ctypes.byref(la), ctypes.byref(sg), _dp(inv))
    if rc != 0:
        return -np.inf, 0, None
    return la.value, sg.value, inv


def philox4x32_10(counter, key):
    ctr = np.ascontiguousarray(counter, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    _load().orc_philox(_up(ctr), _up(k), _up(out))
    return out


def uniforms(seed, walker, step, slot, draw):
    u = np.zeros(2)
    _load().orc_uniforms(ctypes.c_uint64(seed), ctypes.c_uint32(walker), ctypes.c_uint32(step),
                         ctypes.c_uint32(slot), ctypes.c_uint32(draw), _dp(u))
    return u


def weights_chirgwin_coulson(S, c):
    """Sec. 2.4: w_I = sum_J c_I c_J S_IJ / sum_IJ c_I c_J S_IJ."""
    S = np.asarray(S, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    num = c * (S @ c)
    return num / num.sum()


def weights_lowdin(S, c):
    """Sec. 2.4: cbar = S^{1/2} c (symmetric square root), w_K = cbar_K^2 / sum cbar^2."""
    S = np.asarray(S, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    ev, U = np.linalg.eigh(0.5 * (S + S.T))
    half = (U * np.sqrt(np.clip(ev, 0.0, None))) @ U.T
    cb = half @ c
    return cb * cb / np.dot(cb, cb)
