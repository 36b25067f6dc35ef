"""Python binding of libvbqmc (the MI355X JVB QMC library).

Argument marshalling only: every step of the method runs in the HIP kernels
behind the C ABI of ``include/vbqmc.h``.  PyTorch supplies device memory and
the current HIP stream.  The binding refuses to run without the built
library; there is no CPU fallback.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvbqmc.so")

FP64, FP32, BF16, MIXED = 0, 1, 2, 3
_PREC = {"fp64": FP64, "fp32": FP32, "bf16": BF16, "mixed": MIXED}
_L_NFUNC = {0: 1, 1: 3, 2: 5}

_ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "EWORKSPACE", -4: "EHIP", -5: "ESINGULAR", -6: "ENONFINITE",
           -7: "EPOPULATION"}


class VBQMCError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRORS.get(code, code)}: {msg}")
        self.code = code


class _System(ctypes.Structure):
    _fields_ = [("n_nuclei", ctypes.c_int32), ("charge", ctypes.POINTER(ctypes.c_double)),
                ("position", ctypes.POINTER(ctypes.c_double)), ("n_up", ctypes.c_int32),
                ("n_dn", ctypes.c_int32)]


class _Wavefunction(ctypes.Structure):
    _fields_ = [("n_shells", ctypes.c_int32), ("shell_center", ctypes.POINTER(ctypes.c_int32)),
                ("shell_kind", ctypes.POINTER(ctypes.c_int32)), ("shell_l", ctypes.POINTER(ctypes.c_int32)),
                ("shell_nprim", ctypes.POINTER(ctypes.c_int32)), ("prim_exp", ctypes.POINTER(ctypes.c_double)),
                ("prim_coef", ctypes.POINTER(ctypes.c_double)), ("n_orbitals", ctypes.c_int32),
                ("lambda_", ctypes.POINTER(ctypes.c_double)), ("n_structures", ctypes.c_int32),
                ("coef", ctypes.POINTER(ctypes.c_double)), ("n_terms", ctypes.c_int32),
                ("term_structure", ctypes.POINTER(ctypes.c_int32)),
                ("term_counts", ctypes.POINTER(ctypes.c_int32)),
                ("term_orbitals", ctypes.POINTER(ctypes.c_int32)), ("kappa", ctypes.c_double),
                ("ee", ctypes.c_double * 8), ("en", ctypes.POINTER(ctypes.c_double)),
                ("een", ctypes.POINTER(ctypes.c_double))]


class _Ecp(ctypes.Structure):
    _fields_ = [("n_centers", ctypes.c_int32), ("center", ctypes.POINTER(ctypes.c_int32)),
                ("n_channels", ctypes.POINTER(ctypes.c_int32)), ("r_cut", ctypes.POINTER(ctypes.c_double)),
                ("n_terms", ctypes.POINTER(ctypes.c_int32)), ("terms", ctypes.POINTER(ctypes.c_double))]


class _Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("refresh_every", ctypes.c_int32),
                ("walker_lanes", ctypes.c_int32), ("step_kernel", ctypes.c_int32),
                ("dmc_kernel", ctypes.c_int32)]


class _Info(ctypes.Structure):
    _fields_ = [("n_electrons", ctypes.c_int32), ("n_up", ctypes.c_int32), ("n_dn", ctypes.c_int32),
                ("n_nuclei", ctypes.c_int32), ("n_basis", ctypes.c_int32), ("n_orbitals", ctypes.c_int32),
                ("n_structures", ctypes.c_int32), ("n_determinants", ctypes.c_int32),
                ("n_unique_up", ctypes.c_int32), ("n_unique_dn", ctypes.c_int32), ("n_table_up", ctypes.c_int32),
                ("n_table_dn", ctypes.c_int32), ("n_params", ctypes.c_int32),
                ("block_threads", ctypes.c_int32), ("sweep_lanes", ctypes.c_int32),
                ("step_kernel", ctypes.c_int32), ("dmc_kernel", ctypes.c_int32),
                ("walker_state_bytes", ctypes.c_int64),
                ("lds_bytes", ctypes.c_int64)]


class _VmcAcc(ctypes.Structure):
    _fields_ = [("e_sum", ctypes.c_void_p), ("e2_sum", ctypes.c_void_p), ("n_accept", ctypes.c_void_p),
                ("e_last", ctypes.c_void_p), ("sij_sum", ctypes.c_void_p)]


class _DmcLog(ctypes.Structure):
    _fields_ = [("pop", ctypes.c_void_p), ("wsum", ctypes.c_void_p), ("wesum", ctypes.c_void_p),
                ("etrial", ctypes.c_void_p), ("n_accept", ctypes.c_void_p), ("n_prop", ctypes.c_void_p),
                ("step_ms", ctypes.POINTER(ctypes.c_double)), ("wcsum", ctypes.c_void_p),
                ("dr2_acc", ctypes.c_void_p), ("dr2_prop", ctypes.c_void_p)]


# per-step DMC records (device tensors); "wcsum", "dr2_acc" and "dr2_prop"
# may be left out
_DMC_LOG_KEYS = ("pop", "wsum", "wesum", "etrial", "n_accept", "n_prop", "wcsum", "dr2_acc", "dr2_prop")


def _dmc_log(log, step_ms):
    opt = [log[k].data_ptr() if k in log else None for k in _DMC_LOG_KEYS[6:]]
    return _DmcLog(*[log[k].data_ptr() for k in _DMC_LOG_KEYS[:6]], step_ms, *opt)


_lib = None

EXPORTS = ["vbqmc_create", "vbqmc_destroy", "vbqmc_last_error", "vbqmc_get_info", "vbqmc_set_params", "vbqmc_set_ecp",
           "vbqmc_get_params", "vbqmc_evaluate", "vbqmc_walkers_init", "vbqmc_walkers_positions",
           "vbqmc_walkers_eloc", "vbqmc_vmc_advance", "vbqmc_vmc_sweep", "vbqmc_vmc_measure",
           "vbqmc_dmc_workspace_bytes", "vbqmc_dmc_advance", "vbqmc_dmc_advance_noalloc",
           "vbqmc_param_grad_workspace_bytes", "vbqmc_param_grad", "vbqmc_reduce_walkers",
           "vbqmc_weights_chirgwin_coulson", "vbqmc_weights_lowdin", "vbqmc_lm_acc_doubles",
           "vbqmc_lm_accumulate", "vbqmc_lm_estimators", "vbqmc_lm_solve", "vbqmc_det_occupancy",
           "vbqmc_rotation_pairs", "vbqmc_orbital_classes", "vbqmc_rotate_orbitals", "vbqmc_rotation_grad",
           "vbqmc_lm_redundant", "vbqmc_lm_accumulate_cols"]


def load_library(path=LIB_PATH):
    """Load libvbqmc.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libvbqmc.so not found at {path}: build it with "
                           "`python -m paper_2207_14715_amd.build` (there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    vp, i32, i64, dbl, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64
    lib.vbqmc_create.argtypes = [ctypes.POINTER(_System), ctypes.POINTER(_Wavefunction),
                                 ctypes.POINTER(_Options), ctypes.POINTER(vp)]
    lib.vbqmc_destroy.argtypes = [vp]
    lib.vbqmc_destroy.restype = None
    lib.vbqmc_last_error.argtypes = [vp]
    lib.vbqmc_last_error.restype = ctypes.c_char_p
    lib.vbqmc_get_info.argtypes = [vp, ctypes.POINTER(_Info)]
    lib.vbqmc_set_params.argtypes = [vp, ctypes.POINTER(dbl)]
    lib.vbqmc_set_ecp.argtypes = [vp, ctypes.POINTER(_Ecp)]
    lib.vbqmc_get_params.argtypes = [vp, ctypes.POINTER(dbl)]
    lib.vbqmc_evaluate.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp]
    lib.vbqmc_walkers_init.argtypes = [vp, i64, vp, vp, vp]
    lib.vbqmc_walkers_positions.argtypes = [vp, i64, vp, vp, vp]
    lib.vbqmc_walkers_eloc.argtypes = [vp, i64, vp, vp, vp]
    lib.vbqmc_vmc_advance.argtypes = [vp, vp, i64, i32, u64, u64, dbl, i32, ctypes.POINTER(_VmcAcc), vp]
    lib.vbqmc_vmc_sweep.argtypes = [vp, vp, i64, u64, u64, dbl, vp, vp]
    lib.vbqmc_vmc_measure.argtypes = [vp, vp, i64, ctypes.POINTER(_VmcAcc), vp]
    lib.vbqmc_dmc_workspace_bytes.argtypes = [vp, i64, i32, ctypes.POINTER(ctypes.c_size_t)]
    lib.vbqmc_dmc_advance.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(i64), i64, i32, u64, u64, dbl,
                                      ctypes.POINTER(dbl), i64, ctypes.POINTER(_DmcLog), vp, ctypes.c_size_t, vp]
    lib.vbqmc_dmc_advance_noalloc.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(i64), i64, i32, u64, u64, dbl,
                                              ctypes.POINTER(dbl), i64, ctypes.POINTER(_DmcLog), vp]
    lib.vbqmc_param_grad_workspace_bytes.argtypes = [vp, i64, ctypes.POINTER(ctypes.c_size_t)]
    lib.vbqmc_param_grad.argtypes = [vp, i64, vp, vp, vp, vp, ctypes.c_size_t, vp]
    lib.vbqmc_reduce_walkers.argtypes = [vp, i64, i32, vp, vp, vp, vp]
    lib.vbqmc_weights_chirgwin_coulson.argtypes = [i32, ctypes.POINTER(dbl), ctypes.POINTER(dbl),
                                                   ctypes.POINTER(dbl)]
    lib.vbqmc_weights_lowdin.argtypes = lib.vbqmc_weights_chirgwin_coulson.argtypes
    pd = ctypes.POINTER(dbl)
    lib.vbqmc_lm_acc_doubles.argtypes = [i32, ctypes.POINTER(i64)]
    lib.vbqmc_lm_accumulate.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp]
    lib.vbqmc_lm_estimators.argtypes = [i32, pd, pd, pd, pd, pd, pd, pd]
    lib.vbqmc_lm_solve.argtypes = [i32, dbl, pd, pd, pd, pd, dbl, pd, pd]
    pi32, pu8 = ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_uint8)
    lib.vbqmc_det_occupancy.argtypes = [vp, i32, pu8, pi32]
    lib.vbqmc_rotation_pairs.argtypes = [i32, i32, pu8, pi32, i32, pi32, pi32]
    lib.vbqmc_orbital_classes.argtypes = [i32, i32, pd, pi32]
    lib.vbqmc_rotate_orbitals.argtypes = [i32, i32, pd, i32, pi32, pd, pd]
    lib.vbqmc_rotation_grad.argtypes = [vp, i64, i32, vp, vp, vp, vp, vp, vp]
    lib.vbqmc_lm_redundant.argtypes = [i32, pd, dbl, pi32]
    lib.vbqmc_lm_accumulate_cols.argtypes = [i32, i64, vp, vp, vp, vp, vp, vp]
    _lib = lib
    return lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _up(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check_cuda(t, name, dtype=None, shape=None):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous CUDA tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")


class Context:
    """A vbqmc context for one system dict (see the ``systems`` package)."""

    def __init__(self, system, precision="fp64", refresh_every=32, walker_lanes=0, step_kernel=0, dmc_kernel=0):
        lib = load_library()
        self._lib = lib
        self.system = system
        nuc = system["nuclei"]
        self._keep = []

        def keep(a):
            self._keep.append(a)
            return a

        Z = keep(np.ascontiguousarray(nuc["Z"], np.float64))
        pos = keep(np.ascontiguousarray(nuc["pos"], np.float64).reshape(-1))
        sysc = _System(len(Z), _dp(Z), _dp(pos), int(system["n_up"]), int(system["n_dn"]))
        sh = system["shells"]
        cen = keep(np.ascontiguousarray([s["center"] for s in sh], np.int32))
        kind = keep(np.ascontiguousarray([0 if s["kind"] == "gto" else 1 for s in sh], np.int32))
        ls = keep(np.ascontiguousarray([s["l"] for s in sh], np.int32))
        npr = keep(np.ascontiguousarray([len(s["exps"]) for s in sh], np.int32))
        pe = keep(np.ascontiguousarray(np.concatenate([s["exps"] for s in sh]), np.float64))
        pc = keep(np.ascontiguousarray(np.concatenate([s["coefs"] for s in sh]), np.float64))
        lam = keep(np.ascontiguousarray(system["lam"], np.float64))
        st = system["structures"]
        c = keep(np.ascontiguousarray([s["c"] for s in st], np.float64))
        ts, tc, to = [], [], []
        for I, s in enumerate(st):
            for t in s["terms"]:
                ts.append(I)
                tc += [len(t["inactive"]), len(t["pairs"]), len(t["unpaired"])]
                to += list(t["inactive"]) + [o for p in t["pairs"] for o in p] + list(t["unpaired"])
        ts = keep(np.ascontiguousarray(ts, np.int32))
        tc = keep(np.ascontiguousarray(tc, np.int32))
        to = keep(np.ascontiguousarray(to if to else [0], np.int32))
        jas = system["jastrow"]
        ee = jas["ee"]
        ee_arr = (ctypes.c_double * 8)(ee["a_anti"], ee["a_par"], ee["b_anti"], ee["b_par"], *ee["poly"])
        en = keep(np.ascontiguousarray([[e["a1"], e["a2"]] + list(e["poly"]) for e in jas["en"]],
                                       np.float64).reshape(-1))
        # f_een coefficients [n_nuclei][23] in the library's term order, or none
        een = None
        if jas.get("een") is not None:
            een = keep(np.ascontiguousarray(jas["een"], np.float64))
            if een.shape != (len(Z), 23):
                raise ValueError("jastrow een: one row of 23 coefficients per nucleus")
        wfc = _Wavefunction(len(sh), _ip(cen), _ip(kind), _ip(ls), _ip(npr), _dp(pe), _dp(pc), lam.shape[0],
                            _dp(lam), len(st), _dp(c), len(ts), _ip(ts), _ip(tc), _ip(to), float(jas["kappa"]),
                            ee_arr, _dp(en), None if een is None else _dp(een))
        opt = _Options(_PREC[precision] if isinstance(precision, str) else int(precision), int(refresh_every),
                       int(walker_lanes), int(step_kernel), int(dmc_kernel))
        h = ctypes.c_void_p()
        rc = lib.vbqmc_create(ctypes.byref(sysc), ctypes.byref(wfc), ctypes.byref(opt), ctypes.byref(h))
        if rc != 0:
            raise VBQMCError(rc, "vbqmc_create failed (see stderr)")
        self._h = h
        info = _Info()
        lib.vbqmc_get_info(h, ctypes.byref(info))
        self.info = {f: getattr(info, f) for f, _ in _Info._fields_}
        self.N = info.n_electrons
        self.n_struct = info.n_structures
        self.n_params = info.n_params
        self.rec_doubles = info.walker_state_bytes // 8
        self.precision = precision
        if system.get("ecp"):
            self.set_ecp(system["ecp"])

    def __del__(self):
        if getattr(self, "_h", None):
            self._lib.vbqmc_destroy(self._h)
            self._h = None

    def _rc(self, rc):
        if rc != 0:
            raise VBQMCError(rc, self._lib.vbqmc_last_error(self._h).decode())

    # ------------------------------------------------------------------
    def evaluate(self, R, want=("grad", "eloc", "ratio")):
        import torch
        W = R.shape[0]
        _check_cuda(R, "R", torch.float64, (W, self.N, 3))
        dev = R.device
        out = {"logabs": torch.empty(W, dtype=torch.float64, device=dev),
               "sign": torch.empty(W, dtype=torch.int32, device=dev)}
        out["grad"] = torch.empty(W, self.N, 3, dtype=torch.float64, device=dev) if "grad" in want else None
        out["eloc"] = torch.empty(W, dtype=torch.float64, device=dev) if "eloc" in want else None
        out["ratio"] = torch.empty(W, self.n_struct, dtype=torch.float64, device=dev) if "ratio" in want else None
        self._rc(self._lib.vbqmc_evaluate(self._h, W, _ptr(R), _ptr(out["logabs"]), _ptr(out["sign"]),
                                          _ptr(out["grad"]), _ptr(out["eloc"]), _ptr(out["ratio"]), _stream()))
        return out

    def new_state(self, W, device="cuda"):
        import torch
        return torch.zeros(W, self.rec_doubles, dtype=torch.float64, device=device)

    def walkers_init(self, R, state=None):
        import torch
        W = R.shape[0]
        _check_cuda(R, "R", torch.float64, (W, self.N, 3))
        if state is None:
            state = self.new_state(W, R.device)
        _check_cuda(state, "state", torch.float64)
        if state.shape[0] < W or state.shape[1] != self.rec_doubles:
            raise ValueError("state buffer too small")
        self._rc(self._lib.vbqmc_walkers_init(self._h, W, _ptr(R), _ptr(state), _stream()))
        return state

    def positions(self, state, W=None):
        import torch
        W = state.shape[0] if W is None else W
        R = torch.empty(W, self.N, 3, dtype=torch.float64, device=state.device)
        self._rc(self._lib.vbqmc_walkers_positions(self._h, W, _ptr(state), _ptr(R), _stream()))
        return R

    def record_eloc(self, state, W=None):
        import torch
        W = state.shape[0] if W is None else W
        e = torch.empty(W, dtype=torch.float64, device=state.device)
        self._rc(self._lib.vbqmc_walkers_eloc(self._h, W, _ptr(state), _ptr(e), _stream()))
        return e

    def new_vmc_acc(self, W, device="cuda", sij=False):
        import torch
        z = lambda *s: torch.zeros(*s, dtype=torch.float64, device=device)  # noqa: E731
        acc = {"e_sum": z(W), "e2_sum": z(W), "n_accept": z(W), "e_last": z(W)}
        acc["sij_sum"] = z(W, self.n_struct, self.n_struct) if sij else None
        return acc

    def vmc_advance(self, state, n_steps, seed, step0=0, step_size=0.3, all_electron=False, acc=None, W=None):
        W = state.shape[0] if W is None else W
        if acc is None:
            acc = self.new_vmc_acc(W, state.device)
        a = _VmcAcc(acc["e_sum"].data_ptr(), acc["e2_sum"].data_ptr(), acc["n_accept"].data_ptr(),
                    acc["e_last"].data_ptr(), acc["sij_sum"].data_ptr() if acc.get("sij_sum") is not None else None)
        self._rc(self._lib.vbqmc_vmc_advance(self._h, _ptr(state), W, int(n_steps), ctypes.c_uint64(seed),
                                             ctypes.c_uint64(step0), float(step_size), 1 if all_electron else 0,
                                             ctypes.byref(a), _stream()))
        return acc

    def vmc_sweep(self, state, seed, step, step_size, n_accept, W=None):
        """One sweep of single-electron moves of every walker (no E_L)."""
        W = state.shape[0] if W is None else W
        import torch
        _check_cuda(n_accept, "n_accept", torch.float64, (W,))
        self._rc(self._lib.vbqmc_vmc_sweep(self._h, _ptr(state), W, ctypes.c_uint64(seed), ctypes.c_uint64(step),
                                           float(step_size), _ptr(n_accept), _stream()))

    def vmc_measure(self, state, acc, W=None):
        """E_L of every walker from its record, accumulated into acc."""
        W = state.shape[0] if W is None else W
        a = _VmcAcc(acc["e_sum"].data_ptr(), acc["e2_sum"].data_ptr(), acc["n_accept"].data_ptr(),
                    acc["e_last"].data_ptr(), acc["sij_sum"].data_ptr() if acc.get("sij_sum") is not None else None)
        self._rc(self._lib.vbqmc_vmc_measure(self._h, _ptr(state), W, ctypes.byref(a), _stream()))
        return acc

    def dmc_workspace(self, capacity, n_steps, device="cuda"):
        import torch
        nb = ctypes.c_size_t()
        self._rc(self._lib.vbqmc_dmc_workspace_bytes(self._h, capacity, n_steps, ctypes.byref(nb)))
        return torch.zeros((nb.value + 7) // 8, dtype=torch.float64, device=device)

    def dmc_advance(self, states, W, n_steps, seed, step0, tau, e_trial, w_target, workspace=None, log=None,
                    time_steps=False):
        """time_steps: also return "step_ms", the HIP-event duration of each
        step's move-and-energy kernels (numpy, host)."""
        import torch
        cap = states[0].shape[0]
        dev = states[0].device
        if workspace is None:
            workspace = self.dmc_workspace(cap, n_steps, dev)
        if log is None:
            log = {k: torch.zeros(n_steps, dtype=torch.float64, device=dev) for k in _DMC_LOG_KEYS}
        step_ms = np.zeros(max(n_steps, 1)) if time_steps else None
        lg = _dmc_log(log, _dp(step_ms) if time_steps else None)
        arr = (ctypes.c_void_p * 2)(states[0].data_ptr(), states[1].data_ptr())
        Wio = ctypes.c_int64(W)
        et = ctypes.c_double(e_trial)
        rc = self._lib.vbqmc_dmc_advance(self._h, arr, ctypes.byref(Wio), cap, int(n_steps), ctypes.c_uint64(seed),
                                         ctypes.c_uint64(step0), float(tau), ctypes.byref(et), int(w_target),
                                         ctypes.byref(lg), ctypes.c_void_p(workspace.data_ptr()),
                                         workspace.numel() * 8, _stream())
        self._rc(rc)
        out = {"W": Wio.value, "e_trial": et.value, **log}
        if time_steps:
            out["step_ms"] = step_ms[:n_steps]
        return out

    def dmc_advance_noalloc(self, states, W, n_steps, seed, step0, tau, e_trial, w_target, log):
        """vbqmc_dmc_advance on the library's fixed scratch array: the caller
        passes the records and the per-step log, nothing is allocated."""
        cap = states[0].shape[0]
        lg = _dmc_log(log, None)
        arr = (ctypes.c_void_p * 2)(states[0].data_ptr(), states[1].data_ptr())
        Wio = ctypes.c_int64(W)
        et = ctypes.c_double(e_trial)
        self._rc(self._lib.vbqmc_dmc_advance_noalloc(self._h, arr, ctypes.byref(Wio), cap, int(n_steps),
                                                     ctypes.c_uint64(seed), ctypes.c_uint64(step0), float(tau),
                                                     ctypes.byref(et), int(w_target), ctypes.byref(lg), _stream()))
        return {"W": Wio.value, "e_trial": et.value, **log}

    def param_grad(self, R, workspace=None):
        import torch
        W = R.shape[0]
        _check_cuda(R, "R", torch.float64, (W, self.N, 3))
        nb = ctypes.c_size_t()
        self._rc(self._lib.vbqmc_param_grad_workspace_bytes(self._h, W, ctypes.byref(nb)))
        if workspace is None and nb.value:
            workspace = torch.empty((nb.value + 7) // 8, dtype=torch.float64, device=R.device)
        dl = torch.empty(W, self.n_params, dtype=torch.float64, device=R.device)
        de = torch.empty(W, self.n_params, dtype=torch.float64, device=R.device)
        self._rc(self._lib.vbqmc_param_grad(self._h, W, _ptr(R), _ptr(dl), _ptr(de),
                                            _ptr(workspace) if workspace is not None else None,
                                            nb.value, _stream()))
        return dl, de

    def reduce_walkers(self, x, weights=None):
        """Fixed-order sum over the walker axis (optionally weighted)."""
        import torch
        x2 = x.reshape(x.shape[0], -1)
        _check_cuda(x2, "x", torch.float64)
        if weights is not None:
            _check_cuda(weights, "weights", torch.float64, (x2.shape[0],))
        out = torch.empty(x2.shape[1], dtype=torch.float64, device=x.device)
        self._rc(self._lib.vbqmc_reduce_walkers(self._h, x2.shape[0], x2.shape[1], _ptr(weights), _ptr(x2),
                                                _ptr(out), _stream()))
        return out.reshape(x.shape[1:])

    def new_lm_acc(self, device="cuda"):
        """A zeroed accumulator of the linear-method sample sums (3 (P+1)^2 doubles)."""
        import torch
        n = ctypes.c_int64()
        self._rc(self._lib.vbqmc_lm_acc_doubles(self.n_params, ctypes.byref(n)))
        return torch.zeros(n.value, dtype=torch.float64, device=device)

    def lm_accumulate(self, dlogpsi, deloc, eloc, acc, weight=None):
        """Add W samples (vbqmc_param_grad outputs, their E_L, optional weights)
        to the accumulator acc."""
        import torch
        W = dlogpsi.shape[0]
        _check_cuda(dlogpsi, "dlogpsi", torch.float64, (W, self.n_params))
        _check_cuda(deloc, "deloc", torch.float64, (W, self.n_params))
        _check_cuda(eloc, "eloc", torch.float64, (W,))
        _check_cuda(acc, "acc", torch.float64, (3 * (self.n_params + 1) ** 2,))
        if weight is not None:
            _check_cuda(weight, "weight", torch.float64, (W,))
        self._rc(self._lib.vbqmc_lm_accumulate(self._h, W, _ptr(dlogpsi), _ptr(deloc), _ptr(eloc), _ptr(weight),
                                               _ptr(acc), _stream()))

    def det_occupancy(self):
        """The context's determinant products as occupancies [n][2][n_orbitals]
        (vbqmc_det_occupancy)."""
        n = ctypes.c_int32()
        self._rc(self._lib.vbqmc_det_occupancy(self._h, 0, None, ctypes.byref(n)))
        occ = np.zeros((n.value, 2, self.info["n_orbitals"]), np.uint8)
        self._rc(self._lib.vbqmc_det_occupancy(self._h, n.value, _up(occ), ctypes.byref(n)))
        return occ

    def rotation_grad(self, dlogpsi, deloc, pairs):
        """d/d kappa of ln|Psi| and E_L for the rotation pairs [n][3] (numpy
        or tensor) from vbqmc_param_grad outputs (vbqmc_rotation_grad)."""
        import torch
        W = dlogpsi.shape[0]
        _check_cuda(dlogpsi, "dlogpsi", torch.float64, (W, self.n_params))
        _check_cuda(deloc, "deloc", torch.float64, (W, self.n_params))
        pr = torch.as_tensor(np.ascontiguousarray(pairs, np.int32).reshape(-1, 3), device=dlogpsi.device)
        n = pr.shape[0]
        odl = torch.empty(W, n, dtype=torch.float64, device=dlogpsi.device)
        ode = torch.empty(W, n, dtype=torch.float64, device=dlogpsi.device)
        self._rc(self._lib.vbqmc_rotation_grad(self._h, W, n, _ptr(pr), _ptr(dlogpsi), _ptr(deloc), _ptr(odl),
                                               _ptr(ode), _stream()))
        return odl, ode

    def get_params(self):
        p = np.zeros(self.n_params)
        self._rc(self._lib.vbqmc_get_params(self._h, _dp(p)))
        return p

    def set_ecp(self, ecp):
        """Attach pseudopotentials (vbqmc_set_ecp): a list of {"center",
        "r_cut", "local": [[c, n, alpha], ..], "channels": [[[c, n, alpha],
        ..] per l]}, or None / [] to remove them."""
        ecp = ecp or []
        cen = np.ascontiguousarray([e["center"] for e in ecp] or [0], np.int32)
        nch = np.ascontiguousarray([len(e["channels"]) for e in ecp] or [0], np.int32)
        rc = np.ascontiguousarray([e["r_cut"] for e in ecp] or [0.0], np.float64)
        parts = [p for e in ecp for p in [e["local"]] + list(e["channels"])]
        nt = np.ascontiguousarray([len(p) for p in parts] or [0], np.int32)
        terms = np.ascontiguousarray([t for p in parts for t in p] or [[0.0, 0.0, 0.0]], np.float64).reshape(-1)
        arg = _Ecp(len(ecp), _ip(cen), _ip(nch), _dp(rc), _ip(nt), _dp(terms))
        self._rc(self._lib.vbqmc_set_ecp(self._h, ctypes.byref(arg)))

    def set_params(self, p):
        p = np.ascontiguousarray(p, np.float64)
        if p.shape != (self.n_params,):
            raise ValueError("parameter vector has the wrong length")
        self._rc(self._lib.vbqmc_set_params(self._h, _dp(p)))


def weights_chirgwin_coulson(S, c):
    lib = load_library()
    S = np.ascontiguousarray(S, np.float64)
    c = np.ascontiguousarray(c, np.float64)
    w = np.zeros(len(c))
    rc = lib.vbqmc_weights_chirgwin_coulson(len(c), _dp(S), _dp(c), _dp(w))
    if rc != 0:
        raise VBQMCError(rc, "weights_chirgwin_coulson")
    return w


def weights_lowdin(S, c):
    lib = load_library()
    S = np.ascontiguousarray(S, np.float64)
    c = np.ascontiguousarray(c, np.float64)
    w = np.zeros(len(c))
    rc = lib.vbqmc_weights_lowdin(len(c), _dp(S), _dp(c), _dp(w))
    if rc != 0:
        raise VBQMCError(rc, "weights_lowdin")
    return w


def lm_estimators(acc, n_params):
    """E0, g_L, g_R, Hbar, Sbar (and the E_L variance) from an accumulator
    (numpy or tensor; copied to the host)."""
    lib = load_library()
    a = np.ascontiguousarray(acc.cpu().numpy() if hasattr(acc, "cpu") else acc, np.float64)
    P = int(n_params)
    if a.shape != (3 * (P + 1) ** 2,):
        raise ValueError("accumulator has the wrong length")
    e0, var = np.zeros(1), np.zeros(1)
    gl, gr = np.zeros(P), np.zeros(P)
    H, Sb = np.zeros((P, P)), np.zeros((P, P))
    rc = lib.vbqmc_lm_estimators(P, _dp(a), _dp(e0), _dp(gl), _dp(gr), _dp(H), _dp(Sb), _dp(var))
    if rc != 0:
        raise VBQMCError(rc, "lm_estimators")
    return {"e0": float(e0[0]), "g_l": gl, "g_r": gr, "h_bar": H, "s_bar": Sb, "var": float(var[0])}


def lm_solve(e0, g_l, g_r, h_bar, s_bar, a_diag=0.0):
    """(dp, E_lin) of one linear-method step (vbqmc_lm_solve)."""
    lib = load_library()
    g_l, g_r = np.ascontiguousarray(g_l, np.float64), np.ascontiguousarray(g_r, np.float64)
    h_bar, s_bar = np.ascontiguousarray(h_bar, np.float64), np.ascontiguousarray(s_bar, np.float64)
    n = len(g_l)
    if g_r.shape != (n,) or h_bar.shape != (n, n) or s_bar.shape != (n, n):
        raise ValueError("inconsistent shapes")
    dp, el = np.zeros(n), np.zeros(1)
    rc = lib.vbqmc_lm_solve(n, float(e0), _dp(g_l), _dp(g_r), _dp(h_bar), _dp(s_bar), float(a_diag), _dp(dp),
                            _dp(el))
    if rc != 0:
        raise VBQMCError(rc, "lm_solve")
    return dp, float(el[0])


def lm_accumulate_cols(dlogpsi, deloc, eloc, acc, weight=None):
    """vbqmc_lm_accumulate over a caller-assembled parameter set (P = the
    number of columns of dlogpsi)."""
    import torch
    W, P = dlogpsi.shape
    _check_cuda(dlogpsi, "dlogpsi", torch.float64, (W, P))
    _check_cuda(deloc, "deloc", torch.float64, (W, P))
    _check_cuda(eloc, "eloc", torch.float64, (W,))
    _check_cuda(acc, "acc", torch.float64, (3 * (P + 1) ** 2,))
    if weight is not None:
        _check_cuda(weight, "weight", torch.float64, (W,))
    rc = load_library().vbqmc_lm_accumulate_cols(P, W, _ptr(dlogpsi), _ptr(deloc), _ptr(eloc), _ptr(weight),
                                                 _ptr(acc), _stream())
    if rc != 0:
        raise VBQMCError(rc, "lm_accumulate_cols")


def rotation_pairs(occ, loc_class=None):
    """Kept orbital excitations (k, l, kind) [n][3] of a determinant
    occupancy [n_dets][2][n_orb] (vbqmc_rotation_pairs)."""
    lib = load_library()
    occ = np.ascontiguousarray(occ, np.uint8)
    nd, _, no = occ.shape
    cls = None if loc_class is None else np.ascontiguousarray(loc_class, np.int32)
    if cls is not None and cls.shape != (no,):
        raise ValueError("loc_class needs one entry per orbital")
    n = ctypes.c_int32()
    rc = lib.vbqmc_rotation_pairs(no, nd, _up(occ), None if cls is None else _ip(cls), 0, None, ctypes.byref(n))
    if rc != 0 and n.value == 0:
        raise VBQMCError(rc, "rotation_pairs")
    pairs = np.zeros((max(1, n.value), 3), np.int32)
    rc = lib.vbqmc_rotation_pairs(no, nd, _up(occ), None if cls is None else _ip(cls), n.value, _ip(pairs),
                                  ctypes.byref(n))
    if rc != 0:
        raise VBQMCError(rc, "rotation_pairs")
    return pairs[:n.value]


def orbital_classes(lam):
    """Localization class of each orbital (same nonzero pattern, same class)."""
    lib = load_library()
    lam = np.ascontiguousarray(lam, np.float64)
    cls = np.zeros(lam.shape[0], np.int32)
    rc = lib.vbqmc_orbital_classes(lam.shape[0], lam.shape[1], _dp(lam), _ip(cls))
    if rc != 0:
        raise VBQMCError(rc, "orbital_classes")
    return cls


def rotate_orbitals(lam, pairs, theta):
    """lambda' = exp(K)^T lambda for the rotation parameters theta of pairs."""
    lib = load_library()
    lam = np.ascontiguousarray(lam, np.float64)
    pairs = np.ascontiguousarray(pairs, np.int32).reshape(-1, 3)
    theta = np.ascontiguousarray(theta, np.float64)
    if theta.shape != (pairs.shape[0],):
        raise ValueError("one theta per pair")
    out = np.zeros_like(lam)
    rc = lib.vbqmc_rotate_orbitals(lam.shape[0], lam.shape[1], _dp(lam), pairs.shape[0], _ip(pairs), _dp(theta),
                                   _dp(out))
    if rc != 0:
        raise VBQMCError(rc, "rotate_orbitals")
    return out


def lm_redundant(s_bar, tol=1e-8):
    """Mask of the parameters kept (in order) by vbqmc_lm_redundant."""
    lib = load_library()
    s_bar = np.ascontiguousarray(s_bar, np.float64)
    n = s_bar.shape[0]
    if s_bar.shape != (n, n):
        raise ValueError("s_bar must be square")
    keep = np.zeros(n, np.int32)
    rc = lib.vbqmc_lm_redundant(n, _dp(s_bar), float(tol), _ip(keep))
    if rc != 0:
        raise VBQMCError(rc, "lm_redundant")
    return keep.astype(bool)


def _jvb_function():
    import torch

    class JVBFunction(torch.autograd.Function):
        """(ln|Psi|, E_L) of fixed configurations as a differentiable function
        of the parameter vector p = [c | lambda | Jastrow].

        forward: sets p on the context and runs vbqmc_evaluate.
        backward: runs the hand-written adjoint (vbqmc_param_grad, which
        recomputes every determinant inverse from R) at the p this forward
        received, whatever the context holds by then (it is restored after),
        and contracts the per-walker derivatives with the upstream gradients
        by the library's fixed-order walker reduction."""

        @staticmethod
        def forward(ctx_, p, R, vbctx):
            p_host = p.detach().double().cpu().numpy().copy()
            vbctx.set_params(p_host)
            out = vbctx.evaluate(R, want=("eloc",))
            ctx_.save_for_backward(R)
            ctx_.vb = vbctx
            ctx_.p_host = p_host
            ctx_.p_device = p.device
            return out["logabs"], out["eloc"]

        @staticmethod
        def backward(ctx_, g_logpsi, g_eloc):
            (R,) = ctx_.saved_tensors
            vb = ctx_.vb
            held = vb.get_params()
            swap = not np.array_equal(held, ctx_.p_host)
            if swap:
                vb.set_params(ctx_.p_host)
            try:
                dl, de = vb.param_grad(R)
            finally:
                if swap:
                    vb.set_params(held)
            gp = None
            if g_logpsi is not None:
                gp = vb.reduce_walkers(dl, g_logpsi.double().contiguous())
            if g_eloc is not None:
                ge = vb.reduce_walkers(de, g_eloc.double().contiguous())
                gp = ge if gp is None else gp + ge
            return gp.to(ctx_.p_device), None, None

    return JVBFunction


def jvb_apply(p, R, vbctx):
    """Differentiable (ln|Psi|, E_L) for parameters p and configurations R."""
    return _jvb_function().apply(p, R, vbctx)
