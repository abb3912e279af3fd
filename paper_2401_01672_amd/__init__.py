"""MI355X (gfx950) solver for the pore-scale freezing/thawing phase-field model
of Strachota, arXiv 2401.01672 (Sec. 2.2 coupled heat + Allen-Cahn SigmaP1-P
model, Sec. 2.4 micro-scale reduction, Sec. 2.5 finite volumes +
Runge-Kutta-Merson).

This module is a thin ctypes binding of ``libpf.so`` (C ABI in
``include/pf.h``): it marshals arguments only.  Every step of the computation
runs in the library's HIP kernels.  Importing fails loudly when the library is
not built.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpf.so")

PF_OK, PF_EQUILIBRIUM, PF_MAXSTEPS = 0, 1, 2
PF_EINVAL, PF_ENOMEM, PF_EHIP, PF_ENONFINITE, PF_EDTMIN = -1, -2, -3, -4, -5
MODELS = {"ac": 0, "coupled": 1, "temp": 2}
PRECISIONS = {"fp64": 0, "fp32": 1}
REACTIONS = {"sigma": 0, "gradp": 1}
WARM_MODES = {"all": 0, "nucleus": 1, "flood": 2}
STATUS_NAMES = {0: "ok", 1: "equilibrium", 2: "maxsteps", -1: "einval", -2: "enomem",
                -3: "ehip", -4: "enonfinite", -5: "edtmin"}


class PFParams(C.Structure):
    _fields_ = [
        ("n1", C.c_int32), ("n2", C.c_int32), ("n3", C.c_int32),
        ("model", C.c_int32), ("precision", C.c_int32), ("reaction", C.c_int32),
        ("dirichlet_faces", C.c_int32), ("bc_kind", C.c_int32),
        ("h", C.c_double), ("xi", C.c_double), ("alpha", C.c_double), ("mu", C.c_double),
        ("b", C.c_double), ("eps0", C.c_double), ("eps1", C.c_double), ("zeta", C.c_double),
        ("t_star", C.c_double), ("dT", C.c_double), ("gamma", C.c_double),
        ("lam", C.c_double * 3), ("rhoc", C.c_double * 3), ("Lv", C.c_double),
        ("bc_T0", C.c_double), ("bc_T1", C.c_double), ("bc_t0", C.c_double),
        ("bc_t1", C.c_double),
        ("tol", C.c_double), ("safety", C.c_double), ("dt_min", C.c_double),
        ("dt_max", C.c_double),
        ("rho_c_separate", C.c_int32), ("pad_", C.c_int32),
        ("rho", C.c_double * 3), ("cs", C.c_double * 3), ("L", C.c_double),
    ]


class PFStepInfo(C.Structure):
    _fields_ = [("accepted", C.c_int32), ("status", C.c_int32), ("eps", C.c_double),
                ("dt_used", C.c_double), ("dt_next", C.c_double), ("maxk1", C.c_double),
                ("t", C.c_double)]


class PFRunStats(C.Structure):
    _fields_ = [("steps_accepted", C.c_int64), ("steps_rejected", C.c_int64),
                ("t", C.c_double), ("dt", C.c_double), ("ice_count", C.c_int64),
                ("pore_count", C.c_int64), ("sum_phi", C.c_double),
                ("enthalpy", C.c_double), ("maxk1", C.c_double), ("wall_s", C.c_double),
                ("status", C.c_int32), ("pad", C.c_int32)]


_lib = None

# (name, restype, argtypes); every symbol declared in include/pf.h
_VP, _H = C.c_void_p, C.c_void_p
SIGNATURES = [
    ("pf_create", C.c_int, [C.POINTER(PFParams), C.c_void_p, C.POINTER(C.c_void_p)]),
    ("pf_create_field", C.c_int, [C.POINTER(PFParams), C.c_void_p, C.POINTER(C.c_void_p)]),
    ("pf_destroy", None, [_H]),
    ("pf_last_error", C.c_char_p, [_H]),
    ("pf_set_stream", C.c_int, [_H, C.c_size_t]),
    ("pf_set_state", C.c_int, [_H, _VP, _VP, C.c_int, C.c_size_t]),
    ("pf_get_state", C.c_int, [_H, _VP, _VP, C.c_int, C.c_size_t]),
    ("pf_set_time", C.c_int, [_H, C.c_double, C.c_double]),
    ("pf_set_tolerance", C.c_int, [_H, C.c_double]),
    ("pf_rhs", C.c_int, [_H, C.c_double, _VP, _VP, _VP, _VP, C.c_size_t]),
    ("pf_rkm_step", C.c_int, [_H, C.POINTER(C.c_double), C.POINTER(C.c_double),
                              C.POINTER(PFStepInfo)]),
    ("pf_integrate", C.c_int, [_H, C.c_double, C.c_int64, C.c_double, C.POINTER(PFRunStats)]),
    ("pf_diagnostics", C.c_int, [_H, C.POINTER(PFRunStats)]),
    ("pf_diagnostics_planes", C.c_int, [_H, C.c_int32, C.c_int32, C.POINTER(PFRunStats)]),
    ("pf_batch_integrate", C.c_int, [C.POINTER(C.c_void_p), C.c_int32, C.c_double, C.c_int64,
                                     C.c_double, C.POINTER(PFRunStats), C.c_size_t,
                                     C.c_void_p]),
    ("pf_set_loop", C.c_int, [_H, C.c_int32, C.c_int32]),
    ("pf_set_tile", C.c_int, [_H, C.c_int32]),
    ("pf_set_stage_tiles", C.c_int, [_H, C.POINTER(C.c_int32)]),
    ("pf_set_schedule", C.c_int, [_H, C.c_int32]),
    ("pf_set_pair_tile", C.c_int, [_H, C.c_int32, C.c_int32]),
    ("pf_set_vector", C.c_int, [_H, C.c_int32]),
    ("pf_get_config", C.c_int, [_H, C.POINTER(C.c_int32)]),
    ("pf_time_kernels", C.c_int, [_H, C.c_int32, C.POINTER(C.c_double)]),
    ("pf_synchronize", C.c_int, [_H]),
    ("pf_num_cells", C.c_int64, [_H]),
    ("pf_abi_version", C.c_int, []),
    ("pf_unet_create", C.c_int, [C.c_uint64, C.POINTER(C.c_void_p)]),
    ("pf_unet_destroy", None, [_H]),
    ("pf_unet_last_error", C.c_char_p, [_H]),
    ("pf_unet_set_stream", C.c_int, [_H, C.c_size_t]),
    ("pf_unet_set_conv_kernel", C.c_int, [_H, C.c_int32]),
    ("pf_unet_num_params", C.c_int64, []),
    ("pf_unet_get_params", C.c_int, [_H, _VP]),
    ("pf_unet_set_params", C.c_int, [_H, _VP]),
    ("pf_unet_forward", C.c_int, [_H, _VP, C.c_int32, C.c_int32, C.c_int32, C.c_double,
                                  C.c_double, _VP]),
    ("pf_unet_grad", C.c_int, [_H, _VP, _VP, C.c_int32, C.c_int32, C.c_int32, C.c_double,
                               C.c_double, _VP, C.POINTER(C.c_double)]),
    ("pf_unet_train_step", C.c_int, [_H, _VP, _VP, C.c_int32, C.c_int32, C.c_int32,
                                     C.c_double, C.c_double, C.c_double,
                                     C.POINTER(C.c_double)]),
    ("pf_unet_time_layers", C.c_int, [_H, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                      C.POINTER(C.c_double)]),
    ("pf_unet_layer_info", C.c_int, [C.c_int32, C.POINTER(C.c_int32)]),
    ("pf_warmstart", C.c_int, [_H, _H, C.c_double, C.c_double, C.c_int32, C.c_size_t]),
    ("pf_conv3_bf16", C.c_int, [_VP, C.c_int32, _VP, _VP, C.c_int32, _VP, C.c_int32,
                                C.c_int32, C.c_int32, C.c_int32, C.c_size_t]),
    ("pf_conv3_bf16_noalloc", C.c_int, [_VP, C.c_int32, _VP, _VP, C.c_int32, _VP, C.c_int32,
                                        C.c_int32, C.c_int32, C.c_int32, C.c_size_t]),
    ("pf_conv3_bf16_backward", C.c_int, [_VP, C.c_int32, _VP, _VP, C.c_int32, C.c_int32,
                                         C.c_int32, C.c_int32, _VP, _VP, _VP, C.c_size_t]),
    ("pf_mfma_probe", C.c_int, [_VP, _VP, _VP, C.c_size_t]),
]


def lib():
    """Load libpf.so; raises if it has not been built (no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                "(hipcc, gfx950); there is no CPU fallback")
        L = C.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class PFError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def make_params(p: Dict, precision: str = "fp64", run: Optional[Dict] = None) -> PFParams:
    """pf_params from a case parameter dict (keys as in pf_inputs.Case.params)
    plus integration controls (tol, safety, dt_min, dt_max)."""
    run = run or {}
    P = PFParams()
    P.n1, P.n2, P.n3 = int(p["n1"]), int(p["n2"]), int(p["n3"])
    P.model = MODELS[p.get("model", "ac")]
    P.precision = PRECISIONS[precision]
    P.reaction = REACTIONS[p.get("reaction", "sigma")]
    P.dirichlet_faces = int(p.get("dirichlet_faces", 0))
    P.bc_kind = int(p.get("bc_kind", 0))
    for k in ("h", "xi", "alpha", "mu", "b", "eps0", "eps1", "zeta", "t_star", "dT", "Lv",
              "bc_T0", "bc_T1", "bc_t0", "bc_t1"):
        setattr(P, k, float(p.get(k, 0.0)))
    P.gamma = float(p.get("gamma", 2.0))
    P.lam[:] = [float(v) for v in p["lam"]]
    P.rhoc[:] = [float(v) for v in p["rhoc"]]
    P.tol = float(run.get("tol", 0.0))
    P.safety = float(run.get("safety", 0.8))
    P.dt_min = float(run.get("dt_min", 1e-12))
    P.dt_max = float(run.get("dt_max", 1e30))
    P.rho_c_separate = int(p.get("rho_c_separate", 0))
    P.rho[:] = [float(v) for v in p.get("rho", (1.0, 1.0, 1.0))]
    P.cs[:] = [float(v) for v in p.get("cs", (1.0, 1.0, 1.0))]
    P.L = float(p.get("L", 0.0))
    return P


def _ptr(x) -> Tuple[int, int]:
    """(address, on_device) of a torch tensor or numpy array."""
    if x is None:
        return 0, 1
    if isinstance(x, np.ndarray):
        assert x.flags.c_contiguous
        return x.ctypes.data, 0
    assert x.is_contiguous()
    return x.data_ptr(), 1 if x.is_cuda else 0


class Solver:
    """One grid: owns a pf_handle."""

    def __init__(self, params: Dict, mask: np.ndarray, precision: str = "fp64",
                 run: Optional[Dict] = None, glass_field: Optional[np.ndarray] = None):
        """mask: uint8 (n3, n2, n1), nonzero = glass; or glass_field: a smooth
        G in [0, 1] (paper mode, pf_create_field; mask is then ignored)."""
        self.P = make_params(params, precision, run)
        self.precision = precision
        self.model = params.get("model", "ac")
        self.shape = (int(params["n3"]), int(params["n2"]), int(params["n1"]))
        self.np_dtype = np.float64 if precision == "fp64" else np.float32
        h = C.c_void_p()
        if glass_field is not None:
            g = np.ascontiguousarray(glass_field, dtype=np.float64)
            assert g.shape == self.shape, (g.shape, self.shape)
            rc = lib().pf_create_field(C.byref(self.P), g.ctypes.data, C.byref(h))
            if rc != 0:
                raise PFError(rc, lib().pf_last_error(None).decode())
            self.h = h
            return
        m = np.ascontiguousarray(mask, dtype=np.uint8)
        assert m.shape == self.shape, (m.shape, self.shape)
        rc = lib().pf_create(C.byref(self.P), m.ctypes.data, C.byref(h))
        if rc != 0:
            raise PFError(rc, lib().pf_last_error(None).decode())
        self.h = h

    # -- plumbing ------------------------------------------------------------
    def _check(self, rc: int, ok=(PF_OK,)) -> int:
        if rc not in ok:
            raise PFError(rc, lib().pf_last_error(self.h).decode())
        return rc

    def close(self):
        if getattr(self, "h", None):
            lib().pf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def ncells(self) -> int:
        return int(np.prod(self.shape))

    def torch_dtype(self):
        import torch
        return torch.float64 if self.precision == "fp64" else torch.float32

    # -- state ----------------------------------------------------------------
    def set_state(self, phi, theta=None, stream: int = 0):
        """phi, theta (= T - T*): torch tensors (cuda) or numpy arrays in the
        handle's precision, ncells elements each (Temp model: theta only,
        phi may be None).  stream: a hipStream_t as int (0: the handle's)."""
        if isinstance(phi, np.ndarray) or isinstance(theta, np.ndarray):
            if phi is not None:
                phi = np.ascontiguousarray(phi, dtype=self.np_dtype)
            if theta is not None:
                theta = np.ascontiguousarray(theta, dtype=self.np_dtype)
        pp, dev = _ptr(phi)
        tp, dev_t = _ptr(theta)
        if phi is None:
            dev = dev_t
        if dev:  # device inputs written on torch's current stream
            import torch
            torch.cuda.current_stream().synchronize()
        self._check(lib().pf_set_state(self.h, pp, tp, dev, int(stream)))

    def get_state(self, device: bool = False, stream: int = 0):
        """(phi, theta); theta is None for the micro-scale model, phi is None
        for the Temp model."""
        has_phi = self.model != "temp"
        has_th = self.model != "ac"
        if device:
            import torch
            mk = (lambda: torch.empty(self.shape, dtype=self.torch_dtype(), device="cuda"))
            phi = mk() if has_phi else None
            th = mk() if has_th else None
            torch.cuda.current_stream().synchronize()
        else:
            phi = np.empty(self.shape, dtype=self.np_dtype) if has_phi else None
            th = np.empty(self.shape, dtype=self.np_dtype) if has_th else None
        self._check(lib().pf_get_state(self.h, _ptr(phi)[0], _ptr(th)[0], 1 if device else 0,
                                       int(stream)))
        return phi, th

    def set_time(self, t: float, dt: float):
        self._check(lib().pf_set_time(self.h, float(t), float(dt)))

    def set_tolerance(self, tol: float):
        self._check(lib().pf_set_tolerance(self.h, float(tol)))

    # -- computation -----------------------------------------------------------
    def rhs(self, t: float, phi, theta, dphi, dtheta, stream: Optional[int] = None):
        """F(t, phi, theta) into dphi, dtheta (device tensors).  By default on
        the handle's stream, after torch's current stream has finished and
        waited for before returning; with an explicit stream (a hipStream_t as
        a nonzero int) the call is left running on that stream."""
        import torch
        wait = stream is None
        if wait:
            torch.cuda.current_stream().synchronize()
            stream = 0
        self._check(lib().pf_rhs(self.h, float(t), _ptr(phi)[0], _ptr(theta)[0],
                                 _ptr(dphi)[0], _ptr(dtheta)[0], int(stream)))
        if wait:
            self._check(lib().pf_synchronize(self.h))

    def rkm_step(self, t: float, dt: float):
        tt, dd = C.c_double(t), C.c_double(dt)
        info = PFStepInfo()
        self._check(lib().pf_rkm_step(self.h, C.byref(tt), C.byref(dd), C.byref(info)),
                    ok=(PF_OK, PF_ENONFINITE, PF_EDTMIN))
        return tt.value, dd.value, dict(accepted=info.accepted, status=info.status,
                                        eps=info.eps, dt_used=info.dt_used,
                                        dt_next=info.dt_next, maxk1=info.maxk1)

    def integrate(self, t_end: float = float("inf"), max_steps: int = 2**62,
                  eq_tol: float = 0.0, raise_on_error: bool = True) -> Dict:
        st = PFRunStats()
        rc = lib().pf_integrate(self.h, float(t_end), int(max_steps), float(eq_tol), C.byref(st))
        if rc < 0 and raise_on_error:
            self._check(rc)
        return self._stats(st, rc)

    def diagnostics(self) -> Dict:
        st = PFRunStats()
        self._check(lib().pf_diagnostics(self.h, C.byref(st)))
        return self._stats(st, PF_OK)

    def diagnostics_planes(self, i3_lo: int, i3_hi: int) -> Dict:
        """Diagnostics over the planes i3_lo <= i3 < i3_hi."""
        st = PFRunStats()
        self._check(lib().pf_diagnostics_planes(self.h, int(i3_lo), int(i3_hi), C.byref(st)))
        return self._stats(st, PF_OK)

    def uwc_bottom_half(self) -> Dict:
        """Unfrozen water content of the bottom half (the planes below n3/2),
        reduced on the GPU."""
        d = self.diagnostics_planes(0, self.shape[0] // 2)
        return dict(water_cells=d["pore_count"], ice_cells=d["ice_count"], uwc=d["uwc"])

    @staticmethod
    def _stats(st: PFRunStats, rc: int) -> Dict:
        pore = st.pore_count
        return dict(steps_accepted=st.steps_accepted, steps_rejected=st.steps_rejected,
                    t=st.t, dt=st.dt, ice_count=st.ice_count, pore_count=pore,
                    sum_phi=st.sum_phi, enthalpy=st.enthalpy, maxk1=st.maxk1,
                    wall_s=st.wall_s, status=st.status, rc=rc,
                    ice_fraction=(st.ice_count / pore) if pore else 0.0,
                    uwc=(1.0 - st.ice_count / pore) if pore else 0.0)

    def set_loop(self, steps_per_poll: int = 16, use_graph: bool = True):
        self._check(lib().pf_set_loop(self.h, int(steps_per_poll), 1 if use_graph else 0))

    def set_tile(self, z_chunk: int):
        self._check(lib().pf_set_tile(self.h, int(z_chunk)))

    def set_stage_tiles(self, z):
        """Planes per workgroup column of S1..S5 (five ints >= 1)."""
        arr = (C.c_int32 * 5)(*[int(v) for v in z])
        self._check(lib().pf_set_stage_tiles(self.h, arr))

    def set_schedule(self, schedule: str):
        """'five' (one pass per stage) or 'paired' (S1+S2, S3+S4, S5)."""
        self._check(lib().pf_set_schedule(self.h, {"five": 0, "paired": 1}[schedule]))

    def set_vector(self, enable: bool):
        self._check(lib().pf_set_vector(self.h, 1 if enable else 0))

    def set_pair_tile(self, tile_index: int, z_chunk: int):
        self._check(lib().pf_set_pair_tile(self.h, int(tile_index), int(z_chunk)))

    def get_config(self) -> Dict:
        out = (C.c_int32 * 14)()
        self._check(lib().pf_get_config(self.h, out))
        v = list(out)
        return dict(schedule={0: "five", 1: "paired"}[v[0]], passes=v[1], z_chunk=v[2],
                    workgroups=v[3], pair_tile=(v[4], v[5]), pair_z_chunk=v[6],
                    pair_workgroups=v[7], vector=bool(v[8]), stage_z_chunk=v[9:14])

    def time_kernels(self, reps: int = 10):
        out = (C.c_double * 6)()
        self._check(lib().pf_time_kernels(self.h, int(reps), out))
        return list(out)

    def synchronize(self):
        self._check(lib().pf_synchronize(self.h))


class PFBatchOptions(C.Structure):
    _fields_ = [("mode", C.c_int32), ("z_chunk", C.c_int32), ("steps_per_poll", C.c_int32),
                ("branches", C.c_int32)]


BATCH_MODES = {"persistent": 1, "graph": 2}


def batch_integrate(solvers, t_end: float = float("inf"), max_steps: int = 2**62,
                    eq_tol: float = 0.0, raise_on_error: bool = True, mode: str = "graph",
                    z_chunk: int = 0, steps_per_poll: int = 0, branches: int = 0):
    """pf_batch_integrate over Solver objects: 'persistent' (one cooperative
    kernel per poll interval) or 'graph' (per-stage launches replayed as a
    HIP graph, in `branches` parallel chains over instance groups; 0 = the
    library's default).  Returns one stats dict per solver."""
    n = len(solvers)
    hs = (C.c_void_p * n)(*[s.h for s in solvers])
    out = (PFRunStats * n)()
    opts = PFBatchOptions(BATCH_MODES[mode], int(z_chunk), int(steps_per_poll), int(branches))
    rc = lib().pf_batch_integrate(hs, n, float(t_end), int(max_steps), float(eq_tol), out, 0,
                                  C.byref(opts))
    if rc < 0 and raise_on_error:
        raise PFError(rc, lib().pf_last_error(solvers[0].h).decode() or
                      lib().pf_last_error(None).decode())
    return [Solver._stats(out[i], rc) for i in range(n)]


# ---------------------------------------------------------------------------
# Learned warm start


def unet_num_params() -> int:
    return int(lib().pf_unet_num_params())


def unet_layer_info(layer: int) -> Dict:
    out = (C.c_int32 * 8)()
    rc = lib().pf_unet_layer_info(int(layer), out)
    if rc != 0:
        raise PFError(rc, f"no convolution {layer}")
    v = list(out)
    return dict(cin=v[0], cout=v[1], w_off=v[2], b_off=v[3], level=v[4], head_w=v[5],
                head_b=v[6], layers=v[7])


def _dev_ptr(t, dtype=None) -> int:
    """Address of a contiguous CUDA tensor (optionally of a given dtype)."""
    assert t.is_cuda and t.is_contiguous(), "device tensor expected"
    if dtype is not None:
        assert t.dtype == dtype, (t.dtype, dtype)
    return t.data_ptr()


class UNet:
    """Warm-start network: owns a pf_unet (parameters, Adam state, buffers)."""

    def __init__(self, seed: int = 0):
        h = C.c_void_p()
        rc = lib().pf_unet_create(C.c_uint64(int(seed)), C.byref(h))
        if rc != 0:
            raise PFError(rc, "pf_unet_create failed")
        self.h = h

    def _check(self, rc: int) -> int:
        if rc != PF_OK:
            raise PFError(rc, lib().pf_unet_last_error(self.h).decode())
        return rc

    def close(self):
        if getattr(self, "h", None):
            lib().pf_unet_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_conv_kernel(self, variant: str):
        """'reg' (default: register-blocked where it is faster, else tiled),
        'tiled' (LDS-staged input blocks) or 'direct'."""
        self._check(lib().pf_unet_set_conv_kernel(
            self.h, {"direct": 0, "tiled": 1, "reg": 2}[variant]))

    def get_params(self) -> np.ndarray:
        out = np.empty(unet_num_params(), np.float32)
        self._check(lib().pf_unet_get_params(self.h, out.ctypes.data))
        return out

    def set_params(self, p: np.ndarray):
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.size == unet_num_params()
        self._check(lib().pf_unet_set_params(self.h, p.ctypes.data))

    def forward(self, mask, dT: float, log10_s: float, out=None):
        """mask: uint8 CUDA tensor (n3, n2, n1), nonzero = glass; returns the
        FP32 prediction (CUDA tensor of the same shape)."""
        import torch
        n3, n2, n1 = mask.shape
        if out is None:
            out = torch.empty(mask.shape, dtype=torch.float32, device=mask.device)
        self._check(lib().pf_unet_forward(self.h, _dev_ptr(mask, torch.uint8), n1, n2, n3,
                                          float(dT), float(log10_s),
                                          _dev_ptr(out, torch.float32)))
        torch.cuda.synchronize()
        return out

    def grad(self, mask, target, dT: float, log10_s: float):
        """(loss, gradient vector) of the masked MSE, no update."""
        import torch
        n3, n2, n1 = mask.shape
        g = np.empty(unet_num_params(), np.float32)
        loss = C.c_double()
        self._check(lib().pf_unet_grad(self.h, _dev_ptr(mask, torch.uint8),
                                       _dev_ptr(target, torch.float32), n1, n2, n3, float(dT),
                                       float(log10_s), g.ctypes.data, C.byref(loss)))
        return loss.value, g

    def train_step(self, mask, target, dT: float, log10_s: float, lr: float,
                   want_loss: bool = True):
        import torch
        n3, n2, n1 = mask.shape
        loss = C.c_double()
        self._check(lib().pf_unet_train_step(self.h, _dev_ptr(mask, torch.uint8),
                                             _dev_ptr(target, torch.float32), n1, n2, n3,
                                             float(dT), float(log10_s), float(lr),
                                             C.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def time_layers(self, shape, reps: int = 5):
        n3, n2, n1 = shape
        out = (C.c_double * 10)()
        self._check(lib().pf_unet_time_layers(self.h, n1, n2, n3, int(reps), out))
        return list(out)

    def warmstart(self, solver: "Solver", dT: float, log10_s: float, mode: str = "nucleus",
                  stream: int = 0):
        """Write the prediction into the solver's current phi: 'nucleus'
        (default) only on the water cells connected to the current nucleus
        (phi > 1/2), 'all' everywhere, 'flood' the baseline without the
        network (phi = 1 on the nucleus's component)."""
        solver._check(lib().pf_warmstart(solver.h, self.h, float(dT), float(log10_s),
                                         WARM_MODES[mode], int(stream)))


def conv3_bf16(x, w, b, relu: bool, cout: int):
    """Building block: y = act(conv3x3x3(x) + b); x (n3, n2, n1, cin) as
    int16 bit patterns of BF16 (CUDA), w (cout, 27, cin) FP32 CUDA, b (cout,)
    FP32 CUDA or None.  Returns y (n3, n2, n1, cout) BF16 bits."""
    import torch
    n3, n2, n1, cin = x.shape
    y = torch.empty((n3, n2, n1, cout), dtype=torch.int16, device=x.device)
    rc = lib().pf_conv3_bf16(_dev_ptr(x, torch.int16), cin, _dev_ptr(w, torch.float32),
                             0 if b is None else _dev_ptr(b, torch.float32), 1 if relu else 0,
                             _dev_ptr(y), cout, n1, n2, n3, 0)
    if rc != 0:
        raise PFError(rc, "pf_conv3_bf16 failed")
    return y


def conv3_bf16_noalloc(x, w, b, relu: bool, y, stream: int = 0):
    """Building block without allocation: y = act(conv3x3x3(x) + b) into the
    caller's y (n3, n2, n1, cout) BF16 bits, asynchronous on `stream` (a
    hipStream_t as int; 0 = the null stream).  Shapes as conv3_bf16."""
    import torch
    n3, n2, n1, cin = x.shape
    cout = y.shape[-1]
    assert tuple(y.shape[:3]) == (n3, n2, n1)
    rc = lib().pf_conv3_bf16_noalloc(_dev_ptr(x, torch.int16), cin, _dev_ptr(w, torch.float32),
                                     0 if b is None else _dev_ptr(b, torch.float32),
                                     1 if relu else 0, _dev_ptr(y, torch.int16), cout, n1, n2,
                                     n3, int(stream))
    if rc != 0:
        raise PFError(rc, lib().pf_last_error(None).decode())
    return y


def conv3_bf16_backward(x, w, dy, want_dx: bool = True):
    """Building block: (dx BF16 bits or None, dw FP32, db FP32) for
    y = conv3x3x3(x) + b given dy (n3, n2, n1, cout) BF16 bits."""
    import torch
    n3, n2, n1, cin = x.shape
    cout = dy.shape[-1]
    dx = torch.empty_like(x) if want_dx else None
    dw = torch.empty((cout, 27, cin), dtype=torch.float32, device=x.device)
    db = torch.empty((cout,), dtype=torch.float32, device=x.device)
    rc = lib().pf_conv3_bf16_backward(_dev_ptr(x, torch.int16), cin, _dev_ptr(w, torch.float32),
                                      _dev_ptr(dy, torch.int16), cout, n1, n2, n3,
                                      0 if dx is None else _dev_ptr(dx), _dev_ptr(dw),
                                      _dev_ptr(db), 0)
    if rc != 0:
        raise PFError(rc, "pf_conv3_bf16_backward failed")
    return dx, dw, db


def mfma_probe(a, b):
    """c = a b through one 16x16x32 BF16 matrix-core instruction."""
    import torch
    c = torch.empty((16, 16), dtype=torch.float32, device=a.device)
    rc = lib().pf_mfma_probe(_dev_ptr(a, torch.float32), _dev_ptr(b, torch.float32),
                             _dev_ptr(c), 0)
    if rc != 0:
        raise PFError(rc, "pf_mfma_probe failed")
    return c
