"""FP64 CPU oracle of the pore-scale phase-field freezing model.

TEST INFRASTRUCTURE: only the tests, ``__graft_entry__.smoke()`` and the CPU
baseline of ``bench.py`` use this package.  The product path never imports
it.  It shares no code with the GPU path: ``pf_oracle.c`` is plain C compiled
with gcc, this module only marshals numpy arrays into it.

The arithmetic lives in ``pf_oracle.c`` (see its header for the paper
passages each piece follows); ``brute.py`` is an independent dense-matrix
transcription used to pin it on tiny grids.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Dict, Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MODEL = {"ac": 0, "coupled": 1, "temp": 2}
REACTION = {"sigma": 0, "gradp": 1}
OK, EQUILIBRIUM, MAXSTEPS, NONFINITE, DTMIN = 0, 1, 2, -4, -5


class Params(C.Structure):
    _fields_ = [
        ("n1", C.c_int32), ("n2", C.c_int32), ("n3", C.c_int32),
        ("model", C.c_int32), ("reaction", C.c_int32),
        ("phi_face_mask", C.c_int32), ("dirichlet_faces", C.c_int32),
        ("bc_kind", C.c_int32),
        ("h", C.c_double), ("xi", C.c_double), ("alpha", C.c_double),
        ("mu", C.c_double), ("b", C.c_double), ("eps0", C.c_double),
        ("eps1", C.c_double), ("zeta", C.c_double), ("t_star", C.c_double),
        ("dT", C.c_double), ("gamma", C.c_double),
        ("lam", C.c_double * 3), ("rhoc", C.c_double * 3), ("Lv", C.c_double),
        ("bc_T0", C.c_double), ("bc_T1", C.c_double),
        ("bc_t0", C.c_double), ("bc_t1", C.c_double),
        ("rho_c_separate", C.c_int32), ("pad_", C.c_int32),
        ("rho", C.c_double * 3), ("cs", C.c_double * 3), ("L", C.c_double),
    ]


class Ctl(C.Structure):
    _fields_ = [("tol", C.c_double), ("safety", C.c_double),
                ("dt_min", C.c_double), ("dt_max", C.c_double)]


class StepInfo(C.Structure):
    _fields_ = [("accepted", C.c_int32), ("status", C.c_int32), ("eps", C.c_double),
                ("dt_used", C.c_double), ("dt_next", C.c_double), ("maxk1", C.c_double)]


class RunStats(C.Structure):
    _fields_ = [("steps_accepted", C.c_int64), ("steps_rejected", C.c_int64),
                ("t", C.c_double), ("dt", C.c_double), ("status", C.c_int32),
                ("pad", C.c_int32)]


def build(force: bool = False, openmp: bool = True) -> str:
    """Compile pf_oracle.c with gcc into liboracle.so (next to the source)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fno-fast-math",
               "-ffp-contract=off"]
        if openmp:
            cmd.append("-fopenmp")
        tmp = _LIB + f".tmp{os.getpid()}"
        cmd += [_SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        L.or_rhs.argtypes = [C.POINTER(Params), dp, C.c_double, dp, dp, dp, dp]
        L.or_rhs.restype = None
        L.or_rkm_step.argtypes = [C.POINTER(Params), dp, C.POINTER(Ctl), C.c_double,
                                  C.c_double, dp, dp, dp, C.POINTER(StepInfo)]
        L.or_rkm_step.restype = C.c_int
        L.or_integrate.argtypes = [C.POINTER(Params), dp, C.POINTER(Ctl), C.c_double,
                                   C.c_int64, C.c_double, dp, dp, dp, C.POINTER(RunStats)]
        L.or_integrate.restype = C.c_int
        L.or_diagnostics.argtypes = [C.POINTER(Params), dp, dp, dp, dp]
        L.or_diagnostics.restype = None
        L.or_uwc_bottom_half.argtypes = [C.POINTER(Params), dp, dp, dp, dp]
        L.or_uwc_bottom_half.restype = None
        for name in ("or_sigma",):
            getattr(L, name).argtypes = [C.c_double, C.c_double, C.c_double]
            getattr(L, name).restype = C.c_double
        L.or_water_indicator.argtypes = [C.c_double, C.c_double]
        L.or_water_indicator.restype = C.c_double
        L.or_num_threads.argtypes = []
        L.or_num_threads.restype = C.c_int
        L.or_dirichlet_T.argtypes = [C.POINTER(Params), C.c_double]
        L.or_dirichlet_T.restype = C.c_double
        _lib = L
    return _lib


def _dptr(a: Optional[np.ndarray]):
    if a is None:
        return C.POINTER(C.c_double)()
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_params(p: Dict, model: Optional[str] = None, reaction: str = "sigma") -> Params:
    """Oracle parameter block from a case parameter dict (pf_inputs.Case.params)."""
    m = model or p.get("model", "ac")
    P = Params()
    P.n1, P.n2, P.n3 = int(p["n1"]), int(p["n2"]), int(p["n3"])
    P.model = MODEL[m]
    P.reaction = REACTION[p.get("reaction", reaction)]
    P.phi_face_mask = int(p.get("phi_face_mask", 1))
    P.dirichlet_faces = int(p.get("dirichlet_faces", 0))
    P.bc_kind = int(p.get("bc_kind", 0))
    for k in ("h", "xi", "alpha", "mu", "b", "eps0", "eps1", "zeta", "t_star", "dT", "Lv",
              "bc_T0", "bc_T1", "bc_t0", "bc_t1"):
        setattr(P, k, float(p.get(k, 0.0)))
    P.gamma = float(p.get("gamma", 2.0))
    P.lam[:] = [float(v) for v in p["lam"]]
    P.rhoc[:] = [float(v) for v in p["rhoc"]]
    P.rho_c_separate = int(p.get("rho_c_separate", 0))
    P.rho[:] = [float(v) for v in p.get("rho", (1.0, 1.0, 1.0))]
    P.cs[:] = [float(v) for v in p.get("cs", (1.0, 1.0, 1.0))]
    P.L = float(p.get("L", 0.0))
    return P


def _G(mask_or_G: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(mask_or_G, dtype=np.float64)


def _nvar(P: Params) -> int:
    return 2 if P.model == MODEL["coupled"] else 1


def pack(P: Params, phi, T) -> np.ndarray:
    if P.model == MODEL["ac"]:
        return np.ascontiguousarray(phi, dtype=np.float64).ravel().copy()
    if P.model == MODEL["coupled"]:
        return np.concatenate([np.asarray(phi, np.float64).ravel(),
                               np.asarray(T, np.float64).ravel()])
    return np.ascontiguousarray(T, dtype=np.float64).ravel().copy()


def unpack(P: Params, y: np.ndarray, shape) -> Tuple[Optional[np.ndarray], Optional[np.ndarray]]:
    nc = int(np.prod(shape))
    if P.model == MODEL["ac"]:
        return y[:nc].reshape(shape), None
    if P.model == MODEL["coupled"]:
        return y[:nc].reshape(shape), y[nc:].reshape(shape)
    return None, y[:nc].reshape(shape)


def rhs(P: Params, G, t: float, phi, T=None):
    """(kphi, kT) = F(t, phi, T).  kT is None for the micro-scale model."""
    G = _G(G)
    shape = G.shape
    phi_a = None if phi is None else np.ascontiguousarray(phi, dtype=np.float64)
    T_a = None if T is None else np.ascontiguousarray(T, dtype=np.float64)
    kphi = np.zeros(shape)
    kT = None if P.model == MODEL["ac"] else np.zeros(shape)
    lib().or_rhs(C.byref(P), _dptr(G), t, _dptr(phi_a), _dptr(T_a), _dptr(kphi), _dptr(kT))
    return kphi, kT


def make_ctl(tol=1e-6, safety=0.8, dt_min=1e-12, dt_max=1e30) -> Ctl:
    return Ctl(float(tol), float(safety), float(dt_min), float(dt_max))


def rkm_step(P: Params, G, ctl: Ctl, t: float, dt: float, phi, T=None,
             t_end: float = 1e300, eq_tol: float = 0.0):
    """One Merson attempt.  Returns (phi, T, t, dt, info-dict)."""
    G = _G(G)
    y = pack(P, phi, T)
    tt, dd = C.c_double(t), C.c_double(dt)
    info = StepInfo()
    rc = lib().or_rkm_step(C.byref(P), _dptr(G), C.byref(ctl), t_end, eq_tol,
                           C.byref(tt), C.byref(dd), _dptr(y), C.byref(info))
    if rc:
        raise MemoryError("oracle step failed")
    ph, TT = unpack(P, y, G.shape)
    return ph, TT, tt.value, dd.value, dict(
        accepted=info.accepted, status=info.status, eps=info.eps,
        dt_used=info.dt_used, dt_next=info.dt_next, maxk1=info.maxk1)


def integrate(P: Params, G, ctl: Ctl, t: float, dt: float, phi, T=None,
              t_end: float = 1e300, max_steps: int = 10**12, eq_tol: float = 0.0):
    """Adaptive (or fixed-step when ctl.tol <= 0) integration.
    Returns (phi, T, stats-dict)."""
    G = _G(G)
    y = pack(P, phi, T)
    tt, dd = C.c_double(t), C.c_double(dt)
    st = RunStats()
    rc = lib().or_integrate(C.byref(P), _dptr(G), C.byref(ctl), t_end, int(max_steps),
                            eq_tol, C.byref(tt), C.byref(dd), _dptr(y), C.byref(st))
    if rc:
        raise MemoryError("oracle integrate failed")
    ph, TT = unpack(P, y, G.shape)
    return ph, TT, dict(steps_accepted=st.steps_accepted, steps_rejected=st.steps_rejected,
                        t=st.t, dt=st.dt, status=st.status)


def diagnostics(P: Params, G, phi, T=None) -> Dict[str, float]:
    """Ice count, water-cell count, sum of phi over water cells, enthalpy."""
    G = _G(G)
    out = np.zeros(4)
    phi_a = None if phi is None else np.ascontiguousarray(phi, dtype=np.float64)
    T_a = None if T is None else np.ascontiguousarray(T, dtype=np.float64)
    lib().or_diagnostics(C.byref(P), _dptr(G), _dptr(phi_a), _dptr(T_a), _dptr(out))
    ice, pore = out[0], out[1]
    return dict(ice_count=int(ice), pore_count=int(pore), sum_phi=float(out[2]),
                enthalpy=float(out[3]),
                ice_fraction=float(ice / pore) if pore else 0.0,
                uwc=float(1.0 - ice / pore) if pore else 0.0)


def uwc_bottom_half(P: Params, G, phi, T=None) -> Dict[str, float]:
    """Sec. 3.3 eq. UWC-formula over the cells whose centre lies below half
    the vessel height: water cells (G < 1/2), ice cells among them
    (phi > 1/2) and UWC = 1 - ice / water."""
    G = _G(G)
    out = np.zeros(3)
    phi_a = None if phi is None else np.ascontiguousarray(phi, dtype=np.float64)
    T_a = None if T is None else np.ascontiguousarray(T, dtype=np.float64)
    lib().or_uwc_bottom_half(C.byref(P), _dptr(G), _dptr(phi_a), _dptr(T_a), _dptr(out))
    return dict(water_cells=int(out[0]), ice_cells=int(out[1]), uwc=float(out[2]))


def sigma(w: float, e0: float, e1: float) -> float:
    return lib().or_sigma(w, e0, e1)


def water_indicator(G: float, zeta: float) -> float:
    return lib().or_water_indicator(G, zeta)


def num_threads() -> int:
    return int(lib().or_num_threads())


def dirichlet_T(P: Params, t: float) -> float:
    return lib().or_dirichlet_T(C.byref(P), t)
