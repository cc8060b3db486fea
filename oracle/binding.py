"""ctypes binding of the FP64 CPU oracle (test infrastructure only).

The parameter struct below mirrors ``oracle/lbm_oracle.h`` and nothing else; the GPU
library has its own.  A case is described by a plain dict of lattice-unit values (see the
seeded case generators), which is marshalled here field by field.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

FIELDS = ["psi", "ux", "uy", "usx", "usy", "p", "T", "H", "fs", "mdot",
          "psiu_x", "psiu_y", "phi", "fl"]
POPS = {"f": (0, 9), "h": (1, 9), "g": (2, 9), "l": (3, 5), "g_post": (4, 9)}
R_GRAD_S = 1


class OrcParams(C.Structure):
    _fields_ = [
        ("nx", C.c_int), ("ny", C.c_int),
        ("W", C.c_double), ("M", C.c_double), ("gamma", C.c_double),
        ("rho_l", C.c_double), ("rho_g", C.c_double), ("rho_s", C.c_double),
        ("mu_l", C.c_double), ("mu_g", C.c_double), ("mu_s", C.c_double),
        ("cp_l", C.c_double), ("cp_g", C.c_double), ("cp_s", C.c_double),
        ("k_l", C.c_double), ("k_g", C.c_double), ("k_s", C.c_double),
        ("latent", C.c_double),
        ("T_w", C.c_double), ("T_g", C.c_double),
        ("eps_l", C.c_double), ("eps_g", C.c_double), ("eps_s", C.c_double),
        ("sig_l", C.c_double), ("sig_g", C.c_double), ("sig_s", C.c_double),
        ("phi_top", C.c_double), ("phi_bot", C.c_double),
        ("theta_deg", C.c_double),
        ("shape", C.c_int),
        ("R0", C.c_double), ("xc", C.c_double), ("yc", C.c_double), ("h0", C.c_double),
        ("poisson_tol", C.c_double), ("poisson_max_sweeps", C.c_int),
        ("readings", C.c_uint),
    ]


class OrcDiag(C.Structure):
    _fields_ = [
        ("step", C.c_longlong),
        ("sum_psi", C.c_double), ("sum_f", C.c_double), ("sum_g", C.c_double),
        ("V_l", C.c_double), ("V_s", C.c_double),
        ("front_y", C.c_double), ("height", C.c_double), ("max_u", C.c_double),
        ("resid", C.c_double), ("sweeps", C.c_int), ("noconv", C.c_int),
        ("t_fre", C.c_double), ("V_l0", C.c_double), ("nonfinite", C.c_int),
        ("op_resid", C.c_double), ("op_resid_ramp", C.c_double),
    ]


_lib = None


def _bind(L):
    """Declare the argument types of every entry point of an oracle library."""
    dp = C.POINTER(C.c_double)
    L.orc_create.argtypes = [C.POINTER(OrcParams), C.POINTER(C.c_void_p)]
    L.orc_destroy.argtypes = [C.c_void_p]
    L.orc_destroy.restype = None
    L.orc_init.argtypes = [C.c_void_p]
    L.orc_step.argtypes = [C.c_void_p, C.c_int]
    L.orc_solve_potential.argtypes = [C.c_void_p, C.c_double, C.c_int,
                                      C.POINTER(C.c_int), dp]
    L.orc_get_field.argtypes = [C.c_void_p, C.c_int, dp]
    L.orc_set_field.argtypes = [C.c_void_p, C.c_int, dp]
    L.orc_get_pop.argtypes = [C.c_void_p, C.c_int, dp]
    L.orc_set_pop.argtypes = [C.c_void_p, C.c_int, dp]
    L.orc_diagnostics.argtypes = [C.c_void_p, C.POINTER(OrcDiag)]
    L.orc_sweep_log.argtypes = [C.c_void_p, C.POINTER(C.c_int), C.c_int,
                                C.POINTER(C.c_int)]
    L.orc_set_threads.argtypes = [C.c_int]
    L.orc_node_f.argtypes = [C.c_double] * 6 + [dp, dp]
    L.orc_node_f.restype = None
    L.orc_node_h.argtypes = [C.c_double] * 9 + [dp, dp]
    L.orc_node_h.restype = None
    L.orc_node_g.argtypes = [C.c_double] * 6 + [dp]
    L.orc_node_g.restype = None
    L.orc_node_l.argtypes = [C.c_double, dp]
    L.orc_node_l.restype = None
    L.orc_invert_enthalpy.argtypes = [C.POINTER(OrcParams), C.c_double, C.c_double, dp, dp]
    L.orc_stencil.argtypes = [C.POINTER(OrcParams), dp, C.c_int, dp, dp, dp]
    return L


def load(path: str):
    """Another build of the oracle's source (the tests build deliberately broken copies to
    show that the pins catch them); pass the result as `L` to Oracle and the node functions."""
    return _bind(C.CDLL(path))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        _lib = _bind(C.CDLL(LIB_PATH))
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_params(case: dict) -> OrcParams:
    p = OrcParams()
    for name, ctype in OrcParams._fields_:
        if name not in case:
            raise KeyError(f"case is missing '{name}'")
        v = case[name]
        setattr(p, name, int(v) if ctype in (C.c_int, C.c_uint) else float(v))
    return p


def set_threads(n: int, L=None) -> None:
    (L or lib()).orc_set_threads(int(n))


class Oracle:
    """One oracle run.  Mirrors the GPU binding's methods so tests read alike."""

    def __init__(self, case: dict, init: bool = True, L=None):
        self._L = L or lib()
        self.case = dict(case)
        self.params = make_params(case)
        self.nx, self.ny = int(case["nx"]), int(case["ny"])
        h = C.c_void_p()
        rc = self._L.orc_create(C.byref(self.params), C.byref(h))
        if rc != 0:
            raise ValueError(f"orc_create failed ({rc})")
        self._h = h
        if init:
            self.init()

    def close(self):
        if getattr(self, "_h", None):
            self._L.orc_destroy(self._h)
            self._h = None

    __del__ = close

    def init(self):
        rc = self._L.orc_init(self._h)
        if rc != 0:
            raise RuntimeError(f"orc_init failed ({rc})")

    def step(self, n: int = 1):
        rc = self._L.orc_step(self._h, int(n))
        if rc != 0:
            raise RuntimeError(f"orc_step failed ({rc})")

    def solve_potential(self, tol: float, max_sweeps: int):
        k = C.c_int()
        r = C.c_double()
        rc = self._L.orc_solve_potential(self._h, float(tol), int(max_sweeps), C.byref(k), C.byref(r))
        return rc, k.value, r.value

    def field(self, name: str) -> np.ndarray:
        out = np.empty((self.ny, self.nx), dtype=np.float64)
        rc = self._L.orc_get_field(self._h, FIELDS.index(name), _dp(out))
        if rc != 0:
            raise ValueError(name)
        return out

    def set_field(self, name: str, arr):
        a = np.ascontiguousarray(arr, dtype=np.float64).reshape(self.ny, self.nx)
        rc = self._L.orc_set_field(self._h, FIELDS.index(name), _dp(a))
        if rc != 0:
            raise ValueError(name)

    def pop(self, name: str) -> np.ndarray:
        idx, nq = POPS[name]
        out = np.empty((nq, self.ny, self.nx), dtype=np.float64)
        rc = self._L.orc_get_pop(self._h, idx, _dp(out))
        if rc != 0:
            raise ValueError(name)
        return out

    def set_pop(self, name: str, arr):
        idx, nq = POPS[name]
        a = np.ascontiguousarray(arr, dtype=np.float64).reshape(nq, self.ny, self.nx)
        rc = self._L.orc_set_pop(self._h, idx, _dp(a))
        if rc != 0:
            raise ValueError(name)

    def diag(self) -> dict:
        d = OrcDiag()
        self._L.orc_diagnostics(self._h, C.byref(d))
        return {k: getattr(d, k) for k, _ in OrcDiag._fields_}

    def sweep_log(self) -> np.ndarray:
        cnt = C.c_int()
        self._L.orc_sweep_log(self._h, None, 0, C.byref(cnt))
        n = min(cnt.value, 1 << 16)
        buf = (C.c_int * max(n, 1))()
        self._L.orc_sweep_log(self._h, buf, n, C.byref(cnt))
        return np.array(buf[:n], dtype=np.int64)


# ---- node-level pieces -------------------------------------------------------------------

def node_f(psi, ux, uy, Ax, Ay, mdot, L=None):
    feq = np.empty(9); F = np.empty(9)
    (L or lib()).orc_node_f(psi, ux, uy, Ax, Ay, mdot, _dp(feq), _dp(F))
    return feq, F


def node_h(p, rho, ux, uy, S, Ftx, Fty, Gx, Gy, L=None):
    heq = np.empty(9); R = np.empty(9)
    (L or lib()).orc_node_h(p, rho, ux, uy, S, Ftx, Fty, Gx, Gy, _dp(heq), _dp(R))
    return heq, R


def node_g(H, T, Cv, Cref, ux, uy, L=None):
    geq = np.empty(9)
    (L or lib()).orc_node_g(H, T, Cv, Cref, ux, uy, _dp(geq))
    return geq


def node_l(phi, L=None):
    leq = np.empty(5)
    (L or lib()).orc_node_l(phi, _dp(leq))
    return leq


def invert_enthalpy(case: dict, H: float, psi: float, L=None):
    p = make_params(case)
    T = C.c_double(); fl = C.c_double()
    (L or lib()).orc_invert_enthalpy(C.byref(p), float(H), float(psi), C.byref(T), C.byref(fl))
    return T.value, fl.value


def stencil(case: dict, field, ghost: int, L=None):
    p = make_params(case)
    a = np.ascontiguousarray(field, dtype=np.float64)
    gx = np.empty_like(a); gy = np.empty_like(a); lap = np.empty_like(a)
    rc = (L or lib()).orc_stencil(C.byref(p), _dp(a), int(ghost), _dp(gx), _dp(gy), _dp(lap))
    if rc != 0:
        raise ValueError("stencil")
    return gx, gy, lap
