"""Python binding of liblbm.so (the gfx950 HIP library): argument marshalling only.

Every step of the method runs in the library's kernels; PyTorch only provides the device
workspace and the stream.  There is no fallback: if the library is missing or no GPU is
visible, construction raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_ENOCONV, LBM_ENONFINITE, LBM_EHIP, LBM_ESTATE, LBM_ESPACE = 0, -1, -2, -3, -4, -5, -6
FIELDS = ["psi", "ux", "uy", "usx", "usy", "p", "T", "H", "fs", "mdot",
          "psiu_x", "psiu_y", "phi", "fl"]
POPS = {"f": (0, 9), "h": (1, 9), "g": (2, 9), "l": (3, 4)}
PRECISIONS = {"fp64": 0, "fp32": 1, "fp16store": 2}

# every exported symbol of include/lbm.h
SYMBOLS = ["lbm_workspace_bytes", "lbm_init", "lbm_step", "lbm_solve_potential",
           "lbm_diagnostics", "lbm_get_field", "lbm_set_field", "lbm_get_pop", "lbm_set_pop",
           "lbm_sweep_log", "lbm_time_sweeps", "lbm_destroy", "lbm_strerror", "lbm_last_error",
           "lbm_batch_workspace_bytes", "lbm_batch_init", "lbm_batch_step", "lbm_batch_diagnostics",
           "lbm_batch_get_field", "lbm_batch_sweep_log", "lbm_batch_destroy", "lbm_autotune",
           "lbm_nn_param_count", "lbm_nn_workspace_bytes", "lbm_nn_init", "lbm_nn_set_params",
           "lbm_nn_get_params", "lbm_nn_forward", "lbm_nn_gradient", "lbm_nn_train_step",
           "lbm_nn_destroy", "lbm_nn_last_error", "lbm_nn_features", "lbm_nn_target", "lbm_nn_seed",
           "lbm_warm_start", "lbm_set_warm_start", "lbm_batch_nn_sample", "lbm_checkpoint", "lbm_restore",
           "lbm_run_until_frozen", "lbm_batch_run_until_frozen", "lbm_autotune_workspace_bytes",
           "lbm_get_field_device", "lbm_nn_forward_noalloc", "lbm_time_stages", "lbm_stage_name",
           "lbm_batch_warm_start", "lbm_batch_solve_potential", "lbm_launch_shapes", "lbm_time_copy"]

LBM_TUNE_FORCE = 1


class LbmParams(C.Structure):
    _fields_ = [
        ("nx", C.c_int), ("ny", C.c_int), ("precision", C.c_int),
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
        ("sweep_block", C.c_int),
        ("sweep_waves", C.c_int),
        ("skip_initial_solve", C.c_int),
        ("stage_rows", C.c_int),
    ]


LAUNCH_DEFAULTS = {"sweep_block": 0, "sweep_waves": 0, "skip_initial_solve": 0, "stage_rows": 0}


class LbmDiag(C.Structure):
    _fields_ = [
        ("step", C.c_longlong),
        ("sum_psi", C.c_double), ("sum_f", C.c_double), ("sum_g", C.c_double),
        ("V_l", C.c_double), ("V_s", C.c_double),
        ("front_y", C.c_double), ("height", C.c_double), ("max_u", C.c_double),
        ("resid", C.c_double), ("sweeps", C.c_int), ("noconv", C.c_int),
        ("t_fre", C.c_double), ("V_l0", C.c_double), ("nonfinite", C.c_int),
        ("op_resid", C.c_double), ("op_resid_ramp", C.c_double), ("init_converged", C.c_int),
    ]


class LbmTune(C.Structure):
    _fields_ = [
        ("sweep_block", C.c_int), ("sweep_waves", C.c_int), ("cached", C.c_int), ("ncand", C.c_int),
        ("cand_block", C.c_int * 8), ("cand_waves", C.c_int * 8), ("us_per_sweep", C.c_float * 8),
        ("stage_rows", C.c_int), ("nrows", C.c_int), ("cand_rows", C.c_int * 8),
        ("us_per_step_stages", C.c_float * 8),
    ]


class LbmError(RuntimeError):
    def __init__(self, what, code, detail=""):
        self.code = code
        msg = f"{what} failed: {code} ({lib().lbm_strerror(code).decode()})"
        if detail:
            msg += f": {detail}"
        super().__init__(msg)


_lib = None


def lib():
    """Load liblbm.so (built by __graft_entry__.build() or paper_2410_06657_amd/build.py)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it first (python -c "
                               "'import __graft_entry__ as g; g.build()')")
        L = C.CDLL(LIB_PATH)
        vp, dp, ip = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int)
        L.lbm_workspace_bytes.argtypes = [C.POINTER(LbmParams), C.POINTER(C.c_size_t)]
        L.lbm_launch_shapes.argtypes = [C.POINTER(LbmParams), ip, ip, ip]
        L.lbm_time_copy.argtypes = [vp, vp, C.c_size_t, vp, C.c_int, C.POINTER(C.c_float)]
        L.lbm_init.argtypes = [C.POINTER(LbmParams), vp, C.c_size_t, vp, C.POINTER(vp)]
        L.lbm_step.argtypes = [vp, C.c_int]
        L.lbm_solve_potential.argtypes = [vp, C.c_double, C.c_int, ip, dp]
        L.lbm_diagnostics.argtypes = [vp, C.POINTER(LbmDiag)]
        L.lbm_get_field.argtypes = [vp, C.c_int, dp]
        L.lbm_set_field.argtypes = [vp, C.c_int, dp]
        L.lbm_get_pop.argtypes = [vp, C.c_int, dp]
        L.lbm_set_pop.argtypes = [vp, C.c_int, dp]
        L.lbm_sweep_log.argtypes = [vp, ip, C.c_int, ip]
        L.lbm_time_sweeps.argtypes = [vp, C.c_int, C.POINTER(C.c_float)]
        L.lbm_time_stages.argtypes = [vp, C.c_int, C.POINTER(C.c_float), C.c_int, C.POINTER(C.c_int)]
        L.lbm_stage_name.argtypes = [C.c_int]
        L.lbm_stage_name.restype = C.c_char_p
        L.lbm_destroy.argtypes = [vp]
        L.lbm_strerror.argtypes = [C.c_int]
        L.lbm_strerror.restype = C.c_char_p
        L.lbm_last_error.argtypes = [vp]
        L.lbm_last_error.restype = C.c_char_p
        L.lbm_batch_workspace_bytes.argtypes = [C.c_int, C.POINTER(LbmParams), C.POINTER(C.c_size_t)]
        L.lbm_batch_init.argtypes = [C.c_int, C.POINTER(LbmParams), vp, C.c_size_t, vp, C.POINTER(vp)]
        L.lbm_batch_step.argtypes = [vp, C.c_int]
        L.lbm_batch_diagnostics.argtypes = [vp, C.POINTER(LbmDiag)]
        L.lbm_batch_get_field.argtypes = [vp, C.c_int, C.c_int, dp]
        L.lbm_batch_sweep_log.argtypes = [vp, C.c_int, ip, C.c_int, ip]
        L.lbm_batch_destroy.argtypes = [vp]
        L.lbm_autotune_workspace_bytes.argtypes = [C.POINTER(LbmParams), C.POINTER(C.c_size_t)]
        L.lbm_autotune.argtypes = [C.POINTER(LbmParams), vp, C.c_size_t, vp, C.c_int, C.c_int, C.POINTER(LbmTune)]
        L.lbm_get_field_device.argtypes = [vp, C.c_int, vp]
        fp = C.POINTER(C.c_float)
        L.lbm_nn_param_count.argtypes = [ip]
        L.lbm_nn_workspace_bytes.argtypes = [C.c_longlong, C.POINTER(C.c_size_t)]
        L.lbm_nn_init.argtypes = [vp, C.c_size_t, C.c_longlong, C.c_ulonglong, vp, C.POINTER(vp)]
        L.lbm_nn_set_params.argtypes = [vp, fp]
        L.lbm_nn_get_params.argtypes = [vp, fp]
        L.lbm_nn_forward.argtypes = [vp, vp, vp, C.c_int, C.c_int, C.c_int]
        L.lbm_nn_gradient.argtypes = [vp, vp, vp, C.c_int, C.c_int, C.c_int, fp, dp]
        L.lbm_nn_train_step.argtypes = [vp, vp, vp, C.c_int, C.c_int, C.c_int, C.c_float, dp]
        L.lbm_nn_destroy.argtypes = [vp]
        L.lbm_nn_last_error.argtypes = [vp]
        L.lbm_nn_last_error.restype = C.c_char_p
        L.lbm_nn_features.argtypes = [vp, C.c_int, vp]
        L.lbm_nn_target.argtypes = [vp, C.c_int, vp]
        L.lbm_nn_seed.argtypes = [vp, C.c_int, vp]
        L.lbm_warm_start.argtypes = [vp, vp, C.c_int]
        L.lbm_set_warm_start.argtypes = [vp, vp, C.c_int]
        L.lbm_checkpoint.argtypes = [vp, vp, C.POINTER(C.c_size_t)]
        L.lbm_restore.argtypes = [vp, vp, C.c_size_t]
        L.lbm_run_until_frozen.argtypes = [vp, C.c_int, C.c_int, ip]
        L.lbm_batch_run_until_frozen.argtypes = [vp, C.c_int, ip]
        L.lbm_batch_nn_sample.argtypes = [vp, C.c_int, C.c_int, vp, vp]
        L.lbm_batch_warm_start.argtypes = [vp, vp, C.c_int]
        L.lbm_batch_solve_potential.argtypes = [vp, ip]
        _lib = L
    return _lib


def make_params(case: dict, precision: str = "fp64") -> LbmParams:
    p = LbmParams()
    for name, ctype in LbmParams._fields_:
        if name == "precision":
            p.precision = PRECISIONS[precision]
            continue
        if name not in case and name not in LAUNCH_DEFAULTS:
            raise KeyError(f"case is missing '{name}'")
        v = case.get(name, LAUNCH_DEFAULTS.get(name))
        setattr(p, name, int(v) if ctype in (C.c_int, C.c_uint) else float(v))
    return p


def workspace_bytes(case: dict, precision: str = "fp64") -> int:
    p = make_params(case, precision)
    n = C.c_size_t()
    rc = lib().lbm_workspace_bytes(C.byref(p), C.byref(n))
    if rc != LBM_OK:
        raise LbmError("lbm_workspace_bytes", rc)
    return n.value


def launch_shapes(case: dict, precision: str = "fp64") -> dict:
    """The launch shapes a solver of this case takes (lbm_launch_shapes), defaults resolved."""
    p = make_params(case, precision)
    m, w, r = C.c_int(), C.c_int(), C.c_int()
    rc = lib().lbm_launch_shapes(C.byref(p), C.byref(m), C.byref(w), C.byref(r))
    if rc != LBM_OK:
        raise LbmError("lbm_launch_shapes", rc)
    return {"sweep_block": m.value, "sweep_waves": w.value, "stage_rows": r.value}


def time_copy(nbytes: int, reps: int = 10, device: str = "cuda:0") -> float:
    """Average milliseconds of one device-to-device copy of nbytes by the library's streaming
    copy kernel (lbm_time_copy), on fresh torch buffers."""
    import torch
    with torch.cuda.device(torch.device(device)):
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=device)
        dst = torch.empty_like(src)
        ms = C.c_float()
        rc = lib().lbm_time_copy(C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr()), nbytes,
                                 C.c_void_p(torch.cuda.current_stream().cuda_stream), int(reps), C.byref(ms))
        del src, dst
    if rc != LBM_OK:
        raise LbmError("lbm_time_copy", rc)
    return ms.value


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def tune_cache_path() -> str:
    return os.environ.get("LBM_TUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "paper_2410_06657_amd", "launch_shapes.json")


def autotune(case: dict, precision: str = "fp64", launches: int = 20, force: bool = False,
             device: str = "cuda:0", persist: bool = True) -> dict:
    """Fastest launch shapes (potential-sweep shape and stage segment rows) for this grid
    size and precision, from the library's autotuner (lbm_autotune).  Choices are kept in the process (by the library) and
    in a small JSON file (tune_cache_path(), key "nx x ny / precision"), so a shape is timed
    once per machine; force=True re-times."""
    import json

    import torch

    key = f"{int(case['nx'])}x{int(case['ny'])}/{precision}"
    path = tune_cache_path()
    table = {}
    if persist and os.path.exists(path):
        try:
            with open(path) as f:
                table = json.load(f)
        except (OSError, ValueError):
            table = {}
    if not force and key in table:
        return dict(table[key], cached="file")
    p = make_params(case, precision)
    out = LbmTune()
    need = C.c_size_t()
    rc = lib().lbm_autotune_workspace_bytes(C.byref(p), C.byref(need))
    if rc != LBM_OK:
        raise LbmError("lbm_autotune_workspace_bytes", rc)
    with torch.cuda.device(torch.device(device)):
        stream = torch.cuda.current_stream()
        ws = torch.empty(need.value, dtype=torch.uint8, device=device)  # the caller's workspace
        rc = lib().lbm_autotune(C.byref(p), C.c_void_p(ws.data_ptr()), need, C.c_void_p(stream.cuda_stream),
                                int(launches), LBM_TUNE_FORCE if force else 0, C.byref(out))
        del ws
    if rc != LBM_OK:
        raise LbmError("lbm_autotune", rc)
    res = {"sweep_block": out.sweep_block, "sweep_waves": out.sweep_waves, "stage_rows": out.stage_rows,
           "candidates": [{"sweep_block": out.cand_block[k], "sweep_waves": out.cand_waves[k],
                           "us_per_sweep": round(float(out.us_per_sweep[k]), 4)} for k in range(out.ncand)],
           "stage_candidates": [{"stage_rows": out.cand_rows[k],
                                 "us_per_step": round(float(out.us_per_step_stages[k]), 2)}
                                for k in range(out.nrows)]}
    if persist:
        table[key] = res
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + f".{os.getpid()}.tmp"
        with open(tmp, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    return dict(res, cached="library" if out.cached else "")


class Solver:
    """One case on one GPU.  The workspace is a torch uint8 tensor; the stream is torch's
    current stream on `device` at construction."""

    def __init__(self, case: dict, precision: str = "fp64", device: str = "cuda:0", workspace=None,
                 require_converged: bool = False):
        """`precision`: "fp64", "fp32" or "fp16store" (FP32 arithmetic with the f, h and g
        populations stored in binary16).  `workspace`: optional caller-owned uint8 device
        tensor of at least `workspace_bytes(case, precision)` bytes (its contents do not
        matter); by default one is allocated.  An initial potential solve that reaches the
        sweep cap leaves `init_converged` False (lbm_init's LBM_ENOCONV); with
        `require_converged` it raises instead."""
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the HIP library has no CPU path")
        self.case = dict(case)
        self.nx, self.ny = int(case["nx"]), int(case["ny"])
        self.device = torch.device(device)
        self.params = make_params(case, precision)
        nbytes = workspace_bytes(case, precision)
        with torch.cuda.device(self.device):
            if workspace is None:
                self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            else:
                if workspace.dtype != torch.uint8 or workspace.device != self.device or workspace.numel() < nbytes:
                    raise ValueError(f"workspace must be a uint8 tensor on {self.device} of at least {nbytes} bytes")
                self.workspace = workspace
            self.stream = torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        rc = lib().lbm_init(C.byref(self.params), C.c_void_p(self.workspace.data_ptr()),
                            C.c_size_t(nbytes), C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if rc not in (LBM_OK, LBM_ENOCONV):
            raise LbmError("lbm_init", rc)
        self._h = h
        self.init_converged = rc == LBM_OK
        if require_converged and not self.init_converged:
            raise LbmError("lbm_init", rc, f"initial potential solve stopped at the cap "
                                           f"({self.params.poisson_max_sweeps} sweeps)")

    def _check(self, what, rc, ok=(LBM_OK,)):
        if rc not in ok:
            raise LbmError(what, rc, lib().lbm_last_error(self._h).decode())
        return rc

    def close(self):
        if getattr(self, "_h", None):
            lib().lbm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int = 1):
        self._check("lbm_step", lib().lbm_step(self._h, int(n)))

    def solve_potential(self, tol: float, max_sweeps: int):
        k = C.c_int()
        r = C.c_double()
        rc = lib().lbm_solve_potential(self._h, float(tol), int(max_sweeps), C.byref(k), C.byref(r))
        self._check("lbm_solve_potential", rc, ok=(LBM_OK, LBM_ENOCONV))
        return rc, k.value, r.value

    def field(self, name: str) -> np.ndarray:
        out = np.empty((self.ny, self.nx), dtype=np.float64)
        self._check("lbm_get_field", lib().lbm_get_field(self._h, FIELDS.index(name), _dp(out)))
        return out

    def field_device(self, name: str, out=None):
        """One field as a torch FP64 (ny, nx) device tensor, written by the library's kernel
        on the solver's stream (no host copy)."""
        import torch
        if out is None:
            out = torch.empty((self.ny, self.nx), dtype=torch.float64, device=self.device)
        assert out.dtype == torch.float64 and out.is_contiguous() and out.numel() == self.nx * self.ny
        self._check("lbm_get_field_device", lib().lbm_get_field_device(self._h, FIELDS.index(name),
                                                                       C.c_void_p(out.data_ptr())))
        return out

    def set_field(self, name: str, arr):
        a = np.ascontiguousarray(arr, dtype=np.float64).reshape(self.ny, self.nx)
        self._check("lbm_set_field", lib().lbm_set_field(self._h, FIELDS.index(name), _dp(a)))

    def pop(self, name: str) -> np.ndarray:
        idx, nq = POPS[name]
        out = np.empty((nq, self.ny, self.nx), dtype=np.float64)
        self._check("lbm_get_pop", lib().lbm_get_pop(self._h, idx, _dp(out)))
        return out

    def set_pop(self, name: str, arr):
        idx, nq = POPS[name]
        a = np.ascontiguousarray(arr, dtype=np.float64).reshape(nq, self.ny, self.nx)
        self._check("lbm_set_pop", lib().lbm_set_pop(self._h, idx, _dp(a)))

    def diag(self) -> dict:
        d = LbmDiag()
        rc = lib().lbm_diagnostics(self._h, C.byref(d))
        self._check("lbm_diagnostics", rc, ok=(LBM_OK, LBM_ENONFINITE))
        return {k: getattr(d, k) for k, _ in LbmDiag._fields_}

    def time_sweeps(self, n: int) -> float:
        """GPU milliseconds of exactly n sweep launches (HIP events on the solver's stream)."""
        ms = C.c_float()
        self._check("lbm_time_sweeps", lib().lbm_time_sweeps(self._h, int(n), C.byref(ms)))
        return ms.value

    def time_stages(self, n: int) -> dict:
        """Average GPU milliseconds of each stage kernel over n back-to-back launches (HIP
        events on the solver's stream); the state is left as it was."""
        cnt = C.c_int()
        self._check("lbm_time_stages", lib().lbm_time_stages(self._h, int(n), None, 0, C.byref(cnt)))
        ms = (C.c_float * cnt.value)()
        self._check("lbm_time_stages", lib().lbm_time_stages(self._h, int(n), ms, cnt.value, C.byref(cnt)))
        return {lib().lbm_stage_name(k).decode(): float(ms[k]) for k in range(cnt.value)}

    def nn_features(self, factor: int):
        """Coarse input maps of the current state: torch FP32 (ny/f, nx/f, 3) on the device."""
        import torch
        x = torch.empty((self.ny // factor, self.nx // factor, 3), dtype=torch.float32, device=self.device)
        self._check("lbm_nn_features", lib().lbm_nn_features(self._h, int(factor), C.c_void_p(x.data_ptr())))
        return x

    def nn_target(self, factor: int):
        """Coarse potential deviation of the current state: torch FP32 (ny/f, nx/f)."""
        import torch
        t = torch.empty((self.ny // factor, self.nx // factor), dtype=torch.float32, device=self.device)
        self._check("lbm_nn_target", lib().lbm_nn_target(self._h, int(factor), C.c_void_p(t.data_ptr())))
        return t

    def nn_seed(self, factor: int, y):
        """Seed the potential from a coarse deviation map (torch FP32 (ny/f, nx/f) on the device)."""
        y = y.contiguous()
        self._check("lbm_nn_seed", lib().lbm_nn_seed(self._h, int(factor), C.c_void_p(y.data_ptr())))

    def warm_start(self, net: "Net", factor: int):
        """Features -> network -> seeded potential, on this solver's stream."""
        self._check("lbm_warm_start", lib().lbm_warm_start(self._h, net._h, int(factor)))

    def run_until_frozen(self, max_steps: int, check_every: int = 1) -> int:
        """Step until the freezing time is detected; returns the steps taken."""
        k = C.c_int()
        self._check("lbm_run_until_frozen", lib().lbm_run_until_frozen(self._h, int(max_steps), int(check_every),
                                                                       C.byref(k)))
        return k.value

    def checkpoint(self) -> bytes:
        """The whole state as one host image (lbm_checkpoint)."""
        n = C.c_size_t()
        self._check("lbm_checkpoint", lib().lbm_checkpoint(self._h, None, C.byref(n)))
        buf = (C.c_char * n.value)()
        self._check("lbm_checkpoint", lib().lbm_checkpoint(self._h, buf, C.byref(n)))
        return bytes(buf[:n.value])

    def restore(self, image: bytes):
        buf = (C.c_char * len(image)).from_buffer_copy(image)
        self._check("lbm_restore", lib().lbm_restore(self._h, buf, len(image)))

    def set_warm_start(self, net, factor: int = 0):
        """Seed every step's potential solve from `net` (None: the previous step's potential)."""
        self._warm_net = net  # keep the network alive while the library refers to it
        self._check("lbm_set_warm_start", lib().lbm_set_warm_start(self._h, net._h if net else None, int(factor)))

    def sweep_log(self) -> np.ndarray:
        cnt = C.c_int()
        lib().lbm_sweep_log(self._h, None, 0, C.byref(cnt))
        n = cnt.value
        buf = (C.c_int * max(n, 1))()
        lib().lbm_sweep_log(self._h, buf, n, C.byref(cnt))
        return np.array(buf[:n], dtype=np.int64)


class Batch:
    """Many cases advanced together (one launch per stage for all of them).  The stream is a
    dedicated torch stream (default priority) so that the fixed stages can be replayed
    from HIP graphs."""

    def __init__(self, cases: list, precision: str = "fp32", device: str = "cuda:0"):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the HIP library has no CPU path")
        self.cases = [dict(c) for c in cases]
        self.n = len(cases)
        arr = (LbmParams * self.n)(*[make_params(c, precision) for c in cases])
        self._params = arr
        nbytes = C.c_size_t()
        rc = lib().lbm_batch_workspace_bytes(self.n, arr, C.byref(nbytes))
        if rc != LBM_OK:
            raise LbmError("lbm_batch_workspace_bytes", rc)
        self.device = torch.device(device)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
            self.stream = torch.cuda.Stream(self.device)
        torch.cuda.synchronize(self.device)
        h = C.c_void_p()
        rc = lib().lbm_batch_init(self.n, arr, C.c_void_p(self.workspace.data_ptr()), nbytes,
                                  C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if rc != LBM_OK:
            raise LbmError("lbm_batch_init", rc)
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().lbm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int = 1):
        rc = lib().lbm_batch_step(self._h, int(n))
        if rc != LBM_OK:
            raise LbmError("lbm_batch_step", rc)

    def diag(self) -> list:
        arr = (LbmDiag * self.n)()
        rc = lib().lbm_batch_diagnostics(self._h, arr)
        if rc not in (LBM_OK, LBM_ENONFINITE):
            raise LbmError("lbm_batch_diagnostics", rc)
        return [{k: getattr(d, k) for k, _ in LbmDiag._fields_} for d in arr]

    def field(self, c: int, name: str) -> np.ndarray:
        case = self.cases[c]
        out = np.empty((int(case["ny"]), int(case["nx"])), dtype=np.float64)
        rc = lib().lbm_batch_get_field(self._h, int(c), FIELDS.index(name), _dp(out))
        if rc != LBM_OK:
            raise LbmError("lbm_batch_get_field", rc)
        return out

    def run_until_frozen(self, max_steps: int) -> int:
        """Step until every case has frozen (each stops at its own freezing step)."""
        k = C.c_int()
        rc = lib().lbm_batch_run_until_frozen(self._h, int(max_steps), C.byref(k))
        if rc != LBM_OK:
            raise LbmError("lbm_batch_run_until_frozen", rc)
        return k.value

    def warm_start(self, net: "Net", coarse_rows: int = 32):
        """Seed every case's potential from the network (lbm_batch_warm_start)."""
        rc = lib().lbm_batch_warm_start(self._h, net._h, int(coarse_rows))
        if rc != LBM_OK:
            raise LbmError("lbm_batch_warm_start", rc)

    def solve_potential(self) -> int:
        """Every case's potential solve to its own rule; returns the largest sweep count."""
        k = C.c_int()
        rc = lib().lbm_batch_solve_potential(self._h, C.byref(k))
        if rc != LBM_OK:
            raise LbmError("lbm_batch_solve_potential", rc)
        return k.value

    def nn_sample(self, c: int, factor: int):
        """Input maps and target of case c (torch FP32 on the device)."""
        import torch
        case = self.cases[c]
        hc, wc = int(case["ny"]) // factor, int(case["nx"]) // factor
        x = torch.empty((hc, wc, 3), dtype=torch.float32, device=self.device)
        t = torch.empty((hc, wc), dtype=torch.float32, device=self.device)
        rc = lib().lbm_batch_nn_sample(self._h, int(c), int(factor), C.c_void_p(x.data_ptr()),
                                       C.c_void_p(t.data_ptr()))
        if rc != LBM_OK:
            raise LbmError("lbm_batch_nn_sample", rc)
        return x, t

    def sweep_log(self, c: int) -> np.ndarray:
        cnt = C.c_int()
        lib().lbm_batch_sweep_log(self._h, int(c), None, 0, C.byref(cnt))
        n = cnt.value
        buf = (C.c_int * max(n, 1))()
        lib().lbm_batch_sweep_log(self._h, int(c), buf, n, C.byref(cnt))
        return np.array(buf[:n], dtype=np.int64)


class Net:
    """The warm-start network (lbm_nn_*): parameters, forward pass, gradient and Adam steps run
    in the library's kernels on torch's current stream of `device`; inputs and outputs are
    torch FP32 device tensors (x: (n, h, w, 3), y and targets: (n, h, w))."""

    def __init__(self, max_pixels: int, seed: int = 1, device: str = "cuda:0"):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the HIP library has no CPU path")
        self.device = torch.device(device)
        self.max_pixels = int(max_pixels)
        nbytes = C.c_size_t()
        rc = lib().lbm_nn_workspace_bytes(self.max_pixels, C.byref(nbytes))
        if rc != LBM_OK:
            raise LbmError("lbm_nn_workspace_bytes", rc)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
            self.stream = torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        rc = lib().lbm_nn_init(C.c_void_p(self.workspace.data_ptr()), nbytes, self.max_pixels, int(seed),
                               C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if rc != LBM_OK:
            raise LbmError("lbm_nn_init", rc)
        self._h = h
        cnt = C.c_int()
        lib().lbm_nn_param_count(C.byref(cnt))
        self.nparams = cnt.value

    def _check(self, what, rc):
        if rc != LBM_OK:
            raise LbmError(what, rc, lib().lbm_nn_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            lib().lbm_nn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self) -> np.ndarray:
        out = np.empty(self.nparams, dtype=np.float32)
        self._check("lbm_nn_get_params", lib().lbm_nn_get_params(self._h, out.ctypes.data_as(C.POINTER(C.c_float))))
        return out

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.size == self.nparams
        self._check("lbm_nn_set_params", lib().lbm_nn_set_params(self._h, p.ctypes.data_as(C.POINTER(C.c_float))))

    @staticmethod
    def _shape(x):
        n, h, w, c = x.shape
        assert c == 3
        return int(n), int(h), int(w)

    def forward(self, x):
        import torch
        x = x.contiguous()
        n, h, w = self._shape(x)
        y = torch.empty((n, h, w), dtype=torch.float32, device=self.device)
        self._check("lbm_nn_forward", lib().lbm_nn_forward(self._h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                                                           n, h, w))
        return y

    def gradient(self, x, t):
        x, t = x.contiguous(), t.contiguous()
        n, h, w = self._shape(x)
        g = np.empty(self.nparams, dtype=np.float32)
        loss = C.c_double()
        self._check("lbm_nn_gradient", lib().lbm_nn_gradient(self._h, C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()),
                                                             n, h, w, g.ctypes.data_as(C.POINTER(C.c_float)),
                                                             C.byref(loss)))
        return loss.value, g

    def train_step(self, x, t, lr: float, want_loss: bool = False):
        x, t = x.contiguous(), t.contiguous()
        n, h, w = self._shape(x)
        loss = C.c_double()
        self._check("lbm_nn_train_step", lib().lbm_nn_train_step(
            self._h, C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()), n, h, w, float(lr),
            C.byref(loss) if want_loss else None))
        return loss.value if want_loss else None
