"""Python binding of the MI355X library for the multistep BSDE scheme.

Thin ctypes marshalling over the C ABI of ``include/bsde.h``: the functions
below carry the C names and only convert arguments.  Every step of the
backward sweep runs in the HIP kernels of ``libbsde_hip.so``; there is no
CPU fallback, and loading fails loudly when the library is missing.
PyTorch is used only for device memory (tensors) and streams.

A problem is the plain dictionary built by ``workloads`` (keys d, T, n_t,
k_y, k_z, L, n_x, x_min, x_max, drift, vol, driver, p, picard_max,
picard_tol) plus an optional ``prec`` ("fp64" or "fp32_comp").
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbsde_hip.so")

BSDE_OK, BSDE_EINVAL, BSDE_ENOMEM, BSDE_EDEVICE, BSDE_EUNSUPPORTED, BSDE_ENOCONV, \
    BSDE_ENONFINITE, BSDE_ESCRATCH = range(8)
STATIC_WORKSPACE_BYTES = 64 << 20  # BSDE_STATIC_WORKSPACE_BYTES
DRIVERS = {"linear": 0, "bidask": 1, "cubic": 2, "exp": 3}
PRECISIONS = {"fp64": 0, "fp32_comp": 1}
Z_FORMS = {"eq20": 0, "yW": 1}  # bsde_z_form: E[z^{n+1}], E[y^{n+1} dW]/dt
QUADS = {"gh": 0, "exact": 1}  # bsde_quad: Gauss-Hermite (eq (21)), exact Gaussian
INTERPS = {"spline": 0, "bicubic_fd": 1}  # bsde_interp (d = 2: the paper's bicubic)

EXPORTED = ["bsde_plan", "bsde_plan_destroy", "bsde_workspace_bytes", "bsde_solve",
            "bsde_solve_batched", "bsde_profile_kernels", "bsde_status_string",
            "bsde_gauss_hermite", "bsde_gamma", "bsde_autotune", "bsde_problem_info",
            "bsde_initial_layers", "bsde_solve_batched_static", "bsde_checkpoint_layers"]
STABILITY_LIMIT = 16.0  # BSDE_STABILITY_LIMIT


class BsdeError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {bsde_status_string(code)} (status {code})")
        self.code = code


class _Problem(ctypes.Structure):
    _fields_ = [
        ("d", ctypes.c_int),
        ("T", ctypes.c_double),
        ("n_t", ctypes.c_int),
        ("k_y", ctypes.c_int),
        ("k_z", ctypes.c_int),
        ("L", ctypes.c_int),
        ("n_x", ctypes.c_int * 2),
        ("x_min", ctypes.c_double * 2),
        ("x_max", ctypes.c_double * 2),
        ("drift", ctypes.c_double * 2),
        ("vol", ctypes.c_double * 4),
        ("drift_x", ctypes.c_double),
        ("vol_x", ctypes.c_double),
        ("driver", ctypes.c_int),
        ("p", ctypes.c_double * 8),
        ("picard_max", ctypes.c_int),
        ("picard_tol", ctypes.c_double),
        ("prec", ctypes.c_int),
        ("n_stop", ctypes.c_int),
        ("z_form", ctypes.c_int),
        ("quad", ctypes.c_int),
        ("interp", ctypes.c_int),
        ("coef_tab", ctypes.POINTER(ctypes.c_double)),
        ("tab_steps", ctypes.c_int),
    ]


class _Stats(ctypes.Structure):
    _fields_ = [
        ("picard_iter_max", ctypes.c_int),
        ("picard_iter_mean", ctypes.c_double),
        ("picard_nonconverged", ctypes.c_longlong),
        ("nonfinite", ctypes.c_longlong),
        ("stability_ratio", ctypes.c_double),
        ("unstable_instances", ctypes.c_int),
        ("elapsed_ms", ctypes.c_float),
    ]


class _ProblemInfo(ctypes.Structure):
    _fields_ = [("stability_ratio", ctypes.c_double), ("stable", ctypes.c_int),
                ("K", ctypes.c_int), ("node_reach", ctypes.c_int), ("supported", ctypes.c_int)]


class _KernelTimes(ctypes.Structure):
    _fields_ = [("sweep_ms", ctypes.c_double), ("sweep_launches", ctypes.c_int),
                ("spline_ms", ctypes.c_double), ("spline_launches", ctypes.c_int),
                ("path", ctypes.c_int), ("points_per_lane", ctypes.c_int),
                ("node_groups", ctypes.c_int),
                ("blocks", ctypes.c_int), ("lds_bytes", ctypes.c_longlong)]


class _TuneReport(ctypes.Structure):
    _fields_ = [("path", ctypes.c_int), ("points_per_lane", ctypes.c_int),
                ("node_groups", ctypes.c_int), ("best_ms_per_step", ctypes.c_double),
                ("candidates", ctypes.c_int)]


class _Io(ctypes.Structure):
    _fields_ = [("init_y", ctypes.c_void_p), ("init_z", ctypes.c_void_p),
                ("y0", ctypes.c_void_p), ("z0", ctypes.c_void_p)]


_lib = None


def load() -> ctypes.CDLL:
    """Load libbsde_hip.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1909_13560_amd/build.py")
        lib = ctypes.CDLL(LIB_PATH)
        vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int
        lib.bsde_plan.argtypes = [ctypes.POINTER(_Problem), ip, ctypes.POINTER(vp)]
        lib.bsde_plan.restype = ip
        lib.bsde_plan_destroy.argtypes = [vp]
        lib.bsde_plan_destroy.restype = None
        lib.bsde_workspace_bytes.argtypes = [vp]
        lib.bsde_workspace_bytes.restype = ctypes.c_size_t
        lib.bsde_solve.argtypes = [vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(_Stats)]
        lib.bsde_solve.restype = ip
        lib.bsde_solve_batched.argtypes = [vp, vp, ctypes.POINTER(_Io), vp, ctypes.POINTER(_Stats)]
        lib.bsde_solve_batched.restype = ip
        lib.bsde_profile_kernels.argtypes = [vp, vp, ctypes.POINTER(_Io), vp,
                                             ctypes.POINTER(_KernelTimes)]
        lib.bsde_profile_kernels.restype = ip
        lib.bsde_autotune.argtypes = [vp, vp, ctypes.POINTER(_Io), vp, ip,
                                      ctypes.POINTER(_TuneReport)]
        lib.bsde_autotune.restype = ip
        lib.bsde_status_string.argtypes = [ip]
        lib.bsde_status_string.restype = ctypes.c_char_p
        lib.bsde_gauss_hermite.argtypes = [ip, dp, dp]
        lib.bsde_gauss_hermite.restype = ip
        lib.bsde_gamma.argtypes = [ip, ip, dp]
        lib.bsde_gamma.restype = ip
        lib.bsde_problem_info.argtypes = [ctypes.POINTER(_Problem), ctypes.POINTER(_ProblemInfo)]
        lib.bsde_problem_info.restype = ip
        lib.bsde_initial_layers.argtypes = [ctypes.POINTER(_Problem), ip, vp, ctypes.c_size_t,
                                            vp, vp, vp]
        lib.bsde_initial_layers.restype = ip
        lib.bsde_solve_batched_static.argtypes = [vp, ctypes.POINTER(_Io), vp]
        lib.bsde_solve_batched_static.restype = ip
        lib.bsde_checkpoint_layers.argtypes = [vp, vp, ctypes.c_int, vp, vp, vp]
        lib.bsde_checkpoint_layers.restype = ip
        _lib = lib
    return _lib


def _pair(v, fill):
    v = list(v) if isinstance(v, (list, tuple, np.ndarray)) else [v]
    return (v + [fill, fill])[:2]


def problem_struct(pb: dict) -> _Problem:
    s = _Problem()
    s.d = int(pb["d"])
    s.T = float(pb["T"])
    s.n_t = int(pb["n_t"])
    s.k_y = int(pb["k_y"])
    s.k_z = int(pb["k_z"])
    s.L = int(pb["L"])
    s.n_x[:] = [int(v) for v in _pair(pb["n_x"], 0)]
    s.x_min[:] = [float(v) for v in _pair(pb["x_min"], 0.0)]
    s.x_max[:] = [float(v) for v in _pair(pb["x_max"], 0.0)]
    s.drift[:] = [float(v) for v in _pair(pb.get("drift", 0.0), 0.0)]
    vol = np.zeros((2, 2))
    v = np.atleast_2d(np.asarray(pb.get("vol", 1.0), dtype=float))
    vol[: v.shape[0], : v.shape[1]] = v
    s.vol[:] = [float(x) for x in vol.ravel()]
    s.drift_x = float(pb.get("drift_x", 0.0))
    s.vol_x = float(pb.get("vol_x", 0.0))
    s.driver = DRIVERS[pb["driver"]]
    p = list(pb.get("p", [])) + [0.0] * 8
    s.p[:] = [float(x) for x in p[:8]]
    s.picard_max = int(pb.get("picard_max", 30))
    s.picard_tol = float(pb.get("picard_tol", 0.0))
    s.prec = PRECISIONS[pb.get("prec", "fp64")]
    s.n_stop = int(pb.get("n_stop", 0))
    s.z_form = Z_FORMS[pb.get("z_form", "eq20")]
    s.quad = QUADS[pb.get("quad", "gh")]
    s.interp = INTERPS[pb.get("interp", "spline")]
    tab = pb.get("coef_tab")
    if tab is not None:
        # (tab_steps, 2, n_x): rows of a(t, x_i) and b(t, x_i); the struct keeps
        # the array alive while the call that reads it runs
        t = np.ascontiguousarray(tab, dtype=np.float64)
        if t.ndim != 3 or t.shape[1] != 2:
            raise ValueError("coef_tab must have shape (tab_steps, 2, n_x)")
        s.coef_tab = t.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        s.tab_steps = int(t.shape[0])
        s._keep = t
    return s


class Plan:
    """Owns a bsde_plan_t handle."""

    def __init__(self, handle: int, problems: list[dict]):
        self.handle = handle
        self.problems = problems

    def __del__(self):
        # at interpreter exit the module globals may already be gone
        lib = _lib
        if getattr(self, "handle", None) and lib is not None and ctypes is not None:
            lib.bsde_plan_destroy(ctypes.c_void_p(self.handle))
            self.handle = None


# ----------------------------------------------------------------------------
# C ABI, same names
# ----------------------------------------------------------------------------


def bsde_status_string(code: int) -> str:
    return load().bsde_status_string(int(code)).decode()


def bsde_plan(problems) -> Plan:
    """bsde_plan(pb, batch, &out) for a problem dict or a list of them."""
    if isinstance(problems, dict):
        problems = [problems]
    structs = [problem_struct(p) for p in problems]  # they keep any coefficient tables alive
    arr = (_Problem * len(problems))(*structs)
    h = ctypes.c_void_p()
    rc = load().bsde_plan(arr, len(problems), ctypes.byref(h))
    del structs
    if rc != BSDE_OK:
        raise BsdeError(rc, "bsde_plan")
    return Plan(h.value, list(problems))


def bsde_workspace_bytes(plan: Plan) -> int:
    return int(load().bsde_workspace_bytes(ctypes.c_void_p(plan.handle)))


def _stats_dict(st: _Stats) -> dict:
    return {k: getattr(st, k) for k, _ in _Stats._fields_}


def _dptr(t) -> int:
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


def _stream_ptr(stream) -> int | None:
    if stream is None:
        import torch

        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def bsde_solve(plan: Plan, ws, init_y, init_z, y0, z0, stream=None, stats: bool = False,
               check: bool = True):
    """bsde_solve on torch device tensors (float64).  Returns (status, stats or None)."""
    for t in (init_y, init_z, y0, z0):
        if t.dtype != __import__("torch").float64:
            raise TypeError("grid buffers are float64")
    st = _Stats() if stats else None
    rc = load().bsde_solve(ctypes.c_void_p(plan.handle), ctypes.c_void_p(_dptr(ws)),
                           ctypes.c_void_p(_dptr(init_y)), ctypes.c_void_p(_dptr(init_z)),
                           ctypes.c_void_p(_dptr(y0)), ctypes.c_void_p(_dptr(z0)),
                           ctypes.c_void_p(_stream_ptr(stream)),
                           ctypes.byref(st) if st is not None else None)
    if check and rc not in (BSDE_OK, BSDE_ENOCONV, BSDE_ENONFINITE):
        raise BsdeError(rc, "bsde_solve")
    return rc, (_stats_dict(st) if st is not None else None)


def _io_array(ios):
    return (_Io * len(ios))(*[_Io(_dptr(a), _dptr(b), _dptr(c), _dptr(d)) for a, b, c, d in ios])


def bsde_solve_batched(plan: Plan, ws, ios, stream=None, stats: bool = False, check: bool = True):
    """bsde_solve_batched; ``ios`` is a list of (init_y, init_z, y0, z0) tensors."""
    arr = _io_array(ios)
    st = _Stats() if stats else None
    rc = load().bsde_solve_batched(ctypes.c_void_p(plan.handle), ctypes.c_void_p(_dptr(ws)), arr,
                                   ctypes.c_void_p(_stream_ptr(stream)),
                                   ctypes.byref(st) if st is not None else None)
    if check and rc not in (BSDE_OK, BSDE_ENOCONV, BSDE_ENONFINITE):
        raise BsdeError(rc, "bsde_solve_batched")
    return rc, (_stats_dict(st) if st is not None else None)


def bsde_solve_batched_static(plan: Plan, ios, stream=None, check: bool = True) -> int:
    """bsde_solve_batched_static: the batched solve in the library's static
    workspace (allocates nothing).  ``ios`` as for bsde_solve_batched."""
    rc = load().bsde_solve_batched_static(ctypes.c_void_p(plan.handle), _io_array(ios),
                                          ctypes.c_void_p(_stream_ptr(stream)))
    if check and rc not in (BSDE_OK, BSDE_ESCRATCH):
        raise BsdeError(rc, "bsde_solve_batched_static")
    return rc


def bsde_checkpoint_layers(plan: Plan, ws, b: int, layers_y, layers_z, stream=None) -> None:
    """bsde_checkpoint_layers: layers n_stop .. n_stop + K - 1 of instance b into
    device tensors in the initial-layer layout (after a solve with ws)."""
    rc = load().bsde_checkpoint_layers(ctypes.c_void_p(plan.handle), ctypes.c_void_p(_dptr(ws)),
                                       int(b), ctypes.c_void_p(_dptr(layers_y)),
                                       ctypes.c_void_p(_dptr(layers_z)),
                                       ctypes.c_void_p(_stream_ptr(stream)))
    if rc != BSDE_OK:
        raise BsdeError(rc, "bsde_checkpoint_layers")


def bsde_profile_kernels(plan: Plan, ws, ios, stream=None) -> dict:
    """bsde_profile_kernels: per-kernel hipEvent times of one (batched) solve."""
    kt = _KernelTimes()
    rc = load().bsde_profile_kernels(ctypes.c_void_p(plan.handle), ctypes.c_void_p(_dptr(ws)),
                                     _io_array(ios), ctypes.c_void_p(_stream_ptr(stream)),
                                     ctypes.byref(kt))
    if rc != BSDE_OK:
        raise BsdeError(rc, "bsde_profile_kernels")
    return {k: getattr(kt, k) for k, _ in _KernelTimes._fields_}


def bsde_autotune(plan: Plan, ws, ios, stream=None, reps: int = 5) -> dict:
    """bsde_autotune: time the sweep shapes on these buffers and keep the fastest."""
    rep = _TuneReport()
    rc = load().bsde_autotune(ctypes.c_void_p(plan.handle), ctypes.c_void_p(_dptr(ws)),
                              _io_array(ios), ctypes.c_void_p(_stream_ptr(stream)), int(reps),
                              ctypes.byref(rep))
    if rc != BSDE_OK:
        raise BsdeError(rc, "bsde_autotune")
    return {k: getattr(rep, k) for k, _ in _TuneReport._fields_}


def bsde_initial_layers(pb: dict, substeps: int, ws, init_y, init_z, stream=None) -> None:
    """bsde_initial_layers on device tensors: rows 0..K-2 of init_y / init_z from
    row K-1 (the terminal layer) by the 1-step scheme with ``substeps`` steps per dt."""
    rc = load().bsde_initial_layers(ctypes.byref(problem_struct(pb)), int(substeps),
                                    ctypes.c_void_p(_dptr(ws)), ctypes.c_size_t(ws.numel()),
                                    ctypes.c_void_p(_dptr(init_y)), ctypes.c_void_p(_dptr(init_z)),
                                    ctypes.c_void_p(_stream_ptr(stream)))
    if rc != BSDE_OK:
        raise BsdeError(rc, "bsde_initial_layers")


def bsde_problem_info(pb: dict) -> dict:
    """bsde_problem_info: host-only validation and the stability ratio with its flag."""
    info = _ProblemInfo()
    rc = load().bsde_problem_info(ctypes.byref(problem_struct(pb)), ctypes.byref(info))
    if rc != BSDE_OK:
        raise BsdeError(rc, "bsde_problem_info")
    return {k: getattr(info, k) for k, _ in _ProblemInfo._fields_}


def bsde_gauss_hermite(L: int):
    a = np.empty(L)
    w = np.empty(L)
    dp = ctypes.POINTER(ctypes.c_double)
    rc = load().bsde_gauss_hermite(int(L), a.ctypes.data_as(dp), w.ctypes.data_as(dp))
    if rc != BSDE_OK:
        raise BsdeError(rc, "bsde_gauss_hermite")
    return a, w


def bsde_gamma(table: int, K: int):
    g = np.empty(K + 1)
    rc = load().bsde_gamma(int(table), int(K), g.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc != BSDE_OK:
        raise BsdeError(rc, "bsde_gamma")
    return g


# ----------------------------------------------------------------------------
# Convenience: one solve from host arrays (allocation and copies only)
# ----------------------------------------------------------------------------


def workspace(plan: Plan, device="cuda"):
    """A caller-owned workspace tensor, 256-byte aligned (torch allocations are)."""
    import torch

    nbytes = bsde_workspace_bytes(plan)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
    assert ws.data_ptr() % 256 == 0
    return ws


def solve(pb: dict, init_y: np.ndarray, init_z: np.ndarray, device="cuda", stats: bool = True):
    """Plan, copy the K initial layers to the device, solve, copy y0/z0 back."""
    import torch

    plan = bsde_plan(pb)
    ws = workspace(plan, device)
    n = int(np.prod(_pair(pb["n_x"], 1)[: int(pb["d"])]))
    K = max(int(pb["k_y"]), int(pb["k_z"]))
    iy = torch.as_tensor(np.ascontiguousarray(init_y, dtype=np.float64).reshape(K, n), device=device)
    iz = torch.as_tensor(np.ascontiguousarray(init_z, dtype=np.float64).reshape(K, -1), device=device)
    y0 = torch.empty(n, dtype=torch.float64, device=device)
    z0 = torch.empty(iz.shape[1], dtype=torch.float64, device=device)
    rc, st = bsde_solve(plan, ws, iy, iz, y0, z0, stats=stats)
    torch.cuda.synchronize()
    return y0.cpu().numpy(), z0.cpu().numpy().reshape(-1, n), rc, st
