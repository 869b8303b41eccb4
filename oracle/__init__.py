"""Python access to the plain serial FP64 CPU oracle (``bsde_oracle.c``).

TEST INFRASTRUCTURE ONLY.  The oracle is imported by the test suite, by the
smoke check and by the CPU-baseline leg of the benchmark, and by nothing else.
It shares no code with the GPU library: it has its own C source, its own
header, its own Gauss-Hermite rule and its own copy of the paper's Tables 1
and 2.  A problem is passed as the plain dictionary that ``workloads`` builds.

What it computes: the fully discrete multistep scheme of arXiv:1909.13560,
Section 2.2 eq (20) with the Gauss-Hermite expectations of eq (21), run as the
backward loop of Section 3.1.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bsde_oracle.c")
_LIB = os.path.join(_HERE, "libbsde_oracle.so")
_LIB_OMP = os.path.join(_HERE, "libbsde_oracle_omp.so")  # the same source, points shared out

DRIVERS = {"linear": 0, "bidask": 1, "cubic": 2, "exp": 3}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no FMA contraction, no fast-math):
    the serial library, and an OpenMP build of the same source that shares the
    grid points of a layer out over the host's cores (same arithmetic per
    point; used for the all-cores baseline)."""
    flags = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-D_DEFAULT_SOURCE",
             "-fPIC", "-shared", "-Wall"]
    for lib, extra in ((_LIB, []), (_LIB_OMP, ["-fopenmp"])):
        if force or not os.path.exists(lib):
            tmp = lib + ".tmp"
            subprocess.check_call(["gcc", *flags, *extra, "-o", tmp, _SRC, "-lm"])
            os.replace(tmp, lib)
    return _LIB


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
        ("n_stop", ctypes.c_int),
        ("z_form", ctypes.c_int),
        ("quad", ctypes.c_int),
        ("interp2", ctypes.c_int),
        ("coef_tab", ctypes.POINTER(ctypes.c_double)),
        ("tab_steps", ctypes.c_int),
    ]


class _Stats(ctypes.Structure):
    _fields_ = [("picard_iter_max", ctypes.c_int), ("picard_nonconverged", ctypes.c_long)]


_libs = {}


def _load(threads: bool = False):
    """The serial oracle, or with ``threads`` its OpenMP build."""
    if threads not in _libs:
        path = _LIB_OMP if threads else _LIB
        if not os.path.exists(path):
            build(force=False)
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_solve.argtypes = [ctypes.POINTER(_Problem), dp, dp, dp, dp,
                                     ctypes.POINTER(_Stats)]
        lib.oracle_solve.restype = ctypes.c_int
        lib.oracle_gauss_hermite.argtypes = [ctypes.c_int, dp, dp]
        lib.oracle_gauss_hermite.restype = ctypes.c_int
        lib.oracle_gamma.argtypes = [ctypes.c_int, ctypes.c_int, dp]
        lib.oracle_gamma.restype = ctypes.c_int
        lib.oracle_spline_eval.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                           dp, ctypes.c_int, dp, dp]
        lib.oracle_spline_eval.restype = ctypes.c_int
        lib.oracle_first_step_points_2d.argtypes = [
            ctypes.POINTER(_Problem), dp, dp, ctypes.c_int, ctypes.POINTER(ctypes.c_long), dp, dp]
        lib.oracle_first_step_points_2d.restype = ctypes.c_int
        lib.oracle_initial_layers.argtypes = [ctypes.POINTER(_Problem), ctypes.c_int, dp, dp]
        lib.oracle_initial_layers.restype = ctypes.c_int
        lib.oracle_exact_expectation.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                                 dp, dp, ctypes.c_int, dp, ctypes.c_double,
                                                 ctypes.c_double, dp]
        lib.oracle_exact_expectation.restype = ctypes.c_int
        _libs[threads] = lib
    return _libs[threads]


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _pair(v, fill):
    v = list(v) if isinstance(v, (list, tuple, np.ndarray)) else [v]
    return (v + [fill, fill])[:2]


def _to_struct(pb: dict, n_stop: int) -> _Problem:
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
    s.n_stop = int(n_stop)
    s.z_form = {"eq20": 0, "yW": 1}[pb.get("z_form", "eq20")]
    s.quad = {"gh": 0, "exact": 1}[pb.get("quad", "gh")]
    s.interp2 = {"spline": 0, "bicubic_fd": 1}[pb.get("interp", "spline")]
    tab = pb.get("coef_tab")
    if tab is not None:  # (tab_steps, 2, n_x), kept alive by the struct
        t = np.ascontiguousarray(tab, dtype=np.float64)
        if t.ndim != 3 or t.shape[1] != 2:
            raise ValueError("coef_tab must have shape (tab_steps, 2, n_x)")
        s.coef_tab = t.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        s.tab_steps = int(t.shape[0])
        s._keep = t
    return s


def solve(pb: dict, init_y: np.ndarray, init_z: np.ndarray, n_stop: int = 0,
          threads: bool = False):
    """Run the backward sweep down to layer ``n_stop``.

    ``init_y``: (K, points) layers t_{N-K+1} .. t_N;  ``init_z``: (K, d, points).
    Returns ``(y, z, stats)`` with y of shape (points,) and z of shape (d, points).
    ``threads``: the OpenMP build (d = 1: the points of a layer on all cores).
    """
    lib = _load(threads)
    d = int(pb["d"])
    npts = int(np.prod(_pair(pb["n_x"], 1)[:d]))
    K = max(int(pb["k_y"]), int(pb["k_z"]))
    iy = np.ascontiguousarray(init_y, dtype=np.float64).reshape(K, npts)
    iz = np.ascontiguousarray(init_z, dtype=np.float64).reshape(K, d, npts)
    y = np.empty(npts)
    z = np.empty((d, npts))
    st = _Stats()
    s = _to_struct(pb, n_stop)
    rc = lib.oracle_solve(ctypes.byref(s), _ptr(iy), _ptr(iz), _ptr(y), _ptr(z), ctypes.byref(st))
    if rc != 0:
        raise ValueError(f"oracle_solve failed with code {rc}")
    return y, z, {"picard_iter_max": st.picard_iter_max,
                  "picard_nonconverged": st.picard_nonconverged}


def initial_layers(pb: dict, terminal_y: np.ndarray, terminal_z: np.ndarray, sub: int):
    """Section 3.1 step 2: the K initial layers t_{N-K+1} .. t_N from the
    terminal layer, the other K - 1 by the 1-step scheme with ``sub`` steps per
    dt.  ``terminal_y``: (points,); ``terminal_z``: (d, points).  Returns
    (init_y, init_z) of shapes (K, points) and (K, d, points)."""
    lib = _load()
    d = int(pb["d"])
    npts = int(np.prod(_pair(pb["n_x"], 1)[:d]))
    K = max(int(pb["k_y"]), int(pb["k_z"]))
    iy = np.zeros((K, npts))
    iz = np.zeros((K, d, npts))
    iy[K - 1] = np.asarray(terminal_y, dtype=np.float64).reshape(npts)
    iz[K - 1] = np.asarray(terminal_z, dtype=np.float64).reshape(d, npts)
    rc = lib.oracle_initial_layers(ctypes.byref(_to_struct(pb, 0)), int(sub), _ptr(iy), _ptr(iz))
    if rc != 0:
        raise ValueError(f"oracle_initial_layers failed with code {rc}")
    return iy, iz


def first_step_points_2d(pb: dict, init_y: np.ndarray, init_z: np.ndarray, idx):
    """The first backward step (layer N-K) of a d = 2 problem at the flat grid
    indices ``idx`` (i0 * n_x[1] + i1), with the arithmetic of ``solve``.

    Returns ``(y, z)`` with y of shape (m,) and z of shape (2, m).  For checks
    at grid sizes where a whole step of the serial oracle takes minutes.
    """
    lib = _load()
    if int(pb["d"]) != 2:
        raise ValueError("first_step_points_2d needs a d = 2 problem")
    n0, n1 = (int(v) for v in pb["n_x"])
    K = max(int(pb["k_y"]), int(pb["k_z"]))
    iy = np.ascontiguousarray(init_y, dtype=np.float64).reshape(K, n0 * n1)
    iz = np.ascontiguousarray(init_z, dtype=np.float64).reshape(K, 2, n0 * n1)
    ix = np.ascontiguousarray(idx, dtype=np.int64).ravel()
    y = np.empty(ix.size)
    z = np.empty((ix.size, 2))
    s = _to_struct(pb, int(pb["n_t"]) - K)
    rc = lib.oracle_first_step_points_2d(
        ctypes.byref(s), _ptr(iy), _ptr(iz), int(ix.size),
        ix.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), _ptr(y), _ptr(z))
    if rc != 0:
        raise ValueError(f"oracle_first_step_points_2d failed with code {rc}")
    return y, np.ascontiguousarray(z.T)


def gauss_hermite(L: int):
    """Nodes and weights of the L-point Gauss-Hermite rule for exp(-x^2)."""
    lib = _load()
    a = np.empty(L)
    w = np.empty(L)
    rc = lib.oracle_gauss_hermite(int(L), _ptr(a), _ptr(w))
    if rc != 0:
        raise ValueError(f"oracle_gauss_hermite failed with code {rc}")
    return a, w


def gamma(table: int, K: int):
    """Row K of Table 1 (table=1) or Table 2 (table=2) as floats."""
    lib = _load()
    g = np.empty(K + 1)
    if lib.oracle_gamma(int(table), int(K), _ptr(g)) != 0:
        raise ValueError("bad gamma table request")
    return g


def exact_expectation(y, z, x_min: float, x_max: float, c, sd: float, h: float):
    """The oracle's exact Gaussian expectations of the natural splines of y and
    z at X = c + sd xi: rows E[yhat], E[yhat h xi], E[zhat], E[zhat h xi]."""
    lib = _load()
    y = np.ascontiguousarray(y, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    c = np.ascontiguousarray(np.atleast_1d(c), dtype=np.float64)
    out = np.empty((c.size, 4))
    rc = lib.oracle_exact_expectation(len(y), float(x_min), float(x_max), _ptr(y), _ptr(z),
                                      int(c.size), _ptr(c), float(sd), float(h), _ptr(out))
    if rc != 0:
        raise ValueError(f"oracle_exact_expectation failed with code {rc}")
    return out.T.copy()


def spline_eval(y: np.ndarray, x_min: float, x_max: float, X: np.ndarray):
    """The oracle's natural spline of ``y`` on a uniform grid, evaluated at X."""
    lib = _load()
    y = np.ascontiguousarray(y, dtype=np.float64)
    X = np.ascontiguousarray(X, dtype=np.float64)
    out = np.empty_like(X)
    rc = lib.oracle_spline_eval(len(y), float(x_min), float(x_max), _ptr(y), len(X),
                                _ptr(X), _ptr(out))
    if rc != 0:
        raise ValueError(f"oracle_spline_eval failed with code {rc}")
    return out
