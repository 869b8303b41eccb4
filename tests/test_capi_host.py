"""Host-side checks of the C-ABI library (no GPU needed).

The library loads and exports every function declared in include/bsde.h; the
host-only helpers (Gauss-Hermite rule, Tables 1-2) match independent
references; invalid problems are rejected before any device call.
"""
import math
import os
import re
from fractions import Fraction

import numpy as np
import pytest
from conftest import ROOT, read_golden

import paper_1909_13560_amd as B
import workloads as W


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "bsde.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bsde_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = B.load()
    names = _declared_functions()
    assert "bsde_solve" in names and "bsde_plan" in names
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(B.EXPORTED) == sorted(names)


def test_library_has_no_oracle_dependency():
    # the product library must not link or embed the CPU oracle
    data = open(B.LIB_PATH, "rb").read()
    assert b"oracle_solve" not in data and b"bsde_oracle" not in data


@pytest.mark.parametrize("L", [1, 2, 7, 16, 32, 64])
def test_gauss_hermite_rule_matches_numpy(L):
    a, w = B.bsde_gauss_hermite(L)
    a_ref, w_ref = np.polynomial.hermite.hermgauss(L)
    np.testing.assert_allclose(a, a_ref, rtol=0, atol=3e-14 * max(1.0, np.max(abs(a_ref))))
    np.testing.assert_allclose(w, w_ref, rtol=5e-12)
    assert np.sum(w) == pytest.approx(math.sqrt(math.pi), rel=1e-14)


@pytest.mark.parametrize("K", range(1, 7))
def test_gamma_matches_printed_tables(K):
    printed = {}
    for t, k, j, num, den in read_golden("gamma_tables.txt"):
        printed[(int(t), int(k), int(j))] = float(Fraction(int(num), int(den)))
    for table in (1, 2):
        g = B.bsde_gamma(table, K)
        ref = [printed[(table, K, j)] for j in range(K + 1)]
        np.testing.assert_allclose(g, ref, rtol=1e-14, atol=1e-16)


def test_helpers_reject_bad_arguments():
    with pytest.raises(B.BsdeError):
        B.bsde_gauss_hermite(0)
    with pytest.raises(B.BsdeError):
        B.bsde_gauss_hermite(65)
    with pytest.raises(B.BsdeError):
        B.bsde_gamma(3, 2)
    with pytest.raises(B.BsdeError):
        B.bsde_gamma(1, 7)


def test_status_strings():
    for code in range(7):
        assert B.bsde_status_string(code)
    assert B.bsde_status_string(99) == "unknown status"


@pytest.mark.parametrize("field,value", [
    ("k_y", 0), ("k_y", 7), ("k_z", 0), ("L", 0), ("L", 65), ("n_x", 3), ("n_t", 1),
    ("T", -1.0), ("picard_max", 0), ("x_max", -9.0), ("vol", 0.0), ("n_stop", 63),
    ("driver", "bogus"), ("d", 3),
])
def test_plan_rejects_invalid_problems(field, value):
    pb = dict(W.sine_1d().problem)
    if field == "driver":
        s = B.problem_struct(pb)
        s.driver = 9
        arr = (B._Problem * 1)(s)
        import ctypes
        h = ctypes.c_void_p()
        assert B.load().bsde_plan(arr, 1, ctypes.byref(h)) == B.BSDE_EINVAL
        return
    pb[field] = value
    with pytest.raises(B.BsdeError) as e:
        B.bsde_plan(pb)
    assert e.value.code == B.BSDE_EINVAL


def test_plan_rejects_empty_batch():
    import ctypes
    h = ctypes.c_void_p()
    arr = (B._Problem * 1)(B.problem_struct(W.sine_1d().problem))
    assert B.load().bsde_plan(arr, 0, ctypes.byref(h)) == B.BSDE_EINVAL
    assert B.load().bsde_plan(None, 1, ctypes.byref(h)) == B.BSDE_EINVAL


@pytest.mark.parametrize("change", ["vol01", "driver", "fp32_ydw", "exact", "spread"])
def test_plan_2d_reports_unsupported_variants(change):
    # valid two-dimensional problems outside the implemented path are refused
    # before any device call
    pb = dict(W.exchange_2d(n_x=33, n_t=8).problem)
    if change == "vol01":
        pb["vol"] = [[0.25, 0.05], [0.0, 0.3]]
    elif change == "driver":
        pb["driver"] = "cubic"
    elif change == "fp32_ydw":
        pb.update(prec="fp32_comp", z_form="yW", k_y=1, k_z=1)
    elif change == "spread":
        # axis-1 cells of 0.006: the 8 nodes of a row at j = 3 spread over
        # 2 a_max vol11 sqrt(2 j dt) / dx1 = 253 cells, past the 240 of the
        # sweep's LDS window (561 points, 226 cells, passes this check)
        pb["n_x"] = [33, 601]
    else:
        pb["quad"] = "exact"
    with pytest.raises(B.BsdeError) as e:
        B.bsde_plan(pb)
    assert e.value.code == B.BSDE_EUNSUPPORTED


@pytest.mark.parametrize("prec,n_x,limited", [
    ("fp64", 280_000_000, True), ("fp32_comp", 280_000_000, False), ("fp32_comp", 560_000_000, True)])
def test_plan_refuses_ring_planes_past_4gib(prec, n_x, limited):
    # the sweep kernels address a ring plane (16-byte elements in FP64, 8 in
    # FP32) by 32-bit byte offsets; larger grids are refused before any device
    # call, smaller ones get past that check (and here, without a device, fail
    # later or succeed, but not with BSDE_EUNSUPPORTED)
    pb = dict(W.bidask_call_1d(n_x=1024, n_t=16, half_width=None).problem)
    dx = (pb["x_max"] - pb["x_min"]) / 1023  # same cell width, so the nodes stay near
    pb["n_x"] = n_x
    pb["x_max"] = pb["x_min"] + (n_x - 1) * dx
    pb["prec"] = prec
    try:
        B.bsde_plan(pb)
        code = B.BSDE_OK
    except B.BsdeError as e:
        code = e.code
    assert (code == B.BSDE_EUNSUPPORTED) == limited


def test_plan_rejects_mixed_dimensions():
    with pytest.raises(B.BsdeError) as e:
        B.bsde_plan([W.sine_1d().problem, W.sine_2d(n_x=17).problem])
    assert e.value.code == B.BSDE_EINVAL


def test_plan_rejects_invalid_2d_axis():
    pb = dict(W.sine_2d(n_x=17).problem)
    pb["n_x"] = [17, 3]
    with pytest.raises(B.BsdeError) as e:
        B.bsde_plan(pb)
    assert e.value.code == B.BSDE_EINVAL


def test_problem_info_flags_the_stability_ratio():
    # host only: the plan-time stability ratio R = vol sqrt(2 dt)/dx and its
    # flag (R <= 16), for the benchmarked grid, its literal interval and a
    # two-dimensional grid
    cases = [(W.bidask_call_1d(), True), (W.bidask_call_1d(half_width=None), False),
             (W.bidask_call_1d(n_x=3001, n_t=24, half_width=None), False),
             (W.basket_2d(), True), (W.sine_1d(), True)]
    for wl, stable in cases:
        info = B.bsde_problem_info(wl.problem)
        R = W.stability_ratio(wl.problem)
        assert info["stability_ratio"] == pytest.approx(R, rel=1e-12)
        assert info["stable"] == (1 if stable else 0) and info["supported"] == 1
        assert info["K"] == wl.K
    # the literal interval of the benchmark: nodes reach about 9000 cells
    info = B.bsde_problem_info(W.bidask_call_1d(half_width=None).problem)
    assert info["node_reach"] > 9000
    with pytest.raises(B.BsdeError):
        B.bsde_problem_info(dict(W.sine_1d().problem, L=0))
    # a 2-D problem outside the 2-D kernels: reported, not refused
    pb = dict(W.exchange_2d().problem, driver="bidask", p=[0.01, 0.06, 0.2, 0.2, 1.0])
    assert B.bsde_problem_info(pb)["supported"] == 0


def test_problem_info_takes_tabulated_coefficients():
    # the stability ratio follows the table's largest b; invalid tables are
    # refused before any device call
    import numpy as np

    w = W.ou_linear_1d(n_x=401, n_t=16)
    t = W.tabulated(w, time_dependent=True)
    info = B.bsde_problem_info(t.problem)
    dx = (t.problem["x_max"] - t.problem["x_min"]) / 400
    bmax = float(np.max(t.problem["coef_tab"][:, 1]))
    assert info["stability_ratio"] == pytest.approx(bmax * (2 * t.problem["T"] / 16) ** 0.5 / dx,
                                                    rel=1e-12)
    bad = dict(t.problem, coef_tab=t.problem["coef_tab"].copy())
    bad["coef_tab"][3, 1, 7] = -0.1
    with pytest.raises(B.BsdeError) as e:
        B.bsde_problem_info(bad)
    assert e.value.code == B.BSDE_EINVAL
    with pytest.raises(B.BsdeError) as e:  # slopes must be 0 with a table
        B.bsde_problem_info(dict(t.problem, drift_x=0.5))
    assert e.value.code == B.BSDE_EINVAL
    with pytest.raises(B.BsdeError) as e:  # neither 1 nor n_t rows
        B.bsde_problem_info(dict(t.problem, coef_tab=t.problem["coef_tab"][:5]))
    assert e.value.code == B.BSDE_EINVAL
    assert B.bsde_problem_info(dict(t.problem, quad="exact"))["supported"] == 0


def test_stability_flag_tolerates_rounding_of_the_ratio():
    # a grid built for R = 16 computes R = 16 to within a few ulps; it is
    # stable, and R = 16.01 is not
    nx, nt = 3001, 24
    hw = 0.2 * (2 * 0.5 / nt) ** 0.5 / 16.0 * (nx - 1) / 2
    info = B.bsde_problem_info(W.bidask_call_1d(n_x=nx, n_t=nt, half_width=hw).problem)
    assert abs(info["stability_ratio"] - 16.0) < 1e-12 and info["stable"] == 1
    info = B.bsde_problem_info(W.bidask_call_1d(n_x=nx, n_t=nt, half_width=hw / 1.000625).problem)
    assert info["stability_ratio"] > 16.009 and info["stable"] == 0
