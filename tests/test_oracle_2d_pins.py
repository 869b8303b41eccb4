"""Pins of the oracle's two-dimensional sweep (tensor grid, tensor
Gauss-Hermite rule, tensor natural spline, vector z).

- Table 9 (Example 4) errors reproduced to a few per cent;
- a problem that does not depend on x2 reduces to the one-dimensional sweep;
- Example 5: Margrabe's closed form at the printed values, and the sweep
  against it at the smoothed maturity.
"""
import math

import numpy as np
import pytest
from conftest import read_golden

import workloads as W


@pytest.mark.parametrize("row", [r for r in read_golden("table9_example4.txt") if r[1] == "8"],
                         ids=lambda r: "K%s_N%s_M%s" % tuple(r[:3]))
def test_table9_example4(oracle_lib, row):
    K, N, M = (int(v) for v in row[:3])
    y_ref, z_ref = float(row[3]), float(row[4])
    wl = W.sine_2d(n_x=M + 1, n_t=N, k=K, L=8)
    iy, iz = wl.init_layers()
    y, z, _ = oracle_lib.solve(wl.problem, iy, iz)
    i = wl.node_index()
    ey = abs(y[i] - 0.0)
    ez = math.hypot(z[0, i] - 1.0, z[1, i] - 1.0)
    assert ey == pytest.approx(y_ref, rel=0.01)
    assert ez == pytest.approx(z_ref, rel=0.01)
    # symmetric problem: both components of z agree
    assert abs(z[0, i] - z[1, i]) < 1e-12


def test_x2_independent_problem_reduces_to_1d(oracle_lib):
    # f = y/2 - z1, g = sin(x1 + 1), X = W: the solution does not depend on x2
    # and equals the one-dimensional sine problem; z2 vanishes
    n, N, K, L = 65, 10, 3, 8
    pb2 = dict(d=2, T=1.0, n_t=N, k_y=K, k_z=K, L=L, n_x=[n, 33], x_min=[-8.0, -3.0],
               x_max=[8.0, 5.0], drift=[0.0, 0.0], vol=[[1.0, 0.0], [0.0, 1.0]],
               driver="linear", p=[0.5, -1.0, 0.0, 0.0], picard_max=30, picard_tol=0.0)
    wl1 = W.sine_1d(n_x=n, n_t=N, k=K, L=L)
    iy1, iz1 = wl1.init_layers()
    y1, z1, _ = oracle_lib.solve(wl1.problem, iy1, iz1)
    iy2 = np.repeat(iy1[:, :, None], 33, axis=2).reshape(K, -1)
    iz2 = np.zeros((K, 2, n * 33))
    iz2[:, 0] = np.repeat(iz1[:, 0, :, None], 33, axis=2).reshape(K, -1)
    y2, z2, _ = oracle_lib.solve(pb2, iy2, iz2)
    y2 = y2.reshape(n, 33)
    zz = z2.reshape(2, n, 33)
    assert np.max(np.abs(y2 - y1[:, None])) < 1e-13
    assert np.max(np.abs(zz[0] - z1[0][:, None])) < 1e-13
    assert np.max(np.abs(zz[1])) < 1e-13


def test_margrabe_closed_form_matches_printed_values():
    T, y0, z1, z2 = (float(v) for v in read_golden("example5_margrabe.txt")[0])
    wl = W.exchange_2d(n_x=65, n_t=16, T=T, smooth=False)
    y, (a, b) = wl.exact(0.0, (np.array([math.log(100.0)]), np.array([math.log(100.0)])))
    assert y[0] == pytest.approx(y0, abs=1e-5)
    assert a[0] == pytest.approx(z1, abs=1e-4)
    assert b[0] == pytest.approx(z2, abs=1e-4)


@pytest.mark.parametrize("rho", [0.0, 0.5])
def test_exchange_option_sweep_against_margrabe(oracle_lib, rho):
    # rho = 0.5 exercises the off-diagonal of vol (correlated log-prices)
    wl = W.exchange_2d(n_x=129, n_t=8, k=3, L=8, rho=rho)
    iy, iz = wl.init_layers()
    y, z, _ = oracle_lib.solve(wl.problem, iy, iz)
    ye, ze = wl.exact_at_t0()
    i = wl.node_index()
    assert abs(y[i] - ye[i]) < 1e-5
    assert abs(z[0, i] - ze[0, i]) < 1e-4 and abs(z[1, i] - ze[1, i]) < 1e-4


def test_sampled_first_step_equals_whole_grid_step(oracle_lib):
    # the sampled entry (used at grid sizes where a whole serial step takes
    # minutes) returns the whole-grid sweep's first layer bit for bit, at
    # corners, edges, a ragged interior and points whose nodes leave the box
    wl = W.basket_2d(n_x=41, n_t=12, k=3, L=6)
    pb = dict(wl.problem)
    pb["n_x"] = [41, 37]
    pb["x_max"] = [pb["x_max"][0], pb["x_min"][1] + 36 * (pb["x_max"][1] - pb["x_min"][1]) / 40]
    rng = np.random.default_rng(7)  # any layers: the two paths must agree exactly
    K, n = 3, 41 * 37
    iy = rng.standard_normal((K, n))
    iz = rng.standard_normal((K, 2, n))
    y, z, _ = oracle_lib.solve(pb, iy, iz, n_stop=pb["n_t"] - K)
    idx = np.array([0, 36, 40 * 37, 41 * 37 - 1, 18, 20 * 37, 20 * 37 + 36, 777, 1000, 1234])
    ys, zs = oracle_lib.first_step_points_2d(pb, iy, iz, idx)
    assert np.array_equal(ys, y[idx])
    assert np.array_equal(zs[0], z[0, idx]) and np.array_equal(zs[1], z[1, idx])
    with pytest.raises(ValueError):
        oracle_lib.first_step_points_2d(pb, iy, iz, np.array([41 * 37]))


# ----------------------------------------------------------------------------
# The paper's own 2-D interpolation: bicubic with finite-difference derivatives
# ----------------------------------------------------------------------------


def _example4_errors(oracle_lib, K, N, M, interp):
    wl = W.sine_2d(n_x=M + 1, n_t=N, k=K, L=8)
    wl.problem["interp"] = interp
    iy, iz = wl.init_layers()
    y, z, _ = oracle_lib.solve(wl.problem, iy, iz)
    i = wl.node_index()
    return abs(y[i]), math.hypot(z[0, i] - 1.0, z[1, i] - 1.0)


@pytest.mark.parametrize("row", read_golden("table9_example4_k1.txt"),
                         ids=lambda r: "K%s_N%s_M%s" % tuple(r[:3]))
def test_table9_k1_rows_with_the_bicubic(oracle_lib, row):
    # K = 1: y to the printed digits, z to 1% from N = 16 on (the coarsest
    # grid, M = 46 with dx = 0.35, differs by 11%); the tensor spline is
    # further off in z at every N
    K, N, M = (int(v) for v in row[:3])
    y_ref, z_ref = float(row[3]), float(row[4])
    ey, ez = _example4_errors(oracle_lib, K, N, M, "bicubic_fd")
    assert ey == pytest.approx(y_ref, rel=0.01)
    assert ez == pytest.approx(z_ref, rel=0.01 if N >= 16 else 0.15)
    _, ez_spline = _example4_errors(oracle_lib, K, N, M, "spline")
    assert abs(ez - z_ref) < abs(ez_spline - z_ref)


@pytest.mark.parametrize("row", [r for r in read_golden("table9_example4.txt") if r[1] == "8"],
                         ids=lambda r: "K%s_N%s_M%s" % tuple(r[:3]))
def test_table9_rows_with_the_bicubic(oracle_lib, row):
    K, N, M = (int(v) for v in row[:3])
    ey, ez = _example4_errors(oracle_lib, K, N, M, "bicubic_fd")
    assert ey == pytest.approx(float(row[3]), rel=0.01)
    assert ez == pytest.approx(float(row[4]), rel=0.01)


def test_bicubic_fd_is_exact_for_cubic_polynomials(oracle_lib):
    # fourth-order differences are exact for cubics (one-sided ones too), and
    # the bicubic Hermite interpolant of a cubic's values and derivatives is
    # the cubic: f = 0, X = W, g(x) = x1^3 + x1 x2^2 gives y = E[g(X_T)] =
    # x1^3 + x1 x2^2 + (T - t)(3 x1 + x1) = x1^3 + x1 x2^2 + 4 x1 (T - t) at
    # points whose domain of dependence (5 steps of nodes at most 1.35 apart)
    # stays inside the grid
    K, N, n = 2, 6, 81
    pb = dict(d=2, T=1.0, n_t=N, k_y=K, k_z=K, L=4, n_x=[n, n], x_min=[-20.0, -20.0],
              x_max=[20.0, 20.0], drift=[0.0, 0.0], vol=[[1.0, 0.0], [0.0, 1.0]],
              driver="linear", p=[0.0, 0.0, 0.0, 0.0], picard_max=30, picard_tol=0.0,
              interp="bicubic_fd")
    x = np.linspace(-20.0, 20.0, n)
    X1, X2 = np.meshgrid(x, x, indexing="ij")
    dt = 1.0 / N

    def exact(t):
        return (X1 ** 3 + X1 * X2 ** 2 + 4.0 * X1 * (1.0 - t),
                3 * X1 ** 2 + X2 ** 2 + 4.0 * (1.0 - t), 2 * X1 * X2)

    iy = np.stack([exact((N - K + 1 + r) * dt)[0].ravel() for r in range(K)])
    iz = np.stack([np.stack([exact((N - K + 1 + r) * dt)[1].ravel(),
                             exact((N - K + 1 + r) * dt)[2].ravel()]) for r in range(K)])
    y, z, _ = oracle_lib.solve(pb, iy, iz)
    ye, z1e, z2e = exact(0.0)
    inner = (np.abs(X1) <= 5.0) & (np.abs(X2) <= 5.0)
    scale = np.maximum(np.abs(ye), 1.0)
    assert np.max((np.abs(y.reshape(n, n) - ye) / scale)[inner]) < 1e-12
    assert np.max(np.abs(z[0].reshape(n, n) - z1e)[inner]) < 1e-11
    assert np.max(np.abs(z[1].reshape(n, n) - z2e)[inner]) < 1e-11

