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
