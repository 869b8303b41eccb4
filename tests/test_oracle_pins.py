"""Pins of the CPU oracle against facts fixed outside it.

Each test checks the oracle against something it does not compute itself:
values printed in the paper (golden files), a library routine that solves a
special case, exact rational arithmetic from a definition, closed-form
solutions, or invariants of the mathematics.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
from conftest import read_golden
from scipy.interpolate import CubicSpline

import workloads as W

# ----------------------------------------------------------------------------
# Gauss-Hermite rule, eq (21)
# ----------------------------------------------------------------------------


@pytest.mark.parametrize("L", [1, 2, 5, 8, 16, 32, 64])
def test_gauss_hermite_matches_numpy(oracle_lib, L):
    a, w = oracle_lib.gauss_hermite(L)
    a_ref, w_ref = np.polynomial.hermite.hermgauss(L)
    np.testing.assert_allclose(a, a_ref, rtol=0, atol=2e-14 * max(1.0, np.max(abs(a_ref))))
    np.testing.assert_allclose(w, w_ref, rtol=5e-13, atol=1e-300)


@pytest.mark.parametrize("L", [4, 16, 32])
def test_gauss_hermite_gaussian_moments(oracle_lib, L):
    # pi^(-1/2) sum w a^(2m) = E[X^(2m)] for X ~ N(0, 1/2) = (2m-1)!!/2^m, m < L
    a, w = oracle_lib.gauss_hermite(L)
    wh = w / math.sqrt(math.pi)
    for m in range(L):
        exact = 1.0
        for q in range(1, 2 * m, 2):
            exact *= q / 2.0
        got = float(np.sum(wh * a ** (2 * m)))
        assert got == pytest.approx(exact, rel=1e-11), m
        odd = float(np.sum(wh * a ** (2 * m + 1)))
        assert abs(odd) < 1e-12 * max(1.0, exact)


# ----------------------------------------------------------------------------
# Tables 1 and 2
# ----------------------------------------------------------------------------


def _not_a_knot_weights(K: int):
    """Integrals of the K+1 cardinal not-a-knot cubic splines on knots 0..K.

    The spline is written in second-derivative form on unit cells:
    M_{i-1} + 4 M_i + M_{i+1} = 6 (y_{i+1} - 2 y_i + y_{i-1}) inside, third
    derivative continuous at knots 1 and K-1 (not-a-knot); with fewer than
    four knots the interpolant is the polynomial through them.  Returns
    (over [0, K], over [0, 1]) as lists of Fractions, exact.
    """
    def solve(A, b):
        n = len(b)
        M = [row[:] + [b[i]] for i, row in enumerate(A)]
        for c in range(n):
            p = next(r for r in range(c, n) if M[r][c] != 0)
            M[c], M[p] = M[p], M[c]
            for r in range(n):
                if r != c and M[r][c] != 0:
                    f = M[r][c] / M[c][c]
                    M[r] = [x - f * y for x, y in zip(M[r], M[c])]
        return [M[i][n] / M[i][i] for i in range(n)]

    full, first = [], []
    for j in range(K + 1):
        y = [Fraction(int(i == j)) for i in range(K + 1)]
        if K == 1:
            Ms = [Fraction(0)] * 2
        elif K == 2:
            c = y[0] - 2 * y[1] + y[2]
            Ms = [c, c, c]
        else:
            A, b = [], []
            for i in range(1, K):
                row = [Fraction(0)] * (K + 1)
                row[i - 1], row[i], row[i + 1] = Fraction(1), Fraction(4), Fraction(1)
                A.append(row)
                b.append(6 * (y[i + 1] - 2 * y[i] + y[i - 1]))
            for k in (1, K - 1):
                row = [Fraction(0)] * (K + 1)
                row[k - 1], row[k], row[k + 1] = Fraction(1), Fraction(-2), Fraction(1)
                A.append(row)
                b.append(Fraction(0))
            Ms = solve(A, b)
        cell = [(y[i] + y[i + 1]) / 2 - (Ms[i] + Ms[i + 1]) / 24 for i in range(K)]
        full.append(sum(cell) / K)
        first.append(cell[0])
    return full, first


def _printed_tables():
    tab = {}
    for t, K, j, num, den in read_golden("gamma_tables.txt"):
        tab.setdefault((int(t), int(K)), {})[int(j)] = Fraction(int(num), int(den))
    return tab


@pytest.mark.parametrize("K", range(1, 7))
def test_gamma_tables_are_not_a_knot_integrals(oracle_lib, K):
    full, first = _not_a_knot_weights(K)
    printed = _printed_tables()
    assert [printed[(1, K)][j] for j in range(K + 1)] == full
    assert [printed[(2, K)][j] for j in range(K + 1)] == first
    np.testing.assert_allclose(oracle_lib.gamma(1, K), [float(v) for v in full], rtol=1e-15)
    np.testing.assert_allclose(oracle_lib.gamma(2, K), [float(v) for v in first], rtol=1e-15,
                               atol=1e-17)


@pytest.mark.parametrize("K", range(3, 7))
def test_gamma_tables_match_library_spline(oracle_lib, K):
    t = np.arange(K + 1, dtype=float)
    g1 = [CubicSpline(t, np.eye(K + 1)[j], bc_type="not-a-knot").integrate(0, K) / K
          for j in range(K + 1)]
    g2 = [CubicSpline(t, np.eye(K + 1)[j], bc_type="not-a-knot").integrate(0, 1)
          for j in range(K + 1)]
    np.testing.assert_allclose(oracle_lib.gamma(1, K), g1, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(oracle_lib.gamma(2, K), g2, rtol=1e-13, atol=1e-15)


def test_gamma_rows_sum_to_one(oracle_lib):
    for K in range(1, 7):
        assert sum(oracle_lib.gamma(1, K)) == pytest.approx(1.0, abs=1e-15)
        assert sum(oracle_lib.gamma(2, K)) == pytest.approx(1.0, abs=1e-15)


# ----------------------------------------------------------------------------
# Spatial interpolation (natural cubic spline, boundary values outside)
# ----------------------------------------------------------------------------


@pytest.mark.parametrize("n", [4, 7, 33, 1000])
def test_spline_matches_library_natural_spline(oracle_lib, n):
    rng = np.random.default_rng(n)
    x = np.linspace(-2.0, 3.0, n)
    y = np.sin(3 * x) + 0.1 * rng.standard_normal(n)
    X = rng.uniform(-2.0, 3.0, 500)
    X[:3] = [-2.0, 3.0, x[n // 2]]
    ref = CubicSpline(x, y, bc_type="natural")(X)
    got = oracle_lib.spline_eval(y, -2.0, 3.0, X)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13 * np.max(abs(y)))


def test_spline_outside_domain_takes_boundary_values(oracle_lib):
    x = np.linspace(0.0, 1.0, 11)
    y = np.exp(x)
    got = oracle_lib.spline_eval(y, 0.0, 1.0, np.array([-5.0, -1e-9, 1.0 + 1e-9, 7.0]))
    np.testing.assert_array_equal(got, [y[0], y[0], y[-1], y[-1]])


# ----------------------------------------------------------------------------
# The whole scheme against the paper's printed errors
# ----------------------------------------------------------------------------


def _err_at_x0(oracle_lib, wl):
    iy, iz = wl.init_layers()
    y, z, _ = oracle_lib.solve(wl.problem, iy, iz)
    ye, ze = wl.exact_at_t0()
    i = wl.node_index()
    return abs(y[i] - ye[i]), abs(z[0, i] - ze[i])


@pytest.mark.slow
@pytest.mark.parametrize("row", read_golden("table4_example1.txt"), ids=lambda r: "-".join(r[:3]))
def test_table4_example1_errors(oracle_lib, row):
    K, N, M = (int(v) for v in row[:3])
    ey, ez = _err_at_x0(oracle_lib, W.paper_example1(K, N, M))
    # the table prints three significant digits
    assert ey == pytest.approx(float(row[3]), rel=0.02)
    assert ez == pytest.approx(float(row[4]), rel=0.02)


@pytest.mark.slow
@pytest.mark.parametrize("row", read_golden("table5_example2.txt"), ids=lambda r: "-".join(r[:3]))
def test_table5_example2_errors(oracle_lib, row):
    K, N, M = (int(v) for v in row[:3])
    ey, ez = _err_at_x0(oracle_lib, W.paper_example2(K, N, M))
    assert ey == pytest.approx(float(row[3]), rel=0.02)
    assert ez == pytest.approx(float(row[4]), rel=0.02)


def test_grid_rule_reproduces_printed_M():
    for T, xm, K, N, M in read_golden("grid_rule_M.txt"):
        assert W.grid_rule_M(int(K), int(K), int(N), float(T), float(xm)) == int(M)


def test_black_scholes_closed_form_matches_example3():
    (T, K, S0, r, dl, sg, y0, z0), = [[float(v) for v in r] for r in
                                      read_golden("example3_black_scholes.txt")]
    y, z = W.bs_call(T, math.log(S0), K, r, sg, dl)
    assert round(float(y), 4) == y0
    assert round(float(z), 4) == z0


# ----------------------------------------------------------------------------
# Closed forms and special cases
# ----------------------------------------------------------------------------


def test_sine_problem_closed_form(oracle_lib):
    # f = y/2 - z, y = sin(W + t): the default 1025-point, 64-step, k = 2 case
    ey, ez = _err_at_x0(oracle_lib, W.sine_1d())
    assert ey < 1e-4 and ez < 2e-4


@pytest.mark.parametrize("k", [1, 2, 3, 4, 6])
def test_quadratic_terminal_is_reproduced_in_the_interior(oracle_lib, k):
    # f = 0, g = x^2: Gauss-Hermite is exact for quadratics and the spline is
    # exact for them away from the natural boundary condition, so
    # y = x^2 + T - t and z = 2x hold to rounding in the interior.
    # The horizon is short enough that the clamp at +-8 never reaches |x| < 3.
    wl = W.quadratic_heat(k=k, T=0.25)
    iy, iz = wl.init_layers()
    y, z, _ = oracle_lib.solve(wl.problem, iy, iz)
    ye, ze = wl.exact_at_t0()
    inner = np.abs(wl.grid()) < 3.0
    np.testing.assert_allclose(y[inner], ye[inner], rtol=0, atol=1e-12)
    np.testing.assert_allclose(z[0][inner], ze[inner], rtol=0, atol=1e-12)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_space_independent_terminal_gives_zero_z(oracle_lib, k):
    wl = W.discount_const(k=k)
    iy, iz = wl.init_layers()
    y, z, _ = oracle_lib.solve(wl.problem, iy, iz)
    assert np.max(np.abs(z)) < 1e-14
    assert np.ptp(y) < 1e-14
    ye, _ = wl.exact_at_t0()
    assert abs(y[0] - ye[0]) < 1e-5


@pytest.mark.parametrize("k", [1, 2, 3])
def test_time_order_on_space_independent_problem(oracle_lib, k):
    # f = -r y with constant g: the scheme is a linear multistep method for
    # y' = r y; its global error must fall at least like dt^(k+1)
    # (Theorem 1: order min(K_y + 1, 4)).
    errs = []
    for nt in (16, 32, 64):
        wl = W.discount_const(k=k, n_t=nt, r=1.0)
        iy, iz = wl.init_layers()
        y, _, _ = oracle_lib.solve(wl.problem, iy, iz)
        errs.append(abs(y[0] - wl.exact_at_t0()[0][0]))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > k + 1 - 0.3), orders


def test_linear_driver_superposition(oracle_lib):
    # for a linear driver with c = 0 the discrete scheme is linear in the data
    wl = W.sine_1d(n_x=129, n_t=12, k=3, L=8)
    iy, iz = wl.init_layers()
    rng = np.random.default_rng(7)
    dy, dz = rng.standard_normal(iy.shape), rng.standard_normal(iz.shape)
    y1, z1, _ = oracle_lib.solve(wl.problem, iy, iz)
    y2, z2, _ = oracle_lib.solve(wl.problem, dy, dz)
    y3, z3, _ = oracle_lib.solve(wl.problem, iy + 2.0 * dy, iz + 2.0 * dz)
    np.testing.assert_allclose(y3, y1 + 2 * y2, atol=1e-11 * np.max(abs(y3)))
    np.testing.assert_allclose(z3, z1 + 2 * z2, atol=1e-11 * np.max(abs(z3)))


def test_black_scholes_smoothed_problem(oracle_lib):
    # log-price grid with drift and volatility; stability ratio 16
    nx, nt = 2048, 64
    hw = 0.2 * math.sqrt(2 * 0.33 / nt) / 16 * (nx - 1) / 2
    wl = W.bs_call_1d(n_x=nx, n_t=nt, k=3, half_width=hw)
    ey, ez = _err_at_x0(oracle_lib, wl)
    assert ey < 1e-8 and ez < 1e-8


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_bid_ask_call_matches_effective_rate_price(oracle_lib, sign):
    wl = W.bidask_call_1d(n_x=2048, n_t=64, half_width=None, sign=sign)
    ey, ez = _err_at_x0(oracle_lib, wl)
    assert ey < 1e-5 and ez < 1e-6


def test_picard_tolerance_stops_early(oracle_lib):
    wl = W.bidask_call_1d(n_x=257, n_t=16, half_width=None)
    iy, iz = wl.init_layers()
    _, _, st = oracle_lib.solve(wl.problem, iy, iz)
    assert 1 < st["picard_iter_max"] < 10 and st["picard_nonconverged"] == 0


# ----------------------------------------------------------------------------
# The lending branch of the bid-ask driver, and unequal orders K_y != K_z
# ----------------------------------------------------------------------------


def _twin_half_width(sigma, T, n_t, n_x, R=16.0):
    return sigma * math.sqrt(2 * T / n_t) / R * (n_x - 1) / 2


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_bid_ask_put_prices_at_the_lending_rate(oracle_lib, sign):
    # A put's hedge lends (y - z/sigma > 0), so min(y - z/sigma, 0) = 0 and the
    # driver is -r y - theta z whatever the borrowing rate R and the sign s:
    # the exact solution is the Black-Scholes put at the lending rate r.  At
    # the borrowing rate R the price would differ by about 1.1, so a sign or
    # branch error in the min term shows at once.
    nx, nt = 2048, 64
    wl = W.bidask_put_1d(n_x=nx, n_t=nt, sign=sign,
                         half_width=_twin_half_width(0.2, 0.5, nt, nx))
    iy, iz = wl.init_layers()
    y, z, st = oracle_lib.solve(wl.problem, iy, iz)
    ye, ze = wl.exact_at_t0()
    i = wl.node_index()
    assert abs(y[i] - ye[i]) < 1e-5 and abs(z[0, i] - ze[i]) < 1e-8
    tau = wl.problem["T"] + wl.extra["tau_s"]
    y_R, _ = W.bs_put(tau, wl.x0, 100.0, wl.extra["R"], 0.2)
    assert abs(y[i] - y_R) > 0.5
    # the exact solution never reaches the borrowing branch
    assert np.min(ye - ze / 0.2) >= 0.0
    assert st["picard_nonconverged"] == 0


def test_bid_ask_put_does_not_reach_the_borrowing_branch(oracle_lib):
    # min(y - z/sigma, 0) vanishes for a put, so the sign s of the borrowing
    # term must not matter; a branch taken by mistake would move the price
    # towards the rate R (by up to about 1.1 at x0)
    nx, nt = 2048, 32
    out = []
    for sign in (1.0, -1.0):
        wl = W.bidask_put_1d(n_x=nx, n_t=nt, sign=sign,
                             half_width=_twin_half_width(0.2, 0.5, nt, nx))
        iy, iz = wl.init_layers()
        y, z, _ = oracle_lib.solve(wl.problem, iy, iz)
        out.append((y, z[0]))
    assert np.max(np.abs(out[0][0] - out[1][0])) < 1e-12
    assert np.max(np.abs(out[0][1] - out[1][1])) < 1e-12


def _sine_errors(oracle_lib, ky, kz, nt):
    # the sine problem (f = y/2 - z depends on z) on a grid with stability
    # ratio 16: the spatial error stays below the time error
    dx = math.sqrt(2.0 / nt) / 16.0
    nx = int(16.0 / dx) + 1
    nx += 1 - nx % 2  # odd: x = 0 is a node
    wl = W.sine_1d(n_x=nx, n_t=nt, k=ky, L=16)
    wl.problem["k_z"] = kz
    iy, iz = wl.init_layers()
    y, z, _ = oracle_lib.solve(wl.problem, iy, iz)
    ye, ze = wl.exact_at_t0()
    i = wl.node_index()
    return abs(y[i] - ye[i]), abs(z[0, i] - ze[i])


@pytest.mark.slow
@pytest.mark.parametrize("ky,kz", [(3, 1), (1, 3), (2, 4), (4, 2)])
def test_z_order_with_unequal_orders(oracle_lib, ky, kz):
    # Theorem 2: the z error falls like dt^min(K_y + 1, K_z, 3).  The z
    # equation takes row K_z of Table 2 and the y equation row K_y of Table 1
    # with E[y^{n+K_y}]; taking K = max(K_y, K_z) for either, or swapping the
    # rows, changes the observed order (e.g. (3, 1) gives 1, not 3).
    errs = np.array([_sine_errors(oracle_lib, ky, kz, nt)[1] for nt in (16, 32, 64)])
    order = np.log2(errs[:-1] / errs[1:])
    expect = min(ky + 1, kz, 3)
    assert abs(order[-1] - expect) < 0.25, (errs, order)


@pytest.mark.parametrize("ky,kz", [(3, 1), (1, 3)])
def test_y_order_with_unequal_orders_space_independent(oracle_lib, ky, kz):
    # f = -r y, g = 1: z = 0 for any K_z and y follows the row K_y of Table 1
    # alone; the trapezoid row (K_y = 1) is of order 2, the three-eighths row
    # (K_y = 3) of order 4 (Theorem 1: min(K_y + 1, 4)).  Using the row of
    # K_z, or of K = max(K_y, K_z), would swap the two orders.
    errs = []
    for nt in (16, 32, 64, 128):
        wl = W.discount_const(k=ky, n_t=nt, r=1.0)
        wl.problem["k_z"] = kz
        iy, iz = wl.init_layers()
        y, z, _ = oracle_lib.solve(wl.problem, iy, iz)
        assert np.max(np.abs(z)) < 1e-15
        errs.append(abs(y[0] - wl.exact_at_t0()[0][0]))
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert abs(order[-1] - min(ky + 1, 4)) < 0.2, (errs, order)


# ----------------------------------------------------------------------------
# Linear stability in the stability ratio R = vol sqrt(2 dt) / dx
# ----------------------------------------------------------------------------


def _noise_growth(oracle_lib, R, n_t=200, k=4, L=16):
    # the sine problem (f = y/2 - z, X = W) is linear, so the difference of
    # two sweeps whose initial layers differ by grid-scale noise of size 1e-10
    # is that noise as the scheme propagates it (through y and z)
    dx = math.sqrt(2.0 / n_t) / R
    nx = int(6.0 / dx) + 1
    wl = W.sine_1d(n_x=nx, n_t=n_t, k=k, L=L)
    wl.problem.update(x_min=-(nx - 1) * dx / 2, x_max=(nx - 1) * dx / 2)
    iy, iz = wl.init_layers()
    rng = np.random.default_rng(7)
    ny, nz = (1e-10 * rng.standard_normal(a.shape) for a in (iy, iz))
    y0, z0, _ = oracle_lib.solve(wl.problem, iy, iz)
    y1, z1, _ = oracle_lib.solve(wl.problem, iy + ny, iz + nz)
    return max(float(np.max(np.abs(y1 - y0))), float(np.max(np.abs(z1 - z0)))) / 1e-10


def test_stability_ratio_limit():
    # bsde_problem_info flags R above 16; the oracle shows why: at R = 16
    # grid-scale noise in the initial layers is damped, at R = 64 the
    # Gauss-Hermite sums alias it and it grows by orders of magnitude
    import oracle

    oracle.build(force=False)
    stable, unstable = _noise_growth(oracle, 16.0), _noise_growth(oracle, 64.0)
    assert stable < 3.0, stable
    assert unstable > 1e3, unstable


# ----------------------------------------------------------------------------
# Initial layers by the 1-step scheme (Section 3.1 step 2)
# ----------------------------------------------------------------------------


def test_initial_layers_trapezoid_recurrence(oracle_lib):
    # f = -r y, g = 1 (x-independent): z = 0 and the 1-step scheme of eq (20)
    # (K_y = 1: y^n = E[y^{n+1}] + h/2 (f^{n+1} + f^n)) is the trapezoidal
    # rule, y^n = y^{n+1} (1 - r h/2) / (1 + r h/2) with h = dt / sub, so layer
    # t_{N-r} is ((1 - r h/2)/(1 + r h/2))^(r sub) exactly
    r_, sub = 0.7, 5
    wl = W.discount_const(n_x=33, n_t=16, k=4, r=r_)
    wl.problem.update(picard_max=60, picard_tol=1e-15)
    iy_ex, iz_ex = wl.init_layers()
    iy, iz = oracle_lib.initial_layers(wl.problem, iy_ex[-1], iz_ex[-1], sub)
    h = wl.dt() / sub
    q = (1 - r_ * h / 2) / (1 + r_ * h / 2)
    K = wl.K
    for row in range(K):
        steps = (K - 1 - row) * sub
        np.testing.assert_allclose(iy[row], q ** steps, rtol=1e-14)
        assert np.max(np.abs(iz[row])) < 1e-15


def test_initial_layers_one_substep_is_the_one_step_sweep(oracle_lib):
    # with one sub-step the layers are those of the 1-step scheme on the
    # original time grid: a sweep with K_y = K_z = 1 stopped at t_{N-K+1}
    wl = W.bidask_call_1d(n_x=600, n_t=20, half_width=None)
    pb = wl.problem
    iy_ex, iz_ex = wl.init_layers()
    iy, iz = oracle_lib.initial_layers(pb, iy_ex[-1], iz_ex[-1], 1)
    one = dict(pb, k_y=1, k_z=1)
    for row in range(wl.K - 1):
        n_stop = pb["n_t"] - (wl.K - 1 - row)
        y, z, _ = oracle_lib.solve(one, iy_ex[-1:], iz_ex[-1:], n_stop=n_stop)
        assert np.array_equal(iy[row], y) and np.array_equal(iz[row], z)


def test_initial_layers_converge_first_order(oracle_lib):
    # Theorem 2 with K_z = 1: the 1-step scheme's z is first order in its step,
    # so the initial layers approach the exact ones like 1/sub (sine problem,
    # at x = 0, away from the truncated domain's ends)
    wl = W.sine_1d(n_x=1025, n_t=64, k=4)
    iy_ex, iz_ex = wl.init_layers()
    i = wl.node_index()
    errs = []
    for sub in (4, 8, 16):
        iy, iz = oracle_lib.initial_layers(wl.problem, iy_ex[-1], iz_ex[-1], sub)
        errs.append(abs(iz[0, 0, i] - iz_ex[0, 0, i]))
        assert abs(iy[0, i] - iy_ex[0, i]) < 2e-6
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(order - 1.0) < 0.1), (errs, order)


def test_table4_row_with_computed_initial_layers(oracle_lib):
    # Table 4, K = 3, N = 128, M = 4096 (1.44e-11 / 2.77e-8): with initial
    # layers from the 1-step scheme at 16 sub-steps the z error is the printed
    # one to 2%, and y stays within the printed order of magnitude
    wl = W.paper_example1(3, 128, 4096)
    iy_ex, iz_ex = wl.init_layers()
    iy, iz = oracle_lib.initial_layers(wl.problem, iy_ex[-1], iz_ex[-1], 16)
    y, z, _ = oracle_lib.solve(wl.problem, iy, iz)
    i = wl.node_index()
    assert abs(z[0, i] - 0.25) == pytest.approx(2.77e-8, rel=0.02)
    assert abs(y[i] - 0.5) < 1e-10


# ----------------------------------------------------------------------------
# The z form E[y^{n+1} dW]/dt (eq (12) before the relation below it)
# ----------------------------------------------------------------------------


def _sine_errors_zform(oracle_lib, k, nt, z_form):
    dx = math.sqrt(2.0 / nt) / 16.0
    nx = int(16.0 / dx) + 1
    nx += 1 - nx % 2
    wl = W.sine_1d(n_x=nx, n_t=nt, k=k, L=16)
    wl.problem["z_form"] = z_form
    iy, iz = wl.init_layers()
    y, z, _ = oracle_lib.solve(wl.problem, iy, iz)
    ye, ze = wl.exact_at_t0()
    i = wl.node_index()
    return abs(y[i] - ye[i]), abs(z[0, i] - ze[i])


def test_z_form_ydw_second_order_at_one_step(oracle_lib):
    # K = 1: with E[y^{n+1} dW]/dt the z equation is the trapezoidal rule on
    # d/dx y, second order in dt for y and z; the printed form (E[z^{n+1}])
    # is first order there (Theorem 2: min(K_y + 1, K_z, 3) = 1)
    e = np.array([_sine_errors_zform(oracle_lib, 1, nt, "yW") for nt in (16, 32, 64)])
    order = np.log2(e[:-1] / e[1:])
    assert np.all(np.abs(order - 2.0) < 0.1), (e, order)
    e20 = np.array([_sine_errors_zform(oracle_lib, 1, nt, "eq20") for nt in (16, 32, 64)])
    order20 = np.log2(e20[:-1] / e20[1:])
    assert np.all(np.abs(order20[:, 1] - 1.0) < 0.1), (e20, order20)


def test_z_form_ydw_unstable_for_multistep(oracle_lib):
    # K = 2: the multistep z recurrence of Table 2 built on E[y^{n+1} dW]/dt
    # amplifies the O(1/dt) term's errors: refining dt makes the error grow,
    # which is why eq (20) takes dt E[z^{n+1}] in its place
    e = [_sine_errors_zform(oracle_lib, 2, nt, "yW")[1] for nt in (16, 32)]
    assert e[1] > 100 * e[0] and e[1] > 1.0, e
    e20 = [_sine_errors_zform(oracle_lib, 2, nt, "eq20")[1] for nt in (16, 32)]
    assert e20[1] < e20[0] < 2e-3, e20


# ----------------------------------------------------------------------------
# State-dependent forward coefficients (eq (1)): Euler nodes located per point
# ----------------------------------------------------------------------------


@pytest.mark.parametrize("k", [1, 3])
def test_ou_linear_terminal_exact_recurrence(oracle_lib, k):
    # dX = kappa (theta - X) dt + sigma dW, f = 0, g = x.  The Euler node of
    # layer n+k has mean x + kappa (theta - x) k dt; linear data are
    # interpolated exactly (natural spline, M = 0) and Gauss-Hermite sums of
    # linear functions are exact, so y^n = theta + (x - theta) c_n with
    # c_n = (1 - kappa k dt) c_{n+k} from the exact initial layers, at every
    # point whose nodes stay inside the truncated domain
    wl = W.ou_linear_1d(k=k, n_t=32)
    pb = wl.problem
    iy, iz = wl.init_layers()
    y, z, _ = oracle_lib.solve(pb, iy, iz)
    kap, th, N, dt = wl.extra["kappa"], wl.extra["theta"], pb["n_t"], wl.dt()
    c = {N - r: math.exp(-kap * r * dt) for r in range(k)}
    for n in range(N - k, -1, -1):
        c[n] = (1.0 - kap * k * dt) * c[n + k]
    x = wl.grid()
    inner = np.abs(x - th) < 1.5
    np.testing.assert_allclose(y[inner], th + (x[inner] - th) * c[0], rtol=0, atol=1e-12)


def test_ou_z_needs_the_ydw_form(oracle_lib):
    # With a state-dependent drift, E[y^{n+1} dW] = dt E[z^{n+1}] (the relation
    # below eq (12)) no longer holds: for f = 0 the z equation of eq (20)
    # keeps z^n = E[z^{n+1}], so z stays at its terminal value sigma instead
    # of decaying like sigma e^{-kappa (T - t)}; the E[y dW]/dt form (K = 1)
    # follows the decay, first order in dt (the Euler step of X)
    errs = []
    for nt, nx in ((16, 401), (32, 801), (64, 1601)):
        wl = W.ou_linear_1d(k=1, n_t=nt, n_x=nx)
        iy, iz = wl.init_layers()
        i = wl.node_index()
        _, z20, _ = oracle_lib.solve(wl.problem, iy, iz)
        assert abs(z20[0, i] - wl.extra["sigma"]) < 1e-12
        wl.problem["z_form"] = "yW"
        _, z, _ = oracle_lib.solve(wl.problem, iy, iz)
        errs.append(abs(z[0, i] - wl.exact_at_t0()[1][i]))
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(order - 1.0) < 0.15), (errs, order)


def test_black_scholes_on_the_price_grid(oracle_lib):
    # X = S with a(S) = mu S, b(S) = sigma S (the stock-price grid that the
    # paper contrasts with the log-price grid): the Euler nodes give a first
    # order scheme for the Black-Scholes price (weak order of the Euler step)
    errs = []
    for nt in (16, 32, 64):
        dt = 0.33 / nt
        nx = int(300.0 / (0.2 * 300.0 * math.sqrt(2 * dt) / 16.0)) + 1
        wl = W.bs_call_price_1d(n_x=nx, n_t=nt, k=3)
        iy, iz = wl.init_layers()
        y, _, _ = oracle_lib.solve(wl.problem, iy, iz)
        ye, _ = wl.exact_at_t0()
        errs.append(abs(y[wl.node_index()] - ye[wl.node_index()]))
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert errs[-1] < 1e-2 and np.all(np.abs(order - 1.0) < 0.15), (errs, order)


def test_constant_coefficients_reduce_to_the_uniform_path(oracle_lib):
    # drift_x = vol_x = 0 is the constant-coefficient problem
    wl = W.bidask_call_1d(n_x=700, n_t=12, half_width=None)
    iy, iz = wl.init_layers()
    y0, z0, _ = oracle_lib.solve(wl.problem, iy, iz)
    y1, z1, _ = oracle_lib.solve(dict(wl.problem, drift_x=0.0, vol_x=0.0), iy, iz)
    assert np.array_equal(y0, y1) and np.array_equal(z0, z1)


# ----------------------------------------------------------------------------
# Exact Gaussian expectations of the spline (variant of eq (21))
# ----------------------------------------------------------------------------


def test_exact_expectation_closed_forms(oracle_lib):
    # E[sin(c + s xi)] = sin(c) e^{-s^2/2}, E[sin(c + s xi) h xi] = h s cos(c)
    # e^{-s^2/2} (Gaussian integration by parts), up to the spline's
    # interpolation error (dx^4) on a fine grid; constant data give 1 and 0
    # also next to the domain ends (the mass outside goes to the boundary value)
    x = np.linspace(-10.0, 10.0, 4001)
    c = np.array([0.3, 1.0, -2.0])
    sd, h = 0.7, 0.9
    E = oracle_lib.exact_expectation(np.sin(x), np.cos(x), -10.0, 10.0, c, sd, h)
    g = math.exp(-sd * sd / 2)
    np.testing.assert_allclose(E[0], np.sin(c) * g, atol=2e-12)
    np.testing.assert_allclose(E[1], h * sd * np.cos(c) * g, atol=2e-12)
    np.testing.assert_allclose(E[2], np.cos(c) * g, atol=2e-12)
    np.testing.assert_allclose(E[3], -h * sd * np.sin(c) * g, atol=2e-12)
    E = oracle_lib.exact_expectation(np.ones(101), np.full(101, 2.0), 0.0, 1.0,
                                     np.array([0.0, 0.5, 1.0, -3.0]), 0.3, 1.0)
    np.testing.assert_allclose(E[0], 1.0, rtol=1e-14)
    np.testing.assert_allclose(E[2], 2.0, rtol=1e-14)
    assert np.max(np.abs(E[1])) < 1e-14 and np.max(np.abs(E[3])) < 1e-14


def test_exact_expectation_of_a_cubic(oracle_lib):
    # the natural spline of x^3 is x^3 away from the domain ends (the end
    # conditions' influence decays by 0.268 per cell), so the expectations are
    # the Gaussian moments: E[(c + s xi)^3] = c^3 + 3 c s^2 and
    # E[(c + s xi)^3 h xi] = h (3 c^2 s + 3 s^3)
    x = np.linspace(-20.0, 20.0, 4001)
    c = np.array([-1.3, 0.0, 0.7, 2.25])
    sd, h = 0.8, 1.7
    E = oracle_lib.exact_expectation(x ** 3, x ** 2, -20.0, 20.0, c, sd, h)
    np.testing.assert_allclose(E[0], c ** 3 + 3 * c * sd ** 2, rtol=0, atol=1e-10)
    np.testing.assert_allclose(E[1], h * (3 * c ** 2 * sd + 3 * sd ** 3), rtol=0, atol=1e-10)
    np.testing.assert_allclose(E[2], c ** 2 + sd ** 2, rtol=0, atol=1e-10)
    np.testing.assert_allclose(E[3], h * 2 * c * sd, rtol=0, atol=1e-10)


def _noise_growth_exact(oracle_lib, R, quad, n_t=60, k=4):
    dx = math.sqrt(2.0 / n_t) / R
    nx = int(1.5 / dx) + 1
    wl = W.sine_1d(n_x=nx, n_t=n_t, k=k, L=16)
    wl.problem.update(x_min=-(nx - 1) * dx / 2, x_max=(nx - 1) * dx / 2, quad=quad)
    iy, iz = wl.init_layers()
    rng = np.random.default_rng(7)
    ny, nz = (1e-10 * rng.standard_normal(a.shape) for a in (iy, iz))
    # the all-cores build of the oracle: the same arithmetic per point
    y0, z0, _ = oracle_lib.solve(wl.problem, iy, iz, threads=True)
    y1, z1, _ = oracle_lib.solve(wl.problem, iy + ny, iz + nz, threads=True)
    return max(float(np.max(np.abs(y1 - y0))), float(np.max(np.abs(z1 - z0)))) / 1e-10


def test_exact_expectation_stays_stable_at_large_ratio(oracle_lib):
    # at R = 64 Gauss-Hermite (L = 16) aliases grid-scale noise and the sweep
    # amplifies it (x12 over 56 steps here, and without bound as steps are
    # added); the exact expectation damps it (its symbol is the Gaussian's,
    # below 1 for every nonzero frequency)
    gh, ex = _noise_growth_exact(oracle_lib, 64.0, "gh"), _noise_growth_exact(oracle_lib, 64.0, "exact")
    assert gh > 5.0, gh
    assert ex < 1.0, ex


def test_all_cores_oracle_is_the_serial_oracle(oracle_lib):
    # the OpenMP build shares out the points of a layer; each point's
    # arithmetic is unchanged, so the results are identical
    wl = W.bidask_call_1d(n_x=3000, n_t=10, half_width=None)
    iy, iz = wl.init_layers()
    y0, z0, s0 = oracle_lib.solve(wl.problem, iy, iz)
    y1, z1, s1 = oracle_lib.solve(wl.problem, iy, iz, threads=True)
    assert np.array_equal(y0, y1) and np.array_equal(z0, z1) and s0 == s1


# ----------------------------------------------------------------------------
# Forward coefficients tabulated on the grid (eq (1) with any a(t, x), b(t, x))
# ----------------------------------------------------------------------------


@pytest.mark.parametrize("time_dependent", [False, True])
def test_tabulated_coefficients_equal_the_affine_ones(oracle_lib, time_dependent):
    # the Ornstein-Uhlenbeck drift and the stock-price grid's b(S) = sigma S
    # (both pinned above in their affine form) given as tables: the same sweep
    for base in (W.ou_linear_1d(n_x=401, n_t=16), W.bs_call_price_1d(n_x=400, n_t=24)):
        iy, iz = base.init_layers()
        y1, z1, _ = oracle_lib.solve(base.problem, iy, iz)
        t = W.tabulated(base, time_dependent)
        y2, z2, _ = oracle_lib.solve(t.problem, iy, iz)
        assert np.array_equal(y1, y2) and np.array_equal(z1, z2)


def test_tabulated_time_dependent_vol_uses_the_left_point(oracle_lib):
    # dX = sigma(t) dW, g = x^2, f = 0, K = 1: each step adds sigma(t_n)^2 dt at
    # the interior points, so y0 = x^2 + the left Riemann sum of sigma^2; the
    # right sum (coefficients of t_{n+1}) differs by dt (sigma(T)^2 - sigma(0)^2)
    w = W.quadratic_time_varying_vol()
    iy, iz = w.init_layers()
    y, z, _ = oracle_lib.solve(w.problem, iy, iz)
    x = w.grid(0)
    mid = np.abs(x) < 3.0
    left = w.extra["y0_scheme_offset"]
    assert np.max(np.abs(y[mid] - (x[mid] ** 2 + left))) < 1e-7
    dt = w.dt()
    assert dt * (0.75 ** 2 - 0.3 ** 2) > 1e-2
    # and converges at first order in dt to the exact variance integral
    ye, _ = w.exact_at_t0()
    e1 = np.max(np.abs(y[mid] - ye[mid]))
    w2 = W.quadratic_time_varying_vol(n_t=80)
    iy2, iz2 = w2.init_layers()
    y2, _, _ = oracle_lib.solve(w2.problem, iy2, iz2)
    ye2, _ = w2.exact_at_t0()
    e2 = np.max(np.abs(y2[mid] - ye2[mid]))
    assert 1.8 < e1 / e2 < 2.2


def test_tabulated_coefficients_validation(oracle_lib):
    w = W.ou_linear_1d(n_x=101, n_t=8)
    iy, iz = w.init_layers()
    bad = W.tabulated(w)
    bad.problem["coef_tab"] = bad.problem["coef_tab"].copy()
    bad.problem["coef_tab"][0, 1, 50] = 0.0  # b must be positive
    with pytest.raises(ValueError):
        oracle_lib.solve(bad.problem, iy, iz)
    two = W.tabulated(w)
    two.problem["coef_tab"] = np.repeat(two.problem["coef_tab"], 2, axis=0)  # neither 1 nor N rows
    with pytest.raises(ValueError):
        oracle_lib.solve(two.problem, iy, iz)
