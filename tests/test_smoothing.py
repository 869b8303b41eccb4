"""The Kreiss-type smoothing of non-smooth terminal data (Section 5, Example 3)
and the study of it against the time shift, on the oracle.

The smoothing operators are input preparation (the terminal layer the scheme
starts from), so they live with the seeded inputs; here they are pinned to
their definitions by independent integration and to their moment conditions.
The study then runs the oracle's whole algorithm (the method's own initial
layers from the terminal layer, Section 3.1 step 2, then eq (20)) on a call
whose terminal condition has a kink in y and a jump in z at the strike.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad

import workloads as W
from test_gpu_parity import twin_half_width


@pytest.mark.parametrize("order", [2, 4])
def test_kernel_moments(order):
    # integral 1, odd moments 0; second moment 1/6 for the hat, 0 for order 4
    # (so that smooth data change by O(h^4)); fourth moment of order 4 nonzero
    s = 1 if order == 2 else 3
    pts = list(range(-s, s + 1))
    m = [quad(lambda t: t ** q * float(W.kreiss_kernel(t, order)), -s, s, points=pts)[0]
         for q in range(5)]
    assert abs(m[0] - 1.0) < 1e-13 and abs(m[1]) < 1e-13 and abs(m[3]) < 1e-13
    assert abs(m[2] - (1.0 / 6.0 if order == 2 else 0.0)) < 1e-13
    if order == 4:
        assert abs(m[4]) > 1e-3
    # the kernel is continuous and vanishes at the ends of its support
    t = np.array([-s, s], dtype=float)
    assert np.all(W.kreiss_kernel(t, order) == 0.0)


def test_order_four_reproduces_cubics_and_order_two_lines():
    x = np.linspace(-1.0, 1.0, 7)
    h = 0.05
    cubic = lambda u: 1.0 - 2.0 * u + 0.5 * u ** 2 + 3.0 * u ** 3
    np.testing.assert_allclose(W.kreiss_smooth(cubic, x, h, 4), cubic(x), rtol=0, atol=1e-14)
    line = lambda u: 2.0 - 3.0 * u
    np.testing.assert_allclose(W.kreiss_smooth(line, x, h, 2), line(x), rtol=0, atol=1e-14)
    # the hat keeps a quadratic's curvature term: M_h u^2 = u^2 + h^2/6
    np.testing.assert_allclose(W.kreiss_smooth(lambda u: u * u, x, h, 2), x * x + h * h / 6.0,
                               rtol=0, atol=1e-15)


@pytest.mark.parametrize("order", [2, 4])
def test_smoothed_kink_and_jump_match_independent_quadrature(order):
    # the call payoff max(e^x - K, 0) and sigma e^x 1{x > ln K} near the strike
    K, sig, h = 100.0, 0.2, 1.3e-3
    lk = math.log(K)
    x = lk + h * np.array([-3.5, -1.0, -0.25, 0.0, 0.4, 1.0, 2.7])
    pay = lambda u: np.maximum(np.exp(u) - K, 0.0)
    jump = lambda u: sig * np.exp(u) * (u > lk)
    s = 1 if order == 2 else 3
    for v, f in ((pay, lambda u: max(math.exp(u) - K, 0.0)),
                 (jump, lambda u: sig * math.exp(u) * (u > lk))):
        got = W.kreiss_smooth(v, x, h, order, (lk,))
        for xi, g in zip(x, got):
            ref = quad(lambda t: float(W.kreiss_kernel(t, order)) * f(xi - h * t), -s, s,
                       points=sorted(set(range(-s, s + 1)) | {(xi - lk) / h}), limit=200)[0]
            assert abs(g - ref) <= 1e-12 * max(1.0, abs(ref))
    # |x| at its kink: the hat gives h/3 (2 h int_0^1 t (1 - t) dt)
    assert abs(W.kreiss_smooth(np.abs, np.array([0.0]), h, 2, (0.0,))[0] - h / 3.0) < 1e-16


def test_smoothing_study_on_the_oracle(oracle_lib):
    # Black-Scholes call, 4097 points on the stable interval, N = 64, k = 4,
    # L = 32; the K - 1 initial layers by the 1-step scheme with 8 sub-steps
    nx, nt = 4097, 64
    err = {}
    for term, quads in (("raw", ("gh",)), ("kreiss4", ("gh", "exact")), ("shift", ("gh",))):
        wl = W.bs_call_1d(n_x=nx, n_t=nt, k=4, L=32,
                          half_width=twin_half_width(0.2, 0.33, nt, nx), terminal=term)
        ty, tz = W.terminal_layer(wl)
        ye, ze = wl.exact_at_t0()
        i = wl.node_index()
        for q in quads:
            pb = dict(wl.problem, quad=q)
            iy, iz = oracle_lib.initial_layers(pb, ty, tz, 8)
            y, z, _ = oracle_lib.solve(pb, iy, iz, threads=True)
            err[term, q] = (abs(y[i] - ye[i]), abs(z[0, i] - ze[i]))
            print(term, q, "y0 err %.3e z0 err %.3e" % err[term, q])
    # the raw payoff's jump in z leaves a large z error at the money
    assert err["raw", "gh"][1] > 1e-2
    # smoothing over one cell removes it ...
    assert err["kreiss4", "gh"][1] < 1e-5
    # ... but y keeps the Gauss-Hermite error of the still sharp kink, carried
    # to y0 undamped along the y recurrence (y^n from E[y^{n+K_y}])
    assert err["kreiss4", "gh"][0] > 1e-3
    # exact expectations take it away: y0 and z0 at the level of the time shift
    # (both limited by the first-order start-up layers)
    assert err["kreiss4", "exact"][0] < 1e-6 and err["kreiss4", "exact"][1] < 1e-5
    assert err["shift", "gh"][0] < 1e-6 and err["shift", "gh"][1] < 1e-5
