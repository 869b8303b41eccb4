"""Seeded synthetic inputs shared by the GPU path's tests and the oracle's tests.

This module holds problem descriptions, closed-form solutions and the initial
layers built from them.  It holds none of the multistep scheme's arithmetic:
no quadrature, no interpolation, no time stepping.  Both the GPU binding and
the CPU oracle take the plain dictionaries it returns.

A problem dictionary has the keys
    d, T, n_t, k_y, k_z, L, n_x, x_min, x_max, drift, vol, driver, p,
    picard_max, picard_tol
with the forward process X_{t+h} = X_t + drift*h + vol*(W_{t+h} - W_t)
(X = W: drift 0, vol 1; log-price, eq (33): drift mu - sigma^2/2, vol sigma)
and the driver kinds
    "linear"  p = [a, b1, b2, c]          f = a y + b1 z1 + b2 z2 + c
    "bidask"  p = [r, R, theta, sigma, s] f = -r y - theta z + s (R-r) min(y - z/sigma, 0)
    "cubic"   Example 1, eq (22)
    "exp"     Example 2, eq (24)
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable

import numpy as np
from scipy.special import ndtr

# ----------------------------------------------------------------------------
# Closed forms
# ----------------------------------------------------------------------------


def sine_solution(t, x):
    """y = sin(x + t), z = cos(x + t): solves f = y/2 - z with X = W."""
    return np.sin(x + t), np.cos(x + t)


def ex1_solution(t, x):
    """Example 1, eq (23): y = e^{x+t}/(e^{x+t}+1), z = e^{x+t}/(e^{x+t}+1)^2."""
    e = np.exp(-(x + t))  # written with e^{-(x+t)} to stay finite for large x
    y = 1.0 / (1.0 + e)
    return y, y * (1.0 - y)


def ex2_solution(t, x):
    """Example 2, eq (25): y = ln(sin x + 3) e^{t^2}, z = e^{t^2} cos x/(sin x + 3)."""
    et = np.exp(t * t)
    return np.log(np.sin(x) + 3.0) * et, et * np.cos(x) / (np.sin(x) + 3.0)


def bs_call(tau, x, K, r, sigma, delta=0.0):
    """Black-Scholes call on S = e^x with time to expiry tau and dividend yield delta.

    Returns (y, z) with y the price and z = sigma S dV/dS, eq (31) with the
    dividend term kept in d_{1,2}.
    """
    tau = np.asarray(tau, dtype=float)
    S = np.exp(x)
    sq = sigma * np.sqrt(tau)
    d1 = (x - math.log(K) + (r - delta + 0.5 * sigma * sigma) * tau) / sq
    d2 = d1 - sq
    disc_q = np.exp(-delta * tau)
    y = S * disc_q * ndtr(d1) - K * np.exp(-r * tau) * ndtr(d2)
    z = sigma * S * disc_q * ndtr(d1)
    return y, z


def bs_put(tau, x, K, r, sigma, delta=0.0):
    """Black-Scholes put on S = e^x: (price, sigma S dV/dS), written with
    N(-d1), N(-d2) so that both stay accurate far out of the money."""
    tau = np.asarray(tau, dtype=float)
    S = np.exp(x)
    sq = sigma * np.sqrt(tau)
    d1 = (x - math.log(K) + (r - delta + 0.5 * sigma * sigma) * tau) / sq
    d2 = d1 - sq
    disc_q = np.exp(-delta * tau)
    y = K * np.exp(-r * tau) * ndtr(-d2) - S * disc_q * ndtr(-d1)
    z = -sigma * S * disc_q * ndtr(-d1)
    return y, z


def margrabe(tau, x1, x2, sigma1, sigma2, rho):
    """Margrabe exchange option max(S1 - S2, 0), S_k = e^{x_k}; returns (V, dV/dx1, dV/dx2)."""
    s = math.sqrt(sigma1 ** 2 + sigma2 ** 2 - 2 * rho * sigma1 * sigma2)
    S1, S2 = np.exp(x1), np.exp(x2)
    sq = s * np.sqrt(tau)
    d1 = (x1 - x2 + 0.5 * s * s * tau) / sq
    d2 = d1 - sq
    return S1 * ndtr(d1) - S2 * ndtr(d2), S1 * ndtr(d1), -S2 * ndtr(d2)


# ----------------------------------------------------------------------------
# Workload container
# ----------------------------------------------------------------------------


@dataclass
class Workload:
    name: str
    problem: dict
    exact: Callable  # exact(t, x) -> (y, z) on the grid (1-D), or (y, (z1, z2)) (2-D)
    x0: float | tuple = 0.0  # evaluation point of the headline value (a grid node)
    notes: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def K(self) -> int:
        return max(self.problem["k_y"], self.problem["k_z"])

    def grid(self, axis: int = 0) -> np.ndarray:
        pb = self.problem
        n = _as_list(pb["n_x"])[axis]
        lo = _as_list(pb["x_min"])[axis]
        hi = _as_list(pb["x_max"])[axis]
        return lo + np.arange(n) * ((hi - lo) / (n - 1))

    def dt(self) -> float:
        return self.problem["T"] / self.problem["n_t"]

    def init_layers(self):
        """The K newest layers t_{N-K+1}..t_N from the closed form (Section 3.1 step 2).

        Returns (init_y, init_z) of shapes (K, points) and (K, d, points).
        """
        pb = self.problem
        N, K, d = pb["n_t"], self.K, pb["d"]
        dt = self.dt()
        if d == 1:
            x = self.grid(0)
            iy = np.empty((K, x.size))
            iz = np.empty((K, 1, x.size))
            for r in range(K):
                y, z = self.exact((N - K + 1 + r) * dt, x)
                iy[r], iz[r, 0] = y, z
            return iy, iz
        x1, x2 = np.meshgrid(self.grid(0), self.grid(1), indexing="ij")
        iy = np.empty((K, x1.size))
        iz = np.empty((K, 2, x1.size))
        for r in range(K):
            y, (z1, z2) = self.exact((N - K + 1 + r) * dt, (x1, x2))
            iy[r] = np.ravel(y)
            iz[r, 0] = np.ravel(z1)
            iz[r, 1] = np.ravel(z2)
        return iy, iz

    def exact_at_t0(self):
        """Exact (y, z) at t = 0 on the whole grid."""
        if self.problem["d"] == 1:
            return self.exact(0.0, self.grid(0))
        x1, x2 = np.meshgrid(self.grid(0), self.grid(1), indexing="ij")
        y, (z1, z2) = self.exact(0.0, (x1, x2))
        return np.ravel(y), np.stack([np.ravel(z1), np.ravel(z2)])

    def node_index(self) -> int:
        """Flat grid index of x0 (x0 must be a grid node)."""
        if self.problem["d"] == 1:
            x = self.grid(0)
            i = int(round((self.x0 - x[0]) / (x[1] - x[0])))
            assert abs(x[i] - self.x0) < 1e-9 * max(1.0, abs(self.x0)), "x0 is not a node"
            return i
        idx = []
        for a in range(2):
            x = self.grid(a)
            i = int(round((self.x0[a] - x[0]) / (x[1] - x[0])))
            assert abs(x[i] - self.x0[a]) < 1e-9 * max(1.0, abs(self.x0[a]))
            idx.append(i)
        return idx[0] * self.problem["n_x"][1] + idx[1]


def _as_list(v):
    return list(v) if isinstance(v, (list, tuple, np.ndarray)) else [v]


def _problem(**kw) -> dict:
    base = dict(d=1, drift=0.0, vol=1.0, picard_max=30, picard_tol=0.0)
    base.update(kw)
    return base


# ----------------------------------------------------------------------------
# The paper's examples (used as pins of the oracle)
# ----------------------------------------------------------------------------


def paper_example1(K: int, N: int, M: int, L: int = 32, T: float = 1.0) -> Workload:
    """Example 1 (eq (22)-(23)) on [-16, 16] with M intervals, as in Table 4."""
    pb = _problem(T=T, n_t=N, k_y=K, k_z=K, L=L, n_x=M + 1, x_min=-16.0, x_max=16.0,
                  driver="cubic", p=[])
    return Workload(f"ex1_K{K}_N{N}_M{M}", pb, ex1_solution, 0.0)


def paper_example2(K: int, N: int, M: int, L: int = 32, T: float = 1.0) -> Workload:
    """Example 2 (eq (24)-(25)) on [-16, 16] with M intervals, as in Table 5."""
    pb = _problem(T=T, n_t=N, k_y=K, k_z=K, L=L, n_x=M + 1, x_min=-16.0, x_max=16.0,
                  driver="exp", p=[])
    return Workload(f"ex2_K{K}_N{N}_M{M}", pb, ex2_solution, 0.0)


def grid_rule_M(K_y: int, K_z: int, N: int, T: float, x_max: float) -> int:
    """Number of space intervals on [-x_max, x_max] that balances the errors
    (Section 3.1 step 1, with r = 4 for the cubic spline): dx = dt^((q+1)/4)
    with q = min(K_y + 1, K_z, 3), the z order of eq (19)."""
    q = min(K_y + 1, K_z, 3)
    dx = (T / N) ** ((q + 1) / 4.0)
    return 2 * math.ceil(x_max / dx)


# ----------------------------------------------------------------------------
# Workloads of the measured path
# ----------------------------------------------------------------------------


def sine_1d(n_x: int = 1025, n_t: int = 64, k: int = 2, L: int = 16,
            picard_tol: float = 0.0) -> Workload:
    """X = W, T = 1, f = y/2 - z, g = sin(x + 1) on [-8, 8]; exact y = sin(W+t)."""
    pb = _problem(T=1.0, n_t=n_t, k_y=k, k_z=k, L=L, n_x=n_x, x_min=-8.0, x_max=8.0,
                  driver="linear", p=[0.5, -1.0, 0.0, 0.0], picard_tol=picard_tol)
    return Workload(f"sine1d_nx{n_x}_nt{n_t}_k{k}_L{L}", pb, sine_solution, 0.0)


def _snap_domain(c: float, lo: float, hi: float, n_x: int):
    """Shift [lo, hi] (keeping its width) so that c falls on a grid node."""
    dx = (hi - lo) / (n_x - 1)
    i0 = int(round((c - lo) / dx))
    lo = c - i0 * dx
    return lo, lo + (n_x - 1) * dx


# ----------------------------------------------------------------------------
# Smoothing of non-smooth terminal data (Section 5, Example 3: the paper smooths
# the initial condition of the call after Kreiss, Thomee and Widlund (1970)
# without stating the operator).  The operators of that family:
#   (M_h v)(x) = int Phi(t) v(x - h t) dt,
# order 2: Phi the hat function on [-1, 1] (Fourier transform (sin(w/2)/(w/2))^2);
# order 4: Phi = (4/3) B(t) - (1/6) (B(t - 1) + B(t + 1)) with B the cubic
# B-spline on [-2, 2], whose transform is (sin(w/2)/(w/2))^4 (1 + (2/3) sin^2(w/2)):
# it integrates to 1 and has vanishing second moment, so it changes smooth data
# by O(h^4).  With h the grid spacing they act on a cell's scale.
# ----------------------------------------------------------------------------
_GL8 = np.polynomial.legendre.leggauss(8)


def _cubic_bspline(t):
    a = np.abs(t)
    return np.where(a <= 1.0, (4.0 - 6.0 * a * a + 3.0 * a ** 3) / 6.0,
                    np.where(a <= 2.0, (2.0 - a) ** 3 / 6.0, 0.0))


def kreiss_kernel(t, order: int):
    """The smoothing kernel Phi of the given order (2 or 4)."""
    t = np.asarray(t, dtype=float)
    if order == 2:
        return np.maximum(1.0 - np.abs(t), 0.0)
    if order == 4:
        return 4.0 / 3.0 * _cubic_bspline(t) - (_cubic_bspline(t - 1.0) + _cubic_bspline(t + 1.0)) / 6.0
    raise ValueError("order must be 2 or 4")


def kreiss_smooth(v: Callable, x, h: float, order: int, kinks=()):
    """(M_h v)(x) for a vectorised v that is smooth except at the points
    ``kinks``: Gauss-Legendre (8 points) on every unit interval of the kernel's
    support, split where x - h t crosses a kink, so every piece is smooth."""
    x = np.asarray(x, dtype=float)
    s = 1 if order == 2 else 3
    gx, gw = _GL8
    out = np.zeros_like(x)
    for a in range(-s, s):
        cuts = [np.full_like(x, float(a))]
        for xk in kinks:
            cuts.append(np.clip((x - xk) / h, a, a + 1.0))
        cuts.append(np.full_like(x, a + 1.0))
        cuts = np.sort(np.stack(cuts), axis=0)
        for lo, hi in zip(cuts[:-1], cuts[1:]):
            half, mid = 0.5 * (hi - lo), 0.5 * (hi + lo)
            for xg, wg in zip(gx, gw):
                t = mid + half * xg
                out += wg * half * kreiss_kernel(t, order) * v(x - h * t)
    return out


def bs_call_1d(n_x: int = 16384, n_t: int = 256, k: int = 4, L: int = 32,
               half_width: float | None = 5.2, K: float = 100.0, S0: float = 100.0,
               r: float = 0.05, mu: float = 0.1, sigma: float = 0.2, T: float = 0.33,
               delta: float = 0.0, smooth: bool = True, terminal: str | None = None) -> Workload:
    """Black-Scholes call as a linear BSDE on the log-price grid.

    f = -r y - ((mu - r + delta)/sigma) z (eq (29)-(30)), X = ln S (eq (33)).
    With ``smooth`` the terminal layer is the closed-form price with dt left
    to expiry, so the solved problem has maturity T + dt and a smooth terminal
    condition; the exact solution is the price at that maturity.
    ``terminal`` overrides ``smooth``: "shift" (the same), "raw" (the payoff
    and z = sigma S 1{S > K} at T), "kreiss2" or "kreiss4" (those smoothed by
    the Kreiss-type operator of that order over one cell); for the last three
    the exact solution is the price at maturity T and ``terminal_layer()``
    gives the layer at t_N (the other K - 1 initial layers are then the
    method's own, Section 3.1 step 2).
    ``half_width=None`` gives the interval [ln S0 - 6 sigma sqrt(T) - |mu - sigma^2/2| T,
    ln S0 + 6 sigma sqrt(T)]; a number gives ln S0 +- half_width.  The interval
    is shifted by less than one cell so that ln S0 is a grid node.
    """
    if terminal is None:
        terminal = "shift" if smooth else "raw"
    if terminal not in ("shift", "raw", "kreiss2", "kreiss4"):
        raise ValueError(f"unknown terminal condition {terminal}")
    smooth = terminal == "shift"
    c = math.log(S0)
    if half_width is None:
        lo = c - 6 * sigma * math.sqrt(T) - abs(mu - 0.5 * sigma ** 2) * T
        hi = c + 6 * sigma * math.sqrt(T)
    else:
        lo, hi = c - half_width, c + half_width
    lo, hi = _snap_domain(c, lo, hi, n_x)
    tau_s = T / n_t if smooth else 0.0
    theta = (mu - r + delta) / sigma
    pb = _problem(T=T, n_t=n_t, k_y=k, k_z=k, L=L, n_x=n_x, x_min=lo, x_max=hi,
                  drift=mu - 0.5 * sigma ** 2, vol=sigma, driver="linear",
                  p=[-r, -theta, 0.0, 0.0])

    def exact(t, x):
        tau = T + tau_s - t
        if tau <= 0:
            return np.maximum(np.exp(x) - K, 0.0), sigma * np.exp(x) * (x > math.log(K))
        return bs_call(tau, x, K, r, sigma, delta)

    w = Workload(f"bs1d_nx{n_x}_nt{n_t}_k{k}_L{L}" + ("" if smooth else "_" + terminal), pb, exact,
                 math.log(S0))
    w.extra.update(dict(K=K, S0=S0, r=r, mu=mu, sigma=sigma, delta=delta, tau_s=tau_s,
                        terminal=terminal))
    return w


def terminal_layer(w: Workload):
    """The layer at t_N of a Black-Scholes workload: (y, z) of shapes (n,)
    and (1, n), smoothed as its ``terminal`` setting says."""
    x = w.grid(0)
    e = w.extra
    mode = e.get("terminal", "shift")
    if mode == "shift":
        y, z = w.exact(w.problem["T"], x)
        return y, z[None, :]
    K, sigma = e["K"], e["sigma"]
    pay = lambda u: np.maximum(np.exp(u) - K, 0.0)
    dpay = lambda u: sigma * np.exp(u) * (u > math.log(K))
    if mode == "raw":
        return pay(x), dpay(x)[None, :]
    order = int(mode[-1])
    h = x[1] - x[0]
    return (kreiss_smooth(pay, x, h, order, (math.log(K),)),
            kreiss_smooth(dpay, x, h, order, (math.log(K),))[None, :])


def bidask_call_1d(n_x: int = 262144, n_t: int = 1024, k: int = 4, L: int = 16,
                   half_width: float | None = 52.0, K: float = 100.0, S0: float = 100.0,
                   r: float = 0.01, R: float = 0.06, mu: float = 0.05, sigma: float = 0.2,
                   T: float = 0.5, sign: float = 1.0, smooth: bool = True,
                   picard_tol: float = 1e-14, picard_max: int = 30) -> Workload:
    """Call under different lending (r) and borrowing (R) rates.

    f = -r y - theta z + s (R - r) min(y - z/sigma, 0), theta = (mu - r)/sigma.
    A call's replicating portfolio always borrows (y - z/sigma < 0), so the
    exact solution is the Black-Scholes price at rate r' = r - s (R - r):
    s = +1 (the sign as written in the workload statement) gives 2r - R,
    s = -1 (the usual borrowing-rate driver) gives R.
    ``half_width=None`` gives ln S0 +- 6 sigma sqrt(T).
    """
    c = math.log(S0)
    hw = 6 * sigma * math.sqrt(T) if half_width is None else half_width
    lo, hi = _snap_domain(c, c - hw, c + hw, n_x)
    tau_s = T / n_t if smooth else 0.0
    theta = (mu - r) / sigma
    r_eff = r - sign * (R - r)
    pb = _problem(T=T, n_t=n_t, k_y=k, k_z=k, L=L, n_x=n_x, x_min=lo, x_max=hi,
                  drift=mu - 0.5 * sigma ** 2, vol=sigma, driver="bidask",
                  p=[r, R, theta, sigma, sign], picard_tol=picard_tol, picard_max=picard_max)

    def exact(t, x):
        tau = T + tau_s - t
        if tau <= 0:
            return np.maximum(np.exp(x) - K, 0.0), sigma * np.exp(x) * (x > math.log(K))
        return bs_call(tau, x, K, r_eff, sigma)

    w = Workload(f"bidask1d_nx{n_x}_nt{n_t}_k{k}_L{L}", pb, exact, c)
    w.extra.update(dict(K=K, S0=S0, r=r, R=R, mu=mu, sigma=sigma, sign=sign, tau_s=tau_s,
                        r_eff=r_eff))
    return w


def bidask_put_1d(n_x: int = 4096, n_t: int = 64, k: int = 4, L: int = 16,
                  half_width: float | None = None, K: float = 100.0, S0: float = 100.0,
                  r: float = 0.01, R: float = 0.06, mu: float = 0.05, sigma: float = 0.2,
                  T: float = 0.5, sign: float = 1.0, smooth: bool = True,
                  picard_tol: float = 1e-14, picard_max: int = 30) -> Workload:
    """Put under the bid-ask driver of ``bidask_call_1d`` (same parameters).

    A put's replicating portfolio is short the asset and always lends:
    y - z/sigma = K e^{-r tau} N(-d2) > 0, so min(y - z/sigma, 0) = 0 and the
    driver reduces to -r y - theta z for either sign s.  The exact solution is
    the Black-Scholes put at the lending rate r.  The terminal layer is
    smoothed as for the call (maturity T + dt).
    """
    c = math.log(S0)
    hw = 6 * sigma * math.sqrt(T) if half_width is None else half_width
    lo, hi = _snap_domain(c, c - hw, c + hw, n_x)
    tau_s = T / n_t if smooth else 0.0
    theta = (mu - r) / sigma
    pb = _problem(T=T, n_t=n_t, k_y=k, k_z=k, L=L, n_x=n_x, x_min=lo, x_max=hi,
                  drift=mu - 0.5 * sigma ** 2, vol=sigma, driver="bidask",
                  p=[r, R, theta, sigma, sign], picard_tol=picard_tol, picard_max=picard_max)

    def exact(t, x):
        tau = T + tau_s - t
        if tau <= 0:
            return np.maximum(K - np.exp(x), 0.0), -sigma * np.exp(x) * (x < math.log(K))
        return bs_put(tau, x, K, r, sigma)

    w = Workload(f"bidaskput1d_nx{n_x}_nt{n_t}_k{k}_L{L}", pb, exact, c)
    w.extra.update(dict(K=K, S0=S0, r=r, R=R, mu=mu, sigma=sigma, sign=sign, tau_s=tau_s,
                        r_eff=r))
    return w


def bs_call_price_1d(n_x: int = 800, n_t: int = 64, k: int = 3, L: int = 16,
                     S_max: float = 300.0, S_min: float = 1.0, K: float = 100.0,
                     S0: float = 100.0, r: float = 0.05, mu: float = 0.1, sigma: float = 0.2,
                     T: float = 0.33, smooth: bool = True) -> Workload:
    """Black-Scholes call on the stock-price grid (X = S, not ln S): the forward
    coefficients of eq (1) depend on the state, a(S) = mu S and b(S) = sigma S
    (drift_x = mu, vol_x = sigma), so the nodes lie at different cell
    fractions for every grid point (the variant that Table 7 compares with
    the log-price grid).  f = -r y - theta z with theta = (mu - r)/sigma and
    z = sigma S dV/dS.  Grid S_min..S_max; S0 is moved onto a node by shifting
    the interval.  ``smooth`` as in bs_call_1d."""
    lo, hi = _snap_domain(S0, S_min, S_max, n_x)
    tau_s = T / n_t if smooth else 0.0
    theta = (mu - r) / sigma
    pb = _problem(T=T, n_t=n_t, k_y=k, k_z=k, L=L, n_x=n_x, x_min=lo, x_max=hi, drift=0.0,
                  vol=0.0, drift_x=mu, vol_x=sigma, driver="linear", p=[-r, -theta, 0.0, 0.0])

    def exact(t, S):
        tau = T + tau_s - t
        x = np.log(np.maximum(S, 1e-300))
        if tau <= 0:
            return np.maximum(S - K, 0.0), sigma * S * (S > K)
        return bs_call(tau, x, K, r, sigma)

    w = Workload(f"bsprice1d_nx{n_x}_nt{n_t}_k{k}_L{L}", pb, exact, S0)
    w.extra.update(dict(K=K, S0=S0, r=r, mu=mu, sigma=sigma, tau_s=tau_s))
    return w


def ou_linear_1d(n_x: int = 801, n_t: int = 32, k: int = 3, L: int = 16, kappa: float = 1.5,
                 theta: float = 0.4, sigma: float = 0.3, T: float = 1.0,
                 half_width: float = 3.0) -> Workload:
    """Ornstein-Uhlenbeck forward process dX = kappa (theta - X) dt + sigma dW
    (a(x) = kappa theta - kappa x: drift_x = -kappa), f = 0, g(x) = x:
    y = theta + (x - theta) e^{-kappa (T - t)}, z = sigma e^{-kappa (T - t)}."""
    pb = _problem(T=T, n_t=n_t, k_y=k, k_z=k, L=L, n_x=n_x, x_min=theta - half_width,
                  x_max=theta + half_width, drift=kappa * theta, drift_x=-kappa, vol=sigma,
                  driver="linear", p=[0.0, 0.0, 0.0, 0.0])

    def exact(t, x):
        e = math.exp(-kappa * (T - t))
        return theta + (x - theta) * e, np.full_like(x, sigma * e)

    w = Workload(f"ou1d_nx{n_x}_nt{n_t}_k{k}_L{L}", pb, exact, theta)
    w.extra.update(dict(kappa=kappa, theta=theta, sigma=sigma))
    return w


# ----------------------------------------------------------------------------
# Forward coefficients tabulated on the grid (eq (1) with any a(t, x), b(t, x))
# ----------------------------------------------------------------------------


def coef_table(pb: dict, a_fn: Callable, b_fn: Callable, time_dependent: bool) -> np.ndarray:
    """(tab_steps, 2, n_x) rows of a(t_n, x_i) and b(t_n, x_i): one row (t = 0)
    or one per step n = 0..N-1."""
    n = pb["n_x"]
    x = pb["x_min"] + np.arange(n) * ((pb["x_max"] - pb["x_min"]) / (n - 1))
    steps = pb["n_t"] if time_dependent else 1
    dt = pb["T"] / pb["n_t"]
    tab = np.empty((steps, 2, n))
    for r in range(steps):
        t = r * dt
        tab[r, 0] = a_fn(t, x)
        tab[r, 1] = b_fn(t, x)
    return tab


def tabulated(w: Workload, time_dependent: bool = False) -> Workload:
    """The same problem with its affine (or constant) coefficients given as a
    table (rows repeated when time_dependent): the same arithmetic, tabulated."""
    pb = dict(w.problem)
    a0, a1 = pb.get("drift", 0.0), pb.get("drift_x", 0.0)
    b0, b1 = pb.get("vol", 1.0), pb.get("vol_x", 0.0)
    pb["coef_tab"] = coef_table(pb, lambda t, x: a0 + a1 * x, lambda t, x: b0 + b1 * x,
                                time_dependent)
    pb["drift_x"] = pb["vol_x"] = 0.0
    return Workload(w.name + ("_tabt" if time_dependent else "_tab"), pb, w.exact, w.x0,
                    extra=dict(w.extra))


def quadratic_time_varying_vol(n_x: int = 801, n_t: int = 40, L: int = 16, T: float = 1.0,
                               sigma0: float = 0.3, growth: float = 1.5,
                               half_width: float = 6.0) -> Workload:
    """dX = sigma(t) dW with sigma(t) = sigma0 (1 + growth t), f = 0, g(x) = x^2,
    K = 1, tabulated per step: y(t, x) = x^2 + int_t^T sigma^2 ds.  The 1-step
    scheme with the Euler node of step n at sigma(t_n) adds sigma(t_n)^2 dt per
    step (the spline holds x^2 away from the ends), so the computed y0 is
    x^2 + dt sum_{n<N} sigma(t_n)^2, the left Riemann sum (extra["y0_scheme"])."""
    pb = _problem(T=T, n_t=n_t, k_y=1, k_z=1, L=L, n_x=n_x, x_min=-half_width,
                  x_max=half_width, driver="linear", p=[0.0, 0.0, 0.0, 0.0])
    sig = lambda t: sigma0 * (1.0 + growth * t)
    pb["coef_tab"] = coef_table(pb, lambda t, x: np.zeros_like(x),
                                lambda t, x: np.full_like(x, sig(t)), True)
    dt = T / n_t
    left = dt * sum(sig(n * dt) ** 2 for n in range(n_t))

    def exact(t, x):
        # int_t^T sigma0^2 (1 + g s)^2 ds
        F = lambda s: sigma0 ** 2 * ((1.0 + growth * s) ** 3) / (3.0 * growth)
        return x * x + (F(T) - F(t)), 2.0 * sig(t) * x

    w = Workload(f"quadvol_nx{n_x}_nt{n_t}_L{L}", pb, exact, 0.0)
    w.extra.update(dict(y0_scheme_offset=left))
    return w


def local_vol_call_1d(n_x: int = 2001, n_t: int = 48, k: int = 3, L: int = 16, K: float = 100.0,
                      S0: float = 100.0, r: float = 0.03, mu: float = 0.06, T: float = 0.5,
                      half_width: float = 1.2, time_dependent: bool = True,
                      driver: str = "linear") -> Workload:
    """A call under a local volatility with skew and a term structure,
    sigma(t, x) = (0.2 - 0.08 tanh(x - ln K)) (1 + 0.3 t / T), on the
    log-price grid: a = mu - sigma^2 / 2, b = sigma, tabulated per step.
    Driver linear (f = -r y - ((mu - r)/sigma(x)) z is not linear in the table;
    the linear driver takes theta at the money) or bid-ask.  No closed form:
    the terminal layers are the Black-Scholes prices at the money volatility
    (a smooth input for parity)."""
    c = math.log(S0)
    lo, hi = _snap_domain(c, c - half_width, c + half_width, n_x)
    sig = lambda t, x: (0.2 - 0.08 * np.tanh(x - math.log(K))) * (1.0 + 0.3 * t / T)
    s_atm = 0.2
    theta = (mu - r) / s_atm
    p = [-r, -theta, 0.0, 0.0] if driver == "linear" else [r, r + 0.05, theta, s_atm, 1.0]
    pb = _problem(T=T, n_t=n_t, k_y=k, k_z=k, L=L, n_x=n_x, x_min=lo, x_max=hi,
                  driver=driver, p=p)
    pb["coef_tab"] = coef_table(pb, lambda t, x: mu - 0.5 * sig(t, x) ** 2, sig, time_dependent)

    def exact(t, x):
        return bs_call(T + T / n_t - t, x, K, r, s_atm)

    w = Workload(f"lv1d_nx{n_x}_nt{n_t}_k{k}_L{L}_{driver}", pb, exact, c)
    return w


def option_batch(count: int = 4096, seed: int = 1909, log2_nx: tuple = (10.0, 16.0),
                 n_ts: tuple = (64, 128, 256, 512), k: int = 4, L: int = 16,
                 prec: str = "fp32_comp", shared_grid: int = 0,
                 max_half_width: float = 60.0) -> list:
    """Independent European calls of uneven sizes (the batched workload).

    Drawn from numpy's PCG64 generator seeded with ``seed``: strike
    K ~ U[80, 120], sigma ~ U[0.1, 0.5], r ~ U[0, 0.06], T ~ U[0.1, 2],
    n_x = round(2^U[log2_nx]), N uniform over ``n_ts``; S0 = 100,
    mu = r + 0.05; even instances are Black-Scholes (linear driver), odd ones
    the bid-ask call with R = r + 0.05 and the sign as written (s = +1).
    The log-price interval around ln S0 has half-width
    max(6 sigma sqrt(T) + |mu - sigma^2/2| T, sigma sqrt(2 dt) (n_x - 1) / 32),
    so the stability ratio is at most 16 by construction; the half-width is
    capped at ``max_half_width`` (e^(ln 100 + 60) ~ 1e28 keeps prices within
    single precision) and, where the cap binds, n_x is lowered to the
    largest grid with ratio <= 16.  The first
    ``shared_grid`` instances share sigma = 0.2, mu = 0.1, T = 1, N = 256,
    n_x = 16384 and the interval (Black-Scholes; K and r still vary).
    """
    rng = np.random.default_rng(seed)
    out = []
    for b in range(count):
        Kb = rng.uniform(80.0, 120.0)
        sg = rng.uniform(0.1, 0.5)
        r = rng.uniform(0.0, 0.06)
        T = rng.uniform(0.1, 2.0)
        nx = int(round(2.0 ** rng.uniform(*log2_nx)))
        nt = int(rng.choice(np.asarray(n_ts)))
        mu = r + 0.05
        bid_ask = b % 2 == 1
        if b < shared_grid:
            sg, mu, T, nt, nx, bid_ask = 0.2, 0.1, 1.0, 256, 16384, False
        dt = T / nt
        hw = max(6 * sg * math.sqrt(T) + abs(mu - 0.5 * sg ** 2) * T,
                 sg * math.sqrt(2 * dt) * (nx - 1) / 32)
        if hw > max_half_width:
            hw = max_half_width
            nx = int(32 * hw / (sg * math.sqrt(2 * dt))) + 1
        if bid_ask:
            w = bidask_call_1d(n_x=nx, n_t=nt, k=k, L=L, half_width=hw, K=Kb, r=r, R=r + 0.05,
                               mu=mu, sigma=sg, T=T, sign=1.0)
        else:
            w = bs_call_1d(n_x=nx, n_t=nt, k=k, L=L, half_width=hw, K=Kb, r=r, mu=mu, sigma=sg,
                           T=T)
        w.problem["prec"] = prec
        w.name = f"batch{b}_" + w.name
        out.append(w)
    return out


# ----------------------------------------------------------------------------
# Two space dimensions (tensor grid; X = x + drift t + vol W with W in R^2)
# ----------------------------------------------------------------------------


def sine_2d(n_x: int = 129, n_t: int = 8, k: int = 3, L: int = 8, half: float = 8.0) -> Workload:
    """Example 4: X = W in R^2, f = y - (z1 + z2)/2, g = sin(x1 + x2 + T), T = 1, on
    [-half, half]^2; exact y = sin(x1 + x2 + t), z = (cos, cos)(x1 + x2 + t)."""
    pb = _problem(d=2, T=1.0, n_t=n_t, k_y=k, k_z=k, L=L, n_x=[n_x, n_x], x_min=[-half, -half],
                  x_max=[half, half], drift=[0.0, 0.0], vol=[[1.0, 0.0], [0.0, 1.0]],
                  driver="linear", p=[1.0, -0.5, -0.5, 0.0])

    def exact(t, x):
        s = x[0] + x[1] + t
        return np.sin(s), (np.cos(s), np.cos(s))

    return Workload(f"sine2d_nx{n_x}_nt{n_t}_k{k}_L{L}", pb, exact, (0.0, 0.0))


def _vol_2d(sigma, rho):
    """diag(sigma) L_rho with L_rho the Cholesky factor of [[1, rho], [rho, 1]]."""
    return [[sigma[0], 0.0], [rho * sigma[1], sigma[1] * math.sqrt(1.0 - rho * rho)]]


def exchange_2d(n_x: int = 65, n_t: int = 16, k: int = 3, L: int = 8,
                S0: tuple = (100.0, 100.0), r: float = 0.05, mu: tuple = (0.1, 0.1),
                sigma: tuple = (0.25, 0.3), rho: float = 0.0, T: float = 1.0,
                half_width: float | None = None, smooth: bool = True) -> Workload:
    """Example 5: the zero-strike spread (exchange) call max(S1 - S2, 0) on the
    log-price grid.  X = ln S, X_t = x + (mu - sigma^2/2) t + vol B with
    vol = diag(sigma) L_rho, z is taken w.r.t. the independent B and
    f = -r y - theta . z with vol theta = mu - r.  Exact: Margrabe's price,
    z = (grad_x V) vol.  ``smooth`` starts from the price with dt to expiry
    (maturity T + dt); ``half_width=None`` gives ln S0 +- 6 sigma sqrt(T) per axis."""
    vol = _vol_2d(sigma, rho)
    theta = np.linalg.solve(np.asarray(vol), np.asarray(mu) - r)
    lo, hi = [], []
    for a in range(2):
        c = math.log(S0[a])
        hw = 6 * sigma[a] * math.sqrt(T) if half_width is None else half_width
        l_, h_ = _snap_domain(c, c - hw, c + hw, n_x)
        lo.append(l_)
        hi.append(h_)
    tau_s = T / n_t if smooth else 0.0
    pb = _problem(d=2, T=T, n_t=n_t, k_y=k, k_z=k, L=L, n_x=[n_x, n_x], x_min=lo, x_max=hi,
                  drift=[mu[0] - 0.5 * sigma[0] ** 2, mu[1] - 0.5 * sigma[1] ** 2], vol=vol,
                  driver="linear", p=[-r, -theta[0], -theta[1], 0.0])

    def exact(t, x):
        tau = T + tau_s - t
        if tau <= 0:
            S1, S2 = np.exp(x[0]), np.exp(x[1])
            up = S1 > S2
            g1, g2 = S1 * up, -S2 * up
        else:
            _, g1, g2 = margrabe(tau, x[0], x[1], sigma[0], sigma[1], rho)
        V = g1 + g2  # S1 N(d1) - S2 N(d2), and the payoff at expiry
        return V, (vol[0][0] * g1 + vol[1][0] * g2, vol[1][1] * g2)

    w = Workload(f"exchange2d_nx{n_x}_nt{n_t}_k{k}_L{L}", pb, exact,
                 (math.log(S0[0]), math.log(S0[1])))
    w.extra.update(dict(sigma=sigma, rho=rho, r=r, mu=mu, tau_s=tau_s))
    return w


def basket_2d(n_x: int = 1024, n_t: int = 128, k: int = 3, L: int = 16, S0: float = 100.0,
              K: float = 100.0, r: float = 0.05, mu: float = 0.1, sigma: float = 0.2,
              rho: float = 0.5, T: float = 1.0) -> Workload:
    """Basket call max((S1 + S2)/2 - K, 0) on two correlated log-prices with
    equal parameters, f = -r y - theta . z as in exchange_2d, grid
    ln S0 +- 6 sigma sqrt(T) per axis.  There is no closed form: the K initial
    layers are the payoff itself (z its vol-weighted gradient where it is
    differentiable), a deterministic input for parity checks."""
    sg = (sigma, sigma)
    vol = _vol_2d(sg, rho)
    theta = np.linalg.solve(np.asarray(vol), np.asarray([mu, mu]) - r)
    c = math.log(S0)
    lo, hi = _snap_domain(c, c - 6 * sigma * math.sqrt(T), c + 6 * sigma * math.sqrt(T), n_x)
    pb = _problem(d=2, T=T, n_t=n_t, k_y=k, k_z=k, L=L, n_x=[n_x, n_x], x_min=[lo, lo],
                  x_max=[hi, hi], drift=[mu - 0.5 * sigma ** 2] * 2, vol=vol, driver="linear",
                  p=[-r, -theta[0], -theta[1], 0.0])

    def payoff(t, x):
        S1, S2 = np.exp(x[0]), np.exp(x[1])
        itm = 0.5 * (S1 + S2) > K
        g1, g2 = 0.5 * S1 * itm, 0.5 * S2 * itm
        return np.maximum(0.5 * (S1 + S2) - K, 0.0), (vol[0][0] * g1 + vol[1][0] * g2,
                                                     vol[1][1] * g2)

    return Workload(f"basket2d_nx{n_x}_nt{n_t}_k{k}_L{L}", pb, payoff, (c, c))


def quadratic_heat(n_x: int = 513, n_t: int = 32, k: int = 3, L: int = 16,
                   half_width: float = 8.0, T: float = 1.0) -> Workload:
    """f = 0, g = x^2 with X = W: y = x^2 + (T - t), z = 2x (special case)."""
    pb = _problem(T=T, n_t=n_t, k_y=k, k_z=k, L=L, n_x=n_x, x_min=-half_width,
                  x_max=half_width, driver="linear", p=[0.0, 0.0, 0.0, 0.0])

    def exact(t, x):
        return x * x + (T - t), 2.0 * x

    return Workload(f"quad_nx{n_x}_nt{n_t}_k{k}", pb, exact, 0.0)


def discount_const(n_x: int = 65, n_t: int = 32, k: int = 3, L: int = 8, r: float = 0.3,
                   T: float = 1.0) -> Workload:
    """f = -r y, g = 1: y = e^{-r(T - t)}, z = 0 (x-independent special case)."""
    pb = _problem(T=T, n_t=n_t, k_y=k, k_z=k, L=L, n_x=n_x, x_min=-4.0, x_max=4.0,
                  driver="linear", p=[-r, 0.0, 0.0, 0.0])

    def exact(t, x):
        return np.full_like(x, math.exp(-r * (T - t))), np.zeros_like(x)

    return Workload(f"disc_nx{n_x}_nt{n_t}_k{k}", pb, exact, 0.0)


def stability_ratio(pb: dict, axis: int = 0) -> float:
    """R = (spread of one Gauss-Hermite step, vol*sqrt(2 dt)) / dx in cells;
    with state-dependent vol (vol + vol_x x) its largest value on the grid."""
    n = _as_list(pb["n_x"])[axis]
    dx = (_as_list(pb["x_max"])[axis] - _as_list(pb["x_min"])[axis]) / (n - 1)
    vol = np.atleast_2d(np.asarray(pb.get("vol", 1.0), dtype=float))
    v = float(np.sqrt(np.sum(vol[axis] ** 2))) if pb["d"] == 2 else float(vol[0, 0])
    if pb["d"] == 1 and pb.get("vol_x", 0.0):
        v = max(v + pb["vol_x"] * pb["x_min"], v + pb["vol_x"] * pb["x_max"])
    return v * math.sqrt(2.0 * pb["T"] / pb["n_t"]) / dx
