"""GPU parity of the steps around the sweep: the initial layers of Section 3.1
step 2 (1-step scheme with sub-steps).

Same measure and bar as test_gpu_parity: max_i |gpu_i - oracle_i| /
max(|oracle_i|, 1) over every grid point, <= 1e-10 in FP64.
"""
import numpy as np
import pytest

import workloads as W
from test_gpu_parity import TOL64, rel_err, twin_half_width

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1909_13560_amd as B

    B.load()
    return B


@pytest.fixture(scope="module")
def orc():
    import oracle

    oracle.build(force=False)
    return oracle


def _initial_layers_case(lib, orc, wl, sub, terminal=None):
    import torch

    pb = wl.problem
    iy_ex, iz_ex = wl.init_layers()
    if terminal is not None:  # another terminal layer (y of (n,), z of (d, n))
        iy_ex[-1], iz_ex[-1] = terminal
    K, npts = iy_ex.shape
    d = pb["d"]
    print(f"[case] initial layers {wl.name} sub={sub}", flush=True)
    # the oracle's layers from the terminal one
    iy_o, iz_o = orc.initial_layers(pb, iy_ex[-1], iz_ex[-1], sub)
    # the library's, on the device, from the same terminal layer
    plan = lib.bsde_plan(pb)
    ws = lib.workspace(plan)
    t_iy = torch.full((K, npts), float("nan"), dtype=torch.float64, device="cuda")
    t_iz = torch.full((K, d * npts), float("nan"), dtype=torch.float64, device="cuda")
    t_iy[K - 1] = torch.as_tensor(iy_ex[-1], device="cuda")
    t_iz[K - 1] = torch.as_tensor(iz_ex[-1].reshape(-1), device="cuda")
    lib.bsde_initial_layers(pb, sub, ws, t_iy, t_iz)
    iy_g = t_iy.cpu().numpy()
    iz_g = t_iz.cpu().numpy().reshape(K, d, npts)
    e = max(max(rel_err(iy_g[r], iy_o[r]), max(rel_err(iz_g[r, c], iz_o[r, c]) for c in range(d)))
            for r in range(K))
    print(f"  layers: rel err {e:.3e}", flush=True)
    assert e <= TOL64
    # the whole solve from those layers
    y0 = torch.empty(npts, dtype=torch.float64, device="cuda")
    z0 = torch.empty(d * npts, dtype=torch.float64, device="cuda")
    rc, _ = lib.bsde_solve(plan, ws, t_iy, t_iz, y0, z0, stats=True)
    import torch as _t

    _t.cuda.synchronize()
    assert rc == lib.BSDE_OK
    yo, zo, _ = orc.solve(pb, iy_o, iz_o, threads=True)
    zg = z0.cpu().numpy().reshape(d, npts)
    es = max(rel_err(y0.cpu().numpy(), yo), max(rel_err(zg[c], zo[c]) for c in range(d)))
    print(f"  solve: rel err {es:.3e}", flush=True)
    assert es <= TOL64
    return iy_g, iz_g


@pytest.mark.parametrize("sub", [1, 7])
def test_initial_layers_sine(lib, orc, sub):
    _initial_layers_case(lib, orc, W.sine_1d(n_x=1025, n_t=64, k=4), sub)


def test_initial_layers_bid_ask_and_time_dependent_driver(lib, orc):
    nx, nt = 3001, 24
    _initial_layers_case(
        lib, orc, W.bidask_call_1d(n_x=nx, n_t=nt, k=5, half_width=twin_half_width(0.2, 0.5, nt, nx)),
        4)
    # Example 2's driver depends on t: the sub-steps must see absolute times
    _initial_layers_case(lib, orc, W.paper_example2(3, 16, 512), 6)


def test_initial_layers_two_dimensional(lib, orc):
    _initial_layers_case(lib, orc, W.exchange_2d(n_x=49, n_t=8, k=3, L=6, rho=0.5), 3)


def test_initial_layers_from_smoothed_payoffs(lib, orc):
    # Black-Scholes call from its payoff at T (no time shift): raw, and
    # smoothed by the Kreiss-type operator of order 4, with Gauss-Hermite and
    # with exact expectations (the Toeplitz kernel, in the initial layers'
    # 1-step segments too)
    nx, nt = 2049, 32
    for term, q in (("raw", "gh"), ("kreiss4", "gh"), ("kreiss4", "exact")):
        wl = W.bs_call_1d(n_x=nx, n_t=nt, k=4, L=32,
                          half_width=twin_half_width(0.2, 0.33, nt, nx), terminal=term)
        wl.problem["quad"] = q
        _initial_layers_case(lib, orc, wl, 8, terminal=W.terminal_layer(wl))


def test_smoothing_study_full_size(lib):
    # 16384 points, N = 256, k = 4, L = 32 on the stable interval; the method's
    # own initial layers (8 sub-steps) from the terminal layer; errors at the
    # money against the closed form
    import torch

    nx, nt = 16384, 256
    err = {}
    for term, q in (("raw", "gh"), ("kreiss4", "gh"), ("kreiss4", "exact"), ("shift", "gh")):
        wl = W.bs_call_1d(n_x=nx, n_t=nt, k=4, L=32,
                          half_width=twin_half_width(0.2, 0.33, nt, nx), terminal=term)
        pb = dict(wl.problem, quad=q)
        print(f"[case] smoothing study {wl.name} {q}", flush=True)
        ty, tz = W.terminal_layer(wl)
        plan = lib.bsde_plan(pb)
        ws = lib.workspace(plan)
        t_iy = torch.zeros((4, nx), dtype=torch.float64, device="cuda")
        t_iz = torch.zeros((4, nx), dtype=torch.float64, device="cuda")
        t_iy[3] = torch.as_tensor(ty, device="cuda")
        t_iz[3] = torch.as_tensor(tz.reshape(-1), device="cuda")
        lib.bsde_initial_layers(pb, 8, ws, t_iy, t_iz)
        y0 = torch.empty(nx, dtype=torch.float64, device="cuda")
        z0 = torch.empty(nx, dtype=torch.float64, device="cuda")
        rc, _ = lib.bsde_solve(plan, ws, t_iy, t_iz, y0, z0, stats=True)
        torch.cuda.synchronize()
        assert rc == lib.BSDE_OK
        ye, ze = wl.exact_at_t0()
        i = wl.node_index()
        err[term, q] = (abs(float(y0[i]) - ye[i]), abs(float(z0[i]) - ze[i]))
        print("  y0 err %.3e z0 err %.3e" % err[term, q], flush=True)
    assert err["raw", "gh"][1] > 1e-3
    assert err["kreiss4", "gh"][1] < 1e-5 and err["kreiss4", "gh"][0] > 1e-4
    assert err["kreiss4", "exact"][0] < 1e-6 and err["kreiss4", "exact"][1] < 1e-5
    assert err["shift", "gh"][0] < 1e-6 and err["shift", "gh"][1] < 1e-5


def test_initial_layers_reject_small_workspace(lib):
    import torch

    wl = W.sine_1d(n_x=300, n_t=16, k=3)
    ws = torch.empty(256, dtype=torch.uint8, device="cuda")
    iy = torch.zeros((3, 300), dtype=torch.float64, device="cuda")
    iz = torch.zeros((3, 300), dtype=torch.float64, device="cuda")
    with pytest.raises(lib.BsdeError) as ei:
        lib.bsde_initial_layers(wl.problem, 2, ws, iy, iz)
    assert ei.value.code == lib.BSDE_EINVAL


# ----------------------------------------------------------------------------
# The z form E[y^{n+1} dW]/dt
# ----------------------------------------------------------------------------


def _run(lib, orc, wl, prec="fp64", tol=TOL64, threads=False):
    pb = dict(wl.problem, prec=prec)
    print(f"[case] {wl.name} z_form={pb.get('z_form')} {prec}", flush=True)
    iy, iz = wl.init_layers()
    y, z, rc, st = lib.solve(pb, iy, iz)
    yo, zo, _ = orc.solve(pb, iy, iz, n_stop=pb.get("n_stop", 0), threads=threads)
    e = max(rel_err(y, yo), max(rel_err(z[c], zo[c]) for c in range(pb["d"])))
    print(f"  rel err {e:.3e}", flush=True)
    assert rc == lib.BSDE_OK and e <= tol
    return y, z


def test_z_form_ydw_one_step(lib, orc):
    nx, nt = 4001, 64
    wl = W.bidask_call_1d(n_x=nx, n_t=nt, k=1, half_width=twin_half_width(0.2, 0.5, nt, nx))
    wl.problem["z_form"] = "yW"
    _run(lib, orc, wl)
    # the FP32 form is refused: dW/dt weights would amplify its rounding
    with pytest.raises(lib.BsdeError) as ei:
        lib.bsde_plan(dict(wl.problem, prec="fp32_comp"))
    assert ei.value.code == lib.BSDE_EUNSUPPORTED
    wl = W.sine_1d(n_x=1025, n_t=64, k=1)
    wl.problem["z_form"] = "yW"
    y, z = _run(lib, orc, wl)
    # second order: at N = 64 the z error at x = 0 is about 1.2e-4 (5e-4 at
    # N = 32), where the printed form's first order leaves 5e-3
    ye, ze = wl.exact_at_t0()
    assert abs(z[0, wl.node_index()] - ze[wl.node_index()]) < 2e-4


def test_z_form_ydw_multistep_and_two_dimensional(lib, orc):
    # parity of the multistep form over a short sweep (it is unstable over
    # long ones) with unequal orders, and the two-dimensional kernels
    wl = W.sine_1d(n_x=900, n_t=8, k=3)
    wl.problem.update(z_form="yW", k_z=2)
    _run(lib, orc, wl)
    wl = W.exchange_2d(n_x=57, n_t=12, k=1, L=8, rho=0.5)
    wl.problem["z_form"] = "yW"
    _run(lib, orc, wl)
    wl = W.sine_2d(n_x=65, n_t=6, k=2, L=8)
    wl.problem["z_form"] = "yW"
    _run(lib, orc, wl)


# ----------------------------------------------------------------------------
# State-dependent forward coefficients: nodes located per point (gather path)
# ----------------------------------------------------------------------------


@pytest.mark.parametrize("prec,tol", [("fp64", TOL64), ("fp32_comp", 1e-6)])
def test_gather_path_price_grid_and_ou(lib, orc, prec, tol):
    # Black-Scholes on the stock-price grid (b(S) = sigma S), ragged grid
    y, z = _run(lib, orc, W.bs_call_price_1d(n_x=1001, n_t=48, k=3), prec, tol)
    # Ornstein-Uhlenbeck drift with both z forms (the E[y dW]/dt form in
    # FP64 only) and unequal orders
    if prec == "fp64":
        wl = W.ou_linear_1d(n_x=1201, n_t=24, k=1)
        wl.problem["z_form"] = "yW"
        _run(lib, orc, wl, prec, tol)
    wl = W.ou_linear_1d(n_x=777, n_t=20, k=4)
    wl.problem["k_z"] = 2
    _run(lib, orc, wl, prec, tol)


def test_gather_path_nonlinear_driver_and_batch(lib, orc):
    import torch

    # bid-ask driver with an affine volatility (nodes leave the domain at
    # both ends), in a batch with a constant-coefficient instance (which
    # keeps its own LDS-staged kernel)
    g = W.bidask_call_1d(n_x=3001, n_t=16, half_width=None)
    g.problem.update(drift_x=0.01, vol_x=0.02, vol=0.2 - 0.02 * 4.6)
    u = W.bidask_call_1d(n_x=5003, n_t=24, half_width=twin_half_width(0.2, 0.5, 24, 5003))
    plan = lib.bsde_plan([g.problem, u.problem])
    ws = lib.workspace(plan)
    ios = []
    for w in (g, u):
        iy, iz = w.init_layers()
        n = iy.shape[1]
        ios.append((torch.as_tensor(iy, device="cuda").contiguous(),
                    torch.as_tensor(iz.reshape(iy.shape), device="cuda").contiguous(),
                    torch.empty(n, dtype=torch.float64, device="cuda"),
                    torch.empty(n, dtype=torch.float64, device="cuda")))
    print("[case] gather + fused batch", flush=True)
    rc, st = lib.bsde_solve_batched(plan, ws, ios, stats=True)
    torch.cuda.synchronize()
    assert rc == lib.BSDE_OK
    kt = lib.bsde_profile_kernels(plan, ws, ios)
    for w, io in zip((g, u), ios):
        iy, iz = w.init_layers()
        yo, zo, _ = orc.solve(w.problem, iy, iz)
        e = max(rel_err(io[2].cpu().numpy(), yo), rel_err(io[3].cpu().numpy(), zo[0]))
        print(f"  {w.name}: {e:.3e}", flush=True)
        assert e <= TOL64
    assert kt["sweep_launches"] == 13 + 21 and kt["spline_launches"] == 13


# ----------------------------------------------------------------------------
# Exact Gaussian expectations: banded Toeplitz products on FP64 matrix cores
# ----------------------------------------------------------------------------


def test_exact_quadrature_toeplitz(lib, orc):
    import torch

    # sine problem (several 1024-point tiles, ragged end), a Black-Scholes call
    # at stability ratio 40 (bands of several LDS chunks), and the z form
    # E[y dW]/dt with K = 1
    wl = W.sine_1d(n_x=2101, n_t=10, k=3)
    wl.problem["quad"] = "exact"
    _run(lib, orc, wl)
    nx, nt = 3001, 12
    wl = W.bs_call_1d(n_x=nx, n_t=nt, k=4, L=16,
                      half_width=twin_half_width(0.2, 0.33, nt, nx, 40.0))
    wl.problem["quad"] = "exact"
    _run(lib, orc, wl)
    wl = W.sine_1d(n_x=999, n_t=16, k=1)
    wl.problem.update(quad="exact", z_form="yW")
    _run(lib, orc, wl)
    # the plan chose the Toeplitz kernel
    plan = lib.bsde_plan(wl.problem)
    ws = lib.workspace(plan)
    iy, iz = wl.init_layers()
    n = iy.shape[1]
    io = (torch.as_tensor(iy, device="cuda").contiguous(),
          torch.as_tensor(iz.reshape(iy.shape), device="cuda").contiguous(),
          torch.empty(n, dtype=torch.float64, device="cuda"),
          torch.empty(n, dtype=torch.float64, device="cuda"))
    kt = lib.bsde_profile_kernels(plan, ws, [io])
    assert kt["path"] == 4 and kt["node_groups"] > 1


def _toeplitz_splits(lib, pbs):
    import torch

    plan = lib.bsde_plan(pbs)
    ws = lib.workspace(plan)
    ios = []
    for pb in pbs:
        n = pb["n_x"]
        K = max(pb["k_y"], pb["k_z"])
        ios.append((torch.zeros(K * n, dtype=torch.float64, device="cuda"),
                    torch.zeros(K * n, dtype=torch.float64, device="cuda"),
                    torch.empty(n, dtype=torch.float64, device="cuda"),
                    torch.empty(n, dtype=torch.float64, device="cuda")))
    kt = lib.bsde_profile_kernels(plan, ws, ios)
    assert kt["path"] == 4
    return kt["node_groups"]


def test_exact_quadrature_toeplitz_splits_and_batch(lib, orc):
    from test_gpu_parity import batched_solve

    # one band chunk (K = 1 at stability ratio 16: about 220 taps): no
    # split, the sweep kernel finishes the points itself
    nx, nt = 3001, 40
    wl = W.bs_call_1d(n_x=nx, n_t=nt, k=1, L=16, half_width=twin_half_width(0.2, 0.33, nt, nx))
    wl.problem["quad"] = "exact"
    assert _toeplitz_splits(lib, [wl.problem]) == 1
    _run(lib, orc, wl)
    # a batch of exact instances of different sizes and lengths in one group
    # (tile map, splits over several blocks per tile, prefix-active launches)
    wls = [W.sine_1d(n_x=700, n_t=20, k=2), W.sine_1d(n_x=3001, n_t=9, k=3),
           W.bs_call_1d(n_x=1999, n_t=12, k=4, L=16,
                        half_width=twin_half_width(0.2, 0.33, 12, 1999, 30.0))]
    for w in wls:
        w.problem["quad"] = "exact"
    assert _toeplitz_splits(lib, [w.problem for w in wls]) > 1
    rc, st, outs, _ = batched_solve(lib, wls)
    assert rc == lib.BSDE_OK
    for w, (y, z) in zip(wls, outs):
        iy, iz = w.init_layers()
        yo, zo, _ = orc.solve(dict(w.problem, prec="fp64"), iy, iz)
        e = max(rel_err(y, yo), rel_err(z, zo[0]))
        print(f"  {w.name}: rel err {e:.3e}", flush=True)
        assert e <= TOL64


def test_exact_quadrature_black_scholes_full_size_first_steps(lib, orc):
    # 16384 points, N = 256, k = 4 on the stable twin interval, its first
    # eight backward steps against the oracle over the whole grid
    nx, nt = 16384, 256
    wl = W.bs_call_1d(n_x=nx, n_t=nt, k=4, L=32, half_width=twin_half_width(0.2, 0.33, nt, nx))
    wl.problem.update(quad="exact", n_stop=nt - 4 + 1 - 8)
    _run(lib, orc, wl, threads=True)


def test_exact_quadrature_refuses_unsupported(lib):
    wl = W.bidask_call_1d(n_x=500, n_t=8, half_width=None)
    with pytest.raises(lib.BsdeError) as ei:
        lib.bsde_plan(dict(wl.problem, quad="exact"))
    assert ei.value.code == lib.BSDE_EUNSUPPORTED


# ----------------------------------------------------------------------------
# The paper's 2-D interpolation: bicubic with finite-difference derivatives
# ----------------------------------------------------------------------------


def test_bicubic_fd_two_dimensional(lib, orc):
    # Example 4 at Table 9's K = 1 row (the bicubic reproduces it), the
    # exchange option with correlation on a ragged grid with unequal orders,
    # and lines of 5 points (the one-sided stencils only)
    for wl in (W.sine_2d(n_x=65, n_t=16, k=1, L=8), W.exchange_2d(n_x=77, n_t=9, k=3, L=7, rho=0.4)):
        wl.problem["interp"] = "bicubic_fd"
        _run(lib, orc, wl)
    wl = W.exchange_2d(n_x=5, n_t=6, k=2, L=6, rho=0.3)
    pb = wl.problem
    pb["n_x"] = [5, 300]
    pb["x_max"] = [pb["x_max"][0], pb["x_min"][1] + 299 * (pb["x_max"][1] - pb["x_min"][1]) / 4 / 40]
    pb.update(interp="bicubic_fd", k_y=2, k_z=1)
    wl.x0 = (pb["x_min"][0], pb["x_min"][1])
    _run(lib, orc, wl)
    y, z = _run(lib, orc, W.sine_2d(n_x=65, n_t=16, k=1, L=8))  # the spline beside it


# ----------------------------------------------------------------------------
# The FP32 form in 2-D: float ring planes with error feedback, FP64 arithmetic
# ----------------------------------------------------------------------------


def _fp32_2d_cases():
    cases = [W.sine_2d(n_x=129, n_t=8, k=3, L=8), W.exchange_2d(n_x=97, n_t=10, k=3, L=8, rho=0.5)]
    wl = W.exchange_2d(n_x=77, n_t=9, k=2, L=7, rho=0.3)  # ragged, unequal orders
    pb = wl.problem
    pb["n_x"] = [77, 130]
    pb["x_max"] = [pb["x_max"][0], pb["x_min"][1] + 129 * (pb["x_max"][1] - pb["x_min"][1]) / 76]
    pb["k_y"], pb["k_z"] = 3, 2
    cases.append(wl)
    wl = W.exchange_2d(n_x=21, n_t=12, k=2, L=6, rho=0.4)  # short columns, two tiles per row
    pb = wl.problem
    dx1 = (pb["x_max"][0] - pb["x_min"][0]) / 20 / 8
    pb["n_x"] = [21, 700]
    pb["x_max"] = [pb["x_max"][0], pb["x_min"][1] + 699 * dx1]
    cases.append(wl)
    wl = W.exchange_2d(n_x=77, n_t=9, k=3, L=7, rho=0.4)  # the paper's bicubic
    wl.problem["interp"] = "bicubic_fd"
    cases.append(wl)
    return cases


def test_fp32_two_dimensional(lib, orc):
    from test_gpu_parity import TOL32

    for wl in _fp32_2d_cases():
        y, z = _run(lib, orc, wl, prec="fp32_comp", tol=TOL32)
        assert np.all(np.isfinite(y)) and np.all(np.isfinite(z))
    # a checkpoint of the basket (raw payoff layers)
    wl = W.basket_2d(n_x=65, n_t=12, k=3, L=16)
    wl.problem["n_stop"] = 4
    _run(lib, orc, wl, prec="fp32_comp", tol=TOL32)
    # the E[y dW]/dt z form stays refused in the FP32 form
    wl = W.exchange_2d(n_x=33, n_t=6, k=1, L=6, rho=0.2)
    with pytest.raises(lib.BsdeError) as ei:
        lib.bsde_plan(dict(wl.problem, prec="fp32_comp", z_form="yW"))
    assert ei.value.code == lib.BSDE_EUNSUPPORTED


def test_fp32_two_dimensional_full_size(lib, orc):
    # the benchmarked 2-D shape (1024 x 1024, 128 steps, k = 3, 16 x 16 nodes):
    # the first layer against the oracle at sampled points, and the whole
    # solve against the FP64 form over the whole grid
    from test_gpu_parity import TOL32

    wl = W.basket_2d()
    pb = dict(wl.problem)
    K = max(pb["k_y"], pb["k_z"])
    n0, n1 = pb["n_x"]
    iy, iz = wl.init_layers()
    print(f"[case] {wl.name} fp32 first step sampled, whole solve", flush=True)
    y, z, rc, _ = lib.solve(dict(pb, prec="fp32_comp", n_stop=pb["n_t"] - K), iy, iz)
    assert rc == lib.BSDE_OK
    rng = np.random.default_rng(2909)
    rows = np.concatenate([[0, 1, 2, n0 // 2, n0 - 2, n0 - 1], rng.integers(0, n0, 300)])
    cols = np.resize(np.concatenate([[0, 1, 511, 512, n1 - 2, n1 - 1], rng.integers(0, n1, 300)]),
                     rows.size)
    idx = np.unique(rows.astype(np.int64) * n1 + cols)
    ys, zs = orc.first_step_points_2d(dict(pb, n_stop=pb["n_t"] - K), iy, iz, idx)
    e1 = max(rel_err(y[idx], ys), rel_err(z[0, idx], zs[0]), rel_err(z[1, idx], zs[1]))
    y32, z32, rc32, _ = lib.solve(dict(pb, prec="fp32_comp"), iy, iz)
    y64, z64, rc64, _ = lib.solve(dict(pb, prec="fp64"), iy, iz)
    assert rc32 == lib.BSDE_OK and rc64 == lib.BSDE_OK
    e2 = max(rel_err(y32, y64), rel_err(z32[0], z64[0]), rel_err(z32[1], z64[1]))
    print(f"  first step vs oracle {e1:.3e}, whole solve vs FP64 {e2:.3e}", flush=True)
    assert e1 <= TOL32 and e2 <= TOL32


# ----------------------------------------------------------------------------
# Forward coefficients tabulated on the grid and per step (eq (1))
# ----------------------------------------------------------------------------


def test_tabulated_coefficients(lib, orc):
    from test_gpu_parity import TOL32, batched_solve

    # the affine Ornstein-Uhlenbeck drift as a table (one row, and one per step)
    for td in (False, True):
        _run(lib, orc, W.tabulated(W.ou_linear_1d(n_x=801, n_t=32), td))
    # a local volatility with skew and term structure, both drivers, both forms
    for drv in ("linear", "bidask"):
        wl = W.local_vol_call_1d(driver=drv)
        _run(lib, orc, wl)
        _run(lib, orc, wl, prec="fp32_comp", tol=TOL32)
    # time-varying vol on x^2: the left Riemann sum of sigma^2 at the interior
    wl = W.quadratic_time_varying_vol()
    y, _ = _run(lib, orc, wl)
    x = wl.grid(0)
    mid = np.abs(x) < 3.0
    assert np.max(np.abs(y[mid] - (x[mid] ** 2 + wl.extra["y0_scheme_offset"]))) < 1e-7
    # a batch mixing tabulated, affine and constant coefficients (one group on
    # the gather kernel)
    wls = [W.local_vol_call_1d(n_x=1500, n_t=20), W.ou_linear_1d(n_x=700, n_t=24),
           W.tabulated(W.bs_call_price_1d(n_x=900, n_t=16)), W.sine_1d(n_x=600, n_t=12, k=2)]
    rc, st, outs, _ = batched_solve(lib, wls)
    assert rc == lib.BSDE_OK
    for w, (y, z) in zip(wls, outs):
        iy, iz = w.init_layers()
        yo, zo, _ = orc.solve(w.problem, iy, iz)
        e = max(rel_err(y, yo), rel_err(z, zo[0]))
        print(f"  batch {w.name}: rel err {e:.3e}", flush=True)
        assert e <= TOL64


def test_tabulated_coefficients_initial_layers(lib, orc):
    # per-step table: each 1-step segment holds the row of its start time
    _initial_layers_case(lib, orc, W.local_vol_call_1d(n_x=1201, n_t=24, k=4), 5)


# ----------------------------------------------------------------------------
# Checkpoint and resume: the layers of a solve stopped at n_stop, exported and
# used as the initial layers of the remaining sweep
# ----------------------------------------------------------------------------


def _resume_case(lib, orc, wl, n_stop, prec, tol, batch_with=None):
    import torch

    pb = dict(wl.problem, prec=prec)
    K, N, d = max(pb["k_y"], pb["k_z"]), pb["n_t"], pb["d"]
    print(f"[case] resume {wl.name} {prec} at n_stop={n_stop}", flush=True)
    iy, iz = wl.init_layers()
    npts = iy.shape[1]
    y_full, z_full, rc, _ = lib.solve(pb, iy, iz)
    assert rc == lib.BSDE_OK
    # the solve stopped at n_stop, as instance b of a batch when batch_with is given
    probs = [dict(pb, n_stop=n_stop)]
    others = []
    if batch_with is not None:
        probs.insert(0, dict(batch_with.problem, prec=prec))
        others = [batch_with]
    plan = lib.bsde_plan(probs)
    ws = lib.workspace(plan)
    ios = []
    for w, p in zip(others + [wl], probs):
        jy, jz = w.init_layers()
        n = jy.shape[1]
        ios.append((torch.as_tensor(jy, device="cuda").contiguous(),
                    torch.as_tensor(jz.reshape(jy.shape[0], -1), device="cuda").contiguous(),
                    torch.empty(n, dtype=torch.float64, device="cuda"),
                    torch.empty(p["d"] * n, dtype=torch.float64, device="cuda")))
    rc, _ = lib.bsde_solve_batched(plan, ws, ios)
    assert rc == lib.BSDE_OK
    b = len(probs) - 1
    ly = torch.full((K, npts), float("nan"), dtype=torch.float64, device="cuda")
    lz = torch.full((K, d * npts), float("nan"), dtype=torch.float64, device="cuda")
    lib.bsde_checkpoint_layers(plan, ws, b, ly, lz)
    torch.cuda.synchronize()
    ly, lz = ly.cpu().numpy(), lz.cpu().numpy().reshape(K, d, npts)
    # row 0 is layer n_stop, the solve's own output
    assert rel_err(ly[0], ios[b][2].cpu().numpy()) <= (0.0 if prec == "fp64" else 1e-7)
    n2 = n_stop + K - 1
    pb2 = dict(pb, n_t=n2, T=pb["T"] * n2 / N, n_stop=0)
    if pb.get("coef_tab") is not None and len(pb["coef_tab"]) > 1:
        pb2["coef_tab"] = pb["coef_tab"][:n2]  # a per-step table: the remaining steps' rows
    y_r, z_r, rc2, _ = lib.solve(pb2, ly, lz)
    assert rc2 == lib.BSDE_OK
    e = max(rel_err(y_r, y_full), max(rel_err(z_r[c], z_full[c]) for c in range(d)))
    print(f"  resumed vs uninterrupted: rel err {e:.3e}", flush=True)
    assert e <= tol


def test_checkpoint_resume(lib, orc):
    from test_gpu_parity import TOL32

    nx, nt = 3001, 40
    bid = W.bidask_call_1d(n_x=nx, n_t=nt, half_width=twin_half_width(0.2, 0.5, nt, nx))
    _resume_case(lib, orc, bid, 17, "fp64", 1e-12)
    _resume_case(lib, orc, bid, 17, "fp32_comp", TOL32)
    ex = W.bs_call_1d(n_x=2049, n_t=24, k=3, L=16, half_width=twin_half_width(0.2, 0.33, 24, 2049))
    ex.problem["quad"] = "exact"
    _resume_case(lib, orc, ex, 9, "fp64", 1e-12)
    _resume_case(lib, orc, W.local_vol_call_1d(n_x=1201, n_t=24), 8, "fp64", 1e-12)
    _resume_case(lib, orc, W.sine_1d(n_x=900, n_t=30, k=3), 11, "fp64", 1e-12,
                 batch_with=W.sine_1d(n_x=500, n_t=20, k=2))
    two = W.exchange_2d(n_x=49, n_t=12, k=3, L=6, rho=0.4)
    _resume_case(lib, orc, two, 5, "fp64", 1e-12)
    _resume_case(lib, orc, two, 5, "fp32_comp", TOL32)


def test_edge_cases_of_the_newer_paths(lib, orc):
    from test_gpu_parity import TOL32

    # exact expectations (Toeplitz sweep) on the smallest grids, a ragged last
    # tile, a last tile of one point after a full one whose spline window
    # (33 points either side) crosses the domain end, and a single backward
    # step (N = K)
    for nx, nt, k in ((4, 12, 3), (5, 10, 2), (257, 9, 3), (1025, 8, 3), (300, 4, 4)):
        wl = W.sine_1d(n_x=nx, n_t=nt, k=k)
        wl.problem["quad"] = "exact"
        _run(lib, orc, wl)
    # tabulated coefficients (gather sweep) on the smallest grid and one step
    for nx, nt in ((4, 8), (65, 3)):
        wl = W.tabulated(W.ou_linear_1d(n_x=nx, n_t=nt, k=3), True)
        _run(lib, orc, wl)
    # the FP32 form in 2-D on the smallest grids of each interpolant and one step
    for interp, n in (("spline", 4), ("bicubic_fd", 5)):
        wl = W.exchange_2d(n_x=n, n_t=6, k=2, L=4, rho=0.3)
        wl.problem["interp"] = interp
        _run(lib, orc, wl, prec="fp32_comp", tol=TOL32)
    wl = W.exchange_2d(n_x=33, n_t=3, k=3, L=5, rho=0.2)
    _run(lib, orc, wl, prec="fp32_comp", tol=TOL32)
