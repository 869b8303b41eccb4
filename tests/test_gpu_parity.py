"""GPU parity: the HIP path against the CPU oracle, element by element.

Every case runs the same seeded/closed-form inputs through the C ABI (on the
GPU) and through the serial FP64 oracle, and compares the whole output layer.
FP64 bar: max_i |gpu_i - oracle_i| / max(|oracle_i|, 1) <= 1e-10.
FP32 form: the same measure <= 1e-6 (single-precision ring and node
arithmetic; the rounding of one layer, about 6e-8 relative, is averaged
rather than amplified by the quadrature, so the error stays a small
multiple of it over the whole sweep).
"""
import math
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOL32 = 1e-6


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


def rel_err(g, o):
    return float(np.max(np.abs(g - o) / np.maximum(np.abs(o), 1.0)))


def run_both(lib, orc, wl, n_stop=0, tol=TOL64, stats=True, prec="fp64"):
    pb = dict(wl.problem)
    pb["n_stop"] = n_stop
    pb["prec"] = prec
    print(f"[case] {wl.name} {prec} n_stop={n_stop} R={W.stability_ratio(pb):.2f}", flush=True)
    sys.stdout.flush()
    iy, iz = wl.init_layers()
    y, z, rc, st = lib.solve(pb, iy, iz, stats=stats)
    yo, zo, sto = orc.solve(pb, iy, iz, n_stop=n_stop)
    ey, ez = rel_err(y, yo), rel_err(z[0], zo[0])
    print(f"  rel err y {ey:.3e} z {ez:.3e} stats {st}", flush=True)
    assert ey <= tol and ez <= tol, (ey, ez)
    return y, z, yo, zo, rc, st, sto


def twin_half_width(sigma, T, n_t, n_x, R=16.0):
    """Half-width of the log-price interval that gives stability ratio R."""
    return sigma * math.sqrt(2 * T / n_t) / R * (n_x - 1) / 2


def test_sine_problem(lib, orc):
    wl = W.sine_1d()
    y, z, yo, zo, rc, st, _ = run_both(lib, orc, wl)
    assert rc == lib.BSDE_OK and st["picard_iter_max"] == 30
    i = wl.node_index()
    assert abs(y[i] - 0.0) < 1e-4 and abs(z[0, i] - 1.0) < 2e-4


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_black_scholes_all_orders(lib, orc, k):
    nx, nt = 3001, 40
    wl = W.bs_call_1d(n_x=nx, n_t=nt, k=k, L=32, half_width=twin_half_width(0.2, 0.33, nt, nx))
    run_both(lib, orc, wl)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_bid_ask_every_layer_order(lib, orc, k):
    # a grid of 157 tiles: the tiles take every rotation of the layer order
    # (tile / 32 mod 4, reduced mod K), and the windows away from the domain
    # ends take the stencil form of the spline
    nx, nt = 40111, 10
    wl = W.bidask_call_1d(n_x=nx, n_t=nt, k=k, L=16, half_width=twin_half_width(0.2, 0.5, nt, nx))
    _, _, _, _, rc, st, sto = run_both(lib, orc, wl)
    assert rc == lib.BSDE_OK and st["picard_nonconverged"] == 0


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_bid_ask_ragged_grid(lib, orc, sign):
    nx, nt = 5003, 48
    wl = W.bidask_call_1d(n_x=nx, n_t=nt, sign=sign, half_width=twin_half_width(0.2, 0.5, nt, nx))
    _, _, _, _, rc, st, sto = run_both(lib, orc, wl)
    assert rc == lib.BSDE_OK
    assert st["picard_iter_max"] == sto["picard_iter_max"]
    assert st["picard_nonconverged"] == 0


def test_example1_table4_row(lib, orc):
    # Example 1, K = 3, N = 128, M = 4096: the paper prints 1.44e-11 / 2.77e-8
    wl = W.paper_example1(3, 128, 4096)
    y, z, *_ = run_both(lib, orc, wl)
    i = wl.node_index()
    assert abs(y[i] - 0.5) == pytest.approx(1.44e-11, rel=0.03)
    assert abs(z[0, i] - 0.25) == pytest.approx(2.77e-8, rel=0.02)


def test_example2_exp_driver(lib, orc):
    run_both(lib, orc, W.paper_example2(4, 32, 1024))


@pytest.mark.parametrize("ky,kz", [(2, 3), (3, 1), (1, 4)])
def test_unequal_orders(lib, orc, ky, kz):
    wl = W.sine_1d(n_x=777, n_t=30)
    wl.problem.update(k_y=ky, k_z=kz)
    run_both(lib, orc, wl)


@pytest.mark.parametrize("n_x", [4, 5, 63, 64, 65, 513])
def test_small_and_ragged_grids(lib, orc, n_x):
    wl = W.sine_1d(n_x=n_x, n_t=12, k=3)
    run_both(lib, orc, wl)


@pytest.mark.parametrize("L", [1, 2, 7, 64])
def test_quadrature_orders(lib, orc, L):
    wl = W.sine_1d(n_x=300, n_t=10, k=2, L=L)
    run_both(lib, orc, wl)


def test_single_step(lib, orc):
    # N = K: exactly one backward step
    wl = W.sine_1d(n_x=100, n_t=4, k=4)
    run_both(lib, orc, wl)


def test_checkpoint_layer(lib, orc):
    wl = W.bidask_call_1d(n_x=2000, n_t=40, half_width=None)
    run_both(lib, orc, wl, n_stop=17)


def test_wide_reach_literal_domain(lib, orc):
    # large stability ratio: nodes reach far beyond the tile, ghost cells wide
    wl = W.bidask_call_1d(n_x=20000, n_t=16, half_width=None)
    run_both(lib, orc, wl)


def test_full_size_bidask_first_steps(lib, orc):
    # the benchmarked shape: 262144 points, 1024 steps, k = 4, L = 16, stable
    # domain; the oracle follows the first four steps
    nx, nt = 262144, 1024
    wl = W.bidask_call_1d(n_x=nx, n_t=nt, half_width=52.0)
    run_both(lib, orc, wl, n_stop=nt - 4 - 3)


def test_deterministic(lib):
    wl = W.bidask_call_1d(n_x=3000, n_t=20, half_width=None)
    iy, iz = wl.init_layers()
    y1, z1, _, _ = lib.solve(wl.problem, iy, iz)
    y2, z2, _, _ = lib.solve(wl.problem, iy, iz)
    assert np.array_equal(y1, y2) and np.array_equal(z1, z2)


def test_nonfinite_is_reported(lib):
    wl = W.sine_1d(n_x=200, n_t=8)
    iy, iz = wl.init_layers()
    iy[-1, 100] = np.nan
    y, z, rc, st = lib.solve(wl.problem, iy, iz)
    assert rc == lib.BSDE_ENONFINITE and st["nonfinite"] > 0


def test_picard_nonconvergence_is_reported(lib):
    wl = W.bidask_call_1d(n_x=500, n_t=10, half_width=None, picard_tol=1e-300, picard_max=2)
    iy, iz = wl.init_layers()
    y, z, rc, st = lib.solve(wl.problem, iy, iz)
    assert rc == lib.BSDE_ENOCONV
    assert st["picard_nonconverged"] > 0 and st["picard_iter_max"] == 2


def test_batched_equals_single(lib):
    import torch

    # the last instance has 157 tiles, so its tiles take every rotation of the
    # layer order; in the batch they sit behind the other instances' tiles
    wls = [W.sine_1d(n_x=700, n_t=20, k=2), W.bidask_call_1d(n_x=1500, n_t=16, half_width=None),
           W.bs_call_1d(n_x=999, n_t=12, k=5, L=16, half_width=None),
           W.bidask_call_1d(n_x=40111, n_t=12, half_width=twin_half_width(0.2, 0.5, 12, 40111))]
    plan = lib.bsde_plan([w.problem for w in wls])
    ws = lib.workspace(plan)
    ios, outs = [], []
    for w in wls:
        iy, iz = w.init_layers()
        n = iy.shape[1]
        t_iy = torch.as_tensor(iy, device="cuda").contiguous()
        t_iz = torch.as_tensor(iz.reshape(iy.shape[0], n), device="cuda").contiguous()
        y0 = torch.empty(n, dtype=torch.float64, device="cuda")
        z0 = torch.empty(n, dtype=torch.float64, device="cuda")
        ios.append((t_iy, t_iz, y0, z0))
    rc, st = lib.bsde_solve_batched(plan, ws, ios, stats=True)
    torch.cuda.synchronize()
    assert rc == lib.BSDE_OK
    for w, (t_iy, t_iz, y0, z0) in zip(wls, ios):
        iy, iz = w.init_layers()
        y, z, _, _ = lib.solve(w.problem, iy, iz)
        assert np.array_equal(y0.cpu().numpy(), y)
        assert np.array_equal(z0.cpu().numpy(), z[0])


def test_graph_replays_match_direct_launches(lib, monkeypatch):
    # the solve is captured once per buffer set and replayed; every replay,
    # with eager work in between, must equal a directly launched solve
    import torch

    wl = W.bidask_call_1d(n_x=4000, n_t=30, half_width=None)
    iy, iz = wl.init_layers()
    monkeypatch.setenv("BSDE_GRAPH", "0")
    plan_d = lib.bsde_plan(wl.problem)
    monkeypatch.setenv("BSDE_GRAPH", "1")
    plan_g = lib.bsde_plan(wl.problem)
    ws_d, ws_g = lib.workspace(plan_d), lib.workspace(plan_g)
    t_iy = torch.as_tensor(iy, device="cuda").contiguous()
    t_iz = torch.as_tensor(iz.reshape(iy.shape), device="cuda").contiguous()
    n = iy.shape[1]
    yd, zd = (torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(2))
    yg, zg = (torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(2))
    lib.bsde_solve(plan_d, ws_d, t_iy, t_iz, yd, zd)
    torch.cuda.synchronize()
    ref_y, ref_z = yd.clone(), zd.clone()
    for rep in range(4):
        yg.fill_(float("nan"))
        zg.fill_(float("nan"))
        lib.bsde_solve(plan_g, ws_g, t_iy, t_iz, yg, zg)
        lib.bsde_solve(plan_d, ws_d, t_iy, t_iz, yd, zd)  # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(yg, ref_y) and torch.equal(zg, ref_z), rep
        assert torch.equal(yd, ref_y) and torch.equal(zd, ref_z), rep


def test_graph_cache_eviction_keeps_results(lib):
    # a plan keeps the captured solves of its four most recently used buffer
    # sets; cycling through six sets evicts and recaptures on every call, and
    # each solve must still equal the first one bit for bit
    import torch

    wl = W.bidask_call_1d(n_x=2500, n_t=14, half_width=None)
    iy, iz = wl.init_layers()
    n = iy.shape[1]
    plan = lib.bsde_plan(wl.problem)
    sets = []
    for _ in range(6):
        sets.append((lib.workspace(plan), torch.as_tensor(iy, device="cuda").contiguous(),
                     torch.as_tensor(iz.reshape(iy.shape), device="cuda").contiguous(),
                     torch.empty(n, dtype=torch.float64, device="cuda"),
                     torch.empty(n, dtype=torch.float64, device="cuda")))
    ref = None
    for rep in range(2):
        for k, (ws, a, b, y, z) in enumerate(sets):
            y.fill_(float("nan"))
            z.fill_(float("nan"))
            lib.bsde_solve(plan, ws, a, b, y, z)
            torch.cuda.synchronize()
            if ref is None:
                ref = (y.clone(), z.clone())
            assert torch.equal(y, ref[0]) and torch.equal(z, ref[1]), (rep, k)


def test_single_solve_rejects_batched_plan(lib):
    import torch

    wls = [W.sine_1d(n_x=300, n_t=8), W.sine_1d(n_x=400, n_t=8)]
    plan = lib.bsde_plan([w.problem for w in wls])
    ws = lib.workspace(plan)
    iy, iz = wls[0].init_layers()
    t_iy = torch.as_tensor(iy, device="cuda").contiguous()
    t_iz = torch.as_tensor(iz.reshape(iy.shape), device="cuda").contiguous()
    y0 = torch.empty(iy.shape[1], dtype=torch.float64, device="cuda")
    z0 = torch.empty_like(y0)
    rc, _ = lib.bsde_solve(plan, ws, t_iy, t_iz, y0, z0, check=False)
    assert rc == lib.BSDE_EINVAL


# ----------------------------------------------------------------------------
# FP32 form
# ----------------------------------------------------------------------------


def test_fp32_sine_problem(lib, orc):
    run_both(lib, orc, W.sine_1d(), tol=TOL32, prec="fp32_comp")


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_fp32_black_scholes_all_orders(lib, orc, k):
    nx, nt = 3001, 40
    wl = W.bs_call_1d(n_x=nx, n_t=nt, k=k, L=32, half_width=twin_half_width(0.2, 0.33, nt, nx))
    run_both(lib, orc, wl, tol=TOL32, prec="fp32_comp")


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_fp32_bid_ask_ragged_grid(lib, orc, sign):
    nx, nt = 5003, 48
    wl = W.bidask_call_1d(n_x=nx, n_t=nt, sign=sign, half_width=twin_half_width(0.2, 0.5, nt, nx))
    _, _, _, _, rc, st, _ = run_both(lib, orc, wl, tol=TOL32, prec="fp32_comp")
    assert rc == lib.BSDE_OK and st["picard_nonconverged"] == 0


def test_fp32_long_sweep_against_oracle_and_closed_form(lib, orc):
    # the benchmarked time grid and stability ratio (1024 steps, R = 15.75) on
    # a shorter grid the oracle sweeps in seconds
    nx, nt = 4097, 1024
    wl = W.bidask_call_1d(n_x=nx, n_t=nt, half_width=twin_half_width(0.2, 0.5, nt, nx, 15.75))
    y, z, yo, zo, *_ = run_both(lib, orc, wl, tol=TOL32, prec="fp32_comp")
    ye, ze = wl.exact_at_t0()
    i = wl.node_index()
    assert abs(y[i] - ye[i]) / abs(ye[i]) <= TOL32
    assert abs(z[0, i] - ze[i]) / abs(ze[i]) <= TOL32


def test_fp32_direct_path_wide_reach(lib, orc):
    wl = W.bidask_call_1d(n_x=20000, n_t=16, half_width=None)
    run_both(lib, orc, wl, tol=TOL32, prec="fp32_comp")


def test_fp32_full_size_first_steps(lib, orc):
    nx, nt = 262144, 1024
    wl = W.bidask_call_1d(n_x=nx, n_t=nt, half_width=52.0)
    run_both(lib, orc, wl, n_stop=nt - 4 - 3, tol=TOL32, prec="fp32_comp")


def test_fp32_small_grids_and_orders(lib, orc):
    for n_x, L in [(4, 16), (65, 7), (513, 64)]:
        run_both(lib, orc, W.sine_1d(n_x=n_x, n_t=12, k=3, L=L), tol=TOL32, prec="fp32_comp")


# ----------------------------------------------------------------------------
# Batched solves
# ----------------------------------------------------------------------------


def batched_solve(lib, wls, autotune=False):
    import torch

    plan = lib.bsde_plan([w.problem for w in wls])
    ws = lib.workspace(plan)
    ios = []
    for w in wls:
        iy, iz = w.init_layers()
        n = iy.shape[1]
        ios.append((torch.as_tensor(iy, device="cuda").contiguous(),
                    torch.as_tensor(iz.reshape(iy.shape[0], n), device="cuda").contiguous(),
                    torch.empty(n, dtype=torch.float64, device="cuda"),
                    torch.empty(n, dtype=torch.float64, device="cuda")))
    rep = lib.bsde_autotune(plan, ws, ios, reps=2) if autotune else None
    rc, st = lib.bsde_solve_batched(plan, ws, ios, stats=True)
    torch.cuda.synchronize()
    return rc, st, [(io[2].cpu().numpy(), io[3].cpu().numpy()) for io in ios], rep


def test_batched_mixed_precisions_and_lengths(lib, orc):
    wls = [W.sine_1d(n_x=700, n_t=20, k=2), W.bidask_call_1d(n_x=1500, n_t=16, half_width=None),
           W.bs_call_1d(n_x=999, n_t=12, k=5, L=16, half_width=None),
           W.bs_call_1d(n_x=2100, n_t=30, k=3, L=16, half_width=None),
           W.bidask_call_1d(n_x=3001, n_t=40, half_width=None),
           W.sine_1d(n_x=64, n_t=9, k=4)]
    precs = ["fp64", "fp32_comp", "fp64", "fp32_comp", "fp64", "fp32_comp"]
    for w, p in zip(wls, precs):
        w.problem["prec"] = p
    wls[4].problem["n_stop"] = 7
    rc, st, outs, _ = batched_solve(lib, wls)
    assert rc == lib.BSDE_OK
    for w, p, (y, z) in zip(wls, precs, outs):
        iy, iz = w.init_layers()
        yo, zo, _ = orc.solve(w.problem, iy, iz, n_stop=w.problem.get("n_stop", 0))
        tol = TOL64 if p == "fp64" else TOL32
        e = max(rel_err(y, yo), rel_err(z, zo[0]))
        print(f"[case] {w.name} {p}: {e:.3e}", flush=True)
        assert e <= tol, (w.name, e)


def test_option_batch_subsample(lib, orc):
    # the seeded batched workload's recipe at small grids and few steps
    wls = W.option_batch(count=12, log2_nx=(10.0, 12.0), n_ts=(64, 128))
    rc, st, outs, _ = batched_solve(lib, wls)
    assert rc == lib.BSDE_OK and st["picard_nonconverged"] == 0
    assert st["stability_ratio"] <= 16.0 + 1e-9
    for w, (y, z) in zip(wls, outs):
        iy, iz = w.init_layers()
        yo, zo, _ = orc.solve(w.problem, iy, iz)
        e = max(rel_err(y, yo), rel_err(z, zo[0]))
        print(f"[case] {w.name}: {e:.3e}", flush=True)
        assert e <= TOL32, (w.name, e)


def test_autotune_keeps_results(lib, orc):
    wls = [W.bidask_call_1d(n_x=20011, n_t=24, half_width=twin_half_width(0.2, 0.5, 24, 20011)),
           W.bs_call_1d(n_x=5000, n_t=16, k=4, L=16, half_width=None)]
    rc, st, outs, rep = batched_solve(lib, wls, autotune=True)
    print(f"[case] autotune report {rep}", flush=True)
    assert rc == lib.BSDE_OK and rep["candidates"] >= 2 and rep["best_ms_per_step"] > 0
    for w, (y, z) in zip(wls, outs):
        iy, iz = w.init_layers()
        yo, zo, _ = orc.solve(w.problem, iy, iz)
        assert max(rel_err(y, yo), rel_err(z, zo[0])) <= TOL64


# ----------------------------------------------------------------------------
# Two space dimensions
# ----------------------------------------------------------------------------


def test_2d_example4_table9_row(lib, orc):
    # Example 4, K = 3, N = 8, M = 128: the paper prints 3.94e-4 / 1.43e-3
    wl = W.sine_2d(n_x=129, n_t=8, k=3, L=8)
    y, z, yo, zo, *_ = run_both(lib, orc, wl)
    assert rel_err(z[1], zo[1]) <= TOL64
    i = wl.node_index()
    assert abs(y[i]) == pytest.approx(3.94e-4, rel=0.01)
    assert math.hypot(z[0, i] - 1.0, z[1, i] - 1.0) == pytest.approx(1.43e-3, rel=0.01)


@pytest.mark.parametrize("rho", [0.0, 0.5])
def test_2d_exchange_option(lib, orc, rho):
    wl = W.exchange_2d(n_x=97, n_t=10, k=3, L=8, rho=rho)
    y, z, yo, zo, *_ = run_both(lib, orc, wl)
    assert rel_err(z[1], zo[1]) <= TOL64
    ye, ze = wl.exact_at_t0()
    i = wl.node_index()
    assert abs(y[i] - ye[i]) < 1e-4


def test_2d_ragged_grid_unequal_orders(lib, orc):
    wl = W.exchange_2d(n_x=77, n_t=9, k=2, L=7, rho=0.3)
    pb = wl.problem
    pb["n_x"] = [77, 130]
    pb["x_max"] = [pb["x_max"][0], pb["x_min"][1] + 129 * (pb["x_max"][1] - pb["x_min"][1]) / 76]
    pb["k_y"], pb["k_z"] = 3, 2
    wl.x0 = (pb["x_min"][0], pb["x_min"][1])
    y, z, yo, zo, *_ = run_both(lib, orc, wl)
    assert rel_err(z[1], zo[1]) <= TOL64


def test_2d_short_columns_wide_ragged_rows(lib, orc):
    # 21 points along axis 0 (shorter than the spline filter's one-reflection
    # reach: the point-by-point spline form) and 700 along axis 1 (two sweep
    # tiles per row, the second ragged; spline runs ending in a partial run)
    wl = W.exchange_2d(n_x=21, n_t=12, k=2, L=6, rho=0.4)
    pb = wl.problem
    dx1 = (pb["x_max"][0] - pb["x_min"][0]) / 20 / 8
    pb["n_x"] = [21, 700]
    pb["x_max"] = [pb["x_max"][0], pb["x_min"][1] + 699 * dx1]
    y, z, yo, zo, *_ = run_both(lib, orc, wl)
    assert rel_err(z[1], zo[1]) <= TOL64


def test_2d_short_rows(lib, orc):
    # 20 points along axis 1: the axis-1 spline lines are shorter than the
    # filter's one-reflection reach and take the point-by-point form
    wl = W.exchange_2d(n_x=40, n_t=10, k=3, L=6, rho=0.3)
    pb = wl.problem
    dx1 = (pb["x_max"][1] - pb["x_min"][1]) / 39
    pb["n_x"] = [40, 20]
    pb["x_max"] = [pb["x_max"][0], pb["x_min"][1] + 19 * dx1]
    y, z, yo, zo, *_ = run_both(lib, orc, wl)
    assert rel_err(z[1], zo[1]) <= TOL64


@pytest.mark.parametrize("prec", ["fp64", "fp32_comp"])
def test_2d_widest_window(lib, orc, prec):
    # 741 columns (two sweep tiles per row, the second ragged): the 16 x 16
    # nodes of a row at j = 3 spread over 239 cells along axis 1, the widest
    # row the sweep's 240-cell LDS window takes (its largest even/odd column
    # halves), at stability ratio 14.7; six steps to the checkpoint
    wl = W.exchange_2d(n_x=17, n_t=32, k=3, L=16, rho=0.3)
    wl.problem["n_x"] = [17, 741]
    y, z, yo, zo, *_ = run_both(lib, orc, wl, n_stop=24, prec=prec,
                                tol=TOL64 if prec == "fp64" else TOL32)
    assert rel_err(z[1], zo[1]) <= (TOL64 if prec == "fp64" else TOL32)


def test_2d_basket_checkpoint(lib, orc):
    wl = W.basket_2d(n_x=65, n_t=12, k=3, L=16)
    y, z, yo, zo, *_ = run_both(lib, orc, wl, n_stop=4)
    assert rel_err(z[1], zo[1]) <= TOL64


def test_2d_full_size_basket_sampled(lib, orc):
    # the benchmarked 2-D shape (1024 x 1024 grid, 128 steps, k = 3, 16 x 16
    # nodes, the same launch shape): the whole grid's first layer on the GPU
    # against the oracle at sampled points (a whole serial step takes minutes)
    wl = W.basket_2d()
    pb = dict(wl.problem)
    K = max(pb["k_y"], pb["k_z"])
    n0, n1 = pb["n_x"]
    pb["n_stop"] = pb["n_t"] - K
    iy, iz = wl.init_layers()
    print(f"[case] {wl.name} fp64 n_stop={pb['n_stop']} sampled", flush=True)
    y, z, rc, st = lib.solve(pb, iy, iz, stats=True)
    assert rc == lib.BSDE_OK
    rng = np.random.default_rng(1909)
    rows = np.concatenate([[0, 1, 2, n0 // 2, n0 - 2, n0 - 1],
                           np.arange(3, n0 - 2, 4), rng.integers(0, n0, 400)])
    cols = np.concatenate([[0, 1, 63, 64, 65, n1 // 2, n1 - 2, n1 - 1],
                           rng.integers(0, n1, rows.size - 8)])
    cols = np.resize(cols, rows.size)
    idx = np.unique(rows.astype(np.int64) * n1 + cols)
    ys, zs = orc.first_step_points_2d(pb, iy, iz, idx)
    ey = rel_err(y[idx], ys)
    ez = max(rel_err(z[0, idx], zs[0]), rel_err(z[1, idx], zs[1]))
    print(f"  {idx.size} points: rel err y {ey:.3e} z {ez:.3e}", flush=True)
    assert ey <= TOL64 and ez <= TOL64


def test_2d_autotune_reports_single_shape(lib, orc):
    # a two-dimensional plan has one kernel shape: autotune reports it and the
    # solve afterwards is unchanged
    import torch

    wl = W.exchange_2d(n_x=49, n_t=6, k=3, L=6, rho=0.5)
    iy, iz = wl.init_layers()
    n = iy.shape[1]
    plan = lib.bsde_plan(wl.problem)
    ws = lib.workspace(plan)
    io = (torch.as_tensor(iy, device="cuda").contiguous(),
          torch.as_tensor(iz.reshape(iy.shape[0], -1), device="cuda").contiguous(),
          torch.empty(n, dtype=torch.float64, device="cuda"),
          torch.empty(2 * n, dtype=torch.float64, device="cuda"))
    rep = lib.bsde_autotune(plan, ws, [io], reps=2)
    assert rep["path"] == 2 and rep["candidates"] == 0
    rc, _ = lib.bsde_solve_batched(plan, ws, [io])
    torch.cuda.synchronize()
    assert rc == lib.BSDE_OK
    yo, zo, _ = orc.solve(wl.problem, iy, iz)
    zz = io[3].cpu().numpy().reshape(2, n)
    assert rel_err(io[2].cpu().numpy(), yo) <= TOL64
    assert max(rel_err(zz[0], zo[0]), rel_err(zz[1], zo[1])) <= TOL64


def test_2d_picard_tolerance_and_batch(lib, orc):
    import torch

    wls = [W.sine_2d(n_x=33, n_t=6, k=2, L=8), W.exchange_2d(n_x=41, n_t=7, k=4, L=6, rho=0.5)]
    wls[0].problem["picard_tol"] = 1e-14
    plan = lib.bsde_plan([w.problem for w in wls])
    ws = lib.workspace(plan)
    ios = []
    for w in wls:
        iy, iz = w.init_layers()
        n = iy.shape[1]
        ios.append((torch.as_tensor(iy, device="cuda").contiguous(),
                    torch.as_tensor(iz.reshape(iy.shape[0], -1), device="cuda").contiguous(),
                    torch.empty(n, dtype=torch.float64, device="cuda"),
                    torch.empty(2 * n, dtype=torch.float64, device="cuda")))
    rc, st = lib.bsde_solve_batched(plan, ws, ios, stats=True)
    torch.cuda.synchronize()
    assert rc == lib.BSDE_OK and st["picard_nonconverged"] == 0
    for w, io in zip(wls, ios):
        iy, iz = w.init_layers()
        yo, zo, _ = orc.solve(w.problem, iy, iz)
        n = iy.shape[1]
        assert rel_err(io[2].cpu().numpy(), yo) <= TOL64
        zz = io[3].cpu().numpy().reshape(2, n)
        assert max(rel_err(zz[0], zo[0]), rel_err(zz[1], zo[1])) <= TOL64
