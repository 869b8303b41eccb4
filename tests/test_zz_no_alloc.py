"""The entry point that allocates nothing (bsde_solve_batched_static) against
bsde_solve_batched with a caller-owned workspace: the same kernels on the
same inputs, so the outputs must agree bit for bit; two calls in a row, the
second on a smaller problem, and a plan too large for the static buffer.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1909_13560_amd as B

    B.load()
    return B


def _ios(wls):
    import torch

    ios = []
    for w in wls:
        iy, iz = w.init_layers()
        K, n = iy.shape
        ios.append((torch.as_tensor(iy, device="cuda").contiguous(),
                    torch.as_tensor(iz.reshape(K, -1), device="cuda").contiguous(),
                    torch.full((n,), float("nan"), dtype=torch.float64, device="cuda"),
                    torch.full((iz.shape[1] * n,), float("nan"), dtype=torch.float64,
                               device="cuda")))
    return ios


def _case(lib, wls):
    import torch

    print(f"[case] static workspace: {[w.name for w in wls]}", flush=True)
    plan = lib.bsde_plan([w.problem for w in wls])
    assert lib.bsde_workspace_bytes(plan) <= lib.STATIC_WORKSPACE_BYTES
    ref = _ios(wls)
    ws = lib.workspace(plan)
    rc, _ = lib.bsde_solve_batched(plan, ws, ref)
    got = _ios(wls)
    rc2 = lib.bsde_solve_batched_static(plan, got)
    torch.cuda.synchronize()
    assert rc == lib.BSDE_OK and rc2 == lib.BSDE_OK
    for (_, _, y_r, z_r), (_, _, y_s, z_s) in zip(ref, got):
        assert torch.equal(y_r, y_s) and torch.equal(z_r, z_s)
        assert bool(torch.isfinite(y_s).all()) and bool(torch.isfinite(z_s).all())


def test_static_workspace_matches_caller_workspace(lib):
    # first a larger batch (both precisions, a 2-D-free mix of sizes), then a
    # smaller single problem: the second call finds the first one's data in
    # the static buffer and must not depend on it
    big = [W.bidask_call_1d(n_x=40111, n_t=24, half_width=None),
           W.bs_call_1d(n_x=5000, n_t=16, k=5, L=16, half_width=None)]
    big[1].problem["prec"] = "fp32_comp"
    _case(lib, big)
    _case(lib, [W.sine_1d(n_x=700, n_t=20, k=2)])


def test_static_workspace_two_dimensional(lib):
    _case(lib, [W.exchange_2d(n_x=65, n_t=8, k=3, L=8, rho=0.5)])


def test_static_workspace_rejects_large_plans(lib):
    # a ring of 5 slots x 2 planes x 500000 points x 16 bytes is 80 MB
    wl = W.bidask_call_1d(n_x=500000, n_t=8, half_width=None)
    plan = lib.bsde_plan(wl.problem)
    assert lib.bsde_workspace_bytes(plan) > lib.STATIC_WORKSPACE_BYTES
    rc = lib.bsde_solve_batched_static(plan, _ios([wl]), check=False)
    assert rc == lib.BSDE_ESCRATCH
    assert "static" in lib.bsde_status_string(rc)
