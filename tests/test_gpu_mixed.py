"""GPU tests of the mixed-precision path (FP32 Gram assembly with an FP64
residual refinement and FP64 fallback on S2, SO(3) and T3; FP32 MFMA Legendre
contraction on S2).

Bar: within 1e-6 relative L2 of the FP64 path on the same inputs, grid values
and coefficients; the FP64 path itself is held to the oracle elsewhere."""
import sys

import numpy as np
import pytest

from paper_2609_39200_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL_MIXED = 1e-6


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def H():
    import torch  # noqa: F401

    from paper_2609_39200_amd import hamls

    return hamls


def _dev(a):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _rell2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def _fit(H, wl, precision, values=None):
    import torch

    p = H.params_from_workload(wl.params, precision=precision)
    plan = H.hamls_plan(p, _dev(wl.nodes))
    try:
        info = H.hamls_plan_info_get(plan)
        vals = wl.values if values is None else values
        F = vals.shape[0]
        gv = torch.empty((F, info.num_grid), dtype=torch.float64, device="cuda")
        cf = torch.empty((F, info.num_coeffs, 2), dtype=torch.float64, device="cuda")
        H.hamls_mls_to_grid(plan, _dev(vals), gv)
        H.hamls_grid_to_coeffs(plan, gv, cf)
        torch.cuda.synchronize()
        dg = H.hamls_diagnostics(plan)
        return gv.cpu().numpy(), cf.cpu().numpy(), dg
    finally:
        H.hamls_plan_destroy(plan)


def _compare(H, wl, label, values=None):
    _say(f"[gpu-mixed] {label} {wl.name}")
    g64, c64, d64 = _fit(H, wl, "fp64", values)
    g32, c32, d32 = _fit(H, wl, "mixed", values)
    np.testing.assert_array_equal(np.isnan(g64), np.isnan(g32))
    ok = ~np.isnan(g64[0])
    eg = _rell2(g32[:, ok], g64[:, ok])
    _say(f"  grid values rel L2 mixed vs FP64: {eg:.3e}")
    assert eg < TOL_MIXED
    np.testing.assert_array_equal(d32["n"], d64["n"])
    if ok.all():
        ec = _rell2(c32, c64)
        _say(f"  coefficients rel L2 mixed vs FP64: {ec:.3e}")
        assert ec < TOL_MIXED
    return g64, g32, d64, d32


def test_mixed_c2_full(H):
    _compare(H, W.s2_clusters(), "C2")


@pytest.mark.parametrize("K", [0, 1, 2, 3, 4])
def test_mixed_degrees(H, K):
    wl = W.s2_clusters(seed=2600 + K, M=20000, N=24, K=K, n_caps=3, field_degree=40)
    _compare(H, wl, f"K{K}")


def test_mixed_fixed_radius_and_degenerate(H):
    # fixed tau > 0 sends every node to FP64; empty and underdetermined nodes
    rng = np.random.default_rng(5)
    caps = [(np.array([0.0, 0.0, 1.0]), 0.6)]
    nodes = W.cluster_hole_s2(3000, rng, caps=caps, frac_uniform=1.0)
    y = rng.standard_normal(3000)
    for reg, tau in (("fixed", 1e-8), ("none", 0.0)):
        wl = W.Workload("s2-hole-fixed", "s2", nodes, y[None, :],
                        dict(domain="s2", bandwidth=16, degree=2, support_radius=0.12, knn_count=0,
                             reg=reg, tau_fixed=tau))
        g64, _, d64 = _fit(H, wl, "fp64")
        g32, _, d32 = _fit(H, wl, "mixed")
        a, b = g64[0], g32[0]
        np.testing.assert_array_equal(np.isnan(a), np.isnan(b))
        # nodes with chi >= 1e3 are sensitive to rounding in themselves (see
        # the FP64 degenerate-node test); compare the rest
        ok = ~np.isnan(a) & np.isfinite(d64["chi"]) & (d64["chi"] < 1e3)
        e = _rell2(b[ok], a[ok])
        _say(f"  reg={reg}: rel L2 mixed vs FP64 on chi < 1e3: {e:.3e}")
        assert e < TOL_MIXED
        np.testing.assert_array_equal(d32["status"] & 7, d64["status"] & 7)


@pytest.mark.parametrize("F", [3, 19, 64, 70])
def test_mixed_many_fields_mfma_tiles(H, F):
    # the contraction's column chunks: F = 3 (one 32-column chunk), 19 (64),
    # 64 (one 128-column chunk), 70 (a second 128-column chunk)
    rng = np.random.default_rng(100 + F)
    wl = W.s2_clusters(seed=2700, M=30000, N=40, K=2, field_degree=50)
    vals = np.concatenate([wl.values, rng.standard_normal((F - 1, wl.nodes.shape[0]))], axis=0)
    _compare(H, wl, f"F={F}", values=vals)


def test_mixed_c3_full(H):
    _compare(H, W.s2_large(), "C3")


@pytest.mark.parametrize("K", [1, 2, 3])
def test_mixed_so3_degrees(H, K):
    wl = W.so3_clusters(seed=5300 + K, M=20000, N=8, K=K, grid=(0, 0, 0), field_degree=6)
    _compare(H, wl, f"so3 K{K}")


@pytest.mark.parametrize("K", [1, 2, 3])
def test_mixed_t3_degrees(H, K):
    wl = W.t3_clusters(seed=5310 + K, M=20000, N=6, K=K, grid=14, kmax=6)
    _compare(H, wl, f"t3 K{K}")


def test_mixed_grid_fields(H):
    rng = np.random.default_rng(5320)
    wl = W.so3_clusters(seed=5321, M=15000, N=6, K=2, grid=(0, 0, 0), field_degree=5)
    vals = np.concatenate([wl.values, rng.standard_normal((18, wl.nodes.shape[0]))], axis=0)
    _compare(H, wl, "so3 F=19", values=vals)


def test_mixed_so3_full(H):
    # the SO(3) benchmark workload (C5a: M = 10^6, N = 64, K = 2, 130^3)
    _compare(H, W.so3_clusters(), "so3 130^3")


def test_mixed_t3_full(H):
    # the T3 benchmark workload (C5b: M = 2 10^6, N = 64, K = 3, 128^3)
    _compare(H, W.t3_clusters(), "t3 128^3")


def test_mfma_contraction_c3_shape_64_fields(H):
    """Step 3 at the large configuration's shape (N = 512, grid 513 x 1026)
    with 64 fields of random grid values: the matrix-core contraction of the
    mixed path against the FP64 path, every coefficient."""
    import torch

    wl = W.s2_clusters(seed=2800, M=20000, N=512, K=4, n_caps=3, field_degree=40)
    gen = torch.Generator(device="cuda").manual_seed(2801)
    out = {}
    g = None
    for prec in ("fp64", "mixed"):
        p = H.params_from_workload(wl.params, precision=prec)
        plan = H.hamls_plan(p, _dev(wl.nodes))
        try:
            info = H.hamls_plan_info_get(plan)
            if g is None:
                g = torch.randn((64, info.num_grid), dtype=torch.float64, device="cuda", generator=gen)
            cf = torch.empty((64, info.num_coeffs, 2), dtype=torch.float64, device="cuda")
            H.hamls_grid_to_coeffs(plan, g, cf)
            torch.cuda.synchronize()
            out[prec] = cf.cpu().numpy()
        finally:
            H.hamls_plan_destroy(plan)
    e = _rell2(out["mixed"], out["fp64"])
    emax = float(np.abs(out["mixed"] - out["fp64"]).max() / np.abs(out["fp64"]).max())
    _say(f"[gpu-mixed] C3 shape, F = 64: coefficients rel L2 mixed vs FP64 {e:.3e}, max {emax:.3e}")
    assert e < TOL_MIXED and emax < TOL_MIXED
