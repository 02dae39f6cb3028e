"""Voronoi-area node weights on the GPU (hamls_plan_voronoi_areas) against the
oracle's brute-force cells, through the C ABI, and their use as the node
weights of a fit (Sec. 2.2, the remark after Thm. 2.1; Sec. 3)."""
import math

import numpy as np
import pytest

import oracle
from paper_2609_39200_amd import workloads as W

import _parity as PAR

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch  # noqa: F401

    from paper_2609_39200_amd import hamls

    return hamls


def _dev(a):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _areas(H, wl):
    import torch

    p = H.params_from_workload(wl.params)
    plan = H.hamls_plan(p, _dev(wl.nodes))
    a = torch.full((wl.nodes.shape[0],), float("nan"), dtype=torch.float64, device="cuda")
    H.hamls_plan_voronoi_areas(plan, a)
    torch.cuda.synchronize()
    return plan, a


@pytest.mark.parametrize("M,caps", [(3000, 0), (20000, 4)])
def test_voronoi_areas_match_oracle(H, M, caps):
    wl = W.s2_clusters(seed=811 + caps, M=M, N=16, K=2, n_caps=caps, field_degree=10)
    PAR.say(f"[gpu-voronoi] M={M} caps={caps}")
    plan, a = _areas(H, wl)
    try:
        g = a.cpu().numpy()
        o = oracle.voronoi_areas(wl.nodes)
        assert not np.isnan(o).any()
        assert not np.isnan(g).any()
        err = PAR.maxrel(g, o)
        rel = float(np.max(np.abs(g / o - 1)))
        PAR.say(f"  areas: max |diff| / max area {err:.2e}, max relative {rel:.2e}, sum - 4 pi {g.sum() - 4 * math.pi:.2e}")
        assert rel < 1e-10
        assert abs(g.sum() - 4 * math.pi) < 1e-9
    finally:
        H.hamls_plan_destroy(plan)


def test_voronoi_weighted_fit_matches_oracle(H):
    """The areas as node weights of a fit (rebind with them): grid values
    equal the oracle's fit with the oracle's own areas as weights."""
    import torch

    wl = W.s2_clusters(seed=820, M=15000, N=20, K=3, n_caps=3, field_degree=20)
    PAR.say("[gpu-voronoi] weighted fit")
    plan, a = _areas(H, wl)
    try:
        nodes = _dev(wl.nodes)
        H.hamls_plan_rebind(plan, nodes, node_weights=a)
        info = H.hamls_plan_info_get(plan)
        gv = torch.empty((1, info.num_grid), dtype=torch.float64, device="cuda")
        H.hamls_mls_to_grid(plan, _dev(wl.values), gv)
        torch.cuda.synchronize()
        po = oracle.params(**wl.params)
        gpts, _ = H.hamls_plan_grid(plan)
        ow = oracle.voronoi_areas(wl.nodes)
        om = oracle.mls(po, gpts, wl.nodes, wl.values, node_weights=ow)
        g = gv.cpu().numpy()
        err = PAR.rell2(g, om["values"])
        PAR.say(f"  weighted grid values vs oracle: rel L2 {err:.2e}")
        assert err < 1e-10
    finally:
        H.hamls_plan_destroy(plan)


def test_voronoi_full_size_c2(H):
    """The 200,000 clustered nodes with holes: every cell closed (no NaN),
    areas positive and summing to 4 pi, and 400 sampled nodes (and the 100
    largest cells, on the holes' rims) against the oracle's cells built from
    all nodes."""
    wl = W.s2_clusters()
    PAR.say("[gpu-voronoi] C2 nodes")
    plan, a = _areas(H, wl)
    try:
        g = a.cpu().numpy()
        assert not np.isnan(g).any() and (g > 0).all()
        assert abs(g.sum() - 4 * math.pi) < 1e-8
        rng = np.random.default_rng(830)
        rows = np.concatenate([rng.choice(wl.nodes.shape[0], 400, replace=False), np.argsort(g)[-100:]])
        o = oracle.voronoi_areas(wl.nodes, rows=rows)
        rel = float(np.max(np.abs(g[rows] / o - 1)))
        PAR.say(f"  sampled cells vs oracle: max relative {rel:.2e}; largest cell {g.max():.3e} sr")
        assert rel < 1e-10
    finally:
        H.hamls_plan_destroy(plan)
