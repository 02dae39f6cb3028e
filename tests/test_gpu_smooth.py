"""The smoothed adaptive radius (Sec. 2.2, after eq. (12)) on the GPU against
the FP64 oracle: d_n on the auxiliary Fibonacci grid by the plan's radius
search, its degree-zero MLS at every grid node, delta = (1 + eps) times that.

Bars: radii within 1e-12 relative (the Shepard sums run in another order);
neighbour sets bit-exact; grid values and coefficients within 1e-10 relative
L2."""
import sys

import numpy as np
import pytest

import oracle
from paper_2609_39200_amd import workloads as W

pytestmark = pytest.mark.gpu


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
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


@pytest.mark.parametrize("K,naux", [(2, 4000), (3, 1500)])
def test_smoothed_radius_matches_oracle(H, K, naux):
    import torch

    rng = np.random.default_rng(70 + K)
    x = W.cluster_hole_s2(20000, rng, caps=W.random_caps(4, 15.0, 25.0, rng))
    m = (K + 1) * (K + 2) // 2
    wp = dict(domain="s2", bandwidth=24, degree=K, knn_count=4 * m, knn_eps=0.05, reg="chi",
              smooth_aux=naux)
    _say("smooth", K, naux)
    p = H.params_from_workload(wp)
    plan = H.hamls_plan(p, _dev(x))
    try:
        delta, thr = H.hamls_plan_radii(plan)
        rp, idx = H.hamls_plan_neighbors(plan)
        po = oracle.params(**wp)
        g, _w = H.hamls_plan_grid(plan)  # the library's exported grid
        nb = oracle.neighbors(po, g, x, lists=True)
        derr = np.max(np.abs(delta - nb["delta"]) / nb["delta"])
        _say("delta rel", derr, "count min", int(np.diff(rp).min()))
        assert derr <= 1e-12
        assert np.array_equal(rp, nb["row_ptr"]) and np.array_equal(idx, nb["idx"])
        info = H.hamls_plan_info_get(plan)
        vals = _dev(rng.standard_normal((2, x.shape[0])))
        gv = torch.empty((2, info.num_grid), dtype=torch.float64, device="cuda")
        cf = torch.empty((2, info.num_coeffs, 2), dtype=torch.float64, device="cuda")
        H.hamls_mls_to_grid(plan, vals, gv)
        H.hamls_grid_to_coeffs(plan, gv, cf)
        torch.cuda.synchronize()
        ref = oracle.mls(po, g, x, vals.cpu().numpy())
        err = _rell2(gv.cpu().numpy(), ref["values"])
        cref = oracle.coeffs(po, ref["values"])
        c = cf.cpu().numpy()
        cerr = _rell2(c[..., 0] + 1j * c[..., 1], cref)
        _say("values", err, "coeffs", cerr)
        assert err <= 1e-10 and cerr <= 1e-10
        # the radius is smooth: no jumps between neighbouring grid nodes beyond
        # those of the raw kNN radius
        praw = H.params_from_workload(dict(wp, smooth_aux=0))
        plan2 = H.hamls_plan(praw, _dev(x))
        try:
            draw, _ = H.hamls_plan_radii(plan2)
        finally:
            H.hamls_plan_destroy(plan2)
        assert np.max(np.abs(np.diff(delta))) < np.max(np.abs(np.diff(draw)))
    finally:
        H.hamls_plan_destroy(plan)
