"""Captured fits (HIP graphs) on the GPU, through the C ABI.

Every replay of a captured step 2 + step 3 is compared with the eager calls on
the same inputs, with other eager work, new input values and synchronizations
between the replays: bit for bit (the same kernels in the same order; the
re-solve lists are filled by atomics in varying order, but each node's result
does not depend on its place in the list).  A rebind to another node count
makes the graph refuse to launch; a rebind to the same count keeps it valid."""
import sys

import numpy as np
import pytest

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


def _workload(domain):
    rng = np.random.default_rng(71)
    if domain == "s2":
        x = W.cluster_hole_s2(30000, rng, caps=W.random_caps(4, 15.0, 20.0, rng))
        wp = W.serving_params(32, 3)
    elif domain == "so3":
        x = W.clustered_rotations(30000, rng)
        wp = dict(domain="so3", bandwidth=8, degree=2, knn_count=40, knn_eps=0.05, reg="chi")
    else:
        x = W.clustered_torus(30000, rng)
        wp = dict(domain="t3", bandwidth=8, degree=3, knn_count=80, knn_eps=0.05, reg="chi",
                  grid_shape=(16, 16, 16))
    return x, wp


@pytest.mark.parametrize("domain,over", [("s2", {}), ("s2", dict(precision="mixed")), ("so3", {}), ("t3", {})])
def test_captured_fit_replays_equal_eager(H, domain, over):
    import torch

    x, wp = _workload(domain)
    p = H.params_from_workload(wp, **over)
    _say("graph", domain, over)
    s = torch.cuda.Stream()
    rng = np.random.default_rng(3)
    F = 3
    nodes = _dev(x)
    with torch.cuda.stream(s):
        plan = H.hamls_plan(p, nodes, stream=s)
        info = H.hamls_plan_info_get(plan)
        vals = _dev(rng.standard_normal((F, x.shape[0])))
        gv = torch.empty((F, info.num_grid), dtype=torch.float64, device="cuda")
        cf = torch.empty((F, info.num_coeffs, 2), dtype=torch.float64, device="cuda")
        gv_ref = torch.empty_like(gv)
        cf_ref = torch.empty_like(cf)
    s.synchronize()
    graph = H.hamls_fit_capture(plan, vals, gv, cf, s)
    try:
        for rep in range(4):
            # new values (in place), eager reference, other eager work, replay
            vals.copy_(_dev(rng.standard_normal((F, x.shape[0]))))
            torch.cuda.synchronize()
            H.hamls_mls_to_grid(plan, vals, gv_ref, stream=s)
            H.hamls_grid_to_coeffs(plan, gv_ref, cf_ref, stream=s)
            s.synchronize()
            junk = torch.randn(1 << 20, device="cuda", dtype=torch.float64).sum()
            torch.cuda.synchronize()
            gv.fill_(float("nan"))
            cf.fill_(float("nan"))
            torch.cuda.synchronize()
            H.hamls_graph_launch(graph, s)
            s.synchronize()
            assert torch.equal(gv, gv_ref) or bool(torch.all((gv == gv_ref) | (gv.isnan() & gv_ref.isnan())))
            assert torch.equal(cf, cf_ref), (rep, float((cf - cf_ref).abs().max()))
            _say("replay", rep, "ok", float(junk) != 0.0)
        # a rebind to the same node count keeps the graph valid ...
        perm = torch.as_tensor(rng.permutation(x.shape[0]), device="cuda")
        with torch.cuda.stream(s):
            H.hamls_plan_rebind(plan, nodes[perm].contiguous(), stream=s)
            H.hamls_mls_to_grid(plan, vals, gv_ref, stream=s)
            H.hamls_grid_to_coeffs(plan, gv_ref, cf_ref, stream=s)
        H.hamls_graph_launch(graph, s)
        s.synchronize()
        assert torch.equal(cf, cf_ref)
        # ... another count makes it refuse
        with torch.cuda.stream(s):
            H.hamls_plan_rebind(plan, nodes[: x.shape[0] - 1000].contiguous(), stream=s)
        s.synchronize()
        with pytest.raises(H.HamlsError):
            H.hamls_graph_launch(graph, s)
    finally:
        H.hamls_graph_destroy(graph)
        H.hamls_plan_destroy(plan)


def test_capture_refuses_the_default_stream(H):
    import torch

    x, wp = _workload("s2")
    p = H.params_from_workload(wp)
    plan = H.hamls_plan(p, _dev(x))
    try:
        info = H.hamls_plan_info_get(plan)
        vals = _dev(np.ones((1, x.shape[0])))
        gv = torch.empty((1, info.num_grid), dtype=torch.float64, device="cuda")
        cf = torch.empty((1, info.num_coeffs, 2), dtype=torch.float64, device="cuda")
        with pytest.raises(H.HamlsError):
            H.hamls_fit_capture(plan, vals, gv, cf, 0)
    finally:
        H.hamls_plan_destroy(plan)
