"""hamls_grid_to_coeffs_noalloc (step 3 on the library's static device work
array) against hamls_grid_to_coeffs, through the C ABI: the same kernels, so
the coefficients must agree bit for bit, on two calls in a row (the second
with fewer fields and on a smaller plan); no device memory is allocated; a
call whose work memory exceeds the array is refused with a clear error."""
import numpy as np
import pytest

from paper_2609_39200_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def H():
    import torch

    from paper_2609_39200_amd import hamls

    # the static work array is device memory of the library's code object,
    # placed when that object is first loaded on the device: one small call
    # before any free-memory comparison
    wl = W.s2_clusters(seed=9100, M=3000, N=8, K=1, field_degree=4)
    plan = _plan(hamls, wl)
    try:
        info = hamls.hamls_plan_info_get(plan)
        g = torch.zeros((1, info.num_grid), dtype=torch.float64, device="cuda")
        c = torch.zeros((1, info.num_coeffs, 2), dtype=torch.float64, device="cuda")
        hamls.hamls_grid_to_coeffs_noalloc(plan, g, c)
        torch.cuda.synchronize()
    finally:
        hamls.hamls_plan_destroy(plan)
    return hamls


def _plan(H, wl, **over):
    import torch

    p = H.params_from_workload(wl.params, **over)
    nodes = torch.as_tensor(wl.nodes, dtype=torch.float64, device="cuda")
    return H.hamls_plan(p, nodes)


def _both(H, plan, F, seed):
    """Coefficients of F random grid fields by both entry points; the no-alloc
    call runs first, on a plan whose own step-3 work memory is smaller than F
    needs, so the plain call after it has to allocate."""
    import torch

    info = H.hamls_plan_info_get(plan)
    g = torch.as_tensor(np.random.default_rng(seed).standard_normal((F, info.num_grid)), device="cuda")
    a = torch.full((F, info.num_coeffs, 2), float("nan"), dtype=torch.float64, device="cuda")
    b = torch.full_like(a, float("nan"))
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    res0 = H.hamls_plan_info_get(plan).resident_bytes
    H.hamls_grid_to_coeffs_noalloc(plan, g, a)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    res1 = H.hamls_plan_info_get(plan).resident_bytes
    H.hamls_grid_to_coeffs(plan, g, b)
    torch.cuda.synchronize()
    assert free1 == free0, (free0, free1)
    assert res1 == res0
    return a.cpu().numpy(), b.cpu().numpy()


CASES = [
    ("s2-fp64", lambda: W.s2_clusters(seed=9101, M=20000, N=48, K=2, field_degree=20), {}, (9, 2),
     lambda: W.s2_clusters(seed=9102, M=6000, N=20, K=2, field_degree=10)),
    ("s2-mixed", lambda: W.s2_clusters(seed=9103, M=20000, N=48, K=2, field_degree=20), {"precision": "mixed"},
     (21, 3), lambda: W.s2_clusters(seed=9104, M=6000, N=20, K=2, field_degree=10)),
    ("so3", lambda: W.so3_clusters(seed=9105, M=20000, N=10, K=1, grid=(0, 0, 0), field_degree=6), {}, (5, 1),
     lambda: W.so3_clusters(seed=9106, M=8000, N=6, K=1, grid=(0, 0, 0), field_degree=4)),
    ("t3", lambda: W.t3_clusters(seed=9107, M=20000, N=12, K=1, grid=24, kmax=8), {}, (4, 1),
     lambda: W.t3_clusters(seed=9108, M=8000, N=6, K=1, grid=12, kmax=4)),
]


@pytest.mark.parametrize("name,make,over,fields,make_small", CASES, ids=[c[0] for c in CASES])
def test_noalloc_equals_plan_work_memory(H, name, make, over, fields, make_small):
    F1, F2 = fields
    _say(f"[gpu] no-alloc step 3: {name}, F = {F1} then {F2} on a smaller plan")
    plan = _plan(H, make(), **over)
    small = _plan(H, make_small(), **over)
    try:
        a, b = _both(H, plan, F1, 1)
        assert np.isfinite(a).all()
        assert np.array_equal(a, b)
        a2, b2 = _both(H, small, F2, 2)
        assert np.isfinite(a2).all()
        assert np.array_equal(a2, b2)
    finally:
        H.hamls_plan_destroy(plan)
        H.hamls_plan_destroy(small)


def test_noalloc_refuses_work_beyond_the_array(H):
    import torch

    wl = W.t3_clusters(seed=9110, M=20000, N=32, K=1, grid=64, kmax=8)
    plan = _plan(H, wl)
    try:
        info = H.hamls_plan_info_get(plan)
        # T3 64^3: two complex work buffers of 4 MiB per field each
        F = H.hamls_noalloc_scratch_bytes() // (2 * 16 * info.num_grid) + 1
        g = torch.zeros((F, info.num_grid), dtype=torch.float64, device="cuda")
        c = torch.zeros((F, info.num_coeffs, 2), dtype=torch.float64, device="cuda")
        with pytest.raises(H.HamlsError) as e:
            H.hamls_grid_to_coeffs_noalloc(plan, g, c)
        assert e.value.code == -1  # INVALID_ARG
        assert "static work array" in str(e.value)
        # one field fewer fits
        H.hamls_grid_to_coeffs_noalloc(plan, g[: F - 1], c[: F - 1])
        torch.cuda.synchronize()
    finally:
        H.hamls_plan_destroy(plan)
