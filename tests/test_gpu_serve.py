"""Serving loop on the GPU, through the C ABI.

Each result of a request served in a mix (several workers, resident plans
rebound, admission under a byte budget) equals the plain one-request path on
the same inputs: bit for bit on a freshly built plan; within the FP64 bar of
1e-10 relative L2 on a rebound plan, which keeps the cell grid of its first
node set, so that its Gram sums run in another order (rounding differences of
~1e-16 amplified by local condition numbers up to ~1e4 before the
double-double re-solve takes over; ~2e-12 seen).  The footprint estimate
equals the bytes a plan holds; a request that cannot fit, or has invalid
parameters, completes with its error while the others proceed."""
import sys

import numpy as np
import pytest

from paper_2609_39200_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-10


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


def _alone(H, p, nodes, vals):
    import torch

    plan = H.hamls_plan(p, nodes)
    info = H.hamls_plan_info_get(plan)
    F = vals.shape[0]
    gv = torch.empty((F, info.num_grid), dtype=torch.float64, device="cuda")
    cf = torch.empty((F, info.num_coeffs, 2), dtype=torch.float64, device="cuda")
    H.hamls_mls_to_grid(plan, vals, gv)
    H.hamls_grid_to_coeffs(plan, gv, cf)
    torch.cuda.synchronize()
    H.hamls_plan_destroy(plan)
    return cf.cpu().numpy()


def _collect(H, srv, n, timeout=60.0):
    import time

    out = {}
    t_end = time.time() + timeout
    while len(out) < n:
        assert time.time() < t_end, f"only {len(out)} of {n} completions"
        for c in H.hamls_server_wait(srv, 64, 1.0):
            out[c["tag"]] = c
    return out


@pytest.mark.parametrize(
    "domain,over,F",
    [("s2", {}, 1), ("s2", dict(precision="mixed"), 3), ("s2", dict(smooth_aux=3000), 1), ("so3", {}, 2),
     ("t3", {}, 1)],
)
def test_footprint_equals_resident_bytes(H, domain, over, F):
    import torch

    rng = np.random.default_rng(11)
    if domain == "s2":
        x = W.cluster_hole_s2(20000, rng, caps=W.random_caps(3, 20.0, 20.0, rng))
        wp = W.serving_params(24, 3)
    elif domain == "so3":
        x = W.clustered_rotations(20000, rng)
        wp = dict(domain="so3", bandwidth=8, degree=2, knn_count=40, knn_eps=0.05, reg="chi")
    else:
        x = W.clustered_torus(20000, rng)
        wp = dict(domain="t3", bandwidth=8, degree=2, knn_count=40, knn_eps=0.05, reg="chi",
                  grid_shape=(16, 16, 16))
    p = H.params_from_workload(wp, **over)
    _say("footprint", domain, over, F)
    nodes = _dev(x)
    vals = _dev(rng.standard_normal((F, x.shape[0])))
    plan = H.hamls_plan(p, nodes)
    info = H.hamls_plan_info_get(plan)
    gv = torch.empty((F, info.num_grid), dtype=torch.float64, device="cuda")
    cf = torch.empty((F, info.num_coeffs, 2), dtype=torch.float64, device="cuda")
    H.hamls_mls_to_grid(plan, vals, gv)
    H.hamls_grid_to_coeffs(plan, gv, cf)
    torch.cuda.synchronize()
    got = H.hamls_plan_info_get(plan).resident_bytes
    H.hamls_plan_destroy(plan)
    assert got == H.hamls_plan_footprint(p, x.shape[0], F)


def _requests(n_pools=2):
    """Eight small S2 requests: repeated (N, K) pairs so that plans are rebound,
    M from 3000 to 30000, F in {1, 2}."""
    rng = np.random.default_rng(21)
    pools = []
    for k in range(n_pools):
        prng = np.random.default_rng(100 + k)
        x = W.cluster_hole_s2(30000, prng, caps=W.random_caps(4, 15.0, 20.0, prng))
        pools.append(x[prng.permutation(x.shape[0])])
    spec = [(16, 2, 5000, 1), (24, 3, 12000, 2), (16, 2, 4000, 1), (32, 4, 30000, 1),
            (24, 3, 9000, 1), (16, 2, 3000, 2), (32, 4, 20000, 1), (24, 2, 15000, 1)]
    out = []
    for i, (N, K, M, F) in enumerate(spec):
        x = pools[i % n_pools][:M]
        out.append(dict(N=N, K=K, x=x, v=rng.standard_normal((F, M))))
    return out


def test_results_in_the_mix_equal_the_results_alone(H):
    import torch

    reqs = _requests()
    srv = H.hamls_server_create(3, 0)
    try:
        live = []
        for i, r in enumerate(reqs):
            p = H.params_from_workload(W.serving_params(r["N"], r["K"]))
            nodes, vals = _dev(r["x"]), _dev(r["v"])
            ncoef = (r["N"] + 1) ** 2
            cf = torch.full((r["v"].shape[0], ncoef, 2), float("nan"), dtype=torch.float64, device="cuda")
            torch.cuda.synchronize()
            H.hamls_server_submit(srv, p, nodes, vals, cf, tag=i)
            live.append((p, nodes, vals, cf))
        _say("submitted", len(reqs))
        done = _collect(H, srv, len(reqs))
    finally:
        H.hamls_server_destroy(srv)
    assert all(c["status"] == 0 for c in done.values()), done
    assert sum(c["plan_reused"] for c in done.values()) >= 1
    for i, (p, nodes, vals, cf) in enumerate(live):
        c = done[i]
        assert c["t_submit"] <= c["t_admit"] <= c["t_done"]
        ref = _alone(H, p, nodes, vals)
        err = _rell2(cf.cpu().numpy(), ref)
        _say("request", i, "reused", c["plan_reused"], "rel l2", err)
        assert err <= (TOL if c["plan_reused"] else 0.0), (i, err)


def test_admission_budget_and_errors(H):
    import time

    import torch

    reqs = _requests()
    fps = [H.hamls_plan_footprint(H.params_from_workload(W.serving_params(r["N"], r["K"])),
                                  16384 if r["x"].shape[0] <= 16384 else 32768, r["v"].shape[0])
           for r in reqs]
    # room for about one plan at a time (plus grid values)
    budget = int(1.3 * max(fps))
    srv = H.hamls_server_create(4, budget)
    live = []
    try:
        for i, r in enumerate(reqs):
            p = H.params_from_workload(W.serving_params(r["N"], r["K"]))
            nodes, vals = _dev(r["x"]), _dev(r["v"])
            cf = torch.empty((r["v"].shape[0], (r["N"] + 1) ** 2, 2), dtype=torch.float64, device="cuda")
            live.append((p, nodes, vals, cf))
        # an invalid request (degree outside [0, 4]) between valid ones, and one
        # whose footprint alone exceeds the budget
        bad = H.params_from_workload(W.serving_params(16, 2))
        bad.degree = 7
        big = H.params_from_workload(W.serving_params(256, 4))
        bnodes, bvals = live[0][1], live[0][2]
        bcf = torch.empty((1, 257 * 257, 2), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        for i, (p, nodes, vals, cf) in enumerate(live):
            H.hamls_server_submit(srv, p, nodes, vals, cf, tag=i)
            if i == 2:
                H.hamls_server_submit(srv, bad, bnodes, bvals, bcf, tag=100)
            if i == 4:
                H.hamls_server_submit(srv, big, bnodes, bvals, bcf, tag=101)
        peak = 0
        t_end = time.time() + 60
        done = {}
        while len(done) < len(live) + 2:
            assert time.time() < t_end
            _, committed, _ = H.hamls_server_load(srv)
            peak = max(peak, committed)
            for c in H.hamls_server_wait(srv, 64, 0.05):
                done[c["tag"]] = c
    finally:
        H.hamls_server_destroy(srv)
    _say("budget", budget, "peak committed", peak)
    assert peak <= budget
    assert done[100]["status"] == -1
    assert done[101]["status"] == -3
    for i, (p, nodes, vals, cf) in enumerate(live):
        assert done[i]["status"] == 0, (i, done[i])
        err = _rell2(cf.cpu().numpy(), _alone(H, p, nodes, vals))
        assert err <= (TOL if done[i]["plan_reused"] else 0.0), (i, err)


def test_smoothed_and_plain_requests_do_not_share_plans(H):
    """Requests equal in every parameter but the smoothed radius (Sec. 2.2,
    after eq. (12)) must not rebind each other's resident plan: each result
    equals its own request run alone."""
    import torch

    prng = np.random.default_rng(140)
    x = W.cluster_hole_s2(20000, prng, caps=W.random_caps(3, 15.0, 20.0, prng))
    v = prng.standard_normal((1, 20000))
    base = W.serving_params(24, 3)
    srv = H.hamls_server_create(1, 0)  # one worker: strictly sequential, plans stay resident
    live = []
    try:
        for i, aux in enumerate([0, 4000, 0, 4000]):
            p = H.params_from_workload(base, smooth_aux=aux)
            # decreasing M: every later request fits a resident plan's capacity
            nodes, vals = _dev(x[: 15000 - 1000 * i]), _dev(v[:, : 15000 - 1000 * i])
            cf = torch.full((1, 25 * 25, 2), float("nan"), dtype=torch.float64, device="cuda")
            torch.cuda.synchronize()
            H.hamls_server_submit(srv, p, nodes, vals, cf, tag=i)
            live.append((p, nodes, vals, cf))
        done = _collect(H, srv, len(live))
    finally:
        H.hamls_server_destroy(srv)
    assert all(c["status"] == 0 for c in done.values()), done
    # the third and fourth reuse the plans of the first and second
    assert [int(done[i]["plan_reused"]) for i in range(4)] == [0, 0, 1, 1]
    for i, (p, nodes, vals, cf) in enumerate(live):
        err = _rell2(cf.cpu().numpy(), _alone(H, p, nodes, vals))
        _say("smooth_aux", p.smooth_aux, "reused", done[i]["plan_reused"], "rel l2", err)
        assert err <= TOL


def test_served_results_match_the_oracle(H):
    """A sample of served results against the FP64 CPU oracle (steps 2 and 3
    on the library's grid), on small requests of several N and K."""
    import torch

    import oracle

    reqs = _requests()
    sel = [0, 2, 5]  # N = 16, K = 2, M <= 5000
    srv = H.hamls_server_create(2, 0)
    live = []
    try:
        for i, r in enumerate(reqs):
            p = H.params_from_workload(W.serving_params(r["N"], r["K"]))
            nodes, vals = _dev(r["x"]), _dev(r["v"])
            cf = torch.full((r["v"].shape[0], (r["N"] + 1) ** 2, 2), float("nan"), dtype=torch.float64,
                            device="cuda")
            torch.cuda.synchronize()
            H.hamls_server_submit(srv, p, nodes, vals, cf, tag=i)
            live.append((nodes, vals, cf))  # inputs stay valid until completion
        done = _collect(H, srv, len(reqs))
    finally:
        H.hamls_server_destroy(srv)
    for i in sel:
        assert done[i]["status"] == 0
        r = reqs[i]
        wp = W.serving_params(r["N"], r["K"])
        po = oracle.params(**wp)
        plan = H.hamls_plan(H.params_from_workload(wp), _dev(r["x"]))
        gpts, _ = H.hamls_plan_grid(plan)
        H.hamls_plan_destroy(plan)
        om = oracle.mls(po, gpts, r["x"], r["v"])
        oc = oracle.coeffs(po, om["values"])
        c = live[i][2].cpu().numpy()
        err = _rell2(c[..., 0] + 1j * c[..., 1], oc)
        _say("served request", i, "vs oracle rel l2", err)
        assert err < TOL


def test_backfilling_passes_a_blocked_request(H):
    """Under a budget with room for one large plan, a large request that waits
    for a running one to finish is passed by a small request that fits, and
    every result equals its request alone."""
    import torch

    prng = np.random.default_rng(150)
    x = W.cluster_hole_s2(30000, prng, caps=W.random_caps(3, 15.0, 20.0, prng))
    small = (16, 2, 3000)
    large = (64, 4, 30000)
    fp_large = H.hamls_plan_footprint(H.params_from_workload(W.serving_params(64, 4)), 32768, 1)
    fp_small = H.hamls_plan_footprint(H.params_from_workload(W.serving_params(16, 2)), 16384, 1)
    budget = int(1.5 * fp_large)
    assert fp_small < budget - fp_large
    live = []
    for N, K, M in [large, large, small]:
        p = H.params_from_workload(W.serving_params(N, K))
        vals = _dev(prng.standard_normal((1, M)))
        nodes = _dev(x[:M])
        cf = torch.full((1, (N + 1) ** 2, 2), float("nan"), dtype=torch.float64, device="cuda")
        live.append((p, nodes, vals, cf))
    torch.cuda.synchronize()
    srv = H.hamls_server_create(2, budget)
    try:
        # back to back: the small request arrives while the first large one
        # runs and the second waits for its memory
        for i, (p, nodes, vals, cf) in enumerate(live):
            H.hamls_server_submit(srv, p, nodes, vals, cf, tag=i)
        done = _collect(H, srv, len(live))
    finally:
        H.hamls_server_destroy(srv)
    assert all(c["status"] == 0 for c in done.values()), done
    _say("admit times", [round(done[i]["t_admit"] - done[0]["t_admit"], 4) for i in range(3)])
    # the small request was admitted before the second large one
    assert done[2]["t_admit"] < done[1]["t_admit"]
    for i, (p, nodes, vals, cf) in enumerate(live):
        err = _rell2(cf.cpu().numpy(), _alone(H, p, nodes, vals))
        assert err <= (TOL if done[i]["plan_reused"] else 0.0), (i, err)
