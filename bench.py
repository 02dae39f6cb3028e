#!/usr/bin/env python
"""Benchmark of the HAMLS hot path on one MI355X.

Default workload (--workload c2): S2 ill-distributed nodes, M = 200,000 (8
von Mises-Fisher clusters with kappa = 20 plus 20 % uniform, five 20-degree
caps removed), bandwidth N = 128, MLS degree K = 3 (m = 10), Gauss-Legendre
grid 129 x 258 (33,282 local solves), adaptive radius with n = 40, eps = 0.05,
chi-target regularization (chi_T = 10, chi_full = 20), one field, FP64.
Other workloads: c3 (S2, M = 4e6, N = 512, K = 4, grid 513 x 1026, n = 60),
so3 (M = 1e6 rotations, N = 64, K = 2, Euler grid 130^3, n = 40), t3 (M = 2e6
points, N = 64, K = 3, grid 128^3, n = 80).

One step = one whole fit with the inputs resident in device memory:
node binning + sort + support radii (plan rebind), the MLS value at every grid
node (Gram assembly + regularized solve), the quadrature (ring DFTs + Legendre
contraction on S2; axis DFTs + Wigner contraction on SO(3); 3-D DFT on T3).
value = grid nodes solved per second = M_Q * F * steps / wall time of the
timed steps.  Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_VALU_TFLOPS = 78.6  # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
PEAK_FP32_VALU_TFLOPS = 157.3  # published FP32 vector peak (packed)
PEAK_HBM_GBS = 8000.0


def pct(a, q):
    return float(np.percentile(np.asarray(a), q))


# kernel (name prefix) of each phase's main launch, for the counter summary
PHASE_KERNEL = {"binning": None, "radius": "k_s2_radius", "assemble": "k_s2_assemble<",
                "solve": "k_mls_solve<", "ring_dft": "k_s2_ring_dft", "contract": "k_s2_legendre",
                "gather": "k_gather_values"}

WORKLOADS = {
    "c2smooth": ("s2_clusters_smooth", "S2 ill-distributed (C2 nodes, M=200000), N=128, K=3, grid 129x258, smoothed "
                 "adaptive radius: d_n (n=40) on 65536 Fibonacci points, degree-zero MLS at the grid, eps=0.05, "
                 "chi_T=10 chi_full=20, F=1, FP64"),
    "c2fixed": ("s2_clusters_fixed", "S2 ill-distributed under a fixed radius (skewed neighbour counts 0-2400, "
                "median 196), M=200000 (C2 nodes), N=128, K=3, grid 129x258, delta0=0.1 rad, chi_T=10 "
                "chi_full=20, F=1, FP64"),
    "c2": ("s2_clusters", "S2 ill-distributed, M=200000 (8 vMF clusters kappa=20 + 20% uniform, 5 caps of 20 deg "
                          "removed), N=128, K=3, grid 129x258, kNN n=40 eps=0.05, chi_T=10 chi_full=20, F=1, FP64"),
    "c3": ("s2_large", "S2 ill-distributed, M=4000000 (8 vMF clusters kappa=20 + 20% uniform, 12 caps of 10-25 deg "
                       "removed), N=512, K=4, grid 513x1026, kNN n=60 eps=0.05, chi_T=10 chi_full=20, F=1, FP64"),
    "so3": ("so3_clusters", "SO(3), M=1000000 rotations (50% Haar + 4 clusters sigma=0.15), N=64, K=2, Euler grid "
                            "130^3, kNN n=40 eps=0.05, chi_T=10 chi_full=20, F=1, FP64"),
    "t3": ("t3_clusters", "T3, M=2000000 (8 periodic Gaussian clusters sigma=0.05 + 20% uniform, 6 balls removed), "
                          "N=64, K=3, grid 128^3, kNN n=80 eps=0.05, chi_T=10 chi_full=20, F=1, FP64"),
}


def source_sha256():
    import glob
    import hashlib

    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2609_39200_amd", "csrc")
    for f in sorted(glob.glob(os.path.join(csrc, "*.hip")) + glob.glob(os.path.join(csrc, "*.h"))):
        h.update(open(f, "rb").read())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of the kernel whose name starts with `kernel` (the
    FP64 variant) from the committed rocprofv3 counter summary (FETCH_SIZE and
    WRITE_SIZE scaled by the copy calibration), or None when the HIP sources
    changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "s2_c2_hbm_traffic.txt")
    if kernel is None or not os.path.exists(path):
        return None
    info = {}
    kern = {}
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        if line.startswith("kernel "):
            name, rest = line[7:].split(" fetch_kib ")
            f = ("fetch_kib " + rest).split()
            kern[name] = dict(zip(f[0::2], f[1::2]))
        else:
            f = line.split()
            info[f[0]] = f[1]
    if info.get("source_sha256") != source_sha256():
        return None
    for name, k in kern.items():
        # the FP64 pass, not the double-double re-solve (third template argument)
        targs = name[name.index("<") + 1:].rstrip(">").split(", ") if "<" in name else []
        if name.startswith(kernel) and not (len(targs) > 2 and targs[2] == "true"):
            return float(k["bytes"])
    return None


def flops_per_pair(domain, m, F):
    """Algorithmic FLOPs of one (grid node, neighbour) pair in the MLS step:
    membership key (S2 dot 5, SO3 dot 7, T3 min-image distance 12), tangent
    coordinates (S2 12, SO3 24, T3 3), weight 10 (distance, Wendland, node
    weight, square root), monomials and weighting 2m, Gram m(m+1), right-hand
    sides 2mF."""
    key = {"s2": 5, "so3": 7, "t3": 12}[domain]
    crd = {"s2": 12, "so3": 24, "t3": 3}[domain]
    return key + crd + 10 + 2 * m + m * (m + 1) + 2 * m * F


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS) + ["serve"],
                    help="serve: the request loop (continuous batching) on the serving trace")
    ap.add_argument("--requests", type=int, default=512, help="serve: number of requests")
    ap.add_argument("--rate", type=float, default=200.0, help="serve: Poisson arrival rate (1/s)")
    ap.add_argument("--slots", type=int, default=4, help="serve: worker streams of the server")
    ap.add_argument("--fields", type=int, default=1,
                    help="fields per fit: the workload's field plus seeded N(0,1) node values")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="budget of the CPU oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the run, copy a 256 MiB buffer three times (known-size traffic for "
                         "scaling the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; a multi-GPU path is "
                          "not built"}), flush=True)
        sys.exit(2)

    import torch

    from paper_2609_39200_amd import hamls as H
    from paper_2609_39200_amd import workloads as W

    if args.workload == "serve":
        print(json.dumps(serve_bench(args, H, W, torch)), flush=True)
        return

    t_gen = time.time()
    builder, wl_desc = WORKLOADS[args.workload]
    if args.fields > 1:
        wl_desc = wl_desc.replace(", F=1,", f", F={args.fields} (the field + N(0,1) node values),")
    if args.precision == "mixed":
        wl_desc = wl_desc.replace(", FP64", ", mixed (FP32 Gram + FP64 refinement/fallback, FP32 MFMA contraction)")
    wl = getattr(W, builder)()
    domain = wl.domain
    if args.fields > 1:
        extra = np.random.default_rng(77).standard_normal((args.fields - 1, wl.nodes.shape[0]))
        wl.values = np.concatenate([wl.values, extra], axis=0)
    F = wl.values.shape[0]
    dev = torch.device("cuda:0")
    nodes = torch.as_tensor(wl.nodes, dtype=torch.float64, device=dev).contiguous()
    vals = torch.as_tensor(wl.values, dtype=torch.float64, device=dev).contiguous()
    p = H.params_from_workload(wl.params, precision=args.precision)
    stream = torch.cuda.current_stream()
    plan = H.hamls_plan(p, nodes, stream=stream)
    info = H.hamls_plan_info_get(plan)
    MQ = info.num_grid
    gv = torch.empty((F, MQ), dtype=torch.float64, device=dev)
    cf = torch.empty((F, info.num_coeffs, 2), dtype=torch.float64, device=dev)
    gen_s = time.time() - t_gen

    # launch form of the assembly pass (grid order, cost order, S2 FP64 work
    # queue), measured on these nodes and kept by the plan
    tune = None
    q, t = H.hamls_plan_tune(plan, stream=stream)
    tune = {"form": q, "grid_order_ms": t[0], "cost_order_dispatch_ms": t[1]}
    if domain == "s2" and args.precision == "fp64":
        tune["queue_ms"] = {"8/CU": t[2], "12/CU": t[3]}

    def step():
        H.hamls_plan_rebind(plan, nodes, stream=stream)
        H.hamls_mls_to_grid(plan, vals, gv, stream=stream)
        H.hamls_grid_to_coeffs(plan, gv, cf, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    for ph in H.PHASES:
        H.hamls_timing_read(plan, ph)  # clear

    # census (outside the timed region): every phase timed, per-fit latency;
    # each event pair costs a few microseconds of GPU time
    K = args.steps
    nc = max(3, min(10, K))
    H.hamls_timing_phases(plan, None)
    H.hamls_timing_enable(plan, True)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(nc)]
    for i in range(nc):
        ev[i][0].record(stream)
        step()
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    lat = [a.elapsed_time(b) for a, b in ev]
    phases = {}
    for ph in H.PHASES:
        n, ms = H.hamls_timing_read(plan, ph)
        if n:
            phases[ph] = {"launches": n, "avg_ms": ms / n}
    dom = max(phases, key=lambda k: phases[k]["avg_ms"])

    # timed region: K fits, only the dominant phase timed (its launches give
    # the roofline's duration)
    H.hamls_timing_phases(plan, [dom])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(K):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    H.hamls_timing_enable(plan, False)
    H.hamls_timing_phases(plan, None)
    wall = t1 - t0
    n, ms = H.hamls_timing_read(plan, dom)
    phases[dom] = {"launches": n, "avg_ms": ms / n}

    diag = H.hamls_diagnostics(plan)
    pairs = int(diag["n"].astype(np.int64).sum())
    n_reg = int(np.sum(diag["status"] & H.ST_REGULARIZED != 0))
    n_ill = int(np.sum(diag["status"] & H.ST_ILLCOND != 0))

    # roofline of the dominant phase
    m = info.m
    roof = None
    traffic = (measured_traffic(PHASE_KERNEL.get(dom))
               if args.workload == "c2" and args.precision == "fp64" and F == 1 else None)
    if dom == "assemble":
        fpp = flops_per_pair(domain, m, F)
        fl = pairs * fpp
        ach = fl / (phases[dom]["avg_ms"] * 1e-3) / 1e12
        # the mixed pass is priced against the FP32 vector peak
        peak = PEAK_FP64_VALU_TFLOPS if args.precision == "fp64" else PEAK_FP32_VALU_TFLOPS
        roof = {"kernel": "assemble", "bound": "alu", "achieved": ach, "peak": peak,
                "unit": "TFLOP/s", "frac": ach / peak, "traffic": traffic,
                "units_per_launch": {"pairs": pairs, "flop_per_pair": fpp}}
    else:
        # other phases are priced on their algorithmic HBM bytes
        Mn = info.num_nodes
        nt, npf = info.grid_dims[0], info.grid_dims[1]
        N = info.bandwidth
        dimx = 4 if domain == "so3" else 3
        nrec = 2 * Mn if domain == "so3" else Mn
        rec = 8 * dimx
        bytes_by_phase = {
            # keys: read coordinates + write key and index; per radix pass
            # 16 B (key + index, read + write); cell table; gather: index and
            # coordinates read, coordinates and permutation written
            "binning": Mn * 8 * dimx + nrec * (8 + 2 * 16 + 8 + 2 * (4 + rec)),
            # every member record read once; radius, threshold, status, list
            # length and the member lists written
            "radius": pairs * (rec + 4) + MQ * 21,
            "solve": MQ * (8 * (m * (m + 1) // 2 + m * F) + 4 + 8 * F + 17),
            "gather": nrec * (4 + 16 * F),
        }
        if domain == "s2":
            bytes_by_phase["ring_dft"] = MQ * 8 * F + nt * (N + 1) * 16 * F
            bytes_by_phase["contract"] = (((nt + 1) // 2) * ((N + 1) * (N + 2) // 2) * 8
                                          + (N + 1) ** 2 * 16 * F)
        elif domain == "so3":
            K2 = 2 * N + 1
            nb, na, ng = info.grid_dims[0], info.grid_dims[1], info.grid_dims[2]
            # alpha pass: real grid in, (k, gamma) spectra out; gamma pass
            bytes_by_phase["ring_dft"] = F * nb * (na * ng * 8 + 2 * K2 * ng * 16 + K2 * K2 * 16)
            bytes_by_phase["contract"] = nb * info.num_coeffs * 8 + F * (nb * K2 * K2 + info.num_coeffs) * 16
        else:
            # three axis passes: real in / complex out, then complex in / out twice
            bytes_by_phase["ring_dft"] = F * MQ * (8 + 16 + 4 * 16)
        b = bytes_by_phase.get(dom, 0)
        ach = b / (phases[dom]["avg_ms"] * 1e-3) / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": ach / PEAK_HBM_GBS, "traffic": traffic, "units_per_launch": {"bytes": b}}

    out = {
        "metric": "MLS grid nodes solved/s (whole fit: binning + radii + local solves + quadrature)",
        "value": MQ * F * K / wall,
        "unit": "grid nodes/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": wl_desc,
            "grid_nodes": MQ,
            "nodes": int(info.num_nodes),
            "fields": F,
            "precision": args.precision,
        },
        "fits_per_s": K / wall,
        "latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99), "min": float(min(lat))},
        "phases_ms": {k: v["avg_ms"] for k, v in phases.items()},
        "timing": f"value and ms_per_step: wall clock over the {K} timed fits, during which only the "
                  f"dominant phase ({dom}) records HIP events; the other phases and the latency "
                  f"percentiles come from {nc} fits outside the timed region with every phase timed",
        "stats": {"pairs": pairs, "mean_neighbours": pairs / MQ, "regularized": n_reg, "illcond": n_ill},
        "roofline": roof,
    }
    if tune is not None:
        out["assembly_launch"] = tune

    out["captured_fit"] = graph_bench(H, torch, plan, info, vals, K)
    out["generating_functions"] = gen_bench(H, torch, plan, info, vals, gv, stream, K, 1e3 * wall / K)

    if not args.no_cpu_baseline:
        out["cpu_baseline"], out["accuracy"] = cpu_baseline(wl, plan, gv, H, args.cpu_seconds)
    H.hamls_plan_destroy(plan)
    if args.copy_calibration:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = src.numel() * 8
    print(json.dumps(out), flush=True)


def graph_bench(H, torch, plan, info, vals, K):
    """Steps 2 + 3 on the bound nodes (no rebind), K times eagerly and K times
    as replays of one captured graph, on a side stream (capture needs a
    stream other than the default one)."""
    s = torch.cuda.Stream()
    F = vals.shape[0]
    gv = torch.empty((F, info.num_grid), dtype=torch.float64, device=vals.device)
    cf = torch.empty((F, info.num_coeffs, 2), dtype=torch.float64, device=vals.device)
    torch.cuda.synchronize()
    g = H.hamls_fit_capture(plan, vals, gv, cf, s)
    try:
        def eager():
            H.hamls_mls_to_grid(plan, vals, gv, stream=s)
            H.hamls_grid_to_coeffs(plan, gv, cf, stream=s)

        def replay():
            H.hamls_graph_launch(g, s)

        res = {}
        for name, fn in (("eager", eager), ("graph", replay)):
            fn()
            s.synchronize()
            t0 = time.perf_counter()
            for _ in range(K):
                fn()
            s.synchronize()
            res[f"{name}_ms"] = 1e3 * (time.perf_counter() - t0) / K
    finally:
        H.hamls_graph_destroy(g)
    res["note"] = "steps 2 + 3 only (no rebind), wall clock per fit"
    return res


def gen_bench(H, torch, plan, info, vals, gv, stream, K, fit_ms):
    """Generating functions (Rem. 2.5) on the same plan: one build, then K
    fits through the sparse product (value gather + product), timed like the
    main loop; the product kernel's events give its roofline (HBM: every
    entry's 12 bytes, the row pointers, the grid values written, the node
    values read once)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    H.hamls_gen_build(plan, stream=stream)
    torch.cuda.synchronize()
    build_ms = 1e3 * (time.perf_counter() - t0)
    ref = gv.clone()
    H.hamls_mls_to_grid(plan, vals, ref, stream=stream)
    H.hamls_gen_apply(plan, vals, gv, stream=stream)
    torch.cuda.synchronize()
    ok = torch.isfinite(ref)  # empty supports (holes under a fixed radius) are NaN in both
    same_nan = bool(torch.equal(torch.isnan(gv), torch.isnan(ref)))
    err = float(torch.linalg.norm(gv[ok] - ref[ok]) / torch.linalg.norm(ref[ok])) if same_nan else float("inf")
    rp, _, _ = H.hamls_gen_get(plan)
    nnz = int(rp[-1])
    H.hamls_timing_phases(plan, ["gen_apply"])
    H.hamls_timing_enable(plan, True)
    H.hamls_timing_read(plan, "gen_apply")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        H.hamls_gen_apply(plan, vals, gv, stream=stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    n, ms = H.hamls_timing_read(plan, "gen_apply")
    H.hamls_timing_enable(plan, False)
    H.hamls_timing_phases(plan, None)
    gv.copy_(ref)  # the main path's grid values for what follows
    F = vals.shape[0]
    MQ = info.num_grid
    nbytes = nnz * 12 + (MQ + 1) * 8 + MQ * 8 * F + int(info.num_nodes) * 8 * F
    kms = ms / n
    ach = nbytes / (kms * 1e-3) / 1e9
    return {"build_ms": build_ms, "nnz": nnz, "ms_per_fit": 1e3 * wall / K,
            "speedup_vs_full_fit": fit_ms / (1e3 * wall / K), "rel_l2_vs_fit": err,
            "apply_kernel": {"kernel": "k_gen_apply", "avg_ms": kms, "bytes": nbytes, "achieved": ach,
                             "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": ach / PEAK_HBM_GBS}}


def serve_bench(args, H, W, torch):
    """The serving trace through the request loop, then through the plain
    one-request-at-a-time FP64 path (plan, step 2, step 3, destroy per
    request) with the same arrivals.  Latency = completion - arrival."""
    import threading

    tr = W.serving_trace(n=args.requests, rate=args.rate)
    n = len(tr.arrival)
    dev = torch.device("cuda:0")
    pools = [torch.as_tensor(x, dtype=torch.float64, device=dev).contiguous() for x in tr.pools]
    fields = [torch.as_tensor(f, dtype=torch.float64, device=dev).contiguous() for f in tr.fields]
    reqs = []
    for i in range(n):
        M, k = int(tr.M[i]), int(tr.pool[i])
        p = H.params_from_workload(W.serving_params(tr.N[i], tr.K[i]))
        cf = torch.empty((1, (int(tr.N[i]) + 1) ** 2, 2), dtype=torch.float64, device=dev)
        reqs.append((p, pools[k][:M], fields[k][:M].view(1, M), cf))
    torch.cuda.synchronize()

    def summarize(lat, t_first, t_last):
        lat = sorted(lat)
        return {"fits_per_s": n / (t_last - t_first), "p50_ms": 1e3 * pct(lat, 50),
                "p99_ms": 1e3 * pct(lat, 99), "makespan_s": t_last - t_first}

    def serve(arrival):
        """The request loop, starting with no resident plan."""
        srv = H.hamls_server_create(args.slots, 0)
        t0 = H.hamls_server_clock() + 0.05

        def submitter():
            for i, (p, x, v, cf) in enumerate(reqs):
                dt = t0 + arrival[i] - H.hamls_server_clock()
                if dt > 0:
                    time.sleep(dt)
                H.hamls_server_submit(srv, p, x, v, cf, tag=i)

        th = threading.Thread(target=submitter)
        th.start()
        done = {}
        while len(done) < n:
            for c in H.hamls_server_wait(srv, 256, 1.0):
                done[c["tag"]] = c
        th.join()
        _, committed, nplans = H.hamls_server_load(srv)
        H.hamls_server_destroy(srv)
        lat = [done[i]["t_done"] - (t0 + arrival[i]) for i in range(n)]
        out = summarize(lat, t0, max(c["t_done"] for c in done.values()))
        out["plans_reused"] = sum(c["plan_reused"] for c in done.values())
        out["resident_plans_at_end"] = nplans
        out["resident_bytes_at_end"] = committed
        out["failed"] = sum(c["status"] != 0 for c in done.values())
        return out

    # all requests at once: the loop's capacity
    burst = serve(np.zeros(n))
    print(f"burst of {n} requests: {burst}", file=sys.stderr, flush=True)
    # the trace's arrivals
    served = serve(tr.arrival)
    print(f"served {n} requests: {served}", file=sys.stderr, flush=True)
    served_cf = [r[3].clone() for r in reqs]

    # the plain path, one request at a time, same arrivals
    stream = torch.cuda.current_stream()
    t0 = H.hamls_server_clock()
    lat = []
    max_err = 0.0
    for i, (p, x, v, cf) in enumerate(reqs):
        dt = t0 + tr.arrival[i] - H.hamls_server_clock()
        if dt > 0:
            time.sleep(dt)
        plan = H.hamls_plan(p, x, stream=stream)
        info = H.hamls_plan_info_get(plan)
        gv = torch.empty((1, info.num_grid), dtype=torch.float64, device=dev)
        H.hamls_mls_to_grid(plan, v, gv, stream=stream)
        H.hamls_grid_to_coeffs(plan, gv, cf, stream=stream)
        torch.cuda.synchronize()
        H.hamls_plan_destroy(plan)
        lat.append(H.hamls_server_clock() - (t0 + tr.arrival[i]))
        a, b = served_cf[i], cf
        max_err = max(max_err, float(torch.linalg.norm(a - b) / torch.linalg.norm(b)))
    seq = summarize(lat, t0, H.hamls_server_clock())
    print(f"sequential: {seq}", file=sys.stderr, flush=True)

    return {
        "metric": "fits/s + p50/p99 latency, serving (continuous batching) vs the plain "
                  "one-request-at-a-time FP64 path",
        "value": served["fits_per_s"],
        "unit": "fits/s",
        "n_gpus": 1,
        "steps": n,
        "warmup": 0,
        "ms_per_step": 1e3 * served["makespan_s"] / n,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"S2 serving trace: {n} requests, Poisson arrivals at {args.rate:g}/s, N uniform "
                        f"in {{32,64,128,256}}, K uniform in {{2,3,4}}, M log-uniform in [1e4, 1e6] from "
                        f"the cluster + hole generator, kNN n = 4m, chi-target regularization, F = 1",
            "slots": args.slots,
            "hbm_budget": "80% of free device memory",
        },
        "latency_ms": {"p50": served["p50_ms"], "p99": served["p99_ms"]},
        "serving": served,
        "serving_burst": burst,
        "sequential_fp64": seq,
        "vs_sequential": {"fits_per_s": served["fits_per_s"] / seq["fits_per_s"],
                          "p99": served["p99_ms"] / seq["p99_ms"]},
        "max_rel_l2_served_vs_sequential": max_err,
        "timing": "host monotonic clock from each request's scheduled arrival to its completion; "
                  "every run starts with no resident plan; serving_burst submits all requests at "
                  "once (the loop's capacity)",
    }


def cpu_baseline(wl, plan, gv, H, budget_s):
    """The FP64 oracle (untuned) on a bounded sample of the same workload:
    every s-th grid node for step 2 (brute-force neighbours + QR solves), and
    the full step-3 quadrature (direct sums).  Extrapolated to the whole grid."""
    import oracle

    po = oracle.params(**wl.params)
    opts, _ = oracle.grid(po)
    MQ = opts.shape[0]
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    probe = np.arange(0, MQ, max(1, MQ // 256))
    t = time.perf_counter()
    oracle.mls(po, opts, wl.nodes, wl.values, rows=probe)
    per_row = (time.perf_counter() - t) / probe.size
    n_rows = int(min(MQ, max(probe.size, budget_s / max(per_row, 1e-9))))
    rows = np.unique(np.linspace(0, MQ - 1, n_rows).astype(np.int64))
    t = time.perf_counter()
    om = oracle.mls(po, opts, wl.nodes, wl.values, rows=rows)
    t_mls = time.perf_counter() - t
    t = time.perf_counter()
    gcpu = gv.cpu().numpy()
    oracle.coeffs(po, gcpu)
    t_quad = time.perf_counter() - t
    t_fit = t_mls * MQ / rows.size + t_quad
    F = wl.values.shape[0]
    ref = om["values"]
    got = gcpu[:, rows]
    ok = ~np.isnan(ref[0])
    err = float(np.linalg.norm(got[:, ok] - ref[:, ok]) / np.linalg.norm(ref[:, ok]))
    return (
        {"value": MQ * F / t_fit, "unit": "grid nodes/s", "cores": threads, "kind": "oracle",
         "sample": f"step 2 on {rows.size} of {MQ} grid nodes ({t_mls:.1f} s, extrapolated) + full step 3 "
                   f"({t_quad:.1f} s); FP64 C oracle, OpenMP"},
        {"rel_l2_vs_oracle_on_sample": err, "sample_rows": int(rows.size)},
    )


if __name__ == "__main__":
    main()
