#!/usr/bin/env python
"""Benchmark of the HAMLS hot path on one MI355X.

Default workload (--workload c3, the largest configuration): S2 ill-distributed
nodes, M = 4,000,000 (8 von Mises-Fisher clusters with kappa = 20 plus 20 %
uniform, twelve caps of radius 10-25 degrees removed), bandwidth N = 512, MLS
degree K = 4 (m = 15), Gauss-Legendre grid 513 x 1026 (526,338 local solves),
adaptive radius with n = 60, eps = 0.05, chi-target regularization (chi_T = 10,
chi_full = 20), one field, FP64.
Other workloads: c2 (S2, M = 2e5, N = 128, K = 3, grid 129 x 258, n = 40), so3
(M = 1e6 rotations, N = 64, K = 2, Euler grid 130^3, n = 40), t3 (M = 2e6
points, N = 64, K = 3, grid 128^3, n = 80), serve (the request loop).

One step = one whole fit with the inputs resident in device memory:
node binning + sort + support radii (plan rebind), the MLS value at every grid
node (Gram assembly + regularized solve + extended-precision re-solve of the
ill-conditioned centres), the quadrature (ring DFTs + Legendre contraction on
S2; axis DFTs + Wigner contraction on SO(3); 3-D FFT on T3).
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
# FP32 vector peak without packed FP32 instructions (which this build does not
# use): one FP32 FMA per lane per cycle, the FP64 rate
PEAK_FP32_VALU_TFLOPS = 78.6
PEAK_FP32_MFMA_TFLOPS = 157.3  # dense FP32 matrix-core peak
PEAK_HBM_GBS = 8000.0


def pct(a, q):
    return float(np.percentile(np.asarray(a), q))


# kernel (name prefix) of each phase's main launch, for the counter summary
PHASE_KERNEL = {
    "s2": {"binning": None, "radius": "k_s2_radius", "assemble": "k_s2_assemble",
           "solve": "k_mls_solve<", "resolve": "k_s2_dd_gram", "ring_dft": "k_s2_ring_fft",
           "contract": "k_s2_legendre", "gather": "k_gather_values"},
    "so3": {"binning": None, "radius": "k_grid_radius<4", "assemble": "k_grid_mls<4",
            "solve": "k_mls_solve<", "resolve": "k_grid_mls<4", "ring_dft": "k_fft_axis",
            "contract": "k_so3_contract", "gather": "k_gather_values"},
    "t3": {"binning": None, "radius": "k_grid_radius<3", "assemble": "k_grid_mls<3",
           "solve": "k_mls_solve<", "resolve": "k_grid_mls<3", "ring_dft": "k_fft_axis",
           "contract": None, "gather": "k_gather_values"},
}

# the kernels behind each timed phase (the phase's duration is theirs together)
PHASE_LAUNCHES = {
    "s2": {"radius": "k_s2_radius (one launch)",
           "resolve": "cost sort of the list (3 short launches) + k_s2_dd_gram<K, 1> + k_dd_solve<m, 1, false>",
           "assemble": "k_route_list (when routing) + k_s2_assemble_ordered<K> (or the tuned form)",
           "solve": "k_mls_solve<m, 16>"},
}

# file-name stem of a workload's committed rocprofv3 summaries
PROFILE_NAME = {"c3": "s2_c3", "c2": "s2_c2", "c2fixed": "s2_c2_fixed_radius", "c2smooth": "s2_c2_smoothed_radius",
                "c2hybrid": "s2_c2_hybrid_radius", "so3": "so3_m1e6_n64", "t3": "t3_m2e6_n64"}


def _progress(msg):
    """A progress line on stderr (the JSON result alone goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


WORKLOADS = {
    "c2smooth": ("s2_clusters_smooth", "S2 ill-distributed (C2 nodes, M=200000), N=128, K=3, grid 129x258, smoothed "
                 "adaptive radius: d_n (n=40) on 65536 Fibonacci points, degree-zero MLS at the grid, eps=0.05, "
                 "chi_T=10 chi_full=20, F=1, FP64"),
    "c2fixed": ("s2_clusters_fixed", "S2 ill-distributed under a fixed radius (skewed neighbour counts 0-2400, "
                "median 196), M=200000 (C2 nodes), N=128, K=3, grid 129x258, delta0=0.1 rad, chi_T=10 "
                "chi_full=20, F=1, FP64"),
    "c2hybrid": ("s2_clusters_hybrid", "S2 ill-distributed under the hybrid radius max(delta0, (1+eps) d_n) "
                 "(neighbour counts ~44-5700, median ~630), M=200000 (C2 nodes), N=128, K=3, grid 129x258, "
                 "delta0=0.16 rad, kNN n=40 eps=0.05, chi_T=10 chi_full=20, F=1, FP64"),
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


def measured_traffic(workload, kernel):
    """HBM bytes per launch of the kernel whose name starts with `kernel` (the
    FP64 pass; the double-double re-solve when `resolve`) from the committed
    rocprofv3 counter summary of this workload (FETCH_SIZE and WRITE_SIZE
    scaled by the copy calibration), or None when there is none or the HIP
    sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{PROFILE_NAME.get(workload, workload)}_hbm_traffic.txt")
    if kernel is None or not os.path.exists(path):
        return None
    resolve = kernel.startswith("resolve:")
    kernel = kernel.split(":", 1)[-1]
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
        targs = name[name.index("<") + 1:].rstrip(">").split(", ") if "<" in name else []
        if kernel.startswith("k_s2_dd_gram"):
            # the S2 double-double Gram pass of one field: <K, 1>
            if name.startswith(kernel) and len(targs) == 2 and targs[1] == "1":
                return float(k["bytes"])
            continue
        # the grid domains' double-double re-solve instantiations carry
        # "true" as their third template argument
        dd = len(targs) > 2 and targs[2] == "true"
        if name.startswith(kernel) and dd == resolve:
            return float(k["bytes"])
    return None


def flops_per_pair(domain, m, F):
    """Algorithmic FLOPs of one (grid node, neighbour) pair of the MLS step:
    membership key (S2 dot 5, SO3 dot 7, T3 min-image distance 12), tangent
    coordinates (S2 12, SO3 24, T3 3), distance and Wendland weight ~40,
    monomials m - 1, Gram m(m+1) (symmetric m x m, one FMA per entry), right-hand
    sides 2mF."""
    key = {"s2": 5, "so3": 7, "t3": 12}[domain]
    crd = {"s2": 12, "so3": 24, "t3": 3}[domain]
    return key + crd + 40 + (m - 1) + m * (m + 1) + 2 * m * F


def flops_per_solve(m, F):
    """Algorithmic FLOPs of one local solve: Cholesky of the order m-1 block
    ((m-1)^3/3 FMA), two triangular solves per right-hand side, and the tau
    search (64 steps of ~3m)."""
    return 2 * (m - 1) ** 3 // 3 + 2 * (m - 1) ** 2 * (1 + F) + 64 * 3 * m


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS) + ["serve"],
                    help="serve: the request loop (continuous batching) on the serving trace")
    ap.add_argument("--requests", type=int, default=512, help="serve: number of requests")
    ap.add_argument("--rate", type=float, default=200.0, help="serve: Poisson arrival rate (1/s)")
    ap.add_argument("--slots", type=int, default=4, help="serve: worker streams of the server")
    ap.add_argument("--fields", type=int, default=1,
                    help="fields per fit: the workload's field plus seeded N(0,1) node values")
    ap.add_argument("--cpu-seconds", type=float, default=16.0,
                    help="budget of the CPU oracle sample (all cores; a third of it on one core)")
    ap.add_argument("--no-mfma", action="store_true", help="skip the F = 64 contraction measurement")
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

    _progress(f"{args.workload}: inputs and plan ready ({gen_s:.1f} s)")
    # launch form of the assembly pass (grid order, cost order, S2 FP64 work
    # queue), measured on these nodes and kept by the plan
    tune = None
    q, t = H.hamls_plan_tune(plan, stream=stream)
    tune = {"form": q, "grid_order_ms": t[0], "cost_order_dispatch_ms": t[1]}
    if domain == "s2" and args.precision == "fp64":
        tune["queue_ms"] = {"8/CU": t[2], "12/CU": t[3]}
    if domain == "s2":
        en, rt = H.hamls_plan_routing(plan)
        tune["routing"] = {"enabled": en, "step2_ms_without": rt[0], "step2_ms_with": rt[1]}

    def step():
        H.hamls_plan_rebind(plan, nodes, stream=stream)
        H.hamls_mls_to_grid(plan, vals, gv, stream=stream)
        H.hamls_grid_to_coeffs(plan, gv, cf, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    for ph in H.PHASES:
        H.hamls_timing_read(plan, ph)  # clear

    _progress("tuned and warmed up")
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

    # roofline of the dominant phase, priced on the method's algorithmic work
    m = info.m
    illc = (diag["status"] & H.ST_ILLCOND) != 0
    n_ill_pairs = int(diag["n"][illc].astype(np.int64).sum())
    work = phase_work(domain, info, m, F, pairs, MQ, n_ill, n_ill_pairs)
    wk = work.get(dom)
    kern = PHASE_KERNEL[domain].get(dom)
    if dom == "resolve" and kern:
        kern = "resolve:" + kern
    traffic = measured_traffic(args.workload, kern) if args.precision == "fp64" and F == 1 else None
    roof = None
    if wk is not None:
        bound, amount = wk
        sec = phases[dom]["avg_ms"] * 1e-3
        if bound == "hbm":
            ach = amount / sec / 1e9
            roof = {"kernel": dom, "bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                    "frac": ach / PEAK_HBM_GBS, "traffic": traffic, "units_per_launch": {"bytes": amount}}
        else:
            peak = PEAK_FP64_VALU_TFLOPS if args.precision == "fp64" else PEAK_FP32_VALU_TFLOPS
            ach = amount / sec / 1e12
            roof = {"kernel": dom, "bound": "alu", "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                    "frac": ach / peak, "traffic": traffic, "units_per_launch": {"flop": amount}}
        roof["launches"] = PHASE_LAUNCHES.get(domain, {}).get(dom, kern)
    # the whole MLS step (radius + assembly + solve + re-solve) against the
    # FP64 vector peak, on its algorithmic FLOPs
    mls_ms = sum(phases[k]["avg_ms"] for k in ("radius", "assemble", "solve", "resolve") if k in phases)
    mls_fl = pairs * flops_per_pair(domain, m, F) + MQ * flops_per_solve(m, F)
    mls_roof = {"phases": "radius + assemble + solve + resolve", "ms": mls_ms, "flop": mls_fl,
                "achieved": mls_fl / (mls_ms * 1e-3) / 1e12, "peak": PEAK_FP64_VALU_TFLOPS,
                "unit": "TFLOP/s", "frac": mls_fl / (mls_ms * 1e-3) / 1e12 / PEAK_FP64_VALU_TFLOPS}

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
        "mls_step_roofline": mls_roof,
    }
    if tune is not None:
        out["assembly_launch"] = tune

    _progress("census and timed fits done; captured fits, generating functions")
    out["captured_fit"] = graph_bench(H, torch, plan, info, vals, K)
    out["generating_functions"] = gen_bench(H, torch, plan, info, vals, gv, stream, K, 1e3 * wall / K)

    if domain == "s2" and not args.no_mfma:
        out["contraction_f64"] = contraction_bench(H, torch, wl, 64, K)
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


def phase_work(domain, info, m, F, pairs, MQ, n_ill, n_ill_pairs):
    """Algorithmic work of each phase's launch: ("hbm", bytes) or ("alu",
    FLOPs).  Bytes count what the method must move once: coordinates and keys
    of the binning passes, each sorted record read once by the radius search
    plus its outputs, the DFT inputs and outputs, the Legendre / Wigner table
    read once.  FLOPs count the pair and solve arithmetic of the centres a
    launch handles."""
    Mn = info.num_nodes
    nt, npf = info.grid_dims[0], info.grid_dims[1]
    N = info.bandwidth
    dimx = 4 if domain == "so3" else 3
    nrec = 2 * Mn if domain == "so3" else Mn
    rec = 8 * dimx
    w = {
        # keys: read coordinates + write key and index; per radix pass 16 B
        # (key + index, read + write); cell table; gather: index and
        # coordinates read, coordinates and permutation written
        "binning": ("hbm", Mn * 8 * dimx + nrec * (8 + 2 * 16 + 8 + 2 * (4 + rec))),
        # every sorted record read once; radius, threshold and status written
        "radius": ("hbm", nrec * rec + MQ * 17),
        "assemble": ("alu", pairs * flops_per_pair(domain, m, F)),
        "solve": ("alu", MQ * flops_per_solve(m, F)),
        "resolve": ("alu", n_ill_pairs * flops_per_pair(domain, m, F) + n_ill * flops_per_solve(m, F)),
        "gather": ("hbm", nrec * (4 + 16 * F)),
    }
    if domain == "s2":
        w["ring_dft"] = ("hbm", MQ * 8 * F + nt * (N + 1) * 16 * F)
        w["contract"] = ("hbm", ((nt + 1) // 2) * ((N + 1) * (N + 2) // 2) * 8 + (N + 1) ** 2 * 16 * F)
    elif domain == "so3":
        K2 = 2 * N + 1
        nb, na, ng = info.grid_dims[0], info.grid_dims[1], info.grid_dims[2]
        # alpha pass: real grid in, (k, gamma) spectra out; gamma pass
        w["ring_dft"] = ("hbm", F * nb * (na * ng * 8 + 2 * K2 * ng * 16 + K2 * K2 * 16))
        w["contract"] = ("hbm", nb * info.num_coeffs * 8 + F * (nb * K2 * K2 + info.num_coeffs) * 16)
    else:
        # real grid values in, complex coefficients out, one pass each
        w["ring_dft"] = ("hbm", F * MQ * (8 + 16))
    return w


def contraction_bench(H, torch, wl, F, K):
    """The S2 Legendre contraction at F fields on random grid values: the FP64
    kernel of the plain path and the FP32 matrix-core kernel of the mixed path
    (step 3 only; the contraction kernel timed with HIP events, and apart from
    it the ring transforms and, on the mixed path, the fold of the spectra
    into the FP32 blocks and the unfold into the coefficients).  FLOPs: for
    every table entry w_t P_n^k(x_t) of the northern rings (after the
    equatorial fold) and every field, one FMA each for the real and the
    imaginary part of the folded spectrum."""
    res = {"fields": F}
    dev = torch.device("cuda:0")
    nodes = torch.as_tensor(wl.nodes[: max(wl.params["knn_count"], 1000)], dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    g = None
    for prec in ("fp64", "mixed"):
        p = H.params_from_workload(wl.params, precision=prec)
        plan = H.hamls_plan(p, nodes, stream=stream)
        try:
            info = H.hamls_plan_info_get(plan)
            if g is None:  # the same grid values for both paths
                gen = torch.Generator(device=dev).manual_seed(1234)
                g = torch.randn((F, info.num_grid), dtype=torch.float64, device=dev, generator=gen)
            cf = torch.empty((F, info.num_coeffs, 2), dtype=torch.float64, device=dev)
            H.hamls_grid_to_coeffs(plan, g, cf, stream=stream)
            torch.cuda.synchronize()
            H.hamls_timing_phases(plan, ["contract", "ring_dft", "fold"])
            H.hamls_timing_enable(plan, True)
            for ph in ("contract", "ring_dft", "fold"):
                H.hamls_timing_read(plan, ph)
            for _ in range(K):
                H.hamls_grid_to_coeffs(plan, g, cf, stream=stream)
            n, ms = H.hamls_timing_read(plan, "contract")
            nd, msd = H.hamls_timing_read(plan, "ring_dft")
            _, msf = H.hamls_timing_read(plan, "fold")
            H.hamls_timing_enable(plan, False)
            N = info.bandwidth
            th = (info.grid_dims[0] + 1) // 2
            entries = th * (N + 1) * (N + 2) // 2
            fl = 4 * entries * F
            avg = ms / n
            peak = PEAK_FP32_MFMA_TFLOPS if prec == "mixed" else PEAK_FP64_VALU_TFLOPS
            res[prec] = {"kernel": "k_s2_legendre_mfma" if prec == "mixed" else "k_s2_legendre",
                         "avg_ms": avg, "ring_dft_ms": msd / nd, "fold_unfold_ms": msf / K, "flop": fl,
                         "achieved": fl / (avg * 1e-3) / 1e12, "unit": "TFLOP/s", "peak": peak,
                         "frac": fl / (avg * 1e-3) / 1e12 / peak}
            if prec == "mixed":
                ref = res.get("_ref")
                if ref is not None:
                    res["mixed_rel_l2_vs_fp64"] = float(torch.linalg.norm(cf - ref) / torch.linalg.norm(ref))
            else:
                res["_ref"] = cf.clone()
        finally:
            H.hamls_plan_destroy(plan)
    res.pop("_ref", None)
    return res


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


def _omp_threads(n):
    """Set the OpenMP thread count of the oracle's runtime (libgomp)."""
    import ctypes

    try:
        ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))
        return True
    except OSError:
        return False


def cpu_baseline(wl, plan, gv, H, budget_s):
    """The FP64 oracle (untuned) on a bounded sample of the same workload:
    whole rings of the grid, every s-th ring (s chosen to fit the budget; the
    ring subset of the large configuration), for step 2 (brute-force
    neighbours + QR solves) with all host cores, then a smaller sample on one
    core; the full step-3 quadrature (direct sums) with all cores.  Both
    extrapolated to the whole grid."""
    import oracle

    po = oracle.params(**wl.params)
    gpts, _ = H.hamls_plan_grid(plan)
    MQ = gpts.shape[0]
    dims = oracle.grid_dims(po)
    ring = int(np.prod([d for d in dims[1:] if d > 0]))  # grid nodes per ring (first axis)
    nrings = MQ // ring
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    _omp_threads(threads)
    probe = np.arange(0, MQ, max(1, MQ // 128))
    t = time.perf_counter()
    oracle.mls(po, gpts, wl.nodes, wl.values, rows=probe)
    per_row = (time.perf_counter() - t) / probe.size
    want = max(1, int(budget_s / max(per_row, 1e-9) / ring))  # rings that fit the budget
    stride = max(1, -(-nrings // want))
    rings = np.arange(0, nrings, stride)
    rows = (rings[:, None] * ring + np.arange(ring)[None, :]).ravel()
    t = time.perf_counter()
    om = oracle.mls(po, gpts, wl.nodes, wl.values, rows=rows)
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
    emax = float(np.abs(got[:, ok] - ref[:, ok]).max() / np.abs(ref[:, ok]).max())
    base = {"value": MQ * F / t_fit, "unit": "grid nodes/s", "cores": threads, "kind": "oracle",
            "sample": f"step 2 on {rings.size} of {nrings} grid rings (every {stride}th ring, {rows.size} "
                      f"grid nodes, {t_mls:.1f} s, extrapolated) + full step 3 ({t_quad:.1f} s); FP64 C "
                      f"oracle, OpenMP, {threads} threads"}
    # one core: a third of the budget, grid nodes spread over the grid
    if _omp_threads(1):
        n1 = int(min(MQ, max(16, budget_s / 3.0 / max(per_row * threads, 1e-9))))
        rows1 = np.unique(np.linspace(0, MQ - 1, n1).astype(np.int64))
        t = time.perf_counter()
        oracle.mls(po, gpts, wl.nodes, wl.values, rows=rows1)
        t1 = time.perf_counter() - t
        _omp_threads(threads)
        base["one_core"] = {"value": MQ * F / (t1 * MQ / rows1.size + t_quad * threads),
                            "unit": "grid nodes/s", "cores": 1,
                            "sample": f"step 2 on {rows1.size} grid nodes spread over the grid ({t1:.1f} s, "
                                      f"extrapolated) + step 3 taken as {threads} x its all-core time"}
    return base, {"rel_l2_vs_oracle_on_sample": err, "max_rel_vs_oracle_on_sample": emax,
                  "sample_rows": int(rows.size)}


if __name__ == "__main__":
    main()
