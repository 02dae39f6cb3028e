// grid.hip -- step 2 of Alg. 1 on SO(3) and T3 (gfx950).
//
// Both domains bin their nodes on a uniform D-dimensional cell grid:
//   T3   D = 3, [0,1)^3, periodic; key -d^2 with d the min-image distance
//   SO3  D = 4, [-1,1]^4 in quaternion space; every node is stored twice,
//        as q and -q, so that the plain dot product finds exactly the copy on
//        the centre's hemisphere and equals |q.p| bit for bit (negation is
//        exact); key = dot, member iff dot > cos(delta/2) (rotation angle
//        2 arccos|q.p|, Sec. 2.2)
// The cover of a search ball is a box of cells; its rows along the last axis
// are contiguous runs of sorted records, enumerated one row per lane and
// scanned flattened, 64*U slots per step.
#include <math.h>

#include "common.h"
#include "device_common.h"

namespace hamls {

struct GridGeom {
    int dom;             // HAMLS_SO3 or HAMLS_T3
    int nc;              // cells per axis
    double lo, h, ih;    // cell i of an axis covers [lo + i h, lo + (i+1) h); ih = 1/h
    const double* grid;  // M_Q x D (quaternions for SO3, points for T3)
    const double* X;     // sorted records, SoA D x cap
    const double* nu;    // sorted node weights or null
    const int32_t* perm; // sorted record -> original node
    int64_t cap;
    const int32_t* cs;   // cell_start
    const int32_t* mlist;  // member lists of the radius search (kListCap per node) or null
    const int32_t* mcnt;   // their lengths, -1 where the assembly scans the box
};

GridGeom make_grid_geom(const Plan& P) {
    GridGeom g;
    g.dom = P.dom;
    g.nc = P.gbins.nc;
    g.lo = P.gbins.lo;
    g.h = P.gbins.h;
    // exact reciprocal of the cell width: nc per unit length (T3), nc/2 (SO3)
    g.ih = P.dom == HAMLS_T3 ? (double)P.gbins.nc : 0.5 * P.gbins.nc;
    g.grid = P.d_grid;
    g.X = P.d_x;
    g.nu = P.has_nu ? P.d_nu : nullptr;
    g.perm = P.d_perm;
    g.cap = P.cap;
    g.cs = P.d_cell_start;
    g.mlist = P.d_mlist;
    g.mcnt = P.d_mcnt;
    return g;
}

// Closeness key (larger is closer), in a fixed association without fused
// operations: SO3 the 4-D dot product, T3 minus the squared min-image distance.
template <int D>
__device__ __forceinline__ double grid_key(const GridGeom& g, int64_t i, const double* q) {
#pragma clang fp contract(off)
    if (D == 4) {
        double a = g.X[i] * q[0];
        double b = g.X[g.cap + i] * q[1];
        double c = g.X[2 * g.cap + i] * q[2];
        double e = g.X[3 * g.cap + i] * q[3];
        double s = a + b;
        s = s + c;
        s = s + e;
        return s;
    }
    double s = 0.0;
    for (int d = 0; d < 3; d++) {
        double dl = g.X[d * g.cap + i] - q[d];
        dl = dl - rint(dl);
        double sq = dl * dl;
        s = s + sq;
    }
    return -s;
}

// Box half-width (embedding coordinates) and key threshold of a search
// radius r (rotation angle for SO3, distance for T3).
template <int D>
__device__ __forceinline__ double grid_rho(const GridGeom& g, double r) {
    return D == 4 ? 2.0 * sin(0.25 * fmin(r, kPi)) : r;
}
// Key threshold of the box half-width rho (SO3 chordal distance in R^4:
// |p - q|^2 = 2 - 2 p.q; T3 Euclidean) and back.
template <int D>
__device__ __forceinline__ double grid_key_of_rho(double rho) {
    return D == 4 ? 1.0 - 0.5 * rho * rho : -(rho * rho);
}
template <int D>
__device__ __forceinline__ double grid_rho_of_key(double k) {
    return D == 4 ? sqrt(fmax(2.0 - 2.0 * k, 0.0)) : sqrt(fmax(-k, 0.0));
}
// Largest search radius: SO3 the rotation angle pi; T3 0.87, beyond the
// largest min-image distance sqrt(3)/2, so that the ball holds every node.
template <int D>
__device__ __forceinline__ double grid_rmax(const GridGeom& g) {
    return D == 4 ? kPi : 0.87;
}

struct BoxGeo {
    int a[4], n[4];  // per axis first cell and cell count
    bool full[4];
    int rows;        // rows over the first D-1 axes
};

template <int D>
__device__ __forceinline__ BoxGeo box_geo(const GridGeom& g, const double* q, double rho) {
    const double margin = 1e-9;
    BoxGeo B;
    B.rows = 1;
    for (int d = 0; d < D; d++) {
        int a = (int)floor((q[d] - rho - margin - g.lo) * g.ih);
        int b = (int)floor((q[d] + rho + margin - g.lo) * g.ih);
        if (D == 3) {
            if (b - a + 1 >= g.nc) {
                a = 0;
                b = g.nc - 1;
                B.full[d] = true;
            } else {
                B.full[d] = false;
            }
        } else {
            a = a < 0 ? 0 : a;
            b = b > g.nc - 1 ? g.nc - 1 : b;
            B.full[d] = false;
        }
        B.a[d] = a;
        B.n[d] = b - a + 1;
        if (d < D - 1) B.rows *= B.n[d];
    }
    return B;
}

// Record ranges of one row of the box.
template <int D>
__device__ __forceinline__ void box_row_ranges(const GridGeom& g, const BoxGeo& B, int row, int& lo1,
                                               int& len1, int& lo2, int& len2) {
    const int nc = g.nc, L = D - 1;
    int64_t base = 0, mul = nc;
    int rem = row;
#pragma unroll
    for (int d = L - 1; d >= 0; d--) {
        int c = B.a[d] + rem % B.n[d];
        rem /= B.n[d];
        c = c < 0 ? c + nc : (c >= nc ? c - nc : c);
        base += (int64_t)c * mul;
        mul *= nc;
    }
    const int a = B.a[L], b = B.a[L] + B.n[L] - 1;
    // the run [a, b] of the last axis, split in two where it wraps (T3)
    const int a1 = a < 0 ? a + nc : a;
    const int e1 = (a < 0 || b >= nc) ? nc : b + 1;
    const int e2 = a < 0 ? b + 1 : (b >= nc ? b - nc + 1 : 0);
    const int l1 = g.cs[base + a1];
    const int l2 = g.cs[base];
    lo1 = l1;
    len1 = g.cs[base + e1] - l1;
    lo2 = l2;
    len2 = g.cs[base + e2] - l2;
}

template <int D>
__device__ __forceinline__ int grid_cover_count(const GridGeom& g, const double* q, double rho) {
    BoxGeo B = box_geo<D>(g, q, rho);
    const int lane = threadIdx.x & 63;
    int tot = 0;
    for (int rb = 0; rb < B.rows; rb += 64) {
        int r = rb + lane, lo1 = 0, len1 = 0, lo2 = 0, len2 = 0;
        if (r < B.rows) box_row_ranges<D>(g, B, r, lo1, len1, lo2, len2);
        tot += wave_sum_int(len1 + len2);
    }
    return tot;
}

// Visits every record in the box cover, 64*U slots per step (see s2_scan).
template <int D, int U, class Fn>
__device__ __forceinline__ void grid_scan(const GridGeom& g, const double* q, double rho, int* sh,
                                          Fn&& body) {
    BoxGeo B = box_geo<D>(g, q, rho);
    const int lane = threadIdx.x & 63;
    int* s_lo1 = sh;
    int* s_len1 = sh + 64;
    int* s_lo2 = sh + 128;
    int* s_pre = sh + 192;
    for (int rb = 0; rb < B.rows; rb += 64) {
        int r = rb + lane, lo1 = 0, len1 = 0, lo2 = 0, len2 = 0;
        if (r < B.rows) box_row_ranges<D>(g, B, r, lo1, len1, lo2, len2);
        int len = len1 + len2;
        int incl = wave_incl_scan_int(len);
        int total = __shfl(incl, 63, 64);
        s_lo1[lane] = lo1;
        s_len1[lane] = len1;
        s_lo2[lane] = lo2;
        s_pre[lane] = incl - len;
        if (lane == 63) s_pre[64] = incl;
        __syncthreads();
        int kc = 0;
        for (int base = 0; base < total; base += 64 * U) {
            while (s_pre[kc + 1] <= base) kc++;
            bool valid[U];
            int idx[U];
            int k = kc;
#pragma unroll
            for (int u = 0; u < U; u++) {
                int sl = base + 64 * u + lane;
                valid[u] = sl < total;
                idx[u] = 0;
                if (valid[u]) {
                    while (s_pre[k + 1] <= sl) k++;
                    int o = sl - s_pre[k];
                    idx[u] = o < s_len1[k] ? s_lo1[k] + o : s_lo2[k] + (o - s_len1[k]);
                }
            }
            body(valid, idx);
        }
        __syncthreads();
    }
}

// Visits the records of a member list (n entries), 64*U per step, with the
// calling convention of grid_scan.
template <int U, class Fn>
__device__ __forceinline__ void grid_list_scan(const int32_t* list, int n, Fn&& body) {
    const int lane = threadIdx.x & 63;
    for (int base = 0; base < n; base += 64 * U) {
        bool valid[U];
        int idx[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int sl = base + 64 * u + lane;
            valid[u] = sl < n;
            idx[u] = valid[u] ? list[sl] : 0;
        }
        body(valid, idx);
    }
}

// ---------------------------------------------------------------------------
// binning
// ---------------------------------------------------------------------------

// One key per record: T3 one record per node; SO3 two (q and -q, the second
// encoded as index M + i).
__global__ void k_grid_keys(const double* __restrict__ nodes, int64_t M, int dom, int D, int nc,
                            double lo, double ih, uint32_t* __restrict__ keys,
                            int32_t* __restrict__ idx) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t nrec = dom == HAMLS_SO3 ? 2 * M : M;
    if (r >= nrec) return;
    int64_t i = r < M ? r : r - M;
    double sg = r < M ? 1.0 : -1.0;
    uint32_t key = 0;
    for (int d = 0; d < D; d++) {
        double x = sg * nodes[(int64_t)D * i + d];
        int c;
        if (dom == HAMLS_T3) {
            double y = x - floor(x);
            c = (int)(y * nc);
            c = c >= nc ? nc - 1 : (c < 0 ? 0 : c);
        } else {
            c = (int)floor((x - lo) * ih);
            c = c < 0 ? 0 : (c > nc - 1 ? nc - 1 : c);
        }
        key = key * (uint32_t)nc + (uint32_t)c;
    }
    keys[r] = key;
    idx[r] = (int32_t)r;
}

__global__ void k_grid_gather(const int32_t* __restrict__ idx, const double* __restrict__ nodes,
                              const double* __restrict__ nu, int64_t nrec, int64_t M, int D,
                              int64_t cap, double* __restrict__ X, double* __restrict__ NU,
                              int32_t* __restrict__ perm) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrec) return;
    int64_t j = idx[r];
    int64_t i = j < M ? j : j - M;
    double sg = j < M ? 1.0 : -1.0;
    for (int d = 0; d < D; d++) X[d * cap + r] = sg * nodes[(int64_t)D * i + d];
    perm[r] = (int32_t)i;
    if (nu) NU[r] = nu[i];
}

hamls_status launch_grid_keys(const Plan& P, const double* nodes, int64_t M, hipStream_t s) {
    int64_t nrec = P.dom == HAMLS_SO3 ? 2 * M : M;
    int bs = 256;
    hipLaunchKernelGGL(k_grid_keys, dim3((unsigned)((nrec + bs - 1) / bs)), dim3(bs), 0, s, nodes, M,
                       P.dom, P.gbins.D, P.gbins.nc, P.gbins.lo, 0.5 * P.gbins.nc, P.d_key[0], P.d_idx[0]);
    HAMLS_HIP(hipGetLastError());
    return HAMLS_OK;
}

hamls_status launch_grid_gather(const Plan& P, const int32_t* idx, const double* nodes,
                                const double* nu, int64_t M, hipStream_t s) {
    int64_t nrec = P.dom == HAMLS_SO3 ? 2 * M : M;
    int bs = 256;
    hipLaunchKernelGGL(k_grid_gather, dim3((unsigned)((nrec + bs - 1) / bs)), dim3(bs), 0, s, idx,
                       nodes, nu, nrec, M, P.gbins.D, P.cap, P.d_x, P.d_nu, P.d_perm);
    HAMLS_HIP(hipGetLastError());
    return HAMLS_OK;
}

// ---------------------------------------------------------------------------
// support radius (eq. (5), (6), (12))
// ---------------------------------------------------------------------------

// Grid nodes per wave of the radius search.  Consecutive grid nodes are
// neighbours on the product grid (its last axis varies fastest), so every node
// after the first of a group starts from the previous node's n-th distance
// widened by kSeedGrow: the first scan then nearly always holds n nodes, with
// no sizing on the cell table and no second scan.
constexpr int kRadGroup = 8;
constexpr double kSeedGrow = 1.15;

// One wave per group of kRadGroup consecutive grid nodes, one node at a time.
// Adaptive radius: the first node of a group brackets a search radius on the
// cell-cover count (cell table only), the others take the seed above; scan the
// box keeping the keys of the ball, resize until it holds between n and kGCap
// nodes, take the n-th largest key exactly.  SO3: delta = (1+eps) 2
// arccos(t_n), clamped below pi, threshold cos(delta/2).  T3: threshold
// c = (1+eps)^2 d_n^2 on d^2 (no transcendental), delta = sqrt(c).  A fixed
// delta_0 is merged (larger radius wins).  Thresholds are stored on the key:
// SO3 c, T3 -c.
template <int D>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(D == 4 ? 4 : 5))) void k_grid_radius(
    GridGeom g, int64_t M, int64_t MQ, int knn, double eps, double wfac, double delta0, double* thr,
    double* delta, uint8_t* rstatus, int32_t* mlist, int32_t* mcnt) {
    constexpr int U = 4;
    // 416 candidates keep the LDS at 8 KB, five waves per SIMD with 96 VGPRs
    // (the wave-uniform state in scalar registers)
    constexpr int kGCap = kGridCandCap;
    constexpr int kBinCap = 128;
    __shared__ __align__(16) double buf[kGCap];
    __shared__ int ibuf[kGCap];  // record of each kept key
    __shared__ __align__(16) double binbuf[kBinCap];  // also the scan histogram
    __shared__ int ohist[256];
    __shared__ int sh[kScanLds];
    // groups in grid order, dealt over the XCDs
    const int jb = xcd_block(blockIdx.x, gridDim.x);
    const int lane = threadIdx.x;
    // largest search radius and its box half-width
    const double rmax = grid_rmax<D>(g);
    const double rhomax = uni_d(grid_rho<D>(g, rmax));
    double tprev = 0.0;   // n-th largest key of the group's previous node
    bool seeded = false;  // tprev holds one
    for (int gi = 0; gi < kRadGroup; gi++) {
        const int64_t jj = (int64_t)jb * kRadGroup + gi;
        if (jj >= MQ) break;
        const int j = (int)jj;
        double q[4] = {0.0, 0.0, 0.0, 0.0};
        for (int d = 0; d < D; d++) q[d] = uni_d(g.grid[(int64_t)D * j + d]);
        uint8_t st = 0;
        double dl = delta0;
        if (knn > 0) {
            tprev = uni_d(tprev);
            // initial box half-width rho: the seed, or (first node of a group)
            // the radius holding n nodes at the mean density with the box cover
            // count bracketed into [3n, 12n]; a scan with fewer than n nodes in
            // the ball grows it from the histogram of the records outside
            double rho;
            const double rs = grid_rho_of_key<D>(tprev) * kSeedGrow;
            const bool lean = seeded && rs > 0.1 * g.h;
            if (lean) {
                rho = fmin(rs, rhomax);
            } else {
                // radius holding n nodes at the mean density
                double r = fmin(D == 4 ? cbrt(6.0 * kPi * knn / (double)M) : cbrt(3.0 * knn / (4.0 * kPi * M)),
                                rmax);
                {
                    const int target = 3 * knn;
                    double rl = 0.0, rh = 0.0;
                    for (int it = 0; it < 20; it++) {
                        const int cov = grid_cover_count<D>(g, q, grid_rho<D>(g, r));
                        if (cov < target) {
                            if (r >= rmax) break;
                            rl = r;
                            r = rh > 0.0 ? sqrt(r * rh) : fmin(rmax, r * (cov < target / 6 ? 1.6 : 1.25));
                        } else if (cov > 4 * target && r > 1e-6) {
                            rh = r;
                            r = rl > 0.0 ? sqrt(r * rl) : r * 0.7;
                        } else {
                            break;
                        }
                    }
                }
                rho = grid_rho<D>(g, r);
            }
            // Keys at or above ktop are only counted (`above`).  With u = khi - key
            // (khi the largest key: SO3 1, T3 0): a scan that overflows the buffer
            // narrows the kept range to the bin of the n-th key in a 256-bin
            // histogram of u over [khi - ktop, khi - key(r)); a scan with fewer
            // than n keys in the ball grows it from a histogram of the records of
            // the box outside the ball (u over [u0, 16 u0), u0 = khi - key(r)): the
            // smallest bin edge with n records of the box inside holds at least n.
            const double khi = D == 4 ? 1.0 : 0.0;
            double r_hi = 0.0;  // half-width of a box known to overflow the buffer
            double tn = -1e300, ktop = 2.0;
            bool done = false, hemi = false;
            int lcount = -1;  // kept keys of the final scan when it kept them all
            double lkr = 2.0;
            int* hist = (int*)binbuf;  // 256 ints
            if (lean) {
                // seeded first scan: keep the keys of the ball, nothing else;
                // when it holds fewer than n or overflows the buffer, the
                // general loop below takes over (grown or at the same radius)
                const double kr = uni_d(grid_key_of_rho<D>(rho));
                rho = uni_d(rho);
                int count = 0;
                grid_scan<D, U>(g, q, rho, sh, [&](const bool* valid, const int* idx) {
                    double kv[U];
#pragma unroll
                    for (int u = 0; u < U; u++) kv[u] = grid_key<D>(g, idx[u], q);
#pragma unroll
                    for (int u = 0; u < U; u++) kv[u] = valid[u] ? kv[u] : -1e300;
#pragma unroll
                    for (int u = 0; u < U; u++) {
                        const bool in = kv[u] > kr;
                        const uint64_t mk = __ballot(in);
                        const int pos = count + rank_below(mk);
                        if (in && pos < kGCap) {
                            buf[pos] = kv[u];
                            ibuf[pos] = idx[u];
                        }
                        count += __popcll(mk);
                    }
                });
                __syncthreads();
                if (count >= knn && count <= kGCap) {
                    tn = nth_largest(buf, count, knn, kr, khi, sh, binbuf, kBinCap);
                    done = true;
                    lcount = count;
                    lkr = kr;
                } else if (count < knn) {
                    const double grow = 1.15 * cbrt((double)knn / (double)(count > 0 ? count : 1));
                    rho = fmin(rho * fmin(fmax(grow, 1.2), 2.0), rhomax);
                }
                __syncthreads();
            }
            for (int it = 0; it < 40 && !done; it++) {
                const double kr = grid_key_of_rho<D>(rho);
                const double ulo = uni_d(ktop < 2.0 ? khi - ktop : 0.0);
                const double hs = uni_d(256.0 / fmax((khi - kr) - ulo, 1e-300));
                const double u0 = uni_d(khi - kr), ohs = uni_d(256.0 / fmax(15.0 * u0, 1e-300));
                rho = uni_d(rho);
                ktop = uni_d(ktop);
                tn = uni_d(tn);
                r_hi = uni_d(r_hi);
                lkr = uni_d(lkr);
#pragma unroll
                for (int qq = 0; qq < 4; qq++) {
                    hist[4 * lane + qq] = 0;
                    ohist[4 * lane + qq] = 0;
                }
                __syncthreads();
                int count = 0, above = 0, nout = 0;
                grid_scan<D, U>(g, q, rho, sh, [&](const bool* valid, const int* idx) {
                    double kv[U];
#pragma unroll
                    for (int u = 0; u < U; u++) kv[u] = grid_key<D>(g, idx[u], q);
#pragma unroll
                    for (int u = 0; u < U; u++) kv[u] = valid[u] ? kv[u] : -1e300;
#pragma unroll
                    for (int u = 0; u < U; u++) {
                        const bool up = valid[u] && kv[u] >= ktop;
                        const bool in = valid[u] && kv[u] > kr && !up;
                        const bool out = valid[u] && kv[u] <= kr;
                        above += __popcll(__ballot(up));
                        nout += __popcll(__ballot(out));
                        if (out) {
                            int bin = (int)((khi - kv[u] - u0) * ohs);
                            atomicAdd(&ohist[bin < 0 ? 0 : (bin > 255 ? 255 : bin)], 1);
                        }
                        const uint64_t mk = __ballot(in);
                        const int pos = count + rank_below(mk);
                        if (in) {
                            if (pos < kGCap) {
                                buf[pos] = kv[u];
                                ibuf[pos] = idx[u];
                            } else {
                                int bin = (int)((khi - kv[u] - ulo) * hs);
                                atomicAdd(&hist[bin < 0 ? 0 : (bin > 255 ? 255 : bin)], 1);
                            }
                        }
                        count += __popcll(mk);
                    }
                });
                __syncthreads();
                if (above >= knn) {
                    // rounding put the n-th key at or above ktop: drop the bound
                    rho = fmin(grid_rho_of_key<D>(ktop), rhomax);
                    r_hi = 0.0;
                    ktop = 2.0;
                } else if (above + count < knn) {
                    if (rho >= rhomax) {
                        hemi = true;
                        done = true;
                    } else {
                        const int have = above + count;
                        double nr = -1.0;
                        if (have + nout >= knn) {
                            int before;
                            const int B = hist_select_bin(ohist, have, knn, before);
                            // widened by wfac = 1.005 (1 + eps) so that the scan also
                            // holds the support and can hand on its members
                            if (B < 255) nr = grid_rho_of_key<D>(khi - u0 * (1.0 + 15.0 * (B + 1) / 256.0)) * wfac;
                        }
                        if (nr <= rho) {
                            double grow = 1.15 * cbrt((double)knn / (double)(have > 0 ? have : 1));
                            grow = grow < 1.2 ? 1.2 : (grow > 2.0 ? 2.0 : grow);
                            nr = rho * grow;
                            if (r_hi > 0.0 && nr >= r_hi) nr = sqrt(rho * r_hi);
                        } else if (r_hi > 0.0) {
                            nr = fmin(nr, r_hi);
                        }
                        rho = fmin(nr, rhomax);
                    }
                } else if (count <= kGCap) {
                    tn = nth_largest(buf, count, knn - above, kr, fmin(ktop, khi), sh, binbuf, kBinCap);
                    done = true;
                    if (ktop >= 2.0) {
                        lcount = count;  // every key above key(r) is kept
                        lkr = kr;
                    }
                } else {
                    // bin in the histogram of every key of (key(r), ktop)
                    for (int a = lane; a < kGCap; a += 64) {
                        int bin = (int)((khi - buf[a] - ulo) * hs);
                        atomicAdd(&hist[bin < 0 ? 0 : (bin > 255 ? 255 : bin)], 1);
                    }
                    __syncthreads();
                    int before;
                    const int B = hist_select_bin(hist, above, knn, before);
                    r_hi = rho;
                    if (B < 255) rho = fmin(grid_rho_of_key<D>(khi - (ulo + (B + 1) / hs)), rhomax);
                    if (B > 0) ktop = khi - (ulo + B / hs);
                }
                __syncthreads();
            }
            if (!done) {
                // exact fallback: bitwise binary search for the largest key v with
                // #(key >= v) >= n among the keys of the ball of radius r
                const double kr = grid_key_of_rho<D>(rho);
                uint64_t lo = ordered_bits(kr), hi = ordered_bits(D == 4 ? 1.0 : 0.0);
                while (lo < hi) {
                    uint64_t mid = lo + (hi - lo + 1) / 2;
                    double v = from_ordered_bits(mid);
                    int count = 0;
                    grid_scan<D, 1>(g, q, rho, sh, [&](const bool* valid, const int* idx) {
                        bool in = valid[0] && grid_key<D>(g, idx[0], q) >= v;
                        count += __popcll(__ballot(in));
                    });
                    if (count >= knn)
                        lo = mid;
                    else
                        hi = mid - 1;
                }
                tn = from_ordered_bits(lo);
            }
            double tv;  // key threshold of the support
            if (D == 4) {
                double dk = hemi ? kPi : (1.0 + eps) * (2.0 * acos(fmin(1.0, fmax(-1.0, tn))));
                if (!(delta0 > 0.0 && delta0 > dk)) dl = dk;
                if (dl >= kPi) {
                    dl = kPi;
                    st |= HAMLS_ST_HEMISPHERE;
                }
                tv = cos(0.5 * dl);
            } else {
                // T3: the threshold is (1+eps)^2 d_n^2 on d^2; a fixed radius wins
                // when it is larger than the adaptive one
                double e = 1.0 + eps;
                double e2 = e * e;
                double ck = hemi ? 3.0 : e2 * (-tn);
                double dk = sqrt(ck);
                double cc = ck;
                dl = dk;
                if (delta0 > 0.0 && delta0 > dk) {
                    dl = delta0;
                    cc = delta0 * delta0;
                }
                tv = -cc;
            }
            // member list for the assembly: when the final scan kept every key of
            // a ball that holds the support (tv >= key(r)), the members are its
            // kept keys above tv, in scan order
            if (mcnt) {
                int nm = -1;
                if (lcount >= 0 && tv >= lkr && !(st & HAMLS_ST_HEMISPHERE)) {
                    nm = 0;
                    for (int base = 0; base < lcount; base += 64) {
                        const int a = base + lane;
                        const bool in = a < lcount && buf[a] > tv;
                        const uint64_t mk = __ballot(in);
                        const int pos = nm + rank_below(mk);
                        if (in && pos < kListCap) mlist[(int64_t)j * kListCap + pos] = ibuf[a];
                        nm += __popcll(mk);
                    }
                    if (nm > kListCap) nm = -1;
                }
                if (lane == 0) mcnt[j] = nm;
            }
            if (lane == 0) {
                thr[j] = tv;
                delta[j] = dl;
                rstatus[j] = st;
            }
            tprev = tn;
            seeded = !hemi;
            continue;
        }
        if (D == 4) {
            if (dl >= kPi) {
                dl = kPi;
                st |= HAMLS_ST_HEMISPHERE;
            }
            const double c = cos(0.5 * dl);
            if (lane == 0) {
                thr[j] = c;
                delta[j] = dl;
                rstatus[j] = st;
            }
        } else if (lane == 0) {
            thr[j] = -(delta0 * delta0);
            delta[j] = delta0;
            rstatus[j] = st;
        }
    }
}

hamls_status launch_grid_radius(const Plan& P, hipStream_t s) {
    GridGeom g = make_grid_geom(P);
    double d0 = P.prm.support_radius > 0.0 ? P.prm.support_radius : 0.0;
    int knn = P.prm.knn_count > 0 ? P.prm.knn_count : 0;
    auto kern = P.dom == HAMLS_SO3 ? k_grid_radius<4> : k_grid_radius<3>;
    const int64_t groups = (P.MQ + kRadGroup - 1) / kRadGroup;
    hipLaunchKernelGGL(kern, dim3((unsigned)groups), dim3(64), 0, s, g, P.M, P.MQ, knn, P.prm.knn_eps,
                       1.005 * (1.0 + P.prm.knn_eps), d0, P.d_thr, P.d_delta, P.d_rstatus, P.d_mlist,
                       P.d_mcnt);
    HAMLS_HIP(hipGetLastError());
    return HAMLS_OK;
}

// ---------------------------------------------------------------------------
// local problem rows (Sec. 2.3) and assembly (eq. (14))
// ---------------------------------------------------------------------------

// Weight, tangent coordinates (divided by the scale) of record i for centre q.
// SO3: Im(conj(q) p) with p the stored copy (dot > 0), scale delta/2, distance
// 2 arccos(dot).  T3: min-image difference, scale delta, distance |d|.
template <int D>
__device__ __forceinline__ void grid_local(const GridGeom& g, int64_t i, const double* q, double key,
                                           double dl, int wendland, double* u, double& w) {
    if (D == 4) {
        const double x0 = g.X[i], x1 = g.X[g.cap + i], x2 = g.X[2 * g.cap + i], x3 = g.X[3 * g.cap + i];
        const double is = 2.0 / dl;
        u[0] = (q[0] * x1 - x0 * q[1] - (q[2] * x3 - q[3] * x2)) * is;
        u[1] = (q[0] * x2 - x0 * q[2] - (q[3] * x1 - q[1] * x3)) * is;
        u[2] = (q[0] * x3 - x0 * q[3] - (q[1] * x2 - q[2] * x1)) * is;
        w = wendland_phi(wendland, 2.0 * acos(fmin(key, 1.0)) / dl);
    } else {
        const double is = 1.0 / dl;
        for (int d = 0; d < 3; d++) {
            double t = g.X[d * g.cap + i] - q[d];
            u[d] = (t - rint(t)) * is;
        }
        w = wendland_phi(wendland, sqrt(-key) / dl);
    }
    if (g.nu) w *= g.nu[i];
}

// Monomials of degree <= K in 3 variables, by degree, first variable's power
// descending, then the second's.
template <int K>
__device__ __forceinline__ void monomials3(const double* u, double s, double* row) {
    double p0[K + 1], p1[K + 1], p2[K + 1];
    p0[0] = p1[0] = p2[0] = 1.0;
#pragma unroll
    for (int a = 1; a <= K; a++) {
        p0[a] = p0[a - 1] * u[0];
        p1[a] = p1[a - 1] * u[1];
        p2[a] = p2[a - 1] * u[2];
    }
    int c = 0;
#pragma unroll
    for (int l = 0; l <= K; l++)
#pragma unroll
        for (int a = l; a >= 0; a--)
#pragma unroll
            for (int b = l - a; b >= 0; b--) row[c++] = s * p0[a] * p1[b] * p2[l - a - b];
}

// Fused assembly and local solve, one grid node per block (one wave): the
// cover is scanned 64*U records per step; member rows (sqrt(w) g, sqrt(w) y)
// are staged in LDS 64 at a time and each lane owns a few Gram /
// right-hand-side entries (every lane reads valid row positions, so the
// accumulation has no branches); the entries then go to LDS for the solve
// epilogue (normalisation, Cholesky in registers, tau, c_1).
template <int D, int K, int FM, bool DD, bool SPLIT = false, bool UNIT = false>
__device__ __forceinline__ void grid_node(int j, double* rows, int* sh, const GridGeom& g, const double* __restrict__ vals, int F,
                                                int wendland, const double* __restrict__ thr,
                                                const double* __restrict__ delta, const SolveArgs& A,
                                                int32_t* __restrict__ nj,
                                                double* __restrict__ entries_out) {
    constexpr int m = (K + 1) * (K + 2) * (K + 3) / 6;
    constexpr int EG = m * (m + 1) / 2;
    constexpr int ROW = m + FM + 1;
    constexpr int KE = (EG + m * FM + 63) / 64;
    constexpr int U = FM == 1 ? 2 : 1;
    static_assert(2 * (EG + m * FM) + m <= 64 * ROW, "LDS reuse");
    // One FP64 field with at most 64 2x2 blocks (K <= 2): blocked Gram
    // accumulation with interleaved member groups, as on S2
    constexpr int PB = (m + 2) / 2;
    constexpr int NB = PB * (PB + 1) / 2;
    constexpr int GB = 64 / NB > 8 ? 8 : 64 / NB;
    constexpr bool BLK = FM == 1 && !DD && GB >= 1;
    // One FP64 field whose 2x2 blocks do not fit 64 lanes (m = 20): 3x3 blocks
    // of the 21 columns of [V | y] (28 blocks), two interleaved member groups:
    // six LDS reads feed nine FMAs (the packed-entry path: two reads per FMA)
    constexpr int P3 = (m + 3) / 3;
    constexpr int NB3 = P3 * (P3 + 1) / 2;
    constexpr int GB3 = 64 / NB3 > 8 ? 8 : 64 / NB3;
    constexpr bool BLK3 = FM == 1 && !DD && !BLK && (m + 1) % 3 == 0 && GB3 >= 2;
    constexpr int RS = BLK ? 2 * PB : (BLK3 ? m + 1 : ROW);  // LDS row stride
    static_assert(!BLK || (RS <= ROW && RS % 2 == 0 && EG + 2 * m <= 64 * ROW - GB * NB * 4), "blocked LDS");
    static_assert(!BLK3 || EG + 2 * m <= 64 * ROW - GB3 * NB3 * 9, "3x3 blocked LDS");
    const int lane = threadIdx.x;
    double q[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int d = 0; d < D; d++) q[d] = g.grid[(int64_t)D * j + d];
    const double c = thr[j], dl = delta[j];
    const int E = EG + m * F;
    int ca[KE], cb[KE];
    double acc[KE];
    dd accd[KE];
#pragma unroll
    for (int k = 0; k < KE; k++) {
        int e = lane + 64 * k;
        acc[k] = 0.0;
        accd[k] = {0.0, 0.0};
        ca[k] = 0;
        cb[k] = 0;
        if (e < EG) {
            int a = 0, rem = e;
            while (rem >= m - a) {
                rem -= m - a;
                a++;
            }
            ca[k] = a;
            cb[k] = a + rem;
        } else if (e < E) {
            int r = e - EG;
            ca[k] = r / F;
            cb[k] = m + r % F;
        }
    }
    const int grp = lane / NB, blk = lane - (lane / NB) * NB;
    int bI = 0, bJ = 0;
    {
        int rem = blk;
        while (rem >= PB - bI) {
            rem -= PB - bI;
            bI++;
        }
        bJ = bI + rem;
    }
    double a4[4] = {0.0, 0.0, 0.0, 0.0};
    const int grp3 = lane / NB3, blk3 = lane - (lane / NB3) * NB3;
    int cI = 0, cJ = 0;
    {
        int rem = blk3;
        while (rem >= P3 - cI) {
            rem -= P3 - cI;
            cI++;
        }
        cJ = cI + rem;
    }
    double a9[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int count = 0;
    auto body = [&](const bool* valid, const int* idx) {
        double kv[U], y1[U];
        // field values loaded with the coordinates, for every record of the
        // cover (one round trip less than loading the members')
#pragma unroll
        for (int u = 0; u < U; u++) y1[u] = FM == 1 ? vals[idx[u]] : 0.0;
#pragma unroll
        for (int u = 0; u < U; u++) kv[u] = grid_key<D>(g, idx[u], q);
#pragma unroll
        for (int u = 0; u < U; u++) kv[u] = valid[u] ? kv[u] : -1e300;
#pragma unroll
        for (int u = 0; u < U; u++) {
            const bool in = kv[u] > c;
            const uint64_t mk = __ballot(in);
            const int nin = __popcll(mk);
            if (nin == 0) continue;
            if (in) {
                const int i = idx[u];
                double uu[3], w;
                grid_local<D>(g, i, q, kv[u], dl, wendland, uu, w);
                const double sw = sqrt(w);
                double* row = rows + rank_below(mk) * RS;
                if (BLK && RS > m + 1) row[m + 1] = 0.0;
                monomials3<K>(uu, sw, row);
                if (FM == 1)
                    row[m] = sw * y1[u];
                else
                    for (int f = 0; f < F; f++) row[m + f] = sw * vals[(int64_t)f * g.cap + i];
            }
            __syncthreads();
            if (BLK) {
                if (grp < GB) {
                    for (int r = grp; r < nin; r += GB) {
                        const double2 x = *(const double2*)(rows + r * RS + 2 * bI);
                        const double2 y = *(const double2*)(rows + r * RS + 2 * bJ);
                        a4[0] = fma(x.x, y.x, a4[0]);
                        a4[1] = fma(x.x, y.y, a4[1]);
                        a4[2] = fma(x.y, y.x, a4[2]);
                        a4[3] = fma(x.y, y.y, a4[3]);
                    }
                }
            } else if (BLK3) {
                if (grp3 < GB3) {
                    for (int r = grp3; r < nin; r += GB3) {
                        const double* rr = rows + r * RS;
                        const double x0 = rr[3 * cI], x1 = rr[3 * cI + 1], x2 = rr[3 * cI + 2];
                        const double z0 = rr[3 * cJ], z1 = rr[3 * cJ + 1], z2 = rr[3 * cJ + 2];
                        a9[0] = fma(x0, z0, a9[0]);
                        a9[1] = fma(x0, z1, a9[1]);
                        a9[2] = fma(x0, z2, a9[2]);
                        a9[3] = fma(x1, z0, a9[3]);
                        a9[4] = fma(x1, z1, a9[4]);
                        a9[5] = fma(x1, z2, a9[5]);
                        a9[6] = fma(x2, z0, a9[6]);
                        a9[7] = fma(x2, z1, a9[7]);
                        a9[8] = fma(x2, z2, a9[8]);
                    }
                }
            } else {
#pragma unroll 2
                for (int r = 0; r < nin; r++) {
                    const double* row = rows + r * ROW;
#pragma unroll
                    for (int k = 0; k < KE; k++) {
                        if (DD)
                            dd_acc(accd[k], row[ca[k]], row[cb[k]]);
                        else
                            acc[k] = fma(row[ca[k]], row[cb[k]], acc[k]);
                    }
                }
            }
            __syncthreads();
            count += nin;
        }
    };
    // the members from the radius search's list where it left one, else a
    // scan of the ball's box cover
    const int nl = g.mcnt ? g.mcnt[j] : -1;
    if (nl >= 0)
        grid_list_scan<U>(g.mlist + (int64_t)j * kListCap, nl, body);
    else
        grid_scan<D, U>(g, q, grid_rho<D>(g, dl), sh, body);
    if (DD) {
        double* Gh = rows;
        double* Gl = rows + EG + m * FM;
#pragma unroll
        for (int k = 0; k < KE; k++) {
            int e = lane + 64 * k;
            if (e < E) {
                const dd v = fast_two_sum(accd[k].hi, accd[k].lo);
                Gh[e] = v.hi;
                Gl[e] = v.lo;
            }
        }
        __syncthreads();
        mls_dd_epilogue<m, UNIT>(Gh, Gl, rows + 2 * (EG + m * FM), count, F, j, A);
        return;
    }
    if (lane == 0) nj[j] = count;
    if (BLK3) {
        // sum the groups' 3x3 blocks (lanes < NB3), then each block's entries
        // of the upper triangle go to their packed places (y.y is not needed)
        double* part = rows + 64 * ROW - GB3 * NB3 * 9;
        if (grp3 < GB3) {
#pragma unroll
            for (int qq = 0; qq < 9; qq++) part[(grp3 * NB3 + blk3) * 9 + qq] = a9[qq];
        }
        __syncthreads();
        double s9[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        if (lane < NB3) {
            for (int g2 = 0; g2 < GB3; g2++) {
#pragma unroll
                for (int qq = 0; qq < 9; qq++) s9[qq] += part[(g2 * NB3 + lane) * 9 + qq];
            }
        }
        double* dst = SPLIT ? entries_out + (int64_t)j * E : rows;
        if (lane < NB3) {
#pragma unroll
            for (int qq = 0; qq < 9; qq++) {
                const int a = 3 * cI + qq / 3, b = 3 * cJ + qq % 3;
                if (a <= b && b <= m && a < m) {
                    const int e = b < m ? a * m - a * (a - 1) / 2 + (b - a) : EG + a;
                    dst[e] = s9[qq];
                }
            }
        }
        if (SPLIT) return;
        __syncthreads();
        mls_solve_epilogue<m>(rows, rows + EG + m * FM, count, F, j, A, entries_out);
        return;
    }
    if (BLK) {
        // sum the groups' blocks (lanes < NB), then each block's entries of
        // the upper triangle go to their packed places (y.y is not needed)
        double* part = rows + 64 * ROW - GB * NB * 4;
        if (grp < GB) {
#pragma unroll
            for (int qq = 0; qq < 4; qq++) part[(grp * NB + blk) * 4 + qq] = a4[qq];
        }
        __syncthreads();
        double s4[4] = {0.0, 0.0, 0.0, 0.0};
        if (lane < NB) {
            for (int g2 = 0; g2 < GB; g2++) {
#pragma unroll
                for (int qq = 0; qq < 4; qq++) s4[qq] += part[(g2 * NB + lane) * 4 + qq];
            }
        }
        double* dst = SPLIT ? entries_out + (int64_t)j * E : rows;
        if (lane < NB) {
#pragma unroll
            for (int qq = 0; qq < 4; qq++) {
                const int a = 2 * bI + (qq >> 1), b = 2 * bJ + (qq & 1);
                if (a <= b && b <= m && a < m) {
                    const int e = b < m ? a * m - a * (a - 1) / 2 + (b - a) : EG + a;
                    dst[e] = s4[qq];
                }
            }
        }
        if (SPLIT) return;
        __syncthreads();
        mls_solve_epilogue<m>(rows, rows + EG + m * FM, count, F, j, A, entries_out);
        return;
    }
    if (SPLIT) {
        // the solve runs in its own kernel, several nodes per wave: hand on
        // the packed Gram matrix and right-hand side (one field)
#pragma unroll
        for (int k = 0; k < KE; k++) {
            int e = lane + 64 * k;
            if (e < E) entries_out[(int64_t)j * E + e] = acc[k];
        }
        return;
    }
    double* Gs = rows;
#pragma unroll
    for (int k = 0; k < KE; k++) {
        int e = lane + 64 * k;
        if (e < E) Gs[e] = acc[k];
    }
    __syncthreads();
    mls_solve_epilogue<m>(Gs, rows + EG + m * FM, count, F, j, A, entries_out);
}


// LIST: the FP64 pass over the nodes the mixed-precision pass handed on
// (A.in_list), as the re-solve does for its list.
template <int D, int K, int FM, bool DD, bool SPLIT = false, bool UNIT = false, bool LIST = false>
__global__ __launch_bounds__(64) void k_grid_mls(GridGeom g, const double* __restrict__ vals, int F,
                                                int wendland, const double* __restrict__ thr,
                                                const double* __restrict__ delta, SolveArgs A,
                                                int32_t* __restrict__ nj,
                                                double* __restrict__ entries_out,
                                                const int32_t* __restrict__ order) {
    constexpr int m = (K + 1) * (K + 2) * (K + 3) / 6;
    constexpr int EG = m * (m + 1) / 2;
    constexpr int ROW = m + FM + 1;
    static_assert(2 * (EG + m * FM) + m <= 64 * ROW, "LDS reuse");
    __shared__ __align__(16) double rows[64 * ROW];
    __shared__ int sh[kScanLds];
    if (LIST && !DD) {
        const int n = *A.in_count;
        for (int li = blockIdx.x; li < n; li += gridDim.x) {
            grid_node<D, K, FM, false>(A.in_list[li], rows, sh, g, vals, F, wendland, thr, delta, A, nj, entries_out);
            __syncthreads();
        }
    } else if (DD) {
        // the re-solve list: a grid-stride loop over the listed nodes
        const int n = *A.in_count;
        for (int li = blockIdx.x; li < n; li += gridDim.x) {
            grid_node<D, K, FM, DD, false, UNIT>(A.in_list[li], rows, sh, g, vals, F, wendland, thr, delta, A, nj,
                                                 entries_out);
            __syncthreads();
        }
    } else {
        // grid order, or the plan's cost order (heaviest first), dealt over the XCDs
        const int jb = xcd_block(blockIdx.x, gridDim.x);
        const int j = order ? order[jb] : jb;
        grid_node<D, K, FM, DD, SPLIT>(j, rows, sh, g, vals, F, wendland, thr, delta, A, nj, entries_out);
    }
}

// Mixed precision (Rem. 2.4): FP32 Gram, FP64 refinement, or hand-off to the
// FP64 list (mixed_node_core), the members from the radius search's list or a
// scan of the ball's box cover.
template <int D, int K, int FM>
__device__ __forceinline__ void grid_mixed_node(int j, double* lds, int* sh, const GridGeom& g,
                                                const double* __restrict__ vals, int F, int wendland,
                                                const double* __restrict__ thr, const double* __restrict__ delta,
                                                const SolveArgs& A, int32_t* __restrict__ nj) {
    constexpr int m = (K + 1) * (K + 2) * (K + 3) / 6;
    constexpr int U = FM == 1 ? 2 : 1;
    double q[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int d = 0; d < D; d++) q[d] = g.grid[(int64_t)D * j + d];
    const double dl = delta[j];
    auto scan = [&](auto&& body) {
        const int nl = g.mcnt ? g.mcnt[j] : -1;
        if (nl >= 0)
            grid_list_scan<U>(g.mlist + (int64_t)j * kListCap, nl, body);
        else
            grid_scan<D, U>(g, q, grid_rho<D>(g, dl), sh, body);
    };
    auto key = [&](int i) { return grid_key<D>(g, i, q); };
    auto row = [&](int i, double kv, double* r) {
        double uu[3], w;
        grid_local<D>(g, i, q, kv, dl, wendland, uu, w);
        const double sw = sqrt(w);
        monomials3<K>(uu, sw, r);
        return sw;
    };
    mixed_node_core<m, FM, U>(j, lds, thr[j], vals, g.cap, F, A, nj, scan, key, row);
}

template <int D, int K, int FM>
__global__ __launch_bounds__(64) void k_grid_mixed(GridGeom g, const double* __restrict__ vals, int F,
                                                  int wendland, const double* __restrict__ thr,
                                                  const double* __restrict__ delta, SolveArgs A,
                                                  int32_t* __restrict__ nj, const int32_t* __restrict__ order) {
    constexpr int m = (K + 1) * (K + 2) * (K + 3) / 6;
    __shared__ double lds[MixedLayout<m, FM>::size];
    __shared__ int sh[kScanLds];
    // grid order, or the plan's cost order (heaviest first), dealt over the XCDs
    const int jb = xcd_block(blockIdx.x, gridDim.x);
    grid_mixed_node<D, K, FM>(order ? order[jb] : jb, lds, sh, g, vals, F, wendland, thr, delta, A, nj);
}

template <int D, int K>
static void grid_mixed_launch(const Plan& P, const GridGeom& g, const SolveArgs& A, const SolveArgs& B, int F,
                              int wl, hipStream_t s, const int32_t* order) {
    const dim3 grid((unsigned)P.MQ), block(64), lgrid(list_blocks(P.MQ));
    if (F == 1) {
        hipLaunchKernelGGL((k_grid_mixed<D, K, 1>), grid, block, 0, s, g, P.d_vals, F, wl, P.d_thr, P.d_delta, A,
                           P.d_nj, order);
        hipLaunchKernelGGL((k_grid_mls<D, K, 1, false, false, false, true>), lgrid, block, 0, s, g, P.d_vals, F,
                           wl, P.d_thr, P.d_delta, B, P.d_nj, P.d_entries, (const int32_t*)nullptr);
    } else {
        hipLaunchKernelGGL((k_grid_mixed<D, K, kMaxFieldsPerPass>), grid, block, 0, s, g, P.d_vals, F, wl, P.d_thr,
                           P.d_delta, A, P.d_nj, order);
        hipLaunchKernelGGL((k_grid_mls<D, K, kMaxFieldsPerPass, false, false, false, true>), lgrid, block, 0, s, g,
                           P.d_vals, F, wl, P.d_thr, P.d_delta, B, P.d_nj, P.d_entries, (const int32_t*)nullptr);
    }
}

// Mixed precision on SO3 / T3: the FP32 pass over every node (flagging nodes
// for FP64), then the FP64 assembly over the flagged list (which flags its
// own ill-conditioned nodes for the double-double re-solve).
hamls_status launch_grid_mixed(const Plan& P, int F, int f0, double* grid_values, hipStream_t s, int form) {
    GridGeom g = make_grid_geom(P);
    if (form < 0) form = P.asm_queue_blocks;
    const int32_t* order = form == 1 ? P.d_order : nullptr;
    SolveArgs A = make_solve_args(P, F, f0, grid_values);
    SolveArgs B = A;
    A.rs_list = P.d_mx_list;
    A.rs_count = P.d_rs_count + 1;
    B.in_list = P.d_mx_list;
    B.in_count = P.d_rs_count + 1;
    const int wl = P.prm.wendland;
#define HAMLS_GMIX_D(KK)                                               \
    if (P.dom == HAMLS_SO3)                                            \
        grid_mixed_launch<4, KK>(P, g, A, B, F, wl, s, order);         \
    else                                                               \
        grid_mixed_launch<3, KK>(P, g, A, B, F, wl, s, order);
    switch (P.K) {
        case 0: HAMLS_GMIX_D(0) break;
        case 1: HAMLS_GMIX_D(1) break;
        case 2: HAMLS_GMIX_D(2) break;
        case 3: HAMLS_GMIX_D(3) break;
        default: set_error("degree %d unsupported on SO(3)/T3", P.K); return HAMLS_ERR_UNSUPPORTED;
    }
#undef HAMLS_GMIX_D
    HAMLS_HIP(hipGetLastError());
    return HAMLS_OK;
}

// One field with m + 1 <= 16 (K <= 2): the assembly hands the Gram matrices
// to launch_split_solve (four nodes per wave).  K = 3 (m = 20) solves in
// place: handing on 230 entries a node costs more than it saves.
template <int D, int K>
static void grid_mls_launch(const Plan& P, const GridGeom& g, const SolveArgs& A, int F, int wl, hipStream_t s,
                            const int32_t* order, bool split_only) {
    constexpr int m = (K + 1) * (K + 2) * (K + 3) / 6;
    const dim3 grid((unsigned)P.MQ), block(64);
    if (F == 1 && (m + 1 <= 16 || split_only)) {
        hipLaunchKernelGGL((k_grid_mls<D, K, 1, false, true>), grid, block, 0, s, g, P.d_vals, F, wl, P.d_thr,
                           P.d_delta, A, P.d_nj, P.d_entries, order);
        return;
    }
    if (F == 1)
        hipLaunchKernelGGL((k_grid_mls<D, K, 1, false>), grid, block, 0, s, g, P.d_vals, F, wl, P.d_thr, P.d_delta,
                           A, P.d_nj, P.d_entries, order);
    else
        hipLaunchKernelGGL((k_grid_mls<D, K, kMaxFieldsPerPass, false>), grid, block, 0, s, g, P.d_vals, F, wl,
                           P.d_thr, P.d_delta, A, P.d_nj, P.d_entries, order);
}

hamls_status launch_grid_mls(const Plan& P, int F, int f0, double* grid_values, hipStream_t s, int form,
                             bool split_only) {
    GridGeom g = make_grid_geom(P);
    SolveArgs A = make_solve_args(P, F, f0, grid_values);
    int wl = P.prm.wendland;
    if (form < 0) form = P.asm_queue_blocks;
    const int32_t* order = form == 1 ? P.d_order : nullptr;
#define HAMLS_GMLS_D(KK)                                       \
    if (P.dom == HAMLS_SO3)                                    \
        grid_mls_launch<4, KK>(P, g, A, F, wl, s, order, split_only); \
    else                                                       \
        grid_mls_launch<3, KK>(P, g, A, F, wl, s, order, split_only);
    switch (P.K) {
        case 0: HAMLS_GMLS_D(0) break;
        case 1: HAMLS_GMLS_D(1) break;
        case 2: HAMLS_GMLS_D(2) break;
        case 3: HAMLS_GMLS_D(3) break;
        default: set_error("degree %d unsupported on SO(3)/T3", P.K); return HAMLS_ERR_UNSUPPORTED;
    }
#undef HAMLS_GMLS_D
    HAMLS_HIP(hipGetLastError());
    return HAMLS_OK;
}

// Re-solve of the nodes flagged by the FP64 epilogue: the same assembly in
// double-double precision, blocks striding over the list.
hamls_status launch_grid_resolve(const Plan& P, int F, int f0, double* grid_values, hipStream_t s,
                                 int unit_rhs) {
    if (P.m <= 1) return HAMLS_OK;
    GridGeom g = make_grid_geom(P);
    SolveArgs A = make_solve_args(P, F, f0, grid_values);
    dim3 grid(list_blocks(P.MQ)), block(64);
    int wl = P.prm.wendland;
#define HAMLS_GDD(DDIM, KK)                                                                          \
    if (unit_rhs)                                                                                    \
        hipLaunchKernelGGL((k_grid_mls<DDIM, KK, kMaxFieldsPerPass, true, false, true>), grid, block, 0, s, g, \
                           P.d_vals, F, wl, P.d_thr, P.d_delta, A, P.d_nj, P.d_entries, (const int32_t*)nullptr); \
    else if (F == 1)                                                                                 \
        hipLaunchKernelGGL((k_grid_mls<DDIM, KK, 1, true>), grid, block, 0, s, g, P.d_vals, F, wl,      \
                           P.d_thr, P.d_delta, A, P.d_nj, P.d_entries, (const int32_t*)nullptr);     \
    else                                                                                             \
        hipLaunchKernelGGL((k_grid_mls<DDIM, KK, kMaxFieldsPerPass, true>), grid, block, 0, s, g,       \
                           P.d_vals, F, wl, P.d_thr, P.d_delta, A, P.d_nj, P.d_entries, (const int32_t*)nullptr);
#define HAMLS_GDD_D(KK)       \
    if (P.dom == HAMLS_SO3) { \
        HAMLS_GDD(4, KK)      \
    } else {                  \
        HAMLS_GDD(3, KK)      \
    }
    switch (P.K) {
        case 1: HAMLS_GDD_D(1) break;
        case 2: HAMLS_GDD_D(2) break;
        case 3: HAMLS_GDD_D(3) break;
        default: break;
    }
#undef HAMLS_GDD_D
#undef HAMLS_GDD
    HAMLS_HIP(hipGetLastError());
    return HAMLS_OK;
}

// ---------------------------------------------------------------------------
// neighbour export (introspection)
// ---------------------------------------------------------------------------

template <int D>
__global__ __launch_bounds__(64) void k_grid_list(GridGeom g, const double* __restrict__ thr,
                                                 const double* __restrict__ delta,
                                                 const int64_t* __restrict__ row_ptr,
                                                 int32_t* __restrict__ counts, int32_t* __restrict__ idx) {
    __shared__ int sh[kScanLds];
    const int j = blockIdx.x;
    const int lane = threadIdx.x;
    double q[4] = {0.0, 0.0, 0.0, 0.0};
    for (int d = 0; d < D; d++) q[d] = g.grid[(int64_t)D * j + d];
    const double c = thr[j];
    int count = 0;
    grid_scan<D, 1>(g, q, grid_rho<D>(g, delta[j]), sh, [&](const bool* valid, const int* id) {
        bool in = valid[0] && grid_key<D>(g, id[0], q) > c;
        uint64_t mk = __ballot(in);
        if (in && idx) idx[row_ptr[j] + count + rank_below(mk)] = g.perm[id[0]];
        count += __popcll(mk);
    });
    if (lane == 0 && counts) counts[j] = count;
}

hamls_status launch_grid_list(const Plan& P, const int64_t* row_ptr, int32_t* counts, int32_t* idx,
                              hipStream_t s) {
    GridGeom g = make_grid_geom(P);
    auto kern = P.dom == HAMLS_SO3 ? k_grid_list<4> : k_grid_list<3>;
    hipLaunchKernelGGL(kern, dim3((unsigned)P.MQ), dim3(64), 0, s, g, P.d_thr, P.d_delta, row_ptr,
                       counts, idx);
    HAMLS_HIP(hipGetLastError());
    return HAMLS_OK;
}

// Values a*_i = w_i sum_a gamma_a g_a(x_i) of the generating functions
// (Rem. 2.5) at the members of grid node j, with the key, weight and tangent
// monomials formed as in the assembly (grid_key, grid_local, monomials3);
// entries in member order from row_ptr[j] (original node index perm[i] and
// value).  gamma: m x MQ.
template <int D, int K>
__global__ __launch_bounds__(64) void k_grid_gen_values(GridGeom g, int wendland, const double* __restrict__ thr,
                                                       const double* __restrict__ delta,
                                                       const double* __restrict__ gamma, int64_t MQ,
                                                       const int64_t* __restrict__ row_ptr,
                                                       const int32_t* __restrict__ perm,
                                                       int32_t* __restrict__ col, double* __restrict__ val) {
    constexpr int m = (K + 1) * (K + 2) * (K + 3) / 6;
    __shared__ int sh[kScanLds];
    const int j = xcd_block(blockIdx.x, gridDim.x);
    double q[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int d = 0; d < D; d++) q[d] = g.grid[(int64_t)D * j + d];
    const double c = thr[j], dl = delta[j];
    double gm[m];
#pragma unroll
    for (int a = 0; a < m; a++) gm[a] = gamma[(int64_t)a * MQ + j];
    const int64_t base = row_ptr[j], end = row_ptr[j + 1];
    int count = 0;
    auto body = [&](const bool* valid, const int* idx) {
        const int i = idx[0];
        const double kv = valid[0] ? grid_key<D>(g, i, q) : -1e300;
        const bool in = kv > c;
        const uint64_t mk = __ballot(in);
        if (in) {
            double uu[3], w, mono[m];
            grid_local<D>(g, i, q, kv, dl, wendland, uu, w);
            monomials3<K>(uu, 1.0, mono);
            double sum = 0.0;
#pragma unroll
            for (int a = 0; a < m; a++) sum = fma(gm[a], mono[a], sum);
            const int64_t e = base + count + rank_below(mk);
            if (e < end) {
                col[e] = perm[i];
                val[e] = w * sum;
            }
        }
        count += __popcll(mk);
    };
    const int nl = g.mcnt ? g.mcnt[j] : -1;
    if (nl >= 0)
        grid_list_scan<1>(g.mlist + (int64_t)j * kListCap, nl, body);
    else
        grid_scan<D, 1>(g, q, grid_rho<D>(g, dl), sh, body);
}

hamls_status launch_grid_gen_values(const Plan& P, hipStream_t s) {
    GridGeom g = make_grid_geom(P);
    const dim3 grid((unsigned)P.MQ), block(64);
    const int wl = P.prm.wendland;
#define HAMLS_GGV(DDIM, KK)                                                                          \
    hipLaunchKernelGGL((k_grid_gen_values<DDIM, KK>), grid, block, 0, s, g, wl, P.d_thr, P.d_delta,   \
                       P.d_gamma, P.MQ, P.d_grow, P.d_perm, P.d_gcol, P.d_gval);
#define HAMLS_GGV_D(KK)        \
    if (P.dom == HAMLS_SO3) {  \
        HAMLS_GGV(4, KK)       \
    } else {                   \
        HAMLS_GGV(3, KK)       \
    }
    switch (P.K) {
        case 0: HAMLS_GGV_D(0) break;
        case 1: HAMLS_GGV_D(1) break;
        case 2: HAMLS_GGV_D(2) break;
        case 3: HAMLS_GGV_D(3) break;
        default: set_error("degree %d unsupported on SO(3)/T3", P.K); return HAMLS_ERR_UNSUPPORTED;
    }
#undef HAMLS_GGV_D
#undef HAMLS_GGV
    HAMLS_HIP(hipGetLastError());
    return HAMLS_OK;
}

}  // namespace hamls
