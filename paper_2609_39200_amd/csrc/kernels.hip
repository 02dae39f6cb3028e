// kernels.hip -- gfx950 kernels of the HAMLS hot path (S2, FP64).
//
//   binning      cell key per node, stable LSD radix sort (8-bit digits),
//                cell offset table, gather of the sorted node records
//   radius       per grid node support radius: fixed delta_0 or the adaptive
//                radius (1+eps) d_n of eq. (12) by an exact n-th-nearest select
//   assemble     per grid node weighted Gram matrix and right-hand sides of the
//                local problem (eq. (14)) in tangent coordinates (Sec. 2.3)
//   solve        per grid node normalisation, Cholesky of C (eq. (20)),
//                centre amplification chi (eq. (19)), tau (eq. (23)) and the
//                regularized centre value c_1 of eq. (22)
//   ring DFT     step 3 of Alg. 1, the periodic-angle sums of every ring
//   Legendre     step 3, the contraction with the associated Legendre table
//   eval         synthesis of the spherical-harmonic series
#include <math.h>

#include "common.h"
#include "device_common.h"

namespace hamls {

// ---------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------

// Geometry handed to the per-grid-node kernels.
struct S2Geom {
    const double* grid;      // MQ x 3
    const double* theta;     // per ring
    const double* phi;       // per column
    int nphi;
    const double* ring_cs;   // per ring: cos(theta) = x_t, sin(theta)
    const double* col_cs;    // per column: cos(phi), sin(phi)
    const double* X;         // sorted nodes, SoA 3 x cap
    const double* nu;        // sorted node weights or null
    int64_t cap;
    const int32_t* band_off; // nb + 1
    const int32_t* cs;       // cell_start
    const int32_t* mlist;    // member lists of the radius search (kListCap per node) or null
    const int32_t* mcnt;     // their lengths, -1 where the assembly scans the cap
    const uint8_t* route;    // one-field FP64 pass: nodes sent to the re-solve unassembled, or null
    int nb;
    double dtheta, idtheta;  // band height and its reciprocal
};

// Geometry of the cell cover of a geodesic cap (thq, phq, r): the bands it
// meets and its longitude half-width.  Conservative: a margin of 1e-7 rad
// covers every rounding in the cell assignment.
struct CapGeo {
    int b0, b1;
    bool full, pole, north;
    double dphi, cq, sq, crr;
};

__device__ __forceinline__ CapGeo cap_geo(const S2Geom& g, double thq, double cq, double sq, double r) {
    const double margin = 1e-7;
    CapGeo G;
    double rr = r + margin;
    int b0 = (int)floor((thq - rr) * g.idtheta);
    int b1 = (int)floor((thq + rr) * g.idtheta);
    G.b0 = b0 < 0 ? 0 : b0;
    G.b1 = b1 > g.nb - 1 ? g.nb - 1 : b1;
    const bool north = thq - rr <= 0.0, south = thq + rr >= kPi;
    // A cap that holds a pole narrows in longitude away from it: per band the
    // half-width is largest at the band edge nearest the pole, where
    // cos(dphi) = (cos r - cos th cos thq) / (sin th sin thq)  (FP64).
    G.north = north;
    G.pole = (north != south) && rr < 0.5 * kPi;
    G.full = north || south || rr >= 0.5 * kPi;
    G.dphi = kPi;
    if (!G.full) {
        // longitude half-width asin(sin r / sin thq): a bound only, so FP32
        // with the ratio inflated by 1e-5 and 1e-5 rad added covers its error
        float sr = sinf((float)rr) / (float)sq * 1.00001f;
        if (sr >= 1.0f)
            G.full = true;
        else
            G.dphi = (double)asinf(sr) + 1e-5;
    }
    G.cq = cq;
    G.sq = sq;
    G.crr = G.pole ? cos(rr) : 0.0;
    return G;
}

// The (at most two) sector ranges [sa, sb], [sc, sd] (the second empty when
// sd < sc) of band b, ns cells, inside the cover.
__device__ __forceinline__ void band_sectors(const S2Geom& g, const CapGeo& G, int b, int ns, double phq,
                                             int& sa, int& sb, int& sc, int& sd) {
    const double margin = 1e-7;
    bool fullb = G.full;
    double dphi = G.dphi;
    if (G.pole) {
        double te = G.north ? b * g.dtheta : (b + 1) * g.dtheta;  // edge nearest the pole
        fullb = true;
        if (te > 1e-12 && te < kPi - 1e-12) {
            double A = (G.crr - cos(te) * G.cq) / (sin(te) * G.sq);
            if (A > -1.0) {
                fullb = false;
                dphi = A >= 1.0 ? margin : acos(A) + 4.0 * margin;
            }
        }
    }
    sa = 0;
    sb = ns - 1;
    sc = 0;
    sd = -1;
    if (!fullb) {
        const double spr = ns * (0.5 / kPi);  // sectors per radian
        int s0 = (int)floor((phq - dphi) * spr);
        int s1 = (int)floor((phq + dphi) * spr);
        if (s1 - s0 + 1 < ns) {
            if (s0 < 0) {
                sa = s0 + ns;
                sb = ns - 1;
                sc = 0;
                sd = s1;
            } else if (s1 >= ns) {
                sa = s0;
                sb = ns - 1;
                sc = 0;
                sd = s1 - ns;
            } else {
                sa = s0;
                sb = s1;
            }
        }
    }
}

// The (at most two) record ranges [lo1, lo1+len1), [lo2, lo2+len2) of band b
// inside the cover; off, ns: the band's first cell and cell count.
__device__ __forceinline__ void band_ranges_at(const S2Geom& g, const CapGeo& G, int b, int off, int ns,
                                               double phq, int& lo1, int& len1, int& lo2, int& len2) {
    int sa, sb, sc, sd;
    band_sectors(g, G, b, ns, phq, sa, sb, sc, sd);
    lo1 = g.cs[off + sa];
    len1 = g.cs[off + sb + 1] - lo1;
    lo2 = 0;
    len2 = 0;
    if (sd >= sc) {
        lo2 = g.cs[off + sc];
        len2 = g.cs[off + sd + 1] - lo2;
    }
}

__device__ __forceinline__ void band_ranges(const S2Geom& g, const CapGeo& G, int b, double phq,
                                            int& lo1, int& len1, int& lo2, int& len2) {
    const int off = g.band_off[b];
    band_ranges_at(g, G, b, off, g.band_off[b + 1] - off, phq, lo1, len1, lo2, len2);
}

// Radius k of the guess ladder r_k = min(base fac^k, pi/2).
__device__ __forceinline__ double ladder_radius(double base, double fac, int k) {
    double r = base;
    for (int i = 0; i < k; i++) r *= fac;
    return fmin(r, 0.5 * kPi);
}

// Approximate cover counts of the caps of the R <= 64 radii of a ladder
// around one node, in one pass of the cell table.  They only seed
// the radius search (which is exact for whatever cap it scans), so the cover
// is simplified: the bands the cap spans, each over the sectors within the
// cap's widest longitude half-width asin(sin r / sin theta_q) of the node,
// whole bands for caps that reach a pole, no rounding margin.
// Lane k first works out rung k's band range and half-width (broadcast by
// readlane); then the bands of the largest cap go one per lane, each lane
// staging its band's cell ranges for every rung in LDS (16 R bytes per lane)
// and then reading all their cell starts at once.
template <int R>
__device__ __forceinline__ void s2_ladder_counts(const S2Geom& g, double thq, double sq, double phq,
                                                 double base, double fac, int* lds, int (&cov)[R]) {
    const int lane = threadIdx.x & 63;
    const double ih = 1.0 / g.dtheta;
    // rung geometry, lane k < R: bands [kb0, kb1], half-width kdp (< 0: whole bands)
    int kb0 = 0, kb1 = -1;
    double kdp = -1.0;
    {
        const double rk = ladder_radius(base, fac, lane < R ? lane : R - 1);
        kb0 = (int)floor((thq - rk) * ih);
        kb1 = (int)floor((thq + rk) * ih);
        const float sr = sinf((float)rk) * (1.0f / (float)sq);
        if (thq - rk > 0.0 && thq + rk < kPi && sr < 1.0f) kdp = (double)asinf(sr);
    }
    int bl = __shfl(kb0, R - 1, 64), bh = __shfl(kb1, R - 1, 64);
    bl = bl < 0 ? 0 : bl;
    bh = bh > g.nb - 1 ? g.nb - 1 : bh;
    int4* cells = (int4*)lds + lane * R;
    int part[R];
#pragma unroll
    for (int k = 0; k < R; k++) part[k] = 0;
    for (int bb = bl; bb <= bh; bb += 64) {
        const int b = bb + lane;
        const bool valid = b <= bh;
        int off = 0, ns = 1;
        if (valid) {
            off = g.band_off[b];
            ns = g.band_off[b + 1] - off;
        }
        const double spr = ns * (0.5 / kPi);  // sectors per radian of longitude
#pragma unroll 1
        for (int k = 0; k < R; k++) {
            const int b0 = __builtin_amdgcn_readlane(kb0, k), b1 = __builtin_amdgcn_readlane(kb1, k);
            const double dphi = readlane_f64(kdp, k);
            int4 c = make_int4(off, off, off, off);  // empty ranges
            if (valid && b >= b0 && b <= b1) {
                c.y = off + ns;  // whole band
                if (dphi >= 0.0) {
                    const int s0 = (int)floor((phq - dphi) * spr), s1 = (int)floor((phq + dphi) * spr);
                    if (s1 - s0 + 1 < ns) {
                        if (s0 < 0) {
                            c.x = off + s0 + ns;
                            c.z = off;
                            c.w = off + s1 + 1;
                        } else if (s1 >= ns) {
                            c.x = off + s0;
                            c.z = off;
                            c.w = off + s1 - ns + 1;
                        } else {
                            c.x = off + s0;
                            c.y = off + s1 + 1;
                        }
                    }
                }
            }
            cells[k] = c;
        }
        if (valid) {
#pragma unroll
            for (int k = 0; k < R; k++) {
                const int4 c = cells[k];
                part[k] += (g.cs[c.y] - g.cs[c.x]) + (g.cs[c.w] - g.cs[c.z]);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < R; k++) cov[k] = wave_sum_int(part[k]);
}

// Visits every sorted record in the cell cover of the cap, 64*U per step: the
// lanes first enumerate up to 64 bands at once, a wave prefix sum flattens
// their ranges, and every step then hands each lane U slots of the flattened
// list (slot base + 64u + lane), so that U independent record loads per lane
// are in flight before any is used.  body(valid[U], idx[U]) is called by all
// 64 lanes in every step (idx = sorted record index, meaningful when valid),
// so body may synchronise the wave.
template <int U, class Fn>
__device__ __forceinline__ void s2_scan(const S2Geom& g, double thq, double cq, double sq, double phq,
                                        double r, int* sh, Fn&& body) {
    CapGeo G = cap_geo(g, thq, cq, sq, r);
    const int lane = threadIdx.x & 63;
    int* s_lo1 = sh;
    int* s_len1 = sh + 64;
    int* s_lo2 = sh + 128;
    int* s_pre = sh + 192;  // 65 entries
    for (int bb = G.b0; bb <= G.b1; bb += 64) {
        int b = bb + lane, lo1 = 0, len1 = 0, lo2 = 0, len2 = 0;
        if (b <= G.b1) band_ranges(g, G, b, phq, lo1, len1, lo2, len2);
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
            while (s_pre[kc + 1] <= base) kc++;  // band of the step's first slot
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
// calling convention of s2_scan.
template <int U, class Fn>
__device__ __forceinline__ void s2_list_scan(const int32_t* list, int n, Fn&& body) {
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

// The members of grid node j: the radius search's list where it left one,
// else a scan of the cap's cell cover (body sees every record of the cover).
template <int U, class Fn>
__device__ __forceinline__ void s2_members(const S2Geom& g, int j, double thq, double cq, double sq,
                                           double phq, double r, int* sh, Fn&& body) {
    const int nl = g.mcnt ? g.mcnt[j] : -1;
    if (nl >= 0)
        s2_list_scan<U>(g.mlist + (int64_t)j * kListCap, nl, body);
    else
        s2_scan<U>(g, thq, cq, sq, phq, r, sh, body);
}

// ---------------------------------------------------------------------------
// binning
// ---------------------------------------------------------------------------

__global__ void k_s2_keys(const double* __restrict__ nodes, int64_t M,
                          const int32_t* __restrict__ band_off, int nb, double dtheta,
                          uint32_t* __restrict__ keys, int32_t* __restrict__ idx) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    double x = nodes[3 * i], y = nodes[3 * i + 1], z = nodes[3 * i + 2];
    double th = acos(fmin(1.0, fmax(-1.0, z)));
    int b = (int)(th / dtheta);
    b = b < 0 ? 0 : (b > nb - 1 ? nb - 1 : b);
    double ph = atan2(y, x);
    if (ph < 0.0) ph += 2.0 * kPi;
    int off = band_off[b], ns = band_off[b + 1] - off;
    int s = (int)(ph * (ns / (2.0 * kPi)));
    s = s < 0 ? 0 : (s > ns - 1 ? ns - 1 : s);
    keys[i] = (uint32_t)(off + s);
    idx[i] = (int32_t)i;
}

hamls_status launch_s2_keys(const Plan& P, const double* nodes, int64_t M, hipStream_t s) {
    int bs = 256;
    int64_t nbk = (M + bs - 1) / bs;
    hipLaunchKernelGGL(k_s2_keys, dim3((unsigned)nbk), dim3(bs), 0, s, nodes, M, P.d_band_off,
                       P.bins.nb, P.bins.dtheta, P.d_key[0], P.d_idx[0]);
    HAMLS_HIP(hipGetLastError());
    return HAMLS_OK;
}

constexpr int RS_THREADS = 256;
constexpr int RS_TILE = kRadixTile;
constexpr int RS_ITEMS = RS_TILE / RS_THREADS;

__global__ __launch_bounds__(RS_THREADS) void k_radix_count(const uint32_t* __restrict__ keys,
                                                            int64_t n, int shift,
                                                            uint32_t* __restrict__ hist,
                                                            int nblocks) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0u;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_ITEMS; r++) {
        int64_t i = base + (int64_t)r * RS_THREADS + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of the digit-major histogram hist[d][block], first step:
// block d scans its row in place and stores the row total; each scatter block
// then scans the 256 totals into the digit bases and adds both.
__global__ __launch_bounds__(256) void k_scan_rows(uint32_t* __restrict__ hist, int nblocks,
                                                   uint32_t* __restrict__ totals) {
    __shared__ uint32_t part[256];
    uint32_t* row = hist + (int64_t)blockIdx.x * nblocks;
    const int t = threadIdx.x;
    const int chunk = (nblocks + 255) / 256;
    const int lo = t * chunk, hi = lo + chunk < nblocks ? lo + chunk : nblocks;
    uint32_t sum = 0;
    for (int i = lo; i < hi; i++) sum += row[i];
    part[t] = sum;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        uint32_t v = t >= o ? part[t - o] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t run = t > 0 ? part[t - 1] : 0u;
    for (int i = lo; i < hi; i++) {
        uint32_t v = row[i];
        row[i] = run;
        run += v;
    }
    if (t == 255) totals[blockIdx.x] = part[255];
}


// Stable scatter of one 8-bit digit.  Items of a tile are taken in rounds of
// 256 in input order; the rank of an item among equal digits is its rank in
// its wave (ballot matching on the 8 digit bits) plus the counts of the lower
// waves of the round plus everything placed by earlier rounds.
__global__ __launch_bounds__(RS_THREADS) void k_radix_scatter(
    const uint32_t* __restrict__ kin, const int32_t* __restrict__ vin, uint32_t* __restrict__ kout,
    int32_t* __restrict__ vout, int64_t n, int shift, const uint32_t* __restrict__ hist,
    int nblocks, const uint32_t* __restrict__ totals) {
    __shared__ uint32_t off[256];
    __shared__ uint32_t cnt[4][256];
    int t = threadIdx.x, w = t >> 6;
    // digit bases: every block scans the 256 digit totals itself (cheaper
    // than a kernel of its own between the row scan and the scatter)
    const uint32_t own = totals[t];
    off[t] = own;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const uint32_t v = t >= o ? off[t - o] : 0u;
        __syncthreads();
        off[t] += v;
        __syncthreads();
    }
    off[t] += hist[(int64_t)t * nblocks + blockIdx.x] - own;
    int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_ITEMS; r++) {
        int64_t i = base + (int64_t)r * RS_THREADS + t;
        bool valid = i < n;
        uint32_t key = valid ? kin[i] : 0u;
        int32_t val = valid ? vin[i] : 0;
        uint32_t d = (key >> shift) & 255u;
        cnt[0][t] = 0u;
        cnt[1][t] = 0u;
        cnt[2][t] = 0u;
        cnt[3][t] = 0u;
        __syncthreads();
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < 8; b++) {
            uint64_t mb = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? mb : ~mb;
        }
        int rank = rank_below(peers);
        if (valid && rank == 0) cnt[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t pos = off[d] + (uint32_t)rank;
            for (int w2 = 0; w2 < w; w2++) pos += cnt[w2][d];
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        off[t] += cnt[0][t] + cnt[1][t] + cnt[2][t] + cnt[3][t];
        __syncthreads();
    }
}

hamls_status radix_sort(Plan& P, int64_t M, hipStream_t s, int* final_buf) {
    int bits = P.key_bits;
    int passes = (bits + 7) / 8;
    int nblocks = (int)((M + RS_TILE - 1) / RS_TILE);
    // the last 256 entries of the histogram buffer hold the digit totals
    uint32_t* totals = P.d_hist + (P.hist_len - 256);
    if ((int64_t)nblocks * 256 > P.hist_len - 256) {
        set_error("radix histogram too small");
        return HAMLS_ERR_INVALID_ARG;
    }
    int cur = 0;
    for (int ps = 0; ps < passes; ps++) {
        int shift = 8 * ps;
        hipLaunchKernelGGL(k_radix_count, dim3(nblocks), dim3(RS_THREADS), 0, s, P.d_key[cur], M,
                           shift, P.d_hist, nblocks);
        hipLaunchKernelGGL(k_scan_rows, dim3(256), dim3(256), 0, s, P.d_hist, nblocks, totals);
        hipLaunchKernelGGL(k_radix_scatter, dim3(nblocks), dim3(RS_THREADS), 0, s, P.d_key[cur],
                           P.d_idx[cur], P.d_key[cur ^ 1], P.d_idx[cur ^ 1], M, shift, P.d_hist,
                           nblocks, totals);
        cur ^= 1;
    }
    HAMLS_HIP(hipGetLastError());
    *final_buf = cur;
    return HAMLS_OK;
}

// cell_start[c] = first sorted position whose key is >= c, for c in [0, ncells]:
// one thread per cell; the block first brackets the positions of its 256 cells
// by two binary searches, each thread then searches inside the bracket.
__device__ __forceinline__ int64_t lower_bound_key(const uint32_t* keys, int64_t lo, int64_t hi,
                                                   int64_t c) {
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if ((int64_t)keys[mid] < c)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(256) void k_cell_start(const uint32_t* __restrict__ keys, int64_t n,
                                                    int64_t ncells, int32_t* __restrict__ cs) {
    __shared__ int64_t br[2];
    const int64_t c0 = (int64_t)blockIdx.x * 256;
    if (threadIdx.x == 0) br[0] = lower_bound_key(keys, 0, n, c0);
    if (threadIdx.x == 64) br[1] = lower_bound_key(keys, 0, n, c0 + 256);
    __syncthreads();
    const int64_t c = c0 + threadIdx.x;
    if (c > ncells) return;
    cs[c] = (int32_t)lower_bound_key(keys, br[0], br[1], c);
}

// S2 cell table from the key boundaries: position i starts the cells
// keys[i-1]+1 .. keys[i] (cells before the first key start at 0, cells after
// the last at n); every cell is written once.  S2 cells along a band are few
// between two records, so the loops stay short (the 4-D SO3 grid is mostly
// empty and keeps the per-cell search).
__global__ __launch_bounds__(256) void k_cell_start_bounds(const uint32_t* __restrict__ keys, int64_t n,
                                                           int64_t ncells, int32_t* __restrict__ cs) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    const int64_t lo = i == 0 ? 0 : (int64_t)keys[i - 1] + 1;
    const int64_t hi = i == n ? ncells : (int64_t)keys[i];
    for (int64_t c = lo; c <= hi; c++) cs[c] = (int32_t)i;
}

hamls_status launch_cell_start(const Plan& P, const uint32_t* keys, int64_t M, hipStream_t s) {
    if (P.dom == HAMLS_S2) {
        const int64_t nbk = (M + 1 + 255) / 256;
        hipLaunchKernelGGL(k_cell_start_bounds, dim3((unsigned)nbk), dim3(256), 0, s, keys, M, P.ncells,
                           P.d_cell_start);
    } else {
        const int64_t nbk = (P.ncells + 1 + 255) / 256;
        hipLaunchKernelGGL(k_cell_start, dim3((unsigned)nbk), dim3(256), 0, s, keys, M, P.ncells,
                           P.d_cell_start);
    }
    HAMLS_HIP(hipGetLastError());
    return HAMLS_OK;
}

__global__ void k_gather_nodes(const int32_t* __restrict__ idx, const double* __restrict__ nodes,
                               const double* __restrict__ nu, int64_t M, int64_t cap,
                               double* __restrict__ X, double* __restrict__ NU,
                               int32_t* __restrict__ perm) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    int64_t j = idx[i];
    X[i] = nodes[3 * j];
    X[cap + i] = nodes[3 * j + 1];
    X[2 * cap + i] = nodes[3 * j + 2];
    perm[i] = (int32_t)j;
    if (nu) NU[i] = nu[j];
}

hamls_status launch_gather_nodes(const Plan& P, const int32_t* idx, const double* nodes,
                                 const double* nu, int64_t M, hipStream_t s) {
    int bs = 256;
    int64_t nbk = (M + bs - 1) / bs;
    hipLaunchKernelGGL(k_gather_nodes, dim3((unsigned)nbk), dim3(bs), 0, s, idx, nodes, nu, M,
                       P.cap, P.d_x, P.d_nu, P.d_perm);
    HAMLS_HIP(hipGetLastError());
    return HAMLS_OK;
}

__global__ void k_gather_values(const int32_t* __restrict__ perm, const double* __restrict__ values,
                                int F, int64_t ld, int64_t M, int64_t cap,
                                double* __restrict__ out, int32_t* __restrict__ rs_count) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // the solves that follow append their lists from zero ([0], [1]);
    // [2, 10) are the per-XCD node counters of the work-queue assembly
    if (i < 10) rs_count[i] = 0;
    if (i >= M) return;
    int64_t j = perm[i];
    for (int f = 0; f < F; f++) out[f * cap + i] = values[f * ld + j];
}

hamls_status launch_gather_values(const Plan& P, const double* values, int F, int f0, int64_t ld,
                                  hipStream_t s) {
    int bs = 256;
    int64_t nbk = (P.nrec + bs - 1) / bs;
    hipLaunchKernelGGL(k_gather_values, dim3((unsigned)nbk), dim3(bs), 0, s, P.d_perm,
                       values + (int64_t)f0 * ld, F, ld, P.nrec, P.cap, P.d_vals, P.d_rs_count);
    HAMLS_HIP(hipGetLastError());
    return HAMLS_OK;
}

S2Geom make_geom(const Plan& P) {
    S2Geom g;
    g.grid = P.d_grid;
    g.theta = P.d_theta;
    g.phi = P.d_phi;
    g.nphi = P.dims[1];
    g.ring_cs = P.d_ring_cs;
    g.col_cs = P.d_col_cs;
    g.X = P.d_x;
    g.nu = P.has_nu ? P.d_nu : nullptr;
    g.cap = P.cap;
    g.band_off = P.d_band_off;
    g.cs = P.d_cell_start;
    g.mlist = P.d_mlist;
    g.mcnt = P.d_mcnt;
    g.route = nullptr;
    g.nb = P.bins.nb;
    g.dtheta = P.bins.dtheta;
    g.idtheta = 1.0 / P.bins.dtheta;
    return g;
}

// ---------------------------------------------------------------------------
// support radius (eq. (5), (6), (12))
// ---------------------------------------------------------------------------

// Nearest-node distance, relative to d_n, beyond which the search predicts an
// ill-conditioned local system (C3: every centre the FP64 solve flags, and
// 17 700 of the 438 000 others, lie beyond 0.7 d_n).
constexpr double kRouteRatio = 0.7;

// The search keeps its wave-uniform state in scalar registers (uni_d): 128
// VGPRs, four waves per SIMD, with 20 spilled bytes per lane (167 VGPRs and
// three waves otherwise).
// Support radius, one grid node per block (one wave):
//  1. an initial radius from approximate cover counts of a ladder of caps
//     (cell table only, no record reads);
//  2. scan the cap, keeping the keys dot > cos r in LDS; if fewer than n,
//     grow (bracketed) and rescan; if more than kCandCap, narrow the kept key
//     range to the histogram bin of the n-th key and rescan;
//  3. the n-th largest key t_n exactly (rank count); if the search cannot be
//     narrowed (duplicates), a bitwise binary search over the key instead.
// delta = (1+eps) arccos(t_n), merged with a fixed delta_0 if both are set,
// clamped to pi/2 (the tangent projection needs delta < pi/2).
template <bool AUX, bool ROUTE>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void k_s2_radius(S2Geom g, int64_t M, int knn, double eps,
                                                 double delta0, double c_fixed, double* thr,
                                                 double* delta, uint8_t* rstatus, int32_t* mlist,
                                                 int32_t* mcnt, const int32_t* __restrict__ order,
                                                 uint8_t* route) {
    constexpr int U = 4;
    constexpr int kBinCap = 128;
    __shared__ __align__(16) double buf[kCandCap];
    __shared__ int ibuf[kCandCap];  // record of each kept key
    __shared__ __align__(16) double binbuf[kBinCap];  // also the scan histogram
    __shared__ int ohist[256];
    __shared__ int sh[kScanLds];
    // grid order, or the plan's cost order (heaviest first), dealt over the XCDs
    const int jb = xcd_block(blockIdx.x, gridDim.x);
    const int j = order ? order[jb] : jb;
    const int lane = threadIdx.x;
    // AUX: scattered points with their own angles (theta, phi, ring_cs per point)
    const int t = AUX ? j : j / g.nphi, p = AUX ? j : j - t * g.nphi;
    const double q0 = uni_d(g.grid[3 * j]), q1 = uni_d(g.grid[3 * j + 1]), q2 = uni_d(g.grid[3 * j + 2]);
    const double thq = uni_d(g.theta[t]), phq = uni_d(g.phi[p]);
    const double cq = uni_d(g.ring_cs[2 * t]), sq = uni_d(g.ring_cs[2 * t + 1]);
    uint8_t st = 0;
    double dl = delta0, c = c_fixed;
    if (knn > 0) {
        // initial radius from the density of the 3 x 3 cells around the node
        // (lanes 0-8, one cell each): the cap holding 1.44n at that density.
        // Where they hold fewer than 4 records (sparse surroundings, holes),
        // from the approximate cover counts of a ladder of caps r_k = r_0 1.6^k
        // (one pass of the cell table per 8 radii), r_0 one cell: the first
        // cap whose cover holds 3n records (in a hole, where the density sits
        // at the rim, a mean-density estimate would fall short).  Where the
        // count jumps past 8n across that step (the edge of a hole), a finer
        // ladder between r_k-1 and r_k first.
        const double* Xy = g.X + g.cap;
        const double* Xz = g.X + 2 * g.cap;
        double r = 0.5 * kPi;
        int cnt9 = 0;
        float a9 = 0.0f;
        {
            int cnt = 0;
            float ar = 0.0f;
            int bq = (int)(thq * (1.0 / g.dtheta));
            bq = bq > g.nb - 1 ? g.nb - 1 : bq;
            const int b = bq + lane / 3 - 1, ds = lane % 3 - 1;
            if (lane < 9 && b >= 0 && b < g.nb) {
                const int off = g.band_off[b], ns = g.band_off[b + 1] - off;
                const float ca = (float)(4.0 * kPi) / (float)ns * sinf((float)((b + 0.5) * g.dtheta)) *
                                 sinf((float)(0.5 * g.dtheta));
                if (ns <= 3) {
                    if (ds == 0) {
                        cnt = g.cs[off + ns] - g.cs[off];
                        ar = ns * ca;
                    }
                } else {
                    int sc = (int)(phq * (ns * (0.5 / kPi)));
                    sc = sc > ns - 1 ? ns - 1 : sc;
                    const int c = (sc + ds + ns) % ns;
                    cnt = g.cs[off + c + 1] - g.cs[off + c];
                    ar = ca;
                }
            }
            cnt9 = wave_sum_int(cnt);
            a9 = wave_sum_f32(ar);
        }
        if (cnt9 >= 4) {
            r = fmin(1.2 * sqrt((double)knn * a9 / (kPi * cnt9)), 0.5 * kPi);
        } else {
            constexpr int R = 8;
            double base = g.dtheta, fac = 1.6;
            for (int pass = 0; pass < 6; pass++) {
                int ck[R];
                s2_ladder_counts<R>(g, thq, sq, phq, base, fac, (int*)buf, ck);
                // the first radius whose cover holds 3n (counts grow with r)
                int kh = R, cs3 = 1;
#pragma unroll
                for (int k = R - 1; k >= 0; k--)
                    if (ck[k] >= 3 * knn) {
                        kh = k;
                        cs3 = ck[k];
                    }
                if (kh == R) {
                    const double rtop = ladder_radius(base, fac, R - 1);
                    if (rtop >= 0.5 * kPi) break;
                    // the next ladder in steps of 1.25 (spanning 4.8x): a pass
                    // costs the bands of its largest cap, and steps of 1.6
                    // would reach pi/2 (every band) from about 0.13 rad on
                    base = rtop * fac;
                    fac = fmin(fac, 1.25);
                    continue;
                }
                const double rh = ladder_radius(base, fac, kh);
                if (cs3 > 8 * knn && fac > 1.1 && rh < 0.5 * kPi) {
                    // refine between the previous rung and this one
                    base = kh > 0 ? ladder_radius(base, fac, kh - 1) : base / fac;
                    fac = pow(rh / base, 1.0 / R);
                    base *= fac;
                    continue;
                }
                r = rh;
                break;
            }
            __syncthreads();
        }
        // Keys at or above ktop are only counted (`above`): after a scan that
        // overflows the buffer, a 256-bin histogram of u = 1 - key over
        // [1 - ktop, 1 - cos r) locates the bin of the n-th key, and the next
        // scan keeps only that bin's keys (the range shrinks 256-fold a step).
        // A scan that finds fewer than n keys in the cap grows it from a
        // histogram of the records of the cover outside the cap (u over
        // [1 - cos r, 16 (1 - cos r))): the smallest bin edge with n records
        // of the cover inside is a radius that holds at least n.
        // The search runs on the key threshold cr = cos r of the cap.
        double cr = cos(r);
        double uh = 0.0;  // 1 - cos of a cap known to overflow the buffer
        double tn = -2.0, ktop = 2.0;
        bool done = false, hemi = false;
        int lcount = -1;  // kept keys of the final scan when it kept them all
        double lcr = 2.0;
        double kmx = -2.0;  // largest key seen: the nearest node lies in every scanned cover that holds n
        int* hist = (int*)binbuf;  // 256 ints
        for (int it = 0; it < 40 && !done; it++) {
            // cap radius for the cover: an upper bound on arccos(cr) from
            // u = 1 - cr, r = 2 asin(sqrt(u / 2)), in FP32 widened past its
            // error (the cover only has to contain the cap)
            r = (double)(2.0f * asinf(sqrtf((float)(0.5 * (1.0 - cr))))) * (1.0 + 4e-6) + 1e-7;
            const double ulo = uni_d(ktop < 2.0 ? 1.0 - ktop : 0.0);
            const double hs = uni_d(256.0 / fmax((1.0 - cr) - ulo, 1e-300));
            const double u0 = uni_d(1.0 - cr), ohs = uni_d(256.0 / fmax(15.0 * u0, 1e-300));
            r = uni_d(r);
            cr = uni_d(cr);
            ktop = uni_d(ktop);
            uh = uni_d(uh);
            tn = uni_d(tn);
            lcr = uni_d(lcr);
#pragma unroll
            for (int q = 0; q < 4; q++) {
                hist[4 * lane + q] = 0;
                ohist[4 * lane + q] = 0;
            }
            __syncthreads();
            int count = 0, above = 0, nout = 0;
            s2_scan<U>(g, thq, cq, sq, phq, r, sh, [&](const bool* valid, const int* idx) {
                double d[U];
#pragma unroll
                for (int u = 0; u < U; u++) {
                    d[u] = -2.0;
                    if (valid[u]) {
                        int i = idx[u];
                        d[u] = s2_dot(ld_rec(g.X, i), ld_rec(Xy, i), ld_rec(Xz, i), q0, q1, q2);
                    }
                    if (ROUTE) kmx = fmax(kmx, d[u]);
                }
#pragma unroll
                for (int u = 0; u < U; u++) {
                    const bool up = d[u] >= ktop;
                    const bool in = d[u] > cr && !up;
                    const bool out = valid[u] && d[u] <= cr;
                    above += __popcll(__ballot(up));
                    nout += __popcll(__ballot(out));
                    if (out) {
                        int bin = (int)((1.0 - d[u] - u0) * ohs);
                        atomicAdd(&ohist[bin < 0 ? 0 : (bin > 255 ? 255 : bin)], 1);
                    }
                    const uint64_t mk = __ballot(in);
                    const int pos = count + rank_below(mk);
                    if (in) {
                        if (pos < kCandCap) {
                            buf[pos] = d[u];
                            ibuf[pos] = idx[u];
                        } else {
                            int bin = (int)((1.0 - d[u] - ulo) * hs);
                            atomicAdd(&hist[bin < 0 ? 0 : (bin > 255 ? 255 : bin)], 1);
                        }
                    }
                    count += __popcll(mk);
                }
            });
            __syncthreads();
            if (above >= knn) {
                // rounding put the n-th key at or above ktop: drop the bound
                cr = fmin(ktop, 1.0);
                uh = 0.0;
                ktop = 2.0;
            } else if (above + count < knn) {
                if (cr <= 0.0) {
                    hemi = true;
                    done = true;
                } else {
                    const int have = above + count;
                    double nu = -1.0;  // 1 - cos of the next cap
                    if (have + nout >= knn) {
                        int before;
                        const int B = hist_select_bin(ohist, have, knn, before);
                        if (B < 255) nu = u0 * (1.0 + 15.0 * (B + 1) / 256.0);
                    }
                    if (nu < 0.0) {
                        // radius times 1.25 to 2 (u ~ r^2 / 2)
                        double grow = 1.5625 * (double)knn / (double)(have > 0 ? have : 1);
                        grow = grow < 1.5625 ? 1.5625 : (grow > 4.0 ? 4.0 : grow);
                        nu = u0 * grow;
                        if (uh > 0.0 && nu >= uh) nu = sqrt(u0 * uh);
                    } else if (uh > 0.0) {
                        nu = fmin(nu, uh);
                    }
                    cr = fmax(1.0 - nu, 0.0);
                }
            } else if (count <= kCandCap) {
                tn = nth_largest(buf, count, knn - above, cr, fmin(ktop, 1.0), sh, binbuf, kBinCap);
                done = true;
                if (ktop >= 2.0) {
                    lcount = count;  // every key above cos r is kept
                    lcr = cr;
                }
            } else {
                // bin in the histogram of every key of (cos r, ktop)
                for (int a = lane; a < kCandCap; a += 64) {
                    int bin = (int)((1.0 - buf[a] - ulo) * hs);
                    atomicAdd(&hist[bin < 0 ? 0 : (bin > 255 ? 255 : bin)], 1);
                }
                __syncthreads();
                int before;
                const int B = hist_select_bin(hist, above, knn, before);
                uh = u0;
                if (B < 255) cr = 1.0 - (ulo + (B + 1) / hs);
                if (B > 0) ktop = 1.0 - (ulo + B / hs);
            }
            __syncthreads();
        }
        if (!done) {
            // exact fallback: largest key value v with #(dot >= v) >= n, by
            // binary search over the ordered bit patterns in [cos r, 1]
            r = acos(cr);
            uint64_t lo = ordered_bits(cr), hi = ordered_bits(1.0);
            while (lo < hi) {
                uint64_t mid = lo + (hi - lo + 1) / 2;
                double v = from_ordered_bits(mid);
                int count = 0;
                s2_scan<1>(g, thq, cq, sq, phq, r, sh, [&](const bool* valid, const int* idx) {
                    bool in = false;
                    if (valid[0]) {
                        int i = idx[0];
                        in = s2_dot(g.X[i], g.X[g.cap + i], g.X[2 * g.cap + i], q0, q1, q2) >= v;
                    }
                    count += __popcll(__ballot(in));
                });
                if (count >= knn)
                    lo = mid;
                else
                    hi = mid - 1;
            }
            tn = from_ordered_bits(lo);
        }
        double dk = hemi ? kPi : (1.0 + eps) * acos(fmin(1.0, fmax(-1.0, tn)));
        if (!(delta0 > 0.0 && delta0 >= dk)) {
            dl = dk;
            if (dl >= 0.5 * kPi) {
                dl = 0.5 * kPi;
                st |= HAMLS_ST_HEMISPHERE;
            }
            c = cos(dl);
        }
        // member list for the assembly: when the final scan kept every key of
        // a cap that holds the support (c >= cos r), the members are its kept
        // keys above c, in scan order
        if (mcnt) {
            int nm = -1;
            if (lcount >= 0 && c >= lcr && !(st & HAMLS_ST_HEMISPHERE)) {
                nm = 0;
                for (int base = 0; base < lcount; base += 64) {
                    const int a = base + lane;
                    const bool in = a < lcount && buf[a] > c;
                    const uint64_t mk = __ballot(in);
                    const int pos = nm + rank_below(mk);
                    if (in && pos < kListCap) mlist[(int64_t)j * kListCap + pos] = ibuf[a];
                    nm += __popcll(mk);
                }
                if (nm > kListCap) nm = -1;
            }
            if (lane == 0) mcnt[j] = nm;
        }
        // Where even the nearest node lies beyond kRouteRatio d_n, the members
        // form a thin shell about the node (inside a hole of the node set) and
        // the local system is ill-conditioned: the one-field FP64 pass then
        // leaves the node to the double-double re-solve without assembling it
        // in FP64 first (a routing decision only: either path solves any node)
        if (ROUTE) {
            const double kmax = wave_max(kmx);
            bool rt = false;
            if (!hemi) {
                const double d0 = acos(fmin(1.0, fmax(-1.0, kmax)));
                const double dn = acos(fmin(1.0, fmax(-1.0, tn)));
                rt = d0 > kRouteRatio * dn;
            }
            if (lane == 0) route[j] = rt ? 1 : 0;
        }
    }
    if (lane == 0) {
        thr[j] = c;
        delta[j] = dl;
        rstatus[j] = st;
    }
}

// Smoothed adaptive radius (Sec. 2.2, after eq. (12)): d_n at the
// auxiliary points (delta_aux / (1 + eps)) replaced at grid node j by its
// degree-zero MLS approximation, Wendland weights of constant support rs;
// delta_j = (1 + eps) times that, clamped below pi/2 (HEMISPHERE), threshold
// cos(delta_j), members found by the assembly's scan (no list).  One wave per
// grid node.  The Fibonacci points are ordered by z (z_k = 1 - (2k+1)/n), so
// those within rs of q lie in one index range, the band of polar angles
// theta_q -/+ rs (widened by a margin and one index each way); only points
// inside the support (dot > cos rs) need the arc length.
__global__ __launch_bounds__(64) void k_s2_smooth_radius(const double* __restrict__ grid, int64_t MQ,
                                                        const double* __restrict__ aux,
                                                        const double* __restrict__ delta_aux, int naux,
                                                        double eps, double rs, double crs, int wendland,
                                                        double* __restrict__ thr, double* __restrict__ delta,
                                                        uint8_t* __restrict__ rstatus, int32_t* __restrict__ mcnt) {
    const int j = xcd_block(blockIdx.x, gridDim.x);
    const int lane = threadIdx.x;
    const double q0 = grid[3 * j], q1 = grid[3 * j + 1], q2 = grid[3 * j + 2];
    const double ie = 1.0 / (1.0 + eps);
    const double thq = acos(fmin(fmax(q2, -1.0), 1.0));
    const double z_hi = thq - rs - 1e-9 > 0.0 ? cos(thq - rs - 1e-9) : 1.0;
    const double z_lo = thq + rs + 1e-9 < kPi ? cos(thq + rs + 1e-9) : -1.0;
    const int k0 = max(0, (int)floor(0.5 * (1.0 - z_hi) * naux - 0.5) - 1);
    const int k1 = min(naux - 1, (int)ceil(0.5 * (1.0 - z_lo) * naux - 0.5) + 1);
    double sw = 0.0, sv = 0.0;
    for (int k = k0 + lane; k <= k1; k += 64) {
        const double d = s2_dot(aux[3 * k], aux[3 * k + 1], aux[3 * k + 2], q0, q1, q2);
        if (d > crs) {
            const double w = wendland_phi(wendland, acos(fmin(d, 1.0)) / rs);
            sw += w;
            sv += w * (delta_aux[k] * ie);
        }
    }
    sw = wave_sum(sw);
    sv = wave_sum(sv);
    if (lane == 0) {
        double dl = (1.0 + eps) * (sv / sw);
        uint8_t st = 0;
        if (dl >= 0.5 * kPi) {
            dl = 0.5 * kPi;
            st = HAMLS_ST_HEMISPHERE;
        }
        thr[j] = cos(dl);
        delta[j] = dl;
        rstatus[j] = st;
        if (mcnt) mcnt[j] = -1;
    }
}

hamls_status launch_s2_radius(const Plan& P, hipStream_t s, bool route) {
    S2Geom g = make_geom(P);
    double d0 = P.prm.support_radius > 0.0 ? P.prm.support_radius : 0.0;
    double cf = d0 > 0.0 ? cos(d0) : 2.0;
    int knn = P.prm.knn_count > 0 ? P.prm.knn_count : 0;
    // the cost order of the assembly (member counts at tuning) also puts the
    // search's costly nodes (large covers, holes) first
    const int32_t* order = P.asm_queue_blocks == 1 ? P.d_order : nullptr;
    if (P.prm.smooth_aux > 0) {
        // smoothed adaptive radius: d_n on the auxiliary Fibonacci grid (the
        // same search, no member lists), then its degree-zero MLS at the nodes
        S2Geom ga = g;
        ga.grid = P.d_aux;
        ga.theta = P.d_aux_theta;
        ga.phi = P.d_aux_phi;
        ga.ring_cs = P.d_aux_cs;
        ga.nphi = 1;
        ga.mlist = nullptr;
        ga.mcnt = nullptr;
        const int na = P.prm.smooth_aux;
        hipLaunchKernelGGL((k_s2_radius<true, false>), dim3((unsigned)na), dim3(64), 0, s, ga, P.M, knn, P.prm.knn_eps, 0.0,
                           2.0, P.d_aux_thr, P.d_aux_delta, P.d_aux_rst, (int32_t*)nullptr, (int32_t*)nullptr,
                           (const int32_t*)nullptr, (uint8_t*)nullptr);
        const double rs = 3.0 * sqrt(4.0 * kPi / na);
        hipLaunchKernelGGL(k_s2_smooth_radius, dim3((unsigned)P.MQ), dim3(64), 0, s, P.d_grid, P.MQ, P.d_aux,
                           P.d_aux_delta, na, P.prm.knn_eps, rs, cos(rs), P.prm.wendland, P.d_thr, P.d_delta,
                           P.d_rstatus, P.d_mcnt);
        HAMLS_HIP(hipGetLastError());
        return HAMLS_OK;
    }
    // the route flags (nearest-node distance against d_n) only when a fit
    // will route or the tuner times routing: tracking the nearest key costs
    // the search a few percent
    if (route && knn > 0 && P.d_route)
        hipLaunchKernelGGL((k_s2_radius<false, true>), dim3((unsigned)P.MQ), dim3(64), 0, s, g, P.M, knn,
                           P.prm.knn_eps, d0, cf, P.d_thr, P.d_delta, P.d_rstatus, P.d_mlist, P.d_mcnt, order,
                           P.d_route);
    else
        hipLaunchKernelGGL((k_s2_radius<false, false>), dim3((unsigned)P.MQ), dim3(64), 0, s, g, P.M, knn,
                           P.prm.knn_eps, d0, cf, P.d_thr, P.d_delta, P.d_rstatus, P.d_mlist, P.d_mcnt, order,
                           (uint8_t*)nullptr);
    HAMLS_HIP(hipGetLastError());
    return HAMLS_OK;
}

// ---------------------------------------------------------------------------
// assembly of the local problems (eq. (14)), one wave per grid node
// ---------------------------------------------------------------------------

// One-field FP64 passes: a centre the search predicts to be ill-conditioned
// is not assembled (k_route_list hands it to the re-solve list, the split
// solve skips it, the double-double pass counts its members).  A plain early
// exit: appending to the list here raised the assembly's register use.
__device__ __forceinline__ bool routed(const S2Geom& g, int j) { return g.route && g.route[j]; }

// The routed centres onto the re-solve list (one atomic per wave).
__global__ __launch_bounds__(256) void k_route_list(const uint8_t* __restrict__ route, int64_t MQ,
                                                   int32_t* __restrict__ list, int32_t* __restrict__ count) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool r = j < MQ && route[j];
    const uint64_t mk = __ballot(r);
    if (mk == 0) return;
    const int lane = threadIdx.x & 63;
    int base = 0;
    if (lane == __ffsll((unsigned long long)mk) - 1) base = atomicAdd(count, __popcll(mk));
    base = __shfl(base, __ffsll((unsigned long long)mk) - 1, 64);
    if (r) list[base + rank_below(mk)] = (int32_t)j;
}

// Entries per grid node: G_ab = sum_i w_i g_a g_b for a <= b (row-major upper
// triangle, G_00 = sum w), then h_af = sum_i w_i g_a y_if.  Candidates are
// fetched 64*U per step (U record loads per lane in flight); member rows of
// (sqrt(w) g, sqrt(w) y) are staged in LDS 64 at a time and each lane owns a
// few entries, summed over the staged rows.  FM bounds the fields of one pass.
template <int K, int FM, bool DD, bool SPLIT = false, bool UNIT = false>
__device__ __forceinline__ void s2_node(int j, double* rows, int* sh, const S2Geom& g, const double* __restrict__ vals,
                                                   int F, int wendland,
                                                   const double* __restrict__ thr,
                                                   const double* __restrict__ delta, const SolveArgs& A,
                                                   int32_t* __restrict__ nj,
                                                   double* __restrict__ entries_out) {
    constexpr int m = (K + 1) * (K + 2) / 2;
    constexpr int EG = m * (m + 1) / 2;
    constexpr int ROW = m + FM + 1;
    constexpr int KE = (EG + m * FM + 63) / 64;
    constexpr int U = FM == 1 ? 2 : 1;
    static_assert(2 * (EG + m * FM) + m <= 64 * ROW, "LDS reuse");
    // One FP64 field: lanes own 2x2 blocks of the upper triangle of the Gram
    // matrix of [V | y] (PB column pairs, NB blocks), and GB groups of lanes
    // take interleaved members: two 16-byte LDS reads feed four FMAs, and GB
    // members share each instruction.  The groups' partial sums are added in
    // group order at the end.
    constexpr int PB = (m + 2) / 2;
    constexpr int NB = PB * (PB + 1) / 2;
    constexpr int GB = 64 / NB > 8 ? 8 : 64 / NB;
    constexpr bool BLK = FM == 1 && !DD && GB >= 1;
    constexpr int RS = BLK ? 2 * PB : ROW;  // LDS row stride
    static_assert(!BLK || (RS <= ROW && RS % 2 == 0 && m * (m + 1) / 2 + 2 * m <= 64 * ROW - GB * NB * 4), "blocked LDS");
    const int lane = threadIdx.x;
    const int t = j / g.nphi, p = j - t * g.nphi;
    const double q0 = g.grid[3 * j], q1 = g.grid[3 * j + 1], q2 = g.grid[3 * j + 2];
    const double thq = g.theta[t], phq = g.phi[p];
    const double ct = g.ring_cs[2 * t], stt = g.ring_cs[2 * t + 1];
    const double cp = g.col_cs[2 * p], sp = g.col_cs[2 * p + 1];
    const double et0 = ct * cp, et1 = ct * sp, et2 = -stt;
    const double ep0 = -sp, ep1 = cp;
    const double c = thr[j], dl = delta[j];
    const double idl = 1.0 / dl;
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
    int count = 0;
    auto body = [&](const bool* valid, const int* idx) {
        double x0[U], x1[U], x2[U], d[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            x0[u] = 0.0;
            x1[u] = 0.0;
            x2[u] = 0.0;
            d[u] = -2.0;
            if (valid[u]) {
                int i = idx[u];
                x0[u] = g.X[i];
                x1[u] = g.X[g.cap + i];
                x2[u] = g.X[2 * g.cap + i];
            }
        }
        // field values and node weights loaded with the coordinates, for every
        // record of the cover (one round trip less than loading the members')
        double y1[U], nw[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            y1[u] = 0.0;
            nw[u] = 1.0;
            if (valid[u]) {
                if (FM == 1) y1[u] = vals[idx[u]];
                if (g.nu) nw[u] = g.nu[idx[u]];
            }
        }
#pragma unroll
        for (int u = 0; u < U; u++)
            if (valid[u]) d[u] = s2_dot(x0[u], x1[u], x2[u], q0, q1, q2);
#pragma unroll
        for (int u = 0; u < U; u++) {
            const bool in = d[u] > c;
            const uint64_t mk = __ballot(in);
            const int nin = __popcll(mk);
            if (nin == 0) continue;
            if (in) {
                const int i = idx[u];
                double w = wendland_phi(wendland, acos(fmin(d[u], 1.0)) * idl) * nw[u];
                double sw = sqrt(w);
                double uu = (x0[u] * et0 + x1[u] * et1 + x2[u] * et2) * idl;
                double vv = (x0[u] * ep0 + x1[u] * ep1) * idl;
                double pu[K + 1], pv[K + 1];
                pu[0] = 1.0;
                pv[0] = 1.0;
#pragma unroll
                for (int a = 1; a <= K; a++) {
                    pu[a] = pu[a - 1] * uu;
                    pv[a] = pv[a - 1] * vv;
                }
                double* row = rows + rank_below(mk) * RS;
                if (BLK && RS > m + 1) row[m + 1] = 0.0;
                int cidx = 0;
#pragma unroll
                for (int l = 0; l <= K; l++)
#pragma unroll
                    for (int b2 = 0; b2 <= l; b2++) row[cidx++] = sw * pu[l - b2] * pv[b2];
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
    s2_members<U>(g, j, thq, ct, stt, phq, dl, sh, body);
    if (DD && SPLIT) {
        // hand the double-double Gram on to the solve kernel: hi parts at
        // [0, E), lo parts at [EG + m FM, ...), the member count after them
#pragma unroll
        for (int k = 0; k < KE; k++) {
            int e = lane + 64 * k;
            if (e < E) {
                const dd v = fast_two_sum(accd[k].hi, accd[k].lo);
                entries_out[e] = v.hi;
                entries_out[EG + m * FM + e] = v.lo;
            }
        }
        if (lane == 0) {
            entries_out[2 * (EG + m * FM)] = (double)count;
            nj[j] = count;
        }
        return;
    }
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
    if (BLK) {
        // sum the groups' blocks (lanes < NB), then each block's entries of
        // the upper triangle go to their packed places (y.y is not needed)
        double* part = rows + 64 * ROW - GB * NB * 4;
        if (grp < GB) {
#pragma unroll
            for (int q = 0; q < 4; q++) part[(grp * NB + blk) * 4 + q] = a4[q];
        }
        __syncthreads();
        double s4[4] = {0.0, 0.0, 0.0, 0.0};
        if (lane < NB) {
            for (int g2 = 0; g2 < GB; g2++) {
#pragma unroll
                for (int q = 0; q < 4; q++) s4[q] += part[(g2 * NB + lane) * 4 + q];
            }
        }
        double* dst = SPLIT ? entries_out + (int64_t)j * E : rows;
        if (lane < NB) {
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const int a = 2 * bI + (q >> 1), b = 2 * bJ + (q & 1);
                if (a <= b && b <= m && a < m) {
                    const int e = b < m ? a * m - a * (a - 1) / 2 + (b - a) : EG + a;
                    dst[e] = s4[q];
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


template <int K, int FM, bool DD, bool LIST, bool SPLIT = false, bool UNIT = false>
__global__ __launch_bounds__(64) void k_s2_assemble(S2Geom g, const double* __restrict__ vals,
                                                   int F, int wendland,
                                                   const double* __restrict__ thr,
                                                   const double* __restrict__ delta, SolveArgs A,
                                                   int32_t* __restrict__ nj,
                                                   double* __restrict__ entries_out) {
    constexpr int m = (K + 1) * (K + 2) / 2;
    constexpr int EG = m * (m + 1) / 2;
    constexpr int ROW = m + FM + 1;
    static_assert(2 * (EG + m * FM) + m <= 64 * ROW, "LDS reuse");
    __shared__ __align__(16) double rows[64 * ROW];
    __shared__ int sh[kScanLds];
    if (LIST) {
        // a list of nodes (the re-solve list, or the FP64 list of the mixed
        // path): a grid-stride loop over the listed nodes
        const int n = *A.in_count;
        for (int li = blockIdx.x; li < n; li += gridDim.x) {
            s2_node<K, FM, DD, false, UNIT>(A.in_list[li], rows, sh, g, vals, F, wendland, thr, delta, A, nj,
                                            entries_out);
            __syncthreads();
        }
    } else {
        const int j = xcd_block(blockIdx.x, gridDim.x);
        if (SPLIT && FM == 1 && !DD && routed(g, j)) return;
        s2_node<K, FM, DD, SPLIT>(j, rows, sh, g, vals, F, wendland, thr, delta, A, nj, entries_out);
    }
}

// The extended-precision re-solve in two kernels over a chunk [c0, c0 + ch)
// of the re-solve list: the double-double Gram accumulation (the member scan
// and its rows, no solve registers: several waves per SIMD), then the
// double-double factorization and regularized solve from the handed-on Gram
// (per node dd_stride(m, FM) doubles of the hand-off buffer), several nodes a
// wave.
constexpr int dd_stride(int m, int FM) { return 2 * (m * (m + 1) / 2 + m * FM) + 2; }

template <int K, int FM>
__global__ __launch_bounds__(64) void k_s2_dd_gram(S2Geom g, const double* __restrict__ vals, int F, int wendland,
                                                  const double* __restrict__ thr, const double* __restrict__ delta,
                                                  SolveArgs A, int32_t* __restrict__ nj, double* __restrict__ ddg,
                                                  int64_t c0, int64_t ch) {
    constexpr int m = (K + 1) * (K + 2) / 2;
    __shared__ __align__(16) double rows[64 * (m + FM + 1)];
    __shared__ int sh[kScanLds];
    const int64_t n = *A.in_count;
    const int64_t hi = n < c0 + ch ? n : c0 + ch;
    for (int64_t li = c0 + blockIdx.x; li < hi; li += gridDim.x) {
        s2_node<K, FM, true, true>(A.in_list[li], rows, sh, g, vals, F, wendland, thr, delta, A, nj,
                                   ddg + (li - c0) * dd_stride(m, FM));
        __syncthreads();
    }
}

// Lanes per node of the double-double solve (m + F rows on a group).
constexpr int dd_group_size(int m, int FM) { return m + FM <= 16 ? 16 : (m + FM <= 32 ? 32 : 64); }

template <int m, int FM, bool UNIT>
__global__ __launch_bounds__(64) void k_dd_solve(const double* __restrict__ ddg, SolveArgs A, int F, int64_t c0,
                                                int64_t ch) {
    constexpr int EF = m * (m + 1) / 2 + m * FM;
    constexpr int GS = dd_group_size(m, FM);
    constexpr int NG = 64 / GS;
    __shared__ __align__(16) double buf[NG][2 * EF];
    const int g = threadIdx.x / GS, r = threadIdx.x % GS;
    const int E = m * (m + 1) / 2 + m * F;
    const int64_t n = *A.in_count;
    const int64_t hi = n < c0 + ch ? n : c0 + ch;
    for (int64_t b0 = c0 + (int64_t)blockIdx.x * NG; b0 < hi; b0 += (int64_t)gridDim.x * NG) {
        const int64_t li = b0 + g;
        const bool live = li < hi;
        int count = 0;
        if (live) {
            const double* src = ddg + (li - c0) * dd_stride(m, FM);
            for (int e = r; e < E; e += GS) {
                buf[g][e] = src[e];
                buf[g][EF + e] = src[EF + e];
            }
            count = (int)src[2 * EF];
        }
        __syncthreads();
        if (live) mls_dd_group<m, GS, UNIT>(buf[g], buf[g] + EF, count, F, A.in_list[li], A);
        __syncthreads();
    }
}

// Work-queue form of the one-field FP64 assembly pass (split solve): a fixed
// grid of blocks takes grid nodes, heaviest first, from the cost order.  The
// order is dealt over the 8 XCDs (node k of the order to XCD k mod 8; blocks
// are dispatched round-robin over the XCDs, so block b serves XCD b mod 8),
// with one counter per XCD: a single counter for the whole chip serialized
// its atomics (4.6x slower at C2).  The node code is the grid-order kernel's;
// each node's entries do not depend on the order.  counters[0..8) start at
// zero (reset by the value gather that precedes every pass); every block
// leaves once its XCD's share is handed out.
template <int K>
__global__ __launch_bounds__(64) void k_s2_assemble_queue(S2Geom g, const double* __restrict__ vals,
                                                         int wendland, const double* __restrict__ thr,
                                                         const double* __restrict__ delta, SolveArgs A,
                                                         int32_t* __restrict__ nj,
                                                         double* __restrict__ entries_out,
                                                         const int32_t* __restrict__ order,
                                                         int32_t* __restrict__ counters) {
    constexpr int m = (K + 1) * (K + 2) / 2;
    __shared__ __align__(16) double rows[64 * (m + 2)];
    __shared__ int sh[kScanLds];
    __shared__ int next;
    const int64_t MQ = A.MQ;
    const int x = blockIdx.x & 7;
    const int64_t share = (MQ - x + 7) / 8;  // nodes x, x + 8, ... of the order
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(counters + x, 1);
        __syncthreads();
        const int64_t k = next;
        __syncthreads();
        if (k >= share) break;
        const int j = order[8 * k + x];
        if (!routed(g, j))
            s2_node<K, 1, false, true>(j, rows, sh, g, vals, 1, wendland, thr, delta, A, nj, entries_out);
        __syncthreads();
    }
}

// Cost-ordered dispatch of the same pass: the blocks take the cost order
// through the XCD-aware mapping (runs of 64 positions per XCD); the hardware
// dispatcher starts blocks in index order as slots free up, so the heaviest
// nodes start first, with no atomics.
template <int K>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void k_s2_assemble_ordered(S2Geom g, const double* __restrict__ vals,
                                                           int wendland, const double* __restrict__ thr,
                                                           const double* __restrict__ delta, SolveArgs A,
                                                           int32_t* __restrict__ nj,
                                                           double* __restrict__ entries_out,
                                                           const int32_t* __restrict__ order) {
    constexpr int m = (K + 1) * (K + 2) / 2;
    __shared__ __align__(16) double rows[64 * (m + 2)];
    __shared__ int sh[kScanLds];
    const int j = order[xcd_block(blockIdx.x, gridDim.x)];
    if (routed(g, j)) return;
    s2_node<K, 1, false, true>(j, rows, sh, g, vals, 1, wendland, thr, delta, A, nj, entries_out);
}

// Grid nodes ordered by decreasing cost: buckets of floor(log2(n_j + 1))
// (coarse is enough for scheduling), heaviest bucket first, and grid order
// within a bucket (a stable counting sort), so that runs of the order stay
// spatially close for the XCD-aware block mapping.  Three launches over tiles
// of kTileItems grid nodes: per-tile bucket counts (bucket-major), one
// exclusive scan of that count matrix, and a stable scatter that ranks equal
// buckets by ballot matching, round by round in grid order.
__device__ __forceinline__ int cost_bucket(int32_t n) {
    const uint32_t v = (uint32_t)max(n, 0) + 1u;
    return 32 - (31 - __builtin_clz(v));  // 1..32, heavier nodes first
}

// Items i < n (n = *count when count is given, else MQ): grid node
// j = list[i] (or i), bucket of nj[j].
__global__ __launch_bounds__(256) void k_order_count(const int32_t* __restrict__ nj, int64_t MQ,
                                                     const int32_t* __restrict__ list,
                                                     const int32_t* __restrict__ count,
                                                     uint32_t* __restrict__ hist, int ntiles) {
    __shared__ uint32_t h[kOrderBuckets];
    const int t = threadIdx.x;
    if (t < kOrderBuckets) h[t] = 0u;
    __syncthreads();
    const int64_t n = count ? (int64_t)*count : MQ;
    const int64_t base = (int64_t)blockIdx.x * kTileItems;
    for (int r = 0; r < kTileItems / 256; r++) {
        const int64_t i = base + r * 256 + t;
        if (i < n) atomicAdd(&h[cost_bucket(nj[list ? list[i] : i])], 1u);
    }
    __syncthreads();
    if (t < kOrderBuckets) hist[(int64_t)t * ntiles + blockIdx.x] = h[t];
}

__global__ __launch_bounds__(256) void k_order_scatter(const int32_t* __restrict__ nj, int64_t MQ,
                                                       const int32_t* __restrict__ list,
                                                       const int32_t* __restrict__ count,
                                                       const uint32_t* __restrict__ hist, int ntiles,
                                                       int32_t* __restrict__ order) {
    __shared__ uint32_t off[kOrderBuckets];
    __shared__ uint32_t cnt[4][kOrderBuckets];
    const int t = threadIdx.x, w = t >> 6;
    if (t < kOrderBuckets) off[t] = hist[(int64_t)t * ntiles + blockIdx.x];
    const int64_t n = count ? (int64_t)*count : MQ;
    const int64_t base = (int64_t)blockIdx.x * kTileItems;
    for (int r = 0; r < kTileItems / 256; r++) {
        const int64_t i = base + r * 256 + t;
        const bool valid = i < n;
        const int32_t j = valid ? (list ? list[i] : (int32_t)i) : 0;
        const int d = valid ? cost_bucket(nj[j]) : 0;
        if (t < 4 * kOrderBuckets) cnt[t / kOrderBuckets][t % kOrderBuckets] = 0u;
        __syncthreads();
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 6; b++) {
            const uint64_t mb = __ballot((d >> b) & 1);
            peers &= ((d >> b) & 1) ? mb : ~mb;
        }
        const int rank = rank_below(peers);
        if (valid && rank == 0) cnt[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t pos = off[d] + (uint32_t)rank;
            for (int w2 = 0; w2 < w; w2++) pos += cnt[w2][d];
            order[pos] = j;
        }
        __syncthreads();
        if (t < kOrderBuckets) off[t] += cnt[0][t] + cnt[1][t] + cnt[2][t] + cnt[3][t];
        __syncthreads();
    }
}

// The items in cost order: list (or 0..MQ-1) by decreasing bucket of nj, the
// list's order within a bucket; n = *count (or MQ) items, at most MQ.
static hamls_status cost_sort(const Plan& P, const int32_t* list, const int32_t* count, int32_t* out,
                              hipStream_t s) {
    const int nt = tile_count(P.MQ);
    if (!P.d_tiles || (int64_t)kOrderBuckets * nt > P.tiles_len) {
        set_error("tile buffer too small");
        return HAMLS_ERR_INVALID_ARG;
    }
    hipLaunchKernelGGL(k_order_count, dim3(nt), dim3(256), 0, s, P.d_nj, P.MQ, list, count, P.d_tiles, nt);
    hipLaunchKernelGGL((k_exclusive_scan<uint32_t>), dim3(1), dim3(1024), 0, s, P.d_tiles,
                       (int64_t)kOrderBuckets * nt, (uint32_t*)nullptr);
    hipLaunchKernelGGL(k_order_scatter, dim3(nt), dim3(256), 0, s, P.d_nj, P.MQ, list, count, P.d_tiles, nt,
                       out);
    HAMLS_HIP(hipGetLastError());
    return HAMLS_OK;
}

hamls_status launch_cost_order(const Plan& P, hipStream_t s) {
    return cost_sort(P, nullptr, nullptr, P.d_order, s);
}

// Mixed precision, one S2 node per wave (FP32 assembly with FP64 safeguards, Rem. 2.4):
//  1. FP32 pass: member rows (sqrt(w) g, sqrt(w) y) in FP32 (membership and
//     coordinates in FP64), Gram and right-hand sides accumulated in FP32;
//  2. FP64 factorisation of the FP32 system (as in the FP64 epilogue).  A node
//     goes to the FP64 list if it is empty of structure (fewer than m members,
//     a zero column), ill-conditioned (a pivot of the unit-diagonal C below
//     1e-4, condition above ~1e4) or regularized (chi-target with chi above
//     chi_T / 2, or a fixed tau > 0): these are solved from scratch in FP64;
//  3. otherwise the FP32 solution c of the normal equations is refined once in
//     FP64: a second pass over the members forms the residual e = y_w - B c and
//     B^T e with FP64 rows, and the correction solves with the same factor.
//     The error contracts by ~ cond * 6e-8 per refinement, so one step meets
//     1e-6 for cond <= 1e4.
template <int K, int FM>
using MixedLds = MixedLayout<(K + 1) * (K + 2) / 2, FM>;

template <int K>
__device__ __forceinline__ void s2_monomials(double uu, double vv, double s, double* out) {
    double pu[K + 1], pv[K + 1];
    pu[0] = 1.0;
    pv[0] = 1.0;
#pragma unroll
    for (int a = 1; a <= K; a++) {
        pu[a] = pu[a - 1] * uu;
        pv[a] = pv[a - 1] * vv;
    }
    int c = 0;
#pragma unroll
    for (int l = 0; l <= K; l++)
#pragma unroll
        for (int b = 0; b <= l; b++) out[c++] = s * pu[l - b] * pv[b];
}

template <int K, int FM>
__device__ __forceinline__ void s2_mixed_node(int j, double* lds, int* sh, const S2Geom& g,
                                              const double* __restrict__ vals, int F, int wendland,
                                              const double* __restrict__ thr,
                                              const double* __restrict__ delta, const SolveArgs& A,
                                              int32_t* __restrict__ nj) {
    constexpr int m = (K + 1) * (K + 2) / 2;
    constexpr int U = FM == 1 ? 4 : 1;
    const int t = j / g.nphi, p = j - t * g.nphi;
    const double q0 = g.grid[3 * j], q1 = g.grid[3 * j + 1], q2 = g.grid[3 * j + 2];
    const double thq = g.theta[t], phq = g.phi[p];
    const double ct = g.ring_cs[2 * t], stt = g.ring_cs[2 * t + 1];
    const double cp = g.col_cs[2 * p], sp = g.col_cs[2 * p + 1];
    const double et0 = ct * cp, et1 = ct * sp, et2 = -stt;
    const double ep0 = -sp, ep1 = cp;
    const double dl = delta[j];
    const double idl = 1.0 / dl;
    auto scan = [&](auto&& body) { s2_members<U>(g, j, thq, ct, stt, phq, dl, sh, body); };
    auto key = [&](int i) { return s2_dot(g.X[i], g.X[g.cap + i], g.X[2 * g.cap + i], q0, q1, q2); };
    // member row in FP64: sqrt(w) g (m values); returns sqrt(w)
    auto row = [&](int i, double d, double* r) {
        const double x0 = g.X[i], x1 = g.X[g.cap + i], x2 = g.X[2 * g.cap + i];
        const double w = wendland_phi(wendland, acos(fmin(d, 1.0)) * idl) * (g.nu ? g.nu[i] : 1.0);
        const double sw = sqrt(w);
        const double uu = (x0 * et0 + x1 * et1 + x2 * et2) * idl;
        const double vv = (x0 * ep0 + x1 * ep1) * idl;
        s2_monomials<K>(uu, vv, sw, r);
        return sw;
    };
    mixed_node_core<m, FM, U>(j, lds, thr[j], vals, g.cap, F, A, nj, scan, key, row);
}

template <int K, int FM>
__global__ __launch_bounds__(64) void k_s2_mixed(S2Geom g, const double* __restrict__ vals, int F,
                                                int wendland, const double* __restrict__ thr,
                                                const double* __restrict__ delta, SolveArgs A,
                                                int32_t* __restrict__ nj, const int32_t* __restrict__ order) {
    __shared__ double lds[MixedLds<K, FM>::size];
    __shared__ int sh[kScanLds];
    // grid order, or the plan's cost order (heaviest first), dealt over the XCDs
    const int jb = xcd_block(blockIdx.x, gridDim.x);
    s2_mixed_node<K, FM>(order ? order[jb] : jb, lds, sh, g, vals, F, wendland, thr, delta, A, nj);
}

// Mixed precision: the FP32 pass over every node (flagging nodes for FP64),
// then the FP64 assembly over the flagged list (which flags its own
// ill-conditioned nodes for the double-double re-solve).
hamls_status launch_s2_mixed(const Plan& P, int F, int f0, double* grid_values, hipStream_t s, int form) {
    S2Geom g = make_geom(P);
    if (form < 0) form = P.asm_queue_blocks;
    const int32_t* order = form == 1 ? P.d_order : nullptr;
    SolveArgs A = make_solve_args(P, F, f0, grid_values);
    SolveArgs B = A;
    A.rs_list = P.d_mx_list;
    A.rs_count = P.d_rs_count + 1;
    B.in_list = P.d_mx_list;
    B.in_count = P.d_rs_count + 1;
    dim3 grid((unsigned)P.MQ), block(64);
    dim3 lgrid(list_blocks(P.MQ));
    int wl = P.prm.wendland;
#define HAMLS_MIX(KK)                                                                                  \
    if (F == 1) {                                                                                      \
        hipLaunchKernelGGL((k_s2_mixed<KK, 1>), grid, block, 0, s, g, P.d_vals, F, wl, P.d_thr, P.d_delta, A, \
                           P.d_nj, order);                                                             \
        hipLaunchKernelGGL((k_s2_assemble<KK, 1, false, true>), lgrid, block, 0, s, g, P.d_vals, F, wl,     \
                           P.d_thr, P.d_delta, B, P.d_nj, P.d_entries);                                \
    } else {                                                                                           \
        hipLaunchKernelGGL((k_s2_mixed<KK, kMaxFieldsPerPass>), grid, block, 0, s, g, P.d_vals, F, wl,     \
                           P.d_thr, P.d_delta, A, P.d_nj, order);                                      \
        hipLaunchKernelGGL((k_s2_assemble<KK, kMaxFieldsPerPass, false, true>), lgrid, block, 0, s, g,   \
                           P.d_vals, F, wl, P.d_thr, P.d_delta, B, P.d_nj, P.d_entries);               \
    }
    switch (P.K) {
        case 0: HAMLS_MIX(0) break;
        case 1: HAMLS_MIX(1) break;
        case 2: HAMLS_MIX(2) break;
        case 3: HAMLS_MIX(3) break;
        case 4: HAMLS_MIX(4) break;
        default: set_error("degree %d unsupported on S2", P.K); return HAMLS_ERR_UNSUPPORTED;
    }
#undef HAMLS_MIX
    HAMLS_HIP(hipGetLastError());
    return HAMLS_OK;
}

hamls_status launch_s2_assemble(const Plan& P, int F, int f0, double* grid_values, hipStream_t s,
                                int queue_blocks, bool route) {
    S2Geom g = make_geom(P);
    SolveArgs A = make_solve_args(P, F, f0, grid_values);
    if (route && F == 1 && P.route_valid && P.route_enabled) {
        g.route = P.d_route;
        hipLaunchKernelGGL(k_route_list, dim3((unsigned)((P.MQ + 255) / 256)), dim3(256), 0, s, P.d_route, P.MQ,
                           P.d_rs_list, P.d_rs_count);
        HAMLS_HIP(hipGetLastError());
    }
    dim3 grid((unsigned)P.MQ), block(64);
    int wl = P.prm.wendland;
    if (queue_blocks < 0) queue_blocks = P.asm_queue_blocks;
    if (queue_blocks > 1 && queue_blocks < 8) queue_blocks = 8;  // one block per XCD partition at least
    if (F == 1 && queue_blocks > 0 && P.d_order) {
        // one FP64 field in cost order: dispatch order (1) or the work queue
        // (that many blocks); the order is set by hamls_plan_tune
#define HAMLS_ASQ(KK)                                                                                   \
    if (queue_blocks == 1)                                                                              \
        hipLaunchKernelGGL((k_s2_assemble_ordered<KK>), grid, block, 0, s, g, P.d_vals, wl, P.d_thr,   \
                           P.d_delta, A, P.d_nj, P.d_entries, P.d_order);                              \
    else                                                                                                \
        hipLaunchKernelGGL((k_s2_assemble_queue<KK>), dim3((unsigned)queue_blocks), block, 0, s, g, P.d_vals, \
                           wl, P.d_thr, P.d_delta, A, P.d_nj, P.d_entries, P.d_order, P.d_rs_count + 2);
        switch (P.K) {
            case 0: HAMLS_ASQ(0) break;
            case 1: HAMLS_ASQ(1) break;
            case 2: HAMLS_ASQ(2) break;
            case 3: HAMLS_ASQ(3) break;
            case 4: HAMLS_ASQ(4) break;
            default: set_error("degree %d unsupported on S2", P.K); return HAMLS_ERR_UNSUPPORTED;
        }
#undef HAMLS_ASQ
        HAMLS_HIP(hipGetLastError());
        return HAMLS_OK;
    }
    // one field: the assembly hands the Gram matrices to launch_split_solve
#define HAMLS_ASM(KK)                                                                             \
    if (F == 1)                                                                                   \
        hipLaunchKernelGGL((k_s2_assemble<KK, 1, false, false, true>), grid, block, 0, s, g, P.d_vals, F, wl, \
                           P.d_thr, P.d_delta, A, P.d_nj, P.d_entries);                           \
    else                                                                                          \
        hipLaunchKernelGGL((k_s2_assemble<KK, kMaxFieldsPerPass, false, false>), grid, block, 0, s, g, P.d_vals, \
                           F, wl, P.d_thr, P.d_delta, A, P.d_nj, P.d_entries);
    switch (P.K) {
        case 0: HAMLS_ASM(0) break;
        case 1: HAMLS_ASM(1) break;
        case 2: HAMLS_ASM(2) break;
        case 3: HAMLS_ASM(3) break;
        case 4: HAMLS_ASM(4) break;
        default: set_error("degree %d unsupported on S2", P.K); return HAMLS_ERR_UNSUPPORTED;
    }
#undef HAMLS_ASM
    HAMLS_HIP(hipGetLastError());
    return HAMLS_OK;
}

// ---------------------------------------------------------------------------
// local solve (eq. (15)-(23))
// ---------------------------------------------------------------------------
// The solve of an assembly pass that handed on its Gram matrices (one field,
// FP64; S2 any degree, SO3/T3 m + 1 <= 16): four nodes per wave.  Nothing to
// do for the other passes, which solve in place.
bool split_solve(const Plan& P, int F) {
    if (F != 1 || (P.prm.precision != HAMLS_FP64 && !P.mixed_fp64_step2)) return false;
    return P.dom == HAMLS_S2 || P.m + 1 <= 16;
}

hamls_status launch_split_solve(const Plan& P, int F, int f0, double* grid_values, hipStream_t s,
                                bool route) {
    if (!split_solve(P, F)) return HAMLS_OK;
    SolveArgs A = make_solve_args(P, F, f0, grid_values);
    if (route && F == 1 && P.route_valid && P.route_enabled) A.route = P.d_route;
    const dim3 grid((unsigned)((P.MQ + 3) / 4)), block(64);
    const double* G = P.d_entries;
    switch (P.m) {
        case 1: hipLaunchKernelGGL((k_mls_solve<1, 16>), grid, block, 0, s, G, A); break;
        case 3: hipLaunchKernelGGL((k_mls_solve<3, 16>), grid, block, 0, s, G, A); break;
        case 4: hipLaunchKernelGGL((k_mls_solve<4, 16>), grid, block, 0, s, G, A); break;
        case 6: hipLaunchKernelGGL((k_mls_solve<6, 16>), grid, block, 0, s, G, A); break;
        case 10: hipLaunchKernelGGL((k_mls_solve<10, 16>), grid, block, 0, s, G, A); break;
        case 15: hipLaunchKernelGGL((k_mls_solve<15, 16>), grid, block, 0, s, G, A); break;
        default: set_error("no split solve for m = %d", P.m); return HAMLS_ERR_UNSUPPORTED;
    }
    HAMLS_HIP(hipGetLastError());
    return HAMLS_OK;
}


SolveArgs make_solve_args(const Plan& P, int F, int f0, double* grid_values) {
    SolveArgs A;
    A.entries = P.d_entries;
    A.MQ = P.MQ;
    A.F = F;
    A.f0 = f0;
    A.nj = P.d_nj;
    A.rstatus = P.d_rstatus;
    A.reg = P.prm.reg;
    A.tau_fixed = P.prm.tau_fixed;
    A.chi_t = P.prm.chi_target;
    A.chi_f = P.prm.chi_full;
    for (int i = 0; i < 34; i++) A.mu[i] = 0.0;
    // degree multipliers of eq. (21) in monomial order (by degree): S2 and
    // SO3 l(l+1), T3 l^2; one per monomial of degree l in D variables
    int c = 0;
    for (int l = 0; l <= P.K; l++) {
        int cnt = P.D == 2 ? l + 1 : (l + 1) * (l + 2) / 2;
        double mu = P.dom == HAMLS_T3 ? (double)l * l : (double)l * (l + 1);
        for (int b = 0; b < cnt; b++) {
            if (c > 0 && c - 1 < 34) A.mu[c - 1] = mu;
            c++;
        }
    }
    A.out = grid_values;
    A.chi = P.d_chi;
    A.tau = P.d_tau;
    A.status = P.d_status;
    A.write_diag = f0 == 0;
    A.rs_list = P.d_rs_list;
    A.rs_count = P.d_rs_count;
    A.in_list = P.d_rs_list;
    A.in_count = P.d_rs_count;
    A.route = nullptr;
    return A;
}

// Re-solve of the nodes flagged by the FP64 epilogue: the same assembly in
// double-double precision, blocks striding over the list.
// The re-solve list in chunks of the hand-off buffer (the plan's Gram
// hand-off array d_entries, free at this point of the pass): one chunk for
// one field, two for up to 16.
template <int K, int FM, bool UNIT>
static void s2_resolve_chunks(const Plan& P, const S2Geom& g, const SolveArgs& A, int F, hipStream_t s) {
    constexpr int m = (K + 1) * (K + 2) / 2;
    const int64_t cap = P.n_entries_cap * P.MQ;
    int64_t ch = cap / dd_stride(m, FM);
    ch = ch < P.MQ ? ch : P.MQ;
    const dim3 grid(list_blocks(ch)), block(64);
    const dim3 sgrid((grid.x + 64 / dd_group_size(m, FM) - 1) / (64 / dd_group_size(m, FM)));
    for (int64_t c0 = 0; c0 < P.MQ; c0 += ch) {
        hipLaunchKernelGGL((k_s2_dd_gram<K, FM>), grid, block, 0, s, g, P.d_vals, F, P.prm.wendland, P.d_thr,
                           P.d_delta, A, P.d_nj, P.d_entries, c0, ch);
        hipLaunchKernelGGL((k_dd_solve<m, FM, UNIT>), sgrid, block, 0, s, P.d_entries, A, F, c0, ch);
    }
}

hamls_status launch_s2_resolve(const Plan& P, int F, int f0, double* grid_values, hipStream_t s,
                               int unit_rhs) {
    if (P.m <= 1) return HAMLS_OK;
    S2Geom g = make_geom(P);
    SolveArgs A = make_solve_args(P, F, f0, grid_values);
    // heaviest nodes first (the list comes in the order the solve flagged
    // them; a node with thousands of members started late would trail)
    HAMLS_TRY(cost_sort(P, A.in_list, A.in_count, P.d_rs_sorted, s));
    A.in_list = P.d_rs_sorted;
#define HAMLS_DDS(KK)                                                  \
    if (unit_rhs)                                                      \
        s2_resolve_chunks<KK, kMaxFieldsPerPass, true>(P, g, A, F, s); \
    else if (F == 1)                                                   \
        s2_resolve_chunks<KK, 1, false>(P, g, A, F, s);                \
    else                                                               \
        s2_resolve_chunks<KK, kMaxFieldsPerPass, false>(P, g, A, F, s);
    switch (P.K) {
        case 1: HAMLS_DDS(1) break;
        case 2: HAMLS_DDS(2) break;
        case 3: HAMLS_DDS(3) break;
        case 4: HAMLS_DDS(4) break;
        default: break;
    }
#undef HAMLS_DDS
    HAMLS_HIP(hipGetLastError());
    return HAMLS_OK;
}

// ---------------------------------------------------------------------------
// neighbour export (introspection)
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(64) void k_s2_list(S2Geom g, const double* __restrict__ thr,
                                               const double* __restrict__ delta,
                                               const int32_t* __restrict__ perm,
                                               const int64_t* __restrict__ row_ptr,
                                               int32_t* __restrict__ counts,
                                               int32_t* __restrict__ idx) {
    int j = blockIdx.x;
    int lane = threadIdx.x;
    int t = j / g.nphi, p = j - t * g.nphi;
    double q0 = g.grid[3 * j], q1 = g.grid[3 * j + 1], q2 = g.grid[3 * j + 2];
    double c = thr[j];
    int count = 0;
    __shared__ int sh[kScanLds];
    s2_scan<1>(g, g.theta[t], g.ring_cs[2 * t], g.ring_cs[2 * t + 1], g.phi[p], delta[j], sh,
               [&](const bool* valid_, const int* idx_) {
        const bool valid = valid_[0];
        const int i = idx_[0];
        bool in = false;
        if (valid) in = s2_dot(g.X[i], g.X[g.cap + i], g.X[2 * g.cap + i], q0, q1, q2) > c;
        uint64_t mk = __ballot(in);
        if (in && idx) idx[row_ptr[j] + count + rank_below(mk)] = perm[i];
        count += __popcll(mk);
    });
    if (lane == 0 && counts) counts[j] = count;
}

hamls_status launch_s2_count(const Plan& P, int32_t* counts, hipStream_t s) {
    S2Geom g = make_geom(P);
    hipLaunchKernelGGL(k_s2_list, dim3((unsigned)P.MQ), dim3(64), 0, s, g, P.d_thr, P.d_delta,
                       P.d_perm, (const int64_t*)nullptr, counts, (int32_t*)nullptr);
    HAMLS_HIP(hipGetLastError());
    return HAMLS_OK;
}

hamls_status launch_s2_list(const Plan& P, const int64_t* row_ptr, int32_t* idx, hipStream_t s) {
    S2Geom g = make_geom(P);
    hipLaunchKernelGGL(k_s2_list, dim3((unsigned)P.MQ), dim3(64), 0, s, g, P.d_thr, P.d_delta,
                       P.d_perm, row_ptr, (int32_t*)nullptr, idx);
    HAMLS_HIP(hipGetLastError());
    return HAMLS_OK;
}

// ---------------------------------------------------------------------------
// generating functions (Rem. 2.5)
// ---------------------------------------------------------------------------

// Values a*_i = w_i sum_a gamma_a g_a(x_i) of the generating functions at the
// members of grid node j, with the weight w_i and the monomials g_a formed as
// in the assembly; entries in member order from row_ptr[j] (original node
// index perm[i] and value).  gamma: m x MQ (the derivatives of c_1 with respect to the
// right-hand side of the normal equations).
template <int K>
__global__ __launch_bounds__(64) void k_s2_gen_values(S2Geom g, int wendland, const double* __restrict__ thr,
                                                     const double* __restrict__ delta,
                                                     const double* __restrict__ gamma, int64_t MQ,
                                                     const int64_t* __restrict__ row_ptr,
                                                     const int32_t* __restrict__ perm,
                                                     int32_t* __restrict__ col, double* __restrict__ val) {
    constexpr int m = (K + 1) * (K + 2) / 2;
    __shared__ int sh[kScanLds];
    const int j = xcd_block(blockIdx.x, gridDim.x);
    const int t = j / g.nphi, p = j - t * g.nphi;
    const double q0 = g.grid[3 * j], q1 = g.grid[3 * j + 1], q2 = g.grid[3 * j + 2];
    const double thq = g.theta[t], phq = g.phi[p];
    const double ct = g.ring_cs[2 * t], stt = g.ring_cs[2 * t + 1];
    const double cp = g.col_cs[2 * p], sp = g.col_cs[2 * p + 1];
    const double et0 = ct * cp, et1 = ct * sp, et2 = -stt;
    const double ep0 = -sp, ep1 = cp;
    const double c = thr[j], dl = delta[j];
    const double idl = 1.0 / dl;
    double gm[m];
#pragma unroll
    for (int a = 0; a < m; a++) gm[a] = gamma[(int64_t)a * MQ + j];
    const int64_t base = row_ptr[j], end = row_ptr[j + 1];
    int count = 0;
    s2_members<1>(g, j, thq, ct, stt, phq, dl, sh, [&](const bool* valid, const int* idx) {
        const int i = idx[0];
        double x0 = 0.0, x1 = 0.0, x2 = 0.0, d = -2.0;
        if (valid[0]) {
            x0 = g.X[i];
            x1 = g.X[g.cap + i];
            x2 = g.X[2 * g.cap + i];
            d = s2_dot(x0, x1, x2, q0, q1, q2);
        }
        const bool in = d > c;
        const uint64_t mk = __ballot(in);
        if (in) {
            const double w = wendland_phi(wendland, acos(fmin(d, 1.0)) * idl) * (g.nu ? g.nu[i] : 1.0);
            const double uu = (x0 * et0 + x1 * et1 + x2 * et2) * idl;
            const double vv = (x0 * ep0 + x1 * ep1) * idl;
            double pu[K + 1], pv[K + 1];
            pu[0] = 1.0;
            pv[0] = 1.0;
#pragma unroll
            for (int a = 1; a <= K; a++) {
                pu[a] = pu[a - 1] * uu;
                pv[a] = pv[a - 1] * vv;
            }
            double sum = 0.0;
            int cidx = 0;
#pragma unroll
            for (int l = 0; l <= K; l++)
#pragma unroll
                for (int b2 = 0; b2 <= l; b2++) sum = fma(gm[cidx++], pu[l - b2] * pv[b2], sum);
            const int64_t e = base + count + rank_below(mk);
            if (e < end) {
                col[e] = perm[i];
                val[e] = w * sum;
            }
        }
        count += __popcll(mk);
    });
}

hamls_status launch_s2_gen_values(const Plan& P, hipStream_t s) {
    S2Geom g = make_geom(P);
    const dim3 grid((unsigned)P.MQ), block(64);
    const int wl = P.prm.wendland;
#define HAMLS_GENV(KK)                                                                                 \
    hipLaunchKernelGGL((k_s2_gen_values<KK>), grid, block, 0, s, g, wl, P.d_thr, P.d_delta, P.d_gamma, \
                       P.MQ, P.d_grow, P.d_perm, P.d_gcol, P.d_gval);
    switch (P.K) {
        case 0: HAMLS_GENV(0) break;
        case 1: HAMLS_GENV(1) break;
        case 2: HAMLS_GENV(2) break;
        case 3: HAMLS_GENV(3) break;
        case 4: HAMLS_GENV(4) break;
        default: set_error("degree %d unsupported on S2", P.K); return HAMLS_ERR_UNSUPPORTED;
    }
#undef HAMLS_GENV
    HAMLS_HIP(hipGetLastError());
    return HAMLS_OK;
}

// ---------------------------------------------------------------------------
// step 3: ring DFT and Legendre contraction
// ---------------------------------------------------------------------------

// G[f][t][k] = (2 pi / n_phi) sum_p f(t,p) e^{-i k phi_p}, k = 0..N, one block
// per (ring, field).  Twiddles are indexed by k p mod n_phi.
__global__ __launch_bounds__(256) void k_s2_ring_dft(const double* __restrict__ gv, int64_t MQ,
                                                    int nt, int np, int N,
                                                    const double* __restrict__ tw,
                                                    double* __restrict__ G) {
    extern __shared__ double sm[];
    double* ring = sm;
    double* cs = sm + np;
    double* sn = sm + 2 * np;
    int t = blockIdx.x, f = blockIdx.y;
    for (int p = threadIdx.x; p < np; p += blockDim.x) {
        ring[p] = gv[(int64_t)f * MQ + (int64_t)t * np + p];
        cs[p] = tw[p];
        sn[p] = tw[np + p];
    }
    __syncthreads();
    double scale = 2.0 * kPi / np;
    for (int k = threadIdx.x; k <= N; k += blockDim.x) {
        double re = 0.0, im = 0.0;
        int e = 0;
        for (int p = 0; p < np; p++) {
            re = fma(ring[p], cs[e], re);
            im = fma(-ring[p], sn[e], im);
            e += k;
            if (e >= np) e -= np;
        }
        double* o = G + (((int64_t)f * nt + t) * (N + 1) + k) * 2;
        o[0] = re * scale;
        o[1] = im * scale;
    }
}

hamls_status launch_s2_ring_dft(const Plan& P, const double* gv, int F, double* G, hipStream_t s) {
    int nt = P.dims[0], np = P.dims[1];
    // ring lengths that factor into primes up to 19: FFTs of mirrored ring pairs
    if (s2_ring_fft_fits(np)) return launch_s2_ring_fft(P, gv, F, G, s);
    size_t lds = sizeof(double) * 3 * (size_t)np;
    hipLaunchKernelGGL(k_s2_ring_dft, dim3(nt, F), dim3(256), lds, s, gv, P.MQ, nt, np, P.N,
                       P.d_tw, G);
    HAMLS_HIP(hipGetLastError());
    return HAMLS_OK;
}

// fhat_{n,k} = sum_{t < ceil(nt/2)} w_t P_n^k(x_t) (G_t(k) +- G_{nt-1-t}(k)),
// the sign by the parity of n+k (P_n^k(-x) = (-1)^{n+k} P_n^k(x)); negative
// orders from fhat_{n,-k} = (-1)^k conj(fhat_{n,k}) (real fields).
// One coefficient per 8 adjacent lanes: lane p of the group sums the rings
// t = p, p + 8, ... and the group adds its partial sums.
constexpr int kLegSplit = 8;
__global__ __launch_bounds__(256) void k_s2_legendre(const double* __restrict__ tab,
                                                    const double* __restrict__ G, int nt, int N,
                                                    int F, double* __restrict__ coeffs) {
    const int64_t na = (int64_t)(N + 1) * (N + 2) / 2;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int part = (int)(gid % kLegSplit);
    const int64_t cidx = gid / kLegSplit;
    const bool live = cidx < na * F;  // whole groups share this
    const int f = live ? (int)(cidx / na) : 0;
    const int64_t id = live ? cidx - (int64_t)f * na : 0;
    int n = (int)((sqrt(8.0 * (double)id + 1.0) - 1.0) * 0.5);
    while ((int64_t)n * (n + 1) / 2 > id) n--;
    while ((int64_t)(n + 1) * (n + 2) / 2 <= id) n++;
    const int k = (int)(id - (int64_t)n * (n + 1) / 2);
    const int th = (nt + 1) / 2;
    const bool even = ((n + k) & 1) == 0;
    double re = 0.0, im = 0.0;
    if (live) {
        for (int t = part; t < th; t += kLegSplit) {
            const int t2 = nt - 1 - t;
            const double* g1 = G + (((int64_t)f * nt + t) * (N + 1) + k) * 2;
            const double* g2 = G + (((int64_t)f * nt + t2) * (N + 1) + k) * 2;
            double er, ei;
            if (t == t2) {
                er = g1[0];
                ei = g1[1];
            } else if (even) {
                er = g1[0] + g2[0];
                ei = g1[1] + g2[1];
            } else {
                er = g1[0] - g2[0];
                ei = g1[1] - g2[1];
            }
            const double pv = tab[(int64_t)t * na + id];
            re = fma(pv, er, re);
            im = fma(pv, ei, im);
        }
    }
#pragma unroll
    for (int o = 1; o < kLegSplit; o <<= 1) {
        re += __shfl_xor(re, o, 64);
        im += __shfl_xor(im, o, 64);
    }
    if (!live || part != 0) return;
    const int64_t nc = (int64_t)(N + 1) * (N + 1);
    double* o = coeffs + ((int64_t)f * nc + (int64_t)n * n + n + k) * 2;
    o[0] = re;
    o[1] = im;
    if (k > 0) {
        const double sg = (k & 1) ? -1.0 : 1.0;
        double* o2 = coeffs + ((int64_t)f * nc + (int64_t)n * n + n - k) * 2;
        o2[0] = sg * re;
        o2[1] = -sg * im;
    }
}

hamls_status launch_s2_legendre(const Plan& P, int F, const double* G, double* coeffs, hipStream_t s) {
    const int64_t na = (int64_t)(P.N + 1) * (P.N + 2) / 2;
    const int64_t tot = na * F * kLegSplit;
    const int bs = 256;
    hipLaunchKernelGGL(k_s2_legendre, dim3((unsigned)((tot + bs - 1) / bs)), dim3(bs), 0, s,
                       P.d_ptab, G, P.dims[0], P.N, F, coeffs);
    HAMLS_HIP(hipGetLastError());
    return HAMLS_OK;
}

// Step-3 table of the northern rings t < ceil(nt/2):
//   tab[t][n(n+1)/2 + k] = w_t P_n^k(x_t),
// generated on the device from the ring cosines/sines and GL weights: one
// block per order k, one thread per ring, the d^n_{k0} recurrence running
// over the degree (the same trip count on every lane of a block).
__global__ __launch_bounds__(256) void k_s2_legendre_table(const double* __restrict__ ring_cs,
                                                          const double* __restrict__ ring_w, int th,
                                                          int N, double* __restrict__ tab) {
    const int k = blockIdx.x;
    const int t = blockIdx.y * blockDim.x + threadIdx.x;
    if (t >= th) return;
    const int64_t na = (int64_t)(N + 1) * (N + 2) / 2;
    const double x = ring_cs[2 * t], s = ring_cs[2 * t + 1], w = ring_w[t];
    double* col = tab + (int64_t)t * na + k;
    double d = dk0_edge(k, s), dm = 0.0;
    for (int n = k; n <= N; n++) {
        col[(int64_t)n * (n + 1) / 2] = w * sh_norm(n) * d;
        if (n < N) {
            const double nx = dk0_next(n, k, x, d, dm);
            dm = d;
            d = nx;
        }
    }
}

hamls_status launch_s2_legendre_table(const Plan& P, hipStream_t s) {
    const int th = (P.dims[0] + 1) / 2;
    dim3 grid((unsigned)(P.N + 1), (unsigned)((th + 255) / 256));
    hipLaunchKernelGGL(k_s2_legendre_table, grid, dim3(256), 0, s, P.d_ring_cs, P.d_ring_w, th, P.N,
                       P.d_ptab);
    HAMLS_HIP(hipGetLastError());
    return HAMLS_OK;
}

// ---------------------------------------------------------------------------
// synthesis
// ---------------------------------------------------------------------------

// out[f*P + i] = Re sum_{n,k} fhat_{n,k} P_n^{|k|}(cos th) (sign) e^{ik phi};
// the Legendre functions come from the d^n_{k0} recurrence (dk0_edge,
// dk0_next) for each order k.
__global__ __launch_bounds__(128) void k_s2_eval(const double* __restrict__ coeffs, int F, int N,
                                                const double* __restrict__ pts, int64_t np,
                                                double* __restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    double x = pts[3 * i], y = pts[3 * i + 1], z = pts[3 * i + 2];
    double ct = fmin(1.0, fmax(-1.0, z));
    double st = sqrt((1.0 - ct) * (1.0 + ct));
    double ph = atan2(y, x);
    int64_t nc = (int64_t)(N + 1) * (N + 1);
    for (int f = 0; f < F; f++) {
        const double* cf = coeffs + (int64_t)f * nc * 2;
        double acc = 0.0;
        double edge = 1.0;  // d^k_{k0}, updated order by order
        for (int k = 0; k <= N; k++) {
            if (k > 0) edge *= -st * sqrt((2.0 * k - 1.0) / (2.0 * k));
            const double ck = cos(k * ph), sk = sin(k * ph);
            const double sg = (k & 1) ? -1.0 : 1.0;
            double d = edge, dm = 0.0;
            for (int n = k; n <= N; n++) {
                const double* c1 = cf + ((int64_t)n * n + n + k) * 2;
                double v = c1[0] * ck - c1[1] * sk;
                if (k > 0) {
                    const double* c2 = cf + ((int64_t)n * n + n - k) * 2;
                    v += sg * (c2[0] * ck + c2[1] * sk);
                }
                acc = fma(sh_norm(n) * d, v, acc);
                if (n < N) {
                    const double nx = dk0_next(n, k, ct, d, dm);
                    dm = d;
                    d = nx;
                }
            }
        }
        out[(int64_t)f * np + i] = acc;
    }
}

hamls_status launch_s2_eval(const Plan& P, const double* coeffs, int F, const double* pts,
                            int64_t npts, double* out, hipStream_t s) {
    int bs = 128;
    hipLaunchKernelGGL(k_s2_eval, dim3((unsigned)((npts + bs - 1) / bs)), dim3(bs), 0, s, coeffs,
                       F, P.N, pts, npts, out);
    HAMLS_HIP(hipGetLastError());
    return HAMLS_OK;
}

}  // namespace hamls
