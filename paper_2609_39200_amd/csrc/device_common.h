// device_common.h -- device helpers shared by the HIP sources of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace hamls {

// Membership key x.q in a fixed association without fused operations, so that
// the neighbour sets do not depend on instruction selection.
__device__ __forceinline__ double s2_dot(double x0, double x1, double x2, double q0, double q1,
                                         double q2) {
#pragma clang fp contract(off)
    double a = x0 * q0;
    double b = x1 * q1;
    double c = x2 * q2;
    double s = a + b;
    return s + c;
}

__device__ __forceinline__ int rank_below(uint64_t mask) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Workgroups are dealt round-robin over the 8 XCDs (each with its own L2).
// Within every group of 512 workgroups, XCD x takes the 64 consecutive work
// items [64x, 64x + 64): neighbouring grid nodes (sharing candidate records)
// stay on one L2, while expensive regions (holes) still spread over all XCDs.
// A trailing partial group keeps the identity order.
__device__ __forceinline__ int xcd_block(int bid, int nblk) {
    const int g = bid >> 9;
    if ((g + 1) << 9 > nblk) return bid;
    return (g << 9) + ((bid & 7) << 6) + ((bid >> 3) & 63);
}

// Normalised associated Legendre functions through the Wigner small-d
// functions d^n_{k0}(theta): P_n^k(cos theta) = sqrt((2n+1)/(4 pi)) d^n_{k0}
// (orthonormal on S2, Condon-Shortley phase).  The edge value is
// d^k_{k0} = prod_{j=1..k} (-sin theta) sqrt((2j-1)/(2j)), and d obeys the
// three-term recurrence in the degree
//   sqrt((n+1-k)(n+1+k)) d^{n+1} = (2n+1) cos(theta) d^n - sqrt((n-k)(n+k)) d^{n-1}.
__device__ __forceinline__ double dk0_edge(int k, double s) {
    double d = 1.0;
    for (int j = 1; j <= k; j++) d *= -s * sqrt((2.0 * j - 1.0) / (2.0 * j));
    return d;
}

__device__ __forceinline__ double dk0_next(int n, int k, double x, double d, double dm) {
    const double lo = sqrt((double)(n - k) * (double)(n + k));
    const double hi = sqrt((double)(n + 1 - k) * (double)(n + 1 + k));
    return ((2.0 * n + 1.0) * x * d - lo * dm) / hi;
}

__device__ __forceinline__ double sh_norm(int n) { return sqrt((2.0 * n + 1.0) / (4.0 * kPi)); }

__device__ __forceinline__ double wendland_phi(int which, double r) {
    if (r >= 1.0) return 0.0;
    double s = 1.0 - r;
    double s2 = s * s;
    if (which == 2) return s2 * s2 * s2 * (35.0 * r * r + 18.0 * r + 3.0);
    return s2 * s2 * (4.0 * r + 1.0);
}

__device__ __forceinline__ double wave_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Record i of a coordinate array: a 32-bit byte offset from a wave-uniform
// base (one offset register serves every coordinate array).
__device__ __forceinline__ double ld_rec(const double* base, int i) {
    return *(const double*)((const char*)base + (uint32_t)i * 8u);
}

__device__ __forceinline__ float wave_sum_f32(float v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ int wave_sum_int(int v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ int wave_incl_scan_int(int v) {
    const int lane = threadIdx.x & 63;
    for (int o = 1; o < 64; o <<= 1) {
        int t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

__device__ __forceinline__ int64_t wave_incl_scan_i64(int64_t v) {
    const int lane = threadIdx.x & 63;
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t t = __shfl_up((long long)v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// Exclusive prefix sum of v[0, n) in place by one block of 1024 threads
// (each a contiguous chunk); *total receives the sum when not null.  For the
// small per-tile count arrays of the multi-block sorts and scans.
template <class T>
__global__ __launch_bounds__(1024) void k_exclusive_scan(T* __restrict__ v, int64_t n, T* __restrict__ total) {
    __shared__ T part[1024];
    const int t = threadIdx.x;
    const int64_t chunk = (n + 1023) / 1024;
    const int64_t lo = t * chunk < n ? t * chunk : n, hi = lo + chunk < n ? lo + chunk : n;
    T own = 0;
    for (int64_t i = lo; i < hi; i++) own += v[i];
    part[t] = own;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const T x = t >= o ? part[t - o] : (T)0;
        __syncthreads();
        part[t] += x;
        __syncthreads();
    }
    T run = part[t] - own;
    for (int64_t i = lo; i < hi; i++) {
        const T x = v[i];
        v[i] = run;
        run += x;
    }
    if (t == 1023 && total) *total = part[1023];
}

// Ints of LDS one wave needs for s2_scan.
constexpr int kScanLds = 4 * 64 + 1;

// A wave-uniform double moved to scalar registers (bits unchanged).  The
// support-radius searches hold their per-node state (centre, cap, histogram
// parameters) this way, which frees the vector registers for occupancy.
__device__ __forceinline__ double uni_d(double x) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)b);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ double wave_min(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}

// n-th largest of the keys buf[0..count) (LDS, n <= count <= 64 NQ), by rank
// counting with the keys held in registers, NQ per lane.  The n-th largest
// t_n is the smallest key v with fewer than n keys strictly above it: a key at
// or above t_n has at most #(u > t_n) < n keys above it, a key below t_n has
// all the n or more keys at or above t_n above it.  One comparison per pair.
// Slots past count hold -1e300, which has count >= n keys above it.
template <int NQ>
__device__ __forceinline__ double nth_largest_regs(const double* buf, int count, int knn) {
    const int lane = threadIdx.x & 63;
    double v[NQ];
    int gt[NQ];
#pragma unroll
    for (int q = 0; q < NQ; q++) {
        v[q] = lane + 64 * q < count ? buf[lane + 64 * q] : -1e300;
        gt[q] = 0;
    }
#pragma unroll 8
    for (int b = 0; b < count; b++) {
        const double u = buf[b];
#pragma unroll
        for (int q = 0; q < NQ; q++) gt[q] += u > v[q];
    }
    double found = 1e300;
#pragma unroll
    for (int q = 0; q < NQ; q++)
        if (gt[q] < knn) found = fmin(found, v[q]);
    return wave_min(found);
}

// The bin of a 256-bin histogram (LDS, bins in decreasing key order, `above`
// keys beyond bin 0) that holds the n-th largest key: the B with
// above + C(B-1) < n <= above + C(B), C the cumulative count; before =
// above + C(B-1).  Needs above < n <= above + C(255).  Called by a whole wave.
__device__ __forceinline__ int hist_select_bin(const int* hist, int above, int knn, int& before_out) {
    const int lane = threadIdx.x & 63;
    int h4[4], s4 = 0;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        h4[q] = hist[4 * lane + q];
        s4 += h4[q];
    }
    const int incl = wave_incl_scan_int(s4);
    int before = above + incl - s4, bsel = -1, bbefore = 0;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        if (bsel < 0 && before < knn && knn <= before + h4[q]) {
            bsel = 4 * lane + q;
            bbefore = before;
        }
        before += h4[q];
    }
    const uint64_t owner = __ballot(bsel >= 0);
    const int src = __ffsll((unsigned long long)owner) - 1;
    before_out = __shfl(bbefore, src, 64);
    return __shfl(bsel, src, 64);
}

// n-th largest of buf[0..count) (LDS, n <= count), keys in [klo, khi]: rank
// count in registers for up to 64 keys (one comparison per key pair); beyond,
// a 256-bin histogram on khi - key (bins monotone in the key) selects the bin
// holding the n-th key and the rank count runs inside it (a quadratic rank
// count over all keys if that bin holds more than bincap, i.e. heavy
// duplication).  The histogram costs a few instructions per key where the
// rank count costs count / 64 per key.  hist: 256 ints, binbuf: bincap <= 128
// doubles, both LDS.  Called by a whole wave.
__device__ __forceinline__ double nth_largest(double* buf, int count, int knn, double klo, double khi,
                                              int* hist, double* binbuf, int bincap) {
    const int lane = threadIdx.x & 63;
    if (count <= 64) return nth_largest_regs<1>(buf, count, knn);
    const double scale = 256.0 / (khi - klo);
#pragma unroll
    for (int q = 0; q < 4; q++) hist[4 * lane + q] = 0;
    __syncthreads();
    for (int a = lane; a < count; a += 64) {
        int bin = (int)((khi - buf[a]) * scale);
        bin = bin < 0 ? 0 : (bin > 255 ? 255 : bin);
        atomicAdd(&hist[bin], 1);
    }
    __syncthreads();
    int bbefore;
    const int B = hist_select_bin(hist, 0, knn, bbefore);
    const int kth = knn - bbefore;  // rank inside bin B
    const int nB = hist[B];
    __syncthreads();
    if (nB <= bincap) {
        int m = 0;
        for (int base = 0; base < count; base += 64) {
            const int a = base + lane;
            bool inb = false;
            double v = 0.0;
            if (a < count) {
                v = buf[a];
                int bin = (int)((khi - v) * scale);
                bin = bin < 0 ? 0 : (bin > 255 ? 255 : bin);
                inb = bin == B;
            }
            const uint64_t mk = __ballot(inb);
            if (inb) binbuf[m + rank_below(mk)] = v;
            m += __popcll(mk);
        }
        __syncthreads();
        return nB <= 64 ? nth_largest_regs<1>(binbuf, nB, kth) : nth_largest_regs<2>(binbuf, nB, kth);
    }
    double found = 1e300;
    for (int a = lane; a < count; a += 64) {
        const double v = buf[a];
        int gt = 0;
#pragma unroll 8
        for (int b = 0; b < count; b++) gt += buf[b] > v;
        if (gt < knn) found = fmin(found, v);
    }
    return wave_min(found);
}

// Order-preserving map of doubles to unsigned integers.
__device__ __forceinline__ uint64_t ordered_bits(double v) {
    uint64_t b = (uint64_t)__double_as_longlong(v);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double from_ordered_bits(uint64_t u) {
    uint64_t b = (u >> 63) ? (u & 0x7fffffffffffffffull) : ~u;
    return __longlong_as_double((long long)b);
}


// A centre whose FP64 normal-matrix solve is not trustworthy to ~1e-10 is
// re-solved with the Gram matrix in double-double precision: Cholesky
// failure, a pivot of the unit-diagonal C below kPivResolve (condition estimate
// above 1e8), or a Schur denominator below kDenResolve.
constexpr double kPivResolve = 1e-8;
constexpr double kDenResolve = 1e-4;

// sqrt(s) and 1/sqrt(s) of a Cholesky pivot s > 0: the hardware reciprocal
// square-root estimate and two Newton steps y <- y + y (1 - s y^2) / 2 (a
// correctly rounded square root followed by a division is twice as long a
// dependent chain, and the factorization runs one pivot after another)
__device__ __forceinline__ void pivot_roots(double s, double& root, double& inv) {
    double y = __builtin_amdgcn_rsq(s);
    double e = fma(-s * y, y, 1.0);
    y = fma(0.5 * y, e, y);
    e = fma(-s * y, y, 1.0);
    y = fma(0.5 * y, e, y);
    inv = y;
    root = s * y;
}
// |R_jj| of the unit-column V at or below which V is taken as rank deficient
// (compared as the squared pivot of the unit-diagonal C).
constexpr double kRankTol = 1e-11;

// tau of eq. (22), evaluated by a whole wave (all 64 lanes active, uniform
// inputs).  Chi-target: 0 for chi <= chi_T; otherwise the tau with chi_tau =
// chi_T (eq. (23)), times the C^3 smoothstep S(t) = 35t^4 - 84t^5 + 70t^6 -
// 20t^7 of t = (chi - chi_T)/(chi_full - chi_T).  The root of r_tau = 1 -
// 1/chi_T is bracketed between 1e-16 and the first power of two where r_tau
// falls below the target (r_tau decreases in tau), then located on log tau by
// a 64-way search: each round the lanes evaluate r_tau at 64 interior points
// and the bracket shrinks to the sub-interval of the crossing, 65x per round;
// 11 rounds resolve the root beyond 64 halvings.  mu is constant over the
// monomials of one degree: one division per degree.
template <int GS>
__device__ __forceinline__ double choose_tau_grp(int reg, double chi, const double* d2, const double* mu,
                                                 int n, double tau_fixed, double chi_t, double chi_f);

__device__ __forceinline__ double choose_tau(int reg, double chi, const double* d2, const double* mu,
                                         int n, double tau_fixed, double chi_t, double chi_f) {
    return choose_tau_grp<64>(reg, chi, d2, mu, n, tau_fixed, chi_t, chi_f);
}

// a / b for 0 <= a < 2^24 and 1 <= b < 2^24, from rb = 1/b in FP32: the
// product is within one unit of the quotient, and one step each way makes it
// exact (an integer division by a value known only at run time costs several
// times as many instructions, and index arithmetic in the hot loops does one
// per element)
__device__ __forceinline__ int div_small(int a, int b, float rb) {
    int q = (int)((float)a * rb);
    if (q * b > a)
        q--;
    else if ((q + 1) * b <= a)
        q++;
    return q;
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}


// ---------------------------------------------------------------------------
// double-double arithmetic (unevaluated sums hi + lo, |lo| <= ulp(hi)/2), from
// the error-free transformations TwoSum (Knuth), FastTwoSum (Dekker) and the
// FMA form of TwoProduct; written with contraction off so that the compiler
// keeps every rounding step.
// ---------------------------------------------------------------------------
struct dd {
    double hi, lo;
};

__device__ __forceinline__ dd two_sum(double a, double b) {
#pragma clang fp contract(off)
    const double s = a + b;
    const double bb = s - a;
    const double e = (a - (s - bb)) + (b - bb);
    return {s, e};
}
__device__ __forceinline__ dd fast_two_sum(double a, double b) {
#pragma clang fp contract(off)
    const double s = a + b;
    return {s, b - (s - a)};
}
__device__ __forceinline__ dd dd_add(dd a, dd b) {
#pragma clang fp contract(off)
    const dd s = two_sum(a.hi, b.hi);
    return fast_two_sum(s.hi, s.lo + (a.lo + b.lo));
}
__device__ __forceinline__ dd dd_neg(dd a) { return {-a.hi, -a.lo}; }
__device__ __forceinline__ dd dd_mul(dd a, dd b) {
#pragma clang fp contract(off)
    const double p = a.hi * b.hi;
    double e = fma(a.hi, b.hi, -p);
    e = fma(a.hi, b.lo, e);
    e = fma(a.lo, b.hi, e);
    return fast_two_sum(p, e);
}
__device__ __forceinline__ dd dd_mul_d(dd a, double b) {
#pragma clang fp contract(off)
    const double p = a.hi * b;
    double e = fma(a.hi, b, -p);
    e = fma(a.lo, b, e);
    return fast_two_sum(p, e);
}
// 1/b: the double reciprocal and one Newton correction
__device__ __forceinline__ dd dd_recip(dd b) {
#pragma clang fp contract(off)
    const double q = 1.0 / b.hi;
    const dd r = dd_add({1.0, 0.0}, dd_neg(dd_mul_d(b, q)));
    return fast_two_sum(q, r.hi * q);
}
__device__ __forceinline__ dd dd_sqrt(dd a) {
#pragma clang fp contract(off)
    const double x = sqrt(a.hi);
    const double p = x * x;
    const dd xx = {p, fma(x, x, -p)};
    const dd r = dd_add(a, dd_neg(xx));
    return fast_two_sum(x, r.hi / (2.0 * x));
}
// acc += a b for doubles a, b (the product exactly, the sum to ~1e-32)
__device__ __forceinline__ void dd_acc(dd& acc, double a, double b) {
#pragma clang fp contract(off)
    const double p = a * b;
    const double e = fma(a, b, -p);
    const dd s = two_sum(acc.hi, p);
    acc.hi = s.hi;
    acc.lo = acc.lo + (s.lo + e);
}
__device__ __forceinline__ dd readlane_dd(dd v, int l);

// Value of lane l (wave-uniform l) of every lane's v.
__device__ __forceinline__ double readlane_f64(double v, int l) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ __forceinline__ dd readlane_dd(dd v, int l) {
    return {readlane_f64(v.hi, l), readlane_f64(v.lo, l)};
}

// Local solve of one grid node by one wave, from its assembled entries
// (eq. (15)-(23)).  Gs (LDS) holds the Gram matrix of the m weighted
// monomial columns, packed upper [a m - a(a-1)/2 + (b - a)], then the right-hand
// sides [m(m+1)/2 + a F + f]; isc (LDS, m doubles) is scratch.
//  1. normalise: unit weight sum (divide by W = G_00) and unit-norm columns;
//  2. reorder to [V | v1] and append the F right-hand-side rows; lane r holds
//     row r.  The Cholesky factor of the Gram matrix of [V | v1] is
//     [[L, 0], [d^T, rho]] with L L^T = C, d = L^{-1} b and rho^2 = 1 - |d|^2
//     = 1/chi (eq. (19), (20)); eliminated alongside, the right-hand-side rows
//     become z = L^{-1} r[1:] and omega = (r_1 - d.z)/rho.  Columns are
//     broadcast with readlane: no LDS traffic, no barriers;
//  3. with tau from eq. (23),
//       c_1 = (rho omega + sum_j d_j z_j t_j) / (rho^2 + sum_j d_j^2 t_j),
//     t_j = tau mu_j/(1 + tau mu_j): the Schur complement of the first
//     unknown of eq. (22), without the cancellation of 1 - sum d^2/(1 + tau mu).
// Fewer than m neighbours or a zero column: the tau -> infinity limit (the
// weighted mean).  A pivot of C below kPivResolve, chi < 1 by rounding or a Schur
// denominator below kDenResolve: the node goes to the re-solve list.
template <int m>
__device__ void mls_solve_epilogue(const double* Gs, double* isc, int count, int F, int j,
                                   const SolveArgs& A, double* /*unused*/) {
    constexpr int NC = m - 1;
    constexpr int EG = m * (m + 1) / 2;
    const int lane = threadIdx.x & 63;
    const int64_t MQ = A.MQ;
    const uint8_t rst = A.rstatus[j];
    const double W = Gs[0];
    auto gidx = [](int a, int b) { return a * m - a * (a - 1) / 2 + (b - a); };
    if (count == 0 || !(W > 0.0)) {
        if (lane < F) A.out[(int64_t)(A.f0 + lane) * MQ + j] = __builtin_nan("");
        if (lane == 0 && A.write_diag) {
            A.chi[j] = __builtin_nan("");
            A.tau[j] = __builtin_nan("");
            A.status[j] = rst | HAMLS_ST_EMPTY;
        }
        return;
    }
    bool degen = count < m;
    {
        double v = 1.0;
        if (lane < m) v = sqrt(Gs[gidx(lane, lane)] / W);
        if (__ballot(lane < m && !(v > 0.0))) degen = true;
        if (lane < m) isc[lane] = 1.0 / v;
    }
    if (degen) {
        if (lane < F) A.out[(int64_t)(A.f0 + lane) * MQ + j] = Gs[EG + lane] / W;
        if (lane == 0 && A.write_diag) {
            A.chi[j] = __builtin_inf();
            A.tau[j] = __builtin_inf();
            A.status[j] = rst | HAMLS_ST_UNDERDETERMINED;
        }
        return;
    }
    __syncthreads();
    // row `lane` of the normalised, reordered system; p(0) = NC, p(a) = a - 1
    double a[NC + 1];
    {
        const double iW = 1.0 / W;
        const int r = lane;
        const int ar = r >= NC ? 0 : r + 1;
        const double sr = r <= NC ? isc[ar] * iW : iW;
#pragma unroll
        for (int c = 0; c <= NC; c++) {
            const int bc = c == NC ? 0 : c + 1;
            double v = 0.0;
            if (r <= NC) {
                const int lo = ar < bc ? ar : bc, hi = ar < bc ? bc : ar;
                v = Gs[gidx(lo, hi)] * (sr * isc[bc]);
            } else if (r < NC + 1 + F) {
                v = Gs[EG + bc * F + (r - NC - 1)] * (sr * isc[bc]);
            }
            a[c] = v;
        }
    }
    bool ill = false;
    double minpiv = 1.0, s_last = 1.0;
#pragma unroll
    for (int k = 0; k <= NC; k++) {
        const double s = readlane_f64(a[k], k);
        if (k < NC) {
            minpiv = fmin(minpiv, s);
            if (!(s > 1e-300)) {
                ill = true;
                break;
            }
        } else {
            s_last = s;
            if (!(s > 0.0)) {
                ill = true;
                break;
            }
        }
        double lkk, il;
        pivot_roots(s, lkk, il);
        a[k] = lane == k ? lkk : a[k] * il;
#pragma unroll
        for (int c = k + 1; c <= NC; c++) a[c] = fma(-a[k], readlane_f64(a[k], c), a[c]);
    }
    double dv[NC > 0 ? NC : 1], d2[NC > 0 ? NC : 1], tf[NC > 0 ? NC : 1];
    double chi = 1.0, tau = 0.0, den = 1.0;
    if (!ill) {
#pragma unroll
        for (int k = 0; k < NC; k++) {
            dv[k] = readlane_f64(a[k], NC);
            d2[k] = dv[k] * dv[k];
        }
        chi = 1.0 / s_last;
        if (minpiv < kPivResolve) ill = true;
    }
    if (!ill) {
        tau = NC > 0 ? choose_tau(A.reg, chi, d2, A.mu, NC, A.tau_fixed, A.chi_t, A.chi_f) : 0.0;
        den = s_last;
        if (tau > 0.0) {
#pragma unroll
            for (int k = 0; k < NC; k++) {
                const double tm = tau * A.mu[k];
                tf[k] = tm > 0.0 ? tm / (1.0 + tm) : 0.0;
                den += d2[k] * tf[k];
            }
        } else {
#pragma unroll
            for (int k = 0; k < NC; k++) tf[k] = 0.0;
        }
        if (!(den > kDenResolve)) ill = true;
    }
    if (ill) {
        if (lane == 0) {
            const int slot = atomicAdd(A.rs_count, 1);
            A.rs_list[slot] = j;
        }
        return;
    }
    const double rho = readlane_f64(a[NC], NC);
    if (lane > NC && lane < NC + 1 + F) {
        double num = rho * a[NC];
#pragma unroll
        for (int k = 0; k < NC; k++) num += dv[k] * a[k] * tf[k];
        A.out[(int64_t)(A.f0 + lane - NC - 1) * MQ + j] = num / den;
    }
    if (lane == 0 && A.write_diag) {
        A.chi[j] = chi;
        A.tau[j] = tau;
        A.status[j] = rst | (tau > 0.0 ? HAMLS_ST_REGULARIZED : 0);
    }
}

// ---- the same solve for a group of GS lanes (GS = 16 or 32: 64 / GS nodes
// per wave; GS = 64 is mls_solve_epilogue) ---------------------------------

// Lane K of each row of 16 lanes, to the whole row (DPP row_newbcast).
template <int K>
__device__ __forceinline__ double row_bcast(double x) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), 0x150 + K, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), 0x150 + K, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// The value of x on lane k of this lane's group (k a constant after
// unrolling: the switch folds to one broadcast).
template <int GS>
__device__ __forceinline__ double grp_bcast(double x, int k) {
    if (GS == 64) return readlane_f64(x, k);
    if (GS == 16) {
        switch (k) {
            case 0: return row_bcast<0>(x);
            case 1: return row_bcast<1>(x);
            case 2: return row_bcast<2>(x);
            case 3: return row_bcast<3>(x);
            case 4: return row_bcast<4>(x);
            case 5: return row_bcast<5>(x);
            case 6: return row_bcast<6>(x);
            case 7: return row_bcast<7>(x);
            case 8: return row_bcast<8>(x);
            case 9: return row_bcast<9>(x);
            case 10: return row_bcast<10>(x);
            case 11: return row_bcast<11>(x);
            case 12: return row_bcast<12>(x);
            case 13: return row_bcast<13>(x);
            case 14: return row_bcast<14>(x);
            default: return row_bcast<15>(x);
        }
    }
    return __shfl(x, (int)((threadIdx.x & 63) & ~(GS - 1)) + k, 64);
}

// This group's bits of a wave ballot, group lane 0 in bit 0.
template <int GS>
__device__ __forceinline__ uint64_t grp_ballot(bool p) {
    const uint64_t b = __ballot(p);
    if (GS == 64) return b;
    return (b >> ((threadIdx.x & 63) & ~(GS - 1))) & ((1ull << GS) - 1);
}

// choose_tau evaluated by one group (inputs uniform over the group): a
// GS-way search, GS + 1 sub-intervals a round, enough rounds for the same
// resolution of log tau (17 for GS = 16, 14 for GS = 32).
template <int GS>
__device__ __forceinline__ double choose_tau_grp(int reg, double chi, const double* d2, const double* mu,
                                                 int n, double tau_fixed, double chi_t, double chi_f) {
    if (reg == HAMLS_REG_FIXED) return tau_fixed;
    if (reg != HAMLS_REG_CHI_TARGET || !(chi > chi_t)) return 0.0;
    const int r = threadIdx.x & (GS - 1);
    auto coupling = [&](double tau) {
        double acc = 0.0, cur = -1.0, inv = 0.0;
        for (int q = 0; q < n; q++) {
            if (mu[q] != cur) {
                cur = mu[q];
                inv = 1.0 / (1.0 + tau * cur);
            }
            acc += d2[q] * inv;
        }
        return acc;
    };
    const double target = 1.0 - 1.0 / chi_t;
    const uint64_t all = GS == 64 ? ~0ull : ((1ull << GS) - 1);
    double hi = 0.0;
    for (int e0 = 0; e0 < 2048 && hi == 0.0; e0 += GS) {
        const uint64_t over = grp_ballot<GS>(coupling(ldexp(1.0, e0 + r)) > target);
        if (over != all) hi = ldexp(1.0, e0 + __ffsll((unsigned long long)(~over & all)) - 1);
    }
    if (hi == 0.0) hi = ldexp(1.0, 2047);
    // a few rounds of the group search narrow log tau to a relative width of
    // ~1e-4 (65^3, 33^3 or 17^4 sub-intervals) with r_tau > target at the left
    // end a; then Newton steps on tau from exp(a).  r_tau is convex and
    // decreasing in tau, so the steps stay left of the root and rise to it
    // monotonically (quadratic convergence: three steps reach rounding).
    double a = log(1e-16), b = log(hi);
    constexpr int rounds = GS == 64 ? 3 : (GS == 32 ? 3 : 4);
    for (int round = 0; round < rounds; round++) {
        const double step = (b - a) / (GS + 1.0);
        const int cnt = __popcll(grp_ballot<GS>(coupling(exp(a + step * (r + 1))) > target));
        const double na = cnt == 0 ? a : a + step * cnt;
        const double nb = cnt == GS ? b : a + step * (cnt + 1);
        a = na;
        b = nb;
    }
    double t = exp(a);
    const double tmax = exp(b);
    for (int it = 0; it < 5; it++) {
        double f = -target, fp = 0.0, cur = -1.0, inv = 0.0;
        for (int q = 0; q < n; q++) {
            if (mu[q] != cur) {
                cur = mu[q];
                inv = 1.0 / (1.0 + t * cur);
            }
            f += d2[q] * inv;
            fp -= d2[q] * cur * inv * inv;
        }
        if (!(f > 0.0) || !(fp < 0.0)) break;
        const double tn = fmin(t - f / fp, tmax);
        if (!(tn > t)) break;
        t = tn;
    }
    const double tt = (chi - chi_t) / (chi_f - chi_t);
    double sm = 1.0;
    if (tt < 1.0) {
        const double t4 = tt * tt * tt * tt;
        sm = t4 * (35.0 - 84.0 * tt + 70.0 * tt * tt - 20.0 * tt * tt * tt);
    }
    return sm * t;
}

// mls_solve_epilogue for one node per group of GS lanes (m + F <= GS): Gs the
// node's packed Gram matrix and right-hand sides in LDS, group lane r holds
// row r of the normalised, reordered system.  The column scales and every
// pivot go round the group by broadcasts; no barrier, so the groups of a wave
// may take different branches.  UNIT: the F = m right-hand sides are the unit
// vectors e_f instead of those in Gs, so that output f is the derivative of
// c_1 with respect to the right-hand-side entry f (the coefficients of the
// generating functions in the monomial basis, Rem. 2.5).
template <int m, int GS, int F = 1, bool UNIT = false>
__device__ void mls_solve_group(const double* Gs, int count, int64_t j, const SolveArgs& A) {
    constexpr int NC = m - 1;
    constexpr int EG = m * (m + 1) / 2;
    static_assert(m + F <= GS, "group too small");
    static_assert(!UNIT || F == m, "unit right-hand sides: one per monomial");
    const int r = threadIdx.x & (GS - 1);
    const int base = (threadIdx.x & 63) & ~(GS - 1);
    const int64_t MQ = A.MQ;
    const uint8_t rst = A.rstatus[j];
    const double W = Gs[0];
    auto gidx = [](int a, int b) { return a * m - a * (a - 1) / 2 + (b - a); };
    if (count == 0 || !(W > 0.0)) {
        if (r < F) A.out[(int64_t)(A.f0 + r) * MQ + j] = __builtin_nan("");
        if (r == 0 && A.write_diag) {
            A.chi[j] = __builtin_nan("");
            A.tau[j] = __builtin_nan("");
            A.status[j] = rst | HAMLS_ST_EMPTY;
        }
        return;
    }
    bool degen = count < m;
    double inv = 1.0;  // 1 / sqrt(G_rr / W) on group lanes r < m
    {
        double v = 1.0;
        if (r < m) v = sqrt(Gs[gidx(r, r)] / W);
        if (grp_ballot<GS>(r < m && !(v > 0.0))) degen = true;
        inv = 1.0 / v;
    }
    if (degen) {
        if (r < F) A.out[(int64_t)(A.f0 + r) * MQ + j] = (UNIT ? (r == 0 ? 1.0 : 0.0) : Gs[EG + r]) / W;
        if (r == 0 && A.write_diag) {
            A.chi[j] = __builtin_inf();
            A.tau[j] = __builtin_inf();
            A.status[j] = rst | HAMLS_ST_UNDERDETERMINED;
        }
        return;
    }
    // row r of the normalised, reordered system; p(0) = NC, p(a) = a - 1
    double a[NC + 1];
    {
        const double iW = 1.0 / W;
        const int ar = r >= NC ? 0 : r + 1;
        const double sr = (r <= NC ? __shfl(inv, base + ar, 64) : 1.0) * iW;
#pragma unroll
        for (int c = 0; c <= NC; c++) {
            const int bc = c == NC ? 0 : c + 1;
            const double ib = grp_bcast<GS>(inv, bc);
            double v = 0.0;
            if (r <= NC) {
                const int lo = ar < bc ? ar : bc, hi = ar < bc ? bc : ar;
                v = Gs[gidx(lo, hi)] * (sr * ib);
            } else if (r < NC + 1 + F) {
                v = (UNIT ? (bc == r - NC - 1 ? 1.0 : 0.0) : Gs[EG + bc * F + (r - NC - 1)]) * (sr * ib);
            }
            a[c] = v;
        }
    }
    bool ill = false;
    double minpiv = 1.0, s_last = 1.0;
#pragma unroll
    for (int k = 0; k <= NC; k++) {
        const double sk = grp_bcast<GS>(a[k], k);
        if (k < NC) {
            minpiv = fmin(minpiv, sk);
            if (!(sk > 1e-300)) {
                ill = true;
                break;
            }
        } else {
            s_last = sk;
            if (!(sk > 0.0)) {
                ill = true;
                break;
            }
        }
        double lkk, il;
        pivot_roots(sk, lkk, il);
        a[k] = r == k ? lkk : a[k] * il;
#pragma unroll
        for (int c = k + 1; c <= NC; c++) a[c] = fma(-a[k], grp_bcast<GS>(a[k], c), a[c]);
    }
    double dv[NC > 0 ? NC : 1], d2[NC > 0 ? NC : 1], tf[NC > 0 ? NC : 1];
    double chi = 1.0, tau = 0.0, den = 1.0;
    if (!ill) {
#pragma unroll
        for (int k = 0; k < NC; k++) {
            dv[k] = grp_bcast<GS>(a[k], NC);
            d2[k] = dv[k] * dv[k];
        }
        chi = 1.0 / s_last;
        if (minpiv < kPivResolve) ill = true;
    }
    if (!ill) {
        tau = NC > 0 ? choose_tau_grp<GS>(A.reg, chi, d2, A.mu, NC, A.tau_fixed, A.chi_t, A.chi_f) : 0.0;
        den = s_last;
        if (tau > 0.0) {
#pragma unroll
            for (int k = 0; k < NC; k++) {
                const double tm = tau * A.mu[k];
                tf[k] = tm > 0.0 ? tm / (1.0 + tm) : 0.0;
                den += d2[k] * tf[k];
            }
        } else {
#pragma unroll
            for (int k = 0; k < NC; k++) tf[k] = 0.0;
        }
        if (!(den > kDenResolve)) ill = true;
    }
    if (ill) {
        if (r == 0) {
            const int slot = atomicAdd(A.rs_count, 1);
            A.rs_list[slot] = (int32_t)j;
        }
        return;
    }
    const double rho = grp_bcast<GS>(a[NC], NC);
    if (r > NC && r < NC + 1 + F) {
        double num = rho * a[NC];
#pragma unroll
        for (int k = 0; k < NC; k++) num += dv[k] * a[k] * tf[k];
        A.out[(int64_t)(A.f0 + r - NC - 1) * MQ + j] = num / den;
    }
    if (r == 0 && A.write_diag) {
        A.chi[j] = chi;
        A.tau[j] = tau;
        A.status[j] = rst | (tau > 0.0 ? HAMLS_ST_REGULARIZED : 0);
    }
}

// One node per group of GS lanes: the packed Gram matrices gram[j][E]
// (E = m(m+1)/2 + m, one field) of an assembly pass that stopped before the
// solve, and its neighbour counts.
template <int m, int GS>
__global__ __launch_bounds__(64) void k_mls_solve(const double* __restrict__ gram, SolveArgs A) {
    constexpr int NG = 64 / GS;
    constexpr int E = m * (m + 1) / 2 + m;
    __shared__ double gl[NG * E];
    const int g = threadIdx.x / GS, r = threadIdx.x % GS;
    const int64_t j = (int64_t)blockIdx.x * NG + g;
    // centres the assembly left to the re-solve have no entries
    const bool live = j < A.MQ && !(A.route && A.route[j]);
    for (int e = r; e < E; e += GS) gl[g * E + e] = live ? gram[j * E + e] : 0.0;
    __syncthreads();
    if (live) mls_solve_group<m, GS>(gl + g * E, A.nj[j], j, A);
}

// Re-solve of a node flagged by mls_solve_epilogue, from its Gram matrix and
// right-hand sides accumulated in double-double precision (Gh + Gl, same
// packing as the FP64 entries).  The same steps in double-double: the
// normalised system (scales rounded to doubles: d, z, rho and omega do not
// depend on column scaling), the Cholesky factor of [V | v1 | y] in
// registers, then d, 1 - |d|^2 = rho^2 (the last pivot, free of cancellation
// at this precision), z and omega rounded to doubles for tau and c_1.  A
// pivot of the unit-diagonal C at or below kRankTol^2 (|R_jj| of the
// unit-column V at or below kRankTol) or fewer than m neighbours: the weighted
// mean (tau -> infinity).  UNIT: right-hand side f is the unit vector
// e_{f0 + f} (the generating functions' gamma, F = m split into passes of at
// most 16); a separate instantiation, so that the fit's kernels keep their own
// register allocation.
template <int m, bool UNIT = false>
__device__ void mls_dd_epilogue(const double* Gh, const double* Gl, double* isc, int count, int F,
                                int j, const SolveArgs& A) {
    constexpr int NC = m - 1;
    constexpr int EG = m * (m + 1) / 2;
    const int lane = threadIdx.x & 63;
    const int64_t MQ = A.MQ;
    const uint8_t rst = A.rstatus[j] | HAMLS_ST_ILLCOND;
    const double W = Gh[0] + Gl[0];
    auto gidx = [](int a, int b) { return a * m - a * (a - 1) / 2 + (b - a); };
    if (count == 0 || !(W > 0.0)) {
        if (lane < F) A.out[(int64_t)(A.f0 + lane) * MQ + j] = __builtin_nan("");
        if (lane == 0 && A.write_diag) {
            A.chi[j] = __builtin_nan("");
            A.tau[j] = __builtin_nan("");
            A.status[j] = rst | HAMLS_ST_EMPTY;
        }
        return;
    }
    // column factors f_a = 1/sqrt(G_aa), applied entry by entry as two exact
    // double-double scalings, so that the normalised matrix is exactly the
    // congruence diag(f) G diag(f) of the accumulated one
    bool degen = count < m;
    {
        double v = 1.0;
        if (lane < m) v = sqrt(Gh[gidx(lane, lane)] + Gl[gidx(lane, lane)]);
        if (__ballot(lane < m && !(v > 0.0))) degen = true;
        if (lane < m) isc[lane] = 1.0 / v;
    }
    const double ws = 1.0 / sqrt(W);
    __syncthreads();
    dd a[NC + 1];
    bool ill = degen;
    double s_last = 1.0;
    if (!ill) {
        const int r = lane;
        const int ar = r >= NC ? 0 : r + 1;
        const double sr = r <= NC ? isc[ar] : ws;
#pragma unroll
        for (int c = 0; c <= NC; c++) {
            const int bc = c == NC ? 0 : c + 1;
            dd v = {0.0, 0.0};
            if (r <= NC) {
                const int lo = ar < bc ? ar : bc, hi = ar < bc ? bc : ar;
                const int e = gidx(lo, hi);
                v = dd_mul_d(dd_mul_d({Gh[e], Gl[e]}, sr), isc[bc]);
            } else if (r < NC + 1 + F) {
                // right-hand sides of the unit-sum weights: the data scaled by
                // 1/sqrt(W) (unit vectors for the generating functions)
                const int e = EG + bc * F + (r - NC - 1);
                const dd rhs = UNIT ? dd{bc == A.f0 + r - NC - 1 ? 1.0 : 0.0, 0.0} : dd{Gh[e], Gl[e]};
                v = dd_mul_d(dd_mul_d(rhs, sr), isc[bc]);
            }
            a[c] = v;
        }
        const double rank2 = kRankTol * kRankTol;
#pragma unroll
        for (int k = 0; k <= NC; k++) {
            const dd s = readlane_dd(a[k], k);
            if (k < NC) {
                if (!(s.hi > rank2)) {
                    ill = true;
                    break;
                }
            } else {
                s_last = s.hi;
                if (!(s.hi > 0.0)) {
                    s_last = 0.0;
                    break;
                }
            }
            const dd lkk = dd_sqrt(s);
            const dd il = dd_recip(lkk);
            a[k] = lane == k ? lkk : dd_mul(a[k], il);
#pragma unroll
            for (int c = k + 1; c <= NC; c++)
                a[c] = dd_add(a[c], dd_neg(dd_mul(a[k], readlane_dd(a[k], c))));
        }
    }
    if (ill) {
        // rank deficient: the tau -> infinity limit
        if (lane < F)
            A.out[(int64_t)(A.f0 + lane) * MQ + j] =
                (UNIT ? (A.f0 + lane == 0 ? 1.0 : 0.0) : Gh[EG + lane] + Gl[EG + lane]) / W;
        if (lane == 0 && A.write_diag) {
            A.chi[j] = __builtin_inf();
            A.tau[j] = __builtin_inf();
            A.status[j] = rst | HAMLS_ST_UNDERDETERMINED;
        }
        return;
    }
    double dv[NC > 0 ? NC : 1], d2[NC > 0 ? NC : 1], tf[NC > 0 ? NC : 1];
#pragma unroll
    for (int k = 0; k < NC; k++) {
        dv[k] = readlane_f64(a[k].hi, NC);
        d2[k] = dv[k] * dv[k];
    }
    const double chi = 1.0 / s_last;
    const double tau = NC > 0 ? choose_tau(A.reg, chi, d2, A.mu, NC, A.tau_fixed, A.chi_t, A.chi_f) : 0.0;
    double den = s_last;
#pragma unroll
    for (int k = 0; k < NC; k++) {
        const double tm = tau * A.mu[k];
        tf[k] = tm > 0.0 ? tm / (1.0 + tm) : 0.0;
        den += d2[k] * tf[k];
    }
    const double rho = sqrt(s_last);
    if (lane > NC && lane < NC + 1 + F) {
        // rho omega = r_1 - d.z (omega = 0 where rho = 0)
        double num = s_last > 0.0 ? rho * a[NC].hi : 0.0;
#pragma unroll
        for (int k = 0; k < NC; k++) num += dv[k] * a[k].hi * tf[k];
        A.out[(int64_t)(A.f0 + lane - NC - 1) * MQ + j] = num / den;
    }
    if (lane == 0 && A.write_diag) {
        A.chi[j] = chi;
        A.tau[j] = tau;
        A.status[j] = rst | (tau > 0.0 ? HAMLS_ST_REGULARIZED : 0);
    }
}

// mls_dd_epilogue by one group of GS lanes (GS / 64 nodes a wave): the same
// double-double steps, row r of the system on group lane r (m + F <= GS),
// broadcasts within the group, and the group's tau search.
template <int GS>
__device__ __forceinline__ dd grp_bcast_dd(dd x, int k) {
    return {grp_bcast<GS>(x.hi, k), grp_bcast<GS>(x.lo, k)};
}

template <int m, int GS, bool UNIT>
__device__ void mls_dd_group(const double* Gh, const double* Gl, int count, int F, int64_t j,
                             const SolveArgs& A) {
    constexpr int NC = m - 1;
    constexpr int EG = m * (m + 1) / 2;
    const int r = threadIdx.x & (GS - 1);
    const int base = (threadIdx.x & 63) & ~(GS - 1);
    const int64_t MQ = A.MQ;
    const uint8_t rst = A.rstatus[j] | HAMLS_ST_ILLCOND;
    const double W = Gh[0] + Gl[0];
    auto gidx = [](int a, int b) { return a * m - a * (a - 1) / 2 + (b - a); };
    if (count == 0 || !(W > 0.0)) {
        if (r < F) A.out[(int64_t)(A.f0 + r) * MQ + j] = __builtin_nan("");
        if (r == 0 && A.write_diag) {
            A.chi[j] = __builtin_nan("");
            A.tau[j] = __builtin_nan("");
            A.status[j] = rst | HAMLS_ST_EMPTY;
        }
        return;
    }
    bool degen = count < m;
    double inv = 1.0;  // 1 / sqrt(G_rr) on group lanes r < m
    {
        double v = 1.0;
        if (r < m) v = sqrt(Gh[gidx(r, r)] + Gl[gidx(r, r)]);
        if (grp_ballot<GS>(r < m && !(v > 0.0))) degen = true;
        inv = 1.0 / v;
    }
    const double ws = 1.0 / sqrt(W);
    dd a[NC + 1];
    bool ill = degen;
    double s_last = 1.0;
    if (!ill) {
        const int ar = r >= NC ? 0 : r + 1;
        const double sr = r <= NC ? __shfl(inv, base + ar, 64) : ws;
#pragma unroll
        for (int c = 0; c <= NC; c++) {
            const int bc = c == NC ? 0 : c + 1;
            const double ib = grp_bcast<GS>(inv, bc);
            dd v = {0.0, 0.0};
            if (r <= NC) {
                const int lo = ar < bc ? ar : bc, hi = ar < bc ? bc : ar;
                const int e = gidx(lo, hi);
                v = dd_mul_d(dd_mul_d({Gh[e], Gl[e]}, sr), ib);
            } else if (r < NC + 1 + F) {
                const int e = EG + bc * F + (r - NC - 1);
                const dd rhs = UNIT ? dd{bc == A.f0 + r - NC - 1 ? 1.0 : 0.0, 0.0} : dd{Gh[e], Gl[e]};
                v = dd_mul_d(dd_mul_d(rhs, sr), ib);
            }
            a[c] = v;
        }
        const double rank2 = kRankTol * kRankTol;
#pragma unroll
        for (int k = 0; k <= NC; k++) {
            const dd sk = grp_bcast_dd<GS>(a[k], k);
            if (k < NC) {
                if (!(sk.hi > rank2)) {
                    ill = true;
                    break;
                }
            } else {
                s_last = sk.hi;
                if (!(sk.hi > 0.0)) {
                    s_last = 0.0;
                    break;
                }
            }
            const dd lkk = dd_sqrt(sk);
            const dd il = dd_recip(lkk);
            a[k] = r == k ? lkk : dd_mul(a[k], il);
#pragma unroll
            for (int c = k + 1; c <= NC; c++) a[c] = dd_add(a[c], dd_neg(dd_mul(a[k], grp_bcast_dd<GS>(a[k], c))));
        }
    }
    if (ill) {
        // rank deficient: the tau -> infinity limit
        if (r < F)
            A.out[(int64_t)(A.f0 + r) * MQ + j] = (UNIT ? (A.f0 + r == 0 ? 1.0 : 0.0) : Gh[EG + r] + Gl[EG + r]) / W;
        if (r == 0 && A.write_diag) {
            A.chi[j] = __builtin_inf();
            A.tau[j] = __builtin_inf();
            A.status[j] = rst | HAMLS_ST_UNDERDETERMINED;
        }
        return;
    }
    double dv[NC > 0 ? NC : 1], d2[NC > 0 ? NC : 1], tf[NC > 0 ? NC : 1];
#pragma unroll
    for (int k = 0; k < NC; k++) {
        dv[k] = grp_bcast<GS>(a[k].hi, NC);
        d2[k] = dv[k] * dv[k];
    }
    const double chi = 1.0 / s_last;
    const double tau = NC > 0 ? choose_tau_grp<GS>(A.reg, chi, d2, A.mu, NC, A.tau_fixed, A.chi_t, A.chi_f) : 0.0;
    double den = s_last;
#pragma unroll
    for (int k = 0; k < NC; k++) {
        const double tm = tau * A.mu[k];
        tf[k] = tm > 0.0 ? tm / (1.0 + tm) : 0.0;
        den += d2[k] * tf[k];
    }
    const double rho = sqrt(s_last);
    if (r > NC && r < NC + 1 + F) {
        double num = s_last > 0.0 ? rho * a[NC].hi : 0.0;
#pragma unroll
        for (int k = 0; k < NC; k++) num += dv[k] * a[k].hi * tf[k];
        A.out[(int64_t)(A.f0 + r - NC - 1) * MQ + j] = num / den;
    }
    if (r == 0 && A.write_diag) {
        A.chi[j] = chi;
        A.tau[j] = tau;
        A.status[j] = rst | (tau > 0.0 ? HAMLS_ST_REGULARIZED : 0);
    }
}

// ---------------------------------------------------------------------------
// mixed precision (FP32 Gram, FP64 refinement), any domain
// ---------------------------------------------------------------------------

// LDS of one mixed-precision node (doubles): packed Gram + right-hand sides,
// column scales, the factor L, the FP32-data solutions, FP64 member rows; the
// FP32 member rows alias the start.
template <int m, int FM>
struct MixedLayout {
    static constexpr int EG = m * (m + 1) / 2;
    static constexpr int E = EG + m * FM;
    static constexpr int ROW32 = m + FM + 1;
    static constexpr int ROW64 = m + FM;
    static constexpr int oIsc = E, oL = oIsc + m, oC = oL + m * m, oRow = oC + FM * m;
    static constexpr int size = oRow + 64 * ROW64;  // doubles
    static_assert(64 * ROW32 <= 2 * size, "FP32 rows fit");
};

// One node by one wave in the mixed policy (Rem. 2.4: the local system's
// condition decides the precision):
//  1. FP32 Gram of [sqrt(w) g | sqrt(w) y] over the members (FP64 rows
//     rounded to FP32 in LDS, FP32 accumulation);
//  2. its FP64 Cholesky after unit-diagonal scaling; the node goes to the FP64
//     list (appended to A.rs_list) when it is empty-free but degenerate,
//     regularized (chi > chi_T / 2 or a fixed tau > 0) or has a pivot of C
//     below 1e-4;
//  3. otherwise the FP32-data solution c, one FP64 pass for the residual
//     B^T (y_w - B c) and a correction solve with the same factor:
//     value = c_1 + delta_1.
// scan(body) visits the candidate records (body(valid[U], idx[U]));
// key(i) is record i's membership key (member iff key > thr);
// row(i, key, r) writes sqrt(w) g of record i (m values) and returns sqrt(w).
template <int m, int FM, int U, class Scan, class Key, class Row>
__device__ __forceinline__ void mixed_node_core(int j, double* lds, double thr, const double* __restrict__ vals,
                                                int64_t vstride, int F, const SolveArgs& A,
                                                int32_t* __restrict__ nj, Scan&& scan, Key&& key, Row&& row) {
    using L_ = MixedLayout<m, FM>;
    constexpr int NC = m - 1, EG = L_::EG, ROW32 = L_::ROW32, ROW64 = L_::ROW64;
    constexpr int KE = (EG + m * FM + 63) / 64;
    constexpr int KG = (m * FM + 63) / 64;
    float* rows32 = (float*)lds;
    double* Gs = lds;
    double* isc = lds + L_::oIsc;
    double* Lm = lds + L_::oL;
    double* cv = lds + L_::oC;
    double* rows64 = lds + L_::oRow;
    const int lane = threadIdx.x;
    const int64_t MQ = A.MQ;
    const int E = EG + m * F;
    int ca[KE], cb[KE];
    float acc[KE];
#pragma unroll
    for (int k = 0; k < KE; k++) {
        int e = lane + 64 * k;
        acc[k] = 0.0f;
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
    // ---------------- pass 1: FP32 Gram
    int count = 0;
    scan([&](const bool* valid, const int* idx) {
#pragma unroll
        for (int u = 0; u < U; u++) {
            const double d = valid[u] ? key(idx[u]) : -1e300;
            const bool in = d > thr;
            const uint64_t mk = __ballot(in);
            const int nin = __popcll(mk);
            if (nin == 0) continue;
            if (in) {
                const int i = idx[u];
                double r64[m];
                const double sw = row(i, d, r64);
                float* rr = rows32 + rank_below(mk) * ROW32;
#pragma unroll
                for (int a = 0; a < m; a++) rr[a] = (float)r64[a];
                for (int f = 0; f < F; f++) rr[m + f] = (float)(sw * vals[(int64_t)f * vstride + i]);
            }
            __syncthreads();
#pragma unroll 2
            for (int r = 0; r < nin; r++) {
                const float* rr = rows32 + r * ROW32;
#pragma unroll
                for (int k = 0; k < KE; k++) acc[k] = fmaf(rr[ca[k]], rr[cb[k]], acc[k]);
            }
            __syncthreads();
            count += nin;
        }
    });
    if (lane == 0) nj[j] = count;
#pragma unroll
    for (int k = 0; k < KE; k++) {
        int e = lane + 64 * k;
        if (e < E) Gs[e] = (double)acc[k];
    }
    __syncthreads();
    // ---------------- FP64 factorisation of the FP32 system
    const uint8_t rst = A.rstatus[j];
    const double W = Gs[0];
    auto gidx = [](int a, int b) { return a * m - a * (a - 1) / 2 + (b - a); };
    auto to_fp64 = [&]() {
        if (lane == 0) {
            const int slot = atomicAdd(A.rs_count, 1);
            A.rs_list[slot] = j;
        }
    };
    if (count == 0 || !(W > 0.0)) {
        if (lane < F) A.out[(int64_t)(A.f0 + lane) * MQ + j] = __builtin_nan("");
        if (lane == 0 && A.write_diag) {
            A.chi[j] = __builtin_nan("");
            A.tau[j] = __builtin_nan("");
            A.status[j] = rst | HAMLS_ST_EMPTY;
        }
        return;
    }
    bool degen = count < m;
    {
        double v = 1.0;
        if (lane < m) v = sqrt(Gs[gidx(lane, lane)] / W);
        if (__ballot(lane < m && !(v > 0.0))) degen = true;
        if (lane < m) isc[lane] = 1.0 / v;
    }
    if (degen) {
        to_fp64();
        return;
    }
    __syncthreads();
    double a[NC + 1];
    {
        const int r = lane;
        const int ar = r >= NC ? 0 : r + 1;
        const double sr = r <= NC ? isc[ar] : 0.0;
#pragma unroll
        for (int cc = 0; cc <= NC; cc++) {
            const int bc = cc == NC ? 0 : cc + 1;
            double v = 0.0;
            if (r <= NC) {
                const int lo = ar < bc ? ar : bc, hi = ar < bc ? bc : ar;
                v = Gs[gidx(lo, hi)] / W * (sr * isc[bc]);
            } else if (r < NC + 1 + F) {
                v = Gs[EG + bc * F + (r - NC - 1)] / W * isc[bc];
            }
            a[cc] = v;
        }
    }
    bool ill = false;
    double minpiv = 1.0, s_last = 1.0;
#pragma unroll
    for (int k = 0; k <= NC; k++) {
        const double sk = readlane_f64(a[k], k);
        if (k < NC)
            minpiv = fmin(minpiv, sk);
        else
            s_last = sk;
        if (!(sk > 1e-300)) {
            ill = true;
            break;
        }
        double lkk, il;
        pivot_roots(sk, lkk, il);
        a[k] = lane == k ? lkk : a[k] * il;
#pragma unroll
        for (int cc = k + 1; cc <= NC; cc++) a[cc] = fma(-a[k], readlane_f64(a[k], cc), a[cc]);
    }
    const double chi = ill ? 0.0 : 1.0 / s_last;
    const bool regularized = (A.reg == HAMLS_REG_CHI_TARGET && chi > 0.5 * A.chi_t) ||
                             (A.reg == HAMLS_REG_FIXED && A.tau_fixed > 0.0);
    if (ill || minpiv < 1e-4 || regularized) {
        to_fp64();
        return;
    }
    // L (rows of the permuted order [V | v1]) to LDS; the field rows hold
    // y' = L^{-1} r_perm: back substitution gives the FP32-data solution
    if (lane <= NC) {
#pragma unroll
        for (int cc = 0; cc <= NC; cc++) Lm[lane * m + cc] = cc <= lane ? a[cc] : 0.0;
    }
    __syncthreads();
    auto back_subst = [&](double* x) {
        // x (permuted order) := L^{-T} x
#pragma unroll
        for (int i = NC; i >= 0; i--) {
            double v = x[i];
#pragma unroll
            for (int k2 = i + 1; k2 <= NC; k2++) v -= Lm[k2 * m + i] * x[k2];
            x[i] = v / Lm[i * m + i];
        }
    };
    auto fwd_subst = [&](double* x) {
#pragma unroll
        for (int i = 0; i <= NC; i++) {
            double v = x[i];
#pragma unroll
            for (int k2 = 0; k2 < i; k2++) v -= Lm[i * m + k2] * x[k2];
            x[i] = v / Lm[i * m + i];
        }
    };
    if (lane > NC && lane < NC + 1 + F) {
        double x[NC + 1];
#pragma unroll
        for (int i = 0; i <= NC; i++) x[i] = a[i];
        back_subst(x);
        const int f = lane - NC - 1;
        cv[f * m + 0] = x[NC];
#pragma unroll
        for (int i = 0; i < NC; i++) cv[f * m + i + 1] = x[i];
    }
    __syncthreads();
    // ---------------- pass 2: FP64 residual B^T (y_w - B c)
    const double ws = 1.0 / sqrt(W);
    double sc[m];
#pragma unroll
    for (int i = 0; i < m; i++) sc[i] = isc[i] * ws;
    int ga[KG], gf[KG];
    double gacc[KG];
#pragma unroll
    for (int k = 0; k < KG; k++) {
        const int e = lane + 64 * k;
        ga[k] = e < m * F ? e / F : 0;
        gf[k] = e < m * F ? m + e % F : m;
        gacc[k] = 0.0;
    }
    scan([&](const bool* valid, const int* idx) {
#pragma unroll
        for (int u = 0; u < U; u++) {
            const double d = valid[u] ? key(idx[u]) : -1e300;
            const bool in = d > thr;
            const uint64_t mk = __ballot(in);
            const int nin = __popcll(mk);
            if (nin == 0) continue;
            if (in) {
                const int i = idx[u];
                double b[m];
                const double sw = row(i, d, b);
                double* rr = rows64 + rank_below(mk) * ROW64;
#pragma unroll
                for (int a2 = 0; a2 < m; a2++) {
                    b[a2] *= sc[a2];
                    rr[a2] = b[a2];
                }
                for (int f = 0; f < F; f++) {
                    double e = sw * ws * vals[(int64_t)f * vstride + i];
#pragma unroll
                    for (int a2 = 0; a2 < m; a2++) e -= b[a2] * cv[f * m + a2];
                    rr[m + f] = e;
                }
            }
            __syncthreads();
            for (int r = 0; r < nin; r++) {
                const double* rr = rows64 + r * ROW64;
#pragma unroll
                for (int k = 0; k < KG; k++) gacc[k] = fma(rr[ga[k]], rr[gf[k]], gacc[k]);
            }
            __syncthreads();
        }
    });
    // correction: solve with the same factor, value = c_0 + delta_0
    double* gs = rows64;
#pragma unroll
    for (int k = 0; k < KG; k++) {
        const int e = lane + 64 * k;
        if (e < m * F) gs[e] = gacc[k];
    }
    __syncthreads();
    if (lane < F) {
        double x[NC + 1];
#pragma unroll
        for (int i = 0; i < NC; i++) x[i] = gs[(i + 1) * F + lane];
        x[NC] = gs[lane];
        fwd_subst(x);
        back_subst(x);
        A.out[(int64_t)(A.f0 + lane) * MQ + j] = cv[lane * m] + x[NC];
    }
    if (lane == 0 && A.write_diag) {
        A.chi[j] = chi;
        A.tau[j] = 0.0;
        A.status[j] = rst;
    }
}

}  // namespace hamls
