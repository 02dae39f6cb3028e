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

// Ints of LDS one wave needs for s2_scan.
constexpr int kScanLds = 4 * 64 + 1;

// Order-preserving map of doubles to unsigned integers.
__device__ __forceinline__ uint64_t ordered_bits(double v) {
    uint64_t b = (uint64_t)__double_as_longlong(v);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double from_ordered_bits(uint64_t u) {
    uint64_t b = (u >> 63) ? (u & 0x7fffffffffffffffull) : ~u;
    return __longlong_as_double((long long)b);
}


// A centre whose normal-matrix solve is not trustworthy to ~1e-10 is re-solved
// by QR: Cholesky failure, a pivot of the unit-diagonal C below kPivQR
// (condition estimate above 1e8), or a Schur denominator below kDenQR
// (regularized chi_tau above 1e4, where 1 - sum d^2/(1 + tau mu) cancels).
constexpr double kPivQR = 1e-8;
constexpr double kDenQR = 1e-4;
// |R_jj| of the unit-column V at or below which V is taken as rank deficient.
constexpr double kRankTol = 1e-11;

__device__ __forceinline__ double coupling_tau(const double* d2, const double* mu, int n, double tau) {
    double r = 0.0;
    for (int j = 0; j < n; j++) r += d2[j] / (1.0 + tau * mu[j]);
    return r;
}

// tau of eq. (22).  Chi-target: 0 for chi <= chi_T; otherwise the tau with
// chi_tau = chi_T (eq. (23)) by bisection on log tau (64 halvings between 1e-16
// and the first power of two that overshoots), times the C^3 smoothstep
// S(t) = 35t^4 - 84t^5 + 70t^6 - 20t^7 of t = (chi - chi_T)/(chi_full - chi_T).
__device__ inline double choose_tau(int reg, double chi, const double* d2, const double* mu, int n,
                             double tau_fixed, double chi_t, double chi_f) {
    if (reg == HAMLS_REG_FIXED) return tau_fixed;
    if (reg != HAMLS_REG_CHI_TARGET || !(chi > chi_t)) return 0.0;
    double target = 1.0 - 1.0 / chi_t;
    double hi = 1.0;
    int guard = 0;
    while (coupling_tau(d2, mu, n, hi) > target && guard < 2000) {
        hi *= 2.0;
        guard++;
    }
    double a = log(1e-16), b = log(hi);
    for (int it = 0; it < 64; it++) {
        double mid = 0.5 * (a + b);
        if (coupling_tau(d2, mu, n, exp(mid)) > target)
            a = mid;
        else
            b = mid;
    }
    double tt = (chi - chi_t) / (chi_f - chi_t);
    double sm = 1.0;
    if (tt < 1.0) {
        double t4 = tt * tt * tt * tt;
        sm = t4 * (35.0 - 84.0 * tt + 70.0 * tt * tt - 20.0 * tt * tt * tt);
    }
    return sm * exp(0.5 * (a + b));
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}


}  // namespace hamls
