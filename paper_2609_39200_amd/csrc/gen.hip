// Generating functions of MLS (Rem. 2.5): the value at grid node x is the
// linear functional M_y(x) = sum_i a*_i y_i of the data, with a*_i depending
// on the geometry only.  With R_a = sum_i w_i g_a(x_i) y_i the right-hand side
// of the (regularized) normal equations, c_1 is linear in R, so
//   a*_i = w_i sum_a gamma_a g_a(x_i),   gamma_a = d c_1 / d R_a,
// and gamma is c_1 of the solve with the unit vectors e_a as right-hand sides.
// Built once per node set, the values a*_i turn every later fit on the same
// nodes into one sparse product (grid node rows, member columns).
#include <hip/hip_runtime.h>

#include "common.h"
#include "device_common.h"

namespace hamls {

// gamma of GS-lane groups, 64 / GS nodes per wave, from the packed Gram
// matrices of a one-field assembly pass ([j][m(m+1)/2 + m]); the pass's
// right-hand side is not used.
template <int m, int GS>
__global__ __launch_bounds__(64) void k_gen_solve(const double* __restrict__ gram, SolveArgs A) {
    constexpr int NG = 64 / GS;
    constexpr int E = m * (m + 1) / 2 + m;
    __shared__ double gl[NG * E];
    const int g = threadIdx.x / GS, r = threadIdx.x % GS;
    const int64_t j = (int64_t)blockIdx.x * NG + g;
    const bool live = j < A.MQ;
    for (int e = r; e < E; e += GS) gl[g * E + e] = live ? gram[j * E + e] : 0.0;
    __syncthreads();
    if (live) mls_solve_group<m, GS, m, true>(gl + g * E, A.nj[j], j, A);
}

// row_ptr = exclusive prefix sum of the neighbour counts, over tiles of
// kTileItems grid nodes: the tile sums, one scan of them (which also writes
// row_ptr[MQ], the entry count), and each tile's scan from its base.
__global__ __launch_bounds__(256) void k_tile_sums(const int32_t* __restrict__ nj, int64_t MQ,
                                                   int64_t* __restrict__ sums) {
    __shared__ int64_t ws[4];
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kTileItems;
    int64_t own = 0;
    for (int r = 0; r < kTileItems / 256; r++) {
        const int64_t j = base + r * 256 + t;
        if (j < MQ) own += nj[j];
    }
    own = wave_incl_scan_i64(own);
    if ((t & 63) == 63) ws[t >> 6] = own;
    __syncthreads();
    if (t == 0) sums[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

__global__ __launch_bounds__(256) void k_tile_rowptr(const int32_t* __restrict__ nj, int64_t MQ,
                                                     const int64_t* __restrict__ bases,
                                                     int64_t* __restrict__ row_ptr) {
    __shared__ int64_t ws[4];
    const int t = threadIdx.x, w = t >> 6;
    const int64_t base = (int64_t)blockIdx.x * kTileItems;
    int64_t carry = bases[blockIdx.x];
    for (int r = 0; r < kTileItems / 256; r++) {
        const int64_t j = base + r * 256 + t;
        const int64_t x = j < MQ ? (int64_t)nj[j] : 0;
        const int64_t incl = wave_incl_scan_i64(x);
        if ((t & 63) == 63) ws[w] = incl;
        __syncthreads();
        int64_t pre = carry;
        for (int w2 = 0; w2 < w; w2++) pre += ws[w2];
        if (j < MQ) row_ptr[j] = pre + incl - x;
        carry += ws[0] + ws[1] + ws[2] + ws[3];
        __syncthreads();
    }
}

// out[f0 + f][j] = sum_e val[e] vals[f][col[e]] over row j, col the original
// node index (the caller's values are read in place, no gather pass): 32 lanes
// per grid node, 8 nodes per 256-thread block; each lane takes U entries of
// its row at once (entries are read once: non-temporal loads; the values stay
// in L2), then a 32-lane butterfly.  Measured on the S2 cluster workload (47
// entries a row): 16 lanes a row took 1.6x as long, a whole wave 1.2x.  Rows
// without entries (no node in the support) give NaN, as the fit does.  vals:
// row f at vals + f * ldv.
template <int FM, int U>
__global__ __launch_bounds__(256) void k_gen_apply(const int64_t* __restrict__ row_ptr,
                                                   const int32_t* __restrict__ col,
                                                   const double* __restrict__ val,
                                                   const double* __restrict__ vals, int64_t ldv, int F,
                                                   int f0, int64_t MQ, double* __restrict__ out) {
    constexpr int GS = 32;
    const int g = threadIdx.x / GS, r = threadIdx.x % GS;
    const int64_t j = (int64_t)xcd_block(blockIdx.x, gridDim.x) * (256 / GS) + g;
    if (j >= MQ) return;  // whole groups: the butterfly stays within live lanes
    const int64_t b = row_ptr[j], e = row_ptr[j + 1];
    double acc[FM];
#pragma unroll
    for (int f = 0; f < FM; f++) acc[f] = 0.0;
    for (int64_t k0 = b + r; k0 < e; k0 += GS * U) {
        double a[U];
        int64_t i[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int64_t k = k0 + GS * u;
            a[u] = 0.0;
            i[u] = 0;
            if (k < e) {
                a[u] = __builtin_nontemporal_load(val + k);
                i[u] = __builtin_nontemporal_load(col + k);
            }
        }
#pragma unroll
        for (int u = 0; u < U; u++)
#pragma unroll
            for (int f = 0; f < FM; f++)
                if (f < F) acc[f] = fma(a[u], vals[f * ldv + i[u]], acc[f]);
    }
#pragma unroll
    for (int f = 0; f < FM; f++) {
#pragma unroll
        for (int o = GS / 2; o > 0; o >>= 1) acc[f] += __shfl_xor(acc[f], o, GS);
    }
    if (r == 0) {
        const double nan = __builtin_nan("");
#pragma unroll
        for (int f = 0; f < FM; f++)
            if (f < F) out[(int64_t)(f0 + f) * MQ + j] = e > b ? acc[f] : nan;
    }
}

hamls_status launch_gen_solve(const Plan& P, hipStream_t s) {
    SolveArgs A = make_solve_args(P, P.m, 0, P.d_gamma);
    const double* G = P.d_entries;
    // m + m lanes per node: groups of 16 up to m = 8, 32 up to 16, else 64
#define HAMLS_GS(MM, GS)                                                                   \
    hipLaunchKernelGGL((k_gen_solve<MM, GS>), dim3((unsigned)((P.MQ + 64 / GS - 1) / (64 / GS))), \
                       dim3(64), 0, s, G, A);
    switch (P.m) {
        case 1: HAMLS_GS(1, 16) break;
        case 3: HAMLS_GS(3, 16) break;
        case 4: HAMLS_GS(4, 16) break;
        case 6: HAMLS_GS(6, 16) break;
        case 10: HAMLS_GS(10, 32) break;
        case 15: HAMLS_GS(15, 32) break;
        case 20: HAMLS_GS(20, 64) break;
        default: set_error("no generating-function solve for m = %d", P.m); return HAMLS_ERR_UNSUPPORTED;
    }
#undef HAMLS_GS
    HAMLS_HIP(hipGetLastError());
    return HAMLS_OK;
}

hamls_status launch_gen_rowptr(const Plan& P, hipStream_t s) {
    const int nt = tile_count(P.MQ);
    if (!P.d_tiles || 2 * (int64_t)nt > P.tiles_len) {
        set_error("tile buffer too small");
        return HAMLS_ERR_INVALID_ARG;
    }
    int64_t* sums = (int64_t*)P.d_tiles;
    hipLaunchKernelGGL(k_tile_sums, dim3(nt), dim3(256), 0, s, P.d_nj, P.MQ, sums);
    hipLaunchKernelGGL((k_exclusive_scan<int64_t>), dim3(1), dim3(1024), 0, s, sums, (int64_t)nt,
                       P.d_grow + P.MQ);
    hipLaunchKernelGGL(k_tile_rowptr, dim3(nt), dim3(256), 0, s, P.d_nj, P.MQ, sums, P.d_grow);
    HAMLS_HIP(hipGetLastError());
    return HAMLS_OK;
}

hamls_status launch_gen_apply(const Plan& P, const double* values, int64_t ld, int F, int f0,
                              double* grid_values, hipStream_t s) {
    const dim3 grid((unsigned)((P.MQ + 7) / 8)), block(256);
    const double* v = values + (int64_t)f0 * ld;
    if (F == 1)
        hipLaunchKernelGGL((k_gen_apply<1, 2>), grid, block, 0, s, P.d_grow, P.d_gcol, P.d_gval, v, ld, F,
                           f0, P.MQ, grid_values);
    else
        hipLaunchKernelGGL((k_gen_apply<kMaxFieldsPerPass, 2>), grid, block, 0, s, P.d_grow, P.d_gcol,
                           P.d_gval, v, ld, F, f0, P.MQ, grid_values);
    HAMLS_HIP(hipGetLastError());
    return HAMLS_OK;
}

}  // namespace hamls
