// s2_mixed.hip -- the FP32 quadrature contraction of S2 on the matrix cores
// (gfx950 MFMA), used by the mixed-precision path.
//
// Alg. 1 step 3 after the ring DFTs: with the rings folded about the equator
// (P_n^k(-x) = (-1)^{n+k} P_n^k(x)),
//   fhat_{n,k} = sum_{t < th} w_t P_n^k(x_t) X^{par(n+k)}_t(k),
//   X^0_t = G_t + G_{nt-1-t},  X^1_t = G_t - G_{nt-1-t}  (the equator ring once),
// for every order k >= 0 and parity p this is a product of the table block
// T_{k,p}[n][t] = w_t P_n^k(x_t) (rows n = k + p, k + p + 2, ...) with the
// th x 2F matrix of folded spectra (real and imaginary part of every field).
// Negative orders follow from fhat_{n,-k} = (-1)^k conj(fhat_{n,k}).
//
// Layout (built at plan time in FP64, stored in FP32): block (k, p) is
// [t < th_pad][row < R_pad] (row fastest), rows padded to 16, t to 4, zeros in
// the padding; the folded spectra of one (k, p) are [t < th_pad][col < C_pad],
// C_pad = 2F padded to 16.  One wave computes a 16-row tile of one block
// against all column tiles with v_mfma_f32_16x16x4f32 (A 16x4, B 4x16, D
// 16x16, FP32 accumulate): lane l holds A[l % 16][l / 16], B[l / 16][l % 16]
// and D[4 (l / 16) + r][l % 16], r < 4.
#include "common.h"
#include "device_common.h"

namespace hamls {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// X[(k, p)][t][c], c = 2 f + (0 re, 1 im), from the FP64 ring spectra
// G[f][t][k] (complex).
__global__ __launch_bounds__(256) void k_s2_fold32(const double* __restrict__ G, int nt, int N, int F,
                                                   int th, int th_pad, int C_pad, float* __restrict__ X) {
    const int64_t per_k = (int64_t)2 * th_pad * C_pad;
    const int64_t tot = (int64_t)(N + 1) * per_k;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int k = (int)(e / per_k);
        int64_t r = e - (int64_t)k * per_k;
        const int p = (int)(r / ((int64_t)th_pad * C_pad));
        r -= (int64_t)p * th_pad * C_pad;
        const int t = (int)(r / C_pad), c = (int)(r - (int64_t)t * C_pad);
        float v = 0.0f;
        if (t < th && c < 2 * F) {
            const int f = c >> 1, part = c & 1;
            const int t2 = nt - 1 - t;
            const double g1 = G[(((int64_t)f * nt + t) * (N + 1) + k) * 2 + part];
            double x;
            if (t == t2)
                x = p == 0 ? g1 : 0.0;
            else {
                const double g2 = G[(((int64_t)f * nt + t2) * (N + 1) + k) * 2 + part];
                x = p == 0 ? g1 + g2 : g1 - g2;
            }
            v = (float)x;
        }
        X[e] = v;
    }
}

// Work item: order k, parity p, 16-row tile rt of block (k, p).
struct LegItem {
    int k, p, rt, pad;
};

template <int NCT>
__global__ __launch_bounds__(64) void k_s2_legendre_mfma(const float* __restrict__ tab,
                                                         const int64_t* __restrict__ tab_off,
                                                         const LegItem* __restrict__ items,
                                                         const float* __restrict__ X, int N, int F,
                                                         int th_pad, int C_pad, int ct0,
                                                         double* __restrict__ coeffs) {
    const LegItem it = items[blockIdx.x];
    const int k = it.k, p = it.p;
    const int R = N >= k + p ? (N - k - p) / 2 + 1 : 0;
    const int R_pad = (R + 15) & ~15;
    const float* A = tab + tab_off[2 * k + p];
    const float* B = X + ((int64_t)(2 * k + p) * th_pad) * C_pad + ct0 * 16;
    const int lane = threadIdx.x;
    const int row = it.rt * 16 + (lane & 15), kk = lane >> 4;
    const int ncols = 2 * F - ct0 * 16;  // columns left from this launch's first tile
    f32x4 acc[NCT];
#pragma unroll
    for (int c = 0; c < NCT; c++) acc[c] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int t0 = 0; t0 < th_pad; t0 += 4) {
        const float a = A[(int64_t)(t0 + kk) * R_pad + row];
#pragma unroll
        for (int c = 0; c < NCT; c++) {
            const float b = B[(int64_t)(t0 + kk) * C_pad + c * 16 + (lane & 15)];
            acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
        }
    }
    const int64_t nc = (int64_t)(N + 1) * (N + 1);
    const double sg = (k & 1) ? -1.0 : 1.0;
#pragma unroll
    for (int c = 0; c < NCT; c++) {
        const int col = c * 16 + (lane & 15);
        if (col >= ncols) continue;
        const int cg = ct0 * 16 + col;
        const int f = cg >> 1, part = cg & 1;
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int rr = it.rt * 16 + 4 * kk + r;
            if (rr >= R) continue;
            const int n = k + p + 2 * rr;
            const double v = (double)acc[c][r];
            coeffs[((int64_t)f * nc + (int64_t)n * n + n + k) * 2 + part] = v;
            if (k > 0)
                coeffs[((int64_t)f * nc + (int64_t)n * n + n - k) * 2 + part] = part == 0 ? sg * v : -sg * v;
        }
    }
}

hamls_status launch_s2_legendre_mfma(const Plan& P, int F, const double* G, float* X, int64_t xcap,
                                     double* coeffs, hipStream_t s) {
    const int nt = P.dims[0], N = P.N;
    const int th = (nt + 1) / 2, th_pad = (th + 3) & ~3;
    const int C_pad = ((2 * F + 15) / 16) * 16;
    const int64_t xlen = (int64_t)(N + 1) * 2 * th_pad * C_pad;
    if (xlen > xcap) {
        set_error("fold buffer too small");
        return HAMLS_ERR_INVALID_ARG;
    }
    {
        const int bs = 256;
        int64_t nb = (xlen + bs - 1) / bs;
        nb = nb < 65536 ? nb : 65536;
        hipLaunchKernelGGL(k_s2_fold32, dim3((unsigned)nb), dim3(bs), 0, s, G, nt, N, F, th, th_pad, C_pad, X);
        HAMLS_HIP(hipGetLastError());
    }
    const int nct_total = C_pad / 16;
    for (int ct0 = 0; ct0 < nct_total; ct0 += 8) {
        const int nct = nct_total - ct0 < 8 ? nct_total - ct0 : 8;
        dim3 grid((unsigned)P.leg_items), block(64);
#define HAMLS_LEG(NN)                                                                                 \
    hipLaunchKernelGGL(k_s2_legendre_mfma<NN>, grid, block, 0, s, P.d_ptab32, P.d_tab_off,            \
                       (const LegItem*)P.d_leg_items, X, N, F, th_pad, C_pad, ct0, coeffs)
        if (nct <= 1)
            HAMLS_LEG(1);
        else if (nct <= 2)
            HAMLS_LEG(2);
        else if (nct <= 4)
            HAMLS_LEG(4);
        else
            HAMLS_LEG(8);
#undef HAMLS_LEG
        HAMLS_HIP(hipGetLastError());
    }
    return HAMLS_OK;
}

// FP32 table blocks from the resident FP64 table (which holds
// w_t P_n^k(x_t) at [t][n(n+1)/2 + k]): block (k, p) at off[2k + p] is
// [t < th_pad][row < R_pad], row r <-> degree n = k + p + 2r, zero padding.
__global__ __launch_bounds__(256) void k_s2_mfma_table(const double* __restrict__ tab64,
                                                      const int64_t* __restrict__ off, int th, int th_pad,
                                                      int N, float* __restrict__ tab32) {
    const int kp = blockIdx.y;
    const int k = kp >> 1, p = kp & 1;
    const int R = N >= k + p ? (N - k - p) / 2 + 1 : 0;
    const int R_pad = (R + 15) & ~15;
    const int64_t na = (int64_t)(N + 1) * (N + 2) / 2;
    const int64_t len = (int64_t)th_pad * R_pad;
    float* blk = tab32 + off[kp];
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int t = (int)(e / R_pad), r = (int)(e - (int64_t)t * R_pad);
        float v = 0.0f;
        if (t < th && r < R) {
            const int n = k + p + 2 * r;
            v = (float)tab64[(int64_t)t * na + (int64_t)n * (n + 1) / 2 + k];
        }
        blk[e] = v;
    }
}

hamls_status launch_s2_mfma_table(const Plan& P, int64_t len, hipStream_t s) {
    (void)len;
    const int nt = P.dims[0], N = P.N;
    const int th = (nt + 1) / 2, th_pad = (th + 3) & ~3;
    dim3 grid(16u, (unsigned)(2 * (N + 1)));
    hipLaunchKernelGGL(k_s2_mfma_table, grid, dim3(256), 0, s, P.d_ptab, P.d_tab_off, th, th_pad, N,
                       P.d_ptab32);
    HAMLS_HIP(hipGetLastError());
    return HAMLS_OK;
}

// Host: offsets of the FP32 table blocks, their total length and the work
// items.
hamls_status build_s2_mfma_layout(Plan& P, std::vector<int64_t>& off, std::vector<int32_t>& items,
                                  int64_t* len) {
    const int nt = P.dims[0], N = P.N;
    const int th = (nt + 1) / 2, th_pad = (th + 3) & ~3;
    off.assign(2 * (size_t)(N + 1), 0);
    int64_t total = 0;
    items.clear();
    for (int k = 0; k <= N; k++)
        for (int p = 0; p < 2; p++) {
            const int R = N >= k + p ? (N - k - p) / 2 + 1 : 0;
            const int R_pad = (R + 15) & ~15;
            off[2 * k + p] = total;
            total += (int64_t)th_pad * R_pad;
            for (int rt = 0; rt < R_pad / 16; rt++) {
                items.push_back(k);
                items.push_back(p);
                items.push_back(rt);
                items.push_back(0);
            }
        }
    P.leg_items = (int64_t)items.size() / 4;
    *len = total;
    return HAMLS_OK;
}

}  // namespace hamls
