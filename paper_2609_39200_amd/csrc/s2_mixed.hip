// s2_mixed.hip -- the FP32 quadrature contraction of S2 on the matrix cores
// (gfx950 MFMA), used by the mixed-precision path.
//
// Alg. 1 step 3 after the ring transforms: with the rings folded about the
// equator (P_n^k(-x) = (-1)^{n+k} P_n^k(x)),
//   fhat_{n,k} = sum_{t < th} w_t P_n^k(x_t) X^{par(n+k)}_t(k),
//   X^0_t = G_t + G_{nt-1-t},  X^1_t = G_t - G_{nt-1-t}  (the equator ring once),
// for every order k >= 0 and parity p this is a product of the table block
// T_{k,p}[n][t] = w_t P_n^k(x_t) (rows n = k + p, k + p + 2, ...) with the
// th x 2F matrix of folded spectra (real and imaginary part of every field).
// Negative orders follow from fhat_{n,-k} = (-1)^k conj(fhat_{n,k}).
//
// Layout (generated at plan time in FP64, stored in FP32): block (k, p) is
// [t < th_pad][row < R_pad] (row fastest), rows padded to 16, t to 4, zeros in
// the padding; the folded spectra of one (k, p) are [t < th_pad][col < C_pad],
// C_pad = 2F padded to 16.
//
// Kernels: k_s2_fold_x transposes the FP64 ring spectra G[f][t][k] into the
// FP32 folded spectra through an LDS tile (reads coalesced along k, writes
// along the columns); k_s2_legendre_mfma computes a 64-row x CW-column tile
// of one block per workgroup: the K = th_pad reduction runs in chunks of 16
// or 32 rings staged in LDS (double-buffered, one barrier per chunk; the next
// chunk's global loads in flight during the current chunk's MFMAs), and each of
// the four waves accumulates 2 x CW/32 tiles of v_mfma_f32_16x16x4f32
// (A 16x4, B 4x16, D 16x16, FP32 accumulate: lane l holds A[l % 16][l / 16],
// B[l / 16][l % 16] and D[4 (l / 16) + r][l % 16], r < 4).
#include "common.h"
#include "device_common.h"

namespace hamls {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kFoldK = 32;   // orders per fold tile
constexpr int kFoldC = 128;  // columns (64 fields) per fold tile

// X[(k, p)][t][c], c = 2 f + (0 re, 1 im), from the FP64 ring spectra
// G[f][t][k] (complex); grid (t < th_pad, k tiles, column tiles).
__global__ __launch_bounds__(256) void k_s2_fold_x(const double* __restrict__ G, int nt, int N, int F, int th,
                                                   int th_pad, int C_pad, float* __restrict__ X) {
    __shared__ float tile[2][kFoldK][kFoldC + 1];
    const int t = blockIdx.x;
    const int k0 = blockIdx.y * kFoldK;
    const int c0 = blockIdx.z * kFoldC;
    const int f0 = c0 / 2;
    const int nk = min(kFoldK, N + 1 - k0);
    const int t2 = nt - 1 - t;
    // read: for every field of the tile, kFoldK orders of rings t and t2
    // (re, im), consecutive threads on consecutive doubles
    for (int e = threadIdx.x; e < (kFoldC / 2) * kFoldK * 2; e += blockDim.x) {
        const int part = e & 1;
        const int k = (e >> 1) % kFoldK;
        const int fl = (e >> 1) / kFoldK;
        const int f = f0 + fl;
        float ev = 0.0f, od = 0.0f;
        if (t < th && k < nk && f < F) {
            const double g1 = G[(((int64_t)f * nt + t) * (N + 1) + k0 + k) * 2 + part];
            if (t == t2) {
                ev = (float)g1;
            } else {
                const double g2 = G[(((int64_t)f * nt + t2) * (N + 1) + k0 + k) * 2 + part];
                ev = (float)(g1 + g2);
                od = (float)(g1 - g2);
            }
        }
        tile[0][k][2 * fl + part] = ev;
        tile[1][k][2 * fl + part] = od;
    }
    __syncthreads();
    const int ncol = min(kFoldC, C_pad - c0);
    for (int e = threadIdx.x; e < 2 * nk * kFoldC; e += blockDim.x) {
        const int c = e % kFoldC;
        const int pk = e / kFoldC;
        const int p = pk & 1, k = pk >> 1;
        if (c < ncol)
            X[((((int64_t)(k0 + k) * 2 + p) * th_pad) + t) * C_pad + c0 + c] = tile[p][k][c];
    }
}

// Work item: order k, parity p, 64-row tile rt of block (k, p).
struct LegItem {
    int k, p, rt, pad;
};

constexpr int kMfmaRows = 64;  // rows per workgroup tile (4 waves: 2 x 2 row halves / column halves)

// One workgroup (256 threads) per (item, column chunk of CW): rows
// [64 rt, 64 rt + 64) of block (k, p) against columns [cw0, cw0 + CW).
// Wave w owns rows 32 (w / 2) .. + 32 (two 16-row tiles) and columns
// (CW / 2) (w % 2) .. + CW / 2 (CW / 32 tiles of 16).
template <int CW>
__global__ __launch_bounds__(256) void k_s2_legendre_mfma(const float* __restrict__ tab,
                                                         const int64_t* __restrict__ tab_off,
                                                         const LegItem* __restrict__ items,
                                                         const float* __restrict__ X, int N, int F, int th_pad,
                                                         int C_pad, double* __restrict__ coeffs) {
    constexpr int NCT = CW / 32;          // column tiles of 16 per wave
    constexpr int kMfmaTK = CW == 128 ? 16 : 32;  // rings per LDS chunk (LDS for four blocks per CU)
    constexpr int LA = kMfmaRows + 16;    // LDS row strides (padded against bank conflicts)
    constexpr int LB = CW + 16;
    __shared__ __align__(16) float As[2][kMfmaTK * LA];
    __shared__ __align__(16) float Bs[2][kMfmaTK * LB];
    const LegItem it = items[blockIdx.x];
    const int k = it.k, p = it.p;
    const int cw0 = blockIdx.y * CW;
    const int R = N >= k + p ? (N - k - p) / 2 + 1 : 0;
    const int R_pad = (R + 15) & ~15;
    const int r0 = it.rt * kMfmaRows;
    const float* A = tab + tab_off[2 * k + p];
    const float* B = X + ((int64_t)(2 * k + p) * th_pad) * C_pad;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = (w >> 1) * 32, wc = (w & 1) * (CW / 2);
    const int nchunk = (th_pad + kMfmaTK - 1) / kMfmaTK;

    // chunk q of A (kMfmaTK rings x 64 rows) and B (x CW columns) in 16-byte
    // pieces: loaded into registers one chunk ahead (in flight during the
    // MFMAs of the current chunk), then stored to the other LDS buffer
    constexpr int NA = kMfmaTK * kMfmaRows / 4 / 256;  // float4 of A per thread
    constexpr int NBv = kMfmaTK * CW / 4 / 256;        // float4 of B per thread
    static_assert(NA * 256 * 4 == kMfmaTK * kMfmaRows && NBv * 256 * 4 == kMfmaTK * CW, "chunk split");
    float4 ra[NA], rb[NBv];
    auto gload = [&](int q) {
        const int t0 = q * kMfmaTK;
#pragma unroll
        for (int v = 0; v < NA; v++) {
            const int e = (tid + 256 * v) * 4;
            const int tt = e / kMfmaRows, rr = e - tt * kMfmaRows;
            const int t = t0 + tt, r = r0 + rr;
            ra[v] = (t < th_pad && r < R_pad) ? *(const float4*)(A + (int64_t)t * R_pad + r)
                                              : float4{0.0f, 0.0f, 0.0f, 0.0f};
        }
#pragma unroll
        for (int v = 0; v < NBv; v++) {
            const int e = (tid + 256 * v) * 4;
            const int tt = e / CW, cc = e - tt * CW;
            const int t = t0 + tt, c = cw0 + cc;
            rb[v] = (t < th_pad && c < C_pad) ? *(const float4*)(B + (int64_t)t * C_pad + c)
                                              : float4{0.0f, 0.0f, 0.0f, 0.0f};
        }
    };
    auto lstore = [&](int buf) {
#pragma unroll
        for (int v = 0; v < NA; v++) {
            const int e = (tid + 256 * v) * 4;
            const int tt = e / kMfmaRows, rr = e - tt * kMfmaRows;
            *(float4*)(As[buf] + tt * LA + rr) = ra[v];
        }
#pragma unroll
        for (int v = 0; v < NBv; v++) {
            const int e = (tid + 256 * v) * 4;
            const int tt = e / CW, cc = e - tt * CW;
            *(float4*)(Bs[buf] + tt * LB + cc) = rb[v];
        }
    };

    f32x4 acc[2][NCT];
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int c = 0; c < NCT; c++) acc[i][c] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

    gload(0);
    lstore(0);
    __syncthreads();
    for (int q = 0; q < nchunk; q++) {
        const int buf = q & 1;
        if (q + 1 < nchunk) gload(q + 1);
        const float* as = As[buf];
        const float* bs = Bs[buf];
#pragma unroll
        for (int tk = 0; tk < kMfmaTK; tk += 4) {
            const int kr = tk + (lane >> 4);
            const float a0 = as[kr * LA + wr + (lane & 15)];
            const float a1 = as[kr * LA + wr + 16 + (lane & 15)];
#pragma unroll
            for (int c = 0; c < NCT; c++) {
                const float b = bs[kr * LB + wc + c * 16 + (lane & 15)];
                acc[0][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b, acc[0][c], 0, 0, 0);
                acc[1][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b, acc[1][c], 0, 0, 0);
            }
        }
        // the other buffer was last read before the previous barrier
        if (q + 1 < nchunk) lstore(buf ^ 1);
        __syncthreads();
    }

    const int64_t nc = (int64_t)(N + 1) * (N + 1);
    const double sg = (k & 1) ? -1.0 : 1.0;
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int c = 0; c < NCT; c++) {
            const int col = cw0 + wc + c * 16 + (lane & 15);
            if (col >= 2 * F) continue;
            const int f = col >> 1, part = col & 1;
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int rr = r0 + wr + 16 * i + 4 * (lane >> 4) + r;
                if (rr >= R) continue;
                const int n = k + p + 2 * rr;
                const double v = (double)acc[i][c][r];
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
        dim3 grid((unsigned)th_pad, (unsigned)((N + 1 + kFoldK - 1) / kFoldK), (unsigned)((C_pad + kFoldC - 1) / kFoldC));
        hipLaunchKernelGGL(k_s2_fold_x, grid, dim3(256), 0, s, G, nt, N, F, th, th_pad, C_pad, X);
        HAMLS_HIP(hipGetLastError());
    }
    const LegItem* items = (const LegItem*)P.d_leg_items;
    if (C_pad <= 32) {
        hipLaunchKernelGGL(k_s2_legendre_mfma<32>, dim3((unsigned)P.leg_items, 1), dim3(256), 0, s, P.d_ptab32,
                           P.d_tab_off, items, X, N, F, th_pad, C_pad, coeffs);
    } else if (C_pad <= 64) {
        hipLaunchKernelGGL(k_s2_legendre_mfma<64>, dim3((unsigned)P.leg_items, 1), dim3(256), 0, s, P.d_ptab32,
                           P.d_tab_off, items, X, N, F, th_pad, C_pad, coeffs);
    } else {
        hipLaunchKernelGGL(k_s2_legendre_mfma<128>, dim3((unsigned)P.leg_items, (unsigned)((C_pad + 127) / 128)),
                           dim3(256), 0, s, P.d_ptab32, P.d_tab_off, items, X, N, F, th_pad, C_pad, coeffs);
    }
    HAMLS_HIP(hipGetLastError());
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
            for (int rt = 0; rt < (R + kMfmaRows - 1) / kMfmaRows; rt++) {
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
