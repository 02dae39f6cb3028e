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
// of one block per workgroup: the K = th_pad reduction runs in chunks of 32
// rings staged in LDS (double-buffered, one barrier per chunk; the next
// chunk's global loads in flight during the current chunk's MFMAs), and each of
// the four waves accumulates its share in 32 x 32 tiles of
// v_mfma_f32_32x32x2f32 (FP32 accumulate).
#include "common.h"
#include "device_common.h"

namespace hamls {


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

constexpr int kMfmaRows = 64;  // rows per workgroup tile
constexpr int kMfmaTK = 32;    // rings per LDS chunk

typedef float f32x16 __attribute__((ext_vector_type(16)));

// Waves of the contraction's workgroup: two 32-row halves of the 64-row tile
// times CW / 64 column groups (at least one).
constexpr int mfma_waves(int CW) { return 2 * (CW >= 128 ? CW / 64 : 1); }

// One workgroup (64 mfma_waves(CW) threads) per (item, column chunk of CW):
// rows [64 rt, 64 rt + 64) of block (k, p) against columns [cw0, cw0 + CW).
// Each wave owns one 32-row half and CW / WC columns, and accumulates
// 1 x TC tiles of v_mfma_f32_32x32x2f32 (A 32x2, B 2x32, D 32x32 FP32: lane l
// holds A[l % 32][l / 32], B[l / 32][l % 32] and
// D[8 (v / 4) + 4 (l / 32) + v % 4][l % 32] in accumulator v < 16).  The
// K = th_pad reduction runs in chunks of 32 rings staged in LDS, double
// buffered: the next chunk's 16-byte global loads are in flight in registers
// during the current chunk's MFMAs, then stored to the other buffer.
template <int CW>
__global__ __launch_bounds__(256) void k_s2_legendre_mfma(const float* __restrict__ tab,
                                                         const int64_t* __restrict__ tab_off,
                                                         const LegItem* __restrict__ items,
                                                         const float* __restrict__ X, int N, int F, int th_pad,
                                                         int C_pad, float* __restrict__ out) {
    constexpr int NW = mfma_waves(CW);
    constexpr int NT = 64 * NW;                 // threads
    constexpr int WR = 2;                       // waves along the rows
    constexpr int WC = NW / WR;                 // waves along the columns
    constexpr int TR = kMfmaRows / WR / 32;     // 32-row MFMA tiles per wave
    constexpr int TC = CW / WC / 32;            // 32-column MFMA tiles per wave
    static_assert(TR == 1 && TC >= 1 && TC * 32 * WC == CW, "wave tile");
    __shared__ __align__(16) float As[2][kMfmaTK * kMfmaRows];
    __shared__ __align__(16) float Bs[2][kMfmaTK * CW];
    const LegItem it = items[blockIdx.x];
    const int k = it.k, p = it.p;
    const int cw0 = blockIdx.y * CW;
    const int R = N >= k + p ? (N - k - p) / 2 + 1 : 0;
    const int R_pad = (R + 15) & ~15;
    const int r0 = it.rt * kMfmaRows;
    const float* A = tab + tab_off[2 * k + p];
    const float* B = X + ((int64_t)(2 * k + p) * th_pad) * C_pad;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = (w / WC) * (kMfmaRows / WR), wc = (w % WC) * (CW / WC);
    const int nchunk = (th_pad + kMfmaTK - 1) / kMfmaTK;

    constexpr int NA = kMfmaTK * kMfmaRows / 4 / NT;  // float4 of A per thread
    constexpr int NBv = kMfmaTK * CW / 4 / NT;        // float4 of B per thread
    static_assert(NA * NT * 4 == kMfmaTK * kMfmaRows && NBv * NT * 4 == kMfmaTK * CW, "chunk split");
    float4 ra[NA], rb[NBv];
    auto gload = [&](int q) {
        const int t0 = q * kMfmaTK;
#pragma unroll
        for (int v = 0; v < NA; v++) {
            const int e = (tid + NT * v) * 4;
            const int tt = e / kMfmaRows, rr = e - tt * kMfmaRows;
            const int t = t0 + tt, r = r0 + rr;
            ra[v] = (t < th_pad && r < R_pad) ? *(const float4*)(A + (int64_t)t * R_pad + r)
                                              : float4{0.0f, 0.0f, 0.0f, 0.0f};
        }
#pragma unroll
        for (int v = 0; v < NBv; v++) {
            const int e = (tid + NT * v) * 4;
            const int tt = e / CW, cc = e - tt * CW;
            const int t = t0 + tt, c = cw0 + cc;
            rb[v] = (t < th_pad && c < C_pad) ? *(const float4*)(B + (int64_t)t * C_pad + c)
                                              : float4{0.0f, 0.0f, 0.0f, 0.0f};
        }
    };
    auto lstore = [&](int buf) {
#pragma unroll
        for (int v = 0; v < NA; v++) {
            const int e = (tid + NT * v) * 4;
            *(float4*)(As[buf] + e) = ra[v];
        }
#pragma unroll
        for (int v = 0; v < NBv; v++) {
            const int e = (tid + NT * v) * 4;
            *(float4*)(Bs[buf] + e) = rb[v];
        }
    };

    f32x16 acc[TR][TC];
#pragma unroll
    for (int i = 0; i < TR; i++)
#pragma unroll
        for (int c = 0; c < TC; c++)
#pragma unroll
            for (int v = 0; v < 16; v++) acc[i][c][v] = 0.0f;

    gload(0);
    lstore(0);
    __syncthreads();
    for (int q = 0; q < nchunk; q++) {
        const int buf = q & 1;
        if (q + 1 < nchunk) gload(q + 1);
        const float* as = As[buf];
        const float* bs = Bs[buf];
        const int kmax = th_pad - q * kMfmaTK;  // rings of this chunk (a multiple of 4)
#pragma unroll
        for (int tk = 0; tk < kMfmaTK; tk += 2) {
            if (tk >= kmax) break;
            const int kr = tk + (lane >> 5);
            float a[TR], b[TC];
#pragma unroll
            for (int i = 0; i < TR; i++) a[i] = as[kr * kMfmaRows + wr + 32 * i + (lane & 31)];
#pragma unroll
            for (int c = 0; c < TC; c++) b[c] = bs[kr * CW + wc + 32 * c + (lane & 31)];
#pragma unroll
            for (int i = 0; i < TR; i++)
#pragma unroll
                for (int c = 0; c < TC; c++)
                    acc[i][c] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i], b[c], acc[i][c], 0, 0, 0);
        }
        // the other buffer was last read before the previous barrier
        if (q + 1 < nchunk) lstore(buf ^ 1);
        __syncthreads();
    }

    // the tile in the block's own order, [row < R_pad][2F columns] from the
    // block's first row at tab_off / th_pad: lanes 0-31 write 32 consecutive
    // columns of one row (k_s2_unfold scatters it into the coefficients)
    float* o = out + tab_off[2 * k + p] / th_pad * (2 * F);
#pragma unroll
    for (int i = 0; i < TR; i++)
#pragma unroll
        for (int c = 0; c < TC; c++) {
            const int col = cw0 + wc + 32 * c + (lane & 31);
            if (col >= 2 * F) continue;
#pragma unroll
            for (int v = 0; v < 16; v++) {
                const int rr = r0 + wr + 32 * i + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                if (rr < R) o[(int64_t)rr * (2 * F) + col] = acc[i][c][v];
            }
        }
}

// Fields per workgroup of k_s2_unfold.
constexpr int kUnfoldF = 8;

// Orders per LDS stage of k_s2_unfold.
constexpr int kUnfoldK = 256;

// The contraction's blocks (FP32, [row][2F] per (k, p), row r <-> degree
// n = k + p + 2r) into the coefficient layout.  Workgroup (n, field chunk)
// stages kUnfoldK orders k >= 0 of degree n at a time in LDS (one row of
// block (k, (n - k) mod 2) each: 2 kUnfoldF consecutive floats), then
// writes, field by field, the two contiguous runs of (n, +k) and (n, -k),
// with fhat_{n,-k} = (-1)^k conj(fhat_{n,k}).
__global__ __launch_bounds__(256) void k_s2_unfold(const float* __restrict__ blk, const int64_t* __restrict__ tab_off,
                                                  int N, int F, int th_pad, double* __restrict__ coeffs) {
    constexpr int cols = 2 * kUnfoldF;
    __shared__ float v[kUnfoldK * cols];
    const int n = blockIdx.x;
    const int f0 = blockIdx.y * kUnfoldF;
    const int nf = min(kUnfoldF, F - f0);
    const int64_t nc = (int64_t)(N + 1) * (N + 1);
    for (int k0 = 0; k0 <= n; k0 += kUnfoldK) {
        const int nk = min(kUnfoldK, n + 1 - k0);
        for (int e = threadIdx.x; e < nk * cols; e += blockDim.x) {
            const int kl = e / cols, c = e - kl * cols;
            const int k = k0 + kl;
            const int p = (n - k) & 1, rr = (n - k) >> 1;
            float x = 0.0f;
            if (c < 2 * nf) x = blk[tab_off[2 * k + p] / th_pad * (2 * F) + (int64_t)rr * (2 * F) + 2 * f0 + c];
            v[e] = x;
        }
        __syncthreads();
        // per field: entries (k, part) for k in [k0, k0 + nk), then -k
        for (int e = threadIdx.x; e < nf * nk * 4; e += blockDim.x) {
            const int fl = e / (4 * nk), rem = e - fl * 4 * nk;
            const int neg = rem >= 2 * nk;
            const int r2 = neg ? rem - 2 * nk : rem;
            const int kl = r2 >> 1, part = r2 & 1;
            const int k = k0 + kl;
            if (neg && k == 0) continue;
            double x = (double)v[kl * cols + 2 * fl + part];
            if (neg && (((k & 1) != 0) != (part == 1))) x = -x;
            const int64_t idx = (int64_t)n * n + n + (neg ? -k : k);
            coeffs[((int64_t)(f0 + fl) * nc + idx) * 2 + part] = x;
        }
        __syncthreads();
    }
}

// Size (floats) of the contraction's block-ordered output: sum over the
// (k, p) blocks of R_pad rows x 2F.
int64_t s2_mfma_out_len(int N, int F) {
    int64_t rows = 0;
    for (int k = 0; k <= N; k++)
        for (int p = 0; p < 2; p++) {
            const int R = N >= k + p ? (N - k - p) / 2 + 1 : 0;
            rows += (R + 15) & ~15;
        }
    return rows * 2 * F;
}

// Step 3 of the mixed path in three launches: the fold of the ring spectra G
// (FP64) into X (FP32 blocks), the matrix-core contraction, whose
// block-ordered output goes to G's memory (consumed by then; the work size
// provides for both), and the unfold into the coefficients.
static void mfma_dims(const Plan& P, int F, int& th, int& th_pad, int& C_pad) {
    th = (P.dims[0] + 1) / 2;
    th_pad = (th + 3) & ~3;
    C_pad = ((2 * F + 15) / 16) * 16;
}

hamls_status launch_s2_fold(const Plan& P, int F, const double* G, int64_t glen, float* X, int64_t xcap,
                            hipStream_t s) {
    int th, th_pad, C_pad;
    mfma_dims(P, F, th, th_pad, C_pad);
    const int N = P.N;
    const int64_t xlen = (int64_t)(N + 1) * 2 * th_pad * C_pad;
    if (xlen > xcap || s2_mfma_out_len(N, F) > 2 * glen) {
        set_error("fold or contraction buffer too small");
        return HAMLS_ERR_INVALID_ARG;
    }
    dim3 grid((unsigned)th_pad, (unsigned)((N + 1 + kFoldK - 1) / kFoldK), (unsigned)((C_pad + kFoldC - 1) / kFoldC));
    hipLaunchKernelGGL(k_s2_fold_x, grid, dim3(256), 0, s, G, P.dims[0], N, F, th, th_pad, C_pad, X);
    HAMLS_HIP(hipGetLastError());
    return HAMLS_OK;
}

hamls_status launch_s2_legendre_mfma(const Plan& P, int F, const float* X, float* out, hipStream_t s) {
    int th, th_pad, C_pad;
    mfma_dims(P, F, th, th_pad, C_pad);
    const int N = P.N;
    const LegItem* items = (const LegItem*)P.d_leg_items;
    if (C_pad <= 32) {
        hipLaunchKernelGGL(k_s2_legendre_mfma<32>, dim3((unsigned)P.leg_items, 1), dim3(64 * mfma_waves(32)), 0, s,
                           P.d_ptab32, P.d_tab_off, items, X, N, F, th_pad, C_pad, out);
    } else if (C_pad <= 64) {
        hipLaunchKernelGGL(k_s2_legendre_mfma<64>, dim3((unsigned)P.leg_items, 1), dim3(64 * mfma_waves(64)), 0, s,
                           P.d_ptab32, P.d_tab_off, items, X, N, F, th_pad, C_pad, out);
    } else {
        hipLaunchKernelGGL(k_s2_legendre_mfma<128>, dim3((unsigned)P.leg_items, (unsigned)((C_pad + 127) / 128)),
                           dim3(64 * mfma_waves(128)), 0, s, P.d_ptab32, P.d_tab_off, items, X, N, F, th_pad, C_pad,
                           out);
    }
    HAMLS_HIP(hipGetLastError());
    return HAMLS_OK;
}

hamls_status launch_s2_unfold(const Plan& P, int F, const float* out, double* coeffs, hipStream_t s) {
    int th, th_pad, C_pad;
    mfma_dims(P, F, th, th_pad, C_pad);
    hipLaunchKernelGGL(k_s2_unfold, dim3((unsigned)(P.N + 1), (unsigned)((F + kUnfoldF - 1) / kUnfoldF)), dim3(256),
                       0, s, out, P.d_tab_off, P.N, F, th_pad, coeffs);
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
