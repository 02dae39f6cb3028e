// transform.hip -- step 3 of Alg. 1 on SO(3) and T3, and the synthesis
// (evaluation of a harmonic expansion at points) on both (gfx950).
//
// Quadrature (eq. (25)) of real grid values, in separable passes:
//   T3   three axis DFTs, frequencies k - n/2 for k in [0, n), sign -1, the
//        last scaled by 1/n^3 (the equal weights of the periodic grid);
//   SO3  two axis DFTs per beta ring over alpha and gamma (sign +1, scaled by
//        the trapezoid weights 2 pi/n), giving G_t(k, k') for |k|, |k'| <= N,
//        then the Wigner-d contraction over the beta rings
//          fhat^n_{k,k'} = sum_t w_t c_n d^n_{k,k'}(beta_t) G_t(k, k'),
//        c_n = sqrt((2n + 1)/(8 pi^2)), w_t the Gauss-Legendre weights in
//        cos(beta) (Sec. 2.1, the SO(3) basis of Sec. 2.2).
#include <math.h>

#include "common.h"
#include "device_common.h"

namespace hamls {

// ---------------------------------------------------------------------------
// one axis of a separable DFT
// ---------------------------------------------------------------------------

// Lines (a, b) of the [A][nin][B] input are processed TL at a time: the tile
// of TL lines x nin complex values is staged in LDS (loads coalesced along b,
// or along the axis when B = 1), then each output (line, k) is a direct sum
// over the staged line with twiddles from an LDS table of exp(2 pi i e/nin).
__global__ __launch_bounds__(256) void k_dft_axis(const double* __restrict__ in, int real_in,
                                                  double* __restrict__ out, int64_t A, int nin,
                                                  int64_t B, int nout, int koff, double sign,
                                                  double scale, const double* __restrict__ tw, int TL) {
    extern __shared__ double lds[];
    double* stw = lds;                 // 2 nin: cos, sin interleaved
    double* tile = lds + 2 * nin;      // TL x (nin + 1) complex
    const int ldt = 2 * (nin + 1);
    const int tid = threadIdx.x;
    const int64_t nlines = A * B;
    const int64_t L0 = (int64_t)blockIdx.x * TL;
    for (int e = tid; e < nin; e += 256) {
        stw[2 * e] = tw[e];
        stw[2 * e + 1] = tw[nin + e];
    }
    for (int e = tid; e < TL * nin; e += 256) {
        int l, i;
        if (B > 1) {
            l = e % TL;
            i = e / TL;
        } else {
            i = e % nin;
            l = e / nin;
        }
        const int64_t L = L0 + l;
        double re = 0.0, im = 0.0;
        if (L < nlines) {
            const int64_t a = L / B, b = L - a * B;
            const int64_t addr = (a * nin + i) * B + b;
            if (real_in) {
                re = in[addr];
            } else {
                re = in[2 * addr];
                im = in[2 * addr + 1];
            }
        }
        tile[l * ldt + 2 * i] = re;
        tile[l * ldt + 2 * i + 1] = im;
    }
    __syncthreads();
    for (int e = tid; e < TL * nout; e += 256) {
        int l, k;
        if (B > 1) {
            l = e % TL;
            k = e / TL;
        } else {
            k = e % nout;
            l = e / nout;
        }
        const int64_t L = L0 + l;
        if (L >= nlines) continue;
        int step = (k - koff) % nin;
        if (step < 0) step += nin;
        const double* x = tile + l * ldt;
        double re = 0.0, im = 0.0;
        int ei = 0;
        for (int i = 0; i < nin; i++) {
            const double c = stw[2 * ei], s = sign * stw[2 * ei + 1];
            const double xr = x[2 * i], xi = x[2 * i + 1];
            re += xr * c - xi * s;
            im += xr * s + xi * c;
            ei += step;
            if (ei >= nin) ei -= nin;
        }
        const int64_t a = L / B, b = L - a * B;
        const int64_t o = (a * nout + k) * B + b;
        out[2 * o] = re * scale;
        out[2 * o + 1] = im * scale;
    }
}

hamls_status launch_dft_axis(const double* in, bool real_in, double* out, int64_t A, int nin,
                             int64_t B, int nout, int koff, double sign, double scale,
                             const double* tw, hipStream_t s) {
    if (nin < 1 || nout < 1 || A < 1 || B < 1) {
        set_error("dft axis: empty shape");
        return HAMLS_ERR_INVALID_ARG;
    }
    // lengths that factor into primes up to 19: the mixed-radix FFT
    if (fft_axis_fits(nin))
        return launch_fft_axis(in, real_in, out, A, nin, B, nout, koff, sign, scale, tw, s);
    // tile of at most 48 KiB
    int TL = (int)(49152 / (16 * (int64_t)(nin + 1)));
    TL = TL > 16 ? 16 : TL;
    if (TL < 1) {
        set_error("dft axis: length %d too large", nin);
        return HAMLS_ERR_UNSUPPORTED;
    }
    const int64_t nlines = A * B;
    const int64_t nblk = (nlines + TL - 1) / TL;
    if (nblk > 0x7fffffff) {
        set_error("dft axis: too many lines");
        return HAMLS_ERR_UNSUPPORTED;
    }
    size_t lds = sizeof(double) * (2 * (size_t)nin + (size_t)TL * 2 * (nin + 1));
    hipLaunchKernelGGL(k_dft_axis, dim3((unsigned)nblk), dim3(256), lds, s, in, real_in ? 1 : 0, out,
                       A, nin, B, nout, koff, sign, scale, tw, TL);
    HAMLS_HIP(hipGetLastError());
    return HAMLS_OK;
}

// ---------------------------------------------------------------------------
// Wigner d
// ---------------------------------------------------------------------------

// Index of (n, k, k') in the SO3 coefficient order: all (k, k') of degree n
// after those of lower degree, sum_{l<n} (2l+1)^2 = n (2n-1)(2n+1)/3.
__device__ __forceinline__ int64_t so3_index(int n, int k, int kp) {
    return (int64_t)n * (2 * n - 1) * (2 * n + 1) / 3 + (int64_t)(k + n) * (2 * n + 1) + (kp + n);
}

// d^{n0}_{k,k'}(beta) at n0 = max(|k|, |k'|), from the Wigner sum, which has a
// single term at the edge of the index range:
//   k  =  n0:  (-1)^(n0-k') sqrt(C(2n0, n0+k')) cos^(n0+k') sin^(n0-k')
//   k  = -n0:               sqrt(C(2n0, n0-k')) cos^(n0-k') sin^(n0+k')
//   k' =  n0:               sqrt(C(2n0, n0+k))  cos^(n0+k)  sin^(n0-k)
//   k' = -n0:  (-1)^(n0+k)  sqrt(C(2n0, n0-k))  cos^(n0-k)  sin^(n0+k)
// (powers of cos(beta/2), sin(beta/2)), evaluated in logarithms.
__device__ double wigner_edge(int k, int kp, double lc, double ls) {
    const int ak = k < 0 ? -k : k, akp = kp < 0 ? -kp : kp;
    const int n0 = ak > akp ? ak : akp;
    if (n0 == 0) return 1.0;
    int pc, ps, top;
    bool neg;
    if (k == n0) {
        pc = n0 + kp;
        ps = n0 - kp;
        top = n0 + kp;
        neg = ps & 1;
    } else if (k == -n0) {
        pc = n0 - kp;
        ps = n0 + kp;
        top = n0 - kp;
        neg = false;
    } else if (kp == n0) {
        pc = n0 + k;
        ps = n0 - k;
        top = n0 + k;
        neg = false;
    } else {
        pc = n0 - k;
        ps = n0 + k;
        top = n0 - k;
        neg = ps & 1;
    }
    const double lb =
        0.5 * (lgamma(2.0 * n0 + 1.0) - lgamma(top + 1.0) - lgamma(2.0 * n0 - top + 1.0));
    const double v = exp(lb + (pc ? pc * lc : 0.0) + (ps ? ps * ls : 0.0));
    return neg ? -v : v;
}

// d^{j+1} from d^j and d^{j-1} (fixed k, k'), the three-term recurrence in the
// degree; j = 0 only for k = k' = 0, where d^1_{00} = cos(beta).
__device__ __forceinline__ double wigner_next(int j, int k, int kp, double cb, double dj, double djm1) {
    if (j == 0) return cb;
    const double jj = j, kk = (double)k * k, pp = (double)kp * kp, kkp = (double)k * kp;
    const double a = (2.0 * jj + 1.0) * (jj * (jj + 1.0) * cb - kkp);
    const double b = (jj + 1.0) * sqrt((jj * jj - kk) * (jj * jj - pp));
    const double c = jj * sqrt(((jj + 1.0) * (jj + 1.0) - kk) * ((jj + 1.0) * (jj + 1.0) - pp));
    return (a * dj - b * djm1) / c;
}

// Table [ring t][coefficient] = w_t c_n d^n_{k,k'}(beta_t); one thread per
// (k, k') and ring, the recurrence running over the degree.
__global__ __launch_bounds__(256) void k_wigner_table(int N, const double* __restrict__ beta,
                                                      const double* __restrict__ wts, int64_t ncoef,
                                                      double* __restrict__ tab) {
    const int K2 = 2 * N + 1;
    const int pair = blockIdx.x * blockDim.x + threadIdx.x;
    const int t = blockIdx.y;
    if (pair >= K2 * K2) return;
    const int k = pair / K2 - N, kp = pair % K2 - N;
    const double b = beta[t], w = wts[t];
    const double cb = cos(b), lc = log(cos(0.5 * b)), ls = log(sin(0.5 * b));
    const int ak = k < 0 ? -k : k, akp = kp < 0 ? -kp : kp;
    const int n0 = ak > akp ? ak : akp;
    double d = wigner_edge(k, kp, lc, ls), dm = 0.0;
    double* row = tab + (int64_t)t * ncoef;
    for (int n = n0;; n++) {
        row[so3_index(n, k, kp)] = w * sqrt((2.0 * n + 1.0) / (8.0 * kPi * kPi)) * d;
        if (n == N) break;
        const double nx = wigner_next(n, k, kp, cb, d, dm);
        dm = d;
        d = nx;
    }
}

hamls_status launch_wigner_table(const Plan& P, const double* beta, const double* wts, hipStream_t s) {
    const int K2 = 2 * P.N + 1;
    dim3 grid((unsigned)((K2 * K2 + 255) / 256), (unsigned)P.dims[0]);
    hipLaunchKernelGGL(k_wigner_table, grid, dim3(256), 0, s, P.N, beta, wts, P.ncoef, P.d_wtab);
    HAMLS_HIP(hipGetLastError());
    return HAMLS_OK;
}

// fhat[f][(n, k, k')] = sum_t tab[t][(n, k, k')] G[f][t][k + N][k' + N]; one
// thread per coefficient, FB fields per pass sharing the table loads.
template <int FB>
__global__ __launch_bounds__(256) void k_so3_contract(const double* __restrict__ tab,
                                                      const double* __restrict__ G, int F, int f0,
                                                      int N, int nb, int64_t ncoef,
                                                      double* __restrict__ coeffs) {
    const int n = blockIdx.y;
    const int K2n = 2 * n + 1;
    const int pair = blockIdx.x * blockDim.x + threadIdx.x;
    if (pair >= K2n * K2n) return;
    const int k = pair / K2n - n, kp = pair % K2n - n;
    const int K2 = 2 * N + 1;
    const int64_t id = so3_index(n, k, kp);
    const int64_t gofs = (int64_t)(k + N) * K2 + (kp + N);
    const int64_t ring = (int64_t)K2 * K2;
    const int nf = F - f0 < FB ? F - f0 : FB;
    double re[FB], im[FB];
#pragma unroll
    for (int f = 0; f < FB; f++) {
        re[f] = 0.0;
        im[f] = 0.0;
    }
    for (int t = 0; t < nb; t++) {
        const double v = tab[(int64_t)t * ncoef + id];
#pragma unroll
        for (int f = 0; f < FB; f++) {
            if (f < nf) {
                const double* g = G + 2 * (((int64_t)(f0 + f) * nb + t) * ring + gofs);
                re[f] = fma(v, g[0], re[f]);
                im[f] = fma(v, g[1], im[f]);
            }
        }
    }
#pragma unroll
    for (int f = 0; f < FB; f++) {
        if (f < nf) {
            coeffs[2 * ((int64_t)(f0 + f) * ncoef + id)] = re[f];
            coeffs[2 * ((int64_t)(f0 + f) * ncoef + id) + 1] = im[f];
        }
    }
}

hamls_status launch_so3_contract(const Plan& P, const double* G, int F, double* coeffs, hipStream_t s) {
    constexpr int FB = 4;
    const int K2 = 2 * P.N + 1;
    for (int f0 = 0; f0 < F; f0 += FB) {
        dim3 grid((unsigned)((K2 * K2 + 255) / 256), (unsigned)(P.N + 1));
        hipLaunchKernelGGL(k_so3_contract<FB>, grid, dim3(256), 0, s, P.d_wtab, G, F, f0, P.N,
                           P.dims[0], P.ncoef, coeffs);
    }
    HAMLS_HIP(hipGetLastError());
    return HAMLS_OK;
}

// ---------------------------------------------------------------------------
// synthesis
// ---------------------------------------------------------------------------

__device__ __forceinline__ double block_sum256(double v, double* red) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    return red[0] + red[1] + red[2] + red[3];
}

// SO3: f(R) = Re sum fhat^n_{k,k'} c_n d^n_{k,k'}(beta) e^{-i(k alpha + k' gamma)},
// one block per point; the Euler angles come from the quaternion
// q = (cos(b/2) cos((a+g)/2), -sin(b/2) sin((a-g)/2), sin(b/2) cos((a-g)/2),
//      cos(b/2) sin((a+g)/2)).
__global__ __launch_bounds__(256) void k_so3_eval(const double* __restrict__ coeffs, int F, int N,
                                                  int64_t ncoef, const double* __restrict__ pts,
                                                  int64_t npts, double* __restrict__ out) {
    __shared__ double red[4];
    const int64_t i = blockIdx.x;
    const double* q = pts + 4 * i;
    const double be = 2.0 * atan2(sqrt(q[1] * q[1] + q[2] * q[2]), sqrt(q[0] * q[0] + q[3] * q[3]));
    const double sp = atan2(q[3], q[0]), dm = atan2(-q[1], q[2]);
    const double al = sp + dm, ga = sp - dm;
    const double cb = cos(be), lc = log(cos(0.5 * be)), ls = log(sin(0.5 * be));
    const int K2 = 2 * N + 1;
    for (int f = 0; f < F; f++) {
        double acc = 0.0;
        for (int pair = threadIdx.x; pair < K2 * K2; pair += 256) {
            const int k = pair / K2 - N, kp = pair % K2 - N;
            const int ak = k < 0 ? -k : k, akp = kp < 0 ? -kp : kp;
            const int n0 = ak > akp ? ak : akp;
            double ph = -((double)k * al + (double)kp * ga);
            double cph = cos(ph), sph = sin(ph);
            double d = wigner_edge(k, kp, lc, ls), dmv = 0.0;
            for (int n = n0;; n++) {
                const double* c = coeffs + 2 * ((int64_t)f * ncoef + so3_index(n, k, kp));
                acc += sqrt((2.0 * n + 1.0) / (8.0 * kPi * kPi)) * d * (c[0] * cph - c[1] * sph);
                if (n == N) break;
                const double nx = wigner_next(n, k, kp, cb, d, dmv);
                dmv = d;
                d = nx;
            }
        }
        const double tot = block_sum256(acc, red);
        if (threadIdx.x == 0) out[(int64_t)f * npts + i] = tot;
    }
}

hamls_status launch_so3_eval(const Plan& P, const double* coeffs, int F, const double* pts,
                             int64_t npts, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_so3_eval, dim3((unsigned)npts), dim3(256), 0, s, coeffs, F, P.N, P.ncoef, pts,
                       npts, out);
    HAMLS_HIP(hipGetLastError());
    return HAMLS_OK;
}

// T3: f(x) = Re sum_k fhat_k e^{2 pi i k.x}, k in [-n/2, n - n/2)^3, one block
// per point with the per-axis factors in LDS.
__global__ __launch_bounds__(256) void k_t3_eval(const double* __restrict__ coeffs, int F, int n,
                                                 const double* __restrict__ pts, int64_t npts,
                                                 double* __restrict__ out) {
    extern __shared__ double e3[];  // 3 x n complex
    __shared__ double red[4];
    const int64_t i = blockIdx.x;
    const int h = n / 2;
    for (int e = threadIdx.x; e < 3 * n; e += 256) {
        const int ax = e / n, k = e % n;
        double s, c;
        sincos(2.0 * kPi * ((double)(k - h) * pts[3 * i + ax]), &s, &c);
        e3[2 * e] = c;
        e3[2 * e + 1] = s;
    }
    __syncthreads();
    const int64_t nc = (int64_t)n * n * n;
    for (int f = 0; f < F; f++) {
        double acc = 0.0;
        for (int ab = threadIdx.x; ab < n * n; ab += 256) {
            const int a = ab / n, b = ab % n;
            const double ar = e3[2 * a], ai = e3[2 * a + 1];
            const double br = e3[2 * (n + b)], bi = e3[2 * (n + b) + 1];
            const double pr = ar * br - ai * bi, pi = ar * bi + ai * br;
            const double* cf = coeffs + 2 * ((int64_t)f * nc + (int64_t)ab * n);
            for (int c = 0; c < n; c++) {
                const double cr = e3[2 * (2 * n + c)], ci = e3[2 * (2 * n + c) + 1];
                const double er = pr * cr - pi * ci, ei = pr * ci + pi * cr;
                acc += cf[2 * c] * er - cf[2 * c + 1] * ei;
            }
        }
        const double tot = block_sum256(acc, red);
        if (threadIdx.x == 0) out[(int64_t)f * npts + i] = tot;
    }
}

hamls_status launch_t3_eval(const Plan& P, const double* coeffs, int F, const double* pts,
                            int64_t npts, double* out, hipStream_t s) {
    const int n = P.dims[0];
    hipLaunchKernelGGL(k_t3_eval, dim3((unsigned)npts), dim3(256), sizeof(double) * 6 * n, s, coeffs, F, n,
                       pts, npts, out);
    HAMLS_HIP(hipGetLastError());
    return HAMLS_OK;
}

}  // namespace hamls
