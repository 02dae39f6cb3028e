// fft.hip -- mixed-radix FFTs along one axis of a strided array (step 3 of
// Alg. 1: the periodic-angle transforms of Sec. 2.1 on S2, SO(3) and T3).
//
// A line of n complex values is transformed in LDS by Stockham's self-sorting
// formulation: n = r_0 r_1 ... r_{S-1} (radices 2..19), and stage s (span
// Ns = r_0 ... r_{s-1}) maps buffer a to buffer b by, for every j < n/r,
//   v_q = a[j + q n/r] * W(q (j mod Ns) n/(Ns r)),   q < r,
//   b[(j div Ns) Ns r + (j mod Ns) + p Ns] = sum_q v_q W((p q mod r) n/r),
// with W(e) = exp(sign 2 pi i e / n) from the plan's twiddle table of
// cos / sin(2 pi e / n).  After the last stage b holds
//   X_k = sum_j x_j W(j k)
// in natural order.  Work per line ~ n (r_0 + ... + r_{S-1}) complex
// multiply-adds against n^2 for the direct sum.
#include "common.h"
#include "device_common.h"

namespace hamls {

template <class T>
struct cplx {
    T re, im;
};


// X_p = sum_q v_q w^(p q), w = exp(sign 2 pi i / R), for R = 2, 4, 8: the
// even and odd halves transformed at R/2 and joined by the roots
// w^p (w^(p + R/2) = -w^p).
template <class T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> x, cplx<T> y) { return {x.re + y.re, x.im + y.im}; }
template <class T>
__device__ __forceinline__ cplx<T> csub(cplx<T> x, cplx<T> y) { return {x.re - y.re, x.im - y.im}; }
// x times sign i
template <class T>
__device__ __forceinline__ cplx<T> cmul_i(cplx<T> x, T sign) { return {-sign * x.im, sign * x.re}; }
template <int R, class T>
__device__ __forceinline__ void fft_small(const cplx<T>* v, cplx<T>* X, T sign) {
    if constexpr (R == 2) {
        X[0] = cadd(v[0], v[1]);
        X[1] = csub(v[0], v[1]);
    } else if constexpr (R == 4) {
        const cplx<T> a = cadd(v[0], v[2]), bb = csub(v[0], v[2]);
        const cplx<T> c = cadd(v[1], v[3]), d = cmul_i(csub(v[1], v[3]), sign);
        X[0] = cadd(a, c);
        X[2] = csub(a, c);
        X[1] = cadd(bb, d);
        X[3] = csub(bb, d);
    } else {
        const cplx<T> ve[4] = {v[0], v[2], v[4], v[6]}, vo[4] = {v[1], v[3], v[5], v[7]};
        cplx<T> E[4], O[4];
        fft_small<4, T>(ve, E, sign);
        fft_small<4, T>(vo, O, sign);
        const T h = (T)0.70710678118654752440;  // sqrt(1/2)
        // w^1 O_1, w^2 O_2, w^3 O_3 with w = (1 + sign i) / sqrt(2)
        const cplx<T> o1 = {h * (O[1].re - sign * O[1].im), h * (O[1].im + sign * O[1].re)};
        const cplx<T> o2 = cmul_i(O[2], sign);
        const cplx<T> o3 = {-h * (O[3].re + sign * O[3].im), h * (sign * O[3].re - O[3].im)};
        X[0] = cadd(E[0], O[0]);
        X[4] = csub(E[0], O[0]);
        X[1] = cadd(E[1], o1);
        X[5] = csub(E[1], o1);
        X[2] = cadd(E[2], o2);
        X[6] = csub(E[2], o2);
        X[3] = cadd(E[3], o3);
        X[7] = csub(E[3], o3);
    }
}

// One radix-R Stockham butterfly (see the file comment); tw holds cos at
// [e] and sin at [n + e] (FP64 in LDS, rounded to T on use).
template <int R, class T>
__device__ __forceinline__ void fft_butterfly(const cplx<T>* __restrict__ a, cplx<T>* __restrict__ b, int j,
                                              int Ns, float rNs, int tsc, int n, const double* __restrict__ tw,
                                              T sign) {
    const int m = n / R;
    const int jq = div_small(j, Ns, rNs);  // j div Ns
    const int jj = j - jq * Ns;             // j mod Ns
    const int tstep = jj * tsc;             // tsc = n / (Ns R)
    cplx<T> v[R];
#pragma unroll
    for (int q = 0; q < R; q++) {
        const cplx<T> x = a[j + q * m];
        int e = q * tstep;  // < n: q < R, jj < Ns
        const T c = (T)tw[e], s = sign * (T)tw[n + e];
        v[q].re = x.re * c - x.im * s;
        v[q].im = x.re * s + x.im * c;
    }
    const int d0 = jq * Ns * R + jj;
    if constexpr (R == 2 || R == 4 || R == 8) {
        // the R-point DFT factored into radix-2 steps: its roots are 1, +-i
        // and (+-1 +- i)/sqrt(2), so it takes additions and four
        // multiplications instead of the (R - 1)^2 complex products below
        cplx<T> X[R];
        fft_small<R, T>(v, X, sign);
#pragma unroll
        for (int p = 0; p < R; p++) b[d0 + p * Ns] = X[p];
        return;
    }
    // outputs one at a time for the larger radices (register pressure)
    constexpr int kUnrollOut = R <= 8 ? R : 1;
#pragma unroll kUnrollOut
    for (int p = 0; p < R; p++) {
        T re = v[0].re, im = v[0].im;
#pragma unroll
        for (int q = 1; q < R; q++) {
            const int e = ((p * q) % R) * m;
            const T c = (T)tw[e], s = sign * (T)tw[n + e];
            re += v[q].re * c - v[q].im * s;
            im += v[q].re * s + v[q].im * c;
        }
        b[d0 + p * Ns] = cplx<T>{re, im};
    }
}

template <class T>
__device__ __forceinline__ void fft_stage(int R, const cplx<T>* a, cplx<T>* b, int j, int Ns, float rNs, int tsc,
                                          int n, const double* tw, T sign) {
    switch (R) {
#define HAMLS_FFT_CASE(RR) \
    case RR:               \
        fft_butterfly<RR, T>(a, b, j, Ns, rNs, tsc, n, tw, sign); \
        break;
        HAMLS_FFT_CASE(2)
        HAMLS_FFT_CASE(3)
        HAMLS_FFT_CASE(4)
        HAMLS_FFT_CASE(5)
        HAMLS_FFT_CASE(7)
        HAMLS_FFT_CASE(8)
        HAMLS_FFT_CASE(11)
        HAMLS_FFT_CASE(13)
        HAMLS_FFT_CASE(17)
        HAMLS_FFT_CASE(19)
#undef HAMLS_FFT_CASE
        default:
            break;
    }
}

// The TL lines staged at a (row stride ld complex values) are transformed;
// returns the buffer that holds the result (a or b).  Block-cooperative: all
// threads of the block call it.
template <class T>
__device__ cplx<T>* fft_lines(cplx<T>* a, cplx<T>* b, int TL, int ld, int n, const FftPlan& fp,
                              const double* tw, T sign) {
    int Ns = 1;
    for (int s = 0; s < fp.nst; s++) {
        const int R = fp.rad[s];
        const int per = n / R;
        const float rper = 1.0f / (float)per, rNs = 1.0f / (float)Ns;
        const int tsc = n / (Ns * R);
        for (int e = threadIdx.x; e < TL * per; e += blockDim.x) {
            const int l = div_small(e, per, rper), j = e - l * per;
            fft_stage<T>(R, a + l * ld, b + l * ld, j, Ns, rNs, tsc, n, tw, sign);
        }
        __syncthreads();
        cplx<T>* t = a;
        a = b;
        b = t;
        Ns *= R;
    }
    return a;
}

// Lines (a, b) of the [A][nin][B] input (real or complex FP64), TL per
// block: out[(a nout + k) B + b] = scale X_{(k - koff) mod nin}.
// Real input is transformed in pairs: lines l and l + TL/2 of the block go
// into one complex line z = x_l + i x_{l+TL/2}, and X_l(k) = (Z_k + conj
// Z_{-k}) / 2, X_{l+TL/2}(k) = (Z_k - conj Z_{-k}) / (2i).  Strided lines
// (B > 1) are loaded TL consecutive b at a time (128-byte segments for TL =
// 16 real or 8 complex lines).
__global__ __launch_bounds__(256) void k_fft_axis(const double* __restrict__ in, int real_in,
                                                  double* __restrict__ out, int64_t A, int nin, int64_t B,
                                                  int nout, int koff, double sign, double scale,
                                                  const double* __restrict__ tw, int TL, FftPlan fp) {
    extern __shared__ double lds[];
    double* stw = lds;  // cos [nin], sin [nin]
    cplx<double>* buf0 = (cplx<double>*)(lds + 2 * nin);
    const int ld = nin + 1;
    const int NL = real_in ? TL / 2 : TL;  // complex lines transformed
    cplx<double>* buf1 = buf0 + (int64_t)NL * ld;
    const int tid = threadIdx.x;
    const int64_t nlines = A * B;
    const int64_t L0 = (int64_t)blockIdx.x * TL;
    // TL and NL are powers of two (8 or 16 lines; 4, 8 or 16 transforms)
    const int lgTL = 31 - __clz(TL), lgNL = 31 - __clz(NL);
    const float rnin = 1.0f / (float)nin, rnout = 1.0f / (float)nout;
    // line L = (a, b) of the [A][B] lines: L0's split once, then b0 + l < B + TL
    const int64_t a0 = L0 / B, b0 = L0 - a0 * B;
    const float rB = B < (1 << 24) ? 1.0f / (float)B : 0.0f;
    auto split = [&](int l, int64_t& a, int64_t& b) {
        b = b0 + l;
        a = a0;
        if (b >= B) {
            const int64_t w = B < (1 << 24) ? (int64_t)div_small((int)b, (int)B, rB) : b / B;
            a += w;
            b -= w * B;
        }
    };
    for (int e = tid; e < 2 * nin; e += blockDim.x) stw[e] = tw[e];
    for (int e = tid; e < TL * nin; e += blockDim.x) {
        int l, i;
        if (B > 1) {
            l = e & (TL - 1);
            i = e >> lgTL;
        } else {
            l = div_small(e, nin, rnin);
            i = e - l * nin;
        }
        const int64_t L = L0 + l;
        double re = 0.0, im = 0.0;
        if (L < nlines) {
            int64_t a, b;
            split(l, a, b);
            const int64_t addr = (a * nin + i) * B + b;
            if (real_in) {
                re = in[addr];
            } else {
                re = in[2 * addr];
                im = in[2 * addr + 1];
            }
        }
        if (real_in) {
            // line l < NL: real part; line l >= NL: imaginary part of line l - NL
            double* slot = (double*)&buf0[(l & (NL - 1)) * ld + i];
            slot[l >> lgNL] = re;
        } else {
            buf0[l * ld + i] = cplx<double>{re, im};
        }
    }
    __syncthreads();
    const cplx<double>* X = fft_lines<double>(buf0, buf1, NL, ld, nin, fp, stw, sign);
    for (int e = tid; e < TL * nout; e += blockDim.x) {
        int l, k;
        if (B > 1) {
            l = e & (TL - 1);
            k = e >> lgTL;
        } else {
            l = div_small(e, nout, rnout);
            k = e - l * nout;
        }
        const int64_t L = L0 + l;
        if (L >= nlines) continue;
        int f = k - koff;
        if (f < 0 || f >= nin) {
            f %= nin;
            if (f < 0) f += nin;
        }
        cplx<double> x;
        if (real_in) {
            const cplx<double> z = X[(l & (NL - 1)) * ld + f];
            const cplx<double> c = X[(l & (NL - 1)) * ld + (f == 0 ? 0 : nin - f)];  // Z_{-k}
            if (l < NL)
                x = cplx<double>{0.5 * (z.re + c.re), 0.5 * (z.im - c.im)};
            else
                x = cplx<double>{0.5 * (z.im + c.im), -0.5 * (z.re - c.re)};
        } else {
            x = X[l * ld + f];
        }
        int64_t a, b;
        split(l, a, b);
        const int64_t o = (a * nout + k) * B + b;
        out[2 * o] = x.re * scale;
        out[2 * o + 1] = x.im * scale;
    }
}

// S2 ring transforms by pairs of mirrored rings (t, nt-1-t): z = g_t + i g_t'
// is transformed once and split by Z_k = G_t(k) + i G_t'(k) with
// G(-k) = conj G(k) for real rings:
//   G_t(k) = (Z_k + conj Z_{-k}) / 2,  G_t'(k) = (Z_k - conj Z_{-k}) / (2i),
// for k = 0..N, scaled by 2 pi / n_phi, sign -1 (e^{-ik phi}).  The equator
// ring of an odd nt is transformed alone.  Output G[f][ring][k] (complex).
__global__ __launch_bounds__(256) void k_s2_ring_fft(const double* __restrict__ gv, int64_t MQ, int nt, int np,
                                                     int N, const double* __restrict__ tw, FftPlan fp,
                                                     double* __restrict__ G) {
    extern __shared__ double lds[];
    double* stw = lds;
    cplx<double>* buf0 = (cplx<double>*)(lds + 2 * np);
    cplx<double>* buf1 = buf0 + (np + 1);
    const int t = blockIdx.x, f = blockIdx.y;
    const int t2 = nt - 1 - t;
    for (int e = threadIdx.x; e < 2 * np; e += blockDim.x) stw[e] = tw[e];
    const double* r1 = gv + (int64_t)f * MQ + (int64_t)t * np;
    const double* r2 = gv + (int64_t)f * MQ + (int64_t)t2 * np;
    for (int p = threadIdx.x; p < np; p += blockDim.x)
        buf0[p] = cplx<double>{r1[p], t2 != t ? r2[p] : 0.0};
    __syncthreads();
    const cplx<double>* Z = fft_lines<double>(buf0, buf1, 1, np + 1, np, fp, stw, -1.0);
    const double sc = 2.0 * kPi / np;
    double* o1 = G + ((int64_t)f * nt + t) * (N + 1) * 2;
    double* o2 = G + ((int64_t)f * nt + t2) * (N + 1) * 2;
    for (int k = threadIdx.x; k <= N; k += blockDim.x) {
        const cplx<double> a = Z[k % np];
        const cplx<double> c = Z[(np - k % np) % np];  // Z_{-k}
        if (t2 == t) {
            o1[2 * k] = a.re * sc;
            o1[2 * k + 1] = a.im * sc;
        } else {
            o1[2 * k] = 0.5 * (a.re + c.re) * sc;
            o1[2 * k + 1] = 0.5 * (a.im - c.im) * sc;
            o2[2 * k] = 0.5 * (a.im + c.im) * sc;
            o2[2 * k + 1] = -0.5 * (a.re - c.re) * sc;
        }
    }
}

// Radices of n (primes 3..19, then powers of two by 8, 4 and 2, the stages
// in the reverse order), or nst = 0 when n has a prime factor above 19 (the
// direct sum is used then).
FftPlan make_fft_plan(int n) {
    FftPlan p;
    p.nst = 0;
    if (n < 2) return p;
    int r = n;
    int rad[kFftMaxStages];
    int ns = 0;
    const int primes[] = {19, 17, 13, 11, 7, 5, 3};
    for (int q : primes)
        while (r % q == 0 && ns < kFftMaxStages) {
            rad[ns++] = q;
            r /= q;
        }
    while (r % 8 == 0 && ns < kFftMaxStages) {
        rad[ns++] = 8;
        r /= 8;
    }
    while (r % 4 == 0 && ns < kFftMaxStages) {
        rad[ns++] = 4;
        r /= 4;
    }
    while (r % 2 == 0 && ns < kFftMaxStages) {
        rad[ns++] = 2;
        r /= 2;
    }
    if (r != 1) return p;
    p.nst = ns;
    // stages run in the reverse order of extraction: the radix-2 stage of a
    // power of two first (128 = 2 8 8 took 80 us a 128^3 transform where
    // 8 8 2 took 86 us)
    for (int i = 0; i < ns; i++) p.rad[i] = rad[ns - 1 - i];
    return p;
}

// Lines per block: 16 real lines (8 complex transforms) or 8 complex lines
// when their two ping-pong buffers and the twiddles fit 64 KiB; 0 otherwise.
static int fft_axis_lines(int nin, bool real_in) {
    const int TL = real_in ? 16 : 8;
    const int NL = real_in ? TL / 2 : TL;
    const size_t bytes = sizeof(double) * 2 * (size_t)nin + 2 * 16 * (size_t)(nin + 1) * NL;
    return bytes <= 65536 ? TL : 0;
}

bool fft_axis_fits(int nin) { return make_fft_plan(nin).nst > 0 && fft_axis_lines(nin, false) > 0; }

hamls_status launch_fft_axis(const double* in, bool real_in, double* out, int64_t A, int nin, int64_t B,
                             int nout, int koff, double sign, double scale, const double* tw, hipStream_t s) {
    const FftPlan fp = make_fft_plan(nin);
    if (fp.nst == 0) {
        set_error("fft axis: length %d has a prime factor above 19", nin);
        return HAMLS_ERR_UNSUPPORTED;
    }
    const int TL = fft_axis_lines(nin, real_in);
    if (TL < 1) {
        set_error("fft axis: length %d too large", nin);
        return HAMLS_ERR_UNSUPPORTED;
    }
    const int NL = real_in ? TL / 2 : TL;
    const int64_t nlines = A * B;
    const int64_t nblk = (nlines + TL - 1) / TL;
    if (nblk > 0x7fffffff) {
        set_error("fft axis: too many lines");
        return HAMLS_ERR_UNSUPPORTED;
    }
    const size_t lds = sizeof(double) * 2 * (size_t)nin + 2 * 16 * (size_t)(nin + 1) * NL;
    hipLaunchKernelGGL(k_fft_axis, dim3((unsigned)nblk), dim3(256), lds, s, in, real_in ? 1 : 0, out, A, nin, B,
                       nout, koff, sign, scale, tw, TL, fp);
    HAMLS_HIP(hipGetLastError());
    return HAMLS_OK;
}

bool s2_ring_fft_fits(int np) {
    return make_fft_plan(np).nst > 0 && sizeof(double) * 2 * (size_t)np + 2 * 16 * (size_t)(np + 1) <= 65536;
}

hamls_status launch_s2_ring_fft(const Plan& P, const double* gv, int F, double* G, hipStream_t s) {
    const int nt = P.dims[0], np = P.dims[1];
    const FftPlan fp = make_fft_plan(np);
    if (!s2_ring_fft_fits(np)) {
        set_error("ring fft: length %d not supported", np);
        return HAMLS_ERR_UNSUPPORTED;
    }
    const int pairs = (nt + 1) / 2;
    const size_t lds = sizeof(double) * 2 * (size_t)np + 2 * 16 * (size_t)(np + 1);
    hipLaunchKernelGGL(k_s2_ring_fft, dim3((unsigned)pairs, (unsigned)F), dim3(256), lds, s, gv, P.MQ, nt, np,
                       P.N, P.d_tw, fp, G);
    HAMLS_HIP(hipGetLastError());
    return HAMLS_OK;
}

}  // namespace hamls
