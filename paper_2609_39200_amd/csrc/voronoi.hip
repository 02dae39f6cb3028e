// voronoi.hip -- spherical Voronoi-cell areas of the bound S2 nodes, the node
// weights of the paper's ill-distributed recipe (Sec. 2.2, the remark after
// Thm. 2.1: the weight function rescaled by the Voronoi-cell volume of each
// node; Sec. 3: both methods weight the data by Voronoi areas).
//
// One thread per sorted record x.  The cell {y : y.x >= y.x_j for all j} is
// built in the gnomonic chart at x (y ~ x + u e1 + v e2): every other node x_j
// bounds it by the half-plane
//   (x + u e1 + v e2).(x - x_j) >= 0,
// and a square (half-width tan(rho), at most 1e4) is clipped by the
// half-planes of the nodes of a cell cover of the cap of radius rho around x
// (Sutherland-Hodgman; bands outward from x's own, nodes that cannot cut the
// current polygon skipped).  With R the
// largest angle from x to a vertex of the result, a node at angle d >= 2R
// from x cannot cut the cell (its bisector lies beyond every vertex), so the
// result is exact once 2R < rho; otherwise rho grows and the cell is rebuilt.
// The area is the sum of the solid angles of the fan triangles (x, y_k, y_k+1)
// (Van Oosterom-Strackee).  A cell that reaches the chart's edge (~89.99
// degrees from its node), holds more than kVorMaxVerts vertices, or vanishes
// (a duplicate node) gets NaN.
#include "common.h"
#include "device_common.h"

namespace hamls {

constexpr int kVorThreads = 64;
constexpr int kVorMaxVerts = 28;
constexpr double kVorWindow = 1e4;

struct VorGeom {
    const double* X;  // sorted records, structure of arrays [3][cap]
    int64_t cap;
    const int32_t* perm;
    const int32_t* band_off;
    const int32_t* cs;  // cell_start
    int nb;
    double dtheta;
};

// Records [lo, hi) of the sorted array covering sectors [s0, s1] of band b
// (s0 <= s1, no wrap).
__device__ __forceinline__ void vor_range(const VorGeom& g, int b, int s0, int s1, int* lo, int* hi) {
    const int off = g.band_off[b];
    *lo = g.cs[off + s0];
    *hi = g.cs[off + s1 + 1];
}

__global__ __launch_bounds__(kVorThreads) void k_s2_voronoi(VorGeom g, int64_t nrec, double* __restrict__ areas) {
    __shared__ double sbuf[kVorThreads][2][2 * kVorMaxVerts];
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrec) return;
    double* pa = sbuf[threadIdx.x][0];
    double* pb = sbuf[threadIdx.x][1];
    const double x0 = g.X[r], x1 = g.X[g.cap + r], x2 = g.X[2 * g.cap + r];
    // orthonormal tangent frame at x from the reflection that maps the z axis
    // to x (valid for every unit x, also at the poles)
    const double sg = x2 >= 0.0 ? 1.0 : -1.0;
    const double ia = -1.0 / (sg + x2);
    const double bb = x0 * x1 * ia;
    const double e10 = 1.0 + sg * x0 * x0 * ia, e11 = sg * bb, e12 = -sg * x0;
    const double e20 = bb, e21 = sg + x1 * x1 * ia, e22 = -x1;
    const double xx = x0 * x0 + x1 * x1 + x2 * x2;
    const double th0 = acos(fmin(1.0, fmax(-1.0, x2)));
    double ph0 = atan2(x1, x0);
    if (ph0 < 0.0) ph0 += 2.0 * kPi;
    // first cap: about sixteen nodes at the density of x's own cell
    int b0 = (int)(th0 / g.dtheta);
    b0 = b0 < 0 ? 0 : (b0 > g.nb - 1 ? g.nb - 1 : b0);
    const int ns0 = g.band_off[b0 + 1] - g.band_off[b0];
    int s00 = (int)(ph0 * (ns0 / (2.0 * kPi)));
    s00 = s00 < 0 ? 0 : (s00 > ns0 - 1 ? ns0 - 1 : s00);
    int clo, chi;
    vor_range(g, b0, s00, s00, &clo, &chi);
    const double tlo = b0 * g.dtheta, thi = (b0 + 1) * g.dtheta;
    const double acell = (cos(tlo) - cos(thi)) * (2.0 * kPi / ns0);
    double rho = sqrt(16.0 * acell / (kPi * (double)(chi - clo > 0 ? chi - clo : 1)));
    rho = fmin(fmax(rho, 1e-9), kPi);
    double result = nan("");
    double wfix = 0.0;  // > 0: the window of a refining pass
    for (int attempt = 0; attempt < 40; attempt++) {
        // the chart window: a cell accepted below lies within angle rho / 2
        // of x, so a square of half-width tan(rho) holds it with room; a
        // window near the cell's size keeps the clipped vertices accurate
        const double W = wfix > 0.0 ? wfix : (rho < 1.5 ? tan(rho) : kVorWindow);
        int nv = 4;
        pa[0] = -W;
        pa[1] = -W;
        pa[2] = W;
        pa[3] = -W;
        pa[4] = W;
        pa[5] = W;
        pa[6] = -W;
        pa[7] = W;
        bool overflow = false;  // also set when the polygon vanishes (duplicate nodes)
        // the cells covering the cap of radius rho, widened by one band and
        // one sector on each side (rounding of the binning)
        int blo = (int)floor((th0 - rho) / g.dtheta) - 1, bhi = (int)floor((th0 + rho) / g.dtheta) + 1;
        const bool allphi = th0 - rho <= 0.0 || th0 + rho >= kPi;
        blo = blo < 0 ? 0 : blo;
        bhi = bhi > g.nb - 1 ? g.nb - 1 : bhi;
        const double dphi = allphi ? kPi : asin(fmin(1.0, sin(rho) / sin(th0)));
        // cos of the current polygon's largest vertex angle R: a node at angle
        // d >= 2R from x cannot cut it (nor the final cell, which lies inside)
        double cmin_cur = 0.0;
        // bands outward from x's own (near candidates first keep the
        // intermediate polygons small)
        const int nsteps = 2 * max(b0 - blo, bhi - b0) + 1;
        for (int bs = 0; bs < nsteps && !overflow; bs++) {
            const int b = (bs & 1) ? b0 - (bs + 1) / 2 : b0 + bs / 2;
            if (b < blo || b > bhi) continue;
            const int ns = g.band_off[b + 1] - g.band_off[b];
            int ranges[4];
            int nr = 0;
            if (allphi || dphi >= 0.5 * kPi) {
                vor_range(g, b, 0, ns - 1, &ranges[0], &ranges[1]);
                nr = 1;
            } else {
                const double sec = ns / (2.0 * kPi);
                int s0 = (int)floor((ph0 - dphi) * sec) - 1, s1 = (int)floor((ph0 + dphi) * sec) + 1;
                if (s1 - s0 + 1 >= ns) {
                    vor_range(g, b, 0, ns - 1, &ranges[0], &ranges[1]);
                    nr = 1;
                } else {
                    // [s0, s1] modulo ns: one or two runs
                    int a0 = ((s0 % ns) + ns) % ns, a1 = ((s1 % ns) + ns) % ns;
                    if (a0 <= a1) {
                        vor_range(g, b, a0, a1, &ranges[0], &ranges[1]);
                        nr = 1;
                    } else {
                        vor_range(g, b, a0, ns - 1, &ranges[0], &ranges[1]);
                        vor_range(g, b, 0, a1, &ranges[2], &ranges[3]);
                        nr = 2;
                    }
                }
            }
            for (int q = 0; q < nr && !overflow; q++) {
                for (int j = ranges[2 * q]; j < ranges[2 * q + 1]; j++) {
                    if (j == r) continue;
                    const double y0 = g.X[j], y1 = g.X[g.cap + j], y2 = g.X[2 * g.cap + j];
                    const double dot = x0 * y0 + x1 * y1 + x2 * y2;
                    if (dot < 2.0 * cmin_cur * cmin_cur - 1.0 - 1e-12) continue;
                    // the half-plane (x + u e1 + v e2).(x - y) >= 0 through the
                    // difference vector (no cancellation for close nodes)
                    const double d0 = x0 - y0, d1 = x1 - y1, d2 = x2 - y2;
                    const double bj = x0 * d0 + x1 * d1 + x2 * d2;
                    const double cu = -(e10 * d0 + e11 * d1 + e12 * d2);
                    const double cv = -(e20 * d0 + e21 * d1 + e22 * d2);
                    // clip the polygon pa (nv vertices) into pb
                    int no = 0;
                    double u1 = pa[2 * nv - 2], v1 = pa[2 * nv - 1];
                    double f1 = bj - cu * u1 - cv * v1;
                    for (int k = 0; k < nv; k++) {
                        const double u2 = pa[2 * k], v2 = pa[2 * k + 1];
                        const double f2 = bj - cu * u2 - cv * v2;
                        if ((f1 >= 0.0) != (f2 >= 0.0)) {
                            const double t = f1 / (f1 - f2);
                            if (no < kVorMaxVerts) {
                                pb[2 * no] = u1 + t * (u2 - u1);
                                pb[2 * no + 1] = v1 + t * (v2 - v1);
                            }
                            no++;
                        }
                        if (f2 >= 0.0) {
                            if (no < kVorMaxVerts) {
                                pb[2 * no] = u2;
                                pb[2 * no + 1] = v2;
                            }
                            no++;
                        }
                        u1 = u2;
                        v1 = v2;
                        f1 = f2;
                    }
                    if (no > kVorMaxVerts || no == 0) {
                        overflow = true;
                        break;
                    }
                    double* t = pa;
                    pa = pb;
                    pb = t;
                    nv = no;
                    double cm = 1.0;
                    for (int k = 0; k < nv; k++)
                        cm = fmin(cm, sqrt(xx / (xx + pa[2 * k] * pa[2 * k] + pa[2 * k + 1] * pa[2 * k + 1])));
                    cmin_cur = cm;
                }
            }
        }
        if (overflow || nv < 3) break;
        // largest angle from x to a vertex; the chart's edge
        bool edge = false;
        double cmin = 1.0, ext = 0.0;
        for (int k = 0; k < nv; k++) {
            const double u = pa[2 * k], v = pa[2 * k + 1];
            if (fabs(u) >= 0.999999 * W || fabs(v) >= 0.999999 * W) edge = true;
            ext = fmax(ext, fmax(fabs(u), fabs(v)));
            // cos of the angle between x and x + u e1 + v e2
            cmin = fmin(cmin, sqrt(xx) / sqrt(xx + u * u + v * v));
        }
        const double R = acos(fmin(1.0, cmin));
        if (!edge && 2.0 * R < rho * (1.0 - 1e-9) && wfix == 0.0 && W > 4.0 * ext) {
            // exact but clipped from a window much larger than the cell:
            // once more from a square twice the cell's extent
            wfix = 2.0 * ext;
            continue;
        }
        if (!edge && 2.0 * R < rho * (1.0 - 1e-9)) {
            // Van Oosterom-Strackee in the chart: with y = (x + u e1 + v e2)/n,
            // n = |x + u e1 + v e2|, the triple product of (x, y_k, y_l) is
            // (u_k v_l - u_l v_k)/(n_k n_l) and the dot products are
            // |x|/n and (x.x + u_k u_l + v_k v_l)/(n_k n_l): no cancellation
            // for small cells
            double area = 0.0;
            const double xn = sqrt(xx);
            for (int k = 0; k < nv; k++) {
                const int l = k + 1 < nv ? k + 1 : 0;
                const double uk = pa[2 * k], vk = pa[2 * k + 1], ul = pa[2 * l], vl = pa[2 * l + 1];
                const double nk = sqrt(xx + uk * uk + vk * vk), nl = sqrt(xx + ul * ul + vl * vl);
                const double inn = 1.0 / (nk * nl);
                const double det = (uk * vl - ul * vk) * inn;
                const double den = 1.0 + xn / nk + xn / nl + (xx + uk * ul + vk * vl) * inn;
                area += 2.0 * atan2(fabs(det), den);
            }
            result = area;
            break;
        }
        if (wfix > 0.0) break;  // a refining pass that failed: keep NaN
        if (rho >= kPi) break;  // every node was in the cover: the cell reaches the chart's edge
        // a cover too small to close the cell (edge), or one that may miss a
        // node closer than 2R: grow it
        rho = edge ? fmin(kPi, 2.0 * rho) : fmin(kPi, fmax(2.0 * rho, 2.05 * R));
    }
    areas[g.perm[r]] = result;
}

hamls_status launch_s2_voronoi(const Plan& P, double* areas, hipStream_t s) {
    VorGeom g;
    g.X = P.d_x;
    g.cap = P.cap;
    g.perm = P.d_perm;
    g.band_off = P.d_band_off;
    g.cs = P.d_cell_start;
    g.nb = P.bins.nb;
    g.dtheta = P.bins.dtheta;
    const int64_t nb = (P.nrec + kVorThreads - 1) / kVorThreads;
    hipLaunchKernelGGL(k_s2_voronoi, dim3((unsigned)nb), dim3(kVorThreads), 0, s, g, P.nrec, areas);
    HAMLS_HIP(hipGetLastError());
    return HAMLS_OK;
}

}  // namespace hamls
