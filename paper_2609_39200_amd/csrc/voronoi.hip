// voronoi.hip -- spherical Voronoi-cell areas of the bound S2 nodes, the node
// weights of the paper's ill-distributed recipe (Sec. 2.2, the remark after
// Thm. 2.1: the weight function rescaled by the Voronoi-cell volume of each
// node; Sec. 3: both methods weight the data by Voronoi areas).
//
// One thread per sorted record x.  The cell {y : y.x >= y.x_j for all j} is
// built in the gnomonic chart at x (y ~ x + u e1 + v e2): every other node x_j
// bounds it by the half-plane
//   (x.x - x.x_j) - u (e1.x_j) - v (e2.x_j) >= 0,
// and a large square is clipped by the half-planes of the nodes of a cell
// cover of the cap of radius rho around x (Sutherland-Hodgman).  With R the
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
    for (int attempt = 0; attempt < 40; attempt++) {
        int nv = 4;
        pa[0] = -kVorWindow;
        pa[1] = -kVorWindow;
        pa[2] = kVorWindow;
        pa[3] = -kVorWindow;
        pa[4] = kVorWindow;
        pa[5] = kVorWindow;
        pa[6] = -kVorWindow;
        pa[7] = kVorWindow;
        bool overflow = false;  // also set when the polygon vanishes (duplicate nodes)
        // the cells covering the cap of radius rho, widened by one band and
        // one sector on each side (rounding of the binning)
        int blo = (int)floor((th0 - rho) / g.dtheta) - 1, bhi = (int)floor((th0 + rho) / g.dtheta) + 1;
        const bool allphi = th0 - rho <= 0.0 || th0 + rho >= kPi;
        blo = blo < 0 ? 0 : blo;
        bhi = bhi > g.nb - 1 ? g.nb - 1 : bhi;
        const double dphi = allphi ? kPi : asin(fmin(1.0, sin(rho) / sin(th0)));
        for (int b = blo; b <= bhi && !overflow; b++) {
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
                    const double bj = xx - (x0 * y0 + x1 * y1 + x2 * y2);
                    const double cu = e10 * y0 + e11 * y1 + e12 * y2;
                    const double cv = e20 * y0 + e21 * y1 + e22 * y2;
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
                }
            }
        }
        if (overflow || nv < 3) break;
        // largest angle from x to a vertex; the chart's edge
        bool edge = false;
        double cmin = 1.0;
        for (int k = 0; k < nv; k++) {
            const double u = pa[2 * k], v = pa[2 * k + 1];
            if (fabs(u) >= 0.999999 * kVorWindow || fabs(v) >= 0.999999 * kVorWindow) edge = true;
            // cos of the angle between x and x + u e1 + v e2
            cmin = fmin(cmin, sqrt(xx) / sqrt(xx + u * u + v * v));
        }
        const double R = acos(fmin(1.0, cmin));
        if (!edge && 2.0 * R < rho * (1.0 - 1e-9)) {
            double area = 0.0;
            const double xn = sqrt(xx);
            for (int k = 0; k < nv; k++) {
                const int l = k + 1 < nv ? k + 1 : 0;
                double a0 = x0 + pa[2 * k] * e10 + pa[2 * k + 1] * e20;
                double a1 = x1 + pa[2 * k] * e11 + pa[2 * k + 1] * e21;
                double a2 = x2 + pa[2 * k] * e12 + pa[2 * k + 1] * e22;
                double c0 = x0 + pa[2 * l] * e10 + pa[2 * l + 1] * e20;
                double c1 = x1 + pa[2 * l] * e11 + pa[2 * l + 1] * e21;
                double c2 = x2 + pa[2 * l] * e12 + pa[2 * l + 1] * e22;
                const double na = 1.0 / sqrt(a0 * a0 + a1 * a1 + a2 * a2);
                const double nc = 1.0 / sqrt(c0 * c0 + c1 * c1 + c2 * c2);
                a0 *= na;
                a1 *= na;
                a2 *= na;
                c0 *= nc;
                c1 *= nc;
                c2 *= nc;
                const double det = (x0 * (a1 * c2 - a2 * c1) + x1 * (a2 * c0 - a0 * c2) + x2 * (a0 * c1 - a1 * c0)) / xn;
                const double den = 1.0 + (x0 * a0 + x1 * a1 + x2 * a2) / xn + (a0 * c0 + a1 * c1 + a2 * c2) +
                                   (c0 * x0 + c1 * x1 + c2 * x2) / xn;
                area += 2.0 * atan2(fabs(det), den);
            }
            result = area;
            break;
        }
        if (edge || rho >= kPi) break;  // every node was in the cover: the cell reaches the chart's edge
        rho = fmin(kPi, fmax(2.0 * rho, 2.05 * R));
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
