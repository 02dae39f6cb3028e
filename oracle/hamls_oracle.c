/*
 * hamls_oracle.c -- plain, slow FP64 CPU oracle of the HAMLS hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant with
 * the GPU library.  Every routine is written for a reader to check against the
 * paper ("Fast and Stable Harmonic Approximation from Ill-distributed Data
 * using Moving Least Squares", Hielscher, Poeschl, Wuensche), not for speed:
 *
 *   grid          Sec. 2.1 (product quadrature rules exact on Pi_{2L})
 *   neighbours    eq. (5), (6), (12): brute force over every node
 *   local solve   eq. (4), (14)-(23), Sec. 2.3: weights, tangent-space
 *                 monomials, Householder QR (not Cholesky), chi, tau by
 *                 bisection, and c_1 from the regularized problem (22)
 *                 solved as an augmented least-squares problem
 *   quadrature    Alg. 1 step 3 / eq. (25): direct sums, no FFT
 *   evaluation    direct synthesis of the harmonic series
 *
 * Conventions shared with the GPU library only through the documented ABI
 * (layouts, orderings), never through code:
 *   S2   grid ring-major, rings by ascending polar angle (GL nodes in cos(theta)
 *        descending), phi_p = 2 pi p / n_phi; point = (s_t c_p, s_t s_p, x_t)
 *        with s_t = sqrt((1-x_t)(1+x_t)).  Coefficient (n,k) at n*n+n+k.
 *   SO3  unit quaternions (w,x,y,z), q == -q; Euler ZYZ grid laid out
 *        [beta][alpha][gamma]; D^n_{k,k'}(a,b,g) = e^{-ika} d^n_{k,k'}(b)
 *        e^{-ik'g}; coefficient index sum_{l<n}(2l+1)^2 + (k+n)(2n+1) + (k'+n).
 *   T3   [0,1)^3, grid x = i/n laid out [i0][i1][i2], basis e^{2 pi i k.x},
 *        coefficients centred-lexicographic k_d in [-(n/2), n-1-(n/2)].
 *
 * Where the paper is silent, the reading taken is stated at the routine that
 * takes it.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_S2 0
#define ORC_SO3 1
#define ORC_T3 2

#define ORC_REG_NONE 0
#define ORC_REG_FIXED 1
#define ORC_REG_CHI 2

/* per-grid-node status bits */
#define ORC_ST_REGULARIZED 1u
#define ORC_ST_UNDERDETERMINED 2u
#define ORC_ST_EMPTY 4u
#define ORC_ST_HEMISPHERE 8u

static const double ORC_PI = 3.141592653589793238462643383279502884;

typedef struct {
    int32_t domain;         /* ORC_S2 / ORC_SO3 / ORC_T3 */
    int32_t bandwidth;      /* N (the paper's L) */
    int32_t degree;         /* K, MLS polynomial degree */
    int32_t knn_count;      /* n of eq. (12); 0 disables */
    double support_radius;  /* fixed delta_0; 0 disables */
    double knn_eps;         /* epsilon of eq. (12) */
    int32_t wendland;       /* 1: phi_{3,1}, 2: phi_{3,2} */
    int32_t reg;            /* ORC_REG_* */
    double tau_fixed;       /* tau for ORC_REG_FIXED */
    double chi_target;      /* chi_T of Sec. 2.3 */
    double chi_full;        /* chi_full of Sec. 2.3 */
    int32_t grid_shape[3];  /* see orc_grid_dims */
    int32_t smooth_aux;     /* S2 adaptive radius smoothed on this many Fibonacci points; 0 off */
} orc_params;

/* ------------------------------------------------------------------ */
/* small helpers                                                       */
/* ------------------------------------------------------------------ */

static int tangent_dim(int domain) { return domain == ORC_S2 ? 2 : 3; }

/* number of monomials of total degree <= K in D variables: C(K+D, D) */
static int n_monomials(int D, int K)
{
    int m = 1;
    for (int i = 1; i <= D; i++) m = m * (K + i) / i;
    return m;
}

/* Monomial exponents sorted ascending by total degree (Sec. 2.3, "sorted in
 * ascending order by degree"); inside one degree the first variable's power
 * descends.  exps has room for m*3 ints. */
static void monomial_exponents(int D, int K, int* exps, int* degs)
{
    int c = 0;
    for (int l = 0; l <= K; l++) {
        if (D == 2) {
            for (int a = l; a >= 0; a--) {
                exps[3 * c] = a; exps[3 * c + 1] = l - a; exps[3 * c + 2] = 0;
                degs[c++] = l;
            }
        } else {
            for (int a = l; a >= 0; a--)
                for (int b = l - a; b >= 0; b--) {
                    exps[3 * c] = a; exps[3 * c + 1] = b; exps[3 * c + 2] = l - a - b;
                    degs[c++] = l;
                }
        }
    }
}

static double ipow(double x, int e)
{
    double r = 1.0;
    for (int i = 0; i < e; i++) r *= x;
    return r;
}

/* Wendland functions with support [0,1] (the weight profile of eq. (6)). */
static double wendland(int which, double r)
{
    if (r >= 1.0) return 0.0;
    double s = 1.0 - r;
    if (which == 2) {
        double s2 = s * s, s6 = s2 * s2 * s2;
        return s6 * (35.0 * r * r + 18.0 * r + 3.0);
    }
    double s2 = s * s;
    return s2 * s2 * (4.0 * r + 1.0);
}

/* ------------------------------------------------------------------ */
/* Gauss-Legendre rule (Sec. 2.1)                                      */
/* ------------------------------------------------------------------ */

/* P_n(x) and P_n'(x) by the three-term recurrence. */
static void legendre_and_derivative(int n, double x, double* p, double* dp)
{
    double p0 = 1.0, p1 = x;
    if (n == 0) { *p = 1.0; *dp = 0.0; return; }
    for (int k = 2; k <= n; k++) {
        double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
    }
    *p = p1;
    *dp = n * (x * p1 - p0) / (x * x - 1.0);
}

/* Nodes (descending, x[0] nearest +1) and weights of the n-point rule on
 * [-1,1], by Newton's method on P_n.  Exact for polynomials of degree 2n-1. */
int orc_gauss_legendre(int n, double* x, double* w)
{
    if (n < 1) return -1;
    for (int i = 0; i < (n + 1) / 2; i++) {
        double z = cos(ORC_PI * (i + 0.75) / (n + 0.5));
        double p, dp;
        for (int it = 0; it < 100; it++) {
            legendre_and_derivative(n, z, &p, &dp);
            double dz = p / dp;
            z -= dz;
            if (fabs(dz) < 1e-15) {
                legendre_and_derivative(n, z, &p, &dp);
                z -= p / dp;
                break;
            }
        }
        legendre_and_derivative(n, z, &p, &dp);
        double wi = 2.0 / ((1.0 - z * z) * dp * dp);
        x[i] = z;
        x[n - 1 - i] = -z;
        w[i] = wi;
        w[n - 1 - i] = wi;
    }
    if (n % 2 == 1) x[n / 2] = 0.0;
    return 0;
}

/* ------------------------------------------------------------------ */
/* grids (Sec. 2.1)                                                    */
/* ------------------------------------------------------------------ */

/* Resolved grid dimensions.  A zero grid_shape entry takes the paper's minimal
 * exact rule: S2 (L+1) x (2L+2); SO3 (L+1) x (2L+1) x (2L+1); T3 (2L+1)^3. */
int orc_grid_dims(const orc_params* p, int32_t* dims)
{
    int N = p->bandwidth;
    if (N < 0) return -1;
    if (p->domain == ORC_S2) {
        dims[0] = p->grid_shape[0] > 0 ? p->grid_shape[0] : N + 1;
        dims[1] = p->grid_shape[1] > 0 ? p->grid_shape[1] : 2 * N + 2;
        dims[2] = 1;
        if (dims[0] < N + 1 || dims[1] < 2 * N + 1) return -2;
    } else if (p->domain == ORC_SO3) {
        dims[0] = p->grid_shape[0] > 0 ? p->grid_shape[0] : N + 1;
        dims[1] = p->grid_shape[1] > 0 ? p->grid_shape[1] : 2 * N + 1;
        dims[2] = p->grid_shape[2] > 0 ? p->grid_shape[2] : 2 * N + 1;
        if (dims[0] < N + 1 || dims[1] < 2 * N + 1 || dims[2] < 2 * N + 1) return -2;
    } else if (p->domain == ORC_T3) {
        int n = p->grid_shape[0] > 0 ? p->grid_shape[0] : 2 * N + 1;
        dims[0] = dims[1] = dims[2] = n;
        if (n < 2 * N) return -2;
    } else {
        return -1;
    }
    return 0;
}

int64_t orc_grid_size(const orc_params* p)
{
    int32_t d[3];
    if (orc_grid_dims(p, d)) return -1;
    return (int64_t)d[0] * d[1] * d[2];
}

/* unit quaternion of R_z(a) R_y(b) R_z(g) */
static void euler_zyz_quaternion(double a, double b, double g, double* q)
{
    double cb = cos(0.5 * b), sb = sin(0.5 * b);
    double sp = 0.5 * (a + g), dm = 0.5 * (a - g);
    q[0] = cb * cos(sp);
    q[1] = -sb * sin(dm);
    q[2] = sb * cos(dm);
    q[3] = cb * sin(sp);
}

/* Grid points and quadrature weights.  S2/T3 points have 3 doubles, SO3
 * points 4 (quaternion).  Sum of weights: 4 pi (S2), 8 pi^2 (SO3), 1 (T3). */
int orc_grid(const orc_params* p, double* pts, double* wts)
{
    int32_t d[3];
    if (orc_grid_dims(p, d)) return -1;
    if (p->domain == ORC_S2) {
        int nt = d[0], np = d[1];
        double* x = malloc(sizeof(double) * nt);
        double* w = malloc(sizeof(double) * nt);
        orc_gauss_legendre(nt, x, w);
        for (int t = 0; t < nt; t++) {
            double st = sqrt((1.0 - x[t]) * (1.0 + x[t]));
            for (int q = 0; q < np; q++) {
                double phi = 2.0 * ORC_PI * q / np;
                double cp = cos(phi), sp = sin(phi);
                int64_t j = (int64_t)t * np + q;
                pts[3 * j + 0] = st * cp;
                pts[3 * j + 1] = st * sp;
                pts[3 * j + 2] = x[t];
                wts[j] = w[t] * 2.0 * ORC_PI / np;
            }
        }
        free(x);
        free(w);
    } else if (p->domain == ORC_SO3) {
        int nb = d[0], na = d[1], ng = d[2];
        double* x = malloc(sizeof(double) * nb);
        double* w = malloc(sizeof(double) * nb);
        orc_gauss_legendre(nb, x, w);
        for (int t = 0; t < nb; t++) {
            double beta = acos(x[t]);
            for (int a = 0; a < na; a++)
                for (int g = 0; g < ng; g++) {
                    int64_t j = ((int64_t)t * na + a) * ng + g;
                    euler_zyz_quaternion(2.0 * ORC_PI * a / na, beta, 2.0 * ORC_PI * g / ng,
                                         pts + 4 * j);
                    wts[j] = w[t] * (2.0 * ORC_PI / na) * (2.0 * ORC_PI / ng);
                }
        }
        free(x);
        free(w);
    } else {
        int n = d[0];
        for (int a = 0; a < n; a++)
            for (int b = 0; b < n; b++)
                for (int c = 0; c < n; c++) {
                    int64_t j = ((int64_t)a * n + b) * n + c;
                    pts[3 * j + 0] = (double)a / n;
                    pts[3 * j + 1] = (double)b / n;
                    pts[3 * j + 2] = (double)c / n;
                    wts[j] = 1.0 / ((double)n * n * n);
                }
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* distances and the membership predicate (eq. (5), (6), (12))         */
/* ------------------------------------------------------------------ */

/* Proximity key of node x to centre q.  Written without fused operations, in
 * this exact association, so that the membership decision is reproducible:
 *   S2  : dot = (x0 q0 + x1 q1) + x2 q2           (member iff key > c)
 *   SO3 : |dot| over four components              (member iff key > c)
 *   T3  : squared min-image distance              (member iff key < c) */
static double prox_key(int domain, const double* x, const double* q)
{
    if (domain == ORC_S2) {
        double a = x[0] * q[0];
        double b = x[1] * q[1];
        double c = x[2] * q[2];
        double s = a + b;
        return s + c;
    }
    if (domain == ORC_SO3) {
        double a = x[0] * q[0];
        double b = x[1] * q[1];
        double c = x[2] * q[2];
        double e = x[3] * q[3];
        double s = a + b;
        s = s + c;
        s = s + e;
        return fabs(s);
    }
    double s = 0.0;
    for (int i = 0; i < 3; i++) {
        double dlt = x[i] - q[i];
        dlt = dlt - nearbyint(dlt);
        double sq = dlt * dlt;
        s = s + sq;
    }
    return s;
}

static int key_inside(int domain, double key, double c)
{
    return domain == ORC_T3 ? (key < c) : (key > c);
}

/* Geodesic distance from the key: S2 arc length; SO3 rotation angle
 * 2 arccos|q.q'|; T3 Euclidean min-image distance. */
static double key_distance(int domain, double key)
{
    if (domain == ORC_T3) return sqrt(key);
    double k = key > 1.0 ? 1.0 : (key < -1.0 ? -1.0 : key);
    return domain == ORC_S2 ? acos(k) : 2.0 * acos(k);
}

/* The k-th entry (0-based) of a[0..n-1] in descending order (ascending if
 * asc), by quickselect with a median-of-three pivot.  a is permuted. */
static double select_kth(double* a, int64_t n, int64_t k, int asc)
{
    int64_t lo = 0, hi = n - 1;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        double x = a[lo], y = a[mid], z = a[hi];
        double piv = (x < y) ? ((y < z) ? y : ((x < z) ? z : x)) : ((x < z) ? x : ((y < z) ? z : y));
        int64_t i = lo, j = hi;
        while (i <= j) {
            if (asc) {
                while (a[i] < piv) i++;
                while (a[j] > piv) j--;
            } else {
                while (a[i] > piv) i++;
                while (a[j] < piv) j--;
            }
            if (i <= j) {
                double t = a[i];
                a[i] = a[j];
                a[j] = t;
                i++;
                j--;
            }
        }
        if (k <= j)
            hi = j;
        else if (k >= i)
            lo = i;
        else
            return a[k];
    }
    return a[k];
}

/* Support radius delta and membership threshold c of one centre.
 *  fixed radius   : delta = delta_0
 *  adaptive (12)  : delta = (1+eps) d_n, d_n = distance of the n-th nearest
 *                   node (brute force: sort every node's key)
 *  both set       : the larger radius
 * S2 requires delta < pi/2 (tangent projection, Sec. 2.3); a larger radius is
 * clamped to pi/2 and flagged.  Threshold: S2 cos(delta); SO3 cos(delta/2);
 * T3 delta^2, where for the adaptive radius c = (1+eps)^2 d_n^2 directly. */
/* ------------------------------------------------------------------ */
/* Voronoi-area node weights (Sec. 2.2, the remark after Thm. 2.1;    */
/* Sec. 3, where both methods weight the nodes by Voronoi areas)       */
/* ------------------------------------------------------------------ */

/* Area of the spherical Voronoi cell of every node, by its definition
 *   V_i = { x in S2 : x.x_i >= x.x_j for every j },
 * the intersection of the half-spaces x.(x_i - x_j) >= 0 over ALL other
 * nodes (brute force, O(M^2)).  The cell is built in the gnomonic chart
 * centred at x_i (x = x_i + u e1 + v e2, up to a positive factor), where
 * great circles are lines and each half-space is the half-plane
 *   (x_i + u e1 + v e2).(x_i - x_j) >= 0;
 * a large square is clipped by every half-plane in turn (Sutherland-Hodgman),
 * the vertices are mapped back to the sphere, and the area is the sum of the
 * solid angles of the triangles (x_i, y_k, y_k+1) (Van Oosterom-Strackee).
 * A cell that reaches the square's edge (more than ~89.99 degrees from its
 * node) gets NaN; nodes must be distinct unit vectors.  rows (nrows of them)
 * selects the nodes whose cells are computed, or NULL for all M; areas[r]
 * belongs to the r-th selected node.  Returns the number of NaN cells. */
#define ORC_VOR_W 1e4
int64_t orc_voronoi_areas(const double* nodes, int64_t M, const int64_t* rows, int64_t nrows, double* areas)
{
    int64_t bad = 0;
    int64_t nr = rows ? nrows : M;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : bad)
    for (int64_t r = 0; r < nr; r++) {
        const int64_t i = rows ? rows[r] : r;
        double* out_i = areas + r;
        const double* x = nodes + 3 * i;
        int ax = 0;
        for (int d = 1; d < 3; d++)
            if (fabs(x[d]) < fabs(x[ax])) ax = d;
        double a[3] = {0.0, 0.0, 0.0};
        a[ax] = 1.0;
        double ax_x = a[0] * x[0] + a[1] * x[1] + a[2] * x[2];
        double e1[3], e2[3];
        for (int d = 0; d < 3; d++) e1[d] = a[d] - ax_x * x[d];
        double n1 = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
        for (int d = 0; d < 3; d++) e1[d] /= n1;
        e2[0] = x[1] * e1[2] - x[2] * e1[1];
        e2[1] = x[2] * e1[0] - x[0] * e1[2];
        e2[2] = x[0] * e1[1] - x[1] * e1[0];
        double xx = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
        /* the polygon (at most M + 4 vertices), in two ping-pong arrays;
         * pass 0 clips the square of half-width ORC_VOR_W, pass 1 clips again
         * from a square twice the extent of pass 0's cell, so that no vertex
         * is computed from far-away corners (their rounding would swamp a
         * small cell) */
        int cap = 64;
        double* pu = malloc(sizeof(double) * 4 * cap);
        int nv = 0;
        double win = ORC_VOR_W;
        for (int pass = 0; pass < 2; pass++) {
        if (pass == 1) {
            double ext = 0.0;
            for (int k = 0; k < nv; k++) {
                if (fabs(pu[2 * k]) > ext) ext = fabs(pu[2 * k]);
                if (fabs(pu[2 * k + 1]) > ext) ext = fabs(pu[2 * k + 1]);
            }
            if (nv < 3 || ext >= 0.999999 * ORC_VOR_W) break;
            win = 2.0 * ext;
        }
        nv = 4;
        pu[0] = -win; pu[1] = -win;
        pu[2] = win;  pu[3] = -win;
        pu[4] = win;  pu[5] = win;
        pu[6] = -win; pu[7] = win;
        for (int64_t j = 0; j < M && nv > 0; j++) {
            if (j == i) continue;
            const double* y = nodes + 3 * j;
            /* (x + u e1 + v e2).(x - y) >= 0, with the difference vector
             * formed first (accurate for close nodes) */
            double dl[3] = {x[0] - y[0], x[1] - y[1], x[2] - y[2]};
            double b = x[0] * dl[0] + x[1] * dl[1] + x[2] * dl[2];
            double cu = -(e1[0] * dl[0] + e1[1] * dl[1] + e1[2] * dl[2]);
            double cv = -(e2[0] * dl[0] + e2[1] * dl[1] + e2[2] * dl[2]);
            if (nv + 2 > cap) {
                cap *= 2;
                pu = realloc(pu, sizeof(double) * 4 * cap);
            }
            double* out = pu + 2 * cap;
            int no = 0;
            for (int k = 0; k < nv; k++) {
                const double* p1 = pu + 2 * k;
                const double* p2 = pu + 2 * ((k + 1) % nv);
                double f1 = b - cu * p1[0] - cv * p1[1];
                double f2 = b - cu * p2[0] - cv * p2[1];
                if (f1 >= 0.0) {
                    out[2 * no] = p1[0];
                    out[2 * no + 1] = p1[1];
                    no++;
                }
                if ((f1 >= 0.0) != (f2 >= 0.0)) {
                    double t = f1 / (f1 - f2);
                    out[2 * no] = p1[0] + t * (p2[0] - p1[0]);
                    out[2 * no + 1] = p1[1] + t * (p2[1] - p1[1]);
                    no++;
                }
            }
            memcpy(pu, out, sizeof(double) * 2 * no);
            nv = no;
        }
        }
        int reach = nv < 3;
        for (int k = 0; k < nv; k++)
            if (fabs(pu[2 * k]) >= 0.999999 * win || fabs(pu[2 * k + 1]) >= 0.999999 * win) reach = 1;
        if (reach) {
            *out_i = NAN;
            bad++;
            free(pu);
            continue;
        }
        /* solid angle of the fan triangle (x, y_k, y_k+1), y = (x + u e1 +
         * v e2)/n with n = |x + u e1 + v e2|: the Van Oosterom-Strackee
         * formula with its triple product (u_k v_l - u_l v_k)/(n_k n_l) and
         * dot products |x|/n, (x.x + u_k u_l + v_k v_l)/(n_k n_l) written in
         * the chart (e1, e2, x/|x| orthonormal), which avoids the
         * cancellation of the triple product of nearly parallel vectors */
        double area = 0.0;
        double xn = sqrt(xx);
        for (int k = 0; k < nv; k++) {
            const double* p1 = pu + 2 * k;
            const double* p2 = pu + 2 * ((k + 1) % nv);
            double nk = sqrt(xx + p1[0] * p1[0] + p1[1] * p1[1]);
            double nl = sqrt(xx + p2[0] * p2[0] + p2[1] * p2[1]);
            double det = (p1[0] * p2[1] - p2[0] * p1[1]) / (nk * nl);
            double den = 1.0 + xn / nk + xn / nl + (xx + p1[0] * p2[0] + p1[1] * p2[1]) / (nk * nl);
            area += 2.0 * atan2(fabs(det), den);
        }
        *out_i = area;
        free(pu);
    }
    return bad;
}

/* ------------------------------------------------------------------ */
/* smoothed adaptive radius (Sec. 2.2, after eq. (12))                 */
/* ------------------------------------------------------------------ */

/* Fibonacci grid of n points on S2 (the auxiliary grid): z_k = 1 - (2k+1)/n,
 * longitude k times the golden angle pi (3 - sqrt 5). */
void orc_fibonacci(int n, double* pts)
{
    const double ga = ORC_PI * (3.0 - sqrt(5.0));
    for (int k = 0; k < n; k++) {
        double z = 1.0 - (2.0 * k + 1.0) / n;
        double r = sqrt((1.0 - z) * (1.0 + z));
        double ph = ga * k;
        pts[3 * k] = r * cos(ph);
        pts[3 * k + 1] = r * sin(ph);
        pts[3 * k + 2] = z;
    }
}

/* d_n, the distance to the n-th nearest node, at every auxiliary point (brute
 * force, as in centre_radius). */
typedef struct {
    int n;
    double* pts;  /* n x 3 */
    double* dn;   /* n */
    double rs;    /* Shepard support radius: three mean spacings of the grid */
} orc_aux;

static void aux_build(const orc_params* p, const double* nodes, int64_t M, orc_aux* a)
{
    a->n = p->smooth_aux;
    a->pts = malloc(sizeof(double) * 3 * (size_t)a->n);
    a->dn = malloc(sizeof(double) * (size_t)a->n);
    a->rs = 3.0 * sqrt(4.0 * ORC_PI / a->n);
    orc_fibonacci(a->n, a->pts);
#pragma omp parallel
    {
        double* kb = malloc(sizeof(double) * (size_t)(M > 0 ? M : 1));
#pragma omp for schedule(dynamic, 16)
        for (int k = 0; k < a->n; k++) {
            for (int64_t i = 0; i < M; i++) kb[i] = prox_key(ORC_S2, nodes + 3 * i, a->pts + 3 * k);
            a->dn[k] = key_distance(ORC_S2, select_kth(kb, M, p->knn_count - 1, 0));
        }
        free(kb);
    }
}

static void aux_free(orc_aux* a)
{
    free(a->pts);
    free(a->dn);
}

/* The degree-zero MLS (Shepard) approximation of d_n at q from the auxiliary
 * values, Wendland weights of support a->rs (the plan's profile). */
static double aux_smooth(const orc_params* p, const orc_aux* a, const double* q)
{
    double sw = 0.0, sv = 0.0;
    for (int k = 0; k < a->n; k++) {
        double d = key_distance(ORC_S2, prox_key(ORC_S2, a->pts + 3 * k, q));
        double w = wendland(p->wendland, d / a->rs);
        sw += w;
        sv += w * a->dn[k];
    }
    return sv / sw;
}

/* The radius of one centre: fixed, adaptive, both (the larger), or (S2,
 * smooth_aux > 0) the smoothed adaptive radius (1 + eps) * smoothed d_n. */
static void centre_radius(const orc_params* p, const orc_aux* aux, const double* q, const double* nodes,
                          int64_t M, double* keybuf, double* delta, double* c, uint8_t* st)
{
    int dom = p->domain;
    int dimx = dom == ORC_SO3 ? 4 : 3;
    double dl = 0.0, cc = 0.0;
    int have = 0;
    *st = 0;
    if (aux) {
        dl = (1.0 + p->knn_eps) * aux_smooth(p, aux, q);
        have = 1;
    } else if (p->knn_count > 0) {
        for (int64_t i = 0; i < M; i++) keybuf[i] = prox_key(dom, nodes + dimx * i, q);
        double tn = select_kth(keybuf, M, p->knn_count - 1, dom == ORC_T3);
        if (dom == ORC_T3) {
            double e = 1.0 + p->knn_eps;
            double e2 = e * e;
            cc = e2 * tn;
            dl = sqrt(cc);
        } else {
            dl = (1.0 + p->knn_eps) * key_distance(dom, tn);
        }
        have = 1;
    }
    if (p->support_radius > 0.0) {
        double d0 = p->support_radius;
        if (!have || d0 > dl) {
            dl = d0;
            if (dom == ORC_T3) cc = d0 * d0;
        }
    }
    if (dom == ORC_S2) {
        if (dl >= 0.5 * ORC_PI) {
            dl = 0.5 * ORC_PI;
            *st |= ORC_ST_HEMISPHERE;
        }
        cc = cos(dl);
    } else if (dom == ORC_SO3) {
        if (dl >= ORC_PI) {
            dl = ORC_PI;
            *st |= ORC_ST_HEMISPHERE;
        }
        cc = cos(0.5 * dl);
    }
    *delta = dl;
    *c = cc;
}

/* Threshold, radius and neighbour count of each requested centre.  rows lists
 * grid indices (NULL = all MQ centres in order). */
int orc_neighbors(const orc_params* p, const double* grid, int64_t MQ, const int64_t* rows,
                  int64_t nrows, const double* nodes, int64_t M, double* thr, double* delta,
                  int32_t* count, uint8_t* status)
{
    if (p->knn_count > M) return -1;
    int dom = p->domain;
    int dimq = dom == ORC_SO3 ? 4 : 3;
    int64_t R = rows ? nrows : MQ;
    orc_aux aux;
    const orc_aux* auxp = NULL;
    if (p->smooth_aux > 0) {
        if (p->domain != ORC_S2 || p->knn_count <= 0) return -1;
        aux_build(p, nodes, M, &aux);
        auxp = &aux;
    }
#pragma omp parallel
    {
        double* kb = malloc(sizeof(double) * (size_t)(M > 0 ? M : 1));
#pragma omp for schedule(dynamic, 16)
        for (int64_t r = 0; r < R; r++) {
            int64_t j = rows ? rows[r] : r;
            const double* q = grid + dimq * j;
            double dl, c;
            uint8_t st;
            centre_radius(p, auxp, q, nodes, M, kb, &dl, &c, &st);
            int32_t cnt = 0;
            for (int64_t i = 0; i < M; i++)
                if (key_inside(dom, prox_key(dom, nodes + dimq * i, q), c)) cnt++;
            thr[r] = c;
            delta[r] = dl;
            count[r] = cnt;
            status[r] = st;
        }
        free(kb);
    }
    if (auxp) aux_free(&aux);
    return 0;
}

/* Neighbour index lists for the requested centres, ascending original index.
 * row_ptr (R+1) must come from the counts of orc_neighbors. */
int orc_neighbor_lists(const orc_params* p, const double* grid, const int64_t* rows, int64_t nrows,
                       const double* nodes, int64_t M, const double* thr, const int64_t* row_ptr,
                       int32_t* idx)
{
    int dom = p->domain;
    int dimq = dom == ORC_SO3 ? 4 : 3;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < nrows; r++) {
        int64_t j = rows ? rows[r] : r;
        const double* q = grid + dimq * j;
        int64_t o = row_ptr[r];
        for (int64_t i = 0; i < M; i++)
            if (key_inside(dom, prox_key(dom, nodes + dimq * i, q), thr[r])) idx[o++] = (int32_t)i;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* local coordinates (Sec. 2.3, "Locally adapted ansatz space")        */
/* ------------------------------------------------------------------ */

/* Coordinates of node x in the tangent space at centre q, divided by the
 * scale s (any positive scale: the basis is renormalised below).
 * S2 : orthogonal projection P_q x expressed in the frame
 *      e_theta = (cos th cos ph, cos th sin ph, -sin th), e_phi = (-sin ph, cos ph, 0).
 * SO3: projection of the representative on q's hemisphere onto T_q S^3,
 *      expressed in the frame q*i, q*j, q*k, i.e. Im(conj(q) x) sign(q.x).
 * T3 : min-image difference x - q. */
static void tangent_coords(int dom, const double* x, const double* q, double s, double* u)
{
    if (dom == ORC_S2) {
        double rho = sqrt(q[0] * q[0] + q[1] * q[1]);
        double cth = q[2], sth = rho;
        double cph = q[0] / rho, sph = q[1] / rho;
        double et[3] = {cth * cph, cth * sph, -sth};
        double ep[3] = {-sph, cph, 0.0};
        u[0] = (x[0] * et[0] + x[1] * et[1] + x[2] * et[2]) / s;
        u[1] = (x[0] * ep[0] + x[1] * ep[1] + x[2] * ep[2]) / s;
    } else if (dom == ORC_SO3) {
        double dot = q[0] * x[0] + q[1] * x[1] + q[2] * x[2] + q[3] * x[3];
        double sg = dot < 0.0 ? -1.0 : 1.0;
        /* Im(conj(q) x) = q0 x_v - x0 q_v - q_v cross x_v */
        double im0 = q[0] * x[1] - x[0] * q[1] - (q[2] * x[3] - q[3] * x[2]);
        double im1 = q[0] * x[2] - x[0] * q[2] - (q[3] * x[1] - q[1] * x[3]);
        double im2 = q[0] * x[3] - x[0] * q[3] - (q[1] * x[2] - q[2] * x[1]);
        u[0] = sg * im0 / s;
        u[1] = sg * im1 / s;
        u[2] = sg * im2 / s;
    } else {
        for (int i = 0; i < 3; i++) {
            double dlt = x[i] - q[i];
            dlt = dlt - nearbyint(dlt);
            u[i] = dlt / s;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Householder QR (library-primitive step of the local solve)          */
/* ------------------------------------------------------------------ */

/* In-place Householder QR of the column-major n x c matrix A (leading dim
 * lda).  The reflections are also applied to the n x e matrix E (leading dim
 * lde).  On return the upper triangle of A holds R (diagonal may be negative),
 * and E holds Q^T E. */
static void householder_qr(int n, int c, double* A, int lda, int e, double* E, int lde)
{
    for (int k = 0; k < c && k < n; k++) {
        double* a = A + (size_t)k * lda;
        double nrm = 0.0;
        for (int i = k; i < n; i++) nrm += a[i] * a[i];
        nrm = sqrt(nrm);
        if (nrm == 0.0) continue;
        double alpha = a[k] > 0.0 ? -nrm : nrm;
        double v0 = a[k] - alpha;
        double vv = v0 * v0;
        for (int i = k + 1; i < n; i++) vv += a[i] * a[i];
        if (vv == 0.0) {
            a[k] = alpha;
            continue;
        }
        a[k] = v0;
        for (int j = k + 1; j < c + e; j++) {
            double* col = j < c ? A + (size_t)j * lda : E + (size_t)(j - c) * lde;
            double s = 0.0;
            for (int i = k; i < n; i++) s += a[i] * col[i];
            s *= 2.0 / vv;
            for (int i = k; i < n; i++) col[i] -= s * a[i];
        }
        a[k] = alpha;
        for (int i = k + 1; i < n; i++) a[i] = 0.0;
    }
}

/* ------------------------------------------------------------------ */
/* regularization strength (Sec. 2.3, eq. (23))                        */
/* ------------------------------------------------------------------ */

/* r_tau = sum_j d_j^2 / (1 + tau mu_j)  (eq. (23)) */
static double coupling(int n, const double* d, const double* mu, double tau)
{
    double r = 0.0;
    for (int j = 0; j < n; j++) r += d[j] * d[j] / (1.0 + tau * mu[j]);
    return r;
}

/* tau with chi_tau = chi_T by bisection.  Reading (paper: "computed via
 * bisection", no bracket given): bisection on log(tau) between 1e-16 and the
 * first power of two at which r_tau <= 1 - 1/chi_T, 64 halvings, midpoint. */
static double tau_by_bisection(int n, const double* d, const double* mu, double chi_t)
{
    double target = 1.0 - 1.0 / chi_t;
    double hi = 1.0;
    int guard = 0;
    while (coupling(n, d, mu, hi) > target && guard < 2000) {
        hi *= 2.0;
        guard++;
    }
    double a = log(1e-16), b = log(hi);
    for (int it = 0; it < 64; it++) {
        double mid = 0.5 * (a + b);
        if (coupling(n, d, mu, exp(mid)) > target)
            a = mid;
        else
            b = mid;
    }
    return exp(0.5 * (a + b));
}

/* Smooth transition of Sec. 2.3.  Reading (paper gives only the end
 * conditions and C^3): tau~ = S(t) tau with t = (chi - chi_T)/(chi_full -
 * chi_T) clipped to [0,1] and S(t) = 35t^4 - 84t^5 + 70t^6 - 20t^7. */
static double transition(double chi, double chi_t, double chi_f)
{
    double t = (chi - chi_t) / (chi_f - chi_t);
    if (t <= 0.0) return 0.0;
    if (t >= 1.0) return 1.0;
    double t4 = t * t * t * t;
    return t4 * (35.0 - 84.0 * t + 70.0 * t * t - 20.0 * t * t * t);
}

/* Degree multiplier mu of eq. (21): S2 l(l+1) (d = 2, s = 1); SO3 l(l+1);
 * T3 l^2. */
static double degree_multiplier(int dom, int l)
{
    if (dom == ORC_T3) return (double)l * l;
    return (double)l * (l + 1);
}

/* ------------------------------------------------------------------ */
/* the MLS value at one centre (eq. (4), (14)-(23))                    */
/* ------------------------------------------------------------------ */

typedef struct {
    double* B;    /* n x m column-major */
    double* E;    /* n x (1+F) : v_1 and the weighted data */
    double* Aug;  /* (n+m-1) x m augmented matrix */
    double* Rhs;  /* (n+m-1) x F */
    double* w;
    double* g;    /* n x m raw monomial values */
    int32_t* nb;
    int cap;
    int fcap; /* fields E and Rhs hold */
} orc_work;

static void work_reserve(orc_work* wk, int n, int m, int F)
{
    if (n <= wk->cap && F <= wk->fcap) return;
    int cap = n + 64 > wk->cap ? n + 64 : wk->cap;
    if (F < wk->fcap) F = wk->fcap;
    free(wk->B); free(wk->E); free(wk->Aug); free(wk->Rhs); free(wk->w); free(wk->g); free(wk->nb);
    wk->B = malloc(sizeof(double) * (size_t)cap * m);
    wk->E = malloc(sizeof(double) * (size_t)cap * (1 + F));
    wk->Aug = malloc(sizeof(double) * (size_t)(cap + m) * m);
    wk->Rhs = malloc(sizeof(double) * (size_t)(cap + m) * F);
    wk->w = malloc(sizeof(double) * (size_t)cap);
    wk->g = malloc(sizeof(double) * (size_t)cap * m);
    wk->nb = malloc(sizeof(int32_t) * (size_t)cap);
    wk->cap = cap;
    wk->fcap = F;
}

static void work_free(orc_work* wk)
{
    free(wk->B); free(wk->E); free(wk->Aug); free(wk->Rhs); free(wk->w); free(wk->g); free(wk->nb);
}

/* The MLS value(s) at centre q from its neighbours nb[0..n-1].
 * Steps, in the paper's order:
 *  1. weights w_i = phi(d(q,x_i)/delta) nu_i, normalised to sum 1 (Sec. 2.3)
 *  2. monomial basis of Pi_K^tan centred at q, sorted by degree, each scaled
 *     to unit discrete norm; g_1 = 1 (Sec. 2.3)
 *  3. B = (sqrt(w_i) g_j(x_i)), y_w = (sqrt(w_i) y_i)  (eq. (14))
 *  4. B = (v_1 V); the Cholesky factor L of C = V^T V is obtained as R^T
 *     from a Householder QR of V (eq. (20)); d = L^{-1} b with b = V^T v_1
 *     equals S Q^T v_1, S = sign(diag R)
 *  5. chi = 1/(1 - |d|^2)  (eq. (19)), with 1 - |d|^2 taken as the squared
 *     residual of v_1 off span(V)
 *  6. tau: none / fixed / chi-target by bisection + smooth transition
 *  7. c_1 = first coefficient of the minimiser of (22), obtained by a second
 *     Householder QR of the augmented least-squares matrix
 *        [ v_1  V ; 0  sqrt(tau) D^{1/2} L^T ],  right side [ y_w ; 0 ].
 * Degenerate centres: no neighbour -> NaN and EMPTY; fewer than m neighbours,
 * a zero monomial column or |R_jj| <= 1e-11 -> the tau -> infinity limit
 * (Shepard mean, Sec. 2.3) and UNDERDETERMINED.
 * unit = 1: the data are the n unit vectors of the neighbourhood (field f has
 * y = 1 at neighbour f, 0 elsewhere; F = n, vals unused), so that out[f] is
 * the generating function a*_f of Rem. 2.5. */
static void mls_centre(const orc_params* p, const double* q, double delta, int n,
                       const double* nodes, const double* nu, const double* vals, int F,
                       int64_t ld, const int* exps, const int* degs, int m, orc_work* wk,
                       double* out, int64_t out_stride, double* chi_out, double* tau_out,
                       uint8_t* st, int unit)
{
    int dom = p->domain;
    int D = tangent_dim(dom);
    int dimx = dom == ORC_SO3 ? 4 : 3;
    double scale = dom == ORC_SO3 ? 0.5 * delta : delta;
    const int32_t* nb = wk->nb;
    if (n == 0) {
        for (int f = 0; f < F; f++) out[f * out_stride] = NAN;
        *chi_out = NAN;
        *tau_out = NAN;
        *st |= ORC_ST_EMPTY;
        return;
    }
    /* step 1 */
    double W = 0.0;
    for (int i = 0; i < n; i++) {
        const double* x = nodes + (size_t)dimx * nb[i];
        double dist = key_distance(dom, prox_key(dom, x, q));
        double wi = wendland(p->wendland, dist / delta);
        if (nu) wi *= nu[nb[i]];
        wk->w[i] = wi;
        W += wi;
    }
    if (!(W > 0.0)) {
        for (int f = 0; f < F; f++) out[f * out_stride] = NAN;
        *chi_out = NAN;
        *tau_out = NAN;
        *st |= ORC_ST_EMPTY;
        return;
    }
    for (int i = 0; i < n; i++) wk->w[i] /= W;

    /* Shepard mean: the tau -> infinity limit, used for degenerate centres */
    int degenerate = n < m;

    /* step 2 */
    double u[3];
    for (int i = 0; i < n; i++) {
        tangent_coords(dom, nodes + (size_t)dimx * nb[i], q, scale, u);
        for (int a = 0; a < m; a++) {
            double v = 1.0;
            for (int c = 0; c < D; c++) v *= ipow(u[c], exps[3 * a + c]);
            wk->g[(size_t)a * n + i] = v;
        }
    }
    double colscale[64];
    for (int a = 0; a < m; a++) {
        double s = 0.0;
        for (int i = 0; i < n; i++) s += wk->w[i] * wk->g[(size_t)a * n + i] * wk->g[(size_t)a * n + i];
        colscale[a] = sqrt(s);
        if (!(colscale[a] > 0.0)) degenerate = 1;
    }

    if (!degenerate && m > 1) {
        /* step 3: V (columns 2..m) into B, [v_1, y_w] into E */
        int mv = m - 1;
        for (int a = 1; a < m; a++)
            for (int i = 0; i < n; i++)
                wk->B[(size_t)(a - 1) * n + i] = sqrt(wk->w[i]) * wk->g[(size_t)a * n + i] / colscale[a];
        for (int i = 0; i < n; i++) wk->E[i] = sqrt(wk->w[i]);
        const int FE = unit ? 0 : F; /* the data columns of E are not used below */
        for (int f = 0; f < FE; f++)
            for (int i = 0; i < n; i++)
                wk->E[(size_t)(1 + f) * n + i] = sqrt(wk->w[i]) * vals[f * ld + nb[i]];
        /* step 4 */
        householder_qr(n, mv, wk->B, n, 1 + FE, wk->E, n);
        double rmax = 0.0, rmin = INFINITY;
        for (int j = 0; j < mv; j++) {
            double r = fabs(wk->B[(size_t)j * n + j]);
            if (r > rmax) rmax = r;
            if (r < rmin) rmin = r;
        }
        if (!(rmin > 1e-11)) degenerate = 1;
        if (!degenerate) {
            double d[64], mu[64], sgn[64];
            for (int j = 0; j < mv; j++) {
                sgn[j] = wk->B[(size_t)j * n + j] < 0.0 ? -1.0 : 1.0;
                d[j] = sgn[j] * wk->E[j];
                mu[j] = degree_multiplier(dom, degs[j + 1]);
            }
            /* step 5: since |v_1| = 1 (weights normalised to sum 1),
             * 1 - |d|^2 = |(I - P_V) v_1|^2, the squared norm of the entries
             * of Q^T v_1 below the first m-1; summed directly, without the
             * cancellation of 1 - |d|^2 when v_1 is close to span(V) */
            double res = 0.0;
            for (int i = mv; i < n; i++) res += wk->E[i] * wk->E[i];
            double chi = 1.0 / res;
            /* step 6 */
            double tau = 0.0;
            if (p->reg == ORC_REG_FIXED) {
                tau = p->tau_fixed;
            } else if (p->reg == ORC_REG_CHI && chi > p->chi_target) {
                double s = transition(chi, p->chi_target, p->chi_full);
                tau = s * tau_by_bisection(mv, d, mu, p->chi_target);
            }
            /* step 7 */
            int na = n + mv;
            double* A = wk->Aug;
            double* Rh = wk->Rhs;
            for (int i = 0; i < na * m; i++) A[i] = 0.0;
            for (int i = 0; i < n; i++) A[i] = sqrt(wk->w[i]);
            for (int a = 1; a < m; a++)
                for (int i = 0; i < n; i++)
                    A[(size_t)a * na + i] =
                        sqrt(wk->w[i]) * wk->g[(size_t)a * n + i] / colscale[a];
            if (tau > 0.0) {
                /* rows n+j: sqrt(tau mu_j) (L^T)_{j,:} = sqrt(tau mu_j) sgn_j R_{j,:} */
                for (int j = 0; j < mv; j++)
                    for (int c = j; c < mv; c++)
                        A[(size_t)(c + 1) * na + n + j] =
                            sqrt(tau * mu[j]) * sgn[j] * wk->B[(size_t)c * n + j];
            }
            for (int f = 0; f < F; f++) {
                for (int i = 0; i < n; i++)
                    Rh[(size_t)f * na + i] =
                        unit ? (i == f ? sqrt(wk->w[i]) : 0.0) : sqrt(wk->w[i]) * vals[f * ld + nb[i]];
                for (int i = n; i < na; i++) Rh[(size_t)f * na + i] = 0.0;
            }
            householder_qr(na, m, A, na, F, Rh, na);
            for (int f = 0; f < F; f++) {
                double x[64];
                for (int a = m - 1; a >= 0; a--) {
                    double s = Rh[(size_t)f * na + a];
                    for (int c = a + 1; c < m; c++) s -= A[(size_t)c * na + a] * x[c];
                    x[a] = s / A[(size_t)a * na + a];
                }
                out[f * out_stride] = x[0];
            }
            *chi_out = chi;
            *tau_out = tau;
            if (tau > 0.0) *st |= ORC_ST_REGULARIZED;
            return;
        }
    }
    if (m == 1 && !degenerate) {
        /* K = 0: c_1 is the weighted mean itself, chi = 1 */
        for (int f = 0; f < F; f++) {
            double s = 0.0;
            for (int i = 0; i < n; i++) s += wk->w[i] * (unit ? (double)(i == f) : vals[f * ld + nb[i]]);
            out[f * out_stride] = s;
        }
        *chi_out = 1.0;
        *tau_out = 0.0;
        return;
    }
    for (int f = 0; f < F; f++) {
        double s = 0.0;
        for (int i = 0; i < n; i++) s += wk->w[i] * (unit ? (double)(i == f) : vals[f * ld + nb[i]]);
        out[f * out_stride] = s;
    }
    *chi_out = INFINITY;
    *tau_out = INFINITY;
    *st |= ORC_ST_UNDERDETERMINED;
}

/* Step 2 of Alg. 1: MLS values at the requested grid centres.
 * vals is F x M (row f at vals + f*ld).  out is F x R (row stride R).
 * Per-centre diagnostics: n_j, chi, tau, status bits. */
int orc_mls(const orc_params* p, const double* grid, int64_t MQ, const int64_t* rows,
            int64_t nrows, const double* nodes, int64_t M, const double* nu, const double* vals,
            int32_t F, int64_t ld, double* out, int32_t* nj, double* chi, double* tau,
            uint8_t* status)
{
    if (p->knn_count > M || F < 1) return -1;
    if (p->support_radius <= 0.0 && p->knn_count <= 0) return -1;
    int dom = p->domain;
    int D = tangent_dim(dom);
    int K = p->degree;
    if (K < 0 || K > 6) return -1;
    int m = n_monomials(D, K);
    int exps[3 * 128], degs[128];
    monomial_exponents(D, K, exps, degs);
    int dimq = dom == ORC_SO3 ? 4 : 3;
    int64_t R = rows ? nrows : MQ;
    orc_aux aux;
    const orc_aux* auxp = NULL;
    if (p->smooth_aux > 0) {
        if (p->domain != ORC_S2 || p->knn_count <= 0) return -1;
        aux_build(p, nodes, M, &aux);
        auxp = &aux;
    }
#pragma omp parallel
    {
        orc_work wk;
        memset(&wk, 0, sizeof(wk));
        double* kb = malloc(sizeof(double) * (size_t)(M > 0 ? M : 1));
#pragma omp for schedule(dynamic, 8)
        for (int64_t r = 0; r < R; r++) {
            int64_t j = rows ? rows[r] : r;
            const double* q = grid + dimq * j;
            double dl, c;
            uint8_t st;
            centre_radius(p, auxp, q, nodes, M, kb, &dl, &c, &st);
            int n = 0;
            for (int64_t i = 0; i < M; i++)
                if (key_inside(dom, prox_key(dom, nodes + dimq * i, q), c)) n++;
            work_reserve(&wk, n > 0 ? n : 1, m, F);
            n = 0;
            for (int64_t i = 0; i < M; i++)
                if (key_inside(dom, prox_key(dom, nodes + dimq * i, q), c)) wk.nb[n++] = (int32_t)i;
            mls_centre(p, q, dl, n, nodes, nu, vals, F, ld, exps, degs, m, &wk, out + r, R,
                       chi + r, tau + r, &st, 0);
            nj[r] = n;
            status[r] = st;
        }
        work_free(&wk);
        free(kb);
    }
    if (auxp) aux_free(&aux);
    return 0;
}

/* Generating functions of MLS at the requested centres (Rem. 2.5).  The MLS
 * value is linear in the data, M_y(q) = sum_i a*_i y_i, and a*_i is, by that
 * definition, the MLS value of the data vector that is 1 at neighbour i and 0
 * elsewhere: computed exactly so, by the local solve above with the n unit
 * vectors as its fields.  row_ptr (R + 1) comes from the counts of
 * orc_neighbors; idx receives the neighbours (ascending original index) and
 * val the a*_i, row by row; chi, tau and status as for orc_mls. */
int orc_generating(const orc_params* p, const double* grid, int64_t MQ, const int64_t* rows,
                   int64_t nrows, const double* nodes, int64_t M, const double* nu,
                   const int64_t* row_ptr, int32_t* idx, double* val, double* chi, double* tau,
                   uint8_t* status)
{
    if (p->knn_count > M) return -1;
    if (p->support_radius <= 0.0 && p->knn_count <= 0) return -1;
    int dom = p->domain;
    int D = tangent_dim(dom);
    int K = p->degree;
    if (K < 0 || K > 6) return -1;
    int m = n_monomials(D, K);
    int exps[3 * 128], degs[128];
    monomial_exponents(D, K, exps, degs);
    int dimq = dom == ORC_SO3 ? 4 : 3;
    int64_t R = rows ? nrows : MQ;
    int bad = 0;
    orc_aux aux;
    const orc_aux* auxp = NULL;
    if (p->smooth_aux > 0) {
        if (p->domain != ORC_S2 || p->knn_count <= 0) return -1;
        aux_build(p, nodes, M, &aux);
        auxp = &aux;
    }
#pragma omp parallel
    {
        orc_work wk;
        memset(&wk, 0, sizeof(wk));
        double* kb = malloc(sizeof(double) * (size_t)(M > 0 ? M : 1));
#pragma omp for schedule(dynamic, 8)
        for (int64_t r = 0; r < R; r++) {
            int64_t j = rows ? rows[r] : r;
            const double* q = grid + dimq * j;
            double dl, c;
            uint8_t st;
            centre_radius(p, auxp, q, nodes, M, kb, &dl, &c, &st);
            int n = 0;
            for (int64_t i = 0; i < M; i++)
                if (key_inside(dom, prox_key(dom, nodes + dimq * i, q), c)) n++;
            if (n != row_ptr[r + 1] - row_ptr[r]) {
#pragma omp atomic write
                bad = 1;
                continue;
            }
            work_reserve(&wk, n > 0 ? n : 1, m, n > 0 ? n : 1);
            n = 0;
            for (int64_t i = 0; i < M; i++)
                if (key_inside(dom, prox_key(dom, nodes + dimq * i, q), c)) wk.nb[n++] = (int32_t)i;
            for (int k = 0; k < n; k++) idx[row_ptr[r] + k] = wk.nb[k];
            mls_centre(p, q, dl, n, nodes, nu, NULL, n, 0, exps, degs, m, &wk, val + row_ptr[r], 1,
                       chi + r, tau + r, &st, 1);
            status[r] = st;
        }
        work_free(&wk);
        free(kb);
    }
    if (auxp) aux_free(&aux);
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------ */
/* harmonic bases                                                      */
/* ------------------------------------------------------------------ */

/* Fully normalised associated Legendre functions with the Condon-Shortley
 * phase, P_n^k(x) for 0 <= k <= n <= N, stored at n(n+1)/2 + k.  The
 * normalisation makes Y_n^k(theta,phi) = P_n^k(cos theta) e^{ik phi}
 * orthonormal on S2 (surface measure, total 4 pi). */
void orc_alf(int N, double x, double* P)
{
    double s = sqrt((1.0 - x) * (1.0 + x));
    double pkk = 1.0 / sqrt(4.0 * ORC_PI);
    for (int k = 0; k <= N; k++) {
        if (k > 0) pkk = -sqrt((2.0 * k + 1.0) / (2.0 * k)) * s * pkk;
        P[(size_t)k * (k + 1) / 2 + k] = pkk;
        if (k + 1 <= N) P[(size_t)(k + 1) * (k + 2) / 2 + k] = sqrt(2.0 * k + 3.0) * x * pkk;
        for (int n = k + 2; n <= N; n++) {
            double a = sqrt((4.0 * n * n - 1.0) / ((double)n * n - (double)k * k));
            double b = sqrt((((double)n - 1) * (n - 1) - (double)k * k) /
                            (4.0 * ((double)n - 1) * (n - 1) - 1.0));
            P[(size_t)n * (n + 1) / 2 + k] =
                a * (x * P[(size_t)(n - 1) * n / 2 + k] - b * P[(size_t)(n - 2) * (n - 1) / 2 + k]);
        }
    }
}

static double log_sqrt_binom(int n, int k)
{
    return 0.5 * (lgamma(n + 1.0) - lgamma(k + 1.0) - lgamma(n - k + 1.0));
}

/* Wigner d^n_{k,k'}(beta) = <n k| exp(-i beta J_y) |n k'> for all n <= N,
 * |k|,|k'| <= n, stored at sum_{l<n}(2l+1)^2 + (k+n)(2n+1) + (k'+n).
 * Start value at n0 = max(|k|,|k'|) in closed form, then the three-term
 * recurrence in n. */
void orc_wigner_d(int N, double beta, double* d)
{
    double cb = cos(beta);
    double lc = log(cos(0.5 * beta)), ls = log(sin(0.5 * beta));
    double c2 = cos(0.5 * beta), s2 = sin(0.5 * beta);
    for (int k = -N; k <= N; k++)
        for (int kp = -N; kp <= N; kp++) {
            int n0 = abs(k) > abs(kp) ? abs(k) : abs(kp);
            double dn, dm1 = 0.0;
            int j = n0;
            if (n0 == 0) {
                dn = 1.0;
            } else {
                int pc, ps;       /* powers of cos(b/2), sin(b/2) */
                double lb, sign;  /* log sqrt binom and sign */
                if (k == n0) {
                    pc = n0 + kp; ps = n0 - kp; lb = log_sqrt_binom(2 * n0, n0 + kp);
                    sign = (ps % 2) ? -1.0 : 1.0;
                } else if (k == -n0) {
                    pc = n0 - kp; ps = n0 + kp; lb = log_sqrt_binom(2 * n0, n0 - kp);
                    sign = 1.0;
                } else if (kp == n0) {
                    pc = n0 + k; ps = n0 - k; lb = log_sqrt_binom(2 * n0, n0 + k);
                    sign = 1.0;
                } else {
                    pc = n0 - k; ps = n0 + k; lb = log_sqrt_binom(2 * n0, n0 - k);
                    sign = (ps % 2) ? -1.0 : 1.0;
                }
                double v;
                if ((ps > 0 && s2 == 0.0) || (pc > 0 && c2 == 0.0))
                    v = 0.0;
                else
                    v = exp(lb + (pc ? pc * lc : 0.0) + (ps ? ps * ls : 0.0));
                dn = sign * v;
            }
            for (;;) {
                size_t base = 0;
                for (int l = 0; l < j; l++) base += (size_t)(2 * l + 1) * (2 * l + 1);
                d[base + (size_t)(k + j) * (2 * j + 1) + (kp + j)] = dn;
                if (j >= N) break;
                double nx;
                if (j == 0) {
                    nx = cb;
                } else {
                    double jj = j;
                    double num = (2.0 * jj + 1.0) * (jj * (jj + 1.0) * cb - (double)k * kp) * dn -
                                 (jj + 1.0) * sqrt((jj * jj - (double)k * k) * (jj * jj - (double)kp * kp)) * dm1;
                    double den = jj * sqrt(((jj + 1) * (jj + 1) - (double)k * k) *
                                           ((jj + 1) * (jj + 1) - (double)kp * kp));
                    nx = num / den;
                }
                dm1 = dn;
                dn = nx;
                j++;
            }
        }
}

int64_t orc_num_coeffs(const orc_params* p)
{
    int N = p->bandwidth;
    if (p->domain == ORC_S2) return (int64_t)(N + 1) * (N + 1);
    if (p->domain == ORC_SO3) return (int64_t)(N + 1) * (2 * N + 1) * (2 * N + 3) / 3;
    int32_t d[3];
    if (orc_grid_dims(p, d)) return -1;
    return (int64_t)d[0] * d[0] * d[0];
}

/* ------------------------------------------------------------------ */
/* quadrature (Alg. 1 step 3, eq. (25))                                */
/* ------------------------------------------------------------------ */

/* fhat_k = sum_j omega_j f_j conj(phi_k(q_j)), for F real fields given on the
 * grid (gv is F x MQ).  coeffs is F x n_coeff x 2 (re, im).
 * literal != 0 evaluates the double sum term by term (small bandwidths);
 * otherwise the same finite sum is evaluated ring by ring (a direct DFT over
 * the periodic angle(s), then the sum over the remaining angle), which is the
 * same sum reordered, without any FFT. */
int orc_coeffs(const orc_params* p, const double* gv, int32_t F, double* coeffs, int literal)
{
    int32_t dm[3];
    if (orc_grid_dims(p, dm)) return -1;
    int N = p->bandwidth;
    int64_t MQ = (int64_t)dm[0] * dm[1] * dm[2];
    int64_t nc = orc_num_coeffs(p);
    int dimq = p->domain == ORC_SO3 ? 4 : 3;
    double* pts = malloc(sizeof(double) * dimq * MQ);
    double* wts = malloc(sizeof(double) * MQ);
    orc_grid(p, pts, wts);
    memset(coeffs, 0, sizeof(double) * 2 * nc * F);
    if (p->domain == ORC_S2) {
        int nt = dm[0], np = dm[1];
        double* x = malloc(sizeof(double) * nt);
        double* w = malloc(sizeof(double) * nt);
        orc_gauss_legendre(nt, x, w);
        size_t na = (size_t)(N + 1) * (N + 2) / 2;
        if (literal) {
#pragma omp parallel for schedule(dynamic, 1)
            for (int f = 0; f < F; f++) {
                double* P = malloc(sizeof(double) * na);
                for (int t = 0; t < nt; t++) {
                    orc_alf(N, x[t], P);
                    for (int q = 0; q < np; q++) {
                        int64_t j = (int64_t)t * np + q;
                        double phi = 2.0 * ORC_PI * q / np;
                        double fv = wts[j] * gv[f * MQ + j];
                        for (int n = 0; n <= N; n++)
                            for (int k = -n; k <= n; k++) {
                                int ak = abs(k);
                                double pv = P[(size_t)n * (n + 1) / 2 + ak];
                                if (k < 0 && (ak % 2)) pv = -pv;
                                /* conj(Y) = pv e^{-ik phi} */
                                double* c = coeffs + 2 * ((int64_t)f * nc + n * n + n + k);
                                c[0] += fv * pv * cos(k * phi);
                                c[1] -= fv * pv * sin(k * phi);
                            }
                    }
                }
                free(P);
            }
        } else {
#pragma omp parallel for schedule(dynamic, 1)
            for (int f = 0; f < F; f++) {
                double* P = malloc(sizeof(double) * na);
                double* G = malloc(sizeof(double) * 2 * (2 * N + 1));
                for (int t = 0; t < nt; t++) {
                    for (int k = -N; k <= N; k++) {
                        double re = 0.0, im = 0.0;
                        for (int q = 0; q < np; q++) {
                            double phi = 2.0 * ORC_PI * q / np;
                            double fv = gv[f * MQ + (int64_t)t * np + q];
                            re += fv * cos(k * phi);
                            im -= fv * sin(k * phi);
                        }
                        G[2 * (k + N)] = re * 2.0 * ORC_PI / np;
                        G[2 * (k + N) + 1] = im * 2.0 * ORC_PI / np;
                    }
                    orc_alf(N, x[t], P);
                    for (int n = 0; n <= N; n++)
                        for (int k = -n; k <= n; k++) {
                            int ak = abs(k);
                            double pv = w[t] * P[(size_t)n * (n + 1) / 2 + ak];
                            if (k < 0 && (ak % 2)) pv = -pv;
                            double* c = coeffs + 2 * ((int64_t)f * nc + n * n + n + k);
                            c[0] += pv * G[2 * (k + N)];
                            c[1] += pv * G[2 * (k + N) + 1];
                        }
                }
                free(P);
                free(G);
            }
        }
        free(x);
        free(w);
    } else if (p->domain == ORC_SO3) {
        int nb = dm[0], nal = dm[1], ngm = dm[2];
        double* x = malloc(sizeof(double) * nb);
        double* w = malloc(sizeof(double) * nb);
        orc_gauss_legendre(nb, x, w);
        size_t nd = (size_t)nc;
        int K2 = 2 * N + 1;
#pragma omp parallel for schedule(dynamic, 1)
        for (int t = 0; t < nb; t++) {
            double* dd = malloc(sizeof(double) * nd);
            double* G = malloc(sizeof(double) * 2 * K2 * K2);
            double* H = malloc(sizeof(double) * 2 * K2 * ngm);
            double* part = malloc(sizeof(double) * 2 * nc);
            orc_wigner_d(N, acos(x[t]), dd);
            for (int f = 0; f < F; f++) {
                const double* fs = gv + f * MQ + (int64_t)t * nal * ngm;
                /* H(k, g) = dA sum_a f(a,g) e^{+ik alpha_a} */
                for (int k = -N; k <= N; k++)
                    for (int g = 0; g < ngm; g++) {
                        double re = 0.0, im = 0.0;
                        for (int a = 0; a < nal; a++) {
                            double al = 2.0 * ORC_PI * a / nal;
                            re += fs[(int64_t)a * ngm + g] * cos(k * al);
                            im += fs[(int64_t)a * ngm + g] * sin(k * al);
                        }
                        H[2 * ((k + N) * ngm + g)] = re * 2.0 * ORC_PI / nal;
                        H[2 * ((k + N) * ngm + g) + 1] = im * 2.0 * ORC_PI / nal;
                    }
                /* G(k, k') = dG sum_g H(k,g) e^{+ik' gamma_g} */
                for (int k = -N; k <= N; k++)
                    for (int kp = -N; kp <= N; kp++) {
                        double re = 0.0, im = 0.0;
                        for (int g = 0; g < ngm; g++) {
                            double gm = 2.0 * ORC_PI * g / ngm;
                            double hr = H[2 * ((k + N) * ngm + g)], hi = H[2 * ((k + N) * ngm + g) + 1];
                            double c = cos(kp * gm), s = sin(kp * gm);
                            re += hr * c - hi * s;
                            im += hr * s + hi * c;
                        }
                        G[2 * ((k + N) * K2 + kp + N)] = re * 2.0 * ORC_PI / ngm;
                        G[2 * ((k + N) * K2 + kp + N) + 1] = im * 2.0 * ORC_PI / ngm;
                    }
                size_t base = 0;
                for (int n = 0; n <= N; n++) {
                    double cn = sqrt((2.0 * n + 1.0) / (8.0 * ORC_PI * ORC_PI));
                    for (int k = -n; k <= n; k++)
                        for (int kp = -n; kp <= n; kp++) {
                            size_t id = base + (size_t)(k + n) * (2 * n + 1) + (kp + n);
                            double v = w[t] * cn * dd[id];
                            part[2 * id] = v * G[2 * ((k + N) * K2 + kp + N)];
                            part[2 * id + 1] = v * G[2 * ((k + N) * K2 + kp + N) + 1];
                        }
                    base += (size_t)(2 * n + 1) * (2 * n + 1);
                }
#pragma omp critical
                for (int64_t i = 0; i < 2 * nc; i++) coeffs[2 * (int64_t)f * nc + i] += part[i];
            }
            free(dd); free(G); free(H); free(part);
        }
        free(x);
        free(w);
    } else {
        int n = dm[0];
        int h = n / 2;
        /* separable direct DFT along each axis: A1(k0,i1,i2), A2(k0,k1,i2), A3 */
        double* A = malloc(sizeof(double) * 2 * MQ);
        double* Bv = malloc(sizeof(double) * 2 * MQ);
        double* cs = malloc(sizeof(double) * n);
        double* sn = malloc(sizeof(double) * n);
        for (int i = 0; i < n; i++) {
            cs[i] = cos(2.0 * ORC_PI * i / n);
            sn[i] = sin(2.0 * ORC_PI * i / n);
        }
        for (int f = 0; f < F; f++) {
            const double* fs = gv + f * MQ;
            /* axis 0 */
#pragma omp parallel for schedule(static)
            for (int k0 = 0; k0 < n; k0++)
                for (int64_t r = 0; r < (int64_t)n * n; r++) {
                    double re = 0.0, im = 0.0;
                    int kk = k0 - h;
                    for (int i = 0; i < n; i++) {
                        int e = (int)((((int64_t)kk * i) % n + n) % n);
                        re += fs[(int64_t)i * n * n + r] * cs[e];
                        im -= fs[(int64_t)i * n * n + r] * sn[e];
                    }
                    A[2 * ((int64_t)k0 * n * n + r)] = re;
                    A[2 * ((int64_t)k0 * n * n + r) + 1] = im;
                }
            /* axis 1 */
#pragma omp parallel for schedule(static)
            for (int k0 = 0; k0 < n; k0++)
                for (int k1 = 0; k1 < n; k1++)
                    for (int i2 = 0; i2 < n; i2++) {
                        double re = 0.0, im = 0.0;
                        int kk = k1 - h;
                        for (int i = 0; i < n; i++) {
                            int e = (int)((((int64_t)kk * i) % n + n) % n);
                            double ar = A[2 * (((int64_t)k0 * n + i) * n + i2)];
                            double ai = A[2 * (((int64_t)k0 * n + i) * n + i2) + 1];
                            re += ar * cs[e] + ai * sn[e];
                            im += ai * cs[e] - ar * sn[e];
                        }
                        Bv[2 * (((int64_t)k0 * n + k1) * n + i2)] = re;
                        Bv[2 * (((int64_t)k0 * n + k1) * n + i2) + 1] = im;
                    }
            /* axis 2 */
#pragma omp parallel for schedule(static)
            for (int k0 = 0; k0 < n; k0++)
                for (int k1 = 0; k1 < n; k1++)
                    for (int k2 = 0; k2 < n; k2++) {
                        double re = 0.0, im = 0.0;
                        int kk = k2 - h;
                        for (int i = 0; i < n; i++) {
                            int e = (int)((((int64_t)kk * i) % n + n) % n);
                            double ar = Bv[2 * (((int64_t)k0 * n + k1) * n + i)];
                            double ai = Bv[2 * (((int64_t)k0 * n + k1) * n + i) + 1];
                            re += ar * cs[e] + ai * sn[e];
                            im += ai * cs[e] - ar * sn[e];
                        }
                        int64_t id = ((int64_t)k0 * n + k1) * n + k2;
                        coeffs[2 * ((int64_t)f * nc + id)] = re / ((double)n * n * n);
                        coeffs[2 * ((int64_t)f * nc + id) + 1] = im / ((double)n * n * n);
                    }
        }
        free(A); free(Bv); free(cs); free(sn);
    }
    free(pts);
    free(wts);
    return 0;
}

/* ------------------------------------------------------------------ */
/* synthesis                                                           */
/* ------------------------------------------------------------------ */

/* Euler ZYZ angles of a unit quaternion (inverse of euler_zyz_quaternion). */
static void quaternion_euler_zyz(const double* q, double* a, double* b, double* g)
{
    *b = 2.0 * atan2(sqrt(q[1] * q[1] + q[2] * q[2]), sqrt(q[0] * q[0] + q[3] * q[3]));
    double sp = atan2(q[3], q[0]);
    double dm = atan2(-q[1], q[2]);
    *a = sp + dm;
    *g = sp - dm;
}

/* out[f*P + i] = Re sum_k fhat_k phi_k(x_i) (direct summation). */
int orc_eval(const orc_params* p, const double* coeffs, int32_t F, const double* pts, int64_t P,
             double* out)
{
    int N = p->bandwidth;
    int64_t nc = orc_num_coeffs(p);
    if (nc < 0) return -1;
    if (p->domain == ORC_S2) {
#pragma omp parallel
        {
            double* A = malloc(sizeof(double) * (size_t)(N + 1) * (N + 2) / 2);
#pragma omp for schedule(dynamic, 16)
            for (int64_t i = 0; i < P; i++) {
                const double* x = pts + 3 * i;
                double z = x[2] > 1.0 ? 1.0 : (x[2] < -1.0 ? -1.0 : x[2]);
                double phi = atan2(x[1], x[0]);
                orc_alf(N, z, A);
                for (int f = 0; f < F; f++) {
                    double s = 0.0;
                    for (int n = 0; n <= N; n++)
                        for (int k = -n; k <= n; k++) {
                            int ak = abs(k);
                            double pv = A[(size_t)n * (n + 1) / 2 + ak];
                            if (k < 0 && (ak % 2)) pv = -pv;
                            const double* c = coeffs + 2 * ((int64_t)f * nc + n * n + n + k);
                            s += pv * (c[0] * cos(k * phi) - c[1] * sin(k * phi));
                        }
                    out[f * P + i] = s;
                }
            }
            free(A);
        }
    } else if (p->domain == ORC_SO3) {
#pragma omp parallel
        {
            double* dd = malloc(sizeof(double) * (size_t)nc);
#pragma omp for schedule(dynamic, 4)
            for (int64_t i = 0; i < P; i++) {
                double al, be, ga;
                quaternion_euler_zyz(pts + 4 * i, &al, &be, &ga);
                orc_wigner_d(N, be, dd);
                for (int f = 0; f < F; f++) {
                    double s = 0.0;
                    size_t base = 0;
                    for (int n = 0; n <= N; n++) {
                        double cn = sqrt((2.0 * n + 1.0) / (8.0 * ORC_PI * ORC_PI));
                        for (int k = -n; k <= n; k++)
                            for (int kp = -n; kp <= n; kp++) {
                                size_t id = base + (size_t)(k + n) * (2 * n + 1) + (kp + n);
                                double ph = -(k * al + kp * ga);
                                const double* c = coeffs + 2 * ((int64_t)f * nc + (int64_t)id);
                                s += cn * dd[id] * (c[0] * cos(ph) - c[1] * sin(ph));
                            }
                        base += (size_t)(2 * n + 1) * (2 * n + 1);
                    }
                    out[f * P + i] = s;
                }
            }
            free(dd);
        }
    } else {
        int32_t dm[3];
        orc_grid_dims(p, dm);
        int n = dm[0], h = n / 2;
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t i = 0; i < P; i++) {
            const double* x = pts + 3 * i;
            for (int f = 0; f < F; f++) {
                double s = 0.0;
                for (int a = 0; a < n; a++)
                    for (int b = 0; b < n; b++)
                        for (int c = 0; c < n; c++) {
                            double ph = 2.0 * ORC_PI * ((a - h) * x[0] + (b - h) * x[1] + (c - h) * x[2]);
                            const double* cf = coeffs + 2 * ((int64_t)f * nc + ((int64_t)a * n + b) * n + c);
                            s += cf[0] * cos(ph) - cf[1] * sin(ph);
                        }
                out[f * P + i] = s;
            }
        }
    }
    return 0;
}

int orc_num_monomials(int domain, int K) { return n_monomials(tangent_dim(domain), K); }

void orc_monomials(int domain, int K, int32_t* exps, int32_t* degs)
{
    int m = n_monomials(tangent_dim(domain), K);
    int e[3 * 128], d[128];
    monomial_exponents(tangent_dim(domain), K, e, d);
    for (int i = 0; i < m; i++) {
        exps[3 * i] = e[3 * i];
        exps[3 * i + 1] = e[3 * i + 1];
        exps[3 * i + 2] = e[3 * i + 2];
        degs[i] = d[i];
    }
}

/* Local problem of one centre, exposed for the pins: B (n x m, column-major,
 * normalised as in Sec. 2.3) and y_w (n x F) of the given neighbour list. */
int orc_local_system(const orc_params* p, const double* q, double delta, const int32_t* nb, int n,
                     const double* nodes, const double* nu, const double* vals, int32_t F,
                     int64_t ld, double* Bout, double* yw)
{
    int dom = p->domain;
    int D = tangent_dim(dom);
    int m = n_monomials(D, p->degree);
    int exps[3 * 128], degs[128];
    monomial_exponents(D, p->degree, exps, degs);
    int dimx = dom == ORC_SO3 ? 4 : 3;
    double scale = dom == ORC_SO3 ? 0.5 * delta : delta;
    double* w = malloc(sizeof(double) * (n > 0 ? n : 1));
    double W = 0.0;
    for (int i = 0; i < n; i++) {
        const double* x = nodes + (size_t)dimx * nb[i];
        double wi = wendland(p->wendland, key_distance(dom, prox_key(dom, x, q)) / delta);
        if (nu) wi *= nu[nb[i]];
        w[i] = wi;
        W += wi;
    }
    if (!(W > 0.0)) { free(w); return -1; }
    for (int i = 0; i < n; i++) w[i] /= W;
    double u[3];
    for (int a = 0; a < m; a++) {
        double s = 0.0;
        for (int i = 0; i < n; i++) {
            tangent_coords(dom, nodes + (size_t)dimx * nb[i], q, scale, u);
            double v = 1.0;
            for (int c = 0; c < D; c++) v *= ipow(u[c], exps[3 * a + c]);
            Bout[(size_t)a * n + i] = v;
            s += w[i] * v * v;
        }
        s = sqrt(s);
        for (int i = 0; i < n; i++) Bout[(size_t)a * n + i] = sqrt(w[i]) * Bout[(size_t)a * n + i] / s;
    }
    for (int f = 0; f < F; f++)
        for (int i = 0; i < n; i++) yw[(size_t)f * n + i] = sqrt(w[i]) * vals[f * ld + nb[i]];
    free(w);
    return 0;
}
