// host_geometry.h -- plan-time quadrature geometry of Sec. 2.1, host only,
// FP64: the Gauss-Legendre rule in cos(theta) (S2) and cos(beta) (SO3), and
// unit quaternions of Euler ZYZ angles (SO3 grid).
//
// The Gauss-Legendre rule is computed from the Jacobi matrix of the Legendre
// polynomials (symmetric tridiagonal, zero diagonal, off-diagonal
// b_k = k / sqrt(4k^2 - 1)), whose eigenvalues are the nodes:
//   1. each non-negative eigenvalue is isolated by bisection on the Sturm
//      count of the shifted matrix (the number of negative pivots of its LDL^T
//      factorization equals the number of eigenvalues below the shift);
//   2. one Newton correction on the orthonormal polynomial p_n, evaluated by
//      the recurrence b_{k+1} p_{k+1} = x p_k - b_k p_{k-1} of the same matrix;
//   3. the weight is the Christoffel number 1 / sum_{k<n} p_k(x)^2.
// Nodes are returned in descending order (rings by increasing polar angle);
// the rule is symmetric, so the negative half mirrors the positive one and the
// middle node of an odd rule is 0.
#pragma once

#include <math.h>

#include <vector>

namespace hamls {
namespace geom {

// Off-diagonal entry b_k (k >= 1) of the Legendre Jacobi matrix.
inline double jacobi_offdiag(int k) {
    const double kk = (double)k;
    return kk / sqrt((2.0 * kk - 1.0) * (2.0 * kk + 1.0));
}

// Number of eigenvalues of the n x n Legendre Jacobi matrix below lambda.
inline int sturm_count_below(int n, const double* b2, double lambda) {
    int neg = 0;
    double piv = -lambda;
    const double tiny = 1e-300;
    if (piv == 0.0) piv = -tiny;
    if (piv < 0.0) neg++;
    for (int i = 1; i < n; i++) {
        piv = -lambda - b2[i] / piv;
        if (piv == 0.0) piv = -tiny;
        if (piv < 0.0) neg++;
    }
    return neg;
}

// Orthonormal Legendre polynomial p_n(x) (w.r.t. dx on [-1, 1]) and its
// derivative, by the Jacobi-matrix recurrence; also sum_{k<n} p_k(x)^2.
inline void orthonormal_eval(int n, const double* b, double x, double* pn, double* dpn, double* csum) {
    double p_prev = 0.0, p = 1.0 / sqrt(2.0);
    double d_prev = 0.0, d = 0.0;
    double sum = 0.0;
    for (int k = 0; k < n; k++) {
        sum += p * p;
        const double bk = k > 0 ? b[k] : 0.0;
        const double p_next = (x * p - bk * p_prev) / b[k + 1];
        const double d_next = (p + x * d - bk * d_prev) / b[k + 1];
        p_prev = p;
        p = p_next;
        d_prev = d;
        d = d_next;
    }
    *pn = p;
    *dpn = d;
    *csum = sum;
}

// n-point Gauss-Legendre rule on [-1, 1]: x descending, w > 0.
inline void gauss_legendre_rule(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    if (n <= 0) return;
    std::vector<double> b(n + 1, 0.0), b2(n + 1, 0.0);
    for (int k = 1; k <= n; k++) {
        b[k] = jacobi_offdiag(k);
        b2[k] = b[k] * b[k];
    }
    const int half = (n + 1) / 2;
    for (int i = 0; i < half; i++) {
        double xi = 0.0;
        if (!(n % 2 == 1 && i == half - 1)) {
            // the (i+1)-th largest eigenvalue: n-1-i eigenvalues lie below it
            const int below = n - 1 - i;
            double lo = 0.0, hi = 1.0;
            for (int it = 0; it < 200; it++) {
                const double mid = 0.5 * (lo + hi);
                if (mid <= lo || mid >= hi) break;
                if (sturm_count_below(n, b2.data(), mid) > below)
                    hi = mid;
                else
                    lo = mid;
            }
            xi = 0.5 * (lo + hi);
            double pn, dpn, cs;
            orthonormal_eval(n, b.data(), xi, &pn, &dpn, &cs);
            if (dpn != 0.0) {
                const double step = pn / dpn;
                if (fabs(step) < hi - lo + 4e-16) xi -= step;
            }
        }
        double pn, dpn, cs;
        orthonormal_eval(n, b.data(), xi, &pn, &dpn, &cs);
        x[i] = xi;
        x[n - 1 - i] = -xi;
        w[i] = 1.0 / cs;
        w[n - 1 - i] = 1.0 / cs;
    }
}

// Hamilton product r = p q of quaternions (w, x, y, z).
inline void quat_mul(const double* p, const double* q, double* r) {
    const double w = p[0] * q[0] - p[1] * q[1] - p[2] * q[2] - p[3] * q[3];
    const double x = p[0] * q[1] + p[1] * q[0] + p[2] * q[3] - p[3] * q[2];
    const double y = p[0] * q[2] - p[1] * q[3] + p[2] * q[0] + p[3] * q[1];
    const double z = p[0] * q[3] + p[1] * q[2] - p[2] * q[1] + p[3] * q[0];
    r[0] = w;
    r[1] = x;
    r[2] = y;
    r[3] = z;
}

// Rotations about the z and y axes by angle a, as unit quaternions.
inline void quat_rot_z(double a, double* q) {
    q[0] = cos(0.5 * a);
    q[1] = 0.0;
    q[2] = 0.0;
    q[3] = sin(0.5 * a);
}
inline void quat_rot_y(double a, double* q) {
    q[0] = cos(0.5 * a);
    q[1] = 0.0;
    q[2] = sin(0.5 * a);
    q[3] = 0.0;
}

}  // namespace geom
}  // namespace hamls
