// plan.hip -- the C ABI of include/hamls.h: parameter checks, the quadrature
// grid and transform tables (host, FP64), device memory of a plan and the
// order of kernel launches of every call.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>

#include "common.h"
#include "host_geometry.h"

namespace hamls {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

hamls_status hip_status(hipError_t e, const char* what) {
    set_error("%s: %s", what, hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? HAMLS_ERR_OUT_OF_MEMORY : HAMLS_ERR_DEVICE;
}

static hipEvent_t take_event(Plan& P) {
    if (!P.pool.empty()) {
        hipEvent_t e = P.pool.back();
        P.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

PhaseTimer::PhaseTimer(Plan& P, int phase, hipStream_t s, bool allowed) : P_(P), phase_(phase), s_(s) {
    if (!allowed || !P_.timing || !((P_.timing_mask >> phase) & 1u)) return;
    b_ = take_event(P_);
    if (b_) (void)hipEventRecord(b_, s_);
}

PhaseTimer::~PhaseTimer() {
    if (!b_) return;
    hipEvent_t e = take_event(P_);
    if (!e) return;
    (void)hipEventRecord(e, s_);
    P_.pending.push_back({phase_, b_, e});
}

static void drain_timing(Plan& P) {
    for (auto& r : P.pending) {
        float ms = 0.0f;
        if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            P.acc_ms[r.phase] += ms;
            P.acc_n[r.phase] += 1;
        }
        P.pool.push_back(r.a);
        P.pool.push_back(r.b);
    }
    P.pending.clear();
}

// ---------------------------------------------------------------------------
// host geometry (step 1 of Alg. 1, Sec. 2.1)
// ---------------------------------------------------------------------------

static hamls_status check_params(const hamls_params* p, int32_t dims[3]) {
    if (!p || p->struct_size != (int32_t)sizeof(hamls_params)) {
        set_error("params: struct_size mismatch (call hamls_params_init)");
        return HAMLS_ERR_INVALID_ARG;
    }
    const int dom = p->domain;
    if (dom != HAMLS_S2 && dom != HAMLS_SO3 && dom != HAMLS_T3) {
        set_error("unknown domain %d", dom);
        return HAMLS_ERR_INVALID_ARG;
    }
    if (p->precision != HAMLS_FP64 && p->precision != HAMLS_MIXED) {
        set_error("unknown precision %d", p->precision);
        return HAMLS_ERR_INVALID_ARG;
    }
    int N = p->bandwidth;
    const int Nmax = dom == HAMLS_S2 ? 1024 : (dom == HAMLS_SO3 ? 128 : 511);
    if (N < 0 || N > Nmax) {
        set_error("bandwidth %d outside [0, %d]", N, Nmax);
        return HAMLS_ERR_INVALID_ARG;
    }
    const int Kmax = dom == HAMLS_S2 ? 4 : 3;
    if (p->degree < 0 || p->degree > Kmax) {
        set_error("degree %d outside [0, %d]", p->degree, Kmax);
        return HAMLS_ERR_INVALID_ARG;
    }
    int m = n_monomials(dom == HAMLS_S2 ? 2 : 3, p->degree);
    if (p->smooth_aux < 0 || p->smooth_aux > (1 << 24)) {
        set_error("smooth_aux outside [0, 2^24]");
        return HAMLS_ERR_INVALID_ARG;
    }
    if (p->smooth_aux > 0 && (dom != HAMLS_S2 || p->knn_count <= 0 || p->support_radius > 0.0)) {
        set_error("the smoothed radius needs an S2 plan with knn_count > 0 and no fixed radius");
        return HAMLS_ERR_INVALID_ARG;
    }
    if (!(p->support_radius > 0.0) && p->knn_count <= 0) {
        set_error("need a fixed support radius or knn_count");
        return HAMLS_ERR_INVALID_ARG;
    }
    if (p->support_radius < 0.0 || !(p->support_radius == p->support_radius)) {
        set_error("support_radius must be >= 0");
        return HAMLS_ERR_INVALID_ARG;
    }
    if (dom == HAMLS_S2 && p->support_radius >= 0.5 * kPi) {
        set_error("S2 support radius must be < pi/2 (tangent projection)");
        return HAMLS_ERR_DOMAIN;
    }
    if (dom == HAMLS_SO3 && p->support_radius > kPi) {
        set_error("SO3 support radius (rotation angle) must be <= pi");
        return HAMLS_ERR_DOMAIN;
    }
    if (dom == HAMLS_T3 && p->support_radius >= 0.5) {
        set_error("T3 support radius must be < 1/2 (minimum-image chart)");
        return HAMLS_ERR_DOMAIN;
    }
    if (p->knn_count > 0 && (p->knn_count < m || !(p->knn_eps > 0.0))) {
        set_error("knn_count must be >= m = %d and knn_eps > 0", m);
        return HAMLS_ERR_INVALID_ARG;
    }
    const int knn_cap = dom == HAMLS_S2 ? kCandCap : kGridCandCap;
    if (p->knn_count > knn_cap) {
        set_error("knn_count %d above %d (the radius search's candidate buffer)", p->knn_count, knn_cap);
        return HAMLS_ERR_UNSUPPORTED;
    }
    if (p->wendland != 1 && p->wendland != 2) {
        set_error("wendland must be 1 or 2");
        return HAMLS_ERR_INVALID_ARG;
    }
    if (p->reg < HAMLS_REG_NONE || p->reg > HAMLS_REG_CHI_TARGET) {
        set_error("unknown regularization %d", p->reg);
        return HAMLS_ERR_INVALID_ARG;
    }
    if (p->reg == HAMLS_REG_FIXED && !(p->tau_fixed >= 0.0)) {
        set_error("tau_fixed must be >= 0");
        return HAMLS_ERR_INVALID_ARG;
    }
    if (p->reg == HAMLS_REG_CHI_TARGET && !(p->chi_target > 1.0 && p->chi_full > p->chi_target)) {
        set_error("need 1 < chi_target < chi_full");
        return HAMLS_ERR_INVALID_ARG;
    }
    if (dom == HAMLS_S2) {
        dims[0] = p->grid_shape[0] > 0 ? p->grid_shape[0] : N + 1;
        dims[1] = p->grid_shape[1] > 0 ? p->grid_shape[1] : 2 * N + 2;
        dims[2] = 1;
        if (dims[0] < N + 1 || dims[1] < 2 * N + 1) {
            set_error("grid %d x %d is not exact on Pi_2N for N = %d", dims[0], dims[1], N);
            return HAMLS_ERR_NOT_EXACT_GRID;
        }
        if (dims[0] > 8192 || dims[1] > 16384) {
            set_error("grid %d x %d too large", dims[0], dims[1]);
            return HAMLS_ERR_UNSUPPORTED;
        }
    } else if (dom == HAMLS_SO3) {
        dims[0] = p->grid_shape[0] > 0 ? p->grid_shape[0] : N + 1;
        dims[1] = p->grid_shape[1] > 0 ? p->grid_shape[1] : 2 * N + 1;
        dims[2] = p->grid_shape[2] > 0 ? p->grid_shape[2] : 2 * N + 1;
        if (dims[0] < N + 1 || dims[1] < 2 * N + 1 || dims[2] < 2 * N + 1) {
            set_error("grid %d x %d x %d is not exact for N = %d", dims[0], dims[1], dims[2], N);
            return HAMLS_ERR_NOT_EXACT_GRID;
        }
        if (dims[0] > 1024 || dims[1] > 1024 || dims[2] > 1024) {
            set_error("grid %d x %d x %d too large", dims[0], dims[1], dims[2]);
            return HAMLS_ERR_UNSUPPORTED;
        }
    } else {
        int n = p->grid_shape[0] > 0 ? p->grid_shape[0] : 2 * N + 1;
        dims[0] = dims[1] = dims[2] = n;
        if (n < 2 * N || n < 1) {
            set_error("grid %d^3 is not exact for N = %d (need n >= 2N)", n, N);
            return HAMLS_ERR_NOT_EXACT_GRID;
        }
        if (n > 1024) {
            set_error("grid %d^3 too large", n);
            return HAMLS_ERR_UNSUPPORTED;
        }
    }
    return HAMLS_OK;
}

template <class T>
static hamls_status dalloc(Plan& P, T** ptr, size_t count) {
    size_t bytes = sizeof(T) * (count > 0 ? count : 1);
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) return hip_status(e, "hipMalloc");
    P.owned.push_back({p, bytes});
    P.resident += (int64_t)bytes;
    *ptr = (T*)p;
    return HAMLS_OK;
}

static void free_plan(Plan* P) {
    if (!P) return;
    for (auto& r : P->pending) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto e : P->pool) (void)hipEventDestroy(e);
    for (auto& b : P->owned) (void)hipFree(b.p);
    delete P;
}

// S2 binning geometry sized so that a cell is about half the expected support
// radius: nb equal bands in theta, sectors per band proportional to sin(theta).
static void s2_bins(Plan& P, int64_t M) {
    double h = 0.0;
    if (P.prm.knn_count > 0) h = sqrt((double)P.prm.knn_count / (double)M);  // ~ r/2
    if (P.prm.support_radius > 0.0) {
        double hf = 0.5 * P.prm.support_radius;
        h = h > 0.0 ? std::min(h, hf) : hf;
    }
    h = std::max(h, kPi / 4096.0);
    h = std::min(h, kPi / 4.0);
    int nb = (int)ceil(kPi / h);
    nb = std::max(4, std::min(nb, 4096));
    S2Bins& B = P.bins;
    B.nb = nb;
    B.dtheta = kPi / nb;
    B.band_off.assign(nb + 1, 0);
    for (int b = 0; b < nb; b++) {
        double th = (b + 0.5) * B.dtheta;
        int ns = (int)lround(2.0 * kPi * sin(th) / B.dtheta);
        ns = std::max(1, ns);
        B.band_off[b + 1] = B.band_off[b] + ns;
    }
    B.ncells = B.band_off[nb];
    int bits = 1;
    while ((1ll << bits) < B.ncells) bits++;
    B.key_bits = bits;
    P.ncells = B.ncells;
    P.key_bits = bits;
}

// SO3 / T3 cell grid.  T3: cells of about half the expected radius (uniform
// density: n nodes in a ball of radius (3n/(4 pi M))^(1/3)), an integer number
// per unit period.  SO3: records live on the unit 3-sphere in R^4 (2M of them);
// cells of about the expected chordal radius 2 sin(r/4), r = (6 pi n/M)^(1/3)
// the rotation angle holding n of M Haar-uniform rotations.  At most 2^24 cells.
static void grid_bins(Plan& P, int64_t M) {
    GridBins& B = P.gbins;
    const double knn = (double)P.prm.knn_count;
    const double d0 = P.prm.support_radius;
    if (P.dom == HAMLS_T3) {
        double r = knn > 0 ? cbrt(3.0 * knn / (4.0 * kPi * (double)M)) : d0;
        if (d0 > 0.0 && knn > 0) r = std::min(r, d0);
        double h = 0.5 * r;
        int nc = (int)floor(1.0 / std::max(h, 1e-6));
        nc = std::max(1, std::min(nc, 256));
        B.D = 3;
        B.nc = nc;
        B.lo = 0.0;
        B.h = 1.0 / nc;
    } else {
        double r = knn > 0 ? cbrt(6.0 * kPi * knn / (double)M) : d0;
        if (d0 > 0.0 && knn > 0) r = std::min(r, d0);
        r = std::min(r, kPi);
        double rho = 2.0 * sin(0.25 * r);
        int nc = (int)ceil(2.0 / std::max(rho, 1e-6));
        nc = std::max(2, std::min(nc, 64));
        B.D = 4;
        B.nc = nc;
        B.lo = -1.0;
        B.h = 2.0 / nc;
    }
    int64_t nc = 1;
    for (int d = 0; d < B.D; d++) nc *= B.nc;
    B.ncells = nc;
    int bits = 1;
    while ((1ll << bits) < nc) bits++;
    B.key_bits = bits;
    P.ncells = nc;
    P.key_bits = bits;
}

// Routing of predicted ill-conditioned centres applies to S2 plans with the
// plain adaptive radius and degree >= 1 (the re-solve needs m > 1).
static bool route_possible(const Plan& P) {
    return P.dom == HAMLS_S2 && P.d_route && P.prm.knn_count > 0 && P.prm.smooth_aux == 0 && P.m > 1;
}

static hamls_status bind_nodes(Plan& P, const double* nodes, int64_t M, const double* nu,
                               hipStream_t s) {
    P.gen_ready = false;  // generating functions belong to the previous node set
    P.M = M;
    P.nrec = P.dom == HAMLS_SO3 ? 2 * M : M;
    P.has_nu = nu != nullptr;
    const bool s2 = P.dom == HAMLS_S2;
    {
        PhaseTimer pt(P, HAMLS_PHASE_BINNING, s);
        HAMLS_TRY(s2 ? launch_s2_keys(P, nodes, M, s) : launch_grid_keys(P, nodes, M, s));
        int fin = 0;
        HAMLS_TRY(radix_sort(P, P.nrec, s, &fin));
        HAMLS_TRY(launch_cell_start(P, P.d_key[fin], P.nrec, s));
        HAMLS_TRY(s2 ? launch_gather_nodes(P, P.d_idx[fin], nodes, nu, M, s)
                     : launch_grid_gather(P, P.d_idx[fin], nodes, nu, M, s));
    }
    PhaseTimer pt(P, HAMLS_PHASE_RADIUS, s);
    // the plain adaptive search of S2 predicts the ill-conditioned centres
    // when the plan routes them (degree 0 has no re-solve: nothing to route to)
    const bool flags = s2 && P.route_enabled && route_possible(P);
    HAMLS_TRY(s2 ? launch_s2_radius(P, s, flags) : launch_grid_radius(P, s));
    P.route_valid = flags;
    return HAMLS_OK;
}

// Node-side buffers of a plan (sorted records, keys, cells) and the per-centre
// state, shared by all domains.
static hamls_status alloc_common(Plan& P, int dimx) {
    HAMLS_TRY(dalloc(P, &P.d_grid, (size_t)dimx * P.MQ));
    HAMLS_TRY(dalloc(P, &P.d_x, (size_t)dimx * P.cap));
    HAMLS_TRY(dalloc(P, &P.d_nu, P.cap));
    HAMLS_TRY(dalloc(P, &P.d_perm, P.cap));
    HAMLS_TRY(dalloc(P, &P.d_key[0], P.cap));
    HAMLS_TRY(dalloc(P, &P.d_key[1], P.cap));
    HAMLS_TRY(dalloc(P, &P.d_idx[0], P.cap));
    HAMLS_TRY(dalloc(P, &P.d_idx[1], P.cap));
    P.hist_len = 256 * ((P.cap + kRadixTile - 1) / kRadixTile + 2);  // per-block digit counts + digit totals
    HAMLS_TRY(dalloc(P, &P.d_hist, P.hist_len));
    HAMLS_TRY(dalloc(P, &P.d_cell_start, P.ncells + 1));
    HAMLS_TRY(dalloc(P, &P.d_delta, P.MQ));
    HAMLS_TRY(dalloc(P, &P.d_thr, P.MQ));
    HAMLS_TRY(dalloc(P, &P.d_status, P.MQ));
    HAMLS_TRY(dalloc(P, &P.d_rstatus, P.MQ));
    HAMLS_TRY(dalloc(P, &P.d_nj, P.MQ));
    if (P.prm.knn_count > 0) {
        // member lists handed from the adaptive-radius search to the assembly
        HAMLS_TRY(dalloc(P, &P.d_mlist, (size_t)kListCap * P.MQ));
        HAMLS_TRY(dalloc(P, &P.d_mcnt, P.MQ));
        if (P.dom == HAMLS_S2) HAMLS_TRY(dalloc(P, &P.d_route, P.MQ));
    }
    HAMLS_TRY(dalloc(P, &P.d_chi, P.MQ));
    HAMLS_TRY(dalloc(P, &P.d_tau, P.MQ));
    int EG = P.m * (P.m + 1) / 2;
    P.n_entries_cap = EG + (int64_t)P.m * kMaxFieldsPerPass;
    HAMLS_TRY(dalloc(P, &P.d_entries, P.n_entries_cap * P.MQ));
    HAMLS_TRY(dalloc(P, &P.d_rs_list, P.MQ));
    HAMLS_TRY(dalloc(P, &P.d_rs_count, 64));
    HAMLS_TRY(dalloc(P, &P.d_mx_list, P.MQ));
    HAMLS_TRY(dalloc(P, &P.d_rs_sorted, P.MQ));
    P.tiles_len = (int64_t)kOrderBuckets * tile_count(P.MQ);
    HAMLS_TRY(dalloc(P, &P.d_tiles, (size_t)P.tiles_len));
    HAMLS_TRY(dalloc(P, &P.d_vals, (size_t)kMaxFieldsPerPass * P.cap));
    return HAMLS_OK;
}

static void twiddles(int n, std::vector<double>& tw) {
    tw.assign(2 * (size_t)n, 0.0);
    for (int e = 0; e < n; e++) {
        double a = 2.0 * kPi * e / n;
        tw[e] = cos(a);
        tw[n + e] = sin(a);
    }
}

// SO3 and T3 plans: the product grid of Sec. 2.1 (SO3: Gauss-Legendre in
// cos(beta) x trapezoid in alpha and gamma; T3: the equispaced periodic grid),
// the cell grid, and the quadrature tables (axis twiddles; SO3 Wigner table).
static hamls_status build_grid_plan(Plan& P, const double* nodes, int64_t M, int64_t mcap,
                                    const double* nu, hipStream_t s) {
    const bool so3 = P.dom == HAMLS_SO3;
    const int dimx = so3 ? 4 : 3;
    P.D = 3;
    P.m = n_monomials(3, P.K);
    P.MQ = (int64_t)P.dims[0] * P.dims[1] * P.dims[2];
    const int N = P.N;
    if (so3)
        P.ncoef = (int64_t)(N + 1) * (2 * N + 1) * (2 * N + 3) / 3;
    else
        P.ncoef = (int64_t)P.dims[0] * P.dims[0] * P.dims[0];
    P.mcap = mcap;
    P.cap = so3 ? 2 * mcap : mcap;
    P.h_grid.resize((size_t)dimx * P.MQ);
    P.h_wts.resize(P.MQ);
    std::vector<double> tw0, tw1;
    if (so3) {
        const int nb = P.dims[0], na = P.dims[1], ng = P.dims[2];
        geom::gauss_legendre_rule(nb, P.h_glx, P.h_glw);
        P.h_theta.resize(nb);
        // the rotation R_z(alpha) R_y(beta) R_z(gamma) as the quaternion
        // product q_z(alpha) q_y(beta) q_z(gamma)
        std::vector<double> qa(4 * (size_t)na), qg(4 * (size_t)ng);
        for (int a = 0; a < na; a++) geom::quat_rot_z(2.0 * kPi * a / na, &qa[4 * a]);
        for (int g = 0; g < ng; g++) geom::quat_rot_z(2.0 * kPi * g / ng, &qg[4 * g]);
        for (int t = 0; t < nb; t++) {
            const double beta = acos(P.h_glx[t]);
            P.h_theta[t] = beta;
            double qb[4], qab[4];
            geom::quat_rot_y(beta, qb);
            for (int a = 0; a < na; a++) {
                geom::quat_mul(&qa[4 * a], qb, qab);
                for (int g = 0; g < ng; g++) {
                    const int64_t j = ((int64_t)t * na + a) * ng + g;
                    geom::quat_mul(qab, &qg[4 * g], &P.h_grid[4 * j]);
                    P.h_wts[j] = P.h_glw[t] * (2.0 * kPi / na) * (2.0 * kPi / ng);
                }
            }
        }
        twiddles(na, tw0);
        twiddles(ng, tw1);
    } else {
        const int n = P.dims[0];
        const double w = 1.0 / ((double)n * n * n);
        for (int a = 0; a < n; a++)
            for (int b = 0; b < n; b++)
                for (int c = 0; c < n; c++) {
                    const int64_t j = ((int64_t)a * n + b) * n + c;
                    P.h_grid[3 * j + 0] = (double)a / n;
                    P.h_grid[3 * j + 1] = (double)b / n;
                    P.h_grid[3 * j + 2] = (double)c / n;
                    P.h_wts[j] = w;
                }
        twiddles(n, tw0);
    }
    grid_bins(P, M);
    HAMLS_TRY(alloc_common(P, dimx));
    HAMLS_TRY(dalloc(P, &P.d_tw_ax[0], tw0.size()));
    HAMLS_HIP(hipMemcpyAsync(P.d_tw_ax[0], tw0.data(), sizeof(double) * tw0.size(),
                             hipMemcpyHostToDevice, s));
    if (so3) {
        const int nb = P.dims[0];
        HAMLS_TRY(dalloc(P, &P.d_tw_ax[1], tw1.size()));
        HAMLS_TRY(dalloc(P, &P.d_theta, nb));
        HAMLS_TRY(dalloc(P, &P.d_ring_w, nb));
        HAMLS_TRY(dalloc(P, &P.d_wtab, (size_t)nb * P.ncoef));
        HAMLS_HIP(hipMemcpyAsync(P.d_tw_ax[1], tw1.data(), sizeof(double) * tw1.size(),
                                 hipMemcpyHostToDevice, s));
        HAMLS_HIP(hipMemcpyAsync(P.d_theta, P.h_theta.data(), sizeof(double) * nb,
                                 hipMemcpyHostToDevice, s));
        HAMLS_HIP(hipMemcpyAsync(P.d_ring_w, P.h_glw.data(), sizeof(double) * nb,
                                 hipMemcpyHostToDevice, s));
        HAMLS_TRY(launch_wigner_table(P, P.d_theta, P.d_ring_w, s));
    }
    HAMLS_HIP(hipMemcpyAsync(P.d_grid, P.h_grid.data(), sizeof(double) * dimx * P.MQ,
                             hipMemcpyHostToDevice, s));
    HAMLS_HIP(hipStreamSynchronize(s));
    return bind_nodes(P, nodes, M, nu, s);
}

static hamls_status build_plan(Plan& P, const hamls_params* p, const double* nodes, int64_t M,
                               int64_t mcap, const double* nu, hipStream_t s) {
    P.prm = *p;
    HAMLS_HIP(hipGetDevice(&P.device));
    P.dom = p->domain;
    P.N = p->bandwidth;
    P.K = p->degree;
    if (P.dom != HAMLS_S2) return build_grid_plan(P, nodes, M, mcap, nu, s);
    P.D = 2;
    P.m = n_monomials(2, P.K);
    int nt = P.dims[0], np = P.dims[1];
    P.MQ = (int64_t)nt * np;
    P.ncoef = (int64_t)(P.N + 1) * (P.N + 1);
    P.mcap = mcap;
    P.cap = mcap;

    // grid: GL in cos(theta) x trapezoid in phi
    geom::gauss_legendre_rule(nt, P.h_glx, P.h_glw);
    P.h_theta.resize(nt);
    P.h_phi.resize(np);
    P.h_grid.resize(3 * P.MQ);
    P.h_wts.resize(P.MQ);
    std::vector<double> cphi(np), sphi(np);
    for (int q = 0; q < np; q++) {
        P.h_phi[q] = 2.0 * kPi * q / np;
        cphi[q] = cos(P.h_phi[q]);
        sphi[q] = sin(P.h_phi[q]);
    }
    for (int t = 0; t < nt; t++) {
        double x = P.h_glx[t];
        double st = sqrt((1.0 - x) * (1.0 + x));
        P.h_theta[t] = acos(x);
        for (int q = 0; q < np; q++) {
            int64_t j = (int64_t)t * np + q;
            P.h_grid[3 * j + 0] = st * cphi[q];
            P.h_grid[3 * j + 1] = st * sphi[q];
            P.h_grid[3 * j + 2] = x;
            P.h_wts[j] = P.h_glw[t] * 2.0 * kPi / np;
        }
    }
    s2_bins(P, M);

    HAMLS_TRY(alloc_common(P, 3));
    HAMLS_TRY(dalloc(P, &P.d_theta, nt));
    HAMLS_TRY(dalloc(P, &P.d_phi, np));
    HAMLS_TRY(dalloc(P, &P.d_ring_cs, 2 * (size_t)nt));
    HAMLS_TRY(dalloc(P, &P.d_ring_w, nt));
    HAMLS_TRY(dalloc(P, &P.d_col_cs, 2 * (size_t)np));
    HAMLS_TRY(dalloc(P, &P.d_band_off, P.bins.nb + 1));
    std::vector<double> aux, aux_th, aux_ph, aux_cs;
    if (p->smooth_aux > 0) {
        // the auxiliary Fibonacci grid of the smoothed radius: z_k = 1 -
        // (2k+1)/n, longitude k times the golden angle pi (3 - sqrt 5)
        const int na = p->smooth_aux;
        const double ga = kPi * (3.0 - sqrt(5.0));
        aux.resize(3 * (size_t)na);
        aux_th.resize(na);
        aux_ph.resize(na);
        aux_cs.resize(2 * (size_t)na);
        for (int k = 0; k < na; k++) {
            const double z = 1.0 - (2.0 * k + 1.0) / na;
            const double r = sqrt((1.0 - z) * (1.0 + z));
            const double ph = ga * k;
            aux[3 * k] = r * cos(ph);
            aux[3 * k + 1] = r * sin(ph);
            aux[3 * k + 2] = z;
            aux_th[k] = acos(z);
            aux_ph[k] = fmod(ph, 2.0 * kPi);
            aux_cs[2 * k] = z;
            aux_cs[2 * k + 1] = r;
        }
        HAMLS_TRY(dalloc(P, &P.d_aux, aux.size()));
        HAMLS_TRY(dalloc(P, &P.d_aux_theta, aux_th.size()));
        HAMLS_TRY(dalloc(P, &P.d_aux_phi, aux_ph.size()));
        HAMLS_TRY(dalloc(P, &P.d_aux_cs, aux_cs.size()));
        HAMLS_TRY(dalloc(P, &P.d_aux_thr, na));
        HAMLS_TRY(dalloc(P, &P.d_aux_delta, na));
        HAMLS_TRY(dalloc(P, &P.d_aux_rst, na));
        HAMLS_HIP(hipMemcpyAsync(P.d_aux, aux.data(), sizeof(double) * aux.size(), hipMemcpyHostToDevice, s));
        HAMLS_HIP(hipMemcpyAsync(P.d_aux_theta, aux_th.data(), sizeof(double) * na, hipMemcpyHostToDevice, s));
        HAMLS_HIP(hipMemcpyAsync(P.d_aux_phi, aux_ph.data(), sizeof(double) * na, hipMemcpyHostToDevice, s));
        HAMLS_HIP(hipMemcpyAsync(P.d_aux_cs, aux_cs.data(), sizeof(double) * aux_cs.size(), hipMemcpyHostToDevice,
                                 s));
    }

    // step-3 tables: the Legendre table of the northern rings with the GL
    // weights folded in (generated on the device below), and the ring
    // twiddles
    int th = (nt + 1) / 2;
    int64_t na = (int64_t)(P.N + 1) * (P.N + 2) / 2;
    P.ptab_len = (int64_t)th * na;
    std::vector<double> tw(2 * (size_t)np);
    for (int q = 0; q < np; q++) {
        tw[q] = cphi[q];
        tw[np + q] = sphi[q];
    }
    HAMLS_TRY(dalloc(P, &P.d_ptab, P.ptab_len));
    HAMLS_TRY(dalloc(P, &P.d_tw, 2 * (size_t)np));

    HAMLS_HIP(hipMemcpyAsync(P.d_grid, P.h_grid.data(), sizeof(double) * 3 * P.MQ,
                             hipMemcpyHostToDevice, s));
    HAMLS_HIP(hipMemcpyAsync(P.d_theta, P.h_theta.data(), sizeof(double) * nt,
                             hipMemcpyHostToDevice, s));
    HAMLS_HIP(hipMemcpyAsync(P.d_phi, P.h_phi.data(), sizeof(double) * np, hipMemcpyHostToDevice, s));
    std::vector<double> rcs(2 * (size_t)nt), ccs(2 * (size_t)np);
    for (int t = 0; t < nt; t++) {
        rcs[2 * t] = P.h_glx[t];
        rcs[2 * t + 1] = sqrt((1.0 - P.h_glx[t]) * (1.0 + P.h_glx[t]));
    }
    for (int q = 0; q < np; q++) {
        ccs[2 * q] = cphi[q];
        ccs[2 * q + 1] = sphi[q];
    }
    HAMLS_HIP(hipMemcpyAsync(P.d_ring_cs, rcs.data(), sizeof(double) * 2 * nt, hipMemcpyHostToDevice, s));
    HAMLS_HIP(hipMemcpyAsync(P.d_ring_w, P.h_glw.data(), sizeof(double) * nt, hipMemcpyHostToDevice, s));
    HAMLS_HIP(hipMemcpyAsync(P.d_col_cs, ccs.data(), sizeof(double) * 2 * np, hipMemcpyHostToDevice, s));
    HAMLS_HIP(hipMemcpyAsync(P.d_band_off, P.bins.band_off.data(), sizeof(int32_t) * (P.bins.nb + 1),
                             hipMemcpyHostToDevice, s));
    HAMLS_HIP(hipMemcpyAsync(P.d_tw, tw.data(), sizeof(double) * 2 * np, hipMemcpyHostToDevice, s));
    HAMLS_TRY(launch_s2_legendre_table(P, s));
    std::vector<int64_t> toff;
    std::vector<int32_t> titems;
    if (P.prm.precision == HAMLS_MIXED) {
        int64_t len32 = 0;
        HAMLS_TRY(build_s2_mfma_layout(P, toff, titems, &len32));
        HAMLS_TRY(dalloc(P, &P.d_ptab32, len32));
        HAMLS_TRY(dalloc(P, &P.d_tab_off, toff.size()));
        HAMLS_TRY(dalloc(P, &P.d_leg_items, titems.size()));
        HAMLS_HIP(hipMemcpyAsync(P.d_tab_off, toff.data(), sizeof(int64_t) * toff.size(),
                                 hipMemcpyHostToDevice, s));
        HAMLS_HIP(hipMemcpyAsync(P.d_leg_items, titems.data(), sizeof(int32_t) * titems.size(),
                                 hipMemcpyHostToDevice, s));
        HAMLS_TRY(launch_s2_mfma_table(P, len32, s));
    }
    // the host vectors above are pageable: make the copies complete before
    // they go out of scope
    HAMLS_HIP(hipStreamSynchronize(s));
    return bind_nodes(P, nodes, M, nu, s);
}

// A plan whose node buffers hold up to mcap >= M nodes (later rebinds up to
// mcap allocate nothing); the binning geometry follows the first M.
hamls_status plan_create(const hamls_params* p, const double* nodes, int64_t M, int64_t mcap,
                         const double* node_weights, void* stream, hamls_plan_t* out) {
    if (!out || !nodes) {
        set_error("null argument");
        return HAMLS_ERR_INVALID_ARG;
    }
    *out = nullptr;
    int32_t dims[3];
    HAMLS_TRY(check_params(p, dims));
    // sorted records are indexed by int32 (SO3 stores two per node)
    const int64_t rec_max = (((int64_t)1 << 31) - 4096) / (p->domain == HAMLS_SO3 ? 2 : 1);
    if (M < 1 || mcap < M || mcap > rec_max || (p->knn_count > 0 && M < p->knn_count)) {
        set_error("node count %lld / capacity %lld invalid (need 1 <= M <= capacity <= %lld, "
                  "M >= knn_count)", (long long)M, (long long)mcap, (long long)rec_max);
        return HAMLS_ERR_INVALID_ARG;
    }
    Plan* P = new (std::nothrow) Plan();
    if (!P) {
        set_error("host allocation failed");
        return HAMLS_ERR_OUT_OF_MEMORY;
    }
    memcpy(P->dims, dims, sizeof(dims));
    hamls_status st = build_plan(*P, p, nodes, M, mcap, node_weights, (hipStream_t)stream);
    if (st != HAMLS_OK) {
        (void)hipStreamSynchronize((hipStream_t)stream);
        free_plan(P);
        return st;
    }
    *out = (hamls_plan_t)P;
    return HAMLS_OK;
}

// Device bytes a plan of capacity mcap allocates (first bind M) once
// hamls_grid_to_coeffs has run with F fields: the same sizes as the
// allocations of alloc_common, build_plan / build_grid_plan and the
// coefficient work buffers, each at least one element.
hamls_status plan_footprint(const hamls_params* p, int64_t M, int64_t mcap, int32_t F,
                            int64_t* bytes, int64_t* num_grid) {
    int32_t dims[3];
    HAMLS_TRY(check_params(p, dims));
    if (M < 1 || mcap < M || F < 1 || F > 4096) {
        set_error("need 1 <= M <= capacity and 1 <= F <= 4096");
        return HAMLS_ERR_INVALID_ARG;
    }
    Plan P;
    P.prm = *p;
    P.dom = p->domain;
    P.N = p->bandwidth;
    P.K = p->degree;
    memcpy(P.dims, dims, sizeof(dims));
    const bool s2 = P.dom == HAMLS_S2, so3 = P.dom == HAMLS_SO3;
    const int dimx = so3 ? 4 : 3;
    P.m = n_monomials(s2 ? 2 : 3, P.K);
    P.MQ = (int64_t)dims[0] * dims[1] * (s2 ? 1 : dims[2]);
    P.cap = so3 ? 2 * mcap : mcap;
    if (s2)
        s2_bins(P, M);
    else
        grid_bins(P, M);
    int64_t b = 0;
    auto add = [&b](int64_t count, int64_t elem) { b += elem * (count > 0 ? count : 1); };
    const int64_t MQ = P.MQ, cap = P.cap;
    add(dimx * MQ, 8);
    add(dimx * cap, 8);
    add(cap, 8);
    for (int k = 0; k < 5; k++) add(cap, 4);  // perm, two key and two index buffers
    add(256 * ((cap + kRadixTile - 1) / kRadixTile + 2), 4);
    add(P.ncells + 1, 4);
    add(MQ, 8);
    add(MQ, 8);
    add(MQ, 1);
    add(MQ, 1);
    add(MQ, 4);
    if (p->knn_count > 0) {
        add((int64_t)kListCap * MQ, 4);
        add(MQ, 4);
        if (s2) add(MQ, 1);  // route flags
    }
    add(MQ, 8);
    add(MQ, 8);
    add(((int64_t)P.m * (P.m + 1) / 2 + (int64_t)P.m * kMaxFieldsPerPass) * MQ, 8);
    add(MQ, 4);
    add(64, 4);
    add(MQ, 4);
    add(MQ, 4);
    add((int64_t)kOrderBuckets * tile_count(MQ), 4);
    add((int64_t)kMaxFieldsPerPass * cap, 8);
    const int N = P.N, K2 = 2 * N + 1;
    if (s2) {
        const int nt = dims[0], np = dims[1], th = (nt + 1) / 2;
        const int64_t na = (int64_t)(N + 1) * (N + 2) / 2;
        add(nt, 8);
        add(np, 8);
        add(2 * (int64_t)nt, 8);
        add(nt, 8);
        add(2 * (int64_t)np, 8);
        add(P.bins.nb + 1, 4);
        if (p->smooth_aux > 0) {
            const int64_t nx = p->smooth_aux;
            add(3 * nx, 8);
            add(nx, 8);
            add(nx, 8);
            add(2 * nx, 8);
            add(nx, 8);
            add(nx, 8);
            add(nx, 1);
        }
        add((int64_t)th * na, 8);
        add(2 * (int64_t)np, 8);
        add((int64_t)F * nt * (N + 1) * 2, 8);
        if (p->precision == HAMLS_MIXED) {
            const int th_pad = (th + 3) & ~3;
            int64_t total = 0, items = 0;
            for (int k = 0; k <= N; k++)
                for (int q = 0; q < 2; q++) {
                    const int R = N >= k + q ? (N - k - q) / 2 + 1 : 0;
                    const int R_pad = (R + 15) & ~15;
                    total += (int64_t)th_pad * R_pad;
                    items += (R + 63) / 64;
                }
            add(total, 4);
            add(2 * (int64_t)(N + 1), 8);
            add(4 * items, 4);
            const int64_t C_pad = ((2 * (int64_t)F + 15) / 16) * 16;
            add((int64_t)(N + 1) * 2 * th_pad * C_pad, 4);
        }
    } else if (so3) {
        const int nb = dims[0], na = dims[1], ng = dims[2];
        const int64_t ncoef = (int64_t)(N + 1) * (2 * N + 1) * (2 * N + 3) / 3;
        add(2 * (int64_t)na, 8);
        add(2 * (int64_t)ng, 8);
        add(nb, 8);
        add(nb, 8);
        add((int64_t)nb * ncoef, 8);
        add((int64_t)F * nb * K2 * ng * 2, 8);
        add((int64_t)F * nb * K2 * K2 * 2, 8);
    } else {
        add(2 * (int64_t)dims[0], 8);
        add((int64_t)F * MQ * 2, 8);
        add((int64_t)F * MQ * 2, 8);
    }
    *bytes = b;
    if (num_grid) *num_grid = MQ;
    return HAMLS_OK;
}

CoeffWorkSize coeff_work_size(const Plan& P, int F) {
    CoeffWorkSize z;
    const int N = P.N, K2 = 2 * N + 1;
    if (P.dom == HAMLS_S2) {
        z.d0 = (int64_t)F * P.dims[0] * (N + 1) * 2;
        if (P.prm.precision == HAMLS_MIXED) {
            const int th_pad = (((P.dims[0] + 1) / 2) + 3) & ~3;
            const int64_t C_pad = ((2 * (int64_t)F + 15) / 16) * 16;
            z.f0 = (int64_t)(N + 1) * 2 * th_pad * C_pad;
            // the ring spectra's memory later holds the contraction's FP32
            // block-ordered output
            z.d0 = std::max(z.d0, (s2_mfma_out_len(N, F) + 1) / 2);
        }
    } else if (P.dom == HAMLS_SO3) {
        z.d0 = (int64_t)F * P.dims[0] * K2 * P.dims[2] * 2;
        z.d1 = (int64_t)F * P.dims[0] * K2 * K2 * 2;
    } else {
        z.d0 = z.d1 = (int64_t)F * P.MQ * 2;
    }
    return z;
}

// Step-3 work memory for F fields, owned by the plan (grows with the largest
// call; the growth synchronizes the stream).
static hamls_status ensure_coeff_work(Plan* P, int32_t F, hipStream_t s) {
    if (F > P->G_fields) {
        const CoeffWorkSize z = coeff_work_size(*P, F);
        HAMLS_HIP(hipStreamSynchronize(s));
        for (void** slot : {(void**)&P->d_G, (void**)&P->d_work[0], (void**)&P->d_work[1], (void**)&P->d_x32}) {
            if (!*slot) continue;
            for (auto it = P->owned.begin(); it != P->owned.end(); ++it)
                if (it->p == *slot) {
                    (void)hipFree(it->p);
                    P->resident -= (int64_t)it->bytes;
                    P->owned.erase(it);
                    break;
                }
            *slot = nullptr;
        }
        P->x32_len = 0;
        P->G_fields = 0;
        if (P->dom == HAMLS_S2) {
            HAMLS_TRY(dalloc(*P, &P->d_G, z.d0));
            if (z.f0 > 0) {
                P->x32_len = z.f0;
                HAMLS_TRY(dalloc(*P, &P->d_x32, P->x32_len));
            }
        } else {
            HAMLS_TRY(dalloc(*P, &P->d_work[0], z.d0));
            HAMLS_TRY(dalloc(*P, &P->d_work[1], z.d1));
        }
        P->G_fields = F;
    }
    return HAMLS_OK;
}

static CoeffWork plan_coeff_work(const Plan& P) {
    CoeffWork W;
    if (P.dom == HAMLS_S2) {
        W.d0 = P.d_G;
        W.d0_len = P.G_fields > 0 ? coeff_work_size(P, P.G_fields).d0 : 0;
        W.f0 = P.d_x32;
        W.f0_len = P.x32_len;
    } else {
        W.d0 = P.d_work[0];
        W.d1 = P.d_work[1];
    }
    return W;
}

hamls_status run_grid_to_coeffs(Plan* P, const double* grid_values, int F, double* coeffs,
                                const CoeffWork& W, hipStream_t s, bool timed) {
    if (P->dom == HAMLS_S2) {
        {
            PhaseTimer pt(*P, HAMLS_PHASE_RING_DFT, s, timed);
            HAMLS_TRY(launch_s2_ring_dft(*P, grid_values, F, W.d0, s));
        }
        if (P->prm.precision == HAMLS_MIXED) {
            {
                PhaseTimer pt(*P, HAMLS_PHASE_FOLD, s, timed);
                HAMLS_TRY(launch_s2_fold(*P, F, W.d0, W.d0_len, W.f0, W.f0_len, s));
            }
            {
                PhaseTimer pt(*P, HAMLS_PHASE_CONTRACT, s, timed);
                HAMLS_TRY(launch_s2_legendre_mfma(*P, F, W.f0, (float*)W.d0, s));
            }
            PhaseTimer pt(*P, HAMLS_PHASE_FOLD, s, timed);
            return launch_s2_unfold(*P, F, (const float*)W.d0, coeffs, s);
        }
        PhaseTimer pt(*P, HAMLS_PHASE_CONTRACT, s, timed);
        return launch_s2_legendre(*P, F, W.d0, coeffs, s);
    }
    if (P->dom == HAMLS_SO3) {
        const int nb = P->dims[0], na = P->dims[1], ng = P->dims[2], N = P->N, K2 = 2 * N + 1;
        {
            PhaseTimer pt(*P, HAMLS_PHASE_RING_DFT, s, timed);
            // [f][t][a][g] -> [f][t][k][g] -> [f][t][k][k']
            HAMLS_TRY(launch_dft_axis(grid_values, true, W.d0, (int64_t)F * nb, na, ng, K2, N,
                                      1.0, 2.0 * kPi / na, P->d_tw_ax[0], s));
            HAMLS_TRY(launch_dft_axis(W.d0, false, W.d1, (int64_t)F * nb * K2, ng, 1, K2,
                                      N, 1.0, 2.0 * kPi / ng, P->d_tw_ax[1], s));
        }
        PhaseTimer pt(*P, HAMLS_PHASE_CONTRACT, s, timed);
        HAMLS_TRY(launch_so3_contract(*P, W.d1, F, coeffs, s));
        return HAMLS_OK;
    }
    const int n = P->dims[0], h = n / 2;
    const int64_t n2 = (int64_t)n * n;
    PhaseTimer pt(*P, HAMLS_PHASE_RING_DFT, s, timed);
    HAMLS_TRY(launch_dft_axis(grid_values, true, W.d0, F, n, n2, n, h, -1.0, 1.0,
                              P->d_tw_ax[0], s));
    HAMLS_TRY(launch_dft_axis(W.d0, false, W.d1, (int64_t)F * n, n, n, n, h, -1.0, 1.0,
                              P->d_tw_ax[0], s));
    HAMLS_TRY(launch_dft_axis(W.d1, false, coeffs, (int64_t)F * n2, n, 1, n, h, -1.0,
                              1.0 / ((double)n * n2), P->d_tw_ax[0], s));
    return HAMLS_OK;
}

}  // namespace hamls

using namespace hamls;

extern "C" {

hamls_status hamls_params_init(hamls_params* p) {
    if (!p) {
        set_error("null params");
        return HAMLS_ERR_INVALID_ARG;
    }
    memset(p, 0, sizeof(*p));
    p->struct_size = (int32_t)sizeof(hamls_params);
    p->domain = HAMLS_S2;
    p->bandwidth = 16;
    p->degree = 2;
    p->support_radius = 0.0;
    p->knn_count = 24;
    p->wendland = 1;
    p->knn_eps = 0.05;
    p->reg = HAMLS_REG_CHI_TARGET;
    p->precision = HAMLS_FP64;
    p->tau_fixed = 0.0;
    p->chi_target = 10.0;
    p->chi_full = 20.0;
    return HAMLS_OK;
}

hamls_status hamls_plan(const hamls_params* p, const double* nodes, int64_t M,
                        const double* node_weights, void* stream, hamls_plan_t* out) {
    return hamls::plan_create(p, nodes, M, M, node_weights, stream, out);
}

hamls_status hamls_plan_footprint(const hamls_params* p, int64_t M, int32_t F, int64_t* bytes) {
    if (!bytes) {
        set_error("null argument");
        return HAMLS_ERR_INVALID_ARG;
    }
    return hamls::plan_footprint(p, M, M, F, bytes, nullptr);
}

hamls_status hamls_plan_rebind(hamls_plan_t plan, const double* nodes, int64_t M,
                               const double* node_weights, void* stream) {
    Plan* P = (Plan*)plan;
    if (!P || !nodes) {
        set_error("null argument");
        return HAMLS_ERR_INVALID_ARG;
    }
    if (M < 1 || M > P->mcap || (P->prm.knn_count > 0 && M < P->prm.knn_count)) {
        set_error("node count %lld outside [max(1, knn_count), capacity %lld]", (long long)M,
                  (long long)P->mcap);
        return HAMLS_ERR_INVALID_ARG;
    }
    return bind_nodes(*P, nodes, M, node_weights, (hipStream_t)stream);
}

hamls_status hamls_mls_to_grid(hamls_plan_t plan, const double* values, int32_t F, int64_t ld,
                               double* grid_values, void* stream) {
    Plan* P = (Plan*)plan;
    if (!P || !values || !grid_values) {
        set_error("null argument");
        return HAMLS_ERR_INVALID_ARG;
    }
    if (F < 1 || F > 4096 || ld < P->M) {
        set_error("need 1 <= F <= 4096 and ld >= M");
        return HAMLS_ERR_INVALID_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    for (int f0 = 0; f0 < F; f0 += kMaxFieldsPerPass) {
        int Fc = std::min(kMaxFieldsPerPass, F - f0);
        {
            PhaseTimer pt(*P, HAMLS_PHASE_GATHER, s);
            HAMLS_TRY(launch_gather_values(*P, values, Fc, f0, ld, s));
        }
        // assembly (for one FP64 field the solve runs in its own kernel, in the
        // solve phase; otherwise fused with the assembly), then the double-double
        // re-solve of the flagged centres
        {
            PhaseTimer pt(*P, HAMLS_PHASE_ASSEMBLE, s);
            if (P->prm.precision == HAMLS_MIXED && !P->mixed_fp64_step2)
                HAMLS_TRY(P->dom == HAMLS_S2 ? launch_s2_mixed(*P, Fc, f0, grid_values, s)
                                             : launch_grid_mixed(*P, Fc, f0, grid_values, s));
            else
                HAMLS_TRY(P->dom == HAMLS_S2 ? launch_s2_assemble(*P, Fc, f0, grid_values, s, -1, true)
                                             : launch_grid_mls(*P, Fc, f0, grid_values, s));
        }
        {
            PhaseTimer pt(*P, HAMLS_PHASE_SOLVE, s);
            HAMLS_TRY(launch_split_solve(*P, Fc, f0, grid_values, s, true));
        }
        PhaseTimer pt(*P, HAMLS_PHASE_RESOLVE, s);
        HAMLS_TRY(P->dom == HAMLS_S2 ? launch_s2_resolve(*P, Fc, f0, grid_values, s)
                                     : launch_grid_resolve(*P, Fc, f0, grid_values, s));
    }
    return HAMLS_OK;
}

// One one-field FP64 assembly pass on the zero values of the tuning in a given
// launch form (S2: 0 grid order, 1 cost order, > 1 queue; SO3 / T3: 0 or 1).
// out: M_Q doubles for the passes that solve in place (SO3 / T3, m > 15).
static hamls_status tune_pass(Plan* P, hipStream_t s, int form, double* out) {
    const bool fp32 = P->prm.precision == HAMLS_MIXED && !P->mixed_fp64_step2;
    if (P->dom != HAMLS_S2)
        return fp32 ? launch_grid_mixed(*P, 1, 0, out, s, form) : launch_grid_mls(*P, 1, 0, out, s, form);
    return fp32 ? launch_s2_mixed(*P, 1, 0, out, s, form) : launch_s2_assemble(*P, 1, 0, out, s, form);
}

// Step 2 of one field on zero values without the re-solve (the assembly
// pass, plus the split solve where the pass hands one on): the cost compared
// when a mixed plan chooses between its FP32-Gram and FP64 kernels.
static hamls_status tune_step2(Plan* P, hipStream_t s, int form, double* out) {
    HAMLS_TRY(tune_pass(P, s, form, out));
    if (split_solve(*P, 1)) HAMLS_TRY(launch_split_solve(*P, 1, 0, out, s));
    return HAMLS_OK;
}

// The cost order: the member counts of the bound nodes (one grid-order
// assembly pass on zero values), then grid nodes by decreasing count.
// The per-tile count buffer of the tiled cost order and row-pointer scan.
static hamls_status ensure_tiles(Plan* P) {
    if (P->d_tiles) return HAMLS_OK;  // allocated with the plan
    P->tiles_len = (int64_t)kOrderBuckets * tile_count(P->MQ);
    return dalloc(*P, &P->d_tiles, (size_t)P->tiles_len);
}

static hamls_status queue_order(Plan* P, hipStream_t s, double* out) {
    if (!P->d_order) HAMLS_TRY(dalloc(*P, &P->d_order, P->MQ));
    HAMLS_TRY(ensure_tiles(P));
    HAMLS_HIP(hipMemsetAsync(P->d_vals, 0, sizeof(double) * (size_t)P->cap, s));
    HAMLS_HIP(hipMemsetAsync(P->d_rs_count, 0, sizeof(int32_t) * 10, s));
    HAMLS_TRY(tune_pass(P, s, 0, out));
    return launch_cost_order(*P, s);
}

// M_Q doubles of grid values for the tuning passes (freed by the caller)
static hamls_status tune_out(Plan* P, double** out) {
    *out = nullptr;
    HAMLS_HIP(hipMalloc(out, sizeof(double) * (size_t)P->MQ));
    return HAMLS_OK;
}

hamls_status hamls_plan_assembly_form(hamls_plan_t plan, void* stream, int32_t queue_blocks) {
    Plan* P = (Plan*)plan;
    if (!P || queue_blocks < 0 || (queue_blocks > 1 && queue_blocks < 8) || queue_blocks > (1 << 20)) {
        // the queue needs a block on each of the 8 XCD partitions
        set_error("null plan or form not 0, 1 or a block count in [8, 2^20]");
        return HAMLS_ERR_INVALID_ARG;
    }
    if (queue_blocks > 1 && (P->dom != HAMLS_S2 || P->prm.precision != HAMLS_FP64)) {
        set_error("the work-queue assembly exists for FP64 S2 plans only");
        return HAMLS_ERR_UNSUPPORTED;
    }
    if (queue_blocks > 0) {
        hipStream_t s = (hipStream_t)stream;
        double* out = nullptr;
        HAMLS_TRY(tune_out(P, &out));
        hamls_status st = queue_order(P, s, out);
        (void)hipStreamSynchronize(s);
        (void)hipFree(out);
        HAMLS_TRY(st);
    }
    P->asm_queue_blocks = queue_blocks;
    return HAMLS_OK;
}

hamls_status hamls_plan_cost_order(hamls_plan_t plan, int32_t* order) {
    Plan* P = (Plan*)plan;
    if (!P || !order || !P->d_order) {
        set_error("null plan or order, or no cost order computed");
        return HAMLS_ERR_INVALID_ARG;
    }
    HAMLS_HIP(hipDeviceSynchronize());
    HAMLS_HIP(hipMemcpy(order, P->d_order, sizeof(int32_t) * (size_t)P->MQ, hipMemcpyDeviceToHost));
    return HAMLS_OK;
}

// Routing of the centres the search predicts to be ill-conditioned (S2,
// adaptive radius, one FP64 field): step 2 of one field -- assembly in the
// plan's form, split solve, re-solve -- timed without and with it (best of
// three), the faster kept.  Whether it pays depends on how many predicted
// centres really need the re-solve (on the large S2 configuration nearly
// all; where holes are sparsely rimmed, few).
static hamls_status tune_routing(Plan* P, hipStream_t s) {
    P->route_ms[0] = P->route_ms[1] = -1.0f;
    if (!route_possible(*P) || !(P->prm.precision == HAMLS_FP64 || P->mixed_fp64_step2)) {
        P->route_enabled = false;
        return HAMLS_OK;
    }
    // the flags of the bound nodes (the search again; the radii are the same)
    HAMLS_TRY(launch_s2_radius(*P, s, true));
    P->route_valid = true;
    double* out = nullptr;
    HAMLS_TRY(tune_out(P, &out));
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    hamls_status st = HAMLS_OK;
    float t[2] = {1e30f, 1e30f};
    for (int v = 0; v < 2 && e == hipSuccess && st == HAMLS_OK; v++) {
        P->route_enabled = v == 1;
        for (int rep = 0; rep < 3 && e == hipSuccess && st == HAMLS_OK; rep++) {
            e = hipMemsetAsync(P->d_rs_count, 0, sizeof(int32_t) * 10, s);
            if (e == hipSuccess) e = hipEventRecord(a, s);
            if (e != hipSuccess) break;
            st = launch_s2_assemble(*P, 1, 0, out, s, P->asm_queue_blocks, true);
            if (st == HAMLS_OK) st = launch_split_solve(*P, 1, 0, out, s, true);
            if (st == HAMLS_OK) st = launch_s2_resolve(*P, 1, 0, out, s);
            float ms = 0.0f;
            if (st == HAMLS_OK) {
                e = hipEventRecord(b, s);
                if (e == hipSuccess) e = hipEventSynchronize(b);
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
            }
            if (e == hipSuccess && st == HAMLS_OK && ms < t[v]) t[v] = ms;
        }
    }
    (void)hipStreamSynchronize(s);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    (void)hipFree(out);
    P->route_enabled = false;
    if (st != HAMLS_OK) return st;
    if (e != hipSuccess) return hip_status(e, "tune");
    P->route_enabled = t[1] < t[0];
    P->route_ms[0] = t[0];
    P->route_ms[1] = t[1];
    return HAMLS_OK;
}

hamls_status hamls_plan_routing(hamls_plan_t plan, int32_t set, int32_t* enabled, float* times_ms) {
    Plan* P = (Plan*)plan;
    if (!P || set < -1 || set > 1) {
        set_error("null plan or set outside {-1, 0, 1}");
        return HAMLS_ERR_INVALID_ARG;
    }
    if (set >= 0) P->route_enabled = set == 1;
    if (enabled) *enabled = P->route_enabled ? 1 : 0;
    if (times_ms) {
        times_ms[0] = P->route_ms[0];
        times_ms[1] = P->route_ms[1];
    }
    return HAMLS_OK;
}

hamls_status hamls_plan_tune(hamls_plan_t plan, void* stream, int32_t* queue_blocks, float* times_ms) {
    Plan* P = (Plan*)plan;
    if (!P) {
        set_error("null plan");
        return HAMLS_ERR_INVALID_ARG;
    }
    if (times_ms)
        for (int k = 0; k < 4; k++) times_ms[k] = -1.0f;
    hipStream_t s = (hipStream_t)stream;
    int ncu = 0;
    HAMLS_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, P->device));
    double* out = nullptr;
    HAMLS_TRY(tune_out(P, &out));
    hamls_status st0 = queue_order(P, s, out);
    if (st0 != HAMLS_OK) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(out);
        return st0;
    }
    // candidates: grid order, dispatch in cost order, and (S2) the queue at 8
    // and 12 blocks per CU (the queue kernel holds 12 one-wave blocks per CU at
    // a time: three waves per SIMD; bounding it to four spills); best of three
    const int cand[4] = {0, 1, 8 * ncu, 12 * ncu};
    const int ncand = P->dom == HAMLS_S2 && P->prm.precision == HAMLS_FP64 ? 4 : 2;
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e != hipSuccess) {
        if (a) (void)hipEventDestroy(a);
        (void)hipFree(out);
        return hip_status(e, "hipEventCreate");
    }
    float best[4] = {-1.0f, -1.0f, -1.0f, -1.0f};
    hamls_status st = HAMLS_OK;
    for (int c = 0; c < ncand && st == HAMLS_OK; c++) {
        best[c] = 1e30f;
        for (int rep = 0; rep < 3 && st == HAMLS_OK; rep++) {
            // every pass starts with empty re-solve lists (the in-place passes
            // append to them) and zero queue counters
            e = hipMemsetAsync(P->d_rs_count, 0, sizeof(int32_t) * 10, s);
            if (e == hipSuccess) e = hipEventRecord(a, s);
            if (e != hipSuccess) {
                st = hip_status(e, "tune");
                break;
            }
            st = tune_pass(P, s, cand[c], out);
            float ms = 0.0f;
            if (st == HAMLS_OK) {
                e = hipEventRecord(b, s);
                if (e == hipSuccess) e = hipEventSynchronize(b);
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
                if (e != hipSuccess) st = hip_status(e, "tune");
            }
            if (st == HAMLS_OK && ms < best[c]) best[c] = ms;
        }
    }
    (void)hipStreamSynchronize(s);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    (void)hipFree(out);
    if (st != HAMLS_OK) return st;
    int pick = 0;
    for (int c = 1; c < ncand; c++)
        if (best[c] < best[pick]) pick = c;
    P->asm_queue_blocks = cand[pick];
    if (queue_blocks) *queue_blocks = cand[pick];
    if (P->prm.precision == HAMLS_MIXED) {
        // step 2 of a mixed plan: the FP32-Gram pass (with its FP64 list)
        // against the FP64 kernels, in the chosen form; the faster is kept
        hamls_status st2 = tune_out(P, &out);
        if (st2 != HAMLS_OK) return st2;
        e = hipEventCreate(&a);
        if (e == hipSuccess) e = hipEventCreate(&b);
        float t2[2] = {1e30f, 1e30f};
        for (int v = 0; v < 2 && e == hipSuccess && st2 == HAMLS_OK; v++) {
            P->mixed_fp64_step2 = v == 1;
            for (int rep = 0; rep < 3 && e == hipSuccess && st2 == HAMLS_OK; rep++) {
                e = hipMemsetAsync(P->d_rs_count, 0, sizeof(int32_t) * 10, s);
                if (e == hipSuccess) e = hipEventRecord(a, s);
                if (e != hipSuccess) break;
                st2 = tune_step2(P, s, P->asm_queue_blocks, out);
                float ms = 0.0f;
                if (st2 == HAMLS_OK) {
                    e = hipEventRecord(b, s);
                    if (e == hipSuccess) e = hipEventSynchronize(b);
                    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
                }
                if (e == hipSuccess && st2 == HAMLS_OK && ms < t2[v]) t2[v] = ms;
            }
        }
        (void)hipStreamSynchronize(s);
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
        (void)hipFree(out);
        P->mixed_fp64_step2 = false;
        if (st2 != HAMLS_OK) return st2;
        if (e != hipSuccess) return hip_status(e, "tune");
        P->mixed_fp64_step2 = t2[1] < t2[0];
        if (times_ms) {
            times_ms[2] = t2[0];
            times_ms[3] = t2[1];
        }
    }
    if (times_ms)
        for (int c = 0; c < ncand; c++) times_ms[c] = best[c];
    return tune_routing(P, s);
}

hamls_status hamls_gen_build(hamls_plan_t plan, void* stream) {
    Plan* P = (Plan*)plan;
    if (!P) {
        set_error("null plan");
        return HAMLS_ERR_INVALID_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    const bool s2 = P->dom == HAMLS_S2;
    if (!P->d_gamma) {
        HAMLS_TRY(dalloc(*P, &P->d_gamma, (size_t)P->m * P->MQ));
        HAMLS_TRY(dalloc(*P, &P->d_grow, P->MQ + 1));
    }
    HAMLS_TRY(ensure_tiles(P));
    P->gen_ready = false;
    // the assembly pass reads one field of sorted values and the double-double
    // re-solve up to 16 of them: zeros (their right-hand sides are replaced by
    // unit vectors); the re-solve list starts empty
    HAMLS_HIP(hipMemsetAsync(P->d_vals, 0, sizeof(double) * (size_t)kMaxFieldsPerPass * P->cap, s));
    HAMLS_HIP(hipMemsetAsync(P->d_rs_count, 0, sizeof(int32_t) * 10, s));
    if (s2)
        HAMLS_TRY(launch_s2_assemble(*P, 1, 0, nullptr, s));
    else
        HAMLS_TRY(launch_grid_mls(*P, 1, 0, nullptr, s, -1, true));
    HAMLS_TRY(launch_gen_solve(*P, s));
    for (int f0 = 0; f0 < P->m; f0 += kMaxFieldsPerPass) {
        const int Fc = std::min(kMaxFieldsPerPass, P->m - f0);
        HAMLS_TRY(s2 ? launch_s2_resolve(*P, Fc, f0, P->d_gamma, s, 1)
                     : launch_grid_resolve(*P, Fc, f0, P->d_gamma, s, 1));
    }
    HAMLS_TRY(launch_gen_rowptr(*P, s));
    int64_t nnz = 0;
    HAMLS_HIP(hipMemcpyAsync(&nnz, P->d_grow + P->MQ, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HAMLS_HIP(hipStreamSynchronize(s));
    if (nnz > P->gen_cap || !P->d_gval) {
        for (void* q : {(void*)P->d_gcol, (void*)P->d_gval}) {
            if (!q) continue;
            for (auto it = P->owned.begin(); it != P->owned.end(); ++it)
                if (it->p == q) {
                    (void)hipFree(it->p);
                    P->resident -= (int64_t)it->bytes;
                    P->owned.erase(it);
                    break;
                }
        }
        P->d_gcol = nullptr;
        P->d_gval = nullptr;
        P->gen_cap = 0;
        HAMLS_TRY(dalloc(*P, &P->d_gcol, nnz));
        HAMLS_TRY(dalloc(*P, &P->d_gval, nnz));
        P->gen_cap = nnz;
    }
    HAMLS_TRY(s2 ? launch_s2_gen_values(*P, s) : launch_grid_gen_values(*P, s));
    P->gen_nnz = nnz;
    P->gen_ready = true;
    return HAMLS_OK;
}

hamls_status hamls_gen_apply(hamls_plan_t plan, const double* values, int32_t F, int64_t ld,
                             double* grid_values, void* stream) {
    Plan* P = (Plan*)plan;
    if (!P || !values || !grid_values) {
        set_error("null argument");
        return HAMLS_ERR_INVALID_ARG;
    }
    if (!P->gen_ready) {
        set_error("no generating functions for the bound node set (call hamls_gen_build)");
        return HAMLS_ERR_INVALID_ARG;
    }
    if (F < 1 || F > 4096 || ld < P->M) {
        set_error("need 1 <= F <= 4096 and ld >= M");
        return HAMLS_ERR_INVALID_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    for (int f0 = 0; f0 < F; f0 += kMaxFieldsPerPass) {
        const int Fc = std::min(kMaxFieldsPerPass, F - f0);
        PhaseTimer pt(*P, HAMLS_PHASE_GEN_APPLY, s);
        HAMLS_TRY(launch_gen_apply(*P, values, ld, Fc, f0, grid_values, s));
    }
    return HAMLS_OK;
}

hamls_status hamls_gen_get(hamls_plan_t plan, int64_t* row_ptr, int32_t* idx, double* val) {
    Plan* P = (Plan*)plan;
    if (!P || !row_ptr) {
        set_error("null argument");
        return HAMLS_ERR_INVALID_ARG;
    }
    if (!P->gen_ready) {
        set_error("no generating functions for the bound node set (call hamls_gen_build)");
        return HAMLS_ERR_INVALID_ARG;
    }
    HAMLS_HIP(hipDeviceSynchronize());
    HAMLS_HIP(hipMemcpy(row_ptr, P->d_grow, sizeof(int64_t) * (P->MQ + 1), hipMemcpyDeviceToHost));
    if (!idx && !val) return HAMLS_OK;
    const int64_t nnz = P->gen_nnz;
    std::vector<int32_t> col(nnz);
    std::vector<double> v(nnz);
    HAMLS_HIP(hipMemcpy(col.data(), P->d_gcol, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost));
    HAMLS_HIP(hipMemcpy(v.data(), P->d_gval, sizeof(double) * nnz, hipMemcpyDeviceToHost));
    std::vector<std::pair<int32_t, double>> row;
    for (int64_t j = 0; j < P->MQ; j++) {
        row.clear();
        for (int64_t e = row_ptr[j]; e < row_ptr[j + 1]; e++) row.push_back({col[e], v[e]});
        std::sort(row.begin(), row.end());
        for (size_t k = 0; k < row.size(); k++) {
            if (idx) idx[row_ptr[j] + k] = row[k].first;
            if (val) val[row_ptr[j] + k] = row[k].second;
        }
    }
    return HAMLS_OK;
}

// Step-3 work memory for F fields (grows with the largest call; the growth
// synchronizes the stream and reallocates).
hamls_status hamls_grid_to_coeffs(hamls_plan_t plan, const double* grid_values, int32_t F,
                                  double* coeffs, void* stream) {
    Plan* P = (Plan*)plan;
    if (!P || !grid_values || !coeffs) {
        set_error("null argument");
        return HAMLS_ERR_INVALID_ARG;
    }
    if (F < 1 || F > 4096) {
        set_error("F outside [1, 4096]");
        return HAMLS_ERR_INVALID_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    HAMLS_TRY(ensure_coeff_work(P, F, s));
    return run_grid_to_coeffs(P, grid_values, F, coeffs, plan_coeff_work(*P), s);
}

// A captured fit: steps 2 and 3 on one plan with fixed buffers, replayed as
// one graph launch.  The launch choices the host made at capture time from
// the plan's binding (node count, whether node weights enter the kernels)
// are recorded: a replay after a rebind that changes them is refused.
struct hamls_graph_s {
    Plan* P;
    int64_t M;
    bool has_nu;
    hipGraph_t g;
    hipGraphExec_t x;
};

hamls_status hamls_fit_capture(hamls_plan_t plan, const double* values, int32_t F, int64_t ld,
                               double* grid_values, double* coeffs, void* stream, hamls_graph_t* out) {
    Plan* P = (Plan*)plan;
    if (!P || !values || !grid_values || !coeffs || !out) {
        set_error("null argument");
        return HAMLS_ERR_INVALID_ARG;
    }
    if (!stream) {
        set_error("capture needs a stream other than the default stream");
        return HAMLS_ERR_INVALID_ARG;
    }
    if (F < 1 || F > 4096 || ld < P->M) {
        set_error("need 1 <= F <= 4096 and ld >= M");
        return HAMLS_ERR_INVALID_ARG;
    }
    *out = nullptr;
    hipStream_t s = (hipStream_t)stream;
    // everything that allocates or synchronizes happens before the capture
    HAMLS_TRY(ensure_coeff_work(P, F, s));
    HAMLS_HIP(hipStreamSynchronize(s));
    const bool timing = P->timing;
    P->timing = false;
    HAMLS_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    hamls_status st = hamls_mls_to_grid(plan, values, F, ld, grid_values, stream);
    if (st == HAMLS_OK) st = hamls_grid_to_coeffs(plan, grid_values, F, coeffs, stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s, &g);
    P->timing = timing;
    if (st != HAMLS_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return st != HAMLS_OK ? st : hip_status(e, "hipStreamEndCapture");
    }
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_status(e, "hipGraphInstantiate");
    }
    hamls_graph_s* G = new (std::nothrow) hamls_graph_s{P, P->M, P->has_nu, g, x};
    if (!G) {
        (void)hipGraphExecDestroy(x);
        (void)hipGraphDestroy(g);
        set_error("host allocation failed");
        return HAMLS_ERR_OUT_OF_MEMORY;
    }
    *out = G;
    return HAMLS_OK;
}

hamls_status hamls_graph_launch(hamls_graph_t graph, void* stream) {
    if (!graph) {
        set_error("null graph");
        return HAMLS_ERR_INVALID_ARG;
    }
    if (graph->P->M != graph->M) {
        set_error("the plan was rebound to %lld nodes since the capture (%lld)", (long long)graph->P->M,
                  (long long)graph->M);
        return HAMLS_ERR_INVALID_ARG;
    }
    if (graph->P->has_nu != graph->has_nu) {
        set_error("the plan was rebound %s node weights since the capture (captured %s them)",
                  graph->P->has_nu ? "with" : "without", graph->has_nu ? "with" : "without");
        return HAMLS_ERR_INVALID_ARG;
    }
    HAMLS_HIP(hipGraphLaunch(graph->x, (hipStream_t)stream));
    return HAMLS_OK;
}

hamls_status hamls_graph_destroy(hamls_graph_t graph) {
    if (!graph) return HAMLS_OK;
    (void)hipGraphExecDestroy(graph->x);
    (void)hipGraphDestroy(graph->g);
    delete graph;
    return HAMLS_OK;
}

hamls_status hamls_plan_voronoi_areas(hamls_plan_t plan, double* areas, void* stream) {
    Plan* P = (Plan*)plan;
    if (!P || !areas) {
        set_error("null argument");
        return HAMLS_ERR_INVALID_ARG;
    }
    if (P->dom != HAMLS_S2) {
        set_error("Voronoi areas are built for S2 plans");
        return HAMLS_ERR_UNSUPPORTED;
    }
    return launch_s2_voronoi(*P, areas, (hipStream_t)stream);
}

hamls_status hamls_eval(hamls_plan_t plan, const double* coeffs, int32_t F, const double* points,
                        int64_t npts, double* out, void* stream) {
    Plan* P = (Plan*)plan;
    if (!P || !coeffs || !points || !out) {
        set_error("null argument");
        return HAMLS_ERR_INVALID_ARG;
    }
    if (F < 1 || npts < 0) {
        set_error("need F >= 1 and P >= 0");
        return HAMLS_ERR_INVALID_ARG;
    }
    if (npts == 0) return HAMLS_OK;
    if (npts > 0x7fffffff) {
        set_error("too many points");
        return HAMLS_ERR_INVALID_ARG;
    }
    if (P->dom == HAMLS_SO3) return launch_so3_eval(*P, coeffs, F, points, npts, out, (hipStream_t)stream);
    if (P->dom == HAMLS_T3) return launch_t3_eval(*P, coeffs, F, points, npts, out, (hipStream_t)stream);
    return launch_s2_eval(*P, coeffs, F, points, npts, out, (hipStream_t)stream);
}

hamls_status hamls_plan_destroy(hamls_plan_t plan) {
    Plan* P = (Plan*)plan;
    if (!P) return HAMLS_OK;
    (void)hipDeviceSynchronize();
    free_plan(P);
    return HAMLS_OK;
}

hamls_status hamls_plan_info_get(hamls_plan_t plan, hamls_plan_info* o) {
    Plan* P = (Plan*)plan;
    if (!P || !o) {
        set_error("null argument");
        return HAMLS_ERR_INVALID_ARG;
    }
    memset(o, 0, sizeof(*o));
    o->domain = P->dom;
    o->bandwidth = P->N;
    o->degree = P->K;
    o->m = P->m;
    memcpy(o->grid_dims, P->dims, sizeof(P->dims));
    o->precision = P->prm.precision;
    o->num_grid = P->MQ;
    o->num_coeffs = P->ncoef;
    o->num_nodes = P->M;
    o->node_capacity = P->mcap;
    o->resident_bytes = P->resident;
    o->num_cells = P->ncells;
    return HAMLS_OK;
}

hamls_status hamls_plan_grid(hamls_plan_t plan, double* points, double* weights) {
    Plan* P = (Plan*)plan;
    if (!P) {
        set_error("null plan");
        return HAMLS_ERR_INVALID_ARG;
    }
    if (points) memcpy(points, P->h_grid.data(), sizeof(double) * P->h_grid.size());
    if (weights) memcpy(weights, P->h_wts.data(), sizeof(double) * P->h_wts.size());
    return HAMLS_OK;
}

hamls_status hamls_plan_neighbors(hamls_plan_t plan, int64_t* row_ptr, int32_t* idx) {
    Plan* P = (Plan*)plan;
    if (!P || !row_ptr) {
        set_error("null argument");
        return HAMLS_ERR_INVALID_ARG;
    }
    hipStream_t s = nullptr;
    HAMLS_HIP(hipDeviceSynchronize());
    int32_t* d_cnt = nullptr;
    HAMLS_HIP(hipMalloc(&d_cnt, sizeof(int32_t) * P->MQ));
    hamls_status st = P->dom == HAMLS_S2 ? launch_s2_count(*P, d_cnt, s)
                                         : launch_grid_list(*P, nullptr, d_cnt, nullptr, s);
    std::vector<int32_t> cnt(P->MQ);
    if (st == HAMLS_OK) {
        hipError_t e = hipMemcpy(cnt.data(), d_cnt, sizeof(int32_t) * P->MQ, hipMemcpyDeviceToHost);
        if (e != hipSuccess) st = hip_status(e, "hipMemcpy");
    }
    (void)hipFree(d_cnt);
    if (st != HAMLS_OK) return st;
    row_ptr[0] = 0;
    for (int64_t j = 0; j < P->MQ; j++) row_ptr[j + 1] = row_ptr[j] + cnt[j];
    if (!idx) return HAMLS_OK;
    int64_t tot = row_ptr[P->MQ];
    int64_t* d_rp = nullptr;
    int32_t* d_idx = nullptr;
    HAMLS_HIP(hipMalloc(&d_rp, sizeof(int64_t) * (P->MQ + 1)));
    hipError_t e = hipMalloc(&d_idx, sizeof(int32_t) * (tot > 0 ? tot : 1));
    if (e != hipSuccess) {
        (void)hipFree(d_rp);
        return hip_status(e, "hipMalloc");
    }
    e = hipMemcpy(d_rp, row_ptr, sizeof(int64_t) * (P->MQ + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        st = P->dom == HAMLS_S2 ? launch_s2_list(*P, d_rp, d_idx, s)
                                : launch_grid_list(*P, d_rp, nullptr, d_idx, s);
        if (st == HAMLS_OK) e = hipMemcpy(idx, d_idx, sizeof(int32_t) * tot, hipMemcpyDeviceToHost);
    }
    (void)hipFree(d_rp);
    (void)hipFree(d_idx);
    if (e != hipSuccess) return hip_status(e, "neighbour export");
    if (st != HAMLS_OK) return st;
    for (int64_t j = 0; j < P->MQ; j++) std::sort(idx + row_ptr[j], idx + row_ptr[j + 1]);
    return HAMLS_OK;
}

hamls_status hamls_plan_radii(hamls_plan_t plan, double* delta, double* threshold) {
    Plan* P = (Plan*)plan;
    if (!P) {
        set_error("null plan");
        return HAMLS_ERR_INVALID_ARG;
    }
    HAMLS_HIP(hipDeviceSynchronize());
    if (delta) HAMLS_HIP(hipMemcpy(delta, P->d_delta, sizeof(double) * P->MQ, hipMemcpyDeviceToHost));
    if (threshold)
        HAMLS_HIP(hipMemcpy(threshold, P->d_thr, sizeof(double) * P->MQ, hipMemcpyDeviceToHost));
    return HAMLS_OK;
}

hamls_status hamls_diagnostics(hamls_plan_t plan, int32_t* n, double* chi, double* tau,
                               uint8_t* status) {
    Plan* P = (Plan*)plan;
    if (!P) {
        set_error("null plan");
        return HAMLS_ERR_INVALID_ARG;
    }
    HAMLS_HIP(hipDeviceSynchronize());
    if (n) HAMLS_HIP(hipMemcpy(n, P->d_nj, sizeof(int32_t) * P->MQ, hipMemcpyDeviceToHost));
    if (chi) HAMLS_HIP(hipMemcpy(chi, P->d_chi, sizeof(double) * P->MQ, hipMemcpyDeviceToHost));
    if (tau) HAMLS_HIP(hipMemcpy(tau, P->d_tau, sizeof(double) * P->MQ, hipMemcpyDeviceToHost));
    if (status)
        HAMLS_HIP(hipMemcpy(status, P->d_status, sizeof(uint8_t) * P->MQ, hipMemcpyDeviceToHost));
    return HAMLS_OK;
}

hamls_status hamls_timing_enable(hamls_plan_t plan, int32_t enable) {
    Plan* P = (Plan*)plan;
    if (!P) {
        set_error("null plan");
        return HAMLS_ERR_INVALID_ARG;
    }
    P->timing = enable != 0;
    return HAMLS_OK;
}

hamls_status hamls_timing_phases(hamls_plan_t plan, uint32_t mask) {
    Plan* P = (Plan*)plan;
    if (!P) {
        set_error("null plan");
        return HAMLS_ERR_INVALID_ARG;
    }
    P->timing_mask = mask;
    return HAMLS_OK;
}

hamls_status hamls_timing_read(hamls_plan_t plan, int32_t phase, int64_t* launches,
                               double* total_ms) {
    Plan* P = (Plan*)plan;
    if (!P || phase < 0 || phase >= HAMLS_NUM_PHASES) {
        set_error("bad plan or phase");
        return HAMLS_ERR_INVALID_ARG;
    }
    drain_timing(*P);
    if (launches) *launches = P->acc_n[phase];
    if (total_ms) *total_ms = P->acc_ms[phase];
    P->acc_n[phase] = 0;
    P->acc_ms[phase] = 0.0;
    return HAMLS_OK;
}

const char* hamls_status_string(hamls_status s) {
    switch (s) {
        case HAMLS_OK: return "ok";
        case HAMLS_ERR_INVALID_ARG: return "invalid argument";
        case HAMLS_ERR_UNSUPPORTED: return "unsupported";
        case HAMLS_ERR_OUT_OF_MEMORY: return "out of memory";
        case HAMLS_ERR_DEVICE: return "device error";
        case HAMLS_ERR_DOMAIN: return "domain error";
        case HAMLS_ERR_NOT_EXACT_GRID: return "grid not exact";
    }
    return "unknown status";
}

const char* hamls_last_error(void) { return g_err; }

}  // extern "C"
