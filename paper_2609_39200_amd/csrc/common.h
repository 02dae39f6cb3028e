// common.h -- internal declarations of the HAMLS gfx950 library.
//
// Device memory layout of a plan (all FP64 unless noted):
//   grid      M_Q x 3 points (S2), plus per-ring theta and per-column phi
//   nodes     sorted by cell key, structure of arrays x[cap], y[cap], z[cap],
//             perm[cap] (int32, original index), optional weights nu[cap]
//   cells     band_off[nb+1] (int32), cell_start[ncells+1] (int32)
//   radii     delta[M_Q], threshold[M_Q], status[M_Q] (u8)
//   solve     Gram/right-hand-side entries, structure of arrays [entry][M_Q]
//   step 3    Legendre table [ring < ceil(nt/2)][n(n+1)/2 + k] (weights folded
//             in), ring DFT twiddles, ring spectra G[f][ring][k] (complex)
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "hamls.h"

namespace hamls {

constexpr double kPi = 3.141592653589793238462643383279502884;
constexpr int kWave = 64;
constexpr int kMaxFieldsPerPass = 16;  // fields handled by one assembly pass
constexpr int kRadixTile = 1024;       // keys per block of a radix sort pass
constexpr int kTileItems = 2048;       // grid nodes per block of the tiled order / row-pointer passes
constexpr int kOrderBuckets = 33;      // cost-order buckets (floor(log2(n_j + 1)) mapped to 1..32)
inline int tile_count(int64_t n) { return (int)((n + kTileItems - 1) / kTileItems); }
constexpr int kCandCap = 512;          // LDS candidate buffer of the S2 radius search
constexpr int kGridCandCap = 416;      // LDS candidate buffer of the SO3 / T3 radius search
constexpr int kListCap = 128;          // S2 member list of a grid node (radius -> assembly)
constexpr int kResolveBlocks = 131072; // most blocks of a list kernel (grid-stride)

// Blocks of a list kernel over at most MQ nodes: one per listed node up to
// kResolveBlocks, but no more than max(MQ / 4, 8192), so that a short or empty
// list does not pay for launching a block per grid node.
inline unsigned list_blocks(int64_t MQ) {
    int64_t b = MQ / 4 > 8192 ? MQ / 4 : 8192;
    b = b < MQ ? b : MQ;
    return (unsigned)(b < kResolveBlocks ? b : kResolveBlocks);
}

void set_error(const char* fmt, ...);
hamls_status hip_status(hipError_t e, const char* what);

#define HAMLS_HIP(call)                                        \
    do {                                                       \
        hipError_t e_ = (call);                                \
        if (e_ != hipSuccess) return hip_status(e_, #call);    \
    } while (0)

#define HAMLS_TRY(x)                       \
    do {                                   \
        hamls_status s_ = (x);             \
        if (s_ != HAMLS_OK) return s_;     \
    } while (0)

// Geometry of the S2 binning: nb equal-angle bands in theta, band b split into
// ns_b equal sectors in phi; cell key = band_off[b] + sector.
struct S2Bins {
    int nb = 0;
    double dtheta = 0.0;
    std::vector<int32_t> band_off;  // nb + 1
    int64_t ncells = 0;
    int key_bits = 0;
};

// Uniform cell grid of the SO3 and T3 domains: nc cells of width h per axis,
// axis cell i covering [lo + i h, lo + (i+1) h); D = 4 (SO3 quaternions) or
// 3 (T3, periodic).  Cell key = row-major index over the D axes.
struct GridBins {
    int D = 0;
    int nc = 0;
    double lo = 0.0, h = 0.0;
    int64_t ncells = 0;
    int key_bits = 0;
};

struct DeviceBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

struct Plan {
    hamls_params prm{};
    int device = 0;
    int dom = 0, N = 0, K = 0, m = 1, D = 2;
    int32_t dims[3] = {0, 0, 0};
    int64_t MQ = 0, ncoef = 0;
    int64_t M = 0;      // bound nodes
    int64_t nrec = 0;   // sorted records (SO3 stores q and -q: 2M)
    int64_t mcap = 0;   // node capacity of the plan
    int64_t cap = 0;    // record capacity
    bool has_nu = false;
    S2Bins bins;
    GridBins gbins;
    int64_t ncells = 0;
    int key_bits = 0;

    // host copies
    std::vector<double> h_grid, h_wts, h_theta, h_phi, h_glx, h_glw;

    // device allocations (owned)
    std::vector<DeviceBuf> owned;
    double* d_grid = nullptr;       // MQ x 3 (S2, T3) or MQ x 4 (SO3)
    double* d_theta = nullptr;      // per ring
    double* d_phi = nullptr;        // per column
    double* d_ring_cs = nullptr;    // per ring cos(theta), sin(theta)
    double* d_col_cs = nullptr;     // per column cos(phi), sin(phi)
    double* d_x = nullptr;          // sorted node coordinates, SoA dim x cap
    double* d_nu = nullptr;         // sorted node weights (cap) or null
    int32_t* d_perm = nullptr;      // cap
    uint32_t* d_key[2] = {nullptr, nullptr};
    int32_t* d_idx[2] = {nullptr, nullptr};
    uint32_t* d_hist = nullptr;
    int64_t hist_len = 0;
    int32_t* d_band_off = nullptr;
    // smoothed adaptive radius: the auxiliary Fibonacci points (xyz, theta,
    // phi, cos/sin theta) and their search outputs
    double* d_aux = nullptr;
    double* d_aux_theta = nullptr;
    double* d_aux_phi = nullptr;
    double* d_aux_cs = nullptr;
    double* d_aux_thr = nullptr;
    double* d_aux_delta = nullptr;
    uint8_t* d_aux_rst = nullptr;
    int32_t* d_cell_start = nullptr;
    double* d_delta = nullptr;      // MQ
    double* d_thr = nullptr;        // MQ
    uint8_t* d_status = nullptr;    // MQ (radius flags, then solve flags)
    uint8_t* d_rstatus = nullptr;   // MQ radius flags kept across solves
    int32_t* d_nj = nullptr;        // MQ
    int32_t* d_mlist = nullptr;     // S2 adaptive radius: MQ x kListCap member records
    int32_t* d_mcnt = nullptr;      // MQ: member count, or -1 (the assembly scans)
    uint8_t* d_route = nullptr;     // S2 adaptive radius: MQ, 1 where the search predicts an
                                    // ill-conditioned local system (solved in double-double only)
    bool route_valid = false;       // d_route holds the last search's predictions
    bool route_enabled = false;     // fits route (hamls_plan_tune or hamls_plan_routing)
    float route_ms[2] = {-1.0f, -1.0f};  // tuner's step-2 times without / with routing
    double* d_chi = nullptr;        // MQ
    double* d_tau = nullptr;        // MQ
    double* d_entries = nullptr;    // n_entries x MQ
    int32_t* d_rs_list = nullptr;   // MQ, centres re-solved in double-double
    int32_t* d_rs_count = nullptr;  // [0] re-solve list, [1] FP64 list of the mixed path
    int32_t* d_mx_list = nullptr;   // MQ, nodes the mixed path hands to FP64
    int32_t* d_rs_sorted = nullptr; // MQ, the re-solve list by decreasing member count
    int64_t n_entries_cap = 0;
    double* d_vals = nullptr;       // sorted values, kMaxFieldsPerPass x cap
    // generating functions (Rem. 2.5): per grid node the coefficients gamma
    // (m x MQ) of a*_i = w_i sum_a gamma_a g_a(x_i), and a*_i as CSR over the
    // grid (row_ptr MQ + 1, original node index and value per entry)
    double* d_gamma = nullptr;
    int64_t* d_grow = nullptr;
    int32_t* d_gcol = nullptr;
    double* d_gval = nullptr;
    // launch form of the one-field FP64 S2 assembly chosen by hamls_plan_tune:
    // 0 = grid order, 1 = dispatch in cost order, > 1 = work queue of that many
    // blocks over d_order (grid nodes by decreasing member count at tuning time)
    int asm_queue_blocks = 0;
    // mixed plans: step 2 runs the FP64 kernels when hamls_plan_tune measured
    // them faster than the FP32-Gram pass (step 3 stays FP32 on MFMA)
    bool mixed_fp64_step2 = false;
    int32_t* d_order = nullptr;
    // per-tile counts of the tiled cost order and row-pointer scan
    // (kOrderBuckets x tiles uint32, or tiles int64)
    uint32_t* d_tiles = nullptr;
    int64_t tiles_len = 0;
    int64_t gen_cap = 0;            // entries the CSR buffers hold
    int64_t gen_nnz = 0;
    bool gen_ready = false;         // built for the bound node set
    double* d_ptab = nullptr;       // Legendre table
    int64_t ptab_len = 0;
    double* d_tw = nullptr;         // 2 x n_phi twiddles
    double* d_G = nullptr;          // ring spectra, F x nt x (N+1) x 2
    int64_t G_fields = 0;
    // SO3 / T3 quadrature: per-axis twiddles, two complex work buffers, the
    // Wigner table [beta ring][coefficient] (weights and c_n folded in)
    double* d_tw_ax[3] = {nullptr, nullptr, nullptr};
    double* d_work[2] = {nullptr, nullptr};
    int64_t work_len = 0;           // doubles per work buffer
    double* d_wtab = nullptr;
    double* d_ring_w = nullptr;     // Gauss-Legendre weight per ring (S2 theta, SO3 beta)
    // S2 mixed precision: FP32 contraction table in MFMA blocks, block offsets,
    // work items (k, parity, row tile), folded FP32 spectra
    float* d_ptab32 = nullptr;
    int64_t* d_tab_off = nullptr;
    int32_t* d_leg_items = nullptr;
    int64_t leg_items = 0;
    float* d_x32 = nullptr;
    int64_t x32_len = 0;
    int64_t resident = 0;

    // per-phase timing
    bool timing = false;
    uint32_t timing_mask = ~0u;  // phases timed while timing is on (bit 1 << phase)
    struct Rec {
        int phase;
        hipEvent_t a, b;
    };
    std::vector<Rec> pending;
    std::vector<hipEvent_t> pool;
    double acc_ms[HAMLS_NUM_PHASES] = {};
    int64_t acc_n[HAMLS_NUM_PHASES] = {};
};

// Records a start/end event pair around one phase when timing is enabled.
// Records a start and an end event around a phase when the plan's timing is
// on for it; `allowed` = false records nothing (no event is created).
class PhaseTimer {
  public:
    PhaseTimer(Plan& P, int phase, hipStream_t s, bool allowed = true);
    ~PhaseTimer();

  private:
    Plan& P_;
    int phase_;
    hipStream_t s_;
    hipEvent_t b_ = nullptr;
};

// Arguments of the local solve kernels (one set per field pass).
struct SolveArgs {
    const double* entries;
    int64_t MQ;
    int F;
    int f0;
    const int32_t* nj;
    const uint8_t* rstatus;
    int reg;
    double tau_fixed, chi_t, chi_f;
    double mu[34];       // degree multipliers of the non-constant monomials
    double* out;         // F_total x MQ
    double* chi;
    double* tau;
    uint8_t* status;
    int write_diag;
    int32_t* rs_list;    // centres handed on (appended by the FP64 epilogue)
    int32_t* rs_count;
    const int32_t* in_list;   // centres a list-mode kernel works on
    const int32_t* in_count;
    const uint8_t* route;     // split solve: centres left to the re-solve (null: none)
};


SolveArgs make_solve_args(const Plan& P, int F, int f0, double* grid_values);
// one-field FP64 passes whose assembly hands its Gram matrices to a separate
// solve kernel, and that kernel
bool split_solve(const Plan& P, int F);
hamls_status launch_split_solve(const Plan& P, int F, int f0, double* grid_values, hipStream_t s,
                                bool route = false);

// generating functions (Rem. 2.5): gamma by a unit-right-hand-side solve,
// CSR row pointers from the neighbour counts, the values a*_i, and the sparse
// product with gathered values
hamls_status launch_gen_solve(const Plan& P, hipStream_t s);
hamls_status launch_gen_rowptr(const Plan& P, hipStream_t s);
hamls_status launch_s2_gen_values(const Plan& P, hipStream_t s);
hamls_status launch_gen_apply(const Plan& P, const double* values, int64_t ld, int F, int f0,
                              double* grid_values, hipStream_t s);

// Plan construction with a node capacity above the first bind, and the device
// bytes such a plan holds after a coefficient pass of F fields.
hamls_status plan_create(const hamls_params* p, const double* nodes, int64_t M, int64_t mcap,
                         const double* node_weights, void* stream, hamls_plan_t* out);
hamls_status plan_footprint(const hamls_params* p, int64_t M, int64_t mcap, int32_t F,
                            int64_t* bytes, int64_t* num_grid);

// --- kernels (kernels.hip) -------------------------------------------------
hamls_status launch_s2_keys(const Plan& P, const double* nodes, int64_t M, hipStream_t s);
hamls_status radix_sort(Plan& P, int64_t n, hipStream_t s, int* final_buf);
hamls_status launch_cell_start(const Plan& P, const uint32_t* keys, int64_t n, hipStream_t s);
hamls_status launch_gather_nodes(const Plan& P, const int32_t* idx, const double* nodes,
                                 const double* nu, int64_t M, hipStream_t s);
// route: also flag the centres whose nearest node lies beyond 0.7 d_n (d_route)
hamls_status launch_s2_radius(const Plan& P, hipStream_t s, bool route = false);
// queue_blocks: < 0 the plan's tuned launch form, 0 grid order, 1 cost-ordered
// dispatch, > 1 the work queue with that many blocks (one FP64 field)
// route: one field, a fit's pass: the centres the search predicts to be
// ill-conditioned go to the re-solve list unassembled (a tuning or
// generating-function pass assembles every centre)
hamls_status launch_s2_assemble(const Plan& P, int F, int f0, double* grid_values, hipStream_t s,
                                int queue_blocks = -1, bool route = false);
hamls_status launch_cost_order(const Plan& P, hipStream_t s);
hamls_status launch_s2_mixed(const Plan& P, int F, int f0, double* grid_values, hipStream_t s,
                             int form = -1);
hamls_status launch_s2_resolve(const Plan& P, int F, int f0, double* grid_values, hipStream_t s,
                               int unit_rhs = 0);
hamls_status launch_gather_values(const Plan& P, const double* values, int F, int f0, int64_t ld,
                                  hipStream_t s);
hamls_status launch_s2_count(const Plan& P, int32_t* counts, hipStream_t s);
hamls_status launch_s2_list(const Plan& P, const int64_t* row_ptr, int32_t* idx, hipStream_t s);
// Radices of a mixed-radix FFT of length n (product of rad[0..nst-1]);
// nst = 0: no factorization into primes up to 19 (direct sums are used).
constexpr int kFftMaxStages = 16;
struct FftPlan {
    int nst = 0;
    int rad[kFftMaxStages] = {};
};
FftPlan make_fft_plan(int n);
bool fft_axis_fits(int nin);
hamls_status launch_fft_axis(const double* in, bool real_in, double* out, int64_t A, int nin, int64_t B,
                             int nout, int koff, double sign, double scale, const double* tw, hipStream_t s);
bool s2_ring_fft_fits(int np);
hamls_status launch_s2_voronoi(const Plan& P, double* areas, hipStream_t s);
hamls_status launch_s2_ring_fft(const Plan& P, const double* gv, int F, double* G, hipStream_t s);

// Work memory of step 3 for F fields: element counts and pointers.
//   d0  S2: ring spectra G[f][ring][k] (complex); SO3 / T3: first axis pass
//   d1  SO3 / T3: second axis pass
//   f0  S2 mixed: folded FP32 spectra of the matrix-core contraction
struct CoeffWorkSize {
    int64_t d0 = 0, d1 = 0, f0 = 0;
};
struct CoeffWork {
    double* d0 = nullptr;
    int64_t d0_len = 0;  // doubles
    double* d1 = nullptr;
    float* f0 = nullptr;
    int64_t f0_len = 0;
};
CoeffWorkSize coeff_work_size(const Plan& P, int F);
// Step 3 (eq. (25)) of F fields with the given work memory.
// timed = false records no timing events (the no-allocation entry point).
hamls_status run_grid_to_coeffs(Plan* P, const double* grid_values, int F, double* coeffs,
                                const CoeffWork& W, hipStream_t s, bool timed = true);

hamls_status launch_s2_ring_dft(const Plan& P, const double* gv, int F, double* G, hipStream_t s);
hamls_status launch_s2_legendre(const Plan& P, int F, const double* G, double* coeffs, hipStream_t s);
// step 3 of the S2 mixed path: fold (FP64 spectra G -> FP32 blocks X), the
// matrix-core contraction (X -> block-ordered FP32 output in G's memory),
// unfold (-> coefficients)
hamls_status launch_s2_fold(const Plan& P, int F, const double* G, int64_t glen, float* X, int64_t xcap,
                            hipStream_t s);
hamls_status launch_s2_legendre_mfma(const Plan& P, int F, const float* X, float* out, hipStream_t s);
hamls_status launch_s2_unfold(const Plan& P, int F, const float* out, double* coeffs, hipStream_t s);
int64_t s2_mfma_out_len(int N, int F);
hamls_status build_s2_mfma_layout(Plan& P, std::vector<int64_t>& off, std::vector<int32_t>& items,
                                  int64_t* len);
hamls_status launch_s2_mfma_table(const Plan& P, int64_t len, hipStream_t s);
hamls_status launch_s2_legendre_table(const Plan& P, hipStream_t s);
hamls_status launch_s2_eval(const Plan& P, const double* coeffs, int F, const double* pts,
                            int64_t npts, double* out, hipStream_t s);

// --- kernels (grid.hip): SO3 and T3 ----------------------------------------
hamls_status launch_grid_keys(const Plan& P, const double* nodes, int64_t M, hipStream_t s);
hamls_status launch_grid_gather(const Plan& P, const int32_t* idx, const double* nodes,
                                const double* nu, int64_t M, hipStream_t s);
hamls_status launch_grid_radius(const Plan& P, hipStream_t s);
// form: < 0 the plan's tuned launch form, 0 grid order, 1 cost-ordered dispatch
// split_only: one field, the Gram matrices handed on (no solve) at any m
hamls_status launch_grid_mls(const Plan& P, int F, int f0, double* grid_values, hipStream_t s,
                             int form = -1, bool split_only = false);
hamls_status launch_grid_mixed(const Plan& P, int F, int f0, double* grid_values, hipStream_t s, int form = -1);
hamls_status launch_grid_resolve(const Plan& P, int F, int f0, double* grid_values, hipStream_t s,
                                 int unit_rhs = 0);
hamls_status launch_grid_gen_values(const Plan& P, hipStream_t s);
hamls_status launch_grid_list(const Plan& P, const int64_t* row_ptr, int32_t* counts, int32_t* idx,
                              hipStream_t s);

// --- kernels (transform.hip): SO3 and T3 quadrature and synthesis ----------
// out[a][k][b] = scale sum_i in[a][i][b] exp(sign 2 pi i (k - koff) i / nin),
// complex (re, im) pairs, in real when real_in.
hamls_status launch_dft_axis(const double* in, bool real_in, double* out, int64_t A, int nin,
                             int64_t B, int nout, int koff, double sign, double scale,
                             const double* tw, hipStream_t s);
hamls_status launch_wigner_table(const Plan& P, const double* beta, const double* wts, hipStream_t s);
hamls_status launch_so3_contract(const Plan& P, const double* G, int F, double* coeffs,
                                 hipStream_t s);
hamls_status launch_so3_eval(const Plan& P, const double* coeffs, int F, const double* pts,
                             int64_t npts, double* out, hipStream_t s);
hamls_status launch_t3_eval(const Plan& P, const double* coeffs, int F, const double* pts,
                            int64_t npts, double* out, hipStream_t s);

inline int n_monomials(int D, int K) {
    int m = 1;
    for (int i = 1; i <= D; i++) m = m * (K + i) / i;
    return m;
}

}  // namespace hamls
