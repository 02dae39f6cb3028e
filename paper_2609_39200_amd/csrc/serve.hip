// Serving loop: continuous batching of independent fits (steps 2 and 3 of
// Alg. 1 per request) over resident plans.
//
// Host-side runtime only; every step of a request runs in the library's own
// kernels through the plan entry points.  Worker threads each own one HIP
// stream, so the device work of the requests they hold overlaps; admission
// is by device footprint against a byte budget; plans (with their quadrature
// grids and Legendre / Wigner tables) stay resident between requests of
// equal parameters and are evicted least recently used first.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "common.h"


namespace hamls {
namespace {

double now_s() {
    static const auto t0 = std::chrono::steady_clock::now();
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// Parameters that make two plans interchangeable: every field of
// hamls_params (grid, tables, radius rule including the smoothed radius,
// weights, regularization, precision).  A field added to hamls_params must be
// added here; the static_assert below fails when the struct changes size.
bool same_params(const hamls_params& a, const hamls_params& b) {
    static_assert(sizeof(hamls_params) == 88, "hamls_params changed: update same_params");
    return a.domain == b.domain && a.bandwidth == b.bandwidth && a.degree == b.degree &&
           a.support_radius == b.support_radius && a.knn_count == b.knn_count &&
           a.wendland == b.wendland && a.knn_eps == b.knn_eps && a.reg == b.reg &&
           a.precision == b.precision && a.tau_fixed == b.tau_fixed &&
           a.chi_target == b.chi_target && a.chi_full == b.chi_full &&
           a.grid_shape[0] == b.grid_shape[0] && a.grid_shape[1] == b.grid_shape[1] &&
           a.grid_shape[2] == b.grid_shape[2] && a.smooth_aux == b.smooth_aux;
}

// Node capacity of a new plan: the next power of two, at least 16384.
int64_t capacity_for(int64_t M) {
    int64_t c = 16384;
    while (c < M) c *= 2;
    return c;
}

struct Resident {
    hamls_plan_t plan = nullptr;
    hamls_params prm{};
    int64_t mcap = 0;
    int64_t MQ = 0;
    double* grid_vals = nullptr;  // F_grid x MQ
    int32_t F_grid = 0;
    int64_t bytes = 0;            // committed: plan + grid values (or the admission estimate)
    bool busy = false;
    uint64_t last_use = 0;
};

struct Pending {
    hamls_request req;
    double t_submit;
    int bypassed = 0;  // times a later request was admitted ahead of this one at the head
};

// A blocked head of the queue may be passed by later requests that fit now
// (backfilling), at most this many times per head, so that it is not starved.
constexpr int kMaxBypass = 8;
// Later requests examined for backfilling.
constexpr int kBackfillScan = 32;

}  // namespace

struct Server {
    int device = 0;
    int64_t budget = 0;
    std::vector<std::thread> workers;
    std::vector<hipStream_t> streams;
    std::mutex mu;
    std::condition_variable cv_work;  // queue or resident set changed
    std::condition_variable cv_done;  // a completion arrived
    std::deque<Pending> queue;
    std::deque<hamls_completion> done;
    std::vector<Resident*> resident;
    int64_t committed = 0;
    int32_t running = 0;
    uint64_t use_clock = 0;
    uint64_t gen = 0;   // bumped whenever a request finishes
    uint64_t qgen = 0;  // bumped whenever a request arrives
    bool stop = false;

    void worker(int w);
    hamls_status run(Resident& e, const Pending& p, bool reuse, hipStream_t s);
    hamls_status place(const hamls_request& r, Resident** e, int64_t* need, int64_t* mcap);
    int64_t evictable(const Resident* keep) const;
};

namespace {

void free_resident(Resident* e) {
    if (!e) return;
    if (e->plan) (void)hamls_plan_destroy(e->plan);
    if (e->grid_vals) (void)hipFree(e->grid_vals);
    delete e;
}

}  // namespace

// One request on a worker's stream: (re)bind the plan, make room for F grid
// fields, step 2, step 3, wait for the stream.
hamls_status Server::run(Resident& e, const Pending& p, bool reuse, hipStream_t s) {
    const hamls_request& r = p.req;
    if (reuse) {
        HAMLS_TRY(hamls_plan_rebind(e.plan, r.nodes, r.M, r.node_weights, s));
    } else {
        HAMLS_TRY(plan_create(&r.params, r.nodes, r.M, e.mcap, r.node_weights, s, &e.plan));
        e.MQ = ((const Plan*)e.plan)->MQ;
    }
    if (r.F > e.F_grid) {
        if (e.grid_vals) {
            HAMLS_HIP(hipStreamSynchronize(s));
            HAMLS_HIP(hipFree(e.grid_vals));
            e.grid_vals = nullptr;
            e.F_grid = 0;
        }
        HAMLS_HIP(hipMalloc(&e.grid_vals, sizeof(double) * (size_t)r.F * e.MQ));
        e.F_grid = r.F;
    }
    HAMLS_TRY(hamls_mls_to_grid(e.plan, r.values, r.F, r.M, e.grid_vals, s));
    HAMLS_TRY(hamls_grid_to_coeffs(e.plan, e.grid_vals, r.F, r.coeffs, s));
    HAMLS_HIP(hipStreamSynchronize(s));
    return HAMLS_OK;
}

// Where request r would run: an idle resident plan of equal parameters and
// enough capacity, at most four times the capacity a new plan would get (its
// cell grid follows its first node set), the smallest such; else a new plan.
// Sets *e (null: new plan), the device bytes it adds (*need) and the new
// plan's capacity (*mcap); returns the request's own error for invalid
// parameters.
hamls_status Server::place(const hamls_request& r, Resident** e, int64_t* need, int64_t* mcap) {
    *e = nullptr;
    const int64_t cap_new = capacity_for(r.M);
    for (Resident* c : resident)
        if (!c->busy && c->plan && c->mcap >= r.M && c->mcap <= 4 * cap_new && same_params(c->prm, r.params) &&
            (!*e || c->mcap < (*e)->mcap))
            *e = c;
    if (*e) {
        *mcap = (*e)->mcap;
        *need = r.F > (*e)->F_grid ? 8 * (int64_t)(r.F - (*e)->F_grid) * (*e)->MQ : 0;
        return HAMLS_OK;
    }
    *mcap = cap_new;
    int64_t fp = 0, mq = 0;
    HAMLS_TRY(plan_footprint(&r.params, r.M, cap_new, r.F, &fp, &mq));
    *need = fp + 8 * (int64_t)r.F * mq;  // the plan and F x M_Q grid values
    return HAMLS_OK;
}

// Bytes held by idle resident plans other than `keep` (what eviction frees).
int64_t Server::evictable(const Resident* keep) const {
    int64_t b = 0;
    for (const Resident* c : resident)
        if (!c->busy && c != keep) b += c->bytes;
    return b;
}

void Server::worker(int w) {
    (void)hipSetDevice(device);
    hipStream_t s = streams[w];
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        cv_work.wait(lk, [&] { return stop || !queue.empty(); });
        if (queue.empty()) {
            if (stop) return;
            continue;
        }
        // the head of the queue, or (when it cannot fit until running requests
        // finish) the first later request that fits now, if the head has been
        // passed fewer than kMaxBypass times
        size_t pick = 0;
        Resident* e = nullptr;
        int64_t need = 0, mcap = 0;
        {
            hamls_status st = place(queue[0].req, &e, &need, &mcap);
            if (st != HAMLS_OK) {
                // invalid parameters: complete at once with the error
                const Pending& head = queue.front();
                hamls_completion c{head.req.tag, (int32_t)st, 0, head.t_submit, now_s(), now_s()};
                queue.pop_front();
                done.push_back(c);
                cv_done.notify_all();
                continue;
            }
        }
        bool fits = committed - evictable(e) + need <= budget;
        if (!fits && running > 0 && queue[0].bypassed < kMaxBypass) {
            const size_t lim = std::min(queue.size(), (size_t)kBackfillScan + 1);
            for (size_t i = 1; i < lim && !fits; i++) {
                Resident* e2 = nullptr;
                int64_t need2 = 0, mcap2 = 0;
                if (place(queue[i].req, &e2, &need2, &mcap2) != HAMLS_OK) continue;
                if (committed - evictable(e2) + need2 <= budget) {
                    pick = i;
                    e = e2;
                    need = need2;
                    mcap = mcap2;
                    fits = true;
                }
            }
            if (fits) queue[0].bypassed++;
        }
        const bool reuse = e != nullptr;
        if (!fits) {
            const Pending& head = queue.front();
            const uint64_t g0 = gen;
            if (running == 0) {
                // nothing left to finish: the head cannot fit even on an
                // emptied server
                hamls_completion c{head.req.tag, (int32_t)HAMLS_ERR_OUT_OF_MEMORY, 0, head.t_submit, now_s(),
                                   now_s()};
                queue.pop_front();
                done.push_back(c);
                cv_done.notify_all();
                continue;
            }
            // wait until a running request finishes (its plan becomes idle)
            // or a new request arrives (it may fit where the head does not)
            const uint64_t q0 = qgen;
            cv_work.wait(lk, [&] { return stop || gen != g0 || qgen != q0; });
            continue;
        }
        // evict idle plans, least recently used first, until the request fits
        std::vector<Resident*> evicted;
        while (committed + need > budget) {
            Resident* v = nullptr;
            for (Resident* c : resident)
                if (!c->busy && c != e && (!v || c->last_use < v->last_use)) v = c;
            if (!v) break;
            resident.erase(std::find(resident.begin(), resident.end(), v));
            committed -= v->bytes;
            evicted.push_back(v);
        }
        Pending p = queue[pick];
        queue.erase(queue.begin() + (std::ptrdiff_t)pick);
        if (!reuse) {
            e = new Resident();
            e->prm = p.req.params;
            e->mcap = mcap;
            resident.push_back(e);
        }
        e->busy = true;
        e->bytes += need;
        committed += need;
        running++;
        const double t_admit = now_s();
        lk.unlock();
        for (Resident* v : evicted) free_resident(v);
        hamls_status st = run(*e, p, reuse, s);
        int64_t actual = 0;
        if (st == HAMLS_OK) actual = ((const Plan*)e->plan)->resident + 8 * (int64_t)e->F_grid * e->MQ;
        const double t_done = now_s();
        lk.lock();
        running--;
        if (st == HAMLS_OK) {
            committed += actual - e->bytes;
            e->bytes = actual;
            e->busy = false;
            e->last_use = ++use_clock;
        } else {
            // a failed request leaves its plan in an unknown state: drop it
            resident.erase(std::find(resident.begin(), resident.end(), e));
            committed -= e->bytes;
            lk.unlock();
            (void)hipStreamSynchronize(s);
            free_resident(e);
            lk.lock();
        }
        done.push_back(hamls_completion{p.req.tag, (int32_t)st, reuse ? 1 : 0, p.t_submit, t_admit, t_done});
        gen++;
        cv_done.notify_all();
        cv_work.notify_all();
    }
}

}  // namespace hamls

using namespace hamls;

extern "C" {

double hamls_server_clock(void) { return now_s(); }

hamls_status hamls_server_create(int32_t slots, int64_t hbm_budget, hamls_server_t* out) {
    if (!out || slots < 1 || slots > 64) {
        set_error("need 1 <= slots <= 64 and an output pointer");
        return HAMLS_ERR_INVALID_ARG;
    }
    *out = nullptr;
    Server* S = new (std::nothrow) Server();
    if (!S) {
        set_error("host allocation failed");
        return HAMLS_ERR_OUT_OF_MEMORY;
    }
    hipError_t e = hipGetDevice(&S->device);
    if (e == hipSuccess && hbm_budget <= 0) {
        size_t fr = 0, tot = 0;
        e = hipMemGetInfo(&fr, &tot);
        hbm_budget = (int64_t)(0.8 * (double)fr);
    }
    if (e != hipSuccess) {
        delete S;
        return hip_status(e, "server device query");
    }
    S->budget = hbm_budget;
    for (int w = 0; w < slots; w++) {
        hipStream_t s = nullptr;
        e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e != hipSuccess) {
            for (hipStream_t t : S->streams) (void)hipStreamDestroy(t);
            delete S;
            return hip_status(e, "hipStreamCreateWithFlags");
        }
        S->streams.push_back(s);
    }
    for (int w = 0; w < slots; w++) S->workers.emplace_back(&Server::worker, S, w);
    *out = (hamls_server_t)S;
    return HAMLS_OK;
}

hamls_status hamls_server_submit(hamls_server_t server, const hamls_request* r) {
    Server* S = (Server*)server;
    if (!S || !r) {
        set_error("null argument");
        return HAMLS_ERR_INVALID_ARG;
    }
    if (r->struct_size != (int32_t)sizeof(hamls_request) || !r->nodes || !r->values || !r->coeffs ||
        r->F < 1 || r->F > 4096 || r->M < 1) {
        set_error("malformed request (struct_size, null pointers, F in [1, 4096], M >= 1)");
        return HAMLS_ERR_INVALID_ARG;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) {
        set_error("server is shutting down");
        return HAMLS_ERR_INVALID_ARG;
    }
    S->queue.push_back(Pending{*r, now_s()});
    S->qgen++;
    S->cv_work.notify_all();
    return HAMLS_OK;
}

hamls_status hamls_server_wait(hamls_server_t server, hamls_completion* out, int32_t max,
                               int32_t* count, double timeout_s) {
    Server* S = (Server*)server;
    if (!S || !out || !count || max < 1) {
        set_error("null argument or max < 1");
        return HAMLS_ERR_INVALID_ARG;
    }
    std::unique_lock<std::mutex> lk(S->mu);
    if (S->done.empty() && timeout_s > 0.0)
        S->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), [&] { return !S->done.empty(); });
    int32_t n = 0;
    while (n < max && !S->done.empty()) {
        out[n++] = S->done.front();
        S->done.pop_front();
    }
    *count = n;
    return HAMLS_OK;
}

hamls_status hamls_server_load(hamls_server_t server, int32_t* in_flight, int64_t* committed_bytes,
                               int32_t* resident_plans) {
    Server* S = (Server*)server;
    if (!S) {
        set_error("null server");
        return HAMLS_ERR_INVALID_ARG;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    if (in_flight) *in_flight = (int32_t)S->queue.size() + S->running;
    if (committed_bytes) *committed_bytes = S->committed;
    if (resident_plans) *resident_plans = (int32_t)S->resident.size();
    return HAMLS_OK;
}

hamls_status hamls_server_destroy(hamls_server_t server) {
    Server* S = (Server*)server;
    if (!S) return HAMLS_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    for (auto& t : S->workers) t.join();
    for (Resident* e : S->resident) free_resident(e);
    for (hipStream_t s : S->streams) (void)hipStreamDestroy(s);
    delete S;
    return HAMLS_OK;
}

}  // extern "C"
