// Serving with continuous batching (the frequency solves of many requests;
// LU reuse across right-hand sides, Appendix A): requests are queued as they
// are submitted and taken by worker slots, each a host thread with its own
// context, workspace and HIP stream (default priority, non-blocking).  A slot
// takes every waiting request, in arrival order, while their matrices fit its
// share of the HBM budget, plans all their systems at once, factors them in
// shared launches and solves each request on the resident factors for its
// right-hand sides; a request is complete as soon as its own solves are.
// While one slot plans, factors or solves, the others take the requests that
// arrived meanwhile, so rounds overlap on the device.  Submission refuses a
// request (FHW_E_BUSY) while the waiting requests already hold more matrix
// bytes than the queue limit.  Each slot keeps the factors of its last round
// resident: a round whose requests' systems (curve, frequency, N) are all
// among them, each request's in order, is solved on them with no new plan or
// factorization (a one-round factor cache per slot; the precision is the
// server's).  Host logic only: the arithmetic is the
// library's kernels, through the same calls as a single caller would make.
#include <math.h>
#include <string.h>

#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "fhw_internal.h"

namespace {

struct srv_request {
    int64_t ticket = 0;
    int32_t curve = 0, N = 0;
    std::vector<double> omegas;
    std::vector<fhw_incidence> inc;
    void* psi = nullptr;
    double* resid = nullptr;
    int32_t* sweeps = nullptr;
    size_t bytes = 0;                 // device bytes of its systems in the workspace
    int status = 1;                   // 1 pending, 0 done, < 0 error code
    std::string err;
};

}  // namespace

struct fhw_server {
    int device = 0;
    fhw_problem prob{};
    std::vector<std::vector<double>> coef;   // per curve: cx, sx, cy, sy (degree + 1 each)
    std::vector<fhw_curve> curves;
    size_t slot_budget = 0, queue_limit = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<srv_request*> queue;
    size_t queued_bytes = 0;
    std::unordered_map<int64_t, std::unique_ptr<srv_request>> reqs;
    int64_t next_ticket = 1;
    bool stop = false;
    std::vector<std::thread> workers;
    std::vector<hipStream_t> streams;
    std::vector<fhw_ctx*> ctxs;
    // statistics
    int64_t rounds = 0, done = 0, refused = 0, systems = 0, cache_hits = 0;
    double busy_s = 0.0;

    ~fhw_server() {
        for (fhw_ctx* c : ctxs) fhw_destroy(c);
        for (hipStream_t s : streams) (void)hipStreamDestroy(s);
    }
};

namespace {

size_t request_bytes(const fhw_problem& p, int N, size_t n_freq) {
    const size_t NN = (size_t)N * N;
    size_t b = NN * 16 + (size_t)((N + FHW_LU_NB - 1) / FHW_LU_NB) * FHW_LU_NB * FHW_LU_NB * 16;
    if (p.precision == FHW_FP32_REFINE) b += NN * 8;
    b += (size_t)N * (4 + 16 * 2 * FHW_INC_GROUP) + 256;
    return b * n_freq;
}

// key of a system in a slot's resident factors: (curve, frequency bits, N)
struct sys_key {
    int32_t curve;
    uint64_t omega;
    int32_t N;
    bool operator<(const sys_key& o) const {
        if (curve != o.curve) return curve < o.curve;
        if (omega != o.omega) return omega < o.omega;
        return N < o.N;
    }
};
sys_key key_of(int32_t curve, double omega, int32_t N) {
    sys_key k{curve, 0, N};
    memcpy(&k.omega, &omega, sizeof(double));
    return k;
}

void worker(fhw_server* S, fhw_ctx* ctx) {
    (void)hipSetDevice(S->device);
    std::vector<srv_request*> batch;
    std::vector<fhw_system> sys;
    std::vector<int32_t> first;
    // the factor cache of this slot: the systems of its last round, whose
    // factors stay resident until the next round needs a new plan
    std::map<sys_key, int32_t> resident;
    for (;;) {
        batch.clear();
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_work.wait(lk, [&] { return S->stop || !S->queue.empty(); });
            if (S->queue.empty()) break;   // stop requested and nothing left
            size_t bytes = 0;
            while (!S->queue.empty()) {
                srv_request* r = S->queue.front();
                if (!batch.empty() && bytes + r->bytes > S->slot_budget) break;
                S->queue.pop_front();
                S->queued_bytes -= r->bytes;
                batch.push_back(r);
                bytes += r->bytes;
            }
        }
        const auto t0 = std::chrono::steady_clock::now();
        // every request's systems already resident, in order: no plan, no factorization
        first.assign(batch.size(), -1);
        bool hit = !resident.empty();
        for (size_t b = 0; hit && b < batch.size(); ++b) {
            const srv_request* r = batch[b];
            auto it = resident.find(key_of(r->curve, r->omegas[0], r->N));
            if (it == resident.end()) { hit = false; break; }
            first[b] = it->second;
            for (size_t j = 1; j < r->omegas.size(); ++j) {
                auto jt = resident.find(key_of(r->curve, r->omegas[j], r->N));
                if (jt == resident.end() || jt->second != first[b] + (int32_t)j) { hit = false; break; }
            }
        }
        int rc = FHW_OK;
        int64_t n_sys = 0;
        if (!hit) {
            sys.clear();
            for (srv_request* r : batch)
                for (double om : r->omegas) sys.push_back(fhw_system{r->curve, om, r->N});
            resident.clear();
            rc = fhw_plan_systems(ctx, S->curves.data(), (int32_t)S->curves.size(), sys.data(), (int32_t)sys.size(),
                                  &S->prob, nullptr);
            if (rc == FHW_OK) rc = fhw_factor(ctx);
            int32_t s0 = 0;
            for (size_t b = 0; b < batch.size(); ++b) {
                first[b] = s0;
                s0 += (int32_t)batch[b]->omegas.size();
            }
            if (rc == FHW_OK)
                for (int32_t q = 0; q < (int32_t)sys.size(); ++q)
                    resident.emplace(key_of(sys[q].curve, sys[q].omega, sys[q].N), q);
            n_sys = (int64_t)sys.size();
        }
        {
            // the round's counts go in before any of its requests is reported
            // complete, so that a caller who saw its request finish sees them
            std::lock_guard<std::mutex> lk(S->mu);
            S->rounds += 1;
            S->systems += n_sys;
            if (hit) S->cache_hits += (int64_t)batch.size();
        }
        for (size_t b = 0; b < batch.size(); ++b) {
            srv_request* r = batch[b];
            const int32_t cnt = (int32_t)r->omegas.size();
            int rr = rc;
            if (rr == FHW_OK)
                rr = fhw_solve_range(ctx, first[b], cnt, r->inc.data(), (int32_t)r->inc.size(), r->psi, r->resid,
                                     r->sweeps);
            std::lock_guard<std::mutex> lk(S->mu);
            r->status = rr;
            if (rr != FHW_OK) r->err = fhw_last_error(ctx);
            S->done += 1;
            S->cv_done.notify_all();
        }
        const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        std::lock_guard<std::mutex> lk(S->mu);
        S->busy_s += dt;
    }
}

}  // namespace

extern "C" {

int fhw_server_create(fhw_server** out, const fhw_curve* curves, int32_t n_curves, const fhw_problem* prob,
                      int32_t n_slots, size_t hbm_budget_bytes, size_t queue_limit_bytes) {
    if (!out) return FHW_E_INVALID;
    *out = nullptr;
    if (!curves || n_curves < 1 || !prob || n_slots < 1 || n_slots > 8) return FHW_E_INVALID;
    if (prob->precision != FHW_FP64 && prob->precision != FHW_FP32_REFINE) return FHW_E_INVALID;
    if (!(prob->c > 0) || !std::isfinite(prob->c)) return FHW_E_INVALID;
    for (int k = 0; k < n_curves; ++k)
        if (curves[k].degree < 1 || !curves[k].cx || !curves[k].sx || !curves[k].cy || !curves[k].sy)
            return FHW_E_INVALID;
    std::unique_ptr<fhw_server> S(new (std::nothrow) fhw_server());
    if (!S) return FHW_E_NOMEM;
    if (hipGetDevice(&S->device) != hipSuccess) return FHW_E_HIP;
    S->prob = *prob;
    S->prob.lf_M = 0;
    S->prob.j_first = 0;
    S->prob.formulation = FHW_FORM_DIRECT;
    S->coef.resize(n_curves);
    S->curves.resize(n_curves);
    for (int k = 0; k < n_curves; ++k) {
        const int D1 = curves[k].degree + 1;
        std::vector<double>& v = S->coef[k];
        v.assign(4 * D1, 0.0);
        for (int d = 0; d < D1; ++d) {
            v[d] = curves[k].cx[d];
            v[D1 + d] = curves[k].sx[d];
            v[2 * D1 + d] = curves[k].cy[d];
            v[3 * D1 + d] = curves[k].sy[d];
        }
        S->curves[k] = fhw_curve{curves[k].degree, v.data(), v.data() + D1, v.data() + 2 * D1, v.data() + 3 * D1};
    }
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) return FHW_E_HIP;
    const size_t budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)(0.85 * (double)fr);
    S->slot_budget = budget / (size_t)n_slots;
    S->queue_limit = queue_limit_bytes ? queue_limit_bytes : budget;
    // one stream and context per slot, made here so that a failure is reported
    for (int i = 0; i < n_slots; ++i) {
        hipStream_t st = nullptr;
        fhw_ctx* ctx = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return FHW_E_HIP;
        const int rc = fhw_create(&ctx, st, S->slot_budget);
        if (rc != FHW_OK) {
            (void)hipStreamDestroy(st);
            return rc;
        }
        S->streams.push_back(st);
        S->ctxs.push_back(ctx);
    }
    fhw_server* raw = S.release();
    for (fhw_ctx* ctx : raw->ctxs) raw->workers.emplace_back([raw, ctx] { worker(raw, ctx); });
    *out = raw;
    return FHW_OK;
}

int fhw_server_submit(fhw_server* S, const fhw_request* q, int64_t* ticket) {
    if (!S || !q || !ticket) return FHW_E_INVALID;
    *ticket = 0;
    if (q->curve < 0 || q->curve >= (int32_t)S->curves.size() || q->n_freq < 1 || !q->omegas || q->N < 4 ||
        (q->N & 1) || q->N > 4096 || q->n_inc < 1 || !q->inc || !q->psi)
        return FHW_E_INVALID;
    for (int j = 0; j < q->n_freq; ++j)
        if (!(q->omegas[j] > 0) || !std::isfinite(q->omegas[j])) return FHW_E_INVALID;
    for (int j = 0; j < q->n_inc; ++j) {
        if (q->inc[j].kind != FHW_INC_PLANE && q->inc[j].kind != FHW_INC_POINT) return FHW_E_INVALID;
        if (!std::isfinite(q->inc[j].v[0]) || !std::isfinite(q->inc[j].v[1])) return FHW_E_INVALID;
    }
    std::unique_ptr<srv_request> r(new (std::nothrow) srv_request());
    if (!r) return FHW_E_NOMEM;
    r->curve = q->curve;
    r->N = q->N;
    r->omegas.assign(q->omegas, q->omegas + q->n_freq);
    r->inc.assign(q->inc, q->inc + q->n_inc);
    r->psi = q->psi;
    r->resid = q->resid;
    r->sweeps = q->sweeps;
    r->bytes = request_bytes(S->prob, q->N, (size_t)q->n_freq);
    std::lock_guard<std::mutex> lk(S->mu);
    if (r->bytes > S->slot_budget) return FHW_E_NOMEM;
    if (!S->queue.empty() && S->queued_bytes + r->bytes > S->queue_limit) {
        S->refused += 1;
        return FHW_E_BUSY;
    }
    r->ticket = S->next_ticket++;
    *ticket = r->ticket;
    S->queued_bytes += r->bytes;
    S->queue.push_back(r.get());
    S->reqs.emplace(r->ticket, std::move(r));
    S->cv_work.notify_one();
    return FHW_OK;
}

int fhw_server_poll(fhw_server* S, int64_t ticket, int32_t wait, int32_t* status) {
    if (!S || !status) return FHW_E_INVALID;
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return FHW_E_INVALID;
    srv_request* r = it->second.get();
    if (wait) S->cv_done.wait(lk, [&] { return r->status != 1; });
    *status = r->status;
    if (r->status != 1) S->reqs.erase(it);   // a finished ticket is reported once
    return FHW_OK;
}

int fhw_server_stats(fhw_server* S, int64_t* counts, double* busy_s) {
    if (!S || !counts) return FHW_E_INVALID;
    std::lock_guard<std::mutex> lk(S->mu);
    counts[0] = S->rounds;
    counts[1] = S->done;
    counts[2] = S->refused;
    counts[3] = S->systems;
    counts[4] = (int64_t)S->queue.size();
    counts[5] = S->cache_hits;
    if (busy_s) *busy_s = S->busy_s;
    return FHW_OK;
}

int fhw_server_destroy(fhw_server* S) {
    if (!S) return FHW_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    for (std::thread& t : S->workers)
        if (t.joinable()) t.join();
    delete S;
    return FHW_OK;
}

}  // extern "C"
