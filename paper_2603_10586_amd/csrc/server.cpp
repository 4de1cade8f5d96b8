// Continuous-batching solve server (the library's serving loop over qrvie_solve).
//
// Submission (any thread): the array is copied, its geometry is created on a planning
// context (serialised), and the library's own footprint estimates give the request's
// device bytes; the admission policy (policy.h) then decides.  Each of `slots` workers owns
// a context with its own stream and runs one admitted request at a time: it builds the
// operator (or takes the cached one for that geometry), generates the plane waves, solves,
// and copies the solution to host memory.  Finishing a request updates the policy, keeps
// a newly built operator resident when the cache has room, destroys evicted operators and
// admits whatever now fits.  Every request's kernels run on its worker's stream only and
// read shared operators read-only, so results do not depend on the mix.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.h"
#include "policy.h"

using namespace qrvie;

namespace {

double clock_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Owned copy of an array description.
struct ArrayCopy {
    int32_t n = 0, n_eps = 0, cells = 0, shape = 0, grid = 0;
    std::vector<double> centers, radius, height;
    std::vector<qrvie_c128> eps_r;
    std::vector<int32_t> lattice;
    double pitch = 0, wavelength = 0;
    qrvie_array_desc desc() const {
        return qrvie_array_desc{n, centers.data(), radius.data(), height.data(), eps_r.data(), n_eps,
                                lattice.empty() ? nullptr : lattice.data(), pitch, wavelength, cells, shape, grid};
    }
};

// The bytes that define an operator, appended into one string.  The string itself is the
// cache key, so two requests share an operator only when these bytes are equal (the hash of
// the key only picks a bucket).
struct Key {
    std::string bytes;
    void add(const void* p, size_t n) { bytes.append(static_cast<const char*>(p), n); }
};

struct Cached {
    qrvie_geom* geom = nullptr;
    qrvie_op* op = nullptr;
};

struct Request {
    uint64_t ticket = 0;
    std::string key;
    ArrayCopy arr;
    int32_t nrhs = 0;
    std::vector<double> th, ph;
    std::vector<int32_t> pol;
    double tol = 0;
    qrvie_geom* geom = nullptr;       // planning geometry (owned until handed to the cache)
    int64_t n = 0;
    size_t footprint = 0, op_bytes = 0, build_bytes = 0;
    double arrival = 0, admitted = -1, done_at = -1;
    bool done = false;
    qrvie_status status = QRVIE_OK;
    std::vector<qrvie_c128> x;
    std::vector<qrvie_solve_info> info;
    Cached hit;                       // cached operator pinned for it at admission (op null: build)
};

}  // namespace

struct qrvie_server {
    qrvie_server_opts o{};
    int device = 0;
    std::mutex mu;                    // everything below except the planning context
    std::condition_variable cv;
    qrvie::sched::Policy pol;
    std::mutex plan_mu;               // the planning context, geometry creation/destruction
    qrvie_ctx* plan = nullptr;
    std::vector<qrvie_ctx*> ctx;
    std::vector<std::thread> workers;
    std::deque<uint64_t> ready;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
    std::unordered_map<std::string, Cached> cache;
    bool closing = false;
    uint64_t next = 1;
    int64_t submitted = 0, completed = 0, failed = 0, refused = 0, ops_built = 0, rhs_solved = 0;
    std::vector<double> latencies, waits;
    double first_arrival = -1, last_done = -1;
    std::string err;

    qrvie_server(const qrvie_server_opts& op, int dev)
        : o(op), device(dev), pol(op.slots, op.hbm_budget, op.op_cache, op.max_bypass) {}
};

namespace {

void drop(qrvie_server* s, std::vector<Cached>& items) {
    std::lock_guard<std::mutex> g(s->plan_mu);
    for (Cached& c : items) {
        if (c.op) qrvie_op_destroy(c.op);
        if (c.geom) qrvie_geom_destroy(c.geom);
    }
    items.clear();
}

// mu held: admit what fits and hand evicted operators to `drops`
void admit_locked(qrvie_server* s, std::vector<Cached>& drops) {
    if (s->closing) return;
    std::vector<uint64_t> adm;
    std::vector<std::string> ev;
    s->pol.admit(&adm, &ev);
    for (const std::string& k : ev) {
        auto it = s->cache.find(k);
        if (it != s->cache.end()) {
            drops.push_back(it->second);
            s->cache.erase(it);
        }
    }
    const double now = clock_s();
    for (uint64_t t : adm) {
        Request* r = s->reqs.at(t).get();
        r->admitted = now;
        // only an operator the policy pinned for this request is safe from eviction while it
        // runs: one cached after admission is not used (the request builds its own)
        if (s->pol.pinned(t)) {
            auto it = s->cache.find(r->key);
            if (it != s->cache.end()) r->hit = it->second;
        }
        s->ready.push_back(t);
    }
    if (!adm.empty()) s->cv.notify_all();
}

// Far blocks of more rows are split into child pairs: materialised blocks stay at most
// 1.36 GB, so a build's compression chunks hold many blocks for the one-workgroup-per-block
// kernels (the largest arrays otherwise compress 21.7 GB blocks one at a time).
constexpr int64_t kServerMaxBlockRows = 9216;
// Concurrent builds share the device: each compresses at most 16 GiB of blocks at a time.
constexpr int64_t kServerChunkBytes = (int64_t)16 << 30;

qrvie_compress_opts compress_opts(const qrvie_server* s) {
    qrvie_compress_opts co{};
    co.eps = s->o.eps;
    co.far_prec = QRVIE_PREC_C128;
    co.near_prec = QRVIE_PREC_C128;
    co.max_block_rows = kServerMaxBlockRows;
    co.share_transpose = 0;
    co.seed = s->o.seed;
    co.verbose = 0;
    co.chunk_bytes = kServerChunkBytes;
    return co;
}

qrvie_solve_opts solve_opts(const qrvie_server* s, double tol) {
    qrvie_solve_opts so{};
    so.restart = s->o.restart;
    so.max_iter = s->o.max_iter;
    so.mode = s->o.mode;
    so.tol = tol;
    so.use_x0 = 0;
    so.inner_tol = 0.0;
    so.verbose = 0;
    so.block_width = s->o.block_width;
    return so;
}

// Solve one request on a worker context with a given operator.
qrvie_status run_request(qrvie_ctx* ctx, const qrvie_op* op, const qrvie_geom* g, Request* r, double tol,
                         const qrvie_server* s) {
    const int64_t n = r->n;
    c128 *v = nullptr, *x = nullptr;
    qrvie_status st = dalloc(ctx, (void**)&v, sizeof(c128) * n * r->nrhs, "request rhs");
    if (st == QRVIE_OK) st = dalloc(ctx, (void**)&x, sizeof(c128) * n * r->nrhs, "request x");
    if (st == QRVIE_OK)
        st = qrvie_rhs_plane_waves(ctx, g, r->nrhs, r->th.data(), r->ph.data(), r->pol.data(), (qrvie_c128*)v, n);
    if (st == QRVIE_OK) {
        const qrvie_solve_opts so = solve_opts(s, tol);
        r->info.assign(r->nrhs, qrvie_solve_info{});
        st = qrvie_solve(ctx, op, r->nrhs, (const qrvie_c128*)v, n, (qrvie_c128*)x, n, &so, r->info.data());
        if (st == QRVIE_OK || st == QRVIE_NOT_CONVERGED) {
            r->x.resize((size_t)n * r->nrhs);
            const qrvie_status c = hip_check(ctx, hipMemcpyAsync(r->x.data(), x, sizeof(c128) * n * r->nrhs,
                                                                 hipMemcpyDeviceToHost, ctx->stream), "fetch x");
            const qrvie_status y = c == QRVIE_OK ? hip_check(ctx, hipStreamSynchronize(ctx->stream), "fetch x") : c;
            if (y != QRVIE_OK) st = y;
        }
    }
    (void)hipStreamSynchronize(ctx->stream);
    dfree(ctx, v, sizeof(c128) * n * r->nrhs);
    dfree(ctx, x, sizeof(c128) * n * r->nrhs);
    return st;
}

void worker(qrvie_server* s, int slot) {
    (void)hipSetDevice(s->device);
    qrvie_ctx* ctx = s->ctx[slot];
    for (;;) {
        Request* r = nullptr;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv.wait(lk, [&] { return !s->ready.empty() || s->closing; });
            if (s->ready.empty()) return;
            r = s->reqs.at(s->ready.front()).get();
            s->ready.pop_front();
        }
        const Cached hit = r->hit;
        const bool is_hit = hit.op != nullptr;
        qrvie_op* op = nullptr;
        bool built = false;
        qrvie_status st = QRVIE_OK;
        std::string msg;
        if (is_hit) {
            op = hit.op;
        } else {
            const qrvie_compress_opts co = compress_opts(s);
            st = qrvie_op_create(ctx, r->geom, &co, &op);
            built = st == QRVIE_OK;
            if (!built) msg = qrvie_last_error(ctx);
            // the new operator is private to this worker until it is cached: tune its tiles
            // for this request's width (other widths keep the default shape; one wave is
            // solved by the single-vector solver, which has no tiles)
            if (built && s->o.mode == QRVIE_SOLVE_BLOCK && s->o.tune_tiles && r->nrhs > 1) {
                const int w = std::min(r->nrhs, s->o.block_width > 0 ? s->o.block_width : kMaxBlockRhs);
                qrvie_block_tune t;   // an optimisation only: on failure the default shapes stay
                (void)qrvie_op_tune_block(ctx, op, op->d_fac ? QRVIE_PREC_C128 : QRVIE_PREC_C64, w, 2, &t);
            }
        }
        if (st == QRVIE_OK) {
            st = run_request(ctx, op, is_hit ? hit.geom : r->geom, r, r->tol, s);
            if (st != QRVIE_OK && st != QRVIE_NOT_CONVERGED) msg = qrvie_last_error(ctx);
        }
        std::vector<Cached> drops;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            r->status = st;
            r->done = true;
            r->done_at = clock_s();
            if (st == QRVIE_OK || st == QRVIE_NOT_CONVERGED) {
                ++s->completed;
                s->rhs_solved += r->nrhs;
                s->latencies.push_back(r->done_at - r->arrival);
                s->waits.push_back(r->admitted - r->arrival);
                s->last_done = std::max(s->last_done, r->done_at);
            } else {
                ++s->failed;
                s->err = "request " + std::to_string(r->ticket) + ": " + msg;
            }
            if (built) ++s->ops_built;
            std::vector<std::string> ev;
            const bool kept = s->pol.finish(r->ticket, built, &ev);
            for (const std::string& k : ev) {
                auto it = s->cache.find(k);
                if (it != s->cache.end()) {
                    drops.push_back(it->second);
                    s->cache.erase(it);
                }
            }
            if (built && kept) {
                s->cache[r->key] = Cached{r->geom, op};
            } else {
                drops.push_back(Cached{r->geom, built ? op : nullptr});
            }
            r->geom = nullptr;
            admit_locked(s, drops);
            s->cv.notify_all();
        }
        drop(s, drops);
    }
}

qrvie_status bad(qrvie_server* s, const std::string& m, qrvie_status st = QRVIE_ERR_INVALID_ARG) {
    if (s) {
        std::lock_guard<std::mutex> lk(s->mu);
        s->err = m;
    }
    return st;
}

double percentile(std::vector<double> v, double q) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const double pos = q * (double)(v.size() - 1);
    const size_t i = (size_t)pos;
    const double f = pos - (double)i;
    return i + 1 < v.size() ? v[i] * (1.0 - f) + v[i + 1] * f : v[i];
}

}  // namespace

extern "C" {

qrvie_status qrvie_server_create(int hip_device, const qrvie_server_opts* o, qrvie_server** out) {
    if (!o || !out || o->slots < 1 || o->slots > 16 || o->hbm_budget == 0 || !(o->eps > 0.0 && o->eps < 1.0) ||
        o->restart < 1 || o->max_iter < 1 || o->op_cache < 0 ||
        (o->mode != QRVIE_SOLVE_FP64 && o->mode != QRVIE_SOLVE_BLOCK) || o->block_width < 0 ||
        o->block_width > kMaxBlockRhs || (o->tune_tiles != 0 && o->tune_tiles != 1) || o->max_bypass < 0)
        return QRVIE_ERR_INVALID_ARG;
    *out = nullptr;
    std::unique_ptr<qrvie_server> s(new qrvie_server(*o, hip_device));
    qrvie_status st = qrvie_ctx_create(hip_device, nullptr, 0, &s->plan);
    for (int i = 0; st == QRVIE_OK && i < o->slots; ++i) {
        qrvie_ctx* c = nullptr;
        st = qrvie_ctx_create(hip_device, nullptr, 0, &c);
        if (st == QRVIE_OK) s->ctx.push_back(c);
    }
    if (st != QRVIE_OK) {
        for (qrvie_ctx* c : s->ctx) qrvie_ctx_destroy(c);
        if (s->plan) qrvie_ctx_destroy(s->plan);
        return st;
    }
    for (int i = 0; i < o->slots; ++i) s->workers.emplace_back(worker, s.get(), i);
    *out = s.release();
    return QRVIE_OK;
}

qrvie_status qrvie_server_submit(qrvie_server* s, const qrvie_array_desc* a, int32_t nrhs, const double* th,
                                 const double* ph, const int32_t* pol, double tol, uint64_t* ticket) {
    if (!s || !a || !th || !ph || !pol || !ticket || nrhs < 1 || nrhs > kMaxBlockRhs || !(tol > 0.0) || a->n < 1 ||
        !a->centers || !a->radius || !a->height || !a->eps_r || (!a->lattice_ij && a->grid != QRVIE_GRID_PAPER) ||
        (a->n_eps != 1 && a->n_eps != a->n))
        return bad(s, "submit: invalid argument");
    auto r = std::make_unique<Request>();
    ArrayCopy& c = r->arr;
    c.n = a->n;
    c.n_eps = a->n_eps;
    c.cells = a->cells_per_particle;
    c.pitch = a->pitch;
    c.wavelength = a->wavelength;
    c.centers.assign(a->centers, a->centers + 3 * (size_t)a->n);
    c.radius.assign(a->radius, a->radius + a->n);
    c.height.assign(a->height, a->height + a->n);
    c.eps_r.assign(a->eps_r, a->eps_r + a->n_eps);
    c.shape = a->shape;
    c.grid = a->grid;
    if (a->grid != QRVIE_GRID_PAPER) c.lattice.assign(a->lattice_ij, a->lattice_ij + 2 * (size_t)a->n);
    r->nrhs = nrhs;
    r->th.assign(th, th + nrhs);
    r->ph.assign(ph, ph + nrhs);
    r->pol.assign(pol, pol + nrhs);
    r->tol = tol;
    Key k;
    k.add(&c.n, sizeof c.n);
    k.add(&c.n_eps, sizeof c.n_eps);
    k.add(c.centers.data(), sizeof(double) * c.centers.size());
    k.add(c.radius.data(), sizeof(double) * c.radius.size());
    k.add(c.height.data(), sizeof(double) * c.height.size());
    k.add(c.eps_r.data(), sizeof(qrvie_c128) * c.eps_r.size());
    k.add(c.lattice.data(), sizeof(int32_t) * c.lattice.size());
    k.add(&c.shape, sizeof c.shape);
    k.add(&c.grid, sizeof c.grid);
    k.add(&c.wavelength, sizeof c.wavelength);
    k.add(&s->o.eps, sizeof s->o.eps);
    k.add(&s->o.seed, sizeof s->o.seed);
    r->key = std::move(k.bytes);
    size_t op_b = 0, build_b = 0, sol_b = 0;
    {
        std::lock_guard<std::mutex> g(s->plan_mu);
        const qrvie_array_desc d = c.desc();
        qrvie_status st = qrvie_geom_create(s->plan, &d, &r->geom);
        if (st != QRVIE_OK) return bad(s, std::string("submit: ") + qrvie_last_error(s->plan), st);
        const qrvie_compress_opts co = compress_opts(s);
        const qrvie_solve_opts so = solve_opts(s, tol);
        op_footprint(r->geom, &co, &op_b, &build_b);
        st = qrvie_solve_footprint_estimate(r->geom, nullptr, nrhs, &so, &sol_b);
        if (st != QRVIE_OK) {
            qrvie_geom_destroy(r->geom);
            return bad(s, "submit: footprint estimate failed", st);
        }
        r->n = qrvie_geom_ndof(r->geom);
    }
    // a request that builds its operator holds the build's transient buffers as well; the
    // policy charges a cache hit only its solver bytes
    r->op_bytes = op_b;
    r->build_bytes = build_b;
    r->footprint = op_b + build_b + sol_b + 2 * sizeof(c128) * (size_t)r->n * nrhs;
    std::vector<Cached> drops;
    qrvie_status result = QRVIE_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->closing) {
            drops.push_back(Cached{r->geom, nullptr});
            result = QRVIE_ERR_QUEUE_FULL;
            s->err = "submit: the server is shutting down";
        } else {
            const uint64_t t = s->next++;
            r->ticket = t;
            r->arrival = clock_s();
            if (!s->pol.enqueue(t, r->key, r->footprint, r->op_bytes, r->build_bytes)) {
                ++s->refused;
                drops.push_back(Cached{r->geom, nullptr});
                s->err = "submit: the request's footprint (" + std::to_string(r->footprint) +
                         " bytes) exceeds the HBM budget";
                result = QRVIE_ERR_QUEUE_FULL;
            } else {
                ++s->submitted;
                if (s->first_arrival < 0) s->first_arrival = r->arrival;
                *ticket = t;
                s->reqs[t] = std::move(r);
                admit_locked(s, drops);
            }
        }
    }
    drop(s, drops);
    return result;
}

qrvie_status qrvie_server_poll(qrvie_server* s, uint64_t t, int32_t* done) {
    if (!s || !done) return QRVIE_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(t);
    if (it == s->reqs.end()) return QRVIE_ERR_INVALID_ARG;
    *done = it->second->done ? 1 : 0;
    return QRVIE_OK;
}

qrvie_status qrvie_server_wait(qrvie_server* s, uint64_t t, double timeout_s, int32_t* done) {
    if (!s || !done) return QRVIE_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    // -1: unknown or released, 0: queued or running, 1: finished.  Looked up again after every
    // wake-up, since another thread may fetch (and so free) the request meanwhile.
    auto state = [&]() -> int {
        auto it = s->reqs.find(t);
        return it == s->reqs.end() ? -1 : it->second->done ? 1 : 0;
    };
    if (state() < 0) return QRVIE_ERR_INVALID_ARG;
    auto settled = [&] { return state() != 0; };
    if (timeout_s < 0) {
        s->cv.wait(lk, settled);
    } else {
        s->cv.wait_for(lk, std::chrono::duration<double>(timeout_s), settled);
    }
    const int now = state();
    if (now < 0) {
        s->err = "wait: the ticket was released by another thread";
        return QRVIE_ERR_INVALID_ARG;
    }
    *done = now;
    return QRVIE_OK;
}

qrvie_status qrvie_server_fetch(qrvie_server* s, uint64_t t, qrvie_c128* x, int64_t ldx, qrvie_solve_info* info) {
    if (!s) return QRVIE_ERR_INVALID_ARG;
    std::unique_ptr<Request> r;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->reqs.find(t);
        if (it == s->reqs.end() || !it->second->done) {
            s->err = "fetch: unknown, released or unfinished ticket";
            return QRVIE_ERR_INVALID_ARG;
        }
        if (x && ldx < it->second->n) {
            s->err = "fetch: ldx < n";
            return QRVIE_ERR_INVALID_ARG;
        }
        r = std::move(it->second);
        s->reqs.erase(it);
    }
    if (x && !r->x.empty())
        for (int32_t c = 0; c < r->nrhs; ++c)
            std::memcpy(x + (int64_t)c * ldx, r->x.data() + (size_t)c * r->n, sizeof(qrvie_c128) * r->n);
    if (info && !r->info.empty()) std::memcpy(info, r->info.data(), sizeof(qrvie_solve_info) * r->nrhs);
    return r->status;
}

qrvie_status qrvie_server_get_stats(qrvie_server* s, qrvie_server_stats* out) {
    if (!s || !out) return QRVIE_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    qrvie_server_stats st{};
    st.submitted = s->submitted;
    st.completed = s->completed;
    st.failed = s->failed;
    st.refused = s->refused;
    st.running = s->pol.running();
    st.queued = (int64_t)s->pol.queued();
    st.ops_built = s->ops_built;
    st.cache_hits = s->pol.hits();
    st.evictions = s->pol.evictions();
    st.rhs_solved = s->rhs_solved;
    st.latency_p50_s = percentile(s->latencies, 0.50);
    st.latency_p99_s = percentile(s->latencies, 0.99);
    st.queue_wait_p50_s = percentile(s->waits, 0.50);
    st.makespan_s = (s->first_arrival >= 0 && s->last_done >= 0) ? s->last_done - s->first_arrival : 0.0;
    st.requests_per_s = st.makespan_s > 0 ? s->completed / st.makespan_s : 0.0;
    st.rhs_solves_per_s = st.makespan_s > 0 ? s->rhs_solved / st.makespan_s : 0.0;
    st.peak_bytes = s->pol.peak();
    st.in_use_bytes = s->pol.in_use();
    *out = st;
    return QRVIE_OK;
}

qrvie_status qrvie_server_request_times(qrvie_server* s, uint64_t t, double* arrival, double* admitted,
                                        double* done) {
    if (!s || !arrival || !admitted || !done) return QRVIE_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(t);
    if (it == s->reqs.end()) return QRVIE_ERR_INVALID_ARG;
    *arrival = it->second->arrival;
    *admitted = it->second->admitted;
    *done = it->second->done_at;
    return QRVIE_OK;
}

const char* qrvie_server_last_error(qrvie_server* s) {
    if (!s) return "null server";
    std::lock_guard<std::mutex> lk(s->mu);
    thread_local std::string copy;
    copy = s->err;
    return copy.c_str();
}

void qrvie_server_destroy(qrvie_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->closing = true;
        s->cv.notify_all();
    }
    for (std::thread& t : s->workers) t.join();
    std::vector<Cached> drops;
    for (auto& kv : s->cache) drops.push_back(kv.second);
    s->cache.clear();
    for (auto& kv : s->reqs)
        if (kv.second->geom) drops.push_back(Cached{kv.second->geom, nullptr});
    drop(s, drops);
    for (qrvie_ctx* c : s->ctx) qrvie_ctx_destroy(c);
    qrvie_ctx_destroy(s->plan);
    delete s;
}

}  // extern "C"
