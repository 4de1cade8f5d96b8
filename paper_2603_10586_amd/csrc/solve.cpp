// Product, preconditioner, factor export and the GMRES driver (host side).
//
// The solve is the paper's left-preconditioned GMRES (§6, with Z_D^-1 of §4).  Up to
// eight right-hand sides advance together: each keeps its own Krylov basis, Hessenberg
// matrix and Givens rotations, while every Arnoldi step applies the compressed operator
// and the preconditioner to all of them in one multi-RHS product, so the factor panels
// are streamed from HBM once per step for the whole group.
//
// Per Arnoldi step and RHS: classical Gram-Schmidt with one reorthogonalisation in two
// passes over the basis (the second projection through the Gram matrix of the basis),
// the new vector's norm fused into the update, and a device-side Givens update.  The host
// reads two numbers per RHS and step.  A column is converged when its preconditioned
// estimate is <= tol ||Z_D^-1 v|| and its true residual ||v - Z_QR x|| / ||v|| <= tol.
// When only the estimate meets its target, the target is tightened and the same Krylov
// space keeps growing (no restart); restarts happen only at the configured length m.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "work.h"

using namespace qrvie;

namespace {

constexpr int kGroup = 8;   // right-hand sides advanced together

// Rank-space and level-partial buffers of the product, owned by the caller of a product
// so that one operator can be applied from several streams at once.
struct ProdWork {
    c128* T = nullptr;
    c128* Y = nullptr;
    c128* S = nullptr;            // shared factors: Q^T x (rank space) and the mirror partials
    c128* P = nullptr;
    qrvie_status init(Work& w, const qrvie_op* op, int nr) {
        CHECK(w.alloc(&T, (size_t)op->t_len * nr, "rank-space vector"));
        if (op->shared) {
            CHECK(w.alloc(&S, (size_t)op->t_len, "rank-space Q^T x"));
            CHECK(w.alloc(&P, (size_t)op->p_len, "mirror partials"));
        }
        return w.alloc(&Y, (size_t)std::max(op->n_active, 1) * op->g->ndof() * nr, "level partials");
    }
};

int round_nr(int na) { return na <= 2 ? 2 : (na <= 4 ? 4 : 8); }

// out_r = v - Z x (or Z x when v is null), out_z = Z_D^-1 out_r (optional); internal order.
// lo: far factors from the complex64 panels (the reduced-precision operator).
void apply_one(const qrvie_op* op, hipStream_t s, const ProdWork& pw, const c128* x, const c128* v, c128* out_r,
               c128* out_z, bool lo = false) {
    const qrvie_geom* g = op->g;
    if (op->shared) {
        if (lo) {
            launch_qtphase(s, op->d_qt, op->n_qt, op->d_fac32, x, pw.S);
            launch_rphase_sh(s, op->d_rstrips, op->rlaunch[0].count, op->d_fac32, x, pw.T, op->d_tmap, pw.S, pw.P);
            launch_qphase_sh(s, op->d_qstrips, op->qlaunch[0].count, op->d_fac32, pw.T, pw.P, pw.Y);
        } else {
            launch_qtphase(s, op->d_qt, op->n_qt, op->d_fac, x, pw.S);
            launch_rphase_sh(s, op->d_rstrips, op->rlaunch[0].count, op->d_fac, x, pw.T, op->d_tmap, pw.S, pw.P);
            launch_qphase_sh(s, op->d_qstrips, op->qlaunch[0].count, op->d_fac, pw.T, pw.P, pw.Y);
        }
        launch_final(s, g->N, g->d_ptype, op->d_self, out_z ? op->d_pinv : nullptr, x, pw.Y, op->n_active, g->ndof(),
                     v, out_r, out_z);
        return;
    }
    for (const auto& L : op->rlaunch) {
        if (lo) launch_rphase_c64(s, op->d_rstrips + L.begin, L.count, op->d_fac32, x, pw.T, op->d_tmap);
        else launch_rphase(s, op->d_rstrips + L.begin, L.count, L.waves, op->d_fac, x, pw.T, op->d_tmap);
    }
    for (const auto& L : op->qlaunch) {
        if (lo) launch_qphase_c64(s, op->d_qstrips + L.begin, L.count, op->d_fac32, pw.T, pw.Y);
        else launch_qphase(s, op->d_qstrips + L.begin, L.count, L.waves, op->d_fac, pw.T, pw.Y);
    }
    launch_final(s, g->N, g->d_ptype, op->d_self, out_z ? op->d_pinv : nullptr, x, pw.Y, op->n_active, g->ndof(), v,
                 out_r, out_z);
}

// The same for nr RHS-interleaved vectors.
void apply_multi(const qrvie_op* op, hipStream_t s, const ProdWork& pw, int nr, const c128* X, const c128* V,
                 c128* out_r, c128* out_z, bool lo = false) {
    const qrvie_geom* g = op->g;
    for (const auto& L : op->rlaunch) {
        if (lo) launch_rphase_m_c64(s, nr, op->d_rstrips + L.begin, L.count, op->d_fac32, X, pw.T, op->d_tmap);
        else launch_rphase_m(s, nr, op->d_rstrips + L.begin, L.count, op->d_fac, X, pw.T, op->d_tmap);
    }
    for (const auto& L : op->qlaunch) {
        if (lo) launch_qphase_m_c64(s, nr, op->d_qstrips + L.begin, L.count, op->d_fac32, pw.T, pw.Y);
        else launch_qphase_m(s, nr, op->d_qstrips + L.begin, L.count, op->d_fac, pw.T, pw.Y);
    }
    launch_final_m(s, nr, g->N, g->d_ptype, op->d_self, out_z ? op->d_pinv : nullptr, X, pw.Y, op->n_active,
                   g->ndof(), V, out_r, out_z);
}

qrvie_status check_vec_args(qrvie_ctx* ctx, const qrvie_op* op, int32_t nrhs, const void* a, int64_t lda, const void* b,
                            int64_t ldb, const char* what) {
    if (!ctx || !op || !a || !b || nrhs < 1 || lda < op->g->ndof() || ldb < op->g->ndof()) {
        if (ctx) set_err(ctx, std::string(what) + ": invalid argument");
        return QRVIE_ERR_INVALID_ARG;
    }
    return QRVIE_OK;
}

// ------------------------------------------------------------------ GMRES group engine
struct Col {
    c128 *V, *w, *x, *xc, *v, *r, *h, *H, *sn, *g, *y;
    c128* G;                      // Gram matrix V^H V of the basis, (m+1) x (m+1)
    double *cs, *nrm, *np, *bp;
    double vnorm = 0, pvnorm = 0, prec_tol = 0;
    double tol = 0;               // relative true-residual target of this column's system
    int max_it = 0;               // Arnoldi steps allowed in total
    int iters = 0, j = 0;
    bool active = false, converged = false, start = true;
    double t_apply = 0, t0 = 0;
    qrvie_solve_info inf{};
};

struct Group {
    qrvie_ctx* ctx;
    const qrvie_op* op;
    const qrvie_solve_opts* o;
    hipStream_t s;
    int64_t n;
    int m, nch, nblk, na;
    Work w;
    ProdWork pw;
    std::vector<Col> c;
    c128 *X = nullptr, *Z = nullptr;
    const c128** dcolsX = nullptr;
    c128** dcolsW = nullptr;
    double* status = nullptr;
    double* hstat = nullptr;      // pinned
    const c128** hcols = nullptr; // pinned
    hipEvent_t ev0{}, ev1{};
    bool lo = false;              // products with the complex64 panels

    Group(qrvie_ctx* cx, const qrvie_op* p, const qrvie_solve_opts* opt, int count, bool low)
        : ctx(cx), op(p), o(opt), s(cx->stream), n(p->g->ndof()), m(0), nch(0), nblk(0), na(count), w(cx), c(count),
          lo(low) {}
    ~Group() {
        if (hstat) (void)hipHostFree(hstat);
        if (hcols) (void)hipHostFree(hcols);
        (void)hipEventDestroy(ev0);
        (void)hipEventDestroy(ev1);
    }

    qrvie_status init() {
        m = std::min(o->restart, o->max_iter);
        nch = krylov_nchunks(n);
        nblk = krylov_nblocks(n);
        CHECK(pw.init(w, op, na > 1 ? round_nr(na) : 1));
        for (Col& k : c) {
            CHECK(w.alloc(&k.V, (size_t)n * (m + 1), "krylov basis"));
            CHECK(w.alloc(&k.w, n, "krylov w"));
            CHECK(w.alloc(&k.x, n, "solve x"));
            CHECK(w.alloc(&k.xc, n, "candidate x"));
            CHECK(w.alloc(&k.v, n, "solve v"));
            CHECK(w.alloc(&k.r, n, "solve r"));
            CHECK(w.alloc(&k.h, m + 2, "hessenberg column"));
            CHECK(w.alloc(&k.H, (size_t)(m + 1) * m, "hessenberg"));
            CHECK(w.alloc(&k.sn, m, "givens s"));
            CHECK(w.alloc(&k.g, m + 1, "givens rhs"));
            CHECK(w.alloc(&k.y, std::max(m, 1), "lsq solution"));
            CHECK(w.alloc(&k.cs, m, "givens c"));
            CHECK(w.alloc(&k.nrm, 4, "norms"));
            CHECK(hip_check(ctx, hipMemsetAsync(k.nrm, 0, sizeof(double) * 4, s), "norms"));
            CHECK(w.alloc(&k.np, nch, "norm partials"));
            CHECK(w.alloc(&k.bp, nblk, "update norm partials"));
            CHECK(w.alloc(&k.G, (size_t)(m + 1) * (m + 1), "gram matrix"));
        }
        nchg = krylov_nchunks(m + 1);
        CHECK(w.alloc(&pd_all, (size_t)nch * (m + 1) * na, "dot partials"));
        CHECK(w.alloc(&pu_all, (size_t)nch * (m + 1) * na, "gram partials"));
        CHECK(w.alloc(&pg_all, (size_t)nchg * (m + 1) * na, "gram product partials"));
        CHECK(w.alloc(&status, 2 * (size_t)na, "status"));
        if (na > 1) {
            const int nr = round_nr(na);
            CHECK(w.alloc(&X, (size_t)n * nr, "block x"));
            CHECK(w.alloc(&Z, (size_t)n * nr, "block z"));
            CHECK(w.alloc(&dcolsX, nr, "column pointers"));
            CHECK(w.alloc(&dcolsW, nr, "column pointers"));
        }
        CHECK(hip_check(ctx, hipHostMalloc((void**)&hstat, sizeof(double) * 2 * (na + 2), hipHostMallocDefault), "pinned"));
        CHECK(hip_check(ctx, hipHostMalloc((void**)&hcols, sizeof(void*) * 16, hipHostMallocDefault), "pinned"));
        (void)hipEventCreate(&ev0);
        (void)hipEventCreate(&ev1);
        return QRVIE_OK;
    }
    c128 *pd_all = nullptr, *pu_all = nullptr, *pg_all = nullptr;
    int nchg = 0;
    c128* pd(int k) { return pd_all + (size_t)k * nch * (m + 1); }
    c128* pu(int k) { return pu_all + (size_t)k * nch * (m + 1); }
    c128* pg(int k) { return pg_all + (size_t)k * nchg * (m + 1); }

    qrvie_status read(const double* d, int cnt) {
        CHECK(hip_check(ctx, hipMemcpyAsync(hstat, d, sizeof(double) * cnt, hipMemcpyDeviceToHost, s), "read"));
        return hip_check(ctx, hipStreamSynchronize(s), "sync");
    }
    void norm_to(Col& k, const c128* vec, double* dst) {
        launch_norm2(s, vec, n, k.np);
        launch_reduce_norm(s, k.np, nch, dst);
    }
    float elapsed() {
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, ev0, ev1);
        return ms * 1e-3f;
    }

    qrvie_status finish(c128* const* x, const std::vector<c128*>* src, qrvie_solve_info* info, double t0);

    // Column i's system is k.v with the initial guess in k.x: norms of v and Z_D^-1 v,
    // target tol on the true relative residual, at most max_it Arnoldi steps in total.
    qrvie_status prepare(int i, double tol, int max_it) {
        Col& k = c[i];
        const qrvie_geom* g = op->g;
        norm_to(k, k.v, k.nrm + 0);
        launch_block_apply(s, g->N, g->d_ptype, op->d_pinv, k.v, k.r);
        norm_to(k, k.r, k.nrm + 1);
        CHECK(read(k.nrm, 2));
        k.vnorm = std::sqrt(hstat[0]);
        k.pvnorm = std::sqrt(hstat[1]);
        if (!std::isfinite(k.vnorm)) {
            set_err(ctx, "solve: right-hand side has non-finite entries");
            return QRVIE_ERR_INVALID_ARG;
        }
        k.tol = tol;
        k.max_it = max_it;
        k.prec_tol = tol;
        k.j = 0;
        k.start = true;
        k.active = k.vnorm > 0.0;
        k.converged = !k.active;
        if (!k.active) CHECK(hip_check(ctx, hipMemsetAsync(k.x, 0, sizeof(c128) * n, s), "zero x"));
        return QRVIE_OK;
    }

    // r = v - Z x, w = Z_D^-1 r: starts a cycle (or finishes the column)
    qrvie_status start_cycle(int i) {
        Col& k = c[i];
        (void)hipEventRecord(ev0, s);
        apply_one(op, s, pw, k.x, k.v, k.r, k.w, lo);
        (void)hipEventRecord(ev1, s);
        k.inf.n_apply++;
        k.inf.n_prec++;
        norm_to(k, k.r, k.nrm + 0);
        norm_to(k, k.w, k.nrm + 1);
        CHECK(read(k.nrm, 2));
        k.t_apply += elapsed();
        const double tr = std::sqrt(hstat[0]) / k.vnorm;
        const double beta = std::sqrt(hstat[1]);
        if (!std::isfinite(beta)) { set_err(ctx, "solve: non-finite residual"); return QRVIE_ERR_DEVICE; }
        k.inf.rel_res_true = tr;
        k.inf.rel_res_prec = beta / k.pvnorm;
        if (k.inf.rel_res_prec <= k.prec_tol) {
            if (tr <= k.tol) { k.converged = true; k.active = false; return QRVIE_OK; }
            k.prec_tol = std::max(k.prec_tol * 0.5 * k.tol / tr, 1e-15);
        }
        if (k.iters >= k.max_it) { k.active = false; return QRVIE_OK; }
        launch_scale_into(s, k.w, n, k.nrm + 1, k.V, k.g);       // V0 = w / beta, g0 = beta
        k.j = 0;
        k.start = false;
        return QRVIE_OK;
    }

    // Gram-Schmidt + Givens of column i's step j (w already holds Z_D^-1 Z v_j).
    // Pass 1: h1 = V^H w and G[:, j] = V^H v_j (G[j, :] mirrored); h = 2 h1 - G h1;
    // pass 2: w -= V h with ||w||^2 fused; then the Givens update and v_{j+1} = w / ||w||.
    void arnoldi_tail(int i) {
        Col& k = c[i];
        const int j = k.j;
        const int64_t ldg = m + 1;
        c128* gcol = k.G + (int64_t)j * ldg;
        launch_multidot(s, k.V, n, j + 1, k.w, k.V + (size_t)j * n, n, pd(i), pu(i));
        launch_reduce_dots(s, pd(i), nch, j + 1, k.h, nullptr, 0);
        launch_reduce_dots(s, pu(i), nch, j + 1, gcol, k.G + j, ldg);
        launch_multidot(s, k.G, ldg, j + 1, k.h, nullptr, j + 1, pg(i), nullptr);
        launch_cgs2_coeffs(s, pg(i), krylov_nchunks(j + 1), j + 1, k.h);
        launch_gemv_sub(s, k.V, n, j + 1, k.h, k.w, n, k.bp);
        launch_reduce_norm(s, k.bp, nblk, k.nrm + 2);
        launch_givens(s, j, k.h, k.H, m + 1, k.cs, k.sn, k.g, k.nrm + 2, status + 2 * i);
        launch_scale_into(s, k.w, n, k.nrm + 2, k.V + (size_t)(j + 1) * n, nullptr);
    }

    // candidate x_c = x + V y; accept if the true residual meets tol
    qrvie_status candidate(int i, int kused, bool& accepted) {
        Col& k = c[i];
        launch_trisolve(s, kused, k.H, m + 1, k.g, k.y);
        CHECK(hip_check(ctx, hipMemcpyAsync(k.xc, k.x, sizeof(c128) * n, hipMemcpyDeviceToDevice, s), "x_c"));
        launch_gemv_add(s, k.V, n, kused, k.y, k.xc, n);
        (void)hipEventRecord(ev0, s);
        apply_one(op, s, pw, k.xc, k.v, k.r, nullptr, lo);
        (void)hipEventRecord(ev1, s);
        k.inf.n_apply++;
        norm_to(k, k.r, k.nrm + 0);
        CHECK(read(k.nrm, 1));
        k.t_apply += elapsed();
        const double tr = std::sqrt(hstat[0]) / k.vnorm;
        k.inf.rel_res_true = tr;
        accepted = tr <= k.tol;
        if (accepted) CHECK(hip_check(ctx, hipMemcpyAsync(k.x, k.xc, sizeof(c128) * n, hipMemcpyDeviceToDevice, s), "x"));
        else k.prec_tol = std::max(k.prec_tol * 0.5 * k.tol / tr, 1e-15);
        return QRVIE_OK;
    }

    qrvie_status run() {
        for (;;) {
            for (int i = 0; i < na; ++i)
                if (c[i].active && c[i].start) CHECK(start_cycle(i));
            std::vector<int> act;
            for (int i = 0; i < na; ++i)
                if (c[i].active) act.push_back(i);
            if (act.empty()) return QRVIE_OK;
            // one product + preconditioner for every active column
            (void)hipEventRecord(ev0, s);
            if (act.size() == 1 || op->shared) {
                // one column, or shared factors (no multi-vector kernels): a product per column
                for (int i : act) apply_one(op, s, pw, c[i].V + (size_t)c[i].j * n, nullptr, nullptr, c[i].w, lo);
            } else {
                const int nr = round_nr((int)act.size());
                for (size_t a = 0; a < act.size(); ++a) hcols[a] = c[act[a]].V + (size_t)c[act[a]].j * n;
                for (size_t a = 0; a < act.size(); ++a) hcols[8 + a] = c[act[a]].w;
                CHECK(hip_check(ctx, hipMemcpyAsync(dcolsX, hcols, sizeof(void*) * act.size(), hipMemcpyHostToDevice, s), "cols"));
                CHECK(hip_check(ctx, hipMemcpyAsync(dcolsW, hcols + 8, sizeof(void*) * act.size(), hipMemcpyHostToDevice, s), "cols"));
                launch_interleave(s, nr, n, dcolsX, X, (int)act.size());
                apply_multi(op, s, pw, nr, X, nullptr, nullptr, Z, lo);
                launch_deinterleave(s, nr, n, Z, dcolsW, (int)act.size());
            }
            (void)hipEventRecord(ev1, s);
            for (int i : act) arnoldi_tail(i);
            CHECK(hip_check(ctx, hipGetLastError(), "gmres launch"));
            CHECK(read(status, 2 * na));
            const double tshare = elapsed() / act.size();
            std::vector<double> st(hstat, hstat + 2 * na);
            for (int i : act) {
                Col& k = c[i];
                k.t_apply += tshare;
                k.inf.n_apply++;
                k.inf.n_prec++;
                k.iters++;
                k.j++;
                const int kused = k.j;
                const double est = st[2 * i] / k.pvnorm;
                const bool breakdown = st[2 * i + 1] == 0.0;
                k.inf.rel_res_prec = est;
                bool end_cycle = kused >= m || k.iters >= k.max_it;
                if (est <= k.prec_tol || breakdown) {
                    bool ok = false;
                    CHECK(candidate(i, kused, ok));
                    if (ok) {
                        launch_gram_deviation(s, k.G, m + 1, kused, k.nrm + 3);
                        k.converged = true;
                        k.active = false;
                        continue;
                    }
                    if (breakdown) end_cycle = true;
                }
                if (end_cycle) {
                    launch_gram_deviation(s, k.G, m + 1, kused, k.nrm + 3);
                    launch_trisolve(s, kused, k.H, m + 1, k.g, k.y);
                    launch_gemv_add(s, k.V, n, kused, k.y, k.x, n);
                    k.inf.restarts++;
                    k.start = true;   // the next start_cycle computes the true residual
                }
            }
        }
    }
};

// Unpermute the solutions (from src[i], else each column's x) and fill info.
qrvie_status Group::finish(c128* const* x, const std::vector<c128*>* src, qrvie_solve_info* info, double t0) {
    qrvie_status overall = QRVIE_OK;
    const qrvie_geom* g = op->g;
    for (int i = 0; i < na; ++i) {
        Col& k = c[i];
        launch_permute(s, g->N, g->d_i2c, src ? (*src)[i] : k.x, x[i], 0);
        CHECK(read(k.nrm + 3, 1));
        k.inf.basis_ortho = hstat[0];
        k.inf.iterations = k.iters;
        k.inf.converged = k.converged ? 1 : 0;
        k.inf.n_reorth = k.iters;   // every step carries the second projection (through G)
        k.inf.t_apply_s = k.t_apply;
        k.inf.t_prec_s = 0.0;   // fused into the product pass
        k.inf.t_total_s = now_s() - t0;
        k.inf.t_krylov_s = std::max(0.0, k.inf.t_total_s - k.t_apply);
        if (info) info[i] = k.inf;
        if (!k.converged) overall = QRVIE_NOT_CONVERGED;
    }
    return overall;
}

qrvie_status solve_group(qrvie_ctx* ctx, const qrvie_op* op, int na, const c128* const* v, c128* const* x,
                         const qrvie_solve_opts* o, qrvie_solve_info* info) {
    const double t0 = now_s();
    Group G(ctx, op, o, na, !op->d_fac);   // an operator with only complex64 panels uses them
    CHECK(G.init());
    hipStream_t s = ctx->stream;
    const qrvie_geom* g = op->g;
    for (int i = 0; i < na; ++i) {
        Col& k = G.c[i];
        launch_permute(s, g->N, g->d_i2c, v[i], k.v, 1);
        if (o->use_x0) launch_permute(s, g->N, g->d_i2c, x[i], k.x, 1);
        else CHECK(hip_check(ctx, hipMemsetAsync(k.x, 0, sizeof(c128) * G.n, s), "x0"));
        CHECK(G.prepare(i, o->tol, o->max_iter));
    }
    CHECK(G.run());
    return G.finish(x, nullptr, info, t0);
}

// Mixed-precision iterative refinement (one group of right-hand sides).  Outer step:
// r = v - Z_QR x with the complex128 factors; if ||r|| <= tol ||v|| the column is done.
// Otherwise the correction d of Z_lo d = r comes from the same preconditioned GMRES run
// on the complex64 factors (FP64 accumulation and Krylov algebra), to the relative
// target 0.25 tol ||v|| / ||r||, and x += d.  Since ||r - Z_QR d|| <= ||r - Z_lo d|| +
// ||(Z_lo - Z_QR) d||, one refinement leaves the rounding of the factors, amplified by
// the conditioning, as the remaining residual; the next refinement removes most of it.
constexpr int kMaxRefine = 12;

qrvie_status solve_group_ir(qrvie_ctx* ctx, const qrvie_op* op, int na, const c128* const* v, c128* const* x,
                            const qrvie_solve_opts* o, qrvie_solve_info* info) {
    const double t0 = now_s();
    Group G(ctx, op, o, na, true);
    CHECK(G.init());
    hipStream_t s = ctx->stream;
    const qrvie_geom* g = op->g;
    const int64_t n = G.n;
    std::vector<c128*> vin(na), xh(na);
    std::vector<double> vn(na, 0.0), rel(na, 0.0);
    std::vector<int> state(na, 0);   // 0 refining, 1 converged, 2 stopped
    for (int i = 0; i < na; ++i) {
        Col& k = G.c[i];
        CHECK(G.w.alloc(&vin[i], n, "refinement v"));
        CHECK(G.w.alloc(&xh[i], n, "refinement x"));
        launch_permute(s, g->N, g->d_i2c, v[i], vin[i], 1);
        if (o->use_x0) launch_permute(s, g->N, g->d_i2c, x[i], xh[i], 1);
        else CHECK(hip_check(ctx, hipMemsetAsync(xh[i], 0, sizeof(c128) * n, s), "x0"));
        G.norm_to(k, vin[i], k.nrm + 0);
        CHECK(G.read(k.nrm, 1));
        vn[i] = std::sqrt(G.hstat[0]);
        if (!std::isfinite(vn[i])) {
            set_err(ctx, "solve: right-hand side has non-finite entries");
            return QRVIE_ERR_INVALID_ARG;
        }
        if (vn[i] == 0.0) {
            CHECK(hip_check(ctx, hipMemsetAsync(xh[i], 0, sizeof(c128) * n, s), "zero x"));
            state[i] = 1;
        }
    }
    for (int it = 0;; ++it) {
        std::vector<int> refine;
        for (int i = 0; i < na; ++i) {
            if (state[i] != 0) continue;
            Col& k = G.c[i];
            (void)hipEventRecord(G.ev0, s);
            apply_one(op, s, G.pw, xh[i], vin[i], k.v, nullptr, false);   // inner right-hand side r
            (void)hipEventRecord(G.ev1, s);
            k.inf.n_apply++;
            G.norm_to(k, k.v, k.nrm + 0);
            CHECK(G.read(k.nrm, 1));
            k.t_apply += G.elapsed();
            const double r = std::sqrt(G.hstat[0]) / vn[i];
            if (!std::isfinite(r)) { set_err(ctx, "solve: non-finite residual"); return QRVIE_ERR_DEVICE; }
            const bool stalled = it > 0 && r > 0.5 * rel[i];
            rel[i] = r;
            k.inf.rel_res_true = r;
            if (r <= o->tol) { state[i] = 1; continue; }
            if (it >= kMaxRefine || k.iters >= o->max_iter || stalled) { state[i] = 2; continue; }
            CHECK(hip_check(ctx, hipMemsetAsync(k.x, 0, sizeof(c128) * n, s), "correction"));
            const double eta = o->inner_tol > 0.0 ? o->inner_tol : std::min(0.5, std::max(0.25 * o->tol / r, 1e-14));
            CHECK(G.prepare(i, eta, o->max_iter));
            k.inf.n_refine++;
            refine.push_back(i);
        }
        if (refine.empty()) break;
        CHECK(G.run());
        for (int i : refine) launch_add(s, G.c[i].x, n, xh[i]);
    }
    for (int i = 0; i < na; ++i) {
        G.c[i].converged = state[i] == 1;
        if (state[i] == 1 && vn[i] == 0.0) G.c[i].inf.rel_res_true = 0.0;
    }
    return G.finish(x, &xh, info, t0);
}

// Mixed-precision refinement with block corrections (QRVIE_SOLVE_BLOCK_IR): the residuals
// of all columns with the complex128 factors, then one block GMRES solve on the complex64
// panels for all unconverged columns together (inner tolerance as in solve_group_ir, the
// tightest of the columns), x += d, until every column meets tol, stalls (a correction
// that does not halve its residual), or the limits are reached.  Caller order throughout.
qrvie_status solve_block_ir(qrvie_ctx* ctx, const qrvie_op* op, int nrhs, const c128* v, int64_t ldv, c128* x,
                            int64_t ldx, const qrvie_solve_opts* o, qrvie_solve_info* info) {
    const double t0 = now_s();
    const int64_t n = op->g->ndof();
    hipStream_t s = ctx->stream;
    Work w(ctx);
    c128 *R, *Ra, *D;
    double* dn;
    CHECK(w.alloc(&R, (size_t)n * nrhs, "refinement residuals"));
    CHECK(w.alloc(&Ra, (size_t)n * nrhs, "refinement right-hand sides"));
    CHECK(w.alloc(&D, (size_t)n * nrhs, "refinement corrections"));
    CHECK(w.alloc(&dn, (size_t)nrhs, "refinement norms"));
    std::vector<qrvie_solve_info> inf(nrhs);
    for (auto& i : inf) i = qrvie_solve_info{};
    auto norms = [&](const c128* a, int64_t lda, std::vector<double>& out) -> qrvie_status {
        out.assign(nrhs, 0.0);
        launch_col_norms(s, (int)n, a, lda, nrhs, dn);
        CHECK(hip_check(ctx, hipMemcpyAsync(out.data(), dn, sizeof(double) * nrhs, hipMemcpyDeviceToHost, s), "norms"));
        return hip_check(ctx, hipStreamSynchronize(s), "norms");
    };
    if (!o->use_x0)
        for (int c = 0; c < nrhs; ++c)
            CHECK(hip_check(ctx, hipMemsetAsync(x + (int64_t)c * ldx, 0, sizeof(c128) * n, s), "x0"));
    std::vector<double> vn, rn, rel(nrhs, 0.0);
    CHECK(norms(v, ldv, vn));
    std::vector<int> state(nrhs, 0);   // 0 refining, 1 converged, 2 stopped
    for (int c = 0; c < nrhs; ++c) {
        if (!std::isfinite(vn[c])) {
            set_err(ctx, "solve: right-hand side has non-finite entries");
            return QRVIE_ERR_INVALID_ARG;
        }
        if (vn[c] == 0.0) {
            CHECK(hip_check(ctx, hipMemsetAsync(x + (int64_t)c * ldx, 0, sizeof(c128) * n, s), "zero x"));
            state[c] = 1;
        }
    }
    const int width = o->block_width > 0 ? o->block_width : kMaxBlockRhs;
    // corrections: BF16 planes or complex64 panels on FP32 matrix cores, else the complex64
    // panels widened to FP64
    const int kind = op->d_fac16 ? kBlockBF16 : o->inner_fp32 ? kBlockF32 : kBlockF64;
    for (int it = 0;; ++it) {
        // residuals with the complex128 factors, or the complex64 ones with FP64 accumulation
        CHECK(qrvie_apply_prec(ctx, op, op->d_fac ? QRVIE_PREC_C128 : QRVIE_PREC_C64, nrhs, (const qrvie_c128*)x, ldx,
                               (qrvie_c128*)R, n));
        for (int c = 0; c < nrhs; ++c) launch_rsub(s, v + (int64_t)c * ldv, n, R + (int64_t)c * n);
        CHECK(norms(R, n, rn));
        std::vector<int> act;
        double eta = 0.5;
        for (int c = 0; c < nrhs; ++c) {
            if (state[c] != 0) continue;
            const double r = rn[c] / vn[c];
            if (!std::isfinite(r)) { set_err(ctx, "solve: non-finite residual"); return QRVIE_ERR_DEVICE; }
            const bool stalled = it > 0 && r > 0.5 * rel[c];
            rel[c] = r;
            inf[c].rel_res_true = r;
            if (r <= o->tol) { state[c] = 1; continue; }
            if (it >= kMaxRefine || inf[c].iterations >= o->max_iter || stalled) { state[c] = 2; continue; }
            act.push_back(c);
            eta = std::min(eta, o->inner_tol > 0.0 ? o->inner_tol : std::max(0.25 * o->tol / r, 1e-14));
        }
        // corrections on FP32 matrix cores cannot resolve residuals far below their rounding: a
        // correction aims at no less than 1e-5 (complex64 factors) or 1e-2 (BF16 factors) and
        // further refinements take the rest
        if (o->inner_tol <= 0.0) eta = std::max(eta, kind == kBlockBF16 ? 1e-2 : kind == kBlockF32 ? 1e-5 : 0.0);
        if (act.empty()) break;
        for (size_t j = 0; j < act.size(); ++j)
            CHECK(hip_check(ctx, hipMemcpyAsync(Ra + (int64_t)j * n, R + (int64_t)act[j] * n, sizeof(c128) * n,
                                                hipMemcpyDeviceToDevice, s), "refinement rhs"));
        qrvie_solve_opts oi = *o;
        oi.mode = QRVIE_SOLVE_BLOCK;
        oi.tol = eta;
        oi.use_x0 = 0;
        for (size_t r0 = 0; r0 < act.size(); r0 += (size_t)width) {
            const int cnt = (int)std::min(act.size() - r0, (size_t)width);
            std::vector<qrvie_solve_info> ii(cnt);
            bool broke = false;
            const qrvie_status st = solve_block(ctx, op, cnt, Ra + (int64_t)r0 * n, n, D + (int64_t)r0 * n, n, &oi,
                                                ii.data(), &broke, true, kind);
            if (st != QRVIE_OK && st != QRVIE_NOT_CONVERGED) return st;
            for (int j = 0; j < cnt; ++j) {
                qrvie_solve_info& f = inf[act[r0 + j]];
                f.iterations += ii[j].iterations;
                f.restarts += ii[j].restarts;
                f.n_apply += ii[j].n_apply;
                f.n_prec += ii[j].n_prec;
                f.t_apply_s += ii[j].t_apply_s;
                f.rel_res_prec = ii[j].rel_res_prec;
                f.n_refine++;
                if (broke) state[act[r0 + j]] = 2;   // rank-deficient correction block: keep what it gave
            }
        }
        for (size_t j = 0; j < act.size(); ++j) launch_add(s, D + (int64_t)j * n, n, x + (int64_t)act[j] * ldx);
    }
    CHECK(hip_check(ctx, hipStreamSynchronize(s), "solve"));
    const double t1 = now_s();
    qrvie_status overall = QRVIE_OK;
    for (int c = 0; c < nrhs; ++c) {
        inf[c].converged = state[c] == 1;
        if (state[c] == 1 && vn[c] == 0.0) inf[c].rel_res_true = 0.0;
        inf[c].t_total_s = t1 - t0;
        if (!inf[c].converged) overall = QRVIE_NOT_CONVERGED;
    }
    if (info) std::copy(inf.begin(), inf.end(), info);
    return overall;
}

}  // namespace

namespace qrvie {

void apply_single_into(const qrvie_op* op, hipStream_t s, c128* T, c128* Ylev, c128* Sq, c128* P, c128* xi, c128* yi,
                       const c128* x, c128* y) {
    ProdWork pw;
    pw.T = T;
    pw.Y = Ylev;
    pw.S = Sq;
    pw.P = P;
    launch_permute(s, op->g->N, op->g->d_i2c, x, xi, 1);
    apply_one(op, s, pw, xi, nullptr, yi, nullptr, !op->d_fac);
    launch_permute(s, op->g->N, op->g->d_i2c, yi, y, 0);
}

}  // namespace qrvie

extern "C" {

qrvie_status qrvie_apply(qrvie_ctx* ctx, const qrvie_op* op, int32_t nrhs, const qrvie_c128* x, int64_t ldx,
                         qrvie_c128* y, int64_t ldy) {
    return qrvie_apply_prec(ctx, op, op && !op->d_fac ? QRVIE_PREC_C64 : QRVIE_PREC_C128, nrhs, x, ldx, y, ldy);
}

qrvie_status qrvie_apply_prec(qrvie_ctx* ctx, const qrvie_op* op, int32_t prec, int32_t nrhs, const qrvie_c128* x,
                              int64_t ldx, qrvie_c128* y, int64_t ldy) {
    CHECK(check_vec_args(ctx, op, nrhs, x, ldx, y, ldy, "apply"));
    if (!((prec == QRVIE_PREC_C128 && op->d_fac) || (prec == QRVIE_PREC_C64 && op->d_fac32) ||
          (prec == QRVIE_PREC_C64_F32 && op->d_fac32 && op->d_self32) || (prec == QRVIE_PREC_BF16X2 && op->d_fac16))) {
        set_err(ctx, "apply: the operator holds no far factors of the requested precision");
        return QRVIE_ERR_INVALID_ARG;
    }
    const bool lo = prec == QRVIE_PREC_C64;
    const int kind = prec == QRVIE_PREC_BF16X2 ? kBlockBF16 : prec == QRVIE_PREC_C64_F32 ? kBlockF32 : kBlockF64;
    const int64_t n = op->g->ndof();
    hipStream_t s = ctx->stream;
    Work w(ctx);
    if (nrhs >= 16 || kind != kBlockF64) {
        // blocks of up to 64 right-hand sides on the MFMA kernels
        BlockWork bw;
        CHECK(bw.init(w, op));
        c128 *X, *Y;
        CHECK(w.alloc(&X, (size_t)n * kMaxBlockRhs, "apply block"));
        CHECK(w.alloc(&Y, (size_t)n * kMaxBlockRhs, "apply block"));
        for (int r0 = 0; r0 < nrhs; r0 += kMaxBlockRhs) {
            const int cnt = std::min(kMaxBlockRhs, nrhs - r0);
            const int nt = (cnt + 15) / 16;
            launch_gather_block(s, nt, op->g->N, op->g->d_i2c, (const c128*)x + (int64_t)r0 * ldx, ldx, cnt, X);
            block_product(op, s, bw, nt, X, nullptr, Y, nullptr, lo, kind);
            launch_scatter_block(s, nt, op->g->N, op->g->d_i2c, Y, (c128*)y + (int64_t)r0 * ldy, ldy, cnt);
        }
        CHECK(hip_check(ctx, hipGetLastError(), "apply launch"));
        return hip_check(ctx, hipStreamSynchronize(s), "apply");
    }
    ProdWork pw;
    const int nrmax = nrhs > 1 && !op->shared ? kGroup : 1;
    CHECK(pw.init(w, op, nrmax));
    c128 *xi, *yi, *X = nullptr, *Y = nullptr;
    CHECK(w.alloc(&xi, (size_t)n * nrmax, "apply work"));
    CHECK(w.alloc(&yi, (size_t)n * nrmax, "apply work"));
    if (op->shared) {
        // shared factors: one three-pass product per column
        for (int r0 = 0; r0 < nrhs; ++r0) {
            launch_permute(s, op->g->N, op->g->d_i2c, (const c128*)x + r0 * ldx, xi, 1);
            apply_one(op, s, pw, xi, nullptr, yi, nullptr, lo);
            launch_permute(s, op->g->N, op->g->d_i2c, yi, (c128*)y + r0 * ldy, 0);
        }
    } else if (nrhs == 1) {
        launch_permute(s, op->g->N, op->g->d_i2c, (const c128*)x, xi, 1);
        apply_one(op, s, pw, xi, nullptr, yi, nullptr, lo);
        launch_permute(s, op->g->N, op->g->d_i2c, yi, (c128*)y, 0);
    } else {
        CHECK(w.alloc(&X, (size_t)n * kGroup, "apply block"));
        CHECK(w.alloc(&Y, (size_t)n * kGroup, "apply block"));
        c128** dcols;
        CHECK(w.alloc(&dcols, 2 * kGroup, "column pointers"));
        std::vector<c128*> hc(2 * kGroup);
        for (int r0 = 0; r0 < nrhs; r0 += kGroup) {
            const int cnt = std::min(kGroup, nrhs - r0);
            if (cnt == 1) {
                launch_permute(s, op->g->N, op->g->d_i2c, (const c128*)x + r0 * ldx, xi, 1);
                apply_one(op, s, pw, xi, nullptr, yi, nullptr, lo);
                launch_permute(s, op->g->N, op->g->d_i2c, yi, (c128*)y + r0 * ldy, 0);
                continue;
            }
            const int nr = round_nr(cnt);
            for (int a = 0; a < cnt; ++a) {
                launch_permute(s, op->g->N, op->g->d_i2c, (const c128*)x + (r0 + a) * ldx, xi + (size_t)a * n, 1);
                hc[a] = xi + (size_t)a * n;
                hc[kGroup + a] = yi + (size_t)a * n;
            }
            CHECK(hip_check(ctx, hipMemcpyAsync(dcols, hc.data(), sizeof(void*) * 2 * kGroup, hipMemcpyHostToDevice, s), "cols"));
            CHECK(hip_check(ctx, hipStreamSynchronize(s), "cols"));   // hc is reused next pass
            launch_interleave(s, nr, n, (const c128* const*)dcols, X, cnt);
            apply_multi(op, s, pw, nr, X, nullptr, Y, nullptr, lo);
            launch_deinterleave(s, nr, n, Y, dcols + kGroup, cnt);
            for (int a = 0; a < cnt; ++a)
                launch_permute(s, op->g->N, op->g->d_i2c, yi + (size_t)a * n, (c128*)y + (r0 + a) * ldy, 0);
        }
    }
    CHECK(hip_check(ctx, hipGetLastError(), "apply launch"));
    return hip_check(ctx, hipStreamSynchronize(s), "apply");
}

qrvie_status qrvie_op_profile_apply(qrvie_ctx* ctx, const qrvie_op* op, int32_t prec, int32_t reps, double* ms,
                                    int64_t* bytes) {
    if (!ctx || !op || reps < 1 || !ms || !bytes) return QRVIE_ERR_INVALID_ARG;
    if (!((prec == QRVIE_PREC_C128 && op->d_fac) || (prec == QRVIE_PREC_C64 && op->d_fac32))) {
        set_err(ctx, "profile: the operator holds no far factors of the requested precision");
        return QRVIE_ERR_INVALID_ARG;
    }
    const bool lo = prec == QRVIE_PREC_C64;
    const qrvie_geom* g = op->g;
    const int64_t n = g->ndof();
    hipStream_t s = ctx->stream;
    Work w(ctx);
    ProdWork pw;
    CHECK(pw.init(w, op, 1));
    c128 *xi, *yi;
    CHECK(w.alloc(&xi, n, "profile x"));
    CHECK(w.alloc(&yi, n, "profile y"));
    CHECK(hip_check(ctx, hipMemsetAsync(xi, 0, sizeof(c128) * n, s), "profile x"));
    // Each stage is timed over `reps` back-to-back launches of its own kernel (its average
    // launch duration, as a kernel trace reports it), after one whole product has filled the
    // intermediate vectors; the whole product is timed over `reps` products.
    auto qt = [&]() {
        if (!op->shared) return;
        if (lo) launch_qtphase(s, op->d_qt, op->n_qt, op->d_fac32, xi, pw.S);
        else launch_qtphase(s, op->d_qt, op->n_qt, op->d_fac, xi, pw.S);
    };
    auto rp = [&]() {
        for (const auto& L : op->rlaunch) {
            if (op->shared) {
                if (lo) launch_rphase_sh(s, op->d_rstrips, L.count, op->d_fac32, xi, pw.T, op->d_tmap, pw.S, pw.P);
                else launch_rphase_sh(s, op->d_rstrips, L.count, op->d_fac, xi, pw.T, op->d_tmap, pw.S, pw.P);
            } else if (lo) {
                launch_rphase_c64(s, op->d_rstrips + L.begin, L.count, op->d_fac32, xi, pw.T, op->d_tmap);
            } else {
                launch_rphase(s, op->d_rstrips + L.begin, L.count, L.waves, op->d_fac, xi, pw.T, op->d_tmap);
            }
        }
    };
    auto qp = [&]() {
        for (const auto& L : op->qlaunch) {
            if (op->shared) {
                if (lo) launch_qphase_sh(s, op->d_qstrips, L.count, op->d_fac32, pw.T, pw.P, pw.Y);
                else launch_qphase_sh(s, op->d_qstrips, L.count, op->d_fac, pw.T, pw.P, pw.Y);
            } else if (lo) {
                launch_qphase_c64(s, op->d_qstrips + L.begin, L.count, op->d_fac32, pw.T, pw.Y);
            } else {
                launch_qphase(s, op->d_qstrips + L.begin, L.count, L.waves, op->d_fac, pw.T, pw.Y);
            }
        }
    };
    auto fin = [&]() {
        launch_final(s, g->N, g->d_ptype, op->d_self, nullptr, xi, pw.Y, op->n_active, n, nullptr, yi, nullptr);
    };
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    double acc[5] = {0, 0, 0, 0, 0};   // Q^T, R, Q, final, product
    auto timed = [&](int k, auto&& fn) -> qrvie_status {
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < reps; ++r) fn();
        (void)hipEventRecord(e1, s);
        CHECK(hip_check(ctx, hipEventSynchronize(e1), "profile"));
        float t = 0.f;
        (void)hipEventElapsedTime(&t, e0, e1);
        acc[k] = t;
        return QRVIE_OK;
    };
    qt(); rp(); qp(); fin();
    qrvie_status pst = QRVIE_OK;
    if (op->shared) pst = timed(0, qt);
    if (pst == QRVIE_OK) pst = timed(1, rp);
    if (pst == QRVIE_OK) pst = timed(2, qp);
    if (pst == QRVIE_OK) pst = timed(3, fin);
    if (pst == QRVIE_OK) pst = timed(4, [&]() { qt(); rp(); qp(); fin(); });
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (pst != QRVIE_OK) return pst;
    ms[0] = acc[1] / reps;
    ms[1] = acc[2] / reps;
    ms[2] = acc[3] / reps;
    ms[3] = acc[4] / reps;
    ms[4] = acc[0] / reps;
    ms[5] = 0.0;
    // bytes: [0] R pass, [1] Q pass, [2] final, [3] whole product, [4] Q^T pass (shared), [5] 0
    int64_t rn = 0, mr = 0, sr = 0;
    for (size_t b = 0; b < op->blocks.size(); ++b) {
        if (op->shared && !op->blocks[b].primary) continue;
        const int64_t r = op->rank[b];
        rn += r * op->blocks[b].cn * (int64_t)kNp;
        mr += r * op->blocks[b].rn * (int64_t)kNp;
        sr += r;
    }
    const int64_t cb = (int64_t)sizeof(c128), fb = lo ? (int64_t)sizeof(float2) : cb;
    if (op->shared) {
        bytes[4] = fb * mr + cb * (n + sr);            // Q, x; writes s
        bytes[0] = fb * rn + cb * 2 * sr;              // R; reads s, writes t (x counted once, by pass 1)
        bytes[1] = fb * mr + cb * sr;                  // Q, t
    } else {
        bytes[4] = 0;
        bytes[0] = fb * rn + cb * (sr + n);
        bytes[1] = fb * mr + cb * sr;
    }
    bytes[2] = cb * ((int64_t)op->ntypes * kNp * kNp + n);
    bytes[3] = bytes[0] + bytes[1] + bytes[2] + bytes[4];
    bytes[5] = 0;
    return hip_check(ctx, hipGetLastError(), "profile");
}

qrvie_status qrvie_op_profile_block(qrvie_ctx* ctx, const qrvie_op* op, int32_t nrhs, int32_t reps, double* ms,
                                    int64_t* flops) {
    if (!ctx || !op || reps < 1 || nrhs < 1 || nrhs > kMaxBlockRhs || !ms || !flops || op->shared)
        return QRVIE_ERR_INVALID_ARG;
    return profile_block(ctx, op, nrhs, reps, ms, flops);
}

qrvie_status qrvie_probe_read(qrvie_ctx* ctx, const void* d, size_t bytes, int32_t reps, double* gbs) {
    if (!ctx || !d || !gbs || bytes < 16 || bytes % 16 != 0 || reps < 1 || reps > 100) return QRVIE_ERR_INVALID_ARG;
    hipStream_t s = ctx->stream;
    Work w(ctx);
    double* out;
    CHECK(w.alloc(&out, 1, "probe"));
    hipEvent_t e0, e1;
    CHECK(hip_check(ctx, hipEventCreate(&e0), "probe events"));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_check(ctx, hipErrorOutOfMemory, "probe events");
    }
    const int64_t n = (int64_t)(bytes / 16);
    double best = 0.0;
    qrvie_status st = QRVIE_OK;
    for (int grid : {2048, 8192, 16384})
        for (int u : {8, 16}) {
            if (st != QRVIE_OK) break;
            launch_read_probe(s, (const c128*)d, n, grid, u, out);
            (void)hipEventRecord(e0, s);
            for (int r = 0; r < reps; ++r) launch_read_probe(s, (const c128*)d, n, grid, u, out);
            (void)hipEventRecord(e1, s);
            st = hip_check(ctx, hipEventSynchronize(e1), "probe");
            float ms = 0.f;
            if (st == QRVIE_OK) st = hip_check(ctx, hipEventElapsedTime(&ms, e0, e1), "probe timer");
            if (st == QRVIE_OK && ms > 0.f) best = std::max(best, (double)bytes * reps / (ms * 1e-3) / 1e9);
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    CHECK(st);
    *gbs = best;
    return hip_check(ctx, hipGetLastError(), "probe");
}

qrvie_status qrvie_probe_mfma(qrvie_ctx* ctx, int32_t f64, double* tfs) {
    if (!ctx || !tfs || (f64 != 0 && f64 != 1)) return QRVIE_ERR_INVALID_ARG;
    hipStream_t s = ctx->stream;
    Work w(ctx);
    double* out;
    CHECK(w.alloc(&out, 1, "probe"));
    hipEvent_t e0, e1;
    CHECK(hip_check(ctx, hipEventCreate(&e0), "probe events"));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_check(ctx, hipErrorOutOfMemory, "probe events");
    }
    constexpr int kGrid = 256 * 16, kIters = 4096;
    launch_mfma_probe(s, f64 != 0, kGrid, 64, out);
    (void)hipEventRecord(e0, s);
    launch_mfma_probe(s, f64 != 0, kGrid, kIters, out);
    (void)hipEventRecord(e1, s);
    qrvie_status st = hip_check(ctx, hipEventSynchronize(e1), "probe");
    float ms = 0.f;
    if (st == QRVIE_OK) st = hip_check(ctx, hipEventElapsedTime(&ms, e0, e1), "probe timer");
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    CHECK(st);
    const double flops = (double)kGrid * 4 /* waves */ * kIters * 8 /* chains */ * 2048.0;
    *tfs = ms > 0.f ? flops / (ms * 1e-3) / 1e12 : 0.0;
    return hip_check(ctx, hipGetLastError(), "probe");
}

qrvie_status qrvie_op_tune_block(qrvie_ctx* ctx, qrvie_op* op, int32_t prec, int32_t nrhs, int32_t reps,
                                 qrvie_block_tune* out) {
    if (!ctx || !op || !out || reps < 1 || reps > 100 || nrhs < 1 || nrhs > kMaxBlockRhs) return QRVIE_ERR_INVALID_ARG;
    if (prec != QRVIE_PREC_C128 && prec != QRVIE_PREC_C64) return QRVIE_ERR_INVALID_ARG;
    if (prec == QRVIE_PREC_C64 && !op->d_fac32) {
        set_err(ctx, "qrvie_op_tune_block: the operator holds no complex64 panels");
        return QRVIE_ERR_INVALID_ARG;
    }
    if (op->shared) {
        set_err(ctx, "qrvie_op_tune_block: the block products need an operator built without share_transpose");
        return QRVIE_ERR_INVALID_ARG;
    }
    return tune_block(ctx, op, prec, nrhs, reps, out);
}

qrvie_status qrvie_precondition(qrvie_ctx* ctx, const qrvie_op* op, int32_t nrhs, const qrvie_c128* y, int64_t ldy,
                                qrvie_c128* z, int64_t ldz) {
    CHECK(check_vec_args(ctx, op, nrhs, y, ldy, z, ldz, "precondition"));
    const int64_t n = op->g->ndof();
    Work w(ctx);
    c128 *yi, *zi;
    CHECK(w.alloc(&yi, n, "precondition work"));
    CHECK(w.alloc(&zi, n, "precondition work"));
    for (int r = 0; r < nrhs; ++r) {
        launch_permute(ctx->stream, op->g->N, op->g->d_i2c, (const c128*)y + r * ldy, yi, 1);
        launch_block_apply(ctx->stream, op->g->N, op->g->d_ptype, op->d_pinv, yi, zi);
        launch_permute(ctx->stream, op->g->N, op->g->d_i2c, zi, (c128*)z + r * ldz, 0);
    }
    CHECK(hip_check(ctx, hipGetLastError(), "precondition launch"));
    return hip_check(ctx, hipStreamSynchronize(ctx->stream), "precondition");
}

qrvie_status qrvie_op_export_block(const qrvie_op* op, int64_t b, qrvie_block_info* info, qrvie_c128* Q,
                                   qrvie_c128* R) {
    if (!op || b < 0 || b >= (int64_t)op->rank.size()) return QRVIE_ERR_INVALID_ARG;
    qrvie_ctx* ctx = op->ctx;
    const int r = op->rank[b];
    const BlockRec& e = op->blocks[b];
    const int64_t m = (int64_t)e.rn * kNp, n = (int64_t)e.cn * kNp;
    if (info) {
        info->level = e.level;
        info->m = (int32_t)m;
        info->n = (int32_t)n;
        info->rank = r;
        info->row_first = e.r0; info->row_count = e.rn;
        info->col_first = e.c0; info->col_count = e.cn;
        info->rel_err = op->relerr[b];
    }
    if (op->shared && !e.primary && (Q || R) && r > 0) {
        // shared factors: the mirror's Q is the compressed block's R^T and its R that block's Q^T
        std::vector<qrvie_c128> pq((size_t)n * r), pr((size_t)r * m);
        CHECK(qrvie_op_export_block(op, e.mirror, nullptr, pq.data(), pr.data()));
        if (Q)
            for (int64_t i = 0; i < m; ++i)
                for (int k = 0; k < r; ++k) Q[i + (int64_t)k * m] = pr[k + i * r];
        if (R)
            for (int64_t j = 0; j < n; ++j)
                for (int k = 0; k < r; ++k) R[k + j * r] = pq[j + (int64_t)k * n];
        return QRVIE_OK;
    }
    if (!op->d_fac && (Q || R) && r > 0) {
        // complex64 panels: copy down, widen on the host
        std::vector<float2> tq(Q ? (size_t)m * r : 0), tr(R ? (size_t)r * n : 0);
        if (Q) CHECK(hip_check(ctx, hipMemcpyAsync(tq.data(), op->d_fac32 + op->q_off[b], sizeof(float2) * m * r,
                                                   hipMemcpyDeviceToHost, ctx->stream), "export Q"));
        if (R) CHECK(hip_check(ctx, hipMemcpy2DAsync(tr.data(), sizeof(float2) * r, op->d_fac32 + op->r_off[b],
                                                     sizeof(float2) * op->r_ld[b], sizeof(float2) * r, (size_t)n,
                                                     hipMemcpyDeviceToHost, ctx->stream), "export R"));
        CHECK(hip_check(ctx, hipStreamSynchronize(ctx->stream), "export"));
        for (size_t i = 0; i < tq.size(); ++i) Q[i] = qrvie_c128{(double)tq[i].x, (double)tq[i].y};
        for (size_t i = 0; i < tr.size(); ++i) R[i] = qrvie_c128{(double)tr[i].x, (double)tr[i].y};
        return QRVIE_OK;
    }
    if (Q && r > 0)
        CHECK(hip_check(ctx, hipMemcpyAsync(Q, op->d_fac + op->q_off[b], sizeof(c128) * m * r, hipMemcpyDeviceToHost,
                                            ctx->stream), "export Q"));
    if (R && r > 0)
        CHECK(hip_check(ctx, hipMemcpy2DAsync(R, sizeof(c128) * r, op->d_fac + op->r_off[b], sizeof(c128) * op->r_ld[b],
                                              sizeof(c128) * r, (size_t)n, hipMemcpyDeviceToHost, ctx->stream),
                        "export R"));
    return hip_check(ctx, hipStreamSynchronize(ctx->stream), "export");
}

qrvie_status qrvie_op_export_self(const qrvie_op* op, int32_t p, qrvie_c128* Zpp, qrvie_c128* Zinv) {
    if (!op || p < 0 || p >= op->g->N) return QRVIE_ERR_INVALID_ARG;
    qrvie_ctx* ctx = op->ctx;
    const int t = op->g->ptype[op->g->c2i[p]];
    const size_t bytes = sizeof(c128) * kNp * kNp;
    if (Zpp) CHECK(hip_check(ctx, hipMemcpyAsync(Zpp, op->d_self + (size_t)t * kNp * kNp, bytes, hipMemcpyDeviceToHost, ctx->stream), "export self"));
    if (Zinv) CHECK(hip_check(ctx, hipMemcpyAsync(Zinv, op->d_pinv + (size_t)t * kNp * kNp, bytes, hipMemcpyDeviceToHost, ctx->stream), "export inverse"));
    return hip_check(ctx, hipStreamSynchronize(ctx->stream), "export self");
}

qrvie_status qrvie_solve_footprint_estimate(const qrvie_geom* g, const qrvie_op* op, int32_t nrhs,
                                            const qrvie_solve_opts* o, size_t* bytes) {
    if (!g || !o || !bytes || nrhs < 1 || o->restart < 1 || o->max_iter < 1) return QRVIE_ERR_INVALID_ARG;
    const int64_t n = g->ndof();
    const int64_t m = std::min(o->restart, o->max_iter);
    const int64_t na = std::min(nrhs, kGroup);
    const int64_t nr = na > 1 ? round_nr((int)na) : 1;
    const int64_t nch = krylov_nchunks(n), nblk = krylov_nblocks(n);
    // per column: basis, six vectors, Hessenberg and Gram matrices, partials
    const int64_t col = n * (m + 1) + (o->mode == QRVIE_SOLVE_MIXED_IR ? 8 : 6) * n + (m + 1) * m + (m + 1) * (m + 1) +
                        4 * (m + 2) + 2 * nch * (m + 1) + krylov_nchunks(m + 1) * (m + 1) + nch + nblk;
    // product workspace: rank-space block (sum of ranks <= 2 x 64 per block side when unknown) and level partials
    const int64_t tlen = op ? op->t_len : (int64_t)g->blocks.size() * 64;
    const int64_t nlev = op ? std::max(op->n_active, 1) : std::max(g->L, 1);
    const int64_t prod = tlen * nr + nlev * n * nr + (na > 1 ? 2 * n * nr : 0);
    int64_t elems = na * col + prod;
    if (o->mode == QRVIE_SOLVE_BLOCK || o->mode == QRVIE_SOLVE_BLOCK_IR) {
        // one block of up to block_width right-hand sides at a time (the BlockSolver buffers,
        // the block product workspace, which is sized for 64 right-hand sides, and the split-K
        // partials); a rank-deficient block is finished by the single-vector solver with the
        // same total number of basis vectors, so the larger of the two is the peak
        const int64_t width = o->block_width > 0 ? o->block_width : kMaxBlockRhs;
        const int64_t pb = std::min<int64_t>(nrhs, width), P = 16 * ((pb + 15) / 16);
        const int64_t ldh = (std::max<int64_t>(1, std::min<int64_t>(o->restart / pb, o->max_iter)) + 1) * pb;
        const int64_t blk = n * (5 * pb + ldh + 4 * P) + ldh * (8 * pb + 2 * ldh) + 3 * pb * pb + kBlockPartialElems +
                            tlen * kMaxBlockRhs + (nlev + 1) * n * kMaxBlockRhs;
        qrvie_solve_opts o1 = *o;
        o1.mode = QRVIE_SOLVE_FP64;
        o1.restart = block_fallback_restart(o->restart, (int)pb);
        size_t fb = 0;
        CHECK(qrvie_solve_footprint_estimate(g, op, (int32_t)pb, &o1, &fb));
        elems = std::max<int64_t>(blk, (int64_t)(fb / sizeof(c128)));
        if (o->mode == QRVIE_SOLVE_BLOCK_IR) elems += 3 * n * (int64_t)nrhs;   // residuals, their copy, corrections
    }
    *bytes = (size_t)(elems * (int64_t)sizeof(c128)) + (size_t)(1 << 20);
    return QRVIE_OK;
}

qrvie_status qrvie_solve(qrvie_ctx* ctx, const qrvie_op* op, int32_t nrhs, const qrvie_c128* v, int64_t ldv,
                         qrvie_c128* x, int64_t ldx, const qrvie_solve_opts* o, qrvie_solve_info* info) {
    CHECK(check_vec_args(ctx, op, nrhs, v, ldv, x, ldx, "solve"));
    if (!o || o->restart < 1 || o->restart > 16384 || o->max_iter < 1 || !(o->tol > 0.0) ||
        (o->mode != QRVIE_SOLVE_FP64 && o->mode != QRVIE_SOLVE_MIXED_IR && o->mode != QRVIE_SOLVE_BLOCK &&
         o->mode != QRVIE_SOLVE_BLOCK_IR) ||
        !(o->inner_tol >= 0.0 && o->inner_tol < 1.0) || o->block_width < 0 || o->block_width > kMaxBlockRhs ||
        (o->inner_fp32 != 0 && o->inner_fp32 != 1)) {
        set_err(ctx, "solve: invalid options");
        return QRVIE_ERR_INVALID_ARG;
    }
    if (o->mode == QRVIE_SOLVE_MIXED_IR && !(op->d_fac32 && op->d_fac)) {
        set_err(ctx, "solve: mixed-precision refinement needs an operator built with far_prec = QRVIE_PREC_C64");
        return QRVIE_ERR_INVALID_ARG;
    }
    if (o->mode == QRVIE_SOLVE_BLOCK_IR && !op->d_fac32) {
        set_err(ctx, "solve: block refinement needs complex64 factors (far_prec C64, C64_ONLY or BF16X2)");
        return QRVIE_ERR_INVALID_ARG;
    }
    if (o->mode == QRVIE_SOLVE_BLOCK_IR && !op->d_fac && !op->d_fac16 && !o->inner_fp32) {
        set_err(ctx, "solve: block refinement on complex64-only factors needs inner_fp32 = 1 (the corrections "
                     "would otherwise use the residual operator itself)");
        return QRVIE_ERR_INVALID_ARG;
    }
    if (o->mode == QRVIE_SOLVE_BLOCK_IR) return solve_block_ir(ctx, op, nrhs, (const c128*)v, ldv, (c128*)x, ldx, o, info);
    qrvie_status overall = QRVIE_OK;
    if (o->mode == QRVIE_SOLVE_BLOCK) {
        const int width = o->block_width > 0 ? o->block_width : kMaxBlockRhs;
        for (int r0 = 0; r0 < nrhs; r0 += width) {
            const int cnt = std::min(width, nrhs - r0);
            bool broke = false;
            qrvie_solve_info* inf = info ? info + r0 : nullptr;
            if (cnt == 1) {
                // a block of one column spans the same Krylov space as GMRES, whose HBM-bound
                // single-vector kernels are faster (1729 steps at mid: 6.7 s against 12.5 s)
                qrvie_solve_opts o1 = *o;
                o1.mode = QRVIE_SOLVE_FP64;
                const qrvie_status st = qrvie_solve(ctx, op, 1, (const qrvie_c128*)((const c128*)v + (int64_t)r0 * ldv),
                                                    ldv, (qrvie_c128*)((c128*)x + (int64_t)r0 * ldx), ldx, &o1, inf);
                if (st == QRVIE_NOT_CONVERGED) overall = st;
                else if (st != QRVIE_OK) return st;
                continue;
            }
            qrvie_status st = solve_block(ctx, op, cnt, (const c128*)v + (int64_t)r0 * ldv, ldv,
                                          (c128*)x + (int64_t)r0 * ldx, ldx, o, inf, &broke);
            if (broke) {
                // rank-deficient block (e.g. repeated right-hand sides): finish each column with
                // the single-vector solver, starting from the block iterate
                qrvie_solve_opts o1 = *o;
                o1.mode = QRVIE_SOLVE_FP64;
                o1.use_x0 = 1;
                o1.restart = block_fallback_restart(o->restart, cnt);   // the block path's basis budget
                st = qrvie_solve(ctx, op, cnt, (const qrvie_c128*)((const c128*)v + (int64_t)r0 * ldv), ldv,
                                 (qrvie_c128*)((c128*)x + (int64_t)r0 * ldx), ldx, &o1, inf);
            }
            if (st == QRVIE_NOT_CONVERGED) overall = st;
            else if (st != QRVIE_OK) return st;
        }
        return overall;
    }
    for (int r0 = 0; r0 < nrhs; r0 += kGroup) {
        const int cnt = std::min(kGroup, nrhs - r0);
        std::vector<const c128*> vv(cnt);
        std::vector<c128*> xx(cnt);
        for (int a = 0; a < cnt; ++a) {
            vv[a] = (const c128*)v + (r0 + a) * ldv;
            xx[a] = (c128*)x + (r0 + a) * ldx;
        }
        qrvie_solve_info* inf = info ? info + r0 : nullptr;
        const qrvie_status st = o->mode == QRVIE_SOLVE_MIXED_IR
                                    ? solve_group_ir(ctx, op, cnt, vv.data(), xx.data(), o, inf)
                                    : solve_group(ctx, op, cnt, vv.data(), xx.data(), o, inf);
        if (st == QRVIE_NOT_CONVERGED) overall = st;
        else if (st != QRVIE_OK) return st;
    }
    return overall;
}

}  // extern "C"
