// Product, preconditioner, factor export and the GMRES driver (host side).
//
// The solve is the paper's left-preconditioned GMRES (§6, with Z_D^-1 of §4):
// restarted GMRES(m), x0 = 0 unless given; every Arnoldi step costs one fused
// "product + preconditioner" pass, two classical Gram-Schmidt passes (multi-dot and
// multi-axpy kernels), a norm and a device-side Givens update.  The host reads two
// numbers per step (residual estimate and h_{j+1,j}) to decide convergence.  A column
// is converged when the preconditioned estimate is <= tol ||Z_D^-1 v|| and the true
// residual ||v - Z_QR x|| / ||v|| <= tol; if only the first holds the solver restarts
// with a tightened internal tolerance.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "internal.h"

using namespace qrvie;

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// y_int = Z_QR x_int (out_r), optionally r = v - Z x and z = Z_D^-1 r (internal order).
void apply_internal(const qrvie_op* op, hipStream_t s, const c128* x, const c128* v, c128* out_r, c128* out_z) {
    const qrvie_geom* g = op->g;
    for (const auto& L : op->rlaunch)
        launch_rphase(s, op->d_rstrips + L.begin, L.count, L.waves, op->d_fac, x, op->d_t, op->d_tmap);
    for (const auto& L : op->qlaunch)
        launch_qphase(s, op->d_qstrips + L.begin, L.count, L.waves, op->d_fac, op->d_t, op->d_ylev);
    launch_final(s, g->N, g->d_ptype, op->d_self, out_z ? op->d_pinv : nullptr, x, op->d_ylev, op->n_active,
                 g->ndof(), v, out_r, out_z);
}

struct Work {
    qrvie_ctx* ctx;
    std::vector<std::pair<void*, size_t>> bufs;
    explicit Work(qrvie_ctx* c) : ctx(c) {}
    ~Work() {
        (void)hipStreamSynchronize(ctx->stream);
        for (auto& b : bufs) dfree(ctx, b.first, b.second);
    }
    template <class T>
    qrvie_status alloc(T** p, size_t count, const char* what) {
        *p = nullptr;
        qrvie_status st = dalloc(ctx, (void**)p, sizeof(T) * std::max<size_t>(count, 1), what);
        if (st == QRVIE_OK) bufs.push_back({(void*)*p, sizeof(T) * std::max<size_t>(count, 1)});
        return st;
    }
};

#define CHECK(x)                       \
    do {                               \
        qrvie_status _s = (x);         \
        if (_s != QRVIE_OK) return _s; \
    } while (0)

qrvie_status check_vec_args(qrvie_ctx* ctx, const qrvie_op* op, int32_t nrhs, const void* a, int64_t lda, const void* b,
                            int64_t ldb, const char* what) {
    if (!ctx || !op || !a || !b || nrhs < 1 || lda < op->g->ndof() || ldb < op->g->ndof()) {
        if (ctx) set_err(ctx, std::string(what) + ": invalid argument");
        return QRVIE_ERR_INVALID_ARG;
    }
    return QRVIE_OK;
}

}  // namespace

extern "C" {

qrvie_status qrvie_apply(qrvie_ctx* ctx, const qrvie_op* op, int32_t nrhs, const qrvie_c128* x, int64_t ldx,
                         qrvie_c128* y, int64_t ldy) {
    CHECK(check_vec_args(ctx, op, nrhs, x, ldx, y, ldy, "apply"));
    const int64_t n = op->g->ndof();
    Work w(ctx);
    c128 *xi, *yi;
    CHECK(w.alloc(&xi, n, "apply work"));
    CHECK(w.alloc(&yi, n, "apply work"));
    for (int r = 0; r < nrhs; ++r) {
        launch_permute(ctx->stream, op->g->N, op->g->d_i2c, (const c128*)x + r * ldx, xi, 1);
        apply_internal(op, ctx->stream, xi, nullptr, yi, nullptr);
        launch_permute(ctx->stream, op->g->N, op->g->d_i2c, yi, (c128*)y + r * ldy, 0);
    }
    CHECK(hip_check(ctx, hipGetLastError(), "apply launch"));
    return hip_check(ctx, hipStreamSynchronize(ctx->stream), "apply");
}

qrvie_status qrvie_op_profile_apply(qrvie_ctx* ctx, const qrvie_op* op, int32_t reps, double* ms, int64_t* bytes) {
    if (!ctx || !op || reps < 1 || !ms || !bytes) return QRVIE_ERR_INVALID_ARG;
    const qrvie_geom* g = op->g;
    const int64_t n = g->ndof();
    hipStream_t s = ctx->stream;
    Work w(ctx);
    c128 *xi, *yi;
    CHECK(w.alloc(&xi, n, "profile x"));
    CHECK(w.alloc(&yi, n, "profile y"));
    CHECK(hip_check(ctx, hipMemsetAsync(xi, 0, sizeof(c128) * n, s), "profile x"));
    hipEvent_t ev[4];
    for (auto& e : ev) (void)hipEventCreate(&e);
    double acc[4] = {0, 0, 0, 0};
    for (int r = 0; r < reps; ++r) {
        (void)hipEventRecord(ev[0], s);
        for (const auto& L : op->rlaunch)
            launch_rphase(s, op->d_rstrips + L.begin, L.count, L.waves, op->d_fac, xi, op->d_t, op->d_tmap);
        (void)hipEventRecord(ev[1], s);
        for (const auto& L : op->qlaunch)
            launch_qphase(s, op->d_qstrips + L.begin, L.count, L.waves, op->d_fac, op->d_t, op->d_ylev);
        (void)hipEventRecord(ev[2], s);
        launch_final(s, g->N, g->d_ptype, op->d_self, nullptr, xi, op->d_ylev, op->n_active, n, nullptr, yi, nullptr);
        (void)hipEventRecord(ev[3], s);
        CHECK(hip_check(ctx, hipEventSynchronize(ev[3]), "profile"));
        float t = 0.f;
        for (int k = 0; k < 3; ++k) {
            (void)hipEventElapsedTime(&t, ev[k], ev[k + 1]);
            acc[k] += t;
        }
        (void)hipEventElapsedTime(&t, ev[0], ev[3]);
        acc[3] += t;
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    for (int k = 0; k < 4; ++k) ms[k] = acc[k] / reps;
    int64_t rn = 0, mr = 0, sr = 0;
    for (size_t b = 0; b < op->blocks.size(); ++b) {
        const int64_t r = op->rank[b];
        rn += r * op->blocks[b].cn * (int64_t)kNp;
        mr += r * op->blocks[b].rn * (int64_t)kNp;
        sr += r;
    }
    const int64_t cb = (int64_t)sizeof(c128);
    bytes[0] = cb * (rn + sr + n);
    bytes[1] = cb * (mr + sr);
    bytes[2] = cb * ((int64_t)op->ntypes * kNp * kNp + n);
    bytes[3] = bytes[0] + bytes[1] + bytes[2];
    return hip_check(ctx, hipGetLastError(), "profile");
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
    // recover the block geometry from the panel bookkeeping
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

qrvie_status qrvie_solve(qrvie_ctx* ctx, const qrvie_op* op, int32_t nrhs, const qrvie_c128* v, int64_t ldv,
                         qrvie_c128* x, int64_t ldx, const qrvie_solve_opts* o, qrvie_solve_info* info) {
    CHECK(check_vec_args(ctx, op, nrhs, v, ldv, x, ldx, "solve"));
    if (!o || o->restart < 1 || o->restart > 16384 || o->max_iter < 1 || !(o->tol > 0.0) || o->mode != QRVIE_SOLVE_FP64) {
        set_err(ctx, "solve: invalid options");
        return QRVIE_ERR_INVALID_ARG;
    }
    hipStream_t s = ctx->stream;
    const qrvie_geom* g = op->g;
    const int64_t n = g->ndof();
    const int m = o->restart;
    const int nch = krylov_nchunks(n);
    Work w(ctx);
    c128 *V, *wv, *xi, *vi, *r, *pd, *h, *H, *sn, *gv, *y;
    double *np, *nrm, *cs, *status;
    CHECK(w.alloc(&V, (size_t)n * (m + 1), "krylov basis"));
    CHECK(w.alloc(&wv, n, "krylov w"));
    CHECK(w.alloc(&xi, n, "solve x"));
    c128* xc;
    CHECK(w.alloc(&xc, n, "solve candidate x"));
    CHECK(w.alloc(&vi, n, "solve v"));
    CHECK(w.alloc(&r, n, "solve r"));
    CHECK(w.alloc(&pd, (size_t)nch * (m + 1), "dot partials"));
    CHECK(w.alloc(&np, nch, "norm partials"));
    CHECK(w.alloc(&nrm, 4, "norms"));
    CHECK(w.alloc(&h, m + 2, "hessenberg column"));
    CHECK(w.alloc(&H, (size_t)(m + 1) * m, "hessenberg"));
    CHECK(w.alloc(&cs, m, "givens c"));
    CHECK(w.alloc(&sn, m, "givens s"));
    CHECK(w.alloc(&gv, m + 1, "givens rhs"));
    CHECK(w.alloc(&y, m, "lsq solution"));
    CHECK(w.alloc(&status, 2, "status"));
    double* hstat = nullptr;
    CHECK(hip_check(ctx, hipHostMalloc((void**)&hstat, 4 * sizeof(double), hipHostMallocDefault), "pinned status"));
    struct PinnedFree { double* p; ~PinnedFree() { if (p) (void)hipHostFree(p); } } pf{hstat};

    const int nblk = krylov_nblocks(n);
    double* bp;
    int* gate;
    CHECK(w.alloc(&bp, nblk, "update norm partials"));
    CHECK(w.alloc(&gate, 2, "reorthogonalisation gate"));
    auto norm_to = [&](const c128* vec, double* dst) {
        launch_norm2(s, vec, n, np);
        launch_reduce_norm(s, np, nch, dst, nullptr);
    };
    auto read = [&](const double* d, int cnt) -> qrvie_status {
        CHECK(hip_check(ctx, hipMemcpyAsync(hstat, d, sizeof(double) * cnt, hipMemcpyDeviceToHost, s), "read"));
        return hip_check(ctx, hipStreamSynchronize(s), "sync");
    };

    qrvie_status overall = QRVIE_OK;
    hipEvent_t ev0, ev1;
    (void)hipEventCreate(&ev0);
    (void)hipEventCreate(&ev1);
    for (int rhs = 0; rhs < nrhs; ++rhs) {
        const double t0 = now_s();
        qrvie_solve_info inf{};
        double t_apply = 0.0, t_kry = 0.0;
        launch_permute(s, g->N, g->d_i2c, (const c128*)v + rhs * ldv, vi, 1);
        if (o->use_x0) launch_permute(s, g->N, g->d_i2c, (const c128*)x + rhs * ldx, xi, 1);
        else CHECK(hip_check(ctx, hipMemsetAsync(xi, 0, sizeof(c128) * n, s), "x0"));
        // ||v|| and ||Z_D^-1 v||
        norm_to(vi, nrm + 0);
        launch_block_apply(s, g->N, g->d_ptype, op->d_pinv, vi, r);
        norm_to(r, nrm + 1);
        CHECK(read(nrm, 2));
        const double vnorm = std::sqrt(hstat[0]), pvnorm = std::sqrt(hstat[1]);
        if (!(std::isfinite(vnorm))) {
            set_err(ctx, "solve: right-hand side has non-finite entries");
            return QRVIE_ERR_INVALID_ARG;
        }
        if (vnorm == 0.0) {
            CHECK(hip_check(ctx, hipMemsetAsync((c128*)x + rhs * ldx, 0, sizeof(c128) * n, s), "zero x"));
            inf.converged = 1;
            if (info) info[rhs] = inf;
            continue;
        }
        CHECK(hip_check(ctx, hipMemsetAsync(gate, 0, 2 * sizeof(int), s), "gate"));
        double prec_tol = o->tol;
        int iters = 0;
        bool converged = false;
        while (true) {
            // r = v - Z x (true residual), V0 = Z_D^-1 r
            (void)hipEventRecord(ev0, s);
            apply_internal(op, s, xi, vi, r, wv);
            (void)hipEventRecord(ev1, s);
            inf.n_apply++;
            inf.n_prec++;
            norm_to(r, nrm + 0);
            norm_to(wv, nrm + 1);
            CHECK(read(nrm, 2));
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, ev0, ev1);
            t_apply += ms * 1e-3;
            const double true_rel = std::sqrt(hstat[0]) / vnorm;
            const double beta = std::sqrt(hstat[1]);
            inf.rel_res_true = true_rel;
            inf.rel_res_prec = beta / pvnorm;
            if (!std::isfinite(beta)) { set_err(ctx, "solve: non-finite residual"); return QRVIE_ERR_DEVICE; }
            if (inf.rel_res_prec <= prec_tol) {
                if (true_rel <= o->tol) { converged = true; break; }
                prec_tol = std::max(prec_tol * 0.5 * o->tol / true_rel, 1e-15);
            }
            if (iters >= o->max_iter) break;
            const double tk0 = now_s();
            launch_scale_into(s, wv, n, nrm + 1, V, gv);     // V0 = w / beta, g0 = beta
            int k_used = 0;
            bool cycle_done = false;
            for (int j = 0; j < m && iters < o->max_iter && !cycle_done; ++j) {
                (void)hipEventRecord(ev0, s);
                apply_internal(op, s, V + (size_t)j * n, nullptr, nullptr, wv);   // w = Z_D^-1 Z v_j
                (void)hipEventRecord(ev1, s);
                inf.n_apply++;
                inf.n_prec++;
                // one classical Gram-Schmidt pass with ||w|| and ||w'|| fused in
                launch_multidot(s, V, n, j + 1, wv, n, pd, np, nullptr);
                launch_reduce_dots(s, pd, nch, j + 1, h, 0, nullptr);
                launch_reduce_norm(s, np, nch, nrm + 3, nullptr);
                launch_gemv_sub(s, V, n, j + 1, h, wv, n, bp, nullptr);
                launch_reduce_norm(s, bp, nblk, nrm + 2, nullptr);
                // the second pass runs only if the gate opens (||w'||^2 < ||w||^2 / 2)
                launch_reorth_gate(s, nrm + 2, nrm + 3, gate);
                launch_multidot(s, V, n, j + 1, wv, n, pd, nullptr, gate);
                launch_reduce_dots(s, pd, nch, j + 1, y, 0, gate);
                launch_reduce_dots(s, pd, nch, j + 1, h, 1, gate);
                launch_gemv_sub(s, V, n, j + 1, y, wv, n, bp, gate);
                launch_reduce_norm(s, bp, nblk, nrm + 2, gate);
                launch_givens(s, j, h, H, m + 1, cs, sn, gv, nrm + 2, status);
                launch_scale_into(s, wv, n, nrm + 2, V + (size_t)(j + 1) * n, nullptr);
                CHECK(read(status, 2));
                float ms2 = 0.f;
                (void)hipEventElapsedTime(&ms2, ev0, ev1);
                t_apply += ms2 * 1e-3;
                ++iters;
                k_used = j + 1;
                const double est = hstat[0] / pvnorm;
                const bool breakdown = hstat[1] == 0.0;
                if (est <= prec_tol || breakdown) {
                    // candidate x_c = x + V y: accept it if the true residual meets tol too;
                    // otherwise tighten the preconditioned target and keep extending this
                    // Krylov space instead of restarting
                    launch_trisolve(s, k_used, H, m + 1, gv, y);
                    CHECK(hip_check(ctx, hipMemcpyAsync(xc, xi, sizeof(c128) * n, hipMemcpyDeviceToDevice, s), "x_c"));
                    launch_gemv_add(s, V, n, k_used, y, xc, n);
                    (void)hipEventRecord(ev0, s);
                    apply_internal(op, s, xc, vi, r, nullptr);
                    (void)hipEventRecord(ev1, s);
                    inf.n_apply++;
                    norm_to(r, nrm + 0);
                    CHECK(read(nrm, 1));
                    float ms3 = 0.f;
                    (void)hipEventElapsedTime(&ms3, ev0, ev1);
                    t_apply += ms3 * 1e-3;
                    const double tr = std::sqrt(hstat[0]) / vnorm;
                    inf.rel_res_true = tr;
                    inf.rel_res_prec = est;
                    if (tr <= o->tol) {
                        CHECK(hip_check(ctx, hipMemcpyAsync(xi, xc, sizeof(c128) * n, hipMemcpyDeviceToDevice, s), "x"));
                        converged = true;
                        cycle_done = true;
                        k_used = 0;
                    } else {
                        prec_tol = std::max(prec_tol * 0.5 * o->tol / tr, 1e-15);
                        if (breakdown) cycle_done = true;
                    }
                }
            }
            if (k_used > 0) {
                launch_trisolve(s, k_used, H, m + 1, gv, y);
                launch_gemv_add(s, V, n, k_used, y, xi, n);
            }
            CHECK(hip_check(ctx, hipGetLastError(), "gmres launch"));
            inf.restarts++;
            t_kry += now_s() - tk0;
            if (converged) break;
        }
        inf.iterations = iters;
        int hgate[2] = {0, 0};
        CHECK(hip_check(ctx, hipMemcpyAsync(hgate, gate, sizeof hgate, hipMemcpyDeviceToHost, s), "gate"));
        CHECK(hip_check(ctx, hipStreamSynchronize(s), "gate"));
        inf.n_reorth = hgate[1];
        inf.converged = converged ? 1 : 0;
        launch_permute(s, g->N, g->d_i2c, xi, (c128*)x + rhs * ldx, 0);
        CHECK(hip_check(ctx, hipStreamSynchronize(s), "solve"));
        inf.t_total_s = now_s() - t0;
        inf.t_apply_s = t_apply;
        inf.t_krylov_s = std::max(0.0, t_kry - t_apply);
        inf.t_prec_s = 0.0;  // fused into the product pass
        if (info) info[rhs] = inf;
        if (!converged) overall = QRVIE_NOT_CONVERGED;
    }
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    return overall;
}

}  // extern "C"
