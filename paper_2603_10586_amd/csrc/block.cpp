// Block GMRES: up to 64 right-hand sides share one block Krylov space (the paper's
// left-preconditioned GMRES of §6 with the preconditioner of §4, in block form).
//
// With R0 = Z_D^-1 (B - Z_QR X0) = V_0 S0 (a QR factorisation), each block step multiplies
// the newest block V_k by Z_D^-1 Z_QR (the FP64 MFMA block product), orthogonalises it
// against the whole basis, and factorises what remains as V_{k+1} H_{k+1,k}.  The block
// Hessenberg least-squares problem min ||E_1 S0 - H Y|| is kept in triangular form by one
// block reflector per block column, so every step yields each right-hand side's
// preconditioned residual estimate.  When all estimates meet their targets the candidate
// X + V Y is checked against the true residuals ||B - Z_QR X|| / ||B||, exactly as in the
// single-vector solver; a failing column tightens its target and the space keeps growing.
//
// Orthogonalisation is CGS2 through the Gram matrix of the basis (as in the single-vector
// solver): C = V^H [V_k, W] in one GEMM, H = 2 H1 - G H1 with G = V^H V, W -= V H; the new
// block is factorised by Cholesky QR twice.  The basis GEMMs and triangular solves are
// plain dense BLAS (rocBLAS); the product, the Cholesky factor and the least-squares
// reflectors are this library's kernels.
#include <rocblas/rocblas.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "work.h"

namespace qrvie {

void blas_release(qrvie_ctx* ctx) {
    if (ctx->blas) {
        (void)rocblas_destroy_handle((rocblas_handle)ctx->blas);
        ctx->blas = nullptr;
    }
}

namespace {

typedef rocblas_double_complex zc;

inline const zc* Z(const c128* p) { return reinterpret_cast<const zc*>(p); }
inline zc* Z(c128* p) { return reinterpret_cast<zc*>(p); }

qrvie_status blas_check(qrvie_ctx* ctx, rocblas_status st, const char* what) {
    if (st == rocblas_status_success) return QRVIE_OK;
    set_err(ctx, std::string(what) + ": rocBLAS status " + std::to_string((int)st));
    return QRVIE_ERR_DEVICE;
}

qrvie_status blas_handle(qrvie_ctx* ctx, rocblas_handle* h) {
    if (!ctx->blas) {
        rocblas_handle hh = nullptr;
        CHECK(blas_check(ctx, rocblas_create_handle(&hh), "rocblas handle"));
        ctx->blas = hh;
    }
    *h = (rocblas_handle)ctx->blas;
    CHECK(blas_check(ctx, rocblas_set_pointer_mode(*h, rocblas_pointer_mode_host), "rocblas pointer mode"));
    return blas_check(ctx, rocblas_set_stream(*h, ctx->stream), "rocblas stream");
}

// Relative pivot floor of the Cholesky QR: a block whose Gram matrix has a pivot below
// 1e-20 of its largest diagonal entry (condition number above 1e10) counts as rank deficient.
constexpr double kCholFloor = 1e-20;

struct BlockSolver {
    qrvie_ctx* ctx;
    const qrvie_op* op;
    const qrvie_solve_opts* o;
    rocblas_handle hb = nullptr;
    hipStream_t s;
    int64_t n;
    int p = 0, nt = 0, Kc = 0;
    int64_t ldh = 0;
    Work w;
    BlockWork bw;
    c128 *Bc = nullptr, *X = nullptr, *Xc = nullptr, *Rc = nullptr, *Vb = nullptr;
    c128 *Bi = nullptr, *Xi = nullptr, *Ri = nullptr, *Zi = nullptr;
    c128 *Cb = nullptr, *Hb = nullptr, *G = nullptr, *Rl = nullptr, *gl = nullptr, *Yb = nullptr;
    c128 *Yr = nullptr, *Tr = nullptr, *S = nullptr, *R1 = nullptr, *R2 = nullptr;
    int* dflag = nullptr;
    double* dnrm = nullptr;
    double* hbuf = nullptr;   // pinned
    hipEvent_t ev0{}, ev1{};
    double t_apply = 0.0;
    int products = 0;

    BlockSolver(qrvie_ctx* c, const qrvie_op* p_, const qrvie_solve_opts* o_)
        : ctx(c), op(p_), o(o_), s(c->stream), n(p_->g->ndof()), w(c) {}
    ~BlockSolver() {
        if (hbuf) (void)hipHostFree(hbuf);
        (void)hipEventDestroy(ev0);
        (void)hipEventDestroy(ev1);
    }

    qrvie_status init(int ncols) {
        p = ncols;
        nt = (p + 15) / 16;
        Kc = std::max(1, std::min(o->restart / p, o->max_iter));
        ldh = (int64_t)(Kc + 1) * p;
        const int64_t P = 16 * nt;
        CHECK(blas_handle(ctx, &hb));
        CHECK(bw.init(w, op));
        CHECK(w.alloc(&Bc, (size_t)n * p, "block rhs"));
        CHECK(w.alloc(&X, (size_t)n * p, "block x"));
        CHECK(w.alloc(&Xc, (size_t)n * p, "block candidate"));
        CHECK(w.alloc(&Rc, (size_t)n * p, "block residual"));
        CHECK(w.alloc(&Vb, (size_t)n * ldh, "block krylov basis"));
        CHECK(w.alloc(&Bi, (size_t)n * P, "interleaved rhs"));
        CHECK(w.alloc(&Xi, (size_t)n * P, "interleaved x"));
        CHECK(w.alloc(&Ri, (size_t)n * P, "interleaved residual"));
        CHECK(w.alloc(&Zi, (size_t)n * P, "interleaved product"));
        CHECK(w.alloc(&Cb, (size_t)ldh * 2 * p, "block projections"));
        CHECK(w.alloc(&Hb, (size_t)ldh * p, "block coefficients"));
        CHECK(w.alloc(&G, (size_t)ldh * ldh, "block gram matrix"));
        CHECK(w.alloc(&Rl, (size_t)ldh * Kc * p, "block hessenberg"));
        CHECK(w.alloc(&gl, (size_t)ldh * p, "block least-squares rhs"));
        CHECK(w.alloc(&Yb, (size_t)ldh * p, "block least-squares solution"));
        CHECK(w.alloc(&Yr, (size_t)Kc * 2 * p * p, "block reflectors"));
        CHECK(w.alloc(&Tr, (size_t)Kc * p * p, "block reflector factors"));
        CHECK(w.alloc(&S, (size_t)p * p, "gram block"));
        CHECK(w.alloc(&R1, (size_t)p * p, "cholesky factor"));
        CHECK(w.alloc(&R2, (size_t)p * p, "cholesky factor"));
        CHECK(w.alloc(&dflag, 2, "cholesky flags"));
        CHECK(w.alloc(&dnrm, 2 * (size_t)p, "block norms"));
        CHECK(hip_check(ctx, hipHostMalloc((void**)&hbuf, sizeof(double) * (2 * p + 2), hipHostMallocDefault), "pinned"));
        (void)hipEventCreate(&ev0);
        (void)hipEventCreate(&ev1);
        return QRVIE_OK;
    }

    // host copy of `count` doubles (and optionally the two Cholesky flags), then sync
    qrvie_status read(const double* d, int count, bool flags, int hf[2]) {
        CHECK(hip_check(ctx, hipMemcpyAsync(hbuf, d, sizeof(double) * count, hipMemcpyDeviceToHost, s), "read"));
        if (flags)
            CHECK(hip_check(ctx, hipMemcpyAsync(hbuf + 2 * p, dflag, sizeof(int) * 2, hipMemcpyDeviceToHost, s),
                            "read"));
        CHECK(hip_check(ctx, hipStreamSynchronize(s), "sync"));
        if (flags) std::memcpy(hf, hbuf + 2 * p, sizeof(int) * 2);
        return QRVIE_OK;
    }

    // out = B - Z_QR Xcol (col-major n x p) and, optionally, zcol = Z_D^-1 out; both col-major
    void residual(const c128* Xcol, c128* out, c128* zcol) {
        launch_gather_block(s, nt, op->g->N, nullptr, Xcol, n, p, Xi);
        (void)hipEventRecord(ev0, s);
        block_product(op, s, bw, nt, Xi, Bi, Ri, zcol ? Zi : nullptr);
        (void)hipEventRecord(ev1, s);
        ++products;
        launch_scatter_block(s, nt, op->g->N, nullptr, Ri, out, n, p);
        if (zcol) launch_scatter_block(s, nt, op->g->N, nullptr, Zi, zcol, n, p);
    }
    void add_product_time() {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ev0, ev1) == hipSuccess) t_apply += ms * 1e-3;
    }

    // W (n x p, ld n) = Q R with orthonormal Q (in place) and R (p x p upper) at out;
    // Cholesky QR twice.  Returns the pivot flags of both passes through hf after a read.
    qrvie_status cholqr2(c128* Wp, c128* out, int64_t ldo) {
        const double one = 1.0, zero = 0.0;
        const zc zone = {1.0, 0.0};
        c128* Rs[2] = {R1, R2};
        for (int pass = 0; pass < 2; ++pass) {
            CHECK(blas_check(ctx, rocblas_zherk(hb, rocblas_fill_upper, rocblas_operation_conjugate_transpose, p, (int)n,
                                                &one, Z(Wp), (int)n, &zero, Z(S), p), "zherk"));
            launch_cholesky(s, p, S, p, kCholFloor, Rs[pass], p, dflag + pass);
            CHECK(blas_check(ctx, rocblas_ztrsm(hb, rocblas_side_right, rocblas_fill_upper, rocblas_operation_none,
                                                rocblas_diagonal_non_unit, (int)n, p, &zone, Z(Rs[pass]), p, Z(Wp),
                                                (int)n), "ztrsm"));
        }
        launch_trmm_upper(s, p, R2, p, R1, p, out, ldo, dflag);
        return QRVIE_OK;
    }

    // X_out = X_in + V[:, 0:(k+1)p] R^-1 gl[0:(k+1)p]
    qrvie_status update(int steps, const c128* Xin, c128* Xout) {
        const zc zone = {1.0, 0.0};
        const int64_t m = (int64_t)steps * p;
        if (Xout != Xin)
            CHECK(hip_check(ctx, hipMemcpyAsync(Xout, Xin, sizeof(c128) * n * p, hipMemcpyDeviceToDevice, s), "x"));
        if (steps == 0) return QRVIE_OK;
        CHECK(hip_check(ctx, hipMemcpy2DAsync(Yb, sizeof(c128) * ldh, gl, sizeof(c128) * ldh, sizeof(c128) * m, p,
                                              hipMemcpyDeviceToDevice, s), "y"));
        CHECK(blas_check(ctx, rocblas_ztrsm(hb, rocblas_side_left, rocblas_fill_upper, rocblas_operation_none,
                                            rocblas_diagonal_non_unit, (int)m, p, &zone, Z(Rl), (int)ldh, Z(Yb),
                                            (int)ldh), "ztrsm"));
        return blas_check(ctx, rocblas_zgemm(hb, rocblas_operation_none, rocblas_operation_none, (int)n, p, (int)m,
                                             &zone, Z(Vb), (int)n, Z(Yb), (int)ldh, &zone, Z(Xout), (int)n), "zgemm");
    }
};

}  // namespace

qrvie_status solve_block(qrvie_ctx* ctx, const qrvie_op* op, int na, const c128* v, int64_t ldv, c128* x,
                         int64_t ldx, const qrvie_solve_opts* o, qrvie_solve_info* info, bool* broke) {
    *broke = false;
    const double t0 = now_s();
    const qrvie_geom* g = op->g;
    const int64_t n = g->ndof();
    hipStream_t s = ctx->stream;
    std::vector<qrvie_solve_info> inf(na);
    for (auto& i : inf) i = qrvie_solve_info{};

    // right-hand-side norms; zero columns have x = 0 and take no part in the block
    std::vector<double> vnorm(na);
    {
        Work w0(ctx);
        double* d = nullptr;
        CHECK(w0.alloc(&d, na, "rhs norms"));
        launch_col_norms(s, (int)n, v, ldv, na, d);
        CHECK(hip_check(ctx, hipMemcpyAsync(vnorm.data(), d, sizeof(double) * na, hipMemcpyDeviceToHost, s), "norms"));
        CHECK(hip_check(ctx, hipStreamSynchronize(s), "norms"));
    }
    std::vector<int> cols;
    for (int i = 0; i < na; ++i) {
        if (!std::isfinite(vnorm[i])) {
            set_err(ctx, "solve: right-hand side has non-finite entries");
            return QRVIE_ERR_INVALID_ARG;
        }
        if (vnorm[i] > 0.0) {
            cols.push_back(i);
        } else {
            CHECK(hip_check(ctx, hipMemsetAsync(x + (int64_t)i * ldx, 0, sizeof(c128) * n, s), "zero x"));
            inf[i].converged = 1;
        }
    }
    if (cols.empty()) {
        if (info) std::copy(inf.begin(), inf.end(), info);
        return hip_check(ctx, hipStreamSynchronize(s), "solve");
    }

    BlockSolver B(ctx, op, o);
    CHECK(B.init((int)cols.size()));
    const int p = B.p;
    for (int c = 0; c < p; ++c) {
        launch_permute(s, g->N, g->d_i2c, v + (int64_t)cols[c] * ldv, B.Bc + (int64_t)c * n, 1);
        if (o->use_x0) launch_permute(s, g->N, g->d_i2c, x + (int64_t)cols[c] * ldx, B.X + (int64_t)c * n, 1);
    }
    if (!o->use_x0) CHECK(hip_check(ctx, hipMemsetAsync(B.X, 0, sizeof(c128) * n * p, s), "x0"));
    launch_gather_block(s, B.nt, g->N, nullptr, B.Bc, n, p, B.Bi);
    // ||Z_D^-1 b|| per column: the scale of the preconditioned estimates
    launch_strip_mfma(s, B.nt, op->d_ms, op->n_ms, op->d_pinv, B.Bi, B.Zi, nullptr);
    launch_scatter_block(s, B.nt, g->N, nullptr, B.Zi, B.Rc, n, p);
    launch_col_norms(s, (int)n, B.Rc, n, p, B.dnrm);
    int hf[2] = {0, 0};
    CHECK(B.read(B.dnrm, p, false, hf));
    std::vector<double> bnorm(p), pvnorm(p), ptol(p, o->tol), est(p, 0.0), tres(p, 0.0);
    for (int c = 0; c < p; ++c) {
        bnorm[c] = vnorm[cols[c]];
        pvnorm[c] = B.hbuf[c];
    }

    const zc zone = {1.0, 0.0}, zmone = {-1.0, 0.0}, ztwo = {2.0, 0.0}, zzero = {0.0, 0.0};
    int steps_total = 0, cycles = 0;
    bool done = false, converged = false;
    while (!done) {
        // cycle start: true residual of X and the first block V_0 S0 = Z_D^-1 (B - Z_QR X)
        B.residual(B.X, B.Rc, B.Vb);
        launch_col_norms(s, (int)n, B.Rc, n, p, B.dnrm);
        CHECK(B.read(B.dnrm, p, false, hf));
        B.add_product_time();
        bool all = true;
        for (int c = 0; c < p; ++c) {
            tres[c] = B.hbuf[c] / bnorm[c];
            all = all && tres[c] <= o->tol;
        }
        if (all) { converged = true; break; }
        if (steps_total >= o->max_iter) break;
        CHECK(hip_check(ctx, hipMemsetAsync(B.gl, 0, sizeof(c128) * B.ldh * p, s), "ls rhs"));
        CHECK(B.cholqr2(B.Vb, B.gl, B.ldh));
        CHECK(B.read(B.dnrm, 0, true, hf));
        if (hf[0] || hf[1]) { *broke = true; break; }
        int k = 0;
        bool end_cycle = false;
        for (; k < B.Kc && !end_cycle; ++k) {
            const int64_t m = (int64_t)(k + 1) * p;
            c128* Vk = B.Vb + (int64_t)k * p * n;
            c128* W = Vk + (int64_t)p * n;
            // W = Z_D^-1 Z_QR V_k
            launch_gather_block(s, B.nt, g->N, nullptr, Vk, n, p, B.Xi);
            (void)hipEventRecord(B.ev0, s);
            block_product(op, s, B.bw, B.nt, B.Xi, nullptr, B.Ri, B.Zi);
            (void)hipEventRecord(B.ev1, s);
            ++B.products;
            launch_scatter_block(s, B.nt, g->N, nullptr, B.Zi, W, n, p);
            // pass 1: [V^H V_k, V^H W]; Gram block; H = 2 H1 - G H1; pass 2: W -= V H
            CHECK(blas_check(ctx, rocblas_zgemm(B.hb, rocblas_operation_conjugate_transpose, rocblas_operation_none,
                                                (int)m, 2 * p, (int)n, &zone, Z(B.Vb), (int)n, Z(Vk), (int)n, &zzero,
                                                Z(B.Cb), (int)B.ldh), "zgemm projections"));
            launch_gram_store(s, k, p, B.Cb, B.ldh, B.G, B.ldh);
            const c128* H1 = B.Cb + (int64_t)p * B.ldh;
            CHECK(hip_check(ctx, hipMemcpy2DAsync(B.Hb, sizeof(c128) * B.ldh, H1, sizeof(c128) * B.ldh,
                                                  sizeof(c128) * m, p, hipMemcpyDeviceToDevice, s), "h1"));
            CHECK(blas_check(ctx, rocblas_zgemm(B.hb, rocblas_operation_none, rocblas_operation_none, (int)m, p, (int)m,
                                                &zmone, Z(B.G), (int)B.ldh, Z(H1), (int)B.ldh, &ztwo, Z(B.Hb),
                                                (int)B.ldh), "zgemm gram"));
            CHECK(blas_check(ctx, rocblas_zgemm(B.hb, rocblas_operation_none, rocblas_operation_none, (int)n, p, (int)m,
                                                &zmone, Z(B.Vb), (int)n, Z(B.Hb), (int)B.ldh, &zone, Z(W), (int)n),
                             "zgemm update"));
            // block Hessenberg column k: [H; H_{k+1,k}] with W = V_{k+1} H_{k+1,k}
            c128* col = B.Rl + (int64_t)k * p * B.ldh;
            CHECK(hip_check(ctx, hipMemcpy2DAsync(col, sizeof(c128) * B.ldh, B.Hb, sizeof(c128) * B.ldh,
                                                  sizeof(c128) * m, p, hipMemcpyDeviceToDevice, s), "hcol"));
            CHECK(B.cholqr2(W, col + m, B.ldh));
            // least squares: previous reflectors, the new one, and the transformed right-hand side
            launch_ls_apply(s, 0, k, p, B.Yr, B.Tr, col, B.ldh, p);
            launch_ls_factor(s, k, p, col, B.ldh, B.Yr + (int64_t)k * 2 * p * p, B.Tr + (int64_t)k * p * p);
            launch_ls_apply(s, k, k + 1, p, B.Yr, B.Tr, B.gl, B.ldh, p);
            launch_col_norms(s, p, B.gl + m, B.ldh, p, B.dnrm);
            CHECK(hip_check(ctx, hipGetLastError(), "block step"));
            CHECK(B.read(B.dnrm, p, true, hf));
            B.add_product_time();
            ++steps_total;
            const bool breakdown = hf[0] || hf[1];
            bool met = true;
            for (int c = 0; c < p; ++c) {
                est[c] = B.hbuf[c] / pvnorm[c];
                met = met && est[c] <= ptol[c];
            }
            if (met || breakdown) {
                // candidate X + V Y, accepted when every true residual meets tol
                CHECK(B.update(k + 1, B.X, B.Xc));
                B.residual(B.Xc, B.Rc, nullptr);
                launch_col_norms(s, (int)n, B.Rc, n, p, B.dnrm);
                CHECK(B.read(B.dnrm, p, false, hf));
                B.add_product_time();
                bool ok = true;
                for (int c = 0; c < p; ++c) {
                    tres[c] = B.hbuf[c] / bnorm[c];
                    if (tres[c] > o->tol) {
                        ok = false;
                        ptol[c] = std::max(ptol[c] * 0.5 * o->tol / tres[c], 1e-15);
                    }
                }
                if (ok) {
                    CHECK(hip_check(ctx, hipMemcpyAsync(B.X, B.Xc, sizeof(c128) * n * p, hipMemcpyDeviceToDevice, s),
                                    "x"));
                    converged = true;
                    done = true;
                    ++k;
                    break;
                }
                if (breakdown) end_cycle = true;   // the basis cannot grow: restart from the candidate
            }
            if (steps_total >= o->max_iter) end_cycle = true;
        }
        if (done) break;
        // end of the cycle: X += V Y, then restart (or stop at the step limit)
        CHECK(B.update(k, B.X, B.X));
        ++cycles;
        if (steps_total >= o->max_iter) {
            B.residual(B.X, B.Rc, nullptr);
            launch_col_norms(s, (int)n, B.Rc, n, p, B.dnrm);
            CHECK(B.read(B.dnrm, p, false, hf));
            for (int c = 0; c < p; ++c) tres[c] = B.hbuf[c] / bnorm[c];
            break;
        }
    }
    for (int c = 0; c < p; ++c)
        launch_permute(s, g->N, g->d_i2c, B.X + (int64_t)c * n, x + (int64_t)cols[c] * ldx, 0);
    CHECK(hip_check(ctx, hipStreamSynchronize(s), "solve"));
    const double total = now_s() - t0;
    for (int c = 0; c < p; ++c) {
        qrvie_solve_info& f = inf[cols[c]];
        f.iterations = steps_total;
        f.restarts = cycles;
        f.converged = tres[c] <= o->tol ? 1 : 0;
        f.rel_res_prec = est[c];
        f.rel_res_true = tres[c];
        f.n_apply = B.products;
        f.n_prec = B.products;
        f.t_apply_s = B.t_apply;       // block products, shared by the block's columns
        f.t_prec_s = 0.0;
        f.t_total_s = total;
        f.t_krylov_s = std::max(0.0, total - B.t_apply);
        f.n_reorth = steps_total;
        f.n_refine = 0;
    }
    if (info) std::copy(inf.begin(), inf.end(), info);
    (void)converged;
    for (int c = 0; c < p; ++c)
        if (!inf[cols[c]].converged) return QRVIE_NOT_CONVERGED;
    return QRVIE_OK;
}

}  // namespace qrvie
