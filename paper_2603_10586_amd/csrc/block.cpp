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
// block is factorised by Cholesky QR twice.  Every step runs on this library's kernels: the
// projections as split-K FP64 MFMA partial products with a fixed-order reduction, the basis
// and solution updates W += V H on FP64 MFMA, the right triangular solves of Cholesky QR as a
// product with the inverted small triangle, and the least-squares back substitution.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "work.h"

namespace qrvie {

namespace {

// Pivot floors (relative to the largest diagonal entry of a Gram matrix).  The first block
// of a cycle keeps the directions whose singular values exceed 1e-7 of the largest (a
// rank-revealing pivoted Cholesky): plane waves at nearby angles are numerically dependent,
// and what is dropped stays in the residual and returns at the next cycle.  A new Arnoldi
// block whose Cholesky QR meets a pivot below 1e-15 (condition above 3e7, where Cholesky QR
// twice no longer orthogonalises reliably) ends the cycle.
constexpr double kDeflateFloor = 1e-14;
constexpr double kCholFloor = 1e-15;

// Split-K projections: at most 256 row chunks of at least 512 rows, partial products within
// 32 M complex entries (512 MB).
constexpr int64_t kMaxChunks = 256;
constexpr int64_t kMinChunkRows = 512;
constexpr int64_t kPartialElems = kBlockPartialElems;

struct BlockSolver {
    qrvie_ctx* ctx;
    const qrvie_op* op;
    const qrvie_solve_opts* o;
    hipStream_t s;
    int64_t n;
    int p = 0, ntB = 0;          // right-hand sides and their tile count
    int q = 0, ntK = 0, Kc = 0;  // block width of the current cycle, tiles, block steps per cycle
    int64_t ldh = 0;             // rows of the least-squares arrays: (block steps + 1) x width <= ldh
    Work w;
    BlockWork bw;
    c128 *Bc = nullptr, *X = nullptr, *Xc = nullptr, *Rc = nullptr, *Zc = nullptr, *Vb = nullptr;
    c128 *Bi = nullptr, *Xi = nullptr, *Ri = nullptr, *Zi = nullptr;
    c128 *Cb = nullptr, *Hb = nullptr, *G = nullptr, *Rl = nullptr, *gl = nullptr, *Yb = nullptr;
    c128 *Yr = nullptr, *Tr = nullptr, *S = nullptr, *R1 = nullptr, *R2 = nullptr;
    c128* Pk = nullptr;          // split-K partial products
    c128 *Ui = nullptr, *Wt = nullptr;   // inverted triangle and product of a right solve
    int* dflag = nullptr;        // [0..1] Cholesky flags, [2] rank q, [3..] pivot order
    double* dnrm = nullptr;
    double* hbuf = nullptr;      // pinned
    int* hint = nullptr;         // pinned
    hipEvent_t ev0{}, ev1{};
    double t_apply = 0.0;
    int products = 0;
    bool lo = false;             // products (and residuals) on the complex64 panels
    int kind = kBlockF64;        // or on FP32 matrix cores (complex64 panels or BF16 planes)

    BlockSolver(qrvie_ctx* c, const qrvie_op* p_, const qrvie_solve_opts* o_, bool lo_, int kind_)
        : ctx(c), op(p_), o(o_), s(c->stream), n(p_->g->ndof()), w(c), lo(lo_), kind(kind_) {}
    ~BlockSolver() {
        if (hbuf) (void)hipHostFree(hbuf);
        if (hint) (void)hipHostFree(hint);
        (void)hipEventDestroy(ev0);
        (void)hipEventDestroy(ev1);
    }

    qrvie_status init(int ncols) {
        p = ncols;
        ntB = (p + 15) / 16;
        ldh = (int64_t)(std::max(1, std::min(o->restart / p, o->max_iter)) + 1) * p;
        const int64_t P = 16 * ntB;
        CHECK(bw.init(w, op));
        CHECK(w.alloc(&Bc, (size_t)n * p, "block rhs"));
        CHECK(w.alloc(&X, (size_t)n * p, "block x"));
        CHECK(w.alloc(&Xc, (size_t)n * p, "block candidate"));
        CHECK(w.alloc(&Rc, (size_t)n * p, "block residual"));
        CHECK(w.alloc(&Zc, (size_t)n * p, "block preconditioned residual"));
        CHECK(w.alloc(&Vb, (size_t)n * ldh, "block krylov basis"));
        CHECK(w.alloc(&Bi, (size_t)n * P, "interleaved rhs"));
        CHECK(w.alloc(&Xi, (size_t)n * P, "interleaved x"));
        CHECK(w.alloc(&Ri, (size_t)n * P, "interleaved residual"));
        CHECK(w.alloc(&Zi, (size_t)n * P, "interleaved product"));
        CHECK(w.alloc(&Cb, (size_t)ldh * 2 * p, "block projections"));
        CHECK(w.alloc(&Hb, (size_t)ldh * p, "block coefficients"));
        CHECK(w.alloc(&G, (size_t)ldh * ldh, "block gram matrix"));
        CHECK(w.alloc(&Rl, (size_t)ldh * ldh, "block hessenberg"));
        CHECK(w.alloc(&gl, (size_t)ldh * p, "block least-squares rhs"));
        CHECK(w.alloc(&Yb, (size_t)ldh * p, "block least-squares solution"));
        CHECK(w.alloc(&Yr, (size_t)2 * p * ldh, "block reflectors"));
        CHECK(w.alloc(&Tr, (size_t)p * ldh, "block reflector factors"));
        CHECK(w.alloc(&S, (size_t)p * p, "gram block"));
        CHECK(w.alloc(&R1, (size_t)p * p, "cholesky factor"));
        CHECK(w.alloc(&R2, (size_t)p * p, "cholesky factor"));
        CHECK(w.alloc(&Pk, (size_t)kPartialElems, "split-k partials"));
        CHECK(w.alloc(&Ui, (size_t)p * p, "inverted triangle"));
        CHECK(w.alloc(&Wt, (size_t)n * p, "right-solve product"));
        CHECK(w.alloc(&dflag, 3 + (size_t)p, "cholesky flags"));
        CHECK(w.alloc(&dnrm, 2 * (size_t)p, "block norms"));
        CHECK(hip_check(ctx, hipHostMalloc((void**)&hbuf, sizeof(double) * 2 * p, hipHostMallocDefault), "pinned"));
        CHECK(hip_check(ctx, hipHostMalloc((void**)&hint, sizeof(int) * (3 + p), hipHostMallocDefault), "pinned"));
        (void)hipEventCreate(&ev0);
        (void)hipEventCreate(&ev1);
        return QRVIE_OK;
    }

    // host copies of `count` doubles and `nint` flag words, then sync
    qrvie_status read(const double* d, int count, int nint) {
        if (count > 0)
            CHECK(hip_check(ctx, hipMemcpyAsync(hbuf, d, sizeof(double) * count, hipMemcpyDeviceToHost, s), "read"));
        if (nint > 0)
            CHECK(hip_check(ctx, hipMemcpyAsync(hint, dflag, sizeof(int) * nint, hipMemcpyDeviceToHost, s), "read"));
        return hip_check(ctx, hipStreamSynchronize(s), "sync");
    }

    // out = B - Z_QR Xcol and, optionally, zcol = Z_D^-1 out (col-major n x p)
    void residual(const c128* Xcol, c128* out, c128* zcol) {
        launch_gather_block(s, ntB, op->g->N, nullptr, Xcol, n, p, Xi);
        (void)hipEventRecord(ev0, s);
        block_product(op, s, bw, ntB, Xi, Bi, Ri, zcol ? Zi : nullptr, lo, kind);
        (void)hipEventRecord(ev1, s);
        ++products;
        launch_scatter_block(s, ntB, op->g->N, nullptr, Ri, out, n, p);
        if (zcol) launch_scatter_block(s, ntB, op->g->N, nullptr, Zi, zcol, n, p);
    }
    void add_product_time() {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ev0, ev1) == hipSuccess) t_apply += ms * 1e-3;
    }

    // C (m x c, ldc) = A^H B for n-row A (ld lda) and B (ld ldb).  The outputs of the basis
    // projections are small (m x c with c <= 128) against a 10^5-10^6 long reduction, so the
    // rows are split into chunks: one partial product per chunk (FP64 MFMA) and a fixed-order
    // reduction sums them (deterministic, and the whole device is busy).
    qrvie_status gemm_hn(const c128* A, int64_t lda, int m, const c128* Bm, int64_t ldb, int c, c128* C, int64_t ldc) {
        const int64_t per = (int64_t)m * c;
        if (per == 0) return QRVIE_OK;
        const int64_t nb = std::max<int64_t>(1, std::min<int64_t>({kMaxChunks, kPartialElems / per, n / kMinChunkRows}));
        const int64_t L = ((n + nb - 1) / nb + 15) / 16 * 16;
        const int64_t used = (n + L - 1) / L;
        launch_gemm_hn_part(s, n, m, c, A, lda, Bm, ldb, (int)used, L, Pk);
        launch_sum_batches(s, m, c, (int)used, Pk, C, ldc);
        return hip_check(ctx, hipGetLastError(), "projection");
    }

    qrvie_status gram(const c128* Wp, int cols) { return gemm_hn(Wp, n, cols, Wp, n, cols, S, cols); }
    // W (n x cols) = W R^-1 for the upper triangular R: the inverse of the small triangle, then
    // one MFMA product into a work block copied back.
    qrvie_status right_solve(c128* Wp, int cols, const c128* R, int64_t ldr) {
        launch_tri_inv_upper(s, cols, R, ldr, Ui, cols);
        launch_gemm_nn_acc(s, n, cols, cols, Wp, n, Ui, cols, 0.0, 1.0, Wt, n);
        CHECK(hip_check(ctx, hipMemcpyAsync(Wp, Wt, sizeof(c128) * n * cols, hipMemcpyDeviceToDevice, s), "right solve"));
        return hip_check(ctx, hipGetLastError(), "right solve");
    }

    // W (n x cols, ld n) = Q R, Q in place, R (cols x cols upper) at out; Cholesky QR twice.
    // Sets the two flag words (read later); R = 0 when either pass met a pivot below kCholFloor.
    qrvie_status cholqr2(c128* Wp, int cols, c128* out, int64_t ldo) {
        c128* Rs[2] = {R1, R2};
        for (int pass = 0; pass < 2; ++pass) {
            CHECK(gram(Wp, cols));
            launch_cholesky(s, cols, S, cols, kCholFloor, Rs[pass], cols, dflag + pass);
            CHECK(right_solve(Wp, cols, Rs[pass], cols));
        }
        launch_trmm_upper(s, cols, R2, cols, R1, cols, out, ldo, dflag);
        return QRVIE_OK;
    }

    // First block of a cycle from the preconditioned residuals Zc (n x p).  Repeatedly: take
    // the dominant directions of the remainder E (rank-revealing pivoted Cholesky of E^H E,
    // relative to E's own scale), orthogonalise them against the directions already kept
    // (twice) and normalise them (Cholesky QR twice); then S0 = V_0^H Zc and E = Zc - V_0 S0,
    // until every column's remainder is below 1e-3 tol ||Z_D^-1 b|| or the block is full.
    // Rows 0:q of gl receive S0.  q = 0 means the residuals have no usable direction.
    qrvie_status first_block(const std::vector<double>& pvnorm) {
        q = 0;
        c128* E = Rc;
        CHECK(hip_check(ctx, hipMemcpyAsync(E, Zc, sizeof(c128) * n * p, hipMemcpyDeviceToDevice, s), "remainder"));
        CHECK(hip_check(ctx, hipMemsetAsync(gl, 0, sizeof(c128) * ldh * p, s), "ls rhs"));
        for (int pass = 0; pass < 4 && q < p; ++pass) {
            CHECK(gram(E, p));
            launch_cholesky_piv(s, p, S, p, kDeflateFloor, R1, p, dflag + 3, dflag + 2);
            CHECK(read(nullptr, 0, 3 + p));
            const int q2 = std::min(hint[2], p - q);
            if (q2 == 0) break;
            c128* Vn = Vb + (int64_t)q * n;
            for (int c = 0; c < q2; ++c)
                CHECK(hip_check(ctx, hipMemcpyAsync(Vn + (int64_t)c * n, E + (int64_t)hint[3 + c] * n,
                                                    sizeof(c128) * n, hipMemcpyDeviceToDevice, s), "first block"));
            CHECK(right_solve(Vn, q2, R1, p));
            for (int it = 0; q > 0 && it < 2; ++it) {     // against the kept directions, twice
                CHECK(gemm_hn(Vb, n, q, Vn, n, q2, Cb, q));
                launch_gemm_nn_acc(s, n, q, q2, Vb, n, Cb, q, 1.0, -1.0, Vn, n);
            }
            CHECK(cholqr2(Vn, q2, Hb, q2));
            CHECK(read(nullptr, 0, 2));
            if (hint[0] || hint[1]) break;                // not independent after all: keep what we have
            q += q2;
            // S0 = V_0^H Zc and the remainder E = Zc - V_0 S0
            CHECK(gemm_hn(Vb, n, q, Zc, n, p, gl, ldh));
            CHECK(hip_check(ctx, hipMemcpyAsync(E, Zc, sizeof(c128) * n * p, hipMemcpyDeviceToDevice, s), "remainder"));
            launch_gemm_nn_acc(s, n, q, p, Vb, n, gl, ldh, 1.0, -1.0, E, n);
            launch_col_norms(s, (int)n, E, n, p, dnrm);
            CHECK(read(dnrm, p, 0));
            bool small = true;
            for (int c = 0; c < p; ++c) small = small && hbuf[c] <= 1e-3 * o->tol * pvnorm[c];
            if (small) break;
        }
        if (q > 0) {
            ntK = (q + 15) / 16;
            Kc = std::max(1, std::min((int)(ldh / q) - 1, o->max_iter));
        }
        return QRVIE_OK;
    }

    // X_out = X_in + V[:, 0:steps q] R^-1 gl[0:steps q, :]
    qrvie_status update(int steps, const c128* Xin, c128* Xout) {
        const int64_t m = (int64_t)steps * q;
        if (Xout != Xin)
            CHECK(hip_check(ctx, hipMemcpyAsync(Xout, Xin, sizeof(c128) * n * p, hipMemcpyDeviceToDevice, s), "x"));
        if (steps == 0) return QRVIE_OK;
        CHECK(hip_check(ctx, hipMemcpy2DAsync(Yb, sizeof(c128) * ldh, gl, sizeof(c128) * ldh, sizeof(c128) * m, p,
                                              hipMemcpyDeviceToDevice, s), "y"));
        launch_trsm_upper_left(s, (int)m, p, Rl, ldh, Yb, ldh);
        launch_gemm_nn_acc(s, n, (int)m, p, Vb, n, Yb, ldh, 1.0, 1.0, Xout, n);
        return hip_check(ctx, hipGetLastError(), "solution update");
    }
};

}  // namespace

// Stage timers of the block product for nrhs (<= 64) interleaved right-hand sides.
qrvie_status profile_block(qrvie_ctx* ctx, const qrvie_op* op, int nrhs, int reps, double* ms, int64_t* flops) {
    const qrvie_geom* g = op->g;
    const int64_t n = g->ndof();
    const int nt = (nrhs + 15) / 16, P = 16 * nt;
    hipStream_t s = ctx->stream;
    Work w(ctx);
    BlockWork bw;
    CHECK(bw.init(w, op));
    c128 *X, *Y, *Zp;
    CHECK(w.alloc(&X, (size_t)n * P, "profile block"));
    CHECK(w.alloc(&Y, (size_t)n * P, "profile block"));
    CHECK(w.alloc(&Zp, (size_t)n * P, "profile block"));
    CHECK(hip_check(ctx, hipMemsetAsync(X, 0, sizeof(c128) * n * P, s), "profile block"));
    hipEvent_t ev[5];
    for (auto& e : ev) (void)hipEventCreate(&e);
    double acc[4] = {0, 0, 0, 0};
    const bool l = !op->d_fac;
    const int vr = op->tile_of(l, nt, 0), vq = op->tile_of(l, nt, 1), vs = op->tile_of(l, nt, 2);
    for (int r = 0; r < reps; ++r) {
        (void)hipEventRecord(ev[0], s);
        if (op->d_fac) launch_strip_mfma(s, nt, op->d_mr, op->n_mr, op->d_fac, X, bw.T, op->d_tmap, vr);
        else launch_strip_mfma(s, nt, op->d_mr, op->n_mr, op->d_fac32, X, bw.T, op->d_tmap, vr);
        (void)hipEventRecord(ev[1], s);
        if (op->d_fac) launch_strip_mfma(s, nt, op->d_mq, op->n_mq, op->d_fac, bw.T, bw.Ylev, nullptr, vq);
        else launch_strip_mfma(s, nt, op->d_mq, op->n_mq, op->d_fac32, bw.T, bw.Ylev, nullptr, vq);
        (void)hipEventRecord(ev[2], s);
        launch_strip_mfma(s, nt, op->d_ms, op->n_ms, op->d_self, X, bw.Yself, nullptr, vs);
        launch_block_combine(s, nt, n, bw.Ylev, op->n_active, bw.Yself, X, Y);
        (void)hipEventRecord(ev[3], s);
        launch_strip_mfma(s, nt, op->d_ms, op->n_ms, op->d_pinv, Y, Zp, nullptr, vs);
        (void)hipEventRecord(ev[4], s);
        CHECK(hip_check(ctx, hipEventSynchronize(ev[4]), "profile block"));
        for (int k = 0; k < 4; ++k) {
            float t = 0.f;
            (void)hipEventElapsedTime(&t, ev[k], ev[k + 1]);
            acc[k] += t;
        }
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    for (int k = 0; k < 4; ++k) ms[k] = acc[k] / reps;
    // 8 real flops per complex multiply-add, P right-hand sides (the padded width)
    int64_t rn = 0, mr = 0;
    for (size_t b = 0; b < op->blocks.size(); ++b) {
        rn += (int64_t)op->rank[b] * op->blocks[b].cn * kNp;
        mr += (int64_t)op->rank[b] * op->blocks[b].rn * kNp;
    }
    const int64_t self = (int64_t)g->N * kNp * kNp;
    flops[0] = 8 * P * rn;
    flops[1] = 8 * P * mr;
    flops[2] = 8 * P * self;
    flops[3] = 8 * P * self;
    return hip_check(ctx, hipGetLastError(), "profile block");
}

// Autotuner of the strip tile shapes, one choice per strip group (R panels, Q panels, self
// blocks) for this operator, tile count and panel precision.  Each group's output is
// cleared before every launch so that entries no strip writes compare equal.
qrvie_status tune_block(qrvie_ctx* ctx, qrvie_op* op, int prec, int nrhs, int reps, qrvie_block_tune* out) {
    const qrvie_geom* g = op->g;
    const int64_t n = g->ndof();
    const int nt = (nrhs + 15) / 16, P = 16 * nt;
    const bool l = prec == QRVIE_PREC_C64 || !op->d_fac;
    hipStream_t s = ctx->stream;
    Work w(ctx);
    BlockWork bw;
    CHECK(bw.init(w, op));
    // a fixed pseudo-random input block (64-bit LCG, uniform in [-1, 1) per component)
    std::vector<c128> hx((size_t)n * P);
    uint64_t st = 0x9E3779B97F4A7C15ull;
    auto next = [&st]() {
        st = st * 6364136223846793005ull + 1442695040888963407ull;
        return (double)(st >> 11) * 0x1.0p-52 - 1.0;
    };
    for (auto& e : hx) { e.x = next(); e.y = next(); }
    c128* X;
    unsigned long long* dmis;
    CHECK(w.alloc(&X, hx.size(), "tune input"));
    CHECK(w.alloc(&dmis, 3 * kStripVariants, "tune counts"));
    CHECK(hip_check(ctx, hipMemcpyAsync(X, hx.data(), sizeof(c128) * hx.size(), hipMemcpyHostToDevice, s), "tune"));
    CHECK(hip_check(ctx, hipMemsetAsync(dmis, 0, sizeof(unsigned long long) * 3 * kStripVariants, s), "tune"));
    const size_t out_len[3] = {(size_t)std::max<int64_t>(op->t_len, 1) * P,
                               (size_t)std::max(op->n_active, 1) * n * P, (size_t)n * P};
    c128* outs[3] = {bw.T, bw.Ylev, bw.Yself};
    c128* ref;
    CHECK(w.alloc(&ref, std::max({out_len[0], out_len[1], out_len[2]}), "tune reference"));
    auto run = [&](int grp, int v) {
        switch (grp) {
            case 0:
                if (l) launch_strip_mfma(s, nt, op->d_mr, op->n_mr, op->d_fac32, X, bw.T, op->d_tmap, v);
                else launch_strip_mfma(s, nt, op->d_mr, op->n_mr, op->d_fac, X, bw.T, op->d_tmap, v);
                break;
            case 1:
                if (l) launch_strip_mfma(s, nt, op->d_mq, op->n_mq, op->d_fac32, bw.T, bw.Ylev, nullptr, v);
                else launch_strip_mfma(s, nt, op->d_mq, op->n_mq, op->d_fac, bw.T, bw.Ylev, nullptr, v);
                break;
            default: launch_strip_mfma(s, nt, op->d_ms, op->n_ms, op->d_self, X, bw.Yself, nullptr, v); break;
        }
    };
    hipEvent_t e0, e1;
    CHECK(hip_check(ctx, hipEventCreate(&e0), "tune events"));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_check(ctx, hipErrorOutOfMemory, "tune events");
    }
    qrvie_status status = QRVIE_OK;
    std::memset(out, 0, sizeof(*out));
    out->nrhs_tile = P;
    out->n_variants = kStripVariants;
    for (int v = 0; v < kStripVariants; ++v) {
        out->u[v] = strip_variant_u(v);
        out->rows_per_wave[v] = strip_variant_rows(v);
    }
    const int64_t count[3] = {op->n_mr, op->n_mq, op->n_ms};
    for (int grp = 0; grp < 3 && status == QRVIE_OK; ++grp) {
        if (grp == 1) {   // the Q group reads the rank-space block the R group produced
            run(0, 0);
        }
        for (int v = 0; v < kStripVariants && status == QRVIE_OK; ++v) {
            if (count[grp] == 0) break;
            const size_t bytes = sizeof(c128) * out_len[grp];
            status = hip_check(ctx, hipMemsetAsync(outs[grp], 0, bytes, s), "tune clear");
            if (status != QRVIE_OK) break;
            run(grp, v);
            if (v == 0) status = hip_check(ctx, hipMemcpyAsync(ref, outs[grp], bytes, hipMemcpyDeviceToDevice, s), "tune ref");
            else launch_count_neq(s, 2 * (int64_t)out_len[grp], outs[grp], ref, dmis + grp * kStripVariants + v);
            (void)hipEventRecord(e0, s);
            for (int r = 0; r < reps; ++r) run(grp, v);
            (void)hipEventRecord(e1, s);
            status = hip_check(ctx, hipEventSynchronize(e1), "tune");
            float t = 0.f;
            if (status == QRVIE_OK) status = hip_check(ctx, hipEventElapsedTime(&t, e0, e1), "tune timer");
            out->ms[grp][v] = t / reps;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    CHECK(status);
    unsigned long long hm[3 * kStripVariants];
    CHECK(hip_check(ctx, hipMemcpy(hm, dmis, sizeof(hm), hipMemcpyDeviceToHost), "tune counts"));
    for (int grp = 0; grp < 3; ++grp) {
        int best = 0;
        for (int v = 0; v < kStripVariants; ++v) {
            out->mismatches[grp][v] = (int64_t)hm[grp * kStripVariants + v];
            if (count[grp] > 0 && hm[grp * kStripVariants + v] == 0 && out->ms[grp][v] < out->ms[grp][best]) best = v;
        }
        out->chosen[grp] = best;
        op->tile[l ? 1 : 0][nt - 1][grp].store(best, std::memory_order_relaxed);
    }
    return hip_check(ctx, hipGetLastError(), "tune");
}

qrvie_status solve_block(qrvie_ctx* ctx, const qrvie_op* op, int na, const c128* v, int64_t ldv, c128* x,
                         int64_t ldx, const qrvie_solve_opts* o, qrvie_solve_info* info, bool* broke, bool lo,
                         int kind) {
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

    BlockSolver B(ctx, op, o, lo, kind);
    CHECK(B.init((int)cols.size()));
    const int p = B.p;
    for (int c = 0; c < p; ++c) {
        launch_permute(s, g->N, g->d_i2c, v + (int64_t)cols[c] * ldv, B.Bc + (int64_t)c * n, 1);
        if (o->use_x0) launch_permute(s, g->N, g->d_i2c, x + (int64_t)cols[c] * ldx, B.X + (int64_t)c * n, 1);
    }
    if (!o->use_x0) CHECK(hip_check(ctx, hipMemsetAsync(B.X, 0, sizeof(c128) * n * p, s), "x0"));
    launch_gather_block(s, B.ntB, g->N, nullptr, B.Bc, n, p, B.Bi);
    // ||Z_D^-1 b|| per column: the scale of the preconditioned estimates
    launch_strip_mfma(s, B.ntB, op->d_ms, op->n_ms, op->d_pinv, B.Bi, B.Zi, nullptr);
    launch_scatter_block(s, B.ntB, g->N, nullptr, B.Zi, B.Rc, n, p);
    launch_col_norms(s, (int)n, B.Rc, n, p, B.dnrm);
    CHECK(B.read(B.dnrm, p, 0));
    std::vector<double> bnorm(p), pvnorm(p), ptol(p, o->tol), est(p, 0.0), tres(p, 0.0);
    for (int c = 0; c < p; ++c) {
        bnorm[c] = vnorm[cols[c]];
        pvnorm[c] = B.hbuf[c];
    }

    int steps_total = 0, cycles = 0;
    for (;;) {
        // cycle start: true residual of X and the first block from Z_D^-1 (B - Z_QR X)
        B.residual(B.X, B.Rc, B.Zc);
        launch_col_norms(s, (int)n, B.Rc, n, p, B.dnrm);
        CHECK(B.read(B.dnrm, p, 0));
        B.add_product_time();
        bool all = true;
        for (int c = 0; c < p; ++c) {
            tres[c] = B.hbuf[c] / bnorm[c];
            all = all && tres[c] <= o->tol;
        }
        if (o->verbose) {
            double worst = 0.0;
            for (int c = 0; c < p; ++c) worst = std::max(worst, tres[c]);
            std::fprintf(stderr, "[qrvie] cycle %d start after %d block steps: worst true residual %.3e, %.1f s\n",
                         cycles, steps_total, worst, now_s() - t0);
            std::fflush(stderr);
        }
        if (all || steps_total >= o->max_iter) break;
        CHECK(B.first_block(pvnorm));
        if (B.q == 0) { *broke = true; break; }
        const int q = B.q;
        int k = 0;
        bool end_cycle = false, done = false;
        for (; k < B.Kc && !end_cycle; ++k) {
            const int64_t m = (int64_t)(k + 1) * q;
            c128* Vk = B.Vb + (int64_t)k * q * n;
            c128* W = Vk + (int64_t)q * n;
            // W = Z_D^-1 Z_QR V_k
            launch_gather_block(s, B.ntK, g->N, nullptr, Vk, n, q, B.Xi);
            (void)hipEventRecord(B.ev0, s);
            block_product(op, s, B.bw, B.ntK, B.Xi, nullptr, B.Ri, B.Zi, B.lo, B.kind);
            (void)hipEventRecord(B.ev1, s);
            ++B.products;
            launch_scatter_block(s, B.ntK, g->N, nullptr, B.Zi, W, n, q);
            // pass 1: [V^H V_k, V^H W]; Gram block; H = 2 H1 - G H1; pass 2: W -= V H
            CHECK(B.gemm_hn(B.Vb, n, (int)m, Vk, n, 2 * q, B.Cb, B.ldh));
            launch_gram_store(s, k, q, B.Cb, B.ldh, B.G, B.ldh);
            const c128* H1 = B.Cb + (int64_t)q * B.ldh;
            CHECK(hip_check(ctx, hipMemcpy2DAsync(B.Hb, sizeof(c128) * B.ldh, H1, sizeof(c128) * B.ldh,
                                                  sizeof(c128) * m, q, hipMemcpyDeviceToDevice, s), "h1"));
            launch_gemm_nn_acc(s, m, (int)m, q, B.G, B.ldh, H1, B.ldh, 2.0, -1.0, B.Hb, B.ldh);
            launch_gemm_nn_acc(s, n, (int)m, q, B.Vb, n, B.Hb, B.ldh, 1.0, -1.0, W, n);
            // block Hessenberg column k: [H; H_{k+1,k}] with W = V_{k+1} H_{k+1,k}
            c128* col = B.Rl + (int64_t)k * q * B.ldh;
            CHECK(hip_check(ctx, hipMemcpy2DAsync(col, sizeof(c128) * B.ldh, B.Hb, sizeof(c128) * B.ldh,
                                                  sizeof(c128) * m, q, hipMemcpyDeviceToDevice, s), "hcol"));
            CHECK(B.cholqr2(W, q, col + m, B.ldh));
            // least squares: previous reflectors, the new one, and the transformed right-hand sides
            launch_ls_apply(s, 0, k, q, B.Yr, B.Tr, col, B.ldh, q);
            launch_ls_factor(s, k, q, col, B.ldh, B.Yr + (int64_t)k * 2 * q * q, B.Tr + (int64_t)k * q * q);
            launch_ls_apply(s, k, k + 1, q, B.Yr, B.Tr, B.gl, B.ldh, p);
            launch_col_norms(s, q, B.gl + m, B.ldh, p, B.dnrm);
            CHECK(hip_check(ctx, hipGetLastError(), "block step"));
            CHECK(B.read(B.dnrm, p, 2));
            B.add_product_time();
            ++steps_total;
            const bool breakdown = B.hint[0] || B.hint[1];
            bool met = true;
            double worst = 0.0;
            for (int c = 0; c < p; ++c) {
                est[c] = B.hbuf[c] / pvnorm[c];
                met = met && est[c] <= ptol[c];
                worst = std::max(worst, est[c]);
            }
            if (o->verbose && (steps_total % 10 == 0 || met || breakdown)) {
                std::fprintf(stderr, "[qrvie] block step %d (cycle %d, width %d): worst estimate %.3e, %.1f s\n",
                             steps_total, cycles, q, worst, now_s() - t0);
                std::fflush(stderr);
            }
            if (met || breakdown) {
                // candidate X + V Y, accepted when every true residual meets tol
                CHECK(B.update(k + 1, B.X, B.Xc));
                B.residual(B.Xc, B.Rc, nullptr);
                launch_col_norms(s, (int)n, B.Rc, n, p, B.dnrm);
                CHECK(B.read(B.dnrm, p, 0));
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
                    done = true;
                    break;
                }
                if (breakdown) end_cycle = true;   // the basis cannot grow: restart from the candidate
            }
            if (steps_total >= o->max_iter) end_cycle = true;
        }
        if (done) break;
        // end of the cycle: X += V Y, then restart (the next cycle starts with the true residual)
        CHECK(B.update(k, B.X, B.X));
        ++cycles;
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
    for (int c = 0; c < p; ++c)
        if (!inf[cols[c]].converged) return QRVIE_NOT_CONVERGED;
    return QRVIE_OK;
}

}  // namespace qrvie
