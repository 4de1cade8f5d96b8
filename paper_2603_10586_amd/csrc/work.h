// Host-side helpers shared by the solver drivers: a device workspace arena charged to the
// context's HBM budget, and the block product over up to 64 interleaved right-hand sides.
#pragma once

#include <algorithm>
#include <chrono>
#include <utility>
#include <vector>

#include "internal.h"

namespace qrvie {

#define CHECK(x)                       \
    do {                               \
        qrvie_status _s = (x);         \
        if (_s != QRVIE_OK) return _s; \
    } while (0)

inline double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
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


// Workspaces of the block product (up to kMaxBlockRhs interleaved right-hand sides).
struct BlockWork {
    c128 *T = nullptr, *Ylev = nullptr, *Yself = nullptr, *S = nullptr;
    qrvie_status init(Work& w, const qrvie_op* op) {
        const int64_t n = op->g->ndof(), P = kMaxBlockRhs;
        CHECK(w.alloc(&T, (size_t)std::max<int64_t>(op->t_len, 1) * P, "block rank space"));
        if (op->shared) CHECK(w.alloc(&S, (size_t)std::max<int64_t>(op->t_len, 1) * P, "block rank space Q^T X"));
        CHECK(w.alloc(&Ylev, (size_t)std::max(op->n_active, 1) * n * P, "block level partials"));
        return w.alloc(&Yself, (size_t)n * P, "block self product");
    }
};

// Factor precision of a block product: kBlockF64 FP64 matrix cores on the complex128 panels,
// or on the complex64 panels widened (the operator keeps no complex128 panels, or lo);
// kBlockF32 FP32 matrix cores with FP32 accumulation on the complex64 panels; kBlockBF16 the
// same on the BF16 split-complex planes.  The FP32 forms take the complex64 self blocks.
enum { kBlockF64 = 0, kBlockF32 = 1, kBlockBF16 = 2 };

// out = V - Z X (or Z X when V is null), Z_out = Z_D^-1 out (optional); X, V, out, Z_out are
// n x P interleaved blocks, P = 16 nt, internal order.  Shared factors add two passes: S = Q^T X
// (in the stacked order of the R panels) before the R strips, and the level partials R^T S
// (written first; the Q strips accumulate onto them).
inline void block_product(const qrvie_op* op, hipStream_t s, const BlockWork& bw, int nt, const c128* X, const c128* V,
                          c128* out, c128* zout, bool lo = false, int kind = kBlockF64) {
    const int64_t n = op->g->ndof();
    if (kind != kBlockF64) {
        auto far = [&](const MStrip* st, int64_t cnt, const c128* in, c128* o, const int64_t* map) {
            if (kind == kBlockBF16) launch_strip_mfma32_bf16(s, nt, st, cnt, op->d_fac16, op->fac_elems, in, o, map);
            else launch_strip_mfma32(s, nt, st, cnt, op->d_fac32, in, o, map);
        };
        if (op->shared) far(op->d_mqt, op->n_mqt, X, bw.S, op->d_tinv);
        far(op->d_mr, op->n_mr, X, bw.T, op->d_tmap);
        if (op->shared) far(op->d_mrt, op->n_mrt, bw.S, bw.Ylev, nullptr);
        far(op->d_mq, op->n_mq, bw.T, bw.Ylev, nullptr);
        launch_strip_mfma32(s, nt, op->d_ms, op->n_ms, op->d_self32, X, bw.Yself, nullptr);
        launch_block_combine(s, nt, n, bw.Ylev, op->n_active, bw.Yself, V, out);
        if (zout) launch_strip_mfma32(s, nt, op->d_ms, op->n_ms, op->d_pinv32, out, zout, nullptr);
        return;
    }
    const bool l = lo || !op->d_fac;
    const int vr = op->tile_of(l, nt, 0), vq = op->tile_of(l, nt, 1), vs = op->tile_of(l, nt, 2);
    // transposed strips read 4 consecutive entries per row and step: batches of 4 steps make
    // each row's read 16 entries long (tile variant 2)
    constexpr int kTransVariant = 2;
    if (l) {
        if (op->shared) launch_strip_mfma(s, nt, op->d_mqt, op->n_mqt, op->d_fac32, X, bw.S, op->d_tinv, kTransVariant);
        launch_strip_mfma(s, nt, op->d_mr, op->n_mr, op->d_fac32, X, bw.T, op->d_tmap, vr);
        if (op->shared) launch_strip_mfma(s, nt, op->d_mrt, op->n_mrt, op->d_fac32, bw.S, bw.Ylev, nullptr, kTransVariant);
        launch_strip_mfma(s, nt, op->d_mq, op->n_mq, op->d_fac32, bw.T, bw.Ylev, nullptr, vq);
    } else {
        if (op->shared) launch_strip_mfma(s, nt, op->d_mqt, op->n_mqt, op->d_fac, X, bw.S, op->d_tinv, kTransVariant);
        launch_strip_mfma(s, nt, op->d_mr, op->n_mr, op->d_fac, X, bw.T, op->d_tmap, vr);
        if (op->shared) launch_strip_mfma(s, nt, op->d_mrt, op->n_mrt, op->d_fac, bw.S, bw.Ylev, nullptr, kTransVariant);
        launch_strip_mfma(s, nt, op->d_mq, op->n_mq, op->d_fac, bw.T, bw.Ylev, nullptr, vq);
    }
    launch_strip_mfma(s, nt, op->d_ms, op->n_ms, op->d_self, X, bw.Yself, nullptr, vs);
    launch_block_combine(s, nt, n, bw.Ylev, op->n_active, bw.Yself, V, out);
    if (zout) launch_strip_mfma(s, nt, op->d_ms, op->n_ms, op->d_pinv, out, zout, nullptr, vs);
}


// Split-K partial products of the block solver's basis projections (512 MB).
constexpr int64_t kBlockPartialElems = (int64_t)32 << 20;

// Basis vectors per column when a rank-deficient block of `cnt` right-hand sides is finished
// by the single-vector solver (groups of up to 8 columns), keeping the block path's total.
inline int32_t block_fallback_restart(int32_t restart, int cnt) {
    return std::max<int32_t>(1, restart / std::max(1, std::min(cnt, 8)));
}

// Block GMRES over up to kMaxBlockRhs right-hand sides (block.cpp).  `broke` is set when the
// block of right-hand sides (or of residuals at a restart) is numerically rank deficient; x
// then holds the best iterate and the caller finishes those columns another way.
// lo: products and residuals on the complex64 panels (the corrections of BLOCK_IR).
qrvie_status solve_block(qrvie_ctx* ctx, const qrvie_op* op, int na, const c128* v, int64_t ldv, c128* x,
                         int64_t ldx, const qrvie_solve_opts* o, qrvie_solve_info* info, bool* broke,
                         bool lo = false, int kind = kBlockF64);

qrvie_status profile_block(qrvie_ctx* ctx, const qrvie_op* op, int nrhs, int reps, double* ms, int64_t* flops);
qrvie_status tune_block(qrvie_ctx* ctx, qrvie_op* op, int prec, int nrhs, int reps, qrvie_block_tune* out);

}  // namespace qrvie
