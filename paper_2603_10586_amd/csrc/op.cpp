// Compressed operator: build (assembly + certified low-rank compression of every
// far/finest pair block, §5.2-5.4), panel layout for the product, and the product
// and preconditioner entry points.
//
// Compression of a block B (m x n), relative Frobenius tolerance eps (§5.2, eq. 5.3):
//  * small blocks (both sides <= 2 particles): truncated column-pivoted Householder QR
//    of B itself;
//  * larger blocks: a randomised range sketch Y = B Omega (k columns), an orthonormal
//    basis Q_k of Y (CGS2), W = Q_k^H B, and the truncated pivoted QR of W, whose
//    tolerance is reduced by the sketch residual ||B||^2 - ||W||^2; Q = Q_k Q_W.
// Every block is then certified by recomputing ||B - Q R||_F from B; a block that
// misses eps is redone with a wider sketch.  Only the pairs (I, J) with I before J are
// compressed; (J, I) stores the transposed factors, so Z_QR is exactly symmetric like Z.
#include <algorithm>
#include <array>
#include <cstdio>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>

#include "internal.h"

using namespace qrvie;

namespace qrvie {
std::vector<int32_t> node_children(const qrvie_geom* g, int32_t id);
void launch_gemm_residual(hipStream_t s, const GemmDesc* d, const int32_t* td, const int32_t* tmn, int64_t nt,
                          double* partial);
void launch_form_q(hipStream_t s, const FormQDesc* d, int n, int maxrows);
}  // namespace qrvie

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Device allocations released together.  Host staging copies of uploaded data are kept
// alive until the stream has been synchronised (asynchronous copies may read them late).
struct Arena {
    qrvie_ctx* ctx;
    std::vector<std::pair<void*, size_t>> bufs;
    std::vector<std::vector<char>> staged;
    explicit Arena(qrvie_ctx* c) : ctx(c) {}
    ~Arena() { release(); }
    void release() {
        if (!bufs.empty() || !staged.empty()) (void)hipStreamSynchronize(ctx->stream);
        for (auto& b : bufs) dfree(ctx, b.first, b.second);
        bufs.clear();
        staged.clear();
    }
    template <class T>
    qrvie_status alloc(T** p, size_t count, const char* what) {
        *p = nullptr;
        if (count == 0) return QRVIE_OK;
        qrvie_status st = dalloc(ctx, (void**)p, sizeof(T) * count, what);
        if (st == QRVIE_OK) bufs.push_back({(void*)*p, sizeof(T) * count});
        return st;
    }
    template <class T>
    qrvie_status upload(T** p, const std::vector<T>& v, const char* what) {
        qrvie_status st = alloc(p, v.size(), what);
        if (st != QRVIE_OK || v.empty()) return st;
        staged.emplace_back(reinterpret_cast<const char*>(v.data()),
                            reinterpret_cast<const char*>(v.data()) + sizeof(T) * v.size());
        return hip_check(ctx, hipMemcpyAsync(*p, staged.back().data(), sizeof(T) * v.size(), hipMemcpyHostToDevice,
                                             ctx->stream), what);
    }
};

template <class T>
qrvie_status download(qrvie_ctx* ctx, std::vector<T>& v, const T* d, size_t n, const char* what) {
    v.resize(n);
    if (n == 0) return QRVIE_OK;
    qrvie_status st = hip_check(ctx, hipMemcpyAsync(v.data(), d, sizeof(T) * n, hipMemcpyDeviceToHost, ctx->stream), what);
    if (st == QRVIE_OK) st = hip_check(ctx, hipStreamSynchronize(ctx->stream), what);
    return st;
}

#define CHECK(x)                              \
    do {                                      \
        qrvie_status _s = (x);                \
        if (_s != QRVIE_OK) return _s;        \
    } while (0)

struct Factor {            // compact factors of one primary block
    c128* Q = nullptr;     // m x r, ld m
    c128* R = nullptr;     // r x n, ld r
    float2* Q32 = nullptr; // the same rounded to complex64 (operators that keep only complex64)
    float2* R32 = nullptr;
    int32_t rank = 0;
    double rel_err = 0.0;
};

// Tile list of a batch of GEMM descriptors.
void gemm_tiles(const std::vector<GemmDesc>& d, std::vector<int32_t>& td, std::vector<int32_t>& tmn,
                std::vector<int32_t>* first = nullptr, std::vector<int32_t>* count = nullptr) {
    td.clear();
    tmn.clear();
    if (first) first->clear();
    if (count) count->clear();
    for (size_t i = 0; i < d.size(); ++i) {
        const int nm = (d[i].m + 63) / 64, nn = (d[i].n + 63) / 64;
        if (first) first->push_back((int32_t)td.size());
        if (count) count->push_back(nm * nn);
        for (int a = 0; a < nm; ++a)
            for (int b = 0; b < nn; ++b) {
                td.push_back((int32_t)i);
                tmn.push_back((a << 16) | b);
            }
    }
}

constexpr int kDirectMaxParticles = 2;   // both sides at most this many particles: direct QRCP
constexpr int kSketchStart = 128;
constexpr int kMaxSketch = 512;          // widest sketch the CGS2 kernel orthonormalises
constexpr int kAcaStart = 256;           // crosses per block at first (doubled while all are used)
constexpr double kAcaEps = 0.05;         // stopping tolerance of the crosses, relative to eps
constexpr int64_t kAcaWide = 2 * 4608;   // rows plus columns above which a block gets 16 waves
constexpr int kPhaseWaves = 4;           // waves per strip in the product kernels
constexpr int64_t kAlign = 16;           // R-panel leading dimension multiple: 128 B in complex64, 256 B in complex128

struct Builder {
    qrvie_op* op;
    qrvie_ctx* ctx;
    const qrvie_geom* g;
    std::vector<BlockRec> blocks;
    std::vector<Factor> fac;                        // per block (primary only filled)
    std::vector<std::pair<void*, size_t>> segments; // compact factor storage
    double eps;
    bool compact32 = false;                         // round each chunk's compact factors to complex64
    int64_t n_aca = 0, n_resumed = 0, n_retried = 0; // cross approximation counters
    double aca_eps0 = 0.0;                          // the crosses' first stopping tolerance
    // The materialised blocks of a chunk and the direct blocks' working copies live in two
    // grow-only buffers kept across chunks: allocating and releasing tens of GB per chunk
    // cost about as much host time as the chunk's kernels.
    // slots: 0 blocks / crosses U, 1 work copies / crosses V, 2 bases of the crosses, 3 projected
    // rows, 4 complex128 staging of compact factors that are kept as complex64
    static constexpr int kPools = 5;
    c128* pool[kPools] = {};
    size_t pool_elems[kPools] = {};

    qrvie_status pooled(int which, size_t elems, c128** p, const char* what) {
        *p = nullptr;
        if (elems == 0) return QRVIE_OK;
        if (elems > pool_elems[which]) {
            if (pool[which]) {
                (void)hipStreamSynchronize(ctx->stream);
                dfree(ctx, pool[which], pool_elems[which] * sizeof(c128));
            }
            pool[which] = nullptr;
            pool_elems[which] = 0;
            CHECK(dalloc(ctx, (void**)&pool[which], elems * sizeof(c128), what));
            pool_elems[which] = elems;
        }
        *p = pool[which];
        return QRVIE_OK;
    }
    void release_pools() {
        bool any = false;
        for (int w = 0; w < kPools; ++w) any = any || pool[w];
        if (!any) return;
        (void)hipStreamSynchronize(ctx->stream);
        for (int w = 0; w < kPools; ++w) {
            if (pool[w]) dfree(ctx, pool[w], pool_elems[w] * sizeof(c128));
            pool[w] = nullptr;
            pool_elems[w] = 0;
        }
    }
    ~Builder() { release_pools(); }

    qrvie_status new_segment(size_t elems, c128** p) {
        *p = nullptr;
        if (elems == 0) return QRVIE_OK;
        CHECK(dalloc(ctx, (void**)p, elems * sizeof(c128), "compact factors"));
        segments.push_back({(void*)*p, elems * sizeof(c128)});
        return QRVIE_OK;
    }

    // When the operator keeps only complex64 factors, round a chunk's compact factors (blocks
    // `sel` of `ids`, at offsets qo / ro in seg) as soon as they are certified, so the
    // complex128 ones never accumulate over the whole build.
    qrvie_status round_segment(c128* seg, int64_t ctot, const std::vector<size_t>& sel, const std::vector<int32_t>& ids,
                               const std::vector<int64_t>& qo, const std::vector<int64_t>& ro) {
        if (!compact32 || ctot <= 0) return QRVIE_OK;
        float2* seg32 = nullptr;
        CHECK(dalloc(ctx, (void**)&seg32, sizeof(float2) * (size_t)ctot, "compact complex64 factors"));
        segments.push_back({(void*)seg32, sizeof(float2) * (size_t)ctot});
        launch_to_c64(ctx->stream, seg, seg32, ctot);
        CHECK(hip_check(ctx, hipStreamSynchronize(ctx->stream), "compact complex64 factors"));
        for (size_t k = 0; k < segments.size(); ++k)
            if (segments[k].first == (void*)seg) {
                dfree(ctx, seg, segments[k].second);
                segments.erase(segments.begin() + (int64_t)k);
                break;
            }
        for (size_t i : sel) {
            Factor& f = fac[ids[i]];
            f.Q32 = seg32 + qo[i];
            f.R32 = seg32 + ro[i];
            f.Q = f.R = nullptr;
        }
        return QRVIE_OK;
    }

    qrvie_status compress_aca(const std::vector<int32_t>& ids, const std::vector<int32_t>& kmx,
                              const std::vector<double>& eaca, std::vector<int32_t>& fallback);

    // Compress the primary blocks `ids`; sketch width k[i] (0 = direct QRCP).
    qrvie_status compress(const std::vector<int32_t>& ids, const std::vector<int32_t>& kw) {
        hipStream_t s = ctx->stream;
        Arena ar(ctx);
        const size_t nb = ids.size();
        std::vector<int64_t> m(nb), n(nb), boff(nb);
        int64_t btot = 0;
        for (size_t i = 0; i < nb; ++i) {
            const BlockRec& b = blocks[ids[i]];
            m[i] = (int64_t)b.rn * kNp;
            n[i] = (int64_t)b.cn * kNp;
            boff[i] = btot;
            btot += m[i] * n[i];
        }
        c128* dB;
        CHECK(pooled(0, (size_t)btot, &dB, "block buffer"));
        {   // assembly
            std::vector<AsmDesc> ad(nb);
            std::vector<int32_t> wb, wc;
            for (size_t i = 0; i < nb; ++i) {
                const BlockRec& b = blocks[ids[i]];
                ad[i] = AsmDesc{dB + boff[i], m[i], b.r0, b.rn, b.c0, b.cn};
                for (int q = 0; q < b.cn; ++q) { wb.push_back((int32_t)i); wc.push_back(q); }
            }
            AsmDesc* dad; int32_t *dwb, *dwc;
            CHECK(ar.upload(&dad, ad, "asm descs"));
            CHECK(ar.upload(&dwb, wb, "asm work"));
            CHECK(ar.upload(&dwc, wc, "asm work"));
            launch_assemble_far(s, g, dad, dwb, dwc, (int64_t)wb.size());
            CHECK(hip_check(ctx, hipGetLastError(), "assemble far"));
        }
        std::vector<size_t> dir, sk;
        for (size_t i = 0; i < nb; ++i) (kw[i] == 0 ? dir : sk).push_back(i);
        // Direct blocks are factorised in place, so they get a second copy (assembled
        // again, which is cheaper than storing it) while B stays the certification reference.
        std::vector<int64_t> aoff(nb, 0);
        c128* dA = nullptr;
        if (!dir.empty()) {
            int64_t atot = 0;
            std::vector<AsmDesc> ad;
            std::vector<int32_t> wb, wc;
            for (size_t i : dir) {
                const BlockRec& b = blocks[ids[i]];
                aoff[i] = atot;
                atot += m[i] * n[i];
            }
            CHECK(pooled(1, (size_t)atot, &dA, "factorisation buffer"));
            for (size_t i : dir) {
                const BlockRec& b = blocks[ids[i]];
                ad.push_back(AsmDesc{dA + aoff[i], m[i], b.r0, b.rn, b.c0, b.cn});
                for (int q = 0; q < b.cn; ++q) { wb.push_back((int32_t)ad.size() - 1); wc.push_back(q); }
            }
            AsmDesc* dad; int32_t *dwb, *dwc;
            CHECK(ar.upload(&dad, ad, "asm descs"));
            CHECK(ar.upload(&dwb, wb, "asm work"));
            CHECK(ar.upload(&dwc, wc, "asm work"));
            launch_assemble_far(s, g, dad, dwb, dwc, (int64_t)wb.size());
            CHECK(hip_check(ctx, hipGetLastError(), "assemble far (work copy)"));
        }

        // per-block results
        int32_t* d_rank; double *d_trail, *d_norm2;
        CHECK(ar.alloc(&d_rank, nb, "ranks"));
        CHECK(ar.alloc(&d_trail, nb, "trail"));
        CHECK(ar.alloc(&d_norm2, nb, "norm2"));

        // QRCP workspaces sized per block
        std::vector<int64_t> wsn(nb), wsk(nb);
        int64_t tot_n = 0, tot_k = 0;
        // sketch buffers
        std::vector<int64_t> yoff(nb, 0), woff(nb, 0), kk(nb, 0);
        int64_t ytot = 0;
        for (size_t i : sk) {
            kk[i] = std::min<int64_t>(kw[i], std::min(m[i], n[i]));
            yoff[i] = ytot;
            ytot += m[i] * kk[i];
        }
        c128* dY = nullptr;
        CHECK(ar.alloc(&dY, ytot, "sketch"));
        std::vector<int32_t> kept(nb, 0);
        std::vector<double> normB2(nb, 0.0);
        if (!sk.empty()) {
            // Y = B Omega
            std::vector<GemmDesc> gd;
            for (size_t i : sk)
                gd.push_back(GemmDesc{dB + boff[i], m[i], nullptr, 0, dY + yoff[i], m[i], (int32_t)m[i], (int32_t)kk[i],
                                      (int32_t)n[i], op->opts.seed * 0x9E3779B97F4A7C15ull + (uint64_t)ids[i], nullptr});
            std::vector<int32_t> td, tmn;
            gemm_tiles(gd, td, tmn);
            GemmDesc* dgd; int32_t *dtd, *dtmn;
            CHECK(ar.upload(&dgd, gd, "gemm descs"));
            CHECK(ar.upload(&dtd, td, "gemm tiles"));
            CHECK(ar.upload(&dtmn, tmn, "gemm tiles"));
            launch_gemm(s, 2, dgd, dtd, dtmn, (int64_t)td.size());
            // ||B||^2: every block split into pieces of at most 1 M entries (one workgroup each),
            // then a fixed-order sum per block
            std::vector<const c128*> ptr;
            std::vector<int64_t> len;
            std::vector<int32_t> pfirst, pcount;
            constexpr int64_t kPiece = (int64_t)1 << 20;
            for (size_t i : sk) {
                pfirst.push_back((int32_t)ptr.size());
                const int64_t tot = m[i] * n[i];
                for (int64_t o = 0; o < tot; o += kPiece) {
                    ptr.push_back(dB + boff[i] + o);
                    len.push_back(std::min(kPiece, tot - o));
                }
                pcount.push_back((int32_t)ptr.size() - pfirst.back());
            }
            const c128** dptr; int64_t* dlen; double *dpn2, *dn2; int32_t *dpf, *dpc;
            CHECK(ar.upload(&dptr, ptr, "frob ptrs"));
            CHECK(ar.upload(&dlen, len, "frob lens"));
            CHECK(ar.upload(&dpf, pfirst, "frob pieces"));
            CHECK(ar.upload(&dpc, pcount, "frob pieces"));
            CHECK(ar.alloc(&dpn2, ptr.size(), "frob partials"));
            CHECK(ar.alloc(&dn2, sk.size(), "frob out"));
            launch_frob2(s, dptr, dlen, dpn2, (int)ptr.size());
            launch_sum_partials(s, dpn2, dpf, dpc, dn2, (int)sk.size());
            // orthonormal basis of Y
            std::vector<Cgs2Desc> cd;
            int32_t* dkept;
            CHECK(ar.alloc(&dkept, sk.size(), "kept"));
            for (size_t a = 0; a < sk.size(); ++a) {
                const size_t i = sk[a];
                cd.push_back(Cgs2Desc{dY + yoff[i], (int32_t)m[i], (int32_t)kk[i], (int32_t)m[i], 1e-12, dkept + a});
            }
            Cgs2Desc* dcd;
            CHECK(ar.upload(&dcd, cd, "cgs2 descs"));
            int kmax = 0;
            for (const Cgs2Desc& c : cd) kmax = std::max(kmax, c.k);
            launch_cgs2(s, dcd, (int)cd.size(), kmax);
            CHECK(hip_check(ctx, hipGetLastError(), "sketch"));
            std::vector<int32_t> hk;
            std::vector<double> hn2;
            CHECK(download(ctx, hk, dkept, sk.size(), "kept"));
            CHECK(download(ctx, hn2, dn2, sk.size(), "norms"));
            for (size_t a = 0; a < sk.size(); ++a) { kept[sk[a]] = hk[a]; normB2[sk[a]] = hn2[a]; }
        }
        int64_t wtot = 0;
        for (size_t i : sk) { woff[i] = wtot; wtot += (int64_t)kept[i] * n[i]; }
        c128* dW = nullptr;
        CHECK(ar.alloc(&dW, wtot, "projected block"));
        if (!sk.empty()) {
            std::vector<GemmDesc> gd;
            for (size_t i : sk)
                gd.push_back(GemmDesc{dY + yoff[i], m[i], dB + boff[i], m[i], dW + woff[i], kept[i], kept[i],
                                      (int32_t)n[i], (int32_t)m[i], 0, nullptr});
            std::vector<int32_t> td, tmn;
            gemm_tiles(gd, td, tmn);
            GemmDesc* dgd; int32_t *dtd, *dtmn;
            CHECK(ar.upload(&dgd, gd, "gemm descs"));
            CHECK(ar.upload(&dtd, td, "gemm tiles"));
            CHECK(ar.upload(&dtmn, tmn, "gemm tiles"));
            launch_gemm(s, 1, dgd, dtd, dtmn, (int64_t)td.size());
        }
        // QRCP: direct on B, sketch on W
        std::vector<QrcpDesc> qd(nb);
        std::vector<int64_t> am(nb), an(nb);
        for (size_t i = 0; i < nb; ++i) {
            am[i] = kw[i] == 0 ? m[i] : kept[i];
            an[i] = n[i];
            wsn[i] = tot_n; tot_n += an[i];
            wsk[i] = tot_k; tot_k += std::min(am[i], an[i]);
        }
        double* dcn; int32_t* dperm; double* dtau; c128* dwtop; double* dtol2;
        CHECK(ar.alloc(&dcn, std::max<int64_t>(tot_n, 1), "qrcp norms"));
        CHECK(ar.alloc(&dperm, std::max<int64_t>(tot_n, 1), "qrcp perm"));
        CHECK(ar.alloc(&dtau, std::max<int64_t>(tot_k, 1), "qrcp tau"));
        CHECK(ar.alloc(&dwtop, std::max<int64_t>(tot_k, 1), "qrcp w"));
        CHECK(ar.alloc(&dtol2, std::max<size_t>(nb, 1), "qrcp tolerances"));
        const double rel2 = (0.95 * eps) * (0.95 * eps);
        int maxrows_dir = 0, maxrows_sk = 0, maxcols_sk = 0, maxsteps_sk = 0;
        std::vector<QrcpDesc> qdir, qsk;
        for (size_t i = 0; i < nb; ++i) {
            QrcpDesc q{};
            q.A = kw[i] == 0 ? dA + aoff[i] : dW + woff[i];
            q.m = (int32_t)am[i];
            q.n = (int32_t)an[i];
            q.lda = (int32_t)std::max<int64_t>(am[i], 1);
            q.kmax = (int32_t)std::min(am[i], an[i]);
            q.colnorm2 = dcn + wsn[i];
            q.perm = dperm + wsn[i];
            q.tau = dtau + wsk[i];
            q.wtop = dwtop + wsk[i];
            q.rel2 = rel2;
            if (kw[i] == 0) { q.base2 = 0.0; q.sub2 = 0.0; }
            else { q.base2 = normB2[i]; q.sub2 = -1.0; }     // sub2 < 0: subtract base2 - ||W||^2
            q.rank_out = d_rank + i;
            q.trail2_out = d_trail + i;
            q.norm2_out = d_norm2 + i;
            q.tol2_state = dtol2 + i;
            qd[i] = q;
            if (kw[i] == 0) {
                qdir.push_back(q);
                maxrows_dir = std::max<int>(maxrows_dir, q.m);
            } else {
                qsk.push_back(q);
                maxrows_sk = std::max<int>(maxrows_sk, q.m);
                maxcols_sk = std::max<int>(maxcols_sk, q.n);
                maxsteps_sk = std::max<int>(maxsteps_sk, std::min(q.kmax, std::min(q.m, q.n)));
            }
        }
        QrcpDesc *dqdir, *dqsk;
        CHECK(ar.upload(&dqdir, qdir, "qrcp descs"));
        CHECK(ar.upload(&dqsk, qsk, "qrcp descs"));
        launch_qrcp(s, dqdir, (int)qdir.size(), maxrows_dir);
        launch_qrcp_stepped(s, dqsk, (int)qsk.size(), maxrows_sk, maxcols_sk, maxsteps_sk);
        CHECK(hip_check(ctx, hipGetLastError(), "qrcp"));
        std::vector<int32_t> rank;
        std::vector<double> n2;
        CHECK(download(ctx, rank, d_rank, nb, "ranks"));
        CHECK(download(ctx, n2, d_norm2, nb, "norms"));
        for (size_t i = 0; i < nb; ++i)
            if (kw[i] == 0) normB2[i] = n2[i];

        // compact storage
        int64_t ctot = 0;
        std::vector<int64_t> qo(nb), ro(nb);
        for (size_t i = 0; i < nb; ++i) {
            qo[i] = ctot; ctot += m[i] * rank[i];
            ro[i] = ctot; ctot += (int64_t)rank[i] * n[i];
        }
        c128* seg;
        if (compact32) CHECK(pooled(4, (size_t)ctot, &seg, "compact factor staging"));
        else CHECK(new_segment(ctot, &seg));
        // Q
        {
            std::vector<FormQDesc> fdir, fsk;
            int64_t qwtot = 0;
            std::vector<int64_t> qwo(nb, 0);
            for (size_t i : sk) { qwo[i] = qwtot; qwtot += (int64_t)kept[i] * rank[i]; }
            c128* dQW;
            CHECK(ar.alloc(&dQW, qwtot, "sketch Q"));
            for (size_t i = 0; i < nb; ++i) {
                if (rank[i] == 0) continue;
                if (kw[i] == 0)
                    fdir.push_back(FormQDesc{dA + aoff[i], (int32_t)m[i], (int32_t)m[i], rank[i], dtau + wsk[i],
                                             dwtop + wsk[i], seg + qo[i], (int32_t)m[i]});
                else
                    fsk.push_back(FormQDesc{dW + woff[i], kept[i], std::max(kept[i], 1), rank[i], dtau + wsk[i],
                                            dwtop + wsk[i], dQW + qwo[i], std::max(kept[i], 1)});
            }
            FormQDesc *dfd, *dfs;
            CHECK(ar.upload(&dfd, fdir, "formq descs"));
            CHECK(ar.upload(&dfs, fsk, "formq descs"));
            launch_form_q(s, dfd, (int)fdir.size(), maxrows_dir);
            launch_form_q(s, dfs, (int)fsk.size(), maxrows_sk);
            if (!sk.empty()) {
                std::vector<GemmDesc> gd;
                for (size_t i : sk)
                    if (rank[i] > 0)
                        gd.push_back(GemmDesc{dY + yoff[i], m[i], dQW + qwo[i], std::max(kept[i], 1), seg + qo[i], m[i],
                                              (int32_t)m[i], rank[i], kept[i], 0, nullptr});
                std::vector<int32_t> td, tmn;
                gemm_tiles(gd, td, tmn);
                GemmDesc* dgd; int32_t *dtd, *dtmn;
                CHECK(ar.upload(&dgd, gd, "gemm descs"));
                CHECK(ar.upload(&dtd, td, "gemm tiles"));
                CHECK(ar.upload(&dtmn, tmn, "gemm tiles"));
                launch_gemm(s, 0, dgd, dtd, dtmn, (int64_t)td.size());
            }
            CHECK(hip_check(ctx, hipGetLastError(), "form Q"));
            // R
            std::vector<ExtractRDesc> ed;
            for (size_t i = 0; i < nb; ++i)
                if (rank[i] > 0)
                    ed.push_back(ExtractRDesc{qd[i].A, qd[i].lda, rank[i], (int32_t)n[i], qd[i].perm, seg + ro[i], rank[i]});
            ExtractRDesc* ded;
            CHECK(ar.upload(&ded, ed, "extract descs"));
            launch_extract_r(s, ded, (int)ed.size());
            CHECK(hip_check(ctx, hipGetLastError(), "extract R"));
        }
        // certification: ||B - Q R||_F^2 from B itself
        {
            std::vector<GemmDesc> gd;
            for (size_t i = 0; i < nb; ++i)
                gd.push_back(GemmDesc{seg + qo[i], m[i], seg + ro[i], std::max(rank[i], 1), dB + boff[i], m[i],
                                      (int32_t)m[i], (int32_t)n[i], rank[i], 0, nullptr});
            std::vector<int32_t> td, tmn, first, count;
            gemm_tiles(gd, td, tmn, &first, &count);
            GemmDesc* dgd; int32_t *dtd, *dtmn, *dfirst, *dcount; double *dpart, *derr;
            CHECK(ar.upload(&dgd, gd, "cert descs"));
            CHECK(ar.upload(&dtd, td, "cert tiles"));
            CHECK(ar.upload(&dtmn, tmn, "cert tiles"));
            CHECK(ar.upload(&dfirst, first, "cert tiles"));
            CHECK(ar.upload(&dcount, count, "cert tiles"));
            CHECK(ar.alloc(&dpart, std::max<size_t>(td.size(), 1), "cert partials"));
            CHECK(ar.alloc(&derr, nb, "cert err"));
            launch_gemm_residual(s, dgd, dtd, dtmn, (int64_t)td.size(), dpart);
            launch_sum_partials(s, dpart, dfirst, dcount, derr, (int)nb);
            CHECK(hip_check(ctx, hipGetLastError(), "certify"));
            std::vector<double> err2;
            CHECK(download(ctx, err2, derr, nb, "cert err"));
            for (size_t i = 0; i < nb; ++i) {
                Factor& f = fac[ids[i]];
                f.Q = seg + qo[i];
                f.R = seg + ro[i];
                f.rank = rank[i];
                f.rel_err = normB2[i] > 0.0 ? std::sqrt(err2[i] / normB2[i]) : 0.0;
            }
        }
        {
            std::vector<size_t> all(nb);
            for (size_t i = 0; i < nb; ++i) all[i] = i;
            CHECK(round_segment(seg, ctot, all, ids, qo, ro));
        }
        // retry blocks that missed eps with a wider sketch
        std::vector<int32_t> rids, rk;
        for (size_t i = 0; i < nb; ++i) {
            if (fac[ids[i]].rel_err <= eps) continue;
            const int64_t full = std::min<int64_t>(std::min(m[i], n[i]), kMaxSketch);
            if (kw[i] == 0 || kk[i] >= full) {
                set_err(ctx, "compression: block " + std::to_string(ids[i]) + " misses eps: rel err " +
                                 std::to_string(fac[ids[i]].rel_err) + ", ||B||^2 " + std::to_string(normB2[i]) +
                                 ", rank " + std::to_string(rank[i]) + ", m " + std::to_string(m[i]) + ", n " +
                                 std::to_string(n[i]) + ", sketch " + std::to_string(kk[i]));
                return QRVIE_ERR_DEVICE;
            }
            rids.push_back(ids[i]);
            rk.push_back((int32_t)std::min<int64_t>(2 * kk[i], full));
        }
        ar.release();
        if (!rids.empty()) return compress(rids, rk);
        return QRVIE_OK;
    }
};

// Working buffers of one chunk of cross-approximated blocks, in complex128 elements: U and V
// (m + n) kmax, the orthonormalised copy of U (m kmax) and the projected rows (kmax n).
int64_t aca_elems(const BlockRec& b, int kmax) { return 2 * ((int64_t)b.rn + b.cn) * kNp * kmax; }

// Compression through cross approximation (the default): the block B is never formed.
//  1. U V ~ B from k pivot rows and columns of B (k_aca, stopping tolerance eps_aca);
//  2. Y = orth(U) (CGS2), T = Y^H U, W = T V (so Y W = U V);
//  3. truncated pivoted QR of W at 0.9 eps relative to ||W||_F: W ~ Q_W R, Q = Y Q_W;
//  4. certification of ||B - Q R||_F against the entries of B generated again, tile by tile.
// A block that misses eps is redone with a tighter eps_aca (and twice the crosses when it
// used them all); after that the sketch path compresses it from the assembled block.
qrvie_status Builder::compress_aca(const std::vector<int32_t>& ids, const std::vector<int32_t>& kmx,
                                   const std::vector<double>& eaca, std::vector<int32_t>& fallback) {
    hipStream_t s = ctx->stream;
    Arena ar(ctx);
    for (int32_t id : ids)
        if ((int64_t)blocks[id].rn * kNp > kAcaMaxRows || kmx.empty()) {
            set_err(ctx, "cross approximation: block rows beyond the row flags");
            return QRVIE_ERR_INVALID_ARG;
        }
    const size_t nb = ids.size();
    std::vector<int64_t> m(nb), n(nb), uo(nb), vo(nb);
    int64_t utot = 0, vtot = 0;
    for (size_t i = 0; i < nb; ++i) {
        const BlockRec& b = blocks[ids[i]];
        m[i] = (int64_t)b.rn * kNp;
        n[i] = (int64_t)b.cn * kNp;
        uo[i] = utot; utot += m[i] * kmx[i];
        vo[i] = vtot; vtot += n[i] * kmx[i];
    }
    c128 *dU0, *dV0;
    CHECK(pooled(0, (size_t)utot, &dU0, "cross approximation columns"));
    CHECK(pooled(1, (size_t)vtot, &dV0, "cross approximation rows"));
    std::vector<c128*> U(nb), V(nb);                  // per block: m x cap (ld m), cap x n (by rows, ld n)
    std::vector<int32_t> cap(kmx);
    for (size_t i = 0; i < nb; ++i) { U[i] = dU0 + uo[i]; V[i] = dV0 + vo[i]; }
    int32_t *dk, *dpiv; double* dstate;
    CHECK(ar.alloc(&dk, nb, "cross approximation ranks"));
    CHECK(ar.alloc(&dpiv, nb * (size_t)kAcaMaxRank, "pivot rows"));
    CHECK(ar.alloc(&dstate, 2 * nb, "cross approximation state"));
    std::vector<int32_t> k(nb, 0);
    std::vector<size_t> run(nb);
    for (size_t i = 0; i < nb; ++i) run[i] = i;
    // blocks that use every cross before meeting eps_aca continue in buffers twice as wide
    while (!run.empty()) {
        // blocks of more than kAcaWide rows plus columns get 16 waves (their steps stream the
        // longest rows and columns), the others 4
        std::vector<AcaDesc> ad[2];
        for (size_t i : run) {
            const BlockRec& b = blocks[ids[i]];
            ad[m[i] + n[i] > kAcaWide].push_back(AcaDesc{b.r0, b.rn, b.c0, b.cn, U[i], V[i], cap[i], eaca[i], dk + i,
                                                         k[i], dpiv + i * (size_t)kAcaMaxRank, dstate + 2 * i});
        }
        for (int w = 0; w < 2; ++w) {
            AcaDesc* dad;
            CHECK(ar.upload(&dad, ad[w], "aca descs"));
            launch_aca(s, g, dad, (int)ad[w].size(), w == 1);
        }
        CHECK(hip_check(ctx, hipGetLastError(), "cross approximation"));
        std::vector<int32_t> hk;
        CHECK(download(ctx, hk, dk, nb, "cross approximation ranks"));
        std::vector<size_t> more;
        for (size_t i : run) {
            k[i] = hk[i];
            const int32_t full = (int32_t)std::min<int64_t>(std::min(m[i], n[i]), kAcaMaxRank);
            if (k[i] >= cap[i] && cap[i] < full) more.push_back(i);
        }
        n_resumed += (int64_t)more.size();
        for (size_t i : more) {
            const int32_t c2 = (int32_t)std::min<int64_t>(2 * (int64_t)cap[i], std::min<int64_t>(std::min(m[i], n[i]), kAcaMaxRank));
            c128 *u2, *v2;
            CHECK(ar.alloc(&u2, (size_t)(m[i] * c2), "cross approximation columns"));
            CHECK(ar.alloc(&v2, (size_t)(n[i] * c2), "cross approximation rows"));
            CHECK(hip_check(ctx, hipMemcpyAsync(u2, U[i], sizeof(c128) * m[i] * k[i], hipMemcpyDeviceToDevice, s),
                            "cross approximation columns"));
            CHECK(hip_check(ctx, hipMemcpyAsync(v2, V[i], sizeof(c128) * n[i] * k[i], hipMemcpyDeviceToDevice, s),
                            "cross approximation rows"));
            U[i] = u2;
            V[i] = v2;
            cap[i] = c2;
        }
        run = more;
    }
    std::vector<size_t> act;
    for (size_t i = 0; i < nb; ++i) {
        if (k[i] == 0) fallback.push_back(ids[i]);
        else act.push_back(i);
    }
    const size_t na = act.size();
    std::vector<int64_t> yo(nb, 0), wo(nb, 0);
    int64_t ytot = 0;
    for (size_t i : act) { yo[i] = ytot; ytot += m[i] * k[i]; }
    c128* dY;
    CHECK(pooled(2, (size_t)ytot, &dY, "cross approximation basis"));
    std::vector<int32_t> kept(nb, 0);
    if (na) {
        for (size_t i : act)
            CHECK(hip_check(ctx, hipMemcpyAsync(dY + yo[i], U[i], sizeof(c128) * m[i] * k[i],
                                                hipMemcpyDeviceToDevice, s), "basis copy"));
        std::vector<Cgs2Desc> cd;
        int32_t* dkept;
        CHECK(ar.alloc(&dkept, na, "kept"));
        int kmax = 0;
        for (size_t a = 0; a < na; ++a) {
            const size_t i = act[a];
            cd.push_back(Cgs2Desc{dY + yo[i], (int32_t)m[i], k[i], (int32_t)m[i], 1e-12, dkept + a});
            kmax = std::max(kmax, k[i]);
        }
        Cgs2Desc* dcd;
        CHECK(ar.upload(&dcd, cd, "cgs2 descs"));
        launch_cgs2(s, dcd, (int)na, kmax);
        CHECK(hip_check(ctx, hipGetLastError(), "cross approximation basis"));
        std::vector<int32_t> hk;
        CHECK(download(ctx, hk, dkept, na, "kept"));
        for (size_t a = 0; a < na; ++a) kept[act[a]] = hk[a];
    }
    // T = Y^H U (kept x k), then W = T V (kept x n)
    int64_t ttot = 0, wtot = 0;
    std::vector<int64_t> to(nb, 0);
    for (size_t i : act) {
        to[i] = ttot; ttot += (int64_t)kept[i] * k[i];
        wo[i] = wtot; wtot += (int64_t)kept[i] * n[i];
    }
    c128 *dT, *dW;
    CHECK(ar.alloc(&dT, ttot, "cross approximation T"));
    CHECK(pooled(3, (size_t)wtot, &dW, "projected rows"));
    auto gemm = [&](int mode, const std::vector<GemmDesc>& gd) -> qrvie_status {
        if (gd.empty()) return QRVIE_OK;
        std::vector<int32_t> td, tmn;
        gemm_tiles(gd, td, tmn);
        GemmDesc* dgd; int32_t *dtd, *dtmn;
        CHECK(ar.upload(&dgd, gd, "gemm descs"));
        CHECK(ar.upload(&dtd, td, "gemm tiles"));
        CHECK(ar.upload(&dtmn, tmn, "gemm tiles"));
        launch_gemm(s, mode, dgd, dtd, dtmn, (int64_t)td.size());
        return hip_check(ctx, hipGetLastError(), "gemm");
    };
    {
        std::vector<GemmDesc> g1, g0;
        for (size_t i : act) {
            if (kept[i] == 0) continue;
            g1.push_back(GemmDesc{dY + yo[i], m[i], U[i], m[i], dT + to[i], kept[i], kept[i], k[i],
                                  (int32_t)m[i], 0, nullptr});
            g0.push_back(GemmDesc{dT + to[i], kept[i], V[i], n[i], dW + wo[i], kept[i], kept[i],
                                  (int32_t)n[i], k[i], 0, nullptr});
        }
        CHECK(gemm(1, g1));
        CHECK(gemm(4, g0));
    }
    // truncated pivoted QR of W
    std::vector<int64_t> wsn(nb, 0), wsk(nb, 0);
    int64_t tot_n = 0, tot_k = 0;
    for (size_t i : act) {
        wsn[i] = tot_n; tot_n += n[i];
        wsk[i] = tot_k; tot_k += std::min<int64_t>(kept[i], n[i]);
    }
    double *dcn, *dtau, *dtol2, *dtrail, *dn2; int32_t *dperm, *drank; c128* dwtop;
    CHECK(ar.alloc(&dcn, std::max<int64_t>(tot_n, 1), "qrcp norms"));
    CHECK(ar.alloc(&dperm, std::max<int64_t>(tot_n, 1), "qrcp perm"));
    CHECK(ar.alloc(&dtau, std::max<int64_t>(tot_k, 1), "qrcp tau"));
    CHECK(ar.alloc(&dwtop, std::max<int64_t>(tot_k, 1), "qrcp w"));
    CHECK(ar.alloc(&dtol2, std::max<size_t>(nb, 1), "qrcp tolerances"));
    CHECK(ar.alloc(&dtrail, std::max<size_t>(nb, 1), "trail"));
    CHECK(ar.alloc(&dn2, std::max<size_t>(nb, 1), "norm2"));
    CHECK(ar.alloc(&drank, std::max<size_t>(nb, 1), "ranks"));
    CHECK(hip_check(ctx, hipMemsetAsync(drank, 0, sizeof(int32_t) * nb, s), "ranks"));
    std::vector<QrcpDesc> qd;
    std::vector<size_t> qi;
    int maxrows = 0, maxcols = 0, maxsteps = 0;
    for (size_t i : act) {
        if (kept[i] == 0) continue;
        QrcpDesc q{};
        q.A = dW + wo[i];
        q.m = kept[i];
        q.n = (int32_t)n[i];
        q.lda = kept[i];
        q.kmax = (int32_t)std::min<int64_t>(kept[i], n[i]);
        q.colnorm2 = dcn + wsn[i];
        q.perm = dperm + wsn[i];
        q.tau = dtau + wsk[i];
        q.wtop = dwtop + wsk[i];
        q.rel2 = (0.9 * eps) * (0.9 * eps);
        q.base2 = 0.0;
        q.sub2 = 0.0;
        q.rank_out = drank + i;
        q.trail2_out = dtrail + i;
        q.norm2_out = dn2 + i;
        q.tol2_state = dtol2 + i;
        qd.push_back(q);
        qi.push_back(i);
        maxrows = std::max(maxrows, q.m);
        maxcols = std::max(maxcols, q.n);
        maxsteps = std::max(maxsteps, q.kmax);
    }
    QrcpDesc* dqd;
    CHECK(ar.upload(&dqd, qd, "qrcp descs"));
    launch_qrcp_stepped(s, dqd, (int)qd.size(), maxrows, maxcols, maxsteps);
    CHECK(hip_check(ctx, hipGetLastError(), "qrcp"));
    std::vector<int32_t> rank;
    CHECK(download(ctx, rank, drank, nb, "ranks"));
    // compact factors: Q = Y Q_W, R from W
    int64_t ctot = 0;
    std::vector<int64_t> qo(nb, 0), ro(nb, 0);
    for (size_t i : act) {
        qo[i] = ctot; ctot += m[i] * rank[i];
        ro[i] = ctot; ctot += (int64_t)rank[i] * n[i];
    }
    c128* seg;
    if (compact32) CHECK(pooled(4, (size_t)ctot, &seg, "compact factor staging"));
    else CHECK(new_segment(ctot, &seg));
    {
        int64_t qwtot = 0;
        std::vector<int64_t> qwo(nb, 0);
        for (size_t i : act) { qwo[i] = qwtot; qwtot += (int64_t)kept[i] * rank[i]; }
        c128* dQW;
        CHECK(ar.alloc(&dQW, qwtot, "projected Q"));
        std::vector<FormQDesc> fd;
        std::vector<GemmDesc> gd;
        std::vector<ExtractRDesc> ed;
        for (size_t a = 0; a < qd.size(); ++a) {
            const size_t i = qi[a];
            if (rank[i] == 0) continue;
            fd.push_back(FormQDesc{dW + wo[i], kept[i], kept[i], rank[i], dtau + wsk[i], dwtop + wsk[i], dQW + qwo[i],
                                   kept[i]});
            gd.push_back(GemmDesc{dY + yo[i], m[i], dQW + qwo[i], kept[i], seg + qo[i], m[i], (int32_t)m[i], rank[i],
                                  kept[i], 0, nullptr});
            ed.push_back(ExtractRDesc{dW + wo[i], kept[i], rank[i], (int32_t)n[i], dperm + wsn[i], seg + ro[i], rank[i]});
        }
        FormQDesc* dfd;
        ExtractRDesc* ded;
        CHECK(ar.upload(&dfd, fd, "formq descs"));
        CHECK(ar.upload(&ded, ed, "extract descs"));
        launch_form_q(s, dfd, (int)fd.size(), maxrows);
        CHECK(gemm(0, gd));
        launch_extract_r(s, ded, (int)ed.size());
        CHECK(hip_check(ctx, hipGetLastError(), "form factors"));
    }
    // certification against regenerated entries
    std::vector<double> err2(nb, 0.0), nrm2(nb, 0.0);
    if (na) {
        std::vector<CertDesc> cd;
        std::vector<int64_t> first;
        int64_t nwg = 0;
        for (size_t i : act) {
            const BlockRec& b = blocks[ids[i]];
            cd.push_back(CertDesc{b.r0, b.rn, b.c0, b.cn, seg + qo[i], (int32_t)m[i], seg + ro[i], std::max(rank[i], 1),
                                  rank[i]});
            first.push_back(nwg);
            nwg += cert_workgroups(b.rn, b.cn);
        }
        first.push_back(nwg);
        std::vector<int32_t> pf, pc;
        for (size_t a = 0; a < na; ++a) {
            pf.push_back((int32_t)first[a]);
            pc.push_back((int32_t)(first[a + 1] - first[a]));
        }
        for (size_t a = 0; a < na; ++a) pf.push_back((int32_t)(nwg + first[a]));
        if (2 * nwg >= ((int64_t)1 << 31)) { set_err(ctx, "certification: too many tiles in one chunk"); return QRVIE_ERR_INVALID_ARG; }
        CertDesc* dcd; int64_t* dfirst; int32_t *dpf, *dpc; double *dpart, *dsum;
        CHECK(ar.upload(&dcd, cd, "cert descs"));
        CHECK(ar.upload(&dfirst, first, "cert workgroups"));
        CHECK(ar.upload(&dpf, pf, "cert partials"));
        CHECK(ar.upload(&dpc, pc, "cert partials"));
        CHECK(ar.alloc(&dpart, 2 * (size_t)nwg, "cert partials"));
        CHECK(ar.alloc(&dsum, 2 * na, "cert sums"));
        launch_cert_fused(s, g, dcd, dfirst, (int)na, nwg, dpart);
        launch_sum_partials(s, dpart, dpf, dpc, dsum, (int)na);
        launch_sum_partials(s, dpart, dpf + na, dpc, dsum + na, (int)na);
        CHECK(hip_check(ctx, hipGetLastError(), "certify"));
        std::vector<double> hs;
        CHECK(download(ctx, hs, dsum, 2 * na, "cert sums"));
        for (size_t a = 0; a < na; ++a) { err2[act[a]] = hs[a]; nrm2[act[a]] = hs[na + a]; }
    }
    std::vector<int32_t> retry_ids, retry_k;
    std::vector<double> retry_e;
    for (size_t i : act) {
        Factor& f = fac[ids[i]];
        f.Q = seg + qo[i];
        f.R = seg + ro[i];
        f.rank = rank[i];
        f.rel_err = nrm2[i] > 0.0 ? std::sqrt(err2[i] / nrm2[i]) : 0.0;
        if (f.rel_err <= eps) continue;
        if (eaca[i] > 5e-2 * aca_eps0) {                  // two rounds, each at a tenth of the tolerance
            retry_ids.push_back(ids[i]);
            retry_k.push_back(cap[i]);
            retry_e.push_back(eaca[i] * 0.1);
        } else {
            fallback.push_back(ids[i]);
        }
    }
    CHECK(round_segment(seg, ctot, act, ids, qo, ro));
    ar.release();
    n_retried += (int64_t)retry_ids.size();
    if (!retry_ids.empty()) return compress_aca(retry_ids, retry_k, retry_e, fallback);
    return QRVIE_OK;
}

// Chunk size of the build when chunk_bytes = 0: a quarter of the free device memory (or of
// the context's remaining budget), between 256 MB and 64 GiB.
size_t auto_chunk_bytes(qrvie_ctx* ctx) {
    double room = 8.0 * (1ull << 30);
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) == hipSuccess) room = (double)free_b;
    if (ctx->budget) room = std::min(room, (double)(ctx->budget - std::min(ctx->budget, ctx->in_use.load())));
    return (size_t)std::min(64.0 * (1ull << 30), std::max(2.56e8, room / 4.0));
}

// Rank model of the footprint estimate: above the largest ranks measured per block size at
// eps = 1e-6 (144 rows: 70; 576: 50; 2304: 66; 9216: 89), growing by 14 per decade of a
// tighter eps (QRCP ranks on the 4 x 4 array rise by 11-12 per decade).
double rank_model(double rows, double eps) {
    const double base = rows <= 2304 ? 80.0 : rows <= 9216 ? 100.0 : rows <= 36864 ? 128.0 : 160.0;
    return base + 14.0 * std::max(0.0, -std::log10(eps) - 6.0);
}

}  // namespace

namespace qrvie {

std::vector<BlockRec> split_blocks(const qrvie_geom* g, int64_t cap) {
    std::vector<BlockRec> out;
    std::vector<BlockRec> work(g->blocks.begin(), g->blocks.end());
    while (!work.empty()) {
        BlockRec b = work.back();
        work.pop_back();
        if (cap > 0 && b.level < g->L && ((int64_t)b.rn * kNp > cap || (int64_t)b.cn * kNp > cap)) {
            for (int32_t ci : node_children(g, b.rnode))
                for (int32_t cj : node_children(g, b.cnode)) {
                    const auto& a = g->nodes[ci];
                    const auto& c = g->nodes[cj];
                    work.push_back(BlockRec{b.level + 1, a.first, a.count, c.first, c.count, -1,
                                            a.first < c.first ? 1 : 0, ci, cj});
                }
        } else {
            out.push_back(b);
        }
    }
    std::sort(out.begin(), out.end(), [](const BlockRec& a, const BlockRec& b) {
        if (a.level != b.level) return a.level < b.level;
        if (a.r0 != b.r0) return a.r0 < b.r0;
        return a.c0 < b.c0;
    });
    std::map<std::tuple<int, int, int>, int32_t> idx;
    for (size_t i = 0; i < out.size(); ++i) idx[{out[i].level, out[i].r0, out[i].c0}] = (int32_t)i;
    for (auto& b : out) b.mirror = idx.at({b.level, b.c0, b.r0});
    return out;
}

void op_footprint(const qrvie_geom* g, const qrvie_compress_opts* o, size_t* resident, size_t* transient) {
    const bool aca = o->compression == QRVIE_COMPRESS_ACA;
    const std::vector<BlockRec> blocks = split_blocks(
        g, aca ? (o->max_block_rows > 0 ? std::min<int64_t>(o->max_block_rows, kAcaMaxRows) : kAcaMaxRows)
               : o->max_block_rows);
    const int64_t chunk_elems =
        std::max<int64_t>(1, (o->chunk_bytes > 0 ? o->chunk_bytes : ((int64_t)64 << 30)) / (int64_t)sizeof(c128));
    double fac = 0.0, prim = 0.0, tlen = 0.0, rpad = 0.0, qstrips = 0.0;
    std::map<std::pair<int, int>, int> rpanels;
    // materialised bytes per chunk, in the build's chunk order: block, direct work copy,
    // sketch and projected sketch (doubled for the retries of a wider sketch)
    double acc = 0.0, dir = 0.0, sk = 0.0, best = 0.0;
    double cprim = 0.0;                               // compact factors of the chunk
    auto flush = [&]() {
        best = std::max(best, acc + dir + 2.0 * sk + cprim);
        acc = dir = sk = cprim = 0.0;
    };
    // cross approximation: its chunks hold the crosses, their basis and projected rows
    double aacc = 0.0, acprim = 0.0;
    auto aflush = [&]() {
        best = std::max(best, aacc + acprim);
        aacc = acprim = 0.0;
    };
    for (const BlockRec& b : blocks) {
        const double m = (double)b.rn * kNp, n = (double)b.cn * kNp;
        const double r = std::min(rank_model(std::max(m, n), o->eps), std::min(m, n));
        if (!b.primary && o->share_transpose) continue;   // shared: the pair's factors are stored once
        fac += (m + n) * r;
        tlen += r;
        rpanels[{b.level, b.c0}] = b.cn;
        if (!b.primary) continue;
        prim += (m + n) * r;
        const bool small = b.rn <= kDirectMaxParticles && b.cn <= kDirectMaxParticles;
        if (aca && !small) {
            const double e = (double)aca_elems(b, (int)std::min<double>(o->aca_start > 0 ? o->aca_start : kAcaStart,
                                                                        std::min(m, n)));
            if (aacc > 0.0 && aacc + e > (double)chunk_elems) aflush();
            aacc += e;
            acprim += (m + n) * r;
            continue;
        }
        const double e = m * n;
        if (acc > 0.0 && acc + e > (double)chunk_elems) flush();
        acc += e;
        cprim += (m + n) * r;
        if (b.rn <= kDirectMaxParticles && b.cn <= kDirectMaxParticles) dir += e;
        else {
            const double k = std::min<double>(kSketchStart, std::min(m, n));
            sk += k * (m + n);
        }
    }
    flush();
    aflush();
    for (const auto& kv : rpanels) rpad += (double)(kAlign - 1) * kv.second * kNp;
    for (int32_t id = 0; id < (int32_t)g->nodes.size(); ++id) qstrips += std::ceil(g->nodes[id].count * kNp / 64.0);
    const double panel_elems = fac + rpad;
    double panels = 0.0, panels_final = 0.0;        // bytes while packing, and once built
    if (o->far_prec == QRVIE_PREC_C64_ONLY) panels = panels_final = 8.0 * panel_elems;
    else if (o->far_prec == QRVIE_PREC_BF16X2) panels = 8.0 * panel_elems, panels_final = 12.0 * panel_elems;
    else {
        panels = 16.0 * panel_elems;
        panels_final = panels + (o->far_prec == QRVIE_PREC_C64 ? 8.0 * panel_elems : 0.0);
    }
    // compact factors until they are packed (rounded to complex64 chunk by chunk when the
    // operator keeps only complex64)
    const bool c32 = o->far_prec == QRVIE_PREC_C64_ONLY || o->far_prec == QRVIE_PREC_BF16X2;
    const double seg = (c32 ? 8.0 : 16.0) * prim;
    const double pools = 16.0 * best;
    const double nstrips = tlen / 64.0 + (double)rpanels.size() + qstrips;
    const double other = 2.0 * (double)g->types.size() * kNp * kNp * 16.0 + 8.0 * tlen +
                         nstrips * (double)(sizeof(RStrip) + sizeof(QStrip) + sizeof(MStrip)) +
                         (double)g->N * 3 * sizeof(MStrip) + (1 << 20);
    const double peak = std::max({seg + pools, seg + panels, panels_final}) + other;
    *resident = (size_t)(panels_final + other);
    *transient = (size_t)(peak - panels_final - other);
}

}  // namespace qrvie

extern "C" {

qrvie_status qrvie_op_footprint_estimate(const qrvie_geom* g, const qrvie_compress_opts* o, size_t* bytes) {
    if (!g || !o || !bytes || !(o->eps > 0.0) || o->max_block_rows < 0 || o->chunk_bytes < 0)
        return QRVIE_ERR_INVALID_ARG;
    size_t resident = 0, transient = 0;
    op_footprint(g, o, &resident, &transient);
    *bytes = resident + transient;
    return QRVIE_OK;
}

qrvie_status qrvie_op_create(qrvie_ctx* ctx, const qrvie_geom* g, const qrvie_compress_opts* o, qrvie_op** out) {
    if (!ctx || !g || !o || !out) return QRVIE_ERR_INVALID_ARG;
    *out = nullptr;
    if (!(o->eps > 0.0) || !(o->eps < 1.0)) { set_err(ctx, "op_create: eps must be in (0, 1)"); return QRVIE_ERR_INVALID_ARG; }
    if ((o->far_prec != QRVIE_PREC_C128 && o->far_prec != QRVIE_PREC_C64 && o->far_prec != QRVIE_PREC_C64_ONLY &&
         o->far_prec != QRVIE_PREC_BF16X2) ||
        o->near_prec != QRVIE_PREC_C128 ||
        (o->share_transpose != 0 && o->share_transpose != 1) ||
        (o->compression != QRVIE_COMPRESS_ACA && o->compression != QRVIE_COMPRESS_SKETCH) ||
        o->aca_start < 0 || o->aca_start > kAcaMaxRank || !(o->aca_stop >= 0.0) ||
        o->max_block_rows < 0 || o->chunk_bytes < 0) {
        set_err(ctx, "op_create: unsupported precision or option");
        return QRVIE_ERR_INVALID_ARG;
    }
    {
        // resident operator plus the build's transient buffers at the chunk size it will use
        qrvie_compress_opts oc = *o;
        if (oc.chunk_bytes == 0) oc.chunk_bytes = (int64_t)auto_chunk_bytes(ctx);
        size_t resident = 0, transient = 0;
        op_footprint(g, &oc, &resident, &transient);
        if (ctx->budget && ctx->in_use.load() + resident + transient > ctx->budget) {
            set_err(ctx, "op_create: footprint estimate " + std::to_string(resident + transient) +
                             " exceeds the remaining HBM budget");
            return QRVIE_ERR_OUT_OF_MEMORY;
        }
    }
    hipStream_t s = ctx->stream;
    auto* op = new qrvie_op;
    op->ctx = ctx;
    op->g = g;
    op->opts = *o;
    op->ntypes = (int32_t)g->types.size();
    auto fail = [&](qrvie_status st) {
        qrvie_op_destroy(op);
        return st;
    };
    const double t0 = now_s();
    const size_t selfb = sizeof(c128) * (size_t)op->ntypes * kNp * kNp;
    qrvie_status st = QRVIE_OK;
    auto keep = [&](void** p, size_t bytes, const char* what) {
        if (st != QRVIE_OK) return;
        st = dalloc(ctx, p, bytes, what);
        if (st == QRVIE_OK) op->allocs.push_back({*p, bytes});
    };
    keep((void**)&op->d_self, selfb, "self blocks");
    keep((void**)&op->d_pinv, selfb, "preconditioner");
    if (st != QRVIE_OK) return fail(st);
    launch_assemble_self(s, g, op->d_self, op->ntypes);
    st = hip_check(ctx, hipMemcpyAsync(op->d_pinv, op->d_self, selfb, hipMemcpyDeviceToDevice, s), "copy self");
    if (st != QRVIE_OK) return fail(st);
    int* dinfo = nullptr;
    st = dalloc(ctx, (void**)&dinfo, sizeof(int) * op->ntypes, "invert info");
    if (st != QRVIE_OK) return fail(st);
    (void)hipMemsetAsync(dinfo, 0, sizeof(int) * op->ntypes, s);
    launch_invert(s, op->d_pinv, op->ntypes, dinfo);
    std::vector<int> hinfo;
    st = download(ctx, hinfo, dinfo, op->ntypes, "invert info");
    dfree(ctx, dinfo, sizeof(int) * op->ntypes);
    if (st != QRVIE_OK) return fail(st);
    for (int t = 0; t < op->ntypes; ++t)
        if (hinfo[t] != 0) {
            set_err(ctx, "op_create: singular self block");
            return fail(QRVIE_ERR_DEVICE);
        }
    const double t1 = now_s();
    op->stats.t_precond_setup_s = t1 - t0;

    // block list, with the optional row cap splitting far pairs into child pairs (cross
    // approximation keeps one flag per row in LDS: its blocks have at most kAcaMaxRows rows)
    const bool aca = o->compression == QRVIE_COMPRESS_ACA;
    const int64_t cap = aca ? (o->max_block_rows > 0 ? std::min<int64_t>(o->max_block_rows, kAcaMaxRows) : kAcaMaxRows)
                            : o->max_block_rows;
    Builder bld{op, ctx, g, split_blocks(g, cap), {}, {}, o->eps};
    bld.compact32 = o->far_prec == QRVIE_PREC_C64_ONLY || o->far_prec == QRVIE_PREC_BF16X2;
    bld.aca_eps0 = (o->aca_stop > 0.0 ? o->aca_stop : kAcaEps) * o->eps;
    const size_t NB = bld.blocks.size();
    bld.fac.resize(NB);

    // compress primary blocks in chunks bounded by the materialised block bytes
    // (a quarter of the free device memory, or of the remaining budget, at most 64 GiB: the
    // one-workgroup-per-block kernels of the sketch path are better used with many blocks,
    // and concurrent builds on one device still leave room for each other)
    const int64_t chunk_elems =
        std::max<int64_t>(1, (o->chunk_bytes > 0 ? o->chunk_bytes : (int64_t)auto_chunk_bytes(ctx)) / (int64_t)sizeof(c128));
    std::vector<int32_t> fallback;          // cross approximation: blocks left to the sketch path
    if (aca) {
        // chunks of blocks bounded by the crosses' working buffers
        struct Chunk { std::vector<int32_t> ids, kmx; };
        std::vector<Chunk> chunks(1);
        int64_t acc = 0;
        size_t nprim = 0, ndone = 0;
        for (size_t i = 0; i < NB; ++i) {
            const BlockRec& b = bld.blocks[i];
            if (!b.primary || (b.rn <= kDirectMaxParticles && b.cn <= kDirectMaxParticles)) continue;
            const int kmax = (int)std::min<int64_t>(o->aca_start > 0 ? o->aca_start : kAcaStart,
                                                    (int64_t)std::min(b.rn, b.cn) * kNp);
            const int64_t e = aca_elems(b, kmax);
            if (acc > 0 && acc + e > chunk_elems) {
                chunks.emplace_back();
                acc = 0;
            }
            chunks.back().ids.push_back((int32_t)i);
            chunks.back().kmx.push_back(kmax);
            acc += e;
            ++nprim;
        }
        // size the reused buffers once for the largest chunk: growing them chunk by chunk
        // (release, then allocate tens of GB again) cost seconds of host time in large builds
        size_t mx[2] = {0, 0};
        for (const Chunk& ch : chunks) {
            size_t u = 0, v = 0;
            for (size_t a = 0; a < ch.ids.size(); ++a) {
                const BlockRec& b = bld.blocks[ch.ids[a]];
                u += (size_t)b.rn * kNp * ch.kmx[a];
                v += (size_t)b.cn * kNp * ch.kmx[a];
            }
            mx[0] = std::max(mx[0], u);
            mx[1] = std::max(mx[1], v);
        }
        for (int w = 0; w < 4 && st == QRVIE_OK; ++w) {     // crosses U, V; basis of U (<= U); rows (<= V)
            c128* p = nullptr;
            st = bld.pooled(w, mx[w & 1], &p, "cross approximation buffers");
        }
        if (st != QRVIE_OK) return fail(st);
        for (const Chunk& ch : chunks) {
            if (ch.ids.empty()) continue;
            st = bld.compress_aca(ch.ids, ch.kmx, std::vector<double>(ch.ids.size(), bld.aca_eps0), fallback);
            if (st != QRVIE_OK) {
                for (auto& sg : bld.segments) dfree(ctx, sg.first, sg.second);
                return fail(st);
            }
            ndone += ch.ids.size();
            if (o->verbose) {
                std::fprintf(stderr, "[qrvie] cross approximation: %zu / %zu blocks (%.1f s)\n", ndone, nprim,
                             now_s() - t1);
                std::fflush(stderr);
            }
        }
        op->stats.n_aca = (int64_t)ndone - (int64_t)fallback.size();
        op->stats.n_aca_resumed = bld.n_resumed;
        op->stats.n_aca_retried = bld.n_retried;
        op->stats.n_aca_sketch = (int64_t)fallback.size();
        bld.release_pools();                // the direct and sketch passes size their own
        if (o->verbose && !fallback.empty()) {
            std::fprintf(stderr, "[qrvie] cross approximation: %zu blocks left to the sketch path\n", fallback.size());
            std::fflush(stderr);
        }
    }
    {
        std::vector<int32_t> ids, kw;
        int64_t acc = 0;
        size_t nprim = 0, ndone = 0;
        std::vector<char> sketch_ok(NB, aca ? 0 : 1);
        for (int32_t f : fallback) sketch_ok[f] = 1;
        auto mine = [&](const BlockRec& b, size_t i) {
            return b.primary && (sketch_ok[i] || (b.rn <= kDirectMaxParticles && b.cn <= kDirectMaxParticles));
        };
        for (size_t i = 0; i < NB; ++i) nprim += mine(bld.blocks[i], i) ? 1 : 0;
        for (size_t i = 0; i <= NB; ++i) {
            bool flush = (i == NB);
            if (!flush) {
                const BlockRec& b = bld.blocks[i];
                if (!mine(b, i)) continue;
                const int64_t e = (int64_t)b.rn * kNp * b.cn * kNp;
                if (acc > 0 && acc + e > chunk_elems) flush = true;
                if (!flush) {
                    ids.push_back((int32_t)i);
                    const bool direct = b.rn <= kDirectMaxParticles && b.cn <= kDirectMaxParticles;
                    kw.push_back(direct ? 0 : kSketchStart);
                    acc += e;
                    continue;
                }
            }
            if (!ids.empty()) {
                st = bld.compress(ids, kw);
                if (st != QRVIE_OK) {
                    for (auto& sg : bld.segments) dfree(ctx, sg.first, sg.second);
                    return fail(st);
                }
                ndone += ids.size();
                if (o->verbose) {
                    std::fprintf(stderr, "[qrvie] compressed %zu / %zu blocks (%.1f s)\n", ndone, nprim, now_s() - t1);
                    std::fflush(stderr);
                }
            }
            ids.clear();
            kw.clear();
            acc = 0;
            if (i < NB) --i;   // re-visit the block that did not fit
        }
    }
    bld.release_pools();
    (void)hipStreamSynchronize(s);
    const double t2 = now_s();
    op->stats.t_compression_s = t2 - t1;

    // ranks of mirrors; per-block bookkeeping
    op->blocks = bld.blocks;
    op->rank.assign(NB, 0);
    op->relerr.assign(NB, 0.0);
    for (size_t i = 0; i < NB; ++i) {
        const BlockRec& b = bld.blocks[i];
        const Factor& f = bld.fac[b.primary ? i : b.mirror];
        op->rank[i] = f.rank;
        op->relerr[i] = f.rel_err;
    }

    // panel layout.  With shared factors only the compressed block of each pair (its primary)
    // enters the panels: its Q in the row node's Q panel, its R in the column node's R panel;
    // the mirror (J, I) is applied through the same panels transposed.
    const bool sh = o->share_transpose != 0;
    op->shared = sh;
    auto stored = [&](size_t b) { return !sh || bld.blocks[b].primary; };
    const int64_t n = g->ndof();
    std::vector<int> active(g->L + 2, -1);
    for (const auto& b : bld.blocks) active[b.level] = 1;
    int nact = 0;
    for (int l = 0; l <= g->L + 1; ++l)
        if (active[l] > 0) active[l] = nact++;
    op->n_active = nact;
    op->q_off.assign(NB, 0);
    op->r_off.assign(NB, 0);
    op->r_ld.assign(NB, 0);
    std::vector<int64_t> toff(NB, 0);
    std::vector<RStrip> rstr;
    std::vector<QStrip> qstr;
    std::vector<QtItem> qts;
    std::vector<MStrip> mqt, mrt;          // shared factors: Q^T and R^T strips for blocks of RHS
    std::vector<int64_t> tmap;
    int64_t fcur = 0, tcur = 0, pcur = 0;
    for (int l = 0; l <= g->L; ++l) {
        if (active[l] < 0) continue;
        // Q panels over every occupied node of the level
        int64_t qbegin = (int64_t)qstr.size();
        std::map<int32_t, std::vector<std::pair<size_t, int64_t>>> qstrips_of;   // node first -> (strip, row)
        size_t bi = 0;
        while (bi < NB && bld.blocks[bi].level != l) ++bi;
        for (int32_t I : g->level_nodes[l]) {
            const auto& nd = g->nodes[I];
            const int64_t mI = (int64_t)nd.count * kNp;
            size_t b0 = bi;
            while (b0 < NB && bld.blocks[b0].level == l && bld.blocks[b0].r0 < nd.first) ++b0;
            size_t b1 = b0;
            int64_t K = 0;
            while (b1 < NB && bld.blocks[b1].level == l && bld.blocks[b1].r0 == nd.first) {
                if (stored(b1)) K += op->rank[b1];
                ++b1;
            }
            const int64_t base = fcur;
            fcur += mI * K;
            int64_t col = 0;
            for (size_t b = b0; b < b1; ++b) {
                if (!stored(b)) continue;
                op->q_off[b] = base + mI * col;
                toff[b] = tcur + col;
                col += op->rank[b];
            }
            for (int64_t r0 = 0; r0 < mI; r0 += kStrip) {
                qstrips_of[nd.first].push_back({qstr.size(), r0});
                qstr.push_back(QStrip{base + r0, (int32_t)mI, (int32_t)K, (int32_t)std::min<int64_t>(kStrip, mI - r0),
                                      (int64_t)active[l] * n + (int64_t)nd.first * kNp + r0, tcur, -1, 0, 0});
            }
            if (sh) {
                for (int64_t c0 = 0; c0 < K; c0 += 8)
                    qts.push_back(QtItem{base + mI * c0, (int32_t)mI, (int32_t)mI, (int32_t)std::min<int64_t>(8, K - c0),
                                         nd.first * kNp, tcur + c0});
                for (int64_t c0 = 0; c0 < K; c0 += kStrip)   // rows: the panel's columns; output through tinv
                    mqt.push_back(MStrip{base + mI * c0, (int32_t)mI, (int32_t)mI, (int32_t)std::min<int64_t>(kStrip, K - c0),
                                         kStripTrans, (int64_t)nd.first * kNp, 0, tcur + c0});
            }
            tcur += K;
            bi = b1;
        }
        // R panels per column node
        std::map<int32_t, std::array<int64_t, 4>> rpanel;   // node first -> (base, ld, rows, stacked row base)
        std::map<int32_t, std::vector<size_t>> bycol;
        for (size_t b = 0; b < NB; ++b)
            if (bld.blocks[b].level == l && stored(b)) bycol[bld.blocks[b].c0].push_back(b);
        for (auto& kv : bycol) {
            const BlockRec& b0 = bld.blocks[kv.second.front()];
            const int64_t nJ = (int64_t)b0.cn * kNp;
            int64_t Kp = 0;
            for (size_t b : kv.second) Kp += op->rank[b];
            // leading dimension padded to 16 entries so every wave's 64-row column segment
            // starts on a 128-byte cache-line boundary in the complex128 panels and in
            // their complex64 copy
            const int64_t ldp = (Kp + kAlign - 1) / kAlign * kAlign;
            const int64_t base = fcur;
            fcur += ldp * nJ;
            const int64_t tbase = (int64_t)tmap.size();
            int64_t row = 0;
            for (size_t b : kv.second) {
                op->r_off[b] = base + row;
                op->r_ld[b] = (int32_t)ldp;
                for (int k = 0; k < op->rank[b]; ++k) tmap.push_back(toff[b] + k);
                row += op->rank[b];
            }
            rpanel[b0.c0] = {base, ldp, Kp, tbase};
            const int64_t nstrip = (Kp + kStrip - 1) / kStrip;
            for (int64_t r0 = 0; r0 < Kp; r0 += kStrip)
                rstr.push_back(RStrip{base + r0, (int32_t)ldp, (int32_t)nJ, (int32_t)std::min<int64_t>(kStrip, Kp - r0),
                                      b0.c0 * kNp, tbase + r0, sh ? pcur + (r0 / kStrip) * nJ : -1});
            if (sh && nstrip > 0) {
                // the column node's rows at this level also receive the mirror partials
                for (const auto& sr : qstrips_of.at(b0.c0)) {
                    QStrip& q = qstr[sr.first];
                    q.p_off = pcur + sr.second;
                    q.p_cnt = (int32_t)nstrip;
                    q.p_ld = (int32_t)nJ;
                }
                pcur += nstrip * nJ;
            }
        }
        (void)qbegin;
        if (sh)   // R^T strips over the rows of every node of the level (zero rows where no panel)
            for (int32_t J : g->level_nodes[l]) {
                const auto& nd = g->nodes[J];
                const int64_t nJ = (int64_t)nd.count * kNp;
                const auto it = rpanel.find(nd.first);
                for (int64_t j0 = 0; j0 < nJ; j0 += kStrip) {
                    const int32_t rows = (int32_t)std::min<int64_t>(kStrip, nJ - j0);
                    const int64_t orow = (int64_t)active[l] * n + (int64_t)nd.first * kNp + j0;
                    if (it == rpanel.end())
                        mrt.push_back(MStrip{0, 1, 0, rows, kStripTrans, 0, orow, -1});
                    else
                        mrt.push_back(MStrip{it->second[0] + j0 * it->second[1], (int32_t)it->second[1],
                                             (int32_t)it->second[2], rows, kStripTrans, it->second[3], orow, -1});
                }
            }
    }
    // One launch per phase over all levels: four waves per strip split its columns, and the
    // strips are issued longest first so the long coarse-level strips overlap the many
    // short fine-level ones (largest-first greedy, the load-balancing rule of the paper's
    // appendix C applied to workgroups).
    std::stable_sort(rstr.begin(), rstr.end(), [](const RStrip& a, const RStrip& b) { return a.ncols > b.ncols; });
    std::stable_sort(qstr.begin(), qstr.end(), [](const QStrip& a, const QStrip& b) { return a.ncols > b.ncols; });
    op->rlaunch.assign(1, {-1, 0, (int64_t)rstr.size(), kPhaseWaves});
    op->qlaunch.assign(1, {-1, 0, (int64_t)qstr.size(), kPhaseWaves});
    op->fac_elems = fcur;
    op->t_len = tcur;
    op->tmap_len = (int64_t)tmap.size();
    op->p_len = pcur;
    op->n_qt = (int64_t)qts.size();

    // The same strips for blocks of right-hand sides, plus three strips per particle over
    // its self block (and, with the same offsets, its inverse).
    std::vector<MStrip> mr, mq, ms;
    mr.reserve(rstr.size());
    mq.reserve(qstr.size());
    // (shared factors: the Q strips add to the level partials that the R^T strips wrote)
    for (const RStrip& r : rstr) mr.push_back(MStrip{r.a_off, r.ld, r.ncols, r.nrows, 0, r.x_off, 0, r.tmap_off});
    for (const QStrip& q : qstr)
        mq.push_back(MStrip{q.a_off, q.ld, q.ncols, q.nrows, sh ? kStripAcc : 0, q.t_off, q.y_off, -1});
    auto longest_first = [](const MStrip& a, const MStrip& b) { return a.ncols > b.ncols; };
    std::stable_sort(mqt.begin(), mqt.end(), longest_first);
    std::stable_sort(mrt.begin(), mrt.end(), longest_first);
    op->n_mqt = (int64_t)mqt.size();
    op->n_mrt = (int64_t)mrt.size();
    std::vector<int64_t> tinv(sh ? tmap.size() : 0);
    for (size_t k = 0; k < tinv.size(); ++k) tinv[tmap[k]] = (int64_t)k;
    for (int32_t p = 0; p < g->N; ++p)
        for (int r0 = 0; r0 < kNp; r0 += kStrip)
            ms.push_back(MStrip{(int64_t)g->ptype[p] * kNp * kNp + r0, kNp, kNp, std::min(kStrip, kNp - r0), 0,
                                (int64_t)p * kNp, (int64_t)p * kNp + r0, -1});
    op->n_mr = (int64_t)mr.size();
    op->n_mq = (int64_t)mq.size();
    op->n_ms = (int64_t)ms.size();
    keep((void**)&op->d_mr, sizeof(MStrip) * std::max<size_t>(mr.size(), 1), "block R strips");
    keep((void**)&op->d_mq, sizeof(MStrip) * std::max<size_t>(mq.size(), 1), "block Q strips");
    keep((void**)&op->d_ms, sizeof(MStrip) * std::max<size_t>(ms.size(), 1), "block self strips");
    if (sh) {
        keep((void**)&op->d_mqt, sizeof(MStrip) * std::max<size_t>(mqt.size(), 1), "block Q^T strips");
        keep((void**)&op->d_mrt, sizeof(MStrip) * std::max<size_t>(mrt.size(), 1), "block R^T strips");
        keep((void**)&op->d_tinv, sizeof(int64_t) * std::max<size_t>(tinv.size(), 1), "inverse rank map");
    }

    const bool only32 = o->far_prec == QRVIE_PREC_C64_ONLY || o->far_prec == QRVIE_PREC_BF16X2;
    if (only32) keep((void**)&op->d_fac32, sizeof(float2) * (size_t)std::max<int64_t>(fcur, 1), "complex64 panels");
    else keep((void**)&op->d_fac, sizeof(c128) * (size_t)std::max<int64_t>(fcur, 1), "factor panels");
    keep((void**)&op->d_tmap, sizeof(int64_t) * std::max<size_t>(tmap.size(), 1), "rank map");
    keep((void**)&op->d_rstrips, sizeof(RStrip) * std::max<size_t>(rstr.size(), 1), "R strips");
    keep((void**)&op->d_qstrips, sizeof(QStrip) * std::max<size_t>(qstr.size(), 1), "Q strips");
    if (sh) keep((void**)&op->d_qt, sizeof(QtItem) * std::max<size_t>(qts.size(), 1), "Q^T items");
    if (st != QRVIE_OK) {
        for (auto& sg : bld.segments) dfree(ctx, sg.first, sg.second);
        return fail(st);
    }
    if (!tmap.empty()) (void)hipMemcpyAsync(op->d_tmap, tmap.data(), sizeof(int64_t) * tmap.size(), hipMemcpyHostToDevice, s);
    if (!rstr.empty()) (void)hipMemcpyAsync(op->d_rstrips, rstr.data(), sizeof(RStrip) * rstr.size(), hipMemcpyHostToDevice, s);
    if (!qstr.empty()) (void)hipMemcpyAsync(op->d_qstrips, qstr.data(), sizeof(QStrip) * qstr.size(), hipMemcpyHostToDevice, s);
    if (sh && !qts.empty()) (void)hipMemcpyAsync(op->d_qt, qts.data(), sizeof(QtItem) * qts.size(), hipMemcpyHostToDevice, s);
    if (st == QRVIE_OK && !mr.empty()) (void)hipMemcpyAsync(op->d_mr, mr.data(), sizeof(MStrip) * mr.size(), hipMemcpyHostToDevice, s);
    if (st == QRVIE_OK && !mq.empty()) (void)hipMemcpyAsync(op->d_mq, mq.data(), sizeof(MStrip) * mq.size(), hipMemcpyHostToDevice, s);
    if (st == QRVIE_OK && !ms.empty()) (void)hipMemcpyAsync(op->d_ms, ms.data(), sizeof(MStrip) * ms.size(), hipMemcpyHostToDevice, s);
    if (st == QRVIE_OK && sh) {
        if (!mqt.empty()) (void)hipMemcpyAsync(op->d_mqt, mqt.data(), sizeof(MStrip) * mqt.size(), hipMemcpyHostToDevice, s);
        if (!mrt.empty()) (void)hipMemcpyAsync(op->d_mrt, mrt.data(), sizeof(MStrip) * mrt.size(), hipMemcpyHostToDevice, s);
        if (!tinv.empty()) (void)hipMemcpyAsync(op->d_tinv, tinv.data(), sizeof(int64_t) * tinv.size(), hipMemcpyHostToDevice, s);
    }
    st = hip_check(ctx, hipStreamSynchronize(s), "upload layout");   // the host vectors die at return
    if (st != QRVIE_OK) {
        for (auto& sg : bld.segments) dfree(ctx, sg.first, sg.second);
        return fail(st);
    }

    // pack compact factors into the panels
    {
        std::vector<PackDesc> pd;
        for (size_t i = 0; i < NB; ++i) {
            const BlockRec& b = bld.blocks[i];
            if (!b.primary || op->rank[i] == 0) continue;
            const Factor& f = bld.fac[i];
            const int32_t mm = b.rn * kNp, nn = b.cn * kNp, r = f.rank;
            const size_t j = (size_t)b.mirror;
            // destination: complex128 panels, or their complex64 rounding when only those are kept
            auto at = [&](int64_t off, int64_t ld, int32_t tr) {
                return only32 ? PackDesc{nullptr, 0, 0, 0, nullptr, ld, tr, op->d_fac32 + off, nullptr}
                              : PackDesc{nullptr, 0, 0, 0, op->d_fac + off, ld, tr, nullptr, nullptr};
            };
            // the compact source: complex128, or complex64 when the build rounded it per chunk
            auto with = [](PackDesc d, const c128* src, const float2* src32, int32_t rows, int32_t cols, int32_t lds) {
                d.src = src; d.src32 = src32; d.rows = rows; d.cols = cols; d.lds = lds;
                return d;
            };
            pd.push_back(with(at(op->q_off[i], mm, 0), f.Q, f.Q32, mm, r, mm));            // Q_IJ
            pd.push_back(with(at(op->r_off[i], op->r_ld[i], 0), f.R, f.R32, r, nn, r));    // R_IJ
            if (sh) continue;                                                              // mirrors read these
            pd.push_back(with(at(op->q_off[j], nn, 1), f.R, f.R32, r, nn, r));             // Q_JI = R_IJ^T
            pd.push_back(with(at(op->r_off[j], op->r_ld[j], 1), f.Q, f.Q32, mm, r, mm));   // R_JI = Q_IJ^T
        }
        PackDesc* dpd = nullptr;
        if (!pd.empty()) {
            st = dalloc(ctx, (void**)&dpd, sizeof(PackDesc) * pd.size(), "pack descs");
            if (st == QRVIE_OK)
                st = hip_check(ctx, hipMemcpyAsync(dpd, pd.data(), sizeof(PackDesc) * pd.size(), hipMemcpyHostToDevice, s), "pack");
            if (st == QRVIE_OK) {
                launch_pack(s, dpd, (int)pd.size());
                st = hip_check(ctx, hipGetLastError(), "pack");
            }
            if (st == QRVIE_OK) st = hip_check(ctx, hipStreamSynchronize(s), "pack");
            dfree(ctx, dpd, sizeof(PackDesc) * pd.size());
        }
        for (auto& sg : bld.segments) dfree(ctx, sg.first, sg.second);
        bld.segments.clear();
        if (st != QRVIE_OK) return fail(st);
    }
    if (o->far_prec == QRVIE_PREC_C64) {
        // complex64 copy of the far factors for the reduced-precision inner products
        keep((void**)&op->d_fac32, sizeof(float2) * (size_t)std::max<int64_t>(op->fac_elems, 1), "complex64 panels");
        if (st != QRVIE_OK) return fail(st);
        launch_to_c64(s, op->d_fac, op->d_fac32, op->fac_elems);
        st = hip_check(ctx, hipStreamSynchronize(s), "complex64 panels");
        if (st != QRVIE_OK) return fail(st);
    }
    if (o->far_prec == QRVIE_PREC_BF16X2) {
        // BF16 split-complex planes of the complex64 panels (round to nearest even twice:
        // FP64 -> FP32 -> BF16)
        keep((void**)&op->d_fac16, sizeof(uint16_t) * 2 * (size_t)std::max<int64_t>(op->fac_elems, 1), "bf16 planes");
        if (st != QRVIE_OK) return fail(st);
        launch_to_bf16(s, op->d_fac32, op->d_fac16, op->fac_elems, op->fac_elems);
    }
    if (o->far_prec != QRVIE_PREC_C128) {
        // complex64 self blocks and inverses: the near part of products on FP32 matrix cores
        keep((void**)&op->d_self32, sizeof(float2) * (size_t)op->ntypes * kNp * kNp, "complex64 self blocks");
        keep((void**)&op->d_pinv32, sizeof(float2) * (size_t)op->ntypes * kNp * kNp, "complex64 inverses");
        if (st != QRVIE_OK) return fail(st);
        launch_to_c64(s, op->d_self, op->d_self32, (int64_t)op->ntypes * kNp * kNp);
        launch_to_c64(s, op->d_pinv, op->d_pinv32, (int64_t)op->ntypes * kNp * kNp);
    }
    st = hip_check(ctx, hipStreamSynchronize(s), "reduced-precision copies");
    if (st != QRVIE_OK) return fail(st);
    const double t3 = now_s();
    op->stats.t_compression_s += t3 - t2;

    // statistics (eqs. 5.5-5.6 and the product's algorithmic bytes)
    qrvie_op_stats& S = op->stats;
    S.n_levels = g->L;
    S.n_blocks = (int64_t)NB;
    S.n_self_types = op->ntypes;
    for (int l = 0; l < QRVIE_MAX_LEVELS; ++l) { S.min_rank_level[l] = 0; S.max_rank_level[l] = 0; }
    std::vector<double> rsum(QRVIE_MAX_LEVELS, 0.0);
    int64_t nqr = (int64_t)g->N * kNp * kNp, sum_r = 0;
    double maxerr = 0.0;
    for (size_t i = 0; i < NB; ++i) {
        const BlockRec& b = bld.blocks[i];
        const int l = std::min(b.level, QRVIE_MAX_LEVELS - 1);
        const int r = op->rank[i];
        if (S.n_blocks_level[l] == 0 || r < S.min_rank_level[l]) S.min_rank_level[l] = r;
        S.max_rank_level[l] = std::max(S.max_rank_level[l], r);
        S.n_blocks_level[l]++;
        rsum[l] += r;
        nqr += ((int64_t)b.rn * kNp + (int64_t)b.cn * kNp) * r;
        sum_r += r;
        maxerr = std::max(maxerr, op->relerr[i]);
    }
    for (int l = 0; l < QRVIE_MAX_LEVELS; ++l)
        S.mean_rank_level[l] = S.n_blocks_level[l] ? rsum[l] / S.n_blocks_level[l] : 0.0;
    S.n_qr_entries = nqr;
    S.gain = (double)n * (double)n / (double)nqr;
    S.max_block_rel_err = maxerr;
    // factor entries one product streams: every ordered block's Q and R, or with shared factors
    // each pair's Q twice (Q^T x, then Q t) and its R once (R x and R^T s in one pass)
    int64_t streamed = 0;
    for (size_t i = 0; i < NB; ++i) {
        const BlockRec& b = bld.blocks[i];
        const int64_t r = op->rank[i], m = (int64_t)b.rn * kNp, nn = (int64_t)b.cn * kNp;
        if (!sh) streamed += (m + nn) * r;
        else if (b.primary) streamed += (2 * m + nn) * r;
    }
    const int64_t vec = (int64_t)op->ntypes * kNp * kNp + 2 * n + 2 * sum_r;
    S.apply_bytes = (int64_t)sizeof(c128) * (streamed + vec);
    S.apply_bytes_c64 = op->d_fac32 ? (int64_t)sizeof(float2) * streamed + (int64_t)sizeof(c128) * vec : 0;
    for (auto& a : op->allocs) op->dev_bytes += a.second;
    S.device_bytes = (int64_t)op->dev_bytes;
    S.t_assembly_s = 0.0;  // assembly is fused into compression; see t_compression_s
    *out = op;
    return QRVIE_OK;
}

qrvie_status qrvie_op_stats_get(const qrvie_op* op, qrvie_op_stats* out) {
    if (!op || !out) return QRVIE_ERR_INVALID_ARG;
    *out = op->stats;
    return QRVIE_OK;
}

int64_t qrvie_op_num_blocks(const qrvie_op* op) { return op ? (int64_t)op->rank.size() : 0; }

void qrvie_op_destroy(qrvie_op* op) {
    if (!op) return;
    qrvie_ctx* ctx = op->ctx;
    (void)hipStreamSynchronize(ctx->stream);
    for (auto& a : op->allocs) dfree(ctx, a.first, a.second);
    delete op;
}

}  // extern "C"
