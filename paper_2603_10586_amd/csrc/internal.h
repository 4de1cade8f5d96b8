// Internal structures of libqrvie: context, geometry, operator, kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <string>
#include <vector>

#include "qrvie.h"

namespace qrvie {

constexpr int kCells = 48;          // cells per particle (24 squares x 2 layers)
constexpr int kNp = 144;            // DoFs per particle (48 cells x 3 components)
constexpr int kStrip = 64;          // rows per wavefront strip in the products

typedef double2 c128;

// ---------------------------------------------------------------- host records
struct PType {                      // one distinct particle shape/material
    double radius, height;
    double eps_re, eps_im;
    double vol, aeq;                // cell volume, equal-volume sphere radius
    double off[kCells * 3];         // cell-centre offsets, canonical order
};

struct BlockRec {                   // one ordered pair block (I, J) of the grouping
    int32_t level;
    int32_t r0, rn;                 // internal particle range of the row node
    int32_t c0, cn;                 // internal particle range of the column node
    int32_t mirror;                 // index of the (J, I) block
    int32_t primary;                // 1: compressed here (r0 < c0); 0: transpose of its mirror
    int32_t rnode, cnode;           // node ids within the level
};

struct NodeRec { int32_t level, first, count; };

// Flattened work descriptors of the products ------------------------------
struct RStrip {                     // t[tmap[tmap_off + i]] = sum_j A[i + j*ld] x[x_off + j]
    int64_t a_off;                  // element offset of row `row0` col 0 of the panel
    int32_t ld, ncols, nrows;
    int32_t x_off;                  // DoF start of the column node
    int64_t tmap_off;
    int64_t p_off;                  // shared factors: this strip's row of partials P[p_off + j] =
                                    // sum_i A[i + j*ld] s[tmap[tmap_off + i]] (the mirror blocks'
                                    // R^T s); -1 otherwise
};
// One 64-row strip of a column-major panel applied to an RHS-interleaved block of P
// right-hand sides (element (row e, rhs r) at e * P + r): out rows = A_strip in rows.
// MStrip flags (pad): kStripTrans, the strip is the transpose of a stored panel slice (element
// (row r, column k) at a_off + k + r ld: the Q^T and R^T of transpose-shared factors);
// kStripAcc, the result is added to the output instead of replacing it.
constexpr int kStripTrans = 1, kStripAcc = 2;
struct MStrip {
    int64_t a_off;                  // element offset of the strip's first row, column 0
    int32_t ld, ncols, nrows, pad;  // pad: flags (1: transposed panel slice, 2: accumulate)
    int64_t in_off;                 // input row of panel column 0
    int64_t out_off;                // output row of strip row 0 (when tmap_off < 0)
    int64_t tmap_off;               // >= 0: strip row i goes to output row tmap[tmap_off + i]
};

struct QStrip {                     // y[y_off + i] = sum_j A[i + j*ld] t[t_off + j]
    int64_t a_off;
    int32_t ld, ncols, nrows;
    int64_t y_off;                  // level partial index of the strip's first row
    int64_t t_off;
    int64_t p_off;                  // shared factors: plus sum_{k < p_cnt} P[p_off + k*p_ld + i]
    int32_t p_cnt, p_ld;            // (the mirror blocks of this row node); p_cnt = 0 otherwise
};
// Shared factors, first pass: s[t_off + c] = sum_i A[i + c*ld] x[x_off + i] for the ncols
// (<= 8) columns c of a Q panel starting at a_off (s = Q^T x of the pairs whose Q it holds).
struct QtItem {
    int64_t a_off;
    int32_t ld, nrows, ncols;
    int32_t x_off;
    int64_t t_off;
};

// Batched dense-kernel descriptors -----------------------------------------
struct GemmDesc {                   // C (m x n) = op(A) (m x k) * op(B) (k x n)
    const c128* A; int64_t lda;
    const c128* B; int64_t ldb;
    c128* C; int64_t ldc;
    int32_t m, n, k;
    uint64_t seed;                  // for a generated B
    double* out_norm2;              // residual mode: ||C_ref - A B||^2 partial sink
};
struct QrcpDesc {                   // truncated column-pivoted QR of A (m x n), in place
    c128* A; int32_t m, n, lda, kmax;
    double* colnorm2;               // workspace n
    int32_t* perm;                  // n
    double* tau;                    // kmax
    c128* wtop;                     // kmax
    double rel2;                    // tolerance: trailing^2 <= rel2 * base2 - sub2
    double base2;                   // <= 0: use the initial ||A||_F^2
    double sub2;                    // < 0: use max(0, base2 - initial ||A||_F^2) (sketch residual)
    int32_t* rank_out;
    double* trail2_out;
    double* norm2_out;
    double* tol2_state;             // stepped QRCP: the tolerance, kept between launches
};
struct FormQDesc {                  // Q (m x r) = P_0 ... P_{r-1} [I_r; 0] from QRCP reflectors
    const c128* A; int32_t m, lda, r;
    const double* tau; const c128* wtop;
    c128* Q; int32_t ldq;
};
struct ExtractRDesc {               // R[:, perm[j]] = triu(A[0:r, j])
    const c128* A; int32_t lda, r, n;
    const int32_t* perm;
    c128* R; int32_t ldr;
};
struct Cgs2Desc {                   // orthonormalise the columns of Y (m x k) in place
    c128* Y; int32_t m, k, ldy;
    double drop_rel;
    int32_t* kept_out;
};
struct PackDesc {                   // copy compact factors into panel layouts
    const c128* src; int32_t rows, cols, lds; // src (rows x cols), column-major
    c128* dst; int64_t ldd; int32_t transpose; // dst(i,j) = src(i,j) or src(j,i)
    float2* dst32;                  // when set: complex64 panel, rounded to nearest (dst unused)
    const float2* src32;            // when set: complex64 compact factors (src unused)
};
// Cross approximation of a far block (rows: particles r0.., columns: c0..) without assembling
// it: U (m x kmax, ld m), V (kmax x n, stored by rows, ld n); the number of crosses goes to
// *rank_out.
constexpr int kAcaMaxRows = 147456;        // 1024 particles (used-row flags in LDS)
constexpr int kAcaMaxRank = 512;
struct AcaDesc {
    int32_t r0, rn, c0, cn;
    c128* U; c128* V;
    int32_t kmax;
    double eps;                     // stopping tolerance on the newest cross
    int32_t* rank_out;
    int32_t k0;                     // crosses already in U, V (a resumed approximation)
    int32_t* piv;                   // kmax pivot rows, in order (read for the first k0)
    double* state;                  // [running Frobenius estimate, next pivot row], kept for a resume
};
// Certification of factors Q (m x r, ld ldq) R (r x n, ld ldr) of a far block against its
// entries generated on the fly (48 x 48 tiles).
struct CertDesc {
    int32_t r0, rn, c0, cn;
    const c128* Q; int32_t ldq;
    const c128* R; int32_t ldr;
    int32_t r;
};
struct AsmDesc {                    // far block assembly: rows of particles r0.., cols c0..
    c128* B; int64_t ldb;
    int32_t r0, rn, c0, cn;
};

// ---------------------------------------------------------------- handles
}  // namespace qrvie

struct qrvie_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    size_t budget = 0;
    std::atomic<size_t> in_use{0};  // atomic: the server frees operators from other threads
    std::atomic<size_t> peak{0};    // high-water mark of in_use since creation or the last reset
    std::string err;
    void* scratch = nullptr;        // device address of this device's fixed product scratch
    std::string scratch_err;        // why it is missing, when it is
};

struct qrvie_geom {
    qrvie_ctx* ctx = nullptr;
    int32_t N = 0;
    int32_t L = 0;
    bool paper_grid = false;                  // grouping on the paper's 3 x 3-rooted grid
    double wavelength = 1.0, k = 0.0;
    std::vector<int32_t> i2c, c2i;            // internal <-> caller particle index
    std::vector<int32_t> ptype;               // internal particle -> type
    std::vector<qrvie::PType> types;
    std::vector<double> center;               // internal order, N x 3
    std::vector<qrvie::NodeRec> nodes;        // all occupied nodes, all levels
    std::vector<std::vector<int32_t>> level_nodes;  // level -> node ids (Morton order)
    std::vector<qrvie::BlockRec> blocks;      // sorted by (level, r0, c0)
    // device
    double* d_center = nullptr;               // N x 3
    int32_t* d_ptype = nullptr;               // N
    int32_t* d_i2c = nullptr;                 // N
    double* d_tvol = nullptr;                 // ntypes
    double* d_taeq = nullptr;
    qrvie::c128* d_tchi = nullptr;
    double* d_toff = nullptr;                 // ntypes x 48 x 3
    int32_t* d_trep = nullptr;                // ntypes: a representative internal particle
    size_t dev_bytes = 0;
    int64_t ndof() const { return (int64_t)N * qrvie::kNp; }
};

struct qrvie_op {
    qrvie_ctx* ctx = nullptr;
    const qrvie_geom* g = nullptr;
    qrvie_compress_opts opts{};
    int32_t ntypes = 0;
    qrvie::c128* d_self = nullptr;            // ntypes x 144 x 144 (column-major)
    qrvie::c128* d_pinv = nullptr;            // inverses
    qrvie::c128* d_fac = nullptr;             // all panels
    float2* d_fac32 = nullptr;                // complex64 copy of the panels (far_prec = C64), same offsets
    int64_t fac_elems = 0;
    int64_t t_len = 0;                        // length of the rank-space vector (per-call workspace)
    int64_t* d_tmap = nullptr;                // stacked R row -> t index
    int64_t tmap_len = 0;
    qrvie::RStrip* d_rstrips = nullptr;
    qrvie::QStrip* d_qstrips = nullptr;
    // Transpose-shared factors (share_transpose): one Q, R per unordered pair; the mirror block
    // (J, I) is applied as R^T (Q^T x_I).  The product then runs three passes: s = Q^T x over the
    // Q panels (d_qt), t = R x with the mirror partials R^T s over the R panels, y = Q t plus
    // those partials over the Q panels.
    bool shared = false;
    qrvie::QtItem* d_qt = nullptr;
    int64_t n_qt = 0;
    int64_t p_len = 0;                        // mirror partials per product (complex entries)
    qrvie::MStrip* d_mr = nullptr;            // R, Q and self-block strips for blocks of right-hand sides
    qrvie::MStrip* d_mq = nullptr;
    qrvie::MStrip* d_ms = nullptr;            // offsets into d_self and d_pinv (same layout)
    int64_t n_mr = 0, n_mq = 0, n_ms = 0;
    // shared factors, blocks of right-hand sides: Q^T strips (output through d_tinv, the
    // inverse of the rank map) and R^T strips over every node's rows (they write the level
    // partials, which the Q strips then accumulate into)
    qrvie::MStrip* d_mqt = nullptr;
    qrvie::MStrip* d_mrt = nullptr;
    int64_t n_mqt = 0, n_mrt = 0;
    int64_t* d_tinv = nullptr;
    // reduced-precision copies: self blocks and inverses in complex64 (the FP32 near part of
    // the products on FP32 matrix cores) and BF16 split-complex factor planes (far_prec
    // QRVIE_PREC_BF16X2: the real parts of every panel entry, then the imaginary parts)
    float2* d_self32 = nullptr;
    float2* d_pinv32 = nullptr;
    uint16_t* d_fac16 = nullptr;
    // strip product tile variant per (complex64 panels?, nt - 1, group R / Q / self), set by
    // qrvie_op_tune_block; 0 (the default shape) until tuned
    std::atomic<int> tile[2][4][3]{};
    int tile_of(bool lo, int nt, int group) const {
        return tile[lo ? 1 : 0][std::min(std::max(nt, 1), 4) - 1][group].load(std::memory_order_relaxed);
    }
    struct Launch { int level; int64_t begin, count; int waves; };
    std::vector<Launch> rlaunch, qlaunch;
    int32_t n_active = 0;
    std::vector<qrvie::BlockRec> blocks;      // the compressed pair blocks (after any row cap)
    std::vector<int32_t> rank;                // per block
    std::vector<double> relerr;               // per block
    std::vector<int64_t> q_off;               // Q_b first element in d_fac (ld = m_b)
    std::vector<int64_t> r_off;               // R_b (row 0, col 0) in d_fac
    std::vector<int32_t> r_ld;
    qrvie_op_stats stats{};
    std::vector<std::pair<void*, size_t>> allocs;  // owned device memory
    size_t dev_bytes = 0;
};

namespace qrvie {

// ---------------------------------------------------------------- helpers
bool set_err(qrvie_ctx* ctx, const std::string& msg);
qrvie_status hip_check(qrvie_ctx* ctx, hipError_t e, const char* what);
qrvie_status dalloc(qrvie_ctx* ctx, void** p, size_t bytes, const char* what);
void dfree(qrvie_ctx* ctx, void* p, size_t bytes);

// The compressed pair blocks of an operator: the grouping's far/finest pairs with far pairs of
// more than `cap` rows or columns split into their child pairs (0 = no cap), sorted by
// (level, r0, c0), with mirrors set.
std::vector<BlockRec> split_blocks(const qrvie_geom* g, int64_t cap);
// Device bytes of an operator built with options o: `resident` once built (panels, self
// blocks, preconditioner, strip lists) and `transient` during the build (compact factors
// before packing, the largest chunk of materialised blocks with its sketches).  Ranks follow
// a model bounded by the largest ranks measured per block size; chunk_bytes = 0 is taken as
// its automatic maximum of 64 GiB.
void op_footprint(const qrvie_geom* g, const qrvie_compress_opts* o, size_t* resident, size_t* transient);

// Look up (once per device, with that device current) the device address of the library's
// fixed scratch array used by qrvie_apply_noalloc; false with a message on failure.
bool scratch_setup(int device, void** ptr, std::string* err);
// y = Z_QR x for one caller-order vector on stream s, with caller-provided workspaces: the
// rank-space vector T (t_len), the level partials Ylev (n_active x n), for shared factors the
// rank-space Q^T x Sq (t_len) and the mirror partials P (p_len), and two permuted vectors xi,
// yi (n each).  Launches only.
void apply_single_into(const qrvie_op* op, hipStream_t s, c128* T, c128* Ylev, c128* Sq, c128* P, c128* xi, c128* yi,
                       const c128* x, c128* y);

// ---------------------------------------------------------------- launchers
// assembly (k_assemble.hip)
void launch_assemble_self(hipStream_t s, const qrvie_geom* g, c128* out, int ntypes);
void launch_assemble_far(hipStream_t s, const qrvie_geom* g, const AsmDesc* d_descs,
                         const int32_t* d_work_block, const int32_t* d_work_col, int64_t nwork);
void launch_assemble_lists(hipStream_t s, const qrvie_geom* g, const int32_t* d_rows, int32_t nr,
                           const int32_t* d_cols, int32_t nc, c128* B, int64_t ldb);
void launch_rhs(hipStream_t s, const qrvie_geom* g, int nrhs, const double* d_par, c128* v, int64_t ldv);
// wide: 1024 threads per block (for blocks of many rows and columns), else 256
void launch_aca(hipStream_t s, const qrvie_geom* g, const AcaDesc* d, int n, bool wide);
// Certification of far-block factors against entries generated on the fly: workgroup w of
// the launch writes partial[w] = ||B - Q R||^2 and partial[nwg + w] = ||B||^2 over its region;
// the workgroups of descriptor i are [wg_first[i], wg_first[i + 1]), cert_workgroups(rn, cn)
// of them per block.
void launch_cert_fused(hipStream_t s, const qrvie_geom* g, const CertDesc* d, const int64_t* wg_first, int nd,
                       int64_t nwg, double* partial);
int64_t cert_workgroups(int32_t rn, int32_t cn);
void launch_permute(hipStream_t s, int32_t N, const int32_t* d_i2c, const c128* in, c128* out, int to_internal);

// dense linear algebra (k_linalg.hip)
void launch_gemm(hipStream_t s, int mode, const GemmDesc* d_descs, const int32_t* d_tile_desc,
                 const int32_t* d_tile_mn, int64_t ntiles);
void launch_qrcp(hipStream_t s, const QrcpDesc* d, int n, int maxrows);
// maxrows / maxcols / maxsteps: largest m, n and min(kmax, m, n) over the matrices
void launch_qrcp_stepped(hipStream_t s, const QrcpDesc* d, int n, int maxrows, int maxcols, int maxsteps);
void launch_form_q(hipStream_t s, const FormQDesc* d, int n, int maxrows);
void launch_gemm_residual(hipStream_t s, const GemmDesc* d, const int32_t* td, const int32_t* tmn, int64_t nt,
                          double* partial);
void launch_extract_r(hipStream_t s, const ExtractRDesc* d, int n);
void launch_cgs2(hipStream_t s, const Cgs2Desc* d, int n, int kmax);   // kmax: widest sketch, <= 512
void launch_pack(hipStream_t s, const PackDesc* d, int n);
void launch_frob2(hipStream_t s, const c128* const* d_ptr, const int64_t* d_len, double* out, int n);
void launch_invert(hipStream_t s, c128* A, int nmat, int* d_info);
void launch_sum_partials(hipStream_t s, const double* part, const int32_t* d_first, const int32_t* d_count,
                         double* out, int n);

// products (k_apply.hip)
void launch_rphase(hipStream_t s, const RStrip* st, int64_t n, int waves, const c128* fac,
                   const c128* x, c128* t, const int64_t* tmap);
void launch_qphase(hipStream_t s, const QStrip* st, int64_t n, int waves, const c128* fac,
                   const c128* t, c128* y);
// shared factors: s = Q^T x, then t = R x with the mirror partials P (R^T s), then the Q phase
// (whose strips add the partials)
void launch_qtphase(hipStream_t s, const QtItem* it, int64_t n, const c128* fac, const c128* x, c128* S);
void launch_qtphase(hipStream_t s, const QtItem* it, int64_t n, const float2* fac, const c128* x, c128* S);
void launch_rphase_sh(hipStream_t s, const RStrip* st, int64_t n, const c128* fac, const c128* x, c128* t,
                      const int64_t* tmap, const c128* S, c128* P);
void launch_rphase_sh(hipStream_t s, const RStrip* st, int64_t n, const float2* fac, const c128* x, c128* t,
                      const int64_t* tmap, const c128* S, c128* P);
void launch_qphase_sh(hipStream_t s, const QStrip* st, int64_t n, const c128* fac, const c128* t, const c128* P,
                      c128* y);
void launch_qphase_sh(hipStream_t s, const QStrip* st, int64_t n, const float2* fac, const c128* t, const c128* P,
                      c128* y);
void launch_final(hipStream_t s, int32_t N, const int32_t* ptype, const c128* self, const c128* pinv,
                  const c128* x, const c128* ylev, int nlev, int64_t n, const c128* v,
                  c128* out_r, c128* out_z);
void launch_block_apply(hipStream_t s, int32_t N, const int32_t* ptype, const c128* blocks,
                        const c128* x, c128* y);
// many right-hand sides (nr in {2, 4, 8}), RHS-interleaved blocks
void launch_rphase_m(hipStream_t s, int nr, const RStrip* st, int64_t n, const c128* fac, const c128* X, c128* T,
                     const int64_t* tmap);
void launch_qphase_m(hipStream_t s, int nr, const QStrip* st, int64_t n, const c128* fac, const c128* T, c128* Y);
void launch_final_m(hipStream_t s, int nr, int32_t N, const int32_t* ptype, const c128* self, const c128* pinv,
                    const c128* X, const c128* ylev, int nlev, int64_t n, const c128* V, c128* out_r, c128* out_z);
// complex64 factor panels (the reduced-precision operator), FP64 accumulation
void launch_to_c64(hipStream_t s, const c128* in, float2* out, int64_t n);
// BF16 split-complex planes of complex64 values (round to nearest even): re[i], re[plane + i] = im
void launch_to_bf16(hipStream_t s, const float2* in, uint16_t* out, int64_t n, int64_t plane);
void launch_rphase_c64(hipStream_t s, const RStrip* st, int64_t n, const float2* fac, const c128* x, c128* t,
                       const int64_t* tmap);
void launch_qphase_c64(hipStream_t s, const QStrip* st, int64_t n, const float2* fac, const c128* t, c128* y);
void launch_rphase_m_c64(hipStream_t s, int nr, const RStrip* st, int64_t n, const float2* fac, const c128* X,
                         c128* T, const int64_t* tmap);
void launch_qphase_m_c64(hipStream_t s, int nr, const QStrip* st, int64_t n, const float2* fac, const c128* T,
                         c128* Y);
void launch_interleave(hipStream_t s, int nr, int64_t n, const c128* const* cols, c128* blk, int ncols);
void launch_deinterleave(hipStream_t s, int nr, int64_t n, const c128* blk, c128* const* cols, int ncols);

// Krylov helpers (k_krylov.hip)
int krylov_nchunks(int64_t n);      // multidot / norm2 partial count
int krylov_nblocks(int64_t n);      // gemv_sub partial count
void launch_multidot(hipStream_t s, const c128* V, int64_t ldv, int ncols, const c128* w, const c128* u, int64_t n,
                     c128* partial, c128* upartial);
void launch_reduce_dots(hipStream_t s, const c128* partial, int nchunks, int ncols, c128* h, c128* mirror,
                        int64_t mstride);
void launch_cgs2_coeffs(hipStream_t s, const c128* partial, int nchunks, int ncols, c128* h);
void launch_gemv_sub(hipStream_t s, const c128* V, int64_t ldv, int ncols, const c128* h, c128* w, int64_t n,
                     double* npart);
void launch_norm2(hipStream_t s, const c128* w, int64_t n, double* partial);
void launch_reduce_norm(hipStream_t s, const double* partial, int count, double* out);
void launch_scale_into(hipStream_t s, const c128* w, int64_t n, const double* norm2, c128* out, c128* gslot);
void launch_givens(hipStream_t s, int j, c128* hcol, c128* H, int ldh, double* cs, c128* sn, c128* gvec,
                   const double* hnorm2, double* status);
void launch_trisolve(hipStream_t s, int k, const c128* H, int ldh, const c128* gvec, c128* y);
// *out = max(*out, max_ij |G_ij - delta_ij|) over the leading k x k block (out >= 0 on entry)
void launch_gram_deviation(hipStream_t s, const c128* G, int64_t ldg, int k, double* out);
void launch_gemv_add(hipStream_t s, const c128* V, int64_t ldv, int ncols, const c128* y, c128* x, int64_t n);
void launch_add(hipStream_t s, const c128* d, int64_t n, c128* x);
void launch_rsub(hipStream_t s, const c128* a, int64_t n, c128* y);   // y = a - y
void launch_read_probe(hipStream_t s, const c128* p, int64_t n, int grid, int u, double* out);
void launch_mfma_probe(hipStream_t s, bool f64, int grid, int iters, double* out);

// blocks of right-hand sides (k_block.hip); nt = P / 16 tiles of 16 right-hand sides, 1..4
constexpr int kMaxBlockRhs = 64;
// Strip product tile shapes: variant v loads strip_variant_u(v) 4-column steps per batch and
// gives each wave strip_variant_rows(v) rows; 0 is the untuned default.  All variants give
// bitwise-identical results.
constexpr int kStripVariants = 6;
int strip_variant_u(int v);
int strip_variant_rows(int v);
void launch_strip_mfma(hipStream_t s, int nt, const MStrip* st, int64_t n, const c128* fac, const c128* in,
                       c128* out, const int64_t* tmap, int variant = 0);
void launch_strip_mfma(hipStream_t s, int nt, const MStrip* st, int64_t n, const float2* fac, const c128* in,
                       c128* out, const int64_t* tmap, int variant = 0);
// The strip products on FP32 matrix cores with FP32 accumulation: complex64 panels, or BF16
// split-complex planes (imaginary plane `plane` entries after the real one); one tile shape.
void launch_strip_mfma32(hipStream_t s, int nt, const MStrip* st, int64_t n, const float2* fac, const c128* in,
                         c128* out, const int64_t* tmap);
void launch_strip_mfma32_bf16(hipStream_t s, int nt, const MStrip* st, int64_t n, const uint16_t* fac, int64_t plane,
                              const c128* in, c128* out, const int64_t* tmap);
void launch_count_neq(hipStream_t s, int64_t n, const void* a, const void* b, unsigned long long* count);
void launch_block_combine(hipStream_t s, int nt, int64_t n, const c128* ylev, int nlev, const c128* yself,
                          const c128* V, c128* out);
void launch_gather_block(hipStream_t s, int nt, int32_t N, const int32_t* i2c, const c128* src, int64_t ld,
                         int ncols, c128* blk);
void launch_scatter_block(hipStream_t s, int nt, int32_t N, const int32_t* i2c, const c128* blk, c128* dst,
                          int64_t ld, int ncols);
void launch_gram_store(hipStream_t s, int k, int p, const c128* C, int64_t ldc, c128* G, int64_t ldg);
void launch_cholesky(hipStream_t s, int p, const c128* S, int64_t lds, double rel, c128* out, int64_t ldo, int* flag);
void launch_trmm_upper(hipStream_t s, int p, const c128* A, int64_t lda, const c128* B, int64_t ldb, c128* C,
                       int64_t ldc, const int* flag);
void launch_cholesky_piv(hipStream_t s, int p, const c128* S, int64_t lds, double rel, c128* out, int64_t ldo,
                         int* perm, int* qout);
void launch_trmm_perm(hipStream_t s, int q, int p, const c128* A, int64_t lda, const c128* B, int64_t ldb,
                      const int* perm, c128* out, int64_t ldo);
void launch_ls_apply(hipStream_t s, int j0, int j1, int p, const c128* Y, const c128* T, c128* C, int64_t ldc,
                     int ncols);
void launch_ls_factor(hipStream_t s, int k, int p, c128* C, int64_t ldc, c128* Yk, c128* Tk);
void launch_col_norms(hipStream_t s, int rows, const c128* C, int64_t ldc, int ncols, double* out);
void launch_sum_batches(hipStream_t s, int m, int c, int nb, const c128* P, c128* C, int64_t ldc);
// Split-K partials of C = A^H B (n-row A: m columns, B: c columns): chunk z < nb covers rows
// [z L, min(n, (z + 1) L)) and writes P[z m c + i + j m]; launch_sum_batches reduces them.
void launch_gemm_hn_part(hipStream_t s, int64_t n, int m, int c, const c128* A, int64_t lda, const c128* B, int64_t ldb,
                         int nb, int64_t L, c128* P);
// out (k x k) = U^-1 for an upper triangular k x k U, k <= 256
void launch_tri_inv_upper(hipStream_t s, int k, const c128* U, int64_t ldu, c128* out, int64_t ldo);
// Y (m x p) = U^-1 Y for an upper triangular m x m U
void launch_trsm_upper_left(hipStream_t s, int m, int p, const c128* U, int64_t ldu, c128* Y, int64_t ldy);
// W (n x q, q <= 64) = beta W + sign V H (V: n x m, H: m x q).  FP64 MFMA, fixed accumulation order.
void launch_gemm_nn_acc(hipStream_t s, int64_t n, int m, int q, const c128* V, int64_t ldv, const c128* H,
                        int64_t ldh, double beta, double sign, c128* W, int64_t ldw);

}  // namespace qrvie
