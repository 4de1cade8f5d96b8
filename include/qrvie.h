/*
 * qrvie — compressed volume-integral-equation solver for large arrays of
 * sub-wavelength particles, on one AMD Instinct MI355X (gfx950).
 *
 * C ABI.  Every call returns a qrvie_status; no exception or abort crosses
 * the boundary.  qrvie_last_error(ctx) gives a human-readable detail for the
 * last failing call on that context.
 *
 * Conventions
 *  - Complex numbers are complex128, interleaved {re, im} (torch.complex128).
 *  - Vectors and multi-vectors are DEVICE pointers owned by the caller, laid
 *    out column-major (n x nrhs) with a leading dimension >= n.  The library
 *    never frees caller memory.
 *  - Degree-of-freedom order at the ABI ("caller order"): particle in the order
 *    of qrvie_array_desc, then the particle's 48 cells in canonical order
 *    (lower layer, then upper; within a layer row b ascending, then column a
 *    ascending), then the Cartesian component x, y, z fastest: 144 DoFs per
 *    particle.  Unknowns are grouped particle by particle as in the paper's
 *    block partition of Z (§4, eq. 4.1).  Internally the library reorders
 *    particles along a Morton curve; that order never appears at the ABI
 *    except through qrvie_geom_order and block exports.
 *  - Units: lengths in the same unit as `wavelength`; k = 2 pi / wavelength.
 *  - Handles (ctx, geom, op) are library-owned.  geom and op are immutable
 *    after creation.  All device work is ordered on the context's stream;
 *    calls that return host information synchronise that stream.
 *  - A context is not thread-safe: serialise calls on one context.
 */
#ifndef QRVIE_H
#define QRVIE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QRVIE_OK = 0,
    QRVIE_ERR_INVALID_ARG = 1,   /* null pointer, bad size, NaN/Inf input, eps <= 0 */
    QRVIE_ERR_GEOMETRY = 2,      /* two particles on one lattice site, bad lattice indices */
    QRVIE_ERR_OUT_OF_MEMORY = 3, /* HBM budget of the context or device memory exhausted */
    QRVIE_ERR_DEVICE = 4,        /* a HIP runtime error; see qrvie_last_error */
    QRVIE_NOT_CONVERGED = 5,     /* soft: x holds the best iterate and info is filled */
    QRVIE_ERR_QUEUE_FULL = 6     /* server: no admission slot */
} qrvie_status;

typedef struct { double re, im; } qrvie_c128;

typedef struct qrvie_ctx qrvie_ctx;
typedef struct qrvie_geom qrvie_geom;
typedef struct qrvie_op qrvie_op;

/* Static string for a status code. */
const char* qrvie_status_string(qrvie_status s);

/* ------------------------------------------------------------------ context */
/*
 * Create a context on HIP device `hip_device`.  `hip_stream` is a hipStream_t
 * to order all work on (for instance torch.cuda.current_stream().cuda_stream);
 * NULL makes the library create and own a default-priority stream.
 * `hbm_budget` caps the bytes of device memory the library itself allocates
 * for geometries, operators and solver workspaces (0 = no cap besides the
 * device).  Caller-owned buffers do not count.
 */
qrvie_status qrvie_ctx_create(int hip_device, void* hip_stream, size_t hbm_budget, qrvie_ctx** out);
void         qrvie_ctx_destroy(qrvie_ctx* ctx);
const char*  qrvie_last_error(const qrvie_ctx* ctx);
/* Bytes currently allocated by the library on this context. */
size_t       qrvie_ctx_bytes_in_use(const qrvie_ctx* ctx);
/* High-water mark of the library's bytes on this context since its creation or the last
 * reset; reset != 0 then restarts the mark at the bytes currently in use. */
size_t       qrvie_ctx_peak_bytes(qrvie_ctx* ctx, int32_t reset);

/* ----------------------------------------------------------------- geometry */
/*
 * An array of meta-atoms (the paper's scatterers, §6.1), each voxelised into 48
 * cells with three current components per cell.  All pointers are HOST
 * pointers, read during the call only.
 *   n                  number of particles (>= 1)
 *   centers[n][3]      particle centres; the disks' axes are along z
 *   radius[n]          disk or sphere radius (> 0)
 *   height[n]          disk height (> 0; ignored for spheres)
 *   eps_r[n_eps]       relative permittivity; n_eps is 1 (shared) or n
 *   lattice_ij[n][2]   QRVIE_GRID_LATTICE: integer lattice site of each particle; sites
 *                      must be distinct.  Grouping follows the lattice (§5.4: a particle
 *                      belongs whole to the grid block containing its centre).  Ignored
 *                      (may be NULL) with QRVIE_GRID_PAPER.
 *   pitch              lattice pitch (informational; centres are authoritative)
 *   wavelength         free-space wavelength (> 0)
 *   cells_per_particle must be 48
 *   shape              QRVIE_SHAPE_DISK (0): 24 in-plane squares of side r sqrt(pi/24) in two
 *                      layers of height/2.  QRVIE_SHAPE_SPHERE (1): the voxelised sphere of the
 *                      paper's test arrays (§6.1), 48 cubes of side h = r (pi/36)^(1/3) (the
 *                      sphere's volume) in four layers, each the 12 squares of a 4 x 4 grid
 *                      without its corners.
 *   grid               QRVIE_GRID_LATTICE (0): a quadtree on the lattice sites, padded to 2^L
 *                      per side.  QRVIE_GRID_PAPER (1): the paper's grid for arrays without a
 *                      lattice (§5.3, §5.4): the root is the bounding square of the centres
 *                      (side 1 + 2^-20 times the larger extent, centred on the bounding box),
 *                      level l has 3 2^(l-1) blocks per side, each particle belongs to the block
 *                      containing its centre, and the finest level L is the first at which no
 *                      block holds two particles (at most 20; coincident centres are an error).
 */
enum { QRVIE_SHAPE_DISK = 0, QRVIE_SHAPE_SPHERE = 1 };
enum { QRVIE_GRID_LATTICE = 0, QRVIE_GRID_PAPER = 1 };
typedef struct {
    int32_t n;
    const double* centers;
    const double* radius;
    const double* height;
    const qrvie_c128* eps_r;
    int32_t n_eps;
    const int32_t* lattice_ij;
    double pitch;
    double wavelength;
    int32_t cells_per_particle;
    int32_t shape;
    int32_t grid;
} qrvie_array_desc;

/* Discretise the array (paper §3 / the voxel reading) and build the recursive
 * near/far grouping (§5.1, §5.3, §5.4).  Uploads cell data to the device. */
qrvie_status qrvie_geom_create(qrvie_ctx* ctx, const qrvie_array_desc* desc, qrvie_geom** out);
int64_t      qrvie_geom_ndof(const qrvie_geom* g);
int32_t      qrvie_geom_nlevels(const qrvie_geom* g);
/* internal_to_caller[N] (host): caller particle index of each internal particle. */
qrvie_status qrvie_geom_order(const qrvie_geom* g, int32_t* internal_to_caller);
/* Cell centres [N*48][3] and cell volumes [N*48] in caller order (host buffers). */
qrvie_status qrvie_geom_cells(const qrvie_geom* g, double* centers, double* volumes);
/* The finest-level block (i, j) of each caller particle [N][2] (host buffer): the lattice
 * site shifted to start at 0, or the paper-grid block of its centre. */
qrvie_status qrvie_geom_blocks(const qrvie_geom* g, int32_t* block_ij);
void         qrvie_geom_destroy(qrvie_geom* g);

/*
 * Assemble the dense block of Z for caller particles rows[0..nr) x cols[0..nc)
 * (host index lists) into the DEVICE buffer B (column-major, ldb >= 144*nr),
 * DoFs in the order of the lists.  Entries follow the discretised kernel:
 * Z[(m,a),(n,b)] = -k^2 V_m V_n G_ab(r_m - r_n) for distinct cells, with the
 * dyadic Green's function G = (I + grad grad / k^2) g, g = exp(-jkR)/(4 pi R)
 * (§2, eq. 2.4), and V_m [1/chi_m - s(a_m)] on the cell diagonal.
 * Stream-ordered; B is valid after the stream reaches this point.
 */
qrvie_status qrvie_assemble(qrvie_ctx* ctx, const qrvie_geom* g, int32_t nr, const int32_t* rows,
                            int32_t nc, const int32_t* cols, qrvie_c128* B, int64_t ldb);

/* ----------------------------------------------------------------- operator */
enum { QRVIE_PREC_C128 = 0, QRVIE_PREC_C64 = 1, QRVIE_PREC_BF16X2 = 2, QRVIE_PREC_C64_ONLY = 3,
       QRVIE_PREC_C64_F32 = 4 };
enum { QRVIE_COMPRESS_ACA = 0, QRVIE_COMPRESS_SKETCH = 1 };

/*
 *   eps              per-block relative Frobenius tolerance of the low-rank
 *                    factors, ||B - Q R||_F <= eps ||B||_F (§5.2, eq. 5.3); > 0
 *   far_prec         QRVIE_PREC_C128: complex128 far factors; QRVIE_PREC_C64: in addition a
 *                    complex64 copy (rounded to nearest) used by the inner solves of
 *                    QRVIE_SOLVE_MIXED_IR, which streams half the factor bytes;
 *                    QRVIE_PREC_C64_ONLY: only complex64 far factors (half the memory), used
 *                    by every product with FP64 accumulation (the rounding, 2^-24 relative
 *                    per entry, is far below eps); MIXED_IR and complex128 products are
 *                    then refused, and exports return the complex64 values widened.
 *                    QRVIE_PREC_BF16X2: the complex64 far factors of C64_ONLY (every product and
 *                    residual with FP64 accumulation) plus a BF16 split-complex copy (real parts,
 *                    then imaginary parts; FP64 -> FP32 -> BF16, each rounded to nearest even),
 *                    which the corrections of QRVIE_SOLVE_BLOCK_IR apply on FP32 matrix cores with
 *                    FP32 accumulation and complex64 self blocks (the precision pattern's inner
 *                    operator).  Every operator built with complex64 factors also keeps complex64
 *                    copies of the self blocks and their inverses for the FP32 products.
 *   near_prec        storage of the self blocks: QRVIE_PREC_C128 only for now
 *   max_block_rows   far blocks with more rows are split into their child
 *                    pairs (always far); 0 = no cap (the paper's scheme)
 *   share_transpose  0: every ordered far block (I, J) and its mirror (J, I) keep their own
 *                    panels (the mirror holds the transposed factors).  1: one Q, R per
 *                    unordered pair, the mirror applied as R^T (Q^T x_I) (Z = Z^T, the symmetric
 *                    weak form, §2 eq. 2.5): half the factor memory, and a single-RHS product
 *                    streams each pair's Q twice and its R once instead of both twice.  Every
 *                    product and solver mode takes shared operators (2-15 right-hand sides one
 *                    single-RHS product per column; 16 or more, and the FP32 forms, block products
 *                    with Q^T and R^T strips); qrvie_op_profile_block and qrvie_op_tune_block
 *                    refuse them (QRVIE_ERR_INVALID_ARG).
 *   seed             seed of the random sketches used by compression
 *   verbose          1: print one progress line per compression chunk to stderr
 *   chunk_bytes      device bytes compressed together; 0 = a quarter of the free device
 *                    memory (or of the context's remaining budget), at most 64 GiB.  Larger
 *                    chunks keep more blocks in flight.  Cross approximation counts its working
 *                    buffers (about 32 (m + n) k bytes per block of k crosses), the sketch path
 *                    its materialised blocks.
 *   compression      how blocks of more than 2 x 2 particles are compressed (smaller ones always
 *                    by the truncated pivoted QR of the assembled block):
 *                    QRVIE_COMPRESS_ACA (0, the default): cross approximation, the compression
 *                    of §6.5 (after Kurz et al. 2002).  Only the pivot rows and columns of a
 *                    block are generated (256 crosses at first, continued up to 512 when all are
 *                    used, stopping at 0.05 eps); the crosses are recompressed by a truncated
 *                    pivoted QR at 0.9 eps, and the factors are certified against every entry of
 *                    the block generated again, so eq. 5.3 holds exactly as with the sketch.  A
 *                    block that misses eps is redone twice with a tenfold tighter stopping
 *                    tolerance, then by the sketch path.  aca_start and aca_stop set the first
 *                    number of crosses and the stopping tolerance (the op's stats count the
 *                    continuations, repeats and sketch fallbacks).  No far block is materialised, so
 *                    max_block_rows is not needed for memory; blocks above 147456 rows (1024
 *                    particles) are split into their child pairs by the operator itself.
 *                    QRVIE_COMPRESS_SKETCH (1): every block is assembled and compressed through
 *                    a randomised range sketch (CGS2 basis, projection, truncated pivoted QR),
 *                    certified against the assembled block.
 */
typedef struct {
    double eps;
    int32_t far_prec;
    int32_t near_prec;
    int64_t max_block_rows;
    int32_t share_transpose;
    uint64_t seed;
    int32_t verbose;
    int64_t chunk_bytes;
    int32_t compression;
    int32_t aca_start;       /* crosses per block at first, 1..512 (0 = 256) */
    double  aca_stop;        /* stopping tolerance of the crosses relative to eps, > 0 (0 = 0.05) */
} qrvie_compress_opts;

#define QRVIE_MAX_LEVELS 24

typedef struct {
    int32_t n_levels;
    int64_t n_blocks;                         /* ordered far/finest pairs */
    int64_t n_blocks_level[QRVIE_MAX_LEVELS];
    int32_t min_rank_level[QRVIE_MAX_LEVELS];
    int32_t max_rank_level[QRVIE_MAX_LEVELS];
    double  mean_rank_level[QRVIE_MAX_LEVELS];
    int32_t n_self_types;                     /* distinct self blocks (identical atoms share one) */
    int64_t n_qr_entries;                     /* N_QR of eq. 5.6 (complex entries) */
    double  gain;                             /* G = N_dof^2 / N_QR, eq. 5.5 */
    double  max_block_rel_err;                /* certified max_b ||B - QR||_F / ||B||_F */
    int64_t apply_bytes;                      /* algorithmic HBM bytes of one single-RHS product */
    int64_t device_bytes;                     /* device memory held by the operator */
    double  t_assembly_s, t_compression_s, t_precond_setup_s;
    int64_t apply_bytes_c64;                  /* the same product with complex64 far factors (0: none) */
    int64_t n_aca;                            /* cross approximation: blocks compressed by it */
    int64_t n_aca_resumed;                    /*   continuations in wider buffers (all crosses used) */
    int64_t n_aca_retried;                    /*   repeats with a tighter stopping tolerance */
    int64_t n_aca_sketch;                     /*   blocks left to the sketch path */
} qrvie_op_stats;

typedef struct {
    int32_t level;
    int32_t m, n, rank;
    int32_t row_first, row_count;   /* internal particle range of the row block */
    int32_t col_first, col_count;   /* internal particle range of the column block */
    double rel_err;                 /* certified ||B - QR||_F / ||B||_F */
} qrvie_block_info;

/*
 * Estimate, before the build, of the peak device bytes of qrvie_op_create with options o: the
 * operator once built (factor panels of the precision o->far_prec, self blocks and their
 * inverses, strip lists) plus the build's transient buffers (the compact factors before they
 * are packed; the largest compression chunk of materialised blocks with its direct-QR copies
 * and sketches, chunk_bytes = 0 counted as its 64 GiB maximum).  It follows the same block
 * list as the build (o->max_block_rows applied).  Ranks are not known before compression: the
 * estimate assumes per block min(m, n, r_model) with r_model above the largest ranks measured
 * for each block size at eps = 1e-6 (80 up to 2304 rows, 100 up to 9216, 128 up to 36,864, 160
 * beyond) plus 14 per decade below 1e-6.  It is therefore an estimate, not a guarantee: an
 * array whose ranks exceed the model needs more.  QRVIE_ERR_INVALID_ARG for invalid options.
 */
qrvie_status qrvie_op_footprint_estimate(const qrvie_geom* g, const qrvie_compress_opts* o, size_t* bytes);
/*
 * Build the compressed operator Z_QR: self blocks Z_pp and the preconditioner
 * Z_D^-1 (§4, eq. 4.2), then every far/finest pair block of the recursive
 * grouping as certified low-rank factors Q R (§5.2-5.4).  Z_QR is exactly
 * complex-symmetric: the pair (J, I) stores the transpose of the factors of
 * (I, J).  Fails with QRVIE_ERR_OUT_OF_MEMORY if the footprint estimate (at the chunk size
 * the build will use) exceeds the context's remaining budget.
 */
qrvie_status qrvie_op_create(qrvie_ctx* ctx, const qrvie_geom* g, const qrvie_compress_opts* o, qrvie_op** out);
qrvie_status qrvie_op_stats_get(const qrvie_op* op, qrvie_op_stats* out);
int64_t      qrvie_op_num_blocks(const qrvie_op* op);
/* Export block b's factors to HOST buffers Q[m*rank] and R[rank*n] (column-major;
 * either may be NULL).  Rows/columns in internal DoF order of the particle ranges. */
qrvie_status qrvie_op_export_block(const qrvie_op* op, int64_t b, qrvie_block_info* info,
                                   qrvie_c128* Q, qrvie_c128* R);
/* Export the self block Z_pp and/or its inverse of caller particle p (HOST, 144x144 column-major). */
qrvie_status qrvie_op_export_self(const qrvie_op* op, int32_t p, qrvie_c128* Zpp, qrvie_c128* Zpp_inv);
void         qrvie_op_destroy(qrvie_op* op);

/* ---------------------------------------------------------------- products */
/* y = Z_QR x for nrhs columns (device pointers, caller order): the compressed
 * product Z_D x + sum_b Q_b (R_b x_J) of §5.2. */
qrvie_status qrvie_apply(qrvie_ctx* ctx, const qrvie_op* op, int32_t nrhs,
                         const qrvie_c128* x, int64_t ldx, qrvie_c128* y, int64_t ldy);
/* The same product with the far factors of precision prec: QRVIE_PREC_C128 (as qrvie_apply),
 * QRVIE_PREC_C64 (the complex64 factors; products accumulate in FP64), QRVIE_PREC_C64_F32 (the
 * complex64 factors and self blocks on FP32 matrix cores, right-hand sides rounded to FP32,
 * FP32 accumulation) or QRVIE_PREC_BF16X2 (the BF16 planes, likewise with FP32 self blocks).
 * The two FP32 forms run the block product for any nrhs.  An operator built without factors of
 * that precision gives QRVIE_ERR_INVALID_ARG. */
qrvie_status qrvie_apply_prec(qrvie_ctx* ctx, const qrvie_op* op, int32_t prec, int32_t nrhs,
                              const qrvie_c128* x, int64_t ldx, qrvie_c128* y, int64_t ldy);
/*
 * Stage timers of the single-RHS product (the product stage of the paper's timing
 * table, §6.5), measured with HIP events on the context stream: each stage over `reps`
 * back-to-back launches of its own kernel (its average launch duration), the whole product
 * over `reps` products, on a fixed internal test vector.  ms[0] R-phase (t = R x for every block; with shared
 * factors also the mirror partials R^T s), ms[1] Q-phase (y_l = Q t per level, with shared
 * factors plus the mirror partials), ms[2] final pass (self blocks Z_pp x + level sum), ms[3]
 * whole product, ms[4] the Q^T pass s = Q^T x of shared factors (0 otherwise), ms[5] = 0;
 * averages per product.  bytes[0..5]: algorithmic HBM bytes of the same stages per product
 * (factor, self-block and vector traffic, x counted once; the per-level and mirror partial
 * vectors are counted as overhead, not algorithmic bytes).  Host arrays of 6.  prec selects
 * the far factors as in qrvie_apply_prec (complex64 factors count 8 bytes per entry).
 */
qrvie_status qrvie_op_profile_apply(qrvie_ctx* ctx, const qrvie_op* op, int32_t prec, int32_t reps, double* ms,
                                    int64_t* bytes);
/*
 * Stage timers of the block product used by QRVIE_SOLVE_BLOCK and by qrvie_apply with 16 or
 * more right-hand sides, for nrhs (1..64) right-hand sides padded to a multiple of 16:
 * ms[0] R-phase, ms[1] Q-phase, ms[2] self blocks + level sum, ms[3] block preconditioner,
 * averages over `reps` products of a zero block.  flops[0..3]: real floating-point
 * operations of the same stages (8 per complex multiply-add of a factor or self-block entry
 * with each padded right-hand side).  Host arrays of 4.
 */
qrvie_status qrvie_op_profile_block(qrvie_ctx* ctx, const qrvie_op* op, int32_t nrhs, int32_t reps, double* ms,
                                    int64_t* flops);
/*
 * Autotuner of the block product's tile shapes (the rank-grouped strip GEMMs of the
 * multi-right-hand-side product, §5.2).  The strips fall in three groups: R panels, Q panels
 * and the self blocks (whose choice also serves the block preconditioner).  For each group
 * every tile shape (variant v: u[v] 4-column steps per load batch, rows_per_wave[v] rows per
 * wavefront) is timed over `reps` launches (1..100) on a fixed pseudo-random block of
 * 16 * ceil(nrhs / 16) right-hand sides (nrhs 1..64) and compared bitwise with variant 0, the
 * untuned default; the fastest variant with no differing entry is kept in the operator and
 * used from then on by every block product with that tile count and factor precision
 * (prec QRVIE_PREC_C128 or QRVIE_PREC_C64; an operator holding only complex64 panels tunes
 * those either way).  All variants accumulate in the same order, so tuning never changes a
 * result.  Tuning writes to `op`: no product on the same operator may run concurrently with
 * it.  Synchronises the context stream; `out` (host) receives the measurements.
 */
#define QRVIE_TUNE_VARIANTS 8
typedef struct {
    int32_t nrhs_tile;                          /* right-hand sides per product, 16 * tiles */
    int32_t n_variants;                         /* variants measured (<= QRVIE_TUNE_VARIANTS) */
    int32_t u[QRVIE_TUNE_VARIANTS];             /* 4-column steps per load batch */
    int32_t rows_per_wave[QRVIE_TUNE_VARIANTS]; /* rows of a strip per wavefront */
    double ms[3][QRVIE_TUNE_VARIANTS];          /* average launch time: R group, Q group, self group */
    int64_t mismatches[3][QRVIE_TUNE_VARIANTS]; /* entries differing bitwise from variant 0 */
    int32_t chosen[3];                          /* kept variant per group */
} qrvie_block_tune;
qrvie_status qrvie_op_tune_block(qrvie_ctx* ctx, qrvie_op* op, int32_t prec, int32_t nrhs, int32_t reps,
                                 qrvie_block_tune* out);
/*
 * Streaming-read reference for the product's roofline: reads `bytes` (a multiple of 16) of
 * device memory at `d` with the product kernels' nontemporal 16-byte loads over a few grid
 * sizes and load depths, `reps` (1..100) times each, and returns the best read rate in GB/s
 * (host double).  A measurement helper, not a step of the method.
 */
qrvie_status qrvie_probe_read(qrvie_ctx* ctx, const void* d, size_t bytes, int32_t reps, double* gbs);
/*
 * Matrix-core rate reference: back-to-back 16x16x4 MFMAs (f64 = 1: FP64, 0: FP32) on
 * register data over the whole device; *tfs (host) receives TFLOP/s.  A measurement helper.
 */
qrvie_status qrvie_probe_mfma(qrvie_ctx* ctx, int32_t f64, double* tfs);
/*
 * y = Z_QR x for ONE right-hand side without allocating any device memory: for callers that
 * cannot allocate (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The same kernels and result as qrvie_apply with nrhs = 1.  x and y are device
 * vectors of n entries (caller order), y must not overlap x.  Stream-ordered on the context's
 * stream and asynchronous: the call neither synchronises nor allocates; y is valid once the
 * stream reaches this point.  Workspaces come from a fixed device array of 64 MiB per device,
 * held from the first context created on that device until the process ends; the product
 * needs 16 (2 n + sum of ranks + n x active levels) bytes (the mid-size 32 x 32 array fits,
 * a 48 x 48 array does not), and larger operators are refused with QRVIE_ERR_INVALID_ARG (use
 * qrvie_apply).  Every call on one device shares that array and leaves its contents behind:
 * calls that overlap on a device (other streams, threads or contexts) race, so serialise them.
 * QRVIE_ERR_DEVICE if the array's address could not be looked up at context creation.
 */
qrvie_status qrvie_apply_noalloc(qrvie_ctx* ctx, const qrvie_op* op, const qrvie_c128* x, qrvie_c128* y);
/* z = Z_D^-1 y, the block-diagonal left preconditioner (§4, eq. 4.2). */
qrvie_status qrvie_precondition(qrvie_ctx* ctx, const qrvie_op* op, int32_t nrhs,
                                const qrvie_c128* y, int64_t ldy, qrvie_c128* z, int64_t ldz);
/*
 * Right-hand sides v0 (eq. 3.4) for plane waves: v[(m,a)] = V_m E0_a(r_m),
 * E0(r) = e exp(-j k k^.r), k^ = (sin t cos f, sin t sin f, cos t),
 * pol 0 = TE: e = (-sin f, cos f, 0); pol 1 = TM: e = (cos t cos f, cos t sin f, -sin t).
 * Angles in degrees (host arrays of length nrhs); v is a device n x nrhs buffer.
 */
qrvie_status qrvie_rhs_plane_waves(qrvie_ctx* ctx, const qrvie_geom* g, int32_t nrhs,
                                   const double* theta_deg, const double* phi_deg,
                                   const int32_t* pol, qrvie_c128* v, int64_t ldv);

/* ------------------------------------------------------------------- solve */
/*
 * QRVIE_SOLVE_FP64      GMRES on the complex128 factors.
 * QRVIE_SOLVE_MIXED_IR  iterative refinement: residuals r = v - Z_QR x with the complex128
 *                       factors, corrections from GMRES on the complex64 copy of the far
 *                       factors (FP64 accumulation and Krylov algebra), x += d, until
 *                       ||r|| <= tol ||v||.  Needs an operator built with
 *                       far_prec = QRVIE_PREC_C64; otherwise QRVIE_ERR_INVALID_ARG.
 * QRVIE_SOLVE_BLOCK     block GMRES: up to 64 right-hand sides at a time share one block
 *                       Krylov space; every block step applies the operator to the whole
 *                       block on FP64 matrix cores.  `restart` bounds the basis vectors per
 *                       cycle (restart / block width block steps); `max_iter` bounds the
 *                       block steps.  info: iterations = block steps, n_apply = block
 *                       products, t_apply_s = product time of the whole block.  A
 *                       numerically rank-deficient block (repeated right-hand sides) is
 *                       finished column by column in FP64 mode from the block iterate; a
 *                       block of one column is solved in FP64 mode (the same Krylov space).
 * QRVIE_SOLVE_BLOCK_IR  iterative refinement as MIXED_IR, with each correction from block
 *                       GMRES (as BLOCK) for all unconverged columns together.  Residuals use
 *                       the complex128 factors (far_prec C64) or the complex64 ones with FP64
 *                       accumulation (C64_ONLY, BF16X2).  Corrections: the BF16 planes on FP32
 *                       matrix cores (BF16X2), the complex64 factors on FP32 matrix cores
 *                       (inner_fp32 = 1), else the complex64 factors widened on FP64 matrix
 *                       cores (C64).  An FP32 correction aims at a relative residual of at least
 *                       1e-5 (complex64) or 1e-2 (BF16) and further refinements take the rest.
 *                       info: iterations = block steps over all corrections, n_refine =
 *                       corrections.
 */
enum { QRVIE_SOLVE_FP64 = 0, QRVIE_SOLVE_MIXED_IR = 1, QRVIE_SOLVE_BLOCK = 2, QRVIE_SOLVE_BLOCK_IR = 3 };

typedef struct {
    int32_t restart;      /* GMRES(m) restart length, 1..16384 (m >= max_iter: unrestarted, as in §6);
                             the basis takes (m + 1) x n complex128 of device memory */
    int32_t max_iter;     /* total Arnoldi steps per right-hand side */
    int32_t mode;         /* QRVIE_SOLVE_FP64, _MIXED_IR, _BLOCK or _BLOCK_IR */
    double  tol;          /* relative residual; converged when both the preconditioned
                             estimate and the true residual ||v - Z_QR x||/||v|| meet it */
    int32_t use_x0;       /* 1: x holds the initial guess on entry; 0: x0 = 0 */
    double  inner_tol;    /* MIXED_IR: relative tolerance of each correction solve, in (0, 1);
                             0 = automatic, 0.25 tol ||v|| / ||r|| (one correction reaches tol
                             unless the factor rounding dominates).  Ignored in FP64 mode. */
    int32_t verbose;      /* BLOCK: 1 prints one progress line per 10 block steps and per cycle
                             to stderr */
    int32_t block_width;  /* BLOCK: right-hand sides per block, 1..64 (0 = 64).  Narrower blocks
                             need fewer basis vectors in total for the same accuracy, so a
                             block that must fit a fixed basis without restarting can be
                             split. */
    int32_t inner_fp32;   /* BLOCK_IR: 1 applies the corrections' complex64 factors on FP32 matrix
                             cores (FP32 accumulation) instead of widening them to FP64; 0 or 1 */
} qrvie_solve_opts;

typedef struct {
    int32_t iterations, restarts, converged;
    double  rel_res_prec, rel_res_true;
    int32_t n_apply, n_prec;
    double  t_apply_s, t_prec_s, t_krylov_s, t_total_s;
    int32_t n_reorth;     /* Arnoldi steps whose projection carries the second Gram-Schmidt
                             correction.  The single-vector solver computes it through the Gram
                             matrix G = V^H V of the stored basis (coefficients 2 h1 - G h1, one
                             pass over the basis), not as a second pass; basis_ortho measures
                             what that leaves */
    int32_t n_refine;     /* MIXED_IR: correction solves (iterations and n_apply count all of
                             them; rel_res_prec is the last correction's own estimate) */
    double  basis_ortho;  /* FP64 and MIXED_IR: max_ij |(V^H V - I)_ij| over the Krylov basis of
                             every cycle (the largest), from the Gram matrix of the stored basis;
                             0 in the block modes */
} qrvie_solve_info;

/* Upper bound of the device bytes qrvie_solve allocates for nrhs right-hand sides
 * (Krylov bases, Hessenberg data and product workspaces), for admission control by
 * callers that share one device; `op` may be NULL before the operator exists.  The
 * estimate follows opts->mode: one group of up to 8 columns with `restart` basis vectors
 * each (FP64, MIXED_IR), or one block of up to block_width columns sharing `restart` basis
 * vectors (BLOCK; a rank-deficient block is finished by the single-vector solver with the
 * same total of basis vectors, restart / min(columns, 8) per column). */
qrvie_status qrvie_solve_footprint_estimate(const qrvie_geom* g, const qrvie_op* op, int32_t nrhs,
                                            const qrvie_solve_opts* opts, size_t* bytes);

/*
 * Solve Z_QR x = v with left-preconditioned restarted GMRES (the paper's
 * solver with the preconditioner of §4), one right-hand side after another.
 * v, x: device n x nrhs (caller order).  info: host array of nrhs entries
 * (may be NULL).  Returns QRVIE_NOT_CONVERGED (soft) if any column missed tol.
 */
qrvie_status qrvie_solve(qrvie_ctx* ctx, const qrvie_op* op, int32_t nrhs,
                         const qrvie_c128* v, int64_t ldv, qrvie_c128* x, int64_t ldx,
                         const qrvie_solve_opts* opts, qrvie_solve_info* info);

/* ------------------------------------------------------------------ server */
/*
 * Continuous-batching solve server on one device.  Requests (an array, 1..64 plane waves
 * and a tolerance) may be submitted at any time from any thread.  A request is admitted
 * when one of `slots` workers is free and its device footprint (operator + solver, from
 * qrvie_op_footprint_estimate and qrvie_solve_footprint_estimate, computed before
 * anything else is allocated) fits `hbm_budget` next to the admitted requests and the
 * cached operators; requests are taken in arrival order, but one that does not fit yet
 * does not block later ones that do, until `max_bypass` of them have started ahead of
 * it.  Each worker has its own context and default-priority stream, so admitted
 * requests run concurrently on the device.  Operators are
 * compressed once per geometry (same centres, radii, heights, permittivities, lattice
 * sites and wavelength) and kept resident, at most `op_cache` of them, evicted least
 * recently used when their bytes are needed.  A request's result does not depend on what
 * else runs (the kernels are deterministic and share no mutable state).
 */
typedef struct qrvie_server qrvie_server;

typedef struct {
    int32_t  slots;          /* concurrent requests, 1..16 */
    size_t   hbm_budget;     /* bytes that admitted requests and cached operators may hold */
    double   eps;            /* compression tolerance of every operator (qrvie_compress_opts.eps) */
    int32_t  restart;        /* solve options of every request (qrvie_solve_opts) */
    int32_t  max_iter;
    int32_t  mode;           /* QRVIE_SOLVE_FP64 or QRVIE_SOLVE_BLOCK */
    int32_t  block_width;
    int32_t  op_cache;       /* operators kept resident after their request, >= 0 */
    uint64_t seed;           /* compression sketch seed */
    int32_t  tune_tiles;     /* 1: autotune the block product tiles of each new operator (block mode) */
    int32_t  max_bypass;     /* a queued request is overtaken by at most this many later
                                admissions, then nothing behind it starts before it (0: no limit) */
} qrvie_server_opts;

typedef struct {
    int64_t submitted, completed, failed, refused, running, queued;
    int64_t ops_built, cache_hits, evictions, rhs_solved;
    double  latency_p50_s, latency_p99_s;     /* arrival (submit) to completion, completed requests */
    double  queue_wait_p50_s;                  /* arrival to admission */
    double  makespan_s;                        /* first arrival to last completion */
    double  requests_per_s, rhs_solves_per_s;  /* completed over the makespan */
    size_t  peak_bytes, in_use_bytes;          /* admitted + cached footprint (estimates) */
} qrvie_server_stats;

/* Start the workers on HIP device `hip_device`.  Invalid options: QRVIE_ERR_INVALID_ARG. */
qrvie_status qrvie_server_create(int hip_device, const qrvie_server_opts* opts, qrvie_server** out);
/*
 * Submit a request; the array description and angle arrays are HOST data copied during the
 * call.  *ticket identifies it.  A request whose footprint exceeds hbm_budget is refused
 * (QRVIE_ERR_QUEUE_FULL, no ticket); invalid input gives the status of qrvie_geom_create or
 * QRVIE_ERR_INVALID_ARG.
 */
qrvie_status qrvie_server_submit(qrvie_server* srv, const qrvie_array_desc* array, int32_t nrhs,
                                 const double* theta_deg, const double* phi_deg, const int32_t* pol,
                                 double tol, uint64_t* ticket);
/* *done = 1 when the request has finished (successfully or not). */
qrvie_status qrvie_server_poll(qrvie_server* srv, uint64_t ticket, int32_t* done);
/* Block until the request finishes or timeout_s passes (< 0: no limit); *done as in poll.
 * QRVIE_ERR_INVALID_ARG for an unknown ticket, or one that another thread fetched meanwhile. */
qrvie_status qrvie_server_wait(qrvie_server* srv, uint64_t ticket, double timeout_s, int32_t* done);
/*
 * Copy a finished request's solution to the HOST buffer x (n x nrhs column-major, ldx >= n,
 * n = 144 x particles, caller order) and its per-RHS info (host array of nrhs, may be NULL),
 * then release the request.  Returns the request's own status (QRVIE_OK, QRVIE_NOT_CONVERGED
 * or the error that ended it); QRVIE_ERR_INVALID_ARG for an unknown, released or unfinished
 * ticket.
 */
qrvie_status qrvie_server_fetch(qrvie_server* srv, uint64_t ticket, qrvie_c128* x, int64_t ldx,
                                qrvie_solve_info* info);
/* Snapshot of the server's counters, latency percentiles (finished requests) and admitted
 * bytes into the caller's *out; QRVIE_ERR_INVALID_ARG for a null argument. */
qrvie_status qrvie_server_get_stats(qrvie_server* srv, qrvie_server_stats* out);
/* Arrival (submission), admission and completion times of a request not yet fetched, in
 * seconds on the server's steady clock (admitted/done are -1 until they happen). */
qrvie_status qrvie_server_request_times(qrvie_server* srv, uint64_t ticket, double* arrival_s,
                                        double* admitted_s, double* done_s);
/* Last error text of the server (submission or request failures). */
const char*  qrvie_server_last_error(qrvie_server* srv);
/* Finish the running requests, cancel the queued ones, free every operator and context.
 * No other call on the server may be in progress (a pending qrvie_server_wait included)
 * or follow: the handle is freed. */
void         qrvie_server_destroy(qrvie_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* QRVIE_H */
