// Blocks of right-hand sides: the compressed product Z_QR X and the preconditioner for
// up to 64 right-hand sides at once (§5.2 products, §4 preconditioner), on FP64 MFMA.
// Complex64 factor panels are widened to FP64 on load.
//
// With P right-hand sides every factor entry meets P complex multiply-adds, so the product
// turns from HBM-bound (one right-hand side) into a sequence of small dense GEMMs: each
// 64-row strip of a column-major panel (R panel, Q panel, self block or its inverse) is
// multiplied into an RHS-interleaved block (element (row e, rhs r) at e * P + r).  A
// workgroup takes one strip; each of its four waves owns 16 rows and all P columns, as
// P/16 tiles of v_mfma_f64_16x16x4f64.  A complex product is four real MFMAs:
// re += a.re b.re - a.im b.im, im += a.re b.im + a.im b.re.  The factor stream is read
// once per product; the interleaved input rows are shared by the strip's waves through
// the caches.  Accumulation is FP64 and the order is fixed, so results are reproducible.
#include "stream.h"

namespace qrvie {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

// Operand layout of the 16x16x4 FP64 MFMA on gfx950 (checked on the device):
//   A (16 x 4): lane l holds A[l % 16][l / 16];   B (4 x 16): lane l holds B[l / 16][l % 16];
//   D (16 x 16): lane l, slot i holds D[l / 16 + 4 i][l % 16].
__device__ __forceinline__ void cmfma(v4d& re, v4d& im, c128 a, c128 b) {
    re = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, re, 0, 0, 0);
    re = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, b.y, re, 0, 0, 0);
    im = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.y, im, 0, 0, 0);
    im = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.x, im, 0, 0, 0);
}

// Tile shape (chosen per strip group by the autotuner): U 4-column steps are loaded per batch
// (loads in flight against MFMAs), and each wave owns RT tiles of 16 rows, so a 64-row strip
// takes 4 / RT waves and every loaded right-hand-side tile feeds RT row tiles.  Every
// accumulator sees its columns in ascending order in every variant, so all shapes give
// bitwise-identical results.
template <int NT, int U, int RT, typename F>
__global__ void __launch_bounds__(256) k_strip_mfma(const MStrip* __restrict__ strips, const F* __restrict__ fac,
                                                    const c128* __restrict__ in, c128* __restrict__ out,
                                                    const int64_t* __restrict__ tmap) {
    constexpr int P = 16 * NT;
    const MStrip s = strips[blockIdx.x];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int r0 = 16 * RT * w;
    if (r0 >= s.nrows) return;
    const int rl = lane & 15, kq = lane >> 4;
    const bool trans = s.pad & kStripTrans;
    const int64_t rstep = trans ? s.ld : 1, cstep = trans ? 1 : s.ld;
    const F* A[RT];
#pragma unroll
    for (int q = 0; q < RT; ++q) A[q] = fac + s.a_off + min(r0 + 16 * q + rl, s.nrows - 1) * rstep;
    const c128* X = in + s.in_off * P + rl;
    v4d re[RT][NT], im[RT][NT];
#pragma unroll
    for (int q = 0; q < RT; ++q)
#pragma unroll
        for (int t = 0; t < NT; ++t) re[q][t] = im[q][t] = v4d{0.0, 0.0, 0.0, 0.0};
    const int nsteps = s.ncols / 4;
    int c = 0;
    for (; c + U <= nsteps; c += U) {
        c128 a[U][RT], b[U][NT];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t col = 4 * (c + u) + kq;
#pragma unroll
            for (int q = 0; q < RT; ++q) a[u][q] = widen(load_stream(A[q] + col * cstep));
#pragma unroll
            for (int t = 0; t < NT; ++t) b[u][t] = X[col * P + 16 * t];
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int q = 0; q < RT; ++q)
#pragma unroll
                for (int t = 0; t < NT; ++t) cmfma(re[q][t], im[q][t], a[u][q], b[u][t]);
    }
    for (; 4 * c < s.ncols; ++c) {                      // remaining steps, the last possibly partial
        const int64_t col = 4 * c + kq;
        const bool ok = col < s.ncols;
        const c128 z = make_double2(0.0, 0.0);
        c128 b[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) b[t] = ok ? X[col * P + 16 * t] : z;
#pragma unroll
        for (int q = 0; q < RT; ++q) {
            const c128 a = ok ? widen(A[q][col * cstep]) : z;
#pragma unroll
            for (int t = 0; t < NT; ++t) cmfma(re[q][t], im[q][t], a, b[t]);
        }
    }
#pragma unroll
    for (int q = 0; q < RT; ++q)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = r0 + 16 * q + kq + 4 * i;
            if (row >= s.nrows) continue;
            const int64_t orow = s.tmap_off >= 0 ? tmap[s.tmap_off + row] : s.out_off + row;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                c128* o = out + orow * P + 16 * t + rl;
                c128 v = make_double2(re[q][t][i], im[q][t][i]);
                if (s.pad & kStripAcc) v = make_double2(v.x + o->x, v.y + o->y);
                *o = v;
            }
        }
}

// The same strip products on FP32 matrix cores (v_mfma_f32_16x16x4f32: the A and B operand
// layouts of the FP64 instruction, but lane l, slot i of D holds row 4 (l / 16) + i, as
// measured on the device) with FP32 accumulation: factors from complex64 panels (KIND 0) or
// from BF16 split-complex planes (KIND 1: real parts, then the imaginary parts `plane` entries
// later), the right-hand sides rounded to FP32 on load.  One tile shape (4-column steps in
// batches of 4, one 16-row tile per wave); results are stored in FP64.
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void cmfma32(v4f& re, v4f& im, float2 a, float2 b) {
    re = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, re, 0, 0, 0);
    re = __builtin_amdgcn_mfma_f32_16x16x4f32(-a.y, b.y, re, 0, 0, 0);
    im = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.y, im, 0, 0, 0);
    im = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.x, im, 0, 0, 0);
}

__device__ __forceinline__ float bf16_to_f32(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

template <int KIND>
__device__ __forceinline__ float2 load_fac32(const void* fac, int64_t plane, int64_t i) {
    if (KIND == 0) return load_stream(static_cast<const float2*>(fac) + i);
    const unsigned short* p = static_cast<const unsigned short*>(fac);
    return make_float2(bf16_to_f32(__builtin_nontemporal_load(p + i)), bf16_to_f32(__builtin_nontemporal_load(p + plane + i)));
}

__device__ __forceinline__ float2 narrow(c128 v) { return make_float2((float)v.x, (float)v.y); }

template <int NT, int KIND>
__global__ void __launch_bounds__(256) k_strip_mfma32(const MStrip* __restrict__ strips, const void* __restrict__ fac,
                                                      int64_t plane, const c128* __restrict__ in,
                                                      c128* __restrict__ out, const int64_t* __restrict__ tmap) {
    constexpr int P = 16 * NT, U = 4;
    const MStrip s = strips[blockIdx.x];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int r0 = 16 * w;
    if (r0 >= s.nrows) return;
    const int rl = lane & 15, kq = lane >> 4;
    const bool trans = s.pad & kStripTrans;
    const int64_t rstep = trans ? s.ld : 1, cstep = trans ? 1 : s.ld;
    const int64_t abase = s.a_off + min(r0 + rl, s.nrows - 1) * rstep;
    const c128* X = in + s.in_off * P + rl;
    v4f re[NT], im[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) re[t] = im[t] = v4f{0.f, 0.f, 0.f, 0.f};
    const int nsteps = s.ncols / 4;
    int c = 0;
    for (; c + U <= nsteps; c += U) {
        float2 a[U], b[U][NT];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t col = 4 * (c + u) + kq;
            a[u] = load_fac32<KIND>(fac, plane, abase + col * cstep);
#pragma unroll
            for (int t = 0; t < NT; ++t) b[u][t] = narrow(X[col * P + 16 * t]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int t = 0; t < NT; ++t) cmfma32(re[t], im[t], a[u], b[u][t]);
    }
    for (; 4 * c < s.ncols; ++c) {                      // remaining steps, the last possibly partial
        const int64_t col = 4 * c + kq;
        const bool ok = col < s.ncols;
        const float2 z = make_float2(0.f, 0.f);
        const float2 a = ok ? load_fac32<KIND>(fac, plane, abase + col * cstep) : z;
#pragma unroll
        for (int t = 0; t < NT; ++t) cmfma32(re[t], im[t], a, ok ? narrow(X[col * P + 16 * t]) : z);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int row = r0 + 4 * kq + i;
        if (row >= s.nrows) continue;
        const int64_t orow = s.tmap_off >= 0 ? tmap[s.tmap_off + row] : s.out_off + row;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            c128* o = out + orow * P + 16 * t + rl;
            c128 v = make_double2((double)re[t][i], (double)im[t][i]);
            if (s.pad & kStripAcc) v = make_double2(v.x + o->x, v.y + o->y);
            *o = v;
        }
    }
}

// number of positions where two arrays of doubles differ bitwise (accumulated into *count)
__global__ void __launch_bounds__(256) k_count_neq(int64_t n, const unsigned long long* __restrict__ a,
                                                   const unsigned long long* __restrict__ b,
                                                   unsigned long long* count) {
    __shared__ int red[4];
    int c = 0;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) c += a[e] != b[e];
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int t = red[0] + red[1] + red[2] + red[3];
        if (t) atomicAdd(count, (unsigned long long)t);
    }
}

// ----------------------------------------------------------------- basis updates on FP64 MFMA
// W (n x q) = beta W + sign * V H for V: n x m, H: m x q (q <= 64): the basis update of
// block CGS2, the solution update (long, thin products that rocBLAS runs at about half the
// FP64 matrix rate) and the Gram correction 2 H1 - G H1 (square, small: rocBLAS picked a
// tile shape that ran it at a few TF/s).  Each wave owns 16 rows of W and all q columns (NT tiles of 16); the m
// columns of V are visited in ascending batches of U 4-column steps (fixed order).  V is
// streamed once; H stays in cache.
template <int NT>
__global__ void __launch_bounds__(256) k_gemm_nn_acc(int64_t n, int m, int q, const c128* __restrict__ V,
                                                     int64_t ldv, const c128* __restrict__ H, int64_t ldh,
                                                     double beta, double sign, c128* __restrict__ W,
                                                     int64_t ldw) {
    constexpr int U = 4;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int64_t r0 = 64 * (int64_t)blockIdx.x + 16 * w;
    if (r0 >= n) return;
    const int rl = lane & 15, kq = lane >> 4;
    const c128* Vp = V + min(r0 + rl, n - 1);                        // clamped lanes are discarded
    const c128* Hp[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) Hp[t] = H + (int64_t)min(16 * t + rl, q - 1) * ldh;
    v4d re[NT], im[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) re[t] = im[t] = v4d{0.0, 0.0, 0.0, 0.0};
    int i = 0;
    for (; i + 4 * U <= m; i += 4 * U) {
        c128 a[U], b[U][NT];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int col = i + 4 * u + kq;
            a[u] = load_stream(Vp + (int64_t)col * ldv);
#pragma unroll
            for (int t = 0; t < NT; ++t) b[u][t] = Hp[t][col];
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int t = 0; t < NT; ++t) cmfma(re[t], im[t], a[u], b[u][t]);
    }
    for (; i < m; i += 4) {                                           // remaining steps, the last possibly partial
        const int col = i + kq;
        const bool ok = col < m;
        const c128 z = make_double2(0.0, 0.0);
        const c128 a = ok ? Vp[(int64_t)col * ldv] : z;
#pragma unroll
        for (int t = 0; t < NT; ++t) cmfma(re[t], im[t], a, ok ? Hp[t][col] : z);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int64_t row = r0 + kq + 4 * s;
        if (row >= n) continue;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int j = 16 * t + rl;
            if (j < q) {
                c128* o = W + row + (int64_t)j * ldw;
                const c128 v = beta != 0.0 ? *o : make_double2(0.0, 0.0);     // beta = 0: W may be uninitialised
                *o = make_double2(beta * v.x + sign * re[t][s], beta * v.y + sign * im[t][s]);
            }
        }
    }
}

// out = (V ? V - y : y), y = yself + sum_l ylev[l]; all n x P interleaved
template <int NT>
__global__ void k_block_combine(int64_t n, const c128* __restrict__ ylev, int nlev, const c128* __restrict__ yself,
                                const c128* __restrict__ V, c128* __restrict__ out) {
    constexpr int P = 16 * NT;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * P) return;
    c128 y = yself[e];
    for (int l = 0; l < nlev; ++l) {
        const c128 a = ylev[(int64_t)l * n * P + e];
        y = make_double2(y.x + a.x, y.y + a.y);
    }
    if (V) y = make_double2(V[e].x - y.x, V[e].y - y.y);
    out[e] = y;
}

// blk[(p*144 + d) * P + r] = src[r * ld + c * 144 + d], c = i2c ? i2c[p] : p (zero for r >= ncols)
template <int NT>
__global__ void k_gather_block(int32_t N, const int32_t* __restrict__ i2c, const c128* __restrict__ src, int64_t ld,
                               int ncols, c128* __restrict__ blk) {
    constexpr int P = 16 * NT;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // internal DoF
    if (e >= (int64_t)N * kNp) return;
    const int64_t p = e / kNp, d = e % kNp;
    const int64_t ce = (i2c ? (int64_t)i2c[p] : p) * kNp + d;
#pragma unroll 4
    for (int r = 0; r < P; ++r) blk[e * P + r] = r < ncols ? src[r * ld + ce] : make_double2(0.0, 0.0);
}

template <int NT>
__global__ void k_scatter_block(int32_t N, const int32_t* __restrict__ i2c, const c128* __restrict__ blk,
                                c128* __restrict__ dst, int64_t ld, int ncols) {
    constexpr int P = 16 * NT;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)N * kNp) return;
    const int64_t p = e / kNp, d = e % kNp;
    const int64_t ce = (i2c ? (int64_t)i2c[p] : p) * kNp + d;
    for (int r = 0; r < ncols; ++r) dst[r * ld + ce] = blk[e * P + r];
}

// ---------------------------------------------------------------- block Arnoldi helpers
// Gram matrix of the block basis: G[0:(k+1)p, kp:(k+1)p] = C (the new block column, from
// V^H V_k) and the mirrored block row G[kp:(k+1)p, 0:kp] = C[0:kp, :]^H.
__global__ void k_gram_store(int k, int p, const c128* __restrict__ C, int64_t ldc, c128* __restrict__ G,
                             int64_t ldg) {
    const int64_t rows = (int64_t)(k + 1) * p;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rows * p) return;
    const int64_t i = e % rows, j = e / rows;
    const c128 v = C[i + j * ldc];
    G[i + ((int64_t)k * p + j) * ldg] = v;
    if (i < (int64_t)k * p) G[(int64_t)k * p + j + i * ldg] = make_double2(v.x, -v.y);
}

// Cholesky S = R^H R of a Hermitian p x p matrix (p <= 64, column-major, upper triangle
// used), one workgroup.  R (upper, zeros below) is written to out; flag[0] = 1 when a pivot
// falls below rel * (largest diagonal entry of S), i.e. the block is numerically rank
// deficient, and the factor is then not usable.
__global__ void __launch_bounds__(256) k_cholesky(int p, const c128* __restrict__ S, int64_t lds, double rel,
                                                  c128* __restrict__ out, int64_t ldo, int* flag) {
    __shared__ c128 A[64][65];
    __shared__ double dmax;
    const int tid = threadIdx.x;
    for (int e = tid; e < p * p; e += blockDim.x) {
        const int i = e % p, j = e / p;
        A[i][j] = i <= j ? S[i + j * lds] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    if (tid == 0) {
        double m = 0.0;
        for (int j = 0; j < p; ++j) m = fmax(m, A[j][j].x);
        dmax = m;
        flag[0] = 0;
    }
    __syncthreads();
    for (int j = 0; j < p; ++j) {
        const double d = A[j][j].x;
        const bool bad = !(d > rel * dmax);
        const double r = bad ? 1.0 : sqrt(d);
        __syncthreads();
        if (tid == 0) {
            if (bad) flag[0] = 1;
            A[j][j] = make_double2(r, 0.0);
        }
        for (int c = j + 1 + tid; c < p; c += blockDim.x) A[j][c] = make_double2(A[j][c].x / r, A[j][c].y / r);
        __syncthreads();
        // trailing update: A[i][c] -= conj(R[j][i]) R[j][c], j < i <= c
        for (int e = tid; e < p * p; e += blockDim.x) {
            const int i = e % p, c = e / p;
            if (i > j && i <= c) {
                const c128 a = A[j][i], b = A[j][c];
                A[i][c] = make_double2(A[i][c].x - (a.x * b.x + a.y * b.y), A[i][c].y - (a.x * b.y - a.y * b.x));
            }
        }
        __syncthreads();
    }
    for (int e = tid; e < p * p; e += blockDim.x) {
        const int i = e % p, j = e / p;
        out[i + j * ldo] = i <= j ? A[i][j] : make_double2(0.0, 0.0);
    }
}

// Rank-revealing Cholesky with diagonal pivoting of a Hermitian p x p Gram matrix S (p <= 64,
// upper triangle used): S[perm, perm] = R^H R with R upper trapezoidal of rank q, stopping
// at the first pivot below rel * (largest diagonal entry).  out (ld ldo) receives R in its
// first q rows and zeros below; perm[0:p] the pivot order; qout[0] = q.
__global__ void __launch_bounds__(256) k_cholesky_piv(int p, const c128* __restrict__ S, int64_t lds, double rel,
                                                      c128* __restrict__ out, int64_t ldo, int* perm, int* qout) {
    __shared__ c128 A[64][65];
    __shared__ int pv[64];
    __shared__ double dmax;
    __shared__ int sel, q;
    const int tid = threadIdx.x;
    for (int e = tid; e < p * p; e += blockDim.x) {
        const int i = e % p, j = e / p;
        const c128 v = i <= j ? S[i + j * lds] : S[j + i * lds];
        A[i][j] = i <= j ? v : make_double2(v.x, -v.y);
    }
    if (tid < p) pv[tid] = tid;
    __syncthreads();
    if (tid == 0) {
        double m = 0.0;
        for (int j = 0; j < p; ++j) m = fmax(m, A[j][j].x);
        dmax = m;
        q = p;
    }
    __syncthreads();
    for (int j = 0; j < p; ++j) {
        if (tid == 0) {
            int m = j;
            for (int i = j + 1; i < p; ++i)
                if (A[i][i].x > A[m][m].x) m = i;
            sel = m;
            if (!(A[m][m].x > rel * dmax)) q = j;
        }
        __syncthreads();
        if (q <= j) break;                       // uniform: q is shared
        const int m = sel;
        if (m != j) {                            // symmetric swap of rows/columns j and m
            for (int c = tid; c < p; c += blockDim.x) {
                const c128 t = A[j][c]; A[j][c] = A[m][c]; A[m][c] = t;
            }
            __syncthreads();
            for (int r = tid; r < p; r += blockDim.x) {
                const c128 t = A[r][j]; A[r][j] = A[r][m]; A[r][m] = t;
            }
            if (tid == 0) { const int t = pv[j]; pv[j] = pv[m]; pv[m] = t; }
            __syncthreads();
        }
        const double r = sqrt(A[j][j].x);
        __syncthreads();
        if (tid == 0) A[j][j] = make_double2(r, 0.0);
        for (int c = j + 1 + tid; c < p; c += blockDim.x) A[j][c] = make_double2(A[j][c].x / r, A[j][c].y / r);
        __syncthreads();
        for (int e = tid; e < p * p; e += blockDim.x) {          // A[i][c] -= conj(R[j][i]) R[j][c], i, c > j
            const int i = e % p, c = e / p;
            if (i > j && c > j) {
                const c128 a = A[j][i], b = A[j][c];
                A[i][c] = make_double2(A[i][c].x - (a.x * b.x + a.y * b.y), A[i][c].y - (a.x * b.y - a.y * b.x));
            }
        }
        __syncthreads();
    }
    __syncthreads();
    const int qq = q;
    for (int e = tid; e < p * p; e += blockDim.x) {
        const int i = e % p, j = e / p;
        out[i + j * ldo] = (i < qq && i <= j) ? A[i][j] : make_double2(0.0, 0.0);
    }
    if (tid < p) perm[tid] = pv[tid];
    if (tid == 0) qout[0] = qq;
}

// out[0:q, perm[c]] = (A B)[0:q, c] for upper-triangular q x q A and upper-trapezoidal
// q x p B (column-major): the deflated block's S0 in the original column order.
__global__ void k_trmm_perm(int q, int p, const c128* __restrict__ A, int64_t lda, const c128* __restrict__ B,
                            int64_t ldb, const int* __restrict__ perm, c128* __restrict__ out, int64_t ldo) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= q * p) return;
    const int i = e % q, j = e / q;
    double re = 0.0, im = 0.0;
    for (int l = i; l < q && l <= j; ++l) {
        const c128 a = A[i + (int64_t)l * lda], b = B[l + (int64_t)j * ldb];
        re += a.x * b.x - a.y * b.y;
        im += a.x * b.y + a.y * b.x;
    }
    out[i + (int64_t)perm[j] * ldo] = make_double2(re, im);
}

// C = A B for upper-triangular p x p A, B (column-major); C may not alias A or B.  C = 0
// when either Cholesky flag is set (a rank-deficient block contributes nothing).
__global__ void k_trmm_upper(int p, const c128* __restrict__ A, int64_t lda, const c128* __restrict__ B,
                             int64_t ldb, c128* __restrict__ C, int64_t ldc, const int* __restrict__ flag) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= p * p) return;
    const int i = e % p, j = e / p;
    if (flag && (flag[0] || flag[1])) {
        C[i + (int64_t)j * ldc] = make_double2(0.0, 0.0);
        return;
    }
    double re = 0.0, im = 0.0;
    for (int l = i; l <= j; ++l) {
        const c128 a = A[i + (int64_t)l * lda], b = B[l + (int64_t)j * ldb];
        re += a.x * b.x - a.y * b.y;
        im += a.x * b.y + a.y * b.x;
    }
    C[i + (int64_t)j * ldc] = make_double2(re, im);
}

// Least squares of block GMRES.  The block Hessenberg matrix is reduced to upper triangular
// form by one compact-WY block reflector per block column: Q_j = I - Y_j T_j Y_j^H acting on
// rows [jp, jp + 2p) (Y_j: 2p x p, unit lower trapezoidal; T_j: p x p upper triangular).
//
// Apply Q_j^H for j in [j0, j1), in order, to every column of C (rows indexed from 0, ld
// ldc): one workgroup per column, the 2p-row segment staged in LDS.
__global__ void __launch_bounds__(256) k_ls_apply(int j0, int j1, int p, const c128* __restrict__ Y,
                                                  const c128* __restrict__ T, c128* __restrict__ C, int64_t ldc) {
    __shared__ c128 seg[128];
    __shared__ c128 w[64], w2[64];
    __shared__ c128 part[256];
    const int tid = threadIdx.x;
    c128* col = C + (int64_t)blockIdx.x * ldc;
    const int m = 2 * p;
    for (int j = j0; j < j1; ++j) {
        const c128* Yj = Y + (int64_t)j * m * p;
        const c128* Tj = T + (int64_t)j * p * p;
        c128* sg = col + (int64_t)j * p;
        for (int e = tid; e < m; e += blockDim.x) seg[e] = sg[e];
        __syncthreads();
        // w = Y_j^H seg: 4 threads per entry
        {
            const int i = tid >> 2, q = tid & 3;
            double re = 0.0, im = 0.0;
            if (i < p)
                for (int e = q; e < m; e += 4) {
                    const c128 y = Yj[e + (int64_t)i * m], x = seg[e];
                    re += y.x * x.x + y.y * x.y;
                    im += y.x * x.y - y.y * x.x;
                }
            part[tid] = make_double2(re, im);
        }
        __syncthreads();
        if (tid < p) {
            const c128 a = part[4 * tid], b = part[4 * tid + 1], c = part[4 * tid + 2], d = part[4 * tid + 3];
            w[tid] = make_double2((a.x + b.x) + (c.x + d.x), (a.y + b.y) + (c.y + d.y));
        }
        __syncthreads();
        // w2 = T_j^H w: w2[i] = sum_{l <= i} conj(T[l][i]) w[l]
        if (tid < p) {
            double re = 0.0, im = 0.0;
            for (int l = 0; l <= tid; ++l) {
                const c128 t = Tj[l + (int64_t)tid * p], x = w[l];
                re += t.x * x.x + t.y * x.y;
                im += t.x * x.y - t.y * x.x;
            }
            w2[tid] = make_double2(re, im);
        }
        __syncthreads();
        // seg -= Y_j w2: 2 threads per row
        {
            const int e = tid >> 1, q = tid & 1;
            double re = 0.0, im = 0.0;
            if (e < m)
                for (int i = q; i < p; i += 2) {
                    const c128 y = Yj[e + (int64_t)i * m], x = w2[i];
                    re += y.x * x.x - y.y * x.y;
                    im += y.x * x.y + y.y * x.x;
                }
            part[tid] = make_double2(re, im);
        }
        __syncthreads();
        for (int e = tid; e < m; e += blockDim.x) {
            const c128 a = part[2 * e], b = part[2 * e + 1];
            sg[e] = make_double2(seg[e].x - (a.x + b.x), seg[e].y - (a.y + b.y));
        }
        __syncthreads();
    }
}

// Householder QR of the 2p x p block M = C[kp : kp + 2p, 0 : p] (ld ldc), one workgroup:
// M becomes [R_kk; 0], Y_k and T_k are written for k_ls_apply.  Reflector i maps
// (alpha, x) to (beta, 0) with real beta = -sign(Re alpha) ||(alpha, x)||,
// tau = (beta - alpha) / beta, v = (1, x / (alpha - beta)); H_i = I - tau v v^H and the
// block is reduced by H_i^H.  T follows the forward column-wise recurrence
// T[0:i, i] = -tau_i T[0:i, 0:i] (Y[:, 0:i]^H v_i), T[i][i] = tau_i.
__global__ void __launch_bounds__(256) k_ls_factor(int k, int p, c128* __restrict__ C, int64_t ldc,
                                                   c128* __restrict__ Yk, c128* __restrict__ Tk) {
    __shared__ c128 M[128][64];
    __shared__ c128 tau_s[64];
    __shared__ c128 part[256];
    __shared__ c128 z[64];
    __shared__ double red[256];
    __shared__ c128 beta_s, scale_s;
    const int tid = threadIdx.x;
    const int m = 2 * p;
    c128* base = C + (int64_t)k * p;
    for (int e = tid; e < m * p; e += blockDim.x) {
        const int r = e % m, c = e / m;
        M[r][c] = base[r + (int64_t)c * ldc];
    }
    __syncthreads();
    for (int i = 0; i < p; ++i) {
        // norm of x = M[i+1:m, i]
        double s = 0.0;
        for (int r = i + 1 + tid; r < m; r += blockDim.x) s += M[r][i].x * M[r][i].x + M[r][i].y * M[r][i].y;
        red[tid] = s;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (tid < o) red[tid] += red[tid + o];
            __syncthreads();
        }
        if (tid == 0) {
            const c128 alpha = M[i][i];
            const double xn2 = red[0];
            if (xn2 == 0.0 && alpha.y == 0.0) {
                tau_s[i] = make_double2(0.0, 0.0);
                beta_s = alpha;
                scale_s = make_double2(0.0, 0.0);
            } else {
                const double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + xn2);
                const double beta = alpha.x >= 0.0 ? -nrm : nrm;
                tau_s[i] = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
                const double dr = alpha.x - beta, di = alpha.y, den = dr * dr + di * di;
                scale_s = make_double2(dr / den, -di / den);                 // 1 / (alpha - beta)
                beta_s = make_double2(beta, 0.0);
            }
        }
        __syncthreads();
        for (int r = i + 1 + tid; r < m; r += blockDim.x) {
            const c128 x = M[r][i], sc = scale_s;
            M[r][i] = make_double2(x.x * sc.x - x.y * sc.y, x.x * sc.y + x.y * sc.x);
        }
        if (tid == 0) M[i][i] = beta_s;
        __syncthreads();
        // apply H_i^H = I - conj(tau) v v^H to columns c > i; v = (1, M[i+1:m, i])
        {
            const int c = i + 1 + (tid >> 2), q = tid & 3;
            double re = 0.0, im = 0.0;
            if (c < p)
                for (int r = i + q; r < m; r += 4) {
                    const c128 v = r == i ? make_double2(1.0, 0.0) : M[r][i], x = M[r][c];
                    re += v.x * x.x + v.y * x.y;
                    im += v.x * x.y - v.y * x.x;
                }
            part[tid] = make_double2(re, im);
        }
        __syncthreads();
        {
            const int c = i + 1 + (tid >> 2), q = tid & 3;
            const c128 ta = tau_s[i];
            if (c < p) {
                const c128 a = part[tid & ~3], b = part[(tid & ~3) + 1], cc = part[(tid & ~3) + 2],
                           d = part[(tid & ~3) + 3];
                const c128 sv = make_double2((a.x + b.x) + (cc.x + d.x), (a.y + b.y) + (cc.y + d.y));
                // f = conj(tau) * sv
                const c128 f = make_double2(ta.x * sv.x + ta.y * sv.y, ta.x * sv.y - ta.y * sv.x);
                for (int r = i + q; r < m; r += 4) {
                    const c128 v = r == i ? make_double2(1.0, 0.0) : M[r][i];
                    M[r][c] = make_double2(M[r][c].x - (v.x * f.x - v.y * f.y), M[r][c].y - (v.x * f.y + v.y * f.x));
                }
            }
        }
        __syncthreads();
    }
    // Y_k (unit lower trapezoidal) and R_kk back into C (zeros below the diagonal)
    for (int e = tid; e < m * p; e += blockDim.x) {
        const int r = e % m, c = e / m;
        Yk[r + (int64_t)c * m] = r < c ? make_double2(0.0, 0.0) : (r == c ? make_double2(1.0, 0.0) : M[r][c]);
        base[r + (int64_t)c * ldc] = r <= c ? M[r][c] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    // T_k, column by column
    for (int i = 0; i < p; ++i) {
        // z[l] = Y[:, l]^H v_i for l < i (v_i = Y[:, i], zero above row i)
        {
            const int l = tid >> 2, q = tid & 3;
            double re = 0.0, im = 0.0;
            if (l < i)
                for (int r = i + q; r < m; r += 4) {
                    const c128 a = r == l ? make_double2(1.0, 0.0) : M[r][l];
                    const c128 v = r == i ? make_double2(1.0, 0.0) : M[r][i];
                    re += a.x * v.x + a.y * v.y;
                    im += a.x * v.y - a.y * v.x;
                }
            part[tid] = make_double2(re, im);
        }
        __syncthreads();
        if (tid < i) {
            const c128 a = part[4 * tid], b = part[4 * tid + 1], cc = part[4 * tid + 2], d = part[4 * tid + 3];
            z[tid] = make_double2((a.x + b.x) + (cc.x + d.x), (a.y + b.y) + (cc.y + d.y));
        }
        __syncthreads();
        // T[0:i, i] = -tau_i T[0:i, 0:i] z
        if (tid < p) {
            c128 out = make_double2(0.0, 0.0);
            if (tid < i) {
                double re = 0.0, im = 0.0;
                for (int l = tid; l < i; ++l) {
                    const c128 t = Tk[tid + (int64_t)l * p], x = z[l];
                    re += t.x * x.x - t.y * x.y;
                    im += t.x * x.y + t.y * x.x;
                }
                const c128 ta = tau_s[i];
                out = make_double2(-(ta.x * re - ta.y * im), -(ta.x * im + ta.y * re));
            } else if (tid == i) {
                out = tau_s[i];
            }
            Tk[tid + (int64_t)i * p] = out;
        }
        __syncthreads();
    }
}

// ----------------------------------------------------------------- basis projections
// Split-K partial products of C = A^H B (A: n x m, B: n x c, both column-major): chunk z of
// the rows writes P[z m c + i + j m] = sum over its rows e of conj(A[e, i]) B[e, j].  The
// outputs are small against a reduction over 10^5-10^6 rows, so the rows are split into
// chunks and a fixed-order kernel sums the partials (deterministic).  A workgroup owns a
// tile of C for one chunk (below).  The chunk's rows are consumed 16 at a time: the slices of
// A and B are staged in LDS.
// conj(a) b: re += a.re b.re + a.im b.im, im += a.re b.im - a.im b.re.
__device__ __forceinline__ void cmfma_conj(v4d& re, v4d& im, c128 a, c128 b) {
    re = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, re, 0, 0, 0);
    re = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.y, re, 0, 0, 0);
    im = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.y, im, 0, 0, 0);
    im = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, b.x, im, 0, 0, 0);
}

constexpr int kHnRows = 16;                 // rows per staged slice
constexpr int kHnPad = kHnRows + 1;         // LDS row pitch of a staged column (bank spread)
constexpr int kHnTM = 128, kHnTC = 64;      // workgroup tile of C

// A workgroup owns a 128 x 64 tile of C for one row chunk; wave w a 64 x 32 block of it (4 x 2
// FP64 MFMA tiles, so every staged A element feeds 2 and every B element 4 tiles).  The next
// 16-row slice is loaded into registers while the MFMAs run on the staged one.
__global__ void __launch_bounds__(256, 2) k_gemm_hn_part(int64_t n, int m, int c, const c128* __restrict__ A, int64_t lda,
                                                      const c128* __restrict__ B, int64_t ldb, int64_t L,
                                                      c128* __restrict__ P) {
    __shared__ c128 As[kHnTM * kHnPad];
    __shared__ c128 Bs[kHnTC * kHnPad];
    const int t = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6), lane = t & 63;
    const int rl = lane & 15, kq = lane >> 4;
    const int i0 = blockIdx.x * kHnTM, j0 = blockIdx.y * kHnTC;
    const int64_t e0 = (int64_t)blockIdx.z * L, e1 = min(n, e0 + L);
    const int qi = (w & 1) * 64, qj = (w >> 1) * 32;
    // staging: thread t moves row t % 16 of columns t / 16 + 16 p of both slices
    const int sr = t & 15, sc = t >> 4;
    c128 ra[kHnTM / 16], rb[kHnTC / 16];
    auto load = [&](int64_t e) {
        const int64_t row = e + sr;
        const bool rok = row < e1;
#pragma unroll
        for (int p = 0; p < kHnTM / 16; ++p) {
            const int ci = i0 + sc + 16 * p;
            ra[p] = rok && ci < m ? A[row + (int64_t)ci * lda] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int p = 0; p < kHnTC / 16; ++p) {
            const int cj = j0 + sc + 16 * p;
            rb[p] = rok && cj < c ? B[row + (int64_t)cj * ldb] : make_double2(0.0, 0.0);
        }
    };
    v4d re[4][2], im[4][2];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) re[a][b] = im[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
    if (e0 < e1) load(e0);
    for (int64_t e = e0; e < e1; e += kHnRows) {
        __syncthreads();
#pragma unroll
        for (int p = 0; p < kHnTM / 16; ++p) As[(sc + 16 * p) * kHnPad + sr] = ra[p];
#pragma unroll
        for (int p = 0; p < kHnTC / 16; ++p) Bs[(sc + 16 * p) * kHnPad + sr] = rb[p];
        __syncthreads();
        if (e + kHnRows < e1) load(e + kHnRows);
#pragma unroll
        for (int ks = 0; ks < kHnRows / 4; ++ks) {
            c128 a[4], b[2];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) a[mt] = As[(qi + 16 * mt + rl) * kHnPad + 4 * ks + kq];
#pragma unroll
            for (int ct = 0; ct < 2; ++ct) b[ct] = Bs[(qj + 16 * ct + rl) * kHnPad + 4 * ks + kq];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int ct = 0; ct < 2; ++ct) cmfma_conj(re[mt][ct], im[mt][ct], a[mt], b[ct]);
        }
    }
    const int64_t per = (int64_t)m * c;
    c128* out = P + (int64_t)blockIdx.z * per;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int i = i0 + qi + 16 * mt + kq + 4 * s, j = j0 + qj + 16 * ct + rl;
                if (i < m && j < c) out[i + (int64_t)j * m] = make_double2(re[mt][ct][s], im[mt][ct][s]);
            }
}

// Inverse of an upper triangular k x k matrix U (k <= 256): thread j solves U x = e_j by back
// substitution into column j of out (zero below the diagonal).  A zero pivot gives inf / NaN,
// as a triangular solve would; callers check their Cholesky flags.
__global__ void __launch_bounds__(256) k_tri_inv_upper(int k, const c128* __restrict__ U, int64_t ldu,
                                                       c128* __restrict__ out, int64_t ldo) {
    const int j = threadIdx.x;
    if (j >= k) return;
    c128* x = out + (int64_t)j * ldo;
    for (int i = k - 1; i > j; --i) x[i] = make_double2(0.0, 0.0);
    for (int i = j; i >= 0; --i) {
        double re = i == j ? 1.0 : 0.0, im = 0.0;
        for (int l = i + 1; l <= j; ++l) {
            const c128 u = U[i + (int64_t)l * ldu], v = x[l];
            re -= u.x * v.x - u.y * v.y;
            im -= u.x * v.y + u.y * v.x;
        }
        const c128 d = U[i + (int64_t)i * ldu];
        const double den = d.x * d.x + d.y * d.y;
        x[i] = make_double2((re * d.x + im * d.y) / den, (im * d.x - re * d.y) / den);
    }
}

// Y (m x p, ld ldy) = U^-1 Y for an upper triangular m x m U (ld ldu): one workgroup per column
// of Y.  Back substitution by columns of U (contiguous): y_k = y_k / u_kk, then y_i -= u_ik y_k
// for i < k.  Thread t owns the rows i = t (mod 1024), so only the owner of row k touches it;
// y_k reaches the others through LDS.
__global__ void __launch_bounds__(1024) k_trsm_upper_left(int m, const c128* __restrict__ U, int64_t ldu,
                                                          c128* __restrict__ Y, int64_t ldy) {
    __shared__ c128 yk;
    c128* y = Y + (int64_t)blockIdx.x * ldy;
    const int t = threadIdx.x;
    for (int k = m - 1; k >= 0; --k) {
        if ((k & 1023) == t) {
            const c128 d = U[k + (int64_t)k * ldu], v = y[k];
            const double den = d.x * d.x + d.y * d.y;
            const c128 r = make_double2((v.x * d.x + v.y * d.y) / den, (v.y * d.x - v.x * d.y) / den);
            y[k] = r;
            yk = r;
        }
        __syncthreads();
        const c128 b = yk;
        const c128* u = U + (int64_t)k * ldu;
        for (int i = t; i < k; i += 1024) {
            const c128 a = u[i];
            c128 v = y[i];
            v.x -= a.x * b.x - a.y * b.y;
            v.y -= a.x * b.y + a.y * b.x;
            y[i] = v;
        }
        __syncthreads();
    }
}

// C[i + j ldc] = sum_b P[b per + i + j m] for i < m, j < c, b < nb (fixed order): the
// reduction of split-K partial products.
__global__ void k_sum_batches(int m, int c, int nb, const c128* __restrict__ P, c128* __restrict__ C, int64_t ldc) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = (int64_t)m * c;
    if (e >= per) return;
    const int64_t i = e % m, j = e / m;
    double re = 0.0, im = 0.0;
    for (int b = 0; b < nb; ++b) {
        const c128 v = P[(int64_t)b * per + e];
        re += v.x;
        im += v.y;
    }
    C[i + j * ldc] = make_double2(re, im);
}

// out[c] = ||C[0:rows, c]|| for c < ncols
__global__ void __launch_bounds__(256) k_col_norms(int rows, const c128* __restrict__ C, int64_t ldc, double* out) {
    __shared__ double red[256];
    const c128* col = C + (int64_t)blockIdx.x * ldc;
    double s = 0.0;
    for (int r = threadIdx.x; r < rows; r += blockDim.x) s += col[r].x * col[r].x + col[r].y * col[r].y;
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = sqrt(red[0]);
}

}  // namespace

void launch_gram_store(hipStream_t s, int k, int p, const c128* C, int64_t ldc, c128* G, int64_t ldg) {
    const int64_t tot = (int64_t)(k + 1) * p * p;
    hipLaunchKernelGGL(k_gram_store, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, k, p, C, ldc, G, ldg);
}
void launch_cholesky(hipStream_t s, int p, const c128* S, int64_t lds, double rel, c128* out, int64_t ldo, int* flag) {
    hipLaunchKernelGGL(k_cholesky, dim3(1), dim3(256), 0, s, p, S, lds, rel, out, ldo, flag);
}
void launch_trmm_upper(hipStream_t s, int p, const c128* A, int64_t lda, const c128* B, int64_t ldb, c128* C,
                       int64_t ldc, const int* flag) {
    hipLaunchKernelGGL(k_trmm_upper, dim3((p * p + 255) / 256), dim3(256), 0, s, p, A, lda, B, ldb, C, ldc, flag);
}
void launch_cholesky_piv(hipStream_t s, int p, const c128* S, int64_t lds, double rel, c128* out, int64_t ldo,
                         int* perm, int* qout) {
    hipLaunchKernelGGL(k_cholesky_piv, dim3(1), dim3(256), 0, s, p, S, lds, rel, out, ldo, perm, qout);
}
void launch_trmm_perm(hipStream_t s, int q, int p, const c128* A, int64_t lda, const c128* B, int64_t ldb,
                      const int* perm, c128* out, int64_t ldo) {
    if (q * p <= 0) return;
    hipLaunchKernelGGL(k_trmm_perm, dim3((q * p + 255) / 256), dim3(256), 0, s, q, p, A, lda, B, ldb, perm, out, ldo);
}
void launch_ls_apply(hipStream_t s, int j0, int j1, int p, const c128* Y, const c128* T, c128* C, int64_t ldc,
                     int ncols) {
    if (j1 <= j0 || ncols <= 0) return;
    hipLaunchKernelGGL(k_ls_apply, dim3(ncols), dim3(256), 0, s, j0, j1, p, Y, T, C, ldc);
}
void launch_ls_factor(hipStream_t s, int k, int p, c128* C, int64_t ldc, c128* Yk, c128* Tk) {
    hipLaunchKernelGGL(k_ls_factor, dim3(1), dim3(256), 0, s, k, p, C, ldc, Yk, Tk);
}
void launch_sum_batches(hipStream_t s, int m, int c, int nb, const c128* P, c128* C, int64_t ldc) {
    const int64_t per = (int64_t)m * c;
    if (per <= 0) return;
    hipLaunchKernelGGL(k_sum_batches, dim3((unsigned)((per + 255) / 256)), dim3(256), 0, s, m, c, nb, P, C, ldc);
}
void launch_gemm_hn_part(hipStream_t s, int64_t n, int m, int c, const c128* A, int64_t lda, const c128* B, int64_t ldb,
                         int nb, int64_t L, c128* P) {
    if (n <= 0 || m <= 0 || c <= 0 || nb <= 0) return;
    const dim3 g((unsigned)((m + kHnTM - 1) / kHnTM), (unsigned)((c + kHnTC - 1) / kHnTC), (unsigned)nb);
    hipLaunchKernelGGL(k_gemm_hn_part, g, dim3(256), 0, s, n, m, c, A, lda, B, ldb, L, P);
}
void launch_tri_inv_upper(hipStream_t s, int k, const c128* U, int64_t ldu, c128* out, int64_t ldo) {
    if (k > 0) hipLaunchKernelGGL(k_tri_inv_upper, dim3(1), dim3(256), 0, s, k, U, ldu, out, ldo);
}
void launch_trsm_upper_left(hipStream_t s, int m, int p, const c128* U, int64_t ldu, c128* Y, int64_t ldy) {
    if (m > 0 && p > 0) hipLaunchKernelGGL(k_trsm_upper_left, dim3((unsigned)p), dim3(1024), 0, s, m, U, ldu, Y, ldy);
}
void launch_gemm_nn_acc(hipStream_t s, int64_t n, int m, int q, const c128* V, int64_t ldv, const c128* H,
                        int64_t ldh, double beta, double sign, c128* W, int64_t ldw) {
    if (n <= 0 || m <= 0 || q <= 0) return;
    const dim3 g((unsigned)((n + 63) / 64));
    switch ((q + 15) / 16) {
        case 1: hipLaunchKernelGGL(k_gemm_nn_acc<1>, g, dim3(256), 0, s, n, m, q, V, ldv, H, ldh, beta, sign, W, ldw); break;
        case 2: hipLaunchKernelGGL(k_gemm_nn_acc<2>, g, dim3(256), 0, s, n, m, q, V, ldv, H, ldh, beta, sign, W, ldw); break;
        case 3: hipLaunchKernelGGL(k_gemm_nn_acc<3>, g, dim3(256), 0, s, n, m, q, V, ldv, H, ldh, beta, sign, W, ldw); break;
        default: hipLaunchKernelGGL(k_gemm_nn_acc<4>, g, dim3(256), 0, s, n, m, q, V, ldv, H, ldh, beta, sign, W, ldw); break;
    }
}
void launch_col_norms(hipStream_t s, int rows, const c128* C, int64_t ldc, int ncols, double* out) {
    hipLaunchKernelGGL(k_col_norms, dim3(ncols), dim3(256), 0, s, rows, C, ldc, out);
}

#define QRVIE_NT_SWITCH(nt, KERNEL, ...)                                              \
    switch (nt) {                                                                      \
        case 1: hipLaunchKernelGGL(KERNEL<1>, __VA_ARGS__); break;                     \
        case 2: hipLaunchKernelGGL(KERNEL<2>, __VA_ARGS__); break;                     \
        case 3: hipLaunchKernelGGL(KERNEL<3>, __VA_ARGS__); break;                     \
        default: hipLaunchKernelGGL(KERNEL<4>, __VA_ARGS__); break;                    \
    }

namespace {
// the tile-shape table, in the order the autotuner reports it
constexpr int kTileU[kStripVariants] = {2, 1, 4, 1, 2, 4};
constexpr int kTileRT[kStripVariants] = {1, 1, 1, 2, 2, 2};

template <int NT, typename F>
void strip_nt(hipStream_t s, int v, const MStrip* st, int64_t n, const F* fac, const c128* in, c128* out,
              const int64_t* tmap) {
    const dim3 g((unsigned)n);
    switch (v) {
        case 1: hipLaunchKernelGGL((k_strip_mfma<NT, 1, 1, F>), g, dim3(256), 0, s, st, fac, in, out, tmap); break;
        case 2: hipLaunchKernelGGL((k_strip_mfma<NT, 4, 1, F>), g, dim3(256), 0, s, st, fac, in, out, tmap); break;
        case 3: hipLaunchKernelGGL((k_strip_mfma<NT, 1, 2, F>), g, dim3(128), 0, s, st, fac, in, out, tmap); break;
        case 4: hipLaunchKernelGGL((k_strip_mfma<NT, 2, 2, F>), g, dim3(128), 0, s, st, fac, in, out, tmap); break;
        case 5: hipLaunchKernelGGL((k_strip_mfma<NT, 4, 2, F>), g, dim3(128), 0, s, st, fac, in, out, tmap); break;
        default: hipLaunchKernelGGL((k_strip_mfma<NT, 2, 1, F>), g, dim3(256), 0, s, st, fac, in, out, tmap); break;
    }
}

template <typename F>
void strip_any(hipStream_t s, int nt, int v, const MStrip* st, int64_t n, const F* fac, const c128* in, c128* out,
               const int64_t* tmap) {
    if (n <= 0) return;
    switch (nt) {
        case 1: strip_nt<1>(s, v, st, n, fac, in, out, tmap); break;
        case 2: strip_nt<2>(s, v, st, n, fac, in, out, tmap); break;
        case 3: strip_nt<3>(s, v, st, n, fac, in, out, tmap); break;
        default: strip_nt<4>(s, v, st, n, fac, in, out, tmap); break;
    }
}
}  // namespace

template <int KIND>
void strip32_any(hipStream_t s, int nt, const MStrip* st, int64_t n, const void* fac, int64_t plane, const c128* in,
                 c128* out, const int64_t* tmap) {
    if (n <= 0) return;
    const dim3 g((unsigned)n);
    switch (nt) {
        case 1: hipLaunchKernelGGL((k_strip_mfma32<1, KIND>), g, dim3(256), 0, s, st, fac, plane, in, out, tmap); break;
        case 2: hipLaunchKernelGGL((k_strip_mfma32<2, KIND>), g, dim3(256), 0, s, st, fac, plane, in, out, tmap); break;
        case 3: hipLaunchKernelGGL((k_strip_mfma32<3, KIND>), g, dim3(256), 0, s, st, fac, plane, in, out, tmap); break;
        default: hipLaunchKernelGGL((k_strip_mfma32<4, KIND>), g, dim3(256), 0, s, st, fac, plane, in, out, tmap); break;
    }
}

void launch_strip_mfma32(hipStream_t s, int nt, const MStrip* st, int64_t n, const float2* fac, const c128* in,
                         c128* out, const int64_t* tmap) {
    strip32_any<0>(s, nt, st, n, fac, 0, in, out, tmap);
}
void launch_strip_mfma32_bf16(hipStream_t s, int nt, const MStrip* st, int64_t n, const uint16_t* fac, int64_t plane,
                              const c128* in, c128* out, const int64_t* tmap) {
    strip32_any<1>(s, nt, st, n, fac, plane, in, out, tmap);
}

int strip_variant_u(int v) { return v >= 0 && v < kStripVariants ? kTileU[v] : 0; }
int strip_variant_rows(int v) { return v >= 0 && v < kStripVariants ? 16 * kTileRT[v] : 0; }

void launch_strip_mfma(hipStream_t s, int nt, const MStrip* st, int64_t n, const c128* fac, const c128* in,
                       c128* out, const int64_t* tmap, int variant) {
    strip_any(s, nt, variant, st, n, fac, in, out, tmap);
}
void launch_strip_mfma(hipStream_t s, int nt, const MStrip* st, int64_t n, const float2* fac, const c128* in,
                       c128* out, const int64_t* tmap, int variant) {
    strip_any(s, nt, variant, st, n, fac, in, out, tmap);
}
void launch_count_neq(hipStream_t s, int64_t n, const void* a, const void* b, unsigned long long* count) {
    if (n <= 0) return;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_count_neq, dim3((unsigned)blocks), dim3(256), 0, s, n, (const unsigned long long*)a,
                       (const unsigned long long*)b, count);
}
void launch_block_combine(hipStream_t s, int nt, int64_t n, const c128* ylev, int nlev, const c128* yself,
                          const c128* V, c128* out) {
    const int64_t tot = n * 16 * nt;
    QRVIE_NT_SWITCH(nt, k_block_combine, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, ylev, nlev, yself, V,
                    out);
}
void launch_gather_block(hipStream_t s, int nt, int32_t N, const int32_t* i2c, const c128* src, int64_t ld,
                         int ncols, c128* blk) {
    const int64_t tot = (int64_t)N * kNp;
    QRVIE_NT_SWITCH(nt, k_gather_block, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, N, i2c, src, ld, ncols,
                    blk);
}
void launch_scatter_block(hipStream_t s, int nt, int32_t N, const int32_t* i2c, const c128* blk, c128* dst,
                          int64_t ld, int ncols) {
    const int64_t tot = (int64_t)N * kNp;
    QRVIE_NT_SWITCH(nt, k_scatter_block, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, N, i2c, blk, dst, ld,
                    ncols);
}

}  // namespace qrvie
