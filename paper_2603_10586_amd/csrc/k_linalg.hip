// Dense complex FP64 kernels behind the low-rank compression of far blocks (§5.2,
// eq. 5.3) and the preconditioner setup (§4, eq. 4.2).
//
//  * k_gemm     batched 64x64-tiled complex GEMM (op(A) = A or A^H; B stored or a
//               generated random sketch), plus a residual mode that returns
//               per-tile partials of ||C - A B||_F^2 for certification.
//  * k_qrcp     truncated column-pivoted Householder QR, one workgroup per matrix,
//               stopping at the first rank whose exact trailing Frobenius norm meets
//               the tolerance (the low-rank QR of §5.2).  Column norms of the trailing
//               rows are recomputed exactly in the same pass as the reflector update.
//  * k_form_q   explicit orthonormal Q from the stored reflectors.
//  * k_extract_r  R with the column permutation undone.
//  * k_cgs2     block classical Gram-Schmidt with one reorthogonalisation (FP64 MFMA
//               panel projections), dropping numerically dependent columns (range
//               basis of a sketch).
//  * k_invert   Gauss-Jordan inversion with partial pivoting of 144 x 144 blocks.
// All reductions run in a fixed order: results do not depend on scheduling.
#include "internal.h"

namespace qrvie {

namespace {

__device__ __forceinline__ c128 cmul(c128 a, c128 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ c128 cmulc(c128 a, c128 b) {  // conj(a) * b
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ c128 cadd(c128 a, c128 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ c128 csub(c128 a, c128 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double cabs2(c128 a) { return a.x * a.x + a.y * a.y; }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ c128 wave_sum(c128 v) {
    return make_double2(wave_sum(v.x), wave_sum(v.y));
}

// Block-wide sum of one double per thread over NW waves, fixed order.
template <int NW>
__device__ double block_sum(double v, double* red) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) red[wv] = v;
    __syncthreads();
    double r = red[0];
    for (int w = 1; w < NW; ++w) r += red[w];
    return r;
}

// Block-wide sum of one double per thread (256 threads), fixed order.
__device__ double block_sum256(double v, double* red) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) red[wv] = v;
    __syncthreads();
    const double r = (red[0] + red[1]) + (red[2] + red[3]);
    return r;
}

// Counter-based uniform in [-1, 1): splitmix64 of (seed, i, j).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__device__ __forceinline__ c128 rand_c(uint64_t seed, int64_t i, int64_t j) {
    const uint64_t h = mix64(seed ^ mix64((uint64_t)i * 0x100000001B3ull + (uint64_t)j));
    const uint64_t h2 = mix64(h);
    const double s = 1.0 / 9007199254740992.0;  // 2^-53
    return make_double2((double)(h >> 11) * s * 2.0 - 1.0, (double)(h2 >> 11) * s * 2.0 - 1.0);
}

// --------------------------------------------------------------------- GEMM
// mode 0: C = A B        mode 1: C = A^H B      mode 2: C = A Omega(seed)
// mode 3: partial[tile] = ||C - A B||^2 over the tile (C is read, not written)
// mode 4: C = A B with B stored by rows (B(k, j) at B[j + k ldb])
constexpr int TM = 64, TN = 64, TK = 16;

template <int MODE>
__global__ void __launch_bounds__(256) k_gemm(const GemmDesc* descs, const int32_t* tdesc, const int32_t* tmn,
                                              double* partial) {
    const GemmDesc d = descs[tdesc[blockIdx.x]];
    const int tm = tmn[blockIdx.x] >> 16, tn = tmn[blockIdx.x] & 0xFFFF;
    const int m0 = tm * TM, n0 = tn * TN;
    const int tid = threadIdx.x;
    const int tx = tid & 15, ty = tid >> 4;
    __shared__ c128 As[TK][TM + 1];
    __shared__ c128 Bs[TK][TN + 1];
    c128 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = make_double2(0.0, 0.0);

    for (int k0 = 0; k0 < d.k; k0 += TK) {
        // A tile: op(A)(i, kk), i in [m0, m0+64), kk in [k0, k0+16)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int i, kk;
            if (MODE == 1) { kk = tid & 15; i = (tid >> 4) + 16 * q; }
            else { i = tid & 63; kk = (tid >> 6) + 4 * q; }
            const int gi = m0 + i, gk = k0 + kk;
            c128 v = make_double2(0.0, 0.0);
            if (gi < d.m && gk < d.k) {
                if (MODE == 1) { c128 t = d.A[(int64_t)gk + (int64_t)gi * d.lda]; v = make_double2(t.x, -t.y); }
                else v = d.A[(int64_t)gi + (int64_t)gk * d.lda];
            }
            As[kk][i] = v;
        }
        // B tile: B(kk, j)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int kk, j;
            if (MODE == 4) { j = tid & 63; kk = (tid >> 6) + 4 * q; }
            else { kk = tid & 15; j = (tid >> 4) + 16 * q; }
            const int gk = k0 + kk, gj = n0 + j;
            c128 v = make_double2(0.0, 0.0);
            if (gk < d.k && gj < d.n) {
                if (MODE == 2) v = rand_c(d.seed, gk, gj);
                else if (MODE == 4) v = d.B[(int64_t)gj + (int64_t)gk * d.ldb];
                else v = d.B[(int64_t)gk + (int64_t)gj * d.ldb];
            }
            Bs[kk][j] = v;
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < TK; ++kk) {
            c128 av[4], bv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) av[a] = As[kk][ty + 16 * a];
#pragma unroll
            for (int b = 0; b < 4; ++b) bv[b] = Bs[kk][tx + 16 * b];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    acc[a][b].x = fma(av[a].x, bv[b].x, fma(-av[a].y, bv[b].y, acc[a][b].x));
                    acc[a][b].y = fma(av[a].x, bv[b].y, fma(av[a].y, bv[b].x, acc[a][b].y));
                }
        }
        __syncthreads();
    }
    if (MODE == 3) {
        double s = 0.0;
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int gi = m0 + ty + 16 * a, gj = n0 + tx + 16 * b;
                if (gi < d.m && gj < d.n) s += cabs2(csub(d.C[(int64_t)gi + (int64_t)gj * d.ldc], acc[a][b]));
            }
        __shared__ double red[4];
        s = block_sum256(s, red);
        if (tid == 0) partial[blockIdx.x] = s;
        return;
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int gi = m0 + ty + 16 * a, gj = n0 + tx + 16 * b;
            if (gi < d.m && gj < d.n) d.C[(int64_t)gi + (int64_t)gj * d.ldc] = acc[a][b];
        }
}

// --------------------------------------------------------------------- QRCP
template <int MAXR, int NTH>
__global__ void __launch_bounds__(NTH) k_qrcp(const QrcpDesc* descs) {
    constexpr int NW = NTH / 64;
    const QrcpDesc d = descs[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int m = d.m, n = d.n;
    const int64_t lda = d.lda;
    const int kmax = min(d.kmax, min(m, n));
    __shared__ c128 wl[64 * MAXR];
    __shared__ double rsum[NTH];
    __shared__ double rmax[NTH];
    __shared__ int rarg[NTH];
    __shared__ double s_tau;

    for (int j = wv; j < n; j += NW) {
        double s = 0.0;
        for (int i = lane; i < m; i += 64) s += cabs2(d.A[i + j * lda]);
        s = wave_sum(s);
        if (lane == 0) { d.colnorm2[j] = s; d.perm[j] = j; }
    }
    __syncthreads();

    double tol2 = 0.0;
    int rank = kmax;
    double trail = 0.0;
    for (int s = 0;; ++s) {
        // trailing sum and pivot over j in [s, n)
        double sum = 0.0, best = -1.0;
        int bj = n;
        for (int j = s + tid; j < n; j += NTH) {
            const double v = d.colnorm2[j];
            sum += v;
            if (v > best) { best = v; bj = j; }
        }
        rsum[tid] = sum; rmax[tid] = best; rarg[tid] = bj;
        __syncthreads();
        for (int o = NTH / 2; o > 0; o >>= 1) {
            if (tid < o) {
                rsum[tid] += rsum[tid + o];
                const double b2 = rmax[tid + o];
                const int a2 = rarg[tid + o];
                if (b2 > rmax[tid] || (b2 == rmax[tid] && a2 < rarg[tid])) { rmax[tid] = b2; rarg[tid] = a2; }
            }
            __syncthreads();
        }
        const double total = rsum[0];
        const int p = rarg[0];
        __syncthreads();
        if (s == 0) {
            const double base = d.base2 > 0.0 ? d.base2 : total;
            const double sub = d.sub2 < 0.0 ? fmax(0.0, base - total) : d.sub2;
            tol2 = d.rel2 * base - sub;
            if (tid == 0 && d.norm2_out) *d.norm2_out = total;
        }
        if (total <= tol2 || s >= kmax) { rank = s; trail = total; break; }
        if (p != s) {
            for (int i = tid; i < m; i += NTH) {
                const c128 a = d.A[i + s * lda];
                d.A[i + s * lda] = d.A[i + p * lda];
                d.A[i + p * lda] = a;
            }
            if (tid == 0) {
                const double t = d.colnorm2[s]; d.colnorm2[s] = d.colnorm2[p]; d.colnorm2[p] = t;
                const int q = d.perm[s]; d.perm[s] = d.perm[p]; d.perm[p] = q;
            }
        }
        __syncthreads();
        // Householder reflector from column s (rows s..m-1): P = I - tau w w^H, P x = beta e1
        if (wv == 0) {
            double xn2 = 0.0;
            for (int i = s + lane; i < m; i += 64) xn2 += cabs2(d.A[i + s * lda]);
            xn2 = wave_sum(xn2);
            if (lane == 0) {
                const c128 x0 = d.A[s + s * lda];
                const double xn = sqrt(xn2);
                const double ax0 = sqrt(cabs2(x0));
                const c128 ph = ax0 > 0.0 ? make_double2(x0.x / ax0, x0.y / ax0) : make_double2(1.0, 0.0);
                const c128 w0 = make_double2(x0.x + ph.x * xn, x0.y + ph.y * xn);
                const double tau = xn > 0.0 ? 1.0 / (xn * (xn + ax0)) : 0.0;
                d.tau[s] = tau;
                d.wtop[s] = w0;
                d.A[s + s * lda] = make_double2(-ph.x * xn, -ph.y * xn);
                s_tau = tau;
                wl[0] = w0;
            }
        }
        for (int i = 1 + tid; i < m - s; i += NTH) wl[i] = d.A[s + i + s * lda];
        __syncthreads();
        const double tau = s_tau;
        // trailing columns, each wave taking every NW-th one; CJ columns at a time so that
        // their independent wave reductions overlap
        constexpr int CJ = MAXR <= 4 ? 4 : (MAXR <= 10 ? 2 : 1);
        for (int j0 = s + 1 + wv; j0 < n; j0 += NW * CJ) {
            c128 a[CJ][MAXR];
            c128 dot[CJ];
#pragma unroll
            for (int c = 0; c < CJ; ++c) {
                const int j = j0 + NW * c;
                dot[c] = make_double2(0.0, 0.0);
#pragma unroll
                for (int q = 0; q < MAXR; ++q) {
                    const int i = lane + 64 * q;
                    a[c][q] = make_double2(0.0, 0.0);
                    if (j < n && s + i < m) {
                        a[c][q] = d.A[s + i + (int64_t)j * lda];
                        dot[c] = cadd(dot[c], cmulc(wl[i], a[c][q]));
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < CJ; ++c) dot[c] = wave_sum(dot[c]);
            double nrm[CJ];
#pragma unroll
            for (int c = 0; c < CJ; ++c) {
                const int j = j0 + NW * c;
                const c128 f = make_double2(tau * dot[c].x, tau * dot[c].y);
                nrm[c] = 0.0;
#pragma unroll
                for (int q = 0; q < MAXR; ++q) {
                    const int i = lane + 64 * q;
                    if (j < n && s + i < m) {
                        a[c][q] = csub(a[c][q], cmul(wl[i], f));
                        d.A[s + i + (int64_t)j * lda] = a[c][q];
                        if (i >= 1) nrm[c] += cabs2(a[c][q]);
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < CJ; ++c) nrm[c] = wave_sum(nrm[c]);
            if (lane == 0) {
#pragma unroll
                for (int c = 0; c < CJ; ++c)
                    if (j0 + NW * c < n) d.colnorm2[j0 + NW * c] = nrm[c];
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        *d.rank_out = rank;
        if (d.trail2_out) *d.trail2_out = trail;
    }
}

// Stepped QRCP for the projected sketches W (at most a few hundred rows, up to 10^4
// columns, few matrices per chunk): the same truncated column-pivoted Householder QR, but
// each pivot step is two launches over all matrices, so one matrix's trailing update is
// spread over many workgroups.  k_qrcp_begin computes the column norms and the tolerance;
// k_qrcp_pivot (one workgroup per matrix) picks the pivot, stops at the tolerance, swaps
// and forms the reflector; k_qrcp_apply (workgroups over 128-column chunks) applies it to
// the trailing columns and recomputes their exact trailing norms.  A finished matrix has
// rank_out >= 0 and its workgroups return at once.
constexpr int kQrcpChunk = 128;

__global__ void __launch_bounds__(256) k_qrcp_begin(const QrcpDesc* descs) {
    const QrcpDesc d = descs[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    __shared__ double red[4];
    double part = 0.0;
    for (int j = wv; j < d.n; j += 4) {
        double sj = 0.0;
        for (int i = lane; i < d.m; i += 64) sj += cabs2(d.A[i + (int64_t)j * d.lda]);
        sj = wave_sum(sj);
        if (lane == 0) { d.colnorm2[j] = sj; d.perm[j] = j; }
        part += sj;                     // wave-uniform
    }
    const double total = block_sum<4>(lane == 0 ? part : 0.0, red);
    if (tid == 0) {
        const double base = d.base2 > 0.0 ? d.base2 : total;
        const double sub = d.sub2 < 0.0 ? fmax(0.0, base - total) : d.sub2;
        *d.tol2_state = d.rel2 * base - sub;
        if (d.norm2_out) *d.norm2_out = total;
        *d.rank_out = -1;
    }
}

__global__ void __launch_bounds__(256) k_qrcp_pivot(const QrcpDesc* descs, int s) {
    const QrcpDesc d = descs[blockIdx.x];
    if (*d.rank_out >= 0) return;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int m = d.m, n = d.n;
    const int64_t lda = d.lda;
    const int kmax = min(d.kmax, min(m, n));
    __shared__ double rsum[256];
    __shared__ double rmax[256];
    __shared__ int rarg[256];
    __shared__ double red[4];
    double sum = 0.0, best = -1.0;
    int bj = n;
    for (int j = s + tid; j < n; j += 256) {
        const double v = d.colnorm2[j];
        sum += v;
        if (v > best) { best = v; bj = j; }
    }
    rsum[tid] = sum; rmax[tid] = best; rarg[tid] = bj;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) {
            rsum[tid] += rsum[tid + o];
            const double b2 = rmax[tid + o];
            const int a2 = rarg[tid + o];
            if (b2 > rmax[tid] || (b2 == rmax[tid] && a2 < rarg[tid])) { rmax[tid] = b2; rarg[tid] = a2; }
        }
        __syncthreads();
    }
    const double total = rsum[0];
    const int p = rarg[0];
    if (total <= *d.tol2_state || s >= kmax) {
        if (tid == 0) {
            *d.rank_out = s;
            if (d.trail2_out) *d.trail2_out = total;
        }
        return;
    }
    if (p != s) {
        for (int i = tid; i < m; i += 256) {
            const c128 a = d.A[i + s * lda];
            d.A[i + s * lda] = d.A[i + p * lda];
            d.A[i + p * lda] = a;
        }
        if (tid == 0) {
            const double t = d.colnorm2[s]; d.colnorm2[s] = d.colnorm2[p]; d.colnorm2[p] = t;
            const int q = d.perm[s]; d.perm[s] = d.perm[p]; d.perm[p] = q;
        }
    }
    __syncthreads();
    // reflector P = I - tau w w^H with P x = beta e1 for x = A[s:m, s]; w[0] = wtop[s], the
    // rest of w stays in A[s+1:m, s]
    double xn2 = 0.0;
    for (int i = s + tid; i < m; i += 256) xn2 += cabs2(d.A[i + s * lda]);
    xn2 = block_sum<4>(xn2, red);
    if (tid == 0) {
        const c128 x0 = d.A[s + s * lda];
        const double xn = sqrt(xn2);
        const double ax0 = sqrt(cabs2(x0));
        const c128 ph = ax0 > 0.0 ? make_double2(x0.x / ax0, x0.y / ax0) : make_double2(1.0, 0.0);
        d.tau[s] = xn > 0.0 ? 1.0 / (xn * (xn + ax0)) : 0.0;
        d.wtop[s] = make_double2(x0.x + ph.x * xn, x0.y + ph.y * xn);
        d.A[s + s * lda] = make_double2(-ph.x * xn, -ph.y * xn);
    }
    (void)wv;
    (void)lane;
}

template <int MAXR>
__global__ void __launch_bounds__(256) k_qrcp_apply(const QrcpDesc* descs, int s) {
    const QrcpDesc d = descs[blockIdx.y];
    if (*d.rank_out >= 0) return;
    const int n = d.n;
    const int c0 = s + 1 + blockIdx.x * kQrcpChunk;
    if (c0 >= n) return;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int m = d.m;
    const int64_t lda = d.lda;
    __shared__ c128 wl[64 * MAXR];
    for (int i = tid; i < m - s; i += 256) wl[i] = i == 0 ? d.wtop[s] : d.A[s + i + s * lda];
    __syncthreads();
    const double tau = d.tau[s];
    const int c1 = min(n, c0 + kQrcpChunk);
    constexpr int CJ = MAXR <= 4 ? 4 : (MAXR <= 10 ? 2 : 1);
    for (int j0 = c0 + wv; j0 < c1; j0 += 4 * CJ) {
        c128 a[CJ][MAXR];
        c128 dot[CJ];
#pragma unroll
        for (int c = 0; c < CJ; ++c) {
            const int j = j0 + 4 * c;
            dot[c] = make_double2(0.0, 0.0);
#pragma unroll
            for (int q = 0; q < MAXR; ++q) {
                const int i = lane + 64 * q;
                a[c][q] = make_double2(0.0, 0.0);
                if (j < c1 && s + i < m) {
                    a[c][q] = d.A[s + i + (int64_t)j * lda];
                    dot[c] = cadd(dot[c], cmulc(wl[i], a[c][q]));
                }
            }
        }
#pragma unroll
        for (int c = 0; c < CJ; ++c) dot[c] = wave_sum(dot[c]);
        double nrm[CJ];
#pragma unroll
        for (int c = 0; c < CJ; ++c) {
            const int j = j0 + 4 * c;
            const c128 f = make_double2(tau * dot[c].x, tau * dot[c].y);
            nrm[c] = 0.0;
#pragma unroll
            for (int q = 0; q < MAXR; ++q) {
                const int i = lane + 64 * q;
                if (j < c1 && s + i < m) {
                    a[c][q] = csub(a[c][q], cmul(wl[i], f));
                    d.A[s + i + (int64_t)j * lda] = a[c][q];
                    if (i >= 1) nrm[c] += cabs2(a[c][q]);
                }
            }
        }
#pragma unroll
        for (int c = 0; c < CJ; ++c) nrm[c] = wave_sum(nrm[c]);
        if (lane == 0) {
#pragma unroll
            for (int c = 0; c < CJ; ++c)
                if (j0 + 4 * c < c1) d.colnorm2[j0 + 4 * c] = nrm[c];
        }
    }
}

// Q = P_0 ... P_{r-1} [I_r; 0]
template <int MAXR>
__global__ void __launch_bounds__(256) k_form_q(const FormQDesc* descs) {
    const FormQDesc d = descs[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int m = d.m, r = d.r;
    __shared__ c128 wl[64 * MAXR];
    for (int64_t e = tid; e < (int64_t)m * r; e += 256) {
        const int i = (int)(e % m), c = (int)(e / m);
        d.Q[i + (int64_t)c * d.ldq] = make_double2(i == c ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    for (int s = r - 1; s >= 0; --s) {
        for (int i = tid; i < m - s; i += 256) wl[i] = (i == 0) ? d.wtop[s] : d.A[s + i + (int64_t)s * d.lda];
        __syncthreads();
        const double tau = d.tau[s];
        for (int c = s + wv; c < r; c += 4) {
            c128 a[MAXR];
            c128 dot = make_double2(0.0, 0.0);
#pragma unroll
            for (int q = 0; q < MAXR; ++q) {
                const int i = lane + 64 * q;
                a[q] = make_double2(0.0, 0.0);
                if (s + i < m) {
                    a[q] = d.Q[s + i + (int64_t)c * d.ldq];
                    dot = cadd(dot, cmulc(wl[i], a[q]));
                }
            }
            dot = wave_sum(dot);
            const c128 f = make_double2(tau * dot.x, tau * dot.y);
#pragma unroll
            for (int q = 0; q < MAXR; ++q) {
                const int i = lane + 64 * q;
                if (s + i < m) d.Q[s + i + (int64_t)c * d.ldq] = csub(a[q], cmul(wl[i], f));
            }
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(256) k_extract_r(const ExtractRDesc* descs) {
    const ExtractRDesc d = descs[blockIdx.x];
    const int64_t tot = (int64_t)d.r * d.n;
    for (int64_t e = threadIdx.x; e < tot; e += 256) {
        const int i = (int)(e % d.r), j = (int)(e / d.r);
        const c128 v = (i <= j) ? d.A[i + (int64_t)j * d.lda] : make_double2(0.0, 0.0);
        d.R[i + (int64_t)d.perm[j] * d.ldr] = v;
    }
}

// Block CGS2 with dropping; the kept columns are compacted to the front of Y.  The sketch is
// taken in panels of 16 columns.  Each panel is projected against all kept columns Q twice
// (H = Q^H P, P -= Q H) on FP64 MFMA: the waves split the 16-column tiles of Q for H and
// the 16-row tiles of P for the update, with H in LDS.  The panel's columns are then
// orthogonalised one by one against the panel's earlier kept columns, twice (one sweep over
// the rows per pass for all dot products), and a column is kept when its remaining norm
// exceeds drop_rel times its norm before any projection.  Every reduction has a fixed order.
typedef double v4d __attribute__((ext_vector_type(4)));

// Operand layout of the 16x16x4 FP64 MFMA: A (16 x 4): lane l holds A[l % 16][l / 16];
// B (4 x 16): lane l holds B[l / 16][l % 16]; D (16 x 16): lane l, slot i holds
// D[l / 16 + 4 i][l % 16].  A complex product is four real MFMAs.
__device__ __forceinline__ void cmfma(v4d& re, v4d& im, c128 a, c128 b) {
    re = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, re, 0, 0, 0);
    re = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, b.y, re, 0, 0, 0);
    im = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.y, im, 0, 0, 0);
    im = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.x, im, 0, 0, 0);
}

constexpr int kPanel = 16;

template <int KMAX, int NTH>
__global__ void __launch_bounds__(NTH) k_cgs2(const Cgs2Desc* descs) {
    constexpr int NW = NTH / 64;
    const Cgs2Desc d = descs[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int rl = lane & 15, kq = lane >> 4;
    const int m = d.m;
    const int64_t ld = d.ldy;
    c128* Y = d.Y;
    __shared__ c128 Hs[KMAX * kPanel];          // H = Q^H P, row q at Hs[q * 16]
    __shared__ c128 red16[NW][kPanel];
    __shared__ c128 hcol[kPanel];
    __shared__ double n0s[kPanel];
    __shared__ double red[NW];
    const c128 z = make_double2(0.0, 0.0);
    int kept = 0;
    for (int c0 = 0; c0 < d.k; c0 += kPanel) {
        const int pc = min(kPanel, d.k - c0);
        c128* P = Y + (int64_t)c0 * ld;
        for (int j = wv; j < pc; j += NW) {
            double s = 0.0;
            for (int i = lane; i < m; i += 64) s += cabs2(P[i + j * ld]);
            s = wave_sum(s);
            if (lane == 0) n0s[j] = s;
        }
        __syncthreads();
        for (int pass = 0; pass < 2 && kept > 0; ++pass) {
            // H = Q^H P: tile t of 16 kept columns per wave, 4-row steps over m
            const int pj = min(rl, pc - 1);
            for (int t = wv; 16 * t < kept; t += NW) {
                const int qa = min(16 * t + rl, kept - 1);
                v4d re = v4d{0.0, 0.0, 0.0, 0.0}, im = re;
                // batches of 4 four-row steps: the loads of a batch are issued together
                for (int i = 0; i < m; i += 16) {
                    c128 a[4], b[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int row = i + 4 * u + kq;
                        const bool ok = row < m;
                        a[u] = ok ? Y[row + qa * ld] : z;
                        b[u] = ok ? P[row + pj * ld] : z;
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        a[u].y = -a[u].y;
                        cmfma(re, im, a[u], b[u]);
                    }
                }
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int q = 16 * t + kq + 4 * s;
                    if (q < kept) Hs[q * kPanel + rl] = make_double2(re[s], im[s]);
                }
            }
            __syncthreads();
            // P -= Q H: row tile r of 16 rows per wave, 4-column steps over the kept columns
            for (int r = wv; 16 * r < m; r += NW) {
                const int r0 = 16 * r;
                const int ra = min(r0 + rl, m - 1);
                v4d re = v4d{0.0, 0.0, 0.0, 0.0}, im = re;
                for (int q = 0; q < kept; q += 16) {
                    c128 a[4], b[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int qq = q + 4 * u + kq;
                        const bool ok = qq < kept;
                        a[u] = ok ? Y[ra + qq * ld] : z;
                        b[u] = ok ? Hs[qq * kPanel + rl] : z;
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) cmfma(re, im, a[u], b[u]);
                }
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int row = r0 + kq + 4 * s;
                    if (row < m && rl < pc) {
                        const c128 v = P[row + rl * ld];
                        P[row + rl * ld] = make_double2(v.x - re[s], v.y - im[s]);
                    }
                }
            }
            __syncthreads();
        }
        // within the panel, column by column
        const int kept0 = kept;
        for (int j = 0; j < pc; ++j) {
            c128* y = P + (int64_t)j * ld;
            const int np = kept - kept0;
            for (int pass = 0; pass < 2 && np > 0; ++pass) {
                c128 part[kPanel - 1];
#pragma unroll
                for (int q = 0; q < kPanel - 1; ++q) part[q] = z;
                for (int i = tid; i < m; i += NTH) {
                    const c128 v = y[i];
#pragma unroll
                    for (int q = 0; q < kPanel - 1; ++q)
                        if (q < np) part[q] = cadd(part[q], cmulc(Y[i + (int64_t)(kept0 + q) * ld], v));
                }
#pragma unroll
                for (int q = 0; q < kPanel - 1; ++q)
                    if (q < np) {
                        const c128 w = wave_sum(part[q]);
                        if (lane == 0) red16[wv][q] = w;
                    }
                __syncthreads();
                if (tid < np) {
                    c128 h = red16[0][tid];
                    for (int w = 1; w < NW; ++w) h = cadd(h, red16[w][tid]);
                    hcol[tid] = h;
                }
                __syncthreads();
                for (int i = tid; i < m; i += NTH) {
                    c128 v = y[i];
#pragma unroll
                    for (int q = 0; q < kPanel - 1; ++q)
                        if (q < np) v = csub(v, cmul(Y[i + (int64_t)(kept0 + q) * ld], hcol[q]));
                    y[i] = v;
                }
                __syncthreads();
            }
            double nr = 0.0;
            for (int i = tid; i < m; i += NTH) nr += cabs2(y[i]);
            nr = block_sum<NW>(nr, red);
            if (nr > 0.0 && nr > d.drop_rel * d.drop_rel * n0s[j] && kept < KMAX) {
                const double inv = 1.0 / sqrt(nr);
                c128* dst = Y + (int64_t)kept * ld;
                for (int i = tid; i < m; i += NTH) dst[i] = make_double2(y[i].x * inv, y[i].y * inv);
                ++kept;
            }
            __syncthreads();
        }
    }
    if (tid == 0) *d.kept_out = kept;
}

__global__ void __launch_bounds__(256) k_pack(const PackDesc* descs) {
    const PackDesc d = descs[blockIdx.x];
    const int64_t tot = (int64_t)d.rows * d.cols;
    for (int64_t e = threadIdx.x; e < tot; e += 256) {
        const int i = (int)(e % d.rows), j = (int)(e / d.rows);
        const int64_t o = d.transpose ? j + i * d.ldd : i + j * d.ldd;
        const int64_t si = i + (int64_t)j * d.lds;
        const c128 v = d.src32 ? make_double2((double)d.src32[si].x, (double)d.src32[si].y) : d.src[si];
        if (d.dst32) d.dst32[o] = make_float2((float)v.x, (float)v.y);
        else d.dst[o] = v;
    }
}

__global__ void __launch_bounds__(256) k_frob2(const c128* const* ptr, const int64_t* len, double* out) {
    const c128* p = ptr[blockIdx.x];
    const int64_t n = len[blockIdx.x];
    double s = 0.0;
    for (int64_t e = threadIdx.x; e < n; e += 256) s += cabs2(p[e]);
    __shared__ double red[4];
    s = block_sum256(s, red);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// In-place Gauss-Jordan inversion with partial pivoting, 144 x 144 column-major.
__global__ void __launch_bounds__(256) k_invert(c128* mats, int* info) {
    constexpr int n = kNp;
    c128* A = mats + (size_t)blockIdx.x * n * n;
    const int tid = threadIdx.x;
    __shared__ c128 col[n];
    __shared__ c128 row[n];
    __shared__ int piv[n];
    __shared__ double rmax[256];
    __shared__ int rarg[256];
    for (int k = 0; k < n; ++k) {
        double best = -1.0;
        int bi = n;
        for (int i = k + tid; i < n; i += 256) {
            const double v = cabs2(A[i + k * n]);
            if (v > best) { best = v; bi = i; }
        }
        rmax[tid] = best; rarg[tid] = bi;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (tid < o) {
                if (rmax[tid + o] > rmax[tid] || (rmax[tid + o] == rmax[tid] && rarg[tid + o] < rarg[tid])) {
                    rmax[tid] = rmax[tid + o]; rarg[tid] = rarg[tid + o];
                }
            }
            __syncthreads();
        }
        const int p = rarg[0];
        if (tid == 0) {
            piv[k] = p;
            if (!(rmax[0] > 0.0) && info) info[blockIdx.x] = k + 1;
        }
        __syncthreads();
        if (p != k)
            for (int j = tid; j < n; j += 256) {
                const c128 t = A[k + j * n]; A[k + j * n] = A[p + j * n]; A[p + j * n] = t;
            }
        __syncthreads();
        const c128 pv = A[k + k * n];
        const double den = cabs2(pv);
        const c128 ipv = make_double2(pv.x / den, -pv.y / den);
        for (int j = tid; j < n; j += 256) row[j] = (j == k) ? ipv : cmul(A[k + j * n], ipv);
        for (int i = tid; i < n; i += 256) col[i] = A[i + k * n];
        __syncthreads();
        for (int e = tid; e < n * n; e += 256) {
            const int i = e % n, j = e / n;
            if (i == k) A[i + j * n] = row[j];
            else {
                const c128 base = (j == k) ? make_double2(0.0, 0.0) : A[i + j * n];
                A[i + j * n] = csub(base, cmul(col[i], row[j]));
            }
        }
        __syncthreads();
    }
    for (int k = n - 1; k >= 0; --k) {
        const int p = piv[k];
        if (p != k)
            for (int i = tid; i < n; i += 256) {
                const c128 t = A[i + k * n]; A[i + k * n] = A[i + p * n]; A[i + p * n] = t;
            }
        __syncthreads();
    }
}

__global__ void k_sum_partials(const double* part, const int32_t* first, const int32_t* count, double* out, int n) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    double s = 0.0;
    for (int t = 0; t < count[b]; ++t) s += part[first[b] + t];
    out[b] = s;
}

}  // namespace

void launch_gemm(hipStream_t s, int mode, const GemmDesc* d, const int32_t* td, const int32_t* tmn, int64_t nt) {
    if (nt <= 0) return;
    dim3 g((unsigned)nt), b(256);
    // residual partials are written at the tile index; the sink is the first desc's out_norm2
    switch (mode) {
        case 0: hipLaunchKernelGGL(k_gemm<0>, g, b, 0, s, d, td, tmn, nullptr); break;
        case 1: hipLaunchKernelGGL(k_gemm<1>, g, b, 0, s, d, td, tmn, nullptr); break;
        case 2: hipLaunchKernelGGL(k_gemm<2>, g, b, 0, s, d, td, tmn, nullptr); break;
        case 4: hipLaunchKernelGGL(k_gemm<4>, g, b, 0, s, d, td, tmn, nullptr); break;
        default: break;
    }
}

void launch_gemm_residual(hipStream_t s, const GemmDesc* d, const int32_t* td, const int32_t* tmn, int64_t nt,
                          double* partial) {
    if (nt <= 0) return;
    hipLaunchKernelGGL(k_gemm<3>, dim3((unsigned)nt), dim3(256), 0, s, d, td, tmn, partial);
}

void launch_qrcp(hipStream_t s, const QrcpDesc* d, int n, int maxrows) {
    if (n <= 0) return;
    if (maxrows <= 192) hipLaunchKernelGGL((k_qrcp<3, 256>), dim3(n), dim3(256), 0, s, d);
    else if (maxrows <= 256) hipLaunchKernelGGL((k_qrcp<4, 256>), dim3(n), dim3(256), 0, s, d);
    else if (maxrows <= 640) hipLaunchKernelGGL((k_qrcp<10, 256>), dim3(n), dim3(256), 0, s, d);
    else hipLaunchKernelGGL((k_qrcp<16, 256>), dim3(n), dim3(256), 0, s, d);
}

void launch_qrcp_stepped(hipStream_t s, const QrcpDesc* d, int n, int maxrows, int maxcols, int maxsteps) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_qrcp_begin, dim3(n), dim3(256), 0, s, d);
    const unsigned chunks = (unsigned)((maxcols + kQrcpChunk - 1) / kQrcpChunk);
    for (int st = 0; st <= maxsteps; ++st) {
        hipLaunchKernelGGL(k_qrcp_pivot, dim3(n), dim3(256), 0, s, d, st);
        if (st == maxsteps) break;
        const dim3 g(chunks, (unsigned)n);
        if (maxrows <= 192) hipLaunchKernelGGL(k_qrcp_apply<3>, g, dim3(256), 0, s, d, st);
        else if (maxrows <= 256) hipLaunchKernelGGL(k_qrcp_apply<4>, g, dim3(256), 0, s, d, st);
        else if (maxrows <= 640) hipLaunchKernelGGL(k_qrcp_apply<10>, g, dim3(256), 0, s, d, st);
        else hipLaunchKernelGGL(k_qrcp_apply<16>, g, dim3(256), 0, s, d, st);
    }
}

void launch_form_q(hipStream_t s, const FormQDesc* d, int n, int maxrows) {
    if (n <= 0) return;
    if (maxrows <= 192) hipLaunchKernelGGL(k_form_q<3>, dim3(n), dim3(256), 0, s, d);
    else if (maxrows <= 256) hipLaunchKernelGGL(k_form_q<4>, dim3(n), dim3(256), 0, s, d);
    else if (maxrows <= 640) hipLaunchKernelGGL(k_form_q<10>, dim3(n), dim3(256), 0, s, d);
    else hipLaunchKernelGGL(k_form_q<16>, dim3(n), dim3(256), 0, s, d);
}

void launch_extract_r(hipStream_t s, const ExtractRDesc* d, int n) {
    if (n > 0) hipLaunchKernelGGL(k_extract_r, dim3(n), dim3(256), 0, s, d);
}
void launch_cgs2(hipStream_t s, const Cgs2Desc* d, int n, int kmax) {
    if (n <= 0) return;
    if (kmax <= 128) hipLaunchKernelGGL((k_cgs2<128, 512>), dim3(n), dim3(512), 0, s, d);
    else hipLaunchKernelGGL((k_cgs2<512, 512>), dim3(n), dim3(512), 0, s, d);
}
void launch_pack(hipStream_t s, const PackDesc* d, int n) {
    if (n > 0) hipLaunchKernelGGL(k_pack, dim3(n), dim3(256), 0, s, d);
}
void launch_frob2(hipStream_t s, const c128* const* p, const int64_t* len, double* out, int n) {
    if (n > 0) hipLaunchKernelGGL(k_frob2, dim3(n), dim3(256), 0, s, p, len, out);
}
void launch_invert(hipStream_t s, c128* A, int nmat, int* info) {
    if (nmat > 0) hipLaunchKernelGGL(k_invert, dim3(nmat), dim3(256), 0, s, A, info);
}
void launch_sum_partials(hipStream_t s, const double* part, const int32_t* first, const int32_t* count,
                         double* out, int n) {
    if (n > 0) hipLaunchKernelGGL(k_sum_partials, dim3((n + 255) / 256), dim3(256), 0, s, part, first, count, out, n);
}

}  // namespace qrvie
