// The compressed product y = Z_QR x (§5.2: each far block applied as Q (R x)) and the
// block-diagonal preconditioner z = Z_D^-1 y (§4, eq. 4.2).
//
// Layout (internal Morton order, complex128):
//  * R panels: for each (level, column node J) the R factors of every block with
//    column J stacked vertically, column-major with ld = total rank.  R-phase:
//    t = R_panel x_J, one 64-row strip per workgroup, the workgroup's waves
//    splitting the columns, x_J read as a wave-uniform broadcast.
//  * Q panels: for each (level, row node I) the Q factors of every block with row I
//    side by side, column-major with ld = rows of I.  Q-phase: y_l = Q_panel t_I,
//    the same strip/split scheme; one partial vector per active level.
//  * Final: per particle, y_p = Z_pp x_p + sum over levels of y_l (fixed order),
//    optionally r = v - y and z = Z_pp^-1 r, so a preconditioned residual or a
//    preconditioned product costs one pass.
// Every lane streams 16-byte complex loads down a column (coalesced 1 KiB per wave
// per column); no atomics, so results are bitwise reproducible.
#include "stream.h"

namespace qrvie {

namespace {

// Columns per batch: the same bytes in flight for 16- and 8-byte entries.
template <typename F> struct Unroll { static constexpr int U = sizeof(F) == 16 ? 8 : 16; };

template <int U>
__device__ __forceinline__ void wave_columns(int ncols, int waves, int wv, int& j0, int& j1) {
    const int per = (ncols + waves * U - 1) / (waves * U) * U;
    j0 = min(ncols, wv * per);
    j1 = min(ncols, j0 + per);
}

// acc += sum_{j in [j0, j1)} A[j*ld] * v[j]   (A already offset to this lane's row).
template <typename F>
__device__ __forceinline__ c128 column_stream(const F* __restrict__ A, int64_t ld, const c128* __restrict__ v,
                                              int j0, int j1) {
    constexpr int U = Unroll<F>::U;
    c128 acc0 = make_double2(0.0, 0.0), acc1 = acc0;
    const int nb = (j1 - j0) / U;
    stream_batches<F, U>(A + (int64_t)j0 * ld, ld, nb, [&](const F* w, int k) {
        const c128* vv = v + j0 + k * U;
#pragma unroll
        for (int u = 0; u < U; u += 2) {
            cfma(acc0, widen(w[u]), vv[u]);
            cfma(acc1, widen(w[u + 1]), vv[u + 1]);
        }
    });
    for (int j = j0 + nb * U; j < j1; ++j) cfma(acc0, widen(A[(int64_t)j * ld]), v[j]);
    return make_double2(acc0.x + acc1.x, acc0.y + acc1.y);
}

template <typename F, int WAVES>
__device__ __forceinline__ void rphase_body(const RStrip& s, const F* __restrict__ fac, const c128* __restrict__ x,
                                            c128* __restrict__ t, const int64_t* __restrict__ tmap) {
    const int lane = threadIdx.x & 63, wv = wave_id();
    const int row = min(lane, s.nrows - 1);
    int j0, j1;
    wave_columns<Unroll<F>::U>(s.ncols, WAVES, wv, j0, j1);
    const c128 acc = column_stream<F>(fac + s.a_off + row, s.ld, x + s.x_off, j0, j1);
    if (WAVES == 1) {
        if (lane < s.nrows) t[tmap[s.tmap_off + lane]] = acc;
        return;
    }
    __shared__ c128 red[WAVES][64];
    red[wv][lane] = acc;
    __syncthreads();
    if (wv == 0 && lane < s.nrows) {
        c128 sum = red[0][lane];
#pragma unroll
        for (int w = 1; w < WAVES; ++w) sum = make_double2(sum.x + red[w][lane].x, sum.y + red[w][lane].y);
        t[tmap[s.tmap_off + lane]] = sum;
    }
}

template <typename F, int WAVES>
__device__ __forceinline__ void qphase_body(const QStrip& s, const F* __restrict__ fac, const c128* __restrict__ t,
                                            c128* __restrict__ y) {
    const int lane = threadIdx.x & 63, wv = wave_id();
    const int row = min(lane, max(s.nrows - 1, 0));
    int j0, j1;
    wave_columns<Unroll<F>::U>(s.ncols, WAVES, wv, j0, j1);
    const c128 acc = column_stream<F>(fac + s.a_off + row, s.ld, t + s.t_off, j0, j1);
    if (WAVES == 1) {
        if (lane < s.nrows) y[s.y_off + lane] = acc;
        return;
    }
    __shared__ c128 red[WAVES][64];
    red[wv][lane] = acc;
    __syncthreads();
    if (wv == 0 && lane < s.nrows) {
        c128 sum = red[0][lane];
#pragma unroll
        for (int w = 1; w < WAVES; ++w) sum = make_double2(sum.x + red[w][lane].x, sum.y + red[w][lane].y);
        y[s.y_off + lane] = sum;
    }
}

template <int WAVES>
__global__ void __launch_bounds__(64 * WAVES) k_rphase(const RStrip* __restrict__ strips, const c128* __restrict__ fac,
                                                       const c128* __restrict__ x, c128* __restrict__ t,
                                                       const int64_t* __restrict__ tmap) {
    rphase_body<c128, WAVES>(strips[blockIdx.x], fac, x, t, tmap);
}
template <int WAVES>
__global__ void __launch_bounds__(64 * WAVES) k_rphase_c64(const RStrip* __restrict__ strips,
                                                           const float2* __restrict__ fac, const c128* __restrict__ x,
                                                           c128* __restrict__ t, const int64_t* __restrict__ tmap) {
    rphase_body<float2, WAVES>(strips[blockIdx.x], fac, x, t, tmap);
}
template <int WAVES>
__global__ void __launch_bounds__(64 * WAVES) k_qphase(const QStrip* __restrict__ strips, const c128* __restrict__ fac,
                                                       const c128* __restrict__ t, c128* __restrict__ y) {
    qphase_body<c128, WAVES>(strips[blockIdx.x], fac, t, y);
}
template <int WAVES>
__global__ void __launch_bounds__(64 * WAVES) k_qphase_c64(const QStrip* __restrict__ strips,
                                                           const float2* __restrict__ fac, const c128* __restrict__ t,
                                                           c128* __restrict__ y) {
    qphase_body<float2, WAVES>(strips[blockIdx.x], fac, t, y);
}

// ------------------------------------------------------------------ transpose-shared factors
// One Q (m x r) and R (r x n) per unordered pair (I, J); the mirror block (J, I) = R^T Q^T
// (symmetric weak form, Z = Z^T).  Three passes per product:
//  1. s = Q^T x_I for every Q panel column (column dot products: each wave owns 8 columns of a
//     panel, lanes own rows, one transposed reduction at the end);
//  2. one pass over every R panel strip computes both t = R x_J (per row, as the plain R
//     phase) and the strip's share of the mirror product R^T s (per column: each lane's
//     products are reduced over the wave, 8 columns at a time), written as one row of partials;
//  3. the Q phase y_I = Q t, whose strips add the partials of their rows in a fixed order.
// Q is streamed twice and R once, against twice each for stored mirror factors.

__device__ __forceinline__ c128 shfl_xor_c(c128 v, int m) {
    return make_double2(__shfl_xor(v.x, m, 64), __shfl_xor(v.y, m, 64));
}
__device__ __forceinline__ c128 cadd(c128 a, c128 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ c128 cmul(c128 a, c128 b) {
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}

// Cross-lane exchanges without LDS.  swap32_c: gfx950's v_permlane32_swap on the pair (a, b):
// lanes 32-63 of a trade places with lanes 0-31 of b.  swap16_c: v_permlane16_swap, odd
// 16-lane rows of a with even rows of b.  dpp_c: a DPP lane permutation within 16-lane rows.
__device__ __forceinline__ void swap_halves(double& a, double& b, bool wide) {
    const unsigned long long ua = (unsigned long long)__double_as_longlong(a);
    const unsigned long long ub = (unsigned long long)__double_as_longlong(b);
    const unsigned al = (unsigned)ua, ah = (unsigned)(ua >> 32), bl = (unsigned)ub, bh = (unsigned)(ub >> 32);
    unsigned rl0, rl1, rh0, rh1;
    if (wide) {
        const auto l = __builtin_amdgcn_permlane32_swap(al, bl, false, false);
        const auto h = __builtin_amdgcn_permlane32_swap(ah, bh, false, false);
        rl0 = l[0]; rl1 = l[1]; rh0 = h[0]; rh1 = h[1];
    } else {
        const auto l = __builtin_amdgcn_permlane16_swap(al, bl, false, false);
        const auto h = __builtin_amdgcn_permlane16_swap(ah, bh, false, false);
        rl0 = l[0]; rl1 = l[1]; rh0 = h[0]; rh1 = h[1];
    }
    a = __longlong_as_double((long long)(((unsigned long long)rh0 << 32) | rl0));
    b = __longlong_as_double((long long)(((unsigned long long)rh1 << 32) | rl1));
}
// a + (the pair partner's b), where the partner of lane L is L ^ 32 (wide) or L ^ 16; each
// lane keeps the half the swap leaves in place, so the sum is that of the kept column.
__device__ __forceinline__ c128 fold_swap(c128 a, c128 b, bool wide) {
    swap_halves(a.x, b.x, wide);
    swap_halves(a.y, b.y, wide);
    return make_double2(a.x + b.x, a.y + b.y);
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, 0xf, 0xf, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
template <int CTRL>
__device__ __forceinline__ c128 dpp_c(c128 v) { return make_double2(dpp_d<CTRL>(v.x), dpp_d<CTRL>(v.y)); }

constexpr int kDppRor8 = 0x128;        // row_ror:8, lane i of a row reads lane i ^ 8
constexpr int kDppHalfMirror = 0x141;  // row_half_mirror, lane i of 8 reads lane 7 - i
constexpr int kDppQuadXor1 = 0xB1;     // quad_perm [1, 0, 3, 2]
constexpr int kDppQuadXor2 = 0x4E;     // quad_perm [2, 3, 0, 1]

// Sums of 8 values per lane over the 64 lanes of a wave: every lane L returns the total of
// v[L >> 3].  Each of the first three steps halves the values a lane keeps (lanes with bit
// 5, 4, 3 set keep the upper half), then the 8 lanes of a group reduce their common column.
// The same from the second fold on: w2[p] = fold_swap(fold_swap(v[p], v[4 + p], true),
// fold_swap(v[2 + p], v[6 + p], true), false) already taken.
__device__ __forceinline__ c128 transpose_sum2(const c128 w2[2], int lane) {
    const c128 s0 = cadd(w2[0], dpp_c<kDppRor8>(w2[0]));
    const c128 s1 = cadd(w2[1], dpp_c<kDppRor8>(w2[1]));
    c128 w = (lane & 8) ? s1 : s0;
    w = cadd(w, dpp_c<kDppHalfMirror>(w));
    w = cadd(w, dpp_c<kDppQuadXor1>(w));
    return cadd(w, dpp_c<kDppQuadXor2>(w));
}

__device__ __forceinline__ c128 transpose_sum8(const c128 v[8], int lane) {
    c128 w4[4], w2[2];
#pragma unroll
    for (int u = 0; u < 4; ++u) w4[u] = fold_swap(v[u], v[4 + u], true);
#pragma unroll
    for (int u = 0; u < 2; ++u) w2[u] = fold_swap(w4[u], w4[2 + u], false);
    const c128 s0 = cadd(w2[0], dpp_c<kDppRor8>(w2[0]));
    const c128 s1 = cadd(w2[1], dpp_c<kDppRor8>(w2[1]));
    c128 w = (lane & 8) ? s1 : s0;
    w = cadd(w, dpp_c<kDppHalfMirror>(w));
    w = cadd(w, dpp_c<kDppQuadXor1>(w));
    return cadd(w, dpp_c<kDppQuadXor2>(w));
}

__device__ __forceinline__ c128 wave_sum_c(c128 w) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) w = cadd(w, shfl_xor_c(w, o));
    return w;
}

// Pass 1: one wave per item (8 columns of a Q panel), four items per workgroup.  Rows past the
// panel re-read its last row and meet x = 0; columns past ncols re-read the last column and are
// not stored.  The next 64-row chunk's loads are issued before the current chunk's FMAs.
template <typename F>
__global__ void __launch_bounds__(256) k_qtphase(const QtItem* __restrict__ items, int64_t nitems,
                                                 const F* __restrict__ fac, const c128* __restrict__ x,
                                                 c128* __restrict__ S) {
    const int lane = threadIdx.x & 63;
    const int64_t it = (int64_t)blockIdx.x * 4 + wave_id();
    if (it >= nitems) return;
    const QtItem q = items[it];
    const F* col[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) col[u] = fac + q.a_off + (int64_t)min(u, q.ncols - 1) * q.ld;
    const int nch = (q.nrows + 63) / 64;
    const c128* xv = x + q.x_off;
    c128 acc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] = make_double2(0.0, 0.0);
    auto load = [&](int ch, F a[8], c128& xr) {
        const int row = ch * 64 + lane;
        const int rr = min(row, q.nrows - 1);
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = load_stream(col[u] + rr);
        xr = row < q.nrows ? xv[rr] : make_double2(0.0, 0.0);
    };
    auto fmas = [&](const F a[8], c128 xr) {
#pragma unroll
        for (int u = 0; u < 8; ++u) cfma(acc[u], widen(a[u]), xr);
    };
    F a[8], b[8];
    c128 xa, xb;
    load(0, a, xa);
    int ch = 0;
    for (; ch + 2 < nch; ch += 2) {
        load(ch + 1, b, xb);
        __builtin_amdgcn_sched_barrier(0);
        fmas(a, xa);
        load(ch + 2, a, xa);
        __builtin_amdgcn_sched_barrier(0);
        fmas(b, xb);
    }
    if (ch + 1 < nch) {
        load(ch + 1, b, xb);
        __builtin_amdgcn_sched_barrier(0);
        fmas(a, xa);
        fmas(b, xb);
    } else {
        fmas(a, xa);
    }
    const c128 tot = transpose_sum8(acc, lane);
    const int c = lane >> 3;
    if ((lane & 7) == 0 && c < q.ncols) S[q.t_off + c] = tot;
}

// Pass 2: a strip of an R panel, four waves splitting its columns in whole batches of U.  Per
// batch: t += A x (per lane) and, per column, the wave's sum of A s (the strip's partial of the
// mirror product), reduced 8 columns at a time and stored by lanes 0, 8, ..., 56.
template <typename F, int WAVES>
__global__ void __launch_bounds__(64 * WAVES) k_rphase_sh(const RStrip* __restrict__ strips,
                                                          const F* __restrict__ fac, const c128* __restrict__ x,
                                                          c128* __restrict__ t, const int64_t* __restrict__ tmap,
                                                          const c128* __restrict__ S, c128* __restrict__ P) {
    constexpr int U = Unroll<F>::U;                  // 8 or 16: whole groups of 8 columns
    const RStrip s = strips[blockIdx.x];
    const int lane = threadIdx.x & 63, wv = wave_id();
    const int row = min(lane, s.nrows - 1);
    const c128 sv = lane < s.nrows ? S[tmap[s.tmap_off + lane]] : make_double2(0.0, 0.0);
    int j0, j1;
    wave_columns<U>(s.ncols, WAVES, wv, j0, j1);
    const F* A = fac + s.a_off + row;
    const c128* xv = x + s.x_off;
    c128* pr = P + s.p_off;
    c128 acc0 = make_double2(0.0, 0.0), acc1 = acc0;
    const int nb = (j1 - j0) / U;
    stream_batches<F, U>(A + (int64_t)j0 * s.ld, s.ld, nb, [&](const F* w, int k) {
        const int jb = j0 + k * U;
        const c128* vv = xv + jb;
#pragma unroll
        for (int h = 0; h < U; h += 8) {
            // the eight products are folded as soon as they exist (columns p, p + 4, p + 2, p + 6
            // into w2[p]), so few of them are live at once
            c128 w2[2];
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                c128 f[2];
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    const int u = p + 2 * r;
                    const c128 a0 = widen(w[h + u]), a1 = widen(w[h + u + 4]);
                    cfma(acc0, a0, vv[h + u]);
                    cfma(acc1, a1, vv[h + u + 4]);
                    f[r] = fold_swap(cmul(a0, sv), cmul(a1, sv), true);
                }
                w2[p] = fold_swap(f[0], f[1], false);
            }
            const c128 tot = transpose_sum2(w2, lane);
            if ((lane & 7) == 0) pr[jb + h + (lane >> 3)] = tot;
        }
    });
    for (int j = j0 + nb * U; j < j1; ++j) {          // columns past whole batches (not for 144-wide nodes)
        const c128 a = widen(A[(int64_t)j * s.ld]);
        cfma(acc0, a, xv[j]);
        const c128 tot = wave_sum_c(cmul(a, sv));
        if (lane == 0) pr[j] = tot;
    }
    const c128 acc = make_double2(acc0.x + acc1.x, acc0.y + acc1.y);
    __shared__ c128 red[WAVES][64];
    red[wv][lane] = acc;
    __syncthreads();
    if (wv == 0 && lane < s.nrows) {
        c128 sum = red[0][lane];
#pragma unroll
        for (int w = 1; w < WAVES; ++w) sum = cadd(sum, red[w][lane]);
        t[tmap[s.tmap_off + lane]] = sum;
    }
}

// Pass 3: the Q phase with the mirror partials of the strip's rows added in a fixed order.
template <typename F, int WAVES>
__global__ void __launch_bounds__(64 * WAVES) k_qphase_sh(const QStrip* __restrict__ strips,
                                                          const F* __restrict__ fac, const c128* __restrict__ t,
                                                          const c128* __restrict__ P, c128* __restrict__ y) {
    const QStrip s = strips[blockIdx.x];
    const int lane = threadIdx.x & 63, wv = wave_id();
    const int row = min(lane, max(s.nrows - 1, 0));
    int j0, j1;
    wave_columns<Unroll<F>::U>(s.ncols, WAVES, wv, j0, j1);
    const c128 acc = column_stream<F>(fac + s.a_off + row, s.ld, t + s.t_off, j0, j1);
    __shared__ c128 red[WAVES][64];
    red[wv][lane] = acc;
    __syncthreads();
    if (wv == 0 && lane < s.nrows) {
        c128 sum = red[0][lane];
#pragma unroll
        for (int w = 1; w < WAVES; ++w) sum = cadd(sum, red[w][lane]);
        for (int k = 0; k < s.p_cnt; ++k) sum = cadd(sum, P[s.p_off + (int64_t)k * s.p_ld + lane]);
        y[s.y_off + lane] = sum;
    }
}

// 576 threads per particle: thread -> (row = tid % 144, column group = tid / 144).
constexpr int kGroups = 4;
constexpr int kColsPerGroup = kNp / kGroups;

__device__ __forceinline__ c128 block_row_product(const c128* __restrict__ M, const c128* vin, int row, int grp) {
    c128 acc = make_double2(0.0, 0.0);
    const c128* a = M + row + (int64_t)grp * kColsPerGroup * kNp;
#pragma unroll 6
    for (int j = 0; j < kColsPerGroup; ++j) cfma(acc, a[(int64_t)j * kNp], vin[grp * kColsPerGroup + j]);
    return acc;
}

__global__ void __launch_bounds__(kNp * kGroups) k_final(const int32_t* __restrict__ ptype, const c128* __restrict__ self,
                                                         const c128* __restrict__ pinv, const c128* __restrict__ x,
                                                         const c128* __restrict__ ylev, int nlev, int64_t n,
                                                         const c128* __restrict__ v, c128* __restrict__ out_r,
                                                         c128* __restrict__ out_z) {
    const int p = blockIdx.x;
    const int tid = threadIdx.x;
    const int row = tid % kNp, grp = tid / kNp;
    const int64_t base = (int64_t)p * kNp;
    const int ty = ptype[p];
    __shared__ c128 vin[kNp];
    __shared__ c128 part[kGroups][kNp];
    if (tid < kNp) vin[tid] = x[base + tid];
    __syncthreads();
    part[grp][row] = block_row_product(self + (size_t)ty * kNp * kNp, vin, row, grp);
    __syncthreads();
    if (tid < kNp) {
        c128 y = part[0][row];
#pragma unroll
        for (int g = 1; g < kGroups; ++g) y = make_double2(y.x + part[g][row].x, y.y + part[g][row].y);
        for (int l = 0; l < nlev; ++l) {
            const c128 a = ylev[(int64_t)l * n + base + row];
            y = make_double2(y.x + a.x, y.y + a.y);
        }
        if (v) {
            const c128 b = v[base + row];
            y = make_double2(b.x - y.x, b.y - y.y);
        }
        if (out_r) out_r[base + row] = y;
        vin[row] = y;
    }
    if (!out_z) return;
    __syncthreads();
    part[grp][row] = block_row_product(pinv + (size_t)ty * kNp * kNp, vin, row, grp);
    __syncthreads();
    if (tid < kNp) {
        c128 z = part[0][row];
#pragma unroll
        for (int g = 1; g < kGroups; ++g) z = make_double2(z.x + part[g][row].x, z.y + part[g][row].y);
        out_z[base + row] = z;
    }
}

// y_p = M_type(p) x_p for every particle (the standalone preconditioner).
__global__ void __launch_bounds__(kNp * kGroups) k_block_apply(const int32_t* __restrict__ ptype,
                                                               const c128* __restrict__ mats, const c128* __restrict__ x,
                                                               c128* __restrict__ y) {
    const int p = blockIdx.x;
    const int tid = threadIdx.x;
    const int row = tid % kNp, grp = tid / kNp;
    const int64_t base = (int64_t)p * kNp;
    __shared__ c128 vin[kNp];
    __shared__ c128 part[kGroups][kNp];
    if (tid < kNp) vin[tid] = x[base + tid];
    __syncthreads();
    part[grp][row] = block_row_product(mats + (size_t)ptype[p] * kNp * kNp, vin, row, grp);
    __syncthreads();
    if (tid < kNp) {
        c128 z = part[0][row];
#pragma unroll
        for (int g = 1; g < kGroups; ++g) z = make_double2(z.x + part[g][row].x, z.y + part[g][row].y);
        y[base + row] = z;
    }
}

// ------------------------------------------------------------------ many right-hand sides
// Blocks of NR vectors are stored RHS-interleaved (element (e, r) at e * NR + r), so the
// NR entries a lane needs for one column are one contiguous wave-uniform row.  Each
// factor element is loaded once and applied to all NR vectors: the streaming pattern and
// the HBM bytes of the factors are those of the single-RHS product.
template <typename F> struct UnrollM { static constexpr int U = sizeof(F) == 16 ? 4 : 8; };

template <typename F, int NR>
__device__ __forceinline__ void column_stream_m(const F* __restrict__ A, int64_t ld, const c128* __restrict__ v,
                                                int j0, int j1, c128 acc[NR]) {
    constexpr int U = UnrollM<F>::U;
    const int nb = (j1 - j0) / U;
    stream_batches<F, U>(A + (int64_t)j0 * ld, ld, nb, [&](const F* w, int k) {
        const c128* vv = v + (int64_t)(j0 + k * U) * NR;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const c128 m = widen(w[u]);
#pragma unroll
            for (int r = 0; r < NR; ++r) cfma(acc[r], m, vv[u * NR + r]);
        }
    });
    for (int j = j0 + nb * U; j < j1; ++j) {
        const c128 m = widen(A[(int64_t)j * ld]);
#pragma unroll
        for (int r = 0; r < NR; ++r) cfma(acc[r], m, v[(int64_t)j * NR + r]);
    }
}

template <typename F, int NR>
__device__ __forceinline__ void rphase_m_body(const RStrip& s, const F* __restrict__ fac, const c128* __restrict__ X,
                                              c128* __restrict__ T, const int64_t* __restrict__ tmap) {
    const int lane = threadIdx.x & 63, wv = wave_id();
    const int row = min(lane, s.nrows - 1);
    int j0, j1;
    wave_columns<UnrollM<F>::U>(s.ncols, 4, wv, j0, j1);
    c128 acc[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = make_double2(0.0, 0.0);
    column_stream_m<F, NR>(fac + s.a_off + row, s.ld, X + (int64_t)s.x_off * NR, j0, j1, acc);
    __shared__ c128 red[4][64 * NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) red[wv][lane * NR + r] = acc[r];
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * NR; e += 256) {
        const int l = e / NR, r = e % NR;
        if (l < s.nrows) {
            c128 sum = red[0][e];
#pragma unroll
            for (int w = 1; w < 4; ++w) sum = make_double2(sum.x + red[w][e].x, sum.y + red[w][e].y);
            T[tmap[s.tmap_off + l] * NR + r] = sum;
        }
    }
}

template <int NR>
__global__ void __launch_bounds__(256) k_rphase_m(const RStrip* __restrict__ strips, const c128* __restrict__ fac,
                                                  const c128* __restrict__ X, c128* __restrict__ T,
                                                  const int64_t* __restrict__ tmap) {
    rphase_m_body<c128, NR>(strips[blockIdx.x], fac, X, T, tmap);
}
template <int NR>
__global__ void __launch_bounds__(256) k_rphase_m_c64(const RStrip* __restrict__ strips, const float2* __restrict__ fac,
                                                      const c128* __restrict__ X, c128* __restrict__ T,
                                                      const int64_t* __restrict__ tmap) {
    rphase_m_body<float2, NR>(strips[blockIdx.x], fac, X, T, tmap);
}

template <typename F, int NR>
__device__ __forceinline__ void qphase_m_body(const QStrip& s, const F* __restrict__ fac, const c128* __restrict__ T,
                                              c128* __restrict__ Y) {
    const int lane = threadIdx.x & 63, wv = wave_id();
    const int row = min(lane, max(s.nrows - 1, 0));
    int j0, j1;
    wave_columns<UnrollM<F>::U>(s.ncols, 4, wv, j0, j1);
    c128 acc[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = make_double2(0.0, 0.0);
    column_stream_m<F, NR>(fac + s.a_off + row, s.ld, T + s.t_off * NR, j0, j1, acc);
    __shared__ c128 red[4][64 * NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) red[wv][lane * NR + r] = acc[r];
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * NR; e += 256) {
        const int l = e / NR, r = e % NR;
        if (l < s.nrows) {
            c128 sum = red[0][e];
#pragma unroll
            for (int w = 1; w < 4; ++w) sum = make_double2(sum.x + red[w][e].x, sum.y + red[w][e].y);
            Y[(s.y_off + l) * NR + r] = sum;
        }
    }
}

template <int NR>
__global__ void __launch_bounds__(256) k_qphase_m(const QStrip* __restrict__ strips, const c128* __restrict__ fac,
                                                  const c128* __restrict__ T, c128* __restrict__ Y) {
    qphase_m_body<c128, NR>(strips[blockIdx.x], fac, T, Y);
}
template <int NR>
__global__ void __launch_bounds__(256) k_qphase_m_c64(const QStrip* __restrict__ strips, const float2* __restrict__ fac,
                                                      const c128* __restrict__ T, c128* __restrict__ Y) {
    qphase_m_body<float2, NR>(strips[blockIdx.x], fac, T, Y);
}

// Per particle: Y = Z_pp X + sum_l Y_l for NR interleaved vectors; optionally R = V - Y and
// Z = Z_pp^-1 R.  576 threads: row = tid % 144, column group = tid / 144.
template <int NR>
__global__ void __launch_bounds__(kNp * kGroups) k_final_m(const int32_t* __restrict__ ptype,
                                                           const c128* __restrict__ self, const c128* __restrict__ pinv,
                                                           const c128* __restrict__ X, const c128* __restrict__ ylev,
                                                           int nlev, int64_t n, const c128* __restrict__ V,
                                                           c128* __restrict__ out_r, c128* __restrict__ out_z) {
    const int p = blockIdx.x;
    const int tid = threadIdx.x;
    const int row = tid % kNp, grp = tid / kNp;
    const int64_t base = (int64_t)p * kNp;
    const int ty = ptype[p];
    __shared__ c128 vin[kNp * NR];
    __shared__ c128 part[kGroups][kNp * NR];
    for (int e = tid; e < kNp * NR; e += kNp * kGroups) vin[e] = X[base * NR + e];
    __syncthreads();
    auto product = [&](const c128* M) {
        c128 acc[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) acc[r] = make_double2(0.0, 0.0);
        const c128* a = M + row + (int64_t)grp * kColsPerGroup * kNp;
        for (int j = 0; j < kColsPerGroup; ++j) {
            const c128 m = a[(int64_t)j * kNp];
            const c128* vv = vin + (grp * kColsPerGroup + j) * NR;
#pragma unroll
            for (int r = 0; r < NR; ++r) cfma(acc[r], m, vv[r]);
        }
#pragma unroll
        for (int r = 0; r < NR; ++r) part[grp][row * NR + r] = acc[r];
    };
    product(self + (size_t)ty * kNp * kNp);
    __syncthreads();
    for (int e = tid; e < kNp * NR; e += kNp * kGroups) {
        c128 y = part[0][e];
#pragma unroll
        for (int g = 1; g < kGroups; ++g) y = make_double2(y.x + part[g][e].x, y.y + part[g][e].y);
        for (int l = 0; l < nlev; ++l) {
            const c128 a = ylev[((int64_t)l * n + base) * NR + e];
            y = make_double2(y.x + a.x, y.y + a.y);
        }
        if (V) {
            const c128 b = V[base * NR + e];
            y = make_double2(b.x - y.x, b.y - y.y);
        }
        if (out_r) out_r[base * NR + e] = y;
        vin[e] = y;
    }
    if (!out_z) return;
    __syncthreads();
    product(pinv + (size_t)ty * kNp * kNp);
    __syncthreads();
    for (int e = tid; e < kNp * NR; e += kNp * kGroups) {
        c128 z = part[0][e];
#pragma unroll
        for (int g = 1; g < kGroups; ++g) z = make_double2(z.x + part[g][e].x, z.y + part[g][e].y);
        out_z[base * NR + e] = z;
    }
}

// Interleave NR columns (stride ld) into an RHS-interleaved block and back; `map`
// optionally permutes particles (caller <-> internal order).
template <int NR>
__global__ void k_interleave(int64_t n, const c128* const* __restrict__ cols, c128* __restrict__ blk, int ncols) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
#pragma unroll
    for (int r = 0; r < NR; ++r) blk[e * NR + r] = r < ncols ? cols[r][e] : make_double2(0.0, 0.0);
}
template <int NR>
__global__ void k_deinterleave(int64_t n, const c128* __restrict__ blk, c128* const* __restrict__ cols, int ncols) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
#pragma unroll
    for (int r = 0; r < NR; ++r)
        if (r < ncols) cols[r][e] = blk[e * NR + r];
}

}  // namespace

// Round the complex128 panels to complex64 (round to nearest even).
// Grid-stride, so any panel size fits one launch.
__global__ void k_to_c64(const c128* __restrict__ in, float2* __restrict__ out, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride)
        out[e] = make_float2((float)in[e].x, (float)in[e].y);
}

// BF16 (8-bit mantissa) of an FP32 value, round to nearest even; NaN stays a quiet NaN.
__device__ __forceinline__ unsigned short f32_to_bf16(float f) {
    const unsigned u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (unsigned short)((u >> 16) | 0x40);
    return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__global__ void k_to_bf16(const float2* __restrict__ in, uint16_t* __restrict__ out, int64_t n, int64_t plane) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        const float2 v = in[e];
        out[e] = f32_to_bf16(v.x);
        out[plane + e] = f32_to_bf16(v.y);
    }
}
void launch_to_bf16(hipStream_t s, const float2* in, uint16_t* out, int64_t n, int64_t plane) {
    if (n <= 0) return;
    const int64_t want = (n + 255) / 256, blocks = want < (1 << 20) ? want : (1 << 20);
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)blocks), dim3(256), 0, s, in, out, n, plane);
}

void launch_to_c64(hipStream_t s, const c128* in, float2* out, int64_t n) {
    if (n <= 0) return;
    const int64_t want = (n + 255) / 256, blocks = want < (1 << 20) ? want : (1 << 20);
    hipLaunchKernelGGL(k_to_c64, dim3((unsigned)blocks), dim3(256), 0, s, in, out, n);
}
void launch_rphase_c64(hipStream_t s, const RStrip* st, int64_t n, const float2* fac, const c128* x, c128* t,
                       const int64_t* tmap) {
    if (n > 0) hipLaunchKernelGGL(k_rphase_c64<4>, dim3((unsigned)n), dim3(256), 0, s, st, fac, x, t, tmap);
}
void launch_qphase_c64(hipStream_t s, const QStrip* st, int64_t n, const float2* fac, const c128* t, c128* y) {
    if (n > 0) hipLaunchKernelGGL(k_qphase_c64<4>, dim3((unsigned)n), dim3(256), 0, s, st, fac, t, y);
}
void launch_rphase_m_c64(hipStream_t s, int nr, const RStrip* st, int64_t n, const float2* fac, const c128* X, c128* T,
                         const int64_t* tmap) {
    if (n <= 0) return;
    dim3 g((unsigned)n);
    switch (nr) {
        case 2: hipLaunchKernelGGL(k_rphase_m_c64<2>, g, dim3(256), 0, s, st, fac, X, T, tmap); break;
        case 4: hipLaunchKernelGGL(k_rphase_m_c64<4>, g, dim3(256), 0, s, st, fac, X, T, tmap); break;
        default: hipLaunchKernelGGL(k_rphase_m_c64<8>, g, dim3(256), 0, s, st, fac, X, T, tmap); break;
    }
}
void launch_qphase_m_c64(hipStream_t s, int nr, const QStrip* st, int64_t n, const float2* fac, const c128* T, c128* Y) {
    if (n <= 0) return;
    dim3 g((unsigned)n);
    switch (nr) {
        case 2: hipLaunchKernelGGL(k_qphase_m_c64<2>, g, dim3(256), 0, s, st, fac, T, Y); break;
        case 4: hipLaunchKernelGGL(k_qphase_m_c64<4>, g, dim3(256), 0, s, st, fac, T, Y); break;
        default: hipLaunchKernelGGL(k_qphase_m_c64<8>, g, dim3(256), 0, s, st, fac, T, Y); break;
    }
}

void launch_rphase_m(hipStream_t s, int nr, const RStrip* st, int64_t n, const c128* fac, const c128* X, c128* T,
                     const int64_t* tmap) {
    if (n <= 0) return;
    dim3 g((unsigned)n);
    switch (nr) {
        case 2: hipLaunchKernelGGL(k_rphase_m<2>, g, dim3(256), 0, s, st, fac, X, T, tmap); break;
        case 4: hipLaunchKernelGGL(k_rphase_m<4>, g, dim3(256), 0, s, st, fac, X, T, tmap); break;
        default: hipLaunchKernelGGL(k_rphase_m<8>, g, dim3(256), 0, s, st, fac, X, T, tmap); break;
    }
}
void launch_qphase_m(hipStream_t s, int nr, const QStrip* st, int64_t n, const c128* fac, const c128* T, c128* Y) {
    if (n <= 0) return;
    dim3 g((unsigned)n);
    switch (nr) {
        case 2: hipLaunchKernelGGL(k_qphase_m<2>, g, dim3(256), 0, s, st, fac, T, Y); break;
        case 4: hipLaunchKernelGGL(k_qphase_m<4>, g, dim3(256), 0, s, st, fac, T, Y); break;
        default: hipLaunchKernelGGL(k_qphase_m<8>, g, dim3(256), 0, s, st, fac, T, Y); break;
    }
}
void launch_final_m(hipStream_t s, int nr, int32_t N, const int32_t* ptype, const c128* self, const c128* pinv,
                    const c128* X, const c128* ylev, int nlev, int64_t n, const c128* V, c128* out_r, c128* out_z) {
    dim3 g(N), b(kNp * kGroups);
    switch (nr) {
        case 2: hipLaunchKernelGGL(k_final_m<2>, g, b, 0, s, ptype, self, pinv, X, ylev, nlev, n, V, out_r, out_z); break;
        case 4: hipLaunchKernelGGL(k_final_m<4>, g, b, 0, s, ptype, self, pinv, X, ylev, nlev, n, V, out_r, out_z); break;
        default: hipLaunchKernelGGL(k_final_m<8>, g, b, 0, s, ptype, self, pinv, X, ylev, nlev, n, V, out_r, out_z); break;
    }
}
void launch_interleave(hipStream_t s, int nr, int64_t n, const c128* const* cols, c128* blk, int ncols) {
    dim3 g((unsigned)((n + 255) / 256));
    switch (nr) {
        case 2: hipLaunchKernelGGL(k_interleave<2>, g, dim3(256), 0, s, n, cols, blk, ncols); break;
        case 4: hipLaunchKernelGGL(k_interleave<4>, g, dim3(256), 0, s, n, cols, blk, ncols); break;
        default: hipLaunchKernelGGL(k_interleave<8>, g, dim3(256), 0, s, n, cols, blk, ncols); break;
    }
}
void launch_deinterleave(hipStream_t s, int nr, int64_t n, const c128* blk, c128* const* cols, int ncols) {
    dim3 g((unsigned)((n + 255) / 256));
    switch (nr) {
        case 2: hipLaunchKernelGGL(k_deinterleave<2>, g, dim3(256), 0, s, n, blk, cols, ncols); break;
        case 4: hipLaunchKernelGGL(k_deinterleave<4>, g, dim3(256), 0, s, n, blk, cols, ncols); break;
        default: hipLaunchKernelGGL(k_deinterleave<8>, g, dim3(256), 0, s, n, blk, cols, ncols); break;
    }
}

void launch_rphase(hipStream_t s, const RStrip* st, int64_t n, int waves, const c128* fac, const c128* x, c128* t,
                   const int64_t* tmap) {
    if (n <= 0) return;
    dim3 g((unsigned)n);
    switch (waves) {
        case 1: hipLaunchKernelGGL(k_rphase<1>, g, dim3(64), 0, s, st, fac, x, t, tmap); break;
        case 2: hipLaunchKernelGGL(k_rphase<2>, g, dim3(128), 0, s, st, fac, x, t, tmap); break;
        case 4: hipLaunchKernelGGL(k_rphase<4>, g, dim3(256), 0, s, st, fac, x, t, tmap); break;
        case 8: hipLaunchKernelGGL(k_rphase<8>, g, dim3(512), 0, s, st, fac, x, t, tmap); break;
        default: hipLaunchKernelGGL(k_rphase<16>, g, dim3(1024), 0, s, st, fac, x, t, tmap); break;
    }
}

void launch_qphase(hipStream_t s, const QStrip* st, int64_t n, int waves, const c128* fac, const c128* t, c128* y) {
    if (n <= 0) return;
    dim3 g((unsigned)n);
    switch (waves) {
        case 1: hipLaunchKernelGGL(k_qphase<1>, g, dim3(64), 0, s, st, fac, t, y); break;
        case 2: hipLaunchKernelGGL(k_qphase<2>, g, dim3(128), 0, s, st, fac, t, y); break;
        case 4: hipLaunchKernelGGL(k_qphase<4>, g, dim3(256), 0, s, st, fac, t, y); break;
        case 8: hipLaunchKernelGGL(k_qphase<8>, g, dim3(512), 0, s, st, fac, t, y); break;
        default: hipLaunchKernelGGL(k_qphase<16>, g, dim3(1024), 0, s, st, fac, t, y); break;
    }
}

void launch_qtphase(hipStream_t s, const QtItem* it, int64_t n, const c128* fac, const c128* x, c128* S) {
    if (n > 0) hipLaunchKernelGGL(k_qtphase<c128>, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, it, n, fac, x, S);
}
void launch_qtphase(hipStream_t s, const QtItem* it, int64_t n, const float2* fac, const c128* x, c128* S) {
    if (n > 0) hipLaunchKernelGGL(k_qtphase<float2>, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, it, n, fac, x, S);
}
void launch_rphase_sh(hipStream_t s, const RStrip* st, int64_t n, const c128* fac, const c128* x, c128* t,
                      const int64_t* tmap, const c128* S, c128* P) {
    if (n > 0)
        hipLaunchKernelGGL((k_rphase_sh<c128, 4>), dim3((unsigned)n), dim3(256), 0, s, st, fac, x, t, tmap, S, P);
}
void launch_rphase_sh(hipStream_t s, const RStrip* st, int64_t n, const float2* fac, const c128* x, c128* t,
                      const int64_t* tmap, const c128* S, c128* P) {
    if (n > 0)
        hipLaunchKernelGGL((k_rphase_sh<float2, 4>), dim3((unsigned)n), dim3(256), 0, s, st, fac, x, t, tmap, S, P);
}
void launch_qphase_sh(hipStream_t s, const QStrip* st, int64_t n, const c128* fac, const c128* t, const c128* P,
                      c128* y) {
    if (n > 0) hipLaunchKernelGGL((k_qphase_sh<c128, 4>), dim3((unsigned)n), dim3(256), 0, s, st, fac, t, P, y);
}
void launch_qphase_sh(hipStream_t s, const QStrip* st, int64_t n, const float2* fac, const c128* t, const c128* P,
                      c128* y) {
    if (n > 0) hipLaunchKernelGGL((k_qphase_sh<float2, 4>), dim3((unsigned)n), dim3(256), 0, s, st, fac, t, P, y);
}

void launch_final(hipStream_t s, int32_t N, const int32_t* ptype, const c128* self, const c128* pinv, const c128* x,
                  const c128* ylev, int nlev, int64_t n, const c128* v, c128* out_r, c128* out_z) {
    hipLaunchKernelGGL(k_final, dim3(N), dim3(kNp * kGroups), 0, s, ptype, self, pinv, x, ylev, nlev, n, v, out_r, out_z);
}

void launch_block_apply(hipStream_t s, int32_t N, const int32_t* ptype, const c128* mats, const c128* x, c128* y) {
    hipLaunchKernelGGL(k_block_apply, dim3(N), dim3(kNp * kGroups), 0, s, ptype, mats, x, y);
}

}  // namespace qrvie
