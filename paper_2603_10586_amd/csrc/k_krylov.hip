// Krylov building blocks of left-preconditioned GMRES (the paper's solver of §6 with
// the preconditioner of §4): Gram-Schmidt projections as multi-dot / multi-axpy kernels
// over the column-major basis V (n x (m+1)) with the vector norms fused in, and the
// Hessenberg least-squares update by complex Givens rotations, all in FP64 on the device.
// Reductions are two-stage with a fixed order, so results are bitwise reproducible.
//
// Orthogonalisation is classical Gram-Schmidt with one reorthogonalisation (CGS2) in two
// passes over the basis instead of four.  With h1 = V^H w, the second projection
// V^H (w - V h1) equals h1 - G h1 for the Gram matrix G = V^H V of the stored basis, so
// CGS2's coefficients are h = 2 h1 - G h1 and its vector is w - V h.  G gains one column
// per step (V^H v_j, computed in the same pass as V^H w), and G h1 is a small
// (j+1) x (j+1) product.  The result equals CGS2 up to rounding: in both, the component
// of the new vector left along the basis is (I - G)^2 h1.
#include "stream.h"

namespace qrvie {

namespace {

constexpr int kChunk = 1024;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double block_sum(double v, double* red) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

// partial[c * ncols + i] = sum_{e in chunk c} conj(V_i[e]) w[e], and the same with u into
// upartial when u is given (two projections per pass over V).  Grid: (row chunks of 1024,
// groups of 64 basis vectors).  The w (and u) chunk is staged in LDS, zero past n; a wave
// issues all 16 loads of one basis vector's chunk before its FMAs (rows past n re-read
// row n-1 and meet a zero).
constexpr int kPerLane = kChunk / 64;
constexpr int kVecGroup = 64;

template <bool TWO>
__global__ void __launch_bounds__(256) k_multidot(const c128* __restrict__ V, int64_t ldv, int ncols,
                                                  const c128* __restrict__ w, const c128* __restrict__ u, int64_t n,
                                                  c128* __restrict__ partial, c128* __restrict__ upartial) {
    __shared__ c128 ws[kChunk];
    __shared__ c128 us[TWO ? kChunk : 1];
    const int c = blockIdx.x;
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t e0 = (int64_t)c * kChunk;
    const int cnt = (n - e0) < kChunk ? (int)(n - e0) : kChunk;
    for (int o = threadIdx.x; o < kChunk; o += 256) {
        ws[o] = o < cnt ? w[e0 + o] : make_double2(0.0, 0.0);
        if (TWO) us[o] = o < cnt ? u[e0 + o] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const int i1 = min(ncols, (int)(blockIdx.y + 1) * kVecGroup);
    for (int i = blockIdx.y * kVecGroup + wv; i < i1; i += 4) {
        const c128* vi = V + (int64_t)i * ldv + e0;
        c128 a[kPerLane];
#pragma unroll
        for (int t = 0; t < kPerLane; ++t) a[t] = load_stream(vi + min(lane + 64 * t, cnt - 1));
        __builtin_amdgcn_sched_barrier(0);
        double re0 = 0.0, im0 = 0.0, re1 = 0.0, im1 = 0.0;
#pragma unroll
        for (int t = 0; t < kPerLane; ++t) {
            const c128 x = ws[lane + 64 * t];
            re0 = fma(a[t].x, x.x, fma(a[t].y, x.y, re0));
            im0 = fma(a[t].x, x.y, fma(-a[t].y, x.x, im0));
            if (TWO) {
                const c128 y = us[lane + 64 * t];
                re1 = fma(a[t].x, y.x, fma(a[t].y, y.y, re1));
                im1 = fma(a[t].x, y.y, fma(-a[t].y, y.x, im1));
            }
        }
        const double re = wave_sum(re0), im = wave_sum(im0);
        if (lane == 0) partial[(int64_t)c * ncols + i] = make_double2(re, im);
        if (TWO) {
            const double ur = wave_sum(re1), ui = wave_sum(im1);
            if (lane == 0) upartial[(int64_t)c * ncols + i] = make_double2(ur, ui);
        }
    }
}

// h[i] = sum_c partial[c * ncols + i]; when mirror is given, also mirror[i * mstride] =
// conj(h[i]) for i < ncols - 1 (the row of a Hermitian matrix whose column is h).
__global__ void k_reduce_dots(const c128* __restrict__ partial, int nchunks, int ncols, c128* h, c128* mirror,
                              int64_t mstride) {
    const int i = threadIdx.x + blockIdx.x * blockDim.x;
    if (i >= ncols) return;
    double re = 0.0, im = 0.0;
#pragma unroll 8
    for (int c = 0; c < nchunks; ++c) {
        const c128 p = partial[(int64_t)c * ncols + i];
        re += p.x;
        im += p.y;
    }
    h[i] = make_double2(re, im);
    if (mirror && i < ncols - 1) mirror[(int64_t)i * mstride] = make_double2(re, -im);
}

// h[i] = 2 h1[i] - sum_c partial[c * ncols + i]  (CGS2 coefficients from G h1 partials)
__global__ void k_cgs2_coeffs(const c128* __restrict__ partial, int nchunks, int ncols, c128* h) {
    const int i = threadIdx.x + blockIdx.x * blockDim.x;
    if (i >= ncols) return;
    double re = 0.0, im = 0.0;
    for (int c = 0; c < nchunks; ++c) {
        const c128 p = partial[(int64_t)c * ncols + i];
        re += p.x;
        im += p.y;
    }
    h[i] = make_double2(2.0 * h[i].x - re, 2.0 * h[i].y - im);
}

// w += SIGN * V h; npart[block] = ||w_block||^2 after (when given).  One row per lane and one
// wave per workgroup: every wave streams all the basis columns for its 64 rows, so n / 64
// equal workgroups spread evenly over the compute units (n / 256 four-wave groups left some
// units a third more work than others).  The coefficients are wave-uniform scalar loads and the
// basis columns stream in double-buffered batches of 8 (rows past n re-read row n-1 and are
// not stored).
template <int SIGN>
__global__ void __launch_bounds__(64) k_gemv_acc(const c128* __restrict__ V, int64_t ldv, int ncols,
                                                 const c128* __restrict__ h, c128* __restrict__ w, int64_t n,
                                                 double* __restrict__ npart) {
    constexpr int U = 8;
    const int64_t e = (int64_t)blockIdx.x * 64 + threadIdx.x;
    const bool live = e < n;
    const int64_t row = live ? e : n - 1;
    c128 acc0 = live ? w[e] : make_double2(0.0, 0.0), acc1 = make_double2(0.0, 0.0);
    const int nb = ncols / U;
    stream_batches<c128, U>(V + row, ldv, nb, [&](const c128* a, int k) {
        const c128* hh = h + k * U;
#pragma unroll
        for (int u = 0; u < U; u += 2) {
            const c128 h0 = make_double2(SIGN * hh[u].x, SIGN * hh[u].y);
            const c128 h1 = make_double2(SIGN * hh[u + 1].x, SIGN * hh[u + 1].y);
            cfma(acc0, a[u], h0);
            cfma(acc1, a[u + 1], h1);
        }
    });
    for (int i = nb * U; i < ncols; ++i)
        cfma(acc0, V[row + (int64_t)i * ldv], make_double2(SIGN * h[i].x, SIGN * h[i].y));
    const double re = acc0.x + acc1.x, im = acc0.y + acc1.y;
    if (live) w[e] = make_double2(re, im);
    if (npart) {
        const double s = wave_sum(live ? re * re + im * im : 0.0);
        if (threadIdx.x == 0) npart[blockIdx.x] = s;
    }
}

__global__ void __launch_bounds__(256) k_norm2(const c128* __restrict__ w, int64_t n, double* __restrict__ partial) {
    const int c = blockIdx.x;
    const int64_t e0 = (int64_t)c * kChunk, e1 = min(n, e0 + kChunk);
    double s = 0.0;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) s = fma(w[e].x, w[e].x, fma(w[e].y, w[e].y, s));
    __shared__ double red[4];
    s = block_sum(s, red);
    if (threadIdx.x == 0) partial[c] = s;
}

__global__ void __launch_bounds__(256) k_reduce_norm(const double* __restrict__ partial, int count, double* out) {
    __shared__ double red[256];
    const int tid = threadIdx.x;
    double s = 0.0;
    for (int c = tid; c < count; c += 256) s += partial[c];
    red[tid] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) red[tid] += red[tid + o];
        __syncthreads();
    }
    if (tid == 0) out[0] = red[0];
}

// out = w / sqrt(norm2); gslot (optional) = sqrt(norm2)
__global__ void k_scale_into(const c128* __restrict__ w, int64_t n, const double* norm2, c128* __restrict__ out,
                             c128* gslot) {
    const double nr = sqrt(norm2[0]);
    const double inv = nr > 0.0 ? 1.0 / nr : 0.0;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e == 0 && gslot) gslot[0] = make_double2(nr, 0.0);
    if (e >= n) return;
    out[e] = make_double2(w[e].x * inv, w[e].y * inv);
}

// Loss of orthogonality of the first k basis vectors, max_ij |G_ij - delta_ij| over the Gram
// matrix G = V^H V that the projections maintain, folded into *out (a non-negative double
// kept as its bit pattern, so the maximum is an exact, order-independent integer max).
__global__ void __launch_bounds__(256) k_gram_deviation(const c128* __restrict__ G, int64_t ldg, int k,
                                                        unsigned long long* out) {
    double m = 0.0;
    const int64_t tot = (int64_t)k * k;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256) {
        const int64_t i = e % k, j = e / k;
        const c128 g = G[i + j * ldg];
        const double re = g.x - (i == j ? 1.0 : 0.0);
        m = fmax(m, sqrt(re * re + g.y * g.y));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(out, (unsigned long long)__double_as_longlong(m));
}

// x += d (the update of an iterative-refinement step)
// Streaming read of n 16-byte entries with the product kernels' nontemporal loads, U loads
// in flight per lane, grid-stride; the sum is kept only so that the loads are not removed.
template <int U>
__global__ void __launch_bounds__(256) k_read_probe(const c128* __restrict__ p, int64_t n, double* out) {
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * 256;
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    for (; i + (U - 1) * stride < n; i += U * stride) {
        c128 a[U];
#pragma unroll
        for (int u = 0; u < U; ++u) a[u] = load_stream(p + i + u * stride);
#pragma unroll
        for (int u = 0; u < U; ++u) acc += a[u].x + a[u].y;
    }
    for (; i < n; i += stride) acc += p[i].x + p[i].y;
    if (acc == -1.0) out[0] = acc;       // practically never: keeps the reads live
}

// Matrix-core rate reference: every wave runs `iters` rounds of eight independent 16x16x4
// MFMA chains (FP64 when F64, else FP32) on register data; 2048 flops per instruction.
typedef double p4d __attribute__((ext_vector_type(4)));
typedef float p4f __attribute__((ext_vector_type(4)));
template <bool F64>
__global__ void __launch_bounds__(256) k_mfma_probe(int iters, double* out) {
    const int lane = threadIdx.x & 63;
    if (F64) {
        p4d c[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) c[j] = p4d{0, 0, 0, 0};
        const double a = 1.0 + 1e-9 * lane, b = 1.0 - 1e-9 * lane;
        for (int i = 0; i < iters; ++i) {
#pragma unroll
            for (int j = 0; j < 8; ++j) c[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(j & 1 ? a : b, j & 2 ? a : b, c[j], 0, 0, 0);
        }
        double t = 0.0;
#pragma unroll
        for (int j = 0; j < 8; ++j) t += c[j][j & 3];
        if (t == -1.0) out[0] = t;
    } else {
        p4f c[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) c[j] = p4f{0, 0, 0, 0};
        const float a = 1.0f + 1e-6f * lane, b = 1.0f - 1e-6f * lane;
        for (int i = 0; i < iters; ++i) {
#pragma unroll
            for (int j = 0; j < 8; ++j) c[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(j & 1 ? a : b, j & 2 ? a : b, c[j], 0, 0, 0);
        }
        float t = 0.0f;
#pragma unroll
        for (int j = 0; j < 8; ++j) t += c[j][j & 3];
        if (t == -1.0f) out[0] = t;
    }
}

// y = a - y
__global__ void k_rsub(const c128* __restrict__ a, int64_t n, c128* __restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = make_double2(a[i].x - y[i].x, a[i].y - y[i].y);
}

__global__ void k_add(const c128* __restrict__ d, int64_t n, c128* __restrict__ x) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    x[e] = make_double2(x[e].x + d[e].x, x[e].y + d[e].y);
}

// Column j of the Hessenberg matrix: hcol[0..j] from Gram-Schmidt, h_{j+1,j} = sqrt(hnorm2).
// Apply the previous rotations, build rotation j so that [[c, s], [-conj(s), c]] zeroes
// h_{j+1,j} (c real), and rotate the right-hand side g.  status = {|g_{j+1}|, h_{j+1,j}}.
//
// Rotation t maps the running entry a_t and the next entry b_t = h_{t+1} to the output
// c_t a_t + s_t b_t and the next running entry a_{t+1} = -conj(s_t) a_t + c_t b_t, an affine
// recurrence in a.  One wave applies the j rotations as a scan: each lane composes the affine
// maps of its contiguous chunk, a 6-step shuffle scan gives every lane the running entry at
// the start of its chunk, and each lane then produces its chunk's outputs.  The critical path
// is about 2 j / 64 + 6 dependent steps instead of j.
__device__ __forceinline__ c128 cmul_k(c128 x, c128 y) {
    return make_double2(x.x * y.x - x.y * y.y, x.x * y.y + x.y * y.x);
}

__global__ void __launch_bounds__(256) k_givens(int j, c128* hcol, c128* H, int ldh, double* cs, c128* sn, c128* g,
                                                const double* hnorm2, double* status) {
    __shared__ c128 carry;
    const int tid = threadIdx.x;
    const double hn = sqrt(hnorm2[0]);
    c128* Hj = H + (int64_t)j * ldh;
    if (tid < 64) {
        const int lane = tid;
        const int len = (j + 63) / 64;
        const int t0 = min(j, lane * len), t1 = min(j, t0 + len);
        // compose this chunk's maps a -> A a + B
        c128 A = make_double2(1.0, 0.0), B = make_double2(0.0, 0.0);
        for (int t = t0; t < t1; ++t) {
            const c128 st = sn[t];
            const double ct = cs[t];
            const c128 al = make_double2(-st.x, st.y);               // -conj(s)
            const c128 bt = hcol[t + 1];
            B = cmul_k(al, B);
            B = make_double2(B.x + ct * bt.x, B.y + ct * bt.y);
            A = cmul_k(al, A);
        }
        // inclusive scan of the maps over the lanes (lane l: chunks 0..l composed)
        for (int o = 1; o < 64; o <<= 1) {
            const c128 Ao = make_double2(__shfl_up(A.x, o, 64), __shfl_up(A.y, o, 64));
            const c128 Bo = make_double2(__shfl_up(B.x, o, 64), __shfl_up(B.y, o, 64));
            if (lane >= o) {                                          // mine after theirs
                const c128 nb = cmul_k(A, Bo);
                B = make_double2(nb.x + B.x, nb.y + B.y);
                A = cmul_k(A, Ao);
            }
        }
        // the running entry at the start of this chunk: the previous lanes' maps applied to h_0
        const c128 h0 = hcol[0];
        c128 Ap = make_double2(__shfl_up(A.x, 1, 64), __shfl_up(A.y, 1, 64));
        c128 Bp = make_double2(__shfl_up(B.x, 1, 64), __shfl_up(B.y, 1, 64));
        if (lane == 0) { Ap = make_double2(1.0, 0.0); Bp = make_double2(0.0, 0.0); }
        const c128 pa = cmul_k(Ap, h0);
        c128 a = make_double2(pa.x + Bp.x, pa.y + Bp.y);
        for (int t = t0; t < t1; ++t) {
            const c128 st = sn[t];
            const double ct = cs[t];
            const c128 bt = hcol[t + 1];
            const c128 sb = cmul_k(st, bt);
            const c128 out = make_double2(ct * a.x + sb.x, ct * a.y + sb.y);
            a = make_double2(-(st.x * a.x + st.y * a.y) + ct * bt.x, -(st.x * a.y - st.y * a.x) + ct * bt.y);
            Hj[t] = out;                // rotated entries go to H; hcol is only read
        }
        if (lane == 63) carry = j == 0 ? h0 : a;
    }
    __syncthreads();
    if (tid == 0) {
        const c128 a = carry, b = make_double2(hn, 0.0);
        const double aa = sqrt(a.x * a.x + a.y * a.y), ab = sqrt(b.x * b.x + b.y * b.y);
        double c;
        c128 s;
        if (ab == 0.0) { c = 1.0; s = make_double2(0.0, 0.0); }
        else if (aa == 0.0) { c = 0.0; s = make_double2(b.x / ab, -b.y / ab); }
        else {
            const double rho = hypot(aa, ab);
            c = aa / rho;
            const c128 ph = make_double2(a.x / aa, a.y / aa);
            // s = ph * conj(b) / rho
            s = make_double2((ph.x * b.x + ph.y * b.y) / rho, (ph.y * b.x - ph.x * b.y) / rho);
        }
        cs[j] = c;
        sn[j] = s;
        Hj[j] = make_double2(c * a.x + (s.x * b.x - s.y * b.y), c * a.y + (s.x * b.y + s.y * b.x));
        const c128 gj = g[j];
        g[j + 1] = make_double2(-(s.x * gj.x + s.y * gj.y), -(s.x * gj.y - s.y * gj.x));
        g[j] = make_double2(c * gj.x, c * gj.y);
        status[0] = sqrt(g[j + 1].x * g[j + 1].x + g[j + 1].y * g[j + 1].y);
        status[1] = hn;
    }
}

// Solve the k x k upper-triangular system H y = g by column sweeps (one workgroup):
// y_i = r_i / H_ii, then r_l -= H_li y_i for l < i in parallel.
__global__ void __launch_bounds__(256) k_trisolve(int k, const c128* H, int ldh, const c128* g, c128* y) {
    __shared__ c128 yi_s;
    for (int l = threadIdx.x; l < k; l += blockDim.x) y[l] = g[l];
    __syncthreads();
    for (int i = k - 1; i >= 0; --i) {
        if (threadIdx.x == 0) {
            const c128 r = y[i], d = H[i + (int64_t)i * ldh];
            const double den = d.x * d.x + d.y * d.y;
            const c128 v = make_double2((r.x * d.x + r.y * d.y) / den, (r.y * d.x - r.x * d.y) / den);
            y[i] = v;
            yi_s = v;
        }
        __syncthreads();
        const c128 v = yi_s;
        for (int l = threadIdx.x; l < i; l += blockDim.x) {
            const c128 h = H[l + (int64_t)i * ldh];
            y[l] = make_double2(y[l].x - (h.x * v.x - h.y * v.y), y[l].y - (h.x * v.y + h.y * v.x));
        }
        __syncthreads();
    }
}

}  // namespace

int krylov_nchunks(int64_t n) { return (int)((n + kChunk - 1) / kChunk); }
int krylov_nblocks(int64_t n) { return (int)((n + 63) / 64); }

void launch_multidot(hipStream_t s, const c128* V, int64_t ldv, int ncols, const c128* w, const c128* u, int64_t n,
                     c128* partial, c128* upartial) {
    dim3 grid(krylov_nchunks(n), (ncols + kVecGroup - 1) / kVecGroup);
    if (u) hipLaunchKernelGGL(k_multidot<true>, grid, dim3(256), 0, s, V, ldv, ncols, w, u, n, partial, upartial);
    else hipLaunchKernelGGL(k_multidot<false>, grid, dim3(256), 0, s, V, ldv, ncols, w, u, n, partial, upartial);
}
void launch_reduce_dots(hipStream_t s, const c128* partial, int nchunks, int ncols, c128* h, c128* mirror,
                        int64_t mstride) {
    hipLaunchKernelGGL(k_reduce_dots, dim3((ncols + 255) / 256), dim3(256), 0, s, partial, nchunks, ncols, h, mirror,
                       mstride);
}
void launch_cgs2_coeffs(hipStream_t s, const c128* partial, int nchunks, int ncols, c128* h) {
    hipLaunchKernelGGL(k_cgs2_coeffs, dim3((ncols + 255) / 256), dim3(256), 0, s, partial, nchunks, ncols, h);
}
void launch_gemv_sub(hipStream_t s, const c128* V, int64_t ldv, int ncols, const c128* h, c128* w, int64_t n,
                     double* npart) {
    hipLaunchKernelGGL(k_gemv_acc<-1>, dim3(krylov_nblocks(n)), dim3(64), 0, s, V, ldv, ncols, h, w, n, npart);
}
void launch_gemv_add(hipStream_t s, const c128* V, int64_t ldv, int ncols, const c128* y, c128* x, int64_t n) {
    hipLaunchKernelGGL(k_gemv_acc<1>, dim3(krylov_nblocks(n)), dim3(64), 0, s, V, ldv, ncols, y, x, n, nullptr);
}
void launch_norm2(hipStream_t s, const c128* w, int64_t n, double* partial) {
    hipLaunchKernelGGL(k_norm2, dim3(krylov_nchunks(n)), dim3(256), 0, s, w, n, partial);
}
void launch_reduce_norm(hipStream_t s, const double* partial, int count, double* out) {
    hipLaunchKernelGGL(k_reduce_norm, dim3(1), dim3(256), 0, s, partial, count, out);
}
void launch_scale_into(hipStream_t s, const c128* w, int64_t n, const double* norm2, c128* out, c128* gslot) {
    hipLaunchKernelGGL(k_scale_into, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, w, n, norm2, out, gslot);
}
void launch_gram_deviation(hipStream_t s, const c128* G, int64_t ldg, int k, double* out) {
    if (k <= 0) return;
    const int64_t tot = (int64_t)k * k;
    const unsigned grid = (unsigned)std::min<int64_t>(1024, (tot + 255) / 256);
    hipLaunchKernelGGL(k_gram_deviation, dim3(grid), dim3(256), 0, s, G, ldg, k,
                       reinterpret_cast<unsigned long long*>(out));
}
void launch_mfma_probe(hipStream_t s, bool f64, int grid, int iters, double* out) {
    if (f64) hipLaunchKernelGGL(k_mfma_probe<true>, dim3(grid), dim3(256), 0, s, iters, out);
    else hipLaunchKernelGGL(k_mfma_probe<false>, dim3(grid), dim3(256), 0, s, iters, out);
}
void launch_read_probe(hipStream_t s, const c128* p, int64_t n, int grid, int u, double* out) {
    if (u >= 16) hipLaunchKernelGGL(k_read_probe<16>, dim3(grid), dim3(256), 0, s, p, n, out);
    else hipLaunchKernelGGL(k_read_probe<8>, dim3(grid), dim3(256), 0, s, p, n, out);
}
void launch_rsub(hipStream_t s, const c128* a, int64_t n, c128* y) {
    hipLaunchKernelGGL(k_rsub, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, n, y);
}
void launch_add(hipStream_t s, const c128* d, int64_t n, c128* x) {
    hipLaunchKernelGGL(k_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d, n, x);
}
void launch_givens(hipStream_t s, int j, c128* hcol, c128* H, int ldh, double* cs, c128* sn, c128* g,
                   const double* hnorm2, double* status) {
    hipLaunchKernelGGL(k_givens, dim3(1), dim3(256), 0, s, j, hcol, H, ldh, cs, sn, g, hnorm2, status);
}
void launch_trisolve(hipStream_t s, int k, const c128* H, int ldh, const c128* g, c128* y) {
    hipLaunchKernelGGL(k_trisolve, dim3(1), dim3(256), 0, s, k, H, ldh, g, y);
}

}  // namespace qrvie
