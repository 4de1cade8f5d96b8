// Krylov building blocks of left-preconditioned restarted GMRES (the paper's solver
// of §6 with the preconditioner of §4): classical Gram-Schmidt passes as multi-dot /
// multi-axpy kernels over the column-major basis V (n x (m+1)), norms, and the
// Hessenberg least-squares update by complex Givens rotations, all in FP64 and on
// the device.  Reductions are two-stage with a fixed order (bitwise reproducible).
#include "internal.h"

namespace qrvie {

namespace {

constexpr int kChunk = 1024;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// partial[c * ncols + i] = sum_{e in chunk c} conj(V_i[e]) w[e]
__global__ void __launch_bounds__(256) k_multidot(const c128* __restrict__ V, int64_t ldv, int ncols,
                                                  const c128* __restrict__ w, int64_t n, c128* __restrict__ partial) {
    const int c = blockIdx.x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t e0 = (int64_t)c * kChunk, e1 = min(n, e0 + kChunk);
    for (int i = wv; i < ncols; i += 4) {
        const c128* vi = V + (int64_t)i * ldv;
        double re = 0.0, im = 0.0;
        for (int64_t e = e0 + lane; e < e1; e += 64) {
            const c128 a = vi[e], b = w[e];
            re = fma(a.x, b.x, fma(a.y, b.y, re));
            im = fma(a.x, b.y, fma(-a.y, b.x, im));
        }
        re = wave_sum(re);
        im = wave_sum(im);
        if (lane == 0) partial[(int64_t)c * ncols + i] = make_double2(re, im);
    }
}

__global__ void k_reduce_dots(const c128* __restrict__ partial, int nchunks, int ncols, c128* h, int accumulate) {
    const int i = threadIdx.x + blockIdx.x * blockDim.x;
    if (i >= ncols) return;
    double re = 0.0, im = 0.0;
    for (int c = 0; c < nchunks; ++c) {
        const c128 p = partial[(int64_t)c * ncols + i];
        re += p.x;
        im += p.y;
    }
    if (accumulate) { re += h[i].x; im += h[i].y; }
    h[i] = make_double2(re, im);
}

// w -= V h  (h length ncols)
__global__ void __launch_bounds__(256) k_gemv_sub(const c128* __restrict__ V, int64_t ldv, int ncols,
                                                  const c128* __restrict__ h, c128* __restrict__ w, int64_t n) {
    __shared__ c128 hs[512];
    for (int i = threadIdx.x; i < ncols; i += blockDim.x) hs[i] = h[i];
    __syncthreads();
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    double re = w[e].x, im = w[e].y;
    for (int i = 0; i < ncols; ++i) {
        const c128 a = V[e + (int64_t)i * ldv];
        re = fma(-a.x, hs[i].x, fma(a.y, hs[i].y, re));
        im = fma(-a.x, hs[i].y, fma(-a.y, hs[i].x, im));
    }
    w[e] = make_double2(re, im);
}

// x += V y
__global__ void __launch_bounds__(256) k_gemv_add(const c128* __restrict__ V, int64_t ldv, int ncols,
                                                  const c128* __restrict__ y, c128* __restrict__ x, int64_t n) {
    __shared__ c128 ys[512];
    for (int i = threadIdx.x; i < ncols; i += blockDim.x) ys[i] = y[i];
    __syncthreads();
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    double re = x[e].x, im = x[e].y;
    for (int i = 0; i < ncols; ++i) {
        const c128 a = V[e + (int64_t)i * ldv];
        re = fma(a.x, ys[i].x, fma(-a.y, ys[i].y, re));
        im = fma(a.x, ys[i].y, fma(a.y, ys[i].x, im));
    }
    x[e] = make_double2(re, im);
}

__global__ void __launch_bounds__(256) k_norm2(const c128* __restrict__ w, int64_t n, double* __restrict__ partial) {
    const int c = blockIdx.x;
    const int64_t e0 = (int64_t)c * kChunk, e1 = min(n, e0 + kChunk);
    double s = 0.0;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) s = fma(w[e].x, w[e].x, fma(w[e].y, w[e].y, s));
    __shared__ double red[4];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) partial[c] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void k_reduce_norm(const double* __restrict__ partial, int nchunks, double* out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int c = 0; c < nchunks; ++c) s += partial[c];
    out[0] = s;
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

// Column j of the Hessenberg matrix: hcol[0..j] from Gram-Schmidt, h_{j+1,j} = sqrt(hnorm2).
// Apply the previous rotations, build rotation j so that [[c, s], [-conj(s), c]] zeroes
// h_{j+1,j} (c real), and rotate the right-hand side g.  status = {|g_{j+1}|, h_{j+1,j}}.
__global__ void k_givens(int j, c128* hcol, c128* H, int ldh, double* cs, c128* sn, c128* g, const double* hnorm2,
                         double* status) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double hn = sqrt(hnorm2[0]);
    hcol[j + 1] = make_double2(hn, 0.0);
    for (int i = 0; i < j; ++i) {
        const c128 a = hcol[i], b = hcol[i + 1];
        const double c = cs[i];
        const c128 s = sn[i];
        // [c a + s b, -conj(s) a + c b]
        const c128 na = make_double2(c * a.x + (s.x * b.x - s.y * b.y), c * a.y + (s.x * b.y + s.y * b.x));
        const c128 nb = make_double2(-(s.x * a.x + s.y * a.y) + c * b.x, -(s.x * a.y - s.y * a.x) + c * b.y);
        hcol[i] = na;
        hcol[i + 1] = nb;
    }
    const c128 a = hcol[j], b = hcol[j + 1];
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
    hcol[j] = make_double2(c * a.x + (s.x * b.x - s.y * b.y), c * a.y + (s.x * b.y + s.y * b.x));
    hcol[j + 1] = make_double2(0.0, 0.0);
    for (int i = 0; i <= j; ++i) H[i + (int64_t)j * ldh] = hcol[i];
    const c128 gj = g[j];
    g[j + 1] = make_double2(-(s.x * gj.x + s.y * gj.y), -(s.x * gj.y - s.y * gj.x));
    g[j] = make_double2(c * gj.x, c * gj.y);
    status[0] = sqrt(g[j + 1].x * g[j + 1].x + g[j + 1].y * g[j + 1].y);
    status[1] = hn;
}

// Solve the k x k upper-triangular system H y = g.
__global__ void k_trisolve(int k, const c128* H, int ldh, const c128* g, c128* y) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (int i = k - 1; i >= 0; --i) {
        double re = g[i].x, im = g[i].y;
        for (int l = i + 1; l < k; ++l) {
            const c128 h = H[i + (int64_t)l * ldh], v = y[l];
            re -= h.x * v.x - h.y * v.y;
            im -= h.x * v.y + h.y * v.x;
        }
        const c128 d = H[i + (int64_t)i * ldh];
        const double den = d.x * d.x + d.y * d.y;
        y[i] = make_double2((re * d.x + im * d.y) / den, (im * d.x - re * d.y) / den);
    }
}

}  // namespace

int krylov_nchunks(int64_t n) { return (int)((n + kChunk - 1) / kChunk); }

void launch_multidot(hipStream_t s, const c128* V, int64_t ldv, int ncols, const c128* w, int64_t n, c128* partial) {
    hipLaunchKernelGGL(k_multidot, dim3(krylov_nchunks(n)), dim3(256), 0, s, V, ldv, ncols, w, n, partial);
}
void launch_reduce_dots(hipStream_t s, const c128* partial, int nchunks, int ncols, c128* h, int accumulate) {
    hipLaunchKernelGGL(k_reduce_dots, dim3((ncols + 255) / 256), dim3(256), 0, s, partial, nchunks, ncols, h, accumulate);
}
void launch_gemv_sub(hipStream_t s, const c128* V, int64_t ldv, int ncols, const c128* h, c128* w, int64_t n) {
    hipLaunchKernelGGL(k_gemv_sub, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, V, ldv, ncols, h, w, n);
}
void launch_gemv_add(hipStream_t s, const c128* V, int64_t ldv, int ncols, const c128* y, c128* x, int64_t n) {
    hipLaunchKernelGGL(k_gemv_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, V, ldv, ncols, y, x, n);
}
void launch_norm2(hipStream_t s, const c128* w, int64_t n, double* partial) {
    hipLaunchKernelGGL(k_norm2, dim3(krylov_nchunks(n)), dim3(256), 0, s, w, n, partial);
}
void launch_reduce_norm(hipStream_t s, const double* partial, int nchunks, double* out) {
    hipLaunchKernelGGL(k_reduce_norm, dim3(1), dim3(64), 0, s, partial, nchunks, out);
}
void launch_scale_into(hipStream_t s, const c128* w, int64_t n, const double* norm2, c128* out, c128* gslot) {
    hipLaunchKernelGGL(k_scale_into, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, w, n, norm2, out, gslot);
}
void launch_givens(hipStream_t s, int j, c128* hcol, c128* H, int ldh, double* cs, c128* sn, c128* g,
                   const double* hnorm2, double* status) {
    hipLaunchKernelGGL(k_givens, dim3(1), dim3(64), 0, s, j, hcol, H, ldh, cs, sn, g, hnorm2, status);
}
void launch_trisolve(hipStream_t s, int k, const c128* H, int ldh, const c128* g, c128* y) {
    hipLaunchKernelGGL(k_trisolve, dim3(1), dim3(64), 0, s, k, H, ldh, g, y);
}

}  // namespace qrvie
