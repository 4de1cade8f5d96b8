// Device helpers shared by the streaming kernels (compressed product, Krylov basis
// sweeps): complex FMA, nontemporal loads of complex128/complex64 entries widened to
// FP64, and a double-buffered column-batch driver.
#pragma once

#include "internal.h"

namespace qrvie {

__device__ __forceinline__ void cfma(c128& acc, c128 a, c128 b) {
    acc.x = fma(a.x, b.x, fma(-a.y, b.y, acc.x));
    acc.y = fma(a.x, b.y, fma(a.y, b.x, acc.y));
}

typedef double v2d __attribute__((ext_vector_type(2)));
typedef float v2f __attribute__((ext_vector_type(2)));

// Streaming loads: data read once per pass stays out of the caches.  Complex64 entries
// are widened to FP64 when used; accumulation is FP64 either way.
__device__ __forceinline__ c128 load_stream(const c128* p) {
    const v2d v = __builtin_nontemporal_load(reinterpret_cast<const v2d*>(p));
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ float2 load_stream(const float2* p) {
    const v2f v = __builtin_nontemporal_load(reinterpret_cast<const v2f*>(p));
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ c128 widen(c128 a) { return a; }
__device__ __forceinline__ c128 widen(float2 a) { return make_double2((double)a.x, (double)a.y); }

// The wave's column range must be wave-uniform so that the vector entries v[j] are
// scalar loads (a separate counter from the factor loads, and no per-lane addressing).
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// Column range of wave wv when WAVES waves share ncols columns: whole batches of U
// columns per wave, so only the last wave can have a partial batch.
template <typename F, int U>
__device__ __forceinline__ void load_batch(const F* __restrict__ p, int64_t ld, F a[U]) {
#pragma unroll
    for (int u = 0; u < U; ++u) a[u] = load_stream(p + (int64_t)u * ld);
}

// Runs fmas(batch, k) over nb batches of U columns starting at p (stride ld between
// columns).  Batches are double-buffered: the loads of batch k+1 are issued before the
// FMAs of batch k, with a scheduling barrier so the compiler does not interleave them.
// The steady-state loop issues both loads unconditionally, so the wait before each FMA
// only covers its own batch (the loads of the next batch stay in flight).
template <typename F, int U, typename Fmas>
__device__ __forceinline__ void stream_batches(const F* __restrict__ p, int64_t ld, int nb, Fmas&& fmas) {
    const int64_t step = (int64_t)U * ld;
    F a[U], b[U];
    if (nb <= 0) return;
    load_batch<F, U>(p, ld, a);
    int k = 0;
    for (; k + 2 < nb; k += 2) {
        load_batch<F, U>(p + step, ld, b);
        __builtin_amdgcn_sched_barrier(0);
        fmas(a, k);
        p += step;
        load_batch<F, U>(p + step, ld, a);
        __builtin_amdgcn_sched_barrier(0);
        fmas(b, k + 1);
        p += step;
    }
    if (k + 1 < nb) {
        load_batch<F, U>(p + step, ld, b);
        __builtin_amdgcn_sched_barrier(0);
        fmas(a, k);
        fmas(b, k + 1);
    } else {
        fmas(a, k);
    }
}

}  // namespace qrvie
