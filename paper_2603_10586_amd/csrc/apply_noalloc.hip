// The compressed product y = Z_QR x (§5.2) for callers that cannot allocate device memory:
// the same kernels as qrvie_apply, with every workspace in one fixed, file-scope device
// array instead of memory allocated per call.
//
// The array lives in device memory from the library's load until the process ends, one copy
// per device.  Its device address is looked up once per device (hipGetSymbolAddress, with the
// device current) when a context is created on that device; host code uses only that
// address.  Layout per call, in complex128 entries, each part aligned to 256 bytes: the
// permuted input (n), the permuted output (n), the rank-space vector (the sum of the ranks),
// one partial vector per active level (n each) and, for transpose-shared factors, the
// rank-space Q^T x and the mirror blocks' partial rows.  Every part is written before it is read
// within one product, so nothing needs clearing between calls.  All calls on one device share
// the array: calls that overlap on the device (several streams, threads or contexts) race.
#include <mutex>

#include "internal.h"

namespace qrvie {

namespace {

constexpr int64_t kScratchBytes = (int64_t)64 << 20;                 // 64 MiB per device
constexpr int64_t kScratchElems = kScratchBytes / (int64_t)sizeof(c128);
constexpr int kMaxDevices = 64;

static __device__ __align__(256) c128 scratch[kScratchElems];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};
bool g_done[kMaxDevices] = {};

int64_t round16(int64_t e) { return (e + 15) / 16 * 16; }

// Scratch bytes one product of `op` takes.
size_t scratch_need(const qrvie_op* op) {
    const int64_t n = op->g->ndof();
    int64_t need = 2 * round16(n) + round16(std::max<int64_t>(op->t_len, 1)) +
                   (int64_t)std::max(op->n_active, 1) * round16(n);
    if (op->shared) need += round16(std::max<int64_t>(op->t_len, 1)) + round16(std::max<int64_t>(op->p_len, 1));
    return (size_t)need * sizeof(c128);
}

}  // namespace

bool scratch_setup(int device, void** ptr, std::string* err) {
    *ptr = nullptr;
    if (device < 0 || device >= kMaxDevices) {
        *err = "device index out of range for the fixed scratch";
        return false;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_done[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            *err = std::string("hipGetSymbolAddress of the fixed scratch failed: ") + hipGetErrorString(e);
            return false;
        }
        g_ptr[device] = p;
        g_done[device] = true;
    }
    *ptr = g_ptr[device];
    return true;
}

}  // namespace qrvie

using namespace qrvie;

extern "C" {

qrvie_status qrvie_apply_noalloc(qrvie_ctx* ctx, const qrvie_op* op, const qrvie_c128* x, qrvie_c128* y) {
    if (!ctx || !op || !x || !y) {
        if (ctx) set_err(ctx, "apply_noalloc: invalid argument");
        return QRVIE_ERR_INVALID_ARG;
    }
    if (!ctx->scratch) {
        set_err(ctx, "apply_noalloc: " + ctx->scratch_err);
        return QRVIE_ERR_DEVICE;
    }
    const size_t need = scratch_need(op);
    if (need > (size_t)kScratchBytes) {
        set_err(ctx, "apply_noalloc: the operator needs " + std::to_string(need) + " bytes of scratch, above the fixed " +
                         std::to_string(kScratchBytes) + "; use qrvie_apply");
        return QRVIE_ERR_INVALID_ARG;
    }
    const int64_t n = op->g->ndof();
    c128* base = static_cast<c128*>(ctx->scratch);
    c128* xi = base;
    c128* yi = xi + round16(n);
    c128* T = yi + round16(n);
    c128* Ylev = T + round16(std::max<int64_t>(op->t_len, 1));
    c128* Sq = Ylev + (int64_t)std::max(op->n_active, 1) * round16(n);
    c128* P = Sq + round16(std::max<int64_t>(op->t_len, 1));
    apply_single_into(op, ctx->stream, T, Ylev, op->shared ? Sq : nullptr, op->shared ? P : nullptr, xi, yi,
                      reinterpret_cast<const c128*>(x), reinterpret_cast<c128*>(y));
    return hip_check(ctx, hipGetLastError(), "apply_noalloc launch");
}

}  // extern "C"
