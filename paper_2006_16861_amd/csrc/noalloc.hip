// Allocation-free preconditioner application (tdp_precond_apply_noalloc).
//
// The recurrence fields of Table 1 (and the complex64 copy of F for FP32
// fields) live in one file-scope device array instead of buffers that the
// library allocates.  Each device holds its own copy of the array for the
// life of the process; host code never uses the array's name as a device
// address, only the address hipGetSymbolAddress returns for the device that
// was current when it was looked up (at tdp_op_create).
#include <hip/hip_runtime.h>

#include <mutex>

#include "tdp_internal.h"

static __device__ __align__(256) unsigned char scratch[TDP_NOALLOC_MAX_BYTES];

namespace tdp {

static const int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];
static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace tdp

using namespace tdp;

int noalloc_setup_device(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device %d beyond the %d devices the library supports", dev, kMaxDevices);
        return TDP_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev]) return TDP_OK;
    void *p = nullptr;
    TDP_CHECK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) {
        set_error("hipGetSymbolAddress returned no address for the scratch array on device %d", dev);
        return TDP_EHIP;
    }
    g_scratch_ptr[dev] = p;
    return TDP_OK;
}

extern "C" int tdp_precond_apply_noalloc(const tdp_op *cop, int periods_T, double rho,
                                         const void *F, void *U)
{
    clear_error();
    if (!cop || !F || !U) {
        set_error("NULL argument");
        return TDP_EINVAL;
    }
    if (F == U) {
        set_error("F and U must not alias");
        return TDP_EINVAL;
    }
    if (misaligned16(F) || misaligned16(U)) {
        set_error("complex arrays must be 16-byte aligned");
        return TDP_EINVAL;
    }
    tdp_op *op = const_cast<tdp_op *>(cop);
    void *base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (op->device >= 0 && op->device < kMaxDevices) base = g_scratch_ptr[op->device];
    }
    if (!base) {
        set_error("no scratch address recorded for device %d", op->device);
        return TDP_EHIP;
    }
    // four field planes of the field precision, then (FP32) F as complex64
    const size_t w = op->prec == TDP_F64 ? sizeof(double) : sizeof(float);
    const size_t plane = align256(w * (size_t)op->N);
    const size_t stage = op->prec == TDP_F32 ? align256(2 * sizeof(float) * (size_t)op->N) : 0;
    const size_t need = 4 * plane + stage;
    if (need > (size_t)TDP_NOALLOC_MAX_BYTES) {
        set_error("grid of %lld nodes needs %zu bytes of scratch; the allocation-free entry "
                  "point holds %zu (TDP_NOALLOC_MAX_BYTES)",
                  (long long)op->N, need, (size_t)TDP_NOALLOC_MAX_BYTES);
        return TDP_EINVAL;
    }
    unsigned char *b = (unsigned char *)base;
    const LoopBufs lb{b, b + plane, b + 2 * plane, b + 3 * plane, true};
    StreamJoin join(op->user_stream, op->stream, op->ev);
    return precond_noalloc_impl(op, periods_T, rho, F, U, lb, stage ? b + 4 * plane : nullptr);
}
