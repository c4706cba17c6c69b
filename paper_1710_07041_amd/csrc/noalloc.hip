// dd_sap_noalloc: the Schwarz smoother of dd_sap for callers that cannot
// allocate device memory.  Its scratch -- the face buffers through which a
// block passes its boundary half spinors to the other colour, and the block
// residual carried from one visit to the next -- lives in a fixed device
// array of this file instead of a hipMalloc'd buffer of the context.
//
// In host code the array's name is only a host-side stand-in; its device
// address (one per GPU, each GPU holding its own copy) is looked up once per
// device with hipGetSymbolAddress and cached, and only that address is handed
// to kernels.
#include <algorithm>
#include <mutex>
#include <string>

#include "dd_internal.h"

namespace dd {

namespace {

constexpr size_t NOALLOC_SCRATCH_BYTES = DD_SAP_NOALLOC_SCRATCH_BYTES;

__device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

// psi = 0 without hipMemsetAsync (stays valid under stream capture)
__global__ void k_zero16(uint4 *__restrict__ p, size_t n16)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (size_t)gridDim.x * blockDim.x)
        p[i] = make_uint4(0u, 0u, 0u, 0u);
}

} // namespace

// Device address of this device's scratch array; looked up on the first call
// for a device (with that device current) and cached.
Status noalloc_scratch(int device, void **out)
{
    if (device < 0 || device >= MAX_DEVICES) return Status{DD_INVALID_ARG, "no-alloc scratch: device index out of range"};
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        DD_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return Status{DD_HIP_ERROR, "no-alloc scratch: no device address"};
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return Status::ok();
}

Status run_sap_noalloc(dd_ctx *ctx, const double *m0, int nrhs, const void *eta, void *psi, int ncy, int nmr,
                       int prec)
{
    const size_t need = sap_scratch_bytes(ctx->g, prec, nrhs);
    if (need > NOALLOC_SCRATCH_BYTES)
        return Status{DD_INVALID_ARG, "dd_sap_noalloc: the smoother needs " + std::to_string(need) +
                                          " bytes of scratch, more than the fixed " +
                                          std::to_string(NOALLOC_SCRATCH_BYTES)};
    void *p = nullptr;
    DD_TRY(noalloc_scratch(ctx->device, &p));
    if (ncy == 0) {
        const size_t n16 = spinor_bytes(ctx->g, prec, nrhs) / 16; // whole blocks of 256 sites: a multiple of 16
        const unsigned grid = (unsigned)std::min<size_t>((n16 + 255) / 256, 8192);
        k_zero16<<<grid, 256, 0, ctx->stream>>>(static_cast<uint4 *>(psi), n16);
        DD_HIP_TRY(hipGetLastError());
        return Status::ok();
    }
    SapSlots sl;
    sl.scratch = p;
    sl.quiet = true; // no profiler events: nothing is created on this path
    return run_sap(ctx, m0, nrhs, eta, psi, ncy, nmr, prec, &sl, false);
}

} // namespace dd
