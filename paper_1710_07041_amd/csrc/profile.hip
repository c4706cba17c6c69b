// Optional per-kernel-class timing: HIP events recorded on the context stream
// around each launch, resolved after the stream has been synchronised.
#include <algorithm>

#include "dd_device.h"
#include "dd_internal.h"

namespace dd {

const char *kclass_name(int k)
{
    static const char *names[K_NCLASS] = {
        "dslash_f64", "dslash_f32in_f64", "dslash_f32", "dslash_f16", "dslash_block",
        "sap_sweep_f64", "sap_sweep_f32", "sap_sweep_f16", "sap_sweep_eo_f64", "sap_sweep_eo_f32", "sap_sweep_eo_f16",
        "cgs_dots", "cgs_update", "restart_norm", "reduce", "combine", "convert", "pack",
        "amg_restrict", "amg_coarse_solve", "amg_prolong",
    };
    return (k >= 0 && k < K_NCLASS) ? names[k] : "?";
}

Prof::~Prof()
{
    for (auto &r : pending) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto e : pool) (void)hipEventDestroy(e);
}

hipEvent_t Prof::get()
{
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void Prof::resolve()
{
    for (auto &r : pending) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
            launches[r.cls] += 1;
            ms[r.cls] += t;
            bytes[r.cls] += r.bytes;
            flops[r.cls] += r.flops;
        }
        pool.push_back(r.a);
        pool.push_back(r.b);
    }
    pending.clear();
}

void Prof::reset()
{
    resolve();
    for (int k = 0; k < K_NCLASS; ++k) {
        launches[k] = 0;
        ms[k] = bytes[k] = flops[k] = 0.0;
    }
}

ProfScope::ProfScope(Prof &pr, hipStream_t s, int c, double by, double fl, bool enable)
    : p(pr.on && enable ? &pr : nullptr), st(s), cls(c), bytes(by), flops(fl)
{
    if (!p) return;
    a = p->get();
    if (a) (void)hipEventRecord(a, st);
}

ProfScope::~ProfScope()
{
    if (!p || !a) return;
    hipEvent_t b = p->get();
    if (!b) {
        p->pool.push_back(a);
        return;
    }
    (void)hipEventRecord(b, st);
    p->pending.push_back({cls, a, b, bytes, flops});
}

namespace {

// Streaming copy: 16-byte non-temporal loads and stores, a tile of 1024
// vectors per workgroup (four per thread, all loads issued before the
// stores); the achievable-HBM-bandwidth reference the kernels are compared
// with.
__global__ __launch_bounds__(256) void k_stream_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst, size_t n)
{
    const size_t i = (size_t)blockIdx.x * 1024 + threadIdx.x;
    if (i + 3 * 256 < n) {
        uint4 v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = ld_stream(src + i + k * 256);
#pragma unroll
        for (int k = 0; k < 4; ++k) st_stream(dst + i + k * 256, v[k]);
    } else {
        for (int k = 0; k < 4; ++k)
            if (i + k * 256 < n) st_stream(dst + i + k * 256, ld_stream(src + i + k * 256));
    }
}

} // namespace

Status stream_copy(const void *src, void *dst, size_t bytes, hipStream_t st)
{
    const size_t n = bytes / 16;
    const size_t grid = (n + 1023) / 1024;
    if (grid > 0x7fffffffu) return Status{DD_INVALID_ARG, "stream copy: too large"};
    k_stream_copy<<<(unsigned)grid, 256, 0, st>>>(static_cast<const uint4 *>(src), static_cast<uint4 *>(dst), n);
    DD_HIP_TRY(hipGetLastError());
    return Status::ok();
}

} // namespace dd
