// Host-side internals of libddsap: the context, launch wrappers of the HIP
// kernels and error plumbing.  Nothing here crosses the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <memory>
#include <string>
#include <vector>

#include "../../include/ddsap.h"

namespace dd {

// A named range on the host timeline around one library call or one phase of
// the solver (shown by rocprofv3 --marker-trace; a no-op without a tool).
struct TraceRange {
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

constexpr int BS_HOST = 256; // sites per 4^4 Schwarz block

struct Status {
    dd_status code = DD_OK;
    std::string msg;
    static Status ok() { return {}; }
    bool good() const { return code == DD_OK; }
};

#define DD_HIP_TRY(expr)                                                                               \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess)                                                                          \
            return dd::Status{e_ == hipErrorOutOfMemory ? DD_OOM : DD_HIP_ERROR,                        \
                              std::string(#expr) + ": " + hipGetErrorString(e_)};                      \
    } while (0)

#define DD_TRY(expr)                                                                                   \
    do {                                                                                               \
        dd::Status s_ = (expr);                                                                        \
        if (!s_.good()) return s_;                                                                     \
    } while (0)

// Owned device allocation.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    Status alloc(size_t n)
    {
        if (n == bytes && p) return Status::ok();
        release();
        if (n == 0) return Status::ok();
        DD_HIP_TRY(hipMalloc(&p, n));
        bytes = n;
        return Status::ok();
    }
    template <typename T> T *as() const { return static_cast<T *>(p); }
};

struct GeomHost {
    int L[4];
    int nb[4];
    int bstride[4];
    int nblocks;
    long V;
    int bcs[4];
};

// Kernel classes timed by the optional profiler (HIP events on the context
// stream around every launch), with the algorithmic bytes and flops of each
// launch as defined by the method (not the bytes the hardware moved).
enum KClass {
    K_DSLASH_F64 = 0, K_DSLASH_F32IN_F64, K_DSLASH_F32, K_DSLASH_F16, K_DSLASH_BLOCK,
    K_SAP_F64, K_SAP_F32, K_SAP_F16, K_SAP_EO_F64, K_SAP_EO_F32, K_SAP_EO_F16,
    K_CGS_DOTS, K_CGS_UPDATE, K_CGS_NORMALIZE, K_REDUCE, K_COMBINE, K_CONVERT, K_PACK,
    K_AMG_RESTRICT, K_AMG_COARSE, K_AMG_PROLONG,
    K_NCLASS
};
const char *kclass_name(int k);

struct Prof {
    bool on = false;
    struct Rec {
        int cls;
        hipEvent_t a, b;
        double bytes, flops;
    };
    std::vector<Rec> pending;
    std::vector<hipEvent_t> pool;
    long launches[K_NCLASS] = {};
    double ms[K_NCLASS] = {}, bytes[K_NCLASS] = {}, flops[K_NCLASS] = {};
    ~Prof();
    hipEvent_t get();
    void resolve(); // caller has synchronised the stream
    void reset();
};

// Brackets one launch with events when profiling is on.
struct ProfScope {
    Prof *p;
    hipStream_t st;
    int cls;
    double bytes, flops;
    hipEvent_t a = nullptr;
    // enable = false: no events are recorded (and none created)
    ProfScope(Prof &pr, hipStream_t s, int c, double by, double fl, bool enable = true);
    ~ProfScope();
};

class Engine; // engine.hip
struct EngineDeleter {
    void operator()(Engine *e) const; // engine.hip
};
struct AmgData; // coarse.hip: interpolation, coarse operator, workspace
struct AmgDeleter {
    void operator()(AmgData *a) const;
};
struct AmgWork; // coarse.hip: the two-grid preconditioner's workspace for W slots
struct AmgWorkDeleter {
    void operator()(AmgWork *w) const;
};

} // namespace dd

struct dd_ctx {
    dd::GeomHost g{};
    hipStream_t stream = nullptr;
    int device = 0;
    bool has_field = false;
    double csw = 0;
    bool link_su3 = false; // every link is SU(3) to FP64 rounding (checked at ingest)
    bool link_r12 = false; // kernels read two rows per link and rebuild the third
    bool sap_half_fields = false; // the plain FP32 smoother reads the FP16 links and clover
    int debug_poison_half = 0;    // test hook: FP16 smoother outputs to poison (-1: all)
    dd::DevBuf links[3];  // blocked links per dd_prec
    dd::DevBuf clover[3]; // blocked clover per dd_prec
    dd::DevBuf colour_blocks[2]; // int block ids of each colour, XCD-friendly order
    int ncolour[2] = {0, 0};
    std::string err;
    dd::DevBuf sap_scratch; // face buffers and carried residual of the Schwarz sweeps of dd_sap
    dd::Prof prof;
    std::unique_ptr<dd::Engine, dd::EngineDeleter> engine; // reused by dd_solve
    std::unique_ptr<dd::AmgData, dd::AmgDeleter> amg;      // coarse level of dd_amg_setup
};

namespace dd {

size_t real_bytes(int prec); // 8, 4, 2
size_t spinor_bytes(const GeomHost &g, int prec, int nrhs);

// fields.hip
// Packs the links (and builds the clover term) in every precision and checks
// whether all links are SU(3) to within 1e-13 (then link_su3 and link_r12).
Status build_fields(dd_ctx *ctx, const double *U_dev_canon, double csw);
Status set_clover_canon(dd_ctx *ctx, const double *C_dev_canon);
Status pack_spinor(dd_ctx *ctx, const double *canon, void *blocked, int prec, int nrhs);
Status unpack_spinor(dd_ctx *ctx, const void *blocked, double *canon, int prec, int nrhs);
// one FP64 right-hand side <-> slot `slot` of a `width`-wide blocked FP64 buffer
// nonzero (device, optional): set to 1 if any entry of canon is nonzero
Status pack_slot(dd_ctx *ctx, hipStream_t st, const double *canon, void *blocked, int width, int slot,
                 int *nonzero = nullptr);
Status unpack_slot(dd_ctx *ctx, hipStream_t st, const void *blocked, double *canon, int width, int slot);
Status any_nonfinite(dd_ctx *ctx, const double *p, size_t n, bool &bad);

// dslash.hip
// out = D in (resid == nullptr) or out = resid - D in (the residual form:
// FP64 or FP32 throughout).  in_prec may differ from out_prec only for
// (F32 in, F64 out) and (F64 in, F64 out).  Masses
// come from the host array m0 or, when m0_dev is set, from device memory;
// in_off (device, nullable) adds a per-rhs element offset to the input.
// active (device, nullable): right-hand sides with active[r] == 0 are skipped
// (their output is left as it was).
Status launch_dslash(dd_ctx *ctx, const double *m0, int nrhs, const void *in, int in_prec, void *out, int out_prec,
                     int field_prec, const double *resid, const double *m0_dev = nullptr,
                     const long *in_off = nullptr, const int *active = nullptr);
Status launch_dslash_block(dd_ctx *ctx, double m0, int block_id, const void *in, void *out, int prec);

// sap.hip
// Per-slot device data for batched use: masses and element offsets of each
// right-hand side's eta and psi chunks (all device pointers, nullable).
struct SapSlots {
    const double *m0_dev = nullptr;
    const long *eta_off = nullptr;
    const long *psi_off = nullptr;
    const int *active = nullptr; // slots with active[r] == 0 are skipped (psi left as it was)
    // the sweeps' scratch (face buffers and the carried block residual,
    // sap_scratch_bytes), owned by the caller; must be set with per-slot data
    void *scratch = nullptr;
    bool quiet = false; // no profiler events (the no-allocation path)
};
size_t sap_scratch_bytes(const GeomHost &g, int prec, int nrhs);
// grows the context's scratch (used when no SapSlots::scratch is given)
Status reserve_sap_scratch(dd_ctx *ctx, int prec, int nrhs);
// eo selects the even-odd preconditioned block solve
Status run_sap(dd_ctx *ctx, const double *m0, int nrhs, const void *eta, void *psi, int ncy, int nmr, int prec,
               const SapSlots *slots = nullptr, bool eo = false);

// noalloc.hip (the fixed array holds DD_SAP_NOALLOC_SCRATCH_BYTES, ddsap.h)
// Device address of `device`'s fixed scratch array (looked up once per device).
Status noalloc_scratch(int device, void **out);
// dd_sap with the scratch in the fixed array: no device memory is allocated.
Status run_sap_noalloc(dd_ctx *ctx, const double *m0, int nrhs, const void *eta, void *psi, int ncy, int nmr,
                       int prec);

// coarse.hip
Status amg_setup(dd_ctx *ctx, double m0, const double *v0, const dd_amg_params &p);
// P and D_c (FP64) to host memory (either may be null)
Status amg_export(dd_ctx *ctx, double *P_host, double *A_host);
size_t amg_coarse_size(const dd_ctx *ctx);
// op: 0 restrict, 1 prolong, 2 coarse apply, 3 coarse solve (k steps), 4 two-grid
Status amg_standalone(dd_ctx *ctx, int op, const double *m0, int nrhs, const void *in, void *out, int prec, int k);
AmgWork *amg_work_new();
// sizes the workspace for W slots of precision prec and a coarse basis of
// max(kmax, the setup's coarse_k) + 1 vectors
Status amg_reserve(dd_ctx *ctx, AmgWork &wk, int W, int prec, int kmax);
// z = B eta for W slots (slot r of eta at eta + eta_off[r], of z at z +
// z_off[r], in the blocked layout with W right-hand sides; offsets nullable)
Status run_two_grid(dd_ctx *ctx, AmgWork &wk, int W, const void *eta, const long *eta_off, int prec, void *z,
                    const long *z_off, const double *m0_dev, const int *active);

// profile.hip: streaming device copy (bytes a multiple of 16)
Status stream_copy(const void *src, void *dst, size_t bytes, hipStream_t st);

// engine.hip
Status solve(dd_ctx *ctx, const double *m0, const double *b, double *x, int nrhs, const dd_params &p,
             dd_solve_info *info);

} // namespace dd
