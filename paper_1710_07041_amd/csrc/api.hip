// C ABI of libddsap (declarations and contracts in include/ddsap.h).  Every
// entry point validates its arguments, converts internal failures into a
// dd_status plus a message, and never lets a C++ exception cross the boundary.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "dd_internal.h"

namespace dd {

size_t real_bytes(int prec) { return prec == DD_F64 ? 8 : prec == DD_F32 ? 4 : 2; }

size_t spinor_bytes(const GeomHost &g, int prec, int nrhs)
{
    return (size_t)g.V * 12 * 2 * real_bytes(prec) * (size_t)nrhs;
}

} // namespace dd

namespace {

thread_local std::string g_create_error;

// Diagnostics on stderr, off unless DDSAP_LOG is set (read once): 1 prints a
// line per failed call and per solve (iterations, residual, wall time).
int log_level()
{
    static const int level = [] {
        const char *e = std::getenv("DDSAP_LOG");
        return e ? std::atoi(e) : 0;
    }();
    return level;
}

dd_status fail(dd_ctx *ctx, const dd::Status &s)
{
    if (ctx) ctx->err = s.msg;
    if (log_level() >= 1) std::fprintf(stderr, "[ddsap] error %d: %s\n", (int)s.code, s.msg.c_str());
    return s.code;
}

dd_status fail(dd_ctx *ctx, dd_status code, const std::string &msg) { return fail(ctx, dd::Status{code, msg}); }

bool prec_ok(int p) { return p == DD_F64 || p == DD_F32 || p == DD_F16; }

template <typename F> dd_status guarded(dd_ctx *ctx, F &&f)
{
    try {
        dd::Status s = f();
        if (!s.good()) return fail(ctx, s);
        return DD_OK;
    } catch (const std::bad_alloc &) {
        return fail(ctx, DD_OOM, "host allocation failed");
    } catch (...) {
        return fail(ctx, DD_HIP_ERROR, "unexpected internal error");
    }
}

dd::Status set_device(dd_ctx *ctx)
{
    DD_HIP_TRY(hipSetDevice(ctx->device));
    return dd::Status::ok();
}

} // namespace

extern "C" {

int dd_abi_version(void) { return DD_ABI_VERSION; }

void dd_default_params(dd_params *p)
{
    if (!p) return;
    p->m = 20;
    p->tol = 1e-10;
    p->max_restarts = 100;
    // twelve SAP cycles: on the 32^3x64 and 48^3x96 workloads the solve time
    // falls from four cycles to ten or twelve (fewer FP64 outer iterations,
    // each an operator application and a Gram-Schmidt step) and rises beyond
    p->ncy = 12;
    p->nmr = 4;
    p->sap_prec = DD_F32;
    p->sap_eo = 0;
    p->amg = 0;
}

void dd_amg_default_params(dd_amg_params *p)
{
    if (!p) return;
    // from a scan on the 32^3x64 workload (m0 = -0.35, -0.42, -0.47): twelve
    // test vectors, six inverse-iteration steps and two adaptive rounds give
    // the fewest outer iterations per setup second; eight post-smoothing
    // cycles balance the smoother against the coarse solve
    p->nvec = 12;
    p->setup_iters = 6;
    p->setup_ncy = 4;
    p->setup_nmr = 4;
    p->setup_prec = DD_F32;
    p->adapt = 2;
    p->coarse_k = 16;
    p->post_ncy = 8;
    p->post_nmr = 4;
}

const char *dd_last_error(const dd_ctx *ctx) { return ctx ? ctx->err.c_str() : g_create_error.c_str(); }

dd_status dd_create(const int dims[4], const int block[4], const int bcs[4], void *stream, dd_ctx **out)
{
    g_create_error.clear();
    if (!dims || !bcs || !out) {
        g_create_error = "dd_create: null argument";
        return DD_INVALID_ARG;
    }
    *out = nullptr;
    if (block)
        for (int mu = 0; mu < 4; ++mu)
            if (block[mu] != 4) {
                g_create_error = "dd_create: only 4x4x4x4 Schwarz blocks are implemented";
                return DD_INVALID_ARG;
            }
    dd::GeomHost g{};
    long V = 1;
    for (int mu = 0; mu < 4; ++mu) {
        if (dims[mu] < 4 || dims[mu] % 4 != 0) {
            g_create_error = "dd_create: every extent must be a positive multiple of the block extent 4";
            return DD_INVALID_ARG;
        }
        int nb = dims[mu] / 4;
        if (nb != 1 && nb % 2 != 0) {
            g_create_error = "dd_create: the number of blocks per direction must be even or one";
            return DD_INVALID_ARG;
        }
        if (bcs[mu] != 1 && bcs[mu] != -1) {
            g_create_error = "dd_create: boundary signs must be +1 or -1";
            return DD_INVALID_ARG;
        }
        g.L[mu] = dims[mu];
        g.nb[mu] = nb;
        g.bcs[mu] = bcs[mu];
        V *= dims[mu];
    }
    if (V > (1L << 28)) {
        g_create_error = "dd_create: lattice too large";
        return DD_INVALID_ARG;
    }
    g.V = V;
    g.nblocks = (int)(V / dd::BS_HOST);
    g.bstride[0] = 1;
    for (int mu = 1; mu < 4; ++mu) g.bstride[mu] = g.bstride[mu - 1] * g.nb[mu - 1];
    dd_ctx *ctx = nullptr;
    try {
        ctx = new dd_ctx();
    } catch (...) {
        g_create_error = "dd_create: host allocation failed";
        return DD_OOM;
    }
    ctx->g = g;
    ctx->stream = static_cast<hipStream_t>(stream);
    if (hipGetDevice(&ctx->device) != hipSuccess) {
        g_create_error = "dd_create: no HIP device";
        delete ctx;
        return DD_HIP_ERROR;
    }
    {
        // the device address of dd_sap_noalloc's fixed scratch array, looked
        // up once per device while that device is current
        void *scr = nullptr;
        dd::Status s = dd::noalloc_scratch(ctx->device, &scr);
        if (!s.good()) {
            g_create_error = "dd_create: " + s.msg;
            delete ctx;
            return s.code;
        }
    }
    // colour lists in canonical block order: the sweep kernels map contiguous
    // ranges of these lists onto one XCD each
    std::vector<int> lists[2];
    for (int b = 0; b < g.nblocks; ++b) {
        int t = b, sum = 0;
        for (int mu = 0; mu < 4; ++mu) {
            sum += t % g.nb[mu];
            t /= g.nb[mu];
        }
        lists[sum & 1].push_back(b);
    }
    for (int c = 0; c < 2; ++c) {
        ctx->ncolour[c] = (int)lists[c].size();
        if (lists[c].empty()) continue;
        dd::Status s = ctx->colour_blocks[c].alloc(lists[c].size() * sizeof(int));
        if (s.good() && hipMemcpy(ctx->colour_blocks[c].p, lists[c].data(), lists[c].size() * sizeof(int),
                                  hipMemcpyHostToDevice) != hipSuccess)
            s = dd::Status{DD_HIP_ERROR, "copy of the colour lists failed"};
        if (!s.good()) {
            g_create_error = "dd_create: " + s.msg;
            delete ctx;
            return s.code;
        }
    }
    *out = ctx;
    return DD_OK;
}

dd_status dd_destroy(dd_ctx *ctx)
{
    if (!ctx) return DD_INVALID_ARG;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    delete ctx;
    return DD_OK;
}

dd_status dd_synchronize(dd_ctx *ctx)
{
    if (!ctx) return DD_INVALID_ARG;
    return guarded(ctx, [&]() -> dd::Status {
        DD_TRY(set_device(ctx));
        DD_HIP_TRY(hipStreamSynchronize(ctx->stream));
        return dd::Status::ok();
    });
}

dd_status dd_set_gauge(dd_ctx *ctx, const double *U_host, double csw)
{
    if (!ctx) return DD_INVALID_ARG;
    if (!U_host || !std::isfinite(csw)) return fail(ctx, DD_INVALID_ARG, "dd_set_gauge: null field or bad csw");
    return guarded(ctx, [&]() -> dd::Status {
        DD_TRY(set_device(ctx));
        size_t n = (size_t)ctx->g.V * 72;
        for (size_t i = 0; i < n; ++i)
            if (!std::isfinite(U_host[i])) return dd::Status{DD_NAN, "dd_set_gauge: gauge field holds NaN or Inf"};
        dd::DevBuf U;
        DD_TRY(U.alloc(n * sizeof(double)));
        DD_HIP_TRY(hipMemcpyAsync(U.p, U_host, n * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
        DD_TRY(dd::build_fields(ctx, U.as<double>(), csw));
        DD_HIP_TRY(hipStreamSynchronize(ctx->stream));
        ctx->has_field = true;
        ctx->csw = csw;
        return dd::Status::ok();
    });
}

dd_status dd_set_link_compression(dd_ctx *ctx, int enable)
{
    if (!ctx) return DD_INVALID_ARG;
    if (enable && !(ctx->has_field && ctx->link_su3))
        return fail(ctx, DD_INVALID_ARG, "dd_set_link_compression: the gauge field is not SU(3)");
    ctx->link_r12 = enable != 0;
    return DD_OK;
}

int dd_link_compression(const dd_ctx *ctx) { return ctx ? (ctx->link_r12 ? 1 : 0) : -1; }

dd_status dd_set_sap_half_fields(dd_ctx *ctx, int enable)
{
    if (!ctx) return DD_INVALID_ARG;
    ctx->sap_half_fields = enable != 0;
    return DD_OK;
}

int dd_sap_half_fields(const dd_ctx *ctx) { return ctx ? (ctx->sap_half_fields ? 1 : 0) : -1; }

dd_status dd_set_clover(dd_ctx *ctx, const double *C_host)
{
    if (!ctx) return DD_INVALID_ARG;
    if (!C_host) return fail(ctx, DD_INVALID_ARG, "dd_set_clover: null clover");
    if (!ctx->has_field) return fail(ctx, DD_NO_FIELD, "dd_set_clover: call dd_set_gauge first");
    return guarded(ctx, [&]() -> dd::Status {
        DD_TRY(set_device(ctx));
        size_t n = (size_t)ctx->g.V * 144;
        for (size_t i = 0; i < n; ++i)
            if (!std::isfinite(C_host[i])) return dd::Status{DD_NAN, "dd_set_clover: clover holds NaN or Inf"};
        dd::DevBuf C;
        DD_TRY(C.alloc(n * sizeof(double)));
        DD_HIP_TRY(hipMemcpyAsync(C.p, C_host, n * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
        DD_TRY(dd::set_clover_canon(ctx, C.as<double>()));
        DD_HIP_TRY(hipStreamSynchronize(ctx->stream));
        return dd::Status::ok();
    });
}

size_t dd_spinor_bytes(const dd_ctx *ctx, int prec, int nrhs)
{
    if (!ctx || !prec_ok(prec) || nrhs < 1) return 0;
    return dd::spinor_bytes(ctx->g, prec, nrhs);
}

dd_status dd_pack_spinor(dd_ctx *ctx, const double *canon, void *blocked, int prec, int nrhs)
{
    if (!ctx) return DD_INVALID_ARG;
    if (!canon || !blocked || !prec_ok(prec) || nrhs < 1 || nrhs > DD_MAX_RHS)
        return fail(ctx, DD_INVALID_ARG, "dd_pack_spinor: bad argument");
    return guarded(ctx, [&]() -> dd::Status {
        DD_TRY(set_device(ctx));
        return dd::pack_spinor(ctx, canon, blocked, prec, nrhs);
    });
}

dd_status dd_unpack_spinor(dd_ctx *ctx, const void *blocked, double *canon, int prec, int nrhs)
{
    if (!ctx) return DD_INVALID_ARG;
    if (!canon || !blocked || !prec_ok(prec) || nrhs < 1 || nrhs > DD_MAX_RHS)
        return fail(ctx, DD_INVALID_ARG, "dd_unpack_spinor: bad argument");
    return guarded(ctx, [&]() -> dd::Status {
        DD_TRY(set_device(ctx));
        return dd::unpack_spinor(ctx, blocked, canon, prec, nrhs);
    });
}

dd_status dd_apply_D(dd_ctx *ctx, const double *m0, const void *x, void *y, int prec, int nrhs)
{
    if (!ctx) return DD_INVALID_ARG;
    if (!m0 || !x || !y || x == y || !prec_ok(prec) || nrhs < 1 || nrhs > DD_MAX_RHS)
        return fail(ctx, DD_INVALID_ARG, "dd_apply_D: bad argument");
    if (!ctx->has_field) return fail(ctx, DD_NO_FIELD, "dd_apply_D: no gauge field");
    for (int r = 0; r < nrhs; ++r)
        if (!std::isfinite(m0[r])) return fail(ctx, DD_INVALID_ARG, "dd_apply_D: non-finite mass");
    return guarded(ctx, [&]() -> dd::Status {
        DD_TRY(set_device(ctx));
        dd::TraceRange tr("dd_apply_D");
        return dd::launch_dslash(ctx, m0, nrhs, x, prec, y, prec, prec, nullptr);
    });
}

dd_status dd_apply_D_block(dd_ctx *ctx, double m0, long block_id, const void *x, void *y, int prec)
{
    if (!ctx) return DD_INVALID_ARG;
    if (!x || !y || x == y || !prec_ok(prec) || !std::isfinite(m0))
        return fail(ctx, DD_INVALID_ARG, "dd_apply_D_block: bad argument");
    if (block_id < 0 || block_id >= ctx->g.nblocks) return fail(ctx, DD_INVALID_ARG, "dd_apply_D_block: bad block id");
    if (!ctx->has_field) return fail(ctx, DD_NO_FIELD, "dd_apply_D_block: no gauge field");
    return guarded(ctx, [&]() -> dd::Status {
        DD_TRY(set_device(ctx));
        return dd::launch_dslash_block(ctx, m0, (int)block_id, x, y, prec);
    });
}

dd_status dd_sap(dd_ctx *ctx, const double *m0, const void *eta, void *psi, int ncy, int nmr, int prec, int nrhs)
{
    if (!ctx) return DD_INVALID_ARG;
    if (!m0 || !eta || !psi || eta == psi || !prec_ok(prec) || nrhs < 1 || nrhs > DD_MAX_RHS || ncy < 0 || nmr < 0)
        return fail(ctx, DD_INVALID_ARG, "dd_sap: bad argument");
    if (!ctx->has_field) return fail(ctx, DD_NO_FIELD, "dd_sap: no gauge field");
    for (int r = 0; r < nrhs; ++r)
        if (!std::isfinite(m0[r])) return fail(ctx, DD_INVALID_ARG, "dd_sap: non-finite mass");
    return guarded(ctx, [&]() -> dd::Status {
        DD_TRY(set_device(ctx));
        dd::TraceRange tr("dd_sap");
        return dd::run_sap(ctx, m0, nrhs, eta, psi, ncy, nmr, prec);
    });
}

dd_status dd_sap_eo(dd_ctx *ctx, const double *m0, const void *eta, void *psi, int ncy, int nmr, int prec, int nrhs)
{
    if (!ctx) return DD_INVALID_ARG;
    if (!m0 || !eta || !psi || eta == psi || !prec_ok(prec) || nrhs < 1 || nrhs > DD_MAX_RHS || ncy < 0 || nmr < 0)
        return fail(ctx, DD_INVALID_ARG, "dd_sap_eo: bad argument");
    if (!ctx->has_field) return fail(ctx, DD_NO_FIELD, "dd_sap_eo: no gauge field");
    for (int r = 0; r < nrhs; ++r)
        if (!std::isfinite(m0[r])) return fail(ctx, DD_INVALID_ARG, "dd_sap_eo: non-finite mass");
    return guarded(ctx, [&]() -> dd::Status {
        DD_TRY(set_device(ctx));
        dd::TraceRange tr("dd_sap_eo");
        return dd::run_sap(ctx, m0, nrhs, eta, psi, ncy, nmr, prec, nullptr, true);
    });
}

dd_status dd_sap_noalloc(dd_ctx *ctx, const double *m0, const void *eta, void *psi, int ncy, int nmr, int prec,
                         int nrhs)
{
    if (!ctx) return DD_INVALID_ARG;
    if (!m0 || !eta || !psi || eta == psi || !prec_ok(prec) || nrhs < 1 || nrhs > DD_MAX_RHS || ncy < 0 || nmr < 0)
        return fail(ctx, DD_INVALID_ARG, "dd_sap_noalloc: bad argument");
    if (!ctx->has_field) return fail(ctx, DD_NO_FIELD, "dd_sap_noalloc: no gauge field");
    for (int r = 0; r < nrhs; ++r)
        if (!std::isfinite(m0[r])) return fail(ctx, DD_INVALID_ARG, "dd_sap_noalloc: non-finite mass");
    return guarded(ctx, [&]() -> dd::Status {
        DD_TRY(set_device(ctx));
        dd::TraceRange tr("dd_sap_noalloc");
        return dd::run_sap_noalloc(ctx, m0, nrhs, eta, psi, ncy, nmr, prec);
    });
}

dd_status dd_solve(dd_ctx *ctx, const double *m0, const double *b, double *x, int nrhs, const dd_params *params,
                   dd_solve_info *info)
{
    if (!ctx) return DD_INVALID_ARG;
    dd_params p;
    dd_default_params(&p);
    if (params) p = *params;
    if (!m0 || !b || !x || (const void *)b == (const void *)x || nrhs < 1 || nrhs > DD_MAX_RHS)
        return fail(ctx, DD_INVALID_ARG, "dd_solve: bad argument");
    if (p.m < 1 || p.m > 32 || !(p.tol > 0) || p.max_restarts < 0 || p.ncy < 0 || p.nmr < 0 || !prec_ok(p.sap_prec))
        return fail(ctx, DD_INVALID_ARG, "dd_solve: bad parameters (1 <= m <= 32, tol > 0, ...)");
    if (p.amg && !ctx->amg) return fail(ctx, DD_INVALID_ARG, "dd_solve: amg = 1 needs dd_amg_setup first");
    if (p.amg && p.sap_prec == DD_F16)
        return fail(ctx, DD_INVALID_ARG, "dd_solve: the two-grid preconditioner smooths in FP32 or FP64");
    if (!ctx->has_field) return fail(ctx, DD_NO_FIELD, "dd_solve: no gauge field");
    for (int r = 0; r < nrhs; ++r)
        if (!std::isfinite(m0[r])) return fail(ctx, DD_INVALID_ARG, "dd_solve: non-finite mass");
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<dd_solve_info> own(log_level() >= 1 && !info ? nrhs : 0);
    dd_solve_info *inf = info ? info : (own.empty() ? nullptr : own.data());
    const dd_status st = guarded(ctx, [&]() -> dd::Status {
        DD_TRY(set_device(ctx));
        dd::TraceRange tr("dd_solve");
        return dd::solve(ctx, m0, b, x, nrhs, p, inf);
    });
    if (log_level() >= 1 && inf) {
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        std::fprintf(stderr, "[ddsap] dd_solve: %d right-hand side(s), status %d, %.3f ms\n", nrhs, (int)st, ms);
        for (int r = 0; r < nrhs; ++r)
            std::fprintf(stderr, "[ddsap]   rhs %d: status %d, %d iterations, %d restarts, %d smoother calls, "
                                 "residual %.3e\n",
                         r, inf[r].status, inf[r].iterations, inf[r].restarts, inf[r].sap_calls, inf[r].rel_residual);
    }
    return st;
}

dd_status dd_amg_setup(dd_ctx *ctx, double m0, const double *v0, const dd_amg_params *p)
{
    if (!ctx) return DD_INVALID_ARG;
    if (!v0 || !p || !std::isfinite(m0)) return fail(ctx, DD_INVALID_ARG, "dd_amg_setup: bad argument");
    if (!ctx->has_field) return fail(ctx, DD_NO_FIELD, "dd_amg_setup: no gauge field");
    return guarded(ctx, [&]() -> dd::Status {
        DD_TRY(set_device(ctx));
        ctx->engine.reset(); // an engine's two-grid workspace belongs to the previous setup
        dd::Status s = dd::amg_setup(ctx, m0, v0, *p);
        if (!s.good()) ctx->amg.reset();
        return s;
    });
}

size_t dd_amg_coarse_size(const dd_ctx *ctx) { return ctx ? dd::amg_coarse_size(ctx) : 0; }

dd_status dd_amg_interpolation(dd_ctx *ctx, double *P_host)
{
    if (!ctx) return DD_INVALID_ARG;
    if (!P_host || !ctx->amg) return fail(ctx, DD_INVALID_ARG, "dd_amg_interpolation: no setup or null pointer");
    return guarded(ctx, [&]() -> dd::Status {
        DD_TRY(set_device(ctx));
        DD_HIP_TRY(hipStreamSynchronize(ctx->stream));
        return dd::amg_export(ctx, P_host, nullptr);
    });
}

dd_status dd_amg_coarse_operator(dd_ctx *ctx, double *Dc_host)
{
    if (!ctx) return DD_INVALID_ARG;
    if (!Dc_host || !ctx->amg) return fail(ctx, DD_INVALID_ARG, "dd_amg_coarse_operator: no setup or null pointer");
    return guarded(ctx, [&]() -> dd::Status {
        DD_TRY(set_device(ctx));
        DD_HIP_TRY(hipStreamSynchronize(ctx->stream));
        return dd::amg_export(ctx, nullptr, Dc_host);
    });
}

namespace {
dd_status amg_call(dd_ctx *ctx, const char *name, int op, const double *m0, int nrhs, const void *in, void *out,
                   int prec, int k)
{
    if (!ctx) return DD_INVALID_ARG;
    if (!in || !out || in == out || nrhs < 1 || nrhs > DD_MAX_RHS || (prec != DD_F64 && prec != DD_F32) ||
        ((op >= 2) && !m0))
        return fail(ctx, DD_INVALID_ARG, std::string(name) + ": bad argument");
    if (!ctx->amg) return fail(ctx, DD_INVALID_ARG, std::string(name) + ": call dd_amg_setup first");
    if (m0)
        for (int r = 0; r < nrhs; ++r)
            if (!std::isfinite(m0[r])) return fail(ctx, DD_INVALID_ARG, std::string(name) + ": non-finite mass");
    return guarded(ctx, [&]() -> dd::Status {
        DD_TRY(set_device(ctx));
        return dd::amg_standalone(ctx, op, m0, nrhs, in, out, prec, k);
    });
}
} // namespace

dd_status dd_amg_restrict(dd_ctx *ctx, const void *x, double *xc, int prec, int nrhs)
{
    return amg_call(ctx, "dd_amg_restrict", 0, nullptr, nrhs, x, xc, prec, 0);
}

dd_status dd_amg_prolong(dd_ctx *ctx, const double *xc, void *x, int prec, int nrhs)
{
    return amg_call(ctx, "dd_amg_prolong", 1, nullptr, nrhs, xc, x, prec, 0);
}

dd_status dd_amg_coarse_apply(dd_ctx *ctx, const double *m0, const double *xc, double *yc, int nrhs)
{
    return amg_call(ctx, "dd_amg_coarse_apply", 2, m0, nrhs, xc, yc, DD_F64, 0);
}

dd_status dd_amg_coarse_solve(dd_ctx *ctx, const double *m0, const double *bc, double *xc, int k, int nrhs)
{
    return amg_call(ctx, "dd_amg_coarse_solve", 3, m0, nrhs, bc, xc, DD_F64, k);
}

dd_status dd_amg_precondition(dd_ctx *ctx, const double *m0, const void *eta, void *psi, int prec, int nrhs)
{
    return amg_call(ctx, "dd_amg_precondition", 4, m0, nrhs, eta, psi, prec, 0);
}

dd_status dd_debug_poison_half_smoother(dd_ctx *ctx, int count)
{
    if (!ctx) return DD_INVALID_ARG;
    ctx->debug_poison_half = count < 0 ? -1 : count;
    return DD_OK;
}

dd_status dd_stream_copy(const void *src, void *dst, size_t bytes, void *stream)
{
    if (!src || !dst || bytes == 0 || bytes % 16 != 0) return DD_INVALID_ARG;
    try {
        dd::Status s = dd::stream_copy(src, dst, bytes, static_cast<hipStream_t>(stream));
        return s.code;
    } catch (...) {
        return DD_HIP_ERROR;
    }
}

dd_status dd_profile_enable(dd_ctx *ctx, int enable)
{
    if (!ctx) return DD_INVALID_ARG;
    return guarded(ctx, [&]() -> dd::Status {
        DD_TRY(set_device(ctx));
        DD_HIP_TRY(hipStreamSynchronize(ctx->stream));
        ctx->prof.reset();
        ctx->prof.on = enable != 0;
        return dd::Status::ok();
    });
}

int dd_profile_read(dd_ctx *ctx, dd_kernel_stat *out, int max)
{
    if (!ctx || (!out && max > 0)) return -1;
    if (hipSetDevice(ctx->device) != hipSuccess || hipStreamSynchronize(ctx->stream) != hipSuccess) {
        ctx->err = "dd_profile_read: stream synchronisation failed";
        return -1;
    }
    ctx->prof.resolve();
    int n = 0;
    for (int k = 0; k < dd::K_NCLASS && n < max; ++k) {
        if (ctx->prof.launches[k] == 0) continue;
        dd_kernel_stat &st = out[n++];
        std::memset(&st, 0, sizeof(st));
        std::strncpy(st.name, dd::kclass_name(k), sizeof(st.name) - 1);
        st.launches = ctx->prof.launches[k];
        st.total_ms = ctx->prof.ms[k];
        st.bytes = ctx->prof.bytes[k];
        st.flops = ctx->prof.flops[k];
    }
    return n;
}

} // extern "C"
