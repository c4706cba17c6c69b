// Wilson-clover operator on the blocked layout.
//
//   (D psi)(x) = (4 + m0) psi(x) + C(x) psi(x)
//              - 1/2 sum_mu [ (1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu(x-mu)^+ psi(x-mu) ]
//
// One thread per (site, right-hand side); one 256-thread workgroup per
// (Schwarz block, right-hand side).  The hop uses the chiral-basis spin
// projection so each of the eight SU(3) products acts on two spins only.
// Bandwidth bound: per site the algorithmic traffic is links 72 + clover 72 +
// spinor in 24 + out 24 reals.  Workgroups are remapped so that each XCD
// sweeps a contiguous range of blocks (shared L2 for the neighbour faces);
// clover terms and outputs, used once, go through streaming loads/stores.
#include "dd_device.h"
#include "dd_internal.h"

namespace dd {

namespace {

struct DArgs {
    Geom g;
    int nrhs;
    int block_id;
    double m0[MAXRHS];
    const double *m0_dev; // per-rhs masses in device memory (overrides m0 when set)
    const long *in_off;   // per-rhs element offset added to the input (nullable)
};

// The eight hops run as a loop that is deliberately not unrolled: unrolled,
// the compiler hoists all 168 loads ahead of the arithmetic and spills.
template <bool BLOCKONLY, typename SI, typename SF, typename A>
__device__ __forceinline__ void hops(const vec2_t<SI> *__restrict__ in, const vec2_t<SF> *__restrict__ links,
                                     const DArgs &a, int b, const int bc[4], int r, int s, cx<A> acc[12])
{
#pragma unroll 1
    for (int k = 0; k < 8; ++k) {
        const int mu = k >> 1, dir = (k & 1) ? -1 : 1;
        int bn, sn, sign;
        bool inb;
        neighbour_rt(a.g, b, bc, s, mu, dir, bn, sn, sign, inb);
        if (BLOCKONLY && !inb) continue;
        const vec2_t<SI> *p = in + ((long)bn * a.nrhs + r) * 12 * BS + sn;
        cx<A> psi[12], h[6], uh[6], U[9];
#pragma unroll
        for (int c = 0; c < 12; ++c) psi[c] = ldc<A>(p + c * BS);
        const int lb = dir > 0 ? b : bn, ls = dir > 0 ? s : sn;
        const vec2_t<SF> *u = links + ((long)lb * 4 + mu) * 9 * BS + ls;
#pragma unroll
        for (int e = 0; e < 9; ++e) U[e] = ldc<A>(u + e * BS);
        const A kk = (A)(-0.5 * sign);
        switch (k) {
        case 0: proj_minus<0>(psi, h); su3_mul(U, h, uh); recon_minus<0>(acc, uh, kk); break;
        case 1: proj_plus<0>(psi, h); su3_mul_adj(U, h, uh); recon_plus<0>(acc, uh, kk); break;
        case 2: proj_minus<1>(psi, h); su3_mul(U, h, uh); recon_minus<1>(acc, uh, kk); break;
        case 3: proj_plus<1>(psi, h); su3_mul_adj(U, h, uh); recon_plus<1>(acc, uh, kk); break;
        case 4: proj_minus<2>(psi, h); su3_mul(U, h, uh); recon_minus<2>(acc, uh, kk); break;
        case 5: proj_plus<2>(psi, h); su3_mul_adj(U, h, uh); recon_plus<2>(acc, uh, kk); break;
        case 6: proj_minus<3>(psi, h); su3_mul(U, h, uh); recon_minus<3>(acc, uh, kk); break;
        default: proj_plus<3>(psi, h); su3_mul_adj(U, h, uh); recon_plus<3>(acc, uh, kk); break;
        }
    }
}

// occupancy target per precision: enough waves per SIMD to keep HBM busy
// without letting the scheduler hoist all eight hops' loads at once
template <typename A> struct DslashWaves { static constexpr int value = 4; };
template <> struct DslashWaves<double> { static constexpr int value = 2; };

template <typename SI, typename SO, typename SF, typename A, bool BLOCKONLY, bool RESID>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(DslashWaves<A>::value))) void k_dslash(const vec2_t<SI> *__restrict__ in, vec2_t<SO> *__restrict__ out,
                                               const vec2_t<SF> *__restrict__ links,
                                               const vec2_t<SF> *__restrict__ clov,
                                               const vec2_t<SO> *__restrict__ resid, DArgs a)
{
    int b, r;
    if (BLOCKONLY) {
        b = a.block_id;
        r = 0;
    } else {
        int wg = xcd_remap(blockIdx.x, gridDim.x);
        b = wg / a.nrhs;
        r = wg - b * a.nrhs;
    }
    const int s = threadIdx.x;
    int bc[4];
    block_coords(a.g, b, bc);
    if (a.in_off) in += a.in_off[r];
    cx<A> acc[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] = mk<A>(0, 0);
    hops<BLOCKONLY, SI, SF, A>(in, links, a, b, bc, r, s, acc);
    const long sp = ((long)b * a.nrhs + r) * 12 * BS + s;
    const A diag = (A)(4.0 + (a.m0_dev ? a.m0_dev[r] : a.m0[r]));
    // one chiral half at a time: halves the registers the clover needs
#pragma unroll 1
    for (int k = 0; k < 2; ++k) {
        cx<A> psi[6], cl[18];
#pragma unroll
        for (int c = 0; c < 6; ++c) psi[c] = ldc<A>(in + sp + (6 * k + c) * BS);
        const vec2_t<SF> *cp = clov + ((long)b * 36 + 18 * k) * BS + s;
#pragma unroll
        for (int e = 0; e < 18; ++e) cl[e] = ldc_stream<A>(cp + e * BS);
        if (k == 0) clover_half_mac(cl, diag, psi, acc);
        else clover_half_mac(cl, diag, psi, acc + 6);
    }
    if (RESID) {
#pragma unroll
        for (int c = 0; c < 12; ++c) stc_stream(out + sp + c * BS, ldc_stream<A>(resid + sp + c * BS) - acc[c]);
    } else {
#pragma unroll
        for (int c = 0; c < 12; ++c) stc_stream(out + sp + c * BS, acc[c]);
    }
}

DArgs make_args(const dd_ctx *ctx, const double *m0, int nrhs)
{
    DArgs a{};
    for (int i = 0; i < 4; ++i) {
        a.g.nb[i] = ctx->g.nb[i];
        a.g.bstride[i] = ctx->g.bstride[i];
        a.g.bcs[i] = ctx->g.bcs[i];
    }
    a.g.nblocks = ctx->g.nblocks;
    a.nrhs = nrhs;
    for (int r = 0; r < nrhs && r < MAXRHS && m0; ++r) a.m0[r] = m0[r];
    return a;
}

template <typename SI, typename SO, typename SF, typename A, bool RESID>
Status launch(dd_ctx *ctx, const DArgs &a, const void *in, void *out, int field_prec, const void *resid)
{
    int grid = ctx->g.nblocks * a.nrhs;
    const double V = (double)ctx->g.V, n = a.nrhs;
    const double by = V * (144.0 * sizeof(SF) + 24.0 * n * (sizeof(SI) + sizeof(SO) * (RESID ? 2 : 1)));
    int cls = sizeof(SF) == 8 ? (sizeof(SI) == 8 ? K_DSLASH_F64 : K_DSLASH_F32IN_F64)
                              : (sizeof(SF) == 4 ? K_DSLASH_F32 : K_DSLASH_F16);
    ProfScope ps(ctx->prof, ctx->stream, cls, by, 1848.0 * V * n);
    k_dslash<SI, SO, SF, A, false, RESID><<<grid, BS, 0, ctx->stream>>>(
        static_cast<const vec2_t<SI> *>(in), static_cast<vec2_t<SO> *>(out),
        static_cast<const vec2_t<SF> *>(ctx->links[field_prec].p), static_cast<const vec2_t<SF> *>(ctx->clover[field_prec].p),
        static_cast<const vec2_t<SO> *>(resid), a);
    DD_HIP_TRY(hipGetLastError());
    return Status::ok();
}

} // namespace

Status launch_dslash(dd_ctx *ctx, const double *m0, int nrhs, const void *in, int in_prec, void *out, int out_prec,
                     int field_prec, const double *resid, const double *m0_dev, const long *in_off)
{
    if (!in || !out || !ctx->links[field_prec].p || !ctx->clover[field_prec].p || (!m0 && !m0_dev))
        return Status{DD_INVALID_ARG, "operator: missing buffer"};
    DArgs a = make_args(ctx, m0, nrhs);
    a.m0_dev = m0_dev;
    a.in_off = in_off;
    bool rs = resid != nullptr;
    if (in_prec == DD_F64 && out_prec == DD_F64 && field_prec == DD_F64)
        return rs ? launch<double, double, double, double, true>(ctx, a, in, out, DD_F64, resid)
                  : launch<double, double, double, double, false>(ctx, a, in, out, DD_F64, resid);
    if (in_prec == DD_F32 && out_prec == DD_F64 && field_prec == DD_F64 && !rs)
        return launch<float, double, double, double, false>(ctx, a, in, out, DD_F64, nullptr);
    if (in_prec == DD_F32 && out_prec == DD_F32 && field_prec == DD_F32 && !rs)
        return launch<float, float, float, float, false>(ctx, a, in, out, DD_F32, nullptr);
    if (in_prec == DD_F16 && out_prec == DD_F16 && field_prec == DD_F16 && !rs)
        return launch<__half, __half, __half, float, false>(ctx, a, in, out, DD_F16, nullptr);
    return Status{DD_INVALID_ARG, "unsupported precision combination for the operator"};
}

Status launch_dslash_block(dd_ctx *ctx, double m0, int block_id, const void *in, void *out, int prec)
{
    DArgs a = make_args(ctx, &m0, 1);
    a.block_id = block_id;
    ProfScope ps(ctx->prof, ctx->stream, K_DSLASH_BLOCK, 256.0 * (144.0 + 48.0) * real_bytes(prec), 1848.0 * 256);
    if (prec == DD_F64)
        k_dslash<double, double, double, double, true, false><<<1, BS, 0, ctx->stream>>>(
            static_cast<const double2 *>(in), static_cast<double2 *>(out), ctx->links[DD_F64].as<double2>(),
            ctx->clover[DD_F64].as<double2>(), nullptr, a);
    else if (prec == DD_F32)
        k_dslash<float, float, float, float, true, false><<<1, BS, 0, ctx->stream>>>(
            static_cast<const float2 *>(in), static_cast<float2 *>(out), ctx->links[DD_F32].as<float2>(),
            ctx->clover[DD_F32].as<float2>(), nullptr, a);
    else
        k_dslash<__half, __half, __half, float, true, false><<<1, BS, 0, ctx->stream>>>(
            static_cast<const __half2 *>(in), static_cast<__half2 *>(out), ctx->links[DD_F16].as<__half2>(),
            ctx->clover[DD_F16].as<__half2>(), nullptr, a);
    DD_HIP_TRY(hipGetLastError());
    return Status::ok();
}

} // namespace dd
