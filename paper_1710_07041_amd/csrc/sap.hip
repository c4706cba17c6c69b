// Red-black Schwarz alternating procedure (SAP) with block-local minimal
// residual (MR) solves -- the "MR inversion within a domain" and the "entire
// Schwarz method" whose per-core rates the paper reports (Sec. 3.1, Tables 1
// and 2); the algorithm is Luescher's multiplicative SAP (Comput. Phys.
// Commun. 156 (2004) 209) with Saad's MR iteration on each block.
//
// One launch sweeps every block of one colour.  One 256-thread workgroup owns
// one 4^4 block, one thread one site, and keeps everything the MR loop needs
// on chip:
//   * the site's four forward links (and, below FP64, its clover term) live
//     in registers for the whole sweep and every right-hand side;
//   * D_BB is applied direction by direction: each thread publishes the
//     spin-projected half spinor of its site for the +mu hop of site x-mu and
//     U_mu(x)^+ times the projected half spinor for the -mu hop of site x+mu
//     through LDS, so no spinor leaves the chip inside the MR loop;
//   * the two block dot products per MR step reduce with wavefront shuffles
//     and a fixed-order combine of the four wavefronts (deterministic).
// The block residual eta_B - (D psi)_B is formed on entry: the in-block part
// by the same LDS exchange, the hops that leave the block by reading the
// other colour's psi (and, for -mu hops, the neighbour's link) from memory.
// Blocks of one colour share no site and read only the other colour's psi,
// so a sweep needs no synchronisation between workgroups.
#include "block_ops.h"
#include "dd_device.h"
#include "dd_internal.h"

namespace dd {

namespace {

struct SArgs {
    Geom g;
    const int *blocks; // block ids of the swept colour
    int nblk;
    int nrhs;
    int nmr;
    int mode; // 0: psi = 0 everywhere; 1: psi_B = 0 on this colour; 2: general
    double m0[MAXRHS];
    const double *m0_dev; // per-rhs masses in device memory (overrides m0 when set)
    const long *eta_off;  // per-rhs element offsets of eta and psi (nullable)
    const long *psi_off;
};

// The MR coefficient of one right-hand side: the dot products <q, r> and
// <q, q> over the block (wavefront shuffles, then a fixed-order combine of the
// four wavefronts through LDS), alpha = <q, r>/<q, q>; returns false when
// <q, q> vanishes (uniform over the workgroup).
template <typename A>
__device__ __forceinline__ bool mr_alpha(Lds<A> &L, int lane, int wave, const cx<A> q[12], const cx<A> rr[12],
                                         cx<A> &alpha)
{
    A qr_re = 0, qr_im = 0, qq = 0;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        qr_re = fma(q[c].re, rr[c].re, qr_re);
        qr_re = fma(q[c].im, rr[c].im, qr_re);
        qr_im = fma(q[c].re, rr[c].im, qr_im);
        qr_im = fma(-q[c].im, rr[c].re, qr_im);
        qq = fma(q[c].re, q[c].re, qq);
        qq = fma(q[c].im, q[c].im, qq);
    }
    qr_re = wave_sum(qr_re);
    qr_im = wave_sum(qr_im);
    qq = wave_sum(qq);
    if (lane == 0) {
        L.red[wave][0] = qr_re;
        L.red[wave][1] = qr_im;
        L.red[wave][2] = qq;
    }
    __syncthreads();
    qr_re = ((L.red[0][0] + L.red[1][0]) + L.red[2][0]) + L.red[3][0];
    qr_im = ((L.red[0][1] + L.red[1][1]) + L.red[2][1]) + L.red[3][1];
    qq = ((L.red[0][2] + L.red[1][2]) + L.red[2][2]) + L.red[3][2];
    if (qq == (A)0) return false;
    alpha = mk<A>(qr_re / qq, qr_im / qq);
    return true;
}

// With the half clover in registers, the MR accumulator delta lives in LDS
// (each thread touches only its own site's entries, so no barrier guards it).
template <typename A, typename RES> struct DelStore {
    cx<A> d[RES::clover_half ? 12 : 1][RES::clover_half ? BS : 1];
};

template <typename S, typename A, typename RES>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(RES::waves))) void k_sap_sweep(
    const vec2_t<S> *__restrict__ eta0, vec2_t<S> *__restrict__ psi0, const vec2_t<S> *__restrict__ links,
    const vec2_t<S> *__restrict__ clov, SArgs a)
{
    constexpr bool REGLINKS = RES::links;
    __shared__ Lds<A> L;
    __shared__ DelStore<A, RES> D;
    const int i = xcd_remap(blockIdx.x, gridDim.x);
    const int b = a.blocks[i];
    const int s = threadIdx.x;
    const int lane = s & 63, wave = s >> 6;
    int bc[4];
    block_coords(a.g, b, bc);

    // register-resident links carry the hop factor -1/2
    cx<A> U[REGLINKS ? 4 : 1][9];
    if (REGLINKS) {
#pragma unroll
        for (int mu = 0; mu < (REGLINKS ? 4 : 1); ++mu) {
            const vec2_t<S> *u = links + ((long)b * 4 + mu) * 9 * BS + s;
#pragma unroll
            for (int e = 0; e < 9; ++e) U[mu][e] = (A)(-0.5) * ldc_stream<A>(u + e * BS);
        }
    }
    cx<A> cl[RES::ncl];
    if (RES::clover || RES::clover_half) {
        const vec2_t<S> *cp = clov + (long)b * 36 * BS + s;
#pragma unroll
        for (int e = 0; e < RES::ncl; ++e) cl[e] = ldc_stream<A>(cp + e * BS);
    }

    for (int r = 0; r < a.nrhs; ++r) {
        const A diag = (A)(4.0 + (a.m0_dev ? a.m0_dev[r] : a.m0[r]));
        const vec2_t<S> *__restrict__ eta = eta0 + (a.eta_off ? a.eta_off[r] : 0);
        vec2_t<S> *__restrict__ psi = psi0 + (a.psi_off ? a.psi_off[r] : 0);
        const long sp = ((long)b * a.nrhs + r) * 12 * BS + s;
        cx<A> rr[12], q[12];
        // del = psi_B on entry; MR adds alpha * r to it
        cx<A> del[RES::clover_half ? 1 : 12];
        {
            cx<A> d0[12];
            if (a.mode == 2) {
#pragma unroll
                for (int c = 0; c < 12; ++c) d0[c] = ldc_stream<A>(psi + sp + c * BS);
            } else {
#pragma unroll
                for (int c = 0; c < 12; ++c) d0[c] = mk<A>(0, 0);
            }
            // q = (D psi)_B: the block part, then the hops from the other colour
            if (a.mode == 2) {
                block_apply<S, A, RES>(L, a.g, b, bc, s, U, cl, links, clov, diag, d0, q);
            } else {
#pragma unroll
                for (int c = 0; c < 12; ++c) q[c] = mk<A>(0, 0);
            }
            if constexpr (RES::clover_half) {
#pragma unroll
                for (int c = 0; c < 12; ++c) D.d[c][s] = d0[c];
            } else {
#pragma unroll
                for (int c = 0; c < 12; ++c) del[c] = d0[c];
            }
        }
        if (a.mode != 0) face_hops<S, S, A, REGLINKS>(a.g, b, bc, s, r, a.nrhs, psi, links, U, q);
        // rho = eta - (D psi)_B
#pragma unroll
        for (int c = 0; c < 12; ++c) rr[c] = ldc_stream<A>(eta + sp + c * BS) - q[c];
        // MR on D_BB
        for (int it = 0; it < a.nmr; ++it) {
            block_apply<S, A, RES>(L, a.g, b, bc, s, U, cl, links, clov, diag, rr, q);
            cx<A> alpha;
            if (!mr_alpha(L, lane, wave, q, rr, alpha)) break;
            // delta += alpha r, then r -= alpha q
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                if constexpr (RES::clover_half) {
                    cx<A> d = D.d[c][s];
                    cmac(d, alpha, rr[c]);
                    D.d[c][s] = d;
                } else {
                    cmac(del[c], alpha, rr[c]);
                }
                rr[c] = rr[c] - alpha * q[c];
            }
        }
        if constexpr (RES::clover_half) {
#pragma unroll
            for (int c = 0; c < 12; ++c) stc_stream(psi + sp + c * BS, D.d[c][s]);
        } else {
#pragma unroll
            for (int c = 0; c < 12; ++c) stc_stream(psi + sp + c * BS, del[c]);
        }
    }
}

template <typename S, typename A, typename RES>
Status sweep(dd_ctx *ctx, const SArgs &a, int prec, const void *eta, void *psi)
{
    // algorithmic traffic of one colour sweep: links + clover once, eta, psi
    // (read only when nonzero) and psi written, per swept site and rhs
    const double sites = 256.0 * a.nblk, sb = (double)sizeof(S), n = a.nrhs;
    const double by = sites * (144.0 * sb + n * sb * (24.0 + 24.0 + (a.mode == 2 ? 24.0 : 0.0)));
    const double fl = sites * n * (a.nmr * 2184.0 + (a.mode == 2 ? 1848.0 : 0.0));
    ProfScope ps(ctx->prof, ctx->stream, prec == DD_F64 ? K_SAP_F64 : prec == DD_F32 ? K_SAP_F32 : K_SAP_F16, by, fl);
    k_sap_sweep<S, A, RES><<<a.nblk, BS, 0, ctx->stream>>>(
        static_cast<const vec2_t<S> *>(eta), static_cast<vec2_t<S> *>(psi),
        static_cast<const vec2_t<S> *>(ctx->links[prec].p), static_cast<const vec2_t<S> *>(ctx->clover[prec].p), a);
    DD_HIP_TRY(hipGetLastError());
    return Status::ok();
}

// Chosen by measurement on MI355X (32^3x64 colour sweep, single RHS):
// links in registers and the clover re-read from L2 per block application
// beat both "everything in registers" (one workgroup per CU, register
// pressure) and "everything from L2".
typedef Residency<true, false, 2, true> ResF32;
typedef Residency<true, false, 2, true> ResF16;
typedef Residency<true, false, 1, true> ResF64;

} // namespace

Status run_sap(dd_ctx *ctx, const double *m0, int nrhs, const void *eta, void *psi, int ncy, int nmr, int prec,
               const SapSlots *slots)
{
    if (!eta || !psi || !ctx->links[prec].p || !ctx->clover[prec].p || (!m0 && !(slots && slots->m0_dev)))
        return Status{DD_INVALID_ARG, "SAP: missing buffer"};
    if (ncy == 0) {
        if (slots) return Status{DD_INVALID_ARG, "SAP: zero cycles with per-slot offsets"};
        DD_HIP_TRY(hipMemsetAsync(psi, 0, spinor_bytes(ctx->g, prec, nrhs), ctx->stream));
        return Status::ok();
    }
    SArgs a{};
    for (int k = 0; k < 4; ++k) {
        a.g.nb[k] = ctx->g.nb[k];
        a.g.bstride[k] = ctx->g.bstride[k];
        a.g.bcs[k] = ctx->g.bcs[k];
    }
    a.g.nblocks = ctx->g.nblocks;
    a.nrhs = nrhs;
    a.nmr = nmr;
    for (int r = 0; r < nrhs && m0; ++r) a.m0[r] = m0[r];
    if (slots) {
        a.m0_dev = slots->m0_dev;
        a.eta_off = slots->eta_off;
        a.psi_off = slots->psi_off;
    }
    for (int cy = 0; cy < ncy; ++cy)
        for (int col = 0; col < 2; ++col) {
            if (ctx->ncolour[col] == 0) continue;
            a.blocks = ctx->colour_blocks[col].as<int>();
            a.nblk = ctx->ncolour[col];
            a.mode = (cy == 0 && col == 0) ? 0 : (cy == 0 ? 1 : 2);
            if (prec == DD_F64) DD_TRY((sweep<double, double, ResF64>(ctx, a, prec, eta, psi)));
            else if (prec == DD_F32) DD_TRY((sweep<float, float, ResF32>(ctx, a, prec, eta, psi)));
            else DD_TRY((sweep<__half, float, ResF16>(ctx, a, prec, eta, psi)));
        }
    return Status::ok();
}

} // namespace dd
