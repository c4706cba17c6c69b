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

template <typename A> struct Lds {
    cx<A> hf[6][BS]; // projected half spinors for +mu hops
    cx<A> hb[6][BS]; // U^+ times projected half spinors for -mu hops
    A red[4][4];
};

// Direction-dispatched spin algebra for run-time loops over mu (a switch on a
// uniform value; each case is the compile-time specialisation).
template <typename A> __device__ __forceinline__ void proj_m(int mu, const cx<A> v[12], cx<A> h[6])
{
    switch (mu) {
    case 0: proj_minus<0>(v, h); break;
    case 1: proj_minus<1>(v, h); break;
    case 2: proj_minus<2>(v, h); break;
    default: proj_minus<3>(v, h); break;
    }
}
template <typename A> __device__ __forceinline__ void proj_p(int mu, const cx<A> v[12], cx<A> h[6])
{
    switch (mu) {
    case 0: proj_plus<0>(v, h); break;
    case 1: proj_plus<1>(v, h); break;
    case 2: proj_plus<2>(v, h); break;
    default: proj_plus<3>(v, h); break;
    }
}
template <typename A> __device__ __forceinline__ void recon_m(int mu, cx<A> q[12], const cx<A> t[6], A k)
{
    switch (mu) {
    case 0: recon_minus<0>(q, t, k); break;
    case 1: recon_minus<1>(q, t, k); break;
    case 2: recon_minus<2>(q, t, k); break;
    default: recon_minus<3>(q, t, k); break;
    }
}
template <typename A> __device__ __forceinline__ void recon_p(int mu, cx<A> q[12], const cx<A> t[6], A k)
{
    switch (mu) {
    case 0: recon_plus<0>(q, t, k); break;
    case 1: recon_plus<1>(q, t, k); break;
    case 2: recon_plus<2>(q, t, k); break;
    default: recon_plus<3>(q, t, k); break;
    }
}

// Where the per-site fields live during a sweep: in registers for the whole
// sweep, or re-read (from L2: one block's fields stay resident while its
// workgroup runs) at every block application.
template <bool REGLINKS, bool REGCLOV, int WAVES> struct Residency {
    static constexpr bool links = REGLINKS, clover = REGCLOV;
    static constexpr int waves = WAVES;
};

template <bool REG, typename S, typename A>
__device__ __forceinline__ void get_link(const cx<A> Ur[4][9], const vec2_t<S> *__restrict__ links, int b, int s,
                                         int mu, cx<A> U[9])
{
    if (REG) {
        switch (mu) {
        case 0:
#pragma unroll
            for (int e = 0; e < 9; ++e) U[e] = Ur[0][e];
            break;
        case 1:
#pragma unroll
            for (int e = 0; e < 9; ++e) U[e] = Ur[REG ? 1 : 0][e];
            break;
        case 2:
#pragma unroll
            for (int e = 0; e < 9; ++e) U[e] = Ur[REG ? 2 : 0][e];
            break;
        default:
#pragma unroll
            for (int e = 0; e < 9; ++e) U[e] = Ur[REG ? 3 : 0][e];
            break;
        }
    } else {
        const vec2_t<S> *u = links + ((long)b * 4 + mu) * 9 * BS + s;
#pragma unroll
        for (int e = 0; e < 9; ++e) U[e] = ldc<A>(u + e * BS);
    }
}

// One direction of the LDS exchange with the link given in registers, already
// multiplied by the hop factor -1/2.  In-block neighbours carry the boundary
// sign only when the block spans the whole direction (one block per
// direction); otherwise the reconstruction is a plain sum.
template <int MU, typename S, typename A>
__device__ __forceinline__ void exchange_dir(Lds<A> &L, const Geom &g, int b, const int bc[4], int s,
                                             const cx<A> U[9], const cx<A> v[12], cx<A> q[12])
{
    const bool wraps = g.nb[MU] == 1; // uniform
    cx<A> h[6], t[6];
    proj_minus<MU>(v, h);
#pragma unroll
    for (int c = 0; c < 6; ++c) L.hf[c][s] = h[c];
    proj_plus<MU>(v, h);
    su3_mul_adj(U, h, t);
#pragma unroll
    for (int c = 0; c < 6; ++c) L.hb[c][s] = t[c];
    __syncthreads();
    int bn, sn, sign;
    bool inb;
    neighbour<MU, +1>(g, b, bc, s, bn, sn, sign, inb);
    if (inb) {
#pragma unroll
        for (int c = 0; c < 6; ++c) h[c] = L.hf[c][sn];
        su3_mul(U, h, t);
        if (wraps) recon_minus<MU>(q, t, (A)sign);
        else recon_minus1<MU>(q, t);
    }
    neighbour<MU, -1>(g, b, bc, s, bn, sn, sign, inb);
    if (inb) {
#pragma unroll
        for (int c = 0; c < 6; ++c) t[c] = L.hb[c][sn];
        if (wraps) recon_plus<MU>(q, t, (A)sign);
        else recon_plus1<MU>(q, t);
    }
    __syncthreads();
}

// q = D_BB v on the block (all threads of the workgroup take part).  The
// loops over clover halves and directions are kept as loops so that only one
// step's loads are in flight per thread (unrolled, the compiler hoists them
// all and spills).
template <typename S, typename A, typename RES>
__device__ __forceinline__ void block_apply(Lds<A> &L, const Geom &g, int b, const int bc[4], int s,
                                            const cx<A> Ur[RES::links ? 4 : 1][9], const cx<A> cl[36],
                                            const vec2_t<S> *__restrict__ links_g,
                                            const vec2_t<S> *__restrict__ clov_g, A diag, const cx<A> v[12],
                                            cx<A> q[12])
{
#pragma unroll
    for (int c = 0; c < 12; ++c) q[c] = mk<A>(0, 0);
    if (RES::clover) {
        clover_mac(cl, diag, v, q);
    } else {
#pragma unroll 1
        for (int k = 0; k < 2; ++k) {
            cx<A> c2[18];
            const vec2_t<S> *cp = clov_g + ((long)b * 36 + 18 * k) * BS + s;
#pragma unroll
            for (int e = 0; e < 18; ++e) c2[e] = ldc<A>(cp + e * BS);
            if (k == 0) clover_half_mac<A>(c2, diag, v, q);
            else clover_half_mac<A>(c2, diag, v + 6, q + 6);
        }
    }
    if constexpr (RES::links) {
        // links already in registers: no loads to hoist, unroll the directions
        exchange_dir<0, S, A>(L, g, b, bc, s, Ur[0], v, q);
        exchange_dir<1, S, A>(L, g, b, bc, s, Ur[RES::links ? 1 : 0], v, q);
        exchange_dir<2, S, A>(L, g, b, bc, s, Ur[RES::links ? 2 : 0], v, q);
        exchange_dir<3, S, A>(L, g, b, bc, s, Ur[RES::links ? 3 : 0], v, q);
    } else {
#pragma unroll 1
    for (int mu = 0; mu < 4; ++mu) {
        cx<A> U[9], h[6], t[6];
        get_link<RES::links, S, A>(Ur, links_g, b, s, mu, U);
        proj_m(mu, v, h);
#pragma unroll
        for (int c = 0; c < 6; ++c) L.hf[c][s] = h[c];
        proj_p(mu, v, h);
        su3_mul_adj(U, h, t);
#pragma unroll
        for (int c = 0; c < 6; ++c) L.hb[c][s] = t[c];
        __syncthreads();
        int bn, sn, sign;
        bool inb;
        neighbour_rt(g, b, bc, s, mu, +1, bn, sn, sign, inb);
        if (inb) {
#pragma unroll
            for (int c = 0; c < 6; ++c) h[c] = L.hf[c][sn];
            su3_mul(U, h, t);
            recon_m(mu, q, t, (A)(sign > 0 ? -0.5f : 0.5f));
        }
        neighbour_rt(g, b, bc, s, mu, -1, bn, sn, sign, inb);
        if (inb) {
#pragma unroll
            for (int c = 0; c < 6; ++c) t[c] = L.hb[c][sn];
            recon_p(mu, q, t, (A)(sign > 0 ? -0.5f : 0.5f));
        }
        __syncthreads();
    }
    }
}

// Hops of site s whose neighbour lies outside the block: read psi (and the
// neighbour's link for -mu hops) from memory and accumulate into q.  One hop
// per loop trip.
template <typename S, typename A, bool REGLINKS>
__device__ __forceinline__ void face_hops(const Geom &g, int b, const int bc[4], int s, int r, int nrhs,
                                          const vec2_t<S> *__restrict__ psi, const vec2_t<S> *__restrict__ links,
                                          const cx<A> Ur[REGLINKS ? 4 : 1][9], cx<A> q[12])
{
#pragma unroll 1
    for (int k = 0; k < 8; ++k) {
        const int mu = k >> 1, dir = (k & 1) ? -1 : 1;
        int bn, sn, sign;
        bool inb;
        neighbour_rt(g, b, bc, s, mu, dir, bn, sn, sign, inb);
        if (inb) continue;
        cx<A> p[12], h[6], t[6], U[9];
        const vec2_t<S> *pp = psi + ((long)bn * nrhs + r) * 12 * BS + sn;
#pragma unroll
        for (int c = 0; c < 12; ++c) p[c] = ldc<A>(pp + c * BS);
        const A kk = (A)(sign > 0 ? -0.5f : 0.5f);
        if (dir > 0) {
            // register links already hold -1/2: only the boundary sign remains
            const A kf = REGLINKS ? (A)sign : kk;
            if (REGLINKS) {
                // explicit branches: a switch would become a dynamic register index
                if (mu == 0) { for (int e = 0; e < 9; ++e) U[e] = Ur[0][e]; }
                else if (mu == 1) { for (int e = 0; e < 9; ++e) U[e] = Ur[REGLINKS ? 1 : 0][e]; }
                else if (mu == 2) { for (int e = 0; e < 9; ++e) U[e] = Ur[REGLINKS ? 2 : 0][e]; }
                else { for (int e = 0; e < 9; ++e) U[e] = Ur[REGLINKS ? 3 : 0][e]; }
            } else {
                get_link<false, S, A>(Ur, links, b, s, mu, U);
            }
            proj_m(mu, p, h);
            su3_mul(U, h, t);
            recon_m(mu, q, t, kf);
        } else {
            const vec2_t<S> *u = links + ((long)bn * 4 + mu) * 9 * BS + sn;
#pragma unroll
            for (int e = 0; e < 9; ++e) U[e] = ldc<A>(u + e * BS);
            proj_p(mu, p, h);
            su3_mul_adj(U, h, t);
            recon_p(mu, q, t, kk);
        }
    }
}

template <typename A> __device__ __forceinline__ A wave_sum(A v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <typename S, typename A, typename RES>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(RES::waves))) void k_sap_sweep(
    const vec2_t<S> *__restrict__ eta0, vec2_t<S> *__restrict__ psi0, const vec2_t<S> *__restrict__ links,
    const vec2_t<S> *__restrict__ clov, SArgs a)
{
    constexpr bool REGCLOV = RES::clover, REGLINKS = RES::links;
    __shared__ Lds<A> L;
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
            for (int e = 0; e < 9; ++e) U[mu][e] = (A)(-0.5) * ldc<A>(u + e * BS);
        }
    }
    cx<A> cl[REGCLOV ? 36 : 1];
    if (REGCLOV) {
        const vec2_t<S> *cp = clov + (long)b * 36 * BS + s;
#pragma unroll
        for (int e = 0; e < (REGCLOV ? 36 : 1); ++e) cl[e] = ldc<A>(cp + e * BS);
    }

    for (int r = 0; r < a.nrhs; ++r) {
        const A diag = (A)(4.0 + (a.m0_dev ? a.m0_dev[r] : a.m0[r]));
        const vec2_t<S> *__restrict__ eta = eta0 + (a.eta_off ? a.eta_off[r] : 0);
        vec2_t<S> *__restrict__ psi = psi0 + (a.psi_off ? a.psi_off[r] : 0);
        const long sp = ((long)b * a.nrhs + r) * 12 * BS + s;
        cx<A> rr[12], del[12], q[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) rr[c] = ldc<A>(eta + sp + c * BS);
        if (a.mode == 2) {
#pragma unroll
            for (int c = 0; c < 12; ++c) del[c] = ldc<A>(psi + sp + c * BS);
        } else {
#pragma unroll
            for (int c = 0; c < 12; ++c) del[c] = mk<A>(0, 0);
        }
        if (a.mode != 0) {
            // rho = eta - (D psi)_B ; psi_B is held in del
            if (a.mode == 2) {
                block_apply<S, A, RES>(L, a.g, b, bc, s, U, cl, links, clov, diag, del, q);
            } else {
#pragma unroll
                for (int c = 0; c < 12; ++c) q[c] = mk<A>(0, 0);
            }
            face_hops<S, A, REGLINKS>(a.g, b, bc, s, r, a.nrhs, psi, links, U, q);
#pragma unroll
            for (int c = 0; c < 12; ++c) rr[c] = rr[c] - q[c];
        }
        // MR on D_BB: del accumulates alpha * r on top of psi_B
        for (int it = 0; it < a.nmr; ++it) {
            block_apply<S, A, RES>(L, a.g, b, bc, s, U, cl, links, clov, diag, rr, q);
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
            if (qq == (A)0) break; // uniform across the workgroup
            const cx<A> alpha = mk<A>(qr_re / qq, qr_im / qq);
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                cmac(del[c], alpha, rr[c]);
                rr[c] = rr[c] - alpha * q[c];
            }
        }
#pragma unroll
        for (int c = 0; c < 12; ++c) stc(psi + sp + c * BS, del[c]);
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
typedef Residency<true, false, 2> ResF32;
typedef Residency<true, false, 1> ResF16;
typedef Residency<true, false, 1> ResF64;

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
