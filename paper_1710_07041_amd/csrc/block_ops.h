// Block-local building blocks shared by the SAP sweep and the operator
// kernel that works block by block: the LDS exchange that applies the hops
// inside a 4^4 block, the clover term, and the hops that leave the block.
//
// One 256-thread workgroup owns one block, one thread one site.  D_BB is
// applied direction by direction: each thread publishes the spin-projected
// half spinor of its site for the +mu hop of site x-mu, and U_mu(x)^+ times
// the projected half spinor for the -mu hop of site x+mu, through LDS; so
// every link of the block is read once and no in-block spinor is re-read
// from memory.
#pragma once

#include "dd_device.h"

namespace dd {

// Two buffers, used by alternate directions: direction mu + 2 overwrites the
// buffer of direction mu only after every thread has passed the barrier of
// direction mu + 1, i.e. after all reads of direction mu; so each direction
// needs one barrier, not two, as long as all four directions go through LDS.
// When the x, y and z hops go across lanes (exchange_dir with LANES) only
// buffer 1 (t) is used, with one barrier per application: two applications
// in a row then need a barrier between them (the caller's), or a slow
// wavefront could still be reading the first one's t hops while a fast one
// writes the second's.  The plain Schwarz sweep keeps each site's psi_B in
// buffer 0 meanwhile.
template <typename A> struct Lds {
    cx<A> hf[2][6][BS]; // projected half spinors for +mu hops
    cx<A> hb[2][6][BS]; // U^+ times projected half spinors for -mu hops
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
// workgroup runs) at every block application.  CLOVH keeps chiral half 0 of
// the clover term in registers and re-reads only half 1, which halves the
// clover footprint that has to stay in L2 across the MR steps.
template <bool REGLINKS, bool REGCLOV, int WAVES, bool CLOVH = false> struct Residency {
    static constexpr bool links = REGLINKS, clover = REGCLOV, clover_half = CLOVH && !REGCLOV;
    static constexpr int waves = WAVES;
    static constexpr int ncl = REGCLOV ? 36 : (CLOVH ? 18 : 1); // clover entries held in registers
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

// The complex value that lane (src4 / 4) of this wavefront holds in v
// (ds_bpermute: a cross-lane read, no LDS storage and no barrier).
template <typename A> __device__ __forceinline__ cx<A> lane_fetch(const cx<A> &v, int src4)
{
    if constexpr (sizeof(A) == 4) {
        return mk<A>(__int_as_float(__builtin_amdgcn_ds_bpermute(src4, __float_as_int(v.re))),
                     __int_as_float(__builtin_amdgcn_ds_bpermute(src4, __float_as_int(v.im))));
    } else {
        const long long r = __double_as_longlong(v.re), i = __double_as_longlong(v.im);
        const int r0 = __builtin_amdgcn_ds_bpermute(src4, (int)r), r1 = __builtin_amdgcn_ds_bpermute(src4, (int)(r >> 32));
        const int i0 = __builtin_amdgcn_ds_bpermute(src4, (int)i), i1 = __builtin_amdgcn_ds_bpermute(src4, (int)(i >> 32));
        return mk<A>(__longlong_as_double(((long long)r1 << 32) | (unsigned)r0),
                     __longlong_as_double(((long long)i1 << 32) | (unsigned)i0));
    }
}

// The x and y neighbours of a 4^4 block (site s = x + 4y + 16z + 64t on
// thread s) are lanes of the same quad (x) or 16-lane row (y): DPP moves
// reach them at VALU rate, rotating within the quad (x +- 1 mod 4) or the row
// (y +- 1 mod 4, i.e. lane +- 4 mod 16).  Lanes whose neighbour lies outside
// the block get their own block's wrapped site and never use it.  z crosses
// rows and keeps ds_bpermute.
template <int CTRL> __device__ __forceinline__ int dpp_mov(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xf, 0xf, false);
}
template <int MU, int DIR, typename A> __device__ __forceinline__ cx<A> lane_hop(const cx<A> &v, int sn)
{
    if constexpr (MU >= 2) {
        return lane_fetch<A>(v, (sn & 63) << 2);
    } else {
        // quad_perm [1,2,3,0] / [3,0,1,2]: lane k reads lane k + 1 / k - 1 of
        // its quad; row_ror:12 / row_ror:4: lane i reads lane i + 4 / i - 4
        // of its row of 16
        constexpr int CTRL = MU == 0 ? (DIR > 0 ? 0x39 : 0x93) : (DIR > 0 ? 0x12C : 0x124);
        if constexpr (sizeof(A) == 4) {
            return mk<A>(__int_as_float(dpp_mov<CTRL>(__float_as_int(v.re))),
                         __int_as_float(dpp_mov<CTRL>(__float_as_int(v.im))));
        } else {
            const long long r = __double_as_longlong(v.re), i = __double_as_longlong(v.im);
            const int r0 = dpp_mov<CTRL>((int)r), r1 = dpp_mov<CTRL>((int)(r >> 32));
            const int i0 = dpp_mov<CTRL>((int)i), i1 = dpp_mov<CTRL>((int)(i >> 32));
            return mk<A>(__longlong_as_double(((long long)r1 << 32) | (unsigned)r0),
                         __longlong_as_double(((long long)i1 << 32) | (unsigned)i0));
        }
    }
}

// One direction of the in-block exchange with the link given in registers,
// already multiplied by the hop factor -1/2.  With LANES (site s = x + 4y +
// 16z + 64t of the 4^4 block is thread s) a wavefront holds one t-slice: the
// x, y and z neighbours are lanes of the same wavefront and are read across
// lanes; only the t direction goes through LDS and a barrier.  Without LANES
// (another site-to-thread map) every direction goes through LDS.  In-block
// neighbours carry the boundary sign only when the block spans the whole
// direction (one block per direction); otherwise the reconstruction is a
// plain sum.
//
// PHASE splits a direction that goes through LDS: 1 posts this site's half
// spinors and returns, 2 waits at the barrier and takes the neighbours'
// (0 does both), so that other work can sit between the two.
template <int MU, typename S, typename A, bool LANES, int PHASE = 0>
__device__ __forceinline__ void exchange_dir(Lds<A> &L, const Geom &g, int b, const int bc[4], int s,
                                             const cx<A> U[9], const cx<A> v[12], cx<A> q[12])
{
    const bool wraps = g.nb[MU] == 1; // uniform
    if constexpr (LANES && MU < 3) {
        cx<A> h[6], t[6];
        int bn, snf, snb, sign_f, sign_b;
        bool inf, inbk;
        neighbour<MU, +1>(g, b, bc, s, bn, snf, sign_f, inf);
        neighbour<MU, -1>(g, b, bc, s, bn, snb, sign_b, inbk);
        // +mu hop: the neighbour's projected half spinor, times this site's link
        proj_minus<MU>(v, h);
#pragma unroll
        for (int c = 0; c < 6; ++c) t[c] = lane_hop<MU, +1, A>(h[c], snf);
        if (inf) {
            su3_mul(U, t, h);
            if (wraps) recon_minus<MU>(q, h, (A)sign_f);
            else recon_minus1<MU>(q, h);
        }
        // -mu hop: U^+ of the neighbour times its projected half spinor
        proj_plus<MU>(v, h);
        su3_mul_adj(U, h, t);
#pragma unroll
        for (int c = 0; c < 6; ++c) h[c] = lane_hop<MU, -1, A>(t[c], snb);
        if (inbk) {
            if (wraps) recon_plus<MU>(q, h, (A)sign_b);
            else recon_plus1<MU>(q, h);
        }
        return;
    }
    constexpr int X = MU & 1;
    cx<A> h[6], t[6];
    if constexpr (PHASE != 2) {
        proj_minus<MU>(v, h);
#pragma unroll
        for (int c = 0; c < 6; ++c) L.hf[X][c][s] = h[c];
        proj_plus<MU>(v, h);
        su3_mul_adj(U, h, t);
#pragma unroll
        for (int c = 0; c < 6; ++c) L.hb[X][c][s] = t[c];
    }
    if constexpr (PHASE == 1) return;
    __syncthreads();
    int bn, sn, sign;
    bool inb;
    neighbour<MU, +1>(g, b, bc, s, bn, sn, sign, inb);
    if (inb) {
#pragma unroll
        for (int c = 0; c < 6; ++c) h[c] = L.hf[X][c][sn];
        su3_mul(U, h, t);
        if (wraps) recon_minus<MU>(q, t, (A)sign);
        else recon_minus1<MU>(q, t);
    }
    neighbour<MU, -1>(g, b, bc, s, bn, sn, sign, inb);
    if (inb) {
#pragma unroll
        for (int c = 0; c < 6; ++c) t[c] = L.hb[X][c][sn];
        if (wraps) recon_plus<MU>(q, t, (A)sign);
        else recon_plus1<MU>(q, t);
    }
}

// q = D_BB v on the block (all threads of the workgroup take part; LANES:
// thread s holds site s, which lets the x, y and z hops stay inside a
// wavefront).  The loops over clover halves and directions are kept as loops
// so that only one step's loads are in flight per thread (unrolled, the
// compiler hoists them all and spills).
template <typename S, typename A, typename RES, bool NTC = false, bool LANES = true>
__device__ __forceinline__ void block_apply(Lds<A> &L, const Geom &g, int b, const int bc[4], int s,
                                            const cx<A> Ur[RES::links ? 4 : 1][9], const cx<A> cl[RES::ncl],
                                            const vec2_t<S> *__restrict__ links_g,
                                            const vec2_t<S> *__restrict__ clov_g, A diag, const cx<A> v[12],
                                            cx<A> q[12])
{
#pragma unroll
    for (int c = 0; c < 12; ++c) q[c] = mk<A>(0, 0);
    // FP16 fields: clover half 1 stays in flight as FP16 pairs across the
    // in-block hops and is applied after them, so its L2 latency hides behind
    // the hops (with FP32 fields the pending loads take twice the registers,
    // and that form measured slower)
    constexpr bool LATE = RES::clover_half && RES::links && sizeof(S) == 2;
    vec2_t<S> c2late[LATE ? 18 : 1];
    if constexpr (RES::clover) {
        clover_mac(cl, diag, v, q);
    } else if constexpr (RES::clover_half) {
        const vec2_t<S> *cp = clov_g + ((long)b * 36 + 18) * BS + s;
        // the address is the same at every MR step: hide that, or the loads
        // are hoisted out of the MR loop and the half is held in registers
        asm volatile("" : "+v"(cp));
        if constexpr (LATE) {
#pragma unroll
            for (int e = 0; e < 18; ++e) c2late[e] = cp[e * BS];
            clover_half_mac<A>(cl, diag, v, q);
        } else {
            // half 1's loads are in flight while half 0 (registers) is applied
            cx<A> c2[18];
#pragma unroll
            for (int e = 0; e < 18; ++e) c2[e] = ldc<A>(cp + e * BS);
            clover_half_mac<A>(cl, diag, v, q);
            clover_half_mac<A>(c2, diag, v + 6, q + 6);
        }
    } else {
#pragma unroll 1
        for (int k = 0; k < 2; ++k) {
            cx<A> c2[18];
            const vec2_t<S> *cp = clov_g + ((long)b * 36 + 18 * k) * BS + s;
#pragma unroll
            for (int e = 0; e < 18; ++e) c2[e] = NTC ? ldc_stream<A>(cp + e * BS) : ldc<A>(cp + e * BS);
            if (k == 0) clover_half_mac<A>(c2, diag, v, q);
            else clover_half_mac<A>(c2, diag, v + 6, q + 6);
        }
    }
    if constexpr (RES::links) {
        // links already in registers: no loads to hoist, unroll the
        // directions.  Across lanes, t alone goes through LDS: its half
        // spinors are posted first and taken last, so the x, y and z hops
        // run while the other wavefronts reach the barrier.
        if constexpr (LANES) {
            exchange_dir<3, S, A, LANES, 1>(L, g, b, bc, s, Ur[RES::links ? 3 : 0], v, q);
            exchange_dir<0, S, A, LANES>(L, g, b, bc, s, Ur[0], v, q);
            exchange_dir<1, S, A, LANES>(L, g, b, bc, s, Ur[RES::links ? 1 : 0], v, q);
            exchange_dir<2, S, A, LANES>(L, g, b, bc, s, Ur[RES::links ? 2 : 0], v, q);
            exchange_dir<3, S, A, LANES, 2>(L, g, b, bc, s, Ur[RES::links ? 3 : 0], v, q);
        } else {
            exchange_dir<0, S, A, LANES>(L, g, b, bc, s, Ur[0], v, q);
            exchange_dir<1, S, A, LANES>(L, g, b, bc, s, Ur[RES::links ? 1 : 0], v, q);
            exchange_dir<2, S, A, LANES>(L, g, b, bc, s, Ur[RES::links ? 2 : 0], v, q);
            exchange_dir<3, S, A, LANES>(L, g, b, bc, s, Ur[RES::links ? 3 : 0], v, q);
        }
        if constexpr (LATE) {
            cx<A> c2[18];
#pragma unroll
            for (int e = 0; e < 18; ++e) c2[e] = ldc<A>(&c2late[e]);
            clover_half_mac<A>(c2, diag, v + 6, q + 6);
        }
    } else {
#pragma unroll 1
    for (int mu = 0; mu < 4; ++mu) {
        cx<A> U[9], h[6], t[6];
        get_link<RES::links, S, A>(Ur, links_g, b, s, mu, U);
        const int X = mu & 1;
        proj_m(mu, v, h);
#pragma unroll
        for (int c = 0; c < 6; ++c) L.hf[X][c][s] = h[c];
        proj_p(mu, v, h);
        su3_mul_adj(U, h, t);
#pragma unroll
        for (int c = 0; c < 6; ++c) L.hb[X][c][s] = t[c];
        __syncthreads();
        int bn, sn, sign;
        bool inb;
        neighbour_rt(g, b, bc, s, mu, +1, bn, sn, sign, inb);
        if (inb) {
#pragma unroll
            for (int c = 0; c < 6; ++c) h[c] = L.hf[X][c][sn];
            su3_mul(U, h, t);
            recon_m(mu, q, t, (A)(sign > 0 ? -0.5f : 0.5f));
        }
        neighbour_rt(g, b, bc, s, mu, -1, bn, sn, sign, inb);
        if (inb) {
#pragma unroll
            for (int c = 0; c < 6; ++c) t[c] = L.hb[X][c][sn];
            recon_p(mu, q, t, (A)(sign > 0 ? -0.5f : 0.5f));
        }
    }
    }
}

// Hops of site s whose neighbour lies outside the block: read psi (and the
// neighbour's link for -mu hops) from memory and accumulate into q.  In a
// 4^4 block a site leaves the block in direction mu at most once (forward
// from the last layer, backward from the first), so one loop trip per
// direction serves both faces with one set of loads.
template <typename SP, typename S, typename A, bool REGLINKS>
__device__ __forceinline__ void face_hops(const Geom &g, int b, const int bc[4], int s, int r, int nrhs,
                                          const vec2_t<SP> *__restrict__ psi, const vec2_t<S> *__restrict__ links,
                                          const cx<A> Ur[REGLINKS ? 4 : 1][9], cx<A> q[12], bool r12)
{
#pragma unroll 1
    for (int mu = 0; mu < 4; ++mu) {
        const int l = (s >> (2 * mu)) & 3;
        if (l != 0 && l != BEXT - 1) continue;
        const int dir = l == 0 ? -1 : 1;
        int bn, sn, sign;
        bool inb;
        neighbour_rt(g, b, bc, s, mu, dir, bn, sn, sign, inb);
        if (inb) continue;
        cx<A> p[12], h[6], t[6], U[9];
        const vec2_t<SP> *pp = psi + ((long)bn * nrhs + r) * 12 * BS + sn;
#pragma unroll
        for (int c = 0; c < 12; ++c) p[c] = ldc<A>(pp + c * BS);
        if (!REGLINKS || dir < 0) {
            // issued before either branch's arithmetic waits on p
            const int lb = dir > 0 ? b : bn, ls = dir > 0 ? s : sn;
            load_link<A>(links + ((long)lb * 4 + mu) * 9 * BS + ls, r12, U);
        } else {
            // explicit branches: a switch would become a dynamic register index
            if (mu == 0) { for (int e = 0; e < 9; ++e) U[e] = Ur[0][e]; }
            else if (mu == 1) { for (int e = 0; e < 9; ++e) U[e] = Ur[REGLINKS ? 1 : 0][e]; }
            else if (mu == 2) { for (int e = 0; e < 9; ++e) U[e] = Ur[REGLINKS ? 2 : 0][e]; }
            else { for (int e = 0; e < 9; ++e) U[e] = Ur[REGLINKS ? 3 : 0][e]; }
        }
        const A kk = (A)(sign > 0 ? -0.5f : 0.5f);
        if (dir > 0) {
            // register links already hold -1/2: only the boundary sign remains
            const A kf = REGLINKS ? (A)sign : kk;
            proj_m(mu, p, h);
            su3_mul(U, h, t);
            recon_m(mu, q, t, kf);
        } else {
            proj_p(mu, p, h);
            su3_mul_adj(U, h, t);
            recon_p(mu, q, t, kk);
        }
    }
}

// ---------------------------------------------------------------------------
// Face buffers of the Schwarz sweep.  A block that has just been solved
// publishes, for each of its boundary sites and a spinor p (its update delta
// in the plain sweep, its psi in the even-odd sweep), the half spinor that
// the neighbouring block (of the other colour) needs for the hop into it:
//   face 2 mu     (sites with l_mu = 0): h = (1 - gamma_mu) p, projected,
//                 for the +mu hop of the block below, which applies its own
//                 link U_mu(x);
//   face 2 mu + 1 (sites with l_mu = 3): t = U~_mu(y)^+ (1 + gamma_mu) p,
//                 projected, with U~ = -U/2 the register-resident link, for
//                 the -mu hop of the block above.
// The consumer then reads six components per boundary hop, dense in a row of
// 64 face sites, instead of the neighbour's twelve (strided) and its link.
// Layout per block and right-hand side: [face 0..7][half-spinor comp. 0..5][64].
constexpr int FACE_ELEMS = 8 * 6 * 64; // = 12 * BS: one spinor's worth per block

// Position of site s in the face of direction mu (the other three
// coordinates, 2 bits each, in order).
__device__ __forceinline__ int face_index(int s, int mu)
{
    const int lo = s & ((1 << (2 * mu)) - 1);
    return lo | ((s >> (2 * mu + 2)) << (2 * mu));
}

// The same hops computed cooperatively by the workgroup: the 8 faces x 64
// sites of a 4^4 block are 512 hops, two per thread, with the face (and so
// mu and the direction) uniform over each wavefront: wavefront w takes face
// w (mu = w/2) and face w + 4 (mu = 2 + w/2), face 2 mu being the sites with
// l_mu = 0 (hop from x - mu) and face 2 mu + 1 those with l_mu = 3.  Each
// hop's transported half spinor, times -1/2 and the boundary sign, goes to
// FB0 (faces 0-3) or FB1 (faces 4-7) at [component][face mod 4][64], i.e. at
// [component][thread]; after the caller's next barrier face_gather adds them
// to their sites.  Compared with the per-site loop this takes two memory
// round trips per right-hand side instead of four, and no lane idles.
template <typename SP, typename SF, typename A>
__device__ __forceinline__ void face_hops_coop(const Geom &g, int b, const int bc[4], int s, int r, int nrhs,
                                               const vec2_t<SP> *__restrict__ psi,
                                               const vec2_t<SF> *__restrict__ links, bool r12, cx<A> *FB0,
                                               cx<A> *FB1)
{
    const int w = s >> 6, k = s & 63;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int f = w + 4 * j;
        const int mu = f >> 1, dir = (f & 1) ? 1 : -1;
        if (g.nb[mu] == 1) continue; // uniform: the in-block exchange wraps
        const int lo = k & ((1 << (2 * mu)) - 1);
        const int x = lo | ((dir > 0 ? BEXT - 1 : 0) << (2 * mu)) | ((k >> (2 * mu)) << (2 * mu + 2));
        int bn, sn, sign;
        bool inb;
        neighbour_rt(g, b, bc, x, mu, dir, bn, sn, sign, inb);
        cx<A> p[12], h[6], t[6], U[9];
        const vec2_t<SP> *pp = psi + ((long)bn * nrhs + r) * 12 * BS + sn;
#pragma unroll
        for (int c = 0; c < 12; ++c) p[c] = ldc<A>(pp + c * BS);
        // the forward hop takes this site's link, the backward one the
        // neighbour's (both as stored: the factor -1/2 is applied below)
        const int lb = dir > 0 ? b : bn, ls = dir > 0 ? x : sn;
        load_link<A>(links + ((long)lb * 4 + mu) * 9 * BS + ls, r12, U);
        if (dir > 0) {
            proj_m(mu, p, h);
            su3_mul(U, h, t);
        } else {
            proj_p(mu, p, h);
            su3_mul_adj(U, h, t);
        }
        const A kk = (A)(-0.5f * sign);
        cx<A> *fb = j == 0 ? FB0 : FB1;
#pragma unroll
        for (int c = 0; c < 6; ++c) fb[c * BS + s] = kk * t[c];
    }
}

// q += the face hops of site s from the buffers face_hops_coop wrote.
template <int MU, typename A>
__device__ __forceinline__ void face_gather_dir(const Geom &g, int s, const cx<A> *FB0, const cx<A> *FB1,
                                                cx<A> q[12])
{
    if (g.nb[MU] == 1) return;
    const int l = (s >> (2 * MU)) & 3;
    if (l != 0 && l != BEXT - 1) return;
    const int f = 2 * MU + (l == 0 ? 0 : 1);
    const cx<A> *fb = (f < 4 ? FB0 : FB1) + (f & 3) * 64 + face_index(s, MU);
    cx<A> t[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) t[c] = fb[c * BS];
    if (l == 0) recon_plus1<MU>(q, t);
    else recon_minus1<MU>(q, t);
}
template <typename A>
__device__ __forceinline__ void face_gather(const Geom &g, int s, const cx<A> *FB0, const cx<A> *FB1, cx<A> q[12])
{
    face_gather_dir<0, A>(g, s, FB0, FB1, q);
    face_gather_dir<1, A>(g, s, FB0, FB1, q);
    face_gather_dir<2, A>(g, s, FB0, FB1, q);
    face_gather_dir<3, A>(g, s, FB0, FB1, q);
}

template <typename S, typename A>
__device__ __forceinline__ void face_publish(vec2_t<S> *__restrict__ F, int b, int nrhs, int r, int s,
                                             const cx<A> p[12], const cx<A> Ur[4][9])
{
    vec2_t<S> *base = F + ((long)b * nrhs + r) * FACE_ELEMS;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        const int l = (s >> (2 * mu)) & 3;
        cx<A> h[6], t[6];
        if (l == 0) {
            proj_m(mu, p, h);
            vec2_t<S> *fp = base + (2 * mu) * 6 * 64 + face_index(s, mu);
#pragma unroll
            for (int e = 0; e < 6; ++e) stc(fp + e * 64, h[e]);
        } else if (l == BEXT - 1) {
            proj_p(mu, p, h);
            su3_mul_adj(Ur[mu], h, t);
            vec2_t<S> *fp = base + (2 * mu + 1) * 6 * 64 + face_index(s, mu);
#pragma unroll
            for (int e = 0; e < 6; ++e) stc(fp + e * 64, t[e]);
        }
    }
}

// The boundary hops of site s from the faces the neighbouring blocks
// published, accumulated into q (one direction per trip: the register
// budget of the sweep has no room for more face data in flight).
template <typename S, typename A>
__device__ __forceinline__ void face_consume(const Geom &g, int b, const int bc[4], int s, int r, int nrhs,
                                             const vec2_t<S> *__restrict__ F, const cx<A> Ur[4][9], cx<A> q[12])
{
#pragma unroll 1
    for (int mu = 0; mu < 4; ++mu) {
        const int l = (s >> (2 * mu)) & 3;
        if (l != 0 && l != BEXT - 1) continue;
        const int dir = l == 0 ? -1 : 1;
        int bn, sn, sign;
        bool inb;
        neighbour_rt(g, b, bc, s, mu, dir, bn, sn, sign, inb);
        if (inb) continue;
        // the +mu face of the block below, or the -mu face of the block above
        const vec2_t<S> *fp =
            F + ((long)bn * nrhs + r) * FACE_ELEMS + (2 * mu + (dir < 0 ? 1 : 0)) * 6 * 64 + face_index(s, mu);
        cx<A> h[6], t[6], U[9];
#pragma unroll
        for (int e = 0; e < 6; ++e) h[e] = ldc<A>(fp + e * 64);
        // U~ and the published t carry -1/2: only the boundary sign remains
        if (dir > 0) {
            // explicit branches: a switch would become a dynamic register index
            if (mu == 0) { for (int e = 0; e < 9; ++e) U[e] = Ur[0][e]; }
            else if (mu == 1) { for (int e = 0; e < 9; ++e) U[e] = Ur[1][e]; }
            else if (mu == 2) { for (int e = 0; e < 9; ++e) U[e] = Ur[2][e]; }
            else { for (int e = 0; e < 9; ++e) U[e] = Ur[3][e]; }
            su3_mul(U, h, t);
            recon_m(mu, q, t, (A)sign);
        } else {
            recon_p(mu, q, h, (A)sign);
        }
    }
}

// One DPP step of the wavefront sum: v + (v moved by ctrl), with rows outside
// row_mask (and invalid source lanes) adding zero.
template <int CTRL, int ROWS> __device__ __forceinline__ float dpp_add(float v)
{
    return v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xf, true));
}
template <int CTRL, int ROWS> __device__ __forceinline__ double dpp_add(double v)
{
    const long long x = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROWS, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(x >> 32), CTRL, ROWS, 0xf, true);
    return v + __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum over the 64 lanes of a wavefront in a fixed order, with cross-lane DPP
// moves (no LDS round trips): pairs, quads, half rows and rows of 16, then
// row 1 += row 0 and row 3 += row 2 (row_bcast:15), then rows 2-3 += the
// first half (row_bcast:31).  The total is valid in lane 63 only.
template <typename A> __device__ __forceinline__ A wave_sum(A v)
{
    v = dpp_add<0xB1, 0xf>(v);  // quad_perm [1,0,3,2]
    v = dpp_add<0x4E, 0xf>(v);  // quad_perm [2,3,0,1]
    v = dpp_add<0x141, 0xf>(v); // row_half_mirror
    v = dpp_add<0x140, 0xf>(v); // row_mirror
    v = dpp_add<0x142, 0xa>(v); // row_bcast:15
    v = dpp_add<0x143, 0xc>(v); // row_bcast:31
    return v;
}


} // namespace dd
