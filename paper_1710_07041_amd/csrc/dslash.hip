// Wilson-clover operator on the blocked layout.
//
//   (D psi)(x) = (4 + m0) psi(x) + C(x) psi(x)
//              - 1/2 sum_mu [ (1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu(x-mu)^+ psi(x-mu) ]
//
// Gather form (k_dslash): one thread per site, one 256-thread workgroup per
// (Schwarz block, group of RT right-hand sides); the RT right-hand sides of a
// thread share every link and clover load.  The hop uses the chiral-basis
// spin projection so each of the eight SU(3) products acts on two spins only.
// Block-wise form (k_dslash_lds, FP32 fields with many right-hand sides):
// links and clover in registers for all right-hand sides, in-block hops
// through the LDS exchange of the smoother.
// Bandwidth bound: per site the algorithmic traffic is links 72 + clover 72 +
// spinor in 24 + out 24 reals per right-hand side.  Workgroups are remapped
// so that each XCD sweeps a contiguous range of blocks (shared L2 for the
// neighbour faces); clover terms and outputs, used once, go through
// streaming loads/stores.
#include "block_ops.h"
#include "dd_device.h"
#include "dd_internal.h"

namespace dd {

namespace {

struct DArgs {
    Geom g;
    int nrhs;
    int ngroups; // groups of RT right-hand sides (ceil(nrhs / RT))
    int block_id;
    double m0[MAXRHS];
    const double *m0_dev; // per-rhs masses in device memory (overrides m0 when set)
    const long *in_off;   // per-rhs element offset added to the input (nullable)
    const int *active;    // right-hand sides with active[r] == 0 are skipped (nullable)
    int r12;              // links stored as SU(3): read two rows, rebuild the third
};

// One hop of direction index k = 2 mu + (0: forward, 1: backward) onto acc.
template <int K, typename A>
__device__ __forceinline__ void hop_k(const cx<A> psi[12], const cx<A> U[9], A kk, cx<A> acc[12])
{
    cx<A> h[6], uh[6];
    if (K & 1) {
        proj_plus<K / 2>(psi, h);
        su3_mul_adj(U, h, uh);
        recon_plus<K / 2>(acc, uh, kk);
    } else {
        proj_minus<K / 2>(psi, h);
        su3_mul(U, h, uh);
        recon_minus<K / 2>(acc, uh, kk);
    }
}

// The RT right-hand sides of one hop share the link: it is loaded once and
// applied to each of them.  All RT spinor loads are issued before any
// arithmetic (no branch between them, so they are in flight together);
// slots beyond the last right-hand side re-read the first one and their
// results are never stored.
template <int K, int RT, typename SI, typename A>
__device__ __forceinline__ void hop_rhs(const vec2_t<SI> *__restrict__ in, const long ro[RT], const cx<A> U[9],
                                        A kk, cx<A> acc[RT][12])
{
    // held in the storage type until used (half the registers for FP32
    // input to FP64 arithmetic)
    vec2_t<SI> raw[RT][12];
#pragma unroll
    for (int rr = 0; rr < RT; ++rr)
#pragma unroll
        for (int c = 0; c < 12; ++c) raw[rr][c] = in[ro[rr] + c * BS];
#pragma unroll
    for (int rr = 0; rr < RT; ++rr) {
        cx<A> psi[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) psi[c] = ldc<A>(&raw[rr][c]);
        hop_k<K, A>(psi, U, kk, acc[rr]);
    }
}

// The eight hops run as a loop that is deliberately not unrolled: unrolled,
// the compiler hoists all hops' loads ahead of the arithmetic and spills.
// With PF the link of the next hop is loaded one trip ahead (registers
// permitting), so only the spinor loads of a hop wait a full round trip.
template <int RT, typename SI, typename A>
__device__ __forceinline__ void hop_switch(int k, const vec2_t<SI> *__restrict__ p, const long ro[RT],
                                           const cx<A> U[9], A kk, cx<A> acc[RT][12])
{
    switch (k) {
    case 0: hop_rhs<0, RT, SI, A>(p, ro, U, kk, acc); break;
    case 1: hop_rhs<1, RT, SI, A>(p, ro, U, kk, acc); break;
    case 2: hop_rhs<2, RT, SI, A>(p, ro, U, kk, acc); break;
    case 3: hop_rhs<3, RT, SI, A>(p, ro, U, kk, acc); break;
    case 4: hop_rhs<4, RT, SI, A>(p, ro, U, kk, acc); break;
    case 5: hop_rhs<5, RT, SI, A>(p, ro, U, kk, acc); break;
    case 6: hop_rhs<6, RT, SI, A>(p, ro, U, kk, acc); break;
    default: hop_rhs<7, RT, SI, A>(p, ro, U, kk, acc); break;
    }
}

// The staged form (one right-hand side per workgroup): the block's own input
// spinor is in LDS, so an in-block neighbour is read from there and only a
// neighbour across the block face comes from memory (those lanes alone).
template <int K, typename SI, typename A>
__device__ __forceinline__ void hop_stg(const vec2_t<SI> *__restrict__ g, const vec2_t<SI> *stg, int sn, bool inb,
                                        const cx<A> U[9], A kk, cx<A> acc[12])
{
    vec2_t<SI> raw[12];
    if (inb) {
#pragma unroll
        for (int c = 0; c < 12; ++c) raw[c] = stg[c * BS + sn];
    } else {
#pragma unroll
        for (int c = 0; c < 12; ++c) raw[c] = g[c * BS];
    }
    cx<A> psi[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) psi[c] = ldc<A>(&raw[c]);
    hop_k<K, A>(psi, U, kk, acc);
}

template <typename SI, typename A>
__device__ __forceinline__ void hop_stg_switch(int k, const vec2_t<SI> *__restrict__ g, const vec2_t<SI> *stg, int sn,
                                               bool inb, const cx<A> U[9], A kk, cx<A> acc[12])
{
    switch (k) {
    case 0: hop_stg<0, SI, A>(g, stg, sn, inb, U, kk, acc); break;
    case 1: hop_stg<1, SI, A>(g, stg, sn, inb, U, kk, acc); break;
    case 2: hop_stg<2, SI, A>(g, stg, sn, inb, U, kk, acc); break;
    case 3: hop_stg<3, SI, A>(g, stg, sn, inb, U, kk, acc); break;
    case 4: hop_stg<4, SI, A>(g, stg, sn, inb, U, kk, acc); break;
    case 5: hop_stg<5, SI, A>(g, stg, sn, inb, U, kk, acc); break;
    case 6: hop_stg<6, SI, A>(g, stg, sn, inb, U, kk, acc); break;
    default: hop_stg<7, SI, A>(g, stg, sn, inb, U, kk, acc); break;
    }
}

template <typename SF, typename A>
__device__ __forceinline__ void load_hop_link(const vec2_t<SF> *__restrict__ links, int b, int s, int k, int bn,
                                              int sn, bool r12, cx<A> U[9])
{
    const int mu = k >> 1;
    const int lb = (k & 1) ? bn : b, ls = (k & 1) ? sn : s;
    load_link<A>(links + ((long)lb * 4 + mu) * 9 * BS + ls, r12, U);
}

template <bool BLOCKONLY, bool PF, bool PAIR, int RT, typename SI, typename SF, typename A, bool STG = false>
__device__ __forceinline__ void hops(const vec2_t<SI> *__restrict__ in, const vec2_t<SF> *__restrict__ links,
                                     const DArgs &a, int b, const int bc[4], int r0, const long ro[RT], int s,
                                     cx<A> acc[RT][12], const vec2_t<SI> *stg = nullptr)
{
    if constexpr (STG && PAIR) {
        // FP32 input: the pair form below with the in-block neighbours from
        // the LDS copy of the block
        static_assert(!BLOCKONLY && RT == 1, "the staged forms take one right-hand side");
#pragma unroll 1
        for (int mu = 0; mu < 4; ++mu) {
            int bf, sf, gf, bb, sb, gb;
            bool inf, inbk;
            neighbour_rt(a.g, b, bc, s, mu, +1, bf, sf, gf, inf);
            neighbour_rt(a.g, b, bc, s, mu, -1, bb, sb, gb, inbk);
            vec2_t<SI> pf[12], pb[12];
            cx<A> Uf[9], Ub[9];
            if (inf) {
#pragma unroll
                for (int c = 0; c < 12; ++c) pf[c] = stg[c * BS + sf];
            } else {
                const vec2_t<SI> *qf = in + ro[0] + ((long)bf * a.nrhs + r0) * 12 * BS + sf;
#pragma unroll
                for (int c = 0; c < 12; ++c) pf[c] = qf[c * BS];
            }
            load_hop_link<SF, A>(links, b, s, 2 * mu, bf, sf, a.r12, Uf);
            if (inbk) {
#pragma unroll
                for (int c = 0; c < 12; ++c) pb[c] = stg[c * BS + sb];
            } else {
                const vec2_t<SI> *qb = in + ro[0] + ((long)bb * a.nrhs + r0) * 12 * BS + sb;
#pragma unroll
                for (int c = 0; c < 12; ++c) pb[c] = qb[c * BS];
            }
            load_hop_link<SF, A>(links, b, s, 2 * mu + 1, bb, sb, a.r12, Ub);
            cx<A> psi[12];
#pragma unroll
            for (int c = 0; c < 12; ++c) psi[c] = ldc<A>(&pf[c]);
            const A kf = (A)(-0.5 * gf), kb = (A)(-0.5 * gb);
            switch (mu) {
            case 0: hop_k<0, A>(psi, Uf, kf, acc[0]); break;
            case 1: hop_k<2, A>(psi, Uf, kf, acc[0]); break;
            case 2: hop_k<4, A>(psi, Uf, kf, acc[0]); break;
            default: hop_k<6, A>(psi, Uf, kf, acc[0]); break;
            }
#pragma unroll
            for (int c = 0; c < 12; ++c) psi[c] = ldc<A>(&pb[c]);
            switch (mu) {
            case 0: hop_k<1, A>(psi, Ub, kb, acc[0]); break;
            case 1: hop_k<3, A>(psi, Ub, kb, acc[0]); break;
            case 2: hop_k<5, A>(psi, Ub, kb, acc[0]); break;
            default: hop_k<7, A>(psi, Ub, kb, acc[0]); break;
            }
        }
    } else if constexpr (STG) {
        static_assert(PF && !BLOCKONLY && RT == 1, "the staged form is the link-prefetch form with one right-hand side");
        // FP64 input: in-block neighbours from the LDS copy of the block
        // (stg), face neighbours from memory; the next hop's link one trip
        // ahead as below
        int bn, sn, sign;
        bool inb;
        neighbour_rt(a.g, b, bc, s, 0, +1, bn, sn, sign, inb);
        cx<A> U[9];
        load_hop_link<SF, A>(links, b, s, 0, bn, sn, a.r12, U);
#pragma unroll 1
        for (int k = 0; k < 8; ++k) {
            const vec2_t<SI> *p = in + ro[0] + ((long)bn * a.nrhs + r0) * 12 * BS + sn;
            const A kk = (A)(-0.5 * sign);
            int bn2 = bn, sn2 = sn, sign2 = sign;
            bool inb2 = inb;
            cx<A> Un[9];
            if (k < 7) { // uniform
                const int k2 = k + 1;
                neighbour_rt(a.g, b, bc, s, k2 >> 1, (k2 & 1) ? -1 : 1, bn2, sn2, sign2, inb2);
                load_hop_link<SF, A>(links, b, s, k2, bn2, sn2, a.r12, Un);
            }
            hop_stg_switch<SI, A>(k, p, stg, sn, inb, U, kk, acc[0]);
#pragma unroll
            for (int e = 0; e < 9; ++e) U[e] = Un[e];
            bn = bn2;
            sn = sn2;
            sign = sign2;
            inb = inb2;
        }
    } else if constexpr (PAIR && !BLOCKONLY && RT == 1 && sizeof(SI) <= 4) {
        // FP32 input, one right-hand side: both hops of a direction in one
        // trip, so the link that site x - mu reads for its forward hop is
        // re-read for the backward hop of site x at once (from L1) rather
        // than a trip later (with FP64 input the pair does not fit in
        // registers, and FP16 input runs faster at four waves per SIMD,
        // where the pair spills; those forms load the next hop's link one
        // trip ahead)
#pragma unroll 1
        for (int mu = 0; mu < 4; ++mu) {
            int bf, sf, gf, bb, sb, gb;
            bool inb;
            neighbour_rt(a.g, b, bc, s, mu, +1, bf, sf, gf, inb);
            neighbour_rt(a.g, b, bc, s, mu, -1, bb, sb, gb, inb);
            vec2_t<SI> pf[12], pb[12];
            cx<A> Uf[9], Ub[9];
            const vec2_t<SI> *qf = in + ro[0] + ((long)bf * a.nrhs + r0) * 12 * BS + sf;
            const vec2_t<SI> *qb = in + ro[0] + ((long)bb * a.nrhs + r0) * 12 * BS + sb;
#pragma unroll
            for (int c = 0; c < 12; ++c) pf[c] = qf[c * BS];
            load_hop_link<SF, A>(links, b, s, 2 * mu, bf, sf, a.r12, Uf);
#pragma unroll
            for (int c = 0; c < 12; ++c) pb[c] = qb[c * BS];
            load_hop_link<SF, A>(links, b, s, 2 * mu + 1, bb, sb, a.r12, Ub);
            cx<A> psi[12];
#pragma unroll
            for (int c = 0; c < 12; ++c) psi[c] = ldc<A>(&pf[c]);
            const A kf = (A)(-0.5 * gf), kb = (A)(-0.5 * gb);
            switch (mu) {
            case 0: hop_k<0, A>(psi, Uf, kf, acc[0]); break;
            case 1: hop_k<2, A>(psi, Uf, kf, acc[0]); break;
            case 2: hop_k<4, A>(psi, Uf, kf, acc[0]); break;
            default: hop_k<6, A>(psi, Uf, kf, acc[0]); break;
            }
#pragma unroll
            for (int c = 0; c < 12; ++c) psi[c] = ldc<A>(&pb[c]);
            switch (mu) {
            case 0: hop_k<1, A>(psi, Ub, kb, acc[0]); break;
            case 1: hop_k<3, A>(psi, Ub, kb, acc[0]); break;
            case 2: hop_k<5, A>(psi, Ub, kb, acc[0]); break;
            default: hop_k<7, A>(psi, Ub, kb, acc[0]); break;
            }
        }
    } else if constexpr (PF && !BLOCKONLY) {
        int bn, sn, sign;
        bool inb;
        neighbour_rt(a.g, b, bc, s, 0, +1, bn, sn, sign, inb);
        cx<A> U[9];
        load_hop_link<SF, A>(links, b, s, 0, bn, sn, a.r12, U);
#pragma unroll 1
        for (int k = 0; k < 8; ++k) {
            const vec2_t<SI> *p = in + ((long)bn * a.nrhs + r0) * 12 * BS + sn;
            const A kk = (A)(-0.5 * sign);
            int bn2 = bn, sn2 = sn, sign2 = sign;
            cx<A> Un[9];
            if (k < 7) { // uniform
                const int k2 = k + 1;
                neighbour_rt(a.g, b, bc, s, k2 >> 1, (k2 & 1) ? -1 : 1, bn2, sn2, sign2, inb);
                load_hop_link<SF, A>(links, b, s, k2, bn2, sn2, a.r12, Un);
            }
            hop_switch<RT, SI, A>(k, p, ro, U, kk, acc);
#pragma unroll
            for (int e = 0; e < 9; ++e) U[e] = Un[e];
            bn = bn2;
            sn = sn2;
            sign = sign2;
        }
    } else {
#pragma unroll 1
        for (int k = 0; k < 8; ++k) {
            const int mu = k >> 1, dir = (k & 1) ? -1 : 1;
            int bn, sn, sign;
            bool inb;
            neighbour_rt(a.g, b, bc, s, mu, dir, bn, sn, sign, inb);
            if (BLOCKONLY && !inb) continue;
            const vec2_t<SI> *p = in + ((long)bn * a.nrhs + r0) * 12 * BS + sn;
            cx<A> U[9];
            load_hop_link<SF, A>(links, b, s, k, bn, sn, a.r12, U);
            hop_switch<RT, SI, A>(k, p, ro, U, (A)(-0.5 * sign), acc);
        }
    }
}

// occupancy target per precision: enough waves per SIMD to keep HBM busy
// without letting the scheduler hoist all eight hops' loads at once (FP16
// input, one right-hand side per lane: four, with the link-prefetch form)
template <typename SI, typename A, int RT> struct DslashWaves {
    static constexpr int value = sizeof(A) == 8 ? 2 : (RT > 1 ? 2 : (sizeof(SI) == 2 ? 4 : 3));
};

// One 256-thread workgroup per (block, group of RT right-hand sides); the
// groups of one block follow each other in the launch order, so the block's
// links and clover terms are re-read from L2.  Streaming clover loads (NTC)
// only when a block has a single group.
// With G > 1 (and RT == 1) G lanes of a wavefront share a site: a wavefront
// covers 64/G sites for G right-hand sides, so every link and clover load of
// the wavefront serves G right-hand sides at once (a group of G right-hand
// sides takes G workgroups per block, of 256/G sites each).
template <typename SI, typename SO, typename SF, typename A, bool BLOCKONLY, bool RESID, int RT, bool NTC, int G = 1>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(DslashWaves<SI, A, RT>::value))) void k_dslash(const vec2_t<SI> *__restrict__ in, vec2_t<SO> *__restrict__ out,
                                               const vec2_t<SF> *__restrict__ links,
                                               const vec2_t<SF> *__restrict__ clov,
                                               const vec2_t<SO> *__restrict__ resid, DArgs a)
{
    static_assert(G == 1 || (RT == 1 && !BLOCKONLY), "lanes share a site only with one right-hand side per lane");
    int b, r0, s = threadIdx.x;
    bool keep = true; // this lane's result is stored
    if (BLOCKONLY) {
        b = a.block_id;
        r0 = 0;
    } else if (G > 1) {
        constexpr int SPW = 64 / G; // sites per wavefront
        const int wg = xcd_remap(blockIdx.x, gridDim.x);
        const int bp = wg / a.ngroups; // block * G + part; the groups of a part are adjacent
        b = bp / G;
        const int l = threadIdx.x & 63;
        s = (bp - b * G) * (4 * SPW) + (threadIdx.x >> 6) * SPW + l % SPW;
        r0 = (wg - bp * a.ngroups) * G + l / SPW;
        if (r0 >= a.nrhs) { // ragged last group: recompute the last right-hand side, store nothing
            r0 = a.nrhs - 1;
            keep = false;
        }
        if (a.active && !a.active[r0]) return; // per lane; the kernel has no barrier
    } else {
        const int wg = xcd_remap(blockIdx.x, gridDim.x);
        b = wg / a.ngroups;
        r0 = (wg - b * a.ngroups) * RT;
        if (RT == 1 && a.active && !a.active[r0]) return; // uniform over the workgroup
    }
    const int nr = !keep ? 0 : (a.nrhs - r0 < RT ? a.nrhs - r0 : RT);
    int bc[4];
    block_coords(a.g, b, bc);
    cx<A> acc[RT][12];
#pragma unroll
    for (int rr = 0; rr < RT; ++rr)
#pragma unroll
        for (int c = 0; c < 12; ++c) acc[rr][c] = mk<A>(0, 0);
    // input of right-hand side r0 + rr relative to that of r0 (plus its own
    // optional element offset)
    long ro[RT];
    A diag[RT];
#pragma unroll
    for (int rr = 0; rr < RT; ++rr) {
        const int r = r0 + (rr < nr ? rr : 0);
        ro[rr] = (long)(r - r0) * 12 * BS + (a.in_off ? a.in_off[r] : 0);
        diag[rr] = (A)(4.0 + (a.m0_dev ? a.m0_dev[r] : a.m0[r]));
    }
    // one right-hand side per workgroup: the block's input spinor is staged
    // in LDS once (coalesced), and the in-block hops and the clover term read
    // it from there; only face neighbours come from memory
    constexpr bool STG = RT == 1 && G == 1 && !BLOCKONLY;
    __shared__ vec2_t<SI> stg[STG ? 12 * BS : 1];
    if constexpr (STG) {
        const vec2_t<SI> *own = in + ro[0] + ((long)b * a.nrhs + r0) * 12 * BS + s;
#pragma unroll
        for (int c = 0; c < 12; ++c) stg[c * BS + s] = own[c * BS];
        __syncthreads();
    }
    hops<BLOCKONLY, (sizeof(A) == 8 || sizeof(SI) == 2) && RT == 1, RT == 1 && sizeof(SI) == 4, RT, SI, SF, A, STG>(
        in, links, a, b, bc, r0, ro, s, acc, stg);
    // one chiral half at a time: halves the registers the clover needs
#pragma unroll 1
    for (int k = 0; k < 2; ++k) {
        cx<A> cl[18];
        const vec2_t<SF> *cp = clov + ((long)b * 36 + 18 * k) * BS + s;
#pragma unroll
        for (int e = 0; e < 18; ++e) cl[e] = NTC ? ldc_stream<A>(cp + e * BS) : ldc<A>(cp + e * BS);
        vec2_t<SI> raw[RT][6];
#pragma unroll
        for (int rr = 0; rr < RT; ++rr) {
            const long sp = ((long)b * a.nrhs + r0) * 12 * BS + s + ro[rr];
#pragma unroll
            for (int c = 0; c < 6; ++c) raw[rr][c] = STG ? stg[(6 * k + c) * BS + s] : in[sp + (6 * k + c) * BS];
        }
#pragma unroll
        for (int rr = 0; rr < RT; ++rr) {
            cx<A> psi[6];
#pragma unroll
            for (int c = 0; c < 6; ++c) psi[c] = ldc<A>(&raw[rr][c]);
            if (k == 0) clover_half_mac(cl, diag[rr], psi, acc[rr]);
            else clover_half_mac(cl, diag[rr], psi, acc[rr] + 6);
        }
    }
#pragma unroll
    for (int rr = 0; rr < RT; ++rr) {
        if (rr < nr) {
            const long sp = ((long)b * a.nrhs + r0 + rr) * 12 * BS + s;
            if (RESID) {
#pragma unroll
                for (int c = 0; c < 12; ++c)
                    stc_stream(out + sp + c * BS, ldc_stream<A>(resid + sp + c * BS) - acc[rr][c]);
            } else {
#pragma unroll
                for (int c = 0; c < 12; ++c) stc_stream(out + sp + c * BS, acc[rr][c]);
            }
        }
    }
}

// Block-wise form of the operator: one workgroup per Schwarz block applies
// the in-block part through the LDS exchange (each link and each in-block
// spinor read once) and adds the hops that leave the block from memory; the
// right-hand sides are processed one after the other, with the fields that
// RES keeps in registers loaded once for all of them.
template <typename SI, typename SO, typename SF, typename A, typename RES, bool RESID, bool NTC>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(RES::waves))) void k_dslash_lds(
    const vec2_t<SI> *__restrict__ in, vec2_t<SO> *__restrict__ out, const vec2_t<SF> *__restrict__ links,
    const vec2_t<SF> *__restrict__ clov, const vec2_t<SO> *__restrict__ resid, DArgs a)
{
    __shared__ Lds<A> L;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int s = threadIdx.x;
    int bc[4];
    block_coords(a.g, b, bc);
    // register-resident links carry the hop factor -1/2
    cx<A> U[RES::links ? 4 : 1][9];
    if constexpr (RES::links) load_links4<A>(links + (long)b * 4 * 9 * BS + s, a.r12, (A)(-0.5), U);
    cx<A> cl[RES::clover ? 36 : 1];
    if (RES::clover) {
        const vec2_t<SF> *cp = clov + (long)b * 36 * BS + s;
#pragma unroll
        for (int e = 0; e < (RES::clover ? 36 : 1); ++e) cl[e] = ldc<A>(cp + e * BS);
    }
    for (int r = 0; r < a.nrhs; ++r) {
        // the previous right-hand side's t hop and face gathers may still
        // read the LDS buffers that this one's writes are about to overwrite
        __syncthreads();
        if (a.active && !a.active[r]) continue; // uniform over the workgroup
        const A diag = (A)(4.0 + (a.m0_dev ? a.m0_dev[r] : a.m0[r]));
        const vec2_t<SI> *__restrict__ inr = in + (a.in_off ? a.in_off[r] : 0);
        const long sp = ((long)b * a.nrhs + r) * 12 * BS + s;
        // the hops that leave the block into the spare LDS buffer (the
        // t-hop barrier inside block_apply publishes them)
        face_hops_coop<SI, SF, A>(a.g, b, bc, s, r, a.nrhs, inr, links, a.r12, &L.hf[0][0][0], &L.hb[0][0][0]);
        cx<A> v[12], q[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) v[c] = ldc<A>(inr + sp + c * BS);
        block_apply<SF, A, RES, NTC>(L, a.g, b, bc, s, U, cl, links, clov, diag, v, q);
        face_gather(a.g, s, &L.hf[0][0][0], &L.hb[0][0][0], q);
        if (RESID) {
#pragma unroll
            for (int c = 0; c < 12; ++c) stc_stream(out + sp + c * BS, ldc_stream<A>(resid + sp + c * BS) - q[c]);
        } else {
#pragma unroll
            for (int c = 0; c < 12; ++c) stc_stream(out + sp + c * BS, q[c]);
        }
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
    a.r12 = ctx->link_r12 ? 1 : 0;
    for (int r = 0; r < nrhs && r < MAXRHS && m0; ++r) a.m0[r] = m0[r];
    return a;
}

// right-hand sides per workgroup: the accumulators of RT right-hand sides
// must fit in registers next to the link (FP64 arithmetic: one -- two already
// spill; FP32 arithmetic: up to three, two when that divides the count and
// three does not, so that no group is mostly empty: four right-hand sides as
// 3 + 1 measured 1.8x slower than as 2 + 2 would be from the 2-RHS time)
template <typename SI, typename A> int pick_rt(int nrhs)
{
    if (sizeof(A) == 8) return 1;
    if (nrhs <= 3) return nrhs;
    return (nrhs % 3 != 0 && nrhs % 2 == 0) ? 2 : 3;
}
// lane-shared sites for several right-hand sides: FP64 input only (with FP32
// input the variant spills and measured no faster; FP32 arithmetic keeps the
// register forms, which measured faster than lane sharing)
template <typename SI> constexpr bool LANE_SHARE = sizeof(SI) == 8;

template <typename SI, typename SO, typename SF, typename A, bool RESID, int RT, bool NTC, int G = 1>
void launch_rt(dd_ctx *ctx, DArgs a, const void *in, void *out, int field_prec, const void *resid)
{
    a.ngroups = (a.nrhs + RT * G - 1) / (RT * G);
    k_dslash<SI, SO, SF, A, false, RESID, RT, NTC, G><<<ctx->g.nblocks * G * a.ngroups, BS, 0, ctx->stream>>>(
        static_cast<const vec2_t<SI> *>(in), static_cast<vec2_t<SO> *>(out),
        static_cast<const vec2_t<SF> *>(ctx->links[field_prec].p), static_cast<const vec2_t<SF> *>(ctx->clover[field_prec].p),
        static_cast<const vec2_t<SO> *>(resid), a);
}

template <typename SI, typename SO, typename SF, typename A, typename RES, bool RESID>
void launch_lds(dd_ctx *ctx, const DArgs &a, const void *in, void *out, int field_prec, const void *resid)
{
    k_dslash_lds<SI, SO, SF, A, RES, RESID, false><<<ctx->g.nblocks, BS, 0, ctx->stream>>>(
        static_cast<const vec2_t<SI> *>(in), static_cast<vec2_t<SO> *>(out),
        static_cast<const vec2_t<SF> *>(ctx->links[field_prec].p), static_cast<const vec2_t<SF> *>(ctx->clover[field_prec].p),
        static_cast<const vec2_t<SO> *>(resid), a);
}

template <typename SI, typename SO, typename SF, typename A, bool RESID>
Status launch(dd_ctx *ctx, const DArgs &a, const void *in, void *out, int field_prec, const void *resid)
{
    const double V = (double)ctx->g.V, n = a.nrhs;
    // the method's data volume: links (72 reals per site) + clover (72) once,
    // input and output spinors per right-hand side; with gauge compression the
    // kernel reads 48 of the 72 link reals, which this figure does not count
    const double by = V * (144.0 * sizeof(SF) + 24.0 * n * (sizeof(SI) + sizeof(SO) * (RESID ? 2 : 1)));
    int cls = sizeof(SF) == 8 ? (sizeof(SI) == 8 ? K_DSLASH_F64 : K_DSLASH_F32IN_F64)
                              : (sizeof(SF) == 4 ? K_DSLASH_F32 : K_DSLASH_F16);
    ProfScope ps(ctx->prof, ctx->stream, cls, by, 1848.0 * V * n);
    if constexpr (sizeof(SF) == 4) {
        if (a.nrhs >= 4) {
            // FP32 fields, many right-hand sides: links and clover in
            // registers for all of them, block-wise LDS form (measured
            // faster than the gather form there; FP16 storage and FP64
            // fields stay with the gather form)
            launch_lds<SI, SO, SF, A, Residency<true, true, 2>, RESID>(ctx, a, in, out, field_prec, resid);
            DD_HIP_TRY(hipGetLastError());
            return Status::ok();
        }
    }
    if constexpr (LANE_SHARE<SI>) {
        if (a.nrhs % 2 == 0) {
            // an even number of right-hand sides: lanes share sites, G = 4
            // when it divides the count, else 2 (a ragged lane group measured
            // slower than G = 1); streaming clover loads when one group covers
            // all right-hand sides
            if (a.nrhs % 4 == 0) {
                if (a.nrhs == 4) launch_rt<SI, SO, SF, A, RESID, 1, true, 4>(ctx, a, in, out, field_prec, resid);
                else launch_rt<SI, SO, SF, A, RESID, 1, false, 4>(ctx, a, in, out, field_prec, resid);
            } else {
                if (a.nrhs == 2) launch_rt<SI, SO, SF, A, RESID, 1, true, 2>(ctx, a, in, out, field_prec, resid);
                else launch_rt<SI, SO, SF, A, RESID, 1, false, 2>(ctx, a, in, out, field_prec, resid);
            }
            DD_HIP_TRY(hipGetLastError());
            return Status::ok();
        }
    }
    const int rt = pick_rt<SI, A>(a.nrhs);
    const bool one = a.nrhs <= rt;
    if (rt == 1) {
        if (one) launch_rt<SI, SO, SF, A, RESID, 1, true>(ctx, a, in, out, field_prec, resid);
        else launch_rt<SI, SO, SF, A, RESID, 1, false>(ctx, a, in, out, field_prec, resid);
    }
    else if constexpr (sizeof(A) == 4) {
        if (rt == 2) {
            if (one) launch_rt<SI, SO, SF, A, RESID, 2, true>(ctx, a, in, out, field_prec, resid);
            else launch_rt<SI, SO, SF, A, RESID, 2, false>(ctx, a, in, out, field_prec, resid);
        }
        else if (one) launch_rt<SI, SO, SF, A, RESID, 3, true>(ctx, a, in, out, field_prec, resid);
        else launch_rt<SI, SO, SF, A, RESID, 3, false>(ctx, a, in, out, field_prec, resid);
    }
    DD_HIP_TRY(hipGetLastError());
    return Status::ok();
}

} // namespace

Status launch_dslash(dd_ctx *ctx, const double *m0, int nrhs, const void *in, int in_prec, void *out, int out_prec,
                     int field_prec, const double *resid, const double *m0_dev, const long *in_off, const int *active)
{
    if (!in || !out || !ctx->links[field_prec].p || !ctx->clover[field_prec].p || (!m0 && !m0_dev))
        return Status{DD_INVALID_ARG, "operator: missing buffer"};
    DArgs a = make_args(ctx, m0, nrhs);
    a.m0_dev = m0_dev;
    a.in_off = in_off;
    a.active = active;
    bool rs = resid != nullptr;
    if (in_prec == DD_F64 && out_prec == DD_F64 && field_prec == DD_F64)
        return rs ? launch<double, double, double, double, true>(ctx, a, in, out, DD_F64, resid)
                  : launch<double, double, double, double, false>(ctx, a, in, out, DD_F64, resid);
    if (in_prec == DD_F32 && out_prec == DD_F64 && field_prec == DD_F64 && !rs)
        return launch<float, double, double, double, false>(ctx, a, in, out, DD_F64, nullptr);
    if (in_prec == DD_F32 && out_prec == DD_F32 && field_prec == DD_F32)
        return rs ? launch<float, float, float, float, true>(ctx, a, in, out, DD_F32, resid)
                  : launch<float, float, float, float, false>(ctx, a, in, out, DD_F32, nullptr);
    if (in_prec == DD_F16 && out_prec == DD_F16 && field_prec == DD_F16 && !rs)
        return launch<__half, __half, __half, float, false>(ctx, a, in, out, DD_F16, nullptr);
    return Status{DD_INVALID_ARG, "unsupported precision combination for the operator"};
}

Status launch_dslash_block(dd_ctx *ctx, double m0, int block_id, const void *in, void *out, int prec)
{
    DArgs a = make_args(ctx, &m0, 1);
    a.ngroups = 1;
    a.block_id = block_id;
    ProfScope ps(ctx->prof, ctx->stream, K_DSLASH_BLOCK, 256.0 * (144.0 + 48.0) * real_bytes(prec), 1848.0 * 256);
    if (prec == DD_F64)
        k_dslash<double, double, double, double, true, false, 1, true><<<1, BS, 0, ctx->stream>>>(
            static_cast<const double2 *>(in), static_cast<double2 *>(out), ctx->links[DD_F64].as<double2>(),
            ctx->clover[DD_F64].as<double2>(), nullptr, a);
    else if (prec == DD_F32)
        k_dslash<float, float, float, float, true, false, 1, true><<<1, BS, 0, ctx->stream>>>(
            static_cast<const float2 *>(in), static_cast<float2 *>(out), ctx->links[DD_F32].as<float2>(),
            ctx->clover[DD_F32].as<float2>(), nullptr, a);
    else
        k_dslash<__half, __half, __half, float, true, false, 1, true><<<1, BS, 0, ctx->stream>>>(
            static_cast<const __half2 *>(in), static_cast<__half2 *>(out), ctx->links[DD_F16].as<__half2>(),
            ctx->clover[DD_F16].as<__half2>(), nullptr, a);
    DD_HIP_TRY(hipGetLastError());
    return Status::ok();
}

} // namespace dd
