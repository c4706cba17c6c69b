// Red-black Schwarz alternating procedure (SAP) with block-local minimal
// residual (MR) solves -- the "MR inversion within a domain" and the "entire
// Schwarz method" whose per-core rates the paper reports (Sec. 3.1, Tables 1
// and 2); the algorithm is Luescher's multiplicative SAP (Comput. Phys.
// Commun. 156 (2004) 209) with Saad's MR iteration on each block.
//
// One launch sweeps every block of one colour.  One 256-thread workgroup owns
// one 4^4 block, one thread one site, and keeps everything the MR loop needs
// on chip:
//   * the site's four forward links (pre-multiplied by the hop factor -1/2)
//     and chiral half 0 of its clover term live in registers for the whole
//     sweep and every right-hand side; clover half 1 is re-read at each block
//     application and stays in L2; the MR accumulator lives in LDS;
//   * D_BB is applied direction by direction: each thread provides the
//     spin-projected half spinor of its site for the +mu hop of site x-mu and
//     U_mu(x)^+ times the projected half spinor for the -mu hop of site x+mu,
//     across lanes of its wavefront for x, y, z (a wavefront is one t-slice)
//     and through LDS for t, so no spinor leaves the chip inside the MR loop;
//   * the two block dot products per MR step reduce with DPP sums within each
//     wavefront and a fixed-order combine of the four wavefronts
//     (deterministic).
// eta and psi go through the caches (they are re-read by the next sweep and
// by the operator that follows the smoother, and fit in the 256 MB
// last-level cache in FP32); links and clover half 0, read once per sweep,
// stream.
// With FP32/FP16 storage the block residual rho_B = eta_B - (D psi)_B is
// carried from visit to visit rather than recomputed (FP64 recomputes it: the
// carried form does not fit its register budget as well).  Luescher's
// formulation of the procedure: after its
// MR steps a block stores its MR residual R_B, and the next visit forms
// rho_B = R_B - D_{B,dB} delta_dB, where delta_dB is the update that the
// neighbouring blocks of the other colour made in between (on the first
// visit R_B = eta_B).  The hops of delta arrive through face buffers that the
// other colour published at the end of its solves (block_ops.h: six dense
// components per boundary hop).  psi_B before the visit waits in the half of
// the LDS exchange buffer that the in-wavefront directions leave free.
// Blocks of one colour share no site and read only the other colour's data,
// so a sweep needs no synchronisation between workgroups.
//
// k_sap_sweep_eo is the same sweep with the even-odd preconditioned block
// solve (MR on the even-site Schur complement, odd sites reconstructed);
// see the comment above it.
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
    const int *active;    // right-hand sides with active[r] == 0 are skipped (nullable)
    int publish;          // write the face buffers for the next sweep
    int r12;              // links stored as SU(3): read two rows, rebuild the third
    int write_r;          // plain sweep: store the block residual for the next visit
};

// The MR coefficient of one right-hand side: the dot products <q, r> and
// <q, q> over the block (DPP sums within each wavefront, then a fixed-order
// combine of the four wavefronts through LDS), alpha = <q, r>/<q, q>; returns
// false when <q, q> vanishes (uniform over the workgroup).
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
    if (lane == 63) { // where wave_sum leaves the total
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

// Whether the plain sweep of storage type S carries the block residual.
template <typename S> constexpr bool SAP_CARRY = !std::is_same<S, double>::value;

// SF is the storage type of the links and the clover term (S, or FP16 fields
// under FP32 spinors).
template <typename S, typename A, typename RES, typename SF = S>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(RES::waves))) void k_sap_sweep(
    const vec2_t<S> *__restrict__ eta0, vec2_t<S> *__restrict__ psi0, const vec2_t<SF> *__restrict__ links,
    const vec2_t<SF> *__restrict__ clov, vec2_t<S> *__restrict__ faces, vec2_t<S> *__restrict__ resid, SArgs a)
{
    constexpr bool REGLINKS = RES::links;
    static_assert(REGLINKS, "the face buffers assume register-resident links");
    static_assert(RES::clover_half, "the MR accumulator lives in LDS");
    // FP32/FP16 storage carries the block residual between visits; FP64
    // recomputes it (the carried form spills in FP64's register budget)
    constexpr bool CARRY = SAP_CARRY<S>;
    __shared__ Lds<A> L;
    __shared__ DelStore<A, RES> D;
    const int i = xcd_remap(blockIdx.x, gridDim.x);
    const int b = a.blocks[i];
    const int s = threadIdx.x;
    const int lane = s & 63, wave = s >> 6;
    int bc[4];
    block_coords(a.g, b, bc);

    // register-resident links carry the hop factor -1/2
    cx<A> U[4][9];
    load_links4<A, true>(links + (long)b * 4 * 9 * BS + s, a.r12, (A)(-0.5), U);
    cx<A> cl[RES::ncl];
    if (RES::clover || RES::clover_half) {
        const vec2_t<SF> *cp = clov + (long)b * 36 * BS + s;
#pragma unroll
        for (int e = 0; e < RES::ncl; ++e) cl[e] = ldc_stream<A>(cp + e * BS);
    }

    for (int r = 0; r < a.nrhs; ++r) {
        // with nmr = 0 the previous right-hand side's last t-hop reads are
        // not yet fenced by an MR barrier
        __syncthreads();
        if (a.active && !a.active[r]) continue; // uniform over the workgroup
        const A diag = (A)(4.0 + (a.m0_dev ? a.m0_dev[r] : a.m0[r]));
        const vec2_t<S> *__restrict__ eta = eta0 + (a.eta_off ? a.eta_off[r] : 0);
        vec2_t<S> *__restrict__ psi = psi0 + (a.psi_off ? a.psi_off[r] : 0);
        const long sp = ((long)b * a.nrhs + r) * 12 * BS + s;
        const long rp = ((long)b * a.nrhs + r) * 12 * BS + s; // the carried residual (no slot offsets)
        cx<A> rr[12], q[12];
        vec2_t<S> er[12];
        if constexpr (CARRY) {
            // psi_B before this visit, in the half of the exchange buffer that
            // the in-wavefront directions leave unused; delta starts at 0
            if (a.mode == 2) {
#pragma unroll
                for (int c = 0; c < 12; ++c) {
                    const cx<A> v = ldc<A>(psi + sp + c * BS);
                    if (c < 6) L.hf[0][c][s] = v;
                    else L.hb[0][c - 6][s] = v;
                }
            }
#pragma unroll
            for (int c = 0; c < 12; ++c) D.d[c][s] = mk<A>(0, 0);
            // rho = R - (hops of the other colour's last update), R being this
            // block's residual after its previous visit (eta on the first)
            const vec2_t<S> *__restrict__ src = a.mode == 2 ? resid + rp : eta + sp;
#pragma unroll
            for (int c = 0; c < 12; ++c) er[c] = src[c * BS];
#pragma unroll
            for (int c = 0; c < 12; ++c) q[c] = mk<A>(0, 0);
        } else {
            // rho = eta - (D psi)_B, recomputed: the block part here, the hops
            // of the other colour's psi below; delta starts at psi_B
            cx<A> d0[12];
#pragma unroll
            for (int c = 0; c < 12; ++c) d0[c] = a.mode == 2 ? ldc<A>(psi + sp + c * BS) : mk<A>(0, 0);
            if (a.mode == 2) {
                block_apply<SF, A, RES>(L, a.g, b, bc, s, U, cl, links, clov, diag, d0, q);
            } else {
#pragma unroll
                for (int c = 0; c < 12; ++c) q[c] = mk<A>(0, 0);
            }
#pragma unroll
            for (int c = 0; c < 12; ++c) D.d[c][s] = d0[c];
            // eta in flight during the face trips (held in the storage type)
#pragma unroll
            for (int c = 0; c < 12; ++c) er[c] = eta[sp + c * BS];
        }
        if (a.mode != 0) face_consume<S, A>(a.g, b, bc, s, r, a.nrhs, faces, U, q);
#pragma unroll
        for (int c = 0; c < 12; ++c) rr[c] = ldc<A>(&er[c]) - q[c];
        // the recomputed residual's t-hop reads end before the first MR
        // application rewrites that LDS buffer
        if (!CARRY && a.mode == 2) __syncthreads();
        // MR on D_BB: delta += alpha r, r -= alpha q
        for (int it = 0; it < a.nmr; ++it) {
            block_apply<SF, A, RES>(L, a.g, b, bc, s, U, cl, links, clov, diag, rr, q);
            cx<A> alpha;
            if (!mr_alpha(L, lane, wave, q, rr, alpha)) break;
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                cx<A> d = D.d[c][s];
                cmac(d, alpha, rr[c]);
                D.d[c][s] = d;
                rr[c] = rr[c] - alpha * q[c];
            }
        }
        cx<A> fin[12];
        if constexpr (CARRY) {
            // psi_B += delta; the residual carried to the next visit; the
            // faces of delta for the other colour
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                fin[c] = D.d[c][s];
                cx<A> v = fin[c];
                if (a.mode == 2) v = v + (c < 6 ? L.hf[0][c][s] : L.hb[0][c - 6][s]);
                stc(psi + sp + c * BS, v);
            }
            if (a.write_r) {
#pragma unroll
                for (int c = 0; c < 12; ++c) stc(resid + rp + c * BS, rr[c]);
            }
        } else {
            // psi_B = delta; the faces of psi as stored
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                vec2_t<S> v;
                stc(&v, D.d[c][s]);
                psi[sp + c * BS] = v;
                fin[c] = ldc<A>(&v);
            }
        }
        if (a.publish) face_publish<S, A>(faces, b, a.nrhs, r, s, fin, U);
    }
}

// ---------------------------------------------------------------------------
// Even-odd preconditioned block solve (site parity p = (x+y+z+t) mod 2).  On
// block B, with A = (4 + m0) + C site-local and H the in-block hops,
//   S = A_ee - H_eo A_oo^-1 H_oe on the even sites,
//   rhat_e = rho_e - H_eo A_oo^-1 rho_o,  nMR MR steps on S,
//   delta_o = A_oo^-1 (rho_o - H_oe delta_e).
// Threads 0-127 (waves 0-1) own the even sites, threads 128-255 (waves 2-3)
// the odd ones, so every parity branch is uniform over a wavefront.  A hop
// exchange between the parities is pipelined: at stage k the publishing
// waves post direction k while the consuming waves take direction k-1 from
// the other LDS buffer.  A_oo^-1 is applied through the Cholesky factor of
// each chiral half (the halves are Hermitian positive definite: the clover
// term is small against 4 + m0).
// ---------------------------------------------------------------------------

// Whether the even-odd sweep of storage type S uses the face buffers.
template <typename S> constexpr bool EO_FACES = !std::is_same<S, double>::value;

// Site of thread t: the pair {2k, 2k+1} (k = t mod 128) holds one even and
// one odd site; which is which follows from (ly + lz + lt) mod 2.
__device__ __forceinline__ int eo_site(int t)
{
    const int k = t & 127, odd = t >> 7;
    const int bit = (((k >> 1) & 3) + ((k >> 3) & 3) + ((k >> 5) & 3)) & 1;
    return 2 * k + (bit ^ odd);
}

// Slot of the upper entry (j, i), j < i, of a packed Hermitian 6x6 half.
__host__ __device__ constexpr int hslot(int j, int i) { return 3 + j * 5 - j * (j - 1) / 2 + (i - j - 1); }

// In place: the packed half c, plus diag on the diagonal, becomes its
// Cholesky factor M = R^+ R (R upper triangular, real positive diagonal):
// slots 0-2 receive 1/R_jj in pairs, the slot of (j, i) receives R_ji.
template <typename A> __device__ __forceinline__ void chol_half(cx<A> c[18], A diag)
{
    A d[6] = {c[0].re + diag, c[0].im + diag, c[1].re + diag, c[1].im + diag, c[2].re + diag, c[2].im + diag};
    A inv[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        A t = d[j];
#pragma unroll
        for (int k = 0; k < j; ++k) {
            const cx<A> u = c[hslot(k, j)];
            t -= u.re * u.re + u.im * u.im;
        }
        inv[j] = (A)1 / sqrt(t);
#pragma unroll
        for (int i = j + 1; i < 6; ++i) {
            cx<A> acc = c[hslot(j, i)];
#pragma unroll
            for (int k = 0; k < j; ++k) {
                // acc -= conj(R_kj) R_ki
                const cx<A> a = c[hslot(k, j)], b2 = c[hslot(k, i)];
                acc.re -= a.re * b2.re + a.im * b2.im;
                acc.im -= a.re * b2.im - a.im * b2.re;
            }
            c[hslot(j, i)] = inv[j] * acc;
        }
    }
    c[0] = mk<A>(inv[0], inv[1]);
    c[1] = mk<A>(inv[2], inv[3]);
    c[2] = mk<A>(inv[4], inv[5]);
}

// x = M^-1 x in place from the factor written by chol_half: R^+ y = x, then
// R x = y.
template <typename A> __device__ __forceinline__ void chol_solve(const cx<A> f[18], cx<A> x[6])
{
    const A inv[6] = {f[0].re, f[0].im, f[1].re, f[1].im, f[2].re, f[2].im};
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        cx<A> acc = x[i];
#pragma unroll
        for (int k = 0; k < i; ++k) {
            // acc -= conj(R_ki) y_k
            const cx<A> a = f[hslot(k, i)];
            acc.re -= a.re * x[k].re + a.im * x[k].im;
            acc.im -= a.re * x[k].im - a.im * x[k].re;
        }
        x[i] = inv[i] * acc;
    }
#pragma unroll
    for (int i = 5; i >= 0; --i) {
        cx<A> acc = x[i];
#pragma unroll
        for (int k = i + 1; k < 6; ++k) acc = acc - f[hslot(i, k)] * x[k];
        x[i] = inv[i] * acc;
    }
}

// LDS of the even-odd sweep.  The residual on entry uses the plain block
// exchange (all 256 sites post); the parity exchanges post only one parity
// at a time, so their buffers are indexed by the ordinal k = s / 2 of the
// posting site and share the memory of the full exchange, next to rho of
// the odd sites.
template <typename A> struct EoLds {
    cx<A> hf[2][6][BS / 2];
    cx<A> hb[2][6][BS / 2];
    cx<A> rho[12][BS / 2]; // rho of the odd sites
};
template <typename A> union SapEoShared {
    Lds<A> full;
    EoLds<A> eo;
};

// Post direction MU of v (this thread's site s) into buffer X.
template <int MU, typename A>
__device__ __forceinline__ void eo_publish(EoLds<A> &L, int X, int s, const cx<A> U[9], const cx<A> v[12])
{
    cx<A> h[6], t[6];
    const int k = s >> 1;
    proj_minus<MU>(v, h);
#pragma unroll
    for (int c = 0; c < 6; ++c) L.hf[X][c][k] = h[c];
    proj_plus<MU>(v, h);
    su3_mul_adj(U, h, t);
#pragma unroll
    for (int c = 0; c < 6; ++c) L.hb[X][c][k] = t[c];
}

// Take direction MU from buffer X: q += the two in-block hops of site s.
template <int MU, typename A>
__device__ __forceinline__ void eo_consume(EoLds<A> &L, int X, const Geom &g, int b, const int bc[4], int s,
                                           const cx<A> U[9], cx<A> q[12])
{
    const bool wraps = g.nb[MU] == 1; // uniform
    cx<A> h[6], t[6];
    int bn, sn, sign;
    bool inb;
    neighbour<MU, +1>(g, b, bc, s, bn, sn, sign, inb);
    if (inb) {
#pragma unroll
        for (int c = 0; c < 6; ++c) h[c] = L.hf[X][c][sn >> 1];
        su3_mul(U, h, t);
        if (wraps) recon_minus<MU>(q, t, (A)sign);
        else recon_minus1<MU>(q, t);
    }
    neighbour<MU, -1>(g, b, bc, s, bn, sn, sign, inb);
    if (inb) {
#pragma unroll
        for (int c = 0; c < 6; ++c) t[c] = L.hb[X][c][sn >> 1];
        if (wraps) recon_plus<MU>(q, t, (A)sign);
        else recon_plus1<MU>(q, t);
    }
}

// q += H v across the parities: the waves with pub set post v, the others
// accumulate the hops into q.  Stage k posts direction k and takes direction
// k - 1 (the two LDS buffers alternate), one barrier per stage.  Buffer reuse
// is safe across consecutive calls: a buffer is rewritten only after a
// barrier that follows its last read.
template <typename A>
__device__ __forceinline__ void eo_exchange(EoLds<A> &L, const Geom &g, int b, const int bc[4], int s,
                                            const cx<A> Ur[4][9], bool pub, const cx<A> v[12], cx<A> q[12])
{
    if (pub) eo_publish<0, A>(L, 0, s, Ur[0], v);
    __syncthreads();
    if (pub) eo_publish<1, A>(L, 1, s, Ur[1], v);
    else eo_consume<0, A>(L, 0, g, b, bc, s, Ur[0], q);
    __syncthreads();
    if (pub) eo_publish<2, A>(L, 0, s, Ur[2], v);
    else eo_consume<1, A>(L, 1, g, b, bc, s, Ur[1], q);
    __syncthreads();
    if (pub) eo_publish<3, A>(L, 1, s, Ur[3], v);
    else eo_consume<2, A>(L, 0, g, b, bc, s, Ur[2], q);
    __syncthreads();
    if (!pub) eo_consume<3, A>(L, 1, g, b, bc, s, Ur[3], q);
}

// x = M^-1 x in place with the factor of chiral half 1 held in LDS.
template <typename A> __device__ __forceinline__ void chol_solve_lds(const cx<A> (*F)[BS / 2], int k, cx<A> x[6])
{
    cx<A> f[18];
#pragma unroll
    for (int e = 0; e < 18; ++e) f[e] = F[e][k];
    chol_solve<A>(f, x);
}

template <typename S, typename A, typename RES>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(RES::waves))) void k_sap_sweep_eo(
    const vec2_t<S> *__restrict__ eta0, vec2_t<S> *__restrict__ psi0, const vec2_t<S> *__restrict__ links,
    const vec2_t<S> *__restrict__ clov, vec2_t<S> *__restrict__ faces, SArgs a)
{
    static_assert(RES::links && RES::clover_half, "even-odd sweep: links and clover half 0 in registers");
    __shared__ SapEoShared<A> SH;
    __shared__ cx<A> Dd[12][BS / 2]; // delta_e of the even sites (by even ordinal)
    __shared__ cx<A> F1[18][BS / 2]; // Cholesky factor of chiral half 1 of the odd sites
    Lds<A> &L = SH.full;
    EoLds<A> &E = SH.eo;
    const int i = xcd_remap(blockIdx.x, gridDim.x);
    const int b = a.blocks[i];
    const int tid = threadIdx.x, s = eo_site(tid), k = tid & (BS / 2 - 1);
    const bool odd = tid >= BS / 2; // uniform over a wavefront
    const int lane = tid & 63, wave = tid >> 6;
    int bc[4];
    block_coords(a.g, b, bc);

    // register-resident links carry the hop factor -1/2
    cx<A> U[4][9];
    load_links4<A, true>(links + (long)b * 4 * 9 * BS + s, a.r12, (A)(-0.5), U);
    const vec2_t<S> *cp0 = clov + (long)b * 36 * BS + s;

    for (int r = 0; r < a.nrhs; ++r) {
        if (a.active && !a.active[r]) continue; // uniform over the workgroup
        const A diag = (A)(4.0 + (a.m0_dev ? a.m0_dev[r] : a.m0[r]));
        const vec2_t<S> *__restrict__ eta = eta0 + (a.eta_off ? a.eta_off[r] : 0);
        vec2_t<S> *__restrict__ psi = psi0 + (a.psi_off ? a.psi_off[r] : 0);
        const long sp = ((long)b * a.nrhs + r) * 12 * BS + s;
        // clover half 0 (odd sites factor it in place below, so it is
        // reloaded for every right-hand side)
        cx<A> cl[18];
#pragma unroll
        for (int e = 0; e < 18; ++e) cl[e] = ldc<A>(cp0 + e * BS);
        if (odd) {
            // factor of chiral half 1 of A_oo = (4 + m0) + C, kept in LDS
            cx<A> c1[18];
#pragma unroll
            for (int e = 0; e < 18; ++e) c1[e] = ldc<A>(cp0 + (18 + e) * BS);
            chol_half<A>(c1, diag);
#pragma unroll
            for (int e = 0; e < 18; ++e) F1[e][k] = c1[e];
        }

        // rho = eta - (D psi)_B
        cx<A> rho[12], q[12];
        {
            cx<A> p0[12];
            if (a.mode == 2) {
#pragma unroll
                for (int c = 0; c < 12; ++c) p0[c] = ldc<A>(psi + sp + c * BS);
                // threads own sites by parity here, not site = thread
                block_apply<S, A, RES, false, false>(L, a.g, b, bc, s, U, cl, links, clov, diag, p0, q);
            } else {
#pragma unroll
                for (int c = 0; c < 12; ++c) q[c] = mk<A>(0, 0);
            }
        }
        // the boundary hops, from the faces the other colour published, with
        // eta in flight during the face trips (in FP64 the other colour's psi
        // and links are read instead, and eta afterwards: the face code does
        // not fit this sweep's FP64 register budget)
        if constexpr (EO_FACES<S>) {
            vec2_t<S> er[12];
#pragma unroll
            for (int c = 0; c < 12; ++c) er[c] = eta[sp + c * BS];
            if (a.mode != 0) face_consume<S, A>(a.g, b, bc, s, r, a.nrhs, faces, U, q);
#pragma unroll
            for (int c = 0; c < 12; ++c) rho[c] = ldc<A>(&er[c]) - q[c];
        } else {
            if (a.mode != 0) face_hops<S, S, A, true>(a.g, b, bc, s, r, a.nrhs, psi, links, U, q, a.r12);
#pragma unroll
            for (int c = 0; c < 12; ++c) rho[c] = ldc<A>(eta + sp + c * BS) - q[c];
        }
        // the parity exchanges reuse the memory of the full one
        __syncthreads();

        // Two vectors per thread from here on: r (even sites) and q.  In each
        // parity exchange the posting waves read q or r and the receiving
        // waves accumulate into q, so one array serves both roles.
        cx<A> rr[12];
        if (odd) {
            // rho_o to LDS; factor chiral half 0 in place; q = A_oo^-1 rho_o
#pragma unroll
            for (int c = 0; c < 12; ++c) E.rho[c][k] = rho[c];
            chol_half<A>(cl, diag);
#pragma unroll
            for (int c = 0; c < 12; ++c) q[c] = rho[c];
            chol_solve<A>(cl, q);
            chol_solve_lds<A>(F1, k, q + 6);
#pragma unroll
            for (int c = 0; c < 12; ++c) rr[c] = mk<A>(0, 0);
        } else {
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                rr[c] = rho[c];
                q[c] = mk<A>(0, 0);
                Dd[c][k] = mk<A>(0, 0);
            }
        }
        // even: r_e = rho_e - H_eo A_oo^-1 rho_o
        eo_exchange<A>(E, a.g, b, bc, s, U, odd, q, q);
        if (!odd) {
#pragma unroll
            for (int c = 0; c < 12; ++c) rr[c] = rr[c] - q[c];
        }

        // MR on S = A_ee - H_eo A_oo^-1 H_oe
        for (int it = 0; it < a.nmr; ++it) {
            // odd: q = H_oe r_e
#pragma unroll
            for (int c = 0; c < 12; ++c) q[c] = mk<A>(0, 0);
            eo_exchange<A>(E, a.g, b, bc, s, U, !odd, rr, q);
            if (odd) {
                // q = -A_oo^-1 H_oe r_e
                chol_solve<A>(cl, q);
                chol_solve_lds<A>(F1, k, q + 6);
#pragma unroll
                for (int c = 0; c < 12; ++c) q[c] = mk<A>(-q[c].re, -q[c].im);
            } else {
                // q = A_ee r_e
                clover_half_mac<A>(cl, diag, rr, q);
                cx<A> c2[18];
                const vec2_t<S> *cp1 = cp0 + 18 * BS;
                // the same address at every MR step: hide that, or the loads
                // leave the loop and the half is held in registers
                asm volatile("" : "+v"(cp1));
#pragma unroll
                for (int e = 0; e < 18; ++e) c2[e] = ldc<A>(cp1 + e * BS);
                clover_half_mac<A>(c2, diag, rr + 6, q + 6);
            }
            // even: q = A_ee r_e - H_eo A_oo^-1 H_oe r_e = S r_e
            eo_exchange<A>(E, a.g, b, bc, s, U, odd, q, q);
            if (odd) {
#pragma unroll
                for (int c = 0; c < 12; ++c) q[c] = mk<A>(0, 0);
            }
            cx<A> alpha;
            if (!mr_alpha(L, lane, wave, q, rr, alpha)) break;
            if (!odd) {
#pragma unroll
                for (int c = 0; c < 12; ++c) {
                    cx<A> d = Dd[c][k];
                    cmac(d, alpha, rr[c]);
                    Dd[c][k] = d;
                    rr[c] = rr[c] - alpha * q[c];
                }
            }
        }

        // odd: delta_o = A_oo^-1 (rho_o - H_oe delta_e); even: delta_e
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            rr[c] = odd ? mk<A>(0, 0) : Dd[c][k];
            q[c] = mk<A>(0, 0);
        }
        eo_exchange<A>(E, a.g, b, bc, s, U, !odd, rr, q);
        if (odd) {
#pragma unroll
            for (int c = 0; c < 12; ++c) rr[c] = E.rho[c][k] - q[c];
            chol_solve<A>(cl, rr);
            chol_solve_lds<A>(F1, k, rr + 6);
        }
        // psi_B += delta_B
        if (a.mode == 2) {
#pragma unroll
            for (int c = 0; c < 12; ++c) rr[c] = rr[c] + ldc<A>(psi + sp + c * BS);
        }
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            vec2_t<S> v;
            stc(&v, rr[c]);
            psi[sp + c * BS] = v;
            rr[c] = ldc<A>(&v); // the stored value, as the other colour would read it
        }
        if constexpr (EO_FACES<S>) {
            if (a.publish) face_publish<S, A>(faces, b, a.nrhs, r, s, rr, U);
        }
        // the next right-hand side's residual reuses the LDS read above
        __syncthreads();
    }
}

template <typename S, typename A, typename RES, bool EO, typename SF = S>
Status sweep(dd_ctx *ctx, const SArgs &a, int prec, const void *eta, void *psi, void *faces, void *resid, bool quiet)
{
    // algorithmic traffic of one colour sweep: links + clover once, eta (or
    // the carried residual), psi (read only when nonzero), psi written and,
    // in the plain form, the residual carried to the next visit
    const double sites = 256.0 * a.nblk, sb = (double)sizeof(S), n = a.nrhs;
    constexpr bool CARRY = !EO && SAP_CARRY<S>;
    const int fprec = sizeof(SF) == 8 ? DD_F64 : (sizeof(SF) == 4 ? DD_F32 : DD_F16);
    // (links count 72 reals per site also when compressed: the method's volume)
    const double by = sites * (144.0 * (double)sizeof(SF) +
                               n * sb * (24.0 + 24.0 + (a.mode == 2 ? 24.0 : 0.0) + (CARRY && a.write_r ? 24.0 : 0.0)));
    // recomputing the block residual costs one operator application when
    // psi_B != 0; carrying it costs none.  The even-odd form adds one
    // in-block hop application (the right-hand side and the odd
    // reconstruction) per block solve.
    const double fl = sites * n * (a.nmr * 2184.0 + (!CARRY && a.mode == 2 ? 1848.0 : 0.0) + (EO ? 1848.0 : 0.0));
    const int cls = EO ? (prec == DD_F64 ? K_SAP_EO_F64 : prec == DD_F32 ? K_SAP_EO_F32 : K_SAP_EO_F16)
                       : (prec == DD_F64 ? K_SAP_F64 : prec == DD_F32 ? K_SAP_F32 : K_SAP_F16);
    ProfScope ps(ctx->prof, ctx->stream, cls, by, fl, !quiet);
    if constexpr (EO)
        k_sap_sweep_eo<S, A, RES><<<a.nblk, BS, 0, ctx->stream>>>(
            static_cast<const vec2_t<S> *>(eta), static_cast<vec2_t<S> *>(psi),
            static_cast<const vec2_t<S> *>(ctx->links[prec].p), static_cast<const vec2_t<S> *>(ctx->clover[prec].p),
            static_cast<vec2_t<S> *>(faces), a);
    else
        k_sap_sweep<S, A, RES, SF><<<a.nblk, BS, 0, ctx->stream>>>(
            static_cast<const vec2_t<S> *>(eta), static_cast<vec2_t<S> *>(psi),
            static_cast<const vec2_t<SF> *>(ctx->links[fprec].p), static_cast<const vec2_t<SF> *>(ctx->clover[fprec].p),
            static_cast<vec2_t<S> *>(faces), static_cast<vec2_t<S> *>(resid), a);
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
// The even-odd sweep holds more per thread (two vectors, the factor or the
// clover, the four links) and runs at one wavefront per SIMD.
typedef Residency<true, false, 1, true> ResEO;

} // namespace

size_t sap_scratch_bytes(const GeomHost &g, int prec, int nrhs)
{
    // face buffers (FACE_ELEMS = 12 * BS per block and rhs) and the carried
    // block residual: one spinor each
    return 2 * spinor_bytes(g, prec, nrhs);
}

Status reserve_sap_scratch(dd_ctx *ctx, int prec, int nrhs)
{
    const size_t need = sap_scratch_bytes(ctx->g, prec, nrhs);
    if (ctx->sap_scratch.p && ctx->sap_scratch.bytes >= need) return Status::ok();
    return ctx->sap_scratch.alloc(need);
}

Status run_sap(dd_ctx *ctx, const double *m0, int nrhs, const void *eta, void *psi, int ncy, int nmr, int prec,
               const SapSlots *slots, bool eo)
{
    if (!eta || !psi || !ctx->links[prec].p || !ctx->clover[prec].p || (!m0 && !(slots && slots->m0_dev)))
        return Status{DD_INVALID_ARG, "SAP: missing buffer"};
    // FP16 links and clover under the plain FP32 sweep (the even-odd sweep
    // keeps its own precision's fields)
    const bool half_fields = prec == DD_F32 && !eo && ctx->sap_half_fields;
    if (half_fields && (!ctx->links[DD_F16].p || !ctx->clover[DD_F16].p))
        return Status{DD_INVALID_ARG, "SAP: missing FP16 fields"};
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
    a.r12 = ctx->link_r12 ? 1 : 0;
    for (int r = 0; r < nrhs && m0; ++r) a.m0[r] = m0[r];
    if (slots) {
        a.m0_dev = slots->m0_dev;
        a.eta_off = slots->eta_off;
        a.psi_off = slots->psi_off;
        a.active = slots->active;
    }
    // face buffers and carried residual: the caller's scratch, else the context's
    void *scratch = slots ? slots->scratch : nullptr;
    if (!scratch) {
        DD_TRY(reserve_sap_scratch(ctx, prec, nrhs));
        scratch = ctx->sap_scratch.p;
    }
    if (!scratch) return Status{DD_INVALID_ARG, "SAP: no scratch buffer"};
    void *faces = scratch;
    void *resid = static_cast<char *>(scratch) + spinor_bytes(ctx->g, prec, nrhs);
    const bool quiet = slots && slots->quiet;
    TraceRange tr(eo ? "sap_eo" : "sap");
    for (int cy = 0; cy < ncy; ++cy)
        for (int col = 0; col < 2; ++col) {
            if (ctx->ncolour[col] == 0) continue;
            a.blocks = ctx->colour_blocks[col].as<int>();
            a.nblk = ctx->ncolour[col];
            a.mode = (cy == 0 && col == 0) ? 0 : (cy == 0 ? 1 : 2);
            a.publish = !(cy == ncy - 1 && col == 1);
            a.write_r = cy < ncy - 1;
            if (eo) {
                if (prec == DD_F64) DD_TRY((sweep<double, double, ResEO, true>(ctx, a, prec, eta, psi, faces, resid, quiet)));
                else if (prec == DD_F32) DD_TRY((sweep<float, float, ResEO, true>(ctx, a, prec, eta, psi, faces, resid, quiet)));
                else DD_TRY((sweep<__half, float, ResEO, true>(ctx, a, prec, eta, psi, faces, resid, quiet)));
            } else {
                if (prec == DD_F64) DD_TRY((sweep<double, double, ResF64, false>(ctx, a, prec, eta, psi, faces, resid, quiet)));
                else if (prec == DD_F32 && half_fields)
                    DD_TRY((sweep<float, float, ResF32, false, __half>(ctx, a, prec, eta, psi, faces, resid, quiet)));
                else if (prec == DD_F32) DD_TRY((sweep<float, float, ResF32, false>(ctx, a, prec, eta, psi, faces, resid, quiet)));
                else DD_TRY((sweep<__half, float, ResF16, false>(ctx, a, prec, eta, psi, faces, resid, quiet)));
            }
        }
    return Status::ok();
}

} // namespace dd
