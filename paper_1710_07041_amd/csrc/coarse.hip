// Two-level coarse correction of DD-alpha-AMG on the GPU: the multigrid
// level the paper's solver puts above the Schwarz smoother (Sec. 1 names the
// method, Sec. 2.1 the smoother as its fine grid, Sec. 5 its coarse grid).
// The method is the published one (Frommer, Kahl, Krieg, Leder, Rottmann,
// SIAM J. Sci. Comput. 36 (2014) A1581):
//   * aggregates: each 4^4 Schwarz block split into its two chiral halves
//     (spins 0-1, spins 2-3), so the interpolation commutes with gamma_5;
//   * interpolation P: N test vectors restricted to every aggregate and
//     orthonormalised there by Gram-Schmidt in their order (P^+ P = 1);
//   * test vectors: inverse iteration with the Schwarz smoother from N
//     starting vectors, optionally refined by rounds of the two-grid method;
//   * coarse operator D_c = P^+ D P: a nearest-neighbour stencil on the
//     lattice of blocks with 2N unknowns per block, nine dense 2N x 2N
//     matrices per block (the block itself and its eight neighbours), built
//     at m0 = 0 -- because P^+ P = 1 the mass enters as + m0 at apply time,
//     so one coarse operator serves every mass;
//   * coarse solve: k steps of GMRES from zero (the least-residual vector of
//     the Krylov space), run entirely on the device for every right-hand
//     side at once (no host round trip, so the preconditioner can be
//     captured in a graph);
//   * two-grid preconditioner: psi_0 = P x_c with x_c the coarse solve of
//     D_c x_c = P^+ eta, then psi = psi_0 + SAP_nu(eta - D psi_0).
//
// Layouts (complex numbers as (re, im) pairs):
//   P      [block][chiral half c][vector i][component 0..5][site 0..255],
//          component = (spin - 2c) * 3 + colour; FP64 master, FP32 copy;
//   D_c    [block][d][column k'][row k], d = 0 the block itself, 1 + 2 mu
//          the +mu neighbour, 2 + 2 mu the -mu neighbour; row/column index
//          k = c * N + i; FP64 master, FP16 copy read by the coarse solve
//          (the coarse system is solved only approximately, and its nine
//          blocks per row are the largest array the solve streams);
//   coarse vectors [slot][block][k], FP64.
// Everything a block or a coarse site reduces is summed in a fixed order
// (DPP within a wavefront, then the wavefronts in order), so results are
// deterministic.
#include <algorithm>
#include <cmath>

#include "block_ops.h"
#include "dd_device.h"
#include "dd_internal.h"

namespace dd {

namespace {

constexpr int NMAX = 16;  // test vectors
constexpr int CK = 32;    // largest coarse GMRES step count
constexpr int CTPB = 256; // threads per coarse workgroup
constexpr int CG = 256;   // workgroups of the coarse reductions (grid-stride; one partial sum each)

// ---------------------------------------------------------------------------
// block reductions: the wavefront sum of each value lands in lane 63, the
// four wavefronts are added in order through LDS
// ---------------------------------------------------------------------------
struct Red {
    double v[4][2 * NMAX][2];
};

__device__ __forceinline__ void wave_put(Red &R, int lane, int wave, int slot, double re, double im)
{
    re = wave_sum(re);
    im = wave_sum(im);
    if (lane == 63) {
        R.v[wave][slot][0] = re;
        R.v[wave][slot][1] = im;
    }
}

__device__ __forceinline__ cx<double> wave_get(const Red &R, int slot)
{
    return mk<double>(((R.v[0][slot][0] + R.v[1][slot][0]) + R.v[2][slot][0]) + R.v[3][slot][0],
                      ((R.v[0][slot][1] + R.v[1][slot][1]) + R.v[2][slot][1]) + R.v[3][slot][1]);
}

__device__ __forceinline__ long pidx(int b, int c, int i, int N, int comp, int s)
{
    return ((((long)b * 2 + c) * N + i) * 6 + comp) * BS + s;
}

// ---------------------------------------------------------------------------
// interpolation: Gram-Schmidt of the test vectors on every aggregate
// ---------------------------------------------------------------------------
// tv: N test vectors in the blocked FP64 layout with N right-hand sides.
__global__ __launch_bounds__(BS) void k_amg_gs(const double2 *__restrict__ tv, double2 *__restrict__ Pd,
                                               float2 *__restrict__ Pf, int N)
{
    __shared__ Red R;
    const int b = blockIdx.x, c = blockIdx.y, s = threadIdx.x, lane = s & 63, wave = s >> 6;
    for (int i = 0; i < N; ++i) {
        cx<double> w[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) w[k] = ldc<double>(tv + (((long)b * N + i) * 12 + 6 * c + k) * BS + s);
        for (int j = 0; j < i; ++j) {
            cx<double> q[6];
            double re = 0, im = 0;
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                q[k] = ldc<double>(Pd + pidx(b, c, j, N, k, s));
                re += q[k].re * w[k].re + q[k].im * w[k].im;
                im += q[k].re * w[k].im - q[k].im * w[k].re;
            }
            wave_put(R, lane, wave, 0, re, im);
            __syncthreads();
            const cx<double> h = wave_get(R, 0);
            __syncthreads();
#pragma unroll
            for (int k = 0; k < 6; ++k) w[k] = w[k] - h * q[k];
        }
        double n2 = 0;
#pragma unroll
        for (int k = 0; k < 6; ++k) n2 += w[k].re * w[k].re + w[k].im * w[k].im;
        wave_put(R, lane, wave, 0, n2, 0.0);
        __syncthreads();
        // a piece that vanishes on the aggregate (dependent vectors) gives a
        // zero column instead of NaN
        const double nn = wave_get(R, 0).re;
        const double inv = nn > 0 ? 1.0 / sqrt(nn) : 0.0;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const cx<double> p = inv * w[k];
            stc(Pd + pidx(b, c, i, N, k, s), p);
            stc(Pf + pidx(b, c, i, N, k, s), p);
        }
    }
}

// ---------------------------------------------------------------------------
// coarse operator: D_c[b][d][k'][k] = <P_{b,k}, (D P_{nbr_d(b),k'})|_b> at m0 = 0
// ---------------------------------------------------------------------------
struct AGeom {
    Geom g;
    int N;
    int r12;
};

// one hop into site s of block b from (bn, sn): forward (dir > 0) applies
// -1/2 (1 - g_mu) U_mu(x), backward -1/2 (1 + g_mu) U_mu(x - mu)^+, both
// times the boundary sign
__device__ __forceinline__ void hop_into(const double2 *__restrict__ links, bool r12, int b, int s, int bn, int sn,
                                         int mu, int dir, int sign, const cx<double> p[12], cx<double> q[12])
{
    cx<double> U[9], h[6], t[6];
    const double kk = sign > 0 ? -0.5 : 0.5;
    if (dir > 0) {
        load_link<double>(links + ((long)b * 4 + mu) * 9 * BS + s, r12, U);
        proj_m(mu, p, h);
        su3_mul(U, h, t);
        recon_m(mu, q, t, kk);
    } else {
        load_link<double>(links + ((long)bn * 4 + mu) * 9 * BS + sn, r12, U);
        proj_p(mu, p, h);
        su3_mul_adj(U, h, t);
        recon_p(mu, q, t, kk);
    }
}

__device__ __forceinline__ void load_col(const double2 *__restrict__ Pd, int b, int kp, int N, int s, cx<double> p[12])
{
    const int c = kp / N, i = kp % N;
#pragma unroll
    for (int k = 0; k < 12; ++k) p[k] = mk<double>(0, 0);
    // explicit halves: a run-time index into p would put it in scratch memory
    if (c == 0) {
#pragma unroll
        for (int k = 0; k < 6; ++k) p[k] = ldc<double>(Pd + pidx(b, 0, i, N, k, s));
    } else {
#pragma unroll
        for (int k = 0; k < 6; ++k) p[6 + k] = ldc<double>(Pd + pidx(b, 1, i, N, k, s));
    }
}

__global__ __launch_bounds__(BS) void k_amg_build(const double2 *__restrict__ Pd, const double2 *__restrict__ links,
                                                  const double2 *__restrict__ clov, double2 *__restrict__ Ad,
                                                  __half2 *__restrict__ Ah, AGeom a)
{
    __shared__ Red R;
    const int b = blockIdx.x, d = blockIdx.y, s = threadIdx.x, lane = s & 63, wave = s >> 6;
    const int N = a.N, N2 = 2 * N;
    int bc[4];
    block_coords(a.g, b, bc);
    const int mu = d == 0 ? 0 : (d - 1) >> 1, dir = (d - 1) & 1 ? -1 : 1;
    // the source block of this matrix
    int src = b;
    if (d > 0) {
        if (a.g.nb[mu] == 1) {
            // all hops of this direction stay in the block: counted in d = 0
            for (int e = s; e < N2 * N2; e += BS) {
                Ad[((long)b * 9 + d) * N2 * N2 + e] = make_double2(0, 0);
                Ah[((long)b * 9 + d) * N2 * N2 + e] = __floats2half2_rn(0.f, 0.f);
            }
            return;
        }
        const int up = bc[mu] + 1 == a.g.nb[mu] ? -(a.g.nb[mu] - 1) : 1;
        const int dn = bc[mu] == 0 ? a.g.nb[mu] - 1 : -1;
        src = b + (dir > 0 ? up : dn) * a.g.bstride[mu];
    }
    // this site's P rows for the dot products are re-read per column (L2)
    for (int kp = 0; kp < N2; ++kp) {
        cx<double> q[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) q[k] = mk<double>(0, 0);
        if (d == 0) {
            cx<double> p[12];
            load_col(Pd, b, kp, N, s, p);
            // (4 + C(x)) p(x): the mass is added at apply time
#pragma unroll 1
            for (int h = 0; h < 2; ++h) {
                cx<double> cl[18];
#pragma unroll
                for (int e = 0; e < 18; ++e) cl[e] = ldc<double>(clov + ((long)b * 36 + 18 * h + e) * BS + s);
                clover_half_mac<double>(cl, 4.0, p + 6 * h, q + 6 * h);
            }
            // hops whose neighbour lies in the block (with the boundary sign
            // when the block spans the whole direction)
#pragma unroll 1
            for (int m = 0; m < 4; ++m)
#pragma unroll 1
                for (int dr = -1; dr <= 1; dr += 2) {
                    int bn, sn, sign;
                    bool inb;
                    neighbour_rt(a.g, b, bc, s, m, dr, bn, sn, sign, inb);
                    if (!inb) continue;
                    cx<double> pn[12];
                    load_col(Pd, b, kp, N, sn, pn);
                    hop_into(links, a.r12, b, s, bn, sn, m, dr, sign, pn, q);
                }
        } else {
            int bn, sn, sign;
            bool inb;
            neighbour_rt(a.g, b, bc, s, mu, dir, bn, sn, sign, inb);
            if (!inb && bn == src) {
                cx<double> pn[12];
                load_col(Pd, src, kp, N, sn, pn);
                hop_into(links, a.r12, b, s, bn, sn, mu, dir, sign, pn, q);
            }
        }
        // entries (k, kp) for every row k = c * N + i
#pragma unroll
        for (int c = 0; c < 2; ++c)
            for (int i = 0; i < N; ++i) {
                double re = 0, im = 0;
#pragma unroll
                for (int e = 0; e < 6; ++e) {
                    const cx<double> pk = ldc<double>(Pd + pidx(b, c, i, N, e, s));
                    const cx<double> qe = q[6 * c + e];
                    re += pk.re * qe.re + pk.im * qe.im;
                    im += pk.re * qe.im - pk.im * qe.re;
                }
                wave_put(R, lane, wave, c * N + i, re, im);
            }
        __syncthreads();
        if (s < N2) {
            const cx<double> v = wave_get(R, s);
            const long o = (((long)b * 9 + d) * N2 + kp) * N2 + s;
            stc(Ad + o, v);
            stc(Ah + o, v);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// restriction x_c = P^+ eta and prolongation psi = P x_c (W slots; a slot's
// fine data at base + off[r] in the blocked layout with W right-hand sides)
// ---------------------------------------------------------------------------
// FP64 data are restricted and prolongated with the FP64 interpolation in
// FP64 arithmetic, FP32 data with the FP32 copy in FP32 arithmetic.
template <typename S> using PT = vec2_t<S>;

template <typename S>
__global__ __launch_bounds__(BS) void k_amg_restrict(const vec2_t<S> *__restrict__ in, const long *__restrict__ off,
                                                     const PT<S> *__restrict__ P, double2 *__restrict__ xc,
                                                     const int *__restrict__ active, int N, int nblocks, int W)
{
    __shared__ Red R;
    const int b = blockIdx.x, r = blockIdx.y, s = threadIdx.x, lane = s & 63, wave = s >> 6;
    if (active && !active[r]) return;
    const vec2_t<S> *e = in + (off ? off[r] : 0) + ((long)b * W + r) * 12 * BS + s;
    cx<S> v[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) v[k] = ldc<S>(e + k * BS);
#pragma unroll
    for (int c = 0; c < 2; ++c)
        for (int i = 0; i < N; ++i) {
            S re = 0, im = 0;
#pragma unroll
            for (int x = 0; x < 6; ++x) {
                const cx<S> p = ldc<S>(P + pidx(b, c, i, N, x, s));
                re = fma(p.re, v[6 * c + x].re, fma(p.im, v[6 * c + x].im, re));
                im = fma(p.re, v[6 * c + x].im, fma(-p.im, v[6 * c + x].re, im));
            }
            wave_put(R, lane, wave, c * N + i, (double)re, (double)im);
        }
    __syncthreads();
    if (s < 2 * N) stc(xc + ((long)r * nblocks + b) * 2 * N + s, wave_get(R, s));
}

template <typename S>
__global__ __launch_bounds__(BS) void k_amg_prolong(const double2 *__restrict__ xc, const PT<S> *__restrict__ P,
                                                    vec2_t<S> *__restrict__ out, const long *__restrict__ off,
                                                    const int *__restrict__ active, int N, int nblocks, int W)
{
    const int b = blockIdx.x, r = blockIdx.y, s = threadIdx.x;
    if (active && !active[r]) return;
    const double2 *x = xc + ((long)r * nblocks + b) * 2 * N;
    vec2_t<S> *o = out + (off ? off[r] : 0) + ((long)b * W + r) * 12 * BS + s;
#pragma unroll 1
    for (int c = 0; c < 2; ++c) {
        cx<S> acc[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) acc[k] = mk<S>(0, 0);
        for (int i = 0; i < N; ++i) {
            const cx<S> xi = ldc<S>(x + c * N + i);
#pragma unroll
            for (int k = 0; k < 6; ++k) cmac(acc[k], ldc<S>(P + pidx(b, c, i, N, k, s)), xi);
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) stc(o + (6 * c + k) * BS, acc[k]);
    }
}

// ---------------------------------------------------------------------------
// coarse vectors: y = (D_c + m0) x, and the device-side GMRES
// ---------------------------------------------------------------------------
struct CArgs {
    Geom g;
    int N;
    int nblocks;
    int W;
    const double *m0_dev;
    const int *active;
};

// neighbour block of b in direction d (1 + 2 mu: +mu, 2 + 2 mu: -mu)
__device__ __forceinline__ int cnbr(const Geom &g, int b, const int bc[4], int d)
{
    const int mu = (d - 1) >> 1;
    if ((d - 1) & 1) return bc[mu] == 0 ? b + (g.nb[mu] - 1) * g.bstride[mu] : b - g.bstride[mu];
    return bc[mu] + 1 == g.nb[mu] ? b - (g.nb[mu] - 1) * g.bstride[mu] : b + g.bstride[mu];
}

// One thread per (coarse site, row): y_r = (D_c + m0_r) x_r for the slots
// (slot r reads x + r * xs and writes y + r * ys; [nblocks][2N] each), the
// FP16 copy of D_c with FP64 vectors and accumulation.
// The nine 2N x 2N blocks of a row are read column by column, so the 2N
// threads of a coarse site read consecutive entries; x of the source block
// is the same for all of them.
struct GState;

// Per-slot state of the device GMRES (k <= CK steps).
struct GState {
    double2 H[(CK + 1) * CK]; // rotated Hessenberg (row i, column j at i * CK + j)
    double2 g[CK + 1];
    double2 sn[CK];
    double cs[CK];
    double bnorm;
    int ncol;   // columns built so far
    int closed; // the Krylov space closed (no further columns)
};

// The totals of values 0..count-1 over the CG group partials
// (part[(r * CG + group) * nvals + v]), computed by the whole workgroup --
// wavefront w takes values w, w + 4, ...; each lane adds CG / 64 partials,
// then a fixed-order DPP sum -- into out[] (shared).  Every workgroup gets
// the same totals.  Ends with a barrier.
__device__ __forceinline__ void group_totals(const double2 *__restrict__ part, int r, int nvals, int count,
                                             double2 *out)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int v = wave; v < count; v += CTPB / 64) {
        double re = 0, im = 0;
#pragma unroll
        for (int q = 0; q < CG / 64; ++q) {
            const double2 x = part[((long)r * CG + q * 64 + lane) * nvals + v];
            re += x.x;
            im += x.y;
        }
        re = wave_sum(re);
        im = wave_sum(im);
        if (lane == 63) out[v] = make_double2(re, im);
    }
    __syncthreads();
}

// |b|^2 partials (stage 0 of the solve)
__global__ __launch_bounds__(CTPB) void k_cg_norm(const double2 *__restrict__ bvec, double2 *__restrict__ part, CArgs a)
{
    __shared__ Red R;
    const int r = blockIdx.y, s = threadIdx.x;
    if (a.active && !a.active[r]) return;
    const long nrow = (long)a.nblocks * 2 * a.N;
    double n2 = 0;
    for (long t = (long)blockIdx.x * CTPB + s; t < nrow; t += (long)gridDim.x * CTPB) {
        const double2 v = bvec[(long)r * nrow + t];
        n2 += v.x * v.x + v.y * v.y;
    }
    wave_put(R, s & 63, s >> 6, 0, n2, 0.0);
    __syncthreads();
    if (s == 0) stc(part + ((long)r * CG + blockIdx.x), wave_get(R, 0));
}

// v_0 = b / |b|, state reset
__global__ __launch_bounds__(CTPB) void k_cg_init(const double2 *__restrict__ bvec, double2 *__restrict__ V,
                                                  const double2 *__restrict__ part, GState *__restrict__ st, CArgs a,
                                                  int kmax)
{
    const int r = blockIdx.y, s = threadIdx.x;
    if (a.active && !a.active[r]) return;
    const long nrow = (long)a.nblocks * 2 * a.N;
    __shared__ double2 tot[1];
    group_totals(part, r, 1, 1, tot);
    const double nb = sqrt(tot[0].x);
    const double inv = nb > 0 ? 1.0 / nb : 0.0;
    for (long t = (long)blockIdx.x * CTPB + s; t < nrow; t += (long)gridDim.x * CTPB) {
        const double2 v = bvec[(long)r * nrow + t];
        V[((long)r * (kmax + 1)) * nrow + t] = make_double2(v.x * inv, v.y * inv);
    }
    if (blockIdx.x == 0) {
        GState &S = st[r];
        for (int e = s; e < (CK + 1) * CK; e += CTPB) S.H[e] = make_double2(0, 0);
        for (int e = s; e <= CK; e += CTPB) S.g[e] = make_double2(0, 0);
        __syncthreads();
        if (s == 0) {
            S.bnorm = nb;
            S.ncol = 0;
            S.closed = nb > 0 ? 0 : 1;
            S.g[0] = make_double2(nb, 0);
        }
    }
}

// dots <v_i, w> for i <= j: partials per group
__global__ __launch_bounds__(CTPB) void k_cg_dots(const double2 *__restrict__ V, const double2 *__restrict__ w,
                                                  double2 *__restrict__ part, const GState *__restrict__ st, CArgs a,
                                                  int kmax, int j)
{
    __shared__ Red R;
    const int r = blockIdx.y, s = threadIdx.x;
    if ((a.active && !a.active[r]) || st[r].closed) return;
    const long nrow = (long)a.nblocks * 2 * a.N;
    const double2 *Vr = V + (long)r * (kmax + 1) * nrow;
    for (int i0 = 0; i0 <= j; i0 += 2 * NMAX) {
        const int ni = min(2 * NMAX, j + 1 - i0);
        for (int i = 0; i < ni; ++i) {
            double re = 0, im = 0;
            for (long t = (long)blockIdx.x * CTPB + s; t < nrow; t += (long)gridDim.x * CTPB) {
                const double2 v = Vr[(long)(i0 + i) * nrow + t], x = w[(long)r * nrow + t];
                re += v.x * x.x + v.y * x.y;
                im += v.x * x.y - v.y * x.x;
            }
            wave_put(R, s & 63, s >> 6, i, re, im);
        }
        __syncthreads();
        if (s < ni) stc(part + ((long)r * CG + blockIdx.x) * (kmax + 1) + i0 + s, wave_get(R, s));
        __syncthreads();
    }
}

// w -= sum_i h_i v_i (i <= j) with h_i the totals of the dot partials of
// the previous kernel; group 0 adds this pass's h into column j of H.  Then
// mode 1: the partial dots <v_i, w> of the updated w (the second pass of
// classical Gram-Schmidt); mode 2: the partials of |w|^2.
__global__ __launch_bounds__(CTPB) void k_cg_orth(const double2 *__restrict__ V, double2 *__restrict__ w,
                                                  const double2 *__restrict__ part, double2 *__restrict__ part_out,
                                                  GState *__restrict__ st, CArgs a, int kmax, int j, int mode)
{
    __shared__ Red R;
    __shared__ double2 h[CK + 1];
    const int r = blockIdx.y, s = threadIdx.x;
    if ((a.active && !a.active[r]) || st[r].closed) return;
    const long nrow = (long)a.nblocks * 2 * a.N;
    group_totals(part, r, kmax + 1, j + 1, h);
    const double2 *Vr = V + (long)r * (kmax + 1) * nrow;
    double2 *wr = w + (long)r * nrow;
    double n2 = 0;
    for (long t = (long)blockIdx.x * CTPB + s; t < nrow; t += (long)gridDim.x * CTPB) {
        cx<double> x = ldc<double>(wr + t);
#pragma unroll 4
        for (int i = 0; i <= j; ++i) x = x - ldc<double>(&h[i]) * ldc<double>(Vr + (long)i * nrow + t);
        stc(wr + t, x);
        n2 += x.re * x.re + x.im * x.im;
    }
    if (blockIdx.x == 0 && s == 0) {
        GState &S = st[r];
        for (int i = 0; i <= j; ++i) {
            double2 &e = S.H[i * CK + j];
            e.x += h[i].x;
            e.y += h[i].y;
        }
    }
    if (mode == 1) {
        // the rows of this thread were written by this thread: no barrier needed
        for (int i0 = 0; i0 <= j; i0 += 2 * NMAX) {
            const int ni = min(2 * NMAX, j + 1 - i0);
            for (int i = 0; i < ni; ++i) {
                double re = 0, im = 0;
                for (long t = (long)blockIdx.x * CTPB + s; t < nrow; t += (long)gridDim.x * CTPB) {
                    const double2 v = Vr[(long)(i0 + i) * nrow + t], x = wr[t];
                    re += v.x * x.x + v.y * x.y;
                    im += v.x * x.y - v.y * x.x;
                }
                wave_put(R, s & 63, s >> 6, i, re, im);
            }
            __syncthreads();
            if (s < ni) stc(part_out + ((long)r * CG + blockIdx.x) * (kmax + 1) + i0 + s, wave_get(R, s));
            __syncthreads();
        }
    } else if (mode == 2) {
        wave_put(R, s & 63, s >> 6, 0, n2, 0.0);
        __syncthreads();
        if (s == 0) stc(part_out + ((long)r * CG + blockIdx.x), wave_get(R, 0));
    }
}

// Givens rotation in the convention of LAPACK's zlartg: [c s; -conj(s) c]
// [f; g] = [r; 0] with c real >= 0
__device__ __forceinline__ void givens(cx<double> f, cx<double> g, double &c, cx<double> &sn, cx<double> &rr)
{
    const double af = sqrt(f.re * f.re + f.im * f.im), ag = sqrt(g.re * g.re + g.im * g.im);
    if (ag == 0.0) {
        c = 1.0;
        sn = mk<double>(0, 0);
        rr = f;
    } else if (af == 0.0) {
        c = 0.0;
        sn = (1.0 / ag) * conjx(g);
        rr = mk<double>(ag, 0);
    } else {
        const double nrm = sqrt(af * af + ag * ag);
        const cx<double> ph = (1.0 / af) * f;
        c = af / nrm;
        sn = (1.0 / nrm) * (ph * conjx(g));
        rr = nrm * ph;
    }
}

// beta = |w|; v_{j+1} = w / beta; column j of H rotated (group 0); a space
// that closed (beta tiny against |b|) stops growing
__global__ __launch_bounds__(CTPB) void k_cg_next(double2 *__restrict__ V, const double2 *__restrict__ w,
                                                  const double2 *__restrict__ part, GState *__restrict__ st, CArgs a,
                                                  int kmax, int j)
{
    const int r = blockIdx.y, s = threadIdx.x;
    if ((a.active && !a.active[r]) || st[r].closed) return;
    const long nrow = (long)a.nblocks * 2 * a.N;
    __shared__ double2 tot[1];
    group_totals(part, r, 1, 1, tot);
    const double beta = sqrt(tot[0].x);
    const bool closes = !(beta > 1e-14 * st[r].bnorm);
    if (!closes && j + 1 <= kmax) {
        const double inv = 1.0 / beta;
        double2 *Vn = V + ((long)r * (kmax + 1) + j + 1) * nrow;
        for (long t = (long)blockIdx.x * CTPB + s; t < nrow; t += (long)gridDim.x * CTPB) {
            const double2 x = w[(long)r * nrow + t];
            Vn[t] = make_double2(x.x * inv, x.y * inv);
        }
    }
    if (blockIdx.x == 0 && s == 0) {
        GState &S = st[r];
        // apply the earlier rotations to column j, then form rotation j
        for (int i = 0; i < j; ++i) {
            const cx<double> x0 = ldc<double>(&S.H[i * CK + j]), x1 = ldc<double>(&S.H[(i + 1) * CK + j]);
            const cx<double> sn = ldc<double>(&S.sn[i]);
            stc(&S.H[i * CK + j], S.cs[i] * x0 + sn * x1);
            stc(&S.H[(i + 1) * CK + j], S.cs[i] * x1 - conjx(sn) * x0);
        }
        double c;
        cx<double> sn, rr;
        givens(ldc<double>(&S.H[j * CK + j]), mk<double>(closes ? 0.0 : beta, 0), c, sn, rr);
        S.cs[j] = c;
        stc(&S.sn[j], sn);
        stc(&S.H[j * CK + j], rr);
        const cx<double> gj = ldc<double>(&S.g[j]);
        stc(&S.g[j], c * gj);
        stc(&S.g[j + 1], mk<double>(0, 0) - conjx(sn) * gj);
        S.ncol = j + 1;
        if (closes) S.closed = 1;
    }
}

// N2 = 2N is a compile-time constant so that the loads of a block row are
// issued together (a run-time loop waits on each pair of loads in turn)
template <int N2>
__global__ __launch_bounds__(CTPB) void k_coarse_apply(const __half2 *__restrict__ Ah, const double2 *__restrict__ x,
                                                       long xs, double2 *__restrict__ y, long ys,
                                                       const GState *__restrict__ st, CArgs a)
{
    const int r = blockIdx.y;
    if ((a.active && !a.active[r]) || (st && st[r].closed)) return;
    const double m0 = a.m0_dev[r];
    const long nrow = (long)a.nblocks * N2;
    const double2 *xr = x + (long)r * xs;
    for (long t = (long)blockIdx.x * CTPB + threadIdx.x; t < nrow; t += (long)gridDim.x * CTPB) {
        const int b = (int)(t / N2), k = (int)(t % N2);
        int bc[4];
        block_coords(a.g, b, bc);
        cx<double> acc = m0 * ldc<double>(xr + t);
#pragma unroll 1
        for (int d = 0; d < 9; ++d) {
            const int src = d == 0 ? b : cnbr(a.g, b, bc, d);
            const __half2 *Ac = Ah + ((long)b * 9 + d) * N2 * N2 + k;
            const double2 *xsrc = xr + (long)src * N2;
#pragma unroll 16
            for (int kp = 0; kp < N2; ++kp) cmac(acc, ldc<double>(Ac + (long)kp * N2), ldc<double>(xsrc + kp));
        }
        stc(y + (long)r * ys + t, acc);
    }
}

void coarse_apply(int N, dim3 grid, hipStream_t st, const __half2 *Ah, const double2 *x, long xs, double2 *y, long ys,
                  const GState *S, const CArgs &a)
{
    switch (N) {
#define DD_CA(n) case n: k_coarse_apply<2 * n><<<grid, CTPB, 0, st>>>(Ah, x, xs, y, ys, S, a); break;
        DD_CA(1) DD_CA(2) DD_CA(3) DD_CA(4) DD_CA(5) DD_CA(6) DD_CA(7) DD_CA(8)
        DD_CA(9) DD_CA(10) DD_CA(11) DD_CA(12) DD_CA(13) DD_CA(14) DD_CA(15) DD_CA(16)
#undef DD_CA
    default: break;
    }
}

// y = R^-1 g over the columns built, then x = V y (one slot per grid row)
__global__ __launch_bounds__(CTPB) void k_cg_finish(const double2 *__restrict__ V, double2 *__restrict__ x,
                                                    const GState *__restrict__ st, CArgs a, int kmax)
{
    __shared__ double2 y[CK];
    const int r = blockIdx.y, s = threadIdx.x;
    if (a.active && !a.active[r]) return;
    const GState &S = st[r];
    const int n = S.ncol;
    if (s == 0) {
        for (int i = n - 1; i >= 0; --i) {
            cx<double> acc = ldc<double>(&S.g[i]);
            for (int k = i + 1; k < n; ++k) acc = acc - ldc<double>(&S.H[i * CK + k]) * ldc<double>(&y[k]);
            const cx<double> d = ldc<double>(&S.H[i * CK + i]);
            const double dd = d.re * d.re + d.im * d.im;
            // a zero pivot only if the coarse operator is singular on the space
            const cx<double> q = dd > 0 ? (1.0 / dd) * (acc * conjx(d)) : mk<double>(0, 0);
            stc(&y[i], q);
        }
    }
    __syncthreads();
    const long nrow = (long)a.nblocks * 2 * a.N;
    const double2 *Vr = V + (long)r * (kmax + 1) * nrow;
    for (long t = (long)blockIdx.x * CTPB + s; t < nrow; t += (long)gridDim.x * CTPB) {
        cx<double> acc = mk<double>(0, 0);
#pragma unroll 4
        for (int i = 0; i < n; ++i) cmac(acc, ldc<double>(&y[i]), ldc<double>(Vr + (long)i * nrow + t));
        stc(x + (long)r * nrow + t, acc);
    }
}

// z (slot offsets) = a + b for the W slots
template <typename S>
__global__ __launch_bounds__(BS) void k_amg_sum(const vec2_t<S> *__restrict__ p, const vec2_t<S> *__restrict__ q,
                                                vec2_t<S> *__restrict__ z, const long *__restrict__ zoff,
                                                const int *__restrict__ active, int nblocks, int W)
{
    const int r = blockIdx.y, s = threadIdx.x;
    if (active && !active[r]) return;
    for (int b = blockIdx.x; b < nblocks; b += gridDim.x) {
        const long base = ((long)b * W + r) * 12 * BS + s;
        for (int c = 0; c < 12; ++c)
            stc(z + (zoff ? zoff[r] : 0) + base + c * BS,
                ldc<double>(p + base + c * BS) + ldc<double>(q + base + c * BS));
    }
}

// contiguous copy of W slots from base + off[r]
template <typename S>
__global__ __launch_bounds__(BS) void k_amg_gather(const vec2_t<S> *__restrict__ in, const long *__restrict__ off,
                                                   vec2_t<S> *__restrict__ out, const int *__restrict__ active,
                                                   int nblocks, int W)
{
    const int r = blockIdx.y, s = threadIdx.x;
    if (active && !active[r]) return;
    for (int b = blockIdx.x; b < nblocks; b += gridDim.x) {
        const long base = ((long)b * W + r) * 12 * BS + s;
        for (int c = 0; c < 12; ++c) out[base + c * BS] = in[(off ? off[r] : 0) + base + c * BS];
    }
}

// test-vector normalisation: per vector |v|^2 partials, then v /= |v|
template <typename S>
__global__ __launch_bounds__(BS) void k_tv_norm(const vec2_t<S> *__restrict__ v, double2 *__restrict__ part, int nblocks,
                                                int W)
{
    __shared__ Red R;
    const int r = blockIdx.y, s = threadIdx.x;
    double n2 = 0;
    for (int b = blockIdx.x; b < nblocks; b += gridDim.x) {
        const long base = ((long)b * W + r) * 12 * BS + s;
        for (int c = 0; c < 12; ++c) {
            const cx<double> x = ldc<double>(v + base + c * BS);
            n2 += x.re * x.re + x.im * x.im;
        }
    }
    wave_put(R, s & 63, s >> 6, 0, n2, 0.0);
    __syncthreads();
    if (s == 0) stc(part + (long)r * CG + blockIdx.x, wave_get(R, 0));
}

template <typename S>
__global__ __launch_bounds__(BS) void k_tv_scale(const vec2_t<S> *__restrict__ v, vec2_t<S> *__restrict__ out,
                                                 const double2 *__restrict__ part, int nblocks, int W)
{
    const int r = blockIdx.y, s = threadIdx.x;
    __shared__ double2 tot[1];
    group_totals(part, r, 1, 1, tot);
    const double inv = 1.0 / sqrt(tot[0].x);
    for (int b = blockIdx.x; b < nblocks; b += gridDim.x) {
        const long base = ((long)b * W + r) * 12 * BS + s;
        for (int c = 0; c < 12; ++c) stc(out + base + c * BS, inv * ldc<double>(v + base + c * BS));
    }
}

// FP32 blocked spinors -> FP64 (same layout)
__global__ __launch_bounds__(BS) void k_f32_to_f64(const float2 *__restrict__ in, double2 *__restrict__ out, long n)
{
    for (long i = (long)blockIdx.x * BS + threadIdx.x; i < n; i += (long)gridDim.x * BS) {
        const float2 v = in[i];
        out[i] = make_double2(v.x, v.y);
    }
}

unsigned grid_for(long n) { return (unsigned)std::min<long>((n + BS - 1) / BS, 8192); }

} // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct AmgWork {
    int W = 0, prec = -1, kmax = 0, N = 0;
    DevBuf xb, xx, V, w, partA, partB, partN, st; // coarse
    DevBuf et, ps, rr, dl, sapscr, m0;           // fine (smoother precision), masses
};

struct AmgData {
    int N = 0;
    dd_amg_params p{};
    DevBuf Pd, Pf, Ad, Ah; // P FP64 / FP32; D_c FP64 / FP16 (the copy the coarse solve reads)
    AmgWork work; // standalone calls and the setup's adaptive rounds
};

void AmgDeleter::operator()(AmgData *a) const { delete a; }

namespace {

CArgs cargs(const dd_ctx *ctx, int W, const double *m0_dev, const int *active)
{
    CArgs a{};
    for (int k = 0; k < 4; ++k) {
        a.g.nb[k] = ctx->g.nb[k];
        a.g.bstride[k] = ctx->g.bstride[k];
        a.g.bcs[k] = ctx->g.bcs[k];
    }
    a.g.nblocks = ctx->g.nblocks;
    a.N = ctx->amg->N;
    a.nblocks = ctx->g.nblocks;
    a.W = W;
    a.m0_dev = m0_dev;
    a.active = active;
    return a;
}

size_t ncoarse(const dd_ctx *ctx) { return (size_t)ctx->g.nblocks * 2 * ctx->amg->N; }

} // namespace

Status amg_reserve(dd_ctx *ctx, AmgWork &wk, int W, int prec, int kmax)
{
    kmax = std::max(kmax, ctx->amg->p.coarse_k);
    if (wk.W == W && wk.prec == prec && wk.kmax == kmax && wk.N == ctx->amg->N) return Status::ok();
    const size_t nc = ncoarse(ctx), cv = nc * 16 * W;
    DD_TRY(wk.xb.alloc(cv));
    DD_TRY(wk.xx.alloc(cv));
    DD_TRY(wk.V.alloc(cv * (kmax + 1)));
    DD_TRY(wk.w.alloc(cv));
    DD_TRY(wk.partA.alloc((size_t)W * CG * (kmax + 1) * 16));
    DD_TRY(wk.partB.alloc((size_t)W * CG * (kmax + 1) * 16));
    DD_TRY(wk.partN.alloc((size_t)W * CG * 16));
    DD_TRY(wk.st.alloc((size_t)W * sizeof(GState)));
    const size_t sb = spinor_bytes(ctx->g, prec, W);
    DD_TRY(wk.et.alloc(sb));
    DD_TRY(wk.ps.alloc(sb));
    DD_TRY(wk.rr.alloc(sb));
    DD_TRY(wk.dl.alloc(sb));
    DD_TRY(wk.sapscr.alloc(sap_scratch_bytes(ctx->g, prec, W)));
    DD_TRY(wk.m0.alloc((size_t)W * sizeof(double)));
    wk.W = W;
    wk.prec = prec;
    wk.kmax = kmax;
    wk.N = ctx->amg->N;
    return Status::ok();
}

AmgWork *amg_work_new() { return new AmgWork(); }
void AmgWorkDeleter::operator()(AmgWork *w) const { delete w; }

size_t amg_work_bytes(const dd_ctx *ctx, int W, int prec, int kmax, int N)
{
    const size_t nc = (size_t)ctx->g.nblocks * 2 * N, cv = nc * 16 * W;
    return cv * (kmax + 4) + (size_t)W * CG * (2 * kmax + 3) * 16 + W * sizeof(GState) +
           4 * spinor_bytes(ctx->g, prec, W) + sap_scratch_bytes(ctx->g, prec, W);
}

// k-step GMRES from zero on (D_c + m0_r) x_r = b_r for the W slots (b in
// wk.xb, x to wk.xx); device only.
Status coarse_gmres(dd_ctx *ctx, AmgWork &wk, int W, int k, const double *m0_dev, const int *active)
{
    AmgData &A = *ctx->amg;
    const CArgs a = cargs(ctx, W, m0_dev, active);
    const int kmax = wk.kmax;
    const dim3 grid(CG, W);
    hipStream_t st = ctx->stream;
    const long nrow = (long)ncoarse(ctx);
    double2 *V = wk.V.as<double2>(), *w = wk.w.as<double2>();
    GState *S = wk.st.as<GState>();
    // the operator: one row per thread (latency-bound at fewer); the
    // reductions: CG workgroups, one partial sum each
    const dim3 agrid((unsigned)std::min<long>((nrow + CTPB - 1) / CTPB, 8192), W);
    k_cg_norm<<<grid, CTPB, 0, st>>>(wk.xb.as<double2>(), wk.partN.as<double2>(), a);
    k_cg_init<<<grid, CTPB, 0, st>>>(wk.xb.as<double2>(), V, wk.partN.as<double2>(), S, a, kmax);
    for (int j = 0; j < k; ++j) {
        // w = (D_c + m0) v_j
        coarse_apply(A.N, agrid, st, A.Ah.as<__half2>(), V + (long)j * nrow, (long)(kmax + 1) * nrow, w, nrow, S, a);
        k_cg_dots<<<grid, CTPB, 0, st>>>(V, w, wk.partA.as<double2>(), S, a, kmax, j);
        k_cg_orth<<<grid, CTPB, 0, st>>>(V, w, wk.partA.as<double2>(), wk.partB.as<double2>(), S, a, kmax, j, 1);
        k_cg_orth<<<grid, CTPB, 0, st>>>(V, w, wk.partB.as<double2>(), wk.partN.as<double2>(), S, a, kmax, j, 2);
        k_cg_next<<<grid, CTPB, 0, st>>>(V, w, wk.partN.as<double2>(), S, a, kmax, j);
    }
    k_cg_finish<<<grid, CTPB, 0, st>>>(V, wk.xx.as<double2>(), S, a, kmax);
    DD_HIP_TRY(hipGetLastError());
    return Status::ok();
}

// The two-grid preconditioner for W slots: z = P x_c + SAP_nu(eta - D P x_c),
// x_c the coarse solve of D_c x_c = P^+ eta.  eta (z): slot r at base +
// off[r] in the blocked layout with W right-hand sides, precision prec.
Status run_two_grid(dd_ctx *ctx, AmgWork &wk, int W, const void *eta, const long *eta_off, int prec, void *z,
                    const long *z_off, const double *m0_dev, const int *active)
{
    AmgData &A = *ctx->amg;
    const int N = A.N, nb = ctx->g.nblocks;
    hipStream_t st = ctx->stream;
    const dim3 bg(nb, W), sg(std::min(nb, 1024), W);
    const void *e = eta;
    if (eta_off) {
        if (prec == DD_F64)
            k_amg_gather<double><<<sg, BS, 0, st>>>(static_cast<const double2 *>(eta), eta_off, wk.et.as<double2>(), active, nb, W);
        else
            k_amg_gather<float><<<sg, BS, 0, st>>>(static_cast<const float2 *>(eta), eta_off, wk.et.as<float2>(), active, nb, W);
        e = wk.et.p;
    }
    {
        ProfScope ps(ctx->prof, st, K_AMG_RESTRICT, (double)spinor_bytes(ctx->g, prec, W) * (1 + N), 0.0);
        if (prec == DD_F64)
            k_amg_restrict<double><<<bg, BS, 0, st>>>(static_cast<const double2 *>(e), nullptr, A.Pd.as<double2>(), wk.xb.as<double2>(), active, N, nb, W);
        else
            k_amg_restrict<float><<<bg, BS, 0, st>>>(static_cast<const float2 *>(e), nullptr, A.Pf.as<float2>(), wk.xb.as<double2>(), active, N, nb, W);
    }
    {
        ProfScope ps(ctx->prof, st, K_AMG_COARSE, 0.0, 0.0);
        DD_TRY(coarse_gmres(ctx, wk, W, A.p.coarse_k, m0_dev, active));
    }
    // psi_0 = P x_c: straight into z when no post-smoothing follows
    const bool post = A.p.post_ncy > 0;
    {
        ProfScope ps(ctx->prof, st, K_AMG_PROLONG, (double)spinor_bytes(ctx->g, prec, W) * (1 + N), 0.0);
        if (prec == DD_F64)
            k_amg_prolong<double><<<bg, BS, 0, st>>>(wk.xx.as<double2>(), A.Pd.as<double2>(),
                                                     post ? wk.ps.as<double2>() : static_cast<double2 *>(z),
                                                     post ? nullptr : z_off, active, N, nb, W);
        else
            k_amg_prolong<float><<<bg, BS, 0, st>>>(wk.xx.as<double2>(), A.Pf.as<float2>(),
                                                    post ? wk.ps.as<float2>() : static_cast<float2 *>(z),
                                                    post ? nullptr : z_off, active, N, nb, W);
    }
    DD_HIP_TRY(hipGetLastError());
    if (!post) return Status::ok();
    // r = eta - D psi_0, delta = SAP(r), z = psi_0 + delta
    DD_TRY(launch_dslash(ctx, nullptr, W, wk.ps.p, prec, wk.rr.p, prec, prec, static_cast<const double *>(e), m0_dev,
                         nullptr, active));
    SapSlots ss;
    ss.m0_dev = m0_dev;
    ss.active = active;
    ss.scratch = wk.sapscr.p;
    DD_TRY(run_sap(ctx, nullptr, W, wk.rr.p, wk.dl.p, A.p.post_ncy, A.p.post_nmr, prec, &ss, false));
    if (prec == DD_F64)
        k_amg_sum<double><<<sg, BS, 0, st>>>(wk.ps.as<double2>(), wk.dl.as<double2>(), static_cast<double2 *>(z), z_off,
                                             active, nb, W);
    else
        k_amg_sum<float><<<sg, BS, 0, st>>>(wk.ps.as<float2>(), wk.dl.as<float2>(), static_cast<float2 *>(z), z_off,
                                            active, nb, W);
    DD_HIP_TRY(hipGetLastError());
    return Status::ok();
}

namespace {

Status build_P_Dc(dd_ctx *ctx, const double2 *tv64)
{
    AmgData &A = *ctx->amg;
    const int N = A.N, nb = ctx->g.nblocks;
    k_amg_gs<<<dim3(nb, 2), BS, 0, ctx->stream>>>(tv64, A.Pd.as<double2>(), A.Pf.as<float2>(), N);
    DD_HIP_TRY(hipGetLastError());
    AGeom ag{};
    for (int k = 0; k < 4; ++k) {
        ag.g.nb[k] = ctx->g.nb[k];
        ag.g.bstride[k] = ctx->g.bstride[k];
        ag.g.bcs[k] = ctx->g.bcs[k];
    }
    ag.g.nblocks = nb;
    ag.N = N;
    ag.r12 = ctx->link_r12 ? 1 : 0;
    k_amg_build<<<dim3(nb, 9), BS, 0, ctx->stream>>>(A.Pd.as<double2>(), ctx->links[DD_F64].as<double2>(),
                                                     ctx->clover[DD_F64].as<double2>(), A.Ad.as<double2>(),
                                                     A.Ah.as<__half2>(), ag);
    DD_HIP_TRY(hipGetLastError());
    return Status::ok();
}

template <typename S> Status normalise(dd_ctx *ctx, const void *in, void *out, DevBuf &part, int N)
{
    const int nb = ctx->g.nblocks;
    const dim3 g(CG, N);
    k_tv_norm<S><<<g, BS, 0, ctx->stream>>>(static_cast<const vec2_t<S> *>(in), part.as<double2>(), nb, N);
    k_tv_scale<S><<<g, BS, 0, ctx->stream>>>(static_cast<const vec2_t<S> *>(in), static_cast<vec2_t<S> *>(out),
                                              part.as<double2>(), nb, N);
    DD_HIP_TRY(hipGetLastError());
    return Status::ok();
}

} // namespace

Status amg_setup(dd_ctx *ctx, double m0, const double *v0, const dd_amg_params &p)
{
    if (p.nvec < 1 || p.nvec > NMAX || p.setup_iters < 0 || p.setup_ncy < 1 || p.setup_nmr < 1 || p.adapt < 0 ||
        p.coarse_k < 1 || p.coarse_k > CK || p.post_ncy < 0 || p.post_nmr < 0 ||
        (p.setup_prec != DD_F64 && p.setup_prec != DD_F32))
        return Status{DD_INVALID_ARG, "dd_amg_setup: bad parameters (1 <= nvec <= 16, 1 <= coarse_k <= 32, "
                                      "setup_prec FP64 or FP32, ...)"};
    bool bad = false;
    DD_TRY(any_nonfinite(ctx, v0, (size_t)ctx->g.V * 24 * p.nvec, bad));
    if (bad) return Status{DD_NAN, "dd_amg_setup: starting vectors hold NaN or Inf"};
    ctx->amg.reset(new AmgData());
    AmgData &A = *ctx->amg;
    A.N = p.nvec;
    A.p = p;
    const int N = A.N, sp = p.setup_prec;
    const size_t pbytes = (size_t)ctx->g.nblocks * 2 * N * 6 * BS;
    DD_TRY(A.Pd.alloc(pbytes * 16));
    DD_TRY(A.Pf.alloc(pbytes * 8));
    const size_t abytes = (size_t)ctx->g.nblocks * 9 * 4 * N * N;
    DD_TRY(A.Ad.alloc(abytes * 16));
    DD_TRY(A.Ah.alloc(abytes * 4));
    DevBuf ta, tb, t64, part;
    DD_TRY(ta.alloc(spinor_bytes(ctx->g, sp, N)));
    DD_TRY(tb.alloc(spinor_bytes(ctx->g, sp, N)));
    DD_TRY(part.alloc((size_t)N * CG * 16));
    DD_TRY(pack_spinor(ctx, v0, ta.p, sp, N));
    std::vector<double> m0s(N, m0);
    // inverse iteration with the Schwarz smoother: v <- SAP(v) / |SAP(v)|
    for (int it = 0; it < p.setup_iters; ++it) {
        DD_TRY(run_sap(ctx, m0s.data(), N, ta.p, tb.p, p.setup_ncy, p.setup_nmr, sp));
        DD_TRY(sp == DD_F64 ? normalise<double>(ctx, tb.p, ta.p, part, N) : normalise<float>(ctx, tb.p, ta.p, part, N));
    }
    auto build = [&]() -> Status {
        const double2 *tv = ta.as<double2>();
        if (sp == DD_F32) {
            DD_TRY(t64.alloc(spinor_bytes(ctx->g, DD_F64, N)));
            const long n = (long)ctx->g.V * 12 * N;
            k_f32_to_f64<<<grid_for(n), BS, 0, ctx->stream>>>(ta.as<float2>(), t64.as<double2>(), n);
            DD_HIP_TRY(hipGetLastError());
            tv = t64.as<double2>();
        }
        return build_P_Dc(ctx, tv);
    };
    DD_TRY(build());
    // adaptive rounds: the current two-grid method in place of the smoother
    if (p.adapt > 0) {
        DD_TRY(amg_reserve(ctx, A.work, N, sp, 0));
        DD_HIP_TRY(hipMemcpyAsync(A.work.m0.p, m0s.data(), N * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
        for (int r = 0; r < p.adapt; ++r) {
            DD_TRY(run_two_grid(ctx, A.work, N, ta.p, nullptr, sp, tb.p, nullptr, A.work.m0.as<double>(), nullptr));
            DD_TRY(sp == DD_F64 ? normalise<double>(ctx, tb.p, ta.p, part, N) : normalise<float>(ctx, tb.p, ta.p, part, N));
            DD_TRY(build());
        }
    }
    DD_HIP_TRY(hipStreamSynchronize(ctx->stream));
    return Status::ok();
}

size_t amg_coarse_size(const dd_ctx *ctx) { return ctx->amg ? ncoarse(ctx) : 0; }

Status amg_export(dd_ctx *ctx, double *P_host, double *A_host)
{
    AmgData &A = *ctx->amg;
    if (P_host) DD_HIP_TRY(hipMemcpy(P_host, A.Pd.p, A.Pd.bytes, hipMemcpyDeviceToHost));
    if (A_host) DD_HIP_TRY(hipMemcpy(A_host, A.Ad.p, A.Ad.bytes, hipMemcpyDeviceToHost));
    return Status::ok();
}

Status amg_standalone(dd_ctx *ctx, int op, const double *m0, int nrhs, const void *in, void *out, int prec, int k)
{
    AmgData &A = *ctx->amg;
    AmgWork &wk = A.work;
    if (op == 3 && (k < 1 || k > CK)) return Status{DD_INVALID_ARG, "dd_amg_coarse_solve: 1 <= k <= 32"};
    DD_TRY(amg_reserve(ctx, wk, nrhs, prec, op == 3 ? k : 0));
    std::vector<double> masses(nrhs, 0.0);
    if (m0) masses.assign(m0, m0 + nrhs);
    DD_HIP_TRY(hipMemcpyAsync(wk.m0.p, masses.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    DD_HIP_TRY(hipStreamSynchronize(ctx->stream)); // masses is a host temporary
    const int N = A.N, nb = ctx->g.nblocks;
    const dim3 bg(nb, nrhs), grid(CG, nrhs);
    const size_t cv = ncoarse(ctx) * 16 * nrhs;
    const CArgs a = cargs(ctx, nrhs, wk.m0.as<double>(), nullptr);
    switch (op) {
    case 0: // restrict: out (coarse) = P^+ in
        if (prec == DD_F64)
            k_amg_restrict<double><<<bg, BS, 0, ctx->stream>>>(static_cast<const double2 *>(in), nullptr, A.Pd.as<double2>(), static_cast<double2 *>(out), nullptr, N, nb, nrhs);
        else
            k_amg_restrict<float><<<bg, BS, 0, ctx->stream>>>(static_cast<const float2 *>(in), nullptr, A.Pf.as<float2>(), static_cast<double2 *>(out), nullptr, N, nb, nrhs);
        break;
    case 1: // prolong: out (fine) = P in
        if (prec == DD_F64)
            k_amg_prolong<double><<<bg, BS, 0, ctx->stream>>>(static_cast<const double2 *>(in), A.Pd.as<double2>(), static_cast<double2 *>(out), nullptr, nullptr, N, nb, nrhs);
        else
            k_amg_prolong<float><<<bg, BS, 0, ctx->stream>>>(static_cast<const double2 *>(in), A.Pf.as<float2>(), static_cast<float2 *>(out), nullptr, nullptr, N, nb, nrhs);
        break;
    case 2: // coarse apply
        coarse_apply(N, dim3((unsigned)std::min<long>(((long)ncoarse(ctx) + CTPB - 1) / CTPB, 8192), nrhs),
                     ctx->stream, A.Ah.as<__half2>(), static_cast<const double2 *>(in), (long)ncoarse(ctx),
                     static_cast<double2 *>(out), (long)ncoarse(ctx), nullptr, a);
        break;
    case 3: // coarse solve with k steps
        DD_HIP_TRY(hipMemcpyAsync(wk.xb.p, in, cv, hipMemcpyDeviceToDevice, ctx->stream));
        DD_TRY(coarse_gmres(ctx, wk, nrhs, k, wk.m0.as<double>(), nullptr));
        DD_HIP_TRY(hipMemcpyAsync(out, wk.xx.p, cv, hipMemcpyDeviceToDevice, ctx->stream));
        break;
    default: // two-grid preconditioner
        DD_TRY(run_two_grid(ctx, wk, nrhs, in, nullptr, prec, out, nullptr, wk.m0.as<double>(), nullptr));
        break;
    }
    DD_HIP_TRY(hipGetLastError());
    return Status::ok();
}

} // namespace dd
