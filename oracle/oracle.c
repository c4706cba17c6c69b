/*
 * Plain FP64 CPU oracle: Wilson-clover operator, block MR, red-black SAP and
 * FGMRES.  TEST INFRASTRUCTURE ONLY (see oracle.h for the rules, the layouts
 * and the literature each definition follows).
 *
 * Everything here is deliberately direct: dense 4x4 gamma matrices, dense
 * 12x12 clover per site, neighbour lookups by coordinates, no blocking, no
 * fusion and no reordering beyond what the definitions state.  OpenMP only
 * distributes independent sites or independent blocks; every reduction is
 * summed in a fixed order so that results do not depend on thread timing.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Gamma matrices, Euclidean chiral basis:                                   */
/*   gamma_k = [[0, -i sigma_k], [i sigma_k, 0]] (k = 1, 2, 3),              */
/*   gamma_4 = [[0, 1], [1, 0]],  gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4  */
/*           = diag(1, 1, -1, -1).                                           */
/* Index 0..3 is x, y, z, t.                                                 */
/* ------------------------------------------------------------------------ */
static const double complex GAMMA[4][4][4] = {
    /* gamma_x */
    {{0, 0, 0, -I}, {0, 0, -I, 0}, {0, I, 0, 0}, {I, 0, 0, 0}},
    /* gamma_y */
    {{0, 0, 0, -1}, {0, 0, 1, 0}, {0, 1, 0, 0}, {-1, 0, 0, 0}},
    /* gamma_z */
    {{0, 0, -I, 0}, {0, 0, 0, I}, {I, 0, 0, 0}, {0, -I, 0, 0}},
    /* gamma_t */
    {{0, 0, 1, 0}, {0, 0, 0, 1}, {1, 0, 0, 0}, {0, 1, 0, 0}},
};

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Geometry                                                                  */
/* ------------------------------------------------------------------------ */
static long volume_of(const int L[4]) { return (long)L[0] * L[1] * L[2] * L[3]; }

static void coords_of(const int L[4], long s, int c[4])
{
    for (int mu = 0; mu < 4; ++mu) {
        c[mu] = (int)(s % L[mu]);
        s /= L[mu];
    }
}

static long index_of(const int L[4], const int c[4])
{
    return c[0] + (long)L[0] * (c[1] + (long)L[1] * (c[2] + (long)L[2] * c[3]));
}

/* Site reached from s by `step` (+1 or -1) in direction mu, periodic.
 * *wrapped is set when the step crosses the lattice boundary. */
static long shift(const int L[4], long s, int mu, int step, int *wrapped)
{
    int c[4];
    coords_of(L, s, c);
    int v = c[mu] + step;
    int w = 0;
    if (v >= L[mu]) { v -= L[mu]; w = 1; }
    if (v < 0) { v += L[mu]; w = 1; }
    c[mu] = v;
    if (wrapped) *wrapped = w;
    return index_of(L, c);
}

/* Gauge links are periodic: no boundary sign. */
static long gshift(const int L[4], long s, int mu, int step) { return shift(L, s, mu, step, NULL); }

static const double complex *link(const double complex *U, long s, int mu) { return U + (s * 4 + mu) * 9; }

/* ------------------------------------------------------------------------ */
/* Small dense helpers                                                       */
/* ------------------------------------------------------------------------ */
/* c = a * b (3x3), with optional adjoints of a and/or b. */
static void mat3_mul(const double complex *a, int adj_a, const double complex *b, int adj_b,
                     double complex *c)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double complex acc = 0;
            for (int k = 0; k < 3; ++k) {
                double complex aik = adj_a ? conj(a[k * 3 + i]) : a[i * 3 + k];
                double complex bkj = adj_b ? conj(b[j * 3 + k]) : b[k * 3 + j];
                acc += aik * bkj;
            }
            c[i * 3 + j] = acc;
        }
}

/* Product of four links, each possibly adjoint. */
static void leaf(const double complex *a, int da, const double complex *b, int db,
                 const double complex *c, int dc, const double complex *d, int dd,
                 double complex *out)
{
    double complex t1[9], t2[9];
    mat3_mul(a, da, b, db, t1);
    mat3_mul(t1, 0, c, dc, t2);
    mat3_mul(t2, 0, d, dd, out);
}

/* out[spin][a] = sum_b M[a][b] in[spin][b] (M or its adjoint). */
static void colour_apply(const double complex *M, int adj, const double complex *in, double complex *out)
{
    for (int s = 0; s < 4; ++s)
        for (int a = 0; a < 3; ++a) {
            double complex acc = 0;
            for (int b = 0; b < 3; ++b) acc += (adj ? conj(M[b * 3 + a]) : M[a * 3 + b]) * in[s * 3 + b];
            out[s * 3 + a] = acc;
        }
}

/* out[s][a] = sum_t G[s][t] in[t][a] */
static void spin_apply(const double complex G[4][4], const double complex *in, double complex *out)
{
    for (int s = 0; s < 4; ++s)
        for (int a = 0; a < 3; ++a) {
            double complex acc = 0;
            for (int t = 0; t < 4; ++t) acc += G[s][t] * in[t * 3 + a];
            out[s * 3 + a] = acc;
        }
}

/* ------------------------------------------------------------------------ */
/* Clover term                                                               */
/*   C(x) = -(csw/32) sum_{mu,nu} gamma_mu gamma_nu (x) (Q_munu(x) - Q_numu(x)) */
/*   Q_munu(x) = U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+                   */
/*             + U_nu(x) U_mu(x-mu+nu)^+ U_nu(x-mu)^+ U_mu(x-mu)             */
/*             + U_mu(x-mu)^+ U_nu(x-mu-nu)^+ U_mu(x-mu-nu) U_nu(x-nu)       */
/*             + U_nu(x-nu)^+ U_mu(x-nu) U_nu(x-nu+mu) U_mu(x)^+             */
/* (Sheikholeslami-Wohlert clover leaves; no colour-trace subtraction.)      */
/* ------------------------------------------------------------------------ */
static void clover_leaves(const int L[4], const double complex *U, long x, int mu, int nu,
                          double complex Q[9])
{
    long xpm = gshift(L, x, mu, +1);
    long xpn = gshift(L, x, nu, +1);
    long xmm = gshift(L, x, mu, -1);
    long xmn = gshift(L, x, nu, -1);
    long xmm_pn = gshift(L, xmm, nu, +1);
    long xmm_mn = gshift(L, xmm, nu, -1);
    long xmn_pm = gshift(L, xmn, mu, +1);
    double complex t[9];
    for (int i = 0; i < 9; ++i) Q[i] = 0;
    leaf(link(U, x, mu), 0, link(U, xpm, nu), 0, link(U, xpn, mu), 1, link(U, x, nu), 1, t);
    for (int i = 0; i < 9; ++i) Q[i] += t[i];
    leaf(link(U, x, nu), 0, link(U, xmm_pn, mu), 1, link(U, xmm, nu), 1, link(U, xmm, mu), 0, t);
    for (int i = 0; i < 9; ++i) Q[i] += t[i];
    leaf(link(U, xmm, mu), 1, link(U, xmm_mn, nu), 1, link(U, xmm_mn, mu), 0, link(U, xmn, nu), 0, t);
    for (int i = 0; i < 9; ++i) Q[i] += t[i];
    leaf(link(U, xmn, nu), 1, link(U, xmn, mu), 0, link(U, xmn_pm, nu), 0, link(U, x, mu), 1, t);
    for (int i = 0; i < 9; ++i) Q[i] += t[i];
}

void or_clover_site(const int L[4], const double complex *U, double csw, long site, double complex *Cx)
{
    for (int i = 0; i < 144; ++i) Cx[i] = 0;
    for (int mu = 0; mu < 4; ++mu)
        for (int nu = 0; nu < 4; ++nu) {
            if (mu == nu) continue; /* Q_mumu - Q_mumu = 0 */
            double complex Qmn[9], Qnm[9], F[9];
            clover_leaves(L, U, site, mu, nu, Qmn);
            clover_leaves(L, U, site, nu, mu, Qnm);
            for (int i = 0; i < 9; ++i) F[i] = Qmn[i] - Qnm[i];
            double complex G[4][4];
            for (int s = 0; s < 4; ++s)
                for (int t = 0; t < 4; ++t) {
                    double complex acc = 0;
                    for (int k = 0; k < 4; ++k) acc += GAMMA[mu][s][k] * GAMMA[nu][k][t];
                    G[s][t] = acc;
                }
            for (int s = 0; s < 4; ++s)
                for (int a = 0; a < 3; ++a)
                    for (int t = 0; t < 4; ++t)
                        for (int b = 0; b < 3; ++b)
                            Cx[(s * 3 + a) * 12 + t * 3 + b] += -(csw / 32.0) * G[s][t] * F[a * 3 + b];
        }
}

void or_clover_field(const int L[4], const double complex *U, double csw, double complex *C)
{
    long V = volume_of(L);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; ++s) or_clover_site(L, U, csw, s, C + s * 144);
}

/* ------------------------------------------------------------------------ */
/* Wilson-clover operator at one site                                        */
/*   (D psi)(x) = (4 + m0) psi(x) + C(x) psi(x)                              */
/*     - 1/2 sum_mu [ (1 - gamma_mu) U_mu(x) psi(x+mu)                       */
/*                  + (1 + gamma_mu) U_mu(x-mu)^+ psi(x-mu) ]                */
/* A hop that crosses the lattice boundary in mu is multiplied by bcs[mu].   */
/* `inblock` (may be NULL) restricts the hops to neighbours inside a block:  */
/* a neighbour for which it returns 0 contributes nothing.                   */
/* ------------------------------------------------------------------------ */
typedef struct {
    const int *L;
    const int *B;
    int bc[4];
} block_filter;

static int in_block(const block_filter *f, long s)
{
    int c[4];
    coords_of(f->L, s, c);
    for (int mu = 0; mu < 4; ++mu)
        if (c[mu] / f->B[mu] != f->bc[mu]) return 0;
    return 1;
}

static void dirac_site(const int L[4], const int bcs[4], const double complex *U, const double complex *Cx,
                       double m0, const double complex *in, long x, const block_filter *filt,
                       double complex *out /* [12] */)
{
    const double complex *px = in + x * 12;
    for (int i = 0; i < 12; ++i) {
        double complex acc = (4.0 + m0) * px[i];
        for (int j = 0; j < 12; ++j) acc += Cx[i * 12 + j] * px[j];
        out[i] = acc;
    }
    for (int mu = 0; mu < 4; ++mu) {
        double complex chi[12], gchi[12];
        int wrapped;
        /* forward hop: -1/2 (1 - gamma_mu) U_mu(x) psi(x+mu) */
        long xf = shift(L, x, mu, +1, &wrapped);
        if (!filt || in_block(filt, xf)) {
            double sign = wrapped ? (double)bcs[mu] : 1.0;
            colour_apply(link(U, x, mu), 0, in + xf * 12, chi);
            spin_apply(GAMMA[mu], chi, gchi);
            for (int i = 0; i < 12; ++i) out[i] -= 0.5 * sign * (chi[i] - gchi[i]);
        }
        /* backward hop: -1/2 (1 + gamma_mu) U_mu(x-mu)^+ psi(x-mu) */
        long xb = shift(L, x, mu, -1, &wrapped);
        if (!filt || in_block(filt, xb)) {
            double sign = wrapped ? (double)bcs[mu] : 1.0;
            colour_apply(link(U, xb, mu), 1, in + xb * 12, chi);
            spin_apply(GAMMA[mu], chi, gchi);
            for (int i = 0; i < 12; ++i) out[i] -= 0.5 * sign * (chi[i] + gchi[i]);
        }
    }
}

void or_apply_D(const int L[4], const int bcs[4], const double complex *U, const double complex *C,
                double m0, const double complex *in, double complex *out)
{
    long V = volume_of(L);
#pragma omp parallel for schedule(static)
    for (long x = 0; x < V; ++x) dirac_site(L, bcs, U, C + x * 144, m0, in, x, NULL, out + x * 12);
}

void or_apply_D_sites(const int L[4], const int bcs[4], const double complex *U, double csw, double m0,
                      const double complex *in, const long *sites, long n, double complex *out)
{
#pragma omp parallel for schedule(static)
    for (long k = 0; k < n; ++k) {
        double complex Cx[144];
        or_clover_site(L, U, csw, sites[k], Cx);
        dirac_site(L, bcs, U, Cx, m0, in, sites[k], NULL, out + k * 12);
    }
}

void or_apply_D_sites_nv(const int L[4], const int bcs[4], const double complex *U, double csw, double m0,
                         const double complex *in, long nvec, const long *sites, long n, double complex *out)
{
    long V = volume_of(L);
#pragma omp parallel for schedule(static)
    for (long k = 0; k < n; ++k) {
        double complex Cx[144];
        or_clover_site(L, U, csw, sites[k], Cx);
        for (long v = 0; v < nvec; ++v)
            dirac_site(L, bcs, U, Cx, m0, in + v * V * 12, sites[k], NULL, out + (v * n + k) * 12);
    }
}

/* ------------------------------------------------------------------------ */
/* Blocks                                                                    */
/* ------------------------------------------------------------------------ */
static int blocking_valid(const int L[4], const int B[4])
{
    for (int mu = 0; mu < 4; ++mu) {
        if (B[mu] < 1 || L[mu] % B[mu] != 0) return 0;
        int nb = L[mu] / B[mu];
        if (nb != 1 && nb % 2 != 0) return 0; /* red-black needs an even count (or one) */
    }
    return 1;
}

static long num_blocks(const int L[4], const int B[4])
{
    long n = 1;
    for (int mu = 0; mu < 4; ++mu) n *= L[mu] / B[mu];
    return n;
}

/* Block coordinates of block id. */
static void block_coords(const int L[4], const int B[4], long id, int bc[4])
{
    for (int mu = 0; mu < 4; ++mu) {
        int nb = L[mu] / B[mu];
        bc[mu] = (int)(id % nb);
        id /= nb;
    }
}

static int block_colour(const int bc[4]) { return (bc[0] + bc[1] + bc[2] + bc[3]) % 2; }

/* Global site of the k-th site of the block (lexicographic inside the block). */
static long block_site(const int L[4], const int B[4], const int bc[4], long k)
{
    int c[4];
    for (int mu = 0; mu < 4; ++mu) {
        c[mu] = bc[mu] * B[mu] + (int)(k % B[mu]);
        k /= B[mu];
    }
    return index_of(L, c);
}

static long block_volume(const int B[4]) { return (long)B[0] * B[1] * B[2] * B[3]; }

/* out = D_BB in on the sites of block bc (whole-lattice arrays). */
static void apply_DBB_coords(const int L[4], const int B[4], const int bcs[4], const double complex *U,
                             const double complex *C, double m0, const int bc[4],
                             const double complex *in, double complex *out)
{
    block_filter f = {L, B, {bc[0], bc[1], bc[2], bc[3]}};
    long nb = block_volume(B);
    for (long k = 0; k < nb; ++k) {
        long x = block_site(L, B, bc, k);
        dirac_site(L, bcs, U, C + x * 144, m0, in, x, &f, out + x * 12);
    }
}

int or_apply_DBB(const int L[4], const int B[4], const int bcs[4], const double complex *U,
                 const double complex *C, double m0, long block_id, const double complex *in,
                 double complex *out)
{
    if (!blocking_valid(L, B) || block_id < 0 || block_id >= num_blocks(L, B)) return -1;
    int bc[4];
    block_coords(L, B, block_id, bc);
    apply_DBB_coords(L, B, bcs, U, C, m0, bc, in, out);
    return 0;
}

/* Algorithm M (minimal residual on one block), Saad Sec. 5.3.2:
 *   delta = 0, r = rho_B
 *   repeat nmr times: q = D_BB r; stop if <q,q> = 0;
 *                     alpha = <q,r>/<q,q>; delta += alpha r; r -= alpha q
 * Work arrays are whole-lattice sized scratch `r`, `q` (only block sites used). */
static int mr_block_coords(const int L[4], const int B[4], const int bcs[4], const double complex *U,
                           const double complex *C, double m0, const int bc[4], int nmr,
                           const double complex *rho, double complex *delta, double complex *r,
                           double complex *q)
{
    long nb = block_volume(B);
    for (long k = 0; k < nb; ++k) {
        long x = block_site(L, B, bc, k);
        for (int i = 0; i < 12; ++i) {
            delta[x * 12 + i] = 0;
            r[x * 12 + i] = rho[x * 12 + i];
        }
    }
    int steps = 0;
    for (int it = 0; it < nmr; ++it) {
        apply_DBB_coords(L, B, bcs, U, C, m0, bc, r, q);
        double complex qr = 0;
        double qq = 0;
        for (long k = 0; k < nb; ++k) {
            long x = block_site(L, B, bc, k);
            for (int i = 0; i < 12; ++i) {
                qr += conj(q[x * 12 + i]) * r[x * 12 + i];
                qq += creal(conj(q[x * 12 + i]) * q[x * 12 + i]);
            }
        }
        if (qq == 0.0) break;
        double complex alpha = qr / qq;
        for (long k = 0; k < nb; ++k) {
            long x = block_site(L, B, bc, k);
            for (int i = 0; i < 12; ++i) {
                delta[x * 12 + i] += alpha * r[x * 12 + i];
                r[x * 12 + i] -= alpha * q[x * 12 + i];
            }
        }
        ++steps;
    }
    return steps;
}

int or_mr_block(const int L[4], const int B[4], const int bcs[4], const double complex *U,
                const double complex *C, double m0, long block_id, int nmr, const double complex *rho,
                double complex *delta, double complex *r_out)
{
    if (!blocking_valid(L, B) || block_id < 0 || block_id >= num_blocks(L, B) || nmr < 0) return -1;
    long V = volume_of(L);
    double complex *r = calloc((size_t)V * 12, sizeof(double complex));
    double complex *q = calloc((size_t)V * 12, sizeof(double complex));
    if (!r || !q) {
        free(r);
        free(q);
        return -1;
    }
    int bc[4];
    block_coords(L, B, block_id, bc);
    int steps = mr_block_coords(L, B, bcs, U, C, m0, bc, nmr, rho, delta, r, q);
    if (r_out) {
        long nb = block_volume(B);
        for (long k = 0; k < nb; ++k) {
            long x = block_site(L, B, bc, k);
            for (int i = 0; i < 12; ++i) r_out[x * 12 + i] = r[x * 12 + i];
        }
    }
    free(r);
    free(q);
    return steps;
}

/* Algorithm S (multiplicative red-black SAP, Luescher 2004):
 *   psi = 0
 *   for each cycle, for colour c = 0 then 1:
 *     rho = eta - D psi on the blocks of colour c
 *     for every block B of colour c (mutually independent): psi_B += M(rho_B)
 * Blocks of one colour touch disjoint sites and read only the other colour's
 * psi, so they may be processed in any order. */
int or_sap(const int L[4], const int B[4], const int bcs[4], const double complex *U,
           const double complex *C, double m0, const double complex *eta, double complex *psi,
           int ncy, int nmr)
{
    if (!blocking_valid(L, B) || ncy < 0 || nmr < 0) return -1;
    long V = volume_of(L);
    long nblk = num_blocks(L, B);
    long nb = block_volume(B);
    double complex *rho = calloc((size_t)V * 12, sizeof(double complex));
    double complex *delta = calloc((size_t)V * 12, sizeof(double complex));
    double complex *r = calloc((size_t)V * 12, sizeof(double complex));
    double complex *q = calloc((size_t)V * 12, sizeof(double complex));
    if (!rho || !delta || !r || !q) {
        free(rho); free(delta); free(r); free(q);
        return -1;
    }
    memset(psi, 0, sizeof(double complex) * (size_t)V * 12);
    for (int cy = 0; cy < ncy; ++cy)
        for (int colour = 0; colour < 2; ++colour) {
            /* residual on the blocks of this colour */
#pragma omp parallel for schedule(dynamic, 1)
            for (long id = 0; id < nblk; ++id) {
                int bc[4];
                block_coords(L, B, id, bc);
                if (block_colour(bc) != colour) continue;
                for (long k = 0; k < nb; ++k) {
                    long x = block_site(L, B, bc, k);
                    double complex dpsi[12];
                    dirac_site(L, bcs, U, C + x * 144, m0, psi, x, NULL, dpsi);
                    for (int i = 0; i < 12; ++i) rho[x * 12 + i] = eta[x * 12 + i] - dpsi[i];
                }
            }
            /* block solves and updates */
#pragma omp parallel for schedule(dynamic, 1)
            for (long id = 0; id < nblk; ++id) {
                int bc[4];
                block_coords(L, B, id, bc);
                if (block_colour(bc) != colour) continue;
                mr_block_coords(L, B, bcs, U, C, m0, bc, nmr, rho, delta, r, q);
                for (long k = 0; k < nb; ++k) {
                    long x = block_site(L, B, bc, k);
                    for (int i = 0; i < 12; ++i) psi[x * 12 + i] += delta[x * 12 + i];
                }
            }
        }
    free(rho); free(delta); free(r); free(q);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Even-odd preconditioned block solve (SAP variant with the site-parity     */
/* Schur complement inside each block; not in the paper, a standard SAP      */
/* refinement, cf. Luescher 2004 Sec. 4 and DeGrand-Rossi even-odd           */
/* preconditioning).  Site parity p(x) = (x + y + z + t) mod 2.  On block B, */
/* with A = (4 + m0) + C (site-local) and H the in-block hops,               */
/*   D_BB = [[A_ee, H_eo], [H_oe, A_oo]],                                    */
/*   S    = A_ee - H_eo A_oo^-1 H_oe          (on the even sites of B),      */
/* the block system D_BB delta = rho is solved approximately as              */
/*   rhat_e  = rho_e - H_eo A_oo^-1 rho_o,                                   */
/*   delta_e = nmr MR steps for S delta_e = rhat_e from delta_e = 0,         */
/*   delta_o = A_oo^-1 (rho_o - H_oe delta_e).                               */
/* ------------------------------------------------------------------------ */
static int site_parity(const int L[4], long x)
{
    int c[4];
    coords_of(L, x, c);
    return (c[0] + c[1] + c[2] + c[3]) & 1;
}

/* y = ((4 + m0) + C_x)^-1 b by Gaussian elimination with partial pivoting. */
static void site_solve(const double complex *Cx, double m0, const double complex *b, double complex *y)
{
    double complex M[12][13];
    for (int i = 0; i < 12; ++i) {
        for (int j = 0; j < 12; ++j) M[i][j] = Cx[i * 12 + j] + (i == j ? 4.0 + m0 : 0.0);
        M[i][12] = b[i];
    }
    for (int k = 0; k < 12; ++k) {
        int piv = k;
        for (int i = k + 1; i < 12; ++i)
            if (cabs(M[i][k]) > cabs(M[piv][k])) piv = i;
        if (piv != k)
            for (int j = 0; j <= 12; ++j) {
                double complex t = M[k][j];
                M[k][j] = M[piv][j];
                M[piv][j] = t;
            }
        for (int i = k + 1; i < 12; ++i) {
            double complex f = M[i][k] / M[k][k];
            for (int j = k; j <= 12; ++j) M[i][j] -= f * M[k][j];
        }
    }
    for (int i = 11; i >= 0; --i) {
        double complex acc = M[i][12];
        for (int j = i + 1; j < 12; ++j) acc -= M[i][j] * y[j];
        y[i] = acc / M[i][i];
    }
}

/* out(x) = sum of the in-block hops of D applied to `in`, at site x only
 * (the same hop terms as dirac_site, without the site-local part). */
static void hop_site(const int L[4], const int bcs[4], const double complex *U, const double complex *in, long x,
                     const block_filter *filt, double complex *out /* [12] */)
{
    for (int i = 0; i < 12; ++i) out[i] = 0;
    for (int mu = 0; mu < 4; ++mu) {
        double complex chi[12], gchi[12];
        int wrapped;
        long xf = shift(L, x, mu, +1, &wrapped);
        if (in_block(filt, xf)) {
            double sign = wrapped ? (double)bcs[mu] : 1.0;
            colour_apply(link(U, x, mu), 0, in + xf * 12, chi);
            spin_apply(GAMMA[mu], chi, gchi);
            for (int i = 0; i < 12; ++i) out[i] -= 0.5 * sign * (chi[i] - gchi[i]);
        }
        long xb = shift(L, x, mu, -1, &wrapped);
        if (in_block(filt, xb)) {
            double sign = wrapped ? (double)bcs[mu] : 1.0;
            colour_apply(link(U, xb, mu), 1, in + xb * 12, chi);
            spin_apply(GAMMA[mu], chi, gchi);
            for (int i = 0; i < 12; ++i) out[i] -= 0.5 * sign * (chi[i] + gchi[i]);
        }
    }
}

/* out = H in on the block sites of parity `par` (in must vanish there). */
static void hop_parity(const int L[4], const int B[4], const int bcs[4], const double complex *U, const int bc[4],
                       int par, const double complex *in, double complex *out)
{
    block_filter f = {L, B, {bc[0], bc[1], bc[2], bc[3]}};
    long nb = block_volume(B);
    for (long k = 0; k < nb; ++k) {
        long x = block_site(L, B, bc, k);
        if (site_parity(L, x) == par) hop_site(L, bcs, U, in, x, &f, out + x * 12);
    }
}

/* Zero the block sites of parity `par` of a whole-lattice array. */
static void zero_parity(const int L[4], const int B[4], const int bc[4], int par, double complex *a)
{
    long nb = block_volume(B);
    for (long k = 0; k < nb; ++k) {
        long x = block_site(L, B, bc, k);
        if (site_parity(L, x) == par)
            for (int i = 0; i < 12; ++i) a[x * 12 + i] = 0;
    }
}

/* q_e = S r_e = A_ee r_e - H_eo A_oo^-1 H_oe r_e.  r, q, t whole-lattice
 * scratch; r must vanish on the odd block sites; q and t are overwritten on
 * the block. */
static void schur_apply(const int L[4], const int B[4], const int bcs[4], const double complex *U,
                        const double complex *C, double m0, const int bc[4], const double complex *r,
                        double complex *q, double complex *t)
{
    long nb = block_volume(B);
    zero_parity(L, B, bc, 0, t);
    hop_parity(L, B, bcs, U, bc, 1, r, t); /* t_o = H_oe r_e */
    for (long k = 0; k < nb; ++k) {        /* t_o = A_oo^-1 t_o */
        long x = block_site(L, B, bc, k);
        if (site_parity(L, x) == 1) {
            double complex y[12];
            site_solve(C + x * 144, m0, t + x * 12, y);
            for (int i = 0; i < 12; ++i) t[x * 12 + i] = y[i];
        }
    }
    zero_parity(L, B, bc, 1, q);
    hop_parity(L, B, bcs, U, bc, 0, t, q); /* q_e = H_eo t_o */
    for (long k = 0; k < nb; ++k) {        /* q_e = A_ee r_e - q_e */
        long x = block_site(L, B, bc, k);
        if (site_parity(L, x) == 0) {
            const double complex *Cx = C + x * 144;
            for (int i = 0; i < 12; ++i) {
                double complex acc = (4.0 + m0) * r[x * 12 + i];
                for (int j = 0; j < 12; ++j) acc += Cx[i * 12 + j] * r[x * 12 + j];
                q[x * 12 + i] = acc - q[x * 12 + i];
            }
        }
    }
}

static int mr_block_eo_coords(const int L[4], const int B[4], const int bcs[4], const double complex *U,
                              const double complex *C, double m0, const int bc[4], int nmr,
                              const double complex *rho, double complex *delta, double complex *r,
                              double complex *q, double complex *t)
{
    long nb = block_volume(B);
    /* t_o = A_oo^-1 rho_o ; r_e = rho_e - H_eo t_o ; delta = 0 */
    for (long k = 0; k < nb; ++k) {
        long x = block_site(L, B, bc, k);
        for (int i = 0; i < 12; ++i) {
            delta[x * 12 + i] = 0;
            t[x * 12 + i] = 0;
        }
        if (site_parity(L, x) == 1) site_solve(C + x * 144, m0, rho + x * 12, t + x * 12);
    }
    zero_parity(L, B, bc, 1, q);
    hop_parity(L, B, bcs, U, bc, 0, t, q);
    for (long k = 0; k < nb; ++k) {
        long x = block_site(L, B, bc, k);
        int even = site_parity(L, x) == 0;
        for (int i = 0; i < 12; ++i) r[x * 12 + i] = even ? rho[x * 12 + i] - q[x * 12 + i] : 0;
    }
    int steps = 0;
    for (int it = 0; it < nmr; ++it) {
        schur_apply(L, B, bcs, U, C, m0, bc, r, q, t);
        double complex qr = 0;
        double qq = 0;
        for (long k = 0; k < nb; ++k) {
            long x = block_site(L, B, bc, k);
            if (site_parity(L, x) != 0) continue;
            for (int i = 0; i < 12; ++i) {
                qr += conj(q[x * 12 + i]) * r[x * 12 + i];
                qq += creal(conj(q[x * 12 + i]) * q[x * 12 + i]);
            }
        }
        if (qq == 0.0) break;
        double complex alpha = qr / qq;
        for (long k = 0; k < nb; ++k) {
            long x = block_site(L, B, bc, k);
            if (site_parity(L, x) != 0) continue;
            for (int i = 0; i < 12; ++i) {
                delta[x * 12 + i] += alpha * r[x * 12 + i];
                r[x * 12 + i] -= alpha * q[x * 12 + i];
            }
        }
        ++steps;
    }
    /* delta_o = A_oo^-1 (rho_o - H_oe delta_e) */
    zero_parity(L, B, bc, 0, t);
    hop_parity(L, B, bcs, U, bc, 1, delta, t);
    for (long k = 0; k < nb; ++k) {
        long x = block_site(L, B, bc, k);
        if (site_parity(L, x) == 1) {
            double complex rhs[12];
            for (int i = 0; i < 12; ++i) rhs[i] = rho[x * 12 + i] - t[x * 12 + i];
            site_solve(C + x * 144, m0, rhs, delta + x * 12);
        }
    }
    return steps;
}

int or_mr_block_eo(const int L[4], const int B[4], const int bcs[4], const double complex *U,
                   const double complex *C, double m0, long block_id, int nmr, const double complex *rho,
                   double complex *delta, double complex *r_out)
{
    if (!blocking_valid(L, B) || block_id < 0 || block_id >= num_blocks(L, B) || nmr < 0) return -1;
    long V = volume_of(L);
    double complex *r = calloc((size_t)V * 12, sizeof(double complex));
    double complex *q = calloc((size_t)V * 12, sizeof(double complex));
    double complex *t = calloc((size_t)V * 12, sizeof(double complex));
    if (!r || !q || !t) {
        free(r); free(q); free(t);
        return -1;
    }
    int bc[4];
    block_coords(L, B, block_id, bc);
    int steps = mr_block_eo_coords(L, B, bcs, U, C, m0, bc, nmr, rho, delta, r, q, t);
    if (r_out) {
        long nb = block_volume(B);
        for (long k = 0; k < nb; ++k) {
            long x = block_site(L, B, bc, k);
            for (int i = 0; i < 12; ++i) r_out[x * 12 + i] = r[x * 12 + i];
        }
    }
    free(r); free(q); free(t);
    return steps;
}

/* Algorithm S with the even-odd block solve in place of Algorithm M. */
int or_sap_eo(const int L[4], const int B[4], const int bcs[4], const double complex *U,
              const double complex *C, double m0, const double complex *eta, double complex *psi,
              int ncy, int nmr)
{
    if (!blocking_valid(L, B) || ncy < 0 || nmr < 0) return -1;
    long V = volume_of(L);
    long nblk = num_blocks(L, B);
    long nb = block_volume(B);
    double complex *rho = calloc((size_t)V * 12, sizeof(double complex));
    double complex *delta = calloc((size_t)V * 12, sizeof(double complex));
    double complex *r = calloc((size_t)V * 12, sizeof(double complex));
    double complex *q = calloc((size_t)V * 12, sizeof(double complex));
    double complex *t = calloc((size_t)V * 12, sizeof(double complex));
    if (!rho || !delta || !r || !q || !t) {
        free(rho); free(delta); free(r); free(q); free(t);
        return -1;
    }
    memset(psi, 0, sizeof(double complex) * (size_t)V * 12);
    for (int cy = 0; cy < ncy; ++cy)
        for (int colour = 0; colour < 2; ++colour) {
#pragma omp parallel for schedule(dynamic, 1)
            for (long id = 0; id < nblk; ++id) {
                int bc[4];
                block_coords(L, B, id, bc);
                if (block_colour(bc) != colour) continue;
                for (long k = 0; k < nb; ++k) {
                    long x = block_site(L, B, bc, k);
                    double complex dpsi[12];
                    dirac_site(L, bcs, U, C + x * 144, m0, psi, x, NULL, dpsi);
                    for (int i = 0; i < 12; ++i) rho[x * 12 + i] = eta[x * 12 + i] - dpsi[i];
                }
            }
#pragma omp parallel for schedule(dynamic, 1)
            for (long id = 0; id < nblk; ++id) {
                int bc[4];
                block_coords(L, B, id, bc);
                if (block_colour(bc) != colour) continue;
                mr_block_eo_coords(L, B, bcs, U, C, m0, bc, nmr, rho, delta, r, q, t);
                for (long k = 0; k < nb; ++k) {
                    long x = block_site(L, B, bc, k);
                    for (int i = 0; i < 12; ++i) psi[x * 12 + i] += delta[x * 12 + i];
                }
            }
        }
    free(rho); free(delta); free(r); free(q); free(t);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Vector helpers for FGMRES (fixed summation order)                         */
/* ------------------------------------------------------------------------ */
static double complex vdot(long n, const double complex *a, const double complex *b)
{
    /* Split into fixed chunks summed in order: deterministic for any thread count. */
    const long chunk = 4096;
    long nchunks = (n + chunk - 1) / chunk;
    double complex *part = malloc(sizeof(double complex) * (size_t)(nchunks > 0 ? nchunks : 1));
#pragma omp parallel for schedule(static)
    for (long c = 0; c < nchunks; ++c) {
        double complex acc = 0;
        long hi = (c + 1) * chunk < n ? (c + 1) * chunk : n;
        for (long i = c * chunk; i < hi; ++i) acc += conj(a[i]) * b[i];
        part[c] = acc;
    }
    double complex s = 0;
    for (long c = 0; c < nchunks; ++c) s += part[c];
    free(part);
    return s;
}

static double vnorm(long n, const double complex *a) { return sqrt(creal(vdot(n, a, a))); }

/* Complex Givens rotation with LAPACK zlartg semantics:
 * [ c  s ] [f]   [r]
 * [-s* c ] [g] = [0],  c real >= 0. */
static void givens(double complex f, double complex g, double *c, double complex *s, double complex *r)
{
    double af = cabs(f), ag = cabs(g);
    if (ag == 0.0) {
        *c = 1.0; *s = 0.0; *r = f;
    } else if (af == 0.0) {
        *c = 0.0; *s = conj(g) / ag; *r = ag;
    } else {
        double nrm = hypot(af, ag);
        double complex ph = f / af;
        *c = af / nrm;
        *s = ph * conj(g) / nrm;
        *r = ph * nrm;
    }
}

/* Algorithm G (FGMRES(m), right preconditioning, MGS), Saad 1993:
 *   r = b - D x; stop when ||r||/||b|| <= tol (true residual, recomputed)
 *   beta = ||r||, v_1 = r/beta, g = beta e_1
 *   for j = 1..m: z_j = M(v_j); w = D z_j;
 *                 for i <= j: h_ij = <v_i, w>; w -= h_ij v_i
 *                 h_{j+1,j} = ||w||; rotate column j by G_1..G_{j-1};
 *                 form G_j to zero h_{j+1,j}; g = G_j g
 *                 leave when h_{j+1,j} = 0 or |g_{j+1}|/||b|| <= tol
 *                 v_{j+1} = w / h_{j+1,j}
 *   y = R^-1 g (back substitution); x += sum y_i z_i; restart. */
int or_fgmres(const int L[4], const int B[4], const int bcs[4], const double complex *U,
              const double complex *C, double m0, const double complex *b, double complex *x,
              int m, double tol, int max_restarts, int ncy, int nmr, or_precond_fn pre,
              void *pre_user, or_info *info)
{
    or_info local = {0, 0, 0, 2, NAN};
    if (!info) info = &local;
    *info = local;
    if (m < 1 || max_restarts < 0 || (!pre && ncy > 0 && !blocking_valid(L, B))) return 2;
    long V = volume_of(L);
    long n = V * 12;
    double complex *Vb = malloc(sizeof(double complex) * (size_t)n * (m + 1));
    double complex *Z = malloc(sizeof(double complex) * (size_t)n * m);
    double complex *w = malloc(sizeof(double complex) * (size_t)n);
    double complex *H = calloc((size_t)(m + 1) * m, sizeof(double complex)); /* H[i*m + j] */
    double complex *g = calloc((size_t)(m + 1), sizeof(double complex));
    double complex *sn = calloc((size_t)m, sizeof(double complex));
    double *cs = calloc((size_t)m, sizeof(double));
    double complex *y = calloc((size_t)m, sizeof(double complex));
    if (!Vb || !Z || !w || !H || !g || !sn || !cs || !y) {
        free(Vb); free(Z); free(w); free(H); free(g); free(sn); free(cs); free(y);
        return 2;
    }
    double bnorm = vnorm(n, b);
    int status = 1;
    if (bnorm == 0.0) {
        memset(x, 0, sizeof(double complex) * (size_t)n);
        info->rel_residual = 0.0;
        status = 0;
        goto done;
    }
    for (int cycle = 0; cycle <= max_restarts; ++cycle) {
        /* true residual */
        or_apply_D(L, bcs, U, C, m0, x, w);
        for (long i = 0; i < n; ++i) w[i] = b[i] - w[i];
        double beta = vnorm(n, w);
        info->rel_residual = beta / bnorm;
        if (beta / bnorm <= tol) {
            status = 0;
            break;
        }
        if (cycle == max_restarts) break;
        info->restarts++;
        for (long i = 0; i < n; ++i) Vb[i] = w[i] / beta;
        for (int i = 0; i <= m; ++i) g[i] = 0;
        g[0] = beta;
        int jdone = 0;
        for (int j = 0; j < m; ++j) {
            double complex *vj = Vb + (long)j * n;
            double complex *zj = Z + (long)j * n;
            if (pre) pre(vj, zj, pre_user);
            else if (ncy > 0) or_sap(L, B, bcs, U, C, m0, vj, zj, ncy, nmr);
            else memcpy(zj, vj, sizeof(double complex) * (size_t)n);
            info->precond_calls++;
            or_apply_D(L, bcs, U, C, m0, zj, w);
            for (int i = 0; i <= j; ++i) {
                double complex *vi = Vb + (long)i * n;
                double complex h = vdot(n, vi, w);
                H[i * m + j] = h;
                for (long k = 0; k < n; ++k) w[k] -= h * vi[k];
            }
            double hn = vnorm(n, w);
            H[(j + 1) * m + j] = hn;
            for (int i = 0; i < j; ++i) {
                double complex a = H[i * m + j], bb = H[(i + 1) * m + j];
                H[i * m + j] = cs[i] * a + sn[i] * bb;
                H[(i + 1) * m + j] = -conj(sn[i]) * a + cs[i] * bb;
            }
            double complex r;
            givens(H[j * m + j], H[(j + 1) * m + j], &cs[j], &sn[j], &r);
            H[j * m + j] = r;
            H[(j + 1) * m + j] = 0;
            g[j + 1] = -conj(sn[j]) * g[j];
            g[j] = cs[j] * g[j];
            info->iterations++;
            jdone = j + 1;
            if (hn == 0.0 || cabs(g[j + 1]) / bnorm <= tol) break;
            double complex *vn = Vb + (long)(j + 1) * n;
            for (long k = 0; k < n; ++k) vn[k] = w[k] / hn;
        }
        /* back substitution R y = g */
        for (int i = jdone - 1; i >= 0; --i) {
            double complex acc = g[i];
            for (int k = i + 1; k < jdone; ++k) acc -= H[i * m + k] * y[k];
            y[i] = acc / H[i * m + i];
        }
        for (int i = 0; i < jdone; ++i) {
            double complex *zi = Z + (long)i * n;
            for (long k = 0; k < n; ++k) x[k] += y[i] * zi[k];
        }
    }
done:
    info->status = status;
    free(Vb); free(Z); free(w); free(H); free(g); free(sn); free(cs); free(y);
    return status;
}
