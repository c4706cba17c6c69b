/*
 * Plain FP64 CPU oracle for the Wilson-clover operator, the block-local MR
 * iteration, the red-black Schwarz alternating procedure (SAP) and
 * SAP-preconditioned FGMRES.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, obviously correct
 * definition that the GPU path is checked against.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It shares
 * no code with the GPU library and includes none of its headers.
 *
 * Paper: DD-alphaAMG on QPACE 3 (Georg, Richtmann, Wettig).  The paper names
 * the method (Sec. 1: solving the discretised Dirac equation; Sec. 3.1: MR
 * inversion within a domain inside the Schwarz method, Tables 1-2) but prints
 * no formula, so every definition below follows standard published
 * mathematics, named at each function:
 *   - Wilson-clover operator: Sheikholeslami & Wohlert, Nucl. Phys. B259
 *     (1985) 572, in the mass form used by DD-alphaAMG (4 + m0 diagonal, hop
 *     factor 1/2, clover -(csw/32) sum gamma_mu gamma_nu (x) (Q_munu - Q_numu));
 *   - minimal residual: Saad, Iterative Methods for Sparse Linear Systems,
 *     2nd ed., Sec. 5.3.2;
 *   - SAP: Luescher, Comput. Phys. Commun. 156 (2004) 209;
 *   - FGMRES: Saad, SIAM J. Sci. Comput. 14 (1993) 461.
 *
 * Canonical layouts (all double complex, i.e. interleaved re/im doubles):
 *   site      s = x + Lx*(y + Ly*(z + Lz*t))
 *   gauge     U[s][mu][a][b]       mu = 0..3 for x, y, z, t
 *   spinor    psi[s][spin][colour] 12 complex per site
 *   clover    C[s][12][12]         row/col index spin*3 + colour
 * Blocks: extents B[mu] divide L[mu]; block coordinates bc[mu] = x[mu]/B[mu];
 * block id = bx + NBx*(by + NBy*(bz + NBz*bt)); colour = sum(bc) mod 2.
 * Fermion boundary signs bcs[mu] in {+1, -1} multiply every hop that wraps.
 */
#ifndef DD_ORACLE_H
#define DD_ORACLE_H

#include <complex.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void (*or_precond_fn)(const double complex *in, double complex *out, void *user);

typedef struct {
    int iterations;      /* Arnoldi steps taken in total               */
    int restarts;        /* outer cycles started                        */
    int precond_calls;   /* applications of the preconditioner          */
    int status;          /* 0 converged, 1 not converged, 2 invalid arg */
    double rel_residual; /* final ||b - D x|| / ||b||, recomputed        */
} or_info;

/* Clover term C(x) for every site, C[V][12][12]. */
void or_clover_field(const int L[4], const double complex *U, double csw, double complex *C);

/* Clover term at one site. */
void or_clover_site(const int L[4], const double complex *U, double csw, long site,
                    double complex *Cx /* [12][12] */);

/* out = D in on the whole lattice. */
void or_apply_D(const int L[4], const int bcs[4], const double complex *U,
                const double complex *C, double m0, const double complex *in,
                double complex *out);

/* (D in)(x) at the listed sites only; the clover is formed on the fly, so no
 * field-sized clover array is needed.  out[n][12]. */
void or_apply_D_sites(const int L[4], const int bcs[4], const double complex *U, double csw,
                      double m0, const double complex *in, const long *sites, long n,
                      double complex *out);

/* The same for nvec vectors in[nvec][V][12] at once (the clover term of a
 * site is formed once for all of them); out[nvec][n][12]. */
void or_apply_D_sites_nv(const int L[4], const int bcs[4], const double complex *U, double csw,
                         double m0, const double complex *in, long nvec, const long *sites, long n,
                         double complex *out);

/* out_B = D_BB in_B for block `block_id`: every hop whose neighbour lies
 * outside the block is dropped.  in/out are whole-lattice canonical arrays;
 * only the sites of the block are read and written.  Returns 0, or -1 if the
 * blocking is invalid. */
int or_apply_DBB(const int L[4], const int B[4], const int bcs[4], const double complex *U,
                 const double complex *C, double m0, long block_id,
                 const double complex *in, double complex *out);

/* Algorithm M on block `block_id`: nmr minimal-residual steps for
 * D_BB delta = rho_B from delta = 0.  rho and delta are whole-lattice arrays
 * (only block sites are touched); r_out (may be NULL) receives the final
 * block residual.  Returns the number of steps taken, -1 on invalid blocking. */
int or_mr_block(const int L[4], const int B[4], const int bcs[4], const double complex *U,
                const double complex *C, double m0, long block_id, int nmr,
                const double complex *rho, double complex *delta, double complex *r_out);

/* Algorithm S: multiplicative red-black SAP, ncy cycles, from psi = 0.
 * Returns 0, or -1 on invalid blocking. */
int or_sap(const int L[4], const int B[4], const int bcs[4], const double complex *U,
           const double complex *C, double m0, const double complex *eta, double complex *psi,
           int ncy, int nmr);

/* Even-odd preconditioned block solve on block `block_id` (site parity
 * (x+y+z+t) mod 2): nmr MR steps on the Schur complement
 * S = A_ee - H_eo A_oo^-1 H_oe for rhat_e = rho_e - H_eo A_oo^-1 rho_o, then
 * delta_o = A_oo^-1 (rho_o - H_oe delta_e); A = (4+m0) + C, H the in-block
 * hops.  r_out (may be NULL) receives the final Schur residual on the even
 * sites (zero on the odd ones).  Returns the MR steps taken, -1 on invalid
 * blocking. */
int or_mr_block_eo(const int L[4], const int B[4], const int bcs[4], const double complex *U,
                   const double complex *C, double m0, long block_id, int nmr,
                   const double complex *rho, double complex *delta, double complex *r_out);

/* Algorithm S with the even-odd block solve in place of Algorithm M. */
int or_sap_eo(const int L[4], const int B[4], const int bcs[4], const double complex *U,
              const double complex *C, double m0, const double complex *eta, double complex *psi,
              int ncy, int nmr);

/* Algorithm G: FGMRES(m) with right preconditioning.  x holds x0 on entry
 * and the solution on exit.  Preconditioner: `pre` if non-NULL, else SAP with
 * (ncy, nmr) if ncy > 0, else the identity. */
int or_fgmres(const int L[4], const int B[4], const int bcs[4], const double complex *U,
              const double complex *C, double m0, const double complex *b, double complex *x,
              int m, double tol, int max_restarts, int ncy, int nmr, or_precond_fn pre,
              void *pre_user, or_info *info);

/* Threads the OpenMP runtime will use (for reporting). */
int or_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
