/*
 * ddsap.h -- C ABI of libddsap.so, an MI355X (gfx950) implementation of the
 * Wilson-clover Dirac operator, the red-black Schwarz alternating procedure
 * (SAP) built from block-local minimal-residual (MR) solves, and
 * SAP-preconditioned flexible GMRES with an FP64 outer iteration.
 *
 * Paper: P. Georg, D. Richtmann, T. Wettig, "DD-alphaAMG on QPACE 3"
 * (Lattice 2017).  Sec. 1 states the task (solve the discretised Dirac
 * equation); Sec. 3.1 names the hot path (the MR inversion within a domain and
 * the entire Schwarz method, Tables 1 and 2), mixed precision with some data
 * structures held in half precision (Listing 1 rounds to nearest even), and
 * Sec. 5 the solver's use as an external library that transforms the data
 * layout at entry.  The operator itself follows Sheikholeslami & Wohlert (1985)
 * in the mass form used by DD-alphaAMG:
 *
 *   (D psi)(x) = (4 + m0) psi(x) + C(x) psi(x)
 *              - 1/2 sum_mu [ (1 - g_mu) U_mu(x) psi(x+mu)
 *                           + (1 + g_mu) U_mu(x-mu)^+ psi(x-mu) ]
 *   C(x) = -(csw/32) sum_{mu,nu} g_mu g_nu (x) (Q_munu(x) - Q_numu(x))
 *
 * with Q the four-leaf clover, Euclidean chiral gamma matrices
 * (g_5 = diag(1,1,-1,-1)), and the fermion boundary sign bcs[mu] on every hop
 * that wraps around the lattice.  SAP follows Luescher, Comput. Phys. Commun.
 * 156 (2004) 209; MR follows Saad's textbook (Sec. 5.3.2); FGMRES follows
 * Saad, SIAM J. Sci. Comput. 14 (1993) 461.
 *
 * ---------------------------------------------------------------------------
 * Conventions shared by every call
 * ---------------------------------------------------------------------------
 * Canonical (caller) layouts, complex numbers as interleaved (re, im) doubles:
 *   site    s = x + Lx*(y + Ly*(z + Lz*t))
 *   gauge   U[s][mu][a][b]            mu = x, y, z, t          (18 doubles/site/mu)
 *   spinor  psi[rhs][s][spin][colour]                          (24 doubles/site)
 *   clover  C[s][k][i][j]  k = chiral half (spins 0-1, spins 2-3),
 *                          i, j = (spin - 2k)*3 + colour       (144 doubles/site)
 * Blocked (device) layout: the library's own, reached through
 * dd_pack_spinor / dd_unpack_spinor; dd_spinor_bytes gives its size.  The
 * Schwarz blocks are 4x4x4x4 sites; the number of blocks per direction must be
 * even or one (red-black colouring).  Block id (canonical) =
 * bx + NBx*(by + NBy*(bz + NBz*bt)); its colour is (bx+by+bz+bt) mod 2.
 *
 * Precision (dd_prec): FP64, FP32, or FP16 storage with FP32 arithmetic.
 * Conversions to lower precision round to nearest even.
 *
 * Ownership: the caller owns every pointer it passes.  Device pointers are
 * HIP device allocations on the context's device (e.g. torch tensors'
 * data_ptr()).  The context copies the gauge/clover fields it is given and
 * owns all workspaces.  Calls enqueue on the context's stream and return
 * without waiting unless stated; device faults surface at the next
 * synchronising call.  One context serves one host thread at a time.
 *
 * Errors: every call returns a dd_status.  The library never aborts and
 * never throws across this boundary; dd_last_error gives the message of the
 * last failure on a context (or of the last failed dd_create when passed
 * NULL).  It prints nothing unless the environment variable DDSAP_LOG is 1
 * or more when the library first checks it: then every failed call and
 * every dd_solve (per right-hand side: status, iterations, restarts,
 * smoother calls, residual; and the call's wall time) write one line each
 * to stderr.
 */
#ifndef DDSAP_H
#define DDSAP_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DD_ABI_VERSION 6
#define DD_MAX_RHS 16 /* right-hand sides fused into one launch */

typedef enum {
    DD_OK = 0,
    DD_INVALID_ARG = 1,   /* bad size, pointer, blocking, precision or parameter */
    DD_OOM = 2,           /* a device allocation failed                           */
    DD_HIP_ERROR = 3,     /* a HIP runtime call failed                            */
    DD_NOT_CONVERGED = 4, /* max restarts reached; x holds the best iterate       */
    DD_BREAKDOWN = 5,     /* the Krylov space closed on a singular projection of D
                             without convergence (e.g. b in the null space of a
                             singular D); x holds the last iterate               */
    DD_NAN = 6,           /* NaN or Inf found in an input or a residual           */
    DD_NO_FIELD = 7       /* the call needs a gauge field that was never set      */
} dd_status;

typedef enum { DD_F64 = 0, DD_F32 = 1, DD_F16 = 2 } dd_prec;

typedef struct dd_ctx dd_ctx;

/* Parameters of dd_solve (FGMRES(m) preconditioned by ncy SAP cycles of nmr
 * MR steps per block, in precision sap_prec; the outer iteration is FP64). */
typedef struct {
    int m;            /* Krylov dimension per restart cycle, 1..32 (20)         */
    double tol;       /* stop when ||b - D x||_2 / ||b||_2 <= tol (1e-10)       */
    int max_restarts; /* restart cycles before DD_NOT_CONVERGED (100)            */
    int ncy;          /* SAP cycles per preconditioner call; 0 = no precond (12)*/
    int nmr;          /* MR steps per block and sweep (4)                        */
    int sap_prec;     /* dd_prec of the smoother (DD_F32)                        */
    int sap_eo;       /* 1: even-odd preconditioned block solves (dd_sap_eo), 0 */
    int amg;          /* 1: precondition with the two-grid method of dd_amg_setup
                         (coarse correction + SAP post-smoothing in sap_prec,
                         DD_F32 or DD_F64; ncy/nmr/sap_eo are then unused), 0  */
} dd_params;

/* Per right-hand-side result of dd_solve. */
typedef struct {
    int status;          /* dd_status of this right-hand side                   */
    int iterations;      /* Arnoldi steps taken                                 */
    int restarts;        /* restart cycles started                              */
    int sap_calls;       /* preconditioner applications                         */
    double rel_residual; /* final true residual ||b - D x|| / ||b|| (FP64, GPU) */
} dd_solve_info;

/* ABI version of the loaded library (DD_ABI_VERSION). */
int dd_abi_version(void);

/* Fill *p with the defaults shown above. */
void dd_default_params(dd_params *p);

/* Create a context for a Lx x Ly x Lz x Lt lattice on the current HIP device.
 *   dims   lattice extents; each a multiple of the block extent;
 *   block  Schwarz block extents (Sec. 3.1: the MR inversion runs within
 *          these domains); NULL or {4,4,4,4} -- the only blocking the kernels
 *          implement (one 256-thread workgroup per 4^4 block, one site per
 *          thread); any other value is DD_INVALID_ARG;
 *   bcs    fermion boundary sign per direction, +1 or -1 (e.g. {1,1,1,-1});
 *   stream hipStream_t to enqueue on (NULL = the null stream);
 *   out    receives the context.
 * DD_INVALID_ARG if an extent is not a positive multiple of 4, a direction
 * has an odd number (>1) of blocks, or block is not 4^4; DD_OOM /
 * DD_HIP_ERROR on device failure. */
dd_status dd_create(const int dims[4], const int block[4], const int bcs[4], void *stream, dd_ctx **out);

/* Release the context and every device buffer it owns (synchronises). */
dd_status dd_destroy(dd_ctx *ctx);

/* Message of the last failure on ctx (or of the last dd_create if NULL). */
const char *dd_last_error(const dd_ctx *ctx);

/* Wait for all work enqueued on the context's stream. */
dd_status dd_synchronize(dd_ctx *ctx);

/* Setup (not timed): copy the canonical FP64 gauge field U (host pointer,
 * 72*V doubles), build the clover term with coefficient csw on the device in
 * FP64, and store links and clover in the blocked layout in FP64, FP32 and
 * FP16.  Synchronises.  DD_NAN if U holds NaN/Inf.  When every link is in
 * SU(3) to within 1e-13 (max |U U^+ - 1| and |det U - 1|), gauge compression
 * is switched on (see dd_set_link_compression). */
dd_status dd_set_gauge(dd_ctx *ctx, const double *U_host, double csw);

/* Gauge compression ("reconstruct-12"): the operator and smoother kernels
 * read the first two rows of each link and rebuild the third as the complex
 * conjugate of their cross product, which holds for SU(3) matrices; this cuts
 * the link bytes per site from 72 to 48 reals.  enable = 0 switches it off
 * (all nine entries are read); enable = 1 switches it on, DD_INVALID_ARG if
 * the current field is not SU(3) (or none is set).  Applies to calls made
 * afterwards; servers and solves capture it when their engines are built. */
dd_status dd_set_link_compression(dd_ctx *ctx, int enable);

/* 1 if gauge compression is on, 0 if off, -1 for a NULL context. */
int dd_link_compression(const dd_ctx *ctx);

/* Half-precision fields under the FP32 smoother (Sec. 3.1 keeps part of its
 * data in 16-bit floating point as a further mixed-precision step).  With
 * enable = 1 the plain FP32 Schwarz sweep -- dd_sap with DD_F32, and dd_solve
 * or a server with an FP32 smoother and sap_eo = 0 -- reads the FP16 copies of
 * the links and the clover term that dd_set_gauge / dd_set_clover store;
 * spinors, the MR arithmetic and the FP64 outer iteration keep their
 * precisions.  The block solves then use D_BB with FP16-rounded entries
 * (relative rounding 2^-11), which the flexible outer iteration absorbs; the
 * solve still stops on the FP64 true residual.  enable = 0 (the default)
 * reads FP32 fields.  Other smoother precisions and the even-odd sweep are
 * unaffected.  Applies to calls made afterwards.  DD_INVALID_ARG for a NULL
 * context. */
dd_status dd_set_sap_half_fields(dd_ctx *ctx, int enable);

/* 1 if the FP32 smoother reads FP16 fields, 0 if not, -1 for a NULL context. */
int dd_sap_half_fields(const dd_ctx *ctx);

/* Replace the clover term by an explicit one (host pointer, canonical clover
 * layout, 144*V doubles; each 6x6 half must be Hermitian, only its upper
 * triangle and real diagonal are read).  Requires dd_set_gauge first. */
dd_status dd_set_clover(dd_ctx *ctx, const double *C_host);

/* Bytes of one blocked spinor buffer holding nrhs right-hand sides. */
size_t dd_spinor_bytes(const dd_ctx *ctx, int prec, int nrhs);

/* Layout transform: canonical FP64 spinors (device pointer, nrhs*24*V
 * doubles) -> blocked buffer of precision prec (device pointer), and back.
 * Down-conversion rounds to nearest even; no scaling is applied. */
dd_status dd_pack_spinor(dd_ctx *ctx, const double *canon, void *blocked, int prec, int nrhs);
dd_status dd_unpack_spinor(dd_ctx *ctx, const void *blocked, double *canon, int prec, int nrhs);

/* y = D x for nrhs right-hand sides, right-hand side r with mass m0[r]
 * (host array of nrhs doubles).  x, y: blocked device buffers of precision
 * prec; they must not overlap. */
dd_status dd_apply_D(dd_ctx *ctx, const double *m0, const void *x, void *y, int prec, int nrhs);

/* y_B = D_BB x_B on one Schwarz block (canonical block id): D restricted to
 * the block, every hop that leaves the block dropped.  x, y: whole-lattice
 * blocked buffers (one right-hand side); only block block_id of x is read
 * and only block block_id of y is written. */
dd_status dd_apply_D_block(dd_ctx *ctx, double m0, long block_id, const void *x, void *y, int prec);

/* psi = SAP(eta): ncy cycles of red-black block sweeps from psi = 0; each
 * sweep forms the block residual eta_B - (D psi)_B and adds nmr MR steps on
 * D_BB to psi_B (colour 0 first).  eta, psi: blocked device buffers of
 * precision prec (nrhs right-hand sides, masses m0[r]); psi is overwritten. */
dd_status dd_sap(dd_ctx *ctx, const double *m0, const void *eta, void *psi, int ncy, int nmr,
                 int prec, int nrhs);

/* dd_sap with the even-odd preconditioned block solve in place of plain MR
 * (a standard refinement of the smoother; the paper's SAP is the plain form).
 * With site parity (x+y+z+t) mod 2, A = (4+m0) + C site-local and H the
 * in-block hops, each block solves D_BB delta = rho as
 *   rhat_e = rho_e - H_eo A_oo^-1 rho_o,
 *   nmr MR steps on S = A_ee - H_eo A_oo^-1 H_oe for S delta_e = rhat_e,
 *   delta_o = A_oo^-1 (rho_o - H_oe delta_e).
 * A_oo^-1 is applied through a Cholesky factor of each chiral half, formed on
 * the device per mass; this needs (4+m0) + C positive definite on every
 * chiral half (true whenever 4+m0 exceeds the clover term's norm, as for all
 * physical masses), otherwise psi holds NaN.  Arguments, layout and errors as
 * dd_sap. */
dd_status dd_sap_eo(dd_ctx *ctx, const double *m0, const void *eta, void *psi, int ncy, int nmr,
                    int prec, int nrhs);

/* dd_sap for callers that cannot allocate device memory -- code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  It
 * computes exactly what dd_sap computes (same kernels, same arguments,
 * layout and errors) but allocates nothing: the smoother's scratch (the face
 * buffers that pass boundary half spinors between the colours and the block
 * residual carried between visits, 2 * dd_spinor_bytes(ctx, prec, nrhs)
 * bytes) lives in a fixed device array of DD_SAP_NOALLOC_SCRATCH_BYTES that
 * the library holds on every GPU it runs on until the process ends, and
 * ncy = 0 clears psi with a kernel.  The caller still passes eta and psi.
 * DD_INVALID_ARG (with a message) if the scratch would exceed the array
 * (e.g. FP32, one right-hand side: up to 663,552 sites = 24^3 x 48).  All
 * calls on one GPU share that GPU's array, whose contents persist between
 * calls (nothing in it needs to start at zero): calls that overlap on one
 * GPU -- from different streams or host threads -- race, so the caller must
 * order them.  No profiler events are recorded for it. */
#define DD_SAP_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
dd_status dd_sap_noalloc(dd_ctx *ctx, const double *m0, const void *eta, void *psi, int ncy, int nmr, int prec,
                         int nrhs);

/* Solve D x_r = b_r (r < nrhs) with FGMRES(m) preconditioned by SAP in
 * params->sap_prec, the Arnoldi basis, orthogonalisation, true residuals and
 * reductions in FP64 on the device.  b, x: canonical FP64 spinors (device
 * pointers, nrhs*24*V doubles); x holds the initial guess on entry (zero it
 * for x0 = 0) and the solution on exit.  m0: host array of nrhs masses.
 * info (host, may be NULL): nrhs entries.  Synchronises.  Returns DD_OK if
 * every right-hand side converged, else the first failing status. */
dd_status dd_solve(dd_ctx *ctx, const double *m0, const double *b, double *x, int nrhs,
                   const dd_params *params, dd_solve_info *info);

/* ---------------------------------------------------------------------------
 * Two-level coarse correction (the multigrid level of DD-alpha-AMG)
 * ---------------------------------------------------------------------------
 * The paper's solver is DD-alpha-AMG (Sec. 1): a multigrid method whose
 * fine-grid smoother is the Schwarz method above (Sec. 2.1) and which has a
 * coarse grid (Sec. 5).  The two-level form here follows the published
 * method (Frommer, Kahl, Krieg, Leder, Rottmann, SIAM J. Sci. Comput. 36
 * (2014) A1581):
 *   aggregates    the 4^4 Schwarz blocks, each split into its chiral halves
 *                 (spins 0-1 and spins 2-3), so P commutes with gamma_5;
 *   test vectors  from the caller's starting vectors by inverse iteration
 *                 with SAP (v <- SAP(v)/|SAP(v)|, setup_iters times), then
 *                 `adapt` rounds with the two-grid method in SAP's place;
 *   P             the test vectors restricted to each aggregate and
 *                 orthonormalised there by Gram-Schmidt in their order;
 *   D_c           P^+ D P: 2 nvec unknowns per block, a nearest-neighbour
 *                 operator on the lattice of blocks, built at m0 = 0 (the
 *                 mass enters as + m0 since P^+ P = 1, so one setup serves
 *                 every mass; the test vectors are tuned to the setup mass);
 *   coarse solve  coarse_k steps of GMRES from zero (the least-residual
 *                 vector of the Krylov space), on the device, FP64 vectors
 *                 and an FP16 copy of D_c;
 *   two-grid B    psi_0 = P x_c with x_c the coarse solve of
 *                 D_c x_c = P^+ eta, then psi = psi_0 + SAP(eta - D psi_0)
 *                 with post_ncy cycles of post_nmr MR steps.
 * Layouts: P (dd_amg_interpolation) [block][c][i][component][site], complex,
 * component = (spin - 2c) * 3 + colour, site = the block-local index
 * x + 4y + 16z + 64t; D_c (dd_amg_coarse_operator) [block][d][k'][k],
 * complex, d = 0 the block, 1 + 2 mu its +mu neighbour, 2 + 2 mu its -mu
 * neighbour, entry (row k, column k') with k = c * nvec + i; coarse vectors
 * [rhs][block][k] complex FP64 (device).  A context holds one setup; a new
 * dd_amg_setup replaces it. */
typedef struct {
    int nvec;        /* test vectors, 1..16 (12): 2 nvec coarse unknowns per block */
    int setup_iters; /* inverse-iteration steps per test vector (6)               */
    int setup_ncy;   /* SAP cycles per setup step (4)                               */
    int setup_nmr;   /* MR steps per block in them (4)                              */
    int setup_prec;  /* precision of the setup's smoother, DD_F32 or DD_F64 (F32)   */
    int adapt;       /* adaptive rounds with the two-grid method (2)                */
    int coarse_k;    /* GMRES steps of the coarse solve, 1..32 (16)                 */
    int post_ncy;    /* SAP cycles after the coarse correction, >= 0 (8)            */
    int post_nmr;    /* MR steps per block in them (4)                              */
} dd_amg_params;

/* Fill *p with the defaults shown above. */
void dd_amg_default_params(dd_amg_params *p);

/* Set up the coarse level on ctx's gauge field.  v0: nvec starting vectors,
 * canonical FP64 (device, nvec * 24 * V doubles), e.g. Gaussian; m0: the
 * mass the test vectors are tuned to.  Synchronises.  DD_NO_FIELD,
 * DD_INVALID_ARG (parameters out of range), DD_NAN (non-finite v0), DD_OOM. */
dd_status dd_amg_setup(dd_ctx *ctx, double m0, const double *v0, const dd_amg_params *p);

/* Complex entries of one coarse vector (nblocks * 2 nvec), 0 without a setup. */
size_t dd_amg_coarse_size(const dd_ctx *ctx);

/* Copy the FP64 interpolation / coarse operator to host memory in the
 * layouts above (P: nblocks*2*nvec*6*256 complex; D_c: nblocks*9*(2 nvec)^2
 * complex).  Synchronises.  DD_INVALID_ARG without a setup. */
dd_status dd_amg_interpolation(dd_ctx *ctx, double *P_host);
dd_status dd_amg_coarse_operator(dd_ctx *ctx, double *Dc_host);

/* xc = P^+ x (restriction) and x = P xc (prolongation) for nrhs right-hand
 * sides: x a blocked spinor buffer of precision prec (DD_F64: FP64
 * interpolation and arithmetic; DD_F32: the FP32 copy and FP32 arithmetic),
 * xc coarse vectors (device, FP64). */
dd_status dd_amg_restrict(dd_ctx *ctx, const void *x, double *xc, int prec, int nrhs);
dd_status dd_amg_prolong(dd_ctx *ctx, const double *xc, void *x, int prec, int nrhs);

/* yc = (D_c + m0[r]) xc for each right-hand side r (m0: host, nrhs values),
 * with the FP16 copy of D_c that the coarse solve uses. */
dd_status dd_amg_coarse_apply(dd_ctx *ctx, const double *m0, const double *xc, double *yc, int nrhs);

/* xc = k steps of GMRES from zero on (D_c + m0[r]) xc = bc (1 <= k <= 32;
 * the Krylov space may close earlier, then xc solves exactly). */
dd_status dd_amg_coarse_solve(dd_ctx *ctx, const double *m0, const double *bc, double *xc, int k, int nrhs);

/* psi = B eta, the two-grid preconditioner, for nrhs right-hand sides of
 * precision prec (DD_F64 or DD_F32 blocked buffers; eta and psi must not
 * overlap). */
dd_status dd_amg_precondition(dd_ctx *ctx, const double *m0, const void *eta, void *psi, int prec, int nrhs);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of solves over resident gauge fields
 * ---------------------------------------------------------------------------
 * A server keeps several gauge fields resident (each with its own HIP stream,
 * its own worker thread and a pool of right-hand-side slots sized from the
 * HBM budget).  Requests are queued first in, first out; a field's worker
 * admits the right-hand sides of that field's requests into free slots as
 * earlier ones finish and fuses all slots of the field into multi-RHS
 * launches (the Arnoldi step is replayed as a captured hipGraph).  Fields
 * advance independently -- a small lattice is not held to the step rate of a
 * large one -- and overlap on the device through their streams.  Each slot
 * runs its own FGMRES(m) to params tol, so a result does not depend on which
 * other requests share the launches beyond rounding. */
typedef struct dd_server dd_server;

typedef struct {
    size_t hbm_budget_bytes; /* solver workspace of all fields together (200 GiB)   */
    int max_width;           /* slots per field, 1..16 (12)                          */
    int m;                   /* FGMRES(m), 1..32 (20)                                 */
    double tol;              /* per right-hand side (1e-10)                          */
    int max_restarts;        /* (100)                                                 */
    int ncy, nmr;            /* SAP cycles and MR steps (12, 4)                       */
    int sap_prec;            /* smoother precision (DD_F32)                           */
    int use_graphs;          /* replay captured hipGraphs for the Arnoldi step (1)    */
    int sap_eo;              /* even-odd preconditioned block solves (0)              */
    int sap_half_fields;     /* FP32 smoother reads FP16 links and clover (0); see
                                dd_set_sap_half_fields                                */
} dd_server_config;

typedef struct {
    long requests_done;
    long rhs_done;
    long iterations;        /* Arnoldi steps over all finished right-hand sides    */
    double p50_ms, p99_ms;  /* request latency, submit to completion               */
    double mean_ms;
    double wall_s;          /* first submit to last completion                     */
    double rhs_per_s;       /* rhs_done / wall_s                                   */
    double busy_s;          /* worker time with work on the device, summed over the
                               fields' workers (can exceed wall_s)                */
    size_t workspace_bytes; /* reserved slot workspace of all fields                */
} dd_server_stats;

void dd_server_default_config(dd_server_config *cfg);

/* Create a server on the current HIP device (cfg may be NULL for defaults). */
dd_status dd_server_create(const dd_server_config *cfg, dd_server **out);

/* Make a gauge field resident (host U as in dd_set_gauge).  width = slots for
 * this field (0 = max_width), reduced to what the remaining HBM budget allows;
 * DD_OOM if not even one slot fits.  Fields must be added before the first
 * submit.  *field_id receives the field's index. */
dd_status dd_server_add_field(dd_server *s, const int dims[4], const int bcs[4], const double *U_host, double csw,
                              int width, int *field_id);

/* Slot count and reserved workspace bytes of a field. */
dd_status dd_server_field_info(const dd_server *s, int field_id, int *width, size_t *workspace_bytes);

/* Queue a request: nrhs right-hand sides b (canonical FP64, device, nrhs*24*V
 * doubles) on field_id with masses m0 (host, nrhs values); solutions go to x
 * (canonical FP64 device buffer of the same size).  b and x belong to the
 * caller and must stay valid until the request completes; the server's
 * streams are not ordered after the caller's, so all writes to b and x must
 * have finished before the call.  Returns at once. */
dd_status dd_server_submit(dd_server *s, int field_id, int nrhs, const double *m0, const double *b, double *x,
                           long *request_id);

/* *done = 1 when the request has finished; then info (host, nrhs entries,
 * may be NULL) and latency_ms (may be NULL) are filled, the request's status
 * is returned and the server forgets the request (its id is then unknown:
 * DD_INVALID_ARG).  *done = 0 and DD_OK while it runs. */
dd_status dd_server_poll(dd_server *s, long request_id, int *done, dd_solve_info *info, double *latency_ms);

/* Block until the request finishes; as dd_server_poll otherwise (the request
 * is forgotten on return).  Safe while other threads submit. */
dd_status dd_server_wait(dd_server *s, long request_id, dd_solve_info *info, double *latency_ms);

/* Latency percentiles and throughput of the requests finished so far. */
dd_status dd_server_get_stats(dd_server *s, dd_server_stats *out);

/* Message of the server's last failure. */
const char *dd_server_last_error(const dd_server *s);

/* Stop the worker (pending requests are abandoned) and free everything. */
dd_status dd_server_destroy(dd_server *s);

/* ---------------------------------------------------------------------------
 * Test hook
 * ---------------------------------------------------------------------------
 * FP16 range (Sec. 3.1 stores part of the data in half precision): dd_solve
 * scales each right-hand side into FP16's range before the smoother, and if
 * a smoother output still turns non-finite the outer iteration drops that
 * step's column, restarts from the last FP64 iterate and runs the FP16
 * smoother in FP32 from then on.  This hook exercises that path from the
 * host: the next `count` FP16 smoother applications of dd_solve on ctx (all
 * of them for count < 0; none for 0, the default) get an FP16 infinity in
 * the first entry of each active right-hand side's output.  A solve under
 * the hook still converges, in FP32, if the fallback works; it never
 * affects FP32/FP64 smoothers.  DD_INVALID_ARG for a NULL context. */
dd_status dd_debug_poison_half_smoother(dd_ctx *ctx, int count);

/* ---------------------------------------------------------------------------
 * Measurement (optional; used to price kernels against the hardware roofline)
 * ---------------------------------------------------------------------------
 * Per kernel class: launches, summed duration of the launches measured with
 * HIP events recorded on the context's stream, and the algorithmic bytes and
 * flops those launches represent (the method's data volume -- links, clover
 * and spinors each counted once per launch -- not the bytes the hardware
 * moved).  Counting conventions: one operator application is 1848 flops per
 * site and right-hand side; one MR step is 2184 flops per site. */
typedef struct {
    char name[32];
    long launches;
    double total_ms;
    double bytes;
    double flops;
} dd_kernel_stat;

/* Copy bytes (a multiple of 16, nonzero) from src to dst (device pointers,
 * not overlapping) on stream with a plain streaming kernel: one workgroup
 * per 16 KiB tile, each thread issuing four 16-byte non-temporal loads
 * before its four stores (a partial last tile element by element).  The
 * HBM bandwidth it reaches (2 * bytes / time) is the reference line the
 * operator and smoother rates are compared with.  DD_INVALID_ARG for null
 * pointers or bad sizes. */
dd_status dd_stream_copy(const void *src, void *dst, size_t bytes, void *stream);

/* Switch event timing on (1) or off (0); switching on clears the counters. */
dd_status dd_profile_enable(dd_ctx *ctx, int enable);

/* Synchronise the context's stream, fold in every finished measurement and
 * copy up to max classes with at least one launch into out (host array).
 * Returns the number of entries written, or -1 on error. */
int dd_profile_read(dd_ctx *ctx, dd_kernel_stat *out, int max);

#ifdef __cplusplus
}
#endif
#endif
