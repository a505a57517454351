/*
 * cmmlfma.h -- C ABI of the MI355X (gfx950) MLFMA library for characteristic-mode
 * analysis of PEC surfaces (Dai, Wu, Meng, Chew, Sha, "Multilevel Fast Multipole
 * Algorithm for Characteristic Mode Analysis").
 *
 * The library builds, from a triangle mesh and a wavenumber k, the RWG
 * discretisation (eq. (4)), an octree with near and far interaction lists
 * (section III-C), and applies to one or more complex vectors
 *   Z = R + iX  (eqs. (5), (7), (11)),   R  (eqs. (19)-(22)),   X (eqs. (15)-(18)),
 *   Z^H,  and dZ/dk,
 * plus the sparse approximate inverse (SAI) preconditioner of the near-field
 * matrix (section IV).  These are the products an implicitly restarted Arnoldi
 * solve of  Z^-1 R J = J / (1 + i lambda)  (eq. (24)) needs at every step; the
 * library also runs that solve (cm_eigs, with GMRES inner solves, cm_gmres),
 * the Arnoldi solve of  X^-1 R J = J / lambda  (eq. (14), cm_eigs_xinv) and a
 * Jacobi-Davidson solve of the pencil  X J = lambda R J  (eqs. (28)-(29),
 * cm_jd).
 *
 * Conventions (all entry points):
 *  - Sign convention.  The public matrix is
 *        Z_mn = ik eta <f_m, [I - grad grad'/k^2] exp(-ikR)/R, f_n>,
 *    i.e. -conj of eq. (5) written with eq. (3), so that R = Re Z is positive
 *    semidefinite and X J = lambda R J has the characteristic values of Table II.
 *  - Unknown order.  RWG n is the n-th interior edge in increasing
 *    (smaller vertex, larger vertex) order; T+ is the lower-numbered triangle
 *    (cm_rwg_table).  f = l/(2A+) (r - p+) on T+, l/(2A-) (p- - r) on T-.
 *  - Vectors.  x and y are DEVICE pointers to interleaved complex numbers,
 *    row-major N x ncols with row stride ld >= ncols (elements): entry (i, c)
 *    at x[i*ld + c].  CM_C64 = complex float (far field in FP32, near field
 *    stored and applied in FP64), CM_C128 = complex double (all FP64).
 *    The caller owns x and y; they must not alias.  y is overwritten.
 *  - Streams.  cm_apply / cm_sai_apply enqueue work on the given HIP stream
 *    (NULL = default stream) and return without synchronising.  Inside an
 *    apply the library forks work to streams of its own (created with the
 *    handle, default priority) and joins them back to the given stream with
 *    events before the call's last kernel, so the given stream alone orders
 *    the call against the caller's other work.  cm_create and cm_sai_build
 *    block until their device work is done.
 *  - Errors.  Every call returns a cm_status; no exception crosses the ABI.
 *    cm_last_error() returns a thread-local message for the last failure.
 *  - Threads.  One handle must not be used by two host threads at once, and
 *    applies that overlap on different streams with the same handle race on
 *    its workspace.
 */
#ifndef CMMLFMA_H
#define CMMLFMA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cm_handle cm_handle;          /* opaque, library-owned */

typedef enum {
  CM_OK = 0,
  CM_E_BADARG = -1,       /* null pointer, size out of range, bad enum          */
  CM_E_MESH = -2,         /* non-manifold edge, zero-area triangle, NaN vertex,
                             or mesh too coarse for the leaf boxes               */
  CM_E_OOM = -3,          /* host or device allocation failed / size overflow   */
  CM_E_HIP = -4,          /* a HIP runtime call failed                          */
  CM_E_NOT_BUILT = -5,    /* handle has no device data (host-only plan) or the
                             SAI has not been built                             */
  CM_E_NUMERIC = -6,      /* non-finite translator or table entry               */
  CM_E_UNSUPPORTED = -7,  /* option combination not implemented                 */
  CM_E_NOT_CONVERGED = -8 /* iterative solver stopped before its tolerance; the
                             outputs hold the last iterate                      */
} cm_status;

typedef enum {
  CM_OP_Z = 0,      /* y = Z x                                                 */
  CM_OP_R = 1,      /* y = R x   (sin kernel, eq. (22); near field = own leaf
                                  box only.  Translations: between children
                                  of the same parent at levels 3..leaf and
                                  between all distinct level-2 boxes, unless
                                  CM_FLAG_R_STANDARD)                        */
  CM_OP_X = 2,      /* y = X x   (cos kernel, eq. (18))                        */
  CM_OP_ZH = 3,     /* y = Z^H x = conj(Z conj(x))  (Z = Z^T)                  */
  CM_OP_DZDK = 4    /* y = (dZ/dk) x, tree and sampling frozen (needs
                       CM_FLAG_DERIV at create)                                */
} cm_op;

typedef enum { CM_C64 = 0, CM_C128 = 1 } cm_dtype;

/* option flags */
#define CM_FLAG_HOST_ONLY 1u   /* build the host plan only (no device work);
                                  cm_apply returns CM_E_NOT_BUILT            */
#define CM_FLAG_DERIV     2u   /* also build dZ_near/dk and derivative tables */
#define CM_FLAG_CHECK     4u   /* brute-force check that every leaf-box pair is
                                  covered exactly once (O(boxes^2))          */
#define CM_FLAG_NO_MATRIX_CORES 8u /* applies use the vector-ALU kernels
                                  only: no MFMA for the near field, the leaf
                                  aggregation/disaggregation and the
                                  interpolation                              */
#define CM_FLAG_NEAR_FP32 16u  /* FP32 applies take the near-field product in
                                  FP32 (an FP32 copy of the FP64-filled
                                  values, FP32 accumulation) instead of
                                  complex128 values with FP64 accumulation:
                                  faster, about 1e-6 relative on the near
                                  part; costs 8 B per near-field entry       */
#define CM_FLAG_WIDE_NEAR 32u  /* two-box buffer at the two finest levels: the
                                  near field takes leaf boxes up to Chebyshev
                                  distance 2, and the translation lists of the
                                  leaf level and the level above start at
                                  distance 3.  RWG supports reach past their
                                  leaf box, so at distance 2 the addition
                                  theorem of eq. (9) is at or past its
                                  convergence limit there and the truncated
                                  translator grows fast with L; this flag
                                  removes both (about 10x smaller error at the
                                  same d0, p) for about 2.8x the near-field
                                  entries and more leaf translations.  The
                                  SAI candidate pattern is the stored near
                                  field, so it widens with it.              */
#define CM_FLAG_AUTOTUNE  64u  /* at create, time every valid slot-chunk width
                                  and load row-group of the matrix-core
                                  interpolation and anterpolation kernels of
                                  each level at the batch width (largest
                                  multiple of 8 up to max_cols, at most 64)
                                  and keep the fastest, and likewise the
                                  translation kernel of each level (16-box
                                  tiles or 64-box tiles whose waves share
                                  their sources through LDS; these give the
                                  same bits) (reported by cm_stats under
                                  "autotune").  Changes only
                                  the summation grouping: results differ
                                  from an untuned handle by FP32 rounding,
                                  and the choice may differ between handles */
#define CM_FLAG_R_STANDARD 128u /* R x with the standard MLFMA lists (the far
                                  lists of Z at every level plus the
                                  neighbouring leaf boxes) instead of the
                                  sibling bookkeeping that the paper
                                  recommends for R after eq. (22); same
                                  operator, several times more leaf
                                  translations                               */

#define CM_FLAG_M2L_TILE16 512u /* keep the autotuner (CM_FLAG_AUTOTUNE) from
                                  trying the 64-box shared-source translation
                                  kernels: FP32 batched translations always
                                  use receiver tiles of 16 boxes (the
                                  default without the autotuner; the kernels
                                  give the same bits)                        */
#define CM_FLAG_M2L_SINGLE_TILES 1024u /* single-column translations use the
                                  receiver tiles of 16 boxes instead of the
                                  receiver-major kernel (one wave per
                                  receiver and 64 directions); the two give
                                  the same bits                              */
#define CM_FLAG_SWEEP_SHARED 2048u /* wavenumber sweeps (n_k > 1): every
                                  wavenumber's plan takes its truncation and
                                  angular sampling at the largest wavenumber
                                  (or k_sampling when set), and FP32 applies
                                  of Z and Z^H whose columns span several
                                  wavenumbers run as one pass: the columns
                                  in slots of four per wavenumber, the near
                                  field, aggregation and disaggregation per
                                  slot with that wavenumber's tables, and the
                                  interpolation, translations and
                                  anterpolation once over all columns with
                                  per-slot translators and shift phases (at
                                  most 16 slots; other ops, FP64 or wider
                                  batches take the per-wavenumber route) */
#define CM_FLAG_VERBOSE   256u /* the eigen-solvers print one progress line to
                                  stderr per Arnoldi restart (cm_eigs,
                                  cm_eigs_xinv) or converged pair (cm_jd) */

typedef struct {
  int32_t nlv;       /* number of octree levels including level 0 (>= 3)        */
  double d0;         /* digits of accuracy in the truncation rule, eq. (30)     */
  int32_t interp_p;  /* local Lagrange interpolation points per direction (even,
                        2..12)                                                  */
  double eta;        /* wave impedance; <= 0 selects 376.730313668 ohm          */
  uint32_t flags;    /* CM_FLAG_*                                               */
  int32_t max_cols;  /* largest ncols any apply will use (1..64)                */
  double k_sampling; /* wavenumber at which eq. (30) sets L and hence the
                        angular sampling of every level; <= 0: each
                        handle's (or sweep point's) own k.  A common value
                        freezes L, the directions and the interpolation
                        tables across handles at nearby wavenumbers, so
                        that they differ only in the k-dependent values
                        (translators, phases, patterns, near field): the
                        discretisation whose k-derivative CM_OP_DZDK
                        applies, e.g. for finite differences in k       */
} cm_opts;

/* Fill opts with defaults: nlv = 0 (must be set), d0 = 3, interp_p = 6,
   eta = 376.730313668, flags = 0, max_cols = 32, k_sampling = 0. */
void cm_default_opts(cm_opts* o);

/* Build a handle.  xyz: host, n_vert x 3 float64 (wavelength units are the
   caller's; k is in the same units).  tri: host, n_tri x 3 int32 vertex
   indices.  k: host array of n_k >= 1 wavenumbers (a sweep): the same tree
   and lists for all, and per wavenumber its own truncation (eq. (30)),
   sampling, translators, leaf patterns, shift phases and near field, so the
   set-up work and device memory grow n_k-fold.  cm_apply picks a wavenumber
   per column (k_index); every other entry point works at k[0].  Blocks until
   all device set-up (near-field fill with singularity extraction, leaf
   radiation patterns, translators) is complete.  The caller keeps ownership
   of xyz/tri/k (copied).  On failure *out is NULL. */
cm_status cm_create(const double* xyz, int64_t n_vert, const int32_t* tri, int64_t n_tri,
                    const double* k, int32_t n_k, const cm_opts* o, void* hip_stream,
                    cm_handle** out);

/* Release all host and device memory of the handle (NULL is a no-op). */
void cm_destroy(cm_handle* h);

/* Number of RWG unknowns N. */
cm_status cm_num_unknowns(const cm_handle* h, int64_t* n);

/* RWG table in the library's unknown order: edge_v (N x 2: smaller, larger
   vertex), tri_pm (N x 2: T+, T-).  Host arrays, caller-allocated. */
cm_status cm_rwg_table(const cm_handle* h, int32_t* edge_v, int32_t* tri_pm);

/* y = op(x) on ncols columns (1 <= ncols <= max_cols).  k_index: NULL (all
   columns at k[0]) or a host array of ncols indices into the handle's k
   array, column j being applied at k[k_index[j]] (columns sharing a
   wavenumber are gathered into one batched apply, padded with zero columns
   to a multiple of 8 where max_cols allows, so that it takes the
   matrix-core kernels; a batch at a single wavenumber runs in place; with
   CM_FLAG_SWEEP_SHARED an FP32 Z or Z^H batch at several wavenumbers runs as
   one pass over slots of four columns per wavenumber, padded with zero
   columns, when 4 x slots <= max_cols and slots <= 16).
   Asynchronous on hip_stream; CM_E_BADARG for an index outside [0, n_k). */
cm_status cm_apply(cm_handle* h, cm_op op, const void* x, void* y, int64_t ld, int32_t ncols,
                   const int32_t* k_index, cm_dtype dt, void* hip_stream);

/* y = op(x) as cm_apply at k[0], for callers that cannot allocate device
   memory (code under HIP graph capture, serving loops, harnesses that forbid
   hipMalloc): the apply's workspace (pattern levels, permuted input,
   near-field output) lives in one fixed 64 MiB device array of the library
   instead of the handle's workspace, and the call allocates nothing.  The
   same kernels as cm_apply in the same order, so the result equals cm_apply's
   bit for bit.  Arguments, layout and ownership as cm_apply (without
   k_index); the current device must be the handle's.  CM_E_BADARG when the
   workspace for this handle, op, dtype and ncols exceeds 64 MiB (the message
   gives the size; e.g. about 3 MiB for 1,920 unknowns and 8 columns).
   Every call on a GPU shares that GPU's array: calls that overlap on one GPU
   (two streams, two handles, two threads) race on it, and the caller orders
   them.  Stage timing is not recorded.  Asynchronous on hip_stream. */
cm_status cm_apply_noalloc(cm_handle* h, cm_op op, const void* x, void* y, int64_t ld, int32_t ncols, cm_dtype dt,
                           void* hip_stream);

/* Build the SAI preconditioner P minimising ||I - A P||_F column by column
   over a prescribed pattern (section IV), for the near field A of the
   operator tau R + i X: tau = 1 gives A = Z_near (the paper's preconditioner
   of the inner solves with Z); other tau > 0 give tau Re Z_near + i Im Z_near
   (the inner solves of cm_eigs with that shift); tau = 0 gives the real
   matrix X_near = Im Z_near (the inner solves with X of cm_eigs_xinv).  The
   shifted operators and their preconditioners are an extension of this
   library (the paper documents no preconditioner for X).  At the wavenumber
   k[k_index] of the handle: a sweep handle keeps, per wavenumber, one SAI of
   Z_near and one of the most recent other tau.  Entries of A with
   |a_ij| < eps1 |a_jj| are dropped, column j's pattern is
   {i : |a_ij| >= eps2 |a_jj|}, and entries of the solution with
   |p_ij| < eps3 max_i |p_ij| are dropped afterwards.  CM_E_BADARG for a
   threshold outside [0, 1], k_index outside [0, n_k) or tau outside
   [0, 1e6].  Rebuilding replaces the previous P of that slot and
   wavenumber.  Blocks. */
cm_status cm_sai_build(cm_handle* h, double eps1, double eps2, double eps3, int32_t k_index, double tau);

/* y = P x for the SAI built with tau (1: of Z_near); vector conventions and
   k_index (per column, NULL = all at k[0]) as cm_apply.  CM_E_NOT_BUILT if
   that SAI was not built for a wavenumber a column uses.  Asynchronous. */
cm_status cm_sai_apply(cm_handle* h, const void* x, void* y, int64_t ld, int32_t ncols, const int32_t* k_index,
                       double tau, cm_dtype dt, void* hip_stream);

/* out = sum_{i < N, c < ncols} conj(x[i*ld + c]) y[i*ld + c]: the complex
   inner product of two N x ncols blocks (CM_C64 or CM_C128, accumulated in
   FP64), written to out (DEVICE pointer, one complex128).  With y =
   (dZ/dk) x this is the wavenumber gradient Re(g^H dZ/dk x) of the backward
   pass (take the real part).  The sum is formed in a fixed order (partial sums
   per block in the handle's reduction buffer, then the blocks in order), so
   it is reproducible; calls that overlap on one handle race on that buffer.
   Asynchronous on hip_stream. */
cm_status cm_vdot(cm_handle* h, const void* x, const void* y, int64_t ld, int32_t ncols, cm_dtype dt, void* out,
                  void* hip_stream);

/* Real characteristic currents (section V): for each of the m complex128
   columns of J (device, N x m row-major, row stride ldj; e.g. Ritz vectors,
   each a real vector times a complex number), the phase that makes
   sum_i J_i^2 real and positive is removed, the real part kept (Jr, with zero
   imaginary parts) and scaled so that Jr^T R Jr = 1; RJr receives R Jr.  Jr
   and RJr: device, N x m complex128, row stride ldo, caller-owned, not
   aliasing J or each other.  All N-vector work on the device (FP64 R
   products and reductions).  CM_E_NUMERIC if a column has no positive R-norm.
   Synchronises with hip_stream. */
cm_status cm_real_currents(cm_handle* h, const void* J, int64_t ldj, int32_t m, void* Jr, void* RJr, int64_t ldo,
                           void* hip_stream);

/* Modal correlation of two sets of currents through R at this handle's
   wavenumber k[0] (the mode correspondence of a frequency sweep, section V):
   C[a*mb + b] = |Ja_a^T R Jb_b| / sqrt(|Ja_a^T R Ja_a| |Jb_b^T R Jb_b|) for the
   ma columns of Ja (device, N x ma complex128, row stride lda) and the mb
   columns of Jb (row stride ldb); C: host, ma x mb.  FP64 R products and
   device reductions.  Synchronises with hip_stream. */
cm_status cm_modal_correlation(cm_handle* h, const void* Ja, int64_t lda, int32_t ma, const void* Jb, int64_t ldb,
                               int32_t mb, double* C, void* hip_stream);

/* d lambda/dk of one characteristic value lambda (real) or of one
   (near-)degenerate cluster of m values around it, from the characteristic
   equation X J = lambda R J differentiated at fixed tree and sampling:
     d lambda/dk = eig( Q^T (X' - lambda R') Q ),   Q^T R Q = I,
   with X' = Im dZ/dk, R' = Re dZ/dk (the dZ/dk pass, CM_FLAG_DERIV) and Q a
   real R-orthonormal basis of the cluster (the m dominant directions of the
   real span of J's real and imaginary parts); for m = 1 this is
   J^T (X' - lambda R') J / J^T R J.  J: device, N x m complex128, row stride
   ldj (1 <= m <= 256).  dldk: host, m values, ascending.  CM_E_NOT_BUILT
   without CM_FLAG_DERIV, CM_E_NUMERIC if the span has no positive R-norm.
   Synchronises with hip_stream. */
cm_status cm_dlambda_dk(cm_handle* h, double lambda, const void* J, int64_t ldj, int32_t m, double* dldk,
                        void* hip_stream);

/* GMRES(restart) for Z x = b (the inner solves Z^-1 u of section IV).
   precond: 0 none; 1 right-preconditioned by the SAI P, x = P u (needs
   cm_sai_build); 2 the Calderon preconditioner of eq. (25), GMRES on
   Z~ G^-1 Z x = Z~ G^-1 b (needs cm_cmp_build; tol and *relres then refer
   to that system).  b, x: device, N complex128 (FP64 Krylov vectors and
   Gram-Schmidt); far_dtype selects the far field of the Z products (CM_C128
   FP64, CM_C64 FP32).  x0 = 0; stops when ||b - Z x|| <= tol ||b|| or after
   maxit iterations (CM_E_NOT_CONVERGED).  *iters and *relres (may be NULL)
   receive the iteration count and the final true relative residual.
   Synchronises with hip_stream. */
cm_status cm_gmres(cm_handle* h, const void* b, void* x, int32_t restart, int32_t maxit, double tol,
                   int32_t precond, cm_dtype far_dtype, int32_t* iters, double* relres, void* hip_stream);

/* Characteristic modes by the implicitly restarted Arnoldi method on
   OP = (tau R + i X)^-1 R: tau = 1 is OP = Z^-1 R of eq. (24), whose
   eigenvalues mu = 1/(1 + i lambda) crowd at 1 when many modes have
   |lambda| << 1 (large bodies); a smaller shift tau > 0 (an extension of
   this library) maps them to mu = 1/(tau + i lambda), spread around a circle
   of diameter 1/tau, so that the modes with |lambda| up to about tau are
   well separated (each inner product then costs an R and an X apply).  The
   nev eigenvalues mu of largest magnitude (smallest |tau + i lambda|) of an
   ncv-vector factorisation with exact-shift restarts (nev < ncv <= N), each
   OP product one R apply and one GMRES solve with tau R + i X
   (gmres_restart, gmres_maxit, gmres_tol), right-preconditioned when
   precond = 1 by the SAI built with the same tau (cm_sai_build), or, with
   precond = 2 and tau = 1, by the Calderon preconditioner (cm_cmp_build).  v0:
   device start vector (N complex128, nonzero; the caller draws it).
   Outputs (host): lambda[2*nev] interleaved complex characteristic values
   lambda = i (tau - 1/mu), smallest |tau + i lambda| first; ritz_resid[nev]
   (may be NULL) the relative Ritz residual estimates; J (device, may be
   NULL) the N x nev Ritz vectors, column-major, unit 2-norm; *nconv the
   number with residual <= tol; counters[6] (may be NULL): OP products,
   GMRES iterations, operator applies, restarts, inner solves redone without
   the preconditioner, inner solves that missed gmres_tol.  A preconditioned
   inner solve that misses gmres_tol within gmres_maxit is redone once
   without the SAI (which can be nearly singular).  Returns
   CM_E_NOT_CONVERGED if fewer than nev converged within maxrestart
   restarts, or if any inner solve missed gmres_tol (the Ritz values then
   belong to an inexact OP).  Synchronises. */
cm_status cm_eigs(cm_handle* h, int32_t nev, int32_t ncv, int32_t maxrestart, double tol, const void* v0,
                  int32_t gmres_restart, int32_t gmres_maxit, double gmres_tol, int32_t precond, double tau,
                  cm_dtype far_dtype, double* lambda, double* ritz_resid, void* J, int32_t* nconv,
                  int64_t* counters, void* hip_stream);

/* Calderon multiplicative preconditioner (section IV, eqs. (25)-(27)) of a
   handle on a closed surface (CM_E_MESH otherwise): builds the barycentric
   refinement of the mesh (each triangle split into six at its edge midpoints
   and centroid), an MLFMA handle on it with nlv_refined levels (0: one more
   than the handle's), interpolation order interp_p_refined and truncation
   parameter d0_refined (0: the handle's) and its other options (one column;
   FP32 products take the near field in FP32, CM_FLAG_NEAR_FP32), the
   Buffa-Christiansen function of every RWG as a combination of the refined
   mesh's RWG functions (the paper names these functions without defining
   them: each carries the RWG's flux l_e from the dual cell of one endpoint
   of the edge to that of the other, with equal charge on every small
   triangle of a cell, half of the flux through each half of the dual edge
   and none through the refined edges along the primal edge), and the mixed
   Gram matrix G_ij = <n x f_i, f~_j> (eq. (27)).  Z~ (eq. (26)) is then
   applied as B Z_ref B^T and G^-1 by GMRES on G.  Z~ only preconditions
   (any fixed Z~ leaves the solution of eq. (25) that of Z x = u), so the
   refined handle may be built coarser and cheaper than the handle itself.
   info (host, may be NULL)
   receives 5 values: refined unknowns, entries of B, entries of G, near-field
   entries of the refined handle, its levels.  A second call rebuilds.  On a
   host-only handle (CM_FLAG_HOST_ONLY) only the host tables are built
   (cm_cmp_export).  Synchronises. */
cm_status cm_cmp_build(cm_handle* h, int32_t nlv_refined, int32_t interp_p_refined, double d0_refined,
                       int64_t* info, void* hip_stream);

/* Host copy of a Calderon table in CSR by rows (public indices): which = 0
   B (N x N_refined: row i holds the coefficients of the i-th BC function on
   the refined mesh's RWG functions, in that handle's public order, i.e.
   interior refined edges in increasing (smaller, larger) vertex order, the
   refined vertices being the mesh's vertices, then one midpoint per RWG in
   RWG order, then one centroid per triangle; refined triangle 6t + 2a is
   (v_a, m(a, a+1), c_t) and 6t + 2a + 1 is (v_a, c_t, m(a-1, a)) for corner a
   of triangle t), 1 G (N x N).  *rows and *nnz always; ptr (rows + 1), col
   and val (nnz) are filled when all three are non-NULL (caller-allocated).
   Needs cm_cmp_build. */
cm_status cm_cmp_export(const cm_handle* h, int32_t which, int64_t* rows, int64_t* nnz, int64_t* ptr, int32_t* col,
                        double* val);

/* One product with the Calderon preconditioner's matrices on a single
   column (x, y: device, N complex128, must not alias): which = 0 y = Z~ x,
   1 y = G x, 2 y = Z~ G^-1 Z x (the matrix of eq. (25); the Gram solve to a
   relative residual of 1e-12, CM_E_NOT_CONVERGED if it misses; inside
   cm_gmres and cm_eigs the Gram solves go to 1e-2 of the outer tolerance,
   within [1e-13, 1e-6]).  far_dtype
   selects the far field of the MLFMA products.  Needs cm_cmp_build.
   Synchronises with hip_stream. */
cm_status cm_cmp_apply(cm_handle* h, int32_t which, const void* x, void* y, cm_dtype far_dtype, void* hip_stream);

/* Characteristic modes by the implicitly restarted Arnoldi method on
   OP = X^-1 R (the standard eigenvalue problem of eq. (14)): mu = 1/lambda,
   so the nev largest |mu| are the smallest |lambda|, well separated in
   magnitude even where Z^-1 R (whose mu = 1/(1 + i lambda) crowd near 1)
   clusters them.  Arguments, outputs and counters[6] as cm_eigs, with inner
   GMRES solves with X, right-preconditioned when precond != 0 by the SAI of
   X_near (cm_sai_build with tau = 0; the paper notes that no efficient
   preconditioner for X is documented: this one is the library's own).  The
   far field of X uses the imaginary part of Z's translator, so X x is as
   accurate as Z x on the same tree (the two-box buffer, CM_FLAG_WIDE_NEAR,
   where leaf boxes are small against the wavelength).  Synchronises. */
cm_status cm_eigs_xinv(cm_handle* h, int32_t nev, int32_t ncv, int32_t maxrestart, double tol, const void* v0,
                       int32_t gmres_restart, int32_t gmres_maxit, double gmres_tol, int32_t precond,
                       cm_dtype far_dtype, double* lambda, double* ritz_resid, void* J, int32_t* nconv,
                       int64_t* counters, void* hip_stream);

/* Characteristic modes by Jacobi-Davidson on the pencil X J = lambda R J
   (eq. (6)) with the R-orthonormal search space and the projected correction
   equation of eqs. (28)-(29): no inner solve with Z or X, each correction an
   approximate solution by inner_steps GMRES steps (one R and one X apply
   each), unpreconditioned (precond 0), right-preconditioned by i P with P the
   SAI of Z_near (precond 1; X - theta R is close to -i (Z - R) for targets
   near 0) or by P the SAI of X_near (precond 2, cm_sai_build with tau = 0;
   X - theta R is close to X near theta = 0).  harmonic = 0 selects the Ritz
   pairs of V^H X V nearest the target; harmonic != 0 the harmonic Ritz pairs
   for the target (W^H (X - theta R) V s = 0 with W = (X - target R) V, the
   smallest |theta - target| first, with the Rayleigh quotient as the value),
   which converge where the target lies inside a dense part of the spectrum
   (an extension of this library).  Finds the nev characteristic values
   closest to target (0 for the significant modes); the search space holds
   at most mmax vectors and restarts from the mmin (harmonic) Ritz vectors
   nearest the target.  A pair is accepted when
   ||X u - theta R u|| <= tol max(1, |theta|) ||R u||, then locked
   (deflated).  v0: device start vector (N complex128; the caller draws it).
   Outputs (host): lambda[nev] real characteristic values in the order found;
   resid[nev] (may be NULL) their relative residuals; J (device, may be NULL)
   the N x nev eigenvectors, column-major, R-normalised (J^H R J = I); *nconv
   the number found; counters[4] (may be NULL): outer iterations, inner GMRES
   steps, operator applies, 1 if the preconditioner was dropped (no new
   converged pair within max(50, maxit / 8) outer iterations: the SAI can be
   nearly singular).  Returns CM_E_NOT_CONVERGED when fewer than nev were
   found within maxit outer iterations (the first *nconv outputs are valid),
   CM_E_NUMERIC when an expansion vector has no R-norm (R is singular on it),
   CM_E_NOT_BUILT for a preconditioner whose SAI was not built.  Synchronises. */
cm_status cm_jd(cm_handle* h, int32_t nev, double target, int32_t mmin, int32_t mmax, int32_t maxit, double tol,
                int32_t inner_steps, int32_t precond, int32_t harmonic, const void* v0, cm_dtype far_dtype,
                double* lambda, double* resid, void* J, int32_t* nconv, int64_t* counters, void* hip_stream);

/* Copy the near-field matrix to host (public unknown order, CSR by row):
   row_ptr (N+1, int64), col (nnz, int32), val (nnz complex128 interleaved).
   Pass NULLs to query *nnz only.  which = 0: Z_near, 1: dZ_near/dk,
   2: the SAI matrix of Z_near, 3: the SAI matrix of the other tau (at
   k[0]; tau = 0: of X_near). */
cm_status cm_export_near(const cm_handle* h, int32_t which, int64_t* nnz, int64_t* row_ptr,
                         int32_t* col, double* val);

/* JSON description of the plan of k[0] (levels with boxes, L, the translator
   truncation L_translator, K and list sizes; nnz; k_sampling), the autotuner's
   choices ("autotune") and, for a sweep with CM_FLAG_SWEEP_SHARED, the number
   of wavenumbers in its one-pass tables ("sweep_tables") and of one-pass
   applies so far ("sweep_one_pass_calls"), NUL-terminated into buf.
   Returns CM_E_BADARG if buf_len is too small (needed size in *needed). */
cm_status cm_stats(const cm_handle* h, char* buf, int64_t buf_len, int64_t* needed);

/* Pin the translation kernel of the FP32 batched applies on every level (of
   every wavenumber of a sweep handle), overriding the default and the
   autotuner's choice: 1 receiver tiles of 16 boxes, each block loading its
   own sources (the default); 2 tiles of 64 boxes whose four waves share
   their sources through LDS, two directions per thread, chunks of 8
   sources; 3 the same with chunks of 4 at three waves per SIMD; 4 one
   direction per thread.  All give the same bits; on the 122,880-unknown
   sphere at 32 columns the 16-box tiles are the fastest.  CM_E_BADARG for
   another value. */
cm_status cm_set_translation_kernel(cm_handle* h, int32_t variant);

/* Per-stage timing of applies: with enable != 0, every later cm_apply /
   cm_sai_apply on this handle brackets each kernel stage with HIP events
   recorded on the apply's own stream (small overhead); enable = 0 turns it
   off.  Either call resets the accumulated times. */
cm_status cm_stage_timing(cm_handle* h, int32_t enable);

/* Accumulated stage times since cm_stage_timing as JSON
   {"near": {"ms": total, "calls": n}, "m2l_l5": {...}, ...}, NUL-terminated
   into buf (needed size in *needed; CM_E_BADARG if buf_len is too small).
   Synchronises with the recorded events. */
cm_status cm_stage_times(cm_handle* h, char* buf, int64_t buf_len, int64_t* needed);

/* Message of the last failure on this thread ("" if none). */
const char* cm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CMMLFMA_H */
