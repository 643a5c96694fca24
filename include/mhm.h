/*
 * mhm.h - C ABI of the MI355X (gfx950) engine for the local problems of the
 * Multiscale Hybrid-Mixed (MHM) method.
 *
 * What the library computes, per coarse element K (the solveLocalProblem
 * primitive of Algorithm 1, Section 3, for the Darcy subproblems of
 * eqs. (8)-(9), Section 4.2), specialised to 2D, continuous P1 elements on a
 * uniform refinement of the triangle K with s subdivisions per edge, and face
 * multipliers of degree l on each of the three faces (m = 1, Section 2):
 *
 *   n   = (s+1)(s+2)/2 sub-mesh nodes,   T = s*s sub-triangles,
 *   N_I = 3(l+1) face DoFs,              r = N_I + 1 right-hand sides.
 *
 *   A      n x n P1 stiffness of (kappa grad u, grad w)_K, kappa constant on
 *          each sub-triangle.
 *   c      c_j = integral of phi_j over K.
 *   Ahat   = A + gamma c c^T with gamma = trace(A) / (n c^T c); symmetric
 *          positive definite, it imposes the zero mean of V_0^perp(K).
 *   B      n x r: columns a = e(l+1)+q hold -sigma_e (P_q, phi_j)_{F_e}
 *          (eq. (9); P_q the Legendre polynomial on the globally oriented
 *          face), the last column holds (f, phi_j)_K (eq. (8)).
 *   Btilde = B - c (1^T B) / |K|   (compatible right-hand sides).
 *   X      n x r: Ahat X = Btilde, then X -= 1 (c^T X)/|K|; the coefficient
 *          vectors d_i and c of eq. (5), face DoFs first, source last.
 *   M, E, B, F: the element's blocks of the skeleton system eq. (6):
 *          M[a][b] = (sigma psi_a, eta^b)_{dK} (N_I x N_I, symmetric,
 *          negative definite), E[a] = -(sigma psi_a, eta^f)_{dK},
 *          B[a] = (sigma psi_a, 1)_{dK}, F = (f, 1)_K.
 *
 * Sub-mesh numbering: node (i,j), i,j >= 0, i+j <= s, lies at
 * v0 + (i/s)(v1-v0) + (j/s)(v2-v0) with index j(s+1) - j(j-1)/2 + i.
 * Sub-triangles are in row strips j = 0..s-1: up triangle (i,j) (nodes
 * (i,j),(i+1,j),(i,j+1)) at j(2s-j)+2i, down triangle (i,j) (nodes
 * (i+1,j+1),(i,j+1),(i+1,j)) at j(2s-j)+2i+1.  Face e is opposite vertex e
 * and runs v[e+1] -> v[e+2]; flip[e] = 1 when that direction goes from the
 * higher to the lower global vertex id (face polynomials use t = -1 at the
 * lower id).  sigma[e] = +1 or -1 is the sign n . n^K_F.
 *
 * Memory: every array pointer in mhm_batch and in the calls below is a
 * DEVICE pointer owned by the caller (the library never frees it).  Matrices
 * are column-major per element at the element's prefix offset.  Calls are
 * asynchronous on the context's HIP stream; outputs are valid once the
 * stream (or mhm_sync) has completed.
 *
 * Errors, two levels:
 *  - call level: the returned mhm_status (argument checks on the host, HIP
 *    launch or allocation failures); mhm_last_error() gives the text.
 *  - element level: info[e] (device int32, written asynchronously):
 *      0   success
 *      k>0 non-positive pivot at column k (1-based) of Ahat: the element's
 *          outputs are filled with NaN (LAPACK potrf convention)
 *     -1   the element's results come from the FP64 path, not from the
 *          FP32 factorisation with FP64 refinement: the refinement did not
 *          reach the tolerance (within max_iters steps, or its observed
 *          contraction said it would not), or, in the fused one-launch
 *          form without a factor store, the element's contrast times s^2
 *          exceeded the bound of MHM_OPT_REFINE64 (s >= 17), so no FP32
 *          attempt was made (ir_iters 0); its outputs are valid
 *     -2   the element's descriptor is inconsistent (s or l out of range,
 *          offsets that disagree with s and l or exceed the *_total sizes,
 *          sign/flip flags out of range, a non-positive area); nothing of
 *          the element is written
 *     -3   the element is larger than the launched kernel supports
 *     -4   (mhm_local_source_step) no stored factor for the element
 *     -5   (mhm_server results) the launch that carried the request failed
 *          (mhm_server_last_error says why): no output was computed, the
 *          result's arrays are NaN, and no factor of that launch is reused
 */
#ifndef MHM_H
#define MHM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MHM_S_LIMIT 64   /* largest s per element          */
#define MHM_INFO_LAUNCH_FAILED (-5)   /* server result of a failed launch */
#define MHM_L_LIMIT 4    /* largest l per element                          */
#define MHM_P_LIMIT 16   /* largest m (l + 1), face DoFs per face (r <= 49):
                            a batch with p_max (or l_max + 1) above 5, that is
                            r above 16, runs on the left-looking kernel only,
                            which takes s <= 48; an element it cannot take
                            reports info -3                                 */

typedef struct mhm_ctx_s* mhm_ctx;
typedef struct mhm_graph_s* mhm_graph;

typedef enum {
  MHM_OK = 0,
  MHM_E_ARG = 1,
  MHM_E_NOMEM = 2,
  MHM_E_DEVICE = 3,
  MHM_E_UNSUPPORTED = 4
} mhm_status;

typedef enum {
  MHM_FP64 = 0,     /* FP64 Cholesky and triangular solves (MFMA f64)          */
  MHM_FP32_IR = 1   /* FP32 Cholesky and solves (MFMA f32) + FP64 refinement    */
} mhm_prec;

/* A ragged batch of local problems p_t = (K_t, {F_t}) (Algorithm 1). */
typedef struct {
  int32_t n_elem;          /* host: number of elements (0 is allowed)          */
  int32_t s_max;           /* host: upper bound on s over the batch            */
  int32_t l_max;           /* host: bound on l                                 */
  int32_t s_min;           /* host: lower bound on s over the batch (0: unknown,
                              taken as 1).  When [s_min, s_max] spans several
                              size classes the batch is binned on the device
                              and every class gets its own launch           */
  const int32_t* s;        /* [n_elem] subdivisions, 1..MHM_S_LIMIT            */
  const int32_t* l;        /* [n_elem] face degree, 0..MHM_L_LIMIT             */
  const double* vert;      /* [n_elem*6] x0 y0 x1 y1 x2 y2, counter-clockwise  */
  const int8_t* sigma;     /* [n_elem*3] +1 / -1                               */
  const int8_t* flip;      /* [n_elem*3] 0 / 1                                 */
  const double* kappa;     /* [tri_total] per sub-triangle, at tri_off[e]      */
  const double* f;         /* [tri_total] per sub-triangle, at tri_off[e]      */
  const int64_t* tri_off;  /* [n_elem+1] prefix sums of s^2                    */
  const int64_t* mat_off;  /* [n_elem+1] prefix sums of n^2   (Ahat, factor)   */
  const int64_t* rhs_off;  /* [n_elem+1] prefix sums of n*r   (Btilde, X)      */
  const int64_t* node_off; /* [n_elem+1] prefix sums of n     (c)              */
  int64_t tri_total;       /* host: element count of kappa and f               */
  int64_t mat_total;       /* host: doubles in the Ahat buffer                 */
  int64_t rhs_total;       /* host: doubles in the Btilde and X buffers        */
  int64_t node_total;      /* host: doubles in the c buffer                    */
  const int32_t* m;        /* [n_elem] segments per face (the m-partition of
                              each face in Section 2: a polynomial of degree l
                              on each of m equal segments, segments and the
                              Legendre variable in the global face orientation),
                              or NULL for m = 1 everywhere.  m must divide s,
                              and m(l+1) <= MHM_P_LIMIT.  N_I = 3 m (l+1)      */
  int32_t p_max;           /* host: bound on m(l+1) over the batch, 0 for
                              l_max + 1; contribution blocks (M, E, B) are
                              padded to NImax = 3 p_max                        */
  int32_t reserved;        /* set to 0                                         */
} mhm_batch;

/* Create a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL means the default stream).  The context owns its
 * workspace and frees it in mhm_destroy. */
mhm_status mhm_create(mhm_ctx* ctx, int device, void* hip_stream);
mhm_status mhm_destroy(mhm_ctx ctx);
/* Change the stream subsequent calls enqueue on. */
mhm_status mhm_set_stream(mhm_ctx ctx, void* hip_stream);

/* Context options (mhm_set_option); every one defaults to 0.
 *  MHM_OPT_REFINE64  the FP64 path's refinement step.  A plain FP64
 *                    Cholesky solve has a forward error that grows with the
 *                    condition number of Ahat, roughly the coefficient
 *                    contrast (max kappa / min kappa over the element) times
 *                    s^2: below 1e-13 for smooth fields, about 1e-10 for a
 *                    contrast of 1e4 at s = 32.  0: elements whose contrast
 *                    times s^2 exceeds 2^20 get one refinement step, its
 *                    residual Btilde - Ahat X accumulated in double-double
 *                    (the solution then matches the exact one of the
 *                    assembled system to about 1e-15); 1: every element;
 *                    -1: none.  ir_iters reports the step (1).  With
 *                    MHM_FP32_IR the same bound (unless -1) sends such an
 *                    element of the fused form straight to the FP64 path
 *                    (info -1): its FP32 refinement would contract slowly
 *                    or stall.
 *  Launch configuration (the results do not depend on them, beyond
 *  rounding; used to exercise kernel families the defaults do not pick, and
 *  reproduced by mhm_autotune's timings):
 *  MHM_OPT_NO_RR     1: never the register-tile kernel
 *  MHM_OPT_NO_LL     1: never the left-looking kernel
 *  MHM_OPT_LL_OCC2   1: left-looking default with two workgroups per CU
 *  MHM_OPT_LL_NW16   1: left-looking default with 16 waves, where built
 *  MHM_OPT_LL_PW     0, 1, 2, 4: left-looking default panel width, where built
 *  MHM_OPT_RR_OCC    0, 2, 3: register-tile kernel's workgroups per CU
 *  MHM_OPT_CONCURRENT_CLASSES  1: run the size classes of a ragged batch
 *                    concurrently, on forked streams, instead of one after
 *                    another on the context's stream (on C4 in FP64 the
 *                    concurrent form took 82 against 78 ms)
 *  MHM_OPT_CLASS_TIMING  1: record HIP timing events on each size class's
 *                    stream around its main kernel launch (not the binning or
 *                    the FP64 pass) in later mhm_local_batch_run and
 *                    mhm_local_factor_solve calls; mhm_class_times reads them.
 *                    Not for use under stream capture.
 * Returns MHM_E_ARG for an unknown option or value.  Applies to later calls
 * (a captured graph keeps the configuration of its capture). */
typedef enum {
  MHM_OPT_REFINE64 = 0,
  MHM_OPT_NO_RR = 1,
  MHM_OPT_NO_LL = 2,
  MHM_OPT_LL_OCC2 = 3,
  MHM_OPT_LL_NW16 = 4,
  MHM_OPT_LL_PW = 5,
  MHM_OPT_RR_OCC = 6,
  MHM_OPT_CLASS_TIMING = 7,
  MHM_OPT_CONCURRENT_CLASSES = 8
} mhm_option;
mhm_status mhm_set_option(mhm_ctx ctx, int option, int value);

/* With MHM_OPT_CLASS_TIMING on: the size classes of the last timed call,
 * largest first, and the duration of each class's main kernel launch in
 * milliseconds (it waits for them).  s_cap[k] is the upper s of class k's
 * launch.  Returns the number of classes (at most max), or -1 when the option
 * is off or no call has been timed. */
int mhm_class_times(mhm_ctx ctx, int32_t* s_cap, float* ms, int max);
/* Text of the last call-level error on this context ("" if none); with a
 * NULL context, the last error of a context-less call (mhm_create) on the
 * calling thread. */
const char* mhm_last_error(mhm_ctx ctx);
/* SHA-256 (64 hex digits) of the sources and compile flags this library was
 * built from, for checking that a built library matches its sources; a
 * static string owned by the library ("unstamped" when built without it). */
const char* mhm_source_hash(void);
/* Block until all work enqueued by this context has finished. */
mhm_status mhm_sync(mhm_ctx ctx);
/* Device workspace (bytes) the context allocates for a batch and precision
 * (elements too large for on-chip storage use a per-workgroup slot). */
size_t mhm_workspace_bytes(mhm_ctx ctx, const mhm_batch* batch, mhm_prec prec);

/* Steps a2-a3: assemble Ahat (n x n, column-major, both triangles),
 * Btilde (n x r, column-major), c (n) and |K| per element.  info as above
 * (only 0 or -2 here).  Defined by eqs. (2)-(3), (8)-(9) and Section 3's
 * shared matrix A with N_I + 1 load vectors. */
mhm_status mhm_local_assemble(mhm_ctx ctx, const mhm_batch* batch,
                              double* Ahat, double* Btilde, double* c,
                              double* area, int32_t* info);

/* Steps a4-a5 (and a5' for MHM_FP32_IR): factor Ahat = L L^T once and solve
 * the r right-hand sides (Section 3: one matrix, factored once, many load
 * vectors), then project X to zero mean.
 *   Ahat_io  in: Ahat from mhm_local_assemble.  out: the lower triangle of
 *            L (MHM_FP64), or the FP32 L, column-major, in the first n*n
 *            floats of the element's slot (MHM_FP32_IR; for elements that
 *            report info == -1 this FP32 L is the one whose refinement did
 *            not converge, and X comes from the FP64 recomputation).  The
 *            strict upper part is unspecified.
 *   Btilde   in: compatible right-hand sides.
 *   X        out: n x r solutions (FP64).
 *   ir_iters out (may be NULL): refinement steps taken per element (FP64:
 *            0, or 1 where MHM_OPT_REFINE64 gave the element its step).
 *   max_iters: refinement step limit (MHM_FP32_IR; ignored for MHM_FP64). */
mhm_status mhm_local_factor_solve(mhm_ctx ctx, const mhm_batch* batch, mhm_prec prec,
                                  double* Ahat_io, const double* Btilde, double* X,
                                  int32_t* info, int32_t* ir_iters, int max_iters);

/* Step a6: the element's contribution to eq. (6) from its solutions X.
 * M [n_elem][NImax*NImax] (column-major NImax x NImax, zero padded),
 * E [n_elem][NImax], B [n_elem][NImax], F [n_elem]; NImax = 3 p_max
 * (3 (l_max+1) when p_max is 0).  Elements whose info[e] on entry is other
 * than 0 or -1 are skipped (info may be NULL). */
mhm_status mhm_skeleton_contrib(mhm_ctx ctx, const mhm_batch* batch, const double* X,
                                double* M, double* E, double* B, double* F,
                                const int32_t* info);

/* Steps a2-a6 fused per element: assemble, factor, solve (and refine),
 * contribute, without writing Ahat or Btilde to memory.  Same contract and
 * layouts as the three calls above.  Under MHM_FP32_IR, elements whose
 * refinement does not converge are recomputed in FP64 (info = -1). */
mhm_status mhm_local_batch_run(mhm_ctx ctx, const mhm_batch* batch, mhm_prec prec,
                               double* X, double* M, double* E, double* B, double* F,
                               int32_t* info, int32_t* ir_iters, int max_iters);

/* No-allocation variant of mhm_local_batch_run, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the same work, contract and
 * results (bit for bit, on the same kernels), with every scratch buffer (the
 * size-class lists of a ragged batch and the per-workgroup workspace slots
 * of large elements) in a device array that the library holds on each GPU
 * it runs on, MHM_NOALLOC_SCRATCH_BYTES in size, until the process ends; the
 * call itself performs no allocation of any kind.  The size classes run one
 * after another on the context's stream, and a launch whose workgroups need
 * slots runs as many workgroups as slots fit in the array (fewer than
 * mhm_local_batch_run for the largest elements: slower, same results).
 * Nothing in the array needs to start at zero.  Every call on one GPU uses
 * that GPU's one array: calls that overlap on a GPU (other streams, other
 * contexts or threads) race and give wrong results; serialise them.
 * Returns MHM_E_ARG, without enqueuing anything, for a batch whose class
 * lists (4 (5 n_elem + 5) bytes) or one workspace slot of its largest
 * elements do not fit in the array. */
#define MHM_NOALLOC_SCRATCH_BYTES (256u << 20)
mhm_status mhm_local_batch_run_noalloc(mhm_ctx ctx, const mhm_batch* batch, mhm_prec prec,
                                       double* X, double* M, double* E, double* B, double* F,
                                       int32_t* info, int32_t* ir_iters, int max_iters);

/* Around the path: the assembly of the skeleton system eq. (6) from the
 * element contributions (the reduce step of reduceLocalProblems,
 * Algorithm 1) and computeSolution, eq. (4).  The global numbering is the
 * caller's; both calls take
 *   gdof   [n_elem * NImax] device int32, NImax as for the blocks: global row
 *          of local face DoF a of element e (entries a >= N_I of the element
 *          are not read),
 *   erow   [n_elem] device int32: global row of the element's constant u_0,
 *   n_rows rows of the skeleton system; an index outside [0, n_rows) is an
 *          error of the data, handled per call below.
 * mhm_skeleton_scatter adds, for every element whose info[e] is 0 or -1
 * (info may be NULL), M[a][b] at (gdof[a], gdof[b]), B[a] at (erow, gdof[a])
 * and (gdof[a], erow), E[a] to rhs[gdof[a]] and F to rhs[erow], into a CSR
 * matrix whose pattern (row_ptr [n_rows+1], col_idx sorted within each row,
 * both device int32) the caller built.  vals [nnz] and rhs [n_rows]
 * accumulate: clear them first for a fresh system.  The additions are FP64
 * atomics, so their order, and with three or more terms per entry the last
 * bits, vary between runs.  An entry absent from the pattern or with an
 * index out of range is skipped and counted in *missing (device int32, may
 * be NULL; it accumulates too).
 * mhm_reconstruct writes u[node_off[e] + p] = sol[erow[e]] +
 * sum_a X[p][a] sol[gdof[e][a]] + X[p][N_I] (the nodal values of u_{H,h} on
 * the element's sub-mesh, in lattice order) for every element whose info is
 * 0 or -1; other elements' nodes are left as they are.  An out-of-range
 * index makes the element's values NaN.  The batch needs node_off. */
mhm_status mhm_skeleton_scatter(mhm_ctx ctx, const mhm_batch* batch, const double* M, const double* E,
                                const double* B, const double* F, const int32_t* gdof, const int32_t* erow,
                                const int32_t* row_ptr, const int32_t* col_idx, int32_t n_rows, double* vals,
                                double* rhs, const int32_t* info, int32_t* missing);
mhm_status mhm_reconstruct(mhm_ctx ctx, const mhm_batch* batch, const double* X, const int32_t* gdof,
                           const int32_t* erow, const double* sol, int32_t n_rows, double* u, const int32_t* info);

/* The skeleton solve (the solve of reduceLocalProblems, Algorithm 1):
 * eq. (6) is symmetric and indefinite, [[M, B^T], [B, 0]] [lambda; u_0] =
 * [E; F] with M negative (semi-)definite.  Preconditioned MINRES (the
 * minimal-residual method for symmetric indefinite systems) with a block
 * diagonal preconditioner diag(D, S~): D the lambda_block x lambda_block
 * diagonal blocks of -M (one face's DoFs), S~^-1 a fixed number of
 * Chebyshev steps on S = B D^-1 B^T (the u_0 rows; diag(S) alone above
 * 8,192 elements); with lambda_block = 1, D = |diag M| and S~ = diag(S).  The paper uses sparse direct solvers and names hybrid
 * direct-iterative ones as future work (Section 6).
 *   n_rows, n_lambda  rows of the system; rows < n_lambda are multiplier
 *             rows (M, B^T), the others u_0 rows (B, 0), as numbered for
 *             mhm_skeleton_scatter.
 *   lambda_block  multiplier rows come in groups of this many consecutive
 *             indices, one group per face (m (l+1) in the numbering of
 *             mhm_skeleton_scatter); 1 to 8, and a divisor of n_lambda, else
 *             MHM_E_ARG.
 *   row_ptr [n_rows+1], col_idx, vals (device): the CSR matrix, e.g. as
 *             accumulated by mhm_skeleton_scatter (both triangles).  The
 *             structure is checked on the device first (row pointers from 0,
 *             non-decreasing; columns in [0, n_rows)); a violation returns
 *             MHM_E_ARG before any product.  vals must hold row_ptr[n_rows]
 *             entries.
 *   rhs [n_rows] (device), sol [n_rows] (device, written; x_0 = 0).
 *   tol       stop when the preconditioned residual norm has fallen by tol.
 *   max_iters bound on the MINRES steps.
 *   iters, relres (host, may be NULL): steps taken and the final true
 *             relative residual ||rhs - K sol||_2 / ||rhs||_2.
 * A singular but consistent system (multiplier block rank deficient, l >= s)
 * is fine: u_0, and u of mhm_reconstruct, are unique.  Uses the context's
 * workspace ((17 + lambda_block) n_rows doubles at most, plus a few KB);
 * synchronises the stream (the host reads the residual estimate every 16
 * steps); deterministic for a given launch configuration. */
mhm_status mhm_skeleton_solve(mhm_ctx ctx, int32_t n_rows, int32_t n_lambda, int32_t lambda_block,
                              const int32_t* row_ptr, const int32_t* col_idx, const double* vals,
                              const double* rhs, double* sol, double tol, int32_t max_iters, int32_t* iters,
                              double* relres);

/* Factor reuse (Section 3: the local matrix is factored once and reused
 * for further load vectors, e.g. over time steps): mhm_local_batch_run with
 * each element's factor kept in a caller-owned device store.
 *   factors       device store; element e's factor occupies
 *                 mhm_factor_bytes(s_e, prec) bytes at byte offset
 *                 factor_off[e] (a multiple of 256; regions of elements in
 *                 one call must not overlap).  The layout is internal
 *                 (16x16 tiles of L with the inverse diagonal blocks) and
 *                 tied to prec.
 *   factor_state  [n_elem] device int8: 0 = factor Ahat and store the factor,
 *                 1 = reuse the stored factor of an earlier call for the same
 *                 element data (s, geometry, kappa); only the right-hand
 *                 sides (any l) are built and solved.
 * A stored factor is valid after a call that reported info[e] == 0 for it
 * (after info > 0 the store holds no factor; after -1 it holds the FP32
 * factor whose refinement did not converge, which a reuse would again
 * recompute in FP64).  Requires s <= 48 (the left-looking kernel).
 * Outputs as mhm_local_batch_run. */
size_t mhm_factor_bytes(int s, mhm_prec prec);
mhm_status mhm_local_batch_run_cached(mhm_ctx ctx, const mhm_batch* batch, mhm_prec prec,
                                      void* factors, const int64_t* factor_off,
                                      const int8_t* factor_state,
                                      double* X, double* M, double* E, double* B, double* F,
                                      int32_t* info, int32_t* ir_iters, int max_iters);

/* Time steps on stored factors (Section 3: with coefficients that do not
 * change in time, the local matrix is assembled and factored only in the
 * first step of a time-marching scheme).  The multiplier load vectors do not
 * change either, so after a first mhm_local_batch_run_cached call (state 0,
 * which stores the factors and computes every column of X, M, E, B, F) a
 * step with a new source f only recomputes the source column: btilde_f of
 * eq. (8), one forward and one backward solve with the stored factor, the
 * zero-mean projection, E = R^T eta^f and F = (1, f)_K of eq. (6).
 *   batch     the same elements (s, l, geometry, kappa, offsets) as the call
 *             that stored the factors and produced X, M and B; f is the new
 *             source.
 *   factors, factor_off, factor_state  as for mhm_local_batch_run_cached
 *             and the same prec; only elements with factor_state[e] == 1 are
 *             solved, the others report info -4 and are left untouched.
 *   X         column N_I (the source) of each element is rewritten; the
 *             multiplier columns are read by nobody and left as they are.
 *   E, F      rewritten.  M and B are not written, except with MHM_FP32_IR
 *             for elements whose refinement does not converge (info -1):
 *             those are recomputed in full in FP64 (X, M, E, B, F), so with
 *             MHM_FP32_IR M and B must be the arrays of the first call.
 *   ir_iters  refinement steps (FP32_IR; may be NULL).
 * info[e] as mhm_local_batch_run, plus -4: no stored factor for the element.
 * Requires s <= 48. */
mhm_status mhm_local_source_step(mhm_ctx ctx, const mhm_batch* batch, mhm_prec prec, const void* factors,
                                 const int64_t* factor_off, const int8_t* factor_state, double* X, double* M,
                                 double* E, double* B, double* F, int32_t* info, int32_t* ir_iters,
                                 int max_iters);

/* Batching: choose, per size class present in the batch, the kernel family
 * and panel width ("tile shape": register-resident tiles, LDS tiles,
 * left-looking panels of 2 or 4 tile columns, or the right-looking
 * workspace kernel) by timing every feasible one on up to 4 x (compute
 * units) elements of that class, keep the fastest in the context for later
 * mhm_local_batch_run and mhm_graph_create calls, then run the batch once
 * (the outputs are those of mhm_local_batch_run).  Synchronises the stream;
 * not for use under stream capture.  Method unchanged (Section 3, Algorithm
 * 1): only the launch configuration is chosen. */
mhm_status mhm_autotune(mhm_ctx ctx, const mhm_batch* batch, mhm_prec prec,
                        double* X, double* M, double* E, double* B, double* F,
                        int32_t* info, int32_t* ir_iters, int max_iters);
/* The last autotuning's measurements as a JSON array (one object per class
 * and candidate: s_max, prec, kernel, pw, ms, elements).  Copies at most
 * len-1 characters plus a terminating zero into buf; returns the full size
 * including the zero. */
size_t mhm_tune_report(mhm_ctx ctx, char* buf, size_t len);

/* Batching: capture the whole mhm_local_batch_run of this batch (binning,
 * one persistent launch per size class, one after another (or on forked
 * streams with MHM_OPT_CONCURRENT_CLASSES), FP64 fallback
 * passes) into a HIP graph that owns its own workspace.  The batch arrays
 * and outputs are bound at capture; their contents may change between
 * launches, their addresses and the host fields of the batch may not.
 * mhm_graph_launch enqueues one replay on the context's stream.  Contract
 * and results as mhm_local_batch_run. */
mhm_status mhm_graph_create(mhm_ctx ctx, const mhm_batch* batch, mhm_prec prec,
                            double* X, double* M, double* E, double* B, double* F,
                            int32_t* info, int32_t* ir_iters, int max_iters,
                            mhm_graph* graph);
mhm_status mhm_graph_launch(mhm_graph graph);
/* Waits for the context's stream, then frees the graph and its workspace. */
mhm_status mhm_graph_destroy(mhm_graph graph);

/* ------------------------------------------------------------- serving
 * A request loop for local problems that arrive one at a time (the
 * solveLocalProblem calls of Algorithm 1 issued as a stream).  A worker
 * thread keeps up to in_flight launches on the device, each on its own
 * stream with its own context; a free launch slot takes every queued
 * request that fits (continuous batching, arrival order) and runs them as
 * one ragged mhm_local_batch_run_cached.  Factors of keyed requests stay in
 * a device LRU cache, so a repeated key solves only its new right-hand sides
 * (any l).  All device memory of the server (slot buffers, an upper bound of
 * the workspaces, the factor arena) fits in hbm_budget; a request whose
 * factor does not fit after evicting every unpinned factor waits until
 * running launches finish. */
typedef struct mhm_server_s* mhm_server;

typedef struct {
  int32_t prec;               /* mhm_prec of every request                     */
  int32_t max_iters;          /* refinement step limit (MHM_FP32_IR)           */
  int32_t max_batch;          /* requests per launch, 1..65536                 */
  int32_t in_flight;          /* launches on the device at once, 1..8          */
  int32_t s_max;              /* largest s accepted, <= 48                     */
  int32_t l_max;              /* largest l accepted, <= MHM_L_LIMIT            */
  int32_t reuse;              /* nonzero: keep factors of keyed requests       */
  int32_t reserved;
  uint64_t hbm_budget;        /* device bytes the server may hold              */
  uint64_t factor_cache_max;  /* cap on the factor arena (0: rest of budget)   */
} mhm_server_config;

typedef struct {
  uint64_t key_hi, key_lo;    /* content key of (geometry, s, kappa); 0,0 = never
                                 reused.  Equal keys must mean equal data.    */
  int32_t s, l;
  double vert[6];             /* as in mhm_batch                               */
  int8_t sigma[3], flip[3];
  int8_t pad[2];
  const double* kappa;        /* HOST [s*s], copied by mhm_server_submit       */
  const double* f;            /* HOST [s*s]                                    */
  double t_arrival;           /* caller's arrival time, mhm_server_now() clock */
} mhm_request;

typedef struct {
  uint64_t ticket;
  int32_t info, ir_iters;     /* as in mhm_local_batch_run                     */
  int32_t cache_hit;          /* the factor came from the cache                */
  int32_t s, l, n, r;
  int32_t pad;
  double t_arrival, t_done;   /* t_done: results on the host (server clock)    */
  const double* X;            /* HOST n x r column-major; M NI x NI, E, B NI   */
  const double* M;            /* (NI = r - 1); valid until the next poll       */
  const double* E;
  const double* B;
  double F;
} mhm_result;

typedef struct {
  int64_t submitted, completed, launches, cache_hits, ir_fallbacks, errors;
  int64_t queued, max_batch_seen, cache_entries, cache_bytes, cache_evictions;
  int64_t arena_bytes, fixed_bytes;
} mhm_server_stats;

double mhm_server_now(void);   /* seconds on the server's monotonic clock */
mhm_status mhm_server_create(int device, const mhm_server_config* cfg, mhm_server* server);
/* Queue n requests; tickets[k] (may be NULL) identifies request k's result. */
mhm_status mhm_server_submit(mhm_server server, const mhm_request* reqs, int n, uint64_t* tickets);
/* Move up to max finished results into out; returns how many (-1 on a bad
 * argument).  Result arrays stay valid until the next poll. */
int mhm_server_poll(mhm_server server, mhm_result* out, int max);
mhm_status mhm_server_stats_get(mhm_server server, mhm_server_stats* stats);
const char* mhm_server_last_error(mhm_server server);
/* Stops the worker (queued requests are dropped), frees everything. */
mhm_status mhm_server_destroy(mhm_server server);

#ifdef __cplusplus
}
#endif

#endif /* MHM_H */
