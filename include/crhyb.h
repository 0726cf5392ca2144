/*
 * crhyb.h - hybridised Crouzeix-Raviart Stokes / Navier-Stokes solve on AMD gfx950.
 *
 * Implements the "hybrid method" of Chenier & Eymard, "Exact pressure
 * elimination for the Crouzeix-Raviart scheme applied to the Stokes and
 * Navier-Stokes problems" (arXiv 2101.03777), Section 3.2:
 *   1. element-wise elimination of the coupled system [A D^t; D 0][U;P] = [R;0]
 *      (Section 3.1, eq. syslin) into G W = S on d unknowns per interior face;
 *   2. Krylov solution of G W = S;
 *   3. element-wise recovery of U and P.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Every function returns cr_status (CR_OK = 0); no C++ exception crosses the ABI.
 *    On failure cr_last_error() returns a message for the calling thread.
 *  - Mesh arrays are HOST pointers, borrowed for the duration of the call and copied.
 *  - Field arrays passed to cr_eliminate / cr_update_rhs and the outputs of
 *    cr_recover are DEVICE pointers (memory of the device the system lives on,
 *    e.g. torch tensors), borrowed for the duration of the enqueued work.
 *  - All device work is enqueued on the HIP stream given to cr_assemble (NULL =
 *    the null stream).  Calls that return host scalars (cr_solve, the exports)
 *    synchronise that stream; the others are asynchronous.
 *  - Device memory of a system comes from the cr_allocator given to cr_assemble
 *    (NULL = hipMalloc/hipFree) and is released by cr_destroy.
 *  - A cr_system is not thread-safe; distinct systems are independent.
 *  - Canonical layouts (never the internal renumbering):
 *      interior faces  ordered lexicographically by their sorted vertex-id tuple
 *                      (cr_interior_faces returns them);
 *      U, W, u_prev, u_lin  [n_int_faces][dim] doubles (face-major);
 *      P, f_mean       in the caller's element order: P [n_elements],
 *                      f_mean [n_elements][dim]; P[k0] = 0 (Section 2, Q_{h,0}).
 *  - Sign choice C_K (eq. propc): +1 on the lower-index element of a face, -1 on
 *    the other; W depends on it, U and P do not.
 */
#ifndef CRHYB_H
#define CRHYB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CR_OK = 0,
  CR_E_INVAL = -1,      /* bad argument or call order */
  CR_E_NOMEM = -2,      /* allocation failed */
  CR_E_MESH = -3,       /* face shared by > 2 elements, zero-volume element, element without interior face */
  CR_E_SINGULAR = -4,   /* B_K <= 0 (Section 3.2 item 4), singular local matrix, zero diagonal of G */
  CR_E_NOCONV = -5,     /* iteration limit reached; best iterate kept, info filled */
  CR_E_BREAKDOWN = -6,  /* Krylov breakdown (p^t G p <= 0 in CG, zero rho/omega in BiCGStab) */
  CR_E_NONFINITE = -7,  /* NaN/Inf in an input or a solver scalar */
  CR_E_DEVICE = -8      /* HIP runtime error */
} cr_status;

/* problem kinds (cr_params.problem) */
enum { CR_STOKES = 0, CR_NS_NEWTON = 1 };
/* face numbering (cr_params.renumber) */
enum { CR_RCM = 0, CR_NATURAL = 1 };
/* Krylov methods (cr_solve_opts.method): CG for symmetric positive definite G;
 * MINRES for symmetric G, definite or not (steady Stokes); for non-symmetric G:
 * BiCGStab, and BiCGStab(2) (two BiCG steps and a degree-two minimal-residual
 * step per iteration, four products with G; it converges on the strongly
 * indefinite G of the steady Newton step where BiCGStab breaks down). */
enum { CR_PCG = 0, CR_BICGSTAB = 1, CR_BICGSTAB2 = 2, CR_MINRES = 3 };
/* arithmetic of the Krylov iterations (cr_solve_opts.precision) */
enum { CR_FP64 = 0, CR_FP32_IR = 1 };
/* how the Krylov iterations apply G (cr_solve_opts.operator_form):
 * CR_OP_AUTO: element factors for CG on transient Stokes, assembled rows otherwise;
 * CR_OP_ASSEMBLED: the assembled block rows of G (Section 3.2 item 5);
 * CR_OP_ELEMENT: G = sum_K H_K G_K H_K^t applied from the element factors of
 *   G_K (Section 3.2 items 4-5), without reading the assembled G (CG on
 *   transient Stokes only). */
enum { CR_OP_AUTO = 0, CR_OP_ASSEMBLED = 1, CR_OP_ELEMENT = 2 };
/* preconditioning (cr_solve_opts.precond).  Every method runs on the Jacobi-
 * scaled system Ds G Ds, one scale per face (Ds_f = (mean over the d components
 * of |diag G|)^{-1/2}; the paper only asks for a Krylov method, Section 3.2
 * items 6-7).  CG with the element form adds an additive aggregate coarse
 * correction M^-1 = I + Z E^-1 Z^t (one column per aggregate: the null vector
 * of the gauge-shifted G restricted to the aggregate's faces):
 * CR_PC_DEFAULT: Jacobi scaling, plus the coarse correction where the mesh has
 *   aggregates (transient Stokes meshes of at least 512 elements in 2D, 1024 in 3D);
 * CR_PC_JACOBI: Jacobi scaling only;
 * CR_PC_COARSE: the coarse correction is required: CR_E_INVAL where it does
 *   not exist (no aggregates, or another method or operator form). */
enum { CR_PC_DEFAULT = 0, CR_PC_JACOBI = 1, CR_PC_COARSE = 2 };

typedef struct cr_system cr_system;

/* Device allocator used for every buffer a system owns.  alloc returns NULL on
 * failure.  stream is the system's hipStream_t. */
typedef struct {
  void* (*alloc)(size_t bytes, void* ctx, void* stream);
  void (*release)(void* ptr, void* ctx, void* stream);
  void* ctx;
} cr_allocator;

/* A simplicial mesh without hanging nodes (Section 2 item 1): triangles (dim 2)
 * or tetrahedra (dim 3), any orientation. */
typedef struct {
  int32_t dim;
  int64_t n_vertices;
  const double* coords;          /* host [n_vertices][dim] */
  int64_t n_elements;
  const int32_t* elem_vertices;  /* host [n_elements][dim+1] */
} cr_mesh_desc;

/* Coefficients of the strong form (Section 2): mu = 1/dt (transient) or 0
 * (steady), nu = 1/Re > 0.  k0 is the element whose pressure is pinned to 0
 * (Section 2 item 5).  problem = CR_NS_NEWTON selects the Newton linearisation
 * of the convection form b_h (eq. defbh) about u_lin (2D and 3D; in 3D the 12 x 12
 * local matrices of the elimination are formed and inverted in LDS). */
typedef struct {
  double mu, nu;
  int32_t k0;
  int32_t problem;
  int32_t renumber;
  /* mu = 0 only: E_K = -lambda_K I on the elements of M1 (Section 3.2 item 7)
   * with lambda_K = lambda_scale * ||A_K||_inf over the interior rows; the
   * paper asks for lambda above every eigenvalue modulus of A_K, which the
   * infinity norm bounds, so lambda_scale must exceed 1.  <= 0: 2. */
  double lambda_scale;
} cr_params;

/* Step a0: face topology, renumbering and upload of the mesh.
 * Builds interior/exterior faces, element<->face tables, the sign choice C_K,
 * reverse Cuthill-McKee face order (or natural), element order, and for mu = 0
 * the element partition M1/M2 of Section 3.2 item 7 (greedy maximal independent
 * set in caller order).  Host work plus host-to-device copies on hip_stream.
 * Errors: CR_E_INVAL (dim not 2/3, nu <= 0, mu < 0, k0 out of range, 0 < lambda_scale <= 1),
 * CR_E_MESH (see above), CR_E_NOMEM, CR_E_DEVICE.  *out is NULL on error. */
cr_status cr_assemble(const cr_mesh_desc* mesh, const cr_params* params,
                      const cr_allocator* alloc, void* hip_stream, cr_system** out);

/* cr_assemble in two parts, for callers that build systems on a host thread
 * while other systems keep the device busy (Section 2 item 1, as cr_assemble).
 * cr_prepare is the host part only: checks, topology, renumbering, the element
 * and face tables in internal order (and, for transient Stokes, the aggregates
 * of the coarse correction); it makes no HIP call and may run on any thread,
 * concurrently with device work of other systems.  *out is NULL on error;
 * errors as cr_assemble except CR_E_DEVICE.
 * cr_assemble_prepared is the device part: allocation and upload on hip_stream;
 * it always consumes prep (also on error), and *out is what cr_assemble would
 * return for the same mesh and parameters.
 * cr_prepared_destroy frees a prepared mesh that is not assembled (NULL: no-op). */
typedef struct cr_prepared cr_prepared;
cr_status cr_prepare(const cr_mesh_desc* mesh, const cr_params* params, cr_prepared** out);
cr_status cr_assemble_prepared(cr_prepared* prep, const cr_allocator* alloc, void* hip_stream, cr_system** out);
void cr_prepared_destroy(cr_prepared* prep);

/* Steps a1-a3: element-wise elimination (Section 3.2 items 4-5) and assembly of
 * G (same block stencil as A) and S.
 * f_mean: device [n_elements][dim], element means of the force (eq. defrhs).
 * u_prev: device [n_int_faces][dim] previous time-step velocity, or NULL; it
 *         enters R_K through the lumped mass mu |K|/(d+1) U^{n-1}.
 * u_lin:  device [n_int_faces][dim] Newton linearisation velocity (CR_NS_NEWTON
 *         only, required there), else NULL.
 * Synchronises the stream to report element errors.
 * Errors: CR_E_SINGULAR (element id in the message), CR_E_NONFINITE, CR_E_INVAL. */
cr_status cr_eliminate(cr_system* sys, const double* f_mean, const double* u_prev,
                       const double* u_lin);

/* Step a6: new right-hand side with the same G (constant time step, Stokes only).
 * In the transient problem of Section 2 the force f carries the velocity of the
 * previous time step, and R_K is its face moment (eq. defrhs): only R_K and
 * s_K change from step to step, G does not (Section 3.2 items 4-5).  Recomputes
 * R_K and s_K from the stored element factors and re-gathers S.  Same argument
 * meaning as cr_eliminate.  Asynchronous.  Errors: CR_E_INVAL (NULL system or
 * f_mean, before cr_eliminate, Navier-Stokes). */
cr_status cr_update_rhs(cr_system* sys, const double* f_mean, const double* u_prev);

typedef struct {
  int32_t method;      /* CR_PCG, CR_MINRES, CR_BICGSTAB or CR_BICGSTAB2 */
  int32_t precision;   /* CR_FP64, or CR_FP32_IR: FP32 Krylov inside FP64 iterative refinement */
  double tol;          /* stop when ||S - G W||_2 <= tol ||S||_2, residual recomputed in FP64 */
  double inner_tol;    /* factor by which the recursive residual falls between FP64 residual
                          replacements (reliable updates); <= 0: automatic (0.1 for FP32
                          iterations and for CG, none otherwise) */
  int32_t maxit;       /* cap on the total number of Krylov iterations */
  int32_t max_outer;   /* cap on refinement passes */
  int32_t check_every; /* iterations per convergence poll (rounded up to even); <= 0: automatic */
  int32_t use_graph;   /* 1: replay the iteration block as a captured hipGraph */
  int32_t warm_start;  /* 1: start from the resident W of the previous solve, 0: from W = 0 */
  int32_t operator_form; /* CR_OP_AUTO, CR_OP_ASSEMBLED or CR_OP_ELEMENT */
  int32_t precond;     /* CR_PC_DEFAULT, CR_PC_JACOBI or CR_PC_COARSE (below) */
  const double* w0;    /* device [n_int_faces][dim] initial W (canonical), or NULL; when
                          given it replaces the resident W and the solve starts from it
                          (warm_start is then implied).  Ignored by cr_batch_add and
                          cr_coupled_solve. */
} cr_solve_opts;

typedef struct {
  int32_t iters;        /* Krylov iterations executed */
  int32_t outer_iters;  /* refinement passes (residual evaluations) */
  double rel_residual;  /* ||S - G W|| / ||S|| in FP64 for the returned W */
  double t_solve_ms;    /* wall time of the call */
  int32_t reason;       /* 1 converged, 3 iteration limit, 4 breakdown, 5 non-finite */
  int32_t fp32_iters;   /* iterations run in FP32 (CR_FP32_IR) */
  int32_t fp64_fallback;/* 1 if CR_FP32_IR stalled and finished with FP64 iterations */
} cr_solve_info;

/* Step a4: Krylov solve of G W = S; W stays resident on the device.
 * PCG applies when mu > 0 and the problem is Stokes (G symmetric positive
 * definite, Section 3.2 item 6); MINRES for symmetric indefinite G (steady
 * Stokes, Section 3.2 item 7), in refinement passes that each restart from the
 * FP64 residual; BiCGStab or BiCGStab(2) otherwise.  Jacobi
 * preconditioning is applied as the symmetric scaling Ds G Ds with one scale
 * per face,
 * Ds_f = (mean over the d components of |diag G|)^{-1/2}.
 * CG with the element form adds an aggregate coarse correction (one column per
 * aggregate: the null vector of the gauge-shifted G restricted to the
 * aggregate's faces; opts.precond); it changes the iterations, not the solution.
 * CR_FP32_IR runs the Krylov recurrences in FP32 with FP64 residual
 * replacements; if the FP32 iterations stop reducing the FP64 residual, the
 * remaining iterations run in FP64 (reported in cr_solve_info.fp64_fallback).
 * Synchronises.  Errors: CR_E_NOCONV, CR_E_BREAKDOWN, CR_E_NONFINITE, CR_E_INVAL
 * (before cr_eliminate).  info may be NULL. */
cr_status cr_solve(cr_system* sys, const cr_solve_opts* opts, cr_solve_info* info);

/* Step a5: recovery (Section 3.2 items 2 and 4):
 *   P_K = r_K^t (R_K - C_K W_K) / B_K (K != K0), P_K0 = 0,
 *   U^_K = A^_K^{-1} (R_K - D_K P_K - C_K W_K);
 * U is the copy of the element with C = +1.
 * U: device [n_int_faces][dim] (canonical), P: device [n_elements] (caller order).
 * jump (optional, device [1] or NULL): ||C^ U^||_2, the copy mismatch, which
 * equals ||S - G W||_2.  Asynchronous. */
cr_status cr_recover(cr_system* sys, double* U, double* P, double* jump);

/* cr_recover for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): same
 * U and P (bit for bit) and the same copy mismatch up to summation order, but
 * no device allocation at all.  cr_recover keeps the second velocity copy in a
 * per-system buffer of n_int_faces*dim doubles allocated on first use; this
 * variant recomputes the non-owner copies in a second element pass and keeps
 * only one partial sum per 128 elements, in a static device array of 256 KiB
 * (32768 doubles) that each device holds until the process ends.
 * Limit: with jump != NULL, at most 4,194,304 elements, else CR_E_INVAL
 * (message names the limit); with jump == NULL no limit and no scratch.
 * Every call on one device shares that device's array: calls that overlap on
 * one device (other streams, other threads) race on it.  Each call writes
 * every partial it reads, so nothing needs clearing between calls.
 * Asynchronous; arguments, layouts and other errors as cr_recover. */
cr_status cr_recover_noalloc(cr_system* sys, double* U, double* P, double* jump);

/* Sizes of the system: interior faces (Section 2 item 1), structural non-zeros
 * of G (d x d blocks of the stencil of A, Section 3.2 item 5: a diagonal block
 * per face and one block per ordered pair of faces of an element), non-zeros of
 * the coupled matrix [A D^t; D 0] of eq. syslin.  Any output pointer may be
 * NULL.  Host only, no device work.  Errors: CR_E_INVAL (NULL system). */
cr_status cr_query_sizes(const cr_system* sys, int64_t* n_int_faces, int64_t* nnz_G,
                         int64_t* nnz_coupled);

/* Host copy of the hybridised system G W = S of Section 3.2 item 5 (G =
 * sum_K H_K G_K H_K^t, S = sum_K H_K s_K), unscaled, FP64 CSR in canonical
 * face-major numbering (row dim*face + component), structural entries of the
 * stencil (zeros kept), columns sorted within a row.  Caller-owned host
 * buffers sized from cr_query_sizes: rowptr [n+1], col [nnz_G], val [nnz_G],
 * S [n] with n = dim * n_int_faces.  Synchronises.  Errors: CR_E_INVAL (NULL
 * system or buffer, before cr_eliminate), CR_E_DEVICE. */
cr_status cr_export_G(const cr_system* sys, int64_t* rowptr, int32_t* col, double* val, double* S);

/* Host copy of the coupled system of Section 3.1 (eq. syslin), Stokes only:
 * [A D^t; D 0] as FP64 CSR and its right-hand side [R; 0].  Rows and columns:
 * the velocity unknowns (canonical face, component), then one pressure per
 * element in caller order without k0 (P_k0 = 0 is not an unknown), so
 * n = dim * n_int_faces + n_elements - 1.  A = sum_K H_K (S_K (x) I_d) H_K^t,
 * D_K = -a_K (rows of K0 dropped), R = sum_K H_K R_K, columns sorted within a
 * row, nnz = nnz_coupled of cr_query_sizes (structural entries, zeros kept).
 * Buffers (host): rowptr [n+1], col [nnz], val [nnz], R [n]; any may be NULL.
 * Assembled on the device with the coupled baseline's kernels (its workspace
 * is allocated on first use); synchronises.  Errors: CR_E_INVAL (NULL system,
 * not eliminated, Navier-Stokes), CR_E_NOMEM, CR_E_DEVICE. */
cr_status cr_export_coupled(cr_system* sys, int64_t* rowptr, int32_t* col, double* val, double* R);

/* Host copy of the resident W [n_int_faces][dim] (canonical): the auxiliary
 * face unknowns of the hybrid system (Section 3.2, eq. syslinhyb), the
 * solution of G W = S after cr_solve.  Synchronises. */
cr_status cr_export_W(const cr_system* sys, double* W);

/* The resident W (as cr_export_W) into a caller-owned DEVICE array
 * [n_int_faces][dim] (canonical), on the system's stream, asynchronous: e.g.
 * the initial guess (cr_solve_opts.w0) of the next solve after a new
 * cr_eliminate, which starts from W = 0 otherwise (a Newton iteration or a time
 * step whose W changes little).  Zero before any solve.  Errors: CR_E_INVAL
 * (NULL system or buffer, not eliminated), CR_E_DEVICE. */
cr_status cr_export_W_device(cr_system* sys, double* W);

/* Set the resident W (Section 3.2, eq. syslinhyb) from a host array
 * [n_int_faces][dim] (canonical), e.g. to recover U and P (Section 3.2 items
 * 2 and 4) from a W computed elsewhere.  Synchronises. */
cr_status cr_import_W(cr_system* sys, const double* W);

/* Host copy of the interior faces of Section 2 item 1 (faces shared by two
 * elements) as sorted vertex ids, [n_int_faces][dim] int32, in the canonical
 * order (lexicographic in those ids) that U, W, u_prev and u_lin use.
 * Caller-owned host buffer.  Errors: CR_E_INVAL (NULL system or buffer). */
cr_status cr_interior_faces(const cr_system* sys, int32_t* face_vertices);

/* Exterior faces of the mesh (faces of one element, Section 2 item 1) as
 * sorted vertex ids [n_bnd_faces][dim] int32, lexicographic in those ids: the
 * order of the boundary data of cr_set_boundary.  face_vertices may be NULL
 * (count only).  Host only.  Errors: CR_E_INVAL (NULL system). */
cr_status cr_boundary_faces(const cr_system* sys, int64_t* n_bnd_faces, int32_t* face_vertices);

/* Non-homogeneous Dirichlet data, as in the tests of Section 4 (the exact
 * velocity imposed on the boundary): g is a DEVICE array [n_bnd_faces][dim]
 * of face-mean velocities on the exterior faces (cr_boundary_faces order),
 * copied on the system's stream; NULL returns to homogeneous data.  It takes
 * effect at the next cr_eliminate / cr_update_rhs: the columns of the exterior
 * faces of A_K times the data leave the velocity rows of R_K, the divergence
 * row of K reads D_K^t U_K = e_K with e_K = -D_K[exterior] . g, and the
 * elimination and recovery of Section 3.2 items 2 and 4 carry e_K (P_K =
 * (r_K^t (R_K - C_K W_K) - e_K) / B_K).  For the Newton step the exterior faces
 * of the linearisation velocity take the data too.  The divergence row of K0
 * is not imposed, so it absorbs the net flux of the data (zero for exact data
 * of a divergence-free field).  In the element-form CG (whose gauge-shifted
 * system keeps a divergence row at K0) that row takes up the net flux, so the
 * element form and its coarse correction serve boundary data too.  Errors:
 * CR_E_INVAL (NULL system, no exterior face), CR_E_NOMEM, CR_E_DEVICE. */
cr_status cr_set_boundary(cr_system* sys, const double* g);

/* Host-only topology (step a0 without any device work), for inspection:
 * n_int_faces, the internal position of every canonical face (perm [n_int_faces],
 * may be NULL), the half bandwidth of the face adjacency in internal order and in
 * canonical order, and the M1 flag of every element (m1 [n_elements], may be
 * NULL; all zero when mu > 0). */
cr_status cr_topology(const cr_mesh_desc* mesh, const cr_params* params, int64_t* n_int_faces,
                      int32_t* perm, int64_t* bandwidth_internal, int64_t* bandwidth_canonical,
                      int32_t* m1);

/* Baseline: a Krylov solve of the original coupled system of Section 3.1
 * (eq. syslin) [A D^t; D 0][U; P] = [R; 0] on the same GPU, FP64, without the
 * hybridisation, preconditioned by the positive diagonal
 * diag|A| (+) diag(D diag|A|^{-1} D^t).  Stokes (symmetric): MINRES on the
 * preconditioned system.  Newton step (non-symmetric A, Jacobian of the
 * convection form included): BiCGStab on the system scaled symmetrically by
 * the square root of that diagonal, in passes that restart from the true
 * residual.  Stops on the coupled residual ||[R;0] - M [U;P]|| <= tol ||R||;
 * opts->tol, maxit, max_outer, check_every are used, the other fields ignored.  U, P as in cr_recover (device, caller-owned).
 * Its workspace (about 12 vectors of the coupled size) is allocated on first
 * use.  Synchronises.  Errors: CR_E_NOCONV (iteration limit; best iterate
 * written), CR_E_BREAKDOWN, CR_E_NONFINITE, CR_E_INVAL (before cr_eliminate). */
cr_status cr_coupled_solve(cr_system* sys, const cr_solve_opts* opts, cr_solve_info* info,
                           double* U, double* P);

/* Average device time of the dominant Krylov kernel (the product with G fused
 * with the CG direction update) over reps launches on the system's stream, measured with
 * HIP events, on scratch copies of the state (the resident solution is
 * untouched; the coarse-correction vectors of the last solve are not kept).
 * Back-to-back launches, except with the coarse correction, where the element
 * kernel runs inside the iteration sequence with events attached to each of its
 * launches.  precision and operator_form as in cr_solve_opts.
 * Also returns the algorithmic bytes one launch moves, each datum counted once:
 * assembled form: values and column indices of G, the gathered input vector,
 * the fused vector reads and writes; element form: element factors, gather
 * indices and flags, r and the previous direction at the faces, the element
 * contributions, the new direction (2D; in 3D the face kernel stores it), and
 * with the coarse correction the face aggregate and Z column read by the
 * elements on aggregate boundaries.  Synchronises.
 * Errors: CR_E_INVAL (not eliminated, reps < 1, element form unavailable). */
cr_status cr_time_spmv(cr_system* sys, int32_t precision, int32_t operator_form, int32_t reps,
                       double* avg_ms, double* bytes_per_launch);

/* Step a7 (serving): batched CG solves of many resident transient-Stokes
 * systems.  Each kernel launch of a batch covers the rows of every active
 * system (a block-diagonal batch, one grid); each system keeps its own partial
 * sums, scalars and stop flag, so its iterates are bitwise those of cr_solve
 * with the same options.  Systems join with cr_batch_add (their right-hand
 * side set by cr_eliminate / cr_update_rhs) and leave when finished; their
 * FP64 residual replacements are serviced between iteration blocks.  All
 * systems of a batch live on the batch's stream and have the same dimension.
 * Systems of a batch use one operator form (the element form for CG on
 * transient Stokes by default).  Not thread-safe.  The batch owns only its own
 * small tables (hipMalloc) and the captured graph. */
typedef struct cr_batch cr_batch;

/* max_systems: capacity (1..4096). */
cr_status cr_batch_create(void* hip_stream, int32_t max_systems, cr_batch** out);

/* Start solving sys's current S (method CR_PCG; opts as for cr_solve, use_graph
 * and check_every ignored).  Asynchronous.  Errors: CR_E_INVAL (system not
 * eliminated, other stream or dimension, not transient Stokes, already in the
 * batch), CR_E_NOMEM (batch full). */
cr_status cr_batch_add(cr_batch* b, cr_system* sys, const cr_solve_opts* opts);

/* Run n_iters iterations (rounded up to even) of every active system in shared
 * launches, then service stops (replacement, restart, FP64 fallback, finish).
 * The iteration block is captured as a hipGraph once per launch shape (block
 * counts of the active systems and n_iters) and replayed; joins and leaves
 * that keep the shape only rewrite the device tables it reads.
 * *n_finished = systems that finished in this call.  Synchronises. */
cr_status cr_batch_advance(cr_batch* b, int32_t n_iters, int32_t* n_finished);

/* Pop one finished system (FIFO): *sys = NULL if none.  info and status (the
 * cr_status cr_solve would have returned) may be NULL.  W is resident in sys. */
cr_status cr_batch_pop(cr_batch* b, cr_system** sys, cr_solve_info* info, int32_t* status);

/* Number of active and of finished-but-not-popped systems. */
cr_status cr_batch_count(const cr_batch* b, int32_t* n_active, int32_t* n_finished);

/* Releases the batch's tables and graphs (not its systems).  NULL is a no-op. */
void cr_batch_destroy(cr_batch* b);

/* Waits for the system's stream, then releases every device buffer of the
 * system through its allocator.  NULL is a no-op. */
void cr_destroy(cr_system* sys);

/* Message of the last failing call on this thread ("" if none). */
const char* cr_last_error(void);

/* Library version string. */
const char* cr_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CRHYB_H */
