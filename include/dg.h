/*
 * dg.h -- C ABI of the matrix-free SIPG Laplacian library for MI355X (gfx950).
 *
 * The operator is the symmetric interior penalty discretisation of
 * -div(c grad u) from Kronbichler & Kormann, "Fast matrix-free evaluation of
 * discontinuous Galerkin finite element operators" (arXiv 1711.03590), Sec. 2,
 * Eq. (2), evaluated as the matrix-vector product y = A u of Sec. 2, Eq. (3)
 * by the cell/face integration loop of Algorithm 1 with sum factorisation
 * (Sec. 2, Eqs. (6)-(7); Sec. 3.3, Eq. (8)).
 *
 * Discretisation fixed by this library:
 *   - mesh: structured brick of ncell[0] x ncell[1] x ncell[2] hexahedra on
 *     the box [lo, hi], optionally deformed by the sine map below;
 *   - basis: Lagrange polynomials of degree k (1 <= k <= 8) on the k+1
 *     Gauss-Lobatto points per direction; quadrature: (k+1)-point
 *     Gauss-Legendre per direction on cells and faces;
 *   - penalty tau = (k+1)^2 / h_a, h_a the unmapped cell size normal to the face;
 *   - Dirichlet faces by the mirror principle u+ = -u-, grad u+ = grad u-
 *     (homogeneous data); Neumann faces (homogeneous) contribute nothing;
 *   - the coefficient c multiplies the cell term and all three face terms.
 *
 * DoF order (all vectors): global = cell * n^3 + i1 + n*i2 + n^2*i3 with
 * n = k + 1 and cell = cx + ncell[0]*(cy + ncell[1]*cz), i.e. cell-contiguous
 * blocks in x-fastest order.
 *
 * Conventions for every call:
 *   - every function returns dg_status; DG_OK == 0.  No exception crosses the
 *     ABI.  dg_last_error() returns a message for the last failure on the
 *     calling thread (empty string if none).
 *   - "stream" is a hipStream_t passed as void* (NULL = the null stream).
 *     Device work is enqueued asynchronously on it unless stated otherwise.
 *   - vectors are dg_vec: a DEVICE pointer owned by the caller, its element
 *     type and its length.  The caller keeps them alive until the stream work
 *     that uses them has completed.
 *   - an op owns its geometry, tables and diagonal, allocated through the
 *     allocator given at setup (NULL: hipMalloc/hipFree) and released by
 *     dg_destroy.
 */
#ifndef DG_H
#define DG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DG_OK = 0,
  DG_ERR_ARG = 1,           /* invalid argument; nothing was enqueued */
  DG_ERR_OOM = 2,           /* allocation failed */
  DG_ERR_HIP = 3,           /* a HIP runtime call failed */
  DG_ERR_UNSUPPORTED = 4,   /* valid but not supported (e.g. degree > 8) */
  DG_ERR_NOT_CONVERGED = 5  /* solver hit its iteration limit; stats are filled */
} dg_status;

typedef enum { DG_F64 = 0, DG_F32 = 1 } dg_dtype;
/* DG_BC_GHOST marks a side where the brick is one partition of a larger
 * mesh: its faces there are interior faces of the larger mesh, and the
 * neighbour's side of them arrives as face traces (see dg_face_traces and
 * dg_apply_ghost).  SIPG ops only. */
typedef enum { DG_BC_DIRICHLET = 0, DG_BC_NEUMANN = 1, DG_BC_GHOST = 2 } dg_bc;

/* Structured brick; bc order x-, x+, y-, y+, z-, z+ (side f = 2a + s: the
 * side of direction a at its low (s = 0) or high (s = 1) end). */
typedef struct {
  int32_t ncell[3];
  double lo[3], hi[3];
  int32_t bc[6];
} dg_mesh;

/* DG_MAP_SINE: x_i = X_i + amplitude * sin(2 pi X) sin(2 pi Y) sin(2 pi Z)
 * for every component i, X the unmapped point.  Jacobians are precomputed at
 * every cell and face quadrature point (inverse Jacobian and determinant:
 * variant G3 of Sec. 5; faces store the normal times inverse Jacobian of
 * Design Choice 5).  DG_MAP_AFFINE stores no geometry per point (the
 * constant-Jacobian compression of Sec. 5). */
typedef enum { DG_MAP_AFFINE = 0, DG_MAP_SINE = 1 } dg_map;
/* What a curved map stores per cell quadrature point (Sec. 5):
 * DG_STORE_JACOBIAN  the inverse Jacobian and c det J w, 10 values (G3);
 * DG_STORE_MERGED    the symmetric effective coefficient
 *                    c det J w J^{-1} J^{-T} of the Laplacian, 6 values (G4);
 * DG_STORE_MIXED     G3 for the FP64 data and G4 for the FP32 data: FP64
 *                    applies (the residuals of mixed-precision refinement)
 *                    see the stored Jacobians, FP32 applies (the inner
 *                    solver) the cheaper merged coefficient.
 * These give the same operator up to rounding.
 * DG_STORE_POSITIONS the physical quadrature-point positions (relative to
 *                    the cell's unmapped corner) and c, 4 values (G2): the
 *                    kernel takes the cell Jacobian as the collocation
 *                    derivative of the positions, i.e. the Jacobian of the
 *                    degree-k interpolant of the map through the Gauss points.
 *                    A slightly different operator (equal on affine maps,
 *                    converging to the others at order k in the Jacobian).
 * Faces store j = J^{-1} n and c ds in every case.  Ignored for
 * DG_MAP_AFFINE. */
typedef enum { DG_STORE_JACOBIAN = 0, DG_STORE_MERGED = 1, DG_STORE_MIXED = 2, DG_STORE_POSITIONS = 3 } dg_storage;
typedef struct {
  dg_map map;
  double amplitude;
  dg_storage storage;
} dg_geometry;

/* DG_COEF_CONST: c = value.  DG_COEF_SINCOS: c = 1 + 0.5 sin(pi x) cos(pi y) z
 * at the physical point.  A variable coefficient is folded into the stored
 * quadrature factors (c * det J * w on cells, c * ds on faces). */
typedef enum { DG_COEF_CONST = 0, DG_COEF_SINCOS = 1 } dg_coef_kind;
typedef struct {
  dg_coef_kind kind;
  double value;
} dg_coefficient;

/* Device allocator callback pair; ctx is passed through unchanged. */
typedef struct {
  void *(*alloc)(size_t bytes, void *ctx);
  void (*free)(void *ptr, void *ctx);
  void *ctx;
} dg_allocator;

typedef struct {
  void *data;     /* device pointer, caller-owned */
  dg_dtype dtype;
  int64_t n;      /* number of elements */
} dg_vec;

typedef struct dg_op dg_op; /* opaque, library-owned */

/* Precision mask for dg_setup / dg_footprint. */
#define DG_PREC_F64 1u
#define DG_PREC_F32 2u

/* Bytes of device memory dg_setup will allocate for this problem: the stored
 * cell and face geometry and the Jacobi diagonal of every enabled precision
 * (solver workspace, which dg_cg_solve and the batch allocate per call or per
 * request, is not included).  Pure host computation. */
dg_status dg_footprint(const dg_mesh *mesh, int degree, const dg_geometry *geom,
                       const dg_coefficient *coef, unsigned precisions, size_t *bytes);

/* Builds the operator: evaluates the geometry at all quadrature points on the
 * device (enqueued on stream; the op is usable by later work on the same
 * stream) and computes the Jacobi diagonal.  The mesh, degree, geometry and
 * coefficient are the problem statement of Sec. 2 (Eq. (2) with the mapping of
 * Eq. (4)).  precisions selects which of FP64 / FP32 data to build. */
dg_status dg_setup(const dg_mesh *mesh, int degree, const dg_geometry *geom,
                   const dg_coefficient *coef, unsigned precisions, const dg_allocator *alloc,
                   void *stream, dg_op **out);

/* Polynomial basis of the SIPG operator.  Both span the tensor-product
 * polynomials of degree k on each cell, so the discrete solution is the same;
 * A changes by the cell-wise change of basis.
 * DG_BASIS_NODAL: Lagrange polynomials on the k+1 Gauss-Lobatto points (the
 *   dg_setup default; DoF = value at a node).
 * DG_BASIS_HERMITE: a Hermite-like basis (k >= 3) in the sense of Sec. 3 and
 *   Sec. 4.4: the 1D functions are dual to the functionals
 *   u(0), s u'(0), u(x_2), ..., u(x_{k-2}), -s u'(1), u(1) with x_m the
 *   Gauss-Lobatto points and s = x_1, so that a face value needs one and a
 *   face derivative one more coefficient per normal line (2 (k+1)^2 of a
 *   neighbour's (k+1)^3 per face). */
typedef enum { DG_BASIS_NODAL = 0, DG_BASIS_HERMITE = 1 } dg_basis;

/* dg_setup in the given basis.  DG_ERR_ARG for an unknown basis or
 * DG_BASIS_HERMITE below degree 3.  The basis does not change the device
 * footprint: dg_footprint applies as it is.  Every call that takes the op (apply,
 * diagonal, right-hand side, error, CG) works in that basis; dg_batch_admit
 * returns DG_ERR_UNSUPPORTED for a Hermite op. */
dg_status dg_setup_basis(const dg_mesh *mesh, int degree, dg_basis basis, const dg_geometry *geom,
                         const dg_coefficient *coef, unsigned precisions, const dg_allocator *alloc, void *stream,
                         dg_op **out);

/* The 1D tables of a basis as the kernels use them, for degree k (n = k+1),
 * written row-major into out: S[q][j] = phi_j(g_q) and D[q][j] = phi_j'(g_q)
 * at the n Gauss points g_q (n*n each), then phi_j(0), phi_j(1), phi_j'(0),
 * phi_j'(1) (n each).  len >= 2 n^2 + 4 n.  Pure host computation. */
dg_status dg_basis_tables(int degree, dg_basis basis, double *out, size_t len);

/* Transport velocity of the advection operator (Sec. 2, Eq. (1)).
 * DG_VEL_CONST: c = value (a constant vector).
 * DG_VEL_ROTATION: c(x) = (1/2 - y, x - 1/2, 1/4), a divergence-free
 * rotation about the unit cube's vertical axis with an upward drift
 * (value ignored). */
typedef enum { DG_VEL_CONST = 0, DG_VEL_ROTATION = 1 } dg_velocity_kind;
typedef struct {
  dg_velocity_kind kind;
  double value[3];
} dg_velocity;

/* Bytes of device memory dg_setup_advection will allocate: 3 values per cell
 * quadrature point (J^{-1} c det J w) and 1 per face point ((c . n) ds for
 * the +e_a orientation of the face), in each enabled precision. */
dg_status dg_footprint_advection(const dg_mesh *mesh, int degree, const dg_geometry *geom,
                                 const dg_velocity *vel, unsigned precisions, size_t *bytes);

/* Builds the DG advection operator with the local Lax-Friedrichs (upwind)
 * flux of Sec. 2, Eq. (1), whose loop structure is Algorithm 1:
 *   y_i = -(grad phi_i, c u_h)_e + <phi_i, 1/2 (c.n)(u- + u+) + 1/2 |c.n| (u- - u+)>_{de}.
 * Boundary faces take u+ = -u- (mirror, homogeneous inflow data) where
 * mesh->bc is DG_BC_DIRICHLET and u+ = u- (outflow) where it is
 * DG_BC_NEUMANN; a DG_BC_GHOST side is DG_ERR_UNSUPPORTED.  geom->storage is ignored.  The op works with dg_apply,
 * dg_n_dofs and dg_destroy; dg_diagonal, dg_rhs, dg_error_manufactured,
 * dg_cg_solve and dg_batch_admit return DG_ERR_UNSUPPORTED for it (the
 * operator is not symmetric). */
dg_status dg_setup_advection(const dg_mesh *mesh, int degree, const dg_geometry *geom, const dg_velocity *vel,
                             unsigned precisions, const dg_allocator *alloc, void *stream, dg_op **out);

/* Number of degrees of freedom (ncells * (k+1)^3); -1 for a NULL op. */
int64_t dg_n_dofs(const dg_op *op);

/* dst := A src (Sec. 2, Eq. (3)) for the op's operator (SIPG Laplacian or
 * advection), one fused pass over all cells: each cell computes its cell
 * integral and the own-side share of its six face integrals (the cell and
 * face loops of Algorithm 1, fused) and writes its dst block once; dst need not be
 * initialised.  src and dst must have the same dtype, which must be enabled in
 * the op, length dg_n_dofs, and must not alias: otherwise DG_ERR_ARG and nothing
 * is enqueued. */
dg_status dg_apply(dg_op *op, dg_vec src, dg_vec dst, void *stream);

/* ---------------------------------------------------------------------------
 * One partition of a larger mesh.  Sec. 2's operator couples a cell to its
 * face neighbours only through the neighbour's value and normal derivative
 * on the shared face (the S_f and D_f rows of Eq. (7) applied to the
 * neighbour's coefficients).  A partition whose side f is DG_BC_GHOST takes
 * those two quantities for every face of side f from a trace buffer that the
 * neighbouring partition computed with dg_face_traces; with the traces of
 * the same global vector, dg_apply_ghost gives the rows of the global A u
 * that the partition owns (up to the rounding of its geometry, which is
 * evaluated from its own box).
 *
 * Trace layout of side f = 2a + s, for a brick with tangential cell counts
 * (m1, m2) on that side (the two directions other than a, in increasing
 * order): (p * 2 + r) * n^2 + j, with p = c1 + m1 * c2 the cell's position
 * in the side's plane, r = 0 the value and r = 1 the reference normal
 * derivative d/dxi_a, and j = j1 + n * j2 the face node (the cell's node
 * indices along the two tangential directions).  Length 2 m1 m2 n^2.
 * ------------------------------------------------------------------------ */

/* traces := the face traces of the op's cells on side `side` (0..5) that the
 * partition across that side needs for its own ghost side (the opposite
 * side of the same direction): for side 2a + 1 the value and the xi_a
 * derivative at xi_a = 1 of every cell in the last layer, for side 2a at
 * xi_a = 0 of the first layer.  src: length dg_n_dofs; traces: the layout
 * above, same dtype as src.  Reads no geometry, so the op need not have the
 * precision enabled and the side's bc does not matter.  SIPG ops (either
 * basis); DG_ERR_UNSUPPORTED for advection ops, DG_ERR_ARG for a bad side,
 * length or dtype, or traces overlapping src; nothing is enqueued then. */
dg_status dg_face_traces(const dg_op *op, int side, dg_vec src, dg_vec traces, void *stream);

/* dst := the partition's rows of A u, like dg_apply, with every
 * DG_BC_GHOST side's neighbour values taken from ghost[f] (the trace layout
 * above, the neighbour's dg_face_traces of the opposite side, same dtype as
 * src).  ghost[f] is read only where bc[f] is DG_BC_GHOST and may be
 * {NULL, ...} elsewhere; an op with no ghost side behaves as dg_apply.
 * DG_ERR_ARG (nothing enqueued) for a missing or mis-sized trace buffer, a
 * wrong dtype, or a trace buffer that overlaps dst.  dg_apply returns
 * DG_ERR_ARG for an op that has a ghost side, and dg_cg_solve and
 * dg_batch_admit return DG_ERR_UNSUPPORTED for one (each apply would need
 * a fresh exchange).  The Jacobi diagonal (dg_diagonal), the load vector and
 * the error norms of such an op treat the ghost faces as interior faces. */
dg_status dg_apply_ghost(dg_op *op, dg_vec src, const dg_vec ghost[6], dg_vec dst, void *stream);

/* diag := diagonal of A (in diag.dtype), the Jacobi preconditioner. */
dg_status dg_diagonal(dg_op *op, dg_vec diag, void *stream);

/* b := load vector of the manufactured solution u* = sin(pi x) sin(pi y) sin(pi z):
 * b_i = sum_q f(x_q) phi_i(x_q) det J w_q with f = -div(c grad u*). FP64 only. */
dg_status dg_rhs(dg_op *op, dg_vec b, void *stream);

/* Squared L2 and broken-H1-seminorm errors of the DG function x (FP64)
 * against u*, by (k+3)-point Gauss quadrature per direction; synchronises
 * the stream and writes the two square roots to err[0], err[1]. */
dg_status dg_error_manufactured(dg_op *op, dg_vec x, void *stream, double err[2]);

/* Jacobi-preconditioned conjugate gradients for A x = b.
 *   mode 0: FP64 CG throughout.
 *   mode 1: FP32 CG (FP32 applies, FP32 accumulation) on the correction
 *           equation inside FP64 iterative refinement: r = b - A x in FP64,
 *           d ~ A^{-1} r in FP32 to rel_tol_inner, x += d in FP64; every
 *           refinement step restarts the FP32 CG.
 *   mode 2: the same split of precisions with reliable updates: one FP32 CG
 *           recurrence whose residual is replaced by the FP64 residual b - A x
 *           (and whose correction is flushed into the FP64 x) each time it has
 *           dropped by the factor rel_tol_inner (e.g. 0.3) since the last
 *           replacement; the search direction is kept across replacements.
 * Stops when ||b - A x||_2 <= rel_tol * ||b||_2 (always checked with an FP64
 * apply).  x holds the initial guess on entry.  Synchronises the stream.
 * Returns DG_ERR_NOT_CONVERGED (stats filled) when the limits are hit. */
typedef struct {
  int mode;
  double rel_tol;
  double rel_tol_inner;
  int max_iter;        /* modes 0, 2: CG iterations; mode 1: inner iterations per refinement step */
  int max_outer;       /* mode 1: refinement steps (must be >= 1 in modes 1, 2) */
  int check_every;     /* read the residual norm back every this many iterations (>= 1) */
} dg_solve_params;

typedef struct {
  int iters_inner;         /* total CG iterations (both modes) */
  int iters_outer;         /* refinement steps (modes 1, 2), 0 in FP64 mode */
  int applies_f64;
  int applies_f32;
  double final_rel_residual;
  double ms;               /* wall time of the call */
} dg_solve_stats;

dg_status dg_cg_solve(dg_op *op, dg_vec b, dg_vec x, const dg_solve_params *params,
                      dg_solve_stats *stats, void *stream);

/* Allocation-free variant of dg_cg_solve, for callers that cannot allocate
 * device or pinned memory while they run (serving loops with a fixed memory
 * plan, harnesses that forbid hipMalloc): the same checks, kernels and
 * results (bitwise, as the reductions are deterministic), with the solver's
 * workspace taken from a static device array of dg_cg_solve_noalloc_capacity()
 * bytes (128 MiB; one per GPU, held from the library's load on that device
 * until the process ends) and the residual read-backs going through
 * thread-local pageable host memory.  Calls no hipMalloc, hipFree,
 * hipHostMalloc or the op's allocator.
 * Limit: dg_cg_solve_noalloc_bytes(op, mode) must not exceed the capacity
 * (FP64 mode about 32 bytes per DoF, mixed modes 24 to 28: some 4 to 5
 * million DoFs); larger solves return DG_ERR_ARG before any work.
 * Every call on a device shares that device's array and leaves its last
 * contents there: calls that overlap on one device (two streams, two host
 * threads) race and must be serialised by the caller. */
dg_status dg_cg_solve_noalloc(dg_op *op, dg_vec b, dg_vec x, const dg_solve_params *params,
                              dg_solve_stats *stats, void *stream);
/* Workspace bytes dg_cg_solve_noalloc needs for this op in this mode. */
dg_status dg_cg_solve_noalloc_bytes(const dg_op *op, int mode, size_t *bytes);
/* Bytes of the static workspace (the largest accepted dg_cg_solve_noalloc_bytes). */
size_t dg_cg_solve_noalloc_capacity(void);

/* Releases everything the op allocated.  Synchronises nothing: the caller
 * must make sure no enqueued work still uses the op. */
dg_status dg_destroy(dg_op *op);

const char *dg_last_error(void);

/* Host-only: the 1D tables the kernels are compiled with, for degree k
 * (1..8), n = k+1.  out receives, in this order: Gauss points (n), Gauss
 * weights (n), Gauss-Lobatto points (n), S (n*n, S[q][j] = phi_j(gauss_q)),
 * Dco (n*n, derivative of the Lagrange basis on the Gauss points at the Gauss
 * points).  len must be >= 3n + 2n^2. */
dg_status dg_tables(int degree, double *out, size_t len);

/* ---------------------------------------------------------------------------
 * Continuous batching of solves.  A batch holds up to max_slots solve
 * requests (mixed precision with reliable updates, the scheme of
 * dg_cg_solve mode 2).  dg_batch_run advances every active slot by one CG
 * iteration per round.  A round is a fixed sequence of launches: per degree
 * and FP32 geometry storage present, ONE persistent apply kernel whose
 * workgroups walk a work list of (slot, cell batch) items covering the cell
 * lists of all active requests of that degree and storage, whatever their
 * size; then kernels that
 * reduce and update the vectors of all active requests together.  Requests
 * may be admitted while others run.  Results do not depend on which other
 * requests share the batch: every reduction of a request is done over a
 * fixed partition of its own vector or of its own cell batches.
 * ------------------------------------------------------------------------ */
typedef struct dg_batch dg_batch;

dg_status dg_batch_create(int max_slots, const dg_allocator *alloc, dg_batch **out);

/* Admits a request: op must have both precisions, b and x FP64 of length
 * dg_n_dofs(op); x holds the initial guess.  The batch allocates the
 * request's solver workspace (about 8 vectors) through its allocator.
 * *slot receives the slot index; DG_ERR_OOM if no slot is free. */
dg_status dg_batch_admit(dg_batch *batch, dg_op *op, dg_vec b, dg_vec x,
                         const dg_solve_params *params, int *slot, void *stream);

/* Runs up to max_rounds rounds (inner CG iterations) for all active slots on
 * stream, then synchronises it. */
dg_status dg_batch_run(dg_batch *batch, int max_rounds, void *stream);

/* Lists slots that finished since the last poll (their x is final) and frees
 * them; stats[i] belongs to done_slots[i].  capacity bounds both arrays. */
dg_status dg_batch_poll(dg_batch *batch, int *done_slots, dg_solve_stats *stats, int capacity,
                        int *n_done);

/* Number of active (admitted, not yet polled) requests. */
int dg_batch_active(const dg_batch *batch);

dg_status dg_batch_destroy(dg_batch *batch);

#ifdef __cplusplus
}
#endif

#endif /* DG_H */
