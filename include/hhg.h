/*
 * hhg.h - C ABI of the MI355X (gfx950) hierarchical-hybrid-grid P1 multigrid
 * library.
 *
 * The method (Kohl et al., "A Scalable and Modular Software Architecture for
 * Finite Elements on Hierarchical Hybrid Grids"):
 *   - an unstructured triangular macro mesh is turned into a graph of
 *     macro-vertices, macro-edges and macro-faces (sec. 2.1);
 *   - every macro-face is refined uniformly by joining edge midpoints, so a
 *     macro-edge at level l carries n = 2^l + 1 micro-vertices (sec. 1.1, 3.1);
 *   - each unknown is owned by exactly one primitive; neighbours keep
 *     read-only ghost copies that are refreshed by communication along the
 *     primitive graph, the higher-dimensional primitive fixing the order
 *     (sec. 2.2, 2.4, 3.3);
 *   - the operator is applied matrix-free with one constant stencil per
 *     primitive, vertices then edges then faces (sec. 4.2, Alg. 3);
 *   - geometric multigrid on the nested levels with pointwise smoothers,
 *     grid transfers and a Krylov coarse solver (sec. 4.3).
 *
 * Conventions shared by every call:
 *   - Return value: HHG_OK (0) or a negative HHG_E* code; the thread-local
 *     text of the last error is returned by hhg_last_error().
 *   - Ownership: the library owns the opaque hhg_mesh and its host metadata.
 *     The caller owns every device buffer (fields and the workspace) and
 *     every stream; the library only borrows device pointers, which must stay
 *     valid until the work enqueued on the stream has finished.  The library
 *     never allocates or frees device memory.  Its one host-side
 *     allocation besides the mesh object is a 64-byte pinned, device-mapped
 *     slot for the solve loop's residual norm, made by the first
 *     hhg_bind_workspace and freed by hhg_destroy_mesh.
 *   - Streams: `stream` is a hipStream_t (NULL = the default stream).  Calls
 *     enqueue work and return, except hhg_solve, which synchronises the
 *     stream once per iteration to read an 8-byte residual norm.
 *   - Concurrency: one mesh object is not thread-safe; separate meshes are
 *     independent.  Calls sharing one bound workspace must not overlap.
 *   - Fields: a field of level l is a device array of hhg_field_elems()
 *     elements of the chosen dtype in the library's level layout (faces,
 *     then edges, then vertices, each with its ghost copies).  Only the
 *     conversion calls hhg_from_canonical / hhg_to_canonical relate it to the
 *     canonical order.
 *   - Canonical order of level l: macro-vertices by id; then macro-edges
 *     sorted by (lower vertex id, higher vertex id), each with its interior
 *     points k = 1..n-2 counted from the lower vertex; then macro-faces in
 *     input order, each with its interior points (i, j), j = 1..n-3,
 *     i = 1..n-2-j, j-major, where face-local point (i, j) sits at
 *     x0 + i/(n-1) (x1 - x0) + j/(n-1) (x2 - x0) after the face has been
 *     made counter-clockwise (vertices 2 and 3 swapped if needed).
 *   - Dirichlet data: every macro-edge with a single adjacent face, and its
 *     two vertices, is a Dirichlet boundary.  Entries of u at Dirichlet
 *     points hold the boundary values; they are read, never written.
 */
#ifndef HHG_H
#define HHG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define HHG_OK        0
#define HHG_EINVAL   -1   /* bad argument, level, mesh, op or dtype        */
#define HHG_ENOMEM   -2   /* workspace missing, too small or unbound        */
#define HHG_EHIP     -3   /* HIP runtime error (message holds its text)     */
#define HHG_ENOTCONV -4   /* iteration cap or divergence; stats are filled  */

/* element types of fields */
#define HHG_F64  0
#define HHG_F32  1
#define HHG_BF16 2

/* operators */
#define HHG_OP_LAPLACE   0   /* -div grad, P1 stiffness (k = 1)              */
#define HHG_OP_DIFFUSION 1   /* -div(k grad), k from hhg_set_coefficient     */
#define HHG_OP_MASS      2   /* P1 consistent mass matrix                    */

/* smoothers */
#define HHG_SMOOTH_GS  0     /* staged multicolour Gauss-Seidel              */
#define HHG_SMOOTH_NET 1     /* learned face smoother (GS on edges/vertices) */

/* workspace feature bits */
#define HHG_FEAT_F64  1u     /* FP64 multigrid hierarchy                     */
#define HHG_FEAT_MP   2u     /* FP32 hierarchy for mixed-precision refinement */
#define HHG_FEAT_VARK 4u     /* per-level coefficient fields                 */
#define HHG_FEAT_NET  8u     /* learned-smoother buffers                     */
#define HHG_FEAT_STOKES 16u  /* Stokes stencils and MINRES vectors (needs F64) */
#define HHG_FEAT_P2   32u    /* P2 stencils and boundary partials (needs F64) */

/* solver modes */
#define HHG_MODE_PLAIN_FP64 0
#define HHG_MODE_MP_IR      1
#define HHG_MODE_LEARNED    2

typedef struct hhg_mesh hhg_mesh;

typedef struct {
    int32_t precision;         /* HHG_F64 or HHG_F32: arithmetic of the
                                  preconditioner's V-cycles                   */
    double rtol;               /* stop when the residual in the norm of the
                                  inverse preconditioner has fallen by rtol   */
    int32_t max_iters;         /* MINRES iteration cap                        */
    int32_t nu1, nu2;          /* smoothing sweeps of the velocity V-cycles   */
    double* res_history;       /* optional host buffer, entry k = residual
                                  norm after k iterations                     */
    int32_t history_capacity;  /* entries available in res_history           */
} hhg_stokes_opts;

typedef struct {
    int32_t iters;             /* MINRES iterations done                      */
    int32_t converged;         /* 1 if rtol was reached                       */
    double res0;               /* initial residual, preconditioned norm       */
    double rel_res;            /* final / initial preconditioned norm         */
    double ms;                 /* host wall time of the call                  */
} hhg_stokes_stats;

typedef struct {
    int32_t mode;              /* HHG_MODE_*                                  */
    int32_t op;                /* HHG_OP_LAPLACE or HHG_OP_DIFFUSION          */
    double rtol;               /* stop when |f - A u| <= rtol |f - A u0|      */
    int32_t max_iters;         /* cycle (or refinement step) cap              */
    int32_t nu1, nu2;          /* pre- and post-smoothing sweeps              */
    double* res_history;       /* optional host buffer for |r_k|, k = 0..     */
    int32_t history_capacity;  /* entries available in res_history           */
} hhg_solve_opts;

typedef struct {
    int32_t iters;             /* V-cycles (or refinement steps) done         */
    int32_t converged;         /* 1 if rtol was reached                       */
    int32_t smoother_used;     /* HHG_SMOOTH_* actually used                  */
    int32_t fallback;          /* 1 if the learned smoother was dropped       */
    double res0;               /* |f - A u0| over interior points             */
    double rel_res;            /* final |f - A u| / res0                      */
    double ms;                 /* host wall time of the call                  */
} hhg_solve_stats;

/* Text of the last error raised on the calling thread ("" if none). */
const char* hhg_last_error(void);

/*
 * Build the macro-primitive graph (sec. 2.1) and the refinement layouts of
 * levels 1..max_level (sec. 3.1, 3.2).
 *   vxy[2*n_vertices]  host, vertex coordinates (x, y), read during the call
 *   tri[3*n_faces]     host, vertex ids of each triangle; clockwise faces are
 *                      reoriented
 *   coarse_level       multigrid coarsest level, 1 <= coarse_level <= max_level
 *   max_level          finest level, 1 <= max_level <= 12
 *   out                receives the new mesh; destroy with hhg_destroy_mesh
 * Errors: HHG_EINVAL for zero-area faces, an edge with more than two faces,
 * out-of-range ids or levels, or a vertex with more than 16 edges.
 */
int hhg_setup_mesh(const double* vxy, int32_t n_vertices, const int32_t* tri,
                   int32_t n_faces, int32_t max_level, int32_t coarse_level,
                   hhg_mesh** out);

/* Free a mesh (NULL is allowed).  Device buffers are the caller's. */
void hhg_destroy_mesh(hhg_mesh* mesh);

/*
 * Bytes of device workspace needed for a set of HHG_FEAT_* features: index
 * and geometry tables, the coarse-level fields of the hierarchy and solver
 * scratch.  *bytes receives the size.
 */
int hhg_workspace_bytes(const hhg_mesh* mesh, uint32_t features, size_t* bytes);

/*
 * Bind a caller-owned device buffer of at least hhg_workspace_bytes(features)
 * bytes (256-byte aligned), clear it to zero and upload the tables into it on
 * `stream` (synchronised before returning).  The buffer must stay alive and
 * unused by the caller while the mesh uses it.
 * Errors: HHG_ENOMEM if bytes is too small, HHG_EHIP on a failed upload.
 */
int hhg_bind_workspace(hhg_mesh* mesh, uint32_t features, void* dptr,
                       size_t bytes, void* stream);

/* Number of elements of one field of `level` in the library layout. */
int hhg_field_elems(const hhg_mesh* mesh, int32_t level, int64_t* n);

/* Interior (non-Dirichlet) and all canonical points of `level`. */
int hhg_n_dofs(const hhg_mesh* mesh, int32_t level, int64_t* n_interior,
               int64_t* n_all);

/*
 * Canonical micro-vertex coordinates of `level` into the host buffer
 * xy[2*n_all] (edge points on the straight macro-edge, face points by the
 * affine face map; sec. 3.1).
 */
int hhg_coords(const hhg_mesh* mesh, int32_t level, double* xy);

/*
 * Copy table of the level layout (sec. 2.2, 3.3: every unknown has one
 * owner; ghost layers hold copies in the receiver's order): n_copies
 * receives the number of copy slots; with dst and src (host arrays of that
 * length, or null to query the count) the field offsets of every copy slot
 * and of the owned value it copies (face rings from edges and vertices, edge
 * end slots from vertices, edge ghost rows from face near-edge rows, vertex
 * ring slots from edge points).  Every library call leaves field[dst] ==
 * field[src] in its outputs.  Host only: needs no workspace.
 */
int hhg_ghost_table(const hhg_mesh* mesh, int32_t level, int64_t* n_copies, int64_t* dst, int64_t* src);

/*
 * Layout conversion (sec. 3.2: the indexing function maps the topological
 * enumeration to memory).  `canon` is a device array of n_all values of
 * `dtype`; `field` a device field of the same dtype.  from_canonical writes
 * every owned value and every ghost copy; to_canonical reads owned values.
 */
int hhg_from_canonical(const hhg_mesh* mesh, int32_t level, int32_t dtype,
                       const void* canon, void* field, void* stream);
int hhg_to_canonical(const hhg_mesh* mesh, int32_t level, int32_t dtype,
                     const void* field, void* canon, void* stream);

/*
 * Nodal coefficient k of -div(k grad u) at the finest level, a device
 * array of n_all(max_level) doubles in canonical order.  Coarser levels take
 * it by injection.  Needs a workspace bound with HHG_FEAT_VARK.  Enables
 * HHG_OP_DIFFUSION (on-the-fly stencils, paper sec. 1.1 and 4.2).  k > 0
 * gives a symmetric positive definite operator; other values are taken as
 * given (an indefinite operator, on which smoothing and solves may diverge:
 * hhg_solve stops after three cycles of rising residual).
 */
int hhg_set_coefficient(hhg_mesh* mesh, const double* k_canon, void* stream);

/*
 * y = A x on `level` (Alg. 3, sec. 4.2): interior rows get the stencil
 * result, Dirichlet rows are set to 0; all ghost copies of y are refreshed.
 * x and y are fields of `dtype` (F64 or F32); x must have consistent ghosts
 * (every library call leaves them so).  x and y must not alias.
 */
int hhg_apply(const hhg_mesh* mesh, int32_t level, int32_t op, int32_t dtype,
              const void* x, void* y, void* stream);

/*
 * r = f - A u on interior points (0 on Dirichlet points) into field r, and
 * optionally |r|_2 over interior points (each unknown once, sec. 4.1 Alg. 2)
 * into the device double *norm (NULL to skip).  With r == NULL only the norm
 * is formed (norm must then be given).
 */
int hhg_residual(const hhg_mesh* mesh, int32_t level, int32_t op, int32_t dtype,
                 const void* u, const void* f, void* r, double* norm,
                 void* stream);

/*
 * `sweeps` Gauss-Seidel sweeps on `level` (sec. 2.4, 3.2, 4.3): stages
 * A = macro-vertices and even-k edge points, B = odd-k edge points, then the
 * face colours, each stage updated at once; backward != 0 reverses the
 * stage order.  u (in/out) and f are fields of `dtype`.
 * smoother HHG_SMOOTH_NET (FP32 fields, weights set) keeps stages A and B
 * and replaces the face stages by u += N(D^-1 (f - A u)); the backward
 * sweep applies the face step first.
 */
int hhg_smooth(const hhg_mesh* mesh, int32_t level, int32_t op,
               int32_t smoother, int32_t dtype, void* u, const void* f,
               int32_t sweeps, int32_t backward, void* stream);

/*
 * One V(nu1, nu2) cycle from `level` down to the coarse level (sec. 4.3):
 * nu1 forward sweeps, residual and restriction (transpose of linear
 * interpolation), recursion with zero initial guess, linear prolongation and
 * correction, nu2 backward sweeps.  The coarse level is solved directly
 * through a stored inverse (built on the GPU by Jacobi-PCG columns the first
 * time it is needed) when it has at most 2048 interior unknowns, else by
 * Jacobi-PCG to a relative residual of 1e-14.  Uses the
 * bound workspace for coarse fields (HHG_FEAT_F64 for dtype F64, HHG_FEAT_MP
 * for F32).
 */
int hhg_vcycle(const hhg_mesh* mesh, int32_t level, int32_t op,
               int32_t smoother, int32_t dtype, void* u, const void* f,
               int32_t nu1, int32_t nu2, void* stream);

/*
 * Solve A u = f on the finest level to a relative residual opts->rtol
 * (sec. 4.3: multigrid as a solver).  u, f are FP64 fields; u holds the
 * initial guess and the Dirichlet values.  Modes: plain FP64 V-cycles;
 * mixed-precision iterative refinement (not in the paper: FP64 residual and
 * update, FP32 V-cycle on the correction whose coarse level is solved in
 * FP64, like hhg_vcycle's, through the stored inverse with one refinement
 * step, or Jacobi-PCG above 2048 unknowns); learned smoother inside the
 * mixed-precision loop with Gauss-Seidel fallback: the learned smoother runs
 * only if a network is loaded and marked accepted, and a learned cycle that
 * does not lower the residual (or makes it non-finite) is undone (the
 * previous iterate is kept) and the solve goes on with Gauss-Seidel
 * (stats->fallback = 1; the undone cycle counts in stats->iters).  The
 * mixed-precision modes alternate the iterate between u and a workspace
 * field and copy it back to u before returning.  Returns HHG_ENOTCONV if
 * max_iters is reached or the residual stops decreasing; stats are filled in
 * every case.
 */
int hhg_solve(hhg_mesh* mesh, const hhg_solve_opts* opts, void* u,
              const void* f, hhg_solve_stats* stats, void* stream);

/*
 * Jacobi-scaled residual rho = D^-1 (f - A u) on interior points (f != NULL)
 * or rho = D^-1 u (f == NULL), 0 on Dirichlet points, all copies written;
 * D is the diagonal of the operator (sec. 4.3: pointwise smoothers use the
 * diagonal, which the stencils provide).  rho must not alias u or f.
 */
int hhg_jacobi(const hhg_mesh* mesh, int32_t level, int32_t op, int32_t dtype,
               const void* u, const void* f, void* rho, void* stream);

/*
 * Dot product x^T y over the owned interior points of `level` (each unknown
 * once), accumulated in FP64 in a fixed order, into the device double *out
 * (sec. 4.1 Alg. 2: local dots per primitive, then a global sum).
 */
int hhg_dot(const hhg_mesh* mesh, int32_t level, int32_t dtype, const void* x,
            const void* y, double* out, void* stream);

/*
 * hhg_dot without the workspace's scratch, for callers that cannot allocate
 * device memory or must not touch the workspace (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * kernels and summation order as hhg_dot, so the same result bit for bit,
 * with the per-block partial sums (at most 9216 doubles, 72 KiB) in a static
 * device array of the library.  It allocates nothing and frees nothing; each
 * device that runs it holds its own copy of the array from the library's
 * first use on that device (workspace binding or the first call) until the
 * process ends.  Every call on a device shares that device's array: calls
 * that overlap on one device (different streams or threads) race.  The
 * tables of a bound workspace are still read (hhg_bind_workspace first).
 * Errors: as hhg_dot; HHG_EINVAL if the level would need more partial sums
 * than the array holds.
 */
int hhg_dot_noalloc(const hhg_mesh* mesh, int32_t level, int32_t dtype, const void* x,
                    const void* y, double* out, void* stream);

/*
 * z = alpha x + beta y over whole fields of `level` (sec. 4.1 Alg. 1,
 * assign; purely local, copies stay consistent).  z may alias x or y.
 */
int hhg_axpby(const hhg_mesh* mesh, int32_t level, int32_t dtype, double alpha,
              const void* x, double beta, const void* y, void* z, void* stream);

/*
 * Full-weighting restriction fc = R r from `level` to level - 1 (sec. 4.3:
 * the transpose of linear interpolation, weight 1 at the coincident point and
 * 1/2 at each of its six fine neighbours), 0 at coarse Dirichlet points,
 * every copy of fc written.  r must carry consistent copies (every library
 * call leaves its outputs so).  2 <= level <= max_level; fc is a field of
 * level - 1 and must not alias r.
 */
int hhg_restrict(const hhg_mesh* mesh, int32_t level, int32_t dtype,
                 const void* r, void* fc, void* stream);

/*
 * u += P uc on `level`: linear interpolation of the level - 1 field uc
 * (sec. 4.3: coarse points are copied, new points on a coarse edge take
 * the mean of its two ends), added on interior points; Dirichlet entries of
 * u are left alone and every copy of u is refreshed.  2 <= level <=
 * max_level.
 */
int hhg_prolong_add(const hhg_mesh* mesh, int32_t level, int32_t dtype,
                    const void* uc, void* u, void* stream);

/*
 * Whole-field precision change dst = (dst_dtype) src on `level` (FP64 to
 * FP32 rounds to nearest even; FP32 to FP64 is exact), the conversion the
 * mixed-precision refinement loop applies to residuals and corrections.
 * Not in the paper, which uses one precision throughout: it belongs to the
 * mixed-precision variant layered on the method.  Only F64 <-> F32;
 * src and dst must not overlap.
 */
int hhg_convert(const hhg_mesh* mesh, int32_t level, int32_t src_dtype,
                const void* src, int32_t dst_dtype, void* dst, void* stream);

/*
 * Learned face smoother (not part of the paper; a smoother variant layered
 * on the method).  N(rho) = HexConv(16->1)(ReLU(HexConv(1->16)(rho))) with
 * 7-tap kernels over the offsets C, E, W, N, S, SE, NW of face-local (i, j),
 * no biases, hidden layer on face-interior points only.  Weights: 224 FP32
 * values, W1[16][7] then W2[16][7], held in the workspace (HHG_FEAT_NET,
 * which needs HHG_FEAT_MP).  The forward pass uses BF16 MFMA operands with
 * FP32 accumulation by default.
 *
 * hhg_net_set_weights: copy w[224] (host) in and reset the Adam moments.
 * hhg_net_get_weights: copy the FP32 master weights out to w[224] (host).
 * hhg_net_set_options: precision HHG_BF16 (MFMA) or HHG_F32 (reference
 *   arithmetic for tests); accepted != 0 lets HHG_MODE_LEARNED use it.
 * hhg_net_forward: out = N(rho) on face interiors, 0 elsewhere (FP32
 *   fields of `level`, copies written).
 * hhg_net_backward: dW[224] (device, accumulated) += gradient of
 *   sum_p g(p) N(rho)(p) over face-interior p; deterministic reduction.
 * hhg_net_adam_step: one Adam step (beta1 0.9, beta2 0.999, eps 1e-8,
 *   bias-corrected, step >= 1) on the master weights with gradient grad
 *   (device, 224 values).
 * Errors: HHG_ENOMEM without HHG_FEAT_NET, HHG_EINVAL for wrong sizes or
 * when no weights have been set.
 */
int hhg_net_set_weights(hhg_mesh* mesh, const float* w, int32_t n, void* stream);
int hhg_net_get_weights(const hhg_mesh* mesh, float* w, int32_t n, void* stream);
int hhg_net_set_options(hhg_mesh* mesh, int32_t precision, int32_t accepted);
int hhg_net_forward(const hhg_mesh* mesh, int32_t level, const void* rho, void* out,
                    void* stream);
int hhg_net_backward(const hhg_mesh* mesh, int32_t level, const void* rho,
                     const void* g, float* dW, void* stream);
int hhg_net_adam_step(hhg_mesh* mesh, const float* grad, float lr, int32_t step,
                      void* stream);

/*
 * Coefficient constant on each macro-face, coef[n_faces] (host, > 0): the
 * stiffness operator HHG_OP_LAPLACE becomes -div(coef grad u) and
 * HHG_OP_DIFFUSION -div(coef k grad u).  The paper's stencils stay one
 * constant stencil per primitive (sec. 4.2): every micro-triangle lies in one
 * macro-face, so each of its stiffness weights is scaled by that face's
 * value, also in the edge and vertex stencils that sum over several faces.
 * The coarse levels use the same coefficient, so their operators remain the
 * Galerkin products of the finer ones.  Coarse operators are rebuilt when a
 * workspace is bound (synchronises the stream).  All ones restores the plain
 * operator.  Errors: HHG_EINVAL for a value that is not positive and finite.
 */
int hhg_set_face_coefficient(hhg_mesh* mesh, const double* coef, void* stream);

/*
 * Equal-order P1-P1 Stokes flow with pressure stabilisation: the monolithic
 * saddle-point system of the paper's energy-transport example (sec. 5.2:
 * P1-P1 with a Petrov-Galerkin pressure stabilisation, velocity zero on the
 * boundary), solved by preconditioned MINRES with multigrid as the
 * preconditioner (sec. 4.3).  Needs a workspace bound with HHG_FEAT_STOKES
 * (and HHG_FEAT_F64; HHG_FEAT_MP for FP32 preconditioning).
 *
 * Unknowns: a Stokes vector is one device array of 3 * hhg_field_elems(level)
 * doubles, the fields u_x | u_y | p one after the other in the level layout.
 * Velocity values at Dirichlet points are boundary data (read, never
 * written); the pressure is an unknown at every point.  With
 *   a(u, v) = sum_c int mu grad u_c . grad v_c,   b(v, q) = -int q div v,
 *   c(p, q) = delta sum_T h_T^2 / mu_T int_T grad p . grad q
 * (h_T the longest edge of micro-triangle T, mu constant per macro-face)
 * the operator is K = [[A, 0, Bx^T], [0, A, By^T], [Bx, By, -C]], symmetric
 * and indefinite, with the constant pressure in its kernel.
 *
 * hhg_stokes_setup: viscosity[n_faces] (host, > 0) and delta > 0 (the
 *   stabilisation parameter); sets the viscosity as the face coefficient of
 *   HHG_OP_LAPLACE (the preconditioner's velocity operator) and builds the
 *   Stokes stencils (host P1 element assembly at the macro scale).
 * hhg_stokes_apply: y = K x on `level`; velocity rows at Dirichlet points 0.
 * hhg_stokes_residual: r = b - K x on `level` (same conventions).
 * hhg_stokes_precond: z = P^-1 r on the finest level, P^-1 = blockdiag(one
 *   V(nu1, nu2) cycle of the viscous operator from zero per velocity
 *   component, in FP64 or FP32 (`precision`), division of the pressure by
 *   the diagonal matrix S = M_l + 4 diag(C): M_l the lumped mass matrix
 *   weighted with 1/mu, C the stabilisation block.  The paper names a
 *   block-diagonal multigrid preconditioner for MINRES (sec. 4.3) but not
 *   its pressure block: the exact Schur complement is B A^-1 B^T + C, and
 *   the C term cut MINRES steps by about a quarter).
 * hhg_stokes_dot: *out (device double) = a . b over every owned point of
 *   the three fields, summed in a fixed order.
 * hhg_stokes_solve: MINRES from the caller's x (b: right-hand side, its
 *   velocity entries at Dirichlet points ignored) until the residual in the
 *   P^-1 norm has fallen by opts->rtol; the pressure correction keeps a zero
 *   mean weighted with the preconditioner's pressure block S.  Synchronises the
 *   stream once per iteration to read that norm.  HHG_ENOTCONV at the cap
 *   (x holds the last iterate; stats are filled in every case).
 * Errors: HHG_ENOMEM without HHG_FEAT_STOKES, HHG_EINVAL before setup or
 * for aliased buffers.
 */
int hhg_stokes_setup(hhg_mesh* mesh, const double* viscosity, double delta, void* stream);
int hhg_stokes_apply(const hhg_mesh* mesh, int32_t level, const void* x, void* y, void* stream);
int hhg_stokes_residual(const hhg_mesh* mesh, int32_t level, const void* x, const void* b, void* r,
                        void* stream);
int hhg_stokes_precond(const hhg_mesh* mesh, int32_t precision, const void* r, void* z, int32_t nu1,
                       int32_t nu2, void* stream);
int hhg_stokes_dot(const hhg_mesh* mesh, int32_t level, const void* a, const void* b, double* out,
                   void* stream);
int hhg_stokes_solve(hhg_mesh* mesh, const hhg_stokes_opts* opts, void* x, const void* b,
                     hhg_stokes_stats* stats, void* stream);

/*
 * Energy transport coupled to the Stokes flow (the paper's sec. 5.2 example:
 * temperature advanced by an explicit upwind finite-volume scheme with the
 * last computed velocity, the Stokes system solved only after every three
 * transport steps, buoyancy forcing -Ra T r_hat).  Finite-volume unknowns
 * sit on the interiors of the micro-triangles (sec. 3.1).  Needs
 * hhg_stokes_setup (workspace with HHG_FEAT_STOKES).
 *
 * Cell fields: one device array of 2 * hhg_field_elems(level) doubles, the
 * up cells {(i,j), (i+1,j), (i,j+1)} of every face at the slots of points
 * (i, j) of the first half, the down cells {(i+1,j), (i+1,j+1), (i,j+1)} at
 * the slots of points (i, j) of the second.  Canonical cell order: per face
 * in input order, up cells j-major (j = 0..n-2, i = 0..n-2-j), then down
 * cells j-major (j = 0..n-3, i = 0..n-3-j): (n-1)^2 per face.
 *
 * Flux through a micro-edge: |e| n . (u_a + u_b) / 2 (outward unit normal n,
 * P1 velocity at the edge's ends: exact for the linear velocity); the two
 * cells of an edge get exactly opposite fluxes.  Micro-edges on the domain
 * boundary carry no flux (zero wall velocity), and there is no diffusion
 * (the paper neglects 1/Pe), so the total heat sum |c| T_c is conserved.
 *
 * hhg_cell_coords: centroids of the cells in canonical order into the host
 *   buffer xy[2 F (n-1)^2] (no workspace needed).
 * hhg_cells_from_canonical / hhg_cells_to_canonical: layout conversion of
 *   cell fields (canonical arrays of F (n-1)^2 doubles, device).
 * hhg_transport_step: T_out = T_in - dt / |c| sum_e F_e T_upwind(e), with the
 *   velocity taken from the Stokes vector x (its u_x and u_y fields).
 * hhg_buoyancy: b (Stokes vector) = (M_T(-Ra T r_hat_x), M_T(-Ra T r_hat_y),
 *   0): b_i = -Ra r_hat(x_i) sum_{cells c at i} T_c |c| / 3, 0 at Dirichlet
 *   points, copies written.
 * hhg_energy_run: opts->steps transport steps from the caller's T (cell
 *   field, updated in place) and x (Stokes vector, the initial guess of the
 *   first solve, the last flow on return); before steps 0, stokes_every,
 *   2 stokes_every, ... the buoyancy of the current T is formed and the
 *   Stokes system solved by MINRES (opts->stokes) warm started from x.
 *   Synchronises the stream.  Returns the first MINRES failure, if any.
 */
typedef struct {
    hhg_stokes_opts stokes;    /* MINRES options of every Stokes solve       */
    double Ra;                 /* Rayleigh number of the buoyancy forcing    */
    double dt;                 /* transport time step                        */
    int32_t steps;             /* transport steps                            */
    int32_t stokes_every;      /* Stokes solve before every k-th step (3)    */
} hhg_energy_opts;

typedef struct {
    int32_t steps;             /* transport steps done                       */
    int32_t stokes_solves;     /* Stokes solves done                         */
    int64_t minres_iters;      /* MINRES iterations over all solves          */
    double worst_rel_res;      /* largest final relative residual of a solve */
    double ms;                 /* host wall time of the call                 */
} hhg_energy_stats;

int hhg_cell_coords(const hhg_mesh* mesh, int32_t level, double* xy);
int hhg_cells_from_canonical(const hhg_mesh* mesh, int32_t level, const double* canon, double* cells,
                             void* stream);
int hhg_cells_to_canonical(const hhg_mesh* mesh, int32_t level, const double* cells, double* canon,
                           void* stream);
int hhg_transport_step(const hhg_mesh* mesh, int32_t level, const double* x, const double* T_in,
                       double* T_out, double dt, void* stream);
int hhg_buoyancy(const hhg_mesh* mesh, int32_t level, const double* T, double Ra, double* b,
                 void* stream);
int hhg_energy_run(hhg_mesh* mesh, const hhg_energy_opts* opts, void* x, void* T,
                   hhg_energy_stats* stats, void* stream);

/*
 * Quadratic (P2) elements and p-multigrid (sec. 3.1: unknowns on the
 * micro-vertices and micro-edges, edge unknowns in three subgroups by edge
 * direction; sec. 4.2, Fig. 8: a stencil per unknown type; sec. 4.3:
 * transfers between P1 and P2 on the same refinement level).
 *
 * The P2 unknowns of level l are the points of level l + 1: a P2 field of
 * level l is a field of the level-(l+1) layout (hhg_field_elems(l + 1)
 * values, owned values and ghost copies, converted with
 * hhg_from_canonical / hhg_to_canonical at level l + 1).  Face-local point
 * (i, j) of that layout is a vertex of level l when i and j are even, else
 * the midpoint of a micro-edge of level l: i odd, j even: i-direction edge;
 * i even, j odd: j-direction edge; both odd: diagonal edge.  Operator: the
 * Laplacian times the coefficient per macro-face of
 * hhg_set_face_coefficient (1 by default); Dirichlet points as for P1.
 * Needs a workspace bound with HHG_FEAT_P2 | HHG_FEAT_F64 on a mesh whose
 * max_level is at least l + 1; P2 calls take the P2 level l, with
 * 1 <= l < max_level.
 *
 * hhg_p2_setup: builds the P2 stencils from the current face coefficients
 *   (host) and uploads them; again after every hhg_set_face_coefficient.
 * hhg_p2_apply: y = A2 x on interior rows, 0 on Dirichlet rows (copies
 *   written).  x and y distinct.
 * hhg_p2_residual: r = f - A2 x, 0 on Dirichlet rows.
 * hhg_p2_jacobi: y = x + omega D^-1 (f - A2 x) on interior points (damped
 *   point Jacobi, all points from the old values), Dirichlet values copied.
 * hhg_p2_solve: p-multigrid cycles until |f - A2 x| <= rtol |f - A2 x0|
 *   (Euclidean norm over interior points): nu1 Jacobi sweeps, residual,
 *   restriction to P1 on level l by the transpose of the P1 -> P2
 *   embedding, one P1 V(vnu1, vnu2) cycle of the h-hierarchy from zero,
 *   prolongation by the embedding and correction, nu2 Jacobi sweeps.  The
 *   embedding coincides with the P1 interpolation from level l to level
 *   l + 1, so the transfers are those of hhg_restrict / hhg_prolong_add at
 *   level l + 1.  Synchronises the stream once per cycle (norm read).
 *   Returns HHG_ENOTCONV if max_iters is reached first; x holds the last
 *   iterate.
 * Errors: HHG_ENOMEM without HHG_FEAT_P2 (or HHG_FEAT_F64 for the solve),
 *   HHG_EINVAL before setup, for a level out of range or bad options.
 */
typedef struct {
    int32_t level;             /* P2 level l (fields of level l + 1)         */
    double rtol;               /* relative residual to reach                 */
    int32_t max_iters;         /* p-multigrid cycles at most                 */
    int32_t nu1, nu2;          /* P2 Jacobi sweeps before / after            */
    int32_t vnu1, vnu2;        /* smoothing of the P1 V-cycle                */
    double omega;              /* Jacobi damping (0.7 suits the Laplacian)   */
    double* res_history;       /* optional host array of residual norms      */
    int32_t history_capacity;  /* its length                                 */
} hhg_p2_opts;

typedef struct {
    int32_t iters;             /* cycles done                                */
    int32_t converged;         /* 1 if rtol was reached                      */
    double res0;               /* initial residual norm                      */
    double rel_res;            /* final / initial                            */
    double ms;                 /* host wall time of the call                 */
} hhg_p2_stats;

int hhg_p2_setup(hhg_mesh* mesh, void* stream);
int hhg_p2_apply(const hhg_mesh* mesh, int32_t level, const void* x, void* y, void* stream);
int hhg_p2_residual(const hhg_mesh* mesh, int32_t level, const void* x, const void* f, void* r,
                    void* stream);
int hhg_p2_jacobi(const hhg_mesh* mesh, int32_t level, double omega, const void* x, const void* f,
                  void* y, void* stream);
int hhg_p2_solve(hhg_mesh* mesh, const hhg_p2_opts* opts, void* x, const void* f, hhg_p2_stats* stats,
                 void* stream);

/*
 * Per-kernel timing of the finest-level smoother launches, for profiling:
 * enable != 0 records a HIP event pair around every finest-level face
 * smoother launch on its stream; hhg_timing_read returns the number of
 * launches and their summed duration in ms since the last reset (it
 * synchronises the recorded events).  Disabled by default.
 */
int hhg_timing_enable(hhg_mesh* mesh, int32_t enable);
int hhg_timing_read(hhg_mesh* mesh, int64_t* launches, double* total_ms,
                    int32_t reset);

#ifdef __cplusplus
}
#endif

#endif /* HHG_H */
