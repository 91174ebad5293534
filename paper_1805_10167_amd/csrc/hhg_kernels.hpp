// Launchers of the HIP kernels of the HHG P1 hot path.  Every launcher
// enqueues on the given stream and returns the launch status.
#pragma once

#include <hip/hip_runtime.h>

#include "hhg_mesh.hpp"

namespace hhg {

enum { OP_LAPLACE = 0, OP_DIFFUSION = 1, OP_MASS = 2 };
enum { DT_F64 = 0, DT_F32 = 1 };

// field[copy] = field[owner] for the ghost classes in `mask` (GM_*).
hipError_t launch_sync(const hhg_mesh* M, int level, int dtype, void* x, int mask,
                       hipStream_t s);
// y = A x (interior rows), 0 on Dirichlet rows, ghosts of y refreshed.
hipError_t launch_apply(const hhg_mesh* M, int level, int op, int dtype, const void* x,
                        void* y, hipStream_t s);
// r = f - A u on interior points, 0 on Dirichlet points, with all copies of
// r; optional |r|_2 over interior points into the device double *norm.
hipError_t launch_residual(const hhg_mesh* M, int level, int op, int dtype, const void* u,
                           const void* f, void* r, double* norm, hipStream_t s);
// One forward or backward staged Gauss-Seidel sweep from field x into field y
// (x is used as scratch; y receives the complete result).
hipError_t launch_gs_sweep(const hhg_mesh* M, int level, int op, int dtype, void* x, void* y,
                           const void* f, int backward, hipStream_t s);
// Mixed-precision outer step (see k_mp_step_tiled): e == nullptr for the first
// residual; xo receives x + e otherwise.
hipError_t launch_mp_step(const hhg_mesh* M, int level, int op, const double* x, const float* e,
                          const double* f, double* xo, float* r, double* norm, hipStream_t s);
// Forward sweep x -> y followed by the restriction of r = f - A y:
// fc (level-1) = P^T r, uc (level-1) = 0.  r is scratch: without two-colour
// faces it receives only what the edge and vertex restriction reads.
hipError_t launch_gs_sweep_restrict(const hhg_mesh* M, int level, int op, int dtype, void* x, void* y,
                                    const void* f, void* r, void* fc, void* uc, hipStream_t s);
// Backward sweep x -> y that also writes |f - A y|_2 over interior points to
// the device double *norm (fixed-order sums: face-core points per tile, then
// the points on and next to the macro-edges).
hipError_t launch_gs_sweep_norm(const hhg_mesh* M, int level, int op, int dtype, void* x, void* y,
                                const void* f, double* norm, hipStream_t s);
// Reduction slots the norm sweep of `level` needs (host data only).
int64_t sweep_norm_partials(const hhg_mesh* M, int level);
// Reduction slots the face-loop kernels (residual norm, dots, the mixed-
// precision outer step) need on `level` (host data only).
int64_t face_loop_partials(const hhg_mesh* M, int level);
// Backward sweep that starts from x + P uc (uc: correction of level - 1):
// prolongation and the first post-smoothing sweep in the same launches.
hipError_t launch_gs_sweep_prolong(const hhg_mesh* M, int level, int op, int dtype, void* x, void* y,
                                   const void* f, const void* uc, hipStream_t s);
// Jacobi-scaled residual at edge and vertex points only (FP32), with their
// copies (face rings included).
hipError_t launch_jacobi_low(const hhg_mesh* M, int level, int op, const float* u, const float* f,
                             float* rho, hipStream_t s);
// Face step of the learned sweep, x -> y (see k_net_step).
hipError_t launch_net_step(const hhg_mesh* M, int level, int op, const float* x, float* y, const float* f,
                           const float* rho_ring, bool mfma, hipStream_t s);
// fc (level-1) = P^T r (level) from r with its copies; uc (level-1) = 0.
hipError_t launch_restrict(const hhg_mesh* M, int level, int dtype, const void* r, void* fc,
                           void* uc, hipStream_t s);
// u (level) += P uc (level-1) on interior points, copies included.
hipError_t launch_prolong_add(const hhg_mesh* M, int level, int dtype, const void* uc,
                              void* u, hipStream_t s);
hipError_t launch_fill(void* x, int64_t n, int dtype, double v, hipStream_t s);
// P2 operator of level fine_level - 1 on the level-fine_level layout (FP64):
// mode 0 y = A x, 1 y = f - A x, 2 y = x + omega D^-1 (f - A x); part holds
// the faces' partial boundary rows.
hipError_t launch_p2(const hhg_mesh* M, int fine_level, int mode, const double* x, const double* f, double* y,
                     double* part, double omega, hipStream_t s);
// ELL values of the coarse operator for `op` into `vals`.
hipError_t launch_coarse_extract(const hhg_mesh* M, int op, double* vals, hipStream_t s);
// u += A_int^-1 (f - A u)_int on the coarse level (stored inverse and one
// refinement step, or Jacobi-PCG), ghosts refreshed.  u_zero: the caller
// guarantees u = 0 (then f is the residual and no residual pass runs).
hipError_t launch_coarse_solve(const hhg_mesh* M, int op, int dtype, void* u, const void* f,
                               const double* vals, hipStream_t s, bool u_zero = false);
// Canonical <-> layout conversion (to_canon = 1: field -> canonical).
hipError_t launch_canon(const hhg_mesh* M, int level, int dtype, const void* src, void* dst,
                        int to_canon, hipStream_t s);
// Coarse coefficient by injection from level to level-1, ghosts refreshed.
hipError_t launch_inject(const hhg_mesh* M, int level, int dtype, const void* kf, void* kc,
                         hipStream_t s);
// Elementwise conversions over whole fields.
hipError_t launch_f64_to_f32(const double* src, float* dst, int64_t n, hipStream_t s);
hipError_t launch_f32_to_f64(const float* src, double* dst, int64_t n, hipStream_t s);
hipError_t launch_add_f32_to_f64(double* u, const float* e, int64_t n, hipStream_t s);

// One Gauss-Seidel stage on edges and vertices (0: A, 1: B), copies written.
hipError_t launch_low_gs(const hhg_mesh* M, int level, int op, int dtype, void* u, const void* f,
                         int stage, hipStream_t s);
// Learned face smoother (net.hip).  mode 0: y = N(rho) on face interiors
// (caller zeroes y first); mode 1: y += N(rho).  Copies are written.
hipError_t launch_net_forward(const hhg_mesh* M, int level, const float* rho, float* y, int mode,
                              bool mfma, hipStream_t s);
// dW[224] += gradient of sum_p g(p) N(rho)(p) with respect to the weights.
hipError_t launch_net_backward(const hhg_mesh* M, int level, const float* rho, const float* g,
                               float* dW, bool bf16, hipStream_t s);
hipError_t launch_net_adam(const hhg_mesh* M, const float* grad, float lr, int step, hipStream_t s);
// rho = D^-1 (f - A u) (f != null) or rho = D^-1 u (f == null) on interior
// points, 0 on Dirichlet points, copies included.
hipError_t launch_jacobi(const hhg_mesh* M, int level, int op, int dtype, const void* u,
                         const void* f, void* rho, hipStream_t s);
// Deterministic dot product over owned interior points into *out (device).
hipError_t launch_dot(const hhg_mesh* M, int level, int dtype, const void* x, const void* y,
                      double* out, hipStream_t s);
// z = alpha x + beta y over whole fields.
hipError_t launch_axpby(int64_t n, int dtype, double alpha, const void* x, double beta, const void* y,
                        void* z, hipStream_t s);

// The dot product of launch_dot with its partial sums in the library's
// static device scratch instead of the workspace (no allocation; calls that
// overlap on one device share that scratch and race).
bool dot_noalloc_fits(const hhg_mesh* M, int level);
hipError_t launch_dot_noalloc(const hhg_mesh* M, int level, int dtype, const void* x, const void* y,
                              double* out, hipStream_t s);
// Device address of the static scratch on the current device (once per
// device; later calls return at once).
hipError_t scratch_init();
// *out = fixed-order sum of partials[0, count).
hipError_t launch_reduce(const double* partials, int64_t count, double* out, hipStream_t s);

// Stokes system and MINRES (stokes.hip).  Stokes vectors are three fields
// u_x | u_y | p of `level`, each of the level's field length.
// Reduction slots the Stokes kernels need.
int64_t stokes_partials();
// mode 0: y = K x; 1: y = K x with partial sums of y . x (count in *nparts);
// 2: y = b - K x.  Velocity rows of Dirichlet points are 0.
hipError_t launch_stokes_apply(const hhg_mesh* M, int level, int mode, const double* x, const double* b,
                               double* y, double* partials, int64_t* nparts, hipStream_t s);
// z_p = r_p / (lumped 1/mu-weighted mass), with partial sums of r . z over
// all three fields (the velocity parts of z must be in place).
hipError_t launch_stokes_pscale_dot(const hhg_mesh* M, int level, const double* r, double* z,
                                    double* partials, int64_t* nparts, hipStream_t s);
// Partial sums of a . b over the owned points of all three fields.
hipError_t launch_stokes_dot(const hhg_mesh* M, int level, const double* a, const double* b,
                             double* partials, int64_t* nparts, hipStream_t s);
// Scalar stages of MINRES (0: start, 1: after the operator, 2: after the
// preconditioner), state in st, residual norms to the host-visible slot.
hipError_t launch_minres_scalars(int stage, const double* partials, int64_t count, double* st, double* slot,
                                 hipStream_t s);
hipError_t launch_minres_rupdate(int64_t n, const double* y, const double* r, double* r_old, const double* st,
                                 hipStream_t s);
hipError_t launch_minres_wupdate(int64_t n, const double* yk, const double* w_old, double* w_older, double* x,
                                 const double* st, hipStream_t s);

// Energy transport (transport.hip).  Cell fields are [up | down], two
// point-layout fields of the level.
// One explicit upwind step Tout = Tin - dt/|c| sum_e F_e T_up(e).
hipError_t launch_fv_step(const hhg_mesh* M, int level, const double* ux, const double* uy, const double* Tin,
                          double* Tout, double dt, hipStream_t s);
// Buoyancy load -Ra r_hat sum T |c| / 3 into the velocity fields of b.
hipError_t launch_fv_buoyancy(const hhg_mesh* M, int level, const double* T, double Ra, double* b,
                              hipStream_t s);
// Canonical cell order <-> cell field (to_canon = 1: field -> canonical).
hipError_t launch_cell_canon(const hhg_mesh* M, int level, const double* src, double* dst, int to_canon,
                             hipStream_t s);

}  // namespace hhg
