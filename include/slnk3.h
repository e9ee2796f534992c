/* slnk3.h -- C ABI of the three-dimensional semi-Lagrangian Newton--Krylov path on MI355X (gfx950).
 *
 * Nothing in the method of arXiv:1604.02153 is specific to two dimensions (section 1,
 * "Limitations and Unresolved Issues"); this interface runs it on a periodic volume.  The
 * operations are those of slnk.h for d = 3: the objective (eq. e:varopt:objective without the
 * mass-source term), the reduced gradient g = beta A v + K int lambda grad m dt (eq. e:control-elim),
 * the Gauss--Newton reduced Hessian matvec (eq. e:hessian-matvec with the lambda terms dropped,
 * section 3.4.1) or the full-Newton one, the preconditioners P_REG (eq. e:reg-precond) and P_2L
 * (section 3.4.2, CHEB(k) or the nested PCG(eps) coarse solve), and the globalised inexact
 * Newton--PCG solve (sections 3.4.1, 3.5).  Transport is the semi-Lagrangian scheme of section 3.3.2
 * (Heun trace of the characteristics, RK2 along them, periodic cubic spline interpolation -- here
 * the tensor-product cubic B-spline in three dimensions, its coefficients from the periodic inverse
 * of the (1, 4, 1)/6 system along each axis, applied as the exponential filter
 * sqrt(3) sum z^|t| f_{i+t}, z = sqrt(3) - 2, truncated below the working precision), or on request
 * the stabilised RK2 scheme of section 3.3.1.
 *
 * Conventions
 *   - Grid: periodic [0, 2 pi)^3 with n1 x n2 x n3 nodes, x_i = 2 pi i / n_i; every n_i a power of
 *     two in [8, 512].  A scalar field is a row-major [n1][n2][n3] array (i3 fastest); a vector
 *     field is three consecutive scalar fields ([3][n1][n2][n3]).
 *   - Element type: double when params.prec == SLNK_PREC_FP64, float when SLNK_PREC_MIXED (fields
 *     and Krylov vectors in FP32; every inner product, norm and the objective in FP64).  Scalar
 *     outputs are double.
 *   - Memory: every field pointer is a DEVICE pointer owned by the caller; the library owns its
 *     workspace (allocated in slnk3_create, released in slnk3_destroy).
 *   - Streams: all device work is enqueued on the stream given to slnk3_create; calls returning
 *     host scalars synchronise it, and any call may synchronise to read a scalar it needs.
 *   - Errors: every call returns an slnk_status (slnk.h); the message of the last failure is
 *     available from slnk3_last_error.  A context is used by one host thread at a time.
 */
#ifndef SLNK3_H
#define SLNK3_H

#include "slnk.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct slnk3_ctx slnk3_ctx;

/* nt: SL time steps on [0, 1] (>= 1); reg: SLNK_REG_H1/H2/H3 (A = -Lap, Lap^2, -Lap^3,
 * eq. e:diffopregv); beta > 0; prec: SLNK_PREC_FP64 or SLNK_PREC_MIXED; proj: SLNK_PROJ_NONE
 * (K = identity) or SLNK_PROJ_LERAY (K = the Leray projection, the incompressible case,
 * section 3.1); sl_path: 0 = each SL step stages its tiles' stencil footprint in LDS whenever the
 * displacement bound lets it fit, else reads the stencils from the global coefficient field;
 * 1 = always the global reads (a tuning choice: both give the same interpolant up to rounding);
 * pc: SLNK_PC_REG (PCG on H with P_REG) or SLNK_PC_2L (PCG on the split system
 * (I + S Q S) s = -S g, S = (beta A')^{-1/2}, with the nested two-level preconditioner of section
 * 3.4.2 on a coarse grid of n_i / 2 points per axis, every n_i / 2 >= 8); cheb_iters, lanczos_steps,
 * emax_safety, lanczos_seed: CHEB(k) and the Lanczos estimate of e_max at v = 0 as in slnk.h
 * (lanczos_steps 1 to 1000 with P_2L); hessian: SLNK_HESS_GN (default) or SLNK_HESS_FN, the
 * full-Newton matvec as in slnk.h (the incremental adjoint with its source div(lambda vt), b~ with
 * lambda grad m~; lambda^0..lambda^nt of the last gradient kept, nt + 8 more fields; the coarse
 * operator of P_2L stays Gauss--Newton); coarse_solver, coarse_eps: P_2L's coarse solver as in
 * slnk.h, SLNK_COARSE_CHEB (default, CHEB(cheb_iters)) or SLNK_COARSE_PCG (the nested PCG(eps) solve:
 * CG on the coarse split operator from zero to coarse_eps times the outer PCG tolerance, 1 in
 * slnk3_precond_apply, at most 200 steps; coarse_eps in (0, 1), default 0.1); transport:
 * SLNK_TRANSPORT_SL (default) or SLNK_TRANSPORT_RK2A, the stabilised RK2 scheme of section 3.3.1
 * and the appendix "Stabilized RK2 Scheme" as in slnk.h (antisymmetric-form state, adjoint and
 * incremental equations with pseudospectral derivatives, Heun's method; conditionally stable, nt by
 * the CFL condition; with P_REG; GN or full Newton; sl_path ignored). */
typedef struct {
  int n1, n2, n3, nt;
  int reg;
  double beta;
  int prec;
  int proj;
  int sl_path;
  int pc;
  int cheb_iters;
  int lanczos_steps;
  double emax_safety;
  unsigned long long lanczos_seed;
  int hessian;
  int coarse_solver;
  double coarse_eps;
  int transport;
} slnk3_params;

/* 64^3, nt = 4, H2, beta = 1e-3, mixed precision, K = identity, P_REG (CHEB(10), 30 Lanczos
 * steps, safety 1.05 for P_2L). */
void slnk3_default_params(slnk3_params* p);

/* Create a context; *out is set on success.  SLNK_EINVAL for sizes outside the conventions,
 * SLNK_ENOMEM when the workspace (about (4 nt + 60) fields of n1 n2 n3 elements) does not fit. */
slnk_status slnk3_create(const slnk3_params* params, void* hip_stream, slnk3_ctx** out);
void slnk3_destroy(slnk3_ctx* ctx);
const char* slnk3_last_error(const slnk3_ctx* ctx);
unsigned long long slnk3_workspace_bytes(const slnk3_ctx* ctx);

/* Reference and template images (scalar fields); copied into the context.  With P_2L also the
 * set-up of section 3.4.2: the spectrally restricted images of the coarse problem and e_max, the
 * largest Ritz value of lanczos_steps Lanczos steps on the coarse split operator at v = 0 from a
 * SplitMix64 start vector, times emax_safety; e_min = min_k 1 + 1 / (beta a'(k)) over the coarse
 * modes. */
slnk_status slnk3_set_images(slnk3_ctx* ctx, const void* m_R, const void* m_T);

/* m1 = m0 transported by the stationary velocity v to t = 1 (the state equation, eq.
 * e:state-slm).  Needs no images.  Changes the context's linearisation point. */
slnk_status slnk3_transport_state(slnk3_ctx* ctx, const void* v, const void* m0, void* m1);

/* J(v) (eq. e:varopt:objective: 1/2 ||m(1) - m_R||^2 + beta/2 <v, A v>, L2 products with the cell
 * volume); linearises at v. */
slnk_status slnk3_objective(slnk3_ctx* ctx, const void* v, double* J);

/* g(v) (eq. e:control-elim) and, if J != NULL, J(v); linearises at v. */
slnk_status slnk3_gradient(slnk3_ctx* ctx, const void* v, void* g, double* J);

/* Hvt = beta A vt + K int lambda~ grad m dt, the Gauss--Newton matvec at the last linearisation
 * point (eqs. e:hessian-matvec, e:inc-state-slm, e:inc-adj-slm); with hessian = SLNK_HESS_FN the
 * full-Newton matvec beta A vt + K int (lambda~ grad m + lambda grad m~) dt.  SLNK_EINVAL before the
 * first slnk3_gradient or slnk3_objective, and for SLNK_HESS_FN unless the last of them at this
 * point was slnk3_gradient (the matvec needs its lambda). */
slnk_status slnk3_hessian_matvec(slnk3_ctx* ctx, const void* vt, void* Hvt);

/* z = P_REG^{-1} r: the spectral inverse of beta A with its zero symbol replaced by 1 (eq.
 * e:reg-precond); with P_2L, z = P_2L^{-1} r = (I - L) r + Pro CHEB(M_c) Res r (section 3.4.2: L
 * the ideal low-pass onto the coarse modes, Res / Pro spectral restriction and prolongation, M_c
 * the coarse split operator linearised at the restricted current point), SLNK_EINVAL before the
 * first slnk3_gradient or slnk3_objective. */
slnk_status slnk3_precond_apply(slnk3_ctx* ctx, const void* r, void* z);

/* out = (I + S Q S) s, S = (beta A')^{-1/2}, Q the transport part of the GN matvec at the last
 * linearisation point: the split spectrally preconditioned Hessian of section 3.4.2. */
slnk_status slnk3_split_matvec(slnk3_ctx* ctx, const void* s, void* out);

/* The Chebyshev bounds of P_2L (the set-up values, or those of the last solve); 0 with P_REG. */
slnk_status slnk3_get_cheb_bounds(const slnk3_ctx* ctx, double* emin, double* emax);

/* Globalised inexact Gauss--Newton--Krylov solve with P_REG or P_2L (params.pc) from v_inout
 * (overwritten by the solution); options and report as in slnk.h (fallback is 0).  Each solve
 * starts from the set-up e_max; a PCG step with r.z <= 0 (CHEB(k) indefinite) re-estimates e_max
 * by Lanczos at the current coarse linearisation and runs PCG again (section 4.2.1).  Returns
 * SLNK_OK, or the status of a solve that ended early (also in report->status):
 * SLNK_ELINESEARCH, SLNK_EMAXIT, SLNK_ECHEB_DIVERGED. */
slnk_status slnk3_newton_solve(slnk3_ctx* ctx, void* v_inout, const slnk_solve_opts* opts,
                               slnk_solve_report* report);

#ifdef __cplusplus
}
#endif

#endif /* SLNK3_H */
