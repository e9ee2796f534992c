// Host-side launchers of the three-dimensional kernels (d3.hip).  The method carries over from
// d = 2 unchanged (section 1, "Limitations and Unresolved Issues"): pseudospectral operators on a
// periodic grid (section 3.2), the semi-Lagrangian transport of section 3.3.2 with the
// tensor-product cubic B-spline in three dimensions, and the reduced gradient and Gauss--Newton
// matvec built from them (eqs. e:control-elim, e:hessian-matvec).
//
// Layout: a scalar field is a row-major [n1][n2][n3] array (i3 fastest, F = n1 n2 n3 values); a
// vector field is three consecutive scalar fields.  A half spectrum is [n1][n2][n3/2 + 1]
// complex (Fh values): the real-to-complex transform runs along x3.  Every n_i is a power of two
// in [8, 512].  Every launcher enqueues on the given stream, never synchronises or allocates,
// and returns the launch status.
#pragma once

#include "common.hpp"

namespace slnk {
namespace d3 {

struct Dims {
  int n1 = 0, n2 = 0, n3 = 0;
  __host__ __device__ size_t F() const { return size_t(n1) * n2 * n3; }
  __host__ __device__ int nh() const { return n3 / 2 + 1; }
  __host__ __device__ size_t Fh() const { return size_t(n1) * n2 * nh(); }
};

// Twiddle tables exp(-2 pi i j / n), j < n / 2, per axis (device memory, computed in FP64).
template <typename T>
struct Twiddles {
  const cplx<T>* t1 = nullptr;
  const cplx<T>* t2 = nullptr;
  const cplx<T>* t3 = nullptr;
};

// Largest transform length supported (LDS tile of the strided passes).
constexpr int kMaxN = 512;

// Forward transform of nf real fields (consecutive, F apart) into nf half spectra (Fh apart):
// unnormalised, exp(-i k x) (numpy's fftn convention).
template <typename T>
hipError_t fft_forward(hipStream_t s, const Dims& d, const Twiddles<T>& tw, int nf, const T* in, cplx<T>* S);
// Inverse transform of nf half spectra into nf real fields, scaled by 1/F; the spectra are
// overwritten.  Each half spectrum must be that of a real field (Hermitian along x3).
template <typename T>
hipError_t fft_inverse(hipStream_t s, const Dims& d, const Twiddles<T>& tw, int nf, cplx<T>* S, T* out);

// Scalar symbols (all real and even in k).
enum class Sym : int {
  One = 0,      // 1
  Reg = 1,      // beta a(k), a = |k|^(2 reg)
  RegInv = 2,   // 1 / (beta a'(k)), a' = a with a(0) replaced by 1 (P_REG^{-1})
  RegInvSqrt = 3,  // (beta a'(k))^{-1/2} (the split preconditioner's half step S)
};
struct SymArgs {
  Sym kind = Sym::One;
  int reg = 2;
  double beta = 1.0;
  int proj = 0;  // nf = 3 only: apply the Leray projection b - k (k . b) / |k|^2 first (odd-order k)
};
// out = op(in) through the transform: Scale (nf = 1 or 3 fields: the symbol, with the Leray
// projection first when a.proj and nf = 3), Grad (one field in, its three derivatives out), Div
// (three fields in, one out).  The forward pass along x1, the operator and the inverse pass along
// x1 run in one LDS kernel where the lines fit.  TF: the fields' element type (float fields
// through an FP64 transform for the mixed context's beta A).  S1, S2: 3 Fh spectra each.
enum class SpecOp : int { Scale = 0, Grad = 1, Div = 2 };
template <typename T, typename TF>
hipError_t spec_apply(hipStream_t s, const Dims& d, const Twiddles<T>& tw, SpecOp op, int nf, SymArgs a, const TF* in,
                      TF* out, cplx<T>* S1, cplx<T>* S2);

// S[c] *= symbol for c < nf (nf = 1 or 3), in place.
template <typename T>
hipError_t spec_symbol(hipStream_t s, const Dims& d, int nf, SymArgs a, cplx<T>* S);
// out[c] = i k_c U (c = 0, 1, 2; Nyquist components zero): the gradient's spectra.
template <typename T>
hipError_t spec_grad(hipStream_t s, const Dims& d, const cplx<T>* U, cplx<T>* out);
// S[0] = sum_c i k_c S[c]: the divergence's spectrum (in place into the first spectrum).
template <typename T>
hipError_t spec_div(hipStream_t s, const Dims& d, cplx<T>* S);

// B-spline coefficients of nf scalar fields (consecutive, F apart), in place allowed: along
// each axis the periodic inverse of the (1, 4, 1)/6 system as the filter
// c_i = sqrt(3) sum_{|t| <= K} z^|t| f_{i+t} (z = sqrt(3) - 2, indices periodic), truncated where
// |z|^K falls below the working precision (K = 13 in FP32, 28 in FP64): three passes, one per axis.
template <typename T>
hipError_t spline_coefficients(hipStream_t s, const Dims& d, int nf, const T* in, T* out);

// Two-grid transfer on half spectra (section 3.4.2, spectral restriction and prolongation): the
// coarse grid has half the points per axis and keeps the fine modes |k_i| < n_i / 4 (its own
// Nyquist modes dropped).  restrict: Sc = those modes of Sf times Fc / F (zero elsewhere);
// prolong_combine: Sf keeps its modes outside that set (the high-pass part of the fine field) and
// takes Sc times F / Fc on it.  nf spectra each.
template <typename T>
hipError_t spec_restrict(hipStream_t s, const Dims& fine, const Dims& coarse, int nf, const cplx<T>* Sf, cplx<T>* Sc);
template <typename T>
hipError_t spec_prolong_combine(hipStream_t s, const Dims& fine, const Dims& coarse, int nf, cplx<T>* Sf,
                                const cplx<T>* Sc);

// One semi-Lagrangian time step (section 3.3.2) at every node x: u = I[coef](x + disp) (the
// cubic spline with B-spline coefficients coef at the departure point, displacement in cells),
// then, by kind:
//   State       dst = u
//   Adjoint     lam = gamma u (+ add); dst = lam; acc += w lam gm
//   IncState    f = -(vt . gm); mt = u + ht/2 f (into 'mt' when given); not last: dst = u + ht f
//               (the next step's transported field m~ + ht/2 f); last: dst = -mt, acc = w (-mt) gm
//   IncAdjoint  lt = gamma u (+ add: the full-Newton source); dst = lt; acc += w lt gm
// (gm: gradient of the state at the output's time level; eqs. e:state-slm, e:adj-slm,
// e:inc-state-slm, e:inc-adj-slm).
enum class Kind : int { State = 0, Adjoint = 1, IncState = 2, IncAdjoint = 3 };
template <typename T>
struct StepArgs {
  Dims d;
  Kind kind = Kind::State;
  const T* coef = nullptr;
  const T* disp = nullptr;
  const T* gamma = nullptr;
  const T* gm = nullptr;
  const T* vt = nullptr;
  T* dst = nullptr;
  T* acc = nullptr;
  const T* add = nullptr;  // Adjoint / IncAdjoint: a field added to gamma u (optional)
  T* mt = nullptr;         // IncState: m~ at the output's time level (optional)
  double w = 0.0, ht = 0.0;
  int last = 0;
  int halo = -1;  // whole cells bounding |disp| (the LDS-staged kernel when its footprint fits), or -1
};
template <typename T>
hipError_t sl_step(hipStream_t s, const StepArgs<T>& a);

// Departure points of both characteristics by Heun's method and the adjoint factor:
//   df = -ht/2 (u(x) + u(x - ht u(x))), da = +ht/2 (u(x) + u(x + ht u(x))) (cells; u the
//   velocity in cells per unit time, its values off the grid from the coefficients cv),
//   gamma = 1 + ht/2 (dD + dx) + ht^2/2 dD dx, dx = div v at x, dD = div v at x + da (from cdiv).
template <typename T>
hipError_t trace(hipStream_t s, const Dims& d, double ht, const T* v, const T* cv, const T* divv, const T* cdiv,
                 T* df, T* da, T* gamma);

// lam = mR - m1; acc = w lam gm (the adjoint's final value and its first b term)
template <typename T>
hipError_t adjoint_start(hipStream_t s, const Dims& d, double w, const T* mR, const T* m1, const T* gm, T* lam,
                         T* acc);
// q = -ht/2 (vt . gm): the incremental state's first transported field (m~(0) = 0)
template <typename T>
hipError_t incstate_start(hipStream_t s, const Dims& d, double ht, const T* vt, const T* gm, T* q);

// out_c = (w . g) g_c (c = 0, 1, 2): the transport part Q w of the GN matvec at v = 0, where m is
// m_T at every time, m~(1) = -(w . grad m_T) and lambda~ = w . grad m_T throughout (g = grad m_T)
template <typename T>
hipError_t q_at_zero(hipStream_t s, const Dims& d, const T* w, const T* g, T* out);

// Full-Newton matvec terms (eq. e:inc-adj-slm with its lambda source; b~ with lambda grad m~):
// out_c = a v_c (c = 0, 1, 2), the product lambda vt whose divergence is the source sigma
template <typename T>
hipError_t scale_vec(hipStream_t s, const Dims& d, const T* a, const T* v, T* out);
// out = ht/2 (1 + ht divv) e + ht/2 sig: Heun's source terms of one incremental adjoint step along the
// adjoint characteristic, e = sigma^j at the departure point, sig = sigma^{j-1} at the node (out may be e)
template <typename T>
hipError_t fn_source(hipStream_t s, const Dims& d, double ht, const T* divv, const T* e, const T* sig, T* out);
// acc_c (init: =, else +=) w lam g_c (c = 0, 1, 2)
template <typename T>
hipError_t acc_scalar_grad(hipStream_t s, const Dims& d, double w, int init, const T* lam, const T* g, T* acc);

// ---- stabilised RK2 transport (section 3.3.1; appendix "Stabilized RK2 Scheme") ----------------
// Antisymmetric-form operators L_s y = 1/2 (v . grad y + div(y v) + s y div v): s = -1 the state
// operator L (d_t m = -L m), s = +1 the adjoint operator A (d_s lam = A lam backward in time); grad y
// and div(y v) come from the spectral Grad and Div passes.  One Heun stage of
// dy/ds = sgn L_dsgn y + src (src optional) at every node: k = sgn L_dsgn y + src from g = grad y,
// dv = div(y v) and y; stage 1: kbuf = k, dst = y + ht k; stage 2: dst = y0 + ht/2 (kbuf + k);
// both: yv = dst v (the product the next evaluation differentiates).
template <typename T>
struct RkStage {
  int stage = 1;
  int sgn = -1, dsgn = -1;
  double ht = 0.0;
  const T* g = nullptr;
  const T* dv = nullptr;
  const T* y = nullptr;
  const T* v = nullptr;
  const T* divv = nullptr;
  const T* src = nullptr;
  const T* y0 = nullptr;
  T* kbuf = nullptr;
  T* dst = nullptr;
  T* yv = nullptr;
};
template <typename T>
hipError_t rk_stage(hipStream_t s, const Dims& d, const RkStage<T>& a);
// out = sgn 1/2 (w . g + dv + dsgn a divw), g = grad a, dv = div(a w): a source of the incremental
// equations (sgn = dsgn = -1: -S(m) vt of the incremental state; +1: the full-Newton incremental
// adjoint's lambda terms)
template <typename T>
hipError_t rk_eval(hipStream_t s, const Dims& d, int sgn, int dsgn, const T* g, const T* dv, const T* a, const T* w,
                   const T* divw, T* out);
// out = a b
template <typename T>
hipError_t mul(hipStream_t s, const Dims& d, const T* a, const T* b, T* out);
// acc_c (init: =, else +=) w/2 (lam gm_c - m gl_c + glm_c), gm = grad m, gl = grad lam,
// glm = grad(lam m): the antisymmetric form of lam grad m in b and b~
template <typename T>
hipError_t rk_accum(hipStream_t s, const Dims& d, double w, int init, const T* lam, const T* m, const T* gm,
                    const T* gl, const T* glm, T* acc);

// out = a x + b y over n values (scalars cast to T; x or y may be null for a zero term)
template <typename T>
hipError_t axpby(hipStream_t s, size_t n, double a, const T* x, double b, const T* y, T* out);

// FP64 reductions over n values into partial[blocks] (reduce_blocks(n) of them), then one
// block sums them in a fixed order into *out: mode 0 sum a b, 1 sum (a - b)^2, 2 max |a|.
int reduce_blocks(size_t n);
template <typename T>
hipError_t reduce(hipStream_t s, size_t n, int mode, const T* a, const T* b, double* partial, double* out);

}  // namespace d3
}  // namespace slnk
