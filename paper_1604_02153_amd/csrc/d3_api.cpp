// Host side of the three-dimensional path (include/slnk3.h): the context, the linearisation
// (trace, state solve, gradients of the state), the reduced gradient, the Gauss--Newton matvec,
// P_REG and the Newton--PCG solve with Armijo backtracking (sections 3.3.2, 3.4.1, 3.5), all on
// the kernels of d3.hip.  Every inner product and norm is an FP64 reduction on the GPU, summed in
// a fixed order (the same inputs give the same bits).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/slnk3.h"
#include "d3.hpp"
#include "kernels.hpp"

namespace slnk {
namespace d3 {
namespace {

struct Err {
  slnk_status st;
  std::string msg;
};

#define D3CHK(expr)                                                                                           \
  do {                                                                                                        \
    hipError_t _e = (expr);                                                                                   \
    if (_e != hipSuccess) throw Err{SLNK_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)};        \
  } while (0)

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

bool size_ok(int n) { return n >= 8 && n <= kMaxN && (n & (n - 1)) == 0; }

// weight of time level j in the composite trapezoid rule on t^0..t^nt (sums to 1)
double trap_w(int j, int nt) { return (j == 0 || j == nt) ? 0.5 / nt : 1.0 / nt; }

// Largest eigenvalue of the symmetric tridiagonal matrix (diagonal a, off-diagonal b): bisection
// on the Sturm count of eigenvalues below x.
double tridiag_max_eig(const std::vector<double>& a, const std::vector<double>& b) {
  const int n = int(a.size());
  double lo = a[0], hi = a[0];
  for (int i = 0; i < n; ++i) {  // Gershgorin bounds
    const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  auto below = [&](double x) {
    int c = 0;
    double q = 1.0;
    for (int i = 0; i < n; ++i) {
      q = a[i] - x - (i > 0 ? b[i - 1] * b[i - 1] / q : 0.0);
      if (q == 0.0) q = -1e-300;
      if (q < 0.0) ++c;
    }
    return c;
  };
  for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(1.0, std::fabs(hi)); ++it) {
    const double mid = 0.5 * (lo + hi);
    (below(mid) == n ? hi : lo) = mid;
  }
  return hi;
}

// Uniform values in [-1/2, 1/2) from SplitMix64 (Steele, Lea, Flood 2014): the state advances by
// 0x9E3779B97F4A7C15; the output is the state after two xor-shift-multiply rounds and a final
// xor-shift; its top 53 bits are the fraction.
std::vector<double> splitmix_uniform(unsigned long long seed, size_t count) {
  std::vector<double> out(count);
  unsigned long long x = seed;
  for (size_t i = 0; i < count; ++i) {
    x += 0x9E3779B97F4A7C15ULL;
    unsigned long long z = x;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z ^= z >> 31;
    out[i] = double(z >> 11) / 9007199254740992.0 - 0.5;
  }
  return out;
}

class Base {
 public:
  virtual ~Base() = default;
  virtual void set_images(const void* mR, const void* mT) = 0;
  virtual void transport_state(const void* v, const void* m0, void* m1) = 0;
  virtual double objective(const void* v) = 0;
  virtual double gradient(const void* v, void* g) = 0;
  virtual void hessian(const void* vt, void* out) = 0;
  virtual void precond(const void* r, void* z) = 0;
  virtual void split_matvec_api(const void* s, void* out) = 0;
  virtual void cheb_bounds(double* emin, double* emax) const = 0;
  virtual slnk_status newton(void* v, const slnk_solve_opts& o, slnk_solve_report& rep) = 0;
  size_t bytes = 0;
};

template <typename T>
class Ctx final : public Base {
 public:
  Ctx(const slnk3_params& p, hipStream_t s) : p_(p), s_(s) {
    d_.n1 = p.n1;
    d_.n2 = p.n2;
    d_.n3 = p.n3;
    F_ = d_.F();
    Fh_ = d_.Fh();
    ht_ = 1.0 / p.nt;
    cell_ = std::pow(2.0 * 3.14159265358979323846, 3) / double(F_);
    fn_ = p.hessian == SLNK_HESS_FN;
    coarse_pcg_ = p.pc == SLNK_PC_2L && p.coarse_solver == SLNK_COARSE_PCG;
    rk_ = p.transport == SLNK_TRANSPORT_RK2A;
    try {
      allocate();
      if (p.pc == SLNK_PC_2L) {  // the coarse level: half the points per axis, GN, its own workspace
        slnk3_params pc = p;
        pc.n1 /= 2;
        pc.n2 /= 2;
        pc.n3 /= 2;
        pc.pc = SLNK_PC_REG;
        pc.hessian = SLNK_HESS_GN;
        coarse_ = std::make_unique<Ctx<T>>(pc, s);
      }
    } catch (...) {
      release();
      throw;
    }
    if (coarse_) bytes += coarse_->bytes;
  }
  ~Ctx() override { release(); }

  void set_images(const void* mR, const void* mT) override {
    D3CHK(hipMemcpyAsync(mR_, mR, F_ * sizeof(T), hipMemcpyDeviceToDevice, s_));
    D3CHK(hipMemcpyAsync(mT_, mT, F_ * sizeof(T), hipMemcpyDeviceToDevice, s_));
    for (const T* img : {mR_, mT_})
      if (!std::isfinite(reduce(0, F_, img, img))) throw Err{SLNK_ENAN, "non-finite image value"};
    images_ = true;
    lin_ = false;
    if (coarse_) setup_two_level();
  }

  void transport_state(const void* v, const void* m0, void* m1) override {
    lin_ = false;
    lam_ok_ = false;
    if (rk_) {  // Heun on d_t m = -L m
      rk_prepare(static_cast<const T*>(v));
      const T* cur = static_cast<const T*>(m0);
      D3CHK(scale_vec<T>(s_, d_, cur, v_, rk_yv_));
      for (int j = 1; j <= p_.nt; ++j) {
        T* out = j == p_.nt ? static_cast<T*>(m1) : rk_y_[j & 1];
        rk_step(-1, -1, cur, out, nullptr, nullptr);
        cur = out;
      }
      D3CHK(hipStreamSynchronize(s_));
      return;
    }
    trace_at(static_cast<const T*>(v));
    const T* cur = static_cast<const T*>(m0);
    T* bufs[2] = {lam0_, lam1_};
    for (int j = 1; j <= p_.nt; ++j) {
      T* out = j == p_.nt ? static_cast<T*>(m1) : bufs[j & 1];
      coefficients(cur, coef_, 1);
      StepArgs<T> a;
      a.d = d_;
      a.halo = halo_;
      a.kind = Kind::State;
      a.coef = coef_;
      a.disp = df_;
      a.dst = out;
      D3CHK(sl_step<T>(s_, a));
      cur = out;
    }
    D3CHK(hipStreamSynchronize(s_));
  }

  double objective(const void* v) override {
    need_images();
    linearize(static_cast<const T*>(v));
    return J_;
  }

  double gradient(const void* v, void* g) override {
    need_images();
    linearize(static_cast<const T*>(v));
    gradient_at(static_cast<T*>(g));
    D3CHK(hipStreamSynchronize(s_));
    return J_;
  }

  void hessian(const void* vt, void* out) override {
    if (!lin_) throw Err{SLNK_EINVAL, "the matvec needs a linearisation (slnk3_gradient or slnk3_objective)"};
    matvec(static_cast<const T*>(vt), static_cast<T*>(out));
  }

  // P_REG^{-1} r, or P_2L^{-1} r at the coarse linearisation of the current point
  void precond(const void* r, void* z) override {
    if (!coarse_) {
      prec_reg(static_cast<const T*>(r), static_cast<T*>(z));
      return;
    }
    if (!lin_) throw Err{SLNK_EINVAL, "P_2L needs a linearisation (slnk3_gradient or slnk3_objective)"};
    coarse_linearize();
    outer_tol_ = 1.0;
    apply_two_level(static_cast<const T*>(r), static_cast<T*>(z));
  }

  void split_matvec_api(const void* sv, void* out) override {
    if (!lin_) throw Err{SLNK_EINVAL, "the matvec needs a linearisation (slnk3_gradient or slnk3_objective)"};
    split_matvec(static_cast<const T*>(sv), static_cast<T*>(out));
  }

  void cheb_bounds(double* emin, double* emax) const override {
    *emin = emin_;
    *emax = emax_;
  }

  slnk_status newton(void* vio, const slnk_solve_opts& o, slnk_solve_report& rep) override {
    need_images();
    std::memset(&rep, 0, sizeof(rep));
    const double t0 = now_ms();
    const size_t V = 3 * F_;
    T* vin = static_cast<T*>(vio);
    D3CHK(hipMemcpyAsync(vk_, vin, V * sizeof(T), hipMemcpyDeviceToDevice, s_));
    if (coarse_) {  // every solve starts from the set-up bound
      emax_ = emax_setup_;
      rep.emin = emin_;
      rep.emax = emax_;
    }
    double g0_inf, g0_two;
    const bool cold = reduce(2, V, vk_, nullptr) == 0.0;
    if (!cold) {  // norms of the gradient at v = 0 for the relative stopping test
      D3CHK(hipMemsetAsync(trial_, 0, V * sizeof(T), s_));
      linearize(trial_);
      gradient_at(gk_);
      g0_inf = reduce(2, V, gk_, nullptr);
      g0_two = std::sqrt(reduce(0, V, gk_, gk_));
    }
    double tg = now_ms();
    linearize(vk_);
    gradient_at(gk_);
    double Jk = J_;
    rep.time_gradient_ms += now_ms() - tg;
    if (cold) {
      g0_inf = reduce(2, V, gk_, nullptr);
      g0_two = std::sqrt(reduce(0, V, gk_, gk_));
    }
    rep.g0_inf = g0_inf;
    rep.g0_two = g0_two;
    if (!(g0_inf > 0.0) || !std::isfinite(g0_two)) throw Err{SLNK_ENAN, "gradient at v = 0 is zero or not finite"};
    slnk_status status = SLNK_OK;
    for (int k = 0; k <= o.max_newton; ++k) {
      const double ginf = reduce(2, V, gk_, nullptr);
      const double gtwo = std::sqrt(reduce(0, V, gk_, gk_));
      if (!std::isfinite(gtwo)) throw Err{SLNK_ENAN, "non-finite gradient"};
      if (k <= SLNK_REPORT_MAX_ITERS) {
        rep.grel[k] = ginf / g0_inf;
        rep.J[k] = Jk;
      }
      if (ginf / g0_inf <= o.gtol_rel || ginf <= o.gtol_abs) break;
      if (k == o.max_newton) {
        status = SLNK_EMAXIT;
        break;
      }
      const double eta = std::min(0.5, gtwo / g0_two);
      const double tp = now_ms();
      int its = 0;
      if (!coarse_) {
        D3CHK(axpby<T>(s_, V, -1.0, gk_, 0.0, nullptr, b_));
        int st = 0;
        its = pcg(
            b_, eta, o.max_pcg, [&](const T* x, T* y) { matvec(x, y); },
            [&](const T* r, T* z) { prec_reg(r, z); }, rep, st);
      } else {
        // the split system (I + S Q S) s = -S g with P_2L, vt = S s; the coarse problem is
        // linearised at the restricted iterate once per Newton step
        coarse_linearize();
        apply_symbol(gk_, b_, SymArgs{Sym::RegInvSqrt, p_.reg, p_.beta, 0});
        D3CHK(axpby<T>(s_, V, -1.0, b_, 0.0, nullptr, b_));
        auto op = [&](const T* x, T* y) { split_matvec(x, y); };
        auto pr = [&](const T* r, T* z) {
          const double t = now_ms();
          apply_two_level(r, z);
          rep.coarse_matvecs += coarse_pcg_ ? last_inner_ : std::max(p_.cheb_iters - 1, 0);
          rep.time_precond_ms += now_ms() - t;
        };
        int st = 0;
        outer_tol_ = eta;  // PCG(eps) solves the coarse system to eps times the forcing term
        its = pcg(b_, eta, o.max_pcg, op, pr, rep, st);
        if (st == kIndefinite && !coarse_pcg_) {  // section 4.2.1: re-estimate the eigenvalues and run again
          reestimate_emax();
          ++rep.cheb_reestimates;
          int its2 = pcg(b_, eta, o.max_pcg, op, pr, rep, st);
          its += its2;
        }
        if (st == kIndefinite) {
          rep.pcg_iters += its;
          status = SLNK_ECHEB_DIVERGED;
          break;
        }
        apply_symbol(x_, x_, SymArgs{Sym::RegInvSqrt, p_.reg, p_.beta, 0});
      }
      rep.time_pcg_ms += now_ms() - tp;
      rep.pcg_iters += its;
      if (k < SLNK_REPORT_MAX_ITERS) rep.pcg[k] = its;
      const double slope = cell_ * reduce(0, V, gk_, x_);
      const double tl = now_ms();
      double alpha = 1.0;
      bool accepted = false;
      for (int h = 0; h <= o.max_halvings; ++h) {
        D3CHK(axpby<T>(s_, V, 1.0, vk_, alpha, x_, trial_));
        linearize(trial_);
        ++rep.line_search_evals;
        if (J_ <= Jk + o.armijo_c1 * alpha * slope) {
          accepted = true;
          break;
        }
        alpha *= 0.5;
      }
      rep.time_linesearch_ms += now_ms() - tl;
      if (!accepted) {
        status = SLNK_ELINESEARCH;
        break;
      }
      std::swap(vk_, trial_);
      Jk = J_;
      tg = now_ms();
      gradient_at(gk_);
      rep.time_gradient_ms += now_ms() - tg;
      rep.newton_iters = k + 1;
    }
    D3CHK(hipMemcpyAsync(vin, vk_, V * sizeof(T), hipMemcpyDeviceToDevice, s_));
    D3CHK(hipStreamSynchronize(s_));
    rep.status = status;
    if (coarse_) rep.emax = emax_;
    rep.time_total_ms = now_ms() - t0;
    rep.time_to_stop_ms = rep.time_total_ms;
    return status;
  }

 private:
  void release() {
    if (hres_) (void)hipHostFree(hres_);
    if (base_) (void)hipFree(base_);
    hres_ = nullptr;
    base_ = nullptr;
  }

  void need_images() const {
    if (!images_) throw Err{SLNK_EINVAL, "slnk3_set_images must come first"};
  }

  template <typename U>
  U* take(size_t n) {
    const size_t off = (used_ + 255) / 256 * 256;
    used_ = off + n * sizeof(U);
    return reinterpret_cast<U*>(base_ + off);
  }

  void carve() {
    used_ = 0;
    const size_t V = 3 * F_;
    const int nt = p_.nt;
    tw1_ = take<cplx<T>>(d_.n1 / 2);
    tw2_ = take<cplx<T>>(d_.n2 / 2);
    tw3_ = take<cplx<T>>(d_.n3 / 2);
    mR_ = take<T>(F_);
    mT_ = take<T>(F_);
    v_ = take<T>(V);
    cv_ = take<T>(V);
    divv_ = take<T>(F_);
    cdiv_ = take<T>(F_);
    df_ = take<T>(V);
    da_ = take<T>(V);
    gamma_ = take<T>(F_);
    Av_ = take<T>(V);
    m_ = take<T>(size_t(nt + 1) * F_);
    gm_ = take<T>(size_t(nt + 1) * V);
    lam0_ = take<T>(F_);
    lam1_ = take<T>(F_);
    coef_ = take<T>(F_);
    acc_ = take<T>(V);
    t3a_ = take<T>(V);
    t3b_ = take<T>(V);
    vk_ = take<T>(V);
    gk_ = take<T>(V);
    trial_ = take<T>(V);
    x_ = take<T>(V);
    r_ = take<T>(V);
    z_ = take<T>(V);
    pp_ = take<T>(V);
    q_ = take<T>(V);
    b_ = take<T>(V);
    st_ = take<T>(V);
    Sr_ = take<cplx<T>>(3 * Fh_);
    S1_ = take<cplx<T>>(3 * Fh_);
    S2_ = take<cplx<T>>(3 * Fh_);
    if constexpr (std::is_same_v<T, float>) {  // FP64 beta A of the mixed context
      twd1_ = take<cplx<double>>(d_.n1 / 2);
      twd2_ = take<cplx<double>>(d_.n2 / 2);
      twd3_ = take<cplx<double>>(d_.n3 / 2);
      Sd_ = take<cplx<double>>(3 * Fh_);
    }
    partial_ = take<double>(size_t(reduce_blocks(V)));
    dres_ = take<double>(8);
    pcg_sc_ = take<double>(8);
    lz_cap_ = std::min(std::max(p_.lanczos_steps, 1), kMaxLanczos);
    lz_ = take<double>(4 + 2 * size_t(lz_cap_));
    lz_live_ = take<int>(1);
    if (rk_) {
      rk_g_ = take<T>(V);
      rk_yv_ = take<T>(V);
      rk_gl_ = take<T>(V);
      rk_glm_ = take<T>(V);
      rk_dv_ = take<T>(F_);
      rk_dvs_ = take<T>(F_);
      rk_tmp_ = take<T>(F_);
      rk_k_ = take<T>(F_);
      rk_p_ = take<T>(F_);
      rk_divt_ = take<T>(F_);
      for (auto& y : rk_y_) y = take<T>(F_);
      for (auto& y : rk_src_) y = take<T>(F_);
    }
    if (fn_) {
      lamk_ = take<T>(size_t(nt + 1) * F_);
      sig_[0] = take<T>(F_);
      sig_[1] = take<T>(F_);
      e_ = take<T>(F_);
      mtj_ = take<T>(F_);
      accfn_ = take<T>(V);
    }
  }

  void allocate() {
    base_ = nullptr;
    carve();  // sizes only (base_ null)
    bytes = used_ + 256;
    if (hipMalloc(reinterpret_cast<void**>(&base_), bytes) != hipSuccess) {
      base_ = nullptr;
      (void)hipGetLastError();
      throw Err{SLNK_ENOMEM, "workspace allocation failed"};
    }
    carve();
    D3CHK(hipHostMalloc(reinterpret_cast<void**>(&hres_), 8 * sizeof(double), hipHostMallocDefault));
    D3CHK(hipMemsetAsync(base_, 0, bytes, s_));
    upload_twiddles(tw1_, d_.n1);
    upload_twiddles(tw2_, d_.n2);
    upload_twiddles(tw3_, d_.n3);
    tw_.t1 = tw1_;
    tw_.t2 = tw2_;
    tw_.t3 = tw3_;
    if constexpr (std::is_same_v<T, float>) {
      upload_twiddles(twd1_, d_.n1);
      upload_twiddles(twd2_, d_.n2);
      upload_twiddles(twd3_, d_.n3);
      twd_.t1 = twd1_;
      twd_.t2 = twd2_;
      twd_.t3 = twd3_;
    }
  }

  // twiddles exp(-2 pi i j / n), j < n/2, computed in FP64 and rounded to U
  template <typename U>
  void upload_twiddles(cplx<U>* dst, int n) {
    std::vector<cplx<U>> h(n / 2);
    for (int j = 0; j < n / 2; ++j) {
      const double a = -2.0 * 3.14159265358979323846 * j / n;
      h[j] = cplx<U>{U(std::cos(a)), U(std::sin(a))};
    }
    D3CHK(hipMemcpyAsync(dst, h.data(), h.size() * sizeof(cplx<U>), hipMemcpyHostToDevice, s_));
    D3CHK(hipStreamSynchronize(s_));
  }

  // out = beta A x (a vector field).  The mixed context forms it in FP64 and rounds once: the
  // symbol beta |k|^(2 reg) would otherwise multiply the FP32 rounding of the transform of x by up
  // to beta max a(k).
  void reg_apply(const T* x, T* out, double beta) {
    const SymArgs a{Sym::Reg, p_.reg, beta, 0};
    if constexpr (std::is_same_v<T, float>) {
      D3CHK((spec_apply<double, float>(s_, d_, twd_, SpecOp::Scale, 3, a, x, out, Sd_, Sd_)));
    } else {
      apply_symbol(x, out, a);
    }
  }

  // FP64 reduction of n values (mode 0: sum a b, 1: sum (a - b)^2, 2: max |a|), read on the host
  double reduce(int mode, size_t n, const T* a, const T* b) {
    D3CHK(d3::reduce<T>(s_, n, mode, a, b, partial_, dres_));
    D3CHK(hipMemcpyAsync(hres_, dres_, sizeof(double), hipMemcpyDeviceToHost, s_));
    D3CHK(hipStreamSynchronize(s_));
    return hres_[0];
  }

  // B-spline coefficients of nf fields (nf = 1 or 3): the periodic inverse of the (1, 4, 1)/6
  // system along each axis (section 3.3.2, "Interpolation") by the truncated exponential filter
  void coefficients(const T* f, T* c, int nf) { D3CHK(spline_coefficients<T>(s_, d_, nf, f, c)); }

  // out = symbol(in) for a vector field (with the Leray projection first when a.proj)
  void apply_symbol(const T* in, T* out, SymArgs a) {
    D3CHK((spec_apply<T, T>(s_, d_, tw_, SpecOp::Scale, 3, a, in, out, S1_, S2_)));
  }

  void gradient_of(const T* f, T* g) {
    D3CHK((spec_apply<T, T>(s_, d_, tw_, SpecOp::Grad, 1, SymArgs{}, f, g, S1_, S2_)));
  }

  void divergence_of(const T* v, T* out) {
    D3CHK((spec_apply<T, T>(s_, d_, tw_, SpecOp::Div, 3, SymArgs{}, v, out, S1_, S2_)));
  }

  // characteristics and adjoint factor of v (copied into v_)
  void trace_at(const T* v) {
    if (v != v_) D3CHK(hipMemcpyAsync(v_, v, 3 * F_ * sizeof(T), hipMemcpyDeviceToDevice, s_));
    if (!std::isfinite(reduce(0, 3 * F_, v_, v_))) throw Err{SLNK_ENAN, "non-finite velocity"};
    coefficients(v_, cv_, 3);
    divergence_of(v_, divv_);
    coefficients(divv_, cdiv_, 1);
    D3CHK(d3::trace<T>(s_, d_, ht_, v_, cv_, divv_, cdiv_, df_, da_, gamma_));
    // whole cells bounding every departure displacement (selects the LDS-staged step kernel)
    const double dmax = std::max(reduce(2, 3 * F_, df_, nullptr), reduce(2, 3 * F_, da_, nullptr));
    halo_ = p_.sl_path == 0 && dmax < 1e6 ? int(std::ceil(dmax)) : -1;
  }

  // trace, state m^0..m^nt (eq. e:state-slm), grad m^j, A v and J
  void linearize(const T* v) {
    const size_t V = 3 * F_;
    if (rk_) {
      rk_prepare(v);
      D3CHK(hipMemcpyAsync(m_, mT_, F_ * sizeof(T), hipMemcpyDeviceToDevice, s_));
      D3CHK(scale_vec<T>(s_, d_, m_, v_, rk_yv_));
      for (int j = 1; j <= p_.nt; ++j) rk_step(-1, -1, m_ + size_t(j - 1) * F_, m_ + size_t(j) * F_, nullptr, nullptr);
    } else {
      trace_at(v);
      D3CHK(hipMemcpyAsync(m_, mT_, F_ * sizeof(T), hipMemcpyDeviceToDevice, s_));
    }
    for (int j = 1; j <= p_.nt && !rk_; ++j) {
      coefficients(m_ + size_t(j - 1) * F_, coef_, 1);
      StepArgs<T> a;
      a.d = d_;
      a.halo = halo_;
      a.kind = Kind::State;
      a.coef = coef_;
      a.disp = df_;
      a.dst = m_ + size_t(j) * F_;
      D3CHK(sl_step<T>(s_, a));
    }
    for (int j = 0; j <= p_.nt; ++j) gradient_of(m_ + size_t(j) * F_, gm_ + size_t(j) * V);
    reg_apply(v_, Av_, 1.0);
    const double mis = reduce(1, F_, m_ + size_t(p_.nt) * F_, mR_);
    const double reg = reduce(0, V, v_, Av_);
    J_ = 0.5 * cell_ * mis + 0.5 * p_.beta * cell_ * reg;
    if (!std::isfinite(J_)) throw Err{SLNK_ENAN, "non-finite objective"};
    lin_ = true;
    lam_ok_ = false;
    coarse_lin_ = false;
  }

  // g = beta A v + K b, b = int lambda grad m dt (adjoint eq. e:adj-slm backward from lambda(1) = m_R - m(1));
  // the full-Newton context keeps lambda^0..lambda^nt in lamk_
  void gradient_at(T* g) {
    const size_t V = 3 * F_;
    const int nt = p_.nt;
    if (rk_) {  // RK2A: lambda^nt = m_R - m^nt, Heun on d_s lam = A lam, b in its antisymmetric form
      D3CHK(axpby<T>(s_, F_, 1.0, mR_, -1.0, m_ + size_t(nt) * F_, rk_level(nt, fn_)));
      rk_adjoint_sweep(fn_, true, nullptr);
      project_and_add(p_.beta, Av_, g);
      lam_ok_ = true;
      return;
    }
    T* lam1 = fn_ ? lamk_ + size_t(nt) * F_ : lam1_;
    D3CHK(adjoint_start<T>(s_, d_, trap_w(nt, nt), mR_, m_ + size_t(nt) * F_, gm_ + size_t(nt) * V, lam1, acc_));
    backward_sweep(lam1, Kind::Adjoint);
    project_and_add(p_.beta, Av_, g);
    lam_ok_ = true;
  }

  // ---- stabilised RK2 (RK2A) transport ---------------------------------------------------------
  // v into v_ and div v (no characteristics)
  void rk_prepare(const T* v) {
    if (v != v_) D3CHK(hipMemcpyAsync(v_, v, 3 * F_ * sizeof(T), hipMemcpyDeviceToDevice, s_));
    if (!std::isfinite(reduce(0, 3 * F_, v_, v_))) throw Err{SLNK_ENAN, "non-finite velocity"};
    divergence_of(v_, divv_);
  }

  // one Heun step of dy/ds = sgn L_dsgn y + src from y0 into dst (src0, src1: the sources at the
  // step's two ends, or null); rk_yv_ holds y0 v on entry and dst v on exit
  void rk_step(int sgn, int dsgn, const T* y0, T* dst, const T* src0, const T* src1) {
    RkStage<T> a;
    a.sgn = sgn;
    a.dsgn = dsgn;
    a.ht = ht_;
    a.g = rk_g_;
    a.dv = rk_dv_;
    a.v = v_;
    a.divv = divv_;
    a.kbuf = rk_k_;
    a.yv = rk_yv_;
    gradient_of(y0, rk_g_);
    divergence_of(rk_yv_, rk_dv_);
    a.stage = 1;
    a.y = y0;
    a.src = src0;
    a.dst = rk_tmp_;
    D3CHK(rk_stage<T>(s_, d_, a));
    gradient_of(rk_tmp_, rk_g_);
    divergence_of(rk_yv_, rk_dv_);
    a.stage = 2;
    a.y = rk_tmp_;
    a.src = src1;
    a.y0 = y0;
    a.dst = dst;
    D3CHK(rk_stage<T>(s_, d_, a));
  }

  // acc (init: =, else +=) w_j 1/2 (lam grad m - m grad lam + grad(lam m)) for m = m~ (its gradient in
  // gm) or the state m^j
  void rk_accumulate(int j, const T* lam, const T* m, const T* gm, bool init) {
    gradient_of(lam, rk_gl_);
    D3CHK(mul<T>(s_, d_, lam, m, rk_p_));
    gradient_of(rk_p_, rk_glm_);
    D3CHK(rk_accum<T>(s_, d_, trap_w(j, p_.nt), init, lam, m, gm, rk_gl_, rk_glm_, acc_));
  }

  // time level j of an RK2A adjoint sweep: every level in lamk_ (keep: the full-Newton gradient),
  // else two rotating fields
  T* rk_level(int j, bool keep) { return keep ? lamk_ + size_t(j) * F_ : rk_y_[j & 1]; }

  // d_s y = A y (+ the full-Newton source when vt is given) from y^nt at rk_level(nt, keep) back to
  // t = 0, acc (init: set by the first term) += w_j 1/2 (y grad m - m grad y + grad(y m)) at every level
  void rk_adjoint_sweep(bool keep, bool init, const T* vt) {
    const size_t V = 3 * F_;
    const int nt = p_.nt;
    // 1/2 (div(lam^j vt) + vt . grad lam^j + lam^j div vt): the full-Newton incremental adjoint's source
    auto source = [&](int j, T* out) -> const T* {
      if (!vt) return nullptr;
      const T* lj = lamk_ + size_t(j) * F_;
      gradient_of(lj, t3b_);
      D3CHK(scale_vec<T>(s_, d_, lj, vt, t3a_));
      divergence_of(t3a_, rk_dvs_);
      D3CHK(rk_eval<T>(s_, d_, +1, +1, t3b_, rk_dvs_, lj, vt, rk_divt_, out));
      return out;
    };
    rk_accumulate(nt, rk_level(nt, keep), m_ + size_t(nt) * F_, gm_ + size_t(nt) * V, init);
    D3CHK(scale_vec<T>(s_, d_, rk_level(nt, keep), v_, rk_yv_));
    const T* s_hi = source(nt, rk_src_[nt & 1]);
    for (int j = nt; j >= 1; --j) {
      const T* s_lo = source(j - 1, rk_src_[(j - 1) & 1]);
      rk_step(+1, +1, rk_level(j, keep), rk_level(j - 1, keep), s_hi, s_lo);
      rk_accumulate(j - 1, rk_level(j - 1, keep), m_ + size_t(j - 1) * F_, gm_ + size_t(j - 1) * V, false);
      s_hi = s_lo;
    }
  }

  // b~ of the RK2A matvec into acc_: the incremental state d_t m~ = -L m~ - S(m) vt from m~ = 0
  // (S(m) vt = 1/2 (div(m vt) + vt . grad m - m div vt)), then the adjoint equation from -m~(1) with b~
  // in its antisymmetric form; full Newton adds the lambda terms (the incremental adjoint's source,
  // and 1/2 (lam grad m~ - m~ grad lam + grad(lam m~)) in b~, added as each m~^j is formed)
  void rk_transport(const T* vt) {
    const size_t V = 3 * F_;
    const int nt = p_.nt;
    divergence_of(vt, rk_divt_);
    auto source = [&](int j, T* out) {
      D3CHK(scale_vec<T>(s_, d_, m_ + size_t(j) * F_, vt, t3a_));
      divergence_of(t3a_, rk_dvs_);
      D3CHK(rk_eval<T>(s_, d_, -1, -1, gm_ + size_t(j) * V, rk_dvs_, m_ + size_t(j) * F_, vt, rk_divt_, out));
    };
    source(0, rk_src_[0]);
    D3CHK(axpby<T>(s_, F_, 0.0, nullptr, 0.0, nullptr, rk_y_[0]));
    D3CHK(axpby<T>(s_, V, 0.0, nullptr, 0.0, nullptr, rk_yv_));
    for (int j = 1; j <= nt; ++j) {
      source(j, rk_src_[j & 1]);
      rk_step(-1, -1, rk_y_[(j - 1) & 1], rk_y_[j & 1], rk_src_[(j - 1) & 1], rk_src_[j & 1]);
      if (fn_) {
        gradient_of(rk_y_[j & 1], t3b_);
        rk_accumulate(j, lamk_ + size_t(j) * F_, rk_y_[j & 1], t3b_, j == 1);
      }
    }
    D3CHK(axpby<T>(s_, F_, -1.0, rk_y_[nt & 1], 0.0, nullptr, rk_y_[nt & 1]));  // lam~(1) = -m~(1)
    rk_adjoint_sweep(false, !fn_, fn_ ? vt : nullptr);
  }

  // sigma^j = div(lambda^j vt), the source of the full-Newton incremental adjoint at time level j
  void sigma_at(int j, const T* vt, T* out) {
    D3CHK(scale_vec<T>(s_, d_, lamk_ + size_t(j) * F_, vt, t3b_));
    divergence_of(t3b_, out);
  }

  // adjoint-type sweep j = nt .. 1 from the field in 'start': lambda^{j-1} = gamma I[lambda^j](x + da),
  // acc += w_{j-1} lambda^{j-1} grad m^{j-1}.  The full-Newton context keeps every adjoint level in
  // lamk_; with vt given (full-Newton incremental adjoint), Heun's step along the adjoint
  // characteristic adds the source sigma = div(lambda vt): ht/2 (1 + ht div v) sigma^j at the
  // departure point and ht/2 sigma^{j-1} at the node.
  void backward_sweep(T* start, Kind kind, const T* vt = nullptr) {
    const size_t V = 3 * F_;
    const bool keep = fn_ && kind == Kind::Adjoint;
    T* cur = start;
    T* nxt = start == lam0_ ? lam1_ : lam0_;
    if (vt) sigma_at(p_.nt, vt, sig_[p_.nt % 2]);
    for (int j = p_.nt; j >= 1; --j) {
      if (keep) nxt = lamk_ + size_t(j - 1) * F_;
      const T* add = nullptr;
      if (vt) {
        sigma_at(j - 1, vt, sig_[(j - 1) % 2]);
        coefficients(sig_[j % 2], coef_, 1);
        StepArgs<T> b;
        b.d = d_;
        b.halo = halo_;
        b.kind = Kind::State;
        b.coef = coef_;
        b.disp = da_;
        b.dst = e_;
        D3CHK(sl_step<T>(s_, b));
        D3CHK(fn_source<T>(s_, d_, ht_, divv_, e_, sig_[(j - 1) % 2], e_));
        add = e_;
      }
      coefficients(cur, coef_, 1);
      StepArgs<T> a;
      a.d = d_;
      a.halo = halo_;
      a.kind = kind;
      a.coef = coef_;
      a.disp = da_;
      a.gamma = gamma_;
      a.gm = gm_ + size_t(j - 1) * V;
      a.dst = nxt;
      a.acc = acc_;
      a.add = add;
      a.w = trap_w(j - 1, p_.nt);
      D3CHK(sl_step<T>(s_, a));
      if (keep)
        cur = nxt;
      else
        std::swap(cur, nxt);
    }
  }

  // out = c add + K acc (K the Leray projection or the identity)
  void project_and_add(double c, const T* add, T* out) {
    const T* kb = acc_;
    if (p_.proj) {
      apply_symbol(acc_, t3b_, SymArgs{Sym::One, p_.reg, 1.0, 1});
      kb = t3b_;
    }
    D3CHK(axpby<T>(s_, 3 * F_, c, add, 1.0, kb, out));  // add may be null (c = 0)
  }

  // Gauss--Newton matvec: incremental state (eq. e:inc-state-slm) forward from m~(0) = 0, the
  // incremental adjoint (eq. e:inc-adj-slm, lambda terms dropped) backward from -m~(1), then
  // beta A vt + K int lambda~ grad m dt (with_reg false: the transport part Q alone).  Full Newton:
  // the incremental adjoint keeps its source div(lambda vt) and b~ adds int lambda grad m~ dt,
  // lambda from the gradient at this linearisation.
  void matvec(const T* vt, T* out, bool with_reg = true) {
    const size_t V = 3 * F_;
    const int nt = p_.nt;
    if (fn_ && !lam_ok_)
      throw Err{SLNK_EINVAL, "the full-Newton matvec needs the gradient at this point (slnk3_gradient)"};
    if (rk_) {
      rk_transport(vt);
      if (with_reg) {
        reg_apply(vt, t3a_, p_.beta);
        project_and_add(1.0, t3a_, out);
      } else {
        project_and_add(0.0, nullptr, out);
      }
      return;
    }
    D3CHK(incstate_start<T>(s_, d_, ht_, vt, gm_, lam0_));
    T* cur = lam0_;
    T* nxt = lam1_;
    for (int j = 1; j <= nt; ++j) {
      coefficients(cur, coef_, 1);
      StepArgs<T> a;
      a.d = d_;
      a.halo = halo_;
      a.kind = Kind::IncState;
      a.coef = coef_;
      a.disp = df_;
      a.gm = gm_ + size_t(j) * V;
      a.vt = vt;
      a.dst = nxt;
      a.acc = acc_;
      a.w = trap_w(nt, nt);
      a.ht = ht_;
      a.last = j == nt;
      a.mt = fn_ ? mtj_ : nullptr;
      D3CHK(sl_step<T>(s_, a));
      if (fn_) {  // lambda^j grad m~^j (m~^0 = 0 adds nothing)
        gradient_of(mtj_, t3a_);
        D3CHK(acc_scalar_grad<T>(s_, d_, trap_w(j, nt), j == 1, lamk_ + size_t(j) * F_, t3a_, accfn_));
      }
      std::swap(cur, nxt);
    }
    backward_sweep(cur, Kind::IncAdjoint, fn_ ? vt : nullptr);
    if (fn_) D3CHK(axpby<T>(s_, V, 1.0, acc_, 1.0, accfn_, acc_));
    if (with_reg) {
      reg_apply(vt, t3a_, p_.beta);
      project_and_add(1.0, t3a_, out);
    } else {
      project_and_add(0.0, nullptr, out);
    }
  }

  void prec_reg(const T* r, T* z) { apply_symbol(r, z, SymArgs{Sym::RegInv, p_.reg, p_.beta, 0}); }

  // M s = s + S Q S s, S = (beta A')^{-1/2}: the split spectrally preconditioned Hessian
  // (section 3.4.2) at this level's linearisation
  void split_matvec(const T* sv, T* out) {
    const SymArgs S{Sym::RegInvSqrt, p_.reg, p_.beta, 0};
    apply_symbol(sv, st_, S);
    matvec(st_, out, false);
    apply_symbol(out, out, S);
    D3CHK(axpby<T>(s_, 3 * F_, 1.0, out, 1.0, sv, out));
  }

  // M s at v = 0 in closed form (the set-up's Lanczos operator): Q S s = K (S s . grad m_T) grad m_T,
  // grad m_T in gm_ (level 0)
  void split_matvec_zero(const T* sv, T* out) {
    const SymArgs S{Sym::RegInvSqrt, p_.reg, p_.beta, 0};
    apply_symbol(sv, st_, S);
    D3CHK(q_at_zero<T>(s_, d_, st_, gm_, acc_));
    project_and_add(0.0, nullptr, out);
    apply_symbol(out, out, S);
    D3CHK(axpby<T>(s_, 3 * F_, 1.0, out, 1.0, sv, out));
  }

  // ---- two-level preconditioner (section 3.4.2, "Nested Preconditioner") ---------------------
  // spectral restriction of nf fine fields into the coarse level's fields
  void restrict_to_coarse(const T* f, T* c, int nf) {
    D3CHK(fft_forward<T>(s_, d_, tw_, nf, f, S1_));
    D3CHK(spec_restrict<T>(s_, d_, coarse_->d_, nf, S1_, coarse_->S1_));
    D3CHK(fft_inverse<T>(s_, coarse_->d_, coarse_->tw_, nf, coarse_->S1_, c));
  }

  // the coarse problem linearised at the restricted current point (once per point)
  void coarse_linearize() {
    if (coarse_lin_) return;
    restrict_to_coarse(v_, coarse_->trial_, 3);
    coarse_->linearize(coarse_->trial_);
    coarse_lin_ = true;
  }

  // coarse images, Lanczos e_max at v = 0, analytic e_min
  void setup_two_level() {
    restrict_to_coarse(mR_, coarse_->mR_, 1);
    restrict_to_coarse(mT_, coarse_->mT_, 1);
    coarse_->images_ = true;
    // the split operator at v = 0 needs grad m_T alone (m is m_T at every time)
    coarse_->gradient_of(coarse_->mT_, coarse_->gm_);
    emax_setup_ = p_.emax_safety * coarse_->lanczos_max(p_.lanczos_steps, p_.lanczos_seed, true);
    emax_ = emax_setup_;
    // e_min = min_k 1 + 1 / (beta a'(k)) over the coarse modes: the largest |k|^2 is at the corner
    const Dims& c = coarse_->d_;
    const double kk = 0.25 * (double(c.n1) * c.n1 + double(c.n2) * c.n2 + double(c.n3) * c.n3);
    emin_ = 1.0 + 1.0 / (p_.beta * std::pow(kk, p_.reg));
    coarse_lin_ = false;
  }

  // a new e_max when CHEB(k) turned out indefinite: Lanczos at the current coarse linearisation
  void reestimate_emax() { emax_ = p_.emax_safety * coarse_->lanczos_max(p_.lanczos_steps, p_.lanczos_seed); }

  // largest Ritz value of 'steps' Lanczos steps on this level's split operator from the
  // SplitMix64 start vector (no re-orthogonalisation; stops at breakdown): at this level's
  // linearisation, or at v = 0 in closed form (at_zero)
  double lanczos_max(int steps, unsigned long long seed, bool at_zero = false) {
    if (steps < 1 || steps > lz_cap_) throw Err{SLNK_EINVAL, "lanczos_steps out of range"};
    const size_t V = 3 * F_;
    const std::vector<double> h = splitmix_uniform(seed, V);
    std::vector<T> ht(h.begin(), h.end());
    T* q = x_;
    T* qp = r_;
    T* w = q_;
    D3CHK(hipMemcpyAsync(q, ht.data(), V * sizeof(T), hipMemcpyHostToDevice, s_));
    const double nq = std::sqrt(reduce(0, V, q, q));  // synchronises before ht is released
    D3CHK(axpby<T>(s_, V, 1.0 / nq, q, 0.0, nullptr, q));
    D3CHK(hipMemsetAsync(qp, 0, V * sizeof(T), s_));
    // the step scalars stay on the device (the 2-D library's k_lanczos_coef, one item); the
    // (alpha, beta) log is read once
    double* alpha = lz_;
    double* beta = lz_ + 1;
    double* inv = lz_ + 2;
    double* log = lz_ + 4;
    const int live = 1;
    D3CHK(set_ints(s_, lz_live_, &live, 1));
    D3CHK(fill<double>(s_, 1, 0.0, beta));
    for (int j = 0; j < steps; ++j) {
      if (at_zero)
        split_matvec_zero(q, w);
      else
        split_matvec(q, w);
      D3CHK((slnk::axpby<T>(s_, 1, V, -1.0, beta, qp, 1.0, nullptr, w)));
      D3CHK(d3::reduce<T>(s_, V, 0, q, w, partial_, dres_));
      D3CHK(lanczos_coef(s_, LANCZOS_ALPHA, 1, j, steps, dres_, lz_live_, alpha, beta, inv, log));
      D3CHK((slnk::axpby<T>(s_, 1, V, -1.0, alpha, q, 1.0, nullptr, w)));
      D3CHK(d3::reduce<T>(s_, V, 0, w, w, partial_, dres_));
      D3CHK(lanczos_coef(s_, LANCZOS_BETA, 1, j, steps, dres_, lz_live_, alpha, beta, inv, log));
      if (j == steps - 1) break;
      std::swap(qp, q);
      D3CHK((slnk::axpby<T>(s_, 1, V, 1.0, inv, w, 0.0, nullptr, q)));  // q <- w / beta
    }
    std::vector<double> lg(2 * size_t(steps));
    D3CHK(hipMemcpyAsync(lg.data(), log, lg.size() * sizeof(double), hipMemcpyDeviceToHost, s_));
    D3CHK(hipStreamSynchronize(s_));
    std::vector<double> al, be;
    for (int j = 0; j < steps; ++j) {
      al.push_back(lg[2 * j]);
      if (lg[2 * j + 1] < 0.0) break;  // last step or breakdown
      be.push_back(lg[2 * j + 1]);
    }
    return tridiag_max_eig(al, be);
  }

  // k steps of the Chebyshev iteration for M x = b from x = 0 on this level (bounds [emin, emax]);
  // the k-th update needs no new residual (k - 1 operator applications); result in x_
  void chebyshev(const T* b, double emin, double emax, int k) {
    const size_t V = 3 * F_;
    const double theta = 0.5 * (emax + emin), delta = 0.5 * (emax - emin);
    const double sigma = theta / delta;
    double rho = 1.0 / sigma;
    D3CHK(hipMemsetAsync(x_, 0, V * sizeof(T), s_));
    D3CHK(hipMemcpyAsync(r_, b, V * sizeof(T), hipMemcpyDeviceToDevice, s_));
    D3CHK(axpby<T>(s_, V, 1.0 / theta, r_, 0.0, nullptr, pp_));
    for (int i = 0; i < k; ++i) {
      D3CHK(axpby<T>(s_, V, 1.0, x_, 1.0, pp_, x_));
      if (i == k - 1) break;
      split_matvec(pp_, q_);
      D3CHK(axpby<T>(s_, V, 1.0, r_, -1.0, q_, r_));
      const double rho_next = 1.0 / (2.0 * sigma - rho);
      D3CHK(axpby<T>(s_, V, rho_next * rho, pp_, 2.0 * rho_next / delta, r_, pp_));
      rho = rho_next;
    }
  }

  // CG on this level's split operator M x = b from x = 0, the nested PCG(eps) coarse solve of
  // section 3.4.2 (M is spectrally preconditioned already: no inner preconditioner), to
  // ||b - M x|| <= tol ||b||, non-positive curvature (rounding only: M is positive definite; the
  // iterate is kept) or maxit steps.  x in x_; uses this level's r_, pp_, q_ and step scalars (the
  // fine level's PCG keeps its own across the call).  Returns the steps.
  int cg(const T* b, double tol, int maxit) {
    const size_t V = 3 * F_;
    D3CHK(hipMemsetAsync(x_, 0, V * sizeof(T), s_));
    D3CHK(hipMemcpyAsync(r_, b, V * sizeof(T), hipMemcpyDeviceToDevice, s_));
    D3CHK(hipMemcpyAsync(pp_, b, V * sizeof(T), hipMemcpyDeviceToDevice, s_));
    const double bnorm = std::sqrt(reduce(0, V, r_, r_));
    if (bnorm == 0.0) return 0;
    double* rr = pcg_sc_;
    double* alpha = pcg_sc_ + 1;
    double* c0 = pcg_sc_ + 2;
    double* c1 = pcg_sc_ + 3;
    D3CHK(d3::reduce<T>(s_, V, 0, r_, r_, partial_, dres_ + 1));
    D3CHK(pcg_coef(s_, PCG_RZ, 1, nullptr, dres_ + 1, rr, nullptr, nullptr));
    for (int it = 1; it <= maxit; ++it) {
      split_matvec(pp_, q_);
      D3CHK(d3::reduce<T>(s_, V, 0, pp_, q_, partial_, dres_));
      D3CHK(pcg_coef(s_, PCG_ALPHA, 1, nullptr, dres_, rr, alpha, nullptr));
      D3CHK((slnk::axpby<T>(s_, 1, V, 1.0, alpha, pp_, 1.0, nullptr, x_)));
      D3CHK((slnk::axpby<T>(s_, 1, V, -1.0, alpha, q_, 1.0, nullptr, r_)));
      D3CHK(d3::reduce<T>(s_, V, 0, r_, r_, partial_, dres_ + 1));
      D3CHK(hipMemcpyAsync(hres_, dres_, 2 * sizeof(double), hipMemcpyDeviceToHost, s_));
      D3CHK(hipStreamSynchronize(s_));
      const double pq = hres_[0], rrh = hres_[1];
      if (!std::isfinite(pq) || !std::isfinite(rrh)) throw Err{SLNK_ENAN, "non-finite coarse CG"};
      if (!(pq > 0.0) || std::sqrt(rrh) <= tol * bnorm) return it;
      // p <- r + (r.r new / r.r) p
      D3CHK(pcg_coef(s_, PCG_BETA, 1, nullptr, dres_ + 1, rr, c0, c1));
      D3CHK((slnk::axpby<T>(s_, 1, V, 1.0, c0, r_, 1.0, c1, pp_)));
    }
    return maxit;
  }

  // P_2L^{-1} r = (I - L) r + Pro C(M_c) Res r, the low/high split and both transfers spectral; C =
  // CHEB(k), or PCG(eps) to eps times outer_tol_ (the forcing term of the outer solve, 1 outside it)
  void apply_two_level(const T* r, T* z) {
    Ctx<T>& c = *coarse_;
    D3CHK(fft_forward<T>(s_, d_, tw_, 3, r, Sr_));
    D3CHK(spec_restrict<T>(s_, d_, c.d_, 3, Sr_, c.S1_));
    D3CHK(fft_inverse<T>(s_, c.d_, c.tw_, 3, c.S1_, c.b_));
    if (coarse_pcg_)
      last_inner_ = c.cg(c.b_, p_.coarse_eps * outer_tol_, kMaxInner);
    else
      c.chebyshev(c.b_, emin_, emax_, p_.cheb_iters);
    D3CHK(fft_forward<T>(s_, c.d_, c.tw_, 3, c.x_, c.S1_));
    D3CHK(spec_prolong_combine<T>(s_, d_, c.d_, 3, Sr_, c.S1_));
    D3CHK(fft_inverse<T>(s_, d_, tw_, 3, Sr_, z));
  }

  static constexpr int kIndefinite = 1;

  // PCG from x = 0 to ||r|| <= tol ||b|| (Euclidean products, the oracle's pcg): stops on
  // non-positive curvature (x = the preconditioned residual at the first step), or with status
  // kIndefinite when the r.z that gave a step was not positive.  Returns the iterations; the
  // step is left in x_.
  template <class Op, class Prec>
  int pcg(const T* b, double tol, int maxit, Op&& op, Prec&& prec, slnk_solve_report& rep, int& status) {
    const size_t V = 3 * F_;
    status = 0;
    D3CHK(hipMemcpyAsync(r_, b, V * sizeof(T), hipMemcpyDeviceToDevice, s_));
    D3CHK(hipMemsetAsync(x_, 0, V * sizeof(T), s_));
    const double bnorm = std::sqrt(reduce(0, V, r_, r_));
    if (bnorm == 0.0) return 0;
    prec(r_, z_);
    D3CHK(hipMemcpyAsync(pp_, z_, V * sizeof(T), hipMemcpyDeviceToDevice, s_));
    // the step coefficients stay on the device (the 2-D library's k_pcg_coef, one item): p.q,
    // r.r and r.z land in dres_[0..2], and one read per iteration returns p.q, r.r and the r.z
    // that made the step
    double* rz = pcg_sc_;
    double* alpha = pcg_sc_ + 1;
    double* c0 = pcg_sc_ + 2;
    double* c1 = pcg_sc_ + 3;
    D3CHK(d3::reduce<T>(s_, V, 0, r_, z_, partial_, dres_ + 2));
    D3CHK(pcg_coef(s_, PCG_RZ, 1, nullptr, dres_ + 2, rz, nullptr, nullptr));
    for (int it = 1; it <= maxit; ++it) {
      op(pp_, q_);
      ++rep.matvecs;
      D3CHK(d3::reduce<T>(s_, V, 0, pp_, q_, partial_, dres_));
      // alpha = rz / pq, 0 where pq is not positive and finite (the updates then leave x, r as
      // they are)
      D3CHK(pcg_coef(s_, PCG_ALPHA, 1, nullptr, dres_, rz, alpha, nullptr));
      D3CHK((slnk::axpby<T>(s_, 1, V, 1.0, alpha, pp_, 1.0, nullptr, x_)));
      D3CHK((slnk::axpby<T>(s_, 1, V, -1.0, alpha, q_, 1.0, nullptr, r_)));
      D3CHK(d3::reduce<T>(s_, V, 0, r_, r_, partial_, dres_ + 1));
      D3CHK(hipMemcpyAsync(hres_, dres_, 2 * sizeof(double), hipMemcpyDeviceToHost, s_));
      D3CHK(hipMemcpyAsync(hres_ + 2, rz, sizeof(double), hipMemcpyDeviceToHost, s_));
      D3CHK(hipStreamSynchronize(s_));
      const double pq = hres_[0], rr = hres_[1], rzh = hres_[2];
      if (!(pq > 0.0)) {
        if (it == 1) D3CHK(hipMemcpyAsync(x_, z_, V * sizeof(T), hipMemcpyDeviceToDevice, s_));
        return it;
      }
      if (std::sqrt(rr) <= tol * bnorm) return it;
      if (!(rzh > 0.0)) {
        status = kIndefinite;
        return it;
      }
      prec(r_, z_);
      D3CHK(d3::reduce<T>(s_, V, 0, r_, z_, partial_, dres_ + 2));
      // p <- z + (rz_new / rz) p, rz <- rz_new
      D3CHK(pcg_coef(s_, PCG_BETA, 1, nullptr, dres_ + 2, rz, c0, c1));
      D3CHK((slnk::axpby<T>(s_, 1, V, 1.0, c0, z_, 1.0, c1, pp_)));
    }
    return maxit;
  }

  slnk3_params p_;
  hipStream_t s_;
  Dims d_;
  size_t F_ = 0, Fh_ = 0;
  double ht_ = 0.0, cell_ = 0.0, J_ = 0.0;
  int halo_ = -1;
  std::unique_ptr<Ctx<T>> coarse_;  // P_2L's coarse level (pc = SLNK_PC_2L)
  bool coarse_lin_ = false;          // the coarse level is linearised at the restricted current point
  double emin_ = 0.0, emax_ = 0.0, emax_setup_ = 0.0;
  bool images_ = false, lin_ = false;
  // full-Newton matvec (this level; the coarse level of P_2L stays Gauss--Newton): lambda^0..nt of
  // the last gradient (lam_ok_: taken at the current linearisation), sigma at two levels, the
  // interpolated source, m~^j, and the lambda grad m~ part of b~
  bool fn_ = false, lam_ok_ = false;
  // P_2L's coarse solver: CHEB(k), or PCG(eps) (at most kMaxInner steps; last_inner_: the steps
  // of the last application) to eps times outer_tol_
  bool coarse_pcg_ = false;
  // RK2A transport (P_REG): derivatives of the Heun stage's input, its products with v, grad lambda and
  // grad(lambda m) of the b-form, div(y v) of the step and of a source, the stage value and slope,
  // lambda m, div vt, two rotating levels and two source levels
  bool rk_ = false;
  T* rk_g_ = nullptr;
  T* rk_yv_ = nullptr;
  T* rk_gl_ = nullptr;
  T* rk_glm_ = nullptr;
  T* rk_dv_ = nullptr;
  T* rk_dvs_ = nullptr;
  T* rk_tmp_ = nullptr;
  T* rk_k_ = nullptr;
  T* rk_p_ = nullptr;
  T* rk_divt_ = nullptr;
  T* rk_y_[2] = {};
  T* rk_src_[2] = {};
  double outer_tol_ = 1.0;
  int last_inner_ = 0;
  static constexpr int kMaxInner = 200;
  T* lamk_ = nullptr;
  T* sig_[2] = {};
  T* e_ = nullptr;
  T* mtj_ = nullptr;
  T* accfn_ = nullptr;
  char* base_ = nullptr;
  size_t used_ = 0;
  double* hres_ = nullptr;
  // PCG: device scalars rz, alpha, (1, beta) of the step updates
  double* pcg_sc_ = nullptr;
  // Lanczos: device scalars alpha, beta, 1 / beta, then the (alpha, beta) log of up to lz_cap_ steps
  static constexpr int kMaxLanczos = 1000;
  int lz_cap_ = 0;
  double* lz_ = nullptr;
  int* lz_live_ = nullptr;
  Twiddles<T> tw_;
  cplx<T>*tw1_ = nullptr, *tw2_ = nullptr, *tw3_ = nullptr;
  T *mR_ = nullptr, *mT_ = nullptr, *v_ = nullptr, *cv_ = nullptr, *divv_ = nullptr, *cdiv_ = nullptr;
  T *df_ = nullptr, *da_ = nullptr, *gamma_ = nullptr, *Av_ = nullptr, *m_ = nullptr, *gm_ = nullptr;
  T *lam0_ = nullptr, *lam1_ = nullptr, *coef_ = nullptr, *acc_ = nullptr, *t3a_ = nullptr, *t3b_ = nullptr;
  T *vk_ = nullptr, *gk_ = nullptr, *trial_ = nullptr, *x_ = nullptr, *r_ = nullptr, *z_ = nullptr, *pp_ = nullptr,
    *q_ = nullptr, *b_ = nullptr, *st_ = nullptr;
  cplx<T>* Sr_ = nullptr;
  cplx<T>*S1_ = nullptr, *S2_ = nullptr;
  Twiddles<double> twd_;
  cplx<double>*twd1_ = nullptr, *twd2_ = nullptr, *twd3_ = nullptr, *Sd_ = nullptr;

  double *partial_ = nullptr, *dres_ = nullptr;
};

}  // namespace
}  // namespace d3
}  // namespace slnk

struct slnk3_ctx {
  std::unique_ptr<slnk::d3::Base> impl;
  std::string err;
};

namespace {

template <class Fn>
slnk_status guard3(slnk3_ctx* ctx, Fn&& fn) {
  if (!ctx || !ctx->impl) return SLNK_EINVAL;
  try {
    fn(*ctx->impl);
    return SLNK_OK;
  } catch (const slnk::d3::Err& e) {
    ctx->err = e.msg;
    return e.st;
  } catch (const std::bad_alloc&) {
    ctx->err = "host allocation failed";
    return SLNK_ENOMEM;
  }
}

}  // namespace

extern "C" {

void slnk3_default_params(slnk3_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->n1 = p->n2 = p->n3 = 64;
  p->nt = 4;
  p->reg = SLNK_REG_H2;
  p->beta = 1e-3;
  p->prec = SLNK_PREC_MIXED;
  p->proj = SLNK_PROJ_NONE;
  p->sl_path = 0;
  p->pc = SLNK_PC_REG;
  p->cheb_iters = 10;
  p->lanczos_steps = 30;
  p->emax_safety = 1.05;
  p->lanczos_seed = 0x5EED;
  p->hessian = SLNK_HESS_GN;
  p->coarse_solver = SLNK_COARSE_CHEB;
  p->coarse_eps = 0.1;
  p->transport = SLNK_TRANSPORT_SL;
}

slnk_status slnk3_create(const slnk3_params* p, void* hip_stream, slnk3_ctx** out) {
  if (!p || !out) return SLNK_EINVAL;
  *out = nullptr;
  using slnk::d3::size_ok;
  if (!size_ok(p->n1) || !size_ok(p->n2) || !size_ok(p->n3) || p->nt < 1 || p->nt > 1000 || p->reg < 1 ||
      p->reg > 3 || !(p->beta > 0.0) || !std::isfinite(p->beta) ||
      (p->prec != SLNK_PREC_FP64 && p->prec != SLNK_PREC_MIXED) || (p->proj != 0 && p->proj != 1) ||
      (p->sl_path != 0 && p->sl_path != 1) || (p->pc != SLNK_PC_REG && p->pc != SLNK_PC_2L) ||
      (p->hessian != SLNK_HESS_GN && p->hessian != SLNK_HESS_FN) ||
      (p->coarse_solver != SLNK_COARSE_CHEB && p->coarse_solver != SLNK_COARSE_PCG) ||
      (p->coarse_solver == SLNK_COARSE_PCG && !(p->coarse_eps > 0.0 && p->coarse_eps < 1.0)) ||
      (p->transport != SLNK_TRANSPORT_SL && p->transport != SLNK_TRANSPORT_RK2A) ||
      (p->transport == SLNK_TRANSPORT_RK2A && p->pc != SLNK_PC_REG))
    return SLNK_EINVAL;
  if (p->pc == SLNK_PC_2L && (!size_ok(p->n1 / 2) || !size_ok(p->n2 / 2) || !size_ok(p->n3 / 2) ||
                              p->cheb_iters < 1 || p->lanczos_steps < 1 || p->lanczos_steps > 1000 ||
                              !(p->emax_safety >= 1.0)))
    return SLNK_EINVAL;
  auto ctx = std::make_unique<slnk3_ctx>();
  try {
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (p->prec == SLNK_PREC_FP64)
      ctx->impl = std::make_unique<slnk::d3::Ctx<double>>(*p, s);
    else
      ctx->impl = std::make_unique<slnk::d3::Ctx<float>>(*p, s);
  } catch (const slnk::d3::Err& e) {
    return e.st;
  } catch (const std::bad_alloc&) {
    return SLNK_ENOMEM;
  }
  *out = ctx.release();
  return SLNK_OK;
}

void slnk3_destroy(slnk3_ctx* ctx) { delete ctx; }

const char* slnk3_last_error(const slnk3_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

unsigned long long slnk3_workspace_bytes(const slnk3_ctx* ctx) {
  return ctx && ctx->impl ? (unsigned long long)ctx->impl->bytes : 0ull;
}

slnk_status slnk3_set_images(slnk3_ctx* ctx, const void* m_R, const void* m_T) {
  if (!m_R || !m_T) return SLNK_EINVAL;
  return guard3(ctx, [&](slnk::d3::Base& c) { c.set_images(m_R, m_T); });
}

slnk_status slnk3_transport_state(slnk3_ctx* ctx, const void* v, const void* m0, void* m1) {
  if (!v || !m0 || !m1) return SLNK_EINVAL;
  return guard3(ctx, [&](slnk::d3::Base& c) { c.transport_state(v, m0, m1); });
}

slnk_status slnk3_objective(slnk3_ctx* ctx, const void* v, double* J) {
  if (!v || !J) return SLNK_EINVAL;
  return guard3(ctx, [&](slnk::d3::Base& c) { *J = c.objective(v); });
}

slnk_status slnk3_gradient(slnk3_ctx* ctx, const void* v, void* g, double* J) {
  if (!v || !g) return SLNK_EINVAL;
  return guard3(ctx, [&](slnk::d3::Base& c) {
    const double j = c.gradient(v, g);
    if (J) *J = j;
  });
}

slnk_status slnk3_hessian_matvec(slnk3_ctx* ctx, const void* vt, void* Hvt) {
  if (!vt || !Hvt) return SLNK_EINVAL;
  return guard3(ctx, [&](slnk::d3::Base& c) { c.hessian(vt, Hvt); });
}

slnk_status slnk3_split_matvec(slnk3_ctx* ctx, const void* s, void* out) {
  if (!s || !out) return SLNK_EINVAL;
  return guard3(ctx, [&](slnk::d3::Base& c) { c.split_matvec_api(s, out); });
}

slnk_status slnk3_get_cheb_bounds(const slnk3_ctx* ctx, double* emin, double* emax) {
  if (!ctx || !ctx->impl || !emin || !emax) return SLNK_EINVAL;
  ctx->impl->cheb_bounds(emin, emax);
  return SLNK_OK;
}

slnk_status slnk3_precond_apply(slnk3_ctx* ctx, const void* r, void* z) {
  if (!r || !z) return SLNK_EINVAL;
  return guard3(ctx, [&](slnk::d3::Base& c) { c.precond(r, z); });
}

slnk_status slnk3_newton_solve(slnk3_ctx* ctx, void* v_inout, const slnk_solve_opts* opts,
                               slnk_solve_report* report) {
  if (!v_inout) return SLNK_EINVAL;
  slnk_solve_opts o;
  slnk_default_opts(&o);
  if (opts) o = *opts;
  if (o.max_newton < 0 || o.max_pcg < 1 || o.max_halvings < 0) return SLNK_EINVAL;
  slnk_solve_report rep;
  slnk_status result = SLNK_OK;
  const slnk_status st = guard3(ctx, [&](slnk::d3::Base& c) { result = c.newton(v_inout, o, rep); });
  if (st != SLNK_OK) return st;
  if (report) *report = rep;
  return result;
}

}  // extern "C"
