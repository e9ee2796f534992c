// Host orchestration of the semi-Lagrangian Gauss--Newton--Krylov path behind the C ABI of
// include/slnk.h.  Everything numerical runs in the gfx950 kernels of spectral_impl.hpp,
// transport.hip and blas.hip; this file sequences them, owns the device workspace and keeps the
// FP64 scalars of the Krylov, Chebyshev, Lanczos and Newton iterations.
//
// A context holds B same-size registration problems ("items").  Every kernel launch covers all
// items (grid z = item); the iterations run in lock step with per-item scalars, and items that
// have stopped are skipped through device-side masks.  B = 1 is the single-problem case.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <thread>
#include <tuple>
#include <type_traits>
#include <type_traits>
#include <vector>

#include "../../include/slnk.h"
#include "fft_plan.hpp"
#include "kernels.hpp"
#include "unet_net.hpp"

namespace slnk {

struct Fail {
  slnk_status st;
  std::string msg;
};

namespace {

constexpr double kPi = 3.14159265358979323846;

#define HIPCHK(expr)                                                                                  \
  do {                                                                                                \
    hipError_t _e = (expr);                                                                           \
    if (_e != hipSuccess) throw ::slnk::Fail{SLNK_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)}; \
  } while (0)


double trapezoid_weight(int j, int nt) {  // weight of level j times ht
  const double ht = 1.0 / nt;
  return (j == 0 || j == nt) ? 0.5 * ht : ht;
}

// Largest eigenvalue of the symmetric tridiagonal matrix (diag a, off-diagonal b) by bisection on
// the Sturm sequence count.
double tridiag_max_eig(const std::vector<double>& a, const std::vector<double>& b) {
  const int n = int(a.size());
  double lo = a[0], hi = a[0];
  for (int i = 0; i < n; ++i) {
    const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  auto count_below = [&](double x) {  // eigenvalues < x
    int c = 0;
    double d = 1.0;
    for (int i = 0; i < n; ++i) {
      const double bb = i > 0 ? b[i - 1] * b[i - 1] : 0.0;
      d = a[i] - x - (i > 0 ? bb / d : 0.0);
      if (d == 0.0) d = -1e-300;
      if (d < 0) ++c;
    }
    return c;
  };
  for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(1.0, std::fabs(hi)); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (count_below(mid) == n)
      hi = mid;
    else
      lo = mid;
  }
  return hi;
}

std::vector<double> splitmix64_uniform(unsigned long long seed, size_t count) {
  std::vector<double> out(count);
  unsigned long long state = seed;
  for (size_t i = 0; i < count; ++i) {
    state += 0x9E3779B97F4A7C15ULL;
    unsigned long long z = state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z = z ^ (z >> 31);
    out[i] = double(z >> 11) * (1.0 / 9007199254740992.0) - 0.5;
  }
  return out;
}

// Bump allocator over one device allocation.
struct Arena {
  char* base = nullptr;
  size_t size = 0, used = 0;
  template <typename U>
  U* take(size_t count) {
    const size_t bytes = (count * sizeof(U) + 255) / 256 * 256;
    if (used + bytes > size) throw Fail{SLNK_ENOMEM, "workspace arena exhausted"};
    U* p = reinterpret_cast<U*>(base + used);
    used += bytes;
    return p;
  }
};

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

bool any_of(const std::vector<int>& m) {
  return std::any_of(m.begin(), m.end(), [](int a) { return a != 0; });
}

// --------------------------------------------------------------------------------------------
// One grid level of B items.  Per item the buffers are consecutive with the sizes noted
// (F = n1 n2 elements); item z of a buffer of size S per item starts at z S.
template <typename T>
struct Level {
  int n1 = 0, n2 = 0, nt = 0, B = 1;
  size_t F = 0;
  double cell = 0;
  SpecGrid<T> sg;
  T* mT = nullptr;  // F
  T* mR = nullptr;  // F
  // slot 0: the current linearisation point; slot 1: the trial point of the line search
  struct Lin {
    T* v = nullptr;      // 2F
    T* df = nullptr;     // 2F  forward displacements (cells)
    T* da = nullptr;     // 2F  adjoint displacements
    T* gamma = nullptr;  // F
    T* m = nullptr;      // (nt+1) F
    T* gm = nullptr;     // 2 (nt+1) F
    T* bAv = nullptr;    // 2F
    std::vector<double> J, Jreg;
    std::vector<int> halo;
    bool valid = false, has_gm = false;
  } lin[2];
  int* halo_dev = nullptr;  // [2][B]: halo of each slot and item, read by the transport kernels
  // work buffers
  T* cv = nullptr;    // 2F
  T* divv = nullptr;  // F
  T* cdiv = nullptr;  // F
  T* lam = nullptr;   // 2F (two time levels)
  T* acc = nullptr;   // 2F
  T* g = nullptr;     // 2F
  T* q = nullptr;     // 2F (two time levels)
  T* bt = nullptr;    // 2F
  T* w = nullptr;     // 2F
  T* coef = nullptr;  // F
  T* coef2 = nullptr; // F
  T* vec[8] = {};     // 2F each: Krylov / Chebyshev / Lanczos vectors
  T* gmT = nullptr;   // 2F: gradient of m_T (Lanczos at v = 0)
  cplx<T>* S1 = nullptr;
  cplx<T>* S2 = nullptr;
  cplx<T>* Sk = nullptr;  // 2 spectra: kept fine spectrum of the two-level combine
  void* tw_row = nullptr;
  void* tw_col = nullptr;
  // largest halo of a slot over the items of 'mask' (empty: all items)
  int max_halo(int slot, const std::vector<int>& mask) const {
    int h = 0;
    for (int z = 0; z < B; ++z)
      if (mask.empty() || mask[z]) h = std::max(h, lin[slot].halo[z]);
    return h;
  }
};

template <typename T>
struct Context {
  slnk_params prm{};
  int B = 1;
  hipStream_t stream = nullptr;
  Arena arena;
  Level<T> fine, coarse;
  bool two_level = false;
  bool images_set = false;
  bool has_grad = false;
  // full-Newton matvec (fine level only; the coarse operator of P_2L stays Gauss--Newton)
  bool full_newton = false;
  // incompressible case: K = Leray projection on b, b~ (section 3.1)
  bool leray = false;
  // P_2L coarse solver: CHEB(k), or PCG(eps) to eps times the outer tolerance of each item
  bool coarse_pcg = false;
  // stabilised RK2 transport instead of the SL scheme (fine level; P_REG)
  bool rk2a = false;
  struct {
    T* w3 = nullptr;      // 3F: (y, y v1, y v2) of the Heun stage's input
    T* d3 = nullptr;      // 3F: its spectral derivatives
    T* w3s = nullptr;     // 3F, 3F: the same for the incremental state's source terms
    T* d3s = nullptr;
    T* k = nullptr;       // F: first-stage slope
    T* y[2] = {};         // F each: current and next time level
    T* src[2] = {};       // F each: incremental-state sources at two time levels
    T* pair = nullptr;    // 2F: (lam, lam m)
    T* g4 = nullptr;      // 4F: (grad lam, grad(lam m))
    T* divt = nullptr;    // F: div of the matvec direction
    T* lam = nullptr;     // (nt+1) F, full Newton: lambda^0..lambda^nt of the last gradient
    T* gmt = nullptr;     // 2F, full Newton: grad m~^j
  } rk;
  std::vector<double> outer_tol;
  static constexpr int kMaxInner = 200;
  struct {
    T* lam = nullptr;    // (nt+1) F per item: lambda^0..lambda^nt of the slot-0 linearisation
    T* mt = nullptr;     // nt F: m~^1..m~^nt
    T* x2 = nullptr;     // 2 (nt+1) F: lambda^j vt, later grad m~^j
    T* sigma = nullptr;  // (nt+1) F: div(lambda^j vt)
    T* e = nullptr;      // nt F: I[sigma^j](X_a), then the source of incremental adjoint step j
    T* divv = nullptr;   // F: div v of the slot-0 linearisation
  } fn;
  std::vector<double> emin, emax;
  // e_max of the set-up (Lanczos at v = 0, the network's head or a caller's value): every solve
  // starts from it, so that a re-estimate inside one solve does not carry over into the next
  std::vector<double> emax_setup;
  double* partial = nullptr;  // reduction partials (two independent halves)
  size_t partial_half = 0;
  double* dres = nullptr;     // device results [2][4B]
  double* hres = nullptr;     // pinned host copy of dres
  double* dsc = nullptr;      // device per-item scalars [16][B]
  double* lz_log = nullptr;   // Lanczos (alpha, beta) per item and step [B][steps][2] (P_2L)
  int* lz_live = nullptr;     // Lanczos: items whose tridiagonal matrix is still growing [B]
  double* hsc = nullptr;      // pinned staging of dsc
  double* cheb_tab = nullptr; // device [2][cheb_iters][B]: Chebyshev d-update coefficients
  double* inv_theta = nullptr;  // device [B]: 1 / theta of each item's Chebyshev interval
  int* masks = nullptr;       // device [4][B]: all ones, PCG, Newton, line search
  // FP64 Newton iterate of the fine level and its regularisation term: beta A amplifies the
  // rounding of v by up to beta max|k|^(2 reg), so v and beta A v are kept in FP64 while the
  // transport reads an FP32 copy (mixed precision; plain copies in the FP64 context)
  SpecGrid<double> sg64;
  void* tw64_row = nullptr;
  void* tw64_col = nullptr;
  double* v64[2] = {};
  double* bAv64[2] = {};
  cplx<double>* S64a = nullptr;
  cplx<double>* S64b = nullptr;
  // captured HIP graphs of the matvec and of the preconditioner, keyed by (operation, input,
  // output, mask); recorded on a private stream, replayed on the caller's stream
  bool use_graphs = true;
  bool capturing = false;
  int halo_cap = 0;  // LDS footprint of graphed SL steps (device halo <= cap)
  hipStream_t cap_stream = nullptr;
  std::map<std::tuple<int, const void*, const void*, const void*>, hipGraphExec_t> graphs;
  // start velocity and head output of the network, kept by slnk_set_images_learned
  T* learned_v = nullptr;     // [B][2F]
  float* learned_y = nullptr; // [B]
  bool learned_ready = false;
  // counters of the current solve
  std::vector<int> n_matvec, n_coarse;
  // preconditioner time: event pairs around each application, summed without stalling the stream
  double t_prec = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prec_ev;
  size_t prec_used = 0;

  enum { kMaskAll = 0, kMaskPcg = 1, kMaskNewton = 2, kMaskLs = 3, kMaskCoarse = 4 };
  int* mask(int k) const { return masks + k * B; }
  double* sc(int k) const { return dsc + k * B; }

  // ---- setup ------------------------------------------------------------------------------
  // plan of length n: radix list and the 2n-entry table of stage twiddles (consecutive butterflies
  // read consecutive entries) and roots of unity (wave-level transforms), in arena memory
  template <typename U>
  void plan(FFTPlanDev& pl, int n, void*& tw) {
    std::vector<cplx<U>> h(2 * size_t(n));
    if (!fft_plan_host(n, pl, [&](int i, double re, double im) { h[i] = {U(re), U(im)}; }))
      throw Fail{SLNK_EINVAL, "FFT length has too many factors"};
    tw = arena.take<cplx<U>>(2 * n);
    HIPCHK(hipMemcpyAsync(tw, h.data(), 2 * n * sizeof(cplx<U>), hipMemcpyHostToDevice, stream));
    HIPCHK(hipStreamSynchronize(stream));  // h is released on return
    pl.tw = tw;
    pl.roots = static_cast<cplx<U>*>(tw) + n;
  }

  static size_t level_bytes(int n1, int n2, int nt, int B) {
    const size_t F = size_t(n1) * n2;
    const size_t spec = size_t(n1) * spec_stride(n2);
    const size_t nspec = std::max<size_t>(6, 2 * (nt + 1));
    // images; two slots of (v, df, da, gamma, m, gm, bAv); cv, divv, cdiv; lam, acc, g, q, bt, w;
    // coef, coef2; vec[8]; gmT
    const size_t fields = 2 + 2 * (2 + 2 + 2 + 1 + (nt + 1) + 2 * (nt + 1) + 2) + 2 + 1 + 1 + 2 * 6 + 2 + 2 * 8 + 2;
    return B * (fields * F * sizeof(T) + (2 * nspec + 2) * spec * sizeof(cplx<T>)) + 2 * (n1 + n2) * sizeof(cplx<T>) +
           96 * 256 + 2 * B * sizeof(int);
  }

  void alloc_level(Level<T>& lv, int n1, int n2, int nt) {
    lv.n1 = n1;
    lv.n2 = n2;
    lv.nt = nt;
    lv.B = B;
    lv.F = size_t(n1) * n2;
    lv.cell = (2.0 * kPi / n1) * (2.0 * kPi / n2);
    lv.sg.n1 = n1;
    lv.sg.n2 = n2;
    plan<T>(lv.sg.row, n2, lv.tw_row);
    plan<T>(lv.sg.col, n1, lv.tw_col);
    const size_t F = lv.F;
    lv.mT = arena.take<T>(B * F);
    lv.mR = arena.take<T>(B * F);
    for (auto& L : lv.lin) {
      L.v = arena.take<T>(B * 2 * F);
      L.df = arena.take<T>(B * 2 * F);
      L.da = arena.take<T>(B * 2 * F);
      L.gamma = arena.take<T>(B * F);
      L.m = arena.take<T>(B * (nt + 1) * F);
      L.gm = arena.take<T>(B * 2 * (nt + 1) * F);
      L.bAv = arena.take<T>(B * 2 * F);
      L.J.assign(B, 0.0);
      L.Jreg.assign(B, 0.0);
      L.halo.assign(B, 0);
    }
    lv.halo_dev = arena.take<int>(2 * B);
    lv.cv = arena.take<T>(B * 2 * F);
    lv.divv = arena.take<T>(B * F);
    lv.cdiv = arena.take<T>(B * F);
    lv.lam = arena.take<T>(B * 2 * F);
    lv.acc = arena.take<T>(B * 2 * F);
    lv.g = arena.take<T>(B * 2 * F);
    lv.q = arena.take<T>(B * 2 * F);
    lv.bt = arena.take<T>(B * 2 * F);
    lv.w = arena.take<T>(B * 2 * F);
    lv.coef = arena.take<T>(B * F);
    lv.coef2 = arena.take<T>(B * F);
    for (auto& p : lv.vec) p = arena.take<T>(B * 2 * F);
    lv.gmT = arena.take<T>(B * 2 * F);
    const size_t nspec = std::max<size_t>(6, 2 * (nt + 1));
    lv.S1 = arena.take<cplx<T>>(B * nspec * lv.sg.spec());
    lv.S2 = arena.take<cplx<T>>(B * nspec * lv.sg.spec());
    lv.Sk = arena.take<cplx<T>>(B * 2 * lv.sg.spec());
  }

  void create(const slnk_params& p, hipStream_t s) {
    prm = p;
    stream = s;
    B = p.batch;
    if (B < 1 || B > 4096) throw Fail{SLNK_EINVAL, "batch must be in [1, 4096]"};
    if (!fft_size_ok(p.n1) || !fft_size_ok(p.n2)) throw Fail{SLNK_EINVAL, "grid sizes must be even products of 2, 3, 5 in [8, 2048]"};
    // the FP64 column transforms (every context has an FP64 part) of n1 > 2000 would need more than
    // the 160 KiB of LDS a gfx950 workgroup has
    if (p.n1 > 2000) throw Fail{SLNK_EINVAL, "n1 must be at most 2000 (LDS of the FP64 column transforms)"};
    if (p.nt < 1 || p.nt > 512) throw Fail{SLNK_EINVAL, "nt must be in [1, 512]"};
    if (p.reg < 1 || p.reg > 3) throw Fail{SLNK_EINVAL, "reg must be 1, 2 or 3"};
    if (!(p.beta > 0)) throw Fail{SLNK_EINVAL, "beta must be positive"};
    if (p.pc != SLNK_PC_REG && p.pc != SLNK_PC_2L) throw Fail{SLNK_EINVAL, "pc must be SLNK_PC_REG or SLNK_PC_2L"};
    if (p.sl_path < 0 || p.sl_path > 3) throw Fail{SLNK_EINVAL, "sl_path must be 0, 1, 2 or 3"};
    if (p.hessian != SLNK_HESS_GN && p.hessian != SLNK_HESS_FN)
      throw Fail{SLNK_EINVAL, "hessian must be SLNK_HESS_GN or SLNK_HESS_FN"};
    full_newton = p.hessian == SLNK_HESS_FN;
    if (p.proj != SLNK_PROJ_NONE && p.proj != SLNK_PROJ_LERAY)
      throw Fail{SLNK_EINVAL, "proj must be SLNK_PROJ_NONE or SLNK_PROJ_LERAY"};
    leray = p.proj == SLNK_PROJ_LERAY;
    if (p.coarse_solver != SLNK_COARSE_CHEB && p.coarse_solver != SLNK_COARSE_PCG)
      throw Fail{SLNK_EINVAL, "coarse_solver must be SLNK_COARSE_CHEB or SLNK_COARSE_PCG"};
    coarse_pcg = p.coarse_solver == SLNK_COARSE_PCG;
    if (coarse_pcg && !(p.coarse_eps > 0.0 && p.coarse_eps < 1.0))
      throw Fail{SLNK_EINVAL, "coarse_eps must lie in (0, 1)"};
    outer_tol.assign(B, 1.0);
    if (p.transport != SLNK_TRANSPORT_SL && p.transport != SLNK_TRANSPORT_RK2A)
      throw Fail{SLNK_EINVAL, "transport must be SLNK_TRANSPORT_SL or SLNK_TRANSPORT_RK2A"};
    rk2a = p.transport == SLNK_TRANSPORT_RK2A;
    if (rk2a && p.pc != SLNK_PC_REG) throw Fail{SLNK_EINVAL, "RK2A transport runs with P_REG"};
    two_level = p.pc == SLNK_PC_2L;
    if (two_level) {
      if (!fft_size_ok(p.n1 / 2) || !fft_size_ok(p.n2 / 2)) throw Fail{SLNK_EINVAL, "coarse grid n/2 not supported"};
      if (p.cheb_iters < 1 || p.cheb_iters > 64 || p.lanczos_steps < 2 || p.lanczos_steps > 1000 ||
          !(p.emax_safety >= 1.0))
        throw Fail{SLNK_EINVAL, "bad P_2L parameters"};
    }
    {
      int dev = 0, lim = 0;
      HIPCHK(hipGetDevice(&dev));
      HIPCHK(hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
      if (spec_lds_bytes<T>(p.n1, p.n2) > size_t(lim) || spec_lds_bytes<double>(p.n1, p.n2) > size_t(lim))
        throw Fail{SLNK_EINVAL, "grid too large for the LDS-resident FFTs of this precision"};
    }
    const size_t F = size_t(p.n1) * p.n2;
    const int tiles = ((p.n1 + 15) / 16) * ((p.n2 + 15) / 16);  // blocks of the 16x16 transport kernels
    partial_half = size_t(B) * (std::max(reduce_blocks(2 * F), tiles) * 4 + 64);
    size_t bytes = level_bytes(p.n1, p.n2, p.nt, B) + (two_level ? level_bytes(p.n1 / 2, p.n2 / 2, p.nt, B) : 0);
    bytes += (2 * partial_half + 8 * B + 16 * B + 2 * 64 * B + B) * sizeof(double) + 5 * B * sizeof(int) + 8192;
    bytes += B * (4 * 2 * F * sizeof(double) + 2 * 2 * size_t(p.n1) * spec_stride(p.n2) * sizeof(cplx<double>)) +
             2 * (p.n1 + p.n2) * sizeof(cplx<double>) + 16 * 256;
    bytes += B * (2 * F * sizeof(T) + sizeof(float)) + 2 * 256;
    if (full_newton && !rk2a) bytes += B * size_t(6 * p.nt + 5) * F * sizeof(T) + 6 * 256;
    if (rk2a) bytes += B * size_t(24) * F * sizeof(T) + 14 * 256;  // w3, d3, w3s, d3s 12; k, y, src 5; pair 2; g4 4; divt 1
    if (rk2a && full_newton) bytes += B * size_t(p.nt + 3) * F * sizeof(T) + 2 * 256;  // lam nt+1; gmt 2
    if (two_level) bytes += B * (2 * size_t(p.lanczos_steps) * sizeof(double) + sizeof(int)) + 2 * 256;  // Lanczos log
    void* base = nullptr;
    if (hipMalloc(&base, bytes) != hipSuccess) throw Fail{SLNK_ENOMEM, "hipMalloc of the workspace failed"};
    arena.base = static_cast<char*>(base);
    arena.size = bytes;
    // every buffer starts finite: items skipped by a mask may still be read by unmasked updates.
    // Cleared on the context's stream, which may be non-blocking: ordered before all of its work
    HIPCHK(hipMemsetAsync(base, 0, bytes, stream));
    partial = arena.take<double>(2 * partial_half);
    dres = arena.take<double>(8 * B);
    dsc = arena.take<double>(16 * B);
    cheb_tab = arena.take<double>(2 * 64 * B);
    inv_theta = arena.take<double>(B);
    masks = arena.take<int>(5 * B);
    if (two_level) {
      lz_log = arena.take<double>(B * 2 * size_t(p.lanczos_steps));
      lz_live = arena.take<int>(B);
    }
    HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&hres), 8 * B * sizeof(double), hipHostMallocDefault));
    HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&hsc), 16 * B * sizeof(double), hipHostMallocDefault));
    alloc_level(fine, p.n1, p.n2, p.nt);
    if (two_level) alloc_level(coarse, p.n1 / 2, p.n2 / 2, p.nt);
    if (full_newton && !rk2a) {
      fn.lam = arena.take<T>(B * (p.nt + 1) * F);
      fn.mt = arena.take<T>(B * p.nt * F);
      fn.x2 = arena.take<T>(B * 2 * (p.nt + 1) * F);
      fn.sigma = arena.take<T>(B * (p.nt + 1) * F);
      fn.e = arena.take<T>(B * p.nt * F);
      fn.divv = arena.take<T>(B * F);
    }
    if (rk2a) {
      rk.w3 = arena.take<T>(B * 3 * F);
      rk.d3 = arena.take<T>(B * 3 * F);
      rk.w3s = arena.take<T>(B * 3 * F);
      rk.d3s = arena.take<T>(B * 3 * F);
      rk.k = arena.take<T>(B * F);
      for (auto& y : rk.y) y = arena.take<T>(B * F);
      for (auto& y : rk.src) y = arena.take<T>(B * F);
      rk.pair = arena.take<T>(B * 2 * F);
      rk.g4 = arena.take<T>(B * 4 * F);
      rk.divt = arena.take<T>(B * F);
      if (full_newton) {
        rk.lam = arena.take<T>(B * (p.nt + 1) * F);
        rk.gmt = arena.take<T>(B * 2 * F);
      }
    }
    sg64.n1 = p.n1;
    sg64.n2 = p.n2;
    plan<double>(sg64.row, p.n2, tw64_row);
    plan<double>(sg64.col, p.n1, tw64_col);
    for (int sl = 0; sl < 2; ++sl) {
      v64[sl] = arena.take<double>(B * 2 * F);
      bAv64[sl] = arena.take<double>(B * 2 * F);
    }
    S64a = arena.take<cplx<double>>(B * 2 * sg64.spec());
    S64b = arena.take<cplx<double>>(B * 2 * sg64.spec());
    learned_v = arena.take<T>(B * 2 * F);
    learned_y = arena.take<float>(B);
    use_graphs = p.use_graphs != 0;
    halo_cap = std::min(8, sl_step_max_halo<T>());
    if (halo_cap < 0) throw Fail{SLNK_EDEVICE, "cannot query the LDS size of the device"};
    HIPCHK(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking));
    std::vector<int> ones(B, 1);
    for (int k = 0; k < 5; ++k) put_mask(k, ones);
    emin.assign(B, 0.0);
    emax.assign(B, 0.0);
    emax_setup.assign(B, 0.0);
    n_matvec.assign(B, 0);
    n_coarse.assign(B, 0);
    HIPCHK(hipStreamSynchronize(stream));
  }

  void clear_graphs() {
    for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
    graphs.clear();
  }

  void destroy() {
    clear_graphs();
    for (auto& e : prec_ev) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
    prec_ev.clear();
    prec_used = 0;
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    cap_stream = nullptr;
    if (hres) (void)hipHostFree(hres);
    if (hsc) (void)hipHostFree(hsc);
    if (arena.base) (void)hipFree(arena.base);
    hres = hsc = nullptr;
    arena.base = nullptr;
  }

  // read one half of dres (4B doubles; item z's results at 4z + c) to the host
  const double* fetch(int half) {
    HIPCHK(hipMemcpyAsync(hres + half * 4 * B, dres + half * 4 * B, 4 * B * sizeof(double), hipMemcpyDeviceToHost,
                          stream));
    HIPCHK(hipStreamSynchronize(stream));
    return hres + half * 4 * B;
  }

  // next free event pair of the preconditioner timer (a full pool is folded into t_prec first)
  const std::pair<hipEvent_t, hipEvent_t>& prec_event() {
    if (prec_used == 256) fold_prec_time();
    if (prec_used == prec_ev.size()) {
      std::pair<hipEvent_t, hipEvent_t> e{nullptr, nullptr};
      HIPCHK(hipEventCreate(&e.first));
      if (hipEventCreate(&e.second) != hipSuccess) {
        (void)hipEventDestroy(e.first);
        throw Fail{SLNK_EDEVICE, "hipEventCreate failed"};
      }
      prec_ev.push_back(e);
    }
    return prec_ev[prec_used++];
  }

  // add the recorded preconditioner intervals to t_prec (waits for the last one)
  void fold_prec_time() {
    if (prec_used == 0) return;
    HIPCHK(hipEventSynchronize(prec_ev[prec_used - 1].second));
    for (size_t i = 0; i < prec_used; ++i) {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, prec_ev[i].first, prec_ev[i].second));
      t_prec += ms;
    }
    prec_used = 0;
  }

  // read both halves of dres to the host
  const double* fetch_both() {
    HIPCHK(hipMemcpyAsync(hres, dres, 8 * B * sizeof(double), hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    return hres;
  }

  // publish per-item scalars as row k of dsc.  The pinned row is reused only after a later
  // synchronisation (every caller reads a reduction before writing the same row again).
  void put_scalars(int k, const std::vector<double>& v) {
    std::memcpy(hsc + k * B, v.data(), B * sizeof(double));
    HIPCHK(hipMemcpyAsync(sc(k), hsc + k * B, B * sizeof(double), hipMemcpyHostToDevice, stream));
  }

  void put_mask(int k, const std::vector<int>& m) { HIPCHK(set_ints(stream, mask(k), m.data(), B)); }

  SymbolParams sym(Symbol k) const { return SymbolParams{k, prm.reg, prm.beta}; }
  // a symbol applied to a transport result b or b~: K (Leray) first in the incompressible case
  SymbolParams symK(Symbol k) const {
    SymbolParams sp = sym(k);
    sp.proj = leray ? 1 : 0;
    return sp;
  }

  // SL step arguments shared by every step of a level: the LDS footprint is sized for the largest
  // item halo of the slot (halo_cap while capturing a graph), and each item stages its own halo
  // read from device memory
  StepArgs<T> step_base(Level<T>& lv, int slot, const int* active, bool graphed_halo) {
    StepArgs<T> a;
    a.n1 = lv.n1;
    a.n2 = lv.n2;
    a.batch = B;
    a.active = active;
    a.halo = graphed_halo ? halo_cap : lv.max_halo(slot, {});
    a.halo_dev = lv.halo_dev + slot * B;
    a.coef = lv.coef;
    a.st_coef = (long long)lv.F;
    a.coef2 = lv.coef2;
    a.st_coef2 = (long long)lv.F;
    a.ht = 1.0 / lv.nt;
    a.force_global = prm.sl_path == 1;
    a.fused_rows = prm.sl_path == 2 ? 16 : prm.sl_path == 3 ? 32 : 0;
    return a;
  }

  // ---- linearisation: trace, state, objective ---------------------------------------------
  // The velocity of lin[slot] comes from v (device, B x 2F of T) or, on the fine level, from the
  // FP64 iterate v64src.  Traces both characteristics, solves the state equation and, with
  // need_J, evaluates J (fine level: beta A v in FP64); grad m is left to ensure_gm.  Only the
  // items of mk (device mask, host copy hmask; nullptr / empty: all) are touched.
  void linearize(Level<T>& lv, int slot, const T* v, bool need_J, const double* v64src, const int* mk,
                 const std::vector<int>& hmask) {
    auto& L = lv.lin[slot];
    const size_t F = lv.F;
    const bool on_fine = &lv == &fine;
    if (on_fine && v64src) {
      if (v64src != v64[slot]) HIPCHK(masked_copy<double>(stream, B, 2 * F, v64src, 2 * F, v64[slot], 2 * F, mk));
      HIPCHK(cast_copy<T>(stream, B * 2 * F, v64[slot], L.v));
    } else {
      if (v != L.v) HIPCHK(masked_copy<T>(stream, B, 2 * F, v, 2 * F, L.v, 2 * F, mk));
      if (on_fine) HIPCHK(cast_back<T>(stream, B * 2 * F, L.v, v64[slot]));
    }
    // RK2A: no characteristics; div v for the antisymmetric operators
    const bool use_rk = rk2a && on_fine;
    int nb = 0;
    const double ht = 1.0 / lv.nt;
    if (use_rk) {
      HIPCHK(spec_div<T>(stream, lv.sg, B, L.v, lv.divv, lv.S1, lv.S2));
    } else {
      HIPCHK(spec_trace_prep<T>(stream, lv.sg, B, mk, L.v, lv.cv, lv.divv, lv.cdiv, lv.S1, lv.S2));
      HIPCHK(sl_trace<T>(stream, lv.n1, lv.n2, B, mk, ht, L.v, lv.cv, lv.divv, lv.cdiv, L.df, L.da, L.gamma,
                         partial, &nb));
      HIPCHK(finish(stream, B, nb, 2, 2LL * nb, 2, 2u, partial, dres));
    }
    const bool reg_term = need_J && on_fine;
    if (reg_term) {
      HIPCHK(spec_scale<double>(stream, sg64, B, mk, sym(Symbol::Reg), 2, v64[slot], bAv64[slot], nullptr, S64a,
                                S64b));
      HIPCHK(dot<double>(stream, B, 2 * F, v64[slot], bAv64[slot], partial + partial_half, dres + 4 * B));
      HIPCHK(cast_copy<T>(stream, B * 2 * F, bAv64[slot], L.bAv));
    }
    const double* r = reg_term ? fetch_both() : fetch(0);  // one synchronisation for both halves
    std::vector<double> maxd(B), vAv(B, 0.0);
    for (int z = 0; z < B; ++z) maxd[z] = use_rk ? 0.0 : r[4 * z + 1];
    if (reg_term)
      for (int z = 0; z < B; ++z) vAv[z] = r[4 * B + 4 * z];
    for (int z = 0; z < B; ++z) {
      if (!hmask.empty() && !hmask[z]) continue;
      if (!std::isfinite(maxd[z]) || !std::isfinite(vAv[z])) throw Fail{SLNK_ENAN, "non-finite velocity or displacement"};
      L.halo[z] = int(std::ceil(maxd[z]));
      L.Jreg[z] = 0.5 * lv.cell * vAv[z];
    }
    HIPCHK(set_ints(stream, lv.halo_dev + slot * B, L.halo.data(), B));
    // state equation
    HIPCHK(masked_copy<T>(stream, B, F, lv.mT, (long long)F, L.m, (long long)((lv.nt + 1) * F), mk));
    if (use_rk) {
      const long long sm = (long long)((lv.nt + 1) * F);
      HIPCHK(rk2a_prod<T>(stream, B, F, L.m, sm, L.v, (long long)(2 * F), rk.w3));
      for (int j = 1; j <= lv.nt; ++j) rk2a_step(lv, slot, -1, -1, L.m + (j - 1) * F, sm, L.m + j * F, sm, nullptr, nullptr);
      if (need_J) {
        HIPCHK(sub_strided<T>(stream, B, F, lv.mR, (long long)F, L.m + lv.nt * F, sm, rk.k, (long long)F));
        HIPCHK(dot<T>(stream, B, F, rk.k, rk.k, partial, dres));
      }
    }
    for (int j = 1; j <= lv.nt && !use_rk; ++j) {
      StepArgs<T> a = step_base(lv, slot, mk, false);
      a.halo = lv.max_halo(slot, hmask);
      a.src = L.m + (j - 1) * F;
      a.dst = L.m + j * F;
      a.st_src = a.st_dst = (long long)((lv.nt + 1) * F);
      a.d1 = L.df;
      a.st_d = (long long)(2 * F);
      a.aux0 = lv.mR;
      a.st_aux0 = (long long)F;
      a.last = (j == lv.nt) && need_J;
      a.partial = partial;
      HIPCHK(sl_step<T>(stream, StepKind::State, a, &nb));
    }
    if (need_J) {
      if (!use_rk) HIPCHK(finish(stream, B, nb, 2, 2LL * nb, 1, 0u, partial, dres));
      const double* r3 = fetch(0);
      for (int z = 0; z < B; ++z) {
        if (!hmask.empty() && !hmask[z]) continue;
        const double mis = r3[4 * z];
        if (!std::isfinite(mis)) throw Fail{SLNK_ENAN, "non-finite state"};
        L.J[z] = 0.5 * lv.cell * mis + L.Jreg[z];
      }
    }
    L.valid = true;
    L.has_gm = false;
  }

  // ---- stabilised RK2 (RK2A) transport ------------------------------------------------------
  // One Heun step of dy/ds = sgn L_dsgn y + src from y0 (rk.w3 holding its products with v) into
  // dst: two evaluations of the antisymmetric operator, each one spectral derivative pass.
  // src0, src1: sources at the start and the end of the step (one field per item, or nullptr).
  void rk2a_step(Level<T>& lv, int slot, int sgn, int dsgn, const T* y0, long long sy0, T* dst, long long sdst,
                 const T* src0, const T* src1) {
    const size_t F = lv.F;
    RK2AStage<T> a;
    a.F = F;
    a.ht = 1.0 / lv.nt;
    a.sgn = sgn;
    a.dsgn = dsgn;
    a.d = rk.d3;
    a.w3 = rk.w3;
    a.v = lv.lin[slot].v;
    a.sv = (long long)(2 * F);
    a.divv = lv.divv;
    a.sdiv = (long long)F;
    a.ssrc = (long long)F;
    a.k = rk.k;
    HIPCHK(spec_rk2a<T>(stream, lv.sg, B, rk.w3, rk.d3, lv.S1, lv.S2));
    a.stage = 1;
    a.src = src0;
    HIPCHK(rk2a_stage<T>(stream, B, a));
    HIPCHK(spec_rk2a<T>(stream, lv.sg, B, rk.w3, rk.d3, lv.S1, lv.S2));
    a.stage = 2;
    a.src = src1;
    a.y0 = y0;
    a.sy0 = sy0;
    a.dst = dst;
    a.sdst = sdst;
    HIPCHK(rk2a_stage<T>(stream, B, a));
  }

  // acc (init: =, else +=) ht w_j 1/2 (lam grad m - m grad lam + grad(lam m)) at time level j for
  // fields lam, m and the gradient gm of m (item strides sl, sm, sgm)
  void rk2a_accumulate(Level<T>& lv, int j, const T* lam, long long sl, const T* m, long long sm, const T* gm,
                       long long sgm, T* acc, bool init) {
    const size_t F = lv.F;
    HIPCHK(rk2a_pair<T>(stream, B, F, lam, sl, m, sm, rk.pair));
    HIPCHK(spec_grad<T>(stream, lv.sg, 2 * B, rk.pair, rk.g4, lv.S1, lv.S2));
    HIPCHK(rk2a_accum<T>(stream, B, F, trapezoid_weight(j, lv.nt), init ? 1 : 0, lam, sl, m, sm, gm, sgm, rk.g4, acc,
                         (long long)(2 * F)));
  }

  // the same with m = m^j, the state of the slot-0 linearisation
  void rk2a_accumulate_state(Level<T>& lv, int j, const T* lam, long long sl, T* acc, bool init) {
    const size_t F = lv.F;
    const long long sm = (long long)((lv.nt + 1) * F);
    auto& L = lv.lin[0];
    rk2a_accumulate(lv, j, lam, sl, L.m + j * F, sm, L.gm + 2 * j * F, 2 * sm, acc, init);
  }

  // time level j of an adjoint sweep: every level in rk.lam (keep: the full-Newton gradient), else
  // two rotating fields
  T* adj_level(const Level<T>& lv, int j, bool keep) const { return keep ? rk.lam + j * lv.F : rk.y[j % 2]; }
  long long adj_stride(const Level<T>& lv, bool keep) const {
    return (long long)(keep ? (lv.nt + 1) * lv.F : lv.F);
  }

  // adjoint equation d_s y = A y + src from y^nt (at adj_level(nt, keep)) backward to t = 0,
  // accumulating b (or b~) into acc (init: its first term sets acc).  source(j, out) writes the
  // equation's source at level j into out and returns out, or returns nullptr (no source).
  template <class Source>
  void rk2a_adjoint_sweep(Level<T>& lv, bool keep, T* acc, bool init, Source source) {
    const size_t F = lv.F;
    const int nt = lv.nt;
    const long long sy = adj_stride(lv, keep);
    rk2a_accumulate_state(lv, nt, adj_level(lv, nt, keep), sy, acc, init);
    HIPCHK(rk2a_prod<T>(stream, B, F, adj_level(lv, nt, keep), sy, lv.lin[0].v, (long long)(2 * F), rk.w3));
    const T* s_hi = source(nt, rk.src[nt % 2]);
    for (int j = nt; j >= 1; --j) {
      const T* s_lo = source(j - 1, rk.src[(j - 1) % 2]);
      rk2a_step(lv, 0, +1, +1, adj_level(lv, j, keep), sy, adj_level(lv, j - 1, keep), sy, s_hi, s_lo);
      rk2a_accumulate_state(lv, j - 1, adj_level(lv, j - 1, keep), sy, acc, false);
      s_hi = s_lo;
    }
  }

  // b = int 1/2 (lam grad m - m grad lam + grad(lam m)) dt at slot 0 into lv.acc; with the
  // full-Newton matvec every lambda^j stays in rk.lam
  void rk2a_gradient(Level<T>& lv) {
    const size_t F = lv.F;
    const int nt = lv.nt;
    auto& L = lv.lin[0];
    const bool keep = full_newton;
    HIPCHK(spec_div<T>(stream, lv.sg, B, L.v, lv.divv, lv.S1, lv.S2));
    HIPCHK(sub_strided<T>(stream, B, F, lv.mR, (long long)F, L.m + nt * F, (long long)((nt + 1) * F),
                          adj_level(lv, nt, keep), adj_stride(lv, keep)));
    rk2a_adjoint_sweep(lv, keep, lv.acc, true, [](int, T*) -> const T* { return nullptr; });
  }

  // b~ of the matvec with RK2A transport at slot 0 into lv.bt: the incremental state
  // d_t m~ = -L m~ - S(m) vt, S(m) vt = 1/2 (div(m vt) + vt . grad m - m div vt), from m~ = 0; then the
  // adjoint equation from -m~(1) with b~ in its antisymmetric form.  Full Newton: the incremental
  // adjoint carries the source 1/2 (div(lam vt) + vt . grad lam + lam div vt) and b~ adds
  // int 1/2 (lam grad m~ - m~ grad lam + grad(lam m~)) dt, lam from the last gradient.
  void rk2a_transport(Level<T>& lv, const T* vt) {
    const size_t F = lv.F;
    const int nt = lv.nt;
    auto& L = lv.lin[0];
    const long long sm = (long long)((nt + 1) * F);
    HIPCHK(spec_div<T>(stream, lv.sg, B, L.v, lv.divv, lv.S1, lv.S2));
    HIPCHK(spec_div<T>(stream, lv.sg, B, vt, rk.divt, lv.S1, lv.S2));
    // sgn 1/2 (div(y vt) + vt . grad y + sgn y div vt) into out
    auto source = [&](const T* y, long long sy, int sgn, T* out) -> const T* {
      HIPCHK(rk2a_prod<T>(stream, B, F, y, sy, vt, (long long)(2 * F), rk.w3s));
      HIPCHK(spec_rk2a<T>(stream, lv.sg, B, rk.w3s, rk.d3s, lv.S1, lv.S2));
      HIPCHK(rk2a_eval<T>(stream, B, F, sgn, sgn, rk.d3s, y, sy, vt, (long long)(2 * F), rk.divt, (long long)F, out,
                          (long long)F));
      return out;
    };
    source(L.m, sm, -1, rk.src[0]);
    HIPCHK(fill<T>(stream, B * F, 0.0, rk.y[0]));
    HIPCHK(fill<T>(stream, B * 3 * F, 0.0, rk.w3));
    int cur = 0;
    for (int j = 1; j <= nt; ++j) {
      source(L.m + j * F, sm, -1, rk.src[j % 2]);
      rk2a_step(lv, 0, -1, -1, rk.y[cur], (long long)F, rk.y[1 - cur], (long long)F, rk.src[(j - 1) % 2],
                rk.src[j % 2]);
      cur = 1 - cur;
      if (full_newton) {  // the lam grad m~ term at level j (m~^0 = 0 adds nothing)
        HIPCHK(spec_grad<T>(stream, lv.sg, B, rk.y[cur], rk.gmt, lv.S1, lv.S2));
        rk2a_accumulate(lv, j, rk.lam + j * F, sm, rk.y[cur], (long long)F, rk.gmt, (long long)(2 * F), lv.bt, j == 1);
      }
    }
    HIPCHK(axpby<T>(stream, B, F, -1.0, nullptr, rk.y[cur], 0.0, nullptr, rk.y[cur]));  // lam~(1) = -m~(1)
    rk2a_adjoint_sweep(lv, false, lv.bt, !full_newton, [&](int j, T* out) -> const T* {
      return full_newton ? source(rk.lam + j * F, sm, +1, out) : nullptr;
    });
  }

  void ensure_gm(Level<T>& lv) {
    auto& L = lv.lin[0];
    if (L.has_gm) return;
    HIPCHK(spec_grad<T>(stream, lv.sg, B * (lv.nt + 1), L.m, L.gm, lv.S1, lv.S2));
    L.has_gm = true;
  }

  // adjoint solve + gradient at slot 0 for the items of mk / hmask; per item sum g^2 and max |g|
  void gradient(Level<T>& lv, const int* mk, const std::vector<int>& hmask, std::vector<double>& g2,
                std::vector<double>& ginf) {
    auto& L = lv.lin[0];
    ensure_gm(lv);
    const size_t F = lv.F;
    const int nt = lv.nt;
    int nb = 0;
    if (rk2a && &lv == &fine) {  // g = beta A v + K b with b from the RK2A adjoint
      rk2a_gradient(lv);
      if (leray) {
        HIPCHK(spec_scale<T>(stream, lv.sg, B, mk, symK(Symbol::One), 2, lv.acc, lv.g, L.bAv, lv.S1, lv.S2));
      } else {
        HIPCHK(xpay<T>(stream, B * 2 * F, lv.acc, 1.0, L.bAv, lv.g));
      }
      HIPCHK(norms<T>(stream, B, 2 * F, lv.g, partial, dres));
      const double* r = fetch(0);
      g2.assign(B, 0.0);
      ginf.assign(B, 0.0);
      for (int z = 0; z < B; ++z) {
        if (!hmask.empty() && !hmask[z]) continue;
        g2[z] = r[4 * z];
        ginf[z] = r[4 * z + 1];
        if (!std::isfinite(g2[z]) || r[4 * z + 2] > 0) throw Fail{SLNK_ENAN, "non-finite gradient"};
      }
      return;
    }
    // the full-Newton matvec needs every adjoint time level (and div v) of this linearisation
    const bool keep = full_newton && &lv == &fine;
    if (keep) {
      HIPCHK(sub_strided<T>(stream, B, F, lv.mR, (long long)F, L.m + nt * F, (long long)((nt + 1) * F),
                            fn.lam + nt * F, (long long)((nt + 1) * F)));
      HIPCHK(spec_div<T>(stream, lv.sg, B, L.v, fn.divv, lv.S1, lv.S2));
    }
    for (int j = nt; j >= 1; --j) {
      StepArgs<T> a = step_base(lv, 0, mk, false);
      a.first = j == nt;
      a.last = j == 1;
      a.src = a.first ? nullptr : lv.lam + (j % 2) * F;
      a.st_src = (long long)(2 * F);
      a.aux0 = lv.mR;
      a.st_aux0 = (long long)F;
      a.aux1 = L.m + nt * F;
      a.st_aux1 = (long long)((nt + 1) * F);
      a.dst = lv.lam + ((j - 1) % 2) * F;
      a.st_dst = (long long)(2 * F);
      if (keep) {
        a.src = a.first ? nullptr : fn.lam + j * F;
        a.dst = fn.lam + (j - 1) * F;
        a.st_src = a.st_dst = (long long)((nt + 1) * F);
      }
      a.d1 = L.da;
      a.st_d = (long long)(2 * F);
      a.gamma = L.gamma;
      a.st_gamma = (long long)F;
      a.gm_new = L.gm + 2 * (j - 1) * F;
      a.gm_old = L.gm + 2 * nt * F;
      a.st_gm = (long long)(2 * (nt + 1) * F);
      a.w_new = trapezoid_weight(j - 1, nt);
      a.w_old = trapezoid_weight(nt, nt);
      a.acc = lv.acc;
      a.st_acc = (long long)(2 * F);
      a.addf = leray ? nullptr : L.bAv;  // with K, beta A v is added after the projection
      a.st_addf = (long long)(2 * F);
      a.out2 = lv.g;
      a.st_out2 = (long long)(2 * F);
      a.partial = partial;
      HIPCHK(sl_step<T>(stream, StepKind::Adjoint, a, &nb));
    }
    if (leray) {  // g = beta A v + K b, then its norms
      HIPCHK(spec_scale<T>(stream, lv.sg, B, mk, symK(Symbol::One), 2, lv.g, lv.g, L.bAv, lv.S1, lv.S2));
      HIPCHK(norms<T>(stream, B, 2 * F, lv.g, partial, dres));
    } else {
      HIPCHK(finish(stream, B, nb, 2, 2LL * nb, 2, 2u, partial, dres));
    }
    const double* r = fetch(0);
    g2.assign(B, 0.0);
    ginf.assign(B, 0.0);
    for (int z = 0; z < B; ++z) {
      if (!hmask.empty() && !hmask[z]) continue;
      g2[z] = r[4 * z];
      ginf[z] = r[4 * z + 1];
      if (!std::isfinite(g2[z]) || (leray && r[4 * z + 2] > 0)) throw Fail{SLNK_ENAN, "non-finite gradient"};
    }
  }

  // bt = Q[vt] (the transport part of the GN matvec) at slot 0 of lv, items of mk
  void gn_transport(Level<T>& lv, const T* vt, const int* mk) {
    auto& L = lv.lin[0];
    ensure_gm(lv);
    const size_t F = lv.F;
    const int nt = lv.nt;
    int nb = 0;
    // while capturing, the LDS is sized for halo_cap so that the graph stays valid for every
    // later linearisation whose halos fit under it
    for (int j = 1; j <= nt; ++j) {  // incremental state, forward
      StepArgs<T> a = step_base(lv, 0, mk, capturing);
      a.first = j == 1;
      a.last = j == nt;
      a.src = a.first ? nullptr : lv.q + ((j - 1) % 2) * F;
      a.dst = lv.q + (j % 2) * F;
      a.st_src = a.st_dst = (long long)(2 * F);
      a.d1 = L.df;
      a.st_d = (long long)(2 * F);
      a.vt = vt;
      a.st_vt = (long long)(2 * F);
      a.gm_old = L.gm;
      a.gm_new = L.gm + 2 * j * F;
      a.st_gm = (long long)(2 * (nt + 1) * F);
      a.w_new = trapezoid_weight(nt, nt);
      a.acc = lv.bt;
      a.st_acc = (long long)(2 * F);
      HIPCHK(sl_step<T>(stream, StepKind::IncState, a, &nb));
    }
    for (int j = nt; j >= 1; --j) {  // incremental adjoint, backward
      StepArgs<T> a = step_base(lv, 0, mk, capturing);
      a.src = lv.q + (j % 2) * F;
      a.dst = j > 1 ? lv.q + ((j - 1) % 2) * F : nullptr;
      a.st_src = a.st_dst = (long long)(2 * F);
      a.d1 = L.da;
      a.st_d = (long long)(2 * F);
      a.gamma = L.gamma;
      a.st_gamma = (long long)F;
      a.gm_new = L.gm + 2 * (j - 1) * F;
      a.st_gm = (long long)(2 * (nt + 1) * F);
      a.w_new = trapezoid_weight(j - 1, nt);
      a.acc = lv.bt;
      a.st_acc = (long long)(2 * F);
      HIPCHK(sl_step<T>(stream, StepKind::IncAdjoint, a, &nb));
    }
  }

  // bt = Q[vt] of the full-Newton matvec at slot 0 of the fine level, items of mk:
  // K int_0^1 (lam~ grad m + lam grad m~) dt, the incremental adjoint carrying the source
  // sigma = div(lam vt) by Heun's step along the adjoint characteristic:
  //   lam~^{j-1} = gamma I[lam~^j](X_a) + ht/2 (1 + ht div v) I[sigma^j](X_a) + ht/2 sigma^{j-1}
  // (eqs. e:hessian-matvec, e:inc-adj-slm).  Needs the adjoint levels kept by gradient().
  void fn_transport(Level<T>& lv, const T* vt, const int* mk) {
    auto& L = lv.lin[0];
    ensure_gm(lv);
    const size_t F = lv.F;
    const int nt = lv.nt;
    const double ht = 1.0 / nt;
    int nb = 0;
    HIPCHK(fn_products<T>(stream, B, F, nt, fn.lam, vt, fn.x2));
    HIPCHK(spec_div<T>(stream, lv.sg, B * (nt + 1), fn.x2, fn.sigma, lv.S1, lv.S2));
    for (int j = 1; j <= nt; ++j) {  // I[sigma^j](X_a)
      StepArgs<T> a = step_base(lv, 0, mk, capturing);
      a.src = fn.sigma + j * F;
      a.st_src = (long long)((nt + 1) * F);
      a.dst = fn.e + (j - 1) * F;
      a.st_dst = (long long)(nt * F);
      a.d1 = L.da;
      a.st_d = (long long)(2 * F);
      HIPCHK(sl_step<T>(stream, StepKind::State, a, &nb));
    }
    HIPCHK(fn_source<T>(stream, B, F, nt, ht, fn.divv, fn.sigma, fn.e));
    for (int j = 1; j <= nt; ++j) {  // incremental state, forward, keeping m~^j
      StepArgs<T> a = step_base(lv, 0, mk, capturing);
      a.first = j == 1;
      a.last = j == nt;
      a.src = a.first ? nullptr : lv.q + ((j - 1) % 2) * F;
      a.dst = lv.q + (j % 2) * F;
      a.st_src = a.st_dst = (long long)(2 * F);
      a.d1 = L.df;
      a.st_d = (long long)(2 * F);
      a.vt = vt;
      a.st_vt = (long long)(2 * F);
      a.gm_old = L.gm;
      a.gm_new = L.gm + 2 * j * F;
      a.st_gm = (long long)(2 * (nt + 1) * F);
      a.w_new = trapezoid_weight(nt, nt);
      a.acc = lv.bt;
      a.st_acc = (long long)(2 * F);
      a.out2 = fn.mt + (j - 1) * F;
      a.st_out2 = (long long)(nt * F);
      HIPCHK(sl_step<T>(stream, StepKind::IncState, a, &nb));
    }
    HIPCHK(spec_grad<T>(stream, lv.sg, B * nt, fn.mt, fn.x2, lv.S1, lv.S2));
    for (int j = nt; j >= 1; --j) {  // incremental adjoint, backward, with its source
      StepArgs<T> a = step_base(lv, 0, mk, capturing);
      a.src = lv.q + (j % 2) * F;
      a.dst = j > 1 ? lv.q + ((j - 1) % 2) * F : nullptr;
      a.st_src = a.st_dst = (long long)(2 * F);
      a.d1 = L.da;
      a.st_d = (long long)(2 * F);
      a.gamma = L.gamma;
      a.st_gamma = (long long)F;
      a.gm_new = L.gm + 2 * (j - 1) * F;
      a.st_gm = (long long)(2 * (nt + 1) * F);
      a.w_new = trapezoid_weight(j - 1, nt);
      a.acc = lv.bt;
      a.st_acc = (long long)(2 * F);
      a.addf = fn.e + (j - 1) * F;
      a.st_addf = (long long)(nt * F);
      HIPCHK(sl_step<T>(stream, StepKind::IncAdjoint, a, &nb));
    }
    HIPCHK(fn_accumulate<T>(stream, B, F, nt, ht, fn.lam, fn.x2, lv.bt, mk));
  }

  // the transport part of the fine matvec the parameters select; the coarse level is always GN
  void transport(Level<T>& lv, const T* vt, const int* mk) {
    if (rk2a && &lv == &fine)
      rk2a_transport(lv, vt);
    else if (full_newton && &lv == &fine)
      fn_transport(lv, vt, mk);
    else
      gn_transport(lv, vt, mk);
  }

  // out = beta A vt + Q vt.  In the mixed context beta A vt is formed in FP64 from the FP32 input
  // and added to the FP32 transport part in FP64 before the one rounding of the output: an FP32
  // transform would leave rounding noise of about eps ||vt|| on every mode, which beta a(k)
  // multiplies by up to beta max|k|^(2 reg) (1e6 for H2 at 256^2, beta = 1e-3).
  void hessian(Level<T>& lv, const T* vt, T* out, const int* mk) {
    transport(lv, vt, mk);
    if (leray) HIPCHK(spec_scale<T>(stream, lv.sg, B, mk, symK(Symbol::One), 2, lv.bt, lv.bt, nullptr, lv.S1, lv.S2));
    if (std::is_same_v<T, float> && &lv == &fine) {  // sg64 belongs to the fine grid
      HIPCHK((spec_scale<double, T>(stream, sg64, B, mk, sym(Symbol::Reg), 2, vt, out, lv.bt, S64a, S64b)));
    } else {
      HIPCHK(spec_scale<T>(stream, lv.sg, B, mk, sym(Symbol::Reg), 2, vt, out, lv.bt, lv.S1, lv.S2));
    }
  }

  // out = s + S Q S s
  void split_matvec(Level<T>& lv, const T* s, T* out, const int* mk) {
    HIPCHK(spec_scale<T>(stream, lv.sg, B, mk, sym(Symbol::RegInvSqrt), 2, s, lv.w, nullptr, lv.S1, lv.S2));
    transport(lv, lv.w, mk);
    HIPCHK(spec_scale<T>(stream, lv.sg, B, mk, symK(Symbol::RegInvSqrt), 2, lv.bt, out, s, lv.S1, lv.S2));
  }

  // out = s + S Q(0) S s on the coarse level (closed form of the v = 0 operator)
  void split_matvec_zero(Level<T>& lv, const T* s, T* out) {
    HIPCHK(spec_scale<T>(stream, lv.sg, B, nullptr, sym(Symbol::RegInvSqrt), 2, s, lv.w, nullptr, lv.S1, lv.S2));
    HIPCHK(q_at_zero<T>(stream, B, lv.F, lv.w, lv.gmT, 1.0, lv.bt));
    HIPCHK(spec_scale<T>(stream, lv.sg, B, nullptr, symK(Symbol::RegInvSqrt), 2, lv.bt, out, s, lv.S1, lv.S2));
  }

  // per-item dot products of two vector fields (host copies; synchronises)
  std::vector<double> dots(const Level<T>& lv, const T* a, const T* b) {
    HIPCHK(dot<T>(stream, B, 2 * lv.F, a, b, partial, dres));
    const double* r = fetch(0);
    std::vector<double> out(B);
    for (int z = 0; z < B; ++z) out[z] = r[4 * z];
    return out;
  }

  // ---- two-level preconditioner -----------------------------------------------------------
  // Lanczos on (I + S Q S) from one SplitMix64 start vector: tridiagonal coefficients (al, be) per
  // item.  Default: Q = Q(0) in closed form, every item.  With mk / hmask: Q at the coarse level's
  // current linearisation (general transport), only the items of hmask (a re-estimate).
  void lanczos(std::vector<std::vector<double>>& al, std::vector<std::vector<double>>& be, const int* mk = nullptr,
               const std::vector<int>& hmask = {}) {
    const bool current = !hmask.empty();
    const size_t n = 2 * coarse.F;
    std::vector<double> h = splitmix64_uniform(prm.lanczos_seed, n);
    std::vector<T> ht(B * n);
    for (int z = 0; z < B; ++z) std::copy(h.begin(), h.end(), ht.begin() + z * n);
    T* q = coarse.vec[0];
    T* qp = coarse.vec[1];
    T* w = coarse.vec[2];
    HIPCHK(hipMemcpyAsync(q, ht.data(), B * n * sizeof(T), hipMemcpyHostToDevice, stream));
    std::vector<double> nq = dots(coarse, q, q);  // synchronises before ht goes out of scope
    for (auto& x : nq) x = 1.0 / std::sqrt(x);
    put_scalars(0, nq);
    HIPCHK(axpby<T>(stream, B, n, 1.0, sc(0), q, 0.0, nullptr, q));
    HIPCHK(fill<T>(stream, B * n, 0.0, qp));
    // the step scalars stay on the device (k_lanczos_coef); the (alpha, beta) log is read once
    const std::vector<int> live0 = current ? hmask : std::vector<int>(B, 1);
    const int steps = prm.lanczos_steps;
    HIPCHK(set_ints(stream, lz_live, live0.data(), B));
    HIPCHK(fill<double>(stream, B, 0.0, sc(1)));  // beta of the step before the first
    for (int j = 0; j < steps; ++j) {
      if (current)
        split_matvec(coarse, q, w, mk);
      else
        split_matvec_zero(coarse, q, w);
      HIPCHK(axpby<T>(stream, B, n, -1.0, sc(1), qp, 1.0, nullptr, w));
      HIPCHK(dot<T>(stream, B, n, q, w, partial, dres));
      HIPCHK(lanczos_coef(stream, LANCZOS_ALPHA, B, j, steps, dres, lz_live, sc(2), sc(1), sc(3), lz_log));
      HIPCHK(axpby<T>(stream, B, n, -1.0, sc(2), q, 1.0, nullptr, w));
      HIPCHK(dot<T>(stream, B, n, w, w, partial, dres));
      HIPCHK(lanczos_coef(stream, LANCZOS_BETA, B, j, steps, dres, lz_live, sc(2), sc(1), sc(3), lz_log));
      if (j == steps - 1) break;
      std::swap(qp, q);  // qp <- q
      HIPCHK(axpby<T>(stream, B, n, 1.0, sc(3), w, 0.0, nullptr, q));  // q <- w / beta
    }
    std::vector<double> log(size_t(B) * steps * 2);
    HIPCHK(hipMemcpyAsync(log.data(), lz_log, log.size() * sizeof(double), hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    for (int z = 0; z < B; ++z) {
      if (!live0[z]) continue;
      for (int j = 0; j < steps; ++j) {
        const double* e = log.data() + (size_t(z) * steps + j) * 2;
        al[z].push_back(e[0]);
        if (e[1] < 0.0) break;  // last step or breakdown
        be[z].push_back(e[1]);
      }
    }
  }

  // e_max from the given per-item values, else from the Lanczos iteration
  void setup_two_level(const std::vector<double>* emax_given = nullptr) {
    // coarse images
    HIPCHK(spec_restrict<T>(stream, fine.sg, coarse.sg, B, nullptr, 1, fine.mT, coarse.mT, nullptr, fine.S1, coarse.S1,
                            coarse.S2));
    HIPCHK(spec_restrict<T>(stream, fine.sg, coarse.sg, B, nullptr, 1, fine.mR, coarse.mR, nullptr, fine.S1, coarse.S1,
                            coarse.S2));
    HIPCHK(spec_grad<T>(stream, coarse.sg, B, coarse.mT, coarse.gmT, coarse.S1, coarse.S2));
    std::vector<std::vector<double>> al(B), be(B);
    if (!emax_given) lanczos(al, be);
    // e_min = min_k 1 + 1 / (beta a'(k)) over the coarse modes: the largest |k|^2 is at the
    // corner (nc1/2, nc2/2)
    const double kk = 0.25 * double(coarse.n1) * coarse.n1 + 0.25 * double(coarse.n2) * coarse.n2;
    for (int z = 0; z < B; ++z) {
      emax[z] = emax_given ? (*emax_given)[z] : prm.emax_safety * tridiag_max_eig(al[z], be[z]);
      emin[z] = 1.0 + 1.0 / (prm.beta * std::pow(kk, prm.reg));
    }
    cheb_tables();
    emax_setup = emax;
  }

  // New e_max for the items of hmask whose CHEB(k) turned out indefinite (section 4.2.1:
  // re-estimate once the preconditioner deteriorates): Lanczos on the coarse split operator at
  // the current coarse linearisation, same start vector and safety factor as the set-up.
  void reestimate_emax(const int* mk, const std::vector<int>& hmask) {
    std::vector<std::vector<double>> al(B), be(B);
    lanczos(al, be, mk, hmask);
    for (int z = 0; z < B; ++z)
      if (hmask[z]) emax[z] = prm.emax_safety * tridiag_max_eig(al[z], be[z]);
    cheb_tables();
  }

  // Chebyshev step coefficients of every item from its bounds (device tables read by the
  // preconditioner, also from captured graphs)
  void cheb_tables() {
    const int k = prm.cheb_iters;
    std::vector<double> itheta(B), tab(2 * size_t(k) * B, 0.0);
    for (int z = 0; z < B; ++z) {
      if (!(emax[z] > emin[z]) || !std::isfinite(emax[z])) throw Fail{SLNK_ENAN, "invalid Chebyshev bound e_max"};
      // Chebyshev recurrence of every step (Saad, Algorithm 12.1): d <- c1[i] d + c2[i] r
      const double theta = 0.5 * (emax[z] + emin[z]), delta = 0.5 * (emax[z] - emin[z]);
      const double sigma = theta / delta;
      double rho = 1.0 / sigma;
      itheta[z] = 1.0 / theta;
      for (int i = 0; i < k; ++i) {
        const double rho_next = 1.0 / (2.0 * sigma - rho);
        tab[size_t(i) * B + z] = rho_next * rho;
        tab[(size_t(k) + i) * B + z] = 2.0 * rho_next / delta;
        rho = rho_next;
      }
    }
    HIPCHK(hipMemcpyAsync(cheb_tab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice, stream));
    HIPCHK(hipMemcpyAsync(inv_theta, itheta.data(), B * sizeof(double), hipMemcpyHostToDevice, stream));
    HIPCHK(hipStreamSynchronize(stream));
  }

  // coarse linearisation at the restriction of the fine slot-0 velocity, items of mk / hmask
  void linearize_coarse(const int* mk, const std::vector<int>& hmask) {
    HIPCHK(spec_restrict<T>(stream, fine.sg, coarse.sg, B, mk, 2, fine.lin[0].v, coarse.vec[7], nullptr, fine.S1,
                            coarse.S1, coarse.S2));
    linearize(coarse, 0, coarse.vec[7], false, nullptr, mk, hmask);
    ensure_gm(coarse);
  }

  // x = CHEB_k(M_c) b on the coarse level (Saad, Algorithm 12.1, from x = 0; x, b distinct).
  // The iteration carries y = S d and u = S r next to d and r: M d = d + S Q y, so each step
  // needs the transport chain Q y and one spectral transform giving S Q y and S^2 Q y, which
  // also update u; one fused kernel then updates r, u, d, y, x.
  void chebyshev(const T* b, T* x, const int* mk) {
    const size_t n = 2 * coarse.F;
    T* r = coarse.vec[3];
    T* d = coarse.vec[4];
    T* u = coarse.vec[5];
    T* y = coarse.vec[0];
    T* sb = coarse.vec[1];
    T* s2b = coarse.w;
    const int k = prm.cheb_iters;
    HIPCHK(axpby<T>(stream, B, n, 1.0, nullptr, b, 0.0, nullptr, r));
    HIPCHK(axpby<T>(stream, B, n, 1.0, inv_theta, b, 0.0, nullptr, d));
    HIPCHK(axpby<T>(stream, B, n, 1.0, nullptr, d, 0.0, nullptr, x));
    if (k == 1) return;
    HIPCHK(spec_scale<T>(stream, coarse.sg, B, mk, sym(Symbol::RegInvSqrt), 2, b, u, nullptr, coarse.S1, coarse.S2));
    HIPCHK(axpby<T>(stream, B, n, 1.0, inv_theta, u, 0.0, nullptr, y));
    const bool fused = spec_fast<T>(coarse.sg);
    for (int i = 0; i < k - 1; ++i) {
      gn_transport(coarse, y, mk);
      const double* c1 = cheb_tab + size_t(i) * B;
      const double* c2 = cheb_tab + (size_t(k) + i) * B;
      if (fused) {
        // the inverse row pass of S Q y, S^2 Q y applies the step in place
        HIPCHK(spec_scale2_cheb<T>(stream, coarse.sg, B, mk, symK(Symbol::RegInvSqrt), sym(Symbol::RegInv), coarse.bt,
                                   ChebTail<T>{r, d, x, u, y, c1, c2}, coarse.S1, coarse.S2));
      } else {
        HIPCHK(spec_scale2<T>(stream, coarse.sg, B, mk, symK(Symbol::RegInvSqrt), sym(Symbol::RegInv), coarse.bt, sb,
                              s2b, coarse.S1, coarse.S2));
        HIPCHK(cheb_step<T>(stream, B, n, c1, c2, r, u, d, y, x, sb, s2b));
      }
    }
  }

  // Run 'body' (device work only, no synchronisation) from a graph captured for 'key', or
  // directly when graphs are off or a current halo exceeds the graphed footprint.
  template <class Fn>
  void graphed(std::tuple<int, const void*, const void*, const void*> key, bool eligible, Fn&& body) {
    if (!use_graphs || !eligible) {
      body();
      return;
    }
    auto it = graphs.find(key);
    if (it == graphs.end()) {
      if (graphs.size() >= 32) clear_graphs();  // callers cycling through many buffers
      hipStream_t user = stream;
      stream = cap_stream;
      capturing = true;
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        try {
          body();
        } catch (...) {
          (void)hipStreamEndCapture(cap_stream, &g);
          if (g) (void)hipGraphDestroy(g);
          stream = user;
          capturing = false;
          throw;
        }
        e = hipStreamEndCapture(cap_stream, &g);
      }
      stream = user;
      capturing = false;
      if (e != hipSuccess) throw Fail{SLNK_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e)};
      hipGraphExec_t ex = nullptr;
      e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) throw Fail{SLNK_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e)};
      it = graphs.emplace(key, ex).first;
    }
    HIPCHK(hipGraphLaunch(it->second, stream));
  }

  bool halo_fits(const Level<T>& lv) const { return prm.sl_path == 1 || lv.max_halo(0, {}) <= halo_cap; }

  void count(std::vector<int>& c, const std::vector<int>& hmask, int by) {
    for (int z = 0; z < B; ++z)
      if (hmask.empty() || hmask[z]) c[z] += by;
  }

  // PCG(eps) coarse solve (section 3.4.2): CG on the coarse split operator M_c x = b (itself
  // spectrally preconditioned, so the inner preconditioner is the identity) from zero, per item to
  // ||b - M_c x|| <= coarse_eps * outer_tol[z] * ||b|| or kMaxInner steps, in lock step over the
  // items of hmask (empty: all); the step coefficients stay in device memory (rows 10-13 of the
  // scalar block) and the host synchronises once per step.
  void coarse_cg(const T* b, T* x, const std::vector<int>& hmask) {
    const size_t n = 2 * coarse.F;
    T* r = coarse.vec[0];
    T* p = coarse.vec[1];
    T* q = coarse.vec[3];
    double* rz = sc(13);
    const int* cm = mask(kMaskCoarse);
    std::vector<int> active = hmask.empty() ? std::vector<int>(B, 1) : hmask;
    HIPCHK(fill<T>(stream, B * n, 0.0, x));
    HIPCHK(axpby<T>(stream, B, n, 1.0, nullptr, b, 0.0, nullptr, r));
    HIPCHK(axpby<T>(stream, B, n, 1.0, nullptr, b, 0.0, nullptr, p));
    std::vector<double> bn = dots(coarse, b, b);
    for (int k = 0; k < B; ++k)
      if (bn[k] == 0.0) active[k] = 0;
    if (!any_of(active)) return;
    put_mask(kMaskCoarse, active);
    HIPCHK(dot<T>(stream, B, n, r, r, partial, dres));
    HIPCHK(pcg_coef(stream, PCG_RZ, B, cm, dres, rz, nullptr, nullptr));
    for (int it = 1; it <= kMaxInner; ++it) {
      graphed({3, p, q, cm}, halo_fits(coarse), [&] { split_matvec(coarse, p, q, cm); });
      count(n_coarse, active, 1);
      HIPCHK(dot<T>(stream, B, n, p, q, partial, dres + 4 * B));
      HIPCHK(pcg_coef(stream, PCG_ALPHA, B, cm, dres + 4 * B, rz, sc(10), nullptr));
      HIPCHK(axpby<T>(stream, B, n, 1.0, sc(10), p, 1.0, nullptr, x));
      HIPCHK(axpby<T>(stream, B, n, -1.0, sc(10), q, 1.0, nullptr, r));
      HIPCHK(dot<T>(stream, B, n, r, r, partial, dres));
      fetch_both();
      bool more = false;
      for (int k = 0; k < B; ++k) {
        if (!active[k]) continue;
        const double pq = hres[4 * B + 4 * k], rr = hres[4 * k];
        if (!std::isfinite(pq) || !std::isfinite(rr)) throw Fail{SLNK_ENAN, "non-finite coarse PCG"};
        // non-positive curvature cannot occur for the positive definite coarse operator but in
        // rounding: stop the item with its current iterate
        if (pq <= 0.0 || std::sqrt(rr) <= prm.coarse_eps * outer_tol[k] * std::sqrt(bn[k]))
          active[k] = 0;
        else
          more = true;
      }
      if (!more) break;
      put_mask(kMaskCoarse, active);
      // p <- r + beta p, beta = (r.r)_new / (r.r)_old
      HIPCHK(pcg_coef(stream, PCG_BETA, B, cm, dres, rz, sc(11), sc(12)));
      HIPCHK(axpby<T>(stream, B, n, 1.0, sc(11), r, 1.0, sc(12), p));
    }
  }

  void precond(const T* r, T* z, const int* mk, const std::vector<int>& hmask) {
    const auto& pe = prec_event();
    HIPCHK(hipEventRecord(pe.first, stream));
    if (!two_level) {
      HIPCHK(spec_scale<T>(stream, fine.sg, B, mk, sym(Symbol::RegInv), 2, r, z, nullptr, fine.S1, fine.S2));
    } else if (coarse_pcg) {
      T* rc = coarse.vec[6];
      T* zc = coarse.vec[2];
      HIPCHK(spec_restrict<T>(stream, fine.sg, coarse.sg, B, mk, 2, r, rc, fine.Sk, fine.S1, coarse.S1, coarse.S2));
      coarse_cg(rc, zc, hmask);
      HIPCHK(spec_prolong_combine<T>(stream, fine.sg, coarse.sg, B, mk, 2, fine.Sk, zc, z, fine.S1, coarse.S1,
                                     coarse.S2));
    } else {
      graphed({1, r, z, mk}, halo_fits(coarse), [&] {
        T* rc = coarse.vec[6];
        T* zc = coarse.vec[2];
        HIPCHK(spec_restrict<T>(stream, fine.sg, coarse.sg, B, mk, 2, r, rc, fine.Sk, fine.S1, coarse.S1, coarse.S2));
        chebyshev(rc, zc, mk);
        HIPCHK(spec_prolong_combine<T>(stream, fine.sg, coarse.sg, B, mk, 2, fine.Sk, zc, z, fine.S1, coarse.S1,
                                       coarse.S2));
      });
      count(n_coarse, hmask, prm.cheb_iters - 1);
    }
    HIPCHK(hipEventRecord(pe.second, stream));
  }

  // fine operator of the Krylov solve: H (P_REG) or the split operator (P_2L)
  void op(const T* x, T* y, const int* mk, const std::vector<int>& hmask) {
    count(n_matvec, hmask, 1);
    ensure_gm(fine);
    graphed({2, x, y, mk}, halo_fits(fine), [&] {
      if (two_level)
        split_matvec(fine, x, y, mk);
      else
        hessian(fine, x, y, mk);
    });
  }

  // Per-item PCG from zero on op x = b (relative tolerances tol[z]), in lock step over the items
  // of 'active'.  Iterations and status of each item in its / st (SLNK_OK, SLNK_EMAXIT,
  // SLNK_ENEGCURV, or SLNK_ECHEB_DIVERGED when the r.z of a step was not positive).  Stopped items see zero step
  // coefficients, which leave their x and r untouched.  The step coefficients are formed in device
  // memory (rz in row 9 of the scalar block); the host synchronises once per iteration, to read the
  // curvature p.q together with the residual norm.
  void pcg(const T* b, T* x, const std::vector<double>& tol, int maxit, std::vector<int> active, std::vector<int>& its,
           std::vector<int>& st) {
    const size_t n = 2 * fine.F;
    T* r = fine.vec[0];
    T* z = fine.vec[1];
    T* p = fine.vec[2];
    T* q = fine.vec[3];
    double* rz = sc(9);
    double* pq_dev = dres + 4 * B;
    its.assign(B, 0);
    st.assign(B, SLNK_OK);
    HIPCHK(fill<T>(stream, B * n, 0.0, x));
    HIPCHK(axpby<T>(stream, B, n, 1.0, nullptr, b, 0.0, nullptr, r));
    std::vector<double> bnorm = dots(fine, b, b);
    for (int k = 0; k < B; ++k) {
      bnorm[k] = std::sqrt(bnorm[k]);
      if (bnorm[k] == 0.0) active[k] = 0;
    }
    if (!any_of(active)) return;
    const int* mk = mask(kMaskPcg);
    put_mask(kMaskPcg, active);
    for (int k = 0; k < B; ++k) outer_tol[k] = tol[k];  // scales the PCG(eps) coarse tolerance
    // r.z goes to slot 1 of the second result half, which the per-iteration fetch returns with
    // p.q: a preconditioner that is not positive definite shows as r.z <= 0
    double* rz_dev = dres + 4 * B + 1;
    precond(r, z, mk, active);
    HIPCHK(axpby<T>(stream, B, n, 1.0, nullptr, z, 0.0, nullptr, p));
    HIPCHK(dot<T>(stream, B, n, r, z, partial, rz_dev));
    HIPCHK(pcg_coef(stream, PCG_RZ, B, mk, rz_dev, rz, nullptr, nullptr));
    std::vector<int> mask_set = active;  // the contents of kMaskPcg (rewritten only on a change)
    for (int it = 1; it <= maxit; ++it) {
      op(p, q, mk, active);
      HIPCHK(dot<T>(stream, B, n, p, q, partial, pq_dev));
      HIPCHK(pcg_coef(stream, PCG_ALPHA, B, mk, pq_dev, rz, sc(4), nullptr));
      HIPCHK(axpby<T>(stream, B, n, 1.0, sc(4), p, 1.0, nullptr, x));
      HIPCHK(axpby<T>(stream, B, n, -1.0, sc(4), q, 1.0, nullptr, r));
      HIPCHK(dot<T>(stream, B, n, r, r, partial, dres));
      fetch_both();
      const double* rr = hres;
      const double* pq = hres + 4 * B;
      bool more = false;
      for (int k = 0; k < B; ++k) {
        if (!active[k]) continue;
        its[k] = it;
        if (!std::isfinite(pq[4 * k])) throw Fail{SLNK_ENAN, "non-finite curvature in PCG"};
        if (pq[4 * k] <= 0.0) {
          // non-positive curvature: stop with the current iterate (at the first step, the
          // preconditioned residual); the step coefficient was zero
          if (it == 1) HIPCHK(masked_copy<T>(stream, 1, n, z + k * n, 0, x + k * n, 0, nullptr));
          st[k] = SLNK_ENEGCURV;
          active[k] = 0;
          continue;
        }
        if (std::sqrt(rr[4 * k]) <= tol[k] * bnorm[k]) {
          active[k] = 0;
        } else if (!(pq[4 * k + 1] > 0.0)) {
          // the r.z that gave this step was not positive: the preconditioner is indefinite and
          // the iterate of no use (the caller re-estimates the Chebyshev bounds)
          st[k] = SLNK_ECHEB_DIVERGED;
          active[k] = 0;
        } else {
          more = true;
        }
      }
      if (!more) return;
      if (it == maxit) break;
      if (active != mask_set) {
        put_mask(kMaskPcg, active);
        mask_set = active;
      }
      precond(r, z, mk, active);
      HIPCHK(dot<T>(stream, B, n, r, z, partial, rz_dev));
      // p <- z + beta p for the running items; stopped items keep p (coefficients 0, 1)
      HIPCHK(pcg_coef(stream, PCG_BETA, B, mk, rz_dev, rz, sc(6), sc(7)));
      HIPCHK(axpby<T>(stream, B, n, 1.0, sc(6), z, 1.0, sc(7), p));
    }
    for (int k = 0; k < B; ++k)
      if (active[k]) st[k] = SLNK_EMAXIT;
  }

  // ---- kernel timing ----------------------------------------------------------------------
  double time_kernel(int which, int reps) {
    auto& lv = fine;
    auto& L = lv.lin[0];
    ensure_gm(lv);
    const size_t F = lv.F;
    const double ht = 1.0 / lv.nt;
    // sources with sane values: the state (twice) and a zeroed accumulator
    HIPCHK(masked_copy<T>(stream, B, F, L.m, (long long)((lv.nt + 1) * F), lv.q, (long long)(2 * F), nullptr));
    HIPCHK(masked_copy<T>(stream, B, F, L.m, (long long)((lv.nt + 1) * F), lv.q + F, (long long)(2 * F), nullptr));
    HIPCHK(fill<T>(stream, B * 2 * F, 0.0, lv.acc));
    auto one = [&](int r) {
      StepArgs<T> a = step_base(lv, 0, nullptr, false);
      a.src = lv.q + (r % 2) * F;
      a.dst = lv.q + ((r + 1) % 2) * F;
      a.st_src = a.st_dst = (long long)(2 * F);
      a.gamma = L.gamma;
      a.st_gamma = (long long)F;
      a.gm_new = L.gm;
      a.st_gm = (long long)(2 * (lv.nt + 1) * F);
      a.w_new = 1e-3;
      a.acc = lv.acc;
      a.st_acc = (long long)(2 * F);
      a.vt = L.v;
      a.st_vt = (long long)(2 * F);
      a.st_d = (long long)(2 * F);
      int nb = 0;
      switch (which) {
        case 0:
          a.d1 = L.df;
          HIPCHK(sl_step<T>(stream, StepKind::State, a, &nb));
          break;
        case 1:
          a.d1 = L.da;
          HIPCHK(sl_step<T>(stream, StepKind::Adjoint, a, &nb));
          break;
        case 2:
          a.d1 = L.df;
          HIPCHK(sl_step<T>(stream, StepKind::IncState, a, &nb));
          break;
        case 3:
          a.d1 = L.da;
          HIPCHK(sl_step<T>(stream, StepKind::IncAdjoint, a, &nb));
          break;
        case 4:  // outputs into work buffers of matching sizes (2F, 2F, F per item)
          HIPCHK(sl_trace<T>(stream, lv.n1, lv.n2, B, nullptr, ht, L.v, lv.cv, lv.divv, lv.cdiv, lv.w, lv.bt, lv.coef,
                             nullptr, &nb));
          break;
        case 5:
          HIPCHK(spec_scale<T>(stream, lv.sg, B, nullptr, sym(Symbol::RegInvSqrt), 2, L.v, lv.w, nullptr, lv.S1,
                               lv.S2));
          break;
        default:  // recomputes grad m in place (same values)
          HIPCHK(spec_grad<T>(stream, lv.sg, B * (lv.nt + 1), L.m, L.gm, lv.S1, lv.S2));
      }
    };
    one(0);  // first launch outside the timed region (LDS attribute, constant upload)
    // back-to-back launches between one pair of events: for a kernel that fills the device this
    // is its average duration (the same figure a kernel trace reports)
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, stream));
    for (int r = 0; r < reps; ++r) one(r);
    HIPCHK(hipEventRecord(e1, stream));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return double(ms) / reps;
  }

  // ---- tuning ---------------------------------------------------------------------------------
  // switch the SL kernel path / graph replay (captured graphs are dropped)
  void retune(int sl_path, int graphs_on) {
    prm.sl_path = sl_path;
    use_graphs = graphs_on != 0;
    clear_graphs();
  }

  // average time (ms) of one application of the Krylov operator at the current linearisation
  // (all items), after one untimed application
  double time_operator(const T* x, T* y, int reps) {
    op(x, y, mask(kMaskAll), {});
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, stream));
    for (int r = 0; r < reps; ++r) op(x, y, mask(kMaskAll), {});
    HIPCHK(hipEventRecord(e1, stream));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return double(ms) / reps;
  }

  // ---- Newton -------------------------------------------------------------------------------
  // slot 1 -> slot 0 for the accepted items (device mask(kMaskLs) == host 'acc')
  void promote_trial(const std::vector<int>& acc) {
    if (!any_of(acc)) return;
    const size_t F = fine.F;
    const int nt = fine.nt;
    const int* mk = mask(kMaskLs);
    auto& L0 = fine.lin[0];
    auto& L1 = fine.lin[1];
    auto cp = [&](const T* a, T* b, size_t cnt) {
      HIPCHK(masked_copy<T>(stream, B, cnt, a, (long long)cnt, b, (long long)cnt, mk));
    };
    cp(L1.v, L0.v, 2 * F);
    cp(L1.df, L0.df, 2 * F);
    cp(L1.da, L0.da, 2 * F);
    cp(L1.gamma, L0.gamma, F);
    cp(L1.m, L0.m, (nt + 1) * F);
    cp(L1.bAv, L0.bAv, 2 * F);
    HIPCHK(masked_copy<double>(stream, B, 2 * F, v64[1], 2 * F, v64[0], 2 * F, mk));
    HIPCHK(masked_copy<double>(stream, B, 2 * F, bAv64[1], 2 * F, bAv64[0], 2 * F, mk));
    for (int z = 0; z < B; ++z)
      if (acc[z]) {
        L0.J[z] = L1.J[z];
        L0.Jreg[z] = L1.Jreg[z];
        L0.halo[z] = L1.halo[z];
      }
    HIPCHK(set_ints(stream, fine.halo_dev, L0.halo.data(), B));
    L0.has_gm = false;  // recomputed for every item (unchanged values for the others)
  }

  slnk_status newton(T* v, const slnk_solve_opts& o, slnk_solve_report* rep) {
    const double t_start = now_ms();
    std::vector<slnk_solve_report> R(B);
    for (auto& r : R) std::memset(&r, 0, sizeof(r));
    std::fill(n_matvec.begin(), n_matvec.end(), 0);
    std::fill(n_coarse.begin(), n_coarse.end(), 0);
    prec_used = 0;
    t_prec = 0;
    const size_t n = 2 * fine.F;
    double t_grad = 0, t_pcg = 0, t_ls = 0;
    const std::vector<int> all(B, 1);
    if (two_level && !coarse_pcg && emax != emax_setup) {  // undo an earlier solve's re-estimates
      emax = emax_setup;
      cheb_tables();
    }
    for (int z = 0; z < B; ++z) {
      R[z].emin = two_level ? emin[z] : 0.0;
      R[z].emax = two_level ? emax[z] : 0.0;
    }
    // gradient at v = 0 fixes ||g_0|| (stopping rule of section 3.4.1)
    std::vector<double> g2, ginf;
    double t0 = now_ms();
    T* zero = fine.vec[4];
    HIPCHK(fill<T>(stream, B * n, 0.0, zero));
    linearize(fine, 0, zero, true, nullptr, nullptr, {});
    gradient(fine, nullptr, {}, g2, ginf);
    for (int z = 0; z < B; ++z) {
      R[z].g0_inf = ginf[z];
      R[z].g0_two = std::sqrt(g2[z]);
    }
    // start point
    HIPCHK(norms<T>(stream, B, n, v, partial, dres));
    const double* r0 = fetch(0);
    const std::vector<double> nv(r0, r0 + 4 * B);
    bool warm = false;
    for (int z = 0; z < B; ++z) {
      if (nv[4 * z + 2] > 0) throw Fail{SLNK_ENAN, "non-finite initial velocity"};
      if (nv[4 * z + 1] > 0.0) warm = true;
    }
    std::vector<int> fallback(B, 0);
    if (warm) {
      linearize(fine, 0, v, true, nullptr, nullptr, {});
      std::vector<double> g2w, ginfw;
      gradient(fine, nullptr, {}, g2w, ginfw);
      // keep a start only where it lowers ||g||_inf; elsewhere start again from v = 0
      for (int z = 0; z < B; ++z) {
        fallback[z] = nv[4 * z + 1] > 0.0 && !(ginfw[z] < ginf[z]);
        if (!fallback[z]) g2[z] = g2w[z], ginf[z] = ginfw[z];
      }
      if (any_of(fallback)) {
        put_mask(kMaskLs, fallback);
        linearize(fine, 0, zero, true, nullptr, mask(kMaskLs), fallback);
        std::vector<double> g2f, ginff;
        gradient(fine, mask(kMaskLs), fallback, g2f, ginff);
        for (int z = 0; z < B; ++z)
          if (fallback[z]) g2[z] = g2f[z], ginf[z] = ginff[z];
      }
    }
    for (int z = 0; z < B; ++z) R[z].fallback = fallback[z];
    t_grad += now_ms() - t0;
    std::vector<int> active(B, 1), kit(B, 0), status(B, SLNK_OK);
    std::vector<double> t_stop(B, 0.0);
    T* vt = fine.vec[5];
    T* rhs = fine.vec[6];
    T* s = fine.vec[7];
    const int* mk = mask(kMaskNewton);
    for (int k = 0;; ++k) {
      std::vector<double> eta(B, 0.0);
      for (int z = 0; z < B; ++z) {
        if (!active[z]) continue;
        const double grel = ginf[z] / R[z].g0_inf;
        if (k <= SLNK_REPORT_MAX_ITERS) {
          R[z].grel[k] = grel;
          R[z].J[k] = fine.lin[0].J[z];
        }
        const bool converged = grel <= o.gtol_rel || ginf[z] <= o.gtol_abs;
        if (converged || k >= o.max_newton || k >= SLNK_REPORT_MAX_ITERS) {
          if (!converged) status[z] = SLNK_EMAXIT;  // the Newton limit, not the stop test, ended it
          active[z] = 0;
          kit[z] = k;
          t_stop[z] = now_ms() - t_start;
          continue;
        }
        eta[z] = std::min(0.5, std::sqrt(g2[z]) / R[z].g0_two);
      }
      if (!any_of(active)) break;
      put_mask(kMaskNewton, active);
      t0 = now_ms();
      std::vector<int> its, st;
      if (two_level) {
        linearize_coarse(mk, active);
        HIPCHK(spec_scale<T>(stream, fine.sg, B, mk, sym(Symbol::RegInvSqrt), 2, fine.g, rhs, nullptr, fine.S1,
                             fine.S2));
        HIPCHK(axpby<T>(stream, B, n, -1.0, nullptr, rhs, 0.0, nullptr, rhs));
        pcg(rhs, s, eta, o.max_pcg, active, its, st);
        // an indefinite CHEB(k): new e_max for those items, then their PCG once more from zero
        std::vector<int> redo(B, 0);
        for (int z = 0; z < B; ++z) redo[z] = active[z] && st[z] == SLNK_ECHEB_DIVERGED && !coarse_pcg;
        if (any_of(redo)) {
          put_mask(kMaskNewton, redo);
          reestimate_emax(mk, redo);
          // pcg() starts every item from zero: the retry writes into a spare vector, whose redone
          // items are copied over their steps
          T* s2 = fine.vec[4];
          std::vector<int> its2, st2;
          pcg(rhs, s2, eta, o.max_pcg, redo, its2, st2);
          HIPCHK(masked_copy<T>(stream, B, n, s2, (long long)n, s, (long long)n, mk));
          for (int z = 0; z < B; ++z)
            if (redo[z]) {
              its[z] += its2[z];
              st[z] = st2[z];
              ++R[z].cheb_reestimates;
            }
          put_mask(kMaskNewton, active);
        }
        HIPCHK(spec_scale<T>(stream, fine.sg, B, mk, sym(Symbol::RegInvSqrt), 2, s, vt, nullptr, fine.S1, fine.S2));
      } else {
        HIPCHK(axpby<T>(stream, B, n, -1.0, nullptr, fine.g, 0.0, nullptr, rhs));
        pcg(rhs, vt, eta, o.max_pcg, active, its, st);
      }
      t_pcg += now_ms() - t0;
      for (int z = 0; z < B; ++z) {
        if (!active[z]) continue;
        R[z].pcg_iters += its[z];
        if (k < SLNK_REPORT_MAX_ITERS) R[z].pcg[k] = its[z];
        if (st[z] == SLNK_ECHEB_DIVERGED) {  // still indefinite after a new e_max: stop the item
          status[z] = SLNK_ECHEB_DIVERGED;
          active[z] = 0;
          kit[z] = k;
          t_stop[z] = now_ms() - t_start;
        }
      }
      if (!any_of(active)) break;
      put_mask(kMaskNewton, active);
      // Armijo backtracking per item: trial v + alpha vt (FP64 iterate) in slot 1
      t0 = now_ms();
      std::vector<double> slope = dots(fine, fine.g, vt);
      for (auto& x : slope) x *= fine.cell;
      std::vector<double> alpha(B, 1.0);
      std::vector<int> searching(active), accepted(B, 0);
      for (int hv = 0; hv <= o.max_halvings && any_of(searching); ++hv) {
        put_mask(kMaskLs, searching);
        put_scalars(8, alpha);
        HIPCHK(xpay_mixed<T>(stream, B, n, v64[0], 1.0, sc(8), vt, v64[1], mask(kMaskLs)));
        linearize(fine, 1, nullptr, true, v64[1], mask(kMaskLs), searching);
        for (int z = 0; z < B; ++z) {
          if (!searching[z]) continue;
          ++R[z].line_search_evals;
          if (fine.lin[1].J[z] <= fine.lin[0].J[z] + o.armijo_c1 * alpha[z] * slope[z]) {
            searching[z] = 0;
            accepted[z] = 1;
          } else {
            alpha[z] *= 0.5;
          }
        }
      }
      t_ls += now_ms() - t0;
      for (int z = 0; z < B; ++z)
        if (active[z] && !accepted[z]) {  // no acceptable step: stop at the last iterate
          status[z] = SLNK_ELINESEARCH;
          active[z] = 0;
          kit[z] = k;
          t_stop[z] = now_ms() - t_start;
        }
      // accepted trials become the current linearisation point
      put_mask(kMaskLs, accepted);
      promote_trial(accepted);
      t0 = now_ms();
      if (any_of(active)) {
        put_mask(kMaskNewton, active);
        std::vector<double> g2n, ginfn;
        gradient(fine, mk, active, g2n, ginfn);
        for (int z = 0; z < B; ++z)
          if (active[z]) {
            g2[z] = g2n[z];
            ginf[z] = ginfn[z];
          }
      }
      t_grad += now_ms() - t0;
    }
    HIPCHK(cast_copy<T>(stream, B * n, v64[0], v));
    if (two_level) {  // the coarse problem follows the final iterate
      put_mask(kMaskNewton, all);
      linearize_coarse(mk, {});
    }
    HIPCHK(hipStreamSynchronize(stream));
    fold_prec_time();
    has_grad = true;
    const double t_total = now_ms() - t_start;
    slnk_status overall = SLNK_OK;
    for (int z = 0; z < B; ++z) {
      R[z].status = status[z];
      R[z].newton_iters = kit[z];
      R[z].matvecs = n_matvec[z];
      R[z].coarse_matvecs = n_coarse[z];
      R[z].time_total_ms = t_total;
      R[z].time_to_stop_ms = t_stop[z];
      R[z].time_gradient_ms = t_grad;
      R[z].time_pcg_ms = t_pcg;
      R[z].time_precond_ms = t_prec;
      R[z].time_linesearch_ms = t_ls;
      // a failed item's status outranks the informational SLNK_EMAXIT
      if (status[z] != SLNK_OK && (overall == SLNK_OK || overall == SLNK_EMAXIT)) overall = slnk_status(status[z]);
      if (rep) rep[z] = R[z];
    }
    return overall;
  }
};

}  // namespace
}  // namespace slnk

// ============================================================================================
// C ABI
// ============================================================================================
struct slnk_ctx {
  std::string err;
  std::unique_ptr<slnk::Context<float>> f;
  std::unique_ptr<slnk::Context<double>> d;
};

namespace {

template <class Fn>
slnk_status guarded(slnk_ctx* c, Fn&& fn) {
  if (!c) return SLNK_EINVAL;
  try {
    fn();
    return SLNK_OK;
  } catch (const slnk::Fail& e) {
    c->err = e.msg;
    return e.st;
  } catch (const std::exception& e) {
    c->err = e.what();
    return SLNK_EDEVICE;
  }
}

template <class Fn>
slnk_status dispatch(slnk_ctx* c, Fn&& fn) {
  return guarded(c, [&] {
    if (c->f)
      fn(*c->f);
    else
      fn(*c->d);
  });
}

}  // namespace

extern "C" {

void slnk_default_params(slnk_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->n1 = p->n2 = 256;
  p->nt = 4;
  p->reg = SLNK_REG_H2;
  p->beta = 1e-3;
  p->prec = SLNK_PREC_MIXED;
  p->pc = SLNK_PC_2L;
  p->cheb_iters = 10;
  p->lanczos_steps = 30;
  p->emax_safety = 1.05;
  p->lanczos_seed = 0x5EED;
  p->use_graphs = 1;
  p->batch = 1;
  p->coarse_solver = SLNK_COARSE_CHEB;
  p->coarse_eps = 0.1;
}

void slnk_default_opts(slnk_solve_opts* o) {
  if (!o) return;
  o->max_newton = 10;
  o->gtol_rel = 1e-2;
  o->gtol_abs = 1e-5;
  o->max_pcg = 500;
  o->armijo_c1 = 1e-4;
  o->max_halvings = 10;
}

slnk_status slnk_create(const slnk_params* params, void* hip_stream, slnk_ctx** out) {
  if (!params || !out) return SLNK_EINVAL;
  *out = nullptr;
  if (params->prec != SLNK_PREC_FP64 && params->prec != SLNK_PREC_MIXED) return SLNK_EINVAL;
  auto c = std::make_unique<slnk_ctx>();
  slnk_status st = guarded(c.get(), [&] {
    if (params->prec == SLNK_PREC_MIXED) {
      c->f = std::make_unique<slnk::Context<float>>();
      c->f->create(*params, static_cast<hipStream_t>(hip_stream));
    } else {
      c->d = std::make_unique<slnk::Context<double>>();
      c->d->create(*params, static_cast<hipStream_t>(hip_stream));
    }
  });
  if (st != SLNK_OK) {
    if (c->f) c->f->destroy();
    if (c->d) c->d->destroy();
    return st;
  }
  *out = c.release();
  return SLNK_OK;
}

void slnk_destroy(slnk_ctx* ctx) {
  if (!ctx) return;
  if (ctx->f) ctx->f->destroy();
  if (ctx->d) ctx->d->destroy();
  delete ctx;
}

const char* slnk_last_error(const slnk_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

unsigned long long slnk_workspace_bytes(const slnk_ctx* ctx) {
  if (!ctx) return 0;
  return ctx->f ? ctx->f->arena.size : ctx->d->arena.size;
}

slnk_status slnk_set_images(slnk_ctx* ctx, const void* m_R, const void* m_T) {
  if (!m_R || !m_T) return SLNK_EINVAL;
  return dispatch(ctx, [&](auto& C) {
    using T = std::remove_reference_t<decltype(*C.fine.mT)>;
    const size_t n = C.B * C.fine.F;
    HIPCHK(hipMemcpyAsync(C.fine.mR, m_R, n * sizeof(T), hipMemcpyDeviceToDevice, C.stream));
    HIPCHK(hipMemcpyAsync(C.fine.mT, m_T, n * sizeof(T), hipMemcpyDeviceToDevice, C.stream));
    for (T* img : {C.fine.mR, C.fine.mT}) {
      HIPCHK(slnk::norms<T>(C.stream, C.B, C.fine.F, img, C.partial, C.dres));
      const double* r = C.fetch(0);
      for (int z = 0; z < C.B; ++z)
        if (r[4 * z + 2] > 0) throw slnk::Fail{SLNK_ENAN, "non-finite image value"};
    }
    C.fine.lin[0].valid = C.fine.lin[1].valid = false;
    C.has_grad = false;
    C.learned_ready = false;
    C.clear_graphs();
    if (C.two_level) C.setup_two_level();
    C.images_set = true;
  });
}

slnk_status slnk_transport_state(slnk_ctx* ctx, const void* v, const void* m0, void* m1) {
  if (!v || !m0 || !m1) return SLNK_EINVAL;
  return dispatch(ctx, [&](auto& C) {
    using T = std::remove_reference_t<decltype(*C.fine.mT)>;
    auto& lv = C.fine;
    const size_t F = lv.F;
    const int B = C.B;
    // run in the trial slot with a temporary template, then restore the images
    T* saved = lv.vec[0];
    HIPCHK(hipMemcpyAsync(saved, lv.mT, B * F * sizeof(T), hipMemcpyDeviceToDevice, C.stream));
    HIPCHK(hipMemcpyAsync(lv.mT, m0, B * F * sizeof(T), hipMemcpyDeviceToDevice, C.stream));
    C.linearize(lv, 1, static_cast<const T*>(v), false, nullptr, nullptr, {});
    HIPCHK(slnk::masked_copy<T>(C.stream, B, F, lv.lin[1].m + lv.nt * F, (long long)((lv.nt + 1) * F),
                                static_cast<T*>(m1), (long long)F, nullptr));
    HIPCHK(hipMemcpyAsync(lv.mT, saved, B * F * sizeof(T), hipMemcpyDeviceToDevice, C.stream));
    lv.lin[1].valid = false;
    HIPCHK(hipStreamSynchronize(C.stream));
  });
}

slnk_status slnk_objective(slnk_ctx* ctx, const void* v, double* J) {
  if (!v || !J) return SLNK_EINVAL;
  return dispatch(ctx, [&](auto& C) {
    using T = std::remove_reference_t<decltype(*C.fine.mT)>;
    if (!C.images_set) throw slnk::Fail{SLNK_EINVAL, "slnk_set_images must come first"};
    C.has_grad = false;
    C.linearize(C.fine, 0, static_cast<const T*>(v), true, nullptr, nullptr, {});
    for (int z = 0; z < C.B; ++z) J[z] = C.fine.lin[0].J[z];
  });
}

slnk_status slnk_gradient(slnk_ctx* ctx, const void* v, void* g, double* J) {
  if (!v || !g) return SLNK_EINVAL;
  return dispatch(ctx, [&](auto& C) {
    using T = std::remove_reference_t<decltype(*C.fine.mT)>;
    if (!C.images_set) throw slnk::Fail{SLNK_EINVAL, "slnk_set_images must come first"};
    C.has_grad = false;
    C.linearize(C.fine, 0, static_cast<const T*>(v), true, nullptr, nullptr, {});
    std::vector<double> g2, ginf;
    C.gradient(C.fine, nullptr, {}, g2, ginf);
    HIPCHK(hipMemcpyAsync(g, C.fine.g, C.B * 2 * C.fine.F * sizeof(T), hipMemcpyDeviceToDevice, C.stream));
    if (C.two_level) {
      C.put_mask(C.kMaskNewton, std::vector<int>(C.B, 1));
      C.linearize_coarse(C.mask(C.kMaskNewton), {});
    }
    HIPCHK(hipStreamSynchronize(C.stream));
    if (J)
      for (int z = 0; z < C.B; ++z) J[z] = C.fine.lin[0].J[z];
    C.has_grad = true;
  });
}

slnk_status slnk_hessian_matvec(slnk_ctx* ctx, const void* vt, void* Hvt) {
  if (!vt || !Hvt) return SLNK_EINVAL;
  return dispatch(ctx, [&](auto& C) {
    using T = std::remove_reference_t<decltype(*C.fine.mT)>;
    if (!C.has_grad) throw slnk::Fail{SLNK_EINVAL, "no linearisation point: call slnk_gradient first"};
    C.hessian(C.fine, static_cast<const T*>(vt), static_cast<T*>(Hvt), nullptr);
  });
}

slnk_status slnk_split_matvec(slnk_ctx* ctx, const void* s, void* out) {
  if (!s || !out) return SLNK_EINVAL;
  return dispatch(ctx, [&](auto& C) {
    using T = std::remove_reference_t<decltype(*C.fine.mT)>;
    if (!C.has_grad) throw slnk::Fail{SLNK_EINVAL, "no linearisation point: call slnk_gradient first"};
    C.split_matvec(C.fine, static_cast<const T*>(s), static_cast<T*>(out), nullptr);
  });
}

slnk_status slnk_precond_apply(slnk_ctx* ctx, const void* r, void* z) {
  if (!r || !z) return SLNK_EINVAL;
  return dispatch(ctx, [&](auto& C) {
    using T = std::remove_reference_t<decltype(*C.fine.mT)>;
    if (C.two_level && !C.has_grad)
      throw slnk::Fail{SLNK_EINVAL, "P_2L needs a linearisation point: call slnk_gradient first"};
    std::fill(C.outer_tol.begin(), C.outer_tol.end(), 1.0);  // PCG(eps): coarse tolerance eps
    C.precond(static_cast<const T*>(r), static_cast<T*>(z), C.mask(C.kMaskAll), {});
  });
}

slnk_status slnk_get_cheb_bounds(const slnk_ctx* ctx, double* emin, double* emax) {
  if (!ctx || !emin || !emax) return SLNK_EINVAL;
  const auto& lo = ctx->f ? ctx->f->emin : ctx->d->emin;
  const auto& hi = ctx->f ? ctx->f->emax : ctx->d->emax;
  for (size_t z = 0; z < lo.size(); ++z) {
    emin[z] = lo[z];
    emax[z] = hi[z];
  }
  return SLNK_OK;
}

slnk_status slnk_set_cheb_emax(slnk_ctx* ctx, const double* emax) {
  if (!emax) return SLNK_EINVAL;
  return dispatch(ctx, [&](auto& C) {
    if (!C.two_level || !C.images_set) throw slnk::Fail{SLNK_EINVAL, "needs a P_2L context with images set"};
    for (int z = 0; z < C.B; ++z)
      if (!(emax[z] > C.emin[z]) || !std::isfinite(emax[z])) throw slnk::Fail{SLNK_EINVAL, "e_max must exceed e_min"};
    for (int z = 0; z < C.B; ++z) C.emax[z] = emax[z];
    C.cheb_tables();
    C.emax_setup = C.emax;
  });
}

slnk_status slnk_get_field(slnk_ctx* ctx, int which, void* out) {
  if (!out) return SLNK_EINVAL;
  return dispatch(ctx, [&](auto& C) {
    using T = std::remove_reference_t<decltype(*C.fine.mT)>;
    auto& lv = C.fine;
    auto& L = lv.lin[0];
    if (!L.valid) throw slnk::Fail{SLNK_EINVAL, "no linearisation point"};
    const size_t F = lv.F;
    const T* src = nullptr;
    size_t cnt = F;
    long long stride = (long long)F;
    switch (which) {
      case 0: src = L.m + lv.nt * F; stride = (long long)((lv.nt + 1) * F); break;
      case 1: src = L.df; cnt = 2 * F; stride = (long long)(2 * F); break;
      case 2: src = L.da; cnt = 2 * F; stride = (long long)(2 * F); break;
      case 3: src = L.gamma; break;
      case 4: src = lv.lam; stride = (long long)(2 * F); break;
      default: throw slnk::Fail{SLNK_EINVAL, "unknown field"};
    }
    HIPCHK(slnk::masked_copy<T>(C.stream, C.B, cnt, src, stride, static_cast<T*>(out), (long long)cnt, nullptr));
    HIPCHK(hipStreamSynchronize(C.stream));
  });
}

slnk_status slnk_time_kernel(slnk_ctx* ctx, int which, int reps, double* avg_ms) {
  if (!avg_ms || reps < 1 || which < 0 || which > 6) return SLNK_EINVAL;
  return dispatch(ctx, [&](auto& C) {
    if (!C.has_grad) throw slnk::Fail{SLNK_EINVAL, "no linearisation point: call slnk_gradient first"};
    *avg_ms = C.time_kernel(which, reps);
  });
}

slnk_status slnk_newton_solve(slnk_ctx* ctx, void* v_inout, const slnk_solve_opts* opts, slnk_solve_report* report) {
  if (!v_inout) return SLNK_EINVAL;
  slnk_solve_opts o;
  slnk_default_opts(&o);
  if (opts) o = *opts;
  slnk_status result = SLNK_OK;
  slnk_status st = dispatch(ctx, [&](auto& C) {
    using T = std::remove_reference_t<decltype(*C.fine.mT)>;
    if (!C.images_set) throw slnk::Fail{SLNK_EINVAL, "slnk_set_images must come first"};
    if (o.max_newton < 0 || o.max_pcg < 1 || o.max_halvings < 0) throw slnk::Fail{SLNK_EINVAL, "bad options"};
    result = C.newton(static_cast<T*>(v_inout), o, report);
  });
  return st != SLNK_OK ? st : result;
}

namespace {

// v = the modes |k| <= start_kmax of the network's velocity for the context's images; head
// outputs into y (device, may be NULL)
void learned_start(slnk::Context<float>& C, slnk_unet* u, float* v, float* y = nullptr) {
  const slnk_status fs = slnk_unet_forward_on(u, C.stream, C.B, C.fine.n1, C.fine.n2, C.fine.mR, C.fine.mT, v, y);
  if (fs != SLNK_OK) throw slnk::Fail{fs, std::string("network: ") + slnk_unet_last_error(u)};
  const int kmax = slnk_unet_start_kmax(u);
  if (kmax > 0) {
    slnk::SymbolParams sp{slnk::Symbol::Cutoff, C.prm.reg, C.prm.beta, kmax};
    HIPCHK(slnk::spec_scale<float>(C.stream, C.fine.sg, C.B, nullptr, sp, 2, v, v, nullptr, C.fine.S1, C.fine.S2));
  }
}

}  // namespace

slnk_status slnk_set_images_learned(slnk_ctx* ctx, slnk_unet* u, const void* m_R, const void* m_T) {
  if (!ctx || !u || !m_R || !m_T) return SLNK_EINVAL;
  if (!ctx->f) {
    ctx->err = "the learned set-up needs a mixed-precision (FP32 field) context";
    return SLNK_EINVAL;
  }
  return guarded(ctx, [&] {
    auto& C = *ctx->f;
    const size_t n = C.B * C.fine.F;
    HIPCHK(hipMemcpyAsync(C.fine.mR, m_R, n * sizeof(float), hipMemcpyDeviceToDevice, C.stream));
    HIPCHK(hipMemcpyAsync(C.fine.mT, m_T, n * sizeof(float), hipMemcpyDeviceToDevice, C.stream));
    for (float* img : {C.fine.mR, C.fine.mT}) {
      HIPCHK(slnk::norms<float>(C.stream, C.B, C.fine.F, img, C.partial, C.dres));
      const double* r = C.fetch(0);
      for (int z = 0; z < C.B; ++z)
        if (r[4 * z + 2] > 0) throw slnk::Fail{SLNK_ENAN, "non-finite image value"};
    }
    C.fine.lin[0].valid = C.fine.lin[1].valid = false;
    C.has_grad = false;
    C.learned_ready = false;
    C.clear_graphs();
    learned_start(C, u, C.learned_v, C.learned_y);
    std::vector<float> y(C.B);
    HIPCHK(hipMemcpyAsync(y.data(), C.learned_y, C.B * sizeof(float), hipMemcpyDeviceToHost, C.stream));
    HIPCHK(hipStreamSynchronize(C.stream));
    if (C.two_level) {
      // e_max = 1 + 1.1 exp(y) / beta: the head predicts log(beta (e_max - 1)); the factor 1.1 on
      // top of the safety factor of the training targets guards against underestimates
      std::vector<double> emax(C.B);
      for (int z = 0; z < C.B; ++z) {
        if (!std::isfinite(y[z])) throw slnk::Fail{SLNK_ENAN, "non-finite network head"};
        emax[z] = 1.0 + 1.1 * std::exp(double(y[z])) / C.prm.beta;
      }
      C.setup_two_level(&emax);
    }
    C.learned_ready = true;
    C.images_set = true;
  });
}

slnk_status slnk_newton_solve_learned(slnk_ctx* ctx, slnk_unet* u, void* v_out, const slnk_solve_opts* opts,
                                      slnk_solve_report* report) {
  if (!ctx || !u || !v_out) return SLNK_EINVAL;
  if (!ctx->f) {
    ctx->err = "the learned solve needs a mixed-precision (FP32 field) context";
    return SLNK_EINVAL;
  }
  slnk_solve_opts o;
  slnk_default_opts(&o);
  if (opts) o = *opts;
  slnk_status result = SLNK_OK;
  slnk_status st = guarded(ctx, [&] {
    auto& C = *ctx->f;
    if (!C.images_set) throw slnk::Fail{SLNK_EINVAL, "slnk_set_images must come first"};
    if (o.max_newton < 0 || o.max_pcg < 1 || o.max_halvings < 0) throw slnk::Fail{SLNK_EINVAL, "bad options"};
    const double t0 = slnk::now_ms();
    if (C.learned_ready) {
      HIPCHK(hipMemcpyAsync(v_out, C.learned_v, C.B * 2 * C.fine.F * sizeof(float), hipMemcpyDeviceToDevice,
                            C.stream));
    } else {
      learned_start(C, u, static_cast<float*>(v_out));
    }
    HIPCHK(hipStreamSynchronize(C.stream));
    const double t_net = slnk::now_ms() - t0;
    result = C.newton(static_cast<float*>(v_out), o, report);
    if (report)
      for (int z = 0; z < C.B; ++z) {
        report[z].time_total_ms += t_net;
        report[z].time_to_stop_ms += t_net;
      }
  });
  return st != SLNK_OK ? st : result;
}

}  // extern "C"

// ============================================================================================
// Ragged batches: pairs of uneven grid sizes.  Pairs of one size form a bucket, held by one
// batched context (B = pairs of that size); every bucket is driven by its own host thread on its
// own HIP stream, so the launches of different buckets overlap on the GPU while each bucket runs
// its items in lock step.  Per-pair device buffers are staged into the bucket's stacked layout.
// ============================================================================================
struct slnk_batch {
  std::string err;
  int npairs = 0;
  size_t elem = 0;
  hipStream_t user = nullptr;
  struct Bucket {
    int n1 = 0, n2 = 0;
    std::vector<int> pairs;    // pair ids, in item order
    slnk_ctx* ctx = nullptr;
    hipStream_t stream = nullptr;
    char* img = nullptr;       // [2][B][F]: m_R then m_T
    char* vin = nullptr;       // [B][2][F]
    char* vout = nullptr;      // [B][2][F]
    int sl_path = 0, use_graphs = 1;
    size_t F() const { return size_t(n1) * n2; }
  };
  std::vector<Bucket> buckets;
};

namespace {

void batch_release(slnk_batch* b) {
  for (auto& k : b->buckets) {
    if (k.ctx) slnk_destroy(k.ctx);
    if (k.img) (void)hipFree(k.img);
    if (k.vin) (void)hipFree(k.vin);
    if (k.vout) (void)hipFree(k.vout);
    if (k.stream) (void)hipStreamDestroy(k.stream);
    k = slnk_batch::Bucket{};
  }
}

// Statuses a solve reports per item without having failed as a call: success, a failed line
// search or a preconditioner that stayed indefinite (the item keeps its last accepted iterate) and
// the Newton limit.
bool solve_outcome(slnk_status st) {
  return st == SLNK_OK || st == SLNK_ELINESEARCH || st == SLNK_EMAXIT || st == SLNK_ECHEB_DIVERGED;
}

// Run fn(bucket) for every bucket, one host thread each, after the caller's stream has reached
// this point; the first failure (in bucket order) is returned with its message.
template <class Fn>
slnk_status batch_run(slnk_batch* b, Fn&& fn) {
  if (!b) return SLNK_EINVAL;
  hipEvent_t ready = nullptr;
  if (hipEventCreateWithFlags(&ready, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(ready, b->user) != hipSuccess) {
    b->err = "cannot order the batch after the caller's stream";
    if (ready) (void)hipEventDestroy(ready);
    return SLNK_EDEVICE;
  }
  const size_t nb = b->buckets.size();
  std::vector<slnk_status> st(nb, SLNK_OK);
  std::vector<std::string> msg(nb);
  std::vector<std::thread> th;
  th.reserve(nb);
  for (size_t i = 0; i < nb; ++i) {
    th.emplace_back([&, i] {
      auto& k = b->buckets[i];
      try {
        HIPCHK(hipStreamWaitEvent(k.stream, ready, 0));
        st[i] = fn(k);
        if (!solve_outcome(st[i])) msg[i] = slnk_last_error(k.ctx);
        HIPCHK(hipStreamSynchronize(k.stream));
      } catch (const slnk::Fail& e) {
        st[i] = e.st;
        msg[i] = e.msg;
      } catch (const std::exception& e) {
        st[i] = SLNK_EDEVICE;
        msg[i] = e.what();
      }
    });
  }
  for (auto& t : th) t.join();
  (void)hipEventDestroy(ready);
  slnk_status res = SLNK_OK;
  for (size_t i = 0; i < nb; ++i)
    if (!solve_outcome(st[i])) {
      b->err = "bucket " + std::to_string(b->buckets[i].n1) + "x" + std::to_string(b->buckets[i].n2) + ": " + msg[i];
      return st[i];
    } else if (st[i] == SLNK_ELINESEARCH || (st[i] == SLNK_EMAXIT && res == SLNK_OK)) {
      res = st[i];
    }
  return res;
}

// copy per-pair buffers (cnt elements each) into / out of a bucket's stacked buffer
void stage_in(const slnk_batch* b, const slnk_batch::Bucket& k, const void* const* src, char* dst, size_t cnt) {
  const size_t bytes = cnt * b->elem;
  for (size_t z = 0; z < k.pairs.size(); ++z)
    HIPCHK(hipMemcpyAsync(dst + z * bytes, src[k.pairs[z]], bytes, hipMemcpyDeviceToDevice, k.stream));
}

void stage_out(const slnk_batch* b, const slnk_batch::Bucket& k, const char* src, void* const* dst, size_t cnt) {
  const size_t bytes = cnt * b->elem;
  for (size_t z = 0; z < k.pairs.size(); ++z)
    HIPCHK(hipMemcpyAsync(dst[k.pairs[z]], src + z * bytes, bytes, hipMemcpyDeviceToDevice, k.stream));
}

}  // namespace

extern "C" {

slnk_status slnk_batch_create(const slnk_params* base, int npairs, const int* n1, const int* n2, void* hip_stream,
                              slnk_batch** out) {
  if (!base || !n1 || !n2 || !out || npairs < 1) return SLNK_EINVAL;
  *out = nullptr;
  auto b = std::make_unique<slnk_batch>();
  b->npairs = npairs;
  b->elem = base->prec == SLNK_PREC_FP64 ? sizeof(double) : sizeof(float);
  b->user = static_cast<hipStream_t>(hip_stream);
  // buckets by size, largest grids first (they start first and take longest)
  std::map<std::pair<long long, long long>, std::vector<int>> by;
  for (int p = 0; p < npairs; ++p) by[{-(long long)n1[p] * n2[p], (long long)n1[p]}].push_back(p);
  for (auto& kv : by) {
    slnk_batch::Bucket k;
    k.n1 = n1[kv.second[0]];
    k.n2 = n2[kv.second[0]];
    k.pairs = kv.second;
    b->buckets.push_back(std::move(k));
  }
  for (auto& k : b->buckets) {
    slnk_params p = *base;
    p.n1 = k.n1;
    p.n2 = k.n2;
    p.batch = int(k.pairs.size());
    k.sl_path = p.sl_path;
    k.use_graphs = p.use_graphs;
    const size_t F = k.F(), B = k.pairs.size();
    if (hipStreamCreateWithFlags(&k.stream, hipStreamNonBlocking) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&k.img), 2 * B * F * b->elem) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&k.vin), 2 * B * F * b->elem) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&k.vout), 2 * B * F * b->elem) != hipSuccess) {
      batch_release(b.get());
      return SLNK_ENOMEM;
    }
    slnk_status st = slnk_create(&p, k.stream, &k.ctx);
    if (st != SLNK_OK) {
      batch_release(b.get());
      return st;
    }
  }
  *out = b.release();
  return SLNK_OK;
}

void slnk_batch_destroy(slnk_batch* b) {
  if (!b) return;
  batch_release(b);
  delete b;
}

const char* slnk_batch_last_error(const slnk_batch* b) { return b ? b->err.c_str() : "null batch"; }

slnk_status slnk_batch_bucket_info(const slnk_batch* b, int k, int* n1, int* n2, int* count, int* sl_path,
                                   int* use_graphs) {
  if (!b) return SLNK_EINVAL;
  if (k < 0) {
    if (count) *count = int(b->buckets.size());
    return SLNK_OK;
  }
  if (k >= int(b->buckets.size())) return SLNK_EINVAL;
  const auto& q = b->buckets[k];
  if (n1) *n1 = q.n1;
  if (n2) *n2 = q.n2;
  if (count) *count = int(q.pairs.size());
  if (sl_path) *sl_path = q.sl_path;
  if (use_graphs) *use_graphs = q.use_graphs;
  return SLNK_OK;
}

slnk_status slnk_batch_set_images(slnk_batch* b, const void* const* m_R, const void* const* m_T) {
  if (!b || !m_R || !m_T) return SLNK_EINVAL;
  for (int p = 0; p < b->npairs; ++p)
    if (!m_R[p] || !m_T[p]) return SLNK_EINVAL;
  return batch_run(b, [&](slnk_batch::Bucket& k) {
    const size_t F = k.F(), B = k.pairs.size();
    stage_in(b, k, m_R, k.img, F);
    stage_in(b, k, m_T, k.img + B * F * b->elem, F);
    return slnk_set_images(k.ctx, k.img, k.img + B * F * b->elem);
  });
}

slnk_status slnk_batch_gradient(slnk_batch* b, const void* const* v, void* const* g, double* J) {
  if (!b || !v || !g) return SLNK_EINVAL;
  return batch_run(b, [&](slnk_batch::Bucket& k) {
    std::vector<double> Jk(k.pairs.size());
    stage_in(b, k, v, k.vin, 2 * k.F());
    slnk_status st = slnk_gradient(k.ctx, k.vin, k.vout, Jk.data());
    if (st != SLNK_OK) return st;
    stage_out(b, k, k.vout, g, 2 * k.F());
    if (J)
      for (size_t z = 0; z < k.pairs.size(); ++z) J[k.pairs[z]] = Jk[z];
    return SLNK_OK;
  });
}

slnk_status slnk_batch_hessian_matvec(slnk_batch* b, const void* const* vt, void* const* Hvt) {
  if (!b || !vt || !Hvt) return SLNK_EINVAL;
  return batch_run(b, [&](slnk_batch::Bucket& k) {
    stage_in(b, k, vt, k.vin, 2 * k.F());
    slnk_status st = slnk_hessian_matvec(k.ctx, k.vin, k.vout);
    if (st != SLNK_OK) return st;
    stage_out(b, k, k.vout, Hvt, 2 * k.F());
    return SLNK_OK;
  });
}

slnk_status slnk_batch_newton_solve(slnk_batch* b, void* const* v_inout, const slnk_solve_opts* opts,
                                    slnk_solve_report* reports) {
  if (!b || !v_inout) return SLNK_EINVAL;
  return batch_run(b, [&](slnk_batch::Bucket& k) {
    std::vector<slnk_solve_report> rk(k.pairs.size());
    stage_in(b, k, v_inout, k.vin, 2 * k.F());
    slnk_status st = slnk_newton_solve(k.ctx, k.vin, opts, rk.data());
    if (!solve_outcome(st)) return st;
    stage_out(b, k, k.vin, v_inout, 2 * k.F());
    if (reports)
      for (size_t z = 0; z < k.pairs.size(); ++z) reports[k.pairs[z]] = rk[z];
    return st;
  });
}

slnk_status slnk_batch_autotune(slnk_batch* b, const void* const* vt, int reps, double* best_ms) {
  if (!b || !vt || reps < 1) return SLNK_EINVAL;
  // one bucket at a time, so that the candidates are timed without interference
  for (size_t i = 0; i < b->buckets.size(); ++i) {
    auto& k = b->buckets[i];
    slnk_status st = guarded(k.ctx, [&] {
      stage_in(b, k, vt, k.vin, 2 * k.F());
      auto tune = [&](auto& C) {
        using T = std::remove_reference_t<decltype(*C.fine.mT)>;
        if (!C.has_grad) throw slnk::Fail{SLNK_EINVAL, "no linearisation point: call slnk_batch_gradient first"};
        double best = 1e300;
        int bp = 0, bg = 1;
        // the two-kernel step, and the fused step with 16 x 16 or 16 x 32 threads per tile
        for (int path = 1; path < 4; ++path)
          for (int gr = 0; gr < 2; ++gr) {
            C.retune(path, gr);
            const double ms = C.time_operator(reinterpret_cast<const T*>(k.vin), reinterpret_cast<T*>(k.vout), reps);
            if (ms < best) best = ms, bp = path, bg = gr;
          }
        C.retune(bp, bg);
        k.sl_path = bp;
        k.use_graphs = bg;
        if (best_ms) best_ms[i] = best;
      };
      if (k.ctx->f)
        tune(*k.ctx->f);
      else
        tune(*k.ctx->d);
    });
    if (st != SLNK_OK) {
      b->err = slnk_last_error(k.ctx);
      return st;
    }
  }
  return SLNK_OK;
}

}  // extern "C"
