// Allocation-free state transport: slnk_transport_state_noalloc, the variant of
// slnk_transport_state for callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops, harnesses that forbid hipMalloc).  Its working memory (twiddle
// tables, spline coefficients of v and div v, both characteristics' displacements, the adjoint
// factor, ping-pong fields, FFT spectra, reduction partials) lives in one file-scope device array,
// 'scratch', of kScratchBytes; every GPU the library runs on holds its own copy until the process
// ends.  The kernels are the context path's own (spectral trace preparation, Heun trace, SL state
// steps), so the results equal slnk_transport_state's up to the twiddle tables' rounding.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "../../include/slnk.h"
#include "fft_plan.hpp"
#include "kernels.hpp"

namespace slnk {
namespace {

constexpr size_t kScratchBytes = size_t(16) << 20;  // 16 MiB per GPU
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

// device address of 'scratch' on each GPU, taken once per device with that device current (in host
// code the array's name is only a stand-in for the symbol, never a device address)
std::mutex g_scratch_mutex;
unsigned char* g_scratch[kMaxDevices] = {};

hipError_t scratch_ptr(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = static_cast<unsigned char*>(p);
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

// 8-byte words carried in the kernel arguments (no host staging buffer)
constexpr int kPackWords = 256;
struct WordPack {
  unsigned long long w[kPackWords];
};

__global__ void k_put_words(unsigned long long* dst, WordPack pack, int count) {
  for (int i = threadIdx.x; i < count; i += blockDim.x) dst[i] = pack.w[i];
}

// Twiddle table of a length-n plan (2n complex entries) written into device memory dst through
// kernel arguments, kPackWords words per launch.
template <typename T>
hipError_t put_plan(hipStream_t s, int n, FFTPlanDev& pl, cplx<T>* dst) {
  static_assert(sizeof(cplx<T>) % sizeof(unsigned long long) == 0, "whole words per entry");
  constexpr int kWordsPer = int(sizeof(cplx<T>) / sizeof(unsigned long long));
  constexpr int kPer = kPackWords / kWordsPer;  // entries per launch
  cplx<T> buf[kPer];
  int base = 0, filled = 0;
  hipError_t err = hipSuccess;
  auto flush = [&] {
    if (filled == 0 || err != hipSuccess) return;
    WordPack pack;
    std::memcpy(pack.w, buf, filled * sizeof(cplx<T>));
    hipLaunchKernelGGL(k_put_words, dim3(1), dim3(256), 0, s, reinterpret_cast<unsigned long long*>(dst + base),
                       pack, filled * kWordsPer);
    err = hipGetLastError();
    base += filled;
    filled = 0;
  };
  // fft_plan_host emits the entries in index order (0, 1, 2, ...): a window of kPer entries is
  // sent whenever it is full
  bool in_order = true;
  const bool ok = fft_plan_host(n, pl, [&](int i, double re, double im) {
    in_order = in_order && i == base + filled;
    buf[filled++] = {T(re), T(im)};
    if (filled == kPer) flush();
  });
  if (!ok || !in_order) return hipErrorInvalidValue;
  flush();
  pl.tw = dst;
  pl.roots = dst + n;
  return err;
}

// bump allocation inside the scratch array (256-byte aligned regions)
struct Carve {
  unsigned char* base;
  size_t used = 0;
  template <typename U>
  U* take(size_t count) {
    U* p = reinterpret_cast<U*>(base + used);
    used += (count * sizeof(U) + 255) / 256 * 256;
    return p;
  }
};

template <typename T>
size_t scratch_need(int n1, int n2, int B) {
  const size_t F = size_t(n1) * n2;
  const size_t spec = size_t(n1) * spec_stride(n2);
  const size_t tiles = size_t((n1 + 15) / 16) * ((n2 + 15) / 16);
  auto r = [](size_t bytes) { return (bytes + 255) / 256 * 256; };
  size_t need = r(2 * n2 * sizeof(cplx<T>)) + r(2 * n1 * sizeof(cplx<T>)) + r(B * sizeof(int)) +
                r(2 * tiles * B * sizeof(double)) + r(4 * B * sizeof(double));
  // per item: cv, df, da (two fields each); divv, cdiv, gamma, ping, pong, coef, coef2 (one each)
  need += 3 * r(B * 2 * F * sizeof(T)) + 7 * r(B * F * sizeof(T));
  need += r(B * 2 * spec * sizeof(cplx<T>)) + r(B * 4 * spec * sizeof(cplx<T>));
  return need;
}

struct Err {
  slnk_status st;
  char msg[160];
};

#define NA_CHECK(expr)                                                                     \
  do {                                                                                     \
    hipError_t _e = (expr);                                                                \
    if (_e != hipSuccess) {                                                                \
      Err _r{SLNK_EDEVICE, {}};                                                            \
      std::snprintf(_r.msg, sizeof(_r.msg), "%s: %s", #expr, hipGetErrorString(_e));      \
      return _r;                                                                           \
    }                                                                                      \
  } while (0)

template <typename T>
Err run(const slnk_params& p, hipStream_t s, const T* v, const T* m0, T* m1, unsigned char* base) {
  const int n1 = p.n1, n2 = p.n2, nt = p.nt, B = p.batch;
  const size_t F = size_t(n1) * n2;
  Carve c{base};
  SpecGrid<T> sg;
  sg.n1 = n1;
  sg.n2 = n2;
  cplx<T>* tw_row = c.take<cplx<T>>(2 * size_t(n2));
  cplx<T>* tw_col = c.take<cplx<T>>(2 * size_t(n1));
  NA_CHECK(put_plan<T>(s, n2, sg.row, tw_row));
  NA_CHECK(put_plan<T>(s, n1, sg.col, tw_col));
  int* halo_dev = c.take<int>(B);
  const int tiles = ((n1 + 15) / 16) * ((n2 + 15) / 16);
  double* partial = c.take<double>(2 * size_t(tiles) * B);
  double* dres = c.take<double>(4 * size_t(B));
  T* cv = c.take<T>(B * 2 * F);
  T* divv = c.take<T>(B * F);
  T* cdiv = c.take<T>(B * F);
  T* df = c.take<T>(B * 2 * F);
  T* da = c.take<T>(B * 2 * F);
  T* gamma = c.take<T>(B * F);
  T* ping = c.take<T>(B * F);
  T* pong = c.take<T>(B * F);
  T* coef = c.take<T>(B * F);
  T* coef2 = c.take<T>(B * F);
  cplx<T>* S1 = c.take<cplx<T>>(B * 2 * sg.spec());
  cplx<T>* S2 = c.take<cplx<T>>(B * 4 * sg.spec());
  // characteristics (both, as the context's linearisation traces them) and the bound on |d|
  const double ht = 1.0 / nt;
  int nb = 0;
  NA_CHECK(spec_trace_prep<T>(s, sg, B, nullptr, v, cv, divv, cdiv, S1, S2));
  NA_CHECK(sl_trace<T>(s, n1, n2, B, nullptr, ht, v, cv, divv, cdiv, df, da, gamma, partial, &nb));
  NA_CHECK(finish(s, B, nb, 2, 2LL * nb, 2, 2u, partial, dres));
  int halo = 0;
  int halos[64];
  for (int z0 = 0; z0 < B; z0 += 64) {
    const int cnt = B - z0 < 64 ? B - z0 : 64;
    double maxd[4 * 64];
    NA_CHECK(hipMemcpyAsync(maxd, dres + 4 * size_t(z0), 4 * cnt * sizeof(double), hipMemcpyDeviceToHost, s));
    NA_CHECK(hipStreamSynchronize(s));
    for (int z = 0; z < cnt; ++z) {
      if (!std::isfinite(maxd[4 * z + 1])) return Err{SLNK_ENAN, "non-finite velocity or displacement"};
      halos[z] = int(std::ceil(maxd[4 * z + 1]));
      halo = halos[z] > halo ? halos[z] : halo;
    }
    NA_CHECK(set_ints(s, halo_dev + z0, halos, cnt));
  }
  // state equation: m^0 = m0 (copied, so that m1 may alias m0), m^j = I[m^(j-1)](X_f)
  NA_CHECK(masked_copy<T>(s, B, F, m0, (long long)F, ping, (long long)F, nullptr));
  T* cur = ping;
  T* nxt = pong;
  for (int j = 1; j <= nt; ++j) {
    StepArgs<T> a;
    a.n1 = n1;
    a.n2 = n2;
    a.batch = B;
    a.halo = halo;
    a.halo_dev = halo_dev;
    a.coef = coef;
    a.st_coef = (long long)F;
    a.coef2 = coef2;
    a.st_coef2 = (long long)F;
    a.ht = ht;
    a.force_global = p.sl_path == 1;
    a.fused_rows = p.sl_path == 2 ? 16 : p.sl_path == 3 ? 32 : 0;
    a.src = cur;
    a.dst = j == nt ? m1 : nxt;
    a.st_src = a.st_dst = (long long)F;
    a.d1 = df;
    a.st_d = (long long)(2 * F);
    NA_CHECK(sl_step<T>(s, StepKind::State, a, &nb));
    T* t = cur;
    cur = nxt;
    nxt = t;
  }
  return Err{SLNK_OK, {}};
}

}  // namespace
}  // namespace slnk

extern "C" slnk_status slnk_transport_state_noalloc(const slnk_params* params, void* hip_stream, const void* v,
                                                    const void* m0, void* m1, char* msg, size_t msg_len) {
  using namespace slnk;
  auto fail = [&](slnk_status st, const char* text) {
    if (msg && msg_len) std::snprintf(msg, msg_len, "%s", text);
    return st;
  };
  if (msg && msg_len) msg[0] = '\0';
  if (!params || !v || !m0 || !m1) return fail(SLNK_EINVAL, "null argument");
  const slnk_params& p = *params;
  if (!fft_size_ok(p.n1) || !fft_size_ok(p.n2)) return fail(SLNK_EINVAL, "grid sizes must be even products of 2, 3, 5 in [8, 2048]");
  if (p.nt < 1 || p.nt > 512) return fail(SLNK_EINVAL, "nt must be in [1, 512]");
  if (p.batch < 1) return fail(SLNK_EINVAL, "batch must be at least 1");
  if (p.sl_path < 0 || p.sl_path > 3) return fail(SLNK_EINVAL, "sl_path must be 0, 1, 2 or 3");
  if (p.prec != SLNK_PREC_FP64 && p.prec != SLNK_PREC_MIXED) return fail(SLNK_EINVAL, "prec must be FP64 or MIXED");
  const bool f64 = p.prec == SLNK_PREC_FP64;
  const size_t need = f64 ? scratch_need<double>(p.n1, p.n2, p.batch) : scratch_need<float>(p.n1, p.n2, p.batch);
  if (need > kScratchBytes) {
    char text[160];
    std::snprintf(text, sizeof(text), "needs %zu bytes of scratch, more than the %zu this entry point holds per GPU",
                  need, kScratchBytes);
    return fail(SLNK_EINVAL, text);
  }
  int dev = 0, lim = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return fail(SLNK_EDEVICE, "cannot query the current device");
  if ((f64 ? spec_lds_bytes<double>(p.n1, p.n2) : spec_lds_bytes<float>(p.n1, p.n2)) > size_t(lim))
    return fail(SLNK_EINVAL, "grid too large for the LDS-resident FFTs of this precision");
  unsigned char* base = nullptr;
  hipError_t e = scratch_ptr(dev, &base);
  if (e != hipSuccess) return fail(SLNK_EDEVICE, hipGetErrorString(e));
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  Err r = f64 ? run<double>(p, s, static_cast<const double*>(v), static_cast<const double*>(m0),
                            static_cast<double*>(m1), base)
              : run<float>(p, s, static_cast<const float*>(v), static_cast<const float*>(m0), static_cast<float*>(m1),
                           base);
  if (r.st != SLNK_OK) return fail(r.st, r.msg);
  return SLNK_OK;
}
