// Three-dimensional kernels on gfx950: FFT passes and spectral symbols (section 3.2), the
// semi-Lagrangian step with the tricubic B-spline (section 3.3.2), the Heun trace, and the
// elementwise and FP64 reduction kernels of the reduced gradient and Gauss--Newton matvec.
//
// FFT: every pass transforms lines of one axis in LDS.  The passes along x1 and x2 stage a tile of
// CL neighbouring lines (consecutive in memory along x3) so that each global access moves CL
// contiguous complex values; the pass along x3 (contiguous rows) stages RL whole rows.  Inside
// LDS each line runs an iterative radix-2 Cooley--Tukey transform from bit-reversed order, with
// twiddles from a table computed in FP64 on the host.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <map>
#include <mutex>

#include "d3.hpp"

namespace slnk {
namespace d3 {
namespace {

constexpr int kThreads = 256;

template <typename T>
struct Tile;
template <>
struct Tile<float> {
  static constexpr int CL = 16;  // lines per strided tile: 128 bytes of each row
  static constexpr int RL = 8;   // rows per contiguous tile
};
template <>
struct Tile<double> {
  static constexpr int CL = 8;
  static constexpr int RL = 4;
};

__device__ __forceinline__ int bitrev(int k, int logn) { return int(__brev(unsigned(k)) >> (32 - logn)); }

__device__ __forceinline__ int ilog2_dev(int n) { return 31 - __clz(n); }

inline int ilog2(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

// Raise a kernel's dynamic LDS limit (once per kernel and size) for launches above the default.
// The sizes already allowed are kept per kernel (kernels of one signature share a function type,
// so a static per type would not tell them apart).
std::mutex g_lds_mutex;
std::map<const void*, size_t> g_lds_allowed;
template <typename K>
hipError_t ensure_lds(K kernel, size_t bytes) {
  if (bytes <= 64 * 1024) return hipSuccess;
  const void* key = reinterpret_cast<const void*>(kernel);
  std::lock_guard<std::mutex> lock(g_lds_mutex);
  size_t& allowed = g_lds_allowed[key];
  if (bytes <= allowed) return hipSuccess;
  const hipError_t e = hipFuncSetAttribute(key, hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
  if (e == hipSuccess) allowed = bytes;
  return e;
}

// In-place transforms of lines line0 .. line0 + NL - 1 of length n held in LDS as
// s[k * STRIDE + line], input in bit-reversed order, output in natural order.
// sign -1: exp(-2 pi i jk/n), +1: exp(+...).
// Radix-2 stages st (blocks of 2h, h = 2^st) are taken two at a time: a thread owns the four
// elements a, a + h, a + 2h, a + 3h of a block of 4h and applies both stages' butterflies to them
// in registers (the same operations in the same order as two separate radix-2 stages, so the
// results are identical), which halves the barriers and the LDS traffic; an odd last stage runs
// alone.
template <typename T, int STRIDE, int NL = STRIDE>
__device__ void lds_fft(cplx<T>* s, int n, int logn, int sign, const cplx<T>* __restrict__ tw, int line0 = 0) {
  constexpr int CL = STRIDE;
  auto twiddle = [&](int m) {
    cplx<T> w = tw[m];
    if (sign > 0) w.y = -w.y;
    return w;
  };
  int st = 0;
  for (; st + 1 < logn; st += 2) {
    const int half = 1 << st;
    const int ng = (n / 4) * NL;
    for (int g = threadIdx.x; g < ng; g += blockDim.x) {
      const int c = line0 + g % NL, q = g / NL;
      const int j = q & (half - 1);
      const int ia = ((q >> st) << (st + 2)) + j;
      const cplx<T> w1 = twiddle(j << (logn - 1 - st));
      const cplx<T> w2a = twiddle(j << (logn - 2 - st));
      const cplx<T> w2b = twiddle((j + half) << (logn - 2 - st));
      const cplx<T> xa = s[ia * CL + c], xb = s[(ia + half) * CL + c];
      const cplx<T> xc = s[(ia + 2 * half) * CL + c], xd = s[(ia + 3 * half) * CL + c];
      // stage st: (a, b) and (c, d), twiddle of offset j
      const cplx<T> tb = cmul(w1, xb), td = cmul(w1, xd);
      const cplx<T> a1 = cadd(xa, tb), b1 = csub(xa, tb), c1 = cadd(xc, td), d1 = csub(xc, td);
      // stage st + 1: (a, c) at offset j, (b, d) at offset j + h
      const cplx<T> tc = cmul(w2a, c1), tdd = cmul(w2b, d1);
      s[ia * CL + c] = cadd(a1, tc);
      s[(ia + 2 * half) * CL + c] = csub(a1, tc);
      s[(ia + half) * CL + c] = cadd(b1, tdd);
      s[(ia + 3 * half) * CL + c] = csub(b1, tdd);
    }
    __syncthreads();
  }
  if (st < logn) {  // the last stage alone
    const int half = 1 << st;
    const int tshift = logn - 1 - st;
    const int nb = (n / 2) * NL;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
      const int c = line0 + b % NL, q = b / NL;
      const int j = q & (half - 1);
      const int i0 = ((q >> st) << (st + 1)) + j;
      const int i1 = i0 + half;
      const cplx<T> w = twiddle(j << tshift);
      const cplx<T> x0 = s[i0 * CL + c];
      const cplx<T> x1 = cmul(w, s[i1 * CL + c]);
      s[i0 * CL + c] = cadd(x0, x1);
      s[i1 * CL + c] = csub(x0, x1);
    }
    __syncthreads();
  }
}

// Transform along a strided axis: line (o, c) holds the elements base + k stride_k, base =
// field z + o stride_o + c, k < n; c < inner runs over consecutive addresses.  Block: lines
// c0 .. c0 + CL - 1 of one o (grid.y) and one field (grid.z).
template <typename T>
__global__ void __launch_bounds__(kThreads) k_fft_strided(cplx<T>* data, size_t fstride, int n, int logn, int inner,
                                                          long long stride_k, long long stride_o, int sign,
                                                          const cplx<T>* __restrict__ tw) {
  constexpr int CL = Tile<T>::CL;
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* s = reinterpret_cast<cplx<T>*>(smem_raw);
  const int c0 = blockIdx.x * CL;
  cplx<T>* base = data + blockIdx.z * fstride + size_t(blockIdx.y) * stride_o + c0;
  const int ncl = min(CL, inner - c0);
  for (int e = threadIdx.x; e < n * CL; e += blockDim.x) {
    const int c = e % CL, k = e / CL;
    cplx<T> v = {T(0), T(0)};
    if (c < ncl) v = base[k * stride_k + c];
    s[bitrev(k, logn) * CL + c] = v;
  }
  __syncthreads();
  lds_fft<T, CL>(s, n, logn, sign, tw);
  for (int e = threadIdx.x; e < n * CL; e += blockDim.x) {
    const int c = e % CL, k = e / CL;
    if (c < ncl) base[k * stride_k + c] = s[k * CL + c];
  }
}

// Real rows of length n (contiguous, element type TF) -> their first n/2 + 1 Fourier coefficients.
template <typename T, typename TF = T>
__global__ void __launch_bounds__(kThreads) k_fft_r2c_rows(const TF* __restrict__ in, size_t fin, cplx<T>* out,
                                                           size_t fout, int rows, int n, int logn,
                                                           const cplx<T>* __restrict__ tw) {
  constexpr int RL = Tile<T>::RL;
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* s = reinterpret_cast<cplx<T>*>(smem_raw);
  const int r0 = blockIdx.x * RL;
  const TF* src = in + blockIdx.z * fin;
  cplx<T>* dst = out + blockIdx.z * fout;
  const int nh = n / 2 + 1;
  for (int e = threadIdx.x; e < n * RL; e += blockDim.x) {
    const int r = e / n, k = e - r * n;
    const T v = r0 + r < rows ? T(src[size_t(r0 + r) * n + k]) : T(0);
    s[bitrev(k, logn) * RL + r] = cplx<T>{v, T(0)};
  }
  __syncthreads();
  lds_fft<T, RL>(s, n, logn, -1, tw);
  for (int e = threadIdx.x; e < nh * RL; e += blockDim.x) {
    const int r = e / nh, k = e - r * nh;
    if (r0 + r < rows) dst[size_t(r0 + r) * nh + k] = s[k * RL + r];
  }
}

// Half spectra of rows -> real rows (the full row spectrum is the Hermitian extension), times scale,
// stored as TF.
template <typename T, typename TF = T>
__global__ void __launch_bounds__(kThreads) k_fft_c2r_rows(const cplx<T>* __restrict__ in, size_t fin, TF* out,
                                                           size_t fout, int rows, int n, int logn, T scale,
                                                           const cplx<T>* __restrict__ tw) {
  constexpr int RL = Tile<T>::RL;
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* s = reinterpret_cast<cplx<T>*>(smem_raw);
  const int r0 = blockIdx.x * RL;
  const cplx<T>* src = in + blockIdx.z * fin;
  TF* dst = out + blockIdx.z * fout;
  const int h = n / 2, nh = h + 1;
  for (int e = threadIdx.x; e < n * RL; e += blockDim.x) {
    const int r = e / n, k = e - r * n;
    cplx<T> v = {T(0), T(0)};
    if (r0 + r < rows) {
      const size_t row = size_t(r0 + r) * nh;
      v = k <= h ? src[row + k] : cconj(src[row + (n - k)]);
    }
    s[bitrev(k, logn) * RL + r] = v;
  }
  __syncthreads();
  lds_fft<T, RL>(s, n, logn, +1, tw);
  for (int e = threadIdx.x; e < n * RL; e += blockDim.x) {
    const int r = e / n, k = e - r * n;
    if (r0 + r < rows) dst[size_t(r0 + r) * n + k] = TF(s[k * RL + r].x * scale);
  }
}

template <typename T>
hipError_t launch_strided(hipStream_t s, int nf, cplx<T>* S, size_t Fh, int n, int inner, int outer,
                          long long stride_k, long long stride_o, int sign, const cplx<T>* tw) {
  constexpr int CL = Tile<T>::CL;
  const dim3 grid((inner + CL - 1) / CL, outer, nf);
  const size_t lds = size_t(n) * CL * sizeof(cplx<T>);
  hipLaunchKernelGGL(k_fft_strided<T>, grid, dim3(kThreads), lds, s, S, Fh, n, ilog2(n), inner, stride_k, stride_o,
                     sign, tw);
  return hipGetLastError();
}

// ---- B-spline prefilter -------------------------------------------------------------------
// Truncation error of the filter relative to max |f|: 2 sqrt(3) |z|^(K+1) / (1 - |z|), 4.7e-8 for
// K = 13 (below FP32 rounding) and 1.2e-16 for K = 28 (FP64).
template <typename T>
struct Fir;
template <>
struct Fir<float> {
  static constexpr int K = 13;
  static constexpr int CL = 16;  // lines per strided tile
  static constexpr int RL = 8;   // rows per contiguous tile
};
template <>
struct Fir<double> {
  static constexpr int K = 28;
  static constexpr int CL = 8;
  static constexpr int RL = 4;
};

// periodic index of k - K for 0 <= k < n + 2K: one addition or subtraction unless n < K
template <int K>
__device__ __forceinline__ int fir_src(int k, int n) {
  int x = k - K;
  x = x < 0 ? x + n : (x >= n ? x - n : x);
  return (x < 0 || x >= n) ? wrap_index(x, n) : x;
}
template <typename T>
struct Taps {
  T t[Fir<T>::K + 1];  // sqrt(3) z^t, t = 0..K
};

// Lines are staged with K wrapped values on each side: s[(k + K) * L + line] holds element
// (k mod n) for -K <= k < n + K, so the filter needs no index arithmetic.  A thread produces R
// consecutive outputs of one line from a register window of R + 2K staged values.
template <typename T, int L, int R>
__device__ __forceinline__ void fir_window(const T* s, int k0, int line, const Taps<T>& tp, T* o) {
  constexpr int K = Fir<T>::K;
  T x[R + 2 * K];
#pragma unroll
  for (int i = 0; i < R + 2 * K; ++i) x[i] = s[(k0 + i) * L + line];
  filter_window_rec<T, R, K>(x, o, [&](int t) { return tp.t[t]; });
}

constexpr int kFirR = 4;  // outputs per thread (every n here is a multiple of 8)

// filter along a strided axis (lines as in k_fft_strided, real values)
template <typename T>
__global__ void __launch_bounds__(kThreads) k_fir_strided(const T* in, T* out, size_t fstride, int n, int inner,
                                                          long long stride_k, long long stride_o, Taps<T> tp) {
  constexpr int CL = Fir<T>::CL, K = Fir<T>::K;
  extern __shared__ unsigned char smem_raw[];
  T* s = reinterpret_cast<T*>(smem_raw);
  const int c0 = blockIdx.x * CL;
  const size_t off = blockIdx.z * fstride + size_t(blockIdx.y) * stride_o + c0;
  const int ncl = min(CL, inner - c0);
  const int P = n + 2 * K;
  for (int e = threadIdx.x; e < P * CL; e += blockDim.x) {
    const int c = e % CL, k = e / CL;
    const int src = fir_src<K>(k, n);
    s[k * CL + c] = c < ncl ? in[off + src * stride_k + c] : T(0);
  }
  __syncthreads();
  const int segs = n / kFirR;
  for (int e = threadIdx.x; e < segs * CL; e += blockDim.x) {
    const int c = e % CL, q = e / CL;
    T o[kFirR];
    fir_window<T, CL, kFirR>(s, q * kFirR, c, tp, o);
    if (c < ncl) {
#pragma unroll
      for (int r = 0; r < kFirR; ++r) out[off + (q * kFirR + r) * stride_k + c] = o[r];
    }
  }
}

// filter along the contiguous axis: RL whole rows per block, staged transposed (s[(k + K) * RL + r])
template <typename T>
__global__ void __launch_bounds__(kThreads) k_fir_rows(const T* in, T* out, size_t fstride, int rows, int n,
                                                       Taps<T> tp) {
  constexpr int RL = Fir<T>::RL, K = Fir<T>::K;
  extern __shared__ unsigned char smem_raw[];
  T* s = reinterpret_cast<T*>(smem_raw);
  const int r0 = blockIdx.x * RL;
  const size_t off = blockIdx.z * fstride;
  const int P = n + 2 * K;
  for (int e = threadIdx.x; e < P * RL; e += blockDim.x) {
    const int r = e / P, k = e - r * P;
    s[k * RL + r] = r0 + r < rows ? in[off + size_t(r0 + r) * n + fir_src<K>(k, n)] : T(0);
  }
  __syncthreads();
  const int segs = n / kFirR;
  for (int e = threadIdx.x; e < segs * RL; e += blockDim.x) {
    const int r = e % RL, q = e / RL;
    T o[kFirR];
    fir_window<T, RL, kFirR>(s, q * kFirR, r, tp, o);
    if (r0 + r < rows) {
#pragma unroll
      for (int j = 0; j < kFirR; ++j) out[off + size_t(r0 + r) * n + q * kFirR + j] = o[j];
    }
  }
}

// Filter along x3 and then x2 in one pass.  A block takes a band of BR rows (x2) of one x1 plane:
// it stages rows r0 - K .. r0 + BR + K - 1 (periodic in x2), each with K wrapped values on either
// side (periodic in x3), filters every staged row along x3 into a second buffer, then every
// column of the band along x2.  One read and one write of the field instead of two of each; the
// 2K halo rows are read twice (from L2).  blockDim = (64, 8).
template <typename T>
struct FirPlane {
  static constexpr int kThreadsX = 64, kThreadsY = 8;
  static int band(int n2) { return std::min(n2, 32); }
  static size_t lds_bytes(int n2, int n3) {
    constexpr int K = Fir<T>::K;
    const int NR = band(n2) + 2 * K, W = n3 + 2 * K;
    return size_t(NR) * ((W | 1) + (n3 | 1)) * sizeof(T);
  }
};

template <typename T>
__global__ void __launch_bounds__(512) k_fir_plane(const T* in, T* out, size_t fstride, int n2, int n3, int BR,
                                                   Taps<T> tp) {
  constexpr int K = Fir<T>::K, R = kFirR;
  constexpr int NT = FirPlane<T>::kThreadsX * FirPlane<T>::kThreadsY;
  extern __shared__ unsigned char smem_raw[];
  // odd row strides: the rows of consecutive threads fall on different banks
  const int NR = BR + 2 * K, W = n3 + 2 * K, SA = W | 1, SB = n3 | 1;
  T* A = reinterpret_cast<T*>(smem_raw);  // [NR][SA] staged
  T* Bf = A + size_t(NR) * SA;            // [NR][SB] filtered along x3
  const int r0 = blockIdx.x * BR;
  const size_t plane = blockIdx.z * fstride + size_t(blockIdx.y) * n2 * n3;
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * FirPlane<T>::kThreadsX + tx;
  for (int r = ty; r < NR; r += FirPlane<T>::kThreadsY) {
    const T* row = in + plane + size_t(wrap_near(r0 - K + r, n2)) * n3;
    for (int k = tx; k < W; k += FirPlane<T>::kThreadsX) A[r * SA + k] = row[fir_src<K>(k, n3)];
  }
  __syncthreads();
  // along x3: task t = q NR + r (staged row r, segment q), consecutive threads on consecutive
  // rows; (q, r) stepped by NT without a division per task
  const int segs3 = n3 / R;
  const int dq3 = NT / NR, dr3 = NT - dq3 * NR;
  int q = tid / NR, r = tid - q * NR;
  for (int t = tid; t < NR * segs3; t += NT) {
    T x[R + 2 * K], o[R];
#pragma unroll
    for (int i = 0; i < R + 2 * K; ++i) x[i] = A[r * SA + q * R + i];
    filter_window_rec<T, R, K>(x, o, [&](int j) { return tp.t[j]; });
#pragma unroll
    for (int j = 0; j < R; ++j) Bf[r * SB + q * R + j] = o[j];
    q += dq3;
    r += dr3;
    if (r >= NR) r -= NR, ++q;
  }
  __syncthreads();
  // along x2: task t = q n3 + c (column c, segment q), consecutive threads on consecutive columns
  const int segs2 = BR / R;
  const int dq2 = NT / n3, dc2 = NT - dq2 * n3;
  q = tid / n3;
  int c = tid - q * n3;
  for (int t = tid; t < n3 * segs2; t += NT) {
    T x[R + 2 * K], o[R];
#pragma unroll
    for (int i = 0; i < R + 2 * K; ++i) x[i] = Bf[(q * R + i) * SB + c];
    filter_window_rec<T, R, K>(x, o, [&](int j) { return tp.t[j]; });
#pragma unroll
    for (int j = 0; j < R; ++j) out[plane + size_t(r0 + q * R + j) * n3 + c] = o[j];
    q += dq2;
    c += dc2;
    if (c >= n3) c -= n3, ++q;
  }
}

template <typename T>
Taps<T> make_taps() {
  Taps<T> tp;
  const double z = std::sqrt(3.0) - 2.0;
  for (int t = 0; t <= Fir<T>::K; ++t) tp.t[t] = T(std::sqrt(3.0) * std::pow(z, t));
  return tp;
}

// ---- spectral symbols ----------------------------------------------------------------------

struct Wave {
  int k1, k2, k3;      // signed wavenumbers (the x3 index of a half spectrum is k3 >= 0)
  int o1, o2, o3;      // the same with the Nyquist components zeroed (odd-order symbols)
};

__device__ __forceinline__ Wave wave_of(size_t idx, const Dims& d) {
  const int nh = d.nh();
  const int i3 = int(idx % nh);
  const size_t t = idx / nh;
  const int i2 = int(t % d.n2), i1 = int(t / d.n2);
  Wave w;
  w.k1 = signed_wavenumber(i1, d.n1);
  w.k2 = signed_wavenumber(i2, d.n2);
  w.k3 = i3;
  w.o1 = i1 == d.n1 / 2 ? 0 : w.k1;
  w.o2 = i2 == d.n2 / 2 ? 0 : w.k2;
  w.o3 = i3 == d.n3 / 2 ? 0 : w.k3;
  return w;
}

__device__ __forceinline__ double symbol_value(const Wave& w, const SymArgs& a) {
  if (a.kind == Sym::One) return 1.0;
  const double kk = double(w.k1) * w.k1 + double(w.k2) * w.k2 + double(w.k3) * w.k3;
  double av = 1.0;
  for (int r = 0; r < a.reg; ++r) av *= kk;
  if (a.kind == Sym::Reg) return a.beta * av;
  const double ap = a.beta * (av == 0.0 ? 1.0 : av);
  return a.kind == Sym::RegInv ? 1.0 / ap : 1.0 / sqrt(ap);
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_symbol(Dims d, int nf, SymArgs a, cplx<T>* S) {
  const size_t Fh = d.Fh();
  const size_t idx = size_t(blockIdx.x) * kThreads + threadIdx.x;
  if (idx >= Fh) return;
  const Wave w = wave_of(idx, d);
  const T sv = T(symbol_value(w, a));
  if (nf == 3 && a.proj) {
    cplx<T> b[3] = {S[idx], S[Fh + idx], S[2 * Fh + idx]};
    const T kk = T(double(w.o1) * w.o1 + double(w.o2) * w.o2 + double(w.o3) * w.o3);
    if (kk > T(0)) {
      const T o[3] = {T(w.o1), T(w.o2), T(w.o3)};
      cplx<T> kb = cadd(cadd(cscale(b[0], o[0]), cscale(b[1], o[1])), cscale(b[2], o[2]));
      kb = cscale(kb, T(1) / kk);
#pragma unroll
      for (int c = 0; c < 3; ++c) b[c] = csub(b[c], cscale(kb, o[c]));
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) S[c * Fh + idx] = cscale(b[c], sv);
    return;
  }
  for (int c = 0; c < nf; ++c) S[c * Fh + idx] = cscale(S[c * Fh + idx], sv);
}

// coarse half-spectrum index -> fine one; keep: the mode is one the coarse grid keeps
__device__ __forceinline__ size_t coarse_to_fine(size_t idx, const Dims& f, const Dims& c, bool& keep) {
  const int nhc = c.nh(), nhf = f.nh();
  const int i3 = int(idx % nhc);
  const size_t t = idx / nhc;
  const int i2 = int(t % c.n2), i1 = int(t / c.n2);
  const int k1 = signed_wavenumber(i1, c.n1), k2 = signed_wavenumber(i2, c.n2);
  keep = i1 != c.n1 / 2 && i2 != c.n2 / 2 && i3 < c.n3 / 2;
  const int f1 = k1 < 0 ? k1 + f.n1 : k1, f2 = k2 < 0 ? k2 + f.n2 : k2;
  return (size_t(f1) * f.n2 + f2) * nhf + i3;
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_restrict(Dims f, Dims c, int nf, const cplx<T>* __restrict__ Sf,
                                                       cplx<T>* __restrict__ Sc) {
  const size_t Fhc = c.Fh(), Fhf = f.Fh();
  const size_t idx = size_t(blockIdx.x) * kThreads + threadIdx.x;
  if (idx >= Fhc) return;
  bool keep;
  const size_t fi = coarse_to_fine(idx, f, c, keep);
  const T scale = T(double(c.F()) / double(f.F()));
  for (int k = 0; k < nf; ++k) Sc[k * Fhc + idx] = keep ? cscale(Sf[k * Fhf + fi], scale) : cplx<T>{T(0), T(0)};
}

// over the coarse half spectrum: every fine mode of the coarse set is written from its coarse
// mode (the others keep the fine values)
template <typename T>
__global__ void __launch_bounds__(kThreads) k_prolong_combine(Dims f, Dims c, int nf, cplx<T>* __restrict__ Sf,
                                                              const cplx<T>* __restrict__ Sc) {
  const size_t Fhc = c.Fh(), Fhf = f.Fh();
  const size_t idx = size_t(blockIdx.x) * kThreads + threadIdx.x;
  if (idx >= Fhc) return;
  bool keep;
  const size_t fi = coarse_to_fine(idx, f, c, keep);
  if (!keep) return;
  const T scale = T(double(f.F()) / double(c.F()));
  for (int k = 0; k < nf; ++k) Sf[k * Fhf + fi] = cscale(Sc[k * Fhc + idx], scale);
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_grad(Dims d, const cplx<T>* __restrict__ U, cplx<T>* out) {
  const size_t Fh = d.Fh();
  const size_t idx = size_t(blockIdx.x) * kThreads + threadIdx.x;
  if (idx >= Fh) return;
  const Wave w = wave_of(idx, d);
  const cplx<T> u = U[idx];
  const cplx<T> iu = cmul_i(u);
  out[idx] = cscale(iu, T(w.o1));
  out[Fh + idx] = cscale(iu, T(w.o2));
  out[2 * Fh + idx] = cscale(iu, T(w.o3));
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_div(Dims d, cplx<T>* S) {
  const size_t Fh = d.Fh();
  const size_t idx = size_t(blockIdx.x) * kThreads + threadIdx.x;
  if (idx >= Fh) return;
  const Wave w = wave_of(idx, d);
  const cplx<T> s = cadd(cadd(cscale(S[idx], T(w.o1)), cscale(S[Fh + idx], T(w.o2))), cscale(S[2 * Fh + idx], T(w.o3)));
  S[idx] = cmul_i(s);
}

// ---- transform along x1 fused with the spectral operator ---------------------------------------
// Every line along x1 of a half spectrum holds all k1 of one (k2, k3): the last forward pass, the
// operator (pointwise in k) and the first inverse pass run on it in LDS.  NB buffers of n x CL
// lines: the NI input fields' lines are transformed, the operator leaves its NO output fields in
// bit-reversed order (each thread handles the pair k, bitrev(k), so the reordering is in place),
// and the outputs are transformed back.  OP 0: symbol (with the Leray projection for three fields);
// 1: gradient (one field in, three out, in buffers 1..3); 2: divergence (three in, one out).
template <typename T, int OP, int NI>
struct X1Op {
  static constexpr int NO = OP == 1 ? 3 : (OP == 2 ? 1 : NI);
  static constexpr int NB = OP == 1 ? 4 : NI;
  static constexpr int OUT0 = OP == 1 ? 1 : 0;  // first output buffer
};

template <typename T, int OP, int NI>
__global__ void __launch_bounds__(kThreads) k_x1_op(Dims d, const cplx<T>* Sin, cplx<T>* Sout, SymArgs a,
                                                    const cplx<T>* __restrict__ tw) {
  constexpr int CL = Tile<T>::CL;
  using X = X1Op<T, OP, NI>;
  constexpr int L = X::NB * CL;  // lines in LDS: buffer b, line c at column b CL + c
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* s = reinterpret_cast<cplx<T>*>(smem_raw);
  const int n = d.n1, logn = ilog2_dev(n);
  const int nh = d.nh();
  const int inner = d.n2 * nh;
  const long long stride_k = inner;
  const size_t Fh = d.Fh();
  const int c0 = blockIdx.x * CL;
  const int ncl = min(CL, inner - c0);
  for (int e = threadIdx.x; e < n * NI * CL; e += blockDim.x) {
    const int c = e % CL, b = (e / CL) % NI, k = e / (CL * NI);
    cplx<T> v = {T(0), T(0)};
    if (c < ncl) v = Sin[b * Fh + size_t(k) * stride_k + c0 + c];
    s[bitrev(k, logn) * L + b * CL + c] = v;
  }
  __syncthreads();
  lds_fft<T, L, NI * CL>(s, n, logn, -1, tw);  // the input buffers
  // operator at natural k, stored at bitrev(k): pairs (k, kb) with k <= kb
  for (int e = threadIdx.x; e < n * CL; e += blockDim.x) {
    const int c = e % CL, k = e / CL;
    const int kb = bitrev(k, logn);
    if (k > kb) continue;
    const int idx2 = min(c0 + c, inner - 1);
    const int i2 = idx2 / nh, i3 = idx2 - i2 * nh;
    cplx<T> res[2][3];
    const int ks[2] = {k, kb};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i1 = ks[h];
      Wave w;
      w.k1 = signed_wavenumber(i1, d.n1);
      w.k2 = signed_wavenumber(i2, d.n2);
      w.k3 = i3;
      w.o1 = i1 == d.n1 / 2 ? 0 : w.k1;
      w.o2 = i2 == d.n2 / 2 ? 0 : w.k2;
      w.o3 = i3 == d.n3 / 2 ? 0 : w.k3;
      cplx<T> x[3];
#pragma unroll
      for (int b = 0; b < NI; ++b) x[b] = s[i1 * L + b * CL + c];
      if constexpr (OP == 0) {
        const T sv = T(symbol_value(w, a));
        if constexpr (NI == 3) {
          if (a.proj) {
            const T kk = T(double(w.o1) * w.o1 + double(w.o2) * w.o2 + double(w.o3) * w.o3);
            if (kk > T(0)) {
              const T o[3] = {T(w.o1), T(w.o2), T(w.o3)};
              cplx<T> kb3 = cadd(cadd(cscale(x[0], o[0]), cscale(x[1], o[1])), cscale(x[2], o[2]));
              kb3 = cscale(kb3, T(1) / kk);
#pragma unroll
              for (int q = 0; q < 3; ++q) x[q] = csub(x[q], cscale(kb3, o[q]));
            }
          }
        }
#pragma unroll
        for (int b = 0; b < NI; ++b) res[h][b] = cscale(x[b], sv);
      } else if constexpr (OP == 1) {
        const cplx<T> iu = cmul_i(x[0]);
        res[h][0] = cscale(iu, T(w.o1));
        res[h][1] = cscale(iu, T(w.o2));
        res[h][2] = cscale(iu, T(w.o3));
      } else {
        res[h][0] = cmul_i(cadd(cadd(cscale(x[0], T(w.o1)), cscale(x[1], T(w.o2))), cscale(x[2], T(w.o3))));
      }
    }
#pragma unroll
    for (int b = 0; b < X::NO; ++b) {
      s[kb * L + (X::OUT0 + b) * CL + c] = res[0][b];
      s[k * L + (X::OUT0 + b) * CL + c] = res[1][b];
    }
  }
  __syncthreads();
  lds_fft<T, L, X::NO * CL>(s, n, logn, +1, tw, X::OUT0 * CL);  // the output buffers
  for (int e = threadIdx.x; e < n * X::NO * CL; e += blockDim.x) {
    const int c = e % CL, b = (e / CL) % X::NO, k = e / (CL * X::NO);
    if (c < ncl) Sout[b * Fh + size_t(k) * stride_k + c0 + c] = s[k * L + (X::OUT0 + b) * CL + c];
  }
}

// ---- semi-Lagrangian transport ---------------------------------------------------------------

template <typename T>
__device__ __forceinline__ void bspline_w(T t, T* w) {
  const T t2 = t * t, t3 = t2 * t;
  const T s = T(1) - t;
  const T sixth = T(1.0 / 6.0);
  w[0] = s * s * s * sixth;
  w[1] = (T(3) * t3 - T(6) * t2 + T(4)) * sixth;
  w[2] = (T(-3) * t3 + T(3) * t2 + T(3) * t + T(1)) * sixth;
  w[3] = t3 * sixth;
}

// Periodic tricubic spline with coefficients c at (s1, s2, s3) (cells): the 4 x 4 x 4 stencil
// from floor(s_i) - 1.  Along x3 a stencil row is four consecutive values away from the end.
template <typename T>
__device__ T interp3(const T* __restrict__ c, const Dims& d, T s1, T s2, T s3) {
  const T f1 = floor(s1), f2 = floor(s2), f3 = floor(s3);
  T w1[4], w2[4], w3[4];
  bspline_w(s1 - f1, w1);
  bspline_w(s2 - f2, w2);
  bspline_w(s3 - f3, w3);
  const int b1 = wrap_near(int(f1) - 1, d.n1), b2 = wrap_near(int(f2) - 1, d.n2);
  const int b3 = wrap_near(int(f3) - 1, d.n3);
  int p[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) p[k] = b3 + k >= d.n3 ? b3 + k - d.n3 : b3 + k;
  const bool straight = b3 + 3 < d.n3;
  T acc = T(0);
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int r = b1 + a >= d.n1 ? b1 + a - d.n1 : b1 + a;
    T pa = T(0);
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int q = b2 + b >= d.n2 ? b2 + b - d.n2 : b2 + b;
      const T* row = c + (size_t(r) * d.n2 + q) * d.n3;
      T v[4];
      if (straight) {  // one 4-wide load (unaligned addresses are legal for global loads on gfx950)
        typedef T V4 __attribute__((ext_vector_type(4), aligned(sizeof(T))));
        const V4 q4 = *reinterpret_cast<const V4*>(row + b3);
        v[0] = q4.x;
        v[1] = q4.y;
        v[2] = q4.z;
        v[3] = q4.w;
      } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = row[p[k]];
      }
      pa += w2[b] * (w3[0] * v[0] + w3[1] * v[1] + w3[2] * v[2] + w3[3] * v[3]);
    }
    acc += w1[a] * pa;
  }
  return acc;
}

// the update of a step at node i from the interpolated value u
template <typename T>
__device__ __forceinline__ void step_update(const StepArgs<T>& a, size_t i, size_t F, T u) {
  switch (a.kind) {
    case Kind::State:
      a.dst[i] = u;
      break;
    case Kind::Adjoint:
    case Kind::IncAdjoint: {
      T l = a.gamma[i] * u;
      if (a.add) l += a.add[i];
      a.dst[i] = l;
      const T wl = T(a.w) * l;
#pragma unroll
      for (int c = 0; c < 3; ++c) a.acc[c * F + i] += wl * a.gm[c * F + i];
      break;
    }
    case Kind::IncState: {
      const T f = -(a.vt[i] * a.gm[i] + a.vt[F + i] * a.gm[F + i] + a.vt[2 * F + i] * a.gm[2 * F + i]);
      const T mt = u + T(0.5 * a.ht) * f;
      if (a.mt) a.mt[i] = mt;
      if (!a.last) {
        a.dst[i] = u + T(a.ht) * f;
      } else {
        const T lt = -mt;
        a.dst[i] = lt;
        const T wl = T(a.w) * lt;
#pragma unroll
        for (int c = 0; c < 3; ++c) a.acc[c * F + i] = wl * a.gm[c * F + i];
      }
      break;
    }
  }
}

// step with the stencil read from the global coefficient field (any displacement)
template <typename T>
__global__ void __launch_bounds__(kThreads) k_sl_step(StepArgs<T> a) {
  const Dims d = a.d;
  const size_t F = d.F();
  const size_t i = size_t(blockIdx.x) * kThreads + threadIdx.x;
  if (i >= F) return;
  const int i3 = int(i % d.n3);
  const size_t t = i / d.n3;
  const int i2 = int(t % d.n2), i1 = int(t / d.n2);
  const T u = interp3(a.coef, d, T(i1) + a.disp[i], T(i2) + a.disp[F + i], T(i3) + a.disp[2 * F + i]);
  step_update(a, i, F, u);
}

// step with the stencil footprint of an 8 x 8 x 16 tile staged in LDS (four nodes per thread:
// x1 = o1 + j1 + 4 h1, x2 = o2 + j2 + 4 h2): every departure point lies within D cells of its
// node, so its 4 x 4 x 4 stencil lies in [origin - D - 1, origin + tile + D + 1] per axis
// (G_i = tile_i + 2D + 3 values), which the block loads once, row by row along x3, instead of 64
// scattered loads per node.  D is a template parameter: every footprint size and LDS offset is a
// compile-time constant.  Indices are 32-bit (every grid here has fewer than 2^31 nodes).
constexpr int kT1 = 8, kT2 = 8, kT3 = 16;
constexpr int kRowLanes = 32;    // threads per staged row (G3 <= 32: D <= 6)
constexpr int kStageBatch = 16;  // rows per thread whose loads are in flight together
constexpr int kMaxStagedHalo = 6;
// periodic index for -n <= x < 2n
__device__ __forceinline__ int wrap1(int x, int n) { return x < 0 ? x + n : (x >= n ? x - n : x); }

template <typename T, int D>
__global__ void __launch_bounds__(kThreads) k_sl_step_lds(StepArgs<T> a) {
  constexpr int G1 = kT1 + 2 * D + 3, G2 = kT2 + 2 * D + 3, G3 = kT3 + 2 * D + 3;
  constexpr int NR = G1 * G2;
  constexpr int kRowsPerPass = kThreads / kRowLanes;
  constexpr int kPasses = (NR + kRowsPerPass - 1) / kRowsPerPass;
  static_assert(G3 <= kRowLanes, "one staged row per lane group");
  static_assert(kT3 * 4 * 4 == kThreads && kT1 == 8 && kT2 == 8, "four nodes per thread");
  __shared__ T C[G1 * G2 * G3];
  const Dims d = a.d;
  const unsigned F = unsigned(d.F());
  const int o1 = blockIdx.z * kT1, o2 = blockIdx.y * kT2, o3 = blockIdx.x * kT3;
  const int tid = threadIdx.x;
  const int j1 = tid / (4 * kT3), j2 = (tid / kT3) % 4, j3 = tid % kT3;
  unsigned node[4];
  T dsp[4][3];
#pragma unroll
  for (int h = 0; h < 4; ++h) {  // per-node displacements first: their latency overlaps the staging
    node[h] = (unsigned(o1 + j1 + 4 * (h >> 1)) * d.n2 + (o2 + j2 + 4 * (h & 1))) * d.n3 + (o3 + j3);
#pragma unroll
    for (int c = 0; c < 3; ++c) dsp[h][c] = a.disp[c * F + node[h]];
  }
  const int b1 = o1 - D - 1, b2 = o2 - D - 1, b3 = o3 - D - 1;
  const int lane = tid % kRowLanes;
  const int col = wrap1(b3 + min(lane, G3 - 1), d.n3);
  // staging: rows r = tid / 32 + 8 k walked incrementally; each batch of loads is issued before
  // any of its stores
  int r = tid / kRowLanes;
  int l1 = r / G2, l2 = r - l1 * G2;
#pragma unroll
  for (int k0 = 0; k0 < kPasses; k0 += kStageBatch) {
    T v[kStageBatch];
    int rr = r, q1 = l1, q2 = l2;
#pragma unroll
    for (int k = 0; k < kStageBatch; ++k) {
      if (k0 + k < kPasses) {
        const int c1 = min(q1, G1 - 1);  // rows past the footprint load a valid row, stored nowhere
        v[k] = a.coef[(unsigned(wrap1(b1 + c1, d.n1)) * d.n2 + wrap1(b2 + q2, d.n2)) * d.n3 + col];
        q2 += kRowsPerPass;
        while (q2 >= G2) {
          q2 -= G2;
          ++q1;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < kStageBatch; ++k) {
      if (k0 + k < kPasses) {
        if (rr < NR && lane < G3) C[rr * G3 + lane] = v[k];
        rr += kRowsPerPass;
      }
    }
    r = rr;
    l1 = q1;
    l2 = q2;
  }
  __syncthreads();
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    const T s1 = T(o1 + j1 + 4 * (h >> 1)) + dsp[h][0], s2 = T(o2 + j2 + 4 * (h & 1)) + dsp[h][1];
    const T s3 = T(o3 + j3) + dsp[h][2];
    const T f1 = floor(s1), f2 = floor(s2), f3 = floor(s3);
    T w1[4], w2[4], w3[4];
    bspline_w(s1 - f1, w1);
    bspline_w(s2 - f2, w2);
    bspline_w(s3 - f3, w3);
    // LDS coordinates of the stencil's first node; the clamp is inactive when |d| <= D
    const int m1 = min(max(int(f1) - 1 - b1, 0), G1 - 4);
    const int m2 = min(max(int(f2) - 1 - b2, 0), G2 - 4);
    const int m3 = min(max(int(f3) - 1 - b3, 0), G3 - 4);
    const T* base = C + (m1 * G2 + m2) * G3 + m3;
    T u = T(0);
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      T pa = T(0);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const T* row = base + (p * G2 + q) * G3;
        pa += w2[q] * (w3[0] * row[0] + w3[1] * row[1] + w3[2] * row[2] + w3[3] * row[3]);
      }
      u += w1[p] * pa;
    }
    step_update(a, node[h], F, u);
  }
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_trace(Dims d, T ht, const T* __restrict__ v, const T* __restrict__ cv,
                                                    const T* __restrict__ divv, const T* __restrict__ cdiv,
                                                    T* __restrict__ df, T* __restrict__ da, T* __restrict__ gamma) {
  const size_t F = d.F();
  const size_t i = size_t(blockIdx.x) * kThreads + threadIdx.x;
  if (i >= F) return;
  const int i3 = int(i % d.n3);
  const size_t t = i / d.n3;
  const int i2 = int(t % d.n2), i1 = int(t / d.n2);
  const T x[3] = {T(i1), T(i2), T(i3)};
  const T cells[3] = {T(d.n1 / (2.0 * 3.14159265358979323846)), T(d.n2 / (2.0 * 3.14159265358979323846)),
                      T(d.n3 / (2.0 * 3.14159265358979323846))};
  T u[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) u[c] = v[c * F + i] * cells[c];
  // forward characteristic: X* = x - ht u; departure x - ht/2 (u + u(X*))
  T w[3];
#pragma unroll
  for (int c = 0; c < 3; ++c)
    w[c] = interp3(cv + c * F, d, x[0] - ht * u[0], x[1] - ht * u[1], x[2] - ht * u[2]) * cells[c];
#pragma unroll
  for (int c = 0; c < 3; ++c) df[c * F + i] = -T(0.5) * ht * (u[c] + w[c]);
  // adjoint characteristic: the same with +ht
#pragma unroll
  for (int c = 0; c < 3; ++c)
    w[c] = interp3(cv + c * F, d, x[0] + ht * u[0], x[1] + ht * u[1], x[2] + ht * u[2]) * cells[c];
  T e[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    e[c] = T(0.5) * ht * (u[c] + w[c]);
    da[c * F + i] = e[c];
  }
  const T dD = interp3(cdiv, d, x[0] + e[0], x[1] + e[1], x[2] + e[2]);
  const T dx = divv[i];
  gamma[i] = T(1) + T(0.5) * ht * (dD + dx) + T(0.5) * ht * ht * dD * dx;
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_adjoint_start(size_t F, T w, const T* __restrict__ mR,
                                                            const T* __restrict__ m1, const T* __restrict__ gm,
                                                            T* __restrict__ lam, T* __restrict__ acc) {
  const size_t i = size_t(blockIdx.x) * kThreads + threadIdx.x;
  if (i >= F) return;
  const T l = mR[i] - m1[i];
  lam[i] = l;
#pragma unroll
  for (int c = 0; c < 3; ++c) acc[c * F + i] = w * l * gm[c * F + i];
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_incstate_start(size_t F, T ht, const T* __restrict__ vt,
                                                             const T* __restrict__ gm, T* __restrict__ q) {
  const size_t i = size_t(blockIdx.x) * kThreads + threadIdx.x;
  if (i >= F) return;
  const T f = -(vt[i] * gm[i] + vt[F + i] * gm[F + i] + vt[2 * F + i] * gm[2 * F + i]);
  q[i] = T(0.5) * ht * f;
}

// out_c = (w . g) g_c: the transport part of the GN matvec at v = 0
template <typename T>
__global__ void __launch_bounds__(kThreads) k_q_at_zero(size_t F, const T* __restrict__ w, const T* __restrict__ g,
                                                        T* __restrict__ out) {
  const size_t i = size_t(blockIdx.x) * kThreads + threadIdx.x;
  if (i >= F) return;
  const T g0 = g[i], g1 = g[F + i], g2 = g[2 * F + i];
  const T wg = w[i] * g0 + w[F + i] * g1 + w[2 * F + i] * g2;
  out[i] = wg * g0;
  out[F + i] = wg * g1;
  out[2 * F + i] = wg * g2;
}

// out_c = a v_c (c = 0, 1, 2)
template <typename T>
__global__ void __launch_bounds__(kThreads) k_scale_vec(size_t F, const T* __restrict__ a, const T* __restrict__ v,
                                                        T* __restrict__ out) {
  const size_t i = size_t(blockIdx.x) * kThreads + threadIdx.x;
  if (i >= F) return;
  const T s = a[i];
#pragma unroll
  for (int c = 0; c < 3; ++c) out[c * F + i] = s * v[c * F + i];
}

// out = ht/2 (1 + ht divv) e + ht/2 sig
template <typename T>
__global__ void __launch_bounds__(kThreads) k_fn_source(size_t F, T ht, const T* __restrict__ divv, const T* e,
                                                        const T* __restrict__ sig, T* out) {  // out may be e
  const size_t i = size_t(blockIdx.x) * kThreads + threadIdx.x;
  if (i >= F) return;
  out[i] = T(0.5) * ht * (T(1) + ht * divv[i]) * e[i] + T(0.5) * ht * sig[i];
}

// acc_c (init: =, else +=) w lam g_c (c = 0, 1, 2)
template <typename T>
__global__ void __launch_bounds__(kThreads) k_acc_scalar_grad(size_t F, T w, int init, const T* __restrict__ lam,
                                                              const T* __restrict__ g, T* __restrict__ acc) {
  const size_t i = size_t(blockIdx.x) * kThreads + threadIdx.x;
  if (i >= F) return;
  const T wl = w * lam[i];
#pragma unroll
  for (int c = 0; c < 3; ++c) acc[c * F + i] = init ? wl * g[c * F + i] : acc[c * F + i] + wl * g[c * F + i];
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_rk_stage(size_t F, RkStage<T> a) {
  const size_t i = size_t(blockIdx.x) * kThreads + threadIdx.x;
  if (i >= F) return;
  const T v0 = a.v[i], v1 = a.v[F + i], v2 = a.v[2 * F + i];
  const T y = a.y[i];
  T k = T(0.5 * a.sgn) * (v0 * a.g[i] + v1 * a.g[F + i] + v2 * a.g[2 * F + i] + a.dv[i] + T(a.dsgn) * y * a.divv[i]);
  if (a.src) k += a.src[i];
  T out;
  if (a.stage == 1) {
    a.kbuf[i] = k;
    out = y + T(a.ht) * k;
  } else {
    out = a.y0[i] + T(0.5 * a.ht) * (a.kbuf[i] + k);
  }
  a.dst[i] = out;
  a.yv[i] = out * v0;
  a.yv[F + i] = out * v1;
  a.yv[2 * F + i] = out * v2;
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_rk_eval(size_t F, int sgn, int dsgn, const T* __restrict__ g,
                                                      const T* __restrict__ dv, const T* __restrict__ a,
                                                      const T* __restrict__ w, const T* __restrict__ divw,
                                                      T* __restrict__ out) {
  const size_t i = size_t(blockIdx.x) * kThreads + threadIdx.x;
  if (i >= F) return;
  out[i] = T(0.5 * sgn) *
           (w[i] * g[i] + w[F + i] * g[F + i] + w[2 * F + i] * g[2 * F + i] + dv[i] + T(dsgn) * a[i] * divw[i]);
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_mul(size_t F, const T* __restrict__ a, const T* __restrict__ b,
                                                  T* __restrict__ out) {
  const size_t i = size_t(blockIdx.x) * kThreads + threadIdx.x;
  if (i >= F) return;
  out[i] = a[i] * b[i];
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_rk_accum(size_t F, T w, int init, const T* __restrict__ lam,
                                                       const T* __restrict__ m, const T* __restrict__ gm,
                                                       const T* __restrict__ gl, const T* __restrict__ glm,
                                                       T* __restrict__ acc) {
  const size_t i = size_t(blockIdx.x) * kThreads + threadIdx.x;
  if (i >= F) return;
  const T l = lam[i], mm = m[i];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const T t = T(0.5) * w * (l * gm[c * F + i] - mm * gl[c * F + i] + glm[c * F + i]);
    acc[c * F + i] = init ? t : acc[c * F + i] + t;
  }
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_axpby(size_t n, T a, const T* __restrict__ x, T b,
                                                    const T* __restrict__ y, T* __restrict__ out) {
  for (size_t i = size_t(blockIdx.x) * kThreads + threadIdx.x; i < n; i += size_t(gridDim.x) * kThreads) {
    T r = T(0);
    if (x) r = a * x[i];
    if (y) r += b * y[i];
    out[i] = r;
  }
}

constexpr int kMaxReduceBlocks = 1024;

template <typename T>
__global__ void __launch_bounds__(kThreads) k_reduce(size_t n, int mode, const T* __restrict__ a,
                                                     const T* __restrict__ b, double* __restrict__ partial) {
  __shared__ double red[kThreads];
  double s = 0.0;
  for (size_t i = size_t(blockIdx.x) * kThreads + threadIdx.x; i < n; i += size_t(gridDim.x) * kThreads) {
    if (mode == 0) {
      s += double(a[i]) * double(b[i]);
    } else if (mode == 1) {
      const double r = double(a[i]) - double(b[i]);
      s += r * r;
    } else {
      s = fmax(s, fabs(double(a[i])));
    }
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = mode == 2 ? fmax(red[threadIdx.x], red[threadIdx.x + w])
                                                      : red[threadIdx.x] + red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(kThreads) k_finish(int nb, int mode, const double* __restrict__ partial,
                                                     double* __restrict__ out) {
  __shared__ double red[kThreads];
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += kThreads) s = mode == 2 ? fmax(s, partial[i]) : s + partial[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = mode == 2 ? fmax(red[threadIdx.x], red[threadIdx.x + w])
                                                      : red[threadIdx.x] + red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

inline unsigned blocks_for(size_t n) { return unsigned((n + kThreads - 1) / kThreads); }

}  // namespace

template <typename T>
hipError_t fft_forward(hipStream_t s, const Dims& d, const Twiddles<T>& tw, int nf, const T* in, cplx<T>* S) {
  constexpr int RL = Tile<T>::RL;
  const int rows = d.n1 * d.n2, nh = d.nh();
  const size_t F = d.F(), Fh = d.Fh();
  hipLaunchKernelGGL(k_fft_r2c_rows<T>, dim3((rows + RL - 1) / RL, 1, nf), dim3(kThreads),
                     size_t(d.n3) * RL * sizeof(cplx<T>), s, in, F, S, Fh, rows, d.n3, ilog2(d.n3), tw.t3);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // along x2: lines (i1, k3), element stride nh
  e = launch_strided<T>(s, nf, S, Fh, d.n2, nh, d.n1, nh, (long long)d.n2 * nh, -1, tw.t2);
  if (e != hipSuccess) return e;
  // along x1: lines (i2, k3) = one contiguous run of n2 nh, element stride n2 nh
  return launch_strided<T>(s, nf, S, Fh, d.n1, d.n2 * nh, 1, (long long)d.n2 * nh, 0, -1, tw.t1);
}

template <typename T>
hipError_t fft_inverse(hipStream_t s, const Dims& d, const Twiddles<T>& tw, int nf, cplx<T>* S, T* out) {
  constexpr int RL = Tile<T>::RL;
  const int rows = d.n1 * d.n2, nh = d.nh();
  const size_t F = d.F(), Fh = d.Fh();
  hipError_t e = launch_strided<T>(s, nf, S, Fh, d.n1, d.n2 * nh, 1, (long long)d.n2 * nh, 0, +1, tw.t1);
  if (e != hipSuccess) return e;
  e = launch_strided<T>(s, nf, S, Fh, d.n2, nh, d.n1, nh, (long long)d.n2 * nh, +1, tw.t2);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fft_c2r_rows<T>, dim3((rows + RL - 1) / RL, 1, nf), dim3(kThreads),
                     size_t(d.n3) * RL * sizeof(cplx<T>), s, S, Fh, out, F, rows, d.n3, ilog2(d.n3),
                     T(1.0 / double(F)), tw.t3);
  return hipGetLastError();
}

size_t device_lds_limit();

template <typename T>
hipError_t spline_coefficients(hipStream_t s, const Dims& d, int nf, const T* in, T* out) {
  const Taps<T> tp = make_taps<T>();
  const size_t F = d.F();
  constexpr int RL = Fir<T>::RL, CL = Fir<T>::CL;
  const int rows = d.n1 * d.n2;
  // along x3 and x2 in one pass where a band of rows fits in LDS (else along x3 (rows), then x2
  // (lines (i1, i3), element stride n3)), then x1 (stride n2 n3); the passes after the first in
  // place
  constexpr int K = Fir<T>::K;
  hipError_t e = hipSuccess;
  const size_t plane_lds = FirPlane<T>::lds_bytes(d.n2, d.n3);
  if (plane_lds <= device_lds_limit()) {
    e = ensure_lds(k_fir_plane<T>, plane_lds);
    if (e != hipSuccess) return e;
    const int BR = FirPlane<T>::band(d.n2);
    hipLaunchKernelGGL(k_fir_plane<T>, dim3(d.n2 / BR, d.n1, nf),
                       dim3(FirPlane<T>::kThreadsX, FirPlane<T>::kThreadsY), plane_lds, s, in, out, F, d.n2, d.n3,
                       BR, tp);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  } else {
    hipLaunchKernelGGL(k_fir_rows<T>, dim3((rows + RL - 1) / RL, 1, nf), dim3(kThreads),
                       size_t(d.n3 + 2 * K) * RL * sizeof(T), s, in, out, F, rows, d.n3, tp);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = ensure_lds(k_fir_strided<T>, size_t(std::max(d.n1, d.n2) + 2 * K) * CL * sizeof(T));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fir_strided<T>, dim3((d.n3 + CL - 1) / CL, d.n1, nf), dim3(kThreads),
                       size_t(d.n2 + 2 * K) * CL * sizeof(T), s, out, out, F, d.n2, d.n3, (long long)d.n3,
                       (long long)d.n2 * d.n3, tp);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  e = ensure_lds(k_fir_strided<T>, size_t(std::max(d.n1, d.n2) + 2 * K) * CL * sizeof(T));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fir_strided<T>, dim3((d.n2 * d.n3 + CL - 1) / CL, 1, nf), dim3(kThreads),
                     size_t(d.n1 + 2 * K) * CL * sizeof(T), s, out, out, F, d.n1, d.n2 * d.n3, (long long)d.n2 * d.n3, 0LL,
                     tp);
  return hipGetLastError();
}

size_t device_lds_limit() {
  static std::atomic<size_t> lim{0};
  size_t v = lim.load(std::memory_order_acquire);
  if (v == 0) {
    int dev = 0, b = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&b, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
                                                hipSuccess)
      return 64 * 1024;
    v = size_t(b);
    lim.store(v, std::memory_order_release);
  }
  return v;
}

template <typename T, int OP, int NI>
hipError_t launch_x1_op(hipStream_t s, const Dims& d, const cplx<T>* Sin, cplx<T>* Sout, SymArgs a,
                        const cplx<T>* tw, bool& done) {
  constexpr int CL = Tile<T>::CL;
  const size_t lds = size_t(X1Op<T, OP, NI>::NB) * CL * d.n1 * sizeof(cplx<T>);
  done = false;
  if (lds > device_lds_limit()) return hipSuccess;
  const hipError_t e = ensure_lds(k_x1_op<T, OP, NI>, lds);
  if (e != hipSuccess) return e;
  const int inner = d.n2 * d.nh();
  hipLaunchKernelGGL((k_x1_op<T, OP, NI>), dim3((inner + CL - 1) / CL), dim3(kThreads), lds, s, d, Sin, Sout, a, tw);
  done = true;
  return hipGetLastError();
}

template <typename T, typename TF>
hipError_t spec_apply(hipStream_t s, const Dims& d, const Twiddles<T>& tw, SpecOp op, int nf, SymArgs a, const TF* in,
                      TF* out, cplx<T>* S1, cplx<T>* S2) {
  constexpr int RL = Tile<T>::RL;
  const int nin = op == SpecOp::Grad ? 1 : nf;
  const int nout = op == SpecOp::Grad ? 3 : (op == SpecOp::Div ? 1 : nf);
  if ((op == SpecOp::Scale && nf != 1 && nf != 3) || (op != SpecOp::Scale && nf != (op == SpecOp::Grad ? 1 : 3)))
    return hipErrorInvalidValue;
  const int rows = d.n1 * d.n2, nh = d.nh();
  const size_t F = d.F(), Fh = d.Fh();
  const long long sx1 = (long long)d.n2 * nh;
  hipLaunchKernelGGL((k_fft_r2c_rows<T, TF>), dim3((rows + RL - 1) / RL, 1, nin), dim3(kThreads),
                     size_t(d.n3) * RL * sizeof(cplx<T>), s, in, F, S1, Fh, rows, d.n3, ilog2(d.n3), tw.t3);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_strided<T>(s, nin, S1, Fh, d.n2, nh, d.n1, nh, sx1, -1, tw.t2);
  if (e != hipSuccess) return e;
  cplx<T>* So = op == SpecOp::Grad ? S2 : S1;
  bool done = false;
  if (op == SpecOp::Scale)
    e = nf == 1 ? launch_x1_op<T, 0, 1>(s, d, S1, So, a, tw.t1, done) : launch_x1_op<T, 0, 3>(s, d, S1, So, a, tw.t1, done);
  else if (op == SpecOp::Grad)
    e = launch_x1_op<T, 1, 1>(s, d, S1, So, a, tw.t1, done);
  else
    e = launch_x1_op<T, 2, 3>(s, d, S1, So, a, tw.t1, done);
  if (e != hipSuccess) return e;
  if (!done) {  // the lines do not fit the LDS: transform, operator and inverse as three passes
    e = launch_strided<T>(s, nin, S1, Fh, d.n1, d.n2 * nh, 1, sx1, 0, -1, tw.t1);
    if (e != hipSuccess) return e;
    if (op == SpecOp::Scale)
      e = spec_symbol<T>(s, d, nf, a, S1);
    else if (op == SpecOp::Grad)
      e = spec_grad<T>(s, d, S1, S2);
    else
      e = spec_div<T>(s, d, S1);
    if (e != hipSuccess) return e;
    e = launch_strided<T>(s, nout, So, Fh, d.n1, d.n2 * nh, 1, sx1, 0, +1, tw.t1);
    if (e != hipSuccess) return e;
  }
  e = launch_strided<T>(s, nout, So, Fh, d.n2, nh, d.n1, nh, sx1, +1, tw.t2);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_fft_c2r_rows<T, TF>), dim3((rows + RL - 1) / RL, 1, nout), dim3(kThreads),
                     size_t(d.n3) * RL * sizeof(cplx<T>), s, So, Fh, out, F, rows, d.n3, ilog2(d.n3),
                     T(1.0 / double(F)), tw.t3);
  return hipGetLastError();
}

template <typename T>
hipError_t spec_symbol(hipStream_t s, const Dims& d, int nf, SymArgs a, cplx<T>* S) {
  hipLaunchKernelGGL(k_symbol<T>, dim3(blocks_for(d.Fh())), dim3(kThreads), 0, s, d, nf, a, S);
  return hipGetLastError();
}

template <typename T>
hipError_t spec_restrict(hipStream_t s, const Dims& fine, const Dims& coarse, int nf, const cplx<T>* Sf, cplx<T>* Sc) {
  hipLaunchKernelGGL(k_restrict<T>, dim3(blocks_for(coarse.Fh())), dim3(kThreads), 0, s, fine, coarse, nf, Sf, Sc);
  return hipGetLastError();
}

template <typename T>
hipError_t spec_prolong_combine(hipStream_t s, const Dims& fine, const Dims& coarse, int nf, cplx<T>* Sf,
                                const cplx<T>* Sc) {
  hipLaunchKernelGGL(k_prolong_combine<T>, dim3(blocks_for(coarse.Fh())), dim3(kThreads), 0, s, fine, coarse, nf, Sf,
                     Sc);
  return hipGetLastError();
}

template <typename T>
hipError_t spec_grad(hipStream_t s, const Dims& d, const cplx<T>* U, cplx<T>* out) {
  hipLaunchKernelGGL(k_grad<T>, dim3(blocks_for(d.Fh())), dim3(kThreads), 0, s, d, U, out);
  return hipGetLastError();
}

template <typename T>
hipError_t spec_div(hipStream_t s, const Dims& d, cplx<T>* S) {
  hipLaunchKernelGGL(k_div<T>, dim3(blocks_for(d.Fh())), dim3(kThreads), 0, s, d, S);
  return hipGetLastError();
}

// the staged kernel for halo D when its footprint fits the default 64 KiB of static LDS, else the
// global-gather kernel
template <typename T, int D>
hipError_t launch_staged(hipStream_t s, const StepArgs<T>& a) {
  constexpr size_t bytes = size_t(kT1 + 2 * D + 3) * (kT2 + 2 * D + 3) * (kT3 + 2 * D + 3) * sizeof(T);
  if constexpr (bytes <= 64 * 1024) {
    hipLaunchKernelGGL((k_sl_step_lds<T, D>), dim3(a.d.n3 / kT3, a.d.n2 / kT2, a.d.n1 / kT1), dim3(kThreads), 0, s,
                       a);
  } else {
    hipLaunchKernelGGL(k_sl_step<T>, dim3(blocks_for(a.d.F())), dim3(kThreads), 0, s, a);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t sl_step(hipStream_t s, const StepArgs<T>& a) {
  // the staged kernel: halo known and small, the grid divisible into tiles, the staged region
  // within one period on each side (halo + 2 <= n, for wrap1)
  const int nmin = std::min(a.d.n1, std::min(a.d.n2, a.d.n3));
  const bool staged = a.halo >= 0 && a.halo <= kMaxStagedHalo && a.halo + 2 <= nmin && a.d.n1 % kT1 == 0 &&
                      a.d.n2 % kT2 == 0 && a.d.n3 % kT3 == 0;
  if (staged) {
    switch (a.halo) {
      case 0: return launch_staged<T, 0>(s, a);
      case 1: return launch_staged<T, 1>(s, a);
      case 2: return launch_staged<T, 2>(s, a);
      case 3: return launch_staged<T, 3>(s, a);
      case 4: return launch_staged<T, 4>(s, a);
      case 5: return launch_staged<T, 5>(s, a);
      default: return launch_staged<T, 6>(s, a);
    }
  }
  hipLaunchKernelGGL(k_sl_step<T>, dim3(blocks_for(a.d.F())), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t trace(hipStream_t s, const Dims& d, double ht, const T* v, const T* cv, const T* divv, const T* cdiv,
                 T* df, T* da, T* gamma) {
  hipLaunchKernelGGL(k_trace<T>, dim3(blocks_for(d.F())), dim3(kThreads), 0, s, d, T(ht), v, cv, divv, cdiv, df, da,
                     gamma);
  return hipGetLastError();
}

template <typename T>
hipError_t adjoint_start(hipStream_t s, const Dims& d, double w, const T* mR, const T* m1, const T* gm, T* lam,
                         T* acc) {
  hipLaunchKernelGGL(k_adjoint_start<T>, dim3(blocks_for(d.F())), dim3(kThreads), 0, s, d.F(), T(w), mR, m1, gm, lam,
                     acc);
  return hipGetLastError();
}

template <typename T>
hipError_t incstate_start(hipStream_t s, const Dims& d, double ht, const T* vt, const T* gm, T* q) {
  hipLaunchKernelGGL(k_incstate_start<T>, dim3(blocks_for(d.F())), dim3(kThreads), 0, s, d.F(), T(ht), vt, gm, q);
  return hipGetLastError();
}

template <typename T>
hipError_t q_at_zero(hipStream_t s, const Dims& d, const T* w, const T* g, T* out) {
  hipLaunchKernelGGL(k_q_at_zero<T>, dim3(blocks_for(d.F())), dim3(kThreads), 0, s, d.F(), w, g, out);
  return hipGetLastError();
}

template <typename T>
hipError_t scale_vec(hipStream_t s, const Dims& d, const T* a, const T* v, T* out) {
  hipLaunchKernelGGL(k_scale_vec<T>, dim3(blocks_for(d.F())), dim3(kThreads), 0, s, d.F(), a, v, out);
  return hipGetLastError();
}

template <typename T>
hipError_t fn_source(hipStream_t s, const Dims& d, double ht, const T* divv, const T* e, const T* sig, T* out) {
  hipLaunchKernelGGL(k_fn_source<T>, dim3(blocks_for(d.F())), dim3(kThreads), 0, s, d.F(), T(ht), divv, e, sig, out);
  return hipGetLastError();
}

template <typename T>
hipError_t acc_scalar_grad(hipStream_t s, const Dims& d, double w, int init, const T* lam, const T* g, T* acc) {
  hipLaunchKernelGGL(k_acc_scalar_grad<T>, dim3(blocks_for(d.F())), dim3(kThreads), 0, s, d.F(), T(w), init, lam, g,
                     acc);
  return hipGetLastError();
}

template <typename T>
hipError_t rk_stage(hipStream_t s, const Dims& d, const RkStage<T>& a) {
  hipLaunchKernelGGL(k_rk_stage<T>, dim3(blocks_for(d.F())), dim3(kThreads), 0, s, d.F(), a);
  return hipGetLastError();
}

template <typename T>
hipError_t rk_eval(hipStream_t s, const Dims& d, int sgn, int dsgn, const T* g, const T* dv, const T* a, const T* w,
                   const T* divw, T* out) {
  hipLaunchKernelGGL(k_rk_eval<T>, dim3(blocks_for(d.F())), dim3(kThreads), 0, s, d.F(), sgn, dsgn, g, dv, a, w, divw,
                     out);
  return hipGetLastError();
}

template <typename T>
hipError_t mul(hipStream_t s, const Dims& d, const T* a, const T* b, T* out) {
  hipLaunchKernelGGL(k_mul<T>, dim3(blocks_for(d.F())), dim3(kThreads), 0, s, d.F(), a, b, out);
  return hipGetLastError();
}

template <typename T>
hipError_t rk_accum(hipStream_t s, const Dims& d, double w, int init, const T* lam, const T* m, const T* gm,
                    const T* gl, const T* glm, T* acc) {
  hipLaunchKernelGGL(k_rk_accum<T>, dim3(blocks_for(d.F())), dim3(kThreads), 0, s, d.F(), T(w), init, lam, m, gm, gl,
                     glm, acc);
  return hipGetLastError();
}

template <typename T>
hipError_t axpby(hipStream_t s, size_t n, double a, const T* x, double b, const T* y, T* out) {
  const unsigned nb = std::min<size_t>(blocks_for(n), 8192);
  hipLaunchKernelGGL(k_axpby<T>, dim3(nb), dim3(kThreads), 0, s, n, T(a), x, T(b), y, out);
  return hipGetLastError();
}

template hipError_t spec_apply<double, float>(hipStream_t, const Dims&, const Twiddles<double>&, SpecOp, int, SymArgs,
                                              const float*, float*, cplx<double>*, cplx<double>*);

int reduce_blocks(size_t n) { return int(std::min<size_t>(blocks_for(n), kMaxReduceBlocks)); }

template <typename T>
hipError_t reduce(hipStream_t s, size_t n, int mode, const T* a, const T* b, double* partial, double* out) {
  const int nb = reduce_blocks(n);
  hipLaunchKernelGGL(k_reduce<T>, dim3(nb), dim3(kThreads), 0, s, n, mode, a, b, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(kThreads), 0, s, nb, mode, partial, out);
  return hipGetLastError();
}

#define INST(T)                                                                                                   \
  template hipError_t fft_forward<T>(hipStream_t, const Dims&, const Twiddles<T>&, int, const T*, cplx<T>*);      \
  template hipError_t fft_inverse<T>(hipStream_t, const Dims&, const Twiddles<T>&, int, cplx<T>*, T*);            \
  template hipError_t spec_symbol<T>(hipStream_t, const Dims&, int, SymArgs, cplx<T>*);                          \
  template hipError_t spec_apply<T, T>(hipStream_t, const Dims&, const Twiddles<T>&, SpecOp, int, SymArgs, const T*, \
                                       T*, cplx<T>*, cplx<T>*);                                                  \
  template hipError_t spline_coefficients<T>(hipStream_t, const Dims&, int, const T*, T*);                       \
  template hipError_t spec_grad<T>(hipStream_t, const Dims&, const cplx<T>*, cplx<T>*);                          \
  template hipError_t spec_restrict<T>(hipStream_t, const Dims&, const Dims&, int, const cplx<T>*, cplx<T>*);    \
  template hipError_t spec_prolong_combine<T>(hipStream_t, const Dims&, const Dims&, int, cplx<T>*,             \
                                              const cplx<T>*);                                                   \
  template hipError_t spec_div<T>(hipStream_t, const Dims&, cplx<T>*);                                           \
  template hipError_t sl_step<T>(hipStream_t, const StepArgs<T>&);                                               \
  template hipError_t trace<T>(hipStream_t, const Dims&, double, const T*, const T*, const T*, const T*, T*, T*,  \
                               T*);                                                                               \
  template hipError_t adjoint_start<T>(hipStream_t, const Dims&, double, const T*, const T*, const T*, T*, T*);  \
  template hipError_t incstate_start<T>(hipStream_t, const Dims&, double, const T*, const T*, T*);               \
  template hipError_t q_at_zero<T>(hipStream_t, const Dims&, const T*, const T*, T*);                           \
  template hipError_t scale_vec<T>(hipStream_t, const Dims&, const T*, const T*, T*);                           \
  template hipError_t rk_stage<T>(hipStream_t, const Dims&, const RkStage<T>&);                                 \
  template hipError_t rk_eval<T>(hipStream_t, const Dims&, int, int, const T*, const T*, const T*, const T*,    \
                                 const T*, T*);                                                                 \
  template hipError_t mul<T>(hipStream_t, const Dims&, const T*, const T*, T*);                                 \
  template hipError_t rk_accum<T>(hipStream_t, const Dims&, double, int, const T*, const T*, const T*,          \
                                  const T*, const T*, T*);                                                      \
  template hipError_t fn_source<T>(hipStream_t, const Dims&, double, const T*, const T*, const T*, T*);         \
  template hipError_t acc_scalar_grad<T>(hipStream_t, const Dims&, double, int, const T*, const T*, T*);        \
  template hipError_t axpby<T>(hipStream_t, size_t, double, const T*, double, const T*, T*);                     \
  template hipError_t reduce<T>(hipStream_t, size_t, int, const T*, const T*, double*, double*);
INST(float)
INST(double)
#undef INST

}  // namespace d3
}  // namespace slnk
