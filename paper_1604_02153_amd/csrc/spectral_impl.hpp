// Pseudospectral operators on the periodic grid: LDS-resident mixed-radix (8, 4, 2, 3, 5)
// Stockham FFTs fused with the spectral diagonal operators of the method (section 3.2: Fourier
// discretisation; eq. e:diffopregv: regulariser symbols; eq. e:reg-precond: P_REG; section
// 3.4.2: split preconditioning, cut-off filters, spectral restriction and prolongation).
//
// Layout.  A real field is [n1][n2].  Two real fields are packed as one complex row (a + i b),
// transformed along x2 and unpacked into two half spectra ("row pass").  The column pass
// transforms the n2/2+1 columns along x1, applies the symbol (which may read several input
// spectra and write several outputs) and transforms back.  The inverse row pass packs two
// Hermitian half spectra into one complex row, inverts it and writes both real fields.
//
// Two implementations.  When n1 and n2 are both common lengths (64..1024 powers of two, 96..768
// three times a power of two) the wave-level passes run, and the half spectra are stored
// transposed, [n2/2+1][n1], so that the column pass reads and writes whole rows.  Otherwise the
// generic passes run on half spectra [n1][spec_stride(n2)], with LDS-resident transforms of any
// 2-3-5 length and workgroup barriers between stages.  The layout never leaves this file; a
// restriction or prolongation takes the wave-level form only when both of its grids do.
//
// Conventions: forward transforms are unnormalised; every symbol carries the 1/(n1 n2) of the
// inverse.  Odd symbols (derivatives) drop the Nyquist modes, even symbols keep them.
//
// Compiled once per precision: spectral_f32.hip and spectral_f64.hip define SLNK_SPECTRAL_REAL
// and include this file.
#pragma once

#include <atomic>
#include <mutex>

#include "kernels.hpp"

namespace slnk {
namespace {

constexpr int kMaxE = 16;          // complex elements per thread held by one FFT stage
constexpr int kLdsBudget = 136 * 1024;  // column-pass panels (gfx950: 160 KiB of LDS per workgroup)
constexpr size_t kLdsDefault = 64 * 1024;  // dynamic LDS a kernel gets without an attribute

std::mutex g_attr_mutex;

// Raise a kernel's dynamic-LDS limit before its first launch above 64 KiB (once per size).
template <typename K>
hipError_t allow_lds(K kfn, size_t lds, std::atomic<size_t>& allowed) {
  if (lds <= kLdsDefault || lds <= allowed.load(std::memory_order_acquire)) return hipSuccess;
  std::lock_guard<std::mutex> lock(g_attr_mutex);
  if (lds <= allowed.load(std::memory_order_relaxed)) return hipSuccess;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kfn), hipFuncAttributeMaxDynamicSharedMemorySize,
                                     int(lds));
  if (e == hipSuccess) allowed.store(lds, std::memory_order_release);
  return e;
}

// ---------------------------------------------------------------------------------------
// small DFTs; sign = -1 forward, +1 inverse
// ---------------------------------------------------------------------------------------
template <typename T, int RAD>
struct Dft;

template <typename T>
struct Dft<T, 2> {
  __device__ static void run(cplx<T>* x, int) {
    cplx<T> a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
  }
};

template <typename T>
struct Dft<T, 4> {
  __device__ static void run(cplx<T>* x, int sign) {
    cplx<T> a = cadd(x[0], x[2]), b = csub(x[0], x[2]);
    cplx<T> c = cadd(x[1], x[3]), d = csub(x[1], x[3]);
    d = sign < 0 ? cmul_mi(d) : cmul_i(d);   // omega = exp(sign 2 pi i / 4) = sign * i
    x[0] = cadd(a, c);
    x[1] = cadd(b, d);
    x[2] = csub(a, c);
    x[3] = csub(b, d);
  }
};

template <typename T>
struct Dft<T, 8> {
  __device__ static void run(cplx<T>* x, int sign) {
    // two radix-4 transforms of the even and odd samples, combined with omega_8^k
    cplx<T> e[4] = {x[0], x[2], x[4], x[6]};
    cplx<T> o[4] = {x[1], x[3], x[5], x[7]};
    Dft<T, 4>::run(e, sign);
    Dft<T, 4>::run(o, sign);
    const T r = T(0.707106781186547524400844362104849);  // sqrt(1/2)
    const T sg = sign < 0 ? T(-1) : T(1);
    const cplx<T> w1 = {r, sg * r}, w3 = {-r, sg * r};
    const cplx<T> o1 = cmul(o[1], w1);
    const cplx<T> o2 = sign < 0 ? cmul_mi(o[2]) : cmul_i(o[2]);
    const cplx<T> o3 = cmul(o[3], w3);
    x[0] = cadd(e[0], o[0]);
    x[4] = csub(e[0], o[0]);
    x[1] = cadd(e[1], o1);
    x[5] = csub(e[1], o1);
    x[2] = cadd(e[2], o2);
    x[6] = csub(e[2], o2);
    x[3] = cadd(e[3], o3);
    x[7] = csub(e[3], o3);
  }
};

template <typename T>
struct Dft<T, 3> {
  __device__ static void run(cplx<T>* x, int sign) {
    const T h = T(0.866025403784438646763723170752936);  // sin(2 pi / 3)
    cplx<T> t1 = cadd(x[1], x[2]), t2 = csub(x[1], x[2]);
    cplx<T> m = {x[0].x - T(0.5) * t1.x, x[0].y - T(0.5) * t1.y};
    cplx<T> r = cscale(sign < 0 ? cmul_mi(t2) : cmul_i(t2), h);
    x[0] = cadd(x[0], t1);
    x[1] = cadd(m, r);
    x[2] = csub(m, r);
  }
};

template <typename T>
struct Dft<T, 5> {
  __device__ static void run(cplx<T>* x, int sign) {
    const T c1 = T(0.309016994374947424102293417182819);   // cos(2 pi / 5)
    const T c2 = T(-0.809016994374947424102293417182819);  // cos(4 pi / 5)
    const T s1 = T(0.951056516295153572116439333379382);   // sin(2 pi / 5)
    const T s2 = T(0.587785252292473129168705954639073);   // sin(4 pi / 5)
    cplx<T> t1 = cadd(x[1], x[4]), t2 = cadd(x[2], x[3]);
    cplx<T> t3 = csub(x[1], x[4]), t4 = csub(x[2], x[3]);
    cplx<T> a1 = {x[0].x + c1 * t1.x + c2 * t2.x, x[0].y + c1 * t1.y + c2 * t2.y};
    cplx<T> a2 = {x[0].x + c2 * t1.x + c1 * t2.x, x[0].y + c2 * t1.y + c1 * t2.y};
    cplx<T> b1 = {s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y};
    cplx<T> b2 = {s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y};
    b1 = sign < 0 ? cmul_mi(b1) : cmul_i(b1);
    b2 = sign < 0 ? cmul_mi(b2) : cmul_i(b2);
    x[0] = cadd(x[0], cadd(t1, t2));
    x[1] = cadd(a1, b1);
    x[4] = csub(a1, b1);
    x[2] = cadd(a2, b2);
    x[3] = csub(a2, b2);
  }
};

// LDS position of element e of a transform: an XOR swizzle of the low five index bits by bits
// 3..7.  It permutes every aligned block of 32 elements, and it spreads both the contiguous reads
// and the stride-RAD writes of the Stockham stages (and the column transposes, with a sequence
// stride of 4 mod 32) over the 64 LDS banks.
__device__ __forceinline__ int swz(int e) { return e ^ ((e >> 3) & 31); }

// sequence stride (complex elements) of LDS-resident transforms of length n: room for the swizzle
// (a multiple of 32) plus 4
__host__ __device__ __forceinline__ int lds_stride(int n) { return (n + 31) / 32 * 32 + 4; }

// One Stockham stage of radix RAD over 'nbatch' transforms of length n held in LDS; element e of
// transform b lives at buf[b * bs + swz(e)].  p is the product of the radices of earlier stages.
// The stage reads every input into registers, synchronises, then writes every output, so it
// works in place.
template <typename T, int RAD, int MAXB>
__device__ void fft_stage(cplx<T>* buf, int n, int p, int nbatch, int bs, const cplx<T>* tw,
                          int sign, int tid, int nthr) {
  const int nb = n / RAD;
  const int total = nbatch * nb;
  cplx<T> y[MAXB][RAD];
  int ob[MAXB], oi[MAXB];
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int t = tid + q * nthr;
    if (t < total) {
      const int b = t / nb;
      const int i = t - b * nb;
      const int k = i % p;
      cplx<T> x[RAD];
#pragma unroll
      for (int j = 0; j < RAD; ++j) {
        cplx<T> val = buf[b * bs + swz(i + j * nb)];
        if (j > 0 && k > 0) {
          cplx<T> w = tw[(j - 1) * p + k];
          if (sign > 0) w.y = -w.y;
          val = cmul(val, w);
        }
        x[j] = val;
      }
      Dft<T, RAD>::run(x, sign);
#pragma unroll
      for (int j = 0; j < RAD; ++j) y[q][j] = x[j];
      ob[q] = b * bs;
      oi[q] = (i - k) * RAD + k;
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int t = tid + q * nthr;
    if (t < total) {
#pragma unroll
      for (int j = 0; j < RAD; ++j) buf[ob[q] + swz(oi[q] + j * p)] = y[q][j];
    }
  }
  __syncthreads();
}

// Copy the twiddle table of a plan into LDS (the caller synchronises before use).
template <typename T>
__device__ __forceinline__ void load_twiddles(cplx<T>* tw_lds, const FFTPlanDev& pl, int tid, int nthr) {
  const cplx<T>* tw = static_cast<const cplx<T>*>(pl.tw);
  for (int q = tid; q < pl.ntw; q += nthr) tw_lds[q] = tw[q];
}

// Full transform of nbatch sequences (nbatch * n <= kMaxE * nthr) with the twiddles in LDS.
template <typename T>
__device__ void fft_lds(cplx<T>* buf, const cplx<T>* tw, const FFTPlanDev& pl, int nbatch, int bs, int sign, int tid,
                        int nthr) {
  int p = 1;
  for (int s = 0; s < pl.nstages; ++s) {
    const int r = pl.radix[s];
    const cplx<T>* tws = tw + pl.twoff[s];
    if (r == 8)
      fft_stage<T, 8, kMaxE / 8>(buf, pl.n, p, nbatch, bs, tws, sign, tid, nthr);
    else if (r == 4)
      fft_stage<T, 4, kMaxE / 4>(buf, pl.n, p, nbatch, bs, tws, sign, tid, nthr);
    else if (r == 2)
      fft_stage<T, 2, kMaxE / 2>(buf, pl.n, p, nbatch, bs, tws, sign, tid, nthr);
    else if (r == 3)
      fft_stage<T, 3, (kMaxE + 2) / 3>(buf, pl.n, p, nbatch, bs, tws, sign, tid, nthr);
    else
      fft_stage<T, 5, (kMaxE + 4) / 5>(buf, pl.n, p, nbatch, bs, tws, sign, tid, nthr);
    p *= r;
  }
}

// ---------------------------------------------------------------------------------------
// row passes
// ---------------------------------------------------------------------------------------
// Up to 8 real fields per batch item; field f of item z is p[f] + z * bstride[f].  Items with
// active[z / item_div] == 0 are skipped (active optional).
template <typename T>
struct RealFields {
  const T* p[8];
  long long bstride[8];
  int count;
  const int* active;
  int item_div;
};

template <typename T>
struct OutFields {
  T* p[8];
  const T* add[8];
  long long bstride[8];
  int count;
  const int* active;
  int item_div;
};

// Forward row pass: fields (2q, 2q+1) of 'in' (batch item z) packed as one complex row, FFT along
// x2, unpacked into half spectra S[z][f][x1][k2] (f = 2q, 2q+1; k2 in [0, n2/2]).
template <typename T, typename TF>
__global__ void __launch_bounds__(256) k_row_fwd(RealFields<TF> in, cplx<T>* __restrict__ S, int n1, int n2,
                                                 int rpb, FFTPlanDev pl) {
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* tw = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* buf = tw + n2;
  const int nh = n2 / 2 + 1;
  const int bs = lds_stride(n2);
  const int q = blockIdx.y;
  const int z = blockIdx.z;
  const int r0 = blockIdx.x * rpb;
  const int rows = min(rpb, n1 - r0);
  const int fa = 2 * q, fb = 2 * q + 1;
  if (in.active && !in.active[z / in.item_div]) return;
  load_twiddles<T>(tw, pl, threadIdx.x, blockDim.x);
  const TF* A = in.p[fa] + z * in.bstride[fa];
  const TF* B = fb < in.count ? in.p[fb] + z * in.bstride[fb] : nullptr;
  const int tid = threadIdx.x, nthr = blockDim.x;
  for (int idx = tid; idx < rows * n2; idx += nthr) {
    const int r = idx / n2, c = idx - r * n2;
    const size_t gi = size_t(r0 + r) * n2 + c;
    buf[r * bs + swz(c)] = {T(A[gi]), B ? T(B[gi]) : T(0)};
  }
  __syncthreads();
  fft_lds<T>(buf, tw, pl, rows, bs, -1, tid, nthr);
  const int nhp = spec_stride(n2);
  const size_t sf = size_t(n1) * nhp;
  cplx<T>* SA = S + (size_t(z) * in.count + fa) * sf;
  cplx<T>* SB = S + (size_t(z) * in.count + fb) * sf;
  for (int idx = tid; idx < rows * nh; idx += nthr) {
    const int r = idx / nh, k = idx - r * nh;
    const cplx<T> zk = buf[r * bs + swz(k)];
    const cplx<T> zm = cconj(buf[r * bs + swz(k == 0 ? 0 : n2 - k)]);
    const size_t o = size_t(r0 + r) * nhp + k;
    SA[o] = cscale(cadd(zk, zm), T(0.5));
    if (B) SB[o] = cscale(cmul_mi(csub(zk, zm)), T(0.5));
  }
}

// Inverse row pass: half spectra (2q, 2q+1) of S[z] -> real fields out (plus optional addend).
template <typename T, typename TF>
__global__ void __launch_bounds__(256) k_row_inv(const cplx<T>* __restrict__ S, int nspec, OutFields<TF> out,
                                                 int n1, int n2, int rpb, FFTPlanDev pl) {
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* tw = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* buf = tw + n2;
  const int nh = n2 / 2 + 1;
  const int bs = lds_stride(n2);
  const int q = blockIdx.y;
  const int z = blockIdx.z;
  const int r0 = blockIdx.x * rpb;
  const int rows = min(rpb, n1 - r0);
  const int fa = 2 * q, fb = 2 * q + 1;
  const bool hasb = fb < out.count;
  if (out.active && !out.active[z / out.item_div]) return;
  load_twiddles<T>(tw, pl, threadIdx.x, blockDim.x);
  const int nhp = spec_stride(n2);
  const size_t sf = size_t(n1) * nhp;
  const cplx<T>* SA = S + (size_t(z) * nspec + fa) * sf;
  const cplx<T>* SB = S + (size_t(z) * nspec + fb) * sf;
  const int tid = threadIdx.x, nthr = blockDim.x;
  for (int idx = tid; idx < rows * n2; idx += nthr) {
    const int r = idx / n2, k = idx - r * n2;
    const bool mirror = k > n2 / 2;
    const int kk = mirror ? n2 - k : k;
    const size_t o = size_t(r0 + r) * nhp + kk;
    cplx<T> a = SA[o];
    cplx<T> b = hasb ? SB[o] : cplx<T>{T(0), T(0)};
    if (kk == 0 || kk == n2 / 2) {  // a real row's DC and Nyquist coefficients are real
      a.y = T(0);
      b.y = T(0);
    }
    if (mirror) {
      a = cconj(a);
      b = cconj(b);
    }
    buf[r * bs + swz(k)] = cadd(a, cmul_i(b));
  }
  __syncthreads();
  fft_lds<T>(buf, tw, pl, rows, bs, +1, tid, nthr);
  TF* OA = out.p[fa] + z * out.bstride[fa];
  TF* OB = hasb ? out.p[fb] + z * out.bstride[fb] : nullptr;
  const TF* AA = out.add[fa] ? out.add[fa] + z * out.bstride[fa] : nullptr;
  const TF* AB = hasb && out.add[fb] ? out.add[fb] + z * out.bstride[fb] : nullptr;
  for (int idx = tid; idx < rows * n2; idx += nthr) {
    const int r = idx / n2, c = idx - r * n2;
    const size_t gi = size_t(r0 + r) * n2 + c;
    const cplx<T> val = buf[r * bs + swz(c)];
    OA[gi] = TF(AA ? val.x + T(AA[gi]) : val.x);
    if (OB) OB[gi] = TF(AB ? val.y + T(AB[gi]) : val.y);
  }
}

// ---------------------------------------------------------------------------------------
// column pass with a symbol
// ---------------------------------------------------------------------------------------
enum ColFlags : int { kInK = 1, kOutK = 2 };

// Column pass over B columns (k2 = c0 .. c0 + B - 1) of every input spectrum of batch item z:
// forward FFT along x1 (unless kInK), op at every (k1, k2), inverse FFT (unless kOutK).
template <typename T, class Op>
__global__ void __launch_bounds__(1024) k_col(const cplx<T>* __restrict__ Sin, cplx<T>* __restrict__ Sout, int n1,
                                              int n2, int B, FFTPlanDev pl, Op op, int flags, const int* active,
                                              int item_div) {
  if (active && !active[blockIdx.z / item_div]) return;
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* tw = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* buf = tw + n1;
  constexpr int NIN = Op::NIN, NOUT = Op::NOUT;
  load_twiddles<T>(tw, pl, threadIdx.x, blockDim.x);
  const int nh = n2 / 2 + 1;
  const int bs = lds_stride(n1);
  const int c0 = blockIdx.x * B;
  const int cols = min(B, nh - c0);
  const int z = blockIdx.z;
  const int nhp = spec_stride(n2);
  const size_t sf = size_t(n1) * nhp;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const cplx<T>* in = Sin + size_t(z) * NIN * sf;
  for (int f = 0; f < NIN; ++f)
    for (int idx = tid; idx < n1 * cols; idx += nthr) {
      const int e = idx / cols, b = idx - e * cols;
      buf[(f * B + b) * bs + swz(e)] = in[f * sf + size_t(e) * nhp + c0 + b];
    }
  __syncthreads();
  if (!(flags & kInK)) fft_lds<T>(buf, tw, pl, NIN * B, bs, -1, tid, nthr);
  for (int idx = tid; idx < n1 * cols; idx += nthr) {
    const int b = idx / n1, e = idx - b * n1;
    cplx<T> vin[NIN > 0 ? NIN : 1];
    cplx<T> vout[NOUT > 0 ? NOUT : 1];
#pragma unroll
    for (int f = 0; f < NIN; ++f) vin[f] = buf[(f * B + b) * bs + swz(e)];
    op(signed_wavenumber(e, n1), c0 + b, e, z, vin, vout);
#pragma unroll
    for (int f = 0; f < NOUT; ++f) buf[(f * B + b) * bs + swz(e)] = vout[f];
  }
  __syncthreads();
  if (NOUT == 0) return;
  if (!(flags & kOutK)) fft_lds<T>(buf, tw, pl, NOUT * B, bs, +1, tid, nthr);
  cplx<T>* out = Sout + size_t(z) * NOUT * sf;
  for (int f = 0; f < NOUT; ++f)
    for (int idx = tid; idx < n1 * cols; idx += nthr) {
      const int e = idx / cols, b = idx - e * cols;
      out[f * sf + size_t(e) * nhp + c0 + b] = buf[(f * B + b) * bs + swz(e)];
    }
}

// ---------------------------------------------------------------------------------------
// Wave-level transforms of the common lengths: powers of two 64..1024 and 3 * 2^k, 96..768.
// A transform belongs to LPT = N / E lanes of one wavefront (E = 8 elements per lane for powers
// of two up to 512, 16 for 1024, 12 otherwise), so a wavefront holds 64 / LPT transforms.  A stage keeps the lane's
// elements in registers; between stages the wavefront exchanges them through its own LDS region,
// so the transforms need no workgroup barrier.  Stockham order: butterfly i (k = i mod p) of a
// radix-r stage reads elements i + j N / r and writes (i - k) r + k + j p.  Lane lp of a
// transform owns butterflies lp + LPT q, so the first stage reads elements lp + LPT q + j N / r1
// and the last stage leaves element lp + LPT q + j N / rL in register q rL + j.  A transform run
// with the radix list reversed starts from exactly that mapping (and ends in the r1 mapping).
// ---------------------------------------------------------------------------------------
template <int N>
struct WPlan {
  static constexpr bool kPow2 = (N & (N - 1)) == 0;
  static constexpr int E = kPow2 ? (N <= 512 ? 8 : 16) : 12;
  static constexpr int LPT = N / E;
  static constexpr int T = 64 / LPT;
  static constexpr int NS = N == 64 ? 2 : N == 128 || N == 256 || N == 512 ? 3 : N == 384 || N == 768 ? 5 : 4;
  static constexpr int radix(int s) {
    switch (N) {
      case 64: return 8;
      case 128: return s == 0 ? 8 : 4;
      case 256: return s < 2 ? 8 : 4;
      case 512: return 8;
      case 1024: return s < 2 ? 8 : 4;
      case 96: return s == 0 ? 3 : (s < 3 ? 4 : 2);
      case 192: return s == 0 ? 3 : 4;
      case 384: return s == 0 ? 3 : (s < 4 ? 4 : 2);
      case 768: return s == 0 ? 3 : 4;
    }
    return 0;
  }
  static constexpr int product() {
    int p = 1;
    for (int s = 0; s < NS; ++s) p *= radix(s);
    return p;
  }
  // LDS strides (complex elements) of a transform's region: exchange only (column passes), and
  // exchange plus the transposed access of the row passes (chosen with a bank model of gfx950's
  // 64 banks)
  static constexpr int col_stride = N + (N == 64 || N == 96 ? 8 : N == 128 || N == 192 ? 16 : 0);
  static constexpr int row_stride = N + (N == 96 ? 8 : N == 64 || N == 1024 || N == 768 ? 4 : 2);
  // element e of a region: XOR swizzle of the low five bits (powers of two), identity otherwise
  __device__ static __forceinline__ int pos(int e) {
    if constexpr (kPow2)
      return e ^ ((e >> 3) & 31);
    else
      return e;
  }
};

// Orders the wavefront's LDS accesses around an exchange (LDS operations of one wavefront complete
// in issue order; the fences keep the compiler from moving them across).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Stage s of the radix list in order REV: radix, product p of the earlier radices, and the offset
// of its twiddles w_(r p)^(j k) at tw[off + (j - 1) p + k] (j = 1..r-1, k < p; N - 1 in all), so
// that consecutive butterflies read consecutive entries.
template <int N, bool REV>
struct WStages {
  static constexpr int NS = WPlan<N>::NS;
  static constexpr int radix(int s) { return WPlan<N>::radix(REV ? NS - 1 - s : s); }
  static constexpr int pprod(int s) {
    int p = 1;
    for (int t = 0; t < s; ++t) p *= radix(t);
    return p;
  }
  static constexpr int off(int s) {
    int o = 0;
    for (int t = 0; t < s; ++t) o += (radix(t) - 1) * pprod(t);
    return o;
  }
};

// Fill the stage twiddle table of order REV (N - 1 entries) from the roots exp(-2 pi i m / N).
template <typename T, int N, bool REV>
__device__ void fill_twiddles(cplx<T>* tw, const cplx<T>* __restrict__ roots, int tid, int nthr) {
  using WS = WStages<N, REV>;
  for (int idx = tid; idx < N - 1; idx += nthr) {
    int p = 1, r = WS::radix(0), base = 0;
#pragma unroll
    for (int t = 1; t < WS::NS; ++t)
      if (idx >= WS::off(t)) {
        p = WS::pprod(t);
        r = WS::radix(t);
        base = WS::off(t);
      }
    const int rel = idx - base;
    const int j = rel / p + 1, k = rel - (j - 1) * p;
    tw[idx] = roots[j * k * (N / (r * p))];
  }
}

// Transform of length N (SIGN -1 forward, +1 inverse, unnormalised) of the elements x held by lane
// lp of a transform in the first stage's mapping; returns the outputs in the last stage's mapping.
// reg: the transform's LDS region (N elements at WPlan::pos); tw: the stage twiddles of order REV.
// LAUNDER recomputes the LDS and twiddle addresses of every stage (they depend on lp alone)
// instead of keeping them live across all transforms of a kernel.
template <typename T, int N, int SIGN, bool REV, bool LAUNDER, int S = 0, int P = 1>
__device__ __forceinline__ void wave_fft(cplx<T> (&x)[WPlan<N>::E], cplx<T>* reg, const cplx<T>* tw, int lp) {
  using PL = WPlan<N>;
  using WS = WStages<N, REV>;
  constexpr int NS = PL::NS;
  static_assert(PL::product() == N, "radix list must multiply to N");
  static_assert(PL::E % PL::radix(S < NS ? (REV ? NS - 1 - S : S) : 0) == 0, "radix must divide E");
  if constexpr (S < NS) {
    constexpr int r = WS::radix(S);
    static_assert(WS::pprod(S) == P, "stage product");
    if constexpr (LAUNDER) asm volatile("" : "+v"(lp));
#pragma unroll
    for (int q = 0; q < PL::E / r; ++q) {
      if constexpr (P > 1) {
        const int k = (lp + PL::LPT * q) % P;
#pragma unroll
        for (int j = 1; j < r; ++j) {
          cplx<T> w = tw[WS::off(S) + (j - 1) * P + k];
          if (SIGN > 0) w.y = -w.y;
          x[q * r + j] = cmul(x[q * r + j], w);
        }
      }
      Dft<T, r>::run(&x[q * r], SIGN);
    }
    if constexpr (S + 1 < NS) {
      constexpr int rn = PL::radix(REV ? NS - 2 - S : S + 1);
#pragma unroll
      for (int q = 0; q < PL::E / r; ++q) {
        const int i = lp + PL::LPT * q;
        const int k = i % P;
#pragma unroll
        for (int j = 0; j < r; ++j) reg[PL::pos((i - k) * r + k + j * P)] = x[q * r + j];
      }
      wave_sync();
#pragma unroll
      for (int q = 0; q < PL::E / rn; ++q)
#pragma unroll
        for (int j = 0; j < rn; ++j) x[q * rn + j] = reg[PL::pos(lp + PL::LPT * q + j * (N / rn))];
      wave_sync();
    }
    wave_fft<T, N, SIGN, REV, LAUNDER, S + 1, P * r>(x, reg, tw, lp);
  }
}

// element index held in register m by lane lp in the mapping of a radix-r first or last stage
template <int N, int r>
__device__ __forceinline__ int wmap(int lp, int m) {
  return lp + WPlan<N>::LPT * (m / r) + (m % r) * (N / r);
}

// ---- wave-level passes -------------------------------------------------------------------
// Intermediate layout: the half spectra are stored transposed, St[k2][x1] (row k2 < n2/2 + 1 of
// n1 contiguous values), so that the column transforms read and write whole rows.

// rows per workgroup of the row passes (transposed segments of R complex values)
template <typename T, int N>
struct FRow {
  static constexpr int R = sizeof(T) == 4 ? (N >= 768 ? 8 : 16) : (N >= 768 ? 4 : N >= 192 ? 8 : 16);
  static constexpr int S = WPlan<N>::row_stride;
  static constexpr int W = R / WPlan<N>::T;
  static constexpr int kThreads = 64 * W;
  static constexpr size_t kLds = (size_t(N) + size_t(R) * S) * sizeof(cplx<T>);
};

// Forward row pass: fields (2q, 2q+1) of item z packed as one complex row, transformed along x2,
// unpacked into the transposed half spectra of fields 2q and 2q+1.
template <typename T, int N, typename TF>
__global__ void __launch_bounds__((FRow<T, N>::kThreads)) k_frow_fwd(RealFields<TF> in, cplx<T>* __restrict__ S, int n1,
                                                                   const cplx<T>* __restrict__ roots) {
  using PL = WPlan<N>;
  using RW = FRow<T, N>;
  constexpr int R = RW::R, nh = N / 2 + 1;
  constexpr int r1 = PL::radix(0), rL = PL::radix(PL::NS - 1);
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* rt = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* zb = rt + N;
  const int z = blockIdx.z;
  if (in.active && !in.active[z / in.item_div]) return;
  const int fa = 2 * blockIdx.y, fb = fa + 1;
  const int r0 = blockIdx.x * R;
  const TF* A = in.p[fa] + z * in.bstride[fa];
  const TF* B = fb < in.count ? in.p[fb] + z * in.bstride[fb] : nullptr;
  const int tid = threadIdx.x, lane = tid & 63;
  const int lp = lane % PL::LPT;
  const int row = (tid >> 6) * PL::T + lane / PL::LPT;
  const size_t gb = size_t(r0 + row) * N;
  cplx<T> x[PL::E];
#pragma unroll
  for (int m = 0; m < PL::E; ++m) {
    const int e = wmap<N, r1>(lp, m);
    x[m] = {T(A[gb + e]), B ? T(B[gb + e]) : T(0)};
  }
  fill_twiddles<T, N, false>(rt, roots, tid, RW::kThreads);
  __syncthreads();
  cplx<T>* reg = zb + row * RW::S;
  wave_fft<T, N, -1, false, false>(x, reg, rt, lp);
#pragma unroll
  for (int m = 0; m < PL::E; ++m) reg[PL::pos(wmap<N, rL>(lp, m))] = x[m];
  __syncthreads();
  const size_t sf = size_t(nh) * n1;
  cplx<T>* SA = S + (size_t(z) * in.count + fa) * sf + r0;
  cplx<T>* SB = S + (size_t(z) * in.count + fb) * sf + r0;
  for (int idx = tid; idx < nh * R; idx += RW::kThreads) {
    const int k = idx / R, rr = idx % R;
    const cplx<T>* zr = zb + rr * RW::S;
    const cplx<T> zk = zr[PL::pos(k)];
    const cplx<T> zm = cconj(zr[PL::pos(k == 0 ? 0 : N - k)]);
    const size_t o = size_t(k) * n1 + rr;
    SA[o] = cscale(cadd(zk, zm), T(0.5));
    if (B) SB[o] = cscale(cmul_mi(csub(zk, zm)), T(0.5));
  }
}

// Inverse row pass: transposed half spectra (2q, 2q+1) of item z -> real fields (plus addend).
// With CHEB the four fields (S Q y, S^2 Q y) are not stored: they complete the Chebyshev step in
// place (pair 0 updates r, d, x; pair 1 updates u, y; the arithmetic of cheb_step).
template <typename T, int N, bool CHEB, typename TF>
__global__ void __launch_bounds__((FRow<T, N>::kThreads)) k_frow_inv(const cplx<T>* __restrict__ S, int nspec,
                                                                   OutFields<TF> out, int n1,
                                                                   const cplx<T>* __restrict__ roots,
                                                                   ChebTail<T> ct) {
  using PL = WPlan<N>;
  using RW = FRow<T, N>;
  constexpr int R = RW::R, nh = N / 2 + 1;
  constexpr int r1 = PL::radix(0), rL = PL::radix(PL::NS - 1);
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* rt = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* zb = rt + N;
  const int z = blockIdx.z;
  if (out.active && !out.active[z / out.item_div]) return;
  const int fa = 2 * blockIdx.y, fb = fa + 1;
  const bool hasb = fb < out.count;
  const int r0 = blockIdx.x * R;
  const int tid = threadIdx.x, lane = tid & 63;
  const size_t sf = size_t(nh) * n1;
  const cplx<T>* SA = S + (size_t(z) * nspec + fa) * sf + r0;
  const cplx<T>* SB = S + (size_t(z) * nspec + fb) * sf + r0;
  fill_twiddles<T, N, false>(rt, roots, tid, RW::kThreads);
  // the loads of several iterations are issued before their LDS stores
#pragma unroll 4
  for (int idx = tid; idx < nh * R; idx += RW::kThreads) {
    const int k = idx / R, rr = idx % R;
    const size_t o = size_t(k) * n1 + rr;
    cplx<T> a = SA[o];
    cplx<T> b = hasb ? SB[o] : cplx<T>{T(0), T(0)};
    if (k == 0 || k == N / 2) {  // a real row's DC and Nyquist coefficients are real
      a.y = T(0);
      b.y = T(0);
    }
    cplx<T>* zr = zb + rr * RW::S;
    zr[PL::pos(k)] = cadd(a, cmul_i(b));
    if (k > 0 && k < N / 2) zr[PL::pos(N - k)] = cadd(cconj(a), cmul_i(cconj(b)));
  }
  __syncthreads();
  const int lp = lane % PL::LPT;
  const int row = (tid >> 6) * PL::T + lane / PL::LPT;
  cplx<T>* reg = zb + row * RW::S;
  cplx<T> x[PL::E];
#pragma unroll
  for (int m = 0; m < PL::E; ++m) x[m] = reg[PL::pos(wmap<N, r1>(lp, m))];
  wave_sync();
  wave_fft<T, N, +1, false, false>(x, reg, rt, lp);
  const size_t gb = size_t(r0 + row) * N;
  if constexpr (CHEB) {
    const T c1 = T(ct.c1[z]), c2 = T(ct.c2[z]);
    const size_t F = size_t(n1) * N;
    const size_t ib = size_t(z) * 2 * F + gb;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const size_t o = ib + c * F;
      if (blockIdx.y == 0) {
        T rv[PL::E], dv[PL::E], xv[PL::E];
#pragma unroll
        for (int m = 0; m < PL::E; ++m) {
          const int e = wmap<N, rL>(lp, m);
          rv[m] = ct.r[o + e];
          dv[m] = ct.d[o + e];
          xv[m] = ct.x[o + e];
        }
#pragma unroll
        for (int m = 0; m < PL::E; ++m) {
          const int e = wmap<N, rL>(lp, m);
          const T r = rv[m] - (dv[m] + (c ? x[m].y : x[m].x));
          const T d = c1 * dv[m] + c2 * r;
          ct.r[o + e] = r;
          ct.d[o + e] = d;
          ct.x[o + e] = xv[m] + d;
        }
      } else {
        T uv[PL::E], yv[PL::E];
#pragma unroll
        for (int m = 0; m < PL::E; ++m) {
          const int e = wmap<N, rL>(lp, m);
          uv[m] = ct.u[o + e];
          yv[m] = ct.y[o + e];
        }
#pragma unroll
        for (int m = 0; m < PL::E; ++m) {
          const int e = wmap<N, rL>(lp, m);
          const T u = uv[m] - (yv[m] + (c ? x[m].y : x[m].x));
          ct.u[o + e] = u;
          ct.y[o + e] = c1 * yv[m] + c2 * u;
        }
      }
    }
    return;
  }
  TF* OA = out.p[fa] + z * out.bstride[fa] + gb;
  TF* OB = hasb ? out.p[fb] + z * out.bstride[fb] + gb : nullptr;
  const TF* AA = out.add[fa] ? out.add[fa] + z * out.bstride[fa] + gb : nullptr;
  const TF* AB = hasb && out.add[fb] ? out.add[fb] + z * out.bstride[fb] + gb : nullptr;
  // addends loaded in full before the first store (the outputs may alias nothing, but the
  // compiler cannot know that, and would otherwise wait for each load in turn)
  if (AA) {
#pragma unroll
    for (int m = 0; m < PL::E; ++m) x[m].x += T(AA[wmap<N, rL>(lp, m)]);
  }
  if (AB) {
#pragma unroll
    for (int m = 0; m < PL::E; ++m) x[m].y += T(AB[wmap<N, rL>(lp, m)]);
  }
#pragma unroll
  for (int m = 0; m < PL::E; ++m) {
    const int e = wmap<N, rL>(lp, m);
    OA[e] = TF(x[m].x);
    if (OB) OB[e] = TF(x[m].y);
  }
}

template <typename T, int N>
struct FCol {
  static constexpr int W = 4;  // wavefronts per workgroup
  static constexpr int KR = W * WPlan<N>::T;  // rows k2 per workgroup
  static constexpr int S = WPlan<N>::col_stride;
  static constexpr int kThreads = 64 * W;
  static constexpr size_t kLds = (2 * size_t(N) + size_t(KR) * S) * sizeof(cplx<T>);
};

// Column pass over rows k2 of the transposed spectra of item z: forward transform along x1 (unless
// kInK: the input is k-space in the last-stage mapping), op at every (k1, k2), inverse transform
// (unless kOutK: the output stays k-space).  Each output is formed and transformed on its own, from
// the inputs held in registers.  With gridDim.y = NOUT (small grids) workgroup row y forms output
// y only, so that more wavefronts share the work (each repeats the forward transforms).
template <typename T, int N, class Op, int FL>
__global__ void __launch_bounds__(256) k_fcol(const cplx<T>* __restrict__ Sin, cplx<T>* __restrict__ Sout, int nh,
                                              Op op, const cplx<T>* __restrict__ roots, const int* active,
                                              int item_div) {
  using PL = WPlan<N>;
  using CW = FCol<T, N>;
  constexpr int NIN = Op::NIN, NOUT = Op::NOUT;
  constexpr int r1 = PL::radix(0), rL = PL::radix(PL::NS - 1);
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* rt = reinterpret_cast<cplx<T>*>(smem_raw);   // forward-order twiddles
  cplx<T>* rtr = rt + N;                                  // reversed-order twiddles
  cplx<T>* xb = rt + 2 * N;
  const int z = blockIdx.z;
  if (active && !active[z / item_div]) return;
  const int tid = threadIdx.x, lane = tid & 63;
  const int lp = lane % PL::LPT;
  const int slot = (tid >> 6) * PL::T + lane / PL::LPT;
  const int k2 = blockIdx.x * CW::KR + slot;
  const bool valid = k2 < nh;
  const int k2c = valid ? k2 : nh - 1;
  const size_t sf = size_t(nh) * N;
  cplx<T>* reg = xb + slot * CW::S;
  if constexpr (!(FL & kInK)) fill_twiddles<T, N, false>(rt, roots, tid, CW::kThreads);
  if constexpr (!(FL & kOutK)) fill_twiddles<T, N, true>(rtr, roots, tid, CW::kThreads);
  cplx<T> vin[NIN][PL::E];
#pragma unroll
  for (int f = 0; f < NIN; ++f) {
    const cplx<T>* src = Sin + (size_t(z) * NIN + f) * sf + size_t(k2c) * N;
#pragma unroll
    for (int m = 0; m < PL::E; ++m) vin[f][m] = src[(FL & kInK) ? wmap<N, rL>(lp, m) : wmap<N, r1>(lp, m)];
  }
  // per-wavenumber coefficients of the operator (symbols), formed once for all outputs while
  // the loads are in flight
  constexpr int NC = Op::NC > 0 ? Op::NC : 1;
  T cf[PL::E][NC];
  if constexpr (Op::NC > 0) {
#pragma unroll
    for (int m = 0; m < PL::E; ++m) {
      op.coef(signed_wavenumber(wmap<N, rL>(lp, m), N), k2c, cf[m]);
#pragma unroll
      for (int c = 0; c < NC; ++c) asm volatile("" : "+v"(cf[m][c]));
    }
  }
  __syncthreads();
  if constexpr (!(FL & kInK)) {
#pragma unroll
    for (int f = 0; f < NIN; ++f) wave_fft<T, N, -1, false, true>(vin[f], reg, rt, lp);
  }
  const bool all_out = gridDim.y == 1;
  if constexpr (Op::kPre) {
    if (valid && (all_out || blockIdx.y == 0)) {
#pragma unroll
      for (int m = 0; m < PL::E; ++m) {
        cplx<T> v[NIN];
#pragma unroll
        for (int f = 0; f < NIN; ++f) v[f] = vin[f][m];
        op.pre(signed_wavenumber(wmap<N, rL>(lp, m), N), k2, z, v);
      }
    }
  }
#pragma unroll
  for (int g = 0; g < NOUT; ++g) {
    if (!all_out && g != int(blockIdx.y)) continue;
    cplx<T> y[PL::E];
    int lpg = lp;
    asm volatile("" : "+v"(lpg));
#pragma unroll
    for (int m = 0; m < PL::E; ++m) {
      cplx<T> v[NIN];
#pragma unroll
      for (int f = 0; f < NIN; ++f) v[f] = vin[f][m];
      y[m] = op.out(g, signed_wavenumber(wmap<N, rL>(lpg, m), N), k2c, z, v, cf[m]);
    }
    cplx<T>* dst = Sout + (size_t(z) * NOUT + g) * sf + size_t(k2c) * N;
    if constexpr (!(FL & kOutK)) {
      wave_fft<T, N, +1, true, true>(y, reg, rtr, lp);
      if (valid) {
#pragma unroll
        for (int m = 0; m < PL::E; ++m) dst[wmap<N, r1>(lp, m)] = y[m];
      }
    } else {
      if (valid) {
#pragma unroll
        for (int m = 0; m < PL::E; ++m) dst[wmap<N, rL>(lp, m)] = y[m];
      }
    }
  }
}

// ---- symbols ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T odd_k(int k, int n) { return (2 * k == -n) ? T(0) : T(k); }  // Nyquist dropped

template <typename T>
__device__ __forceinline__ T spline_symbol(int k1, int n1, int k2, int n2) {
  const T b1 = (T(2) + cospi(T(2) * T(k1) / T(n1))) / T(3);
  const T b2 = (T(2) + cospi(T(2) * T(k2) / T(n2))) / T(3);
  return b1 * b2;
}

template <typename T>
__device__ __forceinline__ T reg_a(int k1, int k2, int reg) {
  const T q = T(k1) * T(k1) + T(k2) * T(k2);
  T a = q;
  for (int r = 1; r < reg; ++r) a *= q;
  return a;
}

template <typename T>
__device__ __forceinline__ T symbol_value(const SymbolParams& sp, int k1, int n1, int k2, int n2) {
  switch (sp.kind) {
    case Symbol::Reg:
      return T(sp.beta) * reg_a<T>(k1, k2, sp.reg);
    case Symbol::RegInv: {
      T a = reg_a<T>(k1, k2, sp.reg);
      if (a == T(0)) a = T(1);
      return T(1) / (T(sp.beta) * a);
    }
    case Symbol::RegInvSqrt: {
      T a = reg_a<T>(k1, k2, sp.reg);
      if (a == T(0)) a = T(1);
      return T(1) / sqrt(T(sp.beta) * a);
    }
    case Symbol::LowPass:
      return (4 * abs(k1) < n1 && 4 * abs(k2) < n2) ? T(1) : T(0);
    case Symbol::HighPass:
      return (4 * abs(k1) < n1 && 4 * abs(k2) < n2) ? T(0) : T(1);
    case Symbol::Cutoff:
      return (k1 * k1 + k2 * k2 <= sp.kmax * sp.kmax) ? T(1) : T(0);
    case Symbol::One:
      return T(1);
    case Symbol::Spline:
    default:
      return T(1) / spline_symbol<T>(k1, n1, k2, n2);
  }
}

// Every operator gives all outputs at one wavenumber (operator(), generic column pass) and output g
// alone (out(), wave-level column pass) from NC real coefficients per wavenumber that coef()
// forms once for all outputs; pre() is a side effect at each wavenumber, run once.
// Leray projection of the vector pair (a, b) at column index k1, half-spectrum index k2:
// (a, b) - k (k . (a, b)) / |k|^2 with the odd-order wavenumbers (Nyquist components zero)
template <typename T>
__device__ __forceinline__ void leray_pair(int k1, int n1, int k2, int n2, cplx<T>& a, cplx<T>& b) {
  const T o1 = odd_k<T>(k1, n1), o2 = (2 * k2 == n2) ? T(0) : T(k2);
  const T kk = o1 * o1 + o2 * o2;
  if (kk > T(0)) {
    const cplx<T> t = cscale(cadd(cscale(a, o1), cscale(b, o2)), T(1) / kk);
    a = csub(a, cscale(t, o1));
    b = csub(b, cscale(t, o2));
  }
}

template <typename T, int NF>
struct OpScale {
  static constexpr int NIN = NF, NOUT = NF, NC = 1;
  static constexpr bool kPre = false;
  SymbolParams sp;
  int n1, n2;
  double inv_n;
  __device__ void coef(int k1, int k2, T* c) const {
    const int k2s = (2 * k2 == n2) ? -k2 : k2;
    c[0] = symbol_value<T>(sp, k1, n1, k2s, n2) * T(inv_n);
  }
  __device__ void operator()(int k1, int k2, int, int, const cplx<T>* in, cplx<T>* out) const {
    T s;
    coef(k1, k2, &s);
    if constexpr (NF == 2) {
      if (sp.proj) {
        cplx<T> a = in[0], b = in[1];
        leray_pair<T>(k1, n1, k2, n2, a, b);
        out[0] = cscale(a, s);
        out[1] = cscale(b, s);
        return;
      }
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) out[f] = cscale(in[f], s);
  }
  __device__ void pre(int, int, int, const cplx<T>*) const {}
  __device__ cplx<T> out(int g, int k1, int k2, int, const cplx<T>* in, const T* c) const {
    if constexpr (NF == 2) {
      if (sp.proj) {
        cplx<T> a = in[0], b = in[1];
        leray_pair<T>(k1, n1, k2, n2, a, b);
        return cscale(g == 0 ? a : b, c[0]);
      }
    }
    return cscale(in[g], c[0]);
  }
};

// two symbols of the same two input fields: out[0..2) = sym1 in, out[2..4) = sym2 in
template <typename T>
struct OpScale2 {
  static constexpr int NIN = 2, NOUT = 4, NC = 2;
  static constexpr bool kPre = false;
  SymbolParams sp1, sp2;
  int n1, n2;
  double inv_n;
  __device__ void operator()(int k1, int k2, int, int, const cplx<T>* in, cplx<T>* out) const {
    const int k2s = (2 * k2 == n2) ? -k2 : k2;
    const T a = symbol_value<T>(sp1, k1, n1, k2s, n2) * T(inv_n);
    const T b = symbol_value<T>(sp2, k1, n1, k2s, n2) * T(inv_n);
    cplx<T> x = in[0], y = in[1];
    if (sp1.proj) leray_pair<T>(k1, n1, k2, n2, x, y);
    out[0] = cscale(x, a);
    out[1] = cscale(y, a);
    out[2] = cscale(x, b);
    out[3] = cscale(y, b);
  }
  __device__ void coef(int k1, int k2, T* c) const {
    const int k2s = (2 * k2 == n2) ? -k2 : k2;
    c[0] = symbol_value<T>(sp1, k1, n1, k2s, n2) * T(inv_n);
    c[1] = symbol_value<T>(sp2, k1, n1, k2s, n2) * T(inv_n);
  }
  __device__ void pre(int, int, int, const cplx<T>*) const {}
  __device__ cplx<T> out(int g, int k1, int k2, int, const cplx<T>* in, const T* c) const {
    if (sp1.proj) {
      cplx<T> x = in[0], y = in[1];
      leray_pair<T>(k1, n1, k2, n2, x, y);
      return cscale((g & 1) ? y : x, c[g >> 1]);
    }
    return cscale(in[g & 1], c[g >> 1]);
  }
};

template <typename T>
struct OpGrad {
  static constexpr int NIN = 1, NOUT = 2, NC = 0;
  static constexpr bool kPre = false;
  int n1, n2;
  double inv_n;
  __device__ void operator()(int k1, int k2, int, int, const cplx<T>* in, cplx<T>* out) const {
    const T s = T(inv_n);
    out[0] = cmul_i(cscale(in[0], odd_k<T>(k1, n1) * s));
    out[1] = cmul_i(cscale(in[0], (2 * k2 == n2 ? T(0) : T(k2)) * s));
  }
  __device__ void coef(int, int, T*) const {}
  __device__ void pre(int, int, int, const cplx<T>*) const {}
  __device__ cplx<T> out(int g, int k1, int k2, int, const cplx<T>* in, const T*) const {
    const T k = g == 0 ? odd_k<T>(k1, n1) : (2 * k2 == n2 ? T(0) : T(k2));
    return cmul_i(cscale(in[0], k * T(inv_n)));
  }
};

template <typename T>
struct OpDiv {
  static constexpr int NIN = 2, NOUT = 1, NC = 0;
  static constexpr bool kPre = false;
  int n1, n2;
  double inv_n;
  __device__ cplx<T> div(int k1, int k2, const cplx<T>* in) const {
    const T o1 = odd_k<T>(k1, n1), o2 = (2 * k2 == n2) ? T(0) : T(k2);
    return cscale(cmul_i(cadd(cscale(in[0], o1), cscale(in[1], o2))), T(inv_n));
  }
  __device__ void operator()(int k1, int k2, int, int, const cplx<T>* in, cplx<T>* out) const {
    out[0] = div(k1, k2, in);
  }
  __device__ void coef(int, int, T*) const {}
  __device__ void pre(int, int, int, const cplx<T>*) const {}
  __device__ cplx<T> out(int, int k1, int k2, int, const cplx<T>* in, const T*) const { return div(k1, k2, in); }
};

// Spatial derivatives of one stabilised RK2 stage: from the spectra of (u, w1, w2) the spectra of
// (d1 u, d2 u, d1 w1 + d2 w2), odd-order wavenumbers (Nyquist dropped).
template <typename T>
struct OpRK2A {
  static constexpr int NIN = 3, NOUT = 3, NC = 0;
  static constexpr bool kPre = false;
  int n1, n2;
  double inv_n;
  __device__ cplx<T> der(int g, int k1, int k2, const cplx<T>* in) const {
    const T o1 = odd_k<T>(k1, n1), o2 = (2 * k2 == n2) ? T(0) : T(k2);
    const cplx<T> d = g == 0 ? cscale(in[0], o1) : g == 1 ? cscale(in[0], o2)
                                                         : cadd(cscale(in[1], o1), cscale(in[2], o2));
    return cscale(cmul_i(d), T(inv_n));
  }
  __device__ void operator()(int k1, int k2, int, int, const cplx<T>* in, cplx<T>* out) const {
#pragma unroll
    for (int g = 0; g < 3; ++g) out[g] = der(g, k1, k2, in);
  }
  __device__ void coef(int, int, T*) const {}
  __device__ void pre(int, int, int, const cplx<T>*) const {}
  __device__ cplx<T> out(int g, int k1, int k2, int, const cplx<T>* in, const T*) const { return der(g, k1, k2, in); }
};

template <typename T>
struct OpTracePrep {
  static constexpr int NIN = 2, NOUT = 4, NC = 1;  // cv1, cv2, div v, c_div
  static constexpr bool kPre = false;
  int n1, n2;
  double inv_n;
  __device__ void operator()(int k1, int k2, int, int, const cplx<T>* in, cplx<T>* out) const {
    const int k2s = (2 * k2 == n2) ? -k2 : k2;
    const T s = T(inv_n);
    const T ib = s / spline_symbol<T>(k1, n1, k2s, n2);
    const T o1 = odd_k<T>(k1, n1), o2 = (2 * k2 == n2) ? T(0) : T(k2);
    const cplx<T> d = cmul_i(cadd(cscale(in[0], o1), cscale(in[1], o2)));
    out[0] = cscale(in[0], ib);
    out[1] = cscale(in[1], ib);
    out[2] = cscale(d, s);
    out[3] = cscale(d, ib);
  }
  __device__ void coef(int k1, int k2, T* c) const {
    const int k2s = (2 * k2 == n2) ? -k2 : k2;
    c[0] = T(inv_n) / spline_symbol<T>(k1, n1, k2s, n2);
  }
  __device__ void pre(int, int, int, const cplx<T>*) const {}
  __device__ cplx<T> out(int g, int k1, int k2, int, const cplx<T>* in, const T* c) const {
    if (g < 2) return cscale(in[g], c[0]);
    const T o1 = odd_k<T>(k1, n1), o2 = (2 * k2 == n2) ? T(0) : T(k2);
    return cscale(cmul_i(cadd(cscale(in[0], o1), cscale(in[1], o2))), g == 2 ? T(inv_n) : c[0]);
  }
};

// k-space identity (used for coarse forward transforms and coarse inverse transforms)
template <typename T, int NF>
struct OpCopy {
  static constexpr int NIN = NF, NOUT = NF, NC = 0;
  static constexpr bool kPre = false;
  __device__ void operator()(int, int, int, int, const cplx<T>* in, cplx<T>* out) const {
#pragma unroll
    for (int f = 0; f < NF; ++f) out[f] = in[f];
  }
  __device__ void coef(int, int, T*) const {}
  __device__ void pre(int, int, int, const cplx<T>*) const {}
  __device__ cplx<T> out(int g, int, int, int, const cplx<T>* in, const T*) const { return in[g]; }
};

// Position of coarse mode (e, k2) of field f of item z in the coarse k-space buffer: rows of the
// half spectrum [nc1][nch] (generic passes) or its transpose [nc2 / 2 + 1][nc1] (wave passes).
__device__ __forceinline__ size_t coarse_at(bool tr, int z, int NF, int f, int e, int k2, int nc1, int nc2) {
  if (tr) return ((size_t(z) * NF + f) * size_t(nc2 / 2 + 1) + k2) * nc1 + e;
  const int nch = spec_stride(nc2);
  return ((size_t(z) * NF + f) * nc1 + e) * nch + k2;
}

// Restriction: writes the surviving modes of the fine spectrum (scaled by 1/N_fine so that the
// coarse inverse needs no further scale) into the coarse k-space buffer, and keeps the fine
// spectrum (output, k-space) when asked.
template <typename T, int NF>
struct OpRestrict {
  static constexpr int NIN = NF, NOUT = NF, NC = 0;
  static constexpr bool kPre = true;
  cplx<T>* coarse;   // [z][NF] coarse k-space spectra (layout: coarse_at)
  int n1, n2, nc1, nc2;
  double inv_n;
  int tr;
  __device__ void pre(int k1, int k2, int z, const cplx<T>* in) const {
    if (4 * abs(k1) < n1 && 4 * k2 < n2) {
      const int e = k1 < 0 ? k1 + nc1 : k1;
#pragma unroll
      for (int f = 0; f < NF; ++f) coarse[coarse_at(tr, z, NF, f, e, k2, nc1, nc2)] = cscale(in[f], T(inv_n));
    } else if (abs(k1) <= nc1 / 2 && k2 <= nc2 / 2) {
      // coarse Nyquist row/column: dropped
      const int e = k1 < 0 ? k1 + nc1 : k1;
      if (e < nc1) {
#pragma unroll
        for (int f = 0; f < NF; ++f) coarse[coarse_at(tr, z, NF, f, e, k2, nc1, nc2)] = {T(0), T(0)};
      }
    }
  }
  __device__ void operator()(int k1, int k2, int, int z, const cplx<T>* in, cplx<T>* out) const {
    pre(k1, k2, z, in);
#pragma unroll
    for (int f = 0; f < NF; ++f) out[f] = in[f];
  }
  __device__ void coef(int, int, T*) const {}
  __device__ cplx<T> out(int g, int, int, int, const cplx<T>* in, const T*) const { return in[g]; }
};

// Two-level combine (input: kept fine spectrum, k-space): high-pass part of it plus the
// zero-padded coarse spectrum; 1/N_fine for the fine inverse, N_fine/N_coarse for the padding.
template <typename T, int NF>
struct OpProlongCombine {
  static constexpr int NIN = NF, NOUT = NF, NC = 0;
  static constexpr bool kPre = false;
  const cplx<T>* coarse;   // [z][NF] coarse k-space spectra (forward transform, unnormalised)
  int n1, n2, nc1, nc2;
  double inv_n, inv_nc;
  int tr;
  __device__ void coef(int, int, T*) const {}
  __device__ cplx<T> out(int g, int k1, int k2, int z, const cplx<T>* in, const T* = nullptr) const {
    if (4 * abs(k1) < n1 && 4 * k2 < n2) {
      const int e = k1 < 0 ? k1 + nc1 : k1;
      return cscale(coarse[coarse_at(tr, z, NF, g, e, k2, nc1, nc2)], T(inv_nc));
    }
    return cscale(in[g], T(inv_n));
  }
  __device__ void operator()(int k1, int k2, int, int z, const cplx<T>* in, cplx<T>* out_) const {
#pragma unroll
    for (int f = 0; f < NF; ++f) out_[f] = out(f, k1, k2, z, in);
  }
  __device__ void pre(int, int, int, const cplx<T>*) const {}
};

// ---------------------------------------------------------------------------------------
// launch helpers
// ---------------------------------------------------------------------------------------
#define RET_IF(e)                  \
  do {                             \
    hipError_t _e = (e);           \
    if (_e != hipSuccess) return _e; \
  } while (0)

inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

// about 8 elements per thread (one radix-8 butterfly per stage), at least one wavefront
template <typename T>
void row_config(int n2, int& nthr, int& rpb) {
  nthr = std::min(256, std::max(64, round_up(n2 / 8, 64)));
  rpb = std::max(1, (nthr * 8) / n2);
  while (rpb * n2 > nthr * kMaxE) --rpb;
}

template <typename T, typename TF>
hipError_t launch_row_fwd(hipStream_t s, const SpecGrid<T>& g, RealFields<TF> in, int batch, cplx<T>* S) {
  int nthr, rpb;
  row_config<T>(g.n2, nthr, rpb);
  dim3 grid((g.n1 + rpb - 1) / rpb, (in.count + 1) / 2, batch);
  size_t lds = (size_t(rpb) * lds_stride(g.n2) + g.n2) * sizeof(cplx<T>);
  static std::atomic<size_t> allowed{0};
  RET_IF(allow_lds(k_row_fwd<T, TF>, lds, allowed));
  hipLaunchKernelGGL((k_row_fwd<T, TF>), grid, dim3(nthr), lds, s, in, S, g.n1, g.n2, rpb, g.row);
  return hipGetLastError();
}

template <typename T, typename TF>
hipError_t launch_row_inv(hipStream_t s, const SpecGrid<T>& g, const cplx<T>* S, int nspec, OutFields<TF> out,
                          int batch) {
  int nthr, rpb;
  row_config<T>(g.n2, nthr, rpb);
  dim3 grid((g.n1 + rpb - 1) / rpb, (out.count + 1) / 2, batch);
  size_t lds = (size_t(rpb) * lds_stride(g.n2) + g.n2) * sizeof(cplx<T>);
  static std::atomic<size_t> allowed{0};
  RET_IF(allow_lds(k_row_inv<T, TF>, lds, allowed));
  hipLaunchKernelGGL((k_row_inv<T, TF>), grid, dim3(nthr), lds, s, S, nspec, out, g.n1, g.n2, rpb, g.row);
  return hipGetLastError();
}

// Column pass shape: B adjacent columns per block.  Small grids keep the block count up (B from
// nh / 64); when the batch already gives enough blocks, B grows to what the LDS budget allows,
// so that each row of a panel is a longer contiguous segment (8 columns: 64 bytes in FP32).
// Every FFT stage stays within kMaxE elements per thread at <= 1024 threads.
template <typename T>
void col_config(int n1, int nh, int nmax, int batch, int& B, int& nthr, size_t& lds) {
  const int col_bytes = lds_stride(n1) * int(sizeof(cplx<T>)) * nmax;
  const int bmax = std::max(1, std::min(16, kLdsBudget / col_bytes));
  B = std::max(1, std::min(std::min(16, std::max(1, nh / 64)), bmax));
  while (B < bmax && ((nh + 2 * B - 1) / (2 * B)) * batch >= 512) B *= 2;
  B = std::min(B, bmax);
  while (B > 1 && nmax * B * n1 > 1024 * kMaxE) --B;
  const int elems = nmax * B * n1;
  nthr = std::min(1024, std::max(64, round_up((elems + 7) / 8, 64)));
  while (nthr < 1024 && elems > nthr * kMaxE) nthr += 64;
  lds = size_t(B) * col_bytes + size_t(n1) * sizeof(cplx<T>);
}

template <typename T, class Op>
hipError_t launch_col(hipStream_t s, const SpecGrid<T>& g, const cplx<T>* Sin, cplx<T>* Sout, Op op, int flags,
                      int batch, const int* active = nullptr, int item_div = 1) {
  constexpr int nmax = Op::NIN > Op::NOUT ? Op::NIN : Op::NOUT;
  const int nh = g.nh();
  int B, nthr;
  size_t lds;
  col_config<T>(g.n1, nh, nmax, batch, B, nthr, lds);
  dim3 grid((nh + B - 1) / B, 1, batch);
  static std::atomic<size_t> allowed{0};
  RET_IF(allow_lds(k_col<T, Op>, lds, allowed));
  hipLaunchKernelGGL((k_col<T, Op>), grid, dim3(nthr), lds, s, Sin, Sout, g.n1, g.n2, B, g.col, op, flags, active,
                     item_div);
  return hipGetLastError();
}


// ---- wave-level launchers ----------------------------------------------------------------
bool fast_len(int n) {
  switch (n) {
    case 64: case 96: case 128: case 192: case 256: case 384: case 512: case 768: case 1024:
      return true;
  }
  return false;
}

// the wave-level passes serve a grid when both lengths are common ones (the row passes take
// rows in groups of at most 16, and every such n1 is a multiple of 16)
template <typename T>
bool fast_grid(const SpecGrid<T>& g) {
  return fast_len(g.n1) && fast_len(g.n2) && g.row.roots && g.col.roots;
}

#define SLNK_FAST_CASES(X) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) X(1024)

template <typename T, int N, typename TF>
hipError_t launch_frow_fwd_n(hipStream_t s, const SpecGrid<T>& g, RealFields<TF> in, int batch, cplx<T>* S) {
  using RW = FRow<T, N>;
  static std::atomic<size_t> allowed{0};
  RET_IF(allow_lds(k_frow_fwd<T, N, TF>, RW::kLds, allowed));
  dim3 grid(g.n1 / RW::R, (in.count + 1) / 2, batch);
  hipLaunchKernelGGL((k_frow_fwd<T, N, TF>), grid, dim3(RW::kThreads), RW::kLds, s, in, S, g.n1,
                     static_cast<const cplx<T>*>(g.row.roots));
  return hipGetLastError();
}

template <typename T, int N, bool CHEB = false, typename TF = T>
hipError_t launch_frow_inv_n(hipStream_t s, const SpecGrid<T>& g, const cplx<T>* S, int nspec, OutFields<TF> out,
                             int batch, ChebTail<T> ct = {}) {
  using RW = FRow<T, N>;
  static std::atomic<size_t> allowed{0};
  RET_IF(allow_lds(k_frow_inv<T, N, CHEB, TF>, RW::kLds, allowed));
  dim3 grid(g.n1 / RW::R, (out.count + 1) / 2, batch);
  hipLaunchKernelGGL((k_frow_inv<T, N, CHEB, TF>), grid, dim3(RW::kThreads), RW::kLds, s, S, nspec, out, g.n1,
                     static_cast<const cplx<T>*>(g.row.roots), ct);
  return hipGetLastError();
}

template <typename T, int N, class Op, int FL>
hipError_t launch_fcol_n(hipStream_t s, const SpecGrid<T>& g, const cplx<T>* Sin, cplx<T>* Sout, Op op, int batch,
                         const int* active, int item_div) {
  using CW = FCol<T, N>;
  static std::atomic<size_t> allowed{0};
  RET_IF(allow_lds(k_fcol<T, N, Op, FL>, CW::kLds, allowed));
  const int nh = g.nh();
  const int blocks = (nh + CW::KR - 1) / CW::KR;
  // grids of fewer than a workgroup per compute unit split the outputs over grid rows
  const int ysplit = (Op::NOUT > 1 && long(blocks) * batch < 256) ? Op::NOUT : 1;
  dim3 grid(blocks, ysplit, batch);
  hipLaunchKernelGGL((k_fcol<T, N, Op, FL>), grid, dim3(CW::kThreads), CW::kLds, s, Sin, Sout, nh, op,
                     static_cast<const cplx<T>*>(g.col.roots), active, item_div);
  return hipGetLastError();
}

// Pass dispatch: wave-level passes (transposed spectra) when 'fast', else the generic ones.
template <typename T, typename TF>
hipError_t row_fwd(bool fast, hipStream_t s, const SpecGrid<T>& g, RealFields<TF> in, int batch, cplx<T>* S) {
  if (!fast) return launch_row_fwd<T, TF>(s, g, in, batch, S);
  switch (g.n2) {
#define X(N) \
  case N:    \
    return launch_frow_fwd_n<T, N, TF>(s, g, in, batch, S);
    SLNK_FAST_CASES(X)
#undef X
  }
  return hipErrorInvalidValue;
}

template <typename T, typename TF>
hipError_t row_inv(bool fast, hipStream_t s, const SpecGrid<T>& g, const cplx<T>* S, int nspec, OutFields<TF> out,
                   int batch) {
  if (!fast) return launch_row_inv<T, TF>(s, g, S, nspec, out, batch);
  switch (g.n2) {
#define X(N) \
  case N:    \
    return launch_frow_inv_n<T, N, false, TF>(s, g, S, nspec, out, batch);
    SLNK_FAST_CASES(X)
#undef X
  }
  return hipErrorInvalidValue;
}

template <int FL, typename T, class Op>
hipError_t col(bool fast, hipStream_t s, const SpecGrid<T>& g, const cplx<T>* Sin, cplx<T>* Sout, Op op, int batch,
               const int* active = nullptr, int item_div = 1) {
  if (!fast) return launch_col<T>(s, g, Sin, Sout, op, FL, batch, active, item_div);
  switch (g.n1) {
#define X(N) \
  case N:    \
    return launch_fcol_n<T, N, Op, FL>(s, g, Sin, Sout, op, batch, active, item_div);
    SLNK_FAST_CASES(X)
#undef X
  }
  return hipErrorInvalidValue;
}

// fields f < nf of a per-item block of nf consecutive fields
template <typename T, class FL>
void set_fields(FL& fl, int nf, T* base, size_t F, const int* active) {
  fl.count = nf;
  fl.active = active;
  fl.item_div = 1;
  for (int f = 0; f < nf; ++f) {
    fl.p[f] = base + f * F;
    fl.bstride[f] = (long long)(nf * F);
  }
}

}  // namespace

template <typename T>
size_t spec_lds_bytes(int n1, int n2) {
  int nthr, rpb, B;
  row_config<T>(n2, nthr, rpb);
  const size_t row = (size_t(rpb) * lds_stride(n2) + n2) * sizeof(cplx<T>);
  size_t col = 0;
  col_config<T>(n1, n2 / 2 + 1, 4, 1 << 20, B, nthr, col);  // widest operator, widest panel
  return std::max(row, col);
}

template <typename T, typename TF>
hipError_t spec_scale(hipStream_t s, const SpecGrid<T>& g, int batch, const int* active, SymbolParams sym, int nf,
                      const TF* in, TF* out, const typename NoDeduce<TF>::type* add, cplx<T>* S1, cplx<T>* S2) {
  const size_t F = g.field();
  const bool fast = fast_grid(g);
  RealFields<TF> rin{};
  set_fields(rin, nf, const_cast<TF*>(in), F, active);
  OutFields<TF> rout{};
  set_fields(rout, nf, out, F, active);
  for (int f = 0; f < nf; ++f) rout.add[f] = add ? add + f * F : nullptr;
  RET_IF((row_fwd<T, TF>(fast, s, g, rin, batch, S1)));
  const double inv_n = 1.0 / double(F);
  if (nf == 1) {
    OpScale<T, 1> op{sym, g.n1, g.n2, inv_n};
    RET_IF(col<0>(fast, s, g, S1, S2, op, batch, active));
  } else {
    OpScale<T, 2> op{sym, g.n1, g.n2, inv_n};
    RET_IF(col<0>(fast, s, g, S1, S2, op, batch, active));
  }
  return row_inv<T, TF>(fast, s, g, S2, nf, rout, batch);
}

template <typename T>
hipError_t spec_grad(hipStream_t s, const SpecGrid<T>& g, int count, const T* m, T* gm, cplx<T>* S1, cplx<T>* S2) {
  const size_t F = g.field();
  const bool fast = fast_grid(g);
  RealFields<T> rin{};
  rin.count = 1;
  rin.p[0] = m;
  rin.bstride[0] = (long long)F;
  rin.item_div = 1;
  RET_IF(row_fwd<T>(fast, s, g, rin, count, S1));
  OpGrad<T> op{g.n1, g.n2, 1.0 / double(F)};
  RET_IF(col<0>(fast, s, g, S1, S2, op, count));
  OutFields<T> rout{};
  rout.count = 2;
  rout.p[0] = gm;
  rout.p[1] = gm + F;
  rout.bstride[0] = rout.bstride[1] = (long long)(2 * F);
  rout.item_div = 1;
  return row_inv<T>(fast, s, g, S2, 2, rout, count);
}

template <typename T>
hipError_t spec_div(hipStream_t s, const SpecGrid<T>& g, int count, const T* w, T* out, cplx<T>* S1, cplx<T>* S2) {
  const size_t F = g.field();
  const bool fast = fast_grid(g);
  RealFields<T> rin{};
  set_fields(rin, 2, const_cast<T*>(w), F, nullptr);
  RET_IF(row_fwd<T>(fast, s, g, rin, count, S1));
  OpDiv<T> op{g.n1, g.n2, 1.0 / double(F)};
  RET_IF(col<0>(fast, s, g, S1, S2, op, count));
  OutFields<T> rout{};
  rout.count = 1;
  rout.p[0] = out;
  rout.bstride[0] = (long long)F;
  rout.item_div = 1;
  return row_inv<T>(fast, s, g, S2, 1, rout, count);
}

template <typename T>
hipError_t spec_rk2a(hipStream_t s, const SpecGrid<T>& g, int count, const T* in, T* out, cplx<T>* S1, cplx<T>* S2) {
  const size_t F = g.field();
  const bool fast = fast_grid(g);
  RealFields<T> rin{};
  set_fields(rin, 3, const_cast<T*>(in), F, nullptr);
  RET_IF(row_fwd<T>(fast, s, g, rin, count, S1));
  OpRK2A<T> op{g.n1, g.n2, 1.0 / double(F)};
  RET_IF(col<0>(fast, s, g, S1, S2, op, count));
  OutFields<T> rout{};
  set_fields(rout, 3, out, F, nullptr);
  return row_inv<T>(fast, s, g, S2, 3, rout, count);
}

template <typename T>
hipError_t spec_trace_prep(hipStream_t s, const SpecGrid<T>& g, int batch, const int* active, const T* v, T* cv,
                           T* divv, T* cdiv, cplx<T>* S1, cplx<T>* S2) {
  const size_t F = g.field();
  const bool fast = fast_grid(g);
  RealFields<T> rin{};
  set_fields(rin, 2, const_cast<T*>(v), F, active);
  RET_IF(row_fwd<T>(fast, s, g, rin, batch, S1));
  OpTracePrep<T> op{g.n1, g.n2, 1.0 / double(F)};
  RET_IF(col<0>(fast, s, g, S1, S2, op, batch, active));
  OutFields<T> rout{};
  rout.count = 4;
  rout.active = active;
  rout.item_div = 1;
  rout.p[0] = cv;
  rout.p[1] = cv + F;
  rout.p[2] = divv;
  rout.p[3] = cdiv;
  rout.bstride[0] = rout.bstride[1] = (long long)(2 * F);
  rout.bstride[2] = rout.bstride[3] = (long long)F;
  return row_inv<T>(fast, s, g, S2, 4, rout, batch);
}

template <typename T>
hipError_t spec_scale2(hipStream_t s, const SpecGrid<T>& g, int batch, const int* active, SymbolParams sym1,
                       SymbolParams sym2, const T* in, T* out1, T* out2, cplx<T>* S1, cplx<T>* S2) {
  const size_t F = g.field();
  const bool fast = fast_grid(g);
  RealFields<T> rin{};
  set_fields(rin, 2, const_cast<T*>(in), F, active);
  RET_IF(row_fwd<T>(fast, s, g, rin, batch, S1));
  OpScale2<T> op{sym1, sym2, g.n1, g.n2, 1.0 / double(F)};
  RET_IF(col<0>(fast, s, g, S1, S2, op, batch, active));
  OutFields<T> rout{};
  rout.count = 4;
  rout.active = active;
  rout.item_div = 1;
  rout.p[0] = out1;
  rout.p[1] = out1 + F;
  rout.p[2] = out2;
  rout.p[3] = out2 + F;
  rout.bstride[0] = rout.bstride[1] = rout.bstride[2] = rout.bstride[3] = (long long)(2 * F);
  return row_inv<T>(fast, s, g, S2, 4, rout, batch);
}

template <typename T>
bool spec_fast(const SpecGrid<T>& g) {
  return fast_grid(g);
}

template <typename T>
hipError_t spec_scale2_cheb(hipStream_t s, const SpecGrid<T>& g, int batch, const int* active, SymbolParams sym1,
                            SymbolParams sym2, const T* in, ChebTail<T> ct, cplx<T>* S1, cplx<T>* S2) {
  if (!fast_grid(g)) return hipErrorNotSupported;
  RealFields<T> rin{};
  set_fields(rin, 2, const_cast<T*>(in), g.field(), active);
  RET_IF(row_fwd<T>(true, s, g, rin, batch, S1));
  OpScale2<T> op{sym1, sym2, g.n1, g.n2, 1.0 / double(g.field())};
  RET_IF(col<0>(true, s, g, S1, S2, op, batch, active));
  OutFields<T> rout{};
  rout.count = 4;
  rout.active = active;
  rout.item_div = 1;
  switch (g.n2) {
#define X(N) \
  case N:    \
    return launch_frow_inv_n<T, N, true>(s, g, S2, 4, rout, batch, ct);
    SLNK_FAST_CASES(X)
#undef X
  }
  return hipErrorInvalidValue;
}

// The fine and the coarse passes of a restriction or prolongation share the coarse k-space buffer
// (and the kept fine spectrum), so both grids take the same kind of pass.
template <typename T>
hipError_t spec_restrict(hipStream_t s, const SpecGrid<T>& g, const SpecGrid<T>& gc, int batch, const int* active,
                         int nf, const T* in, T* out_c, cplx<T>* keep_fine, cplx<T>* S1, cplx<T>* Sc1, cplx<T>* Sc2) {
  const size_t F = g.field(), Fc = gc.field();
  const bool fast = fast_grid(g) && fast_grid(gc);
  RealFields<T> rin{};
  set_fields(rin, nf, const_cast<T*>(in), F, active);
  RET_IF((row_fwd<T>(fast, s, g, rin, batch, S1)));
  const double inv_n = 1.0 / double(F);
  // the fine column pass only writes the coarse k-space (and keeps the fine spectrum if asked)
  if (nf == 1) {
    OpRestrict<T, 1> op{Sc1, g.n1, g.n2, gc.n1, gc.n2, inv_n, fast ? 1 : 0};
    RET_IF(col<kOutK>(fast, s, g, S1, keep_fine ? keep_fine : S1, op, batch, active));
    RET_IF(col<kInK>(fast, s, gc, Sc1, Sc2, OpCopy<T, 1>{}, batch, active));
  } else {
    OpRestrict<T, 2> op{Sc1, g.n1, g.n2, gc.n1, gc.n2, inv_n, fast ? 1 : 0};
    RET_IF(col<kOutK>(fast, s, g, S1, keep_fine ? keep_fine : S1, op, batch, active));
    RET_IF(col<kInK>(fast, s, gc, Sc1, Sc2, OpCopy<T, 2>{}, batch, active));
  }
  OutFields<T> rout{};
  set_fields(rout, nf, out_c, Fc, active);
  return row_inv<T>(fast, s, gc, Sc2, nf, rout, batch);
}

template <typename T>
hipError_t spec_prolong_combine(hipStream_t s, const SpecGrid<T>& g, const SpecGrid<T>& gc, int batch,
                                const int* active, int nf, const cplx<T>* fine_k, const T* zc, T* out, cplx<T>* S1,
                                cplx<T>* Sc1, cplx<T>* Sc2) {
  const size_t F = g.field(), Fc = gc.field();
  const bool fast = fast_grid(g) && fast_grid(gc);
  RealFields<T> rin{};
  set_fields(rin, nf, const_cast<T*>(zc), Fc, active);
  RET_IF(row_fwd<T>(fast, s, gc, rin, batch, Sc1));
  if (nf == 1) {
    RET_IF(col<kOutK>(fast, s, gc, Sc1, Sc2, OpCopy<T, 1>{}, batch, active));
    OpProlongCombine<T, 1> op{Sc2, g.n1, g.n2, gc.n1, gc.n2, 1.0 / double(F), 1.0 / double(Fc), fast ? 1 : 0};
    RET_IF(col<kInK>(fast, s, g, fine_k, S1, op, batch, active));
  } else {
    RET_IF(col<kOutK>(fast, s, gc, Sc1, Sc2, OpCopy<T, 2>{}, batch, active));
    OpProlongCombine<T, 2> op{Sc2, g.n1, g.n2, gc.n1, gc.n2, 1.0 / double(F), 1.0 / double(Fc), fast ? 1 : 0};
    RET_IF(col<kInK>(fast, s, g, fine_k, S1, op, batch, active));
  }
  OutFields<T> rout{};
  set_fields(rout, nf, out, F, active);
  return row_inv<T>(fast, s, g, S1, nf, rout, batch);
}

#define INST(T)                                                                                                 \
  template size_t spec_lds_bytes<T>(int, int);                                                                  \
  template hipError_t spec_scale<T, T>(hipStream_t, const SpecGrid<T>&, int, const int*, SymbolParams, int,      \
                                       const T*, T*, const T*, cplx<T>*, cplx<T>*);                             \
  template hipError_t spec_grad<T>(hipStream_t, const SpecGrid<T>&, int, const T*, T*, cplx<T>*, cplx<T>*);     \
  template hipError_t spec_scale2<T>(hipStream_t, const SpecGrid<T>&, int, const int*, SymbolParams, SymbolParams, \
                                     const T*, T*, T*, cplx<T>*, cplx<T>*);                                     \
  template bool spec_fast<T>(const SpecGrid<T>&);                                                                \
  template hipError_t spec_div<T>(hipStream_t, const SpecGrid<T>&, int, const T*, T*, cplx<T>*, cplx<T>*);      \
  template hipError_t spec_rk2a<T>(hipStream_t, const SpecGrid<T>&, int, const T*, T*, cplx<T>*, cplx<T>*);     \
  template hipError_t spec_scale2_cheb<T>(hipStream_t, const SpecGrid<T>&, int, const int*, SymbolParams,       \
                                          SymbolParams, const T*, ChebTail<T>, cplx<T>*, cplx<T>*);             \
  template hipError_t spec_trace_prep<T>(hipStream_t, const SpecGrid<T>&, int, const int*, const T*, T*, T*, T*, \
                                         cplx<T>*, cplx<T>*);                                                   \
  template hipError_t spec_restrict<T>(hipStream_t, const SpecGrid<T>&, const SpecGrid<T>&, int, const int*, int, \
                                       const T*, T*, cplx<T>*, cplx<T>*, cplx<T>*, cplx<T>*);                   \
  template hipError_t spec_prolong_combine<T>(hipStream_t, const SpecGrid<T>&, const SpecGrid<T>&, int,         \
                                              const int*, int, const cplx<T>*, const T*, T*, cplx<T>*, cplx<T>*, \
                                              cplx<T>*);
#ifdef SLNK_SPECTRAL_REAL
INST(SLNK_SPECTRAL_REAL)
#endif
#undef INST

}  // namespace slnk
