// Shared device/host definitions of the MI355X (gfx950) semi-Lagrangian Newton--Krylov path.
//
// Conventions: a scalar field is a row-major [n1][n2] array (i2 fastest) on the periodic
// grid x_i = 2 pi i / n of [0, 2 pi)^2; a vector field is two consecutive scalar fields.
// 'Real' is float (mixed precision: fields in FP32, reductions in FP64) or double.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace slnk {

template <typename R>
struct alignas(2 * sizeof(R)) cplx {
  R x, y;
};

template <typename R>
__device__ __forceinline__ cplx<R> cmul(cplx<R> a, cplx<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename R>
__device__ __forceinline__ cplx<R> cadd(cplx<R> a, cplx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ cplx<R> csub(cplx<R> a, cplx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__device__ __forceinline__ cplx<R> cscale(cplx<R> a, R s) { return {a.x * s, a.y * s}; }
template <typename R>
__device__ __forceinline__ cplx<R> cconj(cplx<R> a) { return {a.x, -a.y}; }
// multiply by +i / -i
template <typename R>
__device__ __forceinline__ cplx<R> cmul_i(cplx<R> a) { return {-a.y, a.x}; }
template <typename R>
__device__ __forceinline__ cplx<R> cmul_mi(cplx<R> a) { return {a.y, -a.x}; }

__host__ __device__ __forceinline__ int wrap_index(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

// R consecutive outputs o[j] = sum_{|t| <= K} tap(t) x[K + j + t] of the truncated exponential
// filter of the periodic cubic B-spline prefilter (tap(t) = tap(0) z^t, z = sqrt(3) - 2) from a
// window x of R + 2K values.  The causal half P_j = sum_{t=0..K} tap(t) x[K + j - t] of the first
// output and the anticausal half Q_j = sum_{t=1..K} tap(t) x[K + j + t] of the last are summed
// directly; the others follow from the first-order recursions of the exponential taps, which keep
// the truncation exactly:
//   P_{j+1} = tap(0) x[K+j+1] + z P_j - z tap(K) x[j],  Q_j = z (tap(0) x[K+j+1] + Q_{j+1}) - z tap(K) x[2K+j+1]
// (|z| < 0.27, so rounding errors decay along the recursion).  About (2K + 3R) / R operations per
// output instead of 2K + 1.
template <typename T, int R, int K, class Tap>
__device__ __forceinline__ void filter_window_rec(const T* x, T* o, Tap tap) {
  const T z = T(-0.26794919243112270647);
  const T t0 = tap(0), zK = z * tap(K);
  T q[R];
  T acc = T(0);
#pragma unroll
  for (int t = 1; t <= K; ++t) acc += tap(t) * x[K + R - 1 + t];
  q[R - 1] = acc;
#pragma unroll
  for (int j = R - 2; j >= 0; --j) q[j] = z * (t0 * x[K + j + 1] + q[j + 1]) - zK * x[2 * K + j + 1];
  T pc = T(0);
#pragma unroll
  for (int t = 0; t <= K; ++t) pc += tap(t) * x[K - t];
  o[0] = pc + q[0];
#pragma unroll
  for (int j = 0; j < R - 1; ++j) {
    pc = t0 * x[K + j + 1] + z * pc - zK * x[j];
    o[j + 1] = pc + q[j + 1];
  }
}

// The same with one add or subtract for -n <= i < 2n (stencil footprints on grids wider than
// them), the division only otherwise: an integer division costs a few dozen instructions.
__host__ __device__ __forceinline__ int wrap_near(int i, int n) {
  i += i < 0 ? n : 0;
  i -= i >= n ? n : 0;
  if (unsigned(i) >= unsigned(n)) i = wrap_index(i, n);
  return i;
}

// row stride (complex elements) of a half spectrum [n1][n2/2 + 1]: padded to a multiple of 16 so
// that every row starts on a 128-byte boundary (FP32) and the strided column passes move whole
// aligned segments
__host__ __device__ __forceinline__ int spec_stride(int n2) { return (n2 / 2 + 1 + 15) / 16 * 16; }

// signed wavenumber of FFT-ordered index idx in [0, n)
__host__ __device__ __forceinline__ int signed_wavenumber(int idx, int n) { return idx < n / 2 ? idx : idx - n; }

// Error reporting from launchers: every launcher returns hipError_t of its launch.
#define SLNK_LAUNCH_CHECK() return hipGetLastError()

}  // namespace slnk
