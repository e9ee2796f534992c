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
