// Elementwise kernels of the stabilised RK2 (RK2A) transport: the transport equations in
// antisymmetric form (section 3.3.1; appendix "Stabilized RK2 Scheme"), pseudospectral in space
// (the derivatives come from spec_rk2a / spec_grad), Heun's method in time.  Every kernel covers
// 'batch' items (grid y = item; each pointer advances by its own item stride) with one element per
// thread.
#include "kernels.hpp"

namespace slnk {
namespace {

constexpr int kThreadsR = 256;

inline unsigned blocks_r(size_t F) { return unsigned((F + kThreadsR - 1) / kThreadsR); }

// out = (a, a w1, a w2)
template <typename T>
__global__ void __launch_bounds__(kThreadsR) k_rk2a_prod(size_t F, const T* __restrict__ ab, long long sa,
                                                          const T* __restrict__ wb, long long sw,
                                                          T* __restrict__ outb) {
  const size_t i = size_t(blockIdx.x) * kThreadsR + threadIdx.x;
  if (i >= F) return;
  const int z = blockIdx.y;
  const T a = ab[z * sa + i];
  const T* w = wb + z * sw;
  T* out = outb + size_t(z) * 3 * F;
  out[i] = a;
  out[F + i] = a * w[i];
  out[2 * F + i] = a * w[F + i];
}

// value of the operator at a node: sgn 1/2 (w1 d1u + w2 d2u + div(u w) + dsgn u div w)
template <typename T>
__device__ __forceinline__ T rk2a_op(const T* d, size_t F, size_t i, T w1, T w2, T u, T divw, int sgn, int dsgn) {
  const T r = w1 * d[i] + w2 * d[F + i] + d[2 * F + i] + T(dsgn) * u * divw;
  return T(0.5 * sgn) * r;
}

// One Heun stage for dy/ds = sgn L_dsgn y + src with L_dsgn y = 1/2 (v . grad y + div(y v) + dsgn y div v)
// (dsgn = -1, sgn = -1: the state operator -L; dsgn = +1, sgn = +1: the adjoint operator A).
// d: derivatives (d1 y, d2 y, div(y v)) of the stage's input, whose products (y, y v1, y v2) are
// in w3 (w3[0] = the stage input).
// stage 1: k1 = op + src -> kbuf; w3 <- products of y + ht k1.
// stage 2: k2 = op + src; ynew = y0 + ht/2 (kbuf + k2) -> dst; w3 <- products of ynew.
template <typename T>
__global__ void __launch_bounds__(kThreadsR) k_rk2a_stage(int stage, size_t F, double ht, int sgn, int dsgn,
                                                           const T* __restrict__ db, T* __restrict__ w3b,
                                                           const T* __restrict__ vb, long long sv,
                                                           const T* __restrict__ divb, long long sdiv,
                                                           const T* __restrict__ srcb, long long ssrc,
                                                           const T* __restrict__ y0b, long long sy0,
                                                           T* __restrict__ kb, T* __restrict__ dstb,
                                                           long long sdst) {
  const size_t i = size_t(blockIdx.x) * kThreadsR + threadIdx.x;
  if (i >= F) return;
  const int z = blockIdx.y;
  const T* d = db + size_t(z) * 3 * F;
  T* w3 = w3b + size_t(z) * 3 * F;
  const T v1 = vb[z * sv + i], v2 = vb[z * sv + F + i];
  const T y = w3[i];
  T k = rk2a_op(d, F, i, v1, v2, y, divb[z * sdiv + i], sgn, dsgn);
  if (srcb) k += srcb[z * ssrc + i];
  T out;
  if (stage == 1) {
    kb[size_t(z) * F + i] = k;
    out = y + T(ht) * k;
  } else {
    out = y0b[z * sy0 + i] + T(0.5 * ht) * (kb[size_t(z) * F + i] + k);
    dstb[z * sdst + i] = out;
  }
  w3[i] = out;
  w3[F + i] = out * v1;
  w3[2 * F + i] = out * v2;
}

// out = sgn 1/2 (w1 d1a + w2 d2a + div(a w) + dsgn a div w): a source term of the incremental
// equations from the derivatives d of (a, a w1, a w2)
template <typename T>
__global__ void __launch_bounds__(kThreadsR) k_rk2a_eval(size_t F, int sgn, int dsgn, const T* __restrict__ db,
                                                          const T* __restrict__ ab, long long sa,
                                                          const T* __restrict__ wb, long long sw,
                                                          const T* __restrict__ divwb, long long sdw,
                                                          T* __restrict__ outb, long long so) {
  const size_t i = size_t(blockIdx.x) * kThreadsR + threadIdx.x;
  if (i >= F) return;
  const int z = blockIdx.y;
  const T* d = db + size_t(z) * 3 * F;
  const T* w = wb + z * sw;
  outb[z * so + i] = rk2a_op(d, F, i, w[i], w[F + i], ab[z * sa + i], divwb[z * sdw + i], sgn, dsgn);
}

// out = (lam, lam m)
template <typename T>
__global__ void __launch_bounds__(kThreadsR) k_rk2a_pair(size_t F, const T* __restrict__ lb, long long sl,
                                                          const T* __restrict__ mb, long long sm,
                                                          T* __restrict__ outb) {
  const size_t i = size_t(blockIdx.x) * kThreadsR + threadIdx.x;
  if (i >= F) return;
  const int z = blockIdx.y;
  const T l = lb[z * sl + i];
  outb[size_t(z) * 2 * F + i] = l;
  outb[size_t(z) * 2 * F + F + i] = l * mb[z * sm + i];
}

// acc (=, +=) w 1/2 (lam grad m - m grad lam + grad(lam m)); g4 = (grad lam, grad(lam m)) per item
template <typename T>
__global__ void __launch_bounds__(kThreadsR) k_rk2a_accum(size_t F, double w, int init, const T* __restrict__ lb,
                                                           long long sl, const T* __restrict__ mb, long long sm,
                                                           const T* __restrict__ gmb, long long sgm,
                                                           const T* __restrict__ g4b, T* __restrict__ accb,
                                                           long long sacc) {
  const size_t i = size_t(blockIdx.x) * kThreadsR + threadIdx.x;
  if (i >= F) return;
  const int z = blockIdx.y;
  const T l = lb[z * sl + i], m = mb[z * sm + i];
  const T* gm = gmb + z * sgm;
  const T* g4 = g4b + size_t(z) * 4 * F;
  T* acc = accb + z * sacc;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const T t = T(0.5 * w) * (l * gm[c * F + i] - m * g4[c * F + i] + g4[(2 + c) * F + i]);
    acc[c * F + i] = init ? t : acc[c * F + i] + t;
  }
}

}  // namespace

template <typename T>
hipError_t rk2a_prod(hipStream_t s, int batch, size_t F, const T* a, long long sa, const T* w, long long sw, T* out) {
  hipLaunchKernelGGL(k_rk2a_prod<T>, dim3(blocks_r(F), batch), dim3(kThreadsR), 0, s, F, a, sa, w, sw, out);
  return hipGetLastError();
}

template <typename T>
hipError_t rk2a_stage(hipStream_t s, int batch, const RK2AStage<T>& a) {
  hipLaunchKernelGGL(k_rk2a_stage<T>, dim3(blocks_r(a.F), batch), dim3(kThreadsR), 0, s, a.stage, a.F, a.ht, a.sgn,
                     a.dsgn, a.d, a.w3, a.v, a.sv, a.divv, a.sdiv, a.src, a.ssrc, a.y0, a.sy0, a.k, a.dst, a.sdst);
  return hipGetLastError();
}

template <typename T>
hipError_t rk2a_eval(hipStream_t s, int batch, size_t F, int sgn, int dsgn, const T* d, const T* a, long long sa,
                     const T* w, long long sw, const T* divw, long long sdw, T* out, long long so) {
  hipLaunchKernelGGL(k_rk2a_eval<T>, dim3(blocks_r(F), batch), dim3(kThreadsR), 0, s, F, sgn, dsgn, d, a, sa, w, sw,
                     divw, sdw, out, so);
  return hipGetLastError();
}

template <typename T>
hipError_t rk2a_pair(hipStream_t s, int batch, size_t F, const T* lam, long long sl, const T* m, long long sm,
                     T* out) {
  hipLaunchKernelGGL(k_rk2a_pair<T>, dim3(blocks_r(F), batch), dim3(kThreadsR), 0, s, F, lam, sl, m, sm, out);
  return hipGetLastError();
}

template <typename T>
hipError_t rk2a_accum(hipStream_t s, int batch, size_t F, double w, int init, const T* lam, long long sl, const T* m,
                      long long sm, const T* gm, long long sgm, const T* g4, T* acc, long long sacc) {
  hipLaunchKernelGGL(k_rk2a_accum<T>, dim3(blocks_r(F), batch), dim3(kThreadsR), 0, s, F, w, init, lam, sl, m, sm,
                     gm, sgm, g4, acc, sacc);
  return hipGetLastError();
}

#define INST(T)                                                                                               \
  template hipError_t rk2a_prod<T>(hipStream_t, int, size_t, const T*, long long, const T*, long long, T*);    \
  template hipError_t rk2a_stage<T>(hipStream_t, int, const RK2AStage<T>&);                                   \
  template hipError_t rk2a_eval<T>(hipStream_t, int, size_t, int, int, const T*, const T*, long long, const T*, \
                                   long long, const T*, long long, T*, long long);                            \
  template hipError_t rk2a_pair<T>(hipStream_t, int, size_t, const T*, long long, const T*, long long, T*);    \
  template hipError_t rk2a_accum<T>(hipStream_t, int, size_t, double, int, const T*, long long, const T*,      \
                                    long long, const T*, long long, const T*, T*, long long);
INST(float)
INST(double)
#undef INST

}  // namespace slnk
