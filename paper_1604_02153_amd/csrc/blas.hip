// FP64-accumulated reductions and vector updates for the Krylov, Chebyshev and Lanczos layers
// (section 3.4: PCG inner products, norms of the reduced gradient, Armijo objective values).
// Every operation runs on 'batch' same-size items at once (grid y = item).  Every reduction is
// two-stage with a fixed combination order, so results are deterministic.
#include <algorithm>
#include <cfloat>

#include "kernels.hpp"

namespace slnk {
namespace {

constexpr int kThreads = 256;
constexpr int kMaxBlocks = 1024;

enum RedOp : int { kDot = 0, kDot3 = 1, kNorms = 2 };

__device__ void block_reduce4(double v[4], unsigned maxmask, int ncomp, double* out) {
  __shared__ double sh[4][kThreads / 64];
  const int tid = threadIdx.x;
  for (int c = 0; c < ncomp; ++c) {
    double x = v[c];
    const bool mx = (maxmask >> c) & 1u;
    for (int off = 32; off > 0; off >>= 1) {
      const double y = __shfl_down(x, off, 64);
      x = mx ? fmax(x, y) : x + y;
    }
    if ((tid & 63) == 0) sh[c][tid >> 6] = x;
  }
  __syncthreads();
  if (tid == 0) {
    for (int c = 0; c < ncomp; ++c) {
      const bool mx = (maxmask >> c) & 1u;
      double x = sh[c][0];
      for (int w = 1; w < kThreads / 64; ++w) x = mx ? fmax(x, sh[c][w]) : x + sh[c][w];
      out[c] = x;
    }
  }
}

template <typename T, int OP>
__global__ void __launch_bounds__(kThreads) k_reduce(size_t n, const T* __restrict__ ab, const T* __restrict__ bb,
                                                      double* __restrict__ partial) {
  const size_t off = size_t(blockIdx.y) * n;
  const T* a = ab + off;
  const T* b = bb + off;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  const size_t stride = size_t(gridDim.x) * kThreads;
  for (size_t i = size_t(blockIdx.x) * kThreads + threadIdx.x; i < n; i += stride) {
    const double x = double(a[i]);
    if constexpr (OP == kDot) {
      v[0] += x * double(b[i]);
    } else if constexpr (OP == kDot3) {
      const double y = double(b[i]);
      v[0] += x * x;
      v[1] += x * y;
      v[2] += y * y;
    } else {
      if (isfinite(x)) {
        v[0] += x * x;
        v[1] = fmax(v[1], fabs(x));
      } else {
        v[2] += 1.0;
      }
    }
  }
  constexpr int nc = OP == kDot ? 1 : 3;
  constexpr unsigned mm = OP == kNorms ? 2u : 0u;
  block_reduce4(v, mm, nc, partial + 4 * (size_t(blockIdx.y) * gridDim.x + blockIdx.x));
}

// one block per item: combine the item's partials in a fixed order into result[4 item + c]
__global__ void __launch_bounds__(kThreads) k_finish(int nparts, int stride, long long per_item, int ncomp,
                                                      unsigned maxmask, const double* __restrict__ partialb,
                                                      double* __restrict__ resultb) {
  const double* partial = partialb + blockIdx.x * per_item;
  double* result = resultb + 4 * blockIdx.x;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int p = threadIdx.x; p < nparts; p += kThreads)
    for (int c = 0; c < ncomp; ++c) {
      const double x = partial[size_t(p) * stride + c];
      v[c] = ((maxmask >> c) & 1u) ? fmax(v[c], x) : v[c] + x;
    }
  __shared__ double outv[4];
  block_reduce4(v, maxmask, ncomp, outv);
  __syncthreads();
  if (threadIdx.x < ncomp) result[threadIdx.x] = outv[threadIdx.x];
}

// y = (a ad[z]) x + (b bd[z]) y per item z; with a zero y coefficient the old y is not read
template <typename T>
__global__ void k_axpby(size_t n, double a, const double* ad, const T* __restrict__ xb, double b, const double* bd,
                        T* __restrict__ yb) {
  const int z = blockIdx.y;
  const T ca = T(ad ? a * ad[z] : a), cb = T(bd ? b * bd[z] : b);
  const T* x = xb + size_t(z) * n;
  T* y = yb + size_t(z) * n;
  // a zero coefficient drops its operand unread: items frozen by (0, 1) keep y bit for bit
  const bool rx = ca != T(0), ry = cb != T(0);
  if (!rx && cb == T(1)) return;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
    y[i] = rx ? (ry ? ca * x[i] + cb * y[i] : ca * x[i]) : cb * y[i];
}

template <typename T>
__global__ void k_cheb_step(size_t n, const double* c1d, const double* c2d, T* __restrict__ rb, T* __restrict__ ub,
                            T* __restrict__ db, T* __restrict__ yb, T* __restrict__ xb, const T* __restrict__ sbb,
                            const T* __restrict__ s2bb) {
  const int z = blockIdx.y;
  const T c1 = T(c1d[z]), c2 = T(c2d[z]);
  const size_t off = size_t(z) * n;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) {
    const size_t k = off + i;
    const T dk = db[k], yk = yb[k];
    const T r = rb[k] - (dk + sbb[k]);
    const T u = ub[k] - (yk + s2bb[k]);
    const T d = c1 * dk + c2 * r;
    rb[k] = r;
    ub[k] = u;
    db[k] = d;
    yb[k] = c1 * yk + c2 * u;
    xb[k] = xb[k] + d;
  }
}

template <typename T>
__global__ void k_xpay(size_t n, const T* __restrict__ x, T a, const T* __restrict__ y, T* __restrict__ z) {
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
    z[i] = x[i] + a * y[i];
}

template <typename T>
__global__ void k_fill(size_t n, T v, T* __restrict__ y) {
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
    y[i] = v;
}

template <typename T>
__global__ void k_q0(size_t F, const T* __restrict__ wb, const T* __restrict__ gmb, T scale, T* __restrict__ outb) {
  const size_t off = size_t(blockIdx.y) * 2 * F;
  const T* w = wb + off;
  const T* gm = gmb + off;
  T* out = outb + off;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < F; i += size_t(gridDim.x) * blockDim.x) {
    const T g1 = gm[i], g2 = gm[i + F];
    const T d = scale * (w[i] * g1 + w[i + F] * g2);
    out[i] = d * g1;
    out[i + F] = d * g2;
  }
}

template <typename T>
__global__ void k_xpay_mixed(size_t n, const double* __restrict__ xb, double a, const double* ad,
                             const T* __restrict__ yb, double* __restrict__ zb, const int* mask) {
  const int z = blockIdx.y;
  if (mask && !mask[z]) return;
  const double c = ad ? a * ad[z] : a;
  const size_t off = size_t(z) * n;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
    zb[off + i] = xb[off + i] + c * double(yb[off + i]);
}

template <typename T>
__global__ void k_masked_copy(size_t n, const T* __restrict__ src, long long ss, T* __restrict__ dst, long long ds,
                              const int* mask) {
  const int z = blockIdx.y;
  if (mask && !mask[z]) return;
  const T* a = src + z * ss;
  T* b = dst + z * ds;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
    b[i] = a[i];
}

template <typename TI, typename TO>
__global__ void k_cast(size_t n, const TI* __restrict__ x, TO* __restrict__ y) {
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
    y[i] = TO(x[i]);
}

// ---- full-Newton matvec helpers (one element per thread; grid y = item, grid z = time level)
// prod[z][j][c] = lam[z][j] * vt[z][c]   (j = 0..nt, c = 0, 1)
template <typename T>
__global__ void k_fn_products(size_t F, int nt1, const T* __restrict__ lam, const T* __restrict__ vt,
                              T* __restrict__ prod) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= F) return;
  const int z = blockIdx.y, j = blockIdx.z;
  const T l = lam[(size_t(z) * nt1 + j) * F + i];
  const T v1 = vt[size_t(z) * 2 * F + i], v2 = vt[size_t(z) * 2 * F + F + i];
  T* o = prod + (size_t(z) * nt1 + j) * 2 * F;
  o[i] = l * v1;
  o[F + i] = l * v2;
}

// e[z][j-1] = ht/2 (1 + ht divv[z]) e[z][j-1] + ht/2 sigma[z][j-1]   (j = 1..nt; e holds
// I[sigma^j](X_a) on entry)
template <typename T>
__global__ void k_fn_source(size_t F, int nt, double ht, const T* __restrict__ divv, const T* __restrict__ sigma,
                            T* __restrict__ e) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= F) return;
  const int z = blockIdx.y, j = blockIdx.z;  // level j - 1
  const T h = T(0.5 * ht);
  const T d = divv[size_t(z) * F + i];
  const size_t o = (size_t(z) * nt + j) * F + i;
  e[o] = h * (T(1) + T(ht) * d) * e[o] + h * sigma[(size_t(z) * (nt + 1) + j) * F + i];
}

// bt[z][c] += sum_{j=1..nt} w_j lam[z][j] gmt[z][j-1][c]  (trapezoid weights of t^1..t^nt)
template <typename T>
__global__ void k_fn_accumulate(size_t F, int nt, double ht, const T* __restrict__ lam, const T* __restrict__ gmt,
                                T* __restrict__ bt, const int* mask) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int z = blockIdx.y;
  if (i >= F || (mask && !mask[z])) return;
  T a1 = T(0), a2 = T(0);
  for (int j = 1; j <= nt; ++j) {
    const T w = T(j == nt ? 0.5 * ht : ht);
    const T l = w * lam[(size_t(z) * (nt + 1) + j) * F + i];
    const T* g = gmt + (size_t(z) * nt + (j - 1)) * 2 * F;
    a1 += l * g[i];
    a2 += l * g[F + i];
  }
  T* b = bt + size_t(z) * 2 * F;
  b[i] += a1;
  b[F + i] += a2;
}

// out[z] = x[z] - y[z] over n elements, items at strides sx, sy, so
template <typename T>
__global__ void k_sub_strided(size_t n, const T* __restrict__ x, long long sx, const T* __restrict__ y, long long sy,
                              T* __restrict__ out, long long so) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int z = blockIdx.y;
  out[z * so + i] = x[z * sx + i] - y[z * sy + i];
}

// Step coefficients of the preconditioned CG iteration kept in device memory (item z's reduction
// at red[4 z]).  PCG_RZ stores rz[z]; PCG_ALPHA writes c0[z] = rz / pq for running items whose
// curvature pq is positive and finite, else 0 (the host reads pq with the residual norm and acts
// on the rest); PCG_BETA forms beta = rz_new / rz, stores rz_new and writes the coefficients of
// p <- c0 z + c1 p: (1, beta) for running items, (0, 1) for stopped ones.
__global__ void k_pcg_coef(int mode, int batch, const int* mask, const double* red, double* rz, double* c0,
                           double* c1) {
  const int z = threadIdx.x + blockIdx.x * blockDim.x;
  if (z >= batch) return;
  const bool run = !mask || mask[z] != 0;
  const double v = red[4 * z];
  if (mode == PCG_RZ) {
    if (run) rz[z] = v;
  } else if (mode == PCG_ALPHA) {
    c0[z] = (run && v > 0.0 && v <= DBL_MAX) ? rz[z] / v : 0.0;
  } else {
    if (run) {
      c0[z] = 1.0;
      c1[z] = v / rz[z];
      rz[z] = v;
    } else {
      c0[z] = 0.0;
      c1[z] = 1.0;
    }
  }
}

// Device-side scalars of one Lanczos step (item z's reduction at red[4 z], z < batch).
// LANCZOS_ALPHA: alpha[z] = q.w (the coefficient of w <- w - alpha q), logged at
// log[(z * steps + j) * 2] for live items.  LANCZOS_BETA: red = w.w; for a live item beta = sqrt(w.w)
// ends its tridiagonal matrix at the last step or at breakdown (beta <= 1e-14 |alpha|): then the
// item is marked dead, its log entry is -1 and beta[z] = inv[z] = 0; otherwise the log holds beta,
// beta[z] = beta (the next step's coefficient of w <- w - beta q_prev) and inv[z] = 1 / beta.
// Dead items keep beta[z] = 0 and get inv[z] = 0.
__global__ void k_lanczos_coef(int mode, int batch, int j, int steps, const double* red, int* live, double* alpha,
                               double* beta, double* inv, double* log) {
  const int z = threadIdx.x + blockIdx.x * blockDim.x;
  if (z >= batch) return;
  const double v = red[4 * z];
  double* lz = log + (size_t(z) * steps + j) * 2;
  if (mode == LANCZOS_ALPHA) {
    alpha[z] = v;
    if (live[z]) lz[0] = v;
    return;
  }
  if (!live[z]) {
    inv[z] = 0.0;
    return;
  }
  const double b = sqrt(v);
  if (j == steps - 1 || b <= 1e-14 * fabs(alpha[z])) {
    live[z] = 0;
    lz[1] = -1.0;
    beta[z] = 0.0;
    inv[z] = 0.0;
  } else {
    lz[1] = b;
    beta[z] = b;
    inv[z] = 1.0 / b;
  }
}

struct IntPack {
  int v[64];
};

__global__ void k_set_ints(int* p, IntPack pack, int count) {
  if (int(threadIdx.x) < count) p[threadIdx.x] = pack.v[threadIdx.x];
}

// One element per thread up to 64 Ki blocks per item: an elementwise kernel then has no
// loop-carried chain (its loads could not move above the previous element's stores, which may
// alias them), so small fields finish in one memory round trip.
inline unsigned grid_for(size_t n) {
  size_t b = (n + kThreads - 1) / kThreads;
  if (b < 1) b = 1;
  if (b > 65535) b = 65535;
  return unsigned(b);
}

}  // namespace

hipError_t pcg_coef(hipStream_t s, int mode, int batch, const int* mask, const double* red, double* rz, double* c0,
                    double* c1) {
  if (batch <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pcg_coef, dim3((batch + 63) / 64), dim3(64), 0, s, mode, batch, mask, red, rz, c0, c1);
  return hipGetLastError();
}

hipError_t lanczos_coef(hipStream_t s, int mode, int batch, int j, int steps, const double* red, int* live,
                        double* alpha, double* beta, double* inv, double* log) {
  if (batch <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_lanczos_coef, dim3((batch + 63) / 64), dim3(64), 0, s, mode, batch, j, steps, red, live, alpha,
                     beta, inv, log);
  return hipGetLastError();
}

hipError_t set_ints(hipStream_t s, int* p, const int* host_values, int count) {
  for (int base = 0; base < count; base += 64) {
    IntPack pack{};
    const int c = std::min(64, count - base);
    for (int i = 0; i < c; ++i) pack.v[i] = host_values[base + i];
    hipLaunchKernelGGL(k_set_ints, dim3(1), dim3(64), 0, s, p + base, pack, c);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

int reduce_blocks(size_t n) {
  size_t b = (n + kThreads * 8 - 1) / (kThreads * 8);
  if (b < 1) b = 1;
  if (b > kMaxBlocks) b = kMaxBlocks;
  return int(b);
}

hipError_t finish(hipStream_t s, int batch, int nparts, int stride, long long per_item, int ncomp, unsigned maxmask,
                  const double* partial, double* result) {
  hipLaunchKernelGGL(k_finish, dim3(batch), dim3(kThreads), 0, s, nparts, stride, per_item, ncomp, maxmask, partial,
                     result);
  return hipGetLastError();
}

template <typename T>
hipError_t dot(hipStream_t s, int batch, size_t n, const T* a, const T* b, double* partial, double* result) {
  const int nb = reduce_blocks(n);
  hipLaunchKernelGGL((k_reduce<T, kDot>), dim3(nb, batch), dim3(kThreads), 0, s, n, a, b, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return finish(s, batch, nb, 4, 4LL * nb, 1, 0u, partial, result);
}

template <typename T>
hipError_t dot3(hipStream_t s, int batch, size_t n, const T* a, const T* b, double* partial, double* result) {
  const int nb = reduce_blocks(n);
  hipLaunchKernelGGL((k_reduce<T, kDot3>), dim3(nb, batch), dim3(kThreads), 0, s, n, a, b, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return finish(s, batch, nb, 4, 4LL * nb, 3, 0u, partial, result);
}

template <typename T>
hipError_t norms(hipStream_t s, int batch, size_t n, const T* a, double* partial, double* result) {
  const int nb = reduce_blocks(n);
  hipLaunchKernelGGL((k_reduce<T, kNorms>), dim3(nb, batch), dim3(kThreads), 0, s, n, a, a, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return finish(s, batch, nb, 4, 4LL * nb, 3, 2u, partial, result);
}

template <typename T>
hipError_t axpby(hipStream_t s, int batch, size_t n, double a, const double* ad, const T* x, double b,
                 const double* bd, T* y) {
  hipLaunchKernelGGL(k_axpby<T>, dim3(grid_for(n), batch), dim3(kThreads), 0, s, n, a, ad, x, b, bd, y);
  return hipGetLastError();
}

template <typename T>
hipError_t cheb_step(hipStream_t s, int batch, size_t n, const double* c1, const double* c2, T* r, T* u, T* d, T* y,
                     T* x, const T* sb, const T* s2b) {
  hipLaunchKernelGGL(k_cheb_step<T>, dim3(grid_for(n), batch), dim3(kThreads), 0, s, n, c1, c2, r, u, d, y, x, sb, s2b);
  return hipGetLastError();
}

template <typename T>
hipError_t xpay(hipStream_t s, size_t n, const T* x, double a, const T* y, T* z) {
  hipLaunchKernelGGL(k_xpay<T>, dim3(grid_for(n)), dim3(kThreads), 0, s, n, x, T(a), y, z);
  return hipGetLastError();
}

template <typename T>
hipError_t fill(hipStream_t s, size_t n, double value, T* y) {
  hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(n)), dim3(kThreads), 0, s, n, T(value), y);
  return hipGetLastError();
}

template <typename T>
hipError_t q_at_zero(hipStream_t s, int batch, size_t F, const T* w, const T* gm, double scale, T* out) {
  hipLaunchKernelGGL(k_q0<T>, dim3(grid_for(F), batch), dim3(kThreads), 0, s, F, w, gm, T(scale), out);
  return hipGetLastError();
}

template <typename T>
hipError_t cast_copy(hipStream_t s, size_t n, const double* x, T* y) {
  hipLaunchKernelGGL((k_cast<double, T>), dim3(grid_for(n)), dim3(kThreads), 0, s, n, x, y);
  return hipGetLastError();
}

template <typename T>
hipError_t cast_back(hipStream_t s, size_t n, const T* x, double* y) {
  hipLaunchKernelGGL((k_cast<T, double>), dim3(grid_for(n)), dim3(kThreads), 0, s, n, x, y);
  return hipGetLastError();
}

template <typename T>
hipError_t xpay_mixed(hipStream_t s, int batch, size_t n, const double* x, double a, const double* ad, const T* y,
                      double* z, const int* mask) {
  hipLaunchKernelGGL(k_xpay_mixed<T>, dim3(grid_for(n), batch), dim3(kThreads), 0, s, n, x, a, ad, y, z, mask);
  return hipGetLastError();
}

template <typename T>
hipError_t masked_copy(hipStream_t s, int batch, size_t n, const T* src, long long src_stride, T* dst,
                       long long dst_stride, const int* mask) {
  hipLaunchKernelGGL(k_masked_copy<T>, dim3(grid_for(n), batch), dim3(kThreads), 0, s, n, src, src_stride, dst,
                     dst_stride, mask);
  return hipGetLastError();
}

inline unsigned fn_blocks(size_t F) { return unsigned((F + kThreads - 1) / kThreads); }

template <typename T>
hipError_t fn_products(hipStream_t s, int batch, size_t F, int nt, const T* lam, const T* vt, T* prod) {
  hipLaunchKernelGGL(k_fn_products<T>, dim3(fn_blocks(F), batch, nt + 1), dim3(kThreads), 0, s, F, nt + 1, lam, vt,
                     prod);
  return hipGetLastError();
}

template <typename T>
hipError_t fn_source(hipStream_t s, int batch, size_t F, int nt, double ht, const T* divv, const T* sigma, T* e) {
  hipLaunchKernelGGL(k_fn_source<T>, dim3(fn_blocks(F), batch, nt), dim3(kThreads), 0, s, F, nt, ht, divv, sigma, e);
  return hipGetLastError();
}

template <typename T>
hipError_t fn_accumulate(hipStream_t s, int batch, size_t F, int nt, double ht, const T* lam, const T* gmt, T* bt,
                         const int* mask) {
  hipLaunchKernelGGL(k_fn_accumulate<T>, dim3(fn_blocks(F), batch), dim3(kThreads), 0, s, F, nt, ht, lam, gmt, bt,
                     mask);
  return hipGetLastError();
}

template <typename T>
hipError_t sub_strided(hipStream_t s, int batch, size_t n, const T* x, long long sx, const T* y, long long sy, T* out,
                       long long so) {
  hipLaunchKernelGGL(k_sub_strided<T>, dim3(fn_blocks(n), batch), dim3(kThreads), 0, s, n, x, sx, y, sy, out, so);
  return hipGetLastError();
}

#define INST(T)                                                                                            \
  template hipError_t dot<T>(hipStream_t, int, size_t, const T*, const T*, double*, double*);             \
  template hipError_t dot3<T>(hipStream_t, int, size_t, const T*, const T*, double*, double*);            \
  template hipError_t norms<T>(hipStream_t, int, size_t, const T*, double*, double*);                     \
  template hipError_t axpby<T>(hipStream_t, int, size_t, double, const double*, const T*, double,         \
                               const double*, T*);                                                        \
  template hipError_t xpay<T>(hipStream_t, size_t, const T*, double, const T*, T*);                       \
  template hipError_t cheb_step<T>(hipStream_t, int, size_t, const double*, const double*, T*, T*, T*, T*, T*,   \
                                   const T*, const T*);                                                         \
  template hipError_t fill<T>(hipStream_t, size_t, double, T*);                                           \
  template hipError_t q_at_zero<T>(hipStream_t, int, size_t, const T*, const T*, double, T*);             \
  template hipError_t cast_copy<T>(hipStream_t, size_t, const double*, T*);                               \
  template hipError_t cast_back<T>(hipStream_t, size_t, const T*, double*);                               \
  template hipError_t xpay_mixed<T>(hipStream_t, int, size_t, const double*, double, const double*,       \
                                    const T*, double*, const int*);                                       \
  template hipError_t masked_copy<T>(hipStream_t, int, size_t, const T*, long long, T*, long long, const int*); \
  template hipError_t fn_products<T>(hipStream_t, int, size_t, int, const T*, const T*, T*);               \
  template hipError_t fn_source<T>(hipStream_t, int, size_t, int, double, const T*, const T*, T*);         \
  template hipError_t fn_accumulate<T>(hipStream_t, int, size_t, int, double, const T*, const T*, T*,      \
                                       const int*);                                                       \
  template hipError_t sub_strided<T>(hipStream_t, int, size_t, const T*, long long, const T*, long long, T*, \
                                     long long);
INST(float)
INST(double)
#undef INST

}  // namespace slnk
