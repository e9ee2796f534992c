// Semi-Lagrangian transport on gfx950 (section 3.3.2: tracing the characteristic by Heun's
// method, cubic spline interpolation at the departure points, RK2 along the characteristic;
// eqs. e:state-slm, e:adj-slm, e:inc-state-slm, e:inc-adj-slm).
//
// One time step of any of the four transport equations is one kernel.  A 16x16 tile of output
// nodes stages the transported field over its departure-point footprint plus the support of the
// spline prefilter in LDS, computes the periodic cubic B-spline coefficients there with the
// separable exponential filter c = sqrt(3) sum_t z^|t| f[i+t], z = sqrt(3) - 2 (the inverse of
// the circulant (1, 4, 1)/6 operator, truncated where |z|^t falls below the working precision),
// gathers the 4x4 tensor B-spline stencil at every departure point and applies the step's
// update (Heun weights, adjoint factor, time-integral accumulation) in registers.
#include <algorithm>
#include <atomic>
#include <mutex>
#include <type_traits>

#include "kernels.hpp"

namespace slnk {
namespace {

// one-time host set-up (filter taps, LDS limit, kernel LDS attributes) may be reached from
// several host threads driving contexts on different streams
std::mutex g_setup_mutex;

constexpr int kTile = 16;

template <typename T>
struct FilterTaps;
// Truncation error of the filter: 2 sqrt(3) |z|^(K+1) / (1 - |z|) relative to max |f|:
// 4.7e-8 for K = 13 (below FP32 rounding) and 1.2e-16 for K = 28 (FP64).  R: outputs per thread
// of the register-blocked filter passes.
template <>
struct FilterTaps<float> {
  static constexpr int K = 13;
  static constexpr int R = 8;
};
template <>
struct FilterTaps<double> {
  static constexpr int K = 28;
  static constexpr int R = 4;
};
constexpr int kMaxChunks = 12;  // footprint side P <= 16 * kMaxChunks

__constant__ double c_taps_d[FilterTaps<double>::K + 1];
__constant__ float c_taps_f[FilterTaps<float>::K + 1];

template <typename T>
__device__ __forceinline__ T tap(int t);
template <>
__device__ __forceinline__ float tap<float>(int t) { return c_taps_f[t]; }
template <>
__device__ __forceinline__ double tap<double>(int t) { return c_taps_d[t]; }

std::atomic<bool> g_taps_ready{false};

hipError_t upload_taps() {
  if (g_taps_ready.load(std::memory_order_acquire)) return hipSuccess;
  std::lock_guard<std::mutex> lock(g_setup_mutex);
  if (g_taps_ready.load(std::memory_order_relaxed)) return hipSuccess;
  // exact coefficients in FP64 from the closed form
  const double z = std::sqrt(3.0) - 2.0;
  double td[FilterTaps<double>::K + 1];
  float tf[FilterTaps<float>::K + 1];
  for (int t = 0; t <= FilterTaps<double>::K; ++t) td[t] = std::sqrt(3.0) * std::pow(z, t);
  for (int t = 0; t <= FilterTaps<float>::K; ++t) tf[t] = float(td[t]);
  hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_taps_d), td, sizeof(td));
  if (e != hipSuccess) return e;
  e = hipMemcpyToSymbol(HIP_SYMBOL(c_taps_f), tf, sizeof(tf));
  if (e == hipSuccess) g_taps_ready.store(true, std::memory_order_release);
  return e;
}

// Tile of this block.  Workgroups go to the 8 XCDs of the chip round-robin in launch order, so
// the blocks of one XCD are given a contiguous run of tiles (row-major): tile halos shared by
// neighbouring tiles are then fetched once into that XCD's L2.
constexpr int kXcds = 8;
__device__ __forceinline__ void xcd_tile(int& ty, int& tx) {
  const int nb = gridDim.x * gridDim.y;
  const int b = blockIdx.y * gridDim.x + blockIdx.x;
  const int x = b % kXcds, local = b / kXcds;
  const int base = nb / kXcds, rem = nb % kXcds;
  const int t = x * base + min(x, rem) + local;
  ty = t / gridDim.x;
  tx = t - ty * gridDim.x;
}

// cubic B-spline weights of the four stencil nodes at fractional offset t in [0, 1)
// (products with 1/6 rather than divisions: a correctly rounded division costs about ten
// instructions, and the weights of every departure point are formed in the step's critical path)
template <typename T>
__device__ __forceinline__ void bspline_w(T t, T* w) {
  const T c6 = T(1.0 / 6.0);
  const T t2 = t * t, t3 = t2 * t;
  const T s = T(1) - t;
  w[0] = s * s * s * c6;
  w[1] = (T(3) * t3 - T(6) * t2 + T(4)) * c6;
  w[2] = (T(-3) * t3 + T(3) * t2 + T(3) * t + T(1)) * c6;
  w[3] = t3 * c6;
}


// Spline value at (s1, s2) (in cells) from a global coefficient field, periodic.  The stencil's
// first row and column are wrapped once (a division only for departure points outside the
// grid); its other rows and columns then need at most one subtraction.  Away from the last three
// columns a stencil row is four consecutive values, read as one 16-byte (FP32) or two 16-byte
// (FP64) copies: the compiler emits wide loads where the target allows unaligned access and
// element loads otherwise.
template <typename T>
__device__ T interp_global(const T* __restrict__ c, int n1, int n2, T s1, T s2) {
  const T f1 = floor(s1), f2 = floor(s2);
  T w1[4], w2[4];
  bspline_w(s1 - f1, w1);
  bspline_w(s2 - f2, w2);
  int i1 = int(f1) - 1, i2 = int(f2) - 1;
  if (unsigned(i1) >= unsigned(n1)) i1 = wrap_index(i1, n1);
  if (unsigned(i2) >= unsigned(n2)) i2 = wrap_index(i2, n2);
  T acc = T(0);
  if (i2 + 3 < n2) {
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      int r = i1 + a;
      r -= r >= n1 ? n1 : 0;
      T v[4];
      __builtin_memcpy(v, c + size_t(r) * n2 + i2, sizeof(v));
      acc += w1[a] * (w2[0] * v[0] + w2[1] * v[1] + w2[2] * v[2] + w2[3] * v[3]);
    }
  } else {
    int cols[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int cb = i2 + b;
      cols[b] = cb >= n2 ? cb - n2 : cb;
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      int r = i1 + a;
      r -= r >= n1 ? n1 : 0;
      const T* row = c + size_t(r) * n2;
      acc += w1[a] * (w2[0] * row[cols[0]] + w2[1] * row[cols[1]] + w2[2] * row[cols[2]] + w2[3] * row[cols[3]]);
    }
  }
  return acc;
}

// FP64 block reduction of two values: (sum, max).  Writes partial[2 * block + {0, 1}] (block
// within the item's x-y grid; the caller offsets 'partial' by item).
__device__ void block_sum_max(double s, double m, double* partial) {
  __shared__ double rs[16], rm[16];
  for (int off = 32; off > 0; off >>= 1) {
    s += __shfl_down(s, off, 64);
    m = fmax(m, __shfl_down(m, off, 64));
  }
  const int tid = threadIdx.y * blockDim.x + threadIdx.x;
  const int nw = (blockDim.x * blockDim.y + 63) >> 6;
  if ((tid & 63) == 0) {
    rs[tid >> 6] = s;
    rm[tid >> 6] = m;
  }
  __syncthreads();
  if (tid == 0) {
    double ts = 0.0, tm = 0.0;
    for (int w = 0; w < nw; ++w) {
      ts += rs[w];
      tm = fmax(tm, rm[w]);
    }
    const int bid = blockIdx.y * gridDim.x + blockIdx.x;
    partial[2 * bid] = ts;
    partial[2 * bid + 1] = tm;
  }
}

// ------------------------------------------------------------------------------------------
// fused prefilter + gather step
// ------------------------------------------------------------------------------------------
// The arguments as seen by item z: every pointer advanced by z times its stride.
template <typename T>
__device__ __forceinline__ StepArgs<T> item_view(const StepArgs<T>& b, int z) {
  StepArgs<T> a = b;
  auto adv = [z](auto* p, long long st) { return p ? p + z * st : p; };
  a.src = adv(b.src, b.st_src);
  a.dst = adv(b.dst, b.st_dst);
  a.d1 = adv(b.d1, b.st_d);
  a.gamma = adv(b.gamma, b.st_gamma);
  a.aux0 = adv(b.aux0, b.st_aux0);
  a.aux1 = adv(b.aux1, b.st_aux1);
  a.gm_new = adv(b.gm_new, b.st_gm);
  a.gm_old = adv(b.gm_old, b.st_gm);
  a.acc = adv(b.acc, b.st_acc);
  a.vt = adv(b.vt, b.st_vt);
  a.addf = adv(b.addf, b.st_addf);
  a.out2 = adv(b.out2, b.st_out2);
  a.coef = adv(b.coef, b.st_coef);
  a.coef2 = adv(b.coef2, b.st_coef2);
  a.halo_dev = b.halo_dev ? b.halo_dev + z : nullptr;
  a.partial = b.partial ? b.partial + size_t(z) * 2 * gridDim.x * gridDim.y : nullptr;
  return a;
}
template <typename T, int KIND, bool FIRST>
__device__ __forceinline__ T load_src(const StepArgs<T>& a, size_t gi) {
  if constexpr (FIRST && KIND == int(StepKind::Adjoint)) {
    return a.aux0[gi] - a.aux1[gi];  // lambda(1) = m_R - m(1)
  } else if constexpr (FIRST && KIND == int(StepKind::IncState)) {
    const size_t F = size_t(a.n1) * a.n2;
    // q^0 = (ht/2) f^0, f = -vt . grad m^0
    return -T(0.5 * a.ht) * (a.vt[gi] * a.gm_old[gi] + a.vt[gi + F] * a.gm_old[gi + F]);
  } else {
    return a.src[gi];
  }
}

// R consecutive outputs of the truncated exponential filter from a window of R + 2K values (the
// recursive form shared with the three-dimensional passes), taps from constant memory
template <typename T, int R, int K>
__device__ __forceinline__ void filter_window(const T* x, T* o) {
  filter_window_rec<T, R, K>(x, o, [](int t) { return tap<T>(t); });
}

// Staging of a P x P footprint by a 16 x TY block (P <= TY CHR rows, P <= 16 CHC columns): every
// thread issues all of its CHR x CHC loads (rows ty + TY i, columns tx + 16 k, clamped into the
// footprint so that no load needs a branch) before it stores any of them, so the loads overlap
// instead of each waiting for the one before.
template <typename T, int KIND, bool FIRST, int CHR, int CHC, int TY>
__device__ __forceinline__ void stage_batched(const StepArgs<T>& a, T* A, int P, int ry, const int* colw) {
  const int tx = threadIdx.x, ty = threadIdx.y;
  T v[CHR][CHC];
#pragma unroll
  for (int i = 0; i < CHR; ++i) {
    const int r = min(ty + TY * i, P - 1);
    const size_t rowoff = size_t(wrap_near(ry + r, a.n1)) * a.n2;
#pragma unroll
    for (int k = 0; k < CHC; ++k) v[i][k] = load_src<T, KIND, FIRST>(a, rowoff + colw[k]);
  }
#pragma unroll
  for (int i = 0; i < CHR; ++i) {
    const int r = ty + TY * i;
#pragma unroll
    for (int k = 0; k < CHC; ++k) {
      const int c = tx + kTile * k;
      if (r < P && c < P) A[r * P + c] = v[i][k];
    }
  }
}

// Prefilter of a P x P block of staged values A (row stride P, P = G + 2K) into the B-spline
// coefficients of its inner G x G region, left at offset 0 of A (row stride G).
// LDS layout: A = P x P staged values (later the G x G coefficients), R words of slack (zero), then
// B1 = (P + R) x G row-filtered values (the last R rows zero).  Each filter pass gives a thread R
// consecutive outputs from a register window of R + 2K inputs; consecutive threads take
// consecutive rows (row pass) or columns (column pass), so the window loads do not conflict
// across LDS banks.  The last window of a row (column) reaches up to R - 1 values past the
// footprint: into the next staged row, or into the slack words after A and the extra rows of B1,
// which zero_filter_slack clears (before the barrier that ends the staging).  The recursive
// filter carries those values into the valid outputs (multiplied by taps that cancel exactly), so
// they must be finite.
template <typename T, int R>
__device__ __forceinline__ void zero_filter_slack(T* A, int P, int G, int tid, int nth) {
  T* B1 = A + P * P + R;
  for (int i = tid; i < R; i += nth) A[P * P + i] = T(0);
  for (int i = tid; i < R * G; i += nth) B1[P * G + i] = T(0);
}

template <typename T, int NTH, int R>
__device__ __forceinline__ void filter_coefficients(T* A, int P, int G, int tid) {
  constexpr int K = FilterTaps<T>::K;
  T* B1 = A + P * P + R;
  T* C = A;
  const int segs = (G + R - 1) / R;
  // prefilter along x2: thread -> (row r, segment q), outputs at columns q R .. q R + R - 1; task
  // sidx = q P + r, stepped by NTH without a division per task
  const int dq1 = NTH / P, dr1 = NTH - dq1 * P;
  int q = tid / P, r = tid - q * P;
  for (int sidx = tid; sidx < P * segs; sidx += NTH) {
    const T* src = A + r * P + q * R;
    T x[R + 2 * K], o[R];
#pragma unroll
    for (int i = 0; i < R + 2 * K; ++i) x[i] = src[i];
    filter_window<T, R, K>(x, o);
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int c = q * R + j;
      if (c < G) B1[r * G + c] = o[j];
    }
    q += dq1;
    r += dr1;
    if (r >= P) r -= P, ++q;
  }
  __syncthreads();
  // prefilter along x1: thread -> (column c, segment q), outputs at rows q R .. q R + R - 1
  const int dq2 = NTH / G, dc2 = NTH - dq2 * G;
  q = tid / G;
  int c = tid - q * G;
  for (int sidx = tid; sidx < G * segs; sidx += NTH) {
    const T* src = B1 + (q * R) * G + c;
    T x[R + 2 * K], o[R];
#pragma unroll
    for (int i = 0; i < R + 2 * K; ++i) x[i] = src[i * G];
    filter_window<T, R, K>(x, o);
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int rr = q * R + j;
      if (rr < G) C[rr * G + c] = o[j];
    }
    q += dq2;
    c += dc2;
    if (c >= G) c -= G, ++q;
  }
  __syncthreads();
}

// Stage the transported field over the rows [y0 - lo - K, y0 - lo + G + K) (and likewise the
// columns) and filter it into the B-spline coefficients of the inner G x G region, which starts
// at global node (y0 - lo, x0 - lo) and is left at LDS offset 0 of 'A' (layout of
// filter_coefficients).  The step kernel uses lo = D + 1, G = 16 + 2D + 3 (the stencil footprint
// of displacements |d| <= D).  The 16 x 32-thread blocks of small (latency-bound) launches give
// each FP32 filter task 4 outputs rather than 8: twice the tasks for their threads, each with a
// shorter dependence chain.
template <typename T, int KIND, bool FIRST, int TY>
__device__ __forceinline__ void stage_coefficients(const StepArgs<T>& a, T* A, int y0, int x0, int lo, int G) {
  constexpr int K = FilterTaps<T>::K;
  constexpr int R = (sizeof(T) == 4 && TY > kTile) ? 4 : FilterTaps<T>::R;
  const int P = G + 2 * K;
  const int n1 = a.n1, n2 = a.n2;
  const int ry = y0 - lo - K, rx = x0 - lo - K;
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int tid = ty * kTile + tx;
  constexpr int NTH = kTile * TY;
  zero_filter_slack<T, R>(A, P, G, tid, NTH);
  // stage (periodic wrap), rows ty + TY i, columns tx + 16 k
  int colw[kMaxChunks];
#pragma unroll
  for (int k = 0; k < kMaxChunks; ++k) {
    const int c = tx + kTile * k;
    colw[k] = c < P ? wrap_near(rx + c, n2) : 0;
  }
  if (P <= 4 * kTile) {
    stage_batched<T, KIND, FIRST, (4 * kTile + TY - 1) / TY, 4, TY>(a, A, P, ry, colw);
  } else if (P <= 6 * kTile) {
    stage_batched<T, KIND, FIRST, (6 * kTile + TY - 1) / TY, 6, TY>(a, A, P, ry, colw);
  } else {
    for (int r = ty; r < P; r += TY) {
      const size_t rowoff = size_t(wrap_near(ry + r, n1)) * n2;
      T* dst = A + r * P;
#pragma unroll
      for (int k = 0; k < kMaxChunks; ++k) {
        const int c = tx + kTile * k;
        if (c < P) dst[c] = load_src<T, KIND, FIRST>(a, rowoff + colw[k]);
      }
    }
  }
  __syncthreads();
  filter_coefficients<T, NTH, R>(A, P, G, tid);
}

// Coefficient pass of the two-kernel step (whole-field B-spline coefficients into a.coef, read
// by the global-memory gather): the separable exponential filter runs along complete periodic
// rows (into a.coef2), then along columns, so that no output is computed twice.
// Rows: a block filters 'rpb' whole rows staged in LDS with K wrapped values on either side; a
// thread forms kRowSeg consecutive outputs from a register window of kRowSeg + 2K staged values.
// The staged rows carry one slack word after every kRowSeg values, so that the windows of
// consecutive threads (kRowSeg + 1 words apart) fall on different LDS banks.
constexpr int kRowSeg = 8;

__host__ __device__ inline int row_stage_len(int n2, int K) { return (n2 + kRowSeg - 1) / kRowSeg * kRowSeg + 2 * K; }
__host__ __device__ inline int row_stage_stride(int n2, int K) {
  const int W = row_stage_len(n2, K);
  return W + W / kRowSeg + 1;
}

template <typename T, int KIND, bool FIRST>
__global__ void __launch_bounds__(256) k_prefilter_rows(StepArgs<T> args, int rpb) {
  if (args.active && !args.active[blockIdx.z]) return;
  const StepArgs<T> a = item_view(args, blockIdx.z);
  constexpr int K = FilterTaps<T>::K;
  extern __shared__ unsigned char smem_raw[];
  T* L = reinterpret_cast<T*>(smem_raw);
  const int n1 = a.n1, n2 = a.n2;
  const int W = row_stage_len(n2, K), Wp = row_stage_stride(n2, K);
  const int nseg = (n2 + kRowSeg - 1) / kRowSeg;
  const int r0 = blockIdx.x * rpb;
  const int nr = min(rpb, n1 - r0);
  // loads of several iterations are issued before their stores (no loop-carried wait)
  for (int r = 0; r < nr; ++r) {
    const size_t rowoff = size_t(r0 + r) * n2;
    T* Lr = L + r * Wp;
#pragma unroll 4
    for (int c = threadIdx.x; c < W; c += 256) {
      int col = c - K;
      if (col < 0) col += n2;
      if (col >= n2) col -= n2;
      if (unsigned(col) >= unsigned(n2)) col = wrap_index(c - K, n2);  // rows shorter than K
      Lr[c + c / kRowSeg] = load_src<T, KIND, FIRST>(a, rowoff + col);
    }
  }
  __syncthreads();
  for (int task = threadIdx.x; task < nr * nseg; task += 256) {
    const int r = task / nseg, q = task - r * nseg;
    const T* xw = L + r * Wp + q * (kRowSeg + 1);
    T x[kRowSeg + 2 * K];
#pragma unroll
    for (int i = 0; i < kRowSeg + 2 * K; ++i) x[i] = xw[i + i / kRowSeg];
    T* out = a.coef2 + size_t(r0 + r) * n2 + q * kRowSeg;
    T y[kRowSeg];
    filter_window<T, kRowSeg, K>(x, y);
    // a lane's outputs are contiguous: 16-byte stores where the row length keeps them aligned
    if (n2 % kRowSeg == 0) {
      using V = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
      constexpr int PER = 16 / sizeof(T);
#pragma unroll
      for (int j = 0; j < kRowSeg; j += PER) {
        V v;
        T* vp = reinterpret_cast<T*>(&v);
#pragma unroll
        for (int e = 0; e < PER; ++e) vp[e] = y[j + e];
        *reinterpret_cast<V*>(out + j) = v;
      }
    } else {
#pragma unroll
      for (int j = 0; j < kRowSeg; ++j)
        if (q * kRowSeg + j < n2) out[j] = y[j];
    }
  }
}

// Columns: a block filters a panel of kColW columns over kColH rows (plus K wrapped rows above and
// below), each thread R consecutive rows of one column from a register window.
constexpr int kColW = 32, kColH = 64;

template <typename T>
__global__ void __launch_bounds__(256) k_prefilter_cols(StepArgs<T> args) {
  if (args.active && !args.active[blockIdx.z]) return;
  const StepArgs<T> a = item_view(args, blockIdx.z);
  constexpr int K = FilterTaps<T>::K;
  constexpr int R = kColH * kColW / 256;
  __shared__ T L[(kColH + 2 * K) * kColW];
  const int n1 = a.n1, n2 = a.n2;
  const int x0 = blockIdx.x * kColW, y0 = blockIdx.y * kColH;
#pragma unroll
  for (int idx = threadIdx.x; idx < (kColH + 2 * K) * kColW; idx += 256) {  // 256 threads per block
    const int r = idx / kColW, c = idx - r * kColW;
    const int col = min(x0 + c, n2 - 1);
    const T val = a.coef2[size_t(wrap_near(y0 - K + r, n1)) * n2 + col];
    L[idx] = x0 + c < n2 ? val : T(0);
  }
  __syncthreads();
  const int c = threadIdx.x % kColW, q = threadIdx.x / kColW;
  const int col = x0 + c;
  T x[R + 2 * K], o[R];
#pragma unroll
  for (int i = 0; i < R + 2 * K; ++i) x[i] = L[(q * R + i) * kColW + c];
  filter_window<T, R, K>(x, o);
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int row = y0 + q * R + j;
    if (row < n1 && col < n2) a.coef[size_t(row) * n2 + col] = o[j];
  }
}

// One-kernel coefficient pass (the two-kernel step's default): a block stages a TS x TS tile of
// the transported field with K wrapped values on every side in LDS, filters its rows (all PS
// staged rows, TS outputs each) and then its columns, and writes the TS x TS coefficients.  The
// halo re-reads hit L2 (tiles of one XCD are contiguous, as in the step kernels), so HBM sees the
// field once and the coefficients once.  R consecutive outputs per thread from register windows;
// odd LDS row strides keep consecutive threads on different banks.
template <typename T>
struct Prefilter2D {
  static constexpr int K = FilterTaps<T>::K;
  static constexpr int TS = sizeof(T) == 4 ? 64 : 32;  // output tile side
  static constexpr int PS = TS + 2 * K;                 // staged side
  static constexpr int SA = PS + 1, SB = TS + 1;        // LDS row strides (odd)
  static constexpr int R = 8;                           // outputs per thread and pass
  static constexpr int NT = 512;                        // threads per block
  static constexpr int KT = (PS * (TS / R) + NT - 1) / NT;  // row-pass tasks per thread
  // the row-filtered values overwrite the staged ones (after a barrier), so one buffer serves
  static constexpr size_t kLds = size_t(PS) * SA * sizeof(T);
  static_assert(SB <= SA, "row-filtered rows must fit the staged rows");
};

template <typename T, int KIND, bool FIRST>
__global__ void __launch_bounds__(Prefilter2D<T>::NT) k_prefilter_2d(StepArgs<T> args) {
  if (args.active && !args.active[blockIdx.z]) return;
  const StepArgs<T> a = item_view(args, blockIdx.z);
  using P2 = Prefilter2D<T>;
  constexpr int K = P2::K, TS = P2::TS, PS = P2::PS, SA = P2::SA, SB = P2::SB, R = P2::R, NT = P2::NT;
  extern __shared__ unsigned char smem_raw[];
  T* A = reinterpret_cast<T*>(smem_raw);  // [PS][SA] staged values
  T* B = A;                               // [PS][SB] row-filtered values, written over A
  const int n1 = a.n1, n2 = a.n2;
  int by, bx;
  xcd_tile(by, bx);
  const int y0 = by * TS, x0 = bx * TS;
  const int tid = threadIdx.x;
  // 1. stage: wavefront ty takes rows ty + SR i, its lane tx columns tx and tx + 64, so that the
  // wrapped row offsets and column indices are formed once per thread (the kernel is bound by its
  // instruction count, and a per-element division and wrap had been most of it); every load of
  // the thread is issued before any store (no per-load wait).  The grid is at least PS in both
  // directions (caller), so one add or subtract wraps an index.
  constexpr int SR = NT / 64, NRI = (PS + SR - 1) / SR, NCI = (PS + 63) / 64;
  const int tx = tid & 63, ty = tid >> 6;
  int gcol[NCI];
#pragma unroll
  for (int j = 0; j < NCI; ++j) {
    int gc = x0 - K + tx + 64 * j;
    gc += gc < 0 ? n2 : 0;
    gc -= gc >= n2 ? n2 : 0;
    gcol[j] = gc;
  }
  T v[NRI][NCI];
#pragma unroll
  for (int i = 0; i < NRI; ++i) {
    const int r = ty + SR * i;
    int gr = y0 - K + r;
    gr += gr < 0 ? n1 : 0;
    gr -= gr >= n1 ? n1 : 0;
    const size_t rowoff = size_t(gr) * n2;
#pragma unroll
    for (int j = 0; j < NCI; ++j)
      if (r < PS && tx + 64 * j < PS) v[i][j] = load_src<T, KIND, FIRST>(a, rowoff + gcol[j]);
  }
#pragma unroll
  for (int i = 0; i < NRI; ++i) {
    const int r = ty + SR * i;
#pragma unroll
    for (int j = 0; j < NCI; ++j)
      if (r < PS && tx + 64 * j < PS) A[r * SA + tx + 64 * j] = v[i][j];
  }
  __syncthreads();
  // 2. rows: task (row r, segment q), consecutive threads on consecutive rows; every task's
  // outputs stay in registers until all staged values are read
  T y[P2::KT][R];
#pragma unroll
  for (int k = 0; k < P2::KT; ++k) {
    const int task = tid + k * NT;
    if (task < PS * (TS / R)) {
      const int q = task / PS, r = task - q * PS;
      const T* src = A + r * SA + q * R;
      T x[R + 2 * K];
#pragma unroll
      for (int i = 0; i < R + 2 * K; ++i) x[i] = src[i];
      filter_window<T, R, K>(x, y[k]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < P2::KT; ++k) {
    const int task = tid + k * NT;
    if (task < PS * (TS / R)) {
      const int q = task / PS, r = task - q * PS;
#pragma unroll
      for (int j = 0; j < R; ++j) B[r * SB + q * R + j] = y[k][j];
    }
  }
  __syncthreads();
  // 3. columns: task (column c, segment q), consecutive threads on consecutive columns
  for (int task = tid; task < TS * (TS / R); task += NT) {
    const int q = task / TS, c = task - q * TS;
    const T* src = B + (q * R) * SB + c;
    T x[R + 2 * K], o[R];
#pragma unroll
    for (int i = 0; i < R + 2 * K; ++i) x[i] = src[i * SB];
    filter_window<T, R, K>(x, o);
    const int col = x0 + c;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int row = y0 + q * R + j;
      if (row < n1 && col < n2) a.coef[size_t(row) * n2 + col] = o[j];
    }
  }
}

// Thread rows TY of the fused step's 16 x 16 tile.  On launches of at most kWideBlocks blocks
// (grids up to 256^2 per item: about one tile per CU, latency-bound) two threads per node share
// the staging and the prefilter -- the step's longest phase runs one round of filter tasks
// instead of two, with two waves per SIMD to cover each other's LDS latency -- and the gather and
// update take the first 16 rows; larger launches keep 16 x 16 blocks, which fill the CUs better.
constexpr int kFusedRows = 2 * kTile;
// Largest halo the fused step takes: a tile of 16 x 16 nodes filters a (16 + 2 halo + 3 + 2K)^2
// footprint, which past about 8 cells costs more than the two-kernel step's extra coefficient
// pass (measured single-pair matvecs: 512^2 at halo 5, fused 0.19 vs 0.22 ms; 1024^2 at halo 13,
// fused 0.42 vs 0.22 ms).
constexpr int kFusedMaxHalo = 8;
constexpr long long kWideBlocks = 512;

template <typename T, int KIND, bool FIRST, bool GLOBAL, int TY = kTile>
__global__ void __launch_bounds__(kTile * TY) k_sl_step(StepArgs<T> args) {
  if (args.active && !args.active[blockIdx.z]) return;
  const StepArgs<T> a = item_view(args, blockIdx.z);
  extern __shared__ unsigned char smem_raw[];
  T* C = reinterpret_cast<T*>(smem_raw);
  constexpr bool kAdj = KIND == int(StepKind::Adjoint);
  constexpr bool kIncS = KIND == int(StepKind::IncState);
  constexpr bool kIncA = KIND == int(StepKind::IncAdjoint);
  // the footprint actually staged: the device-side bound when given (never above the bound the
  // LDS was sized for)
  const int D = a.halo_dev ? min(*a.halo_dev, a.halo) : a.halo;
  const int G = kTile + 2 * D + 3;
  const int n1 = a.n1, n2 = a.n2;
  const size_t F = size_t(n1) * n2;
  int by, bx;
  xcd_tile(by, bx);
  const int y0 = by * kTile, x0 = bx * kTile;
  const int i1 = y0 + threadIdx.y, i2 = x0 + threadIdx.x;
  const bool inside = threadIdx.y < kTile && i1 < n1 && i2 < n2;
  const size_t gi = inside ? size_t(i1) * n2 + i2 : 0;
  // per-node operands, loaded before the staging so that their latency overlaps it
  const T dd1 = a.d1[gi], dd2 = a.d1[gi + F];
  T gam = T(0), gn1 = T(0), gn2 = T(0), ac1 = T(0), ac2 = T(0), ex0 = T(0), ex1 = T(0), ex2 = T(0);
  if constexpr (kAdj || kIncA) gam = a.gamma[gi];
  if constexpr (kAdj || kIncS || kIncA) {
    gn1 = a.gm_new[gi];
    gn2 = a.gm_new[gi + F];
  }
  if constexpr ((kAdj && !FIRST) || kIncA) {
    ac1 = a.acc[gi];
    ac2 = a.acc[gi + F];
  }
  if constexpr (kIncS) {
    ex1 = a.vt[gi];
    ex2 = a.vt[gi + F];
  }
  if constexpr (kIncA) {
    if (a.addf) ex0 = a.addf[gi];  // full-Newton source term of this step
  }
  if constexpr (kAdj && FIRST) {
    ex0 = a.aux0[gi] - a.aux1[gi];  // lambda(1) at the node
    ac1 = a.gm_old[gi];
    ac2 = a.gm_old[gi + F];
  }
  if constexpr (KIND == int(StepKind::State)) {
    if (a.last) ex0 = a.aux0[gi];
  }
  if constexpr (kAdj) {
    if (a.last && a.addf) {  // no addend: the caller adds beta A v after projecting b
      ex1 = a.addf[gi];
      ex2 = a.addf[gi + F];
    }
  }
  if constexpr (!GLOBAL) stage_coefficients<T, KIND, FIRST, TY>(a, C, y0, x0, D + 1, G);

  // gather at the departure point of this thread's node and update
  double red_s = 0.0, red_m = 0.0;
  if (inside) {
    const T s1 = T(i1) + dd1, s2 = T(i2) + dd2;
    T u = T(0);
    if constexpr (GLOBAL) {
      u = interp_global(a.coef, n1, n2, s1, s2);
    } else {
      const T f1 = floor(s1), f2 = floor(s2);
      T w1[4], w2[4];
      bspline_w(s1 - f1, w1);
      bspline_w(s2 - f2, w2);
      // LDS coordinates of the first stencil row/column (region origin y0 - D - 1); the clamp
      // is inactive whenever |d| <= D, which the caller guarantees
      int l1 = int(f1) - y0 + D;
      int l2 = int(f2) - x0 + D;
      l1 = min(max(l1, 0), G - 4);
      l2 = min(max(l2, 0), G - 4);
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const T* row = C + (l1 + p) * G + l2;
        u += w1[p] * (w2[0] * row[0] + w2[1] * row[1] + w2[2] * row[2] + w2[3] * row[3]);
      }
    }
    if constexpr (KIND == int(StepKind::State)) {
      a.dst[gi] = u;
      if (a.last) {
        const double r = double(u) - double(ex0);
        red_s = r * r;
      }
    } else if constexpr (kAdj) {
      const T lam = gam * u;
      if (a.dst) a.dst[gi] = lam;
      T b1 = T(a.w_new) * lam * gn1;
      T b2 = T(a.w_new) * lam * gn2;
      if constexpr (FIRST) {
        b1 += T(a.w_old) * ex0 * ac1;
        b2 += T(a.w_old) * ex0 * ac2;
      } else {
        b1 += ac1;
        b2 += ac2;
      }
      if (a.last) {
        const T g1 = ex1 + b1, g2 = ex2 + b2;
        a.out2[gi] = g1;
        a.out2[gi + F] = g2;
        red_s = double(g1) * double(g1) + double(g2) * double(g2);
        red_m = fmax(fabs(double(g1)), fabs(double(g2)));
      } else {
        a.acc[gi] = b1;
        a.acc[gi + F] = b2;
      }
    } else if constexpr (kIncS) {
      const T fnew = -(ex1 * gn1 + ex2 * gn2);
      const T mt = u + T(0.5 * a.ht) * fnew;  // m~^j
      if (a.out2) a.out2[gi] = mt;             // kept for the full-Newton matvec
      if (!a.last) {
        a.dst[gi] = u + T(a.ht) * fnew;  // q^j = m~^j + (ht/2) f^j
      } else {
        const T lt = -mt;  // lambda~(1) = -m~(1)
        a.dst[gi] = lt;
        a.acc[gi] = T(a.w_new) * lt * gn1;
        a.acc[gi + F] = T(a.w_new) * lt * gn2;
      }
    } else {  // IncAdjoint (ex0: the full-Newton source term, else 0)
      const T lt = gam * u + ex0;
      if (a.dst) a.dst[gi] = lt;
      a.acc[gi] = ac1 + T(a.w_new) * lt * gn1;
      a.acc[gi + F] = ac2 + T(a.w_new) * lt * gn2;
    }
  }
  if (a.partial && a.last) block_sum_max(red_s, red_m, a.partial);
}

template <typename T>
size_t step_lds_bytes(int G) {
  const int P = G + 2 * FilterTaps<T>::K;
  const int R = FilterTaps<T>::R;
  return size_t(P * P + R + (P + R) * G) * sizeof(T);
}

std::atomic<size_t> g_lds_limit{0};

hipError_t lds_limit(size_t* out) {
  if (g_lds_limit.load(std::memory_order_acquire) == 0) {
    int dev = 0, v = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess) return e;
    g_lds_limit.store(size_t(v), std::memory_order_release);
  }
  *out = g_lds_limit.load(std::memory_order_acquire);
  return hipSuccess;
}

// ------------------------------------------------------------------------------------------
// Heun trace of both characteristics + adjoint factor
// ------------------------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_trace(int n1, int n2, const int* active, T ht, const T* __restrict__ vb,
                                               const T* __restrict__ cvb, const T* __restrict__ divvb,
                                               const T* __restrict__ cdivb, T* __restrict__ dfb,
                                               T* __restrict__ dab, T* __restrict__ gammab, double* partialb) {
  const int z = blockIdx.z;
  if (active && !active[z]) return;
  const size_t F = size_t(n1) * n2;
  const T* v = vb + 2 * F * z;
  const T* cv = cvb + 2 * F * z;
  const T* divv = divvb + F * z;
  const T* cdiv = cdivb + F * z;
  T* df = dfb + 2 * F * z;
  T* da = dab + 2 * F * z;
  T* gamma = gammab + F * z;
  double* partial = partialb ? partialb + size_t(z) * 2 * gridDim.x * gridDim.y : nullptr;
  int by, bx;
  xcd_tile(by, bx);
  const int i1 = by * kTile + threadIdx.y, i2 = bx * kTile + threadIdx.x;
  double red_s = 0.0, red_m = 0.0;
  if (i1 < n1 && i2 < n2) {
    const size_t gi = size_t(i1) * n2 + i2;
    // velocity in cells per unit time
    const T c1 = T(n1) / T(2.0 * 3.14159265358979323846), c2 = T(n2) / T(2.0 * 3.14159265358979323846);
    const T u1 = v[gi] * c1, u2 = v[gi + F] * c2;
    const T* cv1 = cv;
    const T* cv2 = cv + F;
    // forward characteristic: X* = x - ht v(x); X_f = x - ht/2 (v(x) + v(X*))
    T s1 = T(i1) - ht * u1, s2 = T(i2) - ht * u2;
    T w1 = interp_global(cv1, n1, n2, s1, s2) * c1, w2 = interp_global(cv2, n1, n2, s1, s2) * c2;
    const T f1 = -T(0.5) * ht * (u1 + w1), f2 = -T(0.5) * ht * (u2 + w2);
    // adjoint characteristic: the same with +ht
    s1 = T(i1) + ht * u1;
    s2 = T(i2) + ht * u2;
    w1 = interp_global(cv1, n1, n2, s1, s2) * c1;
    w2 = interp_global(cv2, n1, n2, s1, s2) * c2;
    const T e1 = T(0.5) * ht * (u1 + w1), e2 = T(0.5) * ht * (u2 + w2);
    df[gi] = f1;
    df[gi + F] = f2;
    da[gi] = e1;
    da[gi + F] = e2;
    const T dD = interp_global(cdiv, n1, n2, T(i1) + e1, T(i2) + e2);
    const T dx = divv[gi];
    gamma[gi] = T(1) + T(0.5) * ht * (dD + dx) + T(0.5) * ht * ht * dD * dx;
    red_m = fmax(fmax(fabs(double(f1)), fabs(double(f2))), fmax(fabs(double(e1)), fabs(double(e2))));
  }
  if (partial) block_sum_max(red_s, red_m, partial);
}

}  // namespace

template <typename T>
int sl_step_max_halo() {
  size_t lim = 0;
  if (lds_limit(&lim) != hipSuccess) return -1;
  int D = -1;
  auto fits = [&](int d) {
    const int G = kTile + 2 * d + 3;
    return step_lds_bytes<T>(G) <= lim && G + 2 * FilterTaps<T>::K <= kTile * kMaxChunks;
  };
  while (D < 64 && fits(D + 1)) ++D;
  return D;
}

template <typename T, int KIND, bool FIRST, int TY>
hipError_t launch_fused(hipStream_t s, const StepArgs<T>& a, dim3 grid) {
  const size_t lds = step_lds_bytes<T>(kTile + 2 * a.halo + 3);
  auto kfn = k_sl_step<T, KIND, FIRST, false, TY>;
  static std::atomic<size_t> attr_set{0};  // largest dynamic LDS size allowed for this kernel
  if (lds > attr_set.load(std::memory_order_acquire)) {
    std::lock_guard<std::mutex> lock(g_setup_mutex);
    if (lds > attr_set.load(std::memory_order_relaxed)) {
      hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kfn),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
      if (e != hipSuccess) return e;
      attr_set.store(lds, std::memory_order_release);
    }
  }
  hipLaunchKernelGGL(kfn, grid, dim3(kTile, TY), lds, s, a);
  return hipGetLastError();
}

template <typename T, int KIND, bool FIRST>
hipError_t launch_step(hipStream_t s, const StepArgs<T>& a, dim3 grid, dim3 block, bool fused) {
  if (fused) {
    const bool wide = a.fused_rows == kFusedRows ||
                      (a.fused_rows == 0 && (long long)grid.x * grid.y * grid.z <= kWideBlocks);
    if (wide) return launch_fused<T, KIND, FIRST, kFusedRows>(s, a, grid);
    return launch_fused<T, KIND, FIRST, kTile>(s, a, grid);
  } else if (!a.two_pass_coef && a.n1 >= Prefilter2D<T>::PS && a.n2 >= Prefilter2D<T>::PS) {
    using P2 = Prefilter2D<T>;
    static std::atomic<size_t> attr2{0};
    if (P2::kLds > 64 * 1024 && attr2.load(std::memory_order_acquire) < P2::kLds) {
      std::lock_guard<std::mutex> lock(g_setup_mutex);
      if (attr2.load(std::memory_order_relaxed) < P2::kLds) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_prefilter_2d<T, KIND, FIRST>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, int(P2::kLds));
        if (e != hipSuccess) return e;
        attr2.store(P2::kLds, std::memory_order_release);
      }
    }
    hipLaunchKernelGGL((k_prefilter_2d<T, KIND, FIRST>),
                       dim3((a.n2 + P2::TS - 1) / P2::TS, (a.n1 + P2::TS - 1) / P2::TS, a.batch), dim3(P2::NT), P2::kLds,
                       s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_sl_step<T, KIND, FIRST, true>), grid, block, 0, s, a);
  } else {
    constexpr int K = FilterTaps<T>::K;
    // a few thousand staged values per block, at most 48 KiB of LDS, and fewer rows per block when
    // that keeps about 2048 blocks in flight (small batches: each row's loads are one round trip)
    const int Wp = row_stage_stride(a.n2, K);
    const int rows_all = a.n1 * a.batch;
    const int rpb = std::max(1, std::min(std::min(4096 / a.n2, int((48 * 1024) / (Wp * sizeof(T)))), rows_all / 2048));
    const size_t lds = size_t(rpb) * Wp * sizeof(T);
    hipLaunchKernelGGL((k_prefilter_rows<T, KIND, FIRST>), dim3((a.n1 + rpb - 1) / rpb, 1, a.batch), dim3(256), lds,
                       s, a, rpb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_prefilter_cols<T>, dim3((a.n2 + kColW - 1) / kColW, (a.n1 + kColH - 1) / kColH, a.batch),
                       dim3(256), 0, s, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_sl_step<T, KIND, FIRST, true>), grid, block, 0, s, a);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t sl_step(hipStream_t s, StepKind kind, const StepArgs<T>& a, int* nblocks_out) {
  hipError_t e = upload_taps();
  if (e != hipSuccess) return e;
  const int maxh = std::min(sl_step_max_halo<T>(), kFusedMaxHalo);
  if (a.halo < 0) return hipErrorInvalidValue;
  const bool fused = a.halo <= maxh && !a.force_global;
  if (!fused && (a.coef == nullptr || a.coef2 == nullptr)) return hipErrorInvalidValue;
  dim3 grid((a.n2 + kTile - 1) / kTile, (a.n1 + kTile - 1) / kTile, a.batch);
  dim3 block(kTile, kTile);
  if (nblocks_out) *nblocks_out = int(grid.x * grid.y);
  if (a.batch < 1) return hipErrorInvalidValue;
  switch (kind) {
    case StepKind::State:
      return launch_step<T, 0, false>(s, a, grid, block, fused);
    case StepKind::Adjoint:
      return a.first ? launch_step<T, 1, true>(s, a, grid, block, fused)
                     : launch_step<T, 1, false>(s, a, grid, block, fused);
    case StepKind::IncState:
      return a.first ? launch_step<T, 2, true>(s, a, grid, block, fused)
                     : launch_step<T, 2, false>(s, a, grid, block, fused);
    case StepKind::IncAdjoint:
      return launch_step<T, 3, false>(s, a, grid, block, fused);
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t sl_trace(hipStream_t s, int n1, int n2, int batch, const int* active, double ht, const T* v, const T* cv,
                    const T* divv, const T* cdiv, T* df, T* da, T* gamma, double* partial, int* nblocks_out) {
  dim3 grid((n2 + kTile - 1) / kTile, (n1 + kTile - 1) / kTile, batch);
  dim3 block(kTile, kTile);
  if (nblocks_out) *nblocks_out = int(grid.x * grid.y);
  hipLaunchKernelGGL(k_trace<T>, grid, block, 0, s, n1, n2, active, T(ht), v, cv, divv, cdiv, df, da, gamma,
                     partial);
  return hipGetLastError();
}

template int sl_step_max_halo<float>();
template int sl_step_max_halo<double>();
template hipError_t sl_step<float>(hipStream_t, StepKind, const StepArgs<float>&, int*);
template hipError_t sl_step<double>(hipStream_t, StepKind, const StepArgs<double>&, int*);
template hipError_t sl_trace<float>(hipStream_t, int, int, int, const int*, double, const float*, const float*,
                                    const float*, const float*, float*, float*, float*, double*, int*);
template hipError_t sl_trace<double>(hipStream_t, int, int, int, const int*, double, const double*, const double*,
                                     const double*, const double*, double*, double*, double*, double*, int*);

}  // namespace slnk
