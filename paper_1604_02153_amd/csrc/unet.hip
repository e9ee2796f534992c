// Convolutional U-Net kernels on the gfx950 BF16 matrix cores (warm start of the Newton--Krylov
// solve; a form added to the paper's method).  Activations are NHWC BF16 ("views": base pointer,
// channels per pixel, channel offset, so that a concatenation is two views into one tensor),
// weights are [tap][out][in] BF16 with FP32 master copies, accumulation is FP32.
//
// Convolutions are 3x3 with periodic (circular) padding -- the images live on the torus -- and
// run as implicit GEMMs on v_mfma_f32_16x16x32_bf16: M = output pixels, N = output channels,
// K = 9 taps x input channels.  Lane l of a wavefront supplies row l%16 and the eight K values
// 8(l/16)..8(l/16)+7 of the A tile, column l%16 and the same K values of the B tile, and receives
// rows 4(l/16)..4(l/16)+3 of column l%16 of the 16x16 result.
#include "unet_kernels.hpp"

#include <atomic>

namespace slnk {
namespace unet {
namespace {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(bf16 h) { return __uint_as_float(unsigned(h) << 16); }
// round to nearest even (finite values)
__device__ __forceinline__ bf16 f2bf(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return bf16(u >> 16);
}

__device__ __forceinline__ v8bf load8(const bf16* p) { return *reinterpret_cast<const v8bf*>(p); }

__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// ---- convolution (forward, and input gradient with transformed weights) ----------------------
// Epilogue of one lane's share of a 16 x 16 MFMA result: the four values of the 2 x 2 pixel block
// at rows y0, y0 + 1 and columns xb, xb + 1 of image pb, output channel co.  Adds the bias, applies
// the ReLU, stores the BF16 output, its 2 x 2 average (the same BF16 values summed in the order of
// the pooling) and its four upsampled copies, and the FP32 values of the first nv channels.
__device__ __forceinline__ void conv_store(const ConvArgs& a, int pb, int y0, int xb, int co, v4f acc) {
  const int HW = a.H * a.W;
  const float bias = a.bias ? a.bias[co] : 0.f;
  float pooled = 0.f;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int yq = y0 + (q >> 1), xq = xb + (q & 1);
    const size_t p = size_t(pb) * HW + size_t(yq) * a.W + xq;
    float v = acc[q] + bias;
    if (a.relu) v = fmaxf(v, 0.f);
    const bf16 h = f2bf(v);
    pooled += bf2f(h);
    if (a.y) a.y[p * a.ycs + a.yco + co] = h;
    if (a.yu) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const size_t pu = (size_t(pb) * 2 * a.H + 2 * yq + (u >> 1)) * (2 * a.W) + 2 * xq + (u & 1);
        a.yu[pu * a.yucs + a.yuco + co] = h;
      }
    }
    if (a.v && co < a.nv) a.v[(size_t(pb) * a.nv + co) * HW + size_t(yq) * a.W + xq] = v;
  }
  if (a.yp) {
    const size_t po = (size_t(pb) * (a.H >> 1) + (y0 >> 1)) * (a.W >> 1) + (xb >> 1);
    a.yp[po * a.ypcs + a.ypco + co] = f2bf(0.25f * pooled);
  }
}

// Block: four wavefronts.  KS of them (1, 2 or 4) share one output tile of 16 MW pixels x 32
// output channels (MW x 2 MFMA tiles) and split its K = 9 taps x cin/32 channel chunks between
// them; their partial sums meet in LDS and are added in a fixed order.  Small grids (the deep
// levels: few pixels, many channels) take KS > 1 so that enough wavefronts run.  The K loop is
// flat over (tap, chunk) and unrolled, so the loads of several steps are in flight together.
// An output tile is a patch of 2 rows x 8 MW columns: row m of MFMA tile i is the pixel
// (y0 + (m >> 1 & 1), x0 + 8 i + 2 (m >> 2) + (m & 1)), so the four results a lane receives
// (rows 4g .. 4g + 3) form one 2 x 2 block, which the epilogue pools in registers.
template <int MW, int KS>
__global__ void __launch_bounds__(256) k_conv(ConvArgs a) {
  constexpr int PG = 4 / KS;  // output tiles per block
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kpart = wave % KS, pg = wave / KS;
  const int r = lane & 15, g = lane >> 4;
  const int HW = a.H * a.W;
  const int pw = a.W / (8 * MW);       // patches per row pair
  const int npi = (a.H >> 1) * pw;     // patches per image
  const int pt = blockIdx.x * PG + pg;
  const int pb = pt / npi;
  const int prem = pt - pb * npi;
  const int prow = prem / pw;
  const int y0 = 2 * prow, x0 = 8 * MW * (prem - prow * pw);
  const int cobase = blockIdx.y * 32;
  int py[MW], px[MW];
#pragma unroll
  for (int i = 0; i < MW; ++i) {
    py[i] = y0 + ((r >> 1) & 1);
    px[i] = x0 + 8 * i + 2 * (r >> 2) + (r & 1);
  }
  v4f acc[MW][2];
#pragma unroll
  for (int i = 0; i < MW; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
  // this wavefront's K steps st = kpart + KS i (i < nmy), st = 9-tap index t times nk plus the
  // 32-channel chunk kc; the loads run four steps ahead of the MFMAs (a ring of four register
  // buffers); steps past the end load a valid step and multiply it by zero weights
  const int nk = a.cin >> 5;
  const int S = 9 * nk;
  const int nmy = (S - kpart + KS - 1) / KS;
  const float inv_nk = 1.0f / float(nk);
  auto load_step = [&](int i, v8bf* av, v8bf* bv) {
    const int st = kpart + KS * min(i, nmy - 1);
    const int t = int((float(st) + 0.5f) * inv_nk);
    const int kc = st - t * nk;
    const int dy = t / 3 - 1, dx = t - 3 * (t / 3) - 1;
#pragma unroll
    for (int m = 0; m < MW; ++m) {
      const int yy = wrap(py[m] + dy, a.H), xx = wrap(px[m] + dx, a.W);
      av[m] = load8(a.x + (size_t(pb) * HW + size_t(yy) * a.W + xx) * a.xcs + a.xco + 8 * g + 32 * kc);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j)
      bv[j] = load8(a.w + (size_t(t) * a.cout + cobase + 16 * j + r) * a.cin + 8 * g + 32 * kc);
  };
  v8bf ra[4][MW], rb[4][2];
#pragma unroll
  for (int q = 0; q < 4; ++q) load_step(q, ra[q], rb[q]);
  const v8bf zero = {};
  for (int i = 0; i < nmy; i += 4) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const bool live = i + q < nmy;
#pragma unroll
      for (int m = 0; m < MW; ++m)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[m][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ra[q][m], live ? rb[q][j] : zero, acc[m][j], 0, 0, 0);
      load_step(i + q + 4, ra[q], rb[q]);
    }
  }
  if constexpr (KS > 1) {
    __shared__ v4f red[4][MW * 2][64];
    if (kpart > 0) {
#pragma unroll
      for (int i = 0; i < MW; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) red[wave][2 * i + j][lane] = acc[i][j];
    }
    __syncthreads();
    if (kpart > 0) return;
#pragma unroll
    for (int q = 1; q < KS; ++q)
#pragma unroll
      for (int i = 0; i < MW; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] += red[wave + q][2 * i + j][lane];
  }
#pragma unroll
  for (int i = 0; i < MW; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) conv_store(a, pb, y0, x0 + 8 * i + 2 * g, cobase + 16 * j + r, acc[i][j]);
}

// LDS-tiled variant for large launches.  A block computes 2 rows x TW columns of pixels x NC output
// channels (NC = 64: 2 x 2 wavefronts over pixels x channels, TW = 32; NC = 32: 4 x 1, TW = 64);
// each wavefront holds 2 x 2 MFMA tiles (two 2 x 8 pixel patches x 32 channels).  For each chunk of
// 32 input channels the block stages the input's 4 x (TW + 2) halo patch (periodic) and the nine
// taps' weights for its NC channels in LDS once, and every tap then reads its operands there: each
// input value serves nine taps and NC channels, each weight 2 TW pixels.  Operands are 16-byte LDS
// reads at the same lane layout as k_conv (so the same epilogue applies).
template <int NC>
__global__ void __launch_bounds__(256) k_conv_lds(ConvArgs a) {
  constexpr int WM = NC == 64 ? 2 : 4;  // wavefronts along the pixels
  constexpr int TW = 16 * WM;           // tile width in pixels
  constexpr int IW = TW + 2;            // staged halo width
  __shared__ __attribute__((aligned(16))) bf16 sIn[4 * IW * 32];
  __shared__ __attribute__((aligned(16))) bf16 sW[9 * NC * 32];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = lane & 15, g = lane >> 4;
  const int wm = wave % WM, wn = wave / WM;
  const int HW = a.H * a.W;
  const int tpr = a.W / TW;                 // tiles per row pair
  const int tpi = (a.H >> 1) * tpr;         // tiles per image
  const int tile = blockIdx.x;
  const int pb = tile / tpi;
  const int trem = tile - pb * tpi;
  const int prow = trem / tpr;
  const int y0 = 2 * prow, x0 = TW * (trem - prow * tpr);
  const int cobase = blockIdx.y * NC;
  const size_t img = size_t(pb) * HW;
  // this lane's pixel of M-tile i (tile coordinates): row (r >> 1) & 1, column 16 wm + 8 i + 2 (r >> 2) + (r & 1)
  int aoff[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int ly = (r >> 1) & 1, lx = 16 * wm + 8 * i + 2 * (r >> 2) + (r & 1);
    aoff[i] = ((ly + 1) * IW + (lx + 1)) * 32 + 8 * g;  // centre tap; tap (dy, dx) adds (dy IW + dx) 32
  }
  int boff[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) boff[j] = (32 * (WM == 2 ? wn : 0) + 16 * j + r) * 32 + 8 * g;
  v4f acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
  const int nk = a.cin >> 5;
  for (int kc = 0; kc < nk; ++kc) {
    __syncthreads();  // the previous chunk's operands are no longer read
    // input halo: 4 rows x IW columns x 4 vectors of 8 channels
    for (int e = tid; e < 4 * IW * 4; e += 256) {
      const int part = e & 3, pix = e >> 2;
      const int row = pix / IW, col = pix - row * IW;
      const int yy = wrap(y0 - 1 + row, a.H), xx = wrap(x0 - 1 + col, a.W);
      *reinterpret_cast<uint4*>(sIn + pix * 32 + 8 * part) = *reinterpret_cast<const uint4*>(
          a.x + (img + size_t(yy) * a.W + xx) * a.xcs + a.xco + 32 * kc + 8 * part);
    }
    // weights: 9 taps x NC channels x 4 vectors of 8 input channels
    for (int e = tid; e < 9 * NC * 4; e += 256) {
      const int part = e & 3, tc = e >> 2;
      const int t = tc / NC, co = tc - t * NC;
      *reinterpret_cast<uint4*>(sW + tc * 32 + 8 * part) = *reinterpret_cast<const uint4*>(
          a.w + (size_t(t) * a.cout + cobase + co) * a.cin + 32 * kc + 8 * part);
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int shift = ((t / 3 - 1) * IW + (t % 3 - 1)) * 32;
      v8bf av[2], bv[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) av[i] = load8(sIn + aoff[i] + shift);
#pragma unroll
      for (int j = 0; j < 2; ++j) bv[j] = load8(sW + t * NC * 32 + boff[j]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
      conv_store(a, pb, y0, x0 + 16 * wm + 8 * i + 2 * g, cobase + 32 * (WM == 2 ? wn : 0) + 16 * j + r, acc[i][j]);
}

// ---- weight gradient ----------------------------------------------------------------------------
// Partial sums over one pixel chunk of dW[t][co][ci] = sum_p dY[p][co] X[p + d_t][ci] for a 32x32
// (co, ci) tile and one tap; 128-pixel slabs are staged in LDS transposed to [channel][pixel] so
// that every lane reads eight consecutive pixels of one channel.
constexpr int kSlab = 128;
constexpr int kSlabPad = kSlab + 8;  // row stride: keeps 16-byte alignment, spreads LDS banks

__global__ void __launch_bounds__(256) k_wgrad(WgradArgs a) {
  __shared__ bf16 sD[32][kSlabPad];
  __shared__ bf16 sX[32][kSlabPad];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 15, g = lane >> 4;
  const int wy = wave >> 1, wx = wave & 1;
  const int nci = a.cin / 32;
  const int co0 = (blockIdx.x / nci) * 32, ci0 = (blockIdx.x % nci) * 32;
  const int t = blockIdx.y, dy = t / 3 - 1, dx = t % 3 - 1;
  const int p0 = blockIdx.z * a.chunk;
  const int p1 = min(a.P, p0 + a.chunk);
  const int HW = a.H * a.W;
  v4f acc = {0.f, 0.f, 0.f, 0.f};
  for (int ps = p0; ps < p1; ps += kSlab) {
#pragma unroll
    for (int rep = 0; rep < 2; ++rep) {
      const int idx = threadIdx.x + 256 * rep;  // 128 pixels x 4 groups of 8 channels
      const int pl = idx >> 2, c8 = (idx & 3) * 8;
      const int p = ps + pl;
      uint4 dv = {0u, 0u, 0u, 0u}, xv = {0u, 0u, 0u, 0u};
      if (p < p1) {
        dv = *reinterpret_cast<const uint4*>(a.dy + size_t(p) * a.dcs + a.dco + co0 + c8);
        const int b = p / HW, rem = p - b * HW;
        const int y = rem / a.W, x = rem - (rem / a.W) * a.W;
        const int yy = wrap(y + dy, a.H), xx = wrap(x + dx, a.W);
        xv = *reinterpret_cast<const uint4*>(a.x + (size_t(b) * HW + size_t(yy) * a.W + xx) * a.xcs + a.xco + ci0 +
                                              c8);
      }
      const bf16* dh = reinterpret_cast<const bf16*>(&dv);
      const bf16* xh = reinterpret_cast<const bf16*>(&xv);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        sD[c8 + e][pl] = dh[e];
        sX[c8 + e][pl] = xh[e];
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kSlab; kk += 32) {
      const v8bf av = load8(&sD[16 * wy + r][kk + 8 * g]);
      const v8bf bv = load8(&sX[16 * wx + r][kk + 8 * g]);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int co = co0 + 16 * wy + 4 * g + q, ci = ci0 + 16 * wx + r;
    a.partial[((size_t(blockIdx.z) * 9 + t) * a.cout + co) * a.cin + ci] = acc[q];
  }
}

// bias gradient partials: partial[z][c] = sum over chunk z of dY[p][c].  Thread (pixel group pg,
// channels 4 c4 .. 4 c4 + 3) sums every G-th pixel of the chunk (8-byte loads, several in
// flight); the G group sums meet in LDS in a fixed order.  C is a multiple of 4 and at most 1024.
__global__ void __launch_bounds__(256) k_bgrad(const bf16* dy, int dcs, int dco, int C, int P, int chunk,
                                               float* partial) {
  __shared__ float red[256 * 4];
  const int tpp = C / 4, G = 256 / tpp;
  const int c4 = threadIdx.x % tpp, pg = threadIdx.x / tpp;
  const int p0 = blockIdx.x * chunk, p1 = min(P, p0 + chunk);
  float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
  if (pg < G) {
#pragma unroll 8
    for (int p = p0 + pg; p < p1; p += G) {
      const uint2 u = *reinterpret_cast<const uint2*>(dy + size_t(p) * dcs + dco + 4 * c4);
      s0 += __uint_as_float(u.x << 16);
      s1 += __uint_as_float(u.x & 0xFFFF0000u);
      s2 += __uint_as_float(u.y << 16);
      s3 += __uint_as_float(u.y & 0xFFFF0000u);
    }
    red[pg * C + 4 * c4 + 0] = s0;
    red[pg * C + 4 * c4 + 1] = s1;
    red[pg * C + 4 * c4 + 2] = s2;
    red[pg * C + 4 * c4 + 3] = s3;
  }
  __syncthreads();
  for (int c = threadIdx.x; c < C; c += blockDim.x) {
    float t = 0.f;
    for (int q = 0; q < G; ++q) t += red[q * C + c];
    partial[size_t(blockIdx.x) * C + c] = t;
  }
}

// out[i] = sum_z partial[z][i] (fixed order), i < n
__global__ void k_sum_splits(const float* partial, int splits, size_t n, float* out) {
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) {
    float s = 0.f;
#pragma unroll 8
    for (int z = 0; z < splits; ++z) s += partial[size_t(z) * n + i];
    out[i] = s;
  }
}

// Wd[t][ci][co] = W[8 - t][co][ci]: the input gradient is the convolution of dY with the
// spatially flipped, channel-transposed kernel
__global__ void k_wtrans(const bf16* w, int cout, int cin, bf16* wd) {
  const size_t n = size_t(9) * cout * cin;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) {
    const int co = int(i % cout);
    const int ci = int((i / cout) % cin);
    const int t = int(i / (size_t(cout) * cin));
    wd[i] = w[(size_t(8 - t) * cout + co) * cin + ci];
  }
}

// dY[p][c] = 0 where Y[p][c] <= 0 (ReLU derivative), C channels of two views
__global__ void k_relu_mask(bf16* dy, int dcs, int dco, const bf16* y, int ycs, int yco, int C, int P) {
  const size_t n = size_t(P) * C;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) {
    const size_t p = i / C;
    const int c = int(i % C);
    if (!(bf2f(y[p * ycs + yco + c]) > 0.f)) dy[p * dcs + dco + c] = 0;
  }
}

// gradient of the pooling, accumulated: dX[2y+i][2x+j] += dY[y][x] / 4
__global__ void k_pool_bwd_add(const bf16* dy, int dcs, int dco, bf16* dx, int xcs, int xco, int C, int B, int H,
                               int W) {
  const size_t n = size_t(B) * H * W * C;  // input resolution
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) {
    const int c = int(i % C);
    const size_t p = i / C;
    const int x = int(p % W), y = int((p / W) % H), b = int(p / (size_t(W) * H));
    const float gsrc = bf2f(dy[((size_t(b) * (H / 2) + y / 2) * (W / 2) + x / 2) * dcs + dco + c]);
    bf16* d = dx + p * xcs + xco + c;
    *d = f2bf(bf2f(*d) + 0.25f * gsrc);
  }
}

// gradient of the upsampling: dX[y][x] = sum of the four dY it was copied to
__global__ void k_up_bwd(const bf16* dy, int dcs, int dco, bf16* dx, int xcs, int xco, int C, int B, int H, int W) {
  const size_t n = size_t(B) * H * W * C;  // low resolution
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) {
    const int c = int(i % C);
    const size_t p = i / C;
    const int x = int(p % W), y = int((p / W) % H), b = int(p / (size_t(W) * H));
    float s = 0.f;
    for (int dy2 = 0; dy2 < 2; ++dy2)
      for (int dx2 = 0; dx2 < 2; ++dx2)
        s += bf2f(dy[((size_t(b) * 2 * H + 2 * y + dy2) * 2 * W + 2 * x + dx2) * dcs + dco + c]);
    dx[p * xcs + xco + c] = f2bf(s);
  }
}

// network input: channels (m_R, m_T, m_R - m_T, 0, ...) of a C-channel tensor
// (C a multiple of 8: each pixel is written as C / 8 16-byte stores)
__global__ void k_prep(const float* mr, const float* mt, bf16* x, int C, size_t P) {
  for (size_t p = size_t(blockIdx.x) * blockDim.x + threadIdx.x; p < P; p += size_t(gridDim.x) * blockDim.x) {
    const float a = mr[p], b = mt[p];
    uint4* o = reinterpret_cast<uint4*>(x + p * C);
    o[0] = make_uint4(unsigned(f2bf(a)) | (unsigned(f2bf(b)) << 16), unsigned(f2bf(a - b)), 0u, 0u);
    for (int c = 1; c < C / 8; ++c) o[c] = make_uint4(0u, 0u, 0u, 0u);
  }
}

// loss = mean (v - target)^2 over B x 2 x H x W; gradient into the C-channel BF16 tensor dv
// (channels >= 2 zero); per-block FP64 partial sums
__global__ void __launch_bounds__(256) k_loss(const float* v, const float* tgt, int B, int HW, int C, bf16* dv,
                                              double* partial) {
  __shared__ double red[256];
  const size_t P = size_t(B) * HW;
  const float scale = 2.f / float(2 * P);
  double s = 0.0;
  for (size_t p = size_t(blockIdx.x) * blockDim.x + threadIdx.x; p < P; p += size_t(gridDim.x) * blockDim.x) {
    const size_t b = p / HW, q = p % HW;
    bf16* o = dv + p * C;
    for (int c = 0; c < 2; ++c) {
      const size_t k = (b * 2 + c) * HW + q;
      const float d = v[k] - tgt[k];
      s += double(d) * d;
      o[c] = f2bf(scale * d);
    }
    for (int c = 2; c < C; ++c) o[c] = 0;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void k_sum_double(const double* partial, int n, double scale, double* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += partial[i];
    *out = s * scale;
  }
}

// Adam (Kingma & Ba) on the FP32 master parameters, BF16 mirror written alongside
__global__ void k_adam(float* w, bf16* wb, const float* g, float* m, float* v, size_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    wb[i] = f2bf(wi);
  }
}

// scalar head: per item b, f[b][c] = mean and f[b][C + c] = max over the HW pixels of x[b][p][c]
// (C channels, FP32), s[b] = bias + sum_{c < 2C} f[b][c] w[c]; one block of 1024 threads per
// item.  Thread (pixel group pg, channels 4 c4 .. 4 c4 + 3) covers every G-th pixel with 8-byte
// loads, several in flight; the group results meet in LDS in a fixed order.  C is a multiple of
// 4 and at most 4096.
__global__ void __launch_bounds__(1024) k_head(const bf16* x, int C, int HW, const float* w, const float* bias,
                                               float* f, float* s) {
  __shared__ float rs[4096], rm[4096];
  __shared__ float red[1024];
  const int b = blockIdx.x;
  const int tpp = C / 4, G = 1024 / tpp;
  const int c4 = threadIdx.x % tpp, pg = threadIdx.x / tpp;
  if (pg < G) {
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
    float m0 = -3.0e38f, m1 = -3.0e38f, m2 = -3.0e38f, m3 = -3.0e38f;
#pragma unroll 8
    for (int p = pg; p < HW; p += G) {
      const uint2 u = *reinterpret_cast<const uint2*>(x + (size_t(b) * HW + p) * C + 4 * c4);
      const float v0 = __uint_as_float(u.x << 16), v1 = __uint_as_float(u.x & 0xFFFF0000u);
      const float v2 = __uint_as_float(u.y << 16), v3 = __uint_as_float(u.y & 0xFFFF0000u);
      a0 += v0;
      a1 += v1;
      a2 += v2;
      a3 += v3;
      m0 = fmaxf(m0, v0);
      m1 = fmaxf(m1, v1);
      m2 = fmaxf(m2, v2);
      m3 = fmaxf(m3, v3);
    }
    float* ps = rs + pg * 4 * tpp + 4 * c4;
    float* pm = rm + pg * 4 * tpp + 4 * c4;
    ps[0] = a0, ps[1] = a1, ps[2] = a2, ps[3] = a3;
    pm[0] = m0, pm[1] = m1, pm[2] = m2, pm[3] = m3;
  }
  __syncthreads();
  float part = 0.f;
  for (int c = threadIdx.x; c < C; c += blockDim.x) {
    float acc = 0.f, mx = -3.0e38f;
    for (int q = 0; q < G; ++q) {
      acc += rs[q * C + c];
      mx = fmaxf(mx, rm[q * C + c]);
    }
    const float fc = acc / float(HW);
    f[size_t(b) * 2 * C + c] = fc;
    f[size_t(b) * 2 * C + C + c] = mx;
    part += fc * w[c] + mx * w[C + c];
  }
  red[threadIdx.x] = part;
  __syncthreads();
  for (int k = 512; k > 0; k >>= 1) {
    if (int(threadIdx.x) < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) s[b] = red[0] + bias[0];
}

// gradient of mean_b (s[b] - y[b])^2 with respect to the head's weights and bias, and the loss
__global__ void __launch_bounds__(256) k_head_grad(const float* f, const float* s, const float* y, int B, int C,
                                                   float* gw, float* gb, double* loss) {
  for (int c = threadIdx.x; c < C; c += blockDim.x) {
    float acc = 0.f;
    for (int b = 0; b < B; ++b) acc += 2.f * (s[b] - y[b]) / float(B) * f[size_t(b) * C + c];
    gw[c] = acc;
  }
  if (threadIdx.x == 0) {
    float g = 0.f;
    double l = 0.0;
    for (int b = 0; b < B; ++b) {
      const float d = s[b] - y[b];
      g += 2.f * d / float(B);
      l += double(d) * d;
    }
    gb[0] = g;
    *loss = l / B;
  }
}

__global__ void k_to_bf16(const float* w, bf16* wb, size_t n) {
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
    wb[i] = f2bf(w[i]);
}

inline unsigned blocks_for(size_t n) {
  size_t b = (n + 255) / 256;
  return unsigned(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

}  // namespace

namespace {
std::atomic<long long> g_conv_launches[kConvVariants];
}

void conv_variant_counts(long long out[kConvVariants], bool reset) {
  for (int i = 0; i < kConvVariants; ++i)
    out[i] = reset ? g_conv_launches[i].exchange(0) : g_conv_launches[i].load();
}

hipError_t conv(hipStream_t s, const ConvArgs& a) {
  const int HW = a.H * a.W;
  if (a.cin % 32 || a.cout % 32 || a.xcs % 8 || a.xco % 8 || a.H % 2 || a.W % 8 || HW % 64 || a.P % HW)
    return hipErrorInvalidValue;
  // large launches: the LDS-tiled kernel (at least two blocks per compute unit)
  const int nc = a.cout % 64 == 0 && a.W % 32 == 0 ? 64 : (a.W % 64 == 0 ? 32 : 0);
  if (nc) {
    const long blocks = long(a.P / (2 * (nc == 64 ? 32 : 64))) * (a.cout / nc);
    if (blocks >= kLdsConvMinBlocks) {
      const dim3 grid(unsigned(a.P / (2 * (nc == 64 ? 32 : 64))), a.cout / nc);
      g_conv_launches[nc == 64 ? 7 : 6].fetch_add(1);
      if (nc == 64)
        hipLaunchKernelGGL((k_conv_lds<64>), grid, dim3(256), 0, s, a);
      else
        hipLaunchKernelGGL((k_conv_lds<32>), grid, dim3(256), 0, s, a);
      return hipGetLastError();
    }
  }
  // output tiles of 2 x 8 MW pixels x 32 channels; split K when they would not give about eight
  // wavefronts per compute unit
  const int mw = HW % 128 == 0 && a.W % 16 == 0 ? 2 : 1;
  const long tiles = long(a.P / (16 * mw)) * (a.cout / 32);
  const int ks = tiles >= 2048 ? 1 : tiles >= 1024 ? 2 : 4;
  const dim3 grid(a.P / (16 * mw * (4 / ks)), a.cout / 32);
  g_conv_launches[3 * (mw - 1) + (ks == 1 ? 0 : ks == 2 ? 1 : 2)].fetch_add(1);
  if (mw == 2) {
    if (ks == 1)
      hipLaunchKernelGGL((k_conv<2, 1>), grid, dim3(256), 0, s, a);
    else if (ks == 2)
      hipLaunchKernelGGL((k_conv<2, 2>), grid, dim3(256), 0, s, a);
    else
      hipLaunchKernelGGL((k_conv<2, 4>), grid, dim3(256), 0, s, a);
  } else {
    if (ks == 1)
      hipLaunchKernelGGL((k_conv<1, 1>), grid, dim3(256), 0, s, a);
    else if (ks == 2)
      hipLaunchKernelGGL((k_conv<1, 2>), grid, dim3(256), 0, s, a);
    else
      hipLaunchKernelGGL((k_conv<1, 4>), grid, dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

int wgrad_splits(int P, int chunk) { return (P + chunk - 1) / chunk; }

hipError_t wgrad(hipStream_t s, const WgradArgs& a) {
  if (a.cin % 32 || a.cout % 32 || a.xcs % 8 || a.xco % 8 || a.dcs % 8 || a.dco % 8 || a.chunk % kSlab)
    return hipErrorInvalidValue;
  const int splits = wgrad_splits(a.P, a.chunk);
  hipLaunchKernelGGL(k_wgrad, dim3((a.cout / 32) * (a.cin / 32), 9, splits), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t bgrad(hipStream_t s, const bf16* dy, int dcs, int dco, int C, int P, int chunk, float* partial) {
  if (C % 4 || C > 1024 || dcs % 4 || dco % 4) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_bgrad, dim3((P + chunk - 1) / chunk), dim3(256), 0, s, dy, dcs, dco, C, P, chunk, partial);
  return hipGetLastError();
}

hipError_t sum_splits(hipStream_t s, const float* partial, int splits, size_t n, float* out) {
  hipLaunchKernelGGL(k_sum_splits, dim3(blocks_for(n)), dim3(256), 0, s, partial, splits, n, out);
  return hipGetLastError();
}

hipError_t wtrans(hipStream_t s, const bf16* w, int cout, int cin, bf16* wd) {
  hipLaunchKernelGGL(k_wtrans, dim3(blocks_for(size_t(9) * cout * cin)), dim3(256), 0, s, w, cout, cin, wd);
  return hipGetLastError();
}

hipError_t relu_mask(hipStream_t s, bf16* dy, int dcs, int dco, const bf16* y, int ycs, int yco, int C, int P) {
  hipLaunchKernelGGL(k_relu_mask, dim3(blocks_for(size_t(P) * C)), dim3(256), 0, s, dy, dcs, dco, y, ycs, yco, C, P);
  return hipGetLastError();
}

hipError_t pool_bwd_add(hipStream_t s, const bf16* dy, int dcs, int dco, bf16* dx, int xcs, int xco, int C, int B,
                        int H, int W) {
  hipLaunchKernelGGL(k_pool_bwd_add, dim3(blocks_for(size_t(B) * H * W * C)), dim3(256), 0, s, dy, dcs, dco, dx, xcs,
                     xco, C, B, H, W);
  return hipGetLastError();
}

hipError_t up_bwd(hipStream_t s, const bf16* dy, int dcs, int dco, bf16* dx, int xcs, int xco, int C, int B, int H,
                  int W) {
  hipLaunchKernelGGL(k_up_bwd, dim3(blocks_for(size_t(B) * H * W * C)), dim3(256), 0, s, dy, dcs, dco, dx, xcs, xco, C,
                     B, H, W);
  return hipGetLastError();
}

hipError_t prep(hipStream_t s, const float* mr, const float* mt, bf16* x, int C, size_t P) {
  if (C % 8 || C < 8) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_prep, dim3(blocks_for(P)), dim3(256), 0, s, mr, mt, x, C, P);
  return hipGetLastError();
}

int loss_blocks(size_t P) { return int(blocks_for(P) > 1024 ? 1024 : blocks_for(P)); }

hipError_t loss(hipStream_t s, const float* v, const float* tgt, int B, int HW, int C, bf16* dv, double* partial,
                double* out) {
  const int nb = loss_blocks(size_t(B) * HW);
  hipLaunchKernelGGL(k_loss, dim3(nb), dim3(256), 0, s, v, tgt, B, HW, C, dv, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sum_double, dim3(1), dim3(64), 0, s, partial, nb, 1.0 / double(size_t(2) * B * HW), out);
  return hipGetLastError();
}

hipError_t adam(hipStream_t s, float* w, bf16* wb, const float* g, float* m, float* v, size_t n, double lr, double b1,
                double b2, double eps, long long step) {
  const double c1 = 1.0 - std::pow(b1, double(step)), c2 = 1.0 - std::pow(b2, double(step));
  hipLaunchKernelGGL(k_adam, dim3(blocks_for(n)), dim3(256), 0, s, w, wb, g, m, v, n, float(lr), float(b1), float(b2),
                     float(eps), float(c1), float(c2));
  return hipGetLastError();
}

hipError_t head(hipStream_t s, const bf16* x, int C, int HW, int B, const float* w, const float* bias, float* f,
                float* out) {
  if (C % 4 || C > 4096) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_head, dim3(B), dim3(1024), 0, s, x, C, HW, w, bias, f, out);
  return hipGetLastError();
}

hipError_t head_grad(hipStream_t s, const float* f, const float* out, const float* y, int B, int C, float* gw,
                     float* gb, double* loss) {
  hipLaunchKernelGGL(k_head_grad, dim3(1), dim3(256), 0, s, f, out, y, B, C, gw, gb, loss);
  return hipGetLastError();
}

hipError_t to_bf16(hipStream_t s, const float* w, bf16* wb, size_t n) {
  hipLaunchKernelGGL(k_to_bf16, dim3(blocks_for(n)), dim3(256), 0, s, w, wb, n);
  return hipGetLastError();
}

}  // namespace unet
}  // namespace slnk
