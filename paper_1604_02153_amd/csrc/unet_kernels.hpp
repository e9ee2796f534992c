// Host-side launchers of the U-Net kernels (unet.hip).  Every launcher enqueues on the given
// stream and returns the launch status; none of them synchronises or allocates.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>

namespace slnk {
namespace unet {

typedef unsigned short bf16;  // bfloat16 bit pattern

// 3x3 periodic convolution as an implicit GEMM on BF16 MFMA.  Input view: x + pixel * xcs + xco,
// cin channels; weights w[9][cout][cin] (tap t = 3 (dy + 1) + (dx + 1) reads pixel (y + dy,
// x + dx)); output y + pixel * ycs + yco (BF16, optional) and/or v[b][c][pixel] (FP32, channels
// c < nv, optional).  Two optional outputs come from the same BF16 values: yp, their 2x2 average
// pooling on the [H/2][W/2] grid (the same sums, in the same order, as pool()), and yu, their
// nearest upsampling on the [2H][2W] grid (as up()).  cin, cout multiples of 32; H even, W a
// multiple of 8, H W a multiple of 64; P = batch * H * W.
struct ConvArgs {
  const bf16* x = nullptr;
  int xcs = 0, xco = 0, cin = 0;
  const bf16* w = nullptr;
  const float* bias = nullptr;
  int cout = 0, relu = 0;
  bf16* y = nullptr;
  int ycs = 0, yco = 0;
  bf16* yp = nullptr;
  int ypcs = 0, ypco = 0;
  bf16* yu = nullptr;
  int yucs = 0, yuco = 0;
  float* v = nullptr;
  int nv = 0;
  int H = 0, W = 0, P = 0;
};
hipError_t conv(hipStream_t s, const ConvArgs& a);
// Launches of at least this many blocks take the LDS-tiled kernel (when the shape allows it).
constexpr long kLdsConvMinBlocks = 512;
// Process-wide counts of the convolution launches per kernel variant since the last reset:
// out[3 (mw - 1) + j], mw = pixel tiles of 16 or 32 (1, 2), j = 0, 1, 2 for K split 1, 2, 4 ways;
// out[6], out[7]: the LDS-tiled kernel with 32 or 64 output channels per block.
constexpr int kConvVariants = 8;
void conv_variant_counts(long long out[kConvVariants], bool reset);

// Weight-gradient partials: partial[z][t][co][ci] = sum over pixel chunk z of
// dy[p][co] * x[p + d_t][ci]; wgrad_splits(P, chunk) chunks (chunk a multiple of 128).
struct WgradArgs {
  const bf16* dy = nullptr;
  int dcs = 0, dco = 0, cout = 0;
  const bf16* x = nullptr;
  int xcs = 0, xco = 0, cin = 0;
  int H = 0, W = 0, P = 0, chunk = 0;
  float* partial = nullptr;
};
int wgrad_splits(int P, int chunk);
hipError_t wgrad(hipStream_t s, const WgradArgs& a);
// bias-gradient partials partial[z][c] over (P + chunk - 1) / chunk chunks
hipError_t bgrad(hipStream_t s, const bf16* dy, int dcs, int dco, int C, int P, int chunk, float* partial);
// out[i] = sum_z partial[z * n + i]
hipError_t sum_splits(hipStream_t s, const float* partial, int splits, size_t n, float* out);
// wd[t][ci][co] = w[8 - t][co][ci]
hipError_t wtrans(hipStream_t s, const bf16* w, int cout, int cin, bf16* wd);
// dy *= (y > 0), C channels of P pixels
hipError_t relu_mask(hipStream_t s, bf16* dy, int dcs, int dco, const bf16* y, int ycs, int yco, int C, int P);
// gradient of the 2x2 average pooling (of a [B][H][W] view into [B][H/2][W/2]) added into dx
hipError_t pool_bwd_add(hipStream_t s, const bf16* dy, int dcs, int dco, bf16* dx, int xcs, int xco, int C, int B,
                        int H, int W);
// gradient of the nearest upsampling of a [B][H][W] view into [B][2H][2W]
hipError_t up_bwd(hipStream_t s, const bf16* dy, int dcs, int dco, bf16* dx, int xcs, int xco, int C, int B, int H,
                  int W);
// input tensor (m_R, m_T, m_R - m_T, zeros) with C channels from FP32 images of P pixels
hipError_t prep(hipStream_t s, const float* mr, const float* mt, bf16* x, int C, size_t P);
// mean squared error of v against tgt ([B][2][HW] FP32), its gradient into dv (C channels, BF16)
// and the loss into *out (device); partial holds loss_blocks(B HW) doubles
int loss_blocks(size_t P);
hipError_t loss(hipStream_t s, const float* v, const float* tgt, int B, int HW, int C, bf16* dv, double* partial,
                double* out);
// one Adam step (bias-corrected, step >= 1) on n FP32 parameters, BF16 mirror updated
hipError_t adam(hipStream_t s, float* w, bf16* wb, const float* g, float* m, float* v, size_t n, double lr, double b1,
                double b2, double eps, long long step);
hipError_t to_bf16(hipStream_t s, const float* w, bf16* wb, size_t n);
// scalar head on the pixel mean and maximum of a [B][HW][C] BF16 tensor: f [B][2C] = (means,
// maxima), out[b] = bias + f[b] . w (w: 2C values); head_grad: the gradient of
// mean_b (out[b] - y[b])^2 with respect to w and bias, given the feature count 2C (+ the loss)
hipError_t head(hipStream_t s, const bf16* x, int C, int HW, int B, const float* w, const float* bias, float* f,
                float* out);
hipError_t head_grad(hipStream_t s, const float* f, const float* out, const float* y, int B, int C, float* gw,
                     float* gb, double* loss);

}  // namespace unet
}  // namespace slnk
