// Host side of the learned warm start: a periodic convolutional U-Net (encoder of `levels`
// resolutions with two 3x3 convolutions + ReLU each and 2x2 average pooling, decoder with nearest
// upsampling, concatenated skips and two 3x3 convolutions + ReLU, a linear 3x3 output
// convolution) mapping (m_R, m_T) to a velocity v_0 [2][H][W].  Training minimises the mean
// squared error against velocities produced by the solver itself, with Adam on FP32 master
// weights; activations and weights are BF16 on the matrix cores, sums are FP32.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/slnk.h"
#include "unet_kernels.hpp"
#include "unet_net.hpp"

namespace {

using slnk::unet::bf16;

constexpr int kInC = 32;          // channels of the network input (m_R, m_T, m_R - m_T, zero padding)
constexpr int kOutC = 32;         // padded output channels of the last convolution (2 used)
constexpr int kChunkW = 2048;     // pixels per weight-gradient partial
constexpr int kChunkB = 1024;     // pixels per bias-gradient partial

struct Fail {
  slnk_status st;
  std::string msg;
};

#define UCHK(expr)                                                                                   \
  do {                                                                                               \
    hipError_t _e = (expr);                                                                          \
    if (_e != hipSuccess) throw Fail{SLNK_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)}; \
  } while (0)

struct View {
  bf16* p = nullptr;
  int cs = 0, co = 0;
};

struct Layer {
  int cin = 0, cout = 0, relu = 1;
  int cin_real = 0, cout_real = 0;
  size_t woff = 0, boff = 0;
};

struct Tensor {
  bf16* p = nullptr;
  int C = 0, H = 0, W = 0;
  View at(int off = 0) const { return View{p, C, off}; }
};

}  // namespace

struct slnk_unet {
  std::string err;
  slnk_unet_params prm{};
  hipStream_t stream = nullptr;
  int L = 0;
  std::vector<int> C, Hs, Ws;
  std::vector<Layer> layers;
  std::vector<int> enc_a, enc_b, dec_a, dec_b;
  int out_layer = -1;
  size_t nparam = 0;
  // device memory: one allocation
  char* base = nullptr;
  size_t used = 0, cap = 0;
  float* w32 = nullptr;
  bf16* wbf = nullptr;
  float* grad = nullptr;
  float* m1 = nullptr;
  float* m2 = nullptr;
  bf16* wdg = nullptr;
  float* partial = nullptr;
  double* lpart = nullptr;
  double* dloss = nullptr;
  double* hloss = nullptr;
  float* vout = nullptr;
  long long step = 0, head_step = 0;
  // scalar head on the pixel mean and maximum of the bottleneck output: predicts
  // log(beta (e_max - 1)) of the two-level preconditioner's Chebyshev interval (its weights follow
  // the convolution layers)
  size_t trunk_n = 0, hw_off = 0, hb_off = 0;
  float* hf = nullptr;     // [max_batch][2 C_top] pooled features (means, maxima)
  float* hs = nullptr;     // [max_batch] head outputs
  double* hlossd = nullptr;
  // activations and their gradients
  Tensor in0, dv;
  std::vector<Tensor> pin, ea, cat, da, db;  // pin[l]: level input for l > 0 (pooled)
  Tensor eb;
  std::vector<Tensor> gpin, gea, gcat, gda, gdb;
  Tensor geb;

  template <typename U>
  U* take(size_t count) {
    const size_t bytes = (count * sizeof(U) + 255) / 256 * 256;
    if (used + bytes > cap) throw Fail{SLNK_ENOMEM, "U-Net arena exhausted"};
    U* p = reinterpret_cast<U*>(base + used);
    used += bytes;
    return p;
  }
  Tensor tensor(int Cc, int l, bool alloc) {
    Tensor t;
    t.C = Cc;
    t.H = Hs[l];
    t.W = Ws[l];
    if (alloc) t.p = take<bf16>(size_t(prm.max_batch) * t.H * t.W * Cc);
    return t;
  }
};

namespace {

int add_layer(slnk_unet& u, int cin, int cout, int relu, int cin_real, int cout_real) {
  Layer ly;
  ly.cin = cin;
  ly.cout = cout;
  ly.relu = relu;
  ly.cin_real = cin_real;
  ly.cout_real = cout_real;
  ly.woff = u.nparam;
  u.nparam += (size_t(9) * cout * cin + 63) / 64 * 64;
  ly.boff = u.nparam;
  u.nparam += (size_t(cout) + 63) / 64 * 64;
  u.layers.push_back(ly);
  return int(u.layers.size()) - 1;
}

void build(slnk_unet& u) {
  const auto& p = u.prm;
  u.L = p.levels;
  for (int l = 0; l < u.L; ++l) {
    u.C.push_back(p.base_channels << l);
    u.Hs.push_back(p.height >> l);
    u.Ws.push_back(p.width >> l);
  }
  const int L = u.L;
  u.enc_a.assign(L, -1);
  u.enc_b.assign(L, -1);
  u.dec_a.assign(L, -1);
  u.dec_b.assign(L, -1);
  for (int l = 0; l < L; ++l) {
    const int cin = l == 0 ? kInC : u.C[l - 1];
    u.enc_a[l] = add_layer(u, cin, u.C[l], 1, l == 0 ? 3 : cin, u.C[l]);
    u.enc_b[l] = add_layer(u, u.C[l], u.C[l], 1, u.C[l], u.C[l]);
  }
  for (int l = L - 2; l >= 0; --l) {
    const int cin = u.C[l + 1] + u.C[l];
    u.dec_a[l] = add_layer(u, cin, u.C[l], 1, cin, u.C[l]);
    u.dec_b[l] = add_layer(u, u.C[l], u.C[l], 1, u.C[l], u.C[l]);
  }
  u.out_layer = add_layer(u, u.C[0], kOutC, 0, u.C[0], 2);
  u.trunk_n = u.nparam;
  u.hw_off = u.nparam;
  u.nparam += (size_t(2 * u.C[L - 1]) + 63) / 64 * 64;
  u.hb_off = u.nparam;
  u.nparam += 64;
}

int level_of(const slnk_unet& u, int layer);

// largest weight tensor and largest gradient-partial buffer over the layers (each layer at its
// own resolution and the largest batch)
void scratch_need(const slnk_unet& u, size_t& wmax, size_t& part) {
  wmax = part = 0;
  for (size_t k = 0; k < u.layers.size(); ++k) {
    const auto& ly = u.layers[k];
    const int l = level_of(u, int(k));
    const int P = u.prm.max_batch * u.Hs[l] * u.Ws[l];
    wmax = std::max(wmax, size_t(9) * ly.cout * ly.cin);
    part = std::max(part, size_t(slnk::unet::wgrad_splits(P, kChunkW)) * 9 * ly.cout * ly.cin);
    part = std::max(part, size_t((P + kChunkB - 1) / kChunkB) * ly.cout);
  }
}

size_t plan_bytes(slnk_unet& u) {
  const size_t B = size_t(u.prm.max_batch);
  size_t act = 0;
  const int L = u.L;
  auto px = [&](int l) { return B * u.Hs[l] * u.Ws[l]; };
  act += px(0) * (kInC + kOutC);  // input, output gradient
  for (int l = 0; l < L; ++l) {
    act += 2 * px(l) * u.C[l];                                                     // ea + grad
    if (l > 0) act += 2 * px(l) * u.C[l - 1];                                      // pooled input + grad
    if (l < L - 1) act += 2 * px(l) * (u.C[l + 1] + u.C[l]) + 4 * px(l) * u.C[l];  // cat, da, db + grads
    else act += 2 * px(l) * u.C[l];                                                // bottleneck out + grad
  }
  size_t wmax, part;
  scratch_need(u, wmax, part);
  const size_t n = u.nparam;
  return act * sizeof(bf16) + n * (4 * sizeof(float) + sizeof(bf16)) + wmax * sizeof(bf16) + part * sizeof(float) +
         (slnk::unet::loss_blocks(px(0)) + 8) * sizeof(double) + px(0) * 2 * sizeof(float) + 64 * 256 +
         64 * 256 * size_t(4 * L + 8);
}

void allocate(slnk_unet& u) {
  const int L = u.L;
  u.w32 = u.take<float>(u.nparam);
  u.wbf = u.take<bf16>(u.nparam);
  u.grad = u.take<float>(u.nparam);
  u.m1 = u.take<float>(u.nparam);
  u.m2 = u.take<float>(u.nparam);
  size_t wmax, part;
  scratch_need(u, wmax, part);
  const int P0 = u.prm.max_batch * u.Hs[0] * u.Ws[0];
  u.wdg = u.take<bf16>(wmax);
  u.partial = u.take<float>(part);
  u.lpart = u.take<double>(slnk::unet::loss_blocks(size_t(P0)) + 8);
  u.dloss = u.lpart + slnk::unet::loss_blocks(size_t(P0));
  u.vout = u.take<float>(size_t(u.prm.max_batch) * 2 * u.Hs[0] * u.Ws[0]);
  u.hf = u.take<float>(size_t(u.prm.max_batch) * 2 * u.C[L - 1]);
  u.hs = u.take<float>(size_t(u.prm.max_batch));
  u.hlossd = u.take<double>(8);
  u.in0 = u.tensor(kInC, 0, true);
  u.dv = u.tensor(kOutC, 0, true);
  u.pin.resize(L);
  u.gpin.resize(L);
  u.ea.resize(L);
  u.gea.resize(L);
  u.cat.resize(L);
  u.gcat.resize(L);
  u.da.resize(L);
  u.gda.resize(L);
  u.db.resize(L);
  u.gdb.resize(L);
  for (int l = 0; l < L; ++l) {
    if (l > 0) {
      u.pin[l] = u.tensor(u.C[l - 1], l, true);
      u.gpin[l] = u.tensor(u.C[l - 1], l, true);
    }
    u.ea[l] = u.tensor(u.C[l], l, true);
    u.gea[l] = u.tensor(u.C[l], l, true);
    if (l < L - 1) {
      u.cat[l] = u.tensor(u.C[l + 1] + u.C[l], l, true);
      u.gcat[l] = u.tensor(u.C[l + 1] + u.C[l], l, true);
      u.da[l] = u.tensor(u.C[l], l, true);
      u.gda[l] = u.tensor(u.C[l], l, true);
      u.db[l] = u.tensor(u.C[l], l, true);
      u.gdb[l] = u.tensor(u.C[l], l, true);
    } else {
      u.eb = u.tensor(u.C[l], l, true);
      u.geb = u.tensor(u.C[l], l, true);
    }
  }
}

// He-uniform initialisation from a SplitMix64 stream (one draw per parameter index); padded
// channels stay zero, the output layer starts small so that v_0 starts near zero
void init_params(slnk_unet& u, std::vector<float>& h) {
  h.assign(u.nparam, 0.f);
  unsigned long long state = u.prm.seed;
  auto uniform = [&]() {
    state += 0x9E3779B97F4A7C15ULL;
    unsigned long long z = state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z = z ^ (z >> 31);
    return double(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
  };
  for (size_t k = 0; k < u.layers.size(); ++k) {
    const auto& ly = u.layers[k];
    double a = std::sqrt(6.0 / (9.0 * ly.cin_real));
    if (int(k) == u.out_layer) a *= 0.1;
    for (int t = 0; t < 9; ++t)
      for (int co = 0; co < ly.cout; ++co)
        for (int ci = 0; ci < ly.cin; ++ci) {
          const double r = uniform();
          if (co < ly.cout_real && ci < ly.cin_real)
            h[ly.woff + (size_t(t) * ly.cout + co) * ly.cin + ci] = float(a * r);
        }
  }
}

int level_of(const slnk_unet& u, int layer) {
  for (int l = 0; l < u.L; ++l)
    if (u.enc_a[l] == layer || u.enc_b[l] == layer || u.dec_a[l] == layer || u.dec_b[l] == layer) return l;
  return 0;  // output layer
}

// pooled / upsampled: further views that the convolution fills with the 2x2 average pooling or
// the nearest upsampling of its output (the next level's input, the decoder's concatenation)
void run_conv(slnk_unet& u, hipStream_t s, int layer, int B, View in, View out, float* v, int nv,
              View pooled = View{}, View upsampled = View{}) {
  const auto& ly = u.layers[layer];
  const int l = level_of(u, layer);
  slnk::unet::ConvArgs a;
  a.x = in.p;
  a.xcs = in.cs;
  a.xco = in.co;
  a.cin = ly.cin;
  a.w = u.wbf + ly.woff;
  a.bias = u.w32 + ly.boff;
  a.cout = ly.cout;
  a.relu = ly.relu;
  a.y = out.p;
  a.ycs = out.cs;
  a.yco = out.co;
  a.yp = pooled.p;
  a.ypcs = pooled.cs;
  a.ypco = pooled.co;
  a.yu = upsampled.p;
  a.yucs = upsampled.cs;
  a.yuco = upsampled.co;
  a.v = v;
  a.nv = nv;
  a.H = u.Hs[l];
  a.W = u.Ws[l];
  a.P = B * a.H * a.W;
  UCHK(slnk::unet::conv(s, a));
}

// backward of one convolution: gout = dL/d(output) (ReLU mask applied here when the layer has
// one), writes the weight and bias gradients and, when gin.p != nullptr, dL/d(input) into gin
void back_conv(slnk_unet& u, hipStream_t s, int layer, int B, View in, View outv, View gout, View gin) {
  const auto& ly = u.layers[layer];
  const int l = level_of(u, layer);
  const int H = u.Hs[l], W = u.Ws[l], P = B * H * W;
  if (ly.relu) UCHK(slnk::unet::relu_mask(s, gout.p, gout.cs, gout.co, outv.p, outv.cs, outv.co, ly.cout, P));
  slnk::unet::WgradArgs w;
  w.dy = gout.p;
  w.dcs = gout.cs;
  w.dco = gout.co;
  w.cout = ly.cout;
  w.x = in.p;
  w.xcs = in.cs;
  w.xco = in.co;
  w.cin = ly.cin;
  w.H = H;
  w.W = W;
  w.P = P;
  w.chunk = kChunkW;
  w.partial = u.partial;
  UCHK(slnk::unet::wgrad(s, w));
  UCHK(slnk::unet::sum_splits(s, u.partial, slnk::unet::wgrad_splits(P, kChunkW), size_t(9) * ly.cout * ly.cin,
                              u.grad + ly.woff));
  UCHK(slnk::unet::bgrad(s, gout.p, gout.cs, gout.co, ly.cout, P, kChunkB, u.partial));
  UCHK(slnk::unet::sum_splits(s, u.partial, (P + kChunkB - 1) / kChunkB, size_t(ly.cout), u.grad + ly.boff));
  if (gin.p) {
    UCHK(slnk::unet::wtrans(s, u.wbf + ly.woff, ly.cout, ly.cin, u.wdg));
    slnk::unet::ConvArgs a;
    a.x = gout.p;
    a.xcs = gout.cs;
    a.xco = gout.co;
    a.cin = ly.cout;
    a.w = u.wdg;
    a.cout = ly.cin;
    a.relu = 0;
    a.y = gin.p;
    a.ycs = gin.cs;
    a.yco = gin.co;
    a.H = H;
    a.W = W;
    a.P = P;
    UCHK(slnk::unet::conv(s, a));
  }
}

void forward(slnk_unet& u, hipStream_t s, int B, const float* mr, const float* mt, float* v, float* head_out) {
  const int L = u.L;
  UCHK(slnk::unet::prep(s, mr, mt, u.in0.p, kInC, size_t(B) * u.Hs[0] * u.Ws[0]));
  // pooling and upsampling run in the epilogues of the convolutions that produce their inputs:
  // enc_b[l] writes the skip and the pooled input of level l + 1; enc_b[L - 1] and dec_b[l]
  // write their output and its upsampling into the first channels of the concatenation one
  // level up
  for (int l = 0; l < L; ++l) {
    const View in = l == 0 ? u.in0.at() : u.pin[l].at();
    run_conv(u, s, u.enc_a[l], B, in, u.ea[l].at(), nullptr, 0);
    if (l < L - 1)
      run_conv(u, s, u.enc_b[l], B, u.ea[l].at(), u.cat[l].at(u.C[l + 1]), nullptr, 0, u.pin[l + 1].at());
    else
      run_conv(u, s, u.enc_b[l], B, u.ea[l].at(), u.eb.at(), nullptr, 0, View{}, u.cat[L - 2].at());
  }
  for (int l = L - 2; l >= 0; --l) {
    run_conv(u, s, u.dec_a[l], B, u.cat[l].at(), u.da[l].at(), nullptr, 0);
    run_conv(u, s, u.dec_b[l], B, u.da[l].at(), u.db[l].at(), nullptr, 0, View{},
             l > 0 ? u.cat[l - 1].at() : View{});
  }
  run_conv(u, s, u.out_layer, B, u.db[0].at(), View{}, v, 2);
  const int lt = L - 1;
  UCHK(slnk::unet::head(s, u.eb.p, u.C[lt], u.Hs[lt] * u.Ws[lt], B, u.w32 + u.hw_off, u.w32 + u.hb_off, u.hf,
                        head_out ? head_out : u.hs));
}

void backward(slnk_unet& u, hipStream_t s, int B) {
  const int L = u.L;
  back_conv(u, s, u.out_layer, B, u.db[0].at(), View{}, u.dv.at(), u.gdb[0].at());
  for (int l = 0; l <= L - 2; ++l) {
    back_conv(u, s, u.dec_b[l], B, u.da[l].at(), u.db[l].at(), u.gdb[l].at(), u.gda[l].at());
    back_conv(u, s, u.dec_a[l], B, u.cat[l].at(), u.da[l].at(), u.gda[l].at(), u.gcat[l].at());
    Tensor& glow = l == L - 2 ? u.geb : u.gdb[l + 1];
    UCHK(slnk::unet::up_bwd(s, u.gcat[l].p, u.gcat[l].C, 0, glow.p, glow.C, 0, u.C[l + 1], B, u.Hs[l + 1],
                            u.Ws[l + 1]));
  }
  for (int l = L - 1; l >= 0; --l) {
    if (l == L - 1) {
      back_conv(u, s, u.enc_b[l], B, u.ea[l].at(), u.eb.at(), u.geb.at(), u.gea[l].at());
    } else {
      const View gskip = u.gcat[l].at(u.C[l + 1]);
      UCHK(slnk::unet::pool_bwd_add(s, u.gpin[l + 1].p, u.gpin[l + 1].C, 0, gskip.p, gskip.cs, gskip.co, u.C[l], B,
                                    u.Hs[l], u.Ws[l]));
      back_conv(u, s, u.enc_b[l], B, u.ea[l].at(), u.cat[l].at(u.C[l + 1]), gskip, u.gea[l].at());
    }
    const View in = l == 0 ? u.in0.at() : u.pin[l].at();
    back_conv(u, s, u.enc_a[l], B, in, u.ea[l].at(), u.gea[l].at(), l == 0 ? View{} : u.gpin[l].at());
  }
}

template <class Fn>
slnk_status guard(slnk_unet* u, Fn&& fn) {
  if (!u) return SLNK_EINVAL;
  try {
    fn();
    return SLNK_OK;
  } catch (const Fail& e) {
    u->err = e.msg;
    return e.st;
  }
}

void check_batch(const slnk_unet& u, int B) {
  if (B < 1 || B > u.prm.max_batch) throw Fail{SLNK_EINVAL, "batch must be in [1, max_batch]"};
}

}  // namespace

int slnk_unet_start_kmax(const slnk_unet* u) { return u ? u->prm.start_kmax : 0; }

slnk_status slnk_unet_forward_on(slnk_unet* u, void* stream, int batch, int height, int width, const float* m_R,
                                 const float* m_T, float* v, float* head) {
  return guard(u, [&] {
    check_batch(*u, batch);
    if (height != u->prm.height || width != u->prm.width)
      throw Fail{SLNK_EINVAL, "the network was built for another grid size"};
    forward(*u, static_cast<hipStream_t>(stream), batch, m_R, m_T, v, head);
  });
}

extern "C" {

void slnk_unet_default_params(slnk_unet_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->height = p->width = 256;
  p->levels = 4;
  p->base_channels = 32;
  p->max_batch = 16;
  p->seed = 0xC0FFEE;
  p->start_kmax = 8;
}

slnk_status slnk_unet_create(const slnk_unet_params* p, void* hip_stream, slnk_unet** out) {
  if (!p || !out) return SLNK_EINVAL;
  *out = nullptr;
  if (p->levels < 2 || p->levels > 6 || p->base_channels < 32 || p->base_channels % 32 || p->max_batch < 1 ||
      p->max_batch > 4096 || p->height < 8 || p->width < 8 || p->start_kmax < 0)
    return SLNK_EINVAL;
  const int f = 1 << (p->levels - 1);
  if (p->height % f || p->width % f || ((p->height / f) * (p->width / f)) % 64) return SLNK_EINVAL;
  auto u = std::make_unique<slnk_unet>();
  u->prm = *p;
  u->stream = static_cast<hipStream_t>(hip_stream);
  build(*u);
  u->cap = plan_bytes(*u);
  if (hipMalloc(reinterpret_cast<void**>(&u->base), u->cap) != hipSuccess) return SLNK_ENOMEM;
  slnk_status st = guard(u.get(), [&] {
    UCHK(hipMemset(u->base, 0, u->cap));
    allocate(*u);
    UCHK(hipHostMalloc(reinterpret_cast<void**>(&u->hloss), 2 * sizeof(double), hipHostMallocDefault));
    std::vector<float> h;
    init_params(*u, h);
    UCHK(hipMemcpy(u->w32, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice));
    UCHK(slnk::unet::to_bf16(nullptr, u->w32, u->wbf, u->nparam));
    UCHK(hipDeviceSynchronize());
  });
  if (st != SLNK_OK) {
    if (u->hloss) (void)hipHostFree(u->hloss);
    (void)hipFree(u->base);
    return st;
  }
  *out = u.release();
  return SLNK_OK;
}

void slnk_unet_destroy(slnk_unet* u) {
  if (!u) return;
  if (u->hloss) (void)hipHostFree(u->hloss);
  if (u->base) (void)hipFree(u->base);
  delete u;
}

const char* slnk_unet_last_error(const slnk_unet* u) { return u ? u->err.c_str() : "null network"; }

long long slnk_unet_param_count(const slnk_unet* u) { return u ? (long long)u->nparam : 0; }

slnk_status slnk_unet_get_params(slnk_unet* u, float* host) {
  if (!host) return SLNK_EINVAL;
  return guard(u, [&] {
    UCHK(hipStreamSynchronize(u->stream));
    UCHK(hipMemcpy(host, u->w32, u->nparam * sizeof(float), hipMemcpyDeviceToHost));
  });
}

slnk_status slnk_unet_set_params(slnk_unet* u, const float* host) {
  if (!host) return SLNK_EINVAL;
  return guard(u, [&] {
    for (size_t i = 0; i < u->nparam; ++i)
      if (!std::isfinite(host[i])) throw Fail{SLNK_ENAN, "non-finite parameter"};
    UCHK(hipStreamSynchronize(u->stream));
    UCHK(hipMemcpy(u->w32, host, u->nparam * sizeof(float), hipMemcpyHostToDevice));
    UCHK(slnk::unet::to_bf16(u->stream, u->w32, u->wbf, u->nparam));
    UCHK(hipMemsetAsync(u->m1, 0, u->nparam * sizeof(float), u->stream));
    UCHK(hipMemsetAsync(u->m2, 0, u->nparam * sizeof(float), u->stream));
    UCHK(hipStreamSynchronize(u->stream));
    u->step = u->head_step = 0;
  });
}

slnk_status slnk_unet_get_grads(slnk_unet* u, float* host) {
  if (!host) return SLNK_EINVAL;
  return guard(u, [&] {
    UCHK(hipStreamSynchronize(u->stream));
    UCHK(hipMemcpy(host, u->grad, u->nparam * sizeof(float), hipMemcpyDeviceToHost));
  });
}

void slnk_unet_conv_variants(long long counts[8], int reset) {
  if (counts) slnk::unet::conv_variant_counts(counts, reset != 0);
}

slnk_status slnk_unet_forward(slnk_unet* u, int batch, const float* m_R, const float* m_T, float* v, float* head) {
  if (!m_R || !m_T || !v) return SLNK_EINVAL;
  return guard(u, [&] {
    check_batch(*u, batch);
    forward(*u, u->stream, batch, m_R, m_T, v, head);
  });
}

slnk_status slnk_unet_train_step(slnk_unet* u, int batch, const float* m_R, const float* m_T, const float* v_target,
                                 const float* head_target, double lr, double* loss, double* head_loss) {
  if (!m_R || !m_T || (!v_target && !head_target) || !(lr >= 0.0)) return SLNK_EINVAL;
  return guard(u, [&] {
    check_batch(*u, batch);
    hipStream_t s = u->stream;
    forward(*u, s, batch, m_R, m_T, u->vout, nullptr);
    if (v_target) {
      UCHK(slnk::unet::loss(s, u->vout, v_target, batch, u->Hs[0] * u->Ws[0], kOutC, u->dv.p, u->lpart, u->dloss));
      backward(*u, s, batch);
      ++u->step;
      if (lr > 0.0)
        UCHK(slnk::unet::adam(s, u->w32, u->wbf, u->grad, u->m1, u->m2, u->trunk_n, lr, 0.9, 0.999, 1e-8, u->step));
    }
    if (head_target) {
      // the head learns from the trunk's features; its loss does not flow back into the trunk
      const int lt = u->L - 1;
      UCHK(slnk::unet::head_grad(s, u->hf, u->hs, head_target, batch, 2 * u->C[lt], u->grad + u->hw_off,
                                 u->grad + u->hb_off, u->hlossd));
      ++u->head_step;
      const size_t o = u->hw_off, n = u->nparam - u->hw_off;
      if (lr > 0.0)
        UCHK(slnk::unet::adam(s, u->w32 + o, u->wbf + o, u->grad + o, u->m1 + o, u->m2 + o, n, lr, 0.9, 0.999, 1e-8,
                              u->head_step));
    }
    double h[2] = {0.0, 0.0};
    if (v_target) UCHK(hipMemcpyAsync(&u->hloss[0], u->dloss, sizeof(double), hipMemcpyDeviceToHost, s));
    if (head_target) UCHK(hipMemcpyAsync(&u->hloss[1], u->hlossd, sizeof(double), hipMemcpyDeviceToHost, s));
    UCHK(hipStreamSynchronize(s));
    if (v_target) h[0] = u->hloss[0];
    if (head_target) h[1] = u->hloss[1];
    if (!std::isfinite(h[0]) || !std::isfinite(h[1])) throw Fail{SLNK_ENAN, "non-finite training loss"};
    if (loss) *loss = h[0];
    if (head_loss) *head_loss = h[1];
  });
}

}  // extern "C"
