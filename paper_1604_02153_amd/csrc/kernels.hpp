// Host-side launchers of the gfx950 kernels.  Every launcher enqueues on the given stream and
// returns the launch status; none of them synchronises or allocates.
#pragma once

#include "common.hpp"

namespace slnk {

constexpr int kFFTMaxStages = 16;

// Factorisation of one transform length into radix-8/4/2/3/5 stages plus its twiddle table
// (device memory, computed on the host in FP64): stage s, radix R, p = product of the earlier
// radices, holds exp(-2 pi i j k / (p R)) at twoff[s] + (j - 1) p + k (j = 1..R-1, k < p);
// ntw = n - 1 values in all.  'roots' holds exp(-2 pi i m / n), m < n (device memory, same
// precision), for the wave-level transforms of the common lengths.
struct FFTPlanDev {
  int n = 0;
  int nstages = 0;
  int radix[kFFTMaxStages] = {0};
  int twoff[kFFTMaxStages] = {0};
  int ntw = 0;
  const void* tw = nullptr;
  const void* roots = nullptr;
};

// Grid description passed to every spectral launcher.
template <typename T>
struct SpecGrid {
  int n1 = 0, n2 = 0;      // real-space grid
  FFTPlanDev row;          // length n2 transforms (along x2, contiguous)
  FFTPlanDev col;          // length n1 transforms (along x1, strided)
  int nh() const { return n2 / 2 + 1; }        // columns of a half spectrum
  int nhp() const { return spec_stride(n2); }   // their row stride
  size_t field() const { return size_t(n1) * size_t(n2); }
  size_t spec() const { return size_t(n1) * size_t(nhp()); }
};

// Scalar symbols applied by spec_scale (all real and even in k).
enum class Symbol : int {
  Reg = 0,        // beta a(k), a = |k|^(2 reg)
  RegInv = 1,     // 1 / (beta a'(k)), a' = a with a(0) replaced by 1   (P_REG^{-1})
  RegInvSqrt = 2, // (beta a'(k))^{-1/2}                                  (split step S)
  LowPass = 3,    // 1 for |k1| < n1/4 and |k2| < n2/4, else 0
  HighPass = 4,   // 1 - LowPass
  Spline = 5,     // 1 / (B1(k1) B2(k2)), B(k) = (2 + cos(2 pi k / n)) / 3  (B-spline prefilter)
  Cutoff = 6,     // 1 for k1^2 + k2^2 <= kmax^2, else 0 (smooth part of a field)
  One = 7,        // 1
};

// proj = 1: a symbol applied to a vector field (two fields) first projects it onto divergence-free
// fields, b - k (k . b) / |k|^2 per wavenumber (the Leray operator K of the incompressible case,
// section 3.1; odd-order wavenumbers, Nyquist components zero, the mean kept)
struct SymbolParams {
  Symbol kind = Symbol::Reg;
  int reg = 2;
  double beta = 1.0;
  int kmax = 0;
  int proj = 0;
};

// Largest dynamic LDS (bytes) a spectral launch on an n1 x n2 grid asks for.
template <typename T>
size_t spec_lds_bytes(int n1, int n2);

// ---- spectral operators (each: row forward, column forward + symbol + column inverse, row inverse)
// All operate on 'batch' same-size items; per item the fields are consecutive (nf fields of
// field() elements) and items follow each other.  'active' (optional, [batch]) skips items.
// Scratch spectra: S1, S2 hold batch * (fields per item) * spec() complex.
//
// out = symbol(in) + (add ? add : 0), nf = 1 or 2 fields per item.  TF is the fields' element
// type: float fields through the FP64 transform (T = double) read FP32 input, form the symbol and
// the sum in FP64 and round once on the store (the mixed context's beta A); otherwise TF = T.
// (the addend takes no part in deducing TF, so that it may be passed as nullptr)
template <typename U>
struct NoDeduce {
  using type = U;
};
template <typename T, typename TF = T>
hipError_t spec_scale(hipStream_t s, const SpecGrid<T>& g, int batch, const int* active, SymbolParams sym, int nf,
                      const TF* in, TF* out, const typename NoDeduce<TF>::type* add, cplx<T>* S1, cplx<T>* S2);

// out1 = sym1(in), out2 = sym2(in) for vector fields (two fields per item): one forward transform.
// S1 >= 2 batch spec(), S2 >= 4 batch spec().
template <typename T>
hipError_t spec_scale2(hipStream_t s, const SpecGrid<T>& g, int batch, const int* active, SymbolParams sym1,
                       SymbolParams sym2, const T* in, T* out1, T* out2, cplx<T>* S1, cplx<T>* S2);

// Spectral divergence of 'count' consecutive vector fields w[c] (two fields, stride 2 field()):
// out[c] = d1 w1 + d2 w2 with stride field().  S1 >= 2 count spec(), S2 >= count spec().
template <typename T>
hipError_t spec_div(hipStream_t s, const SpecGrid<T>& g, int count, const T* w, T* out, cplx<T>* S1, cplx<T>* S2);

// Spatial derivatives of a stabilised RK2 stage for 'count' consecutive blocks of three fields
// (u, w1, w2), stride 3 field(): out block = (d1 u, d2 u, d1 w1 + d2 w2).  S1, S2 >= 3 count spec().
template <typename T>
hipError_t spec_rk2a(hipStream_t s, const SpecGrid<T>& g, int count, const T* in, T* out, cplx<T>* S1, cplx<T>* S2);

// Vectors of one Chebyshev step on M = I + S Q S (item stride 2 field(), coefficients per item)
template <typename T>
struct ChebTail {
  T* r;
  T* d;
  T* x;
  T* u;
  T* y;
  const double* c1;
  const double* c2;
};

// true when the grid takes the wave-level transform passes (both lengths in the fast set)
template <typename T>
bool spec_fast(const SpecGrid<T>& g);

// spec_scale2 with sym1 = S, sym2 = S^2 of in = Q y, followed by the Chebyshev step of cheb_step on
// ct in the same pass (sb and s2b are never stored).  Fast grids only (else hipErrorNotSupported);
// items with active[z] == 0 are left untouched.  S1 >= 2 batch spec(), S2 >= 4 batch spec().
template <typename T>
hipError_t spec_scale2_cheb(hipStream_t s, const SpecGrid<T>& g, int batch, const int* active, SymbolParams sym1,
                            SymbolParams sym2, const T* in, ChebTail<T> ct, cplx<T>* S1, cplx<T>* S2);

// Spectral gradient of 'count' consecutive scalar fields m[c] (stride field()): gm[c] = (d1 m, d2 m)
// with stride 2 field().  S1 >= count spec(), S2 >= 2 count spec().
template <typename T>
hipError_t spec_grad(hipStream_t s, const SpecGrid<T>& g, int count, const T* m, T* gm, cplx<T>* S1, cplx<T>* S2);

// Per item, from v (two fields): spline coefficients cv (two fields), div v and the spline
// coefficients of div v.  S1 >= 2 batch spec(), S2 >= 4 batch spec().
template <typename T>
hipError_t spec_trace_prep(hipStream_t s, const SpecGrid<T>& g, int batch, const int* active, const T* v, T* cv,
                           T* divv, T* cdiv, cplx<T>* S1, cplx<T>* S2);

// Spectral restriction of nf fields per item to the grid gc (n/2): the modes |k_i| < n_i/4
// survive.  If keep_fine != nullptr the fine spectrum (after both forward passes) is also
// stored there (batch * nf * spec() complex) for a later prolong_combine.  Scratch: S1 (fine),
// Sc1/Sc2 (coarse), batch * nf spectra each.
template <typename T>
hipError_t spec_restrict(hipStream_t s, const SpecGrid<T>& g, const SpecGrid<T>& gc, int batch, const int* active,
                         int nf, const T* in, T* out_c, cplx<T>* keep_fine, cplx<T>* S1, cplx<T>* Sc1, cplx<T>* Sc2);

// out = HighPass(fine spectrum kept by spec_restrict) + Prolong(zc): the two-level combine.
template <typename T>
hipError_t spec_prolong_combine(hipStream_t s, const SpecGrid<T>& g, const SpecGrid<T>& gc, int batch,
                                const int* active, int nf, const cplx<T>* fine_k, const T* zc, T* out, cplx<T>* S1,
                                cplx<T>* Sc1, cplx<T>* Sc2);

// ---- semi-Lagrangian transport ---------------------------------------------------------
// Displacements are stored in cells: departure point of node i is i + d (per axis).
enum class StepKind : int {
  State = 0,      // dst = I[src](X_f)
  Adjoint = 1,    // dst = gamma I[src](X_a); b (+)= ht w lam grad m
  IncState = 2,   // incremental state (see transport.hip)
  IncAdjoint = 3, // dst = gamma I[src](X_a) (+ addf: full-Newton source); bt += ht w lam~ grad m
};

// Arguments of one SL time step of B same-size items (image pairs).  Every pointer addresses item
// 0; item z uses pointer + z * (that pointer's stride, in elements).
template <typename T>
struct StepArgs {
  int n1 = 0, n2 = 0;
  int batch = 1;             // items B (blockIdx.z)
  const int* active = nullptr;  // optional [B] mask: items with 0 are skipped
  int halo = 0;              // bound D on |displacement| in cells: sizes the LDS footprint
  const int* halo_dev = nullptr;  // optional [B] device copy of each item's actual bound (<= halo),
                                  // read by the kernel so captured graphs stay valid across
                                  // linearisations
  const T* src = nullptr;    // field transported (nullptr with a 'first' source, see below)
  T* dst = nullptr;
  const T* d1 = nullptr;     // displacement fields (cells); d2 = d1 + n1 n2
  const T* gamma = nullptr;  // adjoint step factor
  // first-step sources (src == nullptr): Adjoint: aux0 - aux1 (m_R - m(1)); IncState:
  // (ht/2) f(vt, gm_old)
  const T* aux0 = nullptr;
  const T* aux1 = nullptr;
  const T* gm_new = nullptr; // 2 fields, grad m at the time level being produced
  const T* gm_old = nullptr; // 2 fields, grad m at the time level of src (first step only)
  T* acc = nullptr;          // 2 fields accumulator (b or bt)
  const T* vt = nullptr;     // incremental state: direction (2 fields)
  const T* addf = nullptr;   // adjoint last step: beta A v added to the accumulator (2 fields,
                             // optional);
                             // incremental adjoint: source term added to gamma I[src] (1 field)
  T* out2 = nullptr;         // adjoint last step: gradient output (2 fields); incremental
                             // state: m~^j (1 field, optional)
  T* coef = nullptr;         // one-field scratch: coefficients of the two-kernel (global gather) step
  T* coef2 = nullptr;        // one-field scratch: row-filtered values of that coefficient pass
  int two_pass_coef = 0;     // coefficient pass as rows + columns through coef2 (else one 2-D pass)
  long long st_src = 0, st_dst = 0, st_d = 0, st_gamma = 0, st_aux0 = 0, st_aux1 = 0, st_gm = 0,
            st_acc = 0, st_vt = 0, st_addf = 0, st_out2 = 0, st_coef = 0, st_coef2 = 0;
  double ht = 0;
  double w_new = 0;          // trapezoid weight of the produced level (times ht)
  double w_old = 0;          // trapezoid weight of the src level (first step only)
  int first = 0, last = 0;
  int force_global = 0;      // 1: coefficient pass + global gather even when the halo fits LDS
  int fused_rows = 0;        // threads per tile column of the fused step: 16 or 32 (0: by launch size)
  double* partial = nullptr; // FP64 per-block partial sums, item z at partial + z * 2 * tiles
                             // (state last step: misfit; adjoint last step: sum g^2, max |g|)
};

// Maximum halo (in cells) the fused LDS step supports for a given precision on this device.
// Larger halos run as a coefficient pass into a.coef followed by a global-memory gather.
template <typename T>
int sl_step_max_halo();

// One SL time step of every item.  Partial sums (when a.partial and a.last) of item z go to
// partial[z * 2 * tiles + 2 * block + {0, 1}]; *nblocks_out receives the tiles per item.
template <typename T>
hipError_t sl_step(hipStream_t s, StepKind kind, const StepArgs<T>& a, int* nblocks_out);

// Heun trace of both characteristics at once, for B items.  Per item: v, cv (spline
// coefficients of v), df, da are 2 fields (item stride 2F); divv, cdiv (div v and its
// coefficients), gamma are one field (stride F).  partial[z * 2 * tiles + 2 block + 1] = max |d|.
template <typename T>
hipError_t sl_trace(hipStream_t s, int n1, int n2, int batch, const int* active, double ht, const T* v,
                    const T* cv, const T* divv, const T* cdiv, T* df, T* da, T* gamma, double* partial,
                    int* nblocks_out);

// ---- reductions and vector updates -------------------------------------------------------
// Two-stage deterministic FP64 reductions over 'batch' items of n elements each (item stride n):
// per-block partials (reduce_blocks(n) blocks per item, 4 slots each), then one block per item
// that combines them in a fixed order.  'partial' needs 4 * batch * reduce_blocks(n) doubles;
// item z's results land at result[4 z + c] (device memory).
int reduce_blocks(size_t n);
// result[4z] = a.b
template <typename T>
hipError_t dot(hipStream_t s, int batch, size_t n, const T* a, const T* b, double* partial, double* result);
// result[4z + {0,1,2}] = {a.a, a.b, b.b}
template <typename T>
hipError_t dot3(hipStream_t s, int batch, size_t n, const T* a, const T* b, double* partial, double* result);
// result[4z + {0,1,2}] = {sum a^2, max |a|, number of non-finite entries}
template <typename T>
hipError_t norms(hipStream_t s, int batch, size_t n, const T* a, double* partial, double* result);
// combine 'ncomp' components of partial[z * per_item + stride * block + c] for each item z into
// result[4 z + c]: component c is a max if bit c of maxmask is set, else a sum
hipError_t finish(hipStream_t s, int batch, int nparts, int stride, long long per_item, int ncomp, unsigned maxmask,
                  const double* partial, double* result);

// Per item z (n elements each): y = (a * ad[z]) x + (b * bd[z]) y, with ad / bd optional [batch]
// device arrays (nullptr: 1).  An operand whose coefficient is zero is not read, and an item with
// coefficients (0, 1) is left untouched.
template <typename T>
hipError_t axpby(hipStream_t s, int batch, size_t n, double a, const double* ad, const T* x, double b,
                 const double* bd, T* y);
// One step of the Chebyshev iteration on M = I + S Q S carrying y = S d and u = S r, per item z
// (n elements each), given sb = S Q y and s2b = S^2 Q y:
//   r -= d + sb;  u -= y + s2b;  d = c1[z] d + c2[z] r;  y = c1[z] y + c2[z] u;  x += d
template <typename T>
hipError_t cheb_step(hipStream_t s, int batch, size_t n, const double* c1, const double* c2, T* r, T* u, T* d, T* y,
                     T* x, const T* sb, const T* s2b);

// z = x + a y over n elements (one item or all items)
template <typename T>
hipError_t xpay(hipStream_t s, size_t n, const T* x, double a, const T* y, T* z);
template <typename T>
hipError_t fill(hipStream_t s, size_t n, double value, T* y);
// Q(0) w = (w . gm) gm pointwise per item (F nodes, w and gm 2 fields per item): the transport
// part of the GN Hessian at v = 0
template <typename T>
hipError_t q_at_zero(hipStream_t s, int batch, size_t F, const T* w, const T* gm, double scale, T* out);
template <typename T>
hipError_t cast_copy(hipStream_t s, size_t n, const double* x, T* y);
template <typename T>
hipError_t cast_back(hipStream_t s, size_t n, const T* x, double* y);
// per item: z = x + (a * ad[z]) y with x, z in FP64 and y in T (the FP64 Newton iterate plus a
// step); items with mask[z] == 0 are left untouched (mask optional)
template <typename T>
hipError_t xpay_mixed(hipStream_t s, int batch, size_t n, const double* x, double a, const double* ad, const T* y,
                      double* z, const int* mask);
// per item z with mask[z] != 0 (mask optional): n elements from src + z src_stride to
// dst + z dst_stride
template <typename T>
hipError_t masked_copy(hipStream_t s, int batch, size_t n, const T* src, long long src_stride, T* dst,
                       long long dst_stride, const int* mask);

// Device-side step coefficients of the lock-step PCG (item z's reduction at red[4 z], z < batch;
// mask optional): PCG_RZ stores rz; PCG_ALPHA writes c0 = rz / pq, 0 for stopped items and for
// curvature that is not positive and finite; PCG_BETA writes (c0, c1) = (1, rz_new / rz) and stores
// rz_new for running items, (0, 1) for stopped ones
enum { PCG_RZ = 0, PCG_ALPHA = 1, PCG_BETA = 2 };
hipError_t pcg_coef(hipStream_t s, int mode, int batch, const int* mask, const double* red, double* rz, double* c0,
                    double* c1);

// Device-side scalars of Lanczos step j of 'steps' (item z's reduction at red[4 z]), so that the
// iteration needs no host round trip: LANCZOS_ALPHA stores alpha = q.w in alpha[z] (and, for live
// items, in log[(z steps + j) 2]); LANCZOS_BETA takes w.w and, for live items, logs beta =
// sqrt(w.w) at log[(z steps + j) 2 + 1] and sets beta[z] = beta, inv[z] = 1 / beta -- or, at the
// last step or a breakdown (beta <= 1e-14 |alpha|), logs -1, sets both to 0 and clears live[z];
// dead items get inv[z] = 0.
enum { LANCZOS_ALPHA = 0, LANCZOS_BETA = 1 };
hipError_t lanczos_coef(hipStream_t s, int mode, int batch, int j, int steps, const double* red, int* live,
                        double* alpha, double* beta, double* inv, double* log);

// ---- full-Newton matvec (eqs. e:hessian-matvec, e:inc-adj-slm with the lambda terms kept).
// Per item z: lam [nt+1] fields (adjoint lambda^0..lambda^nt), vt 2 fields.
// prod[z][j] = lam[z][j] vt[z] (2 fields per level j = 0..nt)
template <typename T>
hipError_t fn_products(hipStream_t s, int batch, size_t F, int nt, const T* lam, const T* vt, T* prod);
// e[z][j-1] <- ht/2 (1 + ht divv[z]) e[z][j-1] + ht/2 sigma[z][j-1], j = 1..nt (e: nt fields per
// item holding I[sigma^j](X_a) on entry; sigma: nt+1 fields per item)
template <typename T>
hipError_t fn_source(hipStream_t s, int batch, size_t F, int nt, double ht, const T* divv, const T* sigma, T* e);
// bt[z] += sum_{j=1..nt} w_j lam[z][j] gmt[z][j-1] with the trapezoid weights of t^1..t^nt (gmt:
// nt vector fields per item, the gradients of m~^1..m~^nt); items with mask[z] == 0 untouched
template <typename T>
hipError_t fn_accumulate(hipStream_t s, int batch, size_t F, int nt, double ht, const T* lam, const T* gmt, T* bt,
                         const int* mask);
// out + z so = (x + z sx) - (y + z sy) over n elements per item
template <typename T>
hipError_t sub_strided(hipStream_t s, int batch, size_t n, const T* x, long long sx, const T* y, long long sy, T* out,
                       long long so);

// ---- stabilised RK2 transport (section 3.3.1; appendix "Stabilized RK2 Scheme") --------------
// Antisymmetric-form operators, L_s y = 1/2 (v . grad y + div(y v) + s y div v): s = -1 gives the
// state operator L (d_t m = -L m), s = +1 the adjoint operator A (d_s lam = A lam backward).  Per
// item: three-field blocks (stride 3F) hold (y, y v1, y v2) and their spectral derivatives
// (d1 y, d2 y, div(y v)) from spec_rk2a.
// out[z] = (a, a w1, a w2)
template <typename T>
hipError_t rk2a_prod(hipStream_t s, int batch, size_t F, const T* a, long long sa, const T* w, long long sw, T* out);
// One Heun stage of dy/ds = sgn L_dsgn y + src.  stage 1: k = sgn L y + src into k, w3 <- the
// products of y + ht k.  stage 2: y_new = y0 + ht/2 (k + sgn L y* + src) into dst, w3 <- its products
// (w3[0] holds the stage's input y or y*; d its derivatives).
template <typename T>
struct RK2AStage {
  int stage = 1;
  size_t F = 0;
  double ht = 0;
  int sgn = -1, dsgn = -1;
  const T* d = nullptr;
  T* w3 = nullptr;
  const T* v = nullptr;
  long long sv = 0;
  const T* divv = nullptr;
  long long sdiv = 0;
  const T* src = nullptr;  // optional source (one field per item)
  long long ssrc = 0;
  const T* y0 = nullptr;   // stage 2: the step's starting value
  long long sy0 = 0;
  T* k = nullptr;          // one field per item: the first stage's slope
  T* dst = nullptr;        // stage 2 output
  long long sdst = 0;
};
template <typename T>
hipError_t rk2a_stage(hipStream_t s, int batch, const RK2AStage<T>& a);
// out = sgn 1/2 (w1 d1a + w2 d2a + div(a w) + dsgn a div w) from the derivatives d of (a, a w1, a w2)
template <typename T>
hipError_t rk2a_eval(hipStream_t s, int batch, size_t F, int sgn, int dsgn, const T* d, const T* a, long long sa,
                     const T* w, long long sw, const T* divw, long long sdw, T* out, long long so);
// out[z] = (lam, lam m)
template <typename T>
hipError_t rk2a_pair(hipStream_t s, int batch, size_t F, const T* lam, long long sl, const T* m, long long sm, T* out);
// acc (init: =, else +=) w/2 (lam grad m - m grad lam + grad(lam m)), g4[z] = (grad lam, grad(lam m))
template <typename T>
hipError_t rk2a_accum(hipStream_t s, int batch, size_t F, double w, int init, const T* lam, long long sl, const T* m,
                      long long sm, const T* gm, long long sgm, const T* g4, T* acc, long long sacc);

// p[i] = host_values[i], i < count (kernel arguments, no staging buffer): publishes
// per-linearisation integers (halos, masks) to device memory read by captured graphs
hipError_t set_ints(hipStream_t s, int* p, const int* host_values, int count);

}  // namespace slnk
