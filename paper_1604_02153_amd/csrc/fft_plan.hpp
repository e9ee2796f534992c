// Host-side planning of the spectral passes' transforms: supported lengths, the radix list of a
// length and its twiddle table (computed in FP64, stored in the pass precision).  Shared by the
// context set-up (api.cpp) and the allocation-free entry point (noalloc.hip).
#pragma once

#include <cmath>

#include "kernels.hpp"

namespace slnk {

// even products of 2, 3, 5 in [8, 2048]
inline bool fft_size_ok(int n) {
  if (n < 8 || n > 2048 || (n & 1)) return false;
  for (int r : {2, 3, 5})
    while (n % r == 0) n /= r;
  return n == 1;
}

// radix list of a supported length (8s, then 4s, 2s, 3s, 5s); returns the number of stages, or -1
// when it would exceed kFFTMaxStages
inline int fft_factorise(int n, int* radix) {
  int k = 0;
  for (int r : {8, 4, 2, 3, 5})
    while (n % r == 0) {
      if (k == kFFTMaxStages) return -1;
      radix[k++] = r;
      n /= r;
    }
  return k;
}

// Fill the plan of length n (radix list, stage offsets; pl.tw and pl.roots are left to the caller)
// and hand its 2n-entry table to emit(i, re, im): entries [0, n - 1) are the stage twiddles (stage
// s, radix R, p = product of the earlier radices: exp(-2 pi i j k / (p R)) at twoff[s] + (j - 1) p
// + k, j = 1..R-1, k < p), entry n - 1 is 1, entries [n, 2n) the roots exp(-2 pi i m / n).
// Returns false when n has too many factors.
template <class Emit>
bool fft_plan_host(int n, FFTPlanDev& pl, Emit&& emit) {
  constexpr double kTwoPi = 6.28318530717958647692;
  int r[kFFTMaxStages];
  const int ns = fft_factorise(n, r);
  if (ns < 0) return false;
  pl.n = n;
  pl.nstages = ns;
  int p = 1, off = 0;
  for (int st = 0; st < ns; ++st) {
    pl.radix[st] = r[st];
    pl.twoff[st] = off;
    for (int j = 1; j < r[st]; ++j)
      for (int k = 0; k < p; ++k) {
        const double a = kTwoPi * double(j) * double(k) / double(p * r[st]);
        emit(off + (j - 1) * p + k, std::cos(a), -std::sin(a));
      }
    off += (r[st] - 1) * p;
    p *= r[st];
  }
  pl.ntw = off;
  for (int i = off; i < n; ++i) emit(i, 1.0, 0.0);
  for (int m = 0; m < n; ++m) {
    const double a = kTwoPi * double(m) / double(n);
    emit(n + m, std::cos(a), -std::sin(a));
  }
  return true;
}

}  // namespace slnk
