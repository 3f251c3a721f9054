// ppe_plan_util.hpp -- host-side FFT factorisation and twiddle tables.
#pragma once

#include <cmath>
#include <vector>

#include "ppe_device.hpp"

namespace ppe {
namespace {

constexpr int kMaxN = 2048;  // longest FFT / y extent supported

// ---------------------------------------------------------------------------
// FFT plans
// ---------------------------------------------------------------------------
struct HostFft {
  int n = 0, e = 1, tc = 1, nst = 0;
  int radix[kMaxStages] = {0};
  int ns[kMaxStages] = {0};
  int tstep[kMaxStages] = {0};
  float inv_ns[kMaxStages] = {0};
  double* tw = nullptr;  // device, 2n doubles
};

inline int gcd_i(int a, int b) { return b ? gcd_i(b, a % b) : a; }

// Radices for n = 2^a 3^b: all 3s first, then 8s (pure powers of two) or 4s,
// then a final 2 or 4.  E = lcm of the radices.  Returns false if n has
// another prime factor.
inline bool fft_factor(int n, HostFft& f) {
  if (n < 1 || n > kMaxN) return false;
  int m = n, a = 0, b = 0;
  while (m % 2 == 0) { m /= 2; ++a; }
  while (m % 3 == 0) { m /= 3; ++b; }
  if (m != 1) return false;
  // (a fixed array: planning allocates no memory)
  int r[kMaxStages + 16];
  int nr = 0;
  for (int q = 0; q < b; ++q) r[nr++] = 3;
  if (b == 0) {
    while (a >= 3) { r[nr++] = 8; a -= 3; }
    if (a == 2) r[nr++] = 4;
    else if (a == 1) r[nr++] = 2;
  } else {
    while (a >= 2) { r[nr++] = 4; a -= 2; }
    if (a == 1) r[nr++] = 2;
  }
  if (nr > kMaxStages) return false;
  int e = 1;
  for (int q = 0; q < nr; ++q) e = e / gcd_i(e, r[q]) * r[q];
  f.n = n;
  f.e = e;
  f.tc = n / e;
  f.nst = nr;
  int ns = 1;
  for (int s = 0; s < f.nst; ++s) {
    f.radix[s] = r[s];
    f.ns[s] = ns;
    f.tstep[s] = n / (ns * r[s]);
    f.inv_ns[s] = 1.0f / (float)ns;
    ns *= r[s];
  }
  return true;
}

// exp(-2 pi i t / n) for t = 0..n-1, computed in extended precision.
inline std::vector<double> twiddles(int n) {
  std::vector<double> w(2 * (size_t)n);
  const long double two_pi = 6.283185307179586476925286766559005768L;
  for (int t = 0; t < n; ++t) {
    // 64-bit-mantissa evaluation, rounded once to double
    const long double a = two_pi * (long double)t / (long double)n;
    w[2 * t] = (double)cosl(a);
    w[2 * t + 1] = (double)(-sinl(a));
  }
  // exact values where the circle hits the axes
  for (int t = 0; t < n; ++t) {
    long long q4 = 4LL * t;
    if (q4 % n == 0) {
      const long long qq = (q4 / n) % 4;
      const double c[4] = {1, 0, -1, 0}, s[4] = {0, -1, 0, 1};
      w[2 * t] = c[qq];
      w[2 * t + 1] = s[qq];
    }
  }
  return w;
}

}  // namespace
}  // namespace ppe
