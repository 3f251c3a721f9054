// hostcheck.cpp -- host-side driver of the kernels' per-thread stage code.
//
// TEST SUPPORT ONLY (built into libppe_hostcheck.so, loaded by the CPU test
// suite, never by the library).  It runs the same __host__ __device__ stage
// functions the kernels run -- the Stockham FFT stages and the partition-method
// tridiagonal elimination -- thread by thread on the host, with the read and
// write halves of each stage separated exactly where the kernels place their
// barriers.  This checks indexing and algebra without a GPU.
#include <cstring>
#include <vector>

#include "ppe_device.hpp"
#include "ppe_plan_util.hpp"

using namespace ppe;

namespace {

template <int E, int DIR, bool PAD>
void run_fft(const HostFft& h, const std::vector<double>& tw, cplx<double>* buf) {
  FftDev f;
  f.n = h.n;
  f.e = h.e;
  f.tc = h.tc;
  f.nst = h.nst;
  for (int s = 0; s < kMaxStages; ++s) {
    f.radix[s] = h.radix[s];
    f.ns[s] = h.ns[s];
    f.tstep[s] = h.tstep[s];
    f.inv_ns[s] = h.inv_ns[s];
  }
  f.tw = tw.data();
  std::vector<cplx<double>> regs((size_t)f.tc * E);
  for (int s = 0; s < f.nst; ++s) {
    const int R = f.radix[s];
    // read half for every thread, then write half for every thread
    for (int t = 0; t < f.tc; ++t) {
      cplx<double>* v = &regs[(size_t)t * E];
      if constexpr (E % 8 == 0) if (R == 8) stage_read<E, 8, PAD, double>(buf, 1, t, RtStage{f, s}, v);
      if constexpr (E % 4 == 0) if (R == 4) stage_read<E, 4, PAD, double>(buf, 1, t, RtStage{f, s}, v);
      if constexpr (E % 3 == 0) if (R == 3) stage_read<E, 3, PAD, double>(buf, 1, t, RtStage{f, s}, v);
      if constexpr (E % 2 == 0) if (R == 2) stage_read<E, 2, PAD, double>(buf, 1, t, RtStage{f, s}, v);
    }
    for (int t = 0; t < f.tc; ++t) {
      cplx<double>* v = &regs[(size_t)t * E];
      if constexpr (E % 8 == 0) if (R == 8) stage_write<E, 8, DIR, PAD, double>(buf, 1, t, RtStage{f, s}, f.tw, v);
      if constexpr (E % 4 == 0) if (R == 4) stage_write<E, 4, DIR, PAD, double>(buf, 1, t, RtStage{f, s}, f.tw, v);
      if constexpr (E % 3 == 0) if (R == 3) stage_write<E, 3, DIR, PAD, double>(buf, 1, t, RtStage{f, s}, f.tw, v);
      if constexpr (E % 2 == 0) if (R == 2) stage_write<E, 2, DIR, PAD, double>(buf, 1, t, RtStage{f, s}, f.tw, v);
    }
  }
}

// The same transform through a compile-time plan (CtStage), stage by stage.
template <int N, int S, int DIR>
void run_fft_ct(const std::vector<double>& tw, cplx<double>* buf, std::vector<cplx<double>>& regs) {
  constexpr int E = CFft<N>::e;
  constexpr int R = CFft<N>::tab.radix[S];
  const CtStage<N, S> sp;
  for (int t = 0; t < CFft<N>::tc; ++t) stage_read<E, R, true, double>(buf, 1, t, sp, &regs[(size_t)t * E]);
  for (int t = 0; t < CFft<N>::tc; ++t)
    stage_write<E, R, DIR, true, double>(buf, 1, t, sp, tw.data(), &regs[(size_t)t * E]);
  if constexpr (S + 1 < CFft<N>::nst) run_fft_ct<N, S + 1, DIR>(tw, buf, regs);
}

// 0 if CFft<N> has the host plan's stages (radix, ns, tstep), e and tc.
template <int N>
int ct_plan_check() {
  HostFft h;
  if (!fft_factor(N, h)) return -1;
  if (h.e != CFft<N>::e || h.tc != CFft<N>::tc || h.nst != CFft<N>::nst) return -2;
  for (int s = 0; s < h.nst; ++s)
    if (h.radix[s] != CFft<N>::tab.radix[s] || h.ns[s] != CFft<N>::tab.ns[s] || h.tstep[s] != CFft<N>::tab.tstep[s])
      return -3;
  return 0;
}

template <int MC>
void run_tri(int ny, int P, double s, int zero, int outflow, const double* rhs, double* x) {
  std::vector<RedRow<double>> red(2 * (size_t)P);
  std::vector<cplx<double>> r((size_t)P * MC);
  std::vector<int> j0v(P), mv(P);
  for (int p = 0; p < P; ++p) {
    const int j0 = (int)(((long long)p * ny) / P);
    const int j1 = (int)(((long long)(p + 1) * ny) / P) - 1;
    const int m = j1 - j0 + 1;
    j0v[p] = j0;
    mv[p] = m;
    cplx<double>* rr = &r[(size_t)p * MC];
    for (int i = 0; i < MC; ++i) rr[i] = mk(0.0, 0.0);
    for (int i = 0; i < m; ++i) rr[i] = mk(rhs[2 * (j0 + i)], rhs[2 * (j0 + i) + 1]);
    const cplx<double> rf = rr[0], rl = rr[m - 1];
    ChunkEnds<double> e;
    chunk_eliminate<MC>(rr, m, s, e);
    RedRow<double> f, l;
    chunk_reduced_rows<MC>(rr, rf, rl, m, s, p == 0, p == P - 1, outflow != 0, e, f, l);
    if (zero && p == 0) {
      f.a = 0.0;
      f.b = 1.0;
      f.c = 0.0;
      f.d = mk(0.0, 0.0);
    }
    red[2 * p] = f;
    red[2 * p + 1] = l;
  }
  const int n2 = 2 * P;
  red_twisted_sweep(red.data(), n2, 0, 1);
  red_twisted_sweep(red.data(), n2, 1, 1);
  red_twisted_meet(red.data(), n2, 1);
  red_twisted_subst(red.data(), n2, 0, 1);
  red_twisted_subst(red.data(), n2, 1, 1);
  for (int p = 0; p < P; ++p) {
    const cplx<double> xf = red[2 * p].d;
    const cplx<double> xl = red[2 * p + 1].d;
    const int m = mv[p], j0 = j0v[p];
    cplx<double>* rr = &r[(size_t)p * MC];
    chunk_interior<MC>(rr, m, s, xf, xl);
    for (int i = 1; i < m - 1; ++i) {
      x[2 * (j0 + i)] = rr[i].re;
      x[2 * (j0 + i) + 1] = rr[i].im;
    }
    x[2 * j0] = xf.re;
    x[2 * j0 + 1] = xf.im;
    x[2 * (j0 + m - 1)] = xl.re;
    x[2 * (j0 + m - 1) + 1] = xl.im;
  }
  if (zero) {
    double a = 0.0;
    for (int j = 0; j < ny; ++j) a += x[2 * j];
    for (int j = 0; j < ny; ++j) {
      x[2 * j] -= a / ny;
      x[2 * j + 1] = 0.0;
    }
  }
}

}  // namespace

extern "C" {

// Radix plan of length n: returns 0 on success, fills e, tc, nst, radix[16].
int hc_fft_plan(int n, int* e, int* tc, int* nst, int* radix) {
  HostFft h;
  if (!fft_factor(n, h)) return -1;
  *e = h.e;
  *tc = h.tc;
  *nst = h.nst;
  for (int s = 0; s < kMaxStages; ++s) radix[s] = h.radix[s];
  return 0;
}

// Twiddle table exp(-2 pi i t/n), 2n doubles.
int hc_twiddles(int n, double* out) {
  std::vector<double> w = twiddles(n);
  std::memcpy(out, w.data(), w.size() * sizeof(double));
  return 0;
}

// Complex FFT of length n (interleaved re/im), dir = -1 forward, +1 inverse
// (unnormalised), through the kernels' stage code.
int hc_fft(int n, int dir, const double* in, double* out) {
  HostFft h;
  if (!fft_factor(n, h)) return -1;
  std::vector<double> tw = twiddles(n);
  // padded row layout, as the row kernels use it
  std::vector<cplx<double>> buf(padded_len(n));
  for (int i = 0; i < n; ++i) buf[lslot<true>(i, 1)] = mk(in[2 * i], in[2 * i + 1]);
#define HC_CASE(EV)                                          \
  case EV:                                                   \
    if (dir < 0) run_fft<EV, -1, true>(h, tw, buf.data());   \
    else run_fft<EV, +1, true>(h, tw, buf.data());           \
    break;
  switch (h.e) {
    HC_CASE(1)
    HC_CASE(2)
    HC_CASE(3)
    HC_CASE(4)
    HC_CASE(6)
    HC_CASE(8)
    HC_CASE(12)
    default:
      return -2;
  }
#undef HC_CASE
  for (int i = 0; i < n; ++i) {
    out[2 * i] = buf[lslot<true>(i, 1)].re;
    out[2 * i + 1] = buf[lslot<true>(i, 1)].im;
  }
  return 0;
}

// hc_fft through the compile-time plan of n (a power of two in 16..2048, or
// 96, 192, 384).
int hc_fft_ct(int n, int dir, const double* in, double* out) {
  std::vector<double> tw = twiddles(n);
  std::vector<cplx<double>> buf(padded_len(n)), regs((size_t)n);
  for (int i = 0; i < n; ++i) buf[lslot<true>(i, 1)] = mk(in[2 * i], in[2 * i + 1]);
#define HC_CT(NN)                                                   \
  case NN:                                                          \
    if (dir < 0) run_fft_ct<NN, 0, -1>(tw, buf.data(), regs);       \
    else run_fft_ct<NN, 0, +1>(tw, buf.data(), regs);               \
    break;
  switch (n) {
    HC_CT(16)
    HC_CT(32)
    HC_CT(64)
    HC_CT(128)
    HC_CT(256)
    HC_CT(512)
    HC_CT(1024)
    HC_CT(2048)
    HC_CT(96)
    HC_CT(192)
    HC_CT(384)
    default:
      return -1;
  }
#undef HC_CT
  for (int i = 0; i < n; ++i) {
    out[2 * i] = buf[lslot<true>(i, 1)].re;
    out[2 * i + 1] = buf[lslot<true>(i, 1)].im;
  }
  return 0;
}

// 0 if the compile-time plan of n equals the host factorisation.
int hc_ct_plan_check(int n) {
  switch (n) {
    case 16: return ct_plan_check<16>();
    case 32: return ct_plan_check<32>();
    case 64: return ct_plan_check<64>();
    case 128: return ct_plan_check<128>();
    case 256: return ct_plan_check<256>();
    case 512: return ct_plan_check<512>();
    case 1024: return ct_plan_check<1024>();
    case 2048: return ct_plan_check<2048>();
    case 96: return ct_plan_check<96>();
    case 192: return ct_plan_check<192>();
    case 384: return ct_plan_check<384>();
    default: return -1;
  }
}

// One solve followed by one refinement step whose residual is formed in
// difference form, (x_{j+1} - x_j) - (x_j - x_{j-1}) - s x_j: for a smooth x
// the differences are small and nearly exact, where x_{j-1} - (2+s) x_j +
// x_{j+1} cancels.  Regular systems only (flags bit 1: outflow top).
int hc_tri_refined(int ny, int P, double s, int flags, const double* rhs, double* x) {
  if (P < 1 || ny < 2 * P || (flags & 1)) return -1;
  const int outflow = (flags >> 1) & 1;
  const int mmax = (ny + P - 1) / P;
  auto pass = [&](const double* r, double* y) {
    if (mmax <= 4) run_tri<4>(ny, P, s, 0, outflow, r, y);
    else if (mmax <= 8) run_tri<8>(ny, P, s, 0, outflow, r, y);
    else if (mmax <= 16) run_tri<16>(ny, P, s, 0, outflow, r, y);
  };
  if (mmax > 16) return -1;
  pass(rhs, x);
  std::vector<double> res(2 * (size_t)ny), d(2 * (size_t)ny);
  for (int c = 0; c < 2; ++c) {
    for (int j = 0; j < ny; ++j) {
      const double xj = x[2 * j + c];
      const double up = j + 1 < ny ? x[2 * (j + 1) + c] - xj : 0.0;
      const double dn = j > 0 ? xj - x[2 * (j - 1) + c] : 0.0;
      double ax = up - dn - s * xj;
      if (j == ny - 1 && outflow) ax -= 2.0 * xj;
      res[2 * j + c] = rhs[2 * j + c] - ax;
    }
  }
  pass(res.data(), d.data());
  for (int q = 0; q < 2 * ny; ++q) x[q] += d[q];
  return 0;
}

// One y system: x_{j-1} + beta_j x_j + x_{j+1} = rhs_j (scaled form, complex
// interleaved), P chunks.  flags bit 0: apply the pin and the mean removal of
// the singular (0,0) system; bit 1: outflow top row (beta_{ny-1} = -3 - s).
int hc_tri(int ny, int P, double s, int flags, const double* rhs, double* x) {
  if (P < 1 || ny < 2 * P) return -1;
  const int zero = flags & 1, outflow = (flags >> 1) & 1;
  if (zero && outflow) return -1;  // the outflow system is never singular
  const int mmax = (ny + P - 1) / P;
  if (mmax <= 4) run_tri<4>(ny, P, s, zero, outflow, rhs, x);
  else if (mmax <= 8) run_tri<8>(ny, P, s, zero, outflow, rhs, x);
  else if (mmax <= 16) run_tri<16>(ny, P, s, zero, outflow, rhs, x);
  else return -1;
  return 0;
}

// The z transform's paired block order for a gx x gy grid: j[L], by[L] for
// every linear block index L.
void hc_fftz_pair_map(int gx, int gy, int* j, int* by) {
  for (int L = 0; L < gx * gy; ++L) fftz_pair_block((unsigned)L, (unsigned)gx, (unsigned)gy, j[L], by[L]);
}

}  // extern "C"
