// ppe_device.hpp -- device building blocks of the projection library (gfx950).
//
// * complex arithmetic on (re, im) pairs,
// * a mixed-radix (2, 3, 4, 8) Stockham FFT whose data live in LDS, one
//   transform per group of `tc` threads, each thread holding E elements in
//   registers during a stage (E = lcm of the radices used),
// * the per-chunk elimination of the y-tridiagonal solve (partition method:
//   every chunk is reduced to its two end unknowns, the reduced system is
//   solved by a two-ended Thomas sweep per system).
//
// Stage bodies are __host__ __device__ and take the thread index explicitly,
// so the same code can be driven thread by thread on the host for checks;
// the kernels call them with barriers between the read and write halves.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace ppe {

#define PPE_HD __host__ __device__ __forceinline__

template <typename T>
struct cplx {
  T re, im;
};

// One complex value stored with the non-temporal hint, as a single 2-vector
// store (the address must be aligned to the whole value, as every spectrum
// element is).
template <typename T>
__device__ __forceinline__ void store_nt(cplx<T>* p, const cplx<T>& y) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  v2 v;
  v.x = y.re;
  v.y = y.im;
  __builtin_nontemporal_store(v, reinterpret_cast<v2*>(p));
}

template <typename T>
PPE_HD cplx<T> mk(T r, T i) {
  cplx<T> c;
  c.re = r;
  c.im = i;
  return c;
}
template <typename T>
PPE_HD cplx<T> cadd(cplx<T> a, cplx<T> b) { return mk(a.re + b.re, a.im + b.im); }
template <typename T>
PPE_HD cplx<T> csub(cplx<T> a, cplx<T> b) { return mk(a.re - b.re, a.im - b.im); }
template <typename T>
PPE_HD cplx<T> cscale(cplx<T> a, T s) { return mk(a.re * s, a.im * s); }
template <typename T>
PPE_HD cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename T>
PPE_HD cplx<T> cconj(cplx<T> a) { return mk(a.re, -a.im); }
// multiply by -i (DIR = -1) or +i (DIR = +1)
template <int DIR, typename T>
PPE_HD cplx<T> mul_i(cplx<T> a) {
  return DIR < 0 ? mk(a.im, -a.re) : mk(-a.im, a.re);
}

// 1/x for finite non-zero x: the hardware reciprocal estimate refined by two
// Newton steps (each doubles the correct bits), accurate to about one unit in
// the last place and much shorter than a correctly rounded division, which
// matters inside the sequential sweeps.  The host build divides.
PPE_HD double rcp_nr(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  double y = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, y, 1.0);
  y = __builtin_fma(y, e, y);
  e = __builtin_fma(-x, y, 1.0);
  return __builtin_fma(y, e, y);
#else
  return 1.0 / x;
#endif
}
PPE_HD float rcp_nr(float x) { return 1.0f / x; }

// ---------------------------------------------------------------------------
// FFT plan as seen by a kernel (passed by value)
// ---------------------------------------------------------------------------
constexpr int kMaxStages = 16;

struct FftDev {
  int n;                   // transform length
  int e;                   // elements per thread (lcm of the radices)
  int tc;                  // threads per transform = n / e
  int nst;                 // number of stages
  int radix[kMaxStages];   // radix of each stage
  int ns[kMaxStages];      // length of the sub-transforms done before the stage
  int tstep[kMaxStages];   // twiddle index step n / (ns * radix)
  float inv_ns[kMaxStages];  // 1 / ns (quotient estimate, corrected exactly)
  const double* tw;        // 2*n doubles: W_n^t = exp(-2 pi i t / n), t = 0..n-1
                           // (global table; kernels stage a copy in LDS)
};

// Compile-time plan of a power-of-two length N (2 <= N <= 2048), factored as
// the host factors powers of two: radix-8 stages, then one radix-4 or radix-2
// stage for the remaining factor.  Stage counts, radices, sub-transform
// lengths and twiddle steps are constants, so the stage loop unrolls, the
// radix dispatch folds away and j / ns, j mod ns become shifts.  Only the
// twiddle table is a run-time value.
struct StageTab {
  int radix[kMaxStages];
  int ns[kMaxStages];
  int tstep[kMaxStages];
};

constexpr int ilog2_c(int x) { return x <= 1 ? 0 : 1 + ilog2_c(x / 2); }

constexpr StageTab pow2_stages(int n) {
  StageTab t{};
  const int lg = ilog2_c(n);
  int ns = 1, s = 0;
  for (int k = 0; k < lg / 3; ++k, ++s) {
    t.radix[s] = 8;
    t.ns[s] = ns;
    t.tstep[s] = n / (ns * 8);
    ns *= 8;
  }
  if (lg % 3) {
    const int r = 1 << (lg % 3);
    t.radix[s] = r;
    t.ns[s] = ns;
    t.tstep[s] = n / (ns * r);
  }
  return t;
}

// n = 3 * 2^a (a >= 2): the host's order, a radix-3 stage, then radix-4
// stages and a last radix 2 for odd a; 12 elements per thread.
constexpr StageTab three_pow2_stages(int n) {
  StageTab t{};
  int a = ilog2_c(n / 3), ns = 1, s = 0;
  const auto put = [&](int r) {
    t.radix[s] = r;
    t.ns[s] = ns;
    t.tstep[s] = n / (ns * r);
    ns *= r;
    ++s;
  };
  put(3);
  for (; a >= 2; a -= 2) put(4);
  if (a == 1) put(2);
  return t;
}

constexpr bool is_pow2_c(int n) { return n >= 1 && (n & (n - 1)) == 0; }

template <int N>
struct CFft {
  static_assert(N >= 2 && (is_pow2_c(N) || (N % 3 == 0 && N >= 12 && is_pow2_c(N / 3))),
                "a power of two, or three times a power of two of at least 4");
  static constexpr bool pow2 = is_pow2_c(N);
  static constexpr int n = N;
  static constexpr int nst = pow2 ? ilog2_c(N) / 3 + (ilog2_c(N) % 3 ? 1 : 0) : 1 + (ilog2_c(N / 3) + 1) / 2;
  static constexpr int e = pow2 ? (ilog2_c(N) >= 3 ? 8 : N) : 12;  // lcm of the radices
  static constexpr int tc = N / e;
  static constexpr StageTab tab = pow2 ? pow2_stages(N) : three_pow2_stages(N);
  const double* tw;  // as in FftDev
};

// What one Stockham stage needs of its plan: the transform length, threads
// per transform, the sub-transform length ns before the stage, the twiddle
// step, and j / ns, j mod ns.  RtStage reads a run-time plan; CtStage<N, S>
// is stage S of CFft<N>, all constants.
struct RtStage {
  const FftDev& f;
  int st;
  PPE_HD int n() const { return f.n; }
  PPE_HD int tc() const { return f.tc; }
  PPE_HD int ns() const { return f.ns[st]; }
  PPE_HD int tstep() const { return f.tstep[st]; }
  // j / ns and j mod ns for 0 <= j < 2^24 from a float quotient estimate,
  // corrected to the exact integers
  PPE_HD void divmod(int j, int& q, int& r) const {
    const int d = f.ns[st];
    q = (int)((float)j * f.inv_ns[st]);
    r = j - q * d;
    if (r < 0) {
      q -= 1;
      r += d;
    } else if (r >= d) {
      q += 1;
      r -= d;
    }
  }
};

template <int N, int S>
struct CtStage {
  static constexpr int kNs = CFft<N>::tab.ns[S];
  PPE_HD static constexpr int n() { return N; }
  PPE_HD static constexpr int tc() { return CFft<N>::tc; }
  PPE_HD static constexpr int ns() { return kNs; }
  PPE_HD static constexpr int tstep() { return CFft<N>::tab.tstep[S]; }
  PPE_HD static void divmod(int j, int& q, int& r) {
    q = (int)((unsigned)j / (unsigned)kNs);
    r = (int)((unsigned)j % (unsigned)kNs);
  }
};

// Small DFTs on registers.  DIR = -1 forward (exp(-i...)), +1 inverse.
template <int DIR, typename T>
PPE_HD void dft2(cplx<T>* v) {
  cplx<T> a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <int DIR, typename T>
PPE_HD void dft3(cplx<T>* v) {
  const T h = T(0.86602540378443864676372317075294);  // sqrt(3)/2
  cplx<T> a = v[0], b = v[1], c = v[2];
  cplx<T> s = cadd(b, c);
  cplx<T> d = csub(b, c);
  cplx<T> m = mk(a.re - T(0.5) * s.re, a.im - T(0.5) * s.im);
  // X1 = m + DIR * i * h * d ; X2 = m - DIR * i * h * d
  cplx<T> r = cscale(mul_i<DIR>(d), h);
  v[0] = cadd(a, s);
  v[1] = cadd(m, r);
  v[2] = csub(m, r);
}

template <int DIR, typename T>
PPE_HD void dft4(cplx<T>* v) {
  cplx<T> a = v[0], b = v[1], c = v[2], d = v[3];
  cplx<T> s0 = cadd(a, c), d0 = csub(a, c);
  cplx<T> s1 = cadd(b, d), d1 = mul_i<DIR>(csub(b, d));
  v[0] = cadd(s0, s1);
  v[2] = csub(s0, s1);
  v[1] = cadd(d0, d1);
  v[3] = csub(d0, d1);
}

template <int DIR, typename T>
PPE_HD void dft8(cplx<T>* v) {
  const T r2 = T(0.70710678118654752440084436210485);  // 1/sqrt(2)
  cplx<T> a[4], b[4];
  for (int k = 0; k < 4; ++k) {
    a[k] = cadd(v[k], v[k + 4]);
    b[k] = csub(v[k], v[k + 4]);
  }
  // b_k *= W8^{k} (forward) or W8^{-k} (inverse)
  // W8 = (1 - i)/sqrt2 forward; (1 + i)/sqrt2 inverse
  {
    cplx<T> t = b[1];
    cplx<T> ti = mul_i<DIR>(t);  // DIR*i*t
    b[1] = mk((t.re + ti.re) * r2, (t.im + ti.im) * r2);
    b[2] = mul_i<DIR>(b[2]);
    t = b[3];
    ti = mul_i<DIR>(t);
    // W8^3 = (-1 - i)/sqrt2 forward => (-t + DIR*i*t)/sqrt2
    b[3] = mk((ti.re - t.re) * r2, (ti.im - t.im) * r2);
  }
  dft4<DIR>(a);
  dft4<DIR>(b);
  v[0] = a[0];
  v[2] = a[1];
  v[4] = a[2];
  v[6] = a[3];
  v[1] = b[0];
  v[3] = b[1];
  v[5] = b[2];
  v[7] = b[3];
}

template <int R, int DIR, typename T>
PPE_HD void dft(cplx<T>* v) {
  if constexpr (R == 2) dft2<DIR>(v);
  else if constexpr (R == 3) dft3<DIR>(v);
  else if constexpr (R == 4) dft4<DIR>(v);
  else if constexpr (R == 8) dft8<DIR>(v);
}

// LDS slot of element n of a transform.  Rows (es == 1) are padded with one
// slot per 2^kRowPadShift elements: the first Stockham stages write with a
// stride of R elements, which without padding puts every lane of a wavefront
// on the same LDS banks.  Columns (es > 1, several transforms side by side)
// sit at stride es; the z kernel adds kColPad slots to its column count.
#ifndef PPE_ROW_PAD_SHIFT
#define PPE_ROW_PAD_SHIFT 3
#endif
#ifndef PPE_COL_PAD
#define PPE_COL_PAD 0
#endif
constexpr int kRowPadShift = PPE_ROW_PAD_SHIFT;
constexpr int kColPad = PPE_COL_PAD;
template <bool PAD>
PPE_HD int lslot(int n, int es) {
  return PAD ? n + (n >> kRowPadShift) : n * es;
}
// Slots a padded row of n elements occupies.
PPE_HD int padded_len(int n) { return n + (n >> kRowPadShift) + 1; }

// Block order of the z transform when a 128-byte tile row spans two blocks
// (FP32 spectra): blocks go to the XCDs round-robin by linear index L, and
// the two halves (by = 2t, 2t + 1) of tile row (j, t) are given L and L + 8,
// one XCD, dispatched together.  gx = ny (a multiple of 8) blocks per column,
// gy columns; with gy odd the last column keeps the plain order.
PPE_HD void fftz_pair_block(unsigned L, unsigned gx, unsigned gy, int& j, int& by) {
  const unsigned npair = gy & ~1u, head = gx * npair;
  if (L < head) {
    const unsigned q = L >> 3, unit = ((q >> 1) << 3) + (L & 7);
    j = (int)(unit % gx);
    by = 2 * (int)(unit / gx) + (int)(q & 1);
  } else {
    j = (int)(L - head);
    by = (int)npair;
  }
}

// One Stockham stage, split into its read and write halves.
//   element n of the transform lives at buf[lslot(n, es)]
//   butterfly j in [0, n/R): inputs j + r n/R, twiddle exp(DIR 2 pi i r (j mod Ns)/(Ns R)),
//   outputs (j / Ns) Ns R + (j mod Ns) + r Ns.
// Thread t owns butterflies j = t + tc q, q in [0, E/R).  `sp` describes the
// stage (RtStage or CtStage).
template <int E, int R, bool PAD, typename T, typename BufT, typename SP>
PPE_HD void stage_read(const BufT* buf, int es, int t, const SP& sp, cplx<T>* v) {
  constexpr int NB = E / R;
  const int nr = sp.n() / R;
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int j = t + sp.tc() * q;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const BufT x = buf[lslot<PAD>(j + r * nr, es)];
      v[q * R + r] = mk(T(x.re), T(x.im));
    }
  }
}

template <int DIR, typename T>
PPE_HD cplx<T> tw_load(const double* tw, int ti) {
  return mk(T(tw[2 * ti]), DIR > 0 ? T(-tw[2 * ti + 1]) : T(tw[2 * ti + 1]));
}

// Stage twiddles w^r, r = 1..R-1, of w = W_n^{jm tstep}: w, w^2 (and w^4 for
// radix 8) come from the table, the others are products of those (at most
// two roundings more than a table value).
template <int R, int DIR, typename T>
PPE_HD void stage_twiddles_of(const double* tw, int base, cplx<T>* w) {
  w[1] = tw_load<DIR, T>(tw, base);
  if constexpr (R >= 3) w[2] = tw_load<DIR, T>(tw, 2 * base);
  if constexpr (R == 4) w[3] = cmul(w[1], w[2]);
  if constexpr (R == 8) {
    w[3] = cmul(w[1], w[2]);
    w[4] = tw_load<DIR, T>(tw, 4 * base);
    w[5] = cmul(w[1], w[4]);
    w[6] = cmul(w[2], w[4]);
    w[7] = cmul(w[3], w[4]);
  }
}

// Twiddles and butterflies of the thread's group q; returns the index of
// output r = 0 (the others follow at stride ns).
template <int R, int DIR, typename T, typename SP>
PPE_HD int stage_butterfly(int j, const SP& sp, const double* tw, cplx<T>* v) {
  int jd, jm;
  sp.divmod(j, jd, jm);
  if (sp.ns() > 1) {
    // twiddles W_n^{r (j mod ns) n/(ns R)}
    cplx<T> w[R];
    stage_twiddles_of<R, DIR, T>(tw, jm * sp.tstep(), w);
#pragma unroll
    for (int r = 1; r < R; ++r) v[r] = cmul(v[r], w[r]);
  }
  dft<R, DIR>(v);
  return jd * sp.ns() * R + jm;
}

template <int E, int R, int DIR, bool PAD, typename T, typename BufT, typename SP>
PPE_HD void stage_write(BufT* buf, int es, int t, const SP& sp, const double* tw, cplx<T>* v) {
  constexpr int NB = E / R;
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int base = stage_butterfly<R, DIR, T>(t + sp.tc() * q, sp, tw, &v[q * R]);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      BufT o;
      o.re = v[q * R + r].re;
      o.im = v[q * R + r].im;
      buf[lslot<PAD>(base + r * sp.ns(), es)] = o;
    }
  }
}

// Twiddles and butterflies of all the thread's groups, in place: after the
// last stage v[q R + r] is output j + r n/R of the transform, j = t + tc q.
template <int E, int R, int DIR, typename T, typename SP>
PPE_HD void stage_bfly_all(int t, const SP& sp, const double* tw, cplx<T>* v) {
  constexpr int NB = E / R;
#pragma unroll
  for (int q = 0; q < NB; ++q) stage_butterfly<R, DIR, T>(t + sp.tc() * q, sp, tw, &v[q * R]);
}

// The read half of stage 0 from a loader instead of LDS: v[q R + r] =
// load(j + r n/R) for the thread's butterflies j = t + tc q.
template <int E, int R, typename T, typename LoadF, typename SP>
PPE_HD void stage_load(int t, const SP& sp, LoadF load, cplx<T>* v) {
  constexpr int NB = E / R;
  const int nr = sp.n() / R;
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int j = t + sp.tc() * q;
#pragma unroll
    for (int r = 0; r < R; ++r) v[q * R + r] = load(j + r * nr);
  }
}

// The write half of a stage to a storer instead of LDS: store(n, x) for the
// stage's outputs n (same twiddles and butterflies as stage_write).
template <int E, int R, int DIR, typename T, typename StoreF, typename SP>
PPE_HD void stage_store(int t, const SP& sp, const double* tw, cplx<T>* v, StoreF store) {
  constexpr int NB = E / R;
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int base = stage_butterfly<R, DIR, T>(t + sp.tc() * q, sp, tw, &v[q * R]);
#pragma unroll
    for (int r = 0; r < R; ++r) store(base + r * sp.ns(), v[q * R + r]);
  }
}

#if defined(__HIP_DEVICE_COMPILE__) || defined(__HIPCC__)
// Copy the twiddle table of `f` into LDS (all threads of the block; the
// caller's next barrier publishes it).
template <typename F>
__device__ __forceinline__ void stage_twiddles(double* lds_tw, const F& f) {
  for (int q = threadIdx.x; q < 2 * f.n; q += blockDim.x) lds_tw[q] = f.tw[q];
}

// Whole transform in LDS.  Every thread of the block must call this (it
// contains barriers); threads with active == false only join the barriers.
// `tw` is the twiddle table, normally the copy a kernel staged in LDS.
template <int E, int DIR, bool PAD, typename T, typename BufT>
__device__ __forceinline__ void fft_lds(BufT* buf, int es, int t, bool active, const FftDev& f, const double* tw) {
  for (int s = 0; s < f.nst; ++s) {
    const int R = f.radix[s];
    cplx<T> v[E];
    if (R == 8) {
      if constexpr (E % 8 == 0) {
        if (active) stage_read<E, 8, PAD, T>(buf, es, t, RtStage{f, s}, v);
        __syncthreads();
        if (active) stage_write<E, 8, DIR, PAD, T>(buf, es, t, RtStage{f, s}, tw, v);
      }
    } else if (R == 4) {
      if constexpr (E % 4 == 0) {
        if (active) stage_read<E, 4, PAD, T>(buf, es, t, RtStage{f, s}, v);
        __syncthreads();
        if (active) stage_write<E, 4, DIR, PAD, T>(buf, es, t, RtStage{f, s}, tw, v);
      }
    } else if (R == 3) {
      if constexpr (E % 3 == 0) {
        if (active) stage_read<E, 3, PAD, T>(buf, es, t, RtStage{f, s}, v);
        __syncthreads();
        if (active) stage_write<E, 3, DIR, PAD, T>(buf, es, t, RtStage{f, s}, tw, v);
      }
    } else {
      if constexpr (E % 2 == 0) {
        if (active) stage_read<E, 2, PAD, T>(buf, es, t, RtStage{f, s}, v);
        __syncthreads();
        if (active) stage_write<E, 2, DIR, PAD, T>(buf, es, t, RtStage{f, s}, tw, v);
      }
    }
    __syncthreads();
  }
}

// Whole transform whose first stage reads its inputs through load(n) (global
// memory) instead of LDS and, with GSTORE, whose last stage hands its outputs
// to store(n, x) instead of writing LDS.  Compared with staging the data in
// LDS first and copying it out after fft_lds, this saves two LDS passes and
// two barriers.  Every thread of the block must call it; threads with
// active == false only join the barriers.  Without GSTORE the result is in
// buf (padded or strided as for fft_lds) after the final barrier.  With
// GSTORE, buf is dead on return and a caller reusing LDS needs a barrier.
template <int E, int DIR, bool PAD, bool GSTORE, typename T, typename BufT, typename LoadF, typename StoreF>
__device__ __forceinline__ void fft_io(BufT* buf, int es, int t, bool active, const FftDev& f, const double* tw,
                                       LoadF load, StoreF store) {
  cplx<T> v[E];
  const int last = f.nst - 1;
  if (last < 0) {  // length 1: the transform is the identity
    if (active) {
#pragma unroll
      for (int q = 0; q < E; ++q) {
        const int n = t + f.tc * q;
        const cplx<T> x = load(n);
        if constexpr (GSTORE) store(n, x);
        else buf[lslot<PAD>(n, es)] = x;
      }
    }
    if constexpr (!GSTORE) __syncthreads();
    return;
  }
#define PPE_FFT_IO_DISPATCH(...)                          \
  {                                                      \
    const int R_ = f.radix[s];                           \
    if (R_ == 8) {                                       \
      if constexpr (E % 8 == 0) {                        \
        constexpr int R = 8;                             \
        __VA_ARGS__                                      \
      }                                                  \
    } else if (R_ == 4) {                                \
      if constexpr (E % 4 == 0) {                        \
        constexpr int R = 4;                             \
        __VA_ARGS__                                      \
      }                                                  \
    } else if (R_ == 3) {                                \
      if constexpr (E % 3 == 0) {                        \
        constexpr int R = 3;                             \
        __VA_ARGS__                                      \
      }                                                  \
    } else {                                             \
      if constexpr (E % 2 == 0) {                        \
        constexpr int R = 2;                             \
        __VA_ARGS__                                      \
      }                                                  \
    }                                                    \
  }
  {
    const int s = 0;
    PPE_FFT_IO_DISPATCH({
      if (active) stage_load<E, R, T>(t, RtStage{f, 0}, load, v);
      if (GSTORE && last == 0) {
        if (active) stage_store<E, R, DIR, T>(t, RtStage{f, 0}, tw, v, store);
      } else {
        if (active) stage_write<E, R, DIR, PAD, T>(buf, es, t, RtStage{f, 0}, tw, v);
      }
    })
  }
  if (GSTORE && last == 0) return;
  __syncthreads();
  for (int s = 1; s <= last; ++s) {
    PPE_FFT_IO_DISPATCH({
      if (active) stage_read<E, R, PAD, T>(buf, es, t, RtStage{f, s}, v);
      if (GSTORE && s == last) {
        if (active) stage_store<E, R, DIR, T>(t, RtStage{f, s}, tw, v, store);
      } else {
        __syncthreads();
        if (active) stage_write<E, R, DIR, PAD, T>(buf, es, t, RtStage{f, s}, tw, v);
        __syncthreads();
      }
    })
  }
#undef PPE_FFT_IO_DISPATCH
}

// fft_io for a compile-time plan: the same stages and barriers, unrolled.
// PRE: load(v) fills the thread's stage-0 inputs v[q R + r] = x(j + r n/R),
// j = t + tc q, all at once (instead of one call per element).
// POST (with GSTORE): the last stage's butterflies run in registers and
// store(v) receives all of the thread's outputs at once (see stage_bfly_all).
template <int E, int DIR, bool PAD, bool GSTORE, bool PRE, typename T, int N, int S, typename BufT, typename LoadF,
          typename StoreF, bool POST = false>
__device__ __forceinline__ void fft_io_ct_stage(BufT* buf, int es, int t, bool active, const double* tw,
                                                LoadF& load, StoreF& store, cplx<T>* v) {
  constexpr int R = CFft<N>::tab.radix[S];
  constexpr int last = CFft<N>::nst - 1;
  static_assert(E % R == 0, "E must be a multiple of every radix");
  static_assert(!POST || GSTORE, "POST hands the outputs to the storer");
  const CtStage<N, S> sp;
  if constexpr (S == 0) {
    if constexpr (PRE) {
      if (active) load(v);
    } else {
      if (active) stage_load<E, R, T>(t, sp, load, v);
    }
  } else {
    if (active) stage_read<E, R, PAD, T>(buf, es, t, sp, v);
  }
  if constexpr (GSTORE && S == last) {
    if constexpr (POST) {
      if (active) {
        stage_bfly_all<E, R, DIR, T>(t, sp, tw, v);
        store(v);
      }
    } else {
      if (active) stage_store<E, R, DIR, T>(t, sp, tw, v, store);
    }
  } else {
    if constexpr (S > 0) __syncthreads();
    if (active) stage_write<E, R, DIR, PAD, T>(buf, es, t, sp, tw, v);
    __syncthreads();
  }
  if constexpr (S < last)
    fft_io_ct_stage<E, DIR, PAD, GSTORE, PRE, T, N, S + 1, BufT, LoadF, StoreF, POST>(buf, es, t, active, tw, load,
                                                                                      store, v);
}

template <int E, int DIR, bool PAD, bool GSTORE, typename T, int N, typename BufT, typename LoadF, typename StoreF>
__device__ __forceinline__ void fft_io(BufT* buf, int es, int t, bool active, const CFft<N>&, const double* tw,
                                       LoadF load, StoreF store) {
  static_assert(E == CFft<N>::e, "elements per thread of the plan");
  cplx<T> v[E];
  fft_io_ct_stage<E, DIR, PAD, GSTORE, false, T, N, 0>(buf, es, t, active, tw, load, store, v);
}

// fft_io with a whole-thread stage-0 loader (see fft_io_ct_stage's PRE).
template <int E, int DIR, bool PAD, bool GSTORE, typename T, int N, typename BufT, typename LoadV, typename StoreF>
__device__ __forceinline__ void fft_io_v(BufT* buf, int es, int t, bool active, const CFft<N>&, const double* tw,
                                         LoadV loadv, StoreF store) {
  static_assert(E == CFft<N>::e, "elements per thread of the plan");
  cplx<T> v[E];
  fft_io_ct_stage<E, DIR, PAD, GSTORE, true, T, N, 0>(buf, es, t, active, tw, loadv, store, v);
}

// fft_io whose last stage hands all of the thread's outputs to store(v):
// v[q R + r] is output t + tc q + r n/R, R the last radix.
template <int E, int DIR, bool PAD, typename T, int N, typename BufT, typename LoadF, typename StoreV>
__device__ __forceinline__ void fft_io_post(BufT* buf, int es, int t, bool active, const CFft<N>&, const double* tw,
                                            LoadF load, StoreV storev) {
  static_assert(E == CFft<N>::e, "elements per thread of the plan");
  cplx<T> v[E];
  fft_io_ct_stage<E, DIR, PAD, true, false, T, N, 0, BufT, LoadF, StoreV, true>(buf, es, t, active, tw, load, storev,
                                                                               v);
}

// fft_io_v whose last stage hands all of the thread's outputs to store(v),
// laid out as for fft_io_post.
template <int E, int DIR, bool PAD, typename T, int N, typename BufT, typename LoadV, typename StoreV>
__device__ __forceinline__ void fft_io_v_post(BufT* buf, int es, int t, bool active, const CFft<N>&,
                                              const double* tw, LoadV loadv, StoreV storev) {
  static_assert(E == CFft<N>::e, "elements per thread of the plan");
  cplx<T> v[E];
  fft_io_ct_stage<E, DIR, PAD, true, true, T, N, 0, BufT, LoadV, StoreV, true>(buf, es, t, active, tw, loadv,
                                                                              storev, v);
}

template <typename F>
struct is_ct_fft : std::false_type {};
template <int N>
struct is_ct_fft<CFft<N>> : std::true_type {};
#endif

// ---------------------------------------------------------------------------
// y-tridiagonal solve, partition method.
//
// Scaled system for one wavenumber pair (multiplied by dy^2):
//   x_{j-1} + beta_j x_j + x_{j+1} = r_j,  beta_j = -2 - s (interior),
//   beta_0 = -1 - s (zero-flux bottom face), beta_{ny-1} = -1 - s (zero-flux
//   top face) or -3 - s (outflow top face, p = 0 there: ghost x_ny = -x_{ny-1}),
//   s = -(lam_x + lam_z) dy^2 >= 0.
// A chunk [j0, j1] (m = j1 - j0 + 1 rows) eliminates its interior rows as a
// Dirichlet problem with end values x_{j0}, x_{j1}:
//   x_i = y_i + phi_i x_{j0} + psi_i x_{j1},  i = 1..m-2 (local index)
// The pivots are carried as g (den_i = -(1 + g_i)), g_1 = 1 + s,
// g_i = s + g_{i-1}/(1 + g_{i-1}), which has no cancellation for small s.
// The two end rows then form a tridiagonal reduced system in the ends of all
// chunks.
// ---------------------------------------------------------------------------
constexpr int kMaxChunk = 16;   // longest chunk the kernels instantiate

// Pivots of the interior rows (ni = m - 2 of them): q_i = 1/(1+g_i) and the
// forward product fphi_i = q_0 ... q_i.  They depend on s and ni only.
template <int MC, typename T>
PPE_HD void chunk_pivots(int ni, T s, T* q, T* fphi) {
  T g = T(1) + s;
#pragma unroll
  for (int i = 0; i < MC - 2; ++i) {
    if (i < ni) {
      if (i > 0) g = s + g * q[i - 1];
      q[i] = rcp_nr(T(1) + g);
      fphi[i] = i == 0 ? q[0] : fphi[i - 1] * q[i];
    }
  }
}

// The homogeneous solutions at the chunk's two interior end rows (local rows
// 1 and m-2); with fewer than one interior row they are not used.
template <typename T>
struct ChunkEnds {
  T phi1, psi1, phiL, psiL;
};

// Interior elimination, in place.  On entry r[0..m-1] holds the chunk's
// scaled right-hand side; on exit r[1..m-2] holds y and `e` the end values of
// phi and psi (r[0], r[m-1] are untouched).  The full phi_i, psi_i are not
// kept: chunk_interior forms them again from s when the chunk's end values
// are known.
//   forward:  dp_i = (dp_{i-1} - r_i) q_i   (den_i = -(1+g_i))
//   backward: y_i = dp_i + y_{i+1} q_i;  phi_i = fphi_i + phi_{i+1} q_i;
//             psi_i = psi_{i+1} q_i, with phi_last = fphi_last, psi_last = q_last
template <int MC, typename T>
PPE_HD void chunk_eliminate(cplx<T>* r, int m, T s, ChunkEnds<T>& e) {
  const int ni = m - 2;
  if (ni <= 0) return;
  T q[MC], fphi[MC];
  chunk_pivots<MC>(ni, s, q, fphi);
#pragma unroll
  for (int i = 0; i < MC - 2; ++i) {
    if (i < ni) {
      const cplx<T> ri = r[i + 1];
      if (i == 0) r[1] = mk(-ri.re * q[0], -ri.im * q[0]);
      else r[i + 1] = mk((r[i].re - ri.re) * q[i], (r[i].im - ri.im) * q[i]);
    }
  }
  T ph = T(0), ps = T(0);
#pragma unroll
  for (int i = MC - 3; i >= 0; --i) {
    if (i < ni) {
      if (i == ni - 1) {
        ph = fphi[i];
        ps = q[i];
        e.phiL = ph;
        e.psiL = ps;
      } else {
        r[i + 1] = mk(r[i + 1].re + r[i + 2].re * q[i], r[i + 1].im + r[i + 2].im * q[i]);
        ph = fphi[i] + ph * q[i];
        ps = ps * q[i];
      }
    }
  }
  e.phi1 = ph;
  e.psi1 = ps;
}

// x_i = y_i + phi_i x_first + psi_i x_last for the interior rows, in place,
// with phi_i and psi_i formed as in chunk_eliminate (same operations, same
// order, so the same values).
template <int MC, typename T>
PPE_HD void chunk_interior(cplx<T>* r, int m, T s, const cplx<T>& xf, const cplx<T>& xl) {
  const int ni = m - 2;
  if (ni <= 0) return;
  T q[MC], fphi[MC];
  chunk_pivots<MC>(ni, s, q, fphi);
  T ph = T(0), ps = T(0);
#pragma unroll
  for (int i = MC - 3; i >= 0; --i) {
    if (i < ni) {
      if (i == ni - 1) {
        ph = fphi[i];
        ps = q[i];
      } else {
        ph = fphi[i] + ph * q[i];
        ps = ps * q[i];
      }
      r[i + 1] = mk(r[i + 1].re + ph * xf.re + ps * xl.re, r[i + 1].im + ph * xf.im + ps * xl.im);
    }
  }
}

// The two reduced rows of a chunk (m >= 2 rows), after chunk_eliminate.
// Unknown order: (first_0, last_0, first_1, last_1, ...).
// first row: a * last_{p-1} + b * first_p + c * last_p = d
// last row : a * first_p + b * last_p + c * first_{p+1} = d
template <typename T>
struct RedRow {
  T a, b, c;
  cplx<T> d;
};

template <int MC, typename T>
PPE_HD void chunk_reduced_rows(const cplx<T>* r, const cplx<T>& r_first, const cplx<T>& r_last, int m, T s,
                               bool global_first, bool global_last, bool top_outflow, const ChunkEnds<T>& e,
                               RedRow<T>& f, RedRow<T>& l) {
  const T beta_first = global_first ? (-T(1) - s) : (-T(2) - s);
  const T beta_last = global_last ? ((top_outflow ? -T(3) : -T(1)) - s) : (-T(2) - s);
  const int ni = m - 2;
  // x_{j0+1} = y_1 + phi_1 first + psi_1 last   (x_{j1} itself when m == 2)
  T phi1 = T(0), psi1 = T(1), phiL = T(1), psiL = T(0);
  cplx<T> y1 = mk(T(0), T(0)), yL = mk(T(0), T(0));
  if (ni > 0) {
    phi1 = e.phi1;
    psi1 = e.psi1;
    phiL = e.phiL;
    psiL = e.psiL;
    y1 = r[1];
#pragma unroll
    for (int i = 0; i < MC - 2; ++i)
      if (i == ni - 1) yL = r[i + 1];
  }
  f.a = global_first ? T(0) : T(1);
  f.b = beta_first + phi1;
  f.c = psi1;
  f.d = csub(r_first, y1);
  l.a = phiL;
  l.b = beta_last + psiL;
  l.c = global_last ? T(0) : T(1);
  l.d = csub(r_last, yL);
}

// Two-ended (twisted) Thomas solve of the n reduced rows of one system, in
// place; on exit rows[i].d holds unknown i.  Thread `who` = 0 eliminates the
// sub-diagonal from the top over rows [0, h), thread 1 the super-diagonal
// from the bottom over rows [h, n), h = n/2; both chains run at once.  The
// reduced system inherits weak diagonal dominance from the y operator, so the
// sweeps are as stable as one Thomas sweep; cyclic reduction instead lost
// about two digits on the low modes.  The four phases are separated by the
// caller's barriers (red_twisted_meet between phase 1 and 2).
//   top:    x_i = d'_i - c'_i x_{i+1}      (stored as rows[i].c = c', .d = d')
//   bottom: x_i = d''_i - a''_i x_{i-1}    (stored as rows[i].a = a'', .d = d'')
// Row i of the system lives at rows[i * st] (systems of a block interleaved).
template <typename T>
PPE_HD void red_twisted_sweep(RedRow<T>* rows, int n, int who, int st) {
  const int h = n / 2;
  if (who == 0) {
    T cp = T(0);
    cplx<T> dp = mk(T(0), T(0));
    RedRow<T> nxt = rows[0];
    for (int i = 0; i < h; ++i) {
      const RedRow<T> r = nxt;
      if (i + 1 < h) nxt = rows[(i + 1) * st];
      const T inv = rcp_nr(r.b - r.a * cp);
      cp = r.c * inv;
      dp = mk((r.d.re - r.a * dp.re) * inv, (r.d.im - r.a * dp.im) * inv);
      rows[i * st].c = cp;
      rows[i * st].d = dp;
    }
  } else {
    T ap = T(0);
    cplx<T> dp = mk(T(0), T(0));
    RedRow<T> nxt = rows[(n - 1) * st];
    for (int i = n - 1; i >= h; --i) {
      const RedRow<T> r = nxt;
      if (i - 1 >= h) nxt = rows[(i - 1) * st];
      const T inv = rcp_nr(r.b - r.c * ap);
      ap = r.a * inv;
      dp = mk((r.d.re - r.c * dp.re) * inv, (r.d.im - r.c * dp.im) * inv);
      rows[i * st].a = ap;
      rows[i * st].d = dp;
    }
  }
}

// After both sweeps: x_{h-1} and x_h from the two meeting rows (thread 0 only;
// n >= 2).
template <typename T>
PPE_HD void red_twisted_meet(RedRow<T>* rows, int n, int st) {
  const int h = n / 2;
  const T c = rows[(h - 1) * st].c, a = rows[h * st].a;
  const cplx<T> d1 = rows[(h - 1) * st].d, d2 = rows[h * st].d;
  const T inv = rcp_nr(T(1) - c * a);
  const cplx<T> xm = mk((d1.re - c * d2.re) * inv, (d1.im - c * d2.im) * inv);
  rows[(h - 1) * st].d = xm;
  rows[h * st].d = mk(d2.re - a * xm.re, d2.im - a * xm.im);
}

// Substitution outward from the meeting rows.
template <typename T>
PPE_HD void red_twisted_subst(RedRow<T>* rows, int n, int who, int st) {
  const int h = n / 2;
  if (who == 0) {
    cplx<T> x = rows[(h - 1) * st].d;
    for (int i = h - 2; i >= 0; --i) {
      const RedRow<T> r = rows[i * st];
      x = mk(r.d.re - r.c * x.re, r.d.im - r.c * x.im);
      rows[i * st].d = x;
    }
  } else {
    cplx<T> x = rows[h * st].d;
    for (int i = h + 1; i < n; ++i) {
      const RedRow<T> r = rows[i * st];
      x = mk(r.d.re - r.a * x.re, r.d.im - r.a * x.im);
      rows[i * st].d = x;
    }
  }
}

}  // namespace ppe
