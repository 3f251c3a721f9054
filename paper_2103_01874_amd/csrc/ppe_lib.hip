// ppe_lib.hip -- plan, launch orchestration and the C ABI of include/ppe.h.
//
// One projection step of Poblador-Ibanez & Sirignano (arXiv 2103.01874),
// Sec. 5.4: right-hand side of Eq. (29), direct FFT/tridiagonal Poisson
// solve, projection of Eq. (28).  All arithmetic runs in the kernels of
// ppe_kernels.hip.inc; this file validates arguments, owns device memory and
// enqueues launches on the plan's stream.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <utility>
#include <new>
#include <string>
#include <vector>

#include "ppe.h"
#include "ppe_kernels.hpp"
#include "ppe_kernels.hip.inc"
#include "ppe_stencil.hip.inc"
#include "ppe_predict.hip.inc"
#include "ppe_plan_util.hpp"

using namespace ppe;

static_assert(sizeof(ppe_info_t) == sizeof(InfoRec), "ppe_info_t layout");
static_assert(sizeof(PtrTable) <= 4096, "kernel argument table too large");

namespace {

FftDev to_dev(const HostFft& h) {
  FftDev d;
  d.n = h.n;
  d.e = h.e;
  d.tc = h.tc;
  d.nst = h.nst;
  for (int s = 0; s < kMaxStages; ++s) {
    d.radix[s] = h.radix[s];
    d.ns[s] = h.ns[s];
    d.tstep[s] = h.tstep[s];
    d.inv_ns[s] = h.inv_ns[s];
  }
  d.tw = h.tw;
  return d;
}

}  // namespace

// ---------------------------------------------------------------------------
// Plan
// ---------------------------------------------------------------------------
struct ppe_plan_s {
  ppe_desc_t d;
  hipStream_t stream = nullptr;
  int device = 0;
  Geom g;
  HostFft fx, fz;
  // launch shapes
  int rp = 1;            // row pairs per block (x kernels)
  int tx = 1;            // kx columns per block (z FFT)
  int txs = 1, pch = 1;  // systems per block, chunks per system (tri)
  int mc = 16;           // register rows per chunk (template of k_tri)
  int fx_ct = 0, fz_ct = 0;  // lengths with a compile-time FFT plan (0: run-time plan)
  bool tri_refine = false;  // one difference-form refinement step in the y solve
  int spec_chunks = 1;   // kx chunks the spectral chain runs in (see launch_chain)
  int src_pt = 8;        // units per thread of k_source (2, 4 or 8)
  int src_vec = 2;       // cells per unit of k_source (1, or 2 when aligned)
  size_t lds_x = 0, lds_z = 0, lds_t = 0;
  // z-marching stencil tiles, one shape per kernel
  struct MarchCfg {
    March m;
    int grid = 0;    // blocks per instance
    int ppt = 1;     // interior points per thread per plane (kernel template)
    int nt = 256;    // threads per block (kernel template: 256, 512 or 1024)
    int tslots = 0;  // LDS slots of a tile plane with its halo ring
  } mrhs, mcor, mres, mrs;  // mres: k_resid_var; mrs: the refinement residual k_resid
  double* r64 = nullptr;   // refinement / fixed-point residual (mixed, or PPE_FLAG_VARCOEF)
  int r64_elem = 0;        // its bytes per cell: 8 (FP64, PPE_FLAG_VARCOEF) or 4 (mixed refinement only)
  // fixed-point iteration: convergence flags copied to pinned host memory
  // every few sweeps, so the host stops enqueuing once all instances converged
  double* conv_host = nullptr;      // [2][kMaxLaunch * kNScal], hipHostMalloc
  hipEvent_t conv_ev[2] = {nullptr, nullptr};
  // refinement of the y solve: k_tri blocks the plain launch skips (byte per
  // block, [kz][bx]) and the refining launch's block list (kz << 16 | bx)
  unsigned char* tri_skip = nullptr;
  int* tri_rblk = nullptr;
  int n_rblk = 0;
  long long pstride = 0;
  // device memory
  void* spec = nullptr;
  double* b64 = nullptr;
  double* rowsum = nullptr;
  double* colsum = nullptr;
  double* scal = nullptr;
  double* partial = nullptr;
  double* lamx = nullptr;
  double* lamz = nullptr;
  size_t bytes = 0;
  // opt-in per-kernel timing: HIP events around every launch on the stream
  bool prof = false;
  struct Pending {
    const char* name;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  std::map<std::string, std::pair<long, double>> acc;  // name -> (launches, total ms)
};

namespace {

// Launch-shape overrides for tuning sweeps (PPE_TUNE_* environment variables;
// unset = the built-in choice).  They change launch shapes only, never the
// arithmetic.
int tune_env(const char* name) {
  const char* v = std::getenv(name);
  return v ? std::atoi(v) : 0;
}

bool desc_ok(const ppe_desc_t* d) {
  if (!d) return false;
  if (d->nx < 1 || d->nz < 1 || d->ny < 2) return false;
  if (d->nx > kMaxN || d->nz > kMaxN || d->ny > kMaxN) return false;
  if (!(d->lx > 0) || !(d->ly > 0) || !(d->lz > 0)) return false;
  if (d->precision != PPE_PREC_FP64 && d->precision != PPE_PREC_MIXED) return false;
  if (d->ybc != PPE_YBC_WALLS && d->ybc != PPE_YBC_OUTFLOW) return false;
  if ((d->flags & ~(PPE_FLAG_VARCOEF | PPE_FLAG_Y_REFINE)) != 0 || d->reserved != 0) return false;
  if (d->batch < 1 || d->batch > PPE_MAX_BATCH) return false;
  if (d->max_refine < 0 || d->max_refine > 64) return false;
  if (!(d->tol >= 0)) return false;
  return true;
}

size_t spec_elem_bytes(const ppe_desc_t* d) {
  return d->precision == PPE_PREC_FP64 ? 2 * sizeof(double) : 2 * sizeof(float);
}

// Tile of a marching stencil kernel run by `nt` threads per block: TXT = nx
// when nx <= max_txt, else the largest divisor of nx up to max_txt; TJ rows so
// that a tile plane has about `points` interior cells; KC planes per chunk so
// that an instance gets about 2048 blocks.
bool march_shape(const ppe_desc_t& d, int points, int max_txt, const char* env, ppe_plan_s::MarchCfg& c,
                 int nt = kMarchThreads, int max_planes = 16) {
  March& M = c.m;
  c.nt = nt;
  if (tune_env("PPE_TUNE_TXT") > 0) max_txt = tune_env("PPE_TUNE_TXT");
  M.txt = d.nx;
  if (M.txt > max_txt) {
    M.txt = 1;
    for (int q = max_txt; q >= 1; --q)
      if (d.nx % q == 0) {
        M.txt = q;
        break;
      }
  }
  M.tj = std::max(1, std::min(points / M.txt, d.ny));
  if (tune_env(env) > 0) M.tj = std::max(1, std::min(tune_env(env), d.ny));
  while (M.tj > 1 && 2 * M.txt + 2 * M.tj > kRingPT * nt) --M.tj;
  if ((long long)M.tj * M.txt > (long long)nt * kMaxPPT) return false;
  M.ntx = d.nx / M.txt;
  M.ntj = (d.ny + M.tj - 1) / M.tj;
  const int target = tune_env("PPE_TUNE_MARCH_BLOCKS") > 0 ? tune_env("PPE_TUNE_MARCH_BLOCKS") : 2048;
  int nkc = std::max(1, (target + M.ntx * M.ntj - 1) / (M.ntx * M.ntj));
  // and at most 16 planes per block: with fewer, longer marches the final
  // set of resident blocks leaves the GPU idle for longer (512x256x512:
  // 128 planes per block, k_correct 1387 us; 16 planes, 1306 us)
  if (tune_env("PPE_TUNE_MAX_PLANES") > 0) max_planes = tune_env("PPE_TUNE_MAX_PLANES");
  nkc = std::max(nkc, (d.nz + max_planes - 1) / max_planes);
  nkc = std::min(nkc, std::max(1, d.nz / 2));
  M.kc = (d.nz + nkc - 1) / nkc;
  M.nkc = (d.nz + M.kc - 1) / M.kc;
  M.nt = M.ntx * M.ntj * M.nkc;
  M.per_xcd = (M.nt + 7) / 8;
  c.grid = 8 * M.per_xcd;
  const int npt = M.txt * M.tj;
  c.ppt = 1;
  while (c.ppt * nt < npt) c.ppt *= 2;
  c.tslots = (M.txt + 2) * (M.tj + 2);
  return true;
}

// Launch shapes and workspace sizes; fills p (no allocation).  `lds_limit`
// is the largest dynamic LDS a block may use (64 KiB without the per-kernel
// opt-in; 160 KiB on gfx950 with it).
bool shape_plan(ppe_plan_s* p, size_t lds_limit = 65536) {
  const ppe_desc_t& d = p->d;
  if (!fft_factor(d.nx, p->fx) || !fft_factor(d.nz, p->fz)) return false;
  {
    // compile-time plans: powers of two 16..2048, and 96, 192, 384
    const auto ct = [](int n) {
      return ((n >= 16 && n <= 2048 && (n & (n - 1)) == 0) || n == 96 || n == 192 || n == 384) ? n : 0;
    };
    const bool rt = tune_env("PPE_TUNE_RT_FFT") > 0;  // force the run-time plans
    p->fx_ct = rt ? 0 : ct(d.nx);
    p->fz_ct = rt ? 0 : ct(d.nz);
  }
  Geom& g = p->g;
  g.nx = d.nx;
  g.ny = d.ny;
  g.nz = d.nz;
  g.hx = d.nx / 2 + 1;
  g.ybc = d.ybc;
  g.tws = d.precision == PPE_PREC_FP64 ? 3 : 4;  // 128-byte kx tiles
  g.npts = (long long)d.nx * d.ny * d.nz;
  const long long ntile = (g.hx + (1 << g.tws) - 1) >> g.tws;
  g.spec_elems = (ntile << g.tws) * d.ny * d.nz;
  const double dx = d.lx / d.nx, dy = d.ly / d.ny, dz = d.lz / d.nz;
  g.dx = dx;
  g.dy = dy;
  g.dz = dz;
  g.idx = 1.0 / dx;
  g.idy = 1.0 / dy;
  g.idz = 1.0 / dz;
  g.dy2 = dy * dy;
  g.inv_nxnz = 1.0 / ((double)d.nx * (double)d.nz);
  // x kernels: RP row pairs of tc threads
  const int tcx = p->fx.tc;
  if (tcx > 512) return false;
  const size_t plen = (size_t)padded_len(d.nx);
  p->rp = std::max(1, 256 / tcx);
  // at most 40 KB of rows per block, so that four blocks fit a CU's LDS
  // (lengths with a radix-3 stage have 12 values per thread, so 256 threads
  // would hold 55 KB of rows: 192 x 96 x 192 row transforms 7-13% faster)
  while (p->rp > 1 && ((size_t)p->rp * plen * 16 > 40960 || p->rp * tcx > 512)) p->rp /= 2;
  p->lds_x = (size_t)p->rp * plen * 16;  // padded rows (twiddles are read from the global table)
  // z FFT: TX columns of tc threads
  const int tcz = p->fz.tc;
  if (tcz > 512) return false;
  // 8 kx columns per block when LDS allows (TX divides the tile: all of an
  // FP64 tile, half of an FP32 one, which measured faster than a full tile)
  p->tx = std::min(1 << g.tws, 8);
  if (tune_env("PPE_TUNE_TX") > 0) p->tx = std::min(1 << g.tws, tune_env("PPE_TUNE_TX"));
  while (p->tx > 1 && ((size_t)d.nz * (p->tx + kColPad) * 16 + (size_t)d.nz * 16 > lds_limit ||
                       p->tx * tcz > ((p->fz_ct && (p->fz_ct & (p->fz_ct - 1)) == 0) ? 1024 : 512)))
    p->tx /= 2;
  // columns + twiddle table (the plane-sum reduction reuses the column area)
  p->lds_z = std::max((size_t)d.nz * (p->tx + kColPad) * 16, (size_t)p->tx * tcz * 8) + (size_t)d.nz * 16;
  // tri: P chunks of 2..16 rows, TXS systems per block.  A block's time is
  // mostly its sequential reduced sweep over 2P rows, so the longest chunks
  // win despite their registers (16 rows against 8: 512x256x512 FP32 spectra
  // 134 against 196 us per launch; 64x2048x32 FP64 190 against 388 us)
  const int chunk = tune_env("PPE_TUNE_CHUNK") > 0 ? tune_env("PPE_TUNE_CHUNK") : 16;
  int P = (int)std::lround(d.ny / (double)chunk);
  P = std::max(P, (d.ny + kMaxChunk - 1) / kMaxChunk);
  P = std::min(P, d.ny / 2);
  P = std::max(P, 1);
  p->pch = P;
  p->txs = std::max(1, 256 / P);
  // whole 128-byte kx tiles per block where there is room (P = 6: 40 or 32
  // systems rather than 42), so that no line of the spectrum is split
  // between two blocks
  if (p->txs > (1 << g.tws)) p->txs -= p->txs % (1 << g.tws);
  if (p->txs * P > 256) return false;
  const int mmax = (d.ny + P - 1) / P;
  p->mc = mmax <= 4 ? 4 : (mmax <= 8 ? 8 : 16);
  // The elimination leaves about 4 eps / lambda_min relative error on a system
  // whose smallest eigenvalue is lambda_min (s for zero-flux ends, s +
  // 4 sin^2(pi / 4 ny) with the outflow top, 4 sin^2(pi / 2 ny) for the pinned
  // zero mode).  Above 256 rows the last two reach 1e-12 in the pressure of
  // ordinary fields; one refinement step of the y solve restores them.
  p->tri_refine = d.ny > 256 || (d.flags & PPE_FLAG_Y_REFINE) != 0;
  p->lds_t = std::max((size_t)p->txs * 2 * P * sizeof(RedRow<double>), (size_t)p->txs * P * 8);
  if (p->lds_x > 65536 || p->lds_z > lds_limit || p->lds_t > 65536) return false;
  // spectral-chain chunks of at most 192 MiB of spectrum (all instances), so
  // that a chunk stays in the 256 MB last-level cache through its z FFT,
  // tridiagonal and inverse z passes with room for the other streams
  // (512x256x512 FP64: 539 MB in 3 chunks, step 3.41 -> 3.22 ms; FP32
  // spectra there: 2 chunks; grids whose spectrum fits run unchunked)
  {
    const double spec_bytes = (double)d.batch * (double)g.spec_elems * (double)spec_elem_bytes(&d);
    p->spec_chunks = std::max(1, (int)std::ceil(spec_bytes / (192.0 * 1048576.0)));
  }
  if (tune_env("PPE_TUNE_SPEC_CHUNKS") > 0) p->spec_chunks = tune_env("PPE_TUNE_SPEC_CHUNKS");
  // target-divergence pass
  if (tune_env("PPE_TUNE_SRC_PT") > 0) p->src_pt = tune_env("PPE_TUNE_SRC_PT");
  if (tune_env("PPE_TUNE_SRC_VEC") > 0) p->src_vec = tune_env("PPE_TUNE_SRC_VEC");
  if (p->src_pt != 2 && p->src_pt != 4) p->src_pt = 8;
  if (p->src_vec != 1) p->src_vec = 2;
  // z-marching stencils: TXT x TJ tiles (TXT a divisor of nx, <= 128), KC planes
  // per chunk; the tile height per kernel trades halo traffic against registers
  // On large planes the two big stencils take 64x8 tiles, which fetch fewer
  // halo rows per interior row than 64x4 where those rows no longer stay in
  // L2: k_rhs with 512 threads, one point each (planes of >= 16 K cells);
  // k_correct with 256 threads, two points each (held to four waves per SIMD
  // by its launch bounds), marching up to 32 planes per block (planes of
  // >= 64 K cells).  512x256x512 FP64: k_rhs 947 -> 921 us, k_correct
  // 1284 -> 1241 us, step 3.23 -> 3.14 ms.  The residual passes take 64x8
  // tiles (two points per thread) on the same planes: k_resid of the
  // FP32-spectrum path 304 -> 273 us at 512x256x512 (at 256x128 planes
  // k_resid_var ran 60 -> 70 us that way).  On smaller planes the halo rows
  // hit L2 and the 64x4 tiles keep more waves in flight.
  const auto nt_of = [](const char* env, int def) {
    const int v = tune_env(env);
    return (v == 256 || v == 512 || v == 1024) ? v : def;
  };
  const long long plane_cells = (long long)d.nx * d.ny;
  const bool big_rhs = plane_cells >= 16384, big_cor = plane_cells >= 65536;
  const int nt_rhs = nt_of("PPE_TUNE_NT_RHS", big_rhs ? 512 : kMarchThreads);
  const int nt_cor = nt_of("PPE_TUNE_NT_COR", kMarchThreads);
  const int planes_cor =
      tune_env("PPE_TUNE_MAX_PLANES_COR") > 0 ? tune_env("PPE_TUNE_MAX_PLANES_COR") : (big_cor ? 32 : 16);
  if (!march_shape(d, big_rhs ? 512 : 256, 64, "PPE_TUNE_TJ_RHS", p->mrhs, nt_rhs) ||
      !march_shape(d, big_cor ? 512 : 256, 64, "PPE_TUNE_TJ_COR", p->mcor, nt_cor, planes_cor) ||
      !march_shape(d, big_cor ? 512 : 256, 64, "PPE_TUNE_TJ_RES", p->mres) ||
      // the refinement residual: 64 x 8 tiles at every plane size (against
      // 64 x 4 below 64 K cells: 7-17% faster from 64^3 to 256 x 128 x 256)
      !march_shape(d, 512, 64, "PPE_TUNE_TJ_RS", p->mrs))
    return false;
  if ((size_t)3 * p->mcor.tslots * 8 > 65536) return false;
  // per-instance partial-sum stride: the largest grid.x of a reducing kernel
  const long long nrows = (long long)d.ny * d.nz;
  const long long xgrid = (nrows + 1) / 2;  // bound on the row-pair grids, whatever the launch shape
  long long gmax = std::max<long long>(kRedBlocks, xgrid);
  gmax = std::max<long long>(gmax, std::max(p->mrhs.grid, std::max(p->mcor.grid, std::max(p->mres.grid, p->mrs.grid))));
  p->pstride = 4 * gmax;
  return true;
}

// FP64 residual buffer: refinement sweeps and the split fixed-point iteration
// Bytes per cell of the residual buffer: the fixed-point iteration keeps an
// FP64 residual; the mixed refinement alone stores it in FP32.
int r64_elem_bytes(const ppe_desc_t& d) {
  if ((d.flags & PPE_FLAG_VARCOEF) != 0) return 8;
  return d.precision == PPE_PREC_MIXED ? 4 : 0;
}
bool needs_r64(const ppe_desc_t& d) { return r64_elem_bytes(d) > 0; }

// Modified wavenumbers of the periodic directions (closed form of the 3-point
// second difference on its Fourier modes): lam_x over the half spectrum,
// lam_z over every kz.
void eig_tables(const ppe_plan_s* p, std::vector<double>& lx, std::vector<double>& lz) {
  const ppe_desc_t& d = p->d;
  const double dx = d.lx / d.nx, dz = d.lz / d.nz;
  const long double pi = 3.141592653589793238462643383279502884L;
  lx.assign(p->g.hx, 0.0);
  lz.assign(d.nz, 0.0);
  for (int a = 0; a < p->g.hx; ++a) {
    const long double s = sinl(pi * a / d.nx);
    lx[a] = (double)(-4.0L / ((long double)dx * dx) * s * s);
  }
  for (int c = 0; c < d.nz; ++c) {
    const long double s = sinl(pi * c / d.nz);
    lz[c] = (double)(-4.0L / ((long double)dz * dz) * s * s);
  }
}

// Below this s = -(lam_x + lam_z) dy^2 a y system takes the refining launch:
// the elimination alone loses ~4 eps / s there (4e-14 at the threshold).
constexpr double kTriTau = 1e-2;

// The k_tri blocks (TXS consecutive kx at one kz) holding a system with
// s < kTriTau, or the zero mode: skip mask [kz][bx] for the plain launch and
// the refining launch's list, one decision per block for both.
void tri_refine_blocks(const ppe_plan_s* p, const std::vector<double>& lx, const std::vector<double>& lz,
                       std::vector<unsigned char>& mask, std::vector<int>& list) {
  const int nbx = (p->g.hx + p->txs - 1) / p->txs;
  mask.assign((size_t)nbx * p->d.nz, 0);
  list.clear();
  for (int kz = 0; kz < p->d.nz; ++kz)
    for (int bx = 0; bx < nbx; ++bx) {
      bool small = bx == 0 && kz == 0;
      for (int kx = bx * p->txs; kx < std::min(p->g.hx, (bx + 1) * p->txs) && !small; ++kx)
        small = -(lx[kx] + lz[kz]) * p->g.dy2 < kTriTau;
      if (small) {
        mask[(size_t)kz * nbx + bx] = 1;
        list.push_back(kz << 16 | bx);
      }
    }
}

size_t workspace_bytes(const ppe_plan_s* p) {
  const ppe_desc_t& d = p->d;
  const size_t B = (size_t)d.batch;
  size_t s = 0;
  s += B * (size_t)p->g.spec_elems * spec_elem_bytes(&d);
  s += B * (size_t)p->g.npts * 8;                                       // b64
  s += B * (size_t)p->g.npts * r64_elem_bytes(d);                       // r64
  s += B * (size_t)d.ny * d.nz * 8;   // rowsum
  s += B * (size_t)d.ny * 8;          // colsum
  s += B * (size_t)kNScal * 8;        // scalars
  s += B * (size_t)p->pstride * 8;    // partials
  s += (size_t)(d.nx / 2 + 1) * 8 + (size_t)d.nz * 8;  // eigenvalue tables
  s += (size_t)2 * d.nx * 8 + (size_t)2 * d.nz * 8;    // twiddles
  if (p->tri_refine) {  // refining blocks of the y solve
    std::vector<double> lx, lz;
    std::vector<unsigned char> mask;
    std::vector<int> list;
    eig_tables(p, lx, lz);
    tri_refine_blocks(p, lx, lz, mask, list);
    s += std::max<size_t>(mask.size(), 8) + std::max<size_t>(list.size() * 4, 8);
  }
  return s;
}

template <typename T>
hipError_t dalloc(ppe_plan_s* p, T** ptr, size_t bytes) {
  if (bytes == 0) bytes = 8;
  hipError_t e = hipMalloc((void**)ptr, bytes);
  if (e == hipSuccess) p->bytes += bytes;
  return e;
}

void free_plan(ppe_plan_s* p) {
  if (!p) return;
  for (auto& e : p->pending) {
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  for (hipEvent_t e : p->pool) (void)hipEventDestroy(e);
  for (hipEvent_t e : p->conv_ev)
    if (e) (void)hipEventDestroy(e);
  if (p->conv_host) (void)hipHostFree(p->conv_host);
  void* ptrs[] = {p->spec, p->b64, p->r64, p->rowsum, p->colsum, p->scal, p->partial,
                  p->lamx, p->lamz, p->fx.tw, p->fz.tw, p->tri_skip, p->tri_rblk};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  delete p;
}

// LDS of a marching kernel holding `fields` row arrays (at least the block's
// reduction scratch, which reuses the same memory after the march)
size_t march_lds(const ppe_plan_s::MarchCfg& c, int fields) {
  return (size_t)std::max(fields * c.tslots, c.nt) * 8;
}

template <typename TS>
Work<TS> make_work(ppe_plan_s* p, int inst0) {
  Work<TS> w;
  w.spec = reinterpret_cast<cplx<TS>*>(p->spec);
  w.b64 = p->b64;
  w.rowsum = p->rowsum;
  w.colsum = p->colsum;
  w.scal = p->scal;
  w.partial = p->partial;
  w.pstride = p->pstride;
  w.lamx = p->lamx;
  w.lamz = p->lamz;
  w.inst0 = inst0;
  // Grids whose spectrum exceeds the last-level cache (a chunked chain): the
  // row transforms' outputs are next read after other passes have gone
  // through the cache, so they are stored non-temporally (512x256x512:
  // forward z transform 235 -> 221 us per step behind the forward rows;
  // k_correct 1186 -> 1166 us behind the inverse rows).  Where the spectrum
  // fits, the hint made the next pass slower (256x128x256: the forward z
  // transform 28.8 -> 31.8 us).  PPE_TUNE_NT_ROWS=1 forces it on, 2 off.
  const int nt = tune_env("PPE_TUNE_NT_ROWS");
  w.nt_rows = nt == 1 ? 1 : (nt == 2 ? 0 : (p->spec_chunks > 1 ? 1 : 0));
  return w;
}

// ---------------------------------------------------------------------------
// E dispatch for the FFT kernels
// ---------------------------------------------------------------------------
#define PPE_PPT_SWITCH(PVAL, CALL)                  \
  switch (PVAL) {                                   \
    case 1: { constexpr int PPT = 1; CALL; } break; \
    case 2: { constexpr int PPT = 2; CALL; } break; \
    case 4: { constexpr int PPT = 4; CALL; } break; \
    default: return PPE_ERR_UNSUPPORTED;            \
  }

// Launch CALL with PPT and NT the marching kernel's points per thread and
// threads per block of launch shape CFG.
#define PPE_MARCH_SWITCH(CFG, CALL)                                                  \
  switch ((CFG).nt * 8 + (CFG).ppt) {                                               \
    case 256 * 8 + 1: { constexpr int PPT = 1, NT = 256; CALL; } break;            \
    case 256 * 8 + 2: { constexpr int PPT = 2, NT = 256; CALL; } break;            \
    case 256 * 8 + 4: { constexpr int PPT = 4, NT = 256; CALL; } break;            \
    case 512 * 8 + 1: { constexpr int PPT = 1, NT = 512; CALL; } break;            \
    case 512 * 8 + 2: { constexpr int PPT = 2, NT = 512; CALL; } break;            \
    case 1024 * 8 + 1: { constexpr int PPT = 1, NT = 1024; CALL; } break;          \
    default: return PPE_ERR_UNSUPPORTED;                                            \
  }

#define PPE_E_SWITCH(EVAL, CALL)  \
  switch (EVAL) {                 \
    case 1: { constexpr int E = 1; CALL; } break;   \
    case 2: { constexpr int E = 2; CALL; } break;   \
    case 3: { constexpr int E = 3; CALL; } break;   \
    case 4: { constexpr int E = 4; CALL; } break;   \
    case 6: { constexpr int E = 6; CALL; } break;   \
    case 8: { constexpr int E = 8; CALL; } break;   \
    case 12: { constexpr int E = 12; CALL; } break; \
    default: return PPE_ERR_UNSUPPORTED;            \
  }

// Launch CALL with FV the kernels' FFT plan of the host plan HF and E its
// elements per thread: a compile-time CFft<N> when CT (the plan's
// power-of-two length, 16..2048), else the run-time plan.
#define PPE_FFT_CT_CASE(NN, HF, FV, CALL) \
  case NN: {                              \
    constexpr int E = CFft<NN>::e;        \
    const CFft<NN> FV{(HF).tw};           \
    CALL;                                 \
  } break;
#define PPE_FFT_SWITCH(CT, HF, FV, CALL)                                              \
  switch (CT) {                                                                     \
    PPE_FFT_CT_CASE(16, HF, FV, CALL)                                               \
    PPE_FFT_CT_CASE(32, HF, FV, CALL)                                               \
    PPE_FFT_CT_CASE(64, HF, FV, CALL)                                               \
    PPE_FFT_CT_CASE(128, HF, FV, CALL)                                              \
    PPE_FFT_CT_CASE(256, HF, FV, CALL)                                              \
    PPE_FFT_CT_CASE(512, HF, FV, CALL)                                              \
    PPE_FFT_CT_CASE(1024, HF, FV, CALL)                                             \
    PPE_FFT_CT_CASE(2048, HF, FV, CALL)                                             \
    PPE_FFT_CT_CASE(96, HF, FV, CALL)                                               \
    PPE_FFT_CT_CASE(192, HF, FV, CALL)                                              \
    PPE_FFT_CT_CASE(384, HF, FV, CALL)                                              \
    default: {                                                                      \
      const FftDev FV = to_dev(HF);                                                 \
      PPE_E_SWITCH(FV.e, CALL);                                                     \
    } break;                                                                        \
  }

hipEvent_t prof_event(ppe_plan_s* p) {
  if (!p->pool.empty()) {
    hipEvent_t e = p->pool.back();
    p->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

// Fold recorded event pairs into the per-kernel totals (waits for the stream).
void prof_collect(ppe_plan_s* p) {
  if (p->pending.empty()) return;
  (void)hipStreamSynchronize(p->stream);
  for (auto& e : p->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e.a, e.b) == hipSuccess) {
      auto& v = p->acc[e.name];
      v.first += 1;
      v.second += ms;
    }
    p->pool.push_back(e.a);
    p->pool.push_back(e.b);
  }
  p->pending.clear();
}

// Run a launch statement; with profiling on, bracket it with events.
#define PPE_TIMED(P, NAME, ...)                                              \
  do {                                                                       \
    hipEvent_t ev_a_ = nullptr;                                              \
    if ((P)->prof) {                                                         \
      ev_a_ = prof_event(P);                                                 \
      (void)hipEventRecord(ev_a_, (P)->stream);                              \
    }                                                                        \
    __VA_ARGS__;                                                             \
    if ((P)->prof) {                                                         \
      hipEvent_t ev_b_ = prof_event(P);                                      \
      (void)hipEventRecord(ev_b_, (P)->stream);                              \
      (P)->pending.push_back({NAME, ev_a_, ev_b_});                          \
      if ((P)->pending.size() > 4096) prof_collect(P);                       \
    }                                                                        \
  } while (0)

void finish(ppe_plan_s* p, const PtrTable& tab, int inst0, int nb, int nblk, int kind, int check,
            double tol = 0.0, double* out = nullptr, int ostride = 0) {
  PPE_TIMED(p, "k_finish",
            (k_finish<<<nb, kFinishThreads, 0, p->stream>>>(tab, p->g, p->scal, p->partial, p->pstride, nblk, inst0, kind, check,
                                                  tol, out, ostride)));
}

template <typename TS>
ppe_status_t launch_fft_z(ppe_plan_s* p, const Work<TS>& W, int nb, int dir, int check, int kx0, int kx1) {
  const Geom& g = p->g;
  dim3 grid(g.ny, (kx1 - kx0 + p->tx - 1) / p->tx, nb);
  dim3 block(p->tx * p->fz.tc);
  // two blocks per 128-byte tile row: pair them on one XCD (the range starts
  // on a tile; with an odd count the last block is a half tile at hx or the
  // range ends inside a tile, and that block keeps the plain order)
  const int pair = (p->tx * 2 == (1 << g.tws) && g.ny % 8 == 0 && kx0 % (2 * p->tx) == 0) ? 1 : 0;
  if (dir < 0) {
    PPE_TIMED(p, "k_fft_z_fwd",
              PPE_FFT_SWITCH(p->fz_ct, p->fz, fz,
                             (k_fft_z<TS, E, -1><<<grid, block, p->lds_z, p->stream>>>(g, fz, W, p->tx, check, kx0,
                                                                                      pair))));
  } else {
    PPE_TIMED(p, "k_fft_z_inv",
              PPE_FFT_SWITCH(p->fz_ct, p->fz, fz,
                             (k_fft_z<TS, E, +1><<<grid, block, p->lds_z, p->stream>>>(g, fz, W, p->tx, check, kx0,
                                                                                      pair))));
  }
  return PPE_OK;
}

// The spectral chain: forward z FFT, y tridiagonal solves, inverse z FFT.
// With spec_chunks > 1 it runs chunk by chunk over the kx range (boundaries
// on multiples of both the z kernel's and the tridiagonal kernel's kx
// blocks), so that a chunk of the spectrum can stay in the last-level cache
// between its three passes.
template <typename TS>
ppe_status_t launch_chain(ppe_plan_s* p, const Work<TS>& W, int nb, int check) {
  const Geom& g = p->g;
  dim3 tblock(p->txs * p->pch);
  const bool full = g.ny == p->pch * p->mc;
  const int nbx = (g.hx + p->txs - 1) / p->txs;
  // with refinement (ny > 256 or PPE_FLAG_Y_REFINE) the plain launch skips
  // the blocks holding a system of s < kTriTau or the zero mode, and the
  // refining launch runs just those, one block per list entry
  const unsigned char* skip = p->tri_refine ? p->tri_skip : nullptr;
  const dim3 rgrid(std::max(p->n_rblk, 1), 1, nb);
  const int unit = std::lcm(p->tx, p->txs);  // kx per chunk step
  const int units = (g.hx + unit - 1) / unit;
  const int nch = p->tri_refine ? 1 : std::max(1, std::min(p->spec_chunks, units));
  for (int c = 0; c < nch; ++c) {
    const int u0 = (int)((long long)units * c / nch), u1 = (int)((long long)units * (c + 1) / nch);
    const int kx0 = u0 * unit, kx1 = std::min(g.hx, u1 * unit);
    const int bx0 = kx0 / p->txs, bx1 = (c == nch - 1) ? nbx : kx1 / p->txs;
    ppe_status_t st = launch_fft_z<TS>(p, W, nb, -1, check, kx0, kx1);
    if (st != PPE_OK) return st;
    const dim3 tgrid(bx1 - bx0, g.nz, nb);
#define PPE_TRI(MCV, FULLV)                                                                              \
  do {                                                                                                   \
    k_tri<TS, MCV, FULLV, false><<<tgrid, tblock, p->lds_t, p->stream>>>(g, W, p->txs, p->pch, check,    \
                                                                         skip, nullptr, bx0, nbx);       \
    if (p->tri_refine && p->n_rblk > 0)                                                                  \
      k_tri<TS, MCV, FULLV, true><<<rgrid, tblock, p->lds_t, p->stream>>>(g, W, p->txs, p->pch, check,   \
                                                                          nullptr, p->tri_rblk, 0, nbx); \
  } while (0)
    PPE_TIMED(p, "k_tri", {
      if (p->mc == 4 && full) PPE_TRI(4, true);
      else if (p->mc == 4) PPE_TRI(4, false);
      else if (p->mc == 8 && full) PPE_TRI(8, true);
      else if (p->mc == 8) PPE_TRI(8, false);
      else if (full) PPE_TRI(16, true);
      else PPE_TRI(16, false);
    });
#undef PPE_TRI
    st = launch_fft_z<TS>(p, W, nb, +1, check, kx0, kx1);
    if (st != PPE_OK) return st;
  }
  return PPE_OK;
}

// rho0 = min(rho) on the device for the instances that ask for it (Eq. 27)
void rho_min_pass(ppe_plan_s* p, const PtrTable& tab, int inst0, int nb) {
  const Geom& g = p->g;
  bool need_min = false;
  for (int i = 0; i < nb; ++i) need_min |= !(tab.in[i].rho0_in > 0.0);
  if (!need_min) return;
  PPE_TIMED(p, "k_rho_min_init", (k_rho_min_init<<<1, 64, 0, p->stream>>>(p->scal, inst0, nb)));
  const long long blocks = std::min<long long>((g.npts + 255) / 256, 1024);
  PPE_TIMED(p, "k_rho_min", (k_rho_min<<<dim3((unsigned)blocks, 1, nb), 256, 0, p->stream>>>(tab, g, p->scal, inst0)));
  PPE_TIMED(p, "k_rho_min_finish", (k_rho_min_finish<<<1, 64, 0, p->stream>>>(tab, p->scal, inst0, nb)));
}

template <typename TS>
ppe_status_t solve_typed(ppe_plan_s* p, const PtrTable& tab, int inst0, int nb) {
  const Geom& g = p->g;
  Work<TS> W = make_work<TS>(p, inst0);
  const bool mixed = p->d.precision == PPE_PREC_MIXED;
  const double tol = mixed ? p->d.tol : 0.0;
  rho_min_pass(p, tab, inst0, nb);
  const long long nrows = (long long)g.ny * g.nz;
  const long long npairs = (nrows + 1) / 2;
  dim3 xgrid((unsigned)((npairs + p->rp - 1) / p->rp), 1, nb);
  dim3 xblock(p->rp * p->fx.tc);
  PPE_TIMED(p, "k_rhs",
            PPE_MARCH_SWITCH(p->mrhs, (k_rhs<TS, PPT, true, NT><<<dim3(p->mrhs.grid, 1, nb), NT, march_lds(p->mrhs, 2),
                                                              p->stream>>>(tab, g, p->mrhs.m, W))));
  // the right-hand-side sums are reduced by block 0 of the first row FFT
  PPE_TIMED(p, "k_r2c",
            PPE_FFT_SWITCH(p->fx_ct, p->fx, fx, (k_r2c<TS, E><<<xgrid, xblock, p->lds_x, p->stream>>>(
                                   tab, g, fx, W, p->b64, p->rp, 0, FinishArgs{p->mrhs.grid, tol}))));
  ppe_status_t st = launch_chain<TS>(p, W, nb, 0);
  if (st != PPE_OK) return st;
  PPE_TIMED(p, "k_c2r",
            PPE_FFT_SWITCH(p->fx_ct, p->fx, fx, (k_c2r<TS, E><<<xgrid, xblock, p->lds_x, p->stream>>>(
                                   tab, g, fx, W, p->rp, 0, 0))));
  if (mixed) {
    // the refinement residual in the spectrum's precision (the first half of
    // the FP64 residual buffer)
    TS* rs = reinterpret_cast<TS*>(p->r64);
    for (int it = 0; it < p->d.max_refine; ++it) {
      PPE_TIMED(p, "k_resid",
                PPE_PPT_SWITCH(p->mrs.ppt, (k_resid<TS, PPT><<<dim3(p->mrs.grid, 1, nb), kMarchThreads,
                                                               march_lds(p->mrs, 1), p->stream>>>(
                                                tab, g, p->mrs.m, W, rs))));
      finish(p, tab, inst0, nb, p->mrs.grid, FIN_RESID, 1);
      PPE_TIMED(p, "k_r2c",
                PPE_FFT_SWITCH(p->fx_ct, p->fx, fx, (k_r2c<TS, E><<<xgrid, xblock, p->lds_x, p->stream>>>(
                                       tab, g, fx, W, static_cast<const TS*>(rs), p->rp, 1, FinishArgs{0, 0.0}))));
      st = launch_chain<TS>(p, W, nb, 1);
      if (st != PPE_OK) return st;
      PPE_TIMED(p, "k_c2r",
                PPE_FFT_SWITCH(p->fx_ct, p->fx, fx, (k_c2r<TS, E><<<xgrid, xblock, p->lds_x, p->stream>>>(
                                       tab, g, fx, W, p->rp, 1, 1))));
    }
  }
  return hipGetLastError() == hipSuccess ? PPE_OK : PPE_ERR_DEVICE;
}

// Split fixed-point iteration (Sec. 5.4): p_0 = 2 p^n - p^{n-1},
// p_{k+1} = p_k + L^+ [c - rho0 D((1/rho_f) G p_k)], c = (rho0/dt)(D u* - S).
// p_1 is the split solve; the fixed point is the pressure of Eq. (25).
// Residual k is recorded in hist[inst][k] (k = 0 .. max_iters).
template <typename TS>
ppe_status_t varcoef_typed(ppe_plan_s* p, const PtrTable& tab, int inst0, int nb, int max_iters, double tol,
                           double* hist) {
  const Geom& g = p->g;
  Work<TS> W = make_work<TS>(p, inst0);
  rho_min_pass(p, tab, inst0, nb);
  const long long nrows = (long long)g.ny * g.nz;
  const long long npairs = (nrows + 1) / 2;
  dim3 xgrid((unsigned)((npairs + p->rp - 1) / p->rp), 1, nb);
  dim3 xblock(p->rp * p->fx.tc);
  PPE_TIMED(p, "k_rhs",
            PPE_MARCH_SWITCH(p->mrhs, (k_rhs<TS, PPT, false, NT><<<dim3(p->mrhs.grid, 1, nb), NT,
                                                               march_lds(p->mrhs, 1), p->stream>>>(tab, g,
                                                                                                   p->mrhs.m, W))));
  finish(p, tab, inst0, nb, p->mrhs.grid, FIN_RHS, 0, tol);
  const int hs = max_iters + 1;
  double* h0 = hist ? hist + (size_t)inst0 * hs : nullptr;
  if (h0) {
    const long long n = (long long)nb * hs;
    PPE_TIMED(p, "k_fill", (k_fill<<<(unsigned)((n + 255) / 256), 256, 0, p->stream>>>(h0, n, -1.0)));
  }
  // every kPoll sweeps the instances' scalars go to pinned host memory behind
  // an event; before enqueuing more, the host reads the previous chunk's copy
  // (one chunk of run-ahead keeps the device busy) and stops once every
  // instance has converged
  constexpr int kPoll = 4;
  for (int it = 0; it <= max_iters; ++it) {
    if (it > 0 && it % kPoll == 0 && tol > 0.0) {
      const int c = it / kPoll;
      double* h = p->conv_host + (size_t)(c & 1) * kMaxLaunch * kNScal;
      if (hipMemcpyAsync(h, p->scal + (size_t)inst0 * kNScal, (size_t)nb * kNScal * sizeof(double),
                         hipMemcpyDeviceToHost, p->stream) != hipSuccess ||
          hipEventRecord(p->conv_ev[c & 1], p->stream) != hipSuccess)
        return PPE_ERR_DEVICE;
      if (c >= 2) {
        if (hipEventSynchronize(p->conv_ev[(c - 1) & 1]) != hipSuccess) return PPE_ERR_DEVICE;
        const double* hp = p->conv_host + (size_t)((c - 1) & 1) * kMaxLaunch * kNScal;
        bool all = true;
        for (int i = 0; i < nb; ++i) all = all && hp[(size_t)i * kNScal + SC_CONV] != 0.0;
        if (all) break;
      }
    }
    if (it == 0)
      PPE_TIMED(p, "k_resid_var",
                PPE_PPT_SWITCH(p->mres.ppt, (k_resid_var<TS, PPT, 1><<<dim3(p->mres.grid, 1, nb), kMarchThreads,
                                                                         march_lds(p->mres, 2), p->stream>>>(
                                                tab, g, p->mres.m, W, p->r64, 1))));
    else
      PPE_TIMED(p, "k_resid_var",
                PPE_PPT_SWITCH(p->mres.ppt, (k_resid_var<TS, PPT, 0><<<dim3(p->mres.grid, 1, nb), kMarchThreads,
                                                                          march_lds(p->mres, 2), p->stream>>>(
                                                tab, g, p->mres.m, W, p->r64, 1))));
    finish(p, tab, inst0, nb, p->mres.grid, it == max_iters ? FIN_RESID_LAST : FIN_RESID, 1, 0.0,
           h0 ? h0 + it : nullptr, hs);
    if (it == max_iters) break;
    PPE_TIMED(p, "k_r2c",
              PPE_FFT_SWITCH(p->fx_ct, p->fx, fx, (k_r2c<TS, E><<<xgrid, xblock, p->lds_x, p->stream>>>(
                                     tab, g, fx, W, p->r64, p->rp, 1, FinishArgs{0, 0.0}))));
    ppe_status_t st = launch_chain<TS>(p, W, nb, 1);
    if (st != PPE_OK) return st;
    PPE_TIMED(p, "k_c2r",
              PPE_FFT_SWITCH(p->fx_ct, p->fx, fx, (k_c2r<TS, E><<<xgrid, xblock, p->lds_x, p->stream>>>(tab, g, fx, W, p->rp, 1, 1))));
  }
  return hipGetLastError() == hipSuccess ? PPE_OK : PPE_ERR_DEVICE;
}

// Split defect of a projection step (Sec. 5.4): the relative residual of the
// variable-coefficient problem, Eq. (25), for p_hat (out[2 b]) and for the
// split pressure p^{n+1} that ppe_solve left in tab.p (out[2 b + 1]), both in
// FP64.  Runs after that solve, on its scalars (rho0, the stop scale and the
// mean of the right-hand side); c = (rho0/dt)(D u* - S) replaces b in b64.
template <typename TS>
ppe_status_t defect_typed(ppe_plan_s* p, const PtrTable& tab, int inst0, int nb, double* out) {
  Work<TS> W = make_work<TS>(p, inst0);
  PPE_TIMED(p, "k_rhs",
            PPE_MARCH_SWITCH(p->mrhs, (k_rhs<TS, PPT, false, NT><<<dim3(p->mrhs.grid, 1, nb), NT,
                                                               march_lds(p->mrhs, 1), p->stream>>>(tab, p->g,
                                                                                                   p->mrhs.m, W))));
  PPE_TIMED(p, "k_resid_var",
            PPE_PPT_SWITCH(p->mres.ppt, (k_resid_var<TS, PPT, 2><<<dim3(p->mres.grid, 1, nb), kMarchThreads,
                                                                   march_lds(p->mres, 2), p->stream>>>(
                                            tab, p->g, p->mres.m, W, p->r64, 0))));
  finish(p, tab, inst0, nb, p->mres.grid, FIN_DEFECT, 0, 0.0, out + 2 * (size_t)inst0, 2);
  PPE_TIMED(p, "k_resid_var",
            PPE_PPT_SWITCH(p->mres.ppt, (k_resid_var<TS, PPT, 0><<<dim3(p->mres.grid, 1, nb), kMarchThreads,
                                                                   march_lds(p->mres, 2), p->stream>>>(
                                            tab, p->g, p->mres.m, W, p->r64, 0))));
  finish(p, tab, inst0, nb, p->mres.grid, FIN_DEFECT, 0, 0.0, out + 2 * (size_t)inst0 + 1, 2);
  return hipGetLastError() == hipSuccess ? PPE_OK : PPE_ERR_DEVICE;
}

bool ptrs_ok(const void* const* a, int n) {
  if (!a) return false;
  for (int i = 0; i < n; ++i)
    if (!a[i]) return false;
  return true;
}

}  // namespace

namespace {
// Dynamic LDS above 64 KiB must be enabled per kernel (all z-FFT variants).
template <typename TS, int E, typename F = FftDev>
hipError_t allow_big_lds_e(int bytes) {
  const void* fns[] = {reinterpret_cast<const void*>(&k_fft_z<TS, E, -1, F>),
                       reinterpret_cast<const void*>(&k_fft_z<TS, E, +1, F>)};
  for (const void* f : fns) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
template <typename TS>
hipError_t allow_big_lds_t(int bytes) {
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = allow_big_lds_e<TS, 1>(bytes);
  if (e == hipSuccess) e = allow_big_lds_e<TS, 2>(bytes);
  if (e == hipSuccess) e = allow_big_lds_e<TS, 3>(bytes);
  if (e == hipSuccess) e = allow_big_lds_e<TS, 4>(bytes);
  if (e == hipSuccess) e = allow_big_lds_e<TS, 6>(bytes);
  if (e == hipSuccess) e = allow_big_lds_e<TS, 8>(bytes);
  if (e == hipSuccess) e = allow_big_lds_e<TS, 12>(bytes);
  if (e == hipSuccess) e = allow_big_lds_e<TS, CFft<16>::e, CFft<16>>(bytes);
  if (e == hipSuccess) e = allow_big_lds_e<TS, CFft<32>::e, CFft<32>>(bytes);
  if (e == hipSuccess) e = allow_big_lds_e<TS, CFft<64>::e, CFft<64>>(bytes);
  if (e == hipSuccess) e = allow_big_lds_e<TS, CFft<128>::e, CFft<128>>(bytes);
  if (e == hipSuccess) e = allow_big_lds_e<TS, CFft<256>::e, CFft<256>>(bytes);
  if (e == hipSuccess) e = allow_big_lds_e<TS, CFft<512>::e, CFft<512>>(bytes);
  if (e == hipSuccess) e = allow_big_lds_e<TS, CFft<1024>::e, CFft<1024>>(bytes);
  if (e == hipSuccess) e = allow_big_lds_e<TS, CFft<2048>::e, CFft<2048>>(bytes);
  if (e == hipSuccess) e = allow_big_lds_e<TS, CFft<96>::e, CFft<96>>(bytes);
  if (e == hipSuccess) e = allow_big_lds_e<TS, CFft<192>::e, CFft<192>>(bytes);
  if (e == hipSuccess) e = allow_big_lds_e<TS, CFft<384>::e, CFft<384>>(bytes);
  return e;
}
hipError_t allow_big_lds(int bytes) {
  hipError_t e = allow_big_lds_t<double>(bytes);
  return e == hipSuccess ? allow_big_lds_t<float>(bytes) : e;
}

}  // namespace

// ---------------------------------------------------------------------------
// Workspace for callers that cannot allocate: one file-scope device array per
// GPU, held until the process ends.  Host code never uses the array's name as
// an address: its device address comes from hipGetSymbolAddress, looked up
// once per device with that device current, and is what kernels receive.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB per GPU
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {nullptr};

// Device address of `scratch` on device `dev` (the current device), looked up
// and the large-LDS kernel attributes set on the first call for that device.
void* scratch_on(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev]) return g_scratch_ptr[dev];
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
  int lds_max = 65536;
  if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return nullptr;
  if (lds_max > 65536 && allow_big_lds(lds_max) != hipSuccess) return nullptr;
  g_scratch_ptr[dev] = ptr;
  return ptr;
}

// Twiddle tables exp(-2 pi i t / n) and the eigenvalue tables of the periodic
// directions, on the device (sinpi / sincospi in FP64; exact values where the
// circle meets the axes), for a workspace built without host copies.
__global__ __launch_bounds__(256) void k_tables(double* twx, int nx, double* twz, int nz, double* lamx, int hx,
                                                double* lamz, double dx, double dz) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const auto tw = [](double* w, int n, int q) {
    double s, c;
    sincospi(2.0 * q / n, &s, &c);
    if ((4LL * q) % n == 0) {
      const int qq = (int)((4LL * q / n) % 4);
      c = qq == 0 ? 1.0 : (qq == 2 ? -1.0 : 0.0);
      s = qq == 1 ? 1.0 : (qq == 3 ? -1.0 : 0.0);
    }
    w[2 * q] = c;
    w[2 * q + 1] = -s;
  };
  if (t < nx) tw(twx, nx, t);
  if (t < nz) tw(twz, nz, t);
  if (t < hx) {
    const double s = sinpi((double)t / nx);
    lamx[t] = -4.0 / (dx * dx) * s * s;
  }
  if (t < nz) {
    const double s = sinpi((double)t / nz);
    lamz[t] = -4.0 / (dz * dz) * s * s;
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

size_t ppe_plan_workspace_bytes(const ppe_desc_t* desc) {
  if (!desc_ok(desc)) return 0;
  ppe_plan_s tmp;
  tmp.d = *desc;
  if (!shape_plan(&tmp)) return 0;
  return workspace_bytes(&tmp);
}

ppe_status_t ppe_plan(const ppe_desc_t* desc, void* stream, ppe_plan_t* out) {
  if (!out) return PPE_ERR_ARG;
  *out = nullptr;
  if (!desc_ok(desc)) return PPE_ERR_ARG;
  ppe_plan_s* p = new (std::nothrow) ppe_plan_s();
  if (!p) return PPE_ERR_NOMEM;
  p->d = *desc;
  p->stream = reinterpret_cast<hipStream_t>(stream);
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return PPE_ERR_DEVICE;
  }
  int lds_max = 65536;
  if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, p->device) != hipSuccess)
    lds_max = 65536;
  if (!shape_plan(p, (size_t)std::max(lds_max, 65536))) {
    delete p;
    return PPE_ERR_UNSUPPORTED;
  }
  if (p->lds_z > 65536 && allow_big_lds((int)p->lds_z) != hipSuccess) {
    delete p;
    return PPE_ERR_DEVICE;
  }
  const ppe_desc_t& d = p->d;
  const size_t B = (size_t)d.batch;
  bool ok = true;
  ok &= dalloc(p, (char**)&p->spec, B * (size_t)p->g.spec_elems * spec_elem_bytes(&d)) == hipSuccess;
  ok &= dalloc(p, &p->b64, B * (size_t)p->g.npts * 8) == hipSuccess;
  if (needs_r64(d)) {
    p->r64_elem = r64_elem_bytes(d);
    ok &= dalloc(p, &p->r64, B * (size_t)p->g.npts * p->r64_elem) == hipSuccess;
    ok &= hipHostMalloc((void**)&p->conv_host, 2 * kMaxLaunch * kNScal * sizeof(double), hipHostMallocDefault) ==
          hipSuccess;
    for (hipEvent_t& e : p->conv_ev) ok &= hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
  }
  ok &= dalloc(p, &p->rowsum, B * (size_t)d.ny * d.nz * 8) == hipSuccess;
  ok &= dalloc(p, &p->colsum, B * (size_t)d.ny * 8) == hipSuccess;
  ok &= dalloc(p, &p->scal, B * kNScal * 8) == hipSuccess;
  ok &= dalloc(p, &p->partial, B * (size_t)p->pstride * 8) == hipSuccess;
  ok &= dalloc(p, &p->lamx, (size_t)p->g.hx * 8) == hipSuccess;
  ok &= dalloc(p, &p->lamz, (size_t)d.nz * 8) == hipSuccess;
  ok &= dalloc(p, &p->fx.tw, (size_t)2 * d.nx * 8) == hipSuccess;
  ok &= dalloc(p, &p->fz.tw, (size_t)2 * d.nz * 8) == hipSuccess;
  if (!ok) {
    free_plan(p);
    return PPE_ERR_NOMEM;
  }
  std::vector<double> lx, lz;
  eig_tables(p, lx, lz);
  if (p->tri_refine) {
    std::vector<unsigned char> mask;
    std::vector<int> list;
    tri_refine_blocks(p, lx, lz, mask, list);
    p->n_rblk = (int)list.size();
    ok &= dalloc(p, &p->tri_skip, mask.size()) == hipSuccess;
    ok &= dalloc(p, &p->tri_rblk, list.size() * 4) == hipSuccess;
    if (ok) {
      ok &= hipMemcpy(p->tri_skip, mask.data(), mask.size(), hipMemcpyHostToDevice) == hipSuccess;
      if (!list.empty())
        ok &= hipMemcpy(p->tri_rblk, list.data(), list.size() * 4, hipMemcpyHostToDevice) == hipSuccess;
    }
  }
  std::vector<double> twx = twiddles(d.nx), twz = twiddles(d.nz);
  ok &= hipMemcpy(p->lamx, lx.data(), lx.size() * 8, hipMemcpyHostToDevice) == hipSuccess;
  ok &= hipMemcpy(p->lamz, lz.data(), lz.size() * 8, hipMemcpyHostToDevice) == hipSuccess;
  ok &= hipMemcpy(p->fx.tw, twx.data(), twx.size() * 8, hipMemcpyHostToDevice) == hipSuccess;
  ok &= hipMemcpy(p->fz.tw, twz.data(), twz.size() * 8, hipMemcpyHostToDevice) == hipSuccess;
  if (!ok) {
    free_plan(p);
    return PPE_ERR_DEVICE;
  }
  *out = p;
  return PPE_OK;
}

ppe_status_t ppe_plan_destroy(ppe_plan_t plan) {
  if (!plan) return PPE_ERR_ARG;
  (void)hipStreamSynchronize(plan->stream);
  free_plan(plan);
  return PPE_OK;
}

ppe_status_t ppe_plan_set_stream(ppe_plan_t plan, void* stream) {
  if (!plan) return PPE_ERR_ARG;
  plan->stream = reinterpret_cast<hipStream_t>(stream);
  return PPE_OK;
}

ppe_status_t ppe_solve(ppe_plan_t p, const double* rho0, const double* dt, const double* const* us,
                       const double* const* vs, const double* const* ws, const double* const* rho,
                       const double* const* pn, const double* const* pnm1, const double* const* S,
                       double* const* pout, ppe_info_t* info) {
  if (!p || !rho0 || !dt || !info) return PPE_ERR_ARG;
  const int B = p->d.batch;
  if (!ptrs_ok((const void* const*)us, B) || !ptrs_ok((const void* const*)vs, B) ||
      !ptrs_ok((const void* const*)ws, B) || !ptrs_ok((const void* const*)rho, B) ||
      !ptrs_ok((const void* const*)pn, B) || !ptrs_ok((const void* const*)pnm1, B) ||
      !ptrs_ok((const void* const*)S, B) || !ptrs_ok((const void* const*)pout, B))
    return PPE_ERR_ARG;
  for (int i = 0; i < B; ++i)
    if (!(dt[i] > 0) || !std::isfinite(dt[i]) || std::isnan(rho0[i])) return PPE_ERR_ARG;
  if (hipSetDevice(p->device) != hipSuccess) return PPE_ERR_DEVICE;
  for (int i0 = 0; i0 < B; i0 += kMaxLaunch) {
    const int nb = std::min(kMaxLaunch, B - i0);
    PtrTable tab;
    std::memset(&tab, 0, sizeof(tab));
    for (int i = 0; i < nb; ++i) {
      InstPtrs& q = tab.in[i];
      q.us = us[i0 + i];
      q.vs = vs[i0 + i];
      q.ws = ws[i0 + i];
      q.rho = rho[i0 + i];
      q.pn = pn[i0 + i];
      q.pnm1 = pnm1[i0 + i];
      q.S = S[i0 + i];
      q.p = pout[i0 + i];
      q.info = info + i0 + i;
      q.rho0_in = rho0[i0 + i];
      q.dt = dt[i0 + i];
    }
    ppe_status_t st = (p->d.precision == PPE_PREC_FP64) ? solve_typed<double>(p, tab, i0, nb)
                                                         : solve_typed<float>(p, tab, i0, nb);
    if (st != PPE_OK) return st;
  }
  return PPE_OK;
}

ppe_status_t ppe_rhs(ppe_plan_t p, const double* rho0, const double* dt, const double* const* us,
                     const double* const* vs, const double* const* ws, const double* const* rho,
                     const double* const* pn, const double* const* pnm1, const double* const* S, double* const* b,
                     ppe_info_t* info) {
  if (!p || !rho0 || !dt || !info) return PPE_ERR_ARG;
  const int B = p->d.batch;
  if (!ptrs_ok((const void* const*)us, B) || !ptrs_ok((const void* const*)vs, B) ||
      !ptrs_ok((const void* const*)ws, B) || !ptrs_ok((const void* const*)rho, B) ||
      !ptrs_ok((const void* const*)pn, B) || !ptrs_ok((const void* const*)pnm1, B) ||
      !ptrs_ok((const void* const*)S, B) || !ptrs_ok((const void* const*)b, B))
    return PPE_ERR_ARG;
  for (int i = 0; i < B; ++i)
    if (!(dt[i] > 0) || !std::isfinite(dt[i]) || std::isnan(rho0[i])) return PPE_ERR_ARG;
  if (hipSetDevice(p->device) != hipSuccess) return PPE_ERR_DEVICE;
  const Geom& g = p->g;
  for (int i0 = 0; i0 < B; i0 += kMaxLaunch) {
    const int nb = std::min(kMaxLaunch, B - i0);
    PtrTable tab;
    std::memset(&tab, 0, sizeof(tab));
    for (int i = 0; i < nb; ++i) {
      InstPtrs& q = tab.in[i];
      q.us = us[i0 + i];
      q.vs = vs[i0 + i];
      q.ws = ws[i0 + i];
      q.rho = rho[i0 + i];
      q.pn = pn[i0 + i];
      q.pnm1 = pnm1[i0 + i];
      q.S = S[i0 + i];
      q.info = info + i0 + i;
      q.rho0_in = rho0[i0 + i];
      q.dt = dt[i0 + i];
    }
    rho_min_pass(p, tab, i0, nb);
    Work<double> W = make_work<double>(p, i0);
    PPE_TIMED(p, "k_rhs",
              PPE_MARCH_SWITCH(p->mrhs, (k_rhs<double, PPT, true, NT><<<dim3(p->mrhs.grid, 1, nb), NT,
                                                                    march_lds(p->mrhs, 2), p->stream>>>(
                                               tab, g, p->mrhs.m, W))));
    finish(p, tab, i0, nb, p->mrhs.grid, FIN_RHS, 0);
    for (int i = 0; i < nb; ++i)
      if (hipMemcpyAsync(b[i0 + i], p->b64 + (size_t)(i0 + i) * g.npts, (size_t)g.npts * sizeof(double),
                         hipMemcpyDeviceToDevice, p->stream) != hipSuccess)
        return PPE_ERR_DEVICE;
  }
  return hipGetLastError() == hipSuccess ? PPE_OK : PPE_ERR_DEVICE;
}

ppe_status_t ppe_solve_varcoef(ppe_plan_t p, const double* rho0, const double* dt, const double* const* us,
                               const double* const* vs, const double* const* ws, const double* const* rho,
                               const double* const* pn, const double* const* pnm1, const double* const* S,
                               double* const* pout, ppe_info_t* info, int32_t max_iters, double tol,
                               double* hist) {
  if (!p || !rho0 || !dt || !info) return PPE_ERR_ARG;
  if (!p->r64 || p->r64_elem != 8) return PPE_ERR_ARG;  // plan built without the FP64 residual buffer
  if (max_iters < 0 || max_iters > 100000 || !(tol >= 0)) return PPE_ERR_ARG;
  const int B = p->d.batch;
  if (!ptrs_ok((const void* const*)us, B) || !ptrs_ok((const void* const*)vs, B) ||
      !ptrs_ok((const void* const*)ws, B) || !ptrs_ok((const void* const*)rho, B) ||
      !ptrs_ok((const void* const*)pn, B) || !ptrs_ok((const void* const*)pnm1, B) ||
      !ptrs_ok((const void* const*)S, B) || !ptrs_ok((const void* const*)pout, B))
    return PPE_ERR_ARG;
  for (int i = 0; i < B; ++i) {
    if (!(dt[i] > 0) || !std::isfinite(dt[i]) || std::isnan(rho0[i])) return PPE_ERR_ARG;
    if (pout[i] == pn[i] || pout[i] == pnm1[i]) return PPE_ERR_ARG;
  }
  if (hipSetDevice(p->device) != hipSuccess) return PPE_ERR_DEVICE;
  for (int i0 = 0; i0 < B; i0 += kMaxLaunch) {
    const int nb = std::min(kMaxLaunch, B - i0);
    PtrTable tab;
    std::memset(&tab, 0, sizeof(tab));
    for (int i = 0; i < nb; ++i) {
      InstPtrs& q = tab.in[i];
      q.us = us[i0 + i];
      q.vs = vs[i0 + i];
      q.ws = ws[i0 + i];
      q.rho = rho[i0 + i];
      q.pn = pn[i0 + i];
      q.pnm1 = pnm1[i0 + i];
      q.S = S[i0 + i];
      q.p = pout[i0 + i];
      q.info = info + i0 + i;
      q.rho0_in = rho0[i0 + i];
      q.dt = dt[i0 + i];
    }
    ppe_status_t st = (p->d.precision == PPE_PREC_FP64)
                          ? varcoef_typed<double>(p, tab, i0, nb, max_iters, tol, hist)
                          : varcoef_typed<float>(p, tab, i0, nb, max_iters, tol, hist);
    if (st != PPE_OK) return st;
  }
  return PPE_OK;
}

ppe_status_t ppe_correct(ppe_plan_t p, const double* rho0, const double* dt, const double* const* us,
                         const double* const* vs, const double* const* ws, const double* const* rho,
                         const double* const* pn, const double* const* pnm1, const double* const* pin,
                         const double* const* S, double* const* u, double* const* v, double* const* w,
                         ppe_info_t* info) {
  if (!p || !dt || !info) return PPE_ERR_ARG;
  const int B = p->d.batch;
  if (!ptrs_ok((const void* const*)us, B) || !ptrs_ok((const void* const*)vs, B) ||
      !ptrs_ok((const void* const*)ws, B) || !ptrs_ok((const void* const*)rho, B) ||
      !ptrs_ok((const void* const*)pn, B) || !ptrs_ok((const void* const*)pnm1, B) ||
      !ptrs_ok((const void* const*)pin, B) || !ptrs_ok((const void* const*)S, B) ||
      !ptrs_ok((const void* const*)u, B) || !ptrs_ok((const void* const*)v, B) || !ptrs_ok((const void* const*)w, B))
    return PPE_ERR_ARG;
  for (int i = 0; i < B; ++i)
    if (!(dt[i] > 0) || !std::isfinite(dt[i]) || (rho0 && std::isnan(rho0[i]))) return PPE_ERR_ARG;
  if (hipSetDevice(p->device) != hipSuccess) return PPE_ERR_DEVICE;
  const Geom& g = p->g;
  const double tol = p->d.precision == PPE_PREC_MIXED ? p->d.tol : 0.0;
  for (int i0 = 0; i0 < B; i0 += kMaxLaunch) {
    const int nb = std::min(kMaxLaunch, B - i0);
    if (rho0) {
      // the caller's rho0 (Eq. 27): min(rho) where asked, and the
      // compatibility defect mean(D u* - S) into a fresh info record
      PtrTable it;
      std::memset(&it, 0, sizeof(it));
      for (int i = 0; i < nb; ++i) {
        InstPtrs& q = it.in[i];
        q.u = const_cast<double*>(us[i0 + i]);
        q.v = const_cast<double*>(vs[i0 + i]);
        q.w = const_cast<double*>(ws[i0 + i]);
        q.S = S[i0 + i];
        q.rho = rho[i0 + i];
        q.info = info + i0 + i;
        q.rho0_in = rho0[i0 + i];
        q.dt = dt[i0 + i];
      }
      rho_min_pass(p, it, i0, nb);
      const long long blocks = std::min<long long>((g.npts + 255) / 256, kRedBlocks);
      PPE_TIMED(p, "k_div_stats",
                (k_div_stats<<<dim3((unsigned)blocks, 1, nb), 256, 0, p->stream>>>(it, g, p->partial, p->pstride,
                                                                                    nullptr, i0, 0)));
      finish(p, it, i0, nb, (int)blocks, FIN_CORR_INIT, 0);
    }
    PtrTable tab;
    std::memset(&tab, 0, sizeof(tab));
    for (int i = 0; i < nb; ++i) {
      InstPtrs& q = tab.in[i];
      q.us = us[i0 + i];
      q.vs = vs[i0 + i];
      q.ws = ws[i0 + i];
      q.rho = rho[i0 + i];
      q.pn = pn[i0 + i];
      q.pnm1 = pnm1[i0 + i];
      q.S = S[i0 + i];
      q.p = const_cast<double*>(pin[i0 + i]);
      q.u = u[i0 + i];
      q.v = v[i0 + i];
      q.w = w[i0 + i];
      q.info = info + i0 + i;
      q.dt = dt[i0 + i];
    }
    PPE_TIMED(p, "k_correct",
              PPE_MARCH_SWITCH(p->mcor, (k_correct<PPT, NT><<<dim3(p->mcor.grid, 1, nb), NT,
                                                            march_lds(p->mcor, 3), p->stream>>>(
                                               tab, g, p->mcor.m, p->partial, p->pstride, i0))));
    finish(p, tab, i0, nb, p->mcor.grid, FIN_CORRECT, 0, tol);
  }
  return hipGetLastError() == hipSuccess ? PPE_OK : PPE_ERR_DEVICE;
}

ppe_status_t ppe_residual(ppe_plan_t p, const double* const* u, const double* const* v, const double* const* w,
                          const double* const* S, double* out) {
  if (!p || !out) return PPE_ERR_ARG;
  const int B = p->d.batch;
  if (!ptrs_ok((const void* const*)u, B) || !ptrs_ok((const void* const*)v, B) ||
      !ptrs_ok((const void* const*)w, B) || !ptrs_ok((const void* const*)S, B))
    return PPE_ERR_ARG;
  if (hipSetDevice(p->device) != hipSuccess) return PPE_ERR_DEVICE;
  const Geom& g = p->g;
  for (int i0 = 0; i0 < B; i0 += kMaxLaunch) {
    const int nb = std::min(kMaxLaunch, B - i0);
    PtrTable tab;
    std::memset(&tab, 0, sizeof(tab));
    for (int i = 0; i < nb; ++i) {
      InstPtrs& q = tab.in[i];
      q.u = const_cast<double*>(u[i0 + i]);
      q.v = const_cast<double*>(v[i0 + i]);
      q.w = const_cast<double*>(w[i0 + i]);
      q.S = S[i0 + i];
    }
    const long long blocks = std::min<long long>((g.npts + 255) / 256, kRedBlocks);
    for (int pass = 0; pass < 2; ++pass) {
      PPE_TIMED(p, "k_div_stats",
                (k_div_stats<<<dim3((unsigned)blocks, 1, nb), 256, 0, p->stream>>>(tab, g, p->partial, p->pstride,
                                                                                    out + 3 * (size_t)i0, i0, pass)));
      finish(p, tab, i0, nb, (int)blocks, pass == 0 ? FIN_DIV0 : FIN_DIV1, 0, 0.0, out + 3 * (size_t)i0);
    }
  }
  return hipGetLastError() == hipSuccess ? PPE_OK : PPE_ERR_DEVICE;
}

ppe_status_t ppe_source(ppe_plan_t p, const ppe_source_t* src, double* const* S) {
  if (!p || !src || !S) return PPE_ERR_ARG;
  const int B = p->d.batch;
  for (int i = 0; i < B; ++i) {
    const ppe_source_t& q = src[i];
    if (!q.C || !q.div_g || !q.div_l || !q.mdot || !q.area || !q.rho_g || !q.rho_l || !S[i]) return PPE_ERR_ARG;
  }
  if (hipSetDevice(p->device) != hipSuccess) return PPE_ERR_DEVICE;
  const long long n = p->g.npts;
  // paired 16-byte accesses when every array of the call is 16-byte aligned
  bool aligned = true;
  auto al = [&](const void* q) { aligned = aligned && (reinterpret_cast<uintptr_t>(q) & 15) == 0; };
  for (int i = 0; i < B; ++i) {
    const ppe_source_t& q = src[i];
    al(q.C), al(q.div_g), al(q.div_l), al(q.mdot), al(q.area), al(q.rho_g), al(q.rho_l), al(S[i]);
  }
  const int vec = (aligned && p->src_vec == 2) ? 2 : 1;
  const int pt = p->src_pt;
  const long long units = vec == 2 ? std::max(1LL, n >> 1) : n;
  const long long per_block = (long long)pt * kSrcThreads;
  const unsigned blocks = (unsigned)((units + per_block - 1) / per_block);
  for (int i0 = 0; i0 < B; i0 += kMaxLaunch) {
    const int nb = std::min(kMaxLaunch, B - i0);
    SrcTable tab;
    std::memset(&tab, 0, sizeof(tab));
    for (int i = 0; i < nb; ++i) {
      const ppe_source_t& q = src[i0 + i];
      SrcPtrs& t = tab.in[i];
      t.C = q.C;
      t.div_g = q.div_g;
      t.div_l = q.div_l;
      t.mdot = q.mdot;
      t.area = q.area;
      t.rho_g = q.rho_g;
      t.rho_l = q.rho_l;
      t.under = q.under;
      t.S = S[i0 + i];
    }
#define PPE_SRC_LAUNCH(PTV, VV) \
  (k_source<PTV, VV><<<dim3(blocks, 1, nb), kSrcThreads, 0, p->stream>>>(tab, n))
    if (vec == 2) {
      if (pt == 2) PPE_TIMED(p, "k_source", PPE_SRC_LAUNCH(2, 2));
      else if (pt == 4) PPE_TIMED(p, "k_source", PPE_SRC_LAUNCH(4, 2));
      else PPE_TIMED(p, "k_source", PPE_SRC_LAUNCH(8, 2));
    } else {
      if (pt == 2) PPE_TIMED(p, "k_source", PPE_SRC_LAUNCH(2, 1));
      else if (pt == 4) PPE_TIMED(p, "k_source", PPE_SRC_LAUNCH(4, 1));
      else PPE_TIMED(p, "k_source", PPE_SRC_LAUNCH(8, 1));
    }
#undef PPE_SRC_LAUNCH
  }
  return hipGetLastError() == hipSuccess ? PPE_OK : PPE_ERR_DEVICE;
}

// ---------------------------------------------------------------------------
// Pressure ring for time loops
// ---------------------------------------------------------------------------
struct ppe_ring_s {
  ppe_plan_t plan = nullptr;
  double* buf[3] = {nullptr, nullptr, nullptr};  // each batch * npts doubles
  int cur = 0, prev = 1;                          // slots of p^n and p^{n-1}
  int64_t steps = 0;
};

ppe_status_t ppe_ring_create(ppe_plan_t p, const double* const* pn, const double* const* pnm1, ppe_ring_t* out) {
  if (!out) return PPE_ERR_ARG;
  *out = nullptr;
  if (!p || !ptrs_ok((const void* const*)pn, p->d.batch)) return PPE_ERR_ARG;
  if (pnm1 && !ptrs_ok((const void* const*)pnm1, p->d.batch)) return PPE_ERR_ARG;
  if (hipSetDevice(p->device) != hipSuccess) return PPE_ERR_DEVICE;
  ppe_ring_s* r = new (std::nothrow) ppe_ring_s();
  if (!r) return PPE_ERR_NOMEM;
  r->plan = p;
  const size_t n = (size_t)p->g.npts;
  const size_t bytes = (size_t)p->d.batch * n * sizeof(double);
  for (int s = 0; s < 3; ++s) {
    if (hipMalloc((void**)&r->buf[s], bytes) != hipSuccess) {
      for (int q = 0; q < s; ++q) (void)hipFree(r->buf[q]);
      delete r;
      return PPE_ERR_NOMEM;
    }
  }
  bool ok = true;
  for (int i = 0; i < p->d.batch; ++i) {
    ok &= hipMemcpyAsync(r->buf[r->cur] + i * n, pn[i], n * sizeof(double), hipMemcpyDeviceToDevice, p->stream) ==
          hipSuccess;
    ok &= hipMemcpyAsync(r->buf[r->prev] + i * n, pnm1 ? pnm1[i] : pn[i], n * sizeof(double),
                         hipMemcpyDeviceToDevice, p->stream) == hipSuccess;
  }
  if (!ok) {
    (void)hipStreamSynchronize(p->stream);
    for (int s = 0; s < 3; ++s) (void)hipFree(r->buf[s]);
    delete r;
    return PPE_ERR_DEVICE;
  }
  *out = r;
  return PPE_OK;
}

ppe_status_t ppe_ring_step(ppe_ring_t r, const double* rho0, const double* dt, const double* const* us,
                           const double* const* vs, const double* const* ws, const double* const* rho,
                           const double* const* S, double* const* u, double* const* v, double* const* w,
                           ppe_info_t* info, double* split_defect) {
  if (!r) return PPE_ERR_ARG;
  ppe_plan_t p = r->plan;
  const int B = p->d.batch;
  if (B > PPE_MAX_BATCH) return PPE_ERR_ARG;
  const int next = 3 - r->cur - r->prev;
  const size_t n = (size_t)p->g.npts;
  const double* pn[PPE_MAX_BATCH];
  const double* pm[PPE_MAX_BATCH];
  double* pp[PPE_MAX_BATCH];
  for (int i = 0; i < B; ++i) {
    pn[i] = r->buf[r->cur] + i * n;
    pm[i] = r->buf[r->prev] + i * n;
    pp[i] = r->buf[next] + i * n;
  }
  if (split_defect && (!p->r64 || p->r64_elem != 8)) return PPE_ERR_ARG;  // needs PPE_FLAG_VARCOEF
  ppe_status_t st = ppe_solve(p, rho0, dt, us, vs, ws, rho, pn, pm, S, pp, info);
  if (st != PPE_OK) return st;
  if (split_defect) {
    for (int i0 = 0; i0 < B; i0 += kMaxLaunch) {
      const int nb = std::min(kMaxLaunch, B - i0);
      PtrTable tab;
      std::memset(&tab, 0, sizeof(tab));
      for (int i = 0; i < nb; ++i) {
        InstPtrs& q = tab.in[i];
        q.us = us[i0 + i];
        q.vs = vs[i0 + i];
        q.ws = ws[i0 + i];
        q.rho = rho[i0 + i];
        q.pn = pn[i0 + i];
        q.pnm1 = pm[i0 + i];
        q.S = S[i0 + i];
        q.p = pp[i0 + i];
        q.info = info + i0 + i;
        q.rho0_in = rho0[i0 + i];
        q.dt = dt[i0 + i];
      }
      st = p->d.precision == PPE_PREC_FP64 ? defect_typed<double>(p, tab, i0, nb, split_defect)
                                           : defect_typed<float>(p, tab, i0, nb, split_defect);
      if (st != PPE_OK) return st;
    }
  }
  st = ppe_correct(p, nullptr, dt, us, vs, ws, rho, pn, pm, pp, S, u, v, w, info);
  if (st != PPE_OK) return st;
  r->prev = r->cur;
  r->cur = next;
  ++r->steps;
  return PPE_OK;
}

ppe_status_t ppe_ring_pressure(ppe_ring_t r, int32_t lag, double** out) {
  if (!r || !out || (lag != 0 && lag != 1)) return PPE_ERR_ARG;
  const size_t n = (size_t)r->plan->g.npts;
  const int s = lag == 0 ? r->cur : r->prev;
  for (int i = 0; i < r->plan->d.batch; ++i) out[i] = r->buf[s] + i * n;
  return PPE_OK;
}

ppe_status_t ppe_ring_read(ppe_ring_t r, int32_t lag, double* const* out) {
  if (!r || (lag != 0 && lag != 1) || !ptrs_ok((const void* const*)out, r->plan->d.batch)) return PPE_ERR_ARG;
  ppe_plan_t p = r->plan;
  if (hipSetDevice(p->device) != hipSuccess) return PPE_ERR_DEVICE;
  const size_t n = (size_t)p->g.npts;
  const int s = lag == 0 ? r->cur : r->prev;
  for (int i = 0; i < p->d.batch; ++i)
    if (hipMemcpyAsync(out[i], r->buf[s] + i * n, n * sizeof(double), hipMemcpyDeviceToDevice, p->stream) !=
        hipSuccess)
      return PPE_ERR_DEVICE;
  return PPE_OK;
}

int64_t ppe_ring_steps(ppe_ring_t r) { return r ? r->steps : -1; }

ppe_status_t ppe_ring_destroy(ppe_ring_t r) {
  if (!r) return PPE_ERR_ARG;
  (void)hipSetDevice(r->plan->device);
  (void)hipStreamSynchronize(r->plan->stream);
  for (int s = 0; s < 3; ++s) (void)hipFree(r->buf[s]);
  delete r;
  return PPE_OK;
}

ppe_status_t ppe_predict(ppe_plan_t p, const ppe_predict_t* in, double* const* up, double* const* vp,
                         double* const* wp) {
  if (!p || !in || !up || !vp || !wp) return PPE_ERR_ARG;
  if (p->d.ny < 4) return PPE_ERR_UNSUPPORTED;
  const int B = p->d.batch;
  for (int i = 0; i < B; ++i) {
    const ppe_predict_t& q = in[i];
    if (!q.u || !q.v || !q.w || !q.rho_n || !q.rho_np1 || !q.mu || !q.C || !q.sigma || !q.kappa || !up[i] ||
        !vp[i] || !wp[i])
      return PPE_ERR_ARG;
    if (!(q.dt > 0) || !std::isfinite(q.dt) || !(q.rho_mean > 0) || !std::isfinite(q.rho_mean)) return PPE_ERR_ARG;
  }
  if (hipSetDevice(p->device) != hipSuccess) return PPE_ERR_DEVICE;
  const Geom& g = p->g;
  const unsigned blocks = (unsigned)((g.npts + 255) / 256);
  // LDS tiles need whole 64-column x tiles; PPE_TUNE_PREDICT_GLOBAL=1 keeps
  // the one-thread-per-face kernels (the same arithmetic on the same values)
  const bool tiled = tune_env("PPE_TUNE_PREDICT_GLOBAL") == 0 && g.nx % kPredTX == 0;
  for (int i0 = 0; i0 < B; i0 += kMaxLaunch) {
    const int nb = std::min(kMaxLaunch, B - i0);
    PredTable tab;
    std::memset(&tab, 0, sizeof(tab));
    for (int i = 0; i < nb; ++i) {
      const ppe_predict_t& q = in[i0 + i];
      PredPtrs& t = tab.in[i];
      t.u = q.u;
      t.v = q.v;
      t.w = q.w;
      t.uv = q.uv ? q.uv : q.u;
      t.vv = q.vv ? q.vv : q.v;
      t.wv = q.wv ? q.wv : q.w;
      t.rn = q.rho_n;
      t.r1 = q.rho_np1;
      t.mu = q.mu;
      t.C = q.C;
      t.sg = q.sigma;
      t.kp = q.kappa;
      t.fsx = q.fsx;
      t.fsy = q.fsy;
      t.fsz = q.fsz;
      t.up = up[i0 + i];
      t.vp = vp[i0 + i];
      t.wp = wp[i0 + i];
      t.rho_mean = q.rho_mean;
      t.dt = q.dt;
    }
    // the viscous-term velocity is the advected one in every instance
    bool alias = true;
    for (int i = 0; i < nb; ++i) {
      const PredPtrs& t = tab.in[i];
      alias = alias && t.uv == t.u && t.vv == t.v && t.wv == t.w;
    }
    if (tiled && alias && tune_env("PPE_TUNE_PREDICT_NO_MARCH") == 0) {
      const auto run_of = [](const char* env, int def) {
        const int v = tune_env(env) > 0 ? tune_env(env) : tune_env("PPE_TUNE_PREDICT_RUN");
        return v > 0 ? v : def;
      };
      // slabs per block: at 256x128x256 the y marches (u, w) ran fastest with
      // 12 (u/w 281/247 us at 16, 270/239 at 12, 275-287/244-257 at 8-14), the
      // z march (v) with 16 or 32 (293; 315-351 at 20-24)
      const int run_u = run_of("PPE_TUNE_PREDICT_RUN_U", 12), run_v = run_of("PPE_TUNE_PREDICT_RUN_V", 16),
                run_w = run_of("PPE_TUNE_PREDICT_RUN_W", 12);
      const unsigned ntx = (unsigned)(g.nx / kPredTX);
      const unsigned ty = ntx * (unsigned)((g.ny + kPredTR - 1) / kPredTR);
      const unsigned tz = ntx * (unsigned)((g.nz + kPredTR - 1) / kPredTR);
      const auto gy = [&](int run) { return dim3(ty * (unsigned)((g.nz + run - 1) / run), 1, nb); };
      const auto gz = [&](int run) { return dim3(tz * (unsigned)((g.ny + run - 1) / run), 1, nb); };
      constexpr int nt = kPredTX * kPredTR;
      if (tune_env("PPE_TUNE_PREDICT_U_PLANES") == 0 && tune_env("PPE_TUNE_PREDICT_SEPARATE") == 0) {
        // the three components in one launch (u and w through y rows, v
        // through z planes), each block range starting on a multiple of 8
        const unsigned nu = gz(run_u).x, nv = gy(run_v).x, nw = gz(run_w).x;
        const unsigned nblk = ((nu + 7u) & ~7u) + ((nv + 7u) & ~7u) + nw;
        PPE_TIMED(p, "k_predict", {
          k_predict_march_uvw<<<dim3(nblk, 1, nb), nt, 0, p->stream>>>(tab, g, run_u, run_v, run_w, nu, nv, nw);
          if (g.ybc == 1) {  // the outflow top face of v
            const unsigned tblocks = (unsigned)(((long long)g.nx * g.nz + 255) / 256);
            k_predict_vtop<<<dim3(tblocks, 1, nb), 256, 0, p->stream>>>(tab, g);
          }
        });
        continue;
      }
      // u marches through y rows like w (faster than through z planes)
      if (tune_env("PPE_TUNE_PREDICT_U_PLANES") != 0) {
        PPE_TIMED(p, "k_predict_u", (k_predict_march<0><<<gy(run_u), nt, 0, p->stream>>>(tab, g, run_u)));
      } else {
        PPE_TIMED(p, "k_predict_u", (k_predict_march<3><<<gz(run_u), nt, 0, p->stream>>>(tab, g, run_u)));
      }
      PPE_TIMED(p, "k_predict_v", {
        k_predict_march<1><<<gy(run_v), nt, 0, p->stream>>>(tab, g, run_v);
        if (g.ybc == 1) {  // the outflow top face
          const unsigned tblocks = (unsigned)(((long long)g.nx * g.nz + 255) / 256);
          k_predict_vtop<<<dim3(tblocks, 1, nb), 256, 0, p->stream>>>(tab, g);
        }
      });
      PPE_TIMED(p, "k_predict_w", (k_predict_march<2><<<gz(run_w), nt, 0, p->stream>>>(tab, g, run_w)));
      continue;
    }
    if (tiled) {
      const unsigned ntx = (unsigned)(g.nx / kPredTX);
      const dim3 gy(ntx * (unsigned)((g.ny + kPredTR - 1) / kPredTR), (unsigned)g.nz, nb);
      const dim3 gz(ntx * (unsigned)((g.nz + kPredTR - 1) / kPredTR), (unsigned)g.ny, nb);
      constexpr int nt = kPredTX * kPredTR;
      PPE_TIMED(p, "k_predict_u", {
        if (alias) k_predict_tile<0, true><<<gy, nt, 0, p->stream>>>(tab, g);
        else k_predict_tile<0, false><<<gy, nt, 0, p->stream>>>(tab, g);
      });
      PPE_TIMED(p, "k_predict_v", {
        if (alias) k_predict_tile<1, true><<<gy, nt, 0, p->stream>>>(tab, g);
        else k_predict_tile<1, false><<<gy, nt, 0, p->stream>>>(tab, g);
        if (g.ybc == 1) {  // the outflow top face
          const unsigned tblocks = (unsigned)(((long long)g.nx * g.nz + 255) / 256);
          k_predict_vtop<<<dim3(tblocks, 1, nb), 256, 0, p->stream>>>(tab, g);
        }
      });
      PPE_TIMED(p, "k_predict_w", {
        if (alias) k_predict_tile<2, true><<<gz, nt, 0, p->stream>>>(tab, g);
        else k_predict_tile<2, false><<<gz, nt, 0, p->stream>>>(tab, g);
      });
      continue;
    }
    PPE_TIMED(p, "k_predict_u", (k_predict<0><<<dim3(blocks, 1, nb), 256, 0, p->stream>>>(tab, g)));
    PPE_TIMED(p, "k_predict_v", {
      k_predict<1><<<dim3(blocks, 1, nb), 256, 0, p->stream>>>(tab, g);
      if (g.ybc == 1) {  // the outflow top face
        const unsigned tblocks = (unsigned)(((long long)g.nx * g.nz + 255) / 256);
        k_predict_vtop<<<dim3(tblocks, 1, nb), 256, 0, p->stream>>>(tab, g);
      }
    });
    PPE_TIMED(p, "k_predict_w", (k_predict<2><<<dim3(blocks, 1, nb), 256, 0, p->stream>>>(tab, g)));
  }
  return hipGetLastError() == hipSuccess ? PPE_OK : PPE_ERR_DEVICE;
}

ppe_status_t ppe_solve_noalloc(const ppe_desc_t* desc, void* stream, const double* rho0, const double* dt,
                               const double* const* us, const double* const* vs, const double* const* ws,
                               const double* const* rho, const double* const* pn, const double* const* pnm1,
                               const double* const* S, double* const* p, double* const* u, double* const* v,
                               double* const* w, ppe_info_t* info) {
  if (!desc_ok(desc)) return PPE_ERR_ARG;
  if (!u != !v || !u != !w) return PPE_ERR_ARG;
  // every host-checkable argument before anything is enqueued
  {
    const int nb = desc->batch;
    if (!rho0 || !dt || !info) return PPE_ERR_ARG;
    if (!ptrs_ok((const void* const*)us, nb) || !ptrs_ok((const void* const*)vs, nb) ||
        !ptrs_ok((const void* const*)ws, nb) || !ptrs_ok((const void* const*)rho, nb) ||
        !ptrs_ok((const void* const*)pn, nb) || !ptrs_ok((const void* const*)pnm1, nb) ||
        !ptrs_ok((const void* const*)S, nb) || !ptrs_ok((const void* const*)p, nb))
      return PPE_ERR_ARG;
    if (u && (!ptrs_ok((const void* const*)u, nb) || !ptrs_ok((const void* const*)v, nb) ||
              !ptrs_ok((const void* const*)w, nb)))
      return PPE_ERR_ARG;
    for (int i = 0; i < nb; ++i)
      if (!(dt[i] > 0) || !std::isfinite(dt[i]) || std::isnan(rho0[i])) return PPE_ERR_ARG;
  }
  // the refined y solve needs a block list built on the host, and the
  // fixed-point buffer is for ppe_solve_varcoef: neither is offered here
  if (desc->ny > 256 || (desc->flags & (PPE_FLAG_Y_REFINE | PPE_FLAG_VARCOEF)) != 0) return PPE_ERR_UNSUPPORTED;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PPE_ERR_DEVICE;
  ppe_plan_s P;  // (a plan on the stack: no allocation; its pointers go into `scratch`)
  P.d = *desc;
  P.stream = reinterpret_cast<hipStream_t>(stream);
  P.device = dev;
  int lds_max = 65536;
  if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return PPE_ERR_DEVICE;
  if (!shape_plan(&P, (size_t)std::max(lds_max, 65536))) return PPE_ERR_UNSUPPORTED;
  const ppe_desc_t& d = P.d;
  const size_t B = (size_t)d.batch;
  const auto al = [](size_t n) { return (n + 255) & ~size_t(255); };
  const size_t sz[] = {B * (size_t)P.g.spec_elems * spec_elem_bytes(&d),  // spectrum
                       B * (size_t)P.g.npts * 8,                         // b64
                       B * (size_t)P.g.npts * r64_elem_bytes(d),         // refinement residual
                       B * (size_t)d.ny * d.nz * 8,                      // row sums
                       B * (size_t)d.ny * 8,                             // plane sums
                       B * (size_t)kNScal * 8,                           // scalars
                       B * (size_t)P.pstride * 8,                        // partials
                       (size_t)P.g.hx * 8, (size_t)d.nz * 8,            // lam_x, lam_z
                       (size_t)2 * d.nx * 8, (size_t)2 * d.nz * 8};      // twiddles
  size_t need = 0;
  for (size_t x : sz) need += al(std::max<size_t>(x, 8));
  if (need > kScratchBytes) return PPE_ERR_NOMEM;  // larger than the static workspace
  char* base = static_cast<char*>(scratch_on(dev));
  if (!base) return PPE_ERR_DEVICE;
  constexpr int kParts = 11;
  static_assert(sizeof(sz) / sizeof(sz[0]) == kParts, "workspace parts");
  void* parts[kParts];
  size_t off = 0;
  for (int i = 0; i < kParts; ++i) {
    parts[i] = base + off;
    off += al(std::max<size_t>(sz[i], 8));
  }
  P.spec = parts[0];
  P.b64 = static_cast<double*>(parts[1]);
  P.r64_elem = r64_elem_bytes(d);
  P.r64 = P.r64_elem > 0 ? static_cast<double*>(parts[2]) : nullptr;
  P.rowsum = static_cast<double*>(parts[3]);
  P.colsum = static_cast<double*>(parts[4]);
  P.scal = static_cast<double*>(parts[5]);
  P.partial = static_cast<double*>(parts[6]);
  P.lamx = static_cast<double*>(parts[7]);
  P.lamz = static_cast<double*>(parts[8]);
  P.fx.tw = static_cast<double*>(parts[9]);
  P.fz.tw = static_cast<double*>(parts[10]);
  if (hipSetDevice(dev) != hipSuccess) return PPE_ERR_DEVICE;
  // tables for this shape, and the per-instance scalars cleared (the array
  // keeps whatever the previous call on this GPU left)
  const int nt = std::max(std::max(d.nx, d.nz), P.g.hx);
  k_tables<<<(nt + 255) / 256, 256, 0, P.stream>>>(P.fx.tw, d.nx, P.fz.tw, d.nz, P.lamx, P.g.hx, P.lamz, P.g.dx,
                                                   P.g.dz);
  const long long nsc = (long long)B * kNScal;
  k_fill<<<(unsigned)((nsc + 255) / 256), 256, 0, P.stream>>>(P.scal, nsc, 0.0);
  if (hipGetLastError() != hipSuccess) return PPE_ERR_DEVICE;
  ppe_status_t st = ppe_solve(&P, rho0, dt, us, vs, ws, rho, pn, pnm1, S, p, info);
  if (st != PPE_OK || !u) return st;
  return ppe_correct(&P, nullptr, dt, us, vs, ws, rho, pn, pnm1, p, S, u, v, w, info);
}

ppe_status_t ppe_plan_profile(ppe_plan_t p, int32_t enable) {
  if (!p) return PPE_ERR_ARG;
  if (enable) {
    prof_collect(p);
    p->acc.clear();
  }
  p->prof = enable != 0;
  return PPE_OK;
}

ppe_status_t ppe_plan_profile_read(ppe_plan_t p, ppe_kernel_time_t* out, int32_t cap, int32_t* count) {
  if (!p || !count || cap < 0 || (cap > 0 && !out)) return PPE_ERR_ARG;
  prof_collect(p);
  int n = 0;
  for (const auto& kv : p->acc) {
    if (n < cap) {
      std::memset(out[n].name, 0, sizeof(out[n].name));
      std::strncpy(out[n].name, kv.first.c_str(), sizeof(out[n].name) - 1);
      out[n].launches = (int32_t)kv.second.first;
      out[n].total_ms = kv.second.second;
    }
    ++n;
  }
  *count = n;
  return PPE_OK;
}

const char* ppe_version(void) { return "ppe-mi355x 0.1 (gfx950)"; }

}  // extern "C"
