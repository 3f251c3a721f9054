// ppe_kernels.hpp -- HIP kernels of the split pressure-gradient projection
// (Poblador-Ibanez & Sirignano, arXiv 2103.01874, Sec. 5.4).
//
// Pass structure of one solve (every pass is one launch over all instances
// of a batch; blockIdx.z is the instance):
//   k_rhs        b = (rho0/dt)(D u* - S) + D(beta_f G p_hat)  (Eq. 29), a
//                z-marching stencil; writes b and the block sums of D u* - S
//   k_r2c        real FFT along x of b (two rows packed per complex FFT) into
//                the half spectrum, with the FP64 row sums (zero mode)
//   k_fft_z      complex FFT along z, in place on the half spectrum
//   k_tri        one tridiagonal system in y per (kx, kz), partition method;
//                the (0,0) system is solved in FP64 from FP64 plane sums
//                (with zero-flux ends it is singular: compatible-projected,
//                pinned and gauge-fixed)
//   k_fft_z      inverse
//   k_c2r        inverse real FFT along x -> p (or p update when refining)
//   k_resid      FP64 r = b - L p, stored in the spectrum's precision
//                (refinement), then k_r2c .. k_c2r again on r
//   k_correct    u^{n+1} = u* - dt[G p/rho0 + gamma_f G p_hat]  (Eq. 28) and
//                the continuity residual of the result
// and, before a solve when the caller assembles S through the library:
//   k_source     S = (1-C) div_g + C div_l + m' (A/V0)(1/rho_g - 1/rho_l)  (Eq. 26)
// and, producing u* itself:
//   k_predict    the predictor u^p of Eq. (23)
#pragma once

#include "ppe_device.hpp"

namespace ppe {

constexpr int kMaxLaunch = 16;     // instances per launch (kernel-argument table)
constexpr int kNScal = 16;         // per-instance scalar slots
constexpr int kRedBlocks = 2048;   // grid cap of the grid-stride reduction kernels

enum ScalarSlot {
  SC_RHO0 = 0,    // rho0 used
  SC_DT,          // dt
  SC_COMPAT,      // mean(D u* - S) (0 with an outflow top)
  SC_REF2,        // ||(rho0/dt)(D u* - S_c)||^2  (refinement stop scale)
  SC_BMEAN,       // mean(b) (0 with an outflow top: nothing is removed)
  SC_PMEAN,       // mean of the current p (refinement gauge; 0 with an outflow top)
  SC_CONV,        // 1 once the refinement met tol
  SC_RES,         // last relative residual
  SC_ITERS,       // refinement sweeps run
  SC_RHO0_BITS,   // min(rho) accumulator (uint64 bits of a positive double)
  SC_TOL,         // tol
};

struct InstPtrs {
  const double* us;
  const double* vs;
  const double* ws;
  const double* rho;
  const double* pn;
  const double* pnm1;
  const double* S;
  double* p;
  double* u;
  double* v;
  double* w;
  void* info;     // ppe_info_t*
  double rho0_in;
  double dt;
};

struct PtrTable {
  InstPtrs in[kMaxLaunch];
};

struct Geom {
  int nx, ny, nz, hx;
  int ybc;              // 0: zero-flux faces at both y ends; 1: outflow top (p = 0 on the face)
  int tws;              // log2 of the spectrum tile width (128-byte tiles of kx)
  long long npts;       // nx*ny*nz
  long long spec_elems; // ntiles * nz * ny * tile width (>= hx * ny * nz)
  double dx, dy, dz;    // cell sizes
  double idx, idy, idz; // 1/dx, 1/dy, 1/dz
  double dy2;           // dy^2
  double inv_nxnz;      // 1/(nx*nz)
};

// Half-spectrum layout: tiles of 2^tws consecutive kx (128 bytes) hold, for
// every (kz, j), their values contiguously:
//   [tile][kz][j][kx mod 2^tws]
// so a y system of one tile is one contiguous run and a z column strides
// ny * 2^tws values.  `row` = kz * ny + j.
__host__ __device__ __forceinline__ long long sidx(const Geom& g, int kx, long long row) {
  const long long t = kx >> g.tws;
  return ((t * g.nz * g.ny + row) << g.tws) + (kx & ((1 << g.tws) - 1));
}

// The tile shift of a spectrum of TS values, as a constant (g.tws at run time).
template <typename TS>
constexpr int kTileShift = sizeof(TS) == 8 ? 3 : 4;

template <typename TS>
__host__ __device__ __forceinline__ long long sidx_t(const Geom& g, int kx, long long row) {
  constexpr int sh = kTileShift<TS>;
  const long long t = kx >> sh;
  return ((t * g.nz * g.ny + row) << sh) + (kx & ((1 << sh) - 1));
}

// Workspace seen by the kernels (device pointers, per-instance strides).
template <typename TS>
struct Work {
  cplx<TS>* spec;       // [inst][nz][ny][hx]
  double* b64;          // [inst][npts]        (refinement only)
  double* rowsum;       // [inst][nz][ny]      FP64 row sums of the transformed field
  double* colsum;       // [inst][ny]          FP64 plane sums (zero mode)
  double* scal;         // [inst][kNScal]
  double* partial;      // [inst][pstride] per-block partial sums
  long long pstride;    // doubles of partials per instance
  const double* lamx;   // [hx]  lam_x(kx)
  const double* lamz;   // [nz]  lam_z(kz)
  int inst0;            // first instance of this launch in the workspace
  int nt_rows;          // row transforms store with the non-temporal hint
};

// Inputs and output of the target-divergence pass (Eq. 26) for one instance.
struct SrcPtrs {
  const double* C;
  const double* div_g;
  const double* div_l;
  const double* mdot;
  const double* area;
  const double* rho_g;
  const double* rho_l;
  const uint8_t* under;   // may be null
  double* S;
};

struct SrcTable {
  SrcPtrs in[kMaxLaunch];
};

// ppe_info_t as laid out in include/ppe.h
struct InfoRec {
  int32_t status;
  int32_t iters;
  double rho0_used;
  double compat_defect;
  double res_rel;
  double div_l2;
  double div_max;
  double div0_l2;
  double p_mean;
};

}  // namespace ppe
