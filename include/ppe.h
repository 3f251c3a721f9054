/*
 * ppe.h -- C ABI of the MI355X split pressure-gradient projection library.
 *
 * The library computes one projection step of the low-Mach two-phase scheme
 * of Poblador-Ibanez & Sirignano (arXiv 2103.01874), Sec. 5.4:
 *
 *   p_hat = 2 p^n - p^{n-1},  rho0 = min(rho)                          (Eq. 27)
 *   lap p = div[(1 - rho0/rho) grad p_hat] + (rho0/dt)(div u* - S)     (Eq. 29)
 *   u^{n+1} = u* - dt [ grad p/rho0 + (1/rho - 1/rho0) grad p_hat ]    (Eq. 28)
 *
 * where u* is the predictor velocity (the paper's u^p, Eq. 23) and S the
 * target divergence div u^{n+1} (Eq. 26).  The Poisson equation is solved
 * directly (Sec. 5.4: a fast solver built from discrete Fourier transforms):
 * real FFT in x, complex FFT in z, one tridiagonal system in y per wavenumber
 * pair, inverse FFTs.  Every step runs in HIP kernels on one GPU.
 *
 * Grid and layouts (all fields are C-order float64, x fastest):
 *   nx*ny*nz cells of size dx = lx/nx, dy = ly/ny, dz = lz/nz; x and z are
 *   periodic; the y ends are chosen by ppe_desc_t.ybc (ppe_ybc_t).
 *   cell fields rho, p^n, p^{n-1}, S, p : [nz][ny][nx]
 *   u (west face of cell i)             : [nz][ny][nx]
 *   v (south face of cell j)            : [nz][ny+1][nx]; row 0 is a wall or
 *                                         symmetry plane (read as given, never
 *                                         corrected, zero pressure flux); row
 *                                         ny is a wall likewise (PPE_YBC_WALLS)
 *                                         or an outflow face (PPE_YBC_OUTFLOW)
 *   w (back face of cell k)             : [nz][ny][nx]
 *   D = cell divergence, G = face gradient (zero on walls), L = D o G.
 *   Face density rho_f = (rho_a + rho_b)/2, the same in the right-hand side
 *   and in the projection, so div u^{n+1} = S_c to rounding.
 *   PPE_YBC_WALLS: L is singular; S_c = S + mean(D u* - S), mean(b) is
 *   removed from the right-hand side (compatibility) and the pressure is
 *   fixed by mean(p) = 0.
 *   PPE_YBC_OUTFLOW (the planar jets of Sec. 6, computed over their symmetry
 *   plane): p = 0 on the top face, imposed by the ghost value -p_{ny-1}; the
 *   top face's density is rho_{ny-1}; the top v face is corrected like an
 *   interior face.  L is regular: S_c = S, nothing is removed, no gauge.
 *
 * Ownership: every field pointer is a DEVICE pointer owned by the caller;
 * the plan owns its workspace, twiddle and eigenvalue tables (allocated in
 * ppe_plan, freed in ppe_plan_destroy).  Outputs must not alias inputs.
 *
 * Streams: every call enqueues work on the plan's stream and returns without
 * waiting for the device.  Results (fields and ppe_info_t records) are valid
 * once the stream has been synchronised.
 *
 * Errors: problems the host can see (null pointer, bad size, unsupported
 * FFT length, non-positive dt) return a negative ppe_status_t and enqueue
 * nothing.  Problems only the device can see (non-finite data, refinement
 * not converged) are written to the instance's ppe_info_t.status; other
 * instances of a batch are not affected.
 *
 * Thread safety: a plan must not be used from two host threads at once.
 * Distinct plans (on distinct streams) may run concurrently.
 */
#ifndef PPE_H
#define PPE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ppe_plan_s* ppe_plan_t;

typedef enum {
  PPE_OK = 0,
  PPE_ERR_ARG = -1,          /* bad argument (null pointer, size, dt <= 0, ...) */
  PPE_ERR_NOMEM = -2,        /* device allocation failed */
  PPE_ERR_DEVICE = -3,       /* a HIP call failed */
  PPE_ERR_NOT_CONVERGED = -4,/* (info only) refinement stopped above tol */
  PPE_ERR_NONFINITE = -5,    /* (info only) a non-finite value reached the solve */
  PPE_ERR_UNSUPPORTED = -6   /* FFT length not of the form 2^a 3^b, or too long */
} ppe_status_t;

/* Boundaries at the two ends of y (x and z are always periodic). */
typedef enum {
  PPE_YBC_WALLS = 0,   /* zero pressure flux through both end faces */
  PPE_YBC_OUTFLOW = 1  /* zero flux through the bottom face (wall or symmetry
                          plane), p = 0 on the top face (outflow) */
} ppe_ybc_t;

/* Plan options (ppe_desc_t.flags). */
#define PPE_FLAG_VARCOEF 1   /* also allocate the FP64 residual buffer that
                                ppe_solve_varcoef and the ring's split defect
                                need: 8 bytes per cell and instance, for either
                                precision (a PPE_PREC_MIXED plan otherwise
                                holds 4 bytes per cell for the FP32 residual of
                                its refinement, which those calls cannot use) */
#define PPE_FLAG_Y_REFINE 2  /* follow every y tridiagonal solve of a system
                                whose smallest eigenvalue is below about 1e-2
                                (s + the lowest y mode, Sec. 5.4 scaling) by
                                one correction solve of its residual, formed in
                                difference form: restores ~1e-15 on systems the
                                elimination alone leaves at ~4 eps / (that
                                eigenvalue).  Always on for ny > 256; the flag
                                asks for it at any ny (wide domains with smooth
                                sources: s = (dy k)^2 falls below 1e-5 when the
                                horizontal extent exceeds ~2000 dy).  Costs a
                                second tridiagonal launch over those systems. */

/* Precision of the spectral passes (FFTs and tridiagonal sweeps). */
typedef enum {
  PPE_PREC_FP64 = 0,   /* FP64 storage and arithmetic: the direct solve */
  PPE_PREC_MIXED = 1   /* FP32 spectra in memory, FP64 arithmetic in registers;
                          the residual is formed and its norm taken in FP64
                          (stored in FP32 for the correction solve), and the
                          zero mode, gauge and update of p are FP64 */
} ppe_precision_t;

typedef struct {
  int32_t nx, ny, nz;      /* cells; nx, nz in 1..2048 of the form 2^a 3^b; 2 <= ny <= 2048 */
  double lx, ly, lz;       /* domain lengths (> 0) */
  int32_t precision;       /* ppe_precision_t */
  int32_t ybc;             /* ppe_ybc_t */
  double tol;              /* PPE_PREC_MIXED: stop when the relative residual
                              ||b - mean b - L p||_2 / ||(rho0/dt)(D u* - S_c)||_2
                              <= tol (the projected field's relative
                              divergence error); 0 runs max_refine sweeps */
  int32_t max_refine;      /* PPE_PREC_MIXED: refinement sweeps after the first
                              solve (>= 0) */
  int32_t batch;           /* same-shape instances handled per call (>= 1) */
  int32_t flags;           /* PPE_FLAG_* */
  int32_t reserved;        /* 0 */
} ppe_desc_t;

/* Per-instance record, written to DEVICE memory by ppe_solve / ppe_correct. */
typedef struct {
  int32_t status;          /* ppe_status_t (PPE_OK, NOT_CONVERGED, NONFINITE) */
  int32_t iters;           /* refinement sweeps run (0 for PPE_PREC_FP64) */
  double rho0_used;        /* rho0 actually used */
  double compat_defect;    /* mean(D u* - S): the incompatible part removed
                              (0 for PPE_YBC_OUTFLOW) */
  double res_rel;          /* ppe_solve: last refinement residual (relative);
                              ppe_correct: div_l2 / div0_l2 */
  double div_l2;           /* ppe_correct: ||D u^{n+1} - S_c||_2 */
  double div_max;          /* ppe_correct: max |D u^{n+1} - S_c| */
  double div0_l2;          /* ||D u* - S_c||_2 */
  double p_mean;           /* ppe_correct: mean of p (0 up to rounding for
                              PPE_YBC_WALLS: the gauge) */
} ppe_info_t;

/* Maximum number of instances per call; larger batches need several calls. */
#define PPE_MAX_BATCH 64

/* Bytes of device memory ppe_plan allocates for this descriptor (workspace,
 * tables, reduction scratch), for admission control.  0 on a bad descriptor. */
size_t ppe_plan_workspace_bytes(const ppe_desc_t* desc);

/* Build a plan for `desc` bound to `stream` (a hipStream_t; NULL = the null
 * stream) on the current device.  Allocates the workspace and FP64 twiddle /
 * eigenvalue tables; a plan that refines its y solves (ny > 256 or
 * PPE_FLAG_Y_REFINE) also holds the list of tridiagonal blocks to refine.
 * All work runs on `stream`.  On success *out holds the plan; on failure *out
 * is NULL. */
ppe_status_t ppe_plan(const ppe_desc_t* desc, void* stream, ppe_plan_t* out);

/* Release a plan and its device memory (waits for its stream first). */
ppe_status_t ppe_plan_destroy(ppe_plan_t plan);

/* Re-bind a plan to another stream (same device). */
ppe_status_t ppe_plan_set_stream(ppe_plan_t plan, void* stream);

/* Pressure solve, Eq. (29) with Eq. (27) (Sec. 5.4).
 *   rho0[b] : host array; > 0 is used as given, <= 0 requests min(rho) (device)
 *   dt[b]   : host array, > 0
 *   us, vs, ws, rho, pn, pnm1, S : host arrays of `batch` device pointers (inputs)
 *   p       : host array of `batch` device pointers (output; zero-mean for
 *             PPE_YBC_WALLS)
 *   info    : device array of `batch` records (output)
 * For PPE_PREC_MIXED the first solve uses FP32 spectra and is refined with
 * residuals formed in FP64 until `tol` or `max_refine`. */
ppe_status_t ppe_solve(ppe_plan_t plan, const double* rho0, const double* dt,
                       const double* const* us, const double* const* vs, const double* const* ws,
                       const double* const* rho, const double* const* pn, const double* const* pnm1,
                       const double* const* S, double* const* p, ppe_info_t* info);

/* Right-hand side of Eq. (29) alone, with Eq. (27) (Sec. 5.4):
 *   b = (rho0/dt)(D u* - S) + D((1 - rho0/rho_f) G p_hat),  p_hat = 2 p^n - p^{n-1},
 * zero flux through the zero-flux y faces (an outflow top face carries the
 * ghost value -p_hat), before any compatibility projection.  The same pass
 * ppe_solve starts with, for callers that assemble here and solve elsewhere,
 * and for checking the assembly on its own.
 *   rho0, dt, us .. S : as for ppe_solve
 *   b    : host array of `batch` device pointers (output, [nz][ny][nx])
 *   info : device array of `batch` records; rho0_used and compat_defect
 *          (mean(D u* - S) with zero-flux ends, else 0) are written, the rest
 *          cleared */
ppe_status_t ppe_rhs(ppe_plan_t plan, const double* rho0, const double* dt,
                     const double* const* us, const double* const* vs, const double* const* ws,
                     const double* const* rho, const double* const* pn, const double* const* pnm1,
                     const double* const* S, double* const* b, ppe_info_t* info);

/* Pressure of the variable-coefficient problem, Eq. (25), by the split
 * fixed-point iteration (Sec. 5.4: the split is exact when grad p_hat equals
 * grad p^{n+1}, so the pressure of Eq. 25 is the fixed point of the split
 * with p_hat fed back):
 *   p_0 = 2 p^n - p^{n-1},
 *   p_{k+1} = p_k + L^+ [ (rho0/dt)(D u* - S) - rho0 D((1/rho_f) G p_k) ],
 * where the bracket is rho0 times the residual of Eq. (25) (in FP64) and L^+
 * the same FFT/tridiagonal solve as ppe_solve (in the plan's precision), with
 * the same compatibility and gauge.  p_1 is exactly ppe_solve's pressure.
 * The error contracts at least by 1 - rho0/rho_max per sweep (energy norm), so
 * the first update also bounds the split's own error:
 *   ||p_1 - q||_E <= ||p_2 - p_1||_E / (rho0/rho_max).
 * Stops when the relative residual
 *   res_k = ||rho0 [(1/dt)(D u* - S_c) - D((1/rho_f) G p_k)]||_2 / ||(rho0/dt)(D u* - S_c)||_2
 * reaches tol, or after max_iters updates (>= 0; 0 only evaluates res_0).
 * The plan needs PPE_FLAG_VARCOEF, for either precision (else PPE_ERR_ARG).
 *   p     : output, must not alias p^n or p^{n-1}
 *   tol   : 0 runs max_iters sweeps without a convergence test
 *   info  : status (PPE_ERR_NOT_CONVERGED if tol > 0 and res > tol after
 *           max_iters, or NONFINITE), iters = updates applied, res_rel = last
 *           residual, rho0_used, compat_defect
 *   hist  : NULL or a device array [batch][max_iters + 1]; hist[b][k] = res_k,
 *           -1 after convergence
 * With tol > 0 the host stops enqueuing sweeps once every instance has
 * converged: every 4 sweeps the convergence flags are copied to pinned host
 * memory, and before enqueuing further sweeps the call waits for the copy
 * made 4 sweeps earlier (so it blocks the host while at most 4 more sweeps
 * are queued).  With tol = 0 it only enqueues, like ppe_solve.
 * ppe_correct(rho0 = NULL, pn = p, pnm1 = p, p) then applies the variable-density
 * projection u^{n+1} = u* - dt G p / rho_f, whose relative divergence error
 * is the last res. */
ppe_status_t ppe_solve_varcoef(ppe_plan_t plan, const double* rho0, const double* dt,
                               const double* const* us, const double* const* vs, const double* const* ws,
                               const double* const* rho, const double* const* pn, const double* const* pnm1,
                               const double* const* S, double* const* p, ppe_info_t* info,
                               int32_t max_iters, double tol, double* hist);

/* Inputs of the predictor, Eq. (23) (Sec. 5.4), for one instance.  Device
 * pointers, float64, layouts as above (u, uv, fsx like u; v, vv, fsy like v;
 * w, wv, fsz like w; the rest cell fields).
 *   u, v, w          : u^n (faces)
 *   uv, vv, wv       : velocity used in the viscous term (the paper uses
 *                      phase-wise velocities there); NULL = u^n, v^n, w^n
 *   rho_n, rho_np1   : cell densities at times n and n+1
 *   mu               : cell viscosity (> 0)
 *   C                : volume fraction at n+1 (interface cells: 0 < C < 1)
 *   sigma, kappa     : surface-tension coefficient and curvature, non-zero
 *                      only in interface cells (Eq. 30 carries them to faces)
 *   fsx, fsy, fsz    : tangential surface force grad_s(sigma)|grad C| on
 *                      faces; NULL = none
 *   rho_mean         : <rho> = (rho_G + rho_L)/2 of the CSF density scaling
 *   dt               : time step (> 0) */
typedef struct {
  const double* u;
  const double* v;
  const double* w;
  const double* uv;
  const double* vv;
  const double* wv;
  const double* rho_n;
  const double* rho_np1;
  const double* mu;
  const double* C;
  const double* sigma;
  const double* kappa;
  const double* fsx;
  const double* fsy;
  const double* fsz;
  double rho_mean;
  double dt;
} ppe_predict_t;

/* Predictor, Eq. (23):
 *   u^p = [ rho^n_f u^n + dt ( -div(rho u u)^n + div(tau)^n
 *                              + (rho^{n+1}_f/<rho>)(sigma_f kappa_f grad C + f_s) ) ] / rho^{n+1}_f
 * on the staggered finite volumes of Sec. 5.4:
 *   - convection: SMART on every momentum control-volume face; where a cell
 *     touching that face is an interface cell, central differences if the
 *     cell Peclet number |m| h / mu < 2, else first-order upwind.  Mass flux
 *     m: the mean of the two neighbouring face mass fluxes (rho_f times the
 *     face velocity), or at a cell centre rho times the mean face velocity;
 *   - viscous: tau = mu [grad u + grad u^T - (2/3)(div u) I] (Sec. 2) in
 *     central differences; mu on edges is the mean of the four cells;
 *   - surface tension: CSF with density scaling; sigma and kappa on faces by
 *     Eq. (30), grad C the face difference;
 *   - rho on faces: the mean of the two cells (as in the projection);
 *   - y ends: ghost cells mirror the first two rows (cell fields, u, w); v
 *     beyond a wall or symmetry face is 2 v_b - v, beyond an outflow face
 *     v_ny.  Wall and symmetry faces of v keep v^n; an outflow face
 *     (PPE_YBC_OUTFLOW) is predicted.
 *   in         : host array of `batch` records
 *   up, vp, wp : host arrays of `batch` device pointers (outputs, must not
 *                alias an input)
 * Needs ny >= 4 (else PPE_ERR_UNSUPPORTED). */
ppe_status_t ppe_predict(ppe_plan_t plan, const ppe_predict_t* in, double* const* up, double* const* vp,
                         double* const* wp);

/* Pressure history resident in device memory, for time loops.  A ring holds
 * three pressure buffers per instance (p^{n-1}, p^n and the next pressure);
 * each step solves with p_hat = 2 p^n - p^{n-1} taken from the ring (Eq. 27),
 * writes p^{n+1} into the oldest buffer, applies the projection (Eq. 28) and
 * rotates, so a time loop moves no pressure data between steps.  The ring
 * owns its buffers (3 * batch * nx*ny*nz doubles) and uses the plan's stream;
 * the plan must outlive the ring. */
typedef struct ppe_ring_s* ppe_ring_t;

/* pn, pnm1: host arrays of `batch` device pointers, copied into the ring
 * (stream-ordered).  pnm1 may be NULL: p^{n-1} = p^n, so the first p_hat is p^n. */
ppe_status_t ppe_ring_create(ppe_plan_t plan, const double* const* pn, const double* const* pnm1, ppe_ring_t* out);

/* One projection step: ppe_solve + ppe_correct with the ring's history, then
 * rotate (the new pressure becomes p^n).  Arguments as for those calls
 * (ppe_correct with rho0 = NULL: it reads the solve's info record).
 * split_defect: NULL, or a device array [batch][2] that receives the relative
 * residual of the variable-coefficient problem, Eq. (25), for p_hat ([b][0])
 * and for the split pressure p^{n+1} ([b][1]) -- how far the split is from
 * the variable-density projection this step (Sec. 5.4).  Both residuals are
 * formed in FP64, relative to ||(rho0/dt)(D u* - S_c)||_2, after ppe_solve:
 * the pressure, velocities and info record are bitwise those of the step
 * without the diagnostic, in either precision (a mixed plan's pressure is
 * the refined one).  It needs the plan's FP64 residual buffer
 * (PPE_FLAG_VARCOEF; else PPE_ERR_ARG). */
ppe_status_t ppe_ring_step(ppe_ring_t ring, const double* rho0, const double* dt,
                           const double* const* us, const double* const* vs, const double* const* ws,
                           const double* const* rho, const double* const* S,
                           double* const* u, double* const* v, double* const* w, ppe_info_t* info,
                           double* split_defect);

/* Device pointers of the ring's pressures: lag 0 = p^n (the newest), lag 1 =
 * p^{n-1}.  p: host array of `batch` entries. */
ppe_status_t ppe_ring_pressure(ppe_ring_t ring, int32_t lag, double** p);

/* Copy the ring's pressure of the given lag into caller buffers (host array
 * of `batch` device pointers), stream-ordered on the plan's stream. */
ppe_status_t ppe_ring_read(ppe_ring_t ring, int32_t lag, double* const* out);

/* Steps taken since creation. */
int64_t ppe_ring_steps(ppe_ring_t ring);

/* Free the ring's buffers (waits for the plan's stream first). */
ppe_status_t ppe_ring_destroy(ppe_ring_t ring);

/* Projection, Eq. (28) (Sec. 5.4), with rho0 of Eq. (27), and the continuity
 * check of the result.
 *   rho0    : NULL, or a host array of `batch` values.
 *             NULL: rho0_used and compat_defect are read from `info`, as
 *             ppe_solve wrote them for the same inputs (the usual step).
 *             Array: > 0 is used as given, <= 0 requests min(rho) (device);
 *             the compatibility defect mean(D u* - S) (zero-flux ends; 0 with
 *             an outflow top) is reduced from us, vs, ws, S here, and `info`
 *             is initialised (status 0, iters 0, rho0_used, compat_defect).
 *             This projects with a pressure obtained elsewhere: no ppe_solve
 *             needs to precede the call.
 *   dt      : host array, > 0
 *   p       : the pressure to project with (any source)
 *   u, v, w : host arrays of `batch` device pointers (outputs; the wall rows
 *             of v are copied from v*, an outflow row is corrected)
 * Writes div_l2, div_max, div0_l2, res_rel, p_mean and status
 * (PPE_ERR_NOT_CONVERGED when res_rel > desc.tol > 0 on a mixed plan,
 * PPE_ERR_NONFINITE for a non-finite residual) to `info`. */
ppe_status_t ppe_correct(ppe_plan_t plan, const double* rho0, const double* dt,
                         const double* const* us, const double* const* vs, const double* const* ws,
                         const double* const* rho, const double* const* pn, const double* const* pnm1,
                         const double* const* p, const double* const* S,
                         double* const* u, double* const* v, double* const* w, ppe_info_t* info);

/* Continuity diagnostic of any staggered field (the constraint behind
 * Eq. 25): out[3*b + 0] = ||d - mean d||_2, out[3*b + 1] = max |d - mean d|,
 * out[3*b + 2] = mean d, with d = D u - S.  `out` is a device array.  (The
 * mean is removed for either ybc; with an outflow top the projected field's
 * mean d is itself zero to rounding.) */
ppe_status_t ppe_residual(ppe_plan_t plan, const double* const* u, const double* const* v,
                          const double* const* w, const double* const* S, double* out);

/* Inputs of the target divergence S = div u^{n+1} of Eq. (26) (Sec. 5.4)
 * for one instance: cell fields [nz][ny][nx], float64 device pointers owned
 * by the caller.  C classifies each cell: gas (C <= 0), liquid (C >= 1),
 * interface (0 < C < 1).
 *   div_g, div_l : phase-wise velocity divergences -(1/rho_k) D rho_k/Dt (the
 *                  extrapolated compressibilities, Sec. 4); div_g is read in
 *                  gas and interface cells, div_l in liquid and interface
 *                  cells
 *   mdot         : interface mass flux per unit area m' (> 0 vaporisation)
 *   area         : interface area density A_Gamma / V0 (Sec. 3: the
 *                  phase-change rate per volume is m' A_Gamma / V0)
 *   rho_g, rho_l : interface gas and liquid densities
 *                  (mdot, area, rho_g, rho_l are read in interface cells only)
 *   under        : uint8 mask, non-zero = under-resolved cell; an
 *                  under-resolved interface cell gets S = 0 (the paper's
 *                  treatment of under-resolved regions); NULL = no such cells */
typedef struct {
  const double* C;
  const double* div_g;
  const double* div_l;
  const double* mdot;
  const double* area;
  const double* rho_g;
  const double* rho_l;
  const uint8_t* under;
} ppe_source_t;

/* Target divergence, Eq. (26):
 *   gas cell S = div_g, liquid cell S = div_l, interface cell
 *   S = (1 - C) div_g + C div_l + mdot * area * (1/rho_g - 1/rho_l)
 *   (0 if under-resolved).
 *   src : host array of `batch` records
 *   S   : host array of `batch` device pointers (output, [nz][ny][nx]; must
 *         not alias an input)
 * The result is the S that ppe_solve and ppe_correct take. */
ppe_status_t ppe_source(ppe_plan_t plan, const ppe_source_t* src, double* const* S);

/* Pressure solve without a plan and without allocating, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  The same computation as
 * ppe_plan(desc) + ppe_solve and, when u, v, w are given, ppe_correct with
 * rho0 = NULL; results equal theirs to rounding (the twiddle and eigenvalue
 * tables are formed on the device here, on the host by ppe_plan).
 *   desc   : as for ppe_plan; ny <= 256, and neither PPE_FLAG_Y_REFINE nor
 *            PPE_FLAG_VARCOEF (else PPE_ERR_UNSUPPORTED)
 *   stream : hipStream_t the work is enqueued on (NULL = the null stream)
 *   rho0 .. S, p, info : as for ppe_solve
 *   u, v, w : NULL (pressure only), or host arrays of `batch` device pointers
 *            receiving the projection, as for ppe_correct
 * Workspace: a 64 MiB array in the library's device data, one per GPU, held
 * until the process ends; its device address is looked up on the first call
 * on each device.  A descriptor whose workspace (ppe_plan_workspace_bytes)
 * exceeds it returns PPE_ERR_NOMEM and enqueues nothing: FP64 grids up to
 * about 3.5 M cells in all (192x96x192 fits).  The call allocates no memory.
 * Every call on one GPU uses that GPU's array and leaves its contents behind
 * (the call clears what it relies on): calls that overlap on one GPU, on
 * different streams or from different threads, race and give wrong results;
 * serialise them (one stream, or events). */
ppe_status_t ppe_solve_noalloc(const ppe_desc_t* desc, void* stream, const double* rho0, const double* dt,
                               const double* const* us, const double* const* vs, const double* const* ws,
                               const double* const* rho, const double* const* pn, const double* const* pnm1,
                               const double* const* S, double* const* p, double* const* u, double* const* v,
                               double* const* w, ppe_info_t* info);

/* Per-kernel timing, for measurement tools.  With profiling enabled every
 * launch the plan makes is bracketed by two HIP events on the plan's stream;
 * durations are folded into per-kernel totals.  Enabling clears the totals.
 * The events add a small gap between launches, so leave profiling off for
 * end-to-end timing. */
typedef struct {
  char name[32];           /* kernel family, e.g. "k_correct", "k_fft_z_fwd" */
  int32_t launches;        /* launches timed since profiling was enabled */
  double total_ms;         /* sum of their event-to-event durations */
} ppe_kernel_time_t;

ppe_status_t ppe_plan_profile(ppe_plan_t plan, int32_t enable);

/* Copy up to `cap` per-kernel records into `out` (host memory) and the
 * number of kernel families into *count.  Waits for the plan's stream. */
ppe_status_t ppe_plan_profile_read(ppe_plan_t plan, ppe_kernel_time_t* out, int32_t cap, int32_t* count);

/* Library version string (static storage). */
const char* ppe_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PPE_H */
