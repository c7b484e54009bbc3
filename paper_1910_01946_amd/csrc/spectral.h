// Plans and launchers of the spectral path (3-D FFTs, projection, curl, CG updates).
#pragma once

#include "fft.h"
#include "kernels.h"

namespace rve {

// Real 9-component fields (nvox each) <-> half spectrum (nz, ny, nxh), nxh = nx/2 + 1.
struct GridPlan {
  int nx, ny, nz, nxh;
  int64_t nvox, nspec;
  AxisPlan ax, ay, az;
  const void* twx;   // exp(-2 pi i k / n), n entries, in the spectral precision
  const void* twy;
  const void* twz;
  const void* Ex;    // exp(+2 pi i q / n) for the modified frequencies (A.4), FP64
  const void* Ey;
  const void* Ez;
  int ly;            // rows per block in the x passes (even)
  int ty;            // kx columns per block in the y passes
  int tz;            // kx columns per block in the z pass (nine components)
  int tz3;           // kx columns per block in the z pass of the factorised projection (three)
  FastDiv fnx, fnxh, fnz, ftz, ftz3;  // divisions by nx, nxh, nz, tz, tz3
  int freq;          // FREQ_ROTATED (eq. A.4) or FREQ_STANDARD (continuous frequencies)
};

// Frequency vector of the derivative i k / h in the projection and the curl.
//   FREQ_ROTATED:  k_i = 1/4 (-i)(E_i - 1) prod_{j != i} (1 + E_j), E = exp(i xi) (eq. A.4): the
//                  rotated finite-difference scheme the paper uses;
//   FREQ_STANDARD: k_i = xi_i in (-pi, pi), the continuous derivative of the trigonometric
//                  interpolant, with the Nyquist frequency's derivative set to 0 (the
//                  comparison of Appendix B).
enum FreqScheme { FREQ_ROTATED = 0, FREQ_STANDARD = 1 };

// Device-resident scalars of the conjugate-gradient loop (FP64).
//
// The operator is applied to the residual and the search-direction image follows by
// linearity, so that every dot product is taken from stored vectors:
//   forward x pass (iteration k > 0):  r -= alpha q;  partial r.r;  K : r
//   beta kernel:   beta = r.r / (previous r.r);  stop if r.r <= tol2 r0.r0
//   inverse x pass: w = G(K : r);  x += alpha p (iteration k > 0, the previous p and alpha),
//                  q = w + beta q,  p = r + beta p;  partial p.q
//   alpha kernel:  alpha = r.r / p.q
// and after the last iteration k_cg_finish adds the pending alpha p to x.
// (q = G(K : p) by linearity of the projected operator).  Taking p.q from the projected
// q keeps alpha consistent with the operator actually applied (p.Kp equals p.G(Kp) only
// while p lies exactly in the range of G, which FP32 rounding does not preserve), and
// r.r is summed from the stored residual each iteration.
struct CGState {
  double rr;       // r . r of the current residual
  double rr0;      // r . r of the right-hand side
  double pq;
  double alpha, beta;
  double tol2;     // stop when rr <= tol2 * rr0
  double rr_best;  // smallest r.r so far that was at most a quarter of the previous best
  double rr_floor; // also stop once rr <= rr_floor: the rounding floor of the right-hand side
                   // (FP32 spectra), below which no correction is resolved
  int32_t iter;    // completed operator applications
  int32_t done;    // 0 running, 1 converged, 2 breakdown (p.q <= 0), 3 diverging (r.r > 1e4 r0.r0),
                   // 4 max_iter, 5 stalled (|r| not halved within `stall` iterations)
  int32_t max_iter;
  int32_t it_best; // iteration of rr_best
  int32_t stall;   // stalled (5) once |r| has not halved for this many iterations
  int32_t pad;
};

// A solve whose residual norm has not halved for kCgStall iterations has reached the
// rounding floor of the operator (the consistent tangent is not symmetric, and CG on a
// right-hand side at that floor need not converge): it stops with its current iterate.
// FP64 solves wait longer: on a badly conditioned operator (a stiffness contrast of 1e6
// with the standard frequencies) the residual norm of CG can plateau for over a thousand
// iterations far above its rounding floor before it falls again, and a stop there hands
// Newton a correction that has not resolved the residual.  The FP32 form's floor also
// ends the solve through rr_floor.
constexpr int kCgStall = 500;
constexpr int kCgStall64 = 2000;

enum XFwdMode { XF_FIELD64 = 0, XF_CG = 1, XF_FP_MINUS_I = 2 };
enum XInvMode { XI_RESID = 0, XI_CG = 1, XI_NYE = 2, XI_OUT64 = 3 };
// MID_GREEN: the projection of eq. 17 on nine components; MID_CURL: the curl of eq. 12;
// MID_GREEN3: the middle factor of the factorised projection (see PF_DIV) on three
// components, w_i = v_i / |k|^2, with the zero frequency and the modes where k vanishes set
// to zero.
enum MidOp { MID_GREEN = 0, MID_CURL = 1, MID_GREEN3 = 2 };

struct XFwdArgs {
  int mode;
  const double* in64;          // XF_FIELD64 / XF_FP_MINUS_I input, 9 x nvox
  const void* K;               // XF_CG: crystal-frame tangent (T), 81 x nvox
  const int32_t* gid;          // XF_CG: grain ids for the frame rotation
  const double* grainR;
  void* x;                     // XF_CG: solution (T), x += alpha p
  void* xbest;                 // XF_CG: copy of the iterate with the best r.r (T)
  void* r;                     // XF_CG: residual (T), r -= alpha q
  const void* p;               // XF_CG: search direction (T)
  const void* q;               // XF_CG: G(K : p) (T)
  CGState* cg;
  double* partial;             // XF_CG: per-block r.r
  void* spec;                  // out: half spectrum (complex T)
};

struct MidArgs {
  int op;
  void* spec;
  double mask_keep[9];         // 1 where the average is stress-controlled (kept)
  double dc_target[9];         // prescribed average of the kept components
  double inv_n;                // 1 / nvox
  double inv_h;                // MID_CURL: 1 / voxel size
  const CGState* cg;           // skip when cg && cg->done
};

struct XInvArgs {
  int mode;
  const void* spec;
  void* x;                     // XI_RESID (T)
  void* r;                     // XI_RESID: out; XI_CG: in
  void* p;                     // XI_RESID: out; XI_CG: p = r + beta p
  void* q;                     // XI_CG: q = G(K : r) + beta q
  CGState* cg;
  double* partial;             // XI_RESID: per-block r.r; XI_CG: per-block p.q
  double* out64;               // XI_OUT64 / XI_NYE: 9 x nvox FP64
  double* rho_gnd;             // XI_NYE: 12 x nvox
  const int32_t* gid;
  const double* grainR;
  const MatDev* mat;
};

void launch_xfwd(const GridPlan& g, bool fp32, const XFwdArgs& a, hipStream_t st);
void launch_yfft(const GridPlan& g, bool fp32, void* spec, int sign, const CGState* cg, hipStream_t st);
// ---- CG scalar updates (device side) ----------------------------------------------
// beta step, after r.r of the updated residual: beta = r.r / previous r.r; stop when
// r.r <= tol2 r0.r0 (1), when it grows past 1e4 r0.r0 or is not finite (3), at the
// iteration cap (4), or when |r| has stalled (5).  first: the first iteration of the
// solve (beta = 0).
__device__ inline void cg_beta_update(CGState* cg, double rr, bool first) {
  cg->beta = first ? 0.0 : rr / cg->rr;
  cg->rr = rr;
  if (first || rr <= 0.25 * cg->rr_best) {
    cg->rr_best = rr;
    cg->it_best = cg->iter;
  }
  if (rr <= cg->tol2 * cg->rr0 || rr <= cg->rr_floor) cg->done = 1;
  else if (!(rr < 1e4 * cg->rr0)) cg->done = 3;
  else if (cg->iter >= cg->max_iter) cg->done = 4;
  else if (cg->iter - cg->it_best >= cg->stall) cg->done = 5;
}

// alpha step, after p.q: alpha = r.r / p.q; a non-positive (or non-finite) p.q is a
// breakdown (2).
__device__ inline void cg_alpha_update(CGState* cg, double pq) {
  cg->pq = pq;
  cg->iter += 1;
  if (pq > 0.0 && pq < 1e300) {
    cg->alpha = cg->rr / pq;
  } else {
    cg->alpha = 0.0;
    cg->done = 2;
  }
}

void launch_mid(const GridPlan& g, bool fp32, const MidArgs& a, hipStream_t st);
void launch_xinv(const GridPlan& g, bool fp32, const XInvArgs& a, hipStream_t st);
int xfwd_blocks(const GridPlan& g);
int xinv_blocks(const GridPlan& g);

// CG bookkeeping kernels (one block).
void launch_cg_beta(CGState* cg, const double* partial, int n, hipStream_t st);
void launch_cg_alpha(CGState* cg, const double* partial, int n, hipStream_t st);
void launch_cg_start(CGState* cg, const double* partial, int n, double tol2, int max_iter, hipStream_t st);

// Sums of a 9- or 12-component FP64 field (per-block partials, reduced on the host),
// and sum of squares of a T field.
int launch_colsum(const double* f, int ncomp, int64_t nvox, double* partial, hipStream_t st);
int launch_sumsq(const void* f, bool fp32, int64_t n, double* partial, hipStream_t st);
// out[i] = (double)in[i], i < n
void launch_widen(const float* in, double* out, int64_t n, hipStream_t st);
void launch_negate(const double* in, double* out, int64_t n, hipStream_t st);

// ---- plane path (x and y transforms of one component plane in LDS) ----------------
//
// The factorised projection.  With the rotated scheme every component of the modified
// frequency (eq. A.4) is, up to the common factor -i, the symbol d_j of a real stencil on the
// 2 x 2 x 2 voxel cube: a forward difference along axis j averaged over the other two axes,
//   D_j = 1/4 (S_j - 1) prod_{m != j} (1 + S_m),   S_m u(x) = u(x + e_m),
// and conj(d_j) is the symbol of its adjoint D_j^H (shifts by -e_m).  The projection of
// eq. 17 away from the zero frequency, (G:A)_ij = k_j sum_l A_il conj(k_l) / |k|^2, is then
//   G:A = D_j w_i,   w_i = (D^H D)^-1 v_i,   v_i = sum_l D_l^H A_il,   D^H D = |d|^2 = |k|^2,
// so the transforms carry the three components v_i instead of nine:
//   k_plane_fwd<PF_DIV>  v_i = sum_l D_l^H y_il on the fly, x and y transforms of v_i;
//   k_mid<MID_GREEN3>    z transforms, times 1 / (nvox |k|^2), inverse z transforms;
//   k_plane_inv<PI_OUT_T> inverse y and x transforms, w_i stored;
//   k_cg_grad            q_ij = D_j w_i + the zero-frequency term, then the CG epilogue.
// The zero frequency keeps the nine-component rule: its output is mask_keep * <y>, from
// plane sums that the PF_DIV pass writes and the PI_OUT_T pass reduces.
enum PlaneSrc { PF_T = 0, PF_F64 = 1, PF_FPI = 2, PF_DIV = 3 };
enum PlaneMode { PI_CG = 0, PI_RESID = 1, PI_OUT64 = 2, PI_OUT_T = 3 };

struct PlaneArgs {
  int src;                     // PF_T: field of type T; PF_F64: FP64 field; PF_FPI: FP64 Fp - I
  const void* in;              // 9 x nvox
  void* spec;                  // out: half spectrum
  // CG iteration (with a CGState): block 0 sums the r.r partials of k_cg_prep and takes the
  // beta step before the inverse pass reads beta
  const double* rr_partial;
  int n_rr;
  int it;                      // iteration index within the solve (0 = first)
  double* plane_sums;          // PF_DIV: sums of y_il over plane z at [(3 i + l) nz + z]
};

struct PlaneInvArgs {
  int mode;
  const void* spec;
  void* x;                     // PI_RESID: set to 0
  void* r;                     // PI_RESID: out (-w); PI_CG: in
  void* p;                     // PI_RESID: out (= r); PI_CG: p = r + beta p
  void* q;                     // PI_CG: q = w + beta q
  double* out64;               // PI_OUT64
  CGState* cg;
  double* partial;             // per-block (9 x nz) r.r (PI_RESID) or p.q (PI_CG)
  // PI_OUT_T: the real planes of the three components, stored as T (3 x nvox); blocks of
  // plane 0 also reduce the plane sums of PF_DIV to the zero-frequency term
  // dc[c] = mask_keep[c] sum_z plane_sums[c nz + z] / nvox
  void* out;
  const double* plane_sums;
  double* dc;
  double mask_keep[9];
  double inv_n;
};

// q = D w + dc, then the CG epilogue of k_plane_inv<PI_CG>: q = q + beta q_prev,
// p = r + beta p, per-block p.q.  Each thread walks lz consecutive z planes of one (x, y)
// column and carries the corner values of the upper plane to the next step.
struct GradArgs {
  const void* w;               // 3 x nvox (T)
  void* x;                     // the CG iterate: x += alpha p of the previous iteration
  const double* dc;            // 9 values
  const void* r;
  void* p;
  void* q;
  CGState* cg;
  double* partial;             // per-block p.q
  int lz;                      // z planes per thread
};

struct PrepArgs {
  const void* K;               // crystal-frame tangent (T, or FP16 pairs: see launch_cg_prep)
  const int32_t* gid;
  const double* grainR;
  void* x;
  void* xbest;                 // copy of the iterate with the best r.r (T)
  void* r;
  const void* p;
  const void* q;
  void* y;                     // out: K : r (T)
  CGState* cg;
  double* partial;             // per-block r.r
  double k_scale;              // FP16 K: y = k_scale (K16 : r)
};

bool plane_fits(const GridPlan& g, bool fp32);
// Raise the dynamic-LDS limit of every LDS-staged spectral kernel to bytes.  Called once
// per device before the first launch (never concurrently with launches).
hipError_t set_spectral_lds_limits(int bytes);
hipError_t set_plane_lds_limits(int bytes);
int plane_blocks(const GridPlan& g);
int prep_blocks(const GridPlan& g);
// The factorised projection runs with the rotated scheme only, on grids that take the plane
// path and whose planes have at most 9 points per thread of the 1024-thread three-component
// plane kernels (planes to about 128 x 128, all that the plane path holds in LDS); the caller
// checks plane_fits for its precision.
bool factorised_fits(const GridPlan& g);
// most blocks (and p.q partials) of the gradient pass
constexpr int kGradBlocks = 4096;
int grad_blocks(const GridPlan& g, int lz);
int grad_lz(const GridPlan& g);
void launch_cg_grad(const GridPlan& g, bool fp32, const GradArgs& a, hipStream_t st);
// x += alpha p for the last iteration of a CG solve (n = 9 nvox values of the CG precision)
void launch_cg_finish(const CGState* cg, bool fp32, void* x, const void* p, int64_t n, hipStream_t st);
void launch_plane_fwd(const GridPlan& g, bool fp32, const PlaneArgs& a, CGState* cg, hipStream_t st);
void launch_plane_inv(const GridPlan& g, bool fp32, const PlaneInvArgs& a, hipStream_t st);
// k16: the tangent copy is FP16 pairs scaled by 1/k_scale (grouped layout of
// TangentGroups<__half>); otherwise it is in the CG precision.  transpose: apply K^T (FP64
// only, for the adjoint system)
void launch_cg_prep(const GridPlan& g, bool fp32, bool k16, bool transpose, const PrepArgs& a, hipStream_t st);
void launch_gnd(int64_t nv, const double* nye, const int32_t* gid, const double* grainR, const MatDev* mat,
                double* rho_gnd, hipStream_t st);

// Initial guess of an increment: out = 2 F - F_prev + corr (F + corr when F_prev is null).
struct Corr9 {
  double v[9];
};
void launch_predictor(const double* F, const double* F_prev, Corr9 corr, double* out, int64_t nvox,
                      hipStream_t st);

}  // namespace rve
