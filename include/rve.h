/*
 * rve.h -- C ABI of the MI355X (gfx950) library for FFT-based strain-gradient
 * crystal-plasticity homogenization of periodic FCC polycrystal RVEs.
 *
 * Method: Haouala, Lucarini, LLorca, Segurado, "Simulation of the Hall-Petch effect in
 * FCC polycrystals by means of strain gradient crystal plasticity and FFT
 * homogenization" (arXiv 1910.01946).  Section numbers and equation numbers below
 * refer to that paper.
 *
 * Conventions shared by every call
 *  - Units: SI (Pa, m, s, 1/m^2).
 *  - Tensors are row-major 3x3 (component ij at index 3*i + j); x, y, z = 0, 1, 2.
 *  - Voxel fields are component-major ("SoA"): field[c * nvox + v] with the voxel index
 *    v = (z * ny + y) * nx + x (x fastest).
 *  - Every call returns an rve_status; 0 is success.  A failing call leaves the handle's
 *    committed state unchanged and stores a message readable with rve_last_error().
 *  - Host pointers are read during the call only (inputs are copied); output host
 *    buffers are owned and sized by the caller.  Pointers documented as "device" must
 *    point to memory of the handle's device (for instance from torch tensors on cuda:0).
 *  - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef RVE_H
#define RVE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rve_ctx* rve_handle;

enum {
  RVE_OK = 0,
  RVE_EINVAL = -1,   /* bad argument: shape, non-finite value, dt <= 0, unknown index   */
  RVE_ENOMEM = -2,   /* device allocation failed                                       */
  RVE_EDEVICE = -3,  /* a HIP runtime call failed                                      */
  RVE_ENOCONV = -4,  /* Newton / CG / local update did not converge; state rolled back */
  RVE_ESTATE = -5    /* call not valid in the current state                            */
};

enum { RVE_FP64 = 0, RVE_MIXED = 1 };

/* Single-crystal parameters (Section 2.1; Tables 1 and 2). */
typedef struct {
  double C11, C12, C44;  /* cubic elastic constants in the crystal frame, Pa (eq. 4)            */
  double mu;             /* Taylor shear modulus, Pa (eq. 7); <= 0 selects the {111}<110> shear
                            modulus 3 C44 (C11-C12) / (C11-C12+4 C44) (Table 2's mu)           */
  double burgers;        /* Burgers vector magnitude b, m (eqs. 7, 8, 13)                      */
  double y_c;            /* effective annihilation distance, m (eq. 8)                         */
  double K_sim;          /* similitude coefficient K (eq. 9)                                   */
  double gamma0_dot;     /* reference slip rate, 1/s (eq. 6)                                   */
  double m_rate;         /* rate sensitivity m; the flow-rule exponent is 1/m (eq. 6)          */
  double q[6];           /* interaction coefficients: self, coplanar, collinear, Hirth,
                            glissile, Lomer (Table 1, eq. 7)                                  */
  double tau0;           /* Pa: initial critical stress; sets the uniform initial SSD density
                            rho0 = (tau0 / (mu b))^2 / sum_b q^{ab} (used when rho0 <= 0)      */
  double rho0;           /* initial SSD density per slip system, 1/m^2 (> 0 overrides tau0)   */
  double c_gnd;          /* weight of the GND density in eqs. 7 and 9 (1: the paper's model,
                            0: no gradient term, the paper's "infinite grain size")          */
  int32_t hardening;     /* 1: tau_c from the dislocation densities (eqs. 7-9);
                            0: tau_c fixed at tau0 and densities frozen                        */
} rve_material;

/* One RVE: a periodic voxel grid with a grain map (Section 2.2). */
typedef struct {
  int32_t n[3];                  /* voxels along x, y, z; each 1..256 with prime factors 2, 3, 5  */
  double voxel_size;             /* h, m: sets the length scale of the Nye tensor (eq. 12)       */
  int32_t n_grains;
  const int32_t* grain_of_voxel; /* host, nvox entries in [0, n_grains); copied                  */
  const double* grain_quat;      /* host, n_grains x (w, x, y, z), crystal -> sample; copied and
                                    normalised                                                  */
  rve_material material;         /* by value                                                     */
  const double* grain_elastic;   /* host, n_grains x (C11, C12, C44) in Pa, cubic in the crystal
                                    frame (eq. 4), copied; NULL: the material's constants for
                                    every grain.  Lets one RVE hold phases of different stiffness
                                    (for instance the elastic three-phase cell of Appendix B)    */
} rve_desc;

typedef struct {
  int32_t precision;     /* RVE_FP64: every step in FP64.  RVE_MIXED: FFTs, projection,
                            conjugate-gradient vectors and the tangent copy in FP32; the
                            constitutive update, F, Fp and the macroscopic averages in FP64 */
  double newton_tol;     /* stop an increment once the rms of the full Newton correction dF
                            is below this value (that correction is then applied whole)      */
  double cg_tol;         /* relative residual of the conjugate-gradient solve of eq. 18      */
  int32_t max_newton;    /* Newton iterations per increment                                  */
  int32_t max_cg;        /* CG iterations per Newton iteration                               */
  int32_t max_backtrack; /* halvings of a Newton step in the residual line search            */
  int32_t device;        /* HIP device ordinal                                               */
  void* stream;          /* hipStream_t to run on (for instance torch.cuda.current_stream());
                            NULL: the library's own stream                                   */
  int32_t use_graph;     /* 1: the conjugate-gradient iterations of eq. 18 are issued as
                            captured HIP graphs (one graph per chunk of iterations, captured
                            once per RVE and replayed); 0: kernel by kernel.  Same results.  */
  int32_t workers;       /* host threads that drive the RVEs of a handle concurrently, each
                            RVE on its own stream; 0: the default (8, or RVE_WORKERS)         */
  int32_t autotune;      /* 1: time the candidate z-pass tile widths of each grid size once
                            per process at rve_create and keep the fastest (the tile width
                            does not change any result); 0: the fixed rule                   */
  int32_t max_cutbacks;  /* automatic time-step cut-back: an increment that fails with
                            RVE_ENOCONV is replaced by two increments of dt/2 (targets
                            interpolated linearly in time), each committed, halved again up to
                            this many levels; 0 (default): no cut-back.  Changes the time
                            integration where it acts (the result equals explicit half steps) */
  int32_t max_continuation; /* load-continuation stages (1, 2, 4, ... up to this value) that the
                            FP64 path may take to solve a failed increment with the same dt and
                            the same result; 0: 16; 1: none                                   */
  int32_t frequencies;   /* 0: the rotated-scheme frequencies of Appendix A (eq. A.4), the
                            paper's method; 1: standard frequencies (the continuous derivative
                            of the trigonometric interpolant, k = xi, Nyquist derivative 0), the
                            comparison of Appendix B.  Both the projection of eq. 17 and the
                            curl of eq. 12 use the chosen scheme; the reverse pass needs 0    */
  int32_t projection;    /* form of the projection inside the conjugate-gradient iterations:
                            0: factorised where it applies (rotated scheme, plane path): the
                            operator of eq. 17 as a divergence stencil, transforms of three
                            components, 1/|k|^2 and a gradient stencil (the symbols of eq. A.4
                            are those stencils), a third of the transforms of the nine-component
                            form; 1: the nine-component form everywhere.  Same operator: the
                            results differ by rounding only                                  */
} rve_options;

/* Per-RVE statistics of one increment. */
typedef struct {
  int32_t status;            /* rve_status of this RVE                                          */
  int32_t newton_iters;      /* Newton corrections applied                                      */
  int32_t cg_iters;          /* conjugate-gradient iterations (one projected apply each)        */
  int32_t residual_evals;    /* projected residual evaluations (one projected apply each)       */
  int32_t line_search_cuts;  /* step halvings in the residual line search                       */
  int32_t local_iters_max;   /* largest local Newton iteration count of any voxel               */
  double res_norm;           /* rms of the final projected residual G(P - P_bar), Pa           */
  double dF_norm;            /* rms of the last full Newton correction                          */
  double voxel_iterations;   /* nvox * (projected applies: residual evaluations + CG iterations)
                                of the solve that produced the committed increment             */
  int32_t fp64_fallback;     /* RVE_MIXED: 1 if the FP32 attempt failed and the increment was
                                solved with the FP64 spectral path                              */
  int32_t continuation_stages; /* 0: solved directly; m: solved by load continuation in m stages
                                after the direct attempt failed                                 */
  double discarded_voxel_iterations; /* nvox * projected applies of failed attempts before the
                                committed solve (counted in newton_iters, cg_iters and
                                residual_evals, not in voxel_iterations)                       */
  int32_t cutbacks;          /* time-step halvings taken (max_cutbacks > 0): the increment was
                                committed as cutbacks + 1 sub-increments                        */
  int32_t pad;
} rve_step_stats;

/* Create a handle holding n_rve RVEs (Section 2.2).  Per grain: rotation from the
 * quaternion, slip systems s = R s0, m = R m0 (12 {111}<110>), interaction matrix q
 * (Table 1 classes), segment matrix A and its minimum-norm inverse (eq. 13).
 * State: F = Fp = I, rho_SSD = rho0, rho_GND = 0.  opt may be NULL (defaults:
 * RVE_FP64, newton_tol 1e-10, cg_tol 1e-8, max_newton 40, max_cg 2000, max_backtrack 12,
 * device 0, own stream, no graphs, 8 workers, no autotuning).  Errors: RVE_EINVAL (bad shape, grain id out of range,
 * non-finite or non-positive material constant, zero initial density), RVE_ENOMEM,
 * RVE_EDEVICE. */
int32_t rve_create(const rve_desc* descs, int32_t n_rve, const rve_options* opt, rve_handle* out);

/* Advance every RVE by one load increment of length dt (Section 2.2, eqs. 15-18):
 * mixed control with mask[9] (1 = average of F_ij prescribed by F_bar, 0 = average of
 * P_ij prescribed by P_bar); F_bar, P_bar are n_rve x 9 (host).  Solves
 * G(P(F) - P_bar) = 0 by Newton with conjugate-gradient linear solves of eq. 18 and a
 * residual line search, commits Fp and rho_SSD, then computes the Nye tensor of Fp
 * (eq. 12, Appendix B) and the GND densities (eq. 13) used by the next increment.
 * stats: n_rve entries or NULL.  Errors: RVE_EINVAL (dt <= 0, non-finite target);
 * RVE_ENOCONV if any RVE fails (its stats entry says which; no RVE is committed). */
int32_t rve_step_increment(rve_handle h, const double* F_bar, const uint8_t* mask,
                           const double* P_bar, double dt, rve_step_stats* stats);

/* Nye tensor (eq. 12; 1/m, 9 x nvox) and GND density per slip system (eq. 13;
 * 1/m^2, 12 x nvox) of the last committed increment, copied to host buffers; either
 * pointer may be NULL.  Errors: RVE_EINVAL for a bad rve index. */
int32_t rve_nye_gnd(rve_handle h, int32_t rve, double* nye, double* rho_gnd);

/* Volume averages <P>, <F> (eq. 15) of the last committed increment, accumulated in
 * FP64, and the macroscopic Cauchy stress <P><F>^T / det<F>; each a host array of 9,
 * sigma may be NULL. */
int32_t rve_macro_stress(rve_handle h, int32_t rve, double* P_avg, double* F_avg, double* sigma);

/* Adjoint of the linearised equilibrium of eq. 18 at the last converged increment: solves
 * G(K^T : lambda) = G(g) for lambda in the range of G, where K is the consistent tangent
 * dP/dF of that increment's last constitutive evaluation, (K^T)_(ij)(kl) = K_(kl)(ij), and G
 * the projection of eq. 17 with the zero-frequency rule of mask (as in rve_project).  This
 * is the first step of an increment's reverse pass (lambda is the multiplier of the
 * equilibrium constraint for a loss with dL/dF = g).  Same conjugate-gradient kernels as the
 * forward solve, with the tangent read transposed; the handle's cg_tol and max_cg apply.
 * g, lambda: device FP64, 9 x nvox (component-major, as the fields of rve_get_field);
 * lambda may alias g.  mask: host, 9 entries.  cg_iters (host, may be NULL) receives the
 * CG iteration count.  Errors: RVE_EINVAL for a bad argument, a handle that is not
 * RVE_FP64, an RVE with no increment taken yet, or a grid whose planes do not fit in LDS;
 * RVE_ENOCONV when CG ends without reaching cg_tol (breakdown, divergence, iteration cap;
 * lambda then holds the current iterate). */
int32_t rve_adjoint_solve(rve_handle h, int32_t rve, const uint8_t* mask, const double* g, double* lambda,
                          int32_t* cg_iters);

/* Reverse pass of the last committed increment k of RVE rve, for the adjoint form: the
 * implicit-function adjoint of the converged increment (Section 2.2, eqs. 16-18) through
 * the transposed consistent tangent, and the reverse of the constitutive update (Section 2.1,
 * eqs. 2-9 and 14) and of the GND chain of the start-of-increment state (eqs. 10-13, eq. 12
 * with Appendix A).  For a loss L that depends on the increment's macroscopic stress <P>_k
 * (eq. 15) and, through later increments, on its committed Fp_k and rho_SSD,k:
 *   in:  dLdP (host, 9) = dL/d<P>_k (row-major);
 *        Fp_bar (device, 9 x nvox) = dL/dFp_k, rho_bar (device, 12 x nvox) = dL/drho_SSD,k
 *        (zeros for the last increment of a curve);
 *   out: Fp_bar = dL/dFp_{k-1}, rho_bar = dL/drho_SSD,{k-1} (overwritten in place; the
 *        GND densities of increment k-1 are folded into Fp_bar through the curl), and
 *        theta_bar (host, 4) += the increment's contribution to dL/d(tau0, K, y_c, c_gnd):
 *        tau0 the initial critical stress (uniform initial SSD density (tau0/(mu b))^2 /
 *        sum_b q^{ab}, reached at k = 1, or tau_c itself when hardening is off), K of eq. 9,
 *        y_c of eq. 8 and c_gnd of eqs. 7 and 9.
 * Calling it for k = n, n-1, ..., 1 with the committed state of each increment restored
 * (rve_save_state / rve_load_state checkpoints: a checkpoint holds the start-of-increment
 * state too) accumulates the gradient of L with respect to the four parameters.
 * The converged state is re-evaluated from the start-of-increment state (slip increments,
 * stress and tangent in FP64) and the multiplier lam of G(K^T : lam) = G(g) is found by the
 * forward conjugate-gradient kernels with the tangent read transposed (FP64 spectral path;
 * mask as in rve_step_increment; cg_tol and max_cg of the handle).  Works on RVE_FP64 and
 * RVE_MIXED handles (the reverse pass always runs in FP64).  cg_iters (host, may be NULL)
 * receives the CG iteration count.  Device buffers belong to the caller and must not overlap.
 * Errors: RVE_EINVAL (bad argument, planes that do not fit in LDS), RVE_ESTATE (no committed
 * increment), RVE_ENOCONV (local Newton or CG failure); on error the outputs are undefined. */
int32_t rve_adjoint_increment(rve_handle h, int32_t rve, const uint8_t* mask, const double* dLdP, double* Fp_bar,
                              double* rho_bar, double* theta_bar, int32_t* cg_iters);

/* Copy a committed field to a host buffer: which = 0 F (9), 1 P (9), 2 Fp (9),
 * 3 rho_SSD (12), 4 rho_GND (12), 5 Nye tensor (9), 6 slip increments of the last
 * increment (12).  Component-major, nvox per component. */
int32_t rve_get_field(rve_handle h, int32_t rve, int32_t which, double* out);

/* Save / restore the committed state of every RVE (F, Fp, rho_SSD, rho_GND, Nye, slip
 * increments, P, the previous increment's F, and the start-of-increment Fp, rho_SSD, rho_GND
 * and time step of the last increment) byte-exactly.  rve_state_bytes gives the size of the
 * host buffer. */
int64_t rve_state_bytes(rve_handle h);
int32_t rve_save_state(rve_handle h, void* buf);
int32_t rve_load_state(rve_handle h, const void* buf);

/* ---- Measurement support ----
 * Kernel families whose launches can be timed; bit f of a mask selects family f. */
enum {
  RVE_KF_SLIP_FAST = 0,      /* local Newton on the slip increments, first pass (eqs. 5-6)       */
  RVE_KF_SLIP_SLOW = 1,      /* continuation pass over the voxels the first pass left            */
  RVE_KF_STRESS_TANGENT = 2, /* stress (eq. 14) and consistent tangent dP/dF                      */
  RVE_KF_CG_PREP = 3,        /* CG vector update, r.r and K : r (eq. 18)                          */
  RVE_KF_PLANE_FWD = 4,      /* x and y forward FFTs of one component plane                      */
  RVE_KF_MID = 5,            /* z FFTs and the Green operator of eq. 17 with its inverse z FFTs  */
  RVE_KF_PLANE_INV = 6,      /* y and x inverse FFTs and the CG epilogue                          */
  RVE_KF_CG_GRAD = 7,        /* gradient stencil of the factorised projection and the CG epilogue */
  RVE_KF_PLANE_DIV = 8,      /* divergence stencil and x and y forward FFTs (factorised form)     */
  RVE_KF_MID3 = 9,           /* z FFTs and 1/|k|^2 on three components (factorised form)          */
  RVE_KF_PLANE_W = 10        /* y and x inverse FFTs of three components (factorised form)        */
};

/* While mask != 0, every launch of the selected families during rve_step_increment
 * carries a pair of HIP events that the dispatch records at the kernel's start and end
 * (AMD's extended launch, on the stream it is launched on); the kernel durations are
 * accumulated per family.  Launches that a finished CG solve turns into no-ops are not
 * counted.  Each call clears the accumulators; mask 0 stops timing.
 * Errors: RVE_EINVAL (unknown family bit). */
int32_t rve_timing_start(rve_handle h, uint32_t mask);

/* Accumulated figures of one family since the last rve_timing_start, summed over the
 * handle's RVEs: launches, total event-measured duration in ms, and units: the
 * algorithmic bytes of those launches for the spectral families (every input read once,
 * every output written once) or the voxels covered for the constitutive families.  Any
 * output pointer may be NULL.  Errors: RVE_EINVAL (unknown family). */
int32_t rve_timing_read(rve_handle h, int32_t family, int64_t* launches, double* total_ms, double* units);

void rve_destroy(rve_handle h);

/* Message of the last failing call on this thread ("" if none). */
const char* rve_last_error(void);

/* ---- Kernel-level entry points (device pointers; used by tests and benchmarks) ---- */

/* Constitutive update (Section 2.1, eqs. 1-9, 14) of nvox independent material points
 * on the device.  Inputs (device, component-major): gid (nvox int32), F (9), Fp_n (9),
 * rho_ssd_n (12), rho_gnd_n (12); dg (12) holds the starting slip increments and
 * receives the converged ones.  Outputs (device): P (9, FP64), K (81 = dP_ij/dF_kl at
 * index (3i+j)*9 + (3k+l), FP64; NULL to skip), local iteration count per voxel (int32;
 * negative if that voxel did not converge; may be NULL).  Grain rotations come from
 * n_grains host quaternions.  stream: hipStream_t or NULL. */
int32_t rve_constitutive_batch(const rve_material* mat, int32_t n_grains, const double* grain_quat,
                               int64_t nvox, const int32_t* gid, const double* F,
                               const double* Fp_n, const double* rho_ssd_n,
                               const double* rho_gnd_n, double dt, double* dg, double* P,
                               double* K, int32_t* iters, void* stream);

/* Sensitivity of the converged stress to the critical resolved shear stresses, for the
 * adjoint form: dPdtc[(9c + r) * nvox + v] = dP_r / dtau_c,c (device out, 108 x nvox, FP64,
 * sample frame), where r = 3i + j indexes P_ij.  tau_c (eq. 7) is held fixed over an increment,
 * so the slip increments dg (device, 12 x nvox) must be the converged ones that
 * rve_constitutive_batch returned for the same inputs; the root then moves by the implicit
 * function theorem through the flow rule (eq. 6) and the stress follows through Fp (eqs. 2,
 * 14).  Other arguments as for rve_constitutive_batch.  Gradients of a loss with respect to
 * the hardening parameters follow by the chain rule through tau_c (eq. 7).  Errors: RVE_EINVAL
 * for a null pointer or dt <= 0. */
int32_t rve_stress_sensitivity(const rve_material* mat, int32_t n_grains, const double* grain_quat,
                               int64_t nvox, const int32_t* gid, const double* F, const double* Fp_n,
                               const double* rho_ssd_n, const double* rho_gnd_n, double dt,
                               const double* dg, double* dPdtc, void* stream);

/* Transposed application of the stress sensitivity, for the adjoint form: tau_c_bar[c * nvox +
 * v] = sum_r w[r * nvox + v] dP_r / dtau_c,c (device out, 12 x nvox) for an adjoint field w
 * (device, 9 x nvox, sample frame), without forming the 108 entries per voxel.  w and
 * tau_c_bar must not overlap.  Other arguments and errors as for rve_stress_sensitivity. */
int32_t rve_stress_sensitivity_vjp(const rve_material* mat, int32_t n_grains, const double* grain_quat,
                                   int64_t nvox, const int32_t* gid, const double* F,
                                   const double* Fp_n, const double* rho_ssd_n,
                                   const double* rho_gnd_n, double dt, const double* dg,
                                   const double* w, double* tau_c_bar, void* stream);

/* Sensitivity of the SSD density update (eqs. 8-9) to its parameters, for the adjoint form:
 * out[a * nvox + v] = d rho_SSD,a / dK and out[(12 + a) * nvox + v] = d rho_SSD,a / dy_c
 * (device out, 24 x nvox, FP64) at fixed slip increments dg (device, 12 x nvox), from the
 * start-of-increment densities rho_ssd_n, rho_gnd_n (device, 12 x nvox each).  K and y_c do not
 * reach the slip solve of the same increment (tau_c uses the start-of-increment densities),
 * so these are the whole derivatives of the committed densities.  Zero for a material without
 * hardening.  Errors: RVE_EINVAL for a null pointer, nvox < 1 or an invalid material. */
int32_t rve_density_sensitivity(const rve_material* mat, int64_t nvox, const double* rho_ssd_n,
                                const double* rho_gnd_n, const double* dg, double* out, void* stream);

/* Projection G of eq. 17 applied to a real FP64 field A (device, 9 x nvox, grid n) with
 * the mixed-control zero-frequency rule of mask (host, 9) and target dc_target (host, 9;
 * NULL = 0); result in out (device, 9 x nvox).  precision selects FP64 or FP32 spectra. */
int32_t rve_project(const int32_t n[3], int32_t precision, const double* A, const uint8_t* mask,
                    const double* dc_target, double* out, void* stream);

/* rve_project for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same projection with
 * the same kernels, but the half spectrum and the root tables live in one fixed device array
 * of the library, 64 MiB per device, held from the first call on a device until the process
 * ends.  The call allocates nothing: it fills the root tables and runs the projection on
 * stream (or the null stream) and returns once the work is queued (no synchronisation).
 * Limit: the spectrum, 9 x (n0/2 + 1) x n1 x n2 complex values of 16 bytes (RVE_FP64) or 8
 * bytes (RVE_MIXED), must fit in 64 MiB - 64 KiB (for instance 96^3 in FP64, 112^3 in FP32);
 * a larger grid is rejected with RVE_EINVAL before any device work.  Every call on a device
 * shares that device's array and leaves its contents behind: calls that overlap in time on
 * one device (different streams or threads) race and must be serialised by the caller.
 * Arguments, layouts and other errors as for rve_project. */
int32_t rve_project_noalloc(const int32_t n[3], int32_t precision, const double* A, const uint8_t* mask,
                            const double* dc_target, double* out, void* stream);

/* Nye tensor alpha_ij = eps_jml d_m Fp_il (eq. 12 with the rotated-scheme derivative of
 * Appendix A and voxel size h; device in/out, 9 x nvox) and, when gid/grain_quat are
 * given, the GND densities per slip system (eq. 13; device out, 12 x nvox). */
int32_t rve_spectral_curl(const int32_t n[3], int32_t precision, double h, const double* Fp,
                          double* nye, const int32_t* gid, int32_t n_grains,
                          const double* grain_quat, double burgers, double* rho_gnd, void* stream);

/* Reverse of the chain Fp -> Nye tensor -> GND densities (eqs. 10-13 and eq. 12 with the
 * rotated-scheme derivative of Appendix A) for the adjoint form: given rho_bar = dL/d rho_GND
 * (device, 12 x nvox), writes Fp_bar = dL/d Fp (device, 9 x nvox) and, when nye_bar is not
 * NULL, nye_bar = dL/d alpha (device, 9 x nvox).  nye is the Nye tensor at which the chain is
 * linearised (device, 9 x nvox, as written by rve_spectral_curl); the absolute values of the
 * per-system densities take the sign of each segment density (0 at a zero density).  gid
 * (device, nvox) holds grain ids in [0, n_grains); grain_quat (host, 4 x n_grains) the grain
 * orientations; burgers > 0 and h > 0 as for rve_spectral_curl; n (x, y, z sizes) and
 * precision (RVE_FP64, or RVE_MIXED for FP32 spectra) as for rve_project.  All device buffers
 * belong to the caller and must not overlap.  The call allocates its own scratch, runs on stream
 * (or the null stream) and returns after the stream has finished.  RVE_EINVAL for a null
 * pointer, a non-positive h, burgers or n_grains, or an unsupported grid size. */
int32_t rve_gnd_adjoint(const int32_t n[3], int32_t precision, double h, const double* nye,
                        const int32_t* gid, int32_t n_grains, const double* grain_quat, double burgers,
                        const double* rho_bar, double* nye_bar, double* Fp_bar, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* RVE_H */
