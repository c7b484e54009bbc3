// Kernel argument structures and launchers shared by the kernel files and the runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "timing.h"

namespace rve {

// Material constants of one RVE, device resident (read through the scalar cache).
struct MatDev {
  double C11, C12, C44;
  double mu, burgers, y_c, K_sim;
  double gamma0_dot, n_exp;      // n_exp = 1 / m
  double c_gnd, tau_c_frozen;
  int32_t hardening, pad;
  double q[144];                 // interaction matrix, row-major
  double Aplus[18 * 9];          // minimum-norm inverse of the segment matrix (eq. 13)
  int32_t screw_of[12];          // screw segment sharing the Burgers vector of each system
};

// The SSD density update (eq. 8) integrated exactly over one increment's slip u = |dg| with
// the mean free path (eq. 9) frozen at its start-of-increment value:
//   rho = rho_n exp(-x) + u phi(x) / (b l),  x = 2 y_c u / b,  phi(x) = (1 - exp(-x)) / x,
// i.e. rho_n + h u phi(x) with h = (1/b)(1/l - 2 y_c rho_n) the forward-Euler rate.
__device__ __forceinline__ double ssd_phi(double x) { return x > 0.0 ? -expm1(-x) / x : 1.0; }
// phi'(x) = (exp(-x)(1 + x) - 1) / x^2; below x = 0.01 its Taylor series (the closed form
// cancels there)
__device__ __forceinline__ double ssd_dphi(double x) {
  if (x < 0.01)
    return -0.5 + x * (1.0 / 3.0 + x * (-1.0 / 8.0 + x * (1.0 / 30.0 + x * (-1.0 / 144.0 + x * (1.0 / 840.0)))));
  return (exp(-x) * (1.0 + x) - 1.0) / (x * x);
}

struct ConstArgs {
  int64_t nvox;
  const int32_t* gid;
  const double* grainR;          // 9 per grain, crystal -> sample
  const double* grainC;          // C11, C12, C44 per grain, or null: the material's (MatDev)
  const MatDev* mat;
  const double* F;               // evaluated at F + lam * dF (dF may be null)
  const double* dF;              // FP64 correction field, may be null
  double lam;
  double* F_out;                 // optional copy of the evaluated F
  const double* Fp_n;
  const double* rho_ssd;
  const double* rho_gnd;
  double* dg;                    // in: warm start, out: converged slip increments
  double* P;
  void* K;                       // crystal-frame tangent (double or float), may be null
  double dt;
  int32_t* stats;                // device {max local iterations, failures, work-list length, -}
  int32_t* work;                 // device work list, nvox entries
  int32_t* iters;                // per voxel local iterations (negative: failed), may be null
  float* dgdF;                   // d(dg)/dF_c at the converged state, 12 x 9 per voxel (crystal
                                 // frame, index (9a + 3k + l) * nvox + v); written with K, may be null
  double lam_base;               // dg (and dgdF) were computed at F + lam_base * dF
  int32_t predict;               // 1: the first pass starts from dg + (lam - lam_base) dgdF : dF_c
  int32_t k_grouped;             // K layout: 0 entry-major (e * nvox + v), 1 grouped (see tangent_index)
  double k_inv_scale;            // FP16 K only: entries are stored as dP/dF times this factor
};

// Storage type of the tangent copy: FP64, FP32, or FP16 pairs scaled by 1/C11 (entries
// of order one; FP16 rounding, 2^-11 relative, perturbs only the Jacobian that the linear
// solve inverts, not the residual, so it changes the Newton path and not the solution).
enum TangentType : int { KT_F64 = 0, KT_F32 = 1, KT_F16 = 2 };

// Layout of the tangent copy used by the conjugate-gradient kernels.  FP64 and FP16: the
// 81 entries of a voxel in groups of W consecutive entries, group-major over voxels, so that
// one lane reads W entries with one vector load while a wavefront still reads contiguous
// memory (fewer memory instructions in flight per voxel).  FP64: W = 2 (16-byte loads, the
// last group padded); FP16: W = 8 (16-byte loads) over entries 0-79, then entry 80 alone
// (2 bytes per voxel, no padding); FP32: entry-major (W = 1); wider groups there cost more
// registers and occupancy than they gain.
template <typename KT>
struct TangentGroups {
  static constexpr int W = sizeof(KT) == 4 ? 1 : (sizeof(KT) == 2 ? 8 : 2);
  static constexpr int G = (81 + W - 1) / W;                          // groups per voxel
  static constexpr int kStored = sizeof(KT) == 2 ? 81 : G * W;       // entries stored per voxel
};
template <typename KT>
__host__ __device__ __forceinline__ int64_t tangent_index(int e, int64_t v, int64_t nv, bool grouped) {
  constexpr int W = TangentGroups<KT>::W;
  if (!grouped) return (int64_t)e * nv + v;
  if (sizeof(KT) == 2 && e >= 80) return 80 * nv + v;                // FP16 tail entry
  return ((int64_t)(e / W) * nv + v) * W + (e % W);
}

struct CommitArgs {
  int64_t nvox;
  const int32_t* gid;
  const double* grainR;
  const MatDev* mat;
  const double* dg;
  double* Fp;                    // in: Fp_n, out: Fp
  double* rho_ssd;               // in: rho_SSD,n, out: rho_SSD
  const double* rho_gnd;
};

// ktype: storage type of K (TangentType).  dF, when given, is an FP64 field.
void launch_constitutive(const ConstArgs& a, int ktype, hipStream_t st, LaunchTimer* timer = nullptr);
void launch_commit(const CommitArgs& a, hipStream_t st);
void launch_rotate_tangent(int64_t nv, const int32_t* gid, const double* grainR, const double* Kc, double* Ks,
                           hipStream_t st);

}  // namespace rve
