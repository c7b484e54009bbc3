// Launchers of the adjoint form: the reverse of the Nye tensor / GND chain (eqs. 10-13,
// eq. B.3) and the stress sensitivity to the critical resolved shear stresses (eqs. 6, 7, 14).
#ifndef RVE_ADJOINT_H
#define RVE_ADJOINT_H

#include "kernels.h"

namespace rve {

// alpha_bar (9 x nv, component-major) = (d rho_GND / d alpha)^T rho_bar (12 x nv) at the
// Nye tensor nye (9 x nv); grain rotations grainR (9 per grain, sample <- crystal).
void launch_gnd_adjoint(int64_t nv, const double* nye, const int32_t* gid, const double* grainR,
                        const MatDev* mat, const double* rho_bar, double* alpha_bar, hipStream_t st);

// dPdtc (9 x 12 per voxel, sample frame, index (9c + r) * nvox + v) = dP_r / dtau_c,c at the
// slip increments a.dg (constitutive.hip); with w (9 x nvox) not null, dPdtc (12 x nvox) =
// sum_r w_r dP_r / dtau_c,c instead.
void launch_stress_sensitivity(const ConstArgs& a, double* dPdtc, const double* w, hipStream_t st);

// out (24 x nv): d rho_SSD,a / dK (row a) and d rho_SSD,a / dy_c (row 12 + a) of eqs. 8-9 at
// fixed slip increments dg (12 x nv), from the start-of-increment densities.
void launch_density_sensitivity(int64_t nv, const MatDev* mat, const double* rho_ssd, const double* rho_gnd,
                                const double* dg, double* out, hipStream_t st);

// Output weights and results of the reverse constitutive update (k_constitutive_adjoint).
struct AdjointLocalArgs {
  double wP[9];            // uniform part of the stress weight P_bar (sample frame)
  const double* lam;       // field subtracted from it (9 x nv, sample frame), may be null
  const double* Fp_bar;    // weight of the committed Fp (9 x nv, sample frame), may be null
  const double* rho_bar;   // weight of the committed rho_SSD (12 x nv), may be null
  double* g;               // mode 0: dL/dF at fixed start state (9 x nv, sample frame)
  double* Fp_bar_out;      // mode 1: dL/dFp_n (9 x nv; may alias Fp_bar)
  double* rho_bar_out;     // mode 1: dL/drho_SSD,n (12 x nv; may alias rho_bar)
  double* rho_gnd_bar;     // mode 1: dL/drho_GND,n (12 x nv)
  double* theta_partial;   // mode 1: per block sums of dL/dK, dL/dy_c, dL/dc_gnd, dL/dtau0 (4 each)
  int mode;                // 0 or 1
};

// Reverse of the constitutive update at the converged slip increments a.dg (constitutive.hip);
// a.F is the converged F, a.Fp_n, a.rho_ssd, a.rho_gnd the start-of-increment state.  Returns
// the number of blocks (4 theta partials each in mode 1).
int launch_constitutive_adjoint(const ConstArgs& a, const AdjointLocalArgs& b, hipStream_t st);

// out(c, z, y, x) = in(c, z - 1, y - 1, x - 1) with periodic wrap, 9 components (added to out
// when accumulate).
void launch_roll_back(int nx, int ny, int nz, const double* in, double* out, hipStream_t st,
                      bool accumulate = false);

}  // namespace rve

#endif
