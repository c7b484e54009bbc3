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

// out(c, z, y, x) = in(c, z - 1, y - 1, x - 1) with periodic wrap, 9 components.
void launch_roll_back(int nx, int ny, int nz, const double* in, double* out, hipStream_t st);

}  // namespace rve

#endif
