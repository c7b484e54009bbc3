// Adjoint form.  Reverse of the chain Fp -> alpha -> rho_GND (eqs. 10-13 and the curl of
// eq. B.3): given rho_bar = dL/d rho_GND, produce dL/d alpha and dL/d Fp.  And the
// sensitivity of the SSD density update (eqs. 8-9) to its parameters K and y_c.
//
//   k_gnd_adjoint   per voxel: alpha_c = R^T alpha R, segment densities rho = A^+ alpha_c / b,
//                   u = sign(rho) * (system weights: 1 for the edge segment of each system,
//                   1/2 for its screw segment, summed over the two systems sharing it),
//                   alpha_bar = R ((A^+)^T u / b) R^T.  sign(0) = 0.
//   curl transpose  the rotated-scheme derivative i k / h is a difference at the voxel corner
//                   x + h/2 (1,1,1); its transpose has the symbol conj(i k / h) and, since
//                   conj(k) = k exp(-i (xi_x + xi_y + xi_z)), the transposed curl equals the
//                   curl itself taken one voxel back along every axis.  The spectral curl
//                   kernels are reused unchanged and k_roll_back applies the shift.
#include "adjoint.h"

#include "common.h"

namespace rve {

namespace {

__device__ __forceinline__ double sgn(double x) { return (double)((x > 0.0) - (x < 0.0)); }

__global__ void k_gnd_adjoint(int64_t nv, const double* nye, const int32_t* gid, const double* grainR,
                              const MatDev* mat, const double* rho_bar, double* alpha_bar) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  const MatDev& M = *mat;
  double q[9], Rg[9], ac[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) q[c] = nye[c * nv + v];
  const int gi = gid[v];
#pragma unroll
  for (int i = 0; i < 9; ++i) Rg[i] = grainR[9 * gi + i];
  to_crystal(Rg, q, ac);
  double u[18];
#pragma unroll
  for (int s = 12; s < 18; ++s) u[s] = 0.0;
#pragma unroll
  for (int a = 0; a < 12; ++a) {
    const double rb = rho_bar[a * nv + v];
    const int k = M.screw_of[a];
    u[a] = rb;
    // static register indices: the screw segment is selected, not indexed
#pragma unroll
    for (int s = 0; s < 6; ++s) u[12 + s] += k == s ? 0.5 * rb : 0.0;
  }
  const double ib = 1.0 / M.burgers;
#pragma unroll
  for (int s = 0; s < 18; ++s) {
    double t = 0.0;
#pragma unroll
    for (int c = 0; c < 9; ++c) t += M.Aplus[s * 9 + c] * ac[c];
    u[s] *= sgn(t) * ib;
  }
  double cb[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) {
    double t = 0.0;
#pragma unroll
    for (int s = 0; s < 18; ++s) t += M.Aplus[s * 9 + c] * u[s];
    cb[c] = t;
  }
  to_sample(Rg, cb, q);
#pragma unroll
  for (int c = 0; c < 9; ++c) alpha_bar[c * nv + v] = q[c];
}

__global__ void k_roll_back(int nx, int ny, int nz, const double* in, double* out, int accumulate) {
  const int64_t plane = (int64_t)nx * ny, nv = plane * nz;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 9 * nv) return;
  const int64_t c = i / nv, r = i - c * nv;
  const int z = (int)(r / plane);
  const int64_t t = r - z * plane;
  const int y = (int)(t / nx), x = (int)(t - (int64_t)y * nx);
  const int zs = z == 0 ? nz - 1 : z - 1, ys = y == 0 ? ny - 1 : y - 1, xs = x == 0 ? nx - 1 : x - 1;
  const double val = in[c * nv + zs * plane + (int64_t)ys * nx + xs];
  out[i] = accumulate ? out[i] + val : val;
}

// Sensitivity of the committed SSD densities (eqs. 8-9) to the similitude coefficient K and
// the annihilation distance y_c at fixed slip increments: with S_a = sum_{b != a} (rho_SSD,b +
// c_gnd rho_GND,b), u = |dg_a|, x = 2 y_c u / b and the update
// rho_a = rho_SSD,a exp(-x) + u phi(x) sqrt(S_a) / (b K) (ssd_phi),
//   d rho_a / dK = -u phi(x) sqrt(S_a) / (b K^2),
//   d rho_a / dy_c = (2 u / b)(-rho_SSD,a exp(-x) + u sqrt(S_a) phi'(x) / (b K)).
// Rows a (K) and 12 + a (y_c) of out; zero without hardening (the densities do not evolve).
__global__ void k_density_sensitivity(int64_t nv, const MatDev* mat, const double* rho_ssd, const double* rho_gnd,
                                      const double* dg, double* out) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  const MatDev& M = *mat;
  double rs[12], forest[12], tot = 0.0;
#pragma unroll
  for (int a = 0; a < 12; ++a) {
    rs[a] = rho_ssd[a * nv + v];
    forest[a] = rs[a] + M.c_gnd * rho_gnd[a * nv + v];
    tot += forest[a];
  }
  const double ib = 1.0 / M.burgers;
#pragma unroll
  for (int a = 0; a < 12; ++a) {
    const double u = M.hardening ? fabs(dg[a * nv + v]) : 0.0;
    const double x = 2.0 * M.y_c * u * ib, sq = sqrt(tot - forest[a]);
    out[a * nv + v] = -u * ib * ssd_phi(x) * sq / (M.K_sim * M.K_sim);
    out[(12 + a) * nv + v] = 2.0 * u * ib * (-rs[a] * exp(-x) + u * sq * ssd_dphi(x) * ib / M.K_sim);
  }
}

}  // namespace

void launch_gnd_adjoint(int64_t nv, const double* nye, const int32_t* gid, const double* grainR,
                        const MatDev* mat, const double* rho_bar, double* alpha_bar, hipStream_t st) {
  const int bs = 128;
  hipLaunchKernelGGL(k_gnd_adjoint, dim3((unsigned)((nv + bs - 1) / bs)), dim3(bs), 0, st, nv, nye, gid, grainR,
                     mat, rho_bar, alpha_bar);
}

void launch_density_sensitivity(int64_t nv, const MatDev* mat, const double* rho_ssd, const double* rho_gnd,
                                const double* dg, double* out, hipStream_t st) {
  const int bs = 128;
  hipLaunchKernelGGL(k_density_sensitivity, dim3((unsigned)((nv + bs - 1) / bs)), dim3(bs), 0, st, nv, mat, rho_ssd,
                     rho_gnd, dg, out);
}

void launch_roll_back(int nx, int ny, int nz, const double* in, double* out, hipStream_t st, bool accumulate) {
  const int bs = 256;
  const int64_t n = 9 * (int64_t)nx * ny * nz;
  hipLaunchKernelGGL(k_roll_back, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, st, nx, ny, nz, in, out,
                     accumulate ? 1 : 0);
}

}  // namespace rve
