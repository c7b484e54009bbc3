// Constitutive update of the strain-gradient crystal-plasticity model (Section 2.1,
// eqs. 1-9 and 14), one voxel per lane, FP64.
//
// Frames.  A grain with rotation R (crystal -> sample) has slip systems s = R s0,
// m = R m0 and stiffness C = R*R*C0*R*R.  The update is rotation-equivariant, so it is
// evaluated in the crystal frame: F_c = R^T F R, Fp_c = R^T Fp R, with the fixed FCC slip
// systems and the cubic stiffness as compile-time constants, and P = R P_c R^T.  The
// tangent is stored in the crystal frame: K_c[(3i+j)*9 + (3k+l)] = dP_c,ij / dF_c,kl.
//
// Time integration over an increment dt (backward Euler in the slip increments dg):
//   Fp = A Fp_n,  A = I + sum_a dg_a s_a (x) m_a                        (eq. 2)
//   Fe = F Fp^{-1},  Ee = (Fe^T Fe - I)/2,  S = C : Ee,  tau_a = S : (s_a (x) m_a)   (1, 3-5)
//   R_a(dg) = dg_a - dt gdot0 (|tau_a| / tau_c,a)^n sgn(tau_a),  n = 1/m     (eq. 6)
//   tau_c,a = mu b sqrt(sum_b q_ab (rho_SSD,b + c_gnd rho_GND,b)) from the densities at
//   the start of the increment (eq. 7); the densities advance after the increment (eq. 8).
//   P = F Fp^{-1} S Fp^{-T}  (= Fe S Fe^T F^{-T}, eq. 14).
//
// Local solve.  Newton on R(dg) = 0 with the analytic Jacobian
//   J_ab = delta_ab + D_a (u_b . Chat_a w_b),  D_a = d g_a / d tau_a,
//   u_b = Ce s_b, w_b = A^{-T} m_b, Chat_a = C : sym(s_a (x) m_a),
// whose non-identity part has rank at most six: each solve with J runs as a 6x6
// elimination on symmetric tensors (rank6_build below); steps are capped at 0.02 in the
// max norm and backtracked on |R|.  If 12 Newton steps at the final
// exponent do not converge from the warm start, the lane restarts with continuation in
// the exponent (roots at n = 1, 2, 4, 8, 16, then n = 1/m): far from the solution the
// Jacobian rows of overloaded systems carry (|tau|/tau_c)^(n-1) and J becomes
// numerically singular; each continuation stage starts close to its own root.
//
// Tangent.  With the converged J (through the same 6x6 form), for each unit direction
// dF = e_k (x) e_l:
//   dtau_a = Fe_k. Chat_a G_l.  (G = Fp^{-1}),  ddg = J^{-1} (D dtau),  Z = sum_b ddg_b s_b (x) m_b,
//   dEe = sym(Fe_k. (x) G_l.) - sym(Ce Z A^{-1}),  dS = C : dEe,
//   dP = e_k (x) (G S G^T)_l. - Fe Z A^{-1} S G^T + Fe dS G^T - Fe S A^{-T} Z^T G^T.
#include "adjoint.h"
#include "common.h"
#include "kernels.h"

#include <hip/hip_fp16.h>

#include <algorithm>

namespace rve {

namespace {

__device__ __forceinline__ double ipow(double r, int k) {
  double res = 1.0, b = r;
  while (k) {
    if (k & 1) res *= b;
    b *= b;
    k >>= 1;
  }
  return res;
}

__device__ __forceinline__ double powr(double r, double n) {
  if (r == 0.0) return n == 0.0 ? 1.0 : 0.0;
  if (n == floor(n) && n >= 0.0 && n <= 64.0) return ipow(r, (int)n);
  return pow(r, n);
}

struct Point {
  double Fe0[9];   // F_c Fp_n,c^{-1}
  double Gn[9];    // Fp_n,c^{-1}
  double tc[12];
  double a;        // dt * gdot0
  double C11, C12, C44;
};

__device__ __forceinline__ void cubic_stress(const Point& p, const double* E, double* S) {
  const double tr = E[0] + E[4] + E[8];
  const double d = p.C11 - p.C12;
  S[0] = p.C12 * tr + d * E[0];
  S[4] = p.C12 * tr + d * E[4];
  S[8] = p.C12 * tr + d * E[8];
  S[1] = S[3] = 2.0 * p.C44 * E[1];
  S[2] = S[6] = 2.0 * p.C44 * E[2];
  S[5] = S[7] = 2.0 * p.C44 * E[5];
}

// u^T Chat_a w for the cubic stiffness: Chat_a = 2 C44 sym(s m) + (C11-C12-2C44) diag(s_i m_i)
__device__ __forceinline__ double uCw(const Point& p, int a, const double* u, const double* w) {
  const double us = u[0] * kSlipS[a][0] + u[1] * kSlipS[a][1] + u[2] * kSlipS[a][2];
  const double um = u[0] * kSlipM[a][0] + u[1] * kSlipM[a][1] + u[2] * kSlipM[a][2];
  const double ws = w[0] * kSlipS[a][0] + w[1] * kSlipS[a][1] + w[2] * kSlipS[a][2];
  const double wm = w[0] * kSlipM[a][0] + w[1] * kSlipM[a][1] + w[2] * kSlipM[a][2];
  const double dd = u[0] * w[0] * kSlipS[a][0] * kSlipM[a][0] + u[1] * w[1] * kSlipS[a][1] * kSlipM[a][1] +
                    u[2] * w[2] * kSlipS[a][2] * kSlipM[a][2];
  return p.C44 * (us * wm + um * ws) + (p.C11 - p.C12 - 2.0 * p.C44) * dd;
}

struct Kin {
  double A[9], Ainv[9], Fe[9], Ce[9], S[9], tau[12];
};

__device__ __forceinline__ void kinematics(const Point& p, const double* dg, Kin& k) {
#pragma unroll
  for (int i = 0; i < 9; ++i) k.A[i] = (i % 4 == 0) ? 1.0 : 0.0;
#pragma unroll
  for (int a = 0; a < 12; ++a)
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) k.A[3 * i + j] += dg[a] * kSlipS[a][i] * kSlipM[a][j];
  inv3(k.A, k.Ainv);
  mm3(p.Fe0, k.Ainv, k.Fe);
  mtm3(k.Fe, k.Fe, k.Ce);
  double E[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) E[i] = 0.5 * (k.Ce[i] - ((i % 4 == 0) ? 1.0 : 0.0));
  cubic_stress(p, E, k.S);
#pragma unroll
  for (int a = 0; a < 12; ++a) {
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) t += kSlipS[a][i] * k.S[3 * i + j] * kSlipM[a][j];
    k.tau[a] = t;
  }
}

// R = dg - g(tau); returns |R|^2.  D (may be null) receives d g_a / d tau_a.
__device__ __forceinline__ double residual(const Point& p, double n, const double* dg, Kin& k, double* R,
                                           double* D) {
  kinematics(p, dg, k);
  double r2 = 0.0;
#pragma unroll
  for (int a = 0; a < 12; ++a) {
    const double ratio = fabs(k.tau[a]) / p.tc[a];
    const double rn1 = powr(ratio, n - 1.0);
    const double g = p.a * rn1 * ratio * ((k.tau[a] > 0.0) ? 1.0 : ((k.tau[a] < 0.0) ? -1.0 : 0.0));
    R[a] = dg[a] - g;
    r2 += R[a] * R[a];
    if (D) D[a] = p.a * n * rn1 / p.tc[a];
  }
  return r2;
}

__device__ __forceinline__ void jacobian(const Point& p, const Kin& k, const double* D, double J[12][12]) {
#pragma unroll
  for (int b = 0; b < 12; ++b) {
    double u[3], w[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      u[i] = k.Ce[3 * i] * kSlipS[b][0] + k.Ce[3 * i + 1] * kSlipS[b][1] + k.Ce[3 * i + 2] * kSlipS[b][2];
      w[i] = k.Ainv[i] * kSlipM[b][0] + k.Ainv[3 + i] * kSlipM[b][1] + k.Ainv[6 + i] * kSlipM[b][2];
    }
#pragma unroll
    for (int a = 0; a < 12; ++a) J[a][b] = ((a == b) ? 1.0 : 0.0) + D[a] * uCw(p, a, u, w);
  }
}

__device__ __forceinline__ void lu12(double J[12][12]) {
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    const double ip = 1.0 / J[c][c];
#pragma unroll
    for (int r = c + 1; r < 12; ++r) {
      const double f = J[r][c] * ip;
      J[r][c] = f;
#pragma unroll
      for (int cc = c + 1; cc < 12; ++cc) J[r][cc] -= f * J[c][cc];
    }
  }
}

__device__ __forceinline__ void lu12_solve(const double J[12][12], double* x) {
#pragma unroll
  for (int r = 1; r < 12; ++r)
#pragma unroll
    for (int c = 0; c < r; ++c) x[r] -= J[r][c] * x[c];
#pragma unroll
  for (int r = 11; r >= 0; --r) {
#pragma unroll
    for (int c = r + 1; c < 12; ++c) x[r] -= J[r][c] * x[c];
    x[r] /= J[r][r];
  }
}

// Rank-six form of the same Jacobian.  With P_a = sym(s_a (x) m_a) and Chat_a = C : P_a,
//   J = I + D H^T W,   (H^T X)_a = Chat_a : X,   W x = sum_b x_b sym(u_b (x) w_b),
// so J has the identity plus a part of rank at most six (symmetric tensors), and the
// Sherman-Morrison-Woodbury identity turns every solve with J into one with the 6x6 operator
//   N = C^{-1} + G,   G T = sum_a D_a sym(u_a (x) w_a) (P_a : T):
//   J d = -R   <=>   N T = W R,  d_a = -R_a + D_a P_a : T
//   J x = D H^T E (E symmetric)   <=>   N T = E,  x_a = D_a P_a : T.
// Symmetric tensors are held as (11, 22, 33, 23, 13, 12) components; with the weights
// omega = (1, 1, 1, 2, 2, 2) of the double contraction, the rows of N are scaled by omega,
// which makes the stored matrix symmetric where sym(u_a (x) w_a) = P_a (Ce = A = I) and
// positive definite there (compliance plus a Gram matrix with D >= 0), so it is eliminated
// without pivoting like the 12x12 form.
__device__ constexpr int kVi[6] = {0, 1, 2, 1, 0, 0};
__device__ constexpr int kVj[6] = {0, 1, 2, 2, 2, 1};

// omega-weighted component l of P_a
__device__ __forceinline__ double pw(int a, int l) {
  const int i = kVi[l], j = kVj[l];
  return (l < 3) ? kSlipS[a][i] * kSlipM[a][i] : kSlipS[a][i] * kSlipM[a][j] + kSlipS[a][j] * kSlipM[a][i];
}

// N (row-scaled by omega) and, when R is given, y = omega * (W R).
__device__ __forceinline__ void rank6_build(const Point& p, const Kin& k, const double* D, const double* R,
                                            double N[6][6], double* y) {
  const double det = (p.C11 - p.C12) * (p.C11 + 2.0 * p.C12);
  const double s11 = (p.C11 + p.C12) / det, s12 = -p.C12 / det, s44 = 1.0 / p.C44;
#pragma unroll
  for (int r = 0; r < 6; ++r) {
    if (R) y[r] = 0.0;
#pragma unroll
    for (int c = 0; c < 6; ++c)
      N[r][c] = (r < 3 && c < 3) ? ((r == c) ? s11 : s12) : ((r == c) ? s44 : 0.0);
  }
#pragma unroll
  for (int b = 0; b < 12; ++b) {
    double u[3], w[3], wv[6];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      u[i] = k.Ce[3 * i] * kSlipS[b][0] + k.Ce[3 * i + 1] * kSlipS[b][1] + k.Ce[3 * i + 2] * kSlipS[b][2];
      w[i] = k.Ainv[i] * kSlipM[b][0] + k.Ainv[3 + i] * kSlipM[b][1] + k.Ainv[6 + i] * kSlipM[b][2];
    }
#pragma unroll
    for (int l = 0; l < 6; ++l)
      wv[l] = (l < 3) ? u[kVi[l]] * w[kVi[l]] : u[kVi[l]] * w[kVj[l]] + u[kVj[l]] * w[kVi[l]];
#pragma unroll
    for (int r = 0; r < 6; ++r) {
      if (R) y[r] += R[b] * wv[r];
      const double dw = D[b] * wv[r];
#pragma unroll
      for (int c = 0; c < 6; ++c) N[r][c] += dw * pw(b, c);
    }
  }
}

__device__ __forceinline__ void lu6(double N[6][6]) {
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    const double ip = 1.0 / N[c][c];
#pragma unroll
    for (int r = c + 1; r < 6; ++r) {
      const double f = N[r][c] * ip;
      N[r][c] = f;
#pragma unroll
      for (int cc = c + 1; cc < 6; ++cc) N[r][cc] -= f * N[c][cc];
    }
  }
}

__device__ __forceinline__ void lu6_solve(const double N[6][6], double* x) {
#pragma unroll
  for (int r = 1; r < 6; ++r)
#pragma unroll
    for (int c = 0; c < r; ++c) x[r] -= N[r][c] * x[c];
#pragma unroll
  for (int r = 5; r >= 0; --r) {
#pragma unroll
    for (int c = r + 1; c < 6; ++c) x[r] -= N[r][c] * x[c];
    x[r] /= N[r][r];
  }
}

// x_a = D_a P_a : T
__device__ __forceinline__ void rank6_expand(const double* D, const double* T, double* x) {
#pragma unroll
  for (int a = 0; a < 12; ++a) {
    double s = 0.0;
#pragma unroll
    for (int l = 0; l < 6; ++l) s += pw(a, l) * T[l];
    x[a] = D[a] * s;
  }
}

// Newton direction d = -J^{-1} R through the 6x6 form.
__device__ __forceinline__ void newton_direction(const Point& p, const Kin& k, const double* D, const double* R,
                                                 double* d) {
  double N[6][6], T[6];
  rank6_build(p, k, D, R, N, T);
  lu6(N);
  lu6_solve(N, T);
  rank6_expand(D, T, d);
#pragma unroll
  for (int a = 0; a < 12; ++a) d[a] -= R[a];
}

// Newton iterations at exponent n; returns 1 if converged.  iters accumulates.  The line
// search works in place: a rejected trial dg + lam d is pulled back by lam/2 d.
__device__ int newton(const Point& p, double n, double tol, int maxit, double* dg, int& iters) {
  const double floor_ = 1e-10, max_step = 0.02;
  Kin k;
  double R[12], D[12], d[12];
  for (int it = 0; it < maxit; ++it) {
    const double r2 = residual(p, n, dg, k, R, D);
    newton_direction(p, k, D, R, d);
    ++iters;
    // fmax drops NaN operands, so finiteness is tested per component (a NaN compares false)
    double big = 0.0, xmax = 0.0;
    bool finite = true;
#pragma unroll
    for (int a = 0; a < 12; ++a) {
      finite = finite && fabs(d[a]) < 1e300;
      big = fmax(big, fabs(d[a]));
      xmax = fmax(xmax, fabs(dg[a]));
    }
    if (!finite) return 0;  // non-finite step
    if (big > max_step) {
      const double s = max_step / big;
#pragma unroll
      for (int a = 0; a < 12; ++a) d[a] *= s;
      big = max_step;
    }
    if (big <= tol * fmax(xmax, floor_)) {
#pragma unroll
      for (int a = 0; a < 12; ++a) dg[a] += d[a];
      return 1;
    }
    double lam = 1.0;
#pragma unroll
    for (int a = 0; a < 12; ++a) dg[a] += d[a];
    for (int ls = 0; ls < 30; ++ls) {
      const double rt = residual(p, n, dg, k, R, nullptr);
      if (rt <= r2) break;
      lam *= 0.5;
#pragma unroll
      for (int a = 0; a < 12; ++a) dg[a] -= lam * d[a];
    }
  }
  return 0;
}

}  // namespace

// Shared set-up of a voxel: frame rotation, Fe0 = F_c Fp_n,c^{-1}, critical stresses.
__device__ __forceinline__ void setup_point(const ConstArgs& args, const MatDev& M, int64_t v, int64_t nv,
                                            const double* dF, double* Rg, Point& p) {
  const int g = args.gid[v];
#pragma unroll
  for (int i = 0; i < 9; ++i) Rg[i] = args.grainR[9 * g + i];
  double Fs[9], Fps[9], Fc[9], Fpc[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    double f = args.F[i * nv + v];
    if (dF) f += args.lam * dF[i * nv + v];
    Fs[i] = f;
    Fps[i] = args.Fp_n[i * nv + v];
  }
  if (args.F_out) {
#pragma unroll
    for (int i = 0; i < 9; ++i) args.F_out[i * nv + v] = Fs[i];
  }
  to_crystal(Rg, Fs, Fc);
  to_crystal(Rg, Fps, Fpc);
  if (args.grainC) {
    p.C11 = args.grainC[3 * g];
    p.C12 = args.grainC[3 * g + 1];
    p.C44 = args.grainC[3 * g + 2];
  } else {
    p.C11 = M.C11;
    p.C12 = M.C12;
    p.C44 = M.C44;
  }
  p.a = args.dt * M.gamma0_dot;
  inv3(Fpc, p.Gn);
  mm3(Fc, p.Gn, p.Fe0);
  if (M.hardening) {
    double forest[12];
#pragma unroll
    for (int b = 0; b < 12; ++b) forest[b] = args.rho_ssd[b * nv + v] + M.c_gnd * args.rho_gnd[b * nv + v];
#pragma unroll
    for (int a = 0; a < 12; ++a) {
      double s = 0.0;
#pragma unroll
      for (int b = 0; b < 12; ++b) s += M.q[12 * a + b] * forest[b];
      p.tc[a] = M.mu * M.burgers * sqrt(s);
    }
  } else {
#pragma unroll
    for (int a = 0; a < 12; ++a) p.tc[a] = M.tau_c_frozen;
  }
}

// Local solve, pass 1: Newton at n = 1/m from the warm start, at most kFastIters steps.
// With args.predict the start is moved along the linearised response of the previous
// converged evaluation (its slip sensitivity times the change of F): a low critical stress
// makes the power law so steep that a change of F of a few yield strains leaves the
// unmoved start far outside Newton's basin.  Converged voxels write their slip increments;
// the others are appended to a work list (their unmoved warm start stays in memory) for
// the continuation pass, so that a few stiff voxels do not hold whole wavefronts.  stats[0] = largest iteration count (atomic max),
// stats[1] = failures, stats[2] = length of the work list.
constexpr int kFastIters = 12;

__global__ void __launch_bounds__(64) k_slip_fast(ConstArgs args) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nv = args.nvox;
  if (v >= nv) return;
  const MatDev& M = *args.mat;
  double Rg[9];
  Point p;
  setup_point(args, M, v, nv, args.dF, Rg, p);
  double dg[12];
#pragma unroll
  for (int a = 0; a < 12; ++a) dg[a] = args.dg[a * nv + v];
  if (args.predict) {
    // first-order start along the Newton direction: the slip increments respond to a
    // change of F with the sensitivity stored at the last converged evaluation
    double dFs[9], dFc[9];
#pragma unroll
    for (int i = 0; i < 9; ++i)
      dFs[i] = args.dF[i * nv + v];
    to_crystal(Rg, dFs, dFc);
    const double s = args.lam - args.lam_base;
#pragma unroll
    for (int a = 0; a < 12; ++a) {
      double d = 0.0;
#pragma unroll
      for (int c = 0; c < 9; ++c) d += (double)args.dgdF[(int64_t)(9 * a + c) * nv + v] * dFc[c];
      dg[a] += s * d;
    }
  }
  int it = 0;
  const int ok = newton(p, M.n_exp, 1e-10, kFastIters, dg, it);
  if (ok) {
#pragma unroll
    for (int a = 0; a < 12; ++a) args.dg[a * nv + v] = dg[a];
    if (args.iters) args.iters[v] = it;
    atomicMax(&args.stats[0], it);
  } else {
    const int slot = atomicAdd(&args.stats[2], 1);
    args.work[slot] = (int32_t)v;
  }
}

// Local solve, pass 2 (work-list voxels): continuation in the exponent from the warm
// start, roots at n = 1, 2, 4, 8, 16, then Newton at n = 1/m.
__global__ void __launch_bounds__(64) k_slip_slow(ConstArgs args) {
  const int count = args.stats[2];
  const int64_t nv = args.nvox;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < count; idx += gridDim.x * blockDim.x) {
    const int64_t v = args.work[idx];
    const MatDev& M = *args.mat;
    double Rg[9];
    Point p;
    setup_point(args, M, v, nv, args.dF, Rg, p);
    double dg[12];
#pragma unroll
    for (int a = 0; a < 12; ++a) dg[a] = args.dg[a * nv + v];
    const double n_final = M.n_exp;
    int it = kFastIters, ok = 0;
#pragma unroll 1
    for (int pass = 0; pass < 6; ++pass) {
      double n = n_final, tol = 1e-10;
      if (pass < 5) {
        n = (double)(1 << pass);   // 1, 2, 4, 8, 16
        tol = 1e-4;
        if (n >= n_final) continue;
      }
      const int r = newton(p, n, tol, 60, dg, it);
      if (pass == 5) ok = r;
    }
#pragma unroll
    for (int a = 0; a < 12; ++a) args.dg[a * nv + v] = dg[a];
    if (args.iters) args.iters[v] = ok ? it : -it - 1;
    atomicMax(&args.stats[0], it);
    if (!ok) atomicAdd(&args.stats[1], 1);
  }
}

__global__ void k_reset_stats(int32_t* stats) {
  if (threadIdx.x < 4) stats[threadIdx.x] = 0;
}

// Stress and consistent tangent at the converged slip increments.
template <typename KT>
__global__ void __launch_bounds__(64) k_stress_tangent(ConstArgs args) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nv = args.nvox;
  if (v >= nv) return;
  const MatDev& M = *args.mat;
  double Rg[9];
  Point p;
  ConstArgs a2 = args;
  a2.F_out = nullptr;
  setup_point(a2, M, v, nv, args.dF, Rg, p);
  double dg[12];
#pragma unroll
  for (int a = 0; a < 12; ++a) dg[a] = args.dg[a * nv + v];
  Kin k;
  double R[12], D[12];
  residual(p, M.n_exp, dg, k, R, D);
  double G[9], SGt[9], Pc[9], Ps[9];
  mm3(p.Gn, k.Ainv, G);            // Fp^{-1}
  mmt3(k.S, G, SGt);               // S G^T
  mm3(k.Fe, SGt, Pc);              // P_c = Fe S G^T
  to_sample(Rg, Pc, Ps);
#pragma unroll
  for (int i = 0; i < 9; ++i) args.P[i * nv + v] = Ps[i];
  if (!args.K) return;
  double N[6][6];
  rank6_build(p, k, D, nullptr, N, nullptr);
  lu6(N);
  double H[9], Q[9], W[9], AtS[9];
  mm3(G, SGt, H);                  // G S G^T
  mm3(k.Ainv, SGt, Q);             // A^{-1} S G^T
  mmt3(k.S, k.Ainv, AtS);          // S A^{-T}
  mm3(k.Fe, AtS, W);               // Fe S A^{-T}
  KT* Kout = reinterpret_cast<KT*>(args.K);
#pragma unroll 1
  for (int kk = 0; kk < 3; ++kk) {
#pragma unroll 1
    for (int ll = 0; ll < 3; ++ll) {
      // rows kk of Fe and ll of G by selection: a loop-variable index into a register array
      // would place the array in scratch memory
      double av[3], bv[3], hv[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        av[i] = kk == 0 ? k.Fe[i] : (kk == 1 ? k.Fe[3 + i] : k.Fe[6 + i]);
        bv[i] = ll == 0 ? G[i] : (ll == 1 ? G[3 + i] : G[6 + i]);
        hv[i] = ll == 0 ? H[i] : (ll == 1 ? H[3 + i] : H[6 + i]);
      }
      // ddg = J^{-1} D H^T sym(av (x) bv), through the 6x6 form
      double T[6], x[12];
#pragma unroll
      for (int l = 0; l < 6; ++l)
        T[l] = (l < 3) ? av[kVi[l]] * bv[kVi[l]] : av[kVi[l]] * bv[kVj[l]] + av[kVj[l]] * bv[kVi[l]];
      lu6_solve(N, T);
      rank6_expand(D, T, x);
      if (args.dgdF) {
#pragma unroll
        for (int a = 0; a < 12; ++a) args.dgdF[(int64_t)(9 * a + 3 * kk + ll) * nv + v] = (float)x[a];
      }
      double Z[9];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          double z = 0.0;
#pragma unroll
          for (int b = 0; b < 12; ++b) z += x[b] * kSlipS[b][i] * kSlipM[b][j];
          Z[3 * i + j] = z;
        }
      double CeZ[9], CeZA[9], dE[9], dS[9];
      mm3(k.Ce, Z, CeZ);
      mm3(CeZ, k.Ainv, CeZA);
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
          dE[3 * i + j] = 0.5 * (av[i] * bv[j] + av[j] * bv[i]) - 0.5 * (CeZA[3 * i + j] + CeZA[3 * j + i]);
      cubic_stress(p, dE, dS);
      double t1[9], t2[9], dP[9];
      mm3(Z, Q, t1);               // - Fe Z Q
      mm3(k.Fe, t1, dP);
#pragma unroll
      for (int i = 0; i < 9; ++i) dP[i] = -dP[i];
      mmt3(dS, G, t1);             // + Fe dS G^T
      mm3(k.Fe, t1, t2);
#pragma unroll
      for (int i = 0; i < 9; ++i) dP[i] += t2[i];
      mm3(G, Z, t1);               // - W Z^T G^T = - W (G Z)^T
      mmt3(W, t1, t2);
#pragma unroll
      for (int i = 0; i < 9; ++i) dP[i] -= t2[i];
#pragma unroll
      for (int r = 0; r < 9; ++r)
        if (r / 3 == kk) dP[r] += hv[r % 3];                   // + e_k (x) H_l.
      const int col = 3 * kk + ll;
#pragma unroll
      for (int r = 0; r < 9; ++r) {
        const int64_t ki = tangent_index<KT>(r * 9 + col, v, nv, args.k_grouped);
        if constexpr (sizeof(KT) == 2) Kout[ki] = __float2half((float)(dP[r] * args.k_inv_scale));
        else Kout[ki] = (KT)dP[r];
      }
    }
  }
}

// Sensitivity of the converged stress to the critical resolved shear stresses (eqs. 6, 7,
// 14), for the adjoint form.  With tau_c fixed over the increment, R_a depends on tau_c,a
// only through the flow rule: dR_a/dtau_c,a = n g_a / tau_c,a, where g_a = dg_a - R_a is the
// flow value at the evaluated slip increments.  A unit change of tau_c,c moves the root by
// ddg = -J^{-1} e_c n g_c / tau_c,c (implicit function theorem), and the stress responds through
// Fp alone: Z = sum_b ddg_b s_b (x) m_b, dEe = -sym(Ce Z A^{-1}), dS = C : dEe,
// dP = -Fe Z A^{-1} S G^T + Fe dS G^T - Fe S A^{-T} Z^T G^T (the F-direction terms of the
// tangent vanish).  Output in the sample frame, dPdtc[(9c + r) * nvox + v] = dP_r / dtau_c,c;
// or, with an adjoint field w (9 x nvox, sample frame), its transposed application
// dPdtc[c * nvox + v] = sum_r w_r dP_r / dtau_c,c.
__global__ void __launch_bounds__(64) k_stress_sensitivity(ConstArgs args, double* __restrict__ dPdtc,
                                                             const double* __restrict__ w) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nv = args.nvox;
  if (v >= nv) return;
  const MatDev& M = *args.mat;
  double Rg[9];
  Point p;
  ConstArgs a2 = args;
  a2.F_out = nullptr;
  setup_point(a2, M, v, nv, nullptr, Rg, p);
  double dg[12];
#pragma unroll
  for (int a = 0; a < 12; ++a) dg[a] = args.dg[a * nv + v];
  Kin k;
  double R[12], D[12];
  residual(p, M.n_exp, dg, k, R, D);
  double G[9], SGt[9];
  mm3(p.Gn, k.Ainv, G);            // Fp^{-1}
  mmt3(k.S, G, SGt);               // S G^T
  double J[12][12];
  jacobian(p, k, D, J);
  lu12(J);
  double Q[9], W[9], AtS[9];
  mm3(k.Ainv, SGt, Q);             // A^{-1} S G^T
  mmt3(k.S, k.Ainv, AtS);          // S A^{-T}
  mm3(k.Fe, AtS, W);               // Fe S A^{-T}
  // the adjoint field is read once, before any output is written
  double wv[9];
#pragma unroll
  for (int r = 0; r < 9; ++r) wv[r] = w ? w[r * nv + v] : 0.0;
#pragma unroll 1
  for (int c = 0; c < 12; ++c) {
    double x[12];
#pragma unroll
    for (int a = 0; a < 12; ++a) x[a] = 0.0;
    // static register indices: the right-hand side entry is selected, not indexed
#pragma unroll
    for (int a = 0; a < 12; ++a)
      if (a == c) x[a] = -M.n_exp * (dg[a] - R[a]) / p.tc[a];
    lu12_solve(J, x);
    double Z[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        double z = 0.0;
#pragma unroll
        for (int b = 0; b < 12; ++b) z += x[b] * kSlipS[b][i] * kSlipM[b][j];
        Z[3 * i + j] = z;
      }
    double CeZ[9], CeZA[9], dE[9], dS[9];
    mm3(k.Ce, Z, CeZ);
    mm3(CeZ, k.Ainv, CeZA);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) dE[3 * i + j] = -0.5 * (CeZA[3 * i + j] + CeZA[3 * j + i]);
    cubic_stress(p, dE, dS);
    double t1[9], t2[9], dP[9], dPs[9];
    mm3(Z, Q, t1);                 // - Fe Z Q
    mm3(k.Fe, t1, dP);
#pragma unroll
    for (int i = 0; i < 9; ++i) dP[i] = -dP[i];
    mmt3(dS, G, t1);               // + Fe dS G^T
    mm3(k.Fe, t1, t2);
#pragma unroll
    for (int i = 0; i < 9; ++i) dP[i] += t2[i];
    mm3(G, Z, t1);                 // - W (G Z)^T
    mmt3(W, t1, t2);
#pragma unroll
    for (int i = 0; i < 9; ++i) dP[i] -= t2[i];
    to_sample(Rg, dP, dPs);
    if (w) {
      double t = 0.0;
#pragma unroll
      for (int r = 0; r < 9; ++r) t += wv[r] * dPs[r];
      dPdtc[(int64_t)c * nv + v] = t;
    } else {
#pragma unroll
      for (int r = 0; r < 9; ++r) dPdtc[(int64_t)(9 * c + r) * nv + v] = dPs[r];
    }
  }
}

// Reverse of the constitutive update of one increment, for the adjoint form (eqs. 2-9,
// 14, differentiated).  At the converged slip increments dg of an increment with
// start-of-increment state (Fp_n, rho_SSD,n, rho_GND,n), the outputs P (eq. 14), Fp (eq. 2)
// and rho_SSD (eq. 8) depend on F and on that state directly and through the root dg of the
// flow rule (eq. 6).  Given output weights P_bar, Fp_bar, rho_bar, the kernel forms the
// derivative of L = <P_bar, P> + <Fp_bar, Fp> + <rho_bar, rho_SSD> with respect to
//   mode 0: F (the right-hand side g of the adjoint equilibrium), and
//   mode 1: Fp_n, rho_SSD,n, rho_GND,n and the parameters (K, y_c, c_gnd; tau0 when
//           hardening is off), all at fixed F.
// Both modes run the same reverse sweep in the crystal frame:
//   1. at fixed dg, back through P = Fe S G^T, S = C : (Fe^T Fe - I)/2, Fe = Fe0 A^-1,
//      G = Gn A^-1, Fp = A Fp_n, A = I + sum dg_a s_a (x) m_a, rho_SSD = rho_n + h |dg|;
//      this gives dg_bar and the direct bars of Fe0 = F Gn and Gn = Fp_n^-1;
//   2. implicit function: mu = J^-T dg_bar with J = dR/d(dg) (the local Newton's Jacobian);
//      R_a = dg_a - g_a(tau_a, tau_c,a) adds tau_bar = D mu (D_a = dg_a/dtau_a) back through
//      tau_a = s_a . S m_a at fixed dg, and tau_c_bar_a = -mu_a n g_a / tau_c,a;
//   3. Fe0 = F Gn, Gn = Fp_n^-1 give F_bar and Fp_n_bar; tau_c (eq. 7) and h (eqs. 8-9) give
//      the density and parameter bars.
// The absolute value |dg| takes the derivative sgn(dg) with sgn(0) = 0.
__device__ __forceinline__ void lu12_solve_t(const double J[12][12], double* x) {
  // J = L U (unit L below the diagonal, U on and above it); J^T x = b: U^T y = b, L^T x = y
#pragma unroll
  for (int r = 0; r < 12; ++r) {
#pragma unroll
    for (int c = 0; c < r; ++c) x[r] -= J[c][r] * x[c];
    x[r] /= J[r][r];
  }
#pragma unroll
  for (int r = 11; r >= 0; --r)
#pragma unroll
    for (int c = r + 1; c < 12; ++c) x[r] -= J[c][r] * x[c];
}

// Fe_bar += Fe (C : sym(S_bar)): reverse of S = C : (Fe^T Fe - I) / 2
__device__ __forceinline__ void rev_elastic_stress(const Point& p, const double* Fe, const double* Sb, double* Feb) {
  double Ss[9], Eb[9], t[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) Ss[3 * i + j] = 0.5 * (Sb[3 * i + j] + Sb[3 * j + i]);
  cubic_stress(p, Ss, Eb);
  mm3(Fe, Eb, t);
#pragma unroll
  for (int i = 0; i < 9; ++i) Feb[i] += t[i];
}

__global__ void __launch_bounds__(64) k_constitutive_adjoint(ConstArgs args, AdjointLocalArgs b) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nv = args.nvox;
  double th[4] = {0.0, 0.0, 0.0, 0.0};  // K, y_c, c_gnd, tau0 (mode 1)
  if (v < nv) {
    const MatDev& M = *args.mat;
    double Rg[9];
    Point p;
    ConstArgs a2 = args;
    a2.F_out = nullptr;
    setup_point(a2, M, v, nv, nullptr, Rg, p);
    double Fs[9], Fc[9], Fpn_s[9], Fpn[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      Fs[i] = args.F[i * nv + v];
      Fpn_s[i] = args.Fp_n[i * nv + v];
    }
    to_crystal(Rg, Fs, Fc);
    to_crystal(Rg, Fpn_s, Fpn);
    double dg[12];
#pragma unroll
    for (int a = 0; a < 12; ++a) dg[a] = args.dg[a * nv + v];
    Kin k;
    double R[12], D[12];
    residual(p, M.n_exp, dg, k, R, D);
    // output weights in the crystal frame (read before any output is written: in-place safe)
    double Pb[9], Fpb[9], rb[12], t[9], t2[9];
    {
      double ws[9], fs[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        ws[i] = b.wP[i] - (b.lam ? b.lam[i * nv + v] : 0.0);
        fs[i] = b.Fp_bar ? b.Fp_bar[i * nv + v] : 0.0;
      }
      to_crystal(Rg, ws, Pb);
      to_crystal(Rg, fs, Fpb);
    }
#pragma unroll
    for (int a = 0; a < 12; ++a) rb[a] = b.rho_bar ? b.rho_bar[a * nv + v] : 0.0;
    double G[9];
    mm3(p.Gn, k.Ainv, G);  // Fp^-1
    // ---- 1. reverse sweep at fixed dg ----
    double Feb[9], Sb[9], Gb[9];
    mm3(Pb, G, t);
    mm3(t, k.S, Feb);      // Fe_bar = P_bar G S
    mtm3(k.Fe, Pb, t);
    mm3(t, G, Sb);         // S_bar = Fe^T P_bar G
    mtm3(Pb, k.Fe, t);
    mm3(t, k.S, Gb);       // G_bar = P_bar^T Fe S
    rev_elastic_stress(p, k.Fe, Sb, Feb);
    double Fe0b[9], Aib[9], Gnb[9], Ab[9];
    mmt3(Feb, k.Ainv, Fe0b);  // Fe = Fe0 A^-1
    mtm3(p.Fe0, Feb, Aib);
    mmt3(Gb, k.Ainv, Gnb);    // G = Gn A^-1
    mtm3(p.Gn, Gb, t);
#pragma unroll
    for (int i = 0; i < 9; ++i) Aib[i] += t[i];
    mtm3(k.Ainv, Aib, t);     // A_bar = -A^-T Ai_bar A^-T
    mmt3(t, k.Ainv, Ab);
    mmt3(Fpb, Fpn, t);        // Fp = A Fp_n
#pragma unroll
    for (int i = 0; i < 9; ++i) Ab[i] = t[i] - Ab[i];
    double Fpnb[9];
    mtm3(k.A, Fpb, Fpnb);
    // densities: rho_SSD = rho_n exp(-x) + |dg| phi(x) sqrt(S) / (b K) with S the
    // start-of-increment forest of the other systems, x = 2 y_c |dg| / b (ssd_phi)
    double rn[12], rg[12], f[12], sq[12], h[12], ex[12], tot = 0.0;
    const bool hard = M.hardening != 0;
#pragma unroll
    for (int a = 0; a < 12; ++a) {
      rn[a] = args.rho_ssd[a * nv + v];
      rg[a] = args.rho_gnd[a * nv + v];
      f[a] = rn[a] + M.c_gnd * rg[a];
      tot += f[a];
    }
#pragma unroll
    for (int a = 0; a < 12; ++a) {
      sq[a] = sqrt(tot - f[a]);
      h[a] = hard ? (1.0 / M.burgers) * (sq[a] / M.K_sim - 2.0 * M.y_c * rn[a]) : 0.0;
      ex[a] = exp(-2.0 * M.y_c * fabs(dg[a]) / M.burgers);
    }
    double mu[12];
#pragma unroll
    for (int a = 0; a < 12; ++a) {
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) s += kSlipS[a][i] * Ab[3 * i + j] * kSlipM[a][j];
      const double sg = dg[a] > 0.0 ? 1.0 : (dg[a] < 0.0 ? -1.0 : 0.0);
      mu[a] = s + rb[a] * h[a] * ex[a] * sg;   // d rho_a / d|dg_a| = h exp(-x)
    }
    // ---- 2. implicit function of the flow rule ----
    {
      double J[12][12];
      jacobian(p, k, D, J);
      lu12(J);
      lu12_solve_t(J, mu);
    }
    {
      double Sb2[9], Feb2[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) Sb2[i] = 0.0, Feb2[i] = 0.0;
#pragma unroll
      for (int a = 0; a < 12; ++a) {
        const double tb = D[a] * mu[a];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j) Sb2[3 * i + j] += tb * kSlipS[a][i] * kSlipM[a][j];
      }
      rev_elastic_stress(p, k.Fe, Sb2, Feb2);
      mmt3(Feb2, k.Ainv, t);
#pragma unroll
      for (int i = 0; i < 9; ++i) Fe0b[i] += t[i];
    }
    // ---- 3. inputs ----
    if (b.mode == 0) {
      double Fb[9];
      mmt3(Fe0b, p.Gn, Fb);  // Fe0 = F Gn
      to_sample(Rg, Fb, t);
#pragma unroll
      for (int i = 0; i < 9; ++i) b.g[i * nv + v] = t[i];
    } else {
      mtm3(Fc, Fe0b, t);     // Gn_bar += F^T Fe0_bar
#pragma unroll
      for (int i = 0; i < 9; ++i) Gnb[i] += t[i];
      mtm3(p.Gn, Gnb, t);    // Gn = Fp_n^-1: Fp_n_bar -= Gn^T Gn_bar Gn^T
      mmt3(t, p.Gn, t2);
#pragma unroll
      for (int i = 0; i < 9; ++i) Fpnb[i] -= t2[i];
      to_sample(Rg, Fpnb, t);
#pragma unroll
      for (int i = 0; i < 9; ++i) b.Fp_bar_out[i * nv + v] = t[i];
      double tcb[12];
#pragma unroll
      for (int a = 0; a < 12; ++a) tcb[a] = -mu[a] * M.n_exp * (dg[a] - R[a]) / p.tc[a];
      double rnb[12], fb[12];
      if (hard) {
        double wsum = 0.0, wk[12];
#pragma unroll
        for (int a = 0; a < 12; ++a) {
          const double u = fabs(dg[a]), x = 2.0 * M.y_c * u / M.burgers;
          const double w = rb[a] * u * ssd_phi(x);
          wk[a] = w / (2.0 * M.burgers * M.K_sim * sq[a]);   // through sqrt(S_a)
          wsum += wk[a];
          rnb[a] = rb[a] * ex[a];
          th[0] -= w * sq[a] / (M.burgers * M.K_sim * M.K_sim);
          // d rho / d y_c = (2 u / b)(-rho_n exp(-x) + u sqrt(S) phi'(x) / (b K))
          th[1] += rb[a] * (2.0 * u / M.burgers) *
                   (-rn[a] * ex[a] + u * sq[a] * ssd_dphi(x) / (M.burgers * M.K_sim));
        }
        const double mb2 = M.mu * M.burgers * M.mu * M.burgers;
#pragma unroll
        for (int c = 0; c < 12; ++c) {
          double s = wsum - wk[c];
#pragma unroll
          for (int a = 0; a < 12; ++a) s += tcb[a] * mb2 * M.q[12 * a + c] / (2.0 * p.tc[a]);
          fb[c] = s;
        }
#pragma unroll
        for (int c = 0; c < 12; ++c) {
          rnb[c] += fb[c];
          th[2] += fb[c] * rg[c];
          b.rho_bar_out[c * nv + v] = rnb[c];
          b.rho_gnd_bar[c * nv + v] = M.c_gnd * fb[c];
        }
      } else {
#pragma unroll
        for (int a = 0; a < 12; ++a) {
          th[3] += tcb[a];
          b.rho_bar_out[a * nv + v] = rb[a];
          b.rho_gnd_bar[a * nv + v] = 0.0;
        }
      }
    }
  }
  if (b.mode == 1) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      double s = th[i];
      for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
      if (threadIdx.x == 0) b.theta_partial[4 * blockIdx.x + i] = s;
    }
  }
}

// Commit of an increment: Fp = (R A_c R^T) Fp_n and rho_SSD = rho_SSD,n + h |dg| phi(x) (eq. 8
// integrated over the increment, see ssd_phi), h = (1/b)(1/l - 2 y_c rho_SSD,n),
// l = K / sqrt(sum_{b != a} (rho_SSD,n + c_gnd rho_GND,n)), x = 2 y_c |dg| / b.
__global__ void k_commit(CommitArgs args) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nv = args.nvox;
  if (v >= nv) return;
  const MatDev& M = *args.mat;
  const int g = args.gid[v];
  double Rg[9], dg[12], Ac[9], As[9], Fpn[9], Fp[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) Rg[i] = args.grainR[9 * g + i];
#pragma unroll
  for (int a = 0; a < 12; ++a) dg[a] = args.dg[a * nv + v];
#pragma unroll
  for (int i = 0; i < 9; ++i) Ac[i] = (i % 4 == 0) ? 1.0 : 0.0;
#pragma unroll
  for (int a = 0; a < 12; ++a)
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) Ac[3 * i + j] += dg[a] * kSlipS[a][i] * kSlipM[a][j];
  to_sample(Rg, Ac, As);
#pragma unroll
  for (int i = 0; i < 9; ++i) Fpn[i] = args.Fp[i * nv + v];
  mm3(As, Fpn, Fp);
#pragma unroll
  for (int i = 0; i < 9; ++i) args.Fp[i * nv + v] = Fp[i];
  if (M.hardening) {
    double rs[12], forest[12], tot = 0.0;
#pragma unroll
    for (int a = 0; a < 12; ++a) {
      rs[a] = args.rho_ssd[a * nv + v];
      forest[a] = rs[a] + M.c_gnd * args.rho_gnd[a * nv + v];
      tot += forest[a];
    }
#pragma unroll
    for (int a = 0; a < 12; ++a) {
      const double ell = M.K_sim / sqrt(tot - forest[a]);
      const double h = (1.0 / M.burgers) * (1.0 / ell - 2.0 * M.y_c * rs[a]);
      const double u = fabs(dg[a]);
      args.rho_ssd[a * nv + v] = rs[a] + h * u * ssd_phi(2.0 * M.y_c * u / M.burgers);
    }
  }
}

// Rotate crystal-frame tangents to the sample frame (kernel-level test entry point).
__global__ void k_rotate_tangent(int64_t nv, const int32_t* gid, const double* grainR, const double* Kc,
                                 double* Ks) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  const int g = gid[v];
  double Rg[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) Rg[i] = grainR[9 * g + i];
  double T[81];
  // T[pq][kl] = sum_rs Kc[pq][rs] R_kr R_ls
  for (int pq = 0; pq < 9; ++pq) {
    double X[9], Y[9];
    for (int rs = 0; rs < 9; ++rs) X[rs] = Kc[(int64_t)(pq * 9 + rs) * nv + v];
    to_sample(Rg, X, Y);
    for (int kl = 0; kl < 9; ++kl) T[pq * 9 + kl] = Y[kl];
  }
  for (int kl = 0; kl < 9; ++kl) {
    double X[9], Y[9];
    for (int pq = 0; pq < 9; ++pq) X[pq] = T[pq * 9 + kl];
    to_sample(Rg, X, Y);
    for (int ij = 0; ij < 9; ++ij) Ks[(int64_t)(ij * 9 + kl) * nv + v] = Y[ij];
  }
}

void launch_constitutive(const ConstArgs& a, int ktype, hipStream_t st, LaunchTimer* timer) {
  const int bs = 64;
  const int64_t nb = (a.nvox + bs - 1) / bs;
  const int nb_slow = (int)std::min<int64_t>(nb, 4096);
  hipLaunchKernelGGL(k_reset_stats, dim3(1), dim3(64), 0, st, a.stats);
  {
    TimedLaunch t(timer, KF_SLIP_FAST, a.nvox, st);
    launch(k_slip_fast, dim3((unsigned)nb), dim3(bs), 0u, st, a);
  }
  {
    TimedLaunch t(timer, KF_SLIP_SLOW, a.nvox, st);
    launch(k_slip_slow, dim3((unsigned)nb_slow), dim3(bs), 0u, st, a);
  }
  {
    TimedLaunch t(timer, KF_STRESS_TANGENT, a.nvox, st);
    if (ktype == KT_F16) launch(k_stress_tangent<__half>, dim3((unsigned)nb), dim3(bs), 0u, st, a);
    else if (ktype == KT_F32) launch(k_stress_tangent<float>, dim3((unsigned)nb), dim3(bs), 0u, st, a);
    else launch(k_stress_tangent<double>, dim3((unsigned)nb), dim3(bs), 0u, st, a);
  }
}

void launch_stress_sensitivity(const ConstArgs& a, double* dPdtc, const double* w, hipStream_t st) {
  const int bs = 64;
  const int64_t nb = (a.nvox + bs - 1) / bs;
  launch(k_stress_sensitivity, dim3((unsigned)nb), dim3(bs), 0u, st, a, dPdtc, w);
}

int launch_constitutive_adjoint(const ConstArgs& a, const AdjointLocalArgs& b, hipStream_t st) {
  const int bs = 64;
  const int64_t nb = (a.nvox + bs - 1) / bs;
  launch(k_constitutive_adjoint, dim3((unsigned)nb), dim3(bs), 0u, st, a, b);
  return (int)nb;
}

void launch_commit(const CommitArgs& a, hipStream_t st) {
  const int bs = 256;
  const int64_t nb = (a.nvox + bs - 1) / bs;
  hipLaunchKernelGGL(k_commit, dim3((unsigned)nb), dim3(bs), 0, st, a);
}

void launch_rotate_tangent(int64_t nv, const int32_t* gid, const double* grainR, const double* Kc, double* Ks,
                           hipStream_t st) {
  const int bs = 128;
  const int64_t nb = (nv + bs - 1) / bs;
  hipLaunchKernelGGL(k_rotate_tangent, dim3((unsigned)nb), dim3(bs), 0, st, nv, gid, grainR, Kc, Ks);
}

}  // namespace rve
