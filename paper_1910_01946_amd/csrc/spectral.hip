// Spectral path: 3-D real FFTs of 9-component voxel fields, the Galerkin projection of
// eq. 17 with the rotated-scheme frequencies of eq. A.4 and the mixed-control rule of
// Section 2.2, the spectral curl of eq. B.3, and the fused conjugate-gradient updates of
// eq. 18.
//
// Layout.  Real fields are component-major (9 x nvox, x fastest).  The half spectrum is
// (9, nz, ny, nxh) with nxh = nx/2 + 1, complex, interleaved.  A 3-D transform is three
// passes, each holding complete lines in LDS:
//   x pass  (one z, ly rows, all 9 components): two real rows are packed into one complex
//           line (row a + i row b), transformed, and split into the two half spectra;
//           fused with the producer of the field (K:p of eq. 18, the stress, Fp - I).
//   y pass  (one component, one z, ty columns of kx).
//   z pass  (one ky, tz columns of kx, all 9 components): forward z transform, the
//           pointwise operator (projection or curl, including the 1/nvox normalisation),
//           inverse z transform, in one kernel.
// and the inverse y and x passes; the inverse x pass is fused with the consumer (CG
// update and residual norm, Nye tensor and GND densities, or plain output).
#include "spectral.h"


namespace rve {

namespace {

template <typename T>
__device__ __forceinline__ double block_sum(double v, double* sh) {
  // 64-wide wavefront reduction, then across wavefronts through LDS
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int w = 0; w < nw; ++w) s += sh[w];
  }
  return s;
}

// ---------------------------------------------------------------------------------------
// forward x pass
// ---------------------------------------------------------------------------------------
template <typename T, int MODE>
__global__ void k_xfwd(GridPlan g, XFwdArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
  __shared__ double red[16];
  if (MODE == XF_CG && a.cg->done) return;
  const int nx = g.nx, ny = g.ny, nz = g.nz, nxh = g.nxh;
  const int64_t nv = g.nvox;
  const int z = blockIdx.y, y0 = blockIdx.x * g.ly;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int npair = g.ly / 2;
  double acc = 0.0;
  if (tid < g.ly * nx) {
    const int row = tid / nx, x = tid - row * nx, y = y0 + row;
    T val[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) val[c] = (T)0;
    if (y < ny) {
      const int64_t v = ((int64_t)z * ny + y) * nx + x;
      if (MODE == XF_FIELD64) {
#pragma unroll
        for (int c = 0; c < 9; ++c) val[c] = (T)a.in64[c * nv + v];
      } else if (MODE == XF_FP_MINUS_I) {
#pragma unroll
        for (int c = 0; c < 9; ++c) val[c] = (T)(a.in64[c * nv + v] - ((c % 4 == 0) ? 1.0 : 0.0));
      } else {
        T* X = reinterpret_cast<T*>(a.x);
        T* r = reinterpret_cast<T*>(a.r);
        const T* q = reinterpret_cast<const T*>(a.q);
        const T* K = reinterpret_cast<const T*>(a.K);
        double ps[9];
        if (a.cg->iter > 0) {
          const double alpha = a.cg->alpha;
          if (a.cg->it_best == a.cg->iter - 1) {
            T* XB = reinterpret_cast<T*>(a.xbest);
#pragma unroll
            for (int c = 0; c < 9; ++c) XB[c * nv + v] = X[c * nv + v];
          }
#pragma unroll
          for (int c = 0; c < 9; ++c) {
            const int64_t o = c * nv + v;
            const T rn = (T)((double)r[o] - alpha * (double)q[o]);
            r[o] = rn;
            ps[c] = (double)rn;
          }
        } else {
#pragma unroll
          for (int c = 0; c < 9; ++c) ps[c] = (double)r[c * nv + v];
        }
#pragma unroll
        for (int c = 0; c < 9; ++c) acc += ps[c] * ps[c];
        const int gi = a.gid[v];
        double Rg[9], pc[9], yc[9], ys[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) Rg[i] = a.grainR[9 * gi + i];
        to_crystal(Rg, ps, pc);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
          double s = 0.0;
#pragma unroll
          for (int j = 0; j < 9; ++j) s += (double)K[tangent_index<T>(i * 9 + j, v, nv, true)] * pc[j];
          yc[i] = s;
        }
        to_sample(Rg, yc, ys);
#pragma unroll
        for (int c = 0; c < 9; ++c) val[c] = (T)ys[c];
      }
    }
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      cplx<T>* e = &buf[(c * npair + (row >> 1)) * nx + x];
      if (row & 1) e->y = val[c];
      else e->x = val[c];
    }
  }
  __syncthreads();
  LineLayout L{9 * npair, 1, nx, 0, 1};
  fft_lines<T, 5>(buf, L, g.ax, reinterpret_cast<const cplx<T>*>(g.twx), (T)-1);
  cplx<T>* spec = reinterpret_cast<cplx<T>*>(a.spec);
  const int total = 9 * npair * nxh;
  for (int idx = tid; idx < total; idx += nthr) {
    const int k = idx % nxh;
    const int t = idx / nxh;
    const int pair = t % npair, c = t / npair;
    const cplx<T> Zk = buf[(c * npair + pair) * nx + k];
    const cplx<T> Zm = buf[(c * npair + pair) * nx + (nx - k) % nx];
    const T h = (T)0.5;
    const cplx<T> A = cmk(h * (Zk.x + Zm.x), h * (Zk.y - Zm.y));
    const cplx<T> B = cmk(h * (Zk.y + Zm.y), h * (Zm.x - Zk.x));
    const int ya = y0 + 2 * pair;
    const int64_t row0 = ((int64_t)c * nz + z) * ny;
    if (ya < ny) spec[(row0 + ya) * nxh + k] = A;
    if (ya + 1 < ny) spec[(row0 + ya + 1) * nxh + k] = B;
  }
  if (MODE == XF_CG) {
    const double sum = block_sum<T>(acc, red);
    if (tid == 0) a.partial[blockIdx.y * gridDim.x + blockIdx.x] = sum;
  }
}

// ---------------------------------------------------------------------------------------
// y pass (forward or inverse)
// ---------------------------------------------------------------------------------------
template <typename T>
__global__ void k_yfft(GridPlan g, void* spec_, int sign, const CGState* cg) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
  if (cg && cg->done) return;
  const int ny = g.ny, nz = g.nz, nxh = g.nxh, ty = g.ty, typ = g.ty + 1;
  const int c = blockIdx.z, z = blockIdx.y, kx0 = blockIdx.x * ty;
  const int tid = threadIdx.x, nthr = blockDim.x;
  cplx<T>* spec = reinterpret_cast<cplx<T>*>(spec_);
  const int64_t base = (((int64_t)c * nz + z) * ny) * nxh + kx0;
  for (int idx = tid; idx < ny * ty; idx += nthr) {
    const int y = idx / ty, j = idx - y * ty;
    buf[y * typ + j] = (kx0 + j < nxh) ? spec[base + (int64_t)y * nxh + j] : cmk((T)0, (T)0);
  }
  __syncthreads();
  LineLayout L{ty, ty, 0, 1, typ, 0, make_fastdiv(ty)};
  fft_lines<T, 16>(buf, L, g.ay, reinterpret_cast<const cplx<T>*>(g.twy), (T)sign);
  for (int idx = tid; idx < ny * ty; idx += nthr) {
    const int y = idx / ty, j = idx - y * ty;
    if (kx0 + j < nxh) spec[base + (int64_t)y * nxh + j] = buf[y * typ + j];
  }
}

// ---------------------------------------------------------------------------------------
// z pass with the pointwise operator
// ---------------------------------------------------------------------------------------
template <typename T, int OP, int RS>
__global__ void k_mid(GridPlan g, MidArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
  if (a.cg && a.cg->done) return;
  // components carried: nine, or the three of the factorised projection
  constexpr int NC = OP == MID_GREEN3 ? 3 : 9;
  const int ny = g.ny, nz = g.nz, nxh = g.nxh, tz = NC == 3 ? g.tz3 : g.tz, SZ = padded_len(nz);
  const FastDiv ftz = NC == 3 ? g.ftz3 : g.ftz;
  // XCD-aware order: consecutive hardware block ids are dealt to the 8 XCDs in turn; each
  // XCD takes a contiguous range of (ky, kx tile) so that the cache lines shared by
  // neighbouring tiles and rows are fetched and written back through a single L2.
  const int ntile = (nxh + tz - 1) / tz;
  const int nblk = ntile * ny;
  const int per = (nblk + 7) / 8;
  const int logical = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (logical >= nblk) return;
  const int ky = logical / ntile, kx0 = (logical % ntile) * tz;
  const int tid = threadIdx.x, nthr = blockDim.x;
  cplx<T>* spec = reinterpret_cast<cplx<T>*>(a.spec);
  // one contiguous padded z line per (component, kx column): line c * tz + j
  cplx<T>* twz = buf + NC * tz * SZ;
  load_twiddles(twz, g.twz, nz);
  const int nload = NC * nz * tz;
  // 8 independent loads in flight per thread before the LDS writes
  for (int b0 = tid; b0 < nload; b0 += 8 * nthr) {
    cplx<T> val[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = b0 + u * nthr;
      val[u] = cmk((T)0, (T)0);
      if (idx < nload) {
        const int t = fdiv(idx, ftz), j = idx - t * tz;
        const int c = fdiv(t, g.fnz), zz = t - c * nz;
        if (kx0 + j < nxh) val[u] = spec[(((int64_t)c * nz + zz) * ny + ky) * nxh + kx0 + j];
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = b0 + u * nthr;
      if (idx < nload) {
        const int t = fdiv(idx, ftz), j = idx - t * tz;
        const int c = fdiv(t, g.fnz), zz = t - c * nz;
        buf[(c * tz + j) * SZ + padded(zz)] = val[u];
      }
    }
  }
  __syncthreads();
  LineLayout L{NC * tz, 1, SZ, 0, 0};
  fft_lines<T, 9, RS>(buf, L, g.az, twz, (T)-1);
  const cplx<double>* Ex = reinterpret_cast<const cplx<double>*>(g.Ex);
  const cplx<double>* Ey = reinterpret_cast<const cplx<double>*>(g.Ey);
  const cplx<double>* Ez = reinterpret_cast<const cplx<double>*>(g.Ez);
  for (int idx = tid; idx < nz * tz; idx += nthr) {
    const int kz = fdiv(idx, ftz), j = idx - kz * tz, kx = kx0 + j;
    if (kx >= nxh) continue;
    // modified frequency vector of the rotated scheme (eq. A.4):
    // k_i = 1/4 (-i)(E_i - 1) prod_{j != i} (1 + E_j)
    const cplx<double> ex = Ex[kx], ey = Ey[ky], ez = Ez[kz];
    cplx<double> kv[3];
    if (g.freq == FREQ_STANDARD) {
      // xi = arg(E) in (-pi, pi]; the Nyquist angle pi (E = -1, exact in the tables) has no
      // derivative
      const cplx<double> e3[3] = {ex, ey, ez};
#pragma unroll
      for (int d = 0; d < 3; ++d)
        kv[d] = cmk((e3[d].x == -1.0 && e3[d].y == 0.0) ? 0.0 : atan2(e3[d].y, e3[d].x), 0.0);
    } else {
      const cplx<double> px = cmk(1.0 + ex.x, ex.y), py = cmk(1.0 + ey.x, ey.y), pz = cmk(1.0 + ez.x, ez.y);
      const cplx<double> mx = cmk(ex.x - 1.0, ex.y), my = cmk(ey.x - 1.0, ey.y), mz = cmk(ez.x - 1.0, ez.y);
      kv[0] = cmuli(cscale(cmul(mx, cmul(py, pz)), 0.25), -1.0);
      kv[1] = cmuli(cscale(cmul(my, cmul(px, pz)), 0.25), -1.0);
      kv[2] = cmuli(cscale(cmul(mz, cmul(px, py)), 0.25), -1.0);
    }
    const bool dc = kx == 0 && ky == 0 && kz == 0;
    const double k2 = kv[0].x * kv[0].x + kv[0].y * kv[0].y + kv[1].x * kv[1].x + kv[1].y * kv[1].y +
                      kv[2].x * kv[2].x + kv[2].y * kv[2].y;
    if constexpr (OP == MID_GREEN3) {
      // w_i = v_i / (nvox |k|^2); v has no zero-frequency content (a sum of differences)
      const double s = (dc || k2 == 0.0) ? 0.0 : a.inv_n / k2;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        cplx<T>& e = buf[(i * tz + j) * SZ + padded(kz)];
        e = cmk((T)(s * (double)e.x), (T)(s * (double)e.y));
      }
      continue;
    }
    cplx<double> ik[3];
    if (OP != MID_GREEN) {
      // alpha_ij = eps_jml (i k_m / h) Fp_il
      const double s = a.inv_h * a.inv_n;
#pragma unroll
      for (int m = 0; m < 3; ++m) ik[m] = cscale(cmuli(kv[m], 1.0), s);
    }
    // both operators map row i of the input to row i of the output: one row at a time, in place
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      cplx<double> A[3], out[3];
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        const cplx<T> e = buf[((3 * i + l) * tz + j) * SZ + padded(kz)];
        A[l] = cmk((double)e.x, (double)e.y);
      }
      if (OP == MID_GREEN) {
        if (dc) {
          const double nvox = (double)g.nvox;
#pragma unroll
          for (int l = 0; l < 3; ++l)
            out[l] = cscale(cmk(A[l].x - nvox * a.dc_target[3 * i + l], A[l].y), a.mask_keep[3 * i + l] * a.inv_n);
        } else if (k2 == 0.0) {
#pragma unroll
          for (int l = 0; l < 3; ++l) out[l] = cmk(0.0, 0.0);
        } else {
          // u_i = sum_l A_il conj(k_l) / |k|^2 ; (G:A)_ij = u_i k_j
          const double s = a.inv_n / k2;
          cplx<double> u = cmk(0.0, 0.0);
#pragma unroll
          for (int l = 0; l < 3; ++l) u = cadd(u, cmulc(A[l], kv[l]));
          u = cscale(u, s);
#pragma unroll
          for (int jj = 0; jj < 3; ++jj) out[jj] = cmul(u, kv[jj]);
        }
      } else {
        out[0] = csub(cmul(ik[1], A[2]), cmul(ik[2], A[1]));
        out[1] = csub(cmul(ik[2], A[0]), cmul(ik[0], A[2]));
        out[2] = csub(cmul(ik[0], A[1]), cmul(ik[1], A[0]));
      }
#pragma unroll
      for (int l = 0; l < 3; ++l) buf[((3 * i + l) * tz + j) * SZ + padded(kz)] = cmk((T)out[l].x, (T)out[l].y);
    }
  }
  __syncthreads();
  fft_lines<T, 9, RS>(buf, L, g.az, twz, (T)1);
  for (int idx = tid; idx < nload; idx += nthr) {
    const int t = fdiv(idx, ftz), j = idx - t * tz;
    const int c = fdiv(t, g.fnz), zz = t - c * nz;
    if (kx0 + j < nxh) spec[(((int64_t)c * nz + zz) * ny + ky) * nxh + kx0 + j] = buf[(c * tz + j) * SZ + padded(zz)];
  }
}

// ---------------------------------------------------------------------------------------
// inverse x pass with the consumer
// ---------------------------------------------------------------------------------------
template <typename T, int MODE>
__global__ void k_xinv(GridPlan g, XInvArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
  __shared__ double red[16];
  if (MODE == XI_CG && a.cg->done) return;
  const int nx = g.nx, ny = g.ny, nz = g.nz, nxh = g.nxh;
  const int64_t nv = g.nvox;
  const int z = blockIdx.y, y0 = blockIdx.x * g.ly;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int npair = g.ly / 2;
  const cplx<T>* spec = reinterpret_cast<const cplx<T>*>(a.spec);
  const int nload = 9 * npair * nx;
  for (int idx = tid; idx < nload; idx += nthr) {
    const int k = idx % nx, t = idx / nx;
    const int pair = t % npair, c = t / npair;
    const int ya = y0 + 2 * pair;
    const int64_t row0 = ((int64_t)c * nz + z) * ny;
    const bool hi = k >= nxh;
    const int kk = hi ? nx - k : k;
    cplx<T> A = cmk((T)0, (T)0), B = cmk((T)0, (T)0);
    if (ya < ny) A = spec[(row0 + ya) * nxh + kk];
    if (ya + 1 < ny) B = spec[(row0 + ya + 1) * nxh + kk];
    if (hi) {
      A.y = -A.y;
      B.y = -B.y;
    }
    buf[(c * npair + pair) * nx + k] = cmk(A.x - B.y, A.y + B.x);
  }
  __syncthreads();
  LineLayout L{9 * npair, 1, nx, 0, 1};
  fft_lines<T, 5>(buf, L, g.ax, reinterpret_cast<const cplx<T>*>(g.twx), (T)1);
  double acc = 0.0;
  if (tid < g.ly * nx) {
    const int row = tid / nx, x = tid - row * nx, y = y0 + row;
    if (y < ny) {
      const int64_t v = ((int64_t)z * ny + y) * nx + x;
      double q[9];
#pragma unroll
      for (int c = 0; c < 9; ++c) {
        const cplx<T> e = buf[(c * npair + (row >> 1)) * nx + x];
        q[c] = (double)((row & 1) ? e.y : e.x);
      }
      if (MODE == XI_RESID) {
        T* X = reinterpret_cast<T*>(a.x);
        T* R = reinterpret_cast<T*>(a.r);
        T* P = reinterpret_cast<T*>(a.p);
#pragma unroll
        for (int c = 0; c < 9; ++c) {
          const T rv = (T)(-q[c]);
          R[c * nv + v] = rv;
          P[c * nv + v] = rv;
          X[c * nv + v] = (T)0;
          acc += (double)rv * (double)rv;
        }
      } else if (MODE == XI_CG) {
        T* Q = reinterpret_cast<T*>(a.q);
        const T* R = reinterpret_cast<const T*>(a.r);
        T* P = reinterpret_cast<T*>(a.p);
        if (a.cg->iter > 0) {
          const double beta = a.cg->beta, alpha = a.cg->alpha;
          T* X = reinterpret_cast<T*>(a.x);
#pragma unroll
          for (int c = 0; c < 9; ++c) {
            const int64_t o = c * nv + v;
            const T pold = P[o];
            const T qv = (T)(q[c] + beta * (double)Q[o]);
            const T pv = (T)((double)R[o] + beta * (double)pold);
            X[o] = (T)((double)X[o] + alpha * (double)pold);
            Q[o] = qv;
            P[o] = pv;
            acc += (double)pv * (double)qv;
          }
        } else {
#pragma unroll
          for (int c = 0; c < 9; ++c) {
            const int64_t o = c * nv + v;
            const T qv = (T)q[c];
            const T pv = R[o];
            Q[o] = qv;
            P[o] = pv;
            acc += (double)pv * (double)qv;
          }
        }
      } else if (MODE == XI_OUT64) {
#pragma unroll
        for (int c = 0; c < 9; ++c) a.out64[c * nv + v] = q[c];
      } else {
        // Nye tensor and GND densities (eqs. 12, 13)
#pragma unroll
        for (int c = 0; c < 9; ++c) a.out64[c * nv + v] = q[c];
        if (a.rho_gnd) {
          const MatDev& M = *a.mat;
          const int gi = a.gid[v];
          double Rg[9], ac[9];
#pragma unroll
          for (int i = 0; i < 9; ++i) Rg[i] = a.grainR[9 * gi + i];
          to_crystal(Rg, q, ac);
          double seg[18];
#pragma unroll
          for (int s = 0; s < 18; ++s) {
            double t = 0.0;
#pragma unroll
            for (int c = 0; c < 9; ++c) t += M.Aplus[s * 9 + c] * ac[c];
            seg[s] = t / M.burgers;
          }
#pragma unroll
          for (int al = 0; al < 12; ++al)
            a.rho_gnd[al * nv + v] = fabs(seg[al]) + 0.5 * fabs(seg[12 + M.screw_of[al]]);
        }
      }
    }
  }
  if (MODE == XI_RESID || MODE == XI_CG) {
    const double s = block_sum<T>(acc, red);
    if (tid == 0) a.partial[blockIdx.y * gridDim.x + blockIdx.x] = s;
  }
}

// ---------------------------------------------------------------------------------------
// CG bookkeeping (one block of 256 threads)
// ---------------------------------------------------------------------------------------
__device__ double reduce_partials(const double* p, int n) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += p[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  return sh[0];
}

__global__ void k_cg_start(CGState* cg, const double* partial, int n, double tol2, int max_iter) {
  const double rr = reduce_partials(partial, n);
  if (threadIdx.x == 0) {
    cg->rr = rr;
    cg->rr0 = rr;
    cg->tol2 = tol2;
    cg->iter = 0;
    cg->rr_best = rr;
    cg->rr_floor = 0.0;
    cg->it_best = 0;
    cg->max_iter = max_iter;
    cg->stall = kCgStall;
    cg->alpha = 0.0;
    cg->beta = 0.0;
    cg->done = (rr > 0.0 && max_iter > 0) ? 0 : 1;
  }
}

__global__ void k_cg_beta(CGState* cg, const double* partial, int n) {
  if (cg->done) return;
  const double rr = reduce_partials(partial, n);
  if (threadIdx.x == 0) cg_beta_update(cg, rr, cg->iter == 0);
}

__global__ void k_cg_alpha(CGState* cg, const double* partial, int n) {
  if (cg->done) return;
  const double pq = reduce_partials(partial, n);
  if (threadIdx.x == 0) cg_alpha_update(cg, pq);
}

// ---------------------------------------------------------------------------------------
// reductions and small elementwise kernels
// ---------------------------------------------------------------------------------------
__global__ void k_colsum(const double* f, int ncomp, int64_t nvox, double* partial) {
  __shared__ double red[16];
  for (int c = 0; c < ncomp; ++c) {
    double s = 0.0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nvox; v += (int64_t)gridDim.x * blockDim.x)
      s += f[c * nvox + v];
    const double t = block_sum<double>(s, red);
    if (threadIdx.x == 0) partial[blockIdx.x * ncomp + c] = t;
    __syncthreads();
  }
}

template <typename T>
__global__ void k_sumsq(const T* f, int64_t n, double* partial) {
  __shared__ double red[16];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double v = (double)f[i];
    s += v * v;
  }
  const double t = block_sum<double>(s, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ void k_predictor(const double* F, const double* F_prev, Corr9 corr, double* out, int64_t nvox) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nvox) return;
#pragma unroll
  for (int c = 0; c < 9; ++c) {
    const double f = F[c * nvox + v];
    out[c * nvox + v] = F_prev ? (2.0 * f - F_prev[c * nvox + v] + corr.v[c]) : (f + corr.v[c]);
  }
}

}  // namespace

// ---------------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------------
// bytes: LDS per work-group of the device; the kernel's static LDS is taken off it.
template <typename K>
static hipError_t lds_limit(K kernel, int bytes) {
  hipFuncAttributes fa;
  hipError_t e = hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(kernel));
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             bytes - (int)fa.sharedSizeBytes);
}

template <typename T, int RS>
static hipError_t mid_limits(int bytes) {
  hipError_t e = hipSuccess, f;
  if ((f = lds_limit(k_mid<T, MID_GREEN, RS>, bytes)) != hipSuccess) e = f;
  if ((f = lds_limit(k_mid<T, MID_CURL, RS>, bytes)) != hipSuccess) e = f;
  if ((f = lds_limit(k_mid<T, MID_GREEN3, RS>, bytes)) != hipSuccess) e = f;
  return e;
}

template <typename T>
static hipError_t spectral_limits(int bytes) {
  hipError_t e = hipSuccess, f;
  if ((f = lds_limit(k_xfwd<T, XF_FIELD64>, bytes)) != hipSuccess) e = f;
  if ((f = lds_limit(k_xfwd<T, XF_CG>, bytes)) != hipSuccess) e = f;
  if ((f = lds_limit(k_xfwd<T, XF_FP_MINUS_I>, bytes)) != hipSuccess) e = f;
  if ((f = lds_limit(k_yfft<T>, bytes)) != hipSuccess) e = f;
  if ((f = mid_limits<T, RS_ALL>(bytes)) != hipSuccess) e = f;
  if ((f = mid_limits<T, RS_8>(bytes)) != hipSuccess) e = f;
  if ((f = mid_limits<T, RS_8 | RS_4>(bytes)) != hipSuccess) e = f;
  if ((f = mid_limits<T, RS_8 | RS_2>(bytes)) != hipSuccess) e = f;
  if ((f = lds_limit(k_xinv<T, XI_RESID>, bytes)) != hipSuccess) e = f;
  if ((f = lds_limit(k_xinv<T, XI_CG>, bytes)) != hipSuccess) e = f;
  if ((f = lds_limit(k_xinv<T, XI_NYE>, bytes)) != hipSuccess) e = f;
  if ((f = lds_limit(k_xinv<T, XI_OUT64>, bytes)) != hipSuccess) e = f;
  return e;
}

hipError_t set_spectral_lds_limits(int bytes) {
  hipError_t e = spectral_limits<float>(bytes), f = spectral_limits<double>(bytes);
  return e != hipSuccess ? e : f;
}

static int xthreads(const GridPlan& g) {
  const int t = g.ly * g.nx;
  return ((t + 63) / 64) * 64;
}

int xfwd_blocks(const GridPlan& g) { return ((g.ny + g.ly - 1) / g.ly) * g.nz; }
int xinv_blocks(const GridPlan& g) { return xfwd_blocks(g); }

void launch_xfwd(const GridPlan& g, bool fp32, const XFwdArgs& a, hipStream_t st) {
  const dim3 grid((g.ny + g.ly - 1) / g.ly, g.nz);
  const dim3 block(xthreads(g));
  const size_t sh = (size_t)9 * (g.ly / 2) * g.nx * (fp32 ? 8 : 16);
#define XF_CASE(T)                                                                            \
  switch (a.mode) {                                                                           \
    case XF_FIELD64: hipLaunchKernelGGL((k_xfwd<T, XF_FIELD64>), grid, block, sh, st, g, a); break; \
    case XF_CG: hipLaunchKernelGGL((k_xfwd<T, XF_CG>), grid, block, sh, st, g, a); break;     \
    default: hipLaunchKernelGGL((k_xfwd<T, XF_FP_MINUS_I>), grid, block, sh, st, g, a); break; \
  }
  if (fp32) {
    XF_CASE(float)
  } else {
    XF_CASE(double)
  }
#undef XF_CASE
}

void launch_yfft(const GridPlan& g, bool fp32, void* spec, int sign, const CGState* cg, hipStream_t st) {
  const dim3 grid((g.nxh + g.ty - 1) / g.ty, g.nz, 9);
  const size_t sh = (size_t)g.ny * (g.ty + 1) * (fp32 ? 8 : 16);
  if (fp32) {
    hipLaunchKernelGGL(k_yfft<float>, grid, dim3(256), sh, st, g, spec, sign, cg);
  } else {
    hipLaunchKernelGGL(k_yfft<double>, grid, dim3(256), sh, st, g, spec, sign, cg);
  }
}

static int mid_blocks(const GridPlan& g, int tz) {
  const int nblk = ((g.nxh + tz - 1) / tz) * g.ny;
  return 8 * ((nblk + 7) / 8);
}

template <typename T, int OP, int RS>
static void mid_launch(const GridPlan& g, const MidArgs& a, hipStream_t st) {
  const int nc = OP == MID_GREEN3 ? 3 : 9, tz = OP == MID_GREEN3 ? g.tz3 : g.tz;
  const size_t sh = ((size_t)nc * tz * padded_len(g.nz) + g.nz) * sizeof(cplx<T>);
  launch(k_mid<T, OP, RS>, dim3(mid_blocks(g, tz)), dim3(256), (uint32_t)sh, st, g, a);
}

// radix set of the z transform
template <typename T, int OP>
static void mid_dispatch(const GridPlan& g, const MidArgs& a, hipStream_t st) {
  switch (radix_set_for(radix_bits(g.az))) {
    case RS_8: mid_launch<T, OP, RS_8>(g, a, st); break;
    case RS_8 | RS_4: mid_launch<T, OP, RS_8 | RS_4>(g, a, st); break;
    case RS_8 | RS_2: mid_launch<T, OP, RS_8 | RS_2>(g, a, st); break;
    default: mid_launch<T, OP, RS_ALL>(g, a, st); break;
  }
}

void launch_mid(const GridPlan& g, bool fp32, const MidArgs& a, hipStream_t st) {
  if (fp32) {
    if (a.op == MID_GREEN) mid_dispatch<float, MID_GREEN>(g, a, st);
    else if (a.op == MID_GREEN3) mid_dispatch<float, MID_GREEN3>(g, a, st);
    else mid_dispatch<float, MID_CURL>(g, a, st);
  } else {
    if (a.op == MID_GREEN) mid_dispatch<double, MID_GREEN>(g, a, st);
    else if (a.op == MID_GREEN3) mid_dispatch<double, MID_GREEN3>(g, a, st);
    else mid_dispatch<double, MID_CURL>(g, a, st);
  }
}

void launch_xinv(const GridPlan& g, bool fp32, const XInvArgs& a, hipStream_t st) {
  const dim3 grid((g.ny + g.ly - 1) / g.ly, g.nz);
  const dim3 block(xthreads(g));
  const size_t sh = (size_t)9 * (g.ly / 2) * g.nx * (fp32 ? 8 : 16);
#define XI_CASE(T)                                                                             \
  switch (a.mode) {                                                                            \
    case XI_RESID: hipLaunchKernelGGL((k_xinv<T, XI_RESID>), grid, block, sh, st, g, a); break; \
    case XI_CG: hipLaunchKernelGGL((k_xinv<T, XI_CG>), grid, block, sh, st, g, a); break;       \
    case XI_NYE: hipLaunchKernelGGL((k_xinv<T, XI_NYE>), grid, block, sh, st, g, a); break;     \
    default: hipLaunchKernelGGL((k_xinv<T, XI_OUT64>), grid, block, sh, st, g, a); break;       \
  }
  if (fp32) {
    XI_CASE(float)
  } else {
    XI_CASE(double)
  }
#undef XI_CASE
}

void launch_cg_start(CGState* cg, const double* partial, int n, double tol2, int max_iter, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_start, dim3(1), dim3(256), 0, st, cg, partial, n, tol2, max_iter);
}
void launch_cg_beta(CGState* cg, const double* partial, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_beta, dim3(1), dim3(256), 0, st, cg, partial, n);
}
void launch_cg_alpha(CGState* cg, const double* partial, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(256), 0, st, cg, partial, n);
}

int launch_colsum(const double* f, int ncomp, int64_t nvox, double* partial, hipStream_t st) {
  int nb = (int)((nvox + 2047) / 2048);
  if (nb > 1024) nb = 1024;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(k_colsum, dim3(nb), dim3(256), 0, st, f, ncomp, nvox, partial);
  return nb;
}

__global__ void k_widen(const float* in, double* out, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (double)in[i];
}

__global__ void k_negate(const double* in, double* out, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = -in[i];
}

void launch_negate(const double* in, double* out, int64_t n, hipStream_t st) {
  const int64_t nb = std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_negate, dim3((unsigned)nb), dim3(256), 0, st, in, out, n);
}

void launch_widen(const float* in, double* out, int64_t n, hipStream_t st) {
  const int64_t nb = std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_widen, dim3((unsigned)nb), dim3(256), 0, st, in, out, n);
}

int launch_sumsq(const void* f, bool fp32, int64_t n, double* partial, hipStream_t st) {
  int nb = (int)((n + 4095) / 4096);
  if (nb > 1024) nb = 1024;
  if (nb < 1) nb = 1;
  if (fp32)
    hipLaunchKernelGGL(k_sumsq<float>, dim3(nb), dim3(256), 0, st, (const float*)f, n, partial);
  else
    hipLaunchKernelGGL(k_sumsq<double>, dim3(nb), dim3(256), 0, st, (const double*)f, n, partial);
  return nb;
}

void launch_predictor(const double* F, const double* F_prev, Corr9 corr, double* out, int64_t nvox,
                      hipStream_t st) {
  const int bs = 256;
  hipLaunchKernelGGL(k_predictor, dim3((unsigned)((nvox + bs - 1) / bs)), dim3(bs), 0, st, F, F_prev, corr, out,
                     nvox);
}

}  // namespace rve
