// Plane kernels of the spectral path: for one component and one z-plane, the x (real
// to half-complex) and y transforms run back to back in LDS, so that a 3-D transform
// of a 9-component field costs one pass over the plane data plus the z pass.
//
//   forward:  field plane (ny x nx real) -> rows packed in pairs (row a + i row b) ->
//             x transform -> split into the two half spectra, stored transposed
//             [kx][y] -> y transform -> spectrum [c][z][ky][kx]
//   inverse:  the same steps reversed, then the consumer of the real plane.
//
// The conjugate-gradient iteration of eq. 18 becomes
//   k_cg_prep  (all components, streaming): x += alpha p, r -= alpha q, partial r.r,
//              y = K : r (crystal-frame tangent, rotated per grain)
//   k_plane_fwd(y)  ->  z pass with the projection  ->  k_plane_inv: w = G(K : r),
//              q = w + beta q, p = r + beta p, partial p.q
// which touches the spectrum four times per iteration.
#include "spectral.h"

#include <hip/hip_fp16.h>

#include <algorithm>
#include <type_traits>

namespace rve {

namespace {

__device__ __forceinline__ double block_sum2(double v, double* sh) {
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

// Sum of n per-block partials in a fixed order (thread t adds t, t + blockDim, ...), the
// same in every block that calls it with the same blockDim; every thread gets the sum.
__device__ __forceinline__ double sum_partials(const double* p, int n, double* red) {
  __shared__ double total;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += p[i];
  s = block_sum2(s, red);
  if (threadIdx.x == 0) total = s;
  __syncthreads();
  const double t = total;
  __syncthreads();
  return t;
}

// Threads per plane block: the plane transforms are a chain of dependent LDS stages, so
// more threads per plane (fewer points each) shorten the chain.
constexpr int kPlaneThreads = 512;
// The three-component passes of the factorised projection launch a third of the blocks of the
// nine-component ones; twice the threads per plane halve each thread's share of the chain.
constexpr int kPlane3Threads = 1024;
template <bool THREE>
constexpr int plane_threads() { return THREE ? kPlane3Threads : kPlaneThreads; }

// Source of the factorised projection's forward pass: row i of the divergence stencil,
// v_i = sum_l D_l^H y_il with D_l^H = 1/4 (S_l^-1 - 1) prod_{m != l} (1 + S_m^-1), at plane z,
// written into the packed row pairs of A (row 2p in .x, row 2p + 1 in .y).  The z factors
// are taken while loading planes z and z - 1,
//   a0 = y_i0(z) + y_i0(z-1),  a1 = y_i1(z) + y_i1(z-1),  a2 = y_i2(z-1) - y_i2(z),
// then the x factors, e = (a2 - a0)(x) + (a0 + a2)(x-1) and f = a1(x) + a1(x-1), and the y
// factors, v = 1/4 [(e - f)(y) + (e + f)(y-1)] (periodic indices).  The sums of y_il over the
// plane go to plane_sums for the zero-frequency term.  VPT bounds the voxels per thread.
template <typename T, int VPT>
__device__ __forceinline__ void plane_divergence(const GridPlan& g, const PlaneArgs& a, int i, int z, cplx<T>* A,
                                                 cplx<T>* B, int SA, double* red) {
  const int nx = g.nx, ny = g.ny, nz = g.nz, npl = nx * ny;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int64_t nv = g.nvox;
  const int zm = (z == 0 ? nz : z) - 1;
  const T* Y = reinterpret_cast<const T*>(a.in);
  const T* y0 = Y + (int64_t)(3 * i) * nv, *y1 = y0 + nv, *y2 = y1 + nv;
  const int64_t oz = (int64_t)z * npl, om = (int64_t)zm * npl;
  // two scratch planes: a0 + a2 in A's storage, a1 in B's (each holds ny nx values of T)
  T* Pl = reinterpret_cast<T*>(A);
  T* Ql = reinterpret_cast<T*>(B);
  T em[VPT], sp[VPT];
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
  for (int u = 0; u < VPT; ++u) {
    const int idx = tid + u * nthr;
    if (idx < npl) {
      const T u0 = y0[oz + idx], u1 = y1[oz + idx], u2 = y2[oz + idx];
      const T w0 = y0[om + idx], w1 = y1[om + idx], w2 = y2[om + idx];
      s0 += (double)u0;
      s1 += (double)u1;
      s2 += (double)u2;
      const T a0 = u0 + w0, a1 = u1 + w1, a2 = w2 - u2;
      em[u] = a2 - a0;
      sp[u] = a1;
      Pl[idx] = a0 + a2;
      Ql[idx] = a1;
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < VPT; ++u) {
    const int idx = tid + u * nthr;
    if (idx < npl) {
      const int y = fdiv(idx, g.fnx), x = idx - y * nx;
      const int xm = (x == 0 ? nx : x) - 1;
      const T e = em[u] + Pl[y * nx + xm];
      const T f = sp[u] + Ql[y * nx + xm];
      em[u] = e - f;
      sp[u] = e + f;
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < VPT; ++u) {
    const int idx = tid + u * nthr;
    if (idx < npl) Ql[idx] = sp[u];
  }
  __syncthreads();
  const T quarter = (T)0.25;
#pragma unroll
  for (int u = 0; u < VPT; ++u) {
    const int idx = tid + u * nthr;
    if (idx < npl) {
      const int y = fdiv(idx, g.fnx), x = idx - y * nx;
      const int ym = (y == 0 ? ny : y) - 1;
      const T v = quarter * (em[u] + Ql[ym * nx + x]);
      cplx<T>& e = A[(y >> 1) * SA + padded(x)];
      if (y & 1) e.y = v;
      else e.x = v;
    }
  }
  // an odd row count leaves the imaginary half of the last pair unset
  if (ny & 1)
    for (int x = tid; x < nx; x += nthr) A[(ny >> 1) * SA + padded(x)].y = (T)0;
  // plane sums (every thread takes part in the three reductions)
  const double t0 = block_sum2(s0, red);
  __syncthreads();
  const double t1 = block_sum2(s1, red);
  __syncthreads();
  const double t2 = block_sum2(s2, red);
  if (tid == 0) {
    a.plane_sums[(3 * i + 0) * nz + z] = t0;
    a.plane_sums[(3 * i + 1) * nz + z] = t1;
    a.plane_sums[(3 * i + 2) * nz + z] = t2;
  }
}

template <typename T, int SRC, int PPT, int RS>
__global__ void __launch_bounds__(plane_threads<SRC == PF_DIV>()) k_plane_fwd(GridPlan g, PlaneArgs a, CGState* cg) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[16];
  if (cg) {
    if (cg->done) return;
    // beta step of this iteration (one block; the others only read the stop flag, and a
    // block that already sees it set leaves its plane untransformed, which is never used)
    if (blockIdx.x == 0 && blockIdx.y == 0) {
      const double rr = sum_partials(a.rr_partial, a.n_rr, red);
      if (threadIdx.x == 0) cg_beta_update(cg, rr, a.it == 0);
    }
  }
  int c, z;
  if constexpr (SRC == PF_DIV) {
    // XCD-aware order on a 1-D grid padded to a multiple of 8: consecutive hardware block ids
    // go to the 8 XCDs in turn, and each XCD takes a contiguous run of (row, plane) in plane
    // order, so that plane z - 1, which this block reads again, is still in that XCD's L2
    const int nblk = 3 * g.nz, per = (nblk + 7) / 8;
    const int logical = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
    if (logical >= nblk) return;
    c = logical / g.nz;
    z = logical - c * g.nz;
  } else {
    c = blockIdx.x;
    z = blockIdx.y;
  }
  const int nx = g.nx, ny = g.ny, nz = g.nz, nxh = g.nxh;
  // A: npair packed rows (x lines), B: nxh columns (y lines), both padded (see padded());
  // the B lines are also skewed (see skewed_line()): the repack and the spectrum hand-off
  // touch one element of many consecutive B lines at a time
  const int npair = (ny + 1) / 2, SA = padded_len(nx), SB = padded_len(ny);
  cplx<T>* A = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* B = A + npair * SA;
  cplx<T>* twx = B + skewed_line(nxh, SB);
  cplx<T>* twy = twx + nx;
  const int64_t nv = g.nvox;
  const int64_t base = (int64_t)c * nv + (int64_t)z * ny * nx;
  const int tid = threadIdx.x, nthr = blockDim.x;
  load_twiddles(twx, g.twx, nx);
  load_twiddles(twy, g.twy, ny);
  if constexpr (SRC == PF_DIV) {
    plane_divergence<T, 2 * PPT>(g, a, c, z, A, B, SA, red);
  } else {
  // 8 independent loads in flight per thread before the LDS writes
  const int nload = 2 * npair * nx;
  for (int b0 = tid; b0 < nload; b0 += 8 * nthr) {
    T val[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = b0 + u * nthr;
      val[u] = (T)0;
      if (idx < ny * nx) {
        const int64_t o = base + idx;
        if (SRC == PF_T) val[u] = reinterpret_cast<const T*>(a.in)[o];
        else if (SRC == PF_F64) val[u] = (T)reinterpret_cast<const double*>(a.in)[o];
        else val[u] = (T)(reinterpret_cast<const double*>(a.in)[o] - ((c % 4 == 0) ? 1.0 : 0.0));
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = b0 + u * nthr;
      if (idx < nload) {
        const int y = fdiv(idx, g.fnx), x = idx - y * nx;
        cplx<T>& e = A[(y >> 1) * SA + padded(x)];
        if (y & 1) e.y = val[u];
        else e.x = val[u];
      }
    }
  }
  }
  __syncthreads();
  fft_lines<T, PPT, RS>(A, LineLayout{npair, 1, SA, 0, 0}, g.ax, twx, (T)-1);
  for (int idx = tid; idx < npair * nxh; idx += nthr) {
    const int p = fdiv(idx, g.fnxh), k = idx - p * nxh;
    const cplx<T> Zk = A[p * SA + padded(k)];
    const cplx<T> Zm = A[p * SA + padded(k == 0 ? 0 : nx - k)];
    const T h = (T)0.5;
    B[skewed_line(k, SB) + padded(2 * p)] = cmk(h * (Zk.x + Zm.x), h * (Zk.y - Zm.y));
    if (2 * p + 1 < ny) B[skewed_line(k, SB) + padded(2 * p + 1)] = cmk(h * (Zk.y + Zm.y), h * (Zm.x - Zk.x));
  }
  __syncthreads();
  fft_lines<T, PPT, RS>(B, LineLayout{nxh, 1, SB, 0, 0, 1}, g.ay, twy, (T)-1);
  cplx<T>* spec = reinterpret_cast<cplx<T>*>(a.spec);
  const int64_t sbase = ((int64_t)c * nz + z) * ny * nxh;
  for (int idx = tid; idx < ny * nxh; idx += nthr) {
    const int ky = fdiv(idx, g.fnxh), kx = idx - ky * nxh;
    spec[sbase + idx] = B[skewed_line(kx, SB) + padded(ky)];
  }
}

template <typename T, int MODE, int PPT, int RS>
__global__ void __launch_bounds__(plane_threads<MODE == PI_OUT_T>()) k_plane_inv(GridPlan g, PlaneInvArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[16];
  if (MODE == PI_CG && a.cg->done) return;
  if (MODE == PI_OUT_T && a.cg && a.cg->done) return;
  const int c = blockIdx.x, z = blockIdx.y;
  const int nx = g.nx, ny = g.ny, nz = g.nz, nxh = g.nxh;
  // A: npair packed rows (x lines), B: nxh columns (y lines), both padded (see padded());
  // the B lines are also skewed (see skewed_line()): the repack and the spectrum hand-off
  // touch one element of many consecutive B lines at a time
  const int npair = (ny + 1) / 2, SA = padded_len(nx), SB = padded_len(ny);
  cplx<T>* A = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* B = A + npair * SA;
  cplx<T>* twx = B + skewed_line(nxh, SB);
  cplx<T>* twy = twx + nx;
  const int64_t nv = g.nvox;
  const int tid = threadIdx.x, nthr = blockDim.x;
  load_twiddles(twx, g.twx, nx);
  load_twiddles(twy, g.twy, ny);
  const cplx<T>* spec = reinterpret_cast<const cplx<T>*>(a.spec);
  const int64_t sbase = ((int64_t)c * nz + z) * ny * nxh;
  for (int b0 = tid; b0 < ny * nxh; b0 += 8 * nthr) {
    cplx<T> val[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = b0 + u * nthr;
      val[u] = cmk((T)0, (T)0);
      if (idx < ny * nxh) val[u] = spec[sbase + idx];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = b0 + u * nthr;
      if (idx < ny * nxh) {
        const int ky = fdiv(idx, g.fnxh), kx = idx - ky * nxh;
        B[skewed_line(kx, SB) + padded(ky)] = val[u];
      }
    }
  }
  __syncthreads();
  fft_lines<T, PPT, RS>(B, LineLayout{nxh, 1, SB, 0, 0, 1}, g.ay, twy, (T)1);
  for (int idx = tid; idx < npair * nx; idx += nthr) {
    const int p = fdiv(idx, g.fnx), k = idx - p * nx;
    const bool hi = k >= nxh;
    const int kk = hi ? nx - k : k;
    cplx<T> Av = B[skewed_line(kk, SB) + padded(2 * p)];
    cplx<T> Bv = (2 * p + 1 < ny) ? B[skewed_line(kk, SB) + padded(2 * p + 1)] : cmk((T)0, (T)0);
    if (hi) {
      Av.y = -Av.y;
      Bv.y = -Bv.y;
    }
    A[p * SA + padded(k)] = cmk(Av.x - Bv.y, Av.y + Bv.x);
  }
  __syncthreads();
  fft_lines<T, PPT, RS>(A, LineLayout{npair, 1, SA, 0, 0}, g.ax, twx, (T)1);
  const int64_t base = (int64_t)c * nv + (int64_t)z * ny * nx;
  double acc = 0.0;
  const double beta = (MODE == PI_CG) ? a.cg->beta : 0.0;
  const double alpha = (MODE == PI_CG) ? a.cg->alpha : 0.0;   // of the previous iteration
  const bool first = (MODE == PI_CG) ? (a.cg->iter == 0) : true;
  for (int b0 = tid; b0 < ny * nx; b0 += 4 * nthr) {
    double w[4];
    T q0[4], p0[4], r0[4], x0[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = b0 + u * nthr;
      if (idx < ny * nx) {
        const int y = fdiv(idx, g.fnx), x = idx - y * nx;
        const cplx<T> e = A[(y >> 1) * SA + padded(x)];
        w[u] = (double)((y & 1) ? e.y : e.x);
        if (MODE == PI_CG) {
          // every load (x too) before the first store, which the compiler cannot move loads past
          const int64_t o = base + idx;
          r0[u] = reinterpret_cast<const T*>(a.r)[o];
          if (!first) {
            q0[u] = reinterpret_cast<const T*>(a.q)[o];
            p0[u] = reinterpret_cast<const T*>(a.p)[o];
            x0[u] = reinterpret_cast<const T*>(a.x)[o];
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = b0 + u * nthr;
      if (idx >= ny * nx) continue;
      const int64_t o = base + idx;
      if (MODE == PI_CG) {
        const T qv = first ? (T)w[u] : (T)(w[u] + beta * (double)q0[u]);
        const T pv = first ? r0[u] : (T)((double)r0[u] + beta * (double)p0[u]);
        reinterpret_cast<T*>(a.q)[o] = qv;
        reinterpret_cast<T*>(a.p)[o] = pv;
        if (!first) reinterpret_cast<T*>(a.x)[o] = (T)((double)x0[u] + alpha * (double)p0[u]);
        acc += (double)pv * (double)qv;
      } else if (MODE == PI_OUT_T) {
        reinterpret_cast<T*>(a.out)[o] = (T)w[u];
      } else if (MODE == PI_RESID) {
        const T rv = (T)(-w[u]);
        reinterpret_cast<T*>(a.r)[o] = rv;
        reinterpret_cast<T*>(a.p)[o] = rv;
        reinterpret_cast<T*>(a.x)[o] = (T)0;
        acc += (double)rv * (double)rv;
      } else {
        a.out64[o] = w[u];
      }
    }
  }
  if (MODE == PI_CG || MODE == PI_RESID) {
    const double s = block_sum2(acc, red);
    if (tid == 0) a.partial[blockIdx.y * gridDim.x + blockIdx.x] = s;
  }
  if (MODE == PI_OUT_T && z == 0) {
    // zero-frequency term of row c from the plane sums of the forward pass
    for (int l = 0; l < 3; ++l) {
      const int cc = 3 * c + l;
      const double s = sum_partials(a.plane_sums + (int64_t)cc * nz, nz, red);
      if (tid == 0) a.dc[cc] = a.mask_keep[cc] * s * a.inv_n;
    }
  }
}

// Gradient stencil of the factorised projection and the CG epilogue (see GradArgs):
//   q_ij = D_j w_i + dc_ij,  D_j = 1/4 (S_j - 1) prod_{m != j} (1 + S_m),
// from the eight corners x + {0,1}^3 of each voxel (periodic), then the previous iteration's
// x += alpha p, q = q + beta q_prev, p = r + beta p and the per-block p.q.  Grid: (blocks over
// the ny nx columns, z chunks).
template <typename T>
__global__ void __launch_bounds__(256) k_cg_grad(GridPlan g, GradArgs a) {
  __shared__ double red[8];
  const CGState* cg = a.cg;
  if (cg->done) return;
  const double beta = cg->beta;
  const double alpha = cg->alpha;   // of the previous iteration
  const bool first = cg->iter == 0;
  const int nx = g.nx, ny = g.ny, nz = g.nz, npl = nx * ny;
  const int64_t nv = g.nvox;
  const T* W = reinterpret_cast<const T*>(a.w);
  const T* Rr = reinterpret_cast<const T*>(a.r);
  T* P = reinterpret_cast<T*>(a.p);
  T* Q = reinterpret_cast<T*>(a.q);
  T* X = reinterpret_cast<T*>(a.x);
  double dc[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) dc[c] = a.dc[c];
  const int z0 = blockIdx.y * a.lz, z1 = min(z0 + a.lz, nz);
  double acc = 0.0;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < npl; idx += gridDim.x * blockDim.x) {
    const int y = fdiv(idx, g.fnx), x = idx - y * nx;
    const int x1 = x + 1 == nx ? 0 : x + 1, y1 = y + 1 == ny ? 0 : y + 1;
    // corner offsets within a plane: (y, x), (y, x+1), (y+1, x), (y+1, x+1)
    const int off[4] = {y * nx + x, y * nx + x1, y1 * nx + x, y1 * nx + x1};
    double lo[3][4], hi[3][4];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int k = 0; k < 4; ++k) lo[i][k] = (double)W[i * nv + (int64_t)z0 * npl + off[k]];
    for (int z = z0; z < z1; ++z) {
      const int zp = z + 1 == nz ? 0 : z + 1;
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 4; ++k) hi[i][k] = (double)W[i * nv + (int64_t)zp * npl + off[k]];
      const int64_t o = (int64_t)z * npl + idx;
      double qn[9];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        qn[3 * i + 0] = 0.25 * ((lo[i][1] - lo[i][0]) + (lo[i][3] - lo[i][2]) + (hi[i][1] - hi[i][0]) +
                                (hi[i][3] - hi[i][2]));
        qn[3 * i + 1] = 0.25 * ((lo[i][2] - lo[i][0]) + (lo[i][3] - lo[i][1]) + (hi[i][2] - hi[i][0]) +
                                (hi[i][3] - hi[i][1]));
        qn[3 * i + 2] = 0.25 * ((hi[i][0] - lo[i][0]) + (hi[i][1] - lo[i][1]) + (hi[i][2] - lo[i][2]) +
                                (hi[i][3] - lo[i][3]));
      }
      // every load of the voxel is issued before the first store (x too)
      T r0[9], q0[9], p0[9], x0[9];
#pragma unroll
      for (int c = 0; c < 9; ++c) {
        r0[c] = Rr[c * nv + o];
        if (!first) {
          q0[c] = Q[c * nv + o];
          p0[c] = P[c * nv + o];
          x0[c] = X[c * nv + o];
        }
      }
#pragma unroll
      for (int c = 0; c < 9; ++c) {
        const double w = qn[c] + dc[c];
        const T qv = first ? (T)w : (T)(w + beta * (double)q0[c]);
        const T pv = first ? r0[c] : (T)((double)r0[c] + beta * (double)p0[c]);
        Q[c * nv + o] = qv;
        P[c * nv + o] = pv;
        if (!first) X[c * nv + o] = (T)((double)x0[c] + alpha * (double)p0[c]);
        acc += (double)pv * (double)qv;
      }
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 4; ++k) lo[i][k] = hi[i][k];
    }
  }
  const double s = block_sum2(acc, red);
  if (threadIdx.x == 0) a.partial[blockIdx.y * gridDim.x + blockIdx.x] = s;
}

// xb = x over the grid-stride range of this thread
template <typename T>
__device__ __forceinline__ void copy_iterate(const T* X, T* XB, int64_t nv) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int c = 0; c < 9; ++c) XB[c * nv + v] = X[c * nv + v];
  }
}

// r -= alpha q (iteration > 0), partial r.r, y = K : r (sample frame; with TR,
// y = K^T : r, (K^T)_(ij)(kl) = K_(kl)(ij), for the adjoint system); the iterate is copied to
// xbest when the previous iteration set a new best r.r.  The iterate's own update x += alpha p
// is taken by the epilogue pass of the next iteration, which reads p anyway (k_cg_finish adds
// the last one).
template <typename T, int K16, int TR>
__global__ void __launch_bounds__(256, (sizeof(T) == 4 && !K16) ? 6 : 4) k_cg_prep(int64_t nv, PrepArgs a) {
  __shared__ double red[8];
  const CGState* cg = a.cg;
  if (cg->done) return;
  const bool upd = cg->iter > 0;
  // the previous iteration's iterate set a new best r.r: keep a copy before it moves
  const bool keep = upd && cg->it_best == cg->iter - 1;
  const double alpha = cg->alpha;
  T* X = reinterpret_cast<T*>(a.x);
  T* XB = reinterpret_cast<T*>(a.xbest);
  T* Rr = reinterpret_cast<T*>(a.r);
  const T* Q = reinterpret_cast<const T*>(a.q);
  // tangent in the grouped layout: G vector loads of W entries per voxel
  using KG = TangentGroups<T>;
  using KV = typename std::conditional<sizeof(T) == 4, float, double2>::type;
  const KV* K = reinterpret_cast<const KV*>(a.K);
  T* Y = reinterpret_cast<T*>(a.y);
  double acc = 0.0;
  if (keep) copy_iterate(X, XB, nv);
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
    // Every load of the voxel is issued before its first store: a store between loads keeps
    // the compiler (which cannot rule out aliasing) from moving the later loads ahead of it.
    // FP16 tangent, scaled: the tangent stream dominates the kernel's bytes, and this halves
    // it.  Entries 0-79 in ten 16-byte loads of eight, entry 80 in a 2-byte load; the packed
    // words stay packed until their product (41 registers instead of 81).
    unsigned kw[41];
    if constexpr (K16 != 0) {
      const uint4* K8 = reinterpret_cast<const uint4*>(a.K);
      const __half* Kt = reinterpret_cast<const __half*>(a.K) + 80 * nv;
#pragma unroll
      for (int gq = 0; gq < 10; ++gq) {
        const uint4 u = K8[(int64_t)gq * nv + v];
        kw[4 * gq] = u.x;
        kw[4 * gq + 1] = u.y;
        kw[4 * gq + 2] = u.z;
        kw[4 * gq + 3] = u.w;
      }
      kw[40] = (unsigned)__half_as_ushort(Kt[v]);
    }
    int gi = 0;
    if constexpr (sizeof(T) == 4) gi = a.gid[v];
    double rs[9];
    if (upd && sizeof(T) == 4) {
      T r0[9], q0[9];
#pragma unroll
      for (int c = 0; c < 9; ++c) {
        r0[c] = Rr[c * nv + v];
        q0[c] = Q[c * nv + v];
      }
#pragma unroll
      for (int c = 0; c < 9; ++c) {
        const T rn = (T)((double)r0[c] - alpha * (double)q0[c]);
        Rr[c * nv + v] = rn;
        rs[c] = (double)rn;
      }
    } else if (upd) {
      // FP64: component by component (both vectors held at once would spill)
#pragma unroll
      for (int c = 0; c < 9; ++c) {
        const int64_t o = c * nv + v;
        const T rn = (T)((double)Rr[o] - alpha * (double)Q[o]);
        Rr[o] = rn;
        rs[c] = (double)rn;
      }
    } else {
#pragma unroll
      for (int c = 0; c < 9; ++c) rs[c] = (double)Rr[c * nv + v];
    }
#pragma unroll
    for (int c = 0; c < 9; ++c) acc += rs[c] * rs[c];
    if constexpr (sizeof(T) != 4) gi = a.gid[v];
    double Rg[9], rc[9], yc[9], ys[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) Rg[i] = a.grainR[9 * gi + i];
    to_crystal(Rg, rs, rc);
    if constexpr (K16 != 0) {
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < 9; ++j) {
          const int e = TR ? j * 9 + i : i * 9 + j;
          const __half2 h2 = *reinterpret_cast<const __half2*>(&kw[e >> 1]);
          const float kf = (e & 1) ? __high2float(h2) : __low2float(h2);
          s += (double)kf * rc[j];
        }
        yc[i] = s * a.k_scale;
      }
    } else if constexpr (KG::W == 1) {
      // FP32: entry-major, loads interleaved with the products (keeps occupancy)
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < 9; ++j) s += (double)K[(int64_t)(TR ? j * 9 + i : i * 9 + j) * nv + v] * rc[j];
        yc[i] = s;
      }
    } else {
      // FP64: two entries per 16-byte load
      T kv[KG::G * KG::W];
#pragma unroll
      for (int gq = 0; gq < KG::G; ++gq) {
        const KV q = K[(int64_t)gq * nv + v];
        kv[2 * gq] = q.x;
        kv[2 * gq + 1] = q.y;
      }
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < 9; ++j) s += (double)kv[TR ? j * 9 + i : i * 9 + j] * rc[j];
        yc[i] = s;
      }
    }
    to_sample(Rg, yc, ys);
#pragma unroll
    for (int c = 0; c < 9; ++c) Y[c * nv + v] = (T)ys[c];
  }
  const double s = block_sum2(acc, red);
  if (threadIdx.x == 0) a.partial[blockIdx.x] = s;
}

// GND densities per slip system from the Nye tensor (eqs. 10-13).
__global__ void k_gnd(int64_t nv, const double* nye, const int32_t* gid, const double* grainR, const MatDev* mat,
                      double* rho_gnd) {
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
  double seg[18];
#pragma unroll
  for (int s = 0; s < 18; ++s) {
    double t = 0.0;
#pragma unroll
    for (int c = 0; c < 9; ++c) t += M.Aplus[s * 9 + c] * ac[c];
    seg[s] = t / M.burgers;
  }
#pragma unroll
  for (int al = 0; al < 12; ++al) rho_gnd[al * nv + v] = fabs(seg[al]) + 0.5 * fabs(seg[12 + M.screw_of[al]]);
}

}  // namespace

static size_t plane_lds(const GridPlan& g, bool fp32) {
  const size_t cs = fp32 ? 8 : 16;
  const size_t npair = (g.ny + 1) / 2;
  return cs * (npair * padded_len(g.nx) + (size_t)skewed_line(g.nxh, padded_len(g.ny)) + g.nx + g.ny);
}

static int plane_ppt(const GridPlan& g, int threads = kPlaneThreads) {
  const int npts = std::max(((g.ny + 1) / 2) * g.nx, g.nxh * g.ny);
  return (npts + threads - 1) / threads;
}

bool plane_fits(const GridPlan& g, bool fp32) { return plane_lds(g, fp32) <= 159 * 1024 && plane_ppt(g) <= 33; }

// bytes: LDS per work-group of the device; the kernel's static LDS is taken off it.
template <typename K>
static hipError_t lds_limit(K kernel, int bytes) {
  hipFuncAttributes fa;
  hipError_t e = hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(kernel));
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             bytes - (int)fa.sharedSizeBytes);
}

template <typename T, int PPT, int RS>
static hipError_t plane_limits_rs(int bytes) {
  hipError_t e = hipSuccess, f;
  if ((f = lds_limit(k_plane_fwd<T, PF_T, PPT, RS>, bytes)) != hipSuccess) e = f;
  if ((f = lds_limit(k_plane_fwd<T, PF_F64, PPT, RS>, bytes)) != hipSuccess) e = f;
  if ((f = lds_limit(k_plane_fwd<T, PF_FPI, PPT, RS>, bytes)) != hipSuccess) e = f;
  if ((f = lds_limit(k_plane_inv<T, PI_CG, PPT, RS>, bytes)) != hipSuccess) e = f;
  if ((f = lds_limit(k_plane_inv<T, PI_RESID, PPT, RS>, bytes)) != hipSuccess) e = f;
  if ((f = lds_limit(k_plane_inv<T, PI_OUT64, PPT, RS>, bytes)) != hipSuccess) e = f;
  if constexpr (PPT <= 9) {
    if ((f = lds_limit(k_plane_fwd<T, PF_DIV, PPT, RS>, bytes)) != hipSuccess) e = f;
    if ((f = lds_limit(k_plane_inv<T, PI_OUT_T, PPT, RS>, bytes)) != hipSuccess) e = f;
  }
  return e;
}

// planes up to PPT 9 (grids to about 96 x 96) have kernels per radix set, PPT 17 (to
// 128 x 128) for radices 8 and 2 (128 = 8 8 2); the others use the general kernels
template <typename T, int PPT>
static hipError_t plane_limits_ppt(int bytes) {
  hipError_t e = hipSuccess, f;
  if ((f = plane_limits_rs<T, PPT, RS_ALL>(bytes)) != hipSuccess) e = f;
  if constexpr (PPT <= 9) {
    if ((f = plane_limits_rs<T, PPT, RS_8>(bytes)) != hipSuccess) e = f;
    if ((f = plane_limits_rs<T, PPT, RS_8 | RS_4>(bytes)) != hipSuccess) e = f;
  }
  if constexpr (PPT <= 17) {
    if ((f = plane_limits_rs<T, PPT, RS_8 | RS_2>(bytes)) != hipSuccess) e = f;
  }
  return e;
}

hipError_t set_plane_lds_limits(int bytes) {
  hipError_t e = hipSuccess, f;
  if ((f = plane_limits_ppt<float, 5>(bytes)) != hipSuccess) e = f;
  if ((f = plane_limits_ppt<float, 9>(bytes)) != hipSuccess) e = f;
  if ((f = plane_limits_ppt<float, 17>(bytes)) != hipSuccess) e = f;
  if ((f = plane_limits_ppt<float, 33>(bytes)) != hipSuccess) e = f;
  if ((f = plane_limits_ppt<double, 5>(bytes)) != hipSuccess) e = f;
  if ((f = plane_limits_ppt<double, 9>(bytes)) != hipSuccess) e = f;
  if ((f = plane_limits_ppt<double, 17>(bytes)) != hipSuccess) e = f;
  if ((f = plane_limits_ppt<double, 33>(bytes)) != hipSuccess) e = f;
  return e;
}

// radix set of the plane kernels: the x and y transforms of the grid
static int plane_radix_set(const GridPlan& g) { return radix_set_for(radix_bits(g.ax) | radix_bits(g.ay)); }

template <typename T, int SRC, int PPT, int RS>
static void fwd_launch(const GridPlan& g, const PlaneArgs& a, CGState* cg, hipStream_t st) {
  const size_t sh = plane_lds(g, sizeof(T) == 4);
  const dim3 grid = SRC == PF_DIV ? dim3(8 * ((3 * g.nz + 7) / 8)) : dim3(9, g.nz);
  launch(k_plane_fwd<T, SRC, PPT, RS>, grid, dim3(plane_threads<SRC == PF_DIV>()), (uint32_t)sh, st, g, a, cg);
}

template <typename T, int SRC, int PPT>
static void fwd_dispatch_rs(const GridPlan& g, const PlaneArgs& a, CGState* cg, hipStream_t st) {
  switch (plane_radix_set(g)) {
    case RS_8: fwd_launch<T, SRC, PPT, RS_8>(g, a, cg, st); break;
    case RS_8 | RS_4: fwd_launch<T, SRC, PPT, RS_8 | RS_4>(g, a, cg, st); break;
    case RS_8 | RS_2: fwd_launch<T, SRC, PPT, RS_8 | RS_2>(g, a, cg, st); break;
    default: fwd_launch<T, SRC, PPT, RS_ALL>(g, a, cg, st); break;
  }
}

template <typename T, int SRC>
static void fwd_dispatch(const GridPlan& g, const PlaneArgs& a, CGState* cg, hipStream_t st) {
  const int ppt = plane_ppt(g, plane_threads<SRC == PF_DIV>());
  if constexpr (SRC == PF_DIV) {
    // compiled to 9 points per thread of 1024 (factorised_fits)
    if (ppt <= 5) fwd_dispatch_rs<T, SRC, 5>(g, a, cg, st);
    else fwd_dispatch_rs<T, SRC, 9>(g, a, cg, st);
  } else {
  if (ppt <= 5) fwd_dispatch_rs<T, SRC, 5>(g, a, cg, st);
  else if (ppt <= 9) fwd_dispatch_rs<T, SRC, 9>(g, a, cg, st);
  else if (ppt <= 17 && plane_radix_set(g) == (RS_8 | RS_2)) fwd_launch<T, SRC, 17, RS_8 | RS_2>(g, a, cg, st);
  else if (ppt <= 17) fwd_launch<T, SRC, 17, RS_ALL>(g, a, cg, st);
  else fwd_launch<T, SRC, 33, RS_ALL>(g, a, cg, st);
  }
}

void launch_plane_fwd(const GridPlan& g, bool fp32, const PlaneArgs& a, CGState* cg, hipStream_t st) {
  if (fp32) {
    if (a.src == PF_T) fwd_dispatch<float, PF_T>(g, a, cg, st);
    else if (a.src == PF_F64) fwd_dispatch<float, PF_F64>(g, a, cg, st);
    else if (a.src == PF_DIV) fwd_dispatch<float, PF_DIV>(g, a, cg, st);
    else fwd_dispatch<float, PF_FPI>(g, a, cg, st);
  } else {
    if (a.src == PF_T) fwd_dispatch<double, PF_T>(g, a, cg, st);
    else if (a.src == PF_F64) fwd_dispatch<double, PF_F64>(g, a, cg, st);
    else if (a.src == PF_DIV) fwd_dispatch<double, PF_DIV>(g, a, cg, st);
    else fwd_dispatch<double, PF_FPI>(g, a, cg, st);
  }
}

template <typename T, int MODE, int PPT, int RS>
static void inv_launch(const GridPlan& g, const PlaneInvArgs& a, hipStream_t st) {
  const size_t sh = plane_lds(g, sizeof(T) == 4);
  launch(k_plane_inv<T, MODE, PPT, RS>, dim3(MODE == PI_OUT_T ? 3 : 9, g.nz), dim3(plane_threads<MODE == PI_OUT_T>()),
         (uint32_t)sh, st, g, a);
}

template <typename T, int MODE, int PPT>
static void inv_dispatch_rs(const GridPlan& g, const PlaneInvArgs& a, hipStream_t st) {
  switch (plane_radix_set(g)) {
    case RS_8: inv_launch<T, MODE, PPT, RS_8>(g, a, st); break;
    case RS_8 | RS_4: inv_launch<T, MODE, PPT, RS_8 | RS_4>(g, a, st); break;
    case RS_8 | RS_2: inv_launch<T, MODE, PPT, RS_8 | RS_2>(g, a, st); break;
    default: inv_launch<T, MODE, PPT, RS_ALL>(g, a, st); break;
  }
}

template <typename T, int MODE>
static void inv_dispatch(const GridPlan& g, const PlaneInvArgs& a, hipStream_t st) {
  const int ppt = plane_ppt(g, plane_threads<MODE == PI_OUT_T>());
  if constexpr (MODE == PI_OUT_T) {
    if (ppt <= 5) inv_dispatch_rs<T, MODE, 5>(g, a, st);
    else inv_dispatch_rs<T, MODE, 9>(g, a, st);
  } else {
  if (ppt <= 5) inv_dispatch_rs<T, MODE, 5>(g, a, st);
  else if (ppt <= 9) inv_dispatch_rs<T, MODE, 9>(g, a, st);
  else if (ppt <= 17 && plane_radix_set(g) == (RS_8 | RS_2)) inv_launch<T, MODE, 17, RS_8 | RS_2>(g, a, st);
  else if (ppt <= 17) inv_launch<T, MODE, 17, RS_ALL>(g, a, st);
  else inv_launch<T, MODE, 33, RS_ALL>(g, a, st);
  }
}

void launch_plane_inv(const GridPlan& g, bool fp32, const PlaneInvArgs& a, hipStream_t st) {
  if (fp32) {
    if (a.mode == PI_CG) inv_dispatch<float, PI_CG>(g, a, st);
    else if (a.mode == PI_RESID) inv_dispatch<float, PI_RESID>(g, a, st);
    else if (a.mode == PI_OUT_T) inv_dispatch<float, PI_OUT_T>(g, a, st);
    else inv_dispatch<float, PI_OUT64>(g, a, st);
  } else {
    if (a.mode == PI_CG) inv_dispatch<double, PI_CG>(g, a, st);
    else if (a.mode == PI_RESID) inv_dispatch<double, PI_RESID>(g, a, st);
    else if (a.mode == PI_OUT_T) inv_dispatch<double, PI_OUT_T>(g, a, st);
    else inv_dispatch<double, PI_OUT64>(g, a, st);
  }
}

int plane_blocks(const GridPlan& g) { return 9 * g.nz; }

namespace {
// The last pending iterate update of a CG solve: x += alpha p when at least one iteration ran
// (the epilogue pass of the iteration that would have taken it returned on the stop flag, and
// a breakdown leaves alpha = 0).
template <typename T>
__global__ void k_cg_finish(const CGState* cg, T* x, const T* p, int64_t n) {
  if (cg->iter == 0) return;
  const double alpha = cg->alpha;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = (T)((double)x[i] + alpha * (double)p[i]);
}
}  // namespace

void launch_cg_finish(const CGState* cg, bool fp32, void* x, const void* p, int64_t n, hipStream_t st) {
  const int nb = (int)std::min<int64_t>((n + 255) / 256, 2048);
  if (fp32)
    hipLaunchKernelGGL(k_cg_finish<float>, dim3(nb), dim3(256), 0, st, cg, static_cast<float*>(x),
                       static_cast<const float*>(p), n);
  else
    hipLaunchKernelGGL(k_cg_finish<double>, dim3(nb), dim3(256), 0, st, cg, static_cast<double*>(x),
                       static_cast<const double*>(p), n);
}

bool factorised_fits(const GridPlan& g) { return g.freq == FREQ_ROTATED && plane_ppt(g, kPlane3Threads) <= 9; }

// Columns of 256 threads over the plane, z chunks of lz planes: the smallest lz that keeps
// the grid (and the p.q partials) at kGradBlocks blocks.
int grad_lz(const GridPlan& g) {
  const int bx = (g.nx * g.ny + 255) / 256;
  int lz = 1;
  while ((int64_t)bx * ((g.nz + lz - 1) / lz) > kGradBlocks) ++lz;
  return lz;
}

int grad_blocks(const GridPlan& g, int lz) { return ((g.nx * g.ny + 255) / 256) * ((g.nz + lz - 1) / lz); }

void launch_cg_grad(const GridPlan& g, bool fp32, const GradArgs& a, hipStream_t st) {
  const dim3 grid((g.nx * g.ny + 255) / 256, (g.nz + a.lz - 1) / a.lz);
  if (fp32) launch(k_cg_grad<float>, grid, dim3(256), 0u, st, g, a);
  else launch(k_cg_grad<double>, grid, dim3(256), 0u, st, g, a);
}

int prep_blocks(const GridPlan& g) {
  const int64_t nb = (g.nvox + 255) / 256;
  return (int)std::min<int64_t>(nb, 1024);
}

void launch_cg_prep(const GridPlan& g, bool fp32, bool k16, bool transpose, const PrepArgs& a, hipStream_t st) {
  const int nb = prep_blocks(g);
  if (transpose) launch(k_cg_prep<double, 0, 1>, dim3(nb), dim3(256), 0u, st, g.nvox, a);
  else if (fp32 && k16) launch(k_cg_prep<float, 1, 0>, dim3(nb), dim3(256), 0u, st, g.nvox, a);
  else if (fp32) launch(k_cg_prep<float, 0, 0>, dim3(nb), dim3(256), 0u, st, g.nvox, a);
  else launch(k_cg_prep<double, 0, 0>, dim3(nb), dim3(256), 0u, st, g.nvox, a);
}

void launch_gnd(int64_t nv, const double* nye, const int32_t* gid, const double* grainR, const MatDev* mat,
                double* rho_gnd, hipStream_t st) {
  const int bs = 128;
  hipLaunchKernelGGL(k_gnd, dim3((unsigned)((nv + bs - 1) / bs)), dim3(bs), 0, st, nv, nye, gid, grainR, mat,
                     rho_gnd);
}

}  // namespace rve
