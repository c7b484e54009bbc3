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

template <typename T, int SRC, int PPT, int RS>
__global__ void __launch_bounds__(kPlaneThreads) k_plane_fwd(GridPlan g, PlaneArgs a, CGState* cg) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[8];
  if (cg) {
    if (cg->done) return;
    // beta step of this iteration (one block; the others only read the stop flag, and a
    // block that already sees it set leaves its plane untransformed, which is never used)
    if (blockIdx.x == 0 && blockIdx.y == 0) {
      const double rr = sum_partials(a.rr_partial, a.n_rr, red);
      if (threadIdx.x == 0) cg_beta_update(cg, rr, a.it == 0);
    }
  }
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
  const int64_t base = (int64_t)c * nv + (int64_t)z * ny * nx;
  const int tid = threadIdx.x, nthr = blockDim.x;
  load_twiddles(twx, g.twx, nx);
  load_twiddles(twy, g.twy, ny);
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
__global__ void __launch_bounds__(kPlaneThreads) k_plane_inv(GridPlan g, PlaneInvArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[8];
  if (MODE == PI_CG && a.cg->done) return;
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
  const bool first = (MODE == PI_CG) ? (a.cg->iter == 0) : true;
  for (int b0 = tid; b0 < ny * nx; b0 += 4 * nthr) {
    double w[4];
    T q0[4], p0[4], r0[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = b0 + u * nthr;
      if (idx < ny * nx) {
        const int y = fdiv(idx, g.fnx), x = idx - y * nx;
        const cplx<T> e = A[(y >> 1) * SA + padded(x)];
        w[u] = (double)((y & 1) ? e.y : e.x);
        if (MODE == PI_CG) {
          const int64_t o = base + idx;
          r0[u] = reinterpret_cast<const T*>(a.r)[o];
          if (!first) {
            q0[u] = reinterpret_cast<const T*>(a.q)[o];
            p0[u] = reinterpret_cast<const T*>(a.p)[o];
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
        acc += (double)pv * (double)qv;
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
}

// xb = x over the grid-stride range of this thread
template <typename T>
__device__ __forceinline__ void copy_iterate(const T* X, T* XB, int64_t nv) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int c = 0; c < 9; ++c) XB[c * nv + v] = X[c * nv + v];
  }
}

// x += alpha p, r -= alpha q (iteration > 0), partial r.r, y = K : r (sample frame; with TR,
// y = K^T : r, (K^T)_(ij)(kl) = K_(kl)(ij), for the adjoint system); the iterate is copied to
// xbest first when the previous iteration set a new best r.r.
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
  const T* P = reinterpret_cast<const T*>(a.p);
  const T* Q = reinterpret_cast<const T*>(a.q);
  // tangent in the grouped layout: G vector loads of W entries per voxel
  using KG = TangentGroups<T>;
  using KV = typename std::conditional<sizeof(T) == 4, float, double2>::type;
  const KV* K = reinterpret_cast<const KV*>(a.K);
  T* Y = reinterpret_cast<T*>(a.y);
  double acc = 0.0;
  if (keep) copy_iterate(X, XB, nv);
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
    double rs[9];
    if (upd) {
#pragma unroll
      for (int c = 0; c < 9; ++c) {
        const int64_t o = c * nv + v;
        X[o] = (T)((double)X[o] + alpha * (double)P[o]);
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
    const int gi = a.gid[v];
    double Rg[9], rc[9], yc[9], ys[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) Rg[i] = a.grainR[9 * gi + i];
    to_crystal(Rg, rs, rc);
    if constexpr (K16 != 0) {
      // FP16 pairs (41 4-byte loads per voxel), scaled: the tangent stream dominates the
      // kernel's bytes, and this halves it
      const __half2* K2 = reinterpret_cast<const __half2*>(a.K);
      float kv[82];
#pragma unroll
      for (int gq = 0; gq < 41; ++gq) {
        const float2 f = __half22float2(K2[(int64_t)gq * nv + v]);
        kv[2 * gq] = f.x;
        kv[2 * gq + 1] = f.y;
      }
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < 9; ++j) s += (double)kv[TR ? j * 9 + i : i * 9 + j] * rc[j];
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

static int plane_ppt(const GridPlan& g) {
  const int npts = std::max(((g.ny + 1) / 2) * g.nx, g.nxh * g.ny);
  return (npts + kPlaneThreads - 1) / kPlaneThreads;
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
  launch(k_plane_fwd<T, SRC, PPT, RS>, dim3(9, g.nz), dim3(kPlaneThreads), (uint32_t)sh, st, g, a, cg);
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
  const int ppt = plane_ppt(g);
  if (ppt <= 5) fwd_dispatch_rs<T, SRC, 5>(g, a, cg, st);
  else if (ppt <= 9) fwd_dispatch_rs<T, SRC, 9>(g, a, cg, st);
  else if (ppt <= 17 && plane_radix_set(g) == (RS_8 | RS_2)) fwd_launch<T, SRC, 17, RS_8 | RS_2>(g, a, cg, st);
  else if (ppt <= 17) fwd_launch<T, SRC, 17, RS_ALL>(g, a, cg, st);
  else fwd_launch<T, SRC, 33, RS_ALL>(g, a, cg, st);
}

void launch_plane_fwd(const GridPlan& g, bool fp32, const PlaneArgs& a, CGState* cg, hipStream_t st) {
  if (fp32) {
    if (a.src == PF_T) fwd_dispatch<float, PF_T>(g, a, cg, st);
    else if (a.src == PF_F64) fwd_dispatch<float, PF_F64>(g, a, cg, st);
    else fwd_dispatch<float, PF_FPI>(g, a, cg, st);
  } else {
    if (a.src == PF_T) fwd_dispatch<double, PF_T>(g, a, cg, st);
    else if (a.src == PF_F64) fwd_dispatch<double, PF_F64>(g, a, cg, st);
    else fwd_dispatch<double, PF_FPI>(g, a, cg, st);
  }
}

template <typename T, int MODE, int PPT, int RS>
static void inv_launch(const GridPlan& g, const PlaneInvArgs& a, hipStream_t st) {
  const size_t sh = plane_lds(g, sizeof(T) == 4);
  launch(k_plane_inv<T, MODE, PPT, RS>, dim3(9, g.nz), dim3(kPlaneThreads), (uint32_t)sh, st, g, a);
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
  const int ppt = plane_ppt(g);
  if (ppt <= 5) inv_dispatch_rs<T, MODE, 5>(g, a, st);
  else if (ppt <= 9) inv_dispatch_rs<T, MODE, 9>(g, a, st);
  else if (ppt <= 17 && plane_radix_set(g) == (RS_8 | RS_2)) inv_launch<T, MODE, 17, RS_8 | RS_2>(g, a, st);
  else if (ppt <= 17) inv_launch<T, MODE, 17, RS_ALL>(g, a, st);
  else inv_launch<T, MODE, 33, RS_ALL>(g, a, st);
}

void launch_plane_inv(const GridPlan& g, bool fp32, const PlaneInvArgs& a, hipStream_t st) {
  if (fp32) {
    if (a.mode == PI_CG) inv_dispatch<float, PI_CG>(g, a, st);
    else if (a.mode == PI_RESID) inv_dispatch<float, PI_RESID>(g, a, st);
    else inv_dispatch<float, PI_OUT64>(g, a, st);
  } else {
    if (a.mode == PI_CG) inv_dispatch<double, PI_CG>(g, a, st);
    else if (a.mode == PI_RESID) inv_dispatch<double, PI_RESID>(g, a, st);
    else inv_dispatch<double, PI_OUT64>(g, a, st);
  }
}

int plane_blocks(const GridPlan& g) { return 9 * g.nz; }

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
