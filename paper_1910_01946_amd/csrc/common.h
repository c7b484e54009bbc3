// Shared device/host definitions of the gfx950 library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

namespace rve {

// ------------------------------------------------------------------------------------
// Complex numbers (interleaved re/im, 8 or 16 bytes).
// ------------------------------------------------------------------------------------
template <typename T>
struct cplx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cplx<T> cmk(T a, T b) {
  cplx<T> c;
  c.x = a;
  c.y = b;
  return c;
}
template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return cmk(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return cmk(a.x - b.x, a.y - b.y); }
template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return cmk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cplx<T> cmulc(cplx<T> a, cplx<T> b) {
  return cmk(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename T>
__device__ __forceinline__ cplx<T> cscale(cplx<T> a, T s) { return cmk(a.x * s, a.y * s); }
template <typename T>
__device__ __forceinline__ cplx<T> cconj(cplx<T> a) { return cmk(a.x, -a.y); }
// multiply by s*i (s = +1 or -1)
template <typename T>
__device__ __forceinline__ cplx<T> cmuli(cplx<T> a, T s) { return cmk(-s * a.y, s * a.x); }

// ------------------------------------------------------------------------------------
// Division by a divisor fixed for a launch (grid extents, tile widths, FFT stage sizes).
// gfx950 has no integer divide instruction.  A power of two d = 2^s divides by a shift;
// any other d by one multiply-high with m = ceil(2^32 / d): with x = q d + f (0 <= f < d)
// and m = 2^32 / d + e (0 <= e < 1), x m / 2^32 = q + f / d + x e / 2^32, whose floor is
// q while x d < 2^32 (f / d <= 1 - 1/d).  Every use divides an index below 2^17 by a
// divisor below 2^9.
// ------------------------------------------------------------------------------------
struct FastDiv {
  uint32_t m;   // 0: power of two
  int32_t sh;   // log2 d when m == 0
};
__host__ __device__ inline FastDiv make_fastdiv(int d) {
  FastDiv f;
  if ((d & (d - 1)) == 0) {
    f.m = 0u;
    f.sh = d > 1 ? __builtin_ctz((unsigned)d) : 0;
  } else {
    f.m = 0xFFFFFFFFu / (uint32_t)d + 1u;
    f.sh = 0;
  }
  return f;
}
__device__ __forceinline__ int fdiv(int x, FastDiv f) {
  return f.m ? (int)__umulhi((uint32_t)x, f.m) : (x >> f.sh);
}

// ------------------------------------------------------------------------------------
// FCC slip systems {111}<110> in the crystal frame, unit vectors (plane-major order).
// s: slip direction, m: plane normal.
// ------------------------------------------------------------------------------------
#define RVE_I2 0.70710678118654752440
#define RVE_I3 0.57735026918962576451

__device__ constexpr double kSlipS[12][3] = {
    {0, RVE_I2, -RVE_I2}, {-RVE_I2, 0, RVE_I2}, {RVE_I2, -RVE_I2, 0},
    {0, RVE_I2, -RVE_I2}, {RVE_I2, 0, RVE_I2},  {RVE_I2, RVE_I2, 0},
    {0, RVE_I2, RVE_I2},  {RVE_I2, 0, -RVE_I2}, {RVE_I2, RVE_I2, 0},
    {0, RVE_I2, RVE_I2},  {RVE_I2, 0, RVE_I2},  {RVE_I2, -RVE_I2, 0}};
__device__ constexpr double kSlipM[12][3] = {
    {RVE_I3, RVE_I3, RVE_I3},  {RVE_I3, RVE_I3, RVE_I3},  {RVE_I3, RVE_I3, RVE_I3},
    {-RVE_I3, RVE_I3, RVE_I3}, {-RVE_I3, RVE_I3, RVE_I3}, {-RVE_I3, RVE_I3, RVE_I3},
    {RVE_I3, -RVE_I3, RVE_I3}, {RVE_I3, -RVE_I3, RVE_I3}, {RVE_I3, -RVE_I3, RVE_I3},
    {RVE_I3, RVE_I3, -RVE_I3}, {RVE_I3, RVE_I3, -RVE_I3}, {RVE_I3, RVE_I3, -RVE_I3}};

// ------------------------------------------------------------------------------------
// 3x3 FP64 helpers (row-major arrays of 9).
// ------------------------------------------------------------------------------------
__device__ __forceinline__ void mm3(const double* a, const double* b, double* c) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      c[3 * i + j] = a[3 * i] * b[j] + a[3 * i + 1] * b[3 + j] + a[3 * i + 2] * b[6 + j];
}
// c = a^T b
__device__ __forceinline__ void mtm3(const double* a, const double* b, double* c) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      c[3 * i + j] = a[i] * b[j] + a[3 + i] * b[3 + j] + a[6 + i] * b[6 + j];
}
// c = a b^T
__device__ __forceinline__ void mmt3(const double* a, const double* b, double* c) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      c[3 * i + j] = a[3 * i] * b[3 * j] + a[3 * i + 1] * b[3 * j + 1] + a[3 * i + 2] * b[3 * j + 2];
}
__device__ __forceinline__ double inv3(const double* a, double* r) {
  const double c00 = a[4] * a[8] - a[5] * a[7];
  const double c01 = a[2] * a[7] - a[1] * a[8];
  const double c02 = a[1] * a[5] - a[2] * a[4];
  const double c10 = a[5] * a[6] - a[3] * a[8];
  const double c11 = a[0] * a[8] - a[2] * a[6];
  const double c12 = a[2] * a[3] - a[0] * a[5];
  const double c20 = a[3] * a[7] - a[4] * a[6];
  const double c21 = a[1] * a[6] - a[0] * a[7];
  const double c22 = a[0] * a[4] - a[1] * a[3];
  const double det = a[0] * c00 + a[1] * c10 + a[2] * c20;
  const double id = 1.0 / det;
  r[0] = c00 * id; r[1] = c01 * id; r[2] = c02 * id;
  r[3] = c10 * id; r[4] = c11 * id; r[5] = c12 * id;
  r[6] = c20 * id; r[7] = c21 * id; r[8] = c22 * id;
  return det;
}
// out = R^T X R (sample -> crystal frame)
__device__ __forceinline__ void to_crystal(const double* R, const double* X, double* out) {
  double t[9];
  mtm3(R, X, t);
  mm3(t, R, out);
}
// out = R X R^T (crystal -> sample frame)
__device__ __forceinline__ void to_sample(const double* R, const double* X, double* out) {
  double t[9];
  mm3(R, X, t);
  mmt3(t, R, out);
}

}  // namespace rve
