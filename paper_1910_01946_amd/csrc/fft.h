// Batched 1-D complex FFTs of lines held in LDS (device side).
//
// Self-sorting mixed-radix Stockham formulation, radices 8, 4, 2, 3, 5.  For a line of
// length n = R_1 R_2 ... R_s, stage t with radix R and Ns = R_1 ... R_{t-1} maps
//   v_r = x[j + r n/R] * w^(r (j mod Ns) n/(Ns R)),  r = 0..R-1,   w = exp(sign 2 pi i / n)
//   y[(j div Ns) Ns R + (j mod Ns) + s Ns] = sum_r v_r exp(sign 2 pi i r s / R)
// for every j in [0, n/R).  Each stage reads all of its inputs into registers, then a
// barrier, then writes all outputs: the transform runs in place in one LDS buffer.
//
// Lines are addressed as base(l) + e * estride with base(l) = (l / L1) * S1 + (l % L1) * S0,
// or, with estride 0, as base(l) + padded(e).
#pragma once

#include "common.h"

namespace rve {

struct AxisPlan {
  int n;
  int nrad;
  int rad[8];
  uint32_t code;  // rad[s] in bits 4s..4s+3 (read by shifts: no indexed access on the device)
};

// Radix sets.  A kernel compiled for a set carries the stage code of those radices only:
// the FFT kernels are short chains of code that each wave runs once per launch, so code
// that a grid never uses still costs instruction-cache misses at every launch.
enum RadixSet : int { RS_8 = 1, RS_4 = 2, RS_2 = 4, RS_3 = 8, RS_5 = 16, RS_ALL = 31 };
inline int radix_bits(const AxisPlan& a) {
  int m = 0;
  for (int s = 0; s < a.nrad; ++s)
    m |= a.rad[s] == 8 ? RS_8 : a.rad[s] == 4 ? RS_4 : a.rad[s] == 2 ? RS_2 : a.rad[s] == 3 ? RS_3 : RS_5;
  return m;
}
// the compiled set that covers the radices in need
inline int radix_set_for(int need) {
  if ((need & ~RS_8) == 0) return RS_8;
  if ((need & ~(RS_8 | RS_4)) == 0) return RS_8 | RS_4;
  if ((need & ~(RS_8 | RS_2)) == 0) return RS_8 | RS_2;
  return RS_ALL;
}

// LDS slot of element e of a contiguous line with one pad slot after every 8 elements:
// radix-8 stages read 8 consecutive elements of each of several lines and write elements
// 8 apart; with this padding and a line stride of 72 (for 64-point lines) both patterns
// fall on distinct LDS banks.
__device__ __forceinline__ int padded(int e) { return e + (e >> 3); }
// line stride for n padded elements
__host__ __device__ constexpr int padded_len(int n) { return n + (n + 7) / 8; }
// Start of line l at stride S with one more pad slot after every 4 lines.  At S = 72
// (64-point lines) the same element of consecutive lines is 144 words apart, 16 banks
// mod 64, so a transpose that reads or writes one element of 32 consecutive lines per
// half-wave would hit 4 banks 8 times each; the extra slot every 4 lines spreads those 32
// lines over distinct banks, and a radix-8 stage (4 lines per half-wave) is unaffected.
__host__ __device__ constexpr int skewed_line(int l, int S) { return l * S + (l >> 2); }

struct LineLayout {
  int nlines;
  int L1, S1, S0, estride;  // estride 0: contiguous padded lines (element e at padded(e))
  int skew;                 // 1: one more pad slot after every 4 lines (see skewed_line)
  FastDiv dL1;              // division by L1; the zero value divides by 1
  __device__ __forceinline__ int base(int l) const {
    const int q = fdiv(l, dL1);
    return q * S1 + (l - q * L1) * S0 + skew * (l >> 2);
  }
  __device__ __forceinline__ int elem(int e) const { return estride ? e * estride : padded(e); }
};

template <typename T>
__device__ __forceinline__ void dft2(cplx<T>* v, T) {
  const cplx<T> a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <typename T>
__device__ __forceinline__ void dft4(cplx<T>* v, T sign) {
  const cplx<T> t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
  const cplx<T> t2 = cadd(v[1], v[3]), t3 = cmuli(csub(v[1], v[3]), sign);
  v[0] = cadd(t0, t2);
  v[2] = csub(t0, t2);
  v[1] = cadd(t1, t3);
  v[3] = csub(t1, t3);
}

template <typename T>
__device__ __forceinline__ void dft8(cplx<T>* v, T sign) {
  cplx<T> e[4] = {v[0], v[2], v[4], v[6]};
  cplx<T> o[4] = {v[1], v[3], v[5], v[7]};
  dft4(e, sign);
  dft4(o, sign);
  const T h = (T)RVE_I2;
  // w8^k = exp(sign i pi k / 4)
  const cplx<T> o1 = cmk(h * (o[1].x - sign * o[1].y), h * (o[1].y + sign * o[1].x));
  const cplx<T> o2 = cmuli(o[2], sign);
  const cplx<T> o3 = cmk(h * (-o[3].x - sign * o[3].y), h * (-o[3].y + sign * o[3].x));
  v[0] = cadd(e[0], o[0]);
  v[4] = csub(e[0], o[0]);
  v[1] = cadd(e[1], o1);
  v[5] = csub(e[1], o1);
  v[2] = cadd(e[2], o2);
  v[6] = csub(e[2], o2);
  v[3] = cadd(e[3], o3);
  v[7] = csub(e[3], o3);
}

template <typename T>
__device__ __forceinline__ void dft3(cplx<T>* v, T sign) {
  const T c = (T)-0.5, s = (T)0.86602540378443864676 * sign;
  const cplx<T> a = v[0], b = v[1], d = v[2];
  const cplx<T> sum = cadd(b, d), dif = csub(b, d);
  const cplx<T> m = cmk(a.x + c * sum.x, a.y + c * sum.y);
  v[0] = cadd(a, sum);
  v[1] = cmk(m.x - s * dif.y, m.y + s * dif.x);
  v[2] = cmk(m.x + s * dif.y, m.y - s * dif.x);
}

template <typename T>
__device__ __forceinline__ void dft5(cplx<T>* v, T sign) {
  const T c1 = (T)0.30901699437494742410, c2 = (T)-0.80901699437494742410;
  const T s1 = (T)0.95105651629515357212 * sign, s2 = (T)0.58778525229247312917 * sign;
  const cplx<T> a = v[0];
  const cplx<T> p1 = cadd(v[1], v[4]), m1 = csub(v[1], v[4]);
  const cplx<T> p2 = cadd(v[2], v[3]), m2 = csub(v[2], v[3]);
  const cplx<T> r1 = cmk(a.x + c1 * p1.x + c2 * p2.x, a.y + c1 * p1.y + c2 * p2.y);
  const cplx<T> r2 = cmk(a.x + c2 * p1.x + c1 * p2.x, a.y + c2 * p1.y + c1 * p2.y);
  // i (s1 m1 + s2 m2) and i (s2 m1 - s1 m2)
  const cplx<T> i1 = cmk(-(s1 * m1.y + s2 * m2.y), s1 * m1.x + s2 * m2.x);
  const cplx<T> i2 = cmk(-(s2 * m1.y - s1 * m2.y), s2 * m1.x - s1 * m2.x);
  v[0] = cadd(a, cadd(p1, p2));
  v[1] = cadd(r1, i1);
  v[4] = csub(r1, i1);
  v[2] = cadd(r2, i2);
  v[3] = csub(r2, i2);
}

template <typename T, int R>
__device__ __forceinline__ void dftR(cplx<T>* v, T sign) {
  if constexpr (R == 2) dft2(v, sign);
  else if constexpr (R == 3) dft3(v, sign);
  else if constexpr (R == 4) dft4(v, sign);
  else if constexpr (R == 5) dft5(v, sign);
  else dft8(v, sign);
}

// One Stockham stage over all lines.  MAXB bounds the butterflies per thread.  The
// twiddle exponent k r n / (Ns R) stays below n (k < Ns, r < R) and the output slot
// (j / Ns) Ns R + k equals (j - k) R + k, so the only divisions are by M and Ns.
template <typename T, int R, int MAXB>
__device__ __forceinline__ void fft_stage(cplx<T>* buf, const LineLayout& L, int n, int Ns,
                                          const cplx<T>* __restrict__ tw, T sign) {
  const int M = n / R;
  const FastDiv dM = make_fastdiv(M), dNs = make_fastdiv(Ns);
  const int total = L.nlines * M;
  const int nthr = blockDim.x * blockDim.y;
  const int tid = threadIdx.y * blockDim.x + threadIdx.x;
  const int twstep = fdiv(M, dNs);  // n / (Ns R)
  cplx<T> v[MAXB][R];
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    const int idx = tid + b * nthr;
    if (idx < total) {
      const int l = fdiv(idx, dM), j = idx - l * M;
      const int base = L.base(l);
#pragma unroll
      for (int r = 0; r < R; ++r) v[b][r] = buf[base + L.elem(j + r * M)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    const int idx = tid + b * nthr;
    if (idx < total) {
      const int l = fdiv(idx, dM), j = idx - l * M;
      const int base = L.base(l);
      const int k = j - fdiv(j, dNs) * Ns;
      if (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cplx<T> w = tw[k * r * twstep];
          if (sign > 0) w.y = -w.y;
          v[b][r] = cmul(v[b][r], w);
        }
      }
      dftR<T, R>(v[b], sign);
      const int out = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[base + L.elem(out + r * Ns)] = v[b][r];
    }
  }
  __syncthreads();
}

// In-place transform of every line; sign = -1 forward, +1 inverse (unnormalised).
// PPT: upper bound of (lines * n) / threads, fixed at compile time.  RS: the radices
// compiled in; the caller guarantees that it contains every radix of the plan.
template <typename T, int PPT, int RS = RS_ALL>
__device__ __forceinline__ void fft_lines(cplx<T>* buf, const LineLayout& L, const AxisPlan& ap, const cplx<T>* __restrict__ tw,
                          T sign) {
  int Ns = 1;
  for (int s = 0; s < ap.nrad; ++s) {
    const int R = (ap.code >> (4 * s)) & 15;
    if constexpr (RS == RS_8) {
      fft_stage<T, 8, (PPT + 7) / 8>(buf, L, ap.n, Ns, tw, sign);
    } else {
      switch (R) {
        case 8: fft_stage<T, 8, (PPT + 7) / 8>(buf, L, ap.n, Ns, tw, sign); break;
        case 4: if constexpr ((RS & RS_4) != 0) fft_stage<T, 4, (PPT + 3) / 4>(buf, L, ap.n, Ns, tw, sign); break;
        case 2: if constexpr ((RS & RS_2) != 0) fft_stage<T, 2, (PPT + 1) / 2>(buf, L, ap.n, Ns, tw, sign); break;
        case 3: if constexpr ((RS & RS_3) != 0) fft_stage<T, 3, (PPT + 2) / 3>(buf, L, ap.n, Ns, tw, sign); break;
        default: if constexpr ((RS & RS_5) != 0) fft_stage<T, 5, (PPT + 4) / 5>(buf, L, ap.n, Ns, tw, sign); break;
      }
    }
    Ns *= R;
  }
}

// Copy a twiddle table (n entries) into LDS; the caller synchronises before use.
template <typename T>
__device__ __forceinline__ void load_twiddles(cplx<T>* dst, const void* src, int n) {
  const cplx<T>* s = reinterpret_cast<const cplx<T>*>(src);
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = s[i];
}

}  // namespace rve
