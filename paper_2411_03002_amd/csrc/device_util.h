// Device helpers: minimum image, exactly ordered squared distance, f_cut, reductions.
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"
#include "exp_table_gen.h"

namespace apx {

constexpr int kWave = 64;
constexpr int kXcds = 8;  // accelerator complex dies of an MI355X, each with its own L2

// Workgroups are handed to the XCDs round-robin (hardware block b runs on XCD b % 8).
// Gather kernels read the data of spatial neighbours, so consecutive logical blocks
// should share an L2: this maps hardware block b to a logical block such that every XCD
// works through one contiguous range of logical blocks (a bijection on [0, nb)).
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int q = nb / kXcds, r = nb % kXcds;
  const int x = b % kXcds, k = b / kXcds;
  return x * q + (x < r ? x : r) + k;
}

// Minimum image of d = x_j - x_i along one axis of length L (both coordinates in
// [lo, hi)): d -= L if d >= L/2; d += L if d < -L/2.  (Written as branches: few pairs
// wrap, and in the thread-per-atom gathers a branch no lane takes costs less than forming
// both shifted values.)
__device__ __forceinline__ double min_image(double d, double L, double half, int periodic) {
  if (periodic) {
    if (d >= half) d -= L;
    else if (d < -half) d += L;
  }
  return d;
}

// The same value formed without branches (both shifted values and selects): cheaper in the
// ACE basis and force kernels (a wave per atom, lanes over its neighbours), where it took
// 8-9% off each.
__device__ __forceinline__ double min_image_sel(double d, double L, double half, int periodic) {
  const double dm = d - L, dp = d + L;
  double r = d >= half ? dm : d;
  r = d < -half ? dp : r;
  return periodic ? r : d;
}

// (dx*dx + dy*dy) + dz*dz with every product and sum rounded separately.
__device__ __forceinline__ double sq_dist_exact(double dx, double dy, double dz) {
#pragma clang fp contract(off)
  double a = dx * dx;
  double b = dy * dy;
  double c = dz * dz;
  return (a + b) + c;
}

// f_cut of the paper (Appendix B), evaluated as ((1 - 1.875x) + 1.25x^3) - 0.375x^5 with
// x^3 = (x*x)*x and x^5 = x^3*(x*x), no fused operations.
__device__ __forceinline__ double fcut_exact(double x) {
#pragma clang fp contract(off)
  if (x < 0.0) return 1.0;
  if (x > 1.0) return 0.0;
  double x2 = x * x;
  double x3 = x2 * x;
  double x5 = x3 * x2;
  double t1 = 1.875 * x;
  double t3 = 1.25 * x3;
  double t5 = 0.375 * x5;
  return ((1.0 - t1) + t3) - t5;
}

// ------------------------------------------------------- fast FP64 elementary functions
// The pair loops evaluate exponentials, reciprocals and square roots per neighbour; these
// forms give up the last ulp or two for fewer FP64 instructions.

// exp(x) by Tang's table-driven method (ACM TOMS 15(2), 1989) with 32 entries:
// x = (32 m + j) ln2/32 + r, |r| <= ln2/64 (reduction constant in two parts), and
// exp(x) = 2^m 2^(j/32) exp(r) with exp(r) - 1 from its Taylor polynomial to degree 6
// (truncation below 2e-18).  `tab` holds kExp2Table (staged in LDS: the index diverges
// across lanes).  For x below -708 the result underflows to 0 through the scaling.
__device__ __forceinline__ double exp_tab(double x, const double* tab) {
  const double k = rint(x * kInvLn2x32);
  const double r = fma(-k, kLn2d32Lo, fma(-k, kLn2d32Hi, x));
  const int ki = (int)k;
  double p = fma(r, 1.0 / 720.0, 1.0 / 120.0);
  p = fma(r, p, 1.0 / 24.0);
  p = fma(r, p, 1.0 / 6.0);
  p = fma(r, p, 0.5);
  p = fma(r, p, 1.0);
  p *= r;
  const double t = tab[ki & 31];
  return ldexp(fma(t, p, t), ki >> 5);
}

// 1/a from the hardware estimate refined by two Newton steps.
__device__ __forceinline__ double rcp_nr(double a) {
  double y = __builtin_amdgcn_rcp(a);
  double e = fma(-a, y, 1.0);
  y = fma(y, e, y);
  e = fma(-a, y, 1.0);
  return fma(y, e, y);
}

// 1/sqrt(a) from the hardware estimate refined by two Newton steps y (3 - a y^2)/2.
__device__ __forceinline__ double rsq_nr(double a) {
  double y = __builtin_amdgcn_rsq(a);
  const double h = 0.5 * a;
  y = y * fma(-h * y, y, 1.5);
  return y * fma(-h * y, y, 1.5);
}

// Stages kExp2Table in LDS; every thread of the block must call it before any returns.
__device__ __forceinline__ void stage_exp_table(double* sh) {
  if (threadIdx.x < 32) sh[threadIdx.x] = kExp2Table[threadIdx.x];
  __syncthreads();
}

// atomicMax on a single global word that many waves update: a device-scope load (from L2,
// not a stale L1 line) first, and the atomic only when v exceeds the value seen.  Atomics
// to one address serialise in one L2 channel; most callers find the maximum already set.
__device__ __forceinline__ void sparse_atomic_max(int* p, int v) {
  if (v > __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(p, v);
}
__device__ __forceinline__ void sparse_atomic_max(unsigned long long* p, unsigned long long v) {
  if (v > __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(p, v);
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

template <class T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    T o = __shfl_xor(v, off, kWave);
    v = o > v ? o : v;
  }
  return v;
}

// Box lengths for minimum-image displacements.
struct BoxDev {
  double L[3], half[3];
  int per[3];
};

inline BoxDev make_box(const apx_atoms* a) {
  BoxDev b;
  for (int d = 0; d < 3; ++d) {
    b.L[d] = a->hi[d] - a->lo[d];
    b.half[d] = 0.5 * b.L[d];
    b.per[d] = a->periodic[d] ? 1 : 0;
  }
  return b;
}

__device__ __forceinline__ int cell_coord(double x, double lo, double inv_cell, int nc) {
  int c = (int)floor((x - lo) * inv_cell);
  return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

}  // namespace apx
