// Atomic cluster expansion on the active atoms: atomic base, product basis with energy
// and adjoint, force scatter.
//
// Three kernels per evaluation (Sec. III A form E = phi1 + F_eps(phi2), basis defined in
// the ABI header):
//  1. k_ace_basis    one wave per active atom: per neighbour the Chebyshev radial values
//                    and real solid harmonics, A'[k][lm] = sum_j g_k S_lm, then the radial
//                    mixing A[n][lm] = sum_k Wp[l][n][k] A'[k][lm] (Wp folds W, N_l, 1/s_a).
//  2. k_ace_products lane = atom, 64 (fp32) or 32 (fp64) atoms per block held in LDS,
//                    16 (fp32) or 8 (fp64) waves dealt the coupling list round-robin;
//                    the list is sorted by coupling type for instruction-cache locality.  B3 is evaluated by recoupling:
//                    for a label pair (p1, p2) the coupled product
//                    P_LM = sum G(l1 l2 L; m1 m2 M) A_p1m1 A_p2m2 is formed once and every
//                    third block p3 >= p2 of degree L contributes B = sum_M P_LM A_p3M.
//                    The adjoint pass reuses the same structure with
//                    d = c1 + F_eps'(phi2) c2: Abar_p3 += d P, Pbar += d A_p3, then Pbar
//                    is pushed back through the coupling into Abar_p1, Abar_p2.
//  3. k_ace_force    one wave per active atom: back-projection of Abar through Wp, then
//                    per neighbour the gradient of sum Abar'' g_k S_lm, scattered as
//                    F_j -= w_i dE_i/dr_ij, F_i += w_i dE_i/dr_ij (float64 atomics).
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "ace_coupling_gen.h"
#include "ace_model.h"
#include "device_util.h"

namespace apx {

struct AnchorDev {
  double A, alpha, beta, r0, rc, inv_h, rc2;
  int on;
};

template <class T>
struct AceScratch {
  T* A;             // [n_act][na]
  T* Ab;            // [n_act][na], or [tile][na][tile_size] when tile_size > 0
  int tile_size;
  double* e_anch;   // [n_act]
  double* fp_anch;  // [n_act]
  T* fp;            // [tiles * tile_size] embedding slope F_eps'(phi2) per atom (float32 path)
};

// ------------------------------------------------------------ shared helpers
// Reads a read-only table entry (a scalar type) through the constant address space.  The
// product kernels store to global memory, so the compiler cannot prove their table reads
// unclobbered and would issue vector loads; constant-space reads let it use scalar loads.
template <class X>
__device__ __forceinline__ X cld(const X* p) {
  return *(const __attribute__((address_space(4))) X*)p;
}

template <class T, int LMAX, bool GRAD>
__device__ __forceinline__ void solid_harmonics(T x, T y, T z, T* S, T* Sx, T* Sy, T* Sz) {
  S[0] = T(1);
  if constexpr (GRAD) { Sx[0] = T(0); Sy[0] = T(0); Sz[0] = T(0); }
#pragma unroll
  for (int l = 0; l < LMAX; ++l) {
    const T c = (l == 0) ? T(1) : T(sqrt((2.0 * l + 1.0) / (2.0 * l + 2.0)));
    const int sll = l * l + 2 * l;  // (l, l)
    const int slm = l * l;          // (l, -l)
    const int tp = (l + 1) * (l + 1) + 2 * (l + 1);
    const int bt = (l + 1) * (l + 1);
    if (l == 0) {
      S[tp] = c * x * S[sll];
      S[bt] = c * y * S[sll];
      if constexpr (GRAD) {
        Sx[tp] = c * S[sll]; Sy[tp] = T(0); Sz[tp] = T(0);
        Sx[bt] = T(0); Sy[bt] = c * S[sll]; Sz[bt] = T(0);
      }
    } else {
      S[tp] = c * (x * S[sll] - y * S[slm]);
      S[bt] = c * (y * S[sll] + x * S[slm]);
      if constexpr (GRAD) {
        Sx[tp] = c * (S[sll] + x * Sx[sll] - y * Sx[slm]);
        Sy[tp] = c * (x * Sy[sll] - S[slm] - y * Sy[slm]);
        Sz[tp] = c * (x * Sz[sll] - y * Sz[slm]);
        Sx[bt] = c * (y * Sx[sll] + S[slm] + x * Sx[slm]);
        Sy[bt] = c * (S[sll] + y * Sy[sll] + x * Sy[slm]);
        Sz[bt] = c * (y * Sz[sll] + x * Sz[slm]);
      }
    }
#pragma unroll
    for (int m = -l; m <= l; ++m) {
      const int dst = (l + 1) * (l + 1) + (l + 1) + m;
      const int s1 = l * l + l + m;
      const T a = T((2.0 * l + 1.0) / sqrt((l + m + 1.0) * (l - m + 1.0)));
      if (m >= -(l - 1) && m <= l - 1) {
        const int s2 = (l - 1) * (l - 1) + (l - 1) + m;
        const T b = T(sqrt((l + m) * (l - m) * 1.0) / sqrt((l + m + 1.0) * (l - m + 1.0)));
        S[dst] = a * z * S[s1] - b * S[s2];
        if constexpr (GRAD) {
          Sx[dst] = a * z * Sx[s1] - b * (T(2) * x * S[s2] + Sx[s2]);
          Sy[dst] = a * z * Sy[s1] - b * (T(2) * y * S[s2] + Sy[s2]);
          Sz[dst] = a * (S[s1] + z * Sz[s1]) - b * (T(2) * z * S[s2] + Sz[s2]);
        }
      } else {
        S[dst] = a * z * S[s1];
        if constexpr (GRAD) {
          Sx[dst] = a * z * Sx[s1];
          Sy[dst] = a * z * Sy[s1];
          Sz[dst] = a * (S[s1] + z * Sz[s1]);
        }
      }
    }
  }
}

// Reciprocal in the evaluation type: the hardware estimate (1 ulp) in float32, two Newton
// steps on it in float64.
template <class T>
__device__ __forceinline__ T rcp_t(T a) {
  if constexpr (sizeof(T) == 4) return __builtin_amdgcn_rcpf(a);
  else return rcp_nr(a);
}

__device__ __forceinline__ void taper_d(double x, double& p, double& dp) {
  const double x2 = x * x;
  const double x4 = x2 * x2;
  const double den = rcp_nr(1.0 + x4);
  p = x4 * den;
  dp = 4.0 * x2 * x * den * den;
}

template <class T>
__device__ __forceinline__ void taper_t(T x, T& p, T& dp) {
  const T x2 = x * x;
  const T x4 = x2 * x2;
  const T den = rcp_t<T>(T(1) + x4);
  p = x4 * den;
  dp = T(4) * x2 * x * den * den;
}

typedef float floatx4 __attribute__((ext_vector_type(4)));

// LDS layout of the atomic-base kernel: per neighbour slot (columns, row stride kStride)
// the radial values g_k (12 rows) and solid harmonics S_lm (LM rows); A' reuses the space
// once the contraction is done.  Float32 contracts on the matrix cores.
template <class T, int LMAX>
struct BasisLds {
  static constexpr int LM = (LMAX + 1) * (LMAX + 1);
  static constexpr bool kMfma = sizeof(T) == 4;
  static constexpr int kStride = kMfma ? 66 : 65;
  static constexpr int kGRows = 12;
  static constexpr int kSRows = LM;
  static constexpr size_t bytes() { return sizeof(T) * ((size_t)(kGRows + kSRows) * kStride); }
  static_assert(12 * LM <= (kGRows + kSRows) * kStride, "A' fits in the neighbour tables");
};

// ------------------------------------------------------------------ kernel 1
template <class T, int LMAX>
__global__ void __launch_bounds__(64) k_ace_basis(const double* __restrict__ pos, int n, BoxDev b,
                                                  const int* __restrict__ count, const int* __restrict__ idx,
                                                  int max_nb, const int* __restrict__ active, int n_act,
                                                  int K, T rc, T inv_h, double rc2, const T* __restrict__ Wp,
                                                  AnchorDev an, AceScratch<T> sc) {
  constexpr int LM = (LMAX + 1) * (LMAX + 1);
  constexpr int kMaxK = 12;
  constexpr bool MF = BasisLds<T, LMAX>::kMfma;
  constexpr int ST = BasisLds<T, LMAX>::kStride, GR = BasisLds<T, LMAX>::kGRows, SR = BasisLds<T, LMAX>::kSRows;
  extern __shared__ double smem_raw[];
  T* gS = reinterpret_cast<T*>(smem_raw);  // [GR][ST]: g_k per neighbour slot
  T* sS = gS + GR * ST;                    // [SR][ST]: S_lm per neighbour slot
  T* Ap = gS;                              // [K*LM], after the contraction
  __shared__ double etab[32];
  stage_exp_table(etab);
  const int q = xcd_block(blockIdx.x, gridDim.x);
  const int lane = threadIdx.x;
  const int i = active[q];
  const double xi = pos[i], yi = pos[(size_t)n + i], zi = pos[2 * (size_t)n + i];
  int cnt = count[i];
  if (cnt > max_nb) cnt = max_nb;
  const int nout = K * LM;
  T acc[5];
#pragma unroll
  for (int s = 0; s < 5; ++s) acc[s] = T(0);
  floatx4 D0 = {0.f, 0.f, 0.f, 0.f}, D1 = {0.f, 0.f, 0.f, 0.f};
  double rho_a = 0.0, pair_a = 0.0;
  const T two_rc = T(2) / rc;
  for (int c0 = 0; c0 < cnt; c0 += 64) {
    const int k = c0 + lane;
    T g[kMaxK];
    T S[LM];
    bool inside = false;
#pragma unroll
    for (int a = 0; a < kMaxK; ++a) g[a] = T(0);
#pragma unroll
    for (int a = 0; a < LM; ++a) S[a] = T(0);
    if (k < cnt) {
      const int j = idx[(size_t)k * n + i];
      const double dx = min_image_sel(pos[j] - xi, b.L[0], b.half[0], b.per[0]);
      const double dy = min_image_sel(pos[(size_t)n + j] - yi, b.L[1], b.half[1], b.per[1]);
      const double dz = min_image_sel(pos[2 * (size_t)n + j] - zi, b.L[2], b.half[2], b.per[2]);
      const double r2 = dx * dx + dy * dy + dz * dz;
      const double ird = rsq_nr(r2);
      const double rd = r2 * ird;
      inside = r2 < rc2;
      if (inside) {
        const T r = T(rd);
        const T ir = T(ird);
        const T x = r * two_rc - T(1);
        T ps, dps;
        taper_t<T>((r - rc) * inv_h, ps, dps);
        T t0 = T(1), t1 = x;
        g[0] = ps;
        if (K > 1) g[1] = x * ps;
#pragma unroll
        for (int a = 2; a < kMaxK; ++a) {
          const T t2 = T(2) * x * t1 - t0;
          if (a < K) g[a] = t2 * ps;
          t0 = t1;
          t1 = t2;
        }
        solid_harmonics<T, LMAX, false>(T(dx) * ir, T(dy) * ir, T(dz) * ir, S, nullptr, nullptr, nullptr);
      }
      if (an.on && r2 < an.rc2) {
        double ps, dps;
        taper_d((rd - an.rc) * an.inv_h, ps, dps);
        rho_a += exp_tab(-an.beta * (rd - an.r0), etab) * ps;
        pair_a += exp_tab(-an.alpha * (rd - an.r0), etab) * ps;
      }
    }
    // neighbour slot of the lane: float32 compacts the neighbours inside the cutoff to the
    // front (the others, all zero, follow), so that the matrix steps stop after them
    int slot = lane, steps = 0;
    if constexpr (MF) {
      const unsigned long long m = __ballot(inside);
      const int nv = __popcll(m);
      const int below = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
      slot = inside ? below : nv + (lane - below);
      steps = (nv + 3) >> 2;
    }
#pragma unroll
    for (int a = 0; a < kMaxK; ++a)
      if (a < K) gS[a * ST + slot] = g[a];
#pragma unroll
    for (int a = 0; a < LM; ++a) sS[a * ST + slot] = S[a];
    __syncthreads();
    if constexpr (MF) {
      // A'[k][lm] += sum over 4 slots per step of g[k][slot] S[lm][slot] on the matrix
      // cores (16 x 16 x 4 float32): lane = row/column (lane % 16) and slot in the step
      // (lane / 16), operand rows beyond K and LM are zero; the row stride of 66 keeps
      // the two lane halves on distinct banks
      const int col = lane & 15, sub = lane >> 4;
      const bool g_row = col < K, s_row = 16 + col < LM;
      for (int st = 0; st < steps; ++st) {
        const int sl = 4 * st + sub;
        const float av = g_row ? gS[col * ST + sl] : 0.f;
        D0 = __builtin_amdgcn_mfma_f32_16x16x4f32(av, sS[col * ST + sl], D0, 0, 0, 0);
        if constexpr (LM > 16)
          D1 = __builtin_amdgcn_mfma_f32_16x16x4f32(av, s_row ? sS[(16 + col) * ST + sl] : 0.f, D1, 0, 0, 0);
      }
    } else {
      const int lim = (cnt - c0) < 64 ? (cnt - c0) : 64;
#pragma unroll
      for (int s = 0; s < 5; ++s) {
        const int o = lane + 64 * s;
        if (o < nout) {
          const int kk = o / LM, lm = o - kk * LM;
          T v = acc[s];
          for (int nb = 0; nb < lim; ++nb) v += gS[kk * ST + nb] * sS[lm * ST + nb];
          acc[s] = v;
        }
      }
    }
    __syncthreads();
  }
  if constexpr (MF) {
    // accumulator layout: row k = 4 (lane / 16) + r, column lane % 16 (+ 16 for D1)
    const int col = lane & 15, sub = lane >> 4;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int k = 4 * sub + r;
      if (k < K) {
        Ap[k * LM + col] = D0[r];
        if (16 + col < LM) Ap[k * LM + 16 + col] = D1[r];
      }
    }
  } else {
#pragma unroll
    for (int s = 0; s < 5; ++s) {
      const int o = lane + 64 * s;
      if (o < nout) Ap[o] = acc[s];
    }
  }
  __syncthreads();
  const int na = K * LM;
  T* Arow = sc.A + (size_t)q * na;
  for (int o = lane; o < na; o += 64) {
    const int nn = o / LM, lm = o - nn * LM;
    int l = 0;
    while ((l + 1) * (l + 1) <= lm) ++l;
    const T* w = Wp + ((size_t)l * K + nn) * K;
    T v = T(0);
    for (int kk = 0; kk < K; ++kk) v += w[kk] * Ap[kk * LM + lm];
    Arow[o] = v;
  }
  if (an.on) {
    rho_a = wave_sum(rho_a);
    pair_a = wave_sum(pair_a);
    if (lane == 0) {
      const double sq = sqrt(rho_a);
      sc.e_anch[q] = (rho_a > 0.0 ? -sq : 0.0) + 0.5 * an.A * pair_a;
      sc.fp_anch[q] = rho_a > 0.0 ? -0.5 / sq : 0.0;
    }
  } else if (lane == 0) {
    sc.e_anch[q] = 0.0;
    sc.fp_anch[q] = 0.0;
  }
}

// ------------------------------------------------------------------ kernel 2
template <class T>
struct Acc {
  T s1, s2, e1, e2;  // running sums and compensation terms
};

template <class T, bool COMP>
__device__ __forceinline__ void acc_add(T& s, T& e, T c, T B) {
  if constexpr (COMP) {
    // TwoProduct (via fma) and TwoSum: the dot-product compensation of Ogita, Rump and
    // Oishi (2005), accumulating the rounding errors separately
    const T p = c * B;
    const T pe = fma(c, B, -p);
    const T sn = s + p;
    const T bp = sn - s;
    const T se = (s - (sn - bp)) + (p - bp);
    s = sn;
    e += se + pe;
  } else {
    s = fma(c, B, s);
  }
}

// Adds x to the compensated sum (s, e): TwoSum, the rounding error kept in e.
template <class T, bool COMP>
__device__ __forceinline__ void acc_sum(T& s, T& e, T x) {
  if constexpr (COMP) {
    const T sn = s + x;
    const T bp = sn - s;
    e += (s - (sn - bp)) + (x - bp);
    s = sn;
  } else {
    s += x;
  }
}

template <class T, int TILE>
__device__ __forceinline__ void lds_add(T* p, T v, bool on) {
  if (on) atomicAdd(p, v);
}

template <class T, int LMAX, int TILE, bool COMP, int L1, int L2>
__device__ __forceinline__ void pair_fwd(const T* __restrict__ As, const int* rec, const AceTables<T>& tb, int t,
                                         Acc<T>& acc) {
  using C = Couple<LMAX, L1, L2>;
  constexpr int P2 = (LMAX + 1) * (LMAX + 1);
  constexpr int ST = TILE + 1;
  const int o1 = rec[0], o2 = rec[1];
  T a[2 * L1 + 1], bb[2 * L2 + 1], P[P2];
#pragma unroll
  for (int m = 0; m < 2 * L1 + 1; ++m) a[m] = As[(o1 + m) * ST + t];
#pragma unroll
  for (int m = 0; m < 2 * L2 + 1; ++m) bb[m] = As[(o2 + m) * ST + t];
#pragma unroll
  for (int m = 0; m < P2; ++m) P[m] = T(0);
  C::template fwd<T>(a, bb, P);
#pragma unroll
  for (int L = 0; L <= LMAX; ++L) {
    if ((C::kMask >> L) & 1) {
      const int q0 = rec[4 + L], q1 = rec[5 + L];
      const int o3b = rec[10 + L];
#pragma unroll 2
      for (int q = q0; q < q1; ++q) {
        const int o3 = o3b + (q - q0) * P2;
        const Coef2<T> c = tb.tc[q];
        T B = T(0);
#pragma unroll
        for (int mm = 0; mm < 2 * L + 1; ++mm) B = fma(P[L * L + mm], As[(o3 + mm) * ST + t], B);
        acc_add<T, COMP>(acc.s1, acc.e1, c.c1, B);
        acc_add<T, COMP>(acc.s2, acc.e2, c.c2, B);
      }
    }
  }
}

// Energy contribution of one label pair with the third-block loop unrolled over the
// radial index (coefficient loads of a segment issued together).  The pair's terms c.B
// (at most (l_max + 1) n_max of them) are summed by fused multiply-adds, and the pair's
// two partial sums enter the running sums with compensation.
// The pair's third blocks of degree L: P_LM by the per-degree coupling, then B = P.A_n3L
// for the pair's run of n3 (wave-uniform bounds; the loop is unrolled over NMAX).
template <class T, int LMAX, int NMAX, int TILE, int L1, int L2, int L>
__device__ __forceinline__ void pair_fwd_deg(const T* __restrict__ As, const int* rec, const AceTables<T>& tb, int t,
                                             const T* a, const T* bb, T& p1, T& p2) {
  if constexpr ((L1 + L2 + L) % 2 == 0 && L >= (L1 > L2 ? L1 - L2 : L2 - L1) && L <= L1 + L2 && L <= LMAX) {
    constexpr int P2 = (LMAX + 1) * (LMAX + 1);
    constexpr int ST = TILE + 1;
    const int q0 = __builtin_amdgcn_readfirstlane(rec[4 + L]);
    const int q1 = __builtin_amdgcn_readfirstlane(rec[5 + L]);
    if (q0 < q1) {
      const int n30 = __builtin_amdgcn_readfirstlane((rec[10 + L] - L * L) / P2);
      const int n3e = n30 + (q1 - q0);
      // the coefficients of n3 = 0 .. NMAX-1 around the run, read at once (scalar loads
      // from a uniform base; the table is padded on both sides), and the run as a bit mask
      static_assert(NMAX <= kTcPad, "the coefficient table is padded by kTcPad entries");
      const Coef2<T>* cb = tb.tc + (q0 - n30);
      T c1v[NMAX], c2v[NMAX];
#pragma unroll
      for (int n3 = 0; n3 < NMAX; ++n3) {
        c1v[n3] = cld(&cb[n3].c1);
        c2v[n3] = cld(&cb[n3].c2);
      }
      const unsigned run = ((1u << n3e) - 1u) & ~((1u << n30) - 1u);
      T P[2 * L + 1];
#pragma unroll
      for (int m = 0; m < 2 * L + 1; ++m) P[m] = T(0);
      Couple3<LMAX, L1, L2, L>::template fwd<T>(a, bb, P);
#pragma unroll
      for (int n3 = 0; n3 < NMAX; ++n3) {
        if (run & (1u << n3)) {
          T B = T(0);
#pragma unroll
          for (int mm = 0; mm < 2 * L + 1; ++mm) B = fma(P[mm], As[(n3 * P2 + L * L + mm) * ST + t], B);
          p1 = fma(c1v[n3], B, p1);
          p2 = fma(c2v[n3], B, p2);
        }
      }
    }
  }
}

template <class T, int LMAX, int NMAX, int TILE, bool COMP, int L1, int L2>
__device__ __forceinline__ void pair_fwd_n(const T* __restrict__ As, const int* rec, const AceTables<T>& tb, int t,
                                           int n_max, Acc<T>& acc) {
  constexpr int ST = TILE + 1;
  const int o1 = rec[0], o2 = rec[1];
  T a[2 * L1 + 1], bb[2 * L2 + 1];
#pragma unroll
  for (int m = 0; m < 2 * L1 + 1; ++m) a[m] = As[(o1 + m) * ST + t];
#pragma unroll
  for (int m = 0; m < 2 * L2 + 1; ++m) bb[m] = As[(o2 + m) * ST + t];
  T p1 = T(0), p2 = T(0);
  pair_fwd_deg<T, LMAX, NMAX, TILE, L1, L2, 0>(As, rec, tb, t, a, bb, p1, p2);
  pair_fwd_deg<T, LMAX, NMAX, TILE, L1, L2, 1>(As, rec, tb, t, a, bb, p1, p2);
  pair_fwd_deg<T, LMAX, NMAX, TILE, L1, L2, 2>(As, rec, tb, t, a, bb, p1, p2);
  pair_fwd_deg<T, LMAX, NMAX, TILE, L1, L2, 3>(As, rec, tb, t, a, bb, p1, p2);
  pair_fwd_deg<T, LMAX, NMAX, TILE, L1, L2, 4>(As, rec, tb, t, a, bb, p1, p2);
  acc_sum<T, COMP>(acc.s1, acc.e1, p1);
  acc_sum<T, COMP>(acc.s2, acc.e2, p2);
}

template <class T, int LMAX, int TILE, bool DC, int L1, int L2>
__device__ __forceinline__ void pair_bwd(const T* __restrict__ As, T* __restrict__ Ab, const int* rec,
                                         const AceTables<T>& tb, int t, bool own, T fp, double wdc, double wfp,
                                         double* dc1, double* dc2) {
  using C = Couple<LMAX, L1, L2>;
  constexpr int P2 = (LMAX + 1) * (LMAX + 1);
  constexpr int ST = TILE + 1;
  const int o1 = rec[0], o2 = rec[1];
  T a[2 * L1 + 1], bb[2 * L2 + 1], P[P2], Pb[P2];
#pragma unroll
  for (int m = 0; m < 2 * L1 + 1; ++m) a[m] = As[(o1 + m) * ST + t];
#pragma unroll
  for (int m = 0; m < 2 * L2 + 1; ++m) bb[m] = As[(o2 + m) * ST + t];
#pragma unroll
  for (int m = 0; m < P2; ++m) {
    P[m] = T(0);
    Pb[m] = T(0);
  }
  C::template fwd<T>(a, bb, P);
#pragma unroll
  for (int L = 0; L <= LMAX; ++L) {
    if ((C::kMask >> L) & 1) {
      const int q0 = rec[4 + L], q1 = rec[5 + L];
      const int o3b = rec[10 + L];
#pragma unroll 2
      for (int q = q0; q < q1; ++q) {
        const int o3 = o3b + (q - q0) * P2;
        const Coef2<T> c = tb.tc[q];
        const T d = fma(fp, c.c2, c.c1);
        T B = T(0);
#pragma unroll
        for (int mm = 0; mm < 2 * L + 1; ++mm) {
          const T a3 = As[(o3 + mm) * ST + t];
          Pb[L * L + mm] = fma(d, a3, Pb[L * L + mm]);
          lds_add<T, TILE>(&Ab[(o3 + mm) * ST + t], d * P[L * L + mm], own);
          if constexpr (DC) B = fma(P[L * L + mm], a3, B);
        }
        if constexpr (DC) {
          double g1 = own ? wdc * (double)B : 0.0;
          double g2 = own ? wfp * (double)B : 0.0;
          g1 = wave_sum(g1);
          g2 = wave_sum(g2);
          if ((threadIdx.x & 63) == 0) {
            atomicAdd(&dc1[tb.t_v[q]], g1);
            atomicAdd(&dc2[tb.t_v[q]], g2);
          }
        }
      }
    }
  }
  T ga[2 * L1 + 1], gb[2 * L2 + 1];
#pragma unroll
  for (int m = 0; m < 2 * L1 + 1; ++m) ga[m] = T(0);
#pragma unroll
  for (int m = 0; m < 2 * L2 + 1; ++m) gb[m] = T(0);
  C::template bwd<T>(a, bb, Pb, ga, gb);
#pragma unroll
  for (int m = 0; m < 2 * L1 + 1; ++m) lds_add<T, TILE>(&Ab[(o1 + m) * ST + t], ga[m], own);
#pragma unroll
  for (int m = 0; m < 2 * L2 + 1; ++m) lds_add<T, TILE>(&Ab[(o2 + m) * ST + t], gb[m], own);
}

#define APX_PAIR_CASES_3(X) \
  X(0, 0) X(0, 1) X(0, 2) X(0, 3) X(1, 0) X(1, 1) X(1, 2) X(1, 3) X(2, 0) X(2, 1) X(2, 2) X(2, 3) X(3, 0) X(3, 1) X(3, 2) X(3, 3)
#define APX_PAIR_CASES_4(X)                                                                                  \
  X(0, 0) X(0, 1) X(0, 2) X(0, 3) X(0, 4) X(1, 0) X(1, 1) X(1, 2) X(1, 3) X(1, 4) X(2, 0) X(2, 1) X(2, 2) X(2, 3) \
  X(2, 4) X(3, 0) X(3, 1) X(3, 2) X(3, 3) X(3, 4) X(4, 0) X(4, 1) X(4, 2) X(4, 3) X(4, 4)


// B1 and B2 contributions (wave 0 of each block), energy and adjoint.
template <class T, int TILE, bool COMP>
__device__ __forceinline__ void low_order_fwd(const T* __restrict__ As, const AceTables<T>& tb, int nb1, int nb2,
                                              int t, Acc<T>& acc) {
  constexpr int ST = TILE + 1;
  for (int e = 0; e < nb1; ++e) {
    const T a = As[tb.b1_off[e] * ST + t];
    acc_add<T, COMP>(acc.s1, acc.e1, tb.b1_c1[e], a);
    acc_add<T, COMP>(acc.s2, acc.e2, tb.b1_c2[e], a);
  }
  for (int e = 0; e < nb2; ++e) {
    const int o1 = tb.b2_off[3 * e], o2 = tb.b2_off[3 * e + 1], l = tb.b2_off[3 * e + 2];
    T B = T(0);
    for (int m = 0; m < 2 * l + 1; ++m) B = fma(As[(o1 + m) * ST + t], As[(o2 + m) * ST + t], B);
    acc_add<T, COMP>(acc.s1, acc.e1, tb.b2_c1[e], B);
    acc_add<T, COMP>(acc.s2, acc.e2, tb.b2_c2[e], B);
  }
}

template <class T, int TILE, bool DC>
__device__ __forceinline__ void low_order_bwd(const T* __restrict__ As, T* __restrict__ Ab, const AceTables<T>& tb,
                                              int nb1, int nb2, int t, bool own, T fp, double wdc, double wfp,
                                              double* dc1, double* dc2) {
  constexpr int ST = TILE + 1;
  for (int e = 0; e < nb1; ++e) {
    const int o = tb.b1_off[e];
    const T d = fma(fp, tb.b1_c2[e], tb.b1_c1[e]);
    lds_add<T, TILE>(&Ab[o * ST + t], d, own);
    if constexpr (DC) {
      const double B = (double)As[o * ST + t];
      double g1 = own ? wdc * B : 0.0, g2 = own ? wfp * B : 0.0;
      g1 = wave_sum(g1);
      g2 = wave_sum(g2);
      if ((threadIdx.x & 63) == 0) {
        atomicAdd(&dc1[tb.b1_v[e]], g1);
        atomicAdd(&dc2[tb.b1_v[e]], g2);
      }
    }
  }
  for (int e = 0; e < nb2; ++e) {
    const int o1 = tb.b2_off[3 * e], o2 = tb.b2_off[3 * e + 1], l = tb.b2_off[3 * e + 2];
    const T d = fma(fp, tb.b2_c2[e], tb.b2_c1[e]);
    T B = T(0);
    for (int m = 0; m < 2 * l + 1; ++m) {
      const T x1 = As[(o1 + m) * ST + t], x2 = As[(o2 + m) * ST + t];
      lds_add<T, TILE>(&Ab[(o1 + m) * ST + t], d * x2, own);
      lds_add<T, TILE>(&Ab[(o2 + m) * ST + t], d * x1, own);
      if constexpr (DC) B = fma(x1, x2, B);
    }
    if constexpr (DC) {
      double g1 = own ? wdc * (double)B : 0.0, g2 = own ? wfp * (double)B : 0.0;
      g1 = wave_sum(g1);
      g2 = wave_sum(g2);
      if ((threadIdx.x & 63) == 0) {
        atomicAdd(&dc1[tb.b2_v[e]], g1);
        atomicAdd(&dc2[tb.b2_v[e]], g2);
      }
    }
  }
}

template <class T>
__device__ __forceinline__ T feps(T x, T eps, T& dfdx) {
  const T ax = x < T(0) ? -x : x;
  const T s = sqrt(ax + eps * eps);
  dfdx = T(0.5) / s;
  const T v = s - eps;
  return x < T(0) ? -v : v;
}

template <class T, int LMAX, int TILE, int NW, bool COMP, bool DC>
__global__ void __launch_bounds__(NW * 64) k_ace_products(const T* __restrict__ Ag, T* __restrict__ Abg, int n_act,
                                                                 int na, AceTables<T> tb, int nb1, int nb2, T eps,
                                                                 const double* __restrict__ e_anch,
                                                                 const int* __restrict__ active,
                                                                 const double* __restrict__ w,
                                                                 double* __restrict__ e_site,
                                                                 double* __restrict__ dc1, double* __restrict__ dc2) {
  constexpr int ST = TILE + 1;
  extern __shared__ double smem_raw[];
  T* As = reinterpret_cast<T*>(smem_raw);
  T* Ab = As + (size_t)na * ST;
  T* red = Ab + (size_t)na * ST;  // [NW][4][TILE]
  T* fps = red + NW * 4 * TILE;   // [TILE]
  const int tid = threadIdx.x;
  const int nthr = NW * 64;
  const int npairs = tb.npairs;
  const int q0 = blockIdx.x * TILE;
  for (int e = tid; e < TILE * na; e += nthr) {
    const int t = e / na, a = e - t * na;
    const int q = q0 + t;
    As[a * ST + t] = q < n_act ? Ag[(size_t)q * na + a] : T(0);
    Ab[a * ST + t] = T(0);
  }
  __syncthreads();
  const int lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform across the wave
  const int t = lane % TILE;
  const bool own = lane < TILE;
  // pairs are sorted by coupling type and dealt round-robin, so all waves of a block run
  // the same specialised code at about the same time
  const int pb = __builtin_amdgcn_readfirstlane(wv);
  // ------------------------------------------------------------ energy pass
  Acc<T> acc{T(0), T(0), T(0), T(0)};
  // lane k < kPairRec holds word k of the wave's next pair record (one vector load a pair
  // ahead, waited for only when the next pair reads it out)
  int rv = 0;
  if (pb < npairs && lane < kPairRec) rv = tb.pairs[pb * kPairRec + lane];
  if (wv == 0) low_order_fwd<T, TILE, COMP>(As, tb, nb1, nb2, t, acc);
  for (int pi = pb; pi < npairs; pi += NW) {
    int rec[kPairRec];
#pragma unroll
    for (int k = 0; k < kPairRec; ++k) rec[k] = __builtin_amdgcn_readlane(rv, k);
    if (pi + NW < npairs && lane < kPairRec) rv = tb.pairs[(pi + NW) * kPairRec + lane];
    const int type = rec[2];
#define APX_FWD(A_, B_) \
  case A_ * (LMAX + 1) + B_: pair_fwd<T, LMAX, TILE, COMP, A_, B_>(As, rec, tb, t, acc); break;
    if constexpr (LMAX == 3) {
      switch (type) { APX_PAIR_CASES_3(APX_FWD) default: break; }
    } else {
      switch (type) { APX_PAIR_CASES_4(APX_FWD) default: break; }
    }
#undef APX_FWD
  }
  if (own) {
    red[(wv * 4 + 0) * TILE + t] = acc.s1;
    red[(wv * 4 + 1) * TILE + t] = acc.e1;
    red[(wv * 4 + 2) * TILE + t] = acc.s2;
    red[(wv * 4 + 3) * TILE + t] = acc.e2;
  }
  __syncthreads();
  if (wv == 0 && own) {
    T s1 = T(0), e1 = T(0), s2 = T(0), e2 = T(0);
    for (int v = 0; v < NW; ++v) {
      acc_add<T, COMP>(s1, e1, T(1), red[(v * 4 + 0) * TILE + t]);
      e1 += red[(v * 4 + 1) * TILE + t];
      acc_add<T, COMP>(s2, e2, T(1), red[(v * 4 + 2) * TILE + t]);
      e2 += red[(v * 4 + 3) * TILE + t];
    }
    const T phi1 = s1 + e1, phi2 = s2 + e2;
    T dfdx;
    const T f2 = feps<T>(phi2, eps, dfdx);
    fps[t] = dfdx;
    const int q = q0 + t;
    if (q < n_act) e_site[active[q]] = (double)phi1 + (double)f2 + e_anch[q];
  }
  __syncthreads();
  // ----------------------------------------------------------- adjoint pass
  const T fp = fps[t];
  double wdc = 0.0, wfp = 0.0;
  if constexpr (DC) {
    const int q = q0 + t;
    if (q < n_act && own) {
      wdc = w ? w[active[q]] : 1.0;
      wfp = wdc * (double)fp;
    }
  }
  if (pb < npairs && lane < kPairRec) rv = tb.pairs[pb * kPairRec + lane];
  if (wv == 0) low_order_bwd<T, TILE, DC>(As, Ab, tb, nb1, nb2, t, own, fp, wdc, wfp, dc1, dc2);
  for (int pi = pb; pi < npairs; pi += NW) {
    int rec[kPairRec];
#pragma unroll
    for (int k = 0; k < kPairRec; ++k) rec[k] = __builtin_amdgcn_readlane(rv, k);
    if (pi + NW < npairs && lane < kPairRec) rv = tb.pairs[(pi + NW) * kPairRec + lane];
    const int type = rec[2];
#define APX_BWD(A_, B_)                                                                                   \
  case A_ * (LMAX + 1) + B_:                                                                              \
    pair_bwd<T, LMAX, TILE, DC, A_, B_>(As, Ab, rec, tb, t, own, fp, wdc, wfp, dc1, dc2);                 \
    break;
    if constexpr (LMAX == 3) {
      switch (type) { APX_PAIR_CASES_3(APX_BWD) default: break; }
    } else {
      switch (type) { APX_PAIR_CASES_4(APX_BWD) default: break; }
    }
#undef APX_BWD
  }
  __syncthreads();
  for (int e = tid; e < TILE * na; e += nthr) {
    const int tt = e / na, a = e - tt * na;
    const int q = q0 + tt;
    if (q < n_act) Abg[(size_t)q * na + a] = Ab[a * ST + tt];
  }
}

// Back-projection of the adjoint of the float32 unit path, one tile of 64 atoms per block
// (lane = atom): B[k][lm] = sum_n Wp[l][n][k] Abar[n][lm], read and written tile-major
// [tile][a][64], so every load and store of a wave is one coalesced 256-byte segment.  A
// wave takes columns lm = wave, wave + 4, ...; a column's K adjoint values are loaded once
// and serve its K outputs, which are summed in registers; the weights are staged in LDS
// once per block.  The sum runs over n in ascending order.
template <class T, int LMAX>
__global__ void __launch_bounds__(256) k_ace_backproject(const T* __restrict__ Abg, T* __restrict__ Bg,
                                                         const T* __restrict__ Wp, int K, int na) {
  constexpr int LM = (LMAX + 1) * (LMAX + 1);
  constexpr int TILE = 64;
  constexpr int kMaxK = 12;
  // the wave index is uniform across the wave: said so, the column's l is too and the
  // weights become scalar loads (otherwise every lane loads the same weight)
  const int t = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // the weights of every l, rows padded to kMaxK (zeros), read by broadcast LDS loads
  __shared__ T ws[(LMAX + 1) * kMaxK * kMaxK];
  for (int e = threadIdx.x; e < (LMAX + 1) * kMaxK * kMaxK; e += 256) {
    const int l = e / (kMaxK * kMaxK), r = e - l * kMaxK * kMaxK, nn = r / kMaxK, kk = r - nn * kMaxK;
    ws[e] = nn < K && kk < K ? Wp[((size_t)l * K + nn) * K + kk] : T(0);
  }
  __syncthreads();
  const T* Ab = Abg + (size_t)blockIdx.x * na * TILE;
  T* B = Bg + (size_t)blockIdx.x * na * TILE;
  for (int lm = wv; lm < LM; lm += 4) {
    int l = 0;
    while ((l + 1) * (l + 1) <= lm) ++l;
    T a[kMaxK];
#pragma unroll
    for (int nn = 0; nn < kMaxK; ++nn) a[nn] = nn < K ? Ab[(size_t)(nn * LM + lm) * TILE + t] : T(0);
    T v[kMaxK];
#pragma unroll
    for (int kk = 0; kk < kMaxK; ++kk) v[kk] = T(0);
#pragma unroll
    for (int nn = 0; nn < kMaxK; ++nn) {
      if (nn < K) {
        const T* w = ws + (l * kMaxK + nn) * kMaxK;
#pragma unroll
        for (int kk = 0; kk < kMaxK; ++kk) v[kk] += w[kk] * a[nn];
      }
    }
#pragma unroll
    for (int kk = 0; kk < kMaxK; ++kk)
      if (kk < K) B[(size_t)(kk * LM + lm) * TILE + t] = v[kk];
  }
}

// ------------------------------------------------------------------ kernel 3
// Ā' of one atom in LDS: lm-major rows of KP radial values (K rounded up to whole 16-byte
// groups, the padding zero), so that a row is read by a few wide broadcast loads.
template <class T, int NMAX>
struct ForceLds {
  static constexpr int KP = (NMAX * (int)sizeof(T) + 15) / 16 * 16 / (int)sizeof(T);
};

// Float32 is held to 128 VGPRs, four waves per SIMD (a few registers spill; three waves left
// the gathers' latency exposed).
template <class T, int LMAX, int NMAX>
__global__ void __launch_bounds__(64, sizeof(T) == 4 ? 4 : 1) k_ace_force(const double* __restrict__ pos, int n, BoxDev b,
                                                  const int* __restrict__ count, const int* __restrict__ idx,
                                                  int max_nb, const int* __restrict__ active, int n_act, int K,
                                                  T rc, T inv_h, double rc2, const T* __restrict__ Wp, AnchorDev an,
                                                  AceScratch<T> sc, const double* __restrict__ w,
                                                  double* __restrict__ f, const double* __restrict__ w2,
                                                  double* __restrict__ f2) {
  constexpr int LM = (LMAX + 1) * (LMAX + 1);
  constexpr int kMaxK = NMAX;
  constexpr int KP = ForceLds<T, NMAX>::KP;
  extern __shared__ double smem_raw[];
  T* Ab2 = reinterpret_cast<T*>(smem_raw);  // [LM][KP]: Ab2[lm * KP + k], zero for k >= K
  __shared__ double etab[32];
  stage_exp_table(etab);
  const int q = xcd_block(blockIdx.x, gridDim.x);
  const T two_rc = T(2) / rc;
  const int lane = threadIdx.x;
  const int i = active[q];
  const double wi = w ? w[i] : 1.0;
  // second weight set (the integrator's weight difference): scattered only where non-zero
  const double w2i = f2 ? w2[i] : 0.0;
  const int na = K * LM;
  const int ts = sc.tile_size;
  const T* Abr = ts > 0 ? sc.Ab + (size_t)(q / ts) * na * ts + (q % ts) : sc.Ab + (size_t)q * na;
  const int as = ts > 0 ? ts : 1;
  // back-projection: Ab2[k][lm] = sum_n Wp[l][n][k] Abar[n][lm]; the float32 unit path
  // has it precomputed tile-major in sc.A by k_ace_backproject
  for (int o = lane; o < LM * KP; o += 64) Ab2[o] = T(0);
  __syncthreads();
  if (ts > 0) {
    const T* B = sc.A + (size_t)(q / ts) * na * ts + (q % ts);
    for (int o = lane; o < K * LM; o += 64) {
      const int kk = o / LM, lm = o - kk * LM;
      Ab2[lm * KP + kk] = B[(size_t)o * ts];
    }
  }
  for (int o = lane; o < K * LM && ts == 0; o += 64) {
    const int kk = o / LM, lm = o - kk * LM;
    int l = 0;
    while ((l + 1) * (l + 1) <= lm) ++l;
    // the K loads of an output are issued together (unrolled to the largest K)
    T wv_[kMaxK], av_[kMaxK];
#pragma unroll
    for (int nn = 0; nn < kMaxK; ++nn) {
      wv_[nn] = nn < K ? Wp[((size_t)l * K + nn) * K + kk] : T(0);
      av_[nn] = nn < K ? Abr[(size_t)(nn * LM + lm) * as] : T(0);
    }
    T v = T(0);
#pragma unroll
    for (int nn = 0; nn < kMaxK; ++nn) v += wv_[nn] * av_[nn];
    Ab2[lm * KP + kk] = v;
  }
  __syncthreads();
  const double fpa = an.on ? sc.fp_anch[q] : 0.0;
  const double xi = pos[i], yi = pos[(size_t)n + i], zi = pos[2 * (size_t)n + i];
  int cnt = count[i];
  if (cnt > max_nb) cnt = max_nb;
  double fix = 0.0, fiy = 0.0, fiz = 0.0;
  double f2x = 0.0, f2y = 0.0, f2z = 0.0;
  for (int c0 = 0; c0 < cnt; c0 += 64) {
    const int k = c0 + lane;
    if (k < cnt) {
      const int j = idx[(size_t)k * n + i];
      const double dx = min_image_sel(pos[j] - xi, b.L[0], b.half[0], b.per[0]);
      const double dy = min_image_sel(pos[(size_t)n + j] - yi, b.L[1], b.half[1], b.per[1]);
      const double dz = min_image_sel(pos[2 * (size_t)n + j] - zi, b.L[2], b.half[2], b.per[2]);
      const double r2 = dx * dx + dy * dy + dz * dz;
      double gx = 0.0, gy = 0.0, gz = 0.0;
      const double ird = rsq_nr(r2);
      const double rd = r2 * ird;
      if (r2 < rc2) {
        const T r = T(rd), ir = T(ird);
        const T ux = T(dx) * ir, uy = T(dy) * ir, uz = T(dz) * ir;
        const T dxdr = two_rc;
        const T x = r * dxdr - T(1);
        T ps, dps;
        taper_t<T>((r - rc) * inv_h, ps, dps);
        dps *= inv_h;
        T g[kMaxK], gd[kMaxK];
        T t0 = T(1), t1 = x, d0 = T(0), d1 = T(1);
        g[0] = ps;
        gd[0] = dps;
        g[1] = x * ps;
        gd[1] = d1 * dxdr * ps + x * dps;
#pragma unroll
        for (int a = 2; a < kMaxK; ++a) {
          const T t2 = T(2) * x * t1 - t0;
          const T d2 = T(2) * t1 + T(2) * x * d1 - d0;
          g[a] = t2 * ps;
          gd[a] = d2 * dxdr * ps + t2 * dps;
          t0 = t1;
          t1 = t2;
          d0 = d1;
          d1 = d2;
        }
        T S[LM], Sx[LM], Sy[LM], Sz[LM];
        solid_harmonics<T, LMAX, true>(ux, uy, uz, S, Sx, Sy, Sz);
        T radial = T(0), vx = T(0), vy = T(0), vz = T(0);
#pragma unroll
        for (int lm = 0; lm < LM; ++lm) {
          int l = 0;
          while ((l + 1) * (l + 1) <= lm) ++l;
          // the row is the same for every lane (broadcast); entries beyond K are zero
          T c[KP];
#pragma unroll
          for (int kk = 0; kk < KP; kk += 16 / (int)sizeof(T)) {
            if constexpr (sizeof(T) == 4) {
              const float4 v = *reinterpret_cast<const float4*>(&Ab2[lm * KP + kk]);
              c[kk] = v.x;
              c[kk + 1] = v.y;
              c[kk + 2] = v.z;
              c[kk + 3] = v.w;
            } else {
              const double2 v = *reinterpret_cast<const double2*>(&Ab2[lm * KP + kk]);
              c[kk] = v.x;
              c[kk + 1] = v.y;
            }
          }
          T av = T(0), bv = T(0);
#pragma unroll
          for (int kk = 0; kk < NMAX; ++kk) {
            av = fma(c[kk], g[kk], av);
            bv = fma(c[kk], gd[kk], bv);
          }
          radial += (bv - av * T(l) * ir) * S[lm];
          const T ar = av * ir;
          vx = fma(ar, Sx[lm], vx);
          vy = fma(ar, Sy[lm], vy);
          vz = fma(ar, Sz[lm], vz);
        }
        gx = (double)(radial * ux + vx);
        gy = (double)(radial * uy + vy);
        gz = (double)(radial * uz + vz);
      }
      if (an.on && r2 < an.rc2) {
        double ps, dps;
        taper_d((rd - an.rc) * an.inv_h, ps, dps);
        dps *= an.inv_h;
        const double eb = exp_tab(-an.beta * (rd - an.r0), etab);
        const double ea = exp_tab(-an.alpha * (rd - an.r0), etab);
        const double drho = eb * (dps - an.beta * ps);
        const double dphi = an.A * ea * (dps - an.alpha * ps);
        const double s = (fpa * drho + 0.5 * dphi) * ird;
        gx += s * dx;
        gy += s * dy;
        gz += s * dz;
      }
      if (w2i != 0.0) {
        const double hx = gx * w2i, hy = gy * w2i, hz = gz * w2i;
        if (hx != 0.0 || hy != 0.0 || hz != 0.0) {
          unsafeAtomicAdd(&f2[j], -hx);
          unsafeAtomicAdd(&f2[(size_t)n + j], -hy);
          unsafeAtomicAdd(&f2[2 * (size_t)n + j], -hz);
        }
        f2x += hx;
        f2y += hy;
        f2z += hz;
      }
      gx *= wi;
      gy *= wi;
      gz *= wi;
      if (gx != 0.0 || gy != 0.0 || gz != 0.0) {
        unsafeAtomicAdd(&f[j], -gx);
        unsafeAtomicAdd(&f[(size_t)n + j], -gy);
        unsafeAtomicAdd(&f[2 * (size_t)n + j], -gz);
      }
      fix += gx;
      fiy += gy;
      fiz += gz;
    }
  }
  fix = wave_sum(fix);
  fiy = wave_sum(fiy);
  fiz = wave_sum(fiz);
  if (lane == 0) {
    unsafeAtomicAdd(&f[i], fix);
    unsafeAtomicAdd(&f[(size_t)n + i], fiy);
    unsafeAtomicAdd(&f[2 * (size_t)n + i], fiz);
  }
  if (w2i != 0.0) {  // uniform across the wave
    f2x = wave_sum(f2x);
    f2y = wave_sum(f2y);
    f2z = wave_sum(f2z);
    if (lane == 0) {
      unsafeAtomicAdd(&f2[i], f2x);
      unsafeAtomicAdd(&f2[(size_t)n + i], f2y);
      unsafeAtomicAdd(&f2[2 * (size_t)n + i], f2z);
    }
  }
}

// ------------------------------------------------- kernel 2b (float32, unit adjoint)
// Same energy pass as k_ace_products; the adjoint is reorganised so that no LDS atomics
// are needed.  The adjoint work is cut into units (l1, l2, L): all pairs of one coupling
// type, restricted to third blocks of degree L.  A unit is owned by one wave, which keeps
//   acc3[n3][M]  the adjoint of every third block (n3, L)            (registers)
//   accR[m]      the adjoint of the pair label with the larger degree, accumulated over
//                the run of pairs sharing it (pairs are sorted by it)
//   accO[h][m]   the adjoint of the other pair label (one of at most unit_width values in
//                the unit's range of other labels)
// and adds them to the tile's adjoint in global memory with float atomics when a run or
// the unit ends.
// Every lane adds, padded lanes (beyond the last active atom) included: their slots lie
// inside the tile's region and are never read back.
template <class T, int TILE>
__device__ __forceinline__ void gadd(T* __restrict__ Abt, int a, int t, T v) {
  unsafeAtomicAdd(&Abt[(size_t)a * TILE + t], v);
}


// The third blocks of degree L in registers, and the flush of their adjoint.
template <class T, int LMAX, int NMAX, int TILE, int L>
__device__ __forceinline__ void third_load(const T* __restrict__ As, int n_max, int t, T (&A3)[NMAX][2 * L + 1],
                                           T (&acc3)[NMAX][2 * L + 1]) {
  constexpr int ST = TILE + 1;
  constexpr int P2 = (LMAX + 1) * (LMAX + 1);
#pragma unroll
  for (int n = 0; n < NMAX; ++n) {
#pragma unroll
    for (int m = 0; m < 2 * L + 1; ++m) {
      acc3[n][m] = T(0);
      A3[n][m] = n < n_max ? As[(n * P2 + L * L + m) * ST + t] : T(0);
    }
  }
}

// The block's waves sum their third-block adjoints through LDS (the upper half of the
// waves hands its sums to the lower half, which stores the partial sums), then every
// wave adds a share of the elements to global memory: one atomic per element and block.
// lds holds (NW/2) * NMAX * (2L+1) * 64 values; the caller has finished with it.
template <class T, int LMAX, int NMAX, int TILE, int NW, int L>
__device__ __forceinline__ void third_flush(T* __restrict__ Abt, T* lds, int n_max, int t, int wv, int lane,
                                            T (&acc3)[NMAX][2 * L + 1]) {
  constexpr int P2 = (LMAX + 1) * (LMAX + 1);
  constexpr int NL = 2 * L + 1, NE = NMAX * NL, H = NW / 2;
  static_assert(NW % 2 == 0, "waves pair up");
  __syncthreads();
  if (wv >= H) {
#pragma unroll
    for (int n = 0; n < NMAX; ++n)
#pragma unroll
      for (int m = 0; m < NL; ++m) lds[((wv - H) * NE + n * NL + m) * 64 + lane] = acc3[n][m];
  }
  __syncthreads();
  if (wv < H) {
#pragma unroll
    for (int n = 0; n < NMAX; ++n)
#pragma unroll
      for (int m = 0; m < NL; ++m) {
        T* q = &lds[(wv * NE + n * NL + m) * 64 + lane];
        *q = *q + acc3[n][m];
      }
  }
  __syncthreads();
  for (int e = wv; e < NE; e += NW) {
    const int n = e / NL, m = e - n * NL;
    if (n >= n_max) continue;
    T s = T(0);
#pragma unroll
    for (int h = 0; h < H; ++h) s += lds[(h * NE + e) * 64 + lane];
    gadd<T, TILE>(Abt, n * P2 + L * L + m, t, s);
  }
}

// The pairs of one unit (l1, l2, L) for a range of the other label; the third-block
// registers A3 and their adjoint acc3 are the caller's (shared by the units of one degree).
template <class T, int LMAX, int NMAX, int TILE, int L1, int L2, int L>
__device__ __forceinline__ void unit_bwd(const T* __restrict__ As, T* __restrict__ Abt, const AceTables<T>& tb,
                                         int eb, int ee, int obase, int oend, int t, T fp,
                                         const T (&A3)[NMAX][2 * L + 1], T (&acc3)[NMAX][2 * L + 1]) {
  using C = Couple3<LMAX, L1, L2, L>;
  constexpr int ST = TILE + 1;
  constexpr int P2 = (LMAX + 1) * (LMAX + 1);
  constexpr int N1 = 2 * L1 + 1, N2 = 2 * L2 + 1, NL = 2 * L + 1;
  constexpr bool RUN1 = L1 >= L2;
  constexpr int NR = RUN1 ? N1 : N2;
  constexpr int NO = RUN1 ? N2 : N1;
  constexpr int LR = RUN1 ? L1 : L2;
  constexpr int LO = RUN1 ? L2 : L1;
  static_assert(NMAX <= kAdjC2 - kAdjC1, "the pair stream holds coefficients for n3 < 12");
  // this unit covers the pairs whose other label lies in [obase, oend), at most
  // unit_width(L, n_max) <= NH labels
  constexpr int NH = unit_width(L, NMAX);
  T accR[NR];
  T accO[NH][NO];  // adjoint of the other label, by its position in the range
#pragma unroll
  for (int h = 0; h < NH; ++h) {
#pragma unroll
    for (int m = 0; m < NO; ++m) accO[h][m] = T(0);
  }
#pragma unroll
  for (int m = 0; m < NR; ++m) accR[m] = T(0);
  int run_n = -1;
  // PF: the next entry's words are loaded while this entry computes (issued once this
  // entry's LDS operands have arrived, so that their wait does not cover the prefetch)
  constexpr bool PF = L <= kAdjPrefetchMaxL;
  int nx_o1 = 0, nx_o2 = 0, nx_run = 0, nx_oth = 0;
  T nx_c1[NMAX], nx_c2[NMAX];
  auto fetch = [&](int e) {
    const int* E = tb.adj_i + (size_t)e * kAdjRec;
    const T* Ec = reinterpret_cast<const T*>(tb.adj_f) + (size_t)e * kAdjRec;
    nx_o1 = cld(E);
    nx_o2 = cld(E + 1);
    nx_run = cld(E + 2);
    nx_oth = cld(E + 3);
#pragma unroll
    for (int n3 = 0; n3 < NMAX; ++n3) {
      nx_c1[n3] = cld(Ec + kAdjC1 + n3);
      nx_c2[n3] = cld(Ec + kAdjC2 + n3);
    }
  };
  if (PF && eb < ee) fetch(eb);
  for (int e = eb; e < ee; ++e) {
    if (!PF) fetch(e);
    const int nrun = nx_run;
    const int noth = nx_oth;
    T c1[NMAX], c2[NMAX];
#pragma unroll
    for (int n3 = 0; n3 < NMAX; ++n3) {
      c1[n3] = nx_c1[n3];
      c2[n3] = nx_c2[n3];
    }
    if (nrun != run_n) {
      if (run_n >= 0) {
#pragma unroll
        for (int m = 0; m < NR; ++m) gadd<T, TILE>(Abt, run_n * P2 + LR * LR + m, t, accR[m]);
      }
#pragma unroll
      for (int m = 0; m < NR; ++m) accR[m] = T(0);
      run_n = nrun;
    }
    const int o1 = nx_o1, o2 = nx_o2;
    T a[N1], b[N2], P[NL], Pb[NL];
#pragma unroll
    for (int m = 0; m < N1; ++m) a[m] = As[(o1 + m) * ST + t];
#pragma unroll
    for (int m = 0; m < N2; ++m) b[m] = As[(o2 + m) * ST + t];
#pragma unroll
    for (int m = 0; m < NL; ++m) {
      P[m] = T(0);
      Pb[m] = T(0);
    }
    C::template fwd<T>(a, b, P);
    if constexpr (PF) {
      __builtin_amdgcn_sched_barrier(0);
      if (e + 1 < ee) fetch(e + 1);
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int n3 = 0; n3 < NMAX; ++n3) {
      // the stream's coefficients are zero outside the pair's run of n3 and A3 is zero
      // beyond n_max: those terms add exact zeros, which costs less than branching on them
      {
        const T d = fma(fp, c2[n3], c1[n3]);
#pragma unroll
        for (int m = 0; m < NL; ++m) {
          Pb[m] = fma(d, A3[n3][m], Pb[m]);
          acc3[n3][m] = fma(d, P[m], acc3[n3][m]);
        }
      }
    }
    T ga[N1], gb[N2];
#pragma unroll
    for (int m = 0; m < N1; ++m) ga[m] = T(0);
#pragma unroll
    for (int m = 0; m < N2; ++m) gb[m] = T(0);
    C::template bwd<T>(a, b, Pb, ga, gb);
#pragma unroll
    for (int m = 0; m < NR; ++m) accR[m] += RUN1 ? ga[m] : gb[m];
    // the other label is wave-uniform: a scalar branch picks its accumulator
    const int oh = noth - obase;
#pragma unroll
    for (int h = 0; h < NH; ++h) {
      if (h == oh) {
#pragma unroll
        for (int m = 0; m < NO; ++m) accO[h][m] += RUN1 ? gb[m] : ga[m];
      }
    }
  }
  if (run_n >= 0) {
#pragma unroll
    for (int m = 0; m < NR; ++m) gadd<T, TILE>(Abt, run_n * P2 + LR * LR + m, t, accR[m]);
  }
#pragma unroll
  for (int h = 0; h < NH; ++h) {
    if (obase + h < oend) {
#pragma unroll
      for (int m = 0; m < NO; ++m) gadd<T, TILE>(Abt, (obase + h) * P2 + LO * LO + m, t, accO[h][m]);
    }
  }
}

// B1 and B2 adjoint of one label n, output-stationary.  B2_(n1 n2 l) = sum_m A_n1lm A_n2lm
// (n1 <= n2, entries stored in catalogue order (n1, n2, l)), so
//   dE/dA_nlm = sum_n' D_nn'l A_n'lm,  D_nn'l = d_(min, max, l) for n' != n, 2 d_(n n l) for n' = n,
// with d = c1 + F'(phi2) c2 of the entry; plus the B1 entry of label n.  The label's
// adjoint is accumulated in registers and added once per (l, m).
template <class T, int LMAX, int TILE>
__device__ __forceinline__ void low_order_unit(const T* __restrict__ As, T* __restrict__ Abt, const AceTables<T>& tb,
                                               int nb1, int n_max, int n, int t, T fp) {
  constexpr int ST = TILE + 1;
  constexpr int P2 = (LMAX + 1) * (LMAX + 1);
  // first entry of the labels n1: sum over n' < n1 of (n_max - n')(l_max + 1)
  auto base = [&](int n1) { return (LMAX + 1) * (n1 * n_max - n1 * (n1 - 1) / 2); };
#pragma unroll
  for (int l = 0; l <= LMAX; ++l) {
    T acc[2 * l + 1];
#pragma unroll
    for (int m = 0; m < 2 * l + 1; ++m) acc[m] = T(0);
    for (int np = 0; np < n_max; ++np) {
      const int n1 = np < n ? np : n, n2 = np < n ? n : np;
      const int e = base(n1) + (n2 - n1) * (LMAX + 1) + l;
      T d = fma(fp, cld(tb.b2_c2 + e), cld(tb.b2_c1 + e));
      if (np == n) d += d;
      const int o = np * P2 + l * l;
#pragma unroll
      for (int m = 0; m < 2 * l + 1; ++m) acc[m] = fma(d, As[(o + m) * ST + t], acc[m]);
    }
    if (l == 0 && n < nb1) acc[0] += fma(fp, cld(tb.b1_c2 + n), cld(tb.b1_c1 + n));
#pragma unroll
    for (int m = 0; m < 2 * l + 1; ++m) gadd<T, TILE>(Abt, n * P2 + l * l + m, t, acc[m]);
  }
}

// coupled degree triples (l1, l2, L) for l_max 3 and 4
#define APX_UNIT_CASES_3(X) \
  X(0, 0, 0) X(0, 1, 1) X(0, 2, 2) X(0, 3, 3) X(1, 0, 1) X(1, 1, 0) X(1, 1, 2) X(1, 2, 1) \
  X(1, 2, 3) X(1, 3, 2) X(2, 0, 2) X(2, 1, 1) X(2, 1, 3) X(2, 2, 0) X(2, 2, 2) X(2, 3, 1) \
  X(2, 3, 3) X(3, 0, 3) X(3, 1, 2) X(3, 2, 1) X(3, 2, 3) X(3, 3, 0) X(3, 3, 2)
#define APX_UNIT_CASES_4(X) \
  X(0, 0, 0) X(0, 1, 1) X(0, 2, 2) X(0, 3, 3) X(0, 4, 4) X(1, 0, 1) X(1, 1, 0) X(1, 1, 2) \
  X(1, 2, 1) X(1, 2, 3) X(1, 3, 2) X(1, 3, 4) X(1, 4, 3) X(2, 0, 2) X(2, 1, 1) X(2, 1, 3) \
  X(2, 2, 0) X(2, 2, 2) X(2, 2, 4) X(2, 3, 1) X(2, 3, 3) X(2, 4, 2) X(2, 4, 4) X(3, 0, 3) \
  X(3, 1, 2) X(3, 1, 4) X(3, 2, 1) X(3, 2, 3) X(3, 3, 0) X(3, 3, 2) X(3, 3, 4) X(3, 4, 1) \
  X(3, 4, 3) X(4, 0, 4) X(4, 1, 3) X(4, 2, 2) X(4, 2, 4) X(4, 3, 1) X(4, 3, 3) X(4, 4, 0) \
  X(4, 4, 2) X(4, 4, 4)

// Stages the tile's atomic base into LDS, [a][TILE + 1] (atom fastest; the padding
// column keeps the stride odd).  The tile is one contiguous block of the atom-major
// global array (the buffer holds whole tiles); float32 tiles are read 16 bytes at a
// time and transposed on the way, values of atoms beyond n_act are zero.
template <class T, int TILE>
__device__ __forceinline__ void stage_tile(const T* __restrict__ Ag, T* As, int q0, int n_act, int na, int nthr) {
  constexpr int ST = TILE + 1;
  if constexpr (sizeof(T) == 4) {
    const T* src = Ag + (size_t)q0 * na;
    const int total = TILE * na;
    const int rem = n_act - q0;
    const int valid = (rem < TILE ? rem : TILE) * na;
    for (int e4 = threadIdx.x * 4; e4 < total; e4 += nthr * 4) {
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (e4 + 3 < valid) {
        v = *reinterpret_cast<const float4*>(src + e4);
      } else {
        if (e4 < valid) v.x = src[e4];
        if (e4 + 1 < valid) v.y = src[e4 + 1];
        if (e4 + 2 < valid) v.z = src[e4 + 2];
      }
      int t = e4 / na, a = e4 - t * na;
      const T vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (e4 + k < total) As[a * ST + t] = vv[k];
        if (++a == na) {
          a = 0;
          ++t;
        }
      }
    }
  } else {
    for (int e = threadIdx.x; e < TILE * na; e += nthr) {
      const int t = e / na, a = e - t * na;
      const int q = q0 + t;
      As[a * ST + t] = q < n_act ? Ag[(size_t)q * na + a] : T(0);
    }
  }
}

// Energy pass of the float32 product basis: 64 active atoms per block (lane = atom), the
// label pairs dealt round-robin to the waves, compensated sums of c1.B and c2.B, then
// E_i = phi1 + F_eps(phi2) (+ anchor) and the embedding slope F_eps'(phi2) for the adjoint.
template <class T, int LMAX, int NMAX, int TILE, int NW, bool COMP>
__global__ void __launch_bounds__(NW * 64, NW / 2) k_ace_energy(const T* __restrict__ Ag, int n_act, int na, int n_max,
                                                        AceTables<T> tb, int nb1, int nb2, T eps,
                                                        const double* __restrict__ e_anch,
                                                        const int* __restrict__ active, double* __restrict__ e_site,
                                                        T* __restrict__ fp_out) {
  extern __shared__ double smem_raw[];
  T* As = reinterpret_cast<T*>(smem_raw);
  T* red = As;  // [NW][4][TILE], over the tile once every wave is done with it
  const int tid = threadIdx.x;
  const int q0 = blockIdx.x * TILE;
  stage_tile<T, TILE>(Ag, As, q0, n_act, na, NW * 64);
  __syncthreads();
  const int lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform across the wave
  const int t = lane % TILE;
  Acc<T> acc{T(0), T(0), T(0), T(0)};
  // lane k < kPairRec holds word k of the wave's next pair record: one vector load per pair,
  // issued a pair ahead and waited for only when the next pair reads it out
  int rv = 0;
  if (wv < tb.npairs && lane < kPairRec) rv = tb.pairs[wv * kPairRec + lane];
  if (wv == 0) low_order_fwd<T, TILE, COMP>(As, tb, nb1, nb2, t, acc);
  for (int pi = wv; pi < tb.npairs; pi += NW) {
    int rec[kPairRec];
#pragma unroll
    for (int k = 0; k < kPairRec; ++k) rec[k] = __builtin_amdgcn_readlane(rv, k);
    if (pi + NW < tb.npairs && lane < kPairRec) rv = tb.pairs[(pi + NW) * kPairRec + lane];
    const int type = rec[2];
#define APX_FWD(A_, B_) \
  case A_ * (LMAX + 1) + B_: pair_fwd_n<T, LMAX, NMAX, TILE, COMP, A_, B_>(As, rec, tb, t, n_max, acc); break;
    if constexpr (LMAX == 3) {
      switch (type) { APX_PAIR_CASES_3(APX_FWD) default: break; }
    } else {
      switch (type) { APX_PAIR_CASES_4(APX_FWD) default: break; }
    }
#undef APX_FWD
  }
  __syncthreads();
  if (lane < TILE) {
    red[(wv * 4 + 0) * TILE + t] = acc.s1;
    red[(wv * 4 + 1) * TILE + t] = acc.e1;
    red[(wv * 4 + 2) * TILE + t] = acc.s2;
    red[(wv * 4 + 3) * TILE + t] = acc.e2;
  }
  __syncthreads();
  if (wv == 0 && lane < TILE) {
    T s1 = T(0), e1 = T(0), s2 = T(0), e2 = T(0);
    for (int v = 0; v < NW; ++v) {
      acc_add<T, COMP>(s1, e1, T(1), red[(v * 4 + 0) * TILE + t]);
      e1 += red[(v * 4 + 1) * TILE + t];
      acc_add<T, COMP>(s2, e2, T(1), red[(v * 4 + 2) * TILE + t]);
      e2 += red[(v * 4 + 3) * TILE + t];
    }
    T dfdx;
    const T f2 = feps<T>(s2 + e2, eps, dfdx);
    const int q = q0 + t;
    fp_out[q] = q < n_act ? dfdx : T(0);
    if (q < n_act) e_site[active[q]] = (double)(s1 + e1) + (double)f2 + e_anch[q];
  }
}

// Degrees 0..3 run at two waves per SIMD (their units hold at most 3 and 2 other labels in
// degrees 2 and 3); degree 4 needs one wave per SIMD.
// Adjoint of the product basis for the units of one launch group G: the tile's atomic
// base is staged again, the embedding slope is read from the energy pass, and every
// wave runs its units (see unit_bwd), adding to the tile's adjoint in global memory.
template <class T, int LMAX, int NMAX, int TILE, int NW, int G>
__global__ void __launch_bounds__(NW * 64, G <= 3 ? 2 : 1) k_ace_adjoint(const T* __restrict__ Ag, T* __restrict__ Abg,
                                                            int n_act, int na, int n_max, AceTables<T> tb, int nb1,
                                                            const T* __restrict__ fp_in) {
  static_assert(NW == kUnitWaves, "the unit tables are dealt to kUnitWaves waves");
  extern __shared__ double smem_raw[];
  T* As = reinterpret_cast<T*>(smem_raw);
  const int tid = threadIdx.x;
  const int q0 = blockIdx.x * TILE;
  stage_tile<T, TILE>(Ag, As, q0, n_act, na, NW * 64);
  __syncthreads();
  const int lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform across the wave
  const int t = lane % TILE;
  const T fp = fp_in[q0 + t];
  T* Abt = Abg + (size_t)blockIdx.x * na * TILE;
  const int* wu = tb.wave_units;
  const int* lst = wu + kUnitGroups * (NW + 1);
  // the third-block degree of the group's units
  constexpr int LG = G;
  T A3[NMAX][2 * LG + 1], acc3[NMAX][2 * LG + 1];
  third_load<T, LMAX, NMAX, TILE, LG>(As, n_max, t, A3, acc3);
  const int ub = __builtin_amdgcn_readfirstlane(cld(wu + G * (NW + 1) + wv));
  const int ue = __builtin_amdgcn_readfirstlane(cld(wu + G * (NW + 1) + wv + 1));
  for (int k = ub; k < ue; ++k) {
    const int u = cld(lst + k);
    const int* ur = tb.units + u * kUnitRec;
    const int type = cld(ur);
    const int L = cld(ur + 1);
    const int pb = cld(ur + 2);
    const int obase = cld(ur + 4);
    const int eb = cld(ur + 5);
    const int ee = cld(ur + 6);
    const int oend = cld(ur + 7);
    if (L < 0) {
      if constexpr (G == 0) low_order_unit<T, LMAX, TILE>(As, Abt, tb, nb1, n_max, pb, t, fp);
      continue;
    }
    const int key = type * (LMAX + 1) + L;
    // every unit of the group has degree LG; the third-block registers persist across the
    // wave's units
#define APX_UNIT(A_, B_, C_)                                                                              \
  case (A_ * (LMAX + 1) + B_) * (LMAX + 1) + C_:                                                          \
    if constexpr (C_ == LG)                                                                               \
      unit_bwd<T, LMAX, NMAX, TILE, A_, B_, C_>(As, Abt, tb, eb, ee, obase, oend, t, fp, A3, acc3);       \
    break;
    if constexpr (LMAX == 3) {
      switch (key) { APX_UNIT_CASES_3(APX_UNIT) default: break; }
    } else {
      switch (key) { APX_UNIT_CASES_4(APX_UNIT) default: break; }
    }
#undef APX_UNIT
  }
  third_flush<T, LMAX, NMAX, TILE, NW, LG>(Abt, As, n_max, t, wv, lane, acc3);
}

// Clears m values of T at p with 16-byte stores (p 16-byte aligned, m * sizeof(T) a multiple
// of 16: the adjoint's tile regions).
template <class T>
__global__ void k_fill_zero_t(T* __restrict__ p, long long m) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m * (long long)sizeof(T) / 16) reinterpret_cast<float4*>(p)[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

__global__ void k_fill_zero(double* __restrict__ p, long long m) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) p[i] = 0.0;
}

// hipFuncSetAttribute once per kernel (the dynamic LDS size is the same for every call
// with a given model shape; the largest seen is kept)
static apx_status ensure_lds(apx_ctx* ctx, const void* kern, size_t bytes) {
  static std::vector<std::pair<const void*, size_t>> done;
  for (auto& d : done)
    if (d.first == kern && d.second >= bytes) return APX_OK;
  APX_HIP(ctx, hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  for (auto& d : done)
    if (d.first == kern) {
      d.second = bytes;
      return APX_OK;
    }
  done.push_back({kern, bytes});
  return APX_OK;
}

template <class T, int LMAX>
apx_status ace_run(apx_ctx* ctx, const apx_atoms* atoms, const apx_nlist* nl, const apx_ace_model* m,
                   const AceTables<T>& tb, const double* w, const int* active, int n_act, double* e_site,
                   double* f, double* dc1, double* dc2, apx::DevBuf& buf, const double* w2 = nullptr,
                   double* f2 = nullptr) {
  constexpr int TILE = sizeof(T) == 4 ? 64 : 32;
  constexpr int LM = (LMAX + 1) * (LMAX + 1);
  const int n = (int)atoms->n;
  const int na = m->na;
  const long long n_pad = (long long)((n_act + TILE - 1) / TILE) * TILE;
  const size_t bytes_A = sizeof(T) * (size_t)n_pad * na;
  APX_ALLOC(ctx, buf, 2 * bytes_A + 2 * sizeof(double) * (size_t)n_act + sizeof(T) * (size_t)n_pad + 512);
  AceScratch<T> sc;
  sc.A = buf.as<T>();
  sc.Ab = reinterpret_cast<T*>(reinterpret_cast<char*>(buf.p) + bytes_A);
  sc.e_anch = reinterpret_cast<double*>(reinterpret_cast<char*>(buf.p) + 2 * bytes_A);
  sc.fp_anch = sc.e_anch + n_act;
  sc.fp = reinterpret_cast<T*>(sc.fp_anch + n_act + 32);
  // float32 without coefficient gradients: unit adjoint with register accumulation
  const bool use_units = sizeof(T) == 4 && dc1 == nullptr;
  sc.tile_size = use_units ? TILE : 0;
  BoxDev b = make_box(atoms);
  AnchorDev an{};
  an.on = m->anchored;
  if (an.on) {
    an.A = m->anchor.A;
    an.alpha = m->anchor.alpha;
    an.beta = m->anchor.beta;
    an.r0 = m->anchor.r0;
    an.rc = m->anchor.r_cut;
    an.inv_h = 1.0 / m->anchor.h;
    an.rc2 = m->anchor.r_cut * m->anchor.r_cut;
  }
  const T rc = (T)m->r_cut, inv_h = (T)(1.0 / m->h);
  const double rc2 = m->r_cut * m->r_cut;
  const size_t lds1 = BasisLds<T, LMAX>::bytes();
  {
  ProfScope ps(ctx, "ace.basis");
  k_ace_basis<T, LMAX><<<n_act, 64, lds1, ctx->stream>>>(atoms->pos, n, b, nl->count, nl->idx, nl->max_nb, active,
                                                         n_act, m->n_max, rc, inv_h, rc2, tb.Wp, an, sc);
  APX_LAUNCH_CHECK(ctx);
  }
  int lds_max = 0;
  APX_HIP(ctx, hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device));
  if constexpr (sizeof(T) == 4) {
  if (use_units) {
    constexpr int NWU = kUnitWaves;
    const size_t ldsu = sizeof(T) * ((size_t)na * (TILE + 1) + NWU * 4 * TILE + TILE);
    if (ldsu > (size_t)lds_max)
      return fail(ctx, APX_EINVAL, "ACE tile needs %zu bytes of LDS, the device allows %d (reduce n_max)", ldsu, lds_max);
    const long long nab = n_pad * na;
    {
      ProfScope ps(ctx, "ace.zero");
      static_assert(TILE * sizeof(T) % 16 == 0, "tile regions are whole 16-byte groups");
      k_fill_zero_t<T><<<blocks_for(nab * (long long)sizeof(T) / 16, 256), 256, 0, ctx->stream>>>(sc.Ab, nab);
      APX_LAUNCH_CHECK(ctx);
    }
    const unsigned nblk = (unsigned)((n_act + TILE - 1) / TILE);
    // the energy pass needs few registers: 16 waves share a staged tile (at most 64 VGPRs,
    // two tiles per CU, eight waves per SIMD at n_max 10, l_max 4; the reduction buffer
    // reuses the tile)
    constexpr int NWE = 16;
    const size_t ldse = sizeof(T) * std::max((size_t)na * (TILE + 1), (size_t)NWE * 4 * TILE);
    const size_t ldsa = sizeof(T) * (size_t)na * (TILE + 1);
    auto energy = [&](auto kern) -> apx_status {
      if (ensure_lds(ctx, (const void*)kern, ldse) != APX_OK) return APX_EDEVICE;
      ProfScope ps(ctx, "ace.energy");
      kern<<<nblk, NWE * 64, ldse, ctx->stream>>>(sc.A, n_act, na, m->n_max, tb, m->nb1, m->nb2, (T)m->eps,
                                                  sc.e_anch, active, e_site, sc.fp);
      APX_LAUNCH_CHECK(ctx);
      return APX_OK;
    };
    auto adjoint = [&](int nmax_t, auto k0, auto k1, auto k2, auto k3, auto k4) -> apx_status {
      ProfScope ps(ctx, "ace.adjoint");
      static_assert(kUnitGroups == 5, "one kernel per launch group");
      const void* ks[kUnitGroups] = {(const void*)k0, (const void*)k1, (const void*)k2, (const void*)k3,
                                     (const void*)k4};
      for (int g = 0; g < kUnitGroups; ++g) {
        if (m->group_units[g] == 0) continue;
        // the staged tile, or the third-block reduction of the group if larger
        const size_t red = sizeof(T) * (size_t)(NWU / 2) * nmax_t * (2 * g + 1) * 64;
        const size_t ldsg = ldsa > red ? ldsa : red;
        if (ldsg > (size_t)lds_max) return fail(ctx, APX_EINVAL, "ACE adjoint needs %zu bytes of LDS", ldsg);
        if (ensure_lds(ctx, ks[g], ldsg) != APX_OK) return APX_EDEVICE;
        if (g == 0) k0<<<nblk, NWU * 64, ldsg, ctx->stream>>>(sc.A, sc.Ab, n_act, na, m->n_max, tb, m->nb1, sc.fp);
        if (g == 1) k1<<<nblk, NWU * 64, ldsg, ctx->stream>>>(sc.A, sc.Ab, n_act, na, m->n_max, tb, m->nb1, sc.fp);
        if (g == 2) k2<<<nblk, NWU * 64, ldsg, ctx->stream>>>(sc.A, sc.Ab, n_act, na, m->n_max, tb, m->nb1, sc.fp);
        if (g == 3) k3<<<nblk, NWU * 64, ldsg, ctx->stream>>>(sc.A, sc.Ab, n_act, na, m->n_max, tb, m->nb1, sc.fp);
        if (g == 4) k4<<<nblk, NWU * 64, ldsg, ctx->stream>>>(sc.A, sc.Ab, n_act, na, m->n_max, tb, m->nb1, sc.fp);
        APX_LAUNCH_CHECK(ctx);
      }
      return APX_OK;
    };
    apx_status s;
#define APX_PRODUCTS(LM_, NM_)                                                                          \
  s = energy(k_ace_energy<T, LM_, NM_, TILE, NWE, true>);                                               \
  if (s == APX_OK)                                                                                      \
    s = adjoint(NM_, k_ace_adjoint<T, LM_, NM_, TILE, NWU, 0>, k_ace_adjoint<T, LM_, NM_, TILE, NWU, 1>, \
                k_ace_adjoint<T, LM_, NM_, TILE, NWU, 2>, k_ace_adjoint<T, LM_, NM_, TILE, NWU, 3>,     \
                k_ace_adjoint<T, LM_, NM_, TILE, NWU, 4>);
    if constexpr (LMAX == 3) {
      if (m->n_max <= 8) {
        APX_PRODUCTS(3, 8)
      } else {
        APX_PRODUCTS(3, 12)
      }
    } else {
      if (m->n_max <= 10) {
        APX_PRODUCTS(4, 10)
      } else {
        APX_PRODUCTS(4, 12)
      }
    }
#undef APX_PRODUCTS
    if (s != APX_OK) return s;
  }
  }
  if (!use_units) {
    // the LDS version (float64, or float32 with coefficient gradients) stages the tile's
    // A and its adjoint; for large bases the tile is halved so that both fit
    constexpr int NW = sizeof(T) == 4 ? kAceWaves32 : kAceWaves64;
    auto lds_for = [&](int tl) { return sizeof(T) * ((size_t)2 * na * (tl + 1) + NW * 4 * tl + tl); };
    auto products = [&](auto tile_c) -> apx_status {
      constexpr int TL = decltype(tile_c)::value;
      const size_t lds2 = lds_for(TL);
      const unsigned nblk = (unsigned)((n_act + TL - 1) / TL);
      ProfScope ps(ctx, "ace.products");
      if (dc1) {
        auto kern = k_ace_products<T, LMAX, TL, NW, sizeof(T) == 4, true>;
        if (ensure_lds(ctx, (const void*)kern, lds2) != APX_OK) return APX_EDEVICE;
        kern<<<nblk, NW * 64, lds2, ctx->stream>>>(sc.A, sc.Ab, n_act, na, tb, m->nb1, m->nb2, (T)m->eps,
                                                   sc.e_anch, active, w, e_site, dc1, dc2);
      } else {
        auto kern = k_ace_products<T, LMAX, TL, NW, sizeof(T) == 4, false>;
        if (ensure_lds(ctx, (const void*)kern, lds2) != APX_OK) return APX_EDEVICE;
        kern<<<nblk, NW * 64, lds2, ctx->stream>>>(sc.A, sc.Ab, n_act, na, tb, m->nb1, m->nb2, (T)m->eps,
                                                   sc.e_anch, active, w, e_site, nullptr, nullptr);
      }
      APX_LAUNCH_CHECK(ctx);
      return APX_OK;
    };
    apx_status s;
    if (lds_for(TILE) <= (size_t)lds_max)
      s = products(std::integral_constant<int, TILE>{});
    else if (lds_for(TILE / 2) <= (size_t)lds_max)
      s = products(std::integral_constant<int, TILE / 2>{});
    else
      return fail(ctx, APX_EINVAL, "ACE tile needs %zu bytes of LDS, the device allows %d (reduce n_max)",
                  lds_for(TILE / 2), lds_max);
    if (s != APX_OK) return s;
  }
  if (use_units) {
    ProfScope ps(ctx, "ace.backproject");
    k_ace_backproject<T, LMAX><<<(unsigned)(n_pad / TILE), 256, 0, ctx->stream>>>(sc.Ab, sc.A, tb.Wp, m->n_max, na);
    APX_LAUNCH_CHECK(ctx);
  }
  ProfScope ps(ctx, "ace.force");
  auto force = [&](auto nmax_c) {
    constexpr int NM = decltype(nmax_c)::value;
    const size_t lds3 = sizeof(T) * (size_t)ForceLds<T, NM>::KP * LM;
    k_ace_force<T, LMAX, NM><<<n_act, 64, lds3, ctx->stream>>>(atoms->pos, n, b, nl->count, nl->idx, nl->max_nb,
                                                               active, n_act, m->n_max, rc, inv_h, rc2, tb.Wp, an,
                                                               sc, w, f, w2, f2);
  };
  if (m->n_max <= 8) force(std::integral_constant<int, 8>{});
  else if (m->n_max <= 10) force(std::integral_constant<int, 10>{});
  else force(std::integral_constant<int, 12>{});
  APX_LAUNCH_CHECK(ctx);
  return APX_OK;
}

}  // namespace apx

using namespace apx;

namespace {
apx::DevBuf& ace_buffer(apx_ctx* ctx) { return ctx->ace_buf; }
}  // namespace

namespace {
apx_status ace_impl(apx_ctx* ctx, const apx_atoms* atoms, const apx_nlist* nl, const apx_ace_model* m, const double* w,
                    const int32_t* active, int64_t n_active, int32_t precision, double* e_site, double* f,
                    double* dE_dc1, double* dE_dc2, const double* w2, double* f2) {
  if (!ctx) return APX_EINVAL;
  apx_status s = check_atoms(ctx, atoms);
  if (s != APX_OK) return s;
  if (!nl || !m) return fail(ctx, APX_EINVAL, "nl and model are required");
  if (nl->n != atoms->n) return fail(ctx, APX_EINVAL, "nlist size mismatch");
  if (nl->max_nb < 1 || nl->max_nb > 128) return fail(ctx, APX_EINVAL, "nlist max_nb must be in 1..128");
  if (m->r_cut > nl->r_list || (m->anchored && m->anchor.r_cut > nl->r_list))
    return fail(ctx, APX_EINVAL, "ACE cutoff exceeds the neighbour-list cutoff");
  if (precision != APX_FP64 && precision != APX_FP32) return fail(ctx, APX_EINVAL, "precision must be APX_FP64 or APX_FP32");
  if (n_active < 0 || n_active > atoms->n) return fail(ctx, APX_EINVAL, "n_active out of range");
  if ((dE_dc1 == nullptr) != (dE_dc2 == nullptr)) return fail(ctx, APX_EINVAL, "dE_dc1 and dE_dc2 go together");
  const int n = (int)atoms->n;
  if (n > 0 && (!e_site || !f)) return fail(ctx, APX_EINVAL, "e_site and f are required");
  if (n_active > 0 && !active) return fail(ctx, APX_EINVAL, "active is NULL");
  if (n > 0) {
    k_fill_zero<<<blocks_for(3LL * n, 256), 256, 0, ctx->stream>>>(f, 3LL * n);
    k_fill_zero<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(e_site, n);
    if (f2) k_fill_zero<<<blocks_for(3LL * n, 256), 256, 0, ctx->stream>>>(f2, 3LL * n);
    APX_LAUNCH_CHECK(ctx);
  }
  if (dE_dc1) {
    k_fill_zero<<<blocks_for(m->n_basis, 256), 256, 0, ctx->stream>>>(dE_dc1, m->n_basis);
    k_fill_zero<<<blocks_for(m->n_basis, 256), 256, 0, ctx->stream>>>(dE_dc2, m->n_basis);
    APX_LAUNCH_CHECK(ctx);
  }
  if (n_active == 0) return APX_OK;
  const int na_ = (int)n_active;
  if (precision == APX_FP64) {
    if (m->l_max == 3)
      return ace_run<double, 3>(ctx, atoms, nl, m, m->t64, w, active, na_, e_site, f, dE_dc1, dE_dc2, ace_buffer(ctx),
                                w2, f2);
    return ace_run<double, 4>(ctx, atoms, nl, m, m->t64, w, active, na_, e_site, f, dE_dc1, dE_dc2, ace_buffer(ctx),
                              w2, f2);
  }
  if (m->l_max == 3)
    return ace_run<float, 3>(ctx, atoms, nl, m, m->t32, w, active, na_, e_site, f, dE_dc1, dE_dc2, ace_buffer(ctx),
                             w2, f2);
  return ace_run<float, 4>(ctx, atoms, nl, m, m->t32, w, active, na_, e_site, f, dE_dc1, dE_dc2, ace_buffer(ctx),
                           w2, f2);
}
}  // namespace

namespace apx {
apx_status ace_energy_forces_dual(apx_ctx* ctx, const apx_atoms* atoms, const apx_nlist* nl, const apx_ace_model* m,
                                  const double* w, const double* w2, const int32_t* active, int64_t n_active,
                                  int32_t precision, double* e_site, double* f, double* f2) {
  if (!w2 || !f2) return fail(ctx, APX_EINVAL, "the second weight set and its force array are required");
  return ace_impl(ctx, atoms, nl, m, w, active, n_active, precision, e_site, f, nullptr, nullptr, w2, f2);
}
}  // namespace apx

extern "C" apx_status apx_ace_energy_forces(apx_ctx* ctx, const apx_atoms* atoms, const apx_nlist* nl,
                                            const apx_ace_model* m, const double* w, const int32_t* active,
                                            int64_t n_active, int32_t precision, double* e_site, double* f,
                                            double* dE_dc1, double* dE_dc2) {
  return ace_impl(ctx, atoms, nl, m, w, active, n_active, precision, e_site, f, dE_dc1, dE_dc2, nullptr, nullptr);
}
