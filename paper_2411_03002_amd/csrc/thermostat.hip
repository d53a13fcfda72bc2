// Local thermostat: the energy correction of a weight update (Sec. II C 2, Appendix C).
//
// Energy errors (eqs. Delta_V_i, Delta_T_i, Delta_E_i, precise-weight form w = 1 - lambda):
//   dV_i = (w^d_i - w^c_i) (E^fast_i - E^precise_i)
//   dT_i = sum_a [ dt^2/(8m) ((F^c_ia)^2 - (F^d_ia)^2) + (F^c_ia - F^d_ia) v_ia(t+dt/2) dt/2 ]
// with F^c = F^d + dF given as the force of the updated weights plus the difference.
//
// Correction (eqs. p_resc_omega, beta_omega_i): every mobile atom with dE_i != 0 rescales the
// momenta of its group Omega_i (atom i and at most |Omega|-1 mobile atoms within r_omega,
// drawn by Philox4x64-10 priorities) about the group's centre-of-mass velocity by
// beta = sqrt(dE_i / K_rel + 1).  Corrections overlap in their groups and must run in a
// defined order, each on the velocities the previous ones left.  The atoms are coloured by
// the parity pattern of their cell in a grid of cells at least 2 r_omega wide: two atoms of
// one colour in different cells are 2 r_omega apart along some axis, so their groups are
// disjoint.  The groups depend on the positions only, which the correction leaves alone:
// they are drawn for all corrections at once (one workgroup per corrected atom).  Then one
// launch per colour runs one workgroup per cell of that colour, and each workgroup applies
// its cell's corrections one after the other in ascending atom order, each a gather of the
// group's velocities, two reductions and the rescale.
#include <algorithm>
#include <cmath>
#include <cstdint>

#include "common.h"
#include "device_util.h"

namespace apx {

constexpr double kConv = 9648.5332;  // (eV/A)/amu in A/ps^2
constexpr int kThThreads = 256;
constexpr int kSegCap = 8192;    // corrected atoms of one colour cell
constexpr int kCandCap = 4096;   // candidates within r_omega of one atom
constexpr long long kGrpBytes = 1LL << 30;  // drawn groups held at once

// ------------------------------------------------------------------ Philox4x64-10
// Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11): ten
// rounds of (c0, c1, c2, c3) -> (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1,
// lo(M0 c0)), the key bumped by the Weyl constants before every round but the first.
__device__ __forceinline__ uint64_t philox_first_word(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                                      uint64_t k0, uint64_t k1) {
  constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  return c0;
}

// ------------------------------------------------------------------ energy errors
__global__ void k_th_errors(long long n, const uint8_t* __restrict__ frozen, const double* __restrict__ wc,
                            const double* __restrict__ wd, const double* __restrict__ e_fast,
                            const double* __restrict__ e_prec, const double* __restrict__ fd,
                            const double* __restrict__ df, const double* __restrict__ vh, double a, double half_dt,
                            double* __restrict__ dE) {
#pragma clang fp contract(off)
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (frozen && frozen[i]) {
    dE[i] = 0.0;
    return;
  }
  const double c = wc[i], d = wd[i];
  const double dv = c != d ? (d - c) * (e_fast[i] - e_prec[i]) : 0.0;
  double dt = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double f_d = fd[k * n + i];
    const double f_c = f_d + df[k * n + i];
    dt = dt + (a * (f_c * f_c - f_d * f_d) + (f_c - f_d) * vh[k * n + i] * half_dt);
  }
  dE[i] = dv + dt;
}

// ------------------------------------------------------------------ colouring
// Colour cells are numbered colour-major: the cells of colour c (the parity pattern
// (cx & 1) + 2 (cy & 1) + 4 (cz & 1)) are base[c] .. base[c + 1] - 1, so that the corrected
// atoms, listed by cell, come in the order (colour, cell) and each colour is one contiguous
// range of the list.
struct ColourGrid {
  int nc[3];
  double lo[3], inv[3];
  int base[9];
};

__host__ __device__ __forceinline__ int colour_half(int nc, int parity) { return (nc - parity + 1) / 2; }

__device__ __forceinline__ int colour_cell(const ColourGrid& g, double x, int d) {
  int c = (int)floor((x - g.lo[d]) * g.inv[d]);
  return c < 0 ? 0 : (c >= g.nc[d] ? g.nc[d] - 1 : c);
}

// Counts the atoms to correct per colour cell and records each one's cell.
__global__ void k_th_flag(int n, const double* __restrict__ pos, const uint8_t* __restrict__ frozen,
                          const double* __restrict__ dE, ColourGrid g, int* __restrict__ cell_of,
                          int* __restrict__ counts) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if ((frozen && frozen[i]) || dE[i] == 0.0) {
    cell_of[i] = -1;
    return;
  }
  const int cx = colour_cell(g, pos[i], 0);
  const int cy = colour_cell(g, pos[(size_t)n + i], 1);
  const int cz = colour_cell(g, pos[2 * (size_t)n + i], 2);
  const int px = cx & 1, py = cy & 1, pz = cz & 1;
  const int c = g.base[px + 2 * py + 4 * pz] +
                (cx >> 1) + colour_half(g.nc[0], px) * ((cy >> 1) + colour_half(g.nc[1], py) * (cz >> 1));
  cell_of[i] = c;
  atomicAdd(&counts[c], 1);
}

__global__ void k_th_fill(int n, const int* __restrict__ cell_of, const int* __restrict__ start, int* __restrict__ fill,
                          int* __restrict__ list) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = cell_of[i];
  if (c < 0) return;
  list[start[c] + atomicAdd(&fill[c], 1)] = i;
}

// out[0]: the largest count of one cell; out[1 + c], c = 0..8: the first list entry of colour c.
__global__ void k_th_heads(const int* __restrict__ counts, int m, const int* __restrict__ start, ColourGrid g,
                           int* __restrict__ out) {
  int v = 0;
  for (int k = threadIdx.x; k < m; k += blockDim.x) v = counts[k] > v ? counts[k] : v;
  v = wave_max(v);
  if ((threadIdx.x & (kWave - 1)) == 0) atomicMax(out, v);
  if (threadIdx.x < 9) out[1 + threadIdx.x] = start[g.base[threadIdx.x]];
}

// ------------------------------------------------------------------ block helpers
__device__ __forceinline__ int block_exclusive(int v, int* sh, int* total) {
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  int incl = v;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int o = __shfl_up(incl, off, kWave);
    if (lane >= off) incl += o;
  }
  __syncthreads();
  if (lane == kWave - 1) sh[w] = incl;
  __syncthreads();
  int base = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < kThThreads / kWave; ++k) {
    if (k < w) base += sh[k];
    tot += sh[k];
  }
  *total = tot;
  return base + incl - v;
}

// Each list of one cell in ascending atom order (bitonic sort in LDS, padded).
__global__ void __launch_bounds__(kThThreads) k_th_sort(const int* __restrict__ start, int* __restrict__ list) {
  __shared__ int seg[kSegCap];
  const int tid = threadIdx.x;
  const int s0 = start[blockIdx.x], m = start[blockIdx.x + 1] - s0;
  if (m < 2) return;
  int p2 = 1;
  while (p2 < m) p2 <<= 1;
  for (int k = tid; k < p2; k += kThThreads) seg[k] = k < m ? list[s0 + k] : 0x7fffffff;
  __syncthreads();
  for (int size = 2; size <= p2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int k = tid; k < p2; k += kThThreads) {
        const int o = k ^ stride;
        if (o > k) {
          const bool up = (k & size) == 0;
          const int a = seg[k], c = seg[o];
          if ((a > c) == up) {
            seg[k] = c;
            seg[o] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int k = tid; k < m; k += kThThreads) list[s0 + k] = seg[k];
}

struct SearchGrid {
  int nc[3], per[3];
  double lo[3], inv[3], L[3], half[3];
  int reach[3], span[3];
};

struct ThermoArgs {
  const double* pos;
  const uint8_t* frozen;
  const double* dE;
  double* vel;
  int n;
  double r2om;
  int omega_max;
  unsigned long long seed, step;
  double half_m_over_conv;
  const int* cell_start;  // search grid
  const int* cell_atoms;
  const int* seg_start;   // colour cells (colour-major): corrected atoms, ascending per cell
  const int* seg_list;
  int* counters;          // [0] corrected, [1] failed, [2] candidate overflow
};

constexpr int kStCap = 1344;  // stencil cells of one atom (at most 11 per axis)
constexpr int kPer = kCandCap / kThThreads;  // candidate slots per thread

// The search-grid stencil of the atom at (xi, yi, zi): for stencil cell q < total, the
// first slot of its atoms in the cell list (st_base) and the exclusive prefix of the
// stencil's cell sizes (st_pref[q], st_pref[total] = number of slots).  Cells outside a
// non-periodic grid are empty.  Returns the number of slots; every thread calls it.
__device__ int stencil_slots(const ThermoArgs& A, const SearchGrid& g, double xi, double yi, double zi,
                             int* st_base, int* st_pref, int* shi) {
  const int base[3] = {(int)floor((xi - g.lo[0]) * g.inv[0]), (int)floor((yi - g.lo[1]) * g.inv[1]),
                       (int)floor((zi - g.lo[2]) * g.inv[2])};
  const int total = g.span[0] * g.span[1] * g.span[2];
  int carry = 0;
  for (int q0 = 0; q0 < total; q0 += kThThreads) {
    const int q = q0 + (int)threadIdx.x;
    int size = 0;
    if (q < total) {
      const int cc[3] = {q % g.span[0], (q / g.span[0]) % g.span[1], q / (g.span[0] * g.span[1])};
      bool skip = false;
      int cell[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int b = base[d] < 0 ? 0 : (base[d] >= g.nc[d] ? g.nc[d] - 1 : base[d]);
        int c = b + cc[d] + g.reach[d];
        if (g.per[d]) c = ((c % g.nc[d]) + g.nc[d]) % g.nc[d];
        else if (c < 0 || c >= g.nc[d]) skip = true;
        cell[d] = c;
      }
      int first = 0;
      if (!skip) {
        const int c = cell[0] + g.nc[0] * (cell[1] + g.nc[1] * cell[2]);
        first = A.cell_start[c];
        size = A.cell_start[c + 1] - first;
      }
      st_base[q] = first;
    }
    int tot = 0;
    const int ex = block_exclusive(size, shi, &tot);
    if (q < total) st_pref[q] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) st_pref[total] = carry;
  __syncthreads();
  return carry;
}

// The candidates of atom i (mobile j != i with r_ij^2 < r_omega^2) among the thread's
// contiguous range of at most kPer slots, all its loads in flight together: j[u] holds the
// atom of slot e0 + u and bit u of the result marks a candidate.
__device__ unsigned mark_candidates(const ThermoArgs& A, const SearchGrid& g, int i, double xi, double yi,
                                    double zi, const int* st_base, const int* st_pref, int total, int M,
                                    int (&j)[kPer]) {
  const int per = (M + kThThreads - 1) / kThThreads;
  const int e0 = (int)threadIdx.x * per, e1 = e0 + per < M ? e0 + per : M;
#pragma unroll
  for (int u = 0; u < kPer; ++u) j[u] = -1;
  if (e0 >= e1) return 0u;
  // stencil cell of the first slot: the last q with st_pref[q] <= e0
  int lo = 0, hi = total - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (st_pref[mid] <= e0) lo = mid;
    else hi = mid - 1;
  }
  int q = lo;
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    if (e0 + u < e1) {
      while (st_pref[q + 1] <= e0 + u) ++q;
      j[u] = A.cell_atoms[st_base[q] + (e0 + u - st_pref[q])];
    }
  }
  double px[kPer], py[kPer], pz[kPer];
  bool mob[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int jj = j[u] < 0 ? i : j[u];
    px[u] = A.pos[jj];
    py[u] = A.pos[(size_t)A.n + jj];
    pz[u] = A.pos[2 * (size_t)A.n + jj];
    mob[u] = !(A.frozen && A.frozen[jj]);
  }
  unsigned ok = 0u;
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const double dx = min_image(px[u] - xi, g.L[0], g.half[0], g.per[0]);
    const double dy = min_image(py[u] - yi, g.L[1], g.half[1], g.per[1]);
    const double dz = min_image(pz[u] - zi, g.L[2], g.half[2], g.per[2]);
    if (j[u] >= 0 && j[u] != i && mob[u] && sq_dist_exact(dx, dy, dz) < A.r2om) ok |= 1u << u;
  }
  return ok;
}

// The group of list entry e0 + blockIdx.x (one workgroup per corrected atom; positions do
// not change during the correction, so every group is drawn before any rescale): its
// candidates in stencil-slot order, all of them if at most |Omega| - 1, else the
// |Omega| - 1 with the smallest (priority, index), selected by a radix select on the
// priority.  grp row blockIdx.x (stride entries) receives the members other than atom i,
// gsz[blockIdx.x] their number (-1: too many candidates, counted in counters[2]).
__global__ void __launch_bounds__(kThThreads) k_th_groups(ThermoArgs A, SearchGrid sg, int e0, int stride,
                                                         int* __restrict__ grp, int* __restrict__ gsz) {
  __shared__ unsigned long long key[kCandCap];
  __shared__ int cand[kCandCap];
  __shared__ int st_base[kStCap], st_pref[kStCap + 1];
  __shared__ int hist[256];
  __shared__ int shi[kThThreads / kWave];
  __shared__ int sel_state[4];
  const int tid = threadIdx.x;
  const int i = A.seg_list[e0 + (int)blockIdx.x];
  int* out = grp + (size_t)blockIdx.x * stride;
  const double xi = A.pos[i], yi = A.pos[(size_t)A.n + i], zi = A.pos[2 * (size_t)A.n + i];
  const int M = stencil_slots(A, sg, xi, yi, zi, st_base, st_pref, shi);
  if (M > kCandCap) {
    if (tid == 0) {
      atomicAdd(&A.counters[2], 1);
      gsz[blockIdx.x] = -1;
    }
    return;
  }
  int j[kPer];
  const unsigned ok = mark_candidates(A, sg, i, xi, yi, zi, st_base, st_pref, sg.span[0] * sg.span[1] * sg.span[2],
                                      M, j);
  int total = 0;
  const int off = block_exclusive(__popc(ok), shi, &total);
  const int need_max = A.omega_max - 1;
  const bool draw = total > need_max;
  {
    int w = off;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      if (!((ok >> u) & 1u)) continue;
      cand[w] = j[u];
      if (draw)
        key[w] = philox_first_word((unsigned long long)i, (unsigned long long)j[u], A.step, 0ull, A.seed, 0ull);
      ++w;
    }
  }
  __syncthreads();
  if (!draw) {
    for (int k = tid; k < total; k += kThThreads) out[k] = cand[k];
    if (tid == 0) gsz[blockIdx.x] = total;
    return;
  }
  // the need_max smallest (priority, index): radix select on the priority, 8 bits a pass
  unsigned long long prefix = 0ull, mask = 0ull;
  int need = need_max;
  bool exact = false;
  for (int shift = 56; shift >= 0; shift -= 8) {
    for (int k = tid; k < 256; k += kThThreads) hist[k] = 0;
    __syncthreads();
    for (int k = tid; k < total; k += kThThreads)
      if ((key[k] & mask) == prefix) atomicAdd(&hist[(key[k] >> shift) & 255ull], 1);
    __syncthreads();
    {
      // the bucket holding the need-th smallest key: thread = bucket
      static_assert(kThThreads == 256, "one thread per bucket");
      const int h = hist[tid];
      int all = 0;
      const int cum = block_exclusive(h, shi, &all);
      // (need = 0, |Omega| = 1: bucket 0, nothing below it)
      if ((cum < need && cum + h >= need) || (need == 0 && tid == 0)) {
        sel_state[0] = tid;
        sel_state[1] = cum;
        sel_state[2] = h;
      }
    }
    __syncthreads();
    const int bsel = sel_state[0], below = sel_state[1], inb = sel_state[2];
    __syncthreads();
    need -= below;
    prefix |= (unsigned long long)bsel << shift;
    mask |= 255ull << shift;
    if (inb == need) {
      exact = true;
      break;
    }
  }
  if (!exact && tid == 0) {
    // fully equal 64-bit priorities at the threshold: the smallest indices win
    int last = -1;
    for (int r = 0; r < need; ++r) {
      int best = 0x7fffffff;
      for (int k = 0; k < total; ++k)
        if (key[k] == prefix && cand[k] > last && cand[k] < best) best = cand[k];
      last = best;
    }
    sel_state[3] = last;
  }
  __syncthreads();
  // taken: the decided bits smaller, or equal and (the bucket taken whole, or among the
  // `need` smallest indices of fully equal priorities); compacted in slot order
  const int tie_last = sel_state[3];
  const int per = (total + kThThreads - 1) / kThThreads;
  const int k0 = tid * per, k1 = k0 + per < total ? k0 + per : total;
  int mine = 0;
  for (int k = k0; k < k1; ++k) {
    const unsigned long long km = key[k] & mask;
    mine += (km < prefix || (km == prefix && (exact || cand[k] <= tie_last))) ? 1 : 0;
  }
  int taken = 0;
  int w = block_exclusive(mine, shi, &taken);
  for (int k = k0; k < k1; ++k) {
    const unsigned long long km = key[k] & mask;
    if ((km < prefix || (km == prefix && (exact || cand[k] <= tie_last))) && w < stride) out[w++] = cand[k];
  }
  if (tid == 0) gsz[blockIdx.x] = taken < stride ? taken : stride;  // taken = need_max <= stride
}

// Sum over the workgroup of three values, in a fixed order (the waves' sums in wave order).
__device__ __forceinline__ void block_sum3(double& a, double& b, double& c, double* sh) {
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  constexpr int nw = kThThreads / kWave;
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) {
    sh[w] = a;
    sh[nw + w] = b;
    sh[2 * nw + w] = c;
  }
  __syncthreads();
  a = sh[0];
  b = sh[nw];
  c = sh[2 * nw];
#pragma unroll
  for (int k = 1; k < nw; ++k) {
    a += sh[k];
    b += sh[nw + k];
    c += sh[2 * nw + k];
  }
}

__device__ __forceinline__ double block_sum1(double v, double* sh) {
  v = wave_sum(v);
  constexpr int nw = kThThreads / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) sh[threadIdx.x / kWave] = v;
  __syncthreads();
  double t = sh[0];
#pragma unroll
  for (int k = 1; k < nw; ++k) t += sh[k];
  return t;
}

// One workgroup per colour cell of one colour (colour-major cells cbase + blockIdx.x): the
// cell's corrections among list entries [e0, e1), one after the other in list order, on
// the groups that k_th_groups drew for the entries from row0 on (entry e in row e - row0).  Per correction the members'
// velocities are gathered into registers (member k = tid + kThThreads u), reduced twice
// (centre-of-mass velocity, then K_rel), rescaled and written back before the next one.
__global__ void __launch_bounds__(kThThreads) k_th_rescale(ThermoArgs A, int cbase, int row0, int e0, int e1,
                                                          int stride, const int* __restrict__ grp,
                                                          const int* __restrict__ gsz) {
  __shared__ double sh3[3 * (kThThreads / kWave)];
  __shared__ double sh1[kThThreads / kWave];
  const int tid = threadIdx.x;
  const int cell = cbase + (int)blockIdx.x;
  int s = A.seg_start[cell], t = A.seg_start[cell + 1];
  s = s > e0 ? s : e0;
  t = t < e1 ? t : e1;
  int done = 0, failed = 0;
  // the entry, group size, dE and member row of the next correction do not depend on the
  // velocities: they are loaded one correction ahead, while the current gathers are in flight
  int g_n = -1, i_n = 0, jn[kPer];
  double dE_n = 0.0;
  auto fetch = [&](int e) {
    g_n = gsz[e - row0];
    i_n = A.seg_list[e];
    dE_n = A.dE[i_n];
    const int* mem = grp + (size_t)(e - row0) * stride;
#pragma unroll
    for (int u = 0; u < kPer; ++u) jn[u] = tid + kThThreads * u < stride ? mem[tid + kThThreads * u] : -1;
  };
  if (s < t) fetch(s);
  for (int e = s; e < t; ++e) {
    const int g = g_n, i = i_n;
    const double dEi = dE_n;
    int jk[kPer];
    double vx[kPer], vy[kPer], vz[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) jk[u] = tid + kThThreads * u < g ? jn[u] : -1;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      vx[u] = vy[u] = vz[u] = 0.0;
      if (jk[u] >= 0) {
        vx[u] = A.vel[jk[u]];
        vy[u] = A.vel[(size_t)A.n + jk[u]];
        vz[u] = A.vel[2 * (size_t)A.n + jk[u]];
      }
    }
    const double vix = A.vel[i], viy = A.vel[(size_t)A.n + i], viz = A.vel[2 * (size_t)A.n + i];
    if (e + 1 < t) fetch(e + 1);
    if (g < 0) continue;
    double sx = 0.0, sy = 0.0, sz = 0.0;
    if (tid == 0) {
      sx = vix;
      sy = viy;
      sz = viz;
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      sx += vx[u];
      sy += vy[u];
      sz += vz[u];
    }
    block_sum3(sx, sy, sz, sh3);
    const double inv_g = 1.0 / (double)(g + 1);
    const double vcx = sx * inv_g, vcy = sy * inv_g, vcz = sz * inv_g;
    double kr = 0.0;
    if (tid == 0) {
      const double ax = vix - vcx, ay = viy - vcy, az = viz - vcz;
      kr = ax * ax + ay * ay + az * az;
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      if (jk[u] < 0) continue;
      const double ax = vx[u] - vcx, ay = vy[u] - vcy, az = vz[u] - vcz;
      kr += ax * ax + ay * ay + az * az;
    }
    const double k_rel = A.half_m_over_conv * block_sum1(kr, sh1);
    const double rad = dEi / k_rel + 1.0;
    if (!(k_rel > 0.0) || !(rad >= 0.0)) {
      ++failed;
      continue;  // no velocity changed; the reductions' buffers are read before the next writes
    }
    const double beta = sqrt(rad);
    if (tid == 0) {
      A.vel[i] = vcx + beta * (vix - vcx);
      A.vel[(size_t)A.n + i] = vcy + beta * (viy - vcy);
      A.vel[2 * (size_t)A.n + i] = vcz + beta * (viz - vcz);
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int j = jk[u];
      if (j < 0) continue;
      A.vel[j] = vcx + beta * (vx[u] - vcx);
      A.vel[(size_t)A.n + j] = vcy + beta * (vy[u] - vcy);
      A.vel[2 * (size_t)A.n + j] = vcz + beta * (vz[u] - vcz);
    }
    ++done;
    __threadfence_block();
    __syncthreads();
  }
  if (tid == 0) {
    if (done) atomicAdd(&A.counters[0], done);
    if (failed) atomicAdd(&A.counters[1], failed);
  }
}

}  // namespace apx

using namespace apx;

namespace apx {

ColourGrid colour_grid(const apx_atoms* a, double r_omega) {
  ColourGrid g;
  for (int d = 0; d < 3; ++d) {
    const double L = a->hi[d] - a->lo[d];
    long long k = (long long)std::floor(L / (2.0 * r_omega));
    if (k < 1) k = 1;
    if (a->periodic[d] && k > 1 && (k & 1)) k -= 1;
    if (k > 1024) k = 1024;
    g.nc[d] = (int)k;
    g.lo[d] = a->lo[d];
    g.inv[d] = (double)k / L;
  }
  g.base[0] = 0;
  for (int c = 0; c < 8; ++c)
    g.base[c + 1] = g.base[c] + colour_half(g.nc[0], c & 1) * colour_half(g.nc[1], (c >> 1) & 1) *
                                    colour_half(g.nc[2], (c >> 2) & 1);
  return g;
}

apx_status thermostat_errors(apx_ctx* ctx, int64_t n, const uint8_t* frozen, const double* w_c, const double* w_d,
                             const double* e_fast, const double* e_precise, const double* f_d, const double* df,
                             const double* v_half, double dt, double mass, double* dE) {
  if (n <= 0) return APX_OK;
  const double a = dt * dt * kConv / (8.0 * mass);
  ProfScope ps(ctx, "thermo.errors");
  k_th_errors<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(n, frozen, w_c, w_d, e_fast, e_precise, f_d, df, v_half,
                                                          a, 0.5 * dt, dE);
  APX_LAUNCH_CHECK(ctx);
  return APX_OK;
}

apx_status thermostat_correct(apx_ctx* ctx, const apx_atoms* atoms, double* vel, const double* dE,
                              const apx_thermo_params* p, int64_t step, double mass, int64_t* n_corrected,
                              int64_t* n_failed) {
  const int n = (int)atoms->n;
  if (n_corrected) *n_corrected = 0;
  if (n_failed) *n_failed = 0;
  if (n == 0) return APX_OK;
  const ColourGrid cg = colour_grid(atoms, p->r_omega);
  const long long ncc = cg.base[8];
  // scratch: cell of each atom, per-cell counts/fill/start, the lists, counters
  APX_ALLOC(ctx, ctx->itmp, sizeof(int) * ((size_t)n * 2 + (size_t)ncc * 3 + 16));
  int* cell_of = ctx->itmp.as<int>();
  int* list = cell_of + n;
  int* counts = list + n;
  int* fill = counts + ncc;
  int* start = fill + ncc;  // ncc + 1
  int* counters = start + ncc + 1;  // [0] corrected [1] failed [2] overflow [3] max segment [4..12] colour heads
  APX_HIP(ctx, hipMemsetAsync(counts, 0, sizeof(int) * (size_t)ncc * 2, ctx->stream));
  APX_HIP(ctx, hipMemsetAsync(counters, 0, sizeof(int) * 4, ctx->stream));
  {
    ProfScope ps(ctx, "thermo.flag");
    k_th_flag<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(n, atoms->pos, atoms->frozen, dE, cg, cell_of, counts);
    APX_LAUNCH_CHECK(ctx);
  }
  apx_status s = scan_exclusive(ctx, counts, ncc, start);
  if (s != APX_OK) return s;
  k_th_heads<<<1, 256, 0, ctx->stream>>>(counts, (int)ncc, start, cg, counters + 3);
  APX_LAUNCH_CHECK(ctx);
  int head[10];
  s = read_ints(ctx, counters + 3, head, 10);
  if (s != APX_OK) return s;
  const int total = head[9];
  if (total == 0) return APX_OK;
  if (head[0] > kSegCap)
    return fail(ctx, APX_ECAPACITY, "thermostat: %d corrections in one colour cell exceed %d (reduce r_omega)",
                head[0], kSegCap);
  {
    ProfScope ps(ctx, "thermo.order");
    k_th_fill<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(n, cell_of, start, fill, list);
    APX_LAUNCH_CHECK(ctx);
    k_th_sort<<<(unsigned)ncc, kThThreads, 0, ctx->stream>>>(start, list);
    APX_LAUNCH_CHECK(ctx);
  }
  // candidate search grid: cells at least r_omega/2 wide, a stencil of every cell within reach
  Grid g = make_grid(atoms, 0.5 * p->r_omega);
  s = bin_atoms(ctx, atoms, g);
  if (s != APX_OK) return s;
  SearchGrid sg;
  for (int d = 0; d < 3; ++d) {
    sg.nc[d] = g.nc[d];
    sg.per[d] = g.per[d];
    sg.lo[d] = g.lo[d];
    sg.inv[d] = g.inv_cell[d];
    sg.L[d] = g.L[d];
    sg.half[d] = 0.5 * g.L[d];
    const double edge = g.L[d] / g.nc[d];
    const int reach = (int)std::ceil(p->r_omega / edge);
    if (2 * reach + 1 >= g.nc[d]) {
      // every cell once; the stencil starts at the cell below (periodic axes wrap)
      sg.reach[d] = g.per[d] ? -(g.nc[d] / 2) : -g.nc[d];
      sg.span[d] = g.per[d] ? g.nc[d] : 2 * g.nc[d] + 1;
    } else {
      sg.reach[d] = -reach;
      sg.span[d] = 2 * reach + 1;
    }
  }
  ThermoArgs A;
  A.pos = atoms->pos;
  A.frozen = atoms->frozen;
  A.dE = dE;
  A.vel = vel;
  A.n = n;
  A.r2om = p->r_omega * p->r_omega;
  A.omega_max = p->omega_max;
  A.seed = (unsigned long long)p->seed;
  A.step = (unsigned long long)step;
  A.half_m_over_conv = 0.5 * mass / kConv;
  A.cell_start = ctx->cell_start.as<int>();
  A.cell_atoms = ctx->cell_atoms.as<int>();
  A.seg_start = start;
  A.seg_list = list;
  A.counters = counters;
  // groups of at most kGrpBytes at a time: each batch of list entries draws its groups,
  // then rescales them colour by colour (entries of one colour are contiguous, so the
  // corrections keep the order (colour, cell, atom))
  const int stride = std::max(1, std::min(kCandCap, p->omega_max - 1));
  long long batch = std::max(1LL, std::min<long long>(total, kGrpBytes / (4LL * (stride + 1))));
  if (p->group_batch > 0 && p->group_batch < batch) batch = p->group_batch;
  APX_ALLOC(ctx, ctx->thermo_grp, sizeof(int) * (size_t)batch * (stride + 1));
  int* grp = ctx->thermo_grp.as<int>();
  int* gsz = grp + (size_t)batch * stride;
  for (long long b0 = 0; b0 < total; b0 += batch) {
    const int b1 = (int)std::min<long long>(total, b0 + batch);
    {
      ProfScope ps(ctx, "thermo.groups");
      k_th_groups<<<(unsigned)(b1 - b0), kThThreads, 0, ctx->stream>>>(A, sg, (int)b0, stride, grp, gsz);
      APX_LAUNCH_CHECK(ctx);
    }
    for (int colour = 0; colour < 8; ++colour) {
      const int lo = std::max(head[1 + colour], (int)b0), hi = std::min(head[2 + colour], b1);
      if (lo >= hi) continue;
      ProfScope ps(ctx, "thermo.rescale");
      k_th_rescale<<<(unsigned)(cg.base[colour + 1] - cg.base[colour]), kThThreads, 0, ctx->stream>>>(
          A, cg.base[colour], (int)b0, lo, hi, stride, grp, gsz);
      APX_LAUNCH_CHECK(ctx);
    }
  }
  int res[3] = {0, 0, 0};
  s = read_ints(ctx, counters, res, 3);
  if (s != APX_OK) return s;
  if (n_corrected) *n_corrected = res[0];
  if (n_failed) *n_failed = res[1];
  if (res[2] > 0)
    return fail(ctx, APX_ECAPACITY, "thermostat: %d atoms have more than %d candidates within r_omega", res[2],
                kCandCap);
  return APX_OK;
}

}  // namespace apx

extern "C" apx_status apx_thermostat_energy_errors(apx_ctx* ctx, int64_t n, const uint8_t* frozen, const double* w_c,
                                                   const double* w_d, const double* e_fast, const double* e_precise,
                                                   const double* f_d, const double* df, const double* v_half,
                                                   double dt, double mass, double* dE) {
  if (!ctx) return APX_EINVAL;
  if (n < 0 || n > 0x7fffffff) return fail(ctx, APX_EINVAL, "bad atom count");
  if (n > 0 && (!w_c || !w_d || !e_fast || !e_precise || !f_d || !df || !v_half || !dE))
    return fail(ctx, APX_EINVAL, "thermostat arrays are required");
  if (!(dt > 0.0) || !(mass > 0.0)) return fail(ctx, APX_EINVAL, "dt and mass must be positive");
  return thermostat_errors(ctx, n, frozen, w_c, w_d, e_fast, e_precise, f_d, df, v_half, dt, mass, dE);
}

extern "C" apx_status apx_thermostat_correct(apx_ctx* ctx, const apx_atoms* atoms, double* vel, const double* dE,
                                             const apx_thermo_params* p, int64_t step, double mass,
                                             int64_t* n_corrected, int64_t* n_failed) {
  if (!ctx) return APX_EINVAL;
  apx_status s = check_atoms(ctx, atoms);
  if (s != APX_OK) return s;
  if (!p) return fail(ctx, APX_EINVAL, "thermostat parameters are required");
  if (atoms->n > 0 && (!vel || !dE)) return fail(ctx, APX_EINVAL, "vel and dE are required");
  if (!(p->r_omega > 0.0) || !(mass > 0.0)) return fail(ctx, APX_EINVAL, "r_omega and mass must be positive");
  if (p->omega_max < 1) return fail(ctx, APX_EINVAL, "omega_max must be at least 1");
  if (p->group_batch < 0) return fail(ctx, APX_EINVAL, "group_batch must be >= 0");
  if (step < 0) return fail(ctx, APX_EINVAL, "step must be >= 0");
  s = thermostat_correct(ctx, atoms, vel, dE, p, step, mass, n_corrected, n_failed);
  if (s != APX_OK) return s;
  if (n_failed && *n_failed > 0)
    return fail(ctx, APX_ERADICAND, "thermostat: %lld corrections with a negative radicand were skipped",
                (long long)*n_failed);
  return APX_OK;
}
