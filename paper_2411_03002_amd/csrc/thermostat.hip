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
// disjoint.  One launch per colour runs one workgroup per cell of that colour, and each
// workgroup applies its cell's corrections one after the other in ascending atom order.
#include <cmath>
#include <cstdint>

#include "common.h"
#include "device_util.h"

namespace apx {

constexpr double kConv = 9648.5332;  // (eV/A)/amu in A/ps^2
constexpr int kThThreads = 256;
constexpr int kSegCap = 8192;    // corrected atoms of one colour cell
constexpr int kCandCap = 4096;   // candidates within r_omega of one atom

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
struct ColourGrid {
  int nc[3];
  double lo[3], inv[3];
};

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
  const int c = cx + g.nc[0] * (cy + g.nc[1] * cz);
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

__global__ void k_th_max(const int* __restrict__ counts, int m, int* __restrict__ out) {
  int v = 0;
  for (int k = threadIdx.x; k < m; k += blockDim.x) v = counts[k] > v ? counts[k] : v;
  v = wave_max(v);
  if ((threadIdx.x & (kWave - 1)) == 0) atomicMax(out, v);
}

// ------------------------------------------------------------------ block helpers
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int w = threadIdx.x / kWave;
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int k = 0; k < kThThreads / kWave; ++k) t += sh[k];
  return t;
}

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
  const int* seg_start;   // colour cells: corrected atoms
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

// The candidates of atom i (mobile j != i with r_ij^2 < r_omega^2) in slot order: every
// thread tests a contiguous range of at most kPer slots (all its loads in flight together)
// and marks them in ctmp (the atom index, or -1); returns the thread's count.
__device__ int mark_candidates(const ThermoArgs& A, const SearchGrid& g, int i, double xi, double yi, double zi,
                               const int* st_base, const int* st_pref, int total, int M, int* ctmp) {
  const int per = (M + kThThreads - 1) / kThThreads;
  const int e0 = (int)threadIdx.x * per, e1 = e0 + per < M ? e0 + per : M;
  if (e0 >= e1) return 0;
  // stencil cell of the first slot: the last q with st_pref[q] <= e0
  int lo = 0, hi = total - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (st_pref[mid] <= e0) lo = mid;
    else hi = mid - 1;
  }
  int q = lo, mine = 0;
  const int e = e0;
  int j[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    j[u] = -1;
    if (e + u < e1) {
      while (st_pref[q + 1] <= e + u) ++q;
      j[u] = A.cell_atoms[st_base[q] + (e + u - st_pref[q])];
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
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    if (e + u < e1) {
      const double dx = min_image(px[u] - xi, g.L[0], g.half[0], g.per[0]);
      const double dy = min_image(py[u] - yi, g.L[1], g.half[1], g.per[1]);
      const double dz = min_image(pz[u] - zi, g.L[2], g.half[2], g.per[2]);
      const bool ok = j[u] != i && mob[u] && sq_dist_exact(dx, dy, dz) < A.r2om;
      ctmp[e + u] = ok ? j[u] : -1;
      mine += ok ? 1 : 0;
    }
  }
  return mine;
}

// One workgroup per colour cell of one colour: the cell's corrections, one after the other.
__global__ void __launch_bounds__(kThThreads) k_th_rescale(ThermoArgs A, SearchGrid sg, ColourGrid cg, int colour) {
  __shared__ int seg[kSegCap];
  __shared__ unsigned long long key[kCandCap];
  __shared__ int cand[kCandCap];
  __shared__ int ctmp[kCandCap];
  __shared__ int st_base[kStCap], st_pref[kStCap + 1];
  __shared__ int hist[256];
  __shared__ double shd[kThThreads / kWave];
  __shared__ int shi[kThThreads / kWave];
  __shared__ int sel_state[4];
  const int tid = threadIdx.x;
  // the blockIdx-th cell of this colour
  const int h0 = (cg.nc[0] - (colour & 1) + 1) / 2, h1 = (cg.nc[1] - ((colour >> 1) & 1) + 1) / 2;
  const int b = blockIdx.x;
  const int cx = 2 * (b % h0) + (colour & 1), cy = 2 * ((b / h0) % h1) + ((colour >> 1) & 1),
            cz = 2 * (b / (h0 * h1)) + ((colour >> 2) & 1);
  if (cx >= cg.nc[0] || cy >= cg.nc[1] || cz >= cg.nc[2]) return;
  const int cell = cx + cg.nc[0] * (cy + cg.nc[1] * cz);
  const int s0 = A.seg_start[cell], m = A.seg_start[cell + 1] - s0;
  if (m == 0) return;
  // the cell's corrected atoms in ascending order (bitonic sort in LDS, padded)
  int p2 = 1;
  while (p2 < m) p2 <<= 1;
  for (int k = tid; k < p2; k += kThThreads) seg[k] = k < m ? A.seg_list[s0 + k] : 0x7fffffff;
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
  const int need_max = A.omega_max - 1;
  for (int t = 0; t < m; ++t) {
    const int i = seg[t];
    const double xi = A.pos[i], yi = A.pos[(size_t)A.n + i], zi = A.pos[2 * (size_t)A.n + i];
    // candidates in stencil-slot order: mark, scan, compact
    const int M = stencil_slots(A, sg, xi, yi, zi, st_base, st_pref, shi);
    if (M > kCandCap) {
      if (tid == 0) atomicAdd(&A.counters[2], 1);
      __syncthreads();
      continue;
    }
    const int mine = mark_candidates(A, sg, i, xi, yi, zi, st_base, st_pref, sg.span[0] * sg.span[1] * sg.span[2],
                                     M, ctmp);
    int total = 0;
    const int off = block_exclusive(mine, shi, &total);
    const bool draw = total > need_max;
    {
      const int per = (M + kThThreads - 1) / kThThreads;
      const int e0 = tid * per, e1 = e0 + per < M ? e0 + per : M;
      int w = off;
      for (int e = e0; e < e1; ++e) {
        const int j = ctmp[e];
        if (j < 0) continue;
        cand[w] = j;
        if (draw) key[w] = philox_first_word((unsigned long long)i, (unsigned long long)j, A.step, 0ull, A.seed, 0ull);
        ++w;
      }
    }
    __syncthreads();
    // selection of the need_max smallest (priority, index) by radix select on the priority
    if (draw) {
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
      // mark: taken if the decided bits are smaller, or equal and (the bucket is taken
      // whole, or among the `need` smallest indices of fully equal priorities)
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
      const int tie_last = sel_state[3];
      for (int k = tid; k < total; k += kThThreads) {
        const unsigned long long km = key[k] & mask;
        const bool take = km < prefix || (km == prefix && (exact || cand[k] <= tie_last));
        if (!take) cand[k] = -1 - cand[k];
      }
      __syncthreads();
    }
    // centre-of-mass velocity of the group (atom i and the taken candidates); every thread
    // holds the velocities of its candidates k = tid + kThThreads u in registers
    const int gsize = 1 + (draw ? need_max : total);
    int jk[kPer];
    double vx[kPer], vy[kPer], vz[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int k = tid + kThThreads * u;
      jk[u] = k < total ? cand[k] : -1;
      const int jj = jk[u] < 0 ? i : jk[u];
      vx[u] = A.vel[jj];
      vy[u] = A.vel[(size_t)A.n + jj];
      vz[u] = A.vel[2 * (size_t)A.n + jj];
    }
    const double vix = A.vel[i], viy = A.vel[(size_t)A.n + i], viz = A.vel[2 * (size_t)A.n + i];
    double sx = 0.0, sy = 0.0, sz = 0.0;
    if (tid == 0) {
      sx = vix;
      sy = viy;
      sz = viz;
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      if (jk[u] < 0) continue;
      sx += vx[u];
      sy += vy[u];
      sz += vz[u];
    }
    const double inv_g = 1.0 / (double)gsize;
    const double vcx = block_sum(sx, shd) * inv_g;
    const double vcy = block_sum(sy, shd) * inv_g;
    const double vcz = block_sum(sz, shd) * inv_g;
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
    const double k_rel = A.half_m_over_conv * block_sum(kr, shd);
    const double rad = A.dE[i] / k_rel + 1.0;
    if (!(k_rel > 0.0) || !(rad >= 0.0)) {
      if (tid == 0) atomicAdd(&A.counters[1], 1);
      __syncthreads();
      continue;
    }
    const double beta = sqrt(rad);
    if (tid == 0) {
      A.vel[i] = vcx + beta * (vix - vcx);
      A.vel[(size_t)A.n + i] = vcy + beta * (viy - vcy);
      A.vel[2 * (size_t)A.n + i] = vcz + beta * (viz - vcz);
      atomicAdd(&A.counters[0], 1);
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int j = jk[u];
      if (j < 0) continue;
      A.vel[j] = vcx + beta * (vx[u] - vcx);
      A.vel[(size_t)A.n + j] = vcy + beta * (vy[u] - vcy);
      A.vel[2 * (size_t)A.n + j] = vcz + beta * (vz[u] - vcz);
    }
    __threadfence_block();
    __syncthreads();
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
  const long long ncc = (long long)cg.nc[0] * cg.nc[1] * cg.nc[2];
  // scratch: cell of each atom, per-cell counts/fill/start, the lists, counters
  APX_ALLOC(ctx, ctx->itmp, sizeof(int) * ((size_t)n * 2 + (size_t)ncc * 3 + 16));
  int* cell_of = ctx->itmp.as<int>();
  int* list = cell_of + n;
  int* counts = list + n;
  int* fill = counts + ncc;
  int* start = fill + ncc;  // ncc + 1
  int* counters = start + ncc + 1;  // [0] corrected [1] failed [2] overflow [3] max segment
  APX_HIP(ctx, hipMemsetAsync(counts, 0, sizeof(int) * (size_t)ncc * 2, ctx->stream));
  APX_HIP(ctx, hipMemsetAsync(counters, 0, sizeof(int) * 4, ctx->stream));
  {
    ProfScope ps(ctx, "thermo.flag");
    k_th_flag<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(n, atoms->pos, atoms->frozen, dE, cg, cell_of, counts);
    APX_LAUNCH_CHECK(ctx);
    k_th_max<<<1, 256, 0, ctx->stream>>>(counts, (int)ncc, counters + 3);
    APX_LAUNCH_CHECK(ctx);
  }
  apx_status s = scan_exclusive(ctx, counts, ncc, start);
  if (s != APX_OK) return s;
  int head[2] = {0, 0};
  s = read_ints(ctx, counters + 3, head, 1);
  if (s != APX_OK) return s;
  if (head[0] == 0) return APX_OK;
  if (head[0] > kSegCap)
    return fail(ctx, APX_ECAPACITY, "thermostat: %d corrections in one colour cell exceed %d (reduce r_omega)",
                head[0], kSegCap);
  k_th_fill<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(n, cell_of, start, fill, list);
  APX_LAUNCH_CHECK(ctx);
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
  for (int colour = 0; colour < 8; ++colour) {
    const int h0 = (cg.nc[0] - (colour & 1) + 1) / 2, h1 = (cg.nc[1] - ((colour >> 1) & 1) + 1) / 2,
              h2 = (cg.nc[2] - ((colour >> 2) & 1) + 1) / 2;
    const long long blocks = (long long)h0 * h1 * h2;
    if (blocks == 0) continue;
    ProfScope ps(ctx, "thermo.rescale");
    k_th_rescale<<<(unsigned)blocks, kThThreads, 0, ctx->stream>>>(A, sg, cg, colour);
    APX_LAUNCH_CHECK(ctx);
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
  if (step < 0) return fail(ctx, APX_EINVAL, "step must be >= 0");
  s = thermostat_correct(ctx, atoms, vel, dE, p, step, mass, n_corrected, n_failed);
  if (s != APX_OK) return s;
  if (n_failed && *n_failed > 0)
    return fail(ctx, APX_ERADICAND, "thermostat: %lld corrections with a negative radicand were skipped",
                (long long)*n_failed);
  return APX_OK;
}
