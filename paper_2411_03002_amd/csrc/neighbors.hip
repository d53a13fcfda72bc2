// Cell-list neighbour build: full Verlet list in neighbour-major ELL layout, rows in
// ascending neighbour index.
#include <climits>
#include <cmath>

#include "common.h"
#include "device_util.h"

namespace apx {

constexpr int kNbCap = 128;       // largest row capacity (max_nb)
constexpr int kCellWaves = 4;     // waves per block; a block serves the atoms of one cell
constexpr int kCandCap = 1024;    // candidates staged in LDS (more are read from global memory)

// Orders the LDS accesses of one wave (the LDS executes a wave's accesses in issue order;
// this keeps the compiler from moving them across).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One step of a bitonic network across the wave: partner lane = lane ^ j; `up` selects
// ascending order for the lane's block, the lower lane of a pair keeps the smaller key
// there.
__device__ __forceinline__ int bitonic_step(int v, int lane, int j, bool up) {
  const int o = __shfl_xor(v, j, kWave);
  const bool lower = (lane & j) == 0;
  return (lower == up) ? min(v, o) : max(v, o);
}

// Sorts 64 keys (one per lane) ascending by lane.
__device__ __forceinline__ int wave_sort64(int v, int lane) {
#pragma unroll
  for (int k = 2; k <= 64; k <<= 1)
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) v = bitonic_step(v, lane, j, (lane & k) == 0);
  return v;
}

// Sorts 128 keys, element e = lane + 64 h held in v[h], ascending by e.
__device__ __forceinline__ void wave_sort128(int& v0, int& v1, int lane) {
#pragma unroll
  for (int k = 2; k <= 128; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      if (j == 64) {  // partners are the lane's own two elements (k = 128: ascending)
        const int a = min(v0, v1), b = max(v0, v1);
        v0 = a;
        v1 = b;
      } else {
        v0 = bitonic_step(v0, lane, j, (lane & k) == 0);
        v1 = bitonic_step(v1, lane, j, ((lane + 64) & k) == 0);
      }
    }
  }
}

// Rows of the cell's atoms taken by one wave (atoms wv, wv + kCellWaves, ... of the cell):
// candidates from LDS (STAGED) or from global memory; returns the longest row.
template <bool STAGED>
__device__ __forceinline__ int cell_rows(const double* __restrict__ pos, int n, const Grid& g, const int* __restrict__ cell_atoms,
                         double rl2, int max_nb, int* __restrict__ count, int* __restrict__ idx, const int* cand,
                         const double* cpx, const double* cpy, const double* cpz, int* row, const int* sc_start,
                         const int* sc_pref, int b0, int e0, int M, int wv, int lane) {
  const double Lx = g.L[0], Ly = g.L[1], Lz = g.L[2];
  const double hx = 0.5 * Lx, hy = 0.5 * Ly, hz = 0.5 * Lz;
  int longest = 0;
  const int self = sc_pref[13];  // the cell's own atoms among the candidates
  for (int a = wv; a < e0 - b0; a += kCellWaves) {
    int i;
    double xi, yi, zi;
    if constexpr (STAGED) {
      i = cand[self + a];
      xi = cpx[self + a];
      yi = cpy[self + a];
      zi = cpz[self + a];
    } else {
      i = cell_atoms[b0 + a];
      xi = pos[i];
      yi = pos[(size_t)n + i];
      zi = pos[2 * (size_t)n + i];
    }
    int cnt = 0;
    for (int s0 = 0; s0 < M; s0 += 64) {
      const int e = s0 + lane;
      bool ok = false;
      int j = -1;
      if (e < M) {
        double px, py, pz;
        if constexpr (STAGED) {
          j = cand[e];
          px = cpx[e];
          py = cpy[e];
          pz = cpz[e];
        } else {
          int sc = 0;
          while (sc_pref[sc + 1] <= e) ++sc;
          j = cell_atoms[sc_start[sc] + (e - sc_pref[sc])];
          px = pos[j];
          py = pos[(size_t)n + j];
          pz = pos[2 * (size_t)n + j];
        }
        const double dx = min_image(px - xi, Lx, hx, g.per[0]);
        const double dy = min_image(py - yi, Ly, hy, g.per[1]);
        const double dz = min_image(pz - zi, Lz, hz, g.per[2]);
        ok = j != i && sq_dist_exact(dx, dy, dz) < rl2;
      }
      const unsigned long long m = __ballot(ok);
      if (ok) {
        const int p = cnt + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                           __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
        if (p < kNbCap) row[p] = j;
      }
      cnt += __popcll(m);
    }
    wave_lds_sync();
    const int kept = cnt < max_nb ? cnt : max_nb;
    int v0 = lane < kept ? row[lane] : INT_MAX;
    if (kept <= 64) {
      v0 = wave_sort64(v0, lane);
      if (lane < kept) idx[(size_t)lane * n + i] = v0;
    } else {
      int v1 = lane + 64 < kept ? row[lane + 64] : INT_MAX;
      wave_sort128(v0, v1, lane);
      idx[(size_t)lane * n + i] = v0;
      if (lane + 64 < kept) idx[(size_t)(lane + 64) * n + i] = v1;
    }
    if (lane == 0) count[i] = cnt;
    longest = cnt > longest ? cnt : longest;
    wave_lds_sync();
  }
  return longest;
}

// One block per cell.  The candidates (atoms of the up to 27 neighbouring cells, fewer
// for grids with fewer than 3 cells along a periodic axis) are staged in LDS with their
// positions; each wave then takes atoms of the cell in turn: the candidates are tested 64
// at a time, accepted indices are compacted into the wave's LDS row by ballot, and the
// row is sorted by a bitonic network across the wave and written out.  The cell's own
// atoms are among the staged candidates (stencil cell 13, offset (0, 0, 0)), so their
// indices and positions come from LDS as well.  Entries beyond max_nb are only counted,
// so the caller learns the length it needs.
__global__ void __launch_bounds__(kCellWaves * 64) k_build(const double* __restrict__ pos, int n, Grid g,
                                                            const int* __restrict__ cell_start,
                                                            const int* __restrict__ cell_atoms, double rl2,
                                                            int max_nb, int* __restrict__ count,
                                                            int* __restrict__ idx, int* __restrict__ flags) {
  __shared__ int cand[kCandCap];
  __shared__ double cpx[kCandCap], cpy[kCandCap], cpz[kCandCap];
  __shared__ int rows[kCellWaves][kNbCap];
  __shared__ int sc_start[27], sc_pref[28];
  const int c = xcd_block(blockIdx.x, gridDim.x);
  const int b0 = cell_start[c], e0 = cell_start[c + 1];
  if (b0 == e0) return;  // uniform over the block
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (wv == 0) {
    // stencil cell `lane` (< 27): offsets -1..1 per axis, restricted as for the grid
    int sz = 0, st = 0;
    if (lane < 27) {
      const int ci[3] = {c % g.nc[0], (c / g.nc[0]) % g.nc[1], c / (g.nc[0] * g.nc[1])};
      const int o[3] = {lane % 3 - 1, (lane / 3) % 3 - 1, lane / 9 - 1};
      bool ok = true;
      int cc[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        int lo, hi;
        if (g.per[d]) {
          lo = g.nc[d] >= 3 ? -1 : 0;
          hi = g.nc[d] >= 3 ? 1 : g.nc[d] - 1;
        } else {
          lo = ci[d] > 0 ? -1 : 0;
          hi = ci[d] < g.nc[d] - 1 ? 1 : 0;
        }
        ok = ok && o[d] >= lo && o[d] <= hi;
        cc[d] = ci[d] + o[d];
        if (g.per[d]) cc[d] = (cc[d] + g.nc[d]) % g.nc[d];
      }
      if (ok) {
        const int id = cc[0] + g.nc[0] * (cc[1] + g.nc[1] * cc[2]);
        st = cell_start[id];
        sz = cell_start[id + 1] - st;
      }
    }
    int incl = sz;
#pragma unroll
    for (int off = 1; off < 32; off <<= 1) {
      const int u = __shfl_up(incl, off, kWave);
      if (lane >= off) incl += u;
    }
    if (lane < 27) {
      sc_start[lane] = st;
      sc_pref[lane] = incl - sz;
    }
    if (lane == 26) sc_pref[27] = incl;
  }
  __syncthreads();
  const int M = sc_pref[27];
  const bool staged = M <= kCandCap;
  // candidate e lies in stencil cell s with sc_pref[s] <= e < sc_pref[s + 1]
  auto cand_index = [&](int e) {
    int s = 0;
    while (sc_pref[s + 1] <= e) ++s;
    return cell_atoms[sc_start[s] + (e - sc_pref[s])];
  };
  if (staged) {
    for (int e = tid; e < M; e += kCellWaves * 64) {
      const int j = cand_index(e);
      cand[e] = j;
      cpx[e] = pos[j];
      cpy[e] = pos[(size_t)n + j];
      cpz[e] = pos[2 * (size_t)n + j];
    }
  }
  __syncthreads();
  // the two paths are separate instantiations, so that LDS reads stay LDS instructions
  const int longest = staged ? cell_rows<true>(pos, n, g, cell_atoms, rl2, max_nb, count, idx, cand, cpx, cpy, cpz,
                                               rows[wv], sc_start, sc_pref, b0, e0, M, wv, lane)
                             : cell_rows<false>(pos, n, g, cell_atoms, rl2, max_nb, count, idx, cand, cpx, cpy, cpz,
                                                rows[wv], sc_start, sc_pref, b0, e0, M, wv, lane);
  // the longest row and the capacity flag: one atomic per wave (longest is wave-uniform)
  if (lane == 0 && longest > 0) {
    if (longest > max_nb) atomicOr(&flags[0], 4);
    sparse_atomic_max(&flags[1], longest);
  }
}

}  // namespace apx

using namespace apx;

extern "C" apx_status apx_build_neighbors(apx_ctx* ctx, const apx_atoms* atoms, double r_list,
                                          apx_nlist* nl, int32_t* needed) {
  if (!ctx) return APX_EINVAL;
  apx_status s = check_atoms(ctx, atoms);
  if (s != APX_OK) return s;
  if (!nl || !needed) return fail(ctx, APX_EINVAL, "nl and needed are required");
  if (nl->n != atoms->n) return fail(ctx, APX_EINVAL, "nlist size %lld != atoms %lld", (long long)nl->n, (long long)atoms->n);
  if (nl->max_nb < 1 || nl->max_nb > kNbCap) return fail(ctx, APX_EINVAL, "max_nb must be in 1..%d", kNbCap);
  if (atoms->n > 0 && (!nl->count || !nl->idx)) return fail(ctx, APX_EINVAL, "nlist arrays are NULL");
  if (!(r_list > 0.0)) return fail(ctx, APX_EINVAL, "r_list must be positive");
  for (int d = 0; d < 3; ++d)
    if (atoms->periodic[d] && !(r_list < 0.5 * (atoms->hi[d] - atoms->lo[d])))
      return fail(ctx, APX_EINVAL, "r_list %.4f must be below half the periodic box (axis %d)", r_list, d);
  nl->r_list = r_list;
  const int n = (int)atoms->n;
  if (n == 0) {
    *needed = 0;
    return APX_OK;
  }
  Grid g = make_grid(atoms, r_list);
  {
    ProfScope ps(ctx, "nbr.bin");
    s = bin_atoms(ctx, atoms, g);
  }
  if (s != APX_OK) return s;
  ProfScope ps(ctx, "nbr.build");
  const long long ncell = g.ncell();
  if (ncell > INT_MAX) return fail(ctx, APX_EINVAL, "too many cells (%lld)", ncell);
  k_build<<<(unsigned)ncell, kCellWaves * 64, 0, ctx->stream>>>(
      atoms->pos, n, g, ctx->cell_start.as<int>(), ctx->cell_atoms.as<int>(), r_list * r_list, nl->max_nb,
      nl->count, nl->idx, ctx->flags.as<int>());
  APX_LAUNCH_CHECK(ctx);
  int fl[2];
  s = read_ints(ctx, ctx->flags.as<int>(), fl, 2);
  if (s != APX_OK) return s;
  *needed = fl[1];
  if (fl[0] & 1) return fail(ctx, APX_EINVAL, "a coordinate lies outside the box along a non-periodic axis");
  if (fl[0] & 2) return fail(ctx, APX_ENONFINITE, "non-finite position");
  if (fl[0] & 4) return fail(ctx, APX_ECAPACITY, "neighbour row of %d entries exceeds max_nb %d", fl[1], nl->max_nb);
  return APX_OK;
}
