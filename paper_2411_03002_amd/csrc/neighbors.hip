// Cell-list neighbour build: full Verlet list in neighbour-major ELL layout, rows in
// ascending neighbour index.
#include <cmath>

#include "common.h"
#include "device_util.h"

namespace apx {

constexpr int kNbThreads = 64;  // one wave per block: each thread owns one row in LDS
constexpr int kNbCap = 128;     // largest row capacity (max_nb)
constexpr int kBatch = 8;       // candidates whose loads are issued together

// One thread per atom.  Candidate atoms come from the 27 (or fewer, for grids with fewer
// than 3 cells along a periodic axis) neighbouring cells; accepted indices are kept
// sorted in the thread's LDS row by insertion, then written out coalesced.
__global__ void __launch_bounds__(kNbThreads) k_build(const double* __restrict__ pos, int n, Grid g,
                                                      const int* __restrict__ cell_start,
                                                      const int* __restrict__ cell_atoms, double rl2,
                                                      int max_nb, int* __restrict__ count,
                                                      int* __restrict__ idx, int* __restrict__ flags) {
  // the thread's row, max_nb entries in LDS (dynamic size); entries beyond max_nb are
  // only counted, so the caller learns the length it needs
  extern __shared__ int row_lds[];
  const int t = threadIdx.x;
  auto row = [&](int k) -> int& { return row_lds[k * kNbThreads + t]; };
  const int i = xcd_block(blockIdx.x, gridDim.x) * kNbThreads + t;
  const bool valid = i < n;
  int cnt = 0;
  if (valid) {
    const double xi = pos[i], yi = pos[(size_t)n + i], zi = pos[2 * (size_t)n + i];
    const double Lx = g.L[0], Ly = g.L[1], Lz = g.L[2];
    const double hx = 0.5 * Lx, hy = 0.5 * Ly, hz = 0.5 * Lz;
    int ci[3];
    ci[0] = cell_coord(xi, g.lo[0], g.inv_cell[0], g.nc[0]);
    ci[1] = cell_coord(yi, g.lo[1], g.inv_cell[1], g.nc[1]);
    ci[2] = cell_coord(zi, g.lo[2], g.inv_cell[2], g.nc[2]);
    // offsets per axis: -1, 0, +1 when distinct, fewer cells otherwise
    int olo[3], ohi[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (g.per[d]) {
        olo[d] = g.nc[d] >= 3 ? -1 : 0;
        ohi[d] = g.nc[d] >= 3 ? 1 : g.nc[d] - 1;
      } else {
        olo[d] = ci[d] > 0 ? -1 : 0;
        ohi[d] = ci[d] < g.nc[d] - 1 ? 1 : 0;
      }
    }
    for (int oz = olo[2]; oz <= ohi[2]; ++oz) {
      int cz = ci[2] + oz;
      if (g.per[2]) cz = (cz + g.nc[2]) % g.nc[2];
      for (int oy = olo[1]; oy <= ohi[1]; ++oy) {
        int cy = ci[1] + oy;
        if (g.per[1]) cy = (cy + g.nc[1]) % g.nc[1];
        for (int ox = olo[0]; ox <= ohi[0]; ++ox) {
          int cx = ci[0] + ox;
          if (g.per[0]) cx = (cx + g.nc[0]) % g.nc[0];
          const int c = cx + g.nc[0] * (cy + g.nc[1] * cz);
          const int b = cell_start[c], e = cell_start[c + 1];
          // candidates in batches: the batch's indices and positions are loaded first so
          // that their memory accesses are in flight together
          for (int a0 = b; a0 < e; a0 += kBatch) {
            int jb[kBatch];
            double px[kBatch], py[kBatch], pz[kBatch];
#pragma unroll
            for (int q = 0; q < kBatch; ++q) jb[q] = a0 + q < e ? cell_atoms[a0 + q] : i;
#pragma unroll
            for (int q = 0; q < kBatch; ++q) {
              px[q] = pos[jb[q]];
              py[q] = pos[(size_t)n + jb[q]];
              pz[q] = pos[2 * (size_t)n + jb[q]];
            }
#pragma unroll
            for (int q = 0; q < kBatch; ++q) {
              const int j = jb[q];
              const double dx = min_image(px[q] - xi, Lx, hx, g.per[0]);
              const double dy = min_image(py[q] - yi, Ly, hy, g.per[1]);
              const double dz = min_image(pz[q] - zi, Lz, hz, g.per[2]);
              const double r2 = sq_dist_exact(dx, dy, dz);
              if (j != i && r2 < rl2) {
                if (cnt < max_nb) {
                  int k = cnt;
                  while (k > 0 && row(k - 1) > j) {
                    row(k) = row(k - 1);
                    --k;
                  }
                  row(k) = j;
                }
                ++cnt;
              }
            }
          }
        }
      }
    }
  }
  // the longest row and the capacity flag: one atomic per wave (the block is one wave)
  const int longest = wave_max(cnt);
  if (t == 0) {
    if (longest > max_nb) atomicOr(&flags[0], 4);
    atomicMax(&flags[1], longest);
  }
  if (!valid) return;
  count[i] = cnt;
  const int m = cnt < max_nb ? cnt : max_nb;
  for (int k = 0; k < m; ++k) idx[(size_t)k * n + i] = row(k);
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
  k_build<<<blocks_for(n, kNbThreads), kNbThreads, sizeof(int) * kNbThreads * nl->max_nb, ctx->stream>>>(
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
