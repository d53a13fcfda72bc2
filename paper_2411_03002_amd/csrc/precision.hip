// Detection and switching: centro-symmetry parameter, initial weights, spreading,
// mask and the ascending list of atoms that need the precise potential.
#include <cmath>

#include "common.h"
#include "device_util.h"

namespace apx {

constexpr int kMaxM = 16;     // N + N_buffer
constexpr int kMaxHalf = 8;   // N / 2
constexpr int kMaxAvg = 4096; // samples per moving mean

struct PrecDev {
  int n_nn, m, half, kind;
  double csp_lo, width, rc2;
};

__device__ __forceinline__ double switch_w0(double c, const PrecDev& p) {
#pragma clang fp contract(off)
  double x = (c - p.csp_lo) / p.width;
  if (p.kind == 0) return x < 0.0 ? 0.0 : (x > 1.0 ? 1.0 : x);
  return 1.0 - fcut_exact(x);
}

constexpr int kBatch = 8;  // neighbours whose loads are issued together

// One thread per atom.  Keeps the M nearest candidates within r_cut sorted by
// (squared distance, index): the row is in ascending index, so a strict comparison
// keeps the smaller index first among equal distances.  The sorted slots carry the
// squared distance and the row position only; the M displacements are recomputed
// (identically) for the pair stage.  EXACT: M and HALF are the parameters' N + N_buffer
// and N/2; otherwise they are upper bounds and p.m, p.half apply.
template <int M, int HALF, bool EXACT>
__global__ void __launch_bounds__(256) k_csp(const double* __restrict__ pos, int n, Grid g,
                                             const uint8_t* __restrict__ frozen,
                                             const int* __restrict__ count, const int* __restrict__ idx,
                                             int max_nb, PrecDev p, const double* __restrict__ w0_extra,
                                             double* __restrict__ csp, double* __restrict__ w0,
                                             double* __restrict__ w) {
#pragma clang fp contract(off)
  const int i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (frozen && frozen[i]) {
    csp[i] = 0.0;
    w0[i] = 0.0;
    w[i] = 0.0;
    return;
  }
  const double xi = pos[i], yi = pos[(size_t)n + i], zi = pos[2 * (size_t)n + i];
  const double hx = 0.5 * g.L[0], hy = 0.5 * g.L[1], hz = 0.5 * g.L[2];
  const int m = EXACT ? M : p.m;
  double kr[M];
  int ks[M];
#pragma unroll
  for (int a = 0; a < M; ++a) {
    kr[a] = INFINITY;
    ks[a] = 0;
  }
  int found = 0;
  int cnt = count[i];
  if (cnt > max_nb) cnt = max_nb;
  for (int k0 = 0; k0 < cnt; k0 += kBatch) {
    int jb[kBatch];
    double px[kBatch], py[kBatch], pz[kBatch];
#pragma unroll
    for (int q = 0; q < kBatch; ++q) jb[q] = k0 + q < cnt ? idx[(size_t)(k0 + q) * n + i] : i;
#pragma unroll
    for (int q = 0; q < kBatch; ++q) {
      px[q] = pos[jb[q]];
      py[q] = pos[(size_t)n + jb[q]];
      pz[q] = pos[2 * (size_t)n + jb[q]];
    }
#pragma unroll
    for (int q = 0; q < kBatch; ++q) {
      const double dx = min_image(px[q] - xi, g.L[0], hx, g.per[0]);
      const double dy = min_image(py[q] - yi, g.L[1], hy, g.per[1]);
      const double dz = min_image(pz[q] - zi, g.L[2], hz, g.per[2]);
      const double r2 = sq_dist_exact(dx, dy, dz);
      if (!(k0 + q < cnt && r2 < p.rc2)) continue;
      ++found;
      if (!(r2 < kr[M - 1])) continue;
      // insertion into the sorted slots, unrolled so they stay in registers; once the new
      // entry has been placed every later slot shifts by one, which keeps equal distances
      // in arrival (ascending index) order
      double cr = r2;
      int cs = k0 + q;
      bool shifting = false;
#pragma unroll
      for (int a = 0; a < M; ++a) {
        const bool take = shifting || cr < kr[a];
        shifting = take;
        const double tr = kr[a];
        const int ts = ks[a];
        kr[a] = take ? cr : tr;
        ks[a] = take ? cs : ts;
        cr = take ? tr : cr;
        cs = take ? ts : cs;
      }
    }
  }
  double c;
  if (found < m) {
    c = INFINITY;
  } else {
    double kx[M], ky[M], kz[M];
#pragma unroll
    for (int a = 0; a < M; ++a) {
      if (a < m) {
        const int j = idx[(size_t)ks[a] * n + i];
        kx[a] = min_image(pos[j] - xi, g.L[0], hx, g.per[0]);
        ky[a] = min_image(pos[(size_t)n + j] - yi, g.L[1], hy, g.per[1]);
        kz[a] = min_image(pos[2 * (size_t)n + j] - zi, g.L[2], hz, g.per[2]);
      } else {
        kx[a] = ky[a] = kz[a] = 0.0;
      }
    }
    double best[HALF];
#pragma unroll
    for (int a = 0; a < HALF; ++a) best[a] = INFINITY;
#pragma unroll
    for (int a = 0; a < M; ++a) {
#pragma unroll
      for (int b = a + 1; b < M; ++b) {
        if (EXACT || b < m) {
          const double sx = kx[a] + kx[b], sy = ky[a] + ky[b], sz = kz[a] + kz[b];
          double v = sq_dist_exact(sx, sy, sz);
          bool shifting = false;
#pragma unroll
          for (int q = 0; q < HALF; ++q) {
            const bool take = shifting || v < best[q];
            shifting = take;
            const double t = best[q];
            best[q] = take ? v : t;
            v = take ? t : v;
          }
        }
      }
    }
    c = 0.0;
#pragma unroll
    for (int q = 0; q < HALF; ++q)
      if (EXACT || q < p.half) c = c + best[q];
  }
  csp[i] = c;
  double v0 = switch_w0(c, p);
  if (w0_extra) {
    const double e = w0_extra[i];
    v0 = e > v0 ? e : v0;
  }
  w0[i] = v0;
  w[i] = v0;
}

// w0 and w from a given CSP (the CSP pass skipped).
__global__ void k_switch(int n, const uint8_t* __restrict__ frozen, PrecDev p, const double* __restrict__ w0_extra,
                         const double* __restrict__ csp, double* __restrict__ w0, double* __restrict__ w) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (frozen && frozen[i]) {
    w0[i] = 0.0;
    w[i] = 0.0;
    return;
  }
  double v0 = switch_w0(csp[i], p);
  if (w0_extra) {
    const double e = w0_extra[i];
    v0 = e > v0 ? e : v0;
  }
  w0[i] = v0;
  w[i] = v0;
}

// Compacts the spreading sources (w0 > 0, not frozen) in any order.
__global__ void k_sources(int n, const double* __restrict__ w0, const uint8_t* __restrict__ frozen,
                          int* __restrict__ src, int* __restrict__ nsrc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (w0[i] > 0.0 && !(frozen && frozen[i])) src[atomicAdd(nsrc, 1)] = i;
}

struct SpreadDev {
  double r_lo, width, rh2;
  int reach[3];   // cells visited along each axis: offsets lo..lo+span-1
  int span[3];
};

// One wave per source: lanes sweep the cells of the stencil, each lane one cell at a
// time; every target within r_hi receives w0_j f_cut(...) by an atomic maximum on the
// IEEE bit pattern (all candidates are > 0, where the unsigned order equals the
// floating-point order), so the result does not depend on the visiting order.
__global__ void __launch_bounds__(256) k_spread(const double* __restrict__ pos, int n, Grid g, SpreadDev s,
                                                const int* __restrict__ src, int nsrc,
                                                const double* __restrict__ w0, const uint8_t* __restrict__ frozen,
                                                const int* __restrict__ cell_start, const int* __restrict__ cell_atoms,
                                                unsigned long long* __restrict__ wbits) {
#pragma clang fp contract(off)
  const int wid = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (wid >= nsrc) return;
  const int j = src[wid];
  const double xj = pos[j], yj = pos[(size_t)n + j], zj = pos[2 * (size_t)n + j];
  const double wj = w0[j];
  const double hx = 0.5 * g.L[0], hy = 0.5 * g.L[1], hz = 0.5 * g.L[2];
  const int cj0 = cell_coord(xj, g.lo[0], g.inv_cell[0], g.nc[0]);
  const int cj1 = cell_coord(yj, g.lo[1], g.inv_cell[1], g.nc[1]);
  const int cj2 = cell_coord(zj, g.lo[2], g.inv_cell[2], g.nc[2]);
  const int total = s.span[0] * s.span[1] * s.span[2];
  for (int q = lane; q < total; q += kWave) {
    const int ox = q % s.span[0] + s.reach[0];
    const int oy = (q / s.span[0]) % s.span[1] + s.reach[1];
    const int oz = q / (s.span[0] * s.span[1]) + s.reach[2];
    int cx = cj0 + ox, cy = cj1 + oy, cz = cj2 + oz;
    if (g.per[0]) cx = ((cx % g.nc[0]) + g.nc[0]) % g.nc[0];
    else if (cx < 0 || cx >= g.nc[0]) continue;
    if (g.per[1]) cy = ((cy % g.nc[1]) + g.nc[1]) % g.nc[1];
    else if (cy < 0 || cy >= g.nc[1]) continue;
    if (g.per[2]) cz = ((cz % g.nc[2]) + g.nc[2]) % g.nc[2];
    else if (cz < 0 || cz >= g.nc[2]) continue;
    const int c = cx + g.nc[0] * (cy + g.nc[1] * cz);
    const int b = cell_start[c], e = cell_start[c + 1];
    for (int a = b; a < e; ++a) {
      const int i = cell_atoms[a];
      if (frozen && frozen[i]) continue;
      const double dx = min_image(pos[i] - xj, g.L[0], hx, g.per[0]);
      const double dy = min_image(pos[(size_t)n + i] - yj, g.L[1], hy, g.per[1]);
      const double dz = min_image(pos[2 * (size_t)n + i] - zj, g.L[2], hz, g.per[2]);
      const double r2 = sq_dist_exact(dx, dy, dz);
      if (!(r2 < s.rh2)) continue;
      const double r = sqrt(r2);
      const double x = (r - s.r_lo) / s.width;
      const double v = wj * fcut_exact(x);
      if (v > 0.0) atomicMax(&wbits[i], (unsigned long long)__double_as_longlong(v));
    }
  }
}

// The additional detection weight combined with the spread weight (no spreading of its
// own): w = max(w, w0_extra), frozen atoms keep 0.
__global__ void k_extra_local(int n, const uint8_t* __restrict__ frozen, const double* __restrict__ extra,
                              double* __restrict__ w) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || (frozen && frozen[i])) return;
  const double e = extra[i];
  if (e > w[i]) w[i] = e;
}

__global__ void k_mask(int n, const double* __restrict__ w, uint8_t* __restrict__ mask, int* __restrict__ flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int m = w[i] > 0.0 ? 1 : 0;
  mask[i] = (uint8_t)m;
  flag[i] = m;
}

__global__ void k_compact(int n, const int* __restrict__ flag, const int* __restrict__ pos_, int* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (flag[i]) out[pos_[i]] = i;
}

// Time-averaged switching.  A ring of n_avg samples per atom, slot-major ([slot][n], so
// each slot is read coalesced); the sample of this call goes to `slot` and the mean adds
// the m newest samples newest first, starting from 0.0, then divides by m.
__device__ __forceinline__ double ring_mean(const double* __restrict__ ring, size_t n, int i, int slot, int n_avg,
                                            int m, double newest) {
#pragma clang fp contract(off)
  double acc = 0.0;
  acc = acc + newest;
  int s = slot;
  for (int j = 1; j < m; ++j) {
    s = s == 0 ? n_avg - 1 : s - 1;
    acc = acc + ring[(size_t)s * n + i];
  }
  return acc / (double)m;
}

// eq. csp_2_i then eq. lambda_1_i: averages the CSP samples, pushes the new one, switches;
// w0 seeds the spreading target w.  past: the mean holds the m samples before this call
// (read before the new sample overwrites the oldest slot; the new sample alone when there
// is none); current: the new sample and the m - 1 before it.
__global__ void k_avg_csp(int n, const uint8_t* __restrict__ frozen, PrecDev p, const double* __restrict__ w0_extra,
                          const double* __restrict__ csp, double* __restrict__ ring, int slot, int n_avg, int m,
                          int past, double* __restrict__ csp_avg, double* __restrict__ w0, double* __restrict__ w) {
#pragma clang fp contract(off)
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double c = csp[i];
  double a;
  if (past && m > 0) {
    double acc = 0.0;
    int s = slot;
    for (int j = 0; j < m; ++j) {
      s = s == 0 ? n_avg - 1 : s - 1;
      acc = acc + ring[(size_t)s * n + i];
    }
    a = acc / (double)m;
    ring[(size_t)slot * n + i] = c;
  } else {
    ring[(size_t)slot * n + i] = c;
    a = ring_mean(ring, (size_t)n, i, slot, n_avg, past ? 1 : m, c);
  }
  csp_avg[i] = a;
  if (frozen && frozen[i]) {
    w0[i] = 0.0;
    w[i] = 0.0;
    return;
  }
  double v0 = switch_w0(a, p);
  if (w0_extra) {
    const double e = w0_extra[i];
    v0 = e > v0 ? e : v0;
  }
  w0[i] = v0;
  w[i] = v0;
}

// eq. lambda_3_i then eq. lambda_4_i: pushes the spread weight, averages, applies the
// minimum step against the previous filtered weight (in w), writes the mask.
__global__ void k_avg_w(int n, const double* __restrict__ w_min, double* __restrict__ ring, int slot, int n_avg, int m,
                        int first, double dw_min, double* __restrict__ w_avg, double* __restrict__ w,
                        uint8_t* __restrict__ mask, int* __restrict__ flag) {
#pragma clang fp contract(off)
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = w_min[i];
  ring[(size_t)slot * n + i] = v;
  const double a = ring_mean(ring, (size_t)n, i, slot, n_avg, m, v);
  if (w_avg) w_avg[i] = a;
  double out = a;
  if (!first) {
    const double prev = w[i];
    const bool take = fabs(a - prev) >= dw_min || a == 0.0 || a == 1.0;
    out = take ? a : prev;
  }
  w[i] = out;
  const int k = out > 0.0 ? 1 : 0;
  mask[i] = (uint8_t)k;
  flag[i] = k;
}

}  // namespace apx

using namespace apx;

// Spreading stencil: a cell edge no smaller than r_hi/3 (and the list cutoff), so that
// three cells on each side cover r_hi; axes with fewer cells are visited once each.
static void spread_stencil(const Grid& g, double r_hi, SpreadDev& s) {
  for (int d = 0; d < 3; ++d) {
    const double cell = g.L[d] / g.nc[d];
    int reach = (int)std::ceil(r_hi / cell);
    if (2 * reach + 1 >= g.nc[d] && g.per[d]) {
      s.reach[d] = -(g.nc[d] / 2);
      s.span[d] = g.nc[d];
    } else {
      s.reach[d] = -reach;
      s.span[d] = 2 * reach + 1;
    }
  }
}

namespace {

// The averaging stage of a call: ring slot of this sample, samples in the means, and
// the buffers (all device, length n or [n_avg][n]).
struct AvgArgs {
  int n_avg, slot, m, first;
  int past, m_csp;  // window of the CSP mean: past samples only (m_csp of them) or current
  double dw_min;
  double *csp_ring, *w_ring, *csp_avg, *w_min, *w_avg;
};

apx_status precision_impl(apx_ctx* ctx, const apx_atoms* atoms, const apx_nlist* nl, const apx_prec_params* p,
                          const double* w0_extra, double* csp, double* w0, double* w, uint8_t* mask,
                          int32_t* active, int64_t* n_active, const AvgArgs* avg) {
  apx_status s = check_atoms(ctx, atoms);
  if (s != APX_OK) return s;
  if (!nl || !p || !n_active) return fail(ctx, APX_EINVAL, "nl, params and n_active are required");
  if (nl->n != atoms->n) return fail(ctx, APX_EINVAL, "nlist size mismatch");
  const int n = (int)atoms->n;
  if (n > 0 && (!csp || !w0 || !w || !mask || !active)) return fail(ctx, APX_EINVAL, "output arrays are NULL");
  if (p->n_nn < 2 || (p->n_nn & 1) || p->n_buffer < 0 || p->n_nn + p->n_buffer > kMaxM)
    return fail(ctx, APX_EINVAL, "n_nn must be even and n_nn + n_buffer <= %d", kMaxM);
  if (!(p->csp_hi > p->csp_lo)) return fail(ctx, APX_EINVAL, "csp_hi must exceed csp_lo");
  if (p->switch_kind != 0 && p->switch_kind != 1) return fail(ctx, APX_EINVAL, "switch_kind must be 0 or 1");
  if (!(p->r_cut > 0.0) || p->r_cut > nl->r_list) return fail(ctx, APX_EINVAL, "r_cut must be in (0, r_list]");
  if (p->r_hi > 0.0 && !(p->r_hi > p->r_lo)) return fail(ctx, APX_EINVAL, "r_hi must exceed r_lo");
  *n_active = 0;
  if (n == 0) return APX_OK;
  Grid g = make_grid(atoms, nl->r_list);
  PrecDev pd;
  pd.n_nn = p->n_nn;
  pd.m = p->n_nn + p->n_buffer;
  pd.half = p->n_nn / 2;
  pd.kind = p->switch_kind;
  pd.csp_lo = p->csp_lo;
  pd.width = p->csp_hi - p->csp_lo;
  pd.rc2 = p->r_cut * p->r_cut;
  // spreading target: w itself, or the instantaneous weight when averaging
  double* ws = avg ? avg->w_min : w;
  // the extra detection weight enters before spreading, or after it (APX_PREC_EXTRA_LOCAL)
  const bool extra_local = (p->flags & APX_PREC_EXTRA_LOCAL) != 0;
  const double* extra_pre = extra_local ? nullptr : w0_extra;
  if (!(p->flags & APX_PREC_CSP_GIVEN)) {
  ProfScope ps(ctx, "prec.csp");
  if (pd.m == 12 && pd.half == 6)
    k_csp<12, 6, true><<<blocks_for(n, 256), 256, 0, ctx->stream>>>(
        atoms->pos, n, g, atoms->frozen, nl->count, nl->idx, nl->max_nb, pd, avg ? nullptr : extra_pre, csp, w0, ws);
  else
    k_csp<kMaxM, kMaxHalf, false><<<blocks_for(n, 256), 256, 0, ctx->stream>>>(
        atoms->pos, n, g, atoms->frozen, nl->count, nl->idx, nl->max_nb, pd, avg ? nullptr : extra_pre, csp, w0, ws);
  APX_LAUNCH_CHECK(ctx);
  } else if (!avg) {
    ProfScope ps(ctx, "prec.switch");
    k_switch<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(n, atoms->frozen, pd, extra_pre, csp, w0, w);
    APX_LAUNCH_CHECK(ctx);
  }
  if (avg) {
    ProfScope ps(ctx, "prec.avg_csp");
    k_avg_csp<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(n, atoms->frozen, pd, extra_pre, csp, avg->csp_ring,
                                                           avg->slot, avg->n_avg, avg->past ? avg->m_csp : avg->m,
                                                           avg->past, avg->csp_avg, w0, ws);
    APX_LAUNCH_CHECK(ctx);
  }
  if (p->r_hi > 0.0) {
    APX_ALLOC(ctx, ctx->itmp, sizeof(int) * (size_t)n);
    APX_ALLOC(ctx, ctx->itmp2, sizeof(int) * 4);
    APX_HIP(ctx, hipMemsetAsync(ctx->itmp2.p, 0, sizeof(int), ctx->stream));
    k_sources<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(n, w0, atoms->frozen, ctx->itmp.as<int>(),
                                                          ctx->itmp2.as<int>());
    APX_LAUNCH_CHECK(ctx);
    int nsrc = 0;
    s = read_ints(ctx, ctx->itmp2.as<int>(), &nsrc, 1);
    if (s != APX_OK) return s;
    if (nsrc > 0) {
      Grid gs = make_grid(atoms, p->r_hi / 3.0);
      s = bin_atoms(ctx, atoms, gs);
      if (s != APX_OK) return s;
      SpreadDev sd;
      sd.r_lo = p->r_lo;
      sd.width = p->r_hi - p->r_lo;
      sd.rh2 = p->r_hi * p->r_hi;
      spread_stencil(gs, p->r_hi, sd);
      const long long threads = (long long)nsrc * kWave;
      ProfScope ps(ctx, "prec.spread");
      k_spread<<<blocks_for(threads, 256), 256, 0, ctx->stream>>>(
          atoms->pos, n, gs, sd, ctx->itmp.as<int>(), nsrc, w0, atoms->frozen, ctx->cell_start.as<int>(),
          ctx->cell_atoms.as<int>(), reinterpret_cast<unsigned long long*>(ws));
      APX_LAUNCH_CHECK(ctx);
    }
  }
  if (extra_local && w0_extra) {
    k_extra_local<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(n, atoms->frozen, w0_extra, ws);
    APX_LAUNCH_CHECK(ctx);
  }
  APX_ALLOC(ctx, ctx->itmp, sizeof(int) * (size_t)n);
  APX_ALLOC(ctx, ctx->itmp2, sizeof(int) * (size_t)(n + 1));
  if (avg) {
    ProfScope ps(ctx, "prec.avg_w");
    k_avg_w<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(n, ws, avg->w_ring, avg->slot, avg->n_avg, avg->m,
                                                         avg->first, avg->dw_min, avg->w_avg, w, mask,
                                                         ctx->itmp.as<int>());
    APX_LAUNCH_CHECK(ctx);
  }
  ProfScope ps(ctx, "prec.compact");
  if (!avg) {
    k_mask<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(n, w, mask, ctx->itmp.as<int>());
    APX_LAUNCH_CHECK(ctx);
  }
  s = scan_exclusive(ctx, ctx->itmp.as<int>(), n, ctx->itmp2.as<int>());
  if (s != APX_OK) return s;
  k_compact<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(n, ctx->itmp.as<int>(), ctx->itmp2.as<int>(), active);
  APX_LAUNCH_CHECK(ctx);
  int na = 0;
  s = read_ints(ctx, ctx->itmp2.as<int>() + n, &na, 1);
  if (s != APX_OK) return s;
  *n_active = na;
  return APX_OK;
}

}  // namespace

extern "C" apx_status apx_compute_precision(apx_ctx* ctx, const apx_atoms* atoms, const apx_nlist* nl,
                                            const apx_prec_params* p, const double* w0_extra, double* csp,
                                            double* w0, double* w, uint8_t* mask, int32_t* active,
                                            int64_t* n_active) {
  return precision_impl(ctx, atoms, nl, p, w0_extra, csp, w0, w, mask, active, n_active, nullptr);
}

extern "C" apx_status apx_compute_precision_avg(apx_ctx* ctx, const apx_atoms* atoms, const apx_nlist* nl,
                                                const apx_prec_params* p, apx_avg_state* st,
                                                const double* w0_extra, double* csp, double* csp_avg, double* w0,
                                                double* w_min, double* w_avg, double* w, uint8_t* mask,
                                                int32_t* active, int64_t* n_active) {
  if (!ctx) return APX_EINVAL;
  if (!st || !atoms) return fail(ctx, APX_EINVAL, "atoms and the averaging state are required");
  if (st->n_avg < 1 || st->n_avg > kMaxAvg) return fail(ctx, APX_EINVAL, "n_avg must be in 1..%d", kMaxAvg);
  if (st->samples < 0) return fail(ctx, APX_EINVAL, "samples must be >= 0");
  if (st->window != APX_WINDOW_PAST && st->window != APX_WINDOW_CURRENT)
    return fail(ctx, APX_EINVAL, "window must be APX_WINDOW_PAST or APX_WINDOW_CURRENT");
  if (!(st->dw_min >= 0.0)) return fail(ctx, APX_EINVAL, "dw_min must be >= 0");
  if (atoms->n > 0 && (!st->csp_ring || !st->w_ring || !csp_avg || !w_min))
    return fail(ctx, APX_EINVAL, "rings, csp_avg and w_min are required");
  AvgArgs a;
  a.n_avg = st->n_avg;
  a.slot = (int)(st->samples % st->n_avg);
  a.m = st->samples + 1 < st->n_avg ? (int)st->samples + 1 : st->n_avg;
  a.first = st->samples == 0 ? 1 : 0;
  a.past = st->window == APX_WINDOW_PAST ? 1 : 0;
  a.m_csp = st->samples < st->n_avg ? (int)st->samples : st->n_avg;  // samples before this one
  a.dw_min = st->dw_min;
  a.csp_ring = st->csp_ring;
  a.w_ring = st->w_ring;
  a.csp_avg = csp_avg;
  a.w_min = w_min;
  a.w_avg = w_avg;
  apx_status s = precision_impl(ctx, atoms, nl, p, w0_extra, csp, w0, w, mask, active, n_active, &a);
  if (s == APX_OK) st->samples += 1;
  return s;
}
