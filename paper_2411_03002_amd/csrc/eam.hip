// Embedded-atom model: density/embedding pass and site-weighted force pass.
//
// Sec. III B eq. energy_eam with the closed-form synthetic functions; forces are the
// fast-potential part of Appendix C eq. F_i_d:
//   F_i = -d/dx_i sum_k u_k E_k,  u = 1 - w
//       = sum_j [ 1/2 (u_i + u_j) phi'(r_ij) + (u_i F'_i + u_j F'_j) rho'(r_ij) ] r_ij / r_ij
// with r_ij = x_j - x_i.  Both passes gather over the full neighbour list (one thread per
// atom, neighbour-major rows read coalesced), so no atomics are needed.
#include <cmath>

#include "common.h"
#include "device_util.h"

namespace apx {

struct EamDev {
  double A, alpha, beta, r0, rc, inv_h, rc2;
};

// psi(x) = x^4/(1+x^4) for x < 0 and its derivative d psi/dx.
__device__ __forceinline__ void taper(double x, double& p, double& dp) {
  const double x2 = x * x;
  const double x4 = x2 * x2;
  const double den = 1.0 / (1.0 + x4);
  p = x4 * den;
  dp = 4.0 * x2 * x * den * den;
}

// Neighbours are processed in batches of kBatch: the batch's indices and positions are
// loaded first so that their memory accesses are in flight together, then the pairs are
// summed in list order (the same order as one at a time).
constexpr int kBatch = 8;

__global__ void __launch_bounds__(256) k_eam_density(const double* __restrict__ pos, int n, BoxDev b, EamDev p,
                                                     const int* __restrict__ count, const int* __restrict__ idx,
                                                     int max_nb, const double* __restrict__ w,
                                                     double* __restrict__ e_site, double* __restrict__ rho_out,
                                                     double* __restrict__ ufp, double* __restrict__ u_out) {
  const int i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double xi = pos[i], yi = pos[(size_t)n + i], zi = pos[2 * (size_t)n + i];
  int cnt = count[i];
  if (cnt > max_nb) cnt = max_nb;
  double rho = 0.0, pair = 0.0;
  for (int k0 = 0; k0 < cnt; k0 += kBatch) {
    int jb[kBatch];
    double px[kBatch], py[kBatch], pz[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) jb[u] = k0 + u < cnt ? idx[(size_t)(k0 + u) * n + i] : i;
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      px[u] = pos[jb[u]];
      py[u] = pos[(size_t)n + jb[u]];
      pz[u] = pos[2 * (size_t)n + jb[u]];
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const double dx = min_image(px[u] - xi, b.L[0], b.half[0], b.per[0]);
      const double dy = min_image(py[u] - yi, b.L[1], b.half[1], b.per[1]);
      const double dz = min_image(pz[u] - zi, b.L[2], b.half[2], b.per[2]);
      const double r2 = dx * dx + dy * dy + dz * dz;
      if (k0 + u < cnt && r2 < p.rc2) {
        const double r = sqrt(r2);
        double ps, dps;
        taper((r - p.rc) * p.inv_h, ps, dps);
        rho += exp(-p.beta * (r - p.r0)) * ps;
        pair += exp(-p.alpha * (r - p.r0)) * ps;
      }
    }
  }
  const double sq = sqrt(rho);
  const double F = rho > 0.0 ? -sq : 0.0;
  const double Fp = rho > 0.0 ? -0.5 / sq : 0.0;
  e_site[i] = F + 0.5 * p.A * pair;
  if (rho_out) rho_out[i] = rho;
  const double u = w ? 1.0 - w[i] : 1.0;
  ufp[i] = u * Fp;
  u_out[i] = u;
}

__global__ void __launch_bounds__(256) k_eam_force(const double* __restrict__ pos, int n, BoxDev b, EamDev p,
                                                   const int* __restrict__ count, const int* __restrict__ idx,
                                                   int max_nb, const double* __restrict__ ufp,
                                                   const double* __restrict__ u, double* __restrict__ f) {
  const int i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double xi = pos[i], yi = pos[(size_t)n + i], zi = pos[2 * (size_t)n + i];
  const double ui = u[i], ufi = ufp[i];
  int cnt = count[i];
  if (cnt > max_nb) cnt = max_nb;
  double fx = 0.0, fy = 0.0, fz = 0.0;
  for (int k0 = 0; k0 < cnt; k0 += kBatch) {
    int jb[kBatch];
    double px[kBatch], py[kBatch], pz[kBatch], uj[kBatch], fj[kBatch];
#pragma unroll
    for (int q = 0; q < kBatch; ++q) jb[q] = k0 + q < cnt ? idx[(size_t)(k0 + q) * n + i] : i;
#pragma unroll
    for (int q = 0; q < kBatch; ++q) {
      px[q] = pos[jb[q]];
      py[q] = pos[(size_t)n + jb[q]];
      pz[q] = pos[2 * (size_t)n + jb[q]];
      uj[q] = u[jb[q]];
      fj[q] = ufp[jb[q]];
    }
#pragma unroll
    for (int q = 0; q < kBatch; ++q) {
      const double dx = min_image(px[q] - xi, b.L[0], b.half[0], b.per[0]);
      const double dy = min_image(py[q] - yi, b.L[1], b.half[1], b.per[1]);
      const double dz = min_image(pz[q] - zi, b.L[2], b.half[2], b.per[2]);
      const double r2 = dx * dx + dy * dy + dz * dz;
      if (k0 + q < cnt && r2 < p.rc2) {
        const double r = sqrt(r2);
        double ps, dps;
        taper((r - p.rc) * p.inv_h, ps, dps);
        dps *= p.inv_h;
        const double eb = exp(-p.beta * (r - p.r0));
        const double ea = exp(-p.alpha * (r - p.r0));
        const double drho = eb * (dps - p.beta * ps);
        const double dphi = p.A * ea * (dps - p.alpha * ps);
        const double s = 0.5 * (ui + uj[q]) * dphi + (ufi + fj[q]) * drho;
        const double sr = s / r;
        fx += sr * dx;
        fy += sr * dy;
        fz += sr * dz;
      }
    }
  }
  f[i] = fx;
  f[(size_t)n + i] = fy;
  f[2 * (size_t)n + i] = fz;
}

apx_status eam_check(apx_ctx* ctx, const apx_atoms* atoms, const apx_nlist* nl, const apx_eam_params* p) {
  apx_status s = check_atoms(ctx, atoms);
  if (s != APX_OK) return s;
  if (!nl || !p) return fail(ctx, APX_EINVAL, "nl and params are required");
  if (nl->n != atoms->n) return fail(ctx, APX_EINVAL, "nlist size mismatch");
  if (!(p->r_cut > 0.0) || p->r_cut > nl->r_list) return fail(ctx, APX_EINVAL, "EAM cutoff must be in (0, r_list]");
  if (!(p->h > 0.0)) return fail(ctx, APX_EINVAL, "EAM taper width must be positive");
  return APX_OK;
}

EamDev eam_dev(const apx_eam_params* p) {
  EamDev d;
  d.A = p->A;
  d.alpha = p->alpha;
  d.beta = p->beta;
  d.r0 = p->r0;
  d.rc = p->r_cut;
  d.inv_h = 1.0 / p->h;
  d.rc2 = p->r_cut * p->r_cut;
  return d;
}

// Launches both passes; ufp/u are caller-provided scratch of n doubles each.
apx_status eam_launch(apx_ctx* ctx, const apx_atoms* atoms, const apx_nlist* nl, const apx_eam_params* p,
                      const double* w, double* e_site, double* rho, double* f, double* ufp, double* u) {
  const int n = (int)atoms->n;
  if (n == 0) return APX_OK;
  BoxDev b = make_box(atoms);
  EamDev d = eam_dev(p);
  {
  ProfScope ps(ctx, "eam.density");
  k_eam_density<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(atoms->pos, n, b, d, nl->count, nl->idx, nl->max_nb,
                                                             w, e_site, rho, ufp, u);
  APX_LAUNCH_CHECK(ctx);
  }
  ProfScope ps(ctx, "eam.force");
  k_eam_force<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(atoms->pos, n, b, d, nl->count, nl->idx, nl->max_nb,
                                                           ufp, u, f);
  APX_LAUNCH_CHECK(ctx);
  return APX_OK;
}

}  // namespace apx

using namespace apx;

extern "C" apx_status apx_eam_forces(apx_ctx* ctx, const apx_atoms* atoms, const apx_nlist* nl,
                                     const apx_eam_params* p, const double* w, double* e_site, double* rho,
                                     double* f) {
  if (!ctx) return APX_EINVAL;
  apx_status s = eam_check(ctx, atoms, nl, p);
  if (s != APX_OK) return s;
  const int n = (int)atoms->n;
  if (n > 0 && (!e_site || !f)) return fail(ctx, APX_EINVAL, "e_site and f are required");
  APX_ALLOC(ctx, ctx->dtmp, sizeof(double) * 2 * (size_t)(n > 0 ? n : 1));
  double* ufp = ctx->dtmp.as<double>();
  return eam_launch(ctx, atoms, nl, p, w, e_site, rho, f, ufp, ufp + n);
}
