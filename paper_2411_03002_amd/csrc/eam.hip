// Embedded-atom model: density/embedding pass and site-weighted force pass.
//
// Sec. III B eq. energy_eam with the closed-form synthetic functions or the paper's EAM2
// copper potential (Appendix E), chosen at compile time per launch; forces are the
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
  // EAM2 (Appendix E), in the order of apx_eam_params.eam2
  double E1, E2, delta, alpha1, alpha2, r01, r02, S[3], rs[3], a, beta1, beta2, r03, r04, xi0, xi2, q[4], Q1, Q2,
      f0;
};

// psi(x) = x^4/(1+x^4) for x < 0 and its derivative d psi/dx.
__device__ __forceinline__ void taper(double x, double& p, double& dp) {
  const double x2 = x * x;
  const double x4 = x2 * x2;
  const double den = rcp_nr(1.0 + x4);
  p = x4 * den;
  dp = 4.0 * x2 * x * den * den;
}

// EAM2 pair functions at r (tapered parts with the taper value ps and slope dps, dps
// already divided by h): pair potential Phi, density zeta and their derivatives.
__device__ __forceinline__ void eam2_pair(const EamDev& p, double r, double ps, double dps, double& phi,
                                          double& dphi, double& rho, double& drho, const double* etab) {
  const double t1 = exp_tab(-p.alpha1 * (r - p.r01), etab), t2 = exp_tab(-p.alpha2 * (r - p.r02), etab);
  const double m1 = t1 * t1 - 2.0 * t1, m2 = t2 * t2 - 2.0 * t2;
  const double dm1 = 2.0 * p.alpha1 * (t1 - t1 * t1), dm2 = 2.0 * p.alpha2 * (t2 - t2 * t2);
  const double core = p.E1 * m1 + p.E2 * m2 + p.delta;
  phi = core * ps;
  dphi = (p.E1 * dm1 + p.E2 * dm2) * ps + core * dps;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double d = p.rs[k] - r;
    if (d >= 0.0) {
      const double d2 = d * d;
      phi -= p.S[k] * d2 * d2;
      dphi += 4.0 * p.S[k] * d2 * d;
    }
  }
  const double x3 = r - p.r03;
  const double g = p.a * exp_tab(-p.beta1 * x3 * x3, etab);
  // exp(-x) is +0 in double precision for x above 745.2; the refit's second density
  // term (beta2 = 535.661 /A, r04 = -261.984 A) is always there, so it is skipped
  const double xe = p.beta2 * (r - p.r04);
  const double e = xe > 746.0 ? 0.0 : exp_tab(-xe, etab);
  rho = (g + e) * ps;
  drho = (-2.0 * p.beta1 * x3 * g - p.beta2 * e) * ps + (g + e) * dps;
}

// EAM2 embedding xi(x) + f0 and its slope.
__device__ __forceinline__ void eam2_embed(const EamDev& p, double x, double& F, double& Fp) {
  const double d = x - 1.0;
  const double d2 = d * d, d3 = d2 * d;
  if (x <= 1.0) {
    const double d4 = d2 * d2, d5 = d4 * d, d6 = d3 * d3;
    F = p.xi0 + 0.5 * p.xi2 * d2 + p.q[0] * d3 + p.q[1] * d4 + p.q[2] * d5 + p.q[3] * d6;
    Fp = p.xi2 * d + 3.0 * p.q[0] * d2 + 4.0 * p.q[1] * d3 + 5.0 * p.q[2] * d4 + 6.0 * p.q[3] * d5;
  } else {
    const double N = p.xi0 + 0.5 * p.xi2 * d2 + p.q[0] * d3 + p.Q1 * d2 * d2;
    const double Np = p.xi2 * d + 3.0 * p.q[0] * d2 + 4.0 * p.Q1 * d3;
    const double D = 1.0 + p.Q2 * d3;
    const double Dp = 3.0 * p.Q2 * d2;
    F = N / D;
    Fp = (Np * D - N * Dp) / (D * D);
  }
  F += p.f0;
}

// Neighbours are processed in batches of kBatch: the batch's indices and positions are
// loaded first so that their memory accesses are in flight together, then the pairs are
// summed in list order (the same order as one at a time).
constexpr int kBatch = 8;

template <int KIND>
__global__ void __launch_bounds__(256) k_eam_density(const double* __restrict__ pos, int n, BoxDev b, EamDev p,
                                                     const int* __restrict__ count, const int* __restrict__ idx,
                                                     int max_nb, const double* __restrict__ w,
                                                     double* __restrict__ e_site, double* __restrict__ rho_out,
                                                     double2* __restrict__ uf, const double* __restrict__ wl,
                                                     double2* __restrict__ duf) {
  __shared__ double etab[32];
  stage_exp_table(etab);
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
        const double r = r2 * rsq_nr(r2);
        double ps, dps;
        taper((r - p.rc) * p.inv_h, ps, dps);
        if constexpr (KIND == APX_EAM_CLOSED) {
          rho += exp_tab(-p.beta * (r - p.r0), etab) * ps;
          pair += exp_tab(-p.alpha * (r - p.r0), etab) * ps;
        } else {
          double phi, dphi, rr, drr;
          eam2_pair(p, r, ps, dps * p.inv_h, phi, dphi, rr, drr, etab);
          rho += rr;
          pair += phi;
        }
      }
    }
  }
  double F, Fp;
  if constexpr (KIND == APX_EAM_CLOSED) {
    const double sq = sqrt(rho);
    F = rho > 0.0 ? -sq : 0.0;
    Fp = rho > 0.0 ? -0.5 / sq : 0.0;
    e_site[i] = F + 0.5 * p.A * pair;
  } else {
    eam2_embed(p, rho, F, Fp);
    e_site[i] = F + 0.5 * pair;
  }
  if (rho_out) rho_out[i] = rho;
  const double u = w ? 1.0 - w[i] : 1.0;
  uf[i] = make_double2(u, u * Fp);
  if (duf) {
    // weights of a second set wl: the EAM weight difference (1 - wl) - (1 - w) = w - wl
    const double du = w[i] - wl[i];
    duf[i] = make_double2(du, du * Fp);
  }
}

// SKIPZERO: pairs whose two weights are both 0 contribute exactly 0 and are not evaluated
// (the pass over weight differences, which are 0 almost everywhere).
template <int KIND, bool SKIPZERO = false>
__global__ void __launch_bounds__(256) k_eam_force(const double* __restrict__ pos, int n, BoxDev b, EamDev p,
                                                   const int* __restrict__ count, const int* __restrict__ idx,
                                                   int max_nb, const double2* __restrict__ uf,
                                                   double* __restrict__ f) {
  __shared__ double etab[32];
  stage_exp_table(etab);
  const int i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double xi = pos[i], yi = pos[(size_t)n + i], zi = pos[2 * (size_t)n + i];
  const double2 ufs = uf[i];
  const double ui = ufs.x, ufi = ufs.y;
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
      const double2 v = uf[jb[q]];
      uj[q] = v.x;
      fj[q] = v.y;
    }
#pragma unroll
    for (int q = 0; q < kBatch; ++q) {
      const double dx = min_image(px[q] - xi, b.L[0], b.half[0], b.per[0]);
      const double dy = min_image(py[q] - yi, b.L[1], b.half[1], b.per[1]);
      const double dz = min_image(pz[q] - zi, b.L[2], b.half[2], b.per[2]);
      const double r2 = dx * dx + dy * dy + dz * dz;
      if (SKIPZERO && ui == 0.0 && uj[q] == 0.0) continue;
      if (k0 + q < cnt && r2 < p.rc2) {
        const double ir = rsq_nr(r2);
        const double r = r2 * ir;
        double ps, dps;
        taper((r - p.rc) * p.inv_h, ps, dps);
        dps *= p.inv_h;
        double drho, dphi;
        if constexpr (KIND == APX_EAM_CLOSED) {
          const double eb = exp_tab(-p.beta * (r - p.r0), etab);
          const double ea = exp_tab(-p.alpha * (r - p.r0), etab);
          drho = eb * (dps - p.beta * ps);
          dphi = p.A * ea * (dps - p.alpha * ps);
        } else {
          double phi, rr;
          eam2_pair(p, r, ps, dps, phi, dphi, rr, drho, etab);
        }
        const double s = 0.5 * (ui + uj[q]) * dphi + (ufi + fj[q]) * drho;
        const double sr = s * ir;
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
  if (p->kind != APX_EAM_CLOSED && p->kind != APX_EAM2) return fail(ctx, APX_EINVAL, "unknown EAM kind %d", p->kind);
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
  const double* e = p->eam2;
  d.E1 = e[0]; d.E2 = e[1]; d.delta = e[2]; d.alpha1 = e[3]; d.alpha2 = e[4]; d.r01 = e[5]; d.r02 = e[6];
  for (int k = 0; k < 3; ++k) {
    d.S[k] = e[7 + k];
    d.rs[k] = e[10 + k];
  }
  d.a = e[13]; d.beta1 = e[14]; d.beta2 = e[15]; d.r03 = e[16]; d.r04 = e[17]; d.xi0 = e[18]; d.xi2 = e[19];
  for (int k = 0; k < 4; ++k) d.q[k] = e[20 + k];
  d.Q1 = e[24]; d.Q2 = e[25]; d.f0 = e[26];
  return d;
}

// Launches both passes; uf is caller-provided scratch of 2n doubles (per atom u and u F').
// With wl and df (and duf, 2n doubles), a second force pass writes df = the fast-potential
// force with weights wl minus the one with weights w.
apx_status eam_launch(apx_ctx* ctx, const apx_atoms* atoms, const apx_nlist* nl, const apx_eam_params* p,
                      const double* w, double* e_site, double* rho, double* f, double* uf,
                      const double* wl = nullptr, double* df = nullptr, double* duf = nullptr) {
  const int n = (int)atoms->n;
  if (n == 0) return APX_OK;
  BoxDev b = make_box(atoms);
  EamDev d = eam_dev(p);
  double2* uf2 = reinterpret_cast<double2*>(uf);
  double2* duf2 = reinterpret_cast<double2*>(duf);
  {
  ProfScope ps(ctx, "eam.density");
  if (p->kind == APX_EAM2)
    k_eam_density<APX_EAM2><<<blocks_for(n, 256), 256, 0, ctx->stream>>>(atoms->pos, n, b, d, nl->count, nl->idx,
                                                                         nl->max_nb, w, e_site, rho, uf2, wl, duf2);
  else
    k_eam_density<APX_EAM_CLOSED><<<blocks_for(n, 256), 256, 0, ctx->stream>>>(
        atoms->pos, n, b, d, nl->count, nl->idx, nl->max_nb, w, e_site, rho, uf2, wl, duf2);
  APX_LAUNCH_CHECK(ctx);
  }
  ProfScope ps(ctx, "eam.force");
  if (p->kind == APX_EAM2)
    k_eam_force<APX_EAM2><<<blocks_for(n, 256), 256, 0, ctx->stream>>>(atoms->pos, n, b, d, nl->count, nl->idx,
                                                                       nl->max_nb, uf2, f);
  else
    k_eam_force<APX_EAM_CLOSED><<<blocks_for(n, 256), 256, 0, ctx->stream>>>(atoms->pos, n, b, d, nl->count,
                                                                             nl->idx, nl->max_nb, uf2, f);
  APX_LAUNCH_CHECK(ctx);
  if (df) {
    ProfScope pd(ctx, "eam.force_delta");
    if (p->kind == APX_EAM2)
      k_eam_force<APX_EAM2, true><<<blocks_for(n, 256), 256, 0, ctx->stream>>>(atoms->pos, n, b, d, nl->count,
                                                                               nl->idx, nl->max_nb, duf2, df);
    else
      k_eam_force<APX_EAM_CLOSED, true><<<blocks_for(n, 256), 256, 0, ctx->stream>>>(
          atoms->pos, n, b, d, nl->count, nl->idx, nl->max_nb, duf2, df);
    APX_LAUNCH_CHECK(ctx);
  }
  return APX_OK;
}

apx_status eam_forces_dual(apx_ctx* ctx, const apx_atoms* atoms, const apx_nlist* nl, const apx_eam_params* p,
                           const double* w, const double* wl, double* e_site, double* rho, double* f, double* df,
                           double* scratch4) {
  apx_status s = eam_check(ctx, atoms, nl, p);
  if (s != APX_OK) return s;
  if (!w || !wl || !df || !scratch4) return fail(ctx, APX_EINVAL, "dual EAM pass needs both weight sets");
  const size_t n = (size_t)atoms->n;
  return eam_launch(ctx, atoms, nl, p, w, e_site, rho, f, scratch4, wl, df, scratch4 + 2 * n);
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
  return eam_launch(ctx, atoms, nl, p, w, e_site, rho, f, ctx->dtmp.as<double>());
}
