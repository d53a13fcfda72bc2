// Velocity-Verlet integration with the switching-weight update (Sec. II C eq. vv) on one
// GPU.  Per step: half kick + drift (+ wrap, displacement check), neighbour rebuild when
// an atom moved more than skin/2 since the last build, the weight update every k steps
// (before the forces, or after them with time-averaged weights over past samples: the
// force routine's order of Appendix G), EAM for every atom, ACE for the atoms with w > 0,
// blend, indenter, half kick, and the local thermostat when the weights changed
// (Sec. II C 2).
#include <cmath>
#include <cstring>

#include "ace_model.h"
#include "common.h"
#include "device_util.h"

namespace apx {

constexpr double kAccel = 9648.5332;  // (eV/A)/amu in A/ps^2

// Half kick, drift and periodic wrap of the mobile atoms; the largest squared
// displacement since the last neighbour build is reduced per block and combined with an
// atomic maximum on its (non-negative) bit pattern.
__global__ void __launch_bounds__(256) k_kick_drift(long long n, double* __restrict__ pos, double* __restrict__ vel,
                                                    const double* __restrict__ f, const uint8_t* __restrict__ frozen,
                                                    double ck, double dt, BoxDev b, const double* __restrict__ lo,
                                                    const double* __restrict__ xref,
                                                    unsigned long long* __restrict__ maxd2) {
  __shared__ double sh[4];
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double d2 = 0.0;
  if (i < n && !(frozen && frozen[i])) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const long long k = d * n + i;
      const double v = vel[k] + ck * f[k];
      vel[k] = v;
      double x = pos[k] + dt * v;
      if (b.per[d]) {
        if (x >= lo[d] + b.L[d]) x -= b.L[d];
        else if (x < lo[d]) x += b.L[d];
        if (x >= lo[d] + b.L[d] || x < lo[d]) x = lo[d];  // rounding guard
      }
      pos[k] = x;
      const double dd = min_image(x - xref[k], b.L[d], b.half[d], b.per[d]);
      d2 += dd * dd;
    }
  }
  d2 = wave_max(d2);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = d2;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = sh[0];
    for (int k = 1; k < 4; ++k) m = sh[k] > m ? sh[k] : m;
    if (m > 0.0) sparse_atomic_max(maxd2, (unsigned long long)__double_as_longlong(m));
  }
}

__global__ void k_kick(long long n, double* __restrict__ vel, const double* __restrict__ f,
                       const uint8_t* __restrict__ frozen, double ck) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (frozen && frozen[i]) return;
  vel[i] += ck * f[i];
  vel[n + i] += ck * f[n + i];
  vel[2 * n + i] += ck * f[2 * n + i];
}

__global__ void k_indenter(long long n, const double* __restrict__ pos, double* __restrict__ f, BoxDev b,
                           double cx, double cy, double cz, double R, double K, double* __restrict__ energy) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double e = 0.0;
  if (i < n) {
    const double dx = min_image(pos[i] - cx, b.L[0], b.half[0], b.per[0]);
    const double dy = min_image(pos[n + i] - cy, b.L[1], b.half[1], b.per[1]);
    const double dz = min_image(pos[2 * n + i] - cz, b.L[2], b.half[2], b.per[2]);
    const double d = sqrt(dx * dx + dy * dy + dz * dz);
    if (d < R && d > 0.0) {
      const double pen = R - d;
      const double s = K * pen * pen / d;
      f[i] += s * dx;
      f[n + i] += s * dy;
      f[2 * n + i] += s * dz;
      e = K / 3.0 * pen * pen * pen;
    }
  }
  e = wave_sum(e);
  if ((threadIdx.x & 63) == 0 && e != 0.0) atomicAdd(energy, e);
}

__global__ void k_kinetic(long long n, const double* __restrict__ vel, const uint8_t* __restrict__ frozen,
                          double half_m, double* __restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double e = 0.0;
  if (i < n && !(frozen && frozen[i])) {
    const double vx = vel[i], vy = vel[n + i], vz = vel[2 * n + i];
    e = half_m * (vx * vx + vy * vy + vz * vz);
  }
  e = wave_sum(e);
  if ((threadIdx.x & 63) == 0 && e != 0.0) atomicAdd(out, e);
}

__global__ void k_fill_d(long long n, double* __restrict__ p, double v) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_iota(int n, int* __restrict__ p) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = i;
}

__global__ void k_copy_d(long long n, const double* __restrict__ a, double* __restrict__ b) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

// dw = w_c - w_d (the ACE weight of the force difference F^c - F^d) and the flag of the
// atoms ACE is evaluated for when both weight sets are needed (w_c > 0 or w_d > 0).
__global__ void k_union(int n, const double* __restrict__ wd, const double* __restrict__ wc, double* __restrict__ dw,
                        int* __restrict__ flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double a = wd[i], c = wc[i];
  dw[i] = c - a;
  flag[i] = (a > 0.0 || c > 0.0) ? 1 : 0;
}

__global__ void k_compact_flags(int n, const int* __restrict__ flag, const int* __restrict__ pos_,
                                int* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && flag[i]) out[pos_[i]] = i;
}

__global__ void k_add_into(long long n, double* __restrict__ a, const double* __restrict__ b) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] += b[i];
}

}  // namespace apx

using namespace apx;

struct apx_md {
  apx_ctx* ctx = nullptr;
  apx_md_params p{};
  apx_eam_params eam{};
  apx_prec_params prec{};
  const apx_ace_model* ace = nullptr;
  apx_atoms atoms{};
  int n = 0;
  int max_nb = 0;
  double r_list = 0.0;
  long long step = 0;
  long long n_active = 0;
  bool initialized = false;
  DevBuf nl_count, nl_idx, xref, lo_dev;
  DevBuf csp, w0, mask, active;
  DevBuf e_eam, e_ace, e_site, f_eam, f_ace, rho;
  DevBuf scal;  // [0] e_pot, [1] e_kin, [2] e_ind, [3] max displacement^2 bits
  apx_mlp* mlp = nullptr;  // learned criterion (optional)
  double tau_lo = 0.0, tau_hi = 0.0;
  DevBuf feat, pred, w0x;
  DevBuf csp_ring, w_ring, csp_avg, w_min;  // time-averaged weights (avg_samples > 0)
  long long avg_taken = 0;                  // samples in the rings since apx_md_init
  DevBuf wtmp;                              // learned route: the centro-symmetry pass's weights
  // local thermostat: weights of the last force evaluation, their difference, the force
  // differences, energy errors, EAM scratch, the union of active atoms
  DevBuf w_last, dw, df, df_ace, dE, eam4, uactive;
  bool w_dirty = false;        // w differs from the weights of the last force evaluation
  long long ace_count = 0;     // atoms ACE was evaluated for by the last force evaluation
  long long thermo_corrected = 0, thermo_failed = 0;
  hipEvent_t ev[6] = {};
  double t_acc[5] = {0, 0, 0, 0, 0};
};

namespace {

apx_status md_nlist(apx_md* md, apx_nlist& nl) {
  nl.n = md->n;
  nl.max_nb = md->max_nb;
  nl.count = md->nl_count.as<int>();
  nl.idx = md->nl_idx.as<int>();
  nl.r_list = md->r_list;
  return APX_OK;
}

apx_status md_rebuild(apx_md* md, const double* pos) {
  apx_ctx* ctx = md->ctx;
  md->atoms.pos = pos;
  for (int attempt = 0; attempt < 2; ++attempt) {
    apx_nlist nl;
    md_nlist(md, nl);
    int needed = 0;
    apx_status s = apx_build_neighbors(ctx, &md->atoms, md->r_list, &nl, &needed);
    if (s == APX_ECAPACITY && attempt == 0 && needed <= 128) {
      int grown = needed + 8 > 128 ? 128 : needed + 8;
      md->max_nb = grown;
      APX_ALLOC(ctx, md->nl_idx, sizeof(int) * (size_t)grown * md->n);
      continue;
    }
    if (s != APX_OK) return s;
    break;
  }
  const long long m3 = 3LL * md->n;
  k_copy_d<<<blocks_for(m3, 256), 256, 0, ctx->stream>>>(m3, pos, md->xref.as<double>());
  APX_LAUNCH_CHECK(ctx);
  return APX_OK;
}

// The criterion's weights from the given parameters: instantaneous, or one sample of the
// time-averaged pipeline (w holds the previous filtered weights).
apx_status md_precision(apx_md* md, const apx_nlist& nl, const apx_prec_params& p, const double* w0x, double* w,
                        int64_t* na) {
  apx_ctx* ctx = md->ctx;
  if (md->p.avg_samples <= 0)
    return apx_compute_precision(ctx, &md->atoms, &nl, &p, w0x, md->csp.as<double>(), md->w0.as<double>(), w,
                                 md->mask.as<uint8_t>(), md->active.as<int>(), na);
  apx_avg_state st{};
  st.n_avg = md->p.avg_samples;
  st.window = md->p.avg_window;
  st.samples = md->avg_taken;
  st.dw_min = md->p.avg_dw_min;
  st.csp_ring = md->csp_ring.as<double>();
  st.w_ring = md->w_ring.as<double>();
  apx_status s = apx_compute_precision_avg(ctx, &md->atoms, &nl, &p, &st, w0x, md->csp.as<double>(),
                                           md->csp_avg.as<double>(), md->w0.as<double>(), md->w_min.as<double>(),
                                           nullptr, w, md->mask.as<uint8_t>(), md->active.as<int>(), na);
  md->avg_taken = st.samples;
  return s;
}

apx_status md_weights(apx_md* md, const double* pos, double* w) {
  apx_ctx* ctx = md->ctx;
  md->atoms.pos = pos;
  const long long n = md->n;
  if (md->p.mode == APX_MODE_FULL_ACE) {
    k_fill_d<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(n, w, 1.0);
    k_iota<<<blocks_for(n, 256), 256, 0, ctx->stream>>>((int)n, md->active.as<int>());
    APX_LAUNCH_CHECK(ctx);
    md->n_active = n;
    return APX_OK;
  }
  if (md->p.mode == APX_MODE_EAM) {
    k_fill_d<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(n, w, 0.0);
    APX_LAUNCH_CHECK(ctx);
    md->n_active = 0;
    return APX_OK;
  }
  apx_nlist nl;
  md_nlist(md, nl);
  int64_t na = 0;
  if (md->mlp) {
    // learned criterion: unweighted EAM (density, force), CSP without spreading, features,
    // bfloat16 inference -> extra weight, then the full precision pass on the given CSP
    apx_status s = apx_eam_forces(ctx, &md->atoms, &nl, &md->eam, nullptr, md->e_eam.as<double>(),
                                  md->rho.as<double>(), md->f_eam.as<double>());
    if (s != APX_OK) return s;
    apx_prec_params p0 = md->prec;
    p0.r_hi = 0.0;
    p0.flags = 0;
    // the centro-symmetry pass writes its weights to scratch: w holds the previous filtered
    // weights that the time-averaged pipeline reads
    s = apx_compute_precision(ctx, &md->atoms, &nl, &p0, nullptr, md->csp.as<double>(), md->w0.as<double>(),
                              md->wtmp.as<double>(), md->mask.as<uint8_t>(), md->active.as<int>(), &na);
    if (s != APX_OK) return s;
    s = apx_features(ctx, &md->atoms, &nl, md->rho.as<double>(), md->csp.as<double>(), md->f_eam.as<double>(),
                     md->feat.as<float>());
    if (s != APX_OK) return s;
    s = apx_mlp_precision(ctx, md->mlp, md->feat.as<float>(), md->n, md->tau_lo, md->tau_hi, md->pred.as<float>(),
                          md->w0x.as<double>());
    if (s != APX_OK) return s;
    apx_prec_params p1 = md->prec;
    p1.flags = md->prec.flags | APX_PREC_CSP_GIVEN;
    s = md_precision(md, nl, p1, md->w0x.as<double>(), w, &na);
    if (s != APX_OK) return s;
    md->n_active = na;
    return APX_OK;
  }
  apx_status s = md_precision(md, nl, md->prec, nullptr, w, &na);
  if (s != APX_OK) return s;
  md->n_active = na;
  return APX_OK;
}

// Forces (and energies) at `pos` with weights `w`; f receives the total force including
// the indenter at time t.  Events ev[1..4] bracket the kernel classes.  dual: the weights
// changed since the last force evaluation (md->w_last) and the thermostat is on: the
// force difference F(w_last) - F(w) is formed in the same passes and the energy errors
// are written to md->dE, with vel holding v(t + dt/2).
apx_status md_forces(apx_md* md, const double* pos, const double* w, double* f, double t, bool timed,
                     bool dual = false, const double* vel = nullptr) {
  apx_ctx* ctx = md->ctx;
  md->atoms.pos = pos;
  const long long n = md->n;
  apx_nlist nl;
  md_nlist(md, nl);
  double* scal = md->scal.as<double>();
  const double* wl = md->w_last.as<double>();
  if (timed) APX_HIP(ctx, hipEventRecord(md->ev[2], ctx->stream));
  apx_status s;
  if (md->p.mode != APX_MODE_FULL_ACE) {
    if (dual)
      s = eam_forces_dual(ctx, &md->atoms, &nl, &md->eam, w, wl, md->e_eam.as<double>(), md->rho.as<double>(),
                          md->f_eam.as<double>(), md->df.as<double>(), md->eam4.as<double>());
    else
      s = apx_eam_forces(ctx, &md->atoms, &nl, &md->eam, w, md->e_eam.as<double>(), md->rho.as<double>(),
                         md->f_eam.as<double>());
    if (s != APX_OK) return s;
  } else {
    k_fill_d<<<blocks_for(3 * n, 256), 256, 0, ctx->stream>>>(3 * n, md->f_eam.as<double>(), 0.0);
    k_fill_d<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(n, md->e_eam.as<double>(), 0.0);
    APX_LAUNCH_CHECK(ctx);
  }
  if (timed) APX_HIP(ctx, hipEventRecord(md->ev[3], ctx->stream));
  if (md->p.mode != APX_MODE_EAM && md->ace) {
    if (dual) {
      // ACE over the atoms with either weight > 0; the second output is F(w_last) - F(w)
      int* flag = md->uactive.as<int>() + n;
      k_union<<<blocks_for(n, 256), 256, 0, ctx->stream>>>((int)n, w, wl, md->dw.as<double>(), flag);
      APX_LAUNCH_CHECK(ctx);
      APX_ALLOC(ctx, ctx->itmp2, sizeof(int) * (size_t)(n + 1));
      s = scan_exclusive(ctx, flag, n, ctx->itmp2.as<int>());
      if (s != APX_OK) return s;
      k_compact_flags<<<blocks_for(n, 256), 256, 0, ctx->stream>>>((int)n, flag, ctx->itmp2.as<int>(),
                                                                   md->uactive.as<int>());
      APX_LAUNCH_CHECK(ctx);
      int nu = 0;
      s = read_ints(ctx, ctx->itmp2.as<int>() + n, &nu, 1);
      if (s != APX_OK) return s;
      s = ace_energy_forces_dual(ctx, &md->atoms, &nl, md->ace, w, md->dw.as<double>(), md->uactive.as<int>(), nu,
                                 md->p.ace_precision, md->e_ace.as<double>(), md->f_ace.as<double>(),
                                 md->df_ace.as<double>());
      if (s != APX_OK) return s;
      md->ace_count = nu;
    } else {
      s = apx_ace_energy_forces(ctx, &md->atoms, &nl, md->ace, w, md->active.as<int>(), md->n_active,
                                md->p.ace_precision, md->e_ace.as<double>(), md->f_ace.as<double>(), nullptr,
                                nullptr);
      if (s != APX_OK) return s;
      md->ace_count = md->n_active;
    }
  } else {
    md->ace_count = 0;
    k_fill_d<<<blocks_for(3 * n, 256), 256, 0, ctx->stream>>>(3 * n, md->f_ace.as<double>(), 0.0);
    k_fill_d<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(n, md->e_ace.as<double>(), 0.0);
    if (dual) k_fill_d<<<blocks_for(3 * n, 256), 256, 0, ctx->stream>>>(3 * n, md->df_ace.as<double>(), 0.0);
    APX_LAUNCH_CHECK(ctx);
  }
  if (timed) APX_HIP(ctx, hipEventRecord(md->ev[4], ctx->stream));
  s = apx_blend(ctx, n, w, md->e_eam.as<double>(), md->e_ace.as<double>(), md->f_eam.as<double>(),
                md->f_ace.as<double>(), md->e_site.as<double>(), f, scal + 0);
  if (s != APX_OK) return s;
  if (dual) {
    // energy errors from the interatomic forces (f before the indenter is added)
    if (md->p.mode == APX_MODE_FULL_ACE)
      k_fill_d<<<blocks_for(3 * n, 256), 256, 0, ctx->stream>>>(3 * n, md->df.as<double>(), 0.0);
    k_add_into<<<blocks_for(3 * n, 256), 256, 0, ctx->stream>>>(3 * n, md->df.as<double>(),
                                                                md->df_ace.as<double>());
    APX_LAUNCH_CHECK(ctx);
    s = thermostat_errors(ctx, n, md->atoms.frozen, wl, w, md->e_eam.as<double>(), md->e_ace.as<double>(), f,
                          md->df.as<double>(), vel, md->p.dt, md->p.mass, md->dE.as<double>());
    if (s != APX_OK) return s;
  }
  k_fill_d<<<1, 64, 0, ctx->stream>>>(1, scal + 2, 0.0);
  if (md->p.indenter) {
    const double cx = md->p.ind_center[0] + t * md->p.ind_velocity[0];
    const double cy = md->p.ind_center[1] + t * md->p.ind_velocity[1];
    const double cz = md->p.ind_center[2] + t * md->p.ind_velocity[2];
    BoxDev b = make_box(&md->atoms);
    ProfScope ps(ctx, "md.indenter");
    k_indenter<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(n, pos, f, b, cx, cy, cz, md->p.ind_radius,
                                                            md->p.ind_k, scal + 2);
  }
  APX_LAUNCH_CHECK(ctx);
  return APX_OK;
}

bool md_after_forces(const apx_md* md) {
  return md->p.mode == APX_MODE_ADAPTIVE && md->p.avg_samples > 0 && md->p.avg_window == APX_WINDOW_PAST;
}

}  // namespace

extern "C" apx_status apx_md_create(apx_ctx* ctx, const apx_atoms* atoms, const apx_md_params* p,
                                    const apx_eam_params* eam, const apx_ace_model* ace,
                                    const apx_prec_params* prec, apx_md** out) {
  if (!ctx) return APX_EINVAL;
  if (!atoms || !p || !eam || !out) return fail(ctx, APX_EINVAL, "atoms, params, eam and out are required");
  *out = nullptr;
  apx_atoms a = *atoms;
  a.pos = nullptr;
  if (a.n <= 0 || a.n > 0x7fffffff) return fail(ctx, APX_EINVAL, "bad atom count");
  if (p->mode != APX_MODE_ADAPTIVE && p->mode != APX_MODE_FULL_ACE && p->mode != APX_MODE_EAM)
    return fail(ctx, APX_EINVAL, "unknown mode");
  if (p->mode != APX_MODE_EAM && !ace) return fail(ctx, APX_EINVAL, "this mode needs an ACE model");
  if (p->mode == APX_MODE_ADAPTIVE && !prec) return fail(ctx, APX_EINVAL, "adaptive mode needs precision params");
  if (!(p->dt > 0.0) || !(p->mass > 0.0) || !(p->skin >= 0.0)) return fail(ctx, APX_EINVAL, "dt, mass, skin");
  if (p->max_nb < 1 || p->max_nb > 128) return fail(ctx, APX_EINVAL, "max_nb must be in 1..128");
  if (p->avg_samples < 0 || p->avg_samples > 4096) return fail(ctx, APX_EINVAL, "avg_samples must be in 0..4096");
  if (p->avg_samples > 0 && !(p->avg_dw_min >= 0.0)) return fail(ctx, APX_EINVAL, "avg_dw_min must be >= 0");
  if (p->avg_window != APX_WINDOW_PAST && p->avg_window != APX_WINDOW_CURRENT)
    return fail(ctx, APX_EINVAL, "avg_window must be APX_WINDOW_PAST or APX_WINDOW_CURRENT");
  if (p->thermostat != 0 && p->thermostat != 1) return fail(ctx, APX_EINVAL, "thermostat must be 0 or 1");
  if (p->thermostat && (!(p->thermo.r_omega > 0.0) || p->thermo.omega_max < 1 || p->thermo.group_batch < 0))
    return fail(ctx, APX_EINVAL, "thermostat needs r_omega > 0 and omega_max >= 1");
  apx_md* md = new apx_md();
  md->ctx = ctx;
  md->p = *p;
  md->eam = *eam;
  if (prec) md->prec = *prec;
  md->ace = ace;
  md->atoms = a;
  md->n = (int)a.n;
  md->max_nb = p->max_nb;
  double rc = eam->r_cut;
  if (ace) {
    rc = rc > ace->r_cut ? rc : ace->r_cut;
    if (ace->anchored) rc = rc > ace->anchor.r_cut ? rc : ace->anchor.r_cut;
  }
  if (prec && p->mode == APX_MODE_ADAPTIVE) rc = rc > prec->r_cut ? rc : prec->r_cut;
  md->r_list = rc + p->skin;
  const size_t n = md->n;
  bool ok = md->nl_count.ensure(sizeof(int) * n) == hipSuccess &&
            md->nl_idx.ensure(sizeof(int) * n * md->max_nb) == hipSuccess &&
            md->xref.ensure(sizeof(double) * 3 * n) == hipSuccess && md->lo_dev.ensure(sizeof(double) * 3) == hipSuccess &&
            md->csp.ensure(sizeof(double) * n) == hipSuccess && md->w0.ensure(sizeof(double) * n) == hipSuccess &&
            md->mask.ensure(n) == hipSuccess && md->active.ensure(sizeof(int) * n) == hipSuccess &&
            md->e_eam.ensure(sizeof(double) * n) == hipSuccess && md->e_ace.ensure(sizeof(double) * n) == hipSuccess &&
            md->e_site.ensure(sizeof(double) * n) == hipSuccess && md->f_eam.ensure(sizeof(double) * 3 * n) == hipSuccess &&
            md->f_ace.ensure(sizeof(double) * 3 * n) == hipSuccess && md->rho.ensure(sizeof(double) * n) == hipSuccess &&
            md->scal.ensure(sizeof(double) * 8) == hipSuccess;
  if (ok && p->mode == APX_MODE_ADAPTIVE && p->avg_samples > 0) {
    const size_t ring = sizeof(double) * (size_t)p->avg_samples * n;
    ok = md->csp_ring.ensure(ring) == hipSuccess && md->w_ring.ensure(ring) == hipSuccess &&
         md->csp_avg.ensure(sizeof(double) * n) == hipSuccess && md->w_min.ensure(sizeof(double) * n) == hipSuccess;
  }
  if (ok && p->mode == APX_MODE_ADAPTIVE)
    ok = md->wtmp.ensure(sizeof(double) * n) == hipSuccess;
  if (ok && p->thermostat)
    ok = md->w_last.ensure(sizeof(double) * n) == hipSuccess && md->dw.ensure(sizeof(double) * n) == hipSuccess &&
         md->df.ensure(sizeof(double) * 3 * n) == hipSuccess &&
         md->df_ace.ensure(sizeof(double) * 3 * n) == hipSuccess && md->dE.ensure(sizeof(double) * n) == hipSuccess &&
         md->eam4.ensure(sizeof(double) * 4 * n) == hipSuccess && md->uactive.ensure(sizeof(int) * 2 * n) == hipSuccess;
  if (!ok) {
    delete md;
    return fail(ctx, APX_ENOMEM, "integrator buffers");
  }
  if (hipMemcpy(md->lo_dev.p, a.lo, sizeof(double) * 3, hipMemcpyHostToDevice) != hipSuccess) {
    delete md;
    return fail(ctx, APX_EDEVICE, "upload of box origin");
  }
  for (auto& e : md->ev) {
    if (hipEventCreate(&e) != hipSuccess) {
      delete md;
      return fail(ctx, APX_EDEVICE, "event creation");
    }
  }
  *out = md;
  return APX_OK;
}

extern "C" void apx_md_destroy(apx_md* md) {
  if (!md) return;
  (void)hipStreamSynchronize(md->ctx->stream);
  for (auto& e : md->ev)
    if (e) (void)hipEventDestroy(e);
  delete md;
}

extern "C" apx_status apx_md_init(apx_md* md, const double* pos, double* f, double* w) {
  if (!md) return APX_EINVAL;
  apx_ctx* ctx = md->ctx;
  if (!pos || !f || !w) return fail(ctx, APX_EINVAL, "pos, f and w are required");
  apx_status s = md_rebuild(md, pos);
  if (s != APX_OK) return s;
  md->avg_taken = 0;
  s = md_weights(md, pos, w);
  if (s != APX_OK) return s;
  s = md_forces(md, pos, w, f, md->step * md->p.dt, false);
  if (s != APX_OK) return s;
  if (md->p.thermostat) {
    k_copy_d<<<blocks_for(md->n, 256), 256, 0, ctx->stream>>>(md->n, w, md->w_last.as<double>());
    APX_LAUNCH_CHECK(ctx);
  }
  md->w_dirty = false;
  md->initialized = true;
  APX_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return APX_OK;
}

namespace {
apx_status md_stats(apx_md* md, const double* vel, apx_md_stats st, apx_md_stats* out) {
  apx_ctx* ctx = md->ctx;
  const long long n = md->n;
  double* scal = md->scal.as<double>();
  k_fill_d<<<1, 64, 0, ctx->stream>>>(1, scal + 1, 0.0);
  k_kinetic<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(n, vel, md->atoms.frozen, 0.5 * md->p.mass / kAccel,
                                                         scal + 1);
  APX_LAUNCH_CHECK(ctx);
  double h[3];
  APX_HIP(ctx, hipMemcpyAsync(h, scal, sizeof(double) * 3, hipMemcpyDeviceToHost, ctx->stream));
  APX_HIP(ctx, hipStreamSynchronize(ctx->stream));
  st.e_pot = h[0];
  st.e_kin = h[1];
  st.e_indenter = h[2];
  st.n_active = md->n_active;
  *out = st;
  return APX_OK;
}
}  // namespace

extern "C" apx_status apx_verlet_step(apx_md* md, double* pos, double* vel, double* f, double* w, int64_t n_steps,
                                      apx_md_stats* stats) {
  if (!md) return APX_EINVAL;
  apx_ctx* ctx = md->ctx;
  if (!pos || !vel || !f || !w) return fail(ctx, APX_EINVAL, "pos, vel, f and w are required");
  if (!md->initialized) return fail(ctx, APX_EINVAL, "call apx_md_init first");
  if (n_steps < 0) return fail(ctx, APX_EINVAL, "negative step count");
  const long long n = md->n;
  const double ck = 0.5 * md->p.dt * kAccel / md->p.mass;
  double* scal = md->scal.as<double>();
  BoxDev b = make_box(&md->atoms);
  apx_md_stats st{};
  for (int k = 0; k < 5; ++k) md->t_acc[k] = 0.0;
  // class timers only while the context profiles: otherwise the step loop waits on the
  // device once per step, for the rebuild test
  const bool timed = ctx->prof;
  for (int64_t it = 0; it < n_steps; ++it) {
    if (timed) APX_HIP(ctx, hipEventRecord(md->ev[0], ctx->stream));
    k_fill_d<<<1, 64, 0, ctx->stream>>>(1, scal + 3, 0.0);
    {
    ProfScope ps(ctx, "md.kick_drift");
    k_kick_drift<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(n, pos, vel, f, md->atoms.frozen, ck, md->p.dt, b,
                                                             md->lo_dev.as<double>(), md->xref.as<double>(),
                                                             reinterpret_cast<unsigned long long*>(scal + 3));
    APX_LAUNCH_CHECK(ctx);
    }
    double maxd2 = 0.0;
    APX_HIP(ctx, hipMemcpyAsync(ctx->host_pinned, scal + 3, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    APX_HIP(ctx, hipStreamSynchronize(ctx->stream));
    std::memcpy(&maxd2, ctx->host_pinned, sizeof(double));
    prof_flush(ctx, false);
    const double half_skin = 0.5 * md->p.skin;
    if (maxd2 > half_skin * half_skin) {
      apx_status s = md_rebuild(md, pos);
      if (s != APX_OK) return s;
      ++st.rebuilds;
    }
    if (timed) APX_HIP(ctx, hipEventRecord(md->ev[1], ctx->stream));
    md->step += 1;
    const bool due = md->p.mode == APX_MODE_ADAPTIVE && md->p.precision_every > 0 &&
                     md->step % md->p.precision_every == 0;
    const bool after = md_after_forces(md);
    if (due && !after) {
      apx_status s = md_weights(md, pos, w);
      if (s != APX_OK) return s;
      ++st.precision_updates;
      md->w_dirty = true;
    }
    const bool dual = md->p.thermostat && md->w_dirty;
    apx_status s = md_forces(md, pos, w, f, md->step * md->p.dt, timed, dual, vel);
    if (s != APX_OK) return s;
    st.ace_atoms += md->ace_count;
    {
    ProfScope ps(ctx, "md.kick");
    k_kick<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(n, vel, f, md->atoms.frozen, ck);
    APX_LAUNCH_CHECK(ctx);
    }
    bool radicand = false;
    if (dual) {
      int64_t nc = 0, nf = 0;
      s = thermostat_correct(ctx, &md->atoms, vel, md->dE.as<double>(), &md->p.thermo, md->step, md->p.mass, &nc,
                             &nf);
      if (s != APX_OK) return s;
      st.thermo_steps += 1;
      st.thermo_corrected += nc;
      st.thermo_failed += nf;
      radicand = nf > 0;
      k_copy_d<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(n, w, md->w_last.as<double>());
      APX_LAUNCH_CHECK(ctx);
    }
    md->w_dirty = false;
    if (due && after) {
      s = md_weights(md, pos, w);
      if (s != APX_OK) return s;
      ++st.precision_updates;
      md->w_dirty = true;
    }
    if (radicand) {
      // a skipped correction: the step is complete; report it before taking the next one
      ++st.steps;
      if (stats) {
        s = md_stats(md, vel, st, stats);
        if (s != APX_OK) return s;
      }
      return fail(ctx, APX_ERADICAND, "thermostat: %lld corrections at step %lld had a negative radicand",
                  (long long)st.thermo_failed, md->step);
    }
    if (timed) {
      APX_HIP(ctx, hipEventRecord(md->ev[5], ctx->stream));
      APX_HIP(ctx, hipEventSynchronize(md->ev[5]));
      float ms = 0.f;
      // ev0..ev1: integrate + rebuild, ev1..ev2: precision, ev2..ev3: EAM, ev3..ev4: ACE, ev4..ev5: blend+kick
      if (hipEventElapsedTime(&ms, md->ev[0], md->ev[1]) == hipSuccess) md->t_acc[0] += ms;
      if (hipEventElapsedTime(&ms, md->ev[1], md->ev[2]) == hipSuccess) md->t_acc[1] += ms;
      if (hipEventElapsedTime(&ms, md->ev[2], md->ev[3]) == hipSuccess) md->t_acc[2] += ms;
      if (hipEventElapsedTime(&ms, md->ev[3], md->ev[4]) == hipSuccess) md->t_acc[3] += ms;
      if (hipEventElapsedTime(&ms, md->ev[4], md->ev[5]) == hipSuccess) md->t_acc[4] += ms;
    }
    ++st.steps;
  }
  if (stats) {
    apx_status s = md_stats(md, vel, st, stats);
    if (s != APX_OK) return s;
  }
  return APX_OK;
}

extern "C" apx_status apx_md_set_mlp(apx_md* md, apx_mlp* mlp, double tau_lo, double tau_hi) {
  if (!md) return APX_EINVAL;
  apx_ctx* ctx = md->ctx;
  if (mlp && !(tau_hi > tau_lo)) return fail(ctx, APX_EINVAL, "tau_hi must exceed tau_lo");
  if (mlp && md->p.mode != APX_MODE_ADAPTIVE) return fail(ctx, APX_EINVAL, "the learned criterion needs adaptive mode");
  md->mlp = mlp;
  md->tau_lo = tau_lo;
  md->tau_hi = tau_hi;
  if (mlp) {
    APX_ALLOC(ctx, md->feat, sizeof(float) * 4 * (size_t)md->n);
    APX_ALLOC(ctx, md->pred, sizeof(float) * (size_t)md->n);
    APX_ALLOC(ctx, md->w0x, sizeof(double) * (size_t)md->n);
  }
  return APX_OK;
}

extern "C" apx_status apx_md_timings(apx_md* md, double* out5) {
  if (!md || !out5) return APX_EINVAL;
  for (int k = 0; k < 5; ++k) out5[k] = md->t_acc[k];
  return APX_OK;
}
