// Host-side construction of the ACE coupling tables (basis catalogue, pair and triple
// lists, per-wave work split) and their upload to the device.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <tuple>
#include <utility>

#include "ace_coupling_gen.h"
#include "ace_model.h"

namespace apx {
namespace {

template <int LMAX, int L1, int L2>
constexpr int couple_terms() {
  return Couple<LMAX, L1, L2>::kTerms;
}

template <int LMAX>
int terms_of(int l1, int l2) {
  static const int tab4[5][5] = {
      {couple_terms<4, 0, 0>(), couple_terms<4, 0, 1>(), couple_terms<4, 0, 2>(), couple_terms<4, 0, 3>(), couple_terms<4, 0, 4>()},
      {couple_terms<4, 1, 0>(), couple_terms<4, 1, 1>(), couple_terms<4, 1, 2>(), couple_terms<4, 1, 3>(), couple_terms<4, 1, 4>()},
      {couple_terms<4, 2, 0>(), couple_terms<4, 2, 1>(), couple_terms<4, 2, 2>(), couple_terms<4, 2, 3>(), couple_terms<4, 2, 4>()},
      {couple_terms<4, 3, 0>(), couple_terms<4, 3, 1>(), couple_terms<4, 3, 2>(), couple_terms<4, 3, 3>(), couple_terms<4, 3, 4>()},
      {couple_terms<4, 4, 0>(), couple_terms<4, 4, 1>(), couple_terms<4, 4, 2>(), couple_terms<4, 4, 3>(), couple_terms<4, 4, 4>()}};
  static const int tab3[4][4] = {
      {couple_terms<3, 0, 0>(), couple_terms<3, 0, 1>(), couple_terms<3, 0, 2>(), couple_terms<3, 0, 3>()},
      {couple_terms<3, 1, 0>(), couple_terms<3, 1, 1>(), couple_terms<3, 1, 2>(), couple_terms<3, 1, 3>()},
      {couple_terms<3, 2, 0>(), couple_terms<3, 2, 1>(), couple_terms<3, 2, 2>(), couple_terms<3, 2, 3>()},
      {couple_terms<3, 3, 0>(), couple_terms<3, 3, 1>(), couple_terms<3, 3, 2>(), couple_terms<3, 3, 3>()}};
  return LMAX == 4 ? tab4[l1][l2] : tab3[l1][l2];
}

bool coupled(int l1, int l2, int l3) { return ((l1 + l2 + l3) % 2 == 0) && l3 >= std::abs(l1 - l2) && l3 <= l1 + l2; }

// Coupling terms of (l1, l2) -> L alone (the per-degree functions Couple3).
template <int LMAX, int L1, int L2, int L>
constexpr int terms3() {
  if constexpr ((L1 + L2 + L) % 2 == 0 && L >= (L1 > L2 ? L1 - L2 : L2 - L1) && L <= L1 + L2 && L <= LMAX)
    return Couple3<LMAX, L1, L2, L>::kTerms;
  else
    return 0;
}
template <int LMAX, int L1, int L2, int... Ls>
int terms3_L(int L, std::integer_sequence<int, Ls...>) {
  int r = 0;
  ((r = (L == Ls ? terms3<LMAX, L1, L2, Ls>() : r)), ...);
  return r;
}
template <int LMAX, int L1, int... L2s>
int terms3_l2(int l2, int L, std::integer_sequence<int, L2s...>) {
  int r = 0;
  ((r = (l2 == L2s ? terms3_L<LMAX, L1, L2s>(L, std::make_integer_sequence<int, LMAX + 1>{}) : r)), ...);
  return r;
}
template <int LMAX, int... L1s>
int terms3_l1(int l1, int l2, int L, std::integer_sequence<int, L1s...>) {
  int r = 0;
  ((r = (l1 == L1s ? terms3_l2<LMAX, L1s>(l2, L, std::make_integer_sequence<int, LMAX + 1>{}) : r)), ...);
  return r;
}
int terms3_of(int l_max, int l1, int l2, int L) {
  return l_max == 4 ? terms3_l1<4>(l1, l2, L, std::make_integer_sequence<int, 5>{})
                    : terms3_l1<3>(l1, l2, L, std::make_integer_sequence<int, 4>{});
}

struct Catalogue {
  long long n_basis = 0;
  std::vector<int> pairs, t_v, b1_off, b1_v, b2_off, b2_v, units, wave_units, adj_ent;
  int group_units[kUnitGroups] = {};
  int ntrip = 0;
  long long coupling_terms = 0, triple_width = 0;
};

Catalogue build_catalogue(int n_max, int l_max) {
  Catalogue c;
  const int LL = l_max + 1;
  const int P = n_max * LL;
  auto off = [&](int p) { int n = p / LL, l = p % LL; return n * LL * LL + l * l; };
  long long v = 0;
  for (int n = 0; n < n_max; ++n) {
    c.b1_off.push_back(n * LL * LL);
    c.b1_v.push_back((int)v++);
  }
  for (int n1 = 0; n1 < n_max; ++n1)
    for (int n2 = n1; n2 < n_max; ++n2)
      for (int l = 0; l < LL; ++l) {
        c.b2_off.push_back(n1 * LL * LL + l * l);
        c.b2_off.push_back(n2 * LL * LL + l * l);
        c.b2_off.push_back(l);
        c.b2_v.push_back((int)v++);
      }
  // B3: the basis indices follow the enumeration p1 <= p2 <= p3 of labels p = n (l_max+1) + l
  // (the basis definition).  The real Gaunt product of three blocks is symmetric in them,
  // so each triple may be evaluated as any of its labels coupled to the pair of the other
  // two.  Here the third block is the label that comes first in degree-major order
  // (l, then n) and the pair holds the other two: a pair (q2 <= q3) then meets third
  // blocks of degree L < l(q2) for every n, and of degree l(q2) for n <= n(q2).  Each pair
  // and degree thus has a run of third blocks n = 0, 1, ... of full or near-full length,
  // which makes fewer (pair, degree) combinations than the enumeration order would.
  struct PairTmp {
    int rec[kPairRec];
    std::vector<int> v;  // basis indices of its triples, in segment order
    double cost;
  };
  auto lkey = [LL](int p) { return std::make_pair(p % LL, p / LL); };
  std::map<std::pair<int, int>, std::vector<std::vector<std::pair<int, int>>>> groups;  // (n3, v) by L
  for (int p1 = 0; p1 < P; ++p1)
    for (int p2 = p1; p2 < P; ++p2)
      for (int p3 = p2; p3 < P; ++p3) {
        if (!coupled(p1 % LL, p2 % LL, p3 % LL)) continue;
        std::array<int, 3> s3 = {p1, p2, p3};
        std::sort(s3.begin(), s3.end(), [&](int a, int b) { return lkey(a) < lkey(b); });
        auto& g = groups[{s3[1], s3[2]}];
        if (g.empty()) g.resize(LL);
        g[s3[0] % LL].push_back({s3[0] / LL, (int)v++});
      }
  std::vector<PairTmp> tmp;
  for (auto& kv : groups) {
    const int q2 = kv.first.first, q3 = kv.first.second;
    const int l1 = q2 % LL, l2 = q3 % LL;
    auto& byL = kv.second;
    PairTmp pt{};
    pt.rec[0] = off(q2);
    pt.rec[1] = off(q3);
    pt.rec[2] = l1 * LL + l2;
    pt.rec[3] = q2 / LL;
    pt.rec[15] = q3 / LL;
    pt.cost = 8.0;
    int t = 0;
    for (int L = 0; L < LL; ++L) {
      std::sort(byL[L].begin(), byL[L].end());
      pt.rec[4 + L] = t;
      pt.rec[10 + L] = byL[L].empty() ? 0 : byL[L][0].first * LL * LL + L * L;
      if (!byL[L].empty()) {
        const int nterm = terms3_of(l_max, l1, l2, L);
        c.coupling_terms += nterm;
        pt.cost += nterm;
      }
      for (size_t e = 0; e < byL[L].size(); ++e) {
        // third blocks of one degree are consecutive in n: offsets step by (l_max+1)^2
        if (byL[L][e].first != byL[L][0].first + (int)e) throw 1;
        pt.v.push_back(byL[L][e].second);
        pt.cost += 2 * L + 1 + 2;
        c.triple_width += 2 * L + 1;
        ++t;
      }
    }
    for (int L = LL; L <= 5; ++L) pt.rec[4 + L] = t;
    tmp.push_back(pt);
  }
  c.n_basis = v;
  // group the pairs by coupling type so that a wave stays in one specialisation for
  // long runs of pairs (instruction-cache locality); within a type order them by the
  // label of larger degree (the run label of the adjoint units), then the other label
  auto key = [LL](const PairTmp& a) {
    const int l1 = a.rec[2] / LL, l2 = a.rec[2] % LL;
    const int run = l1 >= l2 ? a.rec[3] : a.rec[15];
    const int oth = l1 >= l2 ? a.rec[15] : a.rec[3];
    return std::make_tuple(a.rec[2], run, oth);
  };
  std::stable_sort(tmp.begin(), tmp.end(), [&](const PairTmp& a, const PairTmp& b) { return key(a) < key(b); });
  std::vector<double> cost;
  int base = 0;
  for (auto& pt : tmp) {
    for (int L = 0; L <= 5; ++L) pt.rec[4 + L] += base;
    base += (int)pt.v.size();
    c.pairs.insert(c.pairs.end(), pt.rec, pt.rec + kPairRec);
    c.t_v.insert(c.t_v.end(), pt.v.begin(), pt.v.end());
    cost.push_back(pt.cost);
  }
  c.ntrip = base;
  // adjoint units (type, L) over the contiguous pair range of each type, plus the B1/B2
  // units, dealt to the waves by longest processing time first
  std::vector<std::array<int, kUnitRec>> units;
  std::vector<double> ucost;
  {
    // a unit (type, L) covers the pairs whose other label lies in [obase, oend); the
    // ranges are cut by cost so that every launch group has at least two units per wave
    int ntypes[kUnitGroups] = {};
    for (size_t q = 0; q < tmp.size(); ++q) {
      if (q > 0 && tmp[q].rec[2] == tmp[q - 1].rec[2]) continue;
      const int l1 = tmp[q].rec[2] / LL, l2 = tmp[q].rec[2] % LL;
      for (int L = 0; L < LL; ++L) {
        bool any = false;
        for (size_t k = q; k < tmp.size() && tmp[k].rec[2] == tmp[q].rec[2]; ++k)
          any = any || tmp[k].rec[5 + L] > tmp[k].rec[4 + L];
        if (any && coupled(l1, l2, L)) ++ntypes[unit_group(L)];
      }
    }
    int q = 0;
    const int np = (int)tmp.size();
    while (q < np) {
      int e = q;
      while (e < np && tmp[e].rec[2] == tmp[q].rec[2]) ++e;
      const int type = tmp[q].rec[2];
      const int l1 = type / LL, l2 = type % LL;
      for (int L = 0; L < LL; ++L) {
        if (!coupled(l1, l2, L)) continue;
        std::vector<double> cost_o(n_max, 0.0);
        for (int k = q; k < e; ++k) {
          const int noth = l1 >= l2 ? tmp[k].rec[15] : tmp[k].rec[3];
          const int nt = tmp[k].rec[5 + L] - tmp[k].rec[4 + L];
          if (nt > 0) cost_o[noth] += 40.0 + 6.0 * nt * (2 * L + 1) + 3.0 * (2 * l1 + 1) * (2 * l2 + 1);
        }
        double total = 0.0;
        for (double x : cost_o) total += x;
        if (total <= 0.0) continue;
        const int nt_g = std::max(1, ntypes[unit_group(L)]);
        const int parts = std::max(2, (2 * kUnitWaves + nt_g - 1) / nt_g);
        int b = 0;
        double acc = 0.0;
        int made = 0;
        for (int o = 0; o < n_max; ++o) {
          acc += cost_o[o];
          const bool cut = o == n_max - 1 || o - b + 1 == unit_width(unit_group(L), n_max) ||
                           acc >= total * (made + 1) / parts;
          if (!cut) continue;
          double cst = 0.0;
          for (int x = b; x <= o; ++x) cst += cost_o[x];
          if (cst > 0.0) {
            units.push_back({type, L, q, e, b, 0, 0, o + 1});
            ucost.push_back(cst + 30.0 * n_max * (2 * L + 1));
          }
          ++made;
          b = o + 1;
        }
      }
      q = e;
    }
    // B1/B2: one unit per first label n1 (its B1 entry and its B2 entries n2 >= n1)
    for (int n1 = 0; n1 < n_max; ++n1) {
      double cst = 3.0;
      for (int l = 0; l < LL; ++l) cst += (n_max - n1) * (2 * l + 1) * 6.0 + (2 * l + 1) * 3.0;
      units.push_back({0, -1, n1, 0, 0, 0, 0, 0});
      ucost.push_back(cst);
    }
  }
  // the pair stream of every (type, L) unit: the pairs of its half that have third blocks
  // of degree L, in pair order (by run label, then other label)
  for (auto& u : units) {
    if (u[1] < 0) continue;
    const int L = u[1], type = u[0];
    const int l1 = type / LL, l2 = type % LL;
    u[5] = (int)(c.adj_ent.size() / kAdjEnt);
    for (int k = u[2]; k < u[3]; ++k) {
      const int* r = tmp[k].rec;
      if (r[5 + L] <= r[4 + L]) continue;
      const int nrun = l1 >= l2 ? r[3] : r[15];
      const int noth = l1 >= l2 ? r[15] : r[3];
      if (noth < u[4] || noth >= u[7]) continue;
      const int n30 = (r[10 + L] - L * L) / (LL * LL);
      c.adj_ent.insert(c.adj_ent.end(), {r[0], r[1], nrun, noth, n30, r[4 + L], r[5 + L] - r[4 + L]});
    }
    u[6] = (int)(c.adj_ent.size() / kAdjEnt);
  }
  // each launch group is dealt to the waves separately, longest processing time first
  for (auto& u : units) c.units.insert(c.units.end(), u.begin(), u.end());
  c.wave_units.assign(kUnitGroups * (kUnitWaves + 1), 0);
  std::vector<int> order(units.size());
  for (size_t k = 0; k < order.size(); ++k) order[k] = (int)k;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return ucost[a] > ucost[b]; });
  for (int g = 0; g < kUnitGroups; ++g) {
    std::vector<std::vector<int>> per(kUnitWaves);
    std::vector<double> load(kUnitWaves, 0.0);
    for (int u : order) {
      if (unit_group(units[u][1]) != g) continue;
      int best = 0;
      for (int w = 1; w < kUnitWaves; ++w)
        if (load[w] < load[best]) best = w;
      per[best].push_back(u);
      load[best] += ucost[u];
      ++c.group_units[g];
    }
    int* off = c.wave_units.data() + g * (kUnitWaves + 1);
    off[0] = (int)c.wave_units.size() - kUnitGroups * (kUnitWaves + 1);
    for (int w = 0; w < kUnitWaves; ++w) {
      // within a wave, keep units of one type together
      std::sort(per[w].begin(), per[w].end());
      c.wave_units.insert(c.wave_units.end(), per[w].begin(), per[w].end());
      off = c.wave_units.data() + g * (kUnitWaves + 1);
      off[w + 1] = (int)c.wave_units.size() - kUnitGroups * (kUnitWaves + 1);
    }
  }
  return c;
}

}  // namespace
}  // namespace apx

using namespace apx;

extern "C" int64_t apx_ace_num_basis(int32_t n_max, int32_t l_max) {
  if (n_max < 1 || n_max > 12 || (l_max != 3 && l_max != 4)) return -1;
  try {
    return build_catalogue(n_max, l_max).n_basis;
  } catch (...) {
    return -1;
  }
}

template <class T>
static void fill_reals(std::vector<T>& out, const apx_ace_model* m, const Catalogue& c, const double* c1,
                       const double* c2, size_t* offs) {
  const int LL = m->l_max + 1, nm = m->n_max;
  // order: Wp, (c1, c2) per triple + one padding pair, b1_c1, b1_c2, b2_c1, b2_c2
  out.clear();
  offs[0] = out.size();
  for (int l = 0; l < LL; ++l) {
    const double nl = std::sqrt((2.0 * l + 1.0) / (4.0 * M_PI));
    for (int n = 0; n < nm; ++n)
      for (int k = 0; k < nm; ++k) out.push_back((T)(m->W[((size_t)l * nm + n) * nm + k] * nl / m->s_a));
  }
  while (out.size() % 4) out.push_back((T)0);
  // the triples' coefficients with kTcPad zero pairs on either side: a kernel reads the
  // n_max coefficients around a run at once, whatever part of them the run uses
  for (int k = 0; k < 2 * kTcPad; ++k) out.push_back((T)0);
  offs[1] = out.size();
  for (int v : c.t_v) {
    out.push_back((T)c1[v]);
    out.push_back((T)c2[v]);
  }
  for (int k = 0; k < 2 * kTcPad; ++k) out.push_back((T)0);
  offs[2] = out.size();
  offs[3] = out.size();
  for (int v : c.b1_v) out.push_back((T)c1[v]);
  offs[4] = out.size();
  for (int v : c.b1_v) out.push_back((T)c2[v]);
  offs[5] = out.size();
  for (int v : c.b2_v) out.push_back((T)c1[v]);
  offs[6] = out.size();
  for (int v : c.b2_v) out.push_back((T)c2[v]);
  offs[7] = out.size();
}

// The adjoint pair stream with the coefficients of the current model (kAdjRec words per
// entry; coefficients as float32).
static std::vector<int32_t> adjoint_stream(const apx_ace_model* m, const double* c1, const double* c2) {
  const size_t ne = m->adj_ent.size() / kAdjEnt;
  std::vector<int32_t> out(ne * kAdjRec, 0);
  for (size_t e = 0; e < ne; ++e) {
    const int* a = m->adj_ent.data() + kAdjEnt * e;
    int32_t* o = out.data() + e * kAdjRec;
    for (int k = 0; k < 5; ++k) o[k] = a[k];
    const int n30 = a[4], q0 = a[5], nt = a[6];
    for (int n3 = n30; n3 < n30 + nt; ++n3) {
      const int v = m->t_v[q0 + n3 - n30];
      const float f1 = (float)c1[v], f2 = (float)c2[v];
      std::memcpy(o + kAdjC1 + n3, &f1, 4);
      std::memcpy(o + kAdjC2 + n3, &f2, 4);
    }
  }
  return out;
}

template <class T>
static void set_tables(AceTables<T>& t, const T* base, const size_t* offs, const int* ib, const size_t* ioffs) {
  t.Wp = base + offs[0];
  t.tc = reinterpret_cast<const Coef2<T>*>(base + offs[1]);
  t.b1_c1 = base + offs[3];
  t.b1_c2 = base + offs[4];
  t.b2_c1 = base + offs[5];
  t.b2_c2 = base + offs[6];
  t.pairs = ib + ioffs[0];
  t.t_v = ib + ioffs[1];
  t.b1_off = ib + ioffs[2];
  t.b1_v = ib + ioffs[3];
  t.b2_off = ib + ioffs[4];
  t.b2_v = ib + ioffs[5];
  t.units = ib + ioffs[6];
  t.wave_units = ib + ioffs[7];
}

extern "C" apx_status apx_ace_model_create(apx_ctx* ctx, const apx_ace_desc* d, apx_ace_model** out) {
  if (!ctx) return APX_EINVAL;
  if (!d || !out) return fail(ctx, APX_EINVAL, "desc and out are required");
  *out = nullptr;
  if (d->n_max < 1 || d->n_max > 12) return fail(ctx, APX_EINVAL, "n_max must be in 1..12");
  if (d->l_max != 3 && d->l_max != 4) return fail(ctx, APX_EINVAL, "l_max must be 3 or 4");
  if (!d->W || !d->c1 || !d->c2) return fail(ctx, APX_EINVAL, "W, c1 and c2 are required");
  if (d->anchored && d->anchor.kind != APX_EAM_CLOSED)
    return fail(ctx, APX_EINVAL, "the EAM anchor of an ACE model must use the closed form");
  if (!(d->r_cut > 0.0) || !(d->h > 0.0) || !(d->s_a > 0.0) || !(d->eps > 0.0))
    return fail(ctx, APX_EINVAL, "r_cut, h, s_a and eps must be positive");
  Catalogue c;
  try {
    c = build_catalogue(d->n_max, d->l_max);
  } catch (...) {
    return fail(ctx, APX_EINVAL, "inconsistent coupling catalogue");
  }
  apx_ace_model* m = new apx_ace_model();
  m->device = ctx->device;
  m->n_max = d->n_max;
  m->l_max = d->l_max;
  m->na = d->n_max * (d->l_max + 1) * (d->l_max + 1);
  m->n_basis = c.n_basis;
  m->npairs = (int)(c.pairs.size() / kPairRec);
  m->ntrip = c.ntrip;
  m->nb1 = (int)c.b1_v.size();
  m->nb2 = (int)c.b2_v.size();
  m->coupling_terms = c.coupling_terms;
  for (int g = 0; g < kUnitGroups; ++g) m->group_units[g] = c.group_units[g];
  m->triple_width = c.triple_width;
  m->r_cut = d->r_cut;
  m->h = d->h;
  m->s_a = d->s_a;
  m->eps = d->eps;
  m->anchored = d->anchored ? 1 : 0;
  m->anchor = d->anchor;
  m->W.assign(d->W, d->W + (size_t)(d->l_max + 1) * d->n_max * d->n_max);
  m->t_v = c.t_v;
  m->b1_v = c.b1_v;
  m->b2_v = c.b2_v;
  m->adj_ent = c.adj_ent;
  // integer tables
  std::vector<int> ib;
  size_t ioffs[8];
  const std::vector<int>* parts[8] = {&c.pairs, &c.t_v, &c.b1_off, &c.b1_v, &c.b2_off, &c.b2_v, &c.units, &c.wave_units};
  for (int q = 0; q < 8; ++q) {
    ioffs[q] = ib.size();
    ib.insert(ib.end(), parts[q]->begin(), parts[q]->end());
  }
  std::vector<double> r64;
  std::vector<float> r32;
  size_t o64[8], o32[8];
  fill_reals(r64, m, c, d->c1, d->c2, o64);
  fill_reals(r32, m, c, d->c1, d->c2, o32);
  if (m->ints.ensure(ib.size() * sizeof(int)) != hipSuccess || m->reals64.ensure(r64.size() * sizeof(double)) != hipSuccess ||
      m->reals32.ensure(r32.size() * sizeof(float)) != hipSuccess) {
    delete m;
    return fail(ctx, APX_ENOMEM, "ACE table allocation failed");
  }
  hipError_t e1 = hipMemcpy(m->ints.p, ib.data(), ib.size() * sizeof(int), hipMemcpyHostToDevice);
  hipError_t e2 = hipMemcpy(m->reals64.p, r64.data(), r64.size() * sizeof(double), hipMemcpyHostToDevice);
  hipError_t e3 = hipMemcpy(m->reals32.p, r32.data(), r32.size() * sizeof(float), hipMemcpyHostToDevice);
  if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
    delete m;
    return fail(ctx, APX_EDEVICE, "ACE table upload failed");
  }
  set_tables(m->t64, m->reals64.as<double>(), o64, m->ints.as<int>(), ioffs);
  set_tables(m->t32, m->reals32.as<float>(), o32, m->ints.as<int>(), ioffs);
  m->t64.npairs = m->npairs;
  m->t32.npairs = m->npairs;
  const std::vector<int32_t> adj = adjoint_stream(m, d->c1, d->c2);
  if (m->adj.ensure(adj.size() * 4 + 4) != hipSuccess) {
    delete m;
    return fail(ctx, APX_ENOMEM, "ACE table allocation failed");
  }
  if (hipMemcpy(m->adj.p, adj.data(), adj.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
    delete m;
    return fail(ctx, APX_EDEVICE, "ACE table upload failed");
  }
  m->t32.adj_i = m->adj.as<int>();
  m->t32.adj_f = m->adj.as<float>();
  *out = m;
  return APX_OK;
}

extern "C" apx_status apx_ace_model_set_coeffs(apx_ctx* ctx, apx_ace_model* m, const double* c1, const double* c2) {
  if (!ctx) return APX_EINVAL;
  if (!m || !c1 || !c2) return fail(ctx, APX_EINVAL, "model, c1 and c2 are required");
  Catalogue c;
  c.t_v = m->t_v;
  c.b1_v = m->b1_v;
  c.b2_v = m->b2_v;
  std::vector<double> r64;
  std::vector<float> r32;
  size_t o64[8], o32[8];
  fill_reals(r64, m, c, c1, c2, o64);
  fill_reals(r32, m, c, c1, c2, o32);
  if (r64.size() * sizeof(double) > m->reals64.bytes || r32.size() * sizeof(float) > m->reals32.bytes)
    return fail(ctx, APX_EINVAL, "coefficient table size changed");
  APX_HIP(ctx, hipStreamSynchronize(ctx->stream));
  APX_HIP(ctx, hipMemcpy(m->reals64.p, r64.data(), r64.size() * sizeof(double), hipMemcpyHostToDevice));
  APX_HIP(ctx, hipMemcpy(m->reals32.p, r32.data(), r32.size() * sizeof(float), hipMemcpyHostToDevice));
  const std::vector<int32_t> adj = adjoint_stream(m, c1, c2);
  APX_HIP(ctx, hipMemcpy(m->adj.p, adj.data(), adj.size() * 4, hipMemcpyHostToDevice));
  return APX_OK;
}

extern "C" apx_status apx_ace_model_stats(const apx_ace_model* m, int64_t* out6) {
  if (!m || !out6) return APX_EINVAL;
  out6[0] = m->npairs;
  out6[1] = m->ntrip;
  out6[2] = m->coupling_terms;
  out6[3] = m->triple_width;
  out6[4] = m->n_basis;
  out6[5] = m->na;
  return APX_OK;
}

extern "C" void apx_ace_model_destroy(apx_ace_model* m) {
  if (!m) return;
  (void)hipSetDevice(m->device);
  delete m;
}
