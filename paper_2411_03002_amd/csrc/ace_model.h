// ACE model: device copies of the radial mixing and the coupling tables.
#pragma once

#include "common.h"

namespace apx {

// Waves per block of the product-basis kernel: 16 for float32 (<= 128 VGPRs), 8 for
// float64 (<= 256 VGPRs).
constexpr int kAceWaves32 = 16;
constexpr int kAceWaves64 = 8;
// ints per pair record: [0] off1, [1] off2, [2] type = l1*(l_max+1)+l2, [3] n1,
// [4+L] first triple of degree L (L = 0..l_max+1, the last entry closes the list),
// [10+L] atomic-base offset of the first third block of degree L, [15] n2.
constexpr int kPairRec = 16;
// Waves per block of the unit-adjoint product kernels (float32).
constexpr int kUnitWaves = 4;
// The adjoint units are launched in groups by the degree L of their third block (group L;
// the B1/B2 units join group 0), one kernel per group, so that each kernel is
// register-allocated for its own accumulators and keeps one degree's third blocks.
constexpr int kUnitGroups = 5;
__host__ __device__ constexpr int unit_group(int L) { return L < 0 ? 0 : L; }
// ints per adjoint unit record: type, L (-1: a B1/B2 unit), first pair (B1/B2: the label
// n1), end pair, first other label, first and end entry of the unit's pair stream, end
// other label (the unit holds the pairs whose other label lies in [first, end), a range
// of at most unit_width(L, n_max) labels).
constexpr int kUnitRec = 8;
// Widest range of other labels an adjoint unit of launch group g may hold (the unit
// accumulates their adjoints in registers; narrower ranges leave registers to the larger
// third blocks of the higher degrees).
__host__ __device__ constexpr int unit_width(int g, int nmax) { return g >= 3 ? 2 : (g == 2 ? 3 : (nmax + 1) / 2); }
// Words per entry of the adjoint pair stream (float32 path): one entry per pair of a unit
// that has third blocks of the unit's degree in the unit's half, holding
// [0] off1, [1] off2, [2] run label n, [3] other label n, [4] first radial index n3 of the
// third blocks, [5..7] padding, [8 + n3] c1 and [20 + n3] c2 of the triple (n3 < 12; zero
// where there is no triple), so that a pair costs one batch of independent scalar loads.
constexpr int kAdjRec = 32;
constexpr int kAdjC1 = 8, kAdjC2 = 20;
// Unit-adjoint degrees up to which the next pair-stream entry is loaded during the current one
// (it takes 2 n_max + 4 scalar registers).
constexpr int kAdjPrefetchMaxL = 1;
// host copy of a stream entry: off1, off2, run label, other label, first n3, first triple,
// number of triples
constexpr int kAdjEnt = 7;

template <class T>
struct alignas(2 * sizeof(T)) Coef2 {
  T c1, c2;
};

// Pointers into one precision's copy of the tables.
constexpr int kTcPad = 12;  // zero coefficient pairs around the triple table (>= the largest n_max)

template <class T>
struct AceTables {
  const T* Wp;        // [l_max+1][n_max][n_max], W[l][n][k] * N_l / s_a
  const int* pairs;   // [npairs][kPairRec], sorted by type
  const int* t_v;     // [ntrip] basis index
  const Coef2<T>* tc; // [ntrip] (c1, c2) per triple, kTcPad zero entries before and after
  const int* b1_off;  // [nb1]
  const int* b1_v;
  const T* b1_c1;
  const T* b1_c2;
  const int* b2_off;  // [nb2][3]: off1, off2, l
  const int* b2_v;
  const T* b2_c1;
  const T* b2_c2;
  int npairs;
  const int* units;       // [nunits][kUnitRec]
  const int* adj_i;       // [nentries][kAdjRec] adjoint pair stream (float32 tables only)
  const float* adj_f;     // the same stream, read as coefficients
  const int* wave_units;  // [kUnitGroups][kUnitWaves + 1] offsets, then unit indices per wave
};

}  // namespace apx

struct apx_ace_model {
  int device = 0;
  int n_max = 0, l_max = 0, na = 0;
  long long n_basis = 0;
  int npairs = 0, ntrip = 0, nb1 = 0, nb2 = 0;
  long long coupling_terms = 0, triple_width = 0;  // per-atom work counts
  int group_units[apx::kUnitGroups] = {};           // adjoint units per launch group
  double r_cut = 5.0, h = 0.5, s_a = 1.0, eps = 0.1;
  int anchored = 0;
  apx_eam_params anchor{};
  apx::DevBuf ints;           // pairs, t_v, b1_off, b1_v, b2_off, b2_v, units, wave_units
  apx::DevBuf reals64, reals32;
  apx::AceTables<double> t64{};
  apx::AceTables<float> t32{};
  std::vector<double> W;      // host copy [l][n][k]
  std::vector<int> t_v, b1_v, b2_v;  // basis index of every coefficient slot (host)
  std::vector<int> adj_ent;          // adjoint stream entries, kAdjEnt ints each
  apx::DevBuf adj;                   // adjoint pair stream (kAdjRec words per entry)
};
