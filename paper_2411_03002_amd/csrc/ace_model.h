// ACE model: device copies of the radial mixing and the coupling tables.
#pragma once

#include "common.h"

namespace apx {

constexpr int kAceWaves = 8;     // waves per block in the product-basis kernel
constexpr int kPairRec = 12;     // ints per pair record: off1, off2, type, pad, tb[8]

// Pointers into one precision's copy of the tables.
template <class T>
struct AceTables {
  const T* Wp;        // [l_max+1][n_max][n_max], W[l][n][k] * N_l / s_a
  const int* pairs;   // [npairs][kPairRec]
  const int* t_off;   // [ntrip] A offset of the third block
  const int* t_v;     // [ntrip] basis index
  const T* t_c1;      // [ntrip]
  const T* t_c2;
  const int* b1_off;  // [nb1]
  const int* b1_v;
  const T* b1_c1;
  const T* b1_c2;
  const int* b2_off;  // [nb2][3]: off1, off2, l
  const int* b2_v;
  const T* b2_c1;
  const T* b2_c2;
  const int* split;   // [kAceWaves + 1] pair ranges per wave
};

}  // namespace apx

struct apx_ace_model {
  int device = 0;
  int n_max = 0, l_max = 0, na = 0;
  long long n_basis = 0;
  int npairs = 0, ntrip = 0, nb1 = 0, nb2 = 0;
  double r_cut = 5.0, h = 0.5, s_a = 1.0, eps = 0.1;
  int anchored = 0;
  apx_eam_params anchor{};
  apx::DevBuf ints;           // pairs, t_off, t_v, b1_off, b1_v, b2_off, b2_v, split
  apx::DevBuf reals64, reals32;
  apx::AceTables<double> t64{};
  apx::AceTables<float> t32{};
  std::vector<double> W;      // host copy [l][n][k]
};
