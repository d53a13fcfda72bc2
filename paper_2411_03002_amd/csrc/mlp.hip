// Learned precision indicator: per-atom features, a 4-64-64-64-1 tanh network trained in
// float32 (forward, backward, Adam) and evaluated with bfloat16 MFMA, and the switch from
// its prediction to an additional detection weight.
//
// The paper lets the detection argument of its switching function be replaced by another
// criterion (Appendix B, after eq. lambda_1_i); here the network predicts
// log(|F_ACE - F_EAM| + 1e-3) from [rho_EAM, min(CSP, 50), coordination (r < 3.08 A),
// |F_EAM|] and w0_extra = 1 - f_cut((yhat - tau_lo)/(tau_hi - tau_lo)) with
// yhat = exp(prediction) - 1e-3.  Atoms whose features lie outside the training range get
// w0_extra = 0, i.e. only the centro-symmetry criterion (the fallback).
#include <cmath>
#include <cstring>

#include "common.h"
#include "device_util.h"

namespace apx {

constexpr int kH = 64;                 // hidden width
constexpr int kIn = 4;                 // inputs
constexpr int kOffW1 = 0;              // [64][4]
constexpr int kOffB1 = 256;
constexpr int kOffW2 = 320;            // [64][64]
constexpr int kOffB2 = 4416;
constexpr int kOffW3 = 4480;           // [64][64]
constexpr int kOffB3 = 8576;
constexpr int kOffW4 = 8640;           // [64]
constexpr int kOffB4 = 8704;
constexpr int kNParams = 8705;
constexpr int kSamples = 64;           // samples per training block
constexpr float kCoordR2 = 3.08f * 3.08f;

struct Std4 {
  float mu[4], sd[4];
};

}  // namespace apx

struct apx_mlp {
  int device = 0;
  apx::DevBuf buf;    // params, m, v, grad, loss, bf16 weights
  float* params = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  float* grad = nullptr;
  float* loss = nullptr;
  unsigned short* wb = nullptr;  // bf16: W1 padded [64][16], W2 [64][64], W3 [64][64], W4 [64]
  bool wb_valid = false;
  long long step = 0;
  apx::Std4 st{};
  float fmin[4] = {-INFINITY, -INFINITY, -INFINITY, -INFINITY};
  float fmax[4] = {INFINITY, INFINITY, INFINITY, INFINITY};
};

namespace apx {

// ----------------------------------------------------------------- features
__global__ void __launch_bounds__(256) k_features(const double* __restrict__ pos, int n, BoxDev b,
                                                  const int* __restrict__ count, const int* __restrict__ idx,
                                                  int max_nb, const double* __restrict__ rho,
                                                  const double* __restrict__ csp, const double* __restrict__ f,
                                                  float* __restrict__ feat) {
  const int i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double xi = pos[i], yi = pos[(size_t)n + i], zi = pos[2 * (size_t)n + i];
  int cnt = count[i];
  if (cnt > max_nb) cnt = max_nb;
  const double rc2 = 3.08 * 3.08;
  int coord = 0;
  for (int k = 0; k < cnt; ++k) {
    const int j = idx[(size_t)k * n + i];
    const double dx = min_image(pos[j] - xi, b.L[0], b.half[0], b.per[0]);
    const double dy = min_image(pos[(size_t)n + j] - yi, b.L[1], b.half[1], b.per[1]);
    const double dz = min_image(pos[2 * (size_t)n + j] - zi, b.L[2], b.half[2], b.per[2]);
    if (sq_dist_exact(dx, dy, dz) < rc2) ++coord;
  }
  const double fx = f[i], fy = f[(size_t)n + i], fz = f[2 * (size_t)n + i];
  const double c = csp[i];
  feat[4 * (size_t)i + 0] = (float)rho[i];
  feat[4 * (size_t)i + 1] = (float)(c < 50.0 ? c : 50.0);
  feat[4 * (size_t)i + 2] = (float)coord;
  feat[4 * (size_t)i + 3] = (float)sqrt(fx * fx + fy * fy + fz * fz);
}

// ------------------------------------------------- float32 forward / backward
// One block of 256 threads processes 64 samples; weights and activations live in LDS.
// With BWD the block adds its share of the gradient of the mean squared error
// (mean over `total` samples) to `grad` and its squared residuals to `loss`.
template <bool BWD>
__global__ void __launch_bounds__(256) k_mlp_pass(const float* __restrict__ feat, const float* __restrict__ target,
                                                  const int* __restrict__ sel, int nb, int total,
                                                  const float* __restrict__ P, Std4 st, float* __restrict__ grad,
                                                  float* __restrict__ loss, float* __restrict__ out) {
  __shared__ float W[kNParams];
  __shared__ float X[kSamples][kIn];
  __shared__ float H1[kSamples][kH + 1], H2[kSamples][kH + 1], H3[kSamples][kH + 1];
  __shared__ float dY[kSamples];
  const int tid = threadIdx.x;
  const int s0 = blockIdx.x * kSamples;
  for (int e = tid; e < kNParams; e += 256) W[e] = P[e];
  {
    const int s = tid >> 2, c = tid & 3;
    const int g = s0 + s;
    float x = 0.f;
    if (g < nb) {
      const int id = sel ? sel[g] : g;
      x = (feat[4 * (size_t)id + c] - st.mu[c]) / st.sd[c];
    }
    X[s][c] = x;
  }
  __syncthreads();
  for (int o = tid; o < kSamples * kH; o += 256) {
    const int s = o / kH, j = o % kH;
    float z = W[kOffB1 + j];
#pragma unroll
    for (int k = 0; k < kIn; ++k) z = fmaf(W[kOffW1 + j * kIn + k], X[s][k], z);
    H1[s][j] = tanhf(z);
  }
  __syncthreads();
  for (int o = tid; o < kSamples * kH; o += 256) {
    const int s = o / kH, j = o % kH;
    float z = W[kOffB2 + j];
    for (int k = 0; k < kH; ++k) z = fmaf(W[kOffW2 + j * kH + k], H1[s][k], z);
    H2[s][j] = tanhf(z);
  }
  __syncthreads();
  for (int o = tid; o < kSamples * kH; o += 256) {
    const int s = o / kH, j = o % kH;
    float z = W[kOffB3 + j];
    for (int k = 0; k < kH; ++k) z = fmaf(W[kOffW3 + j * kH + k], H2[s][k], z);
    H3[s][j] = tanhf(z);
  }
  __syncthreads();
  if (tid < kSamples) {
    const int g = s0 + tid;
    float y = W[kOffB4];
    for (int k = 0; k < kH; ++k) y = fmaf(W[kOffW4 + k], H3[tid][k], y);
    float d = 0.f, r2 = 0.f;
    if (g < nb) {
      if (out) out[g] = y;
      if (BWD) {
        const int id = sel ? sel[g] : g;
        const float r = y - target[id];
        d = 2.f * r / (float)total;
        r2 = r * r;
      }
    }
    dY[tid] = d;
    if (BWD) {
      r2 = wave_sum(r2);
      if (tid == 0) atomicAdd(loss, r2 / (float)total);
    }
  }
  if (!BWD) return;
  __syncthreads();
  // output layer
  if (tid < kH) {
    float g = 0.f;
    for (int s = 0; s < kSamples; ++s) g = fmaf(dY[s], H3[s][tid], g);
    atomicAdd(&grad[kOffW4 + tid], g);
  }
  if (tid == kH) {
    float g = 0.f;
    for (int s = 0; s < kSamples; ++s) g += dY[s];
    atomicAdd(&grad[kOffB4], g);
  }
  __syncthreads();
  // delta3 in place of H3
  for (int o = tid; o < kSamples * kH; o += 256) {
    const int s = o / kH, j = o % kH;
    const float h = H3[s][j];
    H3[s][j] = dY[s] * W[kOffW4 + j] * (1.f - h * h);
  }
  __syncthreads();
  for (int o = tid; o < kH * kH; o += 256) {
    const int j = o / kH, k = o % kH;
    float g = 0.f;
    for (int s = 0; s < kSamples; ++s) g = fmaf(H3[s][j], H2[s][k], g);
    atomicAdd(&grad[kOffW3 + o], g);
  }
  if (tid < kH) {
    float g = 0.f;
    for (int s = 0; s < kSamples; ++s) g += H3[s][tid];
    atomicAdd(&grad[kOffB3 + tid], g);
  }
  __syncthreads();
  // delta2 in place of H2
  for (int o = tid; o < kSamples * kH; o += 256) {
    const int s = o / kH, k = o % kH;
    float a = 0.f;
    for (int j = 0; j < kH; ++j) a = fmaf(H3[s][j], W[kOffW3 + j * kH + k], a);
    const float h = H2[s][k];
    H2[s][k] = a * (1.f - h * h);
  }
  __syncthreads();
  for (int o = tid; o < kH * kH; o += 256) {
    const int j = o / kH, k = o % kH;
    float g = 0.f;
    for (int s = 0; s < kSamples; ++s) g = fmaf(H2[s][j], H1[s][k], g);
    atomicAdd(&grad[kOffW2 + o], g);
  }
  if (tid < kH) {
    float g = 0.f;
    for (int s = 0; s < kSamples; ++s) g += H2[s][tid];
    atomicAdd(&grad[kOffB2 + tid], g);
  }
  __syncthreads();
  // delta1 in place of H1
  for (int o = tid; o < kSamples * kH; o += 256) {
    const int s = o / kH, k = o % kH;
    float a = 0.f;
    for (int j = 0; j < kH; ++j) a = fmaf(H2[s][j], W[kOffW2 + j * kH + k], a);
    const float h = H1[s][k];
    H1[s][k] = a * (1.f - h * h);
  }
  __syncthreads();
  {
    const int j = tid >> 2, c = tid & 3;  // 256 = 64 x 4 weights of layer 1
    float g = 0.f;
    for (int s = 0; s < kSamples; ++s) g = fmaf(H1[s][j], X[s][c], g);
    atomicAdd(&grad[kOffW1 + j * kIn + c], g);
  }
  if (tid < kH) {
    float g = 0.f;
    for (int s = 0; s < kSamples; ++s) g += H1[s][tid];
    atomicAdd(&grad[kOffB1 + tid], g);
  }
}

// Adam with bias correction; clears the gradient for the next step.
__global__ void k_adam(float* __restrict__ p, float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       int np, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / c1, vh = vi / c2;
  p[i] = p[i] - lr * mh / (sqrtf(vh) + eps);
  g[i] = 0.f;
}

__global__ void k_zero_f(float* __restrict__ p, int m) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) p[i] = 0.f;
}

// --------------------------------------------------------- bfloat16 inference
__device__ __forceinline__ unsigned short bf16_rne(float x) {
  unsigned u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40);  // quiet NaN
  const unsigned lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (unsigned short)(u >> 16);
}

__device__ __forceinline__ float bf16_to_f(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

__global__ void k_pack_bf16(const float* __restrict__ P, unsigned short* __restrict__ wb) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  // W1 padded to [64][16]
  if (e < kH * 16) {
    const int j = e / 16, k = e % 16;
    wb[e] = k < kIn ? bf16_rne(P[kOffW1 + j * kIn + k]) : (unsigned short)0;
  }
  if (e < kH * kH) {
    wb[kH * 16 + e] = bf16_rne(P[kOffW2 + e]);
    wb[kH * 16 + kH * kH + e] = bf16_rne(P[kOffW3 + e]);
  }
  if (e < kH) wb[kH * 16 + 2 * kH * kH + e] = bf16_rne(P[kOffW4 + e]);
}

typedef short v8s __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4f mfma_bf16_16x16x32(v8s a, v8s b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a), __builtin_bit_cast(v8bf, b), c, 0, 0, 0);
}

// One wave evaluates 16 atoms: every hidden layer is a [16 x K] x [K x 64] product on the
// 16x16x32 bfloat16 matrix cores of gfx950 (four output tiles, K/32 steps; lane = row or
// column (lane % 16) and a group of eight K values (lane / 16)), bias + tanh in float32,
// the activations rounded to bfloat16 in LDS for the next layer.
__global__ void __launch_bounds__(256) k_mlp_bf16(const float* __restrict__ feat, int n, const float* __restrict__ P,
                                                  const unsigned short* __restrict__ wb, Std4 st,
                                                  float* __restrict__ out) {
  __shared__ unsigned short act[4][16][kH + 8];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int a0 = (blockIdx.x * 4 + wv) * 16;
  const int ri = lane & 15;   // row (atom) of A, column (neuron) of B and D
  const int kq = lane >> 4;   // k quad
  // inputs, standardised and rounded, K padded to 32 (the weights hold 16 columns)
  {
    v8s a;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int k = 8 * kq + r;
      float x = 0.f;
      if (k < kIn && a0 + ri < n) x = (feat[4 * (size_t)(a0 + ri) + k] - st.mu[k]) / st.sd[k];
      a[r] = (short)bf16_rne(x);
    }
    const unsigned short* W1 = wb;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      v8s bv;
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int k = 8 * kq + r;
        bv[r] = k < 16 ? (short)W1[(nt * 16 + ri) * 16 + k] : (short)0;
      }
      v4f c = {0.f, 0.f, 0.f, 0.f};
      c = mfma_bf16_16x16x32(a, bv, c);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = nt * 16 + ri;
        act[wv][4 * kq + r][j] = bf16_rne(tanhf(c[r] + P[kOffB1 + j]));
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int layer = 0; layer < 2; ++layer) {
    const unsigned short* Wl = wb + kH * 16 + layer * kH * kH;
    const float* bias = P + (layer == 0 ? kOffB2 : kOffB3);
    v4f c[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) c[nt] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < kH / 32; ++ks) {
      v8s a;
#pragma unroll
      for (int r = 0; r < 8; ++r) a[r] = (short)act[wv][ri][32 * ks + 8 * kq + r];
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        v8s bv;
#pragma unroll
        for (int r = 0; r < 8; ++r) bv[r] = (short)Wl[(nt * 16 + ri) * kH + 32 * ks + 8 * kq + r];
        c[nt] = mfma_bf16_16x16x32(a, bv, c[nt]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = nt * 16 + ri;
        act[wv][4 * kq + r][j] = bf16_rne(tanhf(c[nt][r] + bias[j]));
      }
    __syncthreads();
  }
  if (lane < 16 && a0 + lane < n) {
    const unsigned short* W4 = wb + kH * 16 + 2 * kH * kH;
    float y = P[kOffB4];
    for (int k = 0; k < kH; ++k) y = fmaf(bf16_to_f(W4[k]), bf16_to_f(act[wv][lane][k]), y);
    out[a0 + lane] = y;
  }
}

// prediction -> additional detection weight, with the range fallback
__global__ void k_mlp_w0(const float* __restrict__ pred, const float* __restrict__ feat, int n, double tau_lo,
                         double width, Std4 lims_lo, Std4 lims_hi, double* __restrict__ w0) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  bool in_range = true;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const float f = feat[4 * (size_t)i + c];
    if (!(f >= lims_lo.mu[c] && f <= lims_hi.mu[c])) in_range = false;
  }
  double w = 0.0;
  if (in_range) {
    const double dF = exp((double)pred[i]) - 1e-3;
    w = 1.0 - fcut_exact((dF - tau_lo) / width);
  }
  w0[i] = w;
}

// Training labels: dF_i = |F^precise_i - F^fast_i| (float64), label_i = log(dF_i + 1e-3)
// rounded to float32.
__global__ void k_mlp_labels(long long n, const double* __restrict__ fp, const double* __restrict__ ff,
                             double* __restrict__ dF, float* __restrict__ label) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double dx = fp[i] - ff[i], dy = fp[n + i] - ff[n + i], dz = fp[2 * n + i] - ff[2 * n + i];
  const double d = sqrt(dx * dx + dy * dy + dz * dz);
  if (dF) dF[i] = d;
  label[i] = (float)log(d + 1e-3);
}

// Column statistics of the [n][4] float32 features, one block per column, float64 sums
// reduced in a fixed order: out[c] mean, out[4 + c] standard deviation with n - 1,
// out[8 + c] minimum, out[12 + c] maximum.
constexpr int kStatThreads = 1024;
__global__ void __launch_bounds__(kStatThreads) k_feature_stats(const float* __restrict__ feat, long long n,
                                                                double* __restrict__ out) {
  __shared__ double sh[kStatThreads / kWave];
  __shared__ double shm[kStatThreads / kWave], shx[kStatThreads / kWave];
  const int c = blockIdx.x;
  const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  double s = 0.0, mn = INFINITY, mx = -INFINITY;
  for (long long i = threadIdx.x; i < n; i += kStatThreads) {
    const double v = (double)feat[4 * i + c];
    s += v;
    mn = v < mn ? v : mn;
    mx = v > mx ? v : mx;
  }
  s = wave_sum(s);
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    const double a = __shfl_xor(mn, off, kWave), b = __shfl_xor(mx, off, kWave);
    mn = a < mn ? a : mn;
    mx = b > mx ? b : mx;
  }
  if (lane == 0) {
    sh[w] = s;
    shm[w] = mn;
    shx[w] = mx;
  }
  __syncthreads();
  double tot = 0.0, tmin = INFINITY, tmax = -INFINITY;
  for (int k = 0; k < kStatThreads / kWave; ++k) {
    tot += sh[k];
    tmin = shm[k] < tmin ? shm[k] : tmin;
    tmax = shx[k] > tmax ? shx[k] : tmax;
  }
  const double mean = n > 0 ? tot / (double)n : 0.0;
  __syncthreads();
  double q = 0.0;
  for (long long i = threadIdx.x; i < n; i += kStatThreads) {
    const double d = (double)feat[4 * i + c] - mean;
    q += d * d;
  }
  q = wave_sum(q);
  if (lane == 0) sh[w] = q;
  __syncthreads();
  if (threadIdx.x == 0) {
    double qq = 0.0;
    for (int k = 0; k < kStatThreads / kWave; ++k) qq += sh[k];
    out[c] = mean;
    out[4 + c] = n > 1 ? sqrt(qq / (double)(n - 1)) : 0.0;
    out[8 + c] = tmin;
    out[12 + c] = tmax;
  }
}

}  // namespace apx

using namespace apx;

extern "C" {

apx_status apx_mlp_labels(apx_ctx* ctx, int64_t n, const double* f_precise, const double* f_fast, double* dF,
                          float* label) {
  if (!ctx) return APX_EINVAL;
  if (n < 0) return fail(ctx, APX_EINVAL, "negative size");
  if (n > 0 && (!f_precise || !f_fast || !label)) return fail(ctx, APX_EINVAL, "forces and label are required");
  if (n == 0) return APX_OK;
  k_mlp_labels<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(n, f_precise, f_fast, dF, label);
  APX_LAUNCH_CHECK(ctx);
  return APX_OK;
}

apx_status apx_mlp_feature_stats(apx_ctx* ctx, const float* feat, int64_t n, double* stats) {
  if (!ctx) return APX_EINVAL;
  if (n < 1 || !feat || !stats) return fail(ctx, APX_EINVAL, "features (n >= 1) and stats are required");
  k_feature_stats<<<4, kStatThreads, 0, ctx->stream>>>(feat, n, stats);
  APX_LAUNCH_CHECK(ctx);
  return APX_OK;
}

apx_status apx_mlp_create(apx_ctx* ctx, const float* params, const float* mu, const float* sd, apx_mlp** out) {
  if (!ctx) return APX_EINVAL;
  if (!params || !mu || !sd || !out) return fail(ctx, APX_EINVAL, "params, mu, sd and out are required");
  *out = nullptr;
  for (int c = 0; c < 4; ++c)
    if (!(sd[c] > 0.f)) return fail(ctx, APX_EINVAL, "standard deviations must be positive");
  apx_mlp* m = new apx_mlp();
  m->device = ctx->device;
  const size_t nf = 4 * (size_t)kNParams + 64;
  const size_t nwb = kH * 16 + 2 * kH * kH + kH;
  if (m->buf.ensure(nf * sizeof(float) + nwb * sizeof(unsigned short)) != hipSuccess) {
    delete m;
    return fail(ctx, APX_ENOMEM, "MLP buffers");
  }
  float* base = m->buf.as<float>();
  m->params = base;
  m->m = base + kNParams;
  m->v = base + 2 * kNParams;
  m->grad = base + 3 * kNParams;
  m->loss = base + 4 * kNParams;
  m->wb = reinterpret_cast<unsigned short*>(base + nf);
  for (int c = 0; c < 4; ++c) {
    m->st.mu[c] = mu[c];
    m->st.sd[c] = sd[c];
  }
  if (hipMemcpy(m->params, params, kNParams * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(m->m, 0, 3 * (size_t)kNParams * sizeof(float) + 64 * sizeof(float)) != hipSuccess) {
    delete m;
    return fail(ctx, APX_EDEVICE, "MLP upload");
  }
  *out = m;
  return APX_OK;
}

void apx_mlp_destroy(apx_mlp* m) {
  if (!m) return;
  (void)hipSetDevice(m->device);
  delete m;
}

apx_status apx_mlp_get_params(apx_ctx* ctx, const apx_mlp* m, float* params) {
  if (!ctx || !m || !params) return APX_EINVAL;
  APX_HIP(ctx, hipMemcpyAsync(params, m->params, kNParams * sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
  APX_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return APX_OK;
}

apx_status apx_mlp_set_range(apx_mlp* m, const float* fmin, const float* fmax) {
  if (!m || !fmin || !fmax) return APX_EINVAL;
  for (int c = 0; c < 4; ++c) {
    m->fmin[c] = fmin[c];
    m->fmax[c] = fmax[c];
  }
  return APX_OK;
}

apx_status apx_features(apx_ctx* ctx, const apx_atoms* atoms, const apx_nlist* nl, const double* rho,
                        const double* csp, const double* f_eam, float* feat) {
  if (!ctx) return APX_EINVAL;
  apx_status s = check_atoms(ctx, atoms);
  if (s != APX_OK) return s;
  if (!nl || nl->n != atoms->n) return fail(ctx, APX_EINVAL, "nlist mismatch");
  if (nl->r_list < 3.08) return fail(ctx, APX_EINVAL, "neighbour list shorter than the coordination radius");
  const int n = (int)atoms->n;
  if (n == 0) return APX_OK;
  if (!rho || !csp || !f_eam || !feat) return fail(ctx, APX_EINVAL, "feature inputs are required");
  ProfScope ps(ctx, "mlp.features");
  k_features<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(atoms->pos, n, make_box(atoms), nl->count, nl->idx,
                                                         nl->max_nb, rho, csp, f_eam, feat);
  APX_LAUNCH_CHECK(ctx);
  return APX_OK;
}

apx_status apx_mlp_forward(apx_ctx* ctx, const apx_mlp* m, const float* feat, int64_t n, float* out) {
  if (!ctx || !m) return APX_EINVAL;
  if (n < 0 || n > 0x7fffffff) return fail(ctx, APX_EINVAL, "bad sample count");
  if (n == 0) return APX_OK;
  if (!feat || !out) return fail(ctx, APX_EINVAL, "feat and out are required");
  k_mlp_pass<false><<<blocks_for(n, kSamples), 256, 0, ctx->stream>>>(feat, nullptr, nullptr, (int)n, (int)n,
                                                                      m->params, m->st, nullptr, nullptr, out);
  APX_LAUNCH_CHECK(ctx);
  return APX_OK;
}

apx_status apx_mlp_gradients(apx_ctx* ctx, apx_mlp* m, const float* feat, const float* target, const int32_t* sel,
                             int64_t nb, float* grad, float* loss) {
  if (!ctx || !m) return APX_EINVAL;
  if (nb <= 0 || nb > 0x7fffffff) return fail(ctx, APX_EINVAL, "batch size must be positive");
  if (!feat || !target || !grad || !loss) return fail(ctx, APX_EINVAL, "feat, target, grad and loss are required");
  k_zero_f<<<blocks_for(kNParams, 256), 256, 0, ctx->stream>>>(grad, kNParams);
  k_zero_f<<<1, 64, 0, ctx->stream>>>(loss, 1);
  ProfScope ps(ctx, "mlp.train");
  k_mlp_pass<true><<<blocks_for(nb, kSamples), 256, 0, ctx->stream>>>(feat, target, sel, (int)nb, (int)nb,
                                                                     m->params, m->st, grad, loss, nullptr);
  APX_LAUNCH_CHECK(ctx);
  return APX_OK;
}

apx_status apx_mlp_adam_step(apx_ctx* ctx, apx_mlp* m, const float* grad, float lr, float beta1, float beta2,
                             float eps) {
  if (!ctx || !m || !grad) return APX_EINVAL;
  m->step += 1;
  const float c1 = 1.f - powf(beta1, (float)m->step), c2 = 1.f - powf(beta2, (float)m->step);
  k_adam<<<blocks_for(kNParams, 256), 256, 0, ctx->stream>>>(m->params, const_cast<float*>(grad), m->m, m->v,
                                                             kNParams, lr, beta1, beta2, eps, c1, c2);
  APX_LAUNCH_CHECK(ctx);
  m->wb_valid = false;
  return APX_OK;
}

apx_status apx_mlp_train_step(apx_ctx* ctx, apx_mlp* m, const float* feat, const float* target, const int32_t* sel,
                              int64_t nb, float lr, float* loss) {
  if (!ctx || !m) return APX_EINVAL;
  if (nb <= 0 || nb > 0x7fffffff) return fail(ctx, APX_EINVAL, "batch size must be positive");
  if (!feat || !target) return fail(ctx, APX_EINVAL, "feat and target are required");
  float* ls = loss ? loss : m->loss;
  k_zero_f<<<1, 64, 0, ctx->stream>>>(ls, 1);
  {
    ProfScope ps(ctx, "mlp.train");
    k_mlp_pass<true><<<blocks_for(nb, kSamples), 256, 0, ctx->stream>>>(feat, target, sel, (int)nb, (int)nb,
                                                                       m->params, m->st, m->grad, ls, nullptr);
    APX_LAUNCH_CHECK(ctx);
  }
  return apx_mlp_adam_step(ctx, m, m->grad, lr, 0.9f, 0.999f, 1e-8f);
}

apx_status apx_mlp_infer_bf16(apx_ctx* ctx, apx_mlp* m, const float* feat, int64_t n, float* out) {
  if (!ctx || !m) return APX_EINVAL;
  if (n < 0 || n > 0x7fffffff) return fail(ctx, APX_EINVAL, "bad sample count");
  if (!m->wb_valid) {
    k_pack_bf16<<<blocks_for(kH * kH, 256), 256, 0, ctx->stream>>>(m->params, m->wb);
    APX_LAUNCH_CHECK(ctx);
    m->wb_valid = true;
  }
  if (n == 0) return APX_OK;
  if (!feat || !out) return fail(ctx, APX_EINVAL, "feat and out are required");
  ProfScope ps(ctx, "mlp.infer_bf16");
  k_mlp_bf16<<<blocks_for(n, 64), 256, 0, ctx->stream>>>(feat, (int)n, m->params, m->wb, m->st, out);
  APX_LAUNCH_CHECK(ctx);
  return APX_OK;
}

apx_status apx_mlp_weight(apx_ctx* ctx, const apx_mlp* m, const float* pred, const float* feat, int64_t n,
                          double tau_lo, double tau_hi, double* w0_extra) {
  if (!ctx || !m) return APX_EINVAL;
  if (!(tau_hi > tau_lo)) return fail(ctx, APX_EINVAL, "tau_hi must exceed tau_lo");
  if (n < 0 || n > 0x7fffffff) return fail(ctx, APX_EINVAL, "bad sample count");
  if (n > 0 && (!pred || !feat || !w0_extra)) return fail(ctx, APX_EINVAL, "pred, feat and w0_extra are required");
  if (n == 0) return APX_OK;
  Std4 lo, hi;
  for (int c = 0; c < 4; ++c) {
    lo.mu[c] = m->fmin[c];
    hi.mu[c] = m->fmax[c];
    lo.sd[c] = hi.sd[c] = 0.f;
  }
  k_mlp_w0<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(pred, feat, (int)n, tau_lo, tau_hi - tau_lo, lo, hi, w0_extra);
  APX_LAUNCH_CHECK(ctx);
  return APX_OK;
}

apx_status apx_mlp_precision(apx_ctx* ctx, apx_mlp* m, const float* feat, int64_t n, double tau_lo, double tau_hi,
                             float* pred, double* w0_extra) {
  if (!ctx || !m) return APX_EINVAL;
  if (!(tau_hi > tau_lo)) return fail(ctx, APX_EINVAL, "tau_hi must exceed tau_lo");
  if (n > 0 && (!pred || !w0_extra)) return fail(ctx, APX_EINVAL, "pred and w0_extra are required");
  apx_status s = apx_mlp_infer_bf16(ctx, m, feat, n, pred);
  if (s != APX_OK || n == 0) return s;
  return apx_mlp_weight(ctx, m, pred, feat, n, tau_lo, tau_hi, w0_extra);
}

}  // extern "C"
