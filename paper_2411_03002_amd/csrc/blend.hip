// Site-weighted blend of the two potentials and a deterministic energy reduction.
//
// Sec. II A eq. energy_hyb in the precise-weight form: E_i = (1 - w_i) E_i^EAM + w_i E_i^ACE,
// the ACE term only where w_i > 0; forces are the sum of the two weighted parts
// (Appendix C eq. F_i_d); E_pot = sum_i E_i.
#include <mutex>

#include "common.h"
#include "device_util.h"

namespace apx {

constexpr int kRedThreads = 256;
constexpr int kRedPer = 8;

__global__ void __launch_bounds__(kRedThreads) k_blend(long long n, const double* __restrict__ w,
                                                       const double* __restrict__ e_eam,
                                                       const double* __restrict__ e_ace,
                                                       const double* __restrict__ f_eam,
                                                       const double* __restrict__ f_ace, double* __restrict__ e_site,
                                                       double* __restrict__ f, double* __restrict__ partial) {
  __shared__ double sh[kRedThreads];
  const long long base = (long long)blockIdx.x * kRedThreads * kRedPer;
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < kRedPer; ++k) {
    const long long i = base + (long long)k * kRedThreads + threadIdx.x;
    if (i < n) {
      const double wi = w ? w[i] : 0.0;
      double e = (1.0 - wi) * e_eam[i];
      if (wi > 0.0) e += wi * e_ace[i];
      e_site[i] = e;
      s += e;
      f[i] = f_eam[i] + f_ace[i];
      f[n + i] = f_eam[n + i] + f_ace[n + i];
      f[2 * n + i] = f_eam[2 * n + i] + f_ace[2 * n + i];
    }
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int st = kRedThreads / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

// Block partial sums of w_i e_i (w NULL: 1), reduced in the same fixed order as the blend.
__global__ void __launch_bounds__(kRedThreads) k_wsum(long long n, const double* __restrict__ w,
                                                      const double* __restrict__ e, double* __restrict__ partial) {
  __shared__ double sh[kRedThreads];
  const long long base = (long long)blockIdx.x * kRedThreads * kRedPer;
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < kRedPer; ++k) {
    const long long i = base + (long long)k * kRedThreads + threadIdx.x;
    if (i < n) s += (w ? w[i] : 1.0) * e[i];
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int st = kRedThreads / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

// Fixed-order pairwise sum of m partial values into *out (single block).
__global__ void __launch_bounds__(kRedThreads) k_sum_partials(const double* __restrict__ partial, int m,
                                                              double* __restrict__ out) {
  __shared__ double sh[kRedThreads];
  double s = 0.0;
  for (int i = threadIdx.x; i < m; i += kRedThreads) s += partial[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int st = kRedThreads / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

// Block partial sums of the blend's energy reduction for the entry point that allocates
// nothing: one double per block of kRedThreads * kRedPer atoms, so this array bounds its
// atom count at kNoAllocPartials * 2048.  Every GPU the library runs on holds its own copy
// until the process ends.
constexpr long long kNoAllocPartials = 65536;
static __device__ __align__(256) double scratch[kNoAllocPartials];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Resolves the device address of `scratch` on the context's device (current at the call)
// once per device.  Host code uses only this address: the array's own name is a host-side
// stand-in.
apx_status blend_scratch_setup(apx_ctx* ctx) {
  if (ctx->device < 0 || ctx->device >= kMaxDevices) return fail(ctx, APX_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[ctx->device]) return APX_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return fail(ctx, APX_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
  g_scratch_ptr[ctx->device] = static_cast<double*>(p);
  return APX_OK;
}

}  // namespace apx

using namespace apx;

extern "C" apx_status apx_blend(apx_ctx* ctx, int64_t n, const double* w, const double* e_eam, const double* e_ace,
                                const double* f_eam, const double* f_ace, double* e_site, double* f,
                                double* e_pot) {
  if (!ctx) return APX_EINVAL;
  if (n < 0) return fail(ctx, APX_EINVAL, "negative size");
  if (n > 0 && (!e_eam || !e_ace || !f_eam || !f_ace || !e_site || !f))
    return fail(ctx, APX_EINVAL, "blend arrays are required");
  if (!e_pot) return fail(ctx, APX_EINVAL, "e_pot is required");
  const long long nb = n > 0 ? (n + kRedThreads * kRedPer - 1) / (kRedThreads * kRedPer) : 1;
  APX_ALLOC(ctx, ctx->dtmp, sizeof(double) * (size_t)(nb + 1));
  double* part = ctx->dtmp.as<double>();
  ProfScope ps(ctx, "blend");
  if (n > 0) {
    k_blend<<<(unsigned)nb, kRedThreads, 0, ctx->stream>>>(n, w, e_eam, e_ace, f_eam, f_ace, e_site, f, part);
    APX_LAUNCH_CHECK(ctx);
    k_sum_partials<<<1, kRedThreads, 0, ctx->stream>>>(part, (int)nb, e_pot);
  } else {
    k_sum_partials<<<1, kRedThreads, 0, ctx->stream>>>(part, 0, e_pot);
  }
  APX_LAUNCH_CHECK(ctx);
  return APX_OK;
}

extern "C" apx_status apx_weighted_sum(apx_ctx* ctx, int64_t n, const double* w, const double* e, double* out) {
  if (!ctx) return APX_EINVAL;
  if (n < 0) return fail(ctx, APX_EINVAL, "negative size");
  if ((n > 0 && !e) || !out) return fail(ctx, APX_EINVAL, "e and out are required");
  const long long nb = n > 0 ? (n + kRedThreads * kRedPer - 1) / (kRedThreads * kRedPer) : 1;
  APX_ALLOC(ctx, ctx->dtmp, sizeof(double) * (size_t)(nb + 1));
  double* part = ctx->dtmp.as<double>();
  if (n > 0) {
    k_wsum<<<(unsigned)nb, kRedThreads, 0, ctx->stream>>>(n, w, e, part);
    APX_LAUNCH_CHECK(ctx);
  }
  k_sum_partials<<<1, kRedThreads, 0, ctx->stream>>>(part, n > 0 ? (int)nb : 0, out);
  APX_LAUNCH_CHECK(ctx);
  return APX_OK;
}

extern "C" apx_status apx_blend_noalloc(apx_ctx* ctx, int64_t n, const double* w, const double* e_eam,
                                        const double* e_ace, const double* f_eam, const double* f_ace,
                                        double* e_site, double* f, double* e_pot) {
  if (!ctx) return APX_EINVAL;
  if (n < 0) return fail(ctx, APX_EINVAL, "negative size");
  if (n > 0 && (!e_eam || !e_ace || !f_eam || !f_ace || !e_site || !f))
    return fail(ctx, APX_EINVAL, "blend arrays are required");
  if (!e_pot) return fail(ctx, APX_EINVAL, "e_pot is required");
  const long long per_block = (long long)kRedThreads * kRedPer;
  const long long nb = n > 0 ? (n + per_block - 1) / per_block : 0;
  if (nb > kNoAllocPartials)
    return fail(ctx, APX_EINVAL, "apx_blend_noalloc: n = %lld exceeds the limit of %lld atoms", (long long)n,
                kNoAllocPartials * per_block);
  double* part = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (ctx->device >= 0 && ctx->device < kMaxDevices) part = g_scratch_ptr[ctx->device];
  }
  if (!part) return fail(ctx, APX_EDEVICE, "scratch address of device %d was not resolved", ctx->device);
  // every partial that k_sum_partials reads is written by k_blend first: nothing to clear
  if (n > 0) {
    k_blend<<<(unsigned)nb, kRedThreads, 0, ctx->stream>>>(n, w, e_eam, e_ace, f_eam, f_ace, e_site, f, part);
    APX_LAUNCH_CHECK(ctx);
  }
  k_sum_partials<<<1, kRedThreads, 0, ctx->stream>>>(part, (int)nb, e_pot);
  APX_LAUNCH_CHECK(ctx);
  return APX_OK;
}
