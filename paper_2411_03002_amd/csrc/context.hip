// Context, error reporting, cell binning and prefix scans.
#include <cmath>
#include <cstring>

#include "common.h"
#include "device_util.h"

namespace apx {

apx_status fail(apx_ctx* ctx, apx_status code, const char* fmt, ...) {
  if (ctx) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return code;
}

apx_status check_atoms(apx_ctx* ctx, const apx_atoms* a) {
  if (!a) return fail(ctx, APX_EINVAL, "atoms is NULL");
  if (a->n < 0 || a->n > (int64_t)0x7fffffff) return fail(ctx, APX_EINVAL, "bad atom count %lld", (long long)a->n);
  if (a->n > 0 && !a->pos) return fail(ctx, APX_EINVAL, "atoms->pos is NULL");
  for (int d = 0; d < 3; ++d) {
    if (!(a->hi[d] > a->lo[d]) || !std::isfinite(a->hi[d] - a->lo[d]))
      return fail(ctx, APX_EINVAL, "box dimension %d is empty or not finite", d);
  }
  return APX_OK;
}

Grid make_grid(const apx_atoms* a, double min_cell) {
  Grid g;
  for (int d = 0; d < 3; ++d) {
    g.lo[d] = a->lo[d];
    g.L[d] = a->hi[d] - a->lo[d];
    g.per[d] = a->periodic[d] ? 1 : 0;
    long long nc = (long long)std::floor(g.L[d] / min_cell);
    if (nc < 1) nc = 1;
    if (nc > 1024) nc = 1024;
    g.nc[d] = (int)nc;
    g.inv_cell[d] = (double)nc / g.L[d];
  }
  return g;
}

// ------------------------------------------------------------------- binning
__global__ void k_bin_count(const double* __restrict__ pos, int n, Grid g, int* __restrict__ cell_id,
                            int* __restrict__ counts, int* __restrict__ flags) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int c[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double x = pos[(size_t)d * n + i];
    double t = (x - g.lo[d]) * g.inv_cell[d];
    if (!(t >= 0.0 && t < (double)g.nc[d] + 1e-9) && !g.per[d]) atomicOr(&flags[0], 1);
    if (!(x == x)) atomicOr(&flags[0], 2);
    c[d] = cell_coord(x, g.lo[d], g.inv_cell[d], g.nc[d]);
  }
  int id = c[0] + g.nc[0] * (c[1] + g.nc[1] * c[2]);
  cell_id[i] = id;
  atomicAdd(&counts[id], 1);
}

__global__ void k_bin_fill(int n, const int* __restrict__ cell_id, const int* __restrict__ start,
                           int* __restrict__ fill, int* __restrict__ atoms) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int c = cell_id[i];
  int slot = atomicAdd(&fill[c], 1);
  atoms[start[c] + slot] = i;
}

apx_status bin_atoms(apx_ctx* ctx, const apx_atoms* a, const Grid& g) {
  int n = (int)a->n;
  long long nc = g.ncell();
  APX_ALLOC(ctx, ctx->cell_id, sizeof(int) * (size_t)(n > 0 ? n : 1));
  APX_ALLOC(ctx, ctx->cell_count, sizeof(int) * (size_t)nc);
  APX_ALLOC(ctx, ctx->cell_start, sizeof(int) * (size_t)(nc + 1));
  APX_ALLOC(ctx, ctx->cell_fill, sizeof(int) * (size_t)nc);
  APX_ALLOC(ctx, ctx->cell_atoms, sizeof(int) * (size_t)(n > 0 ? n : 1));
  APX_ALLOC(ctx, ctx->flags, sizeof(int) * 4);
  APX_HIP(ctx, hipMemsetAsync(ctx->cell_count.p, 0, sizeof(int) * nc, ctx->stream));
  APX_HIP(ctx, hipMemsetAsync(ctx->cell_fill.p, 0, sizeof(int) * nc, ctx->stream));
  APX_HIP(ctx, hipMemsetAsync(ctx->flags.p, 0, sizeof(int) * 4, ctx->stream));
  if (n > 0) {
    k_bin_count<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(a->pos, n, g, ctx->cell_id.as<int>(),
                                                            ctx->cell_count.as<int>(), ctx->flags.as<int>());
    APX_LAUNCH_CHECK(ctx);
  }
  apx_status s = scan_exclusive(ctx, ctx->cell_count.as<int>(), nc, ctx->cell_start.as<int>());
  if (s != APX_OK) return s;
  if (n > 0) {
    k_bin_fill<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(n, ctx->cell_id.as<int>(), ctx->cell_start.as<int>(),
                                                           ctx->cell_fill.as<int>(), ctx->cell_atoms.as<int>());
    APX_LAUNCH_CHECK(ctx);
  }
  return APX_OK;
}

// --------------------------------------------------------------------- scans
constexpr int kScanThreads = 1024;
constexpr int kScanPer = 4;
constexpr int kScanChunk = kScanThreads * kScanPer;

// Block-wide exclusive scan of one value per thread; returns the block total in *total.
__device__ int block_exclusive_scan(int v, int* sh_waves, int* total) {
  int lane = threadIdx.x & (kWave - 1);
  int wid = threadIdx.x / kWave;
  int incl = v;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    int o = __shfl_up(incl, off, kWave);
    if (lane >= off) incl += o;
  }
  if (lane == kWave - 1) sh_waves[wid] = incl;
  __syncthreads();
  int nw = blockDim.x / kWave;
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int w = 0; w < nw; ++w) {
      int t = sh_waves[w];
      sh_waves[w] = acc;
      acc += t;
    }
    sh_waves[nw] = acc;
  }
  __syncthreads();
  int res = sh_waves[wid] + incl - v;
  *total = sh_waves[nw];
  __syncthreads();
  return res;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(const int* __restrict__ in, long long m,
                                                              int* __restrict__ block_sums) {
  __shared__ int sh[kScanThreads / kWave + 1];
  long long base = (long long)blockIdx.x * kScanChunk + (long long)threadIdx.x * kScanPer;
  int s = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k)
    if (base + k < m) s += in[base + k];
  int tot;
  block_exclusive_scan(s, sh, &tot);
  if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_sums(int* __restrict__ sums, int nb, int* __restrict__ total) {
  __shared__ int sh[kScanThreads / kWave + 1];
  int carry = 0;
  for (int b0 = 0; b0 < nb; b0 += kScanThreads) {
    int i = b0 + threadIdx.x;
    int v = i < nb ? sums[i] : 0;
    int tot;
    int ex = block_exclusive_scan(v, sh, &tot);
    if (i < nb) sums[i] = ex + carry;
    carry += tot;
  }
  if (threadIdx.x == 0) *total = carry;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_apply(const int* __restrict__ in, long long m,
                                                             const int* __restrict__ block_off, int* __restrict__ out) {
  __shared__ int sh[kScanThreads / kWave + 1];
  long long base = (long long)blockIdx.x * kScanChunk + (long long)threadIdx.x * kScanPer;
  int vals[kScanPer];
  int s = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    vals[k] = (base + k < m) ? in[base + k] : 0;
    s += vals[k];
  }
  int tot;
  int ex = block_exclusive_scan(s, sh, &tot) + block_off[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    if (base + k < m) out[base + k] = ex;
    ex += vals[k];
  }
}

apx_status scan_exclusive(apx_ctx* ctx, const int* in, long long m, int* out) {
  long long nb = (m + kScanChunk - 1) / kScanChunk;
  if (nb < 1) nb = 1;
  APX_ALLOC(ctx, ctx->scan_tmp, sizeof(int) * (size_t)(nb + 1));
  int* sums = ctx->scan_tmp.as<int>();
  if (m > 0) {
    k_scan_reduce<<<(unsigned)nb, kScanThreads, 0, ctx->stream>>>(in, m, sums);
    APX_LAUNCH_CHECK(ctx);
  } else {
    APX_HIP(ctx, hipMemsetAsync(sums, 0, sizeof(int), ctx->stream));
  }
  k_scan_sums<<<1, kScanThreads, 0, ctx->stream>>>(sums, (int)nb, out + m);
  APX_LAUNCH_CHECK(ctx);
  if (m > 0) {
    k_scan_apply<<<(unsigned)nb, kScanThreads, 0, ctx->stream>>>(in, m, sums, out);
    APX_LAUNCH_CHECK(ctx);
  }
  return APX_OK;
}

apx_status read_ints(apx_ctx* ctx, const int* dev, int* host, int count) {
  if (count > 64) return fail(ctx, APX_EINVAL, "read_ints: too many values");
  APX_HIP(ctx, hipMemcpyAsync(ctx->host_pinned, dev, sizeof(int) * count, hipMemcpyDeviceToHost, ctx->stream));
  APX_HIP(ctx, hipStreamSynchronize(ctx->stream));
  std::memcpy(host, ctx->host_pinned, sizeof(int) * count);
  return APX_OK;
}

int prof_id(apx_ctx* ctx, const char* name) {
  for (size_t k = 0; k < ctx->prof_stats.size(); ++k)
    if (ctx->prof_stats[k].name == name) return (int)k;
  ctx->prof_stats.push_back(ProfStat{name, 0, 0.0});
  return (int)ctx->prof_stats.size() - 1;
}

hipEvent_t prof_event(apx_ctx* ctx) {
  if (!ctx->prof_pool.empty()) {
    hipEvent_t e = ctx->prof_pool.back();
    ctx->prof_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Accumulates completed event pairs (all of them when `wait`).
void prof_flush(apx_ctx* ctx, bool wait) {
  if (ctx->prof_pending.empty()) return;
  if (wait) (void)hipStreamSynchronize(ctx->stream);
  size_t keep = 0;
  for (size_t k = 0; k < ctx->prof_pending.size(); ++k) {
    ProfPending& p = ctx->prof_pending[k];
    if (!wait && hipEventQuery(p.b) != hipSuccess) {
      ctx->prof_pending[keep++] = p;
      continue;
    }
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      ctx->prof_stats[p.id].ms += ms;
      ctx->prof_stats[p.id].launches += 1;
    }
    ctx->prof_pool.push_back(p.a);
    ctx->prof_pool.push_back(p.b);
  }
  ctx->prof_pending.resize(keep);
}

__global__ void k_fp64_functions(long long n, const double* __restrict__ x, double* __restrict__ e,
                                 double* __restrict__ rc, double* __restrict__ rs) {
  __shared__ double etab[32];
  stage_exp_table(etab);
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = x[i];
  if (e) e[i] = exp_tab(v, etab);
  if (rc) rc[i] = rcp_nr(v);
  if (rs) rs[i] = rsq_nr(v);
}

}  // namespace apx

using namespace apx;

extern "C" {

apx_status apx_fp64_functions(apx_ctx* ctx, int64_t n, const double* x, double* exp_out, double* rcp_out,
                              double* rsq_out) {
  if (!ctx) return APX_EINVAL;
  if (n < 0 || (n > 0 && !x)) return fail(ctx, APX_EINVAL, "x is required");
  if (n == 0) return APX_OK;
  k_fp64_functions<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(n, x, exp_out, rcp_out, rsq_out);
  APX_LAUNCH_CHECK(ctx);
  return APX_OK;
}

apx_status apx_profile_enable(apx_ctx* ctx, int32_t on) {
  if (!ctx) return APX_EINVAL;
  prof_flush(ctx, true);
  ctx->prof_stats.clear();
  ctx->prof = on != 0;
  return APX_OK;
}

int32_t apx_profile_count(apx_ctx* ctx) {
  if (!ctx) return APX_EINVAL;
  prof_flush(ctx, true);
  return (int32_t)ctx->prof_stats.size();
}

apx_status apx_profile_entry(apx_ctx* ctx, int32_t k, const char** name, int64_t* launches, double* total_ms) {
  if (!ctx || !name || !launches || !total_ms) return APX_EINVAL;
  if (k < 0 || k >= (int32_t)ctx->prof_stats.size()) return fail(ctx, APX_EINVAL, "profile entry out of range");
  *name = ctx->prof_stats[k].name.c_str();
  *launches = ctx->prof_stats[k].launches;
  *total_ms = ctx->prof_stats[k].ms;
  return APX_OK;
}

const char* apx_version(void) { return "apx 0.1 gfx950"; }

apx_status apx_ctx_create(int32_t device, void* stream, apx_ctx** out) {
  if (!out) return APX_EINVAL;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return APX_EDEVICE;
  if (hipSetDevice(device) != hipSuccess) return APX_EDEVICE;
  apx_ctx* c = new apx_ctx();
  c->device = device;
  c->stream = static_cast<hipStream_t>(stream);
  if (hipHostMalloc((void**)&c->host_pinned, 64 * sizeof(int), hipHostMallocDefault) != hipSuccess) {
    delete c;
    return APX_ENOMEM;
  }
  if (blend_scratch_setup(c) != APX_OK) {
    (void)hipHostFree(c->host_pinned);
    delete c;
    return APX_EDEVICE;
  }
  *out = c;
  return APX_OK;
}

apx_status apx_ctx_set_stream(apx_ctx* ctx, void* stream) {
  if (!ctx) return APX_EINVAL;
  ctx->stream = static_cast<hipStream_t>(stream);
  return APX_OK;
}

void apx_ctx_destroy(apx_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  prof_flush(ctx, true);
  for (hipEvent_t e : ctx->prof_pool) (void)hipEventDestroy(e);
  if (ctx->host_pinned) (void)hipHostFree(ctx->host_pinned);
  delete ctx;
}

const char* apx_last_error(const apx_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

apx_status apx_ctx_synchronize(apx_ctx* ctx) {
  if (!ctx) return APX_EINVAL;
  APX_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return APX_OK;
}

}  // extern "C"
