// Internal definitions shared by the library's translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

#include "apx.h"

namespace apx {

// Growable device allocation owned by a context or model.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  hipError_t ensure(size_t b) {
    if (b <= bytes && p) return hipSuccess;
    release();
    hipError_t e = hipMalloc(&p, b ? b : 16);
    if (e == hipSuccess) bytes = b ? b : 16;
    else p = nullptr;
    return e;
  }
  template <class T> T* as() const { return static_cast<T*>(p); }
};

// Cell grid over the box: nc cells per axis of edge L/nc >= the requested size.
struct Grid {
  int nc[3];
  int per[3];
  double lo[3];
  double L[3];
  double inv_cell[3];
  long long ncell() const { return (long long)nc[0] * nc[1] * nc[2]; }
};

}  // namespace apx

namespace apx {
struct ProfPending {
  int id;
  hipEvent_t a, b;
};
struct ProfStat {
  std::string name;
  long long launches = 0;
  double ms = 0.0;
};
}  // namespace apx

struct apx_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  // scratch owned by the context
  apx::DevBuf cell_id, cell_count, cell_start, cell_fill, cell_atoms;
  apx::DevBuf scan_tmp, flags, itmp, itmp2, dtmp, ace_buf, thermo_grp;
  int* host_pinned = nullptr;  // small pinned staging area for readbacks
  // optional per-kernel timing with HIP events on the context stream
  bool prof = false;
  std::vector<apx::ProfPending> prof_pending;
  std::vector<hipEvent_t> prof_pool;
  std::vector<apx::ProfStat> prof_stats;
};

namespace apx {

apx_status fail(apx_ctx* ctx, apx_status code, const char* fmt, ...);

#define APX_HIP(ctx, expr)                                                              \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return ::apx::fail((ctx), APX_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define APX_LAUNCH_CHECK(ctx) APX_HIP(ctx, hipGetLastError())

#define APX_ALLOC(ctx, buf, bytes)                                                     \
  do {                                                                                 \
    if ((buf).ensure(bytes) != hipSuccess)                                             \
      return ::apx::fail((ctx), APX_ENOMEM, "device allocation of %zu bytes failed",   \
                         (size_t)(bytes));                                             \
  } while (0)

// Validates an apx_atoms descriptor.
apx_status check_atoms(apx_ctx* ctx, const apx_atoms* a);

// Grid with cells no smaller than `min_cell` (at least one cell per axis).
Grid make_grid(const apx_atoms* a, double min_cell);

// Bins atoms into the context's cell arrays (cell_start has ncell+1 entries).
// Sets flags bit 0 on the device if a non-periodic coordinate lies outside the box.
apx_status bin_atoms(apx_ctx* ctx, const apx_atoms* a, const Grid& g);

// Exclusive scan of m int32 values `in` into `out` (m+1 entries, out[m] = total).
apx_status scan_exclusive(apx_ctx* ctx, const int* in, long long m, int* out);

// Resolves the per-device address of the blend's static scratch array (blend.hip); called
// by apx_ctx_create with the context's device current.
apx_status blend_scratch_setup(apx_ctx* ctx);

// EAM energies and forces with weights w (as apx_eam_forces) plus, in the same density
// pass, df[3][n] = F(weights wl) - F(weights w) of the fast part; scratch4 holds 4n doubles.
apx_status eam_forces_dual(apx_ctx* ctx, const apx_atoms* atoms, const apx_nlist* nl, const apx_eam_params* p,
                           const double* w, const double* wl, double* e_site, double* rho, double* f, double* df,
                           double* scratch4);

// ACE energies and forces as apx_ace_energy_forces with weights w, plus f2[3][n]
// (overwritten) = -d/dx sum_i w2_i E_i over the same active atoms (w2 may be negative).
apx_status ace_energy_forces_dual(apx_ctx* ctx, const apx_atoms* atoms, const apx_nlist* nl, const apx_ace_model* m,
                                  const double* w, const double* w2, const int32_t* active, int64_t n_active,
                                  int32_t precision, double* e_site, double* f, double* f2);

// Local thermostat (thermostat.hip): energy errors and the group rescale, without the
// argument checks of the entry points.
apx_status thermostat_errors(apx_ctx* ctx, int64_t n, const uint8_t* frozen, const double* w_c, const double* w_d,
                             const double* e_fast, const double* e_precise, const double* f_d, const double* df,
                             const double* v_half, double dt, double mass, double* dE);
apx_status thermostat_correct(apx_ctx* ctx, const apx_atoms* atoms, double* vel, const double* dE,
                              const apx_thermo_params* p, int64_t step, double mass, int64_t* n_corrected,
                              int64_t* n_failed);

// Reads `count` ints from device memory into host memory (synchronising).
apx_status read_ints(apx_ctx* ctx, const int* dev, int* host, int count);

// Per-kernel timing: a scope records an event pair around the launches it encloses
// when profiling is enabled on the context.
int prof_id(apx_ctx* ctx, const char* name);
hipEvent_t prof_event(apx_ctx* ctx);
void prof_flush(apx_ctx* ctx, bool wait);

struct ProfScope {
  apx_ctx* ctx;
  int id = -1;
  hipEvent_t a = nullptr;
  ProfScope(apx_ctx* c, const char* name) : ctx(c) {
    if (ctx && ctx->prof) {
      id = prof_id(ctx, name);
      a = prof_event(ctx);
      if (a) (void)hipEventRecord(a, ctx->stream);
    }
  }
  ~ProfScope() {
    if (a) {
      hipEvent_t b = prof_event(ctx);
      if (b) {
        (void)hipEventRecord(b, ctx->stream);
        ctx->prof_pending.push_back({id, a, b});
      }
    }
  }
};

inline unsigned int blocks_for(long long n, int threads) {
  return (unsigned int)((n + threads - 1) / threads);
}

}  // namespace apx
