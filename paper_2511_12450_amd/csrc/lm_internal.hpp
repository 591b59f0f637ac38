// Internal declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <memory>
#include <string>
#include <vector>

#include "../../include/lmfmm.h"
#include "spectral.hpp"

// ----------------------------------------------------------------- errors --
void lm_set_error(const char* fmt, ...);

#define LM_TRY_HIP(expr)                                                             \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess) {                                                          \
      lm_set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__); \
      return e_ == hipErrorOutOfMemory ? LM_ENOMEM : LM_EHIP;                        \
    }                                                                                \
  } while (0)

#define LM_CHECK(cond, status, ...)  \
  do {                               \
    if (!(cond)) {                   \
      lm_set_error(__VA_ARGS__);     \
      return status;                 \
    }                                \
  } while (0)

#define LM_TRY(expr)               \
  do {                             \
    lm_status s_ = (expr);         \
    if (s_ < 0) return s_;         \
  } while (0)

// ----------------------------------------------------------- device memory --
// Owning device buffer (hipMalloc / hipFree).
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
  lm_status alloc(size_t n) {
    release();
    if (n == 0) return LM_OK;
    hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) {
      p = nullptr;
      lm_set_error("hipMalloc(%zu) failed: %s", n, hipGetErrorString(e));
      return LM_ENOMEM;
    }
    bytes = n;
    return LM_OK;
  }
  template <typename T> T* as() const { return static_cast<T*>(p); }
};

lm_status upload(DevBuf& b, const void* host, size_t bytes, hipStream_t s);

// ------------------------------------------------------------------ layers --
struct lm_layers_s {
  MediumDev m;
};

// Layer of a height y: l with -d_l < y < -d_{l-1}; within 1e-12 of an
// interface the point belongs to the upper layer.
inline int layer_of(const MediumDev& m, double y) {
  int l = 0;
  for (int j = 0; j < m.L; ++j)
    if (y < -m.d[j] - 1e-12) l = j + 1;
  return l;
}

// ----------------------------------------------------------------- geometry --
struct FmmPlan;   // fmm.hip
struct Precond;   // precond.hip

struct lm_geom_s {
  const lm_layers_s* layers = nullptr;
  MediumDev m;
  int64_t N = 0;
  int method = LM_DENSE;
  int p = 20;
  int leaf_size = 48;
  int top_fft = 0;  // level-0 M2L by FFT: 0 when it pays, 1 always, -1 never
  int bc = LM_BC_DIRICHLET;  // boundary condition of the scatterers
  double robin_beta = 0.0;   // impedance of the Robin condition
  int quad = LM_QUAD_LOWEST;  // quadrature of the single-layer operator
  // host element data, input numbering
  std::vector<double> cx, cy, w, nx, ny;  // nx, ny: unit normal out of the element's polygon
  std::vector<int32_t> layer;
  // device element data, input numbering
  DevBuf d_cx, d_cy, d_w, d_layer, d_nx, d_ny;
  // spectral rule: per node its scatterer, local index, the scatterer's node
  // count and |x'(t)|; per scatterer the logarithmic weights R_k, k = 0..M-1,
  // at roff[scatterer] (host and device copies)
  std::vector<int32_t> sid, loc, cnt;
  std::vector<double> speed, logw;
  std::vector<int64_t> roff;
  DevBuf d_sid, d_loc, d_cnt, d_speed, d_logw, d_roff;
  // dense path
  DevBuf d_K;          // complex128 row-major [N][N]
  DevBuf d_K32;        // complex64 copy for the mixed form
  // fast path
  FmmPlan* fmm = nullptr;
  Precond* pre = nullptr;
  int64_t device_bytes() const;
  ~lm_geom_s();
};

// ------------------------------------------------------------ entry points --
lm_status dense_assemble(lm_geom_s* g, hipStream_t s);
lm_status dense_matvec(lm_geom_s* g, int precision, int n_rhs, const void* x, void* y, hipStream_t s);
lm_status geom_matvec(lm_geom_s* g, int precision, int n_rhs, const void* x, void* y, hipStream_t s,
                      hipEvent_t* stage_ev = nullptr);
lm_status rhs_launch(lm_geom_s* g, int n_rhs, const double* theta_host, void* g_dev, hipStream_t s);
lm_status farfield_launch(lm_geom_s* g, int n_rhs, const void* phi, int n_obs, const double* obs_host,
                          void* out, hipStream_t s);
// Queued forms (no allocation, no wait): angles already on the device, and a
// scratch buffer of rhs_scratch_bytes(n_rhs) for the right-hand side.
size_t rhs_scratch_bytes(int n_rhs);
lm_status rhs_launch_dev(lm_geom_s* g, int n_rhs, const double* theta_dev, void* scratch, void* g_dev,
                         hipStream_t s);
lm_status farfield_launch_dev(lm_geom_s* g, int n_rhs, const void* phi, int n_obs, const double* obs_dev,
                              void* out, void* work, hipStream_t s);
// bytes of the work buffer farfield_launch_dev needs (0: none)
size_t farfield_work_bytes(lm_geom_s* g, int n_rhs, int n_obs);
// Copies n doubles from host memory to the device in kernel arguments
// (stream-ordered; the host array may be reused as soon as this returns).
lm_status put_f64_async(const double* host, int n, double* dev, hipStream_t s);
lm_status point_far_field_launch(const MediumDev& m, int n_src, const double* src_xy_host, int n_obs,
                                 const double* obs_host, void* out, hipStream_t s);
struct KmBufs {
  DevBuf x32, y32, mz;
  hipEvent_t* stage_ev = nullptr;  // when set: 16 events bracketing the FMM stages (see fmm_matvec_timed)
  int pre_precision = -1;          // precision of the preconditioner apply (-1: the matvec's)
};
lm_status apply_km(lm_geom_s* g, int precision, int R, const double2* x, double2* y, bool use_pre, KmBufs& b,
                   hipStream_t s);
lm_status check_gmres_opts(const lm_gmres_opts* o);
int64_t fmm_ws_per_rhs(const FmmPlan* f);
lm_status gmres_run(lm_geom_s* g, int precision, int n_rhs, const void* g_dev, const lm_gmres_opts* o,
                    void* phi_dev, lm_solve_report* rep, hipStream_t s);

// Per-launch workspace of the FMM matvec: expansions, P2M partial sums,
// level-0 transforms, per-entry M2L results, the complex64 transpose of x.
enum {
  FMM_WS_ME, FMM_WS_LE, FMM_WS_PART, FMM_WS_TOP_MH, FMM_WS_TOP_LH, FMM_WS_M2L_OUT, FMM_WS_OM_SLOT,
  FMM_WS_MF_PART, FMM_WS_XT, FMM_WS_N
};
struct FmmWs {
  void* p[FMM_WS_N] = {};
};
size_t fmm_ws_bytes(const FmmPlan* f, int r);
lm_status fmm_matvec_in(lm_geom_s* g, int precision, int n_rhs, const void* x, void* y, void* base, size_t cap,
                        hipStream_t s);

lm_status fmm_build(lm_geom_s* g, hipStream_t s);
void fmm_free(FmmPlan* f);
int64_t fmm_bytes(const FmmPlan* f);
void fmm_stats(const FmmPlan* f, int64_t* out);
lm_status fmm_matvec(lm_geom_s* g, int precision, int n_rhs, const void* x, void* y, hipStream_t s);
lm_status fmm_matvec_timed(lm_geom_s* g, int precision, int n_rhs, const void* x, void* y, hipStream_t s,
                           hipEvent_t* ev);
lm_status fmm_stage_times(lm_geom_s* g, int precision, int n_rhs, const void* x, void* y, int reps, hipStream_t s,
                          double* out);

lm_status precond_build(lm_geom_s* g, int coarsen, hipStream_t s);
void precond_free(Precond* p);
int64_t precond_bytes(const Precond* p);
lm_status precond_apply(lm_geom_s* g, int precision, int n_rhs, const void* x, void* y, hipStream_t s);
lm_status precond_subdomains(const lm_geom_s* g, int64_t* info4, int32_t* jptr, int32_t* nb, int32_t* jidx);

inline unsigned div_up(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }
