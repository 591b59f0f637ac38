// Request-serving loop: continuous batching of GMRES solves.
//
// A request is one geometry, a list of incidence angles (one right-hand side
// each) and GMRES options.  Every right-hand side becomes a "column" with its
// own device-resident Krylov basis, and the worker thread advances all
// admitted columns together, one Arnoldi step per round:
//   1. columns that need K M v this round are grouped by (geometry,
//      preconditioner flag); each group's inputs are gathered into one
//      [R][N] block and applied as ONE multi-right-hand-side launch (so
//      incidence angles of different requests on the same geometry share the
//      FMM passes); groups of different geometries go to different streams
//      and overlap on the device;
//   2. one batched two-pass classical Gram-Schmidt over every Arnoldi column
//      (each with its own basis length), residual updates for columns that
//      restart or finish, and one device-to-host copy of the new Hessenberg
//      columns and norms;
//   3. Givens rotations and convergence tests on the host, then batched
//      basis-vector scaling and solution updates.
// Requests that arrive while others run are admitted at the next round as
// soon as right-hand-side slots and the HBM budget allow; a request whose
// footprint can never fit is rejected at submission.  Finished requests keep
// phi and the far field in host memory until released.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "lm_internal.hpp"

namespace {

typedef std::complex<double> C;
constexpr int SRV_STREAMS = 4;
constexpr int SD_SLICE = 2048;  // elements per workgroup in the dot kernel
constexpr int SD_IBLK = 64;     // basis vectors per workgroup in the dot kernel

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Per-column operands of the batched kernels.
struct ColDev {
  double2* V;         // basis [m+1][N]
  double2* w;         // vector being orthogonalised / residual
  const double2* g;   // right-hand side (residual form), or null
  const double2* src; // copy / scale source
  double2* dst;       // copy / scale destination
  double2* z;         // solution accumulator
  const double2* y;   // combination coefficients
  double scale;
  int N, cnt;
};

// dst = src * scale      (grid (ceil(Nmax / 256), ncols))
__global__ void __launch_bounds__(256) k_s_copy(const ColDev* __restrict__ d) {
  const ColDev c = d[blockIdx.y];
  const int n = blockIdx.x * 256 + threadIdx.x;
  if (n >= c.N) return;
  const double2 v = c.src[n];
  c.dst[n] = make_double2(v.x * c.scale, v.y * c.scale);
}

__device__ __forceinline__ double s_wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// w = g - w when g is set; wave partials of |w|^2 into part[col nw + wave].
__global__ void __launch_bounds__(256) k_s_resid(const ColDev* __restrict__ d, double* __restrict__ part, int nw) {
  const ColDev c = d[blockIdx.y];
  const int n = blockIdx.x * 256 + threadIdx.x;
  if (blockIdx.x * 256 >= c.N) return;  // whole workgroup beyond this column
  double q = 0.0;
  if (n < c.N) {
    double2 v = c.w[n];
    if (c.g) {
      const double2 gv = c.g[n];
      v = make_double2(gv.x - v.x, gv.y - v.y);
      c.w[n] = v;
    }
    q = v.x * v.x + v.y * v.y;
  }
  q = s_wave_sum(q);
  if ((threadIdx.x & 63) == 0) part[(int64_t)blockIdx.y * nw + blockIdx.x * 4 + (threadIdx.x >> 6)] = q;
}

// nrm[col] = sum of the column's wave partials (4 per 256 elements).
__global__ void __launch_bounds__(64) k_s_norm_final(const ColDev* __restrict__ d, const double* __restrict__ part,
                                                     int nw, double* __restrict__ nrm) {
  const int nwc = 4 * ((d[blockIdx.x].N + 255) / 256);
  double q = 0.0;
  for (int k = threadIdx.x; k < nwc; k += 64) q += part[(int64_t)blockIdx.x * nw + k];
  q = s_wave_sum(q);
  if (threadIdx.x == 0) nrm[blockIdx.x] = q;
}

// Workgroup partials of conj(V[i]) . w for i in this workgroup's block of
// basis vectors: part[(col ldh + i) nb + blockIdx.x].
__global__ void __launch_bounds__(256) k_s_dots(const ColDev* __restrict__ d, double2* __restrict__ part, int ldh,
                                                int nb) {
  const ColDev c = d[blockIdx.y];
  const int ib = blockIdx.z * SD_IBLK;
  if (ib >= c.cnt || blockIdx.x * SD_SLICE >= c.N) return;  // uniform per workgroup
  const int ie = min(c.cnt, ib + SD_IBLK);
  constexpr int EPT = SD_SLICE / 256;
  double2 x[EPT];
  int idx[EPT];
  bool ok[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int n = blockIdx.x * SD_SLICE + threadIdx.x + 256 * e;
    ok[e] = n < c.N;
    idx[e] = ok[e] ? n : 0;
    x[e] = ok[e] ? c.w[idx[e]] : make_double2(0.0, 0.0);
  }
  __shared__ double red[2][4];
  for (int i = ib; i < ie; ++i) {
    const double2* v = c.V + (int64_t)i * c.N;
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const double2 a = ok[e] ? v[idx[e]] : make_double2(0.0, 0.0);
      re = fma(a.x, x[e].x, re);
      re = fma(a.y, x[e].y, re);
      im = fma(a.x, x[e].y, im);
      im = fma(-a.y, x[e].x, im);
    }
    re = s_wave_sum(re);
    im = s_wave_sum(im);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
      red[0][threadIdx.x >> 6] = re;
      red[1][threadIdx.x >> 6] = im;
    }
    __syncthreads();
    if (threadIdx.x == 0)
      part[((int64_t)blockIdx.y * ldh + i) * nb + blockIdx.x] =
          make_double2((red[0][0] + red[0][1]) + (red[0][2] + red[0][3]), (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]));
  }
}

// h[col hs + off + i] = sum of the column's workgroup partials  (grid (cntmax, ncols)).
__global__ void __launch_bounds__(64) k_s_dots_final(const ColDev* __restrict__ d, const double2* __restrict__ part,
                                                     int ldh, int nb, double2* __restrict__ h, int hs, int off) {
  const ColDev c = d[blockIdx.y];
  const int i = blockIdx.x;
  if (i >= c.cnt) return;
  const int nbc = (c.N + SD_SLICE - 1) / SD_SLICE;
  double re = 0.0, im = 0.0;
  for (int k = threadIdx.x; k < nbc; k += 64) {
    const double2 v = part[((int64_t)blockIdx.y * ldh + i) * nb + k];
    re += v.x;
    im += v.y;
  }
  re = s_wave_sum(re);
  im = s_wave_sum(im);
  if (threadIdx.x == 0) h[(int64_t)blockIdx.y * hs + off + i] = make_double2(re, im);
}

// w -= sum_{i < cnt} V[i] h[i]
__global__ void __launch_bounds__(256) k_s_update(const ColDev* __restrict__ d, const double2* __restrict__ h, int hs,
                                                  int off) {
  const ColDev c = d[blockIdx.y];
  if (blockIdx.x * 256 >= c.N || c.cnt == 0) return;
  const int n = blockIdx.x * 256 + threadIdx.x;
  const bool ok = n < c.N;
  const int o = ok ? n : 0;
  const double2* hc = h + (int64_t)blockIdx.y * hs + off;
  double2 acc = ok ? c.w[o] : make_double2(0.0, 0.0);
  constexpr int U = 8;
  for (int i0 = 0; i0 < c.cnt; i0 += U) {
    double2 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = (i0 + u < c.cnt) ? c.V[(int64_t)(i0 + u) * c.N + o] : make_double2(0.0, 0.0);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (i0 + u < c.cnt) {
        const double2 hv = hc[i0 + u];
        acc.x = fma(-hv.x, v[u].x, acc.x);
        acc.x = fma(hv.y, v[u].y, acc.x);
        acc.y = fma(-hv.x, v[u].y, acc.y);
        acc.y = fma(-hv.y, v[u].x, acc.y);
      }
    }
  }
  if (ok) c.w[o] = acc;
}

// z += sum_{i < cnt} V[i] y[i]
__global__ void __launch_bounds__(256) k_s_lincomb(const ColDev* __restrict__ d) {
  const ColDev c = d[blockIdx.y];
  const int n = blockIdx.x * 256 + threadIdx.x;
  if (n >= c.N) return;
  double2 acc = c.z[n];
  for (int i = 0; i < c.cnt; ++i) {
    const double2 a = c.y[i], v = c.V[(int64_t)i * c.N + n];
    acc.x = fma(a.x, v.x, acc.x);
    acc.x = fma(-a.y, v.y, acc.x);
    acc.y = fma(a.x, v.y, acc.y);
    acc.y = fma(a.y, v.x, acc.y);
  }
  c.z[n] = acc;
}

enum Phase { PH_INIT = 0, PH_ARNOLDI = 1, PH_RESTART = 2, PH_FINAL = 3 };

struct Request;

struct Column {
  Request* req = nullptr;
  int col = 0;
  lm_geom_s* g = nullptr;
  int N = 0, m = 0;
  Phase phase = PH_INIT;
  DevBuf V, z, gv, y;
  int j = 0, its = 0, ncols = 0;
  double gnorm = 0.0, res = 1.0;
  bool converged = false, finished = false;
  std::vector<C> H, cs, sn, e1;
  double2* w = nullptr;  // this round's vector (group output slice or gv)
};

struct Request {
  uint64_t id = 0;
  lm_geom_s* g = nullptr;
  int R = 0;
  std::vector<double> theta, obs;
  lm_gmres_opts o{};
  lm_state state = LM_QUEUED;
  lm_status status = LM_OK;
  std::string err;
  std::vector<lm_solve_report> rep;
  std::vector<double2> phi, ff;
  int cols_left = 0;
  bool cancel = false;
  double t_submit = 0.0, t_done = 0.0;
  int64_t bytes = 0;
};

struct Group {
  DevBuf X, Y;
  KmBufs km;
};

}  // namespace

struct lm_server_s {
  lm_server_opts o{};
  int device = 0;
  std::mutex mu;
  std::condition_variable cv;
  std::thread th;
  bool stop = false;
  std::deque<Request*> queue;
  std::map<uint64_t, Request*> reqs;
  uint64_t next_id = 1;
  int64_t used = 0;
  int active_rhs = 0;
  int64_t rounds = 0, launches = 0, fused_rhs = 0;
  double km_ms = 0.0, gs_ms = 0.0, gs_bytes = 0.0;  // phase times (HIP events) and Gram-Schmidt algorithmic bytes
  double m2l_ms = 0.0, m2l_flops = 0.0;              // M2L launches of the fused matvecs (HIP events)
  int64_t m2l_launches = 0;
  hipEvent_t t0 = nullptr, t1 = nullptr, t2 = nullptr;
  hipEvent_t sev[SRV_STREAMS][14] = {};
  // worker state
  std::vector<Column*> cols;
  std::map<std::pair<lm_geom_s*, int>, Group> groups;
  std::map<lm_geom_s*, int> stream_of;
  hipStream_t s = nullptr;
  hipStream_t gs[SRV_STREAMS] = {};
  hipEvent_t ev_main = nullptr;
  hipEvent_t ev[SRV_STREAMS] = {};
  DevBuf d_desc, d_h, d_nrm, d_dpart, d_npart, d_y;
  std::vector<ColDev> hdesc;
  std::vector<double2> hh;
  std::vector<double> hnrm;
};

namespace {

int64_t footprint(const lm_geom_s* g, const lm_gmres_opts& o, int R) {
  const int64_t N = g->N;
  const int m = std::max(1, std::min(o.restart, o.max_iter));
  const int64_t per = (int64_t)(m + 1 + 2 + 3) * N * 16 + (int64_t)(m + 1) * 16 + 2 * N * 8 +
                      (g->fmm ? fmm_ws_per_rhs(g->fmm) : 0);
  return per * R;
}

void fail_request(lm_server_s* S, Request* q, lm_status st, const std::string& msg) {
  std::lock_guard<std::mutex> lk(S->mu);
  if (q->state == LM_QUEUED || q->state == LM_RUNNING) {
    q->state = LM_FAILED;
    q->status = st;
    q->err = msg;
    q->t_done = now_s();
  }
}

lm_status upload_desc(lm_server_s* S, const std::vector<ColDev>& d) {
  const size_t b = d.size() * sizeof(ColDev);
  if (S->d_desc.bytes < b) LM_TRY(S->d_desc.alloc(std::max<size_t>(b, 64 * sizeof(ColDev))));
  LM_TRY_HIP(hipMemcpyAsync(S->d_desc.p, d.data(), b, hipMemcpyHostToDevice, S->s));
  // the host vector may change before the copy runs: wait for it
  LM_TRY_HIP(hipStreamSynchronize(S->s));
  return LM_OK;
}

lm_status ensure(DevBuf& b, size_t bytes) {
  if (b.bytes < bytes) LM_TRY(b.alloc(bytes));
  return LM_OK;
}

// Allocate the columns of an admitted request and compute its right-hand sides.
lm_status start_request(lm_server_s* S, Request* q) {
  const int m = std::max(1, std::min(q->o.restart, q->o.max_iter));
  const int N = (int)q->g->N;
  for (int c = 0; c < q->R; ++c) {
    Column* col = new (std::nothrow) Column();
    LM_CHECK(col, LM_ENOMEM, "host allocation failed");
    S->cols.push_back(col);
    col->req = q;
    col->col = c;
    col->g = q->g;
    col->N = N;
    col->m = m;
    LM_TRY(col->V.alloc((size_t)(m + 1) * N * sizeof(double2)));
    LM_TRY(col->z.alloc((size_t)N * sizeof(double2)));
    LM_TRY(col->gv.alloc((size_t)N * sizeof(double2)));
    LM_TRY(col->y.alloc((size_t)(m + 1) * sizeof(double2)));
    LM_TRY_HIP(hipMemsetAsync(col->z.p, 0, (size_t)N * sizeof(double2), S->s));
    LM_TRY(rhs_launch(q->g, 1, &q->theta[c], col->gv.p, S->s));
    col->H.assign((size_t)(m + 1) * m, 0.0);
    col->cs.assign(m, 0.0);
    col->sn.assign(m, 0.0);
    col->e1.assign(m + 1, 0.0);
    col->phase = PH_INIT;
  }
  q->rep.assign(q->R, lm_solve_report{0, 0.0});
  q->cols_left = q->R;
  return LM_OK;
}

// phi = M z, far field, copy to host; marks the column finished.
lm_status finish_column(lm_server_s* S, Column* c) {
  Request* q = c->req;
  const int N = c->N;
  DevBuf phi, ff;
  LM_TRY(phi.alloc((size_t)N * sizeof(double2)));
  const bool pre = q->o.precond && c->g->pre;
  if (pre) {
    LM_TRY(precond_apply(c->g, S->o.precision, 1, c->z.p, phi.p, S->s));
  } else {
    LM_TRY_HIP(hipMemcpyAsync(phi.p, c->z.p, (size_t)N * sizeof(double2), hipMemcpyDeviceToDevice, S->s));
  }
  LM_TRY_HIP(hipMemcpyAsync(q->phi.data() + (size_t)c->col * N, phi.p, (size_t)N * sizeof(double2),
                            hipMemcpyDeviceToHost, S->s));
  const int no = (int)q->obs.size();
  if (no) {
    LM_TRY(ff.alloc((size_t)no * sizeof(double2)));
    LM_TRY(farfield_launch(c->g, 1, phi.p, no, q->obs.data(), ff.p, S->s));
    LM_TRY_HIP(hipMemcpyAsync(q->ff.data() + (size_t)c->col * no, ff.p, (size_t)no * sizeof(double2),
                              hipMemcpyDeviceToHost, S->s));
  }
  LM_TRY_HIP(hipStreamSynchronize(S->s));
  q->rep[c->col].iterations = c->its;
  q->rep[c->col].rel_residual = c->res;
  c->finished = true;
  return LM_OK;
}

// One round of the worker (see the file comment).  Returns an error only for
// failures that are not attributable to a single request.
lm_status round(lm_server_s* S) {
  std::vector<Column*> cols;
  for (Column* c : S->cols)
    if (!c->finished) cols.push_back(c);
  if (cols.empty()) return LM_OK;
  const int prec = S->o.precision;
  LM_TRY_HIP(hipEventRecord(S->t0, S->s));
  // ---- 1. K M v for every column that needs it, fused per (geometry, precond)
  std::map<std::pair<lm_geom_s*, int>, std::vector<Column*>> byg;
  for (Column* c : cols) {
    if (c->phase == PH_INIT) {
      c->w = c->gv.as<double2>();
      continue;
    }
    byg[{c->g, c->req->o.precond ? 1 : 0}].push_back(c);
  }
  LM_TRY_HIP(hipEventRecord(S->ev_main, S->s));
  std::vector<char> used_stream(SRV_STREAMS, 0), stream_timed(SRV_STREAMS, 0);
  std::vector<int> timed_streams;
  double m2l_flops_round = 0.0;
  int64_t n_launch = 0, n_fused = 0;
  for (auto& kv : byg) {
    lm_geom_s* g = kv.first.first;
    const bool pre = kv.first.second && g->pre;
    std::vector<Column*>& gc = kv.second;
    const int R = (int)gc.size(), N = (int)g->N;
    auto it = S->stream_of.find(g);
    if (it == S->stream_of.end()) it = S->stream_of.emplace(g, (int)(S->stream_of.size() % SRV_STREAMS)).first;
    const int si = it->second;
    hipStream_t st = S->gs[si];
    if (!used_stream[si]) LM_TRY_HIP(hipStreamWaitEvent(st, S->ev_main, 0));
    used_stream[si] = 1;
    Group& G = S->groups[kv.first];
    LM_TRY(ensure(G.X, (size_t)R * N * sizeof(double2)));
    LM_TRY(ensure(G.Y, (size_t)R * N * sizeof(double2)));
    double2* X = G.X.as<double2>();
    double2* Y = G.Y.as<double2>();
    for (int k = 0; k < R; ++k) {
      Column* c = gc[k];
      const double2* in = c->phase == PH_ARNOLDI ? c->V.as<double2>() + (size_t)c->j * N : c->z.as<double2>();
      LM_TRY_HIP(hipMemcpyAsync(X + (size_t)k * N, in, (size_t)N * sizeof(double2), hipMemcpyDeviceToDevice, st));
      c->w = Y + (size_t)k * N;
    }
    const bool time_m2l = g->method == LM_FMM && !stream_timed[si];
    G.km.stage_ev = time_m2l ? S->sev[si] : nullptr;
    LM_TRY(apply_km(g, prec, R, X, Y, pre, G.km, st));
    G.km.stage_ev = nullptr;
    if (time_m2l) {
      stream_timed[si] = 1;
      int64_t st10[10];
      fmm_stats(g->fmm, st10);
      const double P = 2.0 * g->p + 1.0;
      m2l_flops_round += 8.0 * P * P * std::min(R, 64) * (double)(st10[1] + st10[2]);
      timed_streams.push_back(si);
    }
    n_launch++;
    n_fused += R;
  }
  for (int i = 0; i < SRV_STREAMS; ++i)
    if (used_stream[i]) {
      LM_TRY_HIP(hipEventRecord(S->ev[i], S->gs[i]));
      LM_TRY_HIP(hipStreamWaitEvent(S->s, S->ev[i], 0));
    }
  LM_TRY_HIP(hipEventRecord(S->t1, S->s));
  float km_round = 0.f;
  // ---- 2. residuals, norms and batched CGS2 ------------------------------------
  const int nc = (int)cols.size();
  int Nmax = 0, ldh = 1, cntmax = 0;
  for (Column* c : cols) {
    Nmax = std::max(Nmax, c->N);
    ldh = std::max(ldh, c->m + 1);
    if (c->phase == PH_ARNOLDI) cntmax = std::max(cntmax, c->j + 1);
  }
  const int nwu = 4 * (int)div_up(Nmax, 256), nbd = (int)div_up(Nmax, SD_SLICE);
  LM_TRY(ensure(S->d_npart, (size_t)nc * nwu * sizeof(double)));
  LM_TRY(ensure(S->d_nrm, (size_t)nc * sizeof(double)));
  LM_TRY(ensure(S->d_h, (size_t)nc * 2 * ldh * sizeof(double2)));
  S->hdesc.assign(nc, ColDev{});
  for (int i = 0; i < nc; ++i) {
    Column* c = cols[i];
    ColDev& d = S->hdesc[i];
    d.V = c->V.as<double2>();
    d.w = c->w;
    d.g = (c->phase == PH_RESTART || c->phase == PH_FINAL) ? c->gv.as<double2>() : nullptr;
    d.N = c->N;
    d.cnt = c->phase == PH_ARNOLDI ? c->j + 1 : 0;
  }
  LM_TRY(upload_desc(S, S->hdesc));  // synchronises: the Gram-Schmidt timing starts after it
  LM_TRY_HIP(hipEventElapsedTime(&km_round, S->t0, S->t1));
  LM_TRY_HIP(hipEventRecord(S->t1, S->s));
  const ColDev* dd = S->d_desc.as<ColDev>();
  const int hs = 2 * ldh;
  if (cntmax > 0) {
    LM_TRY(ensure(S->d_dpart, (size_t)nc * ldh * nbd * sizeof(double2)));
    for (int pass = 0; pass < 2; ++pass) {
      hipLaunchKernelGGL(k_s_dots, dim3(nbd, nc, div_up(cntmax, SD_IBLK)), dim3(256), 0, S->s, dd,
                         S->d_dpart.as<double2>(), ldh, nbd);
      hipLaunchKernelGGL(k_s_dots_final, dim3(cntmax, nc), dim3(64), 0, S->s, dd, S->d_dpart.as<double2>(), ldh, nbd,
                         S->d_h.as<double2>(), hs, pass * ldh);
      hipLaunchKernelGGL(k_s_update, dim3(div_up(Nmax, 256), nc), dim3(256), 0, S->s, dd, S->d_h.as<double2>(), hs,
                         pass * ldh);
    }
  }
  // norms: of the orthogonalised vector (Arnoldi), of g - K M z (restart,
  // final) or of g (first round)
  hipLaunchKernelGGL(k_s_resid, dim3(div_up(Nmax, 256), nc), dim3(256), 0, S->s, dd, S->d_npart.as<double>(), nwu);
  hipLaunchKernelGGL(k_s_norm_final, dim3(nc), dim3(64), 0, S->s, dd, S->d_npart.as<double>(), nwu,
                     S->d_nrm.as<double>());
  LM_TRY_HIP(hipGetLastError());
  LM_TRY_HIP(hipEventRecord(S->t2, S->s));
  double gsb = 0.0;
  for (Column* c : cols) {  // bytes the CGS2 passes and the norm pass must move
    const double n16 = 16.0 * c->N;
    gsb += n16 + (c->phase == PH_ARNOLDI ? 2.0 * (2.0 * (c->j + 1) * n16 + 3.0 * n16) : 0.0);
  }
  S->hh.resize((size_t)nc * hs);
  S->hnrm.resize(nc);
  if (cntmax > 0)
    LM_TRY_HIP(hipMemcpyAsync(S->hh.data(), S->d_h.p, (size_t)nc * hs * sizeof(double2), hipMemcpyDeviceToHost, S->s));
  LM_TRY_HIP(hipMemcpyAsync(S->hnrm.data(), S->d_nrm.p, (size_t)nc * sizeof(double), hipMemcpyDeviceToHost, S->s));
  LM_TRY_HIP(hipStreamSynchronize(S->s));
  {
    float b = 0.f, m2l = 0.f;
    LM_TRY_HIP(hipEventElapsedTime(&b, S->t1, S->t2));
    for (int si : timed_streams) {
      float t = 0.f;
      LM_TRY_HIP(hipEventElapsedTime(&t, S->sev[si][4], S->sev[si][5]));
      m2l += t;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    S->km_ms += km_round;
    S->gs_ms += b;
    S->m2l_ms += m2l;
    S->m2l_flops += m2l_flops_round;
    S->m2l_launches += (int64_t)timed_streams.size();
    S->gs_bytes += gsb;
    S->launches += n_launch;
    S->fused_rhs += n_fused;
    S->rounds++;
  }
  // ---- 3. host updates ------------------------------------------------------------
  std::vector<ColDev> scal, comb;
  std::vector<double2> ys;
  std::vector<int> comb_col;
  std::vector<Column*> to_finish;
  for (int i = 0; i < nc; ++i) {
    Column* c = cols[i];
    const double nrm = std::sqrt(S->hnrm[i]);
    const double tol = c->req->o.tol;
    const int N = c->N, m = c->m;
    auto start_cycle = [&](const double2* r, double beta) {
      c->j = 0;
      std::fill(c->e1.begin(), c->e1.end(), C(0.0));
      c->e1[0] = beta;
      ColDev d{};
      d.src = r;
      d.dst = c->V.as<double2>();
      d.scale = 1.0 / beta;
      d.N = N;
      scal.push_back(d);
      c->phase = PH_ARNOLDI;
    };
    if (c->phase == PH_INIT) {
      c->gnorm = nrm;
      if (nrm == 0.0) {
        c->res = 0.0;
        c->converged = true;
        to_finish.push_back(c);
      } else {
        c->res = 1.0;
        start_cycle(c->w, nrm);
      }
    } else if (c->phase == PH_RESTART) {
      c->res = nrm / c->gnorm;
      if (c->res <= tol) {
        c->converged = true;
        to_finish.push_back(c);
      } else {
        start_cycle(c->w, nrm);
      }
    } else if (c->phase == PH_FINAL) {
      c->res = nrm / c->gnorm;  // true residual; convergence was decided by the GMRES estimate
      to_finish.push_back(c);
    } else {  // Arnoldi: Givens on the new column
      const int j = c->j;
      const double2* h1 = &S->hh[(size_t)i * hs];
      const double2* h2 = h1 + ldh;
      C* Hc = &c->H[(size_t)j * (m + 1)];
      for (int k = 0; k <= j; ++k) Hc[k] = C(h1[k].x + h2[k].x, h1[k].y + h2[k].y);
      Hc[j + 1] = nrm;
      for (int k = 0; k < j; ++k) {
        const C a = Hc[k], b = Hc[k + 1];
        Hc[k] = std::conj(c->cs[k]) * a + std::conj(c->sn[k]) * b;
        Hc[k + 1] = -c->sn[k] * a + c->cs[k] * b;
      }
      const C a = Hc[j], b = Hc[j + 1];
      const double rr = std::hypot(std::abs(a), std::abs(b));
      c->cs[j] = rr > 0 ? a / rr : C(1.0);
      c->sn[j] = rr > 0 ? b / rr : C(0.0);
      Hc[j] = std::conj(c->cs[j]) * a + std::conj(c->sn[j]) * b;
      Hc[j + 1] = 0.0;
      c->e1[j + 1] = -c->sn[j] * c->e1[j];
      c->e1[j] = std::conj(c->cs[j]) * c->e1[j];
      c->its++;
      c->res = std::abs(c->e1[j + 1]) / c->gnorm;
      const bool conv = c->res <= tol || nrm <= 1e-300;
      if (conv || j + 1 == m || c->its >= c->req->o.max_iter) {
        // y = H^{-1} e1, z += V y; then the true residual (final) or a restart
        const int cnt = j + 1;
        std::vector<C> yv(cnt);
        for (int k = cnt - 1; k >= 0; --k) {
          C acc = c->e1[k];
          for (int l = k + 1; l < cnt; ++l) acc -= c->H[(size_t)l * (m + 1) + k] * yv[l];
          yv[k] = acc / c->H[(size_t)k * (m + 1) + k];
        }
        comb_col.push_back(i);
        for (int k = 0; k < cnt; ++k) ys.push_back(make_double2(yv[k].real(), yv[k].imag()));
        ColDev d{};
        d.V = c->V.as<double2>();
        d.z = c->z.as<double2>();
        d.N = N;
        d.cnt = cnt;
        comb.push_back(d);
        c->converged = conv;
        c->phase = (conv || c->its >= c->req->o.max_iter) ? PH_FINAL : PH_RESTART;
      } else {
        ColDev d{};
        d.src = c->w;
        d.dst = c->V.as<double2>() + (size_t)(j + 1) * N;
        d.scale = 1.0 / nrm;
        d.N = N;
        scal.push_back(d);
        c->j = j + 1;
      }
    }
  }
  if (!comb.empty()) {
    LM_TRY(ensure(S->d_y, ys.size() * sizeof(double2)));
    LM_TRY_HIP(hipMemcpyAsync(S->d_y.p, ys.data(), ys.size() * sizeof(double2), hipMemcpyHostToDevice, S->s));
    size_t off = 0;
    for (auto& d : comb) {
      d.y = S->d_y.as<double2>() + off;
      off += d.cnt;
    }
  }
  std::vector<ColDev> all(scal);
  all.insert(all.end(), comb.begin(), comb.end());
  if (!all.empty()) {
    LM_TRY(upload_desc(S, all));
    int nm = 0;
    for (auto& d : all) nm = std::max(nm, d.N);
    const ColDev* da = S->d_desc.as<ColDev>();
    if (!scal.empty())
      hipLaunchKernelGGL(k_s_copy, dim3(div_up(nm, 256), scal.size()), dim3(256), 0, S->s, da);
    if (!comb.empty())
      hipLaunchKernelGGL(k_s_lincomb, dim3(div_up(nm, 256), comb.size()), dim3(256), 0, S->s, da + scal.size());
    LM_TRY_HIP(hipGetLastError());
    LM_TRY_HIP(hipStreamSynchronize(S->s));  // d_y / descriptors are reused next round
  }
  for (Column* c : to_finish) {
    lm_status st = finish_column(S, c);
    if (st < 0) fail_request(S, c->req, st, lm_last_error());
  }
  return LM_OK;
}

void release_columns(lm_server_s* S, Request* q) {
  auto& v = S->cols;
  for (auto it = v.begin(); it != v.end();) {
    if ((*it)->req == q) {
      delete *it;
      it = v.erase(it);
    } else {
      ++it;
    }
  }
}

void worker(lm_server_s* S) {
  (void)hipSetDevice(S->device);
  std::vector<Request*> running;
  while (true) {
    std::vector<Request*> admit;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      // drop cancelled requests (queued ones are dropped at cancel time)
      for (auto it = running.begin(); it != running.end();) {
        Request* q = *it;
        if (q->cancel || q->state == LM_FAILED) {
          if (q->state == LM_RUNNING) {
            q->state = LM_CANCELLED;
            q->status = LM_ECANCELLED;
            q->t_done = now_s();
          }
          S->used -= q->bytes;
          S->active_rhs -= q->R;
          lk.unlock();
          release_columns(S, q);
          lk.lock();
          it = running.erase(it);
        } else {
          ++it;
        }
      }
      if (S->stop) break;
      // admission: FIFO while right-hand-side slots and the HBM budget allow
      while (!S->queue.empty()) {
        Request* q = S->queue.front();
        if (S->active_rhs + q->R > S->o.max_active_rhs || S->used + q->bytes > S->o.hbm_budget_bytes) break;
        S->queue.pop_front();
        q->state = LM_RUNNING;
        S->used += q->bytes;
        S->active_rhs += q->R;
        admit.push_back(q);
      }
      if (running.empty() && admit.empty()) {
        S->cv.wait(lk, [&] { return S->stop || !S->queue.empty(); });
        continue;
      }
    }
    for (Request* q : admit) {
      lm_status st = start_request(S, q);
      if (st < 0) {
        fail_request(S, q, st, lm_last_error());
        release_columns(S, q);
      }
      running.push_back(q);
    }
    lm_status st = S->cols.empty() ? LM_OK : round(S);
    if (st < 0) {
      const std::string msg = lm_last_error();
      for (Request* q : running) fail_request(S, q, st, msg);
    }
    // completed requests
    for (auto it = running.begin(); it != running.end();) {
      Request* q = *it;
      bool all = true;
      bool conv = true;
      for (Column* c : S->cols)
        if (c->req == q) {
          all = all && c->finished;
          conv = conv && c->converged;
        }
      if (all && q->state == LM_RUNNING) {
        release_columns(S, q);
        std::lock_guard<std::mutex> lk(S->mu);
        q->state = LM_DONE;
        q->status = conv ? LM_OK : LM_NOT_CONVERGED;
        q->t_done = now_s();
        S->used -= q->bytes;
        S->active_rhs -= q->R;
        it = running.erase(it);
      } else {
        ++it;
      }
    }
  }
  for (Request* q : running) release_columns(S, q);
}

}  // namespace

// ---------------------------------------------------------------- C-ABI --
extern "C" lm_status lm_server_create(const lm_server_opts* o, lm_server* out) {
  LM_CHECK(out, LM_EINVAL, "out is NULL");
  *out = nullptr;
  lm_server_opts so{};
  if (o) so = *o;
  LM_CHECK(so.precision == LM_FP64 || so.precision == LM_MIXED, LM_EINVAL, "precision must be LM_FP64 or LM_MIXED");
  LM_CHECK(so.hbm_budget_bytes >= 0 && so.max_active_rhs >= 0, LM_EINVAL, "negative limits");
  if (so.hbm_budget_bytes == 0) so.hbm_budget_bytes = (int64_t)64 << 30;
  if (so.max_active_rhs == 0) so.max_active_rhs = 64;
  auto* S = new (std::nothrow) lm_server_s();
  LM_CHECK(S, LM_ENOMEM, "host allocation failed");
  S->o = so;
  if (hipGetDevice(&S->device) != hipSuccess) S->device = 0;
  bool ok = hipStreamCreateWithFlags(&S->s, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&S->ev_main, hipEventDisableTiming) == hipSuccess &&
            hipEventCreate(&S->t0) == hipSuccess && hipEventCreate(&S->t1) == hipSuccess &&
            hipEventCreate(&S->t2) == hipSuccess;
  for (int i = 0; ok && i < SRV_STREAMS; ++i)
    for (int e = 0; ok && e < 14; ++e) ok = hipEventCreate(&S->sev[i][e]) == hipSuccess;
  for (int i = 0; ok && i < SRV_STREAMS; ++i)
    ok = hipStreamCreateWithFlags(&S->gs[i], hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&S->ev[i], hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    lm_set_error("stream creation failed");
    delete S;
    return LM_EHIP;
  }
  S->th = std::thread(worker, S);
  *out = S;
  return LM_OK;
}

extern "C" lm_status lm_submit(lm_server S, const lm_request* r, uint64_t* id) {
  LM_CHECK(S && r && id, LM_EINVAL, "bad arguments");
  LM_CHECK(r->geom, LM_EINVAL, "request has no geometry");
  LM_CHECK(r->n_rhs >= 1 && r->theta_rad, LM_EINVAL, "request needs at least one incidence angle");
  LM_TRY(check_gmres_opts(&r->gmres));
  for (int i = 0; i < r->n_rhs; ++i)
    LM_CHECK(std::isfinite(r->theta_rad[i]) && std::sin(r->theta_rad[i]) > 0, LM_EINVAL,
             "incidence angle must be in (0, pi)");
  LM_CHECK(r->n_obs >= 0 && (r->n_obs == 0 || r->obs_rad), LM_EINVAL, "bad observation angles");
  for (int i = 0; i < r->n_obs; ++i)
    LM_CHECK(std::isfinite(r->obs_rad[i]) && std::fabs(std::sin(r->obs_rad[i])) > 1e-12, LM_EINVAL,
             "observation angles must be finite and not horizontal");
  auto* q = new (std::nothrow) Request();
  LM_CHECK(q, LM_ENOMEM, "host allocation failed");
  q->g = r->geom;
  q->R = r->n_rhs;
  q->theta.assign(r->theta_rad, r->theta_rad + r->n_rhs);
  if (r->n_obs) q->obs.assign(r->obs_rad, r->obs_rad + r->n_obs);
  q->o = r->gmres;
  q->bytes = footprint(q->g, q->o, q->R);
  q->phi.assign((size_t)q->R * q->g->N, make_double2(0.0, 0.0));
  q->ff.assign((size_t)q->R * r->n_obs, make_double2(0.0, 0.0));
  if (q->R > S->o.max_active_rhs || q->bytes > S->o.hbm_budget_bytes) {
    const int64_t b = q->bytes;
    delete q;
    LM_CHECK(false, LM_ENOMEM, "request can never be admitted (%d right-hand sides, %lld bytes)", r->n_rhs,
             (long long)b);
  }
  std::lock_guard<std::mutex> lk(S->mu);
  q->id = S->next_id++;
  q->t_submit = now_s();
  S->reqs[q->id] = q;
  S->queue.push_back(q);
  *id = q->id;
  S->cv.notify_all();
  return LM_OK;
}

extern "C" lm_status lm_poll(lm_server S, uint64_t id, lm_state* state, lm_solve_report* reports, double* latency_s,
                             void* phi_host, void* far_field_host) {
  LM_CHECK(S && state, LM_EINVAL, "bad arguments");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(id);
  LM_CHECK(it != S->reqs.end(), LM_ENOTFOUND, "unknown request id %llu", (unsigned long long)id);
  Request* q = it->second;
  *state = q->state;
  if (latency_s) *latency_s = q->t_done > 0 ? q->t_done - q->t_submit : now_s() - q->t_submit;
  if (q->state == LM_DONE) {
    if (reports) std::copy(q->rep.begin(), q->rep.end(), reports);
    if (phi_host) std::memcpy(phi_host, q->phi.data(), q->phi.size() * sizeof(double2));
    if (far_field_host) std::memcpy(far_field_host, q->ff.data(), q->ff.size() * sizeof(double2));
    return q->status;
  }
  if (q->state == LM_FAILED) {
    lm_set_error("%s", q->err.c_str());
    return q->status;
  }
  if (q->state == LM_CANCELLED) return LM_ECANCELLED;
  return LM_OK;
}

extern "C" lm_status lm_cancel(lm_server S, uint64_t id) {
  LM_CHECK(S, LM_EINVAL, "bad arguments");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(id);
  LM_CHECK(it != S->reqs.end(), LM_ENOTFOUND, "unknown request id %llu", (unsigned long long)id);
  Request* q = it->second;
  if (q->state == LM_QUEUED) {
    S->queue.erase(std::remove(S->queue.begin(), S->queue.end(), q), S->queue.end());
    q->state = LM_CANCELLED;
    q->status = LM_ECANCELLED;
    q->t_done = now_s();
  } else if (q->state == LM_RUNNING) {
    q->cancel = true;
  }
  return LM_OK;
}

extern "C" lm_status lm_release(lm_server S, uint64_t id) {
  LM_CHECK(S, LM_EINVAL, "bad arguments");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(id);
  LM_CHECK(it != S->reqs.end(), LM_ENOTFOUND, "unknown request id %llu", (unsigned long long)id);
  Request* q = it->second;
  LM_CHECK(q->state == LM_DONE || q->state == LM_FAILED || q->state == LM_CANCELLED, LM_EINVAL,
           "request %llu is still queued or running", (unsigned long long)id);
  delete q;
  S->reqs.erase(it);
  return LM_OK;
}

extern "C" lm_status lm_request_footprint(lm_geom g, int n_rhs, const lm_gmres_opts* o, int64_t* bytes) {
  LM_CHECK(g && bytes && n_rhs >= 1, LM_EINVAL, "bad arguments");
  LM_TRY(check_gmres_opts(o));
  *bytes = footprint(g, *o, n_rhs);
  return LM_OK;
}

extern "C" lm_status lm_server_stats(lm_server S, int64_t* out6) {
  LM_CHECK(S && out6, LM_EINVAL, "bad arguments");
  std::lock_guard<std::mutex> lk(S->mu);
  out6[0] = (int64_t)S->queue.size();
  out6[1] = S->active_rhs;
  out6[2] = S->used;
  out6[3] = S->rounds;
  out6[4] = S->launches;
  out6[5] = S->fused_rhs;
  return LM_OK;
}

extern "C" lm_status lm_server_phase_times(lm_server S, double* out6) {
  LM_CHECK(S && out6, LM_EINVAL, "bad arguments");
  std::lock_guard<std::mutex> lk(S->mu);
  out6[0] = S->km_ms;
  out6[1] = S->gs_ms;
  out6[2] = S->gs_bytes;
  out6[3] = S->m2l_ms;
  out6[4] = S->m2l_flops;
  out6[5] = (double)S->m2l_launches;
  return LM_OK;
}

extern "C" lm_status lm_server_destroy(lm_server S) {
  if (!S) return LM_OK;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    for (auto& kv : S->reqs)
      if (kv.second->state == LM_RUNNING) kv.second->cancel = true;
    S->cv.notify_all();
  }
  if (S->th.joinable()) S->th.join();
  for (auto& kv : S->reqs) delete kv.second;
  for (Column* c : S->cols) delete c;
  S->cols.clear();
  S->groups.clear();
  (void)hipStreamSynchronize(S->s);
  for (int i = 0; i < SRV_STREAMS; ++i) {
    if (S->gs[i]) (void)hipStreamDestroy(S->gs[i]);
    if (S->ev[i]) (void)hipEventDestroy(S->ev[i]);
  }
  if (S->ev_main) (void)hipEventDestroy(S->ev_main);
  for (hipEvent_t e : {S->t0, S->t1, S->t2})
    if (e) (void)hipEventDestroy(e);
  for (int i = 0; i < SRV_STREAMS; ++i)
    for (int e = 0; e < 14; ++e)
      if (S->sev[i][e]) (void)hipEventDestroy(S->sev[i][e]);
  if (S->s) (void)hipStreamDestroy(S->s);
  delete S;
  return LM_OK;
}
