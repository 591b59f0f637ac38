// C-ABI entry points: argument validation, handles, element construction and
// dispatch to the device paths.
#include <cmath>
#include <cstdarg>
#include <cstring>

#include "lm_internal.hpp"

static thread_local char g_err[1024] = "";

void lm_set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

extern "C" const char* lm_last_error(void) { return g_err; }
extern "C" const char* lm_version(void) { return "lmfmm 0.1 gfx950"; }

lm_status upload(DevBuf& b, const void* host, size_t bytes, hipStream_t s) {
  LM_TRY(b.alloc(bytes));
  if (bytes) LM_TRY_HIP(hipMemcpyAsync(b.p, host, bytes, hipMemcpyHostToDevice, s));
  return LM_OK;
}

static bool finite_all(const double* v, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

// ----------------------------------------------------------------- layers --
extern "C" lm_status lm_create_layers(int n_layers, const double* d, const double* k, const double* eta,
                                      lm_layers* out) {
  LM_CHECK(out, LM_EINVAL, "out is NULL");
  *out = nullptr;
  LM_CHECK(n_layers >= 2 && n_layers <= LM_MAX_LAYERS, LM_EINVAL, "n_layers must be in [2, %d]", LM_MAX_LAYERS);
  LM_CHECK(d && k, LM_EINVAL, "d and k are required");
  const int L = n_layers - 1;
  LM_CHECK(finite_all(d, L) && finite_all(k, n_layers), LM_EINVAL, "non-finite d or k");
  for (int l = 1; l < L; ++l) LM_CHECK(d[l] > d[l - 1], LM_EINVAL, "d must be strictly increasing");
  for (int l = 0; l <= L; ++l) LM_CHECK(k[l] > 0, LM_EINVAL, "k must be positive");
  if (eta) {
    LM_CHECK(finite_all(eta, n_layers), LM_EINVAL, "non-finite eta");
    for (int l = 0; l <= L; ++l) LM_CHECK(eta[l] > 0, LM_EINVAL, "eta must be positive");
  }
  auto* h = new (std::nothrow) lm_layers_s();
  LM_CHECK(h, LM_ENOMEM, "host allocation failed");
  std::memset(&h->m, 0, sizeof(h->m));
  h->m.L = L;
  h->m.kmax = 0;
  for (int l = 0; l < L; ++l) h->m.d[l] = d[l];
  for (int l = 0; l <= L; ++l) {
    h->m.k[l] = k[l];
    h->m.eta[l] = eta ? eta[l] : 1.0;
    h->m.kmax = std::fmax(h->m.kmax, k[l]);
  }
  *out = h;
  return LM_OK;
}

extern "C" lm_status lm_destroy_layers(lm_layers layers) {
  delete layers;
  return LM_OK;
}

// --------------------------------------------------------------- geometry --
lm_geom_s::~lm_geom_s() {
  if (fmm) fmm_free(fmm);
  if (pre) precond_free(pre);
}

int64_t lm_geom_s::device_bytes() const {
  int64_t b = d_cx.bytes + d_cy.bytes + d_w.bytes + d_layer.bytes + d_nx.bytes + d_ny.bytes + d_K.bytes + d_K32.bytes +
              d_sid.bytes + d_loc.bytes + d_cnt.bytes + d_speed.bytes + d_logw.bytes + d_roff.bytes;
  if (fmm) b += fmm_bytes(fmm);
  if (pre) b += precond_bytes(pre);
  return b;
}

// Nodes of the spectral rule: the input nodes, x'(t_j) from the trigonometric
// interpolant of each scatterer's M samples (the differentiation matrix of an
// even M, D_ij = (-1)^(i-j) cot((i - j) pi / M) / 2 and 0 on the diagonal,
// i.e. the unpaired mode dropped), weights (2 pi / M) |x'|, normals x'
// turned out of the curve, and the logarithmic weights
// R_k = -(2 pi / n) sum_{m=1}^{n-1} cos(2 pi k m / M) / m - (pi / n^2) (-1)^k,
// n = M / 2, of the product quadrature.
static lm_status spectral_nodes(lm_geom_s* g, int ns, const int64_t* off, const double* nodes, hipStream_t s) {
  const int64_t N = g->N;
  std::vector<int32_t>& sid = g->sid;
  std::vector<int32_t>& loc = g->loc;
  std::vector<int32_t>& cnt = g->cnt;
  std::vector<double>& speed = g->speed;
  std::vector<double>& logw = g->logw;
  std::vector<int64_t>& roff = g->roff;
  sid.assign(N, 0);
  loc.assign(N, 0);
  cnt.assign(N, 0);
  speed.assign(N, 0.0);
  logw.clear();
  roff.assign(ns, 0);
  for (int j = 0; j < ns; ++j) {
    const int64_t a = off[j];
    const int M = (int)(off[j + 1] - a), n = M / 2;
    std::vector<double> cotv(M, 0.0), dx(M, 0.0), dy(M, 0.0);
    for (int d = 1; d < M; ++d) cotv[d] = 0.5 * ((d & 1) ? -1.0 : 1.0) / std::tan(M_PI * d / M);
    for (int i = 0; i < M; ++i)
      for (int q = 0; q < M; ++q)
        if (q != i) {
          const double c = cotv[(i - q + M) % M];
          dx[i] += c * nodes[2 * (a + q)];
          dy[i] += c * nodes[2 * (a + q) + 1];
        }
    double area2 = 0.0;
    for (int i = 0; i < M; ++i) {
      const int64_t p0 = a + i, p1 = a + (i + 1) % M;
      area2 += nodes[2 * p0] * nodes[2 * p1 + 1] - nodes[2 * p1] * nodes[2 * p0 + 1];
    }
    const double o = area2 > 0 ? 1.0 : -1.0;
    const int l0 = layer_of(g->m, nodes[2 * a + 1]);
    for (int i = 0; i < M; ++i) {
      const int64_t p = a + i;
      const double sp = std::hypot(dx[i], dy[i]);
      LM_CHECK(sp > 0, LM_EINVAL, "scatterer %d: zero speed at node %d", j, i);
      g->cx[p] = nodes[2 * p];
      g->cy[p] = nodes[2 * p + 1];
      g->w[p] = 2.0 * M_PI / M * sp;
      g->nx[p] = o * dy[i] / sp;
      g->ny[p] = -o * dx[i] / sp;
      g->layer[p] = layer_of(g->m, g->cy[p]);
      LM_CHECK(g->layer[p] == l0, LM_EINVAL, "scatterer %d crosses an interface", j);
      sid[p] = j;
      loc[p] = i;
      cnt[p] = M;
      speed[p] = sp;
    }
    roff[j] = (int64_t)logw.size();
    for (int k = 0; k < M; ++k) {
      double r = -(M_PI / ((double)n * n)) * ((k & 1) ? -1.0 : 1.0);
      for (int m = 1; m < n; ++m) r -= 2.0 * M_PI / n * std::cos(2.0 * M_PI * (double)k * m / M) / m;
      logw.push_back(r);
    }
  }
  LM_TRY(upload(g->d_sid, sid.data(), N * sizeof(int32_t), s));
  LM_TRY(upload(g->d_loc, loc.data(), N * sizeof(int32_t), s));
  LM_TRY(upload(g->d_cnt, cnt.data(), N * sizeof(int32_t), s));
  LM_TRY(upload(g->d_speed, speed.data(), N * sizeof(double), s));
  LM_TRY(upload(g->d_logw, logw.data(), logw.size() * sizeof(double), s));
  LM_TRY(upload(g->d_roff, roff.data(), roff.size() * sizeof(int64_t), s));
  return LM_OK;
}

extern "C" lm_status lm_create_geometry(lm_layers layers, int n_scatterers, const int64_t* off,
                                        const double* nodes, const lm_geom_opts* opts, void* hip_stream,
                                        lm_geom* out) {
  LM_CHECK(out, LM_EINVAL, "out is NULL");
  *out = nullptr;
  LM_CHECK(layers, LM_EINVAL, "layers is NULL");
  LM_CHECK(n_scatterers >= 1, LM_EINVAL, "need at least one scatterer");
  LM_CHECK(off && nodes, LM_EINVAL, "node_offsets and nodes are required");
  LM_CHECK(off[0] == 0, LM_EINVAL, "node_offsets[0] must be 0");
  for (int j = 0; j < n_scatterers; ++j)
    LM_CHECK(off[j + 1] - off[j] >= 3, LM_EINVAL, "scatterer %d has fewer than 3 nodes", j);
  const int64_t N = off[n_scatterers];
  LM_CHECK(N < (int64_t)1 << 31, LM_EINVAL, "too many elements");
  LM_CHECK(finite_all(nodes, 2 * N), LM_EINVAL, "non-finite node coordinates");
  hipStream_t s = (hipStream_t)hip_stream;

  std::unique_ptr<lm_geom_s> g(new (std::nothrow) lm_geom_s());
  LM_CHECK(g, LM_ENOMEM, "host allocation failed");
  g->layers = layers;
  g->m = layers->m;
  g->N = N;
  lm_geom_opts o = {LM_AUTO, 20, 48, -1, 0, LM_BC_DIRICHLET, 0.0, LM_QUAD_LOWEST};
  if (opts) o = *opts;
  LM_CHECK(o.quad == LM_QUAD_LOWEST || o.quad == LM_QUAD_SPECTRAL, LM_EINVAL, "bad quadrature");
  g->quad = o.quad;
  if (o.quad == LM_QUAD_SPECTRAL) {
    LM_CHECK(o.bc == LM_BC_DIRICHLET, LM_EINVAL, "the spectral rule is for Dirichlet scatterers");
    for (int j = 0; j < n_scatterers; ++j)
      LM_CHECK((off[j + 1] - off[j]) % 2 == 0 && off[j + 1] - off[j] >= 6, LM_EINVAL,
               "scatterer %d: the spectral rule needs an even number (>= 6) of nodes", j);
  }
  LM_CHECK(o.bc >= LM_BC_DIRICHLET && o.bc <= LM_BC_ROBIN, LM_EINVAL, "bad boundary condition");
  LM_CHECK(std::isfinite(o.robin_beta), LM_EINVAL, "non-finite robin_beta");
  g->bc = o.bc;
  g->robin_beta = o.bc == LM_BC_ROBIN ? o.robin_beta : 0.0;
  LM_CHECK(o.method >= LM_AUTO && o.method <= LM_FMM, LM_EINVAL, "bad method");
  g->method = o.method == LM_AUTO ? (N <= 4096 ? LM_DENSE : LM_FMM) : o.method;
  g->p = o.p > 0 ? o.p : 20;
  LM_CHECK(g->p <= 40, LM_EINVAL, "p must be <= 40");
  g->leaf_size = o.leaf_size > 0 ? o.leaf_size : 48;
  LM_CHECK(o.top_fft >= -1 && o.top_fft <= 1, LM_EINVAL, "top_fft must be -1, 0 or 1");
  g->top_fft = o.top_fft;

  // elements (Sec. 3.3): chord midpoints, chord lengths, layer of the midpoint
  g->cx.resize(N);
  g->cy.resize(N);
  g->w.resize(N);
  g->nx.resize(N);
  g->ny.resize(N);
  g->layer.resize(N);
  if (g->quad == LM_QUAD_SPECTRAL) LM_TRY(spectral_nodes(g.get(), n_scatterers, off, nodes, s));
  for (int j = 0; j < n_scatterers && g->quad == LM_QUAD_LOWEST; ++j) {
    const int64_t a = off[j], n = off[j + 1] - off[j];
    double area2 = 0.0;  // twice the signed area: > 0 for counter-clockwise nodes
    for (int64_t i = 0; i < n; ++i) {
      const int64_t p0 = a + i, p1 = a + (i + 1) % n;
      area2 += nodes[2 * p0] * nodes[2 * p1 + 1] - nodes[2 * p1] * nodes[2 * p0 + 1];
    }
    const double o = area2 > 0 ? 1.0 : -1.0;
    for (int64_t i = 0; i < n; ++i) {
      const int64_t p0 = a + i, p1 = a + (i + 1) % n;
      const double x0 = nodes[2 * p0], y0 = nodes[2 * p0 + 1];
      const double x1 = nodes[2 * p1], y1 = nodes[2 * p1 + 1];
      const double len = std::hypot(x1 - x0, y1 - y0);
      LM_CHECK(len > 0, LM_EINVAL, "degenerate element %lld (repeated node)", (long long)p0);
      g->cx[p0] = 0.5 * (x0 + x1);
      g->cy[p0] = 0.5 * (y0 + y1);
      g->w[p0] = len;
      g->nx[p0] = o * (y1 - y0) / len;
      g->ny[p0] = -o * (x1 - x0) / len;
      g->layer[p0] = layer_of(g->m, g->cy[p0]);
    }
  }
  LM_TRY(upload(g->d_cx, g->cx.data(), N * sizeof(double), s));
  LM_TRY(upload(g->d_cy, g->cy.data(), N * sizeof(double), s));
  LM_TRY(upload(g->d_w, g->w.data(), N * sizeof(double), s));
  LM_TRY(upload(g->d_layer, g->layer.data(), N * sizeof(int32_t), s));
  LM_TRY(upload(g->d_nx, g->nx.data(), N * sizeof(double), s));
  LM_TRY(upload(g->d_ny, g->ny.data(), N * sizeof(double), s));

  LM_CHECK(g->bc == LM_BC_DIRICHLET || g->method == LM_DENSE || o.precond <= 0, LM_EINVAL,
           "no domain-decomposition preconditioner for Neumann and Robin scatterers");
  if (g->method == LM_DENSE) {
    LM_CHECK(N <= 32768, LM_EINVAL, "dense method limited to N <= 32768");
    LM_TRY(dense_assemble(g.get(), s));
  } else {
    LM_TRY(fmm_build(g.get(), s));
    if (o.precond && g->bc == LM_BC_DIRICHLET) LM_TRY(precond_build(g.get(), o.precond < 0 ? -1 : o.precond - 1, s));
  }
  LM_TRY_HIP(hipStreamSynchronize(s));
  *out = g.release();
  return LM_OK;
}

extern "C" lm_status lm_geometry_info(lm_geom g, int64_t* n, int64_t* bytes, int* method) {
  LM_CHECK(g, LM_EINVAL, "geom is NULL");
  if (n) *n = g->N;
  if (bytes) *bytes = g->device_bytes();
  if (method) *method = g->method;
  return LM_OK;
}

extern "C" lm_status lm_geometry_elements(lm_geom g, double* cx, double* cy, double* w, int32_t* layer) {
  LM_CHECK(g, LM_EINVAL, "geom is NULL");
  const size_t n = (size_t)g->N;
  if (cx) std::memcpy(cx, g->cx.data(), n * sizeof(double));
  if (cy) std::memcpy(cy, g->cy.data(), n * sizeof(double));
  if (w) std::memcpy(w, g->w.data(), n * sizeof(double));
  if (layer) std::memcpy(layer, g->layer.data(), n * sizeof(int32_t));
  return LM_OK;
}

extern "C" lm_status lm_geometry_normals(lm_geom g, double* nx, double* ny) {
  LM_CHECK(g, LM_EINVAL, "geom is NULL");
  const size_t n = (size_t)g->N;
  if (nx) std::memcpy(nx, g->nx.data(), n * sizeof(double));
  if (ny) std::memcpy(ny, g->ny.data(), n * sizeof(double));
  return LM_OK;
}

extern "C" lm_status lm_fmm_stats(lm_geom g, int64_t* out10) {
  LM_CHECK(g && out10, LM_EINVAL, "bad arguments");
  fmm_stats(g->fmm, out10);
  return LM_OK;
}

extern "C" lm_status lm_destroy_geometry(lm_geom g) {
  delete g;
  return LM_OK;
}

// ----------------------------------------------------------------- compute --
static lm_status check_prec(int precision) {
  LM_CHECK(precision == LM_FP64 || precision == LM_MIXED, LM_EINVAL, "precision must be LM_FP64 or LM_MIXED");
  return LM_OK;
}

lm_status geom_matvec(lm_geom_s* g, int precision, int n_rhs, const void* x, void* y, hipStream_t s,
                      hipEvent_t* stage_ev) {
  if (g->method == LM_DENSE) return dense_matvec(g, precision, n_rhs, x, y, s);
  return fmm_matvec_timed(g, precision, n_rhs, x, y, s, stage_ev);
}

extern "C" lm_status lm_matvec(lm_geom g, int precision, int n_rhs, const void* x, void* y, void* hip_stream) {
  LM_CHECK(g, LM_EINVAL, "geom is NULL");
  LM_TRY(check_prec(precision));
  LM_CHECK(n_rhs >= 1, LM_EINVAL, "n_rhs must be >= 1");
  LM_CHECK(x && y && x != y, LM_EINVAL, "x and y must be distinct device pointers");
  return geom_matvec(g, precision, n_rhs, x, y, (hipStream_t)hip_stream);
}

extern "C" lm_status lm_precond_apply(lm_geom g, int precision, int n_rhs, const void* x, void* y, void* hip_stream) {
  LM_CHECK(g, LM_EINVAL, "geom is NULL");
  LM_TRY(check_prec(precision));
  LM_CHECK(n_rhs >= 1, LM_EINVAL, "n_rhs must be >= 1");
  LM_CHECK(x && y && x != y, LM_EINVAL, "x and y must be distinct device pointers");
  LM_CHECK(g->pre, LM_EINVAL, "the geometry has no preconditioner");
  return precond_apply(g, precision, n_rhs, x, y, (hipStream_t)hip_stream);
}

extern "C" lm_status lm_precond_subdomains(lm_geom g, int64_t* info4, int32_t* jptr, int32_t* nb, int32_t* jidx) {
  LM_CHECK(g && info4, LM_EINVAL, "bad arguments");
  return precond_subdomains(g, info4, jptr, nb, jidx);
}

extern "C" lm_status lm_matvec_stage_times(lm_geom g, int precision, int n_rhs, const void* x, void* y, int reps,
                                           void* hip_stream, double* out9) {
  LM_CHECK(g && out9 && reps >= 1, LM_EINVAL, "bad arguments");
  LM_TRY(check_prec(precision));
  LM_CHECK(n_rhs >= 1 && x && y && x != y, LM_EINVAL, "x and y must be distinct device pointers");
  LM_CHECK(g->method == LM_FMM, LM_EINVAL, "stage timing is defined for the FMM method");
  return fmm_stage_times(g, precision, n_rhs, x, y, reps, (hipStream_t)hip_stream, out9);
}

extern "C" lm_status lm_rhs(lm_geom g, int n_rhs, const double* theta, void* g_dev, void* hip_stream) {
  LM_CHECK(g, LM_EINVAL, "geom is NULL");
  LM_CHECK(n_rhs >= 1 && theta && g_dev, LM_EINVAL, "bad arguments");
  for (int r = 0; r < n_rhs; ++r)
    LM_CHECK(std::isfinite(theta[r]) && std::sin(theta[r]) > 0, LM_EINVAL, "incidence angle must be in (0, pi)");
  return rhs_launch(g, n_rhs, theta, g_dev, (hipStream_t)hip_stream);
}

lm_status check_gmres_opts(const lm_gmres_opts* o) {
  LM_CHECK(o, LM_EINVAL, "gmres options are required");
  LM_CHECK(std::isfinite(o->tol) && o->tol > 0 && o->tol < 1, LM_EINVAL, "tol must be in (0, 1)");
  LM_CHECK(o->max_iter >= 1 && o->restart >= 1 && o->restart <= 1000, LM_EINVAL, "bad max_iter/restart");
  return LM_OK;
}

extern "C" lm_status lm_gmres_solve_rhs(lm_geom g, int precision, int n_rhs, const void* g_dev,
                                        const lm_gmres_opts* o, void* phi, lm_solve_report* rep,
                                        void* hip_stream) {
  LM_CHECK(g, LM_EINVAL, "geom is NULL");
  LM_TRY(check_prec(precision));
  LM_TRY(check_gmres_opts(o));
  LM_CHECK(n_rhs >= 1 && g_dev && phi && rep, LM_EINVAL, "bad arguments");
  return gmres_run(g, precision, n_rhs, g_dev, o, phi, rep, (hipStream_t)hip_stream);
}

extern "C" lm_status lm_gmres_solve(lm_geom g, int precision, int n_rhs, const double* theta,
                                    const lm_gmres_opts* o, void* phi, lm_solve_report* rep, void* hip_stream) {
  LM_CHECK(g, LM_EINVAL, "geom is NULL");
  LM_TRY(check_prec(precision));
  LM_TRY(check_gmres_opts(o));
  LM_CHECK(n_rhs >= 1 && theta && phi && rep, LM_EINVAL, "bad arguments");
  hipStream_t s = (hipStream_t)hip_stream;
  DevBuf rhs;
  LM_TRY(rhs.alloc((size_t)n_rhs * g->N * 16));
  LM_TRY(lm_rhs(g, n_rhs, theta, rhs.p, hip_stream));
  lm_status st = gmres_run(g, precision, n_rhs, rhs.p, o, phi, rep, s);
  LM_TRY_HIP(hipStreamSynchronize(s));
  return st;
}

extern "C" lm_status lm_far_field(lm_geom g, int n_rhs, const void* phi, int n_obs, const double* obs,
                                  void* out, void* hip_stream) {
  LM_CHECK(g, LM_EINVAL, "geom is NULL");
  LM_CHECK(n_rhs >= 1 && n_obs >= 1 && phi && obs && out, LM_EINVAL, "bad arguments");
  for (int j = 0; j < n_obs; ++j)
    LM_CHECK(std::isfinite(obs[j]) && std::fabs(std::sin(obs[j])) > 1e-12, LM_EINVAL,
             "observation angles must be finite and not horizontal");
  return farfield_launch(g, n_rhs, phi, n_obs, obs, out, (hipStream_t)hip_stream);
}
