/*
 * lmfmm -- layered-medium Nystrom boundary integral solver for 2D Helmholtz
 * scattering on MI355X (gfx950).
 *
 * Method: Xia, Yuan, Wang, Cai, "Fast boundary integral method for acoustic
 * wave scattering in two-dimensional layered media".
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All functions are extern "C" and return lm_status.  Negative values are
 *   errors (outputs undefined), positive values are warnings (outputs
 *   written), LM_OK is 0.  lm_last_error() returns a thread-local message for
 *   the last non-OK status of the calling thread.
 * - Complex numbers are interleaved (re, im) pairs: c128 = 2 x double,
 *   c64 = 2 x float.
 * - "host" pointers are read during the call only and are copied; "device"
 *   pointers are HIP device allocations owned by the caller (for example
 *   torch tensors); the library never frees them.
 * - hip_stream is a hipStream_t passed as void* (NULL = the null stream).
 *   Work is enqueued on that stream; calls that return host results
 *   (reports, info) synchronise it.
 * - Element numbering: element j of scatterer m is the chord from node j to
 *   node j+1 (the last node connects to the first) of the m-th polygon, and
 *   elements are numbered scatterer by scatterer in input order.  Every
 *   [n_rhs][N] array uses this numbering; vector r occupies entries
 *   [r*N, (r+1)*N).
 * - Handles are opaque; create functions copy their inputs; each handle is
 *   freed by its destroy function.  Only the lm_server_* / lm_submit /
 *   lm_poll / lm_cancel entry points are thread-safe.
 */
#ifndef LMFMM_H
#define LMFMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lm_layers_s* lm_layers;
typedef struct lm_geom_s* lm_geom;
typedef struct lm_server_s* lm_server;

typedef enum {
  LM_OK = 0,
  LM_NOT_CONVERGED = 1, /* GMRES stopped at max_iter; outputs written */
  LM_EINVAL = -1,       /* invalid argument (NaN, bad sizes, bad geometry) */
  LM_ENOMEM = -2,       /* device or host allocation failed / over budget */
  LM_EHIP = -3,         /* a HIP runtime call failed */
  LM_ENOTFOUND = -4,    /* unknown request id */
  LM_ECANCELLED = -5,   /* request was cancelled */
  LM_EINTERNAL = -6
} lm_status;

/* LM_FP64: every step in double precision (the plain form).
 * LM_MIXED: near-field and translation arithmetic in FP32 accumulated in
 * FP32; spectral coefficients, singular self terms, GMRES Arnoldi/Givens in
 * FP64 (the served form). */
typedef enum { LM_FP64 = 0, LM_MIXED = 1 } lm_precision;

const char* lm_last_error(void);

/* Library version string, e.g. "lmfmm 0.1 gfx950". */
const char* lm_version(void);

/* ---------------------------------------------------------------- medium --
 * Sec. 2.1: L+1 layers l = 0..L (top to bottom), interfaces y = -d[l] for
 * l = 0..L-1 with d strictly increasing, wavenumbers k[l] > 0, and weights
 * eta[l] > 0 of the transmission condition [eta du/dn] = 0 (eta == NULL means
 * all ones).  n_layers = L+1 >= 2, at most LM_MAX_LAYERS.
 * Errors: LM_EINVAL for NaN/inf, non-increasing d, k <= 0, eta <= 0. */
#define LM_MAX_LAYERS 8
lm_status lm_create_layers(int n_layers, const double* d_host, const double* k_host,
                           const double* eta_host, lm_layers* out);
lm_status lm_destroy_layers(lm_layers layers);

/* -------------------------------------------------------------- geometry --
 * Sec. 3.3 (eq. linearSystem): each scatterer boundary is a closed polygon
 * of nodes; element = chord between consecutive nodes, collocation point =
 * chord midpoint, |Gamma_e| = chord length, layer = layer of the midpoint
 * (a midpoint within 1e-12 of an interface belongs to the upper layer).
 *
 * node_offsets_host: n_scatterers+1 increasing int64, node_offsets[0] = 0,
 *   each polygon has >= 3 nodes.
 * nodes_xy_host: 2*node_offsets[n_scatterers] doubles, (x, y) per node.
 * opts: NULL for defaults.
 *   method: LM_DENSE assembles the full matrix by direct Sommerfeld
 *           quadrature (O(N^2) memory, intended for N <= ~16k);
 *           LM_FMM uses the layered fast multipole method (Sec. 4.1);
 *           LM_AUTO picks DENSE for N <= 4096.
 *   p: expansion order (default 20); leaf_size: target points per leaf
 *   (default 48); precond: build the overlapping domain-decomposition
 *   preconditioner of Sec. 4.2 (FMM only): 0 none, 1 subdomains = the
 *   free-space leaf boxes, c >= 2 subdomains = boxes c-1 levels above the
 *   leaves (larger blocks, fewer iterations); default (-1) = the coarsest
 *   level whose neighbourhoods hold at most 8192 elements and whose blocks
 *   fit a quarter of the free device memory.
 *   top_fft: the interactions of the coarsest level (boxes of width 8 / k_max
 *   that meet every non-adjacent box of their tree and of every side tree)
 *   as a convolution along x, done by FFT: 0 (default) when the direct list
 *   would hold more than twice the frequency-domain products and the
 *   transformed operators fit a quarter of the free device memory, 1 always,
 *   -1 never.  Same operator either way, up to rounding.
 * The handle keeps a reference to `layers`, which must outlive it.
 * Errors: LM_EINVAL (bad offsets, NaN, degenerate chord), LM_ENOMEM, LM_EHIP. */
typedef enum { LM_AUTO = 0, LM_DENSE = 1, LM_FMM = 2 } lm_method;
/* Boundary condition of the scatterers (Sec. 2.1 names all three; the paper
 * develops the Dirichlet one).  Neumann and Robin use the same single-layer
 * representation u^s = S phi and the exterior limit of its normal derivative,
 * (-1/2 + K' + i beta S) phi = -(d_n + i beta)(u^inc + u^b) for the condition
 * (d_n + i beta) u = 0 (n out of the scatterer; beta = robin_beta, 0 for
 * Neumann); collocated at the chord midpoints with the rectangle rule.  On the
 * FMM the expansions are unchanged and the targets evaluate n . grad + i beta
 * of the local expansions and of the near-field kernel; the second-kind
 * system needs no preconditioner and none is built (precond >= 1 with
 * Neumann or Robin on the FMM: LM_EINVAL). */
typedef enum { LM_BC_DIRICHLET = 0, LM_BC_NEUMANN = 1, LM_BC_ROBIN = 2 } lm_bc;
/* Quadrature of the single-layer operator.
 * LM_QUAD_LOWEST: the paper's rule (Sec. 3.3, eqs. ApproximateComputation,
 *   matrixelmemts): chord elements between consecutive nodes, midpoint
 *   collocation, first order in the element size.
 * LM_QUAD_SPECTRAL: beyond the paper, for scatterers that are smooth closed
 *   curves sampled at equal parameter steps (an even number of nodes >= 6
 *   per scatterer, counter-clockwise or clockwise) and lie inside one layer
 *   without touching an interface.  The unknowns are the densities at the
 *   nodes themselves (element i = node i: lm_geometry_elements returns the
 *   nodes, their quadrature weights (2 pi / M) |x'(t_i)| with x' from the
 *   trigonometric interpolant of the scatterer's M nodes, and their layers);
 *   the free-space kernel on a node's own scatterer is split into
 *   -J_0(k r)/(4 pi) ln(4 sin^2((t - s)/2)) plus a smooth part and the
 *   logarithm integrated exactly against the trigonometric interpolant
 *   (Martensen-Kussmaul product quadrature), every other part by the
 *   trapezoidal rule: spectral order for analytic curves.  On the FMM the
 *   expansions and the near field keep the trapezoidal sums and a CSR of
 *   same-scatterer corrections (the difference of the two rules, whose Hankel
 *   parts cancel) plus the spectral self terms complete the operator (the
 *   preconditioner blocks stay those of the lowest-order rule on the nodes).
 *   Dirichlet condition only; LM_EINVAL otherwise, for an odd node count or
 *   for a scatterer whose nodes lie in more than one layer. */
typedef enum { LM_QUAD_LOWEST = 0, LM_QUAD_SPECTRAL = 1 } lm_quad;
typedef struct {
  int method;
  int p;
  int leaf_size;
  int precond;
  int top_fft;
  int bc;            /* lm_bc */
  double robin_beta; /* impedance beta of LM_BC_ROBIN */
  int quad;          /* lm_quad */
} lm_geom_opts;
lm_status lm_create_geometry(lm_layers layers, int n_scatterers, const int64_t* node_offsets_host,
                             const double* nodes_xy_host, const lm_geom_opts* opts, void* hip_stream,
                             lm_geom* out);
/* n_elements, bytes of device memory held by the handle, and the method in use. */
lm_status lm_geometry_info(lm_geom geom, int64_t* n_elements, int64_t* device_bytes, int* method);
/* Element data in input numbering (host outputs, any may be NULL):
 * cx, cy, w: double[N]; layer: int32[N]. */
lm_status lm_geometry_elements(lm_geom geom, double* cx, double* cy, double* w, int32_t* layer);
/* Unit normals of the elements pointing out of their polygon (the sign of the
 * polygon's signed area gives its orientation), host outputs double[N]. */
lm_status lm_geometry_normals(lm_geom geom, double* nx, double* ny);
lm_status lm_destroy_geometry(lm_geom geom);
/* Size of the fast-method plan (all zero for LM_DENSE), host output of 10
 * int64: boxes, free-space M2L list entries, reaction M2L list entries (the
 * lists leave out the coarsest level when its convolution is on),
 * free-space M2L classes, reaction M2L operators (Sommerfeld tables of the
 * lists), reaction near-field
 * element pairs, free-space leaf level, reaction finest level, free-space
 * near-field leaf pairs, free-space near-field element pairs. */
lm_status lm_fmm_stats(lm_geom geom, int64_t* out10);

/* ---------------------------------------------------------------- matvec --
 * y = K x for n_rhs vectors (eq. Llayerscomponent, unscaled form):
 *   (K x)_i = sum_{e != i, layer e == layer i} |Gamma_e| G^f(c_i|c_e) x_e
 *           + sum_e |Gamma_e| G^r(c_i|c_e) x_e + I^s_i x_i,
 * i.e. the paper's system with the eta scaling divided out row by row (the
 * paper's source-first eta-scaled system has the same solution).
 * x_dev, y_dev: device [n_rhs][N]; c128 for LM_FP64, c64 for LM_MIXED.
 * x and y must not overlap. */
lm_status lm_matvec(lm_geom geom, int precision, int n_rhs, const void* x_dev, void* y_dev,
                    void* hip_stream);

/* lm_matvec for callers that cannot allocate device memory (code under
 * stream capture, serving loops or harnesses that forbid hipMalloc): the same
 * operator, arguments and errors as lm_matvec, with the FMM's per-launch
 * workspace (expansions, partial sums, level-0 transforms, the complex64
 * transpose of x) in a static device array of LM_NOALLOC_SCRATCH_BYTES that
 * every GPU the library runs on holds until the process ends, instead of
 * buffers the library allocates.  It calls no hipMalloc / hipFree and no
 * allocating library routine.  The right-hand sides are processed in chunks
 * of as many as the array holds (at most 64); LM_EINVAL when it cannot hold
 * the workspace of one right-hand side (then use lm_matvec).  A dense
 * geometry needs no workspace.  Every call on a device shares that device's
 * array: calls that overlap on one device (any streams, any geometries) race
 * and must be serialised by the caller; calls on one geometry also share its
 * side stream, as with lm_matvec. */
#define LM_NOALLOC_SCRATCH_BYTES (256ull << 20)
lm_status lm_matvec_noalloc(lm_geom geom, int precision, int n_rhs, const void* x_dev, void* y_dev,
                            void* hip_stream);

/* y = M x for n_rhs vectors: M = P^{-1} = sum_B S_B Q_B P_B^{-1} R_B, the
 * overlapping domain-decomposition preconditioner of Sec. 4.2 (built by
 * lm_geometry_create with precond != 0), the operator GMRES applies on the
 * right (solve K M z = g, phi = M z).  LM_FP64 applies the FP64 rows;
 * LM_MIXED the binary16 copy on matrix cores, a fixed complex-linear operator
 * within about 1e-3 of the FP64 one (it only changes iteration counts).
 * x_dev, y_dev: device [n_rhs][N] complex128 for both precisions; x and y
 * must not overlap.  LM_EINVAL when the geometry has no preconditioner. */
lm_status lm_precond_apply(lm_geom geom, int precision, int n_rhs, const void* x_dev, void* y_dev, void* hip_stream);

/* The subdomains of the preconditioner (Sec. 4.2: a box B of a layer's
 * free-space tree, its own elements and the elements of B and its neighbour
 * boxes) as integer lists, host outputs.
 * info4_host (required): 4 int64 = number of subdomains S, tree level of the
 *   subdomain boxes (0 = the coarsest), total length of the neighbourhood
 *   lists, leaf level of the free-space trees.
 * jptr_host (S+1 int32), nb_host (S int32), jidx_host (info4[2] int32), each
 *   written when non-NULL (call once with NULLs to size them): the
 *   neighbourhood of subdomain b is jidx[jptr[b] .. jptr[b+1]) (element
 *   indices in input numbering); its first nb[b] entries are the elements of
 *   B itself, the rows of P_B^{-1} the preconditioner keeps, the rest those of
 *   the neighbour boxes.  Subdomains are ordered by (layer, column, row).
 * Errors: LM_EINVAL when the geometry has no preconditioner. */
lm_status lm_precond_subdomains(lm_geom geom, int64_t* info4_host, int32_t* jptr_host, int32_t* nb_host,
                                int32_t* jidx_host);

/* Runs reps FMM matvecs (as lm_matvec) and returns in out9_host the average
 * duration in ms of each stage, measured with HIP events recorded on
 * hip_stream around the stage's kernels: [0] P2M, [1] M2M, [2] M2L lists
 * (every level below the coarsest when the level-0 convolution is on, every
 * level otherwise; free-space and reaction; the translation kernel alone),
 * [3] L2L, [4] L2P, [5] near-field matrix (free-space near pairs, reaction
 * near pairs and self terms), [6] the sums of the M2L partial results per
 * target box (0 where the M2L writes its targets directly), [7] whole
 * matvec, [8] the level-0 convolution (forward transforms, frequency-domain
 * products, inverse transforms; 0 when it is off).  Synchronises the
 * stream.  LM_EINVAL for a dense geometry. */
lm_status lm_matvec_stage_times(lm_geom geom, int precision, int n_rhs, const void* x_dev, void* y_dev, int reps,
                                void* hip_stream, double* out9_host);

/* ------------------------------------------------------------------- rhs --
 * Dirichlet scatterers: g = -u^inc - u^b on Gamma_0 and -u^b elsewhere
 * (eq. homogeneousscattering); Neumann / Robin scatterers:
 * g = -(d_n + i beta)(u^inc + u^b) at the collocation points
 * for plane waves travelling along (cos t, -sin t), t = theta_host[r] in
 * radians, 0 < t < pi.  g_dev: device c128 [n_rhs][N]. */
lm_status lm_rhs(lm_geom geom, int n_rhs, const double* theta_host, void* g_dev, void* hip_stream);

/* ----------------------------------------------------------------- solve --
 * GMRES for K phi = g (Sec. 3.3, Sec. 5): x0 = 0, restarted every `restart`
 * iterations, right preconditioning by the domain-decomposition
 * preconditioner when precond != 0 and the geometry has one; stops when
 * ||g - K phi|| <= tol ||g|| for every right-hand side or after max_iter.
 * Arnoldi (classical Gram-Schmidt, two passes) and Givens rotations are FP64
 * for both precisions.  phi_dev: device c128 [n_rhs][N] (output).
 * reports_host: n_rhs entries (output).  Returns LM_NOT_CONVERGED if any
 * right-hand side missed the tolerance. */
typedef struct {
  double tol;
  int max_iter;
  int restart;
  int precond;
} lm_gmres_opts;
typedef struct {
  int iterations;
  double rel_residual;
} lm_solve_report;
lm_status lm_gmres_solve(lm_geom geom, int precision, int n_rhs, const double* theta_host,
                         const lm_gmres_opts* opts, void* phi_dev, lm_solve_report* reports_host,
                         void* hip_stream);
/* Same solver for caller-provided right-hand sides g_dev (device c128 [n_rhs][N]). */
lm_status lm_gmres_solve_rhs(lm_geom geom, int precision, int n_rhs, const void* g_dev,
                             const lm_gmres_opts* opts, void* phi_dev, lm_solve_report* reports_host,
                             void* hip_stream);

/* ------------------------------------------------------------- far field --
 * Far-field pattern of the scattered field (eq. integralrep in the
 * stationary-phase limit): for 0 < t < pi (top layer)
 *   u^s(R, t) ~ e^{i k_0 R}/sqrt(R) * u_inf(t),
 *   u_inf(t) = e^{-i pi/4} sqrt(k_0/2pi) sin t sum_e |Gamma_e| phi_e a_e(k_0 cos t),
 * and the mirror formula with k_L for pi < t < 2pi (bottom layer); a_e is the
 * spectral source factor of the free-space part and of every reaction
 * component reaching the top (bottom) layer.
 * phi_dev: device c128 [n_rhs][N]; obs_host: n_obs angles in radians (none
 * horizontal); out_dev: device c128 [n_rhs][n_obs]. */
lm_status lm_far_field(lm_geom geom, int n_rhs, const void* phi_dev, int n_obs, const double* obs_host,
                       void* out_dev, void* hip_stream);

/* --------------------------------------------------------- point sources --
 * The layered Green's function G(r | s) (Sec. 3.1, eq. layeredGreensfun:
 * the free-space part when r and s share a layer plus the reaction
 * components of eq. fourreactions) is the field at r of a unit point source
 * at s.  It satisfies every transmission condition and radiates, so with s
 * inside a scatterer its boundary values are the data of an exterior problem
 * whose solution is G(. | s) (the manufactured solution of Sec. 5, Example 1),
 * and with s outside every scatterer -G(. | s) on the boundary is the data of
 * a point-source incident field.
 *
 * lm_point_source_rhs: g[r][i] = G(c_i | s_r) at the collocation points for
 * n_src sources src_xy_host[2 r], src_xy_host[2 r + 1] (host; a source's layer
 * follows the element rule, ties to the upper layer); the reaction part by
 * direct Sommerfeld quadrature in FP64.  g_dev: device c128 [n_src][N].
 * Errors: LM_EINVAL for a non-finite source or one that coincides with a
 * collocation point. */
lm_status lm_point_source_rhs(lm_geom geom, int n_src, const double* src_xy_host, void* g_dev, void* hip_stream);
/* Far-field patterns of unit point sources (the far field of G(. | s_r), in
 * the convention of lm_far_field: u ~ e^{i k R}/sqrt(R) u_inf, top layer for
 * 0 < t < pi, bottom layer for pi < t < 2 pi).  out_dev: device c128
 * [n_src][n_obs]. */
lm_status lm_point_far_field(lm_layers layers, int n_src, const double* src_xy_host, int n_obs,
                             const double* obs_host, void* out_dev, void* hip_stream);

/* ------------------------------------------------------- off the boundary --
 * Scattered field at receivers off the boundary (eq. integralrep, unscaled
 * form): u^s(p) = sum_e |Gamma_e| phi_e G(p | c_e) with the layered Green's
 * function, for n_rhs densities phi_dev (device c128 [n_rhs][N], e.g. from
 * lm_gmres_solve) at n_pts receivers pts_xy_host (host, (x, y) pairs).
 * Free-space part by a direct sum over the elements of the receiver's layer
 * (O(N) per receiver); reaction part by the spectral form of the components:
 * source spectra sum_e |Gamma_e| phi_e e^{-+i lam x_e} e^{i k_{l',y} h_s(e)} on
 * the nodes of the Sommerfeld contour, then one pass over the nodes per
 * receiver.  The number of nodes grows like (extent of sources and receivers)
 * / (distance of the receiver to the interface its arriving waves come from),
 * receivers being grouped by that distance in powers of two.  FP64.
 * out_dev: device c128 [n_rhs][n_pts].  Errors: LM_EINVAL for a receiver
 * within 1e-4 of an interface or non-finite coordinates. */
lm_status lm_field(lm_geom geom, int n_rhs, const void* phi_dev, int n_pts, const double* pts_xy_host,
                   void* out_dev, void* hip_stream);
/* G(p | s_r) at n_pts receivers for n_src unit point sources (the same
 * evaluation with one term per source).  out_dev: device c128 [n_src][n_pts]. */
lm_status lm_point_field(lm_layers layers, int n_src, const double* src_xy_host, int n_pts,
                         const double* pts_xy_host, void* out_dev, void* hip_stream);

/* --------------------------------------------------------------- serving --
 * Request-serving loop with continuous batching (one worker thread per
 * server, on the device current at lm_server_create).  A request is a
 * geometry (owned by the caller; it must outlive the request and must not be
 * used by other calls while the server holds requests on it), n_rhs incidence
 * angles (one GMRES solve each, as lm_gmres_solve with the server's
 * precision) and optional far-field observation angles.  The worker advances
 * every admitted solve one Arnoldi step per round; solves on the same
 * geometry share one multi-right-hand-side launch per round, solves on
 * different geometries run on separate streams.  Krylov bases stay in device
 * memory (complex64 under LM_MIXED, where the charged footprint below, which
 * counts complex128 bases, is an upper bound).  Requests are admitted first-in first-out while the number of
 * active right-hand sides stays <= max_active_rhs and the estimated device
 * footprint of the admitted requests stays <= hbm_budget_bytes (basis,
 * work vectors and the per-right-hand-side FMM workspace; the geometry itself
 * is not counted).  Zero limits select 64 right-hand sides and 64 GiB.  The
 * device buffers of up to max_active_rhs finished solves are kept for reuse
 * by later solves with the same N and restart length; they count against the
 * same budget and are freed (those no admitted request can reuse first) when
 * an admission needs the room, when an allocation fails and at
 * lm_server_destroy.  The buffers of the fused launches of a geometry are
 * freed once none of its solves is admitted while other solves run; when the
 * last request leaves they are kept, with the per-round buffers, for 20 ms
 * and freed if no request arrives meanwhile (an admission keeps them only for
 * its own geometries and only within the budget), so the device memory the
 * server holds (lm_server_memory) stays within the budget.
 * All server entry points are thread-safe. */
typedef struct {
  int64_t hbm_budget_bytes;
  int max_active_rhs;
  int precision; /* LM_FP64 or LM_MIXED, for every request of the server */
  int precond_fp64; /* nonzero: an LM_MIXED server applies the preconditioner
                       with its FP64 rows instead of the binary16 copy */
} lm_server_opts;
typedef struct {
  lm_geom geom;
  int n_rhs;
  const double* theta_rad; /* host, n_rhs angles in (0, pi) */
  lm_gmres_opts gmres;
  int n_obs;               /* far-field angles (0: none) */
  const double* obs_rad;   /* host, n_obs angles, none horizontal */
} lm_request;
typedef enum { LM_QUEUED = 0, LM_RUNNING = 1, LM_DONE = 2, LM_FAILED = 3, LM_CANCELLED = 4 } lm_state;
lm_status lm_server_create(const lm_server_opts* opts, lm_server* out);
/* Copies the request and queues it; never blocks.  LM_EINVAL for invalid
 * numbers (NaN angles, bad options), LM_ENOMEM if the request can never be
 * admitted under the server's limits. */
lm_status lm_submit(lm_server server, const lm_request* request, uint64_t* request_id);
/* State of a request; once LM_DONE, copies its reports (n_rhs), phi (host
 * c128 [n_rhs][N]) and far field (host c128 [n_rhs][n_obs]) into the
 * non-NULL outputs and returns the solve status (LM_OK or LM_NOT_CONVERGED).
 * latency_s: seconds from submission to completion (or to now while
 * pending).  Returns LM_ECANCELLED for a cancelled request, the failure
 * status for a failed one, LM_ENOTFOUND for an unknown id. */
lm_status lm_poll(lm_server server, uint64_t request_id, lm_state* state, lm_solve_report* reports_host,
                  double* latency_s, void* phi_host, void* far_field_host);
/* Cancels a queued or running request (running ones stop at the next round). */
lm_status lm_cancel(lm_server server, uint64_t request_id);
/* Frees a finished, failed or cancelled request's results. */
lm_status lm_release(lm_server server, uint64_t request_id);
/* The device footprint the server charges for a request of n_rhs solves on
 * geom with these GMRES options (Krylov basis, work vectors, FMM workspace). */
lm_status lm_request_footprint(lm_geom geom, int n_rhs, const lm_gmres_opts* gmres, int64_t* bytes);
/* Host output of 6 int64: queued requests, active right-hand sides, admitted
 * footprint bytes, rounds, fused K M launches, right-hand sides in them. */
lm_status lm_server_stats(lm_server server, int64_t* out6);
/* Host output of 3 int64: device bytes the server's own buffers hold now
 * (Krylov bases and work vectors of admitted and spare solves, fused-launch
 * buffers, round buffers; not the geometries), the part held by spare
 * solves, and the admitted footprint (as lm_server_stats). */
lm_status lm_server_memory(lm_server server, int64_t* out3);
/* Host output of 11 doubles accumulated over the server's rounds, measured
 * with HIP events on the streams the kernels run on: [0] ms in the fused
 * K M phase (gathers, preconditioner, matvecs; every geometry stream
 * joined), [1] ms in the Gram-Schmidt phase (classical Gram-Schmidt with a
 * delayed second pass: one dot pass and one update pass over each basis,
 * plus the norms), [2] bytes that phase must move at minimum: per Arnoldi
 * column at step j, with b = 16 bytes per basis element (LM_FP64) or 8
 * (LM_MIXED: the Krylov basis is stored in complex64, every sum is
 * accumulated in FP64), (2 j + 5) N b + 2 N x 16 (dot pass: V[0..j], u and
 * the K M output; update pass: V[0..j-1], u and the K M output read, v_j
 * and the next vector written; at j = 0 one more N x 16 for the norm of the
 * K M output); [3] ms in the M2L
 * launches of the fused FMM matvecs (first launch of each geometry stream
 * per round), [4] their algorithmic flops, 8 (2p+1)^2 R per M2L list entry,
 * [5] the number of those launches, [6] host wall-clock ms of the rounds
 * (everything but finishing columns), [7] host wall-clock ms spent finishing
 * columns (phi = M z, far field, copies to host memory); the rounds' host
 * time split: [8] ms queueing a round's copies and kernels, [9] ms blocked
 * in the round's one wait (for the dot products and norms), [10] ms of the
 * host step after it (Hessenberg columns, rotations, coefficients) up to the
 * queued update pass. */
lm_status lm_server_phase_times(lm_server server, double* out11);
/* Cancels everything in flight, joins the worker and frees the server. */
lm_status lm_server_destroy(lm_server server);

#ifdef __cplusplus
}
#endif

#endif /* LMFMM_H */
