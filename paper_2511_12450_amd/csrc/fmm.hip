// Layered-medium fast multipole matvec (Sec. 4.1 of the paper).
//
// y = K x with K the unscaled Nystrom matrix (eq. Llayerscomponent):
//   free-space part  -- one quadtree per layer over its elements, classical
//                       Helmholtz FMM (P2M, M2M, M2L, L2L, L2P, near P2P);
//   reaction part    -- for each of the 4L^2 components (target side,
//                       source side) an FMM between the two "side trees":
//                       quadtrees in (x, h) where h is the distance to the
//                       interface of that side (the effective location of
//                       targets / polarization coordinate of sources of
//                       eqs. equivalent_imag_for_source/_for_target, measured
//                       from the interface), with M2L operators built from
//                       Sommerfeld-quadrature tables (eq. metoleimage);
//   self terms       -- I^s (eq. ApproximateComputation).
//
// Tree layout.  All trees share one x-grid (origin x0) and the level widths
// w_l = w_top / 2^l; rows count from h = 0.  A free-space tree refines
// uniformly to level lf.  A side tree refines only boxes of row 0 (those
// touching the interface): in image space (target at +h, source image at -h)
// only row-0 boxes of both trees are ever adjacent, so every other box is a
// leaf; the finest level lr is about one element length wide, which leaves
// only pairs of elements within one element length of the same interface in
// the near field.  Interaction lists at level l >= 1 are the children of
// image-adjacent parents that are not image-adjacent themselves (25 classes
// per level and component: dx in -3..3 boxes, rows 0/1 each); at level 0
// every non-adjacent pair interacts.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <unordered_map>

#include "block_mfma.hpp"
#include "fmm_math.hpp"
#include "lm_internal.hpp"
#include "m2l_table.hpp"

#include "fmm_plan.hpp"

namespace {
// Top-level box width times the largest wavenumber.  Level 0 interacts all
// pairs of non-adjacent boxes, so a wide top level keeps that quadratic list
// short; the box radius k w / sqrt(2) = 5.7 stays well inside the range where
// order p = 20 expansions converge to FP64 accuracy.
constexpr double LM_TOP_KW = 8.0;
constexpr int LM_PTS_ITEM = 64;  // points per P2M / L2P work item
constexpr int WG = 64;
constexpr int MAXPP = 2 * MAXP + 1;
static_assert(LM_PTS_ITEM <= PA_ROWS && MAXPP <= PA_ROWS, "P2M / L2P items must fit one matrix-core block");
inline int64_t bkey(int i, int j) { return ((int64_t)i << 32) | (uint32_t)j; }
}  // namespace

void fmm_free(FmmPlan* f) { delete f; }
int64_t fmm_bytes(const FmmPlan* f) { return f ? f->bytes() : 0; }
void fmm_stats(const FmmPlan* f, int64_t* out) {
  for (int i = 0; i < 10; ++i) out[i] = f ? f->stats[i] : 0;
}

// =========================================================== setup kernels ==
//
// Scaled expansions.  With s = k w_l / 2 for a box of level l in a tree of
// wavenumber k and sig_n = s^|n| / |n|!, the library stores
//   ME  at_n = a_n / sig_n   (|at_n| <~ |q| (rho/w)^|n|),
//   LE  bt_m = b_m * sig_m   (|bt_m| <~ (w/R)^|m|),
// and every translation operator carries the matching factors, so all stored
// numbers stay within a few orders of magnitude of one and FP32 holds them.
// Operators are stored column-major by input index: out_i = sum_j Op[j][i] in_j.

__device__ __forceinline__ double sigma_of(const double* sig, int p, int layer, int nlev, int level, int n) {
  return sig[(int64_t)(layer * nlev + level) * (p + 1) + (n < 0 ? -n : n)];
}

// Free-space M2L operator per class: Op[n][m] = sig^t_m (i/4) G_{n-m}(c_t - c_s) sig^s_n.
__global__ void __launch_bounds__(64) k_free_tables(int p, int nlev, const double* __restrict__ geo,
                                                    const int* __restrict__ lvl, const double* __restrict__ sig,
                                                    double2* __restrict__ out) {
  const int t = blockIdx.x;
  const int P = 2 * p + 1, J = 2 * p;
  __shared__ double2 G[4 * MAXP + 1];
  if (threadIdx.x == 0) {
    zd g[4 * MAXP + 1];
    zd hb[2 * MAXP + 1];
    fm::g_seq(geo[3 * t], geo[3 * t + 1], geo[3 * t + 2], J, g, hb);
    for (int j = 0; j <= 2 * J; ++j) G[j] = make_double2(g[j].re, g[j].im);
  }
  __syncthreads();
  const int layer = lvl[2 * t], level = lvl[2 * t + 1];
  for (int idx = threadIdx.x; idx < P * P; idx += 64) {
    const int n = idx / P - p, mm = idx % P - p;
    const double sc = 0.25 * sigma_of(sig, p, layer, nlev, level, mm) * sigma_of(sig, p, layer, nlev, level, n);
    const double2 gv = G[n - mm + 2 * p];
    out[(int64_t)t * P * P + idx] = make_double2(-gv.y * sc, gv.x * sc);  // (i/4) G
  }
}

// Reaction M2L operator per class: one workgroup per table, nodes in chunks;
// the scale factors of the target and source levels are applied on output.
constexpr int TAB_CHUNK = 16;
__global__ void __launch_bounds__(256) k_reac_tables(MediumDev m, int p, int nlev, const int* __restrict__ meta,
                                                     const double* __restrict__ geo, const double* __restrict__ sig,
                                                     double2* __restrict__ out) {
  const int t = blockIdx.x;
  const int P = 2 * p + 1;
  const int lt = meta[4 * t], ls = meta[4 * t + 1], comp = meta[4 * t + 2], level = meta[4 * t + 3];
  const double dx = geo[3 * t], ht = geo[3 * t + 1], hs = geo[3 * t + 2];
  __shared__ double2 A[TAB_CHUNK][MAXPP];
  __shared__ double2 B[TAB_CHUNK][MAXPP];
  ClassNodes cn;
  class_nodes(cn, m.kmax, dx, ht + hs, p);
  const int Q = cn.total();
  constexpr int EPT = (MAXPP * MAXPP + 255) / 256;
  zd acc[EPT];
  for (int q0 = 0; q0 < Q; q0 += TAB_CHUNK) {
    const int tid = threadIdx.x;
    if (tid < TAB_CHUNK) {
      const int q = q0 + tid;
      if (q < Q) {
        zd f, a, ai, b, bi;
        class_factor(m, lt, ls, comp, cn, ht, hs, q, f, a, ai, b, bi);
        zd up = f, dn = f;
        A[tid][p] = make_double2(f.re, f.im);
        for (int j = 1; j <= p; ++j) {
          up = up * a;
          dn = dn * ai;
          A[tid][p + j] = make_double2(up.re, up.im);
          A[tid][p - j] = make_double2(dn.re, dn.im);
        }
        zd nb = -b, nbi = -bi;
        up = zd(1.0, 0.0);
        dn = zd(1.0, 0.0);
        B[tid][p] = make_double2(1.0, 0.0);
        for (int j = 1; j <= p; ++j) {
          up = up * nb;
          dn = dn * nbi;
          B[tid][p + j] = make_double2(up.re, up.im);
          B[tid][p - j] = make_double2(dn.re, dn.im);
        }
      } else {
        for (int j = 0; j < P; ++j) {
          A[tid][j] = make_double2(0.0, 0.0);
          B[tid][j] = make_double2(0.0, 0.0);
        }
      }
    }
    __syncthreads();
    for (int e = 0; e < EPT; ++e) {
      const int idx = threadIdx.x + 256 * e;
      if (idx >= P * P) break;
      const int n = idx / P, mm = idx % P;  // column-major: [n][m]
      zd s = acc[e];
      for (int q = 0; q < TAB_CHUNK; ++q) {
        const double2 x = A[q][mm], y = B[q][n];
        s.re += x.x * y.x - x.y * y.y;
        s.im += x.x * y.y + x.y * y.x;
      }
      acc[e] = s;
    }
    __syncthreads();
  }
  for (int e = 0; e < EPT; ++e) {
    const int idx = threadIdx.x + 256 * e;
    if (idx >= P * P) break;
    const int n = idx / P - p, mm = idx % P - p;
    const double sc = sigma_of(sig, p, lt, nlev, level, mm) * sigma_of(sig, p, ls, nlev, level, n);
    out[(int64_t)t * P * P + idx] = make_double2(acc[e].re * sc, acc[e].im * sc);
  }
}

// Free-space kernel seen by target i: (i/4) H_0(k r) for Dirichlet
// scatterers, n_i . grad + i beta of it for sound-hard / impedance ones
// (grad_i (i/4) H_0(k r) = -(i/4) k H_1(k r) (c_i - c_e) / r).
struct BcTarget {
  int bc;
  double beta;
  const double *nx, *ny;
};
__device__ __forceinline__ zd free_kernel(double k, double dx, double dy, int i, const BcTarget& t) {
  const double r = hypot(dx, dy), kr = k * r;
  const zd g(-0.25 * y0(kr), 0.25 * j0(kr));
  if (t.bc == LM_BC_DIRICHLET) return g;
  const zd d = zd(0.25 * y1(kr), -0.25 * j1(kr)) * (k / r);
  return d * (dx * t.nx[i] + dy * t.ny[i]) + zd(0.0, t.beta) * g;
}

// Near-field matrix values: kind 0 free-space pair, all ones self term,
// otherwise the component mask of a reaction pair.
__global__ void k_near_values(MediumDev m, int64_t n, const int* __restrict__ tgt, const int* __restrict__ src,
                              const unsigned* __restrict__ kind, const double* __restrict__ cx,
                              const double* __restrict__ cy, const double* __restrict__ w,
                              const int* __restrict__ lay, const double2* __restrict__ self, BcTarget bt,
                              double2* __restrict__ val) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int i = tgt[t], e = src[t];
  const unsigned kd = kind[t];
  zd v(0.0, 0.0);
  if (kd == 0u) {
    v = free_kernel(m.k[lay[i]], cx[i] - cx[e], cy[i] - cy[e], i, bt) * w[e];
  } else if (kd == 0xFFFFFFFFu) {
    const double2 sv = self[i];
    v = zd(sv.x, sv.y);
  } else if (bt.bc == LM_BC_DIRICHLET) {
    v = lmq::reaction_direct(m, lay[i], lay[e], fabs(cx[i] - cx[e]), cy[i], cy[e], kd) * w[e];
  } else {
    zd g, gx, gy;
    lmq::reaction_direct_grad(m, lay[i], lay[e], cx[i] - cx[e], cy[i], cy[e], g, gx, gy, kd);
    v = (gx * bt.nx[i] + gy * bt.ny[i] + zd(0.0, bt.beta) * g) * w[e];
  }
  val[t] = make_double2(v.re, v.im);
}

// Free-space near field + self term as dense blocks, one workgroup per leaf:
// Z_B[r][jj] = self term if J[jj] is the row's element, else the free-space
// kernel (i/4) H_0(k |c_i - c_e|) |Gamma_e| (FP64, stored complex64).
__global__ void k_near_block_values(MediumDev m, const int* __restrict__ jptr, const int* __restrict__ jidx,
                                    const int* __restrict__ nb, const int64_t* __restrict__ zoff,
                                    const double* __restrict__ cx, const double* __restrict__ cy,
                                    const double* __restrict__ w, const int* __restrict__ lay,
                                    const double2* __restrict__ self, BcTarget bt, float2* __restrict__ Z) {
  const int b = blockIdx.x;
  const int* J = jidx + jptr[b];
  const int q = jptr[b + 1] - jptr[b], nB = nb[b];
  float2* Zb = Z + zoff[b];
  for (int64_t idx = threadIdx.x; idx < (int64_t)nB * q; idx += blockDim.x) {
    const int r = (int)(idx / q), jj = (int)(idx % q);
    const int i = J[r], e = J[jj];
    zd v;
    if (i == e) {
      const double2 sv = self[i];
      v = zd(sv.x, sv.y);
    } else {
      v = free_kernel(m.k[lay[i]], cx[i] - cx[e], cy[i] - cy[e], i, bt) * w[e];
    }
    Zb[idx] = make_float2((float)v.re, (float)v.im);
  }
}

// Spectral rule, pairs (i, e != i) of one scatterer: the spectral entry minus
// the trapezoidal w_e G^f the rest of the matvec computes for the pair.  The
// Hankel parts cancel:
//   -J_0(k r) |x'_e| / (4 pi) (R_d - (2 pi / M) ln(4 sin^2(pi d / M))),
// d = (i - e) mod M.
__global__ void k_spectral_corr(MediumDev m, int64_t n, const int* __restrict__ tgt, const int* __restrict__ src,
                                const double* __restrict__ cx, const double* __restrict__ cy,
                                const int* __restrict__ lay, const int* __restrict__ sid, const int* __restrict__ loc,
                                const int* __restrict__ cnt, const double* __restrict__ speed,
                                const double* __restrict__ logw, const int64_t* __restrict__ roff,
                                double2* __restrict__ val) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int i = tgt[t], e = src[t];
  const int M = cnt[i], d = ((loc[i] - loc[e]) % M + M) % M;
  const double kr = m.k[lay[i]] * hypot(cx[i] - cx[e], cy[i] - cy[e]);
  const double sn = sin(M_PI * d / M);
  const double v = -j0(kr) * speed[e] / (4.0 * M_PI) * (logw[roff[sid[i]] + d] - 2.0 * M_PI / M * log(4.0 * sn * sn));
  val[t] = make_double2(v, 0.0);
}

__global__ void k_c128_to_c64_fmm(int64_t n, const double2* __restrict__ a, float2* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = make_float2((float)a[i].x, (float)a[i].y);
}

// ========================================================== matvec kernels ==
// Templated on the storage/arithmetic type RT (double: LM_FP64, float:
// LM_MIXED) with R right-hand sides per launch (R <= LM_RCHUNK).  Expansions
// are stored [box][2p+1][R] and vectors [R][N].  A workgroup owns the (2p+1) R
// outputs of one box; thread t holds outputs t, t + blockDim, ... (at most
// MO of them) in registers, in fully unrolled loops so they stay in VGPRs.

constexpr int LM_RCHUNK = 64;
constexpr int MO = 16;          // (2p+1) R <= MO * 256 for p <= 31, R <= 64

template <typename RT> struct C2T;
template <> struct C2T<double> { typedef double2 T; };
template <> struct C2T<float> { typedef float2 T; };

// re + i im += a b as four chained FMAs.
template <typename RT, typename V>
__device__ __forceinline__ void cmac(RT& re, RT& im, V a, V b) {
  re = fma(a.x, b.x, re);
  re = fma(-a.y, b.y, re);
  im = fma(a.x, b.y, im);
  im = fma(a.y, b.x, im);
}

template <typename V, typename RT>
__device__ __forceinline__ V mk(RT re, RT im) {
  V o;
  o.x = re;
  o.y = im;
  return o;
}

// Bessel values J_j(k rho)/sig_j and e^{+-i j theta}, j = 0..p, for one point
// into LDS rows (FP64 evaluation, stored in RT).
template <typename RT>
__device__ __forceinline__ void point_basis(double k, double dx, double dh, int p, const double* sg, double sign,
                                            RT* js, typename C2T<RT>::T* cs) {
  double J[MAXP + 1];
  fm::bessel_j_seq(k * hypot(dx, dh), p, J);
  const zd e1 = fm::cis(sign * atan2(dh, dx));
  zd ep(1.0, 0.0);
  for (int j = 0; j <= p; ++j) {
    js[j] = (RT)(J[j] / sg[j]);
    cs[j] = mk<typename C2T<RT>::T>((RT)ep.re, (RT)ep.im);
    ep = ep * e1;
  }
}

// P2M: at_n = sum_s q_s J_n(k rho_s) e^{-i n theta_s} / sig_n, q_s = |Gamma_s| x_s.
// Points are taken PCH at a time (64 with one right-hand side, else 32).
// One workgroup per work item (leaf box, first point, count <= LM_PTS_ITEM);
// the partial expansions of a leaf's items are summed by k_p2m_reduce.
template <typename RT, int PCH>
__global__ void __launch_bounds__(256) k_p2m(int p, int R, int nlev, const int* __restrict__ items,
                                             const BoxDev* __restrict__ boxes, const int* __restrict__ tree_layer,
                                             const double* __restrict__ sig, const int* __restrict__ pt_elem,
                                             const double2* __restrict__ pt_xh, const double* __restrict__ w,
                                             const typename C2T<RT>::T* __restrict__ x, int N,
                                             typename C2T<RT>::T* __restrict__ part) {
  typedef typename C2T<RT>::T V;
  const int b = items[3 * blockIdx.x];
  BoxDev B = boxes[b];
  B.pt0 = items[3 * blockIdx.x + 1];
  B.npt = items[3 * blockIdx.x + 2];
  const int P = 2 * p + 1, PR = P * R;
  const double* sg = sig + (int64_t)(tree_layer[B.tree] * nlev + B.level) * (p + 1);
  __shared__ RT js[PCH][MAXP + 1];
  __shared__ V cs[PCH][MAXP + 1];
  extern __shared__ unsigned char dyn[];
  V* qs = reinterpret_cast<V*>(dyn);  // [PCH][R]
  RT are[MO], aim[MO];
#pragma unroll
  for (int i = 0; i < MO; ++i) are[i] = aim[i] = RT(0);
  for (int s0 = 0; s0 < B.npt; s0 += PCH) {
    const int cnt = min(PCH, B.npt - s0);
    __syncthreads();
    if (threadIdx.x < (unsigned)cnt) {
      const double2 xh = pt_xh[B.pt0 + s0 + threadIdx.x];
      point_basis<RT>(B.k, xh.x - B.cx, xh.y - B.ch, p, sg, -1.0, js[threadIdx.x], cs[threadIdx.x]);
    }
    for (int idx = threadIdx.x; idx < cnt * R; idx += blockDim.x) {
      const int j = idx / R, r = idx - j * R;
      const int e = pt_elem[B.pt0 + s0 + j];
      const V xv = x[(int64_t)r * N + e];
      const RT we = (RT)w[e];
      qs[idx] = mk<V>(xv.x * we, xv.y * we);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MO; ++i) {
      const int idx = threadIdx.x + i * blockDim.x;
      if (idx < PR) {
        const int n = idx / R - p, r = idx % R;
        const int an = n < 0 ? -n : n;
        const RT sn = (n < 0 && (an & 1)) ? RT(-1) : RT(1);
        const RT cj = n < 0 ? RT(-1) : RT(1);  // e^{-i n th} = conj(e^{-i |n| th}) for n < 0
        RT re = are[i], im = aim[i];
        for (int j = 0; j < cnt; ++j) {
          const V c = cs[j][an];
          const RT jv = js[j][an] * sn;
          const V q = qs[j * R + r];
          const RT cy = c.y * cj;
          re += jv * (c.x * q.x - cy * q.y);
          im += jv * (c.x * q.y + cy * q.x);
        }
        are[i] = re;
        aim[i] = im;
      }
    }
  }
#pragma unroll
  for (int i = 0; i < MO; ++i) {
    const int idx = threadIdx.x + i * blockDim.x;
    if (idx < PR) part[(int64_t)blockIdx.x * PR + idx] = mk<V>(are[i], aim[i]);
  }
}

// me[leaf] = sum of the partial expansions of its work items.
template <typename RT>
__global__ void __launch_bounds__(256) k_p2m_reduce(int PR, const int* __restrict__ leaves,
                                                    const int* __restrict__ ptr, const int* __restrict__ sel,
                                                    const typename C2T<RT>::T* __restrict__ part,
                                                    typename C2T<RT>::T* __restrict__ me) {
  typedef typename C2T<RT>::T V;
  const int k = sel ? sel[blockIdx.x] : (int)blockIdx.x;  // sel: a subset of the outputs
  const int i0 = ptr[k], i1 = ptr[k + 1];
  V* out = me + (int64_t)leaves[k] * PR;
  for (int idx = threadIdx.x; idx < PR; idx += blockDim.x) {
    RT re = 0, im = 0;
    int i = i0;
    for (; i + 4 <= i1; i += 4) {  // four partial loads in flight, summed in order
      V v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = part[(int64_t)(i + u) * PR + idx];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        re += v[u].x;
        im += v[u].y;
      }
    }
    for (; i < i1; ++i) {
      const V v = part[(int64_t)i * PR + idx];
      re += v.x;
      im += v.y;
    }
    out[idx] = mk<V>(re, im);
  }
}

// acc[o][r] += sum_j Op[j][o] in[j][r] for this thread's outputs; Op is
// column-major by input (global), in is [P][R] in LDS.
template <typename RT>
__device__ __forceinline__ void op_apply(int P, int R, const typename C2T<RT>::T* __restrict__ Op,
                                         const typename C2T<RT>::T* in, RT* are, RT* aim) {
  const int PR = P * R;
#pragma unroll
  for (int i = 0; i < MO; ++i) {
    const int idx = threadIdx.x + i * blockDim.x;
    if (idx < PR) {
      const int o = idx / R, r = idx - o * R;
      RT re = are[i], im = aim[i];
      const typename C2T<RT>::T* op = Op + o;
      int j = 0;
      for (; j + 8 <= P; j += 8) {  // eight operator loads in flight
        typename C2T<RT>::T t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) t[u] = op[(int64_t)(j + u) * P];
#pragma unroll
        for (int u = 0; u < 8; ++u) cmac(re, im, t[u], in[(j + u) * R + r]);
      }
      for (; j < P; ++j) cmac(re, im, op[(int64_t)j * P], in[j * R + r]);
      are[i] = re;
      aim[i] = im;
    }
  }
}

template <typename RT>
__device__ __forceinline__ void acc_zero(RT* are, RT* aim) {
#pragma unroll
  for (int i = 0; i < MO; ++i) are[i] = aim[i] = RT(0);
}

template <typename RT>
__device__ __forceinline__ void acc_store(int PR, const RT* are, const RT* aim, typename C2T<RT>::T* out) {
#pragma unroll
  for (int i = 0; i < MO; ++i) {
    const int idx = threadIdx.x + i * blockDim.x;
    if (idx < PR) out[idx] = mk<typename C2T<RT>::T>(are[i], aim[i]);
  }
}

// M2M: parent at = sum over children of Op_child at_child.
template <typename RT>
__global__ void __launch_bounds__(256) k_m2m(int p, int R, int nlev, const int* __restrict__ parents,
                                             const BoxDev* __restrict__ boxes, const int* __restrict__ children,
                                             const int* __restrict__ tree_layer,
                                             const typename C2T<RT>::T* __restrict__ ops,
                                             typename C2T<RT>::T* __restrict__ me) {
  typedef typename C2T<RT>::T V;
  const int b = parents[blockIdx.x];
  const BoxDev B = boxes[b];
  const int P = 2 * p + 1, PR = P * R;
  extern __shared__ unsigned char dyn[];
  V* a = reinterpret_cast<V*>(dyn);  // [P][R]
  RT are[MO], aim[MO];
  acc_zero(are, aim);
  for (int c = 0; c < B.nchild; ++c) {
    const int cb = children[B.child0 + c];
    const BoxDev C = boxes[cb];
    __syncthreads();
    for (int idx = threadIdx.x; idx < PR; idx += blockDim.x) a[idx] = me[(int64_t)cb * PR + idx];
    __syncthreads();
    const V* Op = ops + ((int64_t)((tree_layer[C.tree] * nlev + C.level) * 4 + C.pos)) * P * P;
    op_apply<RT>(P, R, Op, a, are, aim);
  }
  acc_store(PR, are, aim, me + (int64_t)b * PR);
}

// M2L, target-major: each target box sums Op_entry at_source over its list.
template <typename RT>
__global__ void __launch_bounds__(256) k_m2l_target(int p, int R, const int* __restrict__ tgts,
                                                    const int* __restrict__ ptr, const int* __restrict__ src,
                                                    const int* __restrict__ opi,
                                                    const typename C2T<RT>::T* __restrict__ ops,
                                                    const typename C2T<RT>::T* __restrict__ me,
                                                    typename C2T<RT>::T* __restrict__ le) {
  typedef typename C2T<RT>::T V;
  const int P = 2 * p + 1, PR = P * R;
  extern __shared__ unsigned char dyn[];
  V* a = reinterpret_cast<V*>(dyn);  // [P][R]
  RT are[MO], aim[MO];
  acc_zero(are, aim);
  for (int e = ptr[blockIdx.x]; e < ptr[blockIdx.x + 1]; ++e) {
    __syncthreads();
    const int s = src[e];
    for (int idx = threadIdx.x; idx < PR; idx += blockDim.x) a[idx] = me[(int64_t)s * PR + idx];
    __syncthreads();
    op_apply<RT>(P, R, ops + (int64_t)opi[e] * P * P, a, are, aim);
  }
  acc_store(PR, are, aim, le + (int64_t)tgts[blockIdx.x] * PR);
}

// ---- level-0 convolution along x (see the plan) ---------------------------
// A workgroup transforms CH = 2^lgc columns of one row, of length L = 2^lgL,
// held in LDS as buf[k][c].  Radix-2, decimation in time: inputs are stored
// at bit-reversed positions, then log2 L butterfly passes; tw[t] =
// exp(-2 pi i t / L) for t < L / 2 (conjugated for the inverse).
__device__ __forceinline__ int top_brev(int k, int lgL) { return (int)(__brev((unsigned)k) >> (32 - lgL)); }

template <typename V, bool INV>
__device__ void top_fft_lds(V* buf, int lgL, int lgc, const V* __restrict__ tw) {
  const int L = 1 << lgL, nb = (L >> 1) << lgc;
  for (int lh = 0; lh < lgL; ++lh) {
    __syncthreads();
    const int half = 1 << lh;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
      const int c = b & ((1 << lgc) - 1), bf = b >> lgc;
      const int j = bf & (half - 1), grp = bf >> lh;
      const int i0 = ((grp << (lh + 1)) + j) << lgc | c, i1 = i0 + (half << lgc);
      V w = tw[j << (lgL - 1 - lh)];
      if (INV) w.y = -w.y;
      const V a = buf[i0], x = buf[i1];
      V t;
      t.x = w.x * x.x - w.y * x.y;
      t.y = w.x * x.y + w.y * x.x;
      buf[i0] = mk<V>(a.x + t.x, a.y + t.y);
      buf[i1] = mk<V>(a.x - t.x, a.y - t.y);
    }
  }
  __syncthreads();
}

// Forward transform of the level-0 expansions of row blockIdx.y, columns
// [CH blockIdx.x, +CH) of the P x R block: mh[row][f][c].
template <typename V>
__global__ void __launch_bounds__(256) k_top_fwd(int lgL, int lgc, int nx, int PR, const int* __restrict__ grid,
                                                 const V* __restrict__ me, const V* __restrict__ tw,
                                                 V* __restrict__ mh) {
  extern __shared__ unsigned char dyn[];
  V* buf = reinterpret_cast<V*>(dyn);
  const int L = 1 << lgL, CH = 1 << lgc, r = blockIdx.y, c0 = blockIdx.x * CH;
  for (int idx = threadIdx.x; idx < (L << lgc); idx += blockDim.x) {
    const int k = idx >> lgc, c = idx & (CH - 1);
    V v = mk<V>(0, 0);
    if (k < nx && c0 + c < PR) {
      const int b = grid[(int64_t)r * nx + k];
      if (b >= 0) v = me[(int64_t)b * PR + c0 + c];
    }
    buf[(top_brev(k, lgL) << lgc) | c] = v;
  }
  top_fft_lds<V, false>(buf, lgL, lgc, tw);
  for (int idx = threadIdx.x; idx < (L << lgc); idx += blockDim.x) {
    const int k = idx >> lgc, c = idx & (CH - 1);
    if (c0 + c < PR) mh[((int64_t)r * L + k) * PR + c0 + c] = buf[idx];
  }
}

// Inverse transform of row blockIdx.y of lh[row][f][c], scaled by 1/L, into
// the local expansions of that row's level-0 boxes (written, not added: a
// level-0 box has no other M2L source).
template <typename V>
__global__ void __launch_bounds__(256) k_top_inv(int lgL, int lgc, int nx, int PR, const int* __restrict__ grid,
                                                 const V* __restrict__ lh, const V* __restrict__ tw,
                                                 V* __restrict__ le) {
  extern __shared__ unsigned char dyn[];
  V* buf = reinterpret_cast<V*>(dyn);
  const int L = 1 << lgL, CH = 1 << lgc, r = blockIdx.y, c0 = blockIdx.x * CH;
  for (int idx = threadIdx.x; idx < (L << lgc); idx += blockDim.x) {
    const int k = idx >> lgc, c = idx & (CH - 1);
    V v = mk<V>(0, 0);
    if (c0 + c < PR) v = lh[((int64_t)r * L + k) * PR + c0 + c];
    buf[(top_brev(k, lgL) << lgc) | c] = v;
  }
  top_fft_lds<V, true>(buf, lgL, lgc, tw);
  const double sc = 1.0 / L;
  for (int idx = threadIdx.x; idx < (nx << lgc); idx += blockDim.x) {
    const int k = idx >> lgc, c = idx & (CH - 1);
    const int b = grid[(int64_t)r * nx + k];
    if (b >= 0 && c0 + c < PR) {
      const V v = buf[idx];
      le[(int64_t)b * PR + c0 + c] = mk<V>(v.x * sc, v.y * sc);
    }
  }
}

// le[box] = 0 for the boxes of the list (those whose local expansion no
// M2L or level-0 launch writes; the L2L adds into it).
template <typename V>
__global__ void __launch_bounds__(256) k_zero_boxes(int PR, const int* __restrict__ boxes, V* __restrict__ le) {
  V* o = le + (int64_t)boxes[blockIdx.x] * PR;
  for (int idx = threadIdx.x; idx < PR; idx += blockDim.x) o[idx] = mk<V>(0, 0);
}

// Transformed operator sequences (setup, FP64): class blockIdx.y, operator
// entries [CH blockIdx.x, +CH) of P x P.  Offset di in [-(nx-1), nx-1] sits at
// position di mod L; the adjacent offsets of a near class are zero.
__global__ void __launch_bounds__(256) k_top_tables(int lgL, int lgc, int nx, int PP, const double2* __restrict__ tab,
                                                    const int* __restrict__ near, const double2* __restrict__ tw,
                                                    double2* __restrict__ out64, float2* __restrict__ out32) {
  extern __shared__ unsigned char dyn[];
  double2* buf = reinterpret_cast<double2*>(dyn);
  const int L = 1 << lgL, CH = 1 << lgc, cls = blockIdx.y, c0 = blockIdx.x * CH, D = 2 * nx - 1;
  const bool nr = near[cls] != 0;
  for (int idx = threadIdx.x; idx < (L << lgc); idx += blockDim.x) {
    const int k = idx >> lgc, c = idx & (CH - 1);
    const int di = k < nx ? k : (k > L - nx ? k - L : L);
    double2 v = make_double2(0.0, 0.0);
    if (di < L && c0 + c < PP && !(nr && di >= -1 && di <= 1))
      v = tab[((int64_t)cls * D + di + nx - 1) * PP + c0 + c];
    buf[(top_brev(k, lgL) << lgc) | c] = v;
  }
  top_fft_lds<double2, false>(buf, lgL, lgc, tw);
  for (int idx = threadIdx.x; idx < (L << lgc); idx += blockDim.x) {
    const int k = idx >> lgc, c = idx & (CH - 1);
    if (c0 + c < PP) {
      const int64_t o = ((int64_t)cls * L + k) * PP + c0 + c;
      out64[o] = buf[idx];
      out32[o] = make_float2((float)buf[idx].x, (float)buf[idx].y);
    }
  }
}

// Columns per workgroup of the level-0 transforms: the largest power of two
// <= 64 whose L x CH block fits 32 KiB of LDS.
inline int top_lgc(int lgL, size_t elem) {
  int lgc = 6;
  while (lgc > 0 && ((size_t)1 << (lgL + lgc)) * elem > 32768) --lgc;
  return lgc;
}

// Translations with matrix cores (FP32, several right-hand sides): M2L, and
// M2M / L2L as items of one parent or child.  A work item (target, first
// entry, end) sums Op_e a_src(e) over its entries; per entry the operator T
// (P x P complex, [n][m] = column n of the input) and the source expansion a
// (P x R complex, [n][j]) are copied to LDS as they lie in memory (flat,
// coalesced, MF_ST loads in flight per lane), and the complex product is
// formed in 16x16x4 FP32 MFMA tiles (FP32 accumulation) by the
// three-multiplication form T1 = Re T Re a, T2 = Im T Im a,
// T3 = (Re T + Im T)(Re a + Im a), T a = (T1 - T2) + i (T3 - T1 - T2): a tile
// is 16 output coefficients x 16 right-hand sides, a k-step 4 input
// coefficients (A[i][k] = T[n][m] with m = lane % 16, n = lane / 16), each
// fragment one 64-bit LDS load.  K is padded to whole k-steps by zero rows
// of a placed after the staged data (rows beyond P read finite staged values
// times those zeros); output rows beyond P are clamped duplicates that are
// not stored.  Each wavefront holds 3 row tiles (48 coefficients) of one
// column tile; WC column tiles and WR row groups form the workgroup.
typedef float v4f __attribute__((ext_vector_type(4)));
constexpr int MF_ST = 8;   // staging loads in flight per lane
constexpr int MF_PT = 7;   // prefetch registers per lane for the operator (P^2 <= 7 x threads: p = 20 on 256)
constexpr int MF_PA = 11;  // and for the source block (P R <= 11 x threads: p = 20, R = 64 on 256)
constexpr int MF_TR = 3;  // row tiles per wave
__host__ __device__ inline int mf_ks(int P) { return (P + 3) / 4; }
// complex slots after the staged T and a that must read as zero
__host__ __device__ inline int mf_zero_tail(int P, int R) {
  const int KS = mf_ks(P), NT = (R + 15) / 16;
  const int zb = (4 * KS - P) * R + 16 * NT;  // B rows n in [P, 4 KS) and column overrun
  const int za = 4 * KS * P - P * P - P * R;  // A columns n in [P, 4 KS)
  return zb > za ? zb : za;
}
inline size_t mf_lds_bytes(int P, int R) { return (size_t)(P * P + P * R + mf_zero_tail(P, R)) * sizeof(float2); }
// KIND only names the instantiation (MF_LIST: M2L lists, MF_TREE: M2M / L2L,
// MF_TOP: the frequency-domain products of the level-0 convolution)
// so that profiles tell the launches apart.
enum { MF_LIST = 0, MF_TREE = 1, MF_TOP = 2 };
template <int WC, int WR, int KIND, bool PRE>
__global__ void __launch_bounds__(64 * WC * WR) __attribute__((amdgpu_waves_per_eu(PRE ? 4 : 1))) k_m2l_mfma(int p, int R, const int* __restrict__ items,
                                                      const int* __restrict__ src, const int* __restrict__ opi,
                                                      const float2* __restrict__ ops, const float2* __restrict__ me,
                                                      float2* __restrict__ part, const int* __restrict__ dtgt,
                                                      int accumulate) {
  constexpr int NTH = 64 * WC * WR;
  const int P = 2 * p + 1, PP = P * P, PR = P * R, NS = PP + PR;
  const int MT = (P + 15) / 16, NT = (R + 15) / 16, KS = mf_ks(P), NZ = mf_zero_tail(P, R);
  extern __shared__ unsigned char dyn[];
  float2* S = reinterpret_cast<float2*>(dyn);  // T [n][m] (stride P), a [n][j] (stride R), zero tail
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int l16 = lane & 15, kq = lane >> 4;
  const int wr = wv / WC, ct = wv % WC;
  for (int idx = threadIdx.x; idx < NZ; idx += NTH) S[NS + idx] = make_float2(0.f, 0.f);
  int aoff[MF_TR];  // complex offsets of this lane's fragments at k-step 0
#pragma unroll
  for (int t = 0; t < MF_TR; ++t) aoff[t] = kq * P + min(16 * (wr * MF_TR + t) + l16, P - 1);
  const int boff = PP + kq * R + min(16 * ct + l16, 16 * NT - 1);
  v4f t1[MF_TR], t2[MF_TR], t3[MF_TR];
#pragma unroll
  for (int t = 0; t < MF_TR; ++t) t1[t] = t2[t] = t3[t] = v4f{0.f, 0.f, 0.f, 0.f};
  const int e0 = items[3 * blockIdx.x + 1], e1 = items[3 * blockIdx.x + 2];
  // PRE (an entry's operator fits MF_PT and its source block MF_PA values per
  // thread): the next entry is loaded into registers while the current one is
  // multiplied.  Every load has a uniform base (operator or source block plus
  // NTH u) and the thread index as offset, so the loop keeps no per-load
  // addresses; lanes past the end re-read the last element.
  const int tid = threadIdx.x;
  float2 pt[PRE ? MF_PT : 1], pa[PRE ? MF_PA : 1];
#define LM_MF_FETCH(e)                                                          \
  do {                                                                          \
    const float2* Tg_ = ops + (int64_t)opi[e] * PP;                             \
    const float2* Ag_ = me + (int64_t)src[e] * PR;                              \
    _Pragma("unroll") for (int u = 0; u < (PRE ? MF_PT : 1); ++u) {             \
      const int o = NTH * u;                                                    \
      if (o < PP) pt[u] = Tg_[o + min(tid, PP - 1 - o)];                        \
    }                                                                           \
    _Pragma("unroll") for (int u = 0; u < (PRE ? MF_PA : 1); ++u) {             \
      const int o = NTH * u;                                                    \
      if (o < PR) pa[u] = Ag_[o + min(tid, PR - 1 - o)];                        \
    }                                                                           \
  } while (0)
  if (PRE && e0 < e1) LM_MF_FETCH(e0);
  for (int e = e0; e < e1; ++e) {
    __syncthreads();
    if (PRE) {
#pragma unroll
      for (int u = 0; u < (PRE ? MF_PT : 1); ++u)
        if (NTH * u + tid < PP) S[NTH * u + tid] = pt[u];
#pragma unroll
      for (int u = 0; u < (PRE ? MF_PA : 1); ++u)
        if (NTH * u + tid < PR) S[PP + NTH * u + tid] = pa[u];
      __syncthreads();
      if (e + 1 < e1) LM_MF_FETCH(e + 1);
    } else {
      const float2* Tg = ops + (int64_t)opi[e] * PP;
      const float2* Ag = me + (int64_t)src[e] * PR;
      for (int base = threadIdx.x; base < NS; base += NTH * MF_ST) {
        float2 v[MF_ST];
#pragma unroll
        for (int u = 0; u < MF_ST; ++u) {
          const int idx = base + NTH * u;
          if (idx < NS) v[u] = idx < PP ? Tg[idx] : Ag[idx - PP];
        }
#pragma unroll
        for (int u = 0; u < MF_ST; ++u) {
          const int idx = base + NTH * u;
          if (idx < NS) S[idx] = v[u];
        }
      }
      __syncthreads();
    }
#pragma unroll 1
    for (int ks = 0; ks < KS; ++ks) {
      const float2 bv = S[boff + 4 * ks * R];
      const float bs = bv.x + bv.y;
#pragma unroll
      for (int t = 0; t < MF_TR; ++t) {
        const float2 av = S[aoff[t] + 4 * ks * P];
        t1[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, bv.x, t1[t], 0, 0, 0);
        t2[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, bv.y, t2[t], 0, 0, 0);
        t3[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x + av.y, bs, t3[t], 0, 0, 0);
      }
    }
  }
#undef LM_MF_FETCH
  // partial slot of this item, or (translations with one item per box) the
  // output expansion itself, overwritten or accumulated; lane rows 4 kq + v
  // of a tile are coefficients m = 16 rt + 4 kq + v
  float2* out = part + (int64_t)(dtgt ? dtgt[blockIdx.x] : (int)blockIdx.x) * PR;
  const int j = 16 * ct + l16;
#pragma unroll
  for (int t = 0; t < MF_TR; ++t) {
    const int rt = wr * MF_TR + t;
    if (rt < MT && j < R) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = 16 * rt + 4 * kq + v;
        if (m < P) {
          float2* o = out + (int64_t)m * R + j;
          const float a = t1[t][v], b = t2[t][v];
          const float2 r = make_float2(a - b, t3[t][v] - a - b);
          *o = accumulate ? make_float2(o->x + r.x, o->y + r.y) : r;
        }
      }
    }
  }
}

// M2L with few right-hand sides (FP32, 2 <= R <= 8), operator-major: the
// list kernel would stage a P x P operator for every entry's P x R block.
// Here a work item (operator, <= M2L_ITEM of its entries) stages the operator
// once and multiplies it by the source blocks of G = 64 / R entries at a
// time, laid side by side as the CB = G R columns of B ([n][c], c = g R + j),
// with the same tiles and three-product form as k_m2l_mfma (WR row groups of
// 3 tiles, 4 column tiles).  Entry g's P x R result goes to its slot (its
// list position), summed per target by k_p2m_reduce.
constexpr int OM_RMAX = 8;  // right-hand sides up to which the M2L runs operator-major
template <int WR>
__global__ void __launch_bounds__(256 * WR) k_m2l_om(int p, int R, const int* __restrict__ items,
                                                     const int* __restrict__ slot, const int* __restrict__ src,
                                                     const float2* __restrict__ ops, const float2* __restrict__ me,
                                                     float2* __restrict__ out) {
  constexpr int NTH = 256 * WR;
  const int P = 2 * p + 1, PP = P * P, PR = P * R, G = 64 / R, CB = G * R;
  const int MT = (P + 15) / 16, NT = (CB + 15) / 16, KS = mf_ks(P), NZ = mf_zero_tail(P, CB);
  extern __shared__ unsigned char dyn[];
  float2* S = reinterpret_cast<float2*>(dyn);  // T [n][m] (stride P), B [n][c] (stride CB), zero tail
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int l16 = lane & 15, kq = lane >> 4;
  const int wr = wv >> 2, ct = wv & 3;
  const int t = items[3 * blockIdx.x], e0 = items[3 * blockIdx.x + 1], e1 = items[3 * blockIdx.x + 2];
  const float2* Tg = ops + (int64_t)t * PP;
  for (int idx = threadIdx.x; idx < PP; idx += NTH) S[idx] = Tg[idx];
  for (int idx = threadIdx.x; idx < NZ; idx += NTH) S[PP + P * CB + idx] = make_float2(0.f, 0.f);
  int aoff[MF_TR];
#pragma unroll
  for (int u = 0; u < MF_TR; ++u) aoff[u] = kq * P + min(16 * (wr * MF_TR + u) + l16, P - 1);
  const int col = 16 * ct + l16;
  const int boff = PP + kq * CB + min(col, 16 * NT - 1);
  for (int eg = e0; eg < e1; eg += G) {
    const int ng = min(G, e1 - eg);
    __syncthreads();
    for (int idx = threadIdx.x; idx < P * CB; idx += NTH) {
      const int n = idx / CB, c = idx - n * CB, g = c / R, j = c - g * R;
      S[PP + idx] = g < ng ? me[(int64_t)src[eg + g] * PR + n * R + j] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    v4f t1[MF_TR], t2[MF_TR], t3[MF_TR];
#pragma unroll
    for (int u = 0; u < MF_TR; ++u) t1[u] = t2[u] = t3[u] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
    for (int ks = 0; ks < KS; ++ks) {
      const float2 bv = S[boff + 4 * ks * CB];
      const float bs = bv.x + bv.y;
#pragma unroll
      for (int u = 0; u < MF_TR; ++u) {
        const float2 av = S[aoff[u] + 4 * ks * P];
        t1[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, bv.x, t1[u], 0, 0, 0);
        t2[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, bv.y, t2[u], 0, 0, 0);
        t3[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x + av.y, bs, t3[u], 0, 0, 0);
      }
    }
    const int g = col / R, j = col - g * R;
    if (col < CB && g < ng) {
      float2* o = out + (int64_t)slot[eg + g] * PR + j;
#pragma unroll
      for (int u = 0; u < MF_TR; ++u) {
        const int rt = wr * MF_TR + u;
        if (rt < MT) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int m = 16 * rt + 4 * kq + v;
            if (m < P) {
              const float a = t1[u][v], b = t2[u][v];
              o[(int64_t)m * R] = make_float2(a - b, t3[u][v] - a - b);
            }
          }
        }
      }
    }
  }
}

// Launch of k_m2l_mfma for R in [1, 64] and P <= 96 (p <= 47): one wavefront
// per column tile of 16 right-hand sides, one or two row groups of 48.
template <int KIND>
inline void m2l_mfma_launch(int n_items, int p, int R, const int* items, const int* src, const int* opi,
                            const float2* ops, const float2* in, float2* out, const int* dtgt, int accumulate,
                            hipStream_t s) {
  const int P = 2 * p + 1, MT = (P + 15) / 16, NT = (R + 15) / 16;
  const size_t lds = mf_lds_bytes(P, R);
  const bool two = MT > MF_TR;
  const int PP = P * P, PR = P * R;
#define LM_MF(WC, WR)                                                                                               \
  do {                                                                                                              \
    if (PP <= MF_PT * 64 * (WC) * (WR) && PR <= MF_PA * 64 * (WC) * (WR))                                           \
      hipLaunchKernelGGL((k_m2l_mfma<WC, WR, KIND, true>), dim3(n_items), dim3(64 * (WC) * (WR)), lds, s, p, R,    \
                         items, src, opi, ops, in, out, dtgt, accumulate);                                          \
    else                                                                                                            \
      hipLaunchKernelGGL((k_m2l_mfma<WC, WR, KIND, false>), dim3(n_items), dim3(64 * (WC) * (WR)), lds, s, p, R,   \
                         items, src, opi, ops, in, out, dtgt, accumulate);                                          \
  } while (0)
  if (NT > 2) {
    if (two) LM_MF(4, 2); else LM_MF(4, 1);
  } else if (NT == 2) {
    if (two) LM_MF(2, 2); else LM_MF(2, 1);
  } else {
    if (two) LM_MF(1, 2); else LM_MF(1, 1);
  }
#undef LM_MF
}

// LDS limit of the k_m2l_mfma and k_m2l_om instantiations (dynamic LDS
// above 64 KiB must be allowed per kernel).
inline hipError_t m2l_mfma_allow_lds(size_t bytes) {
#define LM_MF4(KIND, PRE)                                                                        \
  (const void*)k_m2l_mfma<4, 1, KIND, PRE>, (const void*)k_m2l_mfma<4, 2, KIND, PRE>,            \
      (const void*)k_m2l_mfma<2, 1, KIND, PRE>, (const void*)k_m2l_mfma<2, 2, KIND, PRE>,        \
      (const void*)k_m2l_mfma<1, 1, KIND, PRE>, (const void*)k_m2l_mfma<1, 2, KIND, PRE>
  const void* fs[38] = {LM_MF4(MF_LIST, true), LM_MF4(MF_LIST, false), LM_MF4(MF_TREE, true),
                        LM_MF4(MF_TREE, false), LM_MF4(MF_TOP, true),   LM_MF4(MF_TOP, false),
                        (const void*)k_m2l_om<1>,  (const void*)k_m2l_om<2>};
#undef LM_MF4
  for (const void* f : fs) {
    const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// M2L, operator-major (one right-hand side): one wavefront per operator
// streams its columns from HBM once per batch of M2L_EB entries (lane m holds
// output row m); the source coefficients are wave-uniform, so they come
// through scalar loads and every lane does M2L_EB complex FMAs per column
// load.  Results go to per-entry slots, summed per target by k_m2l_reduce.
// Operators with many entries are split into work items of at most
// M2L_ITEM entries (item = operator, first entry, end), so no wavefront runs
// much longer than the others.
constexpr int M2L_EB = 8;
constexpr int M2L_ITEM = 32;
constexpr int M2L_MF_ITEM = 32;  // entries per item of the matrix-core M2L lists
template <typename RT>
__global__ void __launch_bounds__(64) k_m2l_apply(int p, const int* __restrict__ items, const int* __restrict__ slot,
                                                  const int* __restrict__ src,
                                                  const typename C2T<RT>::T* __restrict__ ops,
                                                  const typename C2T<RT>::T* __restrict__ me,
                                                  typename C2T<RT>::T* __restrict__ out) {
  typedef typename C2T<RT>::T V;
  const int t = items[3 * blockIdx.x];
  const int P = 2 * p + 1;
  const int m = threadIdx.x;
  const bool act = m < P;
  const V* T = ops + (int64_t)t * P * P + (act ? m : 0);
  const int e0 = items[3 * blockIdx.x + 1], e1 = items[3 * blockIdx.x + 2];
  for (int e = e0; e < e1; e += M2L_EB) {
    const int ne = min(M2L_EB, e1 - e);
    const V* a[M2L_EB];
#pragma unroll
    for (int q = 0; q < M2L_EB; ++q) a[q] = me + (int64_t)src[e + min(q, ne - 1)] * P;
    RT re[M2L_EB], im[M2L_EB];
#pragma unroll
    for (int q = 0; q < M2L_EB; ++q) re[q] = im[q] = RT(0);
    constexpr int U = sizeof(RT) == 8 ? 2 : 4;  // columns in flight per lane
    int n = 0;
    for (; n + U <= P; n += U) {
      V tv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) tv[u] = T[(int64_t)(n + u) * P];
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int q = 0; q < M2L_EB; ++q) cmac(re[q], im[q], tv[u], a[q][n + u]);
    }
    for (; n < P; ++n) {
      const V tv = T[(int64_t)n * P];
#pragma unroll
      for (int q = 0; q < M2L_EB; ++q) cmac(re[q], im[q], tv, a[q][n]);
    }
    if (act) {
#pragma unroll
      for (int q = 0; q < M2L_EB; ++q)
        if (q < ne) out[(int64_t)slot[e + q] * P + m] = mk<V>(re[q], im[q]);
    }
  }
}

// le[target] = sum of its entry slots: four wavefronts per target take every
// fourth entry (two independent chains each), then combine through LDS.
template <typename RT>
__global__ void __launch_bounds__(256) k_m2l_reduce(int p, const int* __restrict__ tgts, const int* __restrict__ ptr,
                                                    const typename C2T<RT>::T* __restrict__ out,
                                                    typename C2T<RT>::T* __restrict__ le) {
  typedef typename C2T<RT>::T V;
  const int P = 2 * p + 1;
  const int m = threadIdx.x & 63, part = threadIdx.x >> 6;
  __shared__ RT red[2][4][64];
  RT r0 = 0, i0 = 0, r1 = 0, i1 = 0;
  if (m < P) {
    const int e1 = ptr[blockIdx.x + 1];
    int e = ptr[blockIdx.x] + part;
    for (; e + 4 < e1; e += 8) {
      const V a = out[(int64_t)e * P + m], b = out[(int64_t)(e + 4) * P + m];
      r0 += a.x;
      i0 += a.y;
      r1 += b.x;
      i1 += b.y;
    }
    if (e < e1) {
      const V a = out[(int64_t)e * P + m];
      r0 += a.x;
      i0 += a.y;
    }
  }
  red[0][part][m] = r0 + r1;
  red[1][part][m] = i0 + i1;
  __syncthreads();
  if (part == 0 && m < P)
    le[(int64_t)tgts[blockIdx.x] * P + m] =
        mk<V>((red[0][0][m] + red[0][1][m]) + (red[0][2][m] + red[0][3][m]),
              (red[1][0][m] + red[1][1][m]) + (red[1][2][m] + red[1][3][m]));
}

// L2L: child bt += Op parent bt, for every box of one level.
template <typename RT>
__global__ void __launch_bounds__(256) k_l2l(int p, int R, int nlev, int first, const BoxDev* __restrict__ boxes,
                                             const int* __restrict__ tree_layer,
                                             const typename C2T<RT>::T* __restrict__ ops,
                                             typename C2T<RT>::T* __restrict__ le) {
  typedef typename C2T<RT>::T V;
  const int b = first + blockIdx.x;
  const BoxDev B = boxes[b];
  const int P = 2 * p + 1, PR = P * R;
  extern __shared__ unsigned char dyn[];
  V* a = reinterpret_cast<V*>(dyn);
  for (int idx = threadIdx.x; idx < PR; idx += blockDim.x) a[idx] = le[(int64_t)B.parent * PR + idx];
  __syncthreads();
  RT are[MO], aim[MO];
  acc_zero(are, aim);
  const V* Op = ops + ((int64_t)((tree_layer[B.tree] * nlev + B.level) * 4 + B.pos)) * P * P;
  op_apply<RT>(P, R, Op, a, are, aim);
  V* out = le + (int64_t)b * PR;
#pragma unroll
  for (int i = 0; i < MO; ++i) {
    const int idx = threadIdx.x + i * blockDim.x;
    if (idx < PR) {
      const V o = out[idx];
      out[idx] = mk<V>(o.x + are[i], o.y + aim[i]);
    }
  }
}

// L2P: y_e (=/+=) sum_m (bt_m / sig_m) J_m(k rho) e^{i m theta} for the points of each leaf.
template <typename RT, int PCH>
__global__ void __launch_bounds__(256) k_l2p(int p, int R, int nlev, int accumulate, const int* __restrict__ items,
                                             const BoxDev* __restrict__ boxes, const int* __restrict__ tree_layer,
                                             const double* __restrict__ sig, const int* __restrict__ pt_elem,
                                             const double2* __restrict__ pt_xh,
                                             const typename C2T<RT>::T* __restrict__ le, int N,
                                             typename C2T<RT>::T* __restrict__ y) {
  typedef typename C2T<RT>::T V;
  const int b = items[3 * blockIdx.x];
  BoxDev B = boxes[b];
  B.pt0 = items[3 * blockIdx.x + 1];
  B.npt = items[3 * blockIdx.x + 2];
  const int P = 2 * p + 1, PR = P * R;
  const double* sg = sig + (int64_t)(tree_layer[B.tree] * nlev + B.level) * (p + 1);
  __shared__ RT js[PCH][MAXP + 1];
  __shared__ V cs[PCH][MAXP + 1];
  extern __shared__ unsigned char dyn[];
  V* L = reinterpret_cast<V*>(dyn);  // [P][R]
  for (int idx = threadIdx.x; idx < PR; idx += blockDim.x) L[idx] = le[(int64_t)b * PR + idx];
  for (int s0 = 0; s0 < B.npt; s0 += PCH) {
    const int cnt = min(PCH, B.npt - s0);
    __syncthreads();
    if (threadIdx.x < (unsigned)cnt) {
      const double2 xh = pt_xh[B.pt0 + s0 + threadIdx.x];
      point_basis<RT>(B.k, xh.x - B.cx, xh.y - B.ch, p, sg, 1.0, js[threadIdx.x], cs[threadIdx.x]);
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < cnt * R; idx += blockDim.x) {
      const int j = idx / R, r = idx - j * R;
      const V l0 = L[p * R + r];
      RT re = js[j][0] * l0.x, im = js[j][0] * l0.y;
      for (int m = 1; m <= p; ++m) {
        const V c = cs[j][m];
        const RT jv = js[j][m];
        const RT jn = (m & 1) ? -jv : jv;  // J_{-m} = (-1)^m J_m
        const V lp = L[(p + m) * R + r], ln = L[(p - m) * R + r];
        // lp e^{i m th} J_m + ln e^{-i m th} J_{-m}
        re += jv * (c.x * lp.x - c.y * lp.y) + jn * (c.x * ln.x + c.y * ln.y);
        im += jv * (c.x * lp.y + c.y * lp.x) + jn * (c.x * ln.y - c.y * ln.x);
      }
      const int e = pt_elem[B.pt0 + s0 + j];
      V* yp = y + (int64_t)r * N + e;
      if (accumulate) {
        const V o = *yp;
        *yp = mk<V>(o.x + re, o.y + im);
      } else {
        *yp = mk<V>(re, im);
      }
    }
  }
}

// Point matrices of the P2M and L2P (complex64, evaluated in FP64) for the
// matrix-core form, per work item (leaf, first point pos, count c) at offset
// pos P: P2M [n][j] (P x c) = |Gamma_j| J_n(k rho_j) e^{-i n theta_j} / sig_|n|,
// L2P [j][m] (c x P) = J_m(k rho_j) e^{i m theta_j} / sig_|m|, n, m = -p..p,
// J_{-n} = (-1)^n J_n.  One thread per point.
// Sound-hard / impedance targets (bt.bc != Dirichlet) see n . grad + i beta of
// the local expansion: with F_m = J_m(k rho) e^{i m theta} in the tree's
// (x, h) plane, d/dx F_m = k/2 (F_{m-1} - F_{m+1}), d/dh F_m = i k/2
// (F_{m-1} + F_{m+1}), and h = +-y + const by the tree's side, the L2P row is
// [k/2 ((a + i b) F_{m-1} - (a - i b) F_{m+1}) + i beta F_m] / sig_|m| with
// (a, b) = (n_x, +-n_y); also kept in FP64 (zl64) for the FP64 matvec.
__global__ void __launch_bounds__(64) k_leaf_basis(int p, int nlev, const int* __restrict__ items,
                                                   const BoxDev* __restrict__ boxes,
                                                   const int* __restrict__ tree_layer, const double* __restrict__ sig,
                                                   const int* __restrict__ pt_elem, const double2* __restrict__ pt_xh,
                                                   const double* __restrict__ w, BcTarget bt,
                                                   const int* __restrict__ tree_side, float2* __restrict__ zp,
                                                   float2* __restrict__ zl, double2* __restrict__ zl64) {
  const int b = items[3 * blockIdx.x], pos = items[3 * blockIdx.x + 1], cnt = items[3 * blockIdx.x + 2];
  const int j = threadIdx.x;
  if (j >= cnt) return;
  const BoxDev B = boxes[b];
  const int P = 2 * p + 1;
  const double* sg = sig + (int64_t)(tree_layer[B.tree] * nlev + B.level) * (p + 1);
  const double2 xh = pt_xh[pos + j];
  const double dx = xh.x - B.cx, dh = xh.y - B.ch;
  double J[MAXP + 2];
  fm::bessel_j_seq(B.k * hypot(dx, dh), p + 1, J);
  const zd e1 = fm::cis(atan2(dh, dx));
  const double we = w[pt_elem[pos + j]];
  float2* P2 = zp + (int64_t)pos * P;
  float2* L2 = zl + (int64_t)pos * P + (int64_t)j * P;
  zd ep(1.0, 0.0);  // e^{i m theta}
  for (int m = 0; m <= p; ++m) {
    const double a = J[m] / sg[m], an = (m & 1) ? -a : a;  // J_m / sig_m, J_{-m} / sig_m
    L2[p + m] = make_float2((float)(a * ep.re), (float)(a * ep.im));
    L2[p - m] = make_float2((float)(an * ep.re), (float)(-an * ep.im));
    P2[(int64_t)(p + m) * cnt + j] = make_float2((float)(we * a * ep.re), (float)(-we * a * ep.im));
    P2[(int64_t)(p - m) * cnt + j] = make_float2((float)(we * an * ep.re), (float)(we * an * ep.im));
    ep = ep * e1;
  }
  if (bt.bc == LM_BC_DIRICHLET) return;
  // F_n, n = -(p+1)..p+1, at F[n + p + 1]
  zd F[2 * MAXP + 3];
  zd en(1.0, 0.0);
  for (int n = 0; n <= p + 1; ++n) {
    const double jn = (n & 1) ? -J[n] : J[n];
    F[p + 1 + n] = en * J[n];
    F[p + 1 - n] = zd(en.re, -en.im) * jn;
    en = en * e1;
  }
  const int e = pt_elem[pos + j];
  const double na = bt.nx[e], nb = (tree_side[B.tree] == SIDE_B ? 1.0 : -1.0) * bt.ny[e];
  const zd apb(na, nb), amb(na, -nb);
  double2* L64 = zl64 + (int64_t)pos * P + (int64_t)j * P;
  for (int m = -p; m <= p; ++m) {
    const zd v = (apb * F[p + m] - amb * F[p + m + 2]) * (0.5 * B.k) + zd(0.0, bt.beta) * F[p + 1 + m];
    const double sc = 1.0 / sg[m < 0 ? -m : m];
    L2[p + m] = make_float2((float)(v.re * sc), (float)(v.im * sc));
    L64[p + m] = make_double2(v.re * sc, v.im * sc);
  }
}

// L2P from stored point rows (sound-hard / impedance targets, FP64 or one
// right-hand side): y[r][e_j] += sum_m Z[j][m] le[leaf][m][r], one thread per
// (point, right-hand side) of a work item.
template <typename RT>
__global__ void __launch_bounds__(256) k_l2p_rows(int p, int R, int N, const int* __restrict__ items,
                                                  const int* __restrict__ pt_elem,
                                                  const typename C2T<RT>::T* __restrict__ Z,
                                                  const typename C2T<RT>::T* __restrict__ le,
                                                  typename C2T<RT>::T* __restrict__ y) {
  typedef typename C2T<RT>::T V;
  const int b = items[3 * blockIdx.x], pos = items[3 * blockIdx.x + 1], cnt = items[3 * blockIdx.x + 2];
  const int P = 2 * p + 1;
  const V* L = le + (int64_t)b * P * R;
  for (int idx = threadIdx.x; idx < cnt * R; idx += blockDim.x) {
    const int j = idx / R, r = idx - j * R;
    const V* z = Z + (int64_t)(pos + j) * P;
    RT re = 0, im = 0;
    for (int m = 0; m < P; ++m) cmac(re, im, z[m], L[(int64_t)m * R + r]);
    V* yp = y + (int64_t)r * N + pt_elem[pos + j];
    const V o = *yp;
    *yp = mk<V>(o.x + re, o.y + im);
  }
}

// P2M item on matrix cores: part[item] (P x R) = P2M matrix (P x c) times
// the gathered input rows xt[e_j] (c x R).
struct P2MOp {
  int rows, q, R;
  const float2* Z;
  const int* elem;
  const float2* xt;
  float2* out;
  __device__ const float2* zrow(int r) const { return Z + (int64_t)r * q; }
  __device__ const float2* brow(int c) const { return xt + (int64_t)elem[c] * R; }
  __device__ void store(int r, int j, float re, float im) const { out[(int64_t)r * R + j] = make_float2(re, im); }
};
// The only item of a leaf writes the leaf's expansion itself (dst >= 0);
// the items of larger leaves write partials, summed by k_p2m_reduce.
__global__ void __launch_bounds__(64 * PA_NW) k_p2m_mfma(int p, int R, const int* __restrict__ items,
                                                       const int* __restrict__ dst, const int* __restrict__ pt_elem,
                                                       const float2* __restrict__ zp, const float2* __restrict__ xt,
                                                       float2* __restrict__ part, float2* __restrict__ me) {
  const int pos = items[3 * blockIdx.x + 1], cnt = items[3 * blockIdx.x + 2], d = dst[blockIdx.x];
  const int P = 2 * p + 1;
  float2* out = d >= 0 ? me + (int64_t)d * P * R : part + (int64_t)blockIdx.x * P * R;
  P2MOp op{P, cnt, R, zp + (int64_t)pos * P, pt_elem + pos, xt, out};
  block_mfma_body(op, R);
}

// L2P item on matrix cores: y[j][e_r] (=|+=) L2P matrix (c x P) times the
// leaf's local expansion le[leaf] (P x R).
struct L2POp {
  int rows, q, N, R, acc;
  const float2* Z;
  const float2* L;
  const int* elem;
  float2* y;
  __device__ const float2* zrow(int r) const { return Z + (int64_t)r * q; }
  __device__ const float2* brow(int c) const { return L + (int64_t)c * R; }
  __device__ void store(int r, int j, float re, float im) const {
    float2* o = y + (int64_t)j * N + elem[r];
    if (acc) {
      const float2 v = *o;
      *o = make_float2(v.x + re, v.y + im);
    } else {
      *o = make_float2(re, im);
    }
  }
};
__global__ void __launch_bounds__(64 * PA_NW) k_l2p_mfma(int p, int R, int N, int accumulate,
                                                       const int* __restrict__ items, const int* __restrict__ pt_elem,
                                                       const float2* __restrict__ zl, const float2* __restrict__ le,
                                                       float2* __restrict__ y) {
  const int b = items[3 * blockIdx.x], pos = items[3 * blockIdx.x + 1], cnt = items[3 * blockIdx.x + 2];
  const int P = 2 * p + 1;
  L2POp op{cnt, P, N, R, accumulate, zl + (int64_t)pos * P, le + (int64_t)b * P * R, pt_elem + pos, y};
  block_mfma_body(op, R);
}

// y_i (+)= sum_j Knear_ij x_j for every right-hand side (acc: add, else
// overwrite): one wavefront per row; right-hand sides in groups of G share
// each matrix value and index load.
template <typename RT, int G>
__global__ void __launch_bounds__(256) k_near_csr(int N, int nrow, const int* __restrict__ rows, int R, int acc,
                                                  const int* __restrict__ ptr, const int* __restrict__ src,
                                                  const typename C2T<RT>::T* __restrict__ val,
                                                  const typename C2T<RT>::T* __restrict__ x,
                                                  typename C2T<RT>::T* __restrict__ y) {
  typedef typename C2T<RT>::T V;
  const int ir = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (ir >= nrow) return;
  const int row = rows ? rows[ir] : ir;
  const int e0 = ptr[row], e1 = ptr[row + 1];
  for (int g = 0; g < R; g += G) {
    RT re[G], im[G];
#pragma unroll
    for (int u = 0; u < G; ++u) re[u] = im[u] = RT(0);
    for (int e = e0 + lane; e < e1; e += 64) {
      const V a = val[e];
      const int c = src[e];
#pragma unroll
      for (int u = 0; u < G; ++u)
        if (g + u < R) cmac(re[u], im[u], a, x[(int64_t)(g + u) * N + c]);
    }
#pragma unroll
    for (int u = 0; u < G; ++u)
      if (g + u < R)
        for (int off = 32; off > 0; off >>= 1) {
          re[u] += __shfl_xor(re[u], off, 64);
          im[u] += __shfl_xor(im[u], off, 64);
        }
    if (lane == 0) {
#pragma unroll
      for (int u = 0; u < G; ++u) {
        if (g + u < R) {
          V* yp = y + (int64_t)(g + u) * N + row;
          if (acc) {
            const V o = *yp;
            *yp = mk<V>(o.x + re[u], o.y + im[u]);
          } else {
            *yp = mk<V>(re[u], im[u]);
          }
        }
      }
    }
  }
}

// ================================================================ host side ==

namespace {

struct TreeB {
  int layer, side;
  bool reac;
  double k;
  std::vector<int> el;
  std::vector<double> x, h;
  std::vector<int> leaf_lev;
  std::vector<std::vector<int64_t>> keys;            // per level, sorted
  std::vector<std::unordered_map<int64_t, int>> idx;  // per level: key -> global box id
};

static constexpr double kEulerGamma = 0.57721566490153286061;

template <typename T>
lm_status up(DevBuf& b, const std::vector<T>& v, hipStream_t s) {
  return upload(b, v.data(), v.size() * sizeof(T), s);
}

}  // namespace

lm_status fmm_build(lm_geom_s* g, hipStream_t s) {
  FmmPlan* F = new (std::nothrow) FmmPlan();
  LM_CHECK(F, LM_ENOMEM, "host allocation failed");
  g->fmm = F;
  LM_TRY_HIP(hipStreamCreateWithFlags(&F->s_near, hipStreamNonBlocking));
  LM_TRY_HIP(hipEventCreateWithFlags(&F->ev_fork, hipEventDisableTiming));
  LM_TRY_HIP(hipEventCreateWithFlags(&F->ev_join, hipEventDisableTiming));
  const MediumDev& m = g->m;
  const int L = m.L;
  const int64_t N = g->N;
  const int p = g->p;
  LM_CHECK(p >= 4 && p <= MAXP, LM_EINVAL, "the FMM needs 4 <= p <= %d", MAXP);
  F->p = p;
  F->bc = g->bc;
  F->beta = g->robin_beta;
  F->n_el = N;
  F->P = 2 * p + 1;
  F->n_layers = L + 1;

  // ---- grid -----------------------------------------------------------------
  double xmin = 1e300, xmax = -1e300;
  for (int64_t e = 0; e < N; ++e) {
    xmin = std::min(xmin, g->cx[e]);
    xmax = std::max(xmax, g->cx[e]);
  }
  std::vector<double> wsort(g->w);
  std::nth_element(wsort.begin(), wsort.begin() + N / 2, wsort.end());
  const double hmed = wsort[N / 2];
  F->w_top = LM_TOP_KW / m.kmax;
  F->x0 = xmin - 1e-7 * (1.0 + std::fabs(xmin)) - 0.5 * hmed;

  // trees: free tree per layer (side B, or T for the bottom layer), side trees
  std::vector<TreeB> T;
  std::vector<int> tree_layer;
  for (int l = 0; l <= L; ++l) {
    TreeB t;
    t.layer = l;
    t.side = l < L ? SIDE_B : SIDE_T;
    t.reac = false;
    t.k = m.k[l];
    T.push_back(t);
  }
  for (int l = 0; l <= L; ++l)
    for (int sd = 0; sd < 2; ++sd)
      if (side_exists(m, l, sd)) {
        TreeB t;
        t.layer = l;
        t.side = sd;
        t.reac = true;
        t.k = m.k[l];
        T.push_back(t);
      }
  for (int64_t e = 0; e < N; ++e) {
    const int l = g->layer[e];
    for (auto& t : T) {
      if (t.layer != l) continue;
      t.el.push_back((int)e);
      t.x.push_back(g->cx[e]);
      t.h.push_back(std::max(0.0, side_h(m, l, t.side, g->cy[e])));
    }
  }
  // free leaf level: mean points per non-empty leaf <= leaf_size
  int lf = 0;
  for (; lf < 12; ++lf) {
    const double w = F->w_top / (1 << lf);
    int64_t nbox = 0, npt = 0;
    for (auto& t : T) {
      if (t.reac) continue;
      std::unordered_map<int64_t, int> cnt;
      for (size_t i = 0; i < t.el.size(); ++i)
        cnt[bkey((int)std::floor((t.x[i] - F->x0) / w), (int)std::floor(t.h[i] / w))]++;
      nbox += cnt.size();
      npt += t.el.size();
    }
    if (nbox == 0 || (double)npt / nbox <= g->leaf_size) break;
  }
  int lr = (int)std::ceil(std::log2(F->w_top / hmed));
  lr = std::max(lr, lf);
  lr = std::min(lr, 16);
  F->lf = lf;
  F->lr = lr;
  F->nlev = lr + 1;
  const int nlev = F->nlev;
  auto wl = [&](int l) { return F->w_top / (double)(1 << l); };

  // ---- boxes ----------------------------------------------------------------
  for (auto& t : T) {
    t.keys.assign(nlev, {});
    t.idx.assign(nlev, {});
    t.leaf_lev.resize(t.el.size());
    for (size_t i = 0; i < t.el.size(); ++i) {
      int ll;
      if (!t.reac) {
        ll = lf;
      } else {
        ll = 0;
        while (ll < lr && t.h[i] < wl(ll)) ++ll;
      }
      t.leaf_lev[i] = ll;
      for (int l = 0; l <= ll; ++l) {
        const int64_t kk = bkey((int)std::floor((t.x[i] - F->x0) / wl(l)), (int)std::floor(t.h[i] / wl(l)));
        t.idx[l].emplace(kk, -1);
      }
    }
    for (int l = 0; l < nlev; ++l) {
      for (auto& kv : t.idx[l]) t.keys[l].push_back(kv.first);
      std::sort(t.keys[l].begin(), t.keys[l].end());
    }
  }
  F->level_ptr.assign(nlev + 1, 0);
  for (int l = 0; l < nlev; ++l) {
    F->level_ptr[l] = (int)F->boxes.size();
    for (size_t ti = 0; ti < T.size(); ++ti) {
      auto& t = T[ti];
      for (int64_t kk : t.keys[l]) {
        const int i = (int)(kk >> 32), j = (int)(uint32_t)kk;
        BoxDev b;
        b.cx = F->x0 + (i + 0.5) * wl(l);
        b.ch = (j + 0.5) * wl(l);
        b.k = t.k;
        b.tree = (int)ti;
        b.level = l;
        b.parent = l > 0 ? t.idx[l - 1].at(bkey(i >> 1, j >> 1)) : -1;
        b.pos = (i & 1) + 2 * (j & 1);
        b.pt0 = b.npt = b.child0 = b.nchild = 0;
        t.idx[l][kk] = (int)F->boxes.size();
        F->boxes.push_back(b);
      }
    }
  }
  F->level_ptr[nlev] = (int)F->boxes.size();
  F->n_boxes = (int)F->boxes.size();
  for (auto& t : T) tree_layer.push_back(t.layer);
  // children (CSR)
  {
    std::vector<std::vector<int>> ch(F->n_boxes);
    for (int b = 0; b < F->n_boxes; ++b)
      if (F->boxes[b].parent >= 0) ch[F->boxes[b].parent].push_back(b);
    for (int b = 0; b < F->n_boxes; ++b) {
      F->boxes[b].child0 = (int)F->children.size();
      F->boxes[b].nchild = (int)ch[b].size();
      for (int c : ch[b]) F->children.push_back(c);
    }
    F->parents_ptr.assign(nlev + 1, 0);
    for (int l = 0; l < nlev; ++l) {
      F->parents_ptr[l] = (int)F->parents_by_level.size();
      for (int b = F->level_ptr[l]; b < F->level_ptr[l + 1]; ++b)
        if (F->boxes[b].nchild) F->parents_by_level.push_back(b);
    }
    F->parents_ptr[nlev] = (int)F->parents_by_level.size();
  }
  // points grouped by leaf box
  for (size_t ti = 0; ti < T.size(); ++ti) {
    auto& t = T[ti];
    std::vector<std::pair<int, int>> order;  // (leaf box, local point)
    for (size_t i = 0; i < t.el.size(); ++i) {
      const int l = t.leaf_lev[i];
      const int64_t kk = bkey((int)std::floor((t.x[i] - F->x0) / wl(l)), (int)std::floor(t.h[i] / wl(l)));
      order.push_back({t.idx[l].at(kk), (int)i});
    }
    std::sort(order.begin(), order.end());
    for (size_t q = 0; q < order.size(); ++q) {
      const int b = order[q].first, i = order[q].second;
      if (F->boxes[b].npt == 0) F->boxes[b].pt0 = (int)F->pt_elem.size();
      F->boxes[b].npt++;
      F->pt_elem.push_back(t.el[i]);
      F->pt_xh.push_back(t.x[i]);
      F->pt_xh.push_back(t.h[i]);
    }
  }
  for (int b = 0; b < F->n_boxes; ++b) {
    const BoxDev& B = F->boxes[b];
    if (!B.npt) continue;
    const TreeB& t = T[B.tree];
    if (!t.reac) F->leaf_free.push_back(b);
    else if (t.side == SIDE_B) F->leaf_B.push_back(b);
    else F->leaf_T.push_back(b);
  }
  // point work items (leaf, first point, count) per tree class, and the
  // item ranges of every leaf for the P2M reduction
  {
    const std::vector<int>* cls[3] = {&F->leaf_free, &F->leaf_B, &F->leaf_T};
    F->p2m_ptr.push_back(0);
    for (int c = 0; c < 3; ++c) {
      F->item_ptr[c] = (int)F->pt_item.size() / 3;
      for (int b : *cls[c]) {
        const BoxDev& B = F->boxes[b];
        for (int q = 0; q < B.npt; q += LM_PTS_ITEM) {
          F->pt_item.push_back(b);
          F->pt_item.push_back(B.pt0 + q);
          F->pt_item.push_back(std::min(LM_PTS_ITEM, B.npt - q));
        }
        F->p2m_leaf.push_back(b);
        F->p2m_ptr.push_back((int)F->pt_item.size() / 3);
        const int i0 = F->p2m_ptr[F->p2m_ptr.size() - 2], i1 = F->p2m_ptr.back();
        for (int i = i0; i < i1; ++i) F->p2m_dst.push_back(i1 - i0 == 1 ? b : -1);
        if (i1 - i0 > 1) F->p2m_msel.push_back((int)F->p2m_leaf.size() - 1);
      }
    }
    F->item_ptr[3] = (int)F->pt_item.size() / 3;
  }

  // ---- expansion scales and M2M / L2L operators -----------------------------------
  // sig[layer][level][n] = s^n / n!, s = k w_level / 2.  Child c, parent C,
  // d = c - C:  M2M  Op[m][n] = (-1)^{m-n} F_{m-n}(d) sig^c_m / sig^C_n,
  //             L2L  Op[m][n] = sig^c_n F_{m-n}(d) / sig^C_m.
  const int NL = L + 1;
  F->sig.assign((size_t)NL * nlev * (p + 1), 0.0);
  for (int l = 0; l <= L; ++l)
    for (int lev = 0; lev < nlev; ++lev) {
      const double sc = 0.5 * m.k[l] * wl(lev);
      double v = 1.0;
      for (int n = 0; n <= p; ++n) {
        F->sig[(size_t)(l * nlev + lev) * (p + 1) + n] = v;
        v *= sc / (n + 1);
      }
    }
  auto sgv = [&](int l, int lev, int n) { return F->sig[(size_t)(l * nlev + lev) * (p + 1) + std::abs(n)]; };
  const int P = F->P;
  const size_t PP = (size_t)P * P;
  F->n_tree_ops = NL * nlev * 4;
  std::vector<double2> ops((size_t)2 * F->n_tree_ops * PP, make_double2(0.0, 0.0));
  {
    const int J = 2 * p;
    std::vector<zd> fj(2 * J + 1);
    std::vector<double> jb(J + 1);
    for (int l = 0; l <= L; ++l)
      for (int lev = 1; lev < nlev; ++lev)
        for (int pos = 0; pos < 4; ++pos) {
          const double q = 0.25 * wl(lev - 1);  // child centre - parent centre = (+-q, +-q)
          fm::f_seq(m.k[l], (pos & 1) ? q : -q, (pos & 2) ? q : -q, J, fj.data(), jb.data());
          const size_t o = (size_t)((l * nlev + lev) * 4 + pos);
          double2* M2 = ops.data() + o * PP;
          double2* L2 = ops.data() + ((size_t)F->n_tree_ops + o) * PP;
          for (int mi = -p; mi <= p; ++mi)
            for (int ni = -p; ni <= p; ++ni) {
              const zd f = fj[mi - ni + J];
              const double sm = ((mi - ni) & 1) ? -1.0 : 1.0;
              const double a = sm * sgv(l, lev, mi) / sgv(l, lev - 1, ni);
              const double b = sgv(l, lev, ni) / sgv(l, lev - 1, mi);
              M2[(size_t)(mi + p) * P + (ni + p)] = make_double2(f.re * a, f.im * a);
              L2[(size_t)(mi + p) * P + (ni + p)] = make_double2(f.re * b, f.im * b);
            }
        }
  }

  // ---- interaction lists --------------------------------------------------------
  std::map<std::tuple<int, int, int, int>, int> free_id;               // (layer, level, di, dj)
  std::map<std::tuple<int, int, int, int, int, int>, int> reac_id;     // (tt, ts, level, di, jt, js)
  auto free_tab = [&](int layer, int lev, int di, int dj) {
    auto key = std::make_tuple(layer, lev, di, dj);
    auto it = free_id.find(key);
    if (it != free_id.end()) return it->second;
    const int id = (int)free_id.size();
    free_id[key] = id;
    F->free_geo.push_back(m.k[layer]);
    F->free_geo.push_back(di * wl(lev));
    F->free_geo.push_back(dj * wl(lev));
    F->free_lvl.push_back(layer);
    F->free_lvl.push_back(lev);
    return id;
  };
  auto reac_tab = [&](int tt, int ts, int lev, int di, int jt, int js) {
    auto key = std::make_tuple(tt, ts, lev, di, jt, js);
    auto it = reac_id.find(key);
    if (it != reac_id.end()) return it->second;
    const int id = (int)reac_id.size();
    reac_id[key] = id;
    F->reac_meta.push_back(T[tt].layer);
    F->reac_meta.push_back(T[ts].layer);
    F->reac_meta.push_back(T[tt].side + 2 * T[ts].side);
    F->reac_meta.push_back(lev);
    F->reac_geo.push_back(di * wl(lev));
    F->reac_geo.push_back((jt + 0.5) * wl(lev));
    F->reac_geo.push_back((js + 0.5) * wl(lev));
    return id;
  };
  auto ij = [&](int b) {
    const BoxDev& B = F->boxes[b];
    const double w = wl(B.level);
    return std::make_pair((int)std::lround((B.cx - F->x0) / w - 0.5), (int)std::lround(B.ch / w - 0.5));
  };
  // ---- level 0 as a convolution along x ---------------------------------------
  // A level-0 box meets every non-adjacent level-0 box of its free tree and
  // every level-0 box of every side tree (no coarser level exists).  Its
  // operator depends on the rows (tree, j) of target and source and on the
  // column offset it - is alone, so per pair of rows that part of the M2L is
  // a Toeplitz product along the columns: transform the level-0 expansions
  // of each row (length top_L >= 2 nx - 1, zero padded, so the circular
  // convolution is the linear one on columns 0..nx-1), multiply per
  // frequency by the transformed operator sequence of each row pair, and
  // transform back.
  std::vector<double> top_free_geo, top_reac_geo;
  std::vector<int> top_free_lvl, top_reac_meta, top_cls_near;
  {
    std::map<std::pair<int, int>, int> row_of;  // (tree, j) -> row
    int nx = 0;
    int64_t nreac0 = 0, direct = 0;
    for (size_t ti = 0; ti < T.size(); ++ti) {
      for (int64_t kk : T[ti].keys[0]) {
        nx = std::max(nx, (int)(kk >> 32) + 1);
        row_of.emplace(std::make_pair((int)ti, (int)(uint32_t)kk), 0);
      }
      const int64_t n0 = (int64_t)T[ti].keys[0].size();
      if (T[ti].reac) nreac0 += n0;
      else direct += n0 * n0;
    }
    direct += nreac0 * nreac0;
    std::vector<std::pair<int, int>> rows;
    for (auto& kv : row_of) {
      kv.second = (int)rows.size();
      rows.push_back(kv.first);
    }
    int L = 2;
    while (L < 2 * nx - 1) L <<= 1;
    // row pairs of every target row, with their operator class
    std::map<std::tuple<int, int, int>, int> free_cls;       // (layer, dj, 0)
    std::map<std::tuple<int, int, int, int>, int> reac_cls;  // (tt, ts, jt, js)
    std::vector<std::vector<std::pair<int, int>>> pr(rows.size());  // (source row, class: free < 0)
    int64_t npairs = 0;
    for (size_t rt = 0; rt < rows.size(); ++rt) {
      const int tt = rows[rt].first, jt = rows[rt].second;
      for (size_t rs = 0; rs < rows.size(); ++rs) {
        const int ts = rows[rs].first, js = rows[rs].second;
        if (T[tt].reac != T[ts].reac || (!T[tt].reac && ts != tt)) continue;
        int c;
        if (T[tt].reac) {
          auto q = reac_cls.emplace(std::make_tuple(tt, ts, jt, js), (int)reac_cls.size()).first;
          c = q->second;
        } else {
          auto q = free_cls.emplace(std::make_tuple(T[tt].layer, jt - js, 0), (int)free_cls.size()).first;
          c = -1 - q->second;
        }
        pr[rt].push_back({(int)rs, c});
      }
      npairs += (int64_t)pr[rt].size();
    }
    const size_t ncls = reac_cls.size() + free_cls.size();
    // device bytes: transformed sequences (FP64 + complex64) and, during
    // setup, the tables at every offset
    const double PPd = (double)(2 * p + 1) * (2 * p + 1);
    const double top_bytes = (double)ncls * PPd * (24.0 * L + 16.0 * (2 * nx - 1));
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) fr = 0;
    F->top_on = nx > 0 && L <= 2048 && rows.size() < 65536 && ncls < 65536 &&
                (g->top_fft > 0 || (g->top_fft == 0 && direct > 2 * npairs * L && top_bytes <= 0.25 * (double)fr));
    if (F->top_on) {
      const int nrc = (int)reac_cls.size(), nfc = (int)free_cls.size(), D = 2 * nx - 1;
      F->top_rows = (int)rows.size();
      F->top_nx = nx;
      F->top_L = L;
      F->top_ncls = nrc + nfc;
      F->top_direct = direct;
      F->top_grid.assign((size_t)rows.size() * nx, -1);
      for (size_t ti = 0; ti < T.size(); ++ti)
        for (int64_t kk : T[ti].keys[0]) {
          const int r = row_of.at({(int)ti, (int)(uint32_t)kk});
          F->top_grid[(size_t)r * nx + (int)(kk >> 32)] = T[ti].idx[0].at(kk);
        }
      // tables of every class at every offset di = -(nx-1) .. nx-1 (class
      // c, offset di at c * D + di + nx - 1; reaction classes first).  The
      // offsets of adjacent boxes (|di| <= 1 in a near class) are not
      // interactions: they get a harmless geometry and are masked out.
      top_cls_near.assign(F->top_ncls, 0);
      top_reac_meta.resize((size_t)nrc * D * 4);
      top_reac_geo.resize((size_t)nrc * D * 3);
      top_free_geo.resize((size_t)nfc * D * 3);
      top_free_lvl.resize((size_t)nfc * D * 2);
      const double w0 = wl(0);
      for (auto& kv : reac_cls) {
        const int c = kv.second;
        const int tt = std::get<0>(kv.first), ts = std::get<1>(kv.first);
        const int jt = std::get<2>(kv.first), js = std::get<3>(kv.first);
        const bool near = jt == 0 && js == 0;
        top_cls_near[c] = near;
        for (int di = -(nx - 1); di <= nx - 1; ++di) {
          const size_t t = (size_t)c * D + di + nx - 1;
          const int dd = near && std::abs(di) <= 1 ? 2 : di;
          top_reac_meta[4 * t] = T[tt].layer;
          top_reac_meta[4 * t + 1] = T[ts].layer;
          top_reac_meta[4 * t + 2] = T[tt].side + 2 * T[ts].side;
          top_reac_meta[4 * t + 3] = 0;
          top_reac_geo[3 * t] = dd * w0;
          top_reac_geo[3 * t + 1] = (jt + 0.5) * w0;
          top_reac_geo[3 * t + 2] = (js + 0.5) * w0;
        }
      }
      for (auto& kv : free_cls) {
        const int c = kv.second;
        const int layer = std::get<0>(kv.first), dj = std::get<1>(kv.first);
        const bool near = std::abs(dj) <= 1;
        top_cls_near[nrc + c] = near;
        for (int di = -(nx - 1); di <= nx - 1; ++di) {
          const size_t t = (size_t)c * D + di + nx - 1;
          const int dd = near && std::abs(di) <= 1 ? 2 : di;
          top_free_geo[3 * t] = m.k[layer];
          top_free_geo[3 * t + 1] = dd * w0;
          top_free_geo[3 * t + 2] = dj * w0;
          top_free_lvl[2 * t] = layer;
          top_free_lvl[2 * t + 1] = 0;
        }
      }
      // frequency-domain items: target (row, frequency) sums, over the row
      // pairs of its row, the transformed operator of the pair's class times
      // the transformed source row at the same frequency
      F->top_ptr.push_back(0);
      for (size_t rt = 0; rt < rows.size(); ++rt)
        for (int f = 0; f < L; ++f) {
          const int e0 = (int)F->top_src.size();
          for (auto& q : pr[rt]) {
            const int c = q.second >= 0 ? q.second : nrc + (-1 - q.second);
            F->top_src.push_back(q.first * L + f);
            F->top_op.push_back(c * L + f);
          }
          F->top_item.insert(F->top_item.end(), {(int)(rt * L + f), e0, (int)F->top_src.size()});
          F->top_ptr.push_back((int)F->top_src.size());
        }
    }
  }
  for (int b = 0; b < F->n_boxes; ++b) {
    const BoxDev& B = F->boxes[b];
    const TreeB& tb = T[B.tree];
    const int lev = B.level;
    if (lev == 0 && F->top_on) continue;  // the level-0 convolution covers it
    auto [it, jt] = ij(b);
    std::vector<std::pair<int, int>> lst;  // (source, tab)
    if (!tb.reac) {
      if (lev == 0) {
        for (int64_t kk : tb.keys[0]) {
          const int is = (int)(kk >> 32), js = (int)(uint32_t)kk;
          if (std::abs(is - it) <= 1 && std::abs(js - jt) <= 1) continue;
          lst.push_back({tb.idx[0].at(kk), -1 - free_tab(tb.layer, 0, it - is, jt - js)});
        }
      } else {
        auto [Ip, Jp] = ij(B.parent);
        for (int dI = -1; dI <= 1; ++dI)
          for (int dJ = -1; dJ <= 1; ++dJ) {
            auto q = tb.idx[lev - 1].find(bkey(Ip + dI, Jp + dJ));
            if (Ip + dI < 0 || Jp + dJ < 0 || q == tb.idx[lev - 1].end()) continue;
            const BoxDev& Q = F->boxes[q->second];
            for (int c = 0; c < Q.nchild; ++c) {
              const int cb = F->children[Q.child0 + c];
              auto [is, js] = ij(cb);
              if (std::abs(is - it) <= 1 && std::abs(js - jt) <= 1) continue;
              lst.push_back({cb, -1 - free_tab(tb.layer, lev, it - is, jt - js)});
            }
          }
      }
    } else {
      // reaction: every source side tree
      for (size_t ts = 0; ts < T.size(); ++ts) {
        const TreeB& sb = T[ts];
        if (!sb.reac) continue;
        if (lev == 0) {
          for (int64_t kk : sb.keys[0]) {
            const int is = (int)(kk >> 32), js = (int)(uint32_t)kk;
            if (std::abs(is - it) <= 1 && jt == 0 && js == 0) continue;
            lst.push_back({sb.idx[0].at(kk), reac_tab(B.tree, (int)ts, 0, it - is, jt, js)});
          }
        } else {
          auto [Ip, Jp] = ij(B.parent);
          (void)Jp;
          for (int dI = -1; dI <= 1; ++dI) {
            if (Ip + dI < 0) continue;
            auto q = sb.idx[lev - 1].find(bkey(Ip + dI, 0));
            if (q == sb.idx[lev - 1].end()) continue;
            const BoxDev& Q = F->boxes[q->second];
            for (int c = 0; c < Q.nchild; ++c) {
              const int cb = F->children[Q.child0 + c];
              auto [is, js] = ij(cb);
              if (std::abs(is - it) <= 1 && jt == 0 && js == 0) continue;
              lst.push_back({cb, reac_tab(B.tree, (int)ts, lev, it - is, jt, js)});
            }
          }
        }
      }
    }
    if (lst.empty()) continue;
    F->m2l_tgt.push_back(b);
    F->m2l_ptr.push_back((int)F->m2l_src.size());
    for (auto& e : lst) {
      F->m2l_src.push_back(e.first);
      F->m2l_tab.push_back(e.second);
    }
  }
  F->m2l_ptr.push_back((int)F->m2l_src.size());

  // free near field (leaf level lf)
  for (int b : F->leaf_free) {
    const BoxDev& B = F->boxes[b];
    const TreeB& tb = T[B.tree];
    auto [it, jt] = ij(b);
    F->near_tgt.push_back(b);
    F->near_ptr.push_back((int)F->near_src.size());
    for (int di = -1; di <= 1; ++di)
      for (int dj = -1; dj <= 1; ++dj) {
        if (it + di < 0 || jt + dj < 0) continue;
        auto q = tb.idx[B.level].find(bkey(it + di, jt + dj));
        if (q != tb.idx[B.level].end()) F->near_src.push_back(q->second);
      }
  }
  F->near_ptr.push_back((int)F->near_src.size());

  // reaction near field: row-0 leaves at level lr adjacent in image space
  {
    std::unordered_map<int64_t, unsigned> pairs;
    for (size_t tt = 0; tt < T.size(); ++tt) {
      if (!T[tt].reac) continue;
      for (int64_t kt : T[tt].keys[lr]) {
        if ((uint32_t)kt != 0) continue;
        const int it = (int)(kt >> 32);
        const BoxDev& Bt = F->boxes[T[tt].idx[lr].at(kt)];
        for (size_t ts = 0; ts < T.size(); ++ts) {
          if (!T[ts].reac) continue;
          const unsigned bit = 1u << (T[tt].side + 2 * T[ts].side);
          for (int di = -1; di <= 1; ++di) {
            if (it + di < 0) continue;
            auto q = T[ts].idx[lr].find(bkey(it + di, 0));
            if (q == T[ts].idx[lr].end()) continue;
            const BoxDev& Bs = F->boxes[q->second];
            for (int a = 0; a < Bt.npt; ++a)
              for (int c = 0; c < Bs.npt; ++c) {
                const int64_t key = ((int64_t)F->pt_elem[Bt.pt0 + a] << 32) | (uint32_t)F->pt_elem[Bs.pt0 + c];
                pairs[key] |= bit;
              }
          }
        }
      }
    }
    std::vector<std::pair<int64_t, unsigned>> pv(pairs.begin(), pairs.end());
    std::sort(pv.begin(), pv.end());
    F->rn_ptr.assign(N + 1, 0);
    for (auto& e : pv) {
      F->rn_ptr[(e.first >> 32) + 1]++;
      F->rn_src.push_back((int)(uint32_t)e.first);
      F->rn_mask.push_back(e.second);
    }
    for (int64_t i = 0; i < N; ++i) F->rn_ptr[i + 1] += F->rn_ptr[i];
    for (int64_t i = 0; i < N; ++i)
      if (F->rn_ptr[i + 1] > F->rn_ptr[i]) F->rn_rows.push_back((int)i);
  }

  // ---- near-field matrix (CSR by element): free near, reaction near, self ----
  std::vector<int> nm_tgt;
  std::vector<unsigned> nm_kind;
  {
    std::vector<int> leaf_slot(N, -1);  // index into near_tgt of the element's free leaf
    for (size_t t = 0; t < F->near_tgt.size(); ++t) {
      const BoxDev& B = F->boxes[F->near_tgt[t]];
      for (int i = 0; i < B.npt; ++i) leaf_slot[F->pt_elem[B.pt0 + i]] = (int)t;
    }
    F->nm_ptr.assign(N + 1, 0);
    int64_t nnz = 0;
    for (int64_t i = 0; i < N; ++i) {
      int64_t len = 1 + (F->rn_ptr[i + 1] - F->rn_ptr[i]);
      const int t = leaf_slot[i];
      for (int e = F->near_ptr[t]; e < F->near_ptr[t + 1]; ++e) len += F->boxes[F->near_src[e]].npt;
      len -= 1;  // the element itself
      nnz += len;
      LM_CHECK(nnz < ((int64_t)1 << 31), LM_ENOMEM, "near-field matrix too large");
      F->nm_ptr[i + 1] = (int)nnz;
    }
    F->nm_src.resize(nnz);
    nm_tgt.resize(nnz);
    nm_kind.resize(nnz);
    for (int64_t i = 0; i < N; ++i) {
      int64_t q = F->nm_ptr[i];
      F->nm_src[q] = (int)i;
      nm_kind[q] = 0xFFFFFFFFu;
      nm_tgt[q++] = (int)i;
      for (int e = F->rn_ptr[i]; e < F->rn_ptr[i + 1]; ++e) {
        F->nm_src[q] = F->rn_src[e];
        nm_kind[q] = F->rn_mask[e];
        nm_tgt[q++] = (int)i;
      }
      const int t = leaf_slot[i];
      for (int e = F->near_ptr[t]; e < F->near_ptr[t + 1]; ++e) {
        const BoxDev& C = F->boxes[F->near_src[e]];
        for (int j = 0; j < C.npt; ++j) {
          const int el = F->pt_elem[C.pt0 + j];
          if (el == (int)i) continue;
          F->nm_src[q] = el;
          nm_kind[q] = 0u;
          nm_tgt[q++] = (int)i;
        }
      }
    }
  }
  // ---- free-space near field + self terms as leaf blocks (matrix-core apply) ----
  {
    F->nb_jptr.push_back(0);
    int64_t z = 0;
    for (size_t t = 0; t < F->near_tgt.size(); ++t) {
      const int b = F->near_tgt[t];
      const BoxDev& B = F->boxes[b];
      for (int i = 0; i < B.npt; ++i) F->nb_jidx.push_back(F->pt_elem[B.pt0 + i]);
      for (int e = F->near_ptr[t]; e < F->near_ptr[t + 1]; ++e) {
        const int c = F->near_src[e];
        if (c == b) continue;
        const BoxDev& Cb = F->boxes[c];
        for (int i = 0; i < Cb.npt; ++i) F->nb_jidx.push_back(F->pt_elem[Cb.pt0 + i]);
      }
      LM_CHECK(F->nb_jidx.size() < ((size_t)1 << 31), LM_ENOMEM, "near-field blocks too large");
      const int q = (int)F->nb_jidx.size() - F->nb_jptr.back();
      F->nb_jptr.push_back((int)F->nb_jidx.size());
      F->nb_rows.push_back(B.npt);
      F->nb_zoff.push_back(z);
      for (int r = 0; r < B.npt; r += PA_ROWS) {
        F->nb_item.push_back((int)t);
        F->nb_item.push_back(r);
      }
      z += (int64_t)q * B.npt;
    }
    F->nb_nnz = z;
    // items write disjoint rows: launch the largest (rows x columns) first
    const int nit = (int)F->nb_item.size() / 2;
    std::vector<int64_t> work(nit);
    std::vector<int> ord(nit);
    for (int i = 0; i < nit; ++i) {
      const int t = F->nb_item[2 * i], r = F->nb_item[2 * i + 1];
      work[i] = (int64_t)std::min(PA_ROWS, F->nb_rows[t] - r) * (F->nb_jptr[t + 1] - F->nb_jptr[t]);
      ord[i] = i;
    }
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return work[a] > work[b]; });
    std::vector<int> sorted(F->nb_item.size());
    for (int i = 0; i < nit; ++i) {
      sorted[2 * i] = F->nb_item[2 * ord[i]];
      sorted[2 * i + 1] = F->nb_item[2 * ord[i] + 1];
    }
    F->nb_item.swap(sorted);
  }

  // ---- M2L entries grouped by operator ----------------------------------------
  {
    F->n_reac_tab = (int)reac_id.size();
    F->n_free_tab = (int)free_id.size();
    const int ntab = F->n_reac_tab + F->n_free_tab;
    F->tm_ptr.assign(ntab + 1, 0);
    auto tabidx = [&](int t) { return t >= 0 ? t : F->n_reac_tab + (-t - 1); };
    for (int t : F->m2l_tab) F->tm_ptr[tabidx(t) + 1]++;
    for (int i = 0; i < ntab; ++i) F->tm_ptr[i + 1] += F->tm_ptr[i];
    std::vector<int> fill(F->tm_ptr.begin(), F->tm_ptr.end() - 1);
    F->tm_slot.resize(F->m2l_tab.size());
    F->tm_src.resize(F->m2l_tab.size());
    for (size_t e = 0; e < F->m2l_tab.size(); ++e) {
      const int q = fill[tabidx(F->m2l_tab[e])]++;
      F->tm_slot[q] = (int)e;
      F->tm_src[q] = F->m2l_src[e];
    }
    // matrix-core M2L items: slots in target order; launched longest first so
    // that the short items fill in behind the long ones
    std::vector<int> it;
    F->mf_ptr.push_back(0);
    for (size_t t = 0; t < F->m2l_tgt.size(); ++t) {
      for (int e = F->m2l_ptr[t]; e < F->m2l_ptr[t + 1]; e += M2L_MF_ITEM) {
        it.push_back((int)t);
        it.push_back(e);
        it.push_back(std::min(e + M2L_MF_ITEM, F->m2l_ptr[t + 1]));
      }
      F->mf_ptr.push_back((int)it.size() / 3);
    }
    const int nit = (int)it.size() / 3;
    F->mf_slot.resize(nit);
    for (int i = 0; i < nit; ++i) F->mf_slot[i] = i;
    std::stable_sort(F->mf_slot.begin(), F->mf_slot.end(),
                     [&](int a, int b) { return it[3 * a + 2] - it[3 * a + 1] > it[3 * b + 2] - it[3 * b + 1]; });
    F->mf_item.resize(it.size());
    for (int i = 0; i < nit; ++i)
      for (int c = 0; c < 3; ++c) F->mf_item[3 * i + c] = it[3 * F->mf_slot[i] + c];
    for (int t = 0; t < ntab; ++t)
      for (int e = F->tm_ptr[t]; e < F->tm_ptr[t + 1]; e += M2L_ITEM) {
        F->tm_item.push_back(t);
        F->tm_item.push_back(e);
        F->tm_item.push_back(std::min(e + M2L_ITEM, F->tm_ptr[t + 1]));
      }
    {  // operator-major items write per-entry slots: launch the longest first
      const int n = (int)F->tm_item.size() / 3;
      std::vector<int> ord(n);
      for (int i = 0; i < n; ++i) ord[i] = i;
      const std::vector<int>& ti = F->tm_item;
      std::stable_sort(ord.begin(), ord.end(),
                       [&](int a, int b) { return ti[3 * a + 2] - ti[3 * a + 1] > ti[3 * b + 2] - ti[3 * b + 1]; });
      std::vector<int> sorted(ti.size());
      for (int i = 0; i < n; ++i)
        for (int c = 0; c < 3; ++c) sorted[3 * i + c] = ti[3 * ord[i] + c];
      F->tm_item.swap(sorted);
    }
  }

  // ---- translation items for the matrix-core M2M / L2L ------------------------------
  // M2M: item k = parent parents_by_level[k], entries = its children with
  // their M2M operators; L2L: one item per box of level >= 1 (in box order),
  // entry = its parent with the L2L operator.  Operator indices count from the
  // start of the operator array.
  {
    auto tr_op = [&](const BoxDev& c, int base) { return base + (tree_layer[c.tree] * nlev + c.level) * 4 + c.pos; };
    for (int b : F->parents_by_level) {
      const BoxDev& B = F->boxes[b];
      F->tr_item.push_back(0);
      F->tr_item.push_back((int)F->tr_src.size());
      for (int c = 0; c < B.nchild; ++c) {
        const int cb = F->children[B.child0 + c];
        F->tr_src.push_back(cb);
        F->tr_op.push_back(tr_op(F->boxes[cb], 0));
      }
      F->tr_item.push_back((int)F->tr_src.size());
    }
    F->l2l_item0 = (int)F->tr_item.size() / 3;
    for (int b = F->level_ptr[1]; b < F->n_boxes; ++b) {
      const BoxDev& B = F->boxes[b];
      F->tr_item.push_back(0);
      F->tr_item.push_back((int)F->tr_src.size());
      F->tr_src.push_back(B.parent);
      F->tr_op.push_back(tr_op(B, F->n_tree_ops));
      F->tr_item.push_back((int)F->tr_src.size());
    }
  }
  {
    std::vector<int> ids(F->n_boxes);
    for (int b = 0; b < F->n_boxes; ++b) ids[b] = b;
    LM_TRY(up(F->d_box_id, ids, s));
  }
  LM_TRY(up(F->d_tr_item, F->tr_item, s));
  LM_TRY(up(F->d_tr_src, F->tr_src, s));
  LM_TRY(up(F->d_tr_op, F->tr_op, s));

  // ---- upload and device setup ---------------------------------------------------
  LM_TRY(up(F->d_boxes, F->boxes, s));
  LM_TRY(up(F->d_children, F->children, s));
  LM_TRY(up(F->d_pt_elem, F->pt_elem, s));
  LM_TRY(up(F->d_pt_xh, F->pt_xh, s));
  LM_TRY(up(F->d_pt_item, F->pt_item, s));
  LM_TRY(up(F->d_p2m_leaf, F->p2m_leaf, s));
  LM_TRY(up(F->d_p2m_ptr, F->p2m_ptr, s));
  LM_TRY(up(F->d_p2m_dst, F->p2m_dst, s));
  LM_TRY(up(F->d_p2m_msel, F->p2m_msel, s));
  LM_TRY(up(F->d_parents, F->parents_by_level, s));
  LM_TRY(up(F->d_m2l_tgt, F->m2l_tgt, s));
  {  // every other box starts its local expansion from zero
    std::vector<char> written(F->n_boxes, 0);
    for (int b : F->m2l_tgt) written[b] = 1;
    F->le_zero.clear();
    for (int b = 0; b < F->n_boxes; ++b)
      if (!written[b] && !(F->top_on && F->boxes[b].level == 0)) F->le_zero.push_back(b);
    LM_TRY(up(F->d_le_zero, F->le_zero, s));
  }
  LM_TRY(up(F->d_m2l_ptr, F->m2l_ptr, s));
  LM_TRY(up(F->d_m2l_src, F->m2l_src, s));
  LM_TRY(up(F->d_m2l_tab, F->m2l_tab, s));
  LM_TRY(up(F->d_near_tgt, F->near_tgt, s));
  LM_TRY(up(F->d_near_ptr, F->near_ptr, s));
  LM_TRY(up(F->d_near_src, F->near_src, s));
  LM_TRY(up(F->d_rn_ptr, F->rn_ptr, s));
  LM_TRY(up(F->d_rn_rows, F->rn_rows, s));
  LM_TRY(up(F->d_rn_src, F->rn_src, s));
  F->tree_layer = tree_layer;
  F->tree_side.clear();
  for (const TreeB& t : T) F->tree_side.push_back(t.side);
  LM_TRY(up(F->d_tree_side, F->tree_side, s));
  LM_TRY(up(F->d_tree_layer, F->tree_layer, s));
  LM_TRY(up(F->d_sig, F->sig, s));
  {
    std::vector<double2> self(N);
    for (int64_t e = 0; e < N; ++e) {
      const double k = m.k[g->layer[e]], w = g->w[e];
      if (g->quad == LM_QUAD_SPECTRAL) {
        // free-space diagonal of the spectral rule: R_0 m1 + (2 pi / M) m2 at
        // t = s, m1 = -|x'| / (4 pi), m2 = (i/4 - gamma/(2 pi) - ln(k |x'| / 2)/(2 pi)) |x'|
        const double sp = g->speed[e], M = g->cnt[e], R0 = g->logw[g->roff[g->sid[e]]];
        self[e] = make_double2(-R0 * sp / (4.0 * M_PI) +
                                   2.0 * M_PI / M * (-kEulerGamma - std::log(0.5 * k * sp)) / (2.0 * M_PI) * sp,
                               2.0 * M_PI / M * 0.25 * sp);
      } else {
        self[e] = make_double2(-(kEulerGamma + std::log(k * w / 4.0) - 1.0) / (2.0 * M_PI) * w, 0.25 * w);
      }
      if (g->bc != LM_BC_DIRICHLET)  // -1/2 + i beta I^s (the free-space K' self term of a chord is zero)
        self[e] = make_double2(-0.5 - g->robin_beta * self[e].y, g->robin_beta * self[e].x);
    }
    LM_TRY(up(F->d_self, self, s));
  }
  // operators: [M2M | L2L | reaction M2L | free-space M2L], P x P each
  const int nfree = (int)free_id.size(), nreac = (int)reac_id.size();
  F->op_m2l = 2 * F->n_tree_ops;
  const int64_t nops = (int64_t)F->op_m2l + nreac + nfree;
  LM_TRY(F->d_ops64.alloc((size_t)nops * PP * sizeof(double2)));
  LM_TRY_HIP(hipMemcpyAsync(F->d_ops64.p, ops.data(), ops.size() * sizeof(double2), hipMemcpyHostToDevice, s));
  double2* m2l_ops = F->d_ops64.as<double2>() + (size_t)F->op_m2l * PP;
  if (nreac) {
    DevBuf meta, geo;
    LM_TRY(up(meta, F->reac_meta, s));
    LM_TRY(up(geo, F->reac_geo, s));
    hipLaunchKernelGGL(k_reac_tables, dim3(nreac), dim3(256), 0, s, m, p, nlev, meta.as<int>(), geo.as<double>(),
                       F->d_sig.as<double>(), m2l_ops);
    LM_TRY_HIP(hipGetLastError());
    LM_TRY_HIP(hipStreamSynchronize(s));
  }
  if (nfree) {
    DevBuf geo, lvl;
    LM_TRY(up(geo, F->free_geo, s));
    LM_TRY(up(lvl, F->free_lvl, s));
    hipLaunchKernelGGL(k_free_tables, dim3(nfree), dim3(64), 0, s, p, nlev, geo.as<double>(), lvl.as<int>(),
                       F->d_sig.as<double>(), m2l_ops + (size_t)nreac * PP);
    LM_TRY_HIP(hipGetLastError());
    LM_TRY_HIP(hipStreamSynchronize(s));
  }
  LM_TRY(F->d_ops32.alloc((size_t)nops * PP * sizeof(float2)));
  hipLaunchKernelGGL(k_c128_to_c64_fmm, dim3(div_up(nops * (int64_t)PP, 256)), dim3(256), 0, s,
                     nops * (int64_t)PP, F->d_ops64.as<double2>(), F->d_ops32.as<float2>());
  LM_TRY_HIP(hipGetLastError());
  {
    // per M2L entry: operator index into the M2L part
    std::vector<int> opi(F->m2l_tab.size());
    for (size_t e = 0; e < opi.size(); ++e) {
      const int t = F->m2l_tab[e];
      opi[e] = t >= 0 ? t : nreac + (-t - 1);
    }
    LM_TRY(up(F->d_m2l_op, opi, s));
  }
  if (F->top_on) {
    // level-0 convolution: operator tables at every offset (temporary),
    // their transforms along the offset (FP64 and FP32), the index arrays
    const int nx = F->top_nx, L = F->top_L, D = 2 * nx - 1;
    const int nrc = (int)(top_reac_meta.size() / (4 * (size_t)D)), nfc = (int)(top_free_lvl.size() / (2 * (size_t)D));
    int lgL = 0;
    while ((1 << lgL) < L) ++lgL;
    std::vector<double2> tw(L / 2);
    std::vector<float2> tw32(L / 2);
    for (int t = 0; t < L / 2; ++t) {
      const double a = -2.0 * M_PI * t / L;
      tw[t] = make_double2(std::cos(a), std::sin(a));
      tw32[t] = make_float2((float)tw[t].x, (float)tw[t].y);
    }
    LM_TRY(up(F->d_top_tw64, tw, s));
    LM_TRY(up(F->d_top_tw32, tw32, s));
    DevBuf tab, near;
    LM_TRY(tab.alloc((size_t)F->top_ncls * D * PP * sizeof(double2)));
    if (nrc) {
      DevBuf meta, geo;
      LM_TRY(up(meta, top_reac_meta, s));
      LM_TRY(up(geo, top_reac_geo, s));
      hipLaunchKernelGGL(k_reac_tables, dim3(nrc * D), dim3(256), 0, s, m, p, nlev, meta.as<int>(), geo.as<double>(),
                         F->d_sig.as<double>(), tab.as<double2>());
      LM_TRY_HIP(hipGetLastError());
      LM_TRY_HIP(hipStreamSynchronize(s));
    }
    if (nfc) {
      DevBuf geo, lvl;
      LM_TRY(up(geo, top_free_geo, s));
      LM_TRY(up(lvl, top_free_lvl, s));
      hipLaunchKernelGGL(k_free_tables, dim3(nfc * D), dim3(64), 0, s, p, nlev, geo.as<double>(), lvl.as<int>(),
                         F->d_sig.as<double>(), tab.as<double2>() + (size_t)nrc * D * PP);
      LM_TRY_HIP(hipGetLastError());
      LM_TRY_HIP(hipStreamSynchronize(s));
    }
    LM_TRY(up(near, top_cls_near, s));
    LM_TRY(F->d_top_T64.alloc((size_t)F->top_ncls * L * PP * sizeof(double2)));
    LM_TRY(F->d_top_T32.alloc((size_t)F->top_ncls * L * PP * sizeof(float2)));
    const int lgc = top_lgc(lgL, sizeof(double2));
    hipLaunchKernelGGL(k_top_tables, dim3(div_up((int64_t)PP, 1 << lgc), F->top_ncls), dim3(256),
                       ((size_t)L << lgc) * sizeof(double2), s, lgL, lgc, nx, (int)PP, tab.as<double2>(),
                       near.as<int>(), F->d_top_tw64.as<double2>(), F->d_top_T64.as<double2>(),
                       F->d_top_T32.as<float2>());
    LM_TRY_HIP(hipGetLastError());
    LM_TRY_HIP(hipStreamSynchronize(s));
    std::vector<int> id((size_t)F->top_rows * L);
    for (size_t i = 0; i < id.size(); ++i) id[i] = (int)i;
    LM_TRY(up(F->d_top_id, id, s));
    LM_TRY(up(F->d_top_grid, F->top_grid, s));
    LM_TRY(up(F->d_top_item, F->top_item, s));
    LM_TRY(up(F->d_top_ptr, F->top_ptr, s));
    LM_TRY(up(F->d_top_src, F->top_src, s));
    LM_TRY(up(F->d_top_op, F->top_op, s));
    LM_TRY_HIP(hipStreamSynchronize(s));  // host staging vectors end with this scope
  }
  // near-field matrix values (what the targets see: the operator itself, or
  // n . grad + i beta of it for sound-hard / impedance scatterers)
  const BcTarget bct{g->bc, g->robin_beta, g->d_nx.as<double>(), g->d_ny.as<double>()};
  const int nrn = (int)F->rn_src.size();
  {
    const int64_t nnz = F->nm_ptr[N];
    LM_TRY(up(F->d_nm_ptr, F->nm_ptr, s));
    LM_TRY(up(F->d_nm_src, F->nm_src, s));
    DevBuf dt, dk;
    LM_TRY(up(dt, nm_tgt, s));
    LM_TRY(up(dk, nm_kind, s));
    LM_TRY(F->d_nm_val.alloc(std::max<int64_t>(nnz, 1) * sizeof(double2)));
    hipLaunchKernelGGL(k_near_values, dim3(div_up(nnz, 128)), dim3(128), 0, s, m, nnz, dt.as<int>(),
                       F->d_nm_src.as<int>(), dk.as<unsigned>(), g->d_cx.as<double>(), g->d_cy.as<double>(),
                       g->d_w.as<double>(), g->d_layer.as<int>(), F->d_self.as<double2>(), bct, F->d_nm_val.as<double2>());
    LM_TRY_HIP(hipGetLastError());
    LM_TRY(F->d_nm_val32.alloc(std::max<int64_t>(nnz, 1) * sizeof(float2)));
    hipLaunchKernelGGL(k_c128_to_c64_fmm, dim3(div_up(nnz, 256)), dim3(256), 0, s, nnz, F->d_nm_val.as<double2>(),
                       F->d_nm_val32.as<float2>());
    LM_TRY_HIP(hipGetLastError());
    LM_TRY_HIP(hipStreamSynchronize(s));
  }
  {
    LM_TRY(up(F->d_nb_jptr, F->nb_jptr, s));
    LM_TRY(up(F->d_nb_jidx, F->nb_jidx, s));
    LM_TRY(up(F->d_nb_rows, F->nb_rows, s));
    LM_TRY(up(F->d_nb_zoff, F->nb_zoff, s));
    LM_TRY(up(F->d_nb_item, F->nb_item, s));
    LM_TRY(F->d_nb_Z32.alloc(std::max<int64_t>(F->nb_nnz, 1) * sizeof(float2)));
    if (!F->nb_rows.empty())
      hipLaunchKernelGGL(k_near_block_values, dim3(F->nb_rows.size()), dim3(256), 0, s, m, F->d_nb_jptr.as<int>(),
                         F->d_nb_jidx.as<int>(), F->d_nb_rows.as<int>(), F->d_nb_zoff.as<int64_t>(),
                         g->d_cx.as<double>(), g->d_cy.as<double>(), g->d_w.as<double>(), g->d_layer.as<int>(),
                         F->d_self.as<double2>(), bct, F->d_nb_Z32.as<float2>());
    // reaction near pairs alone, as CSR (the rest of the near field is in the blocks)
    const int64_t nr = (int64_t)F->rn_src.size();
    std::vector<int> rt(nr);
    for (int64_t i = 0; i < N; ++i)
      for (int e = F->rn_ptr[i]; e < F->rn_ptr[i + 1]; ++e) rt[e] = (int)i;
    DevBuf dt, dk, v64;
    LM_TRY(up(dt, rt, s));
    LM_TRY(up(dk, F->rn_mask, s));
    LM_TRY(v64.alloc(std::max<int64_t>(nr, 1) * sizeof(double2)));
    LM_TRY(F->d_rn_val32.alloc(std::max<int64_t>(nr, 1) * sizeof(float2)));
    if (nr) {
      hipLaunchKernelGGL(k_near_values, dim3(div_up(nr, 128)), dim3(128), 0, s, m, nr, dt.as<int>(),
                         F->d_rn_src.as<int>(), dk.as<unsigned>(), g->d_cx.as<double>(), g->d_cy.as<double>(),
                         g->d_w.as<double>(), g->d_layer.as<int>(), F->d_self.as<double2>(), bct, v64.as<double2>());
      hipLaunchKernelGGL(k_c128_to_c64_fmm, dim3(div_up(nr, 256)), dim3(256), 0, s, nr, v64.as<double2>(),
                         F->d_rn_val32.as<float2>());
    }
    LM_TRY_HIP(hipGetLastError());
    LM_TRY_HIP(hipStreamSynchronize(s));
  }
  if (g->quad == LM_QUAD_SPECTRAL) {  // same-scatterer corrections of the spectral rule
    F->sc_ptr.assign(N + 1, 0);
    F->sc_src.clear();
    std::vector<int> st;
    for (int64_t i = 0; i < N; ++i) {
      const int64_t a = i - g->loc[i], M = g->cnt[i];
      for (int64_t e = a; e < a + M; ++e)
        if (e != i) {
          F->sc_src.push_back((int)e);
          st.push_back((int)i);
        }
      LM_CHECK(F->sc_src.size() < ((size_t)1 << 31), LM_ENOMEM, "too many same-scatterer pairs");
      F->sc_ptr[i + 1] = (int)F->sc_src.size();
    }
    const int64_t nc = (int64_t)F->sc_src.size();
    DevBuf dt;
    LM_TRY(up(F->d_sc_ptr, F->sc_ptr, s));
    LM_TRY(up(F->d_sc_src, F->sc_src, s));
    LM_TRY(up(dt, st, s));
    LM_TRY(F->d_sc_val.alloc(std::max<int64_t>(nc, 1) * sizeof(double2)));
    LM_TRY(F->d_sc_val32.alloc(std::max<int64_t>(nc, 1) * sizeof(float2)));
    if (nc) {
      hipLaunchKernelGGL(k_spectral_corr, dim3(div_up(nc, 256)), dim3(256), 0, s, m, nc, dt.as<int>(),
                         F->d_sc_src.as<int>(), g->d_cx.as<double>(), g->d_cy.as<double>(), g->d_layer.as<int>(),
                         g->d_sid.as<int>(), g->d_loc.as<int>(), g->d_cnt.as<int>(), g->d_speed.as<double>(),
                         g->d_logw.as<double>(), g->d_roff.as<int64_t>(), F->d_sc_val.as<double2>());
      hipLaunchKernelGGL(k_c128_to_c64_fmm, dim3(div_up(nc, 256)), dim3(256), 0, s, nc, F->d_sc_val.as<double2>(),
                         F->d_sc_val32.as<float2>());
    }
    LM_TRY_HIP(hipGetLastError());
    LM_TRY_HIP(hipStreamSynchronize(s));
  }
  LM_TRY(up(F->d_tm_ptr, F->tm_ptr, s));
  LM_TRY(up(F->d_tm_item, F->tm_item, s));
  LM_TRY(up(F->d_mf_item, F->mf_item, s));
  LM_TRY(up(F->d_mf_ptr, F->mf_ptr, s));
  LM_TRY(up(F->d_mf_slot, F->mf_slot, s));
  LM_TRY(up(F->d_tm_slot, F->tm_slot, s));
  LM_TRY(up(F->d_tm_src, F->tm_src, s));
  // point matrices of the matrix-core P2M / L2P
  {
    const size_t npt = std::max<size_t>(F->pt_elem.size(), 1) * F->P * sizeof(float2);
    LM_TRY(F->d_p2m_Z32.alloc(npt));
    LM_TRY(F->d_l2p_Z32.alloc(npt));
    if (g->bc != LM_BC_DIRICHLET) LM_TRY(F->d_l2p_Z64.alloc(2 * npt));
    if (F->item_ptr[3])
      hipLaunchKernelGGL(k_leaf_basis, dim3(F->item_ptr[3]), dim3(64), 0, s, p, F->nlev, F->d_pt_item.as<int>(),
                         F->d_boxes.as<BoxDev>(), F->d_tree_layer.as<int>(), F->d_sig.as<double>(),
                         F->d_pt_elem.as<int>(), F->d_pt_xh.as<double2>(), g->d_w.as<double>(),
                         BcTarget{g->bc, g->robin_beta, g->d_nx.as<double>(), g->d_ny.as<double>()},
                         F->d_tree_side.as<int>(), F->d_p2m_Z32.as<float2>(), F->d_l2p_Z32.as<float2>(),
                         F->d_l2p_Z64.as<double2>());
    LM_TRY_HIP(hipGetLastError());
  }
  LM_TRY(fmm_reserve(F, 1));
  {
    size_t lds = 0;
    for (int r = 1; r <= LM_RCHUNK; ++r) lds = std::max(lds, mf_lds_bytes(F->P, r));
    LM_TRY_HIP(m2l_mfma_allow_lds(lds));
  }
  int64_t nf = 0, nr = 0, npp = 0;
  for (int t : F->m2l_tab) (t < 0 ? nf : nr)++;
  for (size_t t = 0; t < F->near_tgt.size(); ++t)
    for (int e = F->near_ptr[t]; e < F->near_ptr[t + 1]; ++e)
      npp += (int64_t)F->boxes[F->near_tgt[t]].npt * F->boxes[F->near_src[e]].npt;
  F->stats[0] = F->n_boxes;
  F->stats[1] = nf;
  F->stats[2] = nr;
  F->stats[3] = nfree;
  F->stats[4] = nreac;
  F->stats[5] = nrn;
  F->stats[6] = F->lf;
  F->stats[7] = F->lr;
  F->stats[8] = (int64_t)F->near_src.size();
  F->stats[9] = npp;
  return LM_OK;
}

// Device bytes the FMM workspace needs per right-hand side of a launch.
int64_t fmm_ws_per_rhs(const FmmPlan* F) {
  if (!F) return 0;
  return (int64_t)F->P * 16 * (2 * (int64_t)F->n_boxes + F->item_ptr[3]) + (int64_t)F->P * 8 * (F->mf_item.size() / 3);
}

// Per-launch workspace of r right-hand sides: byte sizes of the buffers
// (expansions, P2M partial sums, level-0 transforms, per-entry M2L results,
// the complex64 transpose of x).
void fmm_ws_sizes(const FmmPlan* F, int r, size_t sz[FMM_WS_N]) {
  r = std::min(std::max(r, 1), LM_RCHUNK);
  const size_t P = F->P;
  sz[FMM_WS_ME] = sz[FMM_WS_LE] = (size_t)F->n_boxes * P * r * sizeof(double2);
  sz[FMM_WS_PART] = (size_t)std::max(F->item_ptr[3], 1) * P * r * sizeof(double2);
  sz[FMM_WS_TOP_MH] = sz[FMM_WS_TOP_LH] =
      F->top_on ? (size_t)F->top_rows * F->top_L * P * r * sizeof(double2) : 0;
  sz[FMM_WS_M2L_OUT] = std::max<size_t>(F->m2l_src.size(), 1) * P * sizeof(double2);
  sz[FMM_WS_OM_SLOT] = r > 1 ? std::max<size_t>(F->m2l_src.size(), 1) * P * std::min(r, OM_RMAX) * sizeof(float2) : 0;
  sz[FMM_WS_MF_PART] = r > 1 ? std::max<size_t>(F->mf_item.size() / 3, 1) * P * r * sizeof(float2) : 0;
  sz[FMM_WS_XT] = r > 1 ? (size_t)std::max<int64_t>(F->n_el, 1) * r * sizeof(float2) : 0;
}

// Bytes of one contiguous workspace of r right-hand sides (every buffer
// starting at a 256-byte boundary).
size_t fmm_ws_bytes(const FmmPlan* F, int r) {
  size_t sz[FMM_WS_N], t = 0;
  fmm_ws_sizes(F, r, sz);
  for (int i = 0; i < FMM_WS_N; ++i) t += (sz[i] + 255) & ~(size_t)255;
  return t;
}

// The workspace carved from one device region of at least fmm_ws_bytes.
FmmWs fmm_ws_carve(const FmmPlan* F, int r, void* base) {
  size_t sz[FMM_WS_N], off = 0;
  fmm_ws_sizes(F, r, sz);
  FmmWs w;
  for (int i = 0; i < FMM_WS_N; ++i) {
    w.p[i] = sz[i] ? (char*)base + off : nullptr;
    off += (sz[i] + 255) & ~(size_t)255;
  }
  return w;
}

// Expansion buffers for r right-hand sides per launch (grown on demand).
lm_status fmm_reserve(FmmPlan* F, int r) {
  r = std::min(std::max(r, 1), LM_RCHUNK);
  if (r <= F->r_cap) return LM_OK;
  size_t sz[FMM_WS_N];
  fmm_ws_sizes(F, r, sz);
  DevBuf* bufs[FMM_WS_N] = {&F->d_me, &F->d_le, &F->d_p2m_part, &F->d_top_mh, &F->d_top_lh,
                            &F->d_m2l_out, &F->d_om_slot, &F->d_mf_part, &F->d_xt};
  for (int i = 0; i < FMM_WS_N; ++i)
    if (sz[i] > bufs[i]->bytes) LM_TRY(bufs[i]->alloc(sz[i]));
  F->r_cap = r;
  return LM_OK;
}

// The plan's own workspace (after fmm_reserve).
static FmmWs fmm_ws_own(FmmPlan* F) {
  FmmWs w;
  DevBuf* bufs[FMM_WS_N] = {&F->d_me, &F->d_le, &F->d_p2m_part, &F->d_top_mh, &F->d_top_lh,
                            &F->d_m2l_out, &F->d_om_slot, &F->d_mf_part, &F->d_xt};
  for (int i = 0; i < FMM_WS_N; ++i) w.p[i] = bufs[i]->p;
  return w;
}

namespace {

// One matvec of R <= LM_RCHUNK right-hand sides in storage type RT.  When
// ev != nullptr, ev[2 i], ev[2 i + 1] bracket stage i on stream s (0 P2M,
// 1 M2M, 2 M2L lists, 3 L2L, 4 L2P, 5 near field (side stream), 6 M2L
// partial sums, 7 level-0 convolution).
template <typename RT>
lm_status matvec_chunk(lm_geom_s* g, int R, const typename C2T<RT>::T* x, typename C2T<RT>::T* y, const FmmWs& ws,
                       hipStream_t s, hipEvent_t* ev) {
  typedef typename C2T<RT>::T V;
  FmmPlan* F = g->fmm;
  const int N = (int)g->N, p = F->p, P = F->P, PR = P * R, nlev = F->nlev;
  const BoxDev* boxes = F->d_boxes.as<BoxDev>();
  const int* tl = F->d_tree_layer.as<int>();
  const double* sig = F->d_sig.as<double>();
  const V* ops = sizeof(RT) == 8 ? (const V*)F->d_ops64.p : (const V*)F->d_ops32.p;
  const V* nmv = sizeof(RT) == 8 ? (const V*)F->d_nm_val.p : (const V*)F->d_nm_val32.p;
  const size_t PP = (size_t)P * P;
  V* me = (V*)ws.p[FMM_WS_ME];
  V* le = (V*)ws.p[FMM_WS_LE];
  const int blk = std::min(256, 64 * (int)div_up(PR, 64));
  const size_t lds_pr = (size_t)PR * sizeof(V);
#define LM_STAGE(i, open) \
  if (ev) LM_TRY_HIP(hipEventRecord(ev[2 * (i) + ((open) ? 0 : 1)], s))
  LM_STAGE(0, 1);
  // P2M on every leaf (leaves of all trees; internal boxes come from M2M)
  const int n_items = F->item_ptr[3];
  V* part = (V*)ws.p[FMM_WS_PART];
  const bool pt_mfma = sizeof(RT) == 4 && R > 1;  // FP32 multi-RHS: point steps on matrix cores
  if (pt_mfma)  // complex64 transpose of x, shared by the P2M and the near field
    hipLaunchKernelGGL(k_to_nr<float2>, dim3(div_up(N, 32), div_up(R, 32)), dim3(32, 8), 0, s, N, R,
                       (const float2*)x, (float2*)ws.p[FMM_WS_XT]);
  if (n_items) {
    if (pt_mfma)
      hipLaunchKernelGGL(k_p2m_mfma, dim3(n_items), dim3(64 * PA_NW), 0, s, p, R, F->d_pt_item.as<int>(),
                         F->d_p2m_dst.as<int>(), F->d_pt_elem.as<int>(), F->d_p2m_Z32.as<float2>(),
                         (float2*)ws.p[FMM_WS_XT], (float2*)part, (float2*)me);
    else if (R == 1)
      hipLaunchKernelGGL((k_p2m<RT, 64>), dim3(n_items), dim3(blk), (size_t)64 * R * sizeof(V), s, p, R, nlev,
                         F->d_pt_item.as<int>(), boxes, tl, sig, F->d_pt_elem.as<int>(), F->d_pt_xh.as<double2>(),
                         g->d_w.as<double>(), x, N, part);
    else
      hipLaunchKernelGGL((k_p2m<RT, 32>), dim3(n_items), dim3(blk), (size_t)32 * R * sizeof(V), s, p, R, nlev,
                         F->d_pt_item.as<int>(), boxes, tl, sig, F->d_pt_elem.as<int>(), F->d_pt_xh.as<double2>(),
                         g->d_w.as<double>(), x, N, part);
    if (!pt_mfma)
      hipLaunchKernelGGL(k_p2m_reduce<RT>, dim3(F->p2m_leaf.size()), dim3(blk), 0, s, PR, F->d_p2m_leaf.as<int>(),
                         F->d_p2m_ptr.as<int>(), (const int*)nullptr, part, me);
    else if (!F->p2m_msel.empty())  // leaves of one item were written directly
      hipLaunchKernelGGL(k_p2m_reduce<RT>, dim3(F->p2m_msel.size()), dim3(blk), 0, s, PR, F->d_p2m_leaf.as<int>(),
                         F->d_p2m_ptr.as<int>(), F->d_p2m_msel.as<int>(), part, me);
  }
  // The near field and self terms only need x: they run on the plan's side
  // stream, after the P2M (which heads the critical path) and overlapped with
  // M2M .. L2L, and write y first; every L2P launch then accumulates after
  // the join.
  LM_TRY_HIP(hipEventRecord(F->ev_fork, s));
  LM_TRY_HIP(hipStreamWaitEvent(F->s_near, F->ev_fork, 0));
  {
    hipStream_t sn = F->s_near;
    if (ev) LM_TRY_HIP(hipEventRecord(ev[10], sn));
    if (pt_mfma) {
      // FP32, several right-hand sides: free-space near field + self terms as
      // leaf blocks on matrix cores (every element is a row of one leaf
      // block), then the few reaction near pairs
      if (F->nb_item.empty())
        LM_TRY_HIP(hipMemsetAsync(y, 0, (size_t)R * N * sizeof(float2), sn));
      else
        hipLaunchKernelGGL((k_block_mfma<float2, false>), dim3(F->nb_item.size() / 2), dim3(64 * PA_NW), 0, sn, N,
                           R, F->d_nb_item.as<int>(), F->d_nb_jptr.as<int>(), F->d_nb_jidx.as<int>(),
                           F->d_nb_rows.as<int>(), F->d_nb_zoff.as<int64_t>(), F->d_nb_Z32.as<float2>(),
                           (float2*)ws.p[FMM_WS_XT], (float2*)y);
      if (!F->rn_src.empty())
        hipLaunchKernelGGL((k_near_csr<float, 8>), dim3(div_up(F->rn_rows.size(), 4)), dim3(256), 0, sn, N,
                           (int)F->rn_rows.size(), F->d_rn_rows.as<int>(), R, 1, F->d_rn_ptr.as<int>(),
                           F->d_rn_src.as<int>(), F->d_rn_val32.as<float2>(), (const float2*)x, (float2*)y);
    } else if (R >= 8) {  // CSR with the self term in every row
      hipLaunchKernelGGL((k_near_csr<RT, 8>), dim3(div_up(N, 4)), dim3(256), 0, sn, N, N, (const int*)nullptr, R, 0,
                         F->d_nm_ptr.as<int>(), F->d_nm_src.as<int>(), nmv, x, y);
    } else {
      hipLaunchKernelGGL((k_near_csr<RT, 4>), dim3(div_up(N, 4)), dim3(256), 0, sn, N, N, (const int*)nullptr, R, 0,
                         F->d_nm_ptr.as<int>(), F->d_nm_src.as<int>(), nmv, x, y);
    }
    if (!F->sc_src.empty()) {  // spectral rule: same-scatterer corrections, accumulated
      const V* scv = sizeof(RT) == 8 ? (const V*)F->d_sc_val.p : (const V*)F->d_sc_val32.p;
      if (R >= 8)
        hipLaunchKernelGGL((k_near_csr<RT, 8>), dim3(div_up(N, 4)), dim3(256), 0, sn, N, N, (const int*)nullptr, R, 1,
                           F->d_sc_ptr.as<int>(), F->d_sc_src.as<int>(), scv, x, y);
      else
        hipLaunchKernelGGL((k_near_csr<RT, 4>), dim3(div_up(N, 4)), dim3(256), 0, sn, N, N, (const int*)nullptr, R, 1,
                           F->d_sc_ptr.as<int>(), F->d_sc_src.as<int>(), scv, x, y);
    }
    if (ev) LM_TRY_HIP(hipEventRecord(ev[11], sn));
    LM_TRY_HIP(hipEventRecord(F->ev_join, sn));
  }
  LM_STAGE(0, 0);
  LM_STAGE(1, 1);
  // M2M, finest parents first (FP32 with several right-hand sides: matrix
  // cores, one item per parent holding its children)
  const bool tr_mfma = sizeof(RT) == 4 && R > 1;
  for (int l = nlev - 2; l >= 0; --l) {
    const int n = F->parents_ptr[l + 1] - F->parents_ptr[l];
    if (!n) continue;
    if (tr_mfma) {
      const int i0 = F->parents_ptr[l];
      m2l_mfma_launch<MF_TREE>(n, p, R, F->d_tr_item.as<int>() + 3 * i0, F->d_tr_src.as<int>(),
                               F->d_tr_op.as<int>(), (const float2*)ops, (const float2*)me, (float2*)me,
                               F->d_parents.as<int>() + i0, 0, s);
    } else {
      hipLaunchKernelGGL(k_m2m<RT>, dim3(n), dim3(blk), lds_pr, s, p, R, nlev,
                         F->d_parents.as<int>() + F->parents_ptr[l], boxes, F->d_children.as<int>(), tl, ops, me);
    }
  }
  LM_STAGE(1, 0);
  // M2L (every level at once); the M2L and level-0 launches overwrite their
  // targets, boxes without either start from zero
  if (!F->le_zero.empty())
    hipLaunchKernelGGL(k_zero_boxes<V>, dim3(F->le_zero.size()), dim3(256), 0, s, PR, F->d_le_zero.as<int>(), le);
  // level 0 as a convolution along x (stage 7): transform the level-0
  // expansions of every row, one product per row pair and frequency,
  // transform back into the level-0 local expansions
  LM_STAGE(7, 1);
  if (F->top_on) {
    const int L = F->top_L, nx = F->top_nx, nrow = F->top_rows;
    int lgL = 0;
    while ((1 << lgL) < L) ++lgL;
    const int lgc = top_lgc(lgL, sizeof(V));
    const dim3 tg((unsigned)div_up(PR, 1 << lgc), (unsigned)nrow);
    const size_t tlds = ((size_t)L << lgc) * sizeof(V);
    V* mh = (V*)ws.p[FMM_WS_TOP_MH];
    V* lh = (V*)ws.p[FMM_WS_TOP_LH];
    const V* tw = sizeof(RT) == 8 ? (const V*)F->d_top_tw64.p : (const V*)F->d_top_tw32.p;
    const V* tops = sizeof(RT) == 8 ? (const V*)F->d_top_T64.p : (const V*)F->d_top_T32.p;
    hipLaunchKernelGGL(k_top_fwd<V>, tg, dim3(256), tlds, s, lgL, lgc, nx, PR, F->d_top_grid.as<int>(),
                       (const V*)me, tw, mh);
    if (sizeof(RT) == 4 && R > 1)
      m2l_mfma_launch<MF_TOP>(nrow * L, p, R, F->d_top_item.as<int>(), F->d_top_src.as<int>(),
                              F->d_top_op.as<int>(), (const float2*)tops, (const float2*)mh, (float2*)lh,
                              (const int*)nullptr, 0, s);
    else
      hipLaunchKernelGGL(k_m2l_target<RT>, dim3(nrow * L), dim3(blk), lds_pr, s, p, R, F->d_top_id.as<int>(),
                         F->d_top_ptr.as<int>(), F->d_top_src.as<int>(), F->d_top_op.as<int>(), tops,
                         (const V*)mh, lh);
    hipLaunchKernelGGL(k_top_inv<V>, tg, dim3(256), tlds, s, lgL, lgc, nx, PR, F->d_top_grid.as<int>(),
                       (const V*)lh, tw, le);
  }
  LM_STAGE(7, 0);
  LM_STAGE(2, 1);
  if (!F->m2l_tgt.empty()) {
    const V* mops = ops + (size_t)F->op_m2l * PP;
    if (R == 1) {
      V* out = (V*)ws.p[FMM_WS_M2L_OUT];
      hipLaunchKernelGGL(k_m2l_apply<RT>, dim3(F->tm_item.size() / 3), dim3(64), 0, s, p, F->d_tm_item.as<int>(),
                         F->d_tm_slot.as<int>(), F->d_tm_src.as<int>(), mops, me, out);
      LM_STAGE(2, 0);
      LM_STAGE(6, 1);
      hipLaunchKernelGGL(k_m2l_reduce<RT>, dim3(F->m2l_tgt.size()), dim3(256), 0, s, p, F->d_m2l_tgt.as<int>(),
                         F->d_m2l_ptr.as<int>(), out, le);
      LM_STAGE(6, 0);
    } else if (sizeof(RT) == 4 && R <= OM_RMAX) {
      // few right-hand sides: operator-major, one operator staged per item
      float2* slots = (float2*)ws.p[FMM_WS_OM_SLOT];
      const size_t lds = mf_lds_bytes(P, (64 / R) * R);
      if ((P + 15) / 16 > MF_TR)
        hipLaunchKernelGGL(k_m2l_om<2>, dim3(F->tm_item.size() / 3), dim3(512), lds, s, p, R,
                           F->d_tm_item.as<int>(), F->d_tm_slot.as<int>(), F->d_tm_src.as<int>(),
                           (const float2*)mops, (const float2*)me, slots);
      else
        hipLaunchKernelGGL(k_m2l_om<1>, dim3(F->tm_item.size() / 3), dim3(256), lds, s, p, R,
                           F->d_tm_item.as<int>(), F->d_tm_slot.as<int>(), F->d_tm_src.as<int>(),
                           (const float2*)mops, (const float2*)me, slots);
      LM_STAGE(2, 0);
      LM_STAGE(6, 1);
      hipLaunchKernelGGL(k_p2m_reduce<float>, dim3(F->m2l_tgt.size()), dim3(256), 0, s, PR, F->d_m2l_tgt.as<int>(),
                         F->d_m2l_ptr.as<int>(), (const int*)nullptr, slots, (float2*)le);
      LM_STAGE(6, 0);
    } else if (sizeof(RT) == 4) {
      float2* mpart = (float2*)ws.p[FMM_WS_MF_PART];
      m2l_mfma_launch<MF_LIST>((int)(F->mf_item.size() / 3), p, R, F->d_mf_item.as<int>(), F->d_m2l_src.as<int>(),
                               F->d_m2l_op.as<int>(), (const float2*)mops, (const float2*)me, mpart,
                               F->d_mf_slot.as<int>(), 0, s);
      LM_STAGE(2, 0);
      LM_STAGE(6, 1);
      hipLaunchKernelGGL(k_p2m_reduce<float>, dim3(F->m2l_tgt.size()), dim3(256), 0, s, PR, F->d_m2l_tgt.as<int>(),
                         F->d_mf_ptr.as<int>(), (const int*)nullptr, mpart, (float2*)le);
      LM_STAGE(6, 0);
    } else {
      hipLaunchKernelGGL(k_m2l_target<RT>, dim3(F->m2l_tgt.size()), dim3(blk), lds_pr, s, p, R,
                         F->d_m2l_tgt.as<int>(), F->d_m2l_ptr.as<int>(), F->d_m2l_src.as<int>(),
                         F->d_m2l_op.as<int>(), mops, me, le);
      LM_STAGE(2, 0);
      LM_STAGE(6, 1);
      LM_STAGE(6, 0);
    }
  } else {
    LM_STAGE(2, 0);
    LM_STAGE(6, 1);
    LM_STAGE(6, 0);
  }
  LM_STAGE(3, 1);
  // L2L, coarse to fine (matrix cores as for M2M: one item per child box)
  for (int l = 1; l < nlev; ++l) {
    const int n = F->level_ptr[l + 1] - F->level_ptr[l];
    if (!n) continue;
    if (tr_mfma) {
      const int i0 = F->l2l_item0 + F->level_ptr[l] - F->level_ptr[1];
      m2l_mfma_launch<MF_TREE>(n, p, R, F->d_tr_item.as<int>() + 3 * i0, F->d_tr_src.as<int>(),
                               F->d_tr_op.as<int>(), (const float2*)ops, (const float2*)le, (float2*)le,
                               F->d_box_id.as<int>() + F->level_ptr[l], 1, s);
    } else {
      hipLaunchKernelGGL(k_l2l<RT>, dim3(n), dim3(blk), lds_pr, s, p, R, nlev, F->level_ptr[l], boxes, tl,
                         ops + (size_t)F->n_tree_ops * PP, le);
    }
  }
  LM_STAGE(3, 0);
  LM_TRY_HIP(hipStreamWaitEvent(s, F->ev_join, 0));  // y holds the near field
  LM_STAGE(4, 1);
  // L2P: every tree class accumulates (each element once per launch)
  for (int c = 0; c < 3; ++c) {
    const int i0 = F->item_ptr[c], ni = F->item_ptr[c + 1] - i0;
    if (!ni) continue;
    const int* it = F->d_pt_item.as<int>() + 3 * i0;
    if (pt_mfma)
      hipLaunchKernelGGL(k_l2p_mfma, dim3(ni), dim3(64 * PA_NW), 0, s, p, R, N, 1, it,
                         F->d_pt_elem.as<int>(), F->d_l2p_Z32.as<float2>(), (const float2*)le, (float2*)y);
    else if (F->bc != LM_BC_DIRICHLET)  // stored n . grad + i beta rows
      hipLaunchKernelGGL((k_l2p_rows<RT>), dim3(ni), dim3(256), 0, s, p, R, N, it, F->d_pt_elem.as<int>(),
                         sizeof(RT) == 8 ? (const V*)F->d_l2p_Z64.p : (const V*)F->d_l2p_Z32.p, le, y);
    else if (R == 1)
      hipLaunchKernelGGL((k_l2p<RT, 64>), dim3(ni), dim3(blk), lds_pr, s, p, R, nlev, 1, it, boxes, tl,
                         sig, F->d_pt_elem.as<int>(), F->d_pt_xh.as<double2>(), le, N, y);
    else
      hipLaunchKernelGGL((k_l2p<RT, 32>), dim3(ni), dim3(blk), lds_pr, s, p, R, nlev, 1, it, boxes, tl,
                         sig, F->d_pt_elem.as<int>(), F->d_pt_xh.as<double2>(), le, N, y);
  }
  LM_STAGE(4, 0);
#undef LM_STAGE
  LM_TRY_HIP(hipGetLastError());
  return LM_OK;
}

}  // namespace

// Matvec in chunks of at most rc right-hand sides on the workspace ws
// (holding rc right-hand sides).
static lm_status matvec_chunks(lm_geom_s* g, int precision, int n_rhs, int rc, const void* xv, void* yv,
                               const FmmWs& ws, hipStream_t s, hipEvent_t* ev) {
  const int64_t N = g->N;
  for (int r0 = 0; r0 < n_rhs; r0 += rc) {
    const int R = std::min(rc, n_rhs - r0);
    hipEvent_t* e = r0 == 0 ? ev : nullptr;
    if (precision == LM_FP64) {
      LM_TRY(matvec_chunk<double>(g, R, (const double2*)xv + r0 * N, (double2*)yv + r0 * N, ws, s, e));
    } else {
      LM_TRY(matvec_chunk<float>(g, R, (const float2*)xv + r0 * N, (float2*)yv + r0 * N, ws, s, e));
    }
  }
  return LM_OK;
}

lm_status fmm_matvec_timed(lm_geom_s* g, int precision, int n_rhs, const void* xv, void* yv, hipStream_t s,
                           hipEvent_t* ev) {
  FmmPlan* F = g->fmm;
  LM_CHECK(F, LM_EINTERNAL, "no FMM plan");
  LM_TRY(fmm_reserve(F, n_rhs));
  return matvec_chunks(g, precision, n_rhs, LM_RCHUNK, xv, yv, fmm_ws_own(F), s, ev);
}

// Matvec whose workspace is the caller's region [base, base + cap): no
// device allocation.  Chunks of as many right-hand sides as the region holds
// (at most LM_RCHUNK); LM_EINVAL when it cannot hold one.
lm_status fmm_matvec_in(lm_geom_s* g, int precision, int n_rhs, const void* xv, void* yv, void* base, size_t cap,
                        hipStream_t s) {
  FmmPlan* F = g->fmm;
  LM_CHECK(F, LM_EINTERNAL, "no FMM plan");
  int rc = std::min(n_rhs, LM_RCHUNK);
  while (rc > 1 && fmm_ws_bytes(F, rc) > cap) --rc;
  const size_t need = fmm_ws_bytes(F, rc);
  LM_CHECK(need <= cap, LM_EINVAL,
           "the matvec workspace of this geometry (%zu bytes for one right-hand side) exceeds the %zu-byte static "
           "scratch; use lm_matvec",
           need, cap);
  return matvec_chunks(g, precision, n_rhs, rc, xv, yv, fmm_ws_carve(F, rc, base), s, nullptr);
}

lm_status fmm_matvec(lm_geom_s* g, int precision, int n_rhs, const void* xv, void* yv, hipStream_t s) {
  return fmm_matvec_timed(g, precision, n_rhs, xv, yv, s, nullptr);
}

// Average per-stage durations (ms) over reps matvecs, measured with HIP events
// on the stream the kernels run on; out[0..6] = stages 0..6, out[7] = whole
// matvec, out[8] = stage 7 (level-0 convolution).
lm_status fmm_stage_times(lm_geom_s* g, int precision, int n_rhs, const void* x, void* y, int reps, hipStream_t s,
                          double* out) {
  hipEvent_t ev[18];
  for (int i = 0; i < 18; ++i) LM_TRY_HIP(hipEventCreate(&ev[i]));
  for (int i = 0; i < 9; ++i) out[i] = 0.0;
  lm_status st = LM_OK;
  for (int r = 0; r < reps && st == LM_OK; ++r) {
    LM_TRY_HIP(hipEventRecord(ev[16], s));
    st = fmm_matvec_timed(g, precision, n_rhs, x, y, s, ev);
    LM_TRY_HIP(hipEventRecord(ev[17], s));
    LM_TRY_HIP(hipEventSynchronize(ev[17]));
    for (int i = 0; i < 8; ++i) {
      float ms = 0;
      LM_TRY_HIP(hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]));
      out[i == 7 ? 8 : i] += ms / reps;
    }
    float ms = 0;
    LM_TRY_HIP(hipEventElapsedTime(&ms, ev[16], ev[17]));
    out[7] += ms / reps;
  }
  for (int i = 0; i < 18; ++i) (void)hipEventDestroy(ev[i]);
  return st;
}
