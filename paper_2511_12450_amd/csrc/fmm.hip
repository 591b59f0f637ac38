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

#include "fmm_math.hpp"
#include "lm_internal.hpp"
#include "m2l_table.hpp"

#include "fmm_plan.hpp"

namespace {
constexpr int WG = 64;
constexpr int MAXPP = 2 * MAXP + 1;
inline int64_t bkey(int i, int j) { return ((int64_t)i << 32) | (uint32_t)j; }
}  // namespace

void fmm_free(FmmPlan* f) { delete f; }
int64_t fmm_bytes(const FmmPlan* f) { return f ? f->bytes() : 0; }
void fmm_stats(const FmmPlan* f, int64_t* out) {
  for (int i = 0; i < 10; ++i) out[i] = f ? f->stats[i] : 0;
}

// =========================================================== setup kernels ==

// Hankel values G_j(D), j = -2p..2p, for each free-space M2L class.
__global__ void k_free_tables(int n, int p, const double* __restrict__ geo, double2* __restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int J = 2 * p;
  zd G[2 * (2 * MAXP) + 1];
  zd hb[2 * MAXP + 1];
  fm::g_seq(geo[3 * t], geo[3 * t + 1], geo[3 * t + 2], J, G, hb);
  for (int j = 0; j <= 2 * J; ++j) out[(int64_t)t * (2 * J + 1) + j] = make_double2(G[j].re, G[j].im);
}

// Reaction M2L operator per class: one workgroup per table, nodes in chunks.
constexpr int TAB_CHUNK = 16;
__global__ void __launch_bounds__(256) k_reac_tables(MediumDev m, int p, const int* __restrict__ meta,
                                                     const double* __restrict__ geo, double2* __restrict__ out) {
  const int t = blockIdx.x;
  const int P = 2 * p + 1;
  const int lt = meta[3 * t], ls = meta[3 * t + 1], comp = meta[3 * t + 2];
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
    out[(int64_t)t * P * P + idx] = make_double2(acc[e].re, acc[e].im);
  }
}

// ========================================================== matvec kernels ==

// P2M: a_n = sum_s q_s J_n(k rho_s) e^{-i n theta_s}, q_s = |Gamma_s| x_s.
__global__ void __launch_bounds__(WG) k_p2m(int p, const int* __restrict__ leaves, const BoxDev* __restrict__ boxes,
                                            const int* __restrict__ pt_elem, const double2* __restrict__ pt_xh,
                                            const double* __restrict__ w, const double2* __restrict__ x,
                                            double2* __restrict__ me) {
  const int b = leaves[blockIdx.x];
  const BoxDev B = boxes[b];
  const int P = 2 * p + 1;
  __shared__ double Jq_re[WG][MAXP + 1];
  __shared__ double Jq_im[WG][MAXP + 1];
  __shared__ double th[WG];
  const int n = (int)threadIdx.x - p;
  zd acc(0.0, 0.0);
  for (int s0 = 0; s0 < B.npt; s0 += WG) {
    const int s = s0 + threadIdx.x;
    if (s < B.npt) {
      const int pi = B.pt0 + s;
      const double2 xh = pt_xh[pi];
      const double dx = xh.x - B.cx, dh = xh.y - B.ch;
      const int e = pt_elem[pi];
      const double2 xv = x[e];
      const double we = w[e];
      double J[MAXP + 1];
      fm::bessel_j_seq(B.k * hypot(dx, dh), p, J);
      for (int j = 0; j <= p; ++j) {
        Jq_re[threadIdx.x][j] = J[j] * we * xv.x;
        Jq_im[threadIdx.x][j] = J[j] * we * xv.y;
      }
      th[threadIdx.x] = atan2(dh, dx);
    }
    __syncthreads();
    if (threadIdx.x < (unsigned)P) {
      const int cnt = min(WG, B.npt - s0);
      const int an = n < 0 ? -n : n;
      const double sg = (n < 0 && (an & 1)) ? -1.0 : 1.0;
      for (int j = 0; j < cnt; ++j) {
        double sn, cs;
        sincos(-n * th[j], &sn, &cs);
        const double re = Jq_re[j][an] * sg, im = Jq_im[j][an] * sg;
        acc.re += re * cs - im * sn;
        acc.im += re * sn + im * cs;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < (unsigned)P) me[(int64_t)b * P + threadIdx.x] = make_double2(acc.re, acc.im);
}

// Operator F_j(d) for the box's layer/level/position: ftab[((layer*nlev + level)*4 + pos)*(4p+1) + j + 2p]
__device__ __forceinline__ const double2* ftab_row(const double2* ftab, int nlev, int p, int layer, int level, int pos) {
  return ftab + ((int64_t)((layer * nlev + level) * 4 + pos)) * (4 * p + 1) + 2 * p;
}

// M2M: a^C_n = sum_children sum_m F_{m-n}(C - c) a^c_m = sum (-1)^{m-n} F_{m-n}(c - C) a_m.
__global__ void __launch_bounds__(WG) k_m2m(int p, int nlev, const int* __restrict__ parents,
                                            const BoxDev* __restrict__ boxes, const int* __restrict__ children,
                                            const int* __restrict__ tree_layer, const double2* __restrict__ ftab,
                                            double2* __restrict__ me) {
  const int b = parents[blockIdx.x];
  const BoxDev B = boxes[b];
  const int P = 2 * p + 1;
  __shared__ double2 a[MAXPP];
  __shared__ double2 f[4 * MAXP + 1];
  const int n = (int)threadIdx.x - p;
  zd acc(0.0, 0.0);
  for (int c = 0; c < B.nchild; ++c) {
    const int cb = children[B.child0 + c];
    const BoxDev C = boxes[cb];
    if (threadIdx.x < (unsigned)P) a[threadIdx.x] = me[(int64_t)cb * P + threadIdx.x];
    const double2* fr = ftab_row(ftab, nlev, p, tree_layer[C.tree], C.level, C.pos);
    for (int j = threadIdx.x; j <= 4 * p; j += WG) f[j] = fr[j - 2 * p];
    __syncthreads();
    if (threadIdx.x < (unsigned)P) {
      for (int mm = -p; mm <= p; ++mm) {
        const int d = mm - n;
        const double2 fv = f[d + 2 * p];
        const double sg = (d & 1) ? -1.0 : 1.0;
        const double2 av = a[mm + p];
        acc.re += sg * (fv.x * av.x - fv.y * av.y);
        acc.im += sg * (fv.x * av.y + fv.y * av.x);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < (unsigned)P) me[(int64_t)b * P + threadIdx.x] = make_double2(acc.re, acc.im);
}

// L2L: b^c_n += sum_m F_{m-n}(c - C) b^C_m, for every box of one level with a parent.
__global__ void __launch_bounds__(WG) k_l2l(int p, int nlev, int first, const BoxDev* __restrict__ boxes,
                                            const int* __restrict__ tree_layer, const double2* __restrict__ ftab,
                                            double2* __restrict__ le) {
  const int b = first + blockIdx.x;
  const BoxDev B = boxes[b];
  const int P = 2 * p + 1;
  __shared__ double2 a[MAXPP];
  __shared__ double2 f[4 * MAXP + 1];
  if (threadIdx.x < (unsigned)P) a[threadIdx.x] = le[(int64_t)B.parent * P + threadIdx.x];
  const double2* fr = ftab_row(ftab, nlev, p, tree_layer[B.tree], B.level, B.pos);
  for (int j = threadIdx.x; j <= 4 * p; j += WG) f[j] = fr[j - 2 * p];
  __syncthreads();
  if (threadIdx.x < (unsigned)P) {
    const int n = (int)threadIdx.x - p;
    const double2 old = le[(int64_t)b * P + threadIdx.x];
    zd acc(old.x, old.y);
    for (int mm = -p; mm <= p; ++mm) {
      const double2 fv = f[mm - n + 2 * p];
      const double2 av = a[mm + p];
      acc.re += fv.x * av.x - fv.y * av.y;
      acc.im += fv.x * av.y + fv.y * av.x;
    }
    le[(int64_t)b * P + threadIdx.x] = make_double2(acc.re, acc.im);
  }
}

// L2P: y_e (=/+=) sum_m b_m J_m(k rho) e^{i m theta} for the points of each leaf.
__global__ void __launch_bounds__(WG) k_l2p(int p, int accumulate, const int* __restrict__ leaves,
                                            const BoxDev* __restrict__ boxes, const int* __restrict__ pt_elem,
                                            const double2* __restrict__ pt_xh, const double2* __restrict__ le,
                                            double2* __restrict__ y) {
  const int b = leaves[blockIdx.x];
  const BoxDev B = boxes[b];
  const int P = 2 * p + 1;
  __shared__ double2 L[MAXPP];
  if (threadIdx.x < (unsigned)P) L[threadIdx.x] = le[(int64_t)b * P + threadIdx.x];
  __syncthreads();
  for (int s = threadIdx.x; s < B.npt; s += WG) {
    const int pi = B.pt0 + s;
    const double2 xh = pt_xh[pi];
    const double dx = xh.x - B.cx, dh = xh.y - B.ch;
    double J[MAXP + 1];
    fm::bessel_j_seq(B.k * hypot(dx, dh), p, J);
    const zd e1 = fm::cis(atan2(dh, dx));
    double2 l0 = L[p];
    zd acc(l0.x * J[0], l0.y * J[0]);
    zd ep(1.0, 0.0);
    for (int j = 1; j <= p; ++j) {
      ep = ep * e1;
      const double sg = (j & 1) ? -1.0 : 1.0;
      const double2 lp = L[p + j], lm = L[p - j];
      const zd cp = zd(lp.x, lp.y) * ep, cm = zd(lm.x, lm.y) * conj(ep);
      acc += (cp + cm * sg) * J[j];
    }
    const int e = pt_elem[pi];
    if (accumulate) {
      const double2 o = y[e];
      y[e] = make_double2(o.x + acc.re, o.y + acc.im);
    } else {
      y[e] = make_double2(acc.re, acc.im);
    }
  }
}

// Near-field matrix values: kind 0 free-space pair, 1 reaction pair (mask),
// 2 self term.
__global__ void k_near_values(MediumDev m, int64_t n, const int* __restrict__ tgt, const int* __restrict__ src,
                              const unsigned* __restrict__ kind, const double* __restrict__ cx,
                              const double* __restrict__ cy, const double* __restrict__ w,
                              const int* __restrict__ lay, const double2* __restrict__ self,
                              double2* __restrict__ val) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int i = tgt[t], e = src[t];
  const unsigned kd = kind[t];
  zd v(0.0, 0.0);
  if (kd == 0u) {
    const double kr = m.k[lay[i]] * hypot(cx[i] - cx[e], cy[i] - cy[e]);
    v = zd(-0.25 * y0(kr), 0.25 * j0(kr)) * w[e];
  } else if (kd == 0xFFFFFFFFu) {
    const double2 sv = self[i];
    v = zd(sv.x, sv.y);
  } else {
    v = lmq::reaction_direct(m, lay[i], lay[e], fabs(cx[i] - cx[e]), cy[i], cy[e], kd) * w[e];
  }
  val[t] = make_double2(v.re, v.im);
}

// y_i += sum_j Knear_ij x_j: one wavefront per row.
__global__ void __launch_bounds__(256) k_near_csr(int N, const int* __restrict__ ptr, const int* __restrict__ src,
                                                  const double2* __restrict__ val, const double2* __restrict__ x,
                                                  double2* __restrict__ y) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= N) return;
  double re = 0.0, im = 0.0;
  for (int e = ptr[row] + lane; e < ptr[row + 1]; e += 64) {
    const double2 v = val[e], xv = x[src[e]];
    re += v.x * xv.x - v.y * xv.y;
    im += v.x * xv.y + v.y * xv.x;
  }
  for (int off = 32; off > 0; off >>= 1) {
    re += __shfl_down(re, off, 64);
    im += __shfl_down(im, off, 64);
  }
  if (lane == 0) {
    const double2 o = y[row];
    y[row] = make_double2(o.x + re, o.y + im);
  }
}

// M2L grouped by operator: one workgroup per operator (reaction table or
// free-space class) keeps it in LDS and applies it to all its entries,
// four source expansions at a time; results go to the entry's slot.
constexpr int M2L_BATCH = 4;
__global__ void __launch_bounds__(64) k_m2l_apply(int p, int nreac, const int* __restrict__ ptr,
                                                  const int* __restrict__ slot, const int* __restrict__ src,
                                                  const double2* __restrict__ free_tab,
                                                  const double2* __restrict__ reac_tab,
                                                  const double2* __restrict__ me, double2* __restrict__ out) {
  extern __shared__ double2 lds[];
  const int t = blockIdx.x;
  const int P = 2 * p + 1;
  const bool isfree = t >= nreac;
  double2* T = lds;                                    // P*P (reaction) or 4p+1 (free)
  double2* A = lds + (isfree ? (4 * p + 1) : P * P);   // [M2L_BATCH][P]
  if (isfree) {
    const double2* g = free_tab + (int64_t)(t - nreac) * (4 * p + 1);
    for (int j = threadIdx.x; j <= 4 * p; j += 64) T[j] = g[j];
  } else {
    const double2* g = reac_tab + (int64_t)t * P * P;
    for (int j = threadIdx.x; j < P * P; j += 64) T[j] = g[j];
  }
  const int e0 = ptr[t], e1 = ptr[t + 1];
  for (int e = e0; e < e1; e += M2L_BATCH) {
    const int ne = min(M2L_BATCH, e1 - e);
    __syncthreads();
    for (int j = threadIdx.x; j < ne * P; j += 64) {
      const int q = j / P, n = j % P;
      A[q * P + n] = me[(int64_t)src[e + q] * P + n];
    }
    __syncthreads();
    if (threadIdx.x < (unsigned)P) {
      const int mrow = threadIdx.x;
      double re[M2L_BATCH], im[M2L_BATCH];
#pragma unroll
      for (int q = 0; q < M2L_BATCH; ++q) re[q] = im[q] = 0.0;
      if (isfree) {
        for (int n = 0; n < P; ++n) {
          const double2 gv = T[n - mrow + 2 * p];
#pragma unroll
          for (int q = 0; q < M2L_BATCH; ++q) {
            const double2 av = A[q * P + n];
            re[q] += gv.x * av.x - gv.y * av.y;
            im[q] += gv.x * av.y + gv.y * av.x;
          }
        }
#pragma unroll
        for (int q = 0; q < M2L_BATCH; ++q) {  // times i/4
          const double r2 = -0.25 * im[q], i2 = 0.25 * re[q];
          re[q] = r2;
          im[q] = i2;
        }
      } else {
        for (int n = 0; n < P; ++n) {
          const double2 tv = T[n * P + mrow];
#pragma unroll
          for (int q = 0; q < M2L_BATCH; ++q) {
            const double2 av = A[q * P + n];
            re[q] += tv.x * av.x - tv.y * av.y;
            im[q] += tv.x * av.y + tv.y * av.x;
          }
        }
      }
      for (int q = 0; q < ne; ++q) out[(int64_t)slot[e + q] * P + mrow] = make_double2(re[q], im[q]);
    }
  }
}

// LE of each target box = sum of its entries' slots.
__global__ void __launch_bounds__(64) k_m2l_reduce(int p, const int* __restrict__ tgts, const int* __restrict__ ptr,
                                                   const double2* __restrict__ out, double2* __restrict__ le) {
  const int P = 2 * p + 1;
  if (threadIdx.x >= (unsigned)P) return;
  double re = 0.0, im = 0.0;
  for (int e = ptr[blockIdx.x]; e < ptr[blockIdx.x + 1]; ++e) {
    const double2 v = out[(int64_t)e * P + threadIdx.x];
    re += v.x;
    im += v.y;
  }
  le[(int64_t)tgts[blockIdx.x] * P + threadIdx.x] = make_double2(re, im);
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
  const MediumDev& m = g->m;
  const int L = m.L;
  const int64_t N = g->N;
  const int p = g->p;
  LM_CHECK(p >= 4 && p <= MAXP, LM_EINVAL, "the FMM needs 4 <= p <= %d", MAXP);
  F->p = p;
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
  F->w_top = 4.0 / m.kmax;
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

  // ---- M2M / L2L operators F_j(child - parent) ---------------------------------
  {
    const int J = 2 * p;
    F->ftab.assign((size_t)(L + 1) * nlev * 4 * (2 * J + 1), zd(0.0, 0.0));
    std::vector<zd> buf(2 * J + 1);
    std::vector<double> jb(J + 1);
    for (int l = 0; l <= L; ++l)
      for (int lev = 1; lev < nlev; ++lev)
        for (int pos = 0; pos < 4; ++pos) {
          const double d = 0.5 * wl(lev);
          const double dx = (pos & 1) ? 0.5 * d : -0.5 * d;
          const double dh = (pos & 2) ? 0.5 * d : -0.5 * d;
          // child centre - parent centre = (+-w_lev/2, +-w_lev/2)
          fm::f_seq(m.k[l], 2.0 * dx, 2.0 * dh, J, buf.data(), jb.data());
          std::copy(buf.begin(), buf.end(), F->ftab.begin() + ((size_t)((l * nlev + lev) * 4 + pos)) * (2 * J + 1));
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
  for (int b = 0; b < F->n_boxes; ++b) {
    const BoxDev& B = F->boxes[b];
    const TreeB& tb = T[B.tree];
    const int lev = B.level;
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
    for (int64_t i = 0; i < N; ++i) {
      int64_t len = 1 + (F->rn_ptr[i + 1] - F->rn_ptr[i]);
      const int t = leaf_slot[i];
      for (int e = F->near_ptr[t]; e < F->near_ptr[t + 1]; ++e) len += F->boxes[F->near_src[e]].npt;
      len -= 1;  // the element itself
      F->nm_ptr[i + 1] = (int)len;
    }
    for (int64_t i = 0; i < N; ++i) F->nm_ptr[i + 1] += F->nm_ptr[i];
    const int64_t nnz = F->nm_ptr[N];
    LM_CHECK(nnz < ((int64_t)1 << 31), LM_ENOMEM, "near-field matrix too large");
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
  }

  // ---- upload and device setup ---------------------------------------------------
  LM_TRY(up(F->d_boxes, F->boxes, s));
  LM_TRY(up(F->d_children, F->children, s));
  LM_TRY(up(F->d_pt_elem, F->pt_elem, s));
  LM_TRY(up(F->d_pt_xh, F->pt_xh, s));
  LM_TRY(up(F->d_leaf_free, F->leaf_free, s));
  LM_TRY(up(F->d_leaf_B, F->leaf_B, s));
  LM_TRY(up(F->d_leaf_T, F->leaf_T, s));
  LM_TRY(up(F->d_parents, F->parents_by_level, s));
  LM_TRY(up(F->d_m2l_tgt, F->m2l_tgt, s));
  LM_TRY(up(F->d_m2l_ptr, F->m2l_ptr, s));
  LM_TRY(up(F->d_m2l_src, F->m2l_src, s));
  LM_TRY(up(F->d_m2l_tab, F->m2l_tab, s));
  LM_TRY(up(F->d_near_tgt, F->near_tgt, s));
  LM_TRY(up(F->d_near_ptr, F->near_ptr, s));
  LM_TRY(up(F->d_near_src, F->near_src, s));
  LM_TRY(up(F->d_rn_ptr, F->rn_ptr, s));
  LM_TRY(up(F->d_rn_src, F->rn_src, s));
  {
    std::vector<double2> ft(F->ftab.size());
    for (size_t i = 0; i < ft.size(); ++i) ft[i] = make_double2(F->ftab[i].re, F->ftab[i].im);
    LM_TRY(up(F->d_ftab, ft, s));
    F->tree_layer = tree_layer;
    LM_TRY(up(F->d_tree_layer, F->tree_layer, s));
  }
  {
    std::vector<double2> self(N);
    for (int64_t e = 0; e < N; ++e) {
      const double k = m.k[g->layer[e]], w = g->w[e];
      self[e] = make_double2(-(kEulerGamma + std::log(k * w / 4.0) - 1.0) / (2.0 * M_PI) * w, 0.25 * w);
    }
    LM_TRY(up(F->d_self, self, s));
  }
  // free-space Hankel tables
  const int nfree = (int)free_id.size(), nreac = (int)reac_id.size();
  LM_TRY(F->d_free_tab.alloc((size_t)std::max(nfree, 1) * (4 * p + 1) * sizeof(double2)));
  if (nfree) {
    DevBuf geo;
    LM_TRY(up(geo, F->free_geo, s));
    hipLaunchKernelGGL(k_free_tables, dim3(div_up(nfree, 64)), dim3(64), 0, s, nfree, p, geo.as<double>(),
                       F->d_free_tab.as<double2>());
    LM_TRY_HIP(hipGetLastError());
    LM_TRY_HIP(hipStreamSynchronize(s));
  }
  // reaction tables
  LM_TRY(F->d_reac_tab.alloc((size_t)std::max(nreac, 1) * F->P * F->P * sizeof(double2)));
  if (nreac) {
    DevBuf meta, geo;
    LM_TRY(up(meta, F->reac_meta, s));
    LM_TRY(up(geo, F->reac_geo, s));
    hipLaunchKernelGGL(k_reac_tables, dim3(nreac), dim3(256), 0, s, m, p, meta.as<int>(), geo.as<double>(),
                       F->d_reac_tab.as<double2>());
    LM_TRY_HIP(hipGetLastError());
    LM_TRY_HIP(hipStreamSynchronize(s));
  }
  // near-field matrix values
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
                       g->d_w.as<double>(), g->d_layer.as<int>(), F->d_self.as<double2>(), F->d_nm_val.as<double2>());
    LM_TRY_HIP(hipGetLastError());
    LM_TRY_HIP(hipStreamSynchronize(s));
  }
  LM_TRY(up(F->d_tm_ptr, F->tm_ptr, s));
  LM_TRY(up(F->d_tm_slot, F->tm_slot, s));
  LM_TRY(up(F->d_tm_src, F->tm_src, s));
  LM_TRY(F->d_m2l_out.alloc(std::max<size_t>(F->m2l_src.size(), 1) * F->P * sizeof(double2)));
  LM_TRY(F->d_me.alloc((size_t)F->n_boxes * F->P * sizeof(double2)));
  LM_TRY(F->d_le.alloc((size_t)F->n_boxes * F->P * sizeof(double2)));
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

// Stage timing: when ev != nullptr, ev[2*i], ev[2*i+1] bracket stage i on
// stream s (0 P2M, 1 M2M, 2 M2L, 3 L2L, 4 L2P, 5 near-field matrix, 6 unused).
lm_status fmm_matvec_timed(lm_geom_s* g, int precision, int n_rhs, const void* xv, void* yv, hipStream_t s,
                           hipEvent_t* ev);

lm_status fmm_matvec(lm_geom_s* g, int precision, int n_rhs, const void* xv, void* yv, hipStream_t s) {
  return fmm_matvec_timed(g, precision, n_rhs, xv, yv, s, nullptr);
}

lm_status fmm_matvec_timed(lm_geom_s* g, int precision, int n_rhs, const void* xv, void* yv, hipStream_t s,
                           hipEvent_t* ev) {
  FmmPlan* F = g->fmm;
  LM_CHECK(F, LM_EINTERNAL, "no FMM plan");
  LM_CHECK(precision == LM_FP64, LM_EINVAL, "the FMM matvec supports LM_FP64 only in this build");
  const int N = (int)g->N, p = F->p, P = F->P;
  const BoxDev* boxes = F->d_boxes.as<BoxDev>();
  const int* tl = F->d_tree_layer.as<int>();
  for (int r = 0; r < n_rhs; ++r) {
    const double2* x = (const double2*)xv + (int64_t)r * N;
    double2* y = (double2*)yv + (int64_t)r * N;
    double2* me = F->d_me.as<double2>();
    double2* le = F->d_le.as<double2>();
#define LM_STAGE(i, open)                                             \
  if (ev && r == 0) LM_TRY_HIP(hipEventRecord(ev[2 * (i) + ((open) ? 0 : 1)], s))
    LM_STAGE(0, 1);
    // P2M on every leaf (leaves of all trees; internal boxes come from M2M)
    const std::vector<int>* leaves[3] = {&F->leaf_free, &F->leaf_B, &F->leaf_T};
    const DevBuf* dleaves[3] = {&F->d_leaf_free, &F->d_leaf_B, &F->d_leaf_T};
    for (int c = 0; c < 3; ++c)
      if (!leaves[c]->empty())
        hipLaunchKernelGGL(k_p2m, dim3(leaves[c]->size()), dim3(WG), 0, s, p, dleaves[c]->as<int>(), boxes,
                           F->d_pt_elem.as<int>(), F->d_pt_xh.as<double2>(), g->d_w.as<double>(), x, me);
    LM_STAGE(0, 0);
    LM_STAGE(1, 1);
    // M2M, finest parents first
    for (int l = F->nlev - 2; l >= 0; --l) {
      const int n = F->parents_ptr[l + 1] - F->parents_ptr[l];
      if (n)
        hipLaunchKernelGGL(k_m2m, dim3(n), dim3(WG), 0, s, p, F->nlev, F->d_parents.as<int>() + F->parents_ptr[l],
                           boxes, F->d_children.as<int>(), tl, F->d_ftab.as<double2>(), me);
    }
    LM_STAGE(1, 0);
    // M2L (every level at once); boxes without a list start from zero
    LM_TRY_HIP(hipMemsetAsync(le, 0, (size_t)F->n_boxes * P * sizeof(double2), s));
    LM_STAGE(2, 1);
    if (!F->m2l_tgt.empty()) {
      const int ntab = F->n_reac_tab + F->n_free_tab;
      const size_t lds = (size_t)(std::max(P * P, 4 * p + 1) + M2L_BATCH * P) * sizeof(double2);
      hipLaunchKernelGGL(k_m2l_apply, dim3(ntab), dim3(64), lds, s, p, F->n_reac_tab, F->d_tm_ptr.as<int>(),
                         F->d_tm_slot.as<int>(), F->d_tm_src.as<int>(), F->d_free_tab.as<double2>(),
                         F->d_reac_tab.as<double2>(), me, F->d_m2l_out.as<double2>());
      hipLaunchKernelGGL(k_m2l_reduce, dim3(F->m2l_tgt.size()), dim3(64), 0, s, p, F->d_m2l_tgt.as<int>(),
                         F->d_m2l_ptr.as<int>(), F->d_m2l_out.as<double2>(), le);
    }
    LM_STAGE(2, 0);
    LM_STAGE(3, 1);
    // L2L, coarse to fine
    for (int l = 1; l < F->nlev; ++l) {
      const int n = F->level_ptr[l + 1] - F->level_ptr[l];
      if (n)
        hipLaunchKernelGGL(k_l2l, dim3(n), dim3(WG), 0, s, p, F->nlev, F->level_ptr[l], boxes, tl,
                           F->d_ftab.as<double2>(), le);
    }
    LM_STAGE(3, 0);
    LM_STAGE(4, 1);
    // L2P: free trees write, side trees accumulate (each element once per launch)
    for (int c = 0; c < 3; ++c)
      if (!leaves[c]->empty())
        hipLaunchKernelGGL(k_l2p, dim3(leaves[c]->size()), dim3(WG), 0, s, p, c > 0 ? 1 : 0, dleaves[c]->as<int>(),
                           boxes, F->d_pt_elem.as<int>(), F->d_pt_xh.as<double2>(), le, y);
    LM_STAGE(4, 0);
    LM_STAGE(5, 1);
    // near fields and self terms
    hipLaunchKernelGGL(k_near_csr, dim3(div_up(N, 4)), dim3(256), 0, s, N, F->d_nm_ptr.as<int>(),
                       F->d_nm_src.as<int>(), F->d_nm_val.as<double2>(), x, y);
    LM_STAGE(5, 0);
    LM_STAGE(6, 1);
    LM_STAGE(6, 0);
#undef LM_STAGE
    LM_TRY_HIP(hipGetLastError());
  }
  return LM_OK;
}

// Average per-stage durations (ms) over reps matvecs, measured with HIP events
// on the stream the kernels run on; out[7] = whole matvec.
lm_status fmm_stage_times(lm_geom_s* g, int precision, int n_rhs, const void* x, void* y, int reps, hipStream_t s,
                          double* out) {
  hipEvent_t ev[16];
  for (int i = 0; i < 16; ++i) LM_TRY_HIP(hipEventCreate(&ev[i]));
  for (int i = 0; i < 8; ++i) out[i] = 0.0;
  lm_status st = LM_OK;
  for (int r = 0; r < reps && st == LM_OK; ++r) {
    LM_TRY_HIP(hipEventRecord(ev[14], s));
    st = fmm_matvec_timed(g, precision, n_rhs, x, y, s, ev);
    LM_TRY_HIP(hipEventRecord(ev[15], s));
    LM_TRY_HIP(hipEventSynchronize(ev[15]));
    for (int i = 0; i < 7; ++i) {
      float ms = 0;
      LM_TRY_HIP(hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]));
      out[i] += ms / reps;
    }
    float ms = 0;
    LM_TRY_HIP(hipEventElapsedTime(&ms, ev[14], ev[15]));
    out[7] += ms / reps;
  }
  for (int i = 0; i < 16; ++i) (void)hipEventDestroy(ev[i]);
  return st;
}
