// Overlapping domain-decomposition preconditioner (Sec. 4.2 of the paper).
//
// For every leaf box B of a layer's free-space tree: J = the elements of B and
// of its neighbour leaves (B's own first).  The local matrix keeps only the
// free-space interaction and the singular self term (eq. localmatix):
//   P_B[i][j] = |Gamma_j| (i/4) H_0(k |c_i - c_j|)  (i != j),  P_B[i][i] = I^s_i.
// The preconditioner keeps the rows of P_B^{-1} that belong to B and adds
// the local solutions: P^{-1} = sum_B S_B Q_B P_B^{-1} R_B.
//
// P_B = A W with A complex symmetric (A_ij = (i/4) H_0(k r_ij), A_ii = I^s_i /
// |Gamma_i|) and W = diag |Gamma|, so the rows of P_B^{-1} for B are
// (1/|Gamma_r|) (A^{-1} e_r)^T.  Setup, per subdomain: a kernel assembles A
// in device memory, rocSOLVER factors it (LU with partial pivoting, FP64) and
// solves for the |B| unit vectors, and a kernel stores the scaled rows.
// Subdomains are the free-space tree's boxes at the leaf level, or `coarsen`
// levels above it (bigger overlapping blocks: fewer GMRES iterations for a
// larger setup and apply); coarsen < 0 picks the coarsest level that fits.  Apply: y_{B_r} = sum_j Z_B[r][j] x_{J_j} (Z row-major, so
// the lanes of a wavefront read consecutive addresses of one row); the
// mixed form applies an FP32 copy of Z.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <map>
#include <tuple>

#include "block_mfma.hpp"
#include "fmm_plan.hpp"

constexpr int PRE_QMAX = 8192;  // largest subdomain neighbourhood (LU workspace qmax^2 complex128)

struct Precond {
  int nleaf = 0, qmax = 0, bmax = 0;
  std::vector<int> jptr, jidx, nb;
  std::vector<int64_t> zoff;
  std::vector<int> items;  // (subdomain, first row) work items of PA_ROWS rows for the MFMA apply
  DevBuf d_jptr, d_jidx, d_nb, d_zoff, d_Z, d_Z32, d_items;
  DevBuf d_xt;  // transposed complex64 input of the matrix-core apply
  int64_t bytes() const {
    return d_jptr.bytes + d_jidx.bytes + d_nb.bytes + d_zoff.bytes + d_Z.bytes + d_Z32.bytes + d_items.bytes +
           d_xt.bytes;
  }
};

void precond_free(Precond* p) { delete p; }
int64_t precond_bytes(const Precond* p) { return p ? p->bytes() : 0; }

static constexpr double kEulerGamma = 0.57721566490153286061;

// A (q x q, symmetric, so row- and column-major agree) for one subdomain.
__global__ void k_pre_assemble(MediumDev m, int q, const int* __restrict__ J, const double* __restrict__ cx,
                               const double* __restrict__ cy, const double* __restrict__ w,
                               const int* __restrict__ lay, double2* __restrict__ A) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)q * q) return;
  const int i = (int)(idx / q), jj = (int)(idx % q);
  const int ei = J[i], ej = J[jj];
  const double k = m.k[lay[J[0]]];
  double re, im;
  if (i == jj) {
    re = -(kEulerGamma + log(k * w[ei] / 4.0) - 1.0) / (2.0 * M_PI);
    im = 0.25;
  } else {
    const double r = hypot(cx[ei] - cx[ej], cy[ei] - cy[ej]);
    re = -0.25 * y0(k * r);
    im = 0.25 * j0(k * r);
  }
  A[idx] = make_double2(re, im);
}

// X = the first nB unit vectors (q x nB, column-major).
__global__ void k_pre_unit(int q, int nB, double2* __restrict__ X) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)q * nB) return;
  const int r = (int)(idx / q), j = (int)(idx % q);
  X[idx] = make_double2(j == r ? 1.0 : 0.0, 0.0);
}

// Z_B[r][j] = X[j][r] / |Gamma_{J_r}|  (row r of P_B^{-1}).
__global__ void k_pre_store(int q, int nB, const int* __restrict__ J, const double* __restrict__ w,
                            const double2* __restrict__ X, double2* __restrict__ Z) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)q * nB) return;
  const int r = (int)(idx / q);
  const double sc = 1.0 / w[J[r]];
  const double2 v = X[idx];
  Z[idx] = make_double2(v.x * sc, v.y * sc);
}

// y_{B_r} = sum_j Z_B[r][j] x_{J_j}: one workgroup per leaf; x_J of RG
// right-hand sides at a time is staged in LDS (in the arithmetic type), each
// wavefront takes rows r = wave, wave + 4, ... two at a time, lanes run along
// the rows (coalesced Z loads), and a wavefront reduction finishes each row.
template <typename ZT, typename RT, int RG>
__global__ void __launch_bounds__(256) k_pre_apply(int N, int R, const int* __restrict__ jptr,
                                                   const int* __restrict__ jidx, const int* __restrict__ nb,
                                                   const int64_t* __restrict__ zoff, const ZT* __restrict__ Z,
                                                   const double2* __restrict__ x, double2* __restrict__ y) {
  typedef ZT V;
  extern __shared__ unsigned char dyn[];
  V* xs = reinterpret_cast<V*>(dyn);  // [RG][q]
  const int leaf = blockIdx.x;
  const int j0_ = jptr[leaf], q = jptr[leaf + 1] - j0_, nB = nb[leaf];
  const int* J = jidx + j0_;
  const ZT* Zl = Z + zoff[leaf];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int g = 0; g < R; g += RG) {
    const int ng = min(RG, R - g);
    __syncthreads();
    for (int idx = threadIdx.x; idx < ng * q; idx += 256) {
      const int u = idx / q, j = idx - u * q;
      const double2 v = x[(int64_t)(g + u) * N + J[j]];
      V t;
      t.x = (RT)v.x;
      t.y = (RT)v.y;
      xs[u * q + j] = t;
    }
    __syncthreads();
    for (int r = wv; r < nB; r += 8) {
      const int r2 = r + 4;
      const bool two = r2 < nB;
      const ZT* z1 = Zl + (int64_t)r * q;
      const ZT* z2 = Zl + (int64_t)(two ? r2 : r) * q;
      RT a1[RG][2], a2[RG][2];
#pragma unroll
      for (int u = 0; u < RG; ++u) a1[u][0] = a1[u][1] = a2[u][0] = a2[u][1] = RT(0);
#pragma unroll 4
      for (int j = lane; j < q; j += 64) {
        const ZT p1 = z1[j], p2 = z2[j];
#pragma unroll
        for (int u = 0; u < RG; ++u) {
          if (u < ng) {
            const V xv = xs[u * q + j];
            a1[u][0] = fma((RT)p1.x, xv.x, a1[u][0]);
            a1[u][0] = fma(-(RT)p1.y, xv.y, a1[u][0]);
            a1[u][1] = fma((RT)p1.x, xv.y, a1[u][1]);
            a1[u][1] = fma((RT)p1.y, xv.x, a1[u][1]);
            a2[u][0] = fma((RT)p2.x, xv.x, a2[u][0]);
            a2[u][0] = fma(-(RT)p2.y, xv.y, a2[u][0]);
            a2[u][1] = fma((RT)p2.x, xv.y, a2[u][1]);
            a2[u][1] = fma((RT)p2.y, xv.x, a2[u][1]);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < RG; ++u)
#pragma unroll
        for (int c = 0; c < 2; ++c)
          for (int off = 32; off > 0; off >>= 1) {
            a1[u][c] += __shfl_xor(a1[u][c], off, 64);
            a2[u][c] += __shfl_xor(a2[u][c], off, 64);
          }
      if (lane == 0) {
#pragma unroll
        for (int u = 0; u < RG; ++u) {
          if (u < ng) {
            y[(int64_t)(g + u) * N + J[r]] = make_double2((double)a1[u][0], (double)a1[u][1]);
            if (two) y[(int64_t)(g + u) * N + J[r2]] = make_double2((double)a2[u][0], (double)a2[u][1]);
          }
        }
      }
    }
  }
}

__global__ void k_z_to_c64(int64_t n, const double2* __restrict__ a, float2* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = make_float2((float)a[i].x, (float)a[i].y);
}

lm_status precond_build(lm_geom_s* g, int coarsen, hipStream_t s) {
  FmmPlan* F = g->fmm;
  LM_CHECK(F, LM_EINTERNAL, "the preconditioner needs the FMM plan");
  auto* P = new (std::nothrow) Precond();
  LM_CHECK(P, LM_ENOMEM, "host allocation failed");
  g->pre = P;
  // subdomains: free-tree boxes at level lp; each owns the points of its
  // leaves; neighbourhood = the subdomain and its (up to 8) level-lp neighbours
  auto plan = [&](int lp) {
    P->jptr.assign(1, 0);
    P->jidx.clear();
    P->nb.clear();
    P->zoff.clear();
    P->qmax = P->bmax = 0;
    std::map<std::tuple<int, int, int>, std::vector<int>> pts;  // (tree, i, j) -> elements
    for (int b : F->leaf_free) {
      const BoxDev& B = F->boxes[b];
      const int sh = B.level - lp;
      const double wb = F->w_top / (double)(1 << B.level);
      const int i = (int)std::lround((B.cx - F->x0) / wb - 0.5) >> sh;
      const int j = (int)std::lround(B.ch / wb - 0.5) >> sh;
      auto& v = pts[std::make_tuple(B.tree, i, j)];
      for (int k = 0; k < B.npt; ++k) v.push_back(F->pt_elem[B.pt0 + k]);
    }
    int64_t z = 0;
    for (auto& kv : pts) {
      const int t = std::get<0>(kv.first), i = std::get<1>(kv.first), j = std::get<2>(kv.first);
      for (int e : kv.second) P->jidx.push_back(e);
      for (int di = -1; di <= 1; ++di)
        for (int dj = -1; dj <= 1; ++dj) {
          if (!di && !dj) continue;
          auto it = pts.find(std::make_tuple(t, i + di, j + dj));
          if (it == pts.end()) continue;
          for (int e : it->second) P->jidx.push_back(e);
        }
      const int q = (int)P->jidx.size() - P->jptr.back();
      const int nB = (int)kv.second.size();
      P->jptr.push_back((int)P->jidx.size());
      P->nb.push_back(nB);
      P->zoff.push_back(z);
      z += (int64_t)q * nB;
      P->qmax = std::max(P->qmax, q);
      P->bmax = std::max(P->bmax, nB);
    }
    return z;
  };
  int64_t z = 0;  // stored block entries
  if (coarsen >= 0) {
    z = plan(std::max(0, F->lf - coarsen));
  } else {
    // automatic: the coarsest level whose neighbourhoods fit PRE_QMAX and
    // whose blocks (FP64 and FP32 copies) take at most a quarter of the free
    // device memory; the leaf level otherwise
    size_t fr = 0, tot = 0;
    LM_TRY_HIP(hipMemGetInfo(&fr, &tot));
    for (int lp = 0; lp <= F->lf; ++lp) {
      z = plan(lp);
      if (lp == F->lf || (P->qmax <= PRE_QMAX && (double)z * 24.0 <= 0.25 * (double)fr)) break;
    }
  }
  P->nleaf = (int)P->nb.size();
  for (int b = 0; b < P->nleaf; ++b)
    for (int r = 0; r < P->nb[b]; r += PA_ROWS) {
      P->items.push_back(b);
      P->items.push_back(r);
    }
  LM_CHECK(P->qmax <= PRE_QMAX, LM_EINVAL, "preconditioner neighbourhood too large (%d > %d); use a finer level",
           P->qmax, PRE_QMAX);
  {  // the VALU apply stages x_J of one or two right-hand sides in LDS (up to 128 KiB)
    const void* fs[4] = {(const void*)k_pre_apply<double2, double, 1>, (const void*)k_pre_apply<double2, double, 2>,
                         (const void*)k_pre_apply<float2, float, 2>, (const void*)k_pre_apply<float2, float, 4>};
    for (const void* f : fs)
      LM_TRY_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 2 * PRE_QMAX * 8));
  }
  LM_TRY(upload(P->d_jptr, P->jptr.data(), P->jptr.size() * sizeof(int), s));
  LM_TRY(upload(P->d_jidx, P->jidx.data(), P->jidx.size() * sizeof(int), s));
  LM_TRY(upload(P->d_nb, P->nb.data(), P->nb.size() * sizeof(int), s));
  LM_TRY(upload(P->d_zoff, P->zoff.data(), P->zoff.size() * sizeof(int64_t), s));
  LM_TRY(upload(P->d_items, P->items.data(), P->items.size() * sizeof(int), s));
  LM_TRY(P->d_Z.alloc(std::max<int64_t>(z, 1) * sizeof(double2)));
  DevBuf A, X, piv, info;
  LM_TRY(A.alloc((size_t)P->qmax * P->qmax * sizeof(double2)));
  LM_TRY(X.alloc((size_t)P->qmax * P->bmax * sizeof(double2)));
  LM_TRY(piv.alloc((size_t)P->qmax * sizeof(rocblas_int)));
  LM_TRY(info.alloc((size_t)P->nleaf * sizeof(rocblas_int)));
  rocblas_handle h = nullptr;
  LM_CHECK(rocblas_create_handle(&h) == rocblas_status_success, LM_EINTERNAL, "rocblas_create_handle failed");
  struct HandleGuard {
    rocblas_handle h;
    ~HandleGuard() { rocblas_destroy_handle(h); }
  } guard{h};
  LM_CHECK(rocblas_set_stream(h, s) == rocblas_status_success, LM_EINTERNAL, "rocblas_set_stream failed");
  auto* Ad = A.as<rocblas_double_complex>();
  auto* Xd = X.as<rocblas_double_complex>();
  for (int b = 0; b < P->nleaf; ++b) {
    const int q = P->jptr[b + 1] - P->jptr[b], nB = P->nb[b];
    const int* J = P->d_jidx.as<int>() + P->jptr[b];
    hipLaunchKernelGGL(k_pre_assemble, dim3(div_up((int64_t)q * q, 256)), dim3(256), 0, s, g->m, q, J,
                       g->d_cx.as<double>(), g->d_cy.as<double>(), g->d_w.as<double>(), g->d_layer.as<int>(),
                       A.as<double2>());
    hipLaunchKernelGGL(k_pre_unit, dim3(div_up((int64_t)q * nB, 256)), dim3(256), 0, s, q, nB, X.as<double2>());
    LM_TRY_HIP(hipGetLastError());
    LM_CHECK(rocsolver_zgetrf(h, q, q, Ad, q, piv.as<rocblas_int>(), info.as<rocblas_int>() + b) ==
                 rocblas_status_success, LM_EINTERNAL, "rocsolver_zgetrf failed");
    LM_CHECK(rocsolver_zgetrs(h, rocblas_operation_none, q, nB, Ad, q, piv.as<rocblas_int>(), Xd, q) ==
                 rocblas_status_success, LM_EINTERNAL, "rocsolver_zgetrs failed");
    hipLaunchKernelGGL(k_pre_store, dim3(div_up((int64_t)q * nB, 256)), dim3(256), 0, s, q, nB, J, g->d_w.as<double>(),
                       X.as<double2>(), P->d_Z.as<double2>() + P->zoff[b]);
    LM_TRY_HIP(hipGetLastError());
  }
  std::vector<rocblas_int> inf(P->nleaf);
  LM_TRY_HIP(hipMemcpyAsync(inf.data(), info.p, inf.size() * sizeof(rocblas_int), hipMemcpyDeviceToHost, s));
  LM_TRY_HIP(hipStreamSynchronize(s));
  for (int b = 0; b < P->nleaf; ++b)
    LM_CHECK(inf[b] == 0, LM_EINTERNAL, "singular preconditioner block %d (pivot %d)", b, (int)inf[b]);
  LM_TRY(P->d_Z32.alloc(std::max<int64_t>(z, 1) * sizeof(float2)));
  hipLaunchKernelGGL(k_z_to_c64, dim3(div_up(std::max<int64_t>(z, 1), 256)), dim3(256), 0, s, z, P->d_Z.as<double2>(),
                     P->d_Z32.as<float2>());
  LM_TRY_HIP(hipGetLastError());
  LM_TRY_HIP(hipStreamSynchronize(s));
  return LM_OK;
}

lm_status precond_apply(lm_geom_s* g, int precision, int n_rhs, const void* x, void* y, hipStream_t s) {
  Precond* P = g->pre;
  LM_CHECK(P, LM_EINVAL, "no preconditioner");
  if (precision == LM_MIXED && n_rhs > 1) {
    const size_t need = (size_t)g->N * std::min(n_rhs, 64) * sizeof(float2);
    if (P->d_xt.bytes < need) LM_TRY(P->d_xt.alloc(need));
    for (int r0 = 0; r0 < n_rhs; r0 += 64) {
      const int R = std::min(64, n_rhs - r0);
      hipLaunchKernelGGL(k_to_nr<double2>, dim3(div_up(g->N, 32), div_up(R, 32)), dim3(32, 8), 0, s, (int)g->N, R,
                         (const double2*)x + (int64_t)r0 * g->N, P->d_xt.as<float2>());
      hipLaunchKernelGGL((k_block_mfma<double2, false>), dim3(P->items.size() / 2), dim3(64 * PA_NW), 0, s,
                         (int)g->N, R, P->d_items.as<int>(), P->d_jptr.as<int>(), P->d_jidx.as<int>(),
                         P->d_nb.as<int>(), P->d_zoff.as<int64_t>(), P->d_Z32.as<float2>(), P->d_xt.as<float2>(),
                         (double2*)y + (int64_t)r0 * g->N);
    }
    LM_TRY_HIP(hipGetLastError());
    return LM_OK;
  }
  // x_J of RG right-hand sides is staged in LDS: RG q sizeof <= 64 KiB
  const bool big = P->qmax > 2048;
  if (precision == LM_FP64) {
    if (big)
      hipLaunchKernelGGL((k_pre_apply<double2, double, 1>), dim3(P->nleaf), dim3(256),
                         (size_t)P->qmax * sizeof(double2), s, (int)g->N, n_rhs, P->d_jptr.as<int>(),
                         P->d_jidx.as<int>(), P->d_nb.as<int>(), P->d_zoff.as<int64_t>(), P->d_Z.as<double2>(),
                         (const double2*)x, (double2*)y);
    else
      hipLaunchKernelGGL((k_pre_apply<double2, double, 2>), dim3(P->nleaf), dim3(256),
                         (size_t)2 * P->qmax * sizeof(double2), s, (int)g->N, n_rhs, P->d_jptr.as<int>(),
                         P->d_jidx.as<int>(), P->d_nb.as<int>(), P->d_zoff.as<int64_t>(), P->d_Z.as<double2>(),
                         (const double2*)x, (double2*)y);
  } else {
    if (big)
      hipLaunchKernelGGL((k_pre_apply<float2, float, 2>), dim3(P->nleaf), dim3(256),
                         (size_t)2 * P->qmax * sizeof(float2), s, (int)g->N, n_rhs, P->d_jptr.as<int>(),
                         P->d_jidx.as<int>(), P->d_nb.as<int>(), P->d_zoff.as<int64_t>(), P->d_Z32.as<float2>(),
                         (const double2*)x, (double2*)y);
    else
      hipLaunchKernelGGL((k_pre_apply<float2, float, 4>), dim3(P->nleaf), dim3(256),
                         (size_t)4 * P->qmax * sizeof(float2), s, (int)g->N, n_rhs, P->d_jptr.as<int>(),
                         P->d_jidx.as<int>(), P->d_nb.as<int>(), P->d_zoff.as<int64_t>(), P->d_Z32.as<float2>(),
                         (const double2*)x, (double2*)y);
  }
  LM_TRY_HIP(hipGetLastError());
  return LM_OK;
}
