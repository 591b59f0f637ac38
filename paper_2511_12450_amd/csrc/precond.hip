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
// (1/|Gamma_r|) (A^{-1} e_r)^T.  Setup: one workgroup per leaf assembles A in
// device scratch, factors it (LU, partial pivoting) and solves for the |B|
// unit vectors.  Apply: y_{B_r} = sum_j Z_B[r][j] x_{J_j} (Z row-major, so
// the lanes of a wavefront read consecutive addresses of one row); the
// mixed form applies an FP32 copy of Z.
#include <algorithm>

#include "fmm_plan.hpp"

struct Precond {
  int nleaf = 0, qmax = 0, bmax = 0;
  std::vector<int> jptr, jidx, nb;
  std::vector<int64_t> zoff;
  DevBuf d_jptr, d_jidx, d_nb, d_zoff, d_Z, d_Z32, d_tmp;
  int64_t bytes() const {
    return d_jptr.bytes + d_jidx.bytes + d_nb.bytes + d_zoff.bytes + d_Z.bytes + d_Z32.bytes;
  }
};

void precond_free(Precond* p) { delete p; }
int64_t precond_bytes(const Precond* p) { return p ? p->bytes() : 0; }

static constexpr double kEulerGamma = 0.57721566490153286061;

__global__ void __launch_bounds__(256) k_pre_setup(MediumDev m, int first, const int* __restrict__ jptr,
                                                   const int* __restrict__ jidx, const int* __restrict__ nb,
                                                   const int64_t* __restrict__ zoff, const double* __restrict__ cx,
                                                   const double* __restrict__ cy, const double* __restrict__ w,
                                                   const int* __restrict__ lay, double2* __restrict__ scratch,
                                                   int64_t scratch_stride, double2* __restrict__ Z) {
  const int leaf = first + blockIdx.x;
  const int j0_ = jptr[leaf];
  const int q = jptr[leaf + 1] - j0_;
  const int nB = nb[leaf];
  const int* J = jidx + j0_;
  double2* A = scratch + (int64_t)blockIdx.x * scratch_stride;  // q*q row-major, then q*nB solutions
  double2* X = A + (int64_t)q * q;
  const double k = m.k[lay[J[0]]];
  __shared__ int perm[2048];
  __shared__ double rbest[256];
  __shared__ int ibest[256];
  for (int idx = threadIdx.x; idx < q * q; idx += blockDim.x) {
    const int i = idx / q, jj = idx % q;
    const int ei = J[i], ej = J[jj];
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
  for (int i = threadIdx.x; i < q; i += blockDim.x) perm[i] = i;
  __syncthreads();
  for (int kk = 0; kk < q; ++kk) {
    double best = -1.0;
    int bi = kk;
    for (int i = kk + threadIdx.x; i < q; i += blockDim.x) {
      const double2 v = A[(int64_t)i * q + kk];
      const double a = v.x * v.x + v.y * v.y;
      if (a > best) {
        best = a;
        bi = i;
      }
    }
    rbest[threadIdx.x] = best;
    ibest[threadIdx.x] = bi;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if (threadIdx.x < (unsigned)off && rbest[threadIdx.x + off] > rbest[threadIdx.x]) {
        rbest[threadIdx.x] = rbest[threadIdx.x + off];
        ibest[threadIdx.x] = ibest[threadIdx.x + off];
      }
      __syncthreads();
    }
    const int piv = ibest[0];
    if (piv != kk) {
      for (int jj = threadIdx.x; jj < q; jj += blockDim.x) {
        const double2 t = A[(int64_t)kk * q + jj];
        A[(int64_t)kk * q + jj] = A[(int64_t)piv * q + jj];
        A[(int64_t)piv * q + jj] = t;
      }
      if (threadIdx.x == 0) {
        const int t = perm[kk];
        perm[kk] = perm[piv];
        perm[piv] = t;
      }
    }
    __syncthreads();
    const double2 pv = A[(int64_t)kk * q + kk];
    const zd inv = 1.0 / zd(pv.x, pv.y);
    for (int i = kk + 1 + threadIdx.x; i < q; i += blockDim.x) {
      const double2 v = A[(int64_t)i * q + kk];
      const zd l = zd(v.x, v.y) * inv;
      A[(int64_t)i * q + kk] = make_double2(l.re, l.im);
    }
    __syncthreads();
    const int rem = q - kk - 1;
    for (int idx = threadIdx.x; idx < rem * rem; idx += blockDim.x) {
      const int i = kk + 1 + idx / rem, jj = kk + 1 + idx % rem;
      const double2 l = A[(int64_t)i * q + kk], u = A[(int64_t)kk * q + jj];
      double2 a = A[(int64_t)i * q + jj];
      a.x -= l.x * u.x - l.y * u.y;
      a.y -= l.x * u.y + l.y * u.x;
      A[(int64_t)i * q + jj] = a;
    }
    __syncthreads();
  }
  // column r of A^{-1}: solve L U z = P e_r (one thread per right-hand side)
  for (int r = threadIdx.x; r < nB; r += blockDim.x) {
    double2* z = X + (int64_t)r * q;
    for (int i = 0; i < q; ++i) {  // forward, unit lower
      zd acc(perm[i] == r ? 1.0 : 0.0, 0.0);
      for (int jj = 0; jj < i; ++jj) {
        const double2 l = A[(int64_t)i * q + jj], v = z[jj];
        acc -= zd(l.x, l.y) * zd(v.x, v.y);
      }
      z[i] = make_double2(acc.re, acc.im);
    }
    for (int i = q - 1; i >= 0; --i) {  // backward
      const double2 zi = z[i];
      zd acc(zi.x, zi.y);
      for (int jj = i + 1; jj < q; ++jj) {
        const double2 u = A[(int64_t)i * q + jj], v = z[jj];
        acc -= zd(u.x, u.y) * zd(v.x, v.y);
      }
      const double2 d = A[(int64_t)i * q + i];
      acc = acc / zd(d.x, d.y);
      z[i] = make_double2(acc.re, acc.im);
    }
    const double s = 1.0 / w[J[r]];
    double2* Zl = Z + zoff[leaf];
    for (int jj = 0; jj < q; ++jj) Zl[(int64_t)r * q + jj] = make_double2(z[jj].x * s, z[jj].y * s);
  }
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

lm_status precond_build(lm_geom_s* g, hipStream_t s) {
  FmmPlan* F = g->fmm;
  LM_CHECK(F, LM_EINTERNAL, "the preconditioner needs the FMM plan");
  auto* P = new (std::nothrow) Precond();
  LM_CHECK(P, LM_ENOMEM, "host allocation failed");
  g->pre = P;
  // neighbourhoods from the free-space near lists (leaf itself first)
  P->jptr.push_back(0);
  int64_t z = 0;
  for (size_t t = 0; t < F->near_tgt.size(); ++t) {
    const int b = F->near_tgt[t];
    const BoxDev& B = F->boxes[b];
    for (int i = 0; i < B.npt; ++i) P->jidx.push_back(F->pt_elem[B.pt0 + i]);
    for (int e = F->near_ptr[t]; e < F->near_ptr[t + 1]; ++e) {
      const int c = F->near_src[e];
      if (c == b) continue;
      const BoxDev& C = F->boxes[c];
      for (int i = 0; i < C.npt; ++i) P->jidx.push_back(F->pt_elem[C.pt0 + i]);
    }
    const int q = (int)P->jidx.size() - P->jptr.back();
    P->jptr.push_back((int)P->jidx.size());
    P->nb.push_back(B.npt);
    P->zoff.push_back(z);
    z += (int64_t)q * B.npt;
    P->qmax = std::max(P->qmax, q);
    P->bmax = std::max(P->bmax, B.npt);
  }
  P->nleaf = (int)P->nb.size();
  LM_CHECK(P->qmax <= 2048, LM_EINVAL, "preconditioner neighbourhood too large (%d); use a smaller leaf_size", P->qmax);
  LM_TRY(upload(P->d_jptr, P->jptr.data(), P->jptr.size() * sizeof(int), s));
  LM_TRY(upload(P->d_jidx, P->jidx.data(), P->jidx.size() * sizeof(int), s));
  LM_TRY(upload(P->d_nb, P->nb.data(), P->nb.size() * sizeof(int), s));
  LM_TRY(upload(P->d_zoff, P->zoff.data(), P->zoff.size() * sizeof(int64_t), s));
  LM_TRY(P->d_Z.alloc(std::max<int64_t>(z, 1) * sizeof(double2)));
  const int64_t stride = (int64_t)P->qmax * P->qmax + (int64_t)P->qmax * P->bmax;
  const int batch = (int)std::max<int64_t>(1, std::min<int64_t>(P->nleaf, ((int64_t)1 << 29) / (stride * 16)));
  DevBuf scratch;
  LM_TRY(scratch.alloc((size_t)batch * stride * sizeof(double2)));
  for (int first = 0; first < P->nleaf; first += batch) {
    const int n = std::min(batch, P->nleaf - first);
    hipLaunchKernelGGL(k_pre_setup, dim3(n), dim3(256), 0, s, g->m, first, P->d_jptr.as<int>(), P->d_jidx.as<int>(),
                       P->d_nb.as<int>(), P->d_zoff.as<int64_t>(), g->d_cx.as<double>(), g->d_cy.as<double>(),
                       g->d_w.as<double>(), g->d_layer.as<int>(), scratch.as<double2>(), stride,
                       P->d_Z.as<double2>());
    LM_TRY_HIP(hipGetLastError());
  }
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
  if (precision == LM_FP64)
    hipLaunchKernelGGL((k_pre_apply<double2, double, 2>), dim3(P->nleaf), dim3(256),
                       (size_t)2 * P->qmax * sizeof(double2), s, (int)g->N, n_rhs, P->d_jptr.as<int>(),
                       P->d_jidx.as<int>(), P->d_nb.as<int>(), P->d_zoff.as<int64_t>(), P->d_Z.as<double2>(),
                       (const double2*)x, (double2*)y);
  else
    hipLaunchKernelGGL((k_pre_apply<float2, float, 4>), dim3(P->nleaf), dim3(256),
                       (size_t)4 * P->qmax * sizeof(float2), s, (int)g->N, n_rhs, P->d_jptr.as<int>(),
                       P->d_jidx.as<int>(), P->d_nb.as<int>(), P->d_zoff.as<int64_t>(), P->d_Z32.as<float2>(),
                       (const double2*)x, (double2*)y);
  LM_TRY_HIP(hipGetLastError());
  return LM_OK;
}
