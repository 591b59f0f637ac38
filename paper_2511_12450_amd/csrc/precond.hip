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
// larger setup and apply); coarsen < 0 picks the coarsest level that fits.
// Apply: y_{B_r} = sum_j Z_B[r][j] x_{J_j} (Z row-major, so the lanes of a
// wavefront read consecutive addresses of one row); the FP32 form applies a
// binary16 copy of Z on matrix cores (see k_pre_h16).
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <map>
#include <tuple>

#include "fmm_plan.hpp"

constexpr int PRE_QMAX = 8192;  // largest subdomain neighbourhood (LU workspace qmax^2 complex128)

struct Precond {
  int nleaf = 0, qmax = 0, bmax = 0;
  int level = 0, leaf_level = 0;  // tree level of the subdomain boxes; leaf level of the free-space trees
  std::vector<int> jptr, jidx, nb;
  std::vector<int64_t> zoff, rowoff, zhoff;  // zhoff: binary16 blocks (row stride q rounded up to 4)
  // FP32-form apply: work items (subdomain, first row, first column, column
  // end, partial slot) of PH_ROWS rows and at most PH_KSEG columns (the
  // columns of a row block split evenly); per row block (subdomain, first
  // row, first slot, count) the slots are summed in order
  std::vector<int> items, sums;
  int nslot = 0;
  DevBuf d_jptr, d_jidx, d_nb, d_zoff, d_zhoff, d_rowoff, d_Z, d_Zh, d_rsc, d_items, d_sums, d_part;
  DevBuf d_xh, d_xl, d_cmax;  // split half-precision input of the FP32-form apply, column maxima
  int64_t bytes() const {
    return d_jptr.bytes + d_jidx.bytes + d_nb.bytes + d_zoff.bytes + d_zhoff.bytes + d_rowoff.bytes + d_Z.bytes + d_Zh.bytes +
           d_rsc.bytes + d_items.bytes + d_xh.bytes + d_xl.bytes + d_cmax.bytes + d_sums.bytes + d_part.bytes;
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

// y_{B_r} = sum_j Z_B[r][j] x_{J_j}: one workgroup per leaf; x_J of RG
// right-hand sides at a time is staged in LDS (in the arithmetic type), each
// wavefront takes rows r = wave, wave + 4, ... two at a time, lanes run along
// the rows (coalesced Z loads), and a wavefront reduction finishes each row.
constexpr int PA_ROWS_FP64 = 32;  // rows per workgroup of the FP64 apply
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
  // rows [r_lo, r_hi) of the subdomain: PA_ROWS per workgroup, so that every
  // CU has work (a subdomain per workgroup would leave most of them idle)
  const int r_lo = blockIdx.y * PA_ROWS_FP64, r_hi = min(nB, r_lo + PA_ROWS_FP64);
  if (r_lo >= nB) return;
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
    for (int r = r_lo + wv; r < r_hi; r += 8) {
      const int r2 = r + 4;
      const bool two = r2 < r_hi;
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

// ---- FP32-form apply on half-precision matrix cores ------------------------------
// The preconditioner only sets the iteration count, provided that every
// application in a solve is the same fixed complex-linear operator.  The FP32
// form therefore stores the rows of P_B^{-1} once in binary16 (each row
// scaled by a power of two so that its largest part is below 1, the scale
// kept in FP32) and applies them with v_mfma_f32_16x16x16f16 (FP32
// accumulation) to an input split into two binary16 parts x = x_hi + x_lo
// (each right-hand side scaled by a power of two first): the operator is
// fixed, and the input is represented to about 2^-22 of its largest element,
// as in FP32.  The complex product uses the interleaved real embedding (four
// real products, so the operator stays complex-linear): real row 2r + rho,
// real column 2c + kappa, A = Re Z for rho == kappa, -Im Z for (0, 1), Im Z
// for (1, 0); a lane holds the four k of two complex columns, i.e. one
// 8-byte pair (Z[r][c], Z[r][c+1]) with the imaginary sign flipped (rho = 0)
// or the halves swapped (rho = 1).
typedef _Float16 ph4 __attribute__((ext_vector_type(4)));
typedef float pf4 __attribute__((ext_vector_type(4)));
constexpr int PH_ROWS = 128, PH_KC = 32, PH_ZR = 20, PH_XS = 80;  // rows per item; LDS strides
constexpr int PH_XLD = 64;  // row stride of the split input (right-hand sides)
constexpr int PH_KSEG = 1024;  // most columns per work item (a multiple of PH_KC)
constexpr int PH_MAXSEG = 8;    // column ranges of a row block: PRE_QMAX / PH_KSEG
static_assert(PH_MAXSEG * PH_KSEG >= PRE_QMAX, "slots per row block");
// Stored binary16 rows are padded with zeros to a multiple of PH_KC columns
// (128 bytes), so every chunk a work item loads is whole 128-byte lines.
__host__ __device__ inline int h16_qp(int q) { return (q + PH_KC - 1) / PH_KC * PH_KC; }

__device__ __forceinline__ uint32_t h16_pack(float re, float im) {
  const _Float16 a = (_Float16)re, b = (_Float16)im;
  return (uint32_t)__builtin_bit_cast(uint16_t, a) | ((uint32_t)__builtin_bit_cast(uint16_t, b) << 16);
}
__device__ __forceinline__ float h16_lo(uint32_t v) { return (float)__builtin_bit_cast(_Float16, (uint16_t)(v & 0xffffu)); }
__device__ __forceinline__ float h16_hi(uint32_t v) { return (float)__builtin_bit_cast(_Float16, (uint16_t)(v >> 16)); }

// Row r (global index) of the stored blocks: scale 2^e with max |Re|, |Im| < 2^e,
// binary16 entries of the scaled row at rzh[r], zero up to h16_qp(q).
__global__ void __launch_bounds__(256) k_z_to_h16(const int64_t* __restrict__ rz, const int64_t* __restrict__ rzh,
                                                  const int* __restrict__ rq, const double2* __restrict__ Z,
                                                  uint32_t* __restrict__ Zh, float* __restrict__ rsc) {
  const int r = blockIdx.x;
  const int64_t o = rz[r], oh = rzh[r];
  const int q = rq[r], qp = h16_qp(q);
  double m = 0.0;
  for (int c = threadIdx.x; c < q; c += 256) m = fmax(m, fmax(fabs(Z[o + c].x), fabs(Z[o + c].y)));
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  __shared__ double wm[4];
  if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
  __syncthreads();
  m = fmax(fmax(wm[0], wm[1]), fmax(wm[2], wm[3]));
  int e = 0;
  if (m > 0.0) (void)frexp(m, &e);  // m = f 2^e, f in [0.5, 1)
  const double sc = ldexp(1.0, -e);
  for (int c = threadIdx.x; c < qp; c += 256)
    Zh[oh + c] = c < q ? h16_pack((float)(Z[o + c].x * sc), (float)(Z[o + c].y * sc)) : 0u;
  if (threadIdx.x == 0) rsc[r] = (float)ldexp(1.0, e);
}

// cmax[j] = max |Re|, |Im| of right-hand side j (as FP32 bits; cmax zeroed before):
// H16_CM elements per workgroup, one atomic per workgroup.
constexpr int H16_CM = 8192;
__global__ void __launch_bounds__(256) k_h16_colmax(int N, const double2* __restrict__ x, unsigned* __restrict__ cmax) {
  const int j = blockIdx.y;
  float m = 0.f;
  for (int n0 = blockIdx.x * H16_CM + threadIdx.x; n0 < min(N, (int)(blockIdx.x + 1) * H16_CM); n0 += 2048) {
    double2 v[8];  // eight loads in flight before the maxima
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (n0 + 256 * u < N) v[u] = x[(int64_t)j * N + n0 + 256 * u];
      else v[u] = make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) m = fmaxf(m, fmaxf((float)fabs(v[u].x), (float)fabs(v[u].y)));
  }
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
  __shared__ float wm[4];
  if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) atomicMax(cmax + j, __float_as_uint(fmaxf(fmaxf(wm[0], wm[1]), fmaxf(wm[2], wm[3]))));
}

// v where keep, else zeros (component selects: no select between addresses)
__device__ __forceinline__ uint4 ph_keep(bool keep, uint4 v) {
  const uint32_t m = keep ? 0xffffffffu : 0u;
  return make_uint4(v.x & m, v.y & m, v.z & m, v.w & m);
}

__device__ __forceinline__ int h16_col_exp(unsigned bits) {
  const float m = __uint_as_float(bits);
  int e = 0;
  if (m > 0.f) (void)frexpf(m, &e);
  return e;
}

// xh[n][j] + xl[n][j] = 2^-e_j x[j][n] (binary16 pairs, row stride PH_XLD, 32 x 32
// tiles through LDS).
__global__ void __launch_bounds__(256) k_h16_split(int N, int R, const double2* __restrict__ x,
                                                   const unsigned* __restrict__ cmax, uint32_t* __restrict__ xh,
                                                   uint32_t* __restrict__ xl) {
  __shared__ uint2 tile[32][33];
  const int n0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
  for (int k = threadIdx.y; k < 32; k += 8) {
    const int j = j0 + k, n = n0 + threadIdx.x;
    if (j < R && n < N) {
      const float sc = ldexpf(1.f, -h16_col_exp(cmax[j]));
      const double2 v = x[(int64_t)j * N + n];
      const float re = (float)v.x * sc, im = (float)v.y * sc;
      const uint32_t hi = h16_pack(re, im);
      tile[k][threadIdx.x] = make_uint2(hi, h16_pack(re - h16_lo(hi), im - h16_hi(hi)));
    }
  }
  __syncthreads();
  for (int k = threadIdx.y; k < 32; k += 8) {
    const int n = n0 + k, j = j0 + threadIdx.x;
    if (n < N && j < R) {
      const uint2 t = tile[threadIdx.x][k];
      xh[(int64_t)n * PH_XLD + j] = t.x;
      xl[(int64_t)n * PH_XLD + j] = t.y;
    }
  }
}

// y_{B_r}[j] = sum_c Z_B[r][c] x_{J_c}[j] for a (subdomain, PH_ROWS rows,
// PH_KSEG columns) item: 8 wavefronts in a 4 x 2 grid, each 4 x 2 tiles of 16
// real rows (8 complex) x 16 right-hand sides; K in chunks of PH_KC complex
// columns, 8 per k-step.  The next chunk's binary16 data is loaded into
// registers while the current one is multiplied, so one barrier pair per
// chunk is all the staging costs.  Splitting long rows over several items
// keeps every CU busy until the end (neighbourhoods differ by 2-3x in size);
// every item leaves its FP32 sums in a partial slot and k_pre_h16_sum adds
// the slots of a row block in order (so the operator stays fixed), scales
// them and writes y along the rows.
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(6))) k_pre_h16(int R, const int* __restrict__ items, const int* __restrict__ jptr,
                                                 const int* __restrict__ jidx, const int* __restrict__ nb,
                                                 const int64_t* __restrict__ zoff, const uint32_t* __restrict__ Zh,
                                                 const uint32_t* __restrict__ xh, const uint32_t* __restrict__ xl,
                                                 float2* __restrict__ part) {
  constexpr int TR = PH_ROWS / 32, UZ = PH_ROWS * PH_KC / 2048, UX = PH_KC * 64 / 2048;  // 16-byte loads per thread
  // [row][column pair]: a row's 16-byte loads go to LDS as 16-byte stores
  // side by side, and the fragment reads (8 rows x 4 column pairs) meet 32
  // different bank pairs (row stride 40 words).  Chunks of 32 columns keep
  // the LDS of a workgroup at 41 KB and its registers at 79, so three
  // workgroups share a CU
  __shared__ uint2 Zs[PH_ROWS][PH_ZR];
  __shared__ uint2 Xh[PH_KC / 2][PH_XS];  // [column pair][right-hand side]
  __shared__ uint2 Xl[PH_KC / 2][PH_XS];
  const int* it = items + 5 * blockIdx.x;
  const int sd = it[0], r0 = it[1], cb = it[2], ce = it[3], slot = it[4];
  const int j0 = jptr[sd], q = jptr[sd + 1] - j0, qp = h16_qp(q);
  const int rows = min(PH_ROWS, nb[sd] - r0);
  const int* J = jidx + j0;
  const uint32_t* Zl = Zh + zoff[sd] + (int64_t)r0 * qp;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int l16 = lane & 15, kq = lane >> 4;
  const int wr = wv >> 1, wc = wv & 1;
  const bool rho = (l16 & 1) != 0;
  pf4 acc[TR][2];
#pragma unroll
  for (int t = 0; t < TR; ++t)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[t][c] = pf4{0.f, 0.f, 0.f, 0.f};
  uint4 zr[UZ], hr[UX], lr[UX];
// Next chunk into registers: 4 consecutive columns of a Z row (rows padded to
// h16_qp), 4 consecutive right-hand sides of an input row.
#define PH_FETCH(c0)                                                                                                   \
  do {                                                                                                                 \
_Pragma("unroll")                                                                                                      \
    for (int u = 0; u < UZ; ++u) {                                                                                     \
      const int idx = threadIdx.x + 512 * u, rr = idx / (PH_KC / 4), cq = 4 * (idx % (PH_KC / 4));                     \
      const bool okz = rr < rows && c0 + cq < qp;                                                                      \
      const uint4 tz = *reinterpret_cast<const uint4*>(Zl + (okz ? (int64_t)rr * qp + c0 + cq : 0));                   \
      zr[u] = ph_keep(okz, tz);                                                                                        \
    }                                                                                                                  \
_Pragma("unroll")                                                                                                      \
    for (int u = 0; u < UX; ++u) {                                                                                     \
      const int idx = threadIdx.x + 512 * u, cc = idx >> 4, jq = 4 * (idx & 15);                                       \
      const bool ok = c0 + cc < q && jq < R;                                                                           \
      const int64_t o = ok ? (int64_t)J[c0 + cc] * PH_XLD + jq : 0;                                                    \
      const uint4 th = *reinterpret_cast<const uint4*>(xh + o), tl = *reinterpret_cast<const uint4*>(xl + o);          \
      hr[u] = ph_keep(ok, th);                                                                                         \
      lr[u] = ph_keep(ok, tl);                                                                                         \
    }                                                                                                                  \
  } while (0)
  if (cb < ce) PH_FETCH(cb);
  for (int c0 = cb; c0 < ce; c0 += PH_KC) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < UZ; ++u) {
      const int idx = threadIdx.x + 512 * u, rr = idx / (PH_KC / 4), cq = 4 * (idx % (PH_KC / 4));
      *reinterpret_cast<uint4*>(&Zs[rr][cq >> 1]) = zr[u];
    }
#pragma unroll
    for (int u = 0; u < UX; ++u) {
      const int idx = threadIdx.x + 512 * u, cc = idx >> 4, jq = 4 * (idx & 15);
      uint32_t* ph = reinterpret_cast<uint32_t*>(&Xh[cc >> 1][jq]) + (cc & 1);
      uint32_t* pl = reinterpret_cast<uint32_t*>(&Xl[cc >> 1][jq]) + (cc & 1);
      ph[0] = hr[u].x;
      ph[2] = hr[u].y;
      ph[4] = hr[u].z;
      ph[6] = hr[u].w;
      pl[0] = lr[u].x;
      pl[2] = lr[u].y;
      pl[4] = lr[u].z;
      pl[6] = lr[u].w;
    }
    __syncthreads();
    if (c0 + PH_KC < ce) PH_FETCH(c0 + PH_KC);
#pragma unroll
    for (int ks = 0; ks < PH_KC / 8; ++ks) {
      const int pr = 4 * ks + kq;  // column pair of this lane's four k
      ph4 bh[2], bl[2];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        bh[c] = __builtin_bit_cast(ph4, Xh[pr][16 * (2 * wc + c) + l16]);
        bl[c] = __builtin_bit_cast(ph4, Xl[pr][16 * (2 * wc + c) + l16]);
      }
#pragma unroll
      for (int t = 0; t < TR; ++t) {
        uint2 z = Zs[8 * (TR * wr + t) + (l16 >> 1)][pr];
        if (rho) {
          z.x = (z.x >> 16) | (z.x << 16);
          z.y = (z.y >> 16) | (z.y << 16);
        } else {
          z.x ^= 0x80000000u;
          z.y ^= 0x80000000u;
        }
        const ph4 a = __builtin_bit_cast(ph4, z);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x16f16(a, bh[c], acc[t][c], 0, 0, 0);
          acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x16f16(a, bl[c], acc[t][c], 0, 0, 0);
        }
      }
    }
  }
#undef PH_FETCH
  // FP32 sums of this column range into its partial slot (lane rows 4 kq + v
  // of a tile: complex row 8 rt + 2 kq + v / 2, real part for even v)
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int j = 16 * (2 * wc + c) + l16;
    if (j >= R) continue;
#pragma unroll
    for (int t = 0; t < TR; ++t)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int r = 8 * (TR * wr + t) + 2 * kq + h;
        if (r < rows)
          part[((int64_t)slot * PH_ROWS + r) * PH_XLD + j] = make_float2(acc[t][c][2 * h], acc[t][c][2 * h + 1]);
      }
  }
}

// Every row block: y = scales x (sum of its partial slots, in slot order).  Slots are read along the right-hand sides and y is
// written along the rows (through an LDS transpose, 16 right-hand sides at a
// time), so both sides stay coalesced.
__global__ void __launch_bounds__(256) k_pre_h16_sum(int N, int R, const int* __restrict__ sums,
                                                     const int* __restrict__ jptr, const int* __restrict__ jidx,
                                                     const int* __restrict__ nb, const int64_t* __restrict__ rowoff,
                                                     const float* __restrict__ rsc, const unsigned* __restrict__ cmax,
                                                     const float2* __restrict__ part, double2* __restrict__ y) {
  __shared__ double2 T[16][PH_ROWS + 1];
  const int sd = sums[4 * blockIdx.x], r0 = sums[4 * blockIdx.x + 1];
  const int slot0 = sums[4 * blockIdx.x + 2], ns = sums[4 * blockIdx.x + 3];
  const int rows = min(PH_ROWS, nb[sd] - r0);
  const int* J = jidx + jptr[sd];
  const float* rs = rsc + rowoff[sd] + r0;
  for (int jh = 0; jh < R; jh += 16) {
    for (int idx = threadIdx.x; idx < rows * 16; idx += blockDim.x) {
      const int r = idx >> 4, jj = idx & 15;
      double re = 0.0, im = 0.0;
      if (jh + jj < R) {
        // a row block has at most PH_MAXSEG slots; all loads of a pass are
        // issued before the sums (added in slot order)
        float2 v[PH_MAXSEG];
#pragma unroll
        for (int k = 0; k < PH_MAXSEG; ++k)  // clamped addresses (ns >= 1); extra slots are dropped below
          v[k] = part[((int64_t)(slot0 + min(k, ns - 1)) * PH_ROWS + r) * PH_XLD + jh + jj];
#pragma unroll
        for (int k = 0; k < PH_MAXSEG; ++k)
          if (k < ns) {
            re += v[k].x;
            im += v[k].y;
          }
      }
      T[jj][r] = make_double2(re, im);
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < rows * 16; idx += blockDim.x) {
      const int jj = idx / rows, r = idx - jj * rows, j = jh + jj;
      if (j < R) {
        const double sc = ldexp(1.0, h16_col_exp(cmax[j])) * (double)rs[r];
        const double2 v = T[jj][r];
        y[(int64_t)j * N + J[r0 + r]] = make_double2(v.x * sc, v.y * sc);
      }
    }
    __syncthreads();
  }
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
    P->level = lp;
    P->leaf_level = F->lf;
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
  for (int b = 0; b < P->nleaf; ++b) {
    const int q = P->jptr[b + 1] - P->jptr[b], nseg = std::max(1, (q + PH_KSEG - 1) / PH_KSEG);
    const int len = ((q + nseg - 1) / nseg + PH_KC - 1) / PH_KC * PH_KC;  // <= PH_KSEG
    for (int r = 0; r < P->nb[b]; r += PH_ROWS) {
      P->sums.insert(P->sums.end(), {b, r, P->nslot, nseg});
      for (int k = 0; k < nseg; ++k) P->items.insert(P->items.end(), {b, r, k * len, std::min(q, (k + 1) * len), P->nslot++});
    }
  }
  {  // every item has its own slot: launch the largest (rows x columns) first
    const int nit = (int)P->items.size() / 5;
    std::vector<int64_t> work(nit);
    std::vector<int> ord(nit);
    for (int i = 0; i < nit; ++i) {
      const int* it = &P->items[5 * i];
      work[i] = (int64_t)std::min(PH_ROWS, P->nb[it[0]] - it[1]) * (it[3] - it[2]);
      ord[i] = i;
    }
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return work[a] > work[b]; });
    std::vector<int> sorted(P->items.size());
    for (int i = 0; i < nit; ++i)
      for (int c = 0; c < 5; ++c) sorted[5 * i + c] = P->items[5 * ord[i] + c];
    P->items.swap(sorted);
  }
  LM_CHECK(P->qmax <= PRE_QMAX, LM_EINVAL, "preconditioner neighbourhood too large (%d > %d); use a finer level",
           P->qmax, PRE_QMAX);
  {  // the VALU apply stages x_J of one or two right-hand sides in LDS (up to 128 KiB)
    const void* fs[2] = {(const void*)k_pre_apply<double2, double, 1>, (const void*)k_pre_apply<double2, double, 2>};
    for (const void* f : fs)
      LM_TRY_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 2 * PRE_QMAX * 8));
  }
  LM_TRY(upload(P->d_jptr, P->jptr.data(), P->jptr.size() * sizeof(int), s));
  LM_TRY(upload(P->d_jidx, P->jidx.data(), P->jidx.size() * sizeof(int), s));
  LM_TRY(upload(P->d_nb, P->nb.data(), P->nb.size() * sizeof(int), s));
  LM_TRY(upload(P->d_zoff, P->zoff.data(), P->zoff.size() * sizeof(int64_t), s));
  LM_TRY(upload(P->d_items, P->items.data(), P->items.size() * sizeof(int), s));
  LM_TRY(upload(P->d_sums, P->sums.data(), P->sums.size() * sizeof(int), s));
  LM_TRY(P->d_part.alloc((size_t)P->nslot * PH_ROWS * PH_XLD * sizeof(float2)));
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
  // binary16 rows with power-of-two row scales for the FP32-form apply
  {
    std::vector<int64_t> rz, rzh;
    std::vector<int> rq;
    P->rowoff.assign(1, 0);
    P->zhoff.clear();
    int64_t zh = 0;
    for (int b = 0; b < P->nleaf; ++b) {
      const int q = P->jptr[b + 1] - P->jptr[b], qp = h16_qp(q);
      P->zhoff.push_back(zh);
      for (int r = 0; r < P->nb[b]; ++r) {
        rz.push_back(P->zoff[b] + (int64_t)r * q);
        rzh.push_back(zh + (int64_t)r * qp);
        rq.push_back(q);
      }
      zh += (int64_t)P->nb[b] * qp;
      P->rowoff.push_back(P->rowoff.back() + P->nb[b]);
    }
    DevBuf d_rz, d_rzh, d_rq;
    LM_TRY(upload(d_rz, rz.data(), rz.size() * sizeof(int64_t), s));
    LM_TRY(upload(d_rzh, rzh.data(), rzh.size() * sizeof(int64_t), s));
    LM_TRY(upload(d_rq, rq.data(), rq.size() * sizeof(int), s));
    LM_TRY(upload(P->d_rowoff, P->rowoff.data(), P->rowoff.size() * sizeof(int64_t), s));
    LM_TRY(upload(P->d_zhoff, P->zhoff.data(), P->zhoff.size() * sizeof(int64_t), s));
    LM_TRY(P->d_Zh.alloc(std::max<int64_t>(zh, 4) * sizeof(uint32_t)));
    LM_TRY(P->d_rsc.alloc(std::max<size_t>(rz.size(), 1) * sizeof(float)));
    if (!rz.empty())
      hipLaunchKernelGGL(k_z_to_h16, dim3(rz.size()), dim3(256), 0, s, d_rz.as<int64_t>(), d_rzh.as<int64_t>(),
                         d_rq.as<int>(), P->d_Z.as<double2>(), P->d_Zh.as<uint32_t>(), P->d_rsc.as<float>());
    LM_TRY_HIP(hipGetLastError());
    LM_TRY_HIP(hipStreamSynchronize(s));
  }
  return LM_OK;
}

lm_status precond_subdomains(const lm_geom_s* g, int64_t* info4, int32_t* jptr, int32_t* nb, int32_t* jidx) {
  const Precond* P = g->pre;
  LM_CHECK(P, LM_EINVAL, "the geometry has no preconditioner");
  info4[0] = P->nleaf;
  info4[1] = P->level;
  info4[2] = (int64_t)P->jidx.size();
  info4[3] = P->leaf_level;
  if (jptr) std::copy(P->jptr.begin(), P->jptr.end(), jptr);
  if (nb) std::copy(P->nb.begin(), P->nb.end(), nb);
  if (jidx) std::copy(P->jidx.begin(), P->jidx.end(), jidx);
  return LM_OK;
}

lm_status precond_apply(lm_geom_s* g, int precision, int n_rhs, const void* x, void* y, hipStream_t s) {
  Precond* P = g->pre;
  LM_CHECK(P, LM_EINVAL, "no preconditioner");
  if (precision == LM_MIXED) {  // half-precision matrix cores, chunks of 64 right-hand sides
    const int N = (int)g->N, Rc = std::min(n_rhs, 64);
    const size_t need = (size_t)N * PH_XLD * sizeof(uint32_t);
    if (P->d_xh.bytes < need) LM_TRY(P->d_xh.alloc(need));
    if (P->d_xl.bytes < need) LM_TRY(P->d_xl.alloc(need));
    if (!P->d_cmax.p) LM_TRY(P->d_cmax.alloc(64 * sizeof(unsigned)));
    for (int r0 = 0; r0 < n_rhs; r0 += 64) {
      const int R = std::min(64, n_rhs - r0);
      const double2* xr = (const double2*)x + (int64_t)r0 * N;
      LM_TRY_HIP(hipMemsetAsync(P->d_cmax.p, 0, (size_t)R * sizeof(unsigned), s));
      hipLaunchKernelGGL(k_h16_colmax, dim3(div_up(N, H16_CM), R), dim3(256), 0, s, N, xr, P->d_cmax.as<unsigned>());
      hipLaunchKernelGGL(k_h16_split, dim3(div_up(N, 32), div_up(R, 32)), dim3(32, 8), 0, s, N, R, xr,
                         P->d_cmax.as<unsigned>(), P->d_xh.as<uint32_t>(), P->d_xl.as<uint32_t>());
      hipLaunchKernelGGL(k_pre_h16, dim3(P->items.size() / 5), dim3(512), 0, s, R, P->d_items.as<int>(),
                         P->d_jptr.as<int>(), P->d_jidx.as<int>(), P->d_nb.as<int>(), P->d_zhoff.as<int64_t>(),
                         P->d_Zh.as<uint32_t>(), P->d_xh.as<uint32_t>(), P->d_xl.as<uint32_t>(),
                         P->d_part.as<float2>());
      if (!P->sums.empty())
        hipLaunchKernelGGL(k_pre_h16_sum, dim3(P->sums.size() / 4), dim3(256), 0, s, N, R, P->d_sums.as<int>(),
                           P->d_jptr.as<int>(), P->d_jidx.as<int>(), P->d_nb.as<int>(), P->d_rowoff.as<int64_t>(),
                           P->d_rsc.as<float>(), P->d_cmax.as<unsigned>(), P->d_part.as<float2>(),
                           (double2*)y + (int64_t)r0 * N);
    }
    LM_TRY_HIP(hipGetLastError());
    return LM_OK;
  }
  // FP64: x_J of RG right-hand sides is staged in LDS: RG q sizeof <= 128 KiB
  const bool big = P->qmax > 2048;
  if (big)
    hipLaunchKernelGGL((k_pre_apply<double2, double, 1>), dim3(P->nleaf, div_up(P->bmax, PA_ROWS_FP64)), dim3(256),
                       (size_t)P->qmax * sizeof(double2), s, (int)g->N, n_rhs, P->d_jptr.as<int>(),
                       P->d_jidx.as<int>(), P->d_nb.as<int>(), P->d_zoff.as<int64_t>(), P->d_Z.as<double2>(),
                       (const double2*)x, (double2*)y);
  else
    hipLaunchKernelGGL((k_pre_apply<double2, double, 2>), dim3(P->nleaf, div_up(P->bmax, PA_ROWS_FP64)), dim3(256),
                       (size_t)2 * P->qmax * sizeof(double2), s, (int)g->N, n_rhs, P->d_jptr.as<int>(),
                       P->d_jidx.as<int>(), P->d_nb.as<int>(), P->d_zoff.as<int64_t>(), P->d_Z.as<double2>(),
                       (const double2*)x, (double2*)y);
  LM_TRY_HIP(hipGetLastError());
  return LM_OK;
}
