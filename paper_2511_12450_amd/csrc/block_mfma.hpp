// Block-sparse complex products on matrix cores (preconditioner apply and
// near field, several right-hand sides).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

// Block-sparse products with matrix cores, for several right-hand sides:
// Y_B (rows x R) (=|+=) Z_B (rows x q) X_J (q x R) per work item of PA_ROWS
// rows of one block (a subdomain of the preconditioner, a leaf box with its
// neighbours for the near field, a P2M or L2P point block), in 16x16x4 FP32
// MFMA tiles (FP32 accumulation) by the three-multiplication form of the
// complex product: T1 = Re Z Re X, T2 = Im Z Im X, T3 = (Re Z + Im Z)
// (Re X + Im X), Y = (T1 - T2) + i (T3 - T1 - T2), three real products
// instead of four.  A tile is 16 complex rows x 16 right-hand sides; a k-step
// takes 4 complex columns (lane row = lane % 16, column = lane / 16), and one
// 64-bit LDS load gives both parts of a fragment, so the third operand is
// one add.  The input is the complex64 transpose xt [N][R] (k_to_nr), so a
// neighbourhood row of all right-hand sides is one contiguous load; Z_B is
// row-major complex64.  K runs over the neighbourhood in chunks of PA_KC
// complex columns staged in LDS: the Z chunk row-major with row stride PA_ZK
// = 36 complex (a row's loads are stored side by side, and the fragment
// reads of 16 rows x 4 columns meet every bank exactly twice), the X chunk
// [c][j] with row stride 80 complex.  The next chunk is loaded into registers
// while the current one is multiplied.  Eight wavefronts in a 4 x 2 grid
// hold 1 x 2 tiles each.
typedef float pa_v4f __attribute__((ext_vector_type(4)));
constexpr int PA_ROWS = 64, PA_KC = 32, PA_NW = 8, PA_LS = 80, PA_ZK = 36;
constexpr int PA_UZ = PA_ROWS * PA_KC / (64 * PA_NW), PA_UX = PA_KC * 64 / (64 * PA_NW);  // loads per thread
// The product of one work item.  Op describes the item:
//   rows, q                  output rows (<= PA_ROWS) and K length (complex)
//   zrow(r)                  row r of the item's matrix (q complex64)
//   brow(c)                  row c of the right operand (R complex64)
//   store(r, j, re, im)      writes (or adds) output row r, right-hand side j
template <class Op>
__device__ __forceinline__ void block_mfma_body(const Op& op, int R) {
  constexpr int TC = 2, NTH = 64 * PA_NW;
  __shared__ float2 Zs[PA_ROWS][PA_ZK];
  __shared__ float2 Xs[PA_KC][PA_LS];
  const int rows = op.rows, q = op.q;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int l16 = lane & 15, kq = lane >> 4;
  const int rt = wv >> 1, wc = wv & 1;  // row tile, column-tile pair
  const int aoff = (16 * rt + l16) * PA_ZK + kq;  // complex offsets of this lane's fragments at k-step 0
  int boff[TC];
#pragma unroll
  for (int c = 0; c < TC; ++c) boff[c] = kq * PA_LS + 16 * (wc * TC + c) + l16;
  const float2* Zf = &Zs[0][0];
  const float2* Xf = &Xs[0][0];
  pa_v4f t1[TC], t2[TC], t3[TC];
#pragma unroll
  for (int c = 0; c < TC; ++c) t1[c] = t2[c] = t3[c] = pa_v4f{0.f, 0.f, 0.f, 0.f};
  // chunk c0 into registers: consecutive threads along a matrix row, and
  // along the right-hand sides of a neighbourhood row
  float2 zp[PA_UZ], xp[PA_UX];
  auto fetch = [&](int c0) {
    const int kc = min(PA_KC, q - c0);
#pragma unroll
    for (int u = 0; u < PA_UZ; ++u) {
      const int idx = threadIdx.x + NTH * u, rr = idx / PA_KC, jj = idx - rr * PA_KC;
      zp[u] = (rr < rows && jj < kc) ? op.zrow(rr)[c0 + jj] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < PA_UX; ++u) {
      const int idx = threadIdx.x + NTH * u, jj = idx >> 6, rr = idx & 63;
      xp[u] = (jj < kc && rr < R) ? op.brow(c0 + jj)[rr] : make_float2(0.f, 0.f);
    }
  };
  if (q > 0) fetch(0);
  for (int c0 = 0; c0 < q; c0 += PA_KC) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PA_UZ; ++u) {
      const int idx = threadIdx.x + NTH * u, rr = idx / PA_KC, jj = idx - rr * PA_KC;
      Zs[rr][jj] = zp[u];
    }
#pragma unroll
    for (int u = 0; u < PA_UX; ++u) {
      const int idx = threadIdx.x + NTH * u, jj = idx >> 6, rr = idx & 63;
      Xs[jj][rr] = xp[u];
    }
    __syncthreads();
    if (c0 + PA_KC < q) fetch(c0 + PA_KC);
#pragma unroll 2
    for (int ks = 0; ks < PA_KC / 4; ++ks) {
      const float2 av = Zf[aoff + 4 * ks];
      const float as = av.x + av.y;
#pragma unroll
      for (int c = 0; c < TC; ++c) {
        const float2 bv = Xf[boff[c] + 4 * ks * PA_LS];
        t1[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, bv.x, t1[c], 0, 0, 0);
        t2[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, bv.y, t2[c], 0, 0, 0);
        t3[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(as, bv.x + bv.y, t3[c], 0, 0, 0);
      }
    }
  }
  // lane rows 4 kq + v of a tile are output rows 16 rt + 4 kq + v
#pragma unroll
  for (int c = 0; c < TC; ++c) {
    const int j = 16 * (wc * TC + c) + l16;
    if (j < R) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * rt + 4 * kq + v;
        const float a = t1[c][v], b = t2[c][v];
        if (r < rows) op.store(r, j, a - b, t3[c][v] - a - b);
      }
    }
  }
}

// Near field / preconditioner blocks: item (block, first row); Z_B row-major
// (nb rows x q), neighbourhood J (the block's own rows first), output
// y[j][J[r]] of type YT, overwritten or (ACC) accumulated.
template <typename YT, bool ACC>
struct BlockOp {
  int rows, q, N, R;
  const float2* Zl;
  const int* J;
  int r0;
  const float2* xt;
  YT* y;
  __device__ const float2* zrow(int r) const { return Zl + (int64_t)r * q; }
  __device__ const float2* brow(int c) const { return xt + (int64_t)J[c] * R; }
  __device__ void store(int r, int j, float re, float im) const {
    typedef decltype(y->x) YS;
    YT* o = y + (int64_t)j * N + J[r0 + r];
    YT v;
    if (ACC) {
      v = *o;
      v.x += (YS)re;
      v.y += (YS)im;
    } else {
      v.x = (YS)re;
      v.y = (YS)im;
    }
    *o = v;
  }
};

template <typename YT, bool ACC>
__global__ void __launch_bounds__(64 * PA_NW) k_block_mfma(int N, int R, const int* __restrict__ items,
                                                    const int* __restrict__ jptr, const int* __restrict__ jidx,
                                                    const int* __restrict__ nb, const int64_t* __restrict__ zoff,
                                                    const float2* __restrict__ Z, const float2* __restrict__ xt,
                                                    YT* __restrict__ y) {
  const int sd = items[2 * blockIdx.x], r0 = items[2 * blockIdx.x + 1];
  const int j0 = jptr[sd], q = jptr[sd + 1] - j0;
  BlockOp<YT, ACC> op{min(PA_ROWS, nb[sd] - r0), q, N, R, Z + zoff[sd] + (int64_t)r0 * q, jidx + j0, r0, xt, y};
  block_mfma_body(op, R);
}

// xt[n][r] = x[r][n] as complex64 (32 x 32 tiles through LDS; block (32, 8)).
template <typename XT>
__global__ void __launch_bounds__(256) k_to_nr(int N, int R, const XT* __restrict__ x, float2* __restrict__ xt) {
  __shared__ float2 tile[32][33];
  const int n0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
  for (int k = threadIdx.y; k < 32; k += 8) {
    const int r = r0 + k, n = n0 + threadIdx.x;
    if (r < R && n < N) {
      const XT v = x[(int64_t)r * N + n];
      tile[k][threadIdx.x] = make_float2((float)v.x, (float)v.y);
    }
  }
  __syncthreads();
  for (int k = threadIdx.y; k < 32; k += 8) {
    const int n = n0 + k, r = r0 + threadIdx.x;
    if (n < N && r < R) xt[(int64_t)n * R + r] = tile[threadIdx.x][k];
  }
}
