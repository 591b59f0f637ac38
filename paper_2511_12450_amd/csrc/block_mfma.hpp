// Block-sparse complex products on matrix cores (preconditioner apply and
// near field, several right-hand sides).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

// Block-sparse products with matrix cores, for several right-hand sides:
// Y_B (rows x R) (=|+=) Z_B (rows x q) X_J (q x R) per work item of PA_ROWS
// rows of one block (a subdomain of the preconditioner, or a leaf box with
// its neighbours for the near field), as the real product
// [[Re Z, -Im Z], [Im Z, Re Z]] [Re X; Im X] in 16x16x4 FP32 MFMA tiles (FP32
// accumulation).  Z_B is row-major, complex64; the input is the complex64
// transpose xt [N][R] (k_to_nr), so a neighbourhood row of all right-hand
// sides is one contiguous load; y is [R][N] in YT (complex128 or complex64).
// K runs over the neighbourhood in chunks of PA_KC complex columns staged in
// LDS (Z chunk transposed to [j][r]).
typedef float pa_v4f __attribute__((ext_vector_type(4)));
constexpr int PA_ROWS = 64, PA_KC = 32, PA_NW = 8, PA_TPW = 32 / PA_NW;
template <typename YT, bool ACC>
__global__ void __launch_bounds__(64 * PA_NW) k_block_mfma(int N, int R, const int* __restrict__ items,
                                                    const int* __restrict__ jptr, const int* __restrict__ jidx,
                                                    const int* __restrict__ nb, const int64_t* __restrict__ zoff,
                                                    const float2* __restrict__ Z, const float2* __restrict__ xt,
                                                    YT* __restrict__ y) {
  __shared__ float2 Zs[PA_KC][PA_ROWS];
  __shared__ float2 Xs[PA_KC][64];
  const int sd = items[2 * blockIdx.x], r0 = items[2 * blockIdx.x + 1];
  const int j0_ = jptr[sd], q = jptr[sd + 1] - j0_;
  const int rows = min(PA_ROWS, nb[sd] - r0);
  const int* J = jidx + j0_;
  const float2* Zl = Z + zoff[sd] + (int64_t)r0 * q;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int l16 = lane & 15, kq = lane >> 4;
  const int R2 = 2 * rows, MT = (R2 + 15) / 16, NT = (R + 15) / 16, ntile = MT * NT;
  int mrow[PA_TPW], jcol[PA_TPW];
  bool ire[PA_TPW], ival[PA_TPW], jval[PA_TPW];
#pragma unroll
  for (int t = 0; t < PA_TPW; ++t) {
    const int tile = wv + PA_NW * t;
    const int i = 16 * (tile / NT) + l16, jj = 16 * (tile % NT) + l16;
    ival[t] = tile < ntile && i < R2;
    ire[t] = i < rows;
    mrow[t] = ival[t] ? (ire[t] ? i : i - rows) : 0;
    jval[t] = tile < ntile && jj < R;
    jcol[t] = jval[t] ? jj : 0;
  }
  pa_v4f acc[PA_TPW];
#pragma unroll
  for (int t = 0; t < PA_TPW; ++t) acc[t] = pa_v4f{0.f, 0.f, 0.f, 0.f};
  for (int c0 = 0; c0 < q; c0 += PA_KC) {
    const int kc = min(PA_KC, q - c0);
    __syncthreads();
    for (int idx = threadIdx.x; idx < PA_KC * PA_ROWS; idx += 64 * PA_NW) {
      const int rr = idx / PA_KC, jj = idx - rr * PA_KC;  // consecutive threads along a Z row
      Zs[jj][rr] = (rr < rows && jj < kc) ? Zl[(int64_t)rr * q + c0 + jj] : make_float2(0.f, 0.f);
    }
    for (int idx = threadIdx.x; idx < PA_KC * 64; idx += 64 * PA_NW) {
      const int jj = idx >> 6, rr = idx & 63;
      Xs[jj][rr] = (jj < kc && rr < R) ? xt[(int64_t)J[c0 + jj] * R + rr] : make_float2(0.f, 0.f);
    }
    __syncthreads();
#pragma unroll 1
    for (int ks = 0; ks < 2 * PA_KC / 4; ++ks) {
      const int k = 4 * ks + kq;
      const bool kre = k < PA_KC;
      const int n = kre ? k : k - PA_KC;
#pragma unroll
      for (int t = 0; t < PA_TPW; ++t) {
        if (wv + PA_NW * t < ntile) {  // wave-uniform
          const float2 zv = Zs[n][mrow[t]];
          const float2 xv = Xs[n][jcol[t]];
          const float av = ival[t] ? (ire[t] ? (kre ? zv.x : -zv.y) : (kre ? zv.y : zv.x)) : 0.f;
          const float bv = jval[t] ? (kre ? xv.x : xv.y) : 0.f;
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[t], 0, 0, 0);
        }
      }
    }
  }
  typedef decltype(y->x) YS;
  YS* yd = reinterpret_cast<YS*>(y);
#pragma unroll
  for (int t = 0; t < PA_TPW; ++t) {
    const int tile = wv + PA_NW * t;
    if (tile < ntile) {
      const int jj = 16 * (tile % NT) + l16;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * (tile / NT) + 4 * kq + v;
        if (i < R2 && jj < R) {
          const bool ir = i < rows;
          const int row = J[r0 + (ir ? i : i - rows)];
          YS* o = yd + 2 * ((int64_t)jj * N + row) + (ir ? 0 : 1);
          *o = ACC ? (YS)(*o + (YS)acc[t][v]) : (YS)acc[t][v];
        }
      }
    }
  }
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
