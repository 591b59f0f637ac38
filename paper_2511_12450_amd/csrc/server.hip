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
//   2. Arnoldi orthogonalisation by classical Gram-Schmidt with a delayed
//      second pass (each column with its own basis length): the vector u_j
//      sent through K M is orthogonalised once; at the next step one read of
//      the basis computes both V^H u_j (its re-orthogonalisation) and
//      V^H K M u_j, the Hessenberg column of step j-1 is corrected, and one
//      more read produces the re-orthogonalised v_j and the once-projected
//      next vector.  Two passes over the basis per step instead of four,
//      with the accuracy of two-pass CGS; the Hessenberg column (and the
//      residual estimate) lags one step.  Residual updates for columns that
//      restart or finish, and one device-to-host copy of the dot products
//      and norms per round;
//   3. Givens rotations and convergence tests on the host, then the batched
//      update pass and solution updates.
// The host waits once per round (for the dot products); everything else is
// queued behind it without waiting: round buffers that must grow are
// replaced by larger ones and the old ones freed at the next idle point, and
// finished columns copy phi and the far field to pinned staging memory, from
// which the host fills the requests' arrays while the next round runs.
// Requests that arrive while others run are admitted at the next round as
// soon as right-hand-side slots and the HBM budget allow; a request whose
// footprint can never fit is rejected at submission.  Admission, cancel,
// failure and release are the host-only scheduler of sched.hpp, driven here
// by the device work below.  Finished requests keep
// phi and the far field in host memory until released.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <complex>
#include <condition_variable>
#include <cstring>
#include <cstdlib>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "lm_internal.hpp"
#include "sched.hpp"

namespace {

typedef std::complex<double> C;
constexpr int SRV_STREAMS = 4;
// elements per workgroup in the dot kernel: 4096 for the complex64 basis
// (16 elements of each vector in flight per thread), 2048 for complex128
template <typename BT> constexpr int sd_slice() { return sizeof(BT) == 8 ? 4096 : 2048; }
constexpr int SD_IBLK = 64;  // basis vectors per LDS flush of the dot kernel
constexpr int SD_WGS = 1024;  // workgroups a dot launch aims for (split over the basis below that)

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Per-column operands of the batched kernels.  The Krylov basis is stored
// in BT (complex128, or complex64 for the mixed form: half the Gram-Schmidt
// traffic; every dot product and update is still accumulated in FP64); all
// other vectors are complex128.
struct ColDev {
  void* V;            // basis [m+1][N] in BT
  double2* w;         // K M output / residual vector
  const double2* g;   // right-hand side (residual form), or null
  const double2* src; // copy / scale source
  double2* dst;       // gather destination (K M input slot), or null
  double2* z;         // solution accumulator
  const double2* y;   // combination / update coefficients
  const double* nsrc; // squared norm to normalise by (device), or null
  double* ndst;       // squared norm output (device), or null
  double2 dr;         // complex scalar of the update pass
  double scale;
  int N, cnt;
  int vj;             // gather: basis vector to normalise, or -1 (gather w)
  int ld;             // basis stride (elements; a multiple of 64, so pairs are 16-byte aligned)
};

__device__ __forceinline__ double2 bld(const double2* p) { return *p; }
__device__ __forceinline__ double2 bld(const float2* p) {
  const float2 v = *p;
  return make_double2((double)v.x, (double)v.y);
}
__device__ __forceinline__ double2 bcv(double2 v) { return v; }
__device__ __forceinline__ double2 bcv(float2 v) { return make_double2((double)v.x, (double)v.y); }
__device__ __forceinline__ void bst(double2* p, double2 v) { *p = v; }
__device__ __forceinline__ void bst(float2* p, double2 v) { *p = make_float2((float)v.x, (float)v.y); }
// two consecutive basis elements from an even position (one 16-byte load for complex64)
__device__ __forceinline__ void bld2(const double2* p, double2& a, double2& b) {
  a = p[0];
  b = p[1];
}
__device__ __forceinline__ void bld2(const float2* p, double2& a, double2& b) {
  const float4 v = *reinterpret_cast<const float4*>(p);
  a = make_double2((double)v.x, (double)v.y);
  b = make_double2((double)v.z, (double)v.w);
}
__device__ __forceinline__ void bst2(double2* p, double2 a, double2 b) {
  p[0] = a;
  p[1] = b;
}
__device__ __forceinline__ void bst2(float2* p, double2 a, double2 b) {
  *reinterpret_cast<float4*>(p) = make_float4((float)a.x, (float)a.y, (float)b.x, (float)b.y);
}

// V[0] = src * scale      (grid (ceil(Nmax / 256), ncols))
template <typename BT>
__global__ void __launch_bounds__(256) k_s_copy(const ColDev* __restrict__ d) {
  const ColDev c = d[blockIdx.y];
  const int n = blockIdx.x * 256 + threadIdx.x;
  if (n >= c.N) return;
  const double2 v = c.src[n];
  bst((BT*)c.V + n, make_double2(v.x * c.scale, v.y * c.scale));
}

__device__ __forceinline__ double s_wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// w = g - w when g is set; wave partials of |w|^2 into part[col nw + wave].
// Columns whose norm an earlier pass left (nsrc) are skipped: k_s_norm_final
// reports that one.
__global__ void __launch_bounds__(256) k_s_resid(const ColDev* __restrict__ d, double* __restrict__ part, int nw) {
  const ColDev c = d[blockIdx.y];
  const int n = blockIdx.x * 256 + threadIdx.x;
  if (blockIdx.x * 256 >= c.N || !c.w || c.nsrc) return;  // beyond this column, or nothing to do
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

// nrm[col] = sum of the column's wave partials (4 per 256 elements), or the
// norm an earlier pass left at nsrc.
__global__ void __launch_bounds__(64) k_s_norm_final(const ColDev* __restrict__ d, const double* __restrict__ part,
                                                     int nw, double* __restrict__ nrm) {
  const ColDev c = d[blockIdx.x];
  if (c.nsrc) {  // a norm computed by an earlier pass
    if (threadIdx.x == 0) nrm[blockIdx.x] = *c.nsrc;
    return;
  }
  const int nwc = 4 * ((c.N + 255) / 256);
  double q = 0.0;
  for (int k = threadIdx.x; k < nwc; k += 64) q += part[(int64_t)blockIdx.x * nw + k];
  q = s_wave_sum(q);
  if (threadIdx.x == 0) nrm[blockIdx.x] = q;
}

// z += sum_{i < cnt} V[i] y[i]: two consecutive elements per thread (one
// 16-byte load per basis vector for complex64), the coefficients staged in
// LDS 256 at a time as in the update pass (grid (ceil(Nmax / 512), ncols)).
template <typename BT>
__global__ void __launch_bounds__(256) k_s_lincomb(const ColDev* __restrict__ d) {
  const ColDev c = d[blockIdx.y];
  if (blockIdx.x * 512 >= c.N) return;  // uniform per workgroup
  __shared__ double2 cy[256];
  const int n = 2 * (blockIdx.x * 256 + threadIdx.x);
  const bool ok0 = n < c.N, ok1 = n + 1 < c.N;
  const int o = ok0 ? n : 0;
  const BT* V = (const BT*)c.V;
  double2 acc[2] = {ok0 ? c.z[o] : make_double2(0.0, 0.0), ok1 ? c.z[o + 1] : make_double2(0.0, 0.0)};
  for (int ic = 0; ic < c.cnt; ic += 256) {
    const int ie = min(c.cnt, ic + 256);
    if (ic > 0) __syncthreads();  // the previous chunk's coefficients are read
    for (int t = ic + (int)threadIdx.x; t < ie; t += 256) cy[t - ic] = c.y[t];
    __syncthreads();
#pragma unroll 4
    for (int i = ic; i < ie; ++i) {
      double2 v[2];
      bld2(V + (int64_t)i * c.ld + o, v[0], v[1]);  // basis padding past an odd N is allocated
      const double2 a = cy[i - ic];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        acc[h].x = fma(a.x, v[h].x, acc[h].x);
        acc[h].x = fma(-a.y, v[h].y, acc[h].x);
        acc[h].y = fma(a.x, v[h].y, acc[h].y);
        acc[h].y = fma(a.y, v[h].x, acc[h].y);
      }
    }
  }
  if (ok0) c.z[o] = acc[0];
  if (ok1) c.z[o + 1] = acc[1];
}

// Gathers the K M inputs of Arnoldi columns and normalises lagged basis
// vectors: v = V[vj] * s with s = 1/sqrt(*nsrc) (written back to V[vj]), or
// v = w * scale (vj < 0); dst (the fused launch's input slot) may be null.
template <typename BT>
__global__ void __launch_bounds__(256) k_s_gather(const ColDev* __restrict__ d) {
  const ColDev c = d[blockIdx.y];
  const int n = blockIdx.x * 256 + threadIdx.x;
  if (n >= c.N) return;
  double2 v;
  if (c.vj >= 0) {
    BT* vp = (BT*)c.V + (int64_t)c.vj * c.ld + n;
    const double s = c.nsrc ? 1.0 / sqrt(*c.nsrc) : c.scale;
    v = bld(vp);
    v = make_double2(v.x * s, v.y * s);
    if (c.nsrc) bst(vp, v);
  } else {
    v = c.w[n];
    v = make_double2(v.x * c.scale, v.y * c.scale);
  }
  if (c.dst) c.dst[n] = v;
}

// Two consecutive basis elements of one vector, as loaded (converted to
// FP64 when used): the next pair of vectors is loaded while this one is
// reduced.
template <typename BT> struct BPair;
template <> struct BPair<float2> {
  float4 v;
  __device__ void load(const float2* p) { v = *reinterpret_cast<const float4*>(p); }
  __device__ void get(double2& a, double2& b) const {
    a = make_double2((double)v.x, (double)v.y);
    b = make_double2((double)v.z, (double)v.w);
  }
};
template <> struct BPair<double2> {
  double2 x, y;
  __device__ void load(const double2* p) {
    x = p[0];
    y = p[1];
  }
  __device__ void get(double2& a, double2& b) const {
    a = x;
    b = y;
  }
};

// Workgroup partials of conj(V[i]) . u and conj(V[i]) . z, u = V[cnt-1],
// z = the K M output (or none), for basis vectors [z blk, (z+1) blk) of the
// column (grid (ceil(Nmax / slice), ncols, nz)).  Each thread takes EP pairs
// of consecutive elements of a slice; u and z stay in registers while the
// block's vectors stream past, two per step with the next two in flight.
// Partials go through LDS, flushed every SD_IBLK vectors.
template <typename BT>
__global__ void __launch_bounds__(256) k_s_dots2(const ColDev* __restrict__ d, double2* __restrict__ pa,
                                                 double2* __restrict__ pb, int ldh, int nb, int blk) {
  constexpr int SL = sd_slice<BT>();
  const ColDev c = d[blockIdx.y];
  const int ib = blockIdx.z * blk;
  if (ib >= c.cnt || blockIdx.x * SL >= c.N) return;  // uniform per workgroup
  const int ie = min(c.cnt, ib + blk);
  constexpr int EP = SL / 512;  // pairs per thread
  const BT* V = (const BT*)c.V;
  const BT* u = V + (int64_t)(c.cnt - 1) * c.ld;
  double2 xu[2 * EP], xz[2 * EP];
  int idx[EP];
  bool ok[2 * EP];
#pragma unroll
  for (int e = 0; e < EP; ++e) {
    const int n = blockIdx.x * SL + 2 * (threadIdx.x + 256 * e);
    ok[2 * e] = n < c.N;
    ok[2 * e + 1] = n + 1 < c.N;
    idx[e] = ok[2 * e] ? n : 0;
    bld2(u + idx[e], xu[2 * e], xu[2 * e + 1]);
    xz[2 * e] = (ok[2 * e] && c.w) ? c.w[idx[e]] : make_double2(0.0, 0.0);
    xz[2 * e + 1] = (ok[2 * e + 1] && c.w) ? c.w[idx[e] + 1] : make_double2(0.0, 0.0);
#pragma unroll
    for (int h = 0; h < 2; ++h)
      if (!ok[2 * e + h]) xu[2 * e + h] = make_double2(0.0, 0.0);
  }
  // the eight sums of a step (re / im of V^H u and V^H z for each of two
  // vectors) are reduced over the wavefront by a transposing butterfly
  // (after the xor-32, -16 and -8 steps lane l holds sum number l / 8 of its
  // lane group, then three plain steps finish it); the per-wave results of
  // the whole block meet in LDS
  __shared__ double red[SD_IBLK][4][4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  BPair<BT> n0[EP], n1[EP];
  {
    const BT* v0 = V + (int64_t)ib * c.ld;
    const BT* v1 = V + (int64_t)min(ib + 1, ie - 1) * c.ld;
#pragma unroll
    for (int e = 0; e < EP; ++e) {
      n0[e].load(v0 + idx[e]);
      n1[e].load(v1 + idx[e]);
    }
  }
#pragma unroll 1
  for (int i = ib; i < ie; i += 2) {
    const bool two = i + 1 < ie;
    BPair<BT> c0[EP], c1[EP];
#pragma unroll
    for (int e = 0; e < EP; ++e) {
      c0[e] = n0[e];
      c1[e] = n1[e];
    }
    if (i + 2 < ie) {
      const BT* v0 = V + (int64_t)(i + 2) * c.ld;
      const BT* v1 = V + (int64_t)min(i + 3, ie - 1) * c.ld;
#pragma unroll
      for (int e = 0; e < EP; ++e) {
        n0[e].load(v0 + idx[e]);
        n1[e].load(v1 + idx[e]);
      }
    }
    double t[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int e = 0; e < EP; ++e) {
      double2 a0[2], a1[2];
      c0[e].get(a0[0], a0[1]);
      c1[e].get(a1[0], a1[1]);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int k = 2 * e + h;
        const double2 p0 = ok[k] ? a0[h] : make_double2(0.0, 0.0);
        const double2 p1 = (ok[k] && two) ? a1[h] : make_double2(0.0, 0.0);
        t[0] = fma(p0.x, xu[k].x, fma(p0.y, xu[k].y, t[0]));
        t[1] = fma(p0.x, xu[k].y, fma(-p0.y, xu[k].x, t[1]));
        t[2] = fma(p0.x, xz[k].x, fma(p0.y, xz[k].y, t[2]));
        t[3] = fma(p0.x, xz[k].y, fma(-p0.y, xz[k].x, t[3]));
        t[4] = fma(p1.x, xu[k].x, fma(p1.y, xu[k].y, t[4]));
        t[5] = fma(p1.x, xu[k].y, fma(-p1.y, xu[k].x, t[5]));
        t[6] = fma(p1.x, xz[k].x, fma(p1.y, xz[k].y, t[6]));
        t[7] = fma(p1.x, xz[k].y, fma(-p1.y, xz[k].x, t[7]));
      }
    }
    // 8 -> 4 -> 2 -> 1 values per lane (lanes with the step's bit set keep the upper half)
#pragma unroll
    for (int h = 4, o = 32; h >= 1; h >>= 1, o >>= 1) {
      const bool up = (lane & o) != 0;
#pragma unroll
      for (int k = 0; k < h; ++k) {
        const double send = up ? t[k] : t[k + h];
        const double keep = up ? t[k + h] : t[k];
        t[k] = keep + __shfl_xor(send, o, 64);
      }
    }
    double r = t[0];
    r += __shfl_xor(r, 4, 64);
    r += __shfl_xor(r, 2, 64);
    r += __shfl_xor(r, 1, 64);
    const int q = lane >> 3;  // sum number: vector q / 4, component q % 4
    const int slot = (i - ib) % SD_IBLK;  // i - ib is even: both vectors in one chunk
    if ((lane & 7) == 0 && (q < 4 || two)) red[slot + (q >> 2)][wv][q & 3] = r;
    if (slot + 2 == SD_IBLK || i + 2 >= ie) {  // chunk full or block done (uniform)
      __syncthreads();
      const int i0 = i - slot, cn = min(ie, i0 + SD_IBLK) - i0;
      for (int t = threadIdx.x; t < cn; t += 256) {
        const double(*rr)[4] = red[t];
        const int64_t o = ((int64_t)blockIdx.y * ldh + i0 + t) * nb + blockIdx.x;
        pa[o] = make_double2((rr[0][0] + rr[1][0]) + (rr[2][0] + rr[3][0]),
                             (rr[0][1] + rr[1][1]) + (rr[2][1] + rr[3][1]));
        pb[o] = make_double2((rr[0][2] + rr[1][2]) + (rr[2][2] + rr[3][2]),
                             (rr[0][3] + rr[1][3]) + (rr[2][3] + rr[3][3]));
      }
      __syncthreads();
    }
  }
}

// h[col hs + i] = sum of a-partials, h[col hs + ldh + i] = sum of b-partials.
__global__ void __launch_bounds__(64) k_s_dots2_final(const ColDev* __restrict__ d, const double2* __restrict__ pa,
                                                      const double2* __restrict__ pb, int ldh, int nb, int slice,
                                                      double2* __restrict__ h, int hs) {
  const ColDev c = d[blockIdx.y];
  const int i = blockIdx.x;
  if (i >= c.cnt) return;
  const int nbc = (c.N + slice - 1) / slice;
  double ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0;
  for (int k = threadIdx.x; k < nbc; k += 64) {
    const int64_t o = ((int64_t)blockIdx.y * ldh + i) * nb + k;
    ar += pa[o].x;
    ai += pa[o].y;
    br += pb[o].x;
    bi += pb[o].y;
  }
  ar = s_wave_sum(ar);
  ai = s_wave_sum(ai);
  br = s_wave_sum(br);
  bi = s_wave_sum(bi);
  if (threadIdx.x == 0) {
    h[(int64_t)blockIdx.y * hs + i] = make_double2(ar, ai);
    h[(int64_t)blockIdx.y * hs + ldh + i] = make_double2(br, bi);
  }
}

// One read of the basis V[0..cnt-1] (cnt = j) produces
//   V[j]   <- (u - sum_i a_i V[i]) * scale                (re-orthogonalised v_j)
//   V[j+1] <- z * scale - u * dr - sum_i e_i V[i]          (once-projected next vector)
// with u = V[j], z = the K M output, a = y[0..j), e = y[j..2j); wave
// partials of |V[j+1]|^2 into part.  Each thread takes two consecutive
// elements (SU_ELEM per workgroup); the element past N of an odd N is basis
// padding and is left out of the norm.  The coefficients of SU_CH basis
// vectors at a time are staged in LDS: read from there, the loop over the
// basis keeps more loads in flight than with a global load per coefficient
// (5.6 against 4.7 TB/s at j = 128 over 64 columns).
constexpr int SU_ELEM = 512;
constexpr int SU_CH = 256;
template <typename BT>
__global__ void __launch_bounds__(256) k_s_update2(const ColDev* __restrict__ d, double* __restrict__ part, int nw) {
  const ColDev c = d[blockIdx.y];
  if (blockIdx.x * SU_ELEM >= c.N) return;
  __shared__ double2 cy[2][SU_CH];  // a_i, e_i of the current chunk
  const int n = 2 * (blockIdx.x * 256 + threadIdx.x);
  const bool ok0 = n < c.N, ok1 = n + 1 < c.N;
  const int o = ok0 ? n : 0;
  const int j = c.cnt;
  BT* V = (BT*)c.V;
  BT* uj = V + (int64_t)j * c.ld;
  double2 u[2], q[2], w[2];
  bld2(uj + o, u[0], u[1]);
  const double2 zv[2] = {c.w[o], ok1 ? c.w[o + 1] : make_double2(0.0, 0.0)};
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    q[h] = u[h];
    w[h] = make_double2(zv[h].x * c.scale - (u[h].x * c.dr.x - u[h].y * c.dr.y),
                        zv[h].y * c.scale - (u[h].x * c.dr.y + u[h].y * c.dr.x));
  }
  constexpr int U = 4;
  for (int ic = 0; ic < j; ic += SU_CH) {
    const int ie = min(j, ic + SU_CH);
    if (ic > 0) __syncthreads();  // the previous chunk's coefficients are read
    for (int t = ic + (int)threadIdx.x; t < ie; t += 256) {
      cy[0][t - ic] = c.y[t];
      cy[1][t - ic] = c.y[j + t];
    }
    __syncthreads();
    for (int i0 = ic; i0 < ie; i0 += U) {
      double2 v[U][2];
#pragma unroll
      for (int k = 0; k < U; ++k) {
        if (i0 + k < ie) {
          bld2(V + (int64_t)(i0 + k) * c.ld + o, v[k][0], v[k][1]);
        } else {
          v[k][0] = v[k][1] = make_double2(0.0, 0.0);
        }
      }
#pragma unroll
      for (int k = 0; k < U; ++k) {
        if (i0 + k < ie) {
          const double2 a = cy[0][i0 + k - ic], e = cy[1][i0 + k - ic];
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            q[h].x = fma(-a.x, v[k][h].x, q[h].x);
            q[h].x = fma(a.y, v[k][h].y, q[h].x);
            q[h].y = fma(-a.x, v[k][h].y, q[h].y);
            q[h].y = fma(-a.y, v[k][h].x, q[h].y);
            w[h].x = fma(-e.x, v[k][h].x, w[h].x);
            w[h].x = fma(e.y, v[k][h].y, w[h].x);
            w[h].y = fma(-e.x, v[k][h].y, w[h].y);
            w[h].y = fma(-e.y, v[k][h].x, w[h].y);
          }
        }
      }
    }
  }
  if (ok0) {
    bst2(uj + o, make_double2(q[0].x * c.scale, q[0].y * c.scale), make_double2(q[1].x * c.scale, q[1].y * c.scale));
    bst2(uj + c.ld + o, w[0], w[1]);
  }
  const double qn = s_wave_sum((ok0 ? w[0].x * w[0].x + w[0].y * w[0].y : 0.0) +
                               (ok1 ? w[1].x * w[1].x + w[1].y * w[1].y : 0.0));
  if ((threadIdx.x & 63) == 0) part[(int64_t)blockIdx.y * nw + blockIdx.x * 4 + (threadIdx.x >> 6)] = qn;
}

// *ndst = sum of the column's wave partials (4 per SU_ELEM elements).
__global__ void __launch_bounds__(64) k_s_norm_to(const ColDev* __restrict__ d, const double* __restrict__ part,
                                                  int nw) {
  const ColDev c = d[blockIdx.x];
  const int nwc = 4 * ((c.N + SU_ELEM - 1) / SU_ELEM);
  double q = 0.0;
  for (int k = threadIdx.x; k < nwc; k += 64) q += part[(int64_t)blockIdx.x * nw + k];
  q = s_wave_sum(q);
  if (threadIdx.x == 0) *c.ndst = q;
}

// PH_STAGED: solved; phi and the far field are being copied to pinned host
// memory, and the column is marked finished once those copies are done.
enum Phase { PH_INIT = 0, PH_ARNOLDI = 1, PH_RESTART = 2, PH_FINAL = 3, PH_STAGED = 4 };

struct Request;

struct Column {
  Request* req = nullptr;
  int col = 0;
  lm_geom_s* g = nullptr;
  int N = 0, m = 0;
  int ldv = 0;  // basis stride: N rounded up to a multiple of 64
  Phase phase = PH_INIT;
  DevBuf V, z, gv, y, dn;  // dn: squared norm of the once-projected next vector
  int j = 0, its = 0, ncols = 0;
  double gnorm = 0.0, res = 1.0;
  bool converged = false, finished = false;
  bool km = false;        // needs K M this round
  std::vector<C> H, Hraw, cs, sn, e1, cprev;  // rotated / raw Hessenberg, provisional column
  double2* w = nullptr;  // this round's vector (group output slice or gv)
  void reset() {  // solver state of a fresh column (device buffers are kept)
    phase = PH_INIT;
    j = its = ncols = 0;
    gnorm = 0.0;
    res = 1.0;
    converged = finished = km = false;
    w = nullptr;
  }
};

struct Request {
  uint64_t id = 0;
  lm_geom_s* g = nullptr;
  int R = 0;
  std::vector<double> theta, obs;
  lm_gmres_opts o{};
  lm_state state = LM_QUEUED;
  lm_status status = LM_OK, fail_status = LM_OK;  // fail_status: a failure pending until the worker lets go
  std::string err;
  std::vector<lm_solve_report> rep;
  // phi: R x N, malloc'd without touching it (a zero-filled vector costs a
  // page fault and a fill per 4 KiB on the submitting thread); every column's
  // slice is written before the request is done
  struct FreeHost {
    void operator()(double2* p) const { std::free(p); }
  };
  std::unique_ptr<double2, FreeHost> phi;
  size_t phi_n = 0;
  std::vector<double2> ff;
  int cols_left = 0;
  bool cancel = false;
  double t_submit = 0.0, t_done = 0.0;
  int64_t bytes = 0;
};

struct Group {
  DevBuf X, Y;
  KmBufs km;
};

// Pinned host staging (hipHostMalloc) for the per-round copies, grown on demand.
struct HostBuf {
  void* p = nullptr;
  size_t bytes = 0;
  HostBuf() = default;
  HostBuf(const HostBuf&) = delete;
  HostBuf& operator=(const HostBuf&) = delete;
  ~HostBuf() {
    if (p) (void)hipHostFree(p);
  }
  template <typename T> T* as() const { return static_cast<T*>(p); }
};

// One column's host update of a round: descriptors and coefficients with
// offsets local to this column (rebased when the columns are merged).
struct HostStep {
  std::vector<ColDev> scal, comb, upd;
  std::vector<double2> ys, cf;
  std::vector<Column*> to_finish;
  double gsb = 0.0;
  void clear() {
    scal.clear();
    comb.clear();
    upd.clear();
    ys.clear();
    cf.clear();
    to_finish.clear();
    gsb = 0.0;
  }
};

// A few persistent host threads for per-column work: run(n, f) calls f(i)
// for i in [0, n) on the pool and the calling thread and returns when all
// are done.
class HostPool {
 public:
  explicit HostPool(int n) : nt_(std::max(1, n)) {
    for (int t = 1; t < nt_; ++t) th_.emplace_back([this] { loop(); });
  }
  ~HostPool() {
    stop_.store(true, std::memory_order_release);
    {
      std::lock_guard<std::mutex> lk(m_);
      gen_.fetch_add(1, std::memory_order_release);
    }
    cv_.notify_all();
    for (auto& t : th_) t.join();
  }
  void run(int n, const std::function<void(int)>& f) {
    if (nt_ == 1 || n < 4) {
      for (int i = 0; i < n; ++i) f(i);
      return;
    }
    f_ = &f;
    n_ = n;
    next_.store(0, std::memory_order_relaxed);
    busy_.store(nt_ - 1, std::memory_order_relaxed);
    {  // under the lock, so that a worker going to sleep cannot miss it
      std::lock_guard<std::mutex> lk(m_);
      gen_.fetch_add(1, std::memory_order_release);
    }
    cv_.notify_all();
    work();
    // the workers end within microseconds of the last item
    while (busy_.load(std::memory_order_acquire) != 0) std::this_thread::yield();
  }
  // A run() follows within milliseconds: sleeping workers wake now and poll
  // (up to kArmSpin), so that the run does not wait for their wake-up.
  void arm() {
    if (nt_ == 1) return;
    {
      std::lock_guard<std::mutex> lk(m_);
      arm_.fetch_add(1, std::memory_order_release);
    }
    cv_.notify_all();
  }

 private:
  void work() {
    for (int i = next_.fetch_add(1); i < n_; i = next_.fetch_add(1)) (*f_)(i);
  }
  // Waits for the next generation: polls for up to kSpin after a run and up
  // to kArmSpin after an arm(), then sleeps until either comes.
  void loop() {
    constexpr auto kSpin = std::chrono::microseconds(200), kArmSpin = std::chrono::microseconds(20000);
    uint64_t seen = 0, seen_arm = arm_.load(std::memory_order_acquire);
    auto limit = kSpin;
    while (true) {
      auto t0 = std::chrono::steady_clock::now();
      uint64_t g;
      while ((g = gen_.load(std::memory_order_acquire)) == seen) {
        const uint64_t a = arm_.load(std::memory_order_acquire);
        if (a != seen_arm) {
          seen_arm = a;
          t0 = std::chrono::steady_clock::now();
          limit = kArmSpin;
        }
        if (std::chrono::steady_clock::now() - t0 < limit) {
          std::this_thread::yield();
          continue;
        }
        std::unique_lock<std::mutex> lk(m_);
        cv_.wait(lk, [&] {
          return gen_.load(std::memory_order_acquire) != seen || arm_.load(std::memory_order_acquire) != seen_arm;
        });
      }
      limit = kSpin;
      seen = g;
      if (stop_.load(std::memory_order_acquire)) return;
      work();
      busy_.fetch_sub(1, std::memory_order_release);
    }
  }
  int nt_;
  std::vector<std::thread> th_;
  std::mutex m_;
  std::condition_variable cv_;
  const std::function<void(int)>* f_ = nullptr;
  int n_ = 0;
  std::atomic<int> next_{0}, busy_{0};
  std::atomic<uint64_t> gen_{0}, arm_{0};
  std::atomic<bool> stop_{false};
};

}  // namespace

struct lm_server_s {
  lm_server_opts o{};
  int device = 0;
  lmsched::Book<Request> B;  // requests, queue, admission counters and the lock over them
  std::thread th;
  int64_t held = 0, held_spare = 0;  // device bytes of the server's own buffers (all / spare columns), worker-updated
  int64_t rounds = 0, launches = 0, fused_rhs = 0;
  double km_ms = 0.0, gs_ms = 0.0, gs_bytes = 0.0;  // phase times (HIP events) and Gram-Schmidt algorithmic bytes
  double m2l_ms = 0.0, m2l_flops = 0.0;              // M2L launches of the fused matvecs (HIP events)
  double round_ms = 0.0, finish_ms = 0.0;            // host wall time of rounds / of finishing columns
  double launch_ms = 0.0, wait_ms = 0.0, step_ms = 0.0;  // host wall time: queueing a round, its wait, the host step
  int64_t m2l_launches = 0;
  hipEvent_t t0 = nullptr, t1 = nullptr, t2 = nullptr;
  hipEvent_t tu1 = nullptr, tu2 = nullptr;  // update pass of the last round, read after the next wait
  hipEvent_t ev_wait = nullptr;             // end of a round's copies to the host (polled)
  bool tu_pending = false;
  hipEvent_t sev[SRV_STREAMS][16] = {};
  // worker state
  std::vector<Column*> cols;
  std::vector<Column*> spare;  // finished columns that keep their device buffers
  std::map<std::pair<lm_geom_s*, int>, Group> groups;
  std::map<lm_geom_s*, int> stream_of;
  hipStream_t s = nullptr;
  hipStream_t gs[SRV_STREAMS] = {};
  hipEvent_t ev_main = nullptr;
  hipEvent_t ev[SRV_STREAMS] = {};
  // descriptors of a round's kernels (gather, dot products, updates), each
  // with its own device buffer and pinned staging buffer
  // d_desc: descriptors of the gather and the dot products; d_hn: Hessenberg
  // dot products then norms; d_desc_u: update descriptors then coefficients.
  // Each goes through one pinned buffer and one copy per round.
  DevBuf d_desc, d_desc_u, d_hn, d_dpart, d_npart;
  HostBuf h_desc, h_desc_u, h_hn;
  DevBuf d_fz, d_fphi, d_fff;  // finishing columns: z, phi = M z, far fields
  DevBuf d_fobs, d_adm;        // far-field angles; admission: right-hand-side scratch, then angles
  // finishing columns whose phi / far field copies into h_fin are queued
  // (behind ev_fin); their requests' host arrays are filled once it fires
  struct Staged {
    Column* c;
    size_t phi_off, ff_off;  // byte offsets into h_fin
    int no;                  // far-field angles
  };
  std::vector<Staged> staged;
  HostBuf h_fin;
  hipEvent_t ev_fin = nullptr;
  // allocations replaced by larger ones while queued work may still use
  // them: freed at the next point where the streams are idle (quiesce)
  std::vector<void*> retired, retired_host;
  int64_t retired_bytes = 0;
  std::unique_ptr<HostPool> pool;  // per-column host updates
  std::vector<HostStep> steps;
  std::vector<ColDev> hdesc;
};

namespace {

int64_t footprint(const lm_geom_s* g, const lm_gmres_opts& o, int R) {
  const int64_t N = g->N;
  const int m = std::max(1, std::min(o.restart, o.max_iter));
  const int64_t ld = (N + 63) / 64 * 64;  // basis stride
  const int64_t per = (int64_t)(m + 1) * ld * 16 + (int64_t)(2 + 3) * N * 16 + (int64_t)(m + 1) * 16 + 2 * N * 8 +
                      (g->fmm ? fmm_ws_per_rhs(g->fmm) : 0);
  return per * R;
}

// Waits for everything queued on the server's streams (the side streams of
// the fused launches join the main stream every round), before device
// buffers that queued kernels may still use are freed or regrown.
void free_retired(lm_server_s* S) {
  for (void* p : S->retired) (void)hipFree(p);
  for (void* p : S->retired_host) (void)hipHostFree(p);
  S->retired.clear();
  S->retired_host.clear();
  S->retired_bytes = 0;
}

lm_status quiesce(lm_server_s* S) {
  LM_TRY_HIP(hipStreamSynchronize(S->s));
  free_retired(S);
  return LM_OK;
}

// Grows a round buffer without waiting for the kernels queued on it: the old
// allocation is retired (freed at the next quiesce) and the new one is at
// least twice as large, so that buffers growing by a row each round (the
// dot products of a lengthening basis) are reallocated O(log j) times and
// the host keeps queueing ahead of the GPU.
lm_status ensure(lm_server_s* S, DevBuf& b, size_t bytes) {
  if (b.bytes >= bytes) return LM_OK;
  const size_t n = b.p ? std::max(bytes, 2 * b.bytes) : bytes;
  if (b.p) {
    S->retired.push_back(b.p);
    S->retired_bytes += (int64_t)b.bytes;
    b.p = nullptr;
    b.bytes = 0;
  }
  LM_TRY(b.alloc(n));
  return LM_OK;
}

lm_status host_ensure(lm_server_s* S, HostBuf& h, size_t bytes) {
  if (h.bytes >= bytes) return LM_OK;
  if (h.p) {  // a copy from the old buffer may be queued
    S->retired_host.push_back(h.p);
    h.p = nullptr;
    h.bytes = 0;
  }
  const size_t n = std::max<size_t>(2 * bytes, 4096);
  LM_TRY_HIP(hipHostMalloc(&h.p, n, hipHostMallocDefault));
  h.bytes = n;
  return LM_OK;
}

// Queues the copy of n bytes from src to device buffer d through the pinned
// buffer h, without waiting.  Each staging buffer is written once per round,
// after the round's wait, or before it when the previous round's copy from it
// preceded that round's wait; so no queued copy still reads it.
lm_status upload_async(lm_server_s* S, HostBuf& h, DevBuf& d, const void* src, size_t n) {
  LM_TRY(host_ensure(S, h, n));
  LM_TRY(ensure(S, d, std::max<size_t>(n, 64 * sizeof(ColDev))));
  std::memcpy(h.p, src, n);
  LM_TRY_HIP(hipMemcpyAsync(d.p, h.p, n, hipMemcpyHostToDevice, S->s));
  return LM_OK;
}

// Adds the time of the last update pass to the phase times once its events
// are complete (called after a wait that covers them).
lm_status collect_update_time(lm_server_s* S) {
  if (!S->tu_pending) return LM_OK;
  float t = 0.f;
  LM_TRY_HIP(hipEventSynchronize(S->tu2));
  LM_TRY_HIP(hipEventElapsedTime(&t, S->tu1, S->tu2));
  S->tu_pending = false;
  std::lock_guard<std::mutex> lk(S->B.mu);
  S->gs_ms += t;
  return LM_OK;
}

// Precision of the preconditioner apply: the server's, or the FP64 rows when
// asked for.
int pre_precision(const lm_server_s* S) { return S->o.precond_fp64 ? LM_FP64 : S->o.precision; }

// Bytes per element of a column's Krylov basis.
size_t basis_bytes(const lm_server_s* S) { return S->o.precision == LM_MIXED ? sizeof(float2) : sizeof(double2); }

// Allocate the columns of an admitted request and compute its right-hand sides.
void drop_spares(lm_server_s* S) {
  if (!S->spare.empty()) (void)quiesce(S);
  for (Column* c : S->spare) delete c;
  S->spare.clear();
}

int64_t col_bytes(const Column* c) { return (int64_t)(c->V.bytes + c->z.bytes + c->gv.bytes + c->y.bytes + c->dn.bytes); }

bool group_live(const lm_server_s* S, const std::pair<lm_geom_s*, int>& key) {
  for (const Column* c : S->cols)
    if (c->g == key.first && c->req && (c->req->o.precond ? 1 : 0) == key.second) return true;
  return false;
}

int64_t group_bytes(const Group& G) {
  return (int64_t)(G.X.bytes + G.Y.bytes + G.km.x32.bytes + G.km.y32.bytes + G.km.mz.bytes);
}

// Frees the fused-launch buffers of the groups that no admitted column uses
// and `drop` selects, waiting first for queued kernels that may use them.
template <typename F> void drop_groups(lm_server_s* S, F drop) {
  bool synced = false;
  for (auto it = S->groups.begin(); it != S->groups.end();) {
    if (group_live(S, it->first) || !drop(it->first)) {
      ++it;
      continue;
    }
    if (!synced) (void)quiesce(S);
    synced = true;
    it = S->groups.erase(it);
  }
}

// Before admitting: the fused-launch buffers kept from an idle period stay
// only for the admitted requests' (geometry, preconditioner) groups and only
// if they fit beside the spare columns in what the budget leaves (`allow`);
// then spare columns are freed until they hold at most `allow` bytes: first
// those no admitted request can reuse (another N or restart length), oldest
// first.
void trim_spares(lm_server_s* S, int64_t allow, const std::vector<Request*>& admit) {
  auto wanted = [&](const std::pair<lm_geom_s*, int>& key) {
    for (const Request* q : admit)
      if (q->g == key.first && (q->o.precond ? 1 : 0) == key.second) return true;
    return false;
  };
  drop_groups(S, [&](const std::pair<lm_geom_s*, int>& key) { return !wanted(key); });
  int64_t sb = 0, kept = 0;
  for (Column* c : S->spare) sb += col_bytes(c);
  for (const auto& kv : S->groups)
    if (!group_live(S, kv.first)) kept += group_bytes(kv.second);
  if (sb + kept > allow) {
    drop_groups(S, [](const std::pair<lm_geom_s*, int>&) { return true; });
    kept = 0;
  }
  auto reusable = [&](const Column* c) {
    for (const Request* q : admit)
      if (q->g->N == c->N && std::max(1, std::min(q->o.restart, q->o.max_iter)) == c->m) return true;
    return false;
  };
  if (sb > allow) (void)quiesce(S);
  for (int pass = 0; pass < 2 && sb > allow; ++pass)
    for (auto it = S->spare.begin(); it != S->spare.end() && sb > allow;) {
      if (pass == 0 && reusable(*it)) {
        ++it;
        continue;
      }
      sb -= col_bytes(*it);
      delete *it;
      it = S->spare.erase(it);
    }
}

// Records the device bytes the server holds (all / spare columns).
void record_held(lm_server_s* S) {
  int64_t h = 0, hs = 0;
  for (const Column* c : S->cols) h += col_bytes(c);
  for (const Column* c : S->spare) hs += col_bytes(c);
  for (const auto& kv : S->groups) h += group_bytes(kv.second);
  for (const DevBuf* b : {&S->d_desc, &S->d_desc_u, &S->d_hn, &S->d_dpart, &S->d_npart, &S->d_fz, &S->d_fphi,
                          &S->d_fff, &S->d_fobs, &S->d_adm})
    h += (int64_t)b->bytes;
  h += S->retired_bytes;
  std::lock_guard<std::mutex> lk(S->B.mu);
  S->held = h + hs;
  S->held_spare = hs;
}

// After a round.  While requests run, the fused-launch buffers of groups no
// admitted column uses any more are freed.  When the last request has left,
// everything is kept for the next one (the worker calls release_idle_memory
// if none comes soon).
void settle_memory(lm_server_s* S, bool idle) {
  if (idle) {  // nothing is queued behind the last results
    (void)hipStreamSynchronize(S->s);
    (void)collect_update_time(S);
  } else {
    drop_groups(S, [](const std::pair<lm_geom_s*, int>&) { return true; });
  }
  record_held(S);
}

// The worker has stayed idle: frees the fused-launch buffers, the round and
// finishing buffers and the retired allocations.
void release_idle_memory(lm_server_s* S) {
  (void)quiesce(S);
  drop_groups(S, [](const std::pair<lm_geom_s*, int>&) { return true; });
  for (DevBuf* b : {&S->d_desc, &S->d_desc_u, &S->d_hn, &S->d_dpart, &S->d_npart, &S->d_fz, &S->d_fphi,
                    &S->d_fff, &S->d_fobs, &S->d_adm})
    b->release();
  record_held(S);
}

lm_status start_request(lm_server_s* S, Request* q) {
  const int m = std::max(1, std::min(q->o.restart, q->o.max_iter));
  const int N = (int)q->g->N;
  // the angles go down in kernel arguments and the right-hand sides are
  // queued: admission does not wait for the rounds in flight
  const size_t sb = (rhs_scratch_bytes(1) + 255) / 256 * 256;
  LM_TRY(ensure(S, S->d_adm, sb + (size_t)q->R * sizeof(double)));
  double* d_th = reinterpret_cast<double*>(S->d_adm.as<char>() + sb);
  LM_TRY(put_f64_async(q->theta.data(), q->R, d_th, S->s));
  for (int c = 0; c < q->R; ++c) {
    // a spare column of the same shape keeps its device buffers
    Column* col = nullptr;
    for (auto it = S->spare.begin(); it != S->spare.end(); ++it)
      if ((*it)->N == N && (*it)->m == m) {
        col = *it;
        S->spare.erase(it);
        break;
      }
    const bool fresh = col == nullptr;
    if (fresh) col = new (std::nothrow) Column();
    LM_CHECK(col, LM_ENOMEM, "host allocation failed");
    S->cols.push_back(col);
    col->reset();
    col->req = q;
    col->col = c;
    col->g = q->g;
    col->N = N;
    col->m = m;
    col->ldv = (N + 63) / 64 * 64;
    if (fresh) {
      auto alloc = [&]() -> lm_status {
        LM_TRY(col->V.alloc((size_t)(m + 1) * col->ldv * basis_bytes(S)));
        LM_TRY(col->z.alloc((size_t)N * sizeof(double2)));
        LM_TRY(col->gv.alloc((size_t)N * sizeof(double2)));
        LM_TRY(col->y.alloc((size_t)(m + 1) * sizeof(double2)));
        LM_TRY(col->dn.alloc(sizeof(double)));
        return LM_OK;
      };
      if (alloc() < 0) {  // give the spare columns' memory back and try once more
        drop_spares(S);
        LM_TRY(alloc());
      }
    }
    LM_TRY_HIP(hipMemsetAsync(col->z.p, 0, (size_t)N * sizeof(double2), S->s));
    LM_TRY(rhs_launch_dev(q->g, 1, d_th + c, S->d_adm.p, col->gv.p, S->s));
    // an Arnoldi step writes rows 0..j+1 of its Hessenberg column before
    // anything reads them, so a reused column's arrays need no clearing
    col->H.resize((size_t)(m + 1) * m);
    col->Hraw.resize((size_t)(m + 1) * m);
    col->cprev.assign(m + 1, 0.0);
    col->cs.assign(m, 0.0);
    col->sn.assign(m, 0.0);
    col->e1.assign(m + 1, 0.0);
    col->phase = PH_INIT;
  }
  q->rep.assign(q->R, lm_solve_report{0, 0.0});
  q->cols_left = q->R;
  return LM_OK;
}

// Fills the requests' host arrays of the staged columns from h_fin and marks
// the columns finished, once the staging copies are done: at once if `block`,
// else only if ev_fin has fired.  Returns whether nothing stays staged.
bool complete_staged(lm_server_s* S, bool block) {
  if (S->staged.empty()) return true;
  if (block) {
    if (hipEventSynchronize(S->ev_fin) != hipSuccess) return false;
  } else if (hipEventQuery(S->ev_fin) != hipSuccess) {
    return false;
  }
  const char* hb = S->h_fin.as<char>();
  auto copy = [&](int i) {
    const lm_server_s::Staged& e = S->staged[i];
    Column* c = e.c;
    std::memcpy(c->req->phi.get() + (size_t)c->col * c->N, hb + e.phi_off, (size_t)c->N * sizeof(double2));
    if (e.no)
      std::memcpy(c->req->ff.data() + (size_t)c->col * e.no, hb + e.ff_off, (size_t)e.no * sizeof(double2));
  };
  S->pool->run((int)S->staged.size(), copy);
  for (const lm_server_s::Staged& e : S->staged) e.c->finished = true;
  S->staged.clear();
  return true;
}

// Drops the staged entries of a request that leaves (cancelled or failed):
// its columns are about to be released.
void unstage(lm_server_s* S, const Request* q) {
  auto& v = S->staged;
  v.erase(std::remove_if(v.begin(), v.end(), [&](const lm_server_s::Staged& e) { return e.c->req == q; }), v.end());
}

// phi = M z, far fields and their copies to pinned host memory for the
// columns that finished this round; the copies are not waited for (the
// columns are PH_STAGED until complete_staged sees them done, normally while
// the next round runs).  Columns on one geometry share one preconditioner
// launch (several right-hand sides), columns of requests with the same
// observation angles one far-field launch.  Returns the first failure; the
// columns of a failed group are reported through *failed.
lm_status finish_columns(lm_server_s* S, std::vector<Column*>& fin, std::vector<Request*>* failed) {
  LM_CHECK(complete_staged(S, true), LM_EHIP, "HIP error while copying solutions to host memory");
  std::stable_sort(fin.begin(), fin.end(), [](const Column* a, const Column* b) {
    if (a->g != b->g) return a->g < b->g;
    const bool pa = a->req->o.precond != 0, pb = b->req->o.precond != 0;
    if (pa != pb) return pa < pb;
    if (a->req != b->req) return a->req->id < b->req->id;
    return a->col < b->col;
  });
  size_t hbytes = 0;
  for (const Column* c : fin) hbytes += ((size_t)c->N + c->req->obs.size()) * sizeof(double2);
  LM_TRY(host_ensure(S, S->h_fin, hbytes));
  char* hb = S->h_fin.as<char>();
  size_t off = 0;
  lm_status first = LM_OK;
  for (size_t i0 = 0; i0 < fin.size();) {
    lm_geom_s* g = fin[i0]->g;
    const bool pre = fin[i0]->req->o.precond && g->pre;
    size_t i1 = i0;
    while (i1 < fin.size() && fin[i1]->g == g && (fin[i1]->req->o.precond != 0) == (fin[i0]->req->o.precond != 0))
      ++i1;
    const int k = (int)(i1 - i0), N = fin[i0]->N;
    const size_t vb = (size_t)N * sizeof(double2);
    const size_t s0 = S->staged.size();
    auto group = [&]() -> lm_status {
      // d_fz / d_fphi / d_fff: earlier finishing work that used them is
      // queued before this on the one stream, and grown buffers are retired
      LM_TRY(ensure(S, S->d_fz, k * vb));
      LM_TRY(ensure(S, S->d_fphi, k * vb));
      char* zb = (char*)S->d_fz.p;
      char* pb = (char*)S->d_fphi.p;
      for (int i = 0; i < k; ++i)
        LM_TRY_HIP(hipMemcpyAsync((pre ? zb : pb) + i * vb, fin[i0 + i]->z.p, vb, hipMemcpyDeviceToDevice, S->s));
      if (pre) LM_TRY(precond_apply(g, pre_precision(S), k, zb, pb, S->s));
      // phi of the group: one copy (its columns are contiguous in d_fphi)
      const size_t phi0 = off;
      LM_TRY_HIP(hipMemcpyAsync(hb + phi0, pb, k * vb, hipMemcpyDeviceToHost, S->s));
      off += k * vb;
      for (int i = 0; i < k; ++i) S->staged.push_back({fin[i0 + i], phi0 + i * vb, 0, 0});
      for (int a = 0; a < k;) {  // one far-field launch per run of requests with the same angles
        const std::vector<double>& obs = fin[i0 + a]->req->obs;
        int b = a;
        while (b < k && fin[i0 + b]->req->obs == obs) ++b;
        const int no = (int)obs.size();
        if (no) {
          const size_t fb = (size_t)(b - a) * no * sizeof(double2);
          // far fields, then the chunk partials of the launch behind them
          const size_t fw = farfield_work_bytes(g, b - a, no);
          LM_TRY(ensure(S, S->d_fff, fb + fw));
          LM_TRY(ensure(S, S->d_fobs, (size_t)no * sizeof(double)));
          LM_TRY(put_f64_async(obs.data(), no, S->d_fobs.as<double>(), S->s));
          LM_TRY(farfield_launch_dev(g, b - a, pb + a * vb, no, S->d_fobs.as<double>(), S->d_fff.p,
                                     S->d_fff.as<char>() + fb, S->s));
          LM_TRY_HIP(hipMemcpyAsync(hb + off, S->d_fff.p, fb, hipMemcpyDeviceToHost, S->s));
          for (int i = a; i < b; ++i) {
            lm_server_s::Staged& e = S->staged[s0 + i];
            e.ff_off = off + (size_t)(i - a) * no * sizeof(double2);
            e.no = no;
          }
          off += fb;
        }
        a = b;
      }
      return LM_OK;
    };
    const lm_status st = group();
    if (st < 0) S->staged.resize(s0);
    for (size_t i = i0; i < i1; ++i) {
      Column* c = fin[i];
      if (st < 0) {
        if (failed && (failed->empty() || failed->back() != c->req)) failed->push_back(c->req);
        continue;
      }
      c->req->rep[c->col].iterations = c->its;
      c->req->rep[c->col].rel_residual = c->res;
      c->phase = PH_STAGED;
    }
    if (st < 0 && first == LM_OK) first = st;
    i0 = i1;
  }
  if (!S->staged.empty()) LM_TRY_HIP(hipEventRecord(S->ev_fin, S->s));
  return first;
}

// One round of the worker (see the file comment).  Returns an error only for
// failures that are not attributable to a single request.
lm_status run_round(lm_server_s* S) {
  const double tr0 = now_s();
  std::vector<Column*> cols;
  for (Column* c : S->cols)
    if (!c->finished && c->phase != PH_STAGED) cols.push_back(c);
  if (cols.empty()) {  // only staged columns left
    LM_CHECK(complete_staged(S, true), LM_EHIP, "HIP error while copying solutions to host memory");
    return LM_OK;
  }
  const int prec = S->o.precision;
  const bool f32 = prec == LM_MIXED;  // complex64 Krylov basis
  const int nc = (int)cols.size();
  int Nmax = 0, cntmax = 0;
  for (Column* c : cols) {
    Nmax = std::max(Nmax, c->N);
    // an Arnoldi step needs K M u_j unless it can only finalise column j-1
    // (restart length reached or the last allowed iteration)
    c->km = c->phase == PH_RESTART || c->phase == PH_FINAL ||
            (c->phase == PH_ARNOLDI && !(c->j >= 1 && (c->j == c->m || c->its + 1 >= c->req->o.max_iter)));
    if (c->phase == PH_ARNOLDI) cntmax = std::max(cntmax, c->j + 1);
  }
  const int slice = f32 ? sd_slice<float2>() : sd_slice<double2>();
  const int nwu = 4 * (int)div_up(Nmax, 256), nbd = (int)div_up(Nmax, slice);
  // dot products per column: V^H u then V^H z, cntmax each (the longest
  // basis of the round), so the copy to the host holds no unused rows
  const int ldh = std::max(1, cntmax), hs = 2 * ldh;
  LM_TRY_HIP(hipEventRecord(S->t0, S->s));
  // ---- 1. K M v for every column that needs it, fused per (geometry, precond)
  std::map<std::pair<lm_geom_s*, int>, std::vector<Column*>> byg;
  for (Column* c : cols) {
    c->w = c->phase == PH_INIT ? c->gv.as<double2>() : nullptr;
    if (c->km) byg[{c->g, c->req->o.precond ? 1 : 0}].push_back(c);
  }
  // gather the inputs (normalising lagged basis vectors on the way): one kernel
  std::vector<ColDev> gath;
  for (auto& kv : byg) {
    Group& G = S->groups[kv.first];
    const int R = (int)kv.second.size(), N = (int)kv.first.first->N;
    LM_TRY(ensure(S, G.X, (size_t)R * N * sizeof(double2)));
    LM_TRY(ensure(S, G.Y, (size_t)R * N * sizeof(double2)));
    for (int k = 0; k < R; ++k) {
      Column* c = kv.second[k];
      ColDev d{};
      d.N = N;
      d.dst = G.X.as<double2>() + (size_t)k * N;
      d.scale = 1.0;
      if (c->phase == PH_ARNOLDI) {
        d.V = c->V.p;
        d.ld = c->ldv;
        d.vj = c->j;
        d.nsrc = c->j >= 1 ? c->dn.as<double>() : nullptr;
      } else {
        d.vj = -1;
        d.w = c->z.as<double2>();
      }
      gath.push_back(d);
      c->w = G.Y.as<double2>() + (size_t)k * N;
    }
  }
  for (Column* c : cols)  // finalise-only steps still normalise their lagged vector
    if (c->phase == PH_ARNOLDI && !c->km && c->j >= 1) {
      ColDev d{};
      d.N = c->N;
      d.V = c->V.p;
      d.ld = c->ldv;
      d.vj = c->j;
      d.nsrc = c->dn.as<double>();
      gath.push_back(d);
    }
  // descriptors of the dot products (section 2), uploaded with the gather's
  S->hdesc.assign(nc, ColDev{});
  for (int i = 0; i < nc; ++i) {
    Column* c = cols[i];
    ColDev& d = S->hdesc[i];
    d.V = c->V.p;
    d.ld = c->ldv;
    d.N = c->N;
    if (c->phase == PH_ARNOLDI) {
      d.cnt = c->j + 1;  // dots against V[0..j]; u = V[j]
      d.w = c->km ? c->w : nullptr;
      d.nsrc = c->j >= 1 ? c->dn.as<double>() : nullptr;  // norm of u before normalisation
    } else {
      d.w = c->w;
      d.g = (c->phase == PH_RESTART || c->phase == PH_FINAL) ? c->gv.as<double2>() : nullptr;
    }
  }
  const size_t ngath = gath.size();
  gath.insert(gath.end(), S->hdesc.begin(), S->hdesc.end());
  LM_TRY(upload_async(S, S->h_desc, S->d_desc, gath.data(), gath.size() * sizeof(ColDev)));
  if (ngath > 0) {
    if (f32)
      hipLaunchKernelGGL(k_s_gather<float2>, dim3(div_up(Nmax, 256), ngath), dim3(256), 0, S->s,
                         S->d_desc.as<ColDev>());
    else
      hipLaunchKernelGGL(k_s_gather<double2>, dim3(div_up(Nmax, 256), ngath), dim3(256), 0, S->s,
                         S->d_desc.as<ColDev>());
    LM_TRY_HIP(hipGetLastError());
  }
  LM_TRY_HIP(hipEventRecord(S->ev_main, S->s));
  std::vector<char> used_stream(SRV_STREAMS, 0), stream_timed(SRV_STREAMS, 0);
  std::vector<int> timed_streams;
  double m2l_flops_round = 0.0;
  int64_t n_launch = 0, n_fused = 0;
  // one group: its fused launch runs on the round's own stream (a wait on
  // another stream's event costs about 15 us each way); several: one stream
  // per geometry, so that different geometries overlap
  const bool one_group = byg.size() == 1;
  for (auto& kv : byg) {
    lm_geom_s* g = kv.first.first;
    const bool pre = kv.first.second && g->pre;
    const int R = (int)kv.second.size();
    auto it = S->stream_of.find(g);
    if (it == S->stream_of.end()) it = S->stream_of.emplace(g, (int)(S->stream_of.size() % SRV_STREAMS)).first;
    const int si = it->second;
    hipStream_t st = one_group ? S->s : S->gs[si];
    if (!one_group && !used_stream[si]) LM_TRY_HIP(hipStreamWaitEvent(st, S->ev_main, 0));
    used_stream[si] = one_group ? 0 : 1;
    Group& G = S->groups[kv.first];
    const bool time_m2l = g->method == LM_FMM && !stream_timed[si];
    G.km.stage_ev = time_m2l ? S->sev[si] : nullptr;
    G.km.pre_precision = pre_precision(S);
    LM_TRY(apply_km(g, prec, R, G.X.as<double2>(), G.Y.as<double2>(), pre, G.km, st));
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
  // ---- 2. dot products of the delayed two-pass Gram-Schmidt, residuals, norms
  LM_TRY(ensure(S, S->d_npart, (size_t)nc * nwu * sizeof(double)));
  const size_t hbytes = (size_t)nc * hs * sizeof(double2), hnbytes = hbytes + (size_t)nc * sizeof(double);
  LM_TRY(ensure(S, S->d_hn, hnbytes));
  double2* d_h = S->d_hn.as<double2>();
  double* d_nrm = reinterpret_cast<double*>(S->d_hn.as<char>() + hbytes);
  const ColDev* dd = S->d_desc.as<ColDev>() + ngath;
  if (cntmax > 0) {
    LM_TRY(ensure(S, S->d_dpart, (size_t)2 * nc * ldh * nbd * sizeof(double2)));
    double2* pa = S->d_dpart.as<double2>();
    double2* pb = pa + (size_t)nc * ldh * nbd;
    // split the basis over the grid's z only as far as needed for SD_WGS
    // workgroups (each split reloads u and z), in near-equal blocks of at
    // least 16 vectors
    const int nz = std::max(1, std::min((int)div_up(SD_WGS, (int64_t)nbd * nc), (int)div_up(cntmax, 16)));
    const int blk = (int)div_up(cntmax, nz);
    if (f32)
      hipLaunchKernelGGL(k_s_dots2<float2>, dim3(nbd, nc, nz), dim3(256), 0, S->s, dd, pa, pb, ldh, nbd, blk);
    else
      hipLaunchKernelGGL(k_s_dots2<double2>, dim3(nbd, nc, nz), dim3(256), 0, S->s, dd, pa, pb, ldh, nbd, blk);
    hipLaunchKernelGGL(k_s_dots2_final, dim3(cntmax, nc), dim3(64), 0, S->s, dd, pa, pb, ldh, nbd, slice,
                       d_h, hs);
  }
  // norms: of g - K M z (restart, final) or g (first round); Arnoldi columns
  // report the norm the previous update pass left
  hipLaunchKernelGGL(k_s_resid, dim3(div_up(Nmax, 256), nc), dim3(256), 0, S->s, dd, S->d_npart.as<double>(), nwu);
  hipLaunchKernelGGL(k_s_norm_final, dim3(nc), dim3(64), 0, S->s, dd, S->d_npart.as<double>(), nwu,
                     d_nrm);
  LM_TRY_HIP(hipGetLastError());
  LM_TRY(host_ensure(S, S->h_hn, hnbytes));
  if (cntmax > 0)
    LM_TRY_HIP(hipMemcpyAsync(S->h_hn.p, S->d_hn.p, hnbytes, hipMemcpyDeviceToHost, S->s));
  else
    LM_TRY_HIP(hipMemcpyAsync(S->h_hn.as<char>() + hbytes, d_nrm, hnbytes - hbytes, hipMemcpyDeviceToHost, S->s));
  LM_TRY_HIP(hipEventRecord(S->t2, S->s));
  // the round's one wait: the host step needs the dot products and norms.
  // Polled rather than blocked on, so the host step starts within
  // microseconds of the copy (the worker thread is busy-waiting meanwhile)
  const double tw0 = now_s();
  LM_TRY_HIP(hipEventRecord(S->ev_wait, S->s));
  // the previous round's staging copies ran before this round's kernels:
  // copy them out while those run
  (void)complete_staged(S, true);
  S->pool->arm();  // the host step follows the wait
  for (;;) {
    const hipError_t q = hipEventQuery(S->ev_wait);
    if (q == hipSuccess) break;
    LM_CHECK(q == hipErrorNotReady, LM_EHIP, "HIP error: %s", hipGetErrorString(q));
    std::this_thread::yield();
  }
  const double tw1 = now_s();
  float gs_a = 0.f;
  LM_TRY_HIP(hipEventElapsedTime(&km_round, S->t0, S->t1));
  LM_TRY_HIP(hipEventElapsedTime(&gs_a, S->t1, S->t2));
  LM_TRY(collect_update_time(S));  // the previous round's update pass
  const double2* hhv = S->h_hn.as<double2>();
  const double* hnv = reinterpret_cast<const double*>(S->h_hn.as<char>() + hbytes);
  // ---- 3. host updates ------------------------------------------------------------
  // Per column, independent of the others (its Hessenberg correction is
  // O(j^2)): spread over the host pool, each column's descriptors and
  // coefficients into its own HostStep, merged in column order afterwards.
  const double bb = (double)basis_bytes(S);
  S->steps.resize(nc);
  auto host_step = [&](int i) {
    HostStep& o = S->steps[i];
    o.clear();
    Column* c = cols[i];
    const double nrm = std::sqrt(hnv[i]);
    const double tol = c->req->o.tol;
    const int N = c->N, m = c->m;
    const double n16 = 16.0 * N;
    auto start_cycle = [&](const double2* r, double beta) {
      c->j = 0;
      std::fill(c->e1.begin(), c->e1.end(), C(0.0));
      c->e1[0] = beta;
      ColDev d{};
      d.src = r;
      d.V = c->V.p;
      d.ld = c->ldv;
      d.scale = 1.0 / beta;
      d.N = N;
      o.scal.push_back(d);
      c->phase = PH_ARNOLDI;
    };
    auto end_cycle = [&](int cnt, bool conv) {  // y = H^{-1} e1 over cnt columns, z += V y
      std::vector<C> yv(cnt);
      for (int k = cnt - 1; k >= 0; --k) {
        C acc = c->e1[k];
        for (int l = k + 1; l < cnt; ++l) acc -= c->H[(size_t)l * (m + 1) + k] * yv[l];
        yv[k] = acc / c->H[(size_t)k * (m + 1) + k];
      }
      ColDev d{};
      d.V = c->V.p;
      d.ld = c->ldv;
      d.z = c->z.as<double2>();
      d.N = N;
      d.cnt = cnt;
      d.scale = (double)o.ys.size();  // offset into the coefficient upload
      for (int k = 0; k < cnt; ++k) o.ys.push_back(make_double2(yv[k].real(), yv[k].imag()));
      o.comb.push_back(d);
      c->converged = conv;
      c->phase = (conv || c->its >= c->req->o.max_iter) ? PH_FINAL : PH_RESTART;
    };
    if (c->phase == PH_INIT) {
      o.gsb += n16;
      c->gnorm = nrm;
      if (nrm == 0.0) {
        c->res = 0.0;
        c->converged = true;
        o.to_finish.push_back(c);
      } else {
        c->res = 1.0;
        start_cycle(c->w, nrm);
      }
      return;
    }
    if (c->phase == PH_RESTART || c->phase == PH_FINAL) {
      o.gsb += 3.0 * n16;
      c->res = nrm / c->gnorm;
      if (c->phase == PH_FINAL) {
        o.to_finish.push_back(c);  // true residual; convergence was decided by the GMRES estimate
      } else if (c->res <= tol) {
        c->converged = true;
        o.to_finish.push_back(c);
      } else {
        start_cycle(c->w, nrm);
      }
      return;
    }
    // Arnoldi step j: a = V[0..j]^H u_j, b = V[0..j]^H K M u_j
    const int j = c->j;
    // basis vectors (bb bytes per element) and complex128 vectors moved by the
    // dot, residual-norm and update kernels of this step
    o.gsb += (c->km ? (2.0 * j + 5.0) * bb + (j == 0 ? 3.0 : 2.0) * 16.0 : (j + 2.0) * bb) * N;
    const double2* ha = &hhv[(size_t)i * hs];
    const double2* hb = ha + ldh;
    std::vector<C> aQ(j), bQ(j);
    for (int k = 0; k < j; ++k) {
      aQ[k] = C(ha[k].x, ha[k].y);
      bQ[k] = C(hb[k].x, hb[k].y);
    }
    double aa = 0.0;
    for (int k = 0; k < j; ++k) aa += std::norm(aQ[k]);
    const double mu = ha[j].x;  // |u_j|^2 (u_j normalised this round)
    const double rho = std::sqrt(std::max(mu - aa, 0.0));
    if (j >= 1) {
      // corrected Hessenberg column j-1 (from the provisional one and aQ)
      const double bprev = nrm;  // |w| of the once-projected vector before normalisation
      C* Hr = &c->Hraw[(size_t)(j - 1) * (m + 1)];
      for (int k = 0; k < j; ++k) Hr[k] = c->cprev[k] + bprev * aQ[k];
      Hr[j] = bprev * rho;
      C* Hc = &c->H[(size_t)(j - 1) * (m + 1)];
      for (int k = 0; k <= j; ++k) Hc[k] = Hr[k];
      const int jj = j - 1;
      for (int k = 0; k < jj; ++k) {
        const C a = Hc[k], b = Hc[k + 1];
        Hc[k] = std::conj(c->cs[k]) * a + std::conj(c->sn[k]) * b;
        Hc[k + 1] = -c->sn[k] * a + c->cs[k] * b;
      }
      const C a = Hc[jj], b = Hc[jj + 1];
      const double rr = std::hypot(std::abs(a), std::abs(b));
      c->cs[jj] = rr > 0 ? a / rr : C(1.0);
      c->sn[jj] = rr > 0 ? b / rr : C(0.0);
      Hc[jj] = std::conj(c->cs[jj]) * a + std::conj(c->sn[jj]) * b;
      Hc[jj + 1] = 0.0;
      c->e1[jj + 1] = -c->sn[jj] * c->e1[jj];
      c->e1[jj] = std::conj(c->cs[jj]) * c->e1[jj];
      c->its++;
      c->res = std::abs(c->e1[jj + 1]) / c->gnorm;
      const bool conv = c->res <= tol || std::abs(Hr[j]) <= 1e-300;
      if (conv || j == m || c->its >= c->req->o.max_iter || !c->km) {
        end_cycle(j, conv);
        return;
      }
    }
    // continue: re-orthogonalise u_j into v_j and form the once-projected
    // next vector from K M u_j (see the file comment)
    const C gamma(hb[j].x, hb[j].y);
    // Ha = H[0..j-1, 0..j-1] aQ (upper Hessenberg), in plain real arithmetic
    std::vector<C> Ha(j, C(0.0));
    {
      std::vector<double> hr(2 * (size_t)j, 0.0);
      for (int l = 0; l < j; ++l) {
        const double ar = aQ[l].real(), ai = aQ[l].imag();
        const double* H = reinterpret_cast<const double*>(&c->Hraw[(size_t)l * (m + 1)]);
        const int kt = std::min(l + 1, j - 1);
        for (int k = 0; k <= kt; ++k) {
          hr[2 * k] += H[2 * k] * ar - H[2 * k + 1] * ai;
          hr[2 * k + 1] += H[2 * k] * ai + H[2 * k + 1] * ar;
        }
      }
      for (int k = 0; k < j; ++k) Ha[k] = C(hr[2 * k], hr[2 * k + 1]);
    }
    const C hj = j >= 1 ? c->Hraw[(size_t)(j - 1) * (m + 1) + j] * aQ[j - 1] : C(0.0);
    C ab(0.0);
    for (int k = 0; k < j; ++k) ab += std::conj(aQ[k]) * bQ[k];
    const C cj = ((gamma - ab) / rho - hj) / rho;
    const C dd2 = hj / rho + cj;
    ColDev d{};
    d.V = c->V.p;
    d.ld = c->ldv;
    d.w = c->w;
    d.N = N;
    d.cnt = j;
    d.scale = 1.0 / rho;
    d.dr = make_double2((dd2 / rho).real(), (dd2 / rho).imag());
    d.ndst = c->dn.as<double>();
    d.src = reinterpret_cast<const double2*>((size_t)o.cf.size());  // offset, fixed up after the upload
    for (int k = 0; k < j; ++k) o.cf.push_back(make_double2(aQ[k].real(), aQ[k].imag()));
    for (int k = 0; k < j; ++k) {
      const C cq = (bQ[k] - Ha[k]) / rho;
      c->cprev[k] = cq;
      const C e = Ha[k] / rho + cq - aQ[k] * dd2 / rho;
      o.cf.push_back(make_double2(e.real(), e.imag()));
    }
    c->cprev[j] = cj;
    o.upd.push_back(d);
    c->j = j + 1;
  };
  S->pool->run(nc, host_step);
  std::vector<ColDev> scal, comb, upd;
  std::vector<double2> ys, cf;
  std::vector<Column*> to_finish;
  double gsb = 0.0;
  for (int i = 0; i < nc; ++i) {
    HostStep& o = S->steps[i];
    const size_t bys = ys.size(), bcf = cf.size();
    for (ColDev d : o.comb) {
      d.scale += (double)bys;
      comb.push_back(d);
    }
    for (ColDev d : o.upd) {
      d.src = reinterpret_cast<const double2*>(reinterpret_cast<size_t>(d.src) + bcf);
      upd.push_back(d);
    }
    scal.insert(scal.end(), o.scal.begin(), o.scal.end());
    ys.insert(ys.end(), o.ys.begin(), o.ys.end());
    cf.insert(cf.end(), o.cf.begin(), o.cf.end());
    to_finish.insert(to_finish.end(), o.to_finish.begin(), o.to_finish.end());
    gsb += o.gsb;
  }
  // one upload: the descriptors (update passes, copies, solution
  // combinations), then their coefficients (update passes, combinations)
  const size_t ncf = cf.size();
  const size_t nall = upd.size() + scal.size() + comb.size();
  const size_t dbytes = (nall * sizeof(ColDev) + 255) / 256 * 256;
  const size_t ubytes = dbytes + (ncf + ys.size()) * sizeof(double2);
  if (nall > 0) {
    LM_TRY(ensure(S, S->d_desc_u, ubytes));
    LM_TRY(host_ensure(S, S->h_desc_u, ubytes));
  }
  double2* dy = reinterpret_cast<double2*>(S->d_desc_u.as<char>() + dbytes);
  for (auto& d : upd) {
    d.y = dy + (size_t)d.src;
    d.src = nullptr;
  }
  for (auto& d : comb) {
    d.y = dy + ncf + (size_t)d.scale;
    d.scale = 0.0;
  }
  std::vector<ColDev> all(upd);
  all.insert(all.end(), scal.begin(), scal.end());
  all.insert(all.end(), comb.begin(), comb.end());
  if (!all.empty()) {
    char* hb = S->h_desc_u.as<char>();
    std::memcpy(hb, all.data(), all.size() * sizeof(ColDev));
    std::memcpy(hb + dbytes, cf.data(), ncf * sizeof(double2));
    std::memcpy(hb + dbytes + ncf * sizeof(double2), ys.data(), ys.size() * sizeof(double2));
    LM_TRY_HIP(hipMemcpyAsync(S->d_desc_u.p, hb, ubytes, hipMemcpyHostToDevice, S->s));
    int nm = 0;
    for (auto& d : all) nm = std::max(nm, d.N);
    const ColDev* da = S->d_desc_u.as<ColDev>();
    LM_TRY_HIP(hipEventRecord(S->tu1, S->s));
    if (!upd.empty()) {
      if (f32)
        hipLaunchKernelGGL(k_s_update2<float2>, dim3(div_up(nm, SU_ELEM), upd.size()), dim3(256), 0, S->s, da,
                           S->d_npart.as<double>(), nwu);
      else
        hipLaunchKernelGGL(k_s_update2<double2>, dim3(div_up(nm, SU_ELEM), upd.size()), dim3(256), 0, S->s, da,
                           S->d_npart.as<double>(), nwu);
      hipLaunchKernelGGL(k_s_norm_to, dim3(upd.size()), dim3(64), 0, S->s, da, S->d_npart.as<double>(), nwu);
    }
    LM_TRY_HIP(hipEventRecord(S->tu2, S->s));
    S->tu_pending = true;
    if (!scal.empty()) {
      if (f32)
        hipLaunchKernelGGL(k_s_copy<float2>, dim3(div_up(nm, 256), scal.size()), dim3(256), 0, S->s, da + upd.size());
      else
        hipLaunchKernelGGL(k_s_copy<double2>, dim3(div_up(nm, 256), scal.size()), dim3(256), 0, S->s,
                           da + upd.size());
    }
    if (!comb.empty()) {
      if (f32)
        hipLaunchKernelGGL(k_s_lincomb<float2>, dim3(div_up(nm, 512), comb.size()), dim3(256), 0, S->s,
                           da + upd.size() + scal.size());
      else
        hipLaunchKernelGGL(k_s_lincomb<double2>, dim3(div_up(nm, 512), comb.size()), dim3(256), 0, S->s,
                           da + upd.size() + scal.size());
    }
    LM_TRY_HIP(hipGetLastError());
    // no wait here: the next round's copies and kernels are queued behind
    // these on the same stream
  }
  const double tw2 = now_s();
  {
    float m2l = 0.f;
    for (int si : timed_streams) {
      float t = 0.f;
      LM_TRY_HIP(hipEventElapsedTime(&t, S->sev[si][4], S->sev[si][5]));
      m2l += t;
    }
    std::lock_guard<std::mutex> lk(S->B.mu);
    S->km_ms += km_round;
    S->gs_ms += gs_a;
    S->launch_ms += 1e3 * (tw0 - tr0);
    S->wait_ms += 1e3 * (tw1 - tw0);
    S->step_ms += 1e3 * (tw2 - tw1);
    S->m2l_ms += m2l;
    S->m2l_flops += m2l_flops_round;
    S->m2l_launches += (int64_t)timed_streams.size();
    S->gs_bytes += gsb;
    S->launches += n_launch;
    S->fused_rhs += n_fused;
    S->rounds++;
  }
  const double tf0 = now_s();
  if (!to_finish.empty()) {
    std::vector<Request*> failed;
    const lm_status st = finish_columns(S, to_finish, &failed);
    if (st < 0) {
      const std::string msg = lm_last_error();
      for (Request* q : failed) S->B.mark_failed(q, st, msg);
    }
  }
  const double tf1 = now_s();
  std::lock_guard<std::mutex> lk(S->B.mu);
  S->round_ms += 1e3 * (tf0 - tr0);
  S->finish_ms += 1e3 * (tf1 - tf0);
  return LM_OK;
}

// Removes the request's columns; up to max_active_rhs of them stay as spares
// with their device buffers for the next admission of the same shape.  A
// spare is only written by work queued after what may still use it (one
// stream), so only freeing a column waits for the queued kernels.
void release_columns(lm_server_s* S, Request* q) {
  unstage(S, q);
  bool synced = false;
  auto& v = S->cols;
  for (auto it = v.begin(); it != v.end();) {
    if ((*it)->req == q) {
      Column* c = *it;
      const bool whole = c->V.p && c->z.p && c->gv.p && c->y.p && c->dn.p;  // a failed start leaves holes
      if (whole && (int)S->spare.size() < S->o.max_active_rhs) {
        (*it)->req = nullptr;
        S->spare.push_back(*it);
      } else {
        if (!synced) (void)quiesce(S);  // queued kernels may still use the column's buffers
        synced = true;
        delete *it;
      }
      it = v.erase(it);
    } else {
      ++it;
    }
  }
}

// The device side of the worker loop (lmsched::run_worker drives it).
struct GpuDev {
  lm_server_s* S;
  lm_status start(Request* q) { return start_request(S, q); }
  void release(Request* q) { release_columns(S, q); }
  bool has_work() const { return !S->cols.empty(); }
  lm_status round() { return run_round(S); }
  bool finished(Request* q, bool* conv) {
    bool all = true;
    *conv = true;
    for (const Column* c : S->cols)
      if (c->req == q) {
        all = all && c->finished;
        *conv = *conv && c->converged;
      }
    return all;
  }
  // spare columns count against the budget: free what the admitted requests'
  // footprints leave no room for
  void trim(int64_t allow, const std::vector<Request*>& admit) { trim_spares(S, allow, admit); }
  void settle(bool idle) { settle_memory(S, idle); }
  void release_idle() { release_idle_memory(S); }
  double now() const { return now_s(); }
  std::string last_error() const { return lm_last_error(); }
};

void worker(lm_server_s* S) {
  (void)hipSetDevice(S->device);
  GpuDev D{S};
  lmsched::run_worker(S->B, D);
  drop_spares(S);
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
  S->B.max_rhs = so.max_active_rhs;
  S->B.budget = so.hbm_budget_bytes;
  if (hipGetDevice(&S->device) != hipSuccess) S->device = 0;
  bool ok = hipStreamCreateWithFlags(&S->s, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&S->ev_main, hipEventDisableTiming) == hipSuccess &&
            hipEventCreate(&S->t0) == hipSuccess && hipEventCreate(&S->t1) == hipSuccess &&
            hipEventCreate(&S->t2) == hipSuccess && hipEventCreate(&S->tu1) == hipSuccess &&
            hipEventCreate(&S->tu2) == hipSuccess &&
            hipEventCreateWithFlags(&S->ev_wait, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&S->ev_fin, hipEventDisableTiming) == hipSuccess;
  for (int i = 0; ok && i < SRV_STREAMS; ++i)
    for (int e = 0; ok && e < 16; ++e) ok = hipEventCreate(&S->sev[i][e]) == hipSuccess;
  for (int i = 0; ok && i < SRV_STREAMS; ++i)
    ok = hipStreamCreateWithFlags(&S->gs[i], hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&S->ev[i], hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    lm_set_error("stream creation failed");
    delete S;
    return LM_EHIP;
  }
  try {  // host threads for the per-column updates: at most 8, never more than the cores
    const int hc = (int)std::thread::hardware_concurrency();
    S->pool.reset(new HostPool(std::min(8, std::max(1, hc))));
    S->th = std::thread(worker, S);
  } catch (const std::exception& e) {
    lm_set_error("host thread creation failed: %s", e.what());
    delete S;
    return LM_EINTERNAL;
  }
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
  q->phi_n = (size_t)q->R * q->g->N;
  q->phi.reset(static_cast<double2*>(std::malloc(q->phi_n * sizeof(double2))));
  if (!q->phi) {
    delete q;
    LM_CHECK(false, LM_ENOMEM, "host allocation failed");
  }
  q->ff.assign((size_t)q->R * r->n_obs, make_double2(0.0, 0.0));
  if (q->R > S->o.max_active_rhs || q->bytes > S->o.hbm_budget_bytes)
    lm_set_error("request can never be admitted (%d right-hand sides, %lld bytes)", r->n_rhs, (long long)q->bytes);
  return S->B.submit(q, now_s(), id);  // deletes q when it can never be admitted
}

extern "C" lm_status lm_poll(lm_server S, uint64_t id, lm_state* state, lm_solve_report* reports, double* latency_s,
                             void* phi_host, void* far_field_host) {
  LM_CHECK(S && state, LM_EINVAL, "bad arguments");
  std::lock_guard<std::mutex> lk(S->B.mu);
  Request* q = S->B.find(id);
  LM_CHECK(q, LM_ENOTFOUND, "unknown request id %llu", (unsigned long long)id);
  *state = q->state;
  if (latency_s) *latency_s = q->t_done > 0 ? q->t_done - q->t_submit : now_s() - q->t_submit;
  if (q->state == LM_DONE) {
    if (reports) std::copy(q->rep.begin(), q->rep.end(), reports);
    if (phi_host) std::memcpy(phi_host, q->phi.get(), q->phi_n * sizeof(double2));
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
  const lm_status st = S->B.cancel(id, now_s());
  LM_CHECK(st != LM_ENOTFOUND, LM_ENOTFOUND, "unknown request id %llu", (unsigned long long)id);
  return st;
}

extern "C" lm_status lm_release(lm_server S, uint64_t id) {
  LM_CHECK(S, LM_EINVAL, "bad arguments");
  const lm_status st = S->B.release(id);
  LM_CHECK(st != LM_ENOTFOUND, LM_ENOTFOUND, "unknown request id %llu", (unsigned long long)id);
  LM_CHECK(st != LM_EINVAL, LM_EINVAL, "request %llu is still queued or running", (unsigned long long)id);
  return st;
}

extern "C" lm_status lm_request_footprint(lm_geom g, int n_rhs, const lm_gmres_opts* o, int64_t* bytes) {
  LM_CHECK(g && bytes && n_rhs >= 1, LM_EINVAL, "bad arguments");
  LM_TRY(check_gmres_opts(o));
  *bytes = footprint(g, *o, n_rhs);
  return LM_OK;
}

extern "C" lm_status lm_server_stats(lm_server S, int64_t* out6) {
  LM_CHECK(S && out6, LM_EINVAL, "bad arguments");
  std::lock_guard<std::mutex> lk(S->B.mu);
  out6[0] = (int64_t)S->B.queue.size();
  out6[1] = S->B.active;
  out6[2] = S->B.used;
  out6[3] = S->rounds;
  out6[4] = S->launches;
  out6[5] = S->fused_rhs;
  return LM_OK;
}

extern "C" lm_status lm_server_memory(lm_server S, int64_t* out3) {
  LM_CHECK(S && out3, LM_EINVAL, "bad arguments");
  std::lock_guard<std::mutex> lk(S->B.mu);
  out3[0] = S->held;
  out3[1] = S->held_spare;
  out3[2] = S->B.used;
  return LM_OK;
}

extern "C" lm_status lm_server_phase_times(lm_server S, double* out11) {
  LM_CHECK(S && out11, LM_EINVAL, "bad arguments");
  double* out8 = out11;
  std::lock_guard<std::mutex> lk(S->B.mu);
  out8[0] = S->km_ms;
  out8[1] = S->gs_ms;
  out8[2] = S->gs_bytes;
  out8[3] = S->m2l_ms;
  out8[4] = S->m2l_flops;
  out8[5] = (double)S->m2l_launches;
  out8[6] = S->round_ms;
  out8[7] = S->finish_ms;
  out11[8] = S->launch_ms;
  out11[9] = S->wait_ms;
  out11[10] = S->step_ms;
  return LM_OK;
}

extern "C" lm_status lm_server_destroy(lm_server S) {
  if (!S) return LM_OK;
  S->B.request_stop();
  if (S->th.joinable()) S->th.join();
  S->B.clear();
  (void)quiesce(S);
  for (Column* c : S->cols) delete c;
  S->cols.clear();
  S->groups.clear();
  for (int i = 0; i < SRV_STREAMS; ++i) {
    if (S->gs[i]) (void)hipStreamDestroy(S->gs[i]);
    if (S->ev[i]) (void)hipEventDestroy(S->ev[i]);
  }
  if (S->ev_main) (void)hipEventDestroy(S->ev_main);
  S->staged.clear();
  for (hipEvent_t e : {S->t0, S->t1, S->t2, S->tu1, S->tu2, S->ev_wait, S->ev_fin})
    if (e) (void)hipEventDestroy(e);
  for (int i = 0; i < SRV_STREAMS; ++i)
    for (int e = 0; e < 16; ++e)
      if (S->sev[i][e]) (void)hipEventDestroy(S->sev[i][e]);
  if (S->s) (void)hipStreamDestroy(S->s);
  delete S;
  return LM_OK;
}
