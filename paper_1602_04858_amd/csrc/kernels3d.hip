// Kernels of the 3-D (hexahedral) path: the level operators are assembled (CSR, FP64),
// so one set of kernels serves every level.
//
//   k3_csr     y = A x, y = b - A x or y += A x for a CSR matrix (level operator,
//              prolongation P, restriction P^T); eight lanes per row
//   k3_colour  one colour step of the symmetric multiplicative vertex-patch smoother
//              (Section 3, eq. smoother-Multiplicative): a block per patch forms the
//              local residual (b - A x) on the patch rows, applies the patch
//              pseudo-inverse (symmetric, stored as rotated diagonals, FP64 or FP32
//              storage, FP64 arithmetic) and adds the correction into x
//   k3_copy_idx  x[i] = b[i] on the essential rows (identity rows of the operator)
#include <hip/hip_runtime.h>

#include <cstdint>

#include "common3d.hpp"

namespace bmg {
namespace {

constexpr int kRowLanes = 8;

__device__ __forceinline__ double lane_group_sum(double s) {
  s += __shfl_xor(s, 1, kRowLanes);
  s += __shfl_xor(s, 2, kRowLanes);
  s += __shfl_xor(s, 4, kRowLanes);
  return s;
}

// MODE 0: y = A x; 1: y = b - A x; 2: y += A x
template <int MODE>
__global__ __launch_bounds__(256) void k3_csr(int64_t nrows, const int32_t* __restrict__ rp,
                                              const int32_t* __restrict__ ci, const double* __restrict__ v,
                                              const double* __restrict__ x, const double* __restrict__ b,
                                              double* __restrict__ y) {
  const int64_t row = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kRowLanes;
  const int sub = threadIdx.x % kRowLanes;
  double s = 0.0;
  if (row < nrows)
    for (int e = rp[row] + sub; e < rp[row + 1]; e += kRowLanes) s += v[e] * x[ci[e]];
  s = lane_group_sum(s);
  if (row < nrows && sub == 0) {
    if (MODE == 0) y[row] = s;
    else if (MODE == 1) y[row] = b[row] - s;
    else y[row] += s;
  }
}

// Patches of one colour are the contiguous range [p0, p0 + gridDim.x) of the level's
// patch list; patch p has the dofs pdofs[poff[p] .. poff[p+1]) (ascending) and its
// symmetric pseudo-inverse A+ at pinv + ioff[p]: with FP64 storage as rotated
// diagonals, R[d n + t] = A+(t, (t + d) mod n) for d = 0 .. n/2 (n (n/2 + 1) entries,
// about half of n^2; the entry (t, (t - d) mod n) below the diagonal is R[d][(t - d)
// mod n] by symmetry), with FP32 storage as the full column-major block.
//
// A patch's work is two dependent streams (the CSR rows of its dofs, then its
// pseudo-inverse, 175 KB for n = 208 in FP64), so the kernel is built for loads in
// flight: the residual rows take eight lanes each with the row loop unrolled, and in
// the product each of the BS/64 waves takes its share of the diagonals (columns) for
// all rows, issuing 32 loads before their FMAs; the partial sums meet in LDS.  BS =
// 1024 serves levels with fewer patches in a colour than CUs (the chains get 4x
// shorter; the CUs would idle anyway), BS = 256 the fine levels.
template <int BS, typename S>
__global__ __launch_bounds__(BS) void k3_colour(int p0, const int64_t* __restrict__ poff,
                                                 const int32_t* __restrict__ pdofs, const int64_t* __restrict__ ioff,
                                                 const S* __restrict__ pinv, const int32_t* __restrict__ rp,
                                                 const int32_t* __restrict__ ci, const double* __restrict__ v,
                                                 double* __restrict__ x, const double* __restrict__ b) {
  // the local residual, twice over (rs[t + n] = rs[t]) for the rotated FP64 product
  __shared__ double rs[2 * kMaxPatch3];
  constexpr int NW = BS / 64;
  __shared__ double part[NW][kMaxPatch3];
  __shared__ int32_t gs[kMaxPatch3];
  const int p = p0 + (int)blockIdx.x;
  const int64_t o = poff[p];
  const int n = (int)(poff[p + 1] - o);
  for (int t = threadIdx.x; t < n; t += BS) gs[t] = pdofs[o + t];
  __syncthreads();
  // local residual: BS/8 rows at a time, eight lanes per row
  const int sub = threadIdx.x % kRowLanes, rl = threadIdx.x / kRowLanes;
  for (int t0 = 0; t0 < n; t0 += BS / kRowLanes) {
    const int t = t0 + rl;
    double s = 0.0;
    int gi = 0;
    if (t < n) {
      gi = gs[t];
      const int e1 = rp[gi + 1];
#pragma unroll 4
      for (int e = rp[gi] + sub; e < e1; e += kRowLanes) s += v[e] * x[ci[e]];
    }
    s = lane_group_sum(s);
    if (t < n && sub == 0) rs[t] = rs[t + n] = b[gi] - s;
  }
  __syncthreads();
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const S* A = pinv + ioff[p];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if constexpr (sizeof(S) == 8) {
    // correction y = A+ r from the rotated diagonals: wave w takes the diagonals d in
    // [d0, d1) for rows t = lane + 64 i, and for each reads both R[d][t] (entry
    // (t, t + d)) and R[d][(t - d) mod n] (entry (t, t - d) by symmetry) in the same
    // iteration: the second read hits the lines the first brought in, so the block's
    // HBM stream is the stored half.  Diagonal 0 has no second entry, nor has d = n/2
    // for even n (its entries are all (t, t + n/2)).  Loads are masked (rows t < n,
    // diagonals below d1; the second index is formed from min(t, n-1), inside the
    // block); 2 x 4 x KC of them are issued before the first wait.  The residual
    // entries r[(t +- d) mod n] are read from the doubled copy at t + d and t - d + n.
    constexpr int KC = 4;
    const int H = n >> 1, HL = n - 1 - H;
    const int q = (H + NW) / NW, d0 = w * q, d1 = min(H + 1, d0 + q);
    for (int db = d0; db < d1; db += KC) {
      double au[4][KC], al[4][KC];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int t = lane + 64 * i, tc = min(t, n - 1);
#pragma unroll
        for (int k = 0; k < KC; ++k) {
          const int d = min(db + k, d1 - 1);
          const bool ok = t < n && db + k < d1;
          int s = tc - d;
          s += s < 0 ? n : 0;
          au[i][k] = ok ? A[d * n + t] : 0.0;
          al[i][k] = (ok && d >= 1 && d <= HL) ? A[d * n + s] : 0.0;
        }
      }
#pragma unroll
      for (int k = 0; k < KC; ++k) {
        const int d = min(db + k, d1 - 1);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int tc = min(lane + 64 * i, n - 1);
          acc[i] += au[i][k] * rs[tc + d] + al[i][k] * rs[tc - d + n];
        }
      }
    }
  } else {
    // FP32 storage keeps the full column-major block (entry (t, u) at u n + t); its
    // narrower stream was already short, and the rotated product's index arithmetic
    // and per-lane gathers cost more than the bytes it saves.  Wave w sums the columns
    // u in [u0, u1) for rows lane + 64 i.
    const int q = (n + NW - 1) / NW, u0 = w * q, u1 = min(n, u0 + q);
    for (int ub = u0; ub < u1; ub += 8) {
      // all 32 loads are issued before the first wait, unconditionally at clamped
      // (in-bounds) indices and widened only in the FMAs (masked FP32 loads were each
      // compiled into a branch with its own wait and conversion); rows t >= n are
      // never stored and columns u >= u1 meet r = 0 below.
      S a[4][8];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int t = lane + 64 * i;
#pragma unroll
        for (int k = 0; k < 8; ++k) a[i][k] = A[(int64_t)min(ub + k, u1 - 1) * n + min(t, n - 1)];
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const double r = ub + k < u1 ? rs[ub + k] : 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i] += (double)a[i][k] * r;
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (lane + 64 * i < n) part[w][lane + 64 * i] = acc[i];
  __syncthreads();
  // every x read of this block is done, and same-colour patches neither share dofs nor
  // couple through A, so the writes race with nothing
  for (int t = threadIdx.x; t < n; t += BS) {
    double y = 0.0;
#pragma unroll
    for (int k = 0; k < NW; ++k) y += part[k][t];
    x[gs[t]] += y;
  }
}

// Small patches (n <= kSmallPatch3: every RT_0 patch, at most 12 inner faces + 12
// open-side faces + 8 pressures) leave most of a 256-thread block idle, so here one
// wave takes one patch and a block four patches of the colour (patch p0 + 4 blockIdx.x
// + w): the wave's 64 lanes form the residual rows eight at a time (eight lanes per
// row), then lanes (half, t) = (lane / 32, lane mod 32) sum the product for row t over
// the diagonals (FP64 rotated) or columns (FP32 full) of parity `half`, and the two
// halves meet by a cross-lane add.  Same-colour patches share no dof and no matrix
// entry, so the four patches of a block do not interact.
constexpr int kSmallPatch3 = 32;

template <typename S>
__global__ __launch_bounds__(256) void k3_colour_small(int p0, int npatch, const int64_t* __restrict__ poff,
                                                       const int32_t* __restrict__ pdofs,
                                                       const int64_t* __restrict__ ioff, const S* __restrict__ pinv,
                                                       const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                                       const double* __restrict__ v, double* __restrict__ x,
                                                       const double* __restrict__ b) {
  __shared__ double rs[4][2 * kSmallPatch3];
  __shared__ int32_t gs[4][kSmallPatch3];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int q = 4 * (int)blockIdx.x + w;  // patch of the colour taken by this wave
  const bool live = q < npatch;
  int n = 0;
  int64_t o = 0;
  if (live) {
    const int p = p0 + q;
    o = poff[p];
    n = (int)(poff[p + 1] - o);
    if (lane < n) gs[w][lane] = pdofs[o + lane];
  }
  __syncthreads();
  // the pseudo-inverse entries of this lane, loaded before the residual's chain of
  // dependent loads so the two overlap: lane (half, t) takes row t and the diagonals
  // d = half, half + 2, ... (FP64 rotated) or columns u = half, half + 2, ... (FP32 full)
  const int half = lane >> 5, t = lane & 31, tc = min(t, max(n - 1, 0));
  const int H = n >> 1, HL = n - 1 - H;
  constexpr int NJ = sizeof(S) == 8 ? kSmallPatch3 / 4 + 1 : kSmallPatch3 / 2;
  double au[NJ], al[NJ];
  if (live) {
    const S* A = pinv + ioff[p0 + q];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      if constexpr (sizeof(S) == 8) {
        // y[t] = sum_d R[d][t] r[t + d] + sum_{1 <= d <= HL} R[d][(t - d) mod n] r[t - d]
        const int d = half + 2 * j;
        int sft = tc - d;
        sft += sft < 0 ? n : 0;
        au[j] = (t < n && d <= H) ? A[d * n + t] : 0.0;
        al[j] = (t < n && d >= 1 && d <= HL) ? A[d * n + sft] : 0.0;
      } else {
        // full column-major block: y[t] = sum_u A[u n + t] r[u]
        const int u = half + 2 * j;
        au[j] = (t < n && u < n) ? (double)A[(int64_t)u * n + t] : 0.0;
        al[j] = 0.0;
      }
    }
  }
  // residual rows: eight at a time, eight lanes each
  const int sub = lane % kRowLanes, rl = lane / kRowLanes;
  for (int t0 = 0; t0 < n; t0 += 64 / kRowLanes) {
    const int tr = t0 + rl;
    double s = 0.0;
    int gi = 0;
    if (tr < n) {
      gi = gs[w][tr];
      const int e1 = rp[gi + 1];
      for (int e = rp[gi] + sub; e < e1; e += kRowLanes) s += v[e] * x[ci[e]];
    }
    s = lane_group_sum(s);
    if (tr < n && sub == 0) rs[w][tr] = rs[w][tr + n] = b[gi] - s;
  }
  __syncthreads();
  double acc = 0.0;
  if (live) {
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int d = half + 2 * j;
      if constexpr (sizeof(S) == 8) {
        const int dd = min(d, H);  // entries beyond H are zero; keep the LDS index in range
        acc += au[j] * rs[w][tc + dd] + al[j] * rs[w][tc - dd + n];
      } else {
        acc += au[j] * rs[w][min(d, max(n - 1, 0))];
      }
    }
  }
  acc += __shfl_xor(acc, 32);
  if (live && half == 0 && t < n) x[gs[w][t]] += acc;
}

__global__ __launch_bounds__(256) void k3_copy_idx(const int32_t* __restrict__ idx, int64_t n,
                                                   const double* __restrict__ src, double* __restrict__ dst) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) dst[idx[i]] = src[idx[i]];
}

inline unsigned blocks_for(int64_t threads) { return (unsigned)((threads + 255) / 256); }

}  // namespace

void launch3_csr(int mode, int64_t nrows, const int32_t* rp, const int32_t* ci, const double* v, const double* x,
                 const double* b, double* y, hipStream_t s) {
  if (nrows <= 0) return;
  const dim3 g(blocks_for(nrows * kRowLanes)), bl(256);
  if (mode == 0) hipLaunchKernelGGL(k3_csr<0>, g, bl, 0, s, nrows, rp, ci, v, x, b, y);
  else if (mode == 1) hipLaunchKernelGGL(k3_csr<1>, g, bl, 0, s, nrows, rp, ci, v, x, b, y);
  else hipLaunchKernelGGL(k3_csr<2>, g, bl, 0, s, nrows, rp, ci, v, x, b, y);
}

template <typename S>
static void colour_t(int p0, int npatch, const int64_t* poff, const int32_t* pdofs, const int64_t* ioff,
                     const S* pinv, const int32_t* rp, const int32_t* ci, const double* v, double* x,
                     const double* b, hipStream_t s) {
  if (npatch < 256)
    hipLaunchKernelGGL((k3_colour<1024, S>), dim3(npatch), dim3(1024), 0, s, p0, poff, pdofs, ioff, pinv, rp, ci, v,
                       x, b);
  else
    hipLaunchKernelGGL((k3_colour<256, S>), dim3(npatch), dim3(256), 0, s, p0, poff, pdofs, ioff, pinv, rp, ci, v, x,
                       b);
}

void launch3_colour(int p0, int npatch, const int64_t* poff, const int32_t* pdofs, const int64_t* ioff,
                    const void* pinv, int sprec, const int32_t* rp, const int32_t* ci, const double* v, double* x,
                    const double* b, int maxn, hipStream_t s) {
  if (npatch <= 0) return;
  if (maxn <= kSmallPatch3) {
    const dim3 g((unsigned)((npatch + 3) / 4)), bl(256);
    if (sprec == 1)
      hipLaunchKernelGGL(k3_colour_small<float>, g, bl, 0, s, p0, npatch, poff, pdofs, ioff, (const float*)pinv, rp,
                         ci, v, x, b);
    else
      hipLaunchKernelGGL(k3_colour_small<double>, g, bl, 0, s, p0, npatch, poff, pdofs, ioff, (const double*)pinv,
                         rp, ci, v, x, b);
    return;
  }
  if (sprec == 1) colour_t(p0, npatch, poff, pdofs, ioff, (const float*)pinv, rp, ci, v, x, b, s);
  else colour_t(p0, npatch, poff, pdofs, ioff, (const double*)pinv, rp, ci, v, x, b, s);
}

void launch3_copy_idx(const int32_t* idx, int64_t n, const double* src, double* dst, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k3_copy_idx, dim3(blocks_for(n)), dim3(256), 0, s, idx, n, src, dst);
}

}  // namespace bmg
