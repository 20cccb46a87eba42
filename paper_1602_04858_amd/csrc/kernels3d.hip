// Kernels of the 3-D (hexahedral) path: the level operators are assembled (CSR, FP64),
// so one set of kernels serves every level.
//
//   k3_csr     y = A x, y = b - A x or y += A x for a CSR matrix (level operator,
//              prolongation P, restriction P^T); eight lanes per row
//   k3_colour  one colour step of the symmetric multiplicative vertex-patch smoother
//              (Section 3, eq. smoother-Multiplicative): a block per patch forms the
//              local residual (b - A x) on the patch rows, applies the patch
//              pseudo-inverse (dense, column-major) and adds the correction into x
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
// pseudo-inverse at pinv + ioff[p], column-major (entry (t, u) at u n + t).
__global__ __launch_bounds__(256) void k3_colour(int p0, const int64_t* __restrict__ poff,
                                                 const int32_t* __restrict__ pdofs, const int64_t* __restrict__ ioff,
                                                 const double* __restrict__ pinv, const int32_t* __restrict__ rp,
                                                 const int32_t* __restrict__ ci, const double* __restrict__ v,
                                                 double* __restrict__ x, const double* __restrict__ b) {
  __shared__ double rs[kMaxPatch3];
  __shared__ int32_t gs[kMaxPatch3];
  const int p = p0 + (int)blockIdx.x;
  const int64_t o = poff[p];
  const int n = (int)(poff[p + 1] - o);
  for (int t = threadIdx.x; t < n; t += blockDim.x) gs[t] = pdofs[o + t];
  __syncthreads();
  // local residual: 32 rows at a time, eight lanes per row
  const int sub = threadIdx.x % kRowLanes, rl = threadIdx.x / kRowLanes;
  for (int t0 = 0; t0 < n; t0 += 256 / kRowLanes) {
    const int t = t0 + rl;
    double s = 0.0;
    int gi = 0;
    if (t < n) {
      gi = gs[t];
      for (int e = rp[gi] + sub; e < rp[gi + 1]; e += kRowLanes) s += v[e] * x[ci[e]];
    }
    s = lane_group_sum(s);
    if (t < n && sub == 0) rs[t] = b[gi] - s;
  }
  __syncthreads();
  // correction y = A+ r; every x read of this block is done, and same-colour patches
  // neither share dofs nor couple through A, so the writes race with nothing
  const double* A = pinv + ioff[p];
  for (int t = threadIdx.x; t < n; t += blockDim.x) {
    double acc = 0.0;
    for (int u = 0; u < n; ++u) acc += A[(int64_t)u * n + t] * rs[u];
    x[gs[t]] += acc;
  }
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

void launch3_colour(int p0, int npatch, const int64_t* poff, const int32_t* pdofs, const int64_t* ioff,
                    const double* pinv, const int32_t* rp, const int32_t* ci, const double* v, double* x,
                    const double* b, hipStream_t s) {
  if (npatch <= 0) return;
  hipLaunchKernelGGL(k3_colour, dim3(npatch), dim3(256), 0, s, p0, poff, pdofs, ioff, pinv, rp, ci, v, x, b);
}

void launch3_copy_idx(const int32_t* idx, int64_t n, const double* src, double* dst, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k3_copy_idx, dim3(blocks_for(n)), dim3(256), 0, s, idx, n, src, dst);
}

}  // namespace bmg
