// Declarations shared by the 3-D host code and its kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace bmg {

// largest vertex-patch space the 3-D kernels take: an interior RT_1 x dQ_1 patch holds
// 12 inner faces x 4 + 8 cells x (12 interior velocity + 8 pressure) = 208 dofs, and
// each open side its patch touches adds 4 boundary faces x 4 normal dofs (three open
// sides at a corner: 256; larger patches -- opposite open sides on a two-cell level --
// are rejected at setup).  The colour kernel holds rows lane + 64 i, i < 4.
constexpr int kMaxPatch3 = 256;

// mode 0: y = A x; 1: y = b - A x; 2: y += A x (CSR, FP64, nrows rows)
void launch3_csr(int mode, int64_t nrows, const int32_t* rp, const int32_t* ci, const double* v, const double* x,
                 const double* b, double* y, hipStream_t s);
// one colour step over patches p0 .. p0 + npatch - 1 of a level; pinv holds doubles
// (sprec 0) or floats (sprec 1); maxn: the largest patch of the level (<= 32: one
// wave per patch)
void launch3_colour(int p0, int npatch, const int64_t* poff, const int32_t* pdofs, const int64_t* ioff,
                    const void* pinv, int sprec, const int32_t* rp, const int32_t* ci, const double* v, double* x,
                    const double* b, int maxn, hipStream_t s);
// dst[idx[i]] = src[idx[i]], i < n
void launch3_copy_idx(const int32_t* idx, int64_t n, const double* src, double* dst, hipStream_t s);

}  // namespace bmg
