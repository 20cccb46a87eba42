// Shared definitions of the HIP library: compile-time sizes of the RT_k x dQ_k
// cell, the reference-element data the kernels consume, and the launcher
// interface between the host code and the kernels.
#pragma once
#include <cstddef>
#include <cstdint>

#include <hip/hip_runtime.h>

namespace bmg {

// Sizes for Raviart-Thomas degree K (Section 2.3): per velocity component the cell
// carries NA x NB coefficients (psi_a along the component direction, L_b across),
// the pressure NB x NB.  NL = local dofs of one cell.
template <int K>
struct Dims {
  static constexpr int NA = K + 2, NB = K + 1;
  static constexpr int NV = NA * NB;         // one velocity component
  static constexpr int NP = NB * NB;         // pressure
  static constexpr int NL = 2 * NV + NP;     // whole cell
  static constexpr int NI = 2 * K * NB;      // interior velocity dofs of a cell
  // vertex-patch slot layouts (ascending global order of the patch dofs):
  //   regular : 4 patch-internal faces, 4 cell interiors, 4 cell pressures
  //   extended: 12 faces (adds the 8 outer faces, used when an outer face of the
  //             patch lies on an open part of the domain boundary)
  static constexpr int NSR = 4 * NB + 4 * NI + 4 * NP;
  static constexpr int NSE = 12 * NB + 4 * NI + 4 * NP;
};

// Reference-element matrices of one level family, in arithmetic T.  Velocity
// local index of either component: a*NB + b (a = psi index along the component,
// b = Legendre index across); pressure local index pb*NB + pa.
//   cell velocity block   = Kmu + kappa h^2 M         (same for u_x and u_y)
//   cell divergence block = -h Dx (u_x), -h Dy (u_y)  (rows pressure, cols velocity)
//   face blocks F[ts] (t = test side, s = trial side; side 0 = the cell with the
//   smaller index, side 1 = the other), used for the tangential component;
//   Nb[0|1] = Dirichlet (Nitsche) face at normal coordinate 0 | 1.
template <typename T, int K>
struct Elem {
  using D = Dims<K>;
  T Kmu[D::NV * D::NV];
  T M[D::NV * D::NV];
  T Dx[D::NP * D::NV];
  T Dy[D::NP * D::NV];
  T F[4][D::NV * D::NV];  // 00, 01, 10, 11
  T Nb[2][D::NV * D::NV];
};

// The cell operator of a cell whose four faces are interior (every cell of an
// interior vertex patch), FP32, for the several-column colour step: Kint = Kmu + F[0]
// + F[3] (the stiffness and both faces' self blocks of the tangential component), the
// mass block M (times kappa h^2), the neighbour blocks F1 = F[1] (upper / right) and
// F2 = F[2] (lower / left), the divergence blocks by columns (DxT[d][q] = Dx[q][d],
// for the velocity rows) and by rows (Dx, Dy, for the pressure rows).  Rows are padded
// to multiples of four entries (zeros) so that the kernel reads them four at a time.
template <typename T, int K>
struct ElemInt {
  using D = Dims<K>;
  static constexpr int NVP = (D::NV + 3) / 4 * 4, NPP = (D::NP + 3) / 4 * 4;
  T Kint[D::NV][NVP];
  T M[D::NV][NVP];
  T F1[D::NV][NVP];
  T F2[D::NV][NVP];
  T DxT[D::NV][NPP];
  T DyT[D::NV][NPP];
  T Dx[D::NP][NVP];
  T Dy[D::NP][NVP];
};

// 1-D re-expansion of a coarse function on child interval s (s = 0 left, 1 right):
// fine coefficient a' of coarse psi_a is Ppsi[s][a'*NA + a], of coarse L_b is
// PL[s][b'*NB + b].
template <typename T, int K>
struct Xfer {
  using D = Dims<K>;
  T Ppsi[2][D::NA * D::NA];
  T PL[2][D::NB * D::NB];
};

// Bit s of a boundary mask: side s (0 x=0, 1 x=1, 2 y=0, 3 y=1) is Dirichlet.

// bfloat16 storage of patch pseudo-inverses: the upper 16 bits of an FP32 value,
// widened to FP32 on load (arithmetic stays FP32).
struct bf16 {
  uint16_t v;
  __host__ __device__ operator float() const { return __uint_as_float((uint32_t)v << 16); }
};

// ---------------------------------------------------------------------------
// Launchers (kernels.hip).  prec: 0 = double, 1 = float vectors; sprec: storage
// of the patch inverses, 0 = double, 1 = float, 2 = bfloat16.  All pointers are
// device pointers.
// ---------------------------------------------------------------------------
struct LevelArgs {
  int N;
  int bcm;
  double h;
  const void* kap;  // kappa of the level, arithmetic `prec`
  int colouring;    // COLOURING_S9 or COLOURING_L8
  int cpb = 0;      // columns per block of several-column colour launches (0: automatic)
};

// Vertex colourings of the smoother: S9, colour (vx mod 3) + 3 (vy mod 3); L8, the
// 8 cosets of the lattice spanned by (2, 2) and (2, -2) (x, y even, x = y mod 4),
// colour (vx mod 2) + 2 (vy mod 2) + 4 [(vx - vy) mod 4 >= 2].  Patch p of a colour
// is the p-th vertex of its class in row-major order.
enum { COLOURING_S9 = 0, COLOURING_L8 = 1 };
__host__ __device__ inline int colour_count(int scheme) { return scheme == COLOURING_L8 ? 8 : 9; }
__host__ __device__ inline int colour_of(int scheme, int vx, int vy) {
  if (scheme != COLOURING_L8) return (vx % 3) + 3 * (vy % 3);
  return (vx & 1) + 2 * (vy & 1) + 4 * ((((vx - vy) % 4 + 4) % 4) >= 2 ? 1 : 0);
}
// L8, colour c: rows vy = py, py + 2, ...; in row vy the vertices vx = ((vy + m) mod 4) + 4 i
// with m = (vx - vy) mod 4 = 2 (c >> 2) + (px - py mod 2)
__host__ __device__ inline int l8_row_count(int N, int vy, int m) {
  const int v0 = (vy + m) & 3;
  return v0 <= N ? (N - v0) / 4 + 1 : 0;
}
__host__ __device__ inline int npatch_of(int scheme, int N, int colour) {
  if (scheme != COLOURING_L8) {
    const int c3x = colour % 3, c3y = colour / 3;
    if (c3x > N || c3y > N) return 0;
    return ((N - c3x) / 3 + 1) * ((N - c3y) / 3 + 1);
  }
  const int px = colour & 1, py = (colour >> 1) & 1, m = 2 * (colour >> 2) + ((px - py) & 1);
  int n = 0;
  for (int vy = py; vy <= N; vy += 2) n += l8_row_count(N, vy, m);
  return n;
}
__host__ __device__ inline void patch_vertex(int scheme, int N, int colour, int p, int& vx, int& vy) {
  if (scheme != COLOURING_L8) {
    const int c3x = colour % 3, c3y = colour / 3;
    const int nvx = (N - c3x) / 3 + 1;
    vx = c3x + 3 * (p % nvx);
    vy = c3y + 3 * (p / nvx);
    return;
  }
  const int px = colour & 1, py = (colour >> 1) & 1, m = 2 * (colour >> 2) + ((px - py) & 1);
  const int nA = l8_row_count(N, py, m), nB = py + 2 <= N ? l8_row_count(N, py + 2, m) : 0;
  const int pair = p / (nA + nB), rem = p - pair * (nA + nB);
  vy = py + 4 * pair + (rem < nA ? 0 : 2);
  vx = ((vy + m) & 3) + 4 * (rem < nA ? rem : rem - nA);
}

// Level kernels work on nrhs vectors stored ld elements apart (grid.y = vector), or,
// with il > 0 (FP32, K >= 1), on interleaved records of il values (a power of two,
// 4..16): entry g of column c at g * il + c, the il - nrhs trailing columns zero.
void launch_op(int K, int prec, const void* elem, const LevelArgs& L, const void* x, const void* b, void* y,
               bool residual, int nrhs, int64_t ld, hipStream_t s, int il = 0);
// omega == 0: one colour step of the multiplicative smoother (b = right-hand side);
// omega > 0: the colour's share of an additive step, x[S] += omega A_S^+ b[S] (b = residual)
// plist: NULL, or the colour-class indices of the npatch patches to apply (a subset)
void launch_colour(int K, int prec, int sprec, const void* elem, const LevelArgs& L, void* x, const void* b,
                   const void* inv, const void* invx, const int32_t* extidx, int colour, int npatch,
                   bool finest, bool packed, int nrhs, int64_t ld, double omega, hipStream_t s,
                   const int32_t* plist = nullptr, int il = 0);
// columns one block of the colour kernel serves (for the byte count of a launch);
// cpb > 0 (a tile parameter) overrides the automatic choice
int colour_columns_per_block(int N, bool packed, int npatch, int nrhs, int cpb = 0);
// The colour step on the interior patches of a level (K = 1 or 2) for FP32 columns in
// interleaved records of rp = 4, 8 or 16 values, with bfloat16 rotated inverses; the
// other patches of the colour are left alone (launch_colour with their list does
// them).  elem_int: ElemInt<float, K>
//   tab: the level's template table (mr_table_entries(K) int4 entries, see below)
void launch_colour_mr(int K, const void* elem_int, const LevelArgs& L, void* x, const void* b, const void* inv,
                      const int32_t* tab, int colour, int npatch, int rp, hipStream_t s);
// Template table of a level for launch_colour_mr (int4 entries): first, for each of the
// NE = 4 NL + 8 NV + NSR gathered entries of one column (the dofs of the 4 cells, the
// tangential components of the 8 outside neighbours, the patch slots), {global index at
// the interior vertex (2, 2), stream (0 x-faces, 1 y-faces, 2 interiors, 3 pressure),
// position in the column's LDS block, 1 if it is read from b}; then for each slot
// {LDS position of its first row contribution, of its second or -1, 0, 0}.  Positions
// use the kernel's LDS layout (mr_layout: padded cell width cw, x part xs, column cs).
// Both launches of a several-column colour step (launch_colour_mr on the npatch_mr
// interior patches, launch_colour on the nlist listed ones with records of rp values)
// as one launch (K = 1 or 2, FP32 with bfloat16 rotated inverses); for small levels.
void launch_colour_fused(int K, const void* elem_int, const void* elem, const LevelArgs& L, void* x, const void* b,
                         const void* inv, const void* invx, const int32_t* extidx, const int32_t* tab, int colour,
                         int npatch_mr, int nlist, const int32_t* plist, int nrhs, int rp, hipStream_t s);
int mr_table_entries(int K);
void mr_steps(int K, int N, int* ax, int* ay);
void mr_layout(int K, int* cw, int* xs, int* cs);
// Setup: the pseudo-inverses of every vertex patch of one colour of a level, FP64 on the
// device, written in the level's storage (sprec; full column-major or rotated); extidx
// as for launch_colour; L.kap is the FP64 kappa of the level; *status |= 1 on a zero pivot
void launch_patch_pinv(int K, int sprec, const void* elem64, const LevelArgs& L, int colour, int npatch, bool rotated,
                       void* inv, void* invx, const int32_t* extidx, int32_t* status, hipStream_t s);
void launch_restrict(int K, int prec, const void* xfer, int Nc, int bcm, const void* rf, void* bc, int nrhs,
                     int64_t ldf, int64_t ldc, hipStream_t s, int il = 0);
void launch_prolong(int K, int prec, const void* xfer, int Nc, int bcm, const void* xc, void* xf, int nrhs,
                    int64_t ldc, int64_t ldf, hipStream_t s, int il = 0);
void launch_coarse(int prec, int n, const double* inv, const void* b, void* x, int nrhs, hipStream_t s, int il = 0);
void launch_fill_zero(int prec, void* x, int64_t n, hipStream_t s);
void launch_identity(int prec, void* x, int64_t n, int64_t col0, int nrhs, hipStream_t s);
// Y = B X for a dense symmetric n x n matrix and nrhs columns of n entries
void launch_dense_gemv(int prec, const void* B, int64_t n, const void* x, void* y, int nrhs, hipStream_t s,
                       int il = 0);
void launch_cast(int to_prec, int from_prec, const void* src, void* dst, int64_t n, hipStream_t s);
// nrhs column-major vectors of n entries (ld apart) -> FP32 interleaved records of w values
// (to_il; the w - nrhs trailing columns zero), or back (to_prec 0: FP64, 1: FP32)
void launch_cast_il(int to_prec, int from_prec, const void* src, void* dst, int64_t n, int64_t ld, int nrhs, int w,
                    bool to_il, hipStream_t s);
// dst = src on the essential (constrained) rows, nrhs columns ld apart
void launch_copy_constrained(int K, int N, int bcm, const double* src, void* dst, int dst_prec, int nrhs, int64_t ld,
                             hipStream_t s);

// FP64 Krylov helpers for nrhs right-hand sides: column r of Krylov vector k at
// V + k ldv + r n; per-right-hand-side results ostride / cstride / dstride apart
void launch_dots(const double* V, int nvec, int64_t ldv, const double* w, int64_t n, double* partial,
                 double* out, int nrhs, int64_t ostride, hipStream_t s);
// w += sign * sum_v coef_v V_v with FP32-stored V (the preconditioned vectors Z of FGMRES)
void launch_axpys_f32(double* w, const float* V, int nvec, int64_t ldv, const double* coef, int64_t cstride,
                      double sign, int64_t n, int nrhs, hipStream_t s);
// y = A_j x in FP64 for FP32-stored x (the FP64 operator applied to a vector of Z)
void launch_op64_f32x(int K, const void* elem64, const LevelArgs& L, const float* x, double* y, int nrhs, int64_t ld,
                      hipStream_t s);
void launch_axpys(double* w, const double* V, int nvec, int64_t ldv, const double* coef, int64_t cstride,
                  double sign, int64_t n, int nrhs, hipStream_t s);
void launch_scale(double* dst, const double* src, const double* denom, int64_t dstride, const int32_t* live,
                  bool take_sqrt, int64_t n, int nrhs, hipStream_t s);
void launch_sub(double* r, const double* b, const double* ax, int64_t n, hipStream_t s);
int dots_partial_count();

// Static device scratch of the allocation-free entry point (bmg_vcycle_noalloc):
// kStaticScratchBytes per device, in a file-scope __device__ array of kernels.hip.
// static_scratch() returns its device address on the current device (looked up
// with hipGetSymbolAddress on the first call per device, then cached).
constexpr size_t kStaticScratchBytes = size_t(256) << 20;
constexpr int kMaxScratchDevices = 64;
hipError_t static_scratch(void** ptr, size_t* bytes);

}  // namespace bmg
