// HIP kernels of the multigrid V-cycle (gfx950).
//
//   k_op       level operator y = A_j x or residual r = b - A_j x, matrix-free:
//              one thread per cell computes the rows the cell owns (its interior
//              and pressure dofs, its left / bottom faces, and the right / top
//              faces on the domain boundary) from cell and face blocks
//              (Section 2.3, eqs. ipbrinkman and Brinkman-weak).
//   k_colour   one colour step of the symmetric multiplicative vertex-patch
//              smoother (Section 3.3): one 64-wide wavefront per patch gathers the
//              patch cells and their face neighbours into LDS, forms the local
//              residual (b - A_j x) on the patch dofs from the same cell / face
//              blocks, multiplies by the stored patch pseudo-inverse (streamed
//              column by column, coalesced) and adds the correction.  Patches of
//              one colour have disjoint write sets and never read each other's
//              writes, so a colour is one launch with no atomics.
//   k_restrict b_{j-1} = P^T r_j and k_prolong x_j += P x_{j-1} (Section 3.1),
//              one thread per coarse cell, tensor-product 1-D re-expansion.
//   k_coarse   x_0 = A_0^{-1} b_0 with the precomputed FP64 inverse.
//   Krylov     FP64 multi-dot (deterministic two-stage reduction), multi-axpy.
#include <algorithm>
#include <mutex>
#include <type_traits>

#include "common.hpp"

namespace bmg {
namespace {

enum { F_INT = 0, F_DIR = 1, F_OPEN = 2 };

template <int K>
struct Idx {
  using D = Dims<K>;
  __device__ __forceinline__ static int n_u(int N) { return 2 * N * (N + 1) * D::NB + D::NI * N * N; }
  __device__ __forceinline__ static int xface(int N, int i, int cy, int b) { return (cy * (N + 1) + i) * D::NB + b; }
  __device__ __forceinline__ static int yface(int N, int j, int cx, int b) {
    return N * (N + 1) * D::NB + (j * N + cx) * D::NB + b;
  }
  __device__ __forceinline__ static int inter(int N, int c, int comp, int a, int b) {
    return 2 * N * (N + 1) * D::NB + c * D::NI + (comp * K + (a - 2)) * D::NB + b;
  }
  __device__ __forceinline__ static int pres(int N, int c, int q) { return n_u(N) + c * D::NP + q; }
  // global index of the local dof d of cell (cx, cy)
  __device__ __forceinline__ static int g(int N, int cx, int cy, int d) {
    const int c = cy * N + cx;
    if (d < D::NV) {
      const int a = d / D::NB, b = d % D::NB;
      return a == 0 ? xface(N, cx, cy, b) : a == 1 ? xface(N, cx + 1, cy, b) : inter(N, c, 0, a, b);
    }
    if (d < 2 * D::NV) {
      const int e = d - D::NV, a = e / D::NB, b = e % D::NB;
      return a == 0 ? yface(N, cy, cx, b) : a == 1 ? yface(N, cy + 1, cx, b) : inter(N, c, 1, a, b);
    }
    return pres(N, c, d - 2 * D::NV);
  }
  // the local dof is an essential normal dof (normal face dof on a Dirichlet side)
  __device__ __forceinline__ static bool cons(int N, int bcm, int cx, int cy, int d) {
    if (d < D::NV) {
      const int a = d / D::NB;
      return (a == 0 && cx == 0 && (bcm & 1)) || (a == 1 && cx == N - 1 && (bcm & 2));
    }
    if (d < 2 * D::NV) {
      const int a = (d - D::NV) / D::NB;
      return (a == 0 && cy == 0 && (bcm & 4)) || (a == 1 && cy == N - 1 && (bcm & 8));
    }
    return false;
  }
};

__device__ __forceinline__ int boundary_type(int bcm, int side) { return ((bcm >> side) & 1) ? F_DIR : F_OPEN; }

// Workgroup barrier that orders LDS only: global loads issued before it stay in
// flight (a full __syncthreads() would wait for every outstanding global access).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Orders this wave's own LDS accesses (values one lane wrote, another lane of the same
// wave reads): a wave's LDS instructions execute in program order, so this only keeps
// the compiler from moving accesses across it.  Waves of a block do not wait for each
// other here.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// one velocity component (NV values, comp 0 = u_x, 1 = u_y) of a cell; essential dofs read as 0
// One column of a vector in interleaved records: entry g at p[g * s] (p already points
// at the column's first entry).  Column-major vectors are read through plain pointers.
template <typename T>
struct Rec {
  T* p;
  int64_t s;
  __device__ __forceinline__ T& operator[](int64_t g) const { return p[g * s]; }
};
// the view of a column: IL records of width s, or the plain pointer
template <bool IL, typename T>
__device__ __forceinline__ auto col_view(T* p, int64_t s) {
  if constexpr (IL) return Rec<T>{p, s};
  else return p;
}

template <int K, typename T, typename XA>
__device__ __forceinline__ void load_comp(XA x, int N, int bcm, int cx, int cy, int comp, T* out) {
  using D = Dims<K>;
#pragma unroll
  for (int d = 0; d < D::NV; ++d) {
    const int dd = comp * D::NV + d;
    out[d] = Idx<K>::cons(N, bcm, cx, cy, dd) ? T(0) : T(x[Idx<K>::g(N, cx, cy, dd)]);
  }
}

template <int K, typename T, typename XA>
__device__ __forceinline__ void load_pres(XA x, int N, int cx, int cy, T* out) {
  using D = Dims<K>;
  const int base = Idx<K>::pres(N, cy * N + cx, 0);
#pragma unroll
  for (int q = 0; q < D::NP; ++q) out[q] = T(x[base + q]);
}

// Row d of one velocity component of a cell: cell block, divergence coupling and
// the two faces across which this component is tangential ("lower" = normal
// coordinate 0, where the cell is the higher-index side 1; "upper" = 1, side 0).
template <typename T, int K>
__device__ __forceinline__ T comp_row(const Elem<T, K>& E, int d, const T* xs, const T* p, const T* Dm, T khh, T mh,
                                      int tl, const T* nl, int tu, const T* nu) {
  using D = Dims<K>;
  constexpr int NV = D::NV;
  T s = T(0);
#pragma unroll
  for (int e = 0; e < NV; ++e) s += (E.Kmu[d * NV + e] + khh * E.M[d * NV + e]) * xs[e];
#pragma unroll
  for (int q = 0; q < D::NP; ++q) s += mh * Dm[q * NV + d] * p[q];
  if (tl == F_INT) {
#pragma unroll
    for (int e = 0; e < NV; ++e) s += E.F[3][d * NV + e] * xs[e] + E.F[2][d * NV + e] * nl[e];
  } else if (tl == F_DIR) {
#pragma unroll
    for (int e = 0; e < NV; ++e) s += E.Nb[0][d * NV + e] * xs[e];
  }
  if (tu == F_INT) {
#pragma unroll
    for (int e = 0; e < NV; ++e) s += E.F[0][d * NV + e] * xs[e] + E.F[1][d * NV + e] * nu[e];
  } else if (tu == F_DIR) {
#pragma unroll
    for (int e = 0; e < NV; ++e) s += E.Nb[1][d * NV + e] * xs[e];
  }
  return s;
}

template <typename T, int K>
__device__ __forceinline__ T pres_row(const Elem<T, K>& E, int q, const T* ux, const T* uy, T mh) {
  using D = Dims<K>;
  T s = T(0);
#pragma unroll
  for (int e = 0; e < D::NV; ++e) s += E.Dx[q * D::NV + e] * ux[e] + E.Dy[q * D::NV + e] * uy[e];
  return mh * s;
}

// ---------------------------------------------------------------------------
// Level operator
// ---------------------------------------------------------------------------
// XT: element type of x (T, or float for the FP64 operator applied to FP32-stored
// Krylov vectors; loads are widened to T)
// IL: the vectors are interleaved records of ld values (a power of two); thread ->
// (cell, column), column fastest, so that the lanes of a cell read whole records.
// Otherwise one thread per cell and blockIdx.y = column (ld apart).
template <typename T, int K, bool RES, typename XT = T, bool IL = false>
__global__ __launch_bounds__(256) void k_op(const Elem<T, K>* __restrict__ Ep, int N, int bcm, T h,
                                            const T* __restrict__ kap, const XT* __restrict__ x_,
                                            const T* __restrict__ b_, T* __restrict__ y_, int64_t ld) {
  using D = Dims<K>;
  using I = Idx<K>;
  constexpr int NV = D::NV, NP = D::NP, NA = D::NA, NB = D::NB;
  int c;
  int64_t co;
  if constexpr (IL) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    c = (int)(t >> __builtin_ctzll(ld));
    co = t & (ld - 1);
  } else {
    c = blockIdx.x * blockDim.x + threadIdx.x;
    co = blockIdx.y * ld;
  }
  if (c >= N * N) return;
  const auto x = col_view<IL>(x_ + co, ld);
  const auto y = col_view<IL>(y_ + co, ld);
  const auto b = col_view<IL>(RES ? b_ + co : b_, ld);
  const Elem<T, K>& E = *Ep;
  const int cx = c % N, cy = c / N;
  const T mh = -h, hh = h * h;
  const int tL = cx > 0 ? F_INT : boundary_type(bcm, 0);
  const int tR = cx < N - 1 ? F_INT : boundary_type(bcm, 1);
  const int tD = cy > 0 ? F_INT : boundary_type(bcm, 2);
  const int tU = cy < N - 1 ? F_INT : boundary_type(bcm, 3);
  auto out = [&](int gi, T v) {
    if (RES) y[gi] = b[gi] - v;
    else y[gi] = v;
  };
  auto ident = [&](int gi) {
    if (RES) y[gi] = b[gi] - T(x[gi]);
    else y[gi] = T(x[gi]);
  };

  T ux[NV], uy[NV], p[NP], n0[NV], n1[NV];
  load_comp<K>(x, N, bcm, cx, cy, 0, ux);
  load_comp<K>(x, N, bcm, cx, cy, 1, uy);
  load_pres<K>(x, N, cx, cy, p);
  const T khh = kap[c] * hh;

  // u_x rows (tangential across the bottom / top faces)
  if (tD == F_INT) load_comp<K>(x, N, bcm, cx, cy - 1, 0, n0);
  if (tU == F_INT) load_comp<K>(x, N, bcm, cx, cy + 1, 0, n1);
  T zx[NV];
#pragma unroll
  for (int d = 0; d < NV; ++d) zx[d] = comp_row<T, K>(E, d, ux, p, E.Dx, khh, mh, tD, n0, tU, n1);
  // u_y rows (tangential across the left / right faces)
  if (tL == F_INT) load_comp<K>(x, N, bcm, cx - 1, cy, 1, n0);
  if (tR == F_INT) load_comp<K>(x, N, bcm, cx + 1, cy, 1, n1);
  T zy[NV];
#pragma unroll
  for (int d = 0; d < NV; ++d) zy[d] = comp_row<T, K>(E, d, uy, p, E.Dy, khh, mh, tL, n0, tR, n1);

  // interior velocity and pressure rows belong to this cell only
#pragma unroll
  for (int a = 2; a < NA; ++a)
#pragma unroll
    for (int bb = 0; bb < NB; ++bb) {
      out(I::inter(N, c, 0, a, bb), zx[a * NB + bb]);
      out(I::inter(N, c, 1, a, bb), zy[a * NB + bb]);
    }
#pragma unroll
  for (int q = 0; q < NP; ++q) out(I::pres(N, c, q), pres_row<T, K>(E, q, ux, uy, mh));

  // right / top faces on the domain boundary
  if (cx == N - 1) {
#pragma unroll
    for (int bb = 0; bb < NB; ++bb) {
      const int gi = I::xface(N, N, cy, bb);
      if (bcm & 2) ident(gi);
      else out(gi, zx[1 * NB + bb]);
    }
  }
  if (cy == N - 1) {
#pragma unroll
    for (int bb = 0; bb < NB; ++bb) {
      const int gi = I::yface(N, N, cx, bb);
      if (bcm & 8) ident(gi);
      else out(gi, zy[1 * NB + bb]);
    }
  }

  // left face: this cell (a = 0) plus the left neighbour (a = 1)
  T acc[NB];
#pragma unroll
  for (int bb = 0; bb < NB; ++bb) acc[bb] = zx[bb];
  if (cx > 0) {
    T lx[NV], lp[NP];
    load_comp<K>(x, N, bcm, cx - 1, cy, 0, lx);
    load_pres<K>(x, N, cx - 1, cy, lp);
    if (tD == F_INT) load_comp<K>(x, N, bcm, cx - 1, cy - 1, 0, n0);
    if (tU == F_INT) load_comp<K>(x, N, bcm, cx - 1, cy + 1, 0, n1);
    const T lk = kap[c - 1] * hh;
#pragma unroll
    for (int bb = 0; bb < NB; ++bb) acc[bb] += comp_row<T, K>(E, NB + bb, lx, lp, E.Dx, lk, mh, tD, n0, tU, n1);
  }
#pragma unroll
  for (int bb = 0; bb < NB; ++bb) {
    const int gi = I::xface(N, cx, cy, bb);
    if (cx == 0 && (bcm & 1)) ident(gi);
    else out(gi, acc[bb]);
  }
  // bottom face: this cell (a = 0) plus the lower neighbour (a = 1)
#pragma unroll
  for (int bb = 0; bb < NB; ++bb) acc[bb] = zy[bb];
  if (cy > 0) {
    T dy[NV], dp[NP];
    load_comp<K>(x, N, bcm, cx, cy - 1, 1, dy);
    load_pres<K>(x, N, cx, cy - 1, dp);
    if (tL == F_INT) load_comp<K>(x, N, bcm, cx - 1, cy - 1, 1, n0);
    if (tR == F_INT) load_comp<K>(x, N, bcm, cx + 1, cy - 1, 1, n1);
    const T dk = kap[c - N] * hh;
#pragma unroll
    for (int bb = 0; bb < NB; ++bb) acc[bb] += comp_row<T, K>(E, NB + bb, dy, dp, E.Dy, dk, mh, tL, n0, tR, n1);
  }
#pragma unroll
  for (int bb = 0; bb < NB; ++bb) {
    const int gi = I::yface(N, cy, cx, bb);
    if (cy == 0 && (bcm & 4)) ident(gi);
    else out(gi, acc[bb]);
  }
}

// ---------------------------------------------------------------------------
// Smoother colour step
// ---------------------------------------------------------------------------
// Face groups of the extended patch layout (ascending global order):
//   0: x-face (vx-1, vy-1)  slot 0 left          6: y-face (vy-1, vx-1) slot 0 bottom
//   1: x-face (vx,   vy-1)  slot 0 | slot 1      7: y-face (vy-1, vx)   slot 1 bottom
//   2: x-face (vx+1, vy-1)  slot 1 right         8: y-face (vy, vx-1)   slot 0 | slot 2
//   3: x-face (vx-1, vy)    slot 2 left          9: y-face (vy, vx)     slot 1 | slot 3
//   4: x-face (vx,   vy)    slot 2 | slot 3     10: y-face (vy+1, vx-1) slot 2 top
//   5: x-face (vx+1, vy)    slot 3 right        11: y-face (vy+1, vx)   slot 3 top
// The regular layout keeps groups 1, 4, 8, 9.  Slot s is the cell
// (vx - 1 + (s & 1), vy - 1 + (s >> 1)).  Entry: (slotA, kindA, slotB, kindB) with
// kind 0 = u_x at a = 0, 1 = u_x at a = 1, 2 = u_y at a = 0, 3 = u_y at a = 1.
// Packed form of that table (no memory access): byte g of the three words holds
// slotA | kindA << 2 | slotB << 4 | kindB << 6; bit g of kSingle marks groups with
// one cell only; kRegularGroups holds the four regular groups as nibbles.
constexpr uint32_t kGroupW0 = 0x02051400u, kGroupW1 = 0x09080736u, kGroupW2 = 0x0F0EBDACu;
constexpr uint32_t kSingle = 0xCEDu, kRegularGroups = 0x9841u;

__device__ __forceinline__ void group_info(int grp, int& sA, int& kA, int& sB, int& kB) {
  const uint32_t wd = grp < 4 ? kGroupW0 : grp < 8 ? kGroupW1 : kGroupW2;
  const uint32_t by = (wd >> ((grp & 3) * 8)) & 0xffu;
  sA = by & 3;
  kA = (by >> 2) & 3;
  kB = (by >> 6) & 3;
  sB = ((kSingle >> grp) & 1u) ? -1 : (int)((by >> 4) & 3);
}

template <int K>
__device__ __forceinline__ int kind_to_local(int kind, int b) {
  using D = Dims<K>;
  return (kind >= 2 ? D::NV : 0) + (kind & 1) * D::NB + b;
}

// Entry t of the patch layout: global index gi (-1 if not part of the patch
// space) and the positions zA / zB of the row contributions of the patch cells
// (slot * NL + local dof) that sum to row gi (zB >= 0 only for faces inside the patch).
// INT: the vertex is at least two cells from the boundary (every cell and neighbour
// in the domain, nothing essential, regular layout).
template <int K, bool INT = false>
__device__ __forceinline__ void decode_slot(int t, bool ext, int vx, int vy, int N, int bcm, int& gi, int& zA,
                                            int& zB) {
  using D = Dims<K>;
  using I = Idx<K>;
  constexpr int NB = D::NB, NI = D::NI, NP = D::NP, NV = D::NV, NL = D::NL;
  auto in_dom = [&](int cx, int cy) { return INT || (cx >= 0 && cx < N && cy >= 0 && cy < N); };
  gi = -1;
  zA = -1;
  zB = -1;
  const int nf = ext ? 12 : 4;
  if (t < nf * NB) {
    const int grp = ext ? t / NB : (int)((kRegularGroups >> (4 * (t / NB))) & 0xfu);
    const int bb = t % NB;
    int sA, kA, sB, kB;
    group_info(grp, sA, kA, sB, kB);
    const int axA = vx - 1 + (sA & 1), ayA = vy - 1 + (sA >> 1);
    const bool vA = in_dom(axA, ayA);
    bool vB = false;
    int axB = 0, ayB = 0;
    if (sB >= 0) {
      axB = vx - 1 + (sB & 1);
      ayB = vy - 1 + (sB >> 1);
      vB = in_dom(axB, ayB);
    }
    bool ok;
    int cxu, cyu, du;
    if (sB >= 0) {
      ok = vA || vB;
      cxu = vA ? axA : axB;
      cyu = vA ? ayA : ayB;
      du = kind_to_local<K>(vA ? kA : kB, bb);
    } else {
      // outer face: part of the patch space only on the domain boundary
      int ox = axA, oy = ayA;
      if (kA == 0) ox -= 1;
      else if (kA == 1) ox += 1;
      else if (kA == 2) oy -= 1;
      else oy += 1;
      ok = vA && !in_dom(ox, oy);
      cxu = axA;
      cyu = ayA;
      du = kind_to_local<K>(kA, bb);
    }
    if (ok && (INT || !I::cons(N, bcm, cxu, cyu, du))) {
      gi = I::g(N, cxu, cyu, du);
      // zA is always the first existing contribution, zB the second (if any)
      const int za = vA ? sA * NL + kind_to_local<K>(kA, bb) : -1;
      const int zb = vB ? sB * NL + kind_to_local<K>(kB, bb) : -1;
      zA = za >= 0 ? za : zb;
      zB = za >= 0 ? zb : -1;
    }
  } else {
    const int e = t - nf * NB;
    int s, d;
    // RT_0 has no interior dofs (NI = 0): the branch is dead and the divisors are
    // kept nonzero so that it stays well defined
    constexpr int NId = NI > 0 ? NI : 1, KNB = K > 0 ? K * NB : 1;
    if (e < 4 * NI) {
      s = e / NId;
      const int w2 = e % NId, comp = w2 / KNB, rem = w2 % KNB;
      d = comp * NV + (2 + rem / NB) * NB + rem % NB;
    } else {
      s = (e - 4 * NI) / NP;
      d = 2 * NV + (e - 4 * NI) % NP;
    }
    const int cx = vx - 1 + (s & 1), cy = vy - 1 + (s >> 1);
    if (in_dom(cx, cy)) {
      gi = I::g(N, cx, cy, d);
      zA = s * NL + d;
    }
  }
}

// TAG only separates the launches of the finest level (TAG = 1) from the others
// in profiler output; the code is identical.
//
// Latency structure: everything that does not depend on x is issued first -- the
// element matrices are copied to LDS, the patch-inverse column of this lane is
// prefetched into registers (RT_1, regular layout), the patch layout is decoded
// arithmetically and b on the patch is loaded -- so the dependent chain is one
// gather of x, the local residual in LDS, an FMA chain on registers and the store.
template <typename T, typename S, int K, int TAG, bool PKD, bool MC, bool ADD, bool IL = false>
__global__ __launch_bounds__(256) void k_colour(const Elem<T, K>* __restrict__ Ep, int N, int bcm, T h,
                                                const T* __restrict__ kap, T* __restrict__ x,
                                                const T* __restrict__ b, const S* __restrict__ inv,
                                                const S* __restrict__ invx, const int32_t* __restrict__ extidx,
                                                int colour, int scheme, int npatch, int64_t ld, int nrhs,
                                                int ncol, T omega, const int32_t* __restrict__ plist) {
#define BMG_BX (blockIdx.x)
#define BMG_BY (blockIdx.y)
#define BMG_GDIM ((int)gridDim.x)
#include "colour_kernel.inc"
#undef BMG_BX
#undef BMG_BY
#undef BMG_GDIM
}

// ---------------------------------------------------------------------------
// Colour step for several right-hand sides (up to 16 columns, FP32 arithmetic,
// bfloat16 rotated patch inverses), interior vertices only: the patch cells and their
// neighbours are all in the domain and hold no essential dof, so every coefficient of
// the local operator is the same for the whole wave (LDS broadcasts), and the global
// index of every gathered entry is that of the level's template patch (vertex (2, 2),
// table from setup) shifted linearly with the vertex.  One wave per patch:
//   1. x of the 4 cells and of the 8 neighbouring components, and b on the patch, of
//      every column, gathered column by column (coalesced over the entries) into LDS;
//   2. lane (cell s, column c) computes the NL local rows of its cell for its column
//      from registers: the cell-local operator of eq. (ipbrinkman) / (Brinkman-weak)
//      with the interior-face blocks summed into one self block;
//   3. the residual of the patch rows, split into bfloat16 hi + lo parts, is the B
//      operand of v_mfma_f32_16x16x32_bf16; the A operand is gathered from the
//      rotated inverse staged in LDS (A+[i][k] = R[(k - i) mod n][i] for
//      (k - i) mod n <= n/2, else R[(i - k) mod n][k]); Y = A+ (r_hi + r_lo) accumulates
//      in FP32;
//   4. Y goes through LDS to coalesced read-modify-writes x[S] += Y.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float fx4 __attribute__((ext_vector_type(4)));

}  // namespace

template <int K>
struct MrDims {
  using D = Dims<K>;
  static constexpr int CW = (D::NL + 3) / 4 * 4;             // padded cell width in LDS
  static constexpr int XS = 4 * CW + 8 * D::NV;              // x of one column: cells, then neighbours
  static constexpr int CS = XS + D::NSR;                     // one column: x part, then b on the slots
  static constexpr int NE = 4 * D::NL + 8 * D::NV + D::NSR;  // gathered entries per column
  static constexpr int NPR = D::NSR * (D::NSR / 2 + 1);      // stored rotated entries
  static constexpr int NKS = (D::NSR + 31) / 32;             // k-steps of the product
  static constexpr int NRT = (D::NSR + 15) / 16;             // row tiles of the product
};

// stream of a global index (0 x-faces, 1 y-faces, 2 cell interiors, 3 pressure) and the
// per-stream change of the index when the vertex moves by one in x / in y
template <int K>
__host__ __device__ inline void mr_stream_steps(int N, int* ax, int* ay) {
  using D = Dims<K>;
  ax[0] = D::NB;
  ay[0] = (N + 1) * D::NB;
  ax[1] = D::NB;
  ay[1] = N * D::NB;
  ax[2] = D::NI;
  ay[2] = N * D::NI;
  ax[3] = D::NP;
  ay[3] = N * D::NP;
}

namespace {

template <int K>
__global__ __launch_bounds__(256, 4) void k_colour_mr(const ElemInt<float, K>* __restrict__ Ei, int N, float h,
                                                  const float* __restrict__ kap, float* __restrict__ x,
                                                  const float* __restrict__ b, const bf16* __restrict__ inv,
                                                  const int4* __restrict__ tab, int colour, int scheme, int npatch,
                                                  int rp) {
#define BMG_MR_BX (blockIdx.x)
#define BMG_MR_GDIM ((int)gridDim.x)
#include "colour_mr_kernel.inc"
#undef BMG_MR_BX
#undef BMG_MR_GDIM
}

// ---------------------------------------------------------------------------
// One colour step of a small level in one launch: the blocks below mr_blocks run the
// several-column body on the interior patches, the others the general body (one
// column per block, interleaved records) on the listed boundary patches of the same
// colour.  The two sets of patches share no dof (same colour), so they may run at
// once; on the latency-bound small levels this halves the launches of a smoothing
// step.  The two bodies' LDS share one union.
// ---------------------------------------------------------------------------
template <int K>
struct MrShared {
  using M = MrDims<K>;
  __attribute__((aligned(16))) float buf[16 * M::CS + 4];
  __attribute__((aligned(16))) uint16_t apw[(M::NPR + 7) / 8 * 8 + 8];
  int sgi[Dims<K>::NSR + 1], spa[Dims<K>::NSR + 1], spb[Dims<K>::NSR + 1];
};

template <typename T, typename S, int K, bool PKD, bool MC>
struct ColourShared {
  using D = Dims<K>;
  static constexpr int NL = D::NL, NV = D::NV, NP = D::NP, NSR = D::NSR, NSE = D::NSE;
  static constexpr bool PK = PKD && (K <= 1 || sizeof(S) <= 4);
  static constexpr bool MF = MC && !PK && sizeof(T) == 4;
  static constexpr int NPR = NSR * (NSR / 2 + 1);
  static constexpr bool OVL = PK && !MC;
  static constexpr int WSB = (int)sizeof(T) * (4 * NL + 8 * NV + 4 * NL);
  static constexpr int APB = (int)sizeof(S) * (PK ? NPR : 1);
  static constexpr int RB = ((OVL ? (WSB > APB ? WSB : APB) : WSB + APB) + 15) / 16 * 16;
  Elem<T, K> Es;
  T zblk[NP * NV];
  T rs[4][NSE];
  T rsa[MF ? 4 : 1][MF ? 16 : 1][MF ? NSE : 1];
  int gis[MF ? 4 : 1][MF ? NSE : 1];
  __attribute__((aligned(16))) unsigned char wpool[4 * RB];
};

template <int K>
__global__ __launch_bounds__(256) void k_colour_fused(const ElemInt<float, K>* __restrict__ Ei,
                                                      const int4* __restrict__ tab, int mr_npatch, int mr_blocks,
                                                      const Elem<float, K>* __restrict__ Ep, int N, int bcm, float h,
                                                      const float* __restrict__ kap, float* __restrict__ x,
                                                      const float* __restrict__ b, const bf16* __restrict__ inv,
                                                      const bf16* __restrict__ invx,
                                                      const int32_t* __restrict__ extidx, int colour, int scheme,
                                                      int npatch, int64_t ld, int nrhs,
                                                      const int32_t* __restrict__ plist, int nbx) {
  union FusedShared {
    MrShared<K> m;
    ColourShared<float, bf16, K, true, false> c;
  };
  __shared__ FusedShared fsh;
  if ((int)blockIdx.x < mr_blocks) {
    const int rp = (int)ld;
    const int npatch_all = npatch;
    (void)npatch_all;
    {
      const int npatch = mr_npatch;
#define BMG_MR_SHARED fsh.m
#define BMG_MR_BX (blockIdx.x)
#define BMG_MR_GDIM (mr_blocks)
#include "colour_mr_kernel.inc"
#undef BMG_MR_SHARED
#undef BMG_MR_BX
#undef BMG_MR_GDIM
    }
  } else {
    using T = float;
    using S = bf16;
    constexpr bool PKD = true, MC = false, ADD = false, IL = true;
    const int ncol = 1;
    const T omega = 0.0f;
    const unsigned vb = blockIdx.x - (unsigned)mr_blocks;
#define BMG_COLOUR_SHARED fsh.c
#define BMG_BX (vb % (unsigned)nbx)
#define BMG_BY (vb / (unsigned)nbx)
#define BMG_GDIM (nbx)
#include "colour_kernel.inc"
#undef BMG_COLOUR_SHARED
#undef BMG_BX
#undef BMG_BY
#undef BMG_GDIM
  }
}

// ---------------------------------------------------------------------------
// Setup: vertex-patch pseudo-inverses on the device (Section 3.3: the local Ritz
// projection of every vertex patch), one 256-thread block per patch, FP64 throughout.
//   1. the slot layout of the patch (the same decode as the colour step) and the
//      patch matrix A_S = A_j[S, S], assembled from the cell and face blocks: entry
//      (t, u) sums the couplings between the (at most two) cell-local positions of
//      slot t and those of slot u;
//   2. if no free normal dof of the patch lies on the domain boundary, the constant
//      patch pressure (the (0,0) Legendre coefficient of every patch cell,
//      normalised) spans the kernel of A_S: the matrix is bordered with it, and the
//      leading block of the bordered inverse is the pseudo-inverse with zero patch
//      mean pressure;
//   3. Gauss-Jordan elimination in place in LDS with partial (row) pivoting, the
//      row interchanges undone on the columns at the end;
//   4. the inverse written in the storage of the level: full column-major blocks, or
//      the rotated diagonals of its symmetric part, in the storage precision (S).
// A zero pivot sets *status (the host reports BMG_E_SINGULAR).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint16_t bf16_rne(double d) {
  const float f = (float)d;
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
template <typename S>
__device__ __forceinline__ S store_as(double v);
template <>
__device__ __forceinline__ double store_as<double>(double v) { return v; }
template <>
__device__ __forceinline__ float store_as<float>(double v) { return (float)v; }
template <>
__device__ __forceinline__ bf16 store_as<bf16>(double v) { return bf16{bf16_rne(v)}; }

// Coupling of cell-local position pa = s NL + d (test) with pb = s2 NL + e (trial)
// inside the patch around (vx, vy): the cell block, the divergence blocks, the face
// self terms (interior face, Dirichlet Nitsche face, nothing on an open face) and
// the neighbour block across a face shared by two patch cells.
template <int K>
__device__ double patch_coupling(const Elem<double, K>& E, int pa, int pb, int vx, int vy, int N, int bcm, double h,
                                 const double* __restrict__ kap) {
  using D = Dims<K>;
  constexpr int NV = D::NV, NL = D::NL;
  const int s = pa / NL, d = pa % NL, s2 = pb / NL, e = pb % NL;
  const int cx = vx - 1 + (s & 1), cy = vy - 1 + (s >> 1);
  const bool vd = d < 2 * NV, ve = e < 2 * NV;
  if (s == s2) {
    if (vd && ve) {
      const int comp = d / NV;
      if (e / NV != comp) return 0.0;
      const int dd = d % NV, ee = e % NV;
      double v = E.Kmu[dd * NV + ee] + kap[cy * N + cx] * h * h * E.M[dd * NV + ee];
      for (int up = 0; up < 2; ++up) {
        int ncx = cx, ncy = cy, side;
        if (comp == 0) {
          ncy += up ? 1 : -1;
          side = up ? 3 : 2;
        } else {
          ncx += up ? 1 : -1;
          side = up ? 1 : 0;
        }
        if (ncx >= 0 && ncx < N && ncy >= 0 && ncy < N) v += E.F[up ? 0 : 3][dd * NV + ee];
        else if ((bcm >> side) & 1) v += E.Nb[up][dd * NV + ee];
      }
      return v;
    }
    if (vd && !ve) {
      const int comp = d / NV;
      return -h * (comp ? E.Dy : E.Dx)[(e - 2 * NV) * NV + d % NV];
    }
    if (!vd && ve) {
      const int comp = e / NV;
      return -h * (comp ? E.Dy : E.Dx)[(d - 2 * NV) * NV + e % NV];
    }
    return 0.0;
  }
  if (!vd || !ve) return 0.0;
  const int comp = d / NV;
  if (e / NV != comp) return 0.0;
  const int cx2 = vx - 1 + (s2 & 1), cy2 = vy - 1 + (s2 >> 1);
  const int dd = d % NV, ee = e % NV;
  // the component is tangential across horizontal faces (u_x) or vertical ones (u_y)
  if (comp == 0 && cx2 == cx && cy2 == cy + 1) return E.F[1][dd * NV + ee];
  if (comp == 0 && cx2 == cx && cy2 == cy - 1) return E.F[2][dd * NV + ee];
  if (comp == 1 && cy2 == cy && cx2 == cx + 1) return E.F[1][dd * NV + ee];
  if (comp == 1 && cy2 == cy && cx2 == cx - 1) return E.F[2][dd * NV + ee];
  return 0.0;
}

// Face slot t of the layout lies on the domain boundary (its face has one cell in
// the domain); meaningful for slots that belong to the patch space.
template <int K>
__device__ __forceinline__ bool slot_on_boundary(int t, bool ext, int vx, int vy, int N) {
  using D = Dims<K>;
  const int nf = ext ? 12 : 4;
  if (t >= nf * D::NB) return false;
  const int grp = ext ? t / D::NB : (int)((kRegularGroups >> (4 * (t / D::NB))) & 0xfu);
  int sA, kA, sB, kB;
  group_info(grp, sA, kA, sB, kB);
  if (sB < 0) return true;  // outer face: in the patch space only on the domain boundary
  const int axA = vx - 1 + (sA & 1), ayA = vy - 1 + (sA >> 1);
  const int axB = vx - 1 + (sB & 1), ayB = vy - 1 + (sB >> 1);
  const bool inA = axA >= 0 && axA < N && ayA >= 0 && ayA < N;
  const bool inB = axB >= 0 && axB < N && ayB >= 0 && ayB < N;
  return inA != inB;
}

template <int K, typename S, bool ROT>
__global__ __launch_bounds__(512) void k_patch_pinv(const Elem<double, K>* __restrict__ Ep, int N, int bcm, double h,
                                                    const double* __restrict__ kap, int colour, int scheme,
                                                    S* __restrict__ inv, S* __restrict__ invx,
                                                    const int32_t* __restrict__ extidx, int32_t* __restrict__ status) {
  using D = Dims<K>;
  constexpr int NSR = D::NSR, NSE = D::NSE, NL = D::NL, NV = D::NV, NP = D::NP;
  constexpr int MM = NSE + 1;  // largest bordered size
  static_assert(MM <= 128, "the update loop covers columns l and l + 64");
  __shared__ double a[MM * MM];
  __shared__ double fcol[MM], prow[MM];
  __shared__ int zA[NSE], zB[NSE], gis[NSE], cidx[NSE], slot[MM];
  __shared__ int s_n, s_sing, s_piv, s_bad;
  __shared__ int pv[MM];
  const int p = blockIdx.x, tid = threadIdx.x;
  int vx, vy;
  patch_vertex(scheme, N, colour, p, vx, vy);
  const int ext = extidx[p];
  const bool isx = ext >= 0;
  const int ns = isx ? NSE : NSR;
  const Elem<double, K>& E = *Ep;
  // 1. layout
  for (int t = tid; t < ns; t += blockDim.x) {
    int g, za, zb;
    decode_slot<K, false>(t, isx, vx, vy, N, bcm, g, za, zb);
    gis[t] = g;
    zA[t] = za;
    zB[t] = zb;
  }
  __syncthreads();
  if (tid == 0) {
    int n = 0;
    bool bnd = false;
    for (int t = 0; t < ns; ++t) {
      if (gis[t] >= 0) {
        slot[n] = t;
        cidx[t] = n++;
        bnd = bnd || slot_on_boundary<K>(t, isx, vx, vy, N);
      } else {
        cidx[t] = -1;
      }
    }
    s_n = n;
    s_sing = bnd ? 0 : 1;
    s_bad = 0;
  }
  __syncthreads();
  const int n = s_n, m = n + s_sing;
  // constant patch pressure: the (0,0) coefficient of every patch cell's pressure
  int cnt = 0;
  for (int i = 0; i < n; ++i) {
    const int za = zA[slot[i]];
    cnt += (za % NL) == 2 * NV;
  }
  const double cval = cnt > 0 ? 1.0 / sqrt((double)cnt) : 0.0;
  for (int q = tid; q < m * m; q += blockDim.x) {
    const int i = q / m, j = q % m;
    double v = 0.0;
    if (i < n && j < n) {
      const int ti = slot[i], tj = slot[j];
      const int pa[2] = {zA[ti], zB[ti]}, pb[2] = {zA[tj], zB[tj]};
      for (int x1 = 0; x1 < 2; ++x1)
        for (int x2 = 0; x2 < 2; ++x2)
          if (pa[x1] >= 0 && pb[x2] >= 0) v += patch_coupling<K>(E, pa[x1], pb[x2], vx, vy, N, bcm, h, kap);
    } else if (i < n || j < n) {
      const int ii = i < n ? i : j;
      v = (zA[slot[ii]] % NL) == 2 * NV ? cval : 0.0;
    }
    a[i * m + j] = v;
  }
  __syncthreads();
  // 3. Gauss-Jordan in place, partial pivoting
  for (int k = 0; k < m; ++k) {
    if (tid < 64) {
      double best = -1.0;
      int bi = k;
      for (int i = k + tid; i < m; i += 64) {
        const double v = fabs(a[i * m + k]);
        if (v > best) {
          best = v;
          bi = i;
        }
      }
      for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_down(best, o, 64);
        const int oi = __shfl_down(bi, o, 64);
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
        }
      }
      if (tid == 0) {
        s_piv = bi;
        if (!(best > 0.0)) s_bad = 1;
      }
    }
    __syncthreads();
    if (s_bad) break;
    const int pr = s_piv;
    if (tid == 0) pv[k] = pr;
    if (pr != k)
      for (int j = tid; j < m; j += blockDim.x) {
        const double t0 = a[k * m + j];
        a[k * m + j] = a[pr * m + j];
        a[pr * m + j] = t0;
      }
    __syncthreads();
    const double dinv = 1.0 / a[k * m + k];
    for (int i = tid; i < m; i += blockDim.x) {
      fcol[i] = a[i * m + k];
      prow[i] = (i == k ? 1.0 : a[k * m + i]) * dinv;
    }
    __syncthreads();
    // wave wv updates rows wv, wv + NWV, ...; lane l columns l, l + 64 (no index division)
    {
      const int nwv = blockDim.x >> 6, wv = tid >> 6, l = tid & 63;
      const double p0 = l < m ? prow[l] : 0.0, p1 = l + 64 < m ? prow[l + 64] : 0.0;
      for (int i = wv; i < m; i += nwv) {
        const double f = fcol[i];
        double* ar = a + i * m;
        if (i == k) {
          if (l < m) ar[l] = p0;
          if (l + 64 < m) ar[l + 64] = p1;
        } else {
          if (l < m) ar[l] = (l == k ? 0.0 : ar[l]) - f * p0;
          if (l + 64 < m) ar[l + 64] = (l + 64 == k ? 0.0 : ar[l + 64]) - f * p1;
        }
      }
    }
    __syncthreads();
  }
  if (s_bad) {
    if (tid == 0) atomicOr(status, 1);
    return;
  }
  // undo the row interchanges on the columns, last first
  for (int k = m - 1; k >= 0; --k) {
    const int pr = pv[k];
    if (pr != k)
      for (int i = tid; i < m; i += blockDim.x) {
        const double t0 = a[i * m + k];
        a[i * m + k] = a[i * m + pr];
        a[i * m + pr] = t0;
      }
    __syncthreads();
  }
  // 4. the leading n x n block in the layout of the level
  S* dst = isx ? invx + (size_t)ext * (ROT ? NSE * (NSE / 2 + 1) : NSE * NSE)
               : inv + (size_t)p * (ROT ? NSR * (NSR / 2 + 1) : NSR * NSR);
  if (ROT) {
    const int ne = ns * (ns / 2 + 1);
    for (int q = tid; q < ne; q += blockDim.x) {
      const int dg = q / ns, t = q % ns, u = (t + dg) % ns;
      const int ci = cidx[t], cj = cidx[u];
      const double v = (ci >= 0 && cj >= 0) ? 0.5 * (a[ci * m + cj] + a[cj * m + ci]) : 0.0;
      dst[q] = store_as<S>(v);
    }
  } else {
    for (int q = tid; q < ns * ns; q += blockDim.x) {
      const int u = q / ns, t = q % ns;  // column-major: entry (t, u) at u ns + t
      const int ci = cidx[t], cj = cidx[u];
      dst[q] = store_as<S>((ci >= 0 && cj >= 0) ? a[ci * m + cj] : 0.0);
    }
  }
  (void)NP;
}

// ---------------------------------------------------------------------------
// Transfers
// ---------------------------------------------------------------------------
// Sums over the fine dofs strictly inside coarse cell (cxc, cyc) of P[f][coarse dof]
// * r_f, for one velocity component; only rows with psi index `arow` if arow >= 0.
template <typename T, int K, typename RA>
__device__ __forceinline__ void inside_comp(const Xfer<T, K>& X, int Nf, int cxc, int cyc, int comp, RA rf, T* out,
                                            int arow) {
  using D = Dims<K>;
  constexpr int NA = D::NA, NB = D::NB, NV = D::NV;
#pragma unroll
  for (int i = 0; i < NV; ++i) out[i] = T(0);
#pragma unroll
  for (int ch = 0; ch < 4; ++ch) {
    const int sx = ch & 1, sy = ch >> 1;
    const int sn = comp == 0 ? sx : sy;  // child position along the component direction
    const int st = comp == 0 ? sy : sx;  // across
    const int fx = 2 * cxc + sx, fy = 2 * cyc + sy;
#pragma unroll
    for (int ap = 0; ap < NA; ++ap) {
      if ((sn == 0 && ap == 0) || (sn == 1 && ap == 1) || (sn == 1 && ap == 0)) continue;
#pragma unroll
      for (int bp = 0; bp < NB; ++bp) {
        const T r = rf[Idx<K>::g(Nf, fx, fy, comp * NV + ap * NB + bp)];
#pragma unroll
        for (int a = 0; a < NA; ++a) {
          if (arow >= 0 && a != arow) continue;
          const T pa = X.Ppsi[sn][ap * NA + a] * r;
#pragma unroll
          for (int bb = 0; bb < NB; ++bb) out[a * NB + bb] += pa * X.PL[st][bp * NB + bb];
        }
      }
    }
  }
}

// IL: interleaved records of ldf (= ldc) values, thread -> (coarse cell, column) with
// the column fastest; otherwise one thread per coarse cell, blockIdx.y = column
template <typename T, int K, bool IL = false>
__global__ __launch_bounds__(256) void k_restrict(const Xfer<T, K>* __restrict__ Xp, int Nc, int bcm,
                                                  const T* __restrict__ rf_, T* __restrict__ bc_, int64_t ldf,
                                                  int64_t ldc) {
  using D = Dims<K>;
  using I = Idx<K>;
  constexpr int NA = D::NA, NB = D::NB, NV = D::NV, NP = D::NP;
  int c;
  int64_t cof, coc;
  if constexpr (IL) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    c = (int)(t >> __builtin_ctzll(ldf));
    cof = coc = t & (ldf - 1);
  } else {
    c = blockIdx.x * blockDim.x + threadIdx.x;
    cof = blockIdx.y * ldf;
    coc = blockIdx.y * ldc;
  }
  if (c >= Nc * Nc) return;
  const auto rf = col_view<IL>(rf_ + cof, ldf);
  const auto bc = col_view<IL>(bc_ + coc, ldc);
  const Xfer<T, K>& X = *Xp;
  const int cx = c % Nc, cy = c / Nc, Nf = 2 * Nc;
  T in_x[NV], in_y[NV], tmp[NV];
  inside_comp<T, K>(X, Nf, cx, cy, 0, rf, in_x, -1);
  inside_comp<T, K>(X, Nf, cx, cy, 1, rf, in_y, -1);
  // pressure: every child pressure dof, tensor re-expansion in both directions
  T in_p[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) in_p[q] = T(0);
#pragma unroll
  for (int ch = 0; ch < 4; ++ch) {
    const int sx = ch & 1, sy = ch >> 1;
    const int base = I::pres(Nf, (2 * cy + sy) * Nf + 2 * cx + sx, 0);
#pragma unroll
    for (int qb = 0; qb < NB; ++qb)
#pragma unroll
      for (int qa = 0; qa < NB; ++qa) {
        const T r = rf[base + qb * NB + qa];
#pragma unroll
        for (int pb = 0; pb < NB; ++pb)
#pragma unroll
          for (int pa = 0; pa < NB; ++pa) in_p[pb * NB + pa] += X.PL[sx][qa * NB + pa] * X.PL[sy][qb * NB + pb] * r;
      }
  }
#pragma unroll
  for (int q = 0; q < NP; ++q) bc[I::pres(Nc, c, q)] = in_p[q];
#pragma unroll
  for (int a = 2; a < NA; ++a)
#pragma unroll
    for (int bb = 0; bb < NB; ++bb) {
      bc[I::inter(Nc, c, 0, a, bb)] = in_x[a * NB + bb];
      bc[I::inter(Nc, c, 1, a, bb)] = in_y[a * NB + bb];
    }
  // fine face dofs lying on a coarse face only see that face's dofs (1-D Legendre)
  auto face_x = [&](int i, int bb) {
    T s = T(0);
#pragma unroll
    for (int sd = 0; sd < 2; ++sd)
#pragma unroll
      for (int bp = 0; bp < NB; ++bp) s += X.PL[sd][bp * NB + bb] * rf[I::xface(Nf, 2 * i, 2 * cy + sd, bp)];
    return s;
  };
  auto face_y = [&](int j, int bb) {
    T s = T(0);
#pragma unroll
    for (int sd = 0; sd < 2; ++sd)
#pragma unroll
      for (int bp = 0; bp < NB; ++bp) s += X.PL[sd][bp * NB + bb] * rf[I::yface(Nf, 2 * j, 2 * cx + sd, bp)];
    return s;
  };
  // left face
  if (cx > 0) inside_comp<T, K>(X, Nf, cx - 1, cy, 0, rf, tmp, 1);
#pragma unroll
  for (int bb = 0; bb < NB; ++bb) {
    T v = (cx == 0 && (bcm & 1)) ? T(0) : in_x[bb] + (cx > 0 ? tmp[NB + bb] : T(0)) + face_x(cx, bb);
    bc[I::xface(Nc, cx, cy, bb)] = v;
  }
  if (cx == Nc - 1) {
#pragma unroll
    for (int bb = 0; bb < NB; ++bb)
      bc[I::xface(Nc, Nc, cy, bb)] = (bcm & 2) ? T(0) : in_x[NB + bb] + face_x(Nc, bb);
  }
  // bottom face
  if (cy > 0) inside_comp<T, K>(X, Nf, cx, cy - 1, 1, rf, tmp, 1);
#pragma unroll
  for (int bb = 0; bb < NB; ++bb) {
    T v = (cy == 0 && (bcm & 4)) ? T(0) : in_y[bb] + (cy > 0 ? tmp[NB + bb] : T(0)) + face_y(cy, bb);
    bc[I::yface(Nc, cy, cx, bb)] = v;
  }
  if (cy == Nc - 1) {
#pragma unroll
    for (int bb = 0; bb < NB; ++bb)
      bc[I::yface(Nc, Nc, cx, bb)] = (bcm & 8) ? T(0) : in_y[NB + bb] + face_y(Nc, bb);
  }
}

// IL: as k_restrict
template <typename T, int K, bool IL = false>
__global__ __launch_bounds__(256) void k_prolong(const Xfer<T, K>* __restrict__ Xp, int Nc, int bcm,
                                                 const T* __restrict__ xc_, T* __restrict__ xf_, int64_t ldc,
                                                 int64_t ldf) {
  using D = Dims<K>;
  using I = Idx<K>;
  constexpr int NA = D::NA, NB = D::NB, NV = D::NV, NP = D::NP;
  int c;
  int64_t coc, cof;
  if constexpr (IL) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    c = (int)(t >> __builtin_ctzll(ldf));
    coc = cof = t & (ldf - 1);
  } else {
    c = blockIdx.x * blockDim.x + threadIdx.x;
    coc = blockIdx.y * ldc;
    cof = blockIdx.y * ldf;
  }
  if (c >= Nc * Nc) return;
  const auto xc = col_view<IL>(xc_ + coc, ldc);
  const auto xf = col_view<IL>(xf_ + cof, ldf);
  const Xfer<T, K>& X = *Xp;
  const int cx = c % Nc, cy = c / Nc, Nf = 2 * Nc;
  T zx[NV], zy[NV], zp[NP];
  load_comp<K>(xc, Nc, bcm, cx, cy, 0, zx);
  load_comp<K>(xc, Nc, bcm, cx, cy, 1, zy);
  load_pres<K>(xc, Nc, cx, cy, zp);
#pragma unroll
  for (int ch = 0; ch < 4; ++ch) {
    const int sx = ch & 1, sy = ch >> 1;
    const int fx = 2 * cx + sx, fy = 2 * cy + sy;
#pragma unroll
    for (int comp = 0; comp < 2; ++comp) {
      const int sn = comp == 0 ? sx : sy, st = comp == 0 ? sy : sx;
      const bool last = comp == 0 ? (cx == Nc - 1) : (cy == Nc - 1);
      const T* z = comp == 0 ? zx : zy;
#pragma unroll
      for (int ap = 0; ap < NA; ++ap) {
        if (sn == 1 && ap == 0) continue;            // middle face: written by child sn = 0
        if (sn == 1 && ap == 1 && !last) continue;   // outer face: written by the next coarse cell
#pragma unroll
        for (int bp = 0; bp < NB; ++bp) {
          const int d = comp * NV + ap * NB + bp;
          if (I::cons(Nf, bcm, fx, fy, d)) continue;
          T v = T(0);
#pragma unroll
          for (int a = 0; a < NA; ++a) {
            T s = T(0);
#pragma unroll
            for (int bb = 0; bb < NB; ++bb) s += X.PL[st][bp * NB + bb] * z[a * NB + bb];
            v += X.Ppsi[sn][ap * NA + a] * s;
          }
          xf[I::g(Nf, fx, fy, d)] += v;
        }
      }
    }
    const int base = I::pres(Nf, fy * Nf + fx, 0);
#pragma unroll
    for (int qb = 0; qb < NB; ++qb)
#pragma unroll
      for (int qa = 0; qa < NB; ++qa) {
        T v = T(0);
#pragma unroll
        for (int pb = 0; pb < NB; ++pb)
#pragma unroll
          for (int pa = 0; pa < NB; ++pa) v += X.PL[sx][qa * NB + pa] * X.PL[sy][qb * NB + pb] * zp[pb * NB + pa];
        xf[base + qb * NB + qa] += v;
      }
  }
}

// ---------------------------------------------------------------------------
// Coarse solve, casts, constrained copy
// ---------------------------------------------------------------------------
// one block per column; entry i of column c at c * cs + i * es (column-major: cs = n,
// es = 1; interleaved records of width w: cs = 1, es = w)
template <typename T>
__global__ __launch_bounds__(256) void k_coarse(int n, const double* __restrict__ inv, const T* __restrict__ b,
                                                T* __restrict__ x, int64_t cs, int64_t es) {
  extern __shared__ double sb[];
  b += (int64_t)blockIdx.x * cs;
  x += (int64_t)blockIdx.x * cs;
  for (int i = threadIdx.x; i < n; i += blockDim.x) sb[i] = (double)b[i * es];
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += inv[(size_t)j * n + i] * sb[j];
    x[i * es] = (T)s;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_fill(T* __restrict__ x, T v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = v;
}

// columns col0 .. col0 + nrhs - 1 of the identity, stored as nrhs vectors of length n
template <typename T>
__global__ __launch_bounds__(256) void k_identity(T* __restrict__ x, int64_t n, int64_t col0, int nrhs) {
  const int64_t tot = n * nrhs;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / n, e = i % n;
    x[i] = (e == col0 + r) ? T(1) : T(0);
  }
}

// Y = B X for a symmetric n x n matrix stored densely and NR right-hand sides
// (columns of n entries): one wavefront per row, the row streamed once
// (non-temporal loads) for all columns, four independent partial sums per lane and
// column (the summation order of a column does not depend on NR).
template <typename T, int NR>
__global__ __launch_bounds__(256) void k_dense_rows(const T* __restrict__ B, int64_t n, const T* __restrict__ x,
                                                    T* __restrict__ y, int64_t cs, int64_t es) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  const T* r = B + row * n;
  T a0[NR], a1[NR], a2[NR], a3[NR];
#pragma unroll
  for (int c = 0; c < NR; ++c) a0[c] = a1[c] = a2[c] = a3[c] = T(0);
  int64_t j = lane;
  for (; j + 192 < n; j += 256) {
    const T b0 = __builtin_nontemporal_load(r + j), b1 = __builtin_nontemporal_load(r + j + 64);
    const T b2 = __builtin_nontemporal_load(r + j + 128), b3 = __builtin_nontemporal_load(r + j + 192);
#pragma unroll
    for (int c = 0; c < NR; ++c) {
      const T* xc = x + c * cs;
      a0[c] += b0 * xc[j * es];
      a1[c] += b1 * xc[(j + 64) * es];
      a2[c] += b2 * xc[(j + 128) * es];
      a3[c] += b3 * xc[(j + 192) * es];
    }
  }
  for (; j < n; j += 64) {
    const T b0 = __builtin_nontemporal_load(r + j);
#pragma unroll
    for (int c = 0; c < NR; ++c) a0[c] += b0 * x[c * cs + j * es];
  }
#pragma unroll
  for (int c = 0; c < NR; ++c) {
    T s = (a0[c] + a1[c]) + (a2[c] + a3[c]);
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    if (lane == 0) y[c * cs + row * es] = s;
  }
}

template <typename TO, typename TI>
__global__ __launch_bounds__(256) void k_cast(const TI* __restrict__ src, TO* __restrict__ dst, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (TO)src[i];
}

// Interleaved records of w values (w a power of two, at most 16) <-> column-major
// blocks ld apart: to_il writes dst[g w + c] = src[c ld + g] for c < nrhs and 0 for
// nrhs <= c < w; from_il writes dst[c ld + g] = src[g w + c] for c < nrhs.  A block
// moves 64 consecutive entries g of every column through LDS, so that the blocks are
// read / written along g and the records as whole contiguous runs.
template <typename TO, typename TI>
__global__ __launch_bounds__(256) void k_to_il(const TI* __restrict__ src, TO* __restrict__ dst, int64_t n,
                                               int64_t ld, int nrhs, int w) {
  __shared__ TO tile[16][65];
  const int64_t g0 = (int64_t)blockIdx.x * 64;
  const int gl = threadIdx.x & 63;
  for (int c = threadIdx.x >> 6; c < w; c += 4) {
    const int64_t g = g0 + gl;
    tile[c][gl] = (c < nrhs && g < n) ? (TO)src[c * ld + g] : TO(0);
  }
  __syncthreads();
  const int lw = __builtin_ctz(w);
  for (int i = threadIdx.x; i < 64 * w; i += 256) {
    const int gi = i >> lw, c = i & (w - 1);
    const int64_t g = g0 + gi;
    if (g < n) dst[g * w + c] = tile[c][gi];
  }
}

template <typename TO, typename TI>
__global__ __launch_bounds__(256) void k_from_il(const TI* __restrict__ src, TO* __restrict__ dst, int64_t n,
                                                 int64_t ld, int nrhs, int w) {
  __shared__ TI tile[16][65];
  const int64_t g0 = (int64_t)blockIdx.x * 64;
  const int lw = __builtin_ctz(w);
  for (int i = threadIdx.x; i < 64 * w; i += 256) {
    const int gi = i >> lw, c = i & (w - 1);
    const int64_t g = g0 + gi;
    tile[c][gi] = g < n ? src[g * w + c] : TI(0);
  }
  __syncthreads();
  const int gl = threadIdx.x & 63;
  for (int c = threadIdx.x >> 6; c < nrhs; c += 4) {
    const int64_t g = g0 + gl;
    if (g < n) dst[c * ld + g] = (TO)tile[c][gl];
  }
}

template <typename TO, int K>
__global__ __launch_bounds__(256) void k_copy_cons(int N, int bcm, const double* __restrict__ src, TO* __restrict__ dst,
                                                   int64_t ld) {
  using D = Dims<K>;
  src += blockIdx.y * ld;
  dst += blockIdx.y * ld;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 4 * N * D::NB) return;
  const int side = t / (N * D::NB), r = t % (N * D::NB), f = r / D::NB, bb = r % D::NB;
  if (!((bcm >> side) & 1)) return;
  int gi;
  if (side < 2) gi = Idx<K>::xface(N, side == 0 ? 0 : N, f, bb);
  else gi = Idx<K>::yface(N, side == 2 ? 0 : N, f, bb);
  dst[gi] = (TO)src[gi];
}

// ---------------------------------------------------------------------------
// FP64 Krylov helpers
// ---------------------------------------------------------------------------
constexpr int kDotBlocks = 512;
constexpr int kDotChunk = 8;

__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += sh[i];
  return s;
}

// Krylov vectors of several right-hand sides: column r of vector k at V + k ldv + r n
// (blockIdx.y = r); every right-hand side keeps its own results.
__global__ __launch_bounds__(256) void k_dots(const double* __restrict__ V, int nvec, int64_t ldv,
                                              const double* __restrict__ w, int64_t n, double* __restrict__ partial) {
  __shared__ double sh[8];
  V += blockIdx.y * n;
  w += blockIdx.y * n;
  partial += (int64_t)blockIdx.y * nvec * gridDim.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int c0 = 0; c0 < nvec; c0 += kDotChunk) {
    double acc[kDotChunk];
#pragma unroll
    for (int v = 0; v < kDotChunk; ++v) acc[v] = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) {
      const double wi = w[i];
#pragma unroll
      for (int v = 0; v < kDotChunk; ++v)
        if (c0 + v < nvec) acc[v] += V[(int64_t)(c0 + v) * ldv + i] * wi;
    }
#pragma unroll
    for (int v = 0; v < kDotChunk; ++v) {
      if (c0 + v >= nvec) break;
      const double s = block_sum(acc[v], sh);
      if (threadIdx.x == 0) partial[(int64_t)(c0 + v) * gridDim.x + blockIdx.x] = s;
    }
  }
}

__global__ __launch_bounds__(256) void k_dots_final(const double* __restrict__ partial, int nblk,
                                                    double* __restrict__ out, int64_t ostride) {
  __shared__ double sh[8];
  partial += (int64_t)blockIdx.y * gridDim.x * nblk;
  out += blockIdx.y * ostride;
  double s = 0.0;
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) s += partial[(int64_t)blockIdx.x * nblk + i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

template <typename VT>
__global__ __launch_bounds__(256) void k_axpys(double* __restrict__ w, const VT* __restrict__ V, int nvec,
                                               int64_t ldv, const double* __restrict__ coef, int64_t cstride,
                                               double sign, int64_t n) {
  w += blockIdx.y * n;
  V += blockIdx.y * n;
  coef += blockIdx.y * cstride;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int v = 0; v < nvec; ++v) s += coef[v] * (double)V[(int64_t)v * ldv + i];
    w[i] += sign * s;
  }
}

// dst = src / denom (or / sqrt(denom)) per right-hand side; 0 where live[r] == 0
__global__ __launch_bounds__(256) void k_scale(double* __restrict__ dst, const double* __restrict__ src,
                                               const double* __restrict__ denom, int64_t dstride,
                                               const int32_t* __restrict__ live, int take_sqrt, int64_t n) {
  const int r = blockIdx.y;
  dst += r * n;
  src += r * n;
  const double d = denom[r * dstride];
  const double f = live[r] ? 1.0 / (take_sqrt ? sqrt(d) : d) : 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i] * f;
}

__global__ __launch_bounds__(256) void k_sub(double* __restrict__ r, const double* __restrict__ b,
                                             const double* __restrict__ ax, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    r[i] = b[i] - ax[i];
}

inline unsigned grid_for(int64_t n, int bs = 256, int64_t cap = 8192) {
  int64_t g = (n + bs - 1) / bs;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return (unsigned)g;
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <typename T, int K>
static void op_t(const void* elem, const LevelArgs& L, const void* x, const void* b, void* y, bool res, int nrhs,
                 int64_t ld, int il, hipStream_t s) {
  const int n = L.N * L.N;
  if constexpr (K >= 1 && std::is_same<T, float>::value)
    if (il > 0) {
      // interleaved records of il values: one thread per (cell, column)
      const dim3 gi((unsigned)(((int64_t)n * il + 255) / 256)), bi(256);
      if (res)
        hipLaunchKernelGGL((k_op<T, K, true, T, true>), gi, bi, 0, s, (const Elem<T, K>*)elem, L.N, L.bcm, (T)L.h,
                           (const T*)L.kap, (const T*)x, (const T*)b, (T*)y, (int64_t)il);
      else
        hipLaunchKernelGGL((k_op<T, K, false, T, true>), gi, bi, 0, s, (const Elem<T, K>*)elem, L.N, L.bcm, (T)L.h,
                           (const T*)L.kap, (const T*)x, (const T*)b, (T*)y, (int64_t)il);
      return;
    }
  dim3 g((n + 255) / 256, nrhs), bl(256);
  if (res)
    hipLaunchKernelGGL((k_op<T, K, true>), g, bl, 0, s, (const Elem<T, K>*)elem, L.N, L.bcm, (T)L.h,
                       (const T*)L.kap, (const T*)x, (const T*)b, (T*)y, ld);
  else
    hipLaunchKernelGGL((k_op<T, K, false>), g, bl, 0, s, (const Elem<T, K>*)elem, L.N, L.bcm, (T)L.h,
                       (const T*)L.kap, (const T*)x, (const T*)b, (T*)y, ld);
}

template <int K>
static void op64_f32x_t(const void* elem, const LevelArgs& L, const float* x, double* y, int nrhs, int64_t ld,
                        hipStream_t s) {
  const int n = L.N * L.N;
  hipLaunchKernelGGL((k_op<double, K, false, float>), dim3((n + 255) / 256, nrhs), dim3(256), 0, s,
                     (const Elem<double, K>*)elem, L.N, L.bcm, L.h, (const double*)L.kap, x, (const double*)nullptr,
                     y, ld);
}

void launch_op64_f32x(int K, const void* elem64, const LevelArgs& L, const float* x, double* y, int nrhs, int64_t ld,
                      hipStream_t s) {
  if (K == 0) op64_f32x_t<0>(elem64, L, x, y, nrhs, ld, s);
  else if (K == 1) op64_f32x_t<1>(elem64, L, x, y, nrhs, ld, s);
  else op64_f32x_t<2>(elem64, L, x, y, nrhs, ld, s);
}

void launch_op(int K, int prec, const void* elem, const LevelArgs& L, const void* x, const void* b, void* y,
               bool residual, int nrhs, int64_t ld, hipStream_t s, int il) {
  if (K == 0) {
    if (prec == 0) op_t<double, 0>(elem, L, x, b, y, residual, nrhs, ld, il, s);
    else op_t<float, 0>(elem, L, x, b, y, residual, nrhs, ld, il, s);
  } else if (K == 1) {
    if (prec == 0) op_t<double, 1>(elem, L, x, b, y, residual, nrhs, ld, il, s);
    else op_t<float, 1>(elem, L, x, b, y, residual, nrhs, ld, il, s);
  } else {
    if (prec == 0) op_t<double, 2>(elem, L, x, b, y, residual, nrhs, ld, il, s);
    else op_t<float, 2>(elem, L, x, b, y, residual, nrhs, ld, il, s);
  }
}

// Columns one block of k_colour serves: all of them on the bandwidth-bound levels
// (N >= 192: the inverse is read once per patch for all columns) and with rotated
// storage (up to 16 columns); elsewhere enough blocks to fill the device come first.
int colour_columns_per_block(int N, bool packed, int npatch, int nrhs, int cpb) {
  if (nrhs <= 1) return 1;
  // the tile parameter applies to a handle's own columns (at most 16), not to the setup
  // batches of unit vectors
  if (cpb > 0 && nrhs <= 16) return std::min(nrhs, cpb);
  if (N >= 192) return std::min(nrhs, 16);
  // rotated storage on a small level with many columns (the setup batch of unit vectors
  // that builds the dense coarse operator): one column per block, the columns in parallel
  if (packed && nrhs > 16) return 1;
  if (packed) return std::min(nrhs, 16);
  const int nblk = (npatch + 3) / 4;
  return std::max(1, std::min(16, (int)((int64_t)nblk * nrhs / 4096)));
}

template <typename T, typename S, int K>
static void colour_t(const void* elem, const LevelArgs& L, void* x, const void* b, const void* inv, const void* invx,
              const int32_t* extidx, int colour, int npatch, bool finest, bool packed, int nrhs, int64_t ld,
              double omega, const int32_t* plist, int il, hipStream_t s) {
  if (npatch <= 0) return;
  const int nblk = (npatch + 3) / 4;
  if constexpr (K >= 1 && std::is_same<T, float>::value && std::is_same<S, bf16>::value) {
    if (il > 0) {
      // the listed patches of a level whose columns are interleaved records of il values
      // (rotated inverses, one column per block)
      const int gx = nblk >= 64 ? (nblk + 7) / 8 * 8 : (nblk % 8 == 0 ? nblk + 1 : nblk);
      hipLaunchKernelGGL((k_colour<T, S, K, 0, true, false, false, true>), dim3(gx, nrhs), dim3(256), 0, s,
                         (const Elem<T, K>*)elem, L.N, L.bcm, (T)L.h, (const T*)L.kap, (T*)x, (const T*)b,
                         (const S*)inv, (const S*)invx, extidx, colour, L.colouring, npatch, (int64_t)il, nrhs, 1,
                         (T)omega, plist);
      return;
    }
  }
  // a short list of patches (the boundary patches beside the several-column kernel):
  // one column per block, so that the columns run in parallel
  const int ncol = plist ? 1 : colour_columns_per_block(L.N, packed, npatch, nrhs, L.cpb);
  // large grids: a multiple of the 8 XCDs (the kernel then maps blocks to strips);
  // small ones (coarse levels, setup batches): one block per 4 patches, plain order
  // (a count that happens to be a multiple of 8 gets one idle block more)
  const int gxb = nblk >= 64 ? (nblk + 7) / 8 * 8 : (nblk % 8 == 0 ? nblk + 1 : nblk);
  dim3 g(gxb, (nrhs + ncol - 1) / ncol), bl(256);
#define BMG_KC(TAG, PKD, MC, ADD)                                                                               \
  hipLaunchKernelGGL((k_colour<T, S, K, TAG, PKD, MC, ADD>), g, bl, 0, s, (const Elem<T, K>*)elem, L.N, L.bcm,  \
                     (T)L.h, (const T*)L.kap, (T*)x, (const T*)b, (const S*)inv, (const S*)invx, extidx, colour,  \
                     L.colouring, npatch, ld, nrhs, ncol, (T)omega, plist)
  if (omega > 0.0) {
    // additive step: b is the residual of x
    if (packed) {
      if (ncol > 1) BMG_KC(0, true, true, true);
      else BMG_KC(0, true, false, true);
    } else {
      if (ncol > 1) BMG_KC(0, false, true, true);
      else BMG_KC(0, false, false, true);
    }
  } else if (ncol > 1) {
    if (packed) BMG_KC(0, true, true, false);
    else BMG_KC(0, false, true, false);
  } else if (finest) {
    if (packed) BMG_KC(1, true, false, false);
    else BMG_KC(1, false, false, false);
  } else {
    if (packed) BMG_KC(0, true, false, false);
    else BMG_KC(0, false, false, false);
  }
#undef BMG_KC
}

template <int K, typename S>
static void pinv_t(const void* elem64, const LevelArgs& L, int colour, int npatch, bool rotated, void* inv, void* invx,
                   const int32_t* extidx, int32_t* status, hipStream_t s) {
  if (npatch <= 0) return;
  if (rotated)
    hipLaunchKernelGGL((k_patch_pinv<K, S, true>), dim3(npatch), dim3(512), 0, s, (const Elem<double, K>*)elem64,
                       L.N, L.bcm, L.h, (const double*)L.kap, colour, L.colouring, (S*)inv, (S*)invx, extidx, status);
  else
    hipLaunchKernelGGL((k_patch_pinv<K, S, false>), dim3(npatch), dim3(512), 0, s, (const Elem<double, K>*)elem64,
                       L.N, L.bcm, L.h, (const double*)L.kap, colour, L.colouring, (S*)inv, (S*)invx, extidx, status);
}

void launch_patch_pinv(int K, int sprec, const void* elem64, const LevelArgs& L, int colour, int npatch, bool rotated,
                       void* inv, void* invx, const int32_t* extidx, int32_t* status, hipStream_t s) {
#define BMG_PI(KK)                                                                                         \
  if (sprec == 0) pinv_t<KK, double>(elem64, L, colour, npatch, rotated, inv, invx, extidx, status, s);    \
  else if (sprec == 1) pinv_t<KK, float>(elem64, L, colour, npatch, rotated, inv, invx, extidx, status, s); \
  else pinv_t<KK, bf16>(elem64, L, colour, npatch, rotated, inv, invx, extidx, status, s);
  if (K == 0) {
    BMG_PI(0)
  } else if (K == 1) {
    BMG_PI(1)
  } else {
    BMG_PI(2)
  }
#undef BMG_PI
}

template <int K>
static void colour_mr_t(const void* elem_int, const LevelArgs& L, void* x, const void* b, const void* inv,
                        const int32_t* tab, int colour, int npatch, int rp, hipStream_t s) {
  if (npatch <= 0) return;
  hipLaunchKernelGGL((k_colour_mr<K>), dim3((npatch + 7) & ~7), dim3(256), 0, s, (const ElemInt<float, K>*)elem_int, L.N,
                     (float)L.h, (const float*)L.kap, (float*)x, (const float*)b, (const bf16*)inv,
                     (const int4*)tab, colour, L.colouring, npatch, rp);
}

void launch_colour_mr(int K, const void* elem_int, const LevelArgs& L, void* x, const void* b, const void* inv,
                      const int32_t* tab, int colour, int npatch, int rp, hipStream_t s) {
  if (K == 1) colour_mr_t<1>(elem_int, L, x, b, inv, tab, colour, npatch, rp, s);
  else if (K == 2) colour_mr_t<2>(elem_int, L, x, b, inv, tab, colour, npatch, rp, s);
}

template <int K>
static void colour_fused_t(const void* elem_int, const void* elem, const LevelArgs& L, void* x, const void* b,
                           const void* inv, const void* invx, const int32_t* extidx, const int32_t* tab, int colour,
                           int npatch_mr, int nlist, const int32_t* plist, int nrhs, int rp, hipStream_t s) {
  const int mr_blocks = (npatch_mr + 7) & ~7;
  const int nblk = (nlist + 3) / 4;
  const int nbx = nlist <= 0 ? 0 : nblk >= 64 ? (nblk + 7) / 8 * 8 : (nblk % 8 == 0 ? nblk + 1 : nblk);
  const int64_t grid = (int64_t)mr_blocks + (int64_t)nbx * nrhs;
  if (grid <= 0) return;
  hipLaunchKernelGGL((k_colour_fused<K>), dim3((unsigned)grid), dim3(256), 0, s, (const ElemInt<float, K>*)elem_int,
                     (const int4*)tab, npatch_mr, mr_blocks, (const Elem<float, K>*)elem, L.N, L.bcm, (float)L.h,
                     (const float*)L.kap, (float*)x, (const float*)b, (const bf16*)inv, (const bf16*)invx, extidx,
                     colour, L.colouring, nlist, (int64_t)rp, nrhs, plist, nbx > 0 ? nbx : 1);
}

void launch_colour_fused(int K, const void* elem_int, const void* elem, const LevelArgs& L, void* x, const void* b,
                         const void* inv, const void* invx, const int32_t* extidx, const int32_t* tab, int colour,
                         int npatch_mr, int nlist, const int32_t* plist, int nrhs, int rp, hipStream_t s) {
  if (K == 1)
    colour_fused_t<1>(elem_int, elem, L, x, b, inv, invx, extidx, tab, colour, npatch_mr, nlist, plist, nrhs, rp, s);
  else if (K == 2)
    colour_fused_t<2>(elem_int, elem, L, x, b, inv, invx, extidx, tab, colour, npatch_mr, nlist, plist, nrhs, rp, s);
}

int mr_table_entries(int K) {
  return K == 1 ? MrDims<1>::NE + Dims<1>::NSR : MrDims<2>::NE + Dims<2>::NSR;
}

void mr_steps(int K, int N, int* ax, int* ay) {
  if (K == 1) mr_stream_steps<1>(N, ax, ay);
  else mr_stream_steps<2>(N, ax, ay);
}

void mr_layout(int K, int* cw, int* xs, int* cs) {
  if (K == 1) {
    *cw = MrDims<1>::CW;
    *xs = MrDims<1>::XS;
    *cs = MrDims<1>::CS;
  } else {
    *cw = MrDims<2>::CW;
    *xs = MrDims<2>::XS;
    *cs = MrDims<2>::CS;
  }
}

void launch_colour(int K, int prec, int sprec, const void* elem, const LevelArgs& L, void* x, const void* b,
                   const void* inv, const void* invx, const int32_t* extidx, int colour, int npatch, bool finest,
                   bool packed, int nrhs, int64_t ld, double omega, hipStream_t s, const int32_t* plist, int il) {
#define BMG_COL(T, S, KK) \
  colour_t<T, S, KK>(elem, L, x, b, inv, invx, extidx, colour, npatch, finest, packed, nrhs, ld, omega, plist, il, s)
  if (K == 0) {
    if (prec == 0) BMG_COL(double, double, 0);
    else if (sprec == 0) BMG_COL(float, double, 0);
    else if (sprec == 1) BMG_COL(float, float, 0);
    else BMG_COL(float, bf16, 0);
  } else if (K == 1) {
    if (prec == 0) BMG_COL(double, double, 1);
    else if (sprec == 0) BMG_COL(float, double, 1);
    else if (sprec == 1) BMG_COL(float, float, 1);
    else BMG_COL(float, bf16, 1);
  } else {
    if (prec == 0) BMG_COL(double, double, 2);
    else if (sprec == 0) BMG_COL(float, double, 2);
    else if (sprec == 1) BMG_COL(float, float, 2);
    else BMG_COL(float, bf16, 2);
  }
#undef BMG_COL
}

template <typename T, int K>
static void restrict_t(const void* xfer, int Nc, int bcm, const void* rf, void* bc, int nrhs, int64_t ldf,
                       int64_t ldc, int il, hipStream_t s) {
  const int64_t n = (int64_t)Nc * Nc;
  if constexpr (K >= 1 && std::is_same<T, float>::value)
    if (il > 0) {
      hipLaunchKernelGGL((k_restrict<T, K, true>), dim3((unsigned)((n * il + 255) / 256)), dim3(256), 0, s,
                         (const Xfer<T, K>*)xfer, Nc, bcm, (const T*)rf, (T*)bc, (int64_t)il, (int64_t)il);
      return;
    }
  hipLaunchKernelGGL((k_restrict<T, K>), dim3((unsigned)((n + 255) / 256), nrhs), dim3(256), 0, s,
                     (const Xfer<T, K>*)xfer, Nc, bcm, (const T*)rf, (T*)bc, ldf, ldc);
}
void launch_restrict(int K, int prec, const void* xfer, int Nc, int bcm, const void* rf, void* bc, int nrhs,
                     int64_t ldf, int64_t ldc, hipStream_t s, int il) {
  if (K == 0) {
    if (prec == 0) restrict_t<double, 0>(xfer, Nc, bcm, rf, bc, nrhs, ldf, ldc, il, s);
    else restrict_t<float, 0>(xfer, Nc, bcm, rf, bc, nrhs, ldf, ldc, il, s);
  } else if (K == 1) {
    if (prec == 0) restrict_t<double, 1>(xfer, Nc, bcm, rf, bc, nrhs, ldf, ldc, il, s);
    else restrict_t<float, 1>(xfer, Nc, bcm, rf, bc, nrhs, ldf, ldc, il, s);
  } else {
    if (prec == 0) restrict_t<double, 2>(xfer, Nc, bcm, rf, bc, nrhs, ldf, ldc, il, s);
    else restrict_t<float, 2>(xfer, Nc, bcm, rf, bc, nrhs, ldf, ldc, il, s);
  }
}

template <typename T, int K>
static void prolong_t(const void* xfer, int Nc, int bcm, const void* xc, void* xf, int nrhs, int64_t ldc,
                      int64_t ldf, int il, hipStream_t s) {
  const int64_t n = (int64_t)Nc * Nc;
  if constexpr (K >= 1 && std::is_same<T, float>::value)
    if (il > 0) {
      hipLaunchKernelGGL((k_prolong<T, K, true>), dim3((unsigned)((n * il + 255) / 256)), dim3(256), 0, s,
                         (const Xfer<T, K>*)xfer, Nc, bcm, (const T*)xc, (T*)xf, (int64_t)il, (int64_t)il);
      return;
    }
  hipLaunchKernelGGL((k_prolong<T, K>), dim3((unsigned)((n + 255) / 256), nrhs), dim3(256), 0, s,
                     (const Xfer<T, K>*)xfer, Nc, bcm, (const T*)xc, (T*)xf, ldc, ldf);
}
void launch_prolong(int K, int prec, const void* xfer, int Nc, int bcm, const void* xc, void* xf, int nrhs,
                    int64_t ldc, int64_t ldf, hipStream_t s, int il) {
  if (K == 0) {
    if (prec == 0) prolong_t<double, 0>(xfer, Nc, bcm, xc, xf, nrhs, ldc, ldf, il, s);
    else prolong_t<float, 0>(xfer, Nc, bcm, xc, xf, nrhs, ldc, ldf, il, s);
  } else if (K == 1) {
    if (prec == 0) prolong_t<double, 1>(xfer, Nc, bcm, xc, xf, nrhs, ldc, ldf, il, s);
    else prolong_t<float, 1>(xfer, Nc, bcm, xc, xf, nrhs, ldc, ldf, il, s);
  } else {
    if (prec == 0) prolong_t<double, 2>(xfer, Nc, bcm, xc, xf, nrhs, ldc, ldf, il, s);
    else prolong_t<float, 2>(xfer, Nc, bcm, xc, xf, nrhs, ldc, ldf, il, s);
  }
}

void launch_coarse(int prec, int n, const double* inv, const void* b, void* x, int nrhs, hipStream_t s, int il) {
  const size_t sh = (size_t)n * sizeof(double);
  const int64_t cs = il > 0 ? 1 : n, es = il > 0 ? il : 1;
  if (prec == 0)
    hipLaunchKernelGGL((k_coarse<double>), dim3(nrhs), dim3(256), sh, s, n, inv, (const double*)b, (double*)x, cs, es);
  else
    hipLaunchKernelGGL((k_coarse<float>), dim3(nrhs), dim3(256), sh, s, n, inv, (const float*)b, (float*)x, cs, es);
}

void launch_fill_zero(int prec, void* x, int64_t n, hipStream_t s) {
  const unsigned g = grid_for(n);
  if (prec == 0) hipLaunchKernelGGL((k_fill<double>), dim3(g), dim3(256), 0, s, (double*)x, 0.0, n);
  else hipLaunchKernelGGL((k_fill<float>), dim3(g), dim3(256), 0, s, (float*)x, 0.0f, n);
}

void launch_identity(int prec, void* x, int64_t n, int64_t col0, int nrhs, hipStream_t s) {
  const unsigned g = grid_for(n * nrhs);
  if (prec == 0) hipLaunchKernelGGL((k_identity<double>), dim3(g), dim3(256), 0, s, (double*)x, n, col0, nrhs);
  else hipLaunchKernelGGL((k_identity<float>), dim3(g), dim3(256), 0, s, (float*)x, n, col0, nrhs);
}

template <typename T, int NR>
static void dense_t(const void* B, int64_t n, const void* x, void* y, int64_t cs, int64_t es, hipStream_t s) {
  const unsigned g = (unsigned)((n + 3) / 4);
  hipLaunchKernelGGL((k_dense_rows<T, NR>), dim3(g), dim3(256), 0, s, (const T*)B, n, (const T*)x, (T*)y, cs, es);
}
template <typename T>
static void dense_nr(const void* B, int64_t n, const void* x, void* y, int nrhs, int il, hipStream_t s) {
  // columns in groups of at most 8 (registers of the partial sums); column c at c * cs,
  // entries es apart
  const size_t ts = sizeof(T);
  const int64_t cs = il > 0 ? 1 : n, es = il > 0 ? il : 1;
  for (int c0 = 0; c0 < nrhs; c0 += 8) {
    const void* xc = (const char*)x + (size_t)c0 * cs * ts;
    void* yc = (char*)y + (size_t)c0 * cs * ts;
    switch (std::min(8, nrhs - c0)) {
      case 1: dense_t<T, 1>(B, n, xc, yc, cs, es, s); break;
      case 2: dense_t<T, 2>(B, n, xc, yc, cs, es, s); break;
      case 3: dense_t<T, 3>(B, n, xc, yc, cs, es, s); break;
      case 4: dense_t<T, 4>(B, n, xc, yc, cs, es, s); break;
      case 5: dense_t<T, 5>(B, n, xc, yc, cs, es, s); break;
      case 6: dense_t<T, 6>(B, n, xc, yc, cs, es, s); break;
      case 7: dense_t<T, 7>(B, n, xc, yc, cs, es, s); break;
      default: dense_t<T, 8>(B, n, xc, yc, cs, es, s); break;
    }
  }
}
void launch_dense_gemv(int prec, const void* B, int64_t n, const void* x, void* y, int nrhs, hipStream_t s, int il) {
  if (prec == 0) dense_nr<double>(B, n, x, y, nrhs, il, s);
  else dense_nr<float>(B, n, x, y, nrhs, il, s);
}

void launch_cast(int to_prec, int from_prec, const void* src, void* dst, int64_t n, hipStream_t s) {
  const unsigned g = grid_for(n);
  if (to_prec == 0 && from_prec == 1)
    hipLaunchKernelGGL((k_cast<double, float>), dim3(g), dim3(256), 0, s, (const float*)src, (double*)dst, n);
  else if (to_prec == 1 && from_prec == 0)
    hipLaunchKernelGGL((k_cast<float, double>), dim3(g), dim3(256), 0, s, (const double*)src, (float*)dst, n);
  else if (to_prec == 0)
    hipLaunchKernelGGL((k_cast<double, double>), dim3(g), dim3(256), 0, s, (const double*)src, (double*)dst, n);
  else
    hipLaunchKernelGGL((k_cast<float, float>), dim3(g), dim3(256), 0, s, (const float*)src, (float*)dst, n);
}

void launch_cast_il(int to_prec, int from_prec, const void* src, void* dst, int64_t n, int64_t ld, int nrhs, int w,
                    bool to_il, hipStream_t s) {
  const unsigned g = (unsigned)((n + 63) / 64);
  if (to_il) {
    // the interleaved side is FP32 (the arithmetic of a several-column V-cycle)
    if (from_prec == 0)
      hipLaunchKernelGGL((k_to_il<float, double>), dim3(g), dim3(256), 0, s, (const double*)src, (float*)dst, n, ld,
                         nrhs, w);
    else
      hipLaunchKernelGGL((k_to_il<float, float>), dim3(g), dim3(256), 0, s, (const float*)src, (float*)dst, n, ld,
                         nrhs, w);
  } else {
    if (to_prec == 0)
      hipLaunchKernelGGL((k_from_il<double, float>), dim3(g), dim3(256), 0, s, (const float*)src, (double*)dst, n,
                         ld, nrhs, w);
    else
      hipLaunchKernelGGL((k_from_il<float, float>), dim3(g), dim3(256), 0, s, (const float*)src, (float*)dst, n, ld,
                         nrhs, w);
  }
}

void launch_copy_constrained(int K, int N, int bcm, const double* src, void* dst, int dst_prec, int nrhs, int64_t ld,
                             hipStream_t s) {
  const int n = 4 * N * (K + 1);
  dim3 g((n + 255) / 256, nrhs), bl(256);
  if (K == 0) {
    if (dst_prec == 0) hipLaunchKernelGGL((k_copy_cons<double, 0>), g, bl, 0, s, N, bcm, src, (double*)dst, ld);
    else hipLaunchKernelGGL((k_copy_cons<float, 0>), g, bl, 0, s, N, bcm, src, (float*)dst, ld);
  } else if (K == 1) {
    if (dst_prec == 0) hipLaunchKernelGGL((k_copy_cons<double, 1>), g, bl, 0, s, N, bcm, src, (double*)dst, ld);
    else hipLaunchKernelGGL((k_copy_cons<float, 1>), g, bl, 0, s, N, bcm, src, (float*)dst, ld);
  } else {
    if (dst_prec == 0) hipLaunchKernelGGL((k_copy_cons<double, 2>), g, bl, 0, s, N, bcm, src, (double*)dst, ld);
    else hipLaunchKernelGGL((k_copy_cons<float, 2>), g, bl, 0, s, N, bcm, src, (float*)dst, ld);
  }
}

int dots_partial_count() { return kDotBlocks; }

void launch_dots(const double* V, int nvec, int64_t ldv, const double* w, int64_t n, double* partial, double* out,
                 int nrhs, int64_t ostride, hipStream_t s) {
  hipLaunchKernelGGL(k_dots, dim3(kDotBlocks, nrhs), dim3(256), 0, s, V, nvec, ldv, w, n, partial);
  hipLaunchKernelGGL(k_dots_final, dim3(nvec, nrhs), dim3(256), 0, s, partial, kDotBlocks, out, ostride);
}

void launch_axpys(double* w, const double* V, int nvec, int64_t ldv, const double* coef, int64_t cstride, double sign,
                  int64_t n, int nrhs, hipStream_t s) {
  hipLaunchKernelGGL(k_axpys<double>, dim3(grid_for(n), nrhs), dim3(256), 0, s, w, V, nvec, ldv, coef, cstride,
                     sign, n);
}

void launch_axpys_f32(double* w, const float* V, int nvec, int64_t ldv, const double* coef, int64_t cstride,
                      double sign, int64_t n, int nrhs, hipStream_t s) {
  hipLaunchKernelGGL(k_axpys<float>, dim3(grid_for(n), nrhs), dim3(256), 0, s, w, V, nvec, ldv, coef, cstride,
                     sign, n);
}

void launch_scale(double* dst, const double* src, const double* denom, int64_t dstride, const int32_t* live,
                  bool take_sqrt, int64_t n, int nrhs, hipStream_t s) {
  hipLaunchKernelGGL(k_scale, dim3(grid_for(n), nrhs), dim3(256), 0, s, dst, src, denom, dstride, live,
                     (int)take_sqrt, n);
}

void launch_sub(double* r, const double* b, const double* ax, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_sub, dim3(grid_for(n)), dim3(256), 0, s, r, b, ax, n);
}

// ---------------------------------------------------------------------------
// Static scratch of the allocation-free V-cycle entry point: one array per device,
// held from the moment the code object is loaded until the process ends.  Host code
// must not pass `scratch` itself to a kernel (in host code it names a host-side
// stand-in): its device address is looked up once per device and cached.
// ---------------------------------------------------------------------------
}  // namespace bmg

static __device__ __align__(256) unsigned char scratch[bmg::kStaticScratchBytes];

namespace bmg {
namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};
}  // namespace

hipError_t static_scratch(void** ptr, size_t* bytes) {
  *ptr = nullptr;
  if (bytes) *bytes = kStaticScratchBytes;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* a = nullptr;
    e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = a;
  }
  *ptr = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace bmg
