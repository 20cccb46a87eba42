// Host side of the library: parameter checks, workspace layout, setup products
// (kappa hierarchy, reference-element data, vertex-patch pseudo-inverses, coarse
// inverse), the V-cycle schedule, FP64 flexible GMRES and the C ABI (bmg.h).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <new>
#include <cstdio>
#include <cstring>
#include <exception>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/bmg.h"
#include "common.hpp"
#include "refelem.hpp"

using namespace bmg;

namespace {

constexpr size_t kAlign = 256;

struct LevelInfo {
  int N = 0;
  double h = 0.0;
  int64_t n_u = 0, n_p = 0, ndof = 0;
  std::vector<double> kappa;
  // per colour: number of patches, extended-layout patch count
  int npatch[9] = {0};
  int next[9] = {0};
  // device pointers (into the workspace)
  void* kap = nullptr;      // preconditioner arithmetic
  double* kap64 = nullptr;  // FP64 (operator of bmg_apply and of the outer loop)
  void *x = nullptr, *b = nullptr, *r = nullptr;
  void* inv[9] = {nullptr};
  void* invx[9] = {nullptr};
  int32_t* extidx[9] = {nullptr};
  // levels whose interior patches run the several-column kernel: the other patches
  // of each colour (colour-class indices; host copy and device copy)
  std::vector<int32_t> hblist[9];
  int32_t* blist[9] = {nullptr};
  int32_t* mrtab = nullptr;  // template table of the several-column kernel (levels with N >= 4)
};

}  // namespace

struct bmg_ctx {
  bmg_params p{};
  int K = 1, prec = 0, sprec = 0, bcm = 0;
  int R = 1;  // right-hand sides (columns of every vector)
  size_t tsize = 8, ssize = 8;
  hipStream_t stream = nullptr;
  bool own_ws = false;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  std::vector<LevelInfo> lev;
  RefData ref;
  void* elemT = nullptr;
  void* elemInt = nullptr;  // ElemInt<float, K> of the several-column colour step (or null)
  void* elem64 = nullptr;
  void* xferT = nullptr;
  double* coarse_inv = nullptr;
  // dense operator of the coarse sub-cycle: B_jc for level jc (0 = none)
  int jc = 0;
  void* dense = nullptr;  // B_jc, symmetric: the column-major batch output is read by rows
  // setup batch (unit vectors through the V-cycle of level jc), overlapping the Krylov storage
  int batch_chunk = 0;
  char* region = nullptr;
  // Krylov storage: V (restart + 1 FP64 vectors of R columns) and Z (restart vectors,
  // FP64 for the FP64 V-cycle, FP32 otherwise: the V-cycle's output is FP32 then, so
  // storing it as FP32 is exact); zsize = bytes per entry of Z
  double* V = nullptr;
  void* Z = nullptr;
  size_t zsize = 8;
  double *hdev = nullptr, *partial = nullptr;
  int32_t* live = nullptr;  // per right-hand side: 1 while its Arnoldi process runs
  // several-column bfloat16 handles keep the V-cycle's level vectors as interleaved
  // records of il values (n_rhs rounded up to a power of two >= 4; the extra columns
  // zero): entry g of column r at g * il + r.  0: n_rhs column-major blocks
  int il = 0;
  // V-cycle captured as a graph (captured on a private stream, launched on `stream`)
  hipStream_t cap_stream = nullptr;
  hipGraph_t vgraph = nullptr;
  hipGraphExec_t vexec = nullptr;
  bool graph_failed = false;
  bool layout_mismatch = false;  // the kernel's layout rule disagrees with the patch construction
  // optional event timing of the colour launches of one level
  int timing_level = -1;
  std::vector<hipEvent_t> ev;
  size_t ev_used = 0;
  int64_t timed_launches = 0;
  double timed_bytes = 0.0;
  std::string err;
};

// Independent problems solved together: one handle per problem, worker streams
// that the solves are spread over (one host thread per stream).
struct bmg_batch {
  std::vector<bmg_handle> h;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> done;
  hipEvent_t start = nullptr;
  hipStream_t user = nullptr;
  std::string err;
};

namespace {

// message of the last bmg_setup of this thread that failed after validation
thread_local std::string g_setup_err = "null handle";

bmg_status fail(bmg_ctx* c, bmg_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

#define HIPCHK(ctx, call)                                                                       \
  do {                                                                                          \
    hipError_t e_ = (call);                                                                     \
    if (e_ != hipSuccess) return fail(ctx, BMG_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

int64_t n_u_of(int N, int k) { return 2LL * N * (N + 1) * (k + 1) + 2LL * k * (k + 1) * N * N; }
int64_t n_p_of(int N, int k) { return (int64_t)(k + 1) * (k + 1) * N * N; }

constexpr int kMaxRhs = 16;
constexpr int64_t kMaxCoarseDof = 4096;



bmg_status check_params(const bmg_params* p) {
  if (!p) return BMG_E_ARG;
  if (p->k < 0 || p->k > 2) return BMG_E_UNSUPPORTED;
  if (p->n0 < 2 || p->n0 > 64 || p->levels < 0 || p->levels > 12) return BMG_E_ARG;
  // the coarse solve keeps A_0's dense inverse (host Gauss-Jordan at setup, the
  // right-hand side staged in LDS when applied): at most kMaxCoarseDof unknowns
  if (n_u_of(p->n0, p->k) + n_p_of(p->n0, p->k) > kMaxCoarseDof) return BMG_E_UNSUPPORTED;
  if ((int64_t)p->n0 << p->levels > 4096) return BMG_E_ARG;
  if (!(p->mu >= 0.0) || !std::isfinite(p->mu) || !(p->sigma > 0.0) || !std::isfinite(p->sigma)) return BMG_E_ARG;
  for (int s = 0; s < 4; ++s)
    if (p->bc[s] != BMG_BC_DIRICHLET && p->bc[s] != BMG_BC_OPEN) return BMG_E_ARG;
  if (p->cycle != BMG_CYCLE_STANDARD && p->cycle != BMG_CYCLE_VARIABLE) return BMG_E_ARG;
  if (p->m_fine < 1 || p->m_fine > 64) return BMG_E_ARG;
  if (p->precond_prec != BMG_P_FP64 && p->precond_prec != BMG_P_FP32 && p->precond_prec != BMG_P_BF16)
    return BMG_E_ARG;
  if (p->restart < 1 || p->restart > 512) return BMG_E_ARG;
  if (p->dense_coarse_max < 0 || p->dense_coarse_max > 65535) return BMG_E_ARG;
  if (p->n_rhs < 0 || p->n_rhs > kMaxRhs) return BMG_E_ARG;
  if (p->colouring != COLOURING_S9 && p->colouring != COLOURING_L8) return BMG_E_ARG;
  if (p->coarse_kappa < BMG_KAPPA_ARITHMETIC || p->coarse_kappa > BMG_KAPPA_GEOMETRIC) return BMG_E_ARG;
  if (p->smoother != BMG_SMOOTHER_MULTIPLICATIVE && p->smoother != BMG_SMOOTHER_ADDITIVE) return BMG_E_ARG;
  if (p->smoother == BMG_SMOOTHER_ADDITIVE && !(p->omega > 0.0 && p->omega <= 1.0)) return BMG_E_ARG;
  if (p->setup_on_host != 0 && p->setup_on_host != 1) return BMG_E_ARG;
  if (p->rotated_min_n < 0 || p->rotated_min_n > 4096) return BMG_E_ARG;
  if (p->columns_per_block < 0 || p->columns_per_block > 16) return BMG_E_ARG;
  return BMG_OK;
}

// --------------------------------------------------------------------------
// Patch layout on the host (same slot order as the smoother kernel)
// --------------------------------------------------------------------------
struct HostIdx {
  int N, k, NB, NA, NV, NP, NL, NI, bcm;
  HostIdx(int N_, int k_, int bcm_) : N(N_), k(k_), bcm(bcm_) {
    NB = k + 1;
    NA = k + 2;
    NV = NA * NB;
    NP = NB * NB;
    NL = 2 * NV + NP;
    NI = 2 * k * NB;
  }
  int64_t xface(int i, int cy, int b) const { return ((int64_t)cy * (N + 1) + i) * NB + b; }
  int64_t yface(int j, int cx, int b) const { return (int64_t)N * (N + 1) * NB + ((int64_t)j * N + cx) * NB + b; }
  int64_t inter(int64_t c, int comp, int a, int b) const {
    return 2LL * N * (N + 1) * NB + c * NI + (comp * k + (a - 2)) * NB + b;
  }
  int64_t pres(int64_t c, int q) const { return n_u_of(N, k) + c * NP + q; }
  int64_t g(int cx, int cy, int d) const {
    const int64_t c = (int64_t)cy * N + cx;
    if (d < NV) {
      const int a = d / NB, b = d % NB;
      return a == 0 ? xface(cx, cy, b) : a == 1 ? xface(cx + 1, cy, b) : inter(c, 0, a, b);
    }
    if (d < 2 * NV) {
      const int e = d - NV, a = e / NB, b = e % NB;
      return a == 0 ? yface(cy, cx, b) : a == 1 ? yface(cy + 1, cx, b) : inter(c, 1, a, b);
    }
    return pres(c, d - 2 * NV);
  }
  bool cons(int cx, int cy, int d) const {
    if (d < NV) {
      const int a = d / NB;
      return (a == 0 && cx == 0 && (bcm & 1)) || (a == 1 && cx == N - 1 && (bcm & 2));
    }
    if (d < 2 * NV) {
      const int a = (d - NV) / NB;
      return (a == 0 && cy == 0 && (bcm & 4)) || (a == 1 && cy == N - 1 && (bcm & 8));
    }
    return false;
  }
  bool in(int cx, int cy) const { return cx >= 0 && cx < N && cy >= 0 && cy < N; }
};

const int kGroupH[12][4] = {{0, 0, -1, 0}, {0, 1, 1, 0},  {1, 1, -1, 0}, {2, 0, -1, 0},
                            {2, 1, 3, 0},  {3, 1, -1, 0}, {0, 2, -1, 0}, {1, 2, -1, 0},
                            {0, 3, 2, 2},  {1, 3, 3, 2},  {2, 3, -1, 0}, {3, 3, -1, 0}};
const int kRegularH[4] = {1, 4, 8, 9};

struct PatchLayout {
  bool ext = false;
  int ns = 0;
  std::vector<int64_t> g;      // per slot entry, -1 = not part of the patch space
  std::vector<int> boundary;   // per slot entry: a free normal dof on the domain boundary
  std::vector<int> lane;       // per (slot s, local d): entry index or -1
};

PatchLayout build_layout(const HostIdx& I, int vx, int vy, bool ext) {
  PatchLayout P;
  P.ext = ext;
  const int nf = ext ? 12 : 4;
  P.ns = nf * I.NB + 4 * I.NI + 4 * I.NP;
  P.g.assign(P.ns, -1);
  P.boundary.assign(P.ns, 0);
  P.lane.assign(4 * I.NL, -1);
  auto kind_local = [&](int kind, int b) { return (kind >= 2 ? I.NV : 0) + (kind & 1) * I.NB + b; };
  for (int t = 0; t < P.ns; ++t) {
    if (t < nf * I.NB) {
      const int grp = ext ? t / I.NB : kRegularH[t / I.NB];
      const int b = t % I.NB;
      const int sA = kGroupH[grp][0], kA = kGroupH[grp][1], sB = kGroupH[grp][2], kB = kGroupH[grp][3];
      const int axA = vx - 1 + (sA & 1), ayA = vy - 1 + (sA >> 1);
      const bool vA = I.in(axA, ayA);
      bool vB = false;
      int axB = 0, ayB = 0;
      if (sB >= 0) {
        axB = vx - 1 + (sB & 1);
        ayB = vy - 1 + (sB >> 1);
        vB = I.in(axB, ayB);
      }
      bool ok, bnd;
      int cxu, cyu, du;
      if (sB >= 0) {
        ok = vA || vB;
        bnd = vA != vB;
        cxu = vA ? axA : axB;
        cyu = vA ? ayA : ayB;
        du = kind_local(vA ? kA : kB, b);
      } else {
        int ox = axA, oy = ayA;
        if (kA == 0) ox -= 1;
        else if (kA == 1) ox += 1;
        else if (kA == 2) oy -= 1;
        else oy += 1;
        ok = vA && !I.in(ox, oy);
        bnd = true;
        cxu = axA;
        cyu = ayA;
        du = kind_local(kA, b);
      }
      if (ok && !I.cons(cxu, cyu, du)) {
        P.g[t] = I.g(cxu, cyu, du);
        P.boundary[t] = bnd;
        if (vA) P.lane[sA * I.NL + kind_local(kA, b)] = t;
        if (vB) P.lane[sB * I.NL + kind_local(kB, b)] = t;
      }
    } else {
      const int e = t - nf * I.NB;
      int s, d;
      if (e < 4 * I.NI) {
        s = e / I.NI;
        const int w2 = e % I.NI, comp = w2 / (I.k * I.NB), rem = w2 % (I.k * I.NB);
        d = comp * I.NV + (2 + rem / I.NB) * I.NB + rem % I.NB;
      } else {
        s = (e - 4 * I.NI) / I.NP;
        d = 2 * I.NV + (e - 4 * I.NI) % I.NP;
      }
      const int cx = vx - 1 + (s & 1), cy = vy - 1 + (s >> 1);
      if (I.in(cx, cy)) {
        P.g[t] = I.g(cx, cy, d);
        P.lane[s * I.NL + d] = t;
      }
    }
  }
  return P;
}

bool needs_ext(const HostIdx& I, int vx, int vy) {
  PatchLayout P = build_layout(I, vx, vy, true);
  for (int grp : {0, 2, 3, 5, 6, 7, 10, 11})
    for (int b = 0; b < I.NB; ++b)
      if (P.g[grp * I.NB + b] >= 0) return true;
  return false;
}

// The rule the smoother kernel uses to pick the layout without a table lookup:
// an outer face of the patch lies on an open side.
bool ext_rule(const HostIdx& I, int vx, int vy) {
  return (vx == 1 && !(I.bcm & 1)) || (vx == I.N - 1 && !(I.bcm & 2)) || (vy == 1 && !(I.bcm & 4)) ||
         (vy == I.N - 1 && !(I.bcm & 8));
}

// Dense A restricted to the patch layout (invalid entries: zero rows/cols),
// from the same cell and face blocks the kernels use.
void patch_matrix(const HostIdx& I, const RefData& R, const LevelInfo& L, int vx, int vy, const PatchLayout& P,
                  std::vector<double>& A) {
  const int ns = P.ns, NV = I.NV, NP = I.NP, NL = I.NL;
  A.assign((size_t)ns * ns, 0.0);
  auto add = [&](int s, int d, int s2, int e, double v) {
    const int t = P.lane[s * NL + d], u = P.lane[s2 * NL + e];
    if (t >= 0 && u >= 0) A[(size_t)t * ns + u] += v;
  };
  const double h = L.h, hh = h * h;
  for (int s = 0; s < 4; ++s) {
    const int cx = vx - 1 + (s & 1), cy = vy - 1 + (s >> 1);
    if (!I.in(cx, cy)) continue;
    const double khh = L.kappa[(size_t)cy * I.N + cx] * hh;
    for (int comp = 0; comp < 2; ++comp) {
      const int o = comp * NV;
      const std::vector<double>& Dm = comp == 0 ? R.Dx : R.Dy;
      for (int d = 0; d < NV; ++d) {
        for (int e = 0; e < NV; ++e) add(s, o + d, s, o + e, R.Kmu[d * NV + e] + khh * R.M[d * NV + e]);
        for (int q = 0; q < NP; ++q) {
          add(s, o + d, s, 2 * NV + q, -h * Dm[q * NV + d]);
          add(s, 2 * NV + q, s, o + d, -h * Dm[q * NV + d]);
        }
      }
      // faces across which this component is tangential: lower (side 1 of the face) and upper (side 0)
      for (int up = 0; up < 2; ++up) {
        int ncx = cx, ncy = cy, side;
        if (comp == 0) {
          ncy += up ? 1 : -1;
          side = up ? 3 : 2;
        } else {
          ncx += up ? 1 : -1;
          side = up ? 1 : 0;
        }
        if (!I.in(ncx, ncy)) {
          if ((I.bcm >> side) & 1) {
            const std::vector<double>& Nb = R.Nb[up];
            for (int d = 0; d < NV; ++d)
              for (int e = 0; e < NV; ++e) add(s, o + d, s, o + e, Nb[d * NV + e]);
          }
          continue;
        }
        const std::vector<double>& Fs = R.F[up ? 0 : 3];
        const std::vector<double>& Fn = R.F[up ? 1 : 2];
        for (int d = 0; d < NV; ++d)
          for (int e = 0; e < NV; ++e) add(s, o + d, s, o + e, Fs[d * NV + e]);
        const int dx = ncx - (vx - 1), dy = ncy - (vy - 1);
        if (dx >= 0 && dx <= 1 && dy >= 0 && dy <= 1) {
          const int s2 = dy * 2 + dx;
          for (int d = 0; d < NV; ++d)
            for (int e = 0; e < NV; ++e) add(s, o + d, s2, o + e, Fn[d * NV + e]);
        }
      }
    }
  }
}

// Gauss-Jordan inverse with partial pivoting (row-major, in place on a copy).
bool gauss_jordan(int n, std::vector<double>& a, std::vector<double>& inv) {
  inv.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    double best = std::fabs(a[(size_t)c * n + c]);
    for (int r = c + 1; r < n; ++r) {
      const double v = std::fabs(a[(size_t)r * n + c]);
      if (v > best) {
        best = v;
        piv = r;
      }
    }
    if (!(best > 0.0)) return false;
    if (piv != c) {
      std::swap_ranges(a.begin() + (size_t)piv * n, a.begin() + (size_t)piv * n + n, a.begin() + (size_t)c * n);
      std::swap_ranges(inv.begin() + (size_t)piv * n, inv.begin() + (size_t)piv * n + n, inv.begin() + (size_t)c * n);
    }
    const double d = 1.0 / a[(size_t)c * n + c];
    for (int j = 0; j < n; ++j) {
      a[(size_t)c * n + j] *= d;
      inv[(size_t)c * n + j] *= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = a[(size_t)r * n + c];
      if (f == 0.0) continue;
      double* ar = &a[(size_t)r * n];
      double* ir = &inv[(size_t)r * n];
      const double* ac = &a[(size_t)c * n];
      const double* ic = &inv[(size_t)c * n];
      for (int j = 0; j < n; ++j) {
        ar[j] -= f * ac[j];
        ir[j] -= f * ic[j];
      }
    }
  }
  return true;
}

// Pseudo-inverse of the patch matrix in the layout (ns x ns, zero for invalid
// entries).  If no free normal dof of the patch lies on the domain boundary, the
// constant patch pressure spans the kernel: invert the matrix bordered with that
// (normalised) vector and keep the leading block.
bool patch_pinv(const HostIdx& I, const PatchLayout& P, const std::vector<double>& A, std::vector<double>& out,
                bool* singular) {
  std::vector<int> idx;
  bool has_bnd = false;
  for (int t = 0; t < P.ns; ++t)
    if (P.g[t] >= 0) {
      idx.push_back(t);
      if (P.boundary[t]) has_bnd = true;
    }
  const int n = (int)idx.size();
  const bool sing = !has_bnd;
  if (singular) *singular = sing;
  const int m = sing ? n + 1 : n;
  std::vector<double> a((size_t)m * m, 0.0), inv;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) a[(size_t)i * m + j] = A[(size_t)idx[i] * P.ns + idx[j]];
  if (sing) {
    // constant pressure: the L_0 L_0 coefficient of every patch cell
    std::vector<double> c(n, 0.0);
    int cnt = 0;
    for (int i = 0; i < n; ++i) {
      const int64_t gi = P.g[idx[i]];
      const int64_t nu = n_u_of(I.N, I.k);
      if (gi >= nu && (gi - nu) % I.NP == 0) {
        c[i] = 1.0;
        ++cnt;
      }
    }
    for (int i = 0; i < n; ++i) {
      c[i] /= std::sqrt((double)cnt);
      a[(size_t)i * m + n] = c[i];
      a[(size_t)n * m + i] = c[i];
    }
  }
  if (!gauss_jordan(m, a, inv)) return false;
  out.assign((size_t)P.ns * P.ns, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) out[(size_t)idx[i] * P.ns + idx[j]] = inv[(size_t)i * m + j];
  return true;
}

// f(i) for i < n on the host threads; an exception thrown by f (a failed host
// allocation) stops the loop and is rethrown to the caller after the join.
template <typename F>
void parallel_for(int n, F&& f) {
  unsigned nt = std::thread::hardware_concurrency();
  if (nt == 0) nt = 1;
  if (nt > 32) nt = 32;
  if ((int)nt > n) nt = std::max(1, n);
  std::atomic<int> next{0};
  std::exception_ptr first;
  std::mutex mu;
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nt; ++t)
    th.emplace_back([&]() {
      for (;;) {
        const int i = next.fetch_add(1);
        if (i >= n) break;
        try {
          f(i);
        } catch (...) {
          std::lock_guard<std::mutex> g(mu);
          if (!first) first = std::current_exception();
          next.store(n);
        }
      }
    });
  for (auto& t : th) t.join();
  if (first) std::rethrow_exception(first);
}

// --------------------------------------------------------------------------
// Workspace layout
// --------------------------------------------------------------------------
struct Bump {
  char* base;
  size_t off = 0;
  explicit Bump(char* b) : base(b) {}
  void* take(size_t bytes) {
    off = (off + kAlign - 1) / kAlign * kAlign;
    void* p = base ? base + off : nullptr;
    off += bytes;
    return p;
  }
};

template <typename T>
size_t elem_bytes(int K) {
  return K == 0 ? sizeof(Elem<T, 0>) : K == 1 ? sizeof(Elem<T, 1>) : sizeof(Elem<T, 2>);
}
template <typename T>
size_t xfer_bytes(int K) {
  return K == 0 ? sizeof(Xfer<T, 0>) : K == 1 ? sizeof(Xfer<T, 1>) : sizeof(Xfer<T, 2>);
}

int nsr_of(int k) { return 4 * (k + 1) + 8 * k * (k + 1) + 4 * (k + 1) * (k + 1); }
int nse_of(int k) { return 12 * (k + 1) + 8 * k * (k + 1) + 4 * (k + 1) * (k + 1); }
// Stored entries of one patch pseudo-inverse: rotated symmetric block (RT_1 on levels
// with N >= 192, where the smoother is bandwidth-bound; R[d n + t] = A+[t][(t + d)
// mod n] for d = 0 .. n/2, n even) or full column-major block.
bool packed_level(const bmg_ctx* c, int N) {
  // Several columns in FP32 arithmetic keep full blocks where the colour kernel
  // multiplies a block by all columns at once on the matrix cores from memory (FP32
  // entries, and RT_0 bfloat16 entries); RT_1 / RT_2 with bfloat16 entries and several
  // columns are stored rotated on every level (half the memory: 2048^2 RT_2 with 16
  // columns only fits that way), staged per patch in LDS for the product.
  if (c->R > 1 && c->prec != 0) return c->K >= 1 && c->sprec == 2;
  // one column (or FP64): rotated on the bandwidth-bound levels (N >= 192 unless the
  // tile parameter says otherwise); RT_2 in FP64 reads its rotated blocks from memory
  // in the product
  const int nmin = c->p.rotated_min_n > 0 ? c->p.rotated_min_n : 192;
  return N >= nmin && (c->K <= 1 || c->prec == 0);
}
// Interior patches of level j run the several-column kernel (k_colour_mr): 2..16
// FP32 columns, bfloat16 rotated inverses, RT_1 or RT_2, multiplicative smoother.
bool mr_handle(const bmg_ctx* c) {
  return c->R > 1 && c->prec != 0 && c->sprec == 2 && c->K >= 1 && c->p.smoother == BMG_SMOOTHER_MULTIPLICATIVE;
}
bool mr_level(const bmg_ctx* c, int N, int nrhs) { return mr_handle(c) && packed_level(c, N) && nrhs >= 2 && nrhs <= 16; }

int64_t inv_entries(bool packed, int ns) { return packed ? (int64_t)ns * (ns / 2 + 1) : (int64_t)ns * ns; }

// Coarse sub-cycle applied as one dense matrix: the finest level jc >= 1 whose
// dof count is at most dense_coarse_max (0 = none).
int choose_jc(const bmg_ctx* c) {
  int jc = 0;
  for (int j = 1; j < (int)c->lev.size(); ++j)
    if (c->lev[j].ndof <= (int64_t)c->p.dense_coarse_max) jc = j;
  return jc;
}

// per right-hand side in hdev: [0, m+2) first Gram-Schmidt pass, [m+2, 2m+4) second,
// 2m+4: squared norm, then spare entries
int64_t hd_stride(const bmg_ctx* c) { return 2 * (c->p.restart + 2) + 8; }

// assigns every device pointer of the context; with a null base only sizes
size_t layout(bmg_ctx* c, char* base) {
  Bump B(base);
  const int K = c->K;
  const size_t ts = c->tsize, ss = c->ssize;
  const int nsr = nsr_of(K), nse = nse_of(K);
  for (size_t j = 0; j < c->lev.size(); ++j) {
    LevelInfo& L = c->lev[j];
    const int64_t nc = (int64_t)L.N * L.N;
    L.kap = B.take(nc * ts);
    L.kap64 = (double*)B.take(nc * sizeof(double));
    const int64_t w = c->il > 0 ? c->il : c->R;  // columns (record width) of a level vector
    L.x = B.take(L.ndof * w * ts);
    L.b = B.take(L.ndof * w * ts);
    L.r = B.take(L.ndof * w * ts);
    if (j > 0)
      for (int col = 0; col < 9; ++col) {
        const bool pk = packed_level(c, L.N);
        L.inv[col] = B.take((size_t)L.npatch[col] * inv_entries(pk, nsr) * ss);
        L.invx[col] = B.take((size_t)std::max(L.next[col], 1) * inv_entries(pk, nse) * ss);
        L.extidx[col] = (int32_t*)B.take((size_t)std::max(L.npatch[col], 1) * sizeof(int32_t));
        if (mr_handle(c))
          L.blist[col] = (int32_t*)B.take((size_t)std::max<size_t>(L.hblist[col].size(), 1) * sizeof(int32_t));
      if (mr_handle(c) && L.N >= 4) L.mrtab = (int32_t*)B.take((size_t)mr_table_entries(K) * 4 * sizeof(int32_t));
      }
  }
  const int64_t n0 = c->lev[0].ndof;
  c->coarse_inv = (double*)B.take((size_t)n0 * n0 * sizeof(double));
  c->jc = choose_jc(c);
  if (c->jc > 0) {
    const int64_t nd = c->lev[c->jc].ndof;
    c->dense = B.take((size_t)nd * nd * ts);
  }
  c->elemT = B.take(c->prec == 0 ? elem_bytes<double>(K) : elem_bytes<float>(K));
  c->elem64 = B.take(elem_bytes<double>(K));
  c->elemInt = nullptr;
  if (mr_handle(c))
    c->elemInt = B.take(K == 1 ? sizeof(ElemInt<float, 1>) : sizeof(ElemInt<float, 2>));
  c->xferT = B.take(c->prec == 0 ? xfer_bytes<double>(K) : xfer_bytes<float>(K));
  const int64_t n = c->lev.back().ndof * c->R;  // all columns of one Krylov vector
  const int m = c->p.restart;
  c->zsize = c->prec == 0 ? sizeof(double) : sizeof(float);
  // one region shared by the Krylov vectors (solve) and the setup batch; the residual
  // of a cycle start and A z_i are formed in the next free slot of V
  const size_t kry = (size_t)(m + 1) * n * sizeof(double) + (size_t)m * n * c->zsize + 4 * kAlign;
  size_t per_col = 0;
  for (int j = 0; j <= c->jc; ++j) per_col += 3 * (size_t)c->lev[j].ndof * ts;
  int64_t chunk = 0;
  if (c->jc > 0) {
    const int64_t nd = c->lev[c->jc].ndof;
    chunk = std::min<int64_t>(std::min<int64_t>(nd, 65535), (int64_t)(kry / per_col));
    chunk = std::max<int64_t>(chunk, std::min<int64_t>(nd, 256));
  }
  c->batch_chunk = (int)chunk;
  const size_t rbytes = std::max(kry, per_col * (size_t)chunk);
  c->region = (char*)B.take(rbytes);
  {
    Bump R(c->region);
    c->V = (double*)R.take((size_t)(m + 1) * n * sizeof(double));
    c->Z = R.take((size_t)m * n * c->zsize);
  }
  c->hdev = (double*)B.take((size_t)hd_stride(c) * c->R * sizeof(double));
  c->partial = (double*)B.take((size_t)dots_partial_count() * (m + 2) * c->R * sizeof(double));
  c->live = (int32_t*)B.take((size_t)c->R * sizeof(int32_t));
  return B.off + kAlign;
}

void init_levels(bmg_ctx* c) {
  const bmg_params& p = c->p;
  c->lev.assign(p.levels + 1, LevelInfo());
  for (int j = 0; j <= p.levels; ++j) {
    LevelInfo& L = c->lev[j];
    L.N = p.n0 << j;
    L.h = 1.0 / L.N;
    L.n_u = n_u_of(L.N, p.k);
    L.n_p = n_p_of(L.N, p.k);
    L.ndof = L.n_u + L.n_p;
    if (j > 0) {
      HostIdx I(L.N, p.k, c->bcm);
      for (int col = 0; col < 9; ++col) {
        L.npatch[col] = col < colour_count(p.colouring) ? npatch_of(p.colouring, L.N, col) : 0;
        int ne = 0;
        for (int q = 0; q < L.npatch[col]; ++q) {
          int vx, vy;
          patch_vertex(p.colouring, L.N, col, q, vx, vy);
          // only vertices next to an open side can need the extended layout
          const bool near = vx == 1 || vx == L.N - 1 || vy == 1 || vy == L.N - 1;
          const bool e = near && needs_ext(I, vx, vy);
          if (e != ext_rule(I, vx, vy) || colour_of(p.colouring, vx, vy) != col) c->layout_mismatch = true;
          if (e) ++ne;
          if (mr_handle(c) && !(vx >= 2 && vx <= L.N - 2 && vy >= 2 && vy <= L.N - 2)) L.hblist[col].push_back(q);
        }
        L.next[col] = ne;
      }
      // the colour classes enumerate every vertex exactly once
      int total = 0;
      for (int col = 0; col < 9; ++col) total += L.npatch[col];
      if (total != (L.N + 1) * (L.N + 1)) c->layout_mismatch = true;
    }
  }
}

int bc_mask(const bmg_params& p) {
  int m = 0;
  for (int s = 0; s < 4; ++s)
    if (p.bc[s] == BMG_BC_DIRICHLET) m |= 1 << s;
  return m;
}

void setup_types(bmg_ctx* c) {
  c->K = c->p.k;
  c->prec = c->p.precond_prec == BMG_P_FP64 ? 0 : 1;
  // inverses stored in the preconditioner arithmetic, or bfloat16 with FP32 arithmetic
  c->sprec = c->p.precond_prec == BMG_P_BF16 ? 2 : c->prec;
  c->tsize = c->prec == 0 ? 8 : 4;
  c->ssize = c->sprec == 0 ? 8 : c->sprec == 1 ? 4 : 2;
  c->bcm = bc_mask(c->p);
  c->R = std::max(1, c->p.n_rhs);
  c->il = 0;
  if (mr_handle(c)) {
    c->il = 4;
    while (c->il < c->R) c->il *= 2;
  }
}

template <typename T, int K>
void fill_elem(const RefData& R, Elem<T, K>& E) {
  using D = Dims<K>;
  for (int i = 0; i < D::NV * D::NV; ++i) {
    E.Kmu[i] = (T)R.Kmu[i];
    E.M[i] = (T)R.M[i];
    for (int f = 0; f < 4; ++f) E.F[f][i] = (T)R.F[f][i];
    for (int f = 0; f < 2; ++f) E.Nb[f][i] = (T)R.Nb[f][i];
  }
  for (int i = 0; i < D::NP * D::NV; ++i) {
    E.Dx[i] = (T)R.Dx[i];
    E.Dy[i] = (T)R.Dy[i];
  }
}

template <typename T, int K>
void fill_xfer(const RefData& R, Xfer<T, K>& X) {
  using D = Dims<K>;
  for (int s = 0; s < 2; ++s) {
    for (int i = 0; i < D::NA * D::NA; ++i) X.Ppsi[s][i] = (T)R.Ppsi[s][i];
    for (int i = 0; i < D::NB * D::NB; ++i) X.PL[s][i] = (T)R.PL[s][i];
  }
}

template <typename T, int K>
bmg_status upload_consts(bmg_ctx* c, void* dst, bool elem, bool as_double) {
  (void)as_double;
  if (elem) {
    Elem<T, K> E;
    fill_elem<T, K>(c->ref, E);
    HIPCHK(c, hipMemcpy(dst, &E, sizeof(E), hipMemcpyHostToDevice));
  } else {
    Xfer<T, K> X;
    fill_xfer<T, K>(c->ref, X);
    HIPCHK(c, hipMemcpy(dst, &X, sizeof(X), hipMemcpyHostToDevice));
  }
  return BMG_OK;
}

template <int K>
bmg_status upload_elem_int(bmg_ctx* c) {
  using D = Dims<K>;
  constexpr int NV = D::NV, NP = D::NP;
  const RefData& R = c->ref;
  ElemInt<float, K> E;
  std::memset(&E, 0, sizeof(E));
  for (int d = 0; d < NV; ++d)
    for (int e = 0; e < NV; ++e) {
      const int i = d * NV + e;
      E.Kint[d][e] = (float)(R.Kmu[i] + R.F[0][i] + R.F[3][i]);
      E.M[d][e] = (float)R.M[i];
      E.F1[d][e] = (float)R.F[1][i];
      E.F2[d][e] = (float)R.F[2][i];
    }
  for (int q = 0; q < NP; ++q)
    for (int d = 0; d < NV; ++d) {
      E.DxT[d][q] = (float)R.Dx[q * NV + d];
      E.DyT[d][q] = (float)R.Dy[q * NV + d];
      E.Dx[q][d] = (float)R.Dx[q * NV + d];
      E.Dy[q][d] = (float)R.Dy[q * NV + d];
    }
  HIPCHK(c, hipMemcpy(c->elemInt, &E, sizeof(E), hipMemcpyHostToDevice));
  return BMG_OK;
}

bmg_status upload_all_consts(bmg_ctx* c) {
  if (c->elemInt) {
    const bmg_status se = c->K == 1 ? upload_elem_int<1>(c) : upload_elem_int<2>(c);
    if (se) return se;
  }
  bmg_status s;
  if (c->K == 0) {
    s = c->prec == 0 ? upload_consts<double, 0>(c, c->elemT, true, false) : upload_consts<float, 0>(c, c->elemT, true, false);
    if (s) return s;
    s = upload_consts<double, 0>(c, c->elem64, true, true);
    if (s) return s;
    s = c->prec == 0 ? upload_consts<double, 0>(c, c->xferT, false, false) : upload_consts<float, 0>(c, c->xferT, false, false);
  } else if (c->K == 1) {
    s = c->prec == 0 ? upload_consts<double, 1>(c, c->elemT, true, false) : upload_consts<float, 1>(c, c->elemT, true, false);
    if (s) return s;
    s = upload_consts<double, 1>(c, c->elem64, true, true);
    if (s) return s;
    s = c->prec == 0 ? upload_consts<double, 1>(c, c->xferT, false, false) : upload_consts<float, 1>(c, c->xferT, false, false);
  } else {
    s = c->prec == 0 ? upload_consts<double, 2>(c, c->elemT, true, false) : upload_consts<float, 2>(c, c->elemT, true, false);
    if (s) return s;
    s = upload_consts<double, 2>(c, c->elem64, true, true);
    if (s) return s;
    s = c->prec == 0 ? upload_consts<double, 2>(c, c->xferT, false, false) : upload_consts<float, 2>(c, c->xferT, false, false);
  }
  return s;
}

// FP64 -> bfloat16 with round-to-nearest-even (through FP32)
uint16_t to_bf16(double d) {
  const float f = (float)d;
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);  // inf / nan kept
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (uint16_t)(u >> 16);
}

// upload a host FP64 array converted to `prec` (0 double, 1 float, 2 bfloat16)
bmg_status upload_converted(bmg_ctx* c, void* dst, const double* src, size_t n, int prec) {
  if (prec == 0) {
    HIPCHK(c, hipMemcpy(dst, src, n * sizeof(double), hipMemcpyHostToDevice));
  } else if (prec == 2) {
    std::vector<uint16_t> tmp(n);
    for (size_t i = 0; i < n; ++i) tmp[i] = to_bf16(src[i]);
    HIPCHK(c, hipMemcpy(dst, tmp.data(), n * sizeof(uint16_t), hipMemcpyHostToDevice));
  } else {
    std::vector<float> tmp(n);
    for (size_t i = 0; i < n; ++i) tmp[i] = (float)src[i];
    HIPCHK(c, hipMemcpy(dst, tmp.data(), n * sizeof(float), hipMemcpyHostToDevice));
  }
  return BMG_OK;
}

// Dense A_j of a (small) level from the cell and face blocks; rows and columns
// of the essential normal dofs are the identity.
std::vector<double> dense_level(const RefData& R, int k, int bcm, int N, const std::vector<double>& kappa) {
  HostIdx I(N, k, bcm);
  const int64_t n = n_u_of(N, k) + n_p_of(N, k);
  std::vector<double> A((size_t)n * n, 0.0);
  const int NV = I.NV, NP = I.NP;
  auto add = [&](int cx, int cy, int d, int cx2, int cy2, int e, double v) {
    if (I.cons(cx, cy, d) || I.cons(cx2, cy2, e)) return;
    A[(size_t)I.g(cx, cy, d) * n + I.g(cx2, cy2, e)] += v;
  };
  const double h = 1.0 / N, hh = h * h;
  for (int cy = 0; cy < N; ++cy)
    for (int cx = 0; cx < N; ++cx) {
      const double khh = kappa[(size_t)cy * N + cx] * hh;
      for (int comp = 0; comp < 2; ++comp) {
        const int o = comp * NV;
        const std::vector<double>& Dm = comp == 0 ? R.Dx : R.Dy;
        for (int d = 0; d < NV; ++d) {
          for (int e = 0; e < NV; ++e) add(cx, cy, o + d, cx, cy, o + e, R.Kmu[d * NV + e] + khh * R.M[d * NV + e]);
          for (int q = 0; q < NP; ++q) {
            add(cx, cy, o + d, cx, cy, 2 * NV + q, -h * Dm[q * NV + d]);
            add(cx, cy, 2 * NV + q, cx, cy, o + d, -h * Dm[q * NV + d]);
          }
        }
        for (int up = 0; up < 2; ++up) {
          int ncx = cx, ncy = cy, side;
          if (comp == 0) {
            ncy += up ? 1 : -1;
            side = up ? 3 : 2;
          } else {
            ncx += up ? 1 : -1;
            side = up ? 1 : 0;
          }
          if (!I.in(ncx, ncy)) {
            if ((bcm >> side) & 1)
              for (int d = 0; d < NV; ++d)
                for (int e = 0; e < NV; ++e) add(cx, cy, o + d, cx, cy, o + e, R.Nb[up][d * NV + e]);
            continue;
          }
          const std::vector<double>& Fs = R.F[up ? 0 : 3];
          const std::vector<double>& Fn = R.F[up ? 1 : 2];
          for (int d = 0; d < NV; ++d)
            for (int e = 0; e < NV; ++e) {
              add(cx, cy, o + d, cx, cy, o + e, Fs[d * NV + e]);
              add(cx, cy, o + d, ncx, ncy, o + e, Fn[d * NV + e]);
            }
        }
      }
    }
  for (int cy = 0; cy < N; ++cy)
    for (int cx = 0; cx < N; ++cx)
      for (int d = 0; d < I.NL; ++d)
        if (I.cons(cx, cy, d)) {
          const int64_t gi = I.g(cx, cy, d);
          A[(size_t)gi * n + gi] = 1.0;
        }
  return A;
}

// (Pseudo-)inverse of A_0, stored column-major on the device.  With every side
// Dirichlet the constant pressure spans the kernel: bordered inverse.
bmg_status build_coarse(bmg_ctx* c) {
  const LevelInfo& L = c->lev[0];
  HostIdx I(L.N, c->K, c->bcm);
  const int64_t n = L.ndof;
  std::vector<double> A = dense_level(c->ref, c->K, c->bcm, L.N, L.kappa);
  const bool sing = (c->bcm == 15);
  const int64_t m = sing ? n + 1 : n;
  std::vector<double> a((size_t)m * m, 0.0), inv;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) a[(size_t)i * m + j] = A[(size_t)i * n + j];
  if (sing) {
    const double cv = 1.0 / L.N;
    for (int64_t cc = 0; cc < (int64_t)L.N * L.N; ++cc) {
      const int64_t gi = I.pres(cc, 0);
      a[(size_t)gi * m + n] = cv;
      a[(size_t)n * m + gi] = cv;
    }
  }
  if (!gauss_jordan((int)m, a, inv)) return fail(c, BMG_E_SINGULAR, "coarse matrix is singular");
  std::vector<double> cm((size_t)n * n);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) cm[(size_t)j * n + i] = inv[(size_t)i * m + j];
  HIPCHK(c, hipMemcpy(c->coarse_inv, cm.data(), cm.size() * sizeof(double), hipMemcpyHostToDevice));
  return BMG_OK;
}

// Arguments of the level kernels for level j (kappa in FP64 or the preconditioner's arithmetic).
LevelArgs largs(bmg_ctx* c, int j, bool fp64) {
  LevelArgs a;
  a.N = c->lev[j].N;
  a.bcm = c->bcm;
  a.h = c->lev[j].h;
  a.kap = fp64 ? (const void*)c->lev[j].kap64 : c->lev[j].kap;
  a.colouring = c->p.colouring;
  a.cpb = c->p.columns_per_block;
  return a;
}

// Patch pseudo-inverses of level j, colour by colour, uploaded column-major.
bmg_status build_patches(bmg_ctx* c, int j) {
  LevelInfo& L = c->lev[j];
  HostIdx I(L.N, c->K, c->bcm);
  const int nsr = nsr_of(c->K), nse = nse_of(c->K);
  for (int col = 0; col < 9; ++col) {
    const int np = L.npatch[col];
    if (np == 0) continue;
    const int scheme = c->p.colouring;
    std::vector<int32_t> ext(np, -1);
    int ne = 0;
    for (int p = 0; p < np; ++p) {
      int vx, vy;
      patch_vertex(scheme, L.N, col, p, vx, vy);
      const bool near = vx == 1 || vx == L.N - 1 || vy == 1 || vy == L.N - 1;
      if (near && needs_ext(I, vx, vy)) ext[p] = ne++;
    }
    const bool pk = packed_level(c, L.N);
    HIPCHK(c, hipMemcpy(L.extidx[col], ext.data(), np * sizeof(int32_t), hipMemcpyHostToDevice));
    if (!c->p.setup_on_host) {
      // FP64 Gauss-Jordan on the device, one block per patch (zero pivots flagged in c->live[0])
      launch_patch_pinv(c->K, c->sprec, c->elem64, largs(c, j, true), col, np, pk, L.inv[col], L.invx[col],
                        L.extidx[col], c->live, c->stream);
      HIPCHK(c, hipGetLastError());
      continue;
    }
    const int64_t er = inv_entries(pk, nsr), ee = inv_entries(pk, nse);
    std::vector<double> reg((size_t)np * er, 0.0), exd((size_t)std::max(ne, 1) * ee, 0.0);
    std::atomic<int> bad{0};
    parallel_for(np, [&](int p) {
      int vx, vy;
      patch_vertex(scheme, L.N, col, p, vx, vy);
      const bool isx = ext[p] >= 0;
      PatchLayout P = build_layout(I, vx, vy, isx);
      std::vector<double> A, pinv;
      patch_matrix(I, c->ref, L, vx, vy, P, A);
      if (!patch_pinv(I, P, A, pinv, nullptr)) {
        bad.store(1);
        return;
      }
      double* dst = isx ? &exd[(size_t)ext[p] * ee] : &reg[(size_t)p * er];
      const int ns = P.ns;
      if (pk) {
        // rotated diagonals of the symmetrised (A+ + A+^T)/2
        for (int d = 0; d <= ns / 2; ++d)
          for (int t = 0; t < ns; ++t) {
            const int u = (t + d) % ns;
            dst[(size_t)d * ns + t] = 0.5 * (pinv[(size_t)t * ns + u] + pinv[(size_t)u * ns + t]);
          }
      } else {
        for (int t = 0; t < ns; ++t)
          for (int u = 0; u < ns; ++u) dst[(size_t)u * ns + t] = pinv[(size_t)t * ns + u];
      }
    });
    if (bad.load()) return fail(c, BMG_E_SINGULAR, "a patch matrix is singular");
    bmg_status s = upload_converted(c, L.inv[col], reg.data(), reg.size(), c->sprec);
    if (s) return s;
    if (ne > 0) {
      s = upload_converted(c, L.invx[col], exd.data(), (size_t)ne * ee, c->sprec);
      if (s) return s;
    }
  }
  return BMG_OK;
}

// Template table of level j for the several-column kernel (see launch_colour_mr): the
// regular patch of the interior vertex (2, 2).
bmg_status upload_mr_table(bmg_ctx* c, int j) {
  LevelInfo& L = c->lev[j];
  if (!L.mrtab) return BMG_OK;
  const int K = c->K, N = L.N;
  HostIdx I(N, K, c->bcm);
  const int NV = I.NV, NL = I.NL, nsr = nsr_of(K);
  int cw, xs, cs;
  mr_layout(K, &cw, &xs, &cs);
  (void)cs;
  const PatchLayout P = build_layout(I, 2, 2, false);
  const int ne = 4 * NL + 8 * NV + nsr;
  std::vector<int32_t> tab((size_t)mr_table_entries(K) * 4, 0);
  const int64_t nux = (int64_t)N * (N + 1) * I.NB, nu = n_u_of(N, K);
  auto stream = [&](int64_t g) { return g < nux ? 0 : g < 2 * nux ? 1 : g < nu ? 2 : 3; };
  for (int e = 0; e < ne; ++e) {
    int64_t g;
    int pos, fb = 0;
    if (e < 4 * NL) {
      const int sl = e / NL, d = e % NL;
      g = I.g(1 + (sl & 1), 1 + (sl >> 1), d);
      pos = sl * cw + d;
    } else if (e < 4 * NL + 8 * NV) {
      const int e2 = e - 4 * NL, sl = e2 / (2 * NV), r = e2 % (2 * NV), which = r / NV, d = r % NV;
      const int cx = 1 + (sl & 1), cy = 1 + (sl >> 1);
      const int ncx = which == 0 ? cx : ((sl & 1) ? cx + 1 : cx - 1);
      const int ncy = which == 0 ? ((sl < 2) ? cy - 1 : cy + 1) : cy;
      g = I.g(ncx, ncy, which * NV + d);
      pos = 4 * cw + e2;
    } else {
      const int t = e - 4 * NL - 8 * NV;
      g = P.g[t];
      pos = xs + t;
      fb = 1;
      if (g < 0) return fail(c, BMG_E_STATE, "interior template patch has an empty slot");
      int pa = -1, pb = -1;
      for (int sl = 0; sl < 4; ++sl)
        for (int d = 0; d < NL; ++d)
          if (P.lane[sl * NL + d] == t) {
            if (pa < 0) pa = sl * cw + d;
            else pb = sl * cw + d;
          }
      tab[(size_t)(ne + t) * 4 + 0] = pa;
      tab[(size_t)(ne + t) * 4 + 1] = pb;
    }
    tab[(size_t)e * 4 + 0] = (int32_t)g;
    tab[(size_t)e * 4 + 1] = stream(g);
    tab[(size_t)e * 4 + 2] = pos;
    tab[(size_t)e * 4 + 3] = fb;
  }
  HIPCHK(c, hipMemcpy(L.mrtab, tab.data(), tab.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  return BMG_OK;
}

// Outcome of the device builds of the patch pseudo-inverses (all levels).
bmg_status check_patch_status(bmg_ctx* c) {
  if (c->p.setup_on_host) return BMG_OK;
  int32_t flag = 0;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(&flag, c->live, sizeof(flag), hipMemcpyDeviceToHost));
  if (flag) return fail(c, BMG_E_SINGULAR, "a patch matrix is singular");
  return BMG_OK;
}

// --------------------------------------------------------------------------
// Cycle
// --------------------------------------------------------------------------

// Bytes one colour step of level j (nrhs columns) must move: every patch's stored
// pseudo-inverse (once per block of columns a launch serves), and per column the
// gathered x of its cells and of the tangential components across its outer faces,
// kappa of its cells, b on the patch and the read-modify-write of x on the patch.
double colour_bytes(const bmg_ctx* c, int j, int col, int nrhs) {
  const LevelInfo& L = c->lev[j];
  const int K = c->K, NB = K + 1, NI = 2 * K * NB, NP = NB * NB, NV = (K + 2) * NB;
  const int nsr = nsr_of(K), nse = nse_of(K);
  const double gather = 12.0 * NB + 4.0 * NI + 4.0 * NP + 8.0 * NV + 4.0;
  const double reg = L.npatch[col] - L.next[col], ext = L.next[col];
  const bool pk = packed_level(c, L.N);
  // passes over the inverses: one for the several-column kernel, otherwise one per
  // block of columns
  double inv_bytes = (reg * (double)inv_entries(pk, nsr) + ext * (double)inv_entries(pk, nse)) * c->ssize;
  if (mr_level(c, L.N, nrhs)) {
    // the listed boundary patches read their inverse once per column
    const double nb = (double)L.hblist[col].size(), np = std::max(1, L.npatch[col]);
    inv_bytes *= 1.0 + (nrhs - 1) * nb / np;
  } else {
    const int ncol = colour_columns_per_block(L.N, pk, L.npatch[col], nrhs, c->p.columns_per_block);
    inv_bytes *= (double)((nrhs + ncol - 1) / ncol);
  }
  // x on the patch is written once (its old values come with the gather)
  return inv_bytes + nrhs * (reg * (gather + 2.0 * nsr) + ext * (gather + 2.0 * nse)) * c->tsize;
}

constexpr int kFusedColourMaxN = 256;

// One colour step of level j on nrhs columns of x, b (ld = level ndof apart, or with
// il > 0 interleaved records of il values): the several-column kernel on the interior
// patches plus the general kernel on the listed others, or the general kernel on
// every patch of the colour.  omega > 0: additive share.
void colour_launch(bmg_ctx* c, int j, int col, void* x, const void* b, int nrhs, double omega, int il) {
  LevelInfo& L = c->lev[j];
  const LevelArgs a = largs(c, j, c->prec == 0);
  const bool finest = j == (int)c->lev.size() - 1, pk = packed_level(c, L.N);
  if (il > 0) {
    // interleaved records: the several-column handle's own vectors (multiplicative).
    // Levels up to kFusedColourMaxN cells per side, where a launch is a few dozen to a few
    // thousand blocks and its latency dominates, do interior and listed patches in one
    // launch; larger ones in two (the several-column kernel keeps its own, smaller LDS
    // and four blocks per CU there)
    if (L.mrtab && L.N <= kFusedColourMaxN) {
      launch_colour_fused(c->K, c->elemInt, c->elemT, a, x, b, L.inv[col], L.invx[col], L.extidx[col], L.mrtab, col,
                          L.npatch[col], (int)L.hblist[col].size(), L.blist[col], nrhs, il, c->stream);
      return;
    }
    if (L.mrtab) launch_colour_mr(c->K, c->elemInt, a, x, b, L.inv[col], L.mrtab, col, L.npatch[col], il, c->stream);
    launch_colour(c->K, c->prec, c->sprec, c->elemT, a, x, b, L.inv[col], L.invx[col], L.extidx[col], col,
                  (int)L.hblist[col].size(), finest, pk, nrhs, L.ndof, 0.0, c->stream, L.blist[col], il);
    return;
  }
  launch_colour(c->K, c->prec, c->sprec, c->elemT, a, x, b, L.inv[col], L.invx[col], L.extidx[col], col,
                L.npatch[col], finest, pk, nrhs, L.ndof, omega, c->stream);
}

// `steps` smoothing steps on level j (nrhs columns; r: scratch of the same shape).
// Multiplicative: colours 0..C-1 then C-2..0, each one launch.  Additive: the
// residual of x once, then every colour adds its damped patch corrections computed
// from that residual (colour by colour, so that the updates of a launch are disjoint).
void smooth_level(bmg_ctx* c, int j, int steps, void* x, const void* b, void* r, int nrhs, int il) {
  LevelInfo& L = c->lev[j];
  LevelArgs a = largs(c, j, c->prec == 0);
  const bool timed = (c->timing_level == j);
  const bool additive = c->p.smoother == BMG_SMOOTHER_ADDITIVE;
  const int C = colour_count(c->p.colouring);
  const int nl = additive ? C : 2 * C - 1;
  for (int st = 0; st < steps; ++st) {
    if (additive) launch_op(c->K, c->prec, c->elemT, a, x, b, r, true, nrhs, L.ndof, c->stream, il);
    // one event pair around the back-to-back colour launches of a smoothing step, so
    // that no marker sits between two colour kernels
    const bool rec = timed && c->ev_used + 2 <= c->ev.size();
    if (rec) (void)hipEventRecord(c->ev[c->ev_used], c->stream);
    for (int i = 0; i < nl; ++i) {
      const int col = i < C ? i : 2 * C - 2 - i;
      if (additive) colour_launch(c, j, col, x, r, nrhs, c->p.omega, il);
      else colour_launch(c, j, col, x, b, nrhs, 0.0, il);
      if (rec) c->timed_bytes += colour_bytes(c, j, col, nrhs);
    }
    if (rec) {
      (void)hipEventRecord(c->ev[c->ev_used + 1], c->stream);
      c->ev_used += 2;
      c->timed_launches += nl;
    }
  }
}

int smoothing_steps(const bmg_ctx* c, int j) {
  if (c->p.cycle == BMG_CYCLE_VARIABLE) return c->p.m_fine << (c->p.levels - j);
  return c->p.m_fine;
}

// Vectors of every level the cycle works on (nrhs vectors each, ld = level ndof).
struct Vecs {
  std::vector<void*> x, b, r;
  int nrhs = 1;
  int il = 0;  // > 0: interleaved records of il values (the handle's own level vectors)
};

Vecs level_vecs(bmg_ctx* c) {
  Vecs v;
  v.nrhs = c->R;
  v.il = c->il;
  for (auto& L : c->lev) {
    v.x.push_back(L.x);
    v.b.push_back(L.b);
    v.r.push_back(L.r);
  }
  return v;
}

// B_j applied to v.b[j], result in v.x[j] (Section 3.2).  With use_dense the
// sub-cycle of level jc is one product with its precomputed matrix.
void vcycle_level(bmg_ctx* c, int j, const Vecs& v, bool use_dense) {
  LevelInfo& L = c->lev[j];
  const int nr = v.nrhs;
  if (use_dense && c->jc > 0 && j == c->jc) {
    launch_dense_gemv(c->prec, c->dense, L.ndof, v.b[j], v.x[j], nr, c->stream, v.il);
    return;
  }
  if (j == 0) {
    launch_coarse(c->prec, (int)L.ndof, c->coarse_inv, v.b[0], v.x[0], nr, c->stream, v.il);
    return;
  }
  const int m = smoothing_steps(c, j);
  launch_fill_zero(c->prec, v.x[j], L.ndof * (v.il > 0 ? v.il : nr), c->stream);
  smooth_level(c, j, m, v.x[j], v.b[j], v.r[j], nr, v.il);
  LevelArgs a = largs(c, j, c->prec == 0);
  launch_op(c->K, c->prec, c->elemT, a, v.x[j], v.b[j], v.r[j], true, nr, L.ndof, c->stream, v.il);
  LevelInfo& C = c->lev[j - 1];
  launch_restrict(c->K, c->prec, c->xferT, C.N, c->bcm, v.r[j], v.b[j - 1], nr, L.ndof, C.ndof, c->stream, v.il);
  vcycle_level(c, j - 1, v, use_dense);
  launch_prolong(c->K, c->prec, c->xferT, C.N, c->bcm, v.x[j - 1], v.x[j], nr, C.ndof, L.ndof, c->stream, v.il);
  smooth_level(c, j, m, v.x[j], v.b[j], v.r[j], nr, v.il);
}

// Dense B_jc: the V-cycle of level jc applied to the unit vectors, a chunk of
// columns at a time (column-major storage).
bmg_status build_dense(bmg_ctx* c) {
  if (c->jc == 0) return BMG_OK;
  const int64_t nd = c->lev[c->jc].ndof;
  Vecs v;
  Bump R(c->region);
  for (int j = 0; j <= c->jc; ++j) {
    const size_t bytes = (size_t)c->lev[j].ndof * c->batch_chunk * c->tsize;
    v.x.push_back(R.take(bytes));
    v.b.push_back(R.take(bytes));
    v.r.push_back(R.take(bytes));
  }
  for (int64_t col0 = 0; col0 < nd; col0 += c->batch_chunk) {
    v.nrhs = (int)std::min<int64_t>(c->batch_chunk, nd - col0);
    launch_identity(c->prec, v.b[c->jc], nd, col0, v.nrhs, c->stream);
    vcycle_level(c, c->jc, v, false);
    HIPCHK(c, hipMemcpyAsync((char*)c->dense + (size_t)col0 * nd * c->tsize, v.x[c->jc],
                             (size_t)v.nrhs * nd * c->tsize, hipMemcpyDeviceToDevice, c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipGetLastError());
  return BMG_OK;
}

// Capture the finest-level V-cycle (fixed buffers) once; later cycles replay it.
bool capture_vcycle(bmg_ctx* c) {
  if (c->vexec) return true;
  if (c->graph_failed) return false;
  if (!c->cap_stream && hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    c->graph_failed = true;
    return false;
  }
  hipStream_t user = c->stream;
  c->stream = c->cap_stream;
  bool ok = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
  if (ok) {
    vcycle_level(c, (int)c->lev.size() - 1, level_vecs(c), true);
    ok = hipStreamEndCapture(c->cap_stream, &c->vgraph) == hipSuccess;
  }
  c->stream = user;
  if (ok) ok = hipGraphInstantiate(&c->vexec, c->vgraph, nullptr, nullptr, 0) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    if (c->vgraph) (void)hipGraphDestroy(c->vgraph);
    c->vgraph = nullptr;
    c->vexec = nullptr;
    c->graph_failed = true;
  }
  return ok;
}

// FP64 user vectors (R columns of level j, column-major) into a level vector of the
// handle's arithmetic and layout, and back (to_prec 0: FP64, 1: FP32)
void cast_in(bmg_ctx* c, int j, const double* src, void* dst) {
  const int64_t n = c->lev[j].ndof;
  if (c->il > 0) launch_cast_il(1, 0, src, dst, n, n, c->R, c->il, true, c->stream);
  else launch_cast(c->prec, 0, src, dst, n * c->R, c->stream);
}
void cast_out(bmg_ctx* c, int j, const void* src, void* dst, int to_prec) {
  const int64_t n = c->lev[j].ndof;
  if (c->il > 0) launch_cast_il(to_prec, 1, src, dst, n, n, c->R, c->il, false, c->stream);
  else launch_cast(to_prec, c->prec, src, dst, n * c->R, c->stream);
}

// z = B_J r for all R columns (FP64 r on the device; z FP64, or FP32 with
// z_prec = 1, which is exact for the FP32 V-cycle); the essential rows are inverted
// exactly.
void apply_precond(bmg_ctx* c, const double* r, void* z, int z_prec = 0) {
  LevelInfo& L = c->lev.back();
  cast_in(c, (int)c->lev.size() - 1, r, L.b);
  // the captured graph (eager launches while kernel timing is on, or if the graph
  // cannot be built or launched)
  const bool graphed = c->timing_level < 0 && capture_vcycle(c) && hipGraphLaunch(c->vexec, c->stream) == hipSuccess;
  if (!graphed) {
    if (c->timing_level < 0) (void)hipGetLastError();  // a failed graph launch is replaced, not reported
    vcycle_level(c, (int)c->lev.size() - 1, level_vecs(c), true);
  }
  cast_out(c, (int)c->lev.size() - 1, L.x, z, z_prec);
  launch_copy_constrained(c->K, L.N, c->bcm, r, z, z_prec, c->R, L.ndof, c->stream);
}

void apply_op64(bmg_ctx* c, int j, const double* x, double* y) {
  launch_op(c->K, 0, c->elem64, largs(c, j, true), x, nullptr, y, false, c->R, c->lev[j].ndof, c->stream);
}

// y = b - A_J x in FP64 (one fused launch)
void residual64(bmg_ctx* c, const double* b, const double* x, double* y) {
  const int J = (int)c->lev.size() - 1;
  launch_op(c->K, 0, c->elem64, largs(c, J, true), x, b, y, true, c->R, c->lev[J].ndof, c->stream);
}

// y = A_J z for a vector of Z (FP64 or FP32-stored)
void apply_op64_z(bmg_ctx* c, const void* z, double* y) {
  const int J = (int)c->lev.size() - 1;
  if (c->zsize == sizeof(double)) apply_op64(c, J, (const double*)z, y);
  else launch_op64_f32x(c->K, c->elem64, largs(c, J, true), (const float*)z, y, c->R, c->lev[J].ndof, c->stream);
}

// kappa of level j from the finest field, each coarse cell from its 4 children:
// arithmetic mean (Section 4.1), harmonic mean (0 if a child is 0) or geometric mean
double mean4(int mode, double a, double b, double c, double d) {
  if (mode == BMG_KAPPA_HARMONIC) {
    if (a == 0.0 || b == 0.0 || c == 0.0 || d == 0.0) return 0.0;
    return 4.0 / (1.0 / a + 1.0 / b + 1.0 / c + 1.0 / d);
  }
  if (mode == BMG_KAPPA_GEOMETRIC) return std::sqrt(std::sqrt(a * b) * std::sqrt(c * d));
  return 0.25 * (a + b + c + d);
}

std::vector<double> kappa_level(const double* fine, int n0, int J, int j, int mode) {
  int N = n0 << J;
  std::vector<double> cur(fine, fine + (size_t)N * N);
  for (int l = J; l > j; --l) {
    const int Nc = N / 2;
    std::vector<double> nx((size_t)Nc * Nc);
    for (int cy = 0; cy < Nc; ++cy)
      for (int cx = 0; cx < Nc; ++cx) {
        const size_t f = (size_t)(2 * cy) * N + 2 * cx;
        nx[(size_t)cy * Nc + cx] = mean4(mode, cur[f], cur[f + 1], cur[f + N], cur[f + N + 1]);
      }
    cur.swap(nx);
    N = Nc;
  }
  return cur;
}

bmg_status check_kappa(const bmg_params* p, const double* kappa) {
  if (!kappa) return BMG_E_ARG;
  const int N = p->n0 << p->levels;
  // kappa >= 0 with viscosity (kappa = 0: the Stokes end of the Brinkman family),
  // kappa > 0 for Darcy
  const bool stokes_ok = p->mu > 0.0;
  for (int64_t i = 0; i < (int64_t)N * N; ++i) {
    if (!std::isfinite(kappa[i])) return BMG_E_NONFINITE;
    if (stokes_ok ? !(kappa[i] >= 0.0) : !(kappa[i] > 0.0)) return BMG_E_ARG;
  }
  return BMG_OK;
}

bmg_status check_finite_host(const double* v, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return BMG_E_NONFINITE;
  return BMG_OK;
}

bmg_status setup_into(bmg_ctx* c, const bmg_params* p, const double* kappa, void* workspace, size_t bytes,
                      void* stream, bmg_handle* out);

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* bmg_status_string(bmg_status s) {
  switch (s) {
    case BMG_OK: return "ok";
    case BMG_E_ARG: return "invalid argument";
    case BMG_E_UNSUPPORTED: return "unsupported";
    case BMG_E_NOMEM: return "out of memory";
    case BMG_E_HIP: return "HIP error";
    case BMG_E_SINGULAR: return "singular matrix";
    case BMG_E_NOT_CONVERGED: return "not converged";
    case BMG_E_NONFINITE: return "non-finite value";
    case BMG_E_STATE: return "invalid state";
  }
  return "unknown";
}

const char* bmg_last_error(bmg_handle h) { return h ? h->err.c_str() : g_setup_err.c_str(); }

bmg_status bmg_plan(const bmg_params* p, size_t* bytes) try {
  bmg_status s = check_params(p);
  if (s) return s;
  if (!bytes) return BMG_E_ARG;
  bmg_ctx tmp;
  tmp.p = *p;
  setup_types(&tmp);
  init_levels(&tmp);
  if (tmp.layout_mismatch) return BMG_E_STATE;
  *bytes = layout(&tmp, nullptr);
  return BMG_OK;
} catch (const std::bad_alloc&) {
  return BMG_E_NOMEM;
} catch (...) {
  return BMG_E_STATE;
}

bmg_status bmg_setup(const bmg_params* p, const double* kappa, void* workspace, size_t bytes, void* stream,
                     bmg_handle* out) try {
  bmg_status s = check_params(p);
  if (s) return s;
  if (!out) return BMG_E_ARG;
  if ((s = check_kappa(p, kappa))) return s;
  bmg_ctx* c = new bmg_ctx();
  // a host allocation that fails inside setup frees what the handle holds
  try {
    return setup_into(c, p, kappa, workspace, bytes, stream, out);
  } catch (const std::bad_alloc&) {
    g_setup_err = "host memory exhausted during setup";
    if (c->own_ws) (void)hipFree(c->ws);
    delete c;
    return BMG_E_NOMEM;
  }
} catch (const std::bad_alloc&) {
  return BMG_E_NOMEM;
} catch (...) {
  return BMG_E_STATE;
}

}  // extern "C"

namespace {
// The body of bmg_setup after argument validation; c is freed here on every
// failure it reports.
bmg_status setup_into(bmg_ctx* c, const bmg_params* p, const double* kappa, void* workspace, size_t bytes,
                      void* stream, bmg_handle* out) {
  c->p = *p;
  c->stream = (hipStream_t)stream;
  setup_types(c);
  init_levels(c);
  const size_t need = layout(c, nullptr);
  if (workspace) {
    if (bytes < need || ((uintptr_t)workspace % kAlign) != 0) {
      g_setup_err = "workspace smaller than bmg_plan's size or not 256-byte aligned";
      delete c;
      return BMG_E_NOMEM;
    }
    c->ws = (char*)workspace;
  } else {
    if (hipMalloc((void**)&c->ws, need) != hipSuccess) {
      g_setup_err = "hipMalloc of the " + std::to_string(need >> 20) + " MiB workspace failed";
      delete c;
      return BMG_E_NOMEM;
    }
    c->own_ws = true;
  }
  c->ws_bytes = need;
  if (c->layout_mismatch) {
    if (c->own_ws) (void)hipFree(c->ws);
    delete c;
    return BMG_E_STATE;
  }
  layout(c, c->ws);
  c->ref = make_refdata(p->k, p->mu, p->sigma);
  // kappa hierarchy: arithmetic mean of the four children (Section 4.1)
  for (int j = 0; j <= p->levels; ++j) c->lev[j].kappa = kappa_level(kappa, p->n0, p->levels, j, p->coarse_kappa);
  bmg_status st = upload_all_consts(c);
  if (!st) {
    const int32_t zero = 0;  // status word of the device patch builds
    if (hipMemcpy(c->live, &zero, sizeof(zero), hipMemcpyHostToDevice) != hipSuccess)
      st = fail(c, BMG_E_HIP, "hipMemcpy of the setup status failed");
  }
  for (size_t j = 0; !st && j < c->lev.size(); ++j) {
    LevelInfo& L = c->lev[j];
    st = upload_converted(c, L.kap, L.kappa.data(), L.kappa.size(), c->prec);
    if (!st) st = upload_converted(c, L.kap64, L.kappa.data(), L.kappa.size(), 0);
    if (!st && j > 0) st = build_patches(c, (int)j);
    for (int col = 0; !st && j > 0 && col < 9; ++col)
      if (L.blist[col] && !L.hblist[col].empty() &&
          hipMemcpy(L.blist[col], L.hblist[col].data(), L.hblist[col].size() * sizeof(int32_t),
                    hipMemcpyHostToDevice) != hipSuccess)
        st = fail(c, BMG_E_HIP, "hipMemcpy of a boundary patch list failed");
    if (!st && j > 0) st = upload_mr_table(c, (int)j);
  }
  if (!st) st = check_patch_status(c);
  if (!st) st = build_coarse(c);
  if (!st) st = build_dense(c);
  if (!st && hipDeviceSynchronize() != hipSuccess) st = fail(c, BMG_E_HIP, "setup synchronisation failed");
  if (st) {
    g_setup_err = c->err;
    if (c->own_ws) (void)hipFree(c->ws);
    delete c;
    return st;
  }
  *out = c;
  return BMG_OK;
}
}  // namespace

extern "C" {

bmg_status bmg_kernel_timing(bmg_handle h, int32_t level, int32_t max_launches) try {
  if (!h || level < -1 || level >= (int)h->lev.size() || level == 0 || max_launches < 0 || max_launches > 1 << 20)
    return BMG_E_ARG;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  for (auto e : h->ev) (void)hipEventDestroy(e);
  h->ev.clear();
  h->ev_used = 0;
  h->timed_launches = 0;
  h->timed_bytes = 0.0;
  h->timing_level = level;
  if (level < 0) return BMG_OK;
  h->ev.resize((size_t)2 * ((max_launches + 14) / 15));
  for (auto& e : h->ev) HIPCHK(h, hipEventCreate(&e));
  return BMG_OK;
} catch (const std::bad_alloc&) {
  return BMG_E_NOMEM;
} catch (...) {
  return BMG_E_STATE;
}

bmg_status bmg_kernel_timing_read(bmg_handle h, int32_t* launches, double* total_ms, double* bytes) try {
  if (!h || !launches || !total_ms || !bytes) return BMG_E_ARG;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  double ms = 0.0;
  for (size_t i = 0; i + 1 < h->ev_used; i += 2) {
    float t = 0.0f;
    HIPCHK(h, hipEventElapsedTime(&t, h->ev[i], h->ev[i + 1]));
    ms += t;
  }
  *launches = (int32_t)h->timed_launches;
  *total_ms = ms;
  *bytes = h->timed_bytes;
  return BMG_OK;
} catch (const std::bad_alloc&) {
  return BMG_E_NOMEM;
} catch (...) {
  return BMG_E_STATE;
}

bmg_status bmg_destroy(bmg_handle h) try {
  if (!h) return BMG_E_ARG;
  (void)hipStreamSynchronize(h->stream);
  for (auto e : h->ev) (void)hipEventDestroy(e);
  if (h->vexec) (void)hipGraphExecDestroy(h->vexec);
  if (h->vgraph) (void)hipGraphDestroy(h->vgraph);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  if (h->own_ws) {
    (void)hipStreamSynchronize(h->stream);
    (void)hipFree(h->ws);
  }
  delete h;
  return BMG_OK;
} catch (const std::bad_alloc&) {
  return BMG_E_NOMEM;
} catch (...) {
  return BMG_E_STATE;
}

bmg_status bmg_sizes(bmg_handle h, int32_t level, int32_t* N, int64_t* n_u, int64_t* n_p) try {
  if (!h || level < 0 || level >= (int)h->lev.size()) return BMG_E_ARG;
  if (N) *N = h->lev[level].N;
  if (n_u) *n_u = h->lev[level].n_u;
  if (n_p) *n_p = h->lev[level].n_p;
  return BMG_OK;
} catch (const std::bad_alloc&) {
  return BMG_E_NOMEM;
} catch (...) {
  return BMG_E_STATE;
}

bmg_status bmg_apply(bmg_handle h, int32_t level, const double* x, double* y) try {
  if (!h || !x || !y || level < 0 || level >= (int)h->lev.size()) return BMG_E_ARG;
  apply_op64(h, level, x, y);
  HIPCHK(h, hipGetLastError());
  return BMG_OK;
} catch (const std::bad_alloc&) {
  return BMG_E_NOMEM;
} catch (...) {
  return BMG_E_STATE;
}

bmg_status bmg_vcycle_noalloc(bmg_handle h, const double* r, double* z) try {
  if (!h || !r || !z) return BMG_E_ARG;
  void* base = nullptr;
  size_t cap = 0;
  HIPCHK(h, static_scratch(&base, &cap));
  // the level vectors x_j, b_j, r_j of every level (n_rhs columns, preconditioner
  // arithmetic) in the static scratch instead of the handle's workspace
  Vecs v;
  v.nrhs = h->R;
  v.il = h->il;
  Bump B((char*)base);
  for (const LevelInfo& L : h->lev) {
    const size_t bytes = (size_t)L.ndof * (h->il > 0 ? h->il : h->R) * h->tsize;
    v.x.push_back(B.take(bytes));
    v.b.push_back(B.take(bytes));
    v.r.push_back(B.take(bytes));
  }
  if (B.off > cap)
    return fail(h, BMG_E_NOMEM, "bmg_vcycle_noalloc: the level vectors need " + std::to_string(B.off >> 20) +
                                    " MiB, the static scratch holds " + std::to_string(cap >> 20) + " MiB");
  const int J = (int)h->lev.size() - 1;
  // eager launches on the handle's stream (no graph: its nodes hold the workspace's
  // vectors); every level vector is written before it is read
  cast_in(h, J, r, v.b[J]);
  vcycle_level(h, J, v, true);
  cast_out(h, J, v.x[J], z, 0);
  launch_copy_constrained(h->K, h->lev[J].N, h->bcm, r, z, 0, h->R, h->lev[J].ndof, h->stream);
  HIPCHK(h, hipGetLastError());
  return BMG_OK;
} catch (const std::bad_alloc&) {
  return BMG_E_NOMEM;
} catch (...) {
  return BMG_E_STATE;
}

bmg_status bmg_vcycle(bmg_handle h, const double* r, double* z) try {
  if (!h || !r || !z) return BMG_E_ARG;
  apply_precond(h, r, z);
  HIPCHK(h, hipGetLastError());
  return BMG_OK;
} catch (const std::bad_alloc&) {
  return BMG_E_NOMEM;
} catch (...) {
  return BMG_E_STATE;
}

// Step entry points: FP64 vectors in/out, run in the handle's arithmetic.
bmg_status bmg_colour_step(bmg_handle h, int32_t level, int32_t colour, double* x, const double* b) try {
  if (!h || !x || !b || level < 1 || level >= (int)h->lev.size() || colour < 0 ||
      colour >= colour_count(h->p.colouring))
    return BMG_E_ARG;
  LevelInfo& L = h->lev[level];
  cast_in(h, level, x, L.x);
  cast_in(h, level, b, L.b);
  colour_launch(h, level, colour, L.x, L.b, h->R, 0.0, h->il);
  cast_out(h, level, L.x, x, 0);
  HIPCHK(h, hipGetLastError());
  return BMG_OK;
} catch (const std::bad_alloc&) {
  return BMG_E_NOMEM;
} catch (...) {
  return BMG_E_STATE;
}

bmg_status bmg_smooth(bmg_handle h, int32_t level, int32_t steps, double* x, const double* b) try {
  if (!h || !x || !b || level < 1 || level >= (int)h->lev.size() || steps < 0) return BMG_E_ARG;
  LevelInfo& L = h->lev[level];
  cast_in(h, level, x, L.x);
  cast_in(h, level, b, L.b);
  smooth_level(h, level, steps, L.x, L.b, L.r, h->R, h->il);
  cast_out(h, level, L.x, x, 0);
  HIPCHK(h, hipGetLastError());
  return BMG_OK;
} catch (const std::bad_alloc&) {
  return BMG_E_NOMEM;
} catch (...) {
  return BMG_E_STATE;
}

bmg_status bmg_restrict(bmg_handle h, int32_t level, const double* rf, double* bc) try {
  if (!h || !rf || !bc || level < 1 || level >= (int)h->lev.size()) return BMG_E_ARG;
  LevelInfo& F = h->lev[level];
  LevelInfo& C = h->lev[level - 1];
  cast_in(h, level, rf, F.r);
  launch_restrict(h->K, h->prec, h->xferT, C.N, h->bcm, F.r, C.b, h->R, F.ndof, C.ndof, h->stream, h->il);
  cast_out(h, level - 1, C.b, bc, 0);
  HIPCHK(h, hipGetLastError());
  return BMG_OK;
} catch (const std::bad_alloc&) {
  return BMG_E_NOMEM;
} catch (...) {
  return BMG_E_STATE;
}

bmg_status bmg_prolong_add(bmg_handle h, int32_t level, const double* xc, double* xf) try {
  if (!h || !xc || !xf || level < 1 || level >= (int)h->lev.size()) return BMG_E_ARG;
  LevelInfo& F = h->lev[level];
  LevelInfo& C = h->lev[level - 1];
  cast_in(h, level - 1, xc, C.x);
  cast_in(h, level, xf, F.x);
  launch_prolong(h->K, h->prec, h->xferT, C.N, h->bcm, C.x, F.x, h->R, C.ndof, F.ndof, h->stream, h->il);
  cast_out(h, level, F.x, xf, 0);
  HIPCHK(h, hipGetLastError());
  return BMG_OK;
} catch (const std::bad_alloc&) {
  return BMG_E_NOMEM;
} catch (...) {
  return BMG_E_STATE;
}

bmg_status bmg_coarse_solve(bmg_handle h, const double* b, double* x) try {
  if (!h || !b || !x) return BMG_E_ARG;
  LevelInfo& L = h->lev[0];
  cast_in(h, 0, b, L.b);
  launch_coarse(h->prec, (int)L.ndof, h->coarse_inv, L.b, L.x, h->R, h->stream, h->il);
  cast_out(h, 0, L.x, x, 0);
  HIPCHK(h, hipGetLastError());
  return BMG_OK;
} catch (const std::bad_alloc&) {
  return BMG_E_NOMEM;
} catch (...) {
  return BMG_E_STATE;
}

bmg_status bmg_solve(bmg_handle h, const double* b, double* x, double rtol, int32_t maxit, const double* x0,
                     bmg_solve_info* info) try {
  if (!h || !b || !x || !(rtol > 0.0) || maxit < 1) return BMG_E_ARG;
  const int J = (int)h->lev.size() - 1;
  const int R = h->R;
  const int64_t n = h->lev[J].ndof;  // entries of one column
  const int64_t ldv = n * R;         // distance between Krylov vectors
  const int m = h->p.restart;
  const int64_t HS = hd_stride(h), NS = 2 * (m + 2);
  hipStream_t s = h->stream;
  double* hd = h->hdev;  // per column (HS apart): [0, m+2) first Gram-Schmidt pass, [m+2, NS) second, NS: norm^2
  std::vector<double> hh((size_t)HS * R), up((size_t)HS * R, 0.0);
  auto readback = [&]() -> bmg_status {
    HIPCHK(h, hipMemcpyAsync(hh.data(), hd, hh.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    return BMG_OK;
  };
  auto upload = [&]() -> bmg_status {
    HIPCHK(h, hipMemcpyAsync(hd, up.data(), up.size() * sizeof(double), hipMemcpyHostToDevice, s));
    return BMG_OK;
  };
  // which columns the scaling kernels keep (device copy changed only when it changes)
  std::vector<int32_t> live_dev(R, -1);
  auto set_live = [&](const std::vector<int32_t>& l) -> bmg_status {
    if (l == live_dev) return BMG_OK;
    live_dev = l;
    HIPCHK(h, hipMemcpyAsync(h->live, live_dev.data(), R * sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIPCHK(h, hipStreamSynchronize(s));  // live_dev may change before the next synchronisation
    return BMG_OK;
  };
  bmg_status st;
  // ||b_r||
  launch_dots(b, 1, ldv, b, n, h->partial, hd + NS, R, HS, s);
  if ((st = readback())) return st;
  struct Col {
    double bnorm = 0.0, est = 1.0, prev_beta = -1.0;
    int its = 0;
    bool open = true, conv = false, stalled = false;
  };
  std::vector<Col> col(R);
  for (int r = 0; r < R; ++r) {
    col[r].bnorm = std::sqrt(hh[(size_t)r * HS + NS]);
    if (!std::isfinite(col[r].bnorm)) return fail(h, BMG_E_NONFINITE, "right-hand side is not finite");
  }
  if (x0) HIPCHK(h, hipMemcpyAsync(x, x0, ldv * sizeof(double), hipMemcpyDeviceToDevice, s));
  else HIPCHK(h, hipMemsetAsync(x, 0, ldv * sizeof(double), s));
  for (int r = 0; r < R; ++r)
    if (col[r].bnorm == 0.0) {  // b_r = 0: x_r = 0
      HIPCHK(h, hipMemsetAsync(x + (size_t)r * n, 0, n * sizeof(double), s));
      col[r].open = false;
      col[r].conv = true;
      col[r].est = 0.0;
    }
  // per column: Hessenberg matrix (Givens-reduced), rotations, rhs of the LSQ problem
  std::vector<double> H((size_t)(m + 1) * m * R), cs((size_t)m * R), sn((size_t)m * R), g((size_t)(m + 1) * R),
      y(m);
  // Each restart cycle starts from the true residual, so convergence is confirmed on
  // ||b - A x|| itself (iterative refinement when the Arnoldi estimate has drifted
  // from it); a cycle that reduces the true residual by less than 10% ends the
  // column's solve.
  const int zprec = h->zsize == sizeof(double) ? 0 : 1;
  auto zvec = [&](int i) { return (char*)h->Z + (size_t)i * ldv * h->zsize; };
  for (;;) {
    bool any_open = false;
    for (auto& c : col) any_open |= c.open;
    if (!any_open) break;
    // r = b - A x in V_0, ||r||
    residual64(h, b, x, h->V);
    launch_dots(h->V, 1, ldv, h->V, n, h->partial, hd + NS, R, HS, s);
    if ((st = readback())) return st;
    std::vector<int32_t> act(R, 0);
    bool any = false;
    for (int r = 0; r < R; ++r) {
      Col& c = col[r];
      if (!c.open) continue;
      const double beta = std::sqrt(hh[(size_t)r * HS + NS]);
      if (!std::isfinite(beta)) return fail(h, BMG_E_NONFINITE, "residual is not finite");
      c.est = beta / c.bnorm;
      if (beta <= rtol * c.bnorm) {
        c.conv = true;
        c.open = false;
      } else if (c.prev_beta >= 0.0 && beta > 0.9 * c.prev_beta) {
        c.stalled = true;
        c.open = false;
      } else if (c.its >= maxit) {
        c.open = false;
      } else {
        c.prev_beta = beta;
        act[r] = 1;
        any = true;
        up[(size_t)r * HS + NS] = beta;
        double* Hr = &H[(size_t)r * (m + 1) * m];
        std::fill(Hr, Hr + (size_t)(m + 1) * m, 0.0);
        std::fill(&g[(size_t)r * (m + 1)], &g[(size_t)r * (m + 1)] + (m + 1), 0.0);
        g[(size_t)r * (m + 1)] = beta;
      }
    }
    if (!any) break;
    // V_0 = r / beta on the running columns, 0 on the others (in place)
    if ((st = upload())) return st;
    if ((st = set_live(act))) return st;
    launch_scale(h->V, h->V, hd + NS, HS, h->live, false, n, R, s);
    std::vector<int32_t> run = act;
    std::vector<int> icount(R, 0);
    for (int i = 0; i < m; ++i) {
      double* vi = h->V + (size_t)i * ldv;
      void* zi = zvec(i);
      // w = A z_i is formed in V_{i+1} and orthogonalised there
      double* w = h->V + (size_t)(i + 1) * ldv;
      apply_precond(h, vi, zi, zprec);
      apply_op64_z(h, zi, w);
      // classical Gram-Schmidt, two passes
      launch_dots(h->V, i + 1, ldv, w, n, h->partial, hd, R, HS, s);
      launch_axpys(w, h->V, i + 1, ldv, hd, HS, -1.0, n, R, s);
      launch_dots(h->V, i + 1, ldv, w, n, h->partial, hd + (m + 2), R, HS, s);
      launch_axpys(w, h->V, i + 1, ldv, hd + (m + 2), HS, -1.0, n, R, s);
      launch_dots(w, 1, ldv, w, n, h->partial, hd + NS, R, HS, s);
      if ((st = readback())) return st;
      bool still = false;
      for (int r = 0; r < R; ++r) {
        if (!run[r]) continue;
        Col& c = col[r];
        const double* hr = &hh[(size_t)r * HS];
        double* Hr = &H[(size_t)r * (m + 1) * m];
        double* csr = &cs[(size_t)r * m];
        double* snr = &sn[(size_t)r * m];
        double* gr = &g[(size_t)r * (m + 1)];
        const double hn = std::sqrt(hr[NS]);
        for (int k2 = 0; k2 <= i; ++k2) Hr[(size_t)k2 * m + i] = hr[k2] + hr[(m + 2) + k2];
        Hr[(size_t)(i + 1) * m + i] = hn;
        for (int k2 = 0; k2 < i; ++k2) {
          const double a = Hr[(size_t)k2 * m + i], cc = Hr[(size_t)(k2 + 1) * m + i];
          Hr[(size_t)k2 * m + i] = csr[k2] * a + snr[k2] * cc;
          Hr[(size_t)(k2 + 1) * m + i] = -snr[k2] * a + csr[k2] * cc;
        }
        const double a = Hr[(size_t)i * m + i], cc = Hr[(size_t)(i + 1) * m + i];
        const double den = std::hypot(a, cc);
        if (!std::isfinite(den) || den == 0.0) return fail(h, BMG_E_NONFINITE, "Arnoldi breakdown");
        csr[i] = a / den;
        snr[i] = cc / den;
        Hr[(size_t)i * m + i] = den;
        Hr[(size_t)(i + 1) * m + i] = 0.0;
        gr[i + 1] = -snr[i] * gr[i];
        gr[i] = csr[i] * gr[i];
        ++c.its;
        icount[r] = i + 1;
        c.est = std::fabs(gr[i + 1]) / c.bnorm;
        // a column that reaches rtol is confirmed on the true residual by the next cycle
        if (std::fabs(gr[i + 1]) <= rtol * c.bnorm || hn == 0.0 || c.its >= maxit) run[r] = 0;
        else still = true;
      }
      if (!still || i + 1 == m) break;
      if ((st = set_live(run))) return st;
      launch_scale(w, w, hd + NS, HS, h->live, true, n, R, s);
    }
    // x_r += Z_r y_r with y_r from the triangular system of column r
    int imax = 0;
    std::fill(up.begin(), up.end(), 0.0);
    for (int r = 0; r < R; ++r) {
      const int ic = icount[r];
      imax = std::max(imax, ic);
      const double* Hr = &H[(size_t)r * (m + 1) * m];
      const double* gr = &g[(size_t)r * (m + 1)];
      for (int q = ic - 1; q >= 0; --q) {
        double sum = gr[q];
        for (int cc = q + 1; cc < ic; ++cc) sum -= Hr[(size_t)q * m + cc] * y[cc];
        y[q] = sum / Hr[(size_t)q * m + q];
      }
      for (int q = 0; q < ic; ++q) up[(size_t)r * HS + q] = y[q];
    }
    if ((st = upload())) return st;
    if (zprec == 0) launch_axpys(x, (const double*)h->Z, imax, ldv, hd, HS, 1.0, n, R, s);
    else launch_axpys_f32(x, (const float*)h->Z, imax, ldv, hd, HS, 1.0, n, R, s);
    HIPCHK(h, hipStreamSynchronize(s));  // hd and up are reused by the next cycle
  }
  // true residuals (in V_0, whose basis vector is no longer needed)
  residual64(h, b, x, h->V);
  launch_dots(h->V, 1, ldv, h->V, n, h->partial, hd + NS, R, HS, s);
  if ((st = readback())) return st;
  HIPCHK(h, hipGetLastError());
  bool all = true, stalled = false;
  for (int r = 0; r < R; ++r) {
    const Col& c = col[r];
    all &= c.conv;
    stalled |= c.stalled;
    if (info) {
      info[r].iterations = c.its;
      info[r].converged = c.conv;
      info[r].rel_residual_estimate = c.est;
      info[r].rel_residual_true = c.bnorm > 0.0 ? std::sqrt(hh[(size_t)r * HS + NS]) / c.bnorm : 0.0;
    }
  }
  return all ? BMG_OK
             : fail(h, BMG_E_NOT_CONVERGED,
                    stalled ? "true residual stagnates above rtol (attainable accuracy reached)" : "maxit reached");
} catch (const std::bad_alloc&) {
  return BMG_E_NOMEM;
} catch (...) {
  return BMG_E_STATE;
}

bmg_status bmg_quad_points(const bmg_params* p, double* cell_xy, double* face_xy) try {
  bmg_status st = check_params(p);
  if (st) return st;
  if (!cell_xy || !face_xy) return BMG_E_ARG;
  const int q = p->k + 2, N = p->n0 << p->levels;
  double x[4], w[4];
  gauss_points(q, x, w);
  const double hc = 1.0 / N;
  for (int cy = 0; cy < N; ++cy)
    for (int cx = 0; cx < N; ++cx)
      for (int iy = 0; iy < q; ++iy)
        for (int ix = 0; ix < q; ++ix) {
          const size_t o = ((((size_t)cy * N + cx) * q + iy) * q + ix) * 2;
          cell_xy[o] = (cx + x[ix]) * hc;
          cell_xy[o + 1] = (cy + x[iy]) * hc;
        }
  for (int sd = 0; sd < 4; ++sd)
    for (int f = 0; f < N; ++f)
      for (int i = 0; i < q; ++i) {
        const size_t o = (((size_t)sd * N + f) * q + i) * 2;
        const double t = (f + x[i]) * hc;
        if (sd < 2) {
          face_xy[o] = sd == 0 ? 0.0 : 1.0;
          face_xy[o + 1] = t;
        } else {
          face_xy[o] = t;
          face_xy[o + 1] = sd == 2 ? 0.0 : 1.0;
        }
      }
  return BMG_OK;
} catch (const std::bad_alloc&) {
  return BMG_E_NOMEM;
} catch (...) {
  return BMG_E_STATE;
}

bmg_status bmg_assemble_rhs(const bmg_params* p, const double* f_qp, const double* s_qp, const double* g_qp,
                            double* b) try {
  bmg_status st = check_params(p);
  if (st) return st;
  if (!f_qp || !b) return BMG_E_ARG;
  bmg_ctx tmp;
  bmg_ctx* h = &tmp;
  h->p = *p;
  setup_types(h);
  const RefData R = make_refdata(p->k, p->mu, p->sigma);
  const int N = p->n0 << p->levels;
  HostIdx I(N, h->K, h->bcm);
  const int q = h->K + 2, NB = I.NB, NA = I.NA;
  const double mu = p->mu, sigma = p->sigma;
  const double Lh = 1.0 / N;
  const int64_t ndof = n_u_of(N, p->k) + n_p_of(N, p->k);
  double x[4], w[4];
  gauss_points(q, x, w);
  const size_t ncell = (size_t)N * N * q * q;
  if (check_finite_host(f_qp, 2 * ncell)) return BMG_E_NONFINITE;
  if (s_qp && check_finite_host(s_qp, ncell)) return BMG_E_NONFINITE;
  if (g_qp) {
    if (check_finite_host(g_qp, (size_t)4 * N * q * 2)) return BMG_E_NONFINITE;
    for (int sd = 0; sd < 4; ++sd) {
      if (!((h->bcm >> sd) & 1)) continue;
      for (int i = 0; i < N * q; ++i)
        if (g_qp[((size_t)sd * N * q + i) * 2 + (sd < 2 ? 0 : 1)] != 0.0)
          return BMG_E_UNSUPPORTED;
    }
  }
  // 1-D tables at the points
  std::vector<double> Lq(NB * q), Pq(NA * q);
  for (int b2 = 0; b2 < NB; ++b2)
    for (int i = 0; i < q; ++i) Lq[b2 * q + i] = R.L[b2](x[i]);
  for (int a = 0; a < NA; ++a)
    for (int i = 0; i < q; ++i) Pq[a * q + i] = R.P[a](x[i]);
  std::vector<double> out(ndof, 0.0);
  const double hh = Lh * Lh;
  for (int cy = 0; cy < N; ++cy)
    for (int cx = 0; cx < N; ++cx)
      for (int iy = 0; iy < q; ++iy)
        for (int ix = 0; ix < q; ++ix) {
          const size_t pt = (((size_t)cy * N + cx) * q + iy) * q + ix;
          const double wt = w[ix] * w[iy] * hh;
          const double fx = f_qp[2 * pt], fy = f_qp[2 * pt + 1];
          for (int a = 0; a < NA; ++a)
            for (int b2 = 0; b2 < NB; ++b2) {
              const int d = a * NB + b2;
              out[I.g(cx, cy, d)] += wt * fx * Pq[a * q + ix] * Lq[b2 * q + iy];
              out[I.g(cx, cy, I.NV + d)] += wt * fy * Lq[b2 * q + ix] * Pq[a * q + iy];
            }
          if (s_qp)
            for (int pb = 0; pb < NB; ++pb)
              for (int pa = 0; pa < NB; ++pa)
                out[I.pres((int64_t)cy * N + cx, pb * NB + pa)] -= wt * s_qp[pt] * Lq[pa * q + ix] * Lq[pb * q + iy];
        }
  if (g_qp && mu > 0.0) {
    // tangential Nitsche terms on Dirichlet sides: the tangential component's
    // Legendre index runs across the face (value and normal derivative at 0 or 1)
    for (int sd = 0; sd < 4; ++sd) {
      if (!((h->bcm >> sd) & 1)) continue;
      const bool at1 = (sd == 1 || sd == 3);
      for (int f = 0; f < N; ++f) {
        const int cx = sd == 0 ? 0 : sd == 1 ? N - 1 : f;
        const int cy = sd == 2 ? 0 : sd == 3 ? N - 1 : f;
        const int comp = sd < 2 ? 1 : 0;  // tangential component
        for (int b2 = 0; b2 < NB; ++b2) {
          const double Lv = R.L[b2](at1 ? 1.0 : 0.0);
          const double dLv = R.L[b2].deriv()(at1 ? 1.0 : 0.0);
          const double fac = 2.0 * mu * sigma * Lv + (at1 ? -mu * dLv : mu * dLv);
          for (int a = 0; a < NA; ++a) {
            double s = 0.0;
            for (int i = 0; i < q; ++i) s += w[i] * g_qp[(((size_t)sd * N + f) * q + i) * 2 + comp] * Pq[a * q + i];
            out[I.g(cx, cy, comp * I.NV + a * NB + b2)] += fac * s;
          }
        }
      }
    }
  }
  // essential rows: zero normal data
  for (int cy = 0; cy < N; ++cy)
    for (int cx = 0; cx < N; ++cx)
      for (int d = 0; d < 2 * I.NV; ++d)
        if (I.cons(cx, cy, d)) out[I.g(cx, cy, d)] = 0.0;
  std::copy(out.begin(), out.end(), b);
  return BMG_OK;
} catch (const std::bad_alloc&) {
  return BMG_E_NOMEM;
} catch (...) {
  return BMG_E_STATE;
}

bmg_status bmg_export_patch(const bmg_params* p, const double* kappa, int32_t level, int32_t vx, int32_t vy,
                            int32_t* n, int32_t* dofs, double* inv, int32_t* colour) try {
  bmg_status st = check_params(p);
  if (st) return st;
  if ((st = check_kappa(p, kappa))) return st;
  if (!n || !dofs || level < 1 || level > p->levels) return BMG_E_ARG;
  const int N = p->n0 << level;
  if (vx < 0 || vy < 0 || vx > N || vy > N) return BMG_E_ARG;
  HostIdx I(N, p->k, bc_mask(*p));
  const bool near = vx == 1 || vx == N - 1 || vy == 1 || vy == N - 1;
  PatchLayout P = build_layout(I, vx, vy, near && needs_ext(I, vx, vy));
  std::vector<int> idx;
  for (int t = 0; t < P.ns; ++t)
    if (P.g[t] >= 0) idx.push_back(t);
  *n = (int32_t)idx.size();
  for (size_t i = 0; i < idx.size(); ++i) dofs[i] = (int32_t)P.g[idx[i]];
  if (colour) *colour = colour_of(p->colouring, vx, vy);
  if (inv) {
    LevelInfo L;
    L.N = N;
    L.h = 1.0 / N;
    L.kappa = kappa_level(kappa, p->n0, p->levels, level, p->coarse_kappa);
    const RefData R = make_refdata(p->k, p->mu, p->sigma);
    std::vector<double> A, pinv;
    patch_matrix(I, R, L, vx, vy, P, A);
    if (!patch_pinv(I, P, A, pinv, nullptr)) return BMG_E_SINGULAR;
    const size_t m = idx.size();
    for (size_t i = 0; i < m; ++i)
      for (size_t j = 0; j < m; ++j) inv[i * m + j] = pinv[(size_t)idx[i] * P.ns + idx[j]];
  }
  return BMG_OK;
} catch (const std::bad_alloc&) {
  return BMG_E_NOMEM;
} catch (...) {
  return BMG_E_STATE;
}

bmg_status bmg_export_colouring(const bmg_params* p, int32_t level, int32_t* ncolours, int32_t* colour_host) try {
  bmg_status st = check_params(p);
  if (st) return st;
  if (level < 1 || level > p->levels) return BMG_E_ARG;
  const int N = p->n0 << level;
  if (ncolours) *ncolours = colour_count(p->colouring);
  if (colour_host)
    for (int vy = 0; vy <= N; ++vy)
      for (int vx = 0; vx <= N; ++vx) colour_host[vy * (N + 1) + vx] = colour_of(p->colouring, vx, vy);
  return BMG_OK;
} catch (const std::bad_alloc&) {
  return BMG_E_NOMEM;
} catch (...) {
  return BMG_E_STATE;
}

bmg_status bmg_export_level_matrix(const bmg_params* p, const double* kappa, int32_t level, double* out) try {
  bmg_status st = check_params(p);
  if (st) return st;
  if ((st = check_kappa(p, kappa))) return st;
  if (!out || level < 0 || level > p->levels) return BMG_E_ARG;
  const int N = p->n0 << level;
  if (N > 32) return BMG_E_ARG;
  const RefData R = make_refdata(p->k, p->mu, p->sigma);
  std::vector<double> A = dense_level(R, p->k, bc_mask(*p), N, kappa_level(kappa, p->n0, p->levels, level, p->coarse_kappa));
  std::copy(A.begin(), A.end(), out);
  return BMG_OK;
} catch (const std::bad_alloc&) {
  return BMG_E_NOMEM;
} catch (...) {
  return BMG_E_STATE;
}


// ----- batches of independent problems -----
static void batch_free(bmg_batch* b) {
  for (auto h : b->h)
    if (h) bmg_destroy(h);
  for (auto e : b->done)
    if (e) (void)hipEventDestroy(e);
  if (b->start) (void)hipEventDestroy(b->start);
  for (auto s : b->streams)
    if (s) (void)hipStreamDestroy(s);
  delete b;
}

bmg_status bmg_batch_setup(int32_t nprob, const bmg_params* params, const double* const* kappa_host,
                           int32_t nstreams, void* hip_stream, bmg_batch_handle* out) try {
  if (!out || !params || !kappa_host || nprob < 1 || nprob > 4096 || nstreams < 0 || nstreams > 16)
    return BMG_E_ARG;
  for (int i = 0; i < nprob; ++i) {
    bmg_status s = check_params(&params[i]);
    if (s) return s;
    if (!kappa_host[i]) return BMG_E_ARG;
  }
  bmg_batch* b = new bmg_batch();
  b->user = (hipStream_t)hip_stream;
  const int S = std::min(nstreams == 0 ? 4 : nstreams, nprob);
  b->streams.assign(S, nullptr);
  b->done.assign(S, nullptr);
  for (int w = 0; w < S; ++w) {
    hipError_t e = hipStreamCreateWithFlags(&b->streams[w], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->done[w], hipEventDisableTiming);
    if (e != hipSuccess) {
      g_setup_err = std::string("worker stream: ") + hipGetErrorString(e);
      batch_free(b);
      return BMG_E_HIP;
    }
  }
  if (hipEventCreateWithFlags(&b->start, hipEventDisableTiming) != hipSuccess) {
    g_setup_err = "batch event";
    batch_free(b);
    return BMG_E_HIP;
  }
  b->h.assign(nprob, nullptr);
  for (int i = 0; i < nprob; ++i) {
    bmg_status s = bmg_setup(&params[i], kappa_host[i], nullptr, 0, b->streams[i % S], &b->h[i]);
    if (s) {
      g_setup_err = "problem " + std::to_string(i) + ": " + g_setup_err;
      batch_free(b);
      return s;
    }
  }
  *out = b;
  return BMG_OK;
} catch (const std::bad_alloc&) {
  return BMG_E_NOMEM;
} catch (...) {
  return BMG_E_STATE;
}

bmg_status bmg_batch_handle_of(bmg_batch_handle b, int32_t i, bmg_handle* out) try {
  if (!b || !out || i < 0 || i >= (int)b->h.size()) return BMG_E_ARG;
  *out = b->h[i];
  return BMG_OK;
} catch (const std::bad_alloc&) {
  return BMG_E_NOMEM;
} catch (...) {
  return BMG_E_STATE;
}

bmg_status bmg_batch_solve(bmg_batch_handle b, const double* const* b_dev, double* const* x_dev, double rtol,
                           int32_t maxit, bmg_solve_info* info) try {
  if (!b || !b_dev || !x_dev || !(rtol > 0.0) || maxit < 1) return BMG_E_ARG;
  const int n = (int)b->h.size(), S = (int)b->streams.size();
  std::vector<int64_t> info_off(n + 1, 0);
  for (int i = 0; i < n; ++i) {
    if (!b_dev[i] || !x_dev[i]) return BMG_E_ARG;
    info_off[i + 1] = info_off[i] + b->h[i]->R;
  }
  // the worker streams start after the work already queued on the caller's stream
  if (hipEventRecord(b->start, b->user) != hipSuccess) return BMG_E_HIP;
  for (int w = 0; w < S; ++w)
    if (hipStreamWaitEvent(b->streams[w], b->start, 0) != hipSuccess) return BMG_E_HIP;
  std::vector<bmg_status> st(n, BMG_OK);
  std::atomic<int> next{0};
  auto worker = [&](int w) {
    for (int i = next++; i < n; i = next++) {
      bmg_handle h = b->h[i];
      h->stream = b->streams[w];  // a handle is driven by one worker at a time
      st[i] = bmg_solve(h, b_dev[i], x_dev[i], rtol, maxit, nullptr, info ? info + info_off[i] : nullptr);
    }
  };
  std::vector<std::thread> th;
  for (int w = 1; w < S; ++w) th.emplace_back(worker, w);
  worker(0);
  for (auto& t : th) t.join();
  for (int w = 0; w < S; ++w) {
    if (hipEventRecord(b->done[w], b->streams[w]) != hipSuccess) return BMG_E_HIP;
    if (hipStreamWaitEvent(b->user, b->done[w], 0) != hipSuccess) return BMG_E_HIP;
  }
  // the first hard failure in problem order, else the first NOT_CONVERGED
  int pick = -1;
  for (int i = 0; i < n && pick < 0; ++i)
    if (st[i] != BMG_OK && st[i] != BMG_E_NOT_CONVERGED) pick = i;
  for (int i = 0; i < n && pick < 0; ++i)
    if (st[i] != BMG_OK) pick = i;
  if (pick < 0) return BMG_OK;
  b->err = "problem " + std::to_string(pick) + ": " + b->h[pick]->err;
  return st[pick];
} catch (const std::bad_alloc&) {
  return BMG_E_NOMEM;
} catch (...) {
  return BMG_E_STATE;
}

const char* bmg_batch_last_error(bmg_batch_handle b) { return b ? b->err.c_str() : "null batch"; }

bmg_status bmg_batch_destroy(bmg_batch_handle b) try {
  if (!b) return BMG_E_ARG;
  for (auto s : b->streams) (void)hipStreamSynchronize(s);
  batch_free(b);
  return BMG_OK;
} catch (const std::bad_alloc&) {
  return BMG_E_NOMEM;
} catch (...) {
  return BMG_E_STATE;
}


// ----- autotuning of the smoother schedule -----
}  // extern "C"

namespace {

// Time `trials` preconditioner applications (graph replay) of a handle set up with q.
bmg_status time_vcycles(const bmg_params* q, const double* kappa_host, void* hip_stream, int32_t trials,
                        double* ms_per) {
  hipStream_t s = (hipStream_t)hip_stream;
  bmg_handle h = nullptr;
  bmg_status st = bmg_setup(q, kappa_host, nullptr, 0, hip_stream, &h);
  if (st) return st;
  LevelInfo& L = h->lev.back();
  const int64_t n = L.ndof * h->R;
  double* r = nullptr;
  double* z = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  float ms = 0.0f;
  bool ok = hipMalloc((void**)&r, n * sizeof(double)) == hipSuccess &&
            hipMalloc((void**)&z, n * sizeof(double)) == hipSuccess && hipEventCreate(&e0) == hipSuccess &&
            hipEventCreate(&e1) == hipSuccess;
  if (ok) {
    // constant 1 as input (the timing does not depend on the values)
    std::vector<double> one(n, 1.0);
    ok = hipMemcpyAsync(r, one.data(), n * sizeof(double), hipMemcpyHostToDevice, s) == hipSuccess;
    apply_precond(h, r, z);  // captures the graph
    ok = ok && hipEventRecord(e0, s) == hipSuccess;
    for (int t = 0; ok && t < trials; ++t) apply_precond(h, r, z);
    ok = ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
         hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (r) (void)hipFree(r);
  if (z) (void)hipFree(z);
  bmg_destroy(h);
  if (!ok) return BMG_E_HIP;
  *ms_per = ms / trials;
  return BMG_OK;
}

// tile choices found so far in this process, by problem shape
std::mutex g_tune_mu;
std::map<std::vector<int64_t>, bmg_params> g_tune_cache;

std::vector<int64_t> tune_key(const bmg_params* p) {
  return {p->k, (int64_t)p->n0 << p->levels, p->levels, p->precond_prec, std::max(1, p->n_rhs), p->smoother,
          p->cycle, p->dense_coarse_max};
}

}  // namespace

extern "C" {

bmg_status bmg_autotune(const bmg_params* p, const double* kappa_host, void* hip_stream, int32_t trials,
                        bmg_params* best, double* ms_per_vcycle) try {
  bmg_status st = check_params(p);
  if (st) return st;
  if (!best || trials < 1 || trials > 1000) return BMG_E_ARG;
  if ((st = check_kappa(p, kappa_host))) return st;
  double best_ms = -1.0;
  for (int cand = 0; cand < 2; ++cand) {
    bmg_params q = *p;
    q.colouring = cand == 0 ? BMG_COLOURING_S9 : BMG_COLOURING_L8;
    double per = 0.0;
    if ((st = time_vcycles(&q, kappa_host, hip_stream, trials, &per))) return st;
    if (ms_per_vcycle) ms_per_vcycle[cand] = per;
    if (best_ms < 0.0 || per < best_ms) {
      best_ms = per;
      *best = q;
    }
  }
  return BMG_OK;
} catch (const std::bad_alloc&) {
  return BMG_E_NOMEM;
} catch (...) {
  return BMG_E_STATE;
}

bmg_status bmg_autotune_tiles(const bmg_params* p, const double* kappa_host, void* hip_stream, int32_t trials,
                              bmg_params* best, double* report, int32_t max_report, int32_t* n_report) try {
  bmg_status st = check_params(p);
  if (st) return st;
  if (!best || trials < 1 || trials > 1000 || max_report < 0 || (max_report > 0 && !report)) return BMG_E_ARG;
  if ((st = check_kappa(p, kappa_host))) return st;
  if (n_report) *n_report = 0;
  const std::vector<int64_t> key = tune_key(p);
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      *best = *p;
      best->colouring = it->second.colouring;
      best->rotated_min_n = it->second.rotated_min_n;
      best->columns_per_block = it->second.columns_per_block;
      return BMG_OK;
    }
  }
  int rows = 0;
  bmg_params cur = *p;
  double cur_ms = -1.0;
  // one coordinate at a time: each candidate differs from the best so far in one parameter
  auto trial = [&](bmg_params q) -> bmg_status {
    double per = 0.0;
    bmg_status s2 = time_vcycles(&q, kappa_host, hip_stream, trials, &per);
    if (s2) return s2;
    if (rows < max_report) {
      report[4 * rows + 0] = q.colouring;
      report[4 * rows + 1] = q.rotated_min_n;
      report[4 * rows + 2] = q.columns_per_block;
      report[4 * rows + 3] = per;
    }
    ++rows;
    if (cur_ms < 0.0 || per < cur_ms) {
      cur_ms = per;
      cur = q;
    }
    return BMG_OK;
  };
  for (int col : {BMG_COLOURING_S9, BMG_COLOURING_L8}) {
    bmg_params q = cur;
    q.colouring = col;
    if ((st = trial(q))) return st;
  }
  {
    const bmg_params base = cur;
    for (int nmin : {64, 4096}) {
      bmg_params q = base;
      q.rotated_min_n = nmin;
      if ((st = trial(q))) return st;
    }
  }
  bmg_ctx probe;
  probe.p = *p;
  setup_types(&probe);
  if (probe.R > 1 && !mr_handle(&probe)) {
    const bmg_params base = cur;
    for (int cpb : {1, 4, 16}) {
      bmg_params q = base;
      q.columns_per_block = cpb;
      if ((st = trial(q))) return st;
    }
  }
  *best = cur;
  if (n_report) *n_report = std::min(rows, max_report);
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune_cache[key] = cur;
  return BMG_OK;
} catch (const std::bad_alloc&) {
  return BMG_E_NOMEM;
} catch (...) {
  return BMG_E_STATE;
}

}  // extern "C"
