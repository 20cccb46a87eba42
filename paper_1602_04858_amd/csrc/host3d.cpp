// Host side of the 3-D (hexahedral) path: reference integrals of RT_k x dQ_k (k = 0, the
// lowest order of Section 2.3, or 1) on the unit cube, assembly of the level operators (CSR) with essential boundary normals,
// vertex patches and their pseudo-inverses, the exact-embedding transfers, and the
// FGMRES / V-cycle loop whose every vector operation runs in HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <new>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "../../include/bmg3.h"
#include "common.hpp"
#include "common3d.hpp"
#include "refelem.hpp"

namespace bmg {
namespace {

// Sizes of RT_K x dQ_K on one hexahedron (K = 0: 6 face dofs + 1 pressure; K = 1: 36 + 8)
template <int K>
struct Dims3 {
  static constexpr int NA = K + 2, NB = K + 1;
  static constexpr int NU = 3 * NA * NB * NB;  // local velocity dofs of a cell
  static constexpr int NP = NB * NB * NB;      // local pressure dofs
  static constexpr int NL = NU + NP;
  static constexpr int NQ = K + 2;             // Gauss points per direction
};
#define BMG_DIMS3(K)                                                                         \
  constexpr int NA3 = Dims3<K>::NA, NB3 = Dims3<K>::NB, NU3 = Dims3<K>::NU, NP3 = Dims3<K>::NP, \
                NL3 = Dims3<K>::NL, NQ1 = Dims3<K>::NQ;                                     \
  (void)NA3, (void)NB3, (void)NU3, (void)NP3, (void)NL3, (void)NQ1

// transverse axes of component d
inline void axes(int d, int& d1, int& d2) {
  d1 = d == 0 ? 1 : 0;
  d2 = d == 2 ? 1 : 2;
}
// local velocity index of (d, a, b, c): (d NA + a) NB^2 + b + NB c; pressure a + NB b + NB^2 c
inline int lu(int NA, int NB, int d, int a, int b, int c) { return (d * NA + a) * NB * NB + b + NB * c; }

struct Num3 {  // global numbering of one level (the layout documented in bmg3.h), degree k
  int N, k, NA3, NB3, NU3, NP3, NL3;
  int bcs[6];  // per side (2 d + 0 at x_d = 0, 2 d + 1 at x_d = 1): BMG_BC_DIRICHLET or BMG_BC_OPEN
  int64_t NF, NI, n_u, n_p, ndof;
  Num3(int n, int deg, const int32_t* bc = nullptr) : N(n), k(deg), NA3(deg + 2), NB3(deg + 1) {
    for (int q = 0; q < 6; ++q) bcs[q] = bc ? bc[q] : BMG_BC_DIRICHLET;
    NU3 = 3 * NA3 * NB3 * NB3;
    NP3 = NB3 * NB3 * NB3;
    NL3 = NU3 + NP3;
    NF = (int64_t)(N + 1) * N * N * NB3 * NB3;
    NI = 3 * k * NB3 * NB3;
    n_u = 3 * NF + NI * N * N * N;
    n_p = (int64_t)NP3 * N * N * N;
    ndof = n_u + n_p;
  }
  int64_t cell(int cx, int cy, int cz) const { return ((int64_t)cz * N + cy) * N + cx; }
  int64_t face(int d, int i, int t1, int t2, int b, int c) const {
    return d * NF + (((int64_t)t2 * N + t1) * (N + 1) + i) * NB3 * NB3 + b + NB3 * c;
  }
  // global index of local dof l of cell (cx, cy, cz)
  int64_t g(const int cc[3], int l) const {
    if (l >= NU3) return n_u + cell(cc[0], cc[1], cc[2]) * NP3 + (l - NU3);
    const int d = l / (NA3 * NB3 * NB3), r = l % (NA3 * NB3 * NB3), a = r / (NB3 * NB3), bc = r % (NB3 * NB3);
    if (a <= 1) {
      int d1, d2;
      axes(d, d1, d2);
      return face(d, cc[d] + a, cc[d1], cc[d2], bc % NB3, bc / NB3);
    }
    return 3 * NF + cell(cc[0], cc[1], cc[2]) * NI + (d * k + a - 2) * NB3 * NB3 + bc;
  }
  // the boundary side of a normal face dof on the boundary, else -1
  int side(int64_t gi) const {
    if (gi >= 3 * NF) return -1;
    const int d = (int)(gi / NF);
    const int64_t i = ((gi % NF) / (NB3 * NB3)) % (N + 1);
    return i == 0 ? 2 * d : i == N ? 2 * d + 1 : -1;
  }
  // essential: a normal face dof on a Dirichlet side
  bool essential(int64_t gi) const {
    const int q = side(gi);
    return q >= 0 && bcs[q] == BMG_BC_DIRICHLET;
  }
  // a free normal face dof on an open side
  bool open_normal(int64_t gi) const {
    const int q = side(gi);
    return q >= 0 && bcs[q] == BMG_BC_OPEN;
  }
  bool all_dirichlet() const {
    for (int q = 0; q < 6; ++q)
      if (bcs[q] != BMG_BC_DIRICHLET) return false;
    return true;
  }
};

// Local basis on the reference cube: values and gradients of the NU velocity
// functions, values of the NP pressure functions.
template <int K>
struct Basis3 {
  static constexpr int NA3 = Dims3<K>::NA, NB3 = Dims3<K>::NB, NU3 = Dims3<K>::NU, NP3 = Dims3<K>::NP;
  Poly L[NB3], dL[NB3], P[NA3], dP[NA3];
  Basis3() {
    for (int b = 0; b < NB3; ++b) {
      L[b] = legendre01(b);
      dL[b] = L[b].deriv();
    }
    for (int a = 0; a < NA3; ++a) {
      P[a] = psi(a);
      dP[a] = P[a].deriv();
    }
  }
  void vel(const double X[3], double val[NU3][3], double grad[NU3][3][3]) const {
    std::memset(val, 0, sizeof(double) * NU3 * 3);
    std::memset(grad, 0, sizeof(double) * NU3 * 9);
    for (int d = 0; d < 3; ++d) {
      int d1, d2;
      axes(d, d1, d2);
      for (int a = 0; a < NA3; ++a)
        for (int c = 0; c < NB3; ++c)
          for (int b = 0; b < NB3; ++b) {
            const int l = lu(NA3, NB3, d, a, b, c);
            const double pa = P[a](X[d]), lb = L[b](X[d1]), lc = L[c](X[d2]);
            val[l][d] = pa * lb * lc;
            grad[l][d][d] = dP[a](X[d]) * lb * lc;
            grad[l][d][d1] = pa * dL[b](X[d1]) * lc;
            grad[l][d][d2] = pa * lb * dL[c](X[d2]);
          }
    }
  }
  void pres(const double X[3], double val[NP3]) const {
    for (int c = 0; c < NB3; ++c)
      for (int b = 0; b < NB3; ++b)
        for (int a = 0; a < NB3; ++a) val[a + NB3 * b + NB3 * NB3 * c] = L[a](X[0]) * L[b](X[1]) * L[c](X[2]);
  }
};

// Reference integrals (unit cube / unit faces); physical blocks are scaled per level.
template <int KD>
struct Ref3 {
  static constexpr int NU3 = Dims3<KD>::NU, NP3 = Dims3<KD>::NP, NQ1 = Dims3<KD>::NQ;
  std::vector<double> K, M, D;           // NU x NU, NU x NU, NP x NU
  std::vector<double> J[3], C[3];        // interior faces: 2NU x 2NU jumps / consistency
  std::vector<double> Jb[3][2], Cb[3][2];  // boundary faces (low, high): NU x NU
  double gx[NQ1], gw[NQ1];
  Basis3<KD> B;
  Ref3() {
    gauss_points(NQ1, gx, gw);
    K.assign(NU3 * NU3, 0.0);
    M.assign(NU3 * NU3, 0.0);
    D.assign(NP3 * NU3, 0.0);
    double val[NU3][3], grad[NU3][3][3];
    double pv[NP3];
    for (int q3 = 0; q3 < NQ1; ++q3)
      for (int q2 = 0; q2 < NQ1; ++q2)
        for (int q1 = 0; q1 < NQ1; ++q1) {
          const double X[3] = {gx[q1], gx[q2], gx[q3]}, w = gw[q1] * gw[q2] * gw[q3];
          B.vel(X, val, grad);
          B.pres(X, pv);
          for (int i = 0; i < NU3; ++i)
            for (int j = 0; j < NU3; ++j) {
              double gg = 0.0, vv = 0.0;
              for (int a = 0; a < 3; ++a) {
                vv += val[i][a] * val[j][a];
                for (int e = 0; e < 3; ++e) gg += grad[i][a][e] * grad[j][a][e];
              }
              K[i * NU3 + j] += w * gg;
              M[i * NU3 + j] += w * vv;
            }
          for (int p = 0; p < NP3; ++p)
            for (int i = 0; i < NU3; ++i)
              D[p * NU3 + i] += w * pv[p] * (grad[i][0][0] + grad[i][1][1] + grad[i][2][2]);
        }
    double v1[NU3][3], g1[NU3][3][3], v2[NU3][3], g2[NU3][3][3];
    for (int d = 0; d < 3; ++d) {
      int d1, d2;
      axes(d, d1, d2);
      J[d].assign(4 * NU3 * NU3, 0.0);
      C[d].assign(4 * NU3 * NU3, 0.0);
      for (int s = 0; s < 2; ++s) {
        Jb[d][s].assign(NU3 * NU3, 0.0);
        Cb[d][s].assign(NU3 * NU3, 0.0);
      }
      for (int q2 = 0; q2 < NQ1; ++q2)
        for (int q1 = 0; q1 < NQ1; ++q1) {
          const double w = gw[q1] * gw[q2];
          double X1[3], X2[3];
          X1[d] = 1.0;
          X2[d] = 0.0;
          X1[d1] = X2[d1] = gx[q1];
          X1[d2] = X2[d2] = gx[q2];
          B.vel(X1, v1, g1);  // T1 (lower cell) at its face xi_d = 1
          B.vel(X2, v2, g2);  // T2 (upper cell) at its face xi_d = 0
          // stacked dofs: 0..NU-1 of T1, NU..2NU-1 of T2; jump = T1 - T2, average of d_d u
          for (int i = 0; i < 2 * NU3; ++i)
            for (int j = 0; j < 2 * NU3; ++j) {
              double jj = 0.0, cc = 0.0;
              for (int a = 0; a < 3; ++a) {
                const double ji = i < NU3 ? v1[i][a] : -v2[i - NU3][a];
                const double jm = j < NU3 ? v1[j][a] : -v2[j - NU3][a];
                const double aj = 0.5 * (j < NU3 ? g1[j][a][d] : g2[j - NU3][a][d]);
                jj += ji * jm;
                cc += aj * ji;  // {d_n u_j} . [v_i]
              }
              J[d][i * 2 * NU3 + j] += w * jj;
              C[d][i * 2 * NU3 + j] += w * cc;
            }
          // boundary faces: low (xi_d = 0, outward -e_d) and high (xi_d = 1, outward +e_d)
          for (int s = 0; s < 2; ++s) {
            const double sg = s ? 1.0 : -1.0;
            auto& v = s ? v1 : v2;
            auto& gr = s ? g1 : g2;
            for (int i = 0; i < NU3; ++i)
              for (int j = 0; j < NU3; ++j) {
                double jj = 0.0, cc = 0.0;
                for (int a = 0; a < 3; ++a) {
                  jj += v[i][a] * v[j][a];
                  cc += sg * gr[j][a][d] * v[i][a];
                }
                Jb[d][s][i * NU3 + j] += w * jj;
                Cb[d][s][i * NU3 + j] += w * cc;
              }
          }
        }
    }
  }
};

template <int K>
const Ref3<K>& ref3() {
  static const Ref3<K> R;
  return R;
}

template <typename F>
void par_for(int64_t n, F&& f) {
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (n < 64) nt = 1;
  std::atomic<int64_t> next{0};
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nt; ++t)
    th.emplace_back([&] {
      for (int64_t i; (i = next.fetch_add(1)) < n;) f(i);
    });
  for (auto& t : th) t.join();
}

// Gauss-Jordan inverse with partial pivoting (row-major n x n); false if singular.
bool gj_inverse(int n, std::vector<double>& a, std::vector<double>& inv) {
  inv.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
  double scale = 0.0;
  for (double v : a) scale = std::max(scale, std::fabs(v));
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(a[(size_t)r * n + c]) > std::fabs(a[(size_t)piv * n + c])) piv = r;
    if (!(std::fabs(a[(size_t)piv * n + c]) > 1e-14 * scale)) return false;
    if (piv != c)
      for (int j = 0; j < n; ++j) {
        std::swap(a[(size_t)c * n + j], a[(size_t)piv * n + j]);
        std::swap(inv[(size_t)c * n + j], inv[(size_t)piv * n + j]);
      }
    const double d = 1.0 / a[(size_t)c * n + c];
    for (int j = 0; j < n; ++j) {
      a[(size_t)c * n + j] *= d;
      inv[(size_t)c * n + j] *= d;
    }
    auto eliminate = [&](int64_t r) {
      if (r == c) return;
      const double f = a[(size_t)r * n + c];
      if (f == 0.0) return;
      for (int j = 0; j < n; ++j) {
        a[(size_t)r * n + j] -= f * a[(size_t)c * n + j];
        inv[(size_t)r * n + j] -= f * inv[(size_t)c * n + j];
      }
    };
    if (n > 1024) par_for(n, eliminate);  // the coarsest-level matrix
    else
      for (int r = 0; r < n; ++r) eliminate(r);
  }
  return true;
}

struct Csr {
  int64_t n = 0, m = 0;
  std::vector<int32_t> rp, ci;
  std::vector<double> v;
};

// rows of (row, col, value) triplets -> CSR with duplicates summed and zeros dropped
struct Trip {
  int32_t r, c;
  double v;
};
Csr to_csr(int64_t n, int64_t m, std::vector<Trip>& t) {
  Csr A;
  A.n = n;
  A.m = m;
  std::vector<int64_t> cnt(n + 1, 0);
  for (const Trip& e : t) ++cnt[e.r + 1];
  for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
  std::vector<std::pair<int32_t, double>> byrow(t.size());
  {
    std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
    for (const Trip& e : t) byrow[pos[e.r]++] = {e.c, e.v};
  }
  std::vector<Trip>().swap(t);
  std::vector<std::vector<std::pair<int32_t, double>>> rows(n);
  par_for(n, [&](int64_t i) {
    auto* b = byrow.data() + cnt[i];
    auto* e = byrow.data() + cnt[i + 1];
    std::sort(b, e, [](const auto& x, const auto& y) { return x.first < y.first; });
    auto& out = rows[i];
    for (auto* p = b; p < e;) {
      const int32_t c = p->first;
      double s = 0.0;
      for (; p < e && p->first == c; ++p) s += p->second;
      if (s != 0.0) out.push_back({c, s});
    }
  });
  A.rp.assign(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) A.rp[i + 1] = A.rp[i] + (int32_t)rows[i].size();
  A.ci.resize(A.rp[n]);
  A.v.resize(A.rp[n]);
  par_for(n, [&](int64_t i) {
    int32_t o = A.rp[i];
    for (auto& pr : rows[i]) {
      A.ci[o] = pr.first;
      A.v[o++] = pr.second;
    }
  });
  return A;
}

Csr transpose(const Csr& A) {
  std::vector<Trip> t;
  t.reserve(A.v.size());
  for (int64_t i = 0; i < A.n; ++i)
    for (int32_t e = A.rp[i]; e < A.rp[i + 1]; ++e) t.push_back({A.ci[e], (int32_t)i, A.v[e]});
  return to_csr(A.m, A.n, t);
}

// Level operator: the full interior-penalty matrix (eq. ipbrinkman, Brinkman-weak),
// then identity rows and columns on the essential dofs.
template <int K>
Csr assemble_level_k(const Num3& S, double mu, double sigma, const std::vector<double>& kap, Csr* full_out) {
  BMG_DIMS3(K);
  const Ref3<K>& R = ref3<K>();
  const int N = S.N;
  const double h = 1.0 / N;
  std::vector<Trip> t;
  t.reserve((size_t)N * N * N * (NL3 * NL3 + 3 * 1400));
  std::vector<int64_t> gl(2 * NU3 + NP3);
  // face blocks in physical scaling: h (2 mu sigma J - mu (C + C^T)); nonzeros only
  auto face_block = [&](const std::vector<double>& Jm, const std::vector<double>& Cm, int n) {
    std::vector<double> F((size_t)n * n);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)
        F[(size_t)i * n + j] = h * (2.0 * mu * sigma * Jm[(size_t)i * n + j] - mu * (Cm[(size_t)i * n + j] +
                                                                                     Cm[(size_t)j * n + i]));
    return F;
  };
  std::vector<double> Fi[3], Fb[3][2];
  for (int d = 0; d < 3; ++d) {
    Fi[d] = face_block(R.J[d], R.C[d], 2 * NU3);
    for (int s = 0; s < 2; ++s) Fb[d][s] = face_block(R.Jb[d][s], R.Cb[d][s], NU3);
  }
  for (int cz = 0; cz < N; ++cz)
    for (int cy = 0; cy < N; ++cy)
      for (int cx = 0; cx < N; ++cx) {
        const int cc[3] = {cx, cy, cz};
        const double kc = kap[S.cell(cx, cy, cz)];
        for (int l = 0; l < NL3; ++l) gl[l] = S.g(cc, l);
        for (int i = 0; i < NU3; ++i)
          for (int j = 0; j < NU3; ++j) {
            const double v = mu * h * R.K[i * NU3 + j] + kc * h * h * h * R.M[i * NU3 + j];
            if (v != 0.0) t.push_back({(int32_t)gl[i], (int32_t)gl[j], v});
          }
        for (int p = 0; p < NP3; ++p)
          for (int i = 0; i < NU3; ++i) {
            const double v = -h * h * R.D[p * NU3 + i];
            if (v == 0.0) continue;
            t.push_back({(int32_t)gl[NU3 + p], (int32_t)gl[i], v});
            t.push_back({(int32_t)gl[i], (int32_t)gl[NU3 + p], v});
          }
        for (int d = 0; d < 3; ++d) {
          if (cc[d] + 1 < N) {
            int up[3] = {cx, cy, cz};
            up[d] += 1;
            std::vector<int64_t> g2(2 * NU3);
            for (int l = 0; l < NU3; ++l) {
              g2[l] = gl[l];
              g2[NU3 + l] = S.g(up, l);
            }
            const auto& F = Fi[d];
            for (int i = 0; i < 2 * NU3; ++i)
              for (int j = 0; j < 2 * NU3; ++j) {
                const double v = F[(size_t)i * 2 * NU3 + j];
                if (v != 0.0) t.push_back({(int32_t)g2[i], (int32_t)g2[j], v});
              }
          }
          for (int s = 0; s < 2; ++s) {
            if ((s == 0 && cc[d] != 0) || (s == 1 && cc[d] != N - 1)) continue;
            if (S.bcs[2 * d + s] != BMG_BC_DIRICHLET) continue;  // open side: no boundary term
            const auto& F = Fb[d][s];
            for (int i = 0; i < NU3; ++i)
              for (int j = 0; j < NU3; ++j) {
                const double v = F[(size_t)i * NU3 + j];
                if (v != 0.0) t.push_back({(int32_t)gl[i], (int32_t)gl[j], v});
              }
          }
        }
      }
  Csr A = to_csr(S.ndof, S.ndof, t);
  if (full_out) *full_out = A;
  // essential rows and columns -> identity
  for (int64_t i = 0; i < A.n; ++i) {
    const bool ei = S.essential(i);
    for (int32_t e = A.rp[i]; e < A.rp[i + 1]; ++e) {
      const bool ej = S.essential(A.ci[e]);
      if (ei || ej) A.v[e] = (ei && A.ci[e] == i) ? 1.0 : 0.0;
    }
    if (ei) {
      bool has = false;
      for (int32_t e = A.rp[i]; e < A.rp[i + 1]; ++e) has |= A.ci[e] == i;
      if (!has) return Csr();  // cannot happen: the boundary blocks hold the diagonal
    }
  }
  std::vector<Trip> t2;
  for (int64_t i = 0; i < A.n; ++i)
    for (int32_t e = A.rp[i]; e < A.rp[i + 1]; ++e)
      if (A.v[e] != 0.0) t2.push_back({(int32_t)i, A.ci[e], A.v[e]});
  return to_csr(A.n, A.n, t2);
}

// Local transfer of the exact embedding: T[o] (NL x NL) = coefficients on the child
// with offset o (ox + 2 oy + 4 oz) of the parent's local functions, by local L2
// projection (velocity and pressure blocks; the rest zero).
template <int K>
std::vector<double> local_transfers() {
  BMG_DIMS3(K);
  const Ref3<K>& R = ref3<K>();
  const Basis3<K>& B = R.B;
  std::vector<double> Mu(NU3 * NU3, 0.0), Mp(NP3 * NP3, 0.0), T(8 * NL3 * NL3, 0.0);
  double vf[NU3][3], gf[NU3][3][3], vc[NU3][3], gc[NU3][3][3];
  double pf[NP3], pc[NP3];
  for (int q3 = 0; q3 < NQ1; ++q3)
    for (int q2 = 0; q2 < NQ1; ++q2)
      for (int q1 = 0; q1 < NQ1; ++q1) {
        const double X[3] = {R.gx[q1], R.gx[q2], R.gx[q3]}, w = R.gw[q1] * R.gw[q2] * R.gw[q3];
        B.vel(X, vf, gf);
        B.pres(X, pf);
        for (int i = 0; i < NU3; ++i)
          for (int j = 0; j < NU3; ++j)
            Mu[i * NU3 + j] += w * (vf[i][0] * vf[j][0] + vf[i][1] * vf[j][1] + vf[i][2] * vf[j][2]);
        for (int i = 0; i < NP3; ++i)
          for (int j = 0; j < NP3; ++j) Mp[i * NP3 + j] += w * pf[i] * pf[j];
      }
  std::vector<double> a, Miu, Mip;
  a = Mu;
  gj_inverse(NU3, a, Miu);
  a = Mp;
  gj_inverse(NP3, a, Mip);
  for (int o = 0; o < 8; ++o) {
    const double off[3] = {(double)(o & 1), (double)((o >> 1) & 1), (double)(o >> 2)};
    std::vector<double> Xu(NU3 * NU3, 0.0), Xp(NP3 * NP3, 0.0);
    for (int q3 = 0; q3 < NQ1; ++q3)
      for (int q2 = 0; q2 < NQ1; ++q2)
        for (int q1 = 0; q1 < NQ1; ++q1) {
          const double X[3] = {R.gx[q1], R.gx[q2], R.gx[q3]}, w = R.gw[q1] * R.gw[q2] * R.gw[q3];
          const double Xc[3] = {0.5 * (off[0] + X[0]), 0.5 * (off[1] + X[1]), 0.5 * (off[2] + X[2])};
          B.vel(X, vf, gf);
          B.vel(Xc, vc, gc);
          B.pres(X, pf);
          B.pres(Xc, pc);
          for (int i = 0; i < NU3; ++i)
            for (int j = 0; j < NU3; ++j)
              Xu[i * NU3 + j] += w * (vf[i][0] * vc[j][0] + vf[i][1] * vc[j][1] + vf[i][2] * vc[j][2]);
          for (int i = 0; i < NP3; ++i)
            for (int j = 0; j < NP3; ++j) Xp[i * NP3 + j] += w * pf[i] * pc[j];
        }
    double* To = &T[(size_t)o * NL3 * NL3];
    for (int i = 0; i < NU3; ++i)
      for (int j = 0; j < NU3; ++j) {
        double s = 0.0;
        for (int l = 0; l < NU3; ++l) s += Miu[i * NU3 + l] * Xu[l * NU3 + j];
        To[i * NL3 + j] = std::fabs(s) > 1e-14 ? s : 0.0;
      }
    for (int i = 0; i < NP3; ++i)
      for (int j = 0; j < NP3; ++j) {
        double s = 0.0;
        for (int l = 0; l < NP3; ++l) s += Mip[i * NP3 + l] * Xp[l * NP3 + j];
        To[(NU3 + i) * NL3 + NU3 + j] = std::fabs(s) > 1e-14 ? s : 0.0;
      }
  }
  return T;
}

// P (fine x coarse): every free fine dof takes its value from the first child cell
// that holds it (the coarse function is continuous in the normal component, so every
// holder gives the same value); essential rows and columns are left out.
template <int K>
Csr prolongation_k(const Num3& C, const Num3& F) {
  BMG_DIMS3(K);
  static const std::vector<double> T = local_transfers<K>();
  std::vector<char> done(F.ndof, 0);
  std::vector<Trip> t;
  for (int cz = 0; cz < C.N; ++cz)
    for (int cy = 0; cy < C.N; ++cy)
      for (int cx = 0; cx < C.N; ++cx) {
        const int cc[3] = {cx, cy, cz};
        int64_t gc[NL3];
        for (int l = 0; l < NL3; ++l) gc[l] = C.g(cc, l);
        for (int o = 0; o < 8; ++o) {
          const int fc[3] = {2 * cx + (o & 1), 2 * cy + ((o >> 1) & 1), 2 * cz + (o >> 2)};
          const double* To = &T[(size_t)o * NL3 * NL3];
          for (int i = 0; i < NL3; ++i) {
            const int64_t gf = F.g(fc, i);
            if (done[gf]) continue;
            done[gf] = 1;
            if (F.essential(gf)) continue;
            for (int j = 0; j < NL3; ++j)
              if (To[i * NL3 + j] != 0.0 && !C.essential(gc[j]))
                t.push_back({(int32_t)gf, (int32_t)gc[j], To[i * NL3 + j]});
          }
        }
      }
  return to_csr(F.ndof, C.ndof, t);
}

// Right-hand side of eq. (BCh) for constant f and g (free rows), with the lifting of
// the essential values, and the essential values on the essential rows.
template <int K>
std::vector<double> rhs3_k(const Num3& S, double mu, double sigma, const std::vector<double>& kap, const double f[3],
                           const double g[3]) {
  BMG_DIMS3(K);
  const Ref3<K>& R = ref3<K>();
  const Basis3<K>& B = R.B;
  const int N = S.N;
  const double h = 1.0 / N;
  // reference integrals of each velocity function against constant vectors
  double Iv[NU3][3] = {}, Ib[3][2][NU3][3] = {};
  double val[NU3][3], grad[NU3][3][3];
  for (int q3 = 0; q3 < NQ1; ++q3)
    for (int q2 = 0; q2 < NQ1; ++q2)
      for (int q1 = 0; q1 < NQ1; ++q1) {
        const double X[3] = {R.gx[q1], R.gx[q2], R.gx[q3]}, w = R.gw[q1] * R.gw[q2] * R.gw[q3];
        B.vel(X, val, grad);
        for (int i = 0; i < NU3; ++i)
          for (int a = 0; a < 3; ++a) Iv[i][a] += w * val[i][a];
      }
  const double pen = 2.0 * mu * sigma / h;
  for (int d = 0; d < 3; ++d) {
    int d1, d2;
    axes(d, d1, d2);
    for (int s = 0; s < 2; ++s)
      for (int q2 = 0; q2 < NQ1; ++q2)
        for (int q1 = 0; q1 < NQ1; ++q1) {
          double X[3];
          X[d] = s ? 1.0 : 0.0;
          X[d1] = R.gx[q1];
          X[d2] = R.gx[q2];
          const double w = R.gw[q1] * R.gw[q2], sg = s ? 1.0 : -1.0;
          B.vel(X, val, grad);
          // per unit g: h^2 (pen v - mu d_n v), d_n v = sg (d v / d xi_d) / h
          for (int i = 0; i < NU3; ++i)
            for (int a = 0; a < 3; ++a) Ib[d][s][i][a] += w * h * h * (pen * val[i][a] - mu * sg * grad[i][a][d] / h);
        }
  }
  std::vector<double> b(S.ndof, 0.0), ge(S.ndof, 0.0);
  for (int cz = 0; cz < N; ++cz)
    for (int cy = 0; cy < N; ++cy)
      for (int cx = 0; cx < N; ++cx) {
        const int cc[3] = {cx, cy, cz};
        for (int i = 0; i < NU3; ++i) {
          const int64_t gi = S.g(cc, i);
          double s = h * h * h * (Iv[i][0] * f[0] + Iv[i][1] * f[1] + Iv[i][2] * f[2]);
          for (int d = 0; d < 3; ++d)
            for (int sd = 0; sd < 2; ++sd)
              if (((sd == 0 && cc[d] == 0) || (sd == 1 && cc[d] == N - 1)) && S.bcs[2 * d + sd] == BMG_BC_DIRICHLET)
                s += Ib[d][sd][i][0] * g[0] + Ib[d][sd][i][1] * g[1] + Ib[d][sd][i][2] * g[2];
          b[gi] += s;
        }
      }
  // essential values: the face projection of g.n onto L_b L_c (orthonormal): only the
  // constant coefficient (b = c = 0) is nonzero for constant g
  for (int d = 0; d < 3; ++d)
    for (int t2 = 0; t2 < N; ++t2)
      for (int t1 = 0; t1 < N; ++t1)
        for (int sd = 0; sd < 2; ++sd)
          if (S.bcs[2 * d + sd] == BMG_BC_DIRICHLET) ge[S.face(d, sd ? N : 0, t1, t2, 0, 0)] = g[d];
  Csr Af;
  assemble_level_k<K>(S, mu, sigma, kap, &Af);
  for (int64_t i = 0; i < S.ndof; ++i) {
    if (S.essential(i)) {
      b[i] = ge[i];
      continue;
    }
    double s = 0.0;
    for (int32_t e = Af.rp[i]; e < Af.rp[i + 1]; ++e) s += Af.v[e] * ge[Af.ci[e]];
    b[i] -= s;
  }
  return b;
}

// the degree is a run-time parameter of the handle: dispatch to the instantiation
Csr assemble_level(const Num3& S, double mu, double sigma, const std::vector<double>& kap, Csr* full_out) {
  return S.k == 0 ? assemble_level_k<0>(S, mu, sigma, kap, full_out) : assemble_level_k<1>(S, mu, sigma, kap, full_out);
}
Csr prolongation(const Num3& C, const Num3& F) { return F.k == 0 ? prolongation_k<0>(C, F) : prolongation_k<1>(C, F); }
std::vector<double> rhs3(const Num3& S, double mu, double sigma, const std::vector<double>& kap, const double f[3],
                         const double g[3]) {
  return S.k == 0 ? rhs3_k<0>(S, mu, sigma, kap, f, g) : rhs3_k<1>(S, mu, sigma, kap, f, g);
}

}  // namespace
}  // namespace bmg

using namespace bmg;

struct DevCsr {
  int64_t n = 0;
  int32_t *rp = nullptr, *ci = nullptr;
  double* v = nullptr;
};

struct Level3 {
  Num3 S{1, 1};
  DevCsr A, P, R;  // P, R: from / to level j-1 (j >= 1)
  int32_t* cons = nullptr;
  int64_t ncons = 0;
  int64_t npatch = 0;
  int64_t *poff = nullptr, *ioff = nullptr;
  int32_t* pdofs = nullptr;
  void* pinv = nullptr;  // doubles or floats (bmg3_params.precond_prec)
  int cstart[28] = {0};
  int maxn = 0;                          // largest patch of the level
  std::vector<int64_t> patch_of_vertex;  // vertex -> patch index
  std::vector<int64_t> hpoff, hioff;
  std::vector<int32_t> hpdofs;
  double *x = nullptr, *b = nullptr, *r = nullptr;
};

struct bmg3_ctx {
  bmg3_params p{};
  hipStream_t s = nullptr;
  std::vector<Level3> lev;
  std::vector<void*> allocs;
  double* coarse_inv = nullptr;
  int64_t n0dof = 0;
  // Krylov storage
  double *V = nullptr, *Z = nullptr, *w = nullptr, *rr = nullptr, *partial = nullptr, *hd = nullptr, *coef = nullptr;
  int32_t* live = nullptr;
  std::string err;
};

namespace {
thread_local std::string g_err3 = "null handle";

bmg_status fail3(bmg3_ctx* c, bmg_status st, const std::string& m) {
  if (c) c->err = m;
  else g_err3 = m;
  return st;
}

template <typename T>
bmg_status dalloc(bmg3_ctx* c, T** p, size_t count) {
  void* q = nullptr;
  if (hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) return BMG_E_NOMEM;
  c->allocs.push_back(q);
  *p = (T*)q;
  return BMG_OK;
}

template <typename T>
bmg_status upload(bmg3_ctx* c, T** p, const T* src, size_t count) {
  bmg_status s = dalloc(c, p, count);
  if (s) return s;
  if (count && hipMemcpy(*p, src, count * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) return BMG_E_HIP;
  return BMG_OK;
}

bmg_status upload_csr(bmg3_ctx* c, DevCsr& D, const Csr& A) {
  D.n = A.n;
  bmg_status s;
  if ((s = upload(c, &D.rp, A.rp.data(), A.rp.size()))) return s;
  if ((s = upload(c, &D.ci, A.ci.data(), A.ci.size()))) return s;
  return upload(c, &D.v, A.v.data(), A.v.size());
}

bmg_status check3(const bmg3_params* p) {
  if (!p) return BMG_E_ARG;
  if (p->k != 0 && p->k != 1) return BMG_E_UNSUPPORTED;
  if (p->n0 < 1 || p->n0 > 8 || p->levels < 1 || p->levels > 8) return BMG_E_ARG;
  // finest mesh: 64^3 for RT_1 (65 GB of patch inverses), 128^3 for RT_0 (8.5 M unknowns)
  if ((int64_t)p->n0 << (p->levels - 1) > (p->k == 0 ? 128 : 64)) return BMG_E_ARG;
  if (!(p->mu >= 0.0) || !std::isfinite(p->mu) || !(p->sigma > 0.0) || !std::isfinite(p->sigma)) return BMG_E_ARG;
  if ((p->cycle != 0 && p->cycle != 1) || p->m_fine < 1 || p->restart < 1 || p->restart > 200) return BMG_E_ARG;
  if (p->precond_prec != 0 && p->precond_prec != 1) return BMG_E_ARG;
  for (int q = 0; q < 6; ++q)
    if (p->bc[q] != BMG_BC_DIRICHLET && p->bc[q] != BMG_BC_OPEN) return BMG_E_ARG;
  return BMG_OK;
}

// vertex patch of (vx, vy, vz): free dofs whose support lies in the patch cells, ascending
void patch_dofs3(const Num3& S, int vx, int vy, int vz, std::vector<int64_t>& out, std::vector<int>& cells) {
  const int N = S.N, NA3 = S.NA3, NB3 = S.NB3, NU3 = S.NU3, NL3 = S.NL3;
  out.clear();
  cells.clear();
  bool in[2][2][2] = {};
  for (int oz = 0; oz < 2; ++oz)
    for (int oy = 0; oy < 2; ++oy)
      for (int ox = 0; ox < 2; ++ox) {
        const int cx = vx - 1 + ox, cy = vy - 1 + oy, cz = vz - 1 + oz;
        in[oz][oy][ox] = cx >= 0 && cx < N && cy >= 0 && cy < N && cz >= 0 && cz < N;
      }
  auto inpatch = [&](int cx, int cy, int cz) {
    const int ox = cx - vx + 1, oy = cy - vy + 1, oz = cz - vz + 1;
    return ox >= 0 && ox < 2 && oy >= 0 && oy < 2 && oz >= 0 && oz < 2 && in[oz][oy][ox];
  };
  for (int oz = 0; oz < 2; ++oz)
    for (int oy = 0; oy < 2; ++oy)
      for (int ox = 0; ox < 2; ++ox) {
        if (!in[oz][oy][ox]) continue;
        const int cc[3] = {vx - 1 + ox, vy - 1 + oy, vz - 1 + oz};
        cells.push_back((int)S.cell(cc[0], cc[1], cc[2]));
        for (int l = 0; l < NL3; ++l) {
          if (l < NU3) {
            const int d = l / (NA3 * NB3 * NB3), a = (l % (NA3 * NB3 * NB3)) / (NB3 * NB3);
            if (a <= 1) {
              int nb[3] = {cc[0], cc[1], cc[2]};
              nb[d] += a == 1 ? 1 : -1;
              if (nb[d] >= 0 && nb[d] < N && !inpatch(nb[0], nb[1], nb[2])) continue;
            }
          }
          const int64_t gi = S.g(cc, l);
          if (!S.essential(gi)) out.push_back(gi);
        }
      }
  std::sort(out.begin(), out.end());
  out.erase(std::unique(out.begin(), out.end()), out.end());
}

inline int colour3(int vx, int vy, int vz) { return (vx % 3) + 3 * (vy % 3) + 9 * (vz % 3); }

// Pseudo-inverse of A[D, D] (column-major into dst, symmetrised): the leading block of the inverse of
// [[A_D, c], [c^T, 0]] with c the normalised patch-constant pressure (every patch has it
// in its kernel: no patch space holds a boundary normal dof).
bool patch_pinv3(const Num3& S, const Csr& A, const std::vector<int64_t>& D, const std::vector<int>& cells,
                 double* dst) {
  // a patch with a free normal dof on an open side has no pressure constant in its
  // kernel: plain inverse; otherwise bordered with the normalised patch-constant pressure
  bool singular = true;
  for (int64_t gi : D) singular = singular && !S.open_normal(gi);
  const int n = (int)D.size(), m = singular ? n + 1 : n;
  std::vector<double> a((size_t)m * m, 0.0), inv;
  for (int t = 0; t < n; ++t)
    for (int32_t e = A.rp[D[t]]; e < A.rp[D[t] + 1]; ++e) {
      const auto it = std::lower_bound(D.begin(), D.end(), (int64_t)A.ci[e]);
      if (it != D.end() && *it == A.ci[e]) a[(size_t)t * m + (it - D.begin())] = A.v[e];
    }
  if (singular) {
    const double cv = 1.0 / std::sqrt((double)cells.size());
    for (int cl : cells) {
      const int64_t gpres = S.n_u + (int64_t)cl * S.NP3;
      const int t = (int)(std::lower_bound(D.begin(), D.end(), gpres) - D.begin());
      a[(size_t)t * m + n] = cv;
      a[(size_t)n * m + t] = cv;
    }
  }
  if (!gj_inverse(m, a, inv)) return false;
  // the pseudo-inverse of the symmetric patch matrix is symmetric: the two rounded
  // copies of each off-diagonal entry are averaged (exactly symmetric result)
  for (int t = 0; t < n; ++t)
    for (int u = 0; u < n; ++u) dst[(size_t)u * n + t] = 0.5 * (inv[(size_t)t * m + u] + inv[(size_t)u * m + t]);
  return true;
}

// Stored form of a symmetric n x n block F (column-major): its rotated diagonals
// R[d n + t] = F(t, (t + d) mod n), d = 0 .. n/2, n (n/2 + 1) entries; every entry of
// F is F(t, u) or F(u, t) of one of them.
void rotate_sym3(int n, const double* F, double* R) {
  for (int d = 0; d <= n / 2; ++d)
    for (int t = 0; t < n; ++t) R[(size_t)d * n + t] = F[(size_t)((t + d) % n) * n + t];
}

// Inverse of rotate_sym3 into the full column-major block.
void unrotate_sym3(int n, const double* R, double* F) {
  for (int d = 0; d <= n / 2; ++d)
    for (int t = 0; t < n; ++t) {
      const int u = (t + d) % n;
      F[(size_t)u * n + t] = F[(size_t)t * n + u] = R[(size_t)d * n + t];
    }
}

// Patches of one level: dofs, pseudo-inverses (bordered with the normalised patch-
// constant pressure unless the patch holds a normal dof of an open side), colour ranges.
bmg_status build_patches3(bmg3_ctx* c, Level3& L, const Csr& A) {
  const Num3& S = L.S;
  const int N = S.N, nv = N + 1;
  const int64_t nvert = (int64_t)nv * nv * nv;
  std::vector<std::vector<int64_t>> byc(27);
  for (int vz = 0; vz < nv; ++vz)
    for (int vy = 0; vy < nv; ++vy)
      for (int vx = 0; vx < nv; ++vx) byc[colour3(vx, vy, vz)].push_back(((int64_t)vz * nv + vy) * nv + vx);
  std::vector<int64_t> order;
  for (int col = 0; col < 27; ++col) {
    L.cstart[col] = (int)order.size();
    order.insert(order.end(), byc[col].begin(), byc[col].end());
  }
  L.cstart[27] = (int)order.size();
  L.npatch = nvert;
  L.patch_of_vertex.assign(nvert, -1);
  std::vector<std::vector<int64_t>> dofs(nvert);
  std::vector<std::vector<int>> cells(nvert);
  par_for(nvert, [&](int64_t p) {
    const int64_t v = order[p];
    patch_dofs3(S, (int)(v % nv), (int)((v / nv) % nv), (int)(v / ((int64_t)nv * nv)), dofs[p], cells[p]);
  });
  L.hpoff.assign(nvert + 1, 0);
  L.hioff.assign(nvert + 1, 0);
  for (int64_t p = 0; p < nvert; ++p) {
    L.patch_of_vertex[order[p]] = p;
    const int64_t n = (int64_t)dofs[p].size();
    if (n == 0) return fail3(c, BMG_E_ARG, "empty patch");
    if (n > kMaxPatch3)
      return fail3(c, BMG_E_UNSUPPORTED, "a patch holds more than 256 dofs (opposite open sides on a 2-cell level)");
    L.hpoff[p + 1] = L.hpoff[p] + n;
    L.maxn = std::max(L.maxn, (int)n);
    // FP64: rotated diagonals of the symmetric block; FP32: the full block
    L.hioff[p + 1] = L.hioff[p] + (c->p.precond_prec == 1 ? n * n : n * (n / 2 + 1));
  }
  L.hpdofs.resize(L.hpoff[nvert]);
  std::vector<double> pinv(L.hioff[nvert]);
  std::atomic<int> bad{0};
  par_for(nvert, [&](int64_t p) {
    const auto& D = dofs[p];
    for (size_t t = 0; t < D.size(); ++t) L.hpdofs[L.hpoff[p] + t] = (int32_t)D[t];
    if (c->p.precond_prec == 1) {
      if (!patch_pinv3(S, A, D, cells[p], &pinv[L.hioff[p]])) bad.store(1);
    } else {
      std::vector<double> full(D.size() * D.size());
      if (!patch_pinv3(S, A, D, cells[p], full.data())) bad.store(1);
      else rotate_sym3((int)D.size(), full.data(), &pinv[L.hioff[p]]);
    }
  });
  if (bad.load()) return fail3(c, BMG_E_SINGULAR, "a patch matrix is singular");
  bmg_status s;
  if ((s = upload(c, &L.poff, L.hpoff.data(), L.hpoff.size()))) return fail3(c, s, "device allocation failed");
  if ((s = upload(c, &L.ioff, L.hioff.data(), L.hioff.size()))) return fail3(c, s, "device allocation failed");
  if ((s = upload(c, &L.pdofs, L.hpdofs.data(), L.hpdofs.size()))) return fail3(c, s, "device allocation failed");
  if (c->p.precond_prec == 1) {
    std::vector<float> pf(pinv.begin(), pinv.end());
    float* d = nullptr;
    if ((s = upload(c, &d, pf.data(), pf.size()))) return fail3(c, s, "device allocation failed");
    L.pinv = d;
  } else {
    double* d = nullptr;
    if ((s = upload(c, &d, pinv.data(), pinv.size()))) return fail3(c, s, "device allocation failed");
    L.pinv = d;
  }
  return BMG_OK;
}

std::vector<double> coarsen(const std::vector<double>& kf, int Nc) {
  const int Nf = 2 * Nc;
  std::vector<double> kc((size_t)Nc * Nc * Nc);
  for (int z = 0; z < Nc; ++z)
    for (int y = 0; y < Nc; ++y)
      for (int x = 0; x < Nc; ++x) {
        double s = 0.0;
        for (int o = 0; o < 8; ++o)
          s += kf[((size_t)(2 * z + (o >> 2)) * Nf + 2 * y + ((o >> 1) & 1)) * Nf + 2 * x + (o & 1)];
        kc[((size_t)z * Nc + y) * Nc + x] = 0.125 * s;
      }
  return kc;
}

void smooth_step3(bmg3_ctx* c, Level3& L, double* x, const double* b) {
  for (int k = 0; k < 53; ++k) {
    const int col = k < 27 ? k : 52 - k;
    launch3_colour(L.cstart[col], L.cstart[col + 1] - L.cstart[col], L.poff, L.pdofs, L.ioff, L.pinv,
                   c->p.precond_prec, L.A.rp, L.A.ci, L.A.v, x, b, L.maxn, c->s);
  }
}

int msteps(const bmg3_ctx* c, int j) {
  const int J = (int)c->lev.size() - 1;
  return c->p.cycle == 1 ? c->p.m_fine << (J - j) : c->p.m_fine;
}

void vcycle3(bmg3_ctx* c, int j, const double* b, double* x) {
  Level3& L = c->lev[j];
  if (j == 0) {
    launch_dense_gemv(0, c->coarse_inv, c->n0dof, b, x, 1, c->s);
    return;
  }
  Level3& Lc = c->lev[j - 1];
  launch_fill_zero(0, x, L.S.ndof, c->s);
  const int m = msteps(c, j);
  for (int k = 0; k < m; ++k) smooth_step3(c, L, x, b);
  launch3_csr(1, L.S.ndof, L.A.rp, L.A.ci, L.A.v, x, b, L.r, c->s);
  launch3_csr(0, Lc.S.ndof, L.R.rp, L.R.ci, L.R.v, L.r, nullptr, Lc.b, c->s);
  vcycle3(c, j - 1, Lc.b, Lc.x);
  launch3_csr(2, L.S.ndof, L.P.rp, L.P.ci, L.P.v, Lc.x, nullptr, x, c->s);
  for (int k = 0; k < m; ++k) smooth_step3(c, L, x, b);
  launch3_copy_idx(L.cons, L.ncons, b, x, c->s);
}

bool sync_ok(bmg3_ctx* c) { return hipStreamSynchronize(c->s) == hipSuccess; }

}  // namespace

extern "C" {

bmg_status bmg3_setup(const bmg3_params* p, const double* kappa_host, void* hip_stream, bmg3_handle* out) try {
  if (!out) return fail3(nullptr, BMG_E_ARG, "out is NULL");
  *out = nullptr;
  bmg_status st = check3(p);
  if (st) return fail3(nullptr, st, "invalid parameters");
  if (!kappa_host) return fail3(nullptr, BMG_E_ARG, "kappa is NULL");
  const int J = p->levels - 1, Nf = p->n0 << J;
  const size_t nk = (size_t)Nf * Nf * Nf;
  for (size_t i = 0; i < nk; ++i)
    if (!std::isfinite(kappa_host[i]) || kappa_host[i] < 0.0) return fail3(nullptr, BMG_E_ARG, "kappa must be >= 0");
  auto* c = new bmg3_ctx();
  c->p = *p;
  c->s = (hipStream_t)hip_stream;
  auto bail = [&](bmg_status s, const std::string& m) {
    g_err3 = m.empty() ? c->err : m;
    bmg3_destroy(c);
    return s;
  };
  std::vector<std::vector<double>> kap(p->levels);
  kap[J].assign(kappa_host, kappa_host + nk);
  for (int j = J; j > 0; --j) kap[j - 1] = coarsen(kap[j], p->n0 << (j - 1));
  c->lev.resize(p->levels);
  for (int j = 0; j <= J; ++j) {
    Level3& L = c->lev[j];
    L.S = Num3(p->n0 << j, p->k, p->bc);
    Csr A = assemble_level(L.S, p->mu, p->sigma, kap[j], nullptr);
    if (A.n == 0) return bail(BMG_E_SINGULAR, "essential row without diagonal");
    if (upload_csr(c, L.A, A)) return bail(BMG_E_NOMEM, "device allocation failed");
    std::vector<int32_t> cons;
    for (int64_t i = 0; i < L.S.ndof; ++i)
      if (L.S.essential(i)) cons.push_back((int32_t)i);
    L.ncons = (int64_t)cons.size();
    if (upload(c, &L.cons, cons.data(), cons.size())) return bail(BMG_E_NOMEM, "device allocation failed");
    if (dalloc(c, &L.x, L.S.ndof) || dalloc(c, &L.b, L.S.ndof) || dalloc(c, &L.r, L.S.ndof))
      return bail(BMG_E_NOMEM, "device allocation failed");
    if (j == 0) {
      // dense inverse, bordered when every side is Dirichlet (the constant pressure
      // is then in the kernel; an open side fixes it)
      const bool brd = L.S.all_dirichlet();
      const int64_t n = L.S.ndof, m = brd ? n + 1 : n;
      std::vector<double> a((size_t)m * m, 0.0), inv;
      for (int64_t i = 0; i < n; ++i)
        for (int32_t e = A.rp[i]; e < A.rp[i + 1]; ++e) a[(size_t)i * m + A.ci[e]] = A.v[e];
      const double cv = 1.0 / std::sqrt((double)L.S.N * L.S.N * L.S.N);
      for (int64_t cl = 0; brd && cl < (int64_t)L.S.N * L.S.N * L.S.N; ++cl) {
        a[(size_t)(L.S.n_u + cl * L.S.NP3) * m + n] = cv;
        a[(size_t)n * m + L.S.n_u + cl * L.S.NP3] = cv;
      }
      if (!gj_inverse((int)m, a, inv)) return bail(BMG_E_SINGULAR, "coarse matrix is singular");
      std::vector<double> ci((size_t)n * n);  // row-major (applied row by row)
      for (int64_t i = 0; i < n; ++i)
        for (int64_t k = 0; k < n; ++k) ci[(size_t)i * n + k] = inv[(size_t)i * m + k];
      c->n0dof = n;
      if (upload(c, &c->coarse_inv, ci.data(), ci.size())) return bail(BMG_E_NOMEM, "device allocation failed");
    } else {
      // its own status: SINGULAR for a singular patch, NOMEM / HIP for device errors
      if (const bmg_status ps = build_patches3(c, L, A)) return bail(ps, "");
      Csr P = prolongation(c->lev[j - 1].S, L.S);
      Csr R = transpose(P);
      if (upload_csr(c, L.P, P) || upload_csr(c, L.R, R)) return bail(BMG_E_NOMEM, "device allocation failed");
    }
  }
  const int64_t n = c->lev[J].S.ndof, m = p->restart;
  if (dalloc(c, &c->V, (size_t)(m + 1) * n) || dalloc(c, &c->Z, (size_t)m * n) || dalloc(c, &c->w, n) ||
      dalloc(c, &c->rr, n) || dalloc(c, &c->partial, (size_t)dots_partial_count() * (m + 2)) ||
      dalloc(c, &c->hd, 2 * (m + 3)) || dalloc(c, &c->coef, m + 1) || dalloc(c, &c->live, 1))
    return bail(BMG_E_NOMEM, "device allocation failed");
  const int32_t one = 1;
  if (hipMemcpy(c->live, &one, sizeof(one), hipMemcpyHostToDevice) != hipSuccess)
    return bail(BMG_E_HIP, "hipMemcpy failed");
  *out = c;
  return BMG_OK;
} catch (const std::bad_alloc&) {
  return BMG_E_NOMEM;
} catch (...) {
  return BMG_E_STATE;
}

bmg_status bmg3_destroy(bmg3_handle h) try {
  if (!h) return BMG_E_ARG;
  if (h->s) (void)hipStreamSynchronize(h->s);
  else (void)hipDeviceSynchronize();
  for (void* q : h->allocs) (void)hipFree(q);
  delete h;
  return BMG_OK;
} catch (const std::bad_alloc&) {
  return BMG_E_NOMEM;
} catch (...) {
  return BMG_E_STATE;
}

bmg_status bmg3_sizes(bmg3_handle h, int32_t level, int32_t* N, int64_t* n_u, int64_t* n_p, int64_t* npatch) try {
  if (!h || level < 0 || level >= (int)h->lev.size()) return BMG_E_ARG;
  const Level3& L = h->lev[level];
  if (N) *N = L.S.N;
  if (n_u) *n_u = L.S.n_u;
  if (n_p) *n_p = L.S.n_p;
  if (npatch) *npatch = level ? L.npatch : 0;
  return BMG_OK;
} catch (const std::bad_alloc&) {
  return BMG_E_NOMEM;
} catch (...) {
  return BMG_E_STATE;
}

bmg_status bmg3_assemble_rhs(const bmg3_params* p, const double* kappa_host, const double* f, const double* g,
                             double* b_host) try {
  bmg_status st = check3(p);
  if (st) return fail3(nullptr, st, "invalid parameters");
  if (!kappa_host || !f || !g || !b_host) return fail3(nullptr, BMG_E_ARG, "NULL argument");
  const int Nf = p->n0 << (p->levels - 1);
  Num3 S(Nf, p->k, p->bc);
  std::vector<double> kap(kappa_host, kappa_host + (size_t)Nf * Nf * Nf);
  std::vector<double> b = rhs3(S, p->mu, p->sigma, kap, f, g);
  std::memcpy(b_host, b.data(), b.size() * sizeof(double));
  return BMG_OK;
} catch (const std::bad_alloc&) {
  return BMG_E_NOMEM;
} catch (...) {
  return BMG_E_STATE;
}

bmg_status bmg3_apply(bmg3_handle h, int32_t level, const double* x_dev, double* y_dev) try {
  if (!h || level < 0 || level >= (int)h->lev.size() || !x_dev || !y_dev) return BMG_E_ARG;
  const Level3& L = h->lev[level];
  launch3_csr(0, L.S.ndof, L.A.rp, L.A.ci, L.A.v, x_dev, nullptr, y_dev, h->s);
  return hipGetLastError() == hipSuccess ? BMG_OK : fail3(h, BMG_E_HIP, "launch failed");
} catch (const std::bad_alloc&) {
  return BMG_E_NOMEM;
} catch (...) {
  return BMG_E_STATE;
}

bmg_status bmg3_smooth(bmg3_handle h, int32_t level, int32_t steps, double* x_dev, const double* b_dev) try {
  if (!h || level < 1 || level >= (int)h->lev.size() || steps < 0 || !x_dev || !b_dev) return BMG_E_ARG;
  for (int k = 0; k < steps; ++k) smooth_step3(h, h->lev[level], x_dev, b_dev);
  return hipGetLastError() == hipSuccess ? BMG_OK : fail3(h, BMG_E_HIP, "launch failed");
} catch (const std::bad_alloc&) {
  return BMG_E_NOMEM;
} catch (...) {
  return BMG_E_STATE;
}

bmg_status bmg3_vcycle(bmg3_handle h, const double* r_dev, double* z_dev) try {
  if (!h || !r_dev || !z_dev) return BMG_E_ARG;
  vcycle3(h, (int)h->lev.size() - 1, r_dev, z_dev);
  return hipGetLastError() == hipSuccess ? BMG_OK : fail3(h, BMG_E_HIP, "launch failed");
} catch (const std::bad_alloc&) {
  return BMG_E_NOMEM;
} catch (...) {
  return BMG_E_STATE;
}

bmg_status bmg3_solve(bmg3_handle h, const double* b_dev, double* x_dev, double rtol, int32_t maxit,
                      bmg_solve_info* info) try {
  if (!h || !b_dev || !x_dev || !(rtol > 0.0) || maxit < 1) return BMG_E_ARG;
  Level3& L = h->lev.back();
  const int64_t n = L.S.ndof;
  const int m = h->p.restart;
  hipStream_t s = h->s;
  double* hd = h->hd;  // [0 .. m+1]: h column (first pass), [m+2 .. 2m+3]: second pass, [2m+4]: norm
  const int NS = 2 * (m + 2);
  auto norm2 = [&](const double* v, double& out) {
    launch_dots(v, 1, n, v, n, h->partial, hd + NS, 1, 0, s);
    if (hipMemcpyAsync(&out, hd + NS, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess) return false;
    if (!sync_ok(h)) return false;
    out = std::sqrt(out);
    return true;
  };
  double bn = 0.0;
  if (!norm2(b_dev, bn)) return fail3(h, BMG_E_HIP, "device error");
  if (!std::isfinite(bn)) return fail3(h, BMG_E_NONFINITE, "right-hand side is not finite");
  launch_fill_zero(0, x_dev, n, s);
  if (info) *info = bmg_solve_info{0, 0, 0.0, 0.0};
  if (bn == 0.0) {
    if (info) info->converged = 1;
    return BMG_OK;
  }
  int its = 0;
  bool conv = false;
  double est = 1.0, prev = -1.0;
  std::vector<double> H((size_t)(m + 1) * m), g(m + 1), cs(m), sn(m), hcol(2 * (m + 2)), y(m);
  while (its < maxit) {
    launch3_csr(1, n, L.A.rp, L.A.ci, L.A.v, x_dev, b_dev, h->rr, s);
    double beta = 0.0;
    if (!norm2(h->rr, beta)) return fail3(h, BMG_E_HIP, "device error");
    if (!std::isfinite(beta)) return fail3(h, BMG_E_NONFINITE, "residual is not finite");
    if (beta <= rtol * bn) {
      conv = true;
      est = beta / bn;
      break;
    }
    if (prev > 0.0 && beta > 0.9 * prev) break;  // a cycle that no longer reduces the true residual
    prev = beta;
    launch_scale(h->V, h->rr, hd + NS, 0, h->live, true, n, 1, s);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int done = 0;
    for (int i = 0; i < m && its < maxit; ++i) {
      double* Zi = h->Z + (size_t)i * n;
      vcycle3(h, (int)h->lev.size() - 1, h->V + (size_t)i * n, Zi);
      launch3_csr(0, n, L.A.rp, L.A.ci, L.A.v, Zi, nullptr, h->w, s);
      // classical Gram-Schmidt, twice
      launch_dots(h->V, i + 1, n, h->w, n, h->partial, hd, 1, 0, s);
      launch_axpys(h->w, h->V, i + 1, n, hd, 0, -1.0, n, 1, s);
      launch_dots(h->V, i + 1, n, h->w, n, h->partial, hd + (m + 2), 1, 0, s);
      launch_axpys(h->w, h->V, i + 1, n, hd + (m + 2), 0, -1.0, n, 1, s);
      launch_dots(h->w, 1, n, h->w, n, h->partial, hd + NS, 1, 0, s);
      if (hipMemcpyAsync(hcol.data(), hd, sizeof(double) * (NS + 1), hipMemcpyDeviceToHost, s) != hipSuccess ||
          !sync_ok(h))
        return fail3(h, BMG_E_HIP, "device error");
      for (int l = 0; l <= i; ++l) H[(size_t)l * m + i] = hcol[l] + hcol[m + 2 + l];
      const double hn = std::sqrt(std::max(hcol[NS], 0.0));
      launch_scale(h->V + (size_t)(i + 1) * n, h->w, hd + NS, 0, h->live, true, n, 1, s);
      for (int l = 0; l < i; ++l) {
        const double t = cs[l] * H[(size_t)l * m + i] + sn[l] * H[(size_t)(l + 1) * m + i];
        H[(size_t)(l + 1) * m + i] = -sn[l] * H[(size_t)l * m + i] + cs[l] * H[(size_t)(l + 1) * m + i];
        H[(size_t)l * m + i] = t;
      }
      const double den = std::hypot(H[(size_t)i * m + i], hn);
      if (!std::isfinite(den)) return fail3(h, BMG_E_NONFINITE, "Arnoldi step is not finite");
      cs[i] = den > 0 ? H[(size_t)i * m + i] / den : 1.0;
      sn[i] = den > 0 ? hn / den : 0.0;
      H[(size_t)i * m + i] = den;
      g[i + 1] = -sn[i] * g[i];
      g[i] = cs[i] * g[i];
      ++its;
      done = i + 1;
      est = std::fabs(g[i + 1]) / bn;
      if (est <= rtol || hn == 0.0) break;
    }
    for (int i = done - 1; i >= 0; --i) {
      double t = g[i];
      for (int l = i + 1; l < done; ++l) t -= H[(size_t)i * m + l] * y[l];
      y[i] = t / H[(size_t)i * m + i];
    }
    if (hipMemcpyAsync(h->coef, y.data(), sizeof(double) * done, hipMemcpyHostToDevice, s) != hipSuccess)
      return fail3(h, BMG_E_HIP, "device error");
    launch_axpys(x_dev, h->Z, done, n, h->coef, 0, 1.0, n, 1, s);
  }
  launch3_csr(1, n, L.A.rp, L.A.ci, L.A.v, x_dev, b_dev, h->rr, s);
  double tr = 0.0;
  if (!norm2(h->rr, tr)) return fail3(h, BMG_E_HIP, "device error");
  if (tr <= rtol * bn) conv = true;
  if (info) *info = bmg_solve_info{its, conv ? 1 : 0, est, tr / bn};
  return conv ? BMG_OK : fail3(h, BMG_E_NOT_CONVERGED, "not converged");
} catch (const std::bad_alloc&) {
  return BMG_E_NOMEM;
} catch (...) {
  return BMG_E_STATE;
}

bmg_status bmg3_export_patch(bmg3_handle h, int32_t level, int32_t vx, int32_t vy, int32_t vz, int32_t* n,
                             int32_t* dofs_host, double* pinv_host) try {
  if (!h || level < 1 || level >= (int)h->lev.size() || !n || !dofs_host) return BMG_E_ARG;
  const Level3& L = h->lev[level];
  const int nv = L.S.N + 1;
  if (vx < 0 || vy < 0 || vz < 0 || vx >= nv || vy >= nv || vz >= nv) return BMG_E_ARG;
  const int64_t p = L.patch_of_vertex[((int64_t)vz * nv + vy) * nv + vx];
  const int64_t o = L.hpoff[p], cnt = L.hpoff[p + 1] - o;
  *n = (int32_t)cnt;
  std::memcpy(dofs_host, L.hpdofs.data() + o, cnt * sizeof(int32_t));
  if (!pinv_host) return BMG_OK;
  const size_t stored = (size_t)(L.hioff[p + 1] - L.hioff[p]);
  if (h->p.precond_prec == 1) {
    std::vector<float> tmp(stored);
    if (hipMemcpy(tmp.data(), (const float*)L.pinv + L.hioff[p], stored * sizeof(float), hipMemcpyDeviceToHost) !=
        hipSuccess)
      return fail3(h, BMG_E_HIP, "hipMemcpy failed");
    for (size_t i = 0; i < stored; ++i) pinv_host[i] = tmp[i];
  } else {
    std::vector<double> tmp(stored);
    if (hipMemcpy(tmp.data(), (const double*)L.pinv + L.hioff[p], stored * sizeof(double), hipMemcpyDeviceToHost) !=
        hipSuccess)
      return fail3(h, BMG_E_HIP, "hipMemcpy failed");
    unrotate_sym3((int)cnt, tmp.data(), pinv_host);
  }
  return BMG_OK;
} catch (const std::bad_alloc&) {
  return BMG_E_NOMEM;
} catch (...) {
  return BMG_E_STATE;
}

bmg_status bmg3_export_level_csr(const bmg3_params* p, const double* kappa_host, int32_t level, int64_t* nnz,
                                 int32_t* rp_host, int32_t* ci_host, double* v_host) try {
  bmg_status st = check3(p);
  if (st) return fail3(nullptr, st, "invalid parameters");
  if (!kappa_host || !nnz || level < 0 || level >= p->levels) return fail3(nullptr, BMG_E_ARG, "bad argument");
  const int J = p->levels - 1, Nf = p->n0 << J;
  std::vector<double> kap(kappa_host, kappa_host + (size_t)Nf * Nf * Nf);
  for (int j = J; j > level; --j) kap = coarsen(kap, p->n0 << (j - 1));
  Csr A = assemble_level(Num3(p->n0 << level, p->k, p->bc), p->mu, p->sigma, kap, nullptr);
  if (!rp_host) {
    *nnz = (int64_t)A.v.size();
    return BMG_OK;
  }
  if (*nnz != (int64_t)A.v.size() || !ci_host || !v_host) return fail3(nullptr, BMG_E_ARG, "nnz mismatch");
  std::memcpy(rp_host, A.rp.data(), A.rp.size() * sizeof(int32_t));
  std::memcpy(ci_host, A.ci.data(), A.ci.size() * sizeof(int32_t));
  std::memcpy(v_host, A.v.data(), A.v.size() * sizeof(double));
  return BMG_OK;
} catch (const std::bad_alloc&) {
  return BMG_E_NOMEM;
} catch (...) {
  return BMG_E_STATE;
}

bmg_status bmg3_export_patch_host(const bmg3_params* p, const double* kappa_host, int32_t level, int32_t vx,
                                  int32_t vy, int32_t vz, int32_t* n, int32_t* dofs_host, double* pinv_host) try {
  bmg_status st = check3(p);
  if (st) return fail3(nullptr, st, "invalid parameters");
  if (!kappa_host || !n || !dofs_host || level < 1 || level >= p->levels) return fail3(nullptr, BMG_E_ARG, "bad argument");
  const int J = p->levels - 1, Nf = p->n0 << J, N = p->n0 << level;
  if (vx < 0 || vy < 0 || vz < 0 || vx > N || vy > N || vz > N) return fail3(nullptr, BMG_E_ARG, "vertex out of range");
  std::vector<double> kap(kappa_host, kappa_host + (size_t)Nf * Nf * Nf);
  for (int j = J; j > level; --j) kap = coarsen(kap, p->n0 << (j - 1));
  const Num3 S(N, p->k, p->bc);
  Csr A = assemble_level(S, p->mu, p->sigma, kap, nullptr);
  std::vector<int64_t> D;
  std::vector<int> cells;
  patch_dofs3(S, vx, vy, vz, D, cells);
  if ((int)D.size() > kMaxPatch3) return fail3(nullptr, BMG_E_UNSUPPORTED, "patch larger than 256 dofs");
  *n = (int32_t)D.size();
  for (size_t t = 0; t < D.size(); ++t) dofs_host[t] = (int32_t)D[t];
  if (pinv_host && !patch_pinv3(S, A, D, cells, pinv_host)) return fail3(nullptr, BMG_E_SINGULAR, "singular patch");
  return BMG_OK;
} catch (const std::bad_alloc&) {
  return BMG_E_NOMEM;
} catch (...) {
  return BMG_E_STATE;
}

const char* bmg3_last_error(bmg3_handle h) { return h ? h->err.c_str() : g_err3.c_str(); }

}  // extern "C"
