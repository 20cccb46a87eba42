// Plain FP64 CPU oracle for the geometric-multigrid-preconditioned H(div)-DG
// discretisation of the Brinkman/Darcy equations (Kanschat, Lazarov, Mao,
// "Geometric multigrid for Darcy and Brinkman models of flows in highly
// heterogeneous porous media", arXiv 1602.04858).
//
// TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
// baseline leg of the benchmark load this library; the product (the HIP library)
// shares no code with it and never calls it.
//
// Everything here is written to be checked by eye against the paper:
//   * spaces:   RT_k velocity x discontinuous Q_k pressure on a uniform N x N
//               square mesh of (0,1)^2 (Section 2.3); hierarchical basis:
//               L_b = orthonormal Legendre on [0,1], psi_0 = 1-t, psi_1 = t,
//               psi_a = integral of L_{a-1} (a >= 2); u_x = psi_a(xi) L_b(eta),
//               u_y = L_b(xi) psi_a(eta), p = L_a(xi) L_b(eta).
//   * form:     interior-penalty form a_h (Section 2.3, eq. ipbrinkman) plus the
//               divergence coupling of the saddle-point form (eq. Brinkman-weak),
//               assembled cell by cell and face by face with Gauss quadrature.
//   * boundary: on a Dirichlet side the normal velocity is imposed as an
//               essential condition (u.n = g.n, as the paper states for Darcy and
//               as its L^2_0 pressure space requires for Brinkman) and the
//               tangential part by the Nitsche terms of eq. (BCh); an open side
//               carries no boundary term.
//   * hierarchy: uniform refinement, re-discretisation per level, cell kappa
//               averaged over the four children: arithmetically (Section 4.1, the
//               default), or harmonically / geometrically (the other choices the
//               paper allows).
//   * transfer: the natural injection (Section 3.1) computed by applying the fine
//               degree-of-freedom functionals to coarse basis functions;
//               restriction is its transpose (eq. 3 acting on residuals).
//   * smoother: vertex-patch Ritz projections (Section 3.3), symmetric
//               multiplicative (eq. smoother-Multiplicative), patches visited colour
//               by colour, forward then backward.  Two colourings of the vertices:
//               S9, 9 colours (vx mod 3) + 3 (vy mod 3); L8, the 8 cosets of the
//               lattice spanned by (2, 2) and (2, -2).  Same-colour patches never
//               touch each other's dofs, so the order inside a colour is immaterial.
//   * cycle:    standard or variable V-cycle with coarse direct solve (Section 3.2).
//   * Krylov:   right-preconditioned flexible GMRES with modified Gram-Schmidt.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <memory>
#include <numeric>
#include <vector>

namespace {

// ---------------------------------------------------------------------------
// 1-D polynomials on [0,1]
// ---------------------------------------------------------------------------
void legendre_all(int n, double s, double* P, double* dP) {
  // Legendre P_0..P_n at s in [-1,1] and derivatives (Bonnet recurrence).
  P[0] = 1.0;
  dP[0] = 0.0;
  if (n >= 1) { P[1] = s; dP[1] = 1.0; }
  for (int m = 1; m < n; ++m) {
    P[m + 1] = ((2 * m + 1) * s * P[m] - m * P[m - 1]) / (m + 1);
    dP[m + 1] = dP[m - 1] + (2 * m + 1) * P[m];
  }
}

struct Rule {
  std::vector<double> x, w;  // nodes / weights on [0,1], ascending nodes
};

Rule gauss01(int q) {
  // Gauss-Legendre rule: Newton iteration on the roots of P_q.
  Rule r;
  r.x.resize(q);
  r.w.resize(q);
  std::vector<double> P(q + 1), dP(q + 1);
  for (int i = 0; i < q; ++i) {
    double s = std::cos(M_PI * (i + 0.75) / (q + 0.5));
    for (int it = 0; it < 100; ++it) {
      legendre_all(q, s, P.data(), dP.data());
      double ds = P[q] / dP[q];
      s -= ds;
      if (std::fabs(ds) < 1e-16) break;
    }
    legendre_all(q, s, P.data(), dP.data());
    double w = 2.0 / ((1.0 - s * s) * dP[q] * dP[q]);
    r.x[i] = 0.5 * (1.0 - s);  // ascending in t
    r.w[i] = 0.5 * w;
  }
  return r;
}

const Rule& rule8() {
  static Rule r = gauss01(8);
  return r;
}

double Lval(int b, double t) {
  double P[16], dP[16];
  legendre_all(b, 2.0 * t - 1.0, P, dP);
  return std::sqrt(2.0 * b + 1.0) * P[b];
}
double Lder(int b, double t) {
  double P[16], dP[16];
  legendre_all(b, 2.0 * t - 1.0, P, dP);
  return 2.0 * std::sqrt(2.0 * b + 1.0) * dP[b];
}
double psival(int a, double t) {
  if (a == 0) return 1.0 - t;
  if (a == 1) return t;
  // psi_a(t) = int_0^t L_{a-1}(s) ds, by an 8-point Gauss rule on [0,t] (exact).
  const Rule& r = rule8();
  double s = 0.0;
  for (size_t i = 0; i < r.x.size(); ++i) s += r.w[i] * Lval(a - 1, t * r.x[i]);
  return t * s;
}
double psider(int a, double t) {
  if (a == 0) return -1.0;
  if (a == 1) return 1.0;
  return Lval(a - 1, t);
}

// ---------------------------------------------------------------------------
// Sparse matrices
// ---------------------------------------------------------------------------
struct CSR {
  int n = 0, m = 0;
  std::vector<int> rp, ci;
  std::vector<double> v;
  void mult(const double* x, double* y) const {
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int e = rp[i]; e < rp[i + 1]; ++e) s += v[e] * x[ci[e]];
      y[i] = s;
    }
  }
  double row_dot(int i, const double* x) const {
    double s = 0.0;
    for (int e = rp[i]; e < rp[i + 1]; ++e) s += v[e] * x[ci[e]];
    return s;
  }
  double get(int i, int j) const {
    auto b = ci.begin() + rp[i], e = ci.begin() + rp[i + 1];
    auto it = std::lower_bound(b, e, j);
    if (it != e && *it == j) return v[it - ci.begin()];
    return 0.0;
  }
};

struct Trip {
  int i, j;
  double v;
};

CSR from_triplets(int n, int m, std::vector<Trip>& t) {
  // stable: contributions to (i,j) and (j,i) are summed in the same order
  std::stable_sort(t.begin(), t.end(), [](const Trip& a, const Trip& b) {
    return a.i != b.i ? a.i < b.i : a.j < b.j;
  });
  CSR A;
  A.n = n;
  A.m = m;
  A.rp.assign(n + 1, 0);
  for (size_t e = 0; e < t.size();) {
    size_t f = e;
    double s = 0.0;
    while (f < t.size() && t[f].i == t[e].i && t[f].j == t[e].j) s += t[f++].v;
    A.ci.push_back(t[e].j);
    A.v.push_back(s);
    A.rp[t[e].i + 1]++;
    e = f;
  }
  for (int i = 0; i < n; ++i) A.rp[i + 1] += A.rp[i];
  return A;
}

// ---------------------------------------------------------------------------
// Dense helpers
// ---------------------------------------------------------------------------
// Inverse of a dense n x n matrix (row-major) by Gauss-Jordan with partial
// pivoting.  Returns false if a pivot vanishes.
bool gj_inverse(int n, std::vector<double>& a, std::vector<double>& inv) {
  inv.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(a[(size_t)r * n + c]) > std::fabs(a[(size_t)piv * n + c])) piv = r;
    if (a[(size_t)piv * n + c] == 0.0) return false;
    if (piv != c)
      for (int j = 0; j < n; ++j) {
        std::swap(a[(size_t)piv * n + j], a[(size_t)c * n + j]);
        std::swap(inv[(size_t)piv * n + j], inv[(size_t)c * n + j]);
      }
    double d = 1.0 / a[(size_t)c * n + c];
    for (int j = 0; j < n; ++j) {
      a[(size_t)c * n + j] *= d;
      inv[(size_t)c * n + j] *= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      double f = a[(size_t)r * n + c];
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) {
        a[(size_t)r * n + j] -= f * a[(size_t)c * n + j];
        inv[(size_t)r * n + j] -= f * inv[(size_t)c * n + j];
      }
    }
  }
  return true;
}

// Inverse of a symmetric matrix with known one-dimensional null space spanned by
// the unit vector c (or of a regular one when c is empty): the leading block of
// the bordered inverse [[A, c], [c^T, 0]]^{-1}, i.e. the pseudo-inverse.
bool bordered_inverse(int n, const std::vector<double>& A, const std::vector<double>& c,
                      std::vector<double>& out) {
  if (c.empty()) {
    std::vector<double> a = A;
    return gj_inverse(n, a, out);
  }
  int m = n + 1;
  std::vector<double> a((size_t)m * m, 0.0), inv;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) a[(size_t)i * m + j] = A[(size_t)i * n + j];
  for (int i = 0; i < n; ++i) {
    a[(size_t)i * m + n] = c[i];
    a[(size_t)n * m + i] = c[i];
  }
  if (!gj_inverse(m, a, inv)) return false;
  out.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) out[(size_t)i * n + j] = inv[(size_t)i * m + j];
  return true;
}

// ---------------------------------------------------------------------------
// One mesh level: dof numbering, basis, assembly, patches
// ---------------------------------------------------------------------------
enum { BC_DIRICHLET = 0, BC_OPEN = 1 };

struct LocalFn {
  int kind;  // 0 = u_x, 1 = u_y, 2 = pressure
  int a, b;  // u_x: psi_a(xi) L_b(eta); u_y: L_b(xi) psi_a(eta); p: L_a(xi) L_b(eta)
};

struct BVal {
  double v[2];     // velocity value
  double g[2][2];  // g[c][d] = d u_c / d x_d  (physical)
  double div;
  double p;
};

struct Patch {
  int vx, vy, colour;
  bool singular;
  std::vector<int> dofs;     // ascending global indices
  std::vector<double> inv;   // pseudo-inverse, row-major
};

struct Level {
  int N, k;
  int colouring = 0, ncolours = 9;
  int smoother = 0;     // 0: symmetric multiplicative, 1: additive
  double omega = 0.25;  // damping of the additive smoother
  double h, mu, sigma;
  int bc[4];
  int nb, nv, np, nloc;  // k+1, (k+2)(k+1), (k+1)^2, 2nv+np
  int n_u, n_p, ndof;
  std::vector<LocalFn> loc;
  std::vector<double> kappa;
  std::vector<char> cons;
  bool singular = false;  // pressure constant in the kernel (no open side)
  CSR A, Afull;
  std::vector<Patch> patches;
  int colour_start[10];
  CSR P;  // prolongation from the next coarser level
};

int xface(const Level& L, int i, int cy, int b) { return (cy * (L.N + 1) + i) * L.nb + b; }
int yface(const Level& L, int j, int cx, int b) {
  return L.N * (L.N + 1) * L.nb + (j * L.N + cx) * L.nb + b;
}
int interior(const Level& L, int c, int comp, int a, int b) {
  return 2 * L.N * (L.N + 1) * L.nb + c * 2 * L.k * L.nb + (comp * L.k + (a - 2)) * L.nb + b;
}
int pres(const Level& L, int c, int a, int b) { return L.n_u + c * L.np + b * L.nb + a; }

int global_of(const Level& L, int cx, int cy, int l) {
  const LocalFn& f = L.loc[l];
  int c = cy * L.N + cx;
  if (f.kind == 0) {
    if (f.a == 0) return xface(L, cx, cy, f.b);
    if (f.a == 1) return xface(L, cx + 1, cy, f.b);
    return interior(L, c, 0, f.a, f.b);
  }
  if (f.kind == 1) {
    if (f.a == 0) return yface(L, cy, cx, f.b);
    if (f.a == 1) return yface(L, cy + 1, cx, f.b);
    return interior(L, c, 1, f.a, f.b);
  }
  return pres(L, c, f.a, f.b);
}

// Local basis function l of a cell of size h at reference point (xi, eta).
BVal eval_fn(const Level& L, int l, double xi, double eta, double h) {
  const LocalFn& f = L.loc[l];
  BVal r;
  std::memset(&r, 0, sizeof(r));
  if (f.kind == 0) {
    r.v[0] = psival(f.a, xi) * Lval(f.b, eta);
    r.g[0][0] = psider(f.a, xi) * Lval(f.b, eta) / h;
    r.g[0][1] = psival(f.a, xi) * Lder(f.b, eta) / h;
  } else if (f.kind == 1) {
    r.v[1] = Lval(f.b, xi) * psival(f.a, eta);
    r.g[1][0] = Lder(f.b, xi) * psival(f.a, eta) / h;
    r.g[1][1] = Lval(f.b, xi) * psider(f.a, eta) / h;
  } else {
    r.p = Lval(f.a, xi) * Lval(f.b, eta);
  }
  r.div = r.g[0][0] + r.g[1][1];
  return r;
}

void init_level(Level& L, int N, int k, double mu, double sigma, const int* bc) {
  L.N = N;
  L.k = k;
  L.h = 1.0 / N;
  L.mu = mu;
  L.sigma = sigma;
  for (int s = 0; s < 4; ++s) L.bc[s] = bc[s];
  L.nb = k + 1;
  L.nv = (k + 2) * (k + 1);
  L.np = (k + 1) * (k + 1);
  L.nloc = 2 * L.nv + L.np;
  L.n_u = 2 * N * (N + 1) * L.nb + 2 * k * L.nb * N * N;
  L.n_p = L.np * N * N;
  L.ndof = L.n_u + L.n_p;
  L.loc.clear();
  for (int a = 0; a < k + 2; ++a)
    for (int b = 0; b < k + 1; ++b) L.loc.push_back({0, a, b});
  for (int a = 0; a < k + 2; ++a)
    for (int b = 0; b < k + 1; ++b) L.loc.push_back({1, a, b});
  for (int b = 0; b < k + 1; ++b)
    for (int a = 0; a < k + 1; ++a) L.loc.push_back({2, a, b});
  L.cons.assign(L.ndof, 0);
  for (int cy = 0; cy < N; ++cy)
    for (int b = 0; b < L.nb; ++b) {
      if (bc[0] == BC_DIRICHLET) L.cons[xface(L, 0, cy, b)] = 1;
      if (bc[1] == BC_DIRICHLET) L.cons[xface(L, N, cy, b)] = 1;
    }
  for (int cx = 0; cx < N; ++cx)
    for (int b = 0; b < L.nb; ++b) {
      if (bc[2] == BC_DIRICHLET) L.cons[yface(L, 0, cx, b)] = 1;
      if (bc[3] == BC_DIRICHLET) L.cons[yface(L, N, cx, b)] = 1;
    }
  L.singular = (bc[0] == BC_DIRICHLET && bc[1] == BC_DIRICHLET && bc[2] == BC_DIRICHLET &&
                bc[3] == BC_DIRICHLET);
}

// Face description used for both assembly and the right-hand side.
struct FaceSide {
  int cx, cy;        // cell
  double xi, eta;    // reference coordinates of the face line: one of them fixed
  bool along_eta;    // the face is parametrised by eta (vertical face)
};

// Adds the face integrals of a_h on one face.  `nsides` = 2 for an interior face
// (side 0 = T1 with the smaller cell index, side 1 = T2), 1 for a boundary face.
void face_terms(const Level& L, const FaceSide* sides, int nsides, const double n[2],
                std::vector<Trip>& out) {
  const int q = L.k + 2;
  Rule r = gauss01(q);
  // union of velocity dofs with their local index on each side
  std::vector<int> gl;
  std::vector<int> li[2];
  for (int s = 0; s < nsides; ++s)
    for (int l = 0; l < 2 * L.nv; ++l) {
      int g = global_of(L, sides[s].cx, sides[s].cy, l);
      auto it = std::find(gl.begin(), gl.end(), g);
      int idx;
      if (it == gl.end()) {
        gl.push_back(g);
        li[0].push_back(-1);
        li[1].push_back(-1);
        idx = (int)gl.size() - 1;
      } else {
        idx = (int)(it - gl.begin());
      }
      li[s][idx] = l;
    }
  const int m = (int)gl.size();
  std::vector<double> jump((size_t)m * q * 2), agn((size_t)m * q * 2);
  for (int e = 0; e < m; ++e)
    for (int p = 0; p < q; ++p) {
      double jv[2] = {0, 0}, gv[2] = {0, 0};
      for (int s = 0; s < nsides; ++s) {
        if (li[s][e] < 0) continue;
        double xi = sides[s].along_eta ? sides[s].xi : r.x[p];
        double eta = sides[s].along_eta ? r.x[p] : sides[s].eta;
        BVal bv = eval_fn(L, li[s][e], xi, eta, L.h);
        double sign = (s == 0) ? 1.0 : -1.0;
        double wavg = (nsides == 2) ? 0.5 : 1.0;
        for (int c = 0; c < 2; ++c) {
          jv[c] += sign * bv.v[c];
          gv[c] += wavg * (bv.g[c][0] * n[0] + bv.g[c][1] * n[1]);
        }
      }
      for (int c = 0; c < 2; ++c) {
        jump[((size_t)e * q + p) * 2 + c] = jv[c];
        agn[((size_t)e * q + p) * 2 + c] = gv[c];
      }
    }
  const double pen = 2.0 * L.mu * L.sigma / L.h;
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      double s = 0.0;
      for (int p = 0; p < q; ++p) {
        const double* ji = &jump[((size_t)i * q + p) * 2];
        const double* jj = &jump[((size_t)j * q + p) * 2];
        const double* gi = &agn[((size_t)i * q + p) * 2];
        const double* gj = &agn[((size_t)j * q + p) * 2];
        double jj_ji = jj[0] * ji[0] + jj[1] * ji[1];
        double gj_ji = gj[0] * ji[0] + gj[1] * ji[1];
        double gi_jj = gi[0] * jj[0] + gi[1] * jj[1];
        s += r.w[p] * L.h * (pen * jj_ji - L.mu * (gj_ji + gi_jj));
      }
      if (s != 0.0) out.push_back({gl[i], gl[j], s});
    }
}

// Cell integrals of one cell: mu (grad u, grad v) + (kappa u, v) - (p, div v) - (q, div u).
void cell_terms(const Level& L, int cx, int cy, std::vector<Trip>& t) {
  const int N = L.N, q = L.k + 2, nl = L.nloc;
  Rule r = gauss01(q);
  std::vector<BVal> bv((size_t)nl * q * q);
  double kap = L.kappa[cy * N + cx];
  for (int l = 0; l < nl; ++l)
    for (int iy = 0; iy < q; ++iy)
      for (int ix = 0; ix < q; ++ix)
        bv[((size_t)l * q + iy) * q + ix] = eval_fn(L, l, r.x[ix], r.x[iy], L.h);
  for (int i = 0; i < nl; ++i)
    for (int j = 0; j < nl; ++j) {
      const LocalFn &fi = L.loc[i], &fj = L.loc[j];
      double s = 0.0;
      for (int iy = 0; iy < q; ++iy)
        for (int ix = 0; ix < q; ++ix) {
          const BVal& bi = bv[((size_t)i * q + iy) * q + ix];
          const BVal& bj = bv[((size_t)j * q + iy) * q + ix];
          double w = r.w[ix] * r.w[iy] * L.h * L.h;
          double val = 0.0;
          if (fi.kind < 2 && fj.kind < 2) {
            double gg = 0.0, vv = 0.0;
            for (int c = 0; c < 2; ++c) {
              vv += bi.v[c] * bj.v[c];
              for (int d = 0; d < 2; ++d) gg += bi.g[c][d] * bj.g[c][d];
            }
            val = L.mu * gg + kap * vv;
          } else if (fi.kind == 2 && fj.kind < 2) {
            val = -bi.p * bj.div;
          } else if (fi.kind < 2 && fj.kind == 2) {
            val = -bj.p * bi.div;
          }
          s += w * val;
        }
      if (s != 0.0) t.push_back({global_of(L, cx, cy, i), global_of(L, cx, cy, j), s});
    }
}

// Face integrals of one face: vertical face (i, row c) if vertical, horizontal face
// (column c, j = i) otherwise; interior faces and Dirichlet boundary faces.
void one_face(const Level& L, bool vertical, int i, int c, std::vector<Trip>& t) {
  const int N = L.N;
  if (L.mu == 0.0) return;
  if (vertical) {
    if (i > 0 && i < N) {
      FaceSide sd[2] = {{i - 1, c, 1.0, 0.0, true}, {i, c, 0.0, 0.0, true}};
      double n[2] = {1.0, 0.0};
      face_terms(L, sd, 2, n, t);
    } else if (i == 0 && L.bc[0] == BC_DIRICHLET) {
      FaceSide sd = {0, c, 0.0, 0.0, true};
      double n[2] = {-1.0, 0.0};
      face_terms(L, &sd, 1, n, t);
    } else if (i == N && L.bc[1] == BC_DIRICHLET) {
      FaceSide sd = {N - 1, c, 1.0, 0.0, true};
      double n[2] = {1.0, 0.0};
      face_terms(L, &sd, 1, n, t);
    }
  } else {
    if (i > 0 && i < N) {
      FaceSide sd[2] = {{c, i - 1, 0.0, 1.0, false}, {c, i, 0.0, 0.0, false}};
      double n[2] = {0.0, 1.0};
      face_terms(L, sd, 2, n, t);
    } else if (i == 0 && L.bc[2] == BC_DIRICHLET) {
      FaceSide sd = {c, 0, 0.0, 0.0, false};
      double n[2] = {0.0, -1.0};
      face_terms(L, &sd, 1, n, t);
    } else if (i == N && L.bc[3] == BC_DIRICHLET) {
      FaceSide sd = {c, N - 1, 0.0, 1.0, false};
      double n[2] = {0.0, 1.0};
      face_terms(L, &sd, 1, n, t);
    }
  }
}

void assemble(Level& L) {
  const int N = L.N, nl = L.nloc;
  std::vector<Trip> t;
  t.reserve((size_t)N * N * nl * nl / 2);
  for (int cy = 0; cy < N; ++cy)
    for (int cx = 0; cx < N; ++cx) cell_terms(L, cx, cy, t);
  // faces: jump, average and penalty terms (T1 = smaller cell index); Dirichlet
  // boundary faces with {v} = [v] = v and the outward normal
  for (int c = 0; c < N; ++c)
    for (int i = 0; i <= N; ++i) {
      one_face(L, true, i, c, t);
      one_face(L, false, i, c, t);
    }
  L.Afull = from_triplets(L.ndof, L.ndof, t);
  // essential normal condition: identity rows and columns for constrained dofs
  std::vector<Trip> te;
  te.reserve(L.Afull.v.size());
  for (int i = 0; i < L.ndof; ++i) {
    if (L.cons[i]) {
      te.push_back({i, i, 1.0});
      continue;
    }
    for (int e = L.Afull.rp[i]; e < L.Afull.rp[i + 1]; ++e)
      if (!L.cons[L.Afull.ci[e]]) te.push_back({i, L.Afull.ci[e], L.Afull.v[e]});
  }
  L.A = from_triplets(L.ndof, L.ndof, te);
}

// Colour of vertex (vx, vy): S9 (scheme 0) or L8 (scheme 1).  L8 is the coset of the
// lattice {(x, y): x, y even, x - y = 0 mod 4} = span{(2, 2), (2, -2)} containing the
// vertex: parity of vx, parity of vy, and whether (vx - vy) mod 4 is 0/1 or 2/3.
int vertex_colour(int scheme, int vx, int vy) {
  if (scheme == 0) return (vx % 3) + 3 * (vy % 3);
  const int d = ((vx - vy) % 4 + 4) % 4;
  return (vx & 1) + 2 * (vy & 1) + 4 * (d >= 2 ? 1 : 0);
}

// The support of velocity dof g (1 or 2 cells) lies inside the patch cell set?
void build_patches(Level& L) {
  const int N = L.N;
  std::vector<std::pair<int, int>> order;  // (colour, vertex)
  for (int vy = 0; vy <= N; ++vy)
    for (int vx = 0; vx <= N; ++vx) order.push_back({vertex_colour(L.colouring, vx, vy), vy * (N + 1) + vx});
  std::sort(order.begin(), order.end());
  L.patches.assign(order.size(), Patch());
  for (int c = 0; c <= 9; ++c) L.colour_start[c] = 0;
  for (auto& o : order) L.colour_start[o.first + 1]++;
  for (int c = 0; c < 9; ++c) L.colour_start[c + 1] += L.colour_start[c];
#pragma omp parallel for schedule(dynamic, 16)
  for (int pi = 0; pi < (int)order.size(); ++pi) {
    Patch& P = L.patches[pi];
    int v = order[pi].second;
    P.vx = v % (N + 1);
    P.vy = v / (N + 1);
    P.colour = order[pi].first;
    std::vector<std::pair<int, int>> cells;
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        int cx = P.vx - 1 + dx, cy = P.vy - 1 + dy;
        if (cx >= 0 && cx < N && cy >= 0 && cy < N) cells.push_back({cx, cy});
      }
    auto in_patch = [&](int cx, int cy) {
      for (auto& c : cells)
        if (c.first == cx && c.second == cy) return true;
      return false;
    };
    std::vector<int> S;
    bool has_boundary_normal = false;
    for (auto& c : cells)
      for (int l = 0; l < L.nloc; ++l) {
        const LocalFn& f = L.loc[l];
        int g = global_of(L, c.first, c.second, l);
        if (L.cons[g]) continue;
        if (f.kind < 2 && f.a <= 1) {
          // face dof: the neighbour across the face must be in the patch (or absent)
          int ox = c.first, oy = c.second;
          if (f.kind == 0) ox += (f.a == 0) ? -1 : 1;
          else oy += (f.a == 0) ? -1 : 1;
          bool outside = (ox < 0 || ox >= N || oy < 0 || oy >= N);
          if (!outside && !in_patch(ox, oy)) continue;
          if (outside) has_boundary_normal = true;
        }
        S.push_back(g);
      }
    std::sort(S.begin(), S.end());
    S.erase(std::unique(S.begin(), S.end()), S.end());
    P.dofs = S;
    P.singular = !has_boundary_normal;
    const int n = (int)S.size();
    std::vector<double> Ap((size_t)n * n);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) Ap[(size_t)i * n + j] = L.A.get(S[i], S[j]);
    std::vector<double> cvec;
    if (P.singular) {
      cvec.assign(n, 0.0);
      double cnt = 0;
      for (auto& c : cells) {
        int g = pres(L, c.second * N + c.first, 0, 0);
        int idx = (int)(std::lower_bound(S.begin(), S.end(), g) - S.begin());
        cvec[idx] = 1.0;
        cnt += 1;
      }
      for (auto& x : cvec) x /= std::sqrt(cnt);
    }
    bordered_inverse(n, Ap, cvec, P.inv);
  }
}

// ---------------------------------------------------------------------------
// Prolongation: fine dof functionals applied to coarse basis functions
// ---------------------------------------------------------------------------
// Value of fine dof functional (local fn lf of a child cell) applied to the
// coarse local basis function lc; (sx, sy) = child position in the coarse cell.
double fine_functional(const Level& F, const Level& C, int lf, int lc, int sx, int sy) {
  const LocalFn& f = F.loc[lf];
  const LocalFn& g = C.loc[lc];
  if (f.kind != g.kind) return 0.0;
  const int q = F.k + 2;
  Rule r = gauss01(q);
  auto coarse = [&](double xf, double yf) {
    return eval_fn(C, lc, 0.5 * (sx + xf), 0.5 * (sy + yf), C.h);
  };
  double s = 0.0;
  if (f.kind == 0) {
    if (f.a <= 1) {
      for (int i = 0; i < q; ++i) s += r.w[i] * coarse((double)f.a, r.x[i]).v[0] * Lval(f.b, r.x[i]);
    } else {
      for (int i = 0; i < q; ++i)
        for (int j = 0; j < q; ++j)
          s += r.w[i] * r.w[j] * F.h * coarse(r.x[i], r.x[j]).g[0][0] * Lval(f.a - 1, r.x[i]) *
               Lval(f.b, r.x[j]);
    }
  } else if (f.kind == 1) {
    if (f.a <= 1) {
      for (int i = 0; i < q; ++i) s += r.w[i] * coarse(r.x[i], (double)f.a).v[1] * Lval(f.b, r.x[i]);
    } else {
      for (int i = 0; i < q; ++i)
        for (int j = 0; j < q; ++j)
          s += r.w[i] * r.w[j] * F.h * coarse(r.x[i], r.x[j]).g[1][1] * Lval(f.a - 1, r.x[j]) *
               Lval(f.b, r.x[i]);
    }
  } else {
    for (int i = 0; i < q; ++i)
      for (int j = 0; j < q; ++j)
        s += r.w[i] * r.w[j] * coarse(r.x[i], r.x[j]).p * Lval(f.a, r.x[i]) * Lval(f.b, r.x[j]);
  }
  return s;
}

void build_prolongation(Level& F, const Level& C) {
  std::vector<char> done(F.ndof, 0);
  std::vector<Trip> t;
  // the functional values do not depend on the cell: tabulate per child
  const int nl = F.nloc;
  std::vector<double> tab((size_t)4 * nl * nl);
  for (int s = 0; s < 4; ++s)
    for (int lf = 0; lf < nl; ++lf)
      for (int lc = 0; lc < nl; ++lc)
        tab[((size_t)s * nl + lf) * nl + lc] = fine_functional(F, C, lf, lc, s & 1, s >> 1);
  for (int cyc = 0; cyc < C.N; ++cyc)
    for (int cxc = 0; cxc < C.N; ++cxc)
      for (int s = 0; s < 4; ++s) {
        int sx = s & 1, sy = s >> 1;
        int fx = 2 * cxc + sx, fy = 2 * cyc + sy;
        for (int lf = 0; lf < nl; ++lf) {
          int gf = global_of(F, fx, fy, lf);
          if (done[gf]) continue;
          done[gf] = 1;
          if (F.cons[gf]) continue;
          for (int lc = 0; lc < nl; ++lc) {
            int gc = global_of(C, cxc, cyc, lc);
            if (C.cons[gc]) continue;
            double v = tab[((size_t)s * nl + lf) * nl + lc];
            if (v != 0.0) t.push_back({gf, gc, v});
          }
        }
      }
  F.P = from_triplets(F.ndof, C.ndof, t);
}

// ---------------------------------------------------------------------------
// Solver context
// ---------------------------------------------------------------------------
struct Ctx {
  int J, k, cycle, m_fine;
  std::vector<Level> lev;
  std::vector<double> coarse_inv;  // dense inverse of A_0 (pseudo-inverse if singular)
};

double dot(const std::vector<double>& a, const std::vector<double>& b) {
  double s = 0.0;
  for (size_t i = 0; i < a.size(); ++i) s += a[i] * b[i];
  return s;
}

void colour_step(const Level& L, int colour, double* x, const double* b) {
#pragma omp parallel for schedule(dynamic, 8)
  for (int pi = L.colour_start[colour]; pi < L.colour_start[colour + 1]; ++pi) {
    const Patch& P = L.patches[pi];
    const int n = (int)P.dofs.size();
    std::vector<double> r(n);
    for (int i = 0; i < n; ++i) r[i] = b[P.dofs[i]] - L.A.row_dot(P.dofs[i], x);
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int j = 0; j < n; ++j) s += P.inv[(size_t)i * n + j] * r[j];
      x[P.dofs[i]] += s;
    }
  }
}

// One application of the additive Schwarz smoother over the same patch spaces:
// x += omega sum_v R_v^T A_v^+ R_v (b - A x), every local problem solved with the
// residual of the input x (the paper's multiplicative smoother applies the same
// projections one after the other; the damping omega is a parameter of this variant).
void additive_once(const Level& L, double* x, const double* b) {
  std::vector<double> r(L.ndof), y(L.ndof, 0.0);
  for (int i = 0; i < L.ndof; ++i) r[i] = b[i] - L.A.row_dot(i, x);
  for (const Patch& P : L.patches) {
    const int n = (int)P.dofs.size();
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int j = 0; j < n; ++j) s += P.inv[(size_t)i * n + j] * r[P.dofs[j]];
      y[P.dofs[i]] += s;
    }
  }
  for (int i = 0; i < L.ndof; ++i) x[i] += L.omega * y[i];
}

// One application of the symmetric multiplicative smoother: colours 0..C-1, then
// C-2..0 (the last colour once: its local projections are idempotent); or of the
// additive one.
void smooth_once(const Level& L, double* x, const double* b) {
  if (L.smoother == 1) {
    additive_once(L, x, b);
    return;
  }
  for (int c = 0; c < L.ncolours; ++c) colour_step(L, c, x, b);
  for (int c = L.ncolours - 2; c >= 0; --c) colour_step(L, c, x, b);
}

void restrict_(const Level& F, const double* rf, double* bc, int nc) {
  std::fill(bc, bc + nc, 0.0);
  for (int i = 0; i < F.ndof; ++i)
    for (int e = F.P.rp[i]; e < F.P.rp[i + 1]; ++e) bc[F.P.ci[e]] += F.P.v[e] * rf[i];
}

void prolong_add(const Level& F, const double* xc, double* xf) {
  for (int i = 0; i < F.ndof; ++i) xf[i] += F.P.row_dot(i, xc);
}

void coarse_solve(const Ctx& X, const double* b, double* x) {
  const int n = X.lev[0].ndof;
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += X.coarse_inv[(size_t)i * n + j] * b[j];
    x[i] = s;
  }
}

void vcycle_level(const Ctx& X, int j, const double* b, double* x) {
  const Level& L = X.lev[j];
  if (j == 0) {
    coarse_solve(X, b, x);
    return;
  }
  const int m = (X.cycle == 1) ? X.m_fine << (X.J - j) : X.m_fine;
  std::fill(x, x + L.ndof, 0.0);
  for (int s = 0; s < m; ++s) smooth_once(L, x, b);
  std::vector<double> r(L.ndof), bc(X.lev[j - 1].ndof), xc(X.lev[j - 1].ndof);
  L.A.mult(x, r.data());
  for (int i = 0; i < L.ndof; ++i) r[i] = b[i] - r[i];
  restrict_(L, r.data(), bc.data(), (int)bc.size());
  vcycle_level(X, j - 1, bc.data(), xc.data());
  prolong_add(L, xc.data(), x);
  for (int s = 0; s < m; ++s) smooth_once(L, x, b);
  // identity rows of the constrained dofs are inverted exactly
  for (int i = 0; i < L.ndof; ++i)
    if (L.cons[i]) x[i] = b[i];
}

// Coarse kappa of one cell from its four children: 0 arithmetic mean, 1 harmonic
// mean (0 if a child is 0), 2 geometric mean.
double average4(int mode, double a, double b, double c, double d) {
  if (mode == 1) {
    if (a == 0.0 || b == 0.0 || c == 0.0 || d == 0.0) return 0.0;
    return 4.0 / (1.0 / a + 1.0 / b + 1.0 / c + 1.0 / d);
  }
  if (mode == 2) return std::sqrt(std::sqrt(a * b) * std::sqrt(c * d));
  return 0.25 * (a + b + c + d);
}

Ctx* create(int n0, int J, int k, double mu, double sigma, const int* bc, const double* kappa,
            int cycle, int m_fine, int colouring, int kappa_avg) {
  auto X = std::make_unique<Ctx>();
  X->J = J;
  X->k = k;
  X->cycle = cycle;
  X->m_fine = m_fine;
  X->lev.resize(J + 1);
  for (int j = 0; j <= J; ++j) {
    init_level(X->lev[j], n0 << j, k, mu, sigma, bc);
    X->lev[j].colouring = colouring;
    X->lev[j].ncolours = colouring ? 8 : 9;
  }
  // kappa: finest given, coarser levels by averaging the 4 children
  X->lev[J].kappa.assign(kappa, kappa + (size_t)(n0 << J) * (n0 << J));
  for (int j = J; j >= 1; --j) {
    const Level& F = X->lev[j];
    Level& C = X->lev[j - 1];
    C.kappa.assign((size_t)C.N * C.N, 0.0);
    for (int cy = 0; cy < C.N; ++cy)
      for (int cx = 0; cx < C.N; ++cx)
        C.kappa[cy * C.N + cx] = average4(kappa_avg, F.kappa[(2 * cy) * F.N + 2 * cx],
                                          F.kappa[(2 * cy) * F.N + 2 * cx + 1], F.kappa[(2 * cy + 1) * F.N + 2 * cx],
                                          F.kappa[(2 * cy + 1) * F.N + 2 * cx + 1]);
  }
  for (int j = 0; j <= J; ++j) {
    assemble(X->lev[j]);
    if (j > 0) {
      build_patches(X->lev[j]);
      build_prolongation(X->lev[j], X->lev[j - 1]);
    }
  }
  // coarse inverse (bordered with the constant-pressure vector if singular)
  Level& C = X->lev[0];
  int n = C.ndof;
  std::vector<double> A0((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int e = C.A.rp[i]; e < C.A.rp[i + 1]; ++e) A0[(size_t)i * n + C.A.ci[e]] = C.A.v[e];
  std::vector<double> cvec;
  if (C.singular) {
    cvec.assign(n, 0.0);
    for (int c = 0; c < C.N * C.N; ++c) cvec[pres(C, c, 0, 0)] = 1.0 / C.N;
  }
  if (!bordered_inverse(n, A0, cvec, X->coarse_inv)) return nullptr;
  return X.release();
}

}  // namespace

// ---------------------------------------------------------------------------
// C interface for the tests (ctypes)
// ---------------------------------------------------------------------------
extern "C" {

void* orc_create(int n0, int J, int k, double mu, double sigma, const int* bc,
                 const double* kappa, int cycle, int m_fine, int colouring, int kappa_avg) {
  return create(n0, J, k, mu, sigma, bc, kappa, cycle, m_fine, colouring, kappa_avg);
}
void orc_destroy(void* p) { delete static_cast<Ctx*>(p); }

static Level& LV(void* p, int j) { return static_cast<Ctx*>(p)->lev[j]; }

int orc_ndof(void* p, int j) { return LV(p, j).ndof; }
int orc_n_u(void* p, int j) { return LV(p, j).n_u; }
int orc_N(void* p, int j) { return LV(p, j).N; }
int orc_singular(void* p, int j) { return LV(p, j).singular; }
void orc_constrained(void* p, int j, int8_t* out) {
  Level& L = LV(p, j);
  for (int i = 0; i < L.ndof; ++i) out[i] = L.cons[i];
}
void orc_kappa(void* p, int j, double* out) {
  Level& L = LV(p, j);
  std::copy(L.kappa.begin(), L.kappa.end(), out);
}
int orc_nnz(void* p, int j, int full) { return (int)(full ? LV(p, j).Afull : LV(p, j).A).v.size(); }
void orc_csr(void* p, int j, int full, int* rp, int* ci, double* v) {
  const CSR& A = full ? LV(p, j).Afull : LV(p, j).A;
  std::copy(A.rp.begin(), A.rp.end(), rp);
  std::copy(A.ci.begin(), A.ci.end(), ci);
  std::copy(A.v.begin(), A.v.end(), v);
}
void orc_apply(void* p, int j, const double* x, double* y) { LV(p, j).A.mult(x, y); }
// One row of A_j x: lets a test check a sampled output of a large operator.
double orc_apply_row(void* p, int j, int row, const double* x) { return LV(p, j).A.row_dot(row, x); }

int orc_npatch(void* p, int j) { return (int)LV(p, j).patches.size(); }
void orc_patch_info(void* p, int j, int pi, int* info) {
  const Patch& P = LV(p, j).patches[pi];
  info[0] = P.vx;
  info[1] = P.vy;
  info[2] = P.colour;
  info[3] = (int)P.dofs.size();
  info[4] = P.singular;
}
void orc_patch_dofs(void* p, int j, int pi, int* out) {
  const Patch& P = LV(p, j).patches[pi];
  std::copy(P.dofs.begin(), P.dofs.end(), out);
}
void orc_patch_inverse(void* p, int j, int pi, double* out) {
  const Patch& P = LV(p, j).patches[pi];
  std::copy(P.inv.begin(), P.inv.end(), out);
}
void orc_colour_step(void* p, int j, int colour, double* x, const double* b) {
  colour_step(LV(p, j), colour, x, b);
}
void orc_smooth(void* p, int j, int steps, double* x, const double* b) {
  for (int s = 0; s < steps; ++s) smooth_once(LV(p, j), x, b);
}
// smoother 0: multiplicative (default), 1: additive with damping omega; all levels
void orc_set_smoother(void* p, int smoother, double omega) {
  for (Level& L : static_cast<Ctx*>(p)->lev) {
    L.smoother = smoother;
    L.omega = omega;
  }
}
int orc_p_nnz(void* p, int j) { return (int)LV(p, j).P.v.size(); }
void orc_p_csr(void* p, int j, int* rp, int* ci, double* v) {
  const CSR& A = LV(p, j).P;
  std::copy(A.rp.begin(), A.rp.end(), rp);
  std::copy(A.ci.begin(), A.ci.end(), ci);
  std::copy(A.v.begin(), A.v.end(), v);
}
void orc_prolong_add(void* p, int j, const double* xc, double* xf) { prolong_add(LV(p, j), xc, xf); }
void orc_restrict(void* p, int j, const double* rf, double* bc) {
  restrict_(LV(p, j), rf, bc, LV(p, j - 1).ndof);
}
void orc_coarse_solve(void* p, const double* b, double* x) { coarse_solve(*static_cast<Ctx*>(p), b, x); }
void orc_vcycle(void* p, const double* r, double* z) {
  Ctx* X = static_cast<Ctx*>(p);
  vcycle_level(*X, X->J, r, z);
}

// Flexible GMRES(restart), right preconditioned by the V-cycle, x0 given or 0.
// Stops when the Arnoldi residual estimate is <= rtol * ||b||_2.  Returns the
// number of iterations (negative if maxit was reached); hist[i] = residual
// estimate after iteration i (relative), true_rel = ||b - A x|| / ||b||.
int orc_fgmres(void* p, const double* b, const double* x0, double* x, double rtol, int maxit,
               int restart, int precond, double* hist, double* true_rel) {
  Ctx* X = static_cast<Ctx*>(p);
  const Level& L = X->lev[X->J];
  const int n = L.ndof;
  std::vector<double> bb(b, b + n), r(n), w(n);
  if (x0) std::copy(x0, x0 + n, x);
  else std::fill(x, x + n, 0.0);
  const double bnorm = std::sqrt(dot(bb, bb));
  if (bnorm == 0.0) {
    std::fill(x, x + n, 0.0);
    *true_rel = 0.0;
    return 0;
  }
  int its = 0;
  bool conv = false;
  std::vector<std::vector<double>> V, Z;
  while (!conv && its < maxit) {
    L.A.mult(x, r.data());
    for (int i = 0; i < n; ++i) r[i] = b[i] - r[i];
    double beta = std::sqrt(dot(r, r));
    if (beta <= rtol * bnorm) { conv = true; break; }
    V.assign(1, r);
    for (auto& e : V[0]) e /= beta;
    Z.clear();
    std::vector<double> H((size_t)(restart + 1) * restart, 0.0), cs(restart), sn(restart),
        g(restart + 1, 0.0);
    g[0] = beta;
    int i = 0;
    for (; i < restart && its < maxit; ++i) {
      std::vector<double> z(n);
      if (precond) vcycle_level(*X, X->J, V[i].data(), z.data());
      else z = V[i];
      Z.push_back(z);
      L.A.mult(z.data(), w.data());
      for (int jj = 0; jj <= i; ++jj) {  // modified Gram-Schmidt
        double hji = dot(w, V[jj]);
        H[(size_t)jj * restart + i] = hji;
        for (int e = 0; e < n; ++e) w[e] -= hji * V[jj][e];
      }
      double hn = std::sqrt(dot(w, w));
      H[(size_t)(i + 1) * restart + i] = hn;
      for (int jj = 0; jj < i; ++jj) {  // previous Givens rotations
        double a = H[(size_t)jj * restart + i], c = H[(size_t)(jj + 1) * restart + i];
        H[(size_t)jj * restart + i] = cs[jj] * a + sn[jj] * c;
        H[(size_t)(jj + 1) * restart + i] = -sn[jj] * a + cs[jj] * c;
      }
      double a = H[(size_t)i * restart + i], c = H[(size_t)(i + 1) * restart + i];
      double den = std::hypot(a, c);
      cs[i] = a / den;
      sn[i] = c / den;
      H[(size_t)i * restart + i] = den;
      H[(size_t)(i + 1) * restart + i] = 0.0;
      g[i + 1] = -sn[i] * g[i];
      g[i] = cs[i] * g[i];
      if (hist) hist[its] = std::fabs(g[i + 1]) / bnorm;
      ++its;
      if (std::fabs(g[i + 1]) <= rtol * bnorm || hn == 0.0) {
        conv = true;
        ++i;
        break;
      }
      std::vector<double> v(w);
      for (auto& e : v) e /= hn;
      V.push_back(v);
    }
    // x += Z y with H y = g (upper triangular, size i)
    std::vector<double> y(i);
    for (int rr = i - 1; rr >= 0; --rr) {
      double s = g[rr];
      for (int cc = rr + 1; cc < i; ++cc) s -= H[(size_t)rr * restart + cc] * y[cc];
      y[rr] = s / H[(size_t)rr * restart + rr];
    }
    for (int jj = 0; jj < i; ++jj)
      for (int e = 0; e < n; ++e) x[e] += y[jj] * Z[jj][e];
  }
  L.A.mult(x, r.data());
  for (int i = 0; i < n; ++i) r[i] = b[i] - r[i];
  *true_rel = std::sqrt(dot(r, r)) / bnorm;
  return conv ? its : -its;
}

// Dense direct solve of A_J x = b (small meshes only); for the singular case the
// zero-mean pressure solution is returned.  Returns 0 on success.
int orc_direct_solve(void* p, const double* b, double* x) {
  Ctx* X = static_cast<Ctx*>(p);
  const Level& L = X->lev[X->J];
  const int n = L.ndof;
  const int m = L.singular ? n + 1 : n;
  std::vector<double> a((size_t)m * m, 0.0), rhs(m, 0.0);
  for (int i = 0; i < n; ++i) {
    for (int e = L.A.rp[i]; e < L.A.rp[i + 1]; ++e) a[(size_t)i * m + L.A.ci[e]] = L.A.v[e];
    rhs[i] = b[i];
  }
  if (L.singular)
    for (int c = 0; c < L.N * L.N; ++c) {
      a[(size_t)pres(L, c, 0, 0) * m + n] = 1.0;
      a[(size_t)n * m + pres(L, c, 0, 0)] = 1.0;
    }
  // Gaussian elimination with partial pivoting
  for (int c = 0; c < m; ++c) {
    int piv = c;
    for (int r = c + 1; r < m; ++r)
      if (std::fabs(a[(size_t)r * m + c]) > std::fabs(a[(size_t)piv * m + c])) piv = r;
    if (a[(size_t)piv * m + c] == 0.0) return 1;
    if (piv != c) {
      for (int j = 0; j < m; ++j) std::swap(a[(size_t)piv * m + j], a[(size_t)c * m + j]);
      std::swap(rhs[piv], rhs[c]);
    }
    for (int r = c + 1; r < m; ++r) {
      double f = a[(size_t)r * m + c] / a[(size_t)c * m + c];
      if (f == 0.0) continue;
      for (int j = c; j < m; ++j) a[(size_t)r * m + j] -= f * a[(size_t)c * m + j];
      rhs[r] -= f * rhs[c];
    }
  }
  for (int r = m - 1; r >= 0; --r) {
    double s = rhs[r];
    for (int j = r + 1; j < m; ++j) s -= a[(size_t)r * m + j] * rhs[j];
    rhs[r] = s / a[(size_t)r * m + r];
  }
  std::copy(rhs.begin(), rhs.begin() + n, x);
  return 0;
}

// Quadrature points of the right-hand-side integrals.  Cell points: N*N cells
// (c = cy*N + cx) x q*q points (index iy*q + ix) x (x, y).  Boundary points: 4
// sides (x=0, x=1, y=0, y=1) x N faces (ordered along the side) x q points x (x, y).
void orc_quad_points(int N, int k, double* cell_xy, double* face_xy) {
  const int q = k + 2;
  Rule r = gauss01(q);
  const double h = 1.0 / N;
  for (int cy = 0; cy < N; ++cy)
    for (int cx = 0; cx < N; ++cx)
      for (int iy = 0; iy < q; ++iy)
        for (int ix = 0; ix < q; ++ix) {
          size_t o = ((((size_t)cy * N + cx) * q + iy) * q + ix) * 2;
          cell_xy[o] = (cx + r.x[ix]) * h;
          cell_xy[o + 1] = (cy + r.x[iy]) * h;
        }
  for (int s = 0; s < 4; ++s)
    for (int f = 0; f < N; ++f)
      for (int i = 0; i < q; ++i) {
        size_t o = (((size_t)s * N + f) * q + i) * 2;
        double t = (f + r.x[i]) * h;
        if (s < 2) { face_xy[o] = (s == 0) ? 0.0 : 1.0; face_xy[o + 1] = t; }
        else { face_xy[o] = t; face_xy[o + 1] = (s == 2) ? 0.0 : 1.0; }
      }
}

// Right-hand side of the finest level (eq. BCh): (f, v) + 2 mu sigma_h <g, v>
// - mu <grad v n, g> on Dirichlet sides, -(s, q) in the pressure rows, the
// essential normal values on the constrained dofs and their lifting.
// f_qp: cell points x 2; s_qp: cell points (or null); g_qp: boundary points x 2
// (or null = homogeneous).
void orc_rhs(void* p, const double* f_qp, const double* s_qp, const double* g_qp, double* b) {
  Ctx* X = static_cast<Ctx*>(p);
  const Level& L = X->lev[X->J];
  const int N = L.N, q = L.k + 2;
  Rule r = gauss01(q);
  std::vector<double> bb(L.ndof, 0.0), uc(L.ndof, 0.0);
  for (int cy = 0; cy < N; ++cy)
    for (int cx = 0; cx < N; ++cx)
      for (int iy = 0; iy < q; ++iy)
        for (int ix = 0; ix < q; ++ix) {
          size_t pt = (((size_t)cy * N + cx) * q + iy) * q + ix;
          double w = r.w[ix] * r.w[iy] * L.h * L.h;
          for (int l = 0; l < L.nloc; ++l) {
            BVal bv = eval_fn(L, l, r.x[ix], r.x[iy], L.h);
            int g = global_of(L, cx, cy, l);
            if (L.loc[l].kind < 2) {
              bb[g] += w * (f_qp[pt * 2] * bv.v[0] + f_qp[pt * 2 + 1] * bv.v[1]);
            } else if (s_qp) {
              bb[g] -= w * s_qp[pt] * bv.p;
            }
          }
        }
  if (g_qp) {
    const double pen = 2.0 * L.mu * L.sigma / L.h;
    for (int s = 0; s < 4; ++s) {
      if (L.bc[s] != BC_DIRICHLET) continue;
      for (int f = 0; f < N; ++f) {
        int cx = (s == 0) ? 0 : (s == 1) ? N - 1 : f;
        int cy = (s == 2) ? 0 : (s == 3) ? N - 1 : f;
        double nrm[2] = {s == 0 ? -1.0 : s == 1 ? 1.0 : 0.0, s == 2 ? -1.0 : s == 3 ? 1.0 : 0.0};
        for (int i = 0; i < q; ++i) {
          size_t pt = ((size_t)s * N + f) * q + i;
          const double* g = &g_qp[pt * 2];
          double xi = (s == 0) ? 0.0 : (s == 1) ? 1.0 : r.x[i];
          double eta = (s == 2) ? 0.0 : (s == 3) ? 1.0 : r.x[i];
          for (int l = 0; l < 2 * L.nv; ++l) {
            BVal bv = eval_fn(L, l, xi, eta, L.h);
            int gd = global_of(L, cx, cy, l);
            double gn[2];
            for (int c = 0; c < 2; ++c) gn[c] = bv.g[c][0] * nrm[0] + bv.g[c][1] * nrm[1];
            bb[gd] += r.w[i] * L.h *
                      (pen * (g[0] * bv.v[0] + g[1] * bv.v[1]) - L.mu * (gn[0] * g[0] + gn[1] * g[1]));
          }
          // essential normal values: Legendre moments of the normal component
          for (int bdeg = 0; bdeg < L.nb; ++bdeg) {
            int gd = (s < 2) ? xface(L, s == 0 ? 0 : N, f, bdeg) : yface(L, s == 2 ? 0 : N, f, bdeg);
            double comp = (s < 2) ? g[0] : g[1];
            uc[gd] += r.w[i] * comp * Lval(bdeg, r.x[i]);
          }
        }
      }
    }
  }
  // lifting of the essential values into the free rows
  for (int i = 0; i < L.ndof; ++i) {
    if (L.cons[i]) {
      b[i] = uc[i];
      continue;
    }
    double s = 0.0;
    for (int e = L.Afull.rp[i]; e < L.Afull.rp[i + 1]; ++e)
      if (L.cons[L.Afull.ci[e]]) s += L.Afull.v[e] * uc[L.Afull.ci[e]];
    b[i] = bb[i] - s;
  }
}

// One level without hierarchy or stored matrix: rows of A x computed from the cell
// and face integrals touching each requested row (check of large results).
void* orc_level_create(int N, int k, double mu, double sigma, const int* bc, const double* kappa) {
  Level* L = new Level();
  init_level(*L, N, k, mu, sigma, bc);
  L->kappa.assign(kappa, kappa + (size_t)N * N);
  return L;
}
void orc_level_destroy(void* p) { delete static_cast<Level*>(p); }
int orc_level_ndof(void* p) { return static_cast<Level*>(p)->ndof; }

void orc_level_rows(void* p, int nrows, const int* rows, const double* x, double* out) {
  const Level& L = *static_cast<Level*>(p);
  const int N = L.N, nb = L.nb;
  const int nxf = N * (N + 1) * nb, n_int = 2 * N * (N + 1) * nb;
#pragma omp parallel for schedule(dynamic, 4)
  for (int r = 0; r < nrows; ++r) {
    const int g = rows[r];
    if (L.cons[g]) {
      out[r] = x[g];
      continue;
    }
    // cells whose basis functions can couple to dof g: its support cells
    std::vector<std::pair<int, int>> cells;
    if (g < nxf) {
      int f = g / nb, i = f % (N + 1), cy = f / (N + 1);
      if (i > 0) cells.push_back({i - 1, cy});
      if (i < N) cells.push_back({i, cy});
    } else if (g < n_int) {
      int f = (g - nxf) / nb, cx = f % N, j = f / N;
      if (j > 0) cells.push_back({cx, j - 1});
      if (j < N) cells.push_back({cx, j});
    } else if (g < L.n_u) {
      int c = (g - n_int) / (2 * L.k * nb);
      cells.push_back({c % N, c / N});
    } else {
      int c = (g - L.n_u) / L.np;
      cells.push_back({c % N, c / N});
    }
    std::vector<Trip> t;
    std::vector<std::pair<int, int>> faces;  // (vertical?, face id)
    for (auto& cc : cells) {
      cell_terms(L, cc.first, cc.second, t);
      faces.push_back({1, cc.second * (N + 1) + cc.first});
      faces.push_back({1, cc.second * (N + 1) + cc.first + 1});
      faces.push_back({0, cc.first * (N + 1) + cc.second});
      faces.push_back({0, cc.first * (N + 1) + cc.second + 1});
    }
    std::sort(faces.begin(), faces.end());
    faces.erase(std::unique(faces.begin(), faces.end()), faces.end());
    for (auto& f : faces) {
      if (f.first) one_face(L, true, f.second % (N + 1), f.second / (N + 1), t);
      else one_face(L, false, f.second % (N + 1), f.second / (N + 1), t);
    }
    double s = 0.0;
    for (auto& e : t)
      if (e.i == g && !L.cons[e.j]) s += e.v * x[e.j];
    out[r] = s;
  }
}

// Exposed 1-D helpers (for basis pins).
double orc_L(int b, double t) { return Lval(b, t); }
double orc_psi(int a, double t) { return psival(a, t); }
void orc_gauss(int q, double* x, double* w) {
  Rule r = gauss01(q);
  std::copy(r.x.begin(), r.x.end(), x);
  std::copy(r.w.begin(), r.w.end(), w);
}

}  // extern "C"
