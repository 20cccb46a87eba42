// Reference-element matrices by exact integration of polynomials.
//
// Derivation (Section 2.3, eq. ipbrinkman and eq. Brinkman-weak, uniform square
// cells of size h, no mapping beyond scaling):
//   * u_x basis psi_a(xi) L_b(eta); u_y basis L_b(xi) psi_a(eta): in the index
//     (a, b) both components have the same reference matrices.
//   * cell: (grad u, grad v) = Kpsi (x) I + Mpsi (x) KL  (h-independent in 2-D),
//           (u, v) = h^2 Mpsi (x) I,   (q, div u) = h * D (x) I  with D = int L psi'.
//   * face (tangential component, normal coordinate across the face): with the
//     face integral h * int_0^1 and d/dn = (1/h) d/dt the terms
//       2 mu sigma/h <[u],[v]> - mu <{du/dn},[v]> - mu <{dv/dn},[u]>
//     become mu * Mpsi (x) (2 sigma J J - G J - J G) with the trace J and normal
//     derivative average G of L_b on each side; all h-independent.
#include "refelem.hpp"

#include <cmath>
#include <stdexcept>

namespace bmg {

double Poly::operator()(double t) const {
  double s = 0.0;
  for (size_t i = c.size(); i-- > 0;) s = s * t + c[i];
  return s;
}

Poly Poly::deriv() const {
  Poly r;
  for (size_t i = 1; i < c.size(); ++i) r.c.push_back(c[i] * (double)i);
  if (r.c.empty()) r.c.push_back(0.0);
  return r;
}

Poly Poly::antideriv() const {
  Poly r;
  r.c.push_back(0.0);
  for (size_t i = 0; i < c.size(); ++i) r.c.push_back(c[i] / (double)(i + 1));
  return r;
}

Poly Poly::affine(double a, double b) const {
  // Horner in polynomials: p(a t + b)
  Poly r;
  r.c.push_back(0.0);
  Poly lin;
  lin.c = {b, a};
  for (size_t i = c.size(); i-- > 0;) {
    r = r * lin;
    r.c[0] += c[i];
  }
  return r;
}

double Poly::integral01() const {
  double s = 0.0;
  for (size_t i = 0; i < c.size(); ++i) s += c[i] / (double)(i + 1);
  return s;
}

Poly operator*(const Poly& p, const Poly& q) {
  Poly r;
  r.c.assign(p.c.size() + q.c.size() - 1, 0.0);
  for (size_t i = 0; i < p.c.size(); ++i)
    for (size_t j = 0; j < q.c.size(); ++j) r.c[i + j] += p.c[i] * q.c[j];
  return r;
}

static double binom(int n, int k) {
  double r = 1.0;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

Poly legendre01(int b) {
  // shifted Legendre: sum_j (-1)^(b+j) C(b,j) C(b+j,j) t^j, scaled to unit L2 norm
  Poly p;
  for (int j = 0; j <= b; ++j)
    p.c.push_back(((b + j) % 2 ? -1.0 : 1.0) * binom(b, j) * binom(b + j, j) * std::sqrt(2.0 * b + 1.0));
  return p;
}

Poly psi(int a) {
  Poly p;
  if (a == 0) p.c = {1.0, -1.0};
  else if (a == 1) p.c = {0.0, 1.0};
  else p = legendre01(a - 1).antideriv();
  return p;
}

RefData make_refdata(int k, double mu, double sigma) {
  RefData R;
  R.k = k;
  const int NA = k + 2, NB = k + 1, NV = NA * NB, NP = NB * NB;
  R.NA = NA;
  R.NB = NB;
  R.NV = NV;
  R.NP = NP;
  for (int b = 0; b < NB; ++b) R.L.push_back(legendre01(b));
  for (int a = 0; a < NA; ++a) R.P.push_back(psi(a));
  std::vector<Poly> dL, dP;
  for (auto& p : R.L) dL.push_back(p.deriv());
  for (auto& p : R.P) dP.push_back(p.deriv());

  auto m1 = [&](const Poly& p, const Poly& q) { return (p * q).integral01(); };
  std::vector<double> Mpsi(NA * NA), Kpsi(NA * NA), KL(NB * NB), Dm(NB * NA);
  for (int a = 0; a < NA; ++a)
    for (int c = 0; c < NA; ++c) {
      Mpsi[a * NA + c] = m1(R.P[a], R.P[c]);
      Kpsi[a * NA + c] = m1(dP[a], dP[c]);
    }
  for (int b = 0; b < NB; ++b)
    for (int c = 0; c < NB; ++c) KL[b * NB + c] = m1(dL[b], dL[c]);
  for (int q = 0; q < NB; ++q)
    for (int a = 0; a < NA; ++a) Dm[q * NA + a] = m1(R.L[q], dP[a]);

  R.Kmu.assign(NV * NV, 0.0);
  R.M.assign(NV * NV, 0.0);
  for (int a = 0; a < NA; ++a)
    for (int b = 0; b < NB; ++b)
      for (int c = 0; c < NA; ++c)
        for (int d = 0; d < NB; ++d) {
          int i = a * NB + b, j = c * NB + d;
          double stiff = Kpsi[a * NA + c] * (b == d ? 1.0 : 0.0) + Mpsi[a * NA + c] * KL[b * NB + d];
          R.Kmu[i * NV + j] = mu * stiff;
          R.M[i * NV + j] = Mpsi[a * NA + c] * (b == d ? 1.0 : 0.0);
        }
  // divergence: pressure L_pa(xi) L_pb(eta), row pb*NB + pa
  R.Dx.assign(NP * NV, 0.0);
  R.Dy.assign(NP * NV, 0.0);
  for (int pa = 0; pa < NB; ++pa)
    for (int pb = 0; pb < NB; ++pb)
      for (int a = 0; a < NA; ++a)
        for (int b = 0; b < NB; ++b) {
          int q = pb * NB + pa, v = a * NB + b;
          // u_x = psi_a(xi) L_b(eta): d/dxi psi_a, Legendre orthonormality in eta
          R.Dx[q * NV + v] = (pb == b) ? Dm[pa * NA + a] : 0.0;
          // u_y = L_b(xi) psi_a(eta)
          R.Dy[q * NV + v] = (pa == b) ? Dm[pb * NA + a] : 0.0;
        }
  // faces: traces and normal-derivative averages of L_b on each side
  std::vector<double> L0(NB), L1(NB), dL0(NB), dL1(NB);
  for (int b = 0; b < NB; ++b) {
    L0[b] = R.L[b](0.0);
    L1[b] = R.L[b](1.0);
    dL0[b] = dL[b](0.0);
    dL1[b] = dL[b](1.0);
  }
  // side 0 = lower-index cell, its face at normal coordinate 1; side 1 at 0
  auto J = [&](int side, int b) { return side == 0 ? L1[b] : -L0[b]; };
  auto G = [&](int side, int b) { return side == 0 ? 0.5 * dL1[b] : 0.5 * dL0[b]; };
  for (int t = 0; t < 2; ++t)
    for (int s = 0; s < 2; ++s) {
      std::vector<double>& F = R.F[t * 2 + s];
      F.assign(NV * NV, 0.0);
      for (int a = 0; a < NA; ++a)
        for (int b = 0; b < NB; ++b)
          for (int c = 0; c < NA; ++c)
            for (int d = 0; d < NB; ++d) {
              // test (a,b) on side t, trial (c,d) on side s
              double eta = 2.0 * sigma * J(s, d) * J(t, b) - G(s, d) * J(t, b) - G(t, b) * J(s, d);
              F[(a * NB + b) * NV + c * NB + d] = mu * Mpsi[a * NA + c] * eta;
            }
    }
  for (int e = 0; e < 2; ++e) {
    R.Nb[e].assign(NV * NV, 0.0);
    for (int a = 0; a < NA; ++a)
      for (int b = 0; b < NB; ++b)
        for (int c = 0; c < NA; ++c)
          for (int d = 0; d < NB; ++d) {
            double eta;
            if (e == 0)  // outward normal = -direction: d/dn = -(1/h) d/dt
              eta = 2.0 * sigma * L0[d] * L0[b] + dL0[d] * L0[b] + dL0[b] * L0[d];
            else
              eta = 2.0 * sigma * L1[d] * L1[b] - dL1[d] * L1[b] - dL1[b] * L1[d];
            R.Nb[e][(a * NB + b) * NV + c * NB + d] = mu * Mpsi[a * NA + c] * eta;
          }
  }
  // transfers: coarse function restricted to child interval s, t -> (s + t)/2
  for (int s = 0; s < 2; ++s) {
    R.Ppsi[s].assign(NA * NA, 0.0);
    R.PL[s].assign(NB * NB, 0.0);
    for (int a = 0; a < NA; ++a) {
      Poly g = R.P[a].affine(0.5, 0.5 * s);
      Poly dg = g.deriv();
      for (int ap = 0; ap < NA; ++ap) {
        double v;
        if (ap == 0) v = g(0.0);
        else if (ap == 1) v = g(1.0);
        else v = (dg * R.L[ap - 1]).integral01();
        R.Ppsi[s][ap * NA + a] = v;
      }
    }
    for (int b = 0; b < NB; ++b) {
      Poly g = R.L[b].affine(0.5, 0.5 * s);
      for (int bp = 0; bp < NB; ++bp) R.PL[s][bp * NB + b] = (g * R.L[bp]).integral01();
    }
  }
  return R;
}

void gauss_points(int q, double* x, double* w) {
  double s[4], ws[4];
  if (q == 2) {
    const double r = 1.0 / std::sqrt(3.0);
    s[0] = -r; s[1] = r;
    ws[0] = 1.0; ws[1] = 1.0;
  } else if (q == 3) {
    double r = std::sqrt(3.0 / 5.0);
    s[0] = -r; s[1] = 0.0; s[2] = r;
    ws[0] = 5.0 / 9.0; ws[1] = 8.0 / 9.0; ws[2] = 5.0 / 9.0;
  } else if (q == 4) {
    double a = std::sqrt(3.0 / 7.0 - 2.0 / 7.0 * std::sqrt(6.0 / 5.0));
    double b = std::sqrt(3.0 / 7.0 + 2.0 / 7.0 * std::sqrt(6.0 / 5.0));
    double wa = (18.0 + std::sqrt(30.0)) / 36.0, wb = (18.0 - std::sqrt(30.0)) / 36.0;
    s[0] = -b; s[1] = -a; s[2] = a; s[3] = b;
    ws[0] = wb; ws[1] = wa; ws[2] = wa; ws[3] = wb;
  } else {
    throw std::runtime_error("gauss_points: q must be 2, 3 or 4");
  }
  for (int i = 0; i < q; ++i) {
    x[i] = 0.5 * (1.0 + s[i]);
    w[i] = 0.5 * ws[i];
  }
}

}  // namespace bmg
