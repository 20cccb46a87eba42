// Reference-element data of the RT_k x dQ_k discretisation, computed on the host in
// FP64 by exact polynomial arithmetic (monomial coefficients on [0,1]).
#pragma once
#include <vector>

namespace bmg {

// Polynomial in t with monomial coefficients c[i] t^i.
struct Poly {
  std::vector<double> c;
  double operator()(double t) const;
  Poly deriv() const;
  Poly antideriv() const;               // vanishes at t = 0
  Poly affine(double a, double b) const;  // t -> p(a t + b)
  double integral01() const;
};
Poly operator*(const Poly& p, const Poly& q);

// One-dimensional basis (Section 2.3 spaces, canonical basis):
// L_b = sqrt(2b+1) * shifted Legendre, psi_0 = 1 - t, psi_1 = t, psi_a = int L_{a-1}.
Poly legendre01(int b);
Poly psi(int a);

// Host copy of the reference data in FP64 (layouts of Elem / Xfer in common.hpp).
struct RefData {
  int k = 0;
  int NA = 0, NB = 0, NV = 0, NP = 0;
  std::vector<double> Kmu, M, Dx, Dy, F[4], Nb[2];
  std::vector<double> Ppsi[2], PL[2];
  // 1-D values needed by the right-hand side
  std::vector<Poly> L, P;  // L_b, psi_a
};

RefData make_refdata(int k, double mu, double sigma);

// Gauss-Legendre points / weights on [0,1] with q = 3 or 4 points (closed forms).
void gauss_points(int q, double* x, double* w);

}  // namespace bmg
