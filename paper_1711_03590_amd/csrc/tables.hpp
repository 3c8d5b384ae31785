// tables.hpp -- compile-time 1D polynomial data for the sum-factorisation
// kernels (host and device).
//
// For n points per direction (degree k = n-1):
//   gx, gw   n-point Gauss-Legendre rule on [0,1] (the quadrature of Sec. 2, Eq. (4))
//   lx       n Gauss-Lobatto points on [0,1] (the nodal basis phi_j)
//   S        S[q][j]   = phi_j(gx[q])       basis change to the quadrature points
//                                            (the S_i matrices of Sec. 2, Eq. (5)-(6))
//   D        D[q][j]   = phi_j'(gx[q])      (D_i of Eq. (5), D = Dco S)
//   Dco      Dco[q][j] = ell_j'(gx[q])      collocation derivative: ell_j are the
//                                            Lagrange polynomials on the Gauss points (Eq. (6))
//   L0, L1   ell_j(0), ell_j(1)             face values from quadrature-point data
//   dL0, dL1 ell_j'(0), ell_j'(1)           face normal derivatives from quadrature-point data
//   F0, F1   phi_j'(0), phi_j'(1)           D_f of Eq. (7) on the nodal basis (S_f is the
//                                            unit row: Gauss-Lobatto nodes sit on the faces)
//
// Everything is computed by constant evaluation, so the kernels see the
// entries as literals.  Nodes come from Newton's method on the Legendre
// recurrence; Lagrange data from barycentric weights.
#pragma once

namespace dgk {

constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double c_abs(double x) { return x < 0 ? -x : x; }

constexpr double c_cos(double x)
{
  while (x > kPi) x -= 2.0 * kPi;
  while (x < -kPi) x += 2.0 * kPi;
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 40; ++k) {
    term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}

// P_m(t) and P_m'(t) on (-1,1)
struct LegPair {
  double p, dp;
};
constexpr LegPair legendre_pair(int m, double t)
{
  if (m == 0) return {1.0, 0.0};
  double pm1 = 1.0, p = t;
  for (int j = 2; j <= m; ++j) {
    const double pn = ((2.0 * j - 1.0) * t * p - (j - 1.0) * pm1) / j;
    pm1 = p;
    p = pn;
  }
  return {p, m * (t * p - pm1) / (t * t - 1.0)};
}

template <int N>
struct Tables {
  double gx[N], gw[N], lx[N];
  double S[N][N], D[N][N], Dco[N][N];
  double L0[N], L1[N], dL0[N], dL1[N];
  double F0[N], F1[N];
};

// barycentric weights lambda_j = 1 / prod_{m != j} (x_j - x_m)
template <int N>
constexpr void bary_weights(const double (&x)[N], double (&lam)[N])
{
  for (int j = 0; j < N; ++j) {
    double p = 1.0;
    for (int m = 0; m < N; ++m)
      if (m != j) p *= (x[j] - x[m]);
    lam[j] = 1.0 / p;
  }
}

// value and derivative of every Lagrange polynomial on nodes x at point xi
template <int N>
constexpr void lagrange_at(const double (&x)[N], const double (&lam)[N], double xi,
                           double (&val)[N], double (&der)[N])
{
  for (int j = 0; j < N; ++j) {
    double v = lam[j], d = 0.0;
    for (int m = 0; m < N; ++m) {
      if (m == j) continue;
      // d/dxi of prod: product rule accumulated alongside the value
      d = d * (xi - x[m]) + v;
      v *= (xi - x[m]);
    }
    val[j] = v;
    der[j] = d;
  }
}

template <int N>
constexpr Tables<N> make_tables()
{
  Tables<N> T{};
  // Gauss-Legendre: roots of P_N, Newton from the cosine guesses
  for (int i = 0; i < N; ++i) {
    double t = c_cos(kPi * (i + 0.75) / (N + 0.5));
    for (int it = 0; it < 60; ++it) {
      const LegPair L = legendre_pair(N, t);
      const double dt = L.p / L.dp;
      t -= dt;
      if (c_abs(dt) < 1e-17) break;
    }
    const LegPair L = legendre_pair(N, t);
    T.gx[N - 1 - i] = 0.5 * (1.0 + t);
    T.gw[N - 1 - i] = 1.0 / ((1.0 - t * t) * L.dp * L.dp);
  }
  // Gauss-Lobatto: endpoints and the roots of P'_{N-1}
  T.lx[0] = 0.0;
  T.lx[N - 1] = 1.0;
  const int k = N - 1;
  for (int j = 1; j < k; ++j) {
    double t = -c_cos(kPi * j / k);
    for (int it = 0; it < 60; ++it) {
      const LegPair L = legendre_pair(k, t);
      const double d2 = (2.0 * t * L.dp - k * (k + 1.0) * L.p) / (1.0 - t * t);
      const double dt = L.dp / d2;
      t -= dt;
      if (c_abs(dt) < 1e-17) break;
    }
    T.lx[j] = 0.5 * (1.0 + t);
  }
  // symmetrise (both rules are symmetric about 1/2)
  for (int i = 0; i < N / 2; ++i) {
    const double a = 0.5 * (T.gx[i] + 1.0 - T.gx[N - 1 - i]);
    T.gx[i] = a;
    T.gx[N - 1 - i] = 1.0 - a;
    const double w = 0.5 * (T.gw[i] + T.gw[N - 1 - i]);
    T.gw[i] = w;
    T.gw[N - 1 - i] = w;
    const double b = 0.5 * (T.lx[i] + 1.0 - T.lx[N - 1 - i]);
    T.lx[i] = b;
    T.lx[N - 1 - i] = 1.0 - b;
  }
  if (N % 2 == 1) {
    T.gx[N / 2] = 0.5;
    T.lx[N / 2] = 0.5;
  }
  double lamL[N]{}, lamG[N]{};
  bary_weights<N>(T.lx, lamL);
  bary_weights<N>(T.gx, lamG);
  for (int q = 0; q < N; ++q) {
    double v[N]{}, d[N]{};
    lagrange_at<N>(T.lx, lamL, T.gx[q], v, d);
    for (int j = 0; j < N; ++j) {
      T.S[q][j] = v[j];
      T.D[q][j] = d[j];
    }
  }
  // collocation derivative on the Gauss points: off-diagonal from the
  // barycentric formula, diagonal from the zero row sum (derivative of 1)
  for (int q = 0; q < N; ++q) {
    double s = 0.0;
    for (int j = 0; j < N; ++j) {
      if (j == q) continue;
      T.Dco[q][j] = (lamG[j] / lamG[q]) / (T.gx[q] - T.gx[j]);
      s += T.Dco[q][j];
    }
    T.Dco[q][q] = -s;
  }
  {
    double v[N]{}, d[N]{};
    lagrange_at<N>(T.gx, lamG, 0.0, v, d);
    for (int j = 0; j < N; ++j) { T.L0[j] = v[j]; T.dL0[j] = d[j]; }
    lagrange_at<N>(T.gx, lamG, 1.0, v, d);
    for (int j = 0; j < N; ++j) { T.L1[j] = v[j]; T.dL1[j] = d[j]; }
    lagrange_at<N>(T.lx, lamL, 0.0, v, d);
    for (int j = 0; j < N; ++j) T.F0[j] = d[j];
    lagrange_at<N>(T.lx, lamL, 1.0, v, d);
    for (int j = 0; j < N; ++j) T.F1[j] = d[j];
  }
  return T;
}

// The two bases of the SIPG operator, as 1D tables:
//   S[q][j] = phi_j(gx[q]), D[q][j] = phi_j'(gx[q]),
//   V0, V1  phi_j(0), phi_j(1)      S_f of Eq. (7) at the two ends
//   F0, F1  phi_j'(0), phi_j'(1)    D_f of Eq. (7) at the two ends
//   C       phi_j = sum_i C[i][j] l_i with l_i the Lagrange polynomials on the
//           Gauss-Lobatto points (the identity for the nodal basis)
// BASIS_NODAL: Lagrange on the Gauss-Lobatto points (face values from one
// node per normal line, face derivatives from all N).
// BASIS_HERMITE (N >= 4): the Hermite-like basis dual to the functionals
//   u(0), s u'(0), u(lx[2]), ..., u(lx[N-3]), -s u'(1), u(1),   s = lx[1],
// so that a face value needs one coefficient per normal line and a face
// derivative one more (phi_0, phi_1 at 0; phi_{N-1}, phi_{N-2} at 1), which
// is what a Hermite-type basis buys for the face kernels (Sec. 3, Eq. (7)).
enum : int { BASIS_NODAL = 0, BASIS_HERMITE = 1 };

template <int N>
struct BasisTables {
  double S[N][N], D[N][N];
  double V0[N], V1[N], F0[N], F1[N];
  double C[N][N];
};

template <int N>
constexpr BasisTables<N> make_basis(int basis)
{
  const Tables<N> T = make_tables<N>();
  BasisTables<N> B{};
  if (basis == BASIS_NODAL || N < 4) {
    for (int q = 0; q < N; ++q)
      for (int j = 0; j < N; ++j) {
        B.S[q][j] = T.S[q][j];
        B.D[q][j] = T.D[q][j];
        B.C[q][j] = (q == j) ? 1.0 : 0.0;
      }
    for (int j = 0; j < N; ++j) {
      B.V0[j] = (j == 0) ? 1.0 : 0.0;
      B.V1[j] = (j == N - 1) ? 1.0 : 0.0;
      B.F0[j] = T.F0[j];
      B.F1[j] = T.F1[j];
    }
    return B;
  }
  // functional m applied to Lagrange polynomial i: G[m][i]; C = G^{-1}
  const double s = T.lx[1];
  double G[N][N]{}, I[N][N]{};
  for (int m = 0; m < N; ++m) {
    for (int i = 0; i < N; ++i) {
      if (m == 1) G[m][i] = s * T.F0[i];
      else if (m == N - 2) G[m][i] = -s * T.F1[i];
      else G[m][i] = (m == i) ? 1.0 : 0.0;
      I[m][i] = (m == i) ? 1.0 : 0.0;
    }
  }
  // Gauss-Jordan elimination with partial pivoting
  for (int c = 0; c < N; ++c) {
    int p = c;
    for (int r = c + 1; r < N; ++r)
      if (c_abs(G[r][c]) > c_abs(G[p][c])) p = r;
    for (int k = 0; k < N; ++k) {
      const double a = G[c][k], b = I[c][k];
      G[c][k] = G[p][k];
      I[c][k] = I[p][k];
      G[p][k] = a;
      I[p][k] = b;
    }
    const double piv = G[c][c];
    for (int k = 0; k < N; ++k) {
      G[c][k] /= piv;
      I[c][k] /= piv;
    }
    for (int r = 0; r < N; ++r) {
      if (r == c) continue;
      const double f = G[r][c];
      for (int k = 0; k < N; ++k) {
        G[r][k] -= f * G[c][k];
        I[r][k] -= f * I[c][k];
      }
    }
  }
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) B.C[i][j] = I[i][j];
  for (int q = 0; q < N; ++q)
    for (int j = 0; j < N; ++j) {
      double sv = 0.0, dv = 0.0;
      for (int i = 0; i < N; ++i) {
        sv += T.S[q][i] * B.C[i][j];
        dv += T.D[q][i] * B.C[i][j];
      }
      B.S[q][j] = sv;
      B.D[q][j] = dv;
    }
  // the end data are the defining functionals themselves, kept exact so
  // that the kernels skip the zero entries
  for (int j = 0; j < N; ++j) {
    B.V0[j] = (j == 0) ? 1.0 : 0.0;
    B.V1[j] = (j == N - 1) ? 1.0 : 0.0;
    B.F0[j] = (j == 1) ? 1.0 / s : 0.0;
    B.F1[j] = (j == N - 2) ? -1.0 / s : 0.0;
  }
  return B;
}

// Even-odd split of a centro-(skew-)symmetric N x N matrix M with
// M[N-1-i][N-1-j] = sym * M[i][j] (Sec. 3.3, Eq. (8)):
//   E[i][j] = (M[i][j] + M[i][N-1-j]) / 2,  O[i][j] = (M[i][j] - M[i][N-1-j]) / 2
// for i < ceil(N/2), j < N/2, and the middle column Mid[i] = M[i][N/2] for odd N.
template <int N>
struct EvenOdd {
  double E[(N + 1) / 2][N / 2 > 0 ? N / 2 : 1];
  double O[(N + 1) / 2][N / 2 > 0 ? N / 2 : 1];
  double Mid[(N + 1) / 2];
};

template <int N>
constexpr EvenOdd<N> make_even_odd(const double (&M)[N][N], bool transpose)
{
  EvenOdd<N> R{};
  for (int i = 0; i < (N + 1) / 2; ++i) {
    for (int j = 0; j < N / 2; ++j) {
      const double a = transpose ? M[j][i] : M[i][j];
      const double b = transpose ? M[N - 1 - j][i] : M[i][N - 1 - j];
      R.E[i][j] = 0.5 * (a + b);
      R.O[i][j] = 0.5 * (a - b);
    }
    R.Mid[i] = (N % 2 == 1) ? (transpose ? M[N / 2][i] : M[i][N / 2]) : 0.0;
  }
  return R;
}

}  // namespace dgk
