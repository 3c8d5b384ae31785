/*
 * oracle.c -- plain FP64 CPU oracle for the symmetric interior penalty (SIPG)
 * discretisation of -div(c grad u) on a structured hexahedral brick mesh.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant with the GPU library: it has its own 1D rules, its
 * own geometry and its own quadrature loops.
 *
 * What is computed (Kronbichler & Kormann, "Fast matrix-free evaluation of
 * discontinuous Galerkin finite element operators", arXiv 1711.03590):
 *   y = A u, the operator of Sec. 2 Eq. (3) ("matvec"), for the SIPG weak form
 *   of Sec. 2 Eq. (2) ("poisson_sip"), written element by element:
 *     y_i = (grad phi_i, c grad u_h)_{Omega_e}
 *         - <grad phi_i, 1/2 [[u_h]]>_{dOmega_e}      (adjoint consistency)
 *         - <phi_i n, {{grad u_h}}>_{dOmega_e}          (primal consistency)
 *         + <phi_i n, tau [[u_h]]>_{dOmega_e}           (penalty)
 *   with {{.}}, [[.]] and the Dirichlet mirror principle u+ = -u- + 2g (g = 0)
 *   as defined at the start of Sec. 2, and every integral approximated by
 *   tensor-product Gauss quadrature on the reference cell (Sec. 2, Eq. (4)):
 *   reference gradients mapped by J^{-T}, weights multiplied by det J.
 *
 * How: every integral is evaluated point by point.  At each quadrature point
 * the value and reference gradient of u_h are formed by summing over ALL basis
 * functions of the cell (no sum factorisation, no even-odd splitting, no
 * collocation), the geometry comes from the analytic mapping, and the
 * integrand is tested against every basis function of the cell.  Cost is
 * O(n^6) per cell, which is what makes this an obviously-correct reference.
 *
 * Readings where the paper leaves a choice open (all named here once):
 *   - basis: Lagrange polynomials of degree k on the k+1 Gauss-Lobatto points;
 *     quadrature: (k+1)-point Gauss-Legendre per direction on cells and faces.
 *   - penalty tau = (k+1)^2 / h_a with h_a the unmapped cell size along the
 *     face normal axis a (the paper only asks for "sufficiently large").
 *   - Dirichlet faces: u+ = -u-, grad u+ = grad u-  (mirror of the value only).
 *   - the coefficient c multiplies all three face terms, evaluated at the face
 *     quadrature point.
 *   - the face normal and area element come from the element's own side
 *     (Nanson's formula ds = det J |J^{-T} e| w); the neighbour's gradient uses
 *     the neighbour's own Jacobian at the same physical point.
 *   - homogeneous Neumann faces contribute nothing.
 *   - Cell geometry from quadrature-point positions (problem field cellgeo = 1,
 *     SIPG only): Sec. 5 lists, as variant G2, keeping only the physical
 *     positions of the quadrature points and computing the Jacobian from them
 *     by a collocation derivative.  Reading: the cell term uses the Jacobian
 *     of the tensor-product polynomial through the n^3 Gauss-point positions
 *     (degree k per direction), evaluated at those points; the coefficient is
 *     still c at the exact point (the interpolant passes through it).  Face
 *     terms keep the map's own normals and area elements (the paper notes
 *     that faces need data of their own), and so do the load vector and the
 *     error norms.
 *   - Hermite-like basis (problem field basis = 1, degree k >= 3): the paper
 *     asks only that a face value and a face derivative each need at most two
 *     coefficients per normal line (Sec. 3, the face interpolation kernel;
 *     Sec. 4.4).  Reading: the basis dual to the k+1 functionals
 *       u(0), x_1 u'(0), u(x_2), ..., u(x_{k-2}), -x_1 u'(1), u(1)
 *     with x_m the Gauss-Lobatto points (x_1 = 1 - x_{k-1} their first
 *     interior spacing, which scales the derivative functionals like a
 *     value).  Only phi_0 is non-zero at 0 and only phi_1 has a slope there
 *     (mirrored at 1), the interior functions vanish with their slope at both
 *     ends, and phi_{k-j}(x) = phi_j(1-x).  It spans the same polynomials as
 *     the nodal basis, so the discrete solution is the same; A changes by the
 *     cell-wise change of basis.
 *
 * The same library also evaluates the second operator of the paper, the DG
 * discretisation of stationary advection with the local Lax-Friedrichs
 * (upwind) flux, Sec. 2 Eq. (1), in the element form that Algorithm 1 loops
 * over (problem field op = 1):
 *     y_i = -(grad phi_i, c u_h)_{Omega_e}
 *         + <phi_i, 1/2 (c.n)(u- + u+) + 1/2 |c.n| (u- - u+)>_{dOmega_e}
 *   with n the element's outward normal and u+ the neighbour's trace.
 *   Readings for it: the velocity c(x) is either a constant vector or the
 *   divergence-free field c = (1/2 - y, x - 1/2, 1/4) (a rotation about the
 *   cube's vertical axis with an upward drift); boundary faces take the
 *   mirror u+ = -u- (bc 0, homogeneous inflow data, as in Algorithm 1's
 *   boundary loop) or the extrapolation u+ = u- (bc 1, pure outflow).
 *
 * DoF numbering: global = cell * n^3 + i1 + n*i2 + n^2*i3, cell = cx + Nx*(cy + Ny*cz).
 * Local face numbers 0..5 = x-, x+, y-, y+, z-, z+.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_ERR_ARG 1
#define ORC_ERR_GEOM 2
#define ORC_ERR_MEM 3
#define ORC_MAXN 12

static const double ORC_PI = 3.14159265358979323846264338327950288;

typedef struct {
  int32_t ncell[3];
  double lo[3], hi[3];
  int32_t bc[6];      /* 0 = Dirichlet, 1 = homogeneous Neumann; order x-,x+,y-,y+,z-,z+ */
  int32_t degree;     /* polynomial degree k; n = k + 1 points per direction */
  int32_t map;        /* 0 = affine, 1 = x_i + a sin(2 pi X) sin(2 pi Y) sin(2 pi Z) */
  double amplitude;   /* a of the sine map */
  int32_t coef;       /* 0 = constant coef_value, 1 = 1 + 0.5 sin(pi x) cos(pi y) z */
  double coef_value;
  int32_t op;         /* 0 = SIPG Laplacian, 1 = advection with upwind flux */
  int32_t vel;        /* advection velocity: 0 = constant vel_value, 1 = (1/2 - y, x - 1/2, 1/4) */
  double vel_value[3];
  int32_t basis;      /* 0 = Lagrange on the Gauss-Lobatto points, 1 = Hermite-like (k >= 3) */
  int32_t cellgeo;    /* SIPG cell integrals: 0 = Jacobian of the map, 1 = Jacobian of its
                         interpolant through the cell's Gauss points (positions only) */
} orc_problem;

/* ------------------------------------------------------------------------ */
/* 1D polynomial data                                                        */
/* ------------------------------------------------------------------------ */

/* Legendre P_m(t), P_m'(t) on (-1,1) by the three-term (Bonnet) recurrence. */
static void legendre(int m, double t, double *p, double *dp)
{
  double p0 = 1.0, p1 = t;
  if (m == 0) { *p = 1.0; *dp = 0.0; return; }
  for (int j = 2; j <= m; ++j) {
    double p2 = ((2.0 * j - 1.0) * t * p1 - (j - 1.0) * p0) / j;
    p0 = p1;
    p1 = p2;
  }
  *p = p1;
  *dp = m * (t * p1 - p0) / (t * t - 1.0);
}

/* n-point Gauss-Legendre rule mapped to [0,1], ascending nodes. */
int orc_gauss(int n, double *x, double *w)
{
  if (n < 1 || n > 64) return ORC_ERR_ARG;
  for (int i = 0; i < n; ++i) {
    double t = cos(ORC_PI * (i + 0.75) / (n + 0.5)), p, dp;
    for (int it = 0; it < 100; ++it) {
      legendre(n, t, &p, &dp);
      double dt = p / dp;
      t -= dt;
      if (fabs(dt) < 1e-16) break;
    }
    legendre(n, t, &p, &dp);
    x[n - 1 - i] = 0.5 * (1.0 + t);
    w[n - 1 - i] = 1.0 / ((1.0 - t * t) * dp * dp); /* 2/((1-t^2)P'^2), halved for [0,1] */
  }
  return ORC_OK;
}

/* n-point Gauss-Lobatto nodes mapped to [0,1]: 0, 1 and the roots of P'_{n-1}. */
int orc_gll(int n, double *x)
{
  if (n < 2 || n > 64) return ORC_ERR_ARG;
  int k = n - 1;
  x[0] = 0.0;
  x[n - 1] = 1.0;
  for (int j = 1; j < k; ++j) {
    double t = -cos(ORC_PI * j / k), p, dp;
    for (int it = 0; it < 100; ++it) {
      legendre(k, t, &p, &dp);
      double d2p = (2.0 * t * dp - k * (k + 1.0) * p) / (1.0 - t * t);
      double dt = dp / d2p;
      t -= dt;
      if (fabs(dt) < 1e-16) break;
    }
    x[j] = 0.5 * (1.0 + t);
  }
  return ORC_OK;
}

/* Lagrange polynomial j on the given nodes, value and derivative at xi,
 * straight from the product formula. */
static double lag_val(int n, const double *nodes, int j, double xi)
{
  double v = 1.0;
  for (int m = 0; m < n; ++m)
    if (m != j) v *= (xi - nodes[m]) / (nodes[j] - nodes[m]);
  return v;
}

static double lag_der(int n, const double *nodes, int j, double xi)
{
  double s = 0.0;
  for (int l = 0; l < n; ++l) {
    if (l == j) continue;
    double p = 1.0 / (nodes[j] - nodes[l]);
    for (int m = 0; m < n; ++m)
      if (m != j && m != l) p *= (xi - nodes[m]) / (nodes[j] - nodes[m]);
    s += p;
  }
  return s;
}

int orc_lagrange(int n, const double *nodes, int j, double xi, double *val, double *der)
{
  if (n < 1 || j < 0 || j >= n) return ORC_ERR_ARG;
  *val = lag_val(n, nodes, j, xi);
  *der = lag_der(n, nodes, j, xi);
  return ORC_OK;
}

/* The Hermite-like basis written in the Lagrange basis on the n Gauss-Lobatto
 * points x: phi_j = sum_i T[i*n + j] l_i, i.e. T[i*n + j] = phi_j(x_i).  The
 * value functionals at x_0, x_2..x_{n-3}, x_{n-1} pick T's rows directly
 * (T[i*n + j] = delta_ij there); the two derivative functionals leave the
 * rows i = 1 and i = n-2 as the unknowns of a 2x2 system per j, solved by
 * Cramer's rule. */
static int hermite_table(int n, const double *x, double *T)
{
  if (n < 4 || n > ORC_MAXN) return ORC_ERR_ARG;
  const int a = 1, b = n - 2;
  const double s = x[1];
  /* slopes at 0 and at 1 of the two free Lagrange polynomials */
  const double m00 = lag_der(n, x, a, 0.0), m01 = lag_der(n, x, b, 0.0);
  const double m10 = lag_der(n, x, a, 1.0), m11 = lag_der(n, x, b, 1.0);
  const double det = m00 * m11 - m01 * m10;
  if (fabs(det) < 1e-300) return ORC_ERR_ARG;
  for (int j = 0; j < n; ++j) {
    for (int i = 0; i < n; ++i) T[i * n + j] = 0.0;
    /* required slopes phi_j'(0) = r0 and phi_j'(1) = r1, minus what the
     * fixed nodal values already give */
    double r0 = (j == a) ? 1.0 / s : 0.0;
    double r1 = (j == b) ? -1.0 / s : 0.0;
    if (j != a && j != b) {
      T[j * n + j] = 1.0;
      r0 -= lag_der(n, x, j, 0.0);
      r1 -= lag_der(n, x, j, 1.0);
    }
    T[a * n + j] = (r0 * m11 - m01 * r1) / det;
    T[b * n + j] = (m00 * r1 - r0 * m10) / det;
  }
  return ORC_OK;
}

/* 1D basis function j of the given kind (0 Lagrange on Gauss-Lobatto points,
 * 1 Hermite-like) with n functions, value and derivative at xi. */
int orc_basis1d(int n, int basis, int j, double xi, double *val, double *der)
{
  double x[ORC_MAXN], T[ORC_MAXN * ORC_MAXN];
  if (n < 2 || n > ORC_MAXN || j < 0 || j >= n || (basis != 0 && basis != 1)) return ORC_ERR_ARG;
  orc_gll(n, x);
  if (basis == 0) {
    *val = lag_val(n, x, j, xi);
    *der = lag_der(n, x, j, xi);
    return ORC_OK;
  }
  int rc = hermite_table(n, x, T);
  if (rc) return rc;
  double v = 0.0, d = 0.0;
  for (int i = 0; i < n; ++i) {
    v += T[i * n + j] * lag_val(n, x, i, xi);
    d += T[i * n + j] * lag_der(n, x, i, xi);
  }
  *val = v;
  *der = d;
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Problem context: 1D rules and basis tables at the reference points        */
/* ------------------------------------------------------------------------ */

typedef struct {
  orc_problem P;
  int n, n3;
  double h[3];
  double gll[ORC_MAXN];
  double herm[ORC_MAXN * ORC_MAXN]; /* Hermite-like basis in the Lagrange one (basis 1) */
  double gx[ORC_MAXN], gw[ORC_MAXN];
  /* cell tables at the n^3 Gauss points q = q1 + n q2 + n^2 q3:
   * val[q*n3 + i], grad[(q*n3 + i)*3 + d] */
  double *val, *grad;
  /* face tables for local face f at face point qf = q1 + n q2 (tangential
   * axes in increasing order): fval[(f*n2 + qf)*n3 + i], fgrad[...*3 + d] */
  double *fval, *fgrad;
} orc_ctx;

static void ctx_free(orc_ctx *c)
{
  free(c->val);
  free(c->grad);
  free(c->fval);
  free(c->fgrad);
}

static void tangential_axes(int a, int *t1, int *t2)
{
  *t1 = (a == 0) ? 1 : 0;
  *t2 = (a == 2) ? 1 : 2;
}

/* phi_i and its reference gradient at reference point xi (tensor product of
 * 1D Lagrange polynomials on the Gauss-Lobatto nodes, or of the Hermite-like
 * functions built from them). */
static void basis_at(const orc_ctx *c, const double xi[3], int i, double *v, double g[3])
{
  int n = c->n;
  int id[3] = {i % n, (i / n) % n, i / (n * n)};
  double l[3], dl[3];
  for (int d = 0; d < 3; ++d) {
    if (c->P.basis == 1) {
      l[d] = dl[d] = 0.0;
      for (int m = 0; m < n; ++m) {
        l[d] += c->herm[m * n + id[d]] * lag_val(n, c->gll, m, xi[d]);
        dl[d] += c->herm[m * n + id[d]] * lag_der(n, c->gll, m, xi[d]);
      }
    } else {
      l[d] = lag_val(n, c->gll, id[d], xi[d]);
      dl[d] = lag_der(n, c->gll, id[d], xi[d]);
    }
  }
  *v = l[0] * l[1] * l[2];
  g[0] = dl[0] * l[1] * l[2];
  g[1] = l[0] * dl[1] * l[2];
  g[2] = l[0] * l[1] * dl[2];
}

static void face_ref_point(const orc_ctx *c, int f, int q1, int q2, double xi[3])
{
  int a = f / 2, t1, t2;
  tangential_axes(a, &t1, &t2);
  xi[a] = (f % 2) ? 1.0 : 0.0;
  xi[t1] = c->gx[q1];
  xi[t2] = c->gx[q2];
}

static int ctx_init(orc_ctx *c, const orc_problem *P)
{
  memset(c, 0, sizeof(*c));
  c->P = *P;
  if (P->degree < 1 || P->degree + 1 > ORC_MAXN) return ORC_ERR_ARG;
  for (int d = 0; d < 3; ++d) {
    if (P->ncell[d] < 1 || !(P->hi[d] > P->lo[d])) return ORC_ERR_ARG;
    c->h[d] = (P->hi[d] - P->lo[d]) / P->ncell[d];
  }
  for (int f = 0; f < 6; ++f)
    if (P->bc[f] != 0 && P->bc[f] != 1) return ORC_ERR_ARG;
  if (P->map != 0 && P->map != 1) return ORC_ERR_ARG;
  if (P->coef != 0 && P->coef != 1) return ORC_ERR_ARG;
  if (P->op != 0 && P->op != 1) return ORC_ERR_ARG;
  if (P->vel != 0 && P->vel != 1) return ORC_ERR_ARG;
  if (P->basis != 0 && (P->basis != 1 || P->degree < 3)) return ORC_ERR_ARG;
  if (P->cellgeo != 0 && (P->cellgeo != 1 || P->op != 0)) return ORC_ERR_ARG;
  int n = P->degree + 1, n2 = n * n, n3 = n2 * n;
  c->n = n;
  c->n3 = n3;
  orc_gll(n, c->gll);
  if (P->basis == 1 && hermite_table(n, c->gll, c->herm) != ORC_OK) return ORC_ERR_ARG;
  orc_gauss(n, c->gx, c->gw);
  c->val = malloc(sizeof(double) * (size_t)n3 * n3);
  c->grad = malloc(sizeof(double) * (size_t)n3 * n3 * 3);
  c->fval = malloc(sizeof(double) * (size_t)6 * n2 * n3);
  c->fgrad = malloc(sizeof(double) * (size_t)6 * n2 * n3 * 3);
  if (!c->val || !c->grad || !c->fval || !c->fgrad) { ctx_free(c); return ORC_ERR_MEM; }
  for (int q = 0; q < n3; ++q) {
    double xi[3] = {c->gx[q % n], c->gx[(q / n) % n], c->gx[q / n2]};
    for (int i = 0; i < n3; ++i)
      basis_at(c, xi, i, &c->val[(size_t)q * n3 + i], &c->grad[((size_t)q * n3 + i) * 3]);
  }
  for (int f = 0; f < 6; ++f)
    for (int qf = 0; qf < n2; ++qf) {
      double xi[3];
      face_ref_point(c, f, qf % n, qf / n, xi);
      size_t row = (size_t)f * n2 + qf;
      for (int i = 0; i < n3; ++i)
        basis_at(c, xi, i, &c->fval[row * n3 + i], &c->fgrad[(row * n3 + i) * 3]);
    }
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Geometry and coefficient                                                  */
/* ------------------------------------------------------------------------ */

/* Physical point x and Jacobian J = dx/dxi of cell (ci) at reference xi. */
static void geom_at(const orc_ctx *c, const int ci[3], const double xi[3], double x[3], double J[3][3])
{
  const orc_problem *P = &c->P;
  double X[3], G[3][3];
  for (int d = 0; d < 3; ++d) X[d] = P->lo[d] + (ci[d] + xi[d]) * c->h[d];
  if (P->map == 0) {
    for (int i = 0; i < 3; ++i) {
      x[i] = X[i];
      for (int j = 0; j < 3; ++j) G[i][j] = (i == j) ? 1.0 : 0.0;
    }
  } else {
    double s[3], co[3], A = P->amplitude;
    for (int d = 0; d < 3; ++d) {
      s[d] = sin(2.0 * ORC_PI * X[d]);
      co[d] = cos(2.0 * ORC_PI * X[d]);
    }
    double disp = A * s[0] * s[1] * s[2];
    double ds[3] = {A * 2.0 * ORC_PI * co[0] * s[1] * s[2],
                    A * 2.0 * ORC_PI * s[0] * co[1] * s[2],
                    A * 2.0 * ORC_PI * s[0] * s[1] * co[2]};
    for (int i = 0; i < 3; ++i) {
      x[i] = X[i] + disp;
      for (int j = 0; j < 3; ++j) G[i][j] = ((i == j) ? 1.0 : 0.0) + ds[j];
    }
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) J[i][j] = G[i][j] * c->h[j];
}

/* Point x and Jacobian at Gauss point q of cell ci of the interpolant of the
 * map through the cell's n^3 Gauss points: dx_i/dxi_d = sum_m x_i(point q with
 * its index along d replaced by m) l_m'(g_{q_d}), l_m the Lagrange
 * polynomials on the n Gauss points. */
static void geom_interp_at(const orc_ctx *c, const int ci[3], int q, double x[3], double J[3][3])
{
  const int n = c->n;
  const int qi[3] = {q % n, (q / n) % n, q / (n * n)};
  const double xi[3] = {c->gx[qi[0]], c->gx[qi[1]], c->gx[qi[2]]};
  double Jmap[3][3];
  geom_at(c, ci, xi, x, Jmap);
  for (int d = 0; d < 3; ++d) {
    for (int i = 0; i < 3; ++i) J[i][d] = 0.0;
    for (int m = 0; m < n; ++m) {
      double xm_ref[3] = {xi[0], xi[1], xi[2]}, xm[3], Jm[3][3];
      xm_ref[d] = c->gx[m];
      geom_at(c, ci, xm_ref, xm, Jm);
      const double dl = lag_der(n, c->gx, m, xi[d]);
      for (int i = 0; i < 3; ++i) J[i][d] += xm[i] * dl;
    }
  }
}

/* Inverse by the adjugate; returns det. */
static double inv3(double J[3][3], double Ji[3][3])
{
  double cof[3][3];
  cof[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  cof[0][1] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  cof[0][2] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  cof[1][0] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
  cof[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
  cof[1][2] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
  cof[2][0] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
  cof[2][1] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
  cof[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  double det = J[0][0] * cof[0][0] + J[0][1] * cof[0][1] + J[0][2] * cof[0][2];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Ji[i][j] = cof[j][i] / det;
  return det;
}

/* grad_x = J^{-T} grad_xi */
static void map_grad(double Ji[3][3], const double g[3], double out[3])
{
  for (int a = 0; a < 3; ++a) out[a] = Ji[0][a] * g[0] + Ji[1][a] * g[1] + Ji[2][a] * g[2];
}

static double coef_at(const orc_ctx *c, const double x[3])
{
  if (c->P.coef == 0) return c->P.coef_value;
  return 1.0 + 0.5 * sin(ORC_PI * x[0]) * cos(ORC_PI * x[1]) * x[2];
}

/* transport velocity of the advection operator at physical point x */
static void velocity_at(const orc_ctx *c, const double x[3], double v[3])
{
  if (c->P.vel == 0) {
    for (int d = 0; d < 3; ++d) v[d] = c->P.vel_value[d];
  } else {
    v[0] = 0.5 - x[1];
    v[1] = x[0] - 0.5;
    v[2] = 0.25;
  }
}

static void cell_coords(const orc_ctx *c, int64_t e, int ci[3])
{
  const int32_t *N = c->P.ncell;
  ci[0] = (int)(e % N[0]);
  ci[1] = (int)((e / N[0]) % N[1]);
  ci[2] = (int)(e / ((int64_t)N[0] * N[1]));
}

static int64_t cell_index(const orc_ctx *c, const int ci[3])
{
  const int32_t *N = c->P.ncell;
  return ci[0] + (int64_t)N[0] * (ci[1] + (int64_t)N[1] * ci[2]);
}

/* neighbour across local face f, or -1 at the domain boundary */
static int64_t neighbour(const orc_ctx *c, int64_t e, int f)
{
  int ci[3];
  cell_coords(c, e, ci);
  int a = f / 2;
  ci[a] += (f % 2) ? 1 : -1;
  if (ci[a] < 0 || ci[a] >= c->P.ncell[a]) return -1;
  return cell_index(c, ci);
}

/* ------------------------------------------------------------------------ */
/* The element-local SIPG operator                                           */
/* ------------------------------------------------------------------------ */

/* y[i] for the test functions i of cell e (all i, or only i == only_test),
 * for the field with coefficients u_own on e and u_nb[f] on the neighbour
 * across local face f (NULL: that neighbour's coefficients are zero). */
static int local_apply(const orc_ctx *c, int64_t e, const double *u_own,
                       const double *const u_nb[6], double *y, int only_test)
{
  const int n = c->n, n2 = n * n, n3 = c->n3;
  const int ilo = only_test >= 0 ? only_test : 0;
  const int ihi = only_test >= 0 ? only_test + 1 : n3;
  int ci[3];
  cell_coords(c, e, ci);
  for (int i = ilo; i < ihi; ++i) y[i] = 0.0;

  /* cell term (grad phi_i, c grad u_h) */
  for (int q = 0; q < n3; ++q) {
    double xi[3] = {c->gx[q % n], c->gx[(q / n) % n], c->gx[q / n2]};
    double W = c->gw[q % n] * c->gw[(q / n) % n] * c->gw[q / n2];
    double x[3], J[3][3], Ji[3][3];
    if (c->P.cellgeo == 1) geom_interp_at(c, ci, q, x, J);
    else geom_at(c, ci, xi, x, J);
    double det = inv3(J, Ji);
    if (!(det > 0.0)) return ORC_ERR_GEOM;
    double gref[3] = {0.0, 0.0, 0.0}, gu[3];
    for (int j = 0; j < n3; ++j) {
      if (u_own[j] == 0.0) continue;
      const double *gj = &c->grad[((size_t)q * n3 + j) * 3];
      for (int d = 0; d < 3; ++d) gref[d] += u_own[j] * gj[d];
    }
    map_grad(Ji, gref, gu);
    double fac = coef_at(c, x) * det * W;
    for (int i = ilo; i < ihi; ++i) {
      double gi[3];
      map_grad(Ji, &c->grad[((size_t)q * n3 + i) * 3], gi);
      y[i] += fac * (gi[0] * gu[0] + gi[1] * gu[1] + gi[2] * gu[2]);
    }
  }

  /* face terms over the six faces of the element boundary */
  for (int f = 0; f < 6; ++f) {
    const int a = f / 2, side = f % 2;
    const int64_t nb = neighbour(c, e, f);
    if (nb < 0 && c->P.bc[f] == 1) continue; /* homogeneous Neumann */
    const int fo = 2 * a + (1 - side);       /* the neighbour's local face number */
    int cn[3] = {ci[0], ci[1], ci[2]};
    cn[a] += side ? 1 : -1;
    const double sgn = side ? 1.0 : -1.0;
    const double tau = (double)(c->P.degree + 1) * (c->P.degree + 1) / c->h[a];
    for (int qf = 0; qf < n2; ++qf) {
      const int q1 = qf % n, q2 = qf / n;
      double xim[3], x[3], J[3][3], Ji[3][3];
      face_ref_point(c, f, q1, q2, xim);
      geom_at(c, ci, xim, x, J);
      double det = inv3(J, Ji);
      if (!(det > 0.0)) return ORC_ERR_GEOM;
      /* outward normal n = J^{-T} e / |J^{-T} e| and area element (Nanson) */
      double N[3] = {sgn * Ji[a][0], sgn * Ji[a][1], sgn * Ji[a][2]};
      double nrm = sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
      double nv[3] = {N[0] / nrm, N[1] / nrm, N[2] / nrm};
      double ds = det * nrm * c->gw[q1] * c->gw[q2];

      const size_t rowm = (size_t)f * n2 + qf;
      double um = 0.0, grefm[3] = {0.0, 0.0, 0.0}, gm[3];
      for (int j = 0; j < n3; ++j) {
        if (u_own[j] == 0.0) continue;
        um += u_own[j] * c->fval[rowm * n3 + j];
        for (int d = 0; d < 3; ++d) grefm[d] += u_own[j] * c->fgrad[(rowm * n3 + j) * 3 + d];
      }
      map_grad(Ji, grefm, gm);
      double dnm = nv[0] * gm[0] + nv[1] * gm[1] + nv[2] * gm[2];

      double up, dnp;
      if (nb >= 0) {
        double xip[3], xp[3], Jp[3][3], Jip[3][3];
        face_ref_point(c, fo, q1, q2, xip);
        geom_at(c, cn, xip, xp, Jp);
        double detp = inv3(Jp, Jip);
        if (!(detp > 0.0)) return ORC_ERR_GEOM;
        double dx = fabs(xp[0] - x[0]) + fabs(xp[1] - x[1]) + fabs(xp[2] - x[2]);
        if (dx > 1e-12 * (1.0 + fabs(x[0]) + fabs(x[1]) + fabs(x[2]))) return ORC_ERR_GEOM;
        const size_t rowp = (size_t)fo * n2 + qf;
        const double *un = u_nb[f];
        double grefp[3] = {0.0, 0.0, 0.0}, gp[3];
        up = 0.0;
        if (un)
          for (int j = 0; j < n3; ++j) {
            if (un[j] == 0.0) continue;
            up += un[j] * c->fval[rowp * n3 + j];
            for (int d = 0; d < 3; ++d) grefp[d] += un[j] * c->fgrad[(rowp * n3 + j) * 3 + d];
          }
        map_grad(Jip, grefp, gp);
        dnp = nv[0] * gp[0] + nv[1] * gp[1] + nv[2] * gp[2];
      } else { /* Dirichlet mirror, g = 0 */
        up = -um;
        dnp = dnm;
      }
      const double jump = um - up;
      const double avg = 0.5 * (dnm + dnp);
      const double fac = coef_at(c, x) * ds;
      for (int i = ilo; i < ihi; ++i) {
        double gi[3];
        map_grad(Ji, &c->fgrad[(rowm * n3 + i) * 3], gi);
        const double dni = nv[0] * gi[0] + nv[1] * gi[1] + nv[2] * gi[2];
        const double phi = c->fval[rowm * n3 + i];
        y[i] += fac * (-0.5 * jump * dni - phi * avg + tau * phi * jump);
      }
    }
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* The element-local advection operator (Sec. 2 Eq. (1), Algorithm 1)        */
/* ------------------------------------------------------------------------ */

/* Same contract as local_apply, for the advection form.  Cell integral:
 * -sum_q (J^{-T} grad phi_i) . c u_h det J w.  Faces: at each face point the
 * upwind flux f* = 1/2 (c.n)(u- + u+) + 1/2 |c.n| (u- - u+) with the
 * element's outward normal n, tested with phi_i and the area element. */
static int local_apply_adv(const orc_ctx *c, int64_t e, const double *u_own,
                           const double *const u_nb[6], double *y, int only_test)
{
  const int n = c->n, n2 = n * n, n3 = c->n3;
  const int ilo = only_test >= 0 ? only_test : 0;
  const int ihi = only_test >= 0 ? only_test + 1 : n3;
  int ci[3];
  cell_coords(c, e, ci);
  for (int i = ilo; i < ihi; ++i) y[i] = 0.0;

  /* cell term -(grad phi_i, c u_h) */
  for (int q = 0; q < n3; ++q) {
    double xi[3] = {c->gx[q % n], c->gx[(q / n) % n], c->gx[q / n2]};
    double W = c->gw[q % n] * c->gw[(q / n) % n] * c->gw[q / n2];
    double x[3], J[3][3], Ji[3][3], vel[3];
    geom_at(c, ci, xi, x, J);
    double det = inv3(J, Ji);
    if (!(det > 0.0)) return ORC_ERR_GEOM;
    double uq = 0.0;
    for (int j = 0; j < n3; ++j) uq += u_own[j] * c->val[(size_t)q * n3 + j];
    velocity_at(c, x, vel);
    for (int i = ilo; i < ihi; ++i) {
      double gi[3];
      map_grad(Ji, &c->grad[((size_t)q * n3 + i) * 3], gi);
      y[i] -= (gi[0] * vel[0] + gi[1] * vel[1] + gi[2] * vel[2]) * uq * det * W;
    }
  }

  /* face terms: upwind flux through each of the six faces */
  for (int f = 0; f < 6; ++f) {
    const int a = f / 2, side = f % 2;
    const int64_t nb = neighbour(c, e, f);
    const int fo = 2 * a + (1 - side);
    int cn[3] = {ci[0], ci[1], ci[2]};
    cn[a] += side ? 1 : -1;
    const double sgn = side ? 1.0 : -1.0;
    for (int qf = 0; qf < n2; ++qf) {
      const int q1 = qf % n, q2 = qf / n;
      double xim[3], x[3], J[3][3], Ji[3][3], vel[3];
      face_ref_point(c, f, q1, q2, xim);
      geom_at(c, ci, xim, x, J);
      double det = inv3(J, Ji);
      if (!(det > 0.0)) return ORC_ERR_GEOM;
      double N[3] = {sgn * Ji[a][0], sgn * Ji[a][1], sgn * Ji[a][2]};
      double nrm = sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
      double nv[3] = {N[0] / nrm, N[1] / nrm, N[2] / nrm};
      double ds = det * nrm * c->gw[q1] * c->gw[q2];
      const size_t rowm = (size_t)f * n2 + qf;
      double um = 0.0;
      for (int j = 0; j < n3; ++j) um += u_own[j] * c->fval[rowm * n3 + j];
      double up;
      if (nb >= 0) {
        double xip[3], xp[3], Jp[3][3];
        face_ref_point(c, fo, q1, q2, xip);
        geom_at(c, cn, xip, xp, Jp);
        double dx = fabs(xp[0] - x[0]) + fabs(xp[1] - x[1]) + fabs(xp[2] - x[2]);
        if (dx > 1e-12 * (1.0 + fabs(x[0]) + fabs(x[1]) + fabs(x[2]))) return ORC_ERR_GEOM;
        const size_t rowp = (size_t)fo * n2 + qf;
        const double *un = u_nb[f];
        up = 0.0;
        if (un)
          for (int j = 0; j < n3; ++j) up += un[j] * c->fval[rowp * n3 + j];
      } else {
        up = (c->P.bc[f] == 0) ? -um : um;   /* mirror (inflow data 0) or outflow */
      }
      velocity_at(c, x, vel);
      const double vn = vel[0] * nv[0] + vel[1] * nv[1] + vel[2] * nv[2];
      const double flux = 0.5 * vn * (um + up) + 0.5 * fabs(vn) * (um - up);
      for (int i = ilo; i < ihi; ++i) y[i] += c->fval[rowm * n3 + i] * flux * ds;
    }
  }
  return ORC_OK;
}

/* the operator selected by the problem */
static int local_op(const orc_ctx *c, int64_t e, const double *u_own, const double *const u_nb[6], double *y,
                    int only_test)
{
  return c->P.op == 1 ? local_apply_adv(c, e, u_own, u_nb, y, only_test)
                      : local_apply(c, e, u_own, u_nb, y, only_test);
}

/* ------------------------------------------------------------------------ */
/* Exported entry points                                                     */
/* ------------------------------------------------------------------------ */

int64_t orc_n_dofs(const orc_problem *P)
{
  int64_t n = P->degree + 1;
  return (int64_t)P->ncell[0] * P->ncell[1] * P->ncell[2] * n * n * n;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* dst_rows[l*n^3 + i] = (A src) at DoF i of cell cells[l]. */
int orc_apply_cells(const orc_problem *P, const double *src, const int64_t *cells, int64_t ncells,
                    double *dst_rows)
{
  orc_ctx c;
  int rc = ctx_init(&c, P);
  if (rc) return rc;
  const int64_t total = (int64_t)P->ncell[0] * P->ncell[1] * P->ncell[2];
  int err = ORC_OK;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t l = 0; l < ncells; ++l) {
    int64_t e = cells[l];
    if (e < 0 || e >= total) { err = ORC_ERR_ARG; continue; }
    const double *unb[6];
    for (int f = 0; f < 6; ++f) {
      int64_t nb = neighbour(&c, e, f);
      unb[f] = nb >= 0 ? src + nb * c.n3 : NULL;
    }
    int r = local_op(&c, e, src + e * c.n3, unb, dst_rows + l * c.n3, -1);
    if (r) err = r;
  }
  ctx_free(&c);
  return err;
}

int orc_apply(const orc_problem *P, const double *src, double *dst)
{
  const int64_t total = (int64_t)P->ncell[0] * P->ncell[1] * P->ncell[2];
  int64_t *cells = malloc(sizeof(int64_t) * (size_t)(total > 0 ? total : 1));
  if (!cells) return ORC_ERR_MEM;
  for (int64_t e = 0; e < total; ++e) cells[e] = e;
  int rc = orc_apply_cells(P, src, cells, total, dst);
  free(cells);
  return rc;
}

/* diag_rows[l*n^3 + i] = A_ii for DoF i of cell cells[l]: the bilinear form
 * evaluated at (phi_i, phi_i). */
int orc_diag_cells(const orc_problem *P, const int64_t *cells, int64_t ncells, double *diag_rows)
{
  orc_ctx c;
  int rc = ctx_init(&c, P);
  if (rc) return rc;
  const int64_t total = (int64_t)P->ncell[0] * P->ncell[1] * P->ncell[2];
  int err = ORC_OK;
#pragma omp parallel
  {
    double *u = calloc((size_t)c.n3, sizeof(double));
    double *y = calloc((size_t)c.n3, sizeof(double));
    const double *none[6] = {NULL, NULL, NULL, NULL, NULL, NULL};
#pragma omp for schedule(dynamic, 4)
    for (int64_t l = 0; l < ncells; ++l) {
      int64_t e = cells[l];
      if (e < 0 || e >= total) { err = ORC_ERR_ARG; continue; }
      for (int i = 0; i < c.n3; ++i) {
        u[i] = 1.0;
        int r = local_op(&c, e, u, none, y, i);
        if (r) err = r;
        diag_rows[l * c.n3 + i] = y[i];
        u[i] = 0.0;
      }
    }
    free(u);
    free(y);
  }
  ctx_free(&c);
  return err;
}

/* The seven n^3 x n^3 blocks of the block row of cell e: blocks[0] couples
 * to e itself, blocks[1+f] to the neighbour across local face f (left zero at
 * the boundary).  Row-major [i][j] = d y_i / d u_j.  Built column by column
 * from unit coefficient vectors. */
int orc_block_rows(const orc_problem *P, const int64_t *cells, int64_t ncells, double *blocks)
{
  orc_ctx c;
  int rc = ctx_init(&c, P);
  if (rc) return rc;
  const int64_t total = (int64_t)P->ncell[0] * P->ncell[1] * P->ncell[2];
  const int n3 = c.n3;
  const size_t bs = (size_t)n3 * n3;
  int err = ORC_OK;
#pragma omp parallel
  {
    double *zero = calloc((size_t)n3, sizeof(double));
    double *unit = calloc((size_t)n3, sizeof(double));
    double *y = calloc((size_t)n3, sizeof(double));
#pragma omp for schedule(dynamic, 1)
    for (int64_t l = 0; l < ncells; ++l) {
      int64_t e = cells[l];
      double *B = blocks + (size_t)l * 7 * bs;
      memset(B, 0, sizeof(double) * 7 * bs);
      if (e < 0 || e >= total) { err = ORC_ERR_ARG; continue; }
      for (int blk = 0; blk < 7; ++blk) {
        if (blk > 0 && neighbour(&c, e, blk - 1) < 0) continue;
        for (int j = 0; j < n3; ++j) {
          const double *unb[6] = {NULL, NULL, NULL, NULL, NULL, NULL};
          const double *uown = zero;
          unit[j] = 1.0;
          if (blk == 0) uown = unit; else unb[blk - 1] = unit;
          int r = local_op(&c, e, uown, unb, y, -1);
          if (r) err = r;
          for (int i = 0; i < n3; ++i) B[(size_t)blk * bs + (size_t)i * n3 + j] = y[i];
          unit[j] = 0.0;
        }
      }
    }
    free(zero);
    free(unit);
    free(y);
  }
  ctx_free(&c);
  return err;
}

/* Geometry at face point (q1,q2) of local face f of cell e, evaluated from
 * the element's own side and, for interior faces, independently from the
 * neighbour's side.  out[0..2] x, out[3..5] unit outward normal, out[6] ds
 * (area element times weight), out[7..9] x from the neighbour side, out[10]
 * ds from the neighbour side (both zero at the boundary), out[11] = 1 if
 * interior. */
/* The cell Jacobian the SIPG cell term uses at Gauss point q of cell e
 * (J[3*i + d] = dx_i/dxi_d; the interpolant's for cellgeo = 1) and the map's
 * own (Jmap, same layout). */
/* The matrix-based form of y = A u on the rows of the given cells: the
 * block rows of orc_block_rows (the assembled matrix of Sec. 2 Eq. (3),
 * seven n^3 x n^3 blocks per cell) multiplied with the source, a plain
 * block-sparse matrix-vector product with one OpenMP task per block row:
 *   y_l = B[l][0] u_{cells[l]} + sum_f B[l][1+f] u_{neighbour(cells[l], f)}.
 * blocks holds ncells * 7 * n^3 * n^3 values as orc_block_rows writes them;
 * dst receives ncells * n^3 values (the rows of cells[l] at l * n^3). */
int orc_spmv_blocks(const orc_problem *P, const int64_t *cells, int64_t ncells, const double *blocks,
                    const double *src, double *dst)
{
  orc_ctx c;
  int rc = ctx_init(&c, P);
  if (rc) return rc;
  const int64_t total = (int64_t)P->ncell[0] * P->ncell[1] * P->ncell[2];
  const int n3 = c.n3;
  const size_t bs = (size_t)n3 * n3;
  int err = ORC_OK;
#pragma omp parallel for schedule(static)
  for (int64_t l = 0; l < ncells; ++l) {
    const int64_t e = cells[l];
    double *y = dst + (size_t)l * n3;
    if (e < 0 || e >= total) { err = ORC_ERR_ARG; continue; }
    for (int i = 0; i < n3; ++i) y[i] = 0.0;
    for (int blk = 0; blk < 7; ++blk) {
      const int64_t col = blk == 0 ? e : neighbour(&c, e, blk - 1);
      if (col < 0) continue;
      const double *B = blocks + ((size_t)l * 7 + (size_t)blk) * bs;
      const double *u = src + (size_t)col * n3;
      for (int i = 0; i < n3; ++i) {
        double s = 0.0;
        for (int j = 0; j < n3; ++j) s += B[(size_t)i * n3 + j] * u[j];
        y[i] += s;
      }
    }
  }
  ctx_free(&c);
  return err;
}

int orc_cell_jacobian(const orc_problem *P, int64_t e, int q, double *J, double *Jmap)
{
  orc_ctx c;
  int rc = ctx_init(&c, P);
  if (rc) return rc;
  const int64_t total = (int64_t)P->ncell[0] * P->ncell[1] * P->ncell[2];
  if (e < 0 || e >= total || q < 0 || q >= c.n3) {
    ctx_free(&c);
    return ORC_ERR_ARG;
  }
  int ci[3];
  cell_coords(&c, e, ci);
  const int n = c.n;
  const double xi[3] = {c.gx[q % n], c.gx[(q / n) % n], c.gx[q / (n * n)]};
  double x[3], Ja[3][3], Jb[3][3];
  geom_at(&c, ci, xi, x, Ja);
  if (P->cellgeo == 1) geom_interp_at(&c, ci, q, x, Jb);
  else memcpy(Jb, Ja, sizeof(Ja));
  for (int i = 0; i < 3; ++i)
    for (int d = 0; d < 3; ++d) {
      J[3 * i + d] = Jb[i][d];
      Jmap[3 * i + d] = Ja[i][d];
    }
  ctx_free(&c);
  return ORC_OK;
}

int orc_face_point(const orc_problem *P, int64_t e, int f, int q1, int q2, double *out)
{
  orc_ctx c;
  int rc = ctx_init(&c, P);
  if (rc) return rc;
  if (f < 0 || f > 5 || q1 < 0 || q2 < 0 || q1 >= c.n || q2 >= c.n) { ctx_free(&c); return ORC_ERR_ARG; }
  int ci[3], a = f / 2, side = f % 2;
  cell_coords(&c, e, ci);
  double xi[3], x[3], J[3][3], Ji[3][3];
  face_ref_point(&c, f, q1, q2, xi);
  geom_at(&c, ci, xi, x, J);
  double det = inv3(J, Ji), sgn = side ? 1.0 : -1.0;
  double N[3] = {sgn * Ji[a][0], sgn * Ji[a][1], sgn * Ji[a][2]};
  double nrm = sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
  for (int d = 0; d < 3; ++d) { out[d] = x[d]; out[3 + d] = N[d] / nrm; out[7 + d] = 0.0; }
  out[6] = det * nrm * c.gw[q1] * c.gw[q2];
  out[10] = 0.0;
  out[11] = 0.0;
  int64_t nb = neighbour(&c, e, f);
  if (nb >= 0) {
    int cn[3];
    cell_coords(&c, nb, cn);
    double xip[3], xp[3], Jp[3][3], Jip[3][3];
    face_ref_point(&c, 2 * a + (1 - side), q1, q2, xip);
    geom_at(&c, cn, xip, xp, Jp);
    double detp = inv3(Jp, Jip);
    double Np[3] = {Jip[a][0], Jip[a][1], Jip[a][2]};
    for (int d = 0; d < 3; ++d) out[7 + d] = xp[d];
    out[10] = detp * sqrt(Np[0] * Np[0] + Np[1] * Np[1] + Np[2] * Np[2]) * c.gw[q1] * c.gw[q2];
    out[11] = 1.0;
  }
  ctx_free(&c);
  return ORC_OK;
}

/* Sum of det(J) w over all cell quadrature points (the mapped volume). */
int orc_volume(const orc_problem *P, double *vol)
{
  orc_ctx c;
  int rc = ctx_init(&c, P);
  if (rc) return rc;
  const int64_t total = (int64_t)P->ncell[0] * P->ncell[1] * P->ncell[2];
  const int n = c.n, n2 = n * n;
  double s = 0.0;
#pragma omp parallel for reduction(+ : s)
  for (int64_t e = 0; e < total; ++e) {
    int ci[3];
    cell_coords(&c, e, ci);
    for (int q = 0; q < c.n3; ++q) {
      double xi[3] = {c.gx[q % n], c.gx[(q / n) % n], c.gx[q / n2]};
      double x[3], J[3][3], Ji[3][3];
      geom_at(&c, ci, xi, x, J);
      s += inv3(J, Ji) * c.gw[q % n] * c.gw[(q / n) % n] * c.gw[q / n2];
    }
  }
  *vol = s;
  ctx_free(&c);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Manufactured solution u* = sin(pi x) sin(pi y) sin(pi z)                  */
/* ------------------------------------------------------------------------ */

static void exact_u(const double x[3], double *u, double g[3])
{
  double s[3], co[3];
  for (int d = 0; d < 3; ++d) {
    s[d] = sin(ORC_PI * x[d]);
    co[d] = cos(ORC_PI * x[d]);
  }
  *u = s[0] * s[1] * s[2];
  g[0] = ORC_PI * co[0] * s[1] * s[2];
  g[1] = ORC_PI * s[0] * co[1] * s[2];
  g[2] = ORC_PI * s[0] * s[1] * co[2];
}

/* f = -div(c grad u*) = -grad c . grad u* + 3 pi^2 c u* */
static double forcing(const orc_ctx *c, const double x[3])
{
  double u, g[3];
  exact_u(x, &u, g);
  double cv = coef_at(c, x), gc[3] = {0.0, 0.0, 0.0};
  if (c->P.coef == 1) {
    gc[0] = 0.5 * ORC_PI * cos(ORC_PI * x[0]) * cos(ORC_PI * x[1]) * x[2];
    gc[1] = -0.5 * ORC_PI * sin(ORC_PI * x[0]) * sin(ORC_PI * x[1]) * x[2];
    gc[2] = 0.5 * sin(ORC_PI * x[0]) * cos(ORC_PI * x[1]);
  }
  return -(gc[0] * g[0] + gc[1] * g[1] + gc[2] * g[2]) + 3.0 * ORC_PI * ORC_PI * cv * u;
}

/* advection: f = div(c u*) = c . grad u* for the divergence-free velocities */
static double forcing_adv(const orc_ctx *c, const double x[3])
{
  double u, g[3], v[3];
  exact_u(x, &u, g);
  velocity_at(c, x, v);
  return v[0] * g[0] + v[1] * g[1] + v[2] * g[2];
}

static double forcing_op(const orc_ctx *c, const double x[3])
{
  return c->P.op == 1 ? forcing_adv(c, x) : forcing(c, x);
}

double orc_forcing_at(const orc_problem *P, const double *x)
{
  orc_ctx c;
  memset(&c, 0, sizeof(c));
  c.P = *P;
  return forcing_op(&c, x);
}

/* b_i = sum_q f(x_q) phi_i(xi_q) det J w_q  (homogeneous Dirichlet data). */
int orc_rhs(const orc_problem *P, double *b)
{
  orc_ctx c;
  int rc = ctx_init(&c, P);
  if (rc) return rc;
  const int64_t total = (int64_t)P->ncell[0] * P->ncell[1] * P->ncell[2];
  const int n = c.n, n2 = n * n, n3 = c.n3;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t e = 0; e < total; ++e) {
    int ci[3];
    cell_coords(&c, e, ci);
    double *be = b + e * n3;
    for (int i = 0; i < n3; ++i) be[i] = 0.0;
    for (int q = 0; q < n3; ++q) {
      double xi[3] = {c.gx[q % n], c.gx[(q / n) % n], c.gx[q / n2]};
      double x[3], J[3][3], Ji[3][3];
      geom_at(&c, ci, xi, x, J);
      double fac = forcing_op(&c, x) * inv3(J, Ji) * c.gw[q % n] * c.gw[(q / n) % n] * c.gw[q / n2];
      for (int i = 0; i < n3; ++i) be[i] += fac * c.val[(size_t)q * n3 + i];
    }
  }
  ctx_free(&c);
  return ORC_OK;
}

/* L2 error and broken H1-seminorm error of the DG function x against u*,
 * with an (n + extra)-point Gauss rule per direction. */
int orc_errors(const orc_problem *P, const double *x, int extra, double *l2, double *h1)
{
  orc_ctx c;
  int rc = ctx_init(&c, P);
  if (rc) return rc;
  const int n = c.n, n3 = c.n3, m = n + (extra > 0 ? extra : 0), m2 = m * m, m3 = m2 * m;
  if (m > 64) { ctx_free(&c); return ORC_ERR_ARG; }
  double gx[64], gw[64];
  orc_gauss(m, gx, gw);
  double *tv = malloc(sizeof(double) * (size_t)m3 * n3);
  double *tg = malloc(sizeof(double) * (size_t)m3 * n3 * 3);
  if (!tv || !tg) { free(tv); free(tg); ctx_free(&c); return ORC_ERR_MEM; }
  for (int q = 0; q < m3; ++q) {
    double xi[3] = {gx[q % m], gx[(q / m) % m], gx[q / m2]};
    for (int i = 0; i < n3; ++i) basis_at(&c, xi, i, &tv[(size_t)q * n3 + i], &tg[((size_t)q * n3 + i) * 3]);
  }
  const int64_t total = (int64_t)P->ncell[0] * P->ncell[1] * P->ncell[2];
  double s0 = 0.0, s1 = 0.0;
#pragma omp parallel for reduction(+ : s0, s1) schedule(dynamic, 4)
  for (int64_t e = 0; e < total; ++e) {
    int ci[3];
    cell_coords(&c, e, ci);
    const double *xe = x + e * n3;
    for (int q = 0; q < m3; ++q) {
      double xi[3] = {gx[q % m], gx[(q / m) % m], gx[q / m2]};
      double xp[3], J[3][3], Ji[3][3];
      geom_at(&c, ci, xi, xp, J);
      double det = inv3(J, Ji), W = gw[q % m] * gw[(q / m) % m] * gw[q / m2];
      double uh = 0.0, gr[3] = {0.0, 0.0, 0.0}, gh[3], ue, ge[3];
      for (int i = 0; i < n3; ++i) {
        uh += xe[i] * tv[(size_t)q * n3 + i];
        for (int d = 0; d < 3; ++d) gr[d] += xe[i] * tg[((size_t)q * n3 + i) * 3 + d];
      }
      map_grad(Ji, gr, gh);
      exact_u(xp, &ue, ge);
      s0 += (uh - ue) * (uh - ue) * det * W;
      s1 += ((gh[0] - ge[0]) * (gh[0] - ge[0]) + (gh[1] - ge[1]) * (gh[1] - ge[1]) +
             (gh[2] - ge[2]) * (gh[2] - ge[2])) * det * W;
    }
  }
  *l2 = sqrt(s0);
  *h1 = sqrt(s1);
  free(tv);
  free(tg);
  ctx_free(&c);
  return ORC_OK;
}
