// kernels.hpp -- the fused matrix-free SIPG apply and the diagonal kernel,
// templated on the number of 1D points N, the number type and the geometry
// representation.  One translation unit per N instantiates them.
//
// Operator: y = A u (Sec. 2, Eq. (3)) for the SIPG form of Sec. 2, Eq. (2),
// evaluated cell by cell.  Each workgroup owns B = 256 / N^2 cells and maps
// one thread to one 1D line of each cell (N^2 lines per sweep direction).
// Per cell, in one pass (Algorithm 1 steps (ii)-(iv) fused, Design Choice 2):
//   (a) gather the cell's N^3 coefficients into LDS (coalesced block copy);
//   (b) basis change to the Gauss points, S x S x S, then the collocation
//       derivative Dco along x, y, z (Sec. 2, Eq. (6)), every 1D matvec done
//       with the even-odd decomposition (Sec. 3.3, Eq. (8));
//   (c) own-side traces of all six faces: values and reference gradients at
//       the face points, read off the quadrature-point data with the Gauss
//       Lagrange end values (face-normal interpolation of Eq. (7) on the
//       collocation basis: the tangential directions are already at the
//       face's Gauss points);
//   (d) cell quadrature-point operation (Algorithm 1 step (c)):
//       t = J^{-1} (c det J w) J^{-T} grad_xi u, then the transposed collocation
//       derivative sums the three components into the residual;
//   (e) per face direction: the neighbour's trace from its Gauss-Lobatto
//       coefficients (value = end node, normal derivative by D_f of Eq. (7)),
//       then a 2D basis change S x S (plus D for the tangential derivative)
//       to the face Gauss points; numerical flux of Eq. (2) with the stored
//       normal-times-inverse-Jacobian j (Design Choice 5); own-side
//       integration back onto the quadrature-point residual;
//   (f) transposed basis change S^T x S^T x S^T and one coalesced write of
//       the cell's dst block (cells set, never add: Sec. 2.1).
// No atomics: every dst entry is written by exactly one thread, so the
// result is deterministic.  Neighbour blocks are re-read from L2/MALL.
#pragma once

#include "dg_internal.hpp"
#include "tables.hpp"

namespace dgk {

template <int N>
inline constexpr Tables<N> kTab = make_tables<N>();
template <int N>
inline constexpr EvenOdd<N> kEoS = make_even_odd<N>(kTab<N>.S, false);
template <int N>
inline constexpr EvenOdd<N> kEoSt = make_even_odd<N>(kTab<N>.S, true);
template <int N>
inline constexpr EvenOdd<N> kEoDco = make_even_odd<N>(kTab<N>.Dco, false);
template <int N>
inline constexpr EvenOdd<N> kEoDcot = make_even_odd<N>(kTab<N>.Dco, true);

enum : int { M_S = 0, M_ST = 1, M_DCO = 2, M_DCOT = 3 };

template <int N, int M>
__device__ __forceinline__ constexpr double eo_E(int i, int j)
{
  if constexpr (M == M_S) return kEoS<N>.E[i][j];
  else if constexpr (M == M_ST) return kEoSt<N>.E[i][j];
  else if constexpr (M == M_DCO) return kEoDco<N>.E[i][j];
  else return kEoDcot<N>.E[i][j];
}
template <int N, int M>
__device__ __forceinline__ constexpr double eo_O(int i, int j)
{
  if constexpr (M == M_S) return kEoS<N>.O[i][j];
  else if constexpr (M == M_ST) return kEoSt<N>.O[i][j];
  else if constexpr (M == M_DCO) return kEoDco<N>.O[i][j];
  else return kEoDcot<N>.O[i][j];
}
template <int N, int M>
__device__ __forceinline__ constexpr double eo_Mid(int i)
{
  if constexpr (M == M_S) return kEoS<N>.Mid[i];
  else if constexpr (M == M_ST) return kEoSt<N>.Mid[i];
  else if constexpr (M == M_DCO) return kEoDco<N>.Mid[i];
  else return kEoDcot<N>.Mid[i];
}

// out = M in for one line of N values, M one of S, S^T (centro-symmetric) or
// Dco, Dco^T (centro-skew-symmetric), by the even-odd decomposition:
// about N^2/2 multiply-adds instead of N^2.
template <int N, int M, typename Real>
__device__ __forceinline__ void eo_apply(const Real (&in)[N], Real (&out)[N])
{
  constexpr int H = N / 2;
  constexpr bool sym = (M == M_S || M == M_ST);
  Real e[H > 0 ? H : 1], o[H > 0 ? H : 1];
#pragma unroll
  for (int j = 0; j < H; ++j) {
    e[j] = in[j] + in[N - 1 - j];
    o[j] = in[j] - in[N - 1 - j];
  }
#pragma unroll
  for (int i = 0; i < H; ++i) {
    Real se = Real(eo_E<N, M>(i, 0)) * e[0];
    Real so = Real(eo_O<N, M>(i, 0)) * o[0];
#pragma unroll
    for (int j = 1; j < H; ++j) {
      se = fma(Real(eo_E<N, M>(i, j)), e[j], se);
      so = fma(Real(eo_O<N, M>(i, j)), o[j], so);
    }
    if constexpr (N % 2 == 1) se = fma(Real(eo_Mid<N, M>(i)), in[H], se);
    out[i] = se + so;
    out[N - 1 - i] = sym ? se - so : so - se;
  }
  if constexpr (N % 2 == 1) {
    if constexpr (sym) {
      Real s = Real(eo_Mid<N, M>(H)) * in[H];
#pragma unroll
      for (int j = 0; j < H; ++j) s = fma(Real(eo_E<N, M>(H, j)), e[j], s);
      out[H] = s;
    } else {
      Real s = Real(0);
#pragma unroll
      for (int j = 0; j < H; ++j) s = fma(Real(eo_O<N, M>(H, j)), o[j], s);
      out[H] = s;
    }
  }
}

// line l of direction A within a cell block (x fastest): l = p1 + N p2 with
// p1, p2 the coordinates along the two other axes in increasing order.
template <int N, int A>
__device__ __forceinline__ int line_base(int l)
{
  if constexpr (A == 0) return l * N;
  else if constexpr (A == 1) return (l % N) + (l / N) * N * N;
  else return l;
}
template <int N, int A>
inline constexpr int kStride = (A == 0) ? 1 : (A == 1 ? N : N * N);

template <int N, int A, typename Real>
__device__ __forceinline__ void load_line(const Real *buf, int l, Real (&v)[N])
{
  const int b = line_base<N, A>(l);
#pragma unroll
  for (int m = 0; m < N; ++m) v[m] = buf[b + m * kStride<N, A>];
}
template <int N, int A, typename Real>
__device__ __forceinline__ void store_line(Real *buf, int l, const Real (&v)[N])
{
  const int b = line_base<N, A>(l);
#pragma unroll
  for (int m = 0; m < N; ++m) buf[b + m * kStride<N, A>] = v[m];
}
template <int N, int A, int M, typename Real>
__device__ __forceinline__ void sweep(const Real *in, Real *out, int l)
{
  Real v[N], r[N];
  load_line<N, A>(in, l, v);
  eo_apply<N, M>(v, r);
  store_line<N, A>(out, l, r);
}

// sum_m L[m] v[m] for the two ends at once (L1[m] = L0[N-1-m] by symmetry)
template <int N, typename Real>
__device__ __forceinline__ void end_values(const Real (&v)[N], Real &lo, Real &hi)
{
  constexpr const auto &T = kTab<N>;
  Real a = Real(T.L0[0]) * v[0], b = Real(T.L1[0]) * v[0];
#pragma unroll
  for (int m = 1; m < N; ++m) {
    a = fma(Real(T.L0[m]), v[m], a);
    b = fma(Real(T.L1[m]), v[m], b);
  }
  lo = a;
  hi = b;
}

// consecutive workgroups are dispatched round-robin over the 8 XCDs; give
// each XCD a contiguous range of cell batches so that neighbour re-reads hit
// that XCD's L2
__device__ __forceinline__ int xcd_remap(int b, int G)
{
  constexpr int X = 8;
  const int q = G / X, r = G % X;
  const int xcd = b % X, k = b / X;
  return (xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q) + k;
}

template <int N>
struct Blocking {
  static constexpr int N2 = N * N, N3 = N2 * N;
  static constexpr int B = 256 / N2;         // cells per workgroup
  static constexpr int NT = B * N2;          // active threads
  static constexpr int WSZ = (3 * N3 > 14 * N2) ? 3 * N3 : 14 * N2;  // gradient / face scratch per cell
};

// face index of the face of cell ci on side s of direction A
template <int A>
__device__ __forceinline__ int64_t face_id(const int (&nc)[3], const int (&ci)[3], int s)
{
  int p[3] = {ci[0], ci[1], ci[2]};
  int m[3] = {nc[0], nc[1], nc[2]};
  p[A] += s;
  m[A] += 1;
  return p[0] + (int64_t)m[0] * (p[1] + (int64_t)m[1] * p[2]);
}

// Face terms of direction A for the cell owned by this thread's group.
// tr[s][0..3]: own value and reference gradient (x,y,z) at face point l of
// the face on side s (0: xi_A = 0, 1: xi_A = 1).
template <int N, typename Real, int GK, int A>
__device__ __forceinline__ void face_direction(const OpView<Real> &op, const Real *__restrict__ src,
                                               Real *Q, Real *W, int l, int cell, const int (&ci)[3],
                                               bool act, bool valid, const Real (&tr)[2][4])
{
  constexpr int N2 = N * N, N3 = N2 * N;
  constexpr int t1 = (A == 0) ? 1 : 0, t2 = (A == 2) ? 1 : 2;
  constexpr const auto &T = kTab<N>;
  Real *X = W;            // [side][value, normal derivative][N2] at Gauss-Lobatto face nodes
  Real *Y = W + 4 * N2;   // [side][S u, D u, S d][N2] after the sweep along t1
  Real *Z = W + 10 * N2;  // [side][tg_t1, tg_t2][N2]
  const int64_t cstride = (A == 0) ? 1 : (A == 1 ? (int64_t)op.ncell[0] : (int64_t)op.ncell[0] * op.ncell[1]);
  bool interior[2] = {false, false};
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int cn = ci[A] + (s ? 1 : -1);
    interior[s] = valid && cn >= 0 && cn < op.ncell[A];
  }
  // (1) neighbour traces at the Gauss-Lobatto nodes of the shared face
  if (act) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      Real val = Real(0), der = Real(0);
      if (interior[s]) {
        const Real *nb = src + (int64_t)(cell + (s ? cstride : -cstride)) * N3;
        Real v[N];
        load_line<N, A>(nb, l, v);
        if (s == 0) {  // neighbour below: shared face is its xi_A = 1 side
          val = v[N - 1];
          der = Real(T.F1[0]) * v[0];
#pragma unroll
          for (int m = 1; m < N; ++m) der = fma(Real(T.F1[m]), v[m], der);
        } else {       // neighbour above: its xi_A = 0 side
          val = v[0];
          der = Real(T.F0[0]) * v[0];
#pragma unroll
          for (int m = 1; m < N; ++m) der = fma(Real(T.F0[m]), v[m], der);
        }
      }
      X[(2 * s) * N2 + l] = val;
      X[(2 * s + 1) * N2 + l] = der;
    }
  }
  __syncthreads();
  // (2) sweep along t1: S and D on the values, S on the normal derivatives
  if (act) {
    const int q1 = l % N, p2 = l / N;
    Real srow[N], drow[N];
#pragma unroll
    for (int m = 0; m < N; ++m) {
      srow[m] = Real(0);
      drow[m] = Real(0);
#pragma unroll
      for (int q = 0; q < N; ++q)
        if (q == q1) { srow[m] = Real(T.S[q][m]); drow[m] = Real(T.D[q][m]); }
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const Real *xv = X + (2 * s) * N2 + N * p2;
      const Real *xd = X + (2 * s + 1) * N2 + N * p2;
      Real su = Real(0), du = Real(0), sd = Real(0);
#pragma unroll
      for (int m = 0; m < N; ++m) {
        su = fma(srow[m], xv[m], su);
        du = fma(drow[m], xv[m], du);
        sd = fma(srow[m], xd[m], sd);
      }
      Y[(3 * s) * N2 + l] = su;
      Y[(3 * s + 1) * N2 + l] = du;
      Y[(3 * s + 2) * N2 + l] = sd;
    }
  }
  __syncthreads();
  // (3) sweep along t2, numerical flux at face point l
  Real tv[2] = {Real(0), Real(0)}, tga[2] = {Real(0), Real(0)};
  if (act) {
    const int q1 = l % N, q2 = l / N;
    Real srow[N], drow[N];
#pragma unroll
    for (int m = 0; m < N; ++m) {
      srow[m] = Real(0);
      drow[m] = Real(0);
#pragma unroll
      for (int q = 0; q < N; ++q)
        if (q == q2) { srow[m] = Real(T.S[q][m]); drow[m] = Real(T.D[q][m]); }
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      Real up = Real(0), gp[3] = {Real(0), Real(0), Real(0)};
      {
        const Real *y0 = Y + (3 * s) * N2 + q1;
        const Real *y1 = Y + (3 * s + 1) * N2 + q1;
        const Real *y2 = Y + (3 * s + 2) * N2 + q1;
#pragma unroll
        for (int m = 0; m < N; ++m) {
          up = fma(srow[m], y0[N * m], up);
          gp[t2] = fma(drow[m], y0[N * m], gp[t2]);
          gp[t1] = fma(srow[m], y1[N * m], gp[t1]);
          gp[A] = fma(srow[m], y2[N * m], gp[A]);
        }
      }
      // geometry at this face point (normal of direction +e_A)
      Real j[3] = {Real(0), Real(0), Real(0)}, cds = Real(0);
      if (valid) {
        if constexpr (GK == CURVED) {
          const int64_t f = face_id<A>(op.ncell, ci, s) * N2 + l;
          const Real *fg = op.g.face[A];
          const int64_t fs = op.g.face_stride[A];
          j[0] = fg[f];
          j[1] = fg[fs + f];
          j[2] = fg[2 * fs + f];
          cds = fg[3 * fs + f];
        } else if constexpr (GK == AFFINE_VAR) {
          const int64_t f = face_id<A>(op.ncell, ci, s) * N2 + l;
          j[A] = op.inv_h[A];
          cds = op.g.face[A][f];
        } else {
          j[A] = op.inv_h[A];
          Real w1 = Real(0), w2 = Real(0);
#pragma unroll
          for (int q = 0; q < N; ++q) {
            if (q == q1) w1 = Real(T.gw[q]);
            if (q == q2) w2 = Real(T.gw[q]);
          }
          cds = op.c_area[A] * w1 * w2;
        }
      }
      const Real sg = s ? Real(1) : Real(-1);
      const Real je[3] = {sg * j[0], sg * j[1], sg * j[2]};
      const Real um = tr[s][0];
      const Real dnm = je[0] * tr[s][1] + je[1] * tr[s][2] + je[2] * tr[s][3];
      Real uplus, dnp;
      if (interior[s]) {
        uplus = up;
        dnp = je[0] * gp[0] + je[1] * gp[1] + je[2] * gp[2];
      } else {  // boundary: Dirichlet mirror; Neumann contributes nothing
        uplus = -um;
        dnp = dnm;
        if (op.bc[2 * A + s] != 0) cds = Real(0);
      }
      const Real jump = um - uplus;
      const Real avg = Real(0.5) * (dnm + dnp);
      tv[s] = cds * (op.tau[A] * jump - avg);
      const Real gfac = Real(-0.5) * cds * jump;
      tga[s] = gfac * je[A];
      Z[(2 * s) * N2 + l] = gfac * je[t1];
      Z[(2 * s + 1) * N2 + l] = gfac * je[t2];
    }
  }
  __syncthreads();
  // (4) transposed tangential collocation derivatives of the gradient-test
  // terms, then add the face contributions along this thread's normal line
  if (act) {
    const int p1 = l % N, p2 = l / N;
    Real w[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      Real acc = tv[s];
      const Real *z1 = Z + (2 * s) * N2 + N * p2;
      const Real *z2 = Z + (2 * s + 1) * N2 + p1;
#pragma unroll
      for (int q = 0; q < N; ++q) {
        Real d1 = Real(0), d2 = Real(0);
#pragma unroll
        for (int r = 0; r < N; ++r) {
          if (r == p1) d1 = Real(T.Dco[q][r]);
          if (r == p2) d2 = Real(T.Dco[q][r]);
        }
        acc = fma(d1, z1[q], acc);
        acc = fma(d2, z2[N * q], acc);
      }
      w[s] = acc;
    }
    Real r[N];
    load_line<N, A>(Q, l, r);
#pragma unroll
    for (int m = 0; m < N; ++m) {
      Real v = r[m];
      v = fma(Real(T.L0[m]), w[0], v);
      v = fma(Real(T.dL0[m]), tga[0], v);
      v = fma(Real(T.L1[m]), w[1], v);
      v = fma(Real(T.dL1[m]), tga[1], v);
      r[m] = v;
    }
    store_line<N, A>(Q, l, r);
  }
  __syncthreads();
}

template <int N, typename Real, int A>
__device__ __forceinline__ void own_traces(const Real *Q, const Real *G0, const Real *G1,
                                           const Real *G2, int l, Real (&tr)[2][4])
{
  Real v[N];
  load_line<N, A>(Q, l, v);
  end_values<N>(v, tr[0][0], tr[1][0]);
  load_line<N, A>(G0, l, v);
  end_values<N>(v, tr[0][1], tr[1][1]);
  load_line<N, A>(G1, l, v);
  end_values<N>(v, tr[0][2], tr[1][2]);
  load_line<N, A>(G2, l, v);
  end_values<N>(v, tr[0][3], tr[1][3]);
}

template <int N, typename Real, int GK>
__global__ void __launch_bounds__(256)
sipg_apply_kernel(const OpView<Real> op, const Real *__restrict__ src, Real *__restrict__ dst)
{
  using BK = Blocking<N>;
  constexpr int N2 = BK::N2, N3 = BK::N3, B = BK::B, NT = BK::NT, WSZ = BK::WSZ;
  constexpr const auto &T = kTab<N>;
  __shared__ Real smem[B * (N3 + WSZ)];

  const int t = threadIdx.x;
  const bool act = t < NT;
  const int cb = act ? t / N2 : 0;
  const int l = act ? t - cb * N2 : 0;
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int cell0 = blk * B;
  const int cell = cell0 + cb;
  const bool valid = act && cell < op.ncells;
  const int nhere = min(B, op.ncells - cell0);
  Real *Q = smem + cb * N3;
  Real *W = smem + B * N3 + cb * WSZ;
  Real *G0 = W, *G1 = W + N3, *G2 = W + 2 * N3;
  int ci[3];
  ci[0] = cell % op.ncell[0];
  ci[1] = (cell / op.ncell[0]) % op.ncell[1];
  ci[2] = cell / (op.ncell[0] * op.ncell[1]);

  // (a) gather
  const int64_t g0 = (int64_t)cell0 * N3;
  for (int i = t; i < B * N3; i += 256) smem[i] = (i < nhere * N3) ? src[g0 + i] : Real(0);
  __syncthreads();

  // (b) basis change to the Gauss points, then the collocation derivative
  if (act) sweep<N, 0, M_S>(Q, Q, l);
  __syncthreads();
  if (act) sweep<N, 1, M_S>(Q, Q, l);
  __syncthreads();
  Real dz[N];
  if (act) {
    Real v[N], q[N];
    load_line<N, 2>(Q, l, v);
    eo_apply<N, M_S>(v, q);
    store_line<N, 2>(Q, l, q);
    eo_apply<N, M_DCO>(q, dz);
    store_line<N, 2>(G2, l, dz);
  }
  __syncthreads();
  if (act) {
    sweep<N, 0, M_DCO>(Q, G0, l);
    sweep<N, 1, M_DCO>(Q, G1, l);
  }
  __syncthreads();

  // (c) own-side traces of the six faces
  Real tr[3][2][4];
  if (act) {
    own_traces<N, Real, 0>(Q, G0, G1, G2, l, tr[0]);
    own_traces<N, Real, 1>(Q, G0, G1, G2, l, tr[1]);
    own_traces<N, Real, 2>(Q, G0, G1, G2, l, tr[2]);
  }
  __syncthreads();

  // (d) cell quadrature-point operation along this thread's z-line
  if (act) {
    Real t2v[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const int p = l + k * N2;
      const Real g[3] = {G0[p], G1[p], dz[k]};
      Real o[3];
      if constexpr (GK == CURVED) {
        Real jt[9], f = Real(0);
        if (valid) {
          const int64_t ix = (int64_t)cell * N3 + p;
          const int64_t cs = op.g.cell_stride;
#pragma unroll
          for (int m = 0; m < 9; ++m) jt[m] = op.g.cell[m * cs + ix];
          f = op.g.cell[9 * cs + ix];
        } else {
#pragma unroll
          for (int m = 0; m < 9; ++m) jt[m] = Real(0);
        }
        Real gx[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) gx[a] = f * (jt[3 * a] * g[0] + jt[3 * a + 1] * g[1] + jt[3 * a + 2] * g[2]);
#pragma unroll
        for (int b = 0; b < 3; ++b) o[b] = jt[b] * gx[0] + jt[3 + b] * gx[1] + jt[6 + b] * gx[2];
      } else {
        Real f;
        if constexpr (GK == AFFINE_VAR) {
          f = valid ? op.g.cell[(int64_t)cell * N3 + p] : Real(0);
        } else {
          const int i1 = l % N, i2 = l / N;
          Real w1 = Real(0), w2 = Real(0);
#pragma unroll
          for (int q = 0; q < N; ++q) {
            if (q == i1) w1 = Real(T.gw[q]);
            if (q == i2) w2 = Real(T.gw[q]);
          }
          f = op.c_vol * w1 * w2 * Real(T.gw[k]);
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) o[a] = f * op.inv_h[a] * op.inv_h[a] * g[a];
      }
      G0[p] = o[0];
      G1[p] = o[1];
      t2v[k] = o[2];
    }
    Real rz[N];
    eo_apply<N, M_DCOT>(t2v, rz);
    store_line<N, 2>(Q, l, rz);
  }
  __syncthreads();
  if (act) {
    Real v[N], r[N], q[N];
    load_line<N, 0>(G0, l, v);
    eo_apply<N, M_DCOT>(v, r);
    load_line<N, 0>(Q, l, q);
#pragma unroll
    for (int m = 0; m < N; ++m) q[m] += r[m];
    store_line<N, 0>(Q, l, q);
  }
  __syncthreads();
  if (act) {
    Real v[N], r[N], q[N];
    load_line<N, 1>(G1, l, v);
    eo_apply<N, M_DCOT>(v, r);
    load_line<N, 1>(Q, l, q);
#pragma unroll
    for (int m = 0; m < N; ++m) q[m] += r[m];
    store_line<N, 1>(Q, l, q);
  }
  __syncthreads();

  // (e) face terms, direction by direction
  face_direction<N, Real, GK, 0>(op, src, Q, W, l, cell, ci, act, valid, tr[0]);
  face_direction<N, Real, GK, 1>(op, src, Q, W, l, cell, ci, act, valid, tr[1]);
  face_direction<N, Real, GK, 2>(op, src, Q, W, l, cell, ci, act, valid, tr[2]);

  // (f) back to the Gauss-Lobatto basis and write
  if (act) sweep<N, 0, M_ST>(Q, Q, l);
  __syncthreads();
  if (act) sweep<N, 1, M_ST>(Q, Q, l);
  __syncthreads();
  if (act) sweep<N, 2, M_ST>(Q, Q, l);
  __syncthreads();
  for (int i = t; i < nhere * N3; i += 256) dst[g0 + i] = smem[i];
}

// ---------------------------------------------------------------------------
// Diagonal of A: A_ii = a_h(phi_i, phi_i).  One workgroup per cell, one
// thread per basis function; the cell's geometry is staged in LDS.
//   cell:  sum_q c det J w |J^{-T} grad_xi phi_i|^2
//   faces: phi_i vanishes on a face unless i sits on it (nodal basis); there
//          sum_q c ds (tau phi_i^2 - phi_i dn phi_i) (interior neighbour has u = 0),
//          twice that on Dirichlet faces (mirror), nothing on Neumann faces.
// Accumulated in double from the FP64 geometry.
// ---------------------------------------------------------------------------
template <int N, int GK>
__global__ void __launch_bounds__(1024)
sipg_diag_kernel(const OpView<double> op, double *__restrict__ d64, float *__restrict__ d32)
{
  constexpr int N2 = N * N, N3 = N2 * N;
  constexpr const auto &T = kTab<N>;
  constexpr int NG = (GK == CURVED) ? 10 : 1;
  __shared__ double geo[NG * N3];
  const int cell = blockIdx.x;
  const int i = threadIdx.x;
  for (int m = i; m < NG * N3; m += blockDim.x) {
    const int q = m % N3, f = m / N3;
    if constexpr (GK == CURVED) geo[m] = op.g.cell[f * op.g.cell_stride + (int64_t)cell * N3 + q];
    else if constexpr (GK == AFFINE_VAR) geo[m] = op.g.cell[(int64_t)cell * N3 + q];
    else geo[m] = op.c_vol * T.gw[q % N] * T.gw[(q / N) % N] * T.gw[q / N2];
  }
  __syncthreads();
  if (i >= N3) return;
  const int id[3] = {i % N, (i / N) % N, i / N2};
  double Sc[3][N], Dc[3][N];
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int q = 0; q < N; ++q) {
      double s = 0.0, dd = 0.0;
#pragma unroll
      for (int j = 0; j < N; ++j)
        if (j == id[d]) { s = T.S[q][j]; dd = T.D[q][j]; }
      Sc[d][q] = s;
      Dc[d][q] = dd;
    }
  double acc = 0.0;
  for (int q3 = 0; q3 < N; ++q3)
    for (int q2 = 0; q2 < N; ++q2)
#pragma unroll
      for (int q1 = 0; q1 < N; ++q1) {
        const int q = q1 + N * q2 + N2 * q3;
        const double g[3] = {Dc[0][q1] * Sc[1][q2] * Sc[2][q3], Sc[0][q1] * Dc[1][q2] * Sc[2][q3],
                             Sc[0][q1] * Sc[1][q2] * Dc[2][q3]};
        if constexpr (GK == CURVED) {
          double s2 = 0.0;
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            const double gx = geo[(3 * a) * N3 + q] * g[0] + geo[(3 * a + 1) * N3 + q] * g[1] +
                              geo[(3 * a + 2) * N3 + q] * g[2];
            s2 += gx * gx;
          }
          acc += geo[9 * N3 + q] * s2;
        } else {
          acc += geo[q] * (op.inv_h[0] * op.inv_h[0] * g[0] * g[0] + op.inv_h[1] * op.inv_h[1] * g[1] * g[1] +
                           op.inv_h[2] * op.inv_h[2] * g[2] * g[2]);
        }
      }
  int ci[3];
  ci[0] = cell % op.ncell[0];
  ci[1] = (cell / op.ncell[0]) % op.ncell[1];
  ci[2] = cell / (op.ncell[0] * op.ncell[1]);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int t1 = (a == 0) ? 1 : 0, t2 = (a == 2) ? 1 : 2;
    for (int s = 0; s < 2; ++s) {
      if (id[a] != (s ? N - 1 : 0)) continue;
      const int cn = ci[a] + (s ? 1 : -1);
      const bool interior = cn >= 0 && cn < op.ncell[a];
      double mult = 1.0;
      if (!interior) mult = (op.bc[2 * a + s] == 0) ? 2.0 : 0.0;
      if (mult == 0.0) continue;
      double fa = 0.0;
      for (int j = 0; j < N; ++j)
        if (j == id[a]) fa = s ? T.F1[j] : T.F0[j];
      const double sg = s ? 1.0 : -1.0;
      int p[3] = {ci[0], ci[1], ci[2]}, m[3] = {op.ncell[0], op.ncell[1], op.ncell[2]};
      p[a] += s;
      m[a] += 1;
      const int64_t fid = p[0] + (int64_t)m[0] * (p[1] + (int64_t)m[1] * p[2]);
      for (int q2 = 0; q2 < N; ++q2)
        for (int q1 = 0; q1 < N; ++q1) {
          const int lq = q1 + N * q2;
          const double phi = Sc[t1][q1] * Sc[t2][q2];
          double g[3];
          g[a] = fa * Sc[t1][q1] * Sc[t2][q2];
          g[t1] = Dc[t1][q1] * Sc[t2][q2];
          g[t2] = Sc[t1][q1] * Dc[t2][q2];
          double j[3] = {0.0, 0.0, 0.0}, cds;
          if constexpr (GK == CURVED) {
            const double *fg = op.g.face[a];
            const int64_t fs = op.g.face_stride[a], f = fid * N2 + lq;
            j[0] = fg[f];
            j[1] = fg[fs + f];
            j[2] = fg[2 * fs + f];
            cds = fg[3 * fs + f];
          } else if constexpr (GK == AFFINE_VAR) {
            j[a] = op.inv_h[a];
            cds = op.g.face[a][fid * N2 + lq];
          } else {
            j[a] = op.inv_h[a];
            cds = op.c_area[a] * T.gw[q1] * T.gw[q2];
          }
          const double dn = sg * (j[0] * g[0] + j[1] * g[1] + j[2] * g[2]);
          acc += mult * cds * (op.tau[a] * phi * phi - phi * dn);
        }
    }
  }
  const int64_t o = (int64_t)cell * N3 + i;
  if (d64) d64[o] = acc;
  if (d32) d32[o] = (float)acc;
}

template <int N>
hipError_t launch_apply(const dg_op *op, const void *src, void *dst, bool f32, hipStream_t s)
{
  using BK = Blocking<N>;
  const int grid = (int)((op->ncells + BK::B - 1) / BK::B);
  if (grid == 0) return hipSuccess;
  if (f32) {
    const float *x = static_cast<const float *>(src);
    float *y = static_cast<float *>(dst);
    switch (op->gk) {
      case CURVED: hipLaunchKernelGGL((sipg_apply_kernel<N, float, CURVED>), dim3(grid), dim3(256), 0, s, op->v32, x, y); break;
      case AFFINE_VAR: hipLaunchKernelGGL((sipg_apply_kernel<N, float, AFFINE_VAR>), dim3(grid), dim3(256), 0, s, op->v32, x, y); break;
      default: hipLaunchKernelGGL((sipg_apply_kernel<N, float, AFFINE_CONST>), dim3(grid), dim3(256), 0, s, op->v32, x, y); break;
    }
  } else {
    const double *x = static_cast<const double *>(src);
    double *y = static_cast<double *>(dst);
    switch (op->gk) {
      case CURVED: hipLaunchKernelGGL((sipg_apply_kernel<N, double, CURVED>), dim3(grid), dim3(256), 0, s, op->v64, x, y); break;
      case AFFINE_VAR: hipLaunchKernelGGL((sipg_apply_kernel<N, double, AFFINE_VAR>), dim3(grid), dim3(256), 0, s, op->v64, x, y); break;
      default: hipLaunchKernelGGL((sipg_apply_kernel<N, double, AFFINE_CONST>), dim3(grid), dim3(256), 0, s, op->v64, x, y); break;
    }
  }
  return hipGetLastError();
}

template <int N>
hipError_t launch_diag(const dg_op *op, void *diag64, void *diag32, hipStream_t s)
{
  constexpr int N3 = N * N * N;
  const int block = ((N3 + 63) / 64) * 64;
  const int grid = (int)op->ncells;
  if (grid == 0) return hipSuccess;
  double *d64 = static_cast<double *>(diag64);
  float *d32 = static_cast<float *>(diag32);
  switch (op->gk) {
    case CURVED: hipLaunchKernelGGL((sipg_diag_kernel<N, CURVED>), dim3(grid), dim3(block), 0, s, op->v64, d64, d32); break;
    case AFFINE_VAR: hipLaunchKernelGGL((sipg_diag_kernel<N, AFFINE_VAR>), dim3(grid), dim3(block), 0, s, op->v64, d64, d32); break;
    default: hipLaunchKernelGGL((sipg_diag_kernel<N, AFFINE_CONST>), dim3(grid), dim3(block), 0, s, op->v64, d64, d32); break;
  }
  return hipGetLastError();
}

}  // namespace dgk
