// advection.hpp -- the fused matrix-free apply of the DG advection operator
// with the local Lax-Friedrichs (upwind) flux, Sec. 2, Eq. (1), evaluated
// with the loop structure of Algorithm 1.  Included by kernels.hpp, whose
// line, sweep and table helpers it uses.
//
//   y_i = -(grad phi_i, c u_h)_e + <phi_i, f*>_{de},
//   f*  = 1/2 (c.n)(u- + u+) + 1/2 |c.n| (u- - u+),  n the cell's outward normal.
//
// Element-centric like the SIPG apply: a workgroup owns B cells, one thread
// per 1D line.  Per cell, in one pass:
//   (a) gather the N^3 coefficients (the x-direction neighbour face values
//       requested behind them);
//   (b) S x S x S to the Gauss points (values only: the cell term needs no
//       derivative of u);
//   (c) per face direction: own trace u- from the Gauss-point lines with the
//       Gauss Lagrange end values; the neighbour's trace from its
//       Gauss-Lobatto face layer alone (a nodal basis on the Lobatto points
//       has exactly n^2 non-zero functions on a face, so n^2 values are read
//       instead of a block), then the 2D basis change S x S; upwind flux with
//       the stored (c.n) ds; integration onto the own normal line with the
//       end values;
//   (d) quadrature-point operation t = (J^{-1} c det J w) u (the
//       quadrature-point work of Algorithm 1) and the transposed collocation
//       derivatives, subtracted from
//       the residual;
//   (e) S^T x S^T x S^T and one coalesced write.
// Boundary faces: u+ = -u- (mirror, homogeneous inflow data) on bc 0 faces,
// u+ = u- (outflow) on bc 1 faces.
#pragma once

namespace dgk {

// The two neighbours' face values at Gauss-Lobatto face node l for direction
// A: the neighbour below shares its xi_A = 1 layer, the one above its xi_A =
// 0 layer.  Unconditional loads (a missing neighbour reads the cell itself).
template <int N, typename Real, int A>
__device__ __forceinline__ void load_neighbour_faces(const OpView<Real> &op, const Real *__restrict__ src, int cell,
                                                     int l, const int (&ci)[3], Real (&nb)[2])
{
  constexpr int N3 = N * N * N;
  const int64_t cstride = (A == 0) ? 1 : (A == 1 ? (int64_t)op.ncell[0] : (int64_t)op.ncell[0] * op.ncell[1]);
  const int b = line_base<N, A>(l);
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int cn = ci[A] + (s ? 1 : -1);
    const bool inside = cn >= 0 && cn < op.ncell[A];
    const int64_t nbc = inside ? (int64_t)cell + (s ? cstride : -cstride) : (int64_t)cell;
    nb[s] = src[nbc * N3 + b + (s ? 0 : (N - 1) * kStride<N, A>)];
  }
}

// Face terms of direction A for this thread's cell, own side only.  W is
// 4 N^2 of scratch: X (neighbour face values at the Lobatto nodes), Y (after
// the basis change along t1), U (u+ at the face Gauss points, in X's place).
template <int N, typename Real, int A, typename Next>
__device__ __forceinline__ void adv_face_direction(const OpView<Real> &op, const Real *Q, Real *R, Real *W, int l,
                                                   const int (&ci)[3], bool act, bool valid, const Real (&nb)[2],
                                                   Real (&fz)[2], Next &&next)
{
  constexpr int N2 = N * N;
  constexpr Tables<N> T = kTab<N>;
  Real *X = W;            // [s][p1 + N p2]
  Real *Y = W + 2 * N2;   // [s][q1 + N p2]
  Real *U = W;            // [s][q1 + N q2]
  bool interior[2];
  Real cn[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int c = ci[A] + (s ? 1 : -1);
    interior[s] = valid && c >= 0 && c < op.ncell[A];
    cn[s] = op.g.face[A][face_id<A>(op.ncell, ci, s) * N2 + l];  // (c.n) ds for the +e_A normal
  }
  // S1: own trace at this face point from the Gauss-point line; the
  // neighbours' face values into X
  Real um[2] = {Real(0), Real(0)};
  if (act) {
    Real v[N];
    load_line<N, A>(Q, l, v);
    end_values<N>(v, um[0], um[1]);
    X[l] = nb[0];
    X[N2 + l] = nb[1];
  }
  __syncthreads();
  next();
  // S2, S3: 2D basis change of the neighbour traces to the face Gauss points
  for_jobs<N, 2 * N>(l, act, [&](int jb) {
    const int a = jb / N, p2 = jb - a * N;
    Real v[N], r[N];
#pragma unroll
    for (int m = 0; m < N; ++m) v[m] = X[a * N2 + m + N * p2];
    eo_apply<N, M_S>(v, r);
#pragma unroll
    for (int m = 0; m < N; ++m) Y[a * N2 + m + N * p2] = r[m];
  });
  __syncthreads();
  for_jobs<N, 2 * N>(l, act, [&](int jb) {
    const int a = jb / N, q1 = jb - a * N;
    Real v[N], r[N];
#pragma unroll
    for (int m = 0; m < N; ++m) v[m] = Y[a * N2 + q1 + N * m];
    eo_apply<N, M_S>(v, r);
#pragma unroll
    for (int m = 0; m < N; ++m) U[a * N2 + q1 + N * m] = r[m];
  });
  __syncthreads();
  // S4: upwind flux times the area element at this face point (each thread
  // reads only its own point of U, which it alone overwrites next)
  if (act) {
    Real t[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const Real up = interior[s] ? U[s * N2 + l] : (op.bc[2 * A + s] == 0 ? -um[s] : um[s]);
      const Real cnm = s ? cn[s] : -cn[s];   // outward normal: -e_A side below, +e_A above
      t[s] = Real(0.5) * cnm * (um[s] + up) + Real(0.5) * fabs(cnm) * (um[s] - up);
    }
    // S5: integration onto this thread's normal line of R with the end
    // values; the first direction initialises R, the second adds, the third
    // hands its two coefficients to the cell pass that owns the same z-line
    if constexpr (A == 2) {
      fz[0] = t[0];
      fz[1] = t[1];
    } else {
      Real r[N];
      if constexpr (A == 1) load_line<N, A>(R, l, r);
#pragma unroll
      for (int m = 0; m < N; ++m) {
        Real v = (A == 1) ? r[m] : Real(-0.0);
        v = madd(T.L0[m], t[0], v);
        v = madd(T.L1[m], t[1], v);
        r[m] = v;
      }
      store_line<N, A>(R, l, r);
    }
  }
}

template <int N, typename Real, int TPB>
__device__ __forceinline__ void adv_apply_batch(const OpView<Real> &op, const Real *__restrict__ src,
                                                Real *__restrict__ dst, int blk, Real *smem)
{
  using BK = Blocking<N, TPB>;
  constexpr int N2 = BK::N2, N3 = BK::N3, B = BK::B, NT = BK::NT, WSZ = BK::WSZ;
  constexpr Tables<N> T = kTab<N>;
  static_assert(WSZ >= 4 * N2 && WSZ >= 2 * N3, "scratch too small");

  const int t = threadIdx.x;
  const bool act = t < NT;
  const int cb = act ? t / N2 : 0;
  const int l = act ? t - cb * N2 : 0;
  const int cell0 = blk * B;
  const int cell = min(cell0 + cb, op.ncells - 1);
  const bool valid = act && cell0 + cb < op.ncells;
  const int nhere = min(B, op.ncells - cell0);
  Real *Q = smem + cb * N3;
  Real *R = smem + B * N3 + cb * N3;
  Real *W = smem + 2 * B * N3 + cb * WSZ;
  Real *G0 = W, *G1 = W + N3;
  int ci[3];
  ci[0] = cell % op.ncell[0];
  ci[1] = (cell / op.ncell[0]) % op.ncell[1];
  ci[2] = cell / (op.ncell[0] * op.ncell[1]);

  // (a) gather, with the x-direction neighbour face values behind it
  const int64_t g0 = (int64_t)cell0 * N3;
  constexpr int GI = (B * N3 + TPB - 1) / TPB;
  Real gv[GI];
#pragma unroll
  for (int j = 0; j < GI; ++j) gv[j] = src[g0 + min(t + j * TPB, nhere * N3 - 1)];
  __builtin_amdgcn_sched_barrier(0);
  Real nb[2];
  load_neighbour_faces<N, Real, 0>(op, src, cell, l, ci, nb);
  static_assert(GI * TPB <= 2 * B * N3, "gather overrun");
#pragma unroll
  for (int j = 0; j < GI; ++j) {
    const int i = t + j * TPB;
    smem[i] = i < nhere * N3 ? gv[j] : Real(0);  // slots past B N^3 fall into R, overwritten by the x faces
  }
  __syncthreads();

  // (b) values at the Gauss points
  if (act) sweep<N, 0, M_S>(Q, Q, l);
  __syncthreads();
  if (act) sweep<N, 1, M_S>(Q, Q, l);
  __syncthreads();
  if (act) sweep<N, 2, M_S>(Q, Q, l);
  __syncthreads();

  // (c) faces; the stored cell coefficients of the first planes are
  // requested during the last direction
  constexpr int NB = (DG_GEO_BUFS < N) ? DG_GEO_BUFS : N;
  Real gbuf[NB][3];
  auto load_geometry = [&](int k, Real (&gb)[3]) {
    const int64_t ix = geo_base<N>(cell) + l + k * kGeoPlane<N>;
    const int64_t cs = op.g.cell_stride;
#pragma unroll
    for (int m = 0; m < 3; ++m) gb[m] = op.g.cell[m * cs + ix];
  };
  Real fz[2] = {Real(0), Real(0)};
  adv_face_direction<N, Real, 0>(op, Q, R, W, l, ci, act, valid, nb, fz,
                                 [&] { load_neighbour_faces<N, Real, 1>(op, src, cell, l, ci, nb); });
  adv_face_direction<N, Real, 1>(op, Q, R, W, l, ci, act, valid, nb, fz,
                                 [&] { load_neighbour_faces<N, Real, 2>(op, src, cell, l, ci, nb); });
  adv_face_direction<N, Real, 2>(op, Q, R, W, l, ci, act, valid, nb, fz, [&] {
#pragma unroll
    for (int k = 0; k < NB; ++k) load_geometry(k, gbuf[k]);
  });
  __syncthreads();  // the last direction's scratch is free before W takes t_x, t_y

  // (d) t = (J^{-1} c det J w) u along this thread's z-line; t_z integrated
  // in registers, t_x and t_y through W; all subtracted from R
  if (act) {
    Real qz[N], t2v[N];
    load_line<N, 2>(Q, l, qz);
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const int p = l + k * N2;
      const Real *tc = gbuf[k % NB];
      G0[p] = tc[0] * qz[k];
      G1[p] = tc[1] * qz[k];
      t2v[k] = tc[2] * qz[k];
      __builtin_amdgcn_sched_barrier(0);
      if (k + NB < N) load_geometry(k + NB, gbuf[k % NB]);
    }
    Real rz[N], q[N];
    eo_apply<N, M_DCOT>(t2v, rz);
    load_line<N, 2>(R, l, q);
#pragma unroll
    for (int m = 0; m < N; ++m) {
      Real v = q[m] - rz[m];
      v = madd(T.L0[m], fz[0], v);
      v = madd(T.L1[m], fz[1], v);
      q[m] = v;
    }
    store_line<N, 2>(R, l, q);
  }
  __syncthreads();
  if (act) {
    Real v[N], r[N], q[N];
    load_line<N, 0>(G0, l, v);
    eo_apply<N, M_DCOT>(v, r);
    load_line<N, 0>(R, l, q);
#pragma unroll
    for (int m = 0; m < N; ++m) q[m] -= r[m];
    store_line<N, 0>(R, l, q);
  }
  __syncthreads();
  if (act) {
    Real v[N], r[N], q[N];
    load_line<N, 1>(G1, l, v);
    eo_apply<N, M_DCOT>(v, r);
    load_line<N, 1>(R, l, q);
#pragma unroll
    for (int m = 0; m < N; ++m) q[m] -= r[m];
    store_line<N, 1>(R, l, q);
  }
  __syncthreads();

  // (e) back to the Gauss-Lobatto basis and write
  if (act) sweep<N, 0, M_ST>(R, R, l);
  __syncthreads();
  if (act) sweep<N, 1, M_ST>(R, R, l);
  __syncthreads();
  if (act) sweep<N, 2, M_ST>(R, R, l);
  __syncthreads();
  const Real *Rall = smem + B * N3;
  for (int i = t; i < nhere * N3; i += TPB) dst[g0 + i] = Rall[i];
}

template <int N, typename Real>
__global__ void __launch_bounds__(Blocking<N>::TPB, (Occupancy<N, Real>::value))
adv_apply_kernel(const OpView<Real> op, const Real *__restrict__ src, Real *__restrict__ dst)
{
  using BK = Blocking<N>;
  __shared__ Real smem[BK::SMEM];
  adv_apply_batch<N, Real, BK::TPB>(op, src, dst, xcd_remap(blockIdx.x, gridDim.x), smem);
}

}  // namespace dgk
