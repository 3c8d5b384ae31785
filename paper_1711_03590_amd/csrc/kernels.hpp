// kernels.hpp -- the fused matrix-free SIPG apply and the diagonal kernel,
// templated on the number of 1D points N, the number type and the geometry
// representation.  One translation unit per N instantiates them.
//
// Operator: y = A u (Sec. 2, Eq. (3)) for the SIPG form of Sec. 2, Eq. (2),
// evaluated cell by cell, in the nodal Gauss-Lobatto basis or the
// Hermite-like basis (template parameter BS, see tables.hpp).  Each workgroup owns B = TPB / N^2 cells and maps
// one thread to one 1D line of each cell (N^2 lines per sweep direction).
// Per cell, in one pass (the cell and face loops of Algorithm 1 fused,
// Design Choice 2):
//   (a) gather the cell's N^3 coefficients into LDS (coalesced block copy);
//   (b) basis change to the Gauss points, S x S x S (Sec. 2, Eq. (6)), every
//       1D matvec done with the even-odd decomposition (Sec. 3.3, Eq. (8));
//   (c) per face direction: own-side value and reference normal derivative
//       at the face points, read off the Gauss-point data with the Gauss
//       Lagrange end values (the tangential directions already sit at the
//       face's Gauss points); the neighbour's trace from its coefficients
//       on the normal lines (S_f and D_f of Eq. (7): for the nodal basis
//       the end node and all N nodes, for the Hermite-like basis one and
//       two coefficients), then a 2D basis change S x S to the face Gauss points and
//       the collocation derivative along the face for the tangential
//       gradient; numerical flux of Eq. (2) with the stored
//       normal-times-inverse-Jacobian j (Design Choice 5); own-side
//       integration back onto the quadrature-point residual;
//   (d) cell quadrature-point operation (that of Algorithm 1): collocation
//       derivatives Dco along x, y, z, t = J^{-1} (c det J w) J^{-T} grad_xi u,
//       then the transposed derivatives sum the three components into the
//       residual;
//   (e) transposed basis change S^T x S^T x S^T and one coalesced write of
//       the cell's dst block (cells set, never add: Sec. 2.1).
// The faces come before the cell integrals so that the neighbour blocks are
// read while the workgroups that own them, dispatched at about the same
// time, have just read them too (L2 hits rather than fabric traffic); the
// stored cell geometry, the bulk of the traffic, streams in behind.
// No atomics: every dst entry is written by exactly one thread, so the
// result is deterministic.  Neighbour blocks are re-read from L2/MALL.
#pragma once

#include <type_traits>

#include "dg_internal.hpp"
#include "reduce.hpp"
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
template <int N>
inline constexpr EvenOdd<N> kEoD = make_even_odd<N>(kTab<N>.D, false);
template <int N, int BS>
inline constexpr BasisTables<N> kBasis = make_basis<N>(BS);
template <int N>
inline constexpr EvenOdd<N> kEoHS = make_even_odd<N>(kBasis<N, BASIS_HERMITE>.S, false);
template <int N>
inline constexpr EvenOdd<N> kEoHSt = make_even_odd<N>(kBasis<N, BASIS_HERMITE>.S, true);

enum : int { M_S = 0, M_ST = 1, M_DCO = 2, M_DCOT = 3, M_D = 4, M_HS = 5, M_HST = 6 };
// the basis change of basis BS and its transpose
template <int BS>
inline constexpr int kMS = (BS == BASIS_HERMITE) ? M_HS : M_S;
template <int BS>
inline constexpr int kMST = (BS == BASIS_HERMITE) ? M_HST : M_ST;

// acc + c x with c a compile-time constant after unrolling: zero and unit
// coefficients fold away (accumulators start at -0.0, the additive identity)
template <typename Real>
__device__ __forceinline__ Real madd(double c, Real x, Real acc)
{
  if (c == 0.0) return acc;
  if (c == 1.0) return acc + x;
  if (c == -1.0) return acc - x;
  return fma(Real(c), x, acc);
}

// the even-odd table of matrix M (as a value, so that every use below is a
// compile-time constant once the loops are unrolled)
template <int N, int M>
__host__ __device__ constexpr EvenOdd<N> eo_tab()
{
  if constexpr (M == M_S) return kEoS<N>;
  else if constexpr (M == M_ST) return kEoSt<N>;
  else if constexpr (M == M_DCO) return kEoDco<N>;
  else if constexpr (M == M_DCOT) return kEoDcot<N>;
  else if constexpr (M == M_HS) return kEoHS<N>;
  else if constexpr (M == M_HST) return kEoHSt<N>;
  else return kEoD<N>;
}

// out = M in for one line of N values, M one of S, S^T (centro-symmetric) or
// Dco, Dco^T (centro-skew-symmetric), by the even-odd decomposition:
// about N^2/2 multiply-adds instead of N^2.
template <int N, int M, typename Real>
__device__ __forceinline__ void eo_apply(const Real (&in)[N], Real (&out)[N])
{
  constexpr int H = N / 2;
  constexpr bool sym = (M == M_S || M == M_ST || M == M_HS || M == M_HST);
  constexpr EvenOdd<N> C = eo_tab<N, M>();
  Real e[H > 0 ? H : 1], o[H > 0 ? H : 1];
#pragma unroll
  for (int j = 0; j < H; ++j) {
    e[j] = in[j] + in[N - 1 - j];
    o[j] = in[j] - in[N - 1 - j];
  }
#pragma unroll
  for (int i = 0; i < H; ++i) {
    Real se = Real(-0.0), so = Real(-0.0);
#pragma unroll
    for (int j = 0; j < H; ++j) {
      se = madd(C.E[i][j], e[j], se);
      so = madd(C.O[i][j], o[j], so);
    }
    if constexpr (N % 2 == 1) se = madd(C.Mid[i], in[H], se);
    out[i] = se + so;
    out[N - 1 - i] = sym ? se - so : so - se;
  }
  if constexpr (N % 2 == 1) {
    Real s = Real(-0.0);
    if constexpr (sym) {
      s = madd(C.Mid[H], in[H], s);
#pragma unroll
      for (int j = 0; j < H; ++j) s = madd(C.E[H][j], e[j], s);
    } else {
#pragma unroll
      for (int j = 0; j < H; ++j) s = madd(C.O[H][j], o[j], s);
    }
    out[H] = s;
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

// values at xi = 0 and xi = 1 of the polynomial with Gauss-point values v:
// sum_m L0[m] v[m] and sum_m L1[m] v[m], with L1[m] = L0[N-1-m]
template <int N, typename Real>
__device__ __forceinline__ void end_values(const Real (&v)[N], Real &lo, Real &hi)
{
  constexpr Tables<N> T = kTab<N>;
  constexpr int H = N / 2;
  Real se = Real(-0.0), so = Real(-0.0);
#pragma unroll
  for (int m = 0; m < H; ++m) {
    se = madd(0.5 * (T.L0[m] + T.L0[N - 1 - m]), v[m] + v[N - 1 - m], se);
    so = madd(0.5 * (T.L0[m] - T.L0[N - 1 - m]), v[m] - v[N - 1 - m], so);
  }
  if constexpr (N % 2 == 1) se = madd(T.L0[H], v[H], se);
  lo = se + so;
  hi = se - so;
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

// quadrature-point planes of stored cell geometry held in flight per thread
#ifndef DG_GEO_BUFS
#define DG_GEO_BUFS 3
#endif
// of which requested already during the last face direction
#ifndef DG_GEO_PRE
#define DG_GEO_PRE 1
#endif
#ifndef DG_WG_WAVES
#define DG_WG_WAVES 2
#endif
// Threads per workgroup: DG_WG_WAVES waves (more when one cell's N^2 lines
// need them), or a single wave where that keeps the same share of the lanes
// busy (N = 2, 3, 4, 7, 8: whole cells fill one wave as well as two), which
// measures 2-6 % faster there; at N = 5 and 6 one wave would idle a quarter
// and more of its lanes.
template <int N>
constexpr int pick_tpb()
{
  constexpr int n2 = N * N;
  constexpr int base = (64 * DG_WG_WAVES >= n2) ? 64 * DG_WG_WAVES : ((n2 + 63) / 64) * 64;
  if (n2 <= 64 && base > 64 && (64 / n2) * n2 * base == (base / n2) * n2 * 64) return 64;
  return base;
}
template <int N>
inline constexpr int kTpb = pick_tpb<N>();

template <int N, int TPB_ = kTpb<N>>
struct Blocking {
  static constexpr int N2 = N * N, N3 = N2 * N;
  static constexpr int TPB = TPB_;           // threads per workgroup
  static constexpr int B = TPB / N2;         // cells per workgroup
  static constexpr int NT = B * N2;          // active threads
  static constexpr int WSZ = (2 * N3 > 10 * N2) ? 2 * N3 : 10 * N2;  // gradient / face scratch per cell
  static constexpr int SMEM = B * (2 * N3 + WSZ);  // shared memory in Real units
};

// Layout of the stored cell geometry (every quantity array): cells in groups
// of G = Blocking<N>::B, the cells of one apply workgroup; within a group,
// plane k (the N^2 points with i3 = k) of all G cells comes after plane
// k - 1, so that a workgroup's load of one plane of one quantity is one
// contiguous run of G N^2 values.  Point q of cell c sits at
//   ((c / G) N + q / N^2) G N^2 + (c mod G) N^2 + q mod N^2,
// the arrays are padded to whole groups, and the padding is never read.
template <int N>
inline constexpr int kGeoGroup = Blocking<N>::B;
template <int N>
inline constexpr int kGeoPlane = kGeoGroup<N> * N * N;   // distance between planes of one cell
// index of plane 0, point 0 of a cell
template <int N>
__host__ __device__ __forceinline__ int64_t geo_base(int64_t cell)
{
  constexpr int G = kGeoGroup<N>;
  const int c = (int)cell;   // cells < 2^31 (at most 2^31 - 1 DoFs)
  const int g = c / G;
  return ((int64_t)g * N * G + (c - g * G)) * (N * N);
}
// offset of point q of a cell from its geo_base
template <int N>
__host__ __device__ __forceinline__ int geo_off(int q)
{
  return (q / (N * N)) * kGeoPlane<N> + q % (N * N);
}
// the line of direction D through face point l (the same lines as
// line_base): offset of its first point from geo_base, and the stride
template <int N, int D>
__device__ __forceinline__ int geo_line(int l)
{
  if constexpr (D == 2) return l;
  else if constexpr (D == 1) return (l / N) * kGeoPlane<N> + l % N;
  else return (l / N) * kGeoPlane<N> + (l % N) * N;
}
template <int N, int D>
inline constexpr int kGeoStride = (D == 0) ? 1 : (D == 1 ? N : kGeoPlane<N>);

// Workgroups per CU that the LDS footprint allows (160 KiB per CU).  With
// 256-thread workgroups this is also the number of waves per SIMD, which is
// passed to the compiler as the occupancy target so that register
// allocation does not become the tighter limit.
#ifndef DG_MAX_WAVES_F64
#define DG_MAX_WAVES_F64 4
#endif
#ifndef DG_MAX_WAVES_F32
#define DG_MAX_WAVES_F32 5
#endif
template <int N, typename Real>
struct Occupancy {
  static constexpr int lds = Blocking<N>::SMEM * (int)sizeof(Real);
  static constexpr int wgs = 163840 / lds;
  static constexpr int waves = wgs * (Blocking<N>::TPB / 64) / 4;
  static constexpr int cap = sizeof(Real) == 8 ? DG_MAX_WAVES_F64 : DG_MAX_WAVES_F32;
  static constexpr int value = waves < 1 ? 1 : (waves > cap ? cap : waves);
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

// geometry of face point l of the face of cell ci on side s of direction A:
// j = J^{-1} n for the normal pointing along +e_A, and c ds
template <int N, typename Real, int GK, int A>
__device__ __forceinline__ void face_geometry(const OpView<Real> &op, const int (&ci)[3], int s, int l,
                                              Real (&j)[3], Real &cds)
{
  constexpr int N2 = N * N;
  constexpr Tables<N> T = kTab<N>;
  j[0] = j[1] = j[2] = Real(0);
  if constexpr (curved_faces(GK)) {
    const int64_t f = face_id<A>(op.ncell, ci, s) * N2 + l;
    const Real *fg = op.g.face[A];
    const int64_t fs = op.g.face_stride[A];
    j[0] = fg[f];
    j[1] = fg[fs + f];
    j[2] = fg[2 * fs + f];
    cds = fg[3 * fs + f];
  } else if constexpr (GK == AFFINE_VAR) {
    j[A] = op.inv_h[A];
    cds = op.g.face[A][face_id<A>(op.ncell, ci, s) * N2 + l];
  } else {
    j[A] = op.inv_h[A];
    const int q1 = l % N, q2 = l / N;
    Real w1 = Real(0), w2 = Real(0);
#pragma unroll
    for (int q = 0; q < N; ++q) {
      if (q == q1) w1 = Real(T.gw[q]);
      if (q == q2) w2 = Real(T.gw[q]);
    }
    cds = op.c_area[A] * w1 * w2;
  }
}

// sum_m dL0[m] v[m] and sum_m dL1[m] v[m]: derivatives at xi = 0, 1 of the
// polynomial with Gauss-point values v (dL1[m] = -dL0[N-1-m])
template <int N, typename Real>
__device__ __forceinline__ void end_derivatives(const Real (&v)[N], Real &lo, Real &hi)
{
  constexpr Tables<N> T = kTab<N>;
  constexpr int H = N / 2;
  Real se = Real(-0.0), so = Real(-0.0);
#pragma unroll
  for (int m = 0; m < H; ++m) {
    se = madd(0.5 * (T.dL0[m] + T.dL0[N - 1 - m]), v[m] + v[N - 1 - m], se);
    so = madd(0.5 * (T.dL0[m] - T.dL0[N - 1 - m]), v[m] - v[N - 1 - m], so);
  }
  if constexpr (N % 2 == 1) se = madd(T.dL0[H], v[H], se);
  lo = se + so;
  hi = so - se;
}

// The two neighbours' normal lines through face point l for direction A;
// issued ahead of their use so that the loads overlap the preceding phase.
// Only the coefficients with a non-zero S_f or D_f entry at the shared face
// are read: all N for the nodal basis, two for the Hermite-like one.
template <int N, typename Real, int A, int BS>
__device__ __forceinline__ void load_neighbour_lines(const OpView<Real> &op, const Real *__restrict__ src,
                                                     int cell, int l, const int (&ci)[3], Real (&nb)[2][N])
{
  // branch-free: a missing neighbour reads the cell itself (the values are
  // then ignored), so the loads can stay in flight across later phases
  constexpr int N3 = N * N * N;
  constexpr BasisTables<N> BT = kBasis<N, BS>;
  const int64_t cstride = (A == 0) ? 1 : (A == 1 ? (int64_t)op.ncell[0] : (int64_t)op.ncell[0] * op.ncell[1]);
  const int b = line_base<N, A>(l);
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int cn = ci[A] + (s ? 1 : -1);
    const bool inside = cn >= 0 && cn < op.ncell[A];
    const int64_t nbc = inside ? (int64_t)cell + (s ? cstride : -cstride) : (int64_t)cell;
    const Real *line = src + nbc * N3 + b;
#pragma unroll
    for (int m = 0; m < N; ++m) {
      // the neighbour below meets the face with its xi_A = 1 side, the one above with xi_A = 0
      const bool need = s ? (BT.V0[m] != 0.0 || BT.F0[m] != 0.0) : (BT.V1[m] != 0.0 || BT.F1[m] != 0.0);
      nb[s][m] = need ? line[m * kStride<N, A>] : Real(0);
    }
  }
}

// Jobs jb = 0 .. JOBS-1 of one cell spread over its N^2 lanes (a lane takes
// several when JOBS > N^2); unrolled, so that the common single pass has no
// loop around it.
template <int N, int JOBS, typename F>
__device__ __forceinline__ void for_jobs(int l, bool act, F &&f)
{
  constexpr int N2 = N * N, IT = (JOBS + N2 - 1) / N2;
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int jb = l + it * N2;
    if (act && jb < JOBS) f(jb);
  }
}

// Face terms of direction A for this thread group's cell: the face integrals
// of Sec. 2 Eq. (2) over the cell's two faces normal to A, own side only
// (the element's share of Algorithm 1's face loops), added into the
// quadrature-point residual R along the normal lines.  Q holds the cell's
// values at the Gauss points; W is 10 N^2 of scratch.
//   [[u]] = u- - u+, {{grad u}} = (grad u- + grad u+)/2; the average's
//   tangential part is the tangential derivative of V = u- + u+ on the face
//   (V = 2 u- on a Dirichlet face, where u+ = -u- but grad u+ = grad u-).
// On affine meshes (no curved faces) the cell term splits by direction
// (J^{-1} diagonal): fl holds f h_A^{-2} (f = c det J w) at the points of
// this thread's A-line, and the x and y directions add their cell term
// Dco^T (fl Dco Q) on that line in the same pass as the face integration
// (one read and one write of the residual line instead of two each); qz is
// this thread's Gauss-point z-line, kept in registers from the last basis
// change, which the z faces read instead of LDS.
template <int N, typename Real, int GK, int A, int BS, bool GH, typename Next>
__device__ __forceinline__ void face_direction(const OpView<Real> &op, const Real *Q, Real *R, Real *W, int l,
                                               const int (&ci)[3], bool act, bool valid, const Real (&nb)[2][N],
                                               Real (&fz)[4], Next &&next, const Real (&fl)[N], const Real (&qz)[N])
{
  constexpr bool FUSED = !curved_faces(GK);
  constexpr int N2 = N * N;
  constexpr int t1 = (A == 0) ? 1 : 0, t2 = (A == 2) ? 1 : 2;
  constexpr Tables<N> T = kTab<N>;
  constexpr BasisTables<N> BT = kBasis<N, BS>;
  Real *X = W;            // [s][value, normal derivative] of the neighbour as face coefficients p1 + N p2
  Real *Y = W + 4 * N2;   // [s][..] after the basis change along t1: q1 + N p2
  Real *U = W;            // [s][u+, d_A u+] at the face Gauss points q1 + N q2
  Real *V = W + 8 * N2;   // [s] u- + u+
  Real *dV = W + 4 * N2;  // [s][d_t1 V, d_t2 V]
  Real *Z = W;            // [s][tg_t1, tg_t2]
  Real *Z2 = W + 4 * N2;  // [s][Dco^T along t1 of tg_t1, Dco^T along t2 of tg_t2]
  // with GH, a ghost side's faces are interior faces whose neighbour
  // traces come from op.ghost instead of src
  bool interior[2], ghost[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int cn = ci[A] + (s ? 1 : -1);
    const bool inside = cn >= 0 && cn < op.ncell[A];
    ghost[s] = GH && !inside && op.bc[2 * A + s] == kBcGhost;
    interior[s] = valid && (inside || ghost[s]);
  }
  Real jg[2][3], cds[2];
  face_geometry<N, Real, GK, A>(op, ci, 0, l, jg[0], cds[0]);
  face_geometry<N, Real, GK, A>(op, ci, 1, l, jg[1], cds[1]);
  // S1: own value and reference normal derivative at this face point (the
  // Gauss-point data is tangentially at the face's Gauss points already);
  // the neighbour's value and normal derivative on the shared face in the
  // tangential basis: S_f and D_f of Eq. (7) applied to its normal line
  Real um[2], dm[2];
  Real v[N];   // this thread's Gauss-point line along A (kept for the fused cell term)
  if (act) {
    if constexpr (FUSED && A == 2) {
#pragma unroll
      for (int m = 0; m < N; ++m) v[m] = qz[m];
    } else {
      load_line<N, A>(Q, l, v);
    }
    end_values<N>(v, um[0], um[1]);
    end_derivatives<N>(v, dm[0], dm[1]);
    // neighbour below: the shared face is its xi_A = 1 side; above: xi_A = 0
    Real val0 = Real(-0.0), der0 = Real(-0.0), val1 = Real(-0.0), der1 = Real(-0.0);
#pragma unroll
    for (int m = 0; m < N; ++m) {
      val0 = madd(BT.V1[m], nb[0][m], val0);
      der0 = madd(BT.F1[m], nb[0][m], der0);
      val1 = madd(BT.V0[m], nb[1][m], val1);
      der1 = madd(BT.F0[m], nb[1][m], der1);
    }
    if (GH && (ghost[0] || ghost[1])) {  // only cells on a partition's ghost side
      const int64_t p = side_plane_index<A>(op.ncell, ci) * 2 * N2 + l;
      if (ghost[0]) {
        val0 = op.ghost[2 * A][p];
        der0 = op.ghost[2 * A][p + N2];
      }
      if (ghost[1]) {
        val1 = op.ghost[2 * A + 1][p];
        der1 = op.ghost[2 * A + 1][p + N2];
      }
    }
    X[0 * N2 + l] = val0;
    X[1 * N2 + l] = der0;
    X[2 * N2 + l] = val1;
    X[3 * N2 + l] = der1;
  }
  __syncthreads();
  // loads for what follows (the next direction's neighbour lines, or the
  // first planes of cell geometry), in flight through the rest of the faces
  next();
  // S2: neighbour traces, basis change along t1: one line of one of the
  // four arrays [s][value, derivative] per job (4N jobs over the N^2 lanes)
  for_jobs<N, 4 * N>(l, act, [&](int jb) {
    const int a = jb / N, p2 = jb - a * N;
    Real v[N], r[N];
#pragma unroll
    for (int m = 0; m < N; ++m) v[m] = X[a * N2 + m + N * p2];
    eo_apply<N, kMS<BS>>(v, r);
#pragma unroll
    for (int m = 0; m < N; ++m) Y[a * N2 + m + N * p2] = r[m];
  });
  __syncthreads();
  // S3: basis change along t2
  for_jobs<N, 4 * N>(l, act, [&](int jb) {
    const int a = jb / N, q1 = jb - a * N;
    Real v[N], r[N];
#pragma unroll
    for (int m = 0; m < N; ++m) v[m] = Y[a * N2 + q1 + N * m];
    eo_apply<N, kMS<BS>>(v, r);
#pragma unroll
    for (int m = 0; m < N; ++m) U[a * N2 + q1 + N * m] = r[m];
  });
  __syncthreads();
  // S4: jump, sum of values, sum of normal reference derivatives
  Real jump[2] = {Real(0), Real(0)}, dsum[2] = {Real(0), Real(0)};
  if (act) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      Real up, dp;
      if (interior[s]) {
        up = U[(2 * s) * N2 + l];
        dp = U[(2 * s + 1) * N2 + l];
      } else {  // Dirichlet mirror u+ = -u-, grad u+ = grad u-
        up = -um[s];
        dp = dm[s];
      }
      jump[s] = um[s] - up;
      dsum[s] = dm[s] + dp;
      if constexpr (curved_faces(GK)) V[s * N2 + l] = interior[s] ? um[s] + up : Real(2) * um[s];
    }
  }
  __syncthreads();
  // S5: tangential collocation derivatives of V (lines along t1 and t2).
  // On affine meshes j is normal to the face, so the tangential gradient and
  // the tangential gradient-test terms (S5, S7) drop out exactly.
  if constexpr (curved_faces(GK)) {
    for_jobs<N, 4 * N>(l, act, [&](int jb) {
      const int s = jb / (2 * N), c = (jb / N) & 1, i = jb % N;
      const int base = c ? i : N * i, stride = c ? N : 1;
      Real v[N], r[N];
#pragma unroll
      for (int m = 0; m < N; ++m) v[m] = V[s * N2 + base + m * stride];
      eo_apply<N, M_DCO>(v, r);
#pragma unroll
      for (int m = 0; m < N; ++m) dV[(2 * s + c) * N2 + base + m * stride] = r[m];
    });
    __syncthreads();
  }
  // S6: numerical flux at this face point (Algorithm 1's quadrature-point work on faces)
  Real tv[2] = {Real(0), Real(0)}, tga[2] = {Real(0), Real(0)};
  if (act) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const Real c_ds = (!interior[s] && op.bc[2 * A + s] != 0) ? Real(0) : cds[s];  // Neumann: nothing
      const Real sg = s ? Real(1) : Real(-1);
      const Real je[3] = {sg * jg[s][0], sg * jg[s][1], sg * jg[s][2]};
      const Real gfac = Real(-0.5) * c_ds * jump[s];
      tga[s] = gfac * je[A];
      if constexpr (curved_faces(GK)) {
        Real g[3];
        g[t1] = dV[(2 * s) * N2 + l];
        g[t2] = dV[(2 * s + 1) * N2 + l];
        g[A] = dsum[s];
        const Real avg = Real(0.5) * (je[0] * g[0] + je[1] * g[1] + je[2] * g[2]);
        tv[s] = c_ds * (op.tau[A] * jump[s] - avg);
        Z[(2 * s) * N2 + l] = gfac * je[t1];
        Z[(2 * s + 1) * N2 + l] = gfac * je[t2];
      } else {
        tv[s] = c_ds * (op.tau[A] * jump[s] - Real(0.5) * (je[A] * dsum[s]));
      }
    }
  }
  // S7: transposed tangential collocation derivatives of the gradient-test terms
  if constexpr (curved_faces(GK)) {
    __syncthreads();
    for_jobs<N, 4 * N>(l, act, [&](int jb) {
      const int s = jb / (2 * N), c = (jb / N) & 1, i = jb % N;
      const int base = c ? i : N * i, stride = c ? N : 1;
      Real v[N], r[N];
#pragma unroll
      for (int m = 0; m < N; ++m) v[m] = Z[(2 * s + c) * N2 + base + m * stride];
      eo_apply<N, M_DCOT>(v, r);
#pragma unroll
      for (int m = 0; m < N; ++m) Z2[(2 * s + c) * N2 + base + m * stride] = r[m];
    });
    __syncthreads();
  }
  // S8: face-normal integration onto this thread's normal line of R: the
  // rank-4 update L0 w0 + dL0 tga0 + L1 w1 + dL1 tga1.  The first direction
  // initialises R, the second adds to it, and the third hands its four
  // coefficients (fz) to the cell pass, which owns the same z-line.  No
  // barrier follows: the next writer of Z2's storage is two barriers away.
  if (act) {
    Real w[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      w[s] = tv[s];
      if constexpr (curved_faces(GK)) w[s] += Z2[(2 * s) * N2 + l] + Z2[(2 * s + 1) * N2 + l];
    }
    if constexpr (A == 2) {
      fz[0] = w[0];
      fz[1] = tga[0];
      fz[2] = w[1];
      fz[3] = tga[1];
    } else {
      Real r[N], c[N];
      if constexpr (A == 1) load_line<N, A>(R, l, r);
      if constexpr (FUSED) {
        Real g[N];
        eo_apply<N, M_DCO>(v, g);
#pragma unroll
        for (int m = 0; m < N; ++m) g[m] *= fl[m];
        eo_apply<N, M_DCOT>(g, c);
      }
#pragma unroll
      for (int m = 0; m < N; ++m) {
        Real x = (A == 1) ? r[m] : Real(-0.0);
        if constexpr (FUSED) x += c[m];
        x = madd(T.L0[m], w[0], x);
        x = fma(Real(T.dL0[m]), tga[0], x);
        x = madd(T.L1[m], w[1], x);
        x = fma(Real(T.dL1[m]), tga[1], x);
        r[m] = x;
      }
      store_line<N, A>(R, l, r);
    }
  }
}

// Optional output of the solver's product p.(A p) computed inside the apply:
// part[blk] receives each workgroup's share (a fixed-order sum over its
// threads); the caller sums the shares in workgroup order afterwards.
template <typename Real>
struct DotOut {
  Real *part = nullptr;
};

// fixed-order sum over the TPB threads of a workgroup (sh: TPB / 64 values)
template <int TPB, typename Real>
__device__ __forceinline__ Real wg_sum(Real v, Real *sh)
{
  return workgroup_sum<TPB>(v, sh);
}

// The fused pass over the cells of one batch (cells blk*B .. blk*B+B-1) by
// a workgroup of TPB threads; smem holds B * (2 N^3 + WSZ) values.  tid is
// the thread's index in the workgroup (threadIdx.x when negative); a caller
// that applies several batches in a loop passes it redefined per batch, so
// that what the pass derives from it is not hoisted out of the loop and
// kept live across it.
template <int N, typename Real, int GK, int TPB, bool DOT = false, int BS = BASIS_NODAL, bool GH = false>
__device__ __forceinline__ void apply_batch(const OpView<Real> &op, const Real *__restrict__ src,
                                            Real *__restrict__ dst, int blk, Real *smem,
                                            const DotOut<Real> &dot = DotOut<Real>{}, int tid = -1)
{
  using BK = Blocking<N, TPB>;
  constexpr int N2 = BK::N2, N3 = BK::N3, B = BK::B, NT = BK::NT, WSZ = BK::WSZ;
  constexpr Tables<N> T = kTab<N>;

  const int t = tid >= 0 ? tid : (int)threadIdx.x;
  const bool act = t < NT;
  const int cb = act ? t / N2 : 0;
  const int l = act ? t - cb * N2 : 0;
  const int cell0 = blk * B;
  // cells past the end of the mesh (last workgroup) compute on a copy of the
  // last cell and are never written; all global loads stay unconditional
  const int cell = min(cell0 + cb, op.ncells - 1);
  const bool valid = act && cell0 + cb < op.ncells;
  const int nhere = min(B, op.ncells - cell0);
  Real *Q = smem + cb * N3;              // values at the Gauss points (kept to the end of the faces)
  Real *R = smem + B * N3 + cb * N3;     // residual at the Gauss points
  Real *W = smem + 2 * B * N3 + cb * WSZ;
  Real *G0 = W, *G1 = W + N3;
  int ci[3];
  ci[0] = cell % op.ncell[0];
  ci[1] = (cell / op.ncell[0]) % op.ncell[1];
  ci[2] = cell / (op.ncell[0] * op.ncell[1]);

  // (a) gather the workgroup's cells (coalesced), and request the
  // x-direction neighbour lines behind it: the faces come first, while the
  // neighbouring workgroups, started at about the same time, have just read
  // the same blocks (they are then still in L2)
  const int64_t g0 = (int64_t)cell0 * N3;
  constexpr int GI = (B * N3 + TPB - 1) / TPB;
  Real gv[GI];
#pragma unroll
  for (int j = 0; j < GI; ++j) gv[j] = src[g0 + min(t + j * TPB, nhere * N3 - 1)];
  __builtin_amdgcn_sched_barrier(0);  // keep the gather ahead of the neighbour loads
  Real nb[2][N];
  load_neighbour_lines<N, Real, 0, BS>(op, src, cell, l, ci, nb);
  // (slots past B N^3 fall into R, which the first face direction overwrites)
  static_assert(GI * TPB <= 2 * B * N3, "gather overrun");
#pragma unroll
  for (int j = 0; j < GI; ++j) {
    const int i = t + j * TPB;
    smem[i] = i < nhere * N3 ? gv[j] : Real(0);
  }
  __syncthreads();

  // (b) basis change to the Gauss points (Eq. (6), right factor); on affine
  // meshes the thread keeps its z-line of the result in registers (qz)
  constexpr bool FUSED = !curved_faces(GK);
  Real qz[N];
  if (act) sweep<N, 0, kMS<BS>>(Q, Q, l);
  __syncthreads();
  if (act) sweep<N, 1, kMS<BS>>(Q, Q, l);
  __syncthreads();
  if (act) {
    if constexpr (FUSED) {
      Real v[N];
      load_line<N, 2>(Q, l, v);
      eo_apply<N, kMS<BS>>(v, qz);
      store_line<N, 2>(Q, l, qz);
    } else {
      sweep<N, 2, kMS<BS>>(Q, Q, l);
    }
  }
  __syncthreads();

  // (c) face terms, direction by direction, into R; the stored cell geometry
  // of the first planes is requested during the last direction
  constexpr int NB = (DG_GEO_BUFS < N) ? DG_GEO_BUFS : N;
  constexpr int GV = (GK == CURVED || GK == CURVED_MERGED) ? cell_values(GK) : 1;
  Real gbuf[NB][GV];
  auto load_geometry = [&](int k, Real (&gb)[GV]) {
    if constexpr (GK == CURVED || GK == CURVED_MERGED) {
      const int64_t ix = geo_base<N>(cell) + l + k * kGeoPlane<N>;
      const int64_t cs = op.g.cell_stride;
#pragma unroll
      for (int m = 0; m < GV; ++m) gb[m] = op.g.cell[m * cs + ix];
    }
  };
  Real fz[4] = {Real(0), Real(0), Real(0), Real(0)};
  // affine meshes: f h_D^{-2} along this thread's D-line for the fused
  // per-direction cell terms (the loads of direction D issued a direction
  // ahead, like the neighbour lines)
  Real fl[3][N];
  const int i1 = l % N, i2 = l / N;
  Real w12 = Real(0);  // the product of the weights of this thread's two fixed indices
  auto load_fline = [&](auto dir) {
    constexpr int D = decltype(dir)::value;
    if constexpr (GK == AFFINE_VAR) {
      const int64_t gl = geo_base<N>(cell) + geo_line<N, D>(l);
#pragma unroll
      for (int m = 0; m < N; ++m) fl[D][m] = op.g.cell[gl + m * kGeoStride<N, D>];
    }
  };
  auto scale_fline = [&](auto dir) {
    constexpr int D = decltype(dir)::value;
    const Real ih2 = op.inv_h[D] * op.inv_h[D];
#pragma unroll
    for (int m = 0; m < N; ++m) {
      if constexpr (GK == AFFINE_VAR) fl[D][m] *= ih2;
      else fl[D][m] = op.c_vol * w12 * Real(T.gw[m]) * ih2;
    }
  };
  if constexpr (FUSED) {
    Real w1 = Real(0), w2 = Real(0);
#pragma unroll
    for (int q = 0; q < N; ++q) {
      if (q == i1) w1 = Real(T.gw[q]);
      if (q == i2) w2 = Real(T.gw[q]);
    }
    w12 = w1 * w2;
    load_fline(std::integral_constant<int, 0>{});
    scale_fline(std::integral_constant<int, 0>{});
  }
  face_direction<N, Real, GK, 0, BS, GH>(op, Q, R, W, l, ci, act, valid, nb, fz, [&] {
    load_neighbour_lines<N, Real, 1, BS>(op, src, cell, l, ci, nb);
    if constexpr (FUSED) load_fline(std::integral_constant<int, 1>{});
  }, fl[0], qz);
  if constexpr (FUSED) scale_fline(std::integral_constant<int, 1>{});
  face_direction<N, Real, GK, 1, BS, GH>(op, Q, R, W, l, ci, act, valid, nb, fz, [&] {
    load_neighbour_lines<N, Real, 2, BS>(op, src, cell, l, ci, nb);
    if constexpr (FUSED) load_fline(std::integral_constant<int, 2>{});
  }, fl[1], qz);
  constexpr int PRE = (DG_GEO_PRE < NB) ? DG_GEO_PRE : NB;
  face_direction<N, Real, GK, 2, BS, GH>(op, Q, R, W, l, ci, act, valid, nb, fz, [&] {
#pragma unroll
    for (int k = 0; k < PRE; ++k) load_geometry(k, gbuf[k]);
  }, fl[2], qz);

  if constexpr (FUSED) {
    // (d) affine cell integrals: J^{-1} is diagonal, so the cell term splits
    // by direction, R += sum_d Dco_d^T (f h_d^{-2} Dco_d Q) with f = c det J w
    // per point; the x and y terms were added with the x and y faces, the z
    // term goes with the z faces' normal integration onto this thread's
    // z-line, which then takes the transposed basis change along z in
    // registers (the basis changes of a tensor product commute)
    scale_fline(std::integral_constant<int, 2>{});
    if (act) {
      Real g[N], r[N], q[N];
      eo_apply<N, M_DCO>(qz, g);
#pragma unroll
      for (int m = 0; m < N; ++m) g[m] *= fl[2][m];
      eo_apply<N, M_DCOT>(g, r);
      load_line<N, 2>(R, l, q);
#pragma unroll
      for (int m = 0; m < N; ++m) {
        Real x = q[m] + r[m];
        x = madd(T.L0[m], fz[0], x);
        x = fma(Real(T.dL0[m]), fz[1], x);
        x = madd(T.L1[m], fz[2], x);
        x = fma(Real(T.dL1[m]), fz[3], x);
        q[m] = x;
      }
      eo_apply<N, kMST<BS>>(q, r);
      store_line<N, 2>(R, l, r);
    }
    __syncthreads();
  } else {
#pragma unroll
    for (int k = PRE; k < NB; ++k) load_geometry(k, gbuf[k]);
    __syncthreads();  // the z faces' Z2 reads are done before W takes the gradients
    // (d) cell integrals: collocation derivatives along x and y (z is taken
    // in registers below), then the quadrature-point operation along this
    // thread's z-line with the stored geometry (J^{-T} and c det J w per
    // point) software-pipelined NB planes ahead, then the transposed
    // derivatives, all summed into R
    if (act) {
      sweep<N, 0, M_DCO>(Q, G0, l);
      sweep<N, 1, M_DCO>(Q, G1, l);
    }
    __syncthreads();
    if (act) {
      Real qz[N], dz[N], t2v[N];
      // G2: the Dco rows of this thread's x and y indices, and its two weights
      Real d1[N], d2[N], w12 = Real(0);
      if constexpr (GK == CURVED_POS) {
        const int i1 = l % N, i2 = l / N;
        Real w1 = Real(0), w2 = Real(0);
#pragma unroll
        for (int q = 0; q < N; ++q) {
          if (q == i1) w1 = Real(T.gw[q]);
          if (q == i2) w2 = Real(T.gw[q]);
        }
        w12 = w1 * w2;
#pragma unroll
        for (int j = 0; j < N; ++j) {
          d1[j] = Real(0);
          d2[j] = Real(0);
#pragma unroll
          for (int q = 0; q < N; ++q) {
            if (q == i1) d1[j] = Real(T.Dco[q][j]);
            if (q == i2) d2[j] = Real(T.Dco[q][j]);
          }
        }
      }
      load_line<N, 2>(Q, l, qz);
      eo_apply<N, M_DCO>(qz, dz);
#pragma unroll
      for (int k = 0; k < N; ++k) {
        const int p = l + k * N2;
        const Real g[3] = {G0[p], G1[p], dz[k]};
        Real o[3];
        if constexpr (GK == CURVED) {
          const Real *jt = gbuf[k % NB];
          const Real f = gbuf[k % NB][9];
          Real gx[3];
#pragma unroll
          for (int a = 0; a < 3; ++a) gx[a] = f * (jt[3 * a] * g[0] + jt[3 * a + 1] * g[1] + jt[3 * a + 2] * g[2]);
#pragma unroll
          for (int b = 0; b < 3; ++b) o[b] = jt[b] * gx[0] + jt[3 + b] * gx[1] + jt[6 + b] * gx[2];
          __builtin_amdgcn_sched_barrier(0);
          if (k + NB < N) load_geometry(k + NB, gbuf[k % NB]);
        } else if constexpr (GK == CURVED_MERGED) {
          // G4: t = M grad_xi u with the symmetric M = c det J w J^{-1} J^{-T}
          const Real *M = gbuf[k % NB];
          o[0] = M[0] * g[0] + M[1] * g[1] + M[2] * g[2];
          o[1] = M[1] * g[0] + M[3] * g[1] + M[4] * g[2];
          o[2] = M[2] * g[0] + M[4] * g[1] + M[5] * g[2];
          __builtin_amdgcn_sched_barrier(0);
          if (k + NB < N) load_geometry(k + NB, gbuf[k % NB]);
        } else if constexpr (GK == CURVED_POS) {
          // G2 (Sec. 5): columns a_d = dx/dxi_d of the Jacobian by collocation
          // derivatives of the stored positions along the x, y and z lines
          // through this point (L1-resident: the cell's positions are read
          // by all its threads); with C_d = a_{d+1} x a_{d+2} and
          // det = a_0 . C_0, J^{-T} g = sum_d C_d g_d / det and
          // t_e = c w / det * C_e . (sum_d C_d g_d)
          const Real *P = op.g.cell + geo_base<N>(cell);
          const int64_t cs = op.g.cell_stride;
          constexpr int CP = kGeoPlane<N>;
          const int i1 = l % N, i2 = l / N;
          Real a[3][3];
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            // one component at a time, so that at most 3N loads are in flight
            __builtin_amdgcn_sched_barrier(0);
            Real sx = Real(-0.0), sy = Real(-0.0), sz = Real(-0.0);
#pragma unroll
            for (int j = 0; j < N; ++j) {
              sx = fma(d1[j], P[c * cs + j + N * i2 + CP * k], sx);
              sy = fma(d2[j], P[c * cs + i1 + N * j + CP * k], sy);
              sz = madd(T.Dco[k][j], P[c * cs + l + CP * j], sz);
            }
            a[0][c] = sx;
            a[1][c] = sy;
            a[2][c] = sz;
          }
          Real C[3][3];
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            const Real *u = a[(d + 1) % 3], *v = a[(d + 2) % 3];
            C[d][0] = u[1] * v[2] - u[2] * v[1];
            C[d][1] = u[2] * v[0] - u[0] * v[2];
            C[d][2] = u[0] * v[1] - u[1] * v[0];
          }
          const Real det = a[0][0] * C[0][0] + a[0][1] * C[0][1] + a[0][2] * C[0][2];
          const Real cw = P[3 * cs + l + CP * k] * w12 * Real(T.gw[k]) / det;
          Real v[3];
#pragma unroll
          for (int c = 0; c < 3; ++c) v[c] = C[0][c] * g[0] + C[1][c] * g[1] + C[2][c] * g[2];
#pragma unroll
          for (int e = 0; e < 3; ++e) o[e] = cw * (C[e][0] * v[0] + C[e][1] * v[1] + C[e][2] * v[2]);
        }
        G0[p] = o[0];
        G1[p] = o[1];
        t2v[k] = o[2];
      }
      Real rz[N], q[N];
      eo_apply<N, M_DCOT>(t2v, rz);
      load_line<N, 2>(R, l, q);
      // plus the z faces' normal integration onto the same line
#pragma unroll
      for (int m = 0; m < N; ++m) {
        Real v = q[m] + rz[m];
        v = madd(T.L0[m], fz[0], v);
        v = fma(Real(T.dL0[m]), fz[1], v);
        v = madd(T.L1[m], fz[2], v);
        v = fma(Real(T.dL1[m]), fz[3], v);
        q[m] = v;
      }
      store_line<N, 2>(R, l, q);
    }
    __syncthreads();
    // the y part first, so that the x-line pass, the last to add to R, can
    // take the transposed basis change along x before its one store
    if (act) {
      Real v[N], r[N], q[N];
      load_line<N, 1>(G1, l, v);
      eo_apply<N, M_DCOT>(v, r);
      load_line<N, 1>(R, l, q);
#pragma unroll
      for (int m = 0; m < N; ++m) q[m] += r[m];
      store_line<N, 1>(R, l, q);
    }
    __syncthreads();
    if (act) {
      Real v[N], r[N], q[N];
      load_line<N, 0>(G0, l, v);
      eo_apply<N, M_DCOT>(v, r);
      load_line<N, 0>(R, l, q);
#pragma unroll
      for (int m = 0; m < N; ++m) q[m] += r[m];
      eo_apply<N, kMST<BS>>(q, r);
      store_line<N, 0>(R, l, r);
    }
    __syncthreads();
  }

  // (e) back to the Gauss-Lobatto basis (transposed basis change; on affine
  // meshes z is done already, on curved ones x) and write
  if constexpr (FUSED) {
    if (act) sweep<N, 0, kMST<BS>>(R, R, l);
    __syncthreads();
  }
  if (act) sweep<N, 1, kMST<BS>>(R, R, l);
  __syncthreads();
  if constexpr (!FUSED && !DOT) {
    // the last direction (z) in registers, written straight to dst: the
    // z-lines of a cell are its N^2 consecutive points per plane, so each
    // store of a wave covers contiguous runs of its cells' blocks
    if (valid) {
      Real v[N], r[N];
      load_line<N, 2>(R, l, v);
      eo_apply<N, kMST<BS>>(v, r);
      Real *out = dst + (int64_t)cell * N3 + l;
#pragma unroll
      for (int m = 0; m < N; ++m) out[m * N2] = r[m];
    }
    return;
  }
  if constexpr (!FUSED) {
    if (act) sweep<N, 2, kMST<BS>>(R, R, l);
    __syncthreads();
  }
  const Real *Rall = smem + B * N3;
  for (int i = t; i < nhere * N3; i += TPB) dst[g0 + i] = Rall[i];
  if constexpr (DOT) {
    // this workgroup's share of src.(A src): the gathered values gv are
    // src at the same indices the write loop above visits
    Real v = Real(0);
#pragma unroll
    for (int j = 0; j < GI; ++j) {
      const int i = t + j * TPB;
      if (i < nhere * N3) v += gv[j] * Rall[i];
    }
    static_assert(TPB <= B * N3, "Q holds the workgroup sum");
    const Real wsum = wg_sum<TPB>(v, smem);   // Q is free after the last sweep
    if (t == 0) dot.part[blk] = wsum;
  }
}

template <int N, typename Real, int GK, bool DOT = false, int BS = BASIS_NODAL, bool GH = false>
__global__ void __launch_bounds__(Blocking<N>::TPB, (Occupancy<N, Real>::value))
sipg_apply_kernel(const OpView<Real> op, const Real *__restrict__ src, Real *__restrict__ dst,
                  const DotOut<Real> dot = DotOut<Real>{})
{
  using BK = Blocking<N>;
  __shared__ Real smem[BK::SMEM];
  // successive applies walk the cells in opposite orders, so that each
  // starts on the data the previous one touched last (still in the MALL
  // when the operand set exceeds it); the result does not depend on it
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  apply_batch<N, Real, GK, BK::TPB, DOT, BS, GH>(op, src, dst, op.reverse ? (int)gridDim.x - 1 - b : b, smem, dot);
}

// ---------------------------------------------------------------------------
// Diagonal of A: A_ii = a_h(phi_i, phi_i).  One workgroup per cell, one
// thread per basis function.
//   cell:  sum_q grad_xi phi_i^T M grad_xi phi_i with the symmetric effective
//          coefficient M = c det J w J^{-1} J^{-T} per point.  Each component
//          of grad_xi phi_i is a product of 1D factors (D along its own
//          direction, S along the others), so for every pair (b, c) of
//          components the sum over the n^3 points factorises into three 1D
//          contractions with the tables F_d[q][j] = E_b,d[q][j] E_c,d[q][j]:
//          O(n^4) per pair instead of O(n^6) for the whole cell.
//   faces: phi_i vanishes on a face unless its 1D factor normal to the face
//          is the one with value 1 there (the end node of the nodal basis,
//          phi_0 or phi_{N-1} of the Hermite-like one); there
//          sum_q c ds (tau phi_i^2 - phi_i dn phi_i) (interior neighbour has u = 0),
//          twice that on Dirichlet faces (mirror), nothing on Neumann faces.
// Accumulated in double from the FP64 geometry.
// ---------------------------------------------------------------------------
template <int N, int GK, int BS = BASIS_NODAL>
__global__ void __launch_bounds__(1024)
sipg_diag_kernel(const OpView<double> op, double *__restrict__ d64, float *__restrict__ d32)
{
  constexpr int N2 = N * N, N3 = N2 * N;
  constexpr Tables<N> T = kTab<N>;
  constexpr BasisTables<N> BT = kBasis<N, BS>;
  __shared__ double Sl[N2], Dl[N2];      // S[q][j], D[q][j] (basis function j at Gauss point q)
  __shared__ double Fe[2 * N];           // D_f end rows: F0[j], F1[j]
  __shared__ double Dcl[N2];             // Dco[q][m] (positions storage)
  __shared__ double M[6 * N3];           // M00 M01 M02 M11 M12 M22 per point
  __shared__ double T1[N3], T2[N3];
  const int cell = blockIdx.x;
  const int i = threadIdx.x;
  const bool act = i < N3;
  if (i == 0) {
#pragma unroll
    for (int q = 0; q < N; ++q) {
#pragma unroll
      for (int j = 0; j < N; ++j) {
        Sl[q * N + j] = BT.S[q][j];
        Dl[q * N + j] = BT.D[q][j];
      }
      Fe[q] = BT.F0[q];
      Fe[N + q] = BT.F1[q];
#pragma unroll
      for (int m = 0; m < N; ++m) Dcl[q * N + m] = T.Dco[q][m];
    }
  }
  if constexpr (GK == CURVED_POS) __syncthreads();  // Dcl is read below
  // effective coefficient at quadrature point q = i
  if (act) {
    const int64_t ix = geo_base<N>(cell) + geo_off<N>(i);
    const int64_t cs = op.g.cell_stride;
    double m[6];
    if constexpr (GK == CURVED) {
      double jt[9];
#pragma unroll
      for (int a = 0; a < 9; ++a) jt[a] = op.g.cell[a * cs + ix];
      const double f = op.g.cell[9 * cs + ix];
      const int rb[6] = {0, 0, 0, 1, 1, 2}, rc[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
      for (int e = 0; e < 6; ++e)
        m[e] = f * (jt[rb[e]] * jt[rc[e]] + jt[3 + rb[e]] * jt[3 + rc[e]] + jt[6 + rb[e]] * jt[6 + rc[e]]);
    } else if constexpr (GK == CURVED_MERGED) {
#pragma unroll
      for (int e = 0; e < 6; ++e) m[e] = op.g.cell[e * cs + ix];
    } else if constexpr (GK == CURVED_POS) {
      // the Jacobian's columns by collocation derivatives of the positions,
      // then M = c w det J^{-1} J^{-T} = c w / det C^T C (C_d = a_{d+1} x a_{d+2})
      const int qi[3] = {i % N, (i / N) % N, i / N2};
      const int64_t c0 = geo_base<N>(cell);
      double a[3][3];
      for (int d = 0; d < 3; ++d)
        for (int c = 0; c < 3; ++c) {
          double sum = 0.0;
          for (int mm = 0; mm < N; ++mm) {
            int r[3] = {qi[0], qi[1], qi[2]};
            r[d] = mm;
            sum += Dcl[qi[d] * N + mm] * op.g.cell[c * cs + c0 + r[0] + N * r[1] + kGeoPlane<N> * r[2]];
          }
          a[d][c] = sum;
        }
      double C[3][3];
      for (int d = 0; d < 3; ++d) {
        const double *u = a[(d + 1) % 3], *v = a[(d + 2) % 3];
        C[d][0] = u[1] * v[2] - u[2] * v[1];
        C[d][1] = u[2] * v[0] - u[0] * v[2];
        C[d][2] = u[0] * v[1] - u[1] * v[0];
      }
      const double det = a[0][0] * C[0][0] + a[0][1] * C[0][1] + a[0][2] * C[0][2];
      const double f = op.g.cell[3 * cs + ix] * T.gw[qi[0]] * T.gw[qi[1]] * T.gw[qi[2]] / det;
      const int rb[6] = {0, 0, 0, 1, 1, 2}, rc[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
      for (int e = 0; e < 6; ++e)
        m[e] = f * (C[rb[e]][0] * C[rc[e]][0] + C[rb[e]][1] * C[rc[e]][1] + C[rb[e]][2] * C[rc[e]][2]);
    } else {
      double f;
      if constexpr (GK == AFFINE_VAR) f = op.g.cell[ix];
      else f = op.c_vol * T.gw[i % N] * T.gw[(i / N) % N] * T.gw[i / N2];
      m[0] = f * op.inv_h[0] * op.inv_h[0];
      m[3] = f * op.inv_h[1] * op.inv_h[1];
      m[5] = f * op.inv_h[2] * op.inv_h[2];
      m[1] = m[2] = m[4] = 0.0;
    }
#pragma unroll
    for (int e = 0; e < 6; ++e) M[e * N3 + i] = m[e];
  }
  __syncthreads();
  const int id[3] = {i % N, (i / N) % N, i / N2};
  double acc = 0.0;
  // cell term, pair by pair: T1 = contraction over q1, T2 over q2, then q3
  const int pb[6] = {0, 0, 0, 1, 1, 2}, pc[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    const int b = pb[e], c = pc[e];
    if ((GK == AFFINE_VAR || GK == AFFINE_CONST) && b != c) continue;  // M is diagonal there
    auto F = [&](int d, int q, int j) {
      const double eb = (b == d ? Dl : Sl)[q * N + j];
      const double ec = (c == d ? Dl : Sl)[q * N + j];
      return eb * ec;
    };
    if (act) {
      double s = 0.0;
      for (int q1 = 0; q1 < N; ++q1) s += M[e * N3 + q1 + N * id[1] + N2 * id[2]] * F(0, q1, id[0]);
      T1[i] = s;   // [i1, q2, q3]
    }
    __syncthreads();
    if (act) {
      double s = 0.0;
      for (int q2 = 0; q2 < N; ++q2) s += T1[id[0] + N * q2 + N2 * id[2]] * F(1, q2, id[1]);
      T2[i] = s;   // [i1, i2, q3]
    }
    __syncthreads();
    if (act) {
      double s = 0.0;
      for (int q3 = 0; q3 < N; ++q3) s += T2[id[0] + N * id[1] + N2 * q3] * F(2, q3, id[2]);
      acc += (b == c ? 1.0 : 2.0) * s;
    }
    __syncthreads();
  }
  if (!act) return;
  int ci[3];
  ci[0] = cell % op.ncell[0];
  ci[1] = (cell / op.ncell[0]) % op.ncell[1];
  ci[2] = cell / (op.ncell[0] * op.ncell[1]);
  auto sc = [&](int d, int q) { return Sl[q * N + id[d]]; };
  auto dc = [&](int d, int q) { return Dl[q * N + id[d]]; };
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int t1 = (a == 0) ? 1 : 0, t2 = (a == 2) ? 1 : 2;
    for (int s = 0; s < 2; ++s) {
      if (id[a] != (s ? N - 1 : 0)) continue;
      const int cn = ci[a] + (s ? 1 : -1);
      const bool interior = (cn >= 0 && cn < op.ncell[a]) || op.bc[2 * a + s] == kBcGhost;
      double mult = 1.0;
      if (!interior) mult = (op.bc[2 * a + s] == 0) ? 2.0 : 0.0;
      if (mult == 0.0) continue;
      const double fa = Fe[(s ? N : 0) + id[a]];
      const double sg = s ? 1.0 : -1.0;
      int p[3] = {ci[0], ci[1], ci[2]}, m[3] = {op.ncell[0], op.ncell[1], op.ncell[2]};
      p[a] += s;
      m[a] += 1;
      const int64_t fid = p[0] + (int64_t)m[0] * (p[1] + (int64_t)m[1] * p[2]);
      for (int q2 = 0; q2 < N; ++q2)
        for (int q1 = 0; q1 < N; ++q1) {
          const int lq = q1 + N * q2;
          const double phi = sc(t1, q1) * sc(t2, q2);
          double g[3];
          g[a] = fa * phi;
          g[t1] = dc(t1, q1) * sc(t2, q2);
          g[t2] = sc(t1, q1) * dc(t2, q2);
          double j[3] = {0.0, 0.0, 0.0}, cds;
          if constexpr (curved_faces(GK)) {
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

}  // namespace dgk

#include "advection.hpp"

namespace dgk {

// f(gk, bs) with the geometry kind of the op's FP64 or FP32 data and its
// basis as compile-time constants (the Hermite-like basis exists from N = 4 on)
template <int N, typename F>
__host__ void sipg_variant(const dg_op *op, bool f32, F &&f)
{
  auto with_gk = [&](auto bs) {
    switch (f32 ? op->gk32 : op->gk) {
      case CURVED: f(std::integral_constant<int, CURVED>{}, bs); break;
      case CURVED_MERGED: f(std::integral_constant<int, CURVED_MERGED>{}, bs); break;
      case CURVED_POS: f(std::integral_constant<int, CURVED_POS>{}, bs); break;
      case AFFINE_VAR: f(std::integral_constant<int, AFFINE_VAR>{}, bs); break;
      default: f(std::integral_constant<int, AFFINE_CONST>{}, bs); break;
    }
  };
  if constexpr (N >= 4) {
    if (op->basis == BASIS_HERMITE) {
      with_gk(std::integral_constant<int, BASIS_HERMITE>{});
      return;
    }
  }
  with_gk(std::integral_constant<int, BASIS_NODAL>{});
}

// ghost: per side, the trace buffer read where mesh.bc is DG_BC_GHOST (an
// array of 6 device pointers of the vectors' type, or null when no side is)
template <int N>
hipError_t launch_apply(const dg_op *op, const void *src, void *dst, bool f32, hipStream_t s,
                        const void *const *ghost)
{
  using BK = Blocking<N>;
  const int grid = (int)((op->ncells + BK::B - 1) / BK::B);
  if (grid == 0) return hipSuccess;
  auto go = [&](auto zero, const auto &view) {
    using Real = decltype(zero);
    const Real *x = static_cast<const Real *>(src);
    Real *y = static_cast<Real *>(dst);
    if (op->gk == ADVECTION) {
      hipLaunchKernelGGL((adv_apply_kernel<N, Real>), dim3(grid), dim3(BK::TPB), 0, s, view, x, y);
      return;
    }
    auto v = view;
    v.reverse = (int)(op->sweeps.fetch_add(1, std::memory_order_relaxed) & 1u);
    if (ghost) {
      // ops with ghost sides run their own instantiation, so that the
      // others carry no trace of it
      for (int f = 0; f < 6; ++f) v.ghost[f] = static_cast<const Real *>(ghost[f]);
      sipg_variant<N>(op, f32, [&](auto gk, auto bs) {
        hipLaunchKernelGGL((sipg_apply_kernel<N, Real, decltype(gk)::value, false, decltype(bs)::value, true>),
                           dim3(grid), dim3(BK::TPB), 0, s, v, x, y, DotOut<Real>{});
      });
      return;
    }
    sipg_variant<N>(op, f32, [&](auto gk, auto bs) {
      hipLaunchKernelGGL((sipg_apply_kernel<N, Real, decltype(gk)::value, false, decltype(bs)::value>), dim3(grid),
                         dim3(BK::TPB), 0, s, v, x, y, DotOut<Real>{});
    });
  };
  if (f32) go(0.0f, op->v32);
  else go(0.0, op->v64);
  return hipGetLastError();
}

// the SIPG apply that also writes the workgroup shares of src.(A src) (FP32
// or FP64 as the vectors) into part, apply_workgroups(op) entries
template <int N>
hipError_t launch_apply_dot(const dg_op *op, const void *src, void *dst, bool f32, void *part, hipStream_t s)
{
  using BK = Blocking<N>;
  const int grid = (int)((op->ncells + BK::B - 1) / BK::B);
  if (grid == 0) return hipSuccess;
  auto go = [&](auto zero, const auto &view) {
    using Real = decltype(zero);
    const Real *x = static_cast<const Real *>(src);
    Real *y = static_cast<Real *>(dst);
    DotOut<Real> d{static_cast<Real *>(part)};
    auto v = view;
    v.reverse = (int)(op->sweeps.fetch_add(1, std::memory_order_relaxed) & 1u);
    sipg_variant<N>(op, f32, [&](auto gk, auto bs) {
      hipLaunchKernelGGL((sipg_apply_kernel<N, Real, decltype(gk)::value, true, decltype(bs)::value>), dim3(grid),
                         dim3(BK::TPB), 0, s, v, x, y, d);
    });
  };
  if (f32) go(0.0f, op->v32);
  else go(0.0, op->v64);
  return hipGetLastError();
}

template <int N>
int apply_workgroups(const dg_op *op)
{
  return (int)((op->ncells + Blocking<N>::B - 1) / Blocking<N>::B);
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
  sipg_variant<N>(op, false, [&](auto gk, auto bs) {
    hipLaunchKernelGGL((sipg_diag_kernel<N, decltype(gk)::value, decltype(bs)::value>), dim3(grid), dim3(block), 0, s,
                       op->v64, d64, d32);
  });
  return hipGetLastError();
}

// Face traces of side 2A + s for the partition across it: for every cell of
// the side's layer and face node l, the value and the reference normal
// derivative at xi_A = s, i.e. the S_f and D_f rows of Eq. (7) applied to
// the cell's normal line through l.  These are the products, in the same
// order, that a cell of the neighbouring partition forms from an in-memory
// neighbour (the face pass, S1), so a ghost face sees the same numbers.
constexpr int kTraceThreads = 256;
template <int N, typename Real, int A, int BS>
__global__ void __launch_bounds__(kTraceThreads)
face_traces_kernel(const int3 nc, int s, const Real *__restrict__ src, Real *__restrict__ out, int64_t nplane)
{
  constexpr int N2 = N * N, N3 = N2 * N;
  constexpr int t1 = (A == 0) ? 1 : 0, t2 = (A == 2) ? 1 : 2;
  constexpr BasisTables<N> BT = kBasis<N, BS>;
  const int64_t i = (int64_t)blockIdx.x * kTraceThreads + threadIdx.x;
  if (i >= nplane * N2) return;
  const int64_t p = i / N2;
  const int l = (int)(i - p * N2);
  const int n[3] = {nc.x, nc.y, nc.z};
  int ci[3];
  ci[t1] = (int)(p % n[t1]);
  ci[t2] = (int)(p / n[t1]);
  ci[A] = s ? n[A] - 1 : 0;
  const int64_t cell = ci[0] + (int64_t)n[0] * (ci[1] + (int64_t)n[1] * ci[2]);
  const Real *line = src + cell * N3 + line_base<N, A>(l);
  Real val = Real(-0.0), der = Real(-0.0);
#pragma unroll
  for (int m = 0; m < N; ++m) {
    // the high side (s = 1) is the xi_A = 1 end: V1, F1; the low side V0, F0
    const double v = s ? BT.V1[m] : BT.V0[m], f = s ? BT.F1[m] : BT.F0[m];
    const Real u = (v != 0.0 || f != 0.0) ? line[m * kStride<N, A>] : Real(0);
    if (s) {
      val = madd(BT.V1[m], u, val);
      der = madd(BT.F1[m], u, der);
    } else {
      val = madd(BT.V0[m], u, val);
      der = madd(BT.F0[m], u, der);
    }
  }
  out[p * 2 * N2 + l] = val;
  out[p * 2 * N2 + N2 + l] = der;
}

template <int N>
hipError_t launch_face_traces(const dg_op *op, int side, const void *src, void *out, bool f32, hipStream_t s)
{
  const int a = side / 2, hi = side % 2;
  const int t1 = (a == 0) ? 1 : 0, t2 = (a == 2) ? 1 : 2;
  const int64_t nplane = (int64_t)op->mesh.ncell[t1] * op->mesh.ncell[t2];
  const int64_t threads = nplane * N * N;
  const int grid = (int)((threads + kTraceThreads - 1) / kTraceThreads);
  const int3 nc = make_int3(op->mesh.ncell[0], op->mesh.ncell[1], op->mesh.ncell[2]);
  auto go = [&](auto zero, auto bs) {
    using Real = decltype(zero);
    constexpr int BS = decltype(bs)::value;
    const Real *x = static_cast<const Real *>(src);
    Real *y = static_cast<Real *>(out);
    switch (a) {
      case 0: hipLaunchKernelGGL((face_traces_kernel<N, Real, 0, BS>), dim3(grid), dim3(kTraceThreads), 0, s, nc, hi, x, y, nplane); break;
      case 1: hipLaunchKernelGGL((face_traces_kernel<N, Real, 1, BS>), dim3(grid), dim3(kTraceThreads), 0, s, nc, hi, x, y, nplane); break;
      default: hipLaunchKernelGGL((face_traces_kernel<N, Real, 2, BS>), dim3(grid), dim3(kTraceThreads), 0, s, nc, hi, x, y, nplane); break;
    }
  };
  auto with_basis = [&](auto zero) {
    if constexpr (N >= 4) {
      if (op->basis == BASIS_HERMITE) {
        go(zero, std::integral_constant<int, BASIS_HERMITE>{});
        return;
      }
    }
    go(zero, std::integral_constant<int, BASIS_NODAL>{});
  };
  if (grid == 0) return hipSuccess;
  if (f32) with_basis(0.0f);
  else with_basis(0.0);
  return hipGetLastError();
}

}  // namespace dgk
