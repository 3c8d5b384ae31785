// dg_ops.hip -- operator setup (geometry at the quadrature points, on the
// device), the C-ABI entry points for apply / diagonal / load vector / error
// norms, and the per-degree dispatch.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "dg_internal.hpp"
#include "kernels.hpp"

namespace dgk {

// the kernels themselves are instantiated once per N in inst.hip
#define DG_EXTERN_N(N)                                                                  \
  extern template hipError_t launch_apply<N>(const dg_op *, const void *, void *, bool, \
                                             hipStream_t, const void *const *);         \
  extern template hipError_t launch_face_traces<N>(const dg_op *, int, const void *, void *, bool, \
                                                   hipStream_t);                                   \
  extern template hipError_t launch_diag<N>(const dg_op *, void *, void *, hipStream_t);        \
  extern template hipError_t launch_apply_dot<N>(const dg_op *, const void *, void *, bool,    \
                                                 void *, hipStream_t);                          \
  extern template int apply_workgroups<N>(const dg_op *);
DG_EXTERN_N(2)
DG_EXTERN_N(3)
DG_EXTERN_N(4)
DG_EXTERN_N(5)
DG_EXTERN_N(6)
DG_EXTERN_N(7)
DG_EXTERN_N(8)
DG_EXTERN_N(9)
#undef DG_EXTERN_N

static thread_local std::string g_error;

void set_error(const std::string &msg) { g_error = msg; }

dg_status fail(dg_status st, const std::string &msg)
{
  g_error = msg;
  return st;
}

dg_status hip_fail(hipError_t e, const char *what)
{
  g_error = std::string(what) + ": " + hipGetErrorString(e);
  return DG_ERR_HIP;
}

void *op_alloc(dg_op *op, size_t bytes)
{
  if (bytes == 0) bytes = 256;
  if (!op->own_alloc) return op->alloc.alloc(bytes, op->alloc.ctx);
  void *p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
  return p;
}

void op_free(dg_op *op, void *p)
{
  if (!p) return;
  if (!op->own_alloc) op->alloc.free(p, op->alloc.ctx);
  else (void)hipFree(p);
}

hipError_t launch_apply_any(const dg_op *op, const void *src, void *dst, bool f32, hipStream_t s,
                            const void *const *ghost)
{
  switch (op->n) {
    case 2: return launch_apply<2>(op, src, dst, f32, s, ghost);
    case 3: return launch_apply<3>(op, src, dst, f32, s, ghost);
    case 4: return launch_apply<4>(op, src, dst, f32, s, ghost);
    case 5: return launch_apply<5>(op, src, dst, f32, s, ghost);
    case 6: return launch_apply<6>(op, src, dst, f32, s, ghost);
    case 7: return launch_apply<7>(op, src, dst, f32, s, ghost);
    case 8: return launch_apply<8>(op, src, dst, f32, s, ghost);
    case 9: return launch_apply<9>(op, src, dst, f32, s, ghost);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_apply_dot_any(const dg_op *op, const void *src, void *dst, bool f32, void *part, hipStream_t s)
{
  switch (op->n) {
    case 2: return launch_apply_dot<2>(op, src, dst, f32, part, s);
    case 3: return launch_apply_dot<3>(op, src, dst, f32, part, s);
    case 4: return launch_apply_dot<4>(op, src, dst, f32, part, s);
    case 5: return launch_apply_dot<5>(op, src, dst, f32, part, s);
    case 6: return launch_apply_dot<6>(op, src, dst, f32, part, s);
    case 7: return launch_apply_dot<7>(op, src, dst, f32, part, s);
    case 8: return launch_apply_dot<8>(op, src, dst, f32, part, s);
    case 9: return launch_apply_dot<9>(op, src, dst, f32, part, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_face_traces_any(const dg_op *op, int side, const void *src, void *out, bool f32, hipStream_t s)
{
  switch (op->n) {
    case 2: return launch_face_traces<2>(op, side, src, out, f32, s);
    case 3: return launch_face_traces<3>(op, side, src, out, f32, s);
    case 4: return launch_face_traces<4>(op, side, src, out, f32, s);
    case 5: return launch_face_traces<5>(op, side, src, out, f32, s);
    case 6: return launch_face_traces<6>(op, side, src, out, f32, s);
    case 7: return launch_face_traces<7>(op, side, src, out, f32, s);
    case 8: return launch_face_traces<8>(op, side, src, out, f32, s);
    case 9: return launch_face_traces<9>(op, side, src, out, f32, s);
    default: return hipErrorInvalidValue;
  }
}

int apply_workgroups_any(const dg_op *op)
{
  switch (op->n) {
    case 2: return apply_workgroups<2>(op);
    case 3: return apply_workgroups<3>(op);
    case 4: return apply_workgroups<4>(op);
    case 5: return apply_workgroups<5>(op);
    case 6: return apply_workgroups<6>(op);
    case 7: return apply_workgroups<7>(op);
    case 8: return apply_workgroups<8>(op);
    case 9: return apply_workgroups<9>(op);
    default: return 0;
  }
}

hipError_t launch_diag_any(const dg_op *op, void *d64, void *d32, hipStream_t s)
{
  switch (op->n) {
    case 2: return launch_diag<2>(op, d64, d32, s);
    case 3: return launch_diag<3>(op, d64, d32, s);
    case 4: return launch_diag<4>(op, d64, d32, s);
    case 5: return launch_diag<5>(op, d64, d32, s);
    case 6: return launch_diag<6>(op, d64, d32, s);
    case 7: return launch_diag<7>(op, d64, d32, s);
    case 8: return launch_diag<8>(op, d64, d32, s);
    case 9: return launch_diag<9>(op, d64, d32, s);
    default: return hipErrorInvalidValue;
  }
}

// 1D rules for a runtime number of points (from the compile-time tables)
struct Rule1D {
  int n = 0;
  double x[12], w[12];
};
template <int N>
static void fill_rule(Rule1D &r)
{
  r.n = N;
  for (int i = 0; i < N; ++i) {
    r.x[i] = kTab<N>.gx[i];
    r.w[i] = kTab<N>.gw[i];
  }
}
static bool rule_for(int n, Rule1D &r)
{
  switch (n) {
    case 2: fill_rule<2>(r); return true;
    case 3: fill_rule<3>(r); return true;
    case 4: fill_rule<4>(r); return true;
    case 5: fill_rule<5>(r); return true;
    case 6: fill_rule<6>(r); return true;
    case 7: fill_rule<7>(r); return true;
    case 8: fill_rule<8>(r); return true;
    case 9: fill_rule<9>(r); return true;
    case 10: fill_rule<10>(r); return true;
    case 11: fill_rule<11>(r); return true;
    default: return false;
  }
}

// ---------------------------------------------------------------------------
// Geometry on the device.  x = X + a s(X) (1,1,1), s = sin(2 pi X) sin(2 pi Y)
// sin(2 pi Z); grad Phi = I + 1 (a grad s)^T, whose inverse and determinant
// follow from the rank-one structure (Sherman-Morrison, determinant lemma).
// J = grad Phi diag(h) maps the unit reference cell.
// ---------------------------------------------------------------------------
struct GeoArgs {
  int ncell[3];
  double lo[3], h[3];
  int map, coef;
  double amp, cval;
  int vel;            // advection velocity kind
  double vval[3];
  Rule1D rule;
};

__device__ __forceinline__ void map_point(const GeoArgs &g, const double X[3], double x[3],
                                          double Ginv[3][3], double &detG)
{
  if (g.map == DG_MAP_AFFINE) {
    for (int i = 0; i < 3; ++i) {
      x[i] = X[i];
      for (int j = 0; j < 3; ++j) Ginv[i][j] = (i == j) ? 1.0 : 0.0;
    }
    detG = 1.0;
    return;
  }
  const double tp = 2.0 * kPi;
  double sn[3], cs[3];
  for (int d = 0; d < 3; ++d) sincos(tp * X[d], &sn[d], &cs[d]);
  const double disp = g.amp * sn[0] * sn[1] * sn[2];
  const double ds[3] = {g.amp * tp * cs[0] * sn[1] * sn[2], g.amp * tp * sn[0] * cs[1] * sn[2],
                        g.amp * tp * sn[0] * sn[1] * cs[2]};
  detG = 1.0 + ds[0] + ds[1] + ds[2];
  const double inv = 1.0 / detG;
  for (int i = 0; i < 3; ++i) {
    x[i] = X[i] + disp;
    for (int j = 0; j < 3; ++j) Ginv[i][j] = ((i == j) ? 1.0 : 0.0) - ds[j] * inv;
  }
}

// transport velocity of the advection operator at the physical point x
__device__ __forceinline__ void velocity_value(const GeoArgs &g, const double x[3], double v[3])
{
  if (g.vel == DG_VEL_CONST) {
    for (int d = 0; d < 3; ++d) v[d] = g.vval[d];
  } else {
    v[0] = 0.5 - x[1];
    v[1] = x[0] - 0.5;
    v[2] = 0.25;
  }
}

__device__ __forceinline__ double coef_value(const GeoArgs &g, const double x[3])
{
  if (g.coef == DG_COEF_CONST) return g.cval;
  return 1.0 + 0.5 * sin(kPi * x[0]) * cos(kPi * x[1]) * x[2];
}

template <int GK>
__global__ void geom_cells_kernel(const GeoArgs g, int64_t npts, double *o64, float *o32, int64_t stride, int group)
{
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= npts) return;
  const int n = g.rule.n, n2 = n * n, n3 = n2 * n;
  const int64_t cell = idx / n3;
  const int q = (int)(idx - cell * n3);
  // the grouped layout the apply kernels read (geo_base / geo_off)
  const int64_t grp = cell / group;
  const int64_t at = ((grp * n + q / n2) * group + (cell - grp * group)) * n2 + q % n2;
  const int qi[3] = {q % n, (q / n) % n, q / (n * n)};
  const int ci[3] = {(int)(cell % g.ncell[0]), (int)((cell / g.ncell[0]) % g.ncell[1]),
                     (int)(cell / ((int64_t)g.ncell[0] * g.ncell[1]))};
  double X[3], x[3], Gi[3][3], detG;
  for (int d = 0; d < 3; ++d) X[d] = g.lo[d] + (ci[d] + g.rule.x[qi[d]]) * g.h[d];
  map_point(g, X, x, Gi, detG);
  const double W = g.rule.w[qi[0]] * g.rule.w[qi[1]] * g.rule.w[qi[2]];
  const double cjxw = coef_value(g, x) * detG * g.h[0] * g.h[1] * g.h[2] * W;
  if (GK == CURVED) {
    // J^{-T}[a][b] = J^{-1}[b][a] = Ginv[b][a] / h_b
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        const double v = Gi[b][a] / g.h[b];
        if (o64) o64[(3 * a + b) * stride + at] = v;
        if (o32) o32[(3 * a + b) * stride + at] = (float)v;
      }
    if (o64) o64[9 * stride + at] = cjxw;
    if (o32) o32[9 * stride + at] = (float)cjxw;
  } else if (GK == ADVECTION) {
    // t = J^{-1} c det J w: J^{-1}[b][c] = Ginv[b][c] / h_b
    double v[3];
    velocity_value(g, x, v);
    const double jxw = detG * g.h[0] * g.h[1] * g.h[2] * W;
    for (int b = 0; b < 3; ++b) {
      const double t = (Gi[b][0] * v[0] + Gi[b][1] * v[1] + Gi[b][2] * v[2]) / g.h[b] * jxw;
      if (o64) o64[b * stride + at] = t;
      if (o32) o32[b * stride + at] = (float)t;
    }
  } else if (GK == CURVED_POS) {
    // the point relative to the cell's unmapped corner (small numbers, so
    // that FP32 keeps the differences the collocation derivative takes), and c
    for (int d = 0; d < 3; ++d) {
      const double v = x[d] - (g.lo[d] + ci[d] * g.h[d]);
      if (o64) o64[d * stride + at] = v;
      if (o32) o32[d * stride + at] = (float)v;
    }
    const double c = coef_value(g, x);
    if (o64) o64[3 * stride + at] = c;
    if (o32) o32[3 * stride + at] = (float)c;
  } else if (GK == CURVED_MERGED) {
    // M = c det J w J^{-1} J^{-T}: M[b][c] = cjxw sum_a J^{-T}[a][b] J^{-T}[a][c]
    double jt[3][3];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) jt[a][b] = Gi[b][a] / g.h[b];
    const int rb[6] = {0, 0, 0, 1, 1, 2}, rc[6] = {0, 1, 2, 1, 2, 2};
    for (int e = 0; e < 6; ++e) {
      const double v = cjxw * (jt[0][rb[e]] * jt[0][rc[e]] + jt[1][rb[e]] * jt[1][rc[e]] + jt[2][rb[e]] * jt[2][rc[e]]);
      if (o64) o64[e * stride + at] = v;
      if (o32) o32[e * stride + at] = (float)v;
    }
  } else {
    if (o64) o64[at] = cjxw;
    if (o32) o32[at] = (float)cjxw;
  }
}

template <int GK>
__global__ void geom_faces_kernel(const GeoArgs g, int a, int64_t npts, double *o64, float *o32, int64_t stride)
{
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= npts) return;
  const int n = g.rule.n, n2 = n * n;
  const int64_t f = idx / n2;
  const int lq = (int)(idx - f * n2);
  const int q1 = lq % n, q2 = lq / n;
  int m[3] = {g.ncell[0], g.ncell[1], g.ncell[2]};
  m[a] += 1;
  const int p[3] = {(int)(f % m[0]), (int)((f / m[0]) % m[1]), (int)(f / ((int64_t)m[0] * m[1]))};
  const int t1 = (a == 0) ? 1 : 0, t2 = (a == 2) ? 1 : 2;
  double X[3], x[3], Gi[3][3], detG;
  X[a] = g.lo[a] + p[a] * g.h[a];
  X[t1] = g.lo[t1] + (p[t1] + g.rule.x[q1]) * g.h[t1];
  X[t2] = g.lo[t2] + (p[t2] + g.rule.x[q2]) * g.h[t2];
  map_point(g, X, x, Gi, detG);
  const double w = g.rule.w[q1] * g.rule.w[q2];
  const double c = coef_value(g, x);
  if (GK == CURVED) {
    // J^{-T} e_a has components J^{-1}[a][b] = Ginv[a][b] / h_a
    double v[3], nv = 0.0;
    for (int b = 0; b < 3; ++b) {
      v[b] = Gi[a][b] / g.h[a];
      nv += v[b] * v[b];
    }
    nv = sqrt(nv);
    double nrm[3] = {v[0] / nv, v[1] / nv, v[2] / nv};
    const double cds = c * detG * g.h[0] * g.h[1] * g.h[2] * nv * w;
    for (int cc = 0; cc < 3; ++cc) {
      // j = J^{-1} n
      const double jc = (Gi[cc][0] * nrm[0] + Gi[cc][1] * nrm[1] + Gi[cc][2] * nrm[2]) / g.h[cc];
      if (o64) o64[cc * stride + idx] = jc;
      if (o32) o32[cc * stride + idx] = (float)jc;
    }
    if (o64) o64[3 * stride + idx] = cds;
    if (o32) o32[3 * stride + idx] = (float)cds;
  } else if (GK == ADVECTION) {
    // (c . n) ds for the +e_a normal: Nanson, n ds = det J J^{-T} e_a w, and
    // (J^{-T} e_a)_b = J^{-1}[a][b] = Ginv[a][b] / h_a
    double v[3];
    velocity_value(g, x, v);
    const double cn = detG * g.h[0] * g.h[1] * g.h[2] * w *
                      (Gi[a][0] * v[0] + Gi[a][1] * v[1] + Gi[a][2] * v[2]) / g.h[a];
    if (o64) o64[idx] = cn;
    if (o32) o32[idx] = (float)cn;
  } else {
    const double cds = c * g.h[t1] * g.h[t2] * w;
    if (o64) o64[idx] = cds;
    if (o32) o32[idx] = (float)cds;
  }
}

// ---------------------------------------------------------------------------
// Manufactured load vector and error norms (FP64)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double forcing(const GeoArgs &g, const double x[3], double &u, double gu[3])
{
  double sn[3], cs[3];
  for (int d = 0; d < 3; ++d) sincos(kPi * x[d], &sn[d], &cs[d]);
  u = sn[0] * sn[1] * sn[2];
  gu[0] = kPi * cs[0] * sn[1] * sn[2];
  gu[1] = kPi * sn[0] * cs[1] * sn[2];
  gu[2] = kPi * sn[0] * sn[1] * cs[2];
  const double c = coef_value(g, x);
  double gc[3] = {0.0, 0.0, 0.0};
  if (g.coef == DG_COEF_SINCOS) {
    gc[0] = 0.5 * kPi * cs[0] * cs[1] * x[2];
    gc[1] = -0.5 * kPi * sn[0] * sn[1] * x[2];
    gc[2] = 0.5 * sn[0] * cs[1];
  }
  return -(gc[0] * gu[0] + gc[1] * gu[1] + gc[2] * gu[2]) + 3.0 * kPi * kPi * c * u;
}

// one workgroup per cell: f det J w at the Gauss points into LDS, then
// b = (S^T x S^T x S^T) of it, S of the op's basis BS
template <int N, int BS>
__global__ void __launch_bounds__(1024) rhs_kernel(const GeoArgs g, double *__restrict__ b)
{
  constexpr int N2 = N * N, N3 = N2 * N;
  constexpr const auto &T = kTab<N>;
  constexpr const auto &BT = kBasis<N, BS>;
  __shared__ double F[N3];
  const int64_t cell = blockIdx.x;
  const int t = threadIdx.x;
  const int ci[3] = {(int)(cell % g.ncell[0]), (int)((cell / g.ncell[0]) % g.ncell[1]),
                     (int)(cell / ((int64_t)g.ncell[0] * g.ncell[1]))};
  if (t < N3) {
    const int qi[3] = {t % N, (t / N) % N, t / N2};
    double X[3], x[3], Gi[3][3], detG, u, gu[3];
    for (int d = 0; d < 3; ++d) X[d] = g.lo[d] + (ci[d] + T.gx[qi[d]]) * g.h[d];
    map_point(g, X, x, Gi, detG);
    F[t] = forcing(g, x, u, gu) * detG * g.h[0] * g.h[1] * g.h[2] * T.gw[qi[0]] * T.gw[qi[1]] * T.gw[qi[2]];
  }
  __syncthreads();
  if (t >= N3) return;
  const int id[3] = {t % N, (t / N) % N, t / N2};
  double acc = 0.0;
  for (int q = 0; q < N3; ++q) {
    const int q1 = q % N, q2 = (q / N) % N, q3 = q / N2;
    acc += BT.S[q1][id[0]] * BT.S[q2][id[1]] * BT.S[q3][id[2]] * F[q];
  }
  b[cell * N3 + t] = acc;
}

// error integrals with M points per direction; per-cell partial sums; the
// coefficients xv are in the op's basis BS
template <int N, int M, int BS>
__global__ void __launch_bounds__(1024) error_kernel(const GeoArgs g, const double *__restrict__ xv,
                                                     double *__restrict__ part)
{
  constexpr int N2 = N * N, N3 = N2 * N, M3 = M * M * M;
  constexpr const auto &TN = kTab<N>;
  constexpr const auto &TM = kTab<M>;
  constexpr const auto &BT = kBasis<N, BS>;
  __shared__ double u[N3];
  __shared__ double red[2][1024];
  const int64_t cell = blockIdx.x;
  const int t = threadIdx.x;
  for (int i = t; i < N3; i += blockDim.x) u[i] = xv[cell * N3 + i];
  __syncthreads();
  // Gauss-Lobatto Lagrange basis at the M-point Gauss nodes (then the op's basis)
  double lam[N];
  for (int j = 0; j < N; ++j) {
    double p = 1.0;
    for (int m = 0; m < N; ++m)
      if (m != j) p *= (TN.lx[j] - TN.lx[m]);
    lam[j] = 1.0 / p;
  }
  const int ci[3] = {(int)(cell % g.ncell[0]), (int)((cell / g.ncell[0]) % g.ncell[1]),
                     (int)(cell / ((int64_t)g.ncell[0] * g.ncell[1]))};
  double s0 = 0.0, s1 = 0.0;
  for (int q = t; q < M3; q += blockDim.x) {
    const int qi[3] = {q % M, (q / M) % M, q / (M * M)};
    double V[3][N], D[3][N];
    for (int d = 0; d < 3; ++d) {
      const double xi = TM.gx[qi[d]];
      for (int j = 0; j < N; ++j) {
        double v = lam[j], dd = 0.0;
        for (int m = 0; m < N; ++m) {
          if (m == j) continue;
          dd = dd * (xi - TN.lx[m]) + v;
          v *= (xi - TN.lx[m]);
        }
        V[d][j] = v;
        D[d][j] = dd;
      }
      if constexpr (BS != BASIS_NODAL) {
        // phi_j = sum_i C[i][j] l_i
        double v2[N], d2[N];
        for (int j = 0; j < N; ++j) {
          v2[j] = d2[j] = 0.0;
          for (int i = 0; i < N; ++i) {
            v2[j] += V[d][i] * BT.C[i][j];
            d2[j] += D[d][i] * BT.C[i][j];
          }
        }
        for (int j = 0; j < N; ++j) {
          V[d][j] = v2[j];
          D[d][j] = d2[j];
        }
      }
    }
    double uh = 0.0, gr[3] = {0.0, 0.0, 0.0};
    for (int i3 = 0; i3 < N; ++i3)
      for (int i2 = 0; i2 < N; ++i2)
        for (int i1 = 0; i1 < N; ++i1) {
          const double c = u[i1 + N * i2 + N2 * i3];
          uh += c * V[0][i1] * V[1][i2] * V[2][i3];
          gr[0] += c * D[0][i1] * V[1][i2] * V[2][i3];
          gr[1] += c * V[0][i1] * D[1][i2] * V[2][i3];
          gr[2] += c * V[0][i1] * V[1][i2] * D[2][i3];
        }
    double X[3], x[3], Gi[3][3], detG, ue, ge[3];
    for (int d = 0; d < 3; ++d) X[d] = g.lo[d] + (ci[d] + TM.gx[qi[d]]) * g.h[d];
    map_point(g, X, x, Gi, detG);
    (void)forcing(g, x, ue, ge);
    double gh[3];
    for (int a = 0; a < 3; ++a)
      gh[a] = Gi[0][a] * gr[0] / g.h[0] + Gi[1][a] * gr[1] / g.h[1] + Gi[2][a] * gr[2] / g.h[2];
    const double jw = detG * g.h[0] * g.h[1] * g.h[2] * TM.gw[qi[0]] * TM.gw[qi[1]] * TM.gw[qi[2]];
    s0 += (uh - ue) * (uh - ue) * jw;
    s1 += ((gh[0] - ge[0]) * (gh[0] - ge[0]) + (gh[1] - ge[1]) * (gh[1] - ge[1]) +
           (gh[2] - ge[2]) * (gh[2] - ge[2])) * jw;
  }
  red[0][t] = s0;
  red[1][t] = s1;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (t < w) {
      red[0][t] += red[0][t + w];
      red[1][t] += red[1][t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
    part[2 * cell] = red[0][0];
    part[2 * cell + 1] = red[1][0];
  }
}

static GeoArgs geo_args(const dg_op *op)
{
  GeoArgs g{};
  for (int d = 0; d < 3; ++d) {
    g.ncell[d] = op->mesh.ncell[d];
    g.lo[d] = op->mesh.lo[d];
    g.h[d] = op->h[d];
  }
  g.map = op->geom.map;
  g.amp = op->geom.amplitude;
  g.coef = op->coef.kind;
  g.cval = op->coef.value;
  g.vel = op->vel.kind;
  for (int d = 0; d < 3; ++d) g.vval[d] = op->vel.value[d];
  rule_for(op->n, g.rule);
  return g;
}

static int64_t geom_cell_values(int gk) { return cell_values(gk); }
static int64_t geom_face_values(int gk) { return face_values(gk); }

// geometry kind of the FP64 (f32 = false) or FP32 data
static int geom_kind(const dg_geometry *geom, const dg_coefficient *coef, bool f32 = false)
{
  if (geom->map == DG_MAP_SINE) {
    if (geom->storage == DG_STORE_POSITIONS) return CURVED_POS;
    if (geom->storage == DG_STORE_MERGED || (f32 && geom->storage == DG_STORE_MIXED)) return CURVED_MERGED;
    return CURVED;
  }
  return coef->kind == DG_COEF_SINCOS ? AFFINE_VAR : AFFINE_CONST;
}

// cells per group of the stored cell geometry layout (kGeoGroup<n>)
static int geo_group(int n)
{
  switch (n) {
    case 2: return kGeoGroup<2>;
    case 3: return kGeoGroup<3>;
    case 4: return kGeoGroup<4>;
    case 5: return kGeoGroup<5>;
    case 6: return kGeoGroup<6>;
    case 7: return kGeoGroup<7>;
    case 8: return kGeoGroup<8>;
    default: return kGeoGroup<9>;
  }
}

// cells the stored cell geometry arrays hold: ncells rounded up to whole groups
static int64_t geo_cells(int64_t ncells, int n)
{
  const int64_t g = geo_group(n);
  return (ncells + g - 1) / g * g;
}

static size_t footprint_bytes(const int64_t nc[3], int n, int gk64, int gk32, unsigned prec)
{
  const int64_t ncells = nc[0] * nc[1] * nc[2];
  const int64_t n2 = n * n, n3 = n2 * n;
  auto values = [&](int gk) {
    int64_t vals = geom_cell_values(gk) * geo_cells(ncells, n) * n3;
    for (int a = 0; a < 3; ++a) {
      const int64_t nf = ncells / nc[a] * (nc[a] + 1);
      vals += geom_face_values(gk) * nf * n2;
    }
    return vals;
  };
  size_t bytes = 0;
  if (prec & DG_PREC_F64) bytes += values(gk64) * 8 + ncells * n3 * 8;
  if (prec & DG_PREC_F32) bytes += values(gk32) * 4 + ncells * n3 * 4;
  return bytes;
}

static dg_status validate(const dg_mesh *mesh, int degree, const dg_geometry *geom, const dg_coefficient *coef,
                          unsigned precisions)
{
  if (!mesh || !geom || !coef) return fail(DG_ERR_ARG, "null argument");
  if (degree < 1) return fail(DG_ERR_ARG, "degree must be >= 1");
  if (degree + 1 > kMaxN) return fail(DG_ERR_UNSUPPORTED, "degree > 8 is not compiled in");
  int64_t ncells = 1;
  for (int d = 0; d < 3; ++d) {
    if (mesh->ncell[d] < 1) return fail(DG_ERR_ARG, "ncell must be >= 1 in every direction");
    if (!(mesh->hi[d] > mesh->lo[d])) return fail(DG_ERR_ARG, "box must have hi > lo");
    ncells *= mesh->ncell[d];
  }
  for (int f = 0; f < 6; ++f)
    if (mesh->bc[f] != DG_BC_DIRICHLET && mesh->bc[f] != DG_BC_NEUMANN && mesh->bc[f] != DG_BC_GHOST)
      return fail(DG_ERR_ARG, "bad bc");
  if (geom->map != DG_MAP_AFFINE && geom->map != DG_MAP_SINE) return fail(DG_ERR_ARG, "bad map");
  if (geom->storage != DG_STORE_JACOBIAN && geom->storage != DG_STORE_MERGED && geom->storage != DG_STORE_MIXED &&
      geom->storage != DG_STORE_POSITIONS)
    return fail(DG_ERR_ARG, "bad geometry storage");
  if (coef->kind != DG_COEF_CONST && coef->kind != DG_COEF_SINCOS) return fail(DG_ERR_ARG, "bad coefficient");
  if (precisions == 0 || (precisions & ~3u)) return fail(DG_ERR_ARG, "precisions must be a nonempty subset of F64|F32");
  const int64_t n = degree + 1;
  if (ncells * n * n * n > 2147483647LL) return fail(DG_ERR_UNSUPPORTED, "more than 2^31-1 DoFs");
  return DG_OK;
}

}  // namespace dgk

using namespace dgk;

extern "C" {

const char *dg_last_error(void) { return g_error.c_str(); }

dg_status dg_tables(int degree, double *out, size_t len)
{
  const int n = degree + 1;
  if (degree < 1 || n > kMaxN) return fail(DG_ERR_ARG, "degree out of range");
  if (!out || len < (size_t)(3 * n + 2 * n * n)) return fail(DG_ERR_ARG, "output too short");
  auto put = [&](const auto &T) {
    double *o = out;
    for (int i = 0; i < n; ++i) *o++ = T.gx[i];
    for (int i = 0; i < n; ++i) *o++ = T.gw[i];
    for (int i = 0; i < n; ++i) *o++ = T.lx[i];
    for (int q = 0; q < n; ++q)
      for (int j = 0; j < n; ++j) *o++ = T.S[q][j];
    for (int q = 0; q < n; ++q)
      for (int j = 0; j < n; ++j) *o++ = T.Dco[q][j];
  };
  switch (n) {
    case 2: put(kTab<2>); break;
    case 3: put(kTab<3>); break;
    case 4: put(kTab<4>); break;
    case 5: put(kTab<5>); break;
    case 6: put(kTab<6>); break;
    case 7: put(kTab<7>); break;
    case 8: put(kTab<8>); break;
    case 9: put(kTab<9>); break;
  }
  return DG_OK;
}

dg_status dg_basis_tables(int degree, dg_basis basis, double *out, size_t len)
{
  const int n = degree + 1;
  if (degree < 1 || n > kMaxN) return fail(DG_ERR_ARG, "degree out of range");
  if (basis != DG_BASIS_NODAL && basis != DG_BASIS_HERMITE) return fail(DG_ERR_ARG, "bad basis");
  if (basis == DG_BASIS_HERMITE && degree < 3) return fail(DG_ERR_ARG, "the Hermite-like basis needs degree >= 3");
  if (!out || len < (size_t)(2 * n * n + 4 * n)) return fail(DG_ERR_ARG, "output too short");
  auto put = [&](const auto &B) {
    double *o = out;
    for (int q = 0; q < n; ++q)
      for (int j = 0; j < n; ++j) *o++ = B.S[q][j];
    for (int q = 0; q < n; ++q)
      for (int j = 0; j < n; ++j) *o++ = B.D[q][j];
    for (int j = 0; j < n; ++j) *o++ = B.V0[j];
    for (int j = 0; j < n; ++j) *o++ = B.V1[j];
    for (int j = 0; j < n; ++j) *o++ = B.F0[j];
    for (int j = 0; j < n; ++j) *o++ = B.F1[j];
  };
  auto go = [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    if constexpr (N >= 4)
      if (basis == DG_BASIS_HERMITE) {
        put(kBasis<N, BASIS_HERMITE>);
        return;
      }
    put(kBasis<N, BASIS_NODAL>);
  };
  switch (n) {
    case 2: go(std::integral_constant<int, 2>{}); break;
    case 3: go(std::integral_constant<int, 3>{}); break;
    case 4: go(std::integral_constant<int, 4>{}); break;
    case 5: go(std::integral_constant<int, 5>{}); break;
    case 6: go(std::integral_constant<int, 6>{}); break;
    case 7: go(std::integral_constant<int, 7>{}); break;
    case 8: go(std::integral_constant<int, 8>{}); break;
    case 9: go(std::integral_constant<int, 9>{}); break;
  }
  return DG_OK;
}

dg_status dg_footprint(const dg_mesh *mesh, int degree, const dg_geometry *geom, const dg_coefficient *coef,
                       unsigned precisions, size_t *bytes)
{
  dg_status st = validate(mesh, degree, geom, coef, precisions);
  if (st != DG_OK) return st;
  if (!bytes) return fail(DG_ERR_ARG, "bytes is null");
  const int64_t nc[3] = {mesh->ncell[0], mesh->ncell[1], mesh->ncell[2]};
  *bytes = footprint_bytes(nc, degree + 1, geom_kind(geom, coef), geom_kind(geom, coef, true), precisions);
  return DG_OK;
}

dg_status dg_footprint_advection(const dg_mesh *mesh, int degree, const dg_geometry *geom, const dg_velocity *vel,
                                 unsigned precisions, size_t *bytes)
{
  const dg_coefficient one{DG_COEF_CONST, 1.0};
  dg_status st = validate(mesh, degree, geom, &one, precisions);
  if (st != DG_OK) return st;
  if (!vel || (vel->kind != DG_VEL_CONST && vel->kind != DG_VEL_ROTATION)) return fail(DG_ERR_ARG, "bad velocity");
  for (int f = 0; f < 6; ++f)
    if (mesh->bc[f] == DG_BC_GHOST)
      return fail(DG_ERR_UNSUPPORTED, "ghost sides are implemented for the SIPG operator only");
  if (!bytes) return fail(DG_ERR_ARG, "bytes is null");
  const int64_t nc[3] = {mesh->ncell[0], mesh->ncell[1], mesh->ncell[2]};
  *bytes = footprint_bytes(nc, degree + 1, ADVECTION, ADVECTION, precisions) -
           (size_t)(nc[0] * nc[1] * nc[2]) * (degree + 1) * (degree + 1) * (degree + 1) *
               (((precisions & DG_PREC_F64) ? 8 : 0) + ((precisions & DG_PREC_F32) ? 4 : 0));  // no diagonal
  return DG_OK;
}

int64_t dg_n_dofs(const dg_op *op) { return op ? op->ndofs : -1; }

dg_status dg_destroy(dg_op *op)
{
  if (!op) return DG_OK;
  for (int p = 0; p < 2; ++p) {
    op_free(op, op->cell_geo[p]);
    for (int a = 0; a < 3; ++a) op_free(op, op->face_geo[p][a]);
    op_free(op, op->diag[p]);
  }
  op_free(op, op->scratch);
  delete op;
  return DG_OK;
}

}  // extern "C"

// the SIPG op (vel == nullptr) in the given basis or the advection op with
// velocity vel (nodal basis)
static dg_status setup_impl(const dg_mesh *mesh, int degree, int basis, const dg_geometry *geom,
                            const dg_coefficient *coef, const dg_velocity *vel, unsigned precisions,
                            const dg_allocator *alloc, void *stream, dg_op **out)
{
  dg_status st = validate(mesh, degree, geom, coef, precisions);
  if (st != DG_OK) return st;
  bool ghost_sides = false;
  for (int f = 0; f < 6; ++f) ghost_sides = ghost_sides || mesh->bc[f] == DG_BC_GHOST;
  if (vel && ghost_sides) return fail(DG_ERR_UNSUPPORTED, "ghost sides are implemented for the SIPG operator only");
  if (basis != DG_BASIS_NODAL && basis != DG_BASIS_HERMITE) return fail(DG_ERR_ARG, "bad basis");
  if (basis == DG_BASIS_HERMITE && degree < 3) return fail(DG_ERR_ARG, "the Hermite-like basis needs degree >= 3");
  if (!out) return fail(DG_ERR_ARG, "out is null");
  if (alloc && (!alloc->alloc || !alloc->free)) return fail(DG_ERR_ARG, "allocator needs alloc and free");
  hipStream_t s = static_cast<hipStream_t>(stream);
  dg_op *op = new dg_op();
  op->mesh = *mesh;
  op->ghost_sides = ghost_sides;
  op->degree = degree;
  op->n = degree + 1;
  op->geom = *geom;
  op->coef = *coef;
  if (vel) op->vel = *vel;
  op->basis = basis;
  op->precisions = precisions;
  op->gk = vel ? ADVECTION : geom_kind(geom, coef);
  op->gk32 = vel ? ADVECTION : geom_kind(geom, coef, true);
  if (alloc) {
    op->alloc = *alloc;
    op->own_alloc = false;
  }
  (void)hipGetDevice(&op->device);
  const int n = op->n, n2 = n * n, n3 = n2 * n;
  op->ncells = (int64_t)mesh->ncell[0] * mesh->ncell[1] * mesh->ncell[2];
  op->ndofs = op->ncells * n3;
  for (int d = 0; d < 3; ++d) op->h[d] = (mesh->hi[d] - mesh->lo[d]) / mesh->ncell[d];
  for (int a = 0; a < 3; ++a) op->nfaces[a] = op->ncells / mesh->ncell[a] * (mesh->ncell[a] + 1);

  auto fill_view = [&](auto &v, auto zero) {
    using R = decltype(zero);
    for (int d = 0; d < 3; ++d) v.ncell[d] = mesh->ncell[d];
    v.ncells = (int)op->ncells;
    for (int f = 0; f < 6; ++f) v.bc[f] = mesh->bc[f];
    for (int a = 0; a < 3; ++a) {
      const int t1 = (a == 0) ? 1 : 0, t2 = (a == 2) ? 1 : 2;
      v.inv_h[a] = (R)(1.0 / op->h[a]);
      v.tau[a] = (R)((double)n * n / op->h[a]);
      v.c_area[a] = (R)(coef->value * op->h[t1] * op->h[t2]);
    }
    v.c_vol = (R)(coef->value * op->h[0] * op->h[1] * op->h[2]);
  };
  fill_view(op->v64, 0.0);
  fill_view(op->v32, 0.0f);

  // geometry: FP64 is always built (the diagonal is computed from it); it is
  // released again below if only FP32 was asked for
  // (DG_STORE_MIXED: the FP32 cell data is of another kind than the FP64 one)
  const int64_t nfv = geom_face_values(op->gk);
  GeoArgs g = geo_args(op);
  auto cleanup = [&](dg_status e) {
    dg_destroy(op);
    return e;
  };
  for (int p = 0; p < 2; ++p) {
    const bool want = (p == 0) || (precisions & DG_PREC_F32);
    if (!want) continue;
    const size_t es = p == 0 ? 8 : 4;
    const int64_t ncv = geom_cell_values(p == 0 ? op->gk : op->gk32);
    if (ncv) {
      op->cell_geo[p] = op_alloc(op, ncv * geo_cells(op->ncells, op->n) * n3 * es);
      if (!op->cell_geo[p]) return cleanup(fail(DG_ERR_OOM, "cell geometry allocation failed"));
    }
    if (nfv)
      for (int a = 0; a < 3; ++a) {
        op->face_geo[p][a] = op_alloc(op, nfv * op->nfaces[a] * n2 * es);
        if (!op->face_geo[p][a]) return cleanup(fail(DG_ERR_OOM, "face geometry allocation failed"));
      }
  }
  const int64_t gstride = geo_cells(op->ncells, op->n) * n3;   // elements per quantity array
  {
    const int64_t npts = op->ncells * n3;
    const int grid = (int)((npts + 255) / 256);
    const int group = geo_group(op->n);
    auto cells = [&](int gk, double *o64, float *o32) {
      if (!o64 && !o32) return;
      if (gk == CURVED) hipLaunchKernelGGL(geom_cells_kernel<CURVED>, dim3(grid), dim3(256), 0, s, g, npts, o64, o32, gstride, group);
      else if (gk == CURVED_MERGED)
        hipLaunchKernelGGL(geom_cells_kernel<CURVED_MERGED>, dim3(grid), dim3(256), 0, s, g, npts, o64, o32, gstride, group);
      else if (gk == CURVED_POS)
        hipLaunchKernelGGL(geom_cells_kernel<CURVED_POS>, dim3(grid), dim3(256), 0, s, g, npts, o64, o32, gstride, group);
      else if (gk == ADVECTION)
        hipLaunchKernelGGL(geom_cells_kernel<ADVECTION>, dim3(grid), dim3(256), 0, s, g, npts, o64, o32, gstride, group);
      else if (gk == AFFINE_VAR)
        hipLaunchKernelGGL(geom_cells_kernel<AFFINE_VAR>, dim3(grid), dim3(256), 0, s, g, npts, o64, o32, gstride, group);
    };
    double *o64 = static_cast<double *>(op->cell_geo[0]);
    float *o32 = static_cast<float *>(op->cell_geo[1]);
    if (op->gk == op->gk32) {
      cells(op->gk, o64, o32);
    } else {
      cells(op->gk, o64, nullptr);
      cells(op->gk32, nullptr, o32);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return cleanup(hip_fail(e, "geometry kernel"));
  }
  if (nfv)
    for (int a = 0; a < 3; ++a) {
      const int64_t npts = op->nfaces[a] * n2;
      const int grid = (int)((npts + 255) / 256);
      double *o64 = static_cast<double *>(op->face_geo[0][a]);
      float *o32 = static_cast<float *>(op->face_geo[1][a]);
      if (curved_faces(op->gk)) hipLaunchKernelGGL(geom_faces_kernel<CURVED>, dim3(grid), dim3(256), 0, s, g, a, npts, o64, o32, npts);
      else if (op->gk == ADVECTION)
        hipLaunchKernelGGL(geom_faces_kernel<ADVECTION>, dim3(grid), dim3(256), 0, s, g, a, npts, o64, o32, npts);
      else hipLaunchKernelGGL(geom_faces_kernel<AFFINE_VAR>, dim3(grid), dim3(256), 0, s, g, a, npts, o64, o32, npts);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return cleanup(hip_fail(e, "face geometry kernel"));
    }
  op->v64.g.cell = static_cast<const double *>(op->cell_geo[0]);
  op->v64.g.cell_stride = gstride;
  op->v32.g.cell = static_cast<const float *>(op->cell_geo[1]);
  op->v32.g.cell_stride = gstride;
  for (int a = 0; a < 3; ++a) {
    op->v64.g.face[a] = static_cast<const double *>(op->face_geo[0][a]);
    op->v32.g.face[a] = static_cast<const float *>(op->face_geo[1][a]);
    op->v64.g.face_stride[a] = op->nfaces[a] * n2;
    op->v32.g.face_stride[a] = op->nfaces[a] * n2;
  }
  // Jacobi diagonal in the enabled precisions (the SIPG operator only)
  if (!vel) {
    for (int p = 0; p < 2; ++p) {
      if (!(precisions & (1u << p))) continue;
      op->diag[p] = op_alloc(op, op->ndofs * (p == 0 ? 8 : 4));
      if (!op->diag[p]) return cleanup(fail(DG_ERR_OOM, "diagonal allocation failed"));
    }
    hipError_t e = launch_diag_any(op, op->diag[0], op->diag[1], s);
    if (e != hipSuccess) return cleanup(hip_fail(e, "diagonal kernel"));
  }
  if (!(precisions & DG_PREC_F64)) {
    // FP32-only op: drop the FP64 geometry once the diagonal is done
    if (hipStreamSynchronize(s) != hipSuccess) return cleanup(fail(DG_ERR_HIP, "stream synchronize failed"));
    op_free(op, op->cell_geo[0]);
    op->cell_geo[0] = nullptr;
    for (int a = 0; a < 3; ++a) {
      op_free(op, op->face_geo[0][a]);
      op->face_geo[0][a] = nullptr;
    }
    op->v64.g = GeomData<double>{};
  }
  op->scratch_bytes = 4096 * sizeof(double);
  op->scratch = op_alloc(op, op->scratch_bytes);
  if (!op->scratch) return cleanup(fail(DG_ERR_OOM, "scratch allocation failed"));
  *out = op;
  return DG_OK;
}

extern "C" {

dg_status dg_setup(const dg_mesh *mesh, int degree, const dg_geometry *geom, const dg_coefficient *coef,
                   unsigned precisions, const dg_allocator *alloc, void *stream, dg_op **out)
{
  return setup_impl(mesh, degree, DG_BASIS_NODAL, geom, coef, nullptr, precisions, alloc, stream, out);
}

dg_status dg_setup_basis(const dg_mesh *mesh, int degree, dg_basis basis, const dg_geometry *geom,
                         const dg_coefficient *coef, unsigned precisions, const dg_allocator *alloc, void *stream,
                         dg_op **out)
{
  return setup_impl(mesh, degree, (int)basis, geom, coef, nullptr, precisions, alloc, stream, out);
}

dg_status dg_setup_advection(const dg_mesh *mesh, int degree, const dg_geometry *geom, const dg_velocity *vel,
                             unsigned precisions, const dg_allocator *alloc, void *stream, dg_op **out)
{
  if (!vel || (vel->kind != DG_VEL_CONST && vel->kind != DG_VEL_ROTATION)) return fail(DG_ERR_ARG, "bad velocity");
  const dg_coefficient one{DG_COEF_CONST, 1.0};
  return setup_impl(mesh, degree, DG_BASIS_NODAL, geom, &one, vel, precisions, alloc, stream, out);
}

static dg_status check_vec(const dg_op *op, const dg_vec &v, const char *name)
{
  if (!v.data) return fail(DG_ERR_ARG, std::string(name) + " is null");
  if (v.n != op->ndofs) return fail(DG_ERR_ARG, std::string(name) + " length does not match dg_n_dofs");
  if (v.dtype != DG_F64 && v.dtype != DG_F32) return fail(DG_ERR_ARG, std::string(name) + " has a bad dtype");
  return DG_OK;
}

dg_status dg_apply(dg_op *op, dg_vec src, dg_vec dst, void *stream)
{
  if (!op) return fail(DG_ERR_ARG, "op is null");
  dg_status st = check_vec(op, src, "src");
  if (st != DG_OK) return st;
  if ((st = check_vec(op, dst, "dst")) != DG_OK) return st;
  if (src.dtype != dst.dtype) return fail(DG_ERR_ARG, "src and dst dtypes differ");
  const bool f32 = src.dtype == DG_F32;
  if (!(op->precisions & (f32 ? DG_PREC_F32 : DG_PREC_F64)))
    return fail(DG_ERR_ARG, "the op was not set up for this precision");
  const size_t es = f32 ? 4 : 8;
  const char *a = static_cast<const char *>(src.data), *b = static_cast<const char *>(dst.data);
  if (a < b + op->ndofs * es && b < a + op->ndofs * es) return fail(DG_ERR_ARG, "src and dst alias");
  if (op->ghost_sides) return fail(DG_ERR_ARG, "the op has ghost sides: use dg_apply_ghost");
  hipError_t e = launch_apply_any(op, src.data, dst.data, f32, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "apply kernel");
  return DG_OK;
}

// cells in the plane of side f (the product of the two tangential counts)
static int64_t side_cells(const dg_op *op, int f)
{
  const int a = f / 2;
  return (int64_t)op->mesh.ncell[a == 0 ? 1 : 0] * op->mesh.ncell[a == 2 ? 1 : 2];
}

static bool overlap(const void *p, int64_t pbytes, const void *q, int64_t qbytes)
{
  const char *a = static_cast<const char *>(p), *b = static_cast<const char *>(q);
  return a < b + qbytes && b < a + pbytes;
}

dg_status dg_face_traces(const dg_op *op, int side, dg_vec src, dg_vec traces, void *stream)
{
  if (!op) return fail(DG_ERR_ARG, "op is null");
  if (op->gk == ADVECTION) return fail(DG_ERR_UNSUPPORTED, "face traces are implemented for the SIPG operator only");
  if (side < 0 || side > 5) return fail(DG_ERR_ARG, "side must be 0..5");
  dg_status st = check_vec(op, src, "src");
  if (st != DG_OK) return st;
  if (!traces.data) return fail(DG_ERR_ARG, "traces is null");
  if (traces.dtype != src.dtype) return fail(DG_ERR_ARG, "traces and src dtypes differ");
  const int64_t len = side_cells(op, side) * 2 * op->n * op->n;
  if (traces.n != len) return fail(DG_ERR_ARG, "traces length is not 2 n^2 times the cells of the side");
  const bool f32 = src.dtype == DG_F32;
  const int64_t es = f32 ? 4 : 8;
  if (overlap(src.data, op->ndofs * es, traces.data, len * es)) return fail(DG_ERR_ARG, "traces overlap src");
  hipError_t e = launch_face_traces_any(op, side, src.data, traces.data, f32, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "face traces kernel");
  return DG_OK;
}

dg_status dg_apply_ghost(dg_op *op, dg_vec src, const dg_vec ghost[6], dg_vec dst, void *stream)
{
  if (!op) return fail(DG_ERR_ARG, "op is null");
  if (op->gk == ADVECTION) return fail(DG_ERR_UNSUPPORTED, "ghost sides are implemented for the SIPG operator only");
  dg_status st = check_vec(op, src, "src");
  if (st != DG_OK) return st;
  if ((st = check_vec(op, dst, "dst")) != DG_OK) return st;
  if (src.dtype != dst.dtype) return fail(DG_ERR_ARG, "src and dst dtypes differ");
  const bool f32 = src.dtype == DG_F32;
  if (!(op->precisions & (f32 ? DG_PREC_F32 : DG_PREC_F64)))
    return fail(DG_ERR_ARG, "the op was not set up for this precision");
  const int64_t es = f32 ? 4 : 8;
  if (overlap(src.data, op->ndofs * es, dst.data, op->ndofs * es)) return fail(DG_ERR_ARG, "src and dst alias");
  const void *gp[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  for (int f = 0; f < 6; ++f) {
    if (op->mesh.bc[f] != DG_BC_GHOST) continue;
    if (!ghost) return fail(DG_ERR_ARG, "ghost is null but the op has ghost sides");
    const dg_vec &g = ghost[f];
    const std::string name = "ghost[" + std::to_string(f) + "]";
    if (!g.data) return fail(DG_ERR_ARG, name + " is null on a ghost side");
    if (g.dtype != src.dtype) return fail(DG_ERR_ARG, name + " and src dtypes differ");
    const int64_t len = side_cells(op, f) * 2 * op->n * op->n;
    if (g.n != len) return fail(DG_ERR_ARG, name + " length is not 2 n^2 times the cells of the side");
    if (overlap(g.data, len * es, dst.data, op->ndofs * es)) return fail(DG_ERR_ARG, name + " overlaps dst");
    gp[f] = g.data;
  }
  hipError_t e = launch_apply_any(op, src.data, dst.data, f32, static_cast<hipStream_t>(stream),
                                  op->ghost_sides ? gp : nullptr);
  if (e != hipSuccess) return hip_fail(e, "apply kernel");
  return DG_OK;
}

dg_status dg_diagonal(dg_op *op, dg_vec diag, void *stream)
{
  if (!op) return fail(DG_ERR_ARG, "op is null");
  if (op->gk == ADVECTION) return fail(DG_ERR_UNSUPPORTED, "the advection operator has no Jacobi diagonal here");
  dg_status st = check_vec(op, diag, "diag");
  if (st != DG_OK) return st;
  const int p = diag.dtype == DG_F32 ? 1 : 0;
  if (!op->diag[p]) return fail(DG_ERR_ARG, "the op was not set up for this precision");
  DG_HIP(hipMemcpyAsync(diag.data, op->diag[p], op->ndofs * (p ? 4 : 8), hipMemcpyDeviceToDevice,
                        static_cast<hipStream_t>(stream)));
  return DG_OK;
}

dg_status dg_rhs(dg_op *op, dg_vec b, void *stream)
{
  if (!op) return fail(DG_ERR_ARG, "op is null");
  if (op->gk == ADVECTION) return fail(DG_ERR_UNSUPPORTED, "dg_rhs is defined for the SIPG operator");
  dg_status st = check_vec(op, b, "b");
  if (st != DG_OK) return st;
  if (b.dtype != DG_F64) return fail(DG_ERR_ARG, "b must be FP64");
  GeoArgs g = geo_args(op);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int n3 = op->n * op->n * op->n;
  const int block = ((n3 + 63) / 64) * 64;
  double *bp = static_cast<double *>(b.data);
  const int grid = (int)op->ncells;
  auto go = [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    if constexpr (N >= 4)
      if (op->basis == BASIS_HERMITE) {
        hipLaunchKernelGGL((rhs_kernel<N, BASIS_HERMITE>), dim3(grid), dim3(block), 0, s, g, bp);
        return;
      }
    hipLaunchKernelGGL((rhs_kernel<N, BASIS_NODAL>), dim3(grid), dim3(block), 0, s, g, bp);
  };
  switch (op->n) {
    case 2: go(std::integral_constant<int, 2>{}); break;
    case 3: go(std::integral_constant<int, 3>{}); break;
    case 4: go(std::integral_constant<int, 4>{}); break;
    case 5: go(std::integral_constant<int, 5>{}); break;
    case 6: go(std::integral_constant<int, 6>{}); break;
    case 7: go(std::integral_constant<int, 7>{}); break;
    case 8: go(std::integral_constant<int, 8>{}); break;
    case 9: go(std::integral_constant<int, 9>{}); break;
  }
  DG_HIP(hipGetLastError());
  return DG_OK;
}

dg_status dg_error_manufactured(dg_op *op, dg_vec x, void *stream, double err[2])
{
  if (!op) return fail(DG_ERR_ARG, "op is null");
  if (op->gk == ADVECTION) return fail(DG_ERR_UNSUPPORTED, "dg_error_manufactured is defined for the SIPG operator");
  dg_status st = check_vec(op, x, "x");
  if (st != DG_OK) return st;
  if (x.dtype != DG_F64) return fail(DG_ERR_ARG, "x must be FP64");
  if (!err) return fail(DG_ERR_ARG, "err is null");
  hipStream_t s = static_cast<hipStream_t>(stream);
  GeoArgs g = geo_args(op);
  double *part = static_cast<double *>(op_alloc(op, sizeof(double) * 2 * op->ncells));
  if (!part) return fail(DG_ERR_OOM, "error workspace allocation failed");
  const double *xp = static_cast<const double *>(x.data);
  const int grid = (int)op->ncells;
  // M = N + 2 points per direction; the block is the power of two >= M^3
  // (the kernel's tree reduction needs one), at most 1024 threads
  auto go = [&](auto nc) {
    constexpr int N = decltype(nc)::value, M = N + 2;
    constexpr int block = [] {
      int b = 64;
      while (b < M * M * M && b < 1024) b *= 2;
      return b;
    }();
    if constexpr (N >= 4)
      if (op->basis == BASIS_HERMITE) {
        hipLaunchKernelGGL((error_kernel<N, M, BASIS_HERMITE>), dim3(grid), dim3(block), 0, s, g, xp, part);
        return;
      }
    hipLaunchKernelGGL((error_kernel<N, M, BASIS_NODAL>), dim3(grid), dim3(block), 0, s, g, xp, part);
  };
  switch (op->n) {
    case 2: go(std::integral_constant<int, 2>{}); break;
    case 3: go(std::integral_constant<int, 3>{}); break;
    case 4: go(std::integral_constant<int, 4>{}); break;
    case 5: go(std::integral_constant<int, 5>{}); break;
    case 6: go(std::integral_constant<int, 6>{}); break;
    case 7: go(std::integral_constant<int, 7>{}); break;
    case 8: go(std::integral_constant<int, 8>{}); break;
    case 9: go(std::integral_constant<int, 9>{}); break;
  }
  hipError_t e = hipGetLastError();
  std::vector<double> h(2 * op->ncells);
  if (e == hipSuccess) e = hipMemcpyAsync(h.data(), part, sizeof(double) * 2 * op->ncells, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    (void)hipStreamSynchronize(s);  // the kernel may still read part
    op_free(op, part);
    return hip_fail(e, "error kernel");
  }
  op_free(op, part);
  double s0 = 0.0, s1 = 0.0;
  for (int64_t c = 0; c < op->ncells; ++c) {
    s0 += h[2 * c];
    s1 += h[2 * c + 1];
  }
  err[0] = std::sqrt(s0);
  err[1] = std::sqrt(s1);
  return DG_OK;
}

}  // extern "C"
