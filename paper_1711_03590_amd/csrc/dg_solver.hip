// dg_solver.hip -- Jacobi-preconditioned conjugate gradients on the matrix-
// free SIPG operator: FP64 CG, and FP32 CG (FP32 applies, FP32 accumulation)
// on the correction equation inside FP64 iterative refinement.
//
// Every reduction is deterministic: dot products are summed over a fixed
// partition of the vector (kRedBlocks blocks, grid-stride), each block in a
// fixed tree order, and the block partials are reduced in a fixed order by
// every block that needs the result.  The product p.(A p) comes out of the
// apply itself (per-workgroup shares, summed in a fixed order by a
// one-workgroup kernel), which saves one pass over p and q per iteration.  Scalars (alpha, beta) never leave the
// device; the host reads the residual norm back only every check_every
// iterations, asynchronously into pinned memory.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "dg_internal.hpp"
#include "solver_host.hpp"
#include "solver_kernels.hpp"

namespace dgk {

namespace {

// Host memory for the scalars the solver reads back: pinned by default; the
// allocation-free entry point uses a thread-local pageable buffer instead
// (the copies then complete before hipMemcpyAsync returns, which the
// stream synchronisation after each copy waits for anyway).
struct Pinned {
  double *p = nullptr;
  bool own = false;
  explicit Pinned(bool pinned = true)
  {
    if (pinned) {
      own = hipHostMalloc(reinterpret_cast<void **>(&p), 8 * sizeof(double), hipHostMallocDefault) == hipSuccess;
      if (!own) p = nullptr;
    } else {
      thread_local double host[8];
      p = host;
    }
  }
  ~Pinned()
  {
    if (own) (void)hipHostFree(p);
  }
};

// Device workspace of one solve: released through the op's allocator, or
// (region mode) carved in order from a caller-provided region of cap bytes,
// each piece aligned to 256 bytes, with nothing allocated or freed.
constexpr size_t kWsAlign = 256;
inline size_t ws_round(size_t bytes) { return (bytes + kWsAlign - 1) / kWsAlign * kWsAlign; }
struct Workspace {
  dg_op *op;
  std::vector<void *> ptr;
  char *base = nullptr;
  size_t cap = 0, used = 0;
  explicit Workspace(dg_op *o) : op(o) {}
  Workspace(dg_op *o, void *region, size_t bytes) : op(o), base(static_cast<char *>(region)), cap(bytes) {}
  void *get(size_t bytes)
  {
    if (base) {
      const size_t sz = ws_round(bytes);
      if (used + sz > cap) return nullptr;
      void *p = base + used;
      used += sz;
      return p;
    }
    void *p = op_alloc(op, bytes);
    if (p) ptr.push_back(p);
    return p;
  }
  ~Workspace()
  {
    for (void *p : ptr) op_free(op, p);
  }
};

// the vectors of one PCG run in precision Real
template <typename Real, typename Acc>
struct PcgBuffers {
  Real *r = nullptr, *p = nullptr, *q = nullptr;
  Acc *part = nullptr;
  Real *wgpart = nullptr;     // per-workgroup shares of p.(A p)
  int nwg = 0;
  bool alloc(Workspace &ws, dg_op *op)
  {
    const int64_t n = op->ndofs;
    r = static_cast<Real *>(ws.get(n * sizeof(Real)));
    p = static_cast<Real *>(ws.get(n * sizeof(Real)));
    q = static_cast<Real *>(ws.get(n * sizeof(Real)));
    part = static_cast<Acc *>(ws.get(3 * kRedBlocks * sizeof(Acc) + 4 * sizeof(Acc)));
    nwg = apply_workgroups_any(op);
    wgpart = static_cast<Real *>(ws.get((size_t)nwg * sizeof(Real)));
    return r && p && q && part && wgpart;
  }
  // p.q partials: only entry 0 is written (the sum of the apply's shares),
  // the rest stay zero, so the update kernels' fixed-order sum returns it
  hipError_t clear(hipStream_t s) const
  {
    hipLaunchKernelGGL((fill_kernel<Acc>), dim3(1), dim3(kRedThreads), 0, s, part, Acc(0), (int64_t)kRedBlocks);
    return hipGetLastError();
  }
  // q = A p and pq_part[0] = p.q
  hipError_t apply_dot(dg_op *op, const Real *p, Real *q, hipStream_t s) const
  {
    hipError_t e = launch_apply_dot_any(op, p, q, sizeof(Real) == 4, wgpart, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((sum_shares_kernel<Acc>), dim3(1), dim3(kSumThreads), 0, s, wgpart, nwg, part);
    return hipGetLastError();
  }
};

template <typename Acc>
hipError_t norm2(const void *x, bool f32, int64_t n, Acc *part, Acc *out, hipStream_t s)
{
  if (f32) {
    const float *v = static_cast<const float *>(x);
    hipLaunchKernelGGL((dot_partial_kernel<float, Acc>), dim3(kRedBlocks), dim3(kRedThreads), 0, s, v, v, n, part);
  } else {
    const double *v = static_cast<const double *>(x);
    hipLaunchKernelGGL((dot_partial_kernel<double, Acc>), dim3(kRedBlocks), dim3(kRedThreads), 0, s, v, v, n, part);
  }
  hipLaunchKernelGGL((finalize_kernel<Acc>), dim3(1), dim3(kRedThreads), 0, s, part, kRedBlocks, out);
  return hipGetLastError();
}

// Preconditioned CG on A x = rhs in precision Real (accumulation Acc), x and
// rhs device vectors; x holds the initial guess.  Stops when the recurrence
// residual satisfies ||r|| <= tol_abs, or after max_iter iterations.
// Workspace: r, p, q (Real), partials.  Returns iterations done in *iters.
template <typename Real, typename Acc>
dg_status pcg(dg_op *op, const Real *rhs, Real *x, bool x_zero, double tol_abs, int max_iter, int check_every,
              const PcgBuffers<Real, Acc> &buf, Pinned &pin, hipStream_t s, int *iters, double *rnorm)
{
  const int64_t n = op->ndofs;
  const bool f32 = sizeof(Real) == 4;
  Real *r = buf.r, *p = buf.p, *q = buf.q;
  Acc *part = buf.part;
  Acc *pq_part = part;                    // kRedBlocks
  Acc *rz_part = part + kRedBlocks;       // 2 * kRedBlocks: r.z and r.r interleaved
  Acc *scal = part + 3 * kRedBlocks;      // rz[2] (ping-pong), rr, spare
  const Real *d = static_cast<const Real *>(op->diag[f32 ? 1 : 0]);
  const int grid = kRedBlocks;
  DG_HIP(buf.clear(s));
  // r = rhs - A x
  if (x_zero) {
    hipLaunchKernelGGL((copy_kernel<Real>), dim3(grid), dim3(kRedThreads), 0, s, rhs, r, n);
  } else {
    DG_HIP(launch_apply_any(op, x, q, f32, s));
    hipLaunchKernelGGL((sub_kernel<Real>), dim3(grid), dim3(kRedThreads), 0, s, rhs, q, r, n);
  }
  // z = r / d, p = z, rz = r.z, rr = r.r
  hipLaunchKernelGGL((rz_partial_kernel<Real, Acc>), dim3(grid), dim3(kRedThreads), 0, s, r, d, n, rz_part);
  hipLaunchKernelGGL((cg_pupdate_kernel<Real, Acc>), dim3(grid), dim3(kRedThreads), 0, s, p, (Real *)nullptr, r, d, n,
                     pq_part, rz_part, scal, 0, 0);
  DG_HIP(hipGetLastError());
  int par = 1;  // scal[par] holds the current r.z
  int it = 0;
  bool done = false;
  auto read_rr = [&](double *out) -> dg_status {
    DG_HIP(hipMemcpyAsync(pin.p, scal + 2, sizeof(Acc), hipMemcpyDeviceToHost, s));
    DG_HIP(hipStreamSynchronize(s));
    *out = std::sqrt((double)*reinterpret_cast<Acc *>(pin.p));
    return DG_OK;
  };
  double rn = 0.0;
  dg_status st = read_rr(&rn);
  if (st != DG_OK) return st;
  if (!(rn > tol_abs)) done = true;
  while (!done && it < max_iter) {
    DG_HIP(buf.apply_dot(op, p, q, s));
    hipLaunchKernelGGL((cg_update_kernel<Real, Acc>), dim3(grid), dim3(kRedThreads), 0, s, r, q, d, n, pq_part, scal,
                       par, rz_part);
    hipLaunchKernelGGL((cg_pupdate_kernel<Real, Acc>), dim3(grid), dim3(kRedThreads), 0, s, p, x, r, d, n, pq_part,
                       rz_part, scal, 1, par);
    DG_HIP(hipGetLastError());
    par = 1 - par;
    ++it;
    if (it % check_every == 0 || it == max_iter) {
      if ((st = read_rr(&rn)) != DG_OK) return st;
      if (!(rn > tol_abs)) done = true;
      if (!std::isfinite(rn)) return fail(DG_ERR_NOT_CONVERGED, "CG breakdown (non-finite residual)");
    }
  }
  *iters = it;
  *rnorm = rn;
  return done ? DG_OK : DG_ERR_NOT_CONVERGED;
}

// FP32 Jacobi-PCG with reliable updates inside FP64 refinement: the FP32
// recurrence runs on the relative system A e = r / ||b||; each time its
// residual has dropped by the factor delta since the last refinement
// (checked every check_every iterations), the FP32 correction is flushed into the FP64
// solution (x += ||b|| e), the FP64 residual b - A x is recomputed with an
// FP64 apply and replaces the FP32 residual, and the search direction is
// kept, so no Krylov information is lost at a refinement step.
dg_status pcg_reliable(dg_op *op, const double *b, double *x, double nb, double tol, double delta, int max_iter,
                       int check_every, const PcgBuffers<float, float> &buf, float *e, double *r64, double *dpart,
                       Pinned &pin, hipStream_t s, dg_solve_stats &st, double *rel_out)
{
  const int64_t n = op->ndofs;
  const int grid = kRedBlocks;
  float *r = buf.r, *p = buf.p, *q = buf.q;
  float *pq_part = buf.part, *rz_part = buf.part + kRedBlocks, *scal = buf.part + 3 * kRedBlocks;
  double *dscal = dpart + kRedBlocks;
  const float *d = static_cast<const float *>(op->diag[1]);
  auto read = [&](const void *dev, size_t bytes, void *host) -> dg_status {
    DG_HIP(hipMemcpyAsync(pin.p, dev, bytes, hipMemcpyDeviceToHost, s));
    DG_HIP(hipStreamSynchronize(s));
    memcpy(host, pin.p, bytes);
    return DG_OK;
  };
  // FP64 residual r64 = b - A x, its relative norm, and r = r64 / ||b|| in FP32
  auto refresh = [&](double *rel) -> dg_status {
    DG_HIP(rel_residual_async(op, b, x, r64, dpart, dscal, r, nb, s));
    double v;
    dg_status e2 = read(dscal, sizeof(double), &v);
    if (e2 != DG_OK) return e2;
    *rel = std::sqrt(v) / nb;
    st.applies_f64 += 1;
    return DG_OK;
  };
  double rel;
  dg_status rc = refresh(&rel);
  if (rc != DG_OK) return rc;
  *rel_out = rel;
  if (rel <= tol) return DG_OK;
  DG_HIP(buf.clear(s));
  DG_HIP(start_direction_async(n, e, r, p, d, buf.part, s));
  int par = 1;
  double rlast = rel;
  st.iters_outer = 1;
  for (int it = 1; it <= max_iter; ++it) {
    DG_HIP(buf.apply_dot(op, p, q, s));
    hipLaunchKernelGGL((cg_update_kernel<float, float>), dim3(grid), dim3(kRedThreads), 0, s, r, q, d, n, pq_part,
                       scal, par, rz_part);
    hipLaunchKernelGGL((cg_pupdate_kernel<float, float>), dim3(grid), dim3(kRedThreads), 0, s, p, e, r, d, n, pq_part,
                       rz_part, scal, 1, par);
    DG_HIP(hipGetLastError());
    par = 1 - par;
    st.iters_inner += 1;
    st.applies_f32 += 1;
    if (it % check_every != 0 && it != max_iter) continue;
    float rr;
    if ((rc = read(scal + 2, sizeof(float), &rr)) != DG_OK) return rc;
    const double r32 = std::sqrt((double)rr);
    if (!std::isfinite(r32)) return fail(DG_ERR_NOT_CONVERGED, "CG breakdown (non-finite residual)");
    if (r32 <= tol || r32 < delta * rlast || it == max_iter) {
      // refinement step: flush the correction, replace the residual
      DG_HIP(flush_correction_async(n, x, nb, e, s));
      if ((rc = refresh(&rel)) != DG_OK) return rc;
      *rel_out = rel;
      if (rel <= tol) return DG_OK;
      st.iters_outer += 1;
      rlast = rel;
      // r.z of the replaced residual becomes the current r.z
      DG_HIP(restart_rz_async(n, r, d, buf.part, par, s));
    }
  }
  return DG_ERR_NOT_CONVERGED;
}

}  // namespace

}  // namespace dgk

using namespace dgk;

// Workspace of the allocation-free solve (dg_cg_solve_noalloc): one array per
// GPU the library runs on, in the code object's data, so it is there as soon
// as the library is loaded on that device and stays until the process ends.
// Every call on a device shares it.
static constexpr size_t kNoAllocBytes = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

// the argument checks of both solve entry points
dg_status check_solve_args(const dg_op *op, dg_vec b, dg_vec x, const dg_solve_params *prm)
{
  if (!op || !prm) return fail(DG_ERR_ARG, "null argument");
  if (op->gk == ADVECTION) return fail(DG_ERR_UNSUPPORTED, "CG needs the symmetric SIPG operator");
  if (op->ghost_sides) return fail(DG_ERR_UNSUPPORTED, "CG on a partition with ghost sides needs an exchange per apply");
  if (!b.data || !x.data || b.n != op->ndofs || x.n != op->ndofs || b.dtype != DG_F64 || x.dtype != DG_F64)
    return fail(DG_ERR_ARG, "b and x must be FP64 vectors of length dg_n_dofs");
  if (b.data == x.data) return fail(DG_ERR_ARG, "b and x alias");
  if (prm->mode < 0 || prm->mode > 2) return fail(DG_ERR_ARG, "mode must be 0 (FP64), 1 (mixed) or 2 (mixed, reliable updates)");
  if (!(prm->rel_tol > 0) || prm->max_iter < 1 || prm->check_every < 1) return fail(DG_ERR_ARG, "bad solver limits");
  if (!(op->precisions & DG_PREC_F64)) return fail(DG_ERR_ARG, "the op needs FP64 data");
  if (prm->mode >= 1 && (!(op->precisions & DG_PREC_F32) || !(prm->rel_tol_inner > 0) || prm->max_outer < 1))
    return fail(DG_ERR_ARG, "mixed mode needs FP32 data, rel_tol_inner > 0 and max_outer >= 1");
  return DG_OK;
}

// Device workspace bytes of a solve in region mode: the pieces solve() takes
// from its Workspace, in the same order and sizes, each rounded to kWsAlign.
size_t solve_workspace_bytes(const dg_op *op, int mode)
{
  const size_t n = (size_t)op->ndofs;
  const size_t nwg = (size_t)apply_workgroups_any(op);
  auto pcg_bytes = [&](size_t real, size_t acc) {
    return 3 * ws_round(n * real) + ws_round((3 * kRedBlocks + 4) * acc) + ws_round(nwg * real);
  };
  size_t bytes = ws_round((kRedBlocks + 8) * sizeof(double)) + ws_round(n * sizeof(double));
  if (mode == 0) bytes += pcg_bytes(sizeof(double), sizeof(double));
  else if (mode == 2) bytes += ws_round(n * sizeof(float)) + pcg_bytes(sizeof(float), sizeof(float));
  else bytes += 2 * ws_round(n * sizeof(float)) + pcg_bytes(sizeof(float), sizeof(float));
  return bytes;
}

// The solve proper, with its device workspace taken from ws and its
// read-backs going through pin (arguments already checked).
dg_status solve(dg_op *op, dg_vec b, dg_vec x, const dg_solve_params *prm, dg_solve_stats *stats, void *stream,
                Workspace &ws, Pinned &pin, std::chrono::steady_clock::time_point t0)
{
  hipStream_t s = static_cast<hipStream_t>(stream);
  dg_solve_stats st{};
  const int64_t n = op->ndofs;
  const int grid = kRedBlocks;
  if (!pin.p) return fail(DG_ERR_HIP, "pinned host allocation failed");
  double *part = static_cast<double *>(ws.get((kRedBlocks + 8) * sizeof(double)));
  double *r64 = static_cast<double *>(ws.get(n * sizeof(double)));
  if (!part || !r64) return fail(DG_ERR_OOM, "solver workspace allocation failed");
  double *dscal = part + kRedBlocks;
  double *xp = static_cast<double *>(x.data);
  const double *bp = static_cast<const double *>(b.data);
  auto read_scalar = [&](double *out) -> dg_status {
    DG_HIP(hipMemcpyAsync(pin.p, dscal, sizeof(double), hipMemcpyDeviceToHost, s));
    DG_HIP(hipStreamSynchronize(s));
    *out = *pin.p;
    return DG_OK;
  };
  // ||b||
  DG_HIP(norm2<double>(bp, false, n, part, dscal, s));
  double nb = 0.0;
  dg_status rc = read_scalar(&nb);
  if (rc != DG_OK) return rc;
  nb = std::sqrt(nb);
  if (nb == 0.0) {
    hipLaunchKernelGGL((fill_kernel<double>), dim3(grid), dim3(kRedThreads), 0, s, xp, 0.0, n);
    DG_HIP(hipStreamSynchronize(s));
    if (stats) *stats = st;
    return DG_OK;
  }
  // true FP64 residual r64 = b - A x and its norm
  auto true_residual = [&](double *rel) -> dg_status {
    DG_HIP(launch_apply_any(op, xp, r64, false, s));
    hipLaunchKernelGGL((sub_kernel<double>), dim3(grid), dim3(kRedThreads), 0, s, bp, r64, r64, n);
    DG_HIP(norm2<double>(r64, false, n, part, dscal, s));
    double v;
    dg_status e = read_scalar(&v);
    if (e != DG_OK) return e;
    *rel = std::sqrt(v) / nb;
    st.applies_f64 += 1;
    return DG_OK;
  };
  double rel = 0.0;
  dg_status result = DG_ERR_NOT_CONVERGED;
  if (prm->mode == 0) {
    // FP64 Jacobi-PCG; restarted from the true residual if the recurrence
    // residual drifted below the tolerance first
    PcgBuffers<double, double> buf;
    if (!buf.alloc(ws, op)) return fail(DG_ERR_OOM, "solver workspace allocation failed");
    for (int restart = 0; restart < 4; ++restart) {
      int it = 0;
      double rn = 0.0;
      const int left = prm->max_iter - st.iters_inner;
      if (left <= 0) break;
      // solve A e = b - A x for the correction in place: run CG on x directly
      rc = pcg<double, double>(op, bp, xp, false, prm->rel_tol * nb, left, prm->check_every, buf, pin, s, &it, &rn);
      st.iters_inner += it;
      st.applies_f64 += it + 1;
      if (rc != DG_OK && rc != DG_ERR_NOT_CONVERGED) return rc;
      if ((rc = true_residual(&rel)) != DG_OK) return rc;
      if (rel <= prm->rel_tol) {
        result = DG_OK;
        break;
      }
    }
  } else if (prm->mode == 2) {
    float *e32 = static_cast<float *>(ws.get(n * sizeof(float)));
    PcgBuffers<float, float> buf;
    if (!e32 || !buf.alloc(ws, op)) return fail(DG_ERR_OOM, "solver workspace allocation failed");
    rc = pcg_reliable(op, bp, xp, nb, prm->rel_tol, prm->rel_tol_inner, prm->max_iter, prm->check_every, buf, e32,
                      r64, part, pin, s, st, &rel);
    if (rc == DG_OK) result = DG_OK;
    else if (rc != DG_ERR_NOT_CONVERGED) return rc;
  } else {
    // FP32 PCG on the correction equation inside FP64 iterative refinement
    float *r32 = static_cast<float *>(ws.get(n * sizeof(float)));
    float *d32 = static_cast<float *>(ws.get(n * sizeof(float)));
    PcgBuffers<float, float> buf;
    if (!r32 || !d32 || !buf.alloc(ws, op)) return fail(DG_ERR_OOM, "solver workspace allocation failed");
    for (int outer = 0; outer <= prm->max_outer; ++outer) {
      if ((rc = true_residual(&rel)) != DG_OK) return rc;
      if (rel <= prm->rel_tol) {
        result = DG_OK;
        break;
      }
      if (outer == prm->max_outer || st.iters_inner >= prm->max_iter * prm->max_outer) break;
      st.iters_outer += 1;
      // r32 = r64 / ||r64||, d32 = 0
      const double nr = rel * nb;
      hipLaunchKernelGGL(scale_to_f32_kernel, dim3(grid), dim3(kRedThreads), 0, s, r64, 1.0 / nr, r32, n);
      hipLaunchKernelGGL((fill_kernel<float>), dim3(grid), dim3(kRedThreads), 0, s, d32, 0.0f, n);
      DG_HIP(hipGetLastError());
      int it = 0;
      double rn = 0.0;
      rc = pcg<float, float>(op, r32, d32, true, prm->rel_tol_inner, prm->max_iter, prm->check_every, buf, pin, s,
                             &it, &rn);
      st.iters_inner += it;
      st.applies_f32 += it;
      if (rc != DG_OK && rc != DG_ERR_NOT_CONVERGED) return rc;
      // x += ||r64|| * d32
      hipLaunchKernelGGL(axpy_f32_kernel, dim3(grid), dim3(kRedThreads), 0, s, xp, nr, d32, n);
      DG_HIP(hipGetLastError());
    }
  }
  DG_HIP(hipStreamSynchronize(s));
  st.final_rel_residual = rel;
  st.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (stats) *stats = st;
  if (result != DG_OK) return fail(DG_ERR_NOT_CONVERGED, "solver did not reach the tolerance within its limits");
  return DG_OK;
}

// the device address of this device's scratch, looked up once per device
// (the host-side name scratch is not a device address)
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};

dg_status device_scratch(void **out)
{
  int dev = -1;
  DG_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(DG_ERR_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return DG_OK;
}

}  // namespace

extern "C" dg_status dg_cg_solve(dg_op *op, dg_vec b, dg_vec x, const dg_solve_params *prm, dg_solve_stats *stats,
                                 void *stream)
{
  const auto t0 = std::chrono::steady_clock::now();
  dg_status rc = check_solve_args(op, b, x, prm);
  if (rc != DG_OK) return rc;
  Pinned pin;
  Workspace ws(op);
  return solve(op, b, x, prm, stats, stream, ws, pin, t0);
}

extern "C" size_t dg_cg_solve_noalloc_capacity(void) { return kNoAllocBytes; }

extern "C" dg_status dg_cg_solve_noalloc_bytes(const dg_op *op, int mode, size_t *bytes)
{
  if (!op || !bytes) return fail(DG_ERR_ARG, "null argument");
  if (mode < 0 || mode > 2) return fail(DG_ERR_ARG, "mode must be 0, 1 or 2");
  *bytes = solve_workspace_bytes(op, mode);
  return DG_OK;
}

extern "C" dg_status dg_cg_solve_noalloc(dg_op *op, dg_vec b, dg_vec x, const dg_solve_params *prm,
                                         dg_solve_stats *stats, void *stream)
{
  const auto t0 = std::chrono::steady_clock::now();
  dg_status rc = check_solve_args(op, b, x, prm);
  if (rc != DG_OK) return rc;
  const size_t need = solve_workspace_bytes(op, prm->mode);
  if (need > kNoAllocBytes)
    return fail(DG_ERR_ARG, "dg_cg_solve_noalloc: this solve needs " + std::to_string(need) +
                                " bytes of workspace, beyond the " + std::to_string(kNoAllocBytes) +
                                "-byte static scratch (use dg_cg_solve)");
  void *region = nullptr;
  if ((rc = device_scratch(&region)) != DG_OK) return rc;
  Pinned pin(false);
  Workspace ws(op, region, kNoAllocBytes);
  return solve(op, b, x, prm, stats, stream, ws, pin, t0);
}
