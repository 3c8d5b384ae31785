// dg_batch.hip -- continuous batching of mixed-precision SIPG solves.
//
// A batch holds up to max_slots requests, each a reliable-update mixed CG
// (dg_cg_solve mode 2) on its own operator.  dg_batch_run advances all
// active requests by one CG iteration per round; a round is four launches:
//   1. one persistent apply kernel whose workgroups walk a list of
//      (request, cell batch) items spanning every active request, whatever
//      its degree or geometry (q = A p in FP32);
//   2.-4. batched BLAS kernels over (request, chunk) items: p.q partials,
//      the x/r update with r.z, r.r partials, the p update.
// Each request's sums are taken over the same fixed partition of its own
// vectors as in dg_cg_solve, and its check points count its own iterations,
// so its result does not depend on the other requests in the batch.  The
// FP64 refinement steps (flush of the correction, FP64 residual) run per
// request between rounds.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "dg_internal.hpp"
#include "kernels.hpp"
#include "solver_host.hpp"
#include "solver_kernels.hpp"

namespace dgk {

#define DG_EXTERN_N(N)                                                                  \
  extern template hipError_t launch_apply<N>(const dg_op *, const void *, void *, bool, \
                                             hipStream_t);                              \
  extern template hipError_t launch_diag<N>(const dg_op *, void *, void *, hipStream_t);
DG_EXTERN_N(2)
DG_EXTERN_N(3)
DG_EXTERN_N(4)
DG_EXTERN_N(5)
DG_EXTERN_N(6)
DG_EXTERN_N(7)
DG_EXTERN_N(8)
DG_EXTERN_N(9)
#undef DG_EXTERN_N

constexpr int kBatchTpb = 256;
// degrees served by the persistent kernel: 2..7 (3..8 points per direction)
constexpr int kBatchMinN = 3, kBatchMaxN = 8;
#ifndef DG_BATCH_WAVES
#define DG_BATCH_WAVES 4
#endif

template <int N>
constexpr int batch_lds()
{
  using BK = Blocking<N, kBatchTpb>;
  return BK::SMEM;
}
constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int kBatchLds = cmax(cmax(cmax(batch_lds<3>(), batch_lds<4>()), cmax(batch_lds<5>(), batch_lds<6>())),
                               cmax(batch_lds<7>(), batch_lds<8>()));

// device descriptor of one active request
struct BatchSlot {
  OpView<float> v;
  int n, gk;
  int64_t ndofs;
  int item0, nitems;   // apply items [item0, item0 + nitems): cell batches of kBatchTpb / n^2 cells
  int round0;          // batch round of the request's first iteration
  float *e, *r, *p, *q;
  const float *d;
  float *part;         // kRedBlocks p.q partials, 2 kRedBlocks r.z/r.r partials, scal[4]
};

// one function per degree (not inlined into the persistent kernel), so that
// each degree's register allocation stays its own
template <int N>
__device__ __noinline__ void batch_apply_one(const BatchSlot &sl, int blk, float *smem)
{
  switch (sl.gk) {
    case CURVED: apply_batch<N, float, CURVED, kBatchTpb>(sl.v, sl.p, sl.q, blk, smem); break;
    case CURVED_MERGED: apply_batch<N, float, CURVED_MERGED, kBatchTpb>(sl.v, sl.p, sl.q, blk, smem); break;
    case CURVED_POS: apply_batch<N, float, CURVED_POS, kBatchTpb>(sl.v, sl.p, sl.q, blk, smem); break;
    case AFFINE_VAR: apply_batch<N, float, AFFINE_VAR, kBatchTpb>(sl.v, sl.p, sl.q, blk, smem); break;
    default: apply_batch<N, float, AFFINE_CONST, kBatchTpb>(sl.v, sl.p, sl.q, blk, smem); break;
  }
}

// persistent: workgroup b takes items b, b + G, b + 2G, ... (G = gridDim.x);
// every workgroup leaves the loop once the item list is exhausted
__global__ void __launch_bounds__(kBatchTpb, DG_BATCH_WAVES) batch_apply_kernel(const BatchSlot *__restrict__ slots, int nslots,
                                                                int nitems)
{
  __shared__ float smem[kBatchLds];
  for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
    int s = 0;
    while (s + 1 < nslots && slots[s + 1].item0 <= item) ++s;
    const BatchSlot &sl = slots[s];
    const int blk = item - sl.item0;
    switch (sl.n) {
      case 3: batch_apply_one<3>(sl, blk, smem); break;
      case 4: batch_apply_one<4>(sl, blk, smem); break;
      case 5: batch_apply_one<5>(sl, blk, smem); break;
      case 6: batch_apply_one<6>(sl, blk, smem); break;
      case 7: batch_apply_one<7>(sl, blk, smem); break;
      default: batch_apply_one<8>(sl, blk, smem); break;
    }
    __syncthreads();
  }
}

// the current r.z slot of a request at this round (ping-pong by its own
// iteration count: iteration it uses scal[it & 1])
__device__ __forceinline__ int batch_cur(const BatchSlot &sl, int round) { return (round - sl.round0 + 1) & 1; }

__global__ void __launch_bounds__(kRedThreads) batch_dot_kernel(const BatchSlot *__restrict__ slots)
{
  __shared__ float sh[kRedThreads];
  const BatchSlot &sl = slots[blockIdx.x / kRedBlocks];
  dot_partial_body<float, float>(sl.p, sl.q, sl.ndofs, sl.part, blockIdx.x % kRedBlocks, sh);
}

__global__ void __launch_bounds__(kRedThreads) batch_update_kernel(const BatchSlot *__restrict__ slots, int round)
{
  __shared__ float sh[kRedThreads];
  const BatchSlot &sl = slots[blockIdx.x / kRedBlocks];
  cg_update_body<float, float>(sl.r, sl.q, sl.d, sl.ndofs, sl.part, sl.part + 3 * kRedBlocks, batch_cur(sl, round),
                               sl.part + kRedBlocks, blockIdx.x % kRedBlocks, sh);
}

__global__ void __launch_bounds__(kRedThreads) batch_pupdate_kernel(const BatchSlot *__restrict__ slots, int round)
{
  __shared__ float sh[kRedThreads];
  const BatchSlot &sl = slots[blockIdx.x / kRedBlocks];
  cg_pupdate_body<float, float>(sl.p, sl.e, sl.r, sl.d, sl.ndofs, sl.part, sl.part + kRedBlocks,
                                sl.part + 3 * kRedBlocks, 1, batch_cur(sl, round), blockIdx.x % kRedBlocks, sh);
}

// r.r of every request into one array (one read-back per check)
__global__ void batch_gather_rr_kernel(const BatchSlot *__restrict__ slots, int nslots, float *__restrict__ out)
{
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < nslots) out[s] = slots[s].part[3 * kRedBlocks + 2];
}

struct Request {
  bool used = false;    // admitted and not yet polled
  bool done = false;    // finished (converged or not)
  dg_status status = DG_OK;
  dg_op *op = nullptr;
  double *x = nullptr;
  const double *b = nullptr;
  dg_solve_params prm{};
  double nb = 0.0, rel = 0.0, rlast = 0.0;
  int it = 0;           // CG iterations done
  int round0 = 0;
  void *mem[8] = {nullptr};
  float *e = nullptr, *r = nullptr, *p = nullptr, *q = nullptr, *part = nullptr;
  double *r64 = nullptr, *dpart = nullptr;
  dg_solve_stats st{};
  std::chrono::steady_clock::time_point t0;
};

}  // namespace dgk

using namespace dgk;

struct dg_batch {
  int max_slots = 0;
  dg_allocator alloc{};
  bool own_alloc = true;
  std::vector<Request> req;
  BatchSlot *d_desc = nullptr, *h_desc = nullptr;
  float *d_rr = nullptr, *h_rr = nullptr;
  double *h_scalar = nullptr;
  int round = 0;
  bool dirty = true;
  std::vector<int> active;   // request index per descriptor position
  int nitems = 0;
};

namespace {

void *balloc(dg_batch *b, size_t bytes)
{
  if (!b->own_alloc) return b->alloc.alloc(bytes, b->alloc.ctx);
  void *p = nullptr;
  return hipMalloc(&p, bytes) == hipSuccess ? p : nullptr;
}

void bfree(dg_batch *b, void *p)
{
  if (!p) return;
  if (!b->own_alloc) b->alloc.free(p, b->alloc.ctx);
  else (void)hipFree(p);
}

void release(dg_batch *b, Request &r)
{
  for (void *&m : r.mem) {
    bfree(b, m);
    m = nullptr;
  }
  r = Request();
}

dg_status read_scalar(dg_batch *b, const double *dev, double *out, hipStream_t s)
{
  DG_HIP(hipMemcpyAsync(b->h_scalar, dev, sizeof(double), hipMemcpyDeviceToHost, s));
  DG_HIP(hipStreamSynchronize(s));
  *out = *b->h_scalar;
  return DG_OK;
}

// FP64 residual of request r; stores the relative norm in r.rel
dg_status refresh(dg_batch *b, Request &r, hipStream_t s)
{
  double *dscal = r.dpart + kRedBlocks;
  DG_HIP(rel_residual_async(r.op, r.b, r.x, r.r64, r.dpart, dscal, r.r, r.nb, s));
  double v;
  dg_status st = read_scalar(b, dscal, &v, s);
  if (st != DG_OK) return st;
  r.rel = std::sqrt(v) / r.nb;
  r.st.applies_f64 += 1;
  return DG_OK;
}

void finish(Request &r, dg_status status)
{
  r.done = true;
  r.status = status;
  r.st.final_rel_residual = r.rel;
  r.st.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - r.t0).count();
}

dg_status rebuild(dg_batch *b, hipStream_t s)
{
  b->active.clear();
  int item = 0;
  for (int i = 0; i < b->max_slots; ++i) {
    Request &r = b->req[i];
    if (!r.used || r.done) continue;
    BatchSlot &d = b->h_desc[b->active.size()];
    const int n = r.op->n;
    const int cells_per_item = kBatchTpb / (n * n);
    d.v = r.op->v32;
    d.n = n;
    d.gk = r.op->gk32;
    d.ndofs = r.op->ndofs;
    d.item0 = item;
    d.nitems = (int)((r.op->ncells + cells_per_item - 1) / cells_per_item);
    d.round0 = r.round0;
    d.e = r.e;
    d.r = r.r;
    d.p = r.p;
    d.q = r.q;
    d.d = static_cast<const float *>(r.op->diag[1]);
    d.part = r.part;
    item += d.nitems;
    b->active.push_back(i);
  }
  b->nitems = item;
  if (!b->active.empty()) {
    DG_HIP(hipMemcpyAsync(b->d_desc, b->h_desc, sizeof(BatchSlot) * b->active.size(), hipMemcpyHostToDevice, s));
    DG_HIP(hipStreamSynchronize(s));  // the staging buffer is rewritten by the next rebuild
  }
  b->dirty = false;
  return DG_OK;
}

}  // namespace

extern "C" {

dg_status dg_batch_create(int max_slots, const dg_allocator *alloc, dg_batch **out)
{
  if (max_slots < 1 || max_slots > 1024 || !out) return fail(DG_ERR_ARG, "max_slots must be in [1, 1024]");
  if (alloc && (!alloc->alloc || !alloc->free)) return fail(DG_ERR_ARG, "allocator needs alloc and free");
  dg_batch *b = new dg_batch();
  b->max_slots = max_slots;
  if (alloc) {
    b->alloc = *alloc;
    b->own_alloc = false;
  }
  b->req.resize(max_slots);
  bool ok = hipMalloc(reinterpret_cast<void **>(&b->d_desc), sizeof(BatchSlot) * max_slots) == hipSuccess &&
            hipMalloc(reinterpret_cast<void **>(&b->d_rr), sizeof(float) * max_slots) == hipSuccess &&
            hipHostMalloc(reinterpret_cast<void **>(&b->h_desc), sizeof(BatchSlot) * max_slots,
                          hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc(reinterpret_cast<void **>(&b->h_rr), sizeof(float) * max_slots, hipHostMallocDefault) ==
                hipSuccess &&
            hipHostMalloc(reinterpret_cast<void **>(&b->h_scalar), sizeof(double) * 2, hipHostMallocDefault) ==
                hipSuccess;
  if (!ok) {
    dg_batch_destroy(b);
    return fail(DG_ERR_OOM, "batch allocation failed");
  }
  *out = b;
  return DG_OK;
}

int dg_batch_active(const dg_batch *b)
{
  if (!b) return 0;
  int c = 0;
  for (const Request &r : b->req) c += r.used ? 1 : 0;
  return c;
}

dg_status dg_batch_admit(dg_batch *b, dg_op *op, dg_vec bv, dg_vec xv, const dg_solve_params *prm, int *slot,
                         void *stream)
{
  if (!b || !op || !prm || !slot) return fail(DG_ERR_ARG, "null argument");
  if (op->gk == ADVECTION) return fail(DG_ERR_UNSUPPORTED, "batched CG needs the symmetric SIPG operator");
  if (op->ghost_sides) return fail(DG_ERR_UNSUPPORTED, "batched CG on a partition with ghost sides is not supported");
  if (op->basis != DG_BASIS_NODAL) return fail(DG_ERR_UNSUPPORTED, "batched solves serve the nodal basis");
  if (!(op->precisions & DG_PREC_F64) || !(op->precisions & DG_PREC_F32))
    return fail(DG_ERR_ARG, "batched solves need an op with FP64 and FP32 data");
  if (!bv.data || !xv.data || bv.n != op->ndofs || xv.n != op->ndofs || bv.dtype != DG_F64 || xv.dtype != DG_F64)
    return fail(DG_ERR_ARG, "b and x must be FP64 vectors of length dg_n_dofs");
  if (bv.data == xv.data) return fail(DG_ERR_ARG, "b and x alias");
  if (op->n < kBatchMinN || op->n > kBatchMaxN) return fail(DG_ERR_UNSUPPORTED, "batched solves serve degrees 2..7");
  if (!(prm->rel_tol > 0) || !(prm->rel_tol_inner > 0 && prm->rel_tol_inner < 1) || prm->max_iter < 1 ||
      prm->check_every < 1)
    return fail(DG_ERR_ARG, "bad solver parameters (rel_tol > 0, 0 < rel_tol_inner < 1, max_iter, check_every >= 1)");
  int idx = -1;
  for (int i = 0; i < b->max_slots; ++i)
    if (!b->req[i].used) {
      idx = i;
      break;
    }
  if (idx < 0) return fail(DG_ERR_OOM, "no free slot");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Request &r = b->req[idx];
  r = Request();
  r.t0 = std::chrono::steady_clock::now();
  r.op = op;
  r.x = static_cast<double *>(xv.data);
  r.b = static_cast<const double *>(bv.data);
  r.prm = *prm;
  const int64_t n = op->ndofs;
  const size_t sz[7] = {n * sizeof(float), n * sizeof(float), n * sizeof(float), n * sizeof(float),
                        (3 * kRedBlocks + 4) * sizeof(float), n * sizeof(double), (kRedBlocks + 8) * sizeof(double)};
  for (int i = 0; i < 7; ++i) {
    r.mem[i] = balloc(b, sz[i]);
    if (!r.mem[i]) {
      release(b, r);
      return fail(DG_ERR_OOM, "request workspace allocation failed");
    }
  }
  r.e = static_cast<float *>(r.mem[0]);
  r.r = static_cast<float *>(r.mem[1]);
  r.p = static_cast<float *>(r.mem[2]);
  r.q = static_cast<float *>(r.mem[3]);
  r.part = static_cast<float *>(r.mem[4]);
  r.r64 = static_cast<double *>(r.mem[5]);
  r.dpart = static_cast<double *>(r.mem[6]);
  r.used = true;
  // ||b||, then the first FP64 residual and search direction
  double *dscal = r.dpart + kRedBlocks;
  hipLaunchKernelGGL((dot_partial_kernel<double, double>), dim3(kRedBlocks), dim3(kRedThreads), 0, s, r.b, r.b, n,
                     r.dpart);
  hipLaunchKernelGGL((finalize_kernel<double>), dim3(1), dim3(kRedThreads), 0, s, r.dpart, kRedBlocks, dscal);
  double nb2;
  dg_status st = read_scalar(b, dscal, &nb2, s);
  if (st != DG_OK) {
    release(b, r);
    return st;
  }
  r.nb = std::sqrt(nb2);
  *slot = idx;
  if (r.nb == 0.0) {
    hipLaunchKernelGGL((fill_kernel<double>), dim3(kRedBlocks), dim3(kRedThreads), 0, s, r.x, 0.0, n);
    finish(r, DG_OK);
    return DG_OK;
  }
  if ((st = refresh(b, r, s)) != DG_OK) {
    release(b, r);
    return st;
  }
  if (r.rel <= prm->rel_tol) {
    finish(r, DG_OK);
    return DG_OK;
  }
  hipError_t e = start_direction_async(n, r.e, r.r, r.p, static_cast<const float *>(op->diag[1]), r.part, s);
  if (e != hipSuccess) {
    release(b, r);
    return hip_fail(e, "batch admit");
  }
  r.rlast = r.rel;
  r.st.iters_outer = 1;
  r.round0 = b->round + 1;
  b->dirty = true;
  return DG_OK;
}

dg_status dg_batch_run(dg_batch *b, int max_rounds, void *stream)
{
  if (!b || max_rounds < 0) return fail(DG_ERR_ARG, "bad argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  dg_status st;
  for (int rd = 0; rd < max_rounds; ++rd) {
    if (b->dirty && (st = rebuild(b, s)) != DG_OK) return st;
    const int na = (int)b->active.size();
    if (na == 0) break;
    b->round += 1;
    const int grid = b->nitems < 2048 ? b->nitems : 2048;
    hipLaunchKernelGGL(batch_apply_kernel, dim3(grid), dim3(kBatchTpb), 0, s, b->d_desc, na, b->nitems);
    hipLaunchKernelGGL(batch_dot_kernel, dim3(na * kRedBlocks), dim3(kRedThreads), 0, s, b->d_desc);
    hipLaunchKernelGGL(batch_update_kernel, dim3(na * kRedBlocks), dim3(kRedThreads), 0, s, b->d_desc, b->round);
    hipLaunchKernelGGL(batch_pupdate_kernel, dim3(na * kRedBlocks), dim3(kRedThreads), 0, s, b->d_desc, b->round);
    DG_HIP(hipGetLastError());
    bool any_check = false;
    for (int k = 0; k < na; ++k) {
      Request &r = b->req[b->active[k]];
      r.it += 1;
      r.st.iters_inner += 1;
      r.st.applies_f32 += 1;
      if (r.it % r.prm.check_every == 0 || r.it == r.prm.max_iter) any_check = true;
    }
    if (!any_check) continue;
    hipLaunchKernelGGL(batch_gather_rr_kernel, dim3((na + 63) / 64), dim3(64), 0, s, b->d_desc, na, b->d_rr);
    DG_HIP(hipMemcpyAsync(b->h_rr, b->d_rr, sizeof(float) * na, hipMemcpyDeviceToHost, s));
    DG_HIP(hipStreamSynchronize(s));
    for (int k = 0; k < na; ++k) {
      Request &r = b->req[b->active[k]];
      if (!(r.it % r.prm.check_every == 0 || r.it == r.prm.max_iter)) continue;
      const double r32 = std::sqrt((double)b->h_rr[k]);
      if (!std::isfinite(r32)) {
        finish(r, DG_ERR_NOT_CONVERGED);
        b->dirty = true;
        continue;
      }
      if (r32 <= r.prm.rel_tol || r32 < r.prm.rel_tol_inner * r.rlast || r.it == r.prm.max_iter) {
        const int64_t n = r.op->ndofs;
        DG_HIP(flush_correction_async(n, r.x, r.nb, r.e, s));
        if ((st = refresh(b, r, s)) != DG_OK) return st;
        if (r.rel <= r.prm.rel_tol) {
          finish(r, DG_OK);
          b->dirty = true;
          continue;
        }
        if (r.it >= r.prm.max_iter) {
          finish(r, DG_ERR_NOT_CONVERGED);
          b->dirty = true;
          continue;
        }
        r.st.iters_outer += 1;
        r.rlast = r.rel;
        DG_HIP(restart_rz_async(n, r.r, static_cast<const float *>(r.op->diag[1]), r.part, (r.it + 1) & 1, s));
      }
    }
  }
  DG_HIP(hipStreamSynchronize(s));
  return DG_OK;
}

dg_status dg_batch_poll(dg_batch *b, int *done_slots, dg_solve_stats *stats, int capacity, int *n_done)
{
  if (!b || !n_done || capacity < 0 || (capacity > 0 && !done_slots)) return fail(DG_ERR_ARG, "bad argument");
  int c = 0;
  for (int i = 0; i < b->max_slots && c < capacity; ++i) {
    Request &r = b->req[i];
    if (!r.used || !r.done) continue;
    done_slots[c] = i;
    if (stats) stats[c] = r.st;
    ++c;
    release(b, r);
  }
  *n_done = c;
  return DG_OK;
}

dg_status dg_batch_destroy(dg_batch *b)
{
  if (!b) return DG_OK;
  (void)hipDeviceSynchronize();
  for (Request &r : b->req)
    if (r.used) release(b, r);
  if (b->d_desc) (void)hipFree(b->d_desc);
  if (b->d_rr) (void)hipFree(b->d_rr);
  if (b->h_desc) (void)hipHostFree(b->h_desc);
  if (b->h_rr) (void)hipHostFree(b->h_rr);
  if (b->h_scalar) (void)hipHostFree(b->h_scalar);
  delete b;
  return DG_OK;
}

}  // extern "C"
