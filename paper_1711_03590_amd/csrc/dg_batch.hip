// dg_batch.hip -- continuous batching of mixed-precision SIPG solves.
//
// A batch holds up to max_slots requests, each a reliable-update mixed CG
// (dg_cg_solve mode 2) on its own operator.  dg_batch_run advances all
// active requests by one CG iteration per round; a round is:
//   1. per degree and FP32 geometry storage present, one persistent apply
//      kernel whose workgroups walk a list of (request, cell batch) items
//      spanning every active request of that degree and storage, whatever
//      its size (q = A p in FP32, and each item's share of p.q);
//   2. the sum of each request's p.q shares, in item order;
//   3.-4. two batched BLAS kernels over (request, chunk) items of all
//      requests: the x/r update with r.z, r.r partials, and the p update.
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

// threads per workgroup of the batched apply: the stand-alone apply's
// (one wave at 3, 4, 7 and 8 points, two at 5 and 6)
template <int N>
constexpr int kBatchTpb = kTpb<N>;
// degrees served by the persistent kernel: 2..7 (3..8 points per direction)
constexpr int kBatchMinN = 3, kBatchMaxN = 8;
// the same on the host, for a runtime number of points n
inline int batch_tpb(int n)
{
  switch (n) {
    case 3: return kBatchTpb<3>;
    case 4: return kBatchTpb<4>;
    case 5: return kBatchTpb<5>;
    case 6: return kBatchTpb<6>;
    case 7: return kBatchTpb<7>;
    default: return kBatchTpb<8>;
  }
}
// workgroups of the persistent apply launch (a multiple of kXcds): enough
// one-wave workgroups to hold every wave slot the kernels' register use
// leaves (3 or 4 per SIMD); on the serving trace this serves 5-7 % more
// solves per second than 2,048 workgroups of 128 and 256 threads did (a
// grid of one workgroup per item, not persistent, measures about the same)
#ifndef DG_BATCH_GRID
#define DG_BATCH_GRID 12288
#endif
constexpr int kXcds = 8;   // XCDs of an MI355X
static_assert(DG_BATCH_GRID % kXcds == 0, "the persistent grid is a multiple of the XCD count");
#ifndef DG_BATCH_WAVES
#define DG_BATCH_WAVES 4
#endif
#ifndef DG_BATCH_WAVES_HI
#define DG_BATCH_WAVES_HI 3
#endif

template <int N>
constexpr int batch_lds()
{
  using BK = Blocking<N, kBatchTpb<N>>;
  return BK::SMEM;
}
template <int N>
constexpr int kBatchLds = batch_lds<N>();
// occupancy target (waves per SIMD) given to the compiler: the stand-alone
// apply's, at most DG_BATCH_WAVES (DG_BATCH_WAVES_HI from 6 points up)
template <int N>
constexpr int batch_waves()
{
  constexpr int cap = N >= 6 ? DG_BATCH_WAVES_HI : DG_BATCH_WAVES;
  constexpr int occ = Occupancy<N, float>::value;
  return occ < cap ? occ : cap;
}
template <int N>
constexpr int kBatchWaves = batch_waves<N>();

// device descriptor of one active request
struct BatchSlot {
  OpView<float> v;
  int n, gk;
  int64_t ndofs;
  int item0, nitems;   // apply items [item0, item0 + nitems): cell batches of batch_tpb(n) / n^2 cells
  int round0;          // batch round of the request's first iteration
  float *e, *r, *p, *q;
  const float *d;
  float *part;         // kRedBlocks p.q partials (entry 0 the sum, the others zero), 2 kRedBlocks r.z/r.r partials, scal[4]
  float *share;        // per item: its workgroup's share of p.q, written by the apply
};

// A pointer read from the slot table is a generic pointer to the compiler
// (only kernel arguments are known to point to global memory), so every
// access through it would be a flat access, which waits on the LDS counter
// as well and keeps global loads from overlapping LDS work.  Rebuilding it
// from its integer value as a global pointer lets the accesses be global.
template <typename T>
__device__ __forceinline__ T *as_global(T *p)
{
  typedef __attribute__((address_space(1))) T GT;
  return (T *)(GT *)(uintptr_t)p;
}

// the storages a request's FP32 data can have, in descriptor order
constexpr int kBatchKinds = 5;
constexpr int kBatchKind[kBatchKinds] = {AFFINE_CONST, AFFINE_VAR, CURVED, CURVED_MERGED, CURVED_POS};
inline int batch_kind_index(int gk)
{
  for (int g = 0; g < kBatchKinds; ++g)
    if (kBatchKind[g] == gk) return g;
  return -1;
}

// Persistent and XCD-aware, one kernel per degree and storage: the kernel
// for (N, GK) walks the items [item_begin, item_end) of the requests of that
// degree and storage (the descriptors are ordered by both, so these are
// contiguous).  Workgroups are dispatched to the 8 XCDs round robin
// (workgroup b to XCD b mod 8), so the range is cut into 8 contiguous pieces
// and the G/8 workgroups of XCD x walk piece x with stride G/8: neighbouring
// cell batches, which share neighbour blocks and face geometry, then run at
// about the same time on one XCD and meet in its L2.  G is a multiple of 8;
// every workgroup leaves its loop at the end of its piece.  The apply is
// inlined (a call would save and restore the callee-saved registers through
// scratch memory on every item), and a kernel holds one storage's code only,
// so that its register count is that storage's and not the largest one's.
template <int N, int GK>
__global__ void __launch_bounds__(kBatchTpb<N>, (kBatchWaves<N>))
batch_apply_kernel(const BatchSlot *__restrict__ slots, int nslots, int slot0, int item_begin, int item_end)
{
  __shared__ float smem[kBatchLds<N>];
  constexpr int X = kXcds;
  const int xcd = blockIdx.x % X, w = blockIdx.x / X, nw = gridDim.x / X;
  const int nitems = item_end - item_begin;
  const int per = (nitems + X - 1) / X;
  const int lo = item_begin + xcd * per, hi = min(item_end, lo + per);
  for (int item = lo + w; item < hi; item += nw) {
    int s = slot0;
    while (s + 1 < nslots && slots[s + 1].item0 <= item) ++s;
    const BatchSlot &sl = slots[s];
    const DotOut<float> dot{as_global(sl.share)};
    // the thread index, redefined per item (an empty asm statement the
    // compiler cannot see through): otherwise everything the apply derives
    // from it alone (line bases, LDS offsets, the weights of the thread's
    // indices) is hoisted out of this loop and held in registers across it,
    // 96-111 VGPRs instead of 54-83, and the degree-4 and degree-6 applies
    // ran 7-12 % slower than stand-alone
    int tid = (int)threadIdx.x;
    asm volatile("" : "+v"(tid));
    apply_batch<N, float, GK, kBatchTpb<N>, true>(sl.v, as_global(sl.p), as_global(sl.q), item - sl.item0, smem,
                                                  dot, tid);
    __syncthreads();
  }
}

// the current r.z slot of a request at this round (ping-pong by its own
// iteration count: iteration it uses scal[it & 1])
__device__ __forceinline__ int batch_cur(const BatchSlot &sl, int round) { return (round - sl.round0 + 1) & 1; }

// p.q of every request: the sum of its items' shares in item order, into
// part[0] (the other p.q partials stay zero)
__global__ void __launch_bounds__(kSumThreads) batch_shares_kernel(const BatchSlot *__restrict__ slots)
{
  __shared__ float sh[kSumThreads];
  const BatchSlot &sl = slots[blockIdx.x];
  sum_shares_body<float>(sl.share, sl.nitems, sl.part, sh);
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
  float *e = nullptr, *r = nullptr, *p = nullptr, *q = nullptr, *part = nullptr, *share = nullptr;
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
  std::vector<int> active;   // request index per descriptor position (ordered by degree)
  std::vector<int> refreshing;   // descriptor positions taking a refinement step this round
  int nitems = 0;
  // per number of points n and storage g (kBatchKind): descriptors
  // [slot0[n][g], ...) and items [item0[n][g], item1[n][g])
  int slot0[kBatchMaxN + 1][kBatchKinds] = {}, item0[kBatchMaxN + 1][kBatchKinds] = {},
      item1[kBatchMaxN + 1][kBatchKinds] = {};
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

// Enqueue the FP64 residual of request r and the copy of its squared norm
// into host slot *host (pinned); the caller synchronises the stream once for
// all the requests it refreshes, then calls refresh_done.
dg_status refresh_async(Request &r, double *host, hipStream_t s)
{
  double *dscal = r.dpart + kRedBlocks;
  DG_HIP(rel_residual_async(r.op, r.b, r.x, r.r64, r.dpart, dscal, r.r, r.nb, s));
  DG_HIP(hipMemcpyAsync(host, dscal, sizeof(double), hipMemcpyDeviceToHost, s));
  return DG_OK;
}

void refresh_done(Request &r, double norm2)
{
  r.rel = std::sqrt(norm2) / r.nb;
  r.st.applies_f64 += 1;
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
  // descriptors ordered by degree and storage, so that the items of each
  // (degree, storage) are contiguous
  for (int n = kBatchMinN; n <= kBatchMaxN; ++n) for (int g = 0; g < kBatchKinds; ++g) {
    b->slot0[n][g] = (int)b->active.size();
    b->item0[n][g] = item;
    for (int i = 0; i < b->max_slots; ++i) {
      Request &r = b->req[i];
      if (!r.used || r.done || r.op->n != n || batch_kind_index(r.op->gk32) != g) continue;
      BatchSlot &d = b->h_desc[b->active.size()];
      const int cells_per_item = batch_tpb(n) / (n * n);
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
      d.share = r.share;
      item += d.nitems;
      b->active.push_back(i);
    }
    b->item1[n][g] = item;
  }
  b->nitems = item;
  if (!b->active.empty()) {
    DG_HIP(hipMemcpyAsync(b->d_desc, b->h_desc, sizeof(BatchSlot) * b->active.size(), hipMemcpyHostToDevice, s));
    DG_HIP(hipStreamSynchronize(s));  // the staging buffer is rewritten by the next rebuild
  }
  b->dirty = false;
  return DG_OK;
}

// the persistent apply of the requests with N points and storage kBatchKind[g]
template <int N>
void launch_batch_apply(int g, int grid, const dg_batch *b, int na, hipStream_t s)
{
  const int a0 = b->slot0[N][g], a1 = b->item0[N][g], a2 = b->item1[N][g];
  const dim3 gd(grid), bd(kBatchTpb<N>);
  switch (kBatchKind[g]) {
    case AFFINE_CONST: hipLaunchKernelGGL((batch_apply_kernel<N, AFFINE_CONST>), gd, bd, 0, s, b->d_desc, na, a0, a1, a2); break;
    case AFFINE_VAR: hipLaunchKernelGGL((batch_apply_kernel<N, AFFINE_VAR>), gd, bd, 0, s, b->d_desc, na, a0, a1, a2); break;
    case CURVED: hipLaunchKernelGGL((batch_apply_kernel<N, CURVED>), gd, bd, 0, s, b->d_desc, na, a0, a1, a2); break;
    case CURVED_MERGED: hipLaunchKernelGGL((batch_apply_kernel<N, CURVED_MERGED>), gd, bd, 0, s, b->d_desc, na, a0, a1, a2); break;
    default: hipLaunchKernelGGL((batch_apply_kernel<N, CURVED_POS>), gd, bd, 0, s, b->d_desc, na, a0, a1, a2); break;
  }
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
  b->refreshing.resize(max_slots);
  bool ok = hipMalloc(reinterpret_cast<void **>(&b->d_desc), sizeof(BatchSlot) * max_slots) == hipSuccess &&
            hipMalloc(reinterpret_cast<void **>(&b->d_rr), sizeof(float) * max_slots) == hipSuccess &&
            hipHostMalloc(reinterpret_cast<void **>(&b->h_desc), sizeof(BatchSlot) * max_slots,
                          hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc(reinterpret_cast<void **>(&b->h_rr), sizeof(float) * max_slots, hipHostMallocDefault) ==
                hipSuccess &&
            hipHostMalloc(reinterpret_cast<void **>(&b->h_scalar), sizeof(double) * (max_slots + 2),
                          hipHostMallocDefault) ==
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
  if (batch_kind_index(op->gk32) < 0) return fail(DG_ERR_UNSUPPORTED, "no batched apply for this geometry storage");
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
  const int64_t cells_per_item = batch_tpb(op->n) / (op->n * op->n);
  const int64_t items = (op->ncells + cells_per_item - 1) / cells_per_item;
  const size_t sz[8] = {n * sizeof(float), n * sizeof(float), n * sizeof(float), n * sizeof(float),
                        (3 * kRedBlocks + 4) * sizeof(float), n * sizeof(double), (kRedBlocks + 8) * sizeof(double),
                        (size_t)items * sizeof(float)};
  for (int i = 0; i < 8; ++i) {
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
  r.share = static_cast<float *>(r.mem[7]);
  r.used = true;
  // the p.q partials past entry 0 stay zero (entry 0 takes the sum of the shares)
  hipLaunchKernelGGL((fill_kernel<float>), dim3(1), dim3(kRedThreads), 0, s, r.part, 0.0f, (int64_t)kRedBlocks);
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
    for (int n = kBatchMinN; n <= kBatchMaxN; ++n) for (int g = 0; g < kBatchKinds; ++g) {
      const int items = b->item1[n][g] - b->item0[n][g];
      if (items == 0) continue;
      // a multiple of the XCD count, at most DG_BATCH_GRID
      const int want = items < DG_BATCH_GRID ? items : DG_BATCH_GRID;
      const int grid = ((want + kXcds - 1) / kXcds) * kXcds;
      switch (n) {
        case 3: launch_batch_apply<3>(g, grid, b, na, s); break;
        case 4: launch_batch_apply<4>(g, grid, b, na, s); break;
        case 5: launch_batch_apply<5>(g, grid, b, na, s); break;
        case 6: launch_batch_apply<6>(g, grid, b, na, s); break;
        case 7: launch_batch_apply<7>(g, grid, b, na, s); break;
        default: launch_batch_apply<8>(g, grid, b, na, s); break;
      }
    }
    hipLaunchKernelGGL(batch_shares_kernel, dim3(na), dim3(kSumThreads), 0, s, b->d_desc);
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
    // refinement steps of every request that reached one: all their FP64
    // residuals are enqueued first and read back with one synchronisation
    // (each request's own kernels keep their order, so its result does not
    // depend on the others)
    int nref = 0;
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
        DG_HIP(flush_correction_async(r.op->ndofs, r.x, r.nb, r.e, s));
        if ((st = refresh_async(r, b->h_scalar + 2 + k, s)) != DG_OK) return st;
        b->refreshing[nref++] = k;
      }
    }
    if (nref == 0) continue;
    DG_HIP(hipStreamSynchronize(s));
    for (int j = 0; j < nref; ++j) {
      const int k = b->refreshing[j];
      Request &r = b->req[b->active[k]];
      refresh_done(r, b->h_scalar[2 + k]);
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
      DG_HIP(restart_rz_async(r.op->ndofs, r.r, static_cast<const float *>(r.op->diag[1]), r.part, (r.it + 1) & 1,
                              s));
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
