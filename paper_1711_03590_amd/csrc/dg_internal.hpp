// dg_internal.hpp -- shared host/device declarations of the SIPG library.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstddef>
#include <cstdint>
#include <string>

#include "dg.h"

namespace dgk {

// Geometry representation of an op (Sec. 5):
//   AFFINE_CONST  constant Jacobian, constant coefficient: nothing stored per point
//   AFFINE_VAR    constant Jacobian, c * det J * w per cell point, c * ds per face point
//   CURVED        G3: J^{-T} (9) and c * det J * w per cell point;
//                 face: j = J^{-1} n (3, Design Choice 5) and c * ds per face point
//   CURVED_MERGED G4: the symmetric c * det J * w * J^{-1} J^{-T} (6) per cell
//                 point; faces as CURVED
//   ADVECTION     the advection operator (Sec. 2, Eq. (1)): J^{-1} c det J w
//                 (3) per cell point, (c . n) ds for the +e_a normal per face point
//   CURVED_POS    G2: the quadrature-point positions (3, relative to the
//                 cell's unmapped corner) and c per cell point, the Jacobian
//                 taken in the kernel by collocation derivatives; faces as CURVED
enum GeomKind : int { AFFINE_CONST = 0, AFFINE_VAR = 1, CURVED = 2, CURVED_MERGED = 3, ADVECTION = 4, CURVED_POS = 5 };

// faces carry j = J^{-1} n and c ds per point
constexpr bool curved_faces(int gk) { return gk == CURVED || gk == CURVED_MERGED || gk == CURVED_POS; }
// stored values per cell quadrature point
constexpr int cell_values(int gk)
{
  return gk == CURVED ? 10
                      : (gk == CURVED_MERGED ? 6
                                             : (gk == CURVED_POS ? 4 : (gk == ADVECTION ? 3 : (gk == AFFINE_VAR ? 1 : 0))));
}
constexpr int face_values(int gk) { return curved_faces(gk) ? 4 : ((gk == AFFINE_VAR || gk == ADVECTION) ? 1 : 0); }

constexpr int kMinN = 2;  // degree 1
constexpr int kMaxN = 9;  // degree 8

// Per-precision device data of an op.  Cell quantities are stored as
// separate arrays ("structure of arrays", Sec. 5), each ncells * n^3 long in
// cell-then-point order; face quantities per direction a, each
// nfaces[a] * n^2 long, faces of direction a numbered like cells with
// ncell[a] + 1 planes in that direction.
template <typename Real>
struct GeomData {
  const Real *cell = nullptr;          // CURVED: 10 arrays (J^{-T} row-major, then cJxW);
                                       // CURVED_MERGED: 6 (M00, M01, M02, M11, M12, M22);
                                       // CURVED_POS: 4 (x - X0, y - Y0, z - Z0, c); AFFINE_VAR: 1 (cJxW)
  const Real *face[3] = {nullptr, nullptr, nullptr};  // curved: 4 arrays (j0, j1, j2, cds); AFFINE_VAR: 1 (cds)
  int64_t cell_stride = 0;             // elements between successive quantity arrays
  int64_t face_stride[3] = {0, 0, 0};
};

// Everything a kernel needs to know about the problem, passed by value.
template <typename Real>
struct OpView {
  int ncell[3];
  int ncells;
  int bc[6];                // 0 Dirichlet, 1 Neumann, 2 ghost (traces from ghost[side])
  Real inv_h[3];            // 1 / h_a (affine Jacobian)
  Real tau[3];              // (k+1)^2 / h_a
  Real c_vol;               // AFFINE_CONST: c * hx * hy * hz
  Real c_area[3];           // AFFINE_CONST: c * h_t1 * h_t2 for faces normal to a
  GeomData<Real> g;
  int reverse = 0;          // walk the cell batches last to first (set per launch)
  const Real *ghost[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};  // per launch
};

constexpr int kBcGhost = 2;

// position of cell ci in the plane of its faces normal to direction A
template <int A>
__host__ __device__ __forceinline__ int64_t side_plane_index(const int (&nc)[3], const int (&ci)[3])
{
  if constexpr (A == 0) return ci[1] + (int64_t)nc[1] * ci[2];
  else if constexpr (A == 1) return ci[0] + (int64_t)nc[0] * ci[2];
  else return ci[0] + (int64_t)nc[0] * ci[1];
}

}  // namespace dgk

// The opaque op handle.
struct dg_op {
  dg_mesh mesh;
  int degree = 0, n = 0;
  dg_geometry geom;
  dg_coefficient coef;
  dg_velocity vel{};         // advection ops only
  int basis = 0;             // SIPG ops: DG_BASIS_NODAL or DG_BASIS_HERMITE
  bool ghost_sides = false;  // some mesh.bc is DG_BC_GHOST
  mutable std::atomic<unsigned> sweeps{0};  // SIPG applies so far: odd ones walk the cells backwards
  unsigned precisions = 0;
  int gk = 0;                // geometry kind of the FP64 data (and of the op)
  int gk32 = 0;              // geometry kind of the FP32 data (differs for DG_STORE_MIXED)
  int64_t ncells = 0, ndofs = 0, nfaces[3] = {0, 0, 0};
  double h[3] = {0, 0, 0};
  int device = 0;
  dg_allocator alloc{};
  bool own_alloc = true;
  // device allocations (nullptr when absent)
  void *cell_geo[2] = {nullptr, nullptr};   // [0] FP64, [1] FP32
  void *face_geo[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
  void *diag[2] = {nullptr, nullptr};
  void *scratch = nullptr;                  // small reduction workspace
  size_t scratch_bytes = 0;
  dgk::OpView<double> v64{};
  dgk::OpView<float> v32{};
};

namespace dgk {

// error reporting (thread-local message)
void set_error(const std::string &msg);
dg_status fail(dg_status st, const std::string &msg);
dg_status hip_fail(hipError_t e, const char *what);

#define DG_HIP(call)                                        \
  do {                                                      \
    hipError_t e_ = (call);                                 \
    if (e_ != hipSuccess) return ::dgk::hip_fail(e_, #call); \
  } while (0)

void *op_alloc(dg_op *op, size_t bytes);
void op_free(dg_op *op, void *p);

// kernel launchers (one translation unit per n instantiates them; launch_apply
// and launch_face_traces are declared with their definitions in kernels.hpp)
template <int N>
hipError_t launch_diag(const dg_op *op, void *diag64, void *diag32, hipStream_t s);

template <int N>
hipError_t launch_apply_dot(const dg_op *op, const void *src, void *dst, bool f32, void *part, hipStream_t s);
template <int N>
int apply_workgroups(const dg_op *op);

hipError_t launch_apply_any(const dg_op *op, const void *src, void *dst, bool f32, hipStream_t s,
                            const void *const *ghost = nullptr);
// dst = A src for the SIPG operator and the workgroup shares of src.dst in
// part (apply_workgroups_any(op) entries, see DotOut)
hipError_t launch_apply_dot_any(const dg_op *op, const void *src, void *dst, bool f32, void *part, hipStream_t s);
int apply_workgroups_any(const dg_op *op);
hipError_t launch_diag_any(const dg_op *op, void *diag64, void *diag32, hipStream_t s);

}  // namespace dgk
