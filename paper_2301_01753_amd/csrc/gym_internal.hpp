// Internal declarations of the gym library (host side).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/gym.h"
#include "minres_step.hpp"

namespace gym {

constexpr int kMaxR = 4;          // highest degree with compiled kernels
constexpr int kMaxQ = kMaxR + 2;  // widest Gauss rule (load vectors: r + 2)

// Thread-local error message, returned by gym_last_error().
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);

#define GYM_HIP(call)                                              \
  do {                                                             \
    hipError_t _e = (call);                                        \
    if (_e != hipSuccess) return ::gym::hip_fail(_e, #call);       \
  } while (0)

// 1-D tables on [0,1] for degree r (host, FP64): GLL nodes, Gauss rule of q
// points, nodal values phi_i(x_t) and edge values e_j(x_t).
struct Tables1D {
  int r = 0, q = 0;
  std::vector<double> nodes;    // r + 1
  std::vector<double> gx, gw;   // q
  std::vector<double> phi;      // q x (r + 1), row t
  std::vector<double> edge;     // q x r
};
Tables1D make_tables(int r, int q);
// 1-D element masses of degree r from the q = r + 1 Gauss rule: nodal
// (r+1)^2 and edge r^2 entries, row-major.
void element_masses_1d(int r, std::vector<double>& mn, std::vector<double>& me);
std::vector<double> gll_nodes(int r);
void gauss_rule(int q, std::vector<double>& x, std::vector<double>& w);

// Per-component description of a space: which axes are nodal, and the kept
// lattice positions per axis [start, start + count).
struct CompDesc {
  int nodal_mask = 0;        // bit a set -> nodal along axis a
  int64_t start[3] = {0, 0, 0};
  int64_t count[3] = {1, 1, 1};
  int64_t offset = 0;        // first global index of the block
};

struct SpaceDesc {
  int kind = 0, dim = 3, r = 1, bc = 0, ncomp = 1;
  int periodic = 0;  // bit a: axis a closes on itself (position m_a is position 0)
  int64_t m[3] = {1, 1, 1};
  CompDesc comp[3];
  int64_t ndofs = 0;
};
// periodic: bit a makes axis a periodic, with m_a positions for nodal and edge
// functions alike and no boundary condition along it.
SpaceDesc make_space_desc(int kind, int dim, const int64_t nel[3], int r, int bc, int periodic = 0);

}  // namespace gym

struct gym_op;
namespace gym {
struct OpParams;
// Parameters of one block-operator apply (capi.cpp), and the apply itself.
void build_op_params(const gym_op* op, const void* x, void* y, OpParams& p, int& prob);
// Row sums of the mass matrix without boundary conditions at the kept
// unknowns.  On curved cells they come from a device apply of the curved
// mass (curved_exact), or, as a preconditioner only, from the box with the
// same spacing.
std::vector<double> lumped_diag_host(const gym_space* sp, bool curved_exact = true);
// y = d x or d^T x (gym_d_apply) for nrhs contiguous vectors (strides: the
// spaces' ndofs), one launch.
int d_apply_n(const gym_space* from, const gym_space* to, int transpose, int nrhs, const double* x, double* y,
              hipStream_t stream);
// Diagonal of the mass matrix at the kept unknowns (on curved cells that of
// the box with the same spacing).
std::vector<double> mass_diag_host(const gym_space* sp);
// The same row sums in factored form: at lattice position p, component c has
// sc[c] prod_a w_a(p_a), w_a = rn[a] (nodal along axis a, r N_a + 1 values)
// or re[a] (edge, r N_a values); the product is taken in axis order.
struct LumpedTables {
  std::vector<double> rn[3], re[3];
  double sc[3];
};
LumpedTables lumped_tables_host(const gym_space* sp);
// y = A x; with `mr` the launch also carries the first half of that MINRES
// step (partial sums of x . A x, op_workgroups of them per rhs).
// matrix_core = false keeps to kernels that allocate nothing on first use.
int launch_op_apply(const gym_op* op, int prec, int nrhs, const void* x, void* y, hipStream_t s,
                    const MrStep* mr = nullptr, bool matrix_core = true);
// Partial sums per rhs of the launch above for this precision and nrhs.
int op_workgroups(const gym_op* op, int prec, int nrhs, int* wg, bool matrix_core = true);
}  // namespace gym

struct gym_ctx {
  int device = 0;
  int ncu = 0;
  int mass_form = 0;  // GYM_OPT_MASS_FORM
  int tile = 0;       // GYM_OPT_TILE
  int curved_kernel = 0;  // GYM_OPT_CURVED_KERNEL
};

struct gym_mesh {
  gym_ctx* ctx = nullptr;
  int dim = 3;
  int64_t nel[3] = {1, 1, 1};
  double lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1}, h[3] = {1, 1, 1};
  bool curved = false;              // vertex array given
  int periodic = 0;                 // bit a: axis a periodic (affine boxes only)
  double* d_vertices = nullptr;     // device copy, (N+1)^d x d
  std::vector<double> vertices;     // host copy
  // curved: Gauss-point metrics per degree r (q = r + 1), FP64 [0] and FP32
  // [1], built on first use (geom.hpp) and kept until the mesh is destroyed
  mutable void* qd[2][gym::kMaxR + 1] = {};
};

namespace gym {
// The Gauss-point metrics of a curved mesh for degree r (f32: FP32 copy),
// allocated and filled on first use (synchronously).
int mesh_qdata(const gym_mesh* m, int r, int f32, const void** out);
// Device address of the allocation-free solve's scratch array on `device`
// (current), asked once per device (noalloc.hip).
int noalloc_init(int device);
}  // namespace gym

struct gym_space {
  gym_ctx* ctx = nullptr;
  const gym_mesh* mesh = nullptr;
  gym::SpaceDesc desc;
  double* d_diag = nullptr;         // lazily built Jacobi diagonal
  void* band = nullptr;             // periodic spaces: the mass as 1-D band passes (SpaiParams)
  double* band_mem = nullptr;
  // Krylov workspace for mass solves
  std::vector<void*> work;
  int work_nrhs = 0;
};

struct gym_op {
  gym_ctx* ctx = nullptr;
  const gym_mesh* mesh = nullptr;
  int problem = 0, r = 1;
  gym::SpaceDesc sa, sb;             // first / second unknown block
  int64_t na = 0, nb = 0;
  double* d_prec = nullptr;          // 1 / diag, n = na + nb
  std::vector<void*> work;           // Krylov workspace
  int work_nrhs = 0;
  size_t work_bytes = 0;
  void* schur = nullptr;             // gym::SchurPrec, built on first use
  void* mfma = nullptr;              // bf16 matrix-core apply state, built on first use
  double* hc_halo = nullptr;         // curved Hodge matrix-core apply: tile-boundary sums
  long long hc_halo_n = 0;
};
