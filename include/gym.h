/*
 * gym.h -- C ABI of the MI355X matrix-free FEEC operator library.
 *
 * The library applies, inside Krylov solves, the discrete operators of the
 * finite-element de Rham complex of "Generalized Yee methods" (arXiv
 * 2301.01753), section 2: integer incidence matrices G, C, D (eq.
 * discreteDeRham, CG = 0, DC = 0) and the metric mass matrices
 * (M_p)_ij = int (Lambda_i, Lambda_j)_p dx, evaluated matrix-free by
 * sum-factorised tensor contractions at Gauss points.  Spaces are the
 * tensor-product family Q_r^- Lambda^k on structured quad/hex meshes
 * (r = 1 is the generalized Whitney family of section 4.1).
 *
 * Conventions shared by every call:
 *   - Status: 0 = GYM_OK, > 0 warning, < 0 error.  No call aborts or throws;
 *     gym_last_error() returns a message for the calling thread.
 *   - Vectors passed as `void*`/`double*` are DEVICE pointers owned by the
 *     caller, in the canonical layout below; arrays documented as host
 *     pointers are read during the call only.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Apply calls are stream-ordered and asynchronous; *_create, gym_solve
 *     (which synchronises its stream) and the gym_serve_* calls are blocking.
 *   - Canonical layout of a space's vector: component blocks in axis order
 *     (x, y, z); inside a block, lexicographic over the lattice positions
 *     with x fastest.  Per axis the lattice has m = r*N cells; nodal
 *     positions are 0..m (1..m-1 under essential boundary conditions), edge
 *     positions 0..m-1.  A degree of freedom is the integral of the form over
 *     its lattice k-cell (the integral-normalised version of the paper's eq.
 *     WhitneyFormDefn); with this choice incidence is exactly +-1.
 *   - Multiple right-hand sides: `nrhs` vectors stored back to back,
 *     element (rhs, i) at rhs*ndofs + i.
 *   - Handles are not thread-safe; calls on one context from several threads
 *     must be serialised by the caller (the serving loop is the exception:
 *     gym_serve_submit/poll may be called from any thread).
 */
#ifndef GYM_H
#define GYM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define GYM_OK               0
#define GYM_W_NOT_CONVERGED  1   /* solve hit maxit; x holds the last iterate */
#define GYM_E_ARG           -1   /* invalid argument (message says which)     */
#define GYM_E_OOM           -2   /* device allocation failed / over budget    */
#define GYM_E_HIP           -3   /* a HIP runtime call failed                 */
#define GYM_E_INVALID_MESH  -4   /* det J <= 0 at a quadrature point          */
#define GYM_E_BREAKDOWN     -5   /* Krylov breakdown (NaN, indefinite M^-1)   */
#define GYM_E_UNSUPPORTED   -6   /* valid request this build does not handle  */

/* ---- enumerations ---------------------------------------------------- */
#define GYM_H1     0   /* Lambda^0: nodal                                    */
#define GYM_HCURL  1   /* Lambda^1: component c edge along c                 */
#define GYM_HDIV   2   /* Lambda^{d-1}: component c nodal along c (flux)     */
#define GYM_L2     3   /* Lambda^d: cell integrals                           */

#define GYM_BC_NATURAL    0
#define GYM_BC_ESSENTIAL  1   /* drop nodal positions 0 and m (zero trace)   */

#define GYM_F64   0   /* contractions and vectors in FP64                    */
#define GYM_F32   1   /* contractions in FP32, vectors FP32                  */
#define GYM_BF16  2   /* contraction operands rounded to bf16 (round to
                         nearest even), products accumulated in FP32 on the
                         vector ALUs; FP32 vectors; affine meshes only      */

#define GYM_MIXED_POISSON  0  /* H(div) x L2:  [M2, -D^T M3; -M3 D, 0]       */
#define GYM_HODGE1         1  /* H1_0 x H0(curl): [-M0, G^T M1; M1 G, C^T M2 C] */

#define GYM_MINRES  0
#define GYM_CG      1   /* for SPD operators only (mass solves)              */

#define GYM_MODE_F64      0  /* plain FP64 Krylov                            */
#define GYM_MODE_IR_F32   1  /* FP64 iterative refinement, FP32 inner solve   */
#define GYM_MODE_IR_BF16  2  /* FP64 iterative refinement, BF16 contractions  */

/* Preconditioners of gym_solve.  The paper preconditions only with a
 * diagonal (section 5.1, its Sylvester PCG); the block operators take the
 * diagonal of each block's own Gram-type operator:
 *   Poisson: diag(M2 + D^T M3 D), diag(M3);
 *   Hodge:   diag(M0 + G^T M1 G), diag(M1 + C^T M2 C)
 * (gym_op_precond_diag).  NONE runs unpreconditioned MINRES.
 * SCHUR (mixed Poisson on affine 3-D boxes): diag(diag(M2), S) with
 * S = M3 D diag(M2)^-1 D^T M3, the Schur complement of the block system with
 * M2 replaced by its diagonal; S is inverted exactly by simultaneous
 * diagonalisation of its per-axis factors (dense 1-D transforms along the
 * three axes).  Its set-up (three symmetric eigenproblems of size r N_a on
 * the host) runs on first use. */
#define GYM_PRECOND_JACOBI 0
#define GYM_PRECOND_NONE   1
#define GYM_PRECOND_SCHUR  2

typedef struct gym_ctx gym_ctx;
typedef struct gym_mesh gym_mesh;
typedef struct gym_space gym_space;
typedef struct gym_op gym_op;
typedef struct gym_server gym_server;
typedef struct gym_maxwell gym_maxwell;

/* ---- context --------------------------------------------------------- */
/* Bind to HIP device `device`, upload the 1-D basis/quadrature tables.
 * Errors: GYM_E_ARG (bad device), GYM_E_HIP. */
int gym_create(gym_ctx** out, int device);
/* Frees the context.  Meshes, spaces, operators and servers created from it
 * must be destroyed first. */
int gym_destroy(gym_ctx* ctx);
/* Last error message of the calling thread ("" if none).  Valid until the
 * next failing call on this thread. */
const char* gym_last_error(void);

/* Context options (apply to every later call on the context).
 * GYM_OPT_MASS_FORM: 0 = automatic (Kronecker form of the element masses
 *   on affine meshes, Gauss-point form otherwise), 1 = always evaluate at
 *   Gauss points (the paper's mass-matrix definition, quadrature r + 1).
 *   Both forms compute the same operator up to rounding.
 * GYM_OPT_TILE: 0 = automatic (large tiles unless the mesh has fewer of
 *   them than the device has CUs), 1 = large tiles (one workgroup per CU),
 *   2 = small tiles (several workgroups per CU).
 * GYM_OPT_CURVED_KERNEL: 0 = automatic (the FP64 Hodge apply of degree 3 on
 *   curved cells runs its 1-D contractions on the matrix cores, one cell per
 *   4 x 4 block; other curved applies use the tile kernel), 1 = always the
 *   tile kernel.  Both compute the same operator up to rounding.
 * Errors: GYM_E_ARG for an unknown option or value. */
#define GYM_OPT_MASS_FORM 0
#define GYM_OPT_TILE      1
#define GYM_OPT_CURVED_KERNEL 2
int gym_ctx_set(gym_ctx* ctx, int option, int value);

/* ---- mesh (paper section 2: the mesh T_h) ----------------------------- */
/* Structured mesh of nel[0] x nel[1] (x nel[2]) cells, dim = 2 or 3.
 * vertices: HOST array of (nel[0]+1)*...*(nel[d-1]+1)*dim doubles,
 * vertex (i,j,k) at ((k*(ny+1) + j)*(nx+1) + i)*dim, or NULL for the uniform
 * box [lo, hi].  Each cell is the multilinear image of [0,1]^d of its
 * corners.  The array is copied.  A NULL vertex array gives an affine mesh;
 * a non-NULL one is treated as curved (per-quadrature-point Jacobians).
 * Errors: GYM_E_ARG, GYM_E_INVALID_MESH (det J <= 0 at a Gauss point of
 * any degree <= 4 rule), GYM_E_OOM. */
int gym_mesh_create(gym_ctx* ctx, int dim, const int64_t nel[3],
                    const double* vertices, const double lo[3],
                    const double hi[3], gym_mesh** out);
/* Structured mesh of the box [lo, hi] (NULL: the unit box) with seeded
 * vertex perturbations, the perturbed-hexahedron workloads of the paper's
 * unstructured-mesh experiments recast on a lattice (section 7; the shape
 * of M_p on non-affine cells is section 2).  Vertex (i, j, k) moves by
 * (2 u - 1) perturb_frac h_a along axis a, h_a = (hi_a - lo_a) / nel_a, with
 * u = (z >> 11) 2^-53 and z the SplitMix64 word (Steele, Lea & Flood 2014)
 *   z = mix(seed + (w + 1) 0x9E3779B97F4A7C15),  w = dim * v + a,
 *   v = i + (nel_0 + 1) (j + (nel_1 + 1) k),
 * the same word definition as the serving right-hand sides.  The offset is
 * zero along a on the faces i_a = 0 and i_a = nel_a, so boundary vertices
 * slide in their face or edge and corners stay fixed; the unperturbed
 * coordinate is lo_a + ((hi_a - lo_a) i_a) / nel_a.  perturb_frac = 0 gives
 * the affine box (gym_mesh_create with vertices = NULL); perturb_frac > 0 a
 * curved mesh exactly as if its vertex array had been passed to
 * gym_mesh_create.  Below 1/6 every cell is valid; larger values may return
 * GYM_E_INVALID_MESH.  Errors: GYM_E_ARG (perturb_frac outside [0, 0.5)),
 * and those of gym_mesh_create. */
int gym_mesh_structured(gym_ctx* ctx, int dim, const int64_t nel[3],
                        const double lo[3], const double hi[3],
                        double perturb_frac, uint64_t seed, gym_mesh** out);

/* Make the axes in mask (bit a: axis a) of an affine box periodic: position
 * m_a of every lattice closes onto position 0, so spaces created on the mesh
 * afterwards keep r*nel[a] positions along such an axis for nodal and edge
 * functions alike and apply no boundary condition along it (the paper's
 * torus of section 7.3 and the 20 x 20 mesh of section 7.5).  Serves the
 * time stepping (gym_maxwell_*) and its eigenmodes, incidence and mass
 * applies and mass solves (FP64, through 1-D band passes); gym_op_create
 * refuses periodic meshes.  Call before creating spaces on the mesh.
 * Errors: GYM_E_ARG (bits beyond dim), GYM_E_UNSUPPORTED (curved mesh). */
int gym_mesh_set_periodic(gym_mesh* mesh, int mask);
/* Vertex coordinates of a mesh into the HOST array `vertices`
 * ((nel_0+1)...(nel_{d-1}+1) x dim doubles, the layout of gym_mesh_create);
 * for an affine mesh, the uniform lattice of [lo, hi]. */
int gym_mesh_vertices(const gym_mesh* mesh, double* vertices);
int gym_mesh_destroy(gym_mesh* mesh);

/* ---- spaces (paper section 2: Lambda^p(T_h) with basis Lambda^p) ------ */
/* kind: GYM_H1..GYM_L2; degree r in 1..4; bc: GYM_BC_*. */
int gym_space_create(gym_ctx* ctx, const gym_mesh* mesh, int kind, int degree,
                     int bc, gym_space** out);
int64_t gym_space_ndofs(const gym_space* space);
int gym_space_destroy(gym_space* space);

/* The canonical order of a space's vector (the only layout: every kernel
 * reads and writes it directly, see the conventions above).  Component c
 * occupies [offset[c], offset[c] + prod_a count[c][a]); its entry at kept
 * lattice position (p_0, p_1, p_2) sits at
 *   offset[c] + (p_0 - start[c][0]) + count[c][0] ((p_1 - start[c][1]) +
 *   count[c][1] (p_2 - start[c][2])),
 * with p_a in [start[c][a], start[c][a] + count[c][a]).  Bit a of
 * nodal_mask[c] is set when the component is nodal along axis a (positions
 * 0..m_a, m_a = r nel_a) and clear when it is an edge along a (cells
 * 0..m_a-1).  Unused axes (2-D) have start 0, count 1. */
typedef struct gym_layout {
  int kind;             /* GYM_H1 .. GYM_L2                                */
  int dim, degree, bc;
  int ncomp;            /* 1 or dim                                        */
  int nodal_mask[3];
  int64_t m[3];         /* lattice cells per axis, r * nel                 */
  int64_t start[3][3];  /* [component][axis]                               */
  int64_t count[3][3];
  int64_t offset[3];
  int64_t ndofs;
} gym_layout;
int gym_space_layout(const gym_space* space, gym_layout* layout);

/* ---- incidence (paper eq. discreteDeRham) ----------------------------- */
/* y = d x (transpose = 0) or y = d^T x (transpose = 1) where d: from -> to is
 * G (H1 -> HCURL), C (HCURL -> HDIV in 3-D, HCURL -> L2 in 2-D) or
 * D (HDIV -> L2).  FP64, device pointers, sizes from gym_space_ndofs
 * (x has the size of `from` for d and of `to` for d^T).  Each output entry
 * is summed from +0.0 over its +-1 terms in ascending input-index order, so
 * the result is bit-reproducible.  Errors: GYM_E_ARG (spaces not adjacent
 * in the complex, different meshes or degrees). */
int gym_d_apply(const gym_space* from, const gym_space* to, int transpose,
                const double* x, double* y, void* stream);

/* ---- mass (paper section 2: (M_p)_ij) --------------------------------- */
/* y = M x for `nrhs` vectors.  prec GYM_F64: x, y are double*; GYM_F32 and
 * GYM_BF16: x, y are float*.  Quadrature: Gauss, r + 1 points per axis. */
int gym_mass_apply(const gym_space* space, int prec, int nrhs, const void* x,
                   void* y, void* stream);

/* ---- block operators (readings built from G, C, D, M_p) --------------- */
/* problem GYM_MIXED_POISSON: unknowns [s (HDIV, natural); p (L2)].
 * problem GYM_HODGE1 (3-D): unknowns [sigma (H1, essential); u (HCURL,
 * essential)]; its (2,2) block C^T M2 C is the paper's curl-of-curl P2/c^2.
 * Both operators are symmetric indefinite. */
int gym_op_create(gym_ctx* ctx, int problem, const gym_mesh* mesh, int degree,
                  gym_op** out);
int64_t gym_op_ndofs(const gym_op* op);
/* n[0], n[1] = sizes of the two unknown blocks. */
int gym_op_block_sizes(const gym_op* op, int64_t n[2]);
int gym_op_destroy(gym_op* op);
/* y = A x, nrhs vectors; precisions as for gym_mass_apply (incidence exact). */
int gym_op_apply(const gym_op* op, int prec, int nrhs, const void* x, void* y,
                 void* stream);
/* z = M^-1 y for the preconditioner `precond` of gym_solve (GYM_PRECOND_JACOBI
 * or GYM_PRECOND_SCHUR), nrhs FP64 device vectors.  Stream-ordered; the
 * Schur set-up on first use is blocking.  Errors: GYM_E_ARG,
 * GYM_E_UNSUPPORTED (SCHUR on a Hodge operator, a 2-D or a curved mesh). */
int gym_op_precond_apply(gym_op* op, int precond, int nrhs, const double* y,
                         double* z, void* stream);
/* Diagonal of the block-Jacobi preconditioner (FP64, op ndofs entries):
 * diag(M2 + D^T M3 D), diag(M3) for Poisson; diag(M0 + G^T M1 G),
 * diag(M1 + C^T M2 C) for Hodge. */
int gym_op_precond_diag(const gym_op* op, double* diag, void* stream);

/* Load vector of a manufactured field (FP64, op ndofs entries, device):
 * Poisson: b = [0; -F], F_i = int f Lambda^d_i with
 *   u = sum_m c_m prod_a sin(k_ma pi x_a), f = pi^2 |k_m|^2 u_m;
 * Hodge: b = [0; F], F_i = int f . Lambda^1_i with
 *   u_a = sum_m c_ma cos(k_ma pi x_a) prod_{b!=a} sin(k_mb pi x_b).
 * modes: HOST int array (nmodes x dim) of wave numbers; coeffs: HOST array
 * (nmodes x ncomp) with ncomp = 1 (Poisson) or 3 (Hodge).  Gauss rule with
 * r + 2 points per axis.  Synchronous. */
int gym_rhs_manufactured(const gym_op* op, int nmodes, const int* modes,
                         const double* coeffs, double* b, void* stream);

/* ---- solves ----------------------------------------------------------- */
typedef struct gym_solve_opts {
  int method;         /* GYM_MINRES (default) or GYM_CG                    */
  int mode;           /* GYM_MODE_F64 / _IR_F32 / _IR_BF16                 */
  double rtol;        /* stop when ||b - A x|| / ||b|| <= rtol (FP64)       */
  int maxit;          /* Krylov iterations (per inner solve under IR)      */
  double inner_rtol;  /* IR: inner relative residual target (e.g. 1e-4)    */
  int max_outer;      /* IR: outer refinement steps                        */
  int check_every;    /* host reads the device residual estimate every k   */
  int timing;         /* k > 0: bracket every k-th operator apply with HIP
                         events (1: every apply; a larger k keeps the
                         events' own cost out of the solve)                */
  int precond;        /* GYM_PRECOND_JACOBI (default), _NONE or _SCHUR     */
} gym_solve_opts;

typedef struct gym_solve_info {
  int status;          /* GYM_OK, GYM_W_NOT_CONVERGED or an error          */
  int iters;           /* total Krylov iterations (all inner solves)       */
  int outer_iters;     /* IR outer steps (0 in FP64 mode)                  */
  double rel_res;      /* ||b - A x|| / ||b|| in FP64 at exit, per rhs max */
  double seconds;      /* wall time of the call                            */
  int applies;         /* operator applies timed (opts.timing > 0)         */
  double apply_ms;     /* summed HIP-event time of those applies, ms       */
} gym_solve_info;

/* Fill `opts` with defaults: MINRES, FP64, rtol 1e-10, maxit 20000,
 * inner_rtol 1e-4, max_outer 30, check_every 25, timing 0, block Jacobi. */
void gym_solve_opts_default(gym_solve_opts* opts);

/* Solve A x = b for nrhs right-hand sides (device FP64 vectors, x is
 * overwritten; the initial guess is zero).  The Krylov workspace is
 * allocated on the first solve of an operator and kept until
 * gym_op_destroy.  Blocking: returns after the stream is synchronised.
 * Returns info->status. */
int gym_solve(gym_op* op, const gym_solve_opts* opts, int nrhs,
              const double* b, double* x, gym_solve_info* info, void* stream);

/* gym_solve without device allocation, for callers that cannot allocate
 * (HIP graph capture set-up, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments and results as gym_solve in GYM_MODE_F64 (the
 * same kernels in the same order, so x is the same bit for bit); its Krylov
 * workspace is a static device array of 128 MiB that each GPU the library
 * runs on holds until the process ends, instead of the operator's pool.
 * Limits: FP64 mode only (GYM_E_UNSUPPORTED otherwise), nrhs <= 64, and
 * about 11 x ndofs x nrhs doubles plus partial sums must fit the array
 * (roughly 1.4 M unknowns x rhs); larger problems return GYM_E_ARG with the
 * size in the message.  opts->timing is ignored.  Calls on one GPU share the
 * array: calls that overlap on one GPU race (serialise them).  Blocking, like
 * gym_solve. */
int gym_solve_noalloc(gym_op* op, const gym_solve_opts* opts, int nrhs,
                      const double* b, double* x, gym_solve_info* info,
                      void* stream);

/* Mass solve M x = b (CG, Jacobi preconditioner, FP64): the exact-FEEC
 * application of M_1^{-1} in the paper's eq. (exactEOM). */
int gym_mass_solve(const gym_space* space, const gym_solve_opts* opts,
                   int nrhs, const double* b, double* x, gym_solve_info* info,
                   void* stream);

/* ---- time stepping: generalized Yee methods (paper section 3) --------- */
/* The Maxwell system in the canonical pair (a, e), both in Lambda^1 with a
 * perfect-conductor boundary (tangential components zero: H0(curl)), units
 * eps0 = 1, mu0 = 1 / c^2.  Hamiltonian H = 1/2 e^T Q1 e + 1/2 a^T P2 a with
 * P2 = c^2 C^T M2~ C (eq. discTildeHamilSystem); shear maps
 * a <- a - tau Q1 e and e <- e + tau P2 a (eq. shearMaps) composed by Strang
 * splitting, half step in a, full step in e, half step in a (eq.
 * strangSplit).  Stable iff tau <= 2 / omega_max, omega_max^2 the largest
 * eigenvalue of Q1 P2 (Proposition Stability). */
#define GYM_Q1_EXACT  0  /* Q1 = M1^-1, applied by a CG mass solve           */
#define GYM_Q1_LUMPED 1  /* inverse row sums of M1 (section 4.3)            */
#define GYM_Q1_SPAI_DIAG 2 /* symmetrised SPAI of M1, diagonal pattern S(1)
                              (section 5; affine only)                       */
#define GYM_Q1_SPAI_OP 4 /* SPAI-OP (set by gym_maxwell_spai_op only)        */
#define GYM_Q1_SPAI   3  /* symmetrised SPAI of M1, pattern S(M1): columns
                            q_l = argmin ||M1[:, I_l] q - e_l||_2, then
                            (Q + Q^T)/2 (section 5; affine only)            */
#define GYM_M2_EXACT  0  /* M2~ = M2                                         */
#define GYM_M2_LUMPED 1  /* row sums of M2                                   */
/* Lumped row sums are those of the mass matrix without boundary conditions,
 * at the kept unknowns; with Whitney forms (degree 1) on a box, lumped Q1 and
 * M2~ give Yee's leapfrog (section 4). */
typedef struct gym_maxwell_opts {
  int q1;           /* GYM_Q1_*                                            */
  int m2;           /* GYM_M2_*                                            */
  double c;         /* wave speed (> 0)                                    */
  double cg_rtol;   /* exact Q1: relative residual of each M1 solve        */
  int cg_maxit;     /* exact Q1: CG iteration cap per solve                */
} gym_maxwell_opts;
/* Defaults: exact Q1 and M2~, c = 1, cg_rtol 1e-14, cg_maxit 1000. */
void gym_maxwell_opts_default(gym_maxwell_opts* opts);
/* The mesh is 3-D (tangential components zero on non-periodic faces: the
 * perfect conductor), or 2-D with both axes periodic (the torus: Lambda^2 is
 * then the scalar L2 space and C the 2-D curl).  On periodic meshes the
 * masses run as 1-D band passes.  Errors: GYM_E_ARG (other dimensions,
 * degree outside 1..4, bad option), GYM_E_UNSUPPORTED (a SPAI on a curved
 * mesh; lumped masses whose row sums are not all positive, which on curved
 * cells of degree >= 2 can happen), GYM_E_OOM.  On curved meshes the lumped
 * row sums are those of the curved mass matrix (one device apply). */
int gym_maxwell_create(gym_ctx* ctx, const gym_mesh* mesh, int degree,
                       const gym_maxwell_opts* opts, gym_maxwell** out);
/* SPAI-OP (section 5, eqs. SPAIOPobjective to diagonalPreconditioner): the
 * symmetric Q1 on the pattern of M1 minimising ||M1 Q1 - 1||_F^2 +
 * lambda sum_k ||(M1 Q1 - 1) P2 v_k||^2, from the generalized Sylvester
 * equations (U Q1 T + T Q1 U)_ij = (M1 T + T M1)_ij on the pattern, U = M1^2,
 * T = 1 + lambda W W^T, W = P2 V, solved matrix-free by Jacobi-preconditioned
 * CG from the symmetrised column-wise SPAI (Tikhonov shift 1e-12 max diag U).
 * probes: device array of nprobe x ndofs doubles, the modes v_k (nprobe may be
 * 0: the optimal symmetric SPAI).  On success the object's Q1 becomes this
 * SPAI-OP (GYM_Q1_SPAI_OP) for the time stepping, the energy and the
 * eigen-solver.  Affine meshes only; a periodic axis needs more than 4r
 * lattice positions (GYM_E_UNSUPPORTED otherwise).  Returns GYM_W_NOT_CONVERGED (Q1 is
 * still replaced) if maxit came before rtol; *iters and *rel_res may be NULL. */
int gym_maxwell_spai_op(gym_maxwell* mx, int nprobe, const double* probes, double lambda, double rtol,
                        int maxit, int* iters, double* rel_res, void* stream);
/* Unknowns of a and of e (each). */
int64_t gym_maxwell_ndofs(const gym_maxwell* mx);
/* nsteps Strang steps of length tau on device vectors a and e (ndofs
 * doubles each, updated in place).  Consecutive half steps in a are merged,
 * so a step costs one Q1 and one P2 application.  Synchronises the stream
 * when Q1 is exact (the CG solves read their convergence state).
 * Errors: GYM_E_ARG (tau <= 0, nsteps < 0), GYM_W_NOT_CONVERGED if an M1
 * solve missed cg_rtol (the step is still taken). */
int gym_maxwell_step(gym_maxwell* mx, double tau, int nsteps, double* a, double* e, void* stream);
/* *H = 1/2 e^T Q1 e + 1/2 a^T P2 a (host value; synchronises the stream). */
int gym_maxwell_energy(gym_maxwell* mx, const double* a, const double* e, double* H, void* stream);
int gym_maxwell_destroy(gym_maxwell* mx);

/* ---- eigenmodes of the time-stepping operator (paper section 3) -------
 * The lowest non-kernel eigenpairs of K~ = Q1 P2, i.e. of the generalized
 * problem P2 v = omega^2 Q1^-1 v with Q1^-1 = M1 (exact) or the row sums of
 * M1 (lumped) and P2 = c^2 C^T M2~ C.  The eigenvalues set the stability
 * bound tau <= 2 / omega_max (Proposition Stability) and the numerical
 * dispersion of the scheme (section 5).  P2 vanishes on gradients G Lambda^0;
 * the solver works on P2 + c^2 s Q1^-1 G D0^-1 G^T Q1^-1 instead (D0 the
 * diagonal of the Lambda^0 mass matrix M0), which lifts the gradients to
 * c^2 s times the eigenvalues of the Lambda^0 Laplacian G^T Q1^-1 G taken
 * against D0 and leaves every other eigenpair unchanged, s = grad_shift.
 * Method: LOBPCG
 * (Knyazev 2001) with block size `block`, preconditioned by the inverse row
 * sums of M1, from a seeded N(0,1) block. */
typedef struct gym_eig_opts {
  int nev;            /* eigenpairs wanted (1 <= nev <= block)                 */
  int largest;        /* 0: the lowest non-kernel pairs; 1: the largest ones
                         (omega_max: the step is stable iff tau <= 2/omega_max) */
  int block;          /* LOBPCG block size, <= 8; 0: min(nev + 2, 8)           */
  double tol;         /* stop when every wanted pair has
                         ||P2 v - omega^2 B v|| <= tol omega^2 ||B v||         */
  int maxit;          /* iteration cap                                        */
  double grad_shift;  /* s > 0; must lift the gradients above the wanted pairs */
  uint64_t seed;      /* initial block                                        */
} gym_eig_opts;
typedef struct gym_eig_info {
  int iters;          /* LOBPCG iterations                                    */
  int converged;      /* leading pairs that met tol                           */
  double max_resid;   /* largest relative residual over the wanted pairs      */
  int gradient_modes; /* wanted pairs found to be gradients (G^T B v != 0)    */
} gym_eig_info;
/* Defaults: nev 4, largest 0, block 0, tol 1e-8, maxit 3000, grad_shift 4, seed 1. */
void gym_eig_opts_default(gym_eig_opts* opts);
/* omega2: host array of nev values (ascending; descending when largest:
 * then the solver runs on -P2, without the gradient shift, which the
 * largest pairs never meet).  vecs: NULL or a device array
 * of nev x ndofs doubles receiving the Q1^-1-orthonormal eigenvectors, one
 * after another.  Allocates its work space (device, about 18 block vectors,
 * and 16 small pinned host slots for its uploads) per call and synchronises
 * the stream.  Returns GYM_W_NOT_CONVERGED if the
 * cap came first, or if a wanted pair is a gradient (grad_shift too small,
 * info->gradient_modes > 0); GYM_E_ARG for bad options; GYM_E_BREAKDOWN if
 * the search space lost rank (or a SPAI Q1 is not positive definite);
 * GYM_E_OOM.  A SPAI Q1 enters as B = Q1^-1 through CG solves with Q1. */
int gym_maxwell_eigs(gym_maxwell* mx, const gym_eig_opts* opts, double* omega2, double* vecs,
                     gym_eig_info* info, void* stream);

/* ---- serving: continuous batching of independent solves --------------- */
typedef struct gym_serve_opts {
  int device;            /* HIP device                                       */
  int64_t mem_budget;    /* bytes of device memory the server may hold       */
  int max_slots;         /* requests resident at once                        */
  double rtol;           /* per-request relative residual target             */
  int maxit;             /* per-request iteration cap                        */
  int precond;           /* GYM_PRECOND_JACOBI (0) or GYM_PRECOND_SCHUR; the
                            latter serves GYM_MIXED_POISSON requests only
                            (others are refused at submit) and is set up
                            once per operator                              */
} gym_serve_opts;

typedef struct gym_request {
  int problem;           /* GYM_MIXED_POISSON or GYM_HODGE1                  */
  int nel;               /* cubic mesh nel^3 on the unit cube                */
  int degree;            /* 1..3                                             */
  uint64_t seed;         /* right-hand side: N(0,1) on the second block,
                            zero on the first: SplitMix64 words
                            z_k = mix(seed + (k+1) 0x9E3779B97F4A7C15),
                            u = (z >> 11) 2^-53, Box-Muller on pairs        */
  const double* rhs;     /* optional HOST rhs (op ndofs); overrides seed;
                            copied at submit                                */
  int want_solution;     /* 1: keep x on the host until polled             */
} gym_request;

typedef struct gym_result {
  int status;            /* GYM_OK, GYM_W_NOT_CONVERGED, error; 2 = pending  */
  int iters;
  double rel_res;
  double latency_s;      /* submit -> result ready                           */
  int64_t ndofs;
} gym_result;

/* Start the serving loop on opts->device: a host thread that admits
 * requests while fewer than max_slots are active and their device memory
 * (vectors + operator) fits mem_budget, runs one batched MINRES step of all
 * active requests per turn, and retires converged ones (rel. residual <=
 * rtol, true FP64 residual) so that queued requests enter the mix.
 * mem_budget bytes are reserved on the device here, as the pool that holds
 * every request's vectors (GYM_E_OOM if they cannot be); operators are set
 * up outside the pool on first use of a (problem, nel, degree), count
 * against the same budget and stay resident; one that no active request
 * uses is freed only when an admission needs its room. */
int gym_serve_start(const gym_serve_opts* opts, gym_server** out);
/* Enqueue a request; returns its id.  Errors: GYM_E_OOM if one request
 * alone exceeds the memory budget. */
int gym_serve_submit(gym_server* srv, const gym_request* req, uint64_t* id);
/* Non-blocking.  If x_host is not NULL, the result is ready and the request
 * asked for its solution, the solution (op ndofs doubles) is copied there.
 * Returns 0 when the result is ready (the result is then released), 2 while
 * pending.  res->status carries the request's own status. */
int gym_serve_poll(gym_server* srv, uint64_t id, gym_result* res,
                   double* x_host);
/* Drain: wait for all submitted requests, then stop the loop. */
int gym_serve_stop(gym_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* GYM_H */
