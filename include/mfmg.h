/*
 * mfmg.h -- C ABI of the MI355X matrix-free octree multigrid PCG solver.
 *
 * The solver computes p with A p = rhs, where A is the volume-integrated
 * operator -div(beta grad .) on a 2:1-balanced adaptive octree with cut
 * cells (paper: "Matrix-Free Multigrid with Algebraically Consistent
 * Coarsening on Adaptive Octrees", Section 2.1 Eqs. (2)-(3), Section 3.1
 * Eqs. (5)-(10)), by preconditioned conjugate gradients (Algorithm 1) with
 * one FAS-style multigrid cycle (Algorithm 4, coarse operators from
 * Algorithm 3) as the preconditioner.
 *
 * Conventions shared by every call
 *   - Cells: a leaf is a cell (level l, i, j, k) of size h = 2^-l on the
 *     unit cube.  Leaves are grouped in 4x4x4 bricks (the refinement unit).
 *     Canonical leaf order is ascending Morton key of the cell's min corner
 *     on the 2^max_level grid (x in the least significant interleaved bit);
 *     equivalently bricks in Morton order, 64 cells per brick, cells in
 *     local Morton order.  Every leaf vector (rhs, p, lambda, dL/dp) is a
 *     contiguous array of n_leaves doubles in that order.
 *   - Directions 0..5 are -x, +x, -y, +y, -z, +z.
 *   - Faces: a face between leaves of different levels belongs to the finer
 *     leaf, between equal levels to the leaf on its + side, a wall face to
 *     its leaf.  Canonical face order is (owner leaf, direction).
 *   - "device" pointers are HIP device memory of the current device; "host"
 *     pointers are ordinary host memory.  The caller owns every buffer it
 *     passes; the library owns only the objects it returns, which the
 *     matching mfmg_destroy_* call frees.
 *   - stream is a hipStream_t (NULL = the default stream).  Every call
 *     enqueues its device work on that stream and returns after the work it
 *     needs has completed; statistics are valid on return.
 *   - Errors are reported by status code only; nothing throws across the
 *     ABI.  mfmg_last_error() returns a thread-local message for the last
 *     failing call of the calling thread.
 */
#ifndef MFMG_H
#define MFMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MFMG_OK = 0,
  MFMG_NOT_CONVERGED = 1,        /* warning: outputs hold the last iterate   */
  MFMG_ERR_INVALID_ARG = -1,     /* NULL pointer, size or range violation    */
  MFMG_ERR_TOPOLOGY = -2,        /* levels out of range, unbalanced input    */
  MFMG_ERR_HIP = -3,             /* a HIP runtime call failed                */
  MFMG_ERR_OOM = -4,             /* device or host allocation failed         */
  MFMG_ERR_BREAKDOWN = -5,       /* (p,Ap) <= 0, (r,z) <= 0 or non-finite    */
  MFMG_ERR_INCOMPATIBLE_RHS = -6 /* no Dirichlet face, null-space shift off */
                                 /* and 1^T rhs != 0 over the active cells  */
} mfmg_status;

typedef struct mfmg_octree mfmg_octree;
typedef struct mfmg_coeffs mfmg_coeffs;
typedef struct mfmg_hierarchy mfmg_hierarchy;

/* Thread-local message of the last failing call ("" if none). */
const char *mfmg_last_error(void);

/* ------------------------------------------------------------------ octree
 * Refinement predicates of the paper's grid generator (Section 4.1: a tile
 * meeting the surface takes the finest level), applied to 4^3-cell nodes:
 *   MFMG_SPHERE: the closed node box meets the shell
 *                radius - band <= |x - center| <= radius + band;
 *   MFMG_BOX:    the closed node box meets the boundary of the closed box
 *                [lo, hi].
 */
enum { MFMG_SPHERE = 0, MFMG_BOX = 1 };

typedef struct {
  int kind;         /* MFMG_SPHERE or MFMG_BOX                               */
  double center[3]; /* sphere centre                                         */
  double radius;    /* sphere radius                                         */
  double band;      /* half-width of the refinement shell (>= 0)             */
  double lo[3];     /* box corners                                           */
  double hi[3];
} mfmg_prim;

typedef struct {
  int min_level;  /* cell level of the initial uniform grid, >= 2            */
  int max_level;  /* finest cell level, min_level <= max_level <= 12         */
  int node_size;  /* cells per node edge; must be 4                          */
  int n_prims;    /* number of refinement primitives (>= 0)                  */
  const mfmg_prim *prims; /* host array of n_prims                           */
} mfmg_refine_spec;

/* Build the octree on the host (Section 3; 2:1 face balance).  For
 * l = min_level .. max_level-1 every leaf node of level l whose closed box
 * meets some primitive is split into 8; then coarse leaves are split to the
 * least fixed point where face-neighbouring leaves differ by at most one
 * level.  Host memory only; no device call.  *out receives a new object.
 * Errors: INVALID_ARG (NULL, node_size != 4, bad levels or primitive kind). */
mfmg_status mfmg_build_octree(const mfmg_refine_spec *spec, mfmg_octree **out);

/* The same octree (same leaves, faces and orders, bit for bit) built on the
 * device, for a tree that changes every time step (neighbour tables, then
 * re-assembly and Algorithm 3 coarsening on the device).  Refinement by the
 * predicates level by level, then the 2:1 balance as one pass from the
 * finest level down (each node needs the level l-1 node that contains its
 * face neighbour; a missing one is made by splitting its parent), over
 * dense per-level tables of 8^(l-2) bytes and 8^(l-2) int32 (so about
 * 4.4 GB of temporary device memory at max_level 12, 70 MB at 10), freed
 * before return.  Work is queued on stream; the call returns after the
 * stream has drained.  The octree holds device tables only: it serves
 * everything below, and its host leaves/faces are device outputs copied
 * back (null stream).
 * Errors: INVALID_ARG (as mfmg_build_octree), OOM, HIP, TOPOLOGY (an
 * internal invariant failed). */
mfmg_status mfmg_build_octree_device(const mfmg_refine_spec *spec, void *stream,
                                     mfmg_octree **out);

/* Sizes of the octree: leaf cells, faces, leaf bricks (any output may be
 * NULL).  Host only. */
mfmg_status mfmg_octree_info(const mfmg_octree *tree, int64_t *n_leaves,
                             int64_t *n_faces, int64_t *n_leaf_bricks);

/* Leaves in canonical order: level[n] and ijk[3n] (i, j, k at that level).
 * Host buffers of n_leaves and 3 n_leaves entries. */
mfmg_status mfmg_octree_leaves(const mfmg_octree *tree, uint8_t *level,
                               int32_t *ijk);

/* Faces in canonical order (host buffers of n_faces entries each):
 *   owner: owning leaf; dir: direction 0..5 from the owner;
 *   other: leaf across the face (same-level neighbour or coarser leaf) or
 *          -1 for a wall face;
 *   kind:  0 wall, 1 same level, 2 T-junction (owner finer than other). */
mfmg_status mfmg_octree_faces(const mfmg_octree *tree, int64_t *owner,
                              int8_t *dir, int64_t *other, int8_t *kind);

/* mfmg_octree_leaves and mfmg_octree_faces into device buffers of the same
 * sizes, written by kernels queued on stream (not waited for).  For a
 * host-built octree the first call (or the first assembly) uploads its
 * device tables, which the octree keeps. */
mfmg_status mfmg_octree_leaves_device(const mfmg_octree *tree, uint8_t *level,
                                      int32_t *ijk, void *stream);
mfmg_status mfmg_octree_faces_device(const mfmg_octree *tree, int64_t *owner,
                                     int8_t *dir, int64_t *other, int8_t *kind,
                                     void *stream);

void mfmg_destroy_octree(mfmg_octree *tree);

/* ------------------------------------------------------------ coefficients
 * Four coefficients per cell (Eq. 3) as magnitudes: the diagonal c and the
 * -x, -y, -z face coefficients, with face coefficient
 *   same level or T-junction (fine side): beta S / h,
 *   Dirichlet wall: beta S / (theta h), Neumann wall: 0,
 * S = h^2 the owner's face area and h its size; the coarse side of a
 * T-junction face carries the sum of its fine sub-face coefficients over 2
 * (Section 3.1).  A cell is a degree of freedom iff c != 0.
 */
enum { MFMG_NEUMANN = 0, MFMG_DIRICHLET = 1 };

typedef struct {
  int bc[6];      /* per domain wall (-x,+x,-y,+y,-z,+z): MFMG_NEUMANN or    */
                  /* MFMG_DIRICHLET (p = 0 outside)                           */
  double theta;   /* Dirichlet wall distance in cell sizes, (0, 1]; 0.5 puts */
                  /* p = 0 on the face, 1 is the paper's Dirichlet-cell rule  */
} mfmg_bc;

/* Assemble leaf coefficients on the device from per-face beta (device,
 * n_faces doubles in canonical face order, each >= 0).  Uploads the brick
 * topology on first use.  *out receives a new object that references tree
 * (tree must outlive it).  Errors: INVALID_ARG, HIP, OOM. */
mfmg_status mfmg_assemble_coeffs(const mfmg_octree *tree,
                                 const double *face_beta, const mfmg_bc *bc,
                                 void *stream, mfmg_coeffs **out);

/* Copy leaf coefficients to a device buffer of 4 n_leaves doubles laid out
 * as [c | kx | ky | kz], each in canonical leaf order. */
mfmg_status mfmg_coeffs_leaf(const mfmg_coeffs *coeffs, double *out,
                             void *stream);

void mfmg_destroy_coeffs(mfmg_coeffs *coeffs);

/* --------------------------------------------------------------- hierarchy
 * Multigrid levels max_level .. coarsest_level.  Inner-cell coefficients
 * come from Algorithm 3 (Section 2.5) with restriction scale alpha.
 * precision MFMG_FP64: the cycle runs in FP64.  MFMG_MIXED: the cycle runs
 * in FP32 with FP32 leaf coefficients and FP16 inner coefficients stored as
 * c / h_l (round to nearest even through FP32; a non-zero value below FP16's
 * normal range is stored as +-2^-14, so a sliver cut face keeps a positive
 * coupling and no active cell gets a zero diagonal); the outer PCG, its dot
 * products and the true residual stay FP64.  Every cycle kernel forms a
 * cell's diagonal as the sum of the six face coefficients it reads.
 */
enum { MFMG_FP64 = 0, MFMG_MIXED = 1 };

typedef struct {
  int nu_pre;         /* RBGS iterations before the coarse correction (2)    */
  int nu_post;        /* RBGS iterations after it (2)                         */
  int nu_coarse;      /* RBGS iterations on the coarsest level (10)           */
  int mu;             /* cycle index: 1 = V-cycle, 2 = W-cycle               */
  int coarsest_level; /* 2 <= coarsest_level <= min_level (3)                */
  double alpha;       /* restriction scale, R = P^T / alpha (2)              */
  double beta_mg;     /* coarse-correction factor applied at restriction (2) */
  int precision;      /* MFMG_FP64 or MFMG_MIXED                             */
} mfmg_mg_params;

/* Build the hierarchy for coeffs (which must outlive it).  The stencil
 * kernels use 32-bit buffer offsets: INVALID_ARG (nothing allocated) when
 * the FP64 leaf coefficients (read by the outer operator in both
 * precisions), the level coefficients of the chosen precision or the
 * plus-face table exceed 4 GiB, or an FP64 level vector reaches 2 GiB
 * (from 2^21 leaf bricks on; in FP64 from about 2^21 bricks in all). */
mfmg_status mfmg_build_hierarchy(const mfmg_coeffs *coeffs,
                                 const mfmg_mg_params *params, void *stream,
                                 mfmg_hierarchy **out);

/* Inner-cell coefficients of one level, FP64, to a device buffer of
 * 4 * 64 * n_bricks(level) doubles ([c|kx|ky|kz] per brick of 64 cells, in
 * the order returned by mfmg_hierarchy_level_bricks); leaf bricks of that
 * level hold their assembled coefficients. */
mfmg_status mfmg_hierarchy_level_coeffs(const mfmg_hierarchy *h, int level,
                                        double *out, void *stream);

/* Bricks of one level: count, and (if coords != NULL) host int32 triples of
 * brick coordinates (brick size 4 cells) and is_leaf flags (may be NULL). */
mfmg_status mfmg_hierarchy_level_bricks(const mfmg_hierarchy *h, int level,
                                        int64_t *count, int32_t *coords,
                                        uint8_t *is_leaf);

void mfmg_destroy_hierarchy(mfmg_hierarchy *h);

/* ------------------------------------------------------------------- solve */
typedef struct {
  double rtol;    /* stop when ||r_k||_2 <= rtol ||r_0||_2 (1e-10); see the  */
                  /* true-residual rule at mfmg_pcg_solve                     */
  int max_iter;   /* iteration cap (200)                                      */
  int null_space; /* -1 auto (on iff no Dirichlet wall), 0 off, 1 on: shift */
                  /* the residual to zero mean over active cells (Sec. 2.2)  */
  int warm_start; /* 1: p holds an initial guess x0 on input (Algorithm 1   */
                  /* from x0); the stop test becomes ||r_k|| <= rtol ||rhs||  */
                  /* (equal to ||r_0|| for the zero start).  Forward solves */
                  /* without the null-space shift only.  0: start from zero. */
} mfmg_solve_params;

typedef struct {
  int iters;              /* PCG iterations performed                        */
  int status;             /* mfmg_status of the solve                        */
  double rel_resid_recur; /* ||r_k|| / ||r_0|| of the recurrence             */
  double rel_resid_true;  /* ||rhs - A p|| / ||r_0|| recomputed in FP64      */
  double seconds;         /* device time of the solve (HIP events)           */
} mfmg_solve_stats;

/* Solve A p = rhs (Algorithm 1 from x0 = 0, or from p when warm_start).
 * rhs, p: device, n_leaves doubles
 * in canonical order; entries of inactive leaves are ignored on input and
 * set to 0 on output.  hist (host, may be NULL) receives max_iter + 1
 * relative residuals (the first iters + 1 are meaningful).
 * Stop rule (Algorithm 1's residual test, read with a true-residual check):
 * the iteration stops when the recursively updated residual meets rtol;
 * then the FP64 true residual ||rhs - A p|| is formed, and while it exceeds
 * rtol ||r_0|| and fewer than max_iter iterations were taken, the iteration
 * starts again from p with r = rhs - A p (same tolerance, the iteration
 * budget shared).  A restart that does not lower the true residual ends the
 * solve.  OK therefore means both residuals meet rtol.  In MFMG_MIXED the
 * cycle reads the residual multiplied by a power of two that brings its
 * mean square to [1, 4) (undone exactly in FP64), so the solve does not
 * depend on the scale of rhs within FP64's range.
 * Returns OK, NOT_CONVERGED (p holds the last iterate; the recursive or the
 * true residual is above rtol), BREAKDOWN, INCOMPATIBLE_RHS (null_space = 0
 * on a problem without Dirichlet faces and |sum of rhs| > 1e-10 sum of |rhs|
 * over the active cells: A is singular on the constants and the system has
 * no solution; nothing is solved), or an error. */
mfmg_status mfmg_pcg_solve(mfmg_hierarchy *h, const double *rhs, double *p,
                           const mfmg_solve_params *params, void *stream,
                           mfmg_solve_stats *stats, double *hist);

/* Adjoint of the solve: lambda with A^T lambda = dL_dp, preconditioned by
 * the exact transpose of the cycle (same stop rule and residual scaling as
 * mfmg_pcg_solve), then per face
 *   dL/dbeta_f = -lambda^T (dA/dbeta_f) p
 * (0 at Neumann walls and where a side of the face is inactive).
 * p, dL_dp, lambda: device, n_leaves; dL_dbeta: device, n_faces.
 * INCOMPATIBLE_RHS as for mfmg_pcg_solve, with dL_dp in place of rhs. */
mfmg_status mfmg_pcg_solve_adjoint(mfmg_hierarchy *h, const double *p,
                                   const double *dL_dp, double *lambda,
                                   double *dL_dbeta,
                                   const mfmg_solve_params *params,
                                   void *stream, mfmg_solve_stats *stats);

/* --------------------------------------------------------------- projection
 * The steps around a solve that project a face velocity field (Section
 * 2.1: the pressure equation's flux form; Section 4.4: the static
 * projection test; RMS_V of Section 4.2).  Velocities are MAC normal
 * components on the canonical faces, along the + axis of the face's axis;
 * a face's fluid area is beta_f h^2 (h of its owner, the finer side), with
 * the same beta as the assembly.  Device vectors; kernels are queued on
 * stream. */

/* div (n_leaves, canonical): the integrated divergence of face_u (the net
 * outflow sum_f s beta_f h^2 u_f of each leaf, s = +1 where the + axis
 * points out of it): the right-hand side that makes A p = div the
 * projection's pressure equation. */
mfmg_status mfmg_divergence(mfmg_hierarchy *h, const double *face_beta,
                            const double *face_u, double *div, void *stream);

/* face_u -= s_o F_f / (beta_f h^2) on every face with beta_f > 0, F_f the
 * pressure flux of the operator through the face (same level:
 * k (p_o - p_t); T-junction: k (mean of p over the fine owner's active
 * siblings - p_t) / 2; Dirichlet wall: k p_o; Neumann wall or an inactive
 * side: 0), so that div(u_new) = div(u) - A p: after a solve of A p = div(u)
 * the divergence left is the solve's residual.  The first call makes the
 * hierarchy's canonical face list (n_faces x 18 bytes), which it keeps. */
mfmg_status mfmg_project_velocity(mfmg_hierarchy *h, const double *face_beta,
                                  const double *p, double *face_u, void *stream);

/* *rms (host) = sqrt(sum V_i (div_i / V_i)^2 / sum V_i) over the active
 * leaves, V_i = h_i^3.  Returns after the stream has drained. */
mfmg_status mfmg_divergence_rms(mfmg_hierarchy *h, const double *div, double *rms,
                                void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight time-stepping loops, harnesses that forbid allocation):
 * mfmg_divergence_rms with its partial sums in a fixed array of the
 * library's (2 x 2048 doubles = 32 KiB per device, held until the process
 * ends) instead of the hierarchy's work buffers.  rms is a device pointer to
 * one double, written by the last kernel queued on stream; the call
 * allocates nothing, copies nothing and does not wait for the stream.  The
 * device current at the call must be the hierarchy's; the array's device
 * address is looked up on the first call on each device.  Every call on a
 * device shares that device's array, so calls that overlap on one device
 * (other streams, other threads) race.  Errors: INVALID_ARG (NULL argument,
 * or a reduction grid larger than the array, which the fixed grid of at
 * most 2048 workgroups never needs), HIP. */
mfmg_status mfmg_divergence_rms_noalloc(mfmg_hierarchy *h, const double *div, double *rms,
                                        void *stream);

/* ------------------------------------------------ component entry points
 * For parity tests of single steps.  Device vectors of n_leaves doubles. */

/* y = A x (transpose = 0) or y = A^T x (transpose = 1), composite leaf
 * operator with T-junction ghosts (Section 3.1). */
mfmg_status mfmg_apply_operator(mfmg_hierarchy *h, const double *x, double *y,
                                int transpose, void *stream);

/* z = M r (transpose = 0: one cycle of Algorithm 4 from zero) or
 * z = M^T r (transpose = 1); in the hierarchy's precision. */
mfmg_status mfmg_apply_precond(mfmg_hierarchy *h, const double *r, double *z,
                               int transpose, void *stream);

/* ------------------------------------------------------------ measurement
 * Average device time of one launch of a hot-path step, measured with HIP
 * events on `stream` over `reps` back-to-back launches, and the algorithmic
 * HBM bytes of one launch (each array the step must read or write counted
 * once; a half-sweep reads u and the three face coefficients of every cell
 * and the right-hand side and diagonal of the updated half, and writes the
 * updated half).
 *   what = MFMG_PROFILE_SMOOTH: one colour half-sweep of level `level`;
 *   what = MFMG_PROFILE_CYCLE:  one whole cycle (level ignored), its
 *          right-hand side being the current residual buffer;
 *   what = MFMG_PROFILE_COPY:   a plain streaming copy of 1 GiB between two
 *          buffers allocated for the measurement (16-byte accesses; bytes =
 *          read + write), the achievable HBM ceiling the other figures are
 *          compared with.
 * The work vectors of h are overwritten. */
enum { MFMG_PROFILE_SMOOTH = 0, MFMG_PROFILE_CYCLE = 1, MFMG_PROFILE_COPY = 2 };
mfmg_status mfmg_profile(mfmg_hierarchy *h, int what, int level, int reps,
                         void *stream, double *ms_per_launch,
                         double *bytes_per_launch);

#ifdef __cplusplus
}
#endif

#endif /* MFMG_H */
