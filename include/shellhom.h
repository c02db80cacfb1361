/*
 * shellhom.h -- C ABI of libshellhom: periodic voxel homogenization of a
 * charge-parametrized shellular unit cell on one AMD MI355X (gfx950) GPU.
 *
 * The path (Huang, Liu, Wang, "Shellular Metamaterial Design via Compact
 * Electric Potential Parametrization", arXiv 2511.04025):
 *   1. field      F and grad F of the truncated periodic charge series, Eq. (6),
 *                 at the n^3 voxel centers p_e = ((i+1/2)/n, (j+1/2)/n, (k+1/2)/n);
 *   2. threshold  d_e = |F - c| / ||grad F|| (Eq. (7)), beta_e = h(d_e) with the
 *                 hard step [d < t] or the logistic 1/(1+exp(-kappa (t - d)))
 *                 of Sec. 4.1, E_e = E_void + (E - E_void) beta_e;
 *   3. solve      the six periodic unit-strain cell problems K u^(k) = f^(k)
 *                 of Eq. (8) with a matrix-free 8-node-hex stiffness stencil
 *                 inside Jacobi-preconditioned CG;
 *   4. reduce     C^H_ij = (1/n^3) sum_e E_e (chi^i + u^i_e)^T K_0 (chi^j + u^j_e)
 *                 (energy form of Eq. (8)) and V = mean beta.
 *   The adjoint (Eq. (9)) gives dL/d(charge positions, charge values).
 *
 * Conventions shared by every entry point
 *   - Grids are x-fastest: voxel/node (i, j, k) has linear index (k n + j) n + i.
 *     Node (i, j, k) is the lower corner of voxel (i, j, k); the grid is periodic.
 *   - A 6-load-case nodal field is stored [case][component][k][j][i]
 *     (6 * 3 * n^3 values); load cases in Voigt order (11, 22, 33, 23, 13, 12)
 *     with engineering shear; displacements in units of the voxel edge.
 *   - C^H is returned as 36 doubles, row-major, same Voigt order.
 *   - Pointers prefixed d_ are device memory (hipMalloc'd or PyTorch CUDA
 *     tensors); all others are host memory, read during the call only.
 *   - `hip_stream` is a hipStream_t (may be NULL for the default stream).
 *     Calls are blocking: they return after the stream work is complete.
 *   - Every call returns 0 (SHH_OK) or a status below; negative codes leave
 *     outputs undefined.  No exception crosses the ABI.  The library never
 *     allocates device memory: the caller passes workspaces and arenas.
 */
#ifndef SHELLHOM_H
#define SHELLHOM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define SHH_OK                   0
#define SHH_NOT_CONVERGED        1   /* output valid; rel_res above rtol after max_iter */
#define SHH_INVALID_ARG         (-1) /* n < 2, N < 1, NaN/Inf input, nu outside (-1, 0.5),
                                        E <= 0, E_void outside [0, E], K outside [1, 6],
                                        kappa < 0, target_vf outside (0, 1), ...        */
#define SHH_WORKSPACE_TOO_SMALL (-2)
#define SHH_HIP_ERROR           (-3)
#define SHH_OVER_BUDGET         (-4) /* engine: request footprint exceeds the arena      */
#define SHH_UNSUPPORTED         (-5) /* e.g. gradient of the hard step (kappa = 0)       */
#define SHH_BREAKDOWN           (-6) /* CG breakdown: p^T K p <= 0 or NaN                */
#define SHH_NOT_FOUND           (-7) /* engine: unknown request id                       */
#define SHH_SCRATCH_TOO_SMALL   (-8) /* shh_homogenize_noalloc: the design's workspace
                                        exceeds SHH_NOALLOC_SCRATCH_BYTES                */

#define SHH_PREC_FP64  0  /* FP64 stencil, vectors, dots and reductions                 */
#define SHH_PREC_MIXED 1  /* FP32 stencil and CG vectors; FP64 dots, residual
                             recompute, solution accumulator and C^H reduction           */

#define SHH_SOLVER_JACOBI 0  /* CG with the Jacobi preconditioner                        */
#define SHH_SOLVER_MG     1  /* CG with a geometric multigrid V-cycle preconditioner     */
#define SHH_SOLVER_AUTO   2  /* per design: MG where the grid coarsens, else Jacobi      */
#define SHH_SOLVER_SELECTIVE 3 /* the selective solve of Sec. 4.2: voxels with beta <=
                                 1e-3 are culled (no stiffness floor: an active voxel
                                 carries E beta, E_void is ignored), unknowns only on
                                 the active nodes, held as compact lists in ascending
                                 packed-coordinate order; CG on them preconditioned by a
                                 multigrid V-cycle whose coarse levels are the Galerkin
                                 grids of the culled voxel operator where the grid
                                 coarsens (as for SHH_SOLVER_MG), else by Jacobi.  Any n.
                                 Served by the engine like the other solvers; shh_grad
                                 differentiates the culled model.  A load case whose
                                 true residual has not fallen by 1% over 50 residual
                                 recomputes stops with SHH_NOT_CONVERGED (the FP32
                                 floor of a mixed solve on a poorly conditioned
                                 culled design; SHH_PREC_FP64 reaches rtol there)        */
#define SHH_SOLVER_SELECTIVE_JACOBI 4 /* the same culled system, always Jacobi-preconditioned */

/* One design (Eq. (6)-(7) parameters and material). */
typedef struct {
  int32_t n;            /* voxels per axis, 2 <= n <= 512                               */
  int32_t num_charges;  /* N >= 1                                                        */
  const double *pos;    /* host [N][3] charge positions (any real; the field is
                           1-periodic)                                                   */
  const double *q;      /* host [N] charge values (the paper uses +-1, equal counts)     */
  int32_t K;            /* truncation order, 0 <= h, k, l <= K; the paper uses K = 3    */
  const double *alpha;  /* host [(K+1)^3] spectral weights alpha_hkl, index
                           (h (K+1) + k) (K+1) + l; NULL means all ones                 */
  double iso;           /* iso-level c of the surface F = c (the paper uses 0)           */
  double thickness;     /* shell half-thickness t in cell units; < 0: choose t so that
                           the volume fraction equals target_vf                         */
  double target_vf;     /* used when thickness < 0: hard step -> t is the midpoint of
                           the k-th and (k+1)-th smallest d, k = round(vf n^3);
                           logistic -> bisection until |V - vf| <= 1e-12                */
  double kappa;         /* 0: hard step beta = [d < t];  > 0: logistic sharpness         */
  int32_t dist_mode;    /* 0: d = |F - c| / ||grad F|| (Eq. (7));  1: d = |F - c|       */
  double E;             /* solid Young's modulus, > 0                                    */
  double nu;            /* Poisson ratio, -1 < nu < 0.5                                  */
  double E_void;        /* void stiffness floor, 0 <= E_void <= E (0 makes K singular
                           beyond the rigid modes if the solid is not connected)         */
  int32_t symmetry;     /* fundamental bounding volume (Sec. 3.2): the N charges are
                           given in it and mirrored over the cell before anything else:
                           SHH_SYM_NONE as given; SHH_SYM_MIRROR the eight reflections
                           x_d -> 1 - x_d (a one-eighth-cell volume: orthotropic
                           structures); SHH_SYM_CUBIC those with the six axis
                           permutations, 48 images (a tetrahedral volume: cubic
                           structures).  Images keep the charge value; coincident
                           images are not merged.  Gradients are with respect to the
                           N given charges.  N times the image count <= 4096.         */
} shh_design;

#define SHH_SYM_NONE   0
#define SHH_SYM_MIRROR 1
#define SHH_SYM_CUBIC  2

/* Solver options. */
typedef struct {
  int32_t precision;        /* SHH_PREC_FP64 or SHH_PREC_MIXED                            */
  double rtol;              /* stop a load case when ||f - K u||_2 <= rtol ||f||_2        */
  int32_t max_iter;         /* CG iteration cap per load case                            */
  int32_t recompute_every;  /* R: replace the recursive residual by f - K u, computed in
                               FP64, every R iterations (0: default 50 mixed -- 10 for
                               SHH_SOLVER_SELECTIVE -- / 0 FP64; the true residual is
                               always recomputed at the end)                             */
  int32_t save_for_backward;/* keep F, grad F and the solution for shh_grad               */
  int32_t check_every;      /* host polls convergence every this many iterations (0: 16) */
  int32_t solver;           /* SHH_SOLVER_JACOBI (0): Jacobi-preconditioned CG, one fused
                               pass per iteration; SHH_SOLVER_MG (1): CG preconditioned by
                               a geometric multigrid V-cycle (Sec. 4.2's solver family:
                               Galerkin coarse grids, Chebyshev smoothing), for n = m 2^k
                               with k >= 1, m <= 8 and n >= 6 (SHH_UNSUPPORTED otherwise) */
} shh_opts;

/* Result of one homogenization. */
typedef struct {
  double CH[36];        /* homogenized tensor, row-major Voigt                            */
  double vol_frac;      /* V = mean beta                                                  */
  double t_used;        /* half-thickness used                                            */
  int32_t iters[6];     /* CG iterations per load case                                    */
  double rel_res[6];    /* final true relative residual per load case (FP64)             */
  double ms[5];         /* wall time: field+threshold, rhs, solve, C^H, total            */
  int32_t status;       /* SHH_OK, SHH_NOT_CONVERGED or a negative code                  */
  int32_t active_nodes; /* nodes carrying unknowns: n^3, or the active nodes of the
                           selective solve                                               */
} shh_result;

/* Library version (major * 10000 + minor * 100 + patch). */
int32_t shh_version(void);

/* Human-readable text of a status code (static storage). */
const char *shh_strerror(int32_t code);

/* Device workspace bytes that shh_homogenize needs for this design and these
   options.  Validates the arguments (returns SHH_INVALID_ARG if invalid). */
int32_t shh_workspace_bytes(const shh_design *design, const shh_opts *opts, size_t *bytes);

/* The whole path for one design: field -> threshold -> six-case PCG -> C^H.
   d_ws: caller-owned device workspace of at least shh_workspace_bytes bytes,
   256-byte aligned; it must stay allocated until shh_grad if save_for_backward.
   Returns SHH_OK, SHH_NOT_CONVERGED, or an error. */
int32_t shh_homogenize(const shh_design *design, const shh_opts *opts,
                       void *d_ws, size_t ws_bytes, void *hip_stream, shh_result *out);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): the path of
   shh_homogenize with the library's own fixed workspace, a device array of
   SHH_NOALLOC_SCRATCH_BYTES bytes that each GPU the library runs on holds
   until the process ends (its address is resolved on the first call on a
   device).  The call allocates nothing and creates no HIP events, so
   out->ms[] is zero.  Designs whose shh_workspace_bytes exceeds the scratch
   return SHH_SCRATCH_TOO_SMALL before any work.  Every call on one GPU
   shares that GPU's array and overwrites what the previous call left there
   (the call initializes every part it reads): calls that overlap on one GPU
   -- two host threads, or two streams -- race and must be serialized by the
   caller.  save_for_backward is accepted, but a later call overwrites the
   saved state; shh_grad needs a caller-owned workspace.  Results equal
   shh_homogenize's for the same design and options. */
#define SHH_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
int32_t shh_homogenize_noalloc(const shh_design *design, const shh_opts *opts, void *hip_stream,
                               shh_result *out);

/* The same path for `count` designs at once: every phase is one batched launch
   over all designs (different n and charge counts allowed).  d_ws[i] and
   ws_bytes[i] are per-design workspaces as for shh_homogenize; out[i] receives
   design i's result.  Returns the first negative status, else SHH_NOT_CONVERGED
   if any design did not converge, else SHH_OK. */
int32_t shh_homogenize_batch(const shh_design *designs, int32_t count, const shh_opts *opts,
                             void *const *d_ws, const size_t *ws_bytes, void *hip_stream,
                             shh_result *out);

/* Steps 3-4 only, for a given voxel stiffness field: d_E is a device array of
   n^3 doubles (the E_e of Eq. (7), > 0 somewhere).  Workspace size from
   shh_workspace_bytes_stiffness.  out->vol_frac is mean(E)/max(E). */
int32_t shh_workspace_bytes_stiffness(int32_t n, const shh_opts *opts, size_t *bytes);
int32_t shh_homogenize_stiffness(int32_t n, const double *d_E, double nu, const shh_opts *opts,
                                 void *d_ws, size_t ws_bytes, void *hip_stream, shh_result *out);

/* Steps 3-4 for a voxel modulus grid in one of three encodings (e_dtype):
     SHH_EDTYPE_U8   one byte per voxel, a solid/void code: E_e = E where the
                     byte is nonzero, E_void where it is zero (the hard
                     threshold of Eq. (7) in its most compact form; requires
                     E > 0, 0 <= E_void <= E); out->vol_frac = share of solid
                     voxels;
     SHH_EDTYPE_F32  n^3 floats (the moduli rounded to FP32 on entry, e.g. a
                     mixed-precision caller's own grid);
     SHH_EDTYPE_F64  n^3 doubles (the same as shh_homogenize_stiffness).
   For F32/F64, E and E_void are ignored and out->vol_frac is mean(E)/max(E).
   With SHH_SOLVER_SELECTIVE a zero modulus culls the voxel (the U8 code's
   zeros are culled, E_void ignored) and an all-zero grid gives C^H = 0.
   d_E: device array [n][n][n] (x fastest), caller-owned, read only.  Workspace
   from shh_workspace_bytes_stiffness.  SHH_INVALID_ARG for an unknown
   e_dtype, a grid with no positive modulus, or the conditions above. */
#define SHH_EDTYPE_U8  0
#define SHH_EDTYPE_F32 1
#define SHH_EDTYPE_F64 2
int32_t shh_homogenize_field(int32_t n, const void *d_E, int32_t e_dtype, double E, double E_void, double nu,
                             const shh_opts *opts, void *d_ws, size_t ws_bytes, void *hip_stream,
                             shh_result *out);

/* Steps 1-2 only (Eq. (6)-(7)).  Writes the device arrays d_F [n^3],
   d_G [3][n^3] (dF/dx, dF/dy, dF/dz), d_d [n^3] (distance) and d_beta [n^3]
   (occupancy), all doubles; any of them may be NULL.  out->vol_frac and
   out->t_used are set.  Uses the shh_homogenize workspace. */
int32_t shh_field(const shh_design *design, void *d_ws, size_t ws_bytes, double *d_F,
                  double *d_G, double *d_d, double *d_beta, void *hip_stream, shh_result *out);

/* The field F of Eq. (6) (iso-level not subtracted) and its gradient at
   npts arbitrary points, for fitting the charge field to a given surface
   (the objective of Eq. (10)): d_pts device [npts][3] (cell units, any real:
   F is 1-periodic), d_F device [npts], d_G device [3][npts] or NULL.  Only the
   design's charges, alpha, K and symmetry are used.  d_ws: device workspace of
   shh_workspace_bytes_points bytes.  FP64; synchronizes the stream. */
int32_t shh_workspace_bytes_points(const shh_design *design, int32_t npts, size_t *bytes);
int32_t shh_field_points(const shh_design *design, int32_t npts, const double *d_pts, double *d_F, double *d_G,
                         void *d_ws, size_t ws_bytes, void *hip_stream);
/* Adjoint of a functional of those values: given dL/dF at the points
   (device [npts]), writes dL/dpos [N][3], dL/dq [N] (host) and, if not NULL,
   dL/dalpha [(K+1)^3] (host), with respect to the design's own charges (the
   fundamental volume's, under a symmetry mode). */
int32_t shh_field_points_grad(const shh_design *design, int32_t npts, const double *d_pts, const double *d_dL_dF,
                              double *dL_dpos, double *dL_dq, double *dL_dalpha, void *d_ws, size_t ws_bytes,
                              void *hip_stream);

/* Workspace of the operator calls below (shh_apply_stiffness,
   shh_load_vectors, shh_energy): the moduli in the working precision, the
   Jacobi diagonal, reduction partials and descriptors, about 16 B per node
   (the callers' vectors are not part of it).  2 <= n <= 512;
   precision SHH_PREC_FP64 or SHH_PREC_MIXED; SHH_INVALID_ARG otherwise.  A
   shh_workspace_bytes_stiffness workspace of the same precision is larger and
   serves as well. */
int32_t shh_workspace_bytes_operator(int32_t n, int32_t precision, size_t *bytes);

/* The matrix-free periodic stiffness operator: d_q = K d_p for `nrhs` nodal
   vector fields [nrhs][3][n^3], K = sum_e E_e P_e^T K_0 P_e (Sec. 4.1, K_0 the
   unit-voxel 8-node-hex matrix at E = 1 and Poisson ratio nu).  precision
   SHH_PREC_FP64: d_p, d_q are doubles; SHH_PREC_MIXED: floats (E rounded to
   float).  d_E: device n^3 doubles.  d_ws: device scratch of at least
   shh_workspace_bytes_operator(n, precision) bytes (SHH_INVALID_ARG /
   SHH_WORKSPACE_TOO_SMALL otherwise).  Synchronizes the stream before
   returning. */
int32_t shh_apply_stiffness(int32_t n, int32_t precision, const double *d_E, double nu,
                            int32_t nrhs, const void *d_p, void *d_q, void *d_ws, size_t ws_bytes,
                            void *hip_stream);

/* The Galerkin coarse operator of level `level` (1 <= level < number of
   levels; level l halves each axis l times) of the multigrid solver's
   hierarchy for the moduli d_E (device n^3 doubles) at Poisson ratio nu:
   d_q = A_l d_v with A_l = P_l^T ... P_1^T K P_1 ... P_l, P trilinear periodic
   prolongation (Sec. 4.2's coarse grids).  d_v, d_q: device [6][3][(n/2^l)^3]
   in the precision's type (doubles for SHH_PREC_FP64, floats for MIXED).
   d_ws: at least shh_workspace_bytes_stiffness(n, opts) bytes for opts with
   this precision and solver = SHH_SOLVER_MG.  SHH_UNSUPPORTED for grids the
   hierarchy cannot coarsen, SHH_INVALID_ARG for other levels.  Builds the
   hierarchy, so it costs a solver setup; synchronizes the stream. */
int32_t shh_mg_operator(int32_t n, int32_t precision, const double *d_E, double nu, int32_t level,
                        const void *d_v, void *d_q, void *d_ws, size_t ws_bytes, void *hip_stream);

/* Right-hand sides f^(k) = -sum_e E_e P_e^T K_0 chi^k of the six load cases
   (Eq. (8)) in FP64: d_f [6][3][n^3].  d_ws as for shh_apply_stiffness with
   precision SHH_PREC_FP64. */
int32_t shh_load_vectors(int32_t n, const double *d_E, double nu, double *d_f, void *d_ws,
                         size_t ws_bytes, void *hip_stream);

/* Energy form of Eq. (8) for given displacements d_u [6][3][n^3] (doubles):
   CH[36] = (1/n^3) sum_e E_e (chi^i + u^i_e)^T K_0 (chi^j + u^j_e).
   d_ws as for shh_load_vectors. */
int32_t shh_energy(int32_t n, const double *d_E, double nu, const double *d_u, double CH[36],
                   void *d_ws, size_t ws_bytes, void *hip_stream);

/* Adjoint of Eq. (9) for the forward run that used d_ws (which must have had
   save_for_backward = 1 and kappa > 0): given dL/dC^H (36 doubles, row-major)
   and dL/dV, writes the gradient with respect to every design parameter that
   Sec. 4.3 lists, theta in {charge positions, charge values, alpha_hkl, t}:
     dL_dpos   [N][3]        host, required
     dL_dq     [N]           host, required
     dL_dalpha [(K+1)^3]     host or NULL; index (h (K+1) + k) (K+1) + l as for
                             alpha; entry (0,0,0) is 0 (B_000 = 0)
     dL_dt     [1]           host or NULL; t as an independent parameter (for a
                             volume constraint combine it with the gradient of
                             V: call again with dL/dC = 0, dL/dV = 1)
   The forward's own t (given or chosen from target_vf) is the point of
   evaluation.  The workspace's vectors are overwritten (scratch); F, grad F,
   beta and u survive, so several calls may follow one forward.  After a
   selective solve the gradient is that of the culled model: E_e = E beta_e
   on an active voxel (dE_e/dbeta_e = E), nothing on a culled one (a voxel
   crossing beta = 1e-3 is not differentiated).
   Returns SHH_UNSUPPORTED for the hard step. */
int32_t shh_grad(const shh_design *design, const shh_opts *opts, void *d_ws, size_t ws_bytes,
                 const double dL_dCH[36], double dL_dV, double *dL_dpos, double *dL_dq, double *dL_dalpha,
                 double *dL_dt, void *hip_stream);

/* Batched adjoint over the designs of one shh_homogenize_batch call, with one
   synchronization for all of them.  dL_dCH: [count][36]; dL_dV: [count];
   dL_dpos, dL_dq, dL_dalpha: per-design host arrays laid out back to back
   ([sum N_i][3], [sum N_i], [sum (K_i+1)^3]); dL_dt: [count].  dL_dalpha and
   dL_dt may be NULL. */
int32_t shh_grad_batch(const shh_design *designs, int32_t count, const shh_opts *opts,
                       void *const *d_ws, const size_t *ws_bytes, const double *dL_dCH,
                       const double *dL_dV, double *dL_dpos, double *dL_dq, double *dL_dalpha,
                       double *dL_dt, void *hip_stream);

/* ---- instrumentation ------------------------------------------------------
   When enabled, every launch of the solver's main kernel families is
   bracketed by two HIP events on the stream it runs on, and the elapsed time
   is accumulated per family, process-wide, when the solver next
   synchronizes (profiling state is the library's only process-wide mutable
   state besides a small cache of constants per Poisson ratio; neither holds
   design data).  Families: */
#define SHH_PROF_CG_PASS      0  /* Jacobi-PCG: the fused pass, q = K p with the vector updates */
#define SHH_PROF_MG_DIR       1  /* multigrid CG, voxel level: p = z + beta p, q = K p, p.q     */
#define SHH_PROF_MG_STEP1     2  /*   operator fused with the first pre-smoothing sweep         */
#define SHH_PROF_MG_RES       3  /*   r - K d1 (the residual the restriction takes)            */
#define SHH_PROF_MG_POST      4  /*   operator fused with the first post-smoothing sweep        */
#define SHH_PROF_MG_LAST      5  /*   operator fused with the last sweep and the r.z partials   */
#define SHH_PROF_MG_UPDATE    6  /*   CG update x += alpha p, r -= alpha q                     */
#define SHH_PROF_MG_RESTRICT  7  /*   restriction to the first coarse level                    */
#define SHH_PROF_MG_PROLONG   8  /*   prolongation from the first coarse level                 */
#define SHH_PROF_MG_APPLY1    9  /* multigrid, first coarse level: q = A_1 v (27-point blocks)  */
#define SHH_PROF_RESID64     10  /* FP64 residual f - K u (replacement and final check)         */
#define SHH_PROF_SEL_OP      11  /* selective solve: q = K p on the active nodes, with the sums  */
#define SHH_PROF_SEL_UPDATE  12  /*   x += alpha p, r -= alpha q, p = D^-1 r + beta p            */
#define SHH_PROF_SEL_RESID   13  /*   FP64 residual f - K u on the active nodes                  */
#define SHH_PROF_SEL_MG_PQ   14  /* selective multigrid CG: q = K p on the active nodes, p.q     */
#define SHH_PROF_SEL_MG_SMOOTH 15 /*  the four operator passes fused with the Chebyshev sweeps  */
#define SHH_PROF_SEL_MG_VEC  16  /*   x += alpha p, r -= alpha q with D^-1 r; p = z + beta p     */
#define SHH_PROF_SEL_MG_TRANSFER 17 /* restriction to and prolongation from the first coarse level */
#define SHH_PROF_NKIND       18
/* shh_profile_enable(1) also resets the counters.  shh_profile_read gives the
   number of timed launches of one family and their total milliseconds
   (SHH_INVALID_ARG for an unknown family). */
int32_t shh_profile_enable(int32_t on);
int32_t shh_profile_read(int32_t kind, int64_t *launches, double *ms_total);

/* Reference stream for the measurements: copies `bytes` (a multiple of 16,
   both pointers 16-byte aligned) from d_src to d_dst with 16-byte vector
   loads and stores, enqueued on hip_stream (asynchronous, unlike the calls
   above).  Its duration is the read+write rate the GPU sustains, and its
   hardware traffic counters calibrate those of the solver kernels. */
int32_t shh_stream_copy(const void *d_src, void *d_dst, size_t bytes, void *hip_stream);

/* ---- serving engine: continuous batching ------------------------------
   Requests are admitted into slots while a free slot and enough arena memory
   exist (first fit), run together -- every CG phase is one launch over all
   resident designs (one per solver group: dense and selective designs are
   stepped as two batches) -- and leave when their six load cases have
   converged.  A design's result does not depend on what else is resident.
   Admission happens at iteration boundaries inside shh_engine_step.
   d_arena: caller-owned device memory (e.g. a PyTorch uint8 tensor) of
   arena_bytes bytes, the engine's whole HBM budget; it must outlive the engine.
   Designs and options are copied at submit.  Not thread-safe: one host thread
   per engine. */
typedef struct shh_engine shh_engine;

int32_t shh_engine_create(void *d_arena, size_t arena_bytes, int32_t max_slots, void *hip_stream,
                          shh_engine **out);
/* Footprint (arena bytes) a design would take; SHH_OVER_BUDGET from submit if
   it exceeds the whole arena. */
int32_t shh_engine_footprint(const shh_design *design, const shh_opts *opts, size_t *bytes);
int32_t shh_engine_submit(shh_engine *eng, const shh_design *design, const shh_opts *opts,
                          uint64_t request_id);
/* Admit what fits, then run `iters` CG iterations of every resident design,
   retire the converged ones.  *n_resident / *n_queued receive the counts after
   the step (either may be NULL). */
int32_t shh_engine_step(shh_engine *eng, int32_t iters, int32_t *n_resident, int32_t *n_queued);
/* Move up to `max` finished results out: out[i] and ids[i]. */
int32_t shh_engine_poll(shh_engine *eng, shh_result *out, uint64_t *ids, int32_t max,
                        int32_t *n_out);
/* Remove a queued or resident request (its result is dropped). */
int32_t shh_engine_cancel(shh_engine *eng, uint64_t request_id);
void shh_engine_destroy(shh_engine *eng);

#ifdef __cplusplus
}
#endif

#endif /* SHELLHOM_H */
