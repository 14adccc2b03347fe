/*
 * elas3d.h - C-ABI of the MI355X periodic voxel elasticity solver.
 *
 * The library solves the equilibrium problem of ELAS3D-Xtal (arXiv
 * 2602.07354, Sec. 2.1): a periodic grid of nx*ny*nz voxels, each voxel a
 * trilinear 8-node hexahedron with 3 displacement dofs per node, carrying
 * the 6x6 stiffness of its phase (grain or pore).  Under an applied
 * macroscopic strain E the displacement is u = E.X + w, and w minimises the
 * quadratic energy of Eq. (quadratic_form), i.e. solves A w + b = 0
 * (Sec. 2.1.2).  The solve is the matrix-free point-block Jacobi PCG of
 * Algorithm 2, run entirely by hand-written gfx950 HIP kernels.
 *
 * Conventions (all entry points):
 *   - Grid: voxel / node (i,j,k) is flattened as m = i + nx*(j + ny*k),
 *     x fastest (Eq. pbc_indices, 0-based).  Node m sits at the lower corner
 *     of voxel m; voxel m has the nodes ((i+a)%nx, (j+b)%ny, (k+c)%nz),
 *     a,b,c in {0,1}.  Voxel size is 1, so displacements are in voxel units
 *     and stresses in the units of C.
 *   - Stiffness C: per phase a row-major 6x6 Voigt matrix in the order
 *     (11,22,33,23,13,12) mapping engineering strain to stress (Sec. 2.1.1,
 *     Eq. (2)-(3) and Eq. (anisotropic_rotation)).  It must be symmetric and
 *     finite.  A phase whose 36 entries are all zero is a void (pore).
 *   - Strain: tensor components (E11,E22,E33,E23,E13,E12) (Eq. affine_strain).
 *   - Node vectors (displacement, load, operator input/output): SoA, three
 *     planes of N doubles, component c of node m at [c*N + m].
 *   - Voxel stress: six planes of N doubles, Voigt order, [r*N + m].
 *
 * Ownership: setup copies every input, so callers may free or reuse their
 * arrays on return.  Outputs go to caller-allocated buffers (host memory,
 * or device memory when elas3d_options.outputs_on_device is set).  The
 * library owns all device memory of a context and releases it in
 * elas3d_destroy.  A context is not thread-safe; distinct contexts are
 * independent.
 *
 * Errors: 0 = success.  Positive values are soft results whose outputs are
 * still valid (ELAS3D_NOT_CONVERGED, ELAS3D_BREAKDOWN).  Negative values are
 * hard errors with no outputs written; elas3d_last_error gives a message.
 * Argument validation runs before any device call.
 */
#ifndef ELAS3D_H
#define ELAS3D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ELAS3D_OK 0
#define ELAS3D_NOT_CONVERGED 1  /* maxit reached before the tolerance       */
#define ELAS3D_BREAKDOWN 2      /* h.Ah <= 0 or not finite (Algorithm 2, B) */
#define ELAS3D_EBADARG (-1)     /* invalid argument, nothing done           */
#define ELAS3D_ENOMEM (-2)      /* device memory budget exceeded            */
#define ELAS3D_EDEVICE (-3)     /* HIP runtime error                        */
#define ELAS3D_EORDER (-4)      /* call out of order (e.g. stress before solve) */

#define ELAS3D_MAX_RHS 6

/* elas3d_options.precision */
#define ELAS3D_PREC_FP64 0  /* every vector and reduction in FP64 (the paper's, Sec. 2.1.2) */
#define ELAS3D_PREC_MIXED 1 /* FP32 inner PCG inside FP64 iterative refinement            */

/* elas3d_options.convergence */
#define ELAS3D_CONV_RESIDUAL 0 /* stop on ||g||/||b|| <= tol, confirmed by the true residual */
#define ELAS3D_CONV_PAPER 1    /* stop on sqrt(z.g / z0.g0) < tol (Algorithm 2, D)           */

/* elas3d_options.preconditioner */
#define ELAS3D_PRECOND_BLOCK_JACOBI 0 /* 3x3 point-block Jacobi, Eq. (block_precond) */
#define ELAS3D_PRECOND_NONE 1         /* plain CG (M^-1 = I on active nodes)          */

typedef struct elas3d_ctx elas3d_ctx;
typedef struct elas3d_group elas3d_group;

typedef struct elas3d_options {
    int32_t precision;         /* ELAS3D_PREC_*                                      */
    int32_t convergence;       /* ELAS3D_CONV_*                                      */
    int32_t preconditioner;    /* ELAS3D_PRECOND_*                                   */
    int32_t inputs_on_device;  /* nonzero: `phase` of elas3d_setup is a device pointer */
    int32_t outputs_on_device; /* nonzero: output/input vectors of stress, apply,
                                  get_* are device pointers                          */
    int32_t poll_interval;     /* iterations between host checks of the stop flag;
                                  0 = automatic                                      */
    int32_t timing;            /* nonzero: time each fused-operator and update
                                  launch with HIP events (reported in elas3d_info)   */
    int32_t device;            /* HIP device ordinal, -1 = current device            */
    double hbm_budget_bytes;   /* device bytes the context may allocate; 0 = 95 %
                                  of the device's free memory at setup               */
    void* stream;              /* hipStream_t to run on; NULL = a library stream     */
    double inner_tol;          /* mixed: relative residual reduction per refinement
                                  cycle of the FP32 inner PCG (0 = 1e-4)             */
    int32_t inner_maxit;       /* mixed: iteration cap of one inner solve (0 = auto) */
    int32_t batched;           /* nonzero: solve all requested RHS in one multi-RHS
                                  launch sequence sharing the operator               */
    int32_t graphs;            /* nonzero: replay each batch of poll_interval
                                  iterations as a captured HIP graph (ignored
                                  when timing is on); default 1                      */
    int32_t autotune;          /* nonzero: before the first iteration of each
                                  precision, time the candidate workgroup shapes
                                  (options.tile's list; 5, and 6 for the FP32
                                  sweep, where the grid and its phases allow)
                                  and z-chunkings
                                  (about 2048 to 16384 workgroups) of the
                                  direction+operator sweep and
                                  the grid (1024 to 32768 workgroups) and the
                                  plain or non-temporal form of the update sweep
                                  on the live problem,
                                  keep the fastest (cached per process by grid,
                                  precision and RHS count).  The reduction order
                                  then follows the chosen geometry, so results match
                                  the default geometry's to rounding, not bitwise.
                                  2: time the update sweep's candidates only; the
                                  direction+operator sweep keeps options.tile and
                                  zchunk.  Default 0                                 */
    int32_t tile;              /* workgroup shape of the direction+operator sweep
                                  when not autotuned: 0 = 32x8 lanes (default),
                                  1 = 16x16, 2 = 64x4, 3 = 32x16, 4 = 64x8;
                                  5 = 64x6 + two loader wavefronts (the node
                                  planes stream into an LDS ring by direct-to-
                                  LDS loads; nx must be a multiple of 2, of 4
                                  in mixed precision, nx*ny < 2^27, and no
                                  workgroup box may hold more than 96
                                  distinct phases, else EBADARG; setup builds
                                  a phase dictionary per workgroup, about
                                  1.3 bytes per voxel); 6 = 64x8 + two loader
                                  wavefronts, the same for the FP32 sweep of
                                  mixed precision only (EBADARG in FP64; the
                                  FP64 sweeps of that context take 64x8)     */
    int32_t zchunk;            /* z planes per workgroup of that sweep when not
                                  autotuned; 0 = automatic (about 4096 workgroups);
                                  values above nz mean nz                            */
    int32_t update_blocks;     /* workgroups of the update sweep when not
                                  autotuned: 0 = automatic (1024 on grids of at
                                  most 2^21 nodes, else 4096), else 1..32768 (at
                                  most one per 256 nodes)                            */
    int32_t update_nontemporal; /* 1: the update sweep streams its node vectors
                                  non-temporally when not autotuned; 0 (default)
                                  plain loads and stores.  Same results bitwise     */
} elas3d_options;

typedef struct elas3d_info {
    int32_t nrhs;                              /* RHS solved by the call             */
    int32_t status[ELAS3D_MAX_RHS];            /* per RHS: 0, 1 or 2 (see above)    */
    int32_t iters[ELAS3D_MAX_RHS];             /* PCG iterations (inner ones in mixed) */
    int32_t restarts[ELAS3D_MAX_RHS];          /* residual-confirmation restarts /
                                                  refinement cycles (mixed)          */
    double relres_true[ELAS3D_MAX_RHS];        /* ||A w + b||_2 / ||b||_2, recomputed */
    double relres_recursive[ELAS3D_MAX_RHS];   /* ||g||_2 / ||b||_2 of the recursion */
    double relres_precond[ELAS3D_MAX_RHS];     /* sqrt(z.g / z0.g0)                  */
    double t_solve_s;                          /* wall time of the call              */
    double bytes_per_iter;                     /* algorithmic HBM bytes of one PCG
                                                  iteration (all RHS of the call)   */
    double t_operator_ms;                      /* summed fused-operator kernel time  */
    int64_t n_operator;                        /* fused-operator launches timed      */
    double t_update_ms;                        /* summed update-kernel time          */
    int64_t n_update;                          /* update launches timed              */
    int32_t fp64_fallback[ELAS3D_MAX_RHS];     /* mixed: 1 if the refinement stalled
                                                  and the solve finished in FP64    */
    int32_t op_tile[3];                        /* workgroup lanes in x, y and z-chunk
                                                  length of the direction+operator
                                                  sweep (of the inner solve in mixed) */
    int32_t update_blocks;                     /* grid of the update sweep (launched
                                                  with fewer workgroups when the grid
                                                  has under 256 nodes per workgroup) */
    int64_t precond_rows;                      /* rows of the M^-1 dictionary: one per
                                                  phase (shared by the nodes whose
                                                  eight voxels all have it) plus one
                                                  per phase-boundary node            */
    int32_t update_nontemporal;                /* 1 if the update sweep streams its
                                                  node vectors non-temporally        */
    int32_t apply_tile[3];                     /* workgroup lanes in x, y and z-chunk
                                                  length of the true-residual and
                                                  refinement sweeps                   */
    int32_t op_shape;                          /* the options.tile index of the
                                                  direction+operator sweep's shape
                                                  (op_tile's lanes do not tell 4
                                                  from 6)                            */
} elas3d_info;

/* Fill `opt` with the defaults (FP64, residual criterion, block Jacobi,
 * host pointers, automatic polling, no timing, current device, budget from
 * free memory, library stream, not batched, graphs on, no autotuning). */
void elas3d_options_init(elas3d_options* opt);

/*
 * Create a context: copy the inputs to the device, build the per-phase
 * coefficient tables, assemble the load vector b of every RHS (the work of
 * the macroscopic strain, Eq. (discrete_energy)) and the inverse point-block
 * Jacobi preconditioner M^-1 (Eq. (block_precond)).
 *   out     receives the context (set to NULL on error).
 *   nx,ny,nz grid size, each >= 2, 3*N < 2^31 (N = nx*ny*nz <= 715827882).
 *   phase   N phase ids in [0, nphase), x fastest (host, or device when
 *           opt->inputs_on_device).
 *   nphase  number of phases (>= 1).
 *   C       nphase*36 doubles (host), 6x6 per phase as described above.
 *   nrhs    number of macroscopic strains, 1..ELAS3D_MAX_RHS.
 *   strain  nrhs*6 doubles (host), tensor components per RHS.
 *   opt     NULL for defaults.
 * Returns 0, ELAS3D_EBADARG (null pointer, bad size, phase id out of range,
 * non-finite or asymmetric C, non-finite strain), ELAS3D_ENOMEM or
 * ELAS3D_EDEVICE.
 */
int elas3d_setup(elas3d_ctx** out, int32_t nx, int32_t ny, int32_t nz, const int32_t* phase,
                 int32_t nphase, const double* C, int32_t nrhs, const double* strain,
                 const elas3d_options* opt);

/*
 * Solve A w_r = -b_r for the first `nrhs` load cases from w_r = 0 by the PCG
 * of Algorithm 2 (or its mixed-precision refinement) until the criterion of
 * opt->convergence holds with `tol`, or `maxit` iterations per RHS.
 * `info` (may be NULL) receives per-RHS statistics.  Returns the worst
 * per-RHS status (0, ELAS3D_NOT_CONVERGED, ELAS3D_BREAKDOWN) or a negative
 * error.  The solutions stay on the device for elas3d_stress.
 */
int elas3d_solve(elas3d_ctx* ctx, double tol, int32_t maxit, int32_t nrhs, elas3d_info* info);

/*
 * Post-processing of load case `rhs` (Table 1, stress_OpenMP): per voxel the
 * stress at the voxel centroid sigma = C_p (E_hat + B(1/2,1/2,1/2) w_e),
 * which is the voxel average of the trilinear field (0 in voids).
 *   sigma_voxel  6*N doubles or NULL (device memory when outputs_on_device).
 *   sigma_avg    6 doubles (host) or NULL: mean over all N voxels (voids count 0).
 *   u_node       3*N doubles or NULL (device memory when outputs_on_device):
 *                total displacement u = E.X + w with X = (i,j,k) of the node.
 *   energy       1 double (host) or NULL: total potential energy
 *                Pi = 1/2 sum_e (u_e)^T K_e (u_e) (Eq. discrete_energy).
 * Returns 0, ELAS3D_EBADARG, ELAS3D_EORDER (rhs not solved) or ELAS3D_EDEVICE.
 */
int elas3d_stress(elas3d_ctx* ctx, int32_t rhs, double* sigma_voxel, double* sigma_avg,
                  double* u_node, double* energy);

/*
 * Matrix-free operator y = A x (Algorithm 2, step A: the 27-point coupling
 * of every node through its 8 voxels), x and y 3*N doubles.  Also the
 * building block of the true residual.  Returns 0 or a negative error.
 */
int elas3d_apply(elas3d_ctx* ctx, const double* x, double* y);

/* Copy the load vector b of case `rhs` (3*N doubles) out of the context. */
int elas3d_get_load(elas3d_ctx* ctx, int32_t rhs, double* b);

/* Copy the inverse diagonal blocks M^-1 (6*N doubles: planes xx, yy, zz,
 * yz, xz, xy of the symmetric 3x3 per node; 0 on nodes touched only by
 * voids) out of the context. */
int elas3d_get_precond(elas3d_ctx* ctx, double* minv);

/* Copy the fluctuation displacement w of case `rhs` (3*N doubles). */
int elas3d_get_solution(elas3d_ctx* ctx, int32_t rhs, double* w);

/*
 * Von Mises equivalent stress of load case `rhs` per voxel (Sec. 2.1.3,
 * Table 1, stress_fullfield): from the centroid stress sigma of
 * elas3d_stress, sqrt(((s11-s22)^2 + (s22-s33)^2 + (s33-s11)^2)/2
 * + 3 (s23^2 + s13^2 + s12^2)); 0 in voids.
 *   vm       N doubles or NULL (device memory when outputs_on_device).
 *   vm_max   1 double (host) or NULL: the largest value.
 *   argmax   1 int64 (host) or NULL: the lowest voxel index holding it.
 * Returns 0, ELAS3D_EBADARG, ELAS3D_EORDER (rhs not solved) or ELAS3D_EDEVICE.
 */
int elas3d_von_mises(elas3d_ctx* ctx, int32_t rhs, double* vm, double* vm_max, int64_t* argmax);

/*
 * Microstructure generator (Sec. 2.2), context-free.  opt (NULL = defaults)
 * supplies device, stream and outputs_on_device: when set, `phase` is device
 * memory, otherwise host memory.  Errors: ELAS3D_EBADARG (message in
 * elas3d_last_error(NULL)), ELAS3D_EDEVICE.  Seeds and pores are host
 * arrays and are copied.
 *
 * Grain assignment (Sec. 2.2.2, Eq. ellipsoid_dist): voxel (i,j,k), centre
 * x = (i+1/2, j+1/2, k+1/2), gets the grain g minimising
 *   D^2 = (dx^2 + dy^2) / rt_g^2 + dz^2 / rl_g^2
 * over all ngrain grains, d the periodic minimum-image offset of x from seed
 * g (x - s, or (x -+ L) - s when |x - s| > L/2), evaluated in FP64 in that
 * order; the lowest index wins a tie.  The result is exact (the search is cut
 * by a proven distance bound, not by a candidate radius).
 *   seeds  3*ngrain doubles, seed g at (x, y, z), each in [0, n_d).
 *   semi   2*ngrain doubles (rt_g, rl_g > 0), or NULL for all 1 (plain
 *          periodic Voronoi).
 *   phase  N int32 written with grain ids 0..ngrain-1.
 */
int elas3d_generate_grains(int32_t nx, int32_t ny, int32_t nz, int32_t ngrain, const double* seeds,
                           const double* semi, int32_t* phase, const elas3d_options* opt);

/*
 * Allocation-free grain assignment, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments and the same result, bit for bit, as
 * elas3d_generate_grains, but it calls no hipMalloc, hipFree or stream
 * creation: the seeds sorted by search cell go to a static device work area
 * of about 3.4 MB (one copy per GPU, held until the process ends) and the
 * host staging to static host arrays.  Limits and differences:
 *   - opt must be given with outputs_on_device set: `phase` is device
 *     memory (N int32);
 *   - ngrain <= 65536, and at most 131072 search cells (about one per seed;
 *     more only on very flat grids);
 *   - runs on opt->stream, or the default stream when it is NULL, and
 *     returns after the grain map is written (the stream is synchronised);
 *   - calls are serialised within the process (one lock): every call on a
 *     GPU shares that GPU's work area, whose contents the next call
 *     overwrites.
 * Errors: ELAS3D_EBADARG (as elas3d_generate_grains, plus the limits above;
 * checked before any device call), ELAS3D_EDEVICE; the message is in
 * elas3d_last_error(NULL).
 */
int elas3d_generate_grains_static(int32_t nx, int32_t ny, int32_t nz, int32_t ngrain, const double* seeds,
                                  const double* semi, int32_t* phase, const elas3d_options* opt);

/*
 * Pore overwrite (Sec. 2.2.3): pores p = 0, 1, ... are carved in order,
 * setting to void_id every voxel whose centre they cover, until the number of
 * void voxels reaches `target` (target < 0: carve all; none is carved when
 * the count already reaches it).  Pore p is 15 doubles: centre (3, in
 * [0, n_d)), semi-axes a (3, > 0), R (9, row-major, columns = the pore's
 * axes in the sample frame); it covers x when
 *   sum_j (e_j / a_j)^2 <= 1 + 1e-12,  e_j = (d0 R0j + d1 R1j) + d2 R2j,
 * d the minimum-image offset of x from the centre (as above), in FP64.
 *   phase   N int32, read and updated in place.
 *   used    (host, may be NULL) pores carved.
 *   nvoid   (host, may be NULL) void voxels afterwards.
 */
int elas3d_carve_pores(int32_t nx, int32_t ny, int32_t nz, int32_t* phase, int32_t void_id, int32_t npore,
                       const double* pores, double target, int32_t* used, int64_t* nvoid,
                       const elas3d_options* opt);

/*
 * Groups: continuous batching of independent solves.  A group advances the
 * PCG of every member context (its own grid, phases, stiffnesses and load
 * cases, set up with elas3d_setup) in lockstep, with one launch per sweep
 * for many members: the direction + operator sweep (one launch per 8
 * members), the update sweep and their finalizes each run over a work list
 * of (member, workgroup) entries, so four launches per iteration serve up to
 * 8 requests, and one more per further 8.  Members join
 * (elas3d_group_add) and leave (when converged) between batches of
 * iterations.  Each member follows its own precision option exactly as
 * elas3d_solve would (FP64 PCG with true-residual restarts, or FP32 inner
 * PCG cycles with FP64 refinement and FP64 fallback, Algorithm 2); the
 * group changes only which launches carry its sweeps, so a member's result
 * is bitwise the same alone and in any mix.  Sweeps run with workgroup
 * shape 0 and the default chunking (no autotuning inside a group).
 */

/* Create a group.  opt (NULL = defaults): device, stream (NULL = a library
 * stream).  Returns 0, ELAS3D_EBADARG or ELAS3D_EDEVICE. */
int elas3d_group_create(elas3d_group** out, const elas3d_options* opt);

/* Admit ctx (all of its load cases) with the stopping data of elas3d_solve.
 * The context must be on the group's device, not in another group, and set
 * up with options.batched when it has more than one load case.  While the
 * group runs it, it uses the group's stream and its own entry points
 * (solve, stress, von_mises, apply, get_*) return ELAS3D_EORDER;
 * elas3d_destroy withdraws it from the group first.  A member with nothing
 * to solve (zero load) finishes at once.  Members sweep with workgroup shape
 * 0 and the default z-chunking (options.tile, zchunk and autotune apply to
 * elas3d_solve only), so a member's results equal those of elas3d_solve with
 * the default geometry, bit for bit (options.update_blocks and
 * update_nontemporal do not apply to members either).  Returns 0, ELAS3D_EBADARG,
 * ELAS3D_EORDER (in a group, or finished in one and not returned yet) or
 * ELAS3D_EDEVICE. */
int elas3d_group_add(elas3d_group* g, elas3d_ctx* ctx, double tol, int32_t maxit);

/* Run `iters` lockstep iterations (>= 1) of every member, then settle the
 * members whose runs ended (refinement, restarts, completion).  Up to `cap`
 * finished contexts are returned in done[] with their statistics in
 * infos[] (as elas3d_solve's info; t_solve_s is the time since
 * elas3d_group_add); more wait for the next call.  A returned context is
 * solved (elas3d_stress works) and back on its own stream.  *ndone receives
 * the count; *nactive (may be NULL) the members still running.  Returns 0,
 * ELAS3D_EBADARG or ELAS3D_EDEVICE. */
int elas3d_group_run(elas3d_group* g, int32_t iters, elas3d_ctx** done, elas3d_info* infos, int32_t cap,
                     int32_t* ndone, int32_t* nactive);

/* Release the group.  Members still running are abandoned (their contexts
 * stay valid, unsolved, on their own streams). */
void elas3d_group_destroy(elas3d_group* g);

/*
 * Streaming-bandwidth probe (not part of a solve): the HBM rates that plain
 * streams reach on the device, the practical ceiling for the solver's sweeps,
 * which only stream vectors (the operator is matrix-free, Sec. 2.1.2).  The
 * call allocates two buffers of `bytes` each (freed before it returns) and
 * times three kernels on the options' device and stream (opt NULL:
 * defaults): copy (read one buffer, write the other), read-only and
 * write-only.  `blocks` workgroups of 256 lanes walk the buffer in a
 * grid-stride loop, 16 bytes per lane and access; nontemporal = 1 makes
 * every access non-temporal.  Each kernel runs once untimed, then `reps`
 * times between two events.
 *   gbs  (host) 3 doubles written: copy (bytes read + bytes written), read
 *        and write rates, in 1e9 bytes per second.
 * Returns 0, ELAS3D_EBADARG (gbs NULL, bytes < 1 MiB or not a multiple of
 * 16, blocks outside [1, 2^24], reps outside [1, 10000], nontemporal not 0
 * or 1; checked before any device call), ELAS3D_ENOMEM (the buffers do not
 * fit) or ELAS3D_EDEVICE; the message is in elas3d_last_error(NULL).
 */
int elas3d_stream_bandwidth(int64_t bytes, int32_t blocks, int32_t reps, int32_t nontemporal, double* gbs,
                            const elas3d_options* opt);

/* Device bytes a context with these sizes and options allocates at most (0
 * for sizes that elas3d_setup would reject); the bound counts one M^-1 row
 * per node, where setup stores one per phase and per phase-boundary node. */
double elas3d_device_bytes(int32_t nx, int32_t ny, int32_t nz, int32_t nphase, int32_t nrhs,
                           const elas3d_options* opt);

/* Release every device resource of the context (NULL is a no-op).  A
 * context that a group runs, or holds finished and not yet returned, is
 * withdrawn from the group first (after the group's work in flight). */
void elas3d_destroy(elas3d_ctx* ctx);

/* Message of the last error of `ctx`, or of the calling thread's last
 * context-free call (setup, generator) when ctx is NULL.  Never NULL. */
const char* elas3d_last_error(const elas3d_ctx* ctx);

/* Library version string. */
const char* elas3d_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ELAS3D_H */
