/*
 * fp.h -- C ABI of the MI355X (gfx950) library for the free-stream-preserving
 * conservative finite-difference scheme with reformulated upwind dissipation
 * on curvilinear grids (H. Su, J. Cai, S. Pan, X. Hu, "Reformulated
 * dissipation for the free-stream preserving of the conservative finite
 * difference schemes on curvilinear grids", arXiv 2101.05886).
 *
 * Problem statement (Sec. 2 and Sec. 3 of the paper): given a stationary
 * structured curvilinear grid and a conserved state Q of the Euler equations
 * (eqs. NS, Q, F, G, H, EOS without the viscous terms), form the metrics and
 * 1/J by the symmetric conservative metric method of order Y (eqs. JBabc, JB
 * with the central schemes of eq. metric_discret), evaluate the convective
 * residual dQ/dt = -(1/J)^{-1} sum_d (F'_{i+1/2} - F'_{i-1/2}) whose face flux
 * F' is reconstructed by WENO5-JS (eqs. weno, weno_wights) or the fifth-order
 * linear upwind scheme (eq. linear_upwind, eq. new_form_linear_upwind) from
 * reference-subtracted, characteristic, Lax-Friedrichs-split stencil values
 * with the reference flux added back (eqs. Q_star, QdJ_star, 1dJ,
 * flux_split_detail, my_point1, xidJ), and advance it with the third-order
 * TVD Runge-Kutta scheme (Sec. 2.2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Memory: every array argument is DEVICE memory of the current HIP device,
 *   float64, allocated and owned by the caller.  The library keeps no pointer
 *   after the work it enqueued has completed, except the step graphs cached
 *   by fp_solve (released by fp_release_cache).  Hot entry points
 *   (fp_residual, fp_rk3_step, fp_solve, fp_face_fluxes) allocate nothing.
 * Layout: structure of arrays, variable-major, i fastest.
 *   state q      : [nv][Nk][Nj][Ni], N_d = n_d + 2*ghost, nv = 5 (3D) or 4
 *                  (2D: Nk = 1) with variables (rho, rho u, rho v[, rho w], rho E);
 *   metrics met  : [nmet][Nk][Nj][Ni]; nmet = 10 in 3D (xi_x/J, xi_y/J, xi_z/J,
 *                  eta_x/J, eta_y/J, eta_z/J, zeta_x/J, zeta_y/J, zeta_z/J, 1/J),
 *                  5 in 2D (xi_x/J, xi_y/J, eta_x/J, eta_y/J, 1/J);
 *   coordinates  : [ndim][...] with extents n_d + 2*(ghost + Y/2).
 * Boundaries, per axis: FP_BC_PERIODIC -- the ghost layers of q are ignored
 *   (stencils wrap to the periodic image); the coordinate ghosts must hold the
 *   periodic images shifted by the period.  FP_BC_FROZEN -- the ghost layers
 *   of q hold caller values that are read and never written (every RK stage
 *   reads them from q); coordinate ghosts hold the mapping evaluated out of
 *   range.
 * Streams: `stream` is a hipStream_t passed as void* (NULL = legacy default
 *   stream).  Calls only enqueue work; the caller synchronises.
 * Errors: arguments are validated before anything is enqueued; an invalid
 *   call returns FP_EINVAL or FP_EUNSUPPORTED and enqueues nothing.  A launch
 *   failure returns FP_EHIP.  fp_last_error() gives a thread-local message
 *   for the last non-OK return.  No C++ exception crosses this interface.
 * Threads: entry points are reentrant; the graph cache is mutex-guarded.
 */
#ifndef FP_H
#define FP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FP_OK = 0,
    FP_EINVAL = -1,        /* malformed arguments */
    FP_EUNSUPPORTED = -2,  /* well-formed but not provided (e.g. metric order 3) */
    FP_EHIP = -3,          /* a HIP runtime call or kernel launch failed */
    FP_ENOMEM = -4,        /* a setup entry point could not allocate */
    FP_ENONPHYS = -5       /* reserved: no entry point returns it; non-physical
                              states are reported by fp_check_state's device flag */
} fp_status;

/* Reconstruction of the characteristic split fluxes (Sec. 3 and Remark 2):
 * WENO5-JS and the fifth-order linear upwind scheme (ghost >= 3), WENO7-JS
 * (ghost >= 4) and WENOCU6, the sixth-order adaptive central-upwind WENO
 * (ghost >= 3; C = 20, q = 2; in FP_MIXED32 its epsilon is floored at 1e-30). */
enum { FP_WENO5JS = 0, FP_LINUP5 = 1, FP_WENO7JS = 2, FP_WENOCU6 = 3 };
enum { FP_FP64 = 0, FP_MIXED32 = 1 };            /* precision of the characteristic part */
/* Lax-Friedrichs speeds of the characteristic splitting (Sec. 3 and 4):
 * local (the largest sigma |n.u_m + kappa_s c_m| over the face's stencil) or
 * global (the largest of those over every face of the block in the sweep
 * direction, per field class u_n - c, u_n, u_n + c; recomputed for every
 * stage; the paper's choice for the double Mach reflection and the
 * cylinder). */
enum { FP_LLF = 0, FP_GLF = 1 };
enum { FP_BC_PERIODIC = 0, FP_BC_FROZEN = 1 };   /* per axis */

/* One structured block.  ndim = 2 or 3; n[d] >= 1 interior nodes per axis
 * (n[2] = 1 when ndim = 2); ghost >= 3 and ghost >= metric_order/2;
 * a periodic axis needs n[d] >= ghost. */
typedef struct {
    int32_t ndim;
    int32_t n[3];
    int32_t ghost;
    int32_t bc[3];
} fp_grid;

/* The discretisation.  metric_order Y in {2,4,6,8} is used for the metrics
 * AND for the cell-face interpolation of 1/J, Q~ and the metrics inside the
 * flux (Remark 3).  reformulated = 1 is the paper's method; 0 is the
 * standard characteristic scheme (reference state zero), kept as the
 * negative control of the free-stream test.  precision = FP_MIXED32 runs the
 * characteristic projection, splitting, smoothness indicators, weights and
 * back-projection in FP32 on the reference-subtracted differences; metrics,
 * the reference state, subtraction, add-back and all stored state stay FP64. */
typedef struct {
    int32_t recon;
    int32_t metric_order;
    int32_t reformulated;
    int32_t precision;
    double gamma;     /* ratio of specific heats, > 1 (the paper: 1.4) */
    double weno_eps;  /* WENO epsilon, > 0 (the paper: 1e-6, for every WENO scheme) */
    int32_t splitting; /* FP_LLF or FP_GLF; FP_GLF only in fp_rk3_step, fp_solve,
                          fp_solve_bcs and fp_solve_ns (its speeds live in the workspace) */
    int32_t reserved;  /* 0 */
    double mu;         /* shear viscosity; 0 = Euler.  mu > 0 only in fp_viscous_residual and
                          fp_solve_ns, on grids whose axes are all periodic (n >= 7) */
    double prandtl;    /* Prandtl number (> 0 when mu > 0); the gas constant is 1 (T = p/rho),
                          so the conductivity is mu gamma / ((gamma - 1) Pr) */
} fp_scheme;

/* Sizes in bytes of the caller-allocated arrays. */
size_t fp_state_bytes(const fp_grid *grid);
size_t fp_metric_bytes(const fp_grid *grid);
size_t fp_coord_bytes(const fp_grid *grid, int32_t metric_order);
/* Workspace of fp_rk3_step / fp_solve: three state-sized arrays (two RK
 * stage registers and the residual accumulator) and a 2048-byte tail.  With
 * global Lax-Friedrichs speeds, RK stage k (0, 1, 2) reduces the speeds of
 * its input into set k of the tail (direction d's three speeds, for the
 * classes u_n - c, u_n, u_n + c, at doubles 48 k + 16 d .. 48 k + 16 d + 2)
 * and zeroes set k + 1 mod 3 for the next stage; each call zeroes set 0
 * first.  fp_solve_bcs keeps its device time at doubles 144 .. 146.
 * The tail needs no initial contents.  When an axis is frozen, the frozen
 * ghost layers of q are copied into the two stage registers before the
 * first step of each call (no step writes them again). */
size_t fp_work_bytes(const fp_grid *grid);

/* Symmetric conservative metrics and 1/J of order Y (Sec. 2.1, eqs. JBabc and
 * JB; derivatives by eq. metric_discret).  2D: xi_x/J = y_eta, xi_y/J = -x_eta,
 * eta_x/J = -y_xi, eta_y/J = x_xi and 1/J = 1/2[(x y_eta - y x_eta)_xi +
 * (y x_xi - x y_xi)_eta], the reduction of the 3D formulas for z = zeta.
 * Periodic axes: computed on the interior and copied into the ghost layers;
 * frozen axes: computed on the ghost nodes too.  Setup call (not hot). */
fp_status fp_metrics(const fp_grid *grid, int32_t metric_order, const double *xyz,
                     double *met, void *stream);

/* Face fluxes F'_{i+1/2} of one direction (Sec. 3, eq. my_point1 with the
 * reformulated dissipation of eqs. Linear_upwind_LFspliting and
 * flux_split_detail) at every face of every interior line.
 * flux: [nv][..] with extent n_dir + 1 along `dir` (index f <-> face
 * f - 1/2), interior extents on the other axes. */
fp_status fp_face_fluxes(const fp_grid *grid, const fp_scheme *scheme, const double *met,
                         const double *q, int32_t dir, double *flux, void *stream);

/* dQ/dt = -(1/J)^{-1} sum_{d = xi, eta, zeta} (F'_{i+1/2} - F'_{i-1/2})
 * (eq. aderivative, directions summed in that order) at the interior nodes.
 * Ghost entries of dqdt are not written.  q is not modified. */
fp_status fp_residual(const fp_grid *grid, const fp_scheme *scheme, const double *met,
                      const double *q, double *dqdt, void *stream);

/* One direction of the dimension-by-dimension residual (eq. aderivative for
 * direction `dir`): acc = -(F'_{i+1/2} - F'_{i-1/2}) when accumulate = 0, or
 * acc -= (F'_{i+1/2} - F'_{i-1/2}) when accumulate = 1, at the interior nodes
 * (no division by 1/J).  acc has the state layout; ghost entries are not
 * written.  Launches exactly one kernel.  Summing the three directions in
 * the order xi, eta, zeta and dividing by 1/J gives fp_residual. */
fp_status fp_residual_dir(const fp_grid *grid, const fp_scheme *scheme, const double *met,
                          const double *q, int32_t dir, double *acc, int32_t accumulate,
                          void *stream);

/* One step of the third-order TVD Runge-Kutta scheme (Sec. 2.2):
 * Q1 = Qn + dt L(Qn); Q2 = 3/4 Qn + 1/4 (Q1 + dt L(Q1));
 * Qn+1 = 1/3 Qn + 2/3 (Q2 + dt L(Q2)).  In place on the interior of q;
 * work: fp_work_bytes(grid) bytes of device memory. */
fp_status fp_rk3_step(const fp_grid *grid, const fp_scheme *scheme, const double *met,
                      double *q, double *work, double dt, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the step
 * of fp_rk3_step with its workspace in static device memory of the library
 * instead of a caller buffer.  Each GPU the library runs on holds one
 * FP_NOALLOC_WORK_BYTES array from the first call on that GPU until the
 * process ends; the call itself allocates nothing.  Grids whose
 * fp_work_bytes exceeds FP_NOALLOC_WORK_BYTES are rejected with FP_EINVAL
 * before anything is enqueued (64 MiB: up to 76^3 interior nodes in 3D,
 * 830^2 in 2D, with ghost 3).  Every call on one GPU shares that array, so calls that
 * overlap on one GPU (on different streams, or from several threads without
 * ordering) race and give undefined results; calls in one stream order are
 * safe.  The array keeps the last call's contents; a step writes every
 * workspace value it reads before reading it (stage registers, their frozen
 * ghost layers, the residual accumulator, the global speed sets), so no
 * clearing is needed.  Results are bitwise those of fp_rk3_step. */
#define FP_NOALLOC_WORK_BYTES ((size_t)64 << 20)
fp_status fp_rk3_step_noalloc(const fp_grid *grid, const fp_scheme *scheme, const double *met,
                              double *q, double dt, void *stream);

/* nsteps RK3 steps of fixed dt.  The first call for a given (grid, scheme,
 * pointers, dt) captures the stages of one step into a HIP graph that later
 * calls replay; the frozen ghost layers are copied into the stage registers
 * once per call (no step writes them), so ghost values the caller changes
 * take effect at the next call. */
fp_status fp_solve(const fp_grid *grid, const fp_scheme *scheme, const double *met,
                   double *q, double *work, double dt, int64_t nsteps, void *stream);

/* Viscous fluxes (Sec. 2.1 eqs. NSv1-NSv3 with the stress, strain and heat
 * flux definitions), discretised with sixth-order central differences
 * (Sec. 2.2): at every node the gradients of u and T by the chain rule
 * dphi/dx_j = J sum_d (xi_d)_{x_j}/J D6_d(phi), the stress
 * tau_ij = mu (du_i/dx_j + du_j/dx_i - 2/3 delta_ij div u), the physical
 * fluxes (0, tau_1j, .., u_i tau_ij + kappa dT/dx_j) and their
 * contravariant combinations Fv~_d = sum_j (xi_d)_{x_j}/J Fv_j; then
 * dQ/dt gains J sum_d D6_d(Fv~_d) (equal to the difference of sixth-order
 * face interpolations, so conservative).  Periodic axes only: the ghost
 * layers cannot hold the gradient stencils' reach.
 * vwork: fp_viscous_work_bytes(grid) bytes of device memory (the node
 * fluxes: ndim directions x (ndim + 1) components, state layout). */
size_t fp_viscous_work_bytes(const fp_grid *grid);

/* dQ/dt of the Navier-Stokes equations: the convective residual of
 * fp_residual plus the viscous part above (with mu = 0, fp_residual). */
fp_status fp_viscous_residual(const fp_grid *grid, const fp_scheme *scheme, const double *met,
                              const double *q, double *dqdt, double *vwork, void *stream);

/* nsteps RK3 steps (Sec. 2.2) of the Navier-Stokes equations; work as for
 * fp_rk3_step, vwork as above.  Launches eagerly. */
fp_status fp_solve_ns(const fp_grid *grid, const fp_scheme *scheme, const double *met, double *q,
                      double *work, double *vwork, double dt, int64_t nsteps, void *stream);

/* Boundary faces of a block for the wall-bounded problems of Sec. 4 (the
 * double Mach reflection and the supersonic cylinder).  Each face (axis a,
 * side 0 = low, 1 = high) of a FROZEN axis has a kind, applied to the ghost
 * layers of the face before every stage:
 *   FP_FACE_HOLD    ghosts keep the values the caller gave (inflow states);
 *   FP_FACE_EXTRAP  every ghost layer copies the boundary node (zeroth-order
 *                   extrapolation: supersonic outflow);
 *   FP_FACE_WALL    slip wall through the boundary node: ghost layer l takes
 *                   the state of the interior node l from the boundary with
 *                   the momentum's component along the wall normal reversed
 *                   (normal: the boundary node's metric vector of axis a);
 *                   the coordinates' ghost layers should be the mirror image
 *                   of the interior nodes, and n[a] > ghost;
 *   FP_FACE_SHOCK   a planar shock moving along `normal` at `speed`: ghost
 *                   nodes x with normal . x < offset + speed t take the
 *                   conservative state `post`, the others `pre`.
 * mask[a][side], if not NULL, is a device array of one byte per boundary
 * node of the face (interior nodes of the other axes, the lower-numbered
 * axis fastest): where it is 0 the face holds.  nodes: device coordinates of
 * the state nodes (ndim arrays in the state layout), read by FP_FACE_SHOCK
 * only.  Corner ghost regions are not written (no sweep reads them). */
enum { FP_FACE_HOLD = 0, FP_FACE_EXTRAP = 1, FP_FACE_WALL = 2, FP_FACE_SHOCK = 3 };

typedef struct {
    int32_t kind[3][2];
    const uint8_t *mask[3][2];
    const double *nodes;
    double pre[5], post[5];
    double normal[3];
    double offset, speed;
} fp_bcs;

/* The ghost layers of q's boundary faces at time t (one launch over every
 * face whose kind is not FP_FACE_HOLD). */
fp_status fp_apply_bcs(const fp_grid *grid, const fp_bcs *bcs, const double *met, double *q,
                       double t, void *stream);

/* nsteps RK3 steps from time t0 with the boundary faces applied to each
 * stage's input at the stage's time (t, t + dt, t + dt/2, with
 * t = t0 + i dt at step i; Sec. 2.2).  The first call for a given (grid,
 * scheme, faces, pointers, dt) captures one step into a HIP graph that later
 * calls replay: the time lives in the workspace tail, set at the start of
 * each call and advanced by the graph; fp_release_cache frees the graphs. */
fp_status fp_solve_bcs(const fp_grid *grid, const fp_scheme *scheme, const fp_bcs *bcs,
                       const double *met, double *q, double *work, double t0, double dt,
                       int64_t nsteps, void *stream);

/* Instrumented step (a measurement aid; none of the paper's operations is
 * added): one RK3 step of q (Sec. 2.2) exactly as fp_rk3_step launches it,
 * with the boundary faces of fp_solve_bcs at the stage times of a step from
 * t when bcs is non-NULL, and with the viscous part of fp_solve_ns when
 * scheme->mu > 0 (vwork then required, else ignored), and a HIP event
 * recorded on `stream` before the first launch and after each launch.
 * Synchronises, then writes each launch's duration in milliseconds to
 * kernel_ms[i] and its kind to kernel_kind[i], in launch order:
 *   0 xi sweep, 1 eta sweep, 2 zeta sweep, 3 frozen-ghost copy,
 *   5 global Lax-Friedrichs speeds, 6 boundary faces, 7 viscous node fluxes,
 *   8 viscous divergence, 9 reset of the first speed set;
 * and the number of launches (at most 32) to *n_kernels.  q advances one
 * step; work (and vwork) as for the step.  FP_EINVAL if max_kernels < 32 or
 * an argument is invalid (nothing enqueued then). */
fp_status fp_profile_step(const fp_grid *grid, const fp_scheme *scheme, const fp_bcs *bcs,
                          const double *met, double *q, double *work, double *vwork, double t,
                          double dt, float *kernel_ms, int32_t *kernel_kind, int32_t max_kernels,
                          int32_t *n_kernels, void *stream);

/* dt = cfl / max_i sum_d (|s_d . u| + c |s_d|) (1/J)^{-1} over the interior,
 * written to dt_dev (device, one double).  The test cases of Sec. 4 are run
 * at a stated CFL number (Sec. 4.2.1: 0.6) without the rule being printed;
 * this is the convective limit in index space, the characteristic speeds of
 * the transformed equations of Sec. 2.1 (|U_d| + c |grad xi_d| along each
 * index direction) summed over the directions.  FP_EINVAL on a bad grid,
 * scheme or pointer; cfl must be positive. */
fp_status fp_max_dt(const fp_grid *grid, const fp_scheme *scheme, const double *met,
                    const double *q, double cfl, double *dt_dev, void *stream);

/* flag_dev (device int32) is set to 1 if any interior node has a non-finite
 * value, rho <= 0 or p <= 0; it is left unchanged otherwise (the caller
 * clears it).  A diagnostic, not a step of the method: it detects the
 * breakdown (negative density or pressure) that Sec. 4.2 reports for the
 * standard schemes on randomized grids. */
fp_status fp_check_state(const fp_grid *grid, const fp_scheme *scheme, const double *q,
                         int32_t *flag_dev, void *stream);

/* ---- Batches: many independent blocks advanced in shared launches ----
 *
 * A batch advances many blocks, of uneven sizes and possibly mixed 2D/3D,
 * with one scheme, by the RK3 step of fp_rk3_step (Sec. 2.2), each block
 * with its own dt.  Per RK stage every sweep direction is ONE persistent
 * launch over a (block, tile) work list of all blocks of a dimensionality;
 * a step is 1 + 3 x ndim such launches (ghost copy, then per stage the
 * sweeps), plus one interface exchange per stage when blocks of that
 * dimensionality are linked; fp_batch_solve captures the stages once per
 * such configuration into a HIP graph and copies the ghosts once per call.  Per block the arithmetic is that of fp_rk3_step, and the
 * result is bitwise the same as advancing the block alone.
 *
 * Ownership: the batch owns its device work-list tables and a pinned host
 * staging copy (allocated by fp_batch_create, freed by fp_batch_destroy);
 * the blocks' arrays stay the caller's.  fp_batch_set, fp_batch_rk3_step,
 * fp_batch_solve and fp_batch_autotune allocate nothing (the first
 * fp_batch_solve of a given mix of 2D/3D parts captures a graph).  All calls
 * on one batch must use one stream and one thread at a time; different
 * batches are independent.  A block's arrays must not be freed while work of
 * a step that uses them is pending. */
typedef struct {
    fp_grid grid;
    const double *met; /* fp_metric_bytes(&grid), from fp_metrics */
    double *q;         /* fp_state_bytes(&grid), advanced in place */
    double *work;      /* fp_work_bytes(&grid), the block's own workspace */
    double dt;         /* > 0 */
} fp_block;

typedef struct fp_batch fp_batch;

/* A batch for up to max_blocks blocks (1 .. 65536) of `scheme`, on the
 * current HIP device.  FP_ENOMEM if the tables cannot be allocated. */
fp_status fp_batch_create(const fp_scheme *scheme, int32_t max_blocks, fp_batch **out);

/* Replaces the batch's blocks (host array of nblocks entries, 0 .. max
 * blocks; the entries are copied).  Every block is validated as in
 * fp_rk3_step; on an error nothing changes.  The new work list is copied to
 * the device in stream order, so steps enqueued earlier still see the old
 * list.  Graphs captured by fp_batch_solve stay valid. */
fp_status fp_batch_set(fp_batch *batch, const fp_block *blocks, int32_t nblocks, void *stream);

/* One RK3 step of every block of the batch. */
fp_status fp_batch_rk3_step(fp_batch *batch, void *stream);

/* nsteps RK3 steps of every block, replaying the batch's step graph.  The
 * frozen ghost layers of each block's q are copied into its stage registers
 * once, at the start of the call (no step writes them; so ghost values the
 * caller changes take effect at the next call), then the graph, which holds
 * the stages only, runs nsteps times. */
fp_status fp_batch_solve(fp_batch *batch, int64_t nsteps, void *stream);

/* Multi-block interfaces.  A link makes the ghost layers of `block` on
 * `side` (0 low, 1 high) of `axis` the interior layers of block `nbr` next
 * to its opposite side, so that the two blocks form one grid across the
 * face: the blocks must have the same dimensionality and ghost width, equal
 * extents and orientation along the other axes, and FP_BC_FROZEN on the
 * linked axis; an interface shared both ways needs two links.  Every RK
 * stage then starts with one exchange launch over all links (the stage's
 * register: q, then the two stage registers), so both blocks evaluate the
 * same flux on the shared face and the scheme stays conservative across it.
 * (The multi-block topology the paper's multi-block cases use; a single-GPU
 * form of the halo exchange a decomposition over GPUs would need.) */
typedef struct {
    int32_t block; /* index into the blocks of the last fp_batch_set */
    int32_t axis;  /* 0 .. ndim-1 */
    int32_t side;  /* 0: below index 0, 1: above index n-1 */
    int32_t nbr;   /* the neighbouring block */
} fp_link;

/* Replaces the batch's links (at most 6 per block slot; fp_batch_set clears
 * them).  Also copies, once and in stream order, the metric ghost layers of
 * every linked face from the neighbour's interior metrics: the library
 * WRITES those ghost layers of the blocks' met arrays.  The state ghost
 * layers of linked faces (in q and the workspace) are written every step.
 * Validation as described above; on an error nothing changes. */
fp_status fp_batch_set_links(fp_batch *batch, const fp_link *links, int32_t nlinks, void *stream);

/* Chooses the eta and zeta segment lengths of the batch's work lists (the
 * nodes along the sweep direction one workgroup item covers) by timing RK
 * stage 1 on the current blocks for a set of candidate targets, eta first
 * with zeta's held, then zeta (synchronises the stream; the blocks'
 * workspaces are overwritten, q is not).  The choice is kept for later
 * fp_batch_set calls and cached per process, keyed by the scheme and a size
 * class of the batch (its dimensionalities and, per dimensionality, the
 * binary orders of magnitude of its node count and mean eta and zeta line
 * lengths): a later call on a batch of the same class reuses it without
 * timing.  The eta target is written to *segment if non-NULL. */
fp_status fp_batch_autotune(fp_batch *batch, int32_t *segment, void *stream);

/* The batch's current segment-length targets, and whether the last
 * fp_batch_autotune took them from its cache (1) or timed them (0).  NULL
 * outputs are skipped. */
fp_status fp_batch_get_tiles(const fp_batch *batch, int32_t *seg_eta, int32_t *seg_zeta,
                             int32_t *from_cache);

/* Instrumented step: one RK3 step of every block, exactly as
 * fp_batch_rk3_step, with a HIP event recorded on `stream` after each of its
 * launches; synchronises and writes each launch's duration in milliseconds
 * to kernel_ms[i] and its kind to kernel_kind[i] = 16 * ndim + k (k = 0 xi
 * sweep, 1 eta sweep, 2 zeta sweep, 3 frozen-ghost copy, 4 interface
 * exchange), in launch order, and the number of launches (at most 26) to
 * *n_kernels.  FP_EINVAL if max_kernels is too small (nothing enqueued). */
fp_status fp_batch_profile_step(fp_batch *batch, float *kernel_ms, int32_t *kernel_kind,
                                int32_t max_kernels, int32_t *n_kernels, void *stream);

/* Frees the batch (after synchronising its pending work). NULL is a no-op. */
void fp_batch_destroy(fp_batch *batch);

/* Frees the cached step graphs. */
void fp_release_cache(void);

const char *fp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FP_H */
