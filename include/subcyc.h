/* subcyc: subcycled RK4 time integration on nested block-structured mesh
 * refinement, with refinement-boundary ghost zones filled from the coarse
 * level's RK4 dense output, on one AMD Instinct MI355X (gfx950).
 *
 * Method: Ji, Haas, Zlochower, Brandt, Schnetter, Wen, "GPU-accelerated
 * Subcycling Time Integration with the Einstein Toolkit" (arXiv:2503.09629),
 * Sec. II.  The problem is dy/dt = f(y) (Sec. II, first equation) on a
 * hierarchy of levels with refinement ratio 2 in space and time.
 *
 * Conventions shared by every call
 *   - Return value: SC_OK (0) or a negative sc_status.  No call aborts or
 *     throws; sc_last_error() describes the most recent failure.
 *   - Grids are vertex centred.  On level l the index i sits at
 *     x = origin + i * dx0 / 2^l; level l-1 index I coincides with level l
 *     index 2I.  Boxes are inclusive index ranges on their own level.
 *   - Host-side floating point arguments are always double.
 *   - Device memory is owned by the caller: sc_device_bytes() reports the
 *     arena size, the caller allocates it (any allocator) and binds it with
 *     sc_bind_device_memory(); the library never allocates or frees device
 *     memory itself and never creates streams.  Work is enqueued on the
 *     caller's HIP stream given to sc_create(); calls that return host data
 *     synchronise that stream.
 *   - State machine: CREATED -> BUILT (sc_build_hierarchy) -> BOUND
 *     (sc_bind_device_memory) -> READY (first sc_set_initial_data).  A call
 *     made in the wrong state returns SC_E_STATE.
 *   - One thread may use a context at a time.
 */
#ifndef SUBCYC_H
#define SUBCYC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SC_ABI_VERSION 3

typedef enum {
  SC_OK = 0,
  SC_E_ARG = -1,       /* bad argument (null pointer, out-of-range value, CFL > 0.5) */
  SC_E_STATE = -2,     /* call out of order */
  SC_E_NEST = -3,      /* hierarchy not properly nested or not aligned */
  SC_E_MEM = -4,       /* bound arena too small or misaligned */
  SC_E_HIP = -5,       /* a HIP runtime call failed; the message names it */
  SC_E_NONFINITE = -6  /* a NaN or infinity in the state (sc_check_finite, sc_advance) */
} sc_status;

/* Right-hand sides.  SC_RHS_WAVE: the scalar wave as a first-order system,
 * du/dt = Pi, dPi/dt = Laplacian(u) (Sec. IV.A); variables (u, Pi).
 * SC_RHS_Z4C: the Z4c system with the puncture gauge (Sec. III.A), vacuum,
 * 22 variables in the slot order W, gt_xx, gt_xy, gt_xz, gt_yy, gt_yz, gt_zz,
 * Khat, At_xx, At_xy, At_xz, At_yy, At_yz, At_zz, Theta, Gt^x, Gt^y, Gt^z,
 * alpha, beta^x, beta^y, beta^z (FP64, or FP32 right-hand side with
 * SC_MIXED). */
enum { SC_RHS_WAVE = 0, SC_RHS_Z4C = 1 };

/* Precision of the right-hand-side stencil.  The state, the RK4
 * accumulation, dense output, prolongation and restriction stay FP64 in both
 * modes.  SC_MIXED with the wave: the wave right-hand side f is linear, so
 * stage s >= 2 evaluates k_s = k1 + f(Y_s - y_n) with the stage increment
 * Y_s - y_n = c_s dt k_{s-1} (refinement-boundary ghosts: the dense-output
 * stage value minus the stage-1 value) in FP32, and k1 = f(y_n) in FP64;
 * slopes are stored in FP32.  FP32 rounding enters through quantities of size
 * dt |k| instead of |y|, so the stencil's 1/h^2 amplification of it stays
 * below the discretisation error of the benchmark hierarchies.  SC_MIXED
 * with Z4c: the right-hand side reads FP32 shadow copies of the stage
 * vectors and evaluates in FP32 (the system is not linear). */
enum { SC_FP64 = 0, SC_MIXED = 1 };

/* Execution of one coarse step.  PER_BLOCK: one kernel launch per block per
 * stage; BATCHED: one launch per level per stage covering all blocks of the
 * level; GRAPH: BATCHED, captured once as a HIP graph and replayed. */
enum { SC_EXEC_PER_BLOCK = 0, SC_EXEC_BATCHED = 1, SC_EXEC_GRAPH = 2 };

/* Arrays that can be read back: the state y, the stored RK4 slopes k1..k4 of
 * the last step (Sec. II, step 1 "Store k1..k4") and y_n, the state at the
 * start of the last step. */
enum { SC_ARR_Y = 0, SC_ARR_K1 = 1, SC_ARR_K2 = 2, SC_ARR_K3 = 3, SC_ARR_K4 = 4, SC_ARR_YN = 5 };

/* Ghost fills at refinement boundaries: the fine stage vectors Y1..Y4
 * (Sec. II, Eqs. Y1-Y4) and the state after a substep ("end", dense output
 * at theta0 + 1/2, Sec. II steps 3 and 5). */
enum { SC_FILL_Y1 = 1, SC_FILL_Y2 = 2, SC_FILL_Y3 = 3, SC_FILL_Y4 = 4, SC_FILL_END = 5 };

typedef struct sc_ctx sc_ctx;

/* Time stepping (Sec. IV.A compares both).  SC_SUBCYCLED: level l steps with
 * dt_l = cfl dx_l, two fine steps per parent step, fine refinement-boundary
 * ghosts from the parent's cubic dense output (Sec. II).  SC_UNIFORM_DT: every
 * level steps with the finest level's dt, one fine step per parent step, and
 * the fine ghosts of stage s take the parent's own stage value at the same
 * time, y_n + c_s dt k_{s-1} (RK4 nodes c = 0, 1/2, 1/2, 1), prolonged in space;
 * the parent's step is complete before the fine step starts.
 * SC_BUFFER_ZONES: the buffer-zone subcycling the paper compares against
 * (Carpet, Sec. II and Fig. 1; wave RHS, FP64 only).  Steps as SC_SUBCYCLED,
 * but the owned points of a fine level within 3 G (Chebyshev) of a refinement-
 * boundary point are buffer points: before every fine step the parent's state
 * at the step's start time, interpolated in time over the parent's last three
 * states (quadratic; linear over two while the parent has made one step) and
 * prolonged in space, is written into the buffer points and the refinement-
 * boundary ghosts; the ghosts keep that value through all four stages, the
 * buffer points are evolved and then discarded, and restriction skips them.
 * The valid region of a fine box is thus the box minus 3 G layers on each
 * refinement-boundary face, and the stencils of its ghosts and buffer points
 * must avoid the parent's buffer points (SC_E_NEST otherwise).  Only
 * sc_advance steps this mode; the single-step pieces return SC_E_STATE. */
enum { SC_SUBCYCLED = 0, SC_UNIFORM_DT = 1, SC_BUFFER_ZONES = 2 };

/* Outer boundary of a non-periodic domain (Sec. III.A applies an outgoing
 * condition to the dynamical variables).  SC_BC_FROZEN: the physical-boundary
 * ghosts keep the values the caller set with sc_set_phys_data.
 * SC_BC_RADIATIVE (Z4c, FP64, physical-boundary ghosts on level 0 only): the
 * level-0 ghosts are evolved with d_t f = -(v/r)(x^i d_i f + (f - f0)), r the
 * distance from the coordinate origin, f0 = 1 for W, the conformal metric's
 * diagonal and the lapse and 0 otherwise, v = sqrt(2) for the lapse and 1
 * otherwise; derivatives are second-order one-sided (inwards) across the
 * boundary and centred along it; the ghosts take the same RK4 stages as owned
 * points, starting from the values set with sc_set_phys_data. */
enum { SC_BC_FROZEN = 0, SC_BC_RADIATIVE = 1 };

typedef struct {
  int64_t lo[3], hi[3]; /* inclusive vertex indices on the box's level, x, y, z */
} sc_box;

typedef struct {
  int32_t abi_version; /* SC_ABI_VERSION */
  int32_t rhs;         /* SC_RHS_* */
  int32_t precision;   /* SC_FP64 or SC_MIXED */
  int32_t exec;        /* SC_EXEC_* */
  int32_t nghost;      /* ghost width: 3 for fd_order 4, 4 for fd_order 8; 5 for fd_order 8
                          with the ninth-order dissipation */
  int32_t time_stepping; /* SC_SUBCYCLED (default), SC_UNIFORM_DT or SC_BUFFER_ZONES */
  double ko_sigma;     /* Kreiss-Oliger strength sigma (Sec. III.C), e.g. 0.32 */
  double cfl;          /* dt_l = cfl * dx_l, 0 < cfl <= 0.5 */
  double z4c_kappa1;   /* Z4c constraint damping kappa_1 (default 0.02) */
  double z4c_kappa2;   /* kappa_2 (default 0) */
  double z4c_eta_c;    /* shift damping eta(r) = (eta_c - eta_o) exp(-(r/eta_s)^4) + eta_o, */
  double z4c_eta_o;    /*   r the distance from the coordinate origin; defaults 2, 0.25, 40 */
  double z4c_eta_s;    /*   (Sec. III.A, M = 1) */
  int32_t fd_order;    /* derivative order: 4 (default), or 8 with nghost 4 (the
                          production stencil of Sec. III.C: nine-point centred first
                          and second differences, the same fifth-order dissipation;
                          wave or Z4c, FP64, SC_SUBCYCLED or SC_UNIFORM_DT); fd_order 8
                          with nghost 5 selects the ninth-order dissipation of the
                          same section (its Q u with r = 8: sigma/(1024 h) times the
                          eleven-point tenth difference per dimension; wave or Z4c,
                          FP64) */
  int32_t outer_bc;    /* SC_BC_FROZEN (default) or SC_BC_RADIATIVE */
} sc_config;

/* Fill *cfg with the defaults: wave RHS, FP64, batched, nghost 3, fd_order 4,
 * sigma 0.32, cfl 0.25, Z4c kappa1 0.02, kappa2 0, eta 2 / 0.25 / 40. */
int sc_config_default(sc_config* cfg);

/* Create a context that enqueues on hip_stream (a hipStream_t owned by the
 * caller, or NULL for the null stream).  No device memory is touched. */
int sc_create(const sc_config* cfg, void* hip_stream, sc_ctx** out);

/* Destroy a context and its host-side tables and graphs.  Does not free the
 * bound arena (the caller owns it).  NULL is accepted. */
int sc_destroy(sc_ctx* ctx);

/* Text of the last error on ctx, or of the last failed sc_create on this
 * thread when ctx is NULL.  Owned by the library; valid until the next call. */
const char* sc_last_error(const sc_ctx* ctx);

/* Build the hierarchy of levels with refinement ratio 2 in space and time
 * (Sec. II) and every index map (host only, once); the maps hold all grid
 * index arithmetic, so the kernels do arithmetic only (Sec. III.C).
 *   nmembers        independent copies evolved together (ensemble batching)
 *   origin, dx0     coordinates of level-0 index 0 and level-0 spacing
 *   ncells0         level-0 cells per dimension; level 0 holds indices
 *                   [0, n-1] in a periodic dimension and [0, n] otherwise
 *   periodic        per dimension, 0 or 1
 *   nlevels         number of levels (>= 1)
 *   nboxes_per_level  counts for levels 1..nlevels-1 (nlevels-1 entries)
 *   boxes           the boxes of levels 1.. concatenated in level order
 *   block_seed      seed of the block split (SplitMix64 stream per level,
 *                   state block_seed + level)
 *   min_block, max_block  block side limits (max_block >= 2*min_block - 1)
 * Blocks: every level box is split recursively along its longest side (ties
 * x, y, z) at min_block + (draw mod (n - 2 min_block + 1)), left part first.
 * Fine boxes need even bounds (or to span a periodic dimension), must lie in
 * the domain, must not overlap, and every parent point of every
 * refinement-boundary prolongation stencil must be owned by one parent box;
 * otherwise SC_E_NEST. */
int sc_build_hierarchy(sc_ctx* ctx, int32_t nmembers, const double origin[3], double dx0,
                       const int64_t ncells0[3], const int32_t periodic[3], int32_t nlevels,
                       const int32_t* nboxes_per_level, const sc_box* boxes,
                       uint64_t block_seed, int32_t min_block, int32_t max_block);

/* Per level (one member): number of blocks, owned points, and distinct
 * refinement-boundary (RB) points. */
int sc_get_counts(const sc_ctx* ctx, int32_t level, int32_t* nblocks, int64_t* nowned,
                  int64_t* nrb);

/* Per level (one member): number of buffer points (SC_BUFFER_ZONES; 0 in the
 * other modes and on level 0).  Buffer points are owned points, included in
 * sc_get_counts' nowned. */
int sc_buffer_count(const sc_ctx* ctx, int32_t level, int64_t* nbuffer);

/* Canonical little-endian int64 export of all maps; words == NULL returns the
 * size in *nwords.  Layout: header [0x53554243, 1, nlevels, nmembers]; then
 * per level: [level, nblocks, nowned, nrb, nrestrict], the blocks
 * [lo x,y,z, hi x,y,z] in id order, every block's ghost slots in visiting
 * order (z-major, y, x fastest over [lo-G, hi+G]^3 minus the block) as
 * SYNC [0, owner block, owner-local offset] / RB [1, rb index, 0] /
 * PHYS [2, -1, 0], the RB list sorted by (z, y, x) as
 * [qx, qy, qz, qx/2, qy/2, qz/2, odd bits x=1 y=2 z=4], and the restriction
 * pairs sorted by (parent block, parent offset) as
 * [parent block, parent offset, block, offset].  Offsets are
 * ((z - lo_z) n_y + (y - lo_y)) n_x + (x - lo_x) within the owning block.
 * With SC_BUFFER_ZONES the header's second word is 2, restriction pairs
 * leave out buffer points, and each level ends with [nbuffer] and its buffer
 * points sorted by (z, y, x) in the RB-list format. */
int sc_export_maps(const sc_ctx* ctx, int64_t* words, int64_t* nwords);

/* Device arena size in bytes for the built hierarchy and configuration. */
int sc_device_bytes(const sc_ctx* ctx, size_t* nbytes);

/* Bind a caller-owned device allocation of at least sc_device_bytes() bytes,
 * 256-byte aligned, and upload the index tables (asynchronously, on the
 * context's stream).  The caller keeps it alive until sc_destroy. */
int sc_bind_device_memory(sc_ctx* ctx, void* dptr, size_t nbytes);

/* Initial data y(t_0) of the problem dy/dt = f(y) (Sec. II) for one variable
 * on the owned points of one level of one member, n = owned points, in
 * canonical order (the level's boxes in order, each z-major, y, x fastest).
 * The host array is copied before return; the first call moves the context
 * to READY. */
int sc_set_initial_data(sc_ctx* ctx, int32_t member, int32_t level, int32_t var,
                        const double* host, int64_t n);

/* Physical-boundary ghosts (non-periodic domains) hold frozen values set by
 * the caller.  sc_phys_count: number of such halo points of a level (one
 * member); sc_phys_points: their coordinates as xyz triples (3n doubles) in
 * the library's order; sc_set_phys_data: values of one variable at those
 * points, same order, copied into every ghost table of the level. */
int sc_phys_count(const sc_ctx* ctx, int32_t level, int64_t* n);

/* Closed-form initial data evaluated on the GPU at every owned point of every
 * level and member (and at the frozen physical-boundary ghosts of
 * non-periodic levels), for every variable; moves the context to READY.
 * params (host, nparams doubles, copied) by kind:
 *   SC_ID_STANDING_WAVE (wave): an exact standing-wave solution of the wave
 *     system of Sec. IV.A, u = A sin(m_x pi x) sin(m_y pi y) sin(m_z pi z),
 *     Pi = 0: params (A, m_x, m_y, m_z); or nparams = 0: per member, m_d =
 *     1 + (draw mod 3) for x, y, z and A = 0.5 + U[0,1) from SplitMix64(seed)
 *     (U = top 53 bits of a draw times 2^-53), members in order.
 *   SC_ID_GAUSSIAN_PULSES (wave): u = sum_p A_p g_p(x) g_p(y) g_p(z), Pi = 0,
 *     g_p(x) = sum_k exp(-(x - c_p,x - k L)^2 / w_p^2) over the periodic
 *     images k = -1, 0, 1 of period L (L = 0: k = 0 only), a sum of the
 *     Gaussian profiles of the paper's scalar-wave test (Sec. IV.A):
 *     params (npulses <= 32, L, then A, w, c_x, c_y, c_z per pulse); or
 *     (npulses, L, x_t): per pulse A = 0.1 + 0.9 U, w = 0.05 + 0.15 U,
 *     o = -0.1 + 0.2 U three times, c = (-x_t + o_x, o_y, o_z) for even p and
 *     (x_t + o_x, o_y, o_z) for odd p, drawn from SplitMix64(seed) in that order.
 *   SC_ID_BRILL_LINDQUIST (Z4c): two time-symmetric punctures at (x_+, 0, 0)
 *     and (x_-, 0, 0) with bare masses m_+, m_-: psi = 1 + a,
 *     a = m_+/(2 r_+) + m_-/(2 r_-), W = psi^-2, conformally flat, K = 0, zero
 *     shift, and the initial lapse of Sec. III.B, (1 + (1 - a)/(1 + a))/2:
 *     params (m_+, m_-, x_+, x_-).
 *   SC_ID_SPHERICAL_GAUSSIAN (wave): the exact outgoing solution of the
 *     paper's scalar-wave test (Sec. IV.A) at time t, u = (f(t-r) - f(t+r))/r,
 *     Pi = du/dt, f(v) = A exp(-v^2/(2 sigma^2)), with its limits at r = 0:
 *     params (A, sigma, t).
 * SC_E_ARG for an unknown kind, a kind of the other right-hand side or a bad
 * parameter list; SC_E_STATE before sc_bind_device_memory.  Synchronises. */
enum { SC_ID_STANDING_WAVE = 1, SC_ID_GAUSSIAN_PULSES = 2, SC_ID_BRILL_LINDQUIST = 3,
       SC_ID_SPHERICAL_GAUSSIAN = 4 };
int sc_set_initial_data_analytic(sc_ctx* ctx, int32_t kind, const double* params,
                                 int32_t nparams, uint64_t seed);
int sc_phys_points(const sc_ctx* ctx, int32_t level, double* xyz, int64_t n);
int sc_set_phys_data(sc_ctx* ctx, int32_t member, int32_t level, int32_t var,
                     const double* host, int64_t n);

/* Advance the whole hierarchy by ncoarse coarse steps with the recursive
 * subcycling schedule (Sec. II, steps 1-7): a level takes one RK4 step,
 * prolongs (y_n, k1..k4) to its child's refinement boundary, the child takes
 * two steps at theta0 = 0 and 1/2, and the child's solution is restricted by
 * injection.  Asynchronous.  Every RK4 step flags a non-finite y_{n+1} on the
 * device; the flag is copied back after the steps without a wait, and a later
 * sc_advance that finds it set (once the copy has arrived) returns
 * SC_E_NONFINITE and enqueues nothing.  New initial data clear the flag. */
int sc_advance(sc_ctx* ctx, int32_t ncoarse);

/* The pieces of sc_advance, for callers that drive the schedule themselves:
 * one RK4 step of one level with its stage ghosts taken from the prolonged
 * data of the given substep (0: theta0 = 0, 1: theta0 = 1/2; ignored on
 * level 0), without recursion (Sec. II, steps 1, 3, 5); */
int sc_step_level(sc_ctx* ctx, int32_t level, int32_t substep);
/* prolongation of the parent's (y_n, k1..k4) to fine_level's refinement
 * boundary, producing the ghost stage values of both substeps (step 2); */
int sc_prolongate(sc_ctx* ctx, int32_t fine_level);
/* ghost fill of the state y of a level: SYNC copies, and on refinement
 * boundaries the dense-output value `which` (SC_FILL_*) of `substep`; */
int sc_fill_ghosts(sc_ctx* ctx, int32_t level, int32_t which, int32_t substep);
/* injection of fine_level's state into the parent (step 7). */
int sc_restrict(sc_ctx* ctx, int32_t fine_level);

/* Read one array (SC_ARR_*: the state y, the stored RK4 slopes k1..k4 of
 * Sec. II step 1, or y_n) of one variable on the owned points of a level of
 * a member, canonical order, n = owned points (host, caller-owned).
 * Synchronises the stream.
 * The wave stencil keeps k4 only on levels that have a finer level (nothing
 * else reads it); SC_ARR_K4 on the finest level returns SC_E_STATE. */
int sc_read_back(sc_ctx* ctx, int32_t member, int32_t level, int32_t var, int32_t array,
                 double* host, int64_t n);

/* Refinement-boundary ghost values of a level as the stencil would see them
 * for stage `which` (SC_FILL_Y1..Y4 from the stored stage tables,
 * SC_FILL_END recomputed) of `substep`, in RB-list order, n = nrb of the
 * level.  Requires a preceding sc_prolongate.  Synchronises the stream. */
int sc_read_rb(sc_ctx* ctx, int32_t member, int32_t level, int32_t which, int32_t substep,
               int32_t var, double* host, int64_t n);

/* Deterministic norms of one array of one variable over the owned points of
 * a level of a member (the error and constraint norms the paper reports in
 * Sec. IV are of this kind): out[0] = max |a|, out[1] = sqrt(mean a^2),
 * out[2] = number of non-finite values (host, caller-owned).  A fixed-shape
 * two-pass reduction on the GPU, so repeated calls give the same bits.
 * Synchronises the stream. */
int sc_norms(sc_ctx* ctx, int32_t member, int32_t level, int32_t var, int32_t array,
             double out[3]);

/* sc_norms for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same reduction, bit for bit, with its partials and result in a workspace
 * that the library holds in static device memory (one copy per GPU, 128 KiB,
 * kept until the process ends) instead of the context's arena.  It allocates
 * nothing.  Levels of more than 4096 * 8192 = 33,554,432 owned points per
 * member exceed that workspace: SC_E_ARG, with a message.  Every call on a
 * GPU shares its workspace, so calls that overlap on one GPU (two streams,
 * two threads, two contexts) race; the result is copied back before return
 * (synchronises the context's stream). */
int sc_norms_noalloc(sc_ctx* ctx, int32_t member, int32_t level, int32_t var, int32_t array,
                     double out[3]);

/* Error of the state against a closed-form solution at time t, over the owned
 * points of one level of one member, for one variable: out[0] = max |y - exact|,
 * out[1] = sqrt(mean (y - exact)^2), out[2] = number of non-finite state
 * values (host, caller-owned).  The error norms of the paper's scalar-wave
 * test (Sec. IV.A, Fig. 2) are of this kind.  kind and params as in
 * sc_set_initial_data_analytic at time t: SC_ID_STANDING_WAVE with
 * (A, m_x, m_y, m_z, t) (u = A cos(w t) S, Pi = -A w sin(w t) S,
 * w = pi |m|) or SC_ID_SPHERICAL_GAUSSIAN with (A, sigma, t); wave only.
 * The same deterministic reduction as sc_norms.  Synchronises. */
int sc_error_norms(sc_ctx* ctx, int32_t member, int32_t level, int32_t var, int32_t kind,
                   const double* params, int32_t nparams, double out[3]);

/* Z4c only: the composite-grid L2 norm of the Hamiltonian constraint that the
 * paper monitors (Sec. IV.B), over the points with r < rmax (distance from
 * the coordinate origin) where the lapse exceeds alpha_min (outside the
 * horizons), each point counted once on the finest level that has it, with
 * weight dx_l^3: out[0] = sqrt(sum w H^2 / sum w), out[1] = max |H| over
 * those points, out[2] = non-finite H values there (host, caller-owned).  H
 * as in sc_hamiltonian, reduced on the GPU level by level (deterministic
 * order).  Fills the state's ghosts; call it between coarse steps, after the
 * first.  Synchronises. */
int sc_constraint_norm(sc_ctx* ctx, int32_t member, double rmax, double alpha_min,
                       double out[3]);

/* Z4c only: Hamiltonian constraint H = R + 2/3 (Khat + 2 Theta)^2 - At_ij At^ij
 * (vacuum) of the current state on the owned points of a level of a member,
 * canonical order, n = owned points.  Fills the state's ghosts first (SYNC,
 * physical, and the dense-output end value of the second substep on
 * refinement boundaries), so call it between coarse steps.  Synchronises. */
int sc_hamiltonian(sc_ctx* ctx, int32_t member, int32_t level, double* host, int64_t n);

/* SC_E_NONFINITE if any owned value of the state is not finite on any level
 * (a full scan, which names the level, member and variable).  Synchronises. */
int sc_check_finite(sc_ctx* ctx);

/* Simulation time of a level (host bookkeeping). */
int sc_level_time(const sc_ctx* ctx, int32_t level, double* t);

/* Switch the execution mode (SC_EXEC_*) between calls to sc_advance. */
int sc_set_exec(sc_ctx* ctx, int32_t exec);

/* Fill every halo table and every slope array with quiet NaN, so that any
 * read of a ghost value that the schedule did not fill first shows up as a
 * non-finite result (a test aid for fill ordering).  SC_E_STATE if a level
 * has physical-boundary ghosts, whose values this would erase. */
int sc_poison_halos(sc_ctx* ctx);

/* Autotune the batched stencil kernel: for every level, time candidate
 * tile widths (the widest the LDS window and ring allow, 64 and 32 points),
 * z-chunk depths of the tile table, persistent grid sizes and the stencil
 * variant (threads per workgroup, owned points per thread, planes of loads
 * kept in flight ahead of the computed plane: see sc_set_tile_shape) with
 * HIP events (reps times the four stage launches of one RK4 step, on the
 * bound data) and keep the first candidate, in search order, within 1.5 % of
 * the fastest (so that near-equal shapes do not trade places between runs).
 * Overwrites the slopes of every level
 * and the state buffer that the next step writes (call it before a run or
 * between coarse steps).  Invalidates captured graphs.  Synchronises the
 * stream. */
int sc_autotune(sc_ctx* ctx, int32_t reps);
/* Tile shape of a level: out = {widest tile, tallest tile, z-chunk, workgroups
 * launched (a multiple of 8: the kernels give each of the 8 XCDs a contiguous
 * run of tiles), tiles, planes of loads in flight, points per thread, threads
 * per workgroup}.  Until sc_autotune or sc_set_tile_shape changes it, a wave
 * context cuts 16-plane tiles of at most 512 points per plane and a Z4c
 * context two-plane tiles of at most 256 points per plane (its kernels run one
 * wave per SIMD and need many tiles to fill the chip; they launch one
 * workgroup per tile, rounded up to a multiple of 8, which is what a Z4c
 * context reports as its workgroup count).  The FP64 Z4c derivative pass
 * keeps its own fixed columns (64 x 4 points, 16 planes; 32 at eighth
 * order), which neither call reports or changes. */
int sc_tile_shape(const sc_ctx* ctx, int32_t level, int32_t out[8]);
/* Set a level's stencil tile shape without timing (for instance one found by
 * sc_autotune in an earlier run).  Wave contexts: z-chunk tz >= 4, persistent workgroups grid
 * (0: the context default, capped at the tile count), planes of loads in
 * flight ahead of the computed plane (depth), owned points per thread (slots)
 * and threads per workgroup (threads; a tile holds at most threads * slots
 * points), (threads, slots, depth) one of (256, 2, 1), (256, 2, 2),
 * (256, 1, 2), (512, 2, 1), (512, 2, 2); widest tile tx in 1..128 (0: the
 * untuned default, 64; the LDS window and ring slots cap it lower, at 78 for
 * the fourth-order stencil), so that the widths sc_tile_shape reports, set
 * back, cut the same tiles.  SC_E_ARG if a value is out of range
 * or the shape gives more tiles than the tile table was sized for.  Z4c
 * contexts: only tz applies (tz >= 2; the shape sc_tile_shape reports can be
 * set back); grid, depth, slots, threads and tx are ignored, since the Z4c
 * kernels keep their workgroup shape and launch one workgroup per tile.
 * Invalidates captured graphs; synchronises the stream. */
int sc_set_tile_shape(sc_ctx* ctx, int32_t level, int32_t tz, int32_t grid, int32_t depth,
                      int32_t slots, int32_t threads, int32_t tx);

/* Timing of the stencil stage kernel with HIP events recorded on the
 * context's stream (eager modes only; SC_E_STATE in graph mode): one pair
 * around a level step's four batched stage launches when no other kernel
 * runs between them (no intra-level ghost sync), else one pair around each
 * batched stage launch.  Enabling clears the record. */
int sc_profile_enable(sc_ctx* ctx, int32_t on);
/* Synchronise, then return the recorded launches, their summed duration in
 * milliseconds and their summed algorithmic bytes: per owned point and
 * variable, stage 1 reads y_n and writes k1 (16 B), stages 2 and 3 read y_n
 * and the previous slope and write the next (24 B), stage 4 also reads k1,
 * k2 and writes y_{n+1} (48 B).  Clears the record. */
int sc_profile_read(sc_ctx* ctx, int64_t* nlaunches, double* total_ms, double* alg_bytes);

/* Point-updates of one coarse step of one member (sum over levels of owned
 * points times level steps) and launches enqueued by the last sc_advance. */
int sc_stats(const sc_ctx* ctx, int64_t* updates_per_coarse_step, int64_t* launches);

#ifdef __cplusplus
}
#endif
#endif /* SUBCYC_H */
