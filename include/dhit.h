/*
 * dhit.h - C ABI of the MI355X (gfx950) library for the per-time-step update
 * of the lattice Boltzmann equation (LBE) and of the discrete unified
 * gas-kinetic scheme (DUGKS) on a periodic cube, as compared in
 * Wang, Wang & Guo, arXiv 1601.03815.
 *
 * General rules
 *   - Every function returns a status code (DHIT_OK = 0, negative on error;
 *     box_bytes and population_buffer_bytes return a byte count, or a
 *     negative status).  No C++ exception crosses this boundary.  After an
 *     error, dhit_last_error() returns a message for the calling thread.
 *   - Units are lattice units: dx = 1, particle speed c = 1, RT = c_s^2 =
 *     1/3 (Sec. IV.A).  The mean density rho0 is a parameter (the paper
 *     uses 1); velocities are u = j / rho0.
 *   - A box is an n^3 periodic grid of cells; cell (x, y, z) has flat index
 *     idx = (z*n + y)*n + x (x fastest).  Host-side arrays passed to this
 *     library are C arrays of double in that order: a scalar field is
 *     [n^3], a vector field is [3][n^3], a population field is [19][n^3].
 *   - Population order (D3Q19, Sec. II.A; the paper leaves it open, this
 *     order is part of the ABI): q0 = (0,0,0); q1..q6 = +x, -x, +y, -y,
 *     +z, -z; q7..q10 = (1,1,0), (-1,1,0), (1,-1,0), (-1,-1,0); q11..q14 =
 *     (1,0,1), (-1,0,1), (1,0,-1), (-1,0,-1); q15..q18 = (0,1,1),
 *     (0,-1,1), (0,1,-1), (0,-1,-1).
 *   - Populations are the paper's density-fluctuation form: the discrete
 *     equilibrium of Sec. II.A sums to drho, so f already excludes the
 *     W_i rho0 background (the "deviation form").  FP32 boxes store these
 *     same values in float.
 *   - Ownership: a box owns its device state unless the caller supplies
 *     the two population buffers (then the caller keeps ownership and must
 *     keep them alive until destroy_box).  The caller owns all host arrays.
 *   - Streams: all device work of a box is issued on params.stream (a
 *     hipStream_t; NULL makes the library create one).  step_* calls are
 *     asynchronous; calls that return host data synchronise that stream.
 *   - Thread safety: one box must not be used from two threads at once;
 *     different boxes are independent.
 *   - Environment: every entry point first clears a HIP error that other
 *     code left pending on the thread (DHIT_DEBUG=1 prints it to stderr);
 *     DHIT_TUNE_CACHE names the batch autotuner's cache file (create_batch).
 */
#ifndef DHIT_H
#define DHIT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dhit_box dhit_box;

enum dhit_status {
    DHIT_OK = 0,
    DHIT_EINVAL = -1,      /* bad argument (null pointer, size or parameter out of range) */
    DHIT_ENOMEM = -2,      /* device or host allocation failed */
    DHIT_EDEVICE = -3,     /* a HIP or hipFFT call failed */
    DHIT_EMETHOD = -4,     /* a call that does not apply to the box's method or mesh */
    DHIT_ENONFINITE = -5   /* a global reduction became NaN or infinite (the run blew up) */
};

enum dhit_method {
    DHIT_LBE_BGK = 0,      /* LBE with single-relaxation (BGK) collision, tau = 3 nu + 1/2 */
    DHIT_LBE_MRT = 1,      /* LBE with the D3Q19 multiple-relaxation-time collision of Sec. II.B */
    DHIT_DUGKS = 2         /* DUGKS finite-volume step of Sec. II.A, tau = nu / RT */
};

enum dhit_precision {
    DHIT_FP64 = 0,         /* populations stored and updated in double */
    DHIT_FP32 = 1          /* populations stored and updated in float, per-cell moment sums
                              compensated, global reductions in double */
};

/* Kernel variant of a step.  DHIT_VARIANT_DEFAULT picks the fastest
 * implementation; DHIT_VARIANT_TWO_PASS selects the two-kernel DUGKS step
 * (cell transform to a scratch field, then the face loop), kept as a
 * plainer cross-check of the fused kernel.  Ignored by LBE boxes. */
enum dhit_variant { DHIT_VARIANT_DEFAULT = 0, DHIT_VARIANT_TWO_PASS = 1 };

typedef struct dhit_params {
    int32_t n;          /* cells per side, 4 <= n <= 1024 */
    int32_t method;     /* enum dhit_method */
    int32_t precision;  /* enum dhit_precision */
    int32_t variant;    /* enum dhit_variant */
    int32_t tile_width; /* fused DUGKS kernel: width of a block's column tile, 16 or 32
                           (0 = the default, 32) */
    int32_t z_chunk;    /* fused DUGKS kernel, planes one block marches through:
                           c > 0: z-chunks of c planes (c <= n), one block per
                           column tile and chunk;
                           -c < 0: the same chunks, except that when they fill
                           at least one round of the device's resident blocks
                           and the last round at most half, each chunk of the
                           last round is cut in z into parts of
                           ceil(c / min(slots / left-over chunks, c)) planes,
                           so that the round fills the device;
                           0 = chosen at create_box for the current device:
                           among the chunks ceil(n/k) >= min(n, 8), plain or
                           cut, the one that minimises the launch's estimated
                           plane iterations per block.  Every setting gives
                           the same populations; the global sums agree to
                           rounding (the work split groups the cells' sums) */
    double nu;          /* kinematic viscosity, > 0 */
    double rho0;        /* mean density, > 0 (paper: 1) */
    double dt;          /* time step: LBE requires 1; DUGKS requires 0 < dt*sqrt(2) <= 1
                           (CFL number dt*sqrt(2) of Sec. IV.A; the paper uses dt = 0.5) */
    /* MRT relaxation rates, diagonal of S in Sec. II.B (used by DHIT_LBE_MRT only).
     * s9 and s13 are normally 1/(3 nu + 1/2) (Sec. IV.A); default_params sets them so. */
    double s1, s2, s4, s9, s10, s13, s16;
    /* MRT equilibrium constants of Sec. II.B (paper: 0, -475/63, 0). */
    double w_eps, w_epsj, w_xx;
    void *stream;       /* hipStream_t, or NULL */
    void *f_a, *f_b;    /* optional caller-owned device buffers, each of
                           population_buffer_bytes(params) bytes and 256-byte aligned;
                           both NULL makes the library allocate them */
} dhit_params;

/* Fill *out with the paper's parameters for an n^3 box (Sec. IV.A):
 * rho0 = 1; dt = 1 (LBE) or 0.5 (DUGKS); s1 = 1.19, s2 = s10 = 1.4,
 * s4 = 1.2, s16 = 1.98, s9 = s13 = 1/(3 nu + 1/2); w_eps = w_xx = 0,
 * w_epsj = -475/63; variant default; stream and buffers NULL. */
int32_t default_params(int32_t n, int32_t method, int32_t precision, double nu,
                       dhit_params *out);

/* Bytes of one population buffer (19 padded per-population arrays). */
int64_t population_buffer_bytes(const dhit_params *p);

/* Device bytes a box with these parameters needs: both population buffers
 * (counted even when the caller supplies them), plus reduction scratch and,
 * for DUGKS boxes of the two-pass variant, the transform scratch field.
 * The spectrum work space is allocated on the first energy_spectrum call
 * and is not included.  Used by schedulers to admit boxes by HBM budget. */
int64_t box_bytes(const dhit_params *p);

/* Device bytes of a box's spectrum work space (energy_spectrum,
 * vorticity, initial_pressure, and the DUGKS init_consistent allocate it on
 * their first call and keep it until destroy_box): its arrays plus the work
 * areas of its two hipFFT plans, queried from hipFFT for this n (plans made
 * without allocation).  For schedulers that admit boxes by HBM budget and
 * take diagnostics before releasing them.  A negative status on error. */
int64_t spectrum_bytes(const dhit_params *p);

/* Work split of the fused DUGKS step (Sec. II.A update, marched in z by
 * column tiles; the z_chunk field above) of a box with parameters *p, on a
 * device that holds `slots` blocks of the fused kernel at once (compute
 * units x resident blocks: 256 or 512 on a 256-unit device, by precision).
 * Host computation only, for tools and tests; needs no device.
 * fused_work_items: returns the number of work items (one block each) of
 * the step's launch, or a negative status; *z_chunk (may be NULL) receives
 * the setting in effect (p->z_chunk, or the automatic choice for `slots`).
 * fused_work_item: the column tile (numbered x fastest, then y; tiles of
 * tile_width - 2 by 6 updated columns) and the planes [*z0, *z0 + *planes)
 * that item `item` marches (*planes = 0: an empty slot).  Every tile-plane
 * of the box belongs to exactly one item.  Errors: DHIT_EINVAL for null
 * pointers, invalid parameters (as create_box), slots < 1 or an item out of
 * range; DHIT_EMETHOD for an LBE box or the two-pass variant. */
int32_t fused_work_items(const dhit_params *p, int32_t slots, int32_t *z_chunk);
int32_t fused_work_item(const dhit_params *p, int32_t slots, int32_t item, int32_t *tile, int32_t *z0,
                        int32_t *planes);

/* Create a box.  Validates *p; on success *out owns the new box. */
int32_t create_box(const dhit_params *p, dhit_box **out);

/* Destroy a box and free the device memory the library allocated. */
int32_t destroy_box(dhit_box *b);

/* Set the initial state from a velocity field u[3][n^3] (host) and an
 * optional density-fluctuation field drho[n^3] (host, NULL = 0).
 * BGK-LBE and DUGKS start from f = f^eq(drho, rho0 u) (Sec. II.A
 * equilibrium; for DUGKS the tracked f~ equals f when Omega = 0); MRT-LBE
 * starts from f = M^-1 m^eq (the fixed point of its collision, Sec. II.B).
 * Resets the step counter and the reduction history.  Synchronous. */
int32_t init_velocity_field(dhit_box *b, const double *u, const double *drho);

/* The same initial state from fields already in device memory: u[3][n^3]
 * and drho[n^3] (NULL = 0) are device pointers (doubles, the layout of
 * init_velocity_field's host arrays).  Asynchronous: the state is built by
 * one kernel enqueued on the box's stream and the call returns at once; the
 * caller keeps u and drho unchanged until that stream has passed the
 * kernel.  Allocates nothing and waits for nothing, so a scheduler can
 * start a run while other work is queued on the device.  Resets the step
 * counter. */
int32_t init_velocity_field_device(dhit_box *b, const double *u, const double *drho);

/* Stretched mesh for a DUGKS box (the finite-volume scheme's advantage the
 * paper names in Sec. V; the reconstruction of Sec. II.A with the positions
 * of a non-uniform mesh).  widths: host [3][n] doubles, the width of cell i
 * along x, y, z (the box length of an axis is the sum of its widths; the
 * mesh is periodic).  Faces sit at c_i +- w_i/2, with cell centres
 * c_i = w_0/2 + sum_{k<i} (w_k + w_{k+1})/2.  At each face between cells L
 * and R the value is fbp_L + (fbp_R - fbp_L) w_L/(w_L + w_R), the normal
 * gradient (fbp_R - fbp_L)/(c_R - c_L), and each tangential gradient is the
 * cells' central difference over c_{k+1} - c_{k-1}, interpolated with the
 * same weight; the update divides each axis's flux difference by the cell's
 * width along it.  From then on every step of the box runs this path
 * (whatever the variant) and the five sums of the step history and of
 * moments() are weighted by the cell volumes w_x w_y w_z.  Unit widths give
 * the uniform scheme.  widths = NULL returns the box to unit cells.
 * Allocates the mesh tables and, if the box has none, the scratch field of
 * the two-pass form.  Synchronous.  DHIT_EMETHOD on an LBE box;
 * DHIT_EINVAL for a width that is not finite and > 0, or for
 * sqrt(2) dt > min width (CFL above 1; the paper takes
 * dt = CFL dx_min / sqrt(2)).  Boxes with a stretched mesh cannot be batched
 * (create_batch and step_batch reject them, and batch_step of a batch built
 * before the call returns DHIT_EINVAL), and energy_spectrum and vorticity
 * reject them (DHIT_EMETHOD). */
int32_t set_mesh(dhit_box *b, const double *widths);

/* Density fluctuation that belongs to a velocity field (Sec. IV.A: the
 * initial pressure comes from the Poisson equation in spectral space, and
 * the kinetic schemes take it through the equation of state): the
 * incompressible pressure p with lap p = -rho0 d_i d_j (u_i u_j), computed
 * with the box's hipFFT work space on the integer wavevectors of the n^3
 * grid, p_hat = -rho0 sum_ij k_i k_j (u_i u_j)_hat / |k|^2 (zero mean; the
 * Nyquist component of each derivative factor dropped, as for S and F),
 * and drho = p / c_s^2 = 3 p.  u: host [3][n^3], drho: host [n^3], both
 * idx = (z*n + y)*n + x; the box's state is not touched (only its n, rho0,
 * stream and spectrum work space are used).  The natural drho argument of
 * init_velocity_field and init_consistent.  Synchronous; allocates an
 * upload buffer for the call. */
int32_t initial_pressure(dhit_box *b, const double *u, double *drho);

/* Consistent initial state for a prescribed velocity field (Sec. IV.A: the
 * kinetic schemes start from the density fluctuation and the
 * non-equilibrium part that belong to the initial velocity).
 * drho: host [n^3] or NULL = 0 (the spectral pressure of the velocity,
 * initial_pressure, is the natural choice); u: host [3][n^3] doubles,
 * idx = (z*n + y)*n + x.
 * LBE boxes: the scheme iterated with the velocity held.  Starts as
 * init_velocity_field(b, u, drho), then runs `iters` passes of: one LBE
 * step of the box's method, then every cell's momentum put back to rho0 u
 * with its density and non-equilibrium part kept (f += E(drho, rho0 u) -
 * E(drho, j), E the state init_velocity_field builds).  On return the
 * velocity is u (to rounding) and the density and the non-equilibrium part
 * are the scheme's own.  *residual (host, may be NULL) receives the largest
 * change of drho over the last pass (0 for iters = 0).
 * DUGKS boxes: the held-velocity iteration does not converge for the
 * finite-volume fluxes, so the non-equilibrium part is the first-order
 * Chapman-Enskog one of the BGK model (Sec. II.A collision, tau = nu/RT),
 * f1_q = -(tau rho0/RT) W_q (xi_qa xi_qb - RT delta_ab) d_a u_b, with the
 * spectral velocity gradient (i kappa_a u_hat_b, Nyquist component
 * dropped), in the tracked variable: f~ = f^eq(drho, rho0 u) +
 * (1 + dt/(2 tau)) f1 (f~ = f - dt/2 Omega, Sec. II.A).  `iters` is not
 * used (it must still be >= 0) and *residual is 0.  The box needs unit
 * cells (DHIT_EMETHOD after set_mesh).
 * Both: the step counter and the reduction history are reset.
 * Synchronous; allocates device work space for the call (and the spectrum
 * work space, DUGKS).  DHIT_EINVAL for a null u or iters < 0,
 * DHIT_ENONFINITE if the LBE iteration's density stopped being finite. */
int32_t init_consistent(dhit_box *b, const double *u, const double *drho, int32_t iters, double *residual);

/* Advance an LBE box by nsteps >= 0 steps of dt = 1: fused pull
 * streaming + collision (Sec. II.B evolution equation; BGK or MRT).  The
 * stored state is the post-collision population field.  Each step ends
 * with the global FP64 reduction (sum drho, sum jx, sum jy, sum jz,
 * 1/2 sum |u|^2) of the new state, kept in the box's history.
 * Asynchronous.  DHIT_EMETHOD on a DUGKS box. */
int32_t step_lbe(dhit_box *b, int32_t nsteps);

/* Advance a DUGKS box by nsteps >= 0 steps of dt (Sec. II.A finite-volume
 * update): cell transform to f-bar-plus and f~+, face reconstruction with
 * the half-step characteristic, face equilibrium, flux divergence.  The
 * stored state is f~.  Same per-step reduction as step_lbe.
 * Asynchronous.  DHIT_EMETHOD on an LBE box. */
int32_t step_dugks(dhit_box *b, int32_t nsteps);

/* Per-cell density fluctuation drho[n^3] and momentum j[3][n^3] (host,
 * each optional) and the global sums[5] = (sum drho, sum jx, sum jy,
 * sum jz, 1/2 sum |j/rho0|^2) of the current state (optional).  The
 * moments do not depend on the storage phase (collision conserves them).
 * Synchronous.  Returns DHIT_ENONFINITE if a sum is not finite. */
int32_t moments(dhit_box *b, double *drho, double *j, double *sums);

/* Global sums of the reductions run at the end of the last `count` steps,
 * oldest first, into out[count][5]; count <= min(steps taken, 4096).
 * Synchronous.  Returns DHIT_ENONFINITE if any of them is not finite. */
int32_t sums_history(dhit_box *b, double *out, int32_t count);

/* Energy spectrum and statistics of the current velocity field u = j/rho0
 * (Sec. III): u_hat = DFT(u)/n^3 (hipFFT); E[k] for integer shells
 * k = 0..kmax is the sum of 1/2 |u_hat|^2 over modes with round(|k|) = k;
 * stats[4] (optional) = (K, eps, S, F): K = sum of 1/2 |u_hat|^2 over all
 * modes, eps = 2 nu sum |kappa|^2 1/2 |u_hat|^2 with kappa = 2 pi k / n,
 * S and F the direction-averaged velocity-derivative skewness and flatness
 * from spectral derivatives (Nyquist component dropped).  0 <= kmax.
 * Allocates its work space on the first call.  Synchronous. */
int32_t energy_spectrum(dhit_box *b, double *E, int32_t kmax, double *stats);

/* Vorticity omega = curl u of the current velocity field u = j/rho0 (the
 * flow fields shown in Sec. IV.B), in lattice units (cell size 1): spectral
 * derivatives, omega_hat = i kappa x u_hat with kappa = 2 pi k / n, the
 * Nyquist component of each derivative dropped as for S and F.
 * omega: host [3][n^3] doubles, idx = (z*n + y)*n + x.  Shares the
 * spectrum work space (allocated on the first call).  Synchronous. */
int32_t vorticity(dhit_box *b, double *omega);

/* Copy the stored population field to/from host f[19][n^3] (double; FP32
 * boxes convert).  The stored phase is post-collision for LBE boxes and
 * f~ for DUGKS boxes.  set_populations resets the step counter and the
 * reduction history.  Synchronous. */
int32_t get_populations(dhit_box *b, double *f);
int32_t set_populations(dhit_box *b, const double *f);

/* Number of steps taken since the last initialisation. */
int64_t steps_taken(const dhit_box *b);

/* Wait for all queued work of the box.  Returns DHIT_ENONFINITE if the
 * newest reduction is not finite. */
int32_t box_synchronize(dhit_box *b);

/* Device pointer of the buffer that holds the current population field and
 * its per-population stride in elements (for callers that read the state
 * in place, e.g. from PyTorch).  Either output may be NULL. */
int32_t current_populations(const dhit_box *b, void **ptr, int64_t *stride);

/* Batches: many boxes of one method and precision advanced together
 * (an ensemble of independent runs, e.g. of different grid sizes).
 * Each step is one kernel launch over a work list spanning all boxes (LBE:
 * runs of 256 cells, or 512 when every box's n is even in FP64, two cells
 * per thread; DUGKS: tile z-chunks of the fused kernel), on a grid of one
 * block per work item or on a persistent grid whose blocks loop over them,
 * followed by one launch that finalises every box's global sums; the
 * per-box buffer index and step counter are kept on the device, so runs of
 * 8 steps are replayed from one captured hipGraph.  Results equal
 * single-box steps: populations bit for bit (a single DUGKS box runs the
 * same work-list kernel on a table of one entry, and the march rounds
 * alike whatever the z-chunk; a batch of tile width 16 equals boxes of
 * tile_width 16), global sums to rounding (the chunk decides how the cell
 * sums are grouped).
 *
 * create_batch: boxes[nbox] must share method and precision (DUGKS boxes the
 * default variant) and appear once.  With autotune != 0 the grid (one block
 * per work item, or a persistent grid of 1 to 32 blocks per compute unit)
 * and, for DUGKS, the column-tile width (16 or 32) and work-item
 * z-chunk (8, 16 or 32 planes, or per box n planes below n = 32, 16 below
 * n = 128 and 32 from there on, the untuned batch's chunks) are chosen by
 * timing uncommitted trial steps on the boxes
 * themselves (their states are left unchanged); choices are cached per
 * process under (method, precision, compute units of the device, grid
 * sizes) and, if the environment variable DHIT_TUNE_CACHE names a file,
 * read from and appended to it (one line per choice: key, grid, chunk,
 * tile).  Without autotuning a DUGKS batch uses tile width 32 and as many
 * blocks as the device holds at once (LBE: one block per work item).  Work is
 * issued on the first box's stream (or the one batch_set_stream names); on
 * the device, each batch step waits for the work queued on the boxes' own
 * streams before it, and the boxes' streams wait for the step after it (the
 * host waits for neither).  The boxes must outlive the batch.  With
 * autotune, synchronous (the trial steps are timed). */
typedef struct dhit_batch dhit_batch;
int32_t create_batch(dhit_box **boxes, int32_t nbox, int32_t autotune, dhit_batch **out);

/* Replace the batch's boxes by boxes[nbox] (same method and precision as
 * the batch; the rules of create_batch), for callers whose set of runs
 * changes often (a serving loop): the device tables are rebuilt in place
 * (they grow when needed and are never shrunk, so a smaller set frees
 * nothing and waits for nothing), the autotuned tile width and z-chunk are
 * kept, and the captured graph is captured again on the next batch_step of
 * eight steps or more.  Boxes no longer in the set may be destroyed after
 * the call (destroy_box waits for the device).  Asynchronous. */
int32_t batch_update(dhit_batch *bt, dhit_box **boxes, int32_t nbox);

/* Issue the batch's later work on `stream` (a hipStream_t; NULL = the
 * null stream) instead of the first box's stream, e.g. one stream per
 * method in a serving loop whose boxes keep streams of their own (a box's
 * stream then only orders that box's own work, such as its spectrum, after
 * the batch steps it took part in).  Waits for the work already issued on
 * the batch's previous stream. */
int32_t batch_set_stream(dhit_batch *bt, void *stream);

/* Advance every box of the batch by nsteps >= 0 steps.  Asynchronous: the
 * table of buffer indices and step counters goes up through one of two
 * pinned copies, so the call waits at most for the upload two calls back. */
int32_t batch_step(dhit_batch *bt, int32_t nsteps);

/* info[6] = (grid size, DUGKS z-chunk (0 = per-box default),
 * work items per step, steps per graph replay, 1 if autotuned, DUGKS
 * column-tile width (0 for LBE)). */
int32_t batch_info(const dhit_batch *bt, int64_t *info);

int32_t destroy_batch(dhit_batch *bt);

/* One-off form: builds a batch without tuning or graph, runs nsteps, frees it. */
int32_t step_batch(dhit_box **boxes, int32_t nbox, int32_t nsteps);

/* Kernel kinds reported by read_kernel_timings. */
enum dhit_kernel {
    DHIT_K_LBE = 0,              /* LBE pull streaming + collision */
    DHIT_K_DUGKS_TRANSFORM = 1,  /* DUGKS cell transform (two-pass variant) */
    DHIT_K_DUGKS_FACE = 2,       /* DUGKS face fluxes and update (two-pass variant) */
    DHIT_K_DUGKS_FUSED = 3,      /* DUGKS single-kernel step */
    DHIT_K_FINALIZE = 4,         /* global-sum finalisation */
    DHIT_NKERNEL = 5
};

/* Per-kernel timing.  While enabled, every kernel the box launches is
 * bracketed by two HIP events recorded on the box's stream (at most 8192
 * launches are kept; older ones are dropped).  read_kernel_timings waits for
 * the stream, adds the elapsed time of every recorded launch to ms[kind]
 * (milliseconds) and the launch count to launches[kind] (both arrays of
 * DHIT_NKERNEL entries, overwritten), and clears the record.  Enabling or
 * disabling also clears it. */
int32_t set_kernel_timing(dhit_box *b, int32_t enable);
int32_t read_kernel_timings(dhit_box *b, double *ms, int64_t *launches);

/* Allocation-free step, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  One step of the method in *p (LBE: step_lbe's kernel, BGK or
 * MRT; DUGKS: the fused kernel of step_dugks, variant default only) from
 * the population field in src to dst, with the same per-step FP64 global
 * reduction: sums (device double[5], or NULL) receives (sum drho, sum jx,
 * sum jy, sum jz, 1/2 sum |u|^2) of the new state.  No box is involved:
 * src and dst are caller-owned device buffers of
 * population_buffer_bytes(p) bytes each, 256-byte aligned, distinct, laid
 * out as a box's buffers (19 arrays of the padded stride; LBE: the stored
 * post-collision phase; DUGKS: f~); p->f_a and p->f_b are ignored.
 * Work is issued on p->stream (NULL = the null stream), which must belong to
 * the current device; the call returns without waiting.
 * The per-block partial sums of the reduction go to a static work space of
 * the library on the current device (131072 block slots, 5 MiB, held until
 * the process ends); the call makes no allocation of any kind.  Every call
 * on one GPU shares that work space: calls whose work overlaps on one GPU
 * (on different streams, or from different threads) race and must be
 * ordered by the caller.  Each launch writes every slot it reads, so nothing
 * has to be cleared between calls.
 * Errors: DHIT_EINVAL for null pointers, src == dst, misaligned buffers,
 * invalid parameters (as create_box), the two-pass DUGKS variant, or a box
 * whose reduction needs more than 131072 block slots (LBE: n > 322);
 * DHIT_EDEVICE if a launch fails. */
int32_t step_noalloc(const dhit_params *p, const void *src, void *dst, double *sums);

/* Copy `bytes` bytes (a multiple of 16) between two 16-byte-aligned
 * device buffers on `stream` (a hipStream_t, NULL = the null stream) with a
 * plain streaming copy kernel: the reference for achievable HBM bandwidth
 * and for calibrating hardware byte counters.  Asynchronous. */
int32_t device_copy(void *dst, const void *src, int64_t bytes, void *stream);

/* Message of the last error on the calling thread ("" if none). */
const char *dhit_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DHIT_H */
