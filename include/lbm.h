/* lbm.h -- C ABI of the MI355X (gfx950) fine-box lattice-Boltzmann library.
 *
 * The library advances one or many small lattice-Boltzmann boxes that follow
 * the multiscale strategy of Lee, Duenweg and Schumacher ("Multiscale
 * modelling strategy using the lattice Boltzmann method for polymer dynamics
 * in a turbulent flow"):
 *   - standard D3Q19 lattice (Sec. 3), BGK or weighted-orthogonal MRT
 *     collision with Guo-type forcing, fused with pull streaming;
 *   - the velocity field is prescribed on all sites at t = 0 and on the
 *     boundary layer only at t > 0, both by setting populations to the local
 *     equilibrium (Sec. 2); the boundary velocity is a time series sampled
 *     along a Lagrangian tracer in the tracer frame w = u - v(t) (Sec. 2),
 *     interpolated linearly in space and time (Sec. 2, Sec. 3);
 *   - bead-spring (FENE) chains coupled to the fluid by a Stokes friction
 *     coefficient (Sec. 1) with their centre of mass pinned (Sec. 2).
 *
 * Conventions shared by every call
 *   - Every call returns lb_status: LB_OK (0) or a negative error code; the
 *     text of the last error is available from lb_last_error().
 *   - Boxes are indexed 0..n_boxes-1.  Node (x, y, z) of a box with
 *     dimensions (nx, ny, nz) -- boundary layer included -- has linear index
 *     (z*ny + y)*nx + x.  Interior nodes are those whose every non-periodic
 *     coordinate lies in [1, n-2]; only they are evolved.  The boundary layer
 *     is every other node.
 *   - Lattice directions c_i, i = 0..18, in this order: (0,0,0); (1,0,0),
 *     (-1,0,0), (0,1,0), (0,-1,0), (0,0,1), (0,0,-1); (1,1,0), (-1,-1,0),
 *     (1,-1,0), (-1,1,0), (1,0,1), (-1,0,-1), (1,0,-1), (-1,0,1), (0,1,1),
 *     (0,-1,-1), (0,1,-1), (0,-1,1).  Weights 1/3, 1/18 (x6), 1/36 (x12).
 *   - Ownership: input pointers belong to the caller and are copied (or
 *     consumed) before the call returns.  All device memory belongs to the
 *     context.  Output buffers must be exactly the documented size, else
 *     LB_ERR_BUFSIZE.
 *   - Time: the state after n steps is the pre-collision state at t_n = n.
 *     Step n uses the boundary velocity at t_n.
 *   - Streams: all device work is ordered on lb_config.stream (NULL = the
 *     null stream, which PyTorch's default stream also is).  lb_step is asynchronous; lb_sync and
 *     lb_read_fields synchronise.  A context is not thread-safe.
 *   - Errors found on the device (overstretched FENE bond, bead stencil
 *     leaving the interior, non-finite mass or momentum) are latched with the
 *     step at which they occurred and returned by the next lb_sync or
 *     lb_read_fields; the state then stays at the last good step and further
 *     lb_step calls return the latched error.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LB_OK = 0,
  LB_ERR_ARG = -1,       /* invalid argument, or stepping beyond the boundary samples */
  LB_ERR_OOM = -2,       /* device allocation failed */
  LB_ERR_HIP = -3,       /* a HIP runtime call failed */
  LB_ERR_FENE = -4,      /* a FENE bond reached r >= R0 */
  LB_ERR_BEAD_OUT = -5,  /* a bead's interpolation stencil left the interior */
  LB_ERR_UNSTABLE = -6,  /* non-finite mass or momentum at a check */
  LB_ERR_STATE = -7,     /* call out of order (e.g. stepping without a boundary) */
  LB_ERR_BUFSIZE = -8    /* output/input buffer size mismatch */
} lb_status;

typedef struct lb_ctx lb_ctx; /* opaque; owns all device memory */

typedef enum { LB_BGK = 0, LB_MRT = 1 } lb_collision;

/* Population storage.  Collisions are computed in FP64 for LB_STORE_F64 and in
 * FP32 otherwise, always on deviations from rest equilibrium d_i = f_i - w_i rho0;
 * the chains (bead state, impulses, spreading weights, gathered force) in FP64
 * for every storage.  LB_STORE_F16DEV stores h_i = (f_i/w_i - rho0) * 2^s as
 * IEEE half, s = lb_config.fp16_exp: the step rounds stochastically (up with
 * probability equal to the fraction of an ulp; the random bits come from a
 * counter of node, step and direction, so runs are reproducible), state uploads
 * round to nearest even. */
typedef enum { LB_STORE_F64 = 0, LB_STORE_F32 = 1, LB_STORE_F16DEV = 2 } lb_storage;

/* Streaming.  LB_STREAM_AB: two population buffers, each step pulls from one
 * and writes the other.  LB_STREAM_AA: one buffer updated in place (half the
 * memory): an even step reads every node's populations in place and writes
 * its post-collision f*_i into the node's own slot of the opposite direction;
 * an odd step reads those from the neighbours and writes f*_i into slot i of
 * node x + c_i, where the next even step finds the next pre-collision state
 * in place.  Every slot is read and written by one node only, so no step needs
 * a second buffer.  The same arithmetic as LB_STREAM_AB, bit for bit on tile
 * boxes; in-place contexts run every box as tile items (no row items), gather
 * the chains' spread force inside the fused step, and have no autotuner. */
typedef enum { LB_STREAM_AB = 0, LB_STREAM_AA = 1 } lb_streaming;

typedef struct {
  int32_t nx, ny, nz;      /* nodes per axis, boundary layer included (>= 3 on non-periodic axes) */
  uint32_t periodic_mask;  /* bit a set: axis a (x=0, y=1, z=2) is periodic and has no boundary layer */
} lb_box;

typedef struct {
  int32_t n_boxes;
  const lb_box* boxes;     /* [n_boxes], copied */
  lb_collision collision;
  double tau;              /* shear relaxation time; kinematic viscosity (tau - 1/2)/3; > 1/2 */
  double tau_bulk;         /* MRT bulk relaxation time; bulk viscosity (2/9)(tau_bulk - 1/2) */
  double ghost_rate;       /* MRT relaxation rate of the nine ghost modes (1 = reset to 0) */
  lb_storage storage;
  double rho0;             /* rest density; also the density of the boundary equilibrium */
  int32_t reduce_every;    /* K > 0: record mass and momentum of the interior at t_n, n % K == 0 */
  int32_t fp16_exp;        /* s of LB_STORE_F16DEV, 0 = 10; |h| < 65504 needs |f/w - rho0| < 65504 / 2^s */
  void* stream;            /* hipStream_t; NULL = the null stream */
  /* device allocator hook (e.g. PyTorch's caching allocator); NULL = hipMalloc/hipFree */
  void* (*dev_alloc)(size_t bytes, void* user);
  void (*dev_free)(void* ptr, void* user);
  void* alloc_user;
  const char* tune_cache;  /* path of the autotuner cache (JSON lines: item sizes per box-size
                              class, grid per set of classes), read by lb_init, or NULL */
  int32_t graph_steps;     /* > 0: lb_step replays a HIP graph of this many steps; 0 = eager launches.
                              A multiple of reduce_every lets the graphs leave the check pass out of
                              the steps that are not check steps (captured once per check phase). */
  int32_t streaming;       /* lb_streaming: LB_STREAM_AB (0) or LB_STREAM_AA (1) */
} lb_config;

/* Creates a context: validates the configuration, allocates two population
 * buffers per box (structure of arrays pop[19][nz][ny][nx]) and initialises
 * every interior node to rest, f = w rho0 (Sec. 2 initial condition with u = 0). */
lb_status lb_init(const lb_config* cfg, lb_ctx** out);

/* Prescribes the initial velocity on all interior sites of a box: f(x, 0) =
 * f_eq(rho0, u(x)) (Sec. 2: all sites at t = 0, by local equilibrium).
 * u: host FP64 [nz][ny][nx][3], or NULL for rest.  Only before the first lb_step. */
lb_status lb_set_initial(lb_ctx* ctx, int32_t box, const double* u);

typedef enum { LB_BC_AFFINE = 0, LB_BC_SAMPLED = 1, LB_BC_LEARNED = 2 } lb_bc_mode;

/* Boundary velocity history of one box (Sec. 2-3).  Sample k belongs to step
 * t0 + k*dt; the velocity at step n is linear in time between the samples
 * around it, and stepping to an n outside [t0, t0 + (n_samples-1)*dt] fails
 * with LB_ERR_ARG (never extrapolated).
 *   AFFINE:  data = FP64 [n_samples][9], row-major A; u_b(y) = A (y - x_c),
 *            x_c = ((nx-1)/2, (ny-1)/2, (nz-1)/2).
 *   SAMPLED: data = [n_samples][6][res][res][3], faces -x,+x,-y,+y,-z,+z, entry
 *            [v][u] holds the sample at tangential grid point (u, v) (u = the
 *            lower-index tangential axis), grid point p at node coordinate
 *            p (n-1)/(res-1) (corner aligned); u_b is bilinear on the face.
 *            A node on several faces takes the first face in the order above.
 *            FP64 if data_is_f64, else FP32.  2 <= res <= 8192 and
 *            (largest box edge - 1)(res - 1) < 2^31, else LB_ERR_ARG.
 *   LEARNED: data = a DEVICE pointer the caller owns and keeps alive, FP32
 *            [n_samples][6][res][res][3] laid out as SAMPLED, used as a ring:
 *            step n reads slot ((n - t0) / dt) mod n_samples (and the next slot
 *            for the linear time weight when dt > 1), so stepping never runs
 *            out of samples.  The caller refills slots on the context stream
 *            before the steps that read them (the learned upsampler of
 *            lbnet.h writes one window of dt = 1 slots per call).  Not copied;
 *            FP32/FP16 storage only (LB_ERR_ARG for FP64 contexts).
 * The boundary density is rho0.  Boxes with a boundary layer need a boundary
 * before lb_step (LB_ERR_STATE).  May be replaced between lb_step calls. */
typedef struct {
  lb_bc_mode mode;
  int64_t t0;
  int32_t dt, n_samples, res;
  const void* data;
  int32_t data_is_f64;
} lb_boundary;
lb_status lb_set_boundary(lb_ctx* ctx, int32_t box, const lb_boundary* bc);

/* Appends one bead-spring chain to a box (Sec. 1: beads coupled to the fluid
 * by a Stokes friction coefficient; Sec. 2: centre of mass fixed at the
 * tracer).  Per LB step the fluid velocity at each bead is interpolated
 * trilinearly from the pre-collision moments, the chain is advanced by
 * md_substeps substeps of h = 1/md_substeps (FENE springs F = k r/(1 -
 * r^2/R0^2), exact friction update, positions, optional projection of the
 * centre of mass onto anchor with zero mean velocity), and the friction
 * impulse is spread back with the same trilinear weights.  pos: host FP64
 * [n_beads][3] in lattice node coordinates; vel: [n_beads][3] or NULL (zero).
 * 1 <= n_beads <= 256.  Only before the first lb_step. */
typedef struct {
  int32_t n_beads, md_substeps, fix_com;
  double zeta, mass, fene_k, fene_r0, anchor[3];
} lb_chain;
lb_status lb_couple_chain(lb_ctx* ctx, int32_t box, const lb_chain* chain, const double* pos,
                          const double* vel);

/* Accelerated-frame body force of one box (Sec. 2: in the frame of the
 * tracer, which moves with velocity v(t), the transformed field w = u - v
 * obeys the Navier-Stokes equation with the extra force density rho times
 * -dv/dt).  accel: host FP64 [n_samples][3], the tracer acceleration dv/dt in
 * lattice units (velocity per step) at steps t0 + k dt, linear in time
 * between samples; stepping outside [t0, t0 + (n_samples-1) dt] fails with
 * LB_ERR_ARG (no extrapolation).  Every interior node then receives the force
 * density -rho(x, t_n) a(t_n), rho its pre-collision density, through the
 * collision's forcing, on top of the chains' spread force.  n_samples = 0
 * (accel may be NULL) removes it.  Copied; may be replaced between lb_step
 * calls.  While any box has one, the steps run the extended collision. */
lb_status lb_set_body_force(lb_ctx* ctx, int32_t box, int64_t t0, int32_t dt, int32_t n_samples,
                            const double* accel);

/* Sub-volume history files.  The paper couples its two scales through data
 * on disk (Sec. 1): the velocity of the sub-volume around the tracer, stored
 * during the coarse run, Galilei transformed into the tracer frame and
 * linearly interpolated onto the fine lattice (Sec. 2).  Format (little
 * endian), version 1:
 *   char    magic[8]   "LBSUBVOL"
 *   int32   version    1
 *   int32   R          sample-grid points per edge (2..1024)
 *   int32   n_samples
 *   int32   dt         LB steps between samples
 *   int64   t0         LB step of the first sample
 *   int32   flags      bit 0: tracer accelerations follow the velocities
 *   int32   reserved   0
 *   float32 w[n_samples][R][R][R][3]   tracer-frame velocity in lattice
 *                                      units, index [z][y][x][component]
 *   float64 accel[n_samples][3]        (flags bit 0) tracer acceleration
 *                                      dv/dt in lattice units per step
 * Grid point p of an axis lies at node coordinate p (n - 1)/(R - 1) of the box
 * (corner aligned).  lb_load_subvolume reads a file for one box and applies
 * what `what` asks for: LB_SUBVOL_BOUNDARY -- the six faces of the grid as a
 * SAMPLED boundary history (lb_set_boundary); LB_SUBVOL_INITIAL -- sample 0
 * interpolated trilinearly (FP64) onto every node as the initial field
 * (lb_set_initial; only before the first lb_step); LB_SUBVOL_BODY -- the
 * accelerations as the box's body force (lb_set_body_force).  A malformed or
 * truncated file gives LB_ERR_ARG and changes nothing. */
enum { LB_SUBVOL_INITIAL = 1, LB_SUBVOL_BOUNDARY = 2, LB_SUBVOL_BODY = 4 };
lb_status lb_load_subvolume(lb_ctx* ctx, int32_t box, const char* path, int32_t what);

/* Thermal fluctuations at temperature kT (k_B T in lattice units), for the
 * Stokes-friction coupling of beads and fluid the paper builds on (Sec. 1)
 * in its fluctuating form: every relaxed MRT mode k >= 4 gains the noise
 * sqrt(mu rho b_k (1 - gamma_k^2)) r_k, mu = 3 kT, gamma_k its relaxation
 * factor and b_k its norm, and every bead's exact friction update over a
 * substep h gains the Ornstein-Uhlenbeck kick sqrt(kT/m (1 - e^{-2 zeta h/m}))
 * r.  The r are uniform numbers of mean 0 and variance 1 from the
 * counter-based generator Philox4x32-10 under the 64-bit key `seed`, counter
 * (node index (z ny + y) nx + x, box, step, draw 0..3) for the fluid and
 * (bead index among the box's beads, box, step, 16 + substep) for the beads,
 * so a run is reproducible bit for bit.  MRT contexts only (LB_ERR_ARG
 * otherwise); kT = 0 switches it off.  Only before the first lb_step. */
lb_status lb_set_thermal(lb_ctx* ctx, double kT, uint64_t seed);

/* Advances every box by n_steps (asynchronous on the context stream). */
lb_status lb_step(lb_ctx* ctx, int32_t n_steps);

typedef enum {
  LB_F_RHO = 0,       /* FP64 [nz][ny][nx]; boundary nodes read rho0 */
  LB_F_U = 1,         /* FP64 [nz][ny][nx][3], u = j/rho; boundary nodes read 0 */
  LB_F_POP = 2,       /* FP64 [19][nz][ny][nx] pre-collision f; boundary nodes read w_i rho0 */
  LB_F_BEAD_POS = 3,  /* FP64 [beads of the box][3], chains in coupling order */
  LB_F_BEAD_VEL = 4,  /* FP64 [beads of the box][3] */
  LB_F_MASS_MOM = 5,  /* FP64 [5]: step of the latest check, M, Px, Py, Pz */
  LB_F_STEP = 6,      /* int64 [1]: current step (the context's, box ignored) */
  LB_F_POP_DEV = 7,   /* FP64 [19][nz][ny][nx] pre-collision deviations f_i - w_i rho0: the
                         exact image of the stored state (checkpoints); boundary nodes read 0 */
  LB_F_BEAD_REL = 8,  /* FP64 [beads][3] bead position minus its chain's anchor, as stored
                         (exact image; checkpoints) */
  LB_F_VORT = 9       /* FP64 [nz][ny][nx] vorticity magnitude |curl u| (see lb_vorticity) at
                         the nodes whose six axis neighbours are interior; 0 elsewhere */
} lb_field;

/* Copies a field of one box at the current step to dst (host memory, or
 * device memory when dst_on_device).  Synchronises first; a latched device
 * error is returned after the copy (the data are those of the last good step). */
lb_status lb_read_fields(lb_ctx* ctx, int32_t box, lb_field field, void* dst, size_t dst_bytes,
                         int32_t dst_on_device);

/* Pre-collision populations of selected interior nodes: xyz = host int32
 * [n][3], out = host FP64 [n][19]. */
lb_status lb_read_sites(lb_ctx* ctx, int32_t box, int32_t n, const int32_t* xyz, double* out);

/* Vorticity of the fine box, the quantity the paper compares with the DNS
 * (Sec. 3, Figs. 1-2: the vorticity magnitude averaged over control volumes
 * around the tracer).  |omega| = |curl u| of u = j/rho at the current step
 * (the pre-collision moments, as LB_F_U), each derivative the second-order
 * central difference (u_c(q + e_a) - u_c(q - e_a)) / 2, summed in FP64.
 * vol: host int32 [n_vol][6], each control volume's inclusive node range lo
 * x, y, z then hi x, y, z; every node of it needs its six axis neighbours in
 * the interior (on walled axes 2 <= lo <= hi <= n-3), else LB_ERR_ARG.
 * mean: host FP64 [n_vol], the average of |omega| over each volume.
 * Synchronises. */
lb_status lb_vorticity(lb_ctx* ctx, int32_t box, int32_t n_vol, const int32_t* vol, double* mean);

/* Allocation-free variant of lb_read_sites, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid allocation): the same result, with the site list and the
 * output staged in a static device array of the library instead of buffers
 * it allocates per call.  At most 32768 sites per call (LB_ERR_ARG beyond;
 * the array takes about 5.1 MiB per GPU the library runs on, until the
 * process ends).  Needs a context whose device tables exist (it has stepped,
 * or been read by lb_read_sites or lb_read_fields, once; else LB_ERR_STATE)
 * and its own device current (else LB_ERR_STATE).  Every context on one GPU
 * shares that GPU's array: calls that overlap on one GPU (other host threads)
 * race.  No hipMalloc, hipFree or other allocation. */
lb_status lb_read_sites_noalloc(lb_ctx* ctx, int32_t box, int32_t n, const int32_t* xyz,
                                double* out);

/* Restores state for resume: LB_F_POP or LB_F_POP_DEV (FP64 [19][nz][ny][nx],
 * interior used; LB_F_POP_DEV round-trips bit for bit in every storage mode),
 * LB_F_BEAD_REL (FP64 [beads][3], exact),
 * LB_F_BEAD_POS / LB_F_BEAD_VEL (FP64 [beads][3]), LB_F_STEP (int64 [1]).
 * Only before the first lb_step of the context. */
lb_status lb_write_state(lb_ctx* ctx, int32_t box, lb_field field, const void* src, size_t bytes);

/* Waits for queued work and returns a latched device error, if any. */
lb_status lb_sync(lb_ctx* ctx);

/* Times candidate tile shapes and persistent-grid sizes of the fused kernel on
 * the context's own buffers (idempotent trial launches that do not advance
 * the state), keeps the fastest and records it in lb_config.tune_cache. */
lb_status lb_autotune(lb_ctx* ctx, int32_t trials);

/* Averages of the last lb_step call: [0] ms per step of the whole step, [1] ms
 * per launch of the fused collide-stream kernel, [2] ms per step of the
 * kernels that precede it (x-face boundary velocities and chains; 0 if
 * neither), [3] algorithmic bytes per collide-stream launch (2*19*bytes per
 * population per interior node).  Steps launched one by one are timed with
 * HIP events on the context stream; inside graph-replayed chunks the kernels
 * themselves record the device wall clock at their start (one store by the
 * first thread of the first workgroup), so each figure runs from the start of
 * one kernel to the start of the next.  Requires lb_set_timing(ctx, 1) before
 * the lb_step. */
lb_status lb_set_timing(lb_ctx* ctx, int32_t on);
lb_status lb_get_timing(lb_ctx* ctx, double out[4]);

/* Practical HBM ceiling: copies a device buffer of `bytes` (rounded down to a
 * multiple of 16) with 16-byte loads and stores, each workgroup streaming its
 * own contiguous 256 KiB chunk, `iters` times, and returns in
 * gbs the measured (read + write) bytes per second / 1e9.  Allocates and frees
 * its two buffers with hipMalloc; runs on the current device's null stream. */
lb_status lb_copy_probe(size_t bytes, int32_t iters, double* gbs);

/* Independent HBM ceiling: the runtime's own device-to-device copy
 * (hipMemcpyAsync) of `bytes` between two hipMalloc buffers, `iters` times,
 * timed with HIP events on the null stream of the current device; returns
 * in gbs the (read + write) bytes per second / 1e9.  Allocates and frees its
 * two buffers. */
lb_status lb_memcpy_probe(size_t bytes, int32_t iters, double* gbs);

/* Description of the chosen launch configuration (tile shapes, grid size). */
const char* lb_describe(const lb_ctx* ctx);
const char* lb_last_error(const lb_ctx* ctx);
void lb_free(lb_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
