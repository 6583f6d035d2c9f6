/*
 * ddmpm — differentiable MLS-MPM sand simulation on one MI355X (gfx950).
 *
 * C interface of libddmpm.so.  The library simulates granular material with
 * the moving-least-squares material point method and returns exact reverse-mode
 * gradients of a surface loss with respect to material and skill parameters,
 * as set out in DDBot (arXiv 2510.17335):
 *   - the problem: a state s, an action trajectory a(theta) from the digging
 *     skill and deterministic dynamics s' = f(s, a) (Sec. III-A, "Problem
 *     definition"), the objective J(theta) = r(o', g) and its gradient
 *     dr/dtheta by the chain rule of Eq. grad-chain (Sec. III-E);
 *   - the dynamics: the MLS-MPM sub-step of Algorithm 1 (Sec. III-A) with the
 *     SVK-Hencky energy (Eqs. SVK, piola), Drucker-Prager plasticity (Eq. DP),
 *     sigma = P' F'^T / det F' with det F' := 1, a kinematic shovel with
 *     signed-distance contact and Coulomb friction, and container walls;
 *   - the skill: four phases (Eqs. d1 .. delta_d4, Algorithm 2) with free
 *     insert depth, rotate angle and push distance;
 *   - the loss: the height-map distance of Eq. hm (squared) plus a scoop-mass
 *     term.
 *
 * Conventions
 *   Frame: y is up, the domain is [0,1]^dim, the grid has n_grid nodes per
 *   axis (dx = 1/n_grid); the paper's (x, y, z) with z up maps to (x, z, y).
 *   Memory: every device pointer is caller-owned.  ddm_create takes one
 *   device workspace of the size ddm_workspace_query reports and never
 *   allocates device memory; the context itself is a host object owned by
 *   the library.  Host arrays passed in are copied before the call returns.
 *   Streams: a context is bound to one HIP stream; all calls enqueue work on
 *   it and return without waiting, except ddm_validate_config,
 *   ddm_workspace_query, ddm_check, ddm_read_* and ddm_destroy.  A context is
 *   not thread-safe.
 *   Errors: every call returns a ddm_status; nothing throws across the
 *   interface.  Errors found on the device (NaN, a particle whose stencil
 *   leaves the grid, clamped singular values) are latched in a device word and
 *   reported by ddm_check.
 *   Precision: DDM_F32 or DDM_F64 for all particle and grid arithmetic; the
 *   parameter-gradient accumulators are always FP64.
 *   Particle state layout (ddm_get_state / ddm_set_state): structure of
 *   arrays [2*dim + 2*dim*dim][padded_particles] of 4-byte (DDM_F32) or
 *   8-byte (DDM_F64) elements, rows x[dim], v[dim], C[dim*dim],
 *   G[dim*dim] = F - I (the deformation gradient minus the identity, so that
 *   small strains keep their precision; matrices row-major).  In DDM_F32
 *   contexts the x rows are unsigned 32-bit fixed point, x = value * 2^-32;
 *   in DDM_F64 they are doubles.  Instance i owns columns
 *   [ddm_instance_offset(i), + n_particles), each instance's range padded to
 *   a multiple of 256 columns.
 */
#ifndef DDMPM_H
#define DDMPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum ddm_status {
  DDM_OK = 0,
  DDM_EINVAL = 1,   /* bad configuration or parameter (message via ddm_last_error) */
  DDM_ENOMEM = 2,   /* workspace too small */
  DDM_EDEVICE = 3,  /* a HIP call failed */
  DDM_ENAN = 4,     /* NaN or Inf in the state or a gradient (ddm_check) */
  DDM_EDOMAIN = 5,  /* a particle's B-spline stencil left the grid (ddm_check) */
  DDM_ESTATE = 6    /* call out of order, e.g. backward without a recorded rollout */
} ddm_status;

typedef enum ddm_precision { DDM_F32 = 0, DDM_F64 = 1 } ddm_precision;

/* Problem description shared by all instances of a context. */
typedef struct ddm_config {
  int32_t dim;              /* 2 or 3 */
  int32_t n_grid;           /* nodes per axis, power of two, 16..256 */
  int32_t bound;            /* sticky wall layers on every face (nodes with index < bound
                               or >= n_grid - bound get zero velocity) */
  int32_t precision;        /* ddm_precision */
  int32_t n_sub;            /* sub-steps per skill action (Sec. III-A, "Actions") */
  int32_t shovel;           /* 1: kinematic shovel (3D only), 0: none */
  int32_t hm_res;           /* height-map pixels per axis (40 in the paper) */
  int32_t region_sign;      /* side of the blade holding the scoop region: +1 or -1 */
  double gravity;           /* acceleration along y [m/s^2] */
  double ppc;               /* particles per cell: particle volume V_p = dx^dim / ppc */
  double shovel_half[3];    /* blade half extents along (width z, normal, pointing) [m] */
  double contact_skin;      /* nodes closer than this to the blade are in contact [m] */
  double shovel_mu;         /* Coulomb friction coefficient blade/material */
  double v_lin;             /* skill linear speed v_l [m/s] */
  double v_ang;             /* skill angular speed v_w [rad/s] */
  double d_lift;            /* phase-4 lift distance d4 [m] */
  double hm_origin[2];      /* (x, z) corner of the height-map window [m] */
  double hm_size;           /* window edge [m] */
  double hm_offset;         /* stencil offset r_p of the height map [m] */
  double region_depth;      /* thickness of the scoop region in front of the blade [m] */
  double m_target;          /* target scoop mass [kg] */
  double m_ref;             /* mass normalisation [kg] */
  double w_mass;            /* weight of the scoop-mass term */
  double w_hm;              /* weight of the height-map term */
  int32_t checkpoint_every; /* K: snapshot interval of ddm_rollout (>= 1) */
  int32_t max_steps;        /* longest rollout the workspace is sized for */
  int32_t sort_every;       /* R: particles are re-binned (sorted by cell) every R sub-steps, and
                               always after ddm_init_state / ddm_set_state and at every
                               checkpoint of a recorded rollout; 0 = only then */
  int32_t skill_unrounded;  /* 1: the per-action steps of skill phases 1 and 4 divide by the
                               real-valued T_1^float, T_4^float (Sec. III-B, the alternative
                               mapping; the gradient flows through them); 0: by the rounded T_1, T_4 */
  int32_t particle_contact; /* 1: the particle collision of Algorithm 1 after G2P: a particle whose
                               position is within contact_skin of the blade gets the blade's Coulomb
                               contact, one in the wall layers (closer than bound cells to a face)
                               gets zero velocity; 0: grid collision only */
  int32_t record_segments;  /* how many checkpoint segments the workspace can hold whole for the
                               reverse pass (the state, pre-update grid, stress and binning of every
                               sub-step of a segment); 0 counts as 1.  ddm_rollout runs its last
                               record_segments segments straight into these buffers and
                               ddm_backward replays only the segments before them from their
                               checkpoints: fewer replays for more memory.  Each
                               adds about K (S_p n_total + grid + stress) bytes to the
                               workspace; capped at the segments of a max_steps rollout */
  double w_emd;             /* weight of the earth mover's distance (Eq. emd) between the surface
                               observation and the target set by ddm_set_emd_target; 0 = off;
                               dim 3 only */
  int32_t tile_workgroups;  /* workgroups of the P2G tile kernel: 0 = about one per occupied tile;
                               n > 0 = a persistent launch of n workgroups that take the next tile
                               from a counter in the workspace as they finish one (best near the
                               co-resident count); ddm_autotune chooses it.  The G2P adjoint, the
                               other tile kernel, runs one workgroup per tile */
  int32_t grid_record_blocks; /* capacity of the record of one sub-step's pre-update grid in the
                               segment buffers, in blocks of 4^dim nodes over all instances: the
                               record keeps the active blocks only (those within one tile of an
                               occupied tile).  0 = every block of every instance (no limit).  A
                               smaller capacity shrinks each segment set by K (blocks - capacity)
                               4^dim 4 element-size bytes; a recorded sub-step with more active
                               blocks than that sets device error bit 4 and ddm_check then reports
                               DDM_ENOMEM (the gradient of that pass is not valid) */
  int32_t deterministic;    /* 1: every result (states, grids, loss, gradients, pose and material
                               adjoints) is bitwise the same from run to run and for any
                               tile_workgroups: the particles are binned before every sub-step
                               (sort_every is then ignored), a cell's particles in the order of their
                               ids (so that a state set with ddm_set_state continues bitwise as the
                               uninterrupted run), the LDS windows of the tile kernels add
                               their cells' contributions in a fixed order (cells in 3^dim residue
                               classes, one class at a time), the G2P adjoint stages its windows and
                               the grid adjoint's input sums them in a fixed order, and every
                               reduction over particles or grid blocks sums per-workgroup partials
                               in index order (no floating-point atomics).  Slower (about 4x the
                               pass time), for debugging and reproducibility; the sums of
                               ddm_diagnostics and the 2-norms of the adjoint-growth record stay
                               unordered, and the normalisation treatment (whose 2-norm is reduced
                               with atomics) is rejected.  0: the fast unordered sums */
} ddm_config;

/* One simulation instance: material, skill and time step. */
typedef struct ddm_instance {
  int64_t n_particles;      /* particles of this instance (> 0) */
  double E;                 /* Young's modulus [Pa] (> 0) */
  double nu;                /* Poisson's ratio, in (-1, 0.5) */
  double phi_deg;           /* friction angle [deg], in (0, 90) */
  double rho;               /* density [kg/m^3] (> 0) */
  double cohesion;          /* [Pa] (>= 0); 0 is the paper's cohesionless sand */
  double depth;             /* skill: insertion distance d2 [m] */
  double angle_deg;         /* skill: rotation phi1 [deg] */
  double push;              /* skill: push distance d3 [m] */
  double dt;                /* sub-step [s] (> 0) */
  double tip0[3];           /* initial blade tip [m] */
  double displace;          /* skill: phase-1 displacement d1 along x [m] (Eq. d1; 0 = theta_displace 0) */
  double push_angle_deg;    /* skill: push angle phi3 [deg] (Eq. d3; 180 = theta_push_angle 0) */
} ddm_instance;

/* Differentiable inputs per instance, in the order of every gradient output:
 * E, nu, phi_deg, rho, depth, angle_deg, push, displace, push_angle_deg. */
#define DDM_N_PARAMS 9

/* Sizes reported by ddm_workspace_query. */
typedef struct ddm_sizes {
  size_t workspace_bytes;   /* device bytes ddm_create needs */
  size_t state_bytes;       /* bytes of one instance-concatenated particle state */
  int64_t padded_particles; /* particle slots after per-instance padding */
} ddm_sizes;

typedef struct ddm_ctx ddm_ctx;

/* Device-side error report (ddm_check). */
typedef struct ddm_device_error {
  uint32_t flags;           /* bit 0: NaN/Inf, bit 1: stencil left the grid, bit 2: sigma clamped,
                               bit 3: EMD term set to 0: more observed points than targets, or
                               non-finite distances, bit 4: a recorded sub-step had more active
                               grid blocks than grid_record_blocks */
  uint32_t first_instance;  /* instance of the first flagged particle */
  uint64_t clamp_count;     /* singular values clamped to 1e-6 since the last reset */
} ddm_device_error;

/* Checks a configuration and instance list without touching a device.
 * Returns DDM_EINVAL with a message in msg (if msg_len > 0) on: dim not 2/3,
 * n_grid not a power of two in [16, 256], bound out of [0, n_grid/4], shovel
 * with dim 2, E <= 0, nu outside (-1, 0.5), phi outside (0, 90) deg, rho <= 0,
 * cohesion < 0, dt <= 0, n_particles <= 0, checkpoint_every < 1. */
ddm_status ddm_validate_config(const ddm_config* cfg, int32_t n_inst, const ddm_instance* inst,
                               char* msg, size_t msg_len);

/* The blade pose of every sub-step for one instance's skill (Sec. III-B,
 * Eqs. d1 .. delta_d4, Algorithm 2, spread over n_sub sub-steps as in
 * Algorithm 1): pose_out[n_steps][8] = tip xyz, psi, velocity xyz, omega (host
 * memory, build frame, y up), and, if jac_out is not NULL, its Jacobian
 * jac_out[n_steps][8][5] with respect to (depth, angle_deg, push, displace,
 * push_angle_deg).  This is the table the library uploads at ddm_create; host
 * only, for inspection and tests.  DDM_EINVAL for NULL pointers or
 * n_steps < 1. */
ddm_status ddm_skill_pose_table(const ddm_config* cfg, const ddm_instance* inst, int32_t n_steps,
                                double* pose_out, double* jac_out);

/* Device workspace needed for cfg and these instances (host only). */
ddm_status ddm_workspace_query(const ddm_config* cfg, int32_t n_inst, const ddm_instance* inst,
                               ddm_sizes* out);

/* Creates a context on the current HIP device, bound to `stream` (a
 * hipStream_t, or NULL for the default stream).  `workspace` is caller-owned
 * device memory of at least workspace_bytes (256-byte aligned); the context
 * uses it until ddm_destroy.  Builds the per-instance skill pose tables
 * (Eqs. d1 .. delta_d4, Algorithm 2) on the host and uploads them. */
ddm_status ddm_create(const ddm_config* cfg, int32_t n_inst, const ddm_instance* inst,
                      void* workspace, size_t workspace_bytes, void* stream, ddm_ctx** out);

/* Replaces the per-instance parameters (material, skill, dt, tip0) of a
 * context for the next pass, for optimiser loops and parameter sweeps that
 * reuse one workspace (Sec. III-D: the parameters change every iteration, the
 * problem does not).  n_inst and every n_particles must equal those given to
 * ddm_create.  Recomputes and uploads the instance constants and the pose
 * tables with synchronous copies, after waiting for the context's stream.
 * A recorded rollout and its loss are dropped; a graph captured by ddm_pass
 * stays valid and uses the new values.  Errors: DDM_EINVAL as
 * ddm_validate_config, or for a changed count. */
ddm_status ddm_set_instances(ddm_ctx* ctx, int32_t n_inst, const ddm_instance* inst);

/* Initial particle positions, device pointer to x0[n_total][dim] row-major in
 * the context's precision, instances concatenated in order.  Sets v = 0,
 * C = 0, F = I (the flattened bed at rest, Sec. III-A), resets the step
 * counter, the recorded rollout and the device error word. */
ddm_status ddm_init_state(ddm_ctx* ctx, const void* x0_dev);

/* Advances every instance by n_steps sub-steps (Algorithm 1), no recording. */
ddm_status ddm_step(ddm_ctx* ctx, int32_t n_steps);

/* Runs n_steps sub-steps from the current state and records a snapshot every
 * checkpoint_every steps, so that ddm_backward can replay the rollout; the
 * last record_segments checkpoint segments are recorded whole (every
 * sub-step's state, grids, stress and binning) and need no replay.  The
 * steps and results are those of ddm_step.  DDM_EINVAL when the rollout would
 * pass max_steps. */
ddm_status ddm_rollout(ddm_ctx* ctx, int32_t n_steps);

/* Loss of every instance at the current state: height map of Eq. hm (40x40,
 * five-point stencil, max height) against target_hm_dev
 * ([n_inst][hm_res^(dim-1)] in double, device), plus the scoop-mass term,
 * plus w_emd times the earth mover's distance of Eq. emd when w_emd != 0: the
 * surface observation (in each pixel of the height-map window the highest
 * particle whose own (x, z) lies in it, Sec. III-A) against the target point
 * cloud of ddm_set_emd_target, under the cheapest one-to-one assignment
 * (exact: the Hungarian method).  Writes loss_dev[n_inst] (double, device).
 * DDM_ESTATE when w_emd != 0 and no target was set. */
ddm_status ddm_loss(ddm_ctx* ctx, const double* target_hm_dev, double* loss_dev);

/* Target surface point clouds of the EMD term (Eq. emd): points_dev
 * [n_inst][m][3] (double, device, build frame, y up), copied into the
 * workspace on the context's stream; m in [1, hm_res^2].  Kept until replaced.
 * Errors: DDM_EINVAL for NULL, m out of range, or dim != 3. */
ddm_status ddm_set_emd_target(ddm_ctx* ctx, const double* points_dev, int32_t m);

/* Reverse pass of the last ddm_rollout + ddm_loss: with dloss_dev[n_inst]
 * (double, device) the upstream gradient, writes grad_dev[n_inst][DDM_N_PARAMS]
 * (double, device) = d(sum_i dloss_i * loss_i) / d(E, nu, phi_deg, rho, depth,
 * angle_deg, push, displace, push_angle_deg); the skill entries are zero
 * without a shovel.  Recomputes each checkpoint segment forward (except those
 * the rollout recorded whole), then runs the adjoint of every sub-step in
 * reverse (Eq. po/pa).  A second call replays every segment.  DDM_ESTATE
 * without a preceding ddm_rollout and ddm_loss. */
ddm_status ddm_backward(ddm_ctx* ctx, const double* dloss_dev, double* grad_dev);

/* One full pass of a gradient-based optimiser or line search (Sec. III-D,
 * system identification in Sec. IV-B): ddm_init_state(x0_dev),
 * ddm_rollout(n_steps), ddm_loss(target_hm_dev, loss_dev) and
 * ddm_backward(dloss_dev, grad_dev) in one call, with the arguments and
 * outputs of those calls.  use_graph != 0: the pass is captured into a HIP
 * graph on the first call and later calls with the same pointers and n_steps
 * replay it (one launch for the whole pass); other arguments capture afresh.
 * The graph holds only kernels and device-to-device copies.  Timing events are
 * not recorded inside a captured pass.  Errors: those of the four calls;
 * DDM_EINVAL for NULL pointers or n_steps outside [1, max_steps]. */
ddm_status ddm_pass(ddm_ctx* ctx, const void* x0_dev, int32_t n_steps, const double* target_hm_dev,
                    const double* dloss_dev, double* loss_dev, double* grad_dev, int32_t use_graph);

/* Chooses the launch configuration of this context by timing the same
 * forward sub-steps from the current state, after a warm-up round: first the
 * binning interval R (ddm_config.sort_every) in {2, 4, 8, 16, 32}, then, at
 * that R, the workgroup count of P2G (ddm_config.tile_workgroups) in {0
 * (about one per tile), 4, 8, 16 and 32 per compute unit} (the latter are
 * persistent launches that draw tiles from a work queue).  In the
 * deterministic mode R has no effect and only the workgroup count is
 * probed.  The state is
 * restored, and a recorded rollout, its loss and its checkpoints stay valid.
 * With cache_path != NULL, a line "ddmpm dim=.. n_grid=.. prec=.. n_inst=..
 * particles=.. ppc=.. sort_every=R tile_workgroups=W" for this problem is
 * looked up first (no probe when found) and appended after a probe.  The
 * chosen R is written to *sort_every_out (may be NULL) and both values are
 * readable with ddm_get_launch.  Synchronises the stream.  DDM_ESTATE before
 * ddm_init_state.  The results do not depend on R or W beyond the order of
 * floating-point atomic sums (not at all in the deterministic mode). */
ddm_status ddm_autotune(ddm_ctx* ctx, const char* cache_path, int32_t* sort_every_out);

/* The context's current binning interval and tile-kernel workgroup count
 * (either pointer may be NULL). */
ddm_status ddm_get_launch(const ddm_ctx* ctx, int32_t* sort_every, int32_t* tile_workgroups);

/* Copies the current particle state (layout above) of all instances into /
 * from caller device memory of state_bytes.  Particles are exported in their
 * initial order (binning reorders them internally); ddm_set_state takes that
 * order and restarts the binning. */
ddm_status ddm_get_state(ddm_ctx* ctx, void* state_dev);
ddm_status ddm_set_state(ddm_ctx* ctx, const void* state_dev);

/* Binning of the current state without reordering it: keys_dev[padded]
 * receives each slot's cell key inst * (n^dim + 1) + tile * 4^dim +
 * cell-in-tile (4^dim-cell tiles, lexicographic with the last axis fastest,
 * base cell floor(x n - 1/2) per axis; padding slots inst * (n^dim + 1) +
 * n^dim) and perm_dev[padded] the stable sort of the slots by key (uint32,
 * device).  Slots follow the state's internal order, which is the initial
 * order right after ddm_init_state. */
ddm_status ddm_bin_keys(ddm_ctx* ctx, uint32_t* keys_dev, uint32_t* perm_dev);

/* Copies the grid of the last sub-step (per instance, n_grid^dim nodes,
 * 8 values each: m, mv[3], v[3], a) into caller device memory, in the
 * context's precision; a is 1 for a node of an active block (one the grid
 * update processed) and 0 elsewhere, and nodes outside active blocks are
 * zero.  For
 * kernel-level tests.  DDM_ESTATE when no forward sub-step ran since
 * ddm_init_state, ddm_set_state or ddm_backward (the reverse pass reuses the
 * grid buffers). */
ddm_status ddm_get_grid(ddm_ctx* ctx, void* grid_dev);

/* Copies the height map of the last ddm_loss ([n_inst][hm_res^(dim-1)],
 * double) into caller device memory. */
ddm_status ddm_get_heightmap(ddm_ctx* ctx, double* hm_dev);

/* The FP32 elementary functions that the FP32 constitutive update and its
 * adjoint use for ln s = log1p(s^2 - 1)/2, exp(eps') - 1 and the divided
 * differences of the isotropic adjoint (Sec. III-C, Eq. DP, Appendix B):
 * y[i] = log1p(x[i]) (fn 0) or expm1(x[i]) (fn 1), computed on the device
 * exactly as the kernels compute them, for accuracy tests against a
 * reference.  x_dev, y_dev: device float arrays of n elements, caller-owned;
 * asynchronous on `stream` (a hipStream_t, NULL: the default stream); needs
 * no context.  Errors: DDM_EINVAL for fn outside {0, 1}, n < 0, n > 2^40 or a
 * NULL pointer with n > 0; DDM_EDEVICE for a failed launch. */
ddm_status ddm_eval_math(int32_t fn, const float* x_dev, float* y_dev, int64_t n, void* stream);

/* The loss of ddm_loss without a context and without allocating, for callers
 * that cannot allocate device memory (code under stream capture, tight
 * serving loops, harnesses that forbid hipMalloc).  It evaluates the height
 * map of Eq. hm and the scoop-mass term (not the EMD term) for one instance's
 * particle positions x_dev ([inst->n_particles][dim], device, float for
 * DDM_F32 and double for DDM_F64, as ddm_init_state takes them), with the
 * blade at its pose after sub-step final_step of the instance's skill (-1: the
 * initial pose tip0), against target_hm_dev ([hm_res^(dim-1)] double,
 * device), with the same kernels as ddm_loss.  Writes loss_dev[1] and, when
 * hm_dev is not NULL, the height map hm_dev[hm_res^(dim-1)] (double, device).
 * Asynchronous on `stream` (a hipStream_t, NULL: the default stream).
 * Memory: no allocation of any kind.  Every intermediate lives in one static
 * device array of the library, 8 MiB on each device it runs on, held until
 * the process ends; its address is taken on the first call on a device.
 * Calls on one device share that array: calls that overlap on one device
 * (other streams, other threads) race and must be ordered by the caller.
 * Errors: DDM_EINVAL as ddm_validate_config for cfg and inst, for NULL
 * pointers, n_particles above DDM_NOALLOC_MAX_PARTICLES, hm_res^(dim-1) above
 * DDM_NOALLOC_MAX_PIXELS, w_emd != 0, or final_step outside [-1, max_steps);
 * DDM_EDEVICE when the array's address cannot be taken or a launch fails. */
#define DDM_NOALLOC_MAX_PARTICLES 262144
#define DDM_NOALLOC_MAX_PIXELS 4096
ddm_status ddm_loss_noalloc(const ddm_config* cfg, const ddm_instance* inst, int32_t final_step, const void* x_dev,
                            const double* target_hm_dev, double* loss_dev, double* hm_dev, void* stream);

/* Gradient treatments inside the reverse pass (Sec. III-E) and the record of
 * how the adjoints grow backwards in time (Appendix D).
 *   The adjoint of each key variable of a sub-step is treated as one vector
 *   per instance.  Variables: 0 particle positions, 1 particle velocities,
 *   2 particle deformation gradients (the adjoint state of the start of the
 *   sub-step, after its reverse sub-step), 3 grid velocities after the grid
 *   update (once G2P's adjoint is complete), 4 grid momenta and 5 grid masses
 *   as P2G wrote them (once the grid update's adjoint is complete).  Each is
 *   treated where it is complete, before the rest of the reverse pass reads it.
 *   Modes: DDM_TREAT_NONE; DDM_TREAT_CLIP, every element into [-clip, clip];
 *   DDM_TREAT_SCALE, divide the vector by 10^d + delta, d = round(log10(max
 *   |element|)) - oom (halves rounded away from zero), when d > 0;
 *   DDM_TREAT_NORM, divide it by (2-norm + delta).  The paper's values: clip
 *   1e4, oom 4, delta 1e-6.  Treated gradients are not derivatives of the loss.
 *   Record: with stats_dev != NULL (double, device, caller-owned,
 *   [stats_steps][n_inst][6 variables][6], valid until the setting is
 *   replaced), every ddm_backward first zeroes the buffer and then writes, for
 *   each sub-step k < stats_steps of the recorded rollout, the max, min and
 *   2-norm of each vector before the treatment and after it (the values before
 *   it again for DDM_TREAT_NONE).  A vector's max shows a NaN in it.
 *   The setting holds for later ddm_backward and ddm_pass calls; setting it
 *   drops a captured ddm_pass graph.
 *   Errors: DDM_EINVAL for a NULL context, an unknown mode, clip <= 0 with
 *   DDM_TREAT_CLIP, a non-finite oom, delta < 0 or non-finite, stats_steps < 0,
 *   stats_dev and stats_steps > 0 not given together, or DDM_TREAT_NORM in a
 *   deterministic context. */
typedef enum ddm_grad_treatment {
  DDM_TREAT_NONE = 0,
  DDM_TREAT_CLIP = 1,
  DDM_TREAT_SCALE = 2,
  DDM_TREAT_NORM = 3
} ddm_grad_treatment;

ddm_status ddm_set_grad_treatment(ddm_ctx* ctx, int32_t mode, double clip, double oom, double delta,
                                  double* stats_dev, int32_t stats_steps);

/* Kernel timing for measurement: each launch of a selected group is
 * bracketed by HIP events on the context's stream (an event pair costs a few
 * microseconds of stream time, so a timed run selects only the groups it
 * needs).  Groups: 0 P2G, 1 grid update, 2 G2P, 3 binning (keys, sort,
 * gather, tile list), 4 G2P adjoint, 5 grid adjoint, 6 P2G adjoint, 7 grid
 * clears, 8 loss, 9 gradient treatments and their statistics.
 * groups: bit g selects group g; 0 turns timing off; DDM_TIMING_ALL selects
 * every group.  Synchronises the stream and resets the sums.
 * ddm_read_timing synchronises and returns the summed milliseconds and the
 * number of launches of a group since timing was set.
 * Errors: DDM_EINVAL for a NULL context or bits above DDM_TIMING_ALL. */
#define DDM_TIMING_ALL 0x3FF
ddm_status ddm_set_timing(ddm_ctx* ctx, int32_t groups);
ddm_status ddm_read_timing(ddm_ctx* ctx, int32_t group, double* total_ms, int64_t* launches);

/* Synchronises the stream and reads the device error word. */
ddm_status ddm_check(ddm_ctx* ctx, ddm_device_error* out);

/* Per-step diagnostics of the current state, per instance, into out_dev
 * ([n_inst][DDM_N_DIAG] double, device, caller-owned), in this order:
 *   0 particle mass N m_p (m_p = rho dx^dim / ppc),
 *   1-3 momentum sum m_p v_p, 4 kinetic energy sum m_p |v_p|^2 / 2,
 *   5-7 particles whose next constitutive update (on F_tmp = (I + dt C) F of
 *       the current state) takes the return-map case tension/apex, inside the
 *       cone, projection onto the cone (Eq. DP), 8 singular values that update
 *       would clamp,
 *   9 CFL number max_p max_a |v_a| dt / dx,
 *   10 grid mass of the last sub-step's P2G (sum of the nodal masses the grid
 *       update saw; equal to item 0 up to rounding, since each particle's
 *       B-spline weights sum to one), NaN when no sub-step ran since
 *       ddm_init_state, ddm_set_state or ddm_backward.
 * Sums and counts are accumulated in FP64.  Asynchronous on the context's
 * stream.  Errors: DDM_EINVAL for NULL pointers, DDM_ESTATE before
 * ddm_init_state. */
#define DDM_N_DIAG 11
ddm_status ddm_diagnostics(ddm_ctx* ctx, double* out_dev);

/* Sub-steps taken since ddm_init_state. */
int64_t ddm_steps_taken(const ddm_ctx* ctx);

/* First state column of instance i (see the state layout), or -1. */
int64_t ddm_instance_offset(const ddm_ctx* ctx, int32_t i);

/* Releases the host context (the workspace stays the caller's). */
void ddm_destroy(ddm_ctx* ctx);

/* Static description of a status code, and the message of the last failing
 * call on this thread. */
const char* ddm_status_str(ddm_status s);
const char* ddm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DDMPM_H */
