/*
 * crm.h -- C ABI of libcrm: the per-step particle update of the SPH
 * "Continuous Representation Model" for granular media (arXiv 2507.05643,
 * Chrono::CRM) on one AMD Instinct MI355X (gfx950).
 *
 * One call of crm_step advances the soil particles by explicit-midpoint RK2
 * steps (Sec. 2.3) of the SPH-discretised continuity, momentum and Jaumann
 * hypo-elastic stress-rate equations (Sec. 2.2), followed by the cohesive mu(I)
 * return mapping (Sec. 2.4). Rigid bodies are represented by BCE markers whose
 * velocity and stress are extrapolated from the soil (Sec. 2.5.1); the forces
 * and torques the soil exerts on them are returned by crm_get_forces. The
 * neighbour lists are built with the cell-linked list of Sec. 4.1 and kept for
 * ps_freq steps (Alg. 2); with active domains (Sec. 4.2, Alg. 3) only the
 * particles near moving bodies are processed.
 *
 * Conventions for every entry point:
 *   - All pointers passed to the library are HOST pointers; their contents are
 *     copied during the call and the caller keeps ownership.
 *   - Device memory is owned by the library. It is obtained through the
 *     caller's allocator callbacks when given (so that e.g. PyTorch's caching
 *     allocator accounts for it), else with hipMalloc/hipFree.
 *   - A context is bound to one HIP stream (the one given to crm_init) and to
 *     the device current at crm_init; it is not thread-safe.
 *   - Every call returns a crm_status and never throws. CRM_E_INVALID,
 *     CRM_E_NOMEM and CRM_E_STATE leave the context unchanged. CRM_E_DEVICE and
 *     CRM_E_NONFINITE poison the context: later calls return CRM_E_STATE.
 *   - Kernels run asynchronously; a device error surfaces at the next call that
 *     synchronises (crm_get_forces, up to the last step's body sums;
 *     crm_get_state, the debug exports, or a rebuild step).
 *   - Particle ids: the n_soil soil particles of crm_init are ids 0..n_soil-1;
 *     the markers of body b follow in body order (ids n_soil + ...).
 */
#ifndef CRM_H
#define CRM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CRM_ABI_VERSION 4u

typedef enum {
  CRM_OK = 0,
  CRM_E_INVALID = -1,     /* bad argument or parameter */
  CRM_E_NOMEM = -2,       /* an allocation failed */
  CRM_E_DEVICE = -3,      /* a HIP call or kernel failed */
  CRM_E_STATE = -4,       /* context poisoned or call out of order */
  CRM_E_NONFINITE = -5,   /* a body force or torque is not finite */
  CRM_E_UNSUPPORTED = -6  /* valid request this build does not handle */
} crm_status;

/* Artificial viscosity variants of Sec. 2.2 (eqs. artificial_viscosity_*). */
enum { CRM_AV_OFF = 0, CRM_AV_BILATERAL = 1, CRM_AV_UNILATERAL = 2 };

/* Stored form of particle positions. CRM_POS_FP32: FP32 absolute coordinates.
 * CRM_POS_CELL_OFFSET: the integer cell (cell size 2h, from domain_lo) and an
 * FP32 offset inside it, so that motion stays resolved far from the origin
 * (km-scale terrain, Sec. 5); offsets are advanced in FP64 and renormalised into
 * their cell every stage. Requires fewer than 32768 cells along y and z. */
enum { CRM_POS_FP32 = 0, CRM_POS_CELL_OFFSET = 1 };

/* Smoothing kernels (Sec. 4.1; both have support 2h in 3-D). CRM_KERNEL_CUBIC:
 * the cubic spline (Monaghan 1985). CRM_KERNEL_WENDLAND: the quintic Wendland C2
 * kernel (Wendland 1995), W = 21/(16 pi h^3) (1 - q/2)^4 (2q + 1), q = r/h. */
enum { CRM_KERNEL_CUBIC = 0, CRM_KERNEL_WENDLAND = 1 };

typedef struct crm_ctx crm_ctx;

/* Allocator callbacks: return device memory of `bytes` bytes usable on
 * `hip_stream` (or NULL on failure); free memory returned earlier. */
typedef void* (*crm_alloc_fn)(size_t bytes, void* user, void* hip_stream);
typedef void (*crm_free_fn)(void* ptr, void* user, void* hip_stream);

/* Model and solver parameters (SI units). Paper passages:
 *   dx (particle spacing d0), h (smoothing length), dt, gravity: Table 1, Sec. 3;
 *   rho0, E, nu (G = E / (2(1+nu)), K = E / (3(1-2nu))): Sec. 2.1;
 *   mu_s, mu_2, I0, grain_d (d), cohesion (c): Sec. 2.4 (eqs. pcrit, muI, yieldsurf);
 *   av_mode, av_gamma (gamma_a), av_xi_over_h (xi / h): Sec. 2.2;
 *   ps_freq: Sec. 4.1 (persistent neighbour lists);
 *   active_domains, t_delay, grow_G (G), shrink_S (S), shrink_interval (S_I): Sec. 4.2.
 * domain_lo/hi bound the cell grid (cell size 2h); particles outside are
 * binned into the edge cells. bulk_coeff multiplies the bulk term K tr(D) I of
 * the stress rate (1 = the continuum form of eq. stress_rate_hypoelastic).
 * skin = 0: the paper's persistent lists of the pairs within 2h, rebuilt every
 * ps_freq steps (Alg. 2). skin > 0: Verlet lists of the pairs within 2h + skin
 * (cells of that size; active boxes grown by 2h + skin), rebuilt when a
 * processed particle has moved more than skin / 2 since the last rebuild, or
 * after ps_freq steps. Since the kernel vanishes beyond 2h, the sums then equal
 * those over the exact 2h neighbours of every step (up to summation order).
 * activity_scan: the active-domain flags (Sec. 4.2 item 2) are those of a test
 * of every particle against the active boxes; with 0 only the particles that
 * an index of the master store by coarse cell places near a box, and those
 * on the moved list (integrated, or markers of a body that moved, since the
 * index was built), are tested (same flags); with 1 all N are (the paper's
 * pass). moved_cap: entries of the moved list (0: max(16384, N / 32)); the
 * index is rebuilt when the list would overflow, and a rebuild tests all N
 * instead when the last rebuild integrated more than moved_cap / 2 rows. The
 * index takes 4 B per particle and 16 B per coarse cell (8 list cells per
 * axis); with more coarse cells than max(N, 2^20) all N are tested. */
typedef struct {
  uint32_t abi_version;  /* must be CRM_ABI_VERSION */
  uint32_t av_mode;
  double dx, h, dt;
  double gravity[3];
  double rho0, E, nu, mu_s, mu_2, I0, grain_d, cohesion;
  double av_gamma, av_xi_over_h;
  double domain_lo[3], domain_hi[3];
  uint32_t ps_freq;
  uint32_t active_domains;
  double t_delay;
  double grow_G, shrink_S;
  uint32_t shrink_interval;
  uint32_t pos_mode;     /* CRM_POS_FP32 or CRM_POS_CELL_OFFSET */
  double bulk_coeff;
  uint32_t kernel;       /* CRM_KERNEL_CUBIC or CRM_KERNEL_WENDLAND */
  uint32_t activity_scan; /* 0: active-domain flags from an index by coarse cell (default); 1: a scan of all N */
  double skin;           /* Verlet-list skin (m, >= 0), see below */
  int64_t moved_cap;     /* moved-list entries for activity_scan 0 (>= 0; 0: default), see below */
} crm_params;

/* A rigid body: BCE markers fixed in its frame (Sec. 2.5.1: layers at spacing
 * d0, first layer on the collision surface) and an optional active box, an
 * oriented box of half extents active_half centred at the body origin
 * (Sec. 4.2 item 1; all zero = no box). */
typedef struct {
  int64_t n_markers;
  const float* marker_local;  /* 3 * n_markers floats, body frame, copied */
  double active_half[3];
} crm_body_desc;

/* Create a context. pos: 3*n_soil doubles (rounded to FP32 inside); vel: 3*n_soil
 * floats or NULL (zero); sigma: 6*n_soil floats (xx, yy, zz, xy, xz, yz) or
 * NULL (zero); rho: n_soil floats or NULL (rho0). Bodies start at the identity
 * pose with zero velocity until crm_set_bodies is called. alloc/free may both
 * be NULL (hipMalloc/hipFree). hip_stream may be NULL (the null stream).
 * Errors: CRM_E_INVALID (parameters, sizes, NULL where required),
 * CRM_E_NOMEM, CRM_E_DEVICE. On error *out is NULL. */
crm_status crm_init(const crm_params* params, int64_t n_soil, const double* pos, const float* vel,
                    const float* sigma, const float* rho, int32_t n_bodies,
                    const crm_body_desc* bodies, crm_alloc_fn alloc, crm_free_fn free_fn,
                    void* alloc_user, void* hip_stream, crm_ctx** out);

/* Set the state of the bodies (the multibody side's position- and
 * velocity-level state, Sec. 2.5); it stays frozen during crm_step. pos: 3*nb
 * world positions of the body origins; quat: 4*nb unit quaternions (w, x, y, z);
 * linvel, angvel: 3*nb (world frame; NULL = zero); linacc, angacc: 3*nb or NULL.
 * Marker accelerations in the stress extrapolation are a + alpha x r +
 * w x (w x r) when accelerations are given, else the centripetal part only.
 * Errors: CRM_E_INVALID (nb differs from crm_init, NULL pos/quat, non-finite
 * input), CRM_E_STATE. */
crm_status crm_set_bodies(crm_ctx* ctx, int32_t nb, const double* pos, const double* quat,
                          const double* linvel, const double* angvel, const double* linacc,
                          const double* angacc);

/* Materials of the return mapping (Sec. 2.4): for material m, friction
 * mu_s[m], mu_2[m] and cohesion[m] (the other constants stay those of the
 * parameters); material[i] (< n_mat) for each soil particle i. Until called, all
 * soil has one material with the parameters' values. Allowed only before the
 * first step. n_mat <= 256. Errors: CRM_E_INVALID (sizes, ids, values as in
 * crm_init), CRM_E_STATE (after the first step), CRM_E_DEVICE. */
crm_status crm_set_materials(crm_ctx* ctx, int32_t n_mat, const double* mu_s, const double* mu_2,
                             const double* cohesion, const uint16_t* material);

/* Advance n_steps steps (Alg. 3 per step: rebuild when step mod ps_freq == 0,
 * then two RHS evaluations and the return mapping). Enqueued on the context's
 * stream; returns once enqueued, except on rebuild steps, which wait for the
 * particle and neighbour counts. Errors: CRM_E_INVALID (n_steps < 0),
 * CRM_E_NOMEM, CRM_E_DEVICE, CRM_E_STATE. On CRM_E_NOMEM (a growth of the
 * working set or of the neighbour lists failed) the steps before the failing
 * one stay taken (crm_get_counts reports them) and the failing step leaves no
 * trace: the state, the step counter and every later result are those of a
 * context where the allocation never failed, once memory is available. */
crm_status crm_step(crm_ctx* ctx, int32_t n_steps);

/* crm_step for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving or co-simulation loops, harnesses that forbid
 * hipMalloc): the same steps with the same kernels and bit-identical results,
 * but the call allocates nothing. The transient buffers of a step (compaction
 * block counts, the scans' tile totals, the body-force chunk sums) come from
 * one static device array of the library, 16 MiB per device, held on each
 * device the library runs on until the process ends; everything else is the
 * context's memory from earlier calls. So the context must already hold what
 * the steps need: the first step of a context is taken by a call that may
 * allocate (crm_step, crm_cosim_step, crm_record), and when a list rebuild
 * needs a larger working set, neighbour list or force-sum plan the call
 * returns CRM_E_NOMEM with the failing step left out exactly as for a failed
 * allocation in crm_step (a later crm_step grows the buffers and continues
 * bit for bit). A shrink of the working set that the capacity policy asks for
 * waits for a call that may allocate. No graph is captured or replayed and no
 * kernel timing is recorded during the call. Every call on one device shares
 * that device's array and leaves its contents behind (nothing in it needs to
 * start at zero); calls that overlap on one device, from two contexts on
 * different streams or threads, race and must be serialised by the caller.
 * Errors: as crm_step; CRM_E_INVALID if the context's sizes need more scratch
 * than the array holds (the message states both sizes); CRM_E_NOMEM as above. */
crm_status crm_step_noalloc(crm_ctx* ctx, int32_t n_steps);

/* Force (N, world frame) and torque (N m, about the body origin) the soil
 * exerts on each body, from the stage-2 evaluation of the last step
 * (Sec. 2.5.1: sum of marker mass times marker acceleration). force, torque:
 * 3*nb doubles. Waits (by polling) until the stream has written those sums:
 * a step reduces them before its stage 2, which the sums do not depend on, so
 * after a step the call returns while stage 2 still runs, and the caller's
 * next crm_set_bodies and step queue behind it. Errors: CRM_E_INVALID,
 * CRM_E_STATE (no step taken yet), CRM_E_NONFINITE, CRM_E_DEVICE. */
crm_status crm_get_forces(crm_ctx* ctx, int32_t nb, double* force, double* torque);

/* One co-simulation exchange (the FSI loop of Sec. 2.5 with the multibody
 * side on the host): crm_set_bodies with the given states, crm_step(ctx, 1),
 * then crm_get_forces into force and torque; arguments and errors as there.
 * A host loop that calls it once per step makes one library call per step. */
crm_status crm_cosim_step(crm_ctx* ctx, int32_t nb, const double* pos, const double* quat,
                          const double* linvel, const double* angvel, const double* linacc,
                          const double* angacc, double* force, double* torque);

/* State of all n_total particles by id (soil, then markers: world positions,
 * extrapolated velocity and stress of their last evaluation, rho0). Any
 * pointer may be NULL. pos: 3n doubles; vel: 3n; sigma: 6n; rho: n floats.
 * Synchronises. */
crm_status crm_get_state(crm_ctx* ctx, double* pos, float* vel, float* sigma, float* rho);

/* Overwrite the soil state (ids 0..n_soil-1); any pointer may be NULL. Takes
 * effect from the next step; the next step rebuilds the neighbour lists.
 * Positions must be finite (CRM_E_INVALID otherwise). Velocities, stresses and
 * densities are taken as given: a non-finite value spreads through the step
 * and surfaces as CRM_E_NONFINITE at the next force read (crm_get_forces,
 * crm_cosim_step) once it reaches a body. */
crm_status crm_set_state(crm_ctx* ctx, const double* pos, const float* vel, const float* sigma,
                         const float* rho);

/* Checkpoints for an exact restart: the master state of every particle in its
 * stored form (bit for bit, cell-offset positions included), the step counter,
 * the body states of the last crm_set_bodies and the materials. Taken where
 * the next step rebuilds the neighbour lists (step mod ps_freq = 0, or after
 * crm_init, crm_set_state or a restore), so that a context restored from it
 * continues bit-identically: its first step rebuilds the same lists from the
 * same state (Alg. 2 and 3 depend only on the state, the step counter and the
 * bodies). crm_checkpoint_bytes: the size of a checkpoint of ctx.
 * crm_save_checkpoint: writes it into buf (host, `bytes` >= that size);
 * synchronises; errors: CRM_E_INVALID (NULL or small buffer), CRM_E_STATE (not
 * at a list rebuild), CRM_E_DEVICE. crm_load_checkpoint: restores a
 * checkpoint into a context created with the same particles, bodies and
 * parameters (sizes and position form are checked); the next step rebuilds.
 * Errors: CRM_E_INVALID (not a checkpoint, or of another configuration: the
 * context is unchanged), CRM_E_DEVICE. */
crm_status crm_checkpoint_bytes(crm_ctx* ctx, size_t* bytes);
crm_status crm_save_checkpoint(crm_ctx* ctx, void* buf, size_t bytes);
crm_status crm_load_checkpoint(crm_ctx* ctx, const void* buf, size_t bytes);

/* Sizes: out[0] n_total, out[1] n_soil, out[2] processed particles N_{a+e} of
 * the last rebuild, out[3] active soil rows, out[4] processed marker rows,
 * out[5] stored neighbour slots (soil rows + marker rows, including the
 * padding of each wave's block to its longest list), out[6]
 * working-array capacity, out[7] steps taken, out[8] number of cells M,
 * out[9] rebuilds done. out: 10 int64. */
crm_status crm_get_counts(crm_ctx* ctx, int64_t* out);

/* Export of the last rebuild for bit-exact checks (Sec. 4.1 steps 1-4):
 * sorted_ids: N_{a+e} particle ids in cell-sorted order (inside a cell by
 * the stored x coordinate, ties by id);
 * cell_start: M + 1 values, cell_start[c] = first sorted position of cell c
 * (cellEnd[c] = cell_start[c + 1]); rows: ids of the particles that own a list
 * (active soil, then processed markers), off: rows + 1 offsets, nbr: entries
 * as particle ids (order within a row unspecified), cap: capacity of nbr. A
 * soil row lists every particle within 2h (itself included); a marker row
 * lists only the soil particles within 2h, the only ones its extrapolation
 * and force sums use.
 * flags: n_total activity flags (0 inactive, 1 extended, 2 active).
 * Any pointer may be NULL. Errors: CRM_E_INVALID if cap is too small,
 * CRM_E_STATE before the first rebuild. Synchronises. */
crm_status crm_debug_export(crm_ctx* ctx, int32_t* sorted_ids, uint32_t* cell_start, int32_t* rows,
                            int64_t* off, int32_t* nbr, int64_t cap, uint8_t* flags);

/* Reverse mode, part 1 (the step map of Sec. 2.3 over the rates of Sec. 2.2,
 * the BCE of Sec. 2.5.1 and the return mapping of Sec. 2.4, differentiated
 * with the neighbour lists and activity held fixed). Advances n_steps >= 1
 * steps exactly as crm_step does and keeps what the reverse sweep needs: the
 * master state at each list rebuild of the run and the body table (bodies are
 * frozen during the call, as in crm_step). Device memory: 64 bytes per
 * particle per list rebuild of the run. The record must start at a list
 * rebuild (step mod ps_freq = 0, or the first step after crm_init or
 * crm_set_state). A later crm_step or crm_set_state discards the record.
 * Errors: CRM_E_INVALID, CRM_E_UNSUPPORTED (active domains on), CRM_E_STATE
 * (not at a list rebuild), CRM_E_NOMEM, CRM_E_DEVICE. */
crm_status crm_record(crm_ctx* ctx, int32_t n_steps);

/* Body forces and torques of every step of the last crm_record (those
 * crm_get_forces would have returned after each step), in the layout of the
 * adjoint's force seeds: force, torque: 3 nb doubles per recorded step, step
 * by step (host, written). The forward values of the functional that
 * crm_adjoint differentiates (Sec. 2.5.1 body forces). Synchronises.
 * Errors: CRM_E_INVALID (NULL pointer with nb > 0), CRM_E_STATE (no valid
 * record), CRM_E_NONFINITE, CRM_E_DEVICE. */
crm_status crm_record_forces(crm_ctx* ctx, double* force, double* torque);

/* Reverse mode, part 2: the vector-Jacobian product of the recorded run for
 * the linear functional
 *   L = sum_i (lam_pos_i . x_i + lam_vel_i . u_i + lam_sigma_i . s_i + lam_rho_i rho_i)
 *       + sum_k sum_b (lam_force_kb . F_kb + lam_torque_kb . T_kb)
 * of the soil state at the end of the run and of the body forces and torques
 * of each recorded step k (those crm_get_forces would have returned after it).
 * Seeds (host, any may be NULL = zero): lam_pos 3 n_soil doubles, lam_vel
 * 3 n_soil, lam_sigma 6 n_soil (xx, yy, zz, xy, xz, yz), lam_rho n_soil floats,
 * by particle id; lam_force, lam_torque 3 nb doubles per recorded step, step
 * by step. Outputs (host, any may be NULL): dL/d(state at the start of the
 * run) in the same layouts, and out_params = (dL/dE, dL/dnu, then dL/dmu_s,
 * dL/dmu_2, dL/dcohesion for each material), 2 + 3 n_mat doubles (n_mat = 1
 * without crm_set_materials). At a branch of the step (unilateral artificial
 * viscosity, the return-mapping cases, the mu(I) cases) the derivative is that
 * of the branch taken. The sweep re-runs each segment of steps between list
 * rebuilds from its snapshot, keeping y_n, y_mid, the velocity gradients and
 * the trial stresses of the segment (256 bytes per particle per step of the
 * longest segment), and reverses it step by step. The context ends in the
 * recorded end state with its current bodies; the record stays valid.
 * Synchronises. Errors: CRM_E_STATE (no valid record, or the context stepped
 * since), CRM_E_NOMEM, CRM_E_NONFINITE, CRM_E_DEVICE. */
crm_status crm_adjoint(crm_ctx* ctx, const double* lam_pos, const float* lam_vel, const float* lam_sigma,
                       const float* lam_rho, const double* lam_force, const double* lam_torque, double* out_pos,
                       float* out_vel, float* out_sigma, float* out_rho, double* out_params);

/* enable = 1: run the kernels of each step after its rebuild as one hipGraph,
 * captured on a private stream whenever the working set's buffers or row
 * counts change and launched on the context's stream; results are identical
 * to direct launches. Not used while profiling. enable = 0: direct launches. */
crm_status crm_set_graph(crm_ctx* ctx, int32_t enable);

/* LDS tile configurations of the soil-stage kernels (the neighbour records of
 * a block of 32 cell-sorted rows staged in LDS once per stage). */
#define CRM_TILE_NONE 0   /* neighbours read through L1/L2; highest occupancy */
#define CRM_TILE_SMALL 1  /* 787 records (640 with cell-offset positions), 4 blocks per CU */
#define CRM_TILE_LARGE 2  /* 1024 records (832), 3 blocks per CU */

/* Tile configuration of the soil-stage kernels. config = CRM_TILE_NONE,
 * _SMALL or _LARGE selects it; config < 0 times the stage-1 kernel with each
 * on the current state and list (three launches each; only the midpoint
 * state, which the next step recomputes, is written) and keeps the fastest.
 * chosen (may be NULL) receives the configuration in use. Every
 * configuration gives bit-identical results. Default CRM_TILE_SMALL.
 * Errors: CRM_E_INVALID, CRM_E_STATE (autotuning before the first step),
 * CRM_E_DEVICE. Synchronises when autotuning. */
crm_status crm_autotune(crm_ctx* ctx, int32_t config, int32_t* chosen);

/* Kernel timing for measurement. enable = 1 starts recording HIP events around
 * each kernel class of every following step on the context's stream (and
 * clears earlier records); enable = CRM_PROF_CLASSES | m records only the
 * classes k (numbered as in crm_get_profile) whose bit 1 << k is set in m;
 * enable = 0 stops recording. Errors: CRM_E_INVALID (other values). */
#define CRM_PROF_CLASSES 0x100
crm_status crm_set_profiling(crm_ctx* ctx, int32_t enable);

/* Recorded timings, out: 18 doubles. For class k = 0..6, out[2k] = launches and
 * out[2k + 1] = total milliseconds: 0 rebuild (all kernels of a rebuild step),
 * 1 marker placement, 2 BCE extrapolation (stage 1), 3 soil RHS + stage-1
 * update, 4 BCE + body forces (stage 2), 5 soil RHS + stage-2 update + return
 * mapping, 6 body force reduction. out[14] = soil neighbour pairs and out[15] =
 * marker neighbour pairs of the last rebuild. Class 7, the activity flags of
 * all particles (part of a rebuild step with active domains; Sec. 4.2 item 2):
 * out[16] launches, out[17] milliseconds. Synchronises. */
crm_status crm_get_profile(crm_ctx* ctx, double* out);

/* Capacity policy of Sec. 4.2 item 3 (host logic, no device access): grow to
 * ceil(G * n) when n exceeds cap; at steps that are multiples of S_I, shrink
 * to n when n / cap < S. Returns the new capacity. */
int64_t crm_capacity_next(int64_t cap, int64_t n, int64_t step, double G, double S, int64_t S_I);

/* Human-readable description of the last error of ctx (or of the last failed
 * crm_init when ctx is NULL). Never NULL. */
const char* crm_last_error(const crm_ctx* ctx);

/* Release every resource of ctx (NULL is ignored). Synchronises. */
void crm_destroy(crm_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* CRM_H */
