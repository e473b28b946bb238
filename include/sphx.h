/*
 * sphx.h -- C ABI of the MI355X (gfx950) Riemann-WCSPH library.
 *
 * A library context holds a batch of one or more independent cases; each
 * case is one fluid body and one static wall body (bodies made of particles
 * with inner and contact interactions, Section 9 overview of the SPHinXsys
 * paper, arXiv 2010.12375) with its own parameters and clock, advanced with
 * the paper's fluid scheme: Riemann-based continuity and momentum equations
 * (Section 2.2, Eq. riemannsph) with the one-sided wall condition (Section
 * 2.3), density re-initialisation (Eq. eqrhosum), dual-criteria time
 * stepping (Section 2.4) and position-based Verlet (Section 7). All cases of
 * a batch run in the same kernel launches.
 *
 * Conventions, for every call:
 *  - Return 0 on success or a negative SPHX_E* code; sphx_last_error() gives
 *    a message for the last failure on the context (prefixed "case k: " in a
 *    batch of several cases).
 *  - All host pointers belong to the caller and are only read or written
 *    during the call. Device memory belongs to the library.
 *  - Arrays at the boundary are FP64 and in original particle order (the
 *    order of the arrays passed to sphx_set_fluid* / sphx_set_walls*), however
 *    the library orders particles internally. Vectors are packed n * dim.
 *  - Calls without a case index act on case 0, except sphx_build_neighbors,
 *    sphx_density_reinit, sphx_advance, sphx_profile and sphx_counts, which
 *    act on the whole batch. Case indices out of range give SPHX_EINVAL.
 *  - Work is queued on the stream given at creation (or one the library
 *    creates); calls that return data synchronise that stream.
 *  - A context is not thread-safe; separate contexts are independent.
 */
#ifndef SPHX_H
#define SPHX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPHX_OK 0
#define SPHX_EINVAL (-1)    /* bad argument or unsupported parameter */
#define SPHX_ENOMEM (-2)    /* device or host allocation failed */
#define SPHX_EHIP (-3)      /* a HIP runtime call failed */
#define SPHX_EESCAPE (-4)   /* a fluid particle left the domain box */
#define SPHX_ENAN (-5)      /* NaN in the particle state */
#define SPHX_ECAP (-6)      /* caller buffer too small; *n_out holds the size needed */
#define SPHX_EOVERFLOW (-7) /* a particle has more neighbours than the list capacity */
#define SPHX_ESTATE (-8)    /* call out of order (e.g. rates before any particles) */

#define SPHX_FP64 0 /* every field and every pair computation in FP64 */
#define SPHX_FP32 1 /* FP32 fields and pair arithmetic; FP64 positions, clock and diagnostics */

#define SPHX_INNER 0   /* fluid-fluid neighbours */
#define SPHX_CONTACT 1 /* fluid-wall neighbours */

#define SPHX_FIELD_POS 0  /* n * dim */
#define SPHX_FIELD_VEL 1  /* n * dim */
#define SPHX_FIELD_RHO 2  /* n */
#define SPHX_FIELD_P 3    /* n, from the EoS p = c0^2 (rho - rho0) (Eq. eqeos) */
#define SPHX_FIELD_DRHO 4 /* n, drho/dt of the last density relaxation */

typedef struct sphx_ctx sphx_ctx;

typedef struct {
    int32_t dim;         /* 2 or 3 */
    int32_t precision;   /* SPHX_FP64 or SPHX_FP32 */
    int32_t periodic[3]; /* periodic axes (period = hi - lo); need >= 3 cells of 2h */
    int32_t nsub_queue;  /* acoustic sub-steps per queued graph launch (0: default 5; the
                            batch takes case 0's); a step that needs more continues in
                            the next queue, with the same result */
    double dp;           /* initial particle spacing: fluid mass rho0 dp^dim, wall volume dp^dim */
    double h;            /* smoothing length; Wendland C2 support radius 2h */
    double rho0;         /* reference density */
    double c0;           /* artificial sound speed (Eq. eqeos) */
    double u_ref;        /* reference speed: floor of |v|max in the advection criterion */
    double cfl_ad;       /* advection CFL number (Eq. dt-advection; 0.25) */
    double cfl_ac;       /* acoustic CFL number (Eq. dt-relax; 0.6) */
    double gravity[3];   /* body force per unit mass */
    double lo[3], hi[3]; /* domain box: binning grid; fluid outside it is an escape */
    double sigma0;       /* reference kernel sum of Eq. eqrhosum; <= 0: the lattice sum
                            over the dp lattice, self included, computed by the library */
    double eta;          /* dynamic viscosity of Eq. eqviscous (0: inviscid); adds the
                            h^2/nu limit (nu = eta/rho0) to the advection step */
    double p_background; /* background pressure p0 of the transport-velocity correction,
                            Eq. transport (0: off; for flows without free surface) */
    int32_t reinit_mode; /* 0: Eq. eqrhosum (free surface), 1: Eq. eqrhosumnosurface */
    int32_t pad_;        /* unused, 0 */
} sphx_params;

typedef struct {
    double mass;        /* total fluid mass */
    double momentum[3]; /* sum m v */
    double e_kin;       /* sum m |v|^2 / 2 */
    double e_pot;       /* -sum m g . x */
    double e_int;       /* sum m c0^2 (ln(rho/rho0) + rho0/rho - 1): energy of the EoS */
    double front;       /* surge front: max x over fluid particles */
    double max_drho;    /* max |rho/rho0 - 1| */
    double t;           /* clock */
    int64_t n_substeps; /* acoustic sub-steps since sphx_set_fluid */
    int64_t n_steps;    /* advection steps since sphx_set_fluid */
} sphx_diag;

/* Create a context with one case. stream: a hipStream_t to queue work on,
 * or NULL for a library-owned stream (default priority). Fails with
 * SPHX_EINVAL for dim other than 2/3, non-positive sizes, a periodic axis
 * with fewer than 3 cells of size 2h, or an empty box. */
int sphx_create(const sphx_params* params, void* stream, sphx_ctx** out);

/* Create a context with a batch of n_cases >= 1 cases, params[c] for case c
 * (an array of n_cases). Every case must have the same dim and precision;
 * sizes, boxes, sound speeds and every other parameter may differ. The cases
 * start empty; each needs sphx_set_fluid_case before it can run. */
int sphx_create_batch(const sphx_params* params, int32_t n_cases, void* stream, sphx_ctx** out);

/* Number of cases of the context (or SPHX_EINVAL for NULL). */
int sphx_num_cases(const sphx_ctx* ctx);

/* Replace case c's parameters (dim and precision unchanged) when its cell
 * grid stays the same (same box, periodicity and cell count per axis); its
 * particles, clock and walls stay. SPHX_EINVAL otherwise. Invalidates the
 * neighbour configuration of the batch. */
int sphx_set_params_case(sphx_ctx* ctx, int32_t c, const sphx_params* params);

/* Free every device buffer, graph and the owned stream. NULL is a no-op. */
void sphx_destroy(sphx_ctx* ctx);

/* Message of the last failure on ctx (never NULL; "" if none). */
const char* sphx_last_error(const sphx_ctx* ctx);

/* Fluid particles from arrays (direct particle generator, Section 9):
 * pos n*dim (required), vel n*dim (NULL: rest), rho n (NULL: rho0), drho n
 * (NULL: 0, the density rate carried into the first half-step). Resets the
 * clock to 0 and invalidates the neighbour configuration. */
int sphx_set_fluid(sphx_ctx* ctx, int64_t n, const double* pos, const double* vel, const double* rho,
                   const double* drho);

/* The same for case c. Resets that case's clock and counters only; the
 * other cases keep their state (the device layout may grow, moving them).
 * Invalidates the neighbour configuration of the batch. */
int sphx_set_fluid_case(sphx_ctx* ctx, int32_t c, int64_t n, const double* pos, const double* vel,
                        const double* rho, const double* drho);

/* Wall particles: pos n*dim and unit normals n*dim pointing into the fluid
 * (Section 2.3 wall normal), in their reference pose. Every wall particle
 * must lie inside the domain box. The walls are static until
 * sphx_set_wall_motion* gives them a motion (a new wall set drops the
 * case's motion). Invalidates the neighbour configuration. */
int sphx_set_walls(sphx_ctx* ctx, int64_t n, const double* pos, const double* normal);

/* The same for case c (inside case c's box). */
int sphx_set_walls_case(sphx_ctx* ctx, int32_t c, int64_t n, const double* pos, const double* normal);

/* Prescribed rigid motion of a wall body (Section 2.3: the wall velocity
 * u_w of the right state U_R = -U_L + 2 u_w, Eq. eqrienoslip; moving tanks
 * and wave makers of the sloshing cases, Section 10.1):
 *   displacement d(t) = amp sin(omega t),
 *   rotation theta(t) = roll sin(omega t) (radians) in the x-y plane about
 *   the centre pivot + d(t),
 *   x_w(t) = pivot + d(t) + R(theta(t)) (x_w0 - pivot), n_w(t) = R(theta) n_w0,
 *   v_w(t) = d'(t) + theta'(t) z x (x_w - pivot - d(t)).
 * The walls take their pose at every configuration update (at the clock of
 * their case) and keep it, with the rest of the frozen configuration, for
 * the advection step; u_w = -n_w . v_w enters the pressure relaxation at the
 * sub-step's start time and the density relaxation at its end time, and the
 * no-slip shear of Eq. eqviscous at the step's start time. P_R keeps the
 * gravity term of Eq. eqriepright only. In 2D the z components of amp and
 * pivot are ignored. */
typedef struct {
    double amp[3];   /* translation amplitude */
    double omega;    /* angular frequency (>= 0) */
    double roll;     /* rotation amplitude about the z axis (radians) */
    double pivot[3]; /* rotation centre at t = 0 */
} sphx_wall_motion;

/* Give case 0's walls the motion `motion` (NULL: static again). `moving`:
 * one flag per wall particle in the order of sphx_set_walls (0: the
 * particle stays static, e.g. a fixed obstacle in a moving tank; NULL: every
 * wall particle moves). SPHX_EINVAL if the motion could take a wall particle
 * out of the domain box (bound: |amp_k| + |roll| times its distance from the
 * pivot in the x-y plane), moves along a periodic axis, or is not finite.
 * Invalidates the neighbour configuration. The surrogate calls refuse
 * batches with moving walls. */
int sphx_set_wall_motion(sphx_ctx* ctx, const sphx_wall_motion* motion, const int32_t* moving);

/* The same for case c. */
int sphx_set_wall_motion_case(sphx_ctx* ctx, int32_t c, const sphx_wall_motion* motion, const int32_t* moving);

/* Given velocities of case 0's wall particles (Section 2.3: the wall
 * velocity v_w of Eqs. eqrienoslip and eqviscous for walls that do not move,
 * e.g. a lid or belt sliding along itself). `vel`: dim values per wall
 * particle, in the order of sphx_set_walls, host memory, copied; NULL clears
 * them. They add to the velocity of a motion where both are given, are
 * taken in the fixed x-y-z frame (not turned with a roll), and leave the
 * walls where they are. All zero is the same as none (the static code
 * path). sphx_set_walls clears them. SPHX_EINVAL for a non-finite value.
 * Invalidates the neighbour configuration; the surrogate calls refuse
 * batches with wall velocities. */
int sphx_set_wall_velocity(sphx_ctx* ctx, const double* vel);

/* The same for case c. */
int sphx_set_wall_velocity_case(sphx_ctx* ctx, int32_t c, const double* vel);

/* Fluid particles from device memory of the context's device (for example
 * the storage of framework tensors; the caller keeps ownership and may free
 * the buffers when the call returns): the same arrays and meaning as
 * sphx_set_fluid_case, FP64, in original particle order. Before the batch's
 * first device layout the arrays are staged through the host. */
int sphx_set_fluid_device(sphx_ctx* ctx, int32_t c, int64_t n, const double* pos, const double* vel,
                          const double* rho, const double* drho);

/* Field `field` of case c, as sphx_get_field_case, written to device memory
 * `out` of the context's device (FP64, original particle order, n*dim or n
 * values). Returns when the copy is complete. */
int sphx_get_field_device(sphx_ctx* ctx, int32_t c, int field, double* out);

/* Checkpoint (save and load of a run; the restart files of the paper's I/O
 * table, Section 9): sphx_save writes the parameters of
 * every case, its walls, wall motion and given wall velocities, its clock
 * and time step state, and its particle state in the library's current slot
 * order to `path`; sphx_load restores such a file into a context created with the
 * same parameters (same number of cases, dimension, precision and every
 * sphx_params field except nsub_queue; SPHX_EINVAL otherwise or for a
 * truncated or foreign file, and for corrupt contents, checked on the host
 * before anything is uploaded: particle ids that are not a permutation of
 * each case's particles, non-finite positions, state, walls or motion, a
 * negative or non-finite clock or step state, unknown error bits; the
 * context is then unchanged). The neighbour configuration is rebuilt on the
 * next call that needs it; from the restored state the run continues bit for
 * bit as the saved context would have, given the same lanes per particle
 * (sphx_set_lanes; not part of the file). The surrogate's parameters are not
 * part of a checkpoint. */
int sphx_save(sphx_ctx* ctx, const char* path);
int sphx_load(sphx_ctx* ctx, const char* path);

/* Configuration update (Section 2.4: at the advection frequency): wrap
 * periodic coordinates, bin particles into cells of size >= 2h, rebuild the
 * inner and contact neighbour lists with the FP64 predicate r^2 < (2h)^2
 * (dx = x_i - x_j, one minimum-image wrap, left-to-right sum), and freeze
 * the pair geometry, for every case. SPHX_EESCAPE / SPHX_ENAN / SPHX_EOVERFLOW
 * (of the lowest failing case) on failure; then the batch has no
 * configuration until a later call succeeds. Every case needs fluid
 * (SPHX_ESTATE otherwise). */
int sphx_build_neighbors(sphx_ctx* ctx);

/* Neighbour lists (the inner and contact relations of Section 9; the
 * particle table's neighbor_relation unit holds this configuration) as CSR
 * of original ids, ascending within each row.
 * kind: SPHX_INNER or SPHX_CONTACT. off: n_fluid + 1 entries (may be NULL);
 * idx: cap entries (may be NULL). *n_out receives the number of entries;
 * SPHX_ECAP if idx is given and cap < *n_out. */
int sphx_get_neighbors(sphx_ctx* ctx, int kind, int64_t* off, int64_t* idx, int64_t cap, int64_t* n_out);

/* The same for case c (ids relative to that case's own arrays). */
int sphx_get_neighbors_case(sphx_ctx* ctx, int32_t c, int kind, int64_t* off, int64_t* idx, int64_t cap,
                            int64_t* n_out);

/* Density re-initialisation of Eq. eqrhosum on the current configuration:
 * rho = max(rho, rho0 sum W / sum W0), sums over self, fluid and wall
 * neighbours; every case. */
int sphx_density_reinit(sphx_ctx* ctx);

/* The two time-step criteria for the current state (Eq. dt-advection with
 * |v|max floored at u_ref and, for a case with viscosity eta > 0, the
 * h^2/nu limit, nu = eta/rho0; Eq. dt-relax). */
int sphx_time_steps(sphx_ctx* ctx, double* dt_ad, double* dt_ac);
int sphx_time_steps_case(sphx_ctx* ctx, int32_t c, double* dt_ad, double* dt_ac);

/* The rates of one acoustic sub-step of size dt from the current state,
 * which is left unchanged: the pressure relaxation's dv/dt (n*dim, gravity
 * included) and the density relaxation's drho/dt (n), i.e. half-steps of
 * Eq. verlet-first-half, Eq. riemannsph momentum, Eq. verlet-first-mediate,
 * Eq. riemannsph continuity. Requires a configuration. */
int sphx_compute_rates(sphx_ctx* ctx, double dt, double* dvdt, double* drhodt);
int sphx_compute_rates_case(sphx_ctx* ctx, int32_t c, double dt, double* dvdt, double* drhodt);

/* Advance every case by up to n_steps advection steps (the dual-criteria
 * time stepping of Section 2.4; each: dt_ad, density
 * re-initialisation, acoustic sub-steps until the step is covered, the last
 * clipped to land on it, then the configuration update), each case stopping
 * early when its clock reaches t_stop (a step is clipped to end exactly on
 * t_stop). The cases advance together, one advection step per case per
 * queued graph launch; sub-step control stays on the device and the host
 * synchronises once per batch of up to 64 launches. A case that fails (NaN,
 * escape, list overflow) stops where it failed while the others go on; the
 * call then returns the error of the lowest failing case (see
 * sphx_case_status). *n_substeps (may be NULL) receives the acoustic
 * sub-steps done, summed over the cases, *t_out (may be NULL) case 0's
 * clock. */
int sphx_advance(sphx_ctx* ctx, int32_t n_steps, double t_stop, int64_t* n_substeps, double* t_out);

/* Error state of case c: SPHX_OK, or the code of the failure that stopped
 * it (sticky until its fluid is set again or a configuration update of the
 * batch succeeds). */
int sphx_case_status(sphx_ctx* ctx, int32_t c);

/* Field in original order as FP64 (SPHX_FIELD_*; the particle fields the
 * paper's observers and state output write, Section 9 I/O table). */
int sphx_get_field(sphx_ctx* ctx, int field, double* out);
int sphx_get_field_case(sphx_ctx* ctx, int32_t c, int field, double* out);

/* FP64 global observables of the current state (reduced on the device):
 * mass, momentum, kinetic, potential and internal energy (the work of the
 * EoS, Eq. eqeos), surge front and the largest density deviation (the
 * quantity Section 2.1 keeps near 1 %), for the paper's observers
 * (Section 9 I/O table). */
int sphx_diagnostics(sphx_ctx* ctx, sphx_diag* out);

/* The same for case c into out[0]; for c < 0, every case into out[0 ..
 * n_cases). */
int sphx_diagnostics_case(sphx_ctx* ctx, int32_t c, sphx_diag* out);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): sphx_diagnostics_case
 * with no allocation of any kind in the call. Its per-tile partials and
 * per-case sums live in a file-scope device array of 4 MiB per GPU (held
 * until the process ends; its address is taken once per device when a
 * context is created there). Same arguments and results as
 * sphx_diagnostics_case (the same kernels, so the same values).
 * SPHX_ESTATE if the context has no device layout yet (the first call that
 * needs its particles, e.g. sphx_build_neighbors or sphx_diagnostics_case,
 * makes it); SPHX_EINVAL if its tiles of 64 particle slots plus its cases
 * exceed 65 536. All contexts on one GPU share that array: calls that
 * overlap on one GPU (other threads, other streams) race; every value a
 * call reads it has written itself. */
int sphx_diagnostics_noalloc(sphx_ctx* ctx, int32_t c, sphx_diag* out);

/* Average device time per launch (milliseconds) of the hot kernels,
 * measured with HIP events on the context's stream over `reps` launches
 * each, on the current state of every case (each case one acoustic sub-step
 * of its own dt_ac); state and clocks are restored afterwards. ms[0]
 * pressure relaxation, ms[1] density relaxation, ms[2] neighbour-list build,
 * ms[3] density re-initialisation. */
int sphx_profile(sphx_ctx* ctx, int32_t reps, double* ms);

/* Particle and pair counts of the current configuration: out[0] fluid,
 * out[1] wall, out[2] inner pairs (directed), out[3] contact pairs; summed
 * over the batch, or for case c. */
int sphx_counts(sphx_ctx* ctx, int64_t* out);
int sphx_counts_case(sphx_ctx* ctx, int32_t c, int64_t* out);

/* Choose the lanes per particle of the pair kernels (2, 4 or 8 in 2D; 4, 8
 * or 16 in 3D) by timing `reps` launches of the pressure and density
 * relaxation of the batch with each, and rebuild the configuration for the
 * fastest one (*lanes, may be NULL; times, may be NULL: 3 entries, ms per
 * relaxation pair for the three candidates in that order). The lists are the same; the per-particle sums are combined in a
 * different order, so later results can differ from the default's at
 * rounding level. Requires a configuration. */
int sphx_autotune(sphx_ctx* ctx, int32_t reps, int32_t* lanes, double* times);

/* Set the lanes per particle of the pair kernels (2, 4 or 8 in 2D, default
 * 4; 4, 8 or 16 in 3D, default 8), e.g. a value sphx_autotune picked
 * before. An existing configuration is rebuilt from the current state in
 * the new list layout, as by sphx_build_neighbors (the same lists; sums are
 * then combined in another order). Call between advances. SPHX_EINVAL for
 * another value. */
int sphx_set_lanes(sphx_ctx* ctx, int32_t lanes);

/* ---------------------------------------------------------------------
 * Message-passing surrogate (2D contexts only; SPHX_EINVAL in 3D).
 *
 * A network on the SPH neighbour graph of the current configuration (the
 * inner and contact relations, Section 9) predicts for every fluid particle
 * its mean acceleration and density rate over the next two advection steps
 * (about ten acoustic sub-steps). Hidden width 64, three message-passing
 * layers: node features v/u_ref, (rho - rho0)/(0.01 rho0), neighbour counts;
 * edge features (x_j - x_i)/h, r/h, (v_j - v_i)/u_ref, W(r)/W(0), a wall
 * flag, the pressure difference (p_j - p_i)/(rho0 |g| h) (the one-sided wall
 * state for a wall); edge messages relu(P_i + Q_j + R_ij) (a learned vector in place of
 * Q_j for wall edges) summed per particle; residual node updates; output
 * (a_x/g, a_y/g, 1000 Drho h/(rho0 u_ref)). Matrix products take bfloat16
 * operands and accumulate in FP32 (MFMA). Parameters are one flat float32
 * array of sphx_gnn_num_params() values in this order, each matrix K x 64
 * row-major (input dimension first): Wn[32x64] bn[64] We[32x64] be[64], then
 * per layer Wa[64x64] Wb[64x64] Wc[64x64] bm[64] qw[64] Wu[128x64] bu[64],
 * then Wo1[64x64] bo1[64] Wo2[64x3] bo2[3] (rows 8..31 of Wn and We multiply
 * zero padding). One parameter set serves every case of the batch. The plain
 * scheme stays the fallback whenever a case's predicted density deviates from
 * rho0 by more than the caller's bound (1 % is the variation the sound speed
 * is chosen for, Section 2.1). */

int64_t sphx_gnn_num_params(void);

/* Set the parameters (n == sphx_gnn_num_params()); resets Adam's moments. */
int sphx_gnn_set_params(sphx_ctx* ctx, const float* params, int64_t n);

/* Current parameters / the gradient of the last training step. */
int sphx_gnn_get_params(sphx_ctx* ctx, float* params, int64_t n);
int sphx_gnn_get_grad(sphx_ctx* ctx, float* grad, int64_t n);

/* Predictions for every case on the current configuration (SPHX_ESTATE
 * without one); sphx_gnn_get_output_case returns case c's, nf x 3 in
 * original order, valid until the configuration or the parameters change. */
int sphx_gnn_forward(sphx_ctx* ctx);
int sphx_gnn_get_output_case(sphx_ctx* ctx, int32_t c, double* out);

/* Training: targets of case c (nf x 3, original order, same scaling as the
 * output), set on the current configuration (after sphx_build_neighbors;
 * SPHX_ESTATE without one); sphx_gnn_train_step runs the forward and backward passes over
 * every case (loss: mean squared error over all fluid particles and outputs)
 * and one Adam step (beta 0.9 / 0.999, eps 1e-8) with learning rate lr.
 * Every case needs a target set on the current configuration. */
int sphx_gnn_set_target_case(sphx_ctx* ctx, int32_t c, const double* target);
int sphx_gnn_train_step(sphx_ctx* ctx, double lr, double* loss);

/* Per-launch device time (ms, HIP events over `reps` launches) of the
 * surrogate's kernels on the current configuration; ms has 7 entries:
 * ms[0] one fused message-passing layer (edge encoder, edge product,
 * messages and their sums in one kernel, no edge array in device memory),
 * ms[1] the graph's edge features, ms[2] the node update product, ms[3] one
 * whole forward pass as inference runs it (graph and features included, one
 * host synchronisation per pass); for comparison the same with the edge
 * activations through device memory (the training forward's form): ms[4]
 * the whole pass, ms[5] its edge product R = E0 Wc, ms[6] its message sums
 * of one layer. sizes (may be NULL): [0] node rows, [1] edges. */
int sphx_gnn_profile(sphx_ctx* ctx, int32_t reps, double* ms, int64_t* sizes);

/* `windows` surrogate windows: each predicts every case's mean rates over
 * dt = 2 dt_ad (from its current |v|max) and, for the cases whose predicted
 * max |rho/rho0 - 1| stays <= max_drho, applies v += a dt, x += (v + v')/2 dt,
 * rho += Drho dt, advances the clock by dt and the step count by 2 and updates
 * the configuration; every other case takes the two advection steps with the
 * plain scheme. plain_every > 0 also sends every plain_every-th window to the
 * plain scheme. *n_fallback / *n_surrogate (may be NULL) count case-windows
 * of each kind. Errors as for sphx_advance. */
int sphx_surrogate_advance(sphx_ctx* ctx, int32_t windows, double max_drho, int32_t plain_every,
                           int64_t* n_fallback, int64_t* n_surrogate);

#ifdef __cplusplus
}
#endif

#endif /* SPHX_H */
