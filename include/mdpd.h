/*
 * mdpd.h -- C ABI of the MI355X (gfx950) many-body DPD timestep library.
 *
 * One timestep of many-body dissipative particle dynamics (mDPD) on one GPU:
 * cell binning and sort, the many-body density pass, the pair-force pass
 * (attractive A w_c, density-dependent repulsive B (rho_i + rho_j) w_d,
 * dissipative and random terms), the wall treatment for fluid against frozen
 * solid particles, and velocity-Verlet integration.  Model and algorithm:
 * Xia et al., "A GPU-accelerated package for simulation of flow in
 * nanoporous source rocks with many-body dissipative particle dynamics",
 * Sec. 2.1 (Eq. 1 and the density weight), Sec. 2.2 (walls), Sec. 3.2 and
 * Alg. 1 (order of the timestep).
 *
 * Conventions for every call:
 *   - Every function returns an mdpd_status; MDPD_OK is 0, errors are
 *     negative.  A human-readable message for the last error of the calling
 *     thread is returned by mdpd_last_error().  No C++ exception crosses the
 *     ABI.
 *   - Particle ids are input indices 0..n-1.  All per-particle outputs are
 *     returned in input (id) order, whatever the internal sort order.
 *   - Arrays named "pos", "vel", "force" are n x 3, row-major (x, y, z of
 *     particle 0 first), float64.
 *   - mem_kind says where caller arrays live: MDPD_MEM_HOST (pageable or
 *     pinned host memory) or MDPD_MEM_DEVICE (device memory on the current
 *     HIP device).  Caller arrays are borrowed for the duration of the call
 *     only; the library copies what it keeps.
 *   - All device work is enqueued on the stream given to mdpd_create (NULL
 *     means the default stream).  Calls that return data to the host
 *     synchronise that stream.  A handle must not be used from two threads
 *     at once.
 */
#ifndef MDPD_H
#define MDPD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MDPD_MAX_TYPES 8

typedef int32_t mdpd_status;

enum {
    MDPD_OK = 0,
    MDPD_E_INVALID = -1,     /* bad argument (size, range, NULL, non-finite)   */
    MDPD_E_OOM = -2,         /* device or host allocation failed               */
    MDPD_E_HIP = -3,         /* a HIP runtime call failed                      */
    MDPD_E_NONFINITE = -4,   /* a non-finite position or velocity appeared     */
    MDPD_E_STATE = -5,       /* call not valid in the system's current state   */
    MDPD_E_UNSUPPORTED = -6  /* valid input this build does not handle         */
};

enum { MDPD_MEM_HOST = 0, MDPD_MEM_DEVICE = 1 };

/* Arithmetic of the pair passes.  In both forms the neighbour test
 * (r^2 < r_c^2, r^2 < r_d^2) is done in FP64 on FP64 positions, so the
 * neighbour sets do not depend on the form, and positions, velocities,
 * velocity-Verlet and global sums are FP64.
 *   MDPD_FP64         pair math, density and per-particle force sums in FP64
 *   MDPD_FP32_FORCES  pair math, density and per-particle force sums in FP32;
 *                     the force pass takes each pair's position difference
 *                     from fixed-point coordinates (resolution box / 2^32 per
 *                     axis) and its velocity difference from FP32 copies */
enum { MDPD_FP64 = 0, MDPD_FP32_FORCES = 1 };

/* Wall treatment (Sec. 2.2, Sec. 3.2):
 *   MDPD_WALL_OFF   frozen particles interact like any other, nothing else
 *   MDPD_WALL_BVF   boundary volume fraction phi of each fluid particle at its
 *                   predicted position, phi_i = sum_{frozen j, r<r_c} w_c^2 /
 *                   sum_{j != i, r<r_c} w_c^2; if phi_i > phi_c the predicted
 *                   step is rejected: x <- x(t), and the half-step velocity
 *                   is reflected.  With wall_slip = 0 it is negated
 *                   (bounce-back, no slip); otherwise, with the wall normal
 *                   n = unit(sum_{frozen j, r<r_c} w_c^2 (x_i - x_j) / r) at
 *                   the predicted position, the normal part is negated and
 *                   the tangential part scaled by 2 wall_slip - 1: 1 gives
 *                   specular reflection (full slip), 0.5 drops the
 *                   tangential velocity (a zero normal sum, and a particle
 *                   also sent back in the step before, fall back to
 *                   bounce-back, so it leaves the wall the way it came). */
enum { MDPD_WALL_OFF = 0, MDPD_WALL_BVF = 1 };

typedef struct {
    double box[3];        /* periodic box edges L_x, L_y, L_z; each >= 2 r_c      */
    double rc;            /* cutoff of w_c = 1 - r/r_c (Sec. 2.1)                 */
    double rd;            /* cutoff of w_d = 1 - r/r_d and of w_rho; 0 < r_d <= r_c */
    double kT;            /* target temperature; sigma^2 = 2 gamma kT             */
    double dt;            /* timestep                                             */
    double mass;          /* particle mass (all particles)                        */
    double body_force[3]; /* acceleration g on fluid particles (force m g)        */
    double phi_c;         /* wall threshold for MDPD_WALL_BVF, >= 0               */
    double A[MDPD_MAX_TYPES * MDPD_MAX_TYPES];     /* A[t_i*ntypes + t_j], symmetric */
    double B[MDPD_MAX_TYPES * MDPD_MAX_TYPES];     /* B >= 0, symmetric             */
    double gamma[MDPD_MAX_TYPES * MDPD_MAX_TYPES]; /* gamma >= 0, symmetric         */
    uint32_t seed;        /* key word 0 of the pair noise generator               */
    int32_t ntypes;       /* 1..MDPD_MAX_TYPES                                    */
    int32_t precision;    /* MDPD_FP64 or MDPD_FP32_FORCES                        */
    int32_t wall_model;   /* MDPD_WALL_OFF or MDPD_WALL_BVF                       */
    double wall_slip;     /* MDPD_WALL_BVF reflection, 0 (no slip) .. 1 (full)    */
    double skin;          /* neighbour-list skin >= 0: the cells and the list of  */
                          /* pairs closer than r_c + skin are rebuilt only when   */
                          /* a particle has moved skin/2 since the last build     */
                          /* (0: every step); any value gives the same pairs     */
    double diss_ctrl;     /* control of the effective fluid-solid dissipation    */
                          /* (Sec. 2.2), eta >= 0; 0 turns it off.  For a fluid   */
                          /* particle i with frozen neighbours, E_i = sum over    */
                          /* frozen j within r_c of w_c^2 is brought to the       */
                          /* target eta diss_rho W_D phi_i (W_D = 2 pi r_c^3 / 15,*/
                          /* the integral of w_c^2 over the interaction sphere;   */
                          /* phi_i as for MDPD_WALL_BVF, at the positions of the  */
                          /* force evaluation): every fluid-frozen pair of i uses */
                          /* gamma s_i and sigma sqrt(s_i), s_i = target / E_i,   */
                          /* which equals eta diss_rho W_D / sum_{j != i, r<r_c}  */
                          /* w_c^2.  eta = 1: the solid dissipates like fluid at  */
                          /* rest of density diss_rho in its place (no slip);     */
                          /* smaller eta lets the fluid slip.  Independent of     */
                          /* wall_model.                                          */
    double diss_rho;      /* the fluid number density rho_f of the target; > 0   */
                          /* when diss_ctrl > 0                                   */
} mdpd_params;

/* Observables at the current step (all FP64 sums in a fixed order):
 *   ke        = m/2 sum over fluid |v|^2
 *   kT        = 2 ke / (3 dof), dof = N_f - 1 for a periodic fluid with no
 *               frozen particles and no body force, N_f otherwise
 *   pressure  = (sum over fluid m |v|^2 + virial) / (3 V)
 *   virial    = sum over fluid i and neighbours j of c_ij r_ij F^C_ij,
 *               c_ij = 1/2 for fluid j, 1 for frozen j
 *   epot      = the same weighted sum of (A r_c / 2) w_c^2 plus
 *               sum over all particles (pi r_d^4 B_ii / 30) rho_i^2
 *   mean_rho  = mean many-body density of fluid particles
 *   ncorr_*   = wall corrections in the last step and since creation */
typedef struct {
    int64_t step;
    int64_t n, n_fluid;
    int64_t ncorr_last, ncorr_total;
    double ke, kT, pressure, virial, epot, mean_rho;
    double momentum[3];
} mdpd_observables;

typedef struct mdpd_system mdpd_system; /* opaque; owned by the library */

/* Create a system and evaluate density and forces at t = 0 with the given
 * velocities and noise step 0.
 *   p       parameters, copied.  box >= 2 r_c per axis, 0 < rd <= rc, dt > 0,
 *           mass > 0, kT >= 0, symmetric tables with B, gamma >= 0.
 *   n       number of particles, 0 <= n < 2^30 (n = 0 gives an empty system;
 *           the list entries keep 30 bits of slot, far above what one GPU's
 *           memory holds at about 700 bytes per particle)
 *   pos     n x 3 positions, each coordinate in [-L, 2L); wrapped into [0, L)
 *   vel     n x 3 velocities (ignored for frozen particles, which get 0)
 *   type    n type indices in [0, ntypes)
 *   frozen  n flags, nonzero = frozen wall particle (never moves)
 *   stream  hipStream_t to enqueue on (NULL: default stream)
 *   out     receives the handle; *out is NULL on error.
 * Errors: MDPD_E_INVALID (arguments, a box edge below 2 r_c),
 * MDPD_E_UNSUPPORTED (more than 2^24 cells), MDPD_E_OOM, MDPD_E_HIP,
 * MDPD_E_NONFINITE (the evaluation at t = 0 gives a non-finite or out-of-box
 * predicted state). */
mdpd_status mdpd_create(const mdpd_params *p, int64_t n, const double *pos, const double *vel,
                        const int32_t *type, const uint8_t *frozen, int32_t mem_kind,
                        void *stream, mdpd_system **out);

/* Create a batch of nrep independent replicas (separate periodic boxes, each
 * with its own parameters, noise seed and particle count) that every call
 * advances together: each pass of the timestep is one launch over all
 * replicas.  Replica r owns the particles offsets[r] .. offsets[r+1]-1 of the
 * input arrays (offsets: nrep + 1 entries, offsets[0] = 0, non-decreasing;
 * offsets[nrep] < 2^30); inside a replica the particle ids are 0, 1, ...
 * from offsets[r], so that replica r evolves exactly, bit for bit, as a
 * system created alone from its own slice of the arrays with params[r].
 * All replicas need the same precision and wall model.  Per-particle outputs
 * (mdpd_get_state, mdpd_debug_*) come back in input order over the whole
 * batch; observables per replica come from mdpd_read_replica_observables.
 * mdpd_read_observables and mdpd_read_profile need nrep = 1; the adjoint
 * runs per replica (losses and table gradients per replica).
 * Errors as for mdpd_create. */
mdpd_status mdpd_create_batch(int32_t nrep, const mdpd_params *params, const int64_t *offsets,
                              const double *pos, const double *vel, const int32_t *type,
                              const uint8_t *frozen, int32_t mem_kind, void *stream,
                              mdpd_system **out);

/* Advance nsteps >= 0 timesteps in the order of Alg. 1: half kick and drift
 * x(t+dt), [wall: phi and corrector], rho for all particles, forces
 * f(t+dt) with noise step = the new step number, v(t+dt).  Synchronises the
 * stream at the end and returns MDPD_E_NONFINITE if any position or
 * velocity became non-finite (the state is then undefined). */
mdpd_status mdpd_step(mdpd_system *s, int64_t nsteps);

/* Observables of the current state (see mdpd_observables); MDPD_E_STATE
 * for a batch of more than one replica. */
mdpd_status mdpd_read_observables(mdpd_system *s, mdpd_observables *out);

/* Observables of replicas first .. first+count-1 of a batch into out[count].
 * The wall-correction counters are totals over the batch. */
mdpd_status mdpd_read_replica_observables(mdpd_system *s, int32_t first, int32_t count,
                                          mdpd_observables *out);

/* Pressure tensor of replicas first .. first+count-1 (a single system is
 * replica 0) at the current state, six values per replica into out[6 count]:
 * xx, yy, zz, xy, xz, yz of
 *   P_ab = [sum over fluid m v_a v_b + sum over fluid i, neighbours j of
 *           c_ij d_a d_b F^C(r) / r] / V
 * with d = x_i - x_j, F^C = A w_c + B (rho_i + rho_j) w_d (Eq. 1) and c_ij as
 * for the virial; trace / 3 is the pressure of mdpd_observables.  Used for
 * the stress difference across an interface (Sec. 4.1). */
mdpd_status mdpd_read_stress(mdpd_system *s, int32_t first, int32_t count, double *out);

/* The pressure tensor of mdpd_read_stress for callers that cannot allocate
 * memory (code under HIP graph capture, tight serving loops): same result
 * (within rounding: the per-particle terms are summed per block, then per
 * replica), but every intermediate lives in a fixed scratch array of 8 MiB
 * per GPU that the library holds until the process ends, so the call makes
 * no device or host allocation.  out: 6 doubles per replica first ..
 * first + count - 1 (xx, yy, zz, xy, xz, yz), in host memory (mem_kind
 * MDPD_MEM_HOST: the call synchronises the system's stream) or device memory
 * (MDPD_MEM_DEVICE: the results are written on the system's stream and the
 * call returns without waiting).  The system's device must be current.
 * Limit: 6 (blocks + count) doubles, blocks = ceil(4 n_r / 256) summed over
 * the replicas (about 11 million particles); larger systems give
 * MDPD_E_UNSUPPORTED.  All calls on one GPU share the scratch: calls that
 * overlap on one GPU (other threads, other streams) race. */
mdpd_status mdpd_read_stress_noalloc(mdpd_system *s, int32_t first, int32_t count, double *out,
                                     int32_t mem_kind);

/* Number of list builds since creation, summed over the replicas (a build
 * re-sorts a replica into cells of edge >= r_c + skin and rebuilds its skin
 * list; the first evaluation builds every replica once).  builds: host. */
mdpd_status mdpd_read_list_builds(mdpd_system *s, int64_t *builds);

/* Profile of fluid particles in nbins (1..4096) equal bins of L_axis along
 * axis (0..2).  quantity 0: number density; 1..3: mean velocity x, y, z;
 * 4: kinetic temperature of velocities relative to the bin mean; 5: mean
 * many-body density.  Empty bins give 0.  out: nbins doubles, host. */
mdpd_status mdpd_read_profile(mdpd_system *s, int32_t axis, int32_t nbins, int32_t quantity,
                              double *out);

/* Current positions (wrapped into [0, L)), velocities v(t) and, if rho is
 * not NULL, many-body densities (n), in input order, into caller arrays. */
mdpd_status mdpd_get_state(mdpd_system *s, double *pos, double *vel, double *rho,
                           int32_t mem_kind);

/* Neighbour sets of the hot path at the current positions: for each
 * particle the number of j != i with r_ij^2 < cutoff^2 (0 < cutoff <= r_c)
 * and the order-independent hash sum_j mix64(j) mod 2^64, where mix64 is the
 * SplitMix64 output function.  count and hash: n entries, host. */
mdpd_status mdpd_debug_neighbors(mdpd_system *s, double cutoff, int64_t *count, uint64_t *hash);

/* Total force (pairs plus body force) on each particle from the last force
 * evaluation, n x 3, host; zero for frozen particles. */
mdpd_status mdpd_debug_forces(mdpd_system *s, double *force);

/* Kernel timing with HIP events on the system's stream.  enable = 1 records
 * an event pair around every launch of each timed kernel from then on;
 * mdpd_read_kernel_timing returns the summed duration in milliseconds and
 * the number of launches of kernel class k (0: sort, 1: neighbour list,
 * 2: density, 3: force, 4: wall, 5: adjoint pair passes) and resets the
 * counters. */
mdpd_status mdpd_set_kernel_timing(mdpd_system *s, int32_t enable);
mdpd_status mdpd_read_kernel_timing(mdpd_system *s, int32_t kernel, double *total_ms,
                                    int64_t *launches);

/* Work split of the pair passes (lanes = 1, 2, 4, 8 or 16): in pass 1
 * (density and wall fraction) and pass 2 (force) that many lanes of a
 * 64-wide wavefront cooperate on one particle; in pass 0 (the per-step
 * neighbour list, skin 0) that many wavefronts share each cell of the
 * border launch (every cell of a small system), dealing its particles round
 * robin.  Results do not depend on pass 0's setting (default 1); passes 1
 * and 2 (default 4) change only the summation order. */
mdpd_status mdpd_set_lanes(mdpd_system *s, int32_t pass, int32_t lanes);

/* Graph mode (enable = 1): mdpd_step replays a HIP graph of two captured
 * timesteps instead of launching each kernel from the host (an odd last step
 * runs eagerly).  Results are bit for bit those of eager stepping.  The graph
 * is captured on first use and again after the lane split or the buffer
 * parity changed; kernel timing does not see replayed steps.  enable = 0
 * releases the graph. */
mdpd_status mdpd_set_graph(mdpd_system *s, int32_t enable);

/* Autotuner: times `steps` >= 1 timesteps (HIP events around each launch on
 * the system's stream) for every setting of pass 0 (skin 0 only), then of
 * the density pass and then of the force pass (see mdpd_set_lanes), keeps
 * the fastest of each, and restores the state it started from
 * (the trial steps leave no trace; the result only changes summation
 * orders).  The choice is cached for the process per (n, cells, replicas,
 * precision, type count, walls) and reused without timing.  lanes_out
 * (nullable) receives the lanes of passes 0..2. */
mdpd_status mdpd_autotune(mdpd_system *s, int32_t steps, int32_t *lanes_out);

/* Checkpoint and bitwise resume.  A checkpoint holds the complete dynamical
 * state after the last completed step (positions, velocities, forces, the
 * predicted next half-step, densities, ids and types in the internal order,
 * the cell list, the step counter and the wall-correction counters) and a
 * copy of the parameters.  Loading it into a system created with the same
 * parameters and the same n makes every later call return what the saved
 * system would have returned, bit for bit: the noise is keyed on (seed,
 * step, ids) and the internal order and summation orders are functions of
 * the state alone.
 *   mdpd_checkpoint_size   bytes needed for a checkpoint of s
 *   mdpd_save_checkpoint   writes it to buf (bytes >= that size), host or
 *                          device memory per mem_kind
 *   mdpd_load_checkpoint   replaces the state of s with the checkpoint in buf
 * Errors: MDPD_E_INVALID (NULL, buffer too small, not a checkpoint, or saved
 * with other parameters or another n), MDPD_E_HIP. */
mdpd_status mdpd_checkpoint_size(const mdpd_system *s, uint64_t *bytes);
mdpd_status mdpd_save_checkpoint(mdpd_system *s, void *buf, uint64_t bytes, int32_t mem_kind);
mdpd_status mdpd_load_checkpoint(mdpd_system *s, const void *buf, uint64_t bytes, int32_t mem_kind);

/* Adjoint: gradients of trajectory losses by reverse-mode differentiation
 * of the timestep (Eq. 1 forces, the density of Sec. 2.1 and the
 * velocity-Verlet order of Alg. 1).  The pair noise depends on (seed, step,
 * ids) only and is held fixed.  With MDPD_WALL_BVF the corrector's
 * decisions are held fixed as well (events of the recorded trajectory): a
 * particle sent back keeps its position and carries its negated half-step
 * velocity, and the derivative follows that; wall_slip must be 0
 * (MDPD_E_UNSUPPORTED otherwise).  With diss_ctrl > 0 the derivative
 * includes that of the factor s_i through the positions of i's neighbours.
 * The recording starts from the state given
 * to mdpd_create (MDPD_E_STATE after mdpd_step).
 *
 * mdpd_forward_record advances nsteps >= 0 steps from step 0, keeping a
 * device checkpoint every `every` >= 1 steps, and returns in loss[3 nrep]
 * for each replica r (nrep = 1 for a single system)
 *   loss[3r]     = mean many-body density of fluid particles,
 *   loss[3r + 1] = virial pressure (as in mdpd_observables),
 *   loss[3r + 2] = mean x-velocity of fluid particles,
 * of the final state (average = 0) or averaged over the states after steps
 * 1..nsteps (average = 1, nsteps >= 1).  Afterwards the system stands at
 * step nsteps.
 *
 * mdpd_backward returns the gradient of L = sum_r sum_q w[3r + q] loss[3r + q]
 * of the last recording with respect to
 *   dA, dB, dgamma  the pair tables, host: for each replica its ntypes x
 *                   ntypes entries, replica after replica; the derivative of
 *                   L along a symmetric change D of a table is
 *                   sum_ab d[ab] D[ab] (at gamma = 0 the noise amplitude
 *                   sqrt(2 gamma kT) has no derivative and is left out)
 *   dx0, dv0        the positions and velocities given to mdpd_create(_batch),
 *                   n x 3 in input order, host or device per mem_kind (dv0 of
 *                   frozen particles is 0)
 * Any output may be NULL.  Each segment of `every` steps is recomputed from
 * its checkpoint, so the call costs about one forward pass plus the adjoint
 * passes; memory is one checkpoint (about 170 bytes per particle) per
 * segment plus every + 1 stored states (about 90 bytes per particle each).
 * The result is deterministic, and the system is left at the end of the
 * recording. */
mdpd_status mdpd_forward_record(mdpd_system *s, int64_t nsteps, int32_t every, int32_t average,
                                double *loss);
mdpd_status mdpd_backward(mdpd_system *s, const double *w, double *dA, double *dB, double *dgamma,
                          double *dx0, double *dv0, int32_t mem_kind);

/* Release the system and its device memory.  NULL is ignored. */
void mdpd_destroy(mdpd_system *s);

/* Message of the calling thread's last error ("" if none). */
const char *mdpd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MDPD_H */
