/*
 * lbe.h -- C ABI of the MI355X (gfx950) two-component Shan-Chen D3Q19 lattice
 * Boltzmann library with moving rigid ellipsoids.
 *
 * Method: F. Guenther, F. Janoschek, S. Frijters, J. Harting, "Lattice
 * Boltzmann simulations of anisotropic particles at liquid interfaces",
 * arXiv:1109.3277, Sec. 2: LB equation (1) with the BGK operator (2), the
 * Shan-Chen inter-component force (3), moving bounce-back (4) and the particle
 * force (5), shell densities with particle colour (10), particles evolved by
 * Newton's equations.
 *
 * Conventions for every call:
 *  - Return 0 on success or a negative LB_E* code; lb_last_error() then holds
 *    a message. A failed call leaves the handle usable unless it says otherwise.
 *  - Pointers named dev_* are device memory; all others are host memory owned
 *    by the caller, copied in or out before the call returns.
 *  - Fields are indexed [z][y][x], x fastest, N = nx*ny*nz nodes; node (x,y,z)
 *    sits at position (x,y,z) (0-based; the paper counts from 1).
 *  - Quaternions are (w, x, y, z), body -> space, normalised on input. The body
 *    z axis is the ellipsoid's symmetry axis (radius R_par); the other two
 *    radii are R_perp.
 *  - A handle is not thread-safe; all device work of a handle is ordered on
 *    the stream given at creation. Calls that return host data synchronise
 *    that stream.
 *  - The library never allocates device memory: the caller passes a device
 *    workspace of at least lb_workspace_bytes() bytes that must outlive the
 *    handle.
 */
#ifndef LBE_H
#define LBE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LB_OK 0
#define LB_EINVAL (-1)     /* bad argument: dims < 3, tau <= 1/2, non-finite value, NULL where required */
#define LB_ENOMEM (-2)     /* workspace too small, or particle capacity exceeded */
#define LB_EHIP (-3)       /* a HIP runtime error; the message holds hipGetErrorString */
#define LB_EUNSTABLE (-4)  /* NaN or negative density found during lb_step */
#define LB_ESTATE (-5)     /* call-order violation (e.g. lb_step before lb_init_fields) */
#define LB_EGEOM (-6)      /* particle radius <= 0, or bounding radius > max_radius or >= min(nx,ny,nz)/2 */

/* Storage / arithmetic forms of the populations. FP64 stores and computes in
 * double. FP32 stores and computes in float. FP16_DEV / BF16_DEV store the
 * deviation f_i - w_i rho_ref^c (rho_ref^c = the component's initial mean
 * density) in IEEE half / bfloat16 and compute in float. Particle state,
 * force / torque sums and mass reductions are double in every form. */
typedef enum { LB_FP64 = 0, LB_FP32 = 1, LB_FP16_DEV = 2, LB_BF16_DEV = 3 } lb_precision;

/* Problem parameters (Sec. 2 and Sec. 4 of the paper):
 *  tau       BGK relaxation time of both components, Eq. (2); > 1/2.
 *  g_br      cross-component coupling g_AB = g_BA of Eq. (3); > 0 demixes.
 *  psi_kind  effective mass of Eq. (3): 1 -> Psi = 1 - exp(-rho) (recommended),
 *            0 -> Psi = rho.
 *  max_particles  particle capacity reserved in the workspace.
 *  max_radius     largest bounding radius max(R_par, R_perp) any particle
 *                 may have (sizes the per-particle work space; must be > 0
 *                 when max_particles > 0 and < min(nx, ny, nz) / 2). */
typedef struct {
    int32_t nx, ny, nz;
    double tau;
    double g_br;
    int32_t psi_kind;
    int32_t precision; /* lb_precision */
    int32_t max_particles;
    double max_radius;
} lb_params;

typedef struct lb_handle lb_handle;

/* Bytes of device workspace lb_create needs for these parameters (0 if the
 * parameters are invalid). */
size_t lb_workspace_bytes(const lb_params* prm);

/* Create a handle over a caller-owned device workspace (dev_ws, ws_bytes) and
 * a HIP stream (hipStream_t passed as void*, NULL = default stream). The
 * workspace is carved, never freed by the library. *out is NULL on failure. */
int lb_create(const lb_params* prm, void* dev_ws, size_t ws_bytes, void* hip_stream, lb_handle** out);

/* Release host-side state. Does not free the workspace. NULL is a no-op. */
void lb_destroy(lb_handle* h);

/* Initial fields (Sec. 2; populations start at the equilibrium of Eq. (2)):
 * f_i^c = f_i^eq(rho^c, u) on every fluid node. rho_a, rho_b: N doubles each
 * (component A = red, B = blue). u: 3N doubles (x,y,z per node) or NULL for
 * rest. Values are not screened: a NaN or negative density makes the next
 * lb_step return LB_EUNSTABLE. Must precede lb_add_ellipsoids and lb_step. */
int lb_init_fields(lb_handle* h, const double* rho_a, const double* rho_b, const double* u);

/* Add n rigid ellipsoids (Sec. 2: particles discretised on the lattice,
 * coupled by Eq. (4)-(5); colour Delta rho after Eq. (10)). radii: n x 2
 * (R_par, R_perp); pos: n x 3 (wrapped into the box); quat: n x 4; delta_rho:
 * n (may be NULL -> 0); density: n (may be NULL -> 1). Nodes whose body-frame
 * offset d satisfies (d_x^2+d_y^2)/R_perp^2 + d_z^2/R_par^2 <= 1 become solid
 * (smallest particle index wins on overlaps) and the fluid on them is removed.
 * Velocities start at zero. Requires lb_init_fields first. */
int lb_add_ellipsoids(lb_handle* h, int32_t n, const double* radii, const double* pos, const double* quat,
                      const double* delta_rho, const double* density);

/* Advance nsteps >= 0 full time steps (densities, shell fill, Shan-Chen force,
 * BGK collision, streaming with moving bounce-back and particle force/torque,
 * rigid-body update, re-rasterisation with kill/fill). Work is enqueued on
 * the handle's stream; the call then waits for it to check the health flag and
 * returns LB_EUNSTABLE if a NaN or negative density appeared or if a particle
 * moved more than two lattice spacings in one step. */
int lb_step(lb_handle* h, int32_t nsteps);

/* Same as lb_step but does not wait: no health check; the stream is left
 * running (for timing and graph capture by the caller). */
int lb_step_async(lb_handle* h, int32_t nsteps);

/* Macroscopic fields (Sec. 2, the moments defined after Eq. (2): rho^c =
 * sum_i f_i^c and rho^c u^c = sum_i f_i^c c_i): densities rho_a, rho_b (N
 * each), barycentric velocity u = (j^A+j^B) / (rho^A+rho^B) (3N, x y z per
 * node, without a half-force correction) and the owner map (N int32: -1
 * fluid, -2 wall, p >= 0 particle index; particles are discretised on the
 * lattice, Sec. 2). Solid nodes read 0 density and velocity. Any output may
 * be NULL. Host buffers are the caller's. Synchronises the stream. */
int lb_read_fields(lb_handle* h, double* rho_a, double* rho_b, double* u, int32_t* owner);

/* The same fields as lb_read_fields, written to the caller's device memory
 * (dev_rho_a, dev_rho_b: N doubles; dev_u: 3N doubles; dev_owner: N int32;
 * any may be NULL), ordered on the handle's stream without waiting: for
 * analysis on the GPU without a host round trip. The buffers must not
 * overlap the workspace. */
int lb_read_fields_dev(lb_handle* h, double* dev_rho_a, double* dev_rho_b, double* dev_u, int32_t* dev_owner);

/* Number of particles on the handle (or a negative error code). */
int lb_num_particles(const lb_handle* h);

/* Set the motion of particle k (0 <= k < lb_num_particles): velocity V,
 * angular velocity omega and angular momentum L, all in the space frame (the
 * rigid-body state of Sec. 2 that the bounce-back of Eq. (4) and the next
 * body update read). Any of the three may be NULL (left as it is). The body
 * update recomputes omega from L with the current orientation, so a
 * consistent state has omega = R I^-1 R^T L. Host arrays of 3 doubles, the
 * caller's. LB_EINVAL for a bad index or a non-finite value (nothing is
 * changed then). Synchronises the stream. */
int lb_set_particle_motion(lb_handle* h, int32_t k, const double* vel, const double* omega, const double* angmom);

/* Particle state, n x 3 (quat n x 4); force / torque are the totals applied in
 * the last rigid-body update (bounce-back sums of Eq. (5) plus kill/fill
 * impulses). Any output may be NULL. Synchronises the stream. */
int lb_read_particles(lb_handle* h, double* pos, double* quat, double* vel, double* omega, double* force,
                      double* torque);

/* Diagnostics of the conserved quantities of Sec. 2 (per-component mass
 * sum_n rho^c, which the BGK step (2) and streaming (1) conserve, and the
 * total fluid momentum, which the Shan-Chen force (3) leaves unchanged since
 * its pair forces cancel), FP64, deterministic order: out[0..7] = {mass A,
 * mass B, momentum x, y, z over fluid nodes, mass removed by particles
 * (removed at placement plus killed minus filled as they move, cumulative),
 * number of fluid nodes, health (1 = NaN or negative density present)}.
 * out is the caller's host array of 8 doubles. Synchronises the stream. */
int lb_stats(lb_handle* h, double out[8]);

/* Lateral domain size of the order parameter phi~ = rho_A - rho_B (Sec. 4,
 * Eq. (12)), FP64, deterministic order: out[0..7] = {L_x, L_y, L_z,
 * L = (L_x + L_y + L_z) / 3, <k_x^2>, <k_y^2>, <k_z^2>, sum_k S(k)}, with
 * S(k) = |phi'_k|^2 / N the structure function of the fluctuation phi' =
 * phi~ - <phi~> (the squared modulus), k_i = 2 pi n_i / L_i in the symmetric
 * range, <k_i^2> = sum_k k_i^2 S(k) / sum_k S(k), L_i = 2 pi / sqrt(<k_i^2>).
 * Particle and wall nodes hold no fluid and count as phi~ = 0. A component
 * with no variation along its axis gives L_i = +inf; a uniform field gives
 * NaN. out is the caller's host array of 8 doubles. Uses the idle population
 * copy as staging (the state is unchanged). Synchronises the stream.
 * LB_EINVAL if a box side exceeds LB_DOMAIN_MAX_LINE; LB_ESTATE on a batch
 * handle (call it on a system) or before lb_init_fields. */
#define LB_DOMAIN_MAX_LINE 2048
int lb_domain_size(lb_handle* h, double out[8]);

/* Uniform body acceleration a (3 doubles) added to every fluid node's force
 * (test and channel-flow use; default 0). */
int lb_set_body_accel(lb_handle* h, const double a[3]);

/* Particle-particle interactions (Sec. 2, Eqs. (6)-(9)), off by default:
 * Hertz repulsion K_H (2R - r)^{5/2} of equal spheres (Eq. (6)) extended to
 * ellipsoids with the Berne-Pechukas strength and range of Eqs. (7)-(8)
 * (sigma_bar = 2 R_o, eps_bar = K_H sigma_bar^{5/2}; for two particles of
 * different shape R_p and R_o are the means of the pair's), and the
 * lubrication correction of Eq. (9) with the ellipsoid gap |r| - sigma and
 * R = sigma / 2, opposing the normal relative velocity, for gaps below
 * delta_c (taken no smaller than delta_c / 4), viscosity from the initial
 * mean densities. The paper uses K_H = 100 and delta_c = 2/3. The forces and
 * torques join the bounce-back sums at each rigid-body update; pairs are
 * found with a device cell list and summed in a fixed order. on = 0 turns
 * them off. LB_EINVAL for K_H < 0 or delta_c <= 0; LB_ESTATE on a batch or
 * system handle, or when max_particles < 2. */
int lb_set_pair_interactions(lb_handle* h, int on, double K_H, double delta_c);

/* Static solid (wall) nodes, for channel tests (Couette / Poiseuille):
 * mask[n] != 0 (N bytes, x fastest) marks node n as a wall; wall_u (3
 * doubles, NULL for resting walls) is the velocity of every wall node.
 * Links into a wall node take the moving bounce-back of Eq. (4) with that
 * velocity. A wall node next to fluid takes, like a particle node, the mean
 * density of its fluid neighbours (Eq. (10), colour 0). Walls never move or
 * change; particles are not rasterised onto them. Must come before
 * lb_init_fields (LB_ESTATE otherwise), which leaves wall nodes empty. The
 * wall velocity is a property of the handle, not of a checkpoint. */
int lb_set_static_solid(lb_handle* h, const uint8_t* mask, const double* wall_u);

/* Checkpoint: lb_state_bytes() bytes of host memory hold the populations,
 * owner map, particle state and counters; lb_load_state restores them into a
 * handle created with the same parameters. The populations are stored in
 * plain form (each node's values in its own slots; between steps the values
 * bounced into solid nodes are kept there): saving rewrites the device state
 * into that form, which leaves every later result unchanged bit for bit. */
size_t lb_state_bytes(const lb_handle* h);
int lb_save_state(lb_handle* h, void* host_buf, size_t bytes);
int lb_load_state(lb_handle* h, const void* host_buf, size_t bytes);

/* Per-phase timing with HIP events recorded on the handle's stream around
 * every kernel launch of lb_step (phases: 0 densities, 1 shell fill, 2 fused
 * force/collide/stream with bounce-back, 3 particle force sums, 4 rigid
 * bodies, 5 raster (clear + rasterise), 6 kill / fill). lb_profile_enable(h, 1)
 * starts a fresh record, 0 stops recording.
 * lb_profile_read waits for the recorded events and writes, per phase, the
 * summed milliseconds and the number of launches (arrays of LB_NPHASES). */
#define LB_NPHASES 7
int lb_profile_enable(lb_handle* h, int on);
int lb_profile_read(lb_handle* h, double* ms, int64_t* launches);

/* ---- Batches: many independent periodic systems advanced together.
 * The method per system is unchanged (same equations, same arithmetic: a
 * system stepped in a batch ends bit for bit where a lone handle with the
 * same parameters and inputs ends; the one exception is a particle-free box
 * in 4- or 2-byte storage whose width is 64, 128, 256 or 512, which a lone
 * handle runs with its row kernel and a batch with tiles, equal to
 * rounding). Each kernel phase is one launch over all systems, and n steps
 * run as one captured HIP graph, launched on the stream given at creation
 * (the graph is recorded on a private capture stream and runs nowhere else),
 * so many small systems fill the GPU and launch cost is paid once per call.
 * All systems share one precision; dims, tau, g_br, psi_kind and particle
 * capacity may differ per system. */

/* Workspace bytes for nsys systems with parameters per_sys[0..nsys-1] (0 if
 * any is invalid or the precisions differ). */
size_t lb_batch_workspace_bytes(int32_t nsys, const lb_params* per_sys);

/* Create a batch handle over one caller-owned workspace and HIP stream (as
 * lb_create). The systems start empty: initialise each with the *_sys calls
 * below (or through its system handle). *out is NULL on failure. */
int lb_create_batch(int32_t nsys, const lb_params* per_sys, void* dev_ws, size_t ws_bytes, void* hip_stream,
                    lb_handle** out);

/* Per-system calls on a batch handle: the same arguments, layouts, errors
 * and ownership as lb_init_fields, lb_add_ellipsoids, lb_read_fields,
 * lb_read_particles and lb_stats, for system `sys` (0 <= sys < nsys, else
 * LB_EINVAL). lb_step / lb_step_async on the batch handle advance every
 * system; each must have fields first (LB_ESTATE otherwise). */
int lb_init_fields_sys(lb_handle* batch, int32_t sys, const double* rho_a, const double* rho_b, const double* u);
int lb_add_ellipsoids_sys(lb_handle* batch, int32_t sys, int32_t n, const double* radii, const double* pos,
                          const double* quat, const double* delta_rho, const double* density);
int lb_read_fields_sys(lb_handle* batch, int32_t sys, double* rho_a, double* rho_b, double* u, int32_t* owner);
int lb_read_particles_sys(lb_handle* batch, int32_t sys, double* pos, double* quat, double* vel, double* omega,
                          double* force, double* torque);
int lb_stats_sys(lb_handle* batch, int32_t sys, double out[8]);

/* Number of systems of a batch handle (or a negative error code). */
int lb_batch_size(const lb_handle* batch);

/* The handle of system `sys`, owned by the batch (valid until the batch is
 * destroyed; lb_destroy on it is a no-op). It takes every per-system call:
 * lb_init_fields, lb_add_ellipsoids, lb_read_fields, lb_read_particles,
 * lb_stats, lb_set_body_accel, lb_set_static_solid, lb_save_state /
 * lb_load_state. lb_step on it returns LB_ESTATE: systems advance only with
 * lb_step / lb_step_async on the batch handle. Per-system calls on the batch
 * handle itself return LB_ESTATE. */
int lb_batch_system(lb_handle* batch, int32_t sys, lb_handle** out);

/* Autotune the fused kernel's tile shape for this batch: each candidate
 * (BX x 256/BX nodes of one xy-plane per 256-thread block, BX in
 * tile_widths) is timed on the current state over all systems (the timed
 * launches only write the scratch population copy; the state does not
 * change) and the fastest is kept. The choice is cached for the life of the
 * process per precision and system shapes (box, solids or not); a batch of
 * the same shapes takes it without timing. Results do not depend on the
 * choice. Requires fields on every system. out (may be NULL) receives the
 * chosen width, whether it came from the cache, and each candidate's time
 * per fused launch over all systems in ms. */
#define LB_TUNE_CANDIDATES 3
typedef struct {
    int32_t tile_width;
    int32_t cached;
    int32_t tile_widths[LB_TUNE_CANDIDATES];
    double ms[LB_TUNE_CANDIDATES];
} lb_tune_result;
int lb_batch_tune(lb_handle* batch, lb_tune_result* out);

/* The graph of the last lb_step / lb_step_async call on a batch: its number
 * of steps (all run by that one graph launch) and of kernel nodes. */
int lb_batch_last_graph(const lb_handle* batch, int32_t* steps, int64_t* kernel_nodes);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): the diagnostics of
 * lb_stats, computed on the GPU into the caller's DEVICE memory dev_out and
 * enqueued on the handle's stream without waiting. A lone handle writes its 8
 * values (the order of lb_stats); a batch handle writes nsys x 8, system by
 * system. Nothing is allocated on the host or the device: the per-block
 * partial sums live in a static device array of the library, 256 blocks x 8
 * doubles for each of up to LB_NOALLOC_MAX_SYSTEMS systems (4 MiB), which
 * every GPU the library runs on holds until the process ends. A batch of more
 * systems is rejected (LB_EINVAL). Each call rewrites every partial before it
 * reads it; calls that overlap on one GPU race on that array. Values equal
 * lb_stats's to rounding (the partial sums are grouped differently); the
 * fluid count, health flag and removed mass match exactly. The call does no
 * host-device copy and no synchronisation. LB_ESTATE on a system handle of a
 * batch (call it on the batch), before lb_init_fields, or on a batch whose
 * systems changed (fields, particles, walls) since its last lb_step or
 * lb_batch_tune, which upload the batch's tables. */
#define LB_NOALLOC_MAX_SYSTEMS 256
int lb_stats_noalloc(lb_handle* h, double* dev_out);

/* Message of the last failed call on h (or of the last failed lb_create or
 * lb_create_batch when h is NULL); valid until the next call on the same
 * handle. */
const char* lb_last_error(const lb_handle* h);

#ifdef __cplusplus
}
#endif
#endif /* LBE_H */
