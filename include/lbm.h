/*
 * lbm.h -- C interface of the MI355X (gfx950) library that advances a
 * two-component Shan-Chen D3Q19 lattice Boltzmann fluid with suspended,
 * moving, wettable spheres, the coupled method of Jansen & Harting, "From
 * Bijels to Pickering emulsions: a lattice Boltzmann study" (Secs. II-IV).
 *
 * Conventions for every call:
 *  - Return value: LB_OK (0) or a negative LB_E* code; the handle keeps a
 *    message for the last failure, readable with lb_last_error().
 *  - Host arrays passed in or out are plain host memory owned by the caller;
 *    the library copies them and keeps no caller pointer.
 *  - Device memory is owned by the handle, allocated through the caller's
 *    lb_allocator (or hipMalloc when none is given) and released by
 *    lb_destroy().
 *  - All device work of a handle is enqueued on the HIP stream given to
 *    lb_create(); lb_step() returns after enqueueing, and device-side failures
 *    (non-finite mass, list capacity exceeded) surface at the next call that
 *    synchronises (lb_synchronize, lb_observables, the getters).
 *  - A handle is used from one host thread at a time.
 *  - Results are deterministic: identical inputs give bit-identical outputs on
 *    the same device (no floating-point atomics anywhere).
 *
 * Lattice: sites x = (ix, iy, iz), 0 <= ix < nx, ..., periodic in all axes;
 * the linear site index is n = (iz * ny + iy) * nx + ix.
 * Velocity order (index: c_i):  0: (0,0,0);
 *   1: (+1,0,0)  2: (-1,0,0)  3: (0,+1,0)  4: (0,-1,0)  5: (0,0,+1)  6: (0,0,-1)
 *   7: (+1,+1,0) 8: (-1,-1,0) 9: (+1,-1,0) 10: (-1,+1,0)
 *  11: (+1,0,+1) 12: (-1,0,-1) 13: (+1,0,-1) 14: (-1,0,+1)
 *  15: (0,+1,+1) 16: (0,-1,-1) 17: (0,+1,-1) 18: (0,-1,+1)
 * Component 0 is "red", component 1 is "blue" (Sec. II).
 * Population arrays exchanged with the host are double [2][19][nz][ny][nx]:
 * the post-streaming populations f_i^c(x, t) at the start of a step.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    LB_OK = 0,
    LB_EINVAL = -1,    /* invalid argument or parameter */
    LB_ENOMEM = -2,    /* device allocation failed */
    LB_EDEVICE = -3,   /* HIP runtime error */
    LB_EOVERLAP = -4,  /* spheres overlap */
    LB_ESTATE = -5,    /* call not allowed in the current state */
    LB_EUNSTABLE = -6, /* the fluid mass became non-finite, or a sphere moved >= 1 site along an axis */
    LB_ECAPACITY = -7  /* a per-particle list overflowed (a sphere moved too far in one step) */
};

/* Precision of the fluid. LB_FP64 and LB_FP32 store and compute in that type
 * (FP32 stores f_i - zeta_i rho_init to keep rounding relative to the
 * deviations). LB_FP16 and LB_BF16 store those deviations in 16 bits (round to
 * nearest) and compute every update in FP32; densities, forces and all
 * global and per-sphere sums stay FP32 / FP64. */
enum { LB_FP64 = 0, LB_FP32 = 1, LB_FP16 = 2, LB_BF16 = 3 };

/* Fluid kernel variants. LB_KERNEL_FUSED: one sweep per step that computes
 * densities, virtual fluid, Shan-Chen force, collision and streaming with
 * z-marching tiles; LB_KERNEL_TWOPASS: a density sweep, a virtual-fluid pass
 * and a collide-and-stream sweep. Both compute the same step. LB_KERNEL_AUTO
 * takes the two-pass sweep (lb_autotune measures the alternatives for a box). */
enum { LB_KERNEL_AUTO = 0, LB_KERNEL_FUSED = 1, LB_KERNEL_TWOPASS = 2 };

typedef struct lb_handle lb_handle;

/* Device allocator: alloc(bytes, ctx) returns device memory or NULL;
 * free(ptr, ctx) releases it. */
typedef struct {
    void *(*alloc)(size_t bytes, void *ctx);
    void (*free)(void *ptr, void *ctx);
    void *ctx;
} lb_allocator;

typedef struct {
    int32_t nx, ny, nz;      /* periodic box, each >= 4 */
    int32_t precision;       /* LB_FP64, LB_FP32, LB_FP16 or LB_BF16 (storage of the populations) */
    double tau[2];           /* BGK relaxation time per component, Sec. II, > 1/2 */
    double g_br;             /* Shan-Chen coupling g_rb = g_br of Eq. (4); g_rr = g_bb = 0 */
    double rho0;             /* reference density in the effective mass of Eq. (5), > 0 */
    double w_face, w_edge;   /* weights of the 18-neighbour sum of Eq. (4): faces, edges */
    int32_t velocity_mode;   /* 1: per-component u^c = j^c/rho^c as printed in Sec. II;
                                0: common velocity sum_c(j^c/tau^c)/sum_c(rho^c/tau^c) */
    int32_t eq_order;        /* 3: equilibrium of Eq. (3) as printed; 2: without cubic terms */
    double rho_init[2];      /* mean initial density per component */
    double noise_amp;        /* initial density = rho_init + noise_amp*(2U-1), U uniform */
    uint64_t seed;           /* key of the SplitMix64 draws U (draw index 2n + c) */
    double body_accel[3];    /* uniform acceleration of the fluid (channel-flow tests) */
    int32_t wall_axis;       /* -1: none; 0..2: the planes 0 and n-1 of that axis are walls (n >= 3) */
    double wall_vel[2][3];   /* velocities of the low and the high wall */
    double c0_mass_corr;     /* C_0 of the mass correction, Eq. (31); 0 switches it off */
    double k_hertz;          /* K_Hertz of Eq. (21) */
    double lub_hc, lub_hmin; /* lubrication cut-off and clamp gaps of Eq. (22); hc <= 0: off */
    int32_t kernel;          /* LB_KERNEL_* */
    int32_t tile[3];         /* tile of the fused kernel: x is 64, y 4 or 8 (FP64: 4), z the
                                planes of one segment (clamped to nz); other or 0 values
                                take 64, 4, 64 */
    int32_t lub_mode;        /* how Eq. (22) enters the leap-frog of Eqs. (9), (10), which the
                                paper does not fix for a velocity-dependent force:
                                0: explicit force from the velocities U(t - 1/2), as printed;
                                   an isolated pair's approach speed w becomes
                                   w (1 - c (1/m_1 + 1/m_2)), unstable once that factor < -1
                                   (light spheres at the h_min clamp);
                                1 (default): pair impulses J = c w / (1 + c (k_p/m_p + k_q/m_q))
                                   from the velocities after every other force (k: lubrication
                                   contacts of a sphere), backward Euler for an isolated pair */
    int32_t link_writes;     /* where the bounced populations of sphere links (Eq. (16)) are
                                formed, with bitwise the same result: 1 (default): the link
                                kernel writes every one into the solid site's slot; 0: with the
                                two-pass sweep, outside a stream capture, the next step's density
                                sweep forms each from the fluid site's own slot (only links next
                                to a map change are written out by the map update) */
    int32_t force_average;   /* the fluid force and torque that enter Eqs. (9), (10) (the link
                                momentum of Eq. (17) with its moving-wall term, and the Shan-Chen
                                force on the virtual fluid; the covering and refilling impulses
                                are not included), a step the paper leaves to the coupling of the
                                literature it builds on: 0 (default): this step's, as printed;
                                1: the mean of this step's and the previous step's (a sphere's
                                first step after lb_add_particles or lb_set_particle_state uses
                                its own alone), which damps the step-to-step oscillation of the
                                link force that makes light spheres (density near the fluid's)
                                run away in long runs */
} lb_params;

typedef struct {
    double pos[3];    /* centre, in [0, n) per axis */
    double vel[3];    /* velocity U(t - 1/2) */
    double omega[3];  /* angular velocity Omega(t - 1/2) */
    double radius;    /* > 0, <= min(nx, ny, nz)/4 and 2 ceil(radius) + 7 <= each edge */
    double density;   /* mass density, > 0; m = density 4/3 pi r^3 */
    double color;     /* wettability Delta rho of Sec. IV (> 0 prefers red) */
    int32_t prescribed; /* 1: velocities fixed, the sphere moves but is not integrated */
} lb_particle;

typedef struct {
    double pos[3], vel[3], omega[3];
    double force_fluid[3], torque_fluid[3];   /* bounce-back links + Shan-Chen, last step */
    double force_total[3], torque_total[3];   /* everything applied in the last step */
    double pending_impulse[3], pending_angular[3]; /* covering/refilling, applied next step */
} lb_particle_state;

typedef struct {
    int64_t step;
    double mass[2];              /* fluid mass per component (FP64 sums) */
    double fluid_momentum[3];
    double particle_momentum[3]; /* sum m U */
    double pending_impulse[3];
    int64_t n_links, n_shell;    /* bounce-back links and virtual-fluid sites now */
    int64_t covered_total, uncovered_total, refill_fallback;
    int32_t n_particles;
    int32_t unstable;            /* 1 if a step produced a non-finite mass */
} lb_observables_t;

/* Fill p with the defaults: FP32, tau = 1, g_br = 0.08, rho0 = 1, weights
 * (4, 2), velocity_mode 1, eq_order 3, rho_init 0.35 each, noise 0.01,
 * seed 1, no walls, no body force, C_0 = 0, K_Hertz = 100, h_c = 2/3,
 * h_min = 0.1 (the cut-off and clamp stated with Eq. (22)), lub_mode 1,
 * link_writes 1, force_average 0, automatic kernel and tiles; the box is 16^3.  Start every lb_params from
 * here: a zeroed struct selects lub_mode 0. */
void lb_default_params(lb_params *p);

/* Create a lattice: two fluid components with random initial densities (Sec. VI),
 * rho^c(x) = rho_init^c + noise_amp (2U - 1) with U the SplitMix64 draw of
 * index 2n + c, at rest in the equilibrium of Eq. (3) (f_i = zeta_i rho^c),
 * plus the two wall planes if wall_axis >= 0.
 * stream: a hipStream_t (NULL = the null stream); every later call of the
 * handle enqueues its device work there.  alloc may be NULL (hipMalloc).
 * Errors: LB_EINVAL (a parameter out of range: box edge < 1 or more than
 * 2^30 sites, tau <= 1/2, rho0 <= 0, an unknown mode, precision or kernel,
 * walls on an axis shorter than 3), LB_ENOMEM, LB_EDEVICE. */
int lb_create(const lb_params *p, const lb_allocator *alloc, void *stream, lb_handle **out);

/* Release the handle and all its device memory (after the stream drains). */
void lb_destroy(lb_handle *h);

/* Message of the last failure on h ("" if none), valid until the next call;
 * with h == NULL, of the last failed lb_create on the calling thread. */
const char *lb_last_error(const lb_handle *h);

/* Add n spheres (Sec. III: homogeneous spheres, lattice sites inside them
 * are solid); allowed only before the first lb_step.  parts is a host array
 * of n entries, copied.  The sites inside a sphere (strict |x - R| < r on
 * positions rounded to multiples of 2^-20) become solid and their fluid is
 * removed.  Input domain: 0 < radius <= min(nx, ny, nz)/4 and
 * 2 ceil(radius) + 7 <= each box edge (a sphere's bounding box and its
 * neighbour ring fit in one period), density > 0, centre in [0, n) per
 * axis, spheres only in periodic boxes (no walls).
 * Errors: LB_EOVERLAP (two spheres closer than r_a + r_b, minimum image,
 * new against new and old), LB_EINVAL (outside the input domain, or walls
 * present), LB_ESTATE (after stepping, or in a batch). */
int lb_add_particles(lb_handle *h, int32_t n, const lb_particle *parts);

/* Enqueue nsteps time steps (nsteps >= 0) on the handle's stream and return.
 * One step follows Secs. II-IV in this order: moments and densities (Sec.
 * II), virtual fluid on the outermost solid layer (Sec. IV, Eqs. (27),
 * (29), (30)), effective mass Psi (Eq. (5)), Shan-Chen force (Eq. (4)), BGK
 * collision with the velocity shift (Eqs. (2), (3), (6)), streaming with
 * bounce-back and the moving-wall term (Eqs. (11), (12), (16)), momentum
 * exchange and the Shan-Chen force on the spheres (Eqs. (13)-(17), (28)),
 * Hertz and lubrication forces (Eqs. (21), (22)), the leap-frog (Eqs. (9),
 * (10)), then covering and uncovering with refill (Eqs. (18)-(20), (23)-(26),
 * (31)); impulses of covering and refilling act in the next step.  Device
 * failures (a non-finite mass, a sphere moving one site or more along an
 * axis in one step, a list overflow) are reported by the next synchronising
 * call: LB_EUNSTABLE or LB_ECAPACITY. */
int lb_step(lb_handle *h, int32_t nsteps);

/* Wait for the stream; report deferred device failures. */
int lb_synchronize(lb_handle *h);

/* Conserved sums and bookkeeping counters of the current state
 * (synchronises; out is caller-owned host memory).  mass[c] is the fluid
 * mass M^c whose drift from its first-step value is the Delta rho^c of the
 * mass correction, Eq. (31); the momenta are the fluid's sum_i f_i c_i
 * (Sec. II), the spheres' m U (Eq. (9)) and the pending impulses of covering
 * and refilling (Eqs. (18), (20)), whose sum is conserved in a periodic box
 * without walls or body force.  Errors: those of lb_step, deferred. */
int lb_observables(lb_handle *h, lb_observables_t *out);

/* Fields of the current state, each pointer may be NULL:
 * rho [2][N] densities, j [2][N][3] momenta sum_i f c, force [2][N][3] the
 * Shan-Chen (plus body) force on fluid and virtual-fluid sites, u [N][3] the
 * mixture velocity sum_c (j^c + F^c/2) / sum_c rho^c of Eq. (7) on fluid
 * sites (0 elsewhere). N = nx ny nz. (Synchronises.) */
int lb_get_fields(lb_handle *h, double *rho, double *j, double *force, double *u);

/* Post-streaming populations [2][19][N] (zero on solid sites). */
int lb_get_populations(lb_handle *h, double *f);

/* Overwrite the populations on fluid sites (values on solid sites ignored);
 * rounded to the storage precision. */
int lb_set_populations(lb_handle *h, const double *f);

/* Solid map [N]: -1 fluid, p >= 0 owned by sphere p, -2 / -3 low / high wall. */
int lb_get_owner(lb_handle *h, int32_t *owner);

/* Number of spheres. */
int lb_num_particles(const lb_handle *h, int32_t *n);

/* Particle states, lb_num_particles entries. */
int lb_get_particles(lb_handle *h, lb_particle_state *out);

/* Overwrite R, U, Omega and the pending impulses of every sphere (15 doubles
 * per sphere in that order) and rebuild the solid map, virtual-fluid sites
 * and links from the new positions without touching the fluid.  The fluid
 * force of the previous step is forgotten (force_average starts anew). */
int lb_set_particle_state(lb_handle *h, const double *state);

/* Bounce-back links (fluid x, i with x + c_i inside the sphere) and
 * virtual-fluid sites (solid sites of the sphere with a fluid 18-neighbour)
 * of every sphere on the current map. */
int lb_particle_counts(lb_handle *h, int32_t *links, int32_t *shell);

/* Checkpoint (no passage of the paper: storage of the state the method
 * advances).  *bytes in = capacity of buf (caller-owned host memory), out =
 * bytes written (or needed when buf is NULL).  Holds the lb_params the
 * lattice was created with, the step counter, the populations in their
 * storage type, every sphere's state, radius, density, colour and motion
 * flag, the previous step's fluid force and torque of each sphere
 * (force_average), and the mass baseline of Eq. (31).  Errors: LB_EINVAL (buffer too
 * small), LB_EDEVICE. */
int lb_get_state(lb_handle *h, void *buf, size_t *bytes);

/* Restore a checkpoint written by lb_get_state.  The lattice must have the
 * same box, precision and model parameters (tau, g_br, rho0, weights,
 * velocity_mode, eq_order, rho_init, walls, body force, C_0, K_Hertz,
 * lubrication, force averaging; the noise draw, kernel choice and
 * link_writes may differ) and, if it has
 * spheres, the same number with the same radius, density, colour and motion
 * flag; a lattice without spheres that has not stepped takes the
 * checkpoint's spheres.  Errors: LB_EINVAL (not a checkpoint, another format
 * version, other parameters or spheres), LB_ESTATE (other number of spheres,
 * or the lattice is in a batch). */
int lb_set_state(lb_handle *h, const void *buf, size_t bytes);

/* Sec. V: the paper's linear fit theta = 442 Delta rho + 90 (degrees) of the
 * contact angle against the particle colour, inverted; theta in [0, 180]. */
int lb_contact_angle_to_color(double theta_deg, double *color);

/* Kernel timing for measurement, with HIP events recorded on the handle's
 * stream around the launches of one step: which = 0 the sweep that collides
 * and streams the populations, 1 the density sweep of the two-pass variant,
 * 2 the whole step.  lb_enable_timing(h, 1) starts recording (and clears the
 * totals); lb_kernel_timing synchronises and returns the summed milliseconds
 * and the number of launches since then. */
int lb_enable_timing(lb_handle *h, int32_t enable);
int lb_kernel_timing(lb_handle *h, int32_t which, double *ms, int64_t *launches);

/* Device bytes a handle with these parameters and n spheres of radius at most
 * max_radius would allocate, before any lb_get_fields call. */
int lb_footprint_bytes(const lb_params *p, int32_t n_particles, double max_radius, size_t *bytes);

/* ---------------------------------------------------------------------------
 * Analysis observables (off the time-step path; both wait for the handle's
 * stream and copy the result to host memory owned by the caller).
 *
 * lb_domain_size: the lateral domain sizes L_i = 2 pi / sqrt(<k_i^2>) of
 * Sec. VI, Eqs. (33)-(35), with <k_i^2> the second moment along axis i of the
 * structure function S(k) = |phi'_k|^2 / N of the order-parameter fluctuations
 * phi' = phi - <phi>, phi = rho_r - rho_b on fluid sites and 0 on solid ones;
 * k_i = 2 pi m / n_i with |m| <= n_i / 2.  L_out[0..2] (x, y, z), +inf along
 * an axis with no power (phi' constant along it).  Every axis must be at most
 * 2048 (else LB_EINVAL).
 * lb_order_parameter_profile: out[0 .. n_axis-1] = plane averages of phi over
 * the planes normal to `axis` (0 = x, 1 = y, 2 = z), solid sites counted as 0;
 * the zero of this profile locates a flat interface (the contact angle of
 * Sec. V, Eq. (32)).
 * The first call allocates 8 bytes per site of device memory for phi (kept
 * until lb_destroy; not counted by lb_footprint_bytes).  Errors: LB_EINVAL,
 * LB_ENOMEM, LB_EDEVICE (message in lb_last_error).
 * ------------------------------------------------------------------------- */
int lb_domain_size(lb_handle *h, double L_out[3]);
int lb_order_parameter_profile(lb_handle *h, int32_t axis, double *out);

/* lb_order_parameter_profile without any device allocation, for callers that
 * cannot allocate: serving loops that keep a fixed device footprint and
 * harnesses that forbid hipMalloc.  Same arguments and result, bitwise (each
 * site's phi and the plane sums are formed in the same order), but no phi
 * array: the plane averages go to a static device array of 2048 doubles
 * (16 KiB) that each device holds until the process ends.  The axis must be
 * at most 2048 sites long (else LB_EINVAL).  Call it with no device or the
 * handle's device current.  It waits for the handle's stream.  Every call on
 * one device shares that array: calls that overlap on one device, from
 * several threads or streams, race.  Errors: LB_EINVAL, LB_EDEVICE. */
int lb_order_parameter_profile_noalloc(lb_handle *h, int32_t axis, double *out);

/* ---------------------------------------------------------------------------
 * Batches: many lattices advanced by one graph launch.
 *
 * lb_batch_create captures steps_per_launch (even, >= 2) time steps of every
 * member into one HIP graph: members below 2^21 sites with the same
 * precision and collision model, the two-pass sweep and no walls (at least
 * two of them) as one launch per stage over all of them, the others each with
 * its own launches on a branch of its own; lb_batch_step replays it
 * nlaunches times on `stream` (ordered after the members' pending work, and
 * the members' later calls are ordered after it).  A member stepped an odd
 * number of times outside the batch makes lb_batch_step fail (LB_ESTATE).  The kernels are exactly those
 * of lb_step, so every member's result is bitwise the same alone and in a
 * batch.  Members must be fully set up (spheres added); while in a batch they
 * refuse lb_add_particles and lb_set_state, must not record kernel timing,
 * and must outlive the batch.  Errors: LB_EINVAL (bad arguments, a member
 * already in a batch or timing), LB_EDEVICE (capture or launch failed); the
 * message is in lb_batch_last_error (with NULL: of the last failed
 * lb_batch_create on the calling thread).
 * ------------------------------------------------------------------------- */
typedef struct lb_batch lb_batch;
int lb_batch_create(lb_handle **members, int32_t n, int32_t steps_per_launch, void *stream, lb_batch **out);
int lb_batch_step(lb_batch *b, int32_t nlaunches);
int32_t lb_batch_steps_per_launch(const lb_batch *b);
const char *lb_batch_last_error(const lb_batch *b);
void lb_batch_destroy(lb_batch *b);

/* Autotuner: times trial_steps steps of every compiled sweep variant (the
 * two-pass sweep and the fused sweep with each tile shape and z segment that
 * fits the box and precision) on the given box and spheres, and writes the
 * fastest choice into p->kernel and p->tile (and its step time in
 * milliseconds into *best_ms_per_step if non-null).  Each candidate is a
 * lattice of its own, created and destroyed in turn, so device memory for
 * one more lattice must be free.  Returns LB_EDEVICE if no candidate ran. */
int lb_autotune(lb_params *p, int32_t n, const lb_particle *parts, int32_t trial_steps, double *best_ms_per_step);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
