/*
 * hlbm.h -- C ABI of the MI355X (gfx950) library for the four-way coupled
 * homogenized lattice Boltzmann method with a discrete contact model for
 * convex particles (Marquardt, Hafen & Krause, arXiv 2401.10878).
 *
 * The library advances time steps of the paper's Algorithm 1 (one or more
 * contact sub-steps) entirely on one GPU, for spheres, cubes, regular
 * octahedra and convex polyhedra given by vertices and faces:
 *   - D3Q19 BGK stream-collide (Sec. 3.1, eqs. (10)-(13)) with the
 *     exact-difference velocity-shift coupling (Sec. 3.2, eqs. (14)-(15));
 *   - per-node signed-distance evaluation of the particles, which gives
 *     the coupling weight B and the particle velocity at each node
 *     (Sec. 3.2), and the momentum-exchange force and torque on each
 *     particle (eqs. (16)-(18));
 *   - the node-parallel rough contact detection, bounding-box correction
 *     and overlap integration of the discrete contact model (Sec. 3.3.1),
 *     with the lower-id reference for periodic boundaries (Sec. 3.3.2),
 *     and the Nassauer-Kuna contact forces (Sec. 2.3, eqs. (4)-(9));
 *   - Newton-Euler particle motion (eqs. (2)-(3)) with gravity and the
 *     zero-net-flow balance force (Sec. 5.1).
 *
 * Units: lattice units throughout (Delta x = Delta t = 1).  Nodes sit at
 * integer coordinates 0 <= x < nx etc.  x and y are periodic; z is periodic
 * or bounded by half-way bounce-back walls at z = -1/2 and z = nz - 1/2.
 *
 * Layout: host population arrays are FP64 [19][nz][ny][nx] (velocity index
 * slowest), D3Q19 order: rest; +x,-x,+y,-y,+z,-z; (1,1,0),(-1,-1,0),
 * (1,-1,0),(-1,1,0),(1,0,1),(-1,0,-1),(1,0,-1),(-1,0,1),(0,1,1),(0,-1,-1),
 * (0,1,-1),(0,-1,1).  Per-particle vectors are [n][3], quaternions [n][4]
 * in (w, x, y, z) order.  Per-node fields are [nz][ny][nx].
 *
 * Ownership: every pointer argument is a HOST pointer owned by the caller
 * unless stated otherwise; read calls copy and synchronise before return.
 * The context owns its device memory, except population buffers lent with
 * hlbm_bind_populations, which it never frees.
 *
 * Errors: every call returns an hlbm_status; 0 is success.  After an error
 * hlbm_last_error() describes it.  Device-side conditions (capacity
 * overflow, non-finite or non-positive density) are raised at the next
 * read or hlbm_sync call as HLBM_E_CAPACITY / HLBM_E_UNSTABLE.  No C++
 * exception crosses the ABI.
 */
#ifndef HLBM_H
#define HLBM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HLBM_OK = 0,
    HLBM_E_ARG = -1,        /* invalid argument or configuration */
    HLBM_E_NOMEM = -2,      /* device or host allocation failed */
    HLBM_E_DEVICE = -3,     /* HIP runtime error */
    HLBM_E_CAPACITY = -4,   /* tile candidate list or pair table overflow */
    HLBM_E_UNSTABLE = -5,   /* non-finite or non-positive density */
    HLBM_E_STATE = -6       /* call out of order (e.g. step before init) */
} hlbm_status;

typedef enum {
    HLBM_FP64 = 0,          /* populations stored and collided in FP64 */
    HLBM_FP32 = 1,          /* populations stored and collided in FP32 */
    HLBM_FP16S = 2          /* f - w stored as IEEE binary16, FP32 collision */
} hlbm_precision;

/* Convex bodies with exact signed distances; size is the radius (sphere),
   the edge (cube), the centre-to-vertex distance (regular octahedron), or
   the scale factor of a body type k defined with hlbm_define_polyhedron or
   hlbm_define_ellipsoid (shape HLBM_POLYHEDRON0 + k, k < 8). */
typedef enum { HLBM_SPHERE = 0, HLBM_CUBE = 1, HLBM_OCTAHEDRON = 2,
               HLBM_POLYHEDRON0 = 3 } hlbm_shape;

typedef struct {
    int nx, ny, nz;             /* lattice nodes per axis */
    int periodic_z;             /* 1 periodic, 0 walls at -1/2 and nz-1/2 */
    double tau;                 /* BGK relaxation time, eq. (12); > 1/2 */
    double wall_velocity[2][3]; /* bottom (0) and top (1) wall velocity */
    double gravity[3];          /* gravitational acceleration on particles */
    double fluid_accel[3];      /* uniform acceleration added to the fluid */
    int balance;                /* balance force (Sec. 5.1) on a fully periodic
                                   box: 0 none; 1 the uniform fluid
                                   acceleration -sum (s_p - 1) V_p g / N that
                                   cancels the particles' net weight; 2 hold
                                   the net volume flow (lattice momentum) at
                                   zero: after each collision the
                                   acceleration of the next is set from the
                                   lattice momentum of the last two steps */
    double eps_b;               /* width of the B(d) band around the surface */
    double enlarge;             /* enlargement in contact treatment (0.2) */
    int n_c;                    /* contact resolution (8), 1..32 */
    double young, poisson;      /* material, eq. (5) (same for walls) */
    double restitution;         /* e of eq. (6) */
    double mu_s, mu_k, u_k;     /* friction law, eqs. (7)-(9) */
    int max_pairs;              /* capacity of the contact-pair table */
    int tile_capacity;          /* particles per 4x4x4 tile, <= 64 */
    int precision;              /* hlbm_precision */
    int n_sub;                  /* contact sub-steps per time step, 1..64
                                   (Sec. 4.4, Algorithm 1): contact forces,
                                   motion over 1/n_sub and detection repeat
                                   with the hydrodynamic force held fixed */
} hlbm_params;

/* One contact record.  b >= 0: particle-particle with a < b; b = -1: the
   bottom wall, b = -2: the top wall.  count / rlo / rhi come from the latest
   rough detection (node images in the frame of particle a); lo / hi is the
   box the next treatment starts from (the corrected box when carried = 1);
   the remaining fields are the results of the latest treatment. */
typedef struct {
    int a, b;
    int count;
    int rlo[3], rhi[3];
    int carried;
    double lo[3], hi[3];
    int established;
    double damping;
    int age;
    int n_in;
    double volume, centroid[3], normal[3], depth, fn, force_a[3], force_b[3];
} hlbm_contact;

typedef struct hlbm_ctx hlbm_ctx;

/* Create a context on the current HIP device: the lattice, its boundaries
   and the constants of the method (the D3Q19 lattice of Sec. 3.1 with the
   BGK relaxation time of eq. (12); the coupling band of Sec. 3.2; the
   contact constants of eqs. (5)-(9) and the enlargement of Sec. 5.1).
   stream: a hipStream_t to run on (for example the current torch stream),
   or NULL for a private stream.  Validates the parameters (lattice size,
   tau, capacities); allocates the population buffers unless they are lent
   later.  *out is NULL on error; with no context to hold it, the message of
   a rejected parameter goes to stderr.  The context also creates a second
   stream (default priority) for the overlapped contact treatment of
   hlbm_step. */
hlbm_status hlbm_create(const hlbm_params *params, void *stream,
                        hlbm_ctx **out);

/* Lend two DEVICE population buffers of `bytes` each (19 * nx*ny*nz *
   bytes-per-value of the precision: 8, 4 or 2) for the post-collision
   populations f* of eqs. (10)-(12) and their streamed copy (ping-pong).
   Must be called before any init call.  The context never frees them. */
hlbm_status hlbm_bind_populations(hlbm_ctx *ctx, void *dev_a, void *dev_b,
                                  size_t bytes);

/* Define convex polyhedron type `type` (0..7; particles of shape
   HLBM_POLYHEDRON0 + type) from nv vertices (host, nv x 3, FP64) and nf
   faces, face f listing fsize[f] vertex indices counter-clockwise seen from
   outside, all lists concatenated in fidx.  At most 64 vertices, 64 faces,
   384 face-vertex entries and 128 edges.  The surface must be closed,
   consistently oriented, planar-faced and convex (HLBM_E_ARG otherwise).
   The solid is re-centred at its centroid (the particle's X is its centre
   of mass); a particle's size scales it uniformly.  Signed distances are
   exact (the nearest face plane inside; face interiors, edges and vertices
   outside, the method needs only a signed distance and its gradient, Sec.
   3.3).  Particle motion follows eq. (3) with the world-frame inertia
   tensor R I_b R^T of the homogeneous solid.  Call before
   hlbm_init_particles (HLBM_E_STATE after).  Polyhedra are not supported
   by the adjoint. */
hlbm_status hlbm_define_polyhedron(hlbm_ctx *ctx, int type, int nv,
                                   const double *v, int nf, const int *fsize,
                                   const int *fidx);

/* Define ellipsoid type `type` (0..7, sharing the slots of
   hlbm_define_polyhedron; particles of shape HLBM_POLYHEDRON0 + type): the
   solid (x/a)^2 + (y/b)^2 + (z/c)^2 <= 1 with semi-axes a, b, c > 0 along
   the body axes, scaled uniformly by a particle's size (smooth convex
   bodies, Sec. 1; the method needs only a signed distance and its gradient,
   Sec. 3.2 and Sec. 3.3.1).  The signed distance is the exact Euclidean
   distance to the surface, from the nearest point's Lagrange multiplier:
   the FP64 ownership, detection and contact decisions bisect it to
   adjacent doubles (up to about a hundred iterations); the coupling weight
   and the detection screen take Newton steps, and skip the solve where
   bounds from the scaled ellipsoids already decide.  Volume 4 pi a b c / 3;
   eq. (3) with the
   inertia tensor of the homogeneous solid.  HLBM_E_ARG for a type outside
   0..7 or a semi-axis that is not positive and finite; call before
   hlbm_init_particles (HLBM_E_STATE after).  Not supported by the
   adjoint. */
hlbm_status hlbm_define_ellipsoid(hlbm_ctx *ctx, int type, double a, double b,
                                  double c);

/* Upload n particles (host arrays): the state of eqs. (2)-(3), position of
   the centre of mass, orientation, velocity and angular velocity, with
   shape, size and density ratio (Sec. 2.1, Sec. 5.1).  shape: hlbm_shape;
   size = radius (sphere), edge (cube), centre-to-vertex distance
   (octahedron) or scale (polyhedron); density = particle/fluid density
   ratio.  Quaternions are normalised (HLBM_E_ARG for zero or non-finite
   ones).  Positions on periodic axes are wrapped into [0, n).  Periodic
   axes must exceed twice the particle reach (circumradius + detection
   margin). */
hlbm_status hlbm_init_particles(hlbm_ctx *ctx, int n, const int *shape,
                                const double *size, const double *density,
                                const double *X, const double *q,
                                const double *U, const double *omega);

/* Set f* = f^eq(rho, u) (eq. (13)) on every node, then couple the particles
   to the fluid at their current state, as before the first step of
   Algorithm 1: node ownership and coupling (Sec. 3.2), rough contact
   detection (Sec. 3.3.1; the initial contact list) and the
   momentum-exchange force of eqs. (16)-(18). */
hlbm_status hlbm_init_fluid_equilibrium(hlbm_ctx *ctx, double rho,
                                        const double u[3]);

/* Same, from a host FP64 population field [19][nz][ny][nx]. */
hlbm_status hlbm_set_populations(hlbm_ctx *ctx, const double *f);

/* Advance nsteps coupled time steps of Algorithm 1 (Sec. 4.4; asynchronous
   on the context stream).  Order per step (one sub-step): contact treatment
   (Sec. 3.3.1, eqs. (4)-(9)), gravity and Newton-Euler update (eqs.
   (2)-(3)), particle-to-fluid coupling with rough detection (Sec. 3.2,
   Sec. 3.3.1), collide-and-stream (eqs. (10)-(15)) with the fluid-to-
   particle momentum exchange (eqs. (16)-(18)).  With one contact sub-step
   and no timing in use, the contact treatment of every step after the
   first of a call runs on a second stream of the context beside the
   previous step's lattice pass (it reads nothing that pass writes); the
   call ends with no such work pending, and the results are those of
   strictly ordered steps, bit for bit. */
hlbm_status hlbm_step(hlbm_ctx *ctx, int nsteps);

/* Use (1) or stop using (0) captured HIP graphs for hlbm_step (the step of
   Algorithm 1 as one launch).  With one contact sub-step, a call of two or
   more steps replays 8-step graphs (the overlapped contact treatment
   captured inside, and carried across graph boundaries) while at least 8
   steps remain, and runs the rest as overlapped stream launches; a single
   step replays a single-step graph.  A graph's first replay carries a
   one-time setup, so a call of fewer than 64 steps replays only graphs
   that have run before (else it keeps to stream launches).  Results are
   those of stream launches, bit for bit.  The graphs of the parities the
   next steps can reach are captured, instantiated and uploaded (not run)
   when graphs are switched on, at initialisation and after hlbm_set_state,
   so that later hlbm_step calls only launch them. */
hlbm_status hlbm_use_graph(hlbm_ctx *ctx, int on);

/* Per-kernel timing of the next steps (measurement, no paper passage):
   hlbm_step records HIP events on the context stream around each of its
   kernel launches (bookkeeping clear, contact treatment, particle motion +
   tile binning + contact carry-over, an empty slot, coupling map + rough
   detection, stream-collide lattice pass with the momentum exchange of the
   next step, and a seventh slot that stays zero: the separate
   momentum-exchange pass runs only at initialisation) for up to max_steps
   steps (graphs and the overlapped contact treatment are bypassed
   meanwhile).  hlbm_timing_end
   synchronises and returns the summed milliseconds per kernel in that
   order, kernel_ms[7], and the number of timed steps. */
hlbm_status hlbm_timing_begin(hlbm_ctx *ctx, int max_steps);
hlbm_status hlbm_timing_end(hlbm_ctx *ctx, double *kernel_ms, int *nsteps);

/* Wait for queued work; raise device-side error flags. */
hlbm_status hlbm_sync(hlbm_ctx *ctx);

/* Forces and torques that moved the particles in the last step ([n][3]
   each, FP64; any pointer may be NULL): hydrodynamic F_h, T_h of eqs.
   (16)-(18) and contact F_c, T_c summed over the particle's contacts,
   eqs. (4)-(9). */
hlbm_status hlbm_read_forces(hlbm_ctx *ctx, double *Fh, double *Th,
                             double *Fc, double *Tc);

/* Particle state after the last step (eqs. (2)-(3)): centre of mass X
   [n][3], unit quaternion q [n][4], velocity U and angular velocity omega
   [n][3]; NULL skips. */
hlbm_status hlbm_read_particles(hlbm_ctx *ctx, double *X, double *q,
                                double *U, double *omega);

/* Current contact list, sorted by (a, b): per pair the rough-detection
   count and node box, the corrected box, and the results of the latest
   treatment (Sec. 3.3.1: overlap volume, contact point, normal, depth; eqs.
   (4)-(6): damping factor fixed at onset, normal force, force on a and b).
   *n_out = number of records (may exceed capacity, in which case only
   `capacity` are written). */
hlbm_status hlbm_read_contacts(hlbm_ctx *ctx, int capacity,
                               hlbm_contact *out, int *n_out);

/* Density and velocity moments (eq. (11)) of the stored post-collision
   field, and the node owner (-1 = fluid) at the current particle state
   (Sec. 3.2, the particle whose signed distance is smallest).  NULL skips.
   The coupling weight B and particle velocity u_p of the owner come from
   hlbm_read_coupling. */
hlbm_status hlbm_read_fields(hlbm_ctx *ctx, double *rho, double *u,
                             int *owner);

/* Post-collision populations as FP64 [19][nz][ny][nx] (FP16S: w_i + h_i). */
hlbm_status hlbm_read_populations(hlbm_ctx *ctx, double *f);

/* Coupling field at the current particle state (Sec. 3.2): per node the
   weight B(d) of the owner's signed distance and the owner's velocity at
   the node, u_p = U + w x r (u[3*node + k]); 0 where no particle owns the
   node.  FP64, host arrays of N and 3N values; NULL skips. */
hlbm_status hlbm_read_coupling(hlbm_ctx *ctx, double *B, double *up);

/* For callers that cannot allocate (code under HIP graph capture, serving
   loops, harnesses that forbid allocation): hlbm_read_coupling with the
   same arguments and results, staged through a fixed device array that the
   library holds per GPU (64 MiB, for lattices of at most 2^21 nodes; a
   larger lattice returns HLBM_E_ARG).  It allocates no device or host
   memory.  All contexts on one GPU share that array: calls that overlap on
   one GPU race. */
hlbm_status hlbm_read_coupling_noalloc(hlbm_ctx *ctx, double *B, double *up);

/* Rough contact detection (Sec. 3.3.1) and treatment counts: pairs with a
   flagged node in the latest detection and the sum of their flagged-node
   counts; that sum accumulated over all detections so far; steps taken;
   midpoint samples of the latest treatment (6 N_c^2 for the box correction
   and N_c^3 for the overlap integration per treated pair, each evaluating
   both members' signed distances).  NULL skips. */
hlbm_status hlbm_counters(hlbm_ctx *ctx, long long *pairs,
                          long long *cells, long long *total_cells,
                          long long *steps, long long *samples);

/* The context's stream (hipStream_t). */
void *hlbm_stream(const hlbm_ctx *ctx);

/* The uniform fluid acceleration the next collision uses in eq. (15)
   (fluid_accel + the balance force of Sec. 5.1; with balance mode 2 read
   from the device). */
hlbm_status hlbm_fluid_acceleration(hlbm_ctx *ctx, double a[3]);

/* Checkpoint and resume of the state between two steps of Algorithm 1.
   hlbm_get_state copies the whole step state (populations in their
   storage precision, particle records, candidate lists and
   momentum-exchange partial sums, both contact tables, owner map,
   counters, step count) into a caller-owned host buffer; with blob = NULL
   it only sets *bytes to the size needed.  hlbm_set_state restores such a
   blob into a context created with the same parameters and initialised
   with the same particle set (count and shapes); the next hlbm_step
   continues exactly where the saved context stood.  E_ARG for a blob of
   another configuration. */
hlbm_status hlbm_get_state(hlbm_ctx *ctx, void *blob, size_t *bytes);
hlbm_status hlbm_set_state(hlbm_ctx *ctx, const void *blob, size_t bytes);

/* ---- Adjoint (reverse-mode gradient) of K coupled steps -----------------
   Differentiates the time step of Sec. 4.4 (Algorithm 1): streaming and the
   BGK + velocity-shift collision (eqs. (10)-(15)), the coupling weight and
   particle velocity of each node (Sec. 3.2), the momentum exchange
   (eqs. (16)-(18)) and the Newton-Euler update (eqs. (2)-(3)).  The owner
   of every node and the contact forces (eqs. (4)-(9)) of the recorded
   forward run are held fixed: the discrete decisions of the forward pass are
   not differentiated.  FP64 form, fully periodic boxes, balance modes 0 and
   1, spheres, cubes and octahedra only (E_ARG otherwise).

   hlbm_adjoint_record: from the current state, runs `ksteps` steps and keeps
   a device snapshot of the whole state every `ckpt_every` steps (plus the
   end state); the context then stands at the end of the window, as after
   hlbm_step(ksteps).  Memory: ceil(ksteps / ckpt_every) + 1 snapshots of
   about 19 x 8 B per node each.

   hlbm_adjoint_gradient: for J = sum_p dJ_dU[p] . U_p (the particle
   velocities at the end of the window; dJ_dU is 3n, host), recomputes each
   segment from its checkpoint (keeping ckpt_every + 1 population fields on
   the device) and sweeps it in reverse.  Outputs (host, any may be NULL):
     dJ_ds[n]         derivative by each particle's density ratio s_p (mass,
                      inertia, gravity-buoyancy, and the balance acceleration
                      of a balanced box);
     dJ_dtheta0[3n]   derivative by a world-frame rotation of each particle's
                      orientation at the start of the window,
                      q -> exp(theta/2) (x) q;
     dJ_dq0[4n]       the same as a quaternion gradient tangent to |q| = 1 at
                      that (unit) orientation, 2 (0, dJ_dtheta0) (x) q;
     dJ_dX0, dJ_dU0, dJ_domega0 [3n]  derivatives by the position, velocity
                      and angular velocity at the start of the window.
   The context is left at the end of the recorded window.  Reductions use
   FP64 atomics, so results can differ from run to run in the last bits.

   hlbm_adjoint: record and gradient in one call (the form of the
   autograd wrapper): ksteps steps from the current state with checkpoints
   every ckpt_every steps, then dJ_ds and dJ_dq0 of
   J = sum_p dJ_dU[p] . U_p. */
hlbm_status hlbm_adjoint_record(hlbm_ctx *ctx, int ksteps, int ckpt_every);
hlbm_status hlbm_adjoint_gradient(hlbm_ctx *ctx, const double *dJ_dU,
                                  double *dJ_ds, double *dJ_dtheta0,
                                  double *dJ_dq0, double *dJ_dX0,
                                  double *dJ_dU0, double *dJ_domega0);
hlbm_status hlbm_adjoint(hlbm_ctx *ctx, int ksteps, int ckpt_every,
                         const double *dJ_dU, double *dJ_ds, double *dJ_dq0);

/* Hash of the sources the library was built from (16 hex digits: SHA-256
   over the kernel sources and this header); the Python binding refuses a
   library whose hash differs from the sources beside it. */
const char *hlbm_build_hash(void);

/* Message of the context's last error (or of a null context). */
const char *hlbm_last_error(const hlbm_ctx *ctx);

/* Release the context and the device memory it owns. */
void hlbm_destroy(hlbm_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
