/*
 * FP64 CPU oracle of the coupled HLBM + discrete-contact time step of
 * Marquardt, Hafen & Krause, "A novel model for direct numerical simulation
 * of suspension dynamics with arbitrarily shaped convex particles"
 * (arXiv 2401.10878).
 *
 * TEST INFRASTRUCTURE ONLY.  The product library never links, loads or calls
 * this code; only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no source, header, table or helper with
 * the GPU path: every constant below is written out again from the paper.
 *
 * The oracle follows the paper's equations in plain serial loops (OpenMP only
 * over independent per-cell updates).  Where the paper leaves a detail open
 * the reading used is stated at the function that applies it.
 *
 * Conventions: lattice units (Sec. 3, Delta x = Delta t = 1); nodes at integer
 * coordinates 0 <= x < n; populations stored f[i][z][y][x]; x and y are
 * periodic; z is periodic or bounded by walls at z = -1/2 and z = nz - 1/2.
 */
#ifndef HLBM_ORACLE_H
#define HLBM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_Q 19
#define ORC_MAXK 8          /* particles per node in the detection set */

typedef struct {
    int nx, ny, nz;
    int periodic_z;          /* 1 periodic, 0 walls at -1/2 and nz-1/2 */
    double tau;              /* BGK relaxation time, eq. (12) */
    double wall_u[2][3];     /* velocity of the bottom (0) and top (1) wall */
    double gravity[3];       /* gravitational acceleration on particles */
    double fluid_accel[3];   /* uniform acceleration added to the fluid */
    int balance;             /* balance force on a fully periodic box:
                                0 none; 1 cancel the particles' net weight;
                                2 hold the lattice momentum at zero */
    double eps;              /* width of the B(d) transition band */
    double delta_c;          /* enlargement during contact treatment */
    int n_c;                 /* contact resolution */
    double young, poisson, restitution, mu_s, mu_k, u_k;
    int n_sub;               /* contact sub-steps per time step (>= 1) */
} orc_params;

typedef struct {
    int shape;               /* 0 sphere, 1 cube, 2 regular octahedron */
    double size;             /* sphere radius or cube edge */
    double dens;             /* particle / fluid density ratio */
    double X[3], q[4], U[3], w[3];
} orc_particle;

typedef struct {
    int a, b;                /* a < b particle ids; b = -1 bottom, -2 top wall */
    int count;               /* nodes flagged by the latest rough detection */
    int rlo[3], rhi[3];      /* node-image bounds of the latest detection */
    int carried;             /* lo/hi is a corrected box carried over */
    double lo[3], hi[3];     /* box used by the next treatment */
    int established;         /* contact has had V > 0 */
    double damping;          /* c of eq. (6), fixed at onset */
    int age;
    /* results of the latest treatment */
    int n_in;
    double volume, centroid[3], normal[3], depth, fn, force_a[3], force_b[3];
} orc_contact;

typedef struct orc_sim orc_sim;

/* ---- whole-simulation interface ---- */
orc_sim *orc_create(const orc_params *P, int np, const int *shape,
                    const double *size, const double *dens, const double *X,
                    const double *q, const double *U, const double *w);
void orc_destroy(orc_sim *S);
int orc_threads(void);
/* f* := f^eq(rho, u) everywhere, then coupling and detection at S(0) */
int orc_init_equilibrium(orc_sim *S, double rho, const double u[3]);
/* f* := given array [19][nz][ny][nx], then coupling and detection */
int orc_set_populations(orc_sim *S, const double *fs);
int orc_step(orc_sim *S, int nsteps);
long orc_step_count(const orc_sim *S);
const char *orc_error(const orc_sim *S);

void orc_get_populations(const orc_sim *S, double *fs);
void orc_get_fields(const orc_sim *S, double *rho, double *u, int *owner,
                    double *B, double *up);
void orc_get_collision_diag(const orc_sim *S, double *rho, double *J,
                            double *du);
void orc_get_post_stream(const orc_sim *S, double *f);
void orc_get_particles(const orc_sim *S, double *X, double *q, double *U,
                       double *w);
void orc_get_forces(const orc_sim *S, double *Fh, double *Th, double *Fc,
                    double *Tc);
int orc_num_contacts(const orc_sim *S);
void orc_get_contacts(const orc_sim *S, orc_contact *out);
void orc_get_counters(const orc_sim *S, long long *pairs, long long *cells);
void orc_get_mea_cells(const orc_sim *S, double *Scell);
void orc_get_balance(const orc_sim *S, double *a_ext);

/* ---- pieces exposed for closed-form and brute-force checks ---- */
void orc_feq(double rho, const double u[3], double out[ORC_Q]);
void orc_lattice(int c[ORC_Q][3], double w[ORC_Q], int opp[ORC_Q]);
void orc_rotation(const double q[4], double R[9]);
/* Convex polyhedra: shapes ORC_POLY0 .. ORC_POLY0 + ORC_MAXPOLY - 1 refer to
   polyhedron types defined here (before orc_create).  Vertices (nv x 3,
   body frame) and faces (nf vertex lists, counter-clockwise seen from
   outside, fsize[f] entries each, concatenated in fidx).  The solid is
   re-centred at its centroid; a particle's size scales it uniformly.
   Returns 0, or -1 with a message in orc_poly_error() when the input is
   not a closed convex polyhedron within the capacities. */
#define ORC_POLY0 3
#define ORC_MAXPOLY 8
int orc_define_polyhedron(int type, int nv, const double *v, int nf,
                          const int *fsize, const int *fidx);
const char *orc_poly_error(void);
/* Ellipsoid type `type` (same shape codes as the polyhedra): semi-axes a, b,
   c along the body axes at unit scale, scaled by a particle's size. */
int orc_define_ellipsoid(int type, double a, double b, double c);
/* half extent along world axis k of a particle (the node range visited
   around it) */
double orc_half_extent(int shape, double size, const double q[4], int k);
/* unit-scale volume, second moment J = int p p^T dV about the centroid,
   circumradius, and the re-centred vertices (nv x 3) of a defined type */
int orc_poly_info(int type, double *vol, double J[9], double *rc, double *v);
/* R I_b^-1 R^T T for a polyhedron particle (eq. (3), world frame) */
void orc_poly_angular_accel(int shape, double size, double dens,
                            const double q[4], const double T[3], double dw[3]);

double orc_sdf(int shape, double size, const double R[9], const double r[3],
               double grad[3]);
double orc_weight(double d, double eps);
double orc_friction_mu(double a, double mu_s, double mu_k);
double orc_damping(double e, double u0);
double orc_effective_modulus(double Ea, double nua, double Eb, double nub);
/* static treatment of one pair (or particle-wall pair, b < 0) from a box;
   npass correction passes (0 = none) then integration; forces included. */
void orc_treat_pair(const orc_params *P, const orc_particle *pa,
                    const orc_particle *pb, int b_id, int npass,
                    double lo[3], double hi[3], orc_contact *out);
/* eqs. (4)-(9) alone for a contact record whose volume, depth, centroid,
   normal, established flag and damping factor the caller sets (pb NULL: a
   wall partner at rest); writes fn, force_a, force_b and, at onset, the
   damping factor. */
void orc_contact_force_of(const orc_params *P, const orc_particle *pa,
                          const orc_particle *pb, orc_contact *c);

#ifdef __cplusplus
}
#endif
#endif
