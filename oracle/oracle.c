/*
 * FP64 CPU oracle of the coupled HLBM + discrete-contact time step
 * (arXiv 2401.10878).  TEST INFRASTRUCTURE ONLY -- see oracle.h.
 *
 * Build: gcc -O2 -std=c99 -ffp-contract=off -fopenmp -fPIC -shared
 * (no FMA contraction: the signed-distance and predicate arithmetic must be
 * evaluated exactly in the order written, left to right).
 */
#define _POSIX_C_SOURCE 200809L
#include "oracle.h"

#include <float.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ======================================================================
 * D3Q19 velocity set (Sec. 3.1).  The paper names the set but prints no
 * table; these are the textbook velocities and Gauss-Hermite weights with
 * c_s^2 = 1/3.  Order: rest, the six axis directions (+x,-x,+y,-y,+z,-z),
 * then the twelve edge directions, each followed by its opposite.
 * ====================================================================== */
static const int CV[ORC_Q][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
static const double WT[ORC_Q] = {
    1.0 / 3.0,
    1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const double CS2 = 1.0 / 3.0;

static int opposite(int i)
{
    /* the velocity with c = -c_i: find it by search, so the table order
       above is the only place that fixes the layout */
    for (int j = 0; j < ORC_Q; ++j)
        if (CV[j][0] == -CV[i][0] && CV[j][1] == -CV[i][1] &&
            CV[j][2] == -CV[i][2])
            return j;
    return -1;
}

void orc_lattice(int c[ORC_Q][3], double w[ORC_Q], int opp[ORC_Q])
{
    for (int i = 0; i < ORC_Q; ++i) {
        for (int k = 0; k < 3; ++k) c[i][k] = CV[i][k];
        w[i] = WT[i];
        opp[i] = opposite(i);
    }
}

/* eq. (13), with the sign of the u.u term taken as minus: the printed plus
   sign does not conserve mass (sum_i f_i^eq != rho for u != 0), the minus
   sign is the second-order Maxwell-Boltzmann expansion. */
void orc_feq(double rho, const double u[3], double out[ORC_Q])
{
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < ORC_Q; ++i) {
        double cu = CV[i][0] * u[0] + CV[i][1] * u[1] + CV[i][2] * u[2];
        out[i] = WT[i] * rho *
                 (1.0 + cu / CS2 + (cu * cu) / (2.0 * CS2 * CS2) -
                  uu / (2.0 * CS2));
    }
}

/* ======================================================================
 * Geometry: rotation, signed distance functions, coupling weight.
 * ====================================================================== */

/* Rotation matrix of the unit quaternion q = (w, x, y, z); R maps body to
   world coordinates.  Row-major R[3*row + col]. */
void orc_rotation(const double q[4], double R[9])
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1.0 - 2.0 * (y * y + z * z);
    R[1] = 2.0 * (x * y - w * z);
    R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);
    R[4] = 1.0 - 2.0 * (x * x + z * z);
    R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);
    R[7] = 2.0 * (y * z + w * x);
    R[8] = 1.0 - 2.0 * (x * x + y * y);
}

/* Regular octahedron |x| + |y| + |z| <= a (size = a, the centre-to-vertex
   distance), body frame.  Folded into the positive octant (q = |p|), the
   surface there is the triangle A = (a,0,0), B = (0,a,0), C = (0,0,a) on
   the plane x + y + z = a.  Inside, the nearest surface point lies on that
   face plane; outside, it is the closest point of the triangle: on the face
   when the projection onto the plane lands inside it (all coordinates of
   the projection >= 0), else on one of its three edges.  gq receives the
   gradient with respect to q (unit length). */
static double octa_sdf_q(double a, const double q[3], double gq[3])
{
    const double inv3 = 0.57735026918962584;      /* 1 / sqrt(3) */
    double s = (q[0] + q[1]) + q[2];
    double pd = (s - a) * inv3;                    /* signed plane distance */
    double t[3];
    for (int k = 0; k < 3; ++k) t[k] = q[k] - (s - a) / 3.0;
    if (s <= a || (t[0] >= 0.0 && t[1] >= 0.0 && t[2] >= 0.0)) {
        for (int k = 0; k < 3; ++k) gq[k] = inv3;
        return pd;
    }
    /* closest point on the edges A-B, B-C, C-A */
    double best = 1e300, bc[3] = {0.0, 0.0, 0.0};
    for (int e = 0; e < 3; ++e) {
        int i = e, j = (e + 1) % 3;               /* vertex a e_i to a e_j */
        /* segment P0 = a e_i, P1 = a e_j, direction (P1 - P0) */
        double u = ((q[j] - q[i]) + a) / (2.0 * a);
        if (u < 0.0) u = 0.0;
        if (u > 1.0) u = 1.0;
        double cp[3] = {0.0, 0.0, 0.0};
        cp[i] = a * (1.0 - u);
        cp[j] = a * u;
        double dx = q[0] - cp[0], dy = q[1] - cp[1], dz = q[2] - cp[2];
        double d2 = (dx * dx + dy * dy) + dz * dz;
        if (d2 < best) {
            best = d2;
            bc[0] = cp[0]; bc[1] = cp[1]; bc[2] = cp[2];
        }
    }
    double d = sqrt(best);
    for (int k = 0; k < 3; ++k) gq[k] = d > 0.0 ? (q[k] - bc[k]) / d : inv3;
    return d;
}

/* ======================================================================
 * Convex polyhedra (arbitrary convex bodies, Sec. 1 and Sec. 3.3: the
 * method needs only a signed distance and its gradient).  A type is given
 * by vertices and faces; the face planes n_f . p <= h_f follow from the
 * face polygons (Newell's normal, offset through the face's vertex mean).
 * ====================================================================== */
static void cross(const double a[3], const double b[3], double out[3]);

#define ORC_PV 64
#define ORC_PF 64
#define ORC_PFV 384
#define ORC_PE 128

typedef struct {
    int nv, nf, ne;
    int kind;                   /* 0 polyhedron, 1 ellipsoid */
    double ax[3];               /* ellipsoid semi-axes (unit scale) */
    double v[ORC_PV][3];
    double n[ORC_PF][3], h[ORC_PF];
    int fs[ORC_PF + 1], fv[ORC_PFV];
    int e[ORC_PE][2];
    double vol, J[9], rc;
} orc_poly;

static orc_poly g_poly[ORC_MAXPOLY];
static int g_poly_ok[ORC_MAXPOLY];
static char g_poly_err[160];

const char *orc_poly_error(void) { return g_poly_err; }

static int poly_fail(const char *msg)
{
    snprintf(g_poly_err, sizeof g_poly_err, "%s", msg);
    return -1;
}

int orc_define_polyhedron(int type, int nv, const double *v, int nf,
                          const int *fsize, const int *fidx)
{
    if (type < 0 || type >= ORC_MAXPOLY) return poly_fail("type out of range");
    g_poly_ok[type] = 0;
    if (nv < 4 || nv > ORC_PV || nf < 4 || nf > ORC_PF)
        return poly_fail("vertex or face count out of range");
    orc_poly P;
    memset(&P, 0, sizeof P);
    P.nv = nv;
    P.nf = nf;
    for (int i = 0; i < nv; ++i)
        for (int k = 0; k < 3; ++k) P.v[i][k] = v[3 * i + k];
    int m = 0;
    for (int f = 0; f < nf; ++f) {
        if (fsize[f] < 3) return poly_fail("face with fewer than 3 vertices");
        P.fs[f] = m;
        for (int j = 0; j < fsize[f]; ++j) {
            if (m >= ORC_PFV) return poly_fail("too many face-vertex entries");
            int a = fidx[m];
            if (a < 0 || a >= nv) return poly_fail("face vertex index out of range");
            P.fv[m++] = a;
        }
    }
    P.fs[nf] = m;
    /* closed, consistently oriented surface: every directed edge once, and
       its reverse once; collect the undirected edges */
    for (int f = 0; f < nf; ++f) {
        int c = P.fs[f + 1] - P.fs[f];
        for (int j = 0; j < c; ++j) {
            int a = P.fv[P.fs[f] + j], b = P.fv[P.fs[f] + (j + 1) % c];
            if (a == b) return poly_fail("repeated vertex in a face");
            int same = 0, rev = 0;
            for (int g = 0; g < nf; ++g) {
                int cg = P.fs[g + 1] - P.fs[g];
                for (int t = 0; t < cg; ++t) {
                    int x = P.fv[P.fs[g] + t], y = P.fv[P.fs[g] + (t + 1) % cg];
                    if (x == a && y == b) ++same;
                    if (x == b && y == a) ++rev;
                }
            }
            if (same != 1 || rev != 1) return poly_fail("surface not closed or not consistently oriented");
            if (a < b) {
                if (P.ne >= ORC_PE) return poly_fail("too many edges");
                P.e[P.ne][0] = a;
                P.e[P.ne][1] = b;
                ++P.ne;
            }
        }
    }
    if (nv - P.ne + nf != 2) return poly_fail("Euler characteristic is not 2");
    /* volume and centroid: tetrahedra (0, v0, v_j, v_{j+1}) of each face fan */
    double vol = 0.0, cen[3] = {0.0, 0.0, 0.0};
    for (int f = 0; f < nf; ++f) {
        int c = P.fs[f + 1] - P.fs[f];
        const double *a = P.v[P.fv[P.fs[f]]];
        for (int j = 1; j + 1 < c; ++j) {
            const double *b = P.v[P.fv[P.fs[f] + j]], *d = P.v[P.fv[P.fs[f] + j + 1]];
            double t = (a[0] * (b[1] * d[2] - b[2] * d[1]) - a[1] * (b[0] * d[2] - b[2] * d[0]) +
                        a[2] * (b[0] * d[1] - b[1] * d[0])) / 6.0;
            vol += t;
            for (int k = 0; k < 3; ++k) cen[k] += t * (a[k] + b[k] + d[k]) / 4.0;
        }
    }
    if (!(vol > 0.0)) return poly_fail("faces must run counter-clockwise seen from outside");
    for (int k = 0; k < 3; ++k) cen[k] /= vol;
    for (int i = 0; i < nv; ++i)
        for (int k = 0; k < 3; ++k) P.v[i][k] -= cen[k];
    P.vol = vol;
    /* second moment about the centroid: per tetrahedron with a vertex at the
       origin, int p p^T = V/20 (sum_k v_k v_k^T + (sum v_k)(sum v_k)^T) */
    for (int f = 0; f < nf; ++f) {
        int c = P.fs[f + 1] - P.fs[f];
        const double *a = P.v[P.fv[P.fs[f]]];
        for (int j = 1; j + 1 < c; ++j) {
            const double *b = P.v[P.fv[P.fs[f] + j]], *d = P.v[P.fv[P.fs[f] + j + 1]];
            double t = (a[0] * (b[1] * d[2] - b[2] * d[1]) - a[1] * (b[0] * d[2] - b[2] * d[0]) +
                        a[2] * (b[0] * d[1] - b[1] * d[0])) / 6.0;
            for (int r = 0; r < 3; ++r)
                for (int q = 0; q < 3; ++q) {
                    double sv = a[r] + b[r] + d[r], sw = a[q] + b[q] + d[q];
                    P.J[3 * r + q] += t / 20.0 *
                        (a[r] * a[q] + b[r] * b[q] + d[r] * d[q] + sv * sw);
                }
        }
    }
    /* face planes */
    double scale = 0.0;
    for (int i = 0; i < nv; ++i) {
        double r = sqrt(P.v[i][0] * P.v[i][0] + P.v[i][1] * P.v[i][1] + P.v[i][2] * P.v[i][2]);
        if (r > scale) scale = r;
    }
    P.rc = scale;
    /* two distinct vertex indices at the same point make an edge of no length */
    for (int f = 0; f < nf; ++f) {
        int c = P.fs[f + 1] - P.fs[f];
        for (int j = 0; j < c; ++j) {
            const double *a = P.v[P.fv[P.fs[f] + j]], *b = P.v[P.fv[P.fs[f] + (j + 1) % c]];
            double e2 = (b[0] - a[0]) * (b[0] - a[0]) + (b[1] - a[1]) * (b[1] - a[1]) +
                        (b[2] - a[2]) * (b[2] - a[2]);
            if (!(sqrt(e2) > 1e-9 * scale)) return poly_fail("zero-length edge");
        }
    }
    for (int f = 0; f < nf; ++f) {
        int c = P.fs[f + 1] - P.fs[f];
        double nn[3] = {0.0, 0.0, 0.0}, mean[3] = {0.0, 0.0, 0.0};
        for (int j = 0; j < c; ++j) {
            const double *a = P.v[P.fv[P.fs[f] + j]], *b = P.v[P.fv[P.fs[f] + (j + 1) % c]];
            nn[0] += (a[1] - b[1]) * (a[2] + b[2]);
            nn[1] += (a[2] - b[2]) * (a[0] + b[0]);
            nn[2] += (a[0] - b[0]) * (a[1] + b[1]);
            for (int k = 0; k < 3; ++k) mean[k] += a[k] / c;
        }
        double len = sqrt(nn[0] * nn[0] + nn[1] * nn[1] + nn[2] * nn[2]);
        if (!(len > 0.0)) return poly_fail("degenerate face");
        for (int k = 0; k < 3; ++k) P.n[f][k] = nn[k] / len;
        P.h[f] = P.n[f][0] * mean[0] + P.n[f][1] * mean[1] + P.n[f][2] * mean[2];
        /* planar face, every vertex on the inner side (convexity) */
        for (int i = 0; i < nv; ++i) {
            double s = P.n[f][0] * P.v[i][0] + P.n[f][1] * P.v[i][1] + P.n[f][2] * P.v[i][2] - P.h[f];
            if (s > 1e-9 * scale) return poly_fail("not convex (a vertex lies outside a face plane)");
        }
        for (int j = 0; j < c; ++j) {
            const double *a = P.v[P.fv[P.fs[f] + j]];
            double s = P.n[f][0] * a[0] + P.n[f][1] * a[1] + P.n[f][2] * a[2] - P.h[f];
            if (fabs(s) > 1e-9 * scale) return poly_fail("face not planar");
        }
    }
    g_poly[type] = P;
    g_poly_ok[type] = 1;
    g_poly_err[0] = 0;
    return 0;
}

/* Ellipsoid type: the solid sum_k (p_k / e_k)^2 <= 1 with semi-axes e along
   the body axes, scaled uniformly by a particle's size (the smooth convex
   bodies of Sec. 1; the method needs only the signed distance, Sec. 3.2 and
   Sec. 3.3.1).  Volume 4 pi e0 e1 e2 / 3; second moment about the centre
   int p_k^2 dV = V e_k^2 / 5. */
int orc_define_ellipsoid(int type, double a, double b, double c)
{
    if (type < 0 || type >= ORC_MAXPOLY) return poly_fail("type out of range");
    g_poly_ok[type] = 0;
    if (!(a > 0.0 && b > 0.0 && c > 0.0) || !isfinite(a) || !isfinite(b) || !isfinite(c))
        return poly_fail("ellipsoid semi-axes must be positive and finite");
    orc_poly P;
    memset(&P, 0, sizeof P);
    P.kind = 1;
    P.ax[0] = a;
    P.ax[1] = b;
    P.ax[2] = c;
    P.vol = 4.0 / 3.0 * M_PI * a * b * c;
    P.J[0] = P.vol * a * a / 5.0;
    P.J[4] = P.vol * b * b / 5.0;
    P.J[8] = P.vol * c * c / 5.0;
    P.rc = a > b ? (a > c ? a : c) : (b > c ? b : c);
    g_poly[type] = P;
    g_poly_ok[type] = 1;
    g_poly_err[0] = 0;
    return 0;
}

int orc_poly_info(int type, double *vol, double J[9], double *rc, double *v)
{
    if (type < 0 || type >= ORC_MAXPOLY || !g_poly_ok[type]) return -1;
    const orc_poly *P = &g_poly[type];
    if (vol) *vol = P->vol;
    if (J) for (int k = 0; k < 9; ++k) J[k] = P->J[k];
    if (rc) *rc = P->rc;
    if (v) for (int i = 0; i < P->nv; ++i) for (int k = 0; k < 3; ++k) v[3 * i + k] = P->v[i][k];
    return 0;
}

/* Signed distance of the unit-scale polyhedron at body point p, and its
   body-frame gradient gb.  Inside (every plane distance <= 0) the nearest
   boundary point lies on the nearest face plane: d = max_f (n_f . p - h_f),
   gradient n_f of the first maximal face.  Outside, the nearest point is in
   the interior of a face whose plane the point is above (its projection
   inside the face polygon), or on an edge; d is the smallest of those
   candidate distances (first face, then edges in order, on ties). */
static double poly_sdf_unit(const orc_poly *P, const double p[3], double gb[3])
{
    double best = -1e300;
    int fm = 0;
    double dist[ORC_PF];
    for (int f = 0; f < P->nf; ++f) {
        dist[f] = (P->n[f][0] * p[0] + P->n[f][1] * p[1]) + P->n[f][2] * p[2] - P->h[f];
        if (dist[f] > best) {
            best = dist[f];
            fm = f;
        }
    }
    if (best <= 0.0) {
        if (gb) for (int k = 0; k < 3; ++k) gb[k] = P->n[fm][k];
        return best;
    }
    double dmin2 = 1e300, cp[3] = {0.0, 0.0, 0.0};
    int face_hit = -1;
    for (int f = 0; f < P->nf; ++f) {
        if (dist[f] <= 0.0) continue;
        double q[3];
        for (int k = 0; k < 3; ++k) q[k] = p[k] - dist[f] * P->n[f][k];
        int c = P->fs[f + 1] - P->fs[f], inside = 1;
        for (int j = 0; j < c && inside; ++j) {
            const double *a = P->v[P->fv[P->fs[f] + j]], *b = P->v[P->fv[P->fs[f] + (j + 1) % c]];
            double e[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
            double w[3] = {q[0] - a[0], q[1] - a[1], q[2] - a[2]};
            double x[3];
            cross(e, w, x);
            if ((x[0] * P->n[f][0] + x[1] * P->n[f][1]) + x[2] * P->n[f][2] < 0.0) inside = 0;
        }
        if (inside && dist[f] * dist[f] < dmin2) {
            dmin2 = dist[f] * dist[f];
            face_hit = f;
            for (int k = 0; k < 3; ++k) cp[k] = q[k];
        }
    }
    for (int i = 0; i < P->ne; ++i) {
        const double *a = P->v[P->e[i][0]], *b = P->v[P->e[i][1]];
        double e[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
        double w[3] = {p[0] - a[0], p[1] - a[1], p[2] - a[2]};
        double ee = (e[0] * e[0] + e[1] * e[1]) + e[2] * e[2];
        double t = ((w[0] * e[0] + w[1] * e[1]) + w[2] * e[2]) / ee;
        if (t < 0.0) t = 0.0;
        if (t > 1.0) t = 1.0;
        double c[3] = {a[0] + t * e[0], a[1] + t * e[1], a[2] + t * e[2]};
        double dx = p[0] - c[0], dy = p[1] - c[1], dz = p[2] - c[2];
        double d2 = (dx * dx + dy * dy) + dz * dz;
        if (d2 < dmin2) {
            dmin2 = d2;
            face_hit = -1;
            for (int k = 0; k < 3; ++k) cp[k] = c[k];
        }
    }
    double d = sqrt(dmin2);
    if (gb) {
        if (face_hit >= 0) {
            for (int k = 0; k < 3; ++k) gb[k] = P->n[face_hit][k];
        } else {
            for (int k = 0; k < 3; ++k) gb[k] = (p[k] - cp[k]) / d;
        }
    }
    return d;
}

/* Signed distance of the unit-scale ellipsoid with semi-axes e at body
   point p: the Euclidean distance to the nearest surface point x, negative
   inside, and the body-frame gradient (the unit outward normal at x).
   By symmetry p is folded into the positive octant, y_k = |p_k|.  At the
   nearest point y - x is along the normal (x_k / e_k^2), so x_k = e_k^2 y_k /
   (t + e_k^2) for a multiplier t that solves
       G(t) = sum_k (e_k y_k / (t + e_k^2))^2 - 1 = 0
   (t > 0 outside, t < 0 inside).  With m the smallest e_k^2, G decreases
   monotonically on t > -m (terms with y_k = 0 vanish) and its root there is
   the nearest point when some axis with e_k^2 = m has y_k > 0 (G grows
   without bound towards -m), or when all of those have y_k = 0 and the limit
   of G at -m is still positive.  Otherwise (a point near the centre, on the
   plane across the shortest axes) the nearest point has t = -m: the longer
   axes take x_k = e_k^2 y_k / (e_k^2 - m), the first shortest axis the rest
   of the unit sum.  The root is bracketed ([-m + e_k y_k or -m, |e y| - m],
   with G >= 0 and G <= 0 at the ends) and bisected down to adjacent doubles. */
static double ellipsoid_g(const double e[3], const double e2[3], const double y[3], double t)
{
    double g = -1.0;
    for (int k = 0; k < 3; ++k)
        if (y[k] > 0.0) {
            double r = e[k] * y[k] / (t + e2[k]);
            g += r * r;
        }
    return g;
}

static double ellipsoid_sdf_unit(const double e[3], const double p[3], double gb[3])
{
    double y[3], e2[3], x[3], t;
    for (int k = 0; k < 3; ++k) {
        y[k] = fabs(p[k]);
        e2[k] = e[k] * e[k];
    }
    double m = e2[0];
    for (int k = 1; k < 3; ++k)
        if (e2[k] < m) m = e2[k];
    int kmin = -1;                 /* first shortest axis with y_k > 0 */
    for (int k = 0; k < 3; ++k)
        if (kmin < 0 && e2[k] == m && y[k] > 0.0) kmin = k;
    int root = 1;
    if (kmin < 0) {
        double g = -1.0;
        for (int k = 0; k < 3; ++k)
            if (e2[k] > m && y[k] > 0.0) {
                double r = e[k] * y[k] / (e2[k] - m);
                g += r * r;
            }
        root = g > 0.0;
    }
    if (root) {
        double s = 0.0;
        for (int k = 0; k < 3; ++k) s += (e[k] * y[k]) * (e[k] * y[k]);
        double lo = kmin >= 0 ? e[kmin] * y[kmin] - m : -m;
        double hi = sqrt(s) - m;
        if (hi < lo) hi = lo;      /* a single term: the root is lo itself */
        for (int it = 0; it < 2200; ++it) {
            double tm = 0.5 * (lo + hi);
            if (tm == lo || tm == hi) break;
            double g = ellipsoid_g(e, e2, y, tm);
            if (g > 0.0) lo = tm;
            else if (g < 0.0) hi = tm;
            else {
                lo = tm;
                hi = tm;
            }
        }
        t = lo;
        for (int k = 0; k < 3; ++k) x[k] = e2[k] * y[k] / (t + e2[k]);
    } else {
        t = -m;
        double s = 1.0;
        int kf = -1;
        for (int k = 0; k < 3; ++k) {
            if (e2[k] > m) {
                x[k] = e2[k] * y[k] / (e2[k] - m);
                s -= (x[k] / e[k]) * (x[k] / e[k]);
            } else {
                x[k] = 0.0;
                if (kf < 0) kf = k;
            }
        }
        x[kf] = e[kf] * sqrt(s > 0.0 ? s : 0.0);
    }
    double dx = y[0] - x[0], dy = y[1] - x[1], dz = y[2] - x[2];
    double d = sqrt((dx * dx + dy * dy) + dz * dz);
    if (gb) {
        double n[3];
        for (int k = 0; k < 3; ++k) n[k] = x[k] / e2[k];
        double nn = sqrt((n[0] * n[0] + n[1] * n[1]) + n[2] * n[2]);
        for (int k = 0; k < 3; ++k) gb[k] = (p[k] < 0.0 ? -n[k] : n[k]) / nn;
    }
    return t < 0.0 ? -d : d;
}

/* Exact Euclidean signed distance (negative inside) of a sphere (size =
   radius), cube (size = edge) or regular octahedron (size = centre-to-vertex
   distance) at world offset r from its centre.  The paper maps B from a
   level-set function (Sec. 3.2) and evaluates signed distances at nodes
   (Sec. 3.3.1) for arbitrary convex bodies; sphere and cube are the shapes
   of its experiments, the octahedron a further convex body.  grad (may be
   NULL) is the world-frame gradient; inside a cube it is the normal of the
   nearest face (ties to the lowest axis), and at the exact centre of a
   sphere it is zero. */
double orc_sdf(int shape, double size, const double R[9], const double r[3],
               double grad[3])
{
    if (shape >= ORC_POLY0) {
        const orc_poly *P = &g_poly[shape - ORC_POLY0];
        double p[3], gb[3];
        for (int k = 0; k < 3; ++k)
            p[k] = (R[0 + k] * r[0] + R[3 + k] * r[1] + R[6 + k] * r[2]) / size;
        double d = size * (P->kind == 1 ? ellipsoid_sdf_unit(P->ax, p, grad ? gb : NULL)
                                          : poly_sdf_unit(P, p, grad ? gb : NULL));
        if (grad)
            for (int k = 0; k < 3; ++k)
                grad[k] = R[3 * k + 0] * gb[0] + R[3 * k + 1] * gb[1] +
                          R[3 * k + 2] * gb[2];
        return d;
    }
    if (shape == 2) {
        double p[3], q[3], gq[3];
        for (int k = 0; k < 3; ++k) {
            p[k] = R[0 + k] * r[0] + R[3 + k] * r[1] + R[6 + k] * r[2];
            q[k] = fabs(p[k]);
        }
        double d = octa_sdf_q(size, q, gq);
        if (grad) {
            double gb[3];
            for (int k = 0; k < 3; ++k) gb[k] = (p[k] < 0.0 ? -1.0 : 1.0) * gq[k];
            for (int k = 0; k < 3; ++k)
                grad[k] = R[3 * k + 0] * gb[0] + R[3 * k + 1] * gb[1] +
                          R[3 * k + 2] * gb[2];
        }
        return d;
    }
    if (shape == 0) {
        double n2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        double n = sqrt(n2);
        if (grad) {
            for (int k = 0; k < 3; ++k) grad[k] = n > 0.0 ? r[k] / n : 0.0;
        }
        return n - size;
    }
    double h = 0.5 * size;
    double p[3], qd[3], m[3];
    for (int k = 0; k < 3; ++k) {
        /* body frame: p = R^T r */
        p[k] = R[0 + k] * r[0] + R[3 + k] * r[1] + R[6 + k] * r[2];
        qd[k] = fabs(p[k]) - h;
        m[k] = fmax(qd[k], 0.0);
    }
    double outside = sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
    double inside = fmin(fmax(fmax(qd[0], qd[1]), qd[2]), 0.0);
    if (grad) {
        double gb[3] = {0.0, 0.0, 0.0};
        if (outside > 0.0) {
            for (int k = 0; k < 3; ++k)
                gb[k] = (p[k] < 0.0 ? -1.0 : 1.0) * m[k] / outside;
        } else {
            int km = 0;
            for (int k = 1; k < 3; ++k)
                if (qd[k] > qd[km]) km = k;
            gb[km] = p[km] < 0.0 ? -1.0 : 1.0;
        }
        for (int k = 0; k < 3; ++k)
            grad[k] = R[3 * k + 0] * gb[0] + R[3 * k + 1] * gb[1] +
                      R[3 * k + 2] * gb[2];
    }
    return outside + inside;
}

/* Coupling weight B(d) in [0,1] (Sec. 3.2): 1 deep inside, 0 outside, a
   smooth cos^2 ramp over a band of width eps centred on the surface. */
double orc_weight(double d, double eps)
{
    if (d <= -0.5 * eps) return 1.0;
    if (d >= 0.5 * eps) return 0.0;
    double c = cos(M_PI * (d + 0.5 * eps) / (2.0 * eps));
    return c * c;
}

static double minimg(double v, double L, int periodic)
{
    if (!periodic) return v;
    if (v >= 0.5 * L) return v - L;
    if (v < -0.5 * L) return v + L;
    return v;
}

/* integer image shift k (in units of L) applied by minimg to v */
static int image_shift(double v, double L, int periodic)
{
    if (!periodic) return 0;
    if (v >= 0.5 * L) return -1;
    if (v < -0.5 * L) return 1;
    return 0;
}

static void cross(const double a[3], const double b[3], double out[3])
{
    out[0] = a[1] * b[2] - a[2] * b[1];
    out[1] = a[2] * b[0] - a[0] * b[2];
    out[2] = a[0] * b[1] - a[1] * b[0];
}

static double volume_of(const orc_particle *p)
{
    double a = p->size;
    if (p->shape >= ORC_POLY0) return g_poly[p->shape - ORC_POLY0].vol * a * a * a;
    if (p->shape == 0) return 4.0 / 3.0 * M_PI * a * a * a;
    if (p->shape == 2) return 4.0 / 3.0 * a * a * a;   /* two pyramids */
    return a * a * a;
}

/* inverse body-frame inertia tensor of a homogeneous polyhedron of density
   rho and scale s: I_b = rho s^5 (tr(J) 1 - J) with J the unit-scale second
   moment about the centroid; the inverse by cofactors */
static void poly_inv_inertia(const orc_particle *p, double Ii[9])
{
    const orc_poly *P = &g_poly[p->shape - ORC_POLY0];
    double s2 = p->size * p->size, f = p->dens * s2 * s2 * p->size;
    double tr = P->J[0] + P->J[4] + P->J[8], I[9];
    for (int k = 0; k < 9; ++k) I[k] = f * ((k % 4 == 0 ? tr : 0.0) - P->J[k]);
    double c0 = I[4] * I[8] - I[5] * I[7], c1 = I[5] * I[6] - I[3] * I[8],
           c2 = I[3] * I[7] - I[4] * I[6];
    double det = I[0] * c0 + I[1] * c1 + I[2] * c2;
    Ii[0] = c0 / det;
    Ii[1] = (I[2] * I[7] - I[1] * I[8]) / det;
    Ii[2] = (I[1] * I[5] - I[2] * I[4]) / det;
    Ii[3] = c1 / det;
    Ii[4] = (I[0] * I[8] - I[2] * I[6]) / det;
    Ii[5] = (I[2] * I[3] - I[0] * I[5]) / det;
    Ii[6] = c2 / det;
    Ii[7] = (I[1] * I[6] - I[0] * I[7]) / det;
    Ii[8] = (I[0] * I[4] - I[1] * I[3]) / det;
}

/* angular acceleration of eq. (3) for a polyhedron particle under torque T
   (world frame): R I_b^-1 R^T T (exposed for tests) */
void orc_poly_angular_accel(int shape, double size, double dens,
                            const double q[4], const double T[3], double dw[3])
{
    orc_particle p;
    memset(&p, 0, sizeof p);
    p.shape = shape;
    p.size = size;
    p.dens = dens;
    double R[9], Ii[9], tb[3], wb[3];
    orc_rotation(q, R);
    poly_inv_inertia(&p, Ii);
    for (int k = 0; k < 3; ++k)
        tb[k] = (R[0 + k] * T[0] + R[3 + k] * T[1]) + R[6 + k] * T[2];
    for (int k = 0; k < 3; ++k)
        wb[k] = (Ii[3 * k] * tb[0] + Ii[3 * k + 1] * tb[1]) + Ii[3 * k + 2] * tb[2];
    for (int k = 0; k < 3; ++k)
        dw[k] = (R[3 * k] * wb[0] + R[3 * k + 1] * wb[1]) + R[3 * k + 2] * wb[2];
}

/* isotropic moment of inertia of a homogeneous sphere, cube or regular
   octahedron (<x^2> = a^2 / 10 over |x|+|y|+|z| <= a, so I = m a^2 / 5) */
static double inertia_of(const orc_particle *p, double m)
{
    if (p->shape == 0) return 0.4 * m * p->size * p->size;
    if (p->shape == 2) return 0.2 * m * p->size * p->size;
    return m * p->size * p->size / 6.0;
}

/* ======================================================================
 * Contact model pieces (Sec. 2.3, eqs. (4)-(9)).
 * ====================================================================== */
double orc_effective_modulus(double Ea, double nua, double Eb, double nub)
{
    return 1.0 / ((1.0 - nua * nua) / Ea + (1.0 - nub * nub) / Eb); /* (5) */
}

double orc_damping(double e, double u0) /* eq. (6) */
{
    if (u0 > 0.0) return 1.5 * (1.0 - e) * (11.0 - e) / ((1.0 + 9.0 * e) * u0);
    return 0.0;
}

double orc_friction_mu(double a, double mu_s, double mu_k) /* (7)-(9) */
{
    double r = mu_k / mu_s;
    double mus_star = mu_s * (1.0 - 0.09 * (r * r * r * r));
    double a2 = a * a;
    return (2.0 * mus_star - mu_k) * a2 / (a2 * a2 + 1.0) + mu_k -
           mu_k / (a2 + 1.0);
}

/* ======================================================================
 * Simulation state
 * ====================================================================== */
struct orc_sim {
    orc_params P;
    long n;                   /* number of nodes */
    double *fs;               /* post-collision populations (state) */
    double *f;                /* post-stream populations of the current step */
    int np;
    orc_particle *p;
    double *Fh, *Th, *Fc, *Tc;
    double a_ext[3];
    /* zero-net-flux balance (balance mode 2): lattice mass, lattice
       momentum after the last collision, controller part of a_ext */
    double bal_M, bal_P[3], bal_b[3];
    /* coupling fields at the current particle state */
    int *owner;
    double *dist, *B, *up;
    /* detection set per node */
    unsigned char *kn;
    int *kl;
    /* contact list, sorted by (a, b) */
    orc_contact *con;
    int ncon, capcon;
    /* diagnostics of the last collision, for the momentum-exchange check */
    double *rho_c, *J_c, *du_c;
    double *Scell;            /* S(x) of the last momentum exchange */
    long step;
    long long det_pairs, det_cells;
    char err[256];
};

static void set_err(orc_sim *S, const char *msg)
{
    snprintf(S->err, sizeof S->err, "%s", msg);
}

const char *orc_error(const orc_sim *S) { return S->err; }
long orc_step_count(const orc_sim *S) { return S->step; }

int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static long idx_of(const orc_sim *S, int x, int y, int z)
{
    return (long)x + (long)S->P.nx * ((long)y + (long)S->P.ny * (long)z);
}

static int wrapi(int v, int n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

orc_sim *orc_create(const orc_params *P, int np, const int *shape,
                    const double *size, const double *dens, const double *X,
                    const double *q, const double *U, const double *w)
{
    for (int i = 0; i < np; ++i)
        if (shape[i] < 0 || (shape[i] >= ORC_POLY0 &&
                             (shape[i] >= ORC_POLY0 + ORC_MAXPOLY || !g_poly_ok[shape[i] - ORC_POLY0])))
            return NULL;
    orc_sim *S = (orc_sim *)calloc(1, sizeof(orc_sim));
    if (!S) return NULL;
    S->P = *P;
    S->n = (long)P->nx * P->ny * P->nz;
    long n = S->n;
    S->fs = (double *)malloc(sizeof(double) * ORC_Q * n);
    S->f = (double *)malloc(sizeof(double) * ORC_Q * n);
    S->owner = (int *)malloc(sizeof(int) * n);
    S->dist = (double *)malloc(sizeof(double) * n);
    S->B = (double *)malloc(sizeof(double) * n);
    S->up = (double *)malloc(sizeof(double) * 3 * n);
    S->kn = (unsigned char *)malloc(n);
    S->kl = (int *)malloc(sizeof(int) * ORC_MAXK * n);
    S->rho_c = (double *)malloc(sizeof(double) * n);
    S->J_c = (double *)malloc(sizeof(double) * 3 * n);
    S->du_c = (double *)malloc(sizeof(double) * 3 * n);
    S->Scell = (double *)malloc(sizeof(double) * 3 * n);
    S->np = np;
    S->p = (orc_particle *)calloc(np > 0 ? np : 1, sizeof(orc_particle));
    S->Fh = (double *)calloc(3 * (np > 0 ? np : 1), sizeof(double));
    S->Th = (double *)calloc(3 * (np > 0 ? np : 1), sizeof(double));
    S->Fc = (double *)calloc(3 * (np > 0 ? np : 1), sizeof(double));
    S->Tc = (double *)calloc(3 * (np > 0 ? np : 1), sizeof(double));
    S->capcon = 64;
    S->con = (orc_contact *)calloc(S->capcon, sizeof(orc_contact));
    if (!S->fs || !S->f || !S->owner || !S->dist || !S->B || !S->up ||
        !S->kn || !S->kl || !S->rho_c || !S->J_c || !S->du_c || !S->Scell ||
        !S->p || !S->con) {
        orc_destroy(S);
        return NULL;
    }
    memset(S->rho_c, 0, sizeof(double) * n);
    memset(S->J_c, 0, sizeof(double) * 3 * n);
    memset(S->du_c, 0, sizeof(double) * 3 * n);
    memset(S->Scell, 0, sizeof(double) * 3 * n);
    for (int i = 0; i < np; ++i) {
        orc_particle *pp = &S->p[i];
        pp->shape = shape[i];
        pp->size = size[i];
        pp->dens = dens[i];
        for (int k = 0; k < 3; ++k) {
            pp->X[k] = X[3 * i + k];
            pp->U[k] = U[3 * i + k];
            pp->w[k] = w[3 * i + k];
        }
        for (int k = 0; k < 4; ++k) pp->q[k] = q[4 * i + k];
    }
    /* Balance force (Sec. 5.1): a uniform fluid acceleration that cancels
       the particles' net gravity-minus-buoyancy, so that the net external
       force, and hence the net volume flow, stays zero on a fully periodic
       box.  Applied only when requested and the box is fully periodic. */
    for (int k = 0; k < 3; ++k) S->a_ext[k] = P->fluid_accel[k];
    if (P->balance == 1 && P->periodic_z) {
        double tot[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < np; ++i) {
            double V = volume_of(&S->p[i]);
            for (int k = 0; k < 3; ++k)
                tot[k] += (S->p[i].dens - 1.0) * V * P->gravity[k];
        }
        for (int k = 0; k < 3; ++k) S->a_ext[k] -= tot[k] / (double)n;
    }
    return S;
}

void orc_destroy(orc_sim *S)
{
    if (!S) return;
    free(S->fs); free(S->f); free(S->owner); free(S->dist); free(S->B);
    free(S->up); free(S->kn); free(S->kl); free(S->rho_c); free(S->J_c);
    free(S->du_c); free(S->Scell); free(S->p); free(S->Fh); free(S->Th);
    free(S->Fc); free(S->Tc); free(S->con);
    free(S);
}

/* ======================================================================
 * Step phase: streaming, eq. (11), pull form f_i(x) = f_i*(x - c_i).
 * Walls (non-periodic z): half-way bounce-back, the textbook rule
 * f_i(x) = f_opp(i)*(x) + 2 w_i rho_w (c_i . u_w) / c_s^2 with rho_w = 1.
 * ====================================================================== */
static void stream(orc_sim *S)
{
    const orc_params *P = &S->P;
    long n = S->n;
    int opp[ORC_Q];
    for (int i = 0; i < ORC_Q; ++i) opp[i] = opposite(i);
#pragma omp parallel for schedule(static)
    for (int z = 0; z < P->nz; ++z)
        for (int y = 0; y < P->ny; ++y)
            for (int x = 0; x < P->nx; ++x) {
                long id = idx_of(S, x, y, z);
                for (int i = 0; i < ORC_Q; ++i) {
                    int sx = wrapi(x - CV[i][0], P->nx);
                    int sy = wrapi(y - CV[i][1], P->ny);
                    int sz = z - CV[i][2];
                    if (P->periodic_z) {
                        sz = wrapi(sz, P->nz);
                    } else if (sz < 0 || sz >= P->nz) {
                        const double *uw = P->wall_u[sz < 0 ? 0 : 1];
                        double cu = CV[i][0] * uw[0] + CV[i][1] * uw[1] +
                                    CV[i][2] * uw[2];
                        S->f[i * n + id] =
                            S->fs[opp[i] * n + id] + 2.0 * WT[i] * cu / CS2;
                        continue;
                    }
                    S->f[i * n + id] = S->fs[i * n + idx_of(S, sx, sy, sz)];
                }
            }
}

/* ======================================================================
 * Step phase: momentum exchange, eqs. (16)-(18).
 * S(x) = sum_i (c_i - u_p(x)) f_i(x + c_i) + (c_i + u_p(x)) f_opp(i)(x),
 * read with post-streaming populations at the start of the step:
 * f_i(x + c_i) is the population that left x along c_i, i.e. f_i*(x) of the
 * previous collision, and f_opp(i)(x) is the population now at x.  With
 * this reading S(x) is the momentum the node hands to the fluid, so the
 * force on the particle is its negative: F_p = -sum S, T_p = -sum r x S
 * over the nodes x_b the particle owns.
 * ====================================================================== */
static void momentum_exchange(orc_sim *S)
{
    long n = S->n;
    int opp[ORC_Q];
    for (int i = 0; i < ORC_Q; ++i) opp[i] = opposite(i);
    memset(S->Fh, 0, sizeof(double) * 3 * (S->np > 0 ? S->np : 1));
    memset(S->Th, 0, sizeof(double) * 3 * (S->np > 0 ? S->np : 1));
#pragma omp parallel for schedule(static)
    for (long id = 0; id < n; ++id) {
        double s[3] = {0.0, 0.0, 0.0};
        if (S->owner[id] >= 0) {
            const double *u = &S->up[3 * id];
            for (int i = 0; i < ORC_Q; ++i) {
                double fo = S->fs[i * n + id];        /* f_i(x + c_i) */
                double fi = S->f[opp[i] * n + id];    /* f_opp(i)(x)  */
                for (int k = 0; k < 3; ++k)
                    s[k] += (CV[i][k] - u[k]) * fo + (CV[i][k] + u[k]) * fi;
            }
        }
        for (int k = 0; k < 3; ++k) S->Scell[3 * id + k] = s[k];
    }
    /* per-particle sums in node order (serial, deterministic) */
    const orc_params *P = &S->P;
    for (int z = 0; z < P->nz; ++z)
        for (int y = 0; y < P->ny; ++y)
            for (int x = 0; x < P->nx; ++x) {
                long id = idx_of(S, x, y, z);
                int o = S->owner[id];
                if (o < 0) continue;
                const orc_particle *pp = &S->p[o];
                double r[3], t[3];
                r[0] = minimg((double)x - pp->X[0], P->nx, 1);
                r[1] = minimg((double)y - pp->X[1], P->ny, 1);
                r[2] = minimg((double)z - pp->X[2], P->nz, P->periodic_z);
                cross(r, &S->Scell[3 * id], t);
                for (int k = 0; k < 3; ++k) {
                    S->Fh[3 * o + k] -= S->Scell[3 * id + k];
                    S->Th[3 * o + k] -= t[k];
                }
            }
}

/* ======================================================================
 * Step phase: particles to fluid coupling and rough contact detection
 * (Sec. 3.2, Sec. 3.3.1-3.3.2), at the current particle state.
 *
 * Owner: among particles with d < eps/2 at node x, the smallest (d, id)
 * pair.  B(x) = B(d_owner), u_p(x) = U + w x r.  Nodes owned by nobody have
 * B = 0.  The detection set K(x) holds every particle whose enlarged signed
 * distance d - delta_c is below half the cell diagonal sqrt(0.75) (Sec.
 * 3.3.1); a wall joins when its own distance is below that bound.
 *
 * Each particle visits the nodes of its axis-aligned bounding box widened
 * by the largest reach of either test plus one node; nodes outside that box
 * satisfy neither test.  Periodic axes visit every wrapped node once.
 * ====================================================================== */
static int axis_nodes(double c, double reach, int n, int periodic, int *out)
{
    int lo = (int)floor(c - reach), hi = (int)ceil(c + reach);
    int cnt = 0;
    if (periodic) {
        if (hi - lo + 1 >= n) {
            for (int v = 0; v < n; ++v) out[cnt++] = v;
        } else {
            for (int v = lo; v <= hi; ++v) out[cnt++] = wrapi(v, n);
        }
    } else {
        if (lo < 0) lo = 0;
        if (hi > n - 1) hi = n - 1;
        for (int v = lo; v <= hi; ++v) out[cnt++] = v;
    }
    return cnt;
}

static const double DETECT = 0.8660254037844386; /* sqrt(0.75) */

/* half extent along world axis k of a particle with rotation R: exact for
   cubes, polyhedra (largest |world coordinate| of a vertex) and ellipsoids,
   the circumradius for spheres and octahedra */
static double half_extent(const orc_particle *pp, const double R[9], int k)
{
    double e = pp->size;
    if (pp->shape == 1)
        e = 0.5 * pp->size *
            (fabs(R[3 * k]) + fabs(R[3 * k + 1]) + fabs(R[3 * k + 2]));
    if (pp->shape >= ORC_POLY0 && g_poly[pp->shape - ORC_POLY0].kind == 1) {
        /* ellipsoid: max over the surface of a world coordinate,
           |(R_k0 e0, R_k1 e1, R_k2 e2)| */
        const double *ax = g_poly[pp->shape - ORC_POLY0].ax;
        double a0 = R[3 * k] * ax[0], a1 = R[3 * k + 1] * ax[1], a2 = R[3 * k + 2] * ax[2];
        e = pp->size * sqrt((a0 * a0 + a1 * a1) + a2 * a2);
    } else if (pp->shape >= ORC_POLY0) {
        const orc_poly *Q = &g_poly[pp->shape - ORC_POLY0];
        e = 0.0;
        for (int i = 0; i < Q->nv; ++i) {
            double c = fabs((R[3 * k] * Q->v[i][0] + R[3 * k + 1] * Q->v[i][1]) +
                            R[3 * k + 2] * Q->v[i][2]);
            if (c > e) e = c;
        }
        e *= pp->size;
    }
    return e;
}

double orc_half_extent(int shape, double size, const double q[4], int k)
{
    orc_particle p;
    memset(&p, 0, sizeof p);
    p.shape = shape;
    p.size = size;
    double R[9];
    orc_rotation(q, R);
    return half_extent(&p, R, k);
}

static int couple_and_detect_nodes(orc_sim *S)
{
    const orc_params *P = &S->P;
    long n = S->n;
    for (long id = 0; id < n; ++id) {
        S->owner[id] = -1;
        S->dist[id] = DBL_MAX;
        S->kn[id] = 0;
    }
    double margin = fmax(0.5 * P->eps, DETECT + P->delta_c) + 1.0;
    int dims[3] = {P->nx, P->ny, P->nz};
    int per[3] = {1, 1, P->periodic_z};
    int maxd = P->nx;
    if (P->ny > maxd) maxd = P->ny;
    if (P->nz > maxd) maxd = P->nz;
    int *ax[3];
    for (int k = 0; k < 3; ++k) ax[k] = (int *)malloc(sizeof(int) * (maxd + 8));
    int overflow = 0;
    for (int ip = 0; ip < S->np; ++ip) {
        const orc_particle *pp = &S->p[ip];
        double R[9], reach[3];
        orc_rotation(pp->q, R);
        for (int k = 0; k < 3; ++k) reach[k] = half_extent(pp, R, k) + margin;
        int cnt[3];
        for (int k = 0; k < 3; ++k)
            cnt[k] = axis_nodes(pp->X[k], reach[k], dims[k], per[k], ax[k]);
        for (int a = 0; a < cnt[2]; ++a)
            for (int b = 0; b < cnt[1]; ++b)
                for (int c = 0; c < cnt[0]; ++c) {
                    int x = ax[0][c], y = ax[1][b], z = ax[2][a];
                    long id = idx_of(S, x, y, z);
                    double r[3];
                    r[0] = minimg((double)x - pp->X[0], P->nx, 1);
                    r[1] = minimg((double)y - pp->X[1], P->ny, 1);
                    r[2] = minimg((double)z - pp->X[2], P->nz, P->periodic_z);
                    double d = orc_sdf(pp->shape, pp->size, R, r, NULL);
                    if (d < 0.5 * P->eps && d < S->dist[id]) {
                        S->dist[id] = d;   /* strict <: ties keep lower id */
                        S->owner[id] = ip;
                    }
                    if (d - P->delta_c < DETECT) {
                        if (S->kn[id] >= ORC_MAXK) {
                            overflow = 1;
                        } else {
                            S->kl[ORC_MAXK * id + S->kn[id]] = ip;
                            S->kn[id]++;
                        }
                    }
                }
    }
    for (int k = 0; k < 3; ++k) free(ax[k]);
    /* B and u_p from the owner */
    for (int z = 0; z < P->nz; ++z)
        for (int y = 0; y < P->ny; ++y)
            for (int x = 0; x < P->nx; ++x) {
                long id = idx_of(S, x, y, z);
                int o = S->owner[id];
                if (o < 0) {
                    S->B[id] = 0.0;
                    S->up[3 * id] = S->up[3 * id + 1] = S->up[3 * id + 2] = 0.0;
                    continue;
                }
                const orc_particle *pp = &S->p[o];
                double r[3], wr[3];
                r[0] = minimg((double)x - pp->X[0], P->nx, 1);
                r[1] = minimg((double)y - pp->X[1], P->ny, 1);
                r[2] = minimg((double)z - pp->X[2], P->nz, P->periodic_z);
                cross(pp->w, r, wr);
                S->B[id] = orc_weight(S->dist[id], P->eps);
                for (int k = 0; k < 3; ++k) S->up[3 * id + k] = pp->U[k] + wr[k];
            }
    return overflow ? -1 : 0;
}

/* detected pairs, kept per lower id in a small growable list */
typedef struct {
    int b, count, lo[3], hi[3];
} det_entry;
typedef struct {
    det_entry *e;
    int n, cap;
} det_list;

static det_entry *det_get(det_list *L, int b)
{
    for (int i = 0; i < L->n; ++i)
        if (L->e[i].b == b) return &L->e[i];
    if (L->n == L->cap) {
        L->cap = L->cap ? 2 * L->cap : 4;
        L->e = (det_entry *)realloc(L->e, sizeof(det_entry) * L->cap);
    }
    det_entry *d = &L->e[L->n++];
    d->b = b;
    d->count = 0;
    for (int k = 0; k < 3; ++k) {
        d->lo[k] = 2147483647;
        d->hi[k] = -2147483647 - 1;
    }
    return d;
}

static void det_add(det_list *L, int b, const int img[3])
{
    det_entry *d = det_get(L, b);
    d->count++;
    for (int k = 0; k < 3; ++k) {
        if (img[k] < d->lo[k]) d->lo[k] = img[k];
        if (img[k] > d->hi[k]) d->hi[k] = img[k];
    }
}

/* node image in the frame of the lower-id particle (Sec. 3.3.2): the node
   coordinate shifted by whole periods so that it lies at X_a + minimg(x - X_a) */
static void node_image(const orc_sim *S, const orc_particle *pa, int x, int y,
                       int z, int img[3])
{
    const orc_params *P = &S->P;
    img[0] = x + P->nx * image_shift((double)x - pa->X[0], P->nx, 1);
    img[1] = y + P->ny * image_shift((double)y - pa->X[1], P->ny, 1);
    img[2] = z + P->nz * image_shift((double)z - pa->X[2], P->nz, P->periodic_z);
}

static int cmp_int(const void *a, const void *b)
{
    int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}

static void contacts_reserve(orc_sim *S, int need)
{
    if (need <= S->capcon) return;
    while (S->capcon < need) S->capcon *= 2;
    S->con = (orc_contact *)realloc(S->con, sizeof(orc_contact) * S->capcon);
}

/* Rough detection over all nodes, then the new contact list: contacts kept
   from the treatment keep their carried box (already established contacts
   skip the rough detection, Sec. 4.3.2); pairs not in the list start with
   the rough box [min - 1/2, max + 1/2] of their flagged node images. */
static int detect_and_merge(orc_sim *S, int nkeep)
{
    const orc_params *P = &S->P;
    det_list *D = (det_list *)calloc(S->np > 0 ? S->np : 1, sizeof(det_list));
    long long cells = 0;
    for (int z = 0; z < P->nz; ++z)
        for (int y = 0; y < P->ny; ++y)
            for (int x = 0; x < P->nx; ++x) {
                long id = idx_of(S, x, y, z);
                int k = S->kn[id];
                if (k == 0) continue;
                const int *K = &S->kl[ORC_MAXK * id];
                int img[3];
                for (int i = 0; i < k; ++i)
                    for (int j = i + 1; j < k; ++j) {
                        int a = K[i] < K[j] ? K[i] : K[j];
                        int b = K[i] < K[j] ? K[j] : K[i];
                        node_image(S, &S->p[a], x, y, z, img);
                        det_add(&D[a], b, img);
                        cells++;
                    }
                if (!P->periodic_z) {
                    double dbot = (double)z + 0.5;
                    double dtop = ((double)P->nz - 0.5) - (double)z;
                    for (int i = 0; i < k; ++i) {
                        node_image(S, &S->p[K[i]], x, y, z, img);
                        if (dbot < DETECT) { det_add(&D[K[i]], -1, img); cells++; }
                        if (dtop < DETECT) { det_add(&D[K[i]], -2, img); cells++; }
                    }
                }
            }
    /* merge kept contacts (sorted, at S->con[0..nkeep)) with detections */
    int ndet = 0;
    for (int a = 0; a < S->np; ++a) ndet += D[a].n;
    orc_contact *out = (orc_contact *)calloc(nkeep + ndet + 1, sizeof(orc_contact));
    int no = 0, ik = 0;
    long long pairs = 0;
    for (int a = 0; a < S->np; ++a) {
        /* sorted partner ids of a's detections */
        int nb = D[a].n;
        int *bs = (int *)malloc(sizeof(int) * (nb + 1));
        for (int i = 0; i < nb; ++i) bs[i] = D[a].e[i].b;
        qsort(bs, nb, sizeof(int), cmp_int);
        int jb = 0;
        for (;;) {
            int have_k = ik < nkeep && S->con[ik].a == a;
            int have_d = jb < nb;
            if (!have_k && !have_d) break;
            int bk = have_k ? S->con[ik].b : 2147483647;
            int bd = have_d ? bs[jb] : 2147483647;
            orc_contact c;
            if (have_k && bk <= bd) {
                c = S->con[ik++];
                c.count = 0;
                for (int m = 0; m < 3; ++m) c.rlo[m] = c.rhi[m] = 0;
                if (bk == bd) {
                    det_entry *d = det_get(&D[a], bd);
                    c.count = d->count;
                    for (int m = 0; m < 3; ++m) { c.rlo[m] = d->lo[m]; c.rhi[m] = d->hi[m]; }
                    jb++;
                }
            } else {
                det_entry *d = det_get(&D[a], bd);
                memset(&c, 0, sizeof c);
                c.a = a;
                c.b = bd;
                c.count = d->count;
                for (int m = 0; m < 3; ++m) {
                    c.rlo[m] = d->lo[m];
                    c.rhi[m] = d->hi[m];
                    c.lo[m] = (double)d->lo[m] - 0.5;
                    c.hi[m] = (double)d->hi[m] + 0.5;
                }
                jb++;
            }
            if (c.count > 0) pairs++;
            out[no++] = c;
        }
        free(bs);
        free(D[a].e);
    }
    /* kept contacts whose lower id had no detections at all */
    while (ik < nkeep) {
        /* cannot happen: the loop above visits every a; kept for safety */
        out[no] = S->con[ik++];
        out[no].count = 0;
        no++;
    }
    free(D);
    contacts_reserve(S, no + 1);
    memcpy(S->con, out, sizeof(orc_contact) * no);
    S->ncon = no;
    free(out);
    S->det_pairs = pairs;
    S->det_cells = cells;
    return 0;
}

/* ======================================================================
 * Contact treatment of one pair (Sec. 3.3.1, eqs. (4)-(9)).
 * ====================================================================== */
typedef struct {
    int shape;
    double size, X[3], R[9];
} body;

static double body_sdf(const body *b, const double y[3], double grad[3])
{
    double r[3] = {y[0] - b->X[0], y[1] - b->X[1], y[2] - b->X[2]};
    return orc_sdf(b->shape, b->size, b->R, r, grad);
}

/* enlarged signed distance of member a or b (b may be a wall) */
static double member_sdf(const orc_params *P, const body *pb, int b_id,
                         const double y[3], double grad[3])
{
    if (b_id >= 0) return body_sdf(pb, y, grad) - P->delta_c;
    if (b_id == -1) { /* bottom wall, distance z + 1/2 (not enlarged) */
        if (grad) { grad[0] = 0.0; grad[1] = 0.0; grad[2] = 1.0; }
        return y[2] + 0.5;
    }
    if (grad) { grad[0] = 0.0; grad[1] = 0.0; grad[2] = -1.0; }
    return ((double)P->nz - 0.5) - y[2];
}

/* Box correction, one pass (Sec. 3.3.1, "correction"): the six faces in the
   order -x,+x,-y,+y,-z,+z; on each face N_c x N_c midpoint samples of
   phi = max(d'_a, d'_b); the face moves inwards by min phi (outwards if the
   minimum is negative).  Returns 0 if the box became empty. */
static int correct_box(const orc_params *P, const body *A, const body *Bb,
                       int b_id, double lo[3], double hi[3])
{
    int nc = P->n_c;
    for (int face = 0; face < 6; ++face) {
        for (int k = 0; k < 3; ++k)
            if (!(hi[k] > lo[k])) return 0;
        int k = face / 2, plus = face % 2;
        int u = k == 0 ? 1 : 0;
        int v = k == 2 ? 1 : 2;
        double hu = (hi[u] - lo[u]) / (double)nc;
        double hv = (hi[v] - lo[v]) / (double)nc;
        double smin = DBL_MAX;
        for (int j = 0; j < nc; ++j)
            for (int l = 0; l < nc; ++l) {
                double y[3];
                y[k] = plus ? hi[k] : lo[k];
                y[u] = lo[u] + ((double)j + 0.5) * hu;
                y[v] = lo[v] + ((double)l + 0.5) * hv;
                double da = body_sdf(A, y, NULL) - P->delta_c;
                double db = member_sdf(P, Bb, b_id, y, NULL);
                double phi = fmax(da, db);
                if (phi < smin) smin = phi;
            }
        if (plus) hi[k] = hi[k] - smin;
        else lo[k] = lo[k] + smin;
    }
    for (int k = 0; k < 3; ++k)
        if (!(hi[k] > lo[k])) return 0;
    return 1;
}

/* Overlap integration (Sec. 3.3.1, final step): N_c^3 midpoint samples of
   the box; a sample is inside when both enlarged distances are negative.
   V = n_in * cell volume, centroid = mean inside sample, normal = the
   normalised sum of (grad d'_a - grad d'_b) over inside samples (pointing
   from a to b), depth = max over inside samples of -(d'_a + d'_b). */
static void integrate_box(const orc_params *P, const body *A, const body *Bb,
                          int b_id, const double lo[3], const double hi[3],
                          orc_contact *c)
{
    int nc = P->n_c;
    double h[3];
    for (int k = 0; k < 3; ++k) h[k] = (hi[k] - lo[k]) / (double)nc;
    int n_in = 0;
    double sy[3] = {0.0, 0.0, 0.0}, g[3] = {0.0, 0.0, 0.0};
    double dmax = 0.0;
    for (int l = 0; l < nc; ++l)
        for (int k = 0; k < nc; ++k)
            for (int j = 0; j < nc; ++j) {
                double y[3], ga[3], gb[3];
                y[0] = lo[0] + ((double)j + 0.5) * h[0];
                y[1] = lo[1] + ((double)k + 0.5) * h[1];
                y[2] = lo[2] + ((double)l + 0.5) * h[2];
                double da = body_sdf(A, y, ga) - P->delta_c;
                double db = member_sdf(P, Bb, b_id, y, gb);
                if (fmax(da, db) < 0.0) {
                    double dep = -(da + db);
                    if (n_in == 0 || dep > dmax) dmax = dep;
                    n_in++;
                    for (int m = 0; m < 3; ++m) {
                        sy[m] += y[m];
                        g[m] += ga[m] - gb[m];
                    }
                }
            }
    c->n_in = n_in;
    c->volume = (double)n_in * (h[0] * h[1] * h[2]);
    c->depth = n_in > 0 ? dmax : 0.0;
    for (int m = 0; m < 3; ++m) {
        c->centroid[m] = n_in > 0 ? sy[m] / (double)n_in : 0.0;
        c->normal[m] = 0.0;
    }
    double gn = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
    if (n_in > 0 && gn > 0.0) {
        for (int m = 0; m < 3; ++m) c->normal[m] = g[m] / gn;
    } else if (n_in > 0) {
        /* degenerate gradient sum: centre line (particles) or wall normal */
        double dvec[3];
        if (b_id >= 0) {
            for (int m = 0; m < 3; ++m) dvec[m] = Bb->X[m] - A->X[m];
        } else {
            dvec[0] = 0.0; dvec[1] = 0.0; dvec[2] = b_id == -1 ? -1.0 : 1.0;
        }
        double dn = sqrt(dvec[0] * dvec[0] + dvec[1] * dvec[1] + dvec[2] * dvec[2]);
        if (dn > 0.0)
            for (int m = 0; m < 3; ++m) c->normal[m] = dvec[m] / dn;
    }
}

/* Contact forces, eqs. (4)-(9), for a contact with V > 0.  The relative
   velocity is taken at the contact point; its normal component is the
   approach rate (positive when closing).  The damping factor c of eq. (6)
   is fixed at the first treatment with V > 0, with u_0 the normal approach
   rate at that moment, and kept for the contact's lifetime (Sec. 4.3.4).
   The normal force magnitude is clamped at zero (no adhesion). */
static void contact_force(const orc_params *P, const orc_particle *pa,
                          const orc_particle *pb, const double Xb[3],
                          orc_contact *c)
{
    double ra[3], va[3], vb[3] = {0.0, 0.0, 0.0}, t[3];
    for (int m = 0; m < 3; ++m) ra[m] = c->centroid[m] - pa->X[m];
    cross(pa->w, ra, t);
    for (int m = 0; m < 3; ++m) va[m] = pa->U[m] + t[m];
    if (pb) {
        double rb[3];
        for (int m = 0; m < 3; ++m) rb[m] = c->centroid[m] - Xb[m];
        cross(pb->w, rb, t);
        for (int m = 0; m < 3; ++m) vb[m] = pb->U[m] + t[m];
    }
    double v[3];
    for (int m = 0; m < 3; ++m) v[m] = va[m] - vb[m];
    const double *nrm = c->normal;
    double dn = v[0] * nrm[0] + v[1] * nrm[1] + v[2] * nrm[2];
    if (!c->established) {
        c->damping = orc_damping(P->restitution, dn);
        c->established = 1;
    }
    double estar = orc_effective_modulus(P->young, P->poisson, P->young,
                                         P->poisson);
    double fn = 4.0 / (3.0 * M_PI) * estar * sqrt(c->volume * c->depth) *
                (1.0 + c->damping * dn);
    if (fn < 0.0) fn = 0.0;
    double vt[3];
    for (int m = 0; m < 3; ++m) vt[m] = v[m] - dn * nrm[m];
    double vtn = sqrt(vt[0] * vt[0] + vt[1] * vt[1] + vt[2] * vt[2]);
    double ft[3] = {0.0, 0.0, 0.0};
    if (vtn > 0.0) {
        double mu = orc_friction_mu(vtn / P->u_k, P->mu_s, P->mu_k);
        for (int m = 0; m < 3; ++m) ft[m] = -(vt[m] / vtn) * mu * fn;
    }
    c->fn = fn;
    for (int m = 0; m < 3; ++m) {
        c->force_a[m] = -fn * nrm[m] + ft[m];
        c->force_b[m] = -c->force_a[m];
    }
}

static void make_body(const orc_particle *p, const double X[3], body *b)
{
    b->shape = p->shape;
    b->size = p->size;
    for (int k = 0; k < 3; ++k) b->X[k] = X[k];
    orc_rotation(p->q, b->R);
}

void orc_treat_pair(const orc_params *P, const orc_particle *pa,
                    const orc_particle *pb, int b_id, int npass,
                    double lo[3], double hi[3], orc_contact *out)
{
    body A, Bb;
    make_body(pa, pa->X, &A);
    if (b_id >= 0) make_body(pb, pb->X, &Bb);
    int ok = 1;
    for (int it = 0; it < npass && ok; ++it)
        ok = correct_box(P, &A, &Bb, b_id, lo, hi);
    memset(out, 0, sizeof *out);
    out->a = 0;
    out->b = b_id;
    for (int k = 0; k < 3; ++k) { out->lo[k] = lo[k]; out->hi[k] = hi[k]; }
    if (!ok) return;
    integrate_box(P, &A, &Bb, b_id, lo, hi, out);
    if (out->n_in > 0)
        contact_force(P, pa, b_id >= 0 ? pb : NULL, b_id >= 0 ? pb->X : NULL,
                      out);
}

void orc_contact_force_of(const orc_params *P, const orc_particle *pa,
                          const orc_particle *pb, orc_contact *c)
{
    contact_force(P, pa, pb, pb ? pb->X : NULL, c);
}

/* Treatment of the whole contact list at the current particle state; adds
   the contact forces and torques, keeps contacts with V > 0 (sorted order is
   preserved) and returns how many were kept. */
static int treat_contacts(orc_sim *S)
{
    const orc_params *P = &S->P;
    memset(S->Fc, 0, sizeof(double) * 3 * (S->np > 0 ? S->np : 1));
    memset(S->Tc, 0, sizeof(double) * 3 * (S->np > 0 ? S->np : 1));
    int dims[3] = {P->nx, P->ny, P->nz};
    int per[3] = {1, 1, P->periodic_z};
    int nkeep = 0;
    for (int ic = 0; ic < S->ncon; ++ic) {
        orc_contact c = S->con[ic];
        const orc_particle *pa = &S->p[c.a];
        const orc_particle *pb = c.b >= 0 ? &S->p[c.b] : NULL;
        /* the higher-id particle is moved next to the lower-id one
           (Sec. 3.3.2); the stored state is not changed */
        double Xb[3] = {0.0, 0.0, 0.0};
        if (pb)
            for (int k = 0; k < 3; ++k)
                Xb[k] = pa->X[k] + minimg(pb->X[k] - pa->X[k], dims[k], per[k]);
        /* a new particle-wall pair: its flagged nodes all lie on the fluid
           side of the wall plane, while the overlap of the enlarged body
           with the wall's half space lies beyond it; the wall-side face of
           the box starts at the far side of the enlarged body (its half
           extent along z plus the enlargement), and the correction moves it
           onto the body */
        if (!c.carried && c.b < 0) {
            double R[9];
            orc_rotation(pa->q, R);
            double ez = half_extent(pa, R, 2) + P->delta_c;
            if (c.b == -1) c.lo[2] = fmin(c.lo[2], pa->X[2] - ez);
            else c.hi[2] = fmax(c.hi[2], pa->X[2] + ez);
        }
        /* the box stays in the frame of the lower-id particle: if that
           particle has wrapped since the box was made, shift the box along */
        for (int k = 0; k < 3; ++k) {
            double mid = 0.5 * (c.lo[k] + c.hi[k]);
            int sh = image_shift(mid - pa->X[k], dims[k], per[k]);
            c.lo[k] += (double)(sh * dims[k]);
            c.hi[k] += (double)(sh * dims[k]);
        }
        body A, Bb;
        make_body(pa, pa->X, &A);
        if (pb) make_body(pb, Xb, &Bb);
        double lo[3], hi[3];
        for (int k = 0; k < 3; ++k) { lo[k] = c.lo[k]; hi[k] = c.hi[k]; }
        int ok = correct_box(P, &A, &Bb, c.b, lo, hi);
        c.n_in = 0;
        c.volume = 0.0;
        if (ok) integrate_box(P, &A, &Bb, c.b, lo, hi, &c);
        if (!ok || c.n_in == 0) continue; /* contact ends; record deleted */
        contact_force(P, pa, pb, Xb, &c);
        double ta[3], tb[3], r[3];
        for (int k = 0; k < 3; ++k) r[k] = c.centroid[k] - pa->X[k];
        cross(r, c.force_a, ta);
        for (int k = 0; k < 3; ++k) {
            S->Fc[3 * c.a + k] += c.force_a[k];
            S->Tc[3 * c.a + k] += ta[k];
        }
        if (pb) {
            for (int k = 0; k < 3; ++k) r[k] = c.centroid[k] - Xb[k];
            cross(r, c.force_b, tb);
            for (int k = 0; k < 3; ++k) {
                S->Fc[3 * c.b + k] += c.force_b[k];
                S->Tc[3 * c.b + k] += tb[k];
            }
        }
        for (int k = 0; k < 3; ++k) { c.lo[k] = lo[k]; c.hi[k] = hi[k]; }
        c.carried = 1;
        c.age++;
        S->con[nkeep++] = c;
    }
    return nkeep;
}

/* ======================================================================
 * Particle motion, eqs. (2)-(3): symplectic Euler over a sub-step of length
 * dt (1 without sub-steps); gravity minus buoyancy F_g = (rho_p - rho_f) V g
 * (Sec. 5.1) with rho_f = 1; orientation advanced by the exact rotation
 * through |w| dt about w.
 * ====================================================================== */
static void move_particles(orc_sim *S, double dt)
{
    const orc_params *P = &S->P;
    int dims[3] = {P->nx, P->ny, P->nz};
    int per[3] = {1, 1, P->periodic_z};
    for (int ip = 0; ip < S->np; ++ip) {
        orc_particle *pp = &S->p[ip];
        double V = volume_of(pp);
        double m = pp->dens * V;
        double T[3];
        for (int k = 0; k < 3; ++k) {
            double Fg = (pp->dens - 1.0) * V * P->gravity[k];
            double F = S->Fh[3 * ip + k] + S->Fc[3 * ip + k] + Fg;
            T[k] = S->Th[3 * ip + k] + S->Tc[3 * ip + k];
            pp->U[k] += F / m * dt;
            pp->X[k] += pp->U[k] * dt;
            if (per[k]) {
                if (pp->X[k] >= (double)dims[k]) pp->X[k] -= (double)dims[k];
                else if (pp->X[k] < 0.0) pp->X[k] += (double)dims[k];
            }
        }
        if (pp->shape >= ORC_POLY0) {
            /* eq. (3) with the world-frame tensor I_w = R I_b R^T at the
               current orientation: omega += R I_b^-1 R^T T dt */
            double R[9], Ii[9], tb[3], wb[3];
            orc_rotation(pp->q, R);
            poly_inv_inertia(pp, Ii);
            for (int k = 0; k < 3; ++k)
                tb[k] = (R[0 + k] * T[0] + R[3 + k] * T[1]) + R[6 + k] * T[2];
            for (int k = 0; k < 3; ++k)
                wb[k] = (Ii[3 * k] * tb[0] + Ii[3 * k + 1] * tb[1]) + Ii[3 * k + 2] * tb[2];
            for (int k = 0; k < 3; ++k)
                pp->w[k] += ((R[3 * k] * wb[0] + R[3 * k + 1] * wb[1]) + R[3 * k + 2] * wb[2]) * dt;
        } else {
            double I = inertia_of(pp, m);
            for (int k = 0; k < 3; ++k) pp->w[k] += T[k] / I * dt;
        }
        double th = sqrt(pp->w[0] * pp->w[0] + pp->w[1] * pp->w[1] +
                         pp->w[2] * pp->w[2]) * dt;
        if (th > 0.0) {
            double c = cos(0.5 * th), s = sin(0.5 * th) / th * dt;
            double dq[4] = {c, s * pp->w[0], s * pp->w[1], s * pp->w[2]};
            const double *q = pp->q;
            double r[4];
            r[0] = dq[0] * q[0] - (dq[1] * q[1] + dq[2] * q[2] + dq[3] * q[3]);
            r[1] = dq[0] * q[1] + q[0] * dq[1] + (dq[2] * q[3] - dq[3] * q[2]);
            r[2] = dq[0] * q[2] + q[0] * dq[2] + (dq[3] * q[1] - dq[1] * q[3]);
            r[3] = dq[0] * q[3] + q[0] * dq[3] + (dq[1] * q[2] - dq[2] * q[1]);
            double nn = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + r[3] * r[3]);
            for (int k = 0; k < 4; ++k) pp->q[k] = r[k] / nn;
        }
    }
}

/* ======================================================================
 * Collision, eqs. (10), (12), (14), (15): BGK towards f^eq(rho, u) plus the
 * exact-difference source f^eq(rho, u + du) - f^eq(rho, u), with the
 * velocity shift du = B (u_p - u) plus the uniform fluid acceleration.
 * ====================================================================== */
static void collide(orc_sim *S)
{
    const orc_params *P = &S->P;
    long n = S->n;
#pragma omp parallel for schedule(static)
    for (long id = 0; id < n; ++id) {
        double fl[ORC_Q], e1[ORC_Q], e2[ORC_Q];
        double rho = 0.0, J[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < ORC_Q; ++i) {
            fl[i] = S->f[i * n + id];
            rho += fl[i];
            for (int k = 0; k < 3; ++k) J[k] += CV[i][k] * fl[i];
        }
        double u[3], du[3], u2[3];
        double B = S->B[id];
        for (int k = 0; k < 3; ++k) {
            u[k] = J[k] / rho;
            du[k] = B * (S->up[3 * id + k] - u[k]) + S->a_ext[k];
            u2[k] = u[k] + du[k];
        }
        orc_feq(rho, u, e1);
        orc_feq(rho, u2, e2);
        for (int i = 0; i < ORC_Q; ++i)
            S->fs[i * n + id] = fl[i] - (fl[i] - e1[i]) / P->tau + (e2[i] - e1[i]);
        S->rho_c[id] = rho;
        for (int k = 0; k < 3; ++k) {
            S->J_c[3 * id + k] = J[k];
            S->du_c[3 * id + k] = du[k];
        }
    }
}

/* ======================================================================
 * Time step (Sec. 4.4, Algorithm 1): couple fluid to particles; then, in
 * each of n_sub sub-steps of length 1/n_sub with the hydrodynamic force and
 * torque held constant, treat contacts, apply gravity and move particles,
 * couple particles to fluid with contact detection; finally collide.  The
 * stored state between steps is the post-collision field f*, so each step
 * begins with the streaming half of the previous "collide and stream".  The
 * contact forces reported are those of the last sub-step.
 * ====================================================================== */
/* ======================================================================
 * Zero-net-flux balance force (balance mode 2), a reading of Sec. 5.1: the
 * uniform fluid acceleration is chosen so that the suspension keeps a net
 * volume flow rate of zero.  The lattice covers the particles too (their
 * nodes move with u_p), so the net flow is the lattice momentum
 * P = sum_x sum_i c_i f_i*.  Streaming conserves P on a periodic box; the
 * collision of step t adds C_t (coupling and any fluid_accel) plus b_t M,
 * with M = sum_x rho the lattice mass and b_t the controller part of the
 * acceleration.  Aiming at P_{t+1} = 0 with the coupling of step t+1 taken
 * as that of step t:
 *     C_t = P_t - P_{t-1} - b_t M,   b_{t+1} = -(P_t + C_t) / M,
 * and b_0 = -P_{-1} / M from the initial populations.  P stays at the size
 * of the step-to-step change of C instead of accumulating it.
 * ====================================================================== */
static void lattice_momentum(const orc_sim *S, double *M, double *P)
{
    long n = S->n;
    double m = 0.0, p[3] = {0.0, 0.0, 0.0};
    for (long id = 0; id < n; ++id)
        for (int i = 0; i < ORC_Q; ++i) {
            double v = S->fs[i * n + id];
            m += v;
            for (int k = 0; k < 3; ++k) p[k] += CV[i][k] * v;
        }
    if (M) *M = m;
    for (int k = 0; k < 3; ++k) P[k] = p[k];
}

static void balance_start(orc_sim *S)
{
    if (S->P.balance != 2 || !S->P.periodic_z) return;
    lattice_momentum(S, &S->bal_M, S->bal_P);
    for (int k = 0; k < 3; ++k) {
        S->bal_b[k] = -S->bal_P[k] / S->bal_M;
        S->a_ext[k] = S->P.fluid_accel[k] + S->bal_b[k];
    }
}

static void balance_update(orc_sim *S)
{
    if (S->P.balance != 2 || !S->P.periodic_z) return;
    double P[3];
    lattice_momentum(S, NULL, P);
    for (int k = 0; k < 3; ++k) {
        double C = P[k] - S->bal_P[k] - S->bal_b[k] * S->bal_M;
        S->bal_b[k] = -(P[k] + C) / S->bal_M;
        S->bal_P[k] = P[k];
        S->a_ext[k] = S->P.fluid_accel[k] + S->bal_b[k];
    }
}

static int prologue(orc_sim *S)
{
    balance_start(S);
    if (couple_and_detect_nodes(S) != 0) {
        set_err(S, "detection set overflow (more than ORC_MAXK particles at a node)");
        return -1;
    }
    return detect_and_merge(S, 0);
}

int orc_init_equilibrium(orc_sim *S, double rho, const double u[3])
{
    double e[ORC_Q];
    orc_feq(rho, u, e);
    for (int i = 0; i < ORC_Q; ++i)
        for (long id = 0; id < S->n; ++id) S->fs[i * S->n + id] = e[i];
    S->ncon = 0;
    S->step = 0;
    return prologue(S);
}

int orc_set_populations(orc_sim *S, const double *fs)
{
    memcpy(S->fs, fs, sizeof(double) * ORC_Q * S->n);
    S->ncon = 0;
    S->step = 0;
    return prologue(S);
}

int orc_step(orc_sim *S, int nsteps)
{
    for (int it = 0; it < nsteps; ++it) {
        stream(S);
        momentum_exchange(S);
        const int nsub = S->P.n_sub > 1 ? S->P.n_sub : 1;
        for (int sub = 0; sub < nsub; ++sub) {
            int nkeep = treat_contacts(S);
            move_particles(S, 1.0 / (double)nsub);
            if (couple_and_detect_nodes(S) != 0) {
                set_err(S, "detection set overflow (more than ORC_MAXK particles at a node)");
                return -1;
            }
            detect_and_merge(S, nkeep);
        }
        collide(S);
        balance_update(S);
        S->step++;
    }
    return 0;
}

/* ======================================================================
 * Read-out
 * ====================================================================== */
void orc_get_populations(const orc_sim *S, double *fs)
{
    memcpy(fs, S->fs, sizeof(double) * ORC_Q * S->n);
}

void orc_get_post_stream(const orc_sim *S, double *f)
{
    memcpy(f, S->f, sizeof(double) * ORC_Q * S->n);
}

/* density and velocity moments of the stored post-collision field, plus the
   coupling fields at the current particle state */
void orc_get_fields(const orc_sim *S, double *rho, double *u, int *owner,
                    double *B, double *up)
{
    long n = S->n;
    for (long id = 0; id < n; ++id) {
        double r = 0.0, J[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < ORC_Q; ++i) {
            double v = S->fs[i * n + id];
            r += v;
            for (int k = 0; k < 3; ++k) J[k] += CV[i][k] * v;
        }
        if (rho) rho[id] = r;
        if (u)
            for (int k = 0; k < 3; ++k) u[3 * id + k] = J[k] / r;
    }
    if (owner) memcpy(owner, S->owner, sizeof(int) * n);
    if (B) memcpy(B, S->B, sizeof(double) * n);
    if (up) memcpy(up, S->up, sizeof(double) * 3 * n);
}

void orc_get_collision_diag(const orc_sim *S, double *rho, double *J,
                            double *du)
{
    memcpy(rho, S->rho_c, sizeof(double) * S->n);
    memcpy(J, S->J_c, sizeof(double) * 3 * S->n);
    memcpy(du, S->du_c, sizeof(double) * 3 * S->n);
}

void orc_get_mea_cells(const orc_sim *S, double *Scell)
{
    memcpy(Scell, S->Scell, sizeof(double) * 3 * S->n);
}

void orc_get_particles(const orc_sim *S, double *X, double *q, double *U,
                       double *w)
{
    for (int i = 0; i < S->np; ++i) {
        for (int k = 0; k < 3; ++k) {
            X[3 * i + k] = S->p[i].X[k];
            U[3 * i + k] = S->p[i].U[k];
            w[3 * i + k] = S->p[i].w[k];
        }
        for (int k = 0; k < 4; ++k) q[4 * i + k] = S->p[i].q[k];
    }
}

void orc_get_forces(const orc_sim *S, double *Fh, double *Th, double *Fc,
                    double *Tc)
{
    size_t b = sizeof(double) * 3 * S->np;
    memcpy(Fh, S->Fh, b);
    memcpy(Th, S->Th, b);
    memcpy(Fc, S->Fc, b);
    memcpy(Tc, S->Tc, b);
}

int orc_num_contacts(const orc_sim *S) { return S->ncon; }

void orc_get_contacts(const orc_sim *S, orc_contact *out)
{
    memcpy(out, S->con, sizeof(orc_contact) * S->ncon);
}

void orc_get_counters(const orc_sim *S, long long *pairs, long long *cells)
{
    *pairs = S->det_pairs;
    *cells = S->det_cells;
}

void orc_get_balance(const orc_sim *S, double *a_ext)
{
    for (int k = 0; k < 3; ++k) a_ext[k] = S->a_ext[k];
}
