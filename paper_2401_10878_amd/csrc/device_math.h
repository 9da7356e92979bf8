// Device-side building blocks shared by the gfx950 kernels: the D3Q19
// velocity set, particle geometry (rotation, signed distances, coupling
// weight) and small wavefront reductions.
//
// The signed distances and predicates that decide integer results (node
// ownership, detection sets, inside-samples of the overlap integration) are
// written as explicit left-to-right FP64 expressions and the library is
// built with -ffp-contract=off, so every node and sample gets the value the
// formula defines, independent of the launch shape.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hlbm {

constexpr int Q = 19;
// Two tilings of the lattice, each with a per-tile particle candidate list:
//  - detection tiles of 4 x 4 x 4 nodes, one wavefront each (compact, so
//    few particles reach a tile);
//  - lattice blocks of 64 x 4 x 1 nodes, one workgroup of four wavefronts,
//    each wavefront streaming one 64-node x-row (full-width coalesced rows).
//    (A 64 x 1 x 4 block, with most z links inside the block, cut the
//    momentum-exchange pass's L2 fetches by a quarter without making it
//    faster, and slowed the stream-collide pass by 5%.)
constexpr int DX = 4, DY = 4, DZ = 4;
constexpr int LX = 64, LY = 4, LZ = 1;
constexpr int LCAP_MAX = 64;    // lattice-block candidate capacity
constexpr int MAXC = 32;        // contacts per particle in one step
constexpr int BAL_PARTS = 256;  // first-stage workgroups of the balance sums
// FP32 screening record of a particle, per particle: centre (3), rotation
// (9), then the detection thresholds with the particle's FP32 error bound
// tol: eps/2 + tol, eps/2 - tol, sqrt(0.75) + delta_c + tol,
// sqrt(0.75) + delta_c - tol, the larger upper threshold, the size and
// the shape code (its bits)
constexpr int SREC = 20;
// FP32 kinematic record of a particle for the lattice pass (FP32 and
// binary16 storage), 128 bytes (a record address is a shift of the id): the
// integer part of the centre (3, int bits) and its fraction (3), U (3),
// omega (3), the rotation (9), the size and the shape code (its bits), then
// unused words.  A node's offset from the centre is the integer difference
// wrapped to the minimum image minus the fraction: one rounding, as for the
// FP64 offset rounded to FP32.
constexpr int LREC = 32;
// owner-map entry: the owning particle's id, or -1 (no owner)
__device__ inline int owner_id(int v) { return v < 0 ? -1 : v; }
constexpr int WAVE = 64;
constexpr double DETECT = 0.8660254037844386;   // sqrt(0.75), Sec. 3.3.1
constexpr double PI = 3.141592653589793;
constexpr uint64_t EMPTY_KEY = ~0ull;

// D3Q19 (Sec. 3.1): rest, the six axis directions, the twelve edge
// directions; each direction is followed by its opposite.
__host__ __device__ constexpr int cx(int i) {
  constexpr int t[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
  return t[i];
}
__host__ __device__ constexpr int cy(int i) {
  constexpr int t[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
  return t[i];
}
__host__ __device__ constexpr int cz(int i) {
  constexpr int t[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
  return t[i];
}
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
__host__ __device__ constexpr double wgt(int i) {
  return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
}

// Particle record in device memory (structure of arrays, FP64).
// Convex polyhedron type (shape POLY0 + k): vertices re-centred at the
// solid's centroid, face planes n . p <= h (n, h per face), face vertex
// lists (fs[f] .. fs[f+1] into fv, counter-clockwise seen from outside),
// undirected edges, circumradius; all at unit scale.  An ellipsoid type
// (kind 1) uses the same slot: semi-axes in v[0] (vf[0] rounded), rc the
// longest, no faces.
constexpr int POLY0 = 3, MAXPOLY = 8;
constexpr int PV = 64, PF = 64, PFV = 384, PE = 128;
constexpr int KIND_POLY = 0, KIND_ELLIPSOID = 1;
struct PolyDev {
  int nv, nf, ne, kind;
  double rc;
  double v[PV][3];
  double pl[PF][4];
  int fs[PF + 1];
  int fv[PFV];
  int e[PE][2];
  double ed[PFV][4];     // boundary edge of slot m: fv[m] -> next vertex of
                        // its face, as (b - a, 1 / |b - a|^2)
  double sd[PFV][4];     // side plane of slot m: s = n x (b - a), s . a; a
                        // point projects into the face when s . p >= s . a
                        // for each of its slots
  float vf[PV][3];      // v, pl, ed and sd rounded to FP32 (the FP32 forms)
  float plf[PF][4];
  float ef[PFV][4];
  float sf[PFV][4];
};

// Polyhedron tables are read through the constant address space: they do
// not change while a kernel runs, so loads from a wave-uniform type become
// scalar loads.
#define HLBM_CONST __attribute__((address_space(4)))
typedef const HLBM_CONST PolyDev CPoly;
__device__ inline const HLBM_CONST double* poly_vert(CPoly* P, int i, double) { return P->v[i]; }
__device__ inline const HLBM_CONST float* poly_vert(CPoly* P, int i, float) { return P->vf[i]; }
__device__ inline const HLBM_CONST double* poly_plane(CPoly* P, int f, double) { return P->pl[f]; }
__device__ inline const HLBM_CONST float* poly_plane(CPoly* P, int f, float) { return P->plf[f]; }
__device__ inline const HLBM_CONST double* poly_edge(CPoly* P, int m, double) { return P->ed[m]; }
__device__ inline const HLBM_CONST float* poly_edge(CPoly* P, int m, float) { return P->ef[m]; }
__device__ inline const HLBM_CONST double* poly_side(CPoly* P, int m, double) { return P->sd[m]; }
__device__ inline const HLBM_CONST float* poly_side(CPoly* P, int m, float) { return P->sf[m]; }

struct Particles {
  int n;
  const int* shape;     // 0 sphere, 1 cube, 2 octahedron, POLY0 + k polyhedron
  const double* size;   // radius, edge, vertex distance or scale
  const double* dens;   // density ratio s
  const double* vol;    // volume
  const double* mass;   // s * V
  const double* inert;  // isotropic moment of inertia
  double* X;            // [n][3]
  double* q;            // [n][4]
  double* U;            // [n][3]
  double* W;            // [n][3] angular velocity
  double* R;            // [n][9] rotation (body -> world), row-major
  float* XR32;          // [n][SREC] FP32 screening record of detection
  float* LR32;          // [n][LREC] FP32 kinematic record of the lattice pass
  const double* Iinv;   // [n][9] inverse body inertia tensor (polyhedra)
  const PolyDev* poly;  // [MAXPOLY] polyhedron types
};

// Half extent along world axis k of a body with rotation R: exact for
// cubes, polyhedra (largest |world coordinate| of a vertex) and ellipsoids,
// the circumradius for spheres and octahedra.
__device__ inline double half_extent(int shape, double size, const double* R, int k,
                                     const PolyDev* poly) {
  double e = size;
  if (shape == 1) e = 0.5 * size * (fabs(R[3 * k]) + fabs(R[3 * k + 1]) + fabs(R[3 * k + 2]));
  if (poly && shape >= POLY0 && ((CPoly*)poly + (shape - POLY0))->kind == KIND_ELLIPSOID) {
    // ellipsoid: the largest world coordinate over the surface,
    // |(R_k0 e0, R_k1 e1, R_k2 e2)|
    const HLBM_CONST double* ax = ((CPoly*)poly + (shape - POLY0))->v[0];
    const double a0 = R[3 * k] * ax[0], a1 = R[3 * k + 1] * ax[1], a2 = R[3 * k + 2] * ax[2];
    e = size * sqrt((a0 * a0 + a1 * a1) + a2 * a2);
  } else if (poly && shape >= POLY0) {
    CPoly* pd = (CPoly*)poly + (shape - POLY0);
    e = 0.0;
    for (int i = 0; i < pd->nv; ++i) {
      const double c = fabs((R[3 * k] * pd->v[i][0] + R[3 * k + 1] * pd->v[i][1]) +
                            R[3 * k + 2] * pd->v[i][2]);
      e = c > e ? c : e;
    }
    e = size * e;
  }
  return e;
}

// Rotation matrix of q = (w, x, y, z).
__device__ inline void quat_to_rot(const double* q, double* R) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
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

// Minimal image of a coordinate difference on an axis of length L.
// (selects rather than branches: per-lane branches here cost exec-mask
// bookkeeping on every axis of every candidate)
__device__ inline double minimg(double v, double L, bool periodic) {
  const double lo = v + L, hi = v - L;
  double r = (periodic && v >= 0.5 * L) ? hi : v;
  r = (periodic && v < -0.5 * L) ? lo : r;
  return r;
}
__device__ inline float minimg_f(float v, float L, bool periodic) {
  const float lo = v + L, hi = v - L;
  float r = (periodic && v >= 0.5f * L) ? hi : v;
  r = (periodic && v < -0.5f * L) ? lo : r;
  return r;
}
__device__ inline int image_shift(double v, double L, bool periodic) {
  if (!periodic) return 0;
  if (v >= 0.5 * L) return -1;
  if (v < -0.5 * L) return 1;
  return 0;
}

// Regular octahedron |x| + |y| + |z| <= a, folded into the positive octant
// (q = |p|): inside, the distance to the face plane x + y + z = a; outside,
// the distance to the face triangle a e_0, a e_1, a e_2 (its interior when
// the projection onto the plane has no negative coordinate, else the
// nearest of its three edges, first edge kept on ties).  T is double or
// float; gq (may be null) receives the unit gradient with respect to q.
template <typename T>
__device__ inline T octa_edge(T a, T qi, T qj, T& ci, T& cj) {
  T u = ((qj - qi) + a) / ((T)2 * a);
  u = u < (T)0 ? (T)0 : (u > (T)1 ? (T)1 : u);
  ci = a * ((T)1 - u);
  cj = a * u;
  return u;
}
template <typename T>
__device__ inline T octa_q(T a, T q0, T q1, T q2, T& g0, T& g1, T& g2) {
  const T inv3 = (T)0.57735026918962584;
  const T s = (q0 + q1) + q2;
  const T pd = (s - a) * inv3;
  const T t0 = q0 - (s - a) / (T)3, t1 = q1 - (s - a) / (T)3, t2 = q2 - (s - a) / (T)3;
  if (s <= a || (t0 >= (T)0 && t1 >= (T)0 && t2 >= (T)0)) {
    g0 = g1 = g2 = inv3;
    return pd;
  }
  T c0, c1, c2, best, b0, b1, b2;
  {  // edge a e_0 - a e_1
    octa_edge(a, q0, q1, c0, c1);
    const T dx = q0 - c0, dy = q1 - c1, dz = q2;
    best = (dx * dx + dy * dy) + dz * dz;
    b0 = c0; b1 = c1; b2 = (T)0;
  }
  {  // edge a e_1 - a e_2
    octa_edge(a, q1, q2, c1, c2);
    const T dx = q0, dy = q1 - c1, dz = q2 - c2;
    const T d2 = (dx * dx + dy * dy) + dz * dz;
    if (d2 < best) { best = d2; b0 = (T)0; b1 = c1; b2 = c2; }
  }
  {  // edge a e_2 - a e_0
    octa_edge(a, q2, q0, c2, c0);
    const T dx = q0 - c0, dy = q1, dz = q2 - c2;
    const T d2 = (dx * dx + dy * dy) + dz * dz;
    if (d2 < best) { best = d2; b0 = c0; b1 = (T)0; b2 = c2; }
  }
  const T d = sqrt(best);
  g0 = d > (T)0 ? (q0 - b0) / d : inv3;
  g1 = d > (T)0 ? (q1 - b1) / d : inv3;
  g2 = d > (T)0 ? (q2 - b2) / d : inv3;
  return d;
}
template <typename T>
__device__ inline T octa_q(T a, T q0, T q1, T q2) {
  T g0, g1, g2;
  return octa_q<T>(a, q0, q1, q2, g0, g1, g2);
}

// Signed distance of a unit-scale polyhedron at body point p (T = double or
// float, data in the same precision) and, if gb is given, its body-frame
// gradient.  Inside (every plane distance <= 0): the largest plane distance,
// gradient the normal of the first face attaining it.  Outside: the distance
// to the nearest boundary point, which is unique for a convex body.  When
// the projection onto the face of the largest plane distance lies in that
// face, that plane distance (a lower bound of the distance) is attained and
// is the result.  Otherwise the nearest point lies on a face the point is
// above (positive plane distance) or on the boundary of such a face: at a
// nearest point c, p - c is a non-negative combination of the normals of
// the faces through c, so (p - c) . n > 0 for one of them.  Those faces'
// interiors and boundary edges are searched; gradient the face normal or
// (p - c) / d.  With far < inf an outside point whose largest plane
// distance exceeds far returns that lower bound (screening: such a point is
// beyond every threshold).
// Whether body point p projects into face f: (b - a) x (p - a) . n >= 0,
// i.e. (n x (b - a)) . p >= (n x (b - a)) . a, along every boundary edge
// a -> b (counter-clockwise seen from outside; the offset along n drops out
// of the triple product).
template <typename T>
__device__ inline bool poly_face_contains(CPoly* P, int f, const T* p) {
  const int b0 = P->fs[f], cnt = P->fs[f + 1] - b0;
  bool inside = true;
  for (int j = 0; j < cnt; ++j) {
    const HLBM_CONST T* sp = poly_side(P, b0 + j, T());
    inside = inside && ((sp[0] * p[0] + sp[1] * p[1]) + sp[2] * p[2] >= sp[3]);
  }
  return inside;
}

// Signed distance of a unit-scale ellipsoid (semi-axes e) at body point p,
// negative inside, with the body-frame gradient (unit outward normal at the
// nearest surface point x), in the oracle's FP64 arithmetic.  Folded into
// the positive octant (y = |p|), the nearest point is x_k = e_k^2 y_k /
// (t + e_k^2) where G(t) = sum_k (e_k y_k / (t + e_k^2))^2 - 1 vanishes; G
// decreases on t > -m (m the smallest e_k^2; terms with y_k = 0 vanish).
// The root there is the answer when a shortest axis has y_k > 0, or when
// those components are all zero and G's limit at -m is positive; otherwise
// t = -m, the longer axes take x_k = e_k^2 y_k / (e_k^2 - m) and the first
// shortest axis the rest of the unit sum.  The root is bisected from the
// bracket [e_k y_k - m (or -m), |e y| - m] until the midpoint repeats an
// end.  With far < inf, a point with |p| - rc > far returns that lower
// bound with gradient p / |p|.
// G(t) over the three axes in order (terms with y_k = 0 vanish).
// (e_k^2 recomputed rather than held: the same rounded value, fewer live
// registers inside the loop)
__device__ inline double ellip_g(double e0, double e1, double e2, double y0, double y1,
                                 double y2, double t) {
  double g = -1.0;
  if (y0 > 0.0) {
    const double r = e0 * y0 / (t + e0 * e0);
    g += r * r;
  }
  if (y1 > 0.0) {
    const double r = e1 * y1 / (t + e1 * e1);
    g += r * r;
  }
  if (y2 > 0.0) {
    const double r = e2 * y2 / (t + e2 * e2);
    g += r * r;
  }
  return g;
}

// (scalars rather than small arrays, so that nothing lands in scratch)
__device__ inline double ellip_sdf_unit(CPoly* P, const double* p, double* gb, double far) {
  if (far < 1e300) {
    const double r = sqrt((p[0] * p[0] + p[1] * p[1]) + p[2] * p[2]);
    const double lb = r - P->rc;
    if (lb > far) {
      if (gb) {
        gb[0] = p[0] / r;
        gb[1] = p[1] / r;
        gb[2] = p[2] / r;
      }
      return lb;
    }
  }
  const double e0 = P->v[0][0], e1 = P->v[0][1], e2 = P->v[0][2];
  const double y0 = fabs(p[0]), y1 = fabs(p[1]), y2 = fabs(p[2]);
  const double q0 = e0 * e0, q1 = e1 * e1, q2 = e2 * e2;   // e_k^2
  double m = q0;
  if (q1 < m) m = q1;
  if (q2 < m) m = q2;
  // first shortest axis with y_k > 0
  const int kmin = (q0 == m && y0 > 0.0) ? 0
                 : ((q1 == m && y1 > 0.0) ? 1 : ((q2 == m && y2 > 0.0) ? 2 : -1));
  bool root = true;
  if (kmin < 0) {
    double g = -1.0;
    if (q0 > m && y0 > 0.0) {
      const double r = e0 * y0 / (q0 - m);
      g += r * r;
    }
    if (q1 > m && y1 > 0.0) {
      const double r = e1 * y1 / (q1 - m);
      g += r * r;
    }
    if (q2 > m && y2 > 0.0) {
      const double r = e2 * y2 / (q2 - m);
      g += r * r;
    }
    root = g > 0.0;
  }
  double x0, x1, x2, t;
  if (root) {
    double s = 0.0;
    s += (e0 * y0) * (e0 * y0);
    s += (e1 * y1) * (e1 * y1);
    s += (e2 * y2) * (e2 * y2);
    const double ek = kmin == 0 ? e0 : (kmin == 1 ? e1 : e2);
    const double yk = kmin == 0 ? y0 : (kmin == 1 ? y1 : y2);
    double lo = kmin >= 0 ? ek * yk - m : -m;
    double hi = sqrt(s) - m;
    if (hi < lo) hi = lo;
#pragma unroll 1
    for (int it = 0; it < 2200; ++it) {
      const double tm = 0.5 * (lo + hi);
      if (tm == lo || tm == hi) break;
      const double g = ellip_g(e0, e1, e2, y0, y1, y2, tm);
      if (g > 0.0) lo = tm;
      else if (g < 0.0) hi = tm;
      else {
        lo = tm;
        hi = tm;
      }
    }
    t = lo;
    x0 = q0 * y0 / (t + q0);
    x1 = q1 * y1 / (t + q1);
    x2 = q2 * y2 / (t + q2);
  } else {
    t = -m;
    double s = 1.0;
    int kf = -1;
    x0 = 0.0;
    x1 = 0.0;
    x2 = 0.0;
    if (q0 > m) {
      x0 = q0 * y0 / (q0 - m);
      s -= (x0 / e0) * (x0 / e0);
    } else if (kf < 0) {
      kf = 0;
    }
    if (q1 > m) {
      x1 = q1 * y1 / (q1 - m);
      s -= (x1 / e1) * (x1 / e1);
    } else if (kf < 0) {
      kf = 1;
    }
    if (q2 > m) {
      x2 = q2 * y2 / (q2 - m);
      s -= (x2 / e2) * (x2 / e2);
    } else if (kf < 0) {
      kf = 2;
    }
    const double xf = sqrt(s > 0.0 ? s : 0.0);
    if (kf == 0) x0 = e0 * xf;
    if (kf == 1) x1 = e1 * xf;
    if (kf == 2) x2 = e2 * xf;
  }
  const double dx = y0 - x0, dy = y1 - x1, dz = y2 - x2;
  const double d = sqrt((dx * dx + dy * dy) + dz * dz);
  if (gb) {
    const double n0 = x0 / q0, n1 = x1 / q1, n2 = x2 / q2;
    const double nn = sqrt((n0 * n0 + n1 * n1) + n2 * n2);
    gb[0] = (p[0] < 0.0 ? -n0 : n0) / nn;
    gb[1] = (p[1] < 0.0 ? -n1 : n1) / nn;
    gb[2] = (p[2] < 0.0 ? -n2 : n2) / nn;
  }
  return t < 0.0 ? -d : d;
}

// The same distance for the forms that need its value, not the oracle's
// bits (the lattice pass's coupling weight, the detection screen, the
// fields): the multiplier by Newton's method instead of bisection.  G is
// convex and decreasing on t > -m, so Newton steps from the bracket's lower
// end (G >= 0) rise monotonically to the root (each lands at or left of
// it) and stop when a step no longer changes t; the free branch is the
// exact form's.  A few steps against up to a hundred halvings, so a
// wavefront with one band node in it does not wait for the bisection.
template <typename T>
__device__ inline T ellip_sdf_newton(CPoly* P, const T* p, T* gb, T far) {
  if (far < (T)1e30) {
    const T r = sqrt((p[0] * p[0] + p[1] * p[1]) + p[2] * p[2]);
    const T lb = r - (T)P->rc;
    if (lb > far) {
      if (gb) {
        gb[0] = p[0] / r;
        gb[1] = p[1] / r;
        gb[2] = p[2] / r;
      }
      return lb;
    }
  }
  const T e0 = (T)P->v[0][0], e1 = (T)P->v[0][1], e2 = (T)P->v[0][2];
  const T y0 = fabs(p[0]), y1 = fabs(p[1]), y2 = fabs(p[2]);
  const T q0 = e0 * e0, q1 = e1 * e1, q2 = e2 * e2;
  T m = q0;
  if (q1 < m) m = q1;
  if (q2 < m) m = q2;
  const int kmin = (q0 == m && y0 > (T)0) ? 0
                 : ((q1 == m && y1 > (T)0) ? 1 : ((q2 == m && y2 > (T)0) ? 2 : -1));
  bool root = true;
  if (kmin < 0) {
    T g = -(T)1;
    if (q0 > m && y0 > (T)0) g += (e0 * y0 / (q0 - m)) * (e0 * y0 / (q0 - m));
    if (q1 > m && y1 > (T)0) g += (e1 * y1 / (q1 - m)) * (e1 * y1 / (q1 - m));
    if (q2 > m && y2 > (T)0) g += (e2 * y2 / (q2 - m)) * (e2 * y2 / (q2 - m));
    root = g > (T)0;
  }
  T x0 = (T)0, x1 = (T)0, x2 = (T)0, t;
  if (root) {
    const T ek = kmin == 0 ? e0 : (kmin == 1 ? e1 : e2);
    const T yk = kmin == 0 ? y0 : (kmin == 1 ? y1 : y2);
    t = kmin >= 0 ? ek * yk - m : -m;
#pragma unroll 1
    for (int it = 0; it < 100; ++it) {
      const T a0 = y0 > (T)0 ? e0 * y0 / (t + q0) : (T)0;
      const T a1 = y1 > (T)0 ? e1 * y1 / (t + q1) : (T)0;
      const T a2 = y2 > (T)0 ? e2 * y2 / (t + q2) : (T)0;
      const T g = ((a0 * a0 + a1 * a1) + a2 * a2) - (T)1;
      if (!(g > (T)0)) break;
      // -G'(t) / 2 (terms with y_k = 0 are zero; t may start at -m, where
      // such a term's denominator vanishes)
      const T h0 = y0 > (T)0 ? a0 * a0 / (t + q0) : (T)0;
      const T h1 = y1 > (T)0 ? a1 * a1 / (t + q1) : (T)0;
      const T h2 = y2 > (T)0 ? a2 * a2 / (t + q2) : (T)0;
      const T h = (h0 + h1) + h2;
      const T tn = t + (T)0.5 * g / h;
      if (!(tn > t)) break;
      t = tn;
    }
    x0 = y0 > (T)0 ? q0 * y0 / (t + q0) : (T)0;
    x1 = y1 > (T)0 ? q1 * y1 / (t + q1) : (T)0;
    x2 = y2 > (T)0 ? q2 * y2 / (t + q2) : (T)0;
  } else {
    t = -m;
    T s = (T)1;
    int kf = -1;
    if (q0 > m) {
      x0 = q0 * y0 / (q0 - m);
      s -= (x0 / e0) * (x0 / e0);
    } else if (kf < 0) {
      kf = 0;
    }
    if (q1 > m) {
      x1 = q1 * y1 / (q1 - m);
      s -= (x1 / e1) * (x1 / e1);
    } else if (kf < 0) {
      kf = 1;
    }
    if (q2 > m) {
      x2 = q2 * y2 / (q2 - m);
      s -= (x2 / e2) * (x2 / e2);
    } else if (kf < 0) {
      kf = 2;
    }
    const T xf = sqrt(s > (T)0 ? s : (T)0);
    if (kf == 0) x0 = e0 * xf;
    if (kf == 1) x1 = e1 * xf;
    if (kf == 2) x2 = e2 * xf;
  }
  const T dx = y0 - x0, dy = y1 - x1, dz = y2 - x2;
  const T d = sqrt((dx * dx + dy * dy) + dz * dz);
  if (gb) {
    const T n0 = x0 / q0, n1 = x1 / q1, n2 = x2 / q2;
    const T nn = sqrt((n0 * n0 + n1 * n1) + n2 * n2);
    gb[0] = (p[0] < (T)0 ? -n0 : n0) / nn;
    gb[1] = (p[1] < (T)0 ? -n1 : n1) / nn;
    gb[2] = (p[2] < (T)0 ? -n2 : n2) / nn;
  }
  return t < (T)0 ? -d : d;
}

// Bounds of an ellipsoid's signed distance from its scaled copies: with
// s = sqrt(sum_k (p_k / e_k)^2), p lies on the surface of sE, and since E
// = sE + (1 - s)E contains sE plus the ball of radius (1 - s) e_min (and
// sE = E + (s - 1)E for s > 1), d lies in [(s - 1) e_min, (s - 1) e_max]
// outside and in [(s - 1) e_max, (s - 1) e_min] inside (unit scale; the
// nearest point of the scaled surface point is at most (1 - s) |z| <=
// (1 - s) e_max away).  Used to skip the nearest-point solve where only a
// comparison with a threshold far from d is needed.
template <typename T>
__device__ inline void ellip_bounds(CPoly* P, const T* p, T& dlo, T& dhi) {
  const HLBM_CONST double* e = P->v[0];
  const T e0 = (T)e[0], e1 = (T)e[1], e2 = (T)e[2];
  const T q0 = p[0] / e0, q1 = p[1] / e1, q2 = p[2] / e2;
  const T s = sqrt((q0 * q0 + q1 * q1) + q2 * q2);
  const T emin = e0 < e1 ? (e0 < e2 ? e0 : e2) : (e1 < e2 ? e1 : e2);
  const T emax = (T)P->rc;
  const T sm = s - (T)1;
  dlo = sm * (sm >= (T)0 ? emin : emax);
  dhi = sm * (sm >= (T)0 ? emax : emin);
}

template <typename T, bool ELL = false>
__device__ inline T poly_sdf_unit(CPoly* P, const T* p, T* gb, T far) {
  if (ELL && P->kind == KIND_ELLIPSOID) {
    // smooth body: the distance by Newton's method in T (FP32 forms
    // evaluate it only near the surface, where it is well conditioned)
    return ellip_sdf_newton<T>(P, p, gb, far);
  }
  const int nf = P->nf;
  T best = (T)-1e30;
  int fm = 0;
  for (int f = 0; f < nf; ++f) {
    const HLBM_CONST T* pl = poly_plane(P, f, T());
    const T d = (pl[0] * p[0] + pl[1] * p[1]) + pl[2] * p[2] - pl[3];
    if (d > best) {
      best = d;
      fm = f;
    }
  }
  if (best <= (T)0 || best > far) {
    if (gb)
      for (int k = 0; k < 3; ++k) gb[k] = poly_plane(P, fm, T())[k];
    return best;
  }
  {
    // the face test with per-lane face data (a pass per distinct face of the
    // wavefront with the face in scalar registers was slower)
    if (poly_face_contains<T>(P, fm, p)) {
      if (gb)
        for (int k = 0; k < 3; ++k) gb[k] = poly_plane(P, fm, T())[k];
      return best;
    }
  }
  T dmin2 = (T)1e30, c0 = (T)0, c1 = (T)0, c2 = (T)0, dface = (T)0;
  int face_hit = -1;
  for (int f = 0; f < nf; ++f) {
    const HLBM_CONST T* n = poly_plane(P, f, T());
    const T d = (n[0] * p[0] + n[1] * p[1]) + n[2] * p[2] - n[3];
    if (d <= (T)0) continue;
    const int b0 = P->fs[f], cnt = P->fs[f + 1] - b0;
    bool inside = true;
    for (int j = 0; j < cnt; ++j) {
      const HLBM_CONST T* a = poly_vert(P, P->fv[b0 + j], T());
      const HLBM_CONST T* e = poly_edge(P, b0 + j, T());
      const HLBM_CONST T* sp = poly_side(P, b0 + j, T());
      const T e0 = e[0], e1 = e[1], e2 = e[2];
      const T w0 = p[0] - a[0], w1 = p[1] - a[1], w2 = p[2] - a[2];
      inside = inside && ((sp[0] * p[0] + sp[1] * p[1]) + sp[2] * p[2] >= sp[3]);
      // nearest point of the segment a -> a + e
      T t = ((w0 * e0 + w1 * e1) + w2 * e2) * e[3];
      t = t < (T)0 ? (T)0 : (t > (T)1 ? (T)1 : t);
      const T y0 = a[0] + t * e0, y1 = a[1] + t * e1, y2 = a[2] + t * e2;
      const T dx = p[0] - y0, dy = p[1] - y1, dz = p[2] - y2;
      const T d2 = (dx * dx + dy * dy) + dz * dz;
      if (d2 < dmin2) {
        dmin2 = d2;
        face_hit = -1;
        c0 = y0;
        c1 = y1;
        c2 = y2;
      }
    }
    if (inside && d * d < dmin2) {
      dmin2 = d * d;
      dface = d;
      face_hit = f;
    }
  }
  const T d = face_hit >= 0 ? dface : sqrt(dmin2);
  if (gb) {
    if (face_hit >= 0) {
      for (int k = 0; k < 3; ++k) gb[k] = poly_plane(P, face_hit, T())[k];
    } else {
      gb[0] = (p[0] - c0) / d;
      gb[1] = (p[1] - c1) / d;
      gb[2] = (p[2] - c2) / d;
    }
  }
  return d;
}

// poly_sdf_unit for polyhedron type t of the table: when every active lane
// of the wavefront asks for the same type, the table address is uniform.
template <typename T, bool ELL = false>
__device__ inline T poly_sdf(const PolyDev* table, int t, const T* p, T* gb, T far) {
  CPoly* base = (CPoly*)table;
  // ellipsoid types first, one evaluation for every lane (a copy in each
  // branch below would double the inlined code)
  if (ELL && base[t].kind == KIND_ELLIPSOID) return poly_sdf_unit<T, true>(base + t, p, gb, far);
  const int t0 = __builtin_amdgcn_readfirstlane(t);
  if (__ballot(t != t0) == 0) return poly_sdf_unit<T, false>(base + t0, p, gb, far);
  return poly_sdf_unit<T, false>(base + t, p, gb, far);
}

// The same distance in the oracle's own arithmetic, for the FP64 decisions
// that must come out bit for bit alike (node ownership and rough detection,
// and the box correction and overlap integration of a contact): the plane
// distances of every face; inside, the largest; outside, the smallest of
// the distances to the face interiors the point projects into (faces it is
// above, the projection tested against each boundary edge with a cross
// product) and to every undirected edge (segment projection divided by
// |e|^2), faces first and then edges in table order on ties.  With far <
// inf, an outside point whose largest plane distance exceeds far returns
// that lower bound (for the integration's inside test only).
template <bool ELL = false>
__device__ inline double poly_sdf_exact_unit(CPoly* P, const double* p, double* gb,
                                             double far) {
  if (ELL && P->kind == KIND_ELLIPSOID) return ellip_sdf_unit(P, p, gb, far);
  const int nf = P->nf;
  double best = -1e300;
  int fm = 0;
  for (int f = 0; f < nf; ++f) {
    const HLBM_CONST double* n = P->pl[f];
    const double d = (n[0] * p[0] + n[1] * p[1]) + n[2] * p[2] - n[3];
    if (d > best) {
      best = d;
      fm = f;
    }
  }
  if (best <= 0.0 || best > far) {
    if (gb)
      for (int k = 0; k < 3; ++k) gb[k] = P->pl[fm][k];
    return best;
  }
  double dmin2 = 1e300, c0 = 0.0, c1 = 0.0, c2 = 0.0;
  int face_hit = -1;
  for (int f = 0; f < nf; ++f) {
    const HLBM_CONST double* n = P->pl[f];
    const double d = (n[0] * p[0] + n[1] * p[1]) + n[2] * p[2] - n[3];
    if (d <= 0.0) continue;
    const double q0 = p[0] - d * n[0], q1 = p[1] - d * n[1], q2 = p[2] - d * n[2];
    const int b0 = P->fs[f], cnt = P->fs[f + 1] - b0;
    bool inside = true;
    for (int j = 0; j < cnt; ++j) {
      const HLBM_CONST double* a = P->v[P->fv[b0 + j]];
      const HLBM_CONST double* b = P->v[P->fv[b0 + (j + 1 == cnt ? 0 : j + 1)]];
      const double e0 = b[0] - a[0], e1 = b[1] - a[1], e2 = b[2] - a[2];
      const double w0 = q0 - a[0], w1 = q1 - a[1], w2 = q2 - a[2];
      const double x0 = e1 * w2 - e2 * w1, x1 = e2 * w0 - e0 * w2, x2 = e0 * w1 - e1 * w0;
      if ((x0 * n[0] + x1 * n[1]) + x2 * n[2] < 0.0) inside = false;
    }
    if (inside && d * d < dmin2) {
      dmin2 = d * d;
      face_hit = f;
      c0 = q0;
      c1 = q1;
      c2 = q2;
    }
  }
  for (int i = 0; i < P->ne; ++i) {
    const HLBM_CONST double* a = P->v[P->e[i][0]];
    const HLBM_CONST double* b = P->v[P->e[i][1]];
    const double e0 = b[0] - a[0], e1 = b[1] - a[1], e2 = b[2] - a[2];
    const double w0 = p[0] - a[0], w1 = p[1] - a[1], w2 = p[2] - a[2];
    const double ee = (e0 * e0 + e1 * e1) + e2 * e2;
    double t = ((w0 * e0 + w1 * e1) + w2 * e2) / ee;
    t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
    const double y0 = a[0] + t * e0, y1 = a[1] + t * e1, y2 = a[2] + t * e2;
    const double dx = p[0] - y0, dy = p[1] - y1, dz = p[2] - y2;
    const double d2 = (dx * dx + dy * dy) + dz * dz;
    if (d2 < dmin2) {
      dmin2 = d2;
      face_hit = -1;
      c0 = y0;
      c1 = y1;
      c2 = y2;
    }
  }
  const double d = sqrt(dmin2);
  if (gb) {
    if (face_hit >= 0) {
      for (int k = 0; k < 3; ++k) gb[k] = P->pl[face_hit][k];
    } else {
      gb[0] = (p[0] - c0) / d;
      gb[1] = (p[1] - c1) / d;
      gb[2] = (p[2] - c2) / d;
    }
  }
  return d;
}
template <bool ELL = false>
__device__ inline double poly_sdf_exact(const PolyDev* table, int t, const double* p,
                                        double* gb, double far) {
  CPoly* base = (CPoly*)table;
  const int t0 = __builtin_amdgcn_readfirstlane(t);
  if (__ballot(t != t0) == 0) return poly_sdf_exact_unit<ELL>(base + t0, p, gb, far);
  return poly_sdf_exact_unit<ELL>(base + t, p, gb, far);
}

// Exact signed distance (negative inside) at world offset r from the centre.
// sphere: |r| - radius.  cube (edge a): body offset p = R^T r,
// q_k = |p_k| - a/2, d = |max(q, 0)| + min(max_k q_k, 0).
template <bool ELL = false>
__device__ inline double sdf(int shape, double size, const double* R,
                             double r0, double r1, double r2,
                             const PolyDev* poly) {
  if (poly && shape >= POLY0) {
    const double is = 1.0 / size;
    double p[3];
    p[0] = (R[0] * r0 + R[3] * r1 + R[6] * r2) * is;
    p[1] = (R[1] * r0 + R[4] * r1 + R[7] * r2) * is;
    p[2] = (R[2] * r0 + R[5] * r1 + R[8] * r2) * is;
    return size * poly_sdf<double, ELL>(poly, shape - POLY0, p, nullptr, 1e300);
  }
  if (shape == 2) {
    const double p0 = R[0] * r0 + R[3] * r1 + R[6] * r2;
    const double p1 = R[1] * r0 + R[4] * r1 + R[7] * r2;
    const double p2 = R[2] * r0 + R[5] * r1 + R[8] * r2;
    return octa_q<double>(size, fabs(p0), fabs(p1), fabs(p2));
  }
  if (shape == 0) {
    const double n2 = r0 * r0 + r1 * r1 + r2 * r2;
    return sqrt(n2) - size;
  }
  const double h = 0.5 * size;
  const double p0 = R[0] * r0 + R[3] * r1 + R[6] * r2;
  const double p1 = R[1] * r0 + R[4] * r1 + R[7] * r2;
  const double p2 = R[2] * r0 + R[5] * r1 + R[8] * r2;
  const double q0 = fabs(p0) - h, q1 = fabs(p1) - h, q2 = fabs(p2) - h;
  const double m0 = fmax(q0, 0.0), m1 = fmax(q1, 0.0), m2 = fmax(q2, 0.0);
  const double s2 = m0 * m0 + m1 * m1 + m2 * m2;
  const double outside = s2 > 0.0 ? sqrt(s2) : 0.0;
  const double inside = fmin(fmax(fmax(q0, q1), q2), 0.0);
  return outside + inside;
}

// sdf and sdf_grad with a polyhedron evaluated in the oracle's arithmetic
// (the body offset divided by the scale, poly_sdf_exact): the forms of the
// FP64 decisions; the other shapes share sdf / sdf_grad, which already
// follow it.
template <bool ELL = false>
__device__ inline double sdf_exact(int shape, double size, const double* R,
                                   double r0, double r1, double r2, const PolyDev* poly) {
  if (poly && shape >= POLY0) {
    double p[3];
    p[0] = (R[0] * r0 + R[3] * r1 + R[6] * r2) / size;
    p[1] = (R[1] * r0 + R[4] * r1 + R[7] * r2) / size;
    p[2] = (R[2] * r0 + R[5] * r1 + R[8] * r2) / size;
    return size * poly_sdf_exact<ELL>(poly, shape - POLY0, p, nullptr, 1e300);
  }
  return sdf<ELL>(shape, size, R, r0, r1, r2, poly);
}

// The same signed distance in FP32 arithmetic (inputs rounded to FP32, the
// rotation given in FP64 or already rounded; the hardware square root,
// within 1 ulp): its error is below 1e-6 (|r|_1 + size) plus a few units in
// the last place.
template <bool ELL = false, typename RT>
__device__ inline float sdf32(int shape, float size, const RT* R, float r0,
                              float r1, float r2, const PolyDev* poly) {
  if (shape == 0) return __builtin_amdgcn_sqrtf(r0 * r0 + r1 * r1 + r2 * r2) - size;
  if (poly && shape >= POLY0) {
    // exact at every distance (its callers evaluate nodes already known to
    // lie within eps/2 of the body)
    const float is = 1.0f / size;
    float p[3];
    p[0] = ((float)R[0] * r0 + (float)R[3] * r1 + (float)R[6] * r2) * is;
    p[1] = ((float)R[1] * r0 + (float)R[4] * r1 + (float)R[7] * r2) * is;
    p[2] = ((float)R[2] * r0 + (float)R[5] * r1 + (float)R[8] * r2) * is;
    return size * poly_sdf<float, ELL>(poly, shape - POLY0, p, nullptr, 1e30f);
  }
  const float h = 0.5f * size;
  const float p0 = (float)R[0] * r0 + (float)R[3] * r1 + (float)R[6] * r2;
  const float p1 = (float)R[1] * r0 + (float)R[4] * r1 + (float)R[7] * r2;
  const float p2 = (float)R[2] * r0 + (float)R[5] * r1 + (float)R[8] * r2;
  if (shape == 2) return octa_q<float>(size, fabsf(p0), fabsf(p1), fabsf(p2));
  const float q0 = fabsf(p0) - h, q1 = fabsf(p1) - h, q2 = fabsf(p2) - h;
  const float m0 = fmaxf(q0, 0.0f), m1 = fmaxf(q1, 0.0f), m2 = fmaxf(q2, 0.0f);
  return __builtin_amdgcn_sqrtf(m0 * m0 + m1 * m1 + m2 * m2) + fminf(fmaxf(fmaxf(q0, q1), q2), 0.0f);
}

// As sdf32, with the rotation already in FP32 and the hardware square root
// (within 1 ulp; used for screening against an error bound).  Products and
// sums may fuse here: a fused multiply-add rounds once, which keeps the
// error within the same bound.
// With ELL, an ellipsoid type returns a bound instead of the distance when
// the bound settles both thresholds: its lower bound when that exceeds far,
// its upper bound when that lies below inner (the rest, the exact distance).
template <bool ELL = false>
__device__ inline float sdf32_r(int shape, float size, const float* R, float r0,
                                float r1, float r2, const PolyDev* poly, float far,
                                float inner = -1e30f) {
#pragma clang fp contract(fast)
  if (shape == 0) return __builtin_amdgcn_sqrtf(r0 * r0 + r1 * r1 + r2 * r2) - size;
  if (ELL && poly && shape >= POLY0 &&
      ((CPoly*)poly + (shape - POLY0))->kind == KIND_ELLIPSOID) {
    CPoly* P = (CPoly*)poly + (shape - POLY0);
    const float is = 1.0f / size;
    float p[3];
    p[0] = (R[0] * r0 + R[3] * r1 + R[6] * r2) * is;
    p[1] = (R[1] * r0 + R[4] * r1 + R[7] * r2) * is;
    p[2] = (R[2] * r0 + R[5] * r1 + R[8] * r2) * is;
    float dlo, dhi;
    ellip_bounds<float>(P, p, dlo, dhi);
    if (size * dlo > far) return size * dlo;
    if (size * dhi < inner) return size * dhi;
    return size * poly_sdf_unit<float, true>(P, p, nullptr, 1e30f);
  }
  if (poly && shape >= POLY0) {
    // beyond far cells outside the plane lower bound is returned
    const float is = 1.0f / size;
    float p[3];
    p[0] = (R[0] * r0 + R[3] * r1 + R[6] * r2) * is;
    p[1] = (R[1] * r0 + R[4] * r1 + R[7] * r2) * is;
    p[2] = (R[2] * r0 + R[5] * r1 + R[8] * r2) * is;
    return size * poly_sdf<float, ELL>(poly, shape - POLY0, p, nullptr, far * is);
  }
  const float h = 0.5f * size;
  const float p0 = R[0] * r0 + R[3] * r1 + R[6] * r2;
  const float p1 = R[1] * r0 + R[4] * r1 + R[7] * r2;
  const float p2 = R[2] * r0 + R[5] * r1 + R[8] * r2;
  if (shape == 2) return octa_q<float>(size, fabsf(p0), fabsf(p1), fabsf(p2));
  const float q0 = fabsf(p0) - h, q1 = fabsf(p1) - h, q2 = fabsf(p2) - h;
  const float m0 = fmaxf(q0, 0.0f), m1 = fmaxf(q1, 0.0f), m2 = fmaxf(q2, 0.0f);
  return __builtin_amdgcn_sqrtf(m0 * m0 + m1 * m1 + m2 * m2) +
         fminf(fmaxf(fmaxf(q0, q1), q2), 0.0f);
}

// Signed distance with its world-frame gradient.  Inside a cube the
// gradient is the normal of the nearest face (ties to the lowest axis);
// at a sphere's centre it is zero.
// A polyhedron point farther outside than far (cells) may return the largest
// plane distance, a lower bound, with that face's normal.
template <bool ELL = false>
__device__ inline double sdf_grad(int shape, double size, const double* R,
                                  const double* r, double* g, const PolyDev* poly,
                                  double far = 1e300) {
  if (poly && shape >= POLY0) {
    const double is = 1.0 / size;
    double p[3], gb[3];
    #pragma unroll
    for (int k = 0; k < 3; ++k) p[k] = (R[0 + k] * r[0] + R[3 + k] * r[1] + R[6 + k] * r[2]) * is;
    const double d = size * poly_sdf<double, ELL>(poly, shape - POLY0, p, gb, far * is);
    #pragma unroll
    for (int k = 0; k < 3; ++k)
      g[k] = R[3 * k + 0] * gb[0] + R[3 * k + 1] * gb[1] + R[3 * k + 2] * gb[2];
    return d;
  }
  if (shape == 2) {
    const double p0 = R[0] * r[0] + R[3] * r[1] + R[6] * r[2];
    const double p1 = R[1] * r[0] + R[4] * r[1] + R[7] * r[2];
    const double p2 = R[2] * r[0] + R[5] * r[1] + R[8] * r[2];
    double q0, q1, q2;
    const double d = octa_q<double>(size, fabs(p0), fabs(p1), fabs(p2), q0, q1, q2);
    const double b0 = p0 < 0.0 ? -q0 : q0, b1 = p1 < 0.0 ? -q1 : q1, b2 = p2 < 0.0 ? -q2 : q2;
    #pragma unroll
    for (int k = 0; k < 3; ++k) g[k] = R[3 * k + 0] * b0 + R[3 * k + 1] * b1 + R[3 * k + 2] * b2;
    return d;
  }
  if (shape == 0) {
    const double n2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    const double n = sqrt(n2);
    #pragma unroll
    for (int k = 0; k < 3; ++k) g[k] = n > 0.0 ? r[k] / n : 0.0;
    return n - size;
  }
  const double h = 0.5 * size;
  double p[3], qd[3], m[3];
  #pragma unroll
  for (int k = 0; k < 3; ++k) {
    p[k] = R[0 + k] * r[0] + R[3 + k] * r[1] + R[6 + k] * r[2];
    qd[k] = fabs(p[k]) - h;
    m[k] = fmax(qd[k], 0.0);
  }
  const double outside = sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
  const double inside = fmin(fmax(fmax(qd[0], qd[1]), qd[2]), 0.0);
  double gb[3] = {0.0, 0.0, 0.0};
  if (outside > 0.0) {
    #pragma unroll
    for (int k = 0; k < 3; ++k) gb[k] = (p[k] < 0.0 ? -1.0 : 1.0) * m[k] / outside;
  } else {
    // nearest face: largest q_k, ties to the lowest axis (selects, no
    // run-time array index)
    int km = 0;
    double qm = qd[0];
    if (qd[1] > qm) { km = 1; qm = qd[1]; }
    if (qd[2] > qm) km = 2;
    gb[0] = km == 0 ? (p[0] < 0.0 ? -1.0 : 1.0) : 0.0;
    gb[1] = km == 1 ? (p[1] < 0.0 ? -1.0 : 1.0) : 0.0;
    gb[2] = km == 2 ? (p[2] < 0.0 ? -1.0 : 1.0) : 0.0;
  }
  #pragma unroll
  for (int k = 0; k < 3; ++k)
    g[k] = R[3 * k + 0] * gb[0] + R[3 * k + 1] * gb[1] + R[3 * k + 2] * gb[2];
  return outside + inside;
}

template <bool ELL = false>
__device__ inline double sdf_grad_exact(int shape, double size, const double* R,
                                        const double* r, double* g, const PolyDev* poly,
                                        double far = 1e300) {
  if (poly && shape >= POLY0) {
    double p[3], gb[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) p[k] = (R[0 + k] * r[0] + R[3 + k] * r[1] + R[6 + k] * r[2]) / size;
    const double d = size * poly_sdf_exact<ELL>(poly, shape - POLY0, p, gb, far / size);
#pragma unroll
    for (int k = 0; k < 3; ++k)
      g[k] = R[3 * k + 0] * gb[0] + R[3 * k + 1] * gb[1] + R[3 * k + 2] * gb[2];
    return d;
  }
  return sdf_grad<ELL>(shape, size, R, r, g, poly, far);
}

// For an ellipsoid type at world offset r: 1 when its distance bounds put
// r inside by more than eh + margin (B = 1), 0 when outside by more (B =
// 0), -1 otherwise and for other shapes (evaluate the distance).
template <typename T, typename RT>
__device__ inline int ellip_band(const PolyDev* poly, int shape, T size, const RT* R, T r0,
                                 T r1, T r2, T eh, T margin) {
  if (!(poly && shape >= POLY0)) return -1;
  CPoly* P = (CPoly*)poly + (shape - POLY0);
  if (P->kind != KIND_ELLIPSOID) return -1;
  const T is = (T)1 / size;
  T p[3];
  p[0] = ((T)R[0] * r0 + (T)R[3] * r1 + (T)R[6] * r2) * is;
  p[1] = ((T)R[1] * r0 + (T)R[4] * r1 + (T)R[7] * r2) * is;
  p[2] = ((T)R[2] * r0 + (T)R[5] * r1 + (T)R[8] * r2) * is;
  T dlo, dhi;
  ellip_bounds<T>(P, p, dlo, dhi);
  if (size * dhi <= -eh - margin) return 1;
  if (size * dlo >= eh + margin) return 0;
  return -1;
}

// Coupling weight B(d): 1 for d <= -eps/2, 0 for d >= eps/2, cos^2 ramp.
__device__ inline double weight(double d, double eps) {
  if (d <= -0.5 * eps) return 1.0;
  if (d >= 0.5 * eps) return 0.0;
  const double c = cos(PI * (d + 0.5 * eps) / (2.0 * eps));
  return c * c;
}

// FP32 form for the FP32 and binary16 storage: the hardware cosine of the
// angle in revolutions, cos(pi (d + eps/2) / (2 eps)) = cos(2 pi t) with
// t = (d + eps/2) / (4 eps) in [0, 1/4] (absolute error about 1e-6, below
// what the FP32 populations resolve of the velocity shift).
__device__ inline float weight32(float d, float eps_h, float eps_q) {
  // eps_h = eps / 2, eps_q = 1 / (4 eps), both rounded to FP32
  if (d <= -eps_h) return 1.0f;
  if (d >= eps_h) return 0.0f;
  const float c = __builtin_amdgcn_cosf((d + eps_h) * eps_q);
  return c * c;
}

// ---- wavefront reductions (64 lanes) -------------------------------------
// All-lane reductions built from DPP row rotations (row_ror 8, 4, 2, 1 within
// each row of 16 lanes) and four readlanes, so no data goes through LDS and
// the combination order is fixed.  Callers keep all 64 lanes active.
template <int K>
__device__ inline int ror_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x120 + K, 0xf, 0xf, false);
}
template <int K>
__device__ inline double ror_d(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(ror_i<K>(hi), ror_i<K>(lo));
}
__device__ inline double lane_d(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}
__device__ inline double wave_sum(double v) {
  v += ror_d<8>(v);
  v += ror_d<4>(v);
  v += ror_d<2>(v);
  v += ror_d<1>(v);
  return (lane_d(v, 0) + lane_d(v, 16)) + (lane_d(v, 32) + lane_d(v, 48));
}
// DPP move of an FP64 value within each row of 16 lanes.
template <int CTRL>
__device__ inline double dpp_d(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(__builtin_amdgcn_update_dpp(0, hi, CTRL, 0xf, 0xf, false),
                          __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xf, 0xf, false));
}
// Value of lane (l ^ 16) and of lane (l ^ 32).
__device__ inline double xor16_d(double v) {
  return __hiloint2double(__builtin_amdgcn_ds_swizzle(__double2hiint(v), 0x401f),
                          __builtin_amdgcn_ds_swizzle(__double2loint(v), 0x401f));
}
__device__ inline double xor32_d(double v) {
  const int a = ((threadIdx.x & 63) ^ 32) << 2;
  return __hiloint2double(__builtin_amdgcn_ds_bpermute(a, __double2hiint(v)),
                          __builtin_amdgcn_ds_bpermute(a, __double2loint(v)));
}
// Reduce-scatter of six wavefront sums: the sum over all 64 lanes of v[k]
// ends in lanes 2k and 2k + 1 (k < 6).  Each level pairs lanes that differ
// in one bit of their index within the row (row_mirror, row_half_mirror,
// quad_perm 3210, quad_perm 1032); the lane keeps the half of its current
// values that its bit selects and adds the partner's copy of that half, so
// the work halves at every level.  Rows are then combined through lanes
// l ^ 16 and l ^ 32.  Fixed order, all 64 lanes active.
__device__ inline double wave_sum6_scatter(const double* v) {
  const int i = threadIdx.x & 15;
  const bool b3 = (i & 8) != 0, b2 = (i & 4) != 0, b1 = (i & 2) != 0;
  // slots 0..7 (6, 7 are zero): keep 0..3 (b3 = 0) or 4..7 (b3 = 1)
  const double s0 = b3 ? v[0] : v[4], s1 = b3 ? v[1] : v[5];
  const double s2 = b3 ? v[2] : 0.0, s3 = b3 ? v[3] : 0.0;
  double k0 = b3 ? v[4] : v[0], k1 = b3 ? v[5] : v[1];
  double k2 = b3 ? 0.0 : v[2], k3 = b3 ? 0.0 : v[3];
  k0 += dpp_d<0x140>(s0);
  k1 += dpp_d<0x140>(s1);
  k2 += dpp_d<0x140>(s2);
  k3 += dpp_d<0x140>(s3);
  // keep local 0, 1 (b2 = 0) or 2, 3 (b2 = 1)
  const double t0 = b2 ? k0 : k2, t1 = b2 ? k1 : k3;
  double m0 = b2 ? k2 : k0, m1 = b2 ? k3 : k1;
  m0 += dpp_d<0x141>(t0);
  m1 += dpp_d<0x141>(t1);
  // keep local 0 (b1 = 0) or 1 (b1 = 1)
  const double t = b1 ? m0 : m1;
  double n = b1 ? m1 : m0;
  n += dpp_d<0x1b>(t);
  n += dpp_d<0xb1>(n);
  n += xor16_d(n);
  n += xor32_d(n);
  return n;
}

// As wave_sum6_scatter for FP32 inputs: the first level (pairs of lanes)
// adds in FP32, one rounding of a two-lane sum, and the rest in FP64.
template <int CTRL>
__device__ inline float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
__device__ inline double wave_sum6_scatter_f(const float* v) {
  const int i = threadIdx.x & 15;
  const bool b3 = (i & 8) != 0, b2 = (i & 4) != 0, b1 = (i & 2) != 0;
  const float s0 = b3 ? v[0] : v[4], s1 = b3 ? v[1] : v[5];
  const float s2 = b3 ? v[2] : 0.0f, s3 = b3 ? v[3] : 0.0f;
  float k0 = b3 ? v[4] : v[0], k1 = b3 ? v[5] : v[1];
  float k2 = b3 ? 0.0f : v[2], k3 = b3 ? 0.0f : v[3];
  k0 += dpp_f<0x140>(s0);
  k1 += dpp_f<0x140>(s1);
  k2 += dpp_f<0x140>(s2);
  k3 += dpp_f<0x140>(s3);
  const double K0 = k0, K1 = k1, K2 = k2, K3 = k3;
  const double t0 = b2 ? K0 : K2, t1 = b2 ? K1 : K3;
  double m0 = b2 ? K2 : K0, m1 = b2 ? K3 : K1;
  m0 += dpp_d<0x141>(t0);
  m1 += dpp_d<0x141>(t1);
  const double t = b1 ? m0 : m1;
  double n = b1 ? m1 : m0;
  n += dpp_d<0x1b>(t);
  n += dpp_d<0xb1>(n);
  n += xor16_d(n);
  n += xor32_d(n);
  return n;
}

// As wave_sum6_scatter_f with the first three levels (sums of eight lanes)
// in FP32 and the last three in FP64: for per-node contributions that carry
// FP32 rounding already, at about half the instructions of FP64 levels.
__device__ inline double wave_sum6_scatter_f3(const float* v) {
  const int i = threadIdx.x & 15;
  const bool b3 = (i & 8) != 0, b2 = (i & 4) != 0, b1 = (i & 2) != 0;
  const float s0 = b3 ? v[0] : v[4], s1 = b3 ? v[1] : v[5];
  const float s2 = b3 ? v[2] : 0.0f, s3 = b3 ? v[3] : 0.0f;
  float k0 = b3 ? v[4] : v[0], k1 = b3 ? v[5] : v[1];
  float k2 = b3 ? 0.0f : v[2], k3 = b3 ? 0.0f : v[3];
  k0 += dpp_f<0x140>(s0);
  k1 += dpp_f<0x140>(s1);
  k2 += dpp_f<0x140>(s2);
  k3 += dpp_f<0x140>(s3);
  const float t0 = b2 ? k0 : k2, t1 = b2 ? k1 : k3;
  float m0 = b2 ? k2 : k0, m1 = b2 ? k3 : k1;
  m0 += dpp_f<0x141>(t0);
  m1 += dpp_f<0x141>(t1);
  const float t = b1 ? m0 : m1;
  float nf = b1 ? m1 : m0;
  nf += dpp_f<0x1b>(t);
  double n = nf;
  n += dpp_d<0xb1>(n);
  n += xor16_d(n);
  n += xor32_d(n);
  return n;
}

__device__ inline double wave_min(double v) {
  v = fmin(v, ror_d<8>(v));
  v = fmin(v, ror_d<4>(v));
  v = fmin(v, ror_d<2>(v));
  v = fmin(v, ror_d<1>(v));
  return fmin(fmin(lane_d(v, 0), lane_d(v, 16)), fmin(lane_d(v, 32), lane_d(v, 48)));
}
__device__ inline double wave_max(double v) {
  v = fmax(v, ror_d<8>(v));
  v = fmax(v, ror_d<4>(v));
  v = fmax(v, ror_d<2>(v));
  v = fmax(v, ror_d<1>(v));
  return fmax(fmax(lane_d(v, 0), lane_d(v, 16)), fmax(lane_d(v, 32), lane_d(v, 48)));
}
__device__ inline int wave_sum_i(int v) {
  v += ror_i<8>(v);
  v += ror_i<4>(v);
  v += ror_i<2>(v);
  v += ror_i<1>(v);
  return (__builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16)) +
         (__builtin_amdgcn_readlane(v, 32) + __builtin_amdgcn_readlane(v, 48));
}
__device__ inline int wave_min_i(int v) {
  v = min(v, ror_i<8>(v));
  v = min(v, ror_i<4>(v));
  v = min(v, ror_i<2>(v));
  v = min(v, ror_i<1>(v));
  return min(min(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
             min(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}
__device__ inline int wave_max_i(int v) {
  v = max(v, ror_i<8>(v));
  v = max(v, ror_i<4>(v));
  v = max(v, ror_i<2>(v));
  v = max(v, ror_i<1>(v));
  return max(max(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
             max(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}
__device__ inline uint64_t wave_or_u64(uint64_t v) {
  int lo = (int)(uint32_t)v, hi = (int)(uint32_t)(v >> 32);
  lo |= ror_i<8>(lo); hi |= ror_i<8>(hi);
  lo |= ror_i<4>(lo); hi |= ror_i<4>(hi);
  lo |= ror_i<2>(lo); hi |= ror_i<2>(hi);
  lo |= ror_i<1>(lo); hi |= ror_i<1>(hi);
  uint32_t l = 0, h = 0;
  for (int r = 0; r < 64; r += 16) {
    l |= (uint32_t)__builtin_amdgcn_readlane(lo, r);
    h |= (uint32_t)__builtin_amdgcn_readlane(hi, r);
  }
  return ((uint64_t)h << 32) | l;
}

__device__ inline void atomic_add_f64(double* p, double v) {
  unsafeAtomicAdd(p, v);
}

// Hash of a pair key (a << 32 | b + 2) for the open-addressing pair table.
__host__ __device__ inline uint32_t pair_hash(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return (uint32_t)k;
}
__host__ __device__ inline uint64_t pair_key(int a, int b) {
  return ((uint64_t)(uint32_t)a << 32) | (uint64_t)(uint32_t)(b + 2);
}

}  // namespace hlbm
