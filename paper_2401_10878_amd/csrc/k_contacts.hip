// Discrete contact treatment (Sec. 3.3.1, eqs. (4)-(9)) and the per-step
// bookkeeping of the pair tables.
//
// One wavefront treats one contact record (the wavefronts of a fixed grid
// take the table's occupied slots from its list in a stride):
//   box      the carried (corrected) box of an established contact, or the
//            rough box [min - 1/2, max + 1/2] of the flagged node images;
//            kept in the frame of the lower-id particle a (Sec. 3.3.2)
//   correct  faces -x,+x,-y,+y,-z,+z in turn; N_c x N_c midpoint samples of
//            phi = max(d'_a, d'_b) on the face (one per lane); the face
//            moves inwards by the wave minimum of phi
//   integrate N_c^3 midpoint samples of the box; inside = both enlarged
//            distances negative; wave sums of count, position and gradient
//            difference, wave maximum of -(d'_a + d'_b)
//   force    normal force (4, 5, 6) and friction (7-9) at the centroid,
//            appended to both particles' contact slots; k_particles sums a
//            particle's slots in the order of the partner id, so the
//            result does not depend on the order the pairs ran in.
#include <float.h>

#include "context.h"

namespace hlbm {

namespace {

__device__ inline void clear_slot(const PairTable& t, long long i) {
  t.keys[i] = EMPTY_KEY;
  PairRec r = {};
  for (int k = 0; k < 3; ++k) {
    r.rlo[k] = 0x7fffffff;
    r.rhi[k] = (int)0x80000000;
  }
  t.rec[i] = r;
}

// Tile counts (CLEAR_TILES) and, once after allocation, every slot of a
// table (CLEAR_ALL_SLOTS), over a grid.
__global__ void k_clear_step(PairTable next, int* dcount, long long ndt, int* lcount,
                             long long nlt, int what) {
  const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  if (what & CLEAR_TILES) {
    for (long long i = tid; i < ndt; i += stride) dcount[i] = 0;
    for (long long i = tid; i < nlt; i += stride) lcount[i] = 0;
  }
  if (what & CLEAR_ALL_SLOTS)
    for (long long i = tid; i < next.cap; i += stride) clear_slot(next, i);
}

// The next step's contact state (CLEAR_CONTACT), one workgroup: the slots
// the table's list names, the contact forces and slots, and the detection
// counters; the list count is reset after the workgroup barrier, when
// every thread has read it.
constexpr int CLEAR_THREADS = 1024;
__global__ __launch_bounds__(CLEAR_THREADS) void k_clear_contact(PairTable next, double* Fc,
                                                                 double* Tc, int np,
                                                                 int* ccount, Counters* ctr) {
  const int tid = (int)threadIdx.x;
  const int nl = *next.nlist;
  for (int i = tid; i < nl; i += CLEAR_THREADS) clear_slot(next, next.list[i]);
  for (long long i = tid; i < 3LL * np; i += CLEAR_THREADS) {
    Fc[i] = 0.0;
    Tc[i] = 0.0;
  }
  for (int i = tid; i < np; i += CLEAR_THREADS) ccount[i] = 0;
  if (tid == 0) {
    ctr->det_pairs = 0;
    ctr->det_cells = 0;
    ctr->samples = 0;
  }
  __syncthreads();
  if (tid == 0) *next.nlist = 0;
}

__global__ void k_keep(PairTable from, PairTable to, Counters* ctr) {
  const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= from.cap) return;
  keep_slot(from, to, s, ctr);
}

struct Body {
  int shape;
  double size, X[3], R[9];
  const PolyDev* poly;
};

// With a gradient, a point farther outside a polyhedron than far may return
// a lower bound of the distance (far = delta: only points inside the
// enlarged body need the exact value and gradient).
template <bool ELL>
__device__ inline double body_sdf(const Body& b, const double* y, double* g,
                                  double far = 1e300) {
  const double r[3] = {y[0] - b.X[0], y[1] - b.X[1], y[2] - b.X[2]};
  if (g) return sdf_grad_exact<ELL>(b.shape, b.size, b.R, r, g, b.poly, far);
  return sdf_exact<ELL>(b.shape, b.size, b.R, r[0], r[1], r[2], b.poly);
}

// enlarged distance of member b (particle, or wall -1 bottom / -2 top)
template <bool ELL>
__device__ inline double member_sdf(const Body& b, int bid, double delta,
                                    double nz, const double* y, double* g,
                                    double far = 1e300) {
  if (bid >= 0) return body_sdf<ELL>(b, y, g, far) - delta;
  if (bid == -1) {
    if (g) { g[0] = 0.0; g[1] = 0.0; g[2] = 1.0; }
    return y[2] + 0.5;
  }
  if (g) { g[0] = 0.0; g[1] = 0.0; g[2] = -1.0; }
  return (nz - 0.5) - y[2];
}

__device__ inline void cross3(const double* a, const double* b, double* o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

// Append (force, torque) on particle p from its partner `other` to p's slots.
__device__ void add_contact(Tiles tl, Counters* ctr, int p, int other,
                            const double* F, const double* T) {
  const int k = atomicAdd(&tl.ccount[p], 1);
  if (k >= MAXC) {
    atomicOr(&ctr->contact_overflow, 1);
    return;
  }
  const size_t e = (size_t)p * MAXC + k;
  tl.ckey[e] = other;
  for (int m = 0; m < 3; ++m) {
    tl.cval[6 * e + m] = F[m];
    tl.cval[6 * e + 3 + m] = T[m];
  }
}

template <bool POLY, bool ELL>
__device__ void treat_slot(const PairTable& t, const Particles& P, const Geom& g,
                           const Phys& ph, const Tiles& tl, Counters* ctr, int slot) {
  const int lane = threadIdx.x % WAVE;
  PairRec* rec = &t.rec[slot];
  const int a = __builtin_amdgcn_readfirstlane(rec->a);
  const int b = __builtin_amdgcn_readfirstlane(rec->b);
  const bool perz = g.periodic_z != 0;
  const double L[3] = {(double)g.nx, (double)g.ny, (double)g.nz};
  const bool per[3] = {true, true, perz};
  const int nc = ph.n_c;
  const double delta = ph.delta_c;

  Body A, Bb;
  A.poly = Bb.poly = POLY ? P.poly : nullptr;
  A.shape = P.shape[a];
  A.size = P.size[a];
  for (int k = 0; k < 3; ++k) A.X[k] = P.X[3 * a + k];
  for (int k = 0; k < 9; ++k) A.R[k] = P.R[9 * a + k];
  Bb.shape = 0;
  Bb.size = 0.0;
  for (int k = 0; k < 3; ++k) Bb.X[k] = 0.0;
  for (int k = 0; k < 9; ++k) Bb.R[k] = 0.0;
  if (b >= 0) {
    Bb.shape = P.shape[b];
    Bb.size = P.size[b];
    // the higher-id particle is moved next to the lower-id one
    for (int k = 0; k < 3; ++k)
      Bb.X[k] = A.X[k] + minimg(P.X[3 * b + k] - A.X[k], L[k], per[k]);
    for (int k = 0; k < 9; ++k) Bb.R[k] = P.R[9 * b + k];
  }

  double lo[3], hi[3];
  const bool carried = rec->carried != 0;
  // a new particle-wall pair: the flagged nodes lie on the fluid side of
  // the wall plane and the overlap beyond it, so the wall-side face starts
  // at the far side of the enlarged body (half extent along z plus the
  // enlargement) and the correction moves it onto the body
  double wall_lo = 1e300, wall_hi = -1e300;
  if (!carried && b < 0) {
    const double ez = half_extent(A.shape, A.size, A.R, 2, A.poly) + delta;
    if (b == -1) wall_lo = A.X[2] - ez;
    else wall_hi = A.X[2] + ez;
  }
  for (int k = 0; k < 3; ++k) {
    lo[k] = carried ? rec->lo[k] : (double)rec->rlo[k] - 0.5;
    hi[k] = carried ? rec->hi[k] : (double)rec->rhi[k] + 0.5;
    if (k == 2) {
      lo[k] = fmin(lo[k], wall_lo);
      hi[k] = fmax(hi[k], wall_hi);
    }
    const double mid = 0.5 * (lo[k] + hi[k]);
    const int sh = image_shift(mid - A.X[k], L[k], per[k]);
    lo[k] += (double)(sh * (int)L[k]);
    hi[k] += (double)(sh * (int)L[k]);
  }

  // ---- box correction, one pass -----------------------------------------
  bool ok = true;
  int nfaces = 0;   // faces sampled (the box can empty on the way)
  // fully unrolled, so that the face's axis k (and u, v) index registers
#pragma unroll
  for (int face = 0; face < 6; ++face) {
    for (int k = 0; k < 3; ++k)
      if (!(hi[k] > lo[k])) ok = false;
    if (!ok) continue;
    ++nfaces;
    const int k = face / 2, plus = face % 2;
    const int u = k == 0 ? 1 : 0, v = k == 2 ? 1 : 2;
    const double hu = (hi[u] - lo[u]) / (double)nc;
    const double hv = (hi[v] - lo[v]) / (double)nc;
    double smin = DBL_MAX;
    for (int idx = lane; idx < nc * nc; idx += WAVE) {
      const int j = idx / nc, l = idx % nc;
      double y[3];
      y[k] = plus ? hi[k] : lo[k];
      y[u] = lo[u] + ((double)j + 0.5) * hu;
      y[v] = lo[v] + ((double)l + 0.5) * hv;
      const double da = body_sdf<ELL>(A, y, nullptr) - delta;
      const double db = member_sdf<ELL>(Bb, b, delta, L[2], y, nullptr);
      smin = fmin(smin, fmax(da, db));
    }
    smin = wave_min(smin);
    if (plus) hi[k] = hi[k] - smin;
    else lo[k] = lo[k] + smin;
  }
  if (ok)
    for (int k = 0; k < 3; ++k)
      if (!(hi[k] > lo[k])) ok = false;

  // ---- overlap integration ------------------------------------------------
  int n_in = 0;
  double sy[3] = {0.0, 0.0, 0.0}, gs[3] = {0.0, 0.0, 0.0};
  double dmax = -DBL_MAX;
  double h[3] = {0.0, 0.0, 0.0};
  if (ok) {
    for (int k = 0; k < 3; ++k) h[k] = (hi[k] - lo[k]) / (double)nc;
    const int ns = nc * nc * nc;
    for (int idx = lane; idx < ns; idx += WAVE) {
      const int j = idx % nc, kk = (idx / nc) % nc, l = idx / (nc * nc);
      double y[3], ga[3], gb[3];
      y[0] = lo[0] + ((double)j + 0.5) * h[0];
      y[1] = lo[1] + ((double)kk + 0.5) * h[1];
      y[2] = lo[2] + ((double)l + 0.5) * h[2];
      // a sample counts when inside both enlarged bodies: beyond delta
      // outside either, the lower bound decides
      const double da = body_sdf<ELL>(A, y, ga, delta) - delta;
      const double db = member_sdf<ELL>(Bb, b, delta, L[2], y, gb, delta);
      if (fmax(da, db) < 0.0) {
        n_in++;
        dmax = fmax(dmax, -(da + db));
        for (int m = 0; m < 3; ++m) {
          sy[m] += y[m];
          gs[m] += ga[m] - gb[m];
        }
      }
    }
    n_in = wave_sum_i(n_in);
    for (int m = 0; m < 3; ++m) {
      sy[m] = wave_sum(sy[m]);
      gs[m] = wave_sum(gs[m]);
    }
    dmax = wave_max(dmax);
  }
  // midpoint samples of this record (each evaluates both members)
  if (lane == 0)
    atomicAdd(&ctr->samples,
              (unsigned long long)(nfaces * nc * nc + (ok ? nc * nc * nc : 0)));
  if (!ok || n_in == 0) {
    if (lane == 0) {
      rec->keep = 0;
      rec->n_in = 0;
      rec->volume = 0.0;
    }
    return;
  }

  // ---- results and forces (wave-uniform values) ----------------------------
  const double V = (double)n_in * (h[0] * h[1] * h[2]);
  double xc[3], nrm[3] = {0.0, 0.0, 0.0};
  for (int m = 0; m < 3; ++m) xc[m] = sy[m] / (double)n_in;
  const double gn = sqrt(gs[0] * gs[0] + gs[1] * gs[1] + gs[2] * gs[2]);
  if (gn > 0.0) {
    for (int m = 0; m < 3; ++m) nrm[m] = gs[m] / gn;
  } else {
    double dv[3];
    if (b >= 0) {
      for (int m = 0; m < 3; ++m) dv[m] = Bb.X[m] - A.X[m];
    } else {
      dv[0] = 0.0; dv[1] = 0.0; dv[2] = b == -1 ? -1.0 : 1.0;
    }
    const double dn = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
    if (dn > 0.0)
      for (int m = 0; m < 3; ++m) nrm[m] = dv[m] / dn;
  }
  const double depth = dmax;

  double ra[3], t3[3], va[3], vb[3] = {0.0, 0.0, 0.0};
  for (int m = 0; m < 3; ++m) ra[m] = xc[m] - A.X[m];
  cross3(P.W + 3 * a, ra, t3);
  for (int m = 0; m < 3; ++m) va[m] = P.U[3 * a + m] + t3[m];
  double rb[3] = {0.0, 0.0, 0.0};
  if (b >= 0) {
    for (int m = 0; m < 3; ++m) rb[m] = xc[m] - Bb.X[m];
    cross3(P.W + 3 * b, rb, t3);
    for (int m = 0; m < 3; ++m) vb[m] = P.U[3 * b + m] + t3[m];
  }
  double v[3];
  for (int m = 0; m < 3; ++m) v[m] = va[m] - vb[m];
  const double dn = v[0] * nrm[0] + v[1] * nrm[1] + v[2] * nrm[2];
  int established = rec->established;
  double damping = rec->damping;
  if (!established) {
    const double e = ph.restitution;
    damping = dn > 0.0 ? 1.5 * (1.0 - e) * (11.0 - e) / ((1.0 + 9.0 * e) * dn) : 0.0;
    established = 1;
  }
  double fn = 4.0 / (3.0 * PI) * ph.estar * sqrt(V * depth) * (1.0 + damping * dn);
  if (fn < 0.0) fn = 0.0;
  double vt[3];
  for (int m = 0; m < 3; ++m) vt[m] = v[m] - dn * nrm[m];
  const double vtn = sqrt(vt[0] * vt[0] + vt[1] * vt[1] + vt[2] * vt[2]);
  double ft[3] = {0.0, 0.0, 0.0};
  if (vtn > 0.0) {
    const double aa = vtn / ph.u_k;
    const double rr = ph.mu_k / ph.mu_s;
    const double mus = ph.mu_s * (1.0 - 0.09 * (rr * rr * rr * rr));
    const double a2 = aa * aa;
    const double mu = (2.0 * mus - ph.mu_k) * a2 / (a2 * a2 + 1.0) + ph.mu_k -
                      ph.mu_k / (a2 + 1.0);
    for (int m = 0; m < 3; ++m) ft[m] = -(vt[m] / vtn) * mu * fn;
  }
  double Fa[3], Fb[3], Ta[3], Tb[3];
  for (int m = 0; m < 3; ++m) {
    Fa[m] = -fn * nrm[m] + ft[m];
    Fb[m] = -Fa[m];
  }
  cross3(ra, Fa, Ta);
  if (b >= 0) cross3(rb, Fb, Tb);
  if (lane == 0) {
    add_contact(tl, ctr, a, b, Fa, Ta);
    if (b >= 0) add_contact(tl, ctr, b, a, Fb, Tb);
    rec->keep = 1;
    rec->carried = 1;
    rec->established = established;
    rec->damping = damping;
    rec->age = rec->age + 1;
    rec->n_in = n_in;
    rec->volume = V;
    rec->depth = depth;
    rec->fn = fn;
    for (int m = 0; m < 3; ++m) {
      rec->lo[m] = lo[m];
      rec->hi[m] = hi[m];
      rec->centroid[m] = xc[m];
      rec->normal[m] = nrm[m];
      rec->force_a[m] = Fa[m];
    }
  }
}


constexpr int TREAT_BLOCKS = 512;   // 2048 wavefronts
template <bool POLY, bool ELL = false>
__global__ __launch_bounds__(256) void k_treat(PairTable t, Particles P, Geom g,
                                               Phys ph, Tiles tl, Counters* ctr) {
  const int n = *t.nlist;
  const int stride = (int)gridDim.x * 4;
  for (int i = (int)blockIdx.x * 4 + (int)(threadIdx.x / WAVE); i < n; i += stride)
    treat_slot<POLY, ELL>(t, P, g, ph, tl, ctr, __builtin_amdgcn_readfirstlane(t.list[i]));
}

}  // namespace

hipError_t launch_clear_step(Ctx& c, PairTable next, int what, hipStream_t s) {
  const long long ndt = (long long)c.g.dtx * c.g.dty * c.g.dtz;
  const long long nlt = (long long)c.g.ltx * c.g.lty * c.g.ltz;
  if (what & (CLEAR_TILES | CLEAR_ALL_SLOTS)) {
    long long work = (what & CLEAR_ALL_SLOTS) ? next.cap : 0;
    if ((what & CLEAR_TILES) && ndt > work) work = ndt;
    long long blocks = (work + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_clear_step, dim3((unsigned)blocks), dim3(256), 0, s, next,
                       c.tl.dcount, ndt, c.tl.lcount, nlt, what);
  }
  if (what & CLEAR_CONTACT)
    hipLaunchKernelGGL(k_clear_contact, dim3(1), dim3(CLEAR_THREADS), 0, s, next, c.Fc,
                       c.Tc, c.np, c.tl.ccount, c.counters);
  return hipGetLastError();
}

hipError_t launch_keep(Ctx& c, PairTable from, PairTable to) {
  hipLaunchKernelGGL(k_keep, dim3((unsigned)((from.cap + 255) / 256)), dim3(256),
                     0, c.stream, from, to, c.counters);
  return hipGetLastError();
}

hipError_t launch_treat(Ctx& c, PairTable t, hipStream_t s) {
  const unsigned nb = (unsigned)((t.cap + 3) / 4 < TREAT_BLOCKS ? (t.cap + 3) / 4 : TREAT_BLOCKS);
  if (c.has_ellipsoid)
    hipLaunchKernelGGL((k_treat<true, true>), dim3(nb), dim3(256), 0,
                     s, t, c.part, c.g, c.ph, c.tl, c.counters);
  else if (c.has_poly)
    hipLaunchKernelGGL(k_treat<true>, dim3(nb), dim3(256), 0,
                     s, t, c.part, c.g, c.ph, c.tl, c.counters);
  else
    hipLaunchKernelGGL(k_treat<false>, dim3(nb), dim3(256), 0,
                     s, t, c.part, c.g, c.ph, c.tl, c.counters);
  return hipGetLastError();
}

}  // namespace hlbm
