// Particle motion (eqs. (2)-(3)) and tile binning for the node kernels.
//
// One wavefront per particle:
//  1. (moving steps) gather the hydrodynamic force and torque of the last
//     lattice pass: the sum of this particle's per-tile partial sums, in the
//     fixed order of its tile enumeration (deterministic, no atomics);
//  2. every lane evaluates the same FP64 Newton-Euler update (the result is
//     wave-uniform) and lane 0 stores it;
//  3. the lanes enumerate the tiles the particle's reach box touches and
//     append (particle id, enumeration index) to each tile's candidate list.
#include "context.h"

namespace hlbm {

namespace {

// The FP64 value of lane j (j uniform over the wavefront).
__device__ inline double readlane_f64(double v, int j) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), j);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), j);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// A set of at most two disjoint tile intervals on one axis.
struct TileSpan {
  int lo[2], hi[2], n;
  __device__ int count() const {
    return (n > 0 ? hi[0] - lo[0] + 1 : 0) + (n > 1 ? hi[1] - lo[1] + 1 : 0);
  }
  __device__ int at(int i) const {
    const int len0 = hi[0] - lo[0] + 1;
    return i < len0 ? lo[0] + i : lo[1] + (i - len0);
  }
};

__device__ inline int wrapi(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

// Tiles (of ts nodes) touched by the node interval [floor(c-e), ceil(c+e)]
// on an axis of n nodes and nt tiles; periodic axes wrap, bounded axes clip.
__device__ TileSpan axis_tiles(double c, double e, int n, int nt, int ts,
                               bool periodic) {
  TileSpan s;
  s.n = 0;
  int lo = (int)floor(c - e), hi = (int)ceil(c + e);
  if (periodic) {
    if (hi - lo + 1 >= n) {
      s.lo[0] = 0; s.hi[0] = nt - 1; s.n = 1;
      return s;
    }
    const int a = wrapi(lo, n), b = wrapi(hi, n);
    if (a <= b) {
      s.lo[0] = a / ts; s.hi[0] = b / ts; s.n = 1;
    } else {
      const int t0 = a / ts, t1 = b / ts;
      if (t1 >= t0) {
        s.lo[0] = 0; s.hi[0] = nt - 1; s.n = 1;
      } else {
        s.lo[0] = 0; s.hi[0] = t1;
        s.lo[1] = t0; s.hi[1] = nt - 1; s.n = 2;
      }
    }
    return s;
  }
  if (lo < 0) lo = 0;
  if (hi > n - 1) hi = n - 1;
  if (lo > hi) return s;
  s.lo[0] = lo / ts; s.hi[0] = hi / ts; s.n = 1;
  return s;
}

constexpr int UB = 4;   // binning: tiles per lane and round

__global__ __launch_bounds__(64) void k_particles(Particles P, Geom g, Phys ph,
                                                  double* __restrict__ Fh,
                                                  double* __restrict__ Th,
                                                  double* __restrict__ Fc,
                                                  double* __restrict__ Tc,
                                                  int move, Tiles tl, Counters* ctr,
                                                  PairTable keep_from, PairTable keep_to) {
  const int ip = blockIdx.x;
  if (ip >= P.n) {
    // blocks past the particles: the contact carry-over of the pair table,
    // one slot per thread (independent of this kernel's particle work; the
    // detection that follows inserts into the same next table)
    const long long s = (long long)(ip - P.n) * WAVE + threadIdx.x;
    if (s < keep_from.cap) keep_slot(keep_from, keep_to, s, ctr);
    return;
  }
  const int lane = threadIdx.x;
  const bool perz = g.periodic_z != 0;
  const double L[3] = {(double)g.nx, (double)g.ny, (double)g.nz};
  const bool per[3] = {true, true, perz};

  double X[3], U[3], W[3], q[4], R[9];
  for (int k = 0; k < 3; ++k) {
    X[k] = P.X[3 * ip + k];
    U[k] = P.U[3 * ip + k];
    W[k] = P.W[3 * ip + k];
  }
  for (int k = 0; k < 4; ++k) q[k] = P.q[4 * ip + k];

  if (move) {
    // 1. F_p = sum of the per-tile partials (eqs. (17)-(18)); later
    // sub-steps of the step keep the force of the first
    double F[3], T[3];
    if (move == 1) {
      const int ne = tl.nent[ip];
      double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      for (int k = lane; k < ne; k += WAVE) {
        const double* pp = tl.part + ((size_t)ip * g.maxent + k) * 6;
        for (int m = 0; m < 6; ++m) v[m] += pp[m];
      }
      for (int m = 0; m < 3; ++m) {
        F[m] = wave_sum(v[m]) + tl.ovf[6 * ip + m];
        T[m] = wave_sum(v[3 + m]) + tl.ovf[6 * ip + 3 + m];
      }
    } else {
      for (int m = 0; m < 3; ++m) {
        F[m] = Fh[3 * ip + m];
        T[m] = Th[3 * ip + m];
      }
    }
    // contact force and torque: the particle's slots summed in the order
    // of the partner id (lane k holds slot k; partners are distinct)
    double Fcp[3] = {0.0, 0.0, 0.0}, Tcp[3] = {0.0, 0.0, 0.0};
    {
      int nc = tl.ccount[ip];
      nc = nc < MAXC ? nc : MAXC;
      const size_t e0 = (size_t)ip * MAXC;
      // every slot's values are loaded at once (lane k: slot k) and then
      // read from registers in rank order
      const int key = lane < nc ? tl.ckey[e0 + lane] : 0x7fffffff;
      double cv[6];
      for (int m = 0; m < 6; ++m) cv[m] = lane < nc ? tl.cval[6 * (e0 + lane) + m] : 0.0;
      int rank = 0;
      for (int j = 0; j < nc; ++j) rank += __builtin_amdgcn_readlane(key, j) < key ? 1 : 0;
      for (int r = 0; r < nc; ++r) {
        const int j = __ffsll((long long)__ballot(lane < nc && rank == r)) - 1;
        for (int m = 0; m < 3; ++m) {
          Fcp[m] += readlane_f64(cv[m], j);
          Tcp[m] += readlane_f64(cv[3 + m], j);
        }
      }
    }
    // 2. Newton-Euler, symplectic Euler over the sub-step dt (eqs. (2)-(3));
    // gravity minus buoyancy (rho_p - rho_f) V g with rho_f = 1 (Sec. 5.1).
    const double V = P.vol[ip], m = P.mass[ip], I = P.inert[ip];
    const double s = P.dens[ip];
    const double dt = ph.dt_sub;
    double Tt[3];
    for (int k = 0; k < 3; ++k) {
      const double Fg = (s - 1.0) * V * ph.gravity[k];
      const double Ft = F[k] + Fcp[k] + Fg;
      Tt[k] = T[k] + Tcp[k];
      U[k] += Ft / m * dt;
      X[k] += U[k] * dt;
      if (per[k]) {
        if (X[k] >= L[k]) X[k] -= L[k];
        else if (X[k] < 0.0) X[k] += L[k];
      }
    }
    if (P.shape[ip] >= POLY0) {
      // eq. (3) with the world-frame tensor at the current orientation:
      // w += R I_b^-1 R^T T dt
      double Rc[9], tb[3], wb[3];
      quat_to_rot(q, Rc);
      const double* Ii = P.Iinv + 9 * ip;
      for (int k = 0; k < 3; ++k) tb[k] = (Rc[0 + k] * Tt[0] + Rc[3 + k] * Tt[1]) + Rc[6 + k] * Tt[2];
      for (int k = 0; k < 3; ++k) wb[k] = (Ii[3 * k] * tb[0] + Ii[3 * k + 1] * tb[1]) + Ii[3 * k + 2] * tb[2];
      for (int k = 0; k < 3; ++k)
        W[k] += ((Rc[3 * k] * wb[0] + Rc[3 * k + 1] * wb[1]) + Rc[3 * k + 2] * wb[2]) * dt;
    } else {
      for (int k = 0; k < 3; ++k) W[k] += Tt[k] / I * dt;
    }
    // orientation: exact rotation through |w| dt about w, q <- dq (x) q
    const double th = sqrt(W[0] * W[0] + W[1] * W[1] + W[2] * W[2]) * dt;
    if (th > 0.0) {
      const double c = cos(0.5 * th), sn = sin(0.5 * th) / th * dt;
      const double d0 = c, d1 = sn * W[0], d2 = sn * W[1], d3 = sn * W[2];
      double r[4];
      r[0] = d0 * q[0] - (d1 * q[1] + d2 * q[2] + d3 * q[3]);
      r[1] = d0 * q[1] + q[0] * d1 + (d2 * q[3] - d3 * q[2]);
      r[2] = d0 * q[2] + q[0] * d2 + (d3 * q[1] - d1 * q[3]);
      r[3] = d0 * q[3] + q[0] * d3 + (d1 * q[2] - d2 * q[1]);
      const double nn = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + r[3] * r[3]);
      for (int k = 0; k < 4; ++k) q[k] = r[k] / nn;
    }
    if (lane == 0) {
      for (int k = 0; k < 3; ++k) {
        Fh[3 * ip + k] = F[k];
        Th[3 * ip + k] = T[k];
        Fc[3 * ip + k] = Fcp[k];
        Tc[3 * ip + k] = Tcp[k];
      }
      if (move == 1)
        for (int k = 0; k < 6; ++k) tl.ovf[6 * ip + k] = 0.0;
    }
  }
  quat_to_rot(q, R);
  if (lane == 0) {
    for (int k = 0; k < 3; ++k) {
      P.X[3 * ip + k] = X[k];
      P.U[3 * ip + k] = U[k];
      P.W[3 * ip + k] = W[k];
    }
    for (int k = 0; k < 4; ++k) P.q[4 * ip + k] = q[k];
    for (int k = 0; k < 9; ++k) P.R[9 * ip + k] = R[k];
    float* rec = P.XR32 + SREC * ip;
    for (int k = 0; k < 3; ++k) rec[k] = (float)X[k];
    for (int k = 0; k < 9; ++k) rec[3 + k] = (float)R[k];
    // the detection screen's thresholds with this particle's FP32 error
    // bound: 1e-3 + 1e-5 (|r|_1 + size) at |r|_1 = sqrt 3 (R_c + 2), the
    // largest for a node within reach of either threshold (R_c the
    // circumradius)
    const int sh = P.shape[ip];
    const float fs = (float)P.size[ip];
    const float rc = sh >= POLY0 ? (float)P.poly[sh - POLY0].rc * fs
                                 : (sh == 1 ? 0.8660254f * fs : fs);
    const float tol = 1e-3f + 1e-5f * (1.7320508f * (rc + 2.0f) + fs);
    const float ot = (float)(0.5 * ph.eps), dt = (float)(DETECT + ph.delta_c);
    rec[12] = ot + tol;
    rec[13] = ot - tol;
    rec[14] = dt + tol;
    rec[15] = dt - tol;
    rec[16] = fmaxf(ot, dt) + tol;
    rec[17] = fs;
    rec[18] = __int_as_float(sh);
    rec[19] = fminf(ot, dt) - tol;   // below both (the ellipsoid screen's bound)
    // the lattice pass's kinematic record: centre split into an integer part
    // and its fraction (exact in FP64, the fraction then rounded to FP32)
    float* lr = P.LR32 + LREC * ip;
    for (int k = 0; k < 3; ++k) {
      const double fl = floor(X[k]);
      lr[k] = __int_as_float((int)fl);
      lr[3 + k] = (float)(X[k] - fl);
      lr[6 + k] = (float)U[k];
      lr[9 + k] = (float)W[k];
    }
    for (int k = 0; k < 9; ++k) lr[12 + k] = (float)R[k];
    lr[21] = fs;
    lr[22] = __int_as_float(sh);
    for (int k = 23; k < LREC; ++k) lr[k] = 0.0f;
  }

  // 3. Reach box: axis-aligned half extent of the body plus the largest
  // distance at which a node can be owned by it (eps/2) or flagged by the
  // rough detection (sqrt(0.75) + enlargement).
  const double margin = fmax(0.5 * ph.eps, DETECT + ph.delta_c) + 0.25;
  const int shape = P.shape[ip];
  const double size = P.size[ip];
  const int n3[3] = {g.nx, g.ny, g.nz};
  double ext[3];
  // lattice blocks list the particles owning a node within one node of the
  // block (the lattice pass pushes momentum-exchange terms to the owners of
  // each node's neighbours): half extent + eps/2 + 1 node
  const double margin_l = fmax(margin, 0.5 * ph.eps + 1.25);
  double extl[3];
  for (int k = 0; k < 3; ++k) {
    const double e = half_extent(shape, size, R, k, P.poly);
    ext[k] = e + margin;
    extl[k] = e + margin_l;
  }
  // detection tiles
  {
    const int nt3[3] = {g.dtx, g.dty, g.dtz};
    const int ts3[3] = {DX, DY, DZ};
    TileSpan sp[3];
    for (int k = 0; k < 3; ++k) sp[k] = axis_tiles(X[k], ext[k], n3[k], nt3[k], ts3[k], per[k]);
    const int cxn = sp[0].count(), cyn = sp[1].count(), czn = sp[2].count();
    const int total = cxn * cyn * czn;
    // A tile whose centre lies farther from the body than the widest test of
    // the node pass (ownership, eps/2, or detection, sqrt(0.75) + delta_c)
    // plus the tile's radius has no node inside either bound (signed
    // distances are 1-Lipschitz): skip it.
    const double reach = fmax(0.5 * ph.eps, DETECT + ph.delta_c) +
                         0.5 * sqrt((double)(DX - 1) * (DX - 1) + (DY - 1) * (DY - 1) +
                                    (DZ - 1) * (DZ - 1)) + 0.01;
    // UB tiles per lane and round, their slot atomics in flight together
    for (int t0 = lane; t0 < total; t0 += UB * WAVE) {
      long long tile[UB];
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        const int t = t0 + u * WAVE;
        tile[u] = -1;
        if (t >= total) continue;
        const int ix = t % cxn, iy = (t / cxn) % cyn, iz = t / (cxn * cyn);
        const int tx = sp[0].at(ix), ty = sp[1].at(iy), tz = sp[2].at(iz);
        const double rc[3] = {minimg(tx * DX + 0.5 * (DX - 1) - X[0], L[0], true),
                              minimg(ty * DY + 0.5 * (DY - 1) - X[1], L[1], true),
                              minimg(tz * DZ + 0.5 * (DZ - 1) - X[2], L[2], per[2])};
        if (shape >= POLY0) {
          // FP32 with its error bound (as in the detection's screening), the
          // plane lower bound ending the search beyond reach
          const float is = 1.0f / (float)size;
          float pb[3];
          for (int k = 0; k < 3; ++k)
            pb[k] = ((float)R[k] * (float)rc[0] + (float)R[3 + k] * (float)rc[1] +
                     (float)R[6 + k] * (float)rc[2]) * is;
          // (an ellipsoid type: the circumsphere lower bound |p| - rc)
          const CPoly* pt = (CPoly*)P.poly + (shape - POLY0);
          const float d =
              pt->kind == KIND_ELLIPSOID
                  ? (float)size * (sqrtf((pb[0] * pb[0] + pb[1] * pb[1]) + pb[2] * pb[2]) -
                                   (float)pt->rc)
                  : (float)size * poly_sdf<float>(P.poly, shape - POLY0, pb, nullptr,
                                                  (float)reach * is);
          const double tol = 1e-3 + 1e-5 * (fabs(rc[0]) + fabs(rc[1]) + fabs(rc[2]) + size);
          if ((double)d > reach + tol) continue;
        } else if (sdf(shape, size, R, rc[0], rc[1], rc[2], P.poly) > reach) {
          continue;
        }
        tile[u] = tx + (long long)g.dtx * (ty + (long long)g.dty * tz);
      }
      int slot[UB];
#pragma unroll
      for (int u = 0; u < UB; ++u) slot[u] = tile[u] >= 0 ? atomicAdd(&tl.dcount[tile[u]], 1) : 0;
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        if (tile[u] < 0) continue;
        if (slot[u] < g.tile_cap) tl.dlist[tile[u] * g.tile_cap + slot[u]] = ip;
        else atomicOr(&ctr->tile_overflow, 1);
      }
    }
  }
  // lattice blocks, with the particle's own enumeration index
  {
    const int nt3[3] = {g.ltx, g.lty, g.ltz};
    const int ts3[3] = {LX, LY, LZ};
    TileSpan sp[3];
    for (int k = 0; k < 3; ++k) sp[k] = axis_tiles(X[k], extl[k], n3[k], nt3[k], ts3[k], per[k]);
    const int cxn = sp[0].count(), cyn = sp[1].count(), czn = sp[2].count();
    int total = cxn * cyn * czn;
    if (total > g.maxent) {
      if (lane == 0) atomicOr(&ctr->tile_overflow, 1);
      total = g.maxent;
    }
    if (lane == 0) tl.nent[ip] = total;
    for (int t0 = lane; t0 < total; t0 += UB * WAVE) {
      long long tile[UB];
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        const int t = t0 + u * WAVE;
        tile[u] = -1;
        if (t >= total) continue;
        const int ix = t % cxn, iy = (t / cxn) % cyn, iz = t / (cxn * cyn);
        tile[u] = sp[0].at(ix) + (long long)g.ltx * (sp[1].at(iy) + (long long)g.lty * sp[2].at(iz));
      }
      int slot[UB];
#pragma unroll
      for (int u = 0; u < UB; ++u) slot[u] = tile[u] >= 0 ? atomicAdd(&tl.lcount[tile[u]], 1) : 0;
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        if (tile[u] < 0) continue;
        const int t = t0 + u * WAVE;
        if (slot[u] < g.tile_cap) {
          tl.llist[tile[u] * g.tile_cap + slot[u]] = ip;
          tl.lent[tile[u] * g.tile_cap + slot[u]] = t;
        } else {
          atomicOr(&ctr->tile_overflow, 1);
          double* pp = tl.part + ((size_t)ip * g.maxent + t) * 6;
          for (int m = 0; m < 6; ++m) pp[m] = 0.0;
        }
      }
    }
  }
}

}  // namespace

hipError_t launch_particles(Ctx& c, int move, const PairTable* keep_from,
                            const PairTable* keep_to) {
  PairTable none = {nullptr, nullptr, 0, nullptr, nullptr};
  const PairTable from = keep_from ? *keep_from : none;
  const PairTable to = keep_to ? *keep_to : none;
  const unsigned kb = (unsigned)((from.cap + WAVE - 1) / WAVE);
  if (c.np + kb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_particles, dim3(c.np + kb), dim3(64), 0, c.stream, c.part,
                     c.g, c.ph, c.Fh, c.Th, c.Fc, c.Tc, move, c.tl, c.counters, from, to);
  return hipGetLastError();
}

}  // namespace hlbm
