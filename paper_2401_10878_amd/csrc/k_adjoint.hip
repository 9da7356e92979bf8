// Discrete adjoint (reverse mode) of the coupled time step, FP64, fully
// periodic boxes.
//
// Forward step t, as the step kernels compute it (Sec. 4.4, Algorithm 1):
//   f_t      = stream(f*_{t-1})                           eq. (11)
//   F_h, T_h = momentum exchange over the nodes owned by each particle in
//              o_{t-1}, with f*_{t-1}, f_t and u_p at P_{t-1}   eqs. (16)-(18)
//   P_t      = move(P_{t-1}, F_h + F_c, s)                 eqs. (2)-(3)
//   o_t      = owner map at P_t                            (Sec. 3.2)
//   f*_t     = collide(f_t, B(d_{o_t}), u_p(P_t), a(s))    eqs. (10)-(15)
// The adjoint runs these in reverse with the owner maps o and the contact
// forces F_c, T_c of the recorded forward run held fixed (the discrete
// decisions of the forward pass are not differentiated).  Orientation
// adjoints are world-frame rotation vectors: a perturbation of R is
// exp([dtheta]x) R.
//
// Kernels of one reverse step (state adjoints gbar = dJ/df*_t, Pbar):
//   k_adj_collide  per node: hbar = dJ/df_t from gbar, plus the coupling
//                  terms (B, u_p) into the particle adjoints of P_t and the
//                  fluid acceleration adjoint
//   k_adj_move     per particle: Pbar_t -> Pbar_{t-1}, dJ/dF_h, dJ/dT_h, dJ/ds
//   k_adj_mea      per node owned in o_{t-1}: the post-stream terms of the
//                  momentum exchange into hbar, and its u_p and r terms into
//                  Pbar_{t-1}
//   k_adj_stream   per node: gbar_{t-1} = push of hbar plus the own terms of
//                  the momentum exchange
#include "context.h"

namespace hlbm {

namespace {

// Particle adjoint slots: X (0-2), theta (3-5), U (6-8), omega (9-11).
constexpr int PB = 12;

__device__ inline void node_xyz(long long id, const Geom& g, int& x, int& y, int& z) {
  x = (int)(id % g.nx);
  y = (int)((id / g.nx) % g.ny);
  z = (int)(id / ((long long)g.nx * g.ny));
}
__device__ inline long long wrap_id(int x, int y, int z, const Geom& g) {
  x = x < 0 ? x + g.nx : (x >= g.nx ? x - g.nx : x);
  y = y < 0 ? y + g.ny : (y >= g.ny ? y - g.ny : y);
  z = z < 0 ? z + g.nz : (z >= g.nz ? z - g.nz : z);
  return (long long)x + (long long)g.nx * ((long long)y + (long long)g.ny * z);
}

// Wavefront aggregation of per-lane particle adjoint increments v[PB] keyed
// by particle id q (-1 = none), one FP64 atomic per value and distinct id.
__device__ void commit_adjoint(int q, const double* v, double* dst) {
  const int lane = threadIdx.x % WAVE;
  bool pend = q >= 0;
  for (;;) {
    const uint64_t m = __ballot(pend);
    if (m == 0) break;
    const int pick = __builtin_amdgcn_readlane(q, __ffsll((long long)m) - 1);
    const bool take = pend && q == pick;
    for (int k = 0; k < PB; ++k) {
      const double s = wave_sum(take ? v[k] : 0.0);
      if (lane == 0) atomic_add_f64(&dst[PB * pick + k], s);
    }
    if (take) pend = false;
  }
}

// Record layout of one particle state: X 3, q 4, U 3, W 3, R 9.
constexpr int PREC_N = 22;
__device__ inline const double* rec_X(const double* r) { return r; }
__device__ inline const double* rec_U(const double* r) { return r + 7; }
__device__ inline const double* rec_W(const double* r) { return r + 10; }
__device__ inline const double* rec_R(const double* r) { return r + 13; }

__device__ inline void cross(const double* a, const double* b, double* o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

__device__ inline void lever(const Geom& g, int x, int y, int z, const double* X, double* r) {
  r[0] = minimg((double)x - X[0], (double)g.nx, true);
  r[1] = minimg((double)y - X[1], (double)g.ny, true);
  r[2] = minimg((double)z - X[2], (double)g.nz, true);
}

// dJ/df_t at each node from dJ/df*_t (collision, eqs. (10), (12)-(15)) and
// the coupling terms of B(d) and u_p into the adjoints of P_t.
//   f* = (1 - w) f + (w - 1) feq(rho, u) + feq(rho, v),  v = u + B (u_p - u) + a
__global__ __launch_bounds__(256) void k_adj_collide(
    const double* __restrict__ gbar, const double* __restrict__ fprev,
    double* __restrict__ hbar, const int* __restrict__ owner,
    const double* __restrict__ prec, Particles P, Geom g, Phys ph,
    double* __restrict__ pbar, double* __restrict__ abar_part) {
  __shared__ double ared[4][3];
  const long long n = g.ncell;
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = id < n;
  double a_loc[3] = {0.0, 0.0, 0.0};
  double inc[PB];
  for (int k = 0; k < PB; ++k) inc[k] = 0.0;
  int o = -1;
  if (valid) {
    int x, y, z;
    node_xyz(id, g, x, y, z);
    double f[Q], gb[Q];
    double rho = 0.0, J[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      f[i] = fprev[(long long)i * n + wrap_id(x - cx(i), y - cy(i), z - cz(i), g)];
      gb[i] = gbar[(long long)i * n + id];
      rho += f[i];
      J[0] += cx(i) * f[i];
      J[1] += cy(i) * f[i];
      J[2] += cz(i) * f[i];
    }
    const double u[3] = {J[0] / rho, J[1] / rho, J[2] / rho};
    o = owner_id(owner[id]);
    double B = 0.0, Bp = 0.0, up[3] = {0.0, 0.0, 0.0}, r[3] = {0.0, 0.0, 0.0};
    double nrm[3] = {0.0, 0.0, 0.0};
    const double* pr = nullptr;
    if (o >= 0) {
      pr = prec + (size_t)PREC_N * o;
      lever(g, x, y, z, rec_X(pr), r);
      const double d = sdf_grad(P.shape[o], P.size[o], rec_R(pr), r, nrm, nullptr);
      B = weight(d, ph.eps);
      if (d > -0.5 * ph.eps && d < 0.5 * ph.eps)
        Bp = -(PI / (2.0 * ph.eps)) * sin(PI * (d + 0.5 * ph.eps) / ph.eps);
      double wr[3];
      cross(rec_W(pr), r, wr);
      for (int k = 0; k < 3; ++k) up[k] = rec_U(pr)[k] + wr[k];
    }
    double v[3];
    for (int k = 0; k < 3; ++k) v[k] = u[k] + B * (up[k] - u[k]) + ph.a_ext[k];
    // moments of gbar weighted by w_i: s0, s1 (vector), s2 (symmetric)
    double s0 = 0.0, s1[3] = {0.0, 0.0, 0.0};
    double s2[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const double gw = gb[i] * wgt(i);
      const int c[3] = {cx(i), cy(i), cz(i)};
      s0 += gw;
      for (int a = 0; a < 3; ++a) {
        s1[a] += c[a] * gw;
        for (int b = 0; b < 3; ++b) s2[a][b] += c[a] * c[b] * gw;
      }
    }
    // A(w) = d/drho of sum g feq(rho, w); G(w) = d/dw of the same
    auto A = [&](const double* w) {
      double ww = 0.0, s1w = 0.0, wsw = 0.0;
      for (int a = 0; a < 3; ++a) {
        ww += w[a] * w[a];
        s1w += s1[a] * w[a];
        for (int b = 0; b < 3; ++b) wsw += w[a] * s2[a][b] * w[b];
      }
      return s0 + 3.0 * s1w + 4.5 * wsw - 1.5 * ww * s0;
    };
    auto G = [&](const double* w, double* out) {
      for (int a = 0; a < 3; ++a) {
        double sw = 0.0;
        for (int b = 0; b < 3; ++b) sw += s2[a][b] * w[b];
        out[a] = rho * (3.0 * s1[a] + 9.0 * sw - 3.0 * w[a] * s0);
      }
    };
    const double om = ph.omega;
    const double rhob = (om - 1.0) * A(u) + A(v);
    double vb[3], gu[3];
    G(v, vb);
    G(u, gu);
    double ub[3];
    for (int k = 0; k < 3; ++k) ub[k] = (om - 1.0) * gu[k] + (1.0 - B) * vb[k];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const double cu = (cx(i) - u[0]) * ub[0] + (cy(i) - u[1]) * ub[1] + (cz(i) - u[2]) * ub[2];
      hbar[(long long)i * n + id] = (1.0 - om) * gb[i] + rhob + cu / rho;
    }
    for (int k = 0; k < 3; ++k) a_loc[k] = vb[k];
    if (o >= 0) {
      double Bb = 0.0, upb[3];
      for (int k = 0; k < 3; ++k) {
        Bb += vb[k] * (up[k] - u[k]);
        upb[k] = B * vb[k];
      }
      const double db = Bb * Bp;
      double nxr[3], upxw[3], rxup[3];
      cross(nrm, r, nxr);
      cross(upb, rec_W(pr), upxw);
      cross(r, upb, rxup);
      for (int k = 0; k < 3; ++k) {
        inc[k] = -db * nrm[k] - upxw[k];     // X
        inc[3 + k] = db * nxr[k];            // theta
        inc[6 + k] = upb[k];                 // U
        inc[9 + k] = rxup[k];                // omega
      }
    }
  }
  commit_adjoint(o, inc, pbar);
  // fluid acceleration adjoint: per-block partial, fixed order
  const int wave = threadIdx.x / WAVE;
  for (int k = 0; k < 3; ++k) {
    const double s = wave_sum(a_loc[k]);
    if (threadIdx.x % WAVE == 0) ared[wave][k] = s;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const int k = threadIdx.x;
    abar_part[3 * (long long)blockIdx.x + k] =
        ((ared[0][k] + ared[1][k]) + ared[2][k]) + ared[3][k];
  }
}

// Sum of the per-block acceleration adjoints (one block).
__global__ __launch_bounds__(256) void k_adj_reduce_a(const double* __restrict__ part,
                                                      long long nblocks,
                                                      double* __restrict__ abar) {
  __shared__ double red[4][3];
  double s[3] = {0.0, 0.0, 0.0};
  for (long long b = threadIdx.x; b < nblocks; b += blockDim.x)
    for (int k = 0; k < 3; ++k) s[k] += part[3 * b + k];
  const int wave = threadIdx.x / WAVE;
  for (int k = 0; k < 3; ++k) {
    const double t = wave_sum(s[k]);
    if (threadIdx.x % WAVE == 0) red[wave][k] = t;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const int k = threadIdx.x;
    abar[k] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
  }
}

// Particle motion in reverse (eqs. (2)-(3)), one thread per particle:
//   U_t = U + (F_h + F_c)/(s V) + (1 - 1/s) g,   X_t = X + U_t
//   w_t = w + (T_h + T_c)/(s I_1),               R_t = exp([w_t]x) R
// pbar holds Pbar_t (carried) + the increments of k_adj_collide; on return
// it holds Pbar_{t-1} before the momentum-exchange terms, and fhbar the
// adjoints of F_h and T_h (6 per particle).  The fluid acceleration of a
// balanced periodic box, a = -sum (s_p - 1) V_p g / N, adds its s terms.
__global__ void k_adj_move(Particles P, Phys ph, Geom g, int balance,
                           const double* __restrict__ prec_t,
                           const double* __restrict__ frc,
                           const double* __restrict__ abar,
                           double* __restrict__ pbar, double* __restrict__ fhbar,
                           double* __restrict__ sbar) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P.n) return;
  double* pb = pbar + PB * p;
  const double s = P.dens[p], V = P.vol[p];
  const double I1 = P.inert[p] / s;
  const double* f = frc + 12 * p;       // Fh 3, Th 3, Fc 3, Tc 3
  const double* W = rec_W(prec_t + (size_t)PREC_N * p);
  double Xb[3], thb[3], Ub[3], Wb[3];
  for (int k = 0; k < 3; ++k) {
    Xb[k] = pb[k];
    thb[k] = pb[3 + k];
    Ub[k] = pb[6 + k] + pb[k];          // X_t = X + U_t
    Wb[k] = pb[9 + k];
  }
  // rotation: R_t = E R_{t-1} with E = exp([w_t]x)
  const double th2 = W[0] * W[0] + W[1] * W[1] + W[2] * W[2];
  const double th = sqrt(th2);
  double a, b, sa, ca;
  if (th < 1e-4) {
    a = 0.5 - th2 / 24.0;
    b = 1.0 / 6.0 - th2 / 120.0;
  } else {
    a = (1.0 - cos(th)) / th2;
    b = (th - sin(th)) / (th2 * th);
  }
  sa = th < 1e-4 ? 1.0 - th2 / 6.0 : sin(th) / th;
  ca = a;   // (1 - cos)/th^2
  // E^T v = v - sa (w x v) + ca w x (w x v)
  double wxt[3], wwxt[3];
  cross(W, thb, wxt);
  cross(W, wxt, wwxt);
  double thb_prev[3], jt[3];
  for (int k = 0; k < 3; ++k) {
    thb_prev[k] = thb[k] - sa * wxt[k] + ca * wwxt[k];
    jt[k] = thb[k] - a * wxt[k] + b * wwxt[k];   // J_l(w)^T thb
  }
  for (int k = 0; k < 3; ++k) Wb[k] += jt[k];
  double ds = 0.0;
  for (int k = 0; k < 3; ++k) {
    ds += Ub[k] * (-(f[k] + f[6 + k]) / (s * s * V) + ph.gravity[k] / (s * s));
    ds += Wb[k] * (-(f[3 + k] + f[9 + k]) / (s * s * I1));
  }
  if (balance)
    for (int k = 0; k < 3; ++k) ds += abar[k] * (-V * ph.gravity[k] / (double)g.ncell);
  sbar[p] += ds;
  for (int k = 0; k < 3; ++k) {
    fhbar[6 * p + k] = Ub[k] / (s * V);
    fhbar[6 * p + 3 + k] = Wb[k] / (s * I1);
    pb[k] = Xb[k];
    pb[3 + k] = thb_prev[k];
    pb[6 + k] = Ub[k];
    pb[9 + k] = Wb[k];
  }
}

// Momentum exchange in reverse, at nodes owned in o_{t-1}:
//   F_p = -sum S, T_p = -sum r x S,
//   S = sum_i (c_i - u_p) f*_i + (c_i + u_p) f_opp(i)
//     = J* - J_t + u_p (rho_t - rho*)
// with J*, rho* the moments of f*_{t-1} at the node and J_t, rho_t those of
// the streamed f_t.  Sbar = -(Fbar + Tbar x r) goes to hbar (post-stream
// terms) here and to gbar (own terms) in k_adj_stream.
__global__ __launch_bounds__(256) void k_adj_mea(
    const double* __restrict__ fprev, double* __restrict__ hbar,
    const int* __restrict__ owner, const double* __restrict__ prec,
    const double* __restrict__ fhbar, Geom g, double* __restrict__ pbar) {
  const long long n = g.ncell;
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double inc[PB];
  for (int k = 0; k < PB; ++k) inc[k] = 0.0;
  int o = -1;
  if (id < n) o = owner_id(owner[id]);
  if (o >= 0) {
    int x, y, z;
    node_xyz(id, g, x, y, z);
    const double* pr = prec + (size_t)PREC_N * o;
    double r[3], wr[3], up[3];
    lever(g, x, y, z, rec_X(pr), r);
    cross(rec_W(pr), r, wr);
    for (int k = 0; k < 3; ++k) up[k] = rec_U(pr)[k] + wr[k];
    const double* Fb = fhbar + 6 * o;
    double txr[3], Sb[3];
    cross(Fb + 3, r, txr);
    for (int k = 0; k < 3; ++k) Sb[k] = -(Fb[k] + txr[k]);
    double rs = 0.0, rt = 0.0, Js[3] = {0.0, 0.0, 0.0}, Jt[3] = {0.0, 0.0, 0.0};
    const double sbu = Sb[0] * up[0] + Sb[1] * up[1] + Sb[2] * up[2];
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const double fs = fprev[(long long)j * n + id];
      const double ft = fprev[(long long)j * n + wrap_id(x - cx(j), y - cy(j), z - cz(j), g)];
      rs += fs;
      rt += ft;
      Js[0] += cx(j) * fs; Js[1] += cy(j) * fs; Js[2] += cz(j) * fs;
      Jt[0] += cx(j) * ft; Jt[1] += cy(j) * ft; Jt[2] += cz(j) * ft;
      // post-stream population f_j at the node enters S with (u_p - c_j)
      const double sbc = Sb[0] * cx(j) + Sb[1] * cy(j) + Sb[2] * cz(j);
      hbar[(long long)j * n + id] += sbu - sbc;
    }
    double S[3], upb[3];
    for (int k = 0; k < 3; ++k) {
      S[k] = Js[k] - Jt[k] + up[k] * (rt - rs);
      upb[k] = Sb[k] * (rt - rs);
    }
    double sxt[3], upxw[3], rxup[3];
    cross(S, Fb + 3, sxt);
    cross(upb, rec_W(pr), upxw);
    cross(r, upb, rxup);
    for (int k = 0; k < 3; ++k) {
      inc[k] = sxt[k] - upxw[k];    // X
      inc[6 + k] = upb[k];          // U
      inc[9 + k] = rxup[k];         // omega
    }
  }
  commit_adjoint(o, inc, pbar);
}

// Streaming in reverse plus the own terms of the momentum exchange:
//   gbar_{t-1, i}(x) = hbar_i(x + c_i) + [x owned in o_{t-1}] Sbar . (c_i - u_p)
__global__ __launch_bounds__(256) void k_adj_stream(
    const double* __restrict__ hbar, double* __restrict__ gbar,
    const int* __restrict__ owner, const double* __restrict__ prec,
    const double* __restrict__ fhbar, Geom g) {
  const long long n = g.ncell;
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n) return;
  int x, y, z;
  node_xyz(id, g, x, y, z);
  const int o = owner_id(owner[id]);
  double Sb[3] = {0.0, 0.0, 0.0}, up[3] = {0.0, 0.0, 0.0};
  if (o >= 0) {
    const double* pr = prec + (size_t)PREC_N * o;
    double r[3], wr[3];
    lever(g, x, y, z, rec_X(pr), r);
    cross(rec_W(pr), r, wr);
    for (int k = 0; k < 3; ++k) up[k] = rec_U(pr)[k] + wr[k];
    const double* Fb = fhbar + 6 * o;
    double txr[3];
    cross(Fb + 3, r, txr);
    for (int k = 0; k < 3; ++k) Sb[k] = -(Fb[k] + txr[k]);
  }
  const double sbu = Sb[0] * up[0] + Sb[1] * up[1] + Sb[2] * up[2];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const double own = Sb[0] * cx(i) + Sb[1] * cy(i) + Sb[2] * cz(i) - sbu;
    gbar[(long long)i * n + id] =
        hbar[(long long)i * n + wrap_id(x + cx(i), y + cy(i), z + cz(i), g)] + own;
  }
}

// Copy the particle state (X, q, U, W, R) into a record array.
__global__ void k_rec_particles(Particles P, double* __restrict__ out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P.n) return;
  double* r = out + (size_t)PREC_N * p;
  for (int k = 0; k < 3; ++k) r[k] = P.X[3 * p + k];
  for (int k = 0; k < 4; ++k) r[3 + k] = P.q[4 * p + k];
  for (int k = 0; k < 3; ++k) r[7 + k] = P.U[3 * p + k];
  for (int k = 0; k < 3; ++k) r[10 + k] = P.W[3 * p + k];
  for (int k = 0; k < 9; ++k) r[13 + k] = P.R[9 * p + k];
}

// Copy the forces of the last step (F_h, T_h, F_c, T_c) into a record.
__global__ void k_rec_forces(int np, const double* Fh, const double* Th,
                             const double* Fc, const double* Tc,
                             double* __restrict__ out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  for (int k = 0; k < 3; ++k) {
    out[12 * p + k] = Fh[3 * p + k];
    out[12 * p + 3 + k] = Th[3 * p + k];
    out[12 * p + 6 + k] = Fc[3 * p + k];
    out[12 * p + 9 + k] = Tc[3 * p + k];
  }
}

__global__ void k_fill_zero(double* p, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

unsigned nblk(long long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

int adjoint_record_doubles() { return PREC_N; }
int adjoint_slots() { return PB; }

hipError_t launch_rec_particles(Ctx& c, double* out) {
  if (c.np == 0) return hipSuccess;
  hipLaunchKernelGGL(k_rec_particles, dim3(nblk(c.np)), dim3(256), 0, c.stream, c.part, out);
  return hipGetLastError();
}

hipError_t launch_rec_forces(Ctx& c, double* out) {
  if (c.np == 0) return hipSuccess;
  hipLaunchKernelGGL(k_rec_forces, dim3(nblk(c.np)), dim3(256), 0, c.stream, c.np,
                     c.Fh, c.Th, c.Fc, c.Tc, out);
  return hipGetLastError();
}

hipError_t launch_fill_zero(Ctx& c, double* p, long long n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_zero, dim3(nblk(n)), dim3(256), 0, c.stream, p, n);
  return hipGetLastError();
}

// One reverse step.  gbar: dJ/df*_t in, dJ/df*_{t-1} out; hbar: scratch
// lattice; fprev: f*_{t-1}; owner_prev / owner_t: o_{t-1}, o_t; prec_prev /
// prec_t: particle records of P_{t-1}, P_t; frc: forces of step t;
// pbar: particle adjoints (Pbar_t in, Pbar_{t-1} out); sbar: dJ/ds
// accumulated; work: fhbar (6 np) | abar (3) | per-block a partials.
hipError_t launch_adjoint_step(Ctx& c, double* gbar, double* hbar,
                               const double* fprev, const int* owner_prev,
                               const int* owner_t, const double* prec_prev,
                               const double* prec_t, const double* frc,
                               double* pbar, double* sbar, double* work) {
  const long long n = c.g.ncell;
  const unsigned nb = nblk(n);
  double* fhbar = work;
  double* abar = work + 6 * (size_t)(c.np > 0 ? c.np : 1);
  double* apart = abar + 3;
  hipLaunchKernelGGL(k_adj_collide, dim3(nb), dim3(256), 0, c.stream, gbar, fprev,
                     hbar, owner_t, prec_t, c.part, c.g, c.ph, pbar, apart);
  hipLaunchKernelGGL(k_adj_reduce_a, dim3(1), dim3(256), 0, c.stream, apart,
                     (long long)nb, abar);
  if (c.np > 0)
    hipLaunchKernelGGL(k_adj_move, dim3(nblk(c.np)), dim3(256), 0, c.stream, c.part,
                       c.ph, c.g, c.P.balance ? 1 : 0, prec_t, frc, abar, pbar,
                       fhbar, sbar);
  hipLaunchKernelGGL(k_adj_mea, dim3(nb), dim3(256), 0, c.stream, fprev, hbar,
                     owner_prev, prec_prev, fhbar, c.g, pbar);
  hipLaunchKernelGGL(k_adj_stream, dim3(nb), dim3(256), 0, c.stream, hbar, gbar,
                     owner_prev, prec_prev, fhbar, c.g);
  return hipGetLastError();
}

size_t adjoint_work_doubles(const Ctx& c) {
  return 6 * (size_t)(c.np > 0 ? c.np : 1) + 3 + 3 * (size_t)nblk(c.g.ncell);
}

}  // namespace hlbm
