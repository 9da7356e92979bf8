// D3Q19 stream-collide with the HLBM velocity-shift coupling, and the
// momentum exchange of the next step as a pass of its own.
//
// Lattice pass, per node y (one lane), with the particle state already
// advanced:
//   pull     f_i(y) = f_i*(y - c_i)   (half-way bounce-back at z walls)
//   moments  rho = sum f_i, u = sum c_i f_i / rho
//   coupling owner o(y) from the owner map; B = B(d_o(y)),
//            u_p = U_o + w_o x r  (Sec. 3.2)
//   collide  du = B (u_p - u) + a,
//            f_i* = f_i^eq(rho, u + du) + (1 - 1/tau)(f_i - f_i^eq(rho, u))
//            (BGK eq. (12) plus the EDM source eq. (14), rearranged)
//
// Momentum-exchange pass over the populations f* just written, eq. (16)
// read with post-streaming populations: for a node x owned by o,
//   S(x) = sum_i (c_i - u_p(x)) f_i*(x) + (c_i + u_p(x)) f_opp(i)(x)
// where f_opp(i)(x) is the value the next streaming brings to x.  The force
// and torque on particle o are F = -sum S, T = -sum r x S over the nodes it
// owns (eqs. (17)-(18)), summed per lattice block without atomics.
//
// Storage is a template parameter: FP64, FP32, or binary16 deviations
// h_i = f_i - w_i (FP32 arithmetic).
#include <hip/hip_fp16.h>

#include "context.h"

namespace hlbm {

namespace {

// Storage of the populations.  FP64 stores f itself; FP32 and binary16
// store the deviation h = f - w_i from the rest weights ("shifted"), so that
// rounding acts on the small part of f.  ld/st move the stored value h (or
// f), full() turns it into f.  Stores, and the stream-collide pass's loads
// (ldn), are non-temporal: each population is written once and read by the
// next pass, and the arrays are hundreds of times the size of the caches
// (6% less time for the stream-collide pass; the momentum-exchange pass,
// which reads the same lines for neighbouring nodes, keeps ordinary loads).
template <typename S>
struct Store;
template <>
struct Store<double> {
  using C = double;
  static constexpr bool shifted = false;
  __device__ static C ld(const double* p, int k) { return p[k]; }
  __device__ static C ldb(const double* p, unsigned k) {
    return *(const double*)((const char*)p + k * 8u);
  }
  __device__ static void st(double* p, int k, C v) { __builtin_nontemporal_store(v, p + k); }
  __device__ static C ldn(const double* p, int k) { return __builtin_nontemporal_load(p + k); }
};
template <>
struct Store<float> {
  using C = float;
  static constexpr bool shifted = true;
  __device__ static C ld(const float* p, int k) { return p[k]; }
  __device__ static C ldb(const float* p, unsigned k) {
    return *(const float*)((const char*)p + k * 4u);
  }
  __device__ static void st(float* p, int k, C v) { __builtin_nontemporal_store(v, p + k); }
  __device__ static C ldn(const float* p, int k) { return __builtin_nontemporal_load(p + k); }
};
template <>
struct Store<__half> {
  using C = float;
  static constexpr bool shifted = true;
  __device__ static C ld(const __half* p, int k) { return __half2float(p[k]); }
  __device__ static C ldb(const __half* p, unsigned k) {
    return __half2float(*(const __half*)((const char*)p + k * 2u));
  }
  __device__ static void st(__half* p, int k, C v) {
    __builtin_nontemporal_store(__half_as_ushort(__float2half_rn(v)), reinterpret_cast<unsigned short*>(p) + k);
  }
  __device__ static C ldn(const __half* p, int k) {
    return __half2float(__ushort_as_half(__builtin_nontemporal_load(reinterpret_cast<const unsigned short*>(p) + k)));
  }
};
template <typename S>
__device__ inline double full_f(typename Store<S>::C h, int i) {
  return Store<S>::shifted ? wgt(i) + (double)h : (double)h;
}

// Logical block id with consecutive ids kept on one XCD (workgroups are
// dispatched round-robin over the 8 XCDs, each with its own L2).
__device__ inline unsigned xcd_block(unsigned bid, unsigned nblocks) {
  const unsigned m = nblocks / 8, r = nblocks % 8;
  const unsigned xcd = bid % 8, k = bid / 8;
  return xcd * m + (xcd < r ? xcd : r) + k;
}

// Lattice block of the workgroup (LX x LY x LZ nodes, one x-row per
// wavefront, the four rows stacked along y or z), with consecutive block ids
// kept on one XCD.
static_assert(LX == WAVE && LY * LZ == 4 && (LY == 1 || LZ == 1), "block shape");
struct BlockNode {
  long long block;
  int x, y, z, wave;
  bool valid;
};
__device__ inline BlockNode block_node(const Geom& g) {
  BlockNode r;
  // fewer than 2^31 blocks (the cell count is bounded on the host)
  const unsigned nblocks = (unsigned)g.ltx * (unsigned)g.lty * (unsigned)g.ltz;
  const unsigned lb = xcd_block(blockIdx.x, nblocks);
  r.block = lb;
  const unsigned yz = fdiv(lb, g.fltx);
  const unsigned bz = fdiv(yz, g.flty);
  const int bx = (int)(lb - yz * (unsigned)g.ltx);
  const int by = (int)(yz - bz * (unsigned)g.lty);
  r.wave = (int)((unsigned)__builtin_amdgcn_readfirstlane(threadIdx.x) / WAVE);
  r.x = bx * LX + (int)(threadIdx.x % WAVE);
  r.y = by * LY + (LY > 1 ? r.wave : 0);
  r.z = (int)bz * LZ + (LZ > 1 ? r.wave : 0);
  r.valid = r.x < g.nx && r.y < g.ny && r.z < g.nz;
  return r;
}

// Wave-level commit of one group of per-lane (force, torque) contributions
// keyed by particle id q (-1 = none): for each distinct id, the wavefront sum
// is added (by lane 0, in a fixed order) to that candidate's LDS row as
// -sum, the force and torque on the particle (eqs. (17)-(18)).  An id missing
// from the candidate list (not expected) goes to the overflow sums.
__device__ void commit_group(int q, const double* s, const double* t, int lid,
                             double (*row)[6], double* ovf) {
  const int lane = threadIdx.x % WAVE;
  bool pend = q >= 0;
  for (;;) {
    const uint64_t m = __ballot(pend);
    if (m == 0) break;
    const int pick = __builtin_amdgcn_readlane(q, __ffsll((long long)m) - 1);
    const bool take = pend && q == pick;
    double v[6];
    for (int k = 0; k < 3; ++k) {
      v[k] = take ? s[k] : 0.0;
      v[3 + k] = take ? t[k] : 0.0;
    }
    const double sum = wave_sum6_scatter(v);   // component lane/2 in even lanes < 12
    const uint64_t hit = __ballot(lid == pick);
    if (lane < 12 && (lane & 1) == 0) {
      const int k = lane >> 1;
      if (hit) {
        const int c = __ffsll((long long)hit) - 1;
        row[c][k] -= sum;
      } else {
        atomic_add_f64(&ovf[6 * pick + k], -sum);
      }
    }
    if (take) pend = false;
  }
}

// After all wavefronts of the block have committed: add the four LDS rows in
// fixed order and store every (block, particle) partial-sum slot once.
__device__ void store_block(double (*red)[LCAP_MAX][6], const int* list,
                            const int* ent, int cnt, Geom g, double* part) {
  __syncthreads();
  for (int t = threadIdx.x; t < cnt * 6; t += blockDim.x) {
    const int c = t / 6, k = t % 6;
    const double v = ((red[0][c][k] + red[1][c][k]) + red[2][c][k]) + red[3][c][k];
    part[((size_t)list[c] * g.maxent + ent[c]) * 6 + k] = v;
  }
}

// Block sums of four per-lane values (widened to FP64): wavefront sums,
// then the four wavefronts' rows added in fixed order by thread 0 and
// stored at out[4 * block ..].  Every thread of the block must call it.
__device__ void block_sums4(double a, double b, double c, double d,
                            const BlockNode& nd, double* out) {
  __shared__ double rows[4][4];
  const double v[4] = {wave_sum(a), wave_sum(b), wave_sum(c), wave_sum(d)};
  if (threadIdx.x % WAVE == 0)
    for (int k = 0; k < 4; ++k) rows[nd.wave][k] = v[k];
  __syncthreads();
  if (threadIdx.x < 4) {
    const int k = threadIdx.x;
    out[4 * nd.block + k] = ((rows[0][k] + rows[1][k]) + rows[2][k]) + rows[3][k];
  }
}

// Offset of node (x, y, z) and the periodic / walled neighbour indices.
struct Nbr {
  int xs[3], ys[3], zs[3];      // coordinates of x-1, x, x+1 etc. (wrapped)
  int rows[3], planes[3];       // y and z parts of the linear offset
  bool wall_m, wall_p;          // z-1 / z+1 lies beyond a wall
  __device__ int off(int dx, int dy, int dz) const {
    return xs[dx + 1] + rows[dy + 1] + planes[dz + 1];
  }
  __device__ int beyond(int dz) const {   // 0 inside, 1 bottom, 2 top wall
    return dz < 0 ? (wall_m ? 1 : 0) : (dz > 0 ? (wall_p ? 2 : 0) : 0);
  }
};
__device__ inline Nbr neighbours(const Geom& g, int x, int y, int z) {
  Nbr nb;
  const bool perz = g.periodic_z != 0;
  nb.xs[0] = x == 0 ? g.nx - 1 : x - 1;
  nb.xs[1] = x;
  nb.xs[2] = x + 1 >= g.nx ? 0 : x + 1;
  nb.ys[0] = y == 0 ? g.ny - 1 : y - 1;
  nb.ys[1] = y;
  nb.ys[2] = y + 1 >= g.ny ? 0 : y + 1;
  nb.zs[1] = z;
  nb.zs[0] = z - 1;
  nb.zs[2] = z + 1;
  nb.wall_m = nb.wall_p = false;
  if (perz) {
    if (nb.zs[0] < 0) nb.zs[0] = g.nz - 1;
    if (nb.zs[2] >= g.nz) nb.zs[2] = 0;
  } else {
    nb.wall_m = nb.zs[0] < 0;
    nb.wall_p = nb.zs[2] >= g.nz;
    if (nb.wall_m) nb.zs[0] = 0;
    if (nb.wall_p) nb.zs[2] = g.nz - 1;
  }
  for (int k = 0; k < 3; ++k) {
    nb.rows[k] = g.nx * nb.ys[k];
    nb.planes[k] = g.nx * g.ny * nb.zs[k];
  }
  return nb;
}

// At most 128 VGPRs (four wavefronts per SIMD) without spills.  POLY: built
// with the polyhedron signed distance (scenes without polyhedra run the
// form without it, which needs fewer registers).  BAL: with the block sums
// and device acceleration of the zero-net-flux balance force.
template <typename S, bool POLY, bool BAL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_lattice(const S* __restrict__ src,
                                                 S* __restrict__ dst,
                                                 const int* __restrict__ owner,
                                                 Particles P, Geom g, Phys ph,
                                                 Counters* ctr,
                                                 double* __restrict__ bal_part) {
  using C = typename Store<S>::C;
  const BlockNode nd = block_node(g);
  const int x = nd.x, y = nd.y, z = nd.z;
  const bool valid = nd.valid;
  const int n = (int)g.ncell;
  const bool perz = g.periodic_z != 0;
  const Nbr nb = neighbours(g, x, y, z);
  const int self = nb.off(0, 0, 0);

  C f[Q];
  int o = -1;
  if (valid) {
    // one load per direction from a selected index (a branch per direction
    // would make the compiler wait for memory between the loads), then the
    // moving-wall term of the links that bounced back
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int src_i = nb.beyond(-cz(i)) ? opp(i) * n + self
                                          : i * n + nb.off(-cx(i), -cy(i), -cz(i));
      f[i] = Store<S>::ldn(src, src_i);
    }
    o = owner_id(owner[self]);
    if (nb.wall_m || nb.wall_p) {
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const int bw = nb.beyond(-cz(i));
        if (bw) {
          const double* uw = ph.wall_u[bw - 1];
          const double cu = cx(i) * uw[0] + cy(i) * uw[1] + cz(i) * uw[2];
          f[i] += (C)(6.0 * wgt(i) * cu);
        }
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < Q; ++i) f[i] = Store<S>::shifted ? (C)0 : (C)wgt(i);
  }

  // f holds the stored values: f_i itself (FP64) or h_i = f_i - w_i.  The
  // collision below is written for both: with D = sum of stored values,
  // rho = D (+1 when shifted), J = sum c_i h_i = sum c_i f_i, and the
  // equilibrium is shifted by the same w_i.
  C D = 0, J0 = 0, J1 = 0, J2 = 0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    D += f[i];
    if (cx(i)) J0 += cx(i) > 0 ? f[i] : -f[i];
    if (cy(i)) J1 += cy(i) > 0 ? f[i] : -f[i];
    if (cz(i)) J2 += cz(i) > 0 ? f[i] : -f[i];
  }
  const C rho = Store<S>::shifted ? (C)1 + D : D;
  if (valid && !(rho > (C)0 && rho < (C)1e30)) atomicOr(&ctr->unstable, 1);
  const C inv = (C)1 / rho;
  const C u0 = J0 * inv, u1 = J1 * inv, u2 = J2 * inv;

  // coupling: B and u_p of the owner, in FP64 for FP64 storage and in FP32
  // otherwise (the owner itself was decided in FP64)
  C upy[3] = {(C)0, (C)0, (C)0};
  C B = (C)0;
  if (o >= 0) {
    // the owner's record, all loads issued before any use
    const double X0 = P.X[3 * o], X1 = P.X[3 * o + 1], X2 = P.X[3 * o + 2];
    const double U0 = P.U[3 * o], U1 = P.U[3 * o + 1], U2 = P.U[3 * o + 2];
    const double W0 = P.W[3 * o], W1 = P.W[3 * o + 1], W2 = P.W[3 * o + 2];
    const int shape = P.shape[o];
    const double size = P.size[o];
    double Ro[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) Ro[k] = P.R[9 * o + k];
    const C r0 = (C)minimg((double)x - X0, (double)g.nx, true);
    const C r1 = (C)minimg((double)y - X1, (double)g.ny, true);
    const C r2 = (C)minimg((double)z - X2, (double)g.nz, perz);
    C d;
    if constexpr (Store<S>::shifted) {
      d = sdf32(shape, (float)size, Ro, r0, r1, r2, POLY ? P.poly : nullptr);
      B = weight32(d, (float)ph.eps);
    } else {
      d = sdf(shape, size, Ro, r0, r1, r2, POLY ? P.poly : nullptr);
      B = weight(d, ph.eps);
    }
    const C w0 = (C)W0, w1 = (C)W1, w2 = (C)W2;
    upy[0] = (C)U0 + (w1 * r2 - w2 * r1);
    upy[1] = (C)U1 + (w2 * r0 - w0 * r2);
    upy[2] = (C)U2 + (w0 * r1 - w1 * r0);
  }
  // uniform fluid acceleration: fixed, or the zero-net-flux controller's
  double ax = ph.a_ext[0], ay = ph.a_ext[1], az = ph.a_ext[2];
  if (BAL) {
    ax = ctr->bal_a[0];
    ay = ctr->bal_a[1];
    az = ctr->bal_a[2];
  }
  const C du0 = B * (upy[0] - u0) + (C)ax;
  const C du1 = B * (upy[1] - u1) + (C)ay;
  const C du2 = B * (upy[2] - u2) + (C)az;
  const C v0 = u0 + du0, v1 = u1 + du1, v2 = u2 + du2;
  const C uu = u0 * u0 + u1 * u1 + u2 * u2;
  const C vv = v0 * v0 + v1 * v1 + v2 * v2;
  const C keep = (C)1 - (C)ph.omega;
  // equilibrium minus the storage shift: w_i [Ds + rho (3cu + 4.5cu^2 - 1.5u.u)]
  // with Ds = rho - 1 (= D) when shifted, rho otherwise
  const C Ds = Store<S>::shifted ? D : rho;
  // f*_i = e2_i + keep (f_i - e1_i) = keep f_i + (e2_i - keep e1_i), and for
  // the opposite pair (i, opp(i)), c . u changes sign, so
  //   e2 - keep e1 = w_i [A + 4.5 rho ((c.v)^2 - keep (c.u)^2)]   (even)
  //                 +/- 3 w_i rho (c.v - keep c.u)                  (odd)
  // with A = (1 - keep) Ds - 1.5 rho (v.v - keep u.u).
  const C A = ((C)1 - keep) * Ds - (C)1.5 * rho * (vv - keep * uu);
  f[0] = keep * f[0] + (C)wgt(0) * A;
#pragma unroll
  for (int i = 1; i < Q; i += 2) {
    const C cu = (C)cx(i) * u0 + (C)cy(i) * u1 + (C)cz(i) * u2;
    const C cv = (C)cx(i) * v0 + (C)cy(i) * v1 + (C)cz(i) * v2;
    const C wi = (C)wgt(i);
    const C even = wi * (A + (C)4.5 * rho * (cv * cv - keep * (cu * cu)));
    const C odd = (C)3 * wi * rho * (cv - keep * cu);
    f[i] = keep * f[i] + (even + odd);
    f[i + 1] = keep * f[i + 1] + (even - odd);
  }
  if (valid) {
#pragma unroll
    for (int i = 0; i < Q; ++i) Store<S>::st(dst, i * n + self, f[i]);
  }
  if (BAL) {
    // mass and momentum of the collided populations, per block in fixed
    // order, for the zero-net-flux balance controller
    C m = 0, j0 = 0, j1 = 0, j2 = 0;
    if (valid) {
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        m += f[i];
        if (cx(i)) j0 += cx(i) > 0 ? f[i] : -f[i];
        if (cy(i)) j1 += cy(i) > 0 ? f[i] : -f[i];
        if (cz(i)) j2 += cz(i) > 0 ? f[i] : -f[i];
      }
      if constexpr (Store<S>::shifted) m += (C)1;
    }
    block_sums4(m, j0, j1, j2, nd, bal_part);
  }
}

// Momentum exchange, eqs. (16)-(18), over the populations f* of the last
// collision with the owner map and particle state that collision used.  With
// f_i(x) the value the next streaming brings to x (pull from x - c_i, or the
// bounce-back value at a wall) and re-indexing the second sum by opp(i),
//   S(x) = sum_i (c_i - u_p(x)) f_i*(x) + (c_i + u_p(x)) f_opp(i)(x)
//        = sum_{i>=1} (c_i - u_p(x)) d_i,   d_i = f_i*(x) - f_i(x)
// (d_0 = 0).  Shifted storage: both terms of d_i carry the same rest weight,
// so d_i is the difference of two stored values.  d_i and the node sums are
// formed in the compute precision C of the storage (FP64 for FP64 storage,
// FP32 for the shifted forms, whose stored values are small deviations);
// u_p, S, r x S and every reduction are FP64.  Each lane takes one node;
// the wavefront sums -S and -r x S per particle into its LDS row of the
// block's candidate slots, and every (block, particle) slot is stored once.
// Blocks with no candidate particle have no owned node and exit at once.
template <typename S>
__global__ __launch_bounds__(256) void k_mea(const S* __restrict__ fs,
                                             const int* __restrict__ owner,
                                             Particles P, Geom g, Phys ph,
                                             Tiles tl) {
  using C = typename Store<S>::C;
  __shared__ double red[4][LCAP_MAX][6];
  const BlockNode nd = block_node(g);
  const long long tile = nd.block;
  int cnt = tl.lcount[tile];
  cnt = __builtin_amdgcn_readfirstlane(cnt < g.tile_cap ? cnt : g.tile_cap);
  if (cnt == 0) return;                           // uniform over the block
  const int lane = threadIdx.x % WAVE;
  const int* list = tl.llist + tile * g.tile_cap;
  const int* ent = tl.lent + tile * g.tile_cap;
  const int lid = lane < cnt ? list[lane] : -1;   // candidate list, one per lane
  for (int c = lane; c < cnt; c += WAVE)
    for (int k = 0; k < 6; ++k) red[nd.wave][c][k] = 0.0;

  const int x = nd.x, y = nd.y, z = nd.z;
  const int n = (int)g.ncell;
  const Nbr nb = neighbours(g, x, y, z);
  const int self = nb.off(0, 0, 0);
  const int o = nd.valid ? owner_id(owner[self]) : -1;
  double s[3] = {0.0, 0.0, 0.0}, t[3] = {0.0, 0.0, 0.0};
  if (o >= 0) {
    // all population and record loads issued before any use
    // (beyond a wall the neighbour index is clamped into the lattice; that
    // load is replaced by the bounce-back value after all loads are issued)
    C fo[Q], fi[Q];
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      // a scalar base per direction and 32-bit byte offsets (the arrays are
      // under 2^31 values), so the loads need no 64-bit vector address
      // arithmetic (9% less time for binary16, the same for FP32 and FP64)
      const S* base = fs + (size_t)i * (size_t)n;
      fo[i] = Store<S>::ldb(base, (unsigned)self);
      fi[i] = Store<S>::ldb(base, (unsigned)nb.off(-cx(i), -cy(i), -cz(i)));
    }
    const double X0 = P.X[3 * o], X1 = P.X[3 * o + 1], X2 = P.X[3 * o + 2];
    const double U0 = P.U[3 * o], U1 = P.U[3 * o + 1], U2 = P.U[3 * o + 2];
    const double W0 = P.W[3 * o], W1 = P.W[3 * o + 1], W2 = P.W[3 * o + 2];
    C dD = 0, dJ0 = 0, dJ1 = 0, dJ2 = 0;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      const int bw = nb.beyond(-cz(i));
      C d = fo[i] - (bw ? fo[opp(i)] : fi[i]);
      if (bw) {
        const double* uw = ph.wall_u[bw - 1];
        d -= (C)(6.0 * wgt(i) * (cx(i) * uw[0] + cy(i) * uw[1] + cz(i) * uw[2]));
      }
      dD += d;
      if (cx(i)) dJ0 += cx(i) > 0 ? d : -d;
      if (cy(i)) dJ1 += cy(i) > 0 ? d : -d;
      if (cz(i)) dJ2 += cz(i) > 0 ? d : -d;
    }
    const double r0 = minimg((double)x - X0, (double)g.nx, true);
    const double r1 = minimg((double)y - X1, (double)g.ny, true);
    const double r2 = minimg((double)z - X2, (double)g.nz, g.periodic_z != 0);
    const double up0 = U0 + (W1 * r2 - W2 * r1);
    const double up1 = U1 + (W2 * r0 - W0 * r2);
    const double up2 = U2 + (W0 * r1 - W1 * r0);
    s[0] = (double)dJ0 - up0 * (double)dD;
    s[1] = (double)dJ1 - up1 * (double)dD;
    s[2] = (double)dJ2 - up2 * (double)dD;
    t[0] = r1 * s[2] - r2 * s[1];
    t[1] = r2 * s[0] - r0 * s[2];
    t[2] = r0 * s[1] - r1 * s[0];
  }
  commit_group(o, s, t, lid, red[nd.wave], tl.ovf);
  store_block(red, list, ent, cnt, g, tl.part);
}

// Mass and momentum of a population field, per lattice block (the initial
// state of the zero-net-flux balance controller).
template <typename S>
__global__ __launch_bounds__(256) void k_pop_moments(const S* __restrict__ f, Geom g,
                                                     double* __restrict__ out) {
  using C = typename Store<S>::C;
  const BlockNode nd = block_node(g);
  const int n = (int)g.ncell;
  double m = 0.0, j0 = 0.0, j1 = 0.0, j2 = 0.0;
  if (nd.valid) {
    const int self = nd.x + g.nx * (nd.y + g.ny * nd.z);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const double v = full_f<S>(Store<S>::ld(f, i * n + self), i);
      m += v;
      j0 += cx(i) * v;
      j1 += cy(i) * v;
      j2 += cz(i) * v;
    }
  }
  block_sums4(m, j0, j1, j2, nd, out);
}

// Zero-net-flux balance controller (balance mode 2), one workgroup: the
// block sums are added in fixed order (thread t takes blocks t, t + 256, ..,
// then a fixed tree), giving the lattice mass M and momentum P.
// init: M, P_{-1} = P, b_0 = -P / M.  Update after the collision of step t
// (which used b_t): C_t = P_t - P_{t-1} - b_t M, b_{t+1} = -(P_t + C_t) / M.
// The acceleration in use is a = fluid_accel + b.
__global__ __launch_bounds__(256) void k_balance(const double* __restrict__ part,
                                                 unsigned nblocks, Counters* ctr,
                                                 Phys ph, int init) {
  __shared__ double sh[256][4];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (unsigned b = threadIdx.x; b < nblocks; b += 256)
    for (int k = 0; k < 4; ++k) acc[k] += part[4 * (size_t)b + k];
  for (int k = 0; k < 4; ++k) sh[threadIdx.x][k] = acc[k];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int k = 0; k < 4; ++k) sh[threadIdx.x][k] += sh[threadIdx.x + w][k];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (init) ctr->bal_M = sh[0][0];
    const double M = ctr->bal_M;
    for (int k = 0; k < 3; ++k) {
      const double P = sh[0][1 + k];
      double b;
      if (init) {
        b = -P / M;
      } else {
        const double Ct = P - ctr->bal_P[k] - ctr->bal_b[k] * M;
        b = -(P + Ct) / M;
      }
      ctr->bal_b[k] = b;
      ctr->bal_P[k] = P;
      ctr->bal_a[k] = ph.a_ext[k] + b;
    }
  }
}

template <typename S>
__global__ void k_fill_eq(S* f, size_t n, double rho, double u0, double u1,
                          double u2) {
  const size_t id = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (id >= n) return;
  const double uu = u0 * u0 + u1 * u1 + u2 * u2;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const double cu = cx(i) * u0 + cy(i) * u1 + cz(i) * u2;
    const double e = wgt(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    Store<S>::st(f, (int)(i * n + id),
                 (typename Store<S>::C)(Store<S>::shifted ? e - wgt(i) : e));
  }
}

template <typename S>
__global__ void k_store_dir(S* f, size_t n, int i, const double* srcv) {
  const size_t id = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (id >= n) return;
  Store<S>::st(f, (int)(i * n + id),
               (typename Store<S>::C)(Store<S>::shifted ? srcv[id] - wgt(i) : srcv[id]));
}

template <typename S>
__global__ void k_load_dir(const S* f, size_t n, int i, double* out) {
  const size_t id = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (id >= n) return;
  out[id] = full_f<S>(Store<S>::ld(f, (int)(i * n + id)), i);
}

// comp = -1: density; 0..2: velocity component (FP64 moments of f*)
template <typename S>
__global__ void k_moment(const S* f, size_t n, int comp, double* out) {
  const size_t id = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (id >= n) return;
  double rho = 0.0, J = 0.0;
  for (int i = 0; i < Q; ++i) {
    const double v = full_f<S>(Store<S>::ld(f, (int)(i * n + id)), i);
    rho += v;
    const int c = comp == 0 ? cx(i) : (comp == 1 ? cy(i) : cz(i));
    J += c * v;
  }
  out[id] = comp < 0 ? rho : J / rho;
}

unsigned blocks_for(size_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

#define DISPATCH(c, FN, ...)                                        \
  switch ((c).precision) {                                          \
    case HLBM_FP64: FN<double> __VA_ARGS__; break;                  \
    case HLBM_FP32: FN<float> __VA_ARGS__; break;                   \
    default: FN<__half> __VA_ARGS__; break;                         \
  }

static unsigned tile_blocks(const Geom& g) {
  return (unsigned)g.ltx * (unsigned)g.lty * (unsigned)g.ltz;
}

template <typename S>
static void run_lattice(Ctx& c, const void* src, void* dst) {
  const bool bal = c.ph.bal_mode == 2;
  auto k = c.has_poly ? (bal ? k_lattice<S, true, true> : k_lattice<S, true, false>)
                      : (bal ? k_lattice<S, false, true> : k_lattice<S, false, false>);
  hipLaunchKernelGGL(k, dim3(tile_blocks(c.g)), dim3(256), 0, c.stream, (const S*)src,
                     (S*)dst, c.owner, c.part, c.g, c.ph, c.counters, c.bal_part);
}

hipError_t launch_lattice(Ctx& c, const void* src, void* dst) {
  DISPATCH(c, run_lattice, (c, src, dst));
  return hipGetLastError();
}

template <typename S>
static void run_mea(Ctx& c, const void* fs) {
  hipLaunchKernelGGL(k_mea<S>, dim3(tile_blocks(c.g)), dim3(256), 0,
                     c.stream, (const S*)fs, c.owner, c.part, c.g, c.ph, c.tl);
}

hipError_t launch_mea(Ctx& c, const void* fstar) {
  DISPATCH(c, run_mea, (c, fstar));
  return hipGetLastError();
}

template <typename S>
static void run_pop_moments(Ctx& c, const void* f) {
  hipLaunchKernelGGL(k_pop_moments<S>, dim3(tile_blocks(c.g)), dim3(256), 0,
                     c.stream, (const S*)f, c.g, c.bal_part);
}

hipError_t launch_balance(Ctx& c, const void* f, int init) {
  if (init) DISPATCH(c, run_pop_moments, (c, f));
  hipLaunchKernelGGL(k_balance, dim3(1), dim3(256), 0, c.stream, c.bal_part,
                     tile_blocks(c.g), c.counters, c.ph, init);
  return hipGetLastError();
}

template <typename S>
static void run_fill(Ctx& c, void* f, double rho, const double* u) {
  hipLaunchKernelGGL(k_fill_eq<S>, dim3(blocks_for(c.g.ncell)), dim3(256), 0,
                     c.stream, (S*)f, (size_t)c.g.ncell, rho, u[0], u[1], u[2]);
}

hipError_t launch_fill_equilibrium(Ctx& c, void* f, double rho, const double u[3]) {
  DISPATCH(c, run_fill, (c, f, rho, u));
  return hipGetLastError();
}

template <typename S>
static void run_store(Ctx& c, void* f, int i, const double* srcv) {
  hipLaunchKernelGGL(k_store_dir<S>, dim3(blocks_for(c.g.ncell)), dim3(256), 0,
                     c.stream, (S*)f, (size_t)c.g.ncell, i, srcv);
}

hipError_t launch_store_direction(Ctx& c, void* f, int i, const double* srcv) {
  DISPATCH(c, run_store, (c, f, i, srcv));
  return hipGetLastError();
}

template <typename S>
static void run_load(Ctx& c, const void* f, int i, double* out) {
  hipLaunchKernelGGL(k_load_dir<S>, dim3(blocks_for(c.g.ncell)), dim3(256), 0,
                     c.stream, (const S*)f, (size_t)c.g.ncell, i, out);
}

hipError_t launch_load_direction(Ctx& c, const void* f, int i, double* dst) {
  DISPATCH(c, run_load, (c, f, i, dst));
  return hipGetLastError();
}

template <typename S>
static void run_moment(Ctx& c, const void* f, int comp, double* out) {
  hipLaunchKernelGGL(k_moment<S>, dim3(blocks_for(c.g.ncell)), dim3(256), 0,
                     c.stream, (const S*)f, (size_t)c.g.ncell, comp, out);
}

hipError_t launch_moment(Ctx& c, const void* f, int comp, double* out) {
  DISPATCH(c, run_moment, (c, f, comp, out));
  return hipGetLastError();
}

}  // namespace hlbm
