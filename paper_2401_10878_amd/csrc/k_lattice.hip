// D3Q19 stream-collide with the HLBM velocity-shift coupling and the
// momentum exchange of the next step in one pass (and the momentum exchange
// as a pass of its own, for the initial state).
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
// Momentum exchange, eq. (16) read with post-streaming populations: for a
// node x owned by o,
//   S(x) = sum_i (c_i - u_p(x)) f_i*(x) + (c_i + u_p(x)) f_opp(i)(x)
// where f_opp(i)(x) is the value the next streaming brings to x.  The force
// and torque on particle o are F = -sum S, T = -sum r x S over the nodes it
// owns (eqs. (17)-(18)), summed per lattice block without atomics.  The
// lattice pass pushes each value it stores into the two sums it enters (of
// its own node and of the node it streams to); the separate pass pulls
// both for an owned node.
//
// Storage is a template parameter: FP64, FP32, or binary16 deviations
// h_i = f_i - w_i (FP32 arithmetic).
#include <hip/hip_fp16.h>

#include "context.h"

// Multiply-adds in this file may round once (fused): no integer decision is
// taken here from a floating-point value (the owner map and the contact
// decisions come from the other passes), and the vector units run one
// instruction instead of two.
#pragma clang fp contract(fast)

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
  __device__ static C as_stored(C v) { return v; }
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
  __device__ static C as_stored(C v) { return v; }
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
  // the value st writes, read back (round to nearest even)
  __device__ static C as_stored(C v) { return __half2float(__float2half_rn(v)); }
};
__device__ inline int owner_at(const int* owner, unsigned b) {
  return owner_id(*(const int*)((const char*)owner + b));
}
// Loads and stores at byte offset b of an array as raw buffer operations: a
// scalar resource over the array from p (no range check is relied on; every
// offset lies inside the array) and a 32-bit per-lane byte offset, which the
// hardware adds without vector address arithmetic.  Populations
// non-temporal, owner entries cached.
__device__ inline __amdgpu_buffer_rsrc_t rsrc_of(const void* p) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, -1, 0x00020000);
}
constexpr int BUF_NT = 2;
template <typename S>
__device__ inline typename Store<S>::C ld_buf(const S* base, unsigned b) {
  const __amdgpu_buffer_rsrc_t r = rsrc_of(base);
  if constexpr (sizeof(S) == 2)
    return __half2float(__ushort_as_half(__builtin_amdgcn_raw_buffer_load_b16(r, b, 0, BUF_NT)));
  else if constexpr (sizeof(S) == 4)
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, b, 0, BUF_NT));
  else
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, b, 0, BUF_NT));
}
template <typename S>
__device__ inline void st_buf(S* base, unsigned b, typename Store<S>::C v) {
  const __amdgpu_buffer_rsrc_t r = rsrc_of(base);
  if constexpr (sizeof(S) == 2)
    __builtin_amdgcn_raw_buffer_store_b16(__half_as_ushort(__float2half_rn(v)), r, b, 0, BUF_NT);
  else if constexpr (sizeof(S) == 4)
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, b, 0, BUF_NT);
  else
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0)), v), r, b, 0, BUF_NT);
}
__device__ inline int ld_owner_buf(const int* base, unsigned b) {
  return (int)__builtin_amdgcn_raw_buffer_load_b32(rsrc_of(base), b, 0, 0);
}
// c_i . (a, b, c) from the non-zero components of c_i only (a product with
// a zero component is not dropped by the compiler: 0 * inf is not 0).  The
// sum starts from -0, which adds exactly; the direction's components are
// compile-time constants in the unrolled loops.
template <typename C>
__device__ inline C cdot(int i, C a, C b, C c) {
  C r = (C)-0.0;
  if (cx(i)) r += cx(i) > 0 ? a : -a;
  if (cy(i)) r += cy(i) > 0 ? b : -b;
  if (cz(i)) r += cz(i) > 0 ? c : -c;
  return r;
}
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
template <typename V>
__device__ void commit_group(int q, const V* s, const V* t, int lid,
                             double (*row)[6], double* ovf) {
  const int lane = threadIdx.x % WAVE;
  bool pend = q >= 0;
  for (;;) {
    const uint64_t m = __ballot(pend);
    if (m == 0) break;
    const int pick = __builtin_amdgcn_readlane(q, __ffsll((long long)m) - 1);
    const bool take = pend && q == pick;
    V v[6];
    for (int k = 0; k < 3; ++k) {
      v[k] = take ? s[k] : (V)0;
      v[3 + k] = take ? t[k] : (V)0;
    }
    // component lane/2 in even lanes < 12 (FP32 values: first level in FP32)
    double sum;
    if constexpr (sizeof(V) == 4)
      sum = wave_sum6_scatter_f(v);
    else
      sum = wave_sum6_scatter(v);
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

// Block sums of four per-lane values through one reduce-scatter per
// wavefront (the sums land in lanes 0, 2, 4, 6; FP32 values add their first
// level, two lanes, in FP32 and the rest in FP64), then the four
// wavefronts' rows added in fixed order and stored at out[4 * block ..].
// Every thread of the block must call it.
template <typename C>
__device__ void block_sums4s(C a, C b, C c, C d, const BlockNode& nd, double* out) {
  __shared__ double rows[4][4];
  const C v[6] = {a, b, c, d, (C)0, (C)0};
  double sum;
  if constexpr (sizeof(C) == 4)
    sum = wave_sum6_scatter_f(v);
  else
    sum = wave_sum6_scatter(v);
  const int lane = threadIdx.x % WAVE;
  if (lane < 8 && (lane & 1) == 0) rows[nd.wave][lane >> 1] = sum;
  __syncthreads();
  if (threadIdx.x < 4) {
    const int k = threadIdx.x;
    out[4 * nd.block + k] = ((rows[0][k] + rows[1][k]) + rows[2][k]) + rows[3][k];
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

// Velocity c_i of direction i (1..18) for a run-time index, from the order
// rest, +-x, +-y, +-z, then the edge pairs (1,1,0), (-1,-1,0), (1,-1,0),
// (-1,1,0) of the planes xy, xz, yz.
__device__ inline void dir_of(int i, int& d0, int& d1, int& d2) {
  d0 = d1 = d2 = 0;
  if (i <= 6) {
    const int a = (i - 1) >> 1, sg = (i & 1) ? 1 : -1;
    d0 = a == 0 ? sg : 0;
    d1 = a == 1 ? sg : 0;
    d2 = a == 2 ? sg : 0;
  } else {
    const int k = i - 7, grp = k >> 2, j = k & 3;
    const int s1 = (j == 0 || j == 2) ? 1 : -1, s2 = (j == 0 || j == 3) ? 1 : -1;
    d0 = grp == 2 ? 0 : s1;
    d1 = grp == 0 ? s2 : (grp == 2 ? s1 : 0);
    d2 = grp == 0 ? 0 : s2;
  }
}

// Masked moments of the stored post-collision deviations v_i (i >= 1) of
// one node over a set of links: m0 = sum v_i, m1 = sum c_i v_i and the
// second moment Pi = sum c_i c_i^T v_i (six components), added link by link
// (the rare path of a third particle).
template <typename C>
struct LinkMoments {
  C m0, m1[3], pxx, pyy, pzz, pxy, pxz, pyz;
};
template <typename C>
__device__ inline void link_zero(LinkMoments<C>& m) {
  m.m0 = m.m1[0] = m.m1[1] = m.m1[2] = (C)0;
  m.pxx = m.pyy = m.pzz = m.pxy = m.pxz = m.pyz = (C)0;
}

// What the force and torque of a set of links need of its moments: m0, m1,
// the off-diagonal Pi and the sums qx = Pi_yy + Pi_zz, qy = Pi_xx + Pi_zz,
// qz = Pi_xx + Pi_yy (the torque takes (Pi - tr(Pi) 1) w).
template <typename C>
struct Closure {
  C m0, m1[3], pxy, pxz, pyz, qx, qy, qz;
};
template <typename C>
__device__ inline Closure<C> closure_of(const LinkMoments<C>& m) {
  return {m.m0, {m.m1[0], m.m1[1], m.m1[2]}, m.pxy, m.pxz, m.pyz,
          m.pyy + m.pzz, m.pxx + m.pzz, m.pxx + m.pyy};
}

// The closure over the links whose neighbour is owned by particle q
// (nbo[i] == q; ALL: over every link), from the opposite pairs: with a_i
// the masked value and,
// per pair (i, opp(i)) of first link c, s = a_i + a_opp(i) and
// d = a_i - a_opp(i), the pair adds s to m0, c d to m1 and c c^T s to Pi.
// The three axis pairs carry s1, s2, s3; the two pairs of each coordinate
// plane (first links (1, 1, 0) and (1, -1, 0) for xy, and likewise for xz
// and yz) add their sum S to both diagonal entries of the plane and their
// difference to its off-diagonal entry, so that
//   m0 = s1 + s2 + s3 + Sxy + Sxz + Syz,
//   Pi_yy + Pi_zz = m0 - s1 + Syz (and cyclically).
template <typename C, bool ALL = false>
__device__ inline Closure<C> pair_closure(const C* v, const int* nbo, int q) {
  static_assert(cx(1) == 1 && cy(3) == 1 && cz(5) == 1, "axis pairs");
  static_assert(cx(7) == 1 && cy(7) == 1 && cz(7) == 0 && cx(9) == 1 && cy(9) == -1 &&
                    cz(9) == 0, "xy pairs");
  static_assert(cx(11) == 1 && cy(11) == 0 && cz(11) == 1 && cx(13) == 1 && cy(13) == 0 &&
                    cz(13) == -1, "xz pairs");
  static_assert(cx(15) == 0 && cy(15) == 1 && cz(15) == 1 && cx(17) == 0 && cy(17) == 1 &&
                    cz(17) == -1, "yz pairs");
  static_assert(opp(1) == 2 && opp(7) == 8 && opp(17) == 18, "pair order");
  C sp[10], dp[10];
#pragma unroll
  for (int k = 1; k <= 9; ++k) {
    const int i = 2 * k - 1;
    const C a = (ALL || nbo[i] == q) ? v[i] : (C)0;
    const C b = (ALL || nbo[i + 1] == q) ? v[i + 1] : (C)0;
    sp[k] = a + b;
    dp[k] = a - b;
  }
  const C Sxy = sp[4] + sp[5], Sxz = sp[6] + sp[7], Syz = sp[8] + sp[9];
  Closure<C> m;
  m.pxy = sp[4] - sp[5];
  m.pxz = sp[6] - sp[7];
  m.pyz = sp[8] - sp[9];
  m.m0 = ((sp[1] + sp[2]) + sp[3]) + ((Sxy + Sxz) + Syz);
  m.m1[0] = (dp[1] + (dp[4] + dp[5])) + (dp[6] + dp[7]);
  m.m1[1] = (dp[2] + (dp[4] - dp[5])) + (dp[8] + dp[9]);
  m.m1[2] = (dp[3] + (dp[6] - dp[7])) + (dp[8] - dp[9]);
  m.qx = (m.m0 - sp[1]) + Syz;
  m.qy = (m.m0 - sp[2]) + Sxz;
  m.qz = (m.m0 - sp[3]) + Sxy;
  return m;
}

// Force G and torque T that one node y hands to particle q through the
// links in m (y + c_i owned by q), eqs. (16)-(18) summed link by link: the
// post-collision value v_i leaving y enters S(y + c_i) as -(c_i - u_q(y +
// c_i)) v_i, and with r = r_q(y), u = u_q(y), u_q(y + c_i) = u + w x c_i,
// r_q(y + c_i) = r + c_i the sums over the links are
//   G += m1 - u m0 - w x m1,
//   T  = r x G - m1 x u + (Pi - tr(Pi) 1) w
// (c x (w x c) = |c|^2 w - c (c . w)).  G may carry the node's own terms
// already (they act at r).
template <typename C>
__device__ inline void link_force(const Closure<C>& m, const C* r, const C* u,
                                  const C* w, C* G, C* T) {
  G[0] += (m.m1[0] - u[0] * m.m0) - (w[1] * m.m1[2] - w[2] * m.m1[1]);
  G[1] += (m.m1[1] - u[1] * m.m0) - (w[2] * m.m1[0] - w[0] * m.m1[2]);
  G[2] += (m.m1[2] - u[2] * m.m0) - (w[0] * m.m1[1] - w[1] * m.m1[0]);
  T[0] = (r[1] * G[2] - r[2] * G[1]) - (m.m1[1] * u[2] - m.m1[2] * u[1]) +
         ((m.pxy * w[1] + m.pxz * w[2]) - m.qx * w[0]);
  T[1] = (r[2] * G[0] - r[0] * G[2]) - (m.m1[2] * u[0] - m.m1[0] * u[2]) +
         ((m.pxy * w[0] + m.pyz * w[2]) - m.qy * w[1]);
  T[2] = (r[0] * G[1] - r[1] * G[0]) - (m.m1[0] * u[1] - m.m1[1] * u[0]) +
         ((m.pxz * w[0] + m.pyz * w[1]) - m.qz * w[2]);
}

// Kinematics of particle q seen from node (x, y, z): r = minimg(node - X),
// u = U + w x r, w.  FP64 compute precision: from the FP64 state.  FP32:
// from the particle's FP32 kinematic record, the offset as the integer
// difference to the centre's integer part wrapped to the minimum image
// (unambiguous for the nodes within a particle's reach, far below half a
// periodic length) minus the fraction.
__device__ inline int wrap_image(int k, int L, bool periodic) {
  const int h = L >> 1;
  k = (periodic && k > h) ? k - L : k;
  return (periodic && k < -h) ? k + L : k;
}
template <typename C>
__device__ inline void kinematics(const Particles& P, int q, int x, int y, int z,
                                  const Geom& g, C* r, C* u, C* w) {
  if constexpr (sizeof(C) == 4) {
    const float4* rec = (const float4*)(P.LR32 + LREC * q);
    const float4 a = rec[0], b = rec[1], c = rec[2];
    // a: Xi0 Xi1 Xi2 Xf0, b: Xf1 Xf2 U0 U1, c: U2 W0 W1 W2
    r[0] = (float)wrap_image(x - __float_as_int(a.x), g.nx, true) - a.w;
    r[1] = (float)wrap_image(y - __float_as_int(a.y), g.ny, true) - b.x;
    r[2] = (float)wrap_image(z - __float_as_int(a.z), g.nz, g.periodic_z != 0) - b.y;
    w[0] = c.y;
    w[1] = c.z;
    w[2] = c.w;
    u[0] = b.z + (w[1] * r[2] - w[2] * r[1]);
    u[1] = b.w + (w[2] * r[0] - w[0] * r[2]);
    u[2] = c.x + (w[0] * r[1] - w[1] * r[0]);
  } else {
    const double X0 = P.X[3 * q], X1 = P.X[3 * q + 1], X2 = P.X[3 * q + 2];
    const double U0 = P.U[3 * q], U1 = P.U[3 * q + 1], U2 = P.U[3 * q + 2];
    const double W0 = P.W[3 * q], W1 = P.W[3 * q + 1], W2 = P.W[3 * q + 2];
    r[0] = (C)minimg((double)x - X0, (double)g.nx, true);
    r[1] = (C)minimg((double)y - X1, (double)g.ny, true);
    r[2] = (C)minimg((double)z - X2, (double)g.nz, g.periodic_z != 0);
    w[0] = (C)W0;
    w[1] = (C)W1;
    w[2] = (C)W2;
    u[0] = (C)U0 + (w[1] * r[2] - w[2] * r[1]);
    u[1] = (C)U1 + (w[2] * r[0] - w[0] * r[2]);
    u[2] = (C)U2 + (w[0] * r[1] - w[1] * r[0]);
  }
}

// Commit of one round of per-lane (force G, torque T) contributions to the
// block's LDS rows (commit_group adds -sum, so the values go in negated and
// widened to FP64).
template <typename C>
__device__ inline void commit_round(int q, const C* G, const C* T, int lid,
                                    double (*row)[6], double* ovf) {
  double s[3], t[3];
  for (int k = 0; k < 3; ++k) {
    s[k] = -(double)G[k];
    t[k] = -(double)T[k];
  }
  commit_group(q, s, t, lid, row, ovf);
}

// Register budget without spills: FP64 at most 128 VGPRs (four wavefronts
// per SIMD), FP32 and binary16 at most 72 (seven: the pass is faster at
// seven wavefronts than at six or five), 80 with both the polyhedron
// distance and the balance sums.  POLY: built
// with the polyhedron signed distance (scenes without polyhedra run the
// form without it, which needs fewer registers).  BAL: with the block sums
// and device acceleration of the zero-net-flux balance force.  WALL: z
// bounded by walls (half-way bounce-back).
//
// The pass also evaluates the momentum exchange of the NEXT step, eqs.
// (16)-(18), with the owner map and particle state its collision used: every
// post-collision value v_i it stores at node y enters exactly two sums of
// eq. (16) read with post-streaming populations, the own term
// (c_i - u_p(y)) v_i of S(y) and the incoming term -(c_i - u_q(y + c_i)) v_i
// of S(y + c_i) (or, beyond a wall, the bounced term of S(y)).  Each lane
// pushes these terms to the owners of y and of its 18 neighbours (read from
// the owner map), grouped by particle through link masks, and the
// wavefronts reduce them per particle into the block's partial-sum slots
// (F_p = -sum S, T_p = -sum r x S, fixed order, no atomics).  The
// storage's rest weights cancel in every S(x), so the pushed values are the
// stored deviations h_i (FP32, binary16: the values as rounded for storage)
// or f_i - w_i (FP64).  Blocks whose candidate list is empty (no particle
// owns a node within one node of the block), and wavefronts without an owned
// node or a neighbour of one, skip it.
template <typename S, bool POLY, bool BAL, bool WALL, bool ELL = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(
    sizeof(S) == 8 ? 4 : (ELL ? 5 : (POLY && BAL ? 6 : 7)), 8))) void k_lattice(const S* __restrict__ src,
                                                 S* __restrict__ dst,
                                                 const int* __restrict__ owner,
                                                 Particles P, Geom g, Phys ph,
                                                 Counters* ctr,
                                                 double* __restrict__ bal_part,
                                                 Tiles tl) {
  using C = typename Store<S>::C;
  __shared__ double red[4][LCAP_MAX][6];
  // queue of the rare further-particle contributions, per wavefront
  constexpr int XQ = 32;
  __shared__ int xqid[4][XQ];
  __shared__ double xqv[4][XQ][6];
  const BlockNode nd = block_node(g);
  const int x = nd.x, y = nd.y, z = nd.z;
  const bool valid = nd.valid;
  const int n = (int)g.ncell;
  // Every lane loads: a lane outside the lattice reads the nearest node
  // (clamped coordinates) and then stores nothing and adds to no sum.
  const Nbr nb = neighbours(g, x < g.nx ? x : g.nx - 1, y < g.ny ? y : g.ny - 1,
                            z < g.nz ? z : g.nz - 1);
  // walls exist only on a bounded z axis (WALL): elsewhere the wall terms
  // drop out at compile time
  const bool wallm = WALL && nb.wall_m, wallp = WALL && nb.wall_p;
  auto beyond = [&](int dz) { return dz < 0 ? (wallm ? 1 : 0) : (dz > 0 ? (wallp ? 2 : 0) : 0); };
  const int lane = threadIdx.x % WAVE;
  int cnt = tl.lcount[nd.block];
  cnt = __builtin_amdgcn_readfirstlane(cnt < g.tile_cap ? cnt : g.tile_cap);
  const bool mea = cnt > 0;                       // uniform over the block

  // Addresses: the y and z parts of a node's index are uniform over the
  // wavefront (one x-row), so they go into each access's base pointer with
  // the direction; the lanes add only the byte offset of x - 1, x or x + 1.
  constexpr unsigned SB = sizeof(S) == 8 ? 3u : (sizeof(S) == 4 ? 2u : 1u);
  auto rowpl = [&](int dy, int dz) { return nb.rows[dy + 1] + nb.planes[dz + 1]; };
  const unsigned xo[3] = {(unsigned)nb.xs[0] << SB, (unsigned)nb.xs[1] << SB,
                          (unsigned)nb.xs[2] << SB};
  const unsigned xw[3] = {(unsigned)nb.xs[0] << 2, (unsigned)nb.xs[1] << 2,
                          (unsigned)nb.xs[2] << 2};
  const int o = valid ? owner_at(owner + rowpl(0, 0), xw[1]) : -1;

  C f[Q];
  {
    // one load per direction from a selected base and offset (a branch per
    // direction would make the compiler wait for memory between the
    // loads), then the moving-wall term of the links that bounced back
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      // (beyond() is uniform over the wavefront, which holds one x-row)
      const bool bw = beyond(-cz(i)) != 0;
      const S* base = src + (size_t)(bw ? opp(i) : i) * (size_t)n +
                      (bw ? rowpl(0, 0) : rowpl(-cy(i), -cz(i)));
      f[i] = ld_buf<S>(base, bw ? xo[1] : xo[1 - cx(i)]);
    }
    if (wallm || wallp) {
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const int bw = beyond(-cz(i));
        if (bw) {
          const double* uw = ph.wall_u[bw - 1];
          const double cu = cx(i) * uw[0] + cy(i) * uw[1] + cz(i) * uw[2];
          f[i] += (C)(6.0 * wgt(i) * cu);
        }
      }
    }
  }

  // f holds the stored values: f_i itself (FP64) or h_i = f_i - w_i.  The
  // collision below is written for both: with D = sum of stored values,
  // rho = D (+1 when shifted), J = sum c_i h_i = sum c_i f_i, and the
  // equilibrium is shifted by the same w_i.
  // (sums start from -0, which adds exactly)
  C D = (C)-0.0, J0 = (C)-0.0, J1 = (C)-0.0, J2 = (C)-0.0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    D += f[i];
    if (cx(i)) J0 += cx(i) > 0 ? f[i] : -f[i];
    if (cy(i)) J1 += cy(i) > 0 ? f[i] : -f[i];
    if (cz(i)) J2 += cz(i) > 0 ? f[i] : -f[i];
  }
  const C rho = Store<S>::shifted ? (C)1 + D : D;
  if (valid && !(rho > (C)0 && rho < (C)1e30)) atomicOr(&ctr->unstable, 1);
  // (FP32: the hardware reciprocal, within 1 ulp)
  C inv;
  if constexpr (sizeof(C) == 4)
    inv = __builtin_amdgcn_rcpf(rho);
  else
    inv = (C)1 / rho;
  const C u0 = J0 * inv, u1 = J1 * inv, u2 = J2 * inv;

  // coupling: B and u_p of the owner, in FP64 for FP64 storage and in FP32
  // otherwise (the owner itself was decided in FP64)
  C rp[3] = {(C)0, (C)0, (C)0}, upy[3] = {(C)0, (C)0, (C)0}, wp[3] = {(C)0, (C)0, (C)0};
  C B = (C)0;
  if (o >= 0) {
    kinematics<C>(P, o, x, y, z, g, rp, upy, wp);
    if constexpr (Store<S>::shifted) {
      // rotation, size and shape from the FP32 kinematic record
      const float4* rec = (const float4*)(P.LR32 + LREC * o);
      const float4 ra = rec[3], rb = rec[4], rc = rec[5];
      const float Rf[9] = {ra.x, ra.y, ra.z, ra.w, rb.x, rb.y, rb.z, rb.w, rc.x};
      // (an ellipsoid beyond the band either way: B from its bounds)
      const int band = ELL ? ellip_band<float>(P.poly, __float_as_int(rc.z), rc.y, Rf, rp[0],
                                               rp[1], rp[2], ph.eps_h32, 1e-3f)
                           : -1;
      if (band >= 0) {
        B = (C)band;
      } else {
        const C d = sdf32<ELL>(__float_as_int(rc.z), rc.y, Rf, rp[0], rp[1], rp[2],
                               POLY ? P.poly : nullptr);
        B = weight32(d, ph.eps_h32, ph.eps_q32);
      }
    } else {
      const int shape = P.shape[o];
      const double size = P.size[o];
      double Ro[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) Ro[k] = P.R[9 * o + k];
      const int band = ELL ? ellip_band<double>(P.poly, shape, size, Ro, (double)rp[0],
                                                (double)rp[1], (double)rp[2], 0.5 * ph.eps, 1e-9)
                           : -1;
      if (band >= 0) {
        B = (C)band;
      } else {
        const C d = sdf<ELL>(shape, size, Ro, rp[0], rp[1], rp[2], POLY ? P.poly : nullptr);
        B = weight(d, ph.eps);
      }
    }
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
    const C cu = cdot<C>(i, u0, u1, u2);
    const C cv = cdot<C>(i, v0, v1, v2);
    const C wi = (C)wgt(i);
    const C even = wi * (A + (C)4.5 * rho * (cv * cv - keep * (cu * cu)));
    const C odd = (C)3 * wi * rho * (cv - keep * cu);
    f[i] = keep * f[i] + (even + odd);
    f[i + 1] = keep * f[i + 1] + (even - odd);
  }
  if (valid) {
#pragma unroll
    for (int i = 0; i < Q; ++i) st_buf<S>(dst + (size_t)i * (size_t)n + rowpl(0, 0), xo[1], f[i]);
  }
  if (BAL) {
    // mass and momentum of the collided populations, per block in fixed
    // order, for the zero-net-flux balance controller: the collision keeps
    // the mass and sets the momentum to rho v (before the storage rounds the
    // values; with binary16 storage, sums over the rounded values would
    // feed the storage's rounding noise back into the uniform acceleration)
    C m = (C)0, j0 = (C)0, j1 = (C)0, j2 = (C)0;
    if (valid) {
      m = rho;
      j0 = rho * v0;
      j1 = rho * v1;
      j2 = rho * v2;
    }
    block_sums4s<C>(m, j0, j1, j2, nd, bal_part);
  }
  if (!mea) return;                               // uniform over the block

  // ---- momentum exchange of the next step, pushed link by link ----------
  const int* list = tl.llist + nd.block * g.tile_cap;
  const int* ent = tl.lent + nd.block * g.tile_cap;
  const int lid = lane < cnt ? list[lane] : -1;   // candidate list, one per lane
  for (int c = lane; c < cnt; c += WAVE)
    for (int k = 0; k < 6; ++k) red[nd.wave][c][k] = 0.0;
  // Owners of the 18 neighbours (-2: beyond a wall) and the lane's entries:
  // A the node's own particle (own terms and links to its own nodes), or for
  // a fluid node the largest id owning a neighbour; B the largest other id
  // owning a neighbour; further particles around one node (rare) after the
  // commit of A and B.  Selects and extrema only, no branches.
  // (any negative entry means no owner: the extrema and the comparisons
  // below take none of them for a particle)
  int nbo[Q];
  nbo[0] = -1;
  int mx = -1;
  unsigned mn = ~0u;        // smallest id owning a neighbour (negative: none)
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    // (a link beyond a wall reads its clamped neighbour, then replaced)
    const int v = ld_owner_buf(owner + rowpl(cy(i), cz(i)), xw[1 + cx(i)]);
    nbo[i] = beyond(cz(i)) ? -2 : v;
    mx = max(mx, nbo[i]);
    mn = min(mn, (unsigned)nbo[i]);
  }
  const int qa = !valid ? -1 : (o >= 0 ? o : mx);
  // a particle other than A owns a neighbour: the ids owning neighbours are
  // not all A (A = mx for a fluid node)
  const bool two = qa >= 0 && mx >= 0 && (mx != qa || (int)mn != qa);
  const bool multi = __ballot(two) != 0;          // uniform over the wavefront
  int qb = -1;
  bool more = false;
  if (multi) {
#pragma unroll
    for (int i = 1; i < Q; ++i) qb = max(qb, nbo[i] != qa ? nbo[i] : -1);
#pragma unroll
    for (int i = 1; i < Q; ++i) more = more | ((nbo[i] >= 0) & (nbo[i] != qa) & (nbo[i] != qb));
    qb = two ? qb : -1;
    more = more && two;
  }
  if (__ballot(qa >= 0) != 0) {                   // else no lane has an entry
  // One pass over the stored values v_i (FP64: minus the rest weight): the
  // link moments of A (and B), and the own terms of S(y), sum_i (c_i - u) v_i
  // over every link plus, for a link beyond a wall, the bounced value
  // b_i = v_i - 6 w_i c_i . u_w entering as -(c_opp(i) - u) b_i =
  // (c_i + u) b_i: the force on the owner is -(J' + W1) + u (m0' - W0),
  // m0' = sum_{i>=1} v_i, J' = sum c_i v_i, W1 = sum c_i b_i, W0 = sum b_i.
  // The collision conserves mass and moves the momentum to rho v, so
  // m0' = (rho - 1) - v_0 (D - v_0 when shifted) and J' = rho v (to the
  // rounding of the collision); binary16 storage rounds far more, and there
  // m0' and J' are summed over the rounded values.
  constexpr bool ROUNDED = sizeof(S) == 2;
  C vs[Q];
#pragma unroll
  for (int i = 1; i < Q; ++i)
    vs[i] = ROUNDED ? Store<S>::as_stored(f[i]) : (Store<S>::shifted ? f[i] : f[i] - (C)wgt(i));
  C m0, j[3];
  if constexpr (ROUNDED) {
    const Closure<C> own = pair_closure<C, true>(vs, nullptr, 0);
    m0 = own.m0;
    j[0] = own.m1[0];
    j[1] = own.m1[1];
    j[2] = own.m1[2];
  } else {
    const C v_0 = Store<S>::shifted ? f[0] : f[0] - (C)wgt(0);
    m0 = (Store<S>::shifted ? D : rho - (C)1) - v_0;
    j[0] = rho * v0;
    j[1] = rho * v1;
    j[2] = rho * v2;
  }
  if (wallm || wallp) {
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      const int bw = beyond(cz(i));
      if (bw) {
        const double* uw = ph.wall_u[bw - 1];
        const C bi = vs[i] - (C)(6.0 * wgt(i) * (cx(i) * uw[0] + cy(i) * uw[1] + cz(i) * uw[2]));
        m0 -= bi;
        if (cx(i)) j[0] += cx(i) > 0 ? bi : -bi;
        if (cy(i)) j[1] += cy(i) > 0 ? bi : -bi;
        if (cz(i)) j[2] += cz(i) > 0 ? bi : -bi;
      }
    }
  }
  const Closure<C> La = pair_closure<C>(vs, nbo, qa);
  Closure<C> Lb;
  if (multi) Lb = pair_closure<C>(vs, nbo, qb);
  C Ga[3] = {(C)0, (C)0, (C)0}, Ta[3] = {(C)0, (C)0, (C)0};
  C Gb[3] = {(C)0, (C)0, (C)0}, Tb[3] = {(C)0, (C)0, (C)0};
  if (qa >= 0) {
    const bool own = o >= 0;
    C rr[3], uk[3], wk[3];
    // (the coupling's r, u_p, w of the owner are evaluated again here
    // rather than kept live across the collision)
    kinematics<C>(P, qa, x, y, z, g, rr, uk, wk);
    for (int k = 0; k < 3; ++k) Ga[k] = own ? uk[k] * m0 - j[k] : (C)0;
    link_force<C>(La, rr, uk, wk, Ga, Ta);
  }
  if (multi && qb >= 0) {
    C rb[3], ub[3], wb[3];
    kinematics<C>(P, qb, x, y, z, g, rb, ub, wb);
    link_force<C>(Lb, rb, ub, wb, Gb, Tb);
  }
  // one commit for A and B: each distinct particle of the wavefront in
  // turn, the lanes adding the entries that name it (FP64 wave sums into
  // the block's LDS rows, which hold -sum)
  // (pending entries as wavefront masks, the lane predicates taken from
  // them without per-lane bookkeeping; B only in wavefronts that have one)
  {
    uint64_t pa = __ballot(qa >= 0);
    uint64_t pb = multi ? __ballot(qb >= 0) : 0ull;
    while ((pa | pb) != 0) {
      const int pick = pa ? __builtin_amdgcn_readlane(qa, __ffsll((long long)pa) - 1)
                          : __builtin_amdgcn_readlane(qb, __ffsll((long long)pb) - 1);
      // (A and B name different particles: at most one of ta, tb holds)
      const uint64_t ma = pa & __ballot(qa == pick);
      const bool ta = __builtin_amdgcn_inverse_ballot_w64(ma);
      pa &= ~ma;
      const uint64_t mb = pb & __ballot(qb == pick);
      const bool tb = __builtin_amdgcn_inverse_ballot_w64(mb);
      pb &= ~mb;
      C vv[6];
      for (int k = 0; k < 3; ++k) {
        vv[k] = ta ? -Ga[k] : (tb ? -Gb[k] : (C)0);
        vv[3 + k] = ta ? -Ta[k] : (tb ? -Tb[k] : (C)0);
      }
      double sum;
      if constexpr (sizeof(C) == 4)
        sum = wave_sum6_scatter_f3(vv);
      else
        sum = wave_sum6_scatter(vv);
      const uint64_t hit = __ballot(lid == pick);
      if (lane < 12 && (lane & 1) == 0) {
        const int k = lane >> 1;
        if (hit) {
          red[nd.wave][__ffsll((long long)hit) - 1][k] -= sum;
        } else {
          atomic_add_f64(&tl.ovf[6 * pick + k], -sum);
        }
      }
    }
  }
  }
  // further particles around one node (rare): in increasing id order per
  // node, from the node's values read back from what was just stored, one
  // link at a time (a loop the compiler keeps rolled, so that this path
  // adds no registers to the kernel); each lane's contribution goes into a
  // per-wavefront LDS queue in lane order, which is added to the block
  // rows in queue order (a full queue sends the rest to the overflow sums
  // with atomics)
  if (__ballot(more)) {
    int last = -1, nq = 0;
    while (__ballot(more)) {
      int q = -1;
      unsigned mask = 0u;
      if (more) {
#pragma nounroll
        for (int i = 1; i < Q; ++i) {
          int d0, d1, d2;
          dir_of(i, d0, d1, d2);
          // the neighbour's index from its coordinates (periodic wrap; a
          // z beyond a wall has no node)
          int xn = x + d0, yn = y + d1, zn = z + d2;
          xn = xn < 0 ? xn + g.nx : (xn >= g.nx ? xn - g.nx : xn);
          yn = yn < 0 ? yn + g.ny : (yn >= g.ny ? yn - g.ny : yn);
          const bool bw = WALL && (zn < 0 || zn >= g.nz);
          zn = zn < 0 ? zn + g.nz : (zn >= g.nz ? zn - g.nz : zn);
          const int b = bw ? -2 : owner_id(owner[xn + g.nx * (yn + g.ny * zn)]);
          const bool cand = b >= 0 && b != qa && b != qb && b > last;
          const bool lower = cand && (q < 0 || b < q);
          mask = lower ? (1u << i) : ((cand && b == q) ? (mask | (1u << i)) : mask);
          q = lower ? b : q;
        }
        more = q >= 0;
        last = q;
      }
      const uint64_t bq = __ballot(q >= 0);
      if (q >= 0) {
        LinkMoments<C> Lq;
        link_zero(Lq);
#pragma nounroll
        for (int i = 1; i < Q; ++i) {
          if ((mask >> i) & 1u) {
            int d0, d1, d2;
            dir_of(i, d0, d1, d2);
            const C sv = Store<S>::ld(dst, i * n + nb.off(0, 0, 0));
            const C a = Store<S>::shifted ? sv : sv - (C)(i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
            const C e0 = (C)d0, e1 = (C)d1, e2 = (C)d2;
            Lq.m0 += a;
            Lq.m1[0] += e0 * a;
            Lq.m1[1] += e1 * a;
            Lq.m1[2] += e2 * a;
            Lq.pxx += (e0 * e0) * a;
            Lq.pyy += (e1 * e1) * a;
            Lq.pzz += (e2 * e2) * a;
            Lq.pxy += (e0 * e1) * a;
            Lq.pxz += (e0 * e2) * a;
            Lq.pyz += (e1 * e2) * a;
          }
        }
        C G[3] = {(C)0, (C)0, (C)0}, T[3] = {(C)0, (C)0, (C)0}, rq[3], uq[3], wq[3];
        kinematics<C>(P, q, x, y, z, g, rq, uq, wq);
        link_force<C>(closure_of(Lq), rq, uq, wq, G, T);
        const int slot = nq + __builtin_popcountll(bq & ((1ull << lane) - 1ull));
        if (slot < XQ) {
          xqid[nd.wave][slot] = q;
          for (int k = 0; k < 3; ++k) {
            xqv[nd.wave][slot][k] = (double)G[k];
            xqv[nd.wave][slot][3 + k] = (double)T[k];
          }
        } else {
          for (int k = 0; k < 3; ++k) {
            atomic_add_f64(&tl.ovf[6 * q + k], (double)G[k]);
            atomic_add_f64(&tl.ovf[6 * q + 3 + k], (double)T[k]);
          }
        }
      }
      nq += __builtin_popcountll(bq);
    }
    nq = nq < XQ ? nq : XQ;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int e = 0; e < nq; ++e) {
      const int q = xqid[nd.wave][e];
      const uint64_t hit = __ballot(lid == q);
      if (lane < 6) {
        if (hit)
          red[nd.wave][__ffsll((long long)hit) - 1][lane] -= -xqv[nd.wave][e][lane];
        else
          atomic_add_f64(&tl.ovf[6 * q + lane], xqv[nd.wave][e][lane]);
      }
    }
  }
  store_block(red, list, ent, cnt, g, tl.part);
  // every wavefront read the block's count before the barrier in
  // store_block: reset it for the next binning (a block with a zero count
  // has nothing to reset)
  if (threadIdx.x == 0) tl.lcount[nd.block] = 0;
}

// Momentum exchange, eqs. (16)-(18), over the populations f* of the last
// collision with the owner map and particle state that collision used, as a
// pass of its own: the force of the initial state (every later step's comes
// from the stream-collide pass).  With
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
  // S and r x S in the compute precision C (FP64 for FP64 storage); the
  // minimum image in FP64, the reductions across nodes in FP64 (after a
  // first FP32 level for FP32 values)
  C s[3] = {(C)0, (C)0, (C)0}, t[3] = {(C)0, (C)0, (C)0};
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
    C dD = (C)-0.0, dJ0 = (C)-0.0, dJ1 = (C)-0.0, dJ2 = (C)-0.0;
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
    const C r0 = (C)minimg((double)x - X0, (double)g.nx, true);
    const C r1 = (C)minimg((double)y - X1, (double)g.ny, true);
    const C r2 = (C)minimg((double)z - X2, (double)g.nz, g.periodic_z != 0);
    const C w0 = (C)W0, w1 = (C)W1, w2 = (C)W2;
    const C up0 = (C)U0 + (w1 * r2 - w2 * r1);
    const C up1 = (C)U1 + (w2 * r0 - w0 * r2);
    const C up2 = (C)U2 + (w0 * r1 - w1 * r0);
    s[0] = dJ0 - up0 * dD;
    s[1] = dJ1 - up1 * dD;
    s[2] = dJ2 - up2 * dD;
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

// Zero-net-flux balance controller (balance mode 2).  The lattice blocks'
// (mass, momentum) sums are added in two fixed-order stages: BAL_PARTS
// workgroups each sum one contiguous range of blocks (thread t takes
// entries t, t + 256, .. of the range, then a fixed tree), then one
// workgroup sums the BAL_PARTS results the same way, giving the lattice mass
// M and momentum P.  init: M, P_{-1} = P, b_0 = -P / M.  Update after the
// collision of step t (which used b_t): C_t = P_t - P_{t-1} - b_t M,
// b_{t+1} = -(P_t + C_t) / M.  The acceleration in use is a = fluid_accel + b.
__device__ void tree_sum4(double (*sh)[4], double* acc) {
  for (int k = 0; k < 4; ++k) sh[threadIdx.x][k] = acc[k];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int k = 0; k < 4; ++k) sh[threadIdx.x][k] += sh[threadIdx.x + w][k];
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_balance_part(const double* __restrict__ part,
                                                      unsigned nblocks,
                                                      double* __restrict__ out) {
  __shared__ double sh[256][4];
  const unsigned chunk = (nblocks + BAL_PARTS - 1) / BAL_PARTS;
  const unsigned b0 = blockIdx.x * chunk;
  const unsigned b1 = b0 + chunk < nblocks ? b0 + chunk : nblocks;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (unsigned b = b0 + threadIdx.x; b < b1; b += 256)
    for (int k = 0; k < 4; ++k) acc[k] += part[4 * (size_t)b + k];
  tree_sum4(sh, acc);
  if (threadIdx.x < 4) out[4 * blockIdx.x + threadIdx.x] = sh[0][threadIdx.x];
}

__global__ __launch_bounds__(256) void k_balance(const double* __restrict__ parts,
                                                 Counters* ctr, Phys ph, int init) {
  __shared__ double sh[256][4];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (unsigned b = threadIdx.x; b < BAL_PARTS; b += 256)
    for (int k = 0; k < 4; ++k) acc[k] += parts[4 * (size_t)b + k];
  tree_sum4(sh, acc);
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
  const bool bal = c.ph.bal_mode == 2, wall = c.g.periodic_z == 0;
  auto k = c.has_ellipsoid
               ? (bal ? k_lattice<S, true, true, false, true>
                      : (wall ? k_lattice<S, true, false, true, true>
                              : k_lattice<S, true, false, false, true>))
           : c.has_poly
               ? (bal ? k_lattice<S, true, true, false>
                      : (wall ? k_lattice<S, true, false, true> : k_lattice<S, true, false, false>))
               : (bal ? k_lattice<S, false, true, false>
                      : (wall ? k_lattice<S, false, false, true> : k_lattice<S, false, false, false>));
  hipLaunchKernelGGL(k, dim3(tile_blocks(c.g)), dim3(256), 0, c.stream, (const S*)src,
                     (S*)dst, c.owner, c.part, c.g, c.ph, c.counters, c.bal_part, c.tl);
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

hipError_t launch_balance(Ctx& c, const void* f, int init, hipStream_t st) {
  if (init) DISPATCH(c, run_pop_moments, (c, f));
  const unsigned nb = tile_blocks(c.g);
  double* parts = c.bal_part + 4 * (size_t)nb;
  hipLaunchKernelGGL(k_balance_part, dim3(BAL_PARTS), dim3(256), 0, st, c.bal_part,
                     nb, parts);
  hipLaunchKernelGGL(k_balance, dim3(1), dim3(256), 0, st, parts, c.counters, c.ph,
                     init);
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
