// D3Q19 stream-collide with the HLBM velocity-shift coupling and the
// momentum exchange, fused into one pass over the lattice.
//
// Per node y (one lane), with the particle state already advanced:
//   pull     f_i(y) = f_i*(y - c_i)   (half-way bounce-back at z walls)
//   moments  rho = sum f_i, u = sum c_i f_i / rho
//   coupling owner o(y) from the owner map; B = B(d_o(y)),
//            u_p = U_o + w_o x r  (Sec. 3.2)
//   collide  du = B (u_p - u) + a,
//            f_i* = f_i^eq(rho, u + du) + (1 - 1/tau)(f_i - f_i^eq(rho, u))
//            (BGK eq. (12) plus the EDM source eq. (14), rearranged)
//   MEA      the momentum exchange of the NEXT step, eq. (16), read with
//            post-streaming populations: node x contributes
//            S(x) = sum_i (c_i - u_p(x)) f_i*(x) + (c_i + u_p(x)) f_opp(i)(x)
//            after the next streaming.  Every post-collision value f_j*(y)
//            produced here enters exactly two such sums: that of y (own
//            term, c_j - u_p(y)) and that of x = y + c_j, which it reaches
//            by streaming (term -c_j + u_p(x)), or again that of y when it
//            bounces back from a wall.  Each lane scatters these terms to
//            the owners of y and of its 18 neighbours; the wavefront reduces
//            them per particle and commits F_p = -sum S, T_p = -sum r x S
//            with FP64 atomics (eqs. (17)-(18)).
//
// Storage is a template parameter: FP64, FP32, or binary16 deviations
// h_i = f_i - w_i (FP32 arithmetic).  Coupling geometry and all momentum
// exchange terms are FP64.
#include <hip/hip_fp16.h>

#include "context.h"

namespace hlbm {

namespace {

// Storage of the populations.  FP64 stores f itself; FP32 and binary16
// store the deviation h = f - w_i from the rest weights ("shifted"), so that
// rounding acts on the small part of f.  ld/st move the stored value h (or
// f), full() turns it into f.
template <typename S>
struct Store;
template <>
struct Store<double> {
  using C = double;
  static constexpr bool shifted = false;
  __device__ static C ld(const double* p, int k) { return p[k]; }
  __device__ static void st(double* p, int k, C v) { p[k] = v; }
};
template <>
struct Store<float> {
  using C = float;
  static constexpr bool shifted = true;
  __device__ static C ld(const float* p, int k) { return p[k]; }
  __device__ static void st(float* p, int k, C v) { p[k] = v; }
};
template <>
struct Store<__half> {
  using C = float;
  static constexpr bool shifted = true;
  __device__ static C ld(const __half* p, int k) { return __half2float(p[k]); }
  __device__ static void st(__half* p, int k, C v) { p[k] = __float2half_rn(v); }
};
template <typename S>
__device__ inline double full_f(typename Store<S>::C h, int i) {
  return Store<S>::shifted ? wgt(i) + (double)h : (double)h;
}

// Logical block id with consecutive ids kept on one XCD (workgroups are
// dispatched round-robin over the 8 XCDs, each with its own L2).
__device__ inline long long xcd_block(long long bid, long long nblocks) {
  const long long m = nblocks / 8, r = nblocks % 8;
  const long long xcd = bid % 8, k = bid / 8;
  return xcd * m + (xcd < r ? xcd : r) + k;
}

// Two-slot per-lane accumulator of (force, torque) contributions keyed by
// particle id; a third distinct id in one lane goes to the overflow sums.
struct Acc {
  int id0, id1;
  double v0[6], v1[6];
  __device__ void init() {
    id0 = id1 = -1;
    for (int k = 0; k < 6; ++k) v0[k] = v1[k] = 0.0;
  }
  __device__ void add(int q, const double* s, const double* t, double* ovf) {
    if (q == id0 || id0 < 0) {
      id0 = q;
      for (int k = 0; k < 3; ++k) { v0[k] += s[k]; v0[3 + k] += t[k]; }
    } else if (q == id1 || id1 < 0) {
      id1 = q;
      for (int k = 0; k < 3; ++k) { v1[k] += s[k]; v1[3 + k] += t[k]; }
    } else {
      for (int k = 0; k < 3; ++k) {
        atomic_add_f64(&ovf[6 * q + k], -s[k]);
        atomic_add_f64(&ovf[6 * q + 3 + k], -t[k]);
      }
    }
  }
};

// Lattice block of the workgroup (64 x 4 x 1 nodes, one x-row per
// wavefront), with consecutive block ids kept on one XCD.
struct BlockNode {
  long long block;
  int x, y, z, wave;
  bool valid;
};
__device__ inline BlockNode block_node(const Geom& g) {
  BlockNode r;
  const long long nblocks = (long long)g.ltx * g.lty * g.ltz;
  const long long lb = xcd_block(blockIdx.x, nblocks);
  r.block = lb;
  const int bx = (int)(lb % g.ltx);
  const int by = (int)((lb / g.ltx) % g.lty);
  const int bz = (int)(lb / ((long long)g.ltx * g.lty));
  r.wave = threadIdx.x / WAVE;
  r.x = bx * LX + (int)(threadIdx.x % WAVE);
  r.y = by * LY + r.wave;
  r.z = bz;
  r.valid = r.x < g.nx && r.y < g.ny && r.z < g.nz;
  return r;
}

// Block-level commit of the momentum exchange.  Each wavefront reduces its
// lanes' accumulators per particle and writes -sum (force and torque on the
// particle, eqs. (17)-(18)) into its own LDS row of the block's candidate
// slots; after a barrier the four rows are added in fixed order and every
// (block, particle) partial-sum slot is stored exactly once (zeros when
// nothing reached it).  Deterministic: no atomics on this path.
__device__ void commit_block(Acc& a, double (*red)[LCAP_MAX][6], int wave,
                             const int* list, const int* ent, int cnt, Geom g,
                             double* part, double* ovf) {
  const int lane = threadIdx.x % WAVE;
  for (int c = lane; c < cnt; c += WAVE)
    for (int k = 0; k < 6; ++k) red[wave][c][k] = 0.0;
  const int lid = lane < cnt ? list[lane] : -1;     // candidate list, one per lane
  bool p0 = a.id0 >= 0, p1 = a.id1 >= 0;
  for (;;) {
    const uint64_t m0 = __ballot(p0), m1 = __ballot(p1);
    if ((m0 | m1) == 0) break;
    const int pick = m0 ? __builtin_amdgcn_readlane(a.id0, __ffsll((long long)m0) - 1)
                        : __builtin_amdgcn_readlane(a.id1, __ffsll((long long)m1) - 1);
    const bool t0 = p0 && a.id0 == pick, t1 = p1 && a.id1 == pick;
    double v[6];
    for (int k = 0; k < 6; ++k)
      v[k] = wave_sum((t0 ? a.v0[k] : 0.0) + (t1 ? a.v1[k] : 0.0));
    const uint64_t hit = __ballot(lid == pick);
    const int c = hit ? __ffsll((long long)hit) - 1 : -1;
    if (lane == 0) {
      if (c >= 0) {
        for (int k = 0; k < 6; ++k) red[wave][c][k] = -v[k];
      } else {
        for (int k = 0; k < 6; ++k) atomic_add_f64(&ovf[6 * pick + k], -v[k]);
      }
    }
    if (t0) p0 = false;
    if (t1) p1 = false;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < cnt * 6; t += blockDim.x) {
    const int c = t / 6, k = t % 6;
    const double v = ((red[0][c][k] + red[1][c][k]) + red[2][c][k]) + red[3][c][k];
    part[((size_t)list[c] * g.maxent + ent[c]) * 6 + k] = v;
  }
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

// Momentum-exchange sums of node y for one particle q.
// Links j whose far node x = y + c_j q owns (bits of msk): with
// u_p(x) = u_p(y) + w x c_j and r(x) = r(y) + c_j their terms
// (-c_j + u_p(x)) f_j* and r(x) x (...) add up to
//   S_G = -M1 + u_p M0 + w x M1,   T_G = r x S_G + M1 x u_p + w K - M2 w
// with the partial moments M0 = sum f, M1 = sum c f, M2 = sum c c^T f,
// K = trace M2 over those links.  If q also owns y itself, its own terms
// sum_{j>=1} (c_j - u_p(y)) f_j* cancel the M0, M1 parts of every link in
// msk, leaving S = N1 - u_p N0 + w x M1 with the complement sums N0, N1 over
// the links NOT in msk (those leaving the particle).  The complement sums
// are small, so they are accumulated in the compute precision C of the
// populations (exact cancellation in the interior); the combination is FP64.
// Link masks (bits j = 1..18) for the exact rest-weight parts of the
// partial moments: sum over links j in a set G of a_j w_j with w_j = k_j / 36,
// k_j = 2 (axis links) or 1 (edge links) and a_j in {-1, 0, 1}.
struct LinkSel {
  unsigned axp, axm, edp, edm;   // axis / edge links with a_j = +1 / -1
};
template <typename A>
constexpr LinkSel link_sel(A a) {
  LinkSel L{0u, 0u, 0u, 0u};
  for (int j = 1; j < Q; ++j) {
    const bool axis = j < 7;
    const int v = a(j);
    if (v > 0) { if (axis) L.axp |= 1u << j; else L.edp |= 1u << j; }
    if (v < 0) { if (axis) L.axm |= 1u << j; else L.edm |= 1u << j; }
  }
  return L;
}
__device__ inline int wcount36(unsigned G, LinkSel L) {
  return 2 * (__popc(G & L.axp) - __popc(G & L.axm)) + (__popc(G & L.edp) - __popc(G & L.edm));
}

// Momentum-exchange sums of node y for one particle q.  f_j* = base_j + h_j
// with base_j = w_j for shifted storage (0 otherwise) and h_j the stored
// value.  The partial moments over a link set G are sum_G h (accumulated in
// the compute precision C of the storage: the deviations are small) plus the
// exact weight part (integer popcounts of G), combined in FP64.
template <bool SHIFTED, typename H>
__device__ inline void link_group_sums(H hval, unsigned msk, bool own,
                                       const double* up, const double* w,
                                       double* S, double* Tc) {
  using C = decltype(hval(1));
  C M0 = 0, M1x = 0, M1y = 0, M1z = 0, N0 = 0, N1x = 0, N1y = 0, N1z = 0;
  C Mxx = 0, Myy = 0, Mzz = 0, Mxy = 0, Mxz = 0, Myz = 0;
#pragma unroll
  for (int j = 1; j < Q; ++j) {
    const C hj = hval(j);
    const C fG = ((msk >> j) & 1u) ? hj : (C)0;
    const C fN = hj - fG;
    M0 += fG;
    N0 += fN;
    if (cx(j)) {
      M1x += cx(j) > 0 ? fG : -fG;
      N1x += cx(j) > 0 ? fN : -fN;
      Mxx += fG;
    }
    if (cy(j)) {
      M1y += cy(j) > 0 ? fG : -fG;
      N1y += cy(j) > 0 ? fN : -fN;
      Myy += fG;
    }
    if (cz(j)) {
      M1z += cz(j) > 0 ? fG : -fG;
      N1z += cz(j) > 0 ? fN : -fN;
      Mzz += fG;
    }
    if (cx(j) * cy(j)) Mxy += cx(j) * cy(j) > 0 ? fG : -fG;
    if (cx(j) * cz(j)) Mxz += cx(j) * cz(j) > 0 ? fG : -fG;
    if (cy(j) * cz(j)) Myz += cy(j) * cz(j) > 0 ? fG : -fG;
  }
  double m0 = M0, m1[3] = {M1x, M1y, M1z}, n0 = N0, n1[3] = {N1x, N1y, N1z};
  double xx = Mxx, yy = Myy, zz = Mzz, xy = Mxy, xz = Mxz, yz = Myz;
  if (SHIFTED) {
    constexpr LinkSel L0 = link_sel([](int) { return 1; });
    constexpr LinkSel LX = link_sel([](int j) { return cx(j); });
    constexpr LinkSel LY = link_sel([](int j) { return cy(j); });
    constexpr LinkSel LZ = link_sel([](int j) { return cz(j); });
    constexpr LinkSel LXX = link_sel([](int j) { return cx(j) * cx(j); });
    constexpr LinkSel LYY = link_sel([](int j) { return cy(j) * cy(j); });
    constexpr LinkSel LZZ = link_sel([](int j) { return cz(j) * cz(j); });
    constexpr LinkSel LXY = link_sel([](int j) { return cx(j) * cy(j); });
    constexpr LinkSel LXZ = link_sel([](int j) { return cx(j) * cz(j); });
    constexpr LinkSel LYZ = link_sel([](int j) { return cy(j) * cz(j); });
    const unsigned G = msk, N = ~msk & 0x7fffeu;
    const double r36 = 1.0 / 36.0;
    m0 += wcount36(G, L0) * r36;
    n0 += wcount36(N, L0) * r36;
    m1[0] += wcount36(G, LX) * r36;
    m1[1] += wcount36(G, LY) * r36;
    m1[2] += wcount36(G, LZ) * r36;
    n1[0] += wcount36(N, LX) * r36;
    n1[1] += wcount36(N, LY) * r36;
    n1[2] += wcount36(N, LZ) * r36;
    xx += wcount36(G, LXX) * r36;
    yy += wcount36(G, LYY) * r36;
    zz += wcount36(G, LZZ) * r36;
    xy += wcount36(G, LXY) * r36;
    xz += wcount36(G, LXZ) * r36;
    yz += wcount36(G, LYZ) * r36;
  }
  const double wxm[3] = {w[1] * m1[2] - w[2] * m1[1], w[2] * m1[0] - w[0] * m1[2],
                         w[0] * m1[1] - w[1] * m1[0]};
  if (own) {
    S[0] = n1[0] - up[0] * n0 + wxm[0];
    S[1] = n1[1] - up[1] * n0 + wxm[1];
    S[2] = n1[2] - up[2] * n0 + wxm[2];
  } else {
    S[0] = -m1[0] + up[0] * m0 + wxm[0];
    S[1] = -m1[1] + up[1] * m0 + wxm[1];
    S[2] = -m1[2] + up[2] * m0 + wxm[2];
  }
  const double K = (xx + yy) + zz;
  Tc[0] = (m1[1] * up[2] - m1[2] * up[1]) + w[0] * K - (xx * w[0] + xy * w[1] + xz * w[2]);
  Tc[1] = (m1[2] * up[0] - m1[0] * up[2]) + w[1] * K - (xy * w[0] + yy * w[1] + yz * w[2]);
  Tc[2] = (m1[0] * up[1] - m1[1] * up[0]) + w[2] * K - (xz * w[0] + yz * w[1] + zz * w[2]);
}

// link_group_sums for a node whose owner also owns all 18 link neighbours:
// the complement sums vanish, so S = w x M1 and T_c = M1 x u_p + w K - M2 w
// with the full moments of the 18 moving populations.  Their rest-weight
// parts are sum_j w_j c_j = 0 and sum_j w_j c_j c_j^T = I/3 (K = 1).
template <bool SHIFTED, typename H>
__device__ inline void interior_sums(H hval, const double* up, const double* w,
                                     double* S, double* Tc) {
  using C = decltype(hval(1));
  C M1x = 0, M1y = 0, M1z = 0, Mxx = 0, Myy = 0, Mzz = 0, Mxy = 0, Mxz = 0, Myz = 0;
#pragma unroll
  for (int j = 1; j < Q; ++j) {
    const C h = hval(j);
    if (cx(j)) { M1x += cx(j) > 0 ? h : -h; Mxx += h; }
    if (cy(j)) { M1y += cy(j) > 0 ? h : -h; Myy += h; }
    if (cz(j)) { M1z += cz(j) > 0 ? h : -h; Mzz += h; }
    if (cx(j) * cy(j)) Mxy += cx(j) * cy(j) > 0 ? h : -h;
    if (cx(j) * cz(j)) Mxz += cx(j) * cz(j) > 0 ? h : -h;
    if (cy(j) * cz(j)) Myz += cy(j) * cz(j) > 0 ? h : -h;
  }
  const double third = SHIFTED ? 1.0 / 3.0 : 0.0;
  const double m1[3] = {M1x, M1y, M1z};
  const double xx = (double)Mxx + third, yy = (double)Myy + third, zz = (double)Mzz + third;
  const double xy = Mxy, xz = Mxz, yz = Myz;
  S[0] = w[1] * m1[2] - w[2] * m1[1];
  S[1] = w[2] * m1[0] - w[0] * m1[2];
  S[2] = w[0] * m1[1] - w[1] * m1[0];
  const double K = (xx + yy) + zz;
  Tc[0] = (m1[1] * up[2] - m1[2] * up[1]) + w[0] * K - (xx * w[0] + xy * w[1] + xz * w[2]);
  Tc[1] = (m1[2] * up[0] - m1[0] * up[2]) + w[1] * K - (xy * w[0] + yy * w[1] + yz * w[2]);
  Tc[2] = (m1[0] * up[1] - m1[1] * up[0]) + w[2] * K - (xz * w[0] + yz * w[1] + zz * w[2]);
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

// Lattice directions packed as 2-bit fields (c + 1) per direction, so that a
// runtime direction index is decoded with shifts instead of a table lookup.
template <typename A>
constexpr uint64_t pack_dirs(A a) {
  uint64_t v = 0;
  for (int j = 0; j < Q; ++j) v |= (uint64_t)(a(j) + 1) << (2 * j);
  return v;
}
constexpr uint64_t CXP = pack_dirs([](int j) { return cx(j); });
constexpr uint64_t CYP = pack_dirs([](int j) { return cy(j); });
constexpr uint64_t CZP = pack_dirs([](int j) { return cz(j); });
__device__ inline int cdir(uint64_t pk, int j) { return (int)((pk >> (2 * j)) & 3u) - 1; }

// Momentum exchange of the compacted nodes of a lattice block: entry `slot`
// (one per thread, slot < total) holds the node's post-collision populations
// and its link masks.  For each particle that receives terms from the node
// the per-node force and torque (link_group_sums) are committed per
// wavefront.  Threads without an entry take part in the reductions only.
template <typename S, typename C>
__device__ void mea_compacted(C (*fl)[256], int (*meta)[2], int slot, int total,
                              const BlockNode& nd, const Particles& P,
                              const Geom& g, const Phys& ph,
                              const int* __restrict__ owner, int lid,
                              double (*row)[6], double* ovf) {
  const bool have = slot < total;
  int q = -1, q2 = -1, o = -1;
  unsigned msk = 0, msk2 = 0, rem = 0;
  int x = 0, y = 0;
  const int z = nd.z;
  bool inner = false;
  if (have) {
    const int t = meta[slot][0];
    x = nd.x - (int)(threadIdx.x % WAVE) + (t % WAVE);
    y = nd.y - nd.wave + t / WAVE;
    const int code = meta[slot][1];
    o = owner_id(code);
    inner = code >= 0 && (code & OWNER_INTERIOR);
  }
  if (inner) {
    // every link neighbour is owned by o
    q = o;
    msk = 0x7fffeu;
  } else if (have) {
    // owners of the 18 link neighbours (none beyond a wall)
    const Nbr nb = neighbours(g, x, y, z);
    int on[Q];
#pragma unroll
    for (int j = 1; j < Q; ++j) {
      // the neighbour index is clamped at walls, so the load is always valid
      const int v = owner[nb.off(cx(j), cy(j), cz(j))];
      on[j] = nb.beyond(cz(j)) ? -1 : owner_id(v);
    }
    // primary particle: the node's owner, else the largest neighbour owner
    // (any fixed choice would do); links of other particles stay in `rem`
    // and are grouped by the discovery step of the loop below
    int qmax = -1;
#pragma unroll
    for (int j = 1; j < Q; ++j) qmax = on[j] > qmax ? on[j] : qmax;
    q = o >= 0 ? o : qmax;
    unsigned owned = 0;
#pragma unroll
    for (int j = 1; j < Q; ++j) {
      owned |= on[j] >= 0 ? 1u << j : 0u;
      msk |= on[j] == q ? 1u << j : 0u;
    }
    msk &= owned;
    rem = owned & ~msk;
  }
  const bool perz = g.periodic_z != 0;
  const bool wall_m = !perz && z == 0, wall_p = !perz && z == g.nz - 1;
  // post-collision population of the entry: stored value h_j, full f_j*
  auto hval = [&](int j) -> C { return fl[j][slot]; };
  auto fval = [&](int j) -> double { return full_f<S>(fl[j][slot], j); };
  bool own = o >= 0;
  for (;;) {
    if (__ballot(q >= 0) == 0) break;
    // wavefronts made only of interior entries take the unmasked sums
    const bool all_inner = __ballot(q >= 0 && !(inner && own)) == 0;
    double Sv[3] = {0.0, 0.0, 0.0}, T[3] = {0.0, 0.0, 0.0};
    if (q >= 0) {
      const double Xq[3] = {P.X[3 * q], P.X[3 * q + 1], P.X[3 * q + 2]};
      const double Uq[3] = {P.U[3 * q], P.U[3 * q + 1], P.U[3 * q + 2]};
      const double w[3] = {P.W[3 * q], P.W[3 * q + 1], P.W[3 * q + 2]};
      const double r[3] = {minimg((double)x - Xq[0], (double)g.nx, true),
                           minimg((double)y - Xq[1], (double)g.ny, true),
                           minimg((double)z - Xq[2], (double)g.nz, perz)};
      const double up[3] = {Uq[0] + (w[1] * r[2] - w[2] * r[1]),
                            Uq[1] + (w[2] * r[0] - w[0] * r[2]),
                            Uq[2] + (w[0] * r[1] - w[1] * r[0])};
      double Sc[3], Tcc[3];
      if (all_inner)
        interior_sums<Store<S>::shifted>(hval, up, w, Sc, Tcc);
      else
        link_group_sums<Store<S>::shifted>(hval, msk, own, up, w, Sc, Tcc);
      if (own && (wall_m || wall_p)) {
        // links that bounce back from a wall return to y as f_opp(j)(y) of
        // the next step: term (c_j + u_p(y)) f_opp(j)(y)
#pragma unroll
        for (int j = 1; j < Q; ++j) {
          const int bw = cz(j) < 0 ? (wall_m ? 1 : 0) : (cz(j) > 0 ? (wall_p ? 2 : 0) : 0);
          if (!bw) continue;
          const double* uw = ph.wall_u[bw - 1];
          const double cuw = cx(j) * uw[0] + cy(j) * uw[1] + cz(j) * uw[2];
          const double fb = fval(j) - 6.0 * wgt(j) * cuw;
          Sc[0] += ((double)cx(j) + up[0]) * fb;
          Sc[1] += ((double)cy(j) + up[1]) * fb;
          Sc[2] += ((double)cz(j) + up[2]) * fb;
        }
      }
      Sv[0] = Sc[0];
      Sv[1] = Sc[1];
      Sv[2] = Sc[2];
      T[0] = Tcc[0] + (r[1] * Sc[2] - r[2] * Sc[1]);
      T[1] = Tcc[1] + (r[2] * Sc[0] - r[0] * Sc[2]);
      T[2] = Tcc[2] + (r[0] * Sc[1] - r[1] * Sc[0]);
    }
    commit_group(q, Sv, T, lid, row, ovf);
    // next particle
    q = q2;
    msk = msk2;
    own = false;
    q2 = -1;
    msk2 = 0;
    if (q < 0 && rem) {
      // owner of the first remaining link, and all remaining links it owns
      // (links beyond a wall never carry an owner, so z wraps only when
      // periodic)
      auto link_owner = [&](int j) -> int {
        int xj = x + cdir(CXP, j), yj = y + cdir(CYP, j), zj = z + cdir(CZP, j);
        xj = xj < 0 ? xj + g.nx : (xj >= g.nx ? xj - g.nx : xj);
        yj = yj < 0 ? yj + g.ny : (yj >= g.ny ? yj - g.ny : yj);
        zj = zj < 0 ? zj + g.nz : (zj >= g.nz ? zj - g.nz : zj);
        return owner_id(owner[xj + g.nx * (yj + g.ny * zj)]);
      };
      q = link_owner(__ffs(rem) - 1);
      for (unsigned b = rem; b; b &= b - 1) {
        const int j = __ffs(b) - 1;
        if (link_owner(j) == q) msk |= 1u << j;
      }
      rem &= ~msk;
    }
  }
}

// Four wavefronts per SIMD (the LDS footprint of the FP32 / binary16 forms
// allows four blocks per CU); the register allocation is held to 128 VGPRs
// for that, without spills.  The FP64 form is limited to two by its LDS.
template <typename S>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_lattice(const S* __restrict__ src,
                                                 S* __restrict__ dst,
                                                 const int* __restrict__ owner,
                                                 Particles P, Geom g, Phys ph,
                                                 Tiles tl, Counters* ctr) {
  using C = typename Store<S>::C;
  __shared__ double red[4][LCAP_MAX][6];
  __shared__ C fl[Q][256];
  __shared__ int meta[256][2];
  __shared__ int wcount[8];
  const BlockNode nd = block_node(g);
  const int x = nd.x, y = nd.y, z = nd.z;
  const bool valid = nd.valid;
  const long long tile = nd.block;
  const int n = (int)g.ncell;
  const bool perz = g.periodic_z != 0;
  const Nbr nb = neighbours(g, x, y, z);
  const int self = nb.off(0, 0, 0);

  C f[Q];
  int o = -1, ocode = -1;
  if (valid) {
    // one load per direction from a selected index (a branch per direction
    // would make the compiler wait for memory between the loads), then the
    // moving-wall term of the links that bounced back
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int src_i = nb.beyond(-cz(i)) ? opp(i) * n + self
                                          : i * n + nb.off(-cx(i), -cy(i), -cz(i));
      f[i] = Store<S>::ld(src, src_i);
    }
    ocode = owner[self];
    o = owner_id(ocode);
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
      d = sdf32(shape, (float)size, Ro, r0, r1, r2);
      B = weight32(d, (float)ph.eps);
    } else {
      d = sdf(shape, size, Ro, r0, r1, r2);
      B = weight(d, ph.eps);
    }
    const C w0 = (C)W0, w1 = (C)W1, w2 = (C)W2;
    upy[0] = (C)U0 + (w1 * r2 - w2 * r1);
    upy[1] = (C)U1 + (w2 * r0 - w0 * r2);
    upy[2] = (C)U2 + (w0 * r1 - w1 * r0);
  }
  const C du0 = B * (upy[0] - u0) + (C)ph.a_ext[0];
  const C du1 = B * (upy[1] - u1) + (C)ph.a_ext[1];
  const C du2 = B * (upy[2] - u2) + (C)ph.a_ext[2];
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

  // ---- momentum exchange of the next step --------------------------------
  // Compact the block's nodes that may send terms to some particle (owned,
  // or with a possibly owned link neighbour) into LDS, then let the four
  // wavefronts work through that list only.
  const int lane = threadIdx.x % WAVE;
  // Interior nodes (all link neighbours owned by the node's owner) go first,
  // so that wavefronts of the list are mostly of one kind.
  const bool need = valid && ocode != -1;
  const bool inner = need && ocode >= 0 && (ocode & OWNER_INTERIOR);
  const uint64_t in_mask = __ballot(inner);
  const uint64_t bd_mask = __ballot(need && !inner);
  if (lane == 0) {
    wcount[nd.wave] = __popcll(in_mask);
    wcount[4 + nd.wave] = __popcll(bd_mask);
  }
  __syncthreads();
  int base_in = 0, base_bd = 0, n_in = 0, total = 0;
  for (int w = 0; w < 4; ++w) {
    if (w < nd.wave) {
      base_in += wcount[w];
      base_bd += wcount[4 + w];
    }
    n_in += wcount[w];
    total += wcount[w] + wcount[4 + w];
  }
  if (need) {
    const uint64_t below = (1ull << lane) - 1ull;
    const int slot = inner ? base_in + __popcll(in_mask & below)
                           : n_in + base_bd + __popcll(bd_mask & below);
#pragma unroll
    for (int j = 1; j < Q; ++j) fl[j][slot] = f[j];
    meta[slot][0] = (int)threadIdx.x;
    meta[slot][1] = ocode;
  }
  int cnt = tl.lcount[tile];
  cnt = __builtin_amdgcn_readfirstlane(cnt < g.tile_cap ? cnt : g.tile_cap);
  const int* list = tl.llist + tile * g.tile_cap;
  const int* ent = tl.lent + tile * g.tile_cap;
  const int lid = lane < cnt ? list[lane] : -1;     // candidate list, one per lane
  for (int c = lane; c < cnt; c += WAVE)
    for (int k = 0; k < 6; ++k) red[nd.wave][c][k] = 0.0;
  __syncthreads();
  if (total > 0) mea_compacted<S, C>(fl, meta, (int)threadIdx.x, total, nd, P, g, ph,
                                  owner, lid, red[nd.wave], tl.ovf);
  store_block(red, list, ent, cnt, g, tl.part);
}

// Momentum exchange at the current state without collision: used once when
// a population field is set (initial condition) to supply the force of the
// first step.  Node x owned by o: S(x) = sum_i (c_i - u_p) f_i*(x) +
// (c_i + u_p) f_opp(i)(x), f_opp(i)(x) pulled from x + c_i.
template <typename S>
__global__ __launch_bounds__(256) void k_mea_only(const S* __restrict__ fs,
                                                  const int* __restrict__ owner,
                                                  Particles P, Geom g, Phys ph,
                                                  Tiles tl) {
  __shared__ double red[4][LCAP_MAX][6];
  const BlockNode nd = block_node(g);
  const int x = nd.x, y = nd.y, z = nd.z;
  const long long tile = nd.block;
  const size_t n = (size_t)g.ncell;
  const bool perz = g.periodic_z != 0;
  const size_t id = (size_t)x + (size_t)g.nx * ((size_t)y + (size_t)g.ny * z);
  const int o = nd.valid ? owner_id(owner[id]) : -1;
  Acc acc;
  acc.init();
  if (o >= 0) {
    const double* Xo = P.X + 3 * o;
    double r[3];
    r[0] = minimg((double)x - Xo[0], (double)g.nx, true);
    r[1] = minimg((double)y - Xo[1], (double)g.ny, true);
    r[2] = minimg((double)z - Xo[2], (double)g.nz, perz);
    const double* Uo = P.U + 3 * o;
    const double* Wo = P.W + 3 * o;
    double up[3] = {Uo[0] + (Wo[1] * r[2] - Wo[2] * r[1]),
                    Uo[1] + (Wo[2] * r[0] - Wo[0] * r[2]),
                    Uo[2] + (Wo[0] * r[1] - Wo[1] * r[0])};
    double s[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q; ++i) {
      const double fo = full_f<S>(Store<S>::ld(fs, (int)(i * n + id)), i);
      const int sx = (x + cx(i) + g.nx) % g.nx, sy = (y + cy(i) + g.ny) % g.ny;
      int sz = z + cz(i);
      double fi;
      if (!perz && (sz < 0 || sz >= g.nz)) {
        const double* uw = ph.wall_u[sz < 0 ? 0 : 1];
        const int k = opp(i);
        const double cu = cx(k) * uw[0] + cy(k) * uw[1] + cz(k) * uw[2];
        fi = fo + 6.0 * wgt(k) * cu;
      } else {
        sz = (sz + g.nz) % g.nz;
        const size_t sid = (size_t)sx + (size_t)g.nx * ((size_t)sy + (size_t)g.ny * sz);
        fi = full_f<S>(Store<S>::ld(fs, (int)(opp(i) * n + sid)), opp(i));
      }
      const double c3[3] = {(double)cx(i), (double)cy(i), (double)cz(i)};
      for (int k = 0; k < 3; ++k) s[k] += (c3[k] - up[k]) * fo + (c3[k] + up[k]) * fi;
    }
    double t[3] = {r[1] * s[2] - r[2] * s[1], r[2] * s[0] - r[0] * s[2],
                   r[0] * s[1] - r[1] * s[0]};
    acc.add(o, s, t, tl.ovf);
  }
  int cnt = tl.lcount[tile];
  cnt = __builtin_amdgcn_readfirstlane(cnt < g.tile_cap ? cnt : g.tile_cap);
  commit_block(acc, red, nd.wave, tl.llist + tile * g.tile_cap,
               tl.lent + tile * g.tile_cap, cnt, g, tl.part, tl.ovf);
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
  return (unsigned)((long long)g.ltx * g.lty * g.ltz);
}

template <typename S>
static void run_lattice(Ctx& c, const void* src, void* dst) {
  hipLaunchKernelGGL(k_lattice<S>, dim3(tile_blocks(c.g)), dim3(256), 0,
                     c.stream, (const S*)src, (S*)dst, c.owner, c.part, c.g,
                     c.ph, c.tl, c.counters);
}

hipError_t launch_lattice(Ctx& c, const void* src, void* dst) {
  DISPATCH(c, run_lattice, (c, src, dst));
  return hipGetLastError();
}

template <typename S>
static void run_mea(Ctx& c, const void* fs) {
  hipLaunchKernelGGL(k_mea_only<S>, dim3(tile_blocks(c.g)), dim3(256), 0,
                     c.stream, (const S*)fs, c.owner, c.part, c.g, c.ph, c.tl);
}

hipError_t launch_mea_only(Ctx& c, const void* fstar) {
  DISPATCH(c, run_mea, (c, fstar));
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
