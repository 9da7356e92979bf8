// Particle-to-fluid coupling map and rough contact detection (Sec. 3.2,
// Sec. 3.3.1-3.3.2), node-parallel.
//
// One wavefront per tile of TX x TY x TZ nodes.  The tile's candidate list is
// wave-uniform, so each candidate's record is fetched once per wavefront
// through scalar loads, and every lane evaluates that candidate's signed
// distance at its node.  Per node:
//   owner  = argmin over candidates with d < eps/2 of (d, id)
//   K(x)   = candidates with d - delta_c < sqrt(0.75), plus the walls whose
//            distance is below sqrt(0.75)
// Pairs are aggregated over the wavefront with ballots and min/max shuffles
// (count of flagged nodes, bounding box of their images in the frame of the
// lower-id particle) and then committed with one set of atomics per pair
// and tile into the open-addressing pair table.
#include "context.h"

namespace hlbm {

namespace {

__device__ int table_slot(PairTable t, uint64_t key, Counters* ctr) {
  const uint32_t mask = (uint32_t)t.cap - 1u;
  uint32_t h = pair_hash(key) & mask;
  for (int probe = 0; probe < t.cap; ++probe) {
    unsigned long long old = atomicCAS((unsigned long long*)&t.keys[h],
                                       (unsigned long long)EMPTY_KEY,
                                       (unsigned long long)key);
    if (old == EMPTY_KEY) list_slot(t, h);
    if (old == EMPTY_KEY || old == key) return (int)h;
    h = (h + 1u) & mask;
  }
  atomicOr(&ctr->pair_overflow, 1);
  return -1;
}

// Commit one pair seen by the lanes in `bal` with node images img.
__device__ void commit_pair(PairTable t, Counters* ctr, int a, int b,
                            uint64_t bal, bool pred, const int img[3]) {
  const int cnt = __popcll(bal);
  int lo[3], hi[3];
  for (int k = 0; k < 3; ++k) {
    lo[k] = wave_min_i(pred ? img[k] : 0x7fffffff);
    hi[k] = wave_max_i(pred ? img[k] : (int)0x80000000);
  }
  if (threadIdx.x % WAVE == 0) {
    const int s = table_slot(t, pair_key(a, b), ctr);
    if (s >= 0) {
      PairRec* r = &t.rec[s];
      r->a = a;
      r->b = b;
      const int old = atomicAdd(&r->count, cnt);
      if (old == 0) atomicAdd(&ctr->det_pairs, 1ull);
      for (int k = 0; k < 3; ++k) {
        atomicMin(&r->rlo[k], lo[k]);
        atomicMax(&r->rhi[k], hi[k]);
      }
      atomicAdd(&ctr->det_cells, (unsigned long long)cnt);
      atomicAdd(&ctr->total_cells, (unsigned long long)cnt);
    }
  }
}

template <bool POLY, bool ELL = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(POLY ? (ELL ? 4 : 5) : 8, 8))) void k_detect(Particles P, Geom g, Phys ph,
                                                Tiles tl, int* __restrict__ owner,
                                                PairTable tab, Counters* ctr) {
  const int lane = threadIdx.x % WAVE;
  // tile id, uniform over the wavefront (fewer than 2^31 tiles: the cell
  // count is bounded on the host)
  const unsigned ntiles = (unsigned)g.dtx * (unsigned)g.dty * (unsigned)g.dtz;
  const unsigned tile =
      blockIdx.x * 4u + (unsigned)__builtin_amdgcn_readfirstlane(threadIdx.x) / WAVE;
  if (tile >= ntiles) return;                     // whole wavefront exits
  const unsigned tyz = fdiv(tile, g.fdtx);
  const unsigned utz = fdiv(tyz, g.fdty);
  const int tx = (int)(tile - tyz * (unsigned)g.dtx);
  const int ty = (int)(tyz - utz * (unsigned)g.dty);
  const int tz = (int)utz;
  const int x = tx * DX + (lane % DX);
  const int y = ty * DY + (lane / DX) % DY;
  const int z = tz * DZ + lane / (DX * DY);
  const bool valid = x < g.nx && y < g.ny && z < g.nz;
  const bool perz = g.periodic_z != 0;
  const long long node = (long long)x + (long long)g.nx * ((long long)y + (long long)g.ny * z);

  // The tile's count and its first SPEC candidate ids in one round trip
  // (lane c < SPEC reads slot c of the list whatever the count; the rest of
  // a longer list follows); the loops take candidate c's id with readlane
  // and its FP32 screening record (centre, rotation) through scalar loads.
  constexpr int SPEC = 8;
  const int* list = tl.dlist + (size_t)tile * g.tile_cap;
  const int cnt_raw = tl.dcount[tile];
  int my_id = lane < (g.tile_cap < SPEC ? g.tile_cap : SPEC) ? list[lane] : 0;
  int cnt = __builtin_amdgcn_readfirstlane(cnt_raw);
  // this wavefront is the count's only reader: it resets a non-zero count
  // for the next binning as its last store (a store's completion would
  // delay the wavefront's next wait for a load)
  auto reset_count = [&]() {
    if (lane == 0) tl.dcount[tile] = 0;
  };
  cnt = cnt < g.tile_cap ? cnt : g.tile_cap;
  if (cnt == 0) {
    // no particle within reach of the tile: fluid, nothing flagged
    if (valid) owner[node] = -1;
    return;
  }
  if (cnt > SPEC) my_id = lane < cnt ? list[lane] : 0;   // (uniform)
  const bool have = lane < cnt;
  const int pid = have ? my_id : 0;
  const float fxf = (float)x, fyf = (float)y, fzf = (float)z;
  const float Lxf = (float)g.nx, Lyf = (float)g.ny, Lzf = (float)g.nz;
  const double own_t = 0.5 * ph.eps;              // owner:     d < eps/2

  // Pass 1, FP32: classify each candidate against both thresholds with a
  // bound tol on the FP32 error (the thresholds +- tol come with the
  // candidate's screening record).  Per lane: mask = candidates that may
  // be flagged (d < sqrt(0.75) + delta_c + tol; when eps/2 is the smaller
  // threshold, a superset of those that may own the node), nown = how many
  // may own it (d < eps/2 + tol) and bp
  // the last of them; near_own / any_dun = one of them lies within tol of
  // its threshold, so FP32 cannot decide.  Over the wavefront (ballots):
  // det_w = candidates some lane may flag.
  //
  // tol = 1e-3 + 1e-5 (|r|_1 + size) is taken with |r|_1 at its largest for
  // a node within reach of either threshold, sqrt 3 (R + 2) with R the
  // circumradius, so it is uniform per candidate: a node farther out has d
  // far above both thresholds, where the bound is not needed.
  int bp = -1, nown = 0;
  bool near_own = false, any_dun = false;
  uint64_t mask = 0, det_w = 0;
  // with a coupling band wider than the detection reach (eps/2 > sqrt(0.75)
  // + delta_c) a candidate may own a node it cannot flag: those are kept
  // apart for pass 2 (uniform branch)
  const bool own_wider = 0.5 * ph.eps > DETECT + ph.delta_c;
  uint64_t mown = 0;
  for (int c = 0; c < cnt; ++c) {
    const int p = __builtin_amdgcn_readlane(pid, c);
    // the whole record at once (uniform: scalar loads issued together),
    // and bookkeeping without short-circuit branches, so that one wait
    // serves the candidate
    const float* src = P.XR32 + SREC * p;
    float xr[19];
#pragma unroll
    for (int k = 0; k < 19; ++k) xr[k] = src[k];
    __builtin_amdgcn_sched_barrier(0);
    const int shape = __float_as_int(xr[18]);
    const float f0 = minimg_f(fxf - xr[0], Lxf, true);
    const float f1 = minimg_f(fyf - xr[1], Lyf, true);
    const float f2 = minimg_f(fzf - xr[2], Lzf, perz);
    // a polyhedron's plane lower bound beyond both thresholds ends its search
    const float d = sdf32_r<ELL>(shape, xr[17], xr + 3, f0, f1, f2, POLY ? P.poly : nullptr,
                                 xr[16], ELL ? src[19] : -1e30f);
    const bool may_own = valid & (d < xr[12]), may_det = valid & (d < xr[14]);
    nown += may_own ? 1 : 0;
    bp = may_own ? p : bp;
    near_own = near_own | (may_own & (d > xr[13]));
    any_dun = any_dun | (may_det & (d > xr[15]));
    mask |= may_det ? 1ull << c : 0ull;
    if (own_wider) mown |= may_own ? 1ull << c : 0ull;
    if (__ballot(may_det)) det_w |= 1ull << c;
  }
  // Pass 2, FP64, only for lanes pass 1 did not settle: the owner when two
  // or more candidates may own the node or one lies within tol of eps/2
  // (smallest (d, id) among the candidates with d < eps/2), and the
  // detection bits where one lies within tol of its threshold.  Such a lane
  // re-evaluates every candidate it may flag or that may own it, in the
  // oracle's exact expressions (for a candidate clearly inside or outside a
  // threshold the exact decision is the FP32 one).  The wavefront loops over
  // the union of those candidates.
  const bool own_open = near_own || nown > 1;
  const bool open = own_open || any_dun;
  uint64_t orm = det_w;
  if (__ballot(open)) {
    const double fx = (double)x, fy = (double)y, fz = (double)z;
    const double Lx = (double)g.nx, Ly = (double)g.ny, Lz = (double)g.nz;
    const uint64_t m1 = open ? (mask | mown) : 0ull;
    uint64_t todo = wave_or_u64(m1);
    double bd = 1.0e300;
    int ep = -1;
    while (todo) {
      const int c = __builtin_ctzll(todo);
      todo &= todo - 1;
      const int p = __builtin_amdgcn_readlane(pid, c);
      if ((m1 >> c) & 1ull) {
        const double X0 = P.X[3 * p], X1 = P.X[3 * p + 1], X2 = P.X[3 * p + 2];
        const double* R = P.R + 9 * p;
        const double r0 = minimg(fx - X0, Lx, true);
        const double r1 = minimg(fy - X1, Ly, true);
        const double r2 = minimg(fz - X2, Lz, perz);
        const double d = sdf_exact<ELL>(P.shape[p], P.size[p], R, r0, r1, r2, POLY ? P.poly : nullptr);
        if (own_open && d < own_t && (d < bd || (d == bd && p < ep))) {
          bd = d;
          ep = p;
        }
        if (any_dun) {
          if (d - ph.delta_c < DETECT) mask |= 1ull << c;
          else mask &= ~(1ull << c);
        }
      }
    }
    if (own_open) bp = ep;
    orm = wave_or_u64(mask);
  }
  // owner map: the owner's id, or -1
  if (valid) owner[node] = bp;

  // orm: candidates flagged at some node of the tile
  if (orm == 0) {
    reset_count();
    return;
  }
  const double fx = (double)x, fy = (double)y, fz = (double)z;
  const double Lx = (double)g.nx, Ly = (double)g.ny, Lz = (double)g.nz;
  const bool wbot = valid && !perz && (fz + 0.5 < DETECT);
  const bool wtop = valid && !perz && ((Lz - 0.5) - fz < DETECT);
  const bool anywall = __ballot(wbot || wtop) != 0;

  for (int i = 0; i < cnt; ++i) {
    if (!((orm >> i) & 1ull)) continue;
    const int pi = __builtin_amdgcn_readlane(pid, i);
    const bool in_i = (mask >> i) & 1ull;
    for (int j = i + 1; j < cnt; ++j) {
      if (!((orm >> j) & 1ull)) continue;
      const bool pred = in_i && ((mask >> j) & 1ull);
      const uint64_t bal = __ballot(pred);
      if (bal == 0) continue;
      const int pj = __builtin_amdgcn_readlane(pid, j);
      const int a = pi < pj ? pi : pj, b = pi < pj ? pj : pi;
      int img[3];
      img[0] = x + g.nx * image_shift(fx - P.X[3 * a], Lx, true);
      img[1] = y + g.ny * image_shift(fy - P.X[3 * a + 1], Ly, true);
      img[2] = z + g.nz * image_shift(fz - P.X[3 * a + 2], Lz, perz);
      commit_pair(tab, ctr, a, b, bal, pred, img);
    }
    if (anywall) {
      int img[3];
      img[0] = x + g.nx * image_shift(fx - P.X[3 * pi], Lx, true);
      img[1] = y + g.ny * image_shift(fy - P.X[3 * pi + 1], Ly, true);
      img[2] = z;
      const bool pb = in_i && wbot;
      const uint64_t bb = __ballot(pb);
      if (bb) commit_pair(tab, ctr, pi, -1, bb, pb, img);
      const bool pt = in_i && wtop;
      const uint64_t bt = __ballot(pt);
      if (bt) commit_pair(tab, ctr, pi, -2, bt, pt, img);
    }
  }
  reset_count();
}

}  // namespace

hipError_t launch_detect(Ctx& c, PairTable to) {
  const long long ntiles = (long long)c.g.dtx * c.g.dty * c.g.dtz;
  const unsigned blocks = (unsigned)((ntiles + 3) / 4);
  if (c.has_ellipsoid)
    hipLaunchKernelGGL((k_detect<true, true>), dim3(blocks), dim3(256), 0, c.stream, c.part,
                     c.g, c.ph, c.tl, c.owner, to, c.counters);
  else if (c.has_poly)
    hipLaunchKernelGGL(k_detect<true>, dim3(blocks), dim3(256), 0, c.stream, c.part,
                     c.g, c.ph, c.tl, c.owner, to, c.counters);
  else
    hipLaunchKernelGGL(k_detect<false>, dim3(blocks), dim3(256), 0, c.stream, c.part,
                     c.g, c.ph, c.tl, c.owner, to, c.counters);
  return hipGetLastError();
}

}  // namespace hlbm
