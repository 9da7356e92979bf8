// C ABI of the library (declared in include/hlbm.h): context management,
// validation on the host, the per-step launch sequence and read-out.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "context.h"

using namespace hlbm;

struct hlbm_ctx {
  Ctx c;
};

namespace {

hlbm_status fail(Ctx& c, hlbm_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(c.err, sizeof c.err, fmt, ap);
  va_end(ap);
  return st;
}

#define HIPCHECK(call)                                                      \
  do {                                                                      \
    hipError_t e_ = (call);                                                 \
    if (e_ != hipSuccess)                                                   \
      return fail(c, HLBM_E_DEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

size_t value_bytes(int prec) { return prec == HLBM_FP64 ? 8 : (prec == HLBM_FP32 ? 4 : 2); }

int next_pow2(long long v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

// reach beyond the body used for tile binning (must match k_particles)
double margin_of(const Ctx& c) {
  return fmax(0.5 * c.ph.eps, DETECT + c.ph.delta_c) + 0.25;
}

// circumradius of a particle of the given shape and size
double circumradius(const Ctx& c, int shape, double size) {
  if (shape >= POLY0) return size * c.poly_host[shape - POLY0].dev.rc;
  return shape == 1 ? 0.5 * size * sqrt(3.0) : size;
}

// Inverse body inertia tensor of a homogeneous polyhedron of density ratio
// dens and scale s: I_b = dens s^5 (tr(J) 1 - J) with J the unit-scale second
// moment about the centroid (eq. (3)), inverted by cofactors.
void poly_inverse_inertia(const Ctx::PolyHost& P, double s, double dens, double* Ii) {
  const double s2 = s * s, f = dens * s2 * s2 * s;
  const double tr = P.J[0] + P.J[4] + P.J[8];
  double I[9];
  for (int k = 0; k < 9; ++k) I[k] = f * ((k % 4 == 0 ? tr : 0.0) - P.J[k]);
  const double c0 = I[4] * I[8] - I[5] * I[7], c1 = I[5] * I[6] - I[3] * I[8],
               c2 = I[3] * I[7] - I[4] * I[6];
  const double det = I[0] * c0 + I[1] * c1 + I[2] * c2;
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

hlbm_status check_flags(Ctx& c) {
  Counters h;
  HIPCHECK(hipMemcpyAsync(&h, c.counters, sizeof h, hipMemcpyDeviceToHost, c.stream));
  HIPCHECK(hipStreamSynchronize(c.stream));
  if (h.tile_overflow)
    return fail(c, HLBM_E_CAPACITY,
                "tile candidate list overflow: more than tile_capacity=%d particles reach one 4x4x4 tile",
                c.g.tile_cap);
  if (h.pair_overflow)
    return fail(c, HLBM_E_CAPACITY, "contact pair table full (max_pairs=%d)",
                c.P.max_pairs);
  if (h.contact_overflow)
    return fail(c, HLBM_E_CAPACITY, "more than %d contacts on one particle in one step", MAXC);
  if (h.unstable)
    return fail(c, HLBM_E_UNSTABLE, "non-finite or non-positive density on the lattice");
  return HLBM_OK;
}

hlbm_status ensure_populations(Ctx& c) {
  if (c.fbuf[0]) return HLBM_OK;
  const size_t bytes = (size_t)Q * (size_t)c.g.ncell * c.bytes_per_value;
  for (int k = 0; k < 2; ++k) {
    hipError_t e = hipMalloc(&c.fbuf[k], bytes);
    if (e != hipSuccess)
      return fail(c, HLBM_E_NOMEM, "population buffer of %zu bytes: %s", bytes,
                  hipGetErrorString(e));
  }
  c.own_f = true;
  return HLBM_OK;
}

void drop_graphs(Ctx& c) {
  for (int k = 0; k < 4; ++k) {
    if (c.graph_ready[k]) hipGraphExecDestroy(c.gexec[k]);
    c.graph_ready[k] = false;
    for (int v = 0; v < 4; ++v) {
      if (c.graph_n_ready[k][v]) hipGraphExecDestroy(c.gexec_n[k][v]);
      c.graph_n_ready[k][v] = false;
      c.graph_n_run[k][v] = false;
    }
  }
}

// steps per multi-step graph (even: the population and table parities come
// back to their starting values)
constexpr int GRAPH_STEPS = 8;
// The first replay of a multi-step graph carries a one-time setup on the
// device (about 0.15 ms, measured; uploading the graph beforehand does not
// remove it).  A call of fewer steps than this replays only graphs that
// have run before and otherwise keeps to stream launches, which are as fast
// per step; a longer call replays (and so prepares) them.
constexpr int GRAPH_COLD_CALL = 64;

hlbm_status prepare_graphs(Ctx& c);

// Coupling and detection at the current particle state with the current
// populations as f*: ownership map, initial contact list, and the
// momentum-exchange force that moves the particles in the first step.
hlbm_status prologue(Ctx& c) {
  drop_graphs(c);
  const int p = c.tcur;
  const size_t nb = sizeof(double) * 3 * (c.np > 0 ? c.np : 1);
  HIPCHECK(launch_clear_step(c, c.tab[p], CLEAR_CONTACT | CLEAR_TILES, c.stream));
  HIPCHECK(hipMemsetAsync(c.Fh, 0, nb, c.stream));
  HIPCHECK(hipMemsetAsync(c.Th, 0, nb, c.stream));
  HIPCHECK(hipMemsetAsync(c.tl.ovf, 0, 2 * nb, c.stream));
  HIPCHECK(launch_particles(c, 0));
  HIPCHECK(launch_detect(c, c.tab[p]));
  HIPCHECK(launch_mea(c, c.fbuf[c.cur]));
  if (c.ph.bal_mode == 2) HIPCHECK(launch_balance(c, c.fbuf[c.cur], 1, c.stream));
  c.step = 0;
  c.fluid_ready = true;
  const hlbm_status st = check_flags(c);
  return st != HLBM_OK ? st : prepare_graphs(c);
}

// The launch sequence of one time step with population parity p (buffers
// p -> 1-p) starting from contact table t; the table parity flips once per
// sub-step.  ev (optional): 3 + 5 n_sub events recorded around the launches.
// Overlap (one sub-step only): the contact treatment of a step reads the
// particle state and the pair table the previous step's detection left, and
// nothing that the stream-collide or momentum-exchange pass writes, so it
// can run beside them on the side stream.  pre & PRE_DONE: this step's
// treatment already ran there (wait for it, then clear the tile counts the
// previous momentum-exchange pass read); pre & PRE_NEXT: after detection,
// start the next step's treatment on the side stream; pre & PRE_JOINED
// (with PRE_DONE): that treatment, and the balance sums, are complete in
// stream order already (a graph that started them joined them before its
// end), so no event wait.
constexpr int PRE_DONE = 1, PRE_NEXT = 2, PRE_JOINED = 4;
hipError_t enqueue_step(Ctx& c, int p, int t, hipEvent_t* ev, int pre) {
  hipError_t e;
  int m = 0;
  auto mark = [&]() -> hipError_t {
    return ev ? hipEventRecord(ev[m++], c.stream) : hipSuccess;
  };
  if ((e = mark())) return e;
  for (int s = 0; s < c.n_sub; ++s) {
    if (s == 0 && (pre & PRE_DONE)) {
      // (the tile counts need no clearing here: detection and the lattice
      // pass reset the counts they read)
      if (!(pre & PRE_JOINED) && (e = hipStreamWaitEvent(c.stream, c.ev_treat, 0))) return e;
      if ((e = mark())) return e;
    } else {
      if ((e = launch_clear_step(c, c.tab[1 - t], CLEAR_CONTACT | CLEAR_TILES, c.stream)))
        return e;
      if ((e = mark())) return e;
      if ((e = launch_treat(c, c.tab[t], c.stream))) return e;
    }
    if ((e = mark())) return e;
    // particle motion, tile binning and the contact carry-over in one launch
    // (the carry-over's timing slot stays empty)
    if ((e = launch_particles(c, s == 0 ? 1 : 2, &c.tab[t], &c.tab[1 - t]))) return e;
    if ((e = mark())) return e;
    if ((e = mark())) return e;
    if ((e = launch_detect(c, c.tab[1 - t]))) return e;
    if ((e = mark())) return e;
    t = 1 - t;
  }
  if (pre & PRE_NEXT) {
    // the next step's clear of its contact state and its treatment of
    // table t (the one detection just filled)
    if ((e = hipEventRecord(c.ev_det, c.stream))) return e;
    if ((e = hipStreamWaitEvent(c.side, c.ev_det, 0))) return e;
    if ((e = launch_clear_step(c, c.tab[1 - t], CLEAR_CONTACT, c.side))) return e;
    if ((e = launch_treat(c, c.tab[t], c.side))) return e;
    if ((e = hipEventRecord(c.ev_treat, c.side))) return e;
  }
  // the lattice pass also sums the momentum exchange of the next step (the
  // last timing slot stays empty).
  // The balance controller's sums feed only the next collision: with
  // PRE_NEXT they run on the side stream, beside the next step's
  // bookkeeping, particle motion and detection, and the next lattice pass
  // waits for them.
  const bool bal = c.ph.bal_mode == 2;
  if (bal && (pre & PRE_DONE) && !(pre & PRE_JOINED) &&
      (e = hipStreamWaitEvent(c.stream, c.ev_bal, 0)))
    return e;
  if ((e = launch_lattice(c, c.fbuf[p], c.fbuf[1 - p]))) return e;
  if (bal && (pre & PRE_NEXT)) {
    if ((e = hipEventRecord(c.ev_lat, c.stream))) return e;
    if ((e = hipStreamWaitEvent(c.side, c.ev_lat, 0))) return e;
    if ((e = launch_balance(c, nullptr, 0, c.side))) return e;
    if ((e = hipEventRecord(c.ev_bal, c.side))) return e;
  } else if (bal && (e = launch_balance(c, nullptr, 0, c.stream))) {
    return e;
  }
  if ((e = mark())) return e;
  return mark();
}

// Capture and instantiate the graph of one step (multi = false) or of
// GRAPH_STEPS steps with the overlapped contact treatment (multi = true,
// variant v as in Ctx::gexec_n) starting from population parity key / 2 and
// table parity key % 2.  Capturing runs nothing.
hlbm_status capture_graph(Ctx& c, int key, bool multi, int v = 0) {
  const int p = key / 2, t = key % 2;
  hipGraph_t gr;
  HIPCHECK(hipStreamBeginCapture(c.stream, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  if (multi) {
    const bool first_done = v & 1, last_next = v & 2;
    for (int j = 0; j < GRAPH_STEPS && e == hipSuccess; ++j) {
      const int pre = (j > 0 ? PRE_DONE : (first_done ? PRE_DONE | PRE_JOINED : 0)) |
                      (j + 1 < GRAPH_STEPS || last_next ? PRE_NEXT : 0);
      e = enqueue_step(c, p ^ (j & 1), t ^ (j & 1), nullptr, pre);
    }
    // the next step's treatment (and the balance sums after it) joined
    // back, so that the graph ends with nothing pending
    if (e == hipSuccess && last_next)
      e = hipStreamWaitEvent(c.stream, c.ph.bal_mode == 2 ? c.ev_bal : c.ev_treat, 0);
  } else {
    e = enqueue_step(c, p, t, nullptr, 0);
  }
  hipError_t e2 = hipStreamEndCapture(c.stream, &gr);
  if (e != hipSuccess || e2 != hipSuccess)
    return fail(c, HLBM_E_DEVICE, "graph capture: %s",
                hipGetErrorString(e != hipSuccess ? e : e2));
  hipGraphExec_t* slot = multi ? &c.gexec_n[key][v] : &c.gexec[key];
  e = hipGraphInstantiate(slot, gr, nullptr, nullptr, 0);
  hipGraphDestroy(gr);
  if (e != hipSuccess)
    return fail(c, HLBM_E_DEVICE, "graph instantiate: %s", hipGetErrorString(e));
  // upload now, so that the first replay does not carry it
  e = hipGraphUpload(*slot, c.stream);
  if (e != hipSuccess)
    return fail(c, HLBM_E_DEVICE, "graph upload: %s", hipGetErrorString(e));
  if (multi) c.graph_n_ready[key][v] = true;
  else c.graph_ready[key] = true;
  return HLBM_OK;
}

// Capture every graph that steps from the current parities can replay: the
// single-step graphs of the current (population, table) parity and of the
// one after a step, and, with one contact sub-step, the multi-step graphs of
// both (a multi-step graph returns to its starting parities).  A timed window
// of hlbm_step calls then launches graphs only.
hlbm_status prepare_graphs(Ctx& c) {
  if (!c.use_graph || !c.fluid_ready) return HLBM_OK;
  const int k0 = 2 * c.cur + c.tcur;
  const int k1 = 2 * (1 - c.cur) + ((c.n_sub & 1) ? 1 - c.tcur : c.tcur);
  for (int key : {k0, k1}) {
    if (!c.graph_ready[key]) {
      const hlbm_status st = capture_graph(c, key, false);
      if (st != HLBM_OK) return st;
    }
    for (int v = 0; v < 4 && c.n_sub == 1 && c.side; ++v)
      if (!c.graph_n_ready[key][v]) {
        const hlbm_status st = capture_graph(c, key, true, v);
        if (st != HLBM_OK) return st;
      }
  }
  return HLBM_OK;
}

// the step that the next hlbm_step would run, and the parities after it
hipError_t run_step(Ctx& c, hipEvent_t* ev, int pre = 0) {
  hipError_t e = enqueue_step(c, c.cur, c.tcur, ev, pre);
  c.cur = 1 - c.cur;
  c.tcur = (c.n_sub & 1) ? 1 - c.tcur : c.tcur;
  c.step++;
  return e;
}

void free_timing(Ctx& c) {
  if (c.tev) {
    for (int i = 0; i < c.tcap * c.ev_per_step; ++i) hipEventDestroy(c.tev[i]);
    delete[] c.tev;
  }
  c.tev = nullptr;
  c.tcap = c.tused = 0;
  c.timing = false;
}

void free_snapshot(Snapshot& s) {
  void* p[] = {s.f, s.part, s.tiles, s.psums, s.keys[0], s.keys[1], s.rec[0],
               s.rec[1], s.owner, s.ctr};
  for (void* q : p)
    if (q) hipFree(q);
  s = Snapshot();
}

void free_adjoint(Ctx& c) {
  Adjoint& a = c.adj;
  if (c.stream) hipStreamSynchronize(c.stream);
  for (int k = 0; k < a.nseg; ++k) free_snapshot(a.ck[k]);
  delete[] a.ck;
  free_snapshot(a.end);
  void* p[] = {a.fst, a.ost, a.pst, a.frc, a.gbar, a.hbar, a.pbar, a.sbar, a.work};
  for (void* q : p)
    if (q) hipFree(q);
  a = Adjoint();
}

void free_particles(Ctx& c) {
  free_adjoint(c);
  if (c.part_block) hipFree(c.part_block);
  c.part_block = nullptr;
  if (c.part_sums) hipFree(c.part_sums);
  c.part_sums = nullptr;
}

// ---- state snapshots (device-to-device copies on the context stream) ------
size_t pop_bytes(const Ctx& c) { return (size_t)Q * (size_t)c.g.ncell * c.bytes_per_value; }

hipError_t snapshot_alloc(Ctx& c, Snapshot& s) {
  hipError_t e;
  const size_t cap = (size_t)c.tab[0].cap;
  if ((e = hipMalloc(&s.f, pop_bytes(c)))) return e;
  if ((e = hipMalloc(&s.part, c.part_bytes))) return e;
  if ((e = hipMalloc(&s.tiles, c.tile_bytes))) return e;
  if ((e = hipMalloc(&s.psums, c.psum_bytes))) return e;
  for (int k = 0; k < 2; ++k) {
    if ((e = hipMalloc(&s.keys[k], key_block_bytes((int)cap)))) return e;
    if ((e = hipMalloc(&s.rec[k], sizeof(PairRec) * cap))) return e;
  }
  if ((e = hipMalloc(&s.owner, sizeof(int) * (size_t)c.g.ncell))) return e;
  return hipMalloc(&s.ctr, sizeof(Counters));
}

// dir = 0: context -> snapshot, 1: snapshot -> context
hipError_t snapshot_copy(Ctx& c, Snapshot& s, int dir) {
  hipError_t e;
  const size_t cap = (size_t)c.tab[0].cap;
  auto cp = [&](void* snap, void* live, size_t n) {
    return dir == 0 ? hipMemcpyAsync(snap, live, n, hipMemcpyDeviceToDevice, c.stream)
                    : hipMemcpyAsync(live, snap, n, hipMemcpyDeviceToDevice, c.stream);
  };
  if (dir == 0) {
    s.cur = c.cur;
    s.tcur = c.tcur;
    s.step = c.step;
  } else {
    c.cur = s.cur;
    c.tcur = s.tcur;
    c.step = s.step;
  }
  if ((e = cp(s.f, c.fbuf[c.cur], pop_bytes(c)))) return e;
  if ((e = cp(s.part, c.part_block, c.part_bytes))) return e;
  if ((e = cp(s.tiles, c.tile_block, c.tile_bytes))) return e;
  if ((e = cp(s.psums, c.part_sums, c.psum_bytes))) return e;
  for (int k = 0; k < 2; ++k) {
    if ((e = cp(s.keys[k], c.tab[k].keys, key_block_bytes((int)cap)))) return e;
    if ((e = cp(s.rec[k], c.tab[k].rec, sizeof(PairRec) * cap))) return e;
  }
  if ((e = cp(s.owner, c.owner, sizeof(int) * (size_t)c.g.ncell))) return e;
  return cp(s.ctr, c.counters, sizeof(Counters));
}

}  // namespace

extern "C" {

hlbm_status hlbm_create(const hlbm_params* params, void* stream, hlbm_ctx** out) {
  if (!out) return HLBM_E_ARG;
  *out = nullptr;
  if (!params) return HLBM_E_ARG;
  hlbm_ctx* h = new (std::nothrow) hlbm_ctx();
  if (!h) return HLBM_E_NOMEM;
  Ctx& c = h->c;
  c.P = *params;
  const hlbm_params& P = *params;
  auto bad = [&](const char* m) {
    fprintf(stderr, "hlbm_create: %s\n", m);
    delete h;
    return HLBM_E_ARG;
  };
  if (P.nx < 1 || P.ny < 1 || P.nz < 1 || P.nx > 4096 || P.ny > 4096 || P.nz > 4096)
    return bad("lattice size must be 1..4096 per axis");
  const long long ncell = (long long)P.nx * P.ny * P.nz;
  // population offsets i * ncell + node are 32-bit
  if (ncell * Q > (1LL << 31) - 1) return bad("more than (2^31-1)/19 nodes");
  if (!(P.tau > 0.5)) return bad("tau must exceed 1/2");
  if (P.n_c < 1 || P.n_c > 32) return bad("n_c must be 1..32");
  if (P.tile_capacity < 1 || P.tile_capacity > LCAP_MAX) return bad("tile_capacity must be 1..64");
  if (P.max_pairs < 1 || P.max_pairs > (1 << 24)) return bad("max_pairs must be 1..2^24");
  if (P.precision < 0 || P.precision > 2) return bad("precision must be 0, 1 or 2");
  if (P.n_sub < 1 || P.n_sub > 64) return bad("n_sub must be 1..64");
  if (P.balance < 0 || P.balance > 2) return bad("balance must be 0, 1 or 2");
  if (!(P.eps_b > 0.0) || !(P.enlarge >= 0.0)) return bad("eps_b > 0 and enlarge >= 0 required");
  if (!(P.young > 0.0) || !(P.u_k > 0.0) || !(P.mu_s > 0.0))
    return bad("young, u_k and mu_s must be positive");

  c.precision = P.precision;
  c.bytes_per_value = value_bytes(P.precision);
  c.g.nx = P.nx; c.g.ny = P.ny; c.g.nz = P.nz;
  c.g.periodic_z = P.periodic_z ? 1 : 0;
  c.g.dtx = (P.nx + DX - 1) / DX;
  c.g.dty = (P.ny + DY - 1) / DY;
  c.g.dtz = (P.nz + DZ - 1) / DZ;
  c.g.ltx = (P.nx + LX - 1) / LX;
  c.g.lty = (P.ny + LY - 1) / LY;
  c.g.ltz = (P.nz + LZ - 1) / LZ;
  c.g.fdtx = make_fastdiv((unsigned)c.g.dtx);
  c.g.fdty = make_fastdiv((unsigned)c.g.dty);
  c.g.fltx = make_fastdiv((unsigned)c.g.ltx);
  c.g.flty = make_fastdiv((unsigned)c.g.lty);
  c.g.tile_cap = P.tile_capacity;
  c.g.ncell = ncell;
  c.ph.tau = P.tau;
  c.ph.omega = 1.0 / P.tau;
  for (int w = 0; w < 2; ++w)
    for (int k = 0; k < 3; ++k) c.ph.wall_u[w][k] = P.wall_velocity[w][k];
  for (int k = 0; k < 3; ++k) {
    c.ph.gravity[k] = P.gravity[k];
    c.ph.a_ext[k] = P.fluid_accel[k];
  }
  c.ph.eps = P.eps_b;
  c.ph.eps_h32 = (float)(0.5 * P.eps_b);
  c.ph.eps_q32 = (float)(0.25 / P.eps_b);
  c.ph.delta_c = P.enlarge;
  c.ph.n_c = P.n_c;
  // eq. (5) with both bodies (and walls) of the same material
  c.ph.estar = 1.0 / ((1.0 - P.poisson * P.poisson) / P.young +
                      (1.0 - P.poisson * P.poisson) / P.young);
  c.ph.restitution = P.restitution;
  c.ph.mu_s = P.mu_s;
  c.ph.mu_k = P.mu_k;
  c.ph.u_k = P.u_k;
  c.n_sub = P.n_sub;
  c.ph.dt_sub = 1.0 / (double)P.n_sub;
  c.ev_per_step = 3 + 5 * P.n_sub;

  if (stream) {
    c.stream = (hipStream_t)stream;
    c.own_stream = false;
  } else {
    if (hipStreamCreate(&c.stream) != hipSuccess) {
      delete h;
      return HLBM_E_DEVICE;
    }
    c.own_stream = true;
  }
  {
    // the fixed staging array of hlbm_read_coupling_noalloc on this device
    const hipError_t e = noalloc_scratch(&c.fixed_scratch);
    if (e != hipSuccess) {
      fprintf(stderr, "hlbm_create: staging array address: %s\n", hipGetErrorString(e));
      if (c.own_stream) hipStreamDestroy(c.stream);
      delete h;
      return HLBM_E_DEVICE;
    }
  }
  if (hipStreamCreate(&c.side) != hipSuccess ||
      hipEventCreateWithFlags(&c.ev_det, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c.ev_treat, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c.ev_lat, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c.ev_bal, hipEventDisableTiming) != hipSuccess) {
    if (c.side) hipStreamDestroy(c.side);
    if (c.ev_det) hipEventDestroy(c.ev_det);
    if (c.ev_treat) hipEventDestroy(c.ev_treat);
    if (c.ev_lat) hipEventDestroy(c.ev_lat);
    if (c.ev_bal) hipEventDestroy(c.ev_bal);
    if (c.own_stream) hipStreamDestroy(c.stream);
    delete h;
    return HLBM_E_DEVICE;
  }
  const long long ndt = (long long)c.g.dtx * c.g.dty * c.g.dtz;
  const long long nlt = (long long)c.g.ltx * c.g.lty * c.g.ltz;
  const int cap = next_pow2(2LL * P.max_pairs);
  const size_t tbytes = sizeof(int) * (size_t)(ndt + nlt) * (1 + P.tile_capacity) +
                        sizeof(int) * (size_t)nlt * P.tile_capacity;
  c.tile_bytes = tbytes;
  bool okm = hipMalloc(&c.owner, sizeof(int) * ncell) == hipSuccess &&
             hipMalloc(&c.tile_block, tbytes) == hipSuccess &&
             hipMalloc(&c.counters, sizeof(Counters)) == hipSuccess &&
             hipMalloc(&c.scratch, sizeof(double) * ncell) == hipSuccess &&
             (P.balance != 2 ||
              hipMalloc(&c.bal_part, sizeof(double) * 4 * ((size_t)nlt + BAL_PARTS)) == hipSuccess);
  for (int k = 0; k < 2 && okm; ++k) {
    c.tab[k].cap = cap;
    okm = hipMalloc(&c.tab[k].keys, key_block_bytes(cap)) == hipSuccess &&
          hipMalloc(&c.tab[k].rec, sizeof(PairRec) * cap) == hipSuccess;
    if (okm) set_table_views(c.tab[k]);
  }
  if (!okm) {
    *out = h;
    hlbm_destroy(h);
    *out = nullptr;
    return HLBM_E_NOMEM;
  }
  {
    int* t = (int*)c.tile_block;
    c.tl.dcount = t; t += ndt;
    c.tl.dlist = t; t += ndt * P.tile_capacity;
    c.tl.lcount = t; t += nlt;
    c.tl.llist = t; t += nlt * P.tile_capacity;
    c.tl.lent = t;
  }
  hipMemsetAsync(c.counters, 0, sizeof(Counters), c.stream);
  hipMemsetAsync(c.owner, 0xff, sizeof(int) * ncell, c.stream);
  for (int k = 0; k < 2; ++k) {
    hipMemsetAsync(c.tab[k].list, 0, sizeof(int) * ((size_t)cap + 2), c.stream);
    launch_clear_step(c, c.tab[k], CLEAR_ALL_SLOTS, c.stream);
  }
  if (hipStreamSynchronize(c.stream) != hipSuccess) {
    hlbm_destroy(h);
    return HLBM_E_DEVICE;
  }
  *out = h;
  return HLBM_OK;
}

hlbm_status hlbm_bind_populations(hlbm_ctx* h, void* a, void* b, size_t bytes) {
  if (!h) return HLBM_E_ARG;
  Ctx& c = h->c;
  const size_t need = (size_t)Q * (size_t)c.g.ncell * c.bytes_per_value;
  if (!a || !b || a == b || bytes < need)
    return fail(c, HLBM_E_ARG, "bind_populations: need two distinct buffers of %zu bytes", need);
  if (c.fbuf[0] && c.own_f) {
    hipFree(c.fbuf[0]);
    hipFree(c.fbuf[1]);
  }
  c.fbuf[0] = a;
  c.fbuf[1] = b;
  c.own_f = false;
  c.fluid_ready = false;
  drop_graphs(c);
  return HLBM_OK;
}

// A convex polyhedron type from vertices and faces (counter-clockwise seen
// from outside).  Checks a closed, consistently oriented surface (each
// directed edge once, its reverse once, V - E + F = 2), positive volume,
// planar faces and convexity; re-centres the solid at its centroid
// (tetrahedra of each face fan with the origin) and takes its second moment
// J = int p p^T dV there (per tetrahedron V/20 (sum v v^T + (sum v)(sum v)^T)).
// Face planes: Newell's normal through the face's vertex mean.
hlbm_status hlbm_define_polyhedron(hlbm_ctx* h, int type, int nv, const double* v,
                                   int nf, const int* fsize, const int* fidx) {
  if (!h) return HLBM_E_ARG;
  Ctx& c = h->c;
  if (c.particles_ready)
    return fail(c, HLBM_E_STATE, "define polyhedra before init_particles");
  if (type < 0 || type >= MAXPOLY) return fail(c, HLBM_E_ARG, "polyhedron type must be 0..%d", MAXPOLY - 1);
  if (!v || !fsize || !fidx || nv < 4 || nv > PV || nf < 4 || nf > PF)
    return fail(c, HLBM_E_ARG, "polyhedron: 4..%d vertices and 4..%d faces", PV, PF);
  Ctx::PolyHost P;
  PolyDev& D = P.dev;
  memset(&D, 0, sizeof D);
  D.nv = nv;
  D.nf = nf;
  for (int i = 0; i < nv; ++i)
    for (int k = 0; k < 3; ++k) {
      if (!isfinite(v[3 * i + k])) return fail(c, HLBM_E_ARG, "polyhedron: non-finite vertex");
      D.v[i][k] = v[3 * i + k];
    }
  int m = 0;
  for (int f = 0; f < nf; ++f) {
    if (fsize[f] < 3) return fail(c, HLBM_E_ARG, "polyhedron: face %d has fewer than 3 vertices", f);
    D.fs[f] = m;
    for (int j = 0; j < fsize[f]; ++j) {
      if (m >= PFV) return fail(c, HLBM_E_ARG, "polyhedron: more than %d face-vertex entries", PFV);
      if (fidx[m] < 0 || fidx[m] >= nv) return fail(c, HLBM_E_ARG, "polyhedron: vertex index out of range");
      D.fv[m] = fidx[m];
      ++m;
    }
  }
  D.fs[nf] = m;
  auto fvert = [&](int f, int j) {
    const int cnt = D.fs[f + 1] - D.fs[f];
    return D.fv[D.fs[f] + j % cnt];
  };
  for (int f = 0; f < nf; ++f) {
    const int cnt = D.fs[f + 1] - D.fs[f];
    for (int j = 0; j < cnt; ++j) {
      const int a = fvert(f, j), b = fvert(f, j + 1);
      if (a == b) return fail(c, HLBM_E_ARG, "polyhedron: repeated vertex in face %d", f);
      int same = 0, rev = 0;
      for (int g = 0; g < nf; ++g) {
        const int cg = D.fs[g + 1] - D.fs[g];
        for (int t = 0; t < cg; ++t) {
          const int x = fvert(g, t), y = fvert(g, t + 1);
          same += (x == a && y == b);
          rev += (x == b && y == a);
        }
      }
      if (same != 1 || rev != 1)
        return fail(c, HLBM_E_ARG, "polyhedron: surface not closed or not consistently oriented");
      if (a < b) {
        if (D.ne >= PE) return fail(c, HLBM_E_ARG, "polyhedron: more than %d edges", PE);
        D.e[D.ne][0] = a;
        D.e[D.ne][1] = b;
        ++D.ne;
      }
    }
  }
  if (nv - D.ne + nf != 2) return fail(c, HLBM_E_ARG, "polyhedron: Euler characteristic is not 2");
  // signed volume of the tetrahedron (0, a, b, d)
  auto tet = [](const double* a, const double* b, const double* d) {
    return (a[0] * (b[1] * d[2] - b[2] * d[1]) - a[1] * (b[0] * d[2] - b[2] * d[0]) +
            a[2] * (b[0] * d[1] - b[1] * d[0])) / 6.0;
  };
  double vol = 0.0, cen[3] = {0.0, 0.0, 0.0};
  for (int f = 0; f < nf; ++f) {
    const int cnt = D.fs[f + 1] - D.fs[f];
    const double* a = D.v[fvert(f, 0)];
    for (int j = 1; j + 1 < cnt; ++j) {
      const double *b = D.v[fvert(f, j)], *d = D.v[fvert(f, j + 1)];
      const double t = tet(a, b, d);
      vol += t;
      for (int k = 0; k < 3; ++k) cen[k] += t * (a[k] + b[k] + d[k]) / 4.0;
    }
  }
  if (!(vol > 0.0))
    return fail(c, HLBM_E_ARG, "polyhedron: faces must run counter-clockwise seen from outside");
  for (int k = 0; k < 3; ++k) cen[k] /= vol;
  for (int i = 0; i < nv; ++i)
    for (int k = 0; k < 3; ++k) D.v[i][k] -= cen[k];
  P.vol = vol;
  for (int f = 0; f < nf; ++f) {
    const int cnt = D.fs[f + 1] - D.fs[f];
    const double* a = D.v[fvert(f, 0)];
    for (int j = 1; j + 1 < cnt; ++j) {
      const double *b = D.v[fvert(f, j)], *d = D.v[fvert(f, j + 1)];
      const double t = tet(a, b, d);
      for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q) {
          const double sv = a[r] + b[r] + d[r], sw = a[q] + b[q] + d[q];
          P.J[3 * r + q] += t / 20.0 * (a[r] * a[q] + b[r] * b[q] + d[r] * d[q] + sv * sw);
        }
    }
  }
  double scale = 0.0;
  for (int i = 0; i < nv; ++i) {
    const double r = sqrt(D.v[i][0] * D.v[i][0] + D.v[i][1] * D.v[i][1] + D.v[i][2] * D.v[i][2]);
    scale = r > scale ? r : scale;
  }
  D.rc = scale;
  for (int f = 0; f < nf; ++f) {
    const int cnt = D.fs[f + 1] - D.fs[f];
    double nn[3] = {0.0, 0.0, 0.0}, mean[3] = {0.0, 0.0, 0.0};
    for (int j = 0; j < cnt; ++j) {
      const double *a = D.v[fvert(f, j)], *b = D.v[fvert(f, j + 1)];
      nn[0] += (a[1] - b[1]) * (a[2] + b[2]);
      nn[1] += (a[2] - b[2]) * (a[0] + b[0]);
      nn[2] += (a[0] - b[0]) * (a[1] + b[1]);
      for (int k = 0; k < 3; ++k) mean[k] += a[k] / cnt;
    }
    const double len = sqrt(nn[0] * nn[0] + nn[1] * nn[1] + nn[2] * nn[2]);
    if (!(len > 0.0)) return fail(c, HLBM_E_ARG, "polyhedron: degenerate face %d", f);
    for (int k = 0; k < 3; ++k) D.pl[f][k] = nn[k] / len;
    D.pl[f][3] = D.pl[f][0] * mean[0] + D.pl[f][1] * mean[1] + D.pl[f][2] * mean[2];
    for (int i = 0; i < nv; ++i) {
      const double sd = D.pl[f][0] * D.v[i][0] + D.pl[f][1] * D.v[i][1] + D.pl[f][2] * D.v[i][2] - D.pl[f][3];
      if (sd > 1e-9 * scale)
        return fail(c, HLBM_E_ARG, "polyhedron: not convex (a vertex lies outside face %d)", f);
    }
    for (int j = 0; j < cnt; ++j) {
      const double* a = D.v[fvert(f, j)];
      const double sd = D.pl[f][0] * a[0] + D.pl[f][1] * a[1] + D.pl[f][2] * a[2] - D.pl[f][3];
      if (fabs(sd) > 1e-9 * scale) return fail(c, HLBM_E_ARG, "polyhedron: face %d not planar", f);
    }
  }
  for (int i = 0; i < nv; ++i)
    for (int k = 0; k < 3; ++k) D.vf[i][k] = (float)D.v[i][k];
  for (int f = 0; f < nf; ++f)
    for (int k = 0; k < 4; ++k) D.plf[f][k] = (float)D.pl[f][k];
  for (int f = 0; f < nf; ++f) {
    const int cnt = D.fs[f + 1] - D.fs[f];
    for (int j = 0; j < cnt; ++j) {
      const int m = D.fs[f] + j;
      const double* a = D.v[fvert(f, j)];
      const double* b = D.v[fvert(f, j + 1)];
      for (int k = 0; k < 3; ++k) D.ed[m][k] = b[k] - a[k];
      const double ee = D.ed[m][0] * D.ed[m][0] + D.ed[m][1] * D.ed[m][1] + D.ed[m][2] * D.ed[m][2];
      if (!(sqrt(ee) > 1e-9 * scale))
        return fail(c, HLBM_E_ARG, "polyhedron: zero-length edge in face %d", f);
      D.ed[m][3] = 1.0 / ee;
      const double* n = D.pl[f];
      const double* e = D.ed[m];
      D.sd[m][0] = n[1] * e[2] - n[2] * e[1];
      D.sd[m][1] = n[2] * e[0] - n[0] * e[2];
      D.sd[m][2] = n[0] * e[1] - n[1] * e[0];
      D.sd[m][3] = D.sd[m][0] * a[0] + D.sd[m][1] * a[1] + D.sd[m][2] * a[2];
      for (int k = 0; k < 4; ++k) {
        D.ef[m][k] = (float)D.ed[m][k];
        D.sf[m][k] = (float)D.sd[m][k];
      }
    }
  }
  P.ok = true;
  if (!c.poly_dev) HIPCHECK(hipMalloc(&c.poly_dev, sizeof(PolyDev) * MAXPOLY));
  HIPCHECK(hipMemcpy(c.poly_dev + type, &D, sizeof(PolyDev), hipMemcpyHostToDevice));
  c.poly_host[type] = P;
  return HLBM_OK;
}

hlbm_status hlbm_define_ellipsoid(hlbm_ctx* h, int type, double a, double b, double cc) {
  if (!h) return HLBM_E_ARG;
  Ctx& c = h->c;
  if (c.particles_ready)
    return fail(c, HLBM_E_STATE, "define ellipsoids before init_particles");
  if (type < 0 || type >= MAXPOLY) return fail(c, HLBM_E_ARG, "ellipsoid type must be 0..%d", MAXPOLY - 1);
  if (!(a > 0.0 && b > 0.0 && cc > 0.0) || !isfinite(a) || !isfinite(b) || !isfinite(cc))
    return fail(c, HLBM_E_ARG, "ellipsoid semi-axes must be positive and finite");
  Ctx::PolyHost P;
  PolyDev& D = P.dev;
  memset(&D, 0, sizeof D);
  D.kind = KIND_ELLIPSOID;
  D.v[0][0] = a;
  D.v[0][1] = b;
  D.v[0][2] = cc;
  for (int k = 0; k < 3; ++k) D.vf[0][k] = (float)D.v[0][k];
  D.rc = a > b ? (a > cc ? a : cc) : (b > cc ? b : cc);
  // unit-scale volume and second moment about the centre: V = 4 pi abc / 3,
  // int p_k^2 dV = V e_k^2 / 5
  P.vol = 4.0 / 3.0 * PI * a * b * cc;
  P.J[0] = P.vol * a * a / 5.0;
  P.J[4] = P.vol * b * b / 5.0;
  P.J[8] = P.vol * cc * cc / 5.0;
  P.ok = true;
  if (!c.poly_dev) HIPCHECK(hipMalloc(&c.poly_dev, sizeof(PolyDev) * MAXPOLY));
  HIPCHECK(hipMemcpy(c.poly_dev + type, &D, sizeof(PolyDev), hipMemcpyHostToDevice));
  c.poly_host[type] = P;
  return HLBM_OK;
}

hlbm_status hlbm_init_particles(hlbm_ctx* h, int n, const int* shape, const double* size,
                                const double* density, const double* X, const double* q,
                                const double* U, const double* omega) {
  if (!h) return HLBM_E_ARG;
  Ctx& c = h->c;
  if (n < 0 || (n > 0 && (!shape || !size || !density || !X || !q || !U || !omega)))
    return fail(c, HLBM_E_ARG, "init_particles: bad arguments");
  const double L[3] = {(double)c.g.nx, (double)c.g.ny, (double)c.g.nz};
  const bool per[3] = {true, true, c.g.periodic_z != 0};
  const double margin = margin_of(c);
  std::vector<int> sh(n > 0 ? n : 1);
  std::vector<double> sz(n), ds(n), vol(n), mass(n), inert(n), Xh(3 * n), qh(4 * n),
      Uh(3 * n), Wh(3 * n), iinv(9 * (size_t)n, 0.0);
  for (int i = 0; i < n; ++i) {
    const bool poly = shape[i] >= POLY0 && shape[i] < POLY0 + MAXPOLY &&
                      c.poly_host[shape[i] - POLY0].ok;
    if (!poly && (shape[i] < 0 || shape[i] > 2))
      return fail(c, HLBM_E_ARG,
                  "particle %d: shape must be 0 (sphere), 1 (cube), 2 (octahedron) or a "
                  "defined polyhedron type or ellipsoid type (3 + k)", i);
    if (!(size[i] > 0.0) || !(density[i] > 0.0) || !isfinite(size[i]) || !isfinite(density[i]))
      return fail(c, HLBM_E_ARG, "particle %d: size and density must be positive", i);
    sh[i] = shape[i];
    sz[i] = size[i];
    ds[i] = density[i];
    const double circ = circumradius(c, shape[i], size[i]);
    for (int k = 0; k < 3; ++k) {
      if (per[k] && !(L[k] > 2.0 * (circ + margin)))
        return fail(c, HLBM_E_ARG,
                    "particle %d: periodic axis %d (%g nodes) must exceed twice the reach %g",
                    i, k, L[k], circ + margin);
      double x = X[3 * i + k];
      if (!isfinite(x) || !isfinite(U[3 * i + k]) || !isfinite(omega[3 * i + k]))
        return fail(c, HLBM_E_ARG, "particle %d: non-finite state", i);
      if (per[k]) {
        x = fmod(x, L[k]);
        if (x < 0.0) x += L[k];
        if (x >= L[k]) x -= L[k];
      }
      Xh[3 * i + k] = x;
      Uh[3 * i + k] = U[3 * i + k];
      Wh[3 * i + k] = omega[3 * i + k];
    }
    double nq = 0.0;
    for (int k = 0; k < 4; ++k) nq += q[4 * i + k] * q[4 * i + k];
    if (!(nq > 0.0) || !isfinite(nq))
      return fail(c, HLBM_E_ARG, "particle %d: zero or non-finite quaternion", i);
    for (int k = 0; k < 4; ++k) qh[4 * i + k] = q[4 * i + k];
    if (fabs(nq - 1.0) > 1e-12)
      for (int k = 0; k < 4; ++k) qh[4 * i + k] = q[4 * i + k] / sqrt(nq);
    // volume and (isotropic) moment of inertia: sphere 4 pi a^3 / 3,
    // 2 m a^2 / 5; cube a^3, m a^2 / 6; octahedron 4 a^3 / 3, m a^2 / 5
    // polyhedra: V = V_1 s^3 and the inverse inertia tensor (eq. (3))
    const double a = size[i];
    if (poly) {
      const Ctx::PolyHost& P = c.poly_host[shape[i] - POLY0];
      vol[i] = P.vol * a * a * a;
      mass[i] = density[i] * vol[i];
      inert[i] = 1.0;
      poly_inverse_inertia(P, a, density[i], &iinv[9 * (size_t)i]);
      continue;
    }
    vol[i] = shape[i] == 0 ? 4.0 / 3.0 * PI * a * a * a
                           : (shape[i] == 2 ? 4.0 / 3.0 * a * a * a : a * a * a);
    mass[i] = density[i] * vol[i];
    inert[i] = shape[i] == 0 ? 0.4 * mass[i] * a * a
                             : (shape[i] == 2 ? 0.2 * mass[i] * a * a : mass[i] * a * a / 6.0);
  }
  drop_graphs(c);
  free_particles(c);
  const size_t nn = n > 0 ? n : 1;
  // layout of the one particle allocation (doubles, then ints)
  // 5 scalars, X 3, q 4, U 3, W 3, R 9, Fh 3, Th 3, Fc 3, Tc 3
  // (plus SREC / 2 doubles' room for the FP32 screening record), inverse
  // inertia 9; the FP32 kinematic record (LREC / 2 doubles) first, so that
  // its 16-byte rows are aligned
  const size_t nd = nn * (LREC / 2 + 5 + 3 + 4 + 3 + 3 + 9 + 3 + 3 + 3 + 3 + SREC / 2 + 9);
  const size_t bytes = nd * sizeof(double) + nn * sizeof(int);
  c.part_bytes = bytes;
  HIPCHECK(hipMalloc(&c.part_block, bytes));
  HIPCHECK(hipMemsetAsync(c.part_block, 0, bytes, c.stream));
  double* d = (double*)c.part_block;
  auto take = [&](size_t k) { double* p = d; d += k * nn; return p; };
  c.part.LR32 = (float*)take(LREC / 2);
  double* dsz = take(1); double* dds = take(1); double* dvol = take(1);
  double* dmass = take(1); double* dinert = take(1);
  c.part.X = take(3); c.part.q = take(4); c.part.U = take(3); c.part.W = take(3);
  c.part.R = take(9);
  c.part.XR32 = (float*)take(SREC / 2);
  c.Fh = take(3); c.Th = take(3);
  c.Fc = take(3); c.Tc = take(3);
  double* diinv = take(9);
  c.part.Iinv = diinv;
  c.part.poly = c.poly_dev;
  c.has_poly = false;
  c.has_ellipsoid = false;
  for (int i = 0; i < n; ++i) {
    c.has_poly = c.has_poly || sh[i] >= POLY0;
    c.has_ellipsoid = c.has_ellipsoid ||
                      (sh[i] >= POLY0 && c.poly_host[sh[i] - POLY0].dev.kind == KIND_ELLIPSOID);
  }
  int* dsh = (int*)d;
  c.part.n = n;
  c.part.shape = dsh; c.part.size = dsz; c.part.dens = dds; c.part.vol = dvol;
  c.part.mass = dmass; c.part.inert = dinert;
  c.np = n;
  // partial-sum slots: the lattice blocks one particle's reach box can touch
  {
    double emax = 0.0;
    for (int i = 0; i < n; ++i)
      emax = fmax(emax, circumradius(c, sh[i], sz[i]));
    // the lattice-block reach (see k_particles): eps/2 + 1 node beyond the body
    const double span = 2.0 * (emax + fmax(margin, 0.5 * c.ph.eps + 1.25)) + 3.0;
    const int ts[3] = {LX, LY, LZ}, nt[3] = {c.g.ltx, c.g.lty, c.g.ltz};
    const int nn3[3] = {c.g.nx, c.g.ny, c.g.nz};
    const bool per3[3] = {true, true, c.g.periodic_z != 0};
    long long me = 1;
    for (int k = 0; k < 3; ++k) {
      // an interval of length span touches at most span / ts + 2 whole
      // blocks; on a periodic axis whose last block is partial, the
      // interval can wrap through that short block and touch one more
      long long m = (long long)(span / ts[k]) + 2 + (per3[k] && nn3[k] % ts[k] ? 1 : 0);
      if (m > nt[k]) m = nt[k];
      me *= m;
    }
    c.g.maxent = (int)me;
    // doubles: part (nn x me x 6), ovf (nn x 6), cval (nn x MAXC x 6);
    // ints: nent (nn), ccount (nn), ckey (nn x MAXC)
    const size_t nd = nn * 6 * (size_t)me + nn * 6 + nn * MAXC * 6;
    const size_t ni = nn + nn + nn * MAXC;
    const size_t pb = sizeof(double) * nd + sizeof(int) * ni;
    c.psum_bytes = pb;
    HIPCHECK(hipMalloc(&c.part_sums, pb));
    HIPCHECK(hipMemsetAsync(c.part_sums, 0, pb, c.stream));
    double* pd = (double*)c.part_sums;
    c.tl.part = pd;
    c.tl.ovf = pd + nn * 6 * (size_t)me;
    c.tl.cval = c.tl.ovf + nn * 6;
    c.tl.nent = (int*)(c.tl.cval + nn * MAXC * 6);
    c.tl.ccount = c.tl.nent + nn;
    c.tl.ckey = c.tl.ccount + nn;
  }
  if (n > 0) {
    HIPCHECK(hipMemcpyAsync(dsh, sh.data(), sizeof(int) * n, hipMemcpyHostToDevice, c.stream));
    HIPCHECK(hipMemcpyAsync(dsz, sz.data(), sizeof(double) * n, hipMemcpyHostToDevice, c.stream));
    HIPCHECK(hipMemcpyAsync(dds, ds.data(), sizeof(double) * n, hipMemcpyHostToDevice, c.stream));
    HIPCHECK(hipMemcpyAsync(dvol, vol.data(), sizeof(double) * n, hipMemcpyHostToDevice, c.stream));
    HIPCHECK(hipMemcpyAsync(dmass, mass.data(), sizeof(double) * n, hipMemcpyHostToDevice, c.stream));
    HIPCHECK(hipMemcpyAsync(dinert, inert.data(), sizeof(double) * n, hipMemcpyHostToDevice, c.stream));
    HIPCHECK(hipMemcpyAsync(diinv, iinv.data(), sizeof(double) * 9 * n, hipMemcpyHostToDevice, c.stream));
    HIPCHECK(hipMemcpyAsync(c.part.X, Xh.data(), sizeof(double) * 3 * n, hipMemcpyHostToDevice, c.stream));
    HIPCHECK(hipMemcpyAsync(c.part.q, qh.data(), sizeof(double) * 4 * n, hipMemcpyHostToDevice, c.stream));
    HIPCHECK(hipMemcpyAsync(c.part.U, Uh.data(), sizeof(double) * 3 * n, hipMemcpyHostToDevice, c.stream));
    HIPCHECK(hipMemcpyAsync(c.part.W, Wh.data(), sizeof(double) * 3 * n, hipMemcpyHostToDevice, c.stream));
  }
  // zero-net-flow balance force (Sec. 5.1) on fully periodic boxes: mode 1
  // cancels the particles' net weight here; mode 2 is a controller on the
  // lattice momentum, updated on the device after every collision
  for (int k = 0; k < 3; ++k) c.ph.a_ext[k] = c.P.fluid_accel[k];
  c.ph.bal_mode = (c.P.balance == 2 && c.g.periodic_z) ? 2 : 0;
  if (c.P.balance == 1 && c.g.periodic_z) {
    double tot[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < n; ++i)
      for (int k = 0; k < 3; ++k) tot[k] += (ds[i] - 1.0) * vol[i] * c.P.gravity[k];
    for (int k = 0; k < 3; ++k) c.ph.a_ext[k] -= tot[k] / (double)c.g.ncell;
  }
  HIPCHECK(hipStreamSynchronize(c.stream));
  c.particles_ready = true;
  c.fluid_ready = false;
  return HLBM_OK;
}

hlbm_status hlbm_init_fluid_equilibrium(hlbm_ctx* h, double rho, const double u[3]) {
  if (!h) return HLBM_E_ARG;
  Ctx& c = h->c;
  if (!c.particles_ready)
    return fail(c, HLBM_E_STATE, "init_particles must precede the fluid initialisation");
  if (!(rho > 0.0) || !u) return fail(c, HLBM_E_ARG, "rho must be positive");
  hlbm_status st = ensure_populations(c);
  if (st) return st;
  c.cur = 0;
  c.tcur = 0;
  HIPCHECK(launch_fill_equilibrium(c, c.fbuf[c.cur], rho, u));
  return prologue(c);
}

hlbm_status hlbm_set_populations(hlbm_ctx* h, const double* f) {
  if (!h) return HLBM_E_ARG;
  Ctx& c = h->c;
  if (!c.particles_ready)
    return fail(c, HLBM_E_STATE, "init_particles must precede the fluid initialisation");
  if (!f) return fail(c, HLBM_E_ARG, "null population array");
  hlbm_status st = ensure_populations(c);
  if (st) return st;
  c.cur = 0;
  c.tcur = 0;
  const size_t n = (size_t)c.g.ncell;
  for (int i = 0; i < Q; ++i) {
    HIPCHECK(hipMemcpyAsync(c.scratch, f + (size_t)i * n, sizeof(double) * n,
                            hipMemcpyHostToDevice, c.stream));
    HIPCHECK(launch_store_direction(c, c.fbuf[c.cur], i, c.scratch));
  }
  return prologue(c);
}

hlbm_status hlbm_step(hlbm_ctx* h, int nsteps) {
  if (!h) return HLBM_E_ARG;
  Ctx& c = h->c;
  if (!c.fluid_ready) return fail(c, HLBM_E_STATE, "initialise particles and fluid first");
  if (nsteps < 0) return fail(c, HLBM_E_ARG, "nsteps must be >= 0");
  // With graphs on (one contact sub-step), a call of two or more steps
  // replays multi-step graphs first and runs the remaining steps as stream
  // launches; the contact treatment overlaps the previous lattice pass at
  // every step but the call's first, across graph boundaries too (a graph
  // followed by more steps starts the next step's treatment and joins it
  // before it ends; the step after it takes it as done).  The same bits as
  // stream launches.  A single step replays its single-step graph.
  const bool chain = c.use_graph && !c.timing && c.n_sub == 1 && c.side != nullptr;
  bool after_graph = false;   // the previous step ended a graph that joined
  bool streamed = false;      // a stream launch of this call may have left the
                              // next step's treatment pending: no graph after it
  for (int s = 0; s < nsteps; ++s) {
    const int key = 2 * c.cur + c.tcur;
    const int v = (s > 0 ? 1 : 0) | (s + GRAPH_STEPS < nsteps ? 2 : 0);
    if (c.timing) {
      if (c.tused >= c.tcap)
        return fail(c, HLBM_E_CAPACITY, "timing window of %d steps is full", c.tcap);
      HIPCHECK(run_step(c, c.tev + (size_t)c.tused * c.ev_per_step));
      c.tused++;
    } else if (chain && !streamed && nsteps - s >= GRAPH_STEPS &&
               (c.graph_n_run[key][v] || nsteps >= GRAPH_COLD_CALL)) {
      if (!c.graph_n_ready[key][v]) {
        const hlbm_status st = capture_graph(c, key, true, v);
        if (st != HLBM_OK) return st;
      }
      HIPCHECK(hipGraphLaunch(c.gexec_n[key][v], c.stream));
      c.graph_n_run[key][v] = true;
      c.step += GRAPH_STEPS;
      s += GRAPH_STEPS - 1;
      after_graph = true;
    } else if (c.use_graph && !(chain && nsteps >= 2)) {
      if (!c.graph_ready[key]) {
        const hlbm_status st = capture_graph(c, key, false);
        if (st != HLBM_OK) return st;
      }
      HIPCHECK(hipGraphLaunch(c.gexec[key], c.stream));
      c.cur = 1 - c.cur;
      c.tcur = (c.n_sub & 1) ? 1 - c.tcur : c.tcur;
      c.step++;
    } else {
      // steps of one call after the first overlap their contact treatment
      // with the previous step's lattice passes; the last step leaves none
      // pending, so the state after the call is that of whole steps
      const bool ovl = c.n_sub == 1 && c.side != nullptr;
      const int pre = (ovl && s > 0 ? PRE_DONE | (after_graph ? PRE_JOINED : 0) : 0) |
                      (ovl && s + 1 < nsteps ? PRE_NEXT : 0);
      after_graph = false;
      streamed = true;
      const hipError_t e = run_step(c, nullptr, pre);
      if (e != hipSuccess) {
        // whatever the side stream has queued is joined before reporting
        if (ovl) (void)hipStreamWaitEvent(c.stream, c.ev_treat, 0);
        return fail(c, HLBM_E_DEVICE, "step: %s", hipGetErrorString(e));
      }
    }
  }
  return HLBM_OK;
}

hlbm_status hlbm_use_graph(hlbm_ctx* h, int on) {
  if (!h) return HLBM_E_ARG;
  h->c.use_graph = on != 0;
  return prepare_graphs(h->c);
}

hlbm_status hlbm_timing_begin(hlbm_ctx* h, int max_steps) {
  if (!h) return HLBM_E_ARG;
  Ctx& c = h->c;
  if (max_steps < 1 || max_steps > 100000)
    return fail(c, HLBM_E_ARG, "timing window must be 1..100000 steps");
  free_timing(c);
  c.tev = new (std::nothrow) hipEvent_t[(size_t)max_steps * c.ev_per_step];
  if (!c.tev) return fail(c, HLBM_E_NOMEM, "timing events");
  for (int i = 0; i < max_steps * c.ev_per_step; ++i) {
    hipError_t e = hipEventCreate(&c.tev[i]);
    if (e != hipSuccess) {
      c.tcap = i / c.ev_per_step;
      free_timing(c);
      return fail(c, HLBM_E_DEVICE, "hipEventCreate: %s", hipGetErrorString(e));
    }
  }
  c.tcap = max_steps;
  c.tused = 0;
  c.timing = true;
  return HLBM_OK;
}

hlbm_status hlbm_timing_end(hlbm_ctx* h, double* kernel_ms, int* nsteps) {
  if (!h || !kernel_ms || !nsteps) return HLBM_E_ARG;
  Ctx& c = h->c;
  if (!c.timing) return fail(c, HLBM_E_STATE, "timing_begin was not called");
  HIPCHECK(hipStreamSynchronize(c.stream));
  for (int k = 0; k < NKERN; ++k) kernel_ms[k] = 0.0;
  // events: start, then per sub-step after clear, treat, particles, keep,
  // detect; then after the lattice pass and after the momentum exchange
  for (int s = 0; s < c.tused; ++s) {
    hipEvent_t* ev = c.tev + (size_t)s * c.ev_per_step;
    for (int sub = 0; sub < c.n_sub; ++sub)
      for (int k = 0; k < 5; ++k) {
        float ms = 0.0f;
        HIPCHECK(hipEventElapsedTime(&ms, ev[5 * sub + k], ev[5 * sub + k + 1]));
        kernel_ms[k] += (double)ms;
      }
    for (int k = 0; k < 2; ++k) {
      float ms = 0.0f;
      HIPCHECK(hipEventElapsedTime(&ms, ev[c.ev_per_step - 3 + k], ev[c.ev_per_step - 2 + k]));
      kernel_ms[5 + k] += (double)ms;
    }
  }
  *nsteps = c.tused;
  free_timing(c);
  return check_flags(c);
}

hlbm_status hlbm_sync(hlbm_ctx* h) {
  if (!h) return HLBM_E_ARG;
  Ctx& c = h->c;
  HIPCHECK(hipStreamSynchronize(c.stream));
  return check_flags(c);
}

hlbm_status hlbm_read_forces(hlbm_ctx* h, double* Fh, double* Th, double* Fc, double* Tc) {
  if (!h) return HLBM_E_ARG;
  Ctx& c = h->c;
  if (!c.particles_ready) return fail(c, HLBM_E_STATE, "no particles");
  const size_t b = sizeof(double) * 3 * c.np;
  if (c.np > 0) {
    if (Fh) HIPCHECK(hipMemcpyAsync(Fh, c.Fh, b, hipMemcpyDeviceToHost, c.stream));
    if (Th) HIPCHECK(hipMemcpyAsync(Th, c.Th, b, hipMemcpyDeviceToHost, c.stream));
    if (Fc) HIPCHECK(hipMemcpyAsync(Fc, c.Fc, b, hipMemcpyDeviceToHost, c.stream));
    if (Tc) HIPCHECK(hipMemcpyAsync(Tc, c.Tc, b, hipMemcpyDeviceToHost, c.stream));
  }
  HIPCHECK(hipStreamSynchronize(c.stream));
  return check_flags(c);
}

hlbm_status hlbm_read_particles(hlbm_ctx* h, double* X, double* q, double* U, double* W) {
  if (!h) return HLBM_E_ARG;
  Ctx& c = h->c;
  if (!c.particles_ready) return fail(c, HLBM_E_STATE, "no particles");
  const size_t b = sizeof(double) * c.np;
  if (c.np > 0) {
    if (X) HIPCHECK(hipMemcpyAsync(X, c.part.X, 3 * b, hipMemcpyDeviceToHost, c.stream));
    if (q) HIPCHECK(hipMemcpyAsync(q, c.part.q, 4 * b, hipMemcpyDeviceToHost, c.stream));
    if (U) HIPCHECK(hipMemcpyAsync(U, c.part.U, 3 * b, hipMemcpyDeviceToHost, c.stream));
    if (W) HIPCHECK(hipMemcpyAsync(W, c.part.W, 3 * b, hipMemcpyDeviceToHost, c.stream));
  }
  HIPCHECK(hipStreamSynchronize(c.stream));
  return check_flags(c);
}

hlbm_status hlbm_read_contacts(hlbm_ctx* h, int capacity, hlbm_contact* out, int* n_out) {
  if (!h || !n_out || capacity < 0 || (capacity > 0 && !out)) return HLBM_E_ARG;
  Ctx& c = h->c;
  if (!c.fluid_ready) return fail(c, HLBM_E_STATE, "not initialised");
  const PairTable& t = c.tab[c.tcur];
  std::vector<uint64_t> keys(t.cap);
  std::vector<PairRec> rec(t.cap);
  HIPCHECK(hipMemcpyAsync(keys.data(), t.keys, sizeof(uint64_t) * t.cap,
                          hipMemcpyDeviceToHost, c.stream));
  HIPCHECK(hipMemcpyAsync(rec.data(), t.rec, sizeof(PairRec) * t.cap,
                          hipMemcpyDeviceToHost, c.stream));
  HIPCHECK(hipStreamSynchronize(c.stream));
  std::vector<std::pair<uint64_t, int>> order;
  for (int s = 0; s < t.cap; ++s)
    if (keys[s] != EMPTY_KEY) order.push_back({keys[s], s});
  std::sort(order.begin(), order.end());
  *n_out = (int)order.size();
  const int m = std::min(capacity, (int)order.size());
  for (int i = 0; i < m; ++i) {
    const PairRec& r = rec[order[i].second];
    hlbm_contact& o = out[i];
    memset(&o, 0, sizeof o);
    o.a = r.a;
    o.b = r.b;
    o.count = r.count;
    for (int k = 0; k < 3; ++k) {
      o.rlo[k] = r.count > 0 ? r.rlo[k] : 0;
      o.rhi[k] = r.count > 0 ? r.rhi[k] : 0;
      o.lo[k] = r.carried ? r.lo[k] : (double)r.rlo[k] - 0.5;
      o.hi[k] = r.carried ? r.hi[k] : (double)r.rhi[k] + 0.5;
      o.centroid[k] = r.centroid[k];
      o.normal[k] = r.normal[k];
      o.force_a[k] = r.force_a[k];
      o.force_b[k] = -r.force_a[k];
    }
    o.carried = r.carried;
    o.established = r.established;
    o.damping = r.damping;
    o.age = r.age;
    o.n_in = r.n_in;
    o.volume = r.volume;
    o.depth = r.depth;
    o.fn = r.fn;
  }
  return check_flags(c);
}

hlbm_status hlbm_read_fields(hlbm_ctx* h, double* rho, double* u, int* owner) {
  if (!h) return HLBM_E_ARG;
  Ctx& c = h->c;
  if (!c.fluid_ready) return fail(c, HLBM_E_STATE, "not initialised");
  const size_t n = (size_t)c.g.ncell;
  if (rho) {
    HIPCHECK(launch_moment(c, c.fbuf[c.cur], -1, c.scratch));
    HIPCHECK(hipMemcpyAsync(rho, c.scratch, sizeof(double) * n, hipMemcpyDeviceToHost, c.stream));
    HIPCHECK(hipStreamSynchronize(c.stream));
  }
  if (u) {
    std::vector<double> tmp(n);
    for (int k = 0; k < 3; ++k) {
      HIPCHECK(launch_moment(c, c.fbuf[c.cur], k, c.scratch));
      HIPCHECK(hipMemcpyAsync(tmp.data(), c.scratch, sizeof(double) * n,
                              hipMemcpyDeviceToHost, c.stream));
      HIPCHECK(hipStreamSynchronize(c.stream));
      for (size_t i = 0; i < n; ++i) u[3 * i + k] = tmp[i];
    }
  }
  if (owner)
    HIPCHECK(hipMemcpyAsync(owner, c.owner, sizeof(int) * n, hipMemcpyDeviceToHost, c.stream));
  HIPCHECK(hipStreamSynchronize(c.stream));
  return check_flags(c);
}

hlbm_status hlbm_read_coupling(hlbm_ctx* h, double* B, double* up) {
  if (!h) return HLBM_E_ARG;
  Ctx& c = h->c;
  if (!c.fluid_ready) return fail(c, HLBM_E_STATE, "not initialised");
  const size_t n = (size_t)c.g.ncell;
  std::vector<double> tmp(up ? n : 0);
  if (B) {
    HIPCHECK(launch_coupling_field(c, -1, c.scratch, 1));
    HIPCHECK(hipMemcpyAsync(B, c.scratch, sizeof(double) * n, hipMemcpyDeviceToHost, c.stream));
  }
  if (up) {
    for (int k = 0; k < 3; ++k) {
      HIPCHECK(launch_coupling_field(c, k, c.scratch, 1));
      HIPCHECK(hipMemcpyAsync(tmp.data(), c.scratch, sizeof(double) * n,
                              hipMemcpyDeviceToHost, c.stream));
      HIPCHECK(hipStreamSynchronize(c.stream));
      for (size_t i = 0; i < n; ++i) up[3 * i + k] = tmp[i];
    }
  }
  HIPCHECK(hipStreamSynchronize(c.stream));
  return check_flags(c);
}

// The same read-out staged through the fixed device array: no allocation
// on the device or the host (u_p is written interleaved by the kernel, so
// both copies land in the caller's arrays as they are).
hlbm_status hlbm_read_coupling_noalloc(hlbm_ctx* h, double* B, double* up) {
  if (!h) return HLBM_E_ARG;
  Ctx& c = h->c;
  if (!c.fluid_ready) return fail(c, HLBM_E_STATE, "not initialised");
  const long long n = c.g.ncell;
  if (n > NOALLOC_MAX_CELLS)
    return fail(c, HLBM_E_ARG, "hlbm_read_coupling_noalloc: %lld nodes exceed the %lld of "
                "its fixed staging array", n, NOALLOC_MAX_CELLS);
  if (!c.fixed_scratch) return fail(c, HLBM_E_STATE, "no staging array address");
  double* sB = c.fixed_scratch;
  double* sU = c.fixed_scratch + n;
  if (B) {
    HIPCHECK(launch_coupling_field(c, -1, sB, 1));
    HIPCHECK(hipMemcpyAsync(B, sB, sizeof(double) * n, hipMemcpyDeviceToHost, c.stream));
  }
  if (up) {
    for (int k = 0; k < 3; ++k) HIPCHECK(launch_coupling_field(c, k, sU + k, 3));
    HIPCHECK(hipMemcpyAsync(up, sU, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, c.stream));
  }
  HIPCHECK(hipStreamSynchronize(c.stream));
  return check_flags(c);
}

hlbm_status hlbm_read_populations(hlbm_ctx* h, double* f) {
  if (!h || !f) return HLBM_E_ARG;
  Ctx& c = h->c;
  if (!c.fluid_ready) return fail(c, HLBM_E_STATE, "not initialised");
  const size_t n = (size_t)c.g.ncell;
  for (int i = 0; i < Q; ++i) {
    HIPCHECK(launch_load_direction(c, c.fbuf[c.cur], i, c.scratch));
    HIPCHECK(hipMemcpyAsync(f + (size_t)i * n, c.scratch, sizeof(double) * n,
                            hipMemcpyDeviceToHost, c.stream));
    HIPCHECK(hipStreamSynchronize(c.stream));
  }
  return check_flags(c);
}

hlbm_status hlbm_counters(hlbm_ctx* h, long long* pairs, long long* cells,
                          long long* total_cells, long long* steps,
                          long long* samples) {
  if (!h) return HLBM_E_ARG;
  Ctx& c = h->c;
  Counters k;
  HIPCHECK(hipMemcpyAsync(&k, c.counters, sizeof k, hipMemcpyDeviceToHost, c.stream));
  HIPCHECK(hipStreamSynchronize(c.stream));
  if (pairs) *pairs = (long long)k.det_pairs;
  if (cells) *cells = (long long)k.det_cells;
  if (total_cells) *total_cells = (long long)k.total_cells;
  if (steps) *steps = c.step;
  if (samples) *samples = (long long)k.samples;
  return HLBM_OK;
}

void* hlbm_stream(const hlbm_ctx* h) { return h ? (void*)h->c.stream : nullptr; }

hlbm_status hlbm_fluid_acceleration(hlbm_ctx* h, double a[3]) {
  if (!h || !a) return HLBM_E_ARG;
  Ctx& c = h->c;
  if (c.ph.bal_mode == 2) {
    if (!c.fluid_ready) return fail(c, HLBM_E_STATE, "initialise particles and fluid first");
    Counters k;
    HIPCHECK(hipMemcpyAsync(&k, c.counters, sizeof k, hipMemcpyDeviceToHost, c.stream));
    HIPCHECK(hipStreamSynchronize(c.stream));
    for (int i = 0; i < 3; ++i) a[i] = k.bal_a[i];
    return HLBM_OK;
  }
  for (int k = 0; k < 3; ++k) a[k] = c.ph.a_ext[k];
  return HLBM_OK;
}

// ---- host state blob: header, then the device blocks in a fixed order ----
namespace {
struct StateHeader {
  char magic[8];
  int version, precision, nx, ny, nz, np, cur, tcur, cap, n_sub;
  long long step;
  unsigned long long f_bytes, part_bytes, tile_bytes, psum_bytes, tab_bytes,
      owner_bytes;
};
const char kMagic[8] = {'H', 'L', 'B', 'M', 'S', 'T', 'A', '1'};

unsigned long long state_bytes(const Ctx& c) {
  const size_t cap = (size_t)c.tab[0].cap;
  return sizeof(StateHeader) + pop_bytes(c) + c.part_bytes + c.tile_bytes +
         c.psum_bytes + 2 * (key_block_bytes((int)cap) + cap * sizeof(PairRec)) +
         sizeof(int) * (size_t)c.g.ncell + sizeof(Counters);
}
}  // namespace

hlbm_status hlbm_get_state(hlbm_ctx* h, void* blob, size_t* bytes) {
  if (!h || !bytes) return HLBM_E_ARG;
  Ctx& c = h->c;
  if (!c.fluid_ready) return fail(c, HLBM_E_STATE, "initialise particles and fluid first");
  const unsigned long long need = state_bytes(c);
  if (!blob) {
    *bytes = (size_t)need;
    return HLBM_OK;
  }
  if (*bytes < need) return fail(c, HLBM_E_ARG, "state blob needs %llu bytes", need);
  const size_t cap = (size_t)c.tab[0].cap;
  StateHeader hd;
  memset(&hd, 0, sizeof hd);
  memcpy(hd.magic, kMagic, 8);
  hd.version = 2;
  hd.precision = c.precision;
  hd.nx = c.g.nx; hd.ny = c.g.ny; hd.nz = c.g.nz;
  hd.np = c.np;
  hd.cur = c.cur;
  hd.tcur = c.tcur;
  hd.cap = (int)cap;
  hd.n_sub = c.n_sub;
  hd.step = c.step;
  hd.f_bytes = pop_bytes(c);
  hd.part_bytes = c.part_bytes;
  hd.tile_bytes = c.tile_bytes;
  hd.psum_bytes = c.psum_bytes;
  hd.tab_bytes = key_block_bytes((int)cap) + cap * sizeof(PairRec);
  hd.owner_bytes = sizeof(int) * (size_t)c.g.ncell;
  char* o = (char*)blob;
  memcpy(o, &hd, sizeof hd);
  o += sizeof hd;
  auto get = [&](const void* dev, size_t n) {
    hipError_t e = hipMemcpyAsync(o, dev, n, hipMemcpyDeviceToHost, c.stream);
    o += n;
    return e;
  };
  HIPCHECK(get(c.fbuf[c.cur], pop_bytes(c)));
  HIPCHECK(get(c.part_block, c.part_bytes));
  HIPCHECK(get(c.tile_block, c.tile_bytes));
  HIPCHECK(get(c.part_sums, c.psum_bytes));
  for (int k = 0; k < 2; ++k) {
    HIPCHECK(get(c.tab[k].keys, key_block_bytes((int)cap)));
    HIPCHECK(get(c.tab[k].rec, sizeof(PairRec) * cap));
  }
  HIPCHECK(get(c.owner, sizeof(int) * (size_t)c.g.ncell));
  HIPCHECK(get(c.counters, sizeof(Counters)));
  HIPCHECK(hipStreamSynchronize(c.stream));
  *bytes = (size_t)need;
  return HLBM_OK;
}

hlbm_status hlbm_set_state(hlbm_ctx* h, const void* blob, size_t bytes) {
  if (!h || !blob) return HLBM_E_ARG;
  Ctx& c = h->c;
  if (!c.particles_ready)
    return fail(c, HLBM_E_STATE, "initialise the particles (same count and shapes) first");
  StateHeader hd;
  if (bytes < sizeof hd) return fail(c, HLBM_E_ARG, "state blob too short");
  memcpy(&hd, blob, sizeof hd);
  const size_t cap = (size_t)c.tab[0].cap;
  if (memcmp(hd.magic, kMagic, 8) != 0 || hd.version != 2)
    return fail(c, HLBM_E_ARG, "not a state blob of this library");
  if (hd.precision != c.precision || hd.nx != c.g.nx || hd.ny != c.g.ny || hd.nz != c.g.nz ||
      hd.np != c.np || hd.cap != (int)cap || hd.n_sub != c.n_sub || hd.part_bytes != c.part_bytes ||
      hd.tile_bytes != c.tile_bytes || hd.psum_bytes != c.psum_bytes)
    return fail(c, HLBM_E_ARG, "state blob was written by a different configuration");
  if (bytes < state_bytes(c)) return fail(c, HLBM_E_ARG, "state blob truncated");
  hlbm_status st = ensure_populations(c);
  if (st) return st;
  drop_graphs(c);
  c.cur = hd.cur;
  c.tcur = hd.tcur;
  c.step = hd.step;
  const char* o = (const char*)blob + sizeof hd;
  auto put = [&](void* dev, size_t n) {
    hipError_t e = hipMemcpyAsync(dev, o, n, hipMemcpyHostToDevice, c.stream);
    o += n;
    return e;
  };
  HIPCHECK(put(c.fbuf[c.cur], pop_bytes(c)));
  HIPCHECK(put(c.part_block, c.part_bytes));
  HIPCHECK(put(c.tile_block, c.tile_bytes));
  HIPCHECK(put(c.part_sums, c.psum_bytes));
  for (int k = 0; k < 2; ++k) {
    HIPCHECK(put(c.tab[k].keys, key_block_bytes((int)cap)));
    HIPCHECK(put(c.tab[k].rec, sizeof(PairRec) * cap));
  }
  HIPCHECK(put(c.owner, sizeof(int) * (size_t)c.g.ncell));
  HIPCHECK(put(c.counters, sizeof(Counters)));
  HIPCHECK(hipStreamSynchronize(c.stream));
  free_adjoint(c);
  c.fluid_ready = true;
  st = check_flags(c);
  return st != HLBM_OK ? st : prepare_graphs(c);
}

hlbm_status hlbm_adjoint_record(hlbm_ctx* h, int ksteps, int ckpt_every) {
  if (!h) return HLBM_E_ARG;
  Ctx& c = h->c;
  if (!c.fluid_ready) return fail(c, HLBM_E_STATE, "initialise particles and fluid first");
  if (c.precision != HLBM_FP64)
    return fail(c, HLBM_E_ARG, "the adjoint runs on the FP64 form only");
  if (!c.g.periodic_z) return fail(c, HLBM_E_ARG, "the adjoint needs a fully periodic box");
  if (c.n_sub != 1) return fail(c, HLBM_E_ARG, "the adjoint runs without contact sub-steps");
  if (c.ph.bal_mode == 2)
    return fail(c, HLBM_E_ARG, "the adjoint supports balance modes 0 and 1 only");
  {
    std::vector<int> sh(c.np > 0 ? c.np : 1);
    if (c.np > 0) {
      HIPCHECK(hipMemcpy(sh.data(), c.part.shape, sizeof(int) * c.np, hipMemcpyDeviceToHost));
      for (int i = 0; i < c.np; ++i)
        if (sh[i] >= POLY0)
          return fail(c, HLBM_E_ARG, "the adjoint supports spheres, cubes and octahedra only");
    }
  }
  if (c.timing) return fail(c, HLBM_E_STATE, "finish the timing window first");
  if (ksteps < 1 || ckpt_every < 1)
    return fail(c, HLBM_E_ARG, "ksteps and ckpt_every must be >= 1");
  free_adjoint(c);
  Adjoint& a = c.adj;
  a.K = ksteps;
  a.L = ckpt_every < ksteps ? ckpt_every : ksteps;
  a.nseg = (a.K + a.L - 1) / a.L;
  a.ck = new (std::nothrow) Snapshot[a.nseg];
  if (!a.ck) return fail(c, HLBM_E_NOMEM, "checkpoint table");
  for (int k = 0; k < a.nseg; ++k)
    if (snapshot_alloc(c, a.ck[k]) != hipSuccess) {
      free_adjoint(c);
      return fail(c, HLBM_E_NOMEM, "checkpoint %d of %d", k, a.nseg);
    }
  if (snapshot_alloc(c, a.end) != hipSuccess) {
    free_adjoint(c);
    return fail(c, HLBM_E_NOMEM, "end-state snapshot");
  }
  for (int seg = 0; seg < a.nseg; ++seg) {
    HIPCHECK(snapshot_copy(c, a.ck[seg], 0));
    const int n = std::min(a.L, a.K - seg * a.L);
    for (int s = 0; s < n; ++s) HIPCHECK(run_step(c, nullptr));
  }
  HIPCHECK(snapshot_copy(c, a.end, 0));
  hlbm_status st = check_flags(c);
  if (st) return st;
  a.recorded = true;
  return HLBM_OK;
}

hlbm_status hlbm_adjoint_gradient(hlbm_ctx* h, const double* dJ_dU, double* dJ_ds,
                                  double* dJ_dtheta0, double* dJ_dq0,
                                  double* dJ_dX0, double* dJ_dU0,
                                  double* dJ_domega0) {
  if (!h) return HLBM_E_ARG;
  Ctx& c = h->c;
  Adjoint& a = c.adj;
  if (!a.recorded) return fail(c, HLBM_E_STATE, "no recorded forward window");
  if (!dJ_dU) return fail(c, HLBM_E_ARG, "null seed");
  const int np = c.np;
  const size_t npp = np > 0 ? np : 1;
  const long long n = c.g.ncell;
  const int PR = adjoint_record_doubles(), PB = adjoint_slots();
  if (!a.fst) {
    bool ok = hipMalloc(&a.fst, sizeof(double) * (size_t)(a.L + 1) * Q * n) == hipSuccess &&
              hipMalloc(&a.ost, sizeof(int) * (size_t)(a.L + 1) * n) == hipSuccess &&
              hipMalloc(&a.pst, sizeof(double) * (size_t)(a.L + 1) * npp * PR) == hipSuccess &&
              hipMalloc(&a.frc, sizeof(double) * (size_t)a.L * npp * 12) == hipSuccess &&
              hipMalloc(&a.gbar, sizeof(double) * (size_t)Q * n) == hipSuccess &&
              hipMalloc(&a.hbar, sizeof(double) * (size_t)Q * n) == hipSuccess &&
              hipMalloc(&a.pbar, sizeof(double) * npp * PB) == hipSuccess &&
              hipMalloc(&a.sbar, sizeof(double) * npp) == hipSuccess &&
              hipMalloc(&a.work, sizeof(double) * adjoint_work_doubles(c)) == hipSuccess;
    if (!ok) return fail(c, HLBM_E_NOMEM, "adjoint work arrays (segment of %d steps)", a.L);
  }
  // seed: J = sum_p dJ_dU[p] . U_p(K)
  std::vector<double> pb(npp * PB, 0.0);
  for (int p = 0; p < np; ++p)
    for (int k = 0; k < 3; ++k) pb[(size_t)PB * p + 6 + k] = dJ_dU[3 * p + k];
  HIPCHECK(hipMemcpyAsync(a.pbar, pb.data(), sizeof(double) * npp * PB,
                          hipMemcpyHostToDevice, c.stream));
  HIPCHECK(launch_fill_zero(c, a.sbar, (long long)npp));
  HIPCHECK(launch_fill_zero(c, a.gbar, (long long)Q * n));
  const size_t fs = (size_t)Q * n;
  for (int seg = a.nseg - 1; seg >= 0; --seg) {
    HIPCHECK(snapshot_copy(c, a.ck[seg], 1));
    const int L = std::min(a.L, a.K - seg * a.L);
    // recompute the segment, recording what the reverse steps read
    for (int k = 0; k <= L; ++k) {
      if (k < L)
        HIPCHECK(hipMemcpyAsync(a.fst + (size_t)k * fs, c.fbuf[c.cur],
                                sizeof(double) * fs, hipMemcpyDeviceToDevice, c.stream));
      HIPCHECK(hipMemcpyAsync(a.ost + (size_t)k * n, c.owner, sizeof(int) * n,
                              hipMemcpyDeviceToDevice, c.stream));
      HIPCHECK(launch_rec_particles(c, a.pst + (size_t)k * npp * PR));
      if (k == L) break;
      HIPCHECK(run_step(c, nullptr));
      HIPCHECK(launch_rec_forces(c, a.frc + (size_t)k * npp * 12));
    }
    for (int k = L - 1; k >= 0; --k)
      HIPCHECK(launch_adjoint_step(c, a.gbar, a.hbar, a.fst + (size_t)k * fs,
                                   a.ost + (size_t)k * n, a.ost + (size_t)(k + 1) * n,
                                   a.pst + (size_t)k * npp * PR,
                                   a.pst + (size_t)(k + 1) * npp * PR,
                                   a.frc + (size_t)k * npp * 12, a.pbar, a.sbar, a.work));
  }
  // initial orientations, from the particle block of checkpoint 0
  std::vector<double> q0(4 * npp);
  const size_t qoff = (size_t)((char*)c.part.q - (char*)c.part_block);
  HIPCHECK(hipMemcpyAsync(q0.data(), (char*)a.ck[0].part + qoff, sizeof(double) * 4 * npp,
                          hipMemcpyDeviceToHost, c.stream));
  std::vector<double> sb(npp);
  HIPCHECK(hipMemcpyAsync(pb.data(), a.pbar, sizeof(double) * npp * PB,
                          hipMemcpyDeviceToHost, c.stream));
  HIPCHECK(hipMemcpyAsync(sb.data(), a.sbar, sizeof(double) * npp, hipMemcpyDeviceToHost,
                          c.stream));
  HIPCHECK(snapshot_copy(c, a.end, 1));
  HIPCHECK(hipStreamSynchronize(c.stream));
  for (int p = 0; p < np; ++p) {
    const double* v = &pb[(size_t)PB * p];
    if (dJ_ds) dJ_ds[p] = sb[p];
    for (int k = 0; k < 3; ++k) {
      if (dJ_dX0) dJ_dX0[3 * p + k] = v[k];
      if (dJ_dtheta0) dJ_dtheta0[3 * p + k] = v[3 + k];
      if (dJ_dU0) dJ_dU0[3 * p + k] = v[6 + k];
      if (dJ_domega0) dJ_domega0[3 * p + k] = v[9 + k];
    }
    if (dJ_dq0) {
      // gradient in quaternion space, tangent to the unit sphere:
      // 2 (0, theta_bar) (x) q
      const double* q = &q0[4 * p];
      const double t[3] = {v[3], v[4], v[5]};
      dJ_dq0[4 * p + 0] = -2.0 * (t[0] * q[1] + t[1] * q[2] + t[2] * q[3]);
      dJ_dq0[4 * p + 1] = 2.0 * (q[0] * t[0] + (t[1] * q[3] - t[2] * q[2]));
      dJ_dq0[4 * p + 2] = 2.0 * (q[0] * t[1] + (t[2] * q[1] - t[0] * q[3]));
      dJ_dq0[4 * p + 3] = 2.0 * (q[0] * t[2] + (t[0] * q[2] - t[1] * q[1]));
    }
  }
  return check_flags(c);
}

hlbm_status hlbm_adjoint(hlbm_ctx* h, int ksteps, int ckpt_every, const double* dJ_dU,
                         double* dJ_ds, double* dJ_dq0) {
  hlbm_status st = hlbm_adjoint_record(h, ksteps, ckpt_every);
  if (st != HLBM_OK) return st;
  return hlbm_adjoint_gradient(h, dJ_dU, dJ_ds, nullptr, dJ_dq0, nullptr, nullptr, nullptr);
}

// the build passes the hash of the sources (paper_2401_10878_amd/build.py);
// a compile without it reports a hash no source set has
#ifndef HLBM_SOURCE_HASH
#define HLBM_SOURCE_HASH "unhashed"
#endif
const char* hlbm_build_hash(void) { return HLBM_SOURCE_HASH; }

const char* hlbm_last_error(const hlbm_ctx* h) {
  return h ? h->c.err : "null context";
}

void hlbm_destroy(hlbm_ctx* h) {
  if (!h) return;
  Ctx& c = h->c;
  if (c.stream) hipStreamSynchronize(c.stream);
  drop_graphs(c);
  free_timing(c);
  free_particles(c);
  free_adjoint(c);
  if (c.own_f) {
    if (c.fbuf[0]) hipFree(c.fbuf[0]);
    if (c.fbuf[1]) hipFree(c.fbuf[1]);
  }
  if (c.owner) hipFree(c.owner);
  if (c.tile_block) hipFree(c.tile_block);
  if (c.counters) hipFree(c.counters);
  if (c.bal_part) hipFree(c.bal_part);
  if (c.poly_dev) hipFree(c.poly_dev);
  if (c.scratch) hipFree(c.scratch);
  for (int k = 0; k < 2; ++k) {
    if (c.tab[k].keys) hipFree(c.tab[k].keys);
    if (c.tab[k].rec) hipFree(c.tab[k].rec);
  }
  if (c.side) {
    hipStreamSynchronize(c.side);
    hipStreamDestroy(c.side);
  }
  if (c.ev_det) hipEventDestroy(c.ev_det);
  if (c.ev_treat) hipEventDestroy(c.ev_treat);
  if (c.ev_lat) hipEventDestroy(c.ev_lat);
  if (c.ev_bal) hipEventDestroy(c.ev_bal);
  if (c.own_stream && c.stream) hipStreamDestroy(c.stream);
  delete h;
}

}  // extern "C"
