// Host-side context of the library and the launch interface of each kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/hlbm.h"
#include "device_math.h"

namespace hlbm {

// One contact-pair record of the open-addressing pair table.  count, rlo and
// rhi are written with atomics by the rough detection; the rest is written
// by the single wavefront that treats the record, or by the copy that
// carries a kept contact into the next step's table.
struct PairRec {
  int a, b;
  int count;
  int rlo[3], rhi[3];
  int carried, established, age, n_in, keep, pad;
  double lo[3], hi[3];
  double damping;
  double volume, centroid[3], normal[3], depth, fn, force_a[3];
};

struct PairTable {
  uint64_t* keys;   // [cap], EMPTY_KEY when free
  PairRec* rec;     // [cap]
  int cap;          // power of two
  // the occupied slots in order of insertion (list[0 .. *nlist)), so that
  // the treatment and the clearing visit only those; both follow the keys
  // in one allocation (key_block_bytes) and are copied with them
  int* list;
  int* nlist;
};
inline size_t key_block_bytes(int cap) {
  return sizeof(uint64_t) * (size_t)cap + sizeof(int) * ((size_t)cap + 2);
}
inline void set_table_views(PairTable& t) {
  t.list = (int*)(t.keys + t.cap);
  t.nlist = t.list + t.cap;
}
// A key inserted into slot h (by the inserting thread only) joins the list.
__device__ inline void list_slot(const PairTable& t, uint32_t h) {
  t.list[atomicAdd(t.nlist, 1)] = (int)h;
}

// Device counters and flags (one small block of device memory).
struct Counters {
  unsigned long long det_pairs;    // keys with count > 0 (latest detection)
  unsigned long long det_cells;    // sum of counts (latest detection)
  unsigned long long total_cells;  // sum over all detections
  unsigned long long steps;
  unsigned long long samples;      // midpoint samples of the latest treatment
  int tile_overflow;
  int pair_overflow;
  int unstable;
  int contact_overflow;   // more than MAXC contacts on one particle
  // zero-net-flux balance force (balance mode 2): controller part b of the
  // fluid acceleration, lattice momentum P after the last collision,
  // lattice mass M, and the acceleration a = fluid_accel + b in use
  double bal_b[3], bal_P[3], bal_M, bal_a[3];
};

// Carry-over of slot s of the pair table `from` into `to` when its record
// is marked to be kept (an established contact that continues, Sec. 3.3.2):
// the key is inserted by linear probing and the record's contact state
// copied; a full table raises pair_overflow.
__device__ inline void keep_slot(const PairTable& from, const PairTable& to, long long s,
                                 Counters* ctr) {
  const uint64_t key = from.keys[s];
  if (key == EMPTY_KEY) return;
  const PairRec& r = from.rec[s];
  if (!r.keep) return;
  const uint32_t mask = (uint32_t)to.cap - 1u;
  uint32_t h = pair_hash(key) & mask;
  for (int probe = 0; probe < to.cap; ++probe) {
    unsigned long long old = atomicCAS((unsigned long long*)&to.keys[h],
                                       (unsigned long long)EMPTY_KEY,
                                       (unsigned long long)key);
    if (old == EMPTY_KEY) list_slot(to, h);
    if (old == EMPTY_KEY || old == key) {
      PairRec& d = to.rec[h];
      d.a = r.a;
      d.b = r.b;
      d.carried = 1;
      d.established = r.established;
      d.age = r.age;
      d.n_in = r.n_in;
      d.keep = 0;
      for (int k = 0; k < 3; ++k) {
        d.lo[k] = r.lo[k];
        d.hi[k] = r.hi[k];
        d.centroid[k] = r.centroid[k];
        d.normal[k] = r.normal[k];
        d.force_a[k] = r.force_a[k];
      }
      d.damping = r.damping;
      d.volume = r.volume;
      d.depth = r.depth;
      d.fn = r.fn;
      return;
    }
    h = (h + 1u) & mask;
  }
  atomicOr(&ctr->pair_overflow, 1);
}

// Division of 0 <= n < 2^31 by a fixed divisor d >= 1 with one multiply-high
// and a shift (Granlund and Montgomery, PLDI 1994): with s = ceil(log2 d)
// and m = floor(2^32 (2^s - d) / d) + 1, n / d = (mulhi(n, m) + n) >> s; the
// sum stays below 2^32 because mulhi(n, m) <= n.
struct FastDiv {
  unsigned d, m, s;
};
inline FastDiv make_fastdiv(unsigned d) {
  unsigned s = 0;
  while ((1ull << s) < d) ++s;
  const unsigned long long m = ((1ull << 32) * ((1ull << s) - d)) / d + 1;
  return FastDiv{d, (unsigned)m, s};
}
__host__ __device__ inline unsigned fdiv(unsigned n, FastDiv f) {
  return (unsigned)(((((unsigned long long)n * f.m) >> 32) + n) >> f.s);
}

// Scalar parameters handed to every kernel by value.
struct Geom {
  int nx, ny, nz;
  int periodic_z;
  int dtx, dty, dtz;      // detection tiles per axis (DX x DY x DZ nodes)
  int ltx, lty, ltz;      // lattice blocks per axis (LX x LY x LZ nodes)
  FastDiv fdtx, fdty;     // divisions by dtx, dty
  FastDiv fltx, flty;     // divisions by ltx, lty
  int tile_cap;           // particles per candidate list (both tilings)
  int maxent;             // lattice blocks per particle (partial-sum slots)
  long long ncell;
};

// Candidate lists of both tilings and the momentum-exchange partial sums.
// dlist[t*cap + s]: particle ids reaching detection tile t.
// llist[b*cap + s]: particle ids reaching lattice block b, lent[b*cap + s]:
// index k of block b in that particle's own block enumeration;
// part[(p*maxent + k)*6 + 0..5] = the (force, torque) the nodes of that
// block contribute to particle p; nent[p] = blocks enumerated for p;
// ovf[p*6 + ..] collects the rare contributions that do not fit the
// per-lane slots.
struct Tiles {
  int* dcount;
  int* dlist;
  int* lcount;
  int* llist;
  int* lent;
  int* nent;
  double* part;
  double* ovf;
  // contact forces of the step, per particle: ccount[p] entries, each with
  // the partner id ckey[p*MAXC + k] (walls -1, -2) and (force, torque)
  // cval[(p*MAXC + k)*6 + 0..5]; summed in partner order by k_particles
  int* ccount;
  int* ckey;
  double* cval;
};

struct Phys {
  double tau, omega;      // relaxation time and 1/tau
  double wall_u[2][3];
  double gravity[3];
  double a_ext[3];        // uniform fluid acceleration (incl. balance 1)
  int bal_mode;           // 2: the acceleration is Counters::bal_a (device)
  double eps, delta_c;
  float eps_h32, eps_q32;  // eps / 2 and 1 / (4 eps) in FP32 (coupling weight)
  int n_c;
  double estar;           // effective modulus, eq. (5)
  double restitution, mu_s, mu_k, u_k;
  double dt_sub;          // length of a contact sub-step (1 / n_sub)
};

constexpr int NKERN = 7;   // clear, treat, particles, keep, detect, lattice, mea

// Device copy of the whole step state (populations f*, particle block,
// candidate lists and partial sums, both pair tables, owner map, counters).
struct Snapshot {
  void* f = nullptr;
  void* part = nullptr;
  void* tiles = nullptr;
  void* psums = nullptr;
  uint64_t* keys[2] = {nullptr, nullptr};
  PairRec* rec[2] = {nullptr, nullptr};
  int* owner = nullptr;
  Counters* ctr = nullptr;
  int cur = 0, tcur = 0;
  long long step = 0;
};

// Recorded forward window of the adjoint and its work arrays.
struct Adjoint {
  bool recorded = false;
  int K = 0, L = 0;                  // steps, steps per checkpoint
  Snapshot* ck = nullptr;            // checkpoint at the start of each segment
  int nseg = 0;
  Snapshot end;                      // state after the K steps
  double* fst = nullptr;             // (L + 1) x Q x ncell: f* at each step of a segment
  int* ost = nullptr;                // (L + 1) x ncell: owner maps
  double* pst = nullptr;             // (L + 1) x np x 22: particle states
  double* frc = nullptr;             // L x np x 12: forces of each step
  double* gbar = nullptr;            // dJ/df* (Q x ncell)
  double* hbar = nullptr;            // dJ/df  (Q x ncell)
  double* pbar = nullptr;            // np x 12 particle adjoints
  double* sbar = nullptr;            // np: dJ/ds
  double* work = nullptr;
};

struct Ctx {
  hlbm_params P;
  Geom g;
  Phys ph;
  hipStream_t stream;
  bool own_stream;
  // second stream for the next step's contact treatment, which overlaps the
  // stream-collide and momentum-exchange passes (ev_det: detection done on
  // `stream`; ev_treat: treatment done on `side`)
  hipStream_t side = nullptr;
  hipEvent_t ev_det = nullptr, ev_treat = nullptr;
  // balance sums of a step on the side stream: after its lattice pass
  // (ev_lat), before the next step's lattice pass (ev_bal)
  hipEvent_t ev_lat = nullptr, ev_bal = nullptr;
  int precision;
  size_t bytes_per_value;
  // populations (two buffers, ping-pong); fbuf[cur] holds f* of the last step
  void* fbuf[2];
  bool own_f;
  int cur;
  // particles
  int np;
  Particles part;         // device pointers
  void* part_block;       // one allocation for all particle arrays
  double* Fh;             // [np][3] hydrodynamic force of the last step
  double* Th;
  double* Fc;             // contact force / torque of the last step
  double* Tc;
  // lattice-side maps
  int* owner;             // [ncell]
  Tiles tl;
  void* tile_block;       // allocation holding count, list, ent
  void* part_sums;        // allocation holding nent, part, ovf
  // contacts
  PairTable tab[2];
  // convex polyhedron types: host records (volume, second moment about the
  // centroid, circumradius at unit scale) and the device table
  struct PolyHost {
    bool ok = false;
    PolyDev dev;
    double vol = 0.0, J[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  } poly_host[MAXPOLY];
  PolyDev* poly_dev = nullptr;
  bool has_poly = false;  // some particle is a polyhedron: kernels with that path
  bool has_ellipsoid = false;  // some particle is an ellipsoid type: the variants
                               // that also evaluate smooth bodies
  int tcur;               // tab[tcur] = current contact list
  Counters* counters;     // device
  double* scratch;        // [ncell] FP64 staging for host conversions
  double* fixed_scratch;  // device address of the fixed staging array
  double* bal_part = nullptr;  // per-block (mass, momentum) sums, balance mode 2
  // state
  bool particles_ready, fluid_ready;
  long long step;
  // per-kernel timing: ev_per_step events per step, a pool for `tcap` steps
  bool timing;
  int tcap, tused;
  hipEvent_t* tev;
  // sizes of the state blocks (for snapshots)
  size_t part_bytes = 0, tile_bytes = 0, psum_bytes = 0;
  Adjoint adj;
  // graphs: one per (population parity, contact-table parity) for a single
  // step, and (one contact sub-step) GRAPH_STEPS steps with the overlapped
  // contact treatment inside, in four variants v: v & 1, the first step's
  // treatment already ran (the previous graph's last step started it);
  // v & 2, the last step starts the next step's treatment and the graph
  // joins it before it ends
  bool use_graph;
  hipGraphExec_t gexec[4];
  bool graph_ready[4];
  hipGraphExec_t gexec_n[4][4];
  bool graph_n_ready[4][4] = {};
  bool graph_n_run[4][4] = {};   // replayed at least once (its one-time
                                 // setup on the device is done)
  int n_sub;
  int ev_per_step;        // timing events per step: 2 + 5 n_sub
  char err[512] = {};     // last error message (fixed: error paths allocate nothing)
};

// ---- launch wrappers (kernels live in the .hip files) --------------------
// what: CLEAR_CONTACT (next pair table, contact forces and slots, detection
// counters) and/or CLEAR_TILES (detection-tile and lattice-block counts)
constexpr int CLEAR_CONTACT = 1, CLEAR_TILES = 2;
// CLEAR_ALL_SLOTS: every slot of the table (once, after allocation; later
// clears visit the listed slots only)
constexpr int CLEAR_ALL_SLOTS = 4;
hipError_t launch_clear_step(Ctx& c, PairTable next, int what, hipStream_t s);
// move: 0 bin only, 1 gather the hydrodynamic force and move, 2 move with
// the stored hydrodynamic force (later sub-steps)
// keep_from / keep_to (optional, both or neither): the contact carry-over
// from one pair table to the next runs in the same launch
hipError_t launch_particles(Ctx& c, int move, const PairTable* keep_from = nullptr,
                            const PairTable* keep_to = nullptr);
hipError_t launch_keep(Ctx& c, PairTable from, PairTable to);
hipError_t launch_detect(Ctx& c, PairTable to);
// stream-collide src -> dst with the coupling of the current owner map
hipError_t launch_lattice(Ctx& c, const void* src, void* dst);
// momentum exchange over the collided populations fstar (force of the next step)
hipError_t launch_mea(Ctx& c, const void* fstar);
// balance mode 2: lattice mass and momentum of f at the start (init = 1), or
// the controller update after a collision from the lattice pass's block sums
hipError_t launch_balance(Ctx& c, const void* f, int init, hipStream_t st);
hipError_t launch_treat(Ctx& c, PairTable t, hipStream_t s);
hipError_t launch_fill_equilibrium(Ctx& c, void* f, double rho,
                                   const double u[3]);
hipError_t launch_store_direction(Ctx& c, void* f, int i, const double* src);
hipError_t launch_load_direction(Ctx& c, const void* f, int i, double* dst);
// comp = -1: density, 0..2: velocity component of f* (FP64, into out[ncell])
hipError_t launch_moment(Ctx& c, const void* f, int comp, double* out);
// coupling field: comp = -1 weight B, 0..2 particle velocity component
hipError_t launch_coupling_field(Ctx& c, int comp, double* out, int stride);
// nodes the fixed staging array of hlbm_read_coupling_noalloc holds
constexpr long long NOALLOC_MAX_CELLS = 1LL << 21;
hipError_t noalloc_scratch(double** out);
// adjoint (k_adjoint.hip)
int adjoint_record_doubles();
int adjoint_slots();
size_t adjoint_work_doubles(const Ctx& c);
hipError_t launch_rec_particles(Ctx& c, double* out);
hipError_t launch_rec_forces(Ctx& c, double* out);
hipError_t launch_fill_zero(Ctx& c, double* p, long long n);
hipError_t launch_adjoint_step(Ctx& c, double* gbar, double* hbar,
                               const double* fprev, const int* owner_prev,
                               const int* owner_t, const double* prec_prev,
                               const double* prec_t, const double* frc,
                               double* pbar, double* sbar, double* work);

}  // namespace hlbm
