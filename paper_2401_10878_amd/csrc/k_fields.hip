// Read-out of the coupling field (Sec. 3.2) for tests and diagnostics, and
// the fixed device staging array of the read-out that allocates nothing.
#include <mutex>

#include "context.h"

namespace hlbm {

namespace {

// Staging of hlbm_read_coupling_noalloc: B for every node, then u_p
// interleaved per node (4 doubles per node, NOALLOC_MAX_CELLS nodes at most,
// 64 MiB).  Each device holds its own copy for the life of the process; in
// host code the name only stands for the symbol, and kernels get the
// device address that hipGetSymbolAddress returned for the current device.
static __device__ __align__(256) double scratch[4 * (size_t)NOALLOC_MAX_CELLS];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[MAX_DEVICES] = {};

// Coupling field at the current particle state (Sec. 3.2), FP64: comp = -1
// writes B(d_owner), 0..2 the component of u_p = U + w x r of the owner
// (0 where no particle owns the node), at out[stride * node].
__global__ void k_coupling_field(const int* __restrict__ owner, Particles P,
                                 Geom g, Phys ph, int comp, double* __restrict__ out,
                                 int stride) {
  const long long id = (long long)blockIdx.x * 256 + threadIdx.x;
  if (id >= g.ncell) return;
  const int o = owner_id(owner[id]);
  double v = 0.0;
  if (o >= 0) {
    const int x = (int)(id % g.nx), y = (int)((id / g.nx) % g.ny);
    const int z = (int)(id / ((long long)g.nx * g.ny));
    const double r[3] = {minimg((double)x - P.X[3 * o], (double)g.nx, true),
                         minimg((double)y - P.X[3 * o + 1], (double)g.ny, true),
                         minimg((double)z - P.X[3 * o + 2], (double)g.nz, g.periodic_z != 0)};
    if (comp < 0) {
      v = weight(sdf<true>(P.shape[o], P.size[o], P.R + 9 * o, r[0], r[1], r[2], P.poly), ph.eps);
    } else {
      const double* W = P.W + 3 * o;
      const double wr[3] = {W[1] * r[2] - W[2] * r[1], W[2] * r[0] - W[0] * r[2],
                            W[0] * r[1] - W[1] * r[0]};
      v = P.U[3 * o + comp] + wr[comp == 0 ? 0 : (comp == 1 ? 1 : 2)];
    }
  }
  out[stride * id] = v;
}

}  // namespace

hipError_t launch_coupling_field(Ctx& c, int comp, double* out, int stride) {
  hipLaunchKernelGGL(k_coupling_field, dim3((unsigned)((c.g.ncell + 255) / 256)), dim3(256), 0,
                     c.stream, c.owner, c.part, c.g, c.ph, comp, out, stride);
  return hipGetLastError();
}

// Device address of the staging array on the current device, looked up once
// per device (first context created there) and kept.
hipError_t noalloc_scratch(double** out) {
  *out = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    double* ptr = nullptr;
    e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace hlbm
