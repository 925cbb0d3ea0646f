// Allocation-free measurement (mps_measure_static in include/mpsim_static.h): the
// transfer-matrix sweep of <Z_tot> and <Z_tot^2> (eqs. "Z_tot", "z2_tot")
// over an MPS the caller holds in device memory, with the three stacked
// environments and the per-site z sums in a static device array instead of
// memory the library allocates. It launches the same kernels as the
// handle's measurement (batched GEMMs and the z-moment combine).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mpsim_static.h"
#include "common.h"
#include "gemm.h"
#include "mps_kernels.h"

namespace mpsim {
void set_thread_error(const std::string& msg);  // mpsim.cpp
}

using namespace mpsim;

namespace {

// One copy per GPU, held until the process ends. In host code the name is
// only a handle for hipGetSymbolAddress: its device address is looked up per
// device and kept in g_scratch.
static __device__ __align__(256) unsigned char scratch[MPS_MEASURE_STATIC_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`.
hipError_t scratch_address(int dev, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = p;
    bounds_register(p, (size_t)MPS_MEASURE_STATIC_BYTES);
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

constexpr size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// z_p(s) = sum over the fused qubits of (1 - 2 bit) = w - 2 popcount(s), d = 2^w
__global__ void k_zsum_fill(double* z, int d, int w) {
  const int s = threadIdx.x;
  if (s < d) z[s] = (double)(w - 2 * (int)__popc((unsigned)s));  // __popc is unsigned
}

// out = {<psi|psi>, <Z_tot> / n, <Z_tot^2> / n^2} from the three final 1x1
// environments (the last two divided by the norm)
__global__ void k_meas_finish(const cplx* E, double n, double* out) {
  const double nrm = E[0].x;
  out[0] = nrm;
  out[1] = E[1].x / (n * nrm);
  out[2] = E[2].x / (n * n * nrm);
}

int log2_exact(int d) {
  int w = 0;
  while ((1 << w) < d) ++w;
  return (1 << w) == d ? w : -1;
}

mps_status fail_static(mps_status st, const std::string& msg) {
  set_thread_error(msg);
  return st;
}

}  // namespace

extern "C" mps_status mps_measure_static(int32_t nsites, const int32_t* bonds, const int32_t* dims,
                                         const void* const* sites, void* hip_stream, double* out_dev) {
  if (nsites < 1 || !bonds || !dims || !sites || !out_dev)
    return fail_static(MPS_E_INVAL, "mps_measure_static: NULL argument or nsites < 1");
  if (bonds[0] != 1 || bonds[nsites] != 1)
    return fail_static(MPS_E_INVAL, "mps_measure_static: end bonds must be 1");
  long bmax = 1, xmax = 1, zlen = 0;
  int n = 0;
  for (int p = 0; p < nsites; ++p) {
    const int w = log2_exact(dims[p]);
    if (w < 1 || w > 4) return fail_static(MPS_E_INVAL, "mps_measure_static: dims must be 2, 4, 8 or 16");
    if (bonds[p + 1] < 1) return fail_static(MPS_E_INVAL, "mps_measure_static: bonds must be >= 1");
    if (!sites[p]) return fail_static(MPS_E_INVAL, "mps_measure_static: NULL site");
    n += w;
    bmax = std::max(bmax, (long)bonds[p + 1]);
    xmax = std::max(xmax, (long)bonds[p] * dims[p] * bonds[p + 1]);
    zlen += dims[p];
  }
  if (bmax > (1L << 16))  // keeps the size arithmetic below far from overflow
    return fail_static(MPS_E_UNSUPPORTED, "mps_measure_static: bond dimension too large");
  // scratch layout: env0 | env1 (3 b_max^2 complex each) | X (3 max b d b')
  // | z sums (sum of d doubles), each 256-byte aligned
  const size_t env_b = align256(sizeof(cplx) * 3 * (size_t)bmax * bmax);
  const size_t x_b = align256(sizeof(cplx) * 3 * (size_t)xmax);
  const size_t z_b = align256(sizeof(double) * (size_t)zlen);
  const size_t need = 2 * env_b + x_b + z_b;
  if (need > (size_t)MPS_MEASURE_STATIC_BYTES)
    return fail_static(MPS_E_UNSUPPORTED,
                       "mps_measure_static: the environments need " + std::to_string(need) +
                           " bytes, more than the static buffer's " +
                           std::to_string((long long)MPS_MEASURE_STATIC_BYTES));
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return fail_static(MPS_E_DEVICE, "mps_measure_static: no current device");
  void* base = nullptr;
  hipError_t e = scratch_address(dev, &base);
  if (e != hipSuccess)
    return fail_static(MPS_E_DEVICE, std::string("mps_measure_static: hipGetSymbolAddress: ") +
                                         hipGetErrorString(e));
  unsigned char* b8 = (unsigned char*)base;
  cplx* env[2] = {(cplx*)b8, (cplx*)(b8 + env_b)};
  cplx* X = (cplx*)(b8 + 2 * env_b);
  double* zs = (double*)(b8 + 2 * env_b + x_b);
  hipStream_t s = (hipStream_t)hip_stream;
  const cplx one = make_double2(1, 0), zero = make_double2(0, 0);
  // with operand checks on, the caller's sites count as buffers for this call
  std::vector<const void*> added;
  if (bounds_checking())
    for (int p = 0; p < nsites; ++p)
      if (bounds_register_new(sites[p], sizeof(cplx) * (size_t)bonds[p] * dims[p] * bonds[p + 1]))
        added.push_back(sites[p]);
  struct Unregister {
    std::vector<const void*>& v;
    ~Unregister() {
      for (const void* p : v) bounds_unregister(p);
    }
  } unreg{added};
  try {
  // every buffer region read below is written first in this call: the
  // environment starts as {1, 0, 0}, the GEMMs overwrite (beta = 0)
  long zoff = 0;
  for (int p = 0; p < nsites; ++p) {
    hipLaunchKernelGGL(k_zsum_fill, dim3(1), dim3(64), 0, s, zs + zoff, dims[p], log2_exact(dims[p]));
    zoff += dims[p];
  }
  launch_env_init(env[0], s);
  int cur = 0;
  zoff = 0;
  for (int p = 0; p < nsites; ++p) {
    const int b = bonds[p], d = dims[p], b2 = bonds[p + 1];
    const long xs = (long)b * d * b2;
    const cplx* A = (const cplx*)sites[p];
    // X_k = E_k A (three environments in one batched GEMM)
    ZGemm g1 = zgemm_args(b, d * b2, b, zop(env[cur], b, 0), zop(A, (long)d * b2, 0), X, (long)d * b2, 0,
                          one, zero);
    g1.batch = 3;
    g1.A.stride = (long)b * b;
    g1.B.stride = 0;
    g1.strideC = xs;
    zgemm(g1, nullptr, 0, s, nullptr);
    launch_meas_combine(X, b, d, b2, zs + zoff, s);
    // E'_k = A^H Y_k
    ZGemm g2 = zgemm_args(b2, b2, b * d, zop(A, b2, 1, 1), zop(X, b2, 0), env[1 - cur], b2, 0, one, zero);
    g2.batch = 3;
    g2.A.stride = 0;
    g2.B.stride = xs;
    g2.strideC = (long)b2 * b2;
    zgemm(g2, nullptr, 0, s, nullptr);
    cur = 1 - cur;
    zoff += d;
  }
  hipLaunchKernelGGL(k_meas_finish, dim3(1), dim3(1), 0, s, (const cplx*)env[cur], (double)n, out_dev);
  } catch (BoundsError& be) {
    return fail_static(MPS_E_DEVICE, "mps_measure_static: operand out of bounds, not launched: " + be.msg);
  }
  e = hipGetLastError();
  if (e != hipSuccess)
    return fail_static(MPS_E_DEVICE, std::string("mps_measure_static: launch: ") + hipGetErrorString(e));
  return MPS_OK;
}
