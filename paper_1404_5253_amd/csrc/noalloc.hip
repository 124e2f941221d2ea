// Allocation-free variant of wp_lattice_resolvent for callers that cannot allocate device memory
// (code under stream capture, tight serving loops, hosts that forbid allocation after set-up).
//
// The G1 kernels need device memory beyond the caller's output: the G1 values of every channel,
// the energy, and the work list (counter + entries) through which k_g1_lane hands the near-shell
// elements to k_g1_wave. Here that memory is one file-scope device array of WP_NOALLOC_SCRATCH
// bytes. Each GPU holds its own copy of the array until the process ends; its device address is
// looked up once per device (hipGetSymbolAddress, with that device current) and kept, and only
// that address is ever passed to kernels or copies. Calls on one GPU share the array: calls that
// overlap in time on the same GPU race (the library serialises none of them).
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/wpcd.h"
#include "wpcd_objects.h"

namespace {

constexpr size_t kScratchBytes = WP_NOALLOC_SCRATCH;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (looked up on the first call on the device).
wp_status scratch_address(void** out) {
  int dev = 0;
  HIPCHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return wpcd::fail(WP_EDEVICE, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPCHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return wpcd::fail(WP_EDEVICE, "hipGetSymbolAddress returned a null scratch address");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return WP_OK;
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// out[k * N + j] = G[((j * M + k) * nch + ch)]: one channel of the G1 block in the query's order
__global__ void k_pick_channel(const double2* __restrict__ G, int M, int N, int nch, int ch,
                               double2* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)M * N) return;
  const int k = (int)(t / N), j = (int)(t - (int64_t)k * N);
  out[t] = G[((size_t)j * M + k) * nch + ch];
}

}  // namespace

extern "C" wp_status wp_lattice_resolvent_noalloc(const wp_lattice* Lc, double E_lab, int channel, double* G) {
  const wp_lattice* L = Lc;
  if (!L || !G) return wpcd::fail(WP_EINVAL, "NULL argument");
  if (!L->pseudo) return wpcd::fail(WP_ENOTREADY, "twobody_pseudostates has not run");
  if (channel < 0 || channel >= L->nch) return wpcd::fail(WP_EINVAL, "channel out of range");
  if (!(E_lab > 0)) return wpcd::fail(WP_EINVAL, "E_lab must be positive");
  // layout in the scratch array: G1 of every channel [rows] double2 | the requested channel [M N]
  // double2 | E | work list (counter + entries)
  const int64_t rows = (int64_t)L->M * L->N * L->nch;
  const size_t off_c = align256((size_t)rows * sizeof(double2));
  const size_t off_E = off_c + align256((size_t)L->M * L->N * sizeof(double2));
  const size_t off_w = off_E + 256;
  const int64_t nwork = wpcd::g1_work_elems((int)L->waves.size(), L->M, L->N, 1) + 1;
  const size_t need = off_w + (size_t)nwork * sizeof(int64_t);
  if (need > kScratchBytes)
    return wpcd::fail(WP_EINVAL, "wp_lattice_resolvent_noalloc: this lattice needs " + std::to_string(need) +
                                     " bytes of scratch, more than the " + std::to_string(kScratchBytes) +
                                     " the library reserves (use wp_lattice_resolvent)");
  // the device tables (lattice, pseudostates, quadrature rules) must already be resident
  if (!L->d_qe.p || !L->d_O.p || !L->d_bins.p)
    return wpcd::fail(WP_ENOTREADY, "wp_lattice_resolvent_noalloc: the lattice's device tables are not resident "
                                    "(run perm_matrix_build, faddeev_solve or wp_lattice_resolvent once first)");
  void* base = nullptr;
  if (wp_status st = scratch_address(&base)) return st;
  unsigned char* sp = static_cast<unsigned char*>(base);
  double2* dG = reinterpret_cast<double2*>(sp);
  double2* dC = reinterpret_cast<double2*>(sp + off_c);
  double* dE = reinterpret_cast<double*>(sp + off_E);
  int64_t* work = reinterpret_cast<int64_t*>(sp + off_w);
  const double E = L->eps0 + 2.0 * E_lab / 3.0;
  // null stream, synchronous, as wp_lattice_resolvent; the G1 kernels clear the work-list counter
  // themselves and write every element of dG
  HIPCHECK(hipMemcpy(dE, &E, sizeof(double), hipMemcpyHostToDevice));
  HIPCHECK(wpcd::launch_g1(wpcd::g1_args(L, dE, 1, 1, 0, 1, dG, work), nullptr));
  const int64_t MN = (int64_t)L->M * L->N;
  hipLaunchKernelGGL(k_pick_channel, dim3((unsigned)((MN + 255) / 256)), dim3(256), 0, nullptr, dG, L->M, L->N,
                     L->nch, channel, dC);
  HIPCHECK(hipGetLastError());
  // G[2 (k N + j) + {0, 1}]: the byte layout of the picked [k][j] double2 array
  HIPCHECK(hipMemcpy(G, dC, (size_t)MN * sizeof(double2), hipMemcpyDeviceToHost));
  return WP_OK;
}
