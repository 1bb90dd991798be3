// Backscatter / RCS of stored solutions without any device allocation, for callers that
// cannot allocate (code under stream capture, tight serving loops).  It computes exactly
// what cavity_rcs_many computes (Section 7's theta-theta / phi-phi RCS from the aperture
// field, with the same aperture-transform kernel and the same per-block partial sums),
// but its queries, partial sums and results live in one fixed file-scope device array
// instead of a plan-owned block, and the partial sums are reduced on the device.
//
// The array is `scratch` below (kScratchBytes per device, held until the process ends).
// In host code its name is only a host-side stand-in: the device address comes from
// hipGetSymbolAddress, looked up once per device with that device current and kept in
// g_scratch[device]; every kernel argument and copy uses that address.  All calls on one
// device share the array: calls that overlap on a device race and must be serialised by
// the caller.  Every region of it is written before it is read within a call, so nothing
// needs clearing between calls.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>

#include "cavity.h"
#include "kernels.hpp"
#include "runtime.hpp"

namespace {

constexpr size_t kScratchBytes = (size_t)4 << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on device dev (which must be current).
int scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices)
    return cav::record_error(CAVITY_EDEVICE, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return cav::record_error(CAVITY_EDEVICE, (std::string("hipGetSymbolAddress(scratch): ") +
                                                hipGetErrorString(e)).c_str());
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return CAVITY_OK;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Byte offsets of the regions of one call in the scratch array.
struct Regions {
  size_t idx, th, ph, q, part, sig, end;
};

Regions regions(int n, int nblk) {
  Regions r{};
  r.idx = 0;
  r.th = align256(r.idx + (size_t)n * sizeof(int));
  r.ph = align256(r.th + (size_t)n * sizeof(double));
  r.q = align256(r.ph + (size_t)n * sizeof(double));
  r.part = align256(r.q + (size_t)n * sizeof(cav::RcsQuery));
  r.sig = align256(r.part + (size_t)n * 2 * nblk * sizeof(cav::zd));
  r.end = r.sig + (size_t)n * 2 * sizeof(double);
  return r;
}

// Query i: stored solution idx[i] seen from (th[i], ph[i]), u = k (sin t cos f, sin t sin f).
__global__ void k_rcs_setup(int n, const int* __restrict__ idx, const double* __restrict__ th,
                            const double* __restrict__ ph, double k,
                            cav::RcsQuery* __restrict__ q) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double st = sin(th[i]);
  q[i] = {idx[i], k * st * cos(ph[i]), k * st * sin(ph[i])};
}

// Sum the nblk partial aperture transforms of query i in block order, then
//   L = (-E^2, E^1, 0), sigma_theta = k^2/pi |phi^.L|^2, sigma_phi = k^2/pi |theta^.L|^2.
__global__ void k_rcs_finish(int n, int nblk, const cav::zd* __restrict__ part,
                             const double* __restrict__ th, const double* __restrict__ ph,
                             double k, double* __restrict__ sigma) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double e1r = 0.0, e1i = 0.0, e2r = 0.0, e2i = 0.0;
  for (int b = 0; b < nblk; ++b) {
    const cav::zd* pb = part + 2 * ((long long)i * nblk + b);
    e1r += pb[0].re;
    e1i += pb[0].im;
    e2r += pb[1].re;
    e2i += pb[1].im;
  }
  const double ct = cos(th[i]), sp = sin(ph[i]), cp = cos(ph[i]);
  // L1 = -E^2, L2 = E^1
  const double l1r = -e2r, l1i = -e2i, l2r = e1r, l2i = e1i;
  const double phr = -sp * l1r + cp * l2r, phi_ = -sp * l1i + cp * l2i;
  const double thr = ct * cp * l1r + ct * sp * l2r, thi = ct * cp * l1i + ct * sp * l2i;
  const double f = k * k / M_PI;
  sigma[2 * i] = f * (phr * phr + phi_ * phi_);
  sigma[2 * i + 1] = f * (thr * thr + thi * thi);
}

int fail_hip(hipError_t e, const char* what) {
  return cav::record_error(CAVITY_EDEVICE, (std::string(what) + ": " + hipGetErrorString(e)).c_str());
}

}  // namespace

extern "C" int cavity_rcs_many_noalloc(cavity_plan plan, int n, const int* rhs_index,
                                       const double* theta_o, const double* phi_o,
                                       double* sigma) {
  if (!plan || n < 0 || (n > 0 && (!rhs_index || !theta_o || !phi_o || !sigma)))
    return cav::record_error(CAVITY_EINVAL, "bad rcs arguments");
  cav::PlanView v{};
  int s = cav::plan_view(plan, &v);
  if (s) return s;
  for (int i = 0; i < n; ++i)
    if (rhs_index[i] < 0 || rhs_index[i] >= v.nsol)
      return cav::record_error(CAVITY_EINVAL, "no such solution");
  if (n == 0) return CAVITY_OK;
  const Regions r = regions(n, v.rcs_blocks);
  if (r.end > kScratchBytes)
    return cav::record_error(
        CAVITY_EINVAL, ("the pairs need " + std::to_string(r.end) + " bytes of the " +
                        std::to_string(kScratchBytes) + "-byte no-allocation scratch").c_str());
  int prev = 0;
  hipError_t e = hipGetDevice(&prev);
  if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
  if (prev != v.device && (e = hipSetDevice(v.device)) != hipSuccess)
    return fail_hip(e, "hipSetDevice");
  void* base = nullptr;
  s = scratch_address(v.device, &base);
  char* b = static_cast<char*>(base);
  auto* didx = reinterpret_cast<int*>(b + r.idx);
  auto* dth = reinterpret_cast<double*>(b + r.th);
  auto* dph = reinterpret_cast<double*>(b + r.ph);
  auto* dq = reinterpret_cast<cav::RcsQuery*>(b + r.q);
  auto* dpart = reinterpret_cast<cav::zd*>(b + r.part);
  auto* dsig = reinterpret_cast<double*>(b + r.sig);
  const hipStream_t st = v.stream;
  const unsigned nb = (unsigned)((n + 127) / 128);
  if (!s) {
    if ((e = hipMemcpyAsync(didx, rhs_index, (size_t)n * sizeof(int), hipMemcpyHostToDevice,
                            st)) != hipSuccess ||
        (e = hipMemcpyAsync(dth, theta_o, (size_t)n * sizeof(double), hipMemcpyHostToDevice,
                            st)) != hipSuccess ||
        (e = hipMemcpyAsync(dph, phi_o, (size_t)n * sizeof(double), hipMemcpyHostToDevice,
                            st)) != hipSuccess) {
      s = fail_hip(e, "query upload");
    }
  }
  if (!s) {
    hipLaunchKernelGGL(k_rcs_setup, dim3(nb), dim3(128), 0, st, n, didx, dth, dph, v.g.k, dq);
    if ((e = hipGetLastError()) != hipSuccess) s = fail_hip(e, "k_rcs_setup");
  }
  if (!s && (e = cav::launch_rcs_partial(v.g, v.xsol, v.nvec, dq, n, dpart, v.rcs_blocks, st)) !=
                hipSuccess)
    s = fail_hip(e, "k_rcs_partial");
  if (!s) {
    hipLaunchKernelGGL(k_rcs_finish, dim3(nb), dim3(128), 0, st, n, v.rcs_blocks, dpart, dth,
                       dph, v.g.k, dsig);
    if ((e = hipGetLastError()) != hipSuccess) s = fail_hip(e, "k_rcs_finish");
  }
  if (!s && ((e = hipMemcpyAsync(sigma, dsig, (size_t)n * 2 * sizeof(double),
                                 hipMemcpyDeviceToHost, st)) != hipSuccess ||
             (e = hipStreamSynchronize(st)) != hipSuccess))
    s = fail_hip(e, "result copy");
  if (prev != v.device) (void)hipSetDevice(prev);
  return s;
}
