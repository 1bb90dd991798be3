// C ABI of the cavity solver: argument validation, plan (sizes, device memory, FFT
// tables), the host-orchestrated preconditioned GMRES over the device kernels, and the
// inspection entry points.  See include/cavity.h for the contract of each function.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "cavity.h"
#include "kernels.hpp"

using cav::zd;

namespace {

thread_local std::string g_err;

int fail(int status, const std::string& msg) {
  g_err = msg;
  return status;
}

#define HIPCHK(expr)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(CAVITY_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));   \
  } while (0)

bool is_5smooth(long long n) {
  if (n < 1) return false;
  for (int p : {2, 3, 5})
    while (n % p == 0) n /= p;
  return n == 1;
}

int next_5smooth(long long n) {
  if (n < 1) n = 1;
  while (!is_5smooth(n)) ++n;
  return (int)n;
}

cav::FftPlan make_fft_plan(int n) {
  cav::FftPlan p{};
  p.n = n;
  p.nst = 0;
  int m = n;
  while (m % 4 == 0) { p.radix[p.nst++] = 4; m /= 4; }
  while (m % 2 == 0) { p.radix[p.nst++] = 2; m /= 2; }
  while (m % 3 == 0) { p.radix[p.nst++] = 3; m /= 3; }
  while (m % 5 == 0) { p.radix[p.nst++] = 5; m /= 5; }
  return p;
}

}  // namespace

// ---- kernel timing probe (process-wide) ------------------------------------------------
namespace cav {
namespace {
struct ProbeState {
  int which = -1;
  std::vector<hipEvent_t> pool;       // pairs: 2i = start, 2i+1 = stop
  std::vector<double> bytes;          // per recorded launch
  size_t used = 0;                    // launches recorded
  bool overflow = false;
};
ProbeState g_probe;
}  // namespace

void probe_begin(int id, hipStream_t st) {
  if (id != g_probe.which) return;
  if (2 * g_probe.used + 1 >= g_probe.pool.size()) {
    g_probe.overflow = true;
    return;
  }
  (void)hipEventRecord(g_probe.pool[2 * g_probe.used], st);
}

void probe_end(int id, hipStream_t st, double bytes) {
  if (id != g_probe.which) return;
  if (2 * g_probe.used + 1 >= g_probe.pool.size()) return;
  (void)hipEventRecord(g_probe.pool[2 * g_probe.used + 1], st);
  g_probe.bytes.push_back(bytes);
  ++g_probe.used;
}
}  // namespace cav

struct cavity_plan_s {
  cav::Geo g{};
  cav::Trig trig{};
  cavity_opts opts{};
  hipStream_t st = nullptr;
  bool layered = false;
  int nlayers = 1;
  double R = 0.0;
  std::vector<void*> allocs;
  size_t bytes = 0;
  // device data
  zd *khat = nullptr, *rho_d = nullptr, *T = nullptr, *rho_n = nullptr;
  zd *pi_d = nullptr, *theta_d = nullptr, *pi_n = nullptr, *pinv = nullptr, *diag = nullptr;
  double* pivmin = nullptr;
  int* node_code = nullptr;
  zd *kappa2 = nullptr, *ratio = nullptr;
  zd *X = nullptr, *Y = nullptr, *S = nullptr;
  zd *V = nullptr, *w = nullptr, *bvec = nullptr, *r = nullptr;
  zd* xsol = nullptr;
  int nsol_cap = 0, nsol = 0;
  zd *dpart = nullptr, *dh = nullptr;
  double *dnpart = nullptr, *dnorm = nullptr;
  zd* tbuf = nullptr;
  int synth_chunk = 1;
  zd* dy = nullptr;
  // pinned host staging
  zd* hh = nullptr;
  double* hn = nullptr;
  int nblk_red = 256;
  cavity_info info{};
  hipEvent_t ev0 = nullptr, ev1 = nullptr;

  long long nvec() const { return 3LL * g.NM; }
};

namespace {

template <typename T>
int dalloc(cavity_plan p, T** ptr, size_t count) {
  void* q = nullptr;
  const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
  hipError_t e = hipMalloc(&q, bytes);
  if (e != hipSuccess) {
    *ptr = nullptr;
    return fail(CAVITY_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
  }
  p->allocs.push_back(q);
  p->bytes += bytes;
  *ptr = static_cast<T*>(q);
  return CAVITY_OK;
}

void release(cavity_plan p) {
  if (!p) return;
  if (p->st) (void)hipStreamSynchronize(p->st);
  for (void* q : p->allocs) (void)hipFree(q);
  p->allocs.clear();
  if (p->hh) (void)hipHostFree(p->hh);
  if (p->hn) (void)hipHostFree(p->hn);
  if (p->ev0) (void)hipEventDestroy(p->ev0);
  if (p->ev1) (void)hipEventDestroy(p->ev1);
  delete p;
}

double elapsed_ms(cavity_plan p) {
  float ms = 0.f;
  (void)hipEventSynchronize(p->ev1);
  (void)hipEventElapsedTime(&ms, p->ev0, p->ev1);
  return ms;
}

int upload_fft(cavity_plan p, int n, cav::Fft* out) {
  out->p = make_fft_plan(n);
  std::vector<zd> tw(n);
  const long double two_pi = 6.283185307179586476925286766559L;
  for (int t = 0; t < n; ++t) {
    const long double ang = -two_pi * (long double)t / (long double)n;
    tw[t] = cav::mk((double)cosl(ang), (double)sinl(ang));
  }
  zd* d = nullptr;
  int s = dalloc(p, &d, n);
  if (s) return s;
  HIPCHK(hipMemcpy(d, tw.data(), n * sizeof(zd), hipMemcpyHostToDevice));
  out->tw = d;
  return CAVITY_OK;
}

size_t footprint(const cav::Geo& g, bool layered, int restart, int chunk) {
  const size_t z = sizeof(zd);
  const size_t NM = g.NM;
  size_t b = 0;
  b += (size_t)g.P1 * g.P2 * z;                       // spectrum
  b += 3 * NM * z;                                     // Schur data
  b += (size_t)(g.Nz + 1) * NM * z * (layered ? 3 : 2);  // profiles
  b += 12 * NM * z;                                    // preconditioner + diagonals
  b += NM * sizeof(double);
  b += 2 * 3 * (size_t)(g.M + 1) * g.P2 * z;           // TBC workspaces
  b += 3 * NM * z;                                     // S
  b += (size_t)(restart + 1 + 4) * 3 * NM * z;          // Krylov basis, w, b, r, x
  b += 3 * (size_t)chunk * (g.M + 1) * (g.ny + 1) * z; // synthesis staging
  b += (size_t)2 * (g.M + 1) * g.P1 * 8 + (size_t)2 * g.P2 * (g.N + 1) * 8 +
       (size_t)2 * g.P1 * (g.N + 1) * z;               // preconditioner build (transient)
  return b;
}

int run_operator(cavity_plan p, int precond, const zd* v, zd* y) {
  HIPCHK(cav::launch_operator(p->g, p->trig, p->khat, p->rho_d, p->T, p->rho_n, p->pinv, precond,
                              v, p->X, p->Y, p->S, y, p->st));
  return CAVITY_OK;
}

int device_norm2(cavity_plan p, const zd* v, double* out) {
  HIPCHK(cav::launch_norm2(v, p->nvec(), p->dnpart, p->nblk_red, p->dnorm, p->st));
  HIPCHK(hipMemcpyAsync(p->hn, p->dnorm, sizeof(double), hipMemcpyDeviceToHost, p->st));
  HIPCHK(hipStreamSynchronize(p->st));
  *out = p->hn[0];
  return CAVITY_OK;
}

// Right-preconditioned restarted GMRES with classical Gram-Schmidt applied twice.
int gmres(cavity_plan p, zd* x) {
  const long long n = p->nvec();
  const int restart = p->opts.restart;
  const double tol = p->opts.tol;
  HIPCHK(hipMemsetAsync(x, 0, n * sizeof(zd), p->st));
  double bn2 = 0;
  int s = device_norm2(p, p->bvec, &bn2);
  if (s) return s;
  const double bn = std::sqrt(bn2);
  p->info.last_iterations = 0;
  p->info.last_rel_residual = 0.0;
  if (bn == 0.0) return CAVITY_OK;
  std::vector<std::complex<double>> H((size_t)(restart + 1) * restart), cs(restart), sn(restart),
      gv(restart + 1), y(restart);
  int total = 0;
  bool first = true;
  double relres = 1.0;
  while (true) {
    zd* v0 = p->V;
    if (first) {
      HIPCHK(hipMemcpyAsync(v0, p->bvec, n * sizeof(zd), hipMemcpyDeviceToDevice, p->st));
    } else {
      if ((s = run_operator(p, 0, x, p->w))) return s;
      HIPCHK(cav::launch_sub(p->bvec, p->w, v0, n, p->st));
    }
    double beta2 = 0;
    if ((s = device_norm2(p, v0, &beta2))) return s;
    const double beta = std::sqrt(beta2);
    relres = beta / bn;
    if (relres <= tol || total >= p->opts.max_iter) break;
    first = false;
    HIPCHK(cav::launch_scale_copy(v0, p->dnorm, v0, n, p->st));
    std::fill(gv.begin(), gv.end(), 0.0);
    gv[0] = beta;
    int jdone = 0;
    for (int j = 0; j < restart; ++j) {
      zd* vj = p->V + (long long)j * n;
      zd* vn = p->V + (long long)(j + 1) * n;
      if ((s = run_operator(p, 1, vj, p->w))) return s;
      const int nv = j + 1;
      for (int pass = 0; pass < 2; ++pass) {
        zd* hcol = p->dh + pass * 256;
        HIPCHK(cav::launch_dots(p->V, n, nv, p->w, n, p->dpart, p->nblk_red, hcol, p->st));
        HIPCHK(cav::launch_update(p->V, n, nv, hcol, p->w, n, p->st));
      }
      HIPCHK(cav::launch_norm2(p->w, n, p->dnpart, p->nblk_red, p->dnorm, p->st));
      HIPCHK(cav::launch_scale_copy(p->w, p->dnorm, vn, n, p->st));
      HIPCHK(hipMemcpyAsync(p->hh, p->dh, 512 * sizeof(zd), hipMemcpyDeviceToHost, p->st));
      HIPCHK(hipMemcpyAsync(p->hn, p->dnorm, sizeof(double), hipMemcpyDeviceToHost, p->st));
      HIPCHK(hipStreamSynchronize(p->st));
      auto Hc = [&](int i) -> std::complex<double>& { return H[(size_t)j * (restart + 1) + i]; };
      for (int i = 0; i < nv; ++i)
        Hc(i) = std::complex<double>(p->hh[i].re + p->hh[256 + i].re,
                                     p->hh[i].im + p->hh[256 + i].im);
      Hc(j + 1) = std::sqrt(std::max(p->hn[0], 0.0));
      for (int i = 0; i < j; ++i) {
        const std::complex<double> t = cs[i] * Hc(i) + sn[i] * Hc(i + 1);
        Hc(i + 1) = -std::conj(sn[i]) * Hc(i) + std::conj(cs[i]) * Hc(i + 1);
        Hc(i) = t;
      }
      const double den = std::sqrt(std::norm(Hc(j)) + std::norm(Hc(j + 1)));
      if (den == 0.0) {
        cs[j] = 1.0;
        sn[j] = 0.0;
      } else {
        cs[j] = std::conj(Hc(j)) / den;
        sn[j] = std::conj(Hc(j + 1)) / den;
      }
      Hc(j) = den;
      Hc(j + 1) = 0.0;
      gv[j + 1] = -std::conj(sn[j]) * gv[j];
      gv[j] = cs[j] * gv[j];
      ++total;
      jdone = j + 1;
      if (std::abs(gv[j + 1]) <= tol * bn || total >= p->opts.max_iter || den == 0.0) break;
    }
    // back-substitution for y on the jdone x jdone triangle
    for (int i = jdone - 1; i >= 0; --i) {
      std::complex<double> acc = gv[i];
      for (int c = i + 1; c < jdone; ++c) acc -= H[(size_t)c * (restart + 1) + i] * y[c];
      y[i] = acc / H[(size_t)i * (restart + 1) + i];
    }
    std::vector<zd> yh(jdone);
    for (int i = 0; i < jdone; ++i) yh[i] = cav::mk(y[i].real(), y[i].imag());
    HIPCHK(hipMemcpyAsync(p->dy, yh.data(), jdone * sizeof(zd), hipMemcpyHostToDevice, p->st));
    HIPCHK(cav::launch_combine(p->g, p->V, n, jdone, p->dy, p->pinv, x, p->st));
    HIPCHK(hipStreamSynchronize(p->st));
  }
  p->info.last_iterations = total;
  p->info.last_rel_residual = relres;
  if (relres > tol) return fail(CAVITY_ENOCONV, "GMRES did not reach the tolerance");
  return CAVITY_OK;
}

void wave_setup(double k, double theta, double phi, int pol, cav::Wave* wv) {
  const double st = std::sin(theta), ct = std::cos(theta), sp = std::sin(phi), cp = std::cos(phi);
  wv->alpha1 = -k * st * cp;
  wv->alpha2 = -k * st * sp;
  wv->beta = k * ct;
  // theta-hat = (ct cp, ct sp, -st), phi-hat = (-sp, cp, 0)
  if (pol == CAVITY_TM) {
    wv->p1 = ct * cp; wv->p2 = ct * sp; wv->p3 = -st;
  } else {
    wv->p1 = -sp; wv->p2 = cp; wv->p3 = 0.0;
  }
}

int ensure_solutions(cavity_plan p, int count) {
  if (count <= p->nsol_cap) return CAVITY_OK;
  zd* nx = nullptr;
  int s = dalloc(p, &nx, (size_t)count * p->nvec());
  if (s) return s;
  if (p->xsol && p->nsol > 0)
    HIPCHK(hipMemcpyAsync(nx, p->xsol, (size_t)p->nsol * p->nvec() * sizeof(zd),
                          hipMemcpyDeviceToDevice, p->st));
  p->xsol = nx;
  p->nsol_cap = count;
  return CAVITY_OK;
}

int solve_one(cavity_plan p, double theta, double phi, int pol, int slot, cavity_c128* E_out,
              cavity_c128* ap_out) {
  if (!(theta >= 0.0 && theta <= 0.5 * M_PI + 1e-12) || !std::isfinite(phi) ||
      (pol != CAVITY_TM && pol != CAVITY_TE))
    return fail(CAVITY_EINVAL, "theta must lie in [0, pi/2], phi finite, pol TM or TE");
  cav::Wave wv;
  wave_setup(p->g.k, theta, phi, pol, &wv);
  HIPCHK(hipEventRecord(p->ev0, p->st));
  HIPCHK(cav::launch_rhs(p->g, wv, p->bvec, p->st));
  HIPCHK(hipEventRecord(p->ev1, p->st));
  p->info.ms_rhs = elapsed_ms(p);
  zd* x = p->xsol + (long long)slot * p->nvec();
  HIPCHK(hipEventRecord(p->ev0, p->st));
  int status = gmres(p, x);
  if (status != CAVITY_OK && status != CAVITY_ENOCONV) return status;
  HIPCHK(hipEventRecord(p->ev1, p->st));
  p->info.ms_krylov = elapsed_ms(p);
  if (E_out) {
    HIPCHK(hipEventRecord(p->ev0, p->st));
    for (int j0 = 0; j0 <= p->g.Nz; j0 += p->synth_chunk) {
      const int j1 = std::min(p->g.Nz + 1, j0 + p->synth_chunk);
      HIPCHK(cav::launch_synthesis(p->g, p->trig, p->pi_d, p->layered ? p->theta_d : nullptr,
                                   p->pi_n, x, j0, j1, p->tbuf, reinterpret_cast<zd*>(E_out),
                                   p->st));
    }
    HIPCHK(hipEventRecord(p->ev1, p->st));
    p->info.ms_synthesis = elapsed_ms(p);
  }
  if (ap_out) HIPCHK(cav::launch_pack(p->g, x, reinterpret_cast<zd*>(ap_out), p->st));
  return status;
}

}  // namespace

extern "C" {

int cavity_opts_default(cavity_opts* o) {
  if (!o) return fail(CAVITY_EINVAL, "NULL opts");
  o->precision = CAVITY_FP64;
  o->tbc_oversample = 1;
  o->tol = 1e-12;
  o->max_iter = 400;
  o->restart = 60;
  o->hbm_budget = 0;
  o->stream = nullptr;
  return CAVITY_OK;
}

const char* cavity_status_string(int s) {
  switch (s) {
    case CAVITY_OK: return "ok";
    case CAVITY_EINVAL: return "invalid argument";
    case CAVITY_ENOMEM: return "out of device memory / over budget";
    case CAVITY_ERESONANT: return "resonant z-elimination pivot";
    case CAVITY_ENOCONV: return "GMRES did not converge";
    case CAVITY_EDEVICE: return "HIP device error";
    case CAVITY_ENOTIMPL: return "not implemented";
    default: return "unknown status";
  }
}

const char* cavity_last_error(void) { return g_err.c_str(); }

int cavity_plan_create(double a, double b, double c, int Nx, int Ny, int Nz,
                       const cavity_eps* eps, double k, const cavity_opts* opts,
                       cavity_plan* out) {
  if (!out) return fail(CAVITY_EINVAL, "NULL plan output");
  *out = nullptr;
  if (!(a > 0 && b > 0 && c > 0 && k > 0) || !std::isfinite(a) || !std::isfinite(b) ||
      !std::isfinite(c) || !std::isfinite(k))
    return fail(CAVITY_EINVAL, "a, b, c, k must be positive and finite");
  if (Nx < 2 || Ny < 2 || Nz < 1) return fail(CAVITY_EINVAL, "need Nx, Ny >= 2 and Nz >= 1");
  cavity_opts o;
  cavity_opts_default(&o);
  if (opts) o = *opts;
  if (o.precision != CAVITY_FP64)
    return fail(CAVITY_ENOTIMPL, "only CAVITY_FP64 precision is available");
  if (o.tbc_oversample < 1 || o.tbc_oversample > 8)
    return fail(CAVITY_EINVAL, "tbc_oversample must be in 1..8");
  if (!(o.tol > 0 && o.tol < 1) || o.max_iter < 1 || o.restart < 1 || o.restart > 200)
    return fail(CAVITY_EINVAL, "tol in (0,1), max_iter >= 1, restart in 1..200");
  const int s = o.tbc_oversample;
  if (!is_5smooth(2LL * s * Nx) || !is_5smooth(2LL * s * Ny))
    return fail(CAVITY_EINVAL, "2*s*Nx and 2*s*Ny must be products of 2, 3 and 5");
  // layers
  std::vector<int> lnz;
  std::vector<std::complex<double>> leps;
  if (eps) {
    if (eps->n_layers < 1 || !eps->layer_nz || !eps->eps_r)
      return fail(CAVITY_EINVAL, "layer stack needs n_layers >= 1 and both arrays");
    long long sum = 0;
    for (int i = 0; i < eps->n_layers; ++i) {
      if (eps->layer_nz[i] < 1) return fail(CAVITY_EINVAL, "every layer needs >= 1 interval");
      const double er = eps->eps_r[i].re, ei = eps->eps_r[i].im;
      if (!std::isfinite(er) || !std::isfinite(ei) || (er == 0.0 && ei == 0.0))
        return fail(CAVITY_EINVAL, "layer permittivity must be finite and nonzero");
      sum += eps->layer_nz[i];
      lnz.push_back(eps->layer_nz[i]);
      leps.emplace_back(er, ei);
    }
    if (sum != Nz) return fail(CAVITY_EINVAL, "layer intervals must sum to Nz");
  } else {
    lnz.push_back(Nz);
    leps.emplace_back(1.0, 0.0);
  }

  cav::Geo g{};
  g.M = Nx - 1;
  g.N = Ny - 1;
  g.Nz = Nz;
  g.NM = (g.M + 1) * (g.N + 1);
  g.nq1 = s * Nx;
  g.nq2 = s * Ny;
  g.nx = Nx;
  g.ny = Ny;
  g.a = a;
  g.b = b;
  g.h = c / Nz;
  g.k = k;
  g.hq1 = a / g.nq1;
  g.hq2 = b / g.nq2;
  const double R = std::sqrt(2.0) * std::max(a, b);
  g.P1 = next_5smooth((long long)std::ceil((a + R) / g.hq1));
  g.P2 = next_5smooth((long long)std::ceil((b + R) / g.hq2));

  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  int lds_max = 0;
  HIPCHK(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  if ((size_t)2 * std::max(g.P1, g.P2) * sizeof(zd) > (size_t)lds_max)
    return fail(CAVITY_EINVAL, "FFT box too large for one block's LDS");

  const bool layered = lnz.size() > 1;
  int chunk = 1;
  const size_t per_level = 3ull * (g.M + 1) * (g.ny + 1) * sizeof(zd);
  chunk = (int)std::max<size_t>(1, (size_t)(32u << 20) / per_level);
  chunk = std::min(chunk, Nz + 1);
  const size_t need = footprint(g, layered, o.restart, chunk);
  size_t budget = o.hbm_budget;
  if (budget == 0) {
    size_t fr = 0, tot = 0;
    HIPCHK(hipMemGetInfo(&fr, &tot));
    budget = (size_t)(0.9 * (double)fr);
  }
  if (need > budget)
    return fail(CAVITY_ENOMEM, "plan needs " + std::to_string(need) + " bytes, budget " +
                                   std::to_string(budget));

  cavity_plan p = new cavity_plan_s();
  p->g = g;
  p->opts = o;
  p->st = static_cast<hipStream_t>(o.stream);
  p->layered = layered;
  p->nlayers = (int)lnz.size();
  p->R = R;
  p->synth_chunk = chunk;
  int st = CAVITY_OK;
  auto bail = [&](int code) {
    release(p);
    return code;
  };
  if (hipEventCreate(&p->ev0) != hipSuccess || hipEventCreate(&p->ev1) != hipSuccess)
    return bail(fail(CAVITY_EDEVICE, "hipEventCreate failed"));
  if (hipHostMalloc((void**)&p->hh, 512 * sizeof(zd)) != hipSuccess ||
      hipHostMalloc((void**)&p->hn, 8 * sizeof(double)) != hipSuccess)
    return bail(fail(CAVITY_EDEVICE, "hipHostMalloc failed"));

  const long long NM = g.NM, n = 3LL * NM;
  if ((st = dalloc(p, &p->khat, (size_t)g.P1 * g.P2)) || (st = dalloc(p, &p->rho_d, NM)) ||
      (st = dalloc(p, &p->T, NM)) || (st = dalloc(p, &p->rho_n, NM)) ||
      (st = dalloc(p, &p->pi_d, (size_t)(Nz + 1) * NM)) ||
      (st = dalloc(p, &p->pi_n, (size_t)(Nz + 1) * NM)) ||
      (layered && (st = dalloc(p, &p->theta_d, (size_t)(Nz + 1) * NM))) ||
      (st = dalloc(p, &p->pinv, 9 * NM)) || (st = dalloc(p, &p->diag, 3 * NM)) ||
      (st = dalloc(p, &p->pivmin, NM)) || (st = dalloc(p, &p->node_code, Nz + 1)) ||
      (st = dalloc(p, &p->kappa2, lnz.size())) ||
      (st = dalloc(p, &p->ratio, std::max<size_t>(1, lnz.size() - 1))) ||
      (st = dalloc(p, &p->X, 3ull * (g.M + 1) * g.P2)) ||
      (st = dalloc(p, &p->Y, 3ull * (g.M + 1) * g.P2)) || (st = dalloc(p, &p->S, 3 * NM)) ||
      (st = dalloc(p, &p->V, (size_t)(o.restart + 1) * n)) || (st = dalloc(p, &p->w, n)) ||
      (st = dalloc(p, &p->bvec, n)) || (st = dalloc(p, &p->r, n)) ||
      (st = dalloc(p, &p->dpart, (size_t)p->nblk_red * 256)) || (st = dalloc(p, &p->dh, 512)) ||
      (st = dalloc(p, &p->dnpart, p->nblk_red)) || (st = dalloc(p, &p->dnorm, 8)) ||
      (st = dalloc(p, &p->dy, 256)) ||
      (st = dalloc(p, &p->tbuf, (size_t)3 * chunk * (g.M + 1) * (g.ny + 1))))
    return bail(st);
  if ((st = ensure_solutions(p, 1))) return bail(st);
  if ((st = upload_fft(p, 2 * g.nq1, &p->trig.ext1)) ||
      (st = upload_fft(p, 2 * g.nq2, &p->trig.ext2)) ||
      (st = upload_fft(p, g.P1, &p->trig.box1)) || (st = upload_fft(p, g.P2, &p->trig.box2)) ||
      (st = upload_fft(p, 2 * g.nx, &p->trig.out1)) ||
      (st = upload_fft(p, 2 * g.ny, &p->trig.out2)))
    return bail(st);

  // layer tables
  std::vector<int> code(Nz + 1, 0);
  std::vector<zd> kap(lnz.size()), rat(std::max<size_t>(1, lnz.size() - 1), cav::mk(1.0, 0.0));
  {
    int start = 0;
    for (size_t l = 0; l < lnz.size(); ++l) {
      for (int j = start + 1; j < start + lnz[l]; ++j) code[j] = (int)l;
      start += lnz[l];
      if (l + 1 < lnz.size()) {
        code[start] = -(int)(l + 1);  // interface index l -> code -(l+1)
        const std::complex<double> r = leps[l + 1] / leps[l];
        rat[l] = cav::mk(r.real(), r.imag());
      }
    }
    code[0] = 0;
    code[Nz] = (int)lnz.size() - 1;
    for (size_t l = 0; l < lnz.size(); ++l) {
      const std::complex<double> k2 = k * k * leps[l];
      kap[l] = cav::mk(k2.real(), k2.imag());
    }
  }
  if (hipMemcpy(p->node_code, code.data(), code.size() * sizeof(int), hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(p->kappa2, kap.data(), kap.size() * sizeof(zd), hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(p->ratio, rat.data(), rat.size() * sizeof(zd), hipMemcpyHostToDevice) != hipSuccess)
    return bail(fail(CAVITY_EDEVICE, "upload of layer tables failed"));

  auto chk = [&](hipError_t e, const char* what) {
    if (e != hipSuccess) {
      fail(CAVITY_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
      return false;
    }
    return true;
  };
  // spectrum (scaled for the unnormalised inverse FFT and the grid cell)
  const double scale = 1.0 / (g.hq1 * g.hq2 * (double)g.P1 * (double)g.P2);
  if (!chk(hipEventRecord(p->ev0, p->st), "event") ||
      !chk(cav::launch_spectrum(g, R, scale, p->khat, p->st), "spectrum") ||
      !chk(hipEventRecord(p->ev1, p->st), "event"))
    return bail(CAVITY_EDEVICE);
  p->info.ms_spectrum = elapsed_ms(p);
  // elimination
  cav::Layers ly{p->node_code, p->kappa2, p->ratio, layered ? 1 : 0};
  if (!chk(hipEventRecord(p->ev0, p->st), "event") ||
      !chk(cav::launch_elimination(g, ly, p->rho_d, p->T, p->rho_n, p->pi_d, p->theta_d, p->pi_n,
                                   p->pivmin, p->st),
           "elimination") ||
      !chk(hipEventRecord(p->ev1, p->st), "event"))
    return bail(CAVITY_EDEVICE);
  p->info.ms_elimination = elapsed_ms(p);
  {
    std::vector<double> pv(NM);
    if (!chk(hipMemcpy(pv.data(), p->pivmin, NM * sizeof(double), hipMemcpyDeviceToHost),
             "pivot copy"))
      return bail(CAVITY_EDEVICE);
    double mn = 1e300;
    for (double v : pv) mn = std::min(mn, v);
    p->info.min_pivot = mn;
    if (!(mn > 1e-13)) return bail(fail(CAVITY_ERESONANT, "z-elimination pivot below 1e-13"));
  }
  // preconditioner: exact diagonals of the three single-layer families
  {
    double *pw1 = nullptr, *pw2 = nullptr;
    zd* tmp = nullptr;
    void* q = nullptr;
    const size_t b1 = (size_t)2 * (g.M + 1) * g.P1 * sizeof(double);
    const size_t b2 = (size_t)2 * g.P2 * (g.N + 1) * sizeof(double);
    const size_t b3 = (size_t)2 * g.P1 * (g.N + 1) * sizeof(zd);
    if (!chk(hipMalloc(&q, b1 + b2 + b3), "preconditioner scratch")) return bail(CAVITY_ENOMEM);
    pw1 = static_cast<double*>(q);
    pw2 = reinterpret_cast<double*>(static_cast<char*>(q) + b1);
    tmp = reinterpret_cast<zd*>(static_cast<char*>(q) + b1 + b2);
    bool ok = chk(hipEventRecord(p->ev0, p->st), "event") &&
              chk(cav::launch_basis_power(g, p->trig, pw1, pw2, p->st), "basis power") &&
              chk(cav::launch_diag_contract(g, p->khat, pw1, pw2, tmp, p->diag, p->st),
                  "diagonal") &&
              chk(cav::launch_precond_build(g, p->rho_d, p->T, p->rho_n, p->diag, p->pinv, p->st),
                  "preconditioner") &&
              chk(hipEventRecord(p->ev1, p->st), "event");
    if (ok) p->info.ms_preconditioner = elapsed_ms(p);
    (void)hipStreamSynchronize(p->st);
    (void)hipFree(q);
    if (!ok) return bail(CAVITY_EDEVICE);
  }
  p->info.M = g.M;
  p->info.N = g.N;
  p->info.Nz = Nz;
  p->info.P1 = g.P1;
  p->info.P2 = g.P2;
  p->info.n_ap = (long long)(g.M + 1) * g.N + (long long)g.M * (g.N + 1) + (long long)g.M * g.N;
  p->info.unknowns = p->info.n_ap * Nz;
  p->info.device_bytes = p->bytes;
  *out = p;
  return CAVITY_OK;
}

void cavity_plan_destroy(cavity_plan p) { release(p); }

int cavity_plan_info(cavity_plan p, cavity_info* out) {
  if (!p || !out) return fail(CAVITY_EINVAL, "NULL argument");
  p->info.device_bytes = p->bytes;
  *out = p->info;
  return CAVITY_OK;
}

int cavity_solve(cavity_plan p, double theta, double phi, int pol, cavity_c128* E_out) {
  if (!p) return fail(CAVITY_EINVAL, "NULL plan");
  int s = solve_one(p, theta, phi, pol, 0, E_out, nullptr);
  if (s == CAVITY_OK || s == CAVITY_ENOCONV) p->nsol = std::max(p->nsol, 1);
  return s;
}

int cavity_solve_batch(cavity_plan p, int nrhs, const double* theta, const double* phi,
                       const int* pol, cavity_c128* E_out, cavity_c128* aperture_out) {
  if (!p || nrhs < 1 || !theta || !phi || !pol) return fail(CAVITY_EINVAL, "bad batch arguments");
  int s = ensure_solutions(p, nrhs);
  if (s) return s;
  const long long field = 3LL * (p->g.Nz + 1) * (p->g.ny + 1) * (p->g.nx + 1);
  int worst = CAVITY_OK;
  for (int i = 0; i < nrhs; ++i) {
    s = solve_one(p, theta[i], phi[i], pol[i], i, E_out ? E_out + i * field : nullptr,
                  aperture_out ? aperture_out + i * p->info.n_ap : nullptr);
    if (s != CAVITY_OK && s != CAVITY_ENOCONV) return s;
    if (s == CAVITY_ENOCONV) worst = s;
    p->nsol = std::max(p->nsol, i + 1);
  }
  return worst;
}

int cavity_aperture(cavity_plan p, int idx, cavity_c128* out_host) {
  if (!p || !out_host || idx < 0 || idx >= p->nsol) return fail(CAVITY_EINVAL, "no such solution");
  zd* tmp = nullptr;
  HIPCHK(hipMalloc(&tmp, p->info.n_ap * sizeof(zd)));
  hipError_t e = cav::launch_pack(p->g, p->xsol + (long long)idx * p->nvec(), tmp, p->st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(out_host, tmp, p->info.n_ap * sizeof(zd), hipMemcpyDeviceToHost, p->st);
  if (e == hipSuccess) e = hipStreamSynchronize(p->st);
  (void)hipFree(tmp);
  if (e != hipSuccess) return fail(CAVITY_EDEVICE, hipGetErrorString(e));
  return CAVITY_OK;
}

int cavity_rcs(cavity_plan p, int idx, int n_obs, const double* th, const double* ph,
               double* sigma) {
  if (!p || idx < 0 || idx >= p->nsol || n_obs < 0 || (n_obs > 0 && (!th || !ph || !sigma)))
    return fail(CAVITY_EINVAL, "bad rcs arguments");
  const int nblk = 64;
  std::vector<zd> part(2 * nblk);
  const double k = p->g.k;
  const zd* x = p->xsol + (long long)idx * p->nvec();
  for (int i = 0; i < n_obs; ++i) {
    const double st = std::sin(th[i]), ct = std::cos(th[i]), sp = std::sin(ph[i]),
                 cp = std::cos(ph[i]);
    HIPCHK(cav::launch_rcs_partial(p->g, x, k * st * cp, k * st * sp, p->dpart, nblk, p->st));
    HIPCHK(hipMemcpyAsync(part.data(), p->dpart, 2 * nblk * sizeof(zd), hipMemcpyDeviceToHost,
                          p->st));
    HIPCHK(hipStreamSynchronize(p->st));
    std::complex<double> e1 = 0.0, e2 = 0.0;
    for (int b = 0; b < nblk; ++b) {
      e1 += std::complex<double>(part[2 * b].re, part[2 * b].im);
      e2 += std::complex<double>(part[2 * b + 1].re, part[2 * b + 1].im);
    }
    // L = (-E^2, E^1, 0); sigma_theta = k^2/pi |phi^.L|^2, sigma_phi = k^2/pi |theta^.L|^2
    const std::complex<double> L1 = -e2, L2 = e1;
    const std::complex<double> phiL = -sp * L1 + cp * L2;
    const std::complex<double> thL = ct * cp * L1 + ct * sp * L2;
    sigma[2 * i] = k * k / M_PI * std::norm(phiL);
    sigma[2 * i + 1] = k * k / M_PI * std::norm(thL);
  }
  return CAVITY_OK;
}

int cavity_probe_kernel(int which, int capacity) {
  using cav::g_probe;
  for (hipEvent_t e : g_probe.pool) (void)hipEventDestroy(e);
  g_probe = cav::ProbeState();
  if (which < 0) return CAVITY_OK;
  if (which >= cav::K_COUNT || capacity < 1) return fail(CAVITY_EINVAL, "bad probe arguments");
  g_probe.pool.resize(2 * (size_t)capacity + 2);
  for (auto& e : g_probe.pool) HIPCHK(hipEventCreate(&e));
  g_probe.which = which;
  return CAVITY_OK;
}

int cavity_probe_read(int* launches, double* total_ms, double* total_bytes) {
  using cav::g_probe;
  if (!launches || !total_ms || !total_bytes) return fail(CAVITY_EINVAL, "NULL argument");
  if (g_probe.overflow) return fail(CAVITY_ENOMEM, "probe capacity exceeded");
  double ms = 0.0, by = 0.0;
  for (size_t i = 0; i < g_probe.used; ++i) {
    HIPCHK(hipEventSynchronize(g_probe.pool[2 * i + 1]));
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, g_probe.pool[2 * i], g_probe.pool[2 * i + 1]));
    ms += t;
    by += g_probe.bytes[i];
  }
  *launches = (int)g_probe.used;
  *total_ms = ms;
  *total_bytes = by;
  return CAVITY_OK;
}

// ---- inspection entry points ---------------------------------------------------------

static int copy_out(cavity_plan p, const zd* d, cavity_c128* h, size_t count) {
  HIPCHK(hipStreamSynchronize(p->st));
  HIPCHK(hipMemcpy(h, d, count * sizeof(zd), hipMemcpyDeviceToHost));
  return CAVITY_OK;
}

int cavity_debug_columns(cavity_plan p, cavity_c128* rho_d, cavity_c128* T, cavity_c128* rho_n) {
  if (!p || !rho_d || !T || !rho_n) return fail(CAVITY_EINVAL, "NULL argument");
  int s;
  if ((s = copy_out(p, p->rho_d, rho_d, p->g.NM)) || (s = copy_out(p, p->T, T, p->g.NM)) ||
      (s = copy_out(p, p->rho_n, rho_n, p->g.NM)))
    return s;
  return CAVITY_OK;
}

int cavity_debug_profiles(cavity_plan p, cavity_c128* pi_d, cavity_c128* theta_d,
                          cavity_c128* pi_n) {
  if (!p || !pi_d || !theta_d || !pi_n) return fail(CAVITY_EINVAL, "NULL argument");
  const size_t cnt = (size_t)(p->g.Nz + 1) * p->g.NM;
  int s;
  if ((s = copy_out(p, p->pi_d, pi_d, cnt)) || (s = copy_out(p, p->pi_n, pi_n, cnt))) return s;
  if (p->layered) {
    if ((s = copy_out(p, p->theta_d, theta_d, cnt))) return s;
  } else {
    std::memset(theta_d, 0, cnt * sizeof(cavity_c128));
  }
  return CAVITY_OK;
}

int cavity_debug_spectrum(cavity_plan p, cavity_c128* khat) {
  if (!p || !khat) return fail(CAVITY_EINVAL, "NULL argument");
  const size_t cnt = (size_t)p->g.P1 * p->g.P2;
  int s = copy_out(p, p->khat, khat, cnt);
  if (s) return s;
  const double unscale = p->g.hq1 * p->g.hq2 * (double)p->g.P1 * (double)p->g.P2;
  for (size_t i = 0; i < cnt; ++i) {
    khat[i].re *= unscale;
    khat[i].im *= unscale;
  }
  return CAVITY_OK;
}

int cavity_debug_tbc(cavity_plan p, int family, const cavity_c128* in, cavity_c128* out) {
  if (!p || !in || !out || family < 0 || family > 2) return fail(CAVITY_EINVAL, "bad arguments");
  const size_t NM = p->g.NM;
  HIPCHK(hipMemcpy(p->r, in, NM * sizeof(zd), hipMemcpyHostToDevice));
  HIPCHK(cav::launch_single_family(p->g, p->trig, p->khat, family, p->r, p->X, p->Y, p->w, p->st));
  return copy_out(p, p->w, out, NM);
}

int cavity_debug_operator(cavity_plan p, const cavity_c128* in, cavity_c128* out) {
  if (!p || !in || !out) return fail(CAVITY_EINVAL, "NULL argument");
  const size_t n = 3 * (size_t)p->g.NM;
  HIPCHK(hipMemcpy(p->r, in, n * sizeof(zd), hipMemcpyHostToDevice));
  int s = run_operator(p, 0, p->r, p->w);
  if (s) return s;
  return copy_out(p, p->w, out, n);
}

int cavity_debug_rhs(cavity_plan p, double theta, double phi, int pol, cavity_c128* g1,
                     cavity_c128* g2) {
  if (!p || !g1 || !g2) return fail(CAVITY_EINVAL, "NULL argument");
  cav::Wave wv;
  wave_setup(p->g.k, theta, phi, pol, &wv);
  HIPCHK(cav::launch_rhs(p->g, wv, p->r, p->st));
  int s;
  if ((s = copy_out(p, p->r, g1, p->g.NM)) || (s = copy_out(p, p->r + p->g.NM, g2, p->g.NM)))
    return s;
  return CAVITY_OK;
}

}  // extern "C"
