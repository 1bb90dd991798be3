// C ABI of the cavity solver: argument validation, plan (sizes, device memory, FFT
// tables), the host-orchestrated preconditioned GMRES over the device kernels, and the
// inspection entry points.  See include/cavity.h for the contract of each function.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <string>
#include <vector>

#include "cavity.h"
#include "kernels.hpp"
#include "runtime.hpp"

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

// Stages of radix at most 8 (the kernels compiled for radices up to 8 hold about half the
// registers) or up to the largest compiled radix, chosen for the six transform lengths of a
// plan together: one length that needs the larger radices puts every kernel of the plan in
// its larger form.  All six lengths take radices up to 8 when each factors that way in at
// most one stage more than with the larger radices, the extra stage allowed on lengths up
// to 1000 points (the registers saved outweigh one more LDS round trip there: cavities of
// 2, 4 and 12 wavelengths at 32 nodes per wavelength, lengths 128-960, solve 3-11 % faster;
// with 1024 and 1250 points the extra stage cost 3 %).  Otherwise each length takes
// radices up to 8 only when they need no more stages than the larger ones.
constexpr int kExtraStageMaxLen = 1000;
// The planner's two factorisations of a length (radices up to 8, up to the largest
// compiled radix), kept for the process: the searches take 1-8 us per length and every
// plan creation asks for its six lengths several times.
struct FftPlanPair {
  cav::FftPlan small, big;
};
const FftPlanPair& fft_plans(int n) {
  static std::mutex mu;
  static std::map<int, FftPlanPair> cache;   // entries are never erased
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(n);
  if (it == cache.end())
    it = cache.emplace(n, FftPlanPair{cav::plan_fft(n, cav::kSmallRadix),
                                      cav::plan_fft(n, cav::kMaxRadix)}).first;
  return it->second;
}
bool small_radix_plans(const int* len, int count) {
  for (int i = 0; i < count; ++i) {
    if (len[i] <= 1) continue;
    const FftPlanPair& pp = fft_plans(len[i]);
    if (pp.small.nst == 0 || pp.small.nst > pp.big.nst + (len[i] <= kExtraStageMaxLen ? 1 : 0))
      return false;
  }
  return true;
}
cav::FftPlan make_fft_plan(int n, bool small_radices) {
  const FftPlanPair& pp = fft_plans(n);
  if (small_radices || n <= 1) return pp.small;
  return pp.small.nst > 0 && pp.small.nst <= pp.big.nst ? pp.small : pp.big;
}
int plan_max_radix(const cav::FftPlan& p) {
  int r = 1;
  for (int s = 0; s < p.nst; ++s) r = std::max(r, p.radix[s]);
  return r;
}

// LDS of one workgroup on gfx950 (160 KiB); every FFT kernel needs two buffers of its
// longest transform for at least one column.
constexpr size_t kMaxLdsPerBlock = 160 * 1024;

// Largest basis size for which the first Gram-Schmidt update and the second pass's dot
// products share one pass over the basis (the dot kernel's group of vectors).
constexpr int kFusedGsMax = 16;

// Blocks per right-hand side of the fused update + norm pass of the Arnoldi step.
constexpr int kNormBlocks = 1024;

// Blocks per right-hand side (and group of basis vectors) of the dot-product pass: four
// elements per thread (loaded together), 64 to kNormBlocks blocks.
int dot_blocks(long long n) {
  return (int)std::max<long long>(64, std::min<long long>(kNormBlocks, (n + 1023) / 1024));
}

// Most blocks per query of the aperture-transform reduction behind the RCS.
constexpr int kRcsBlocks = 64;
int rcs_blocks(long long NM) {
  return (int)std::max<long long>(1, std::min<long long>(kRcsBlocks, (NM + 255) / 256));
}

// Direct solve limits on n = 3 Nx Ny: the largest system it accepts, and the largest it
// picks by itself (for calls with at least kDenseAutoRhs right-hand sides).
constexpr long long kDenseMax = 4096;
constexpr long long kDenseAuto = 2048;
constexpr int kDenseAutoRhs = 32;
// Right-hand sides per product with the inverse (and per residual check).
constexpr int kDenseGroup = 64;

// Device bytes of the staging slab between the two synthesis passes, per 8 right-hand
// sides of the lockstep batch (at most 4 such units); the (field, level) pairs of one slab
// are synthesised by one pair of launches, and the fewer the launches, the fewer times
// the row pass re-reads the aperture solutions.
constexpr size_t kSynthStagingBytes = (size_t)256 << 20;

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

bool g_probe_active() { return g_probe.which >= 0; }

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

// ---- device memory: one arena per plan part, with a process-wide cache -------------
// Freed arenas are kept (up to a bound) and handed to later plans of similar size, so
// creating plans repeatedly (new geometries, served requests) does not pay hipMalloc.
namespace {

struct CachedBlock {
  void* ptr;
  size_t bytes;
  int device;
};
std::mutex g_cache_mu;
std::vector<CachedBlock> g_cache;
size_t g_cache_bytes = 0;
const size_t kCacheLimit = (size_t)32 << 30;

int arena_acquire(size_t bytes, void** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    int best = -1;
    for (size_t i = 0; i < g_cache.size(); ++i) {
      const CachedBlock& b = g_cache[i];
      if (b.device == dev && b.bytes >= bytes && b.bytes <= 2 * bytes + ((size_t)64 << 20) &&
          (best < 0 || b.bytes < g_cache[best].bytes))
        best = (int)i;
    }
    if (best >= 0) {
      *out = g_cache[best].ptr;
      g_cache_bytes -= g_cache[best].bytes;
      g_cache.erase(g_cache.begin() + best);
      return CAVITY_OK;
    }
  }
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, bytes);
  if (e != hipSuccess) {
    // drop the cache and retry once
    std::vector<CachedBlock> drop;
    {
      std::lock_guard<std::mutex> lk(g_cache_mu);
      drop.swap(g_cache);
      g_cache_bytes = 0;
    }
    for (auto& b : drop) (void)hipFree(b.ptr);
    e = hipMalloc(&q, bytes);
    if (e != hipSuccess)
      return fail(CAVITY_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
  }
  *out = q;
  return CAVITY_OK;
}

// The caller guarantees that no work on the block is pending.
void arena_release(void* ptr, size_t bytes) {
  if (!ptr) return;
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::vector<CachedBlock> drop;
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    g_cache.push_back({ptr, bytes, dev});
    g_cache_bytes += bytes;
    while (g_cache_bytes > kCacheLimit && !g_cache.empty()) {
      drop.push_back(g_cache.front());
      g_cache_bytes -= g_cache.front().bytes;
      g_cache.erase(g_cache.begin());
    }
  }
  for (auto& b : drop) (void)hipFree(b.ptr);
}

// ---- events and pinned host buffers: process-wide free lists -----------------------
// A served request creates a plan and later drops it; the plan's events (phase timers, one
// per Arnoldi step for the convergence polls) and its pinned flag buffers come from these
// lists, so creating plans repeatedly does not pay hipEventCreate and hipHostMalloc
// (about 0.1 ms per plan together).  Returned only when no work on them is pending.
std::mutex g_pool_mu;
struct PooledEvent {
  hipEvent_t ev;
  int device;
  bool timing;
};
std::vector<PooledEvent> g_events;
struct PooledPinned {
  void* ptr;
  size_t bytes;
};
std::vector<PooledPinned> g_pinned;

hipError_t event_get(hipEvent_t* out, bool timing) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    for (size_t i = g_events.size(); i-- > 0;)
      if (g_events[i].device == dev && g_events[i].timing == timing) {
        *out = g_events[i].ev;
        g_events.erase(g_events.begin() + i);
        return hipSuccess;
      }
  }
  return timing ? hipEventCreate(out) : hipEventCreateWithFlags(out, hipEventDisableTiming);
}

void event_put(hipEvent_t ev, bool timing) {
  if (!ev) return;
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(g_pool_mu);
  g_events.push_back({ev, dev, timing});
}

hipError_t pinned_get(size_t bytes, void** out) {
  {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    for (size_t i = g_pinned.size(); i-- > 0;)
      if (g_pinned[i].bytes == bytes) {
        *out = g_pinned[i].ptr;
        g_pinned.erase(g_pinned.begin() + i);
        return hipSuccess;
      }
  }
  return hipHostMalloc(out, bytes);
}

void pinned_put(void* ptr, size_t bytes) {
  if (!ptr) return;
  std::lock_guard<std::mutex> lk(g_pool_mu);
  g_pinned.push_back({ptr, bytes});
}

// Two-phase layout: register every buffer, then bind them into one arena.
struct Layout {
  struct Item {
    void** slot;
    size_t offset;
  };
  std::vector<Item> items;
  size_t bytes = 0;
  template <typename T>
  void add(T** slot, size_t count) {
    bytes = (bytes + 255) & ~(size_t)255;
    items.push_back({reinterpret_cast<void**>(slot), bytes});
    bytes += std::max<size_t>(count, 1) * sizeof(T);
  }
  void bind(void* base) const {
    for (const Item& it : items) *it.slot = static_cast<char*>(base) + it.offset;
  }
};

struct Arena {
  void* ptr = nullptr;
  size_t bytes = 0;
};

}  // namespace

namespace cav {
int device_block_acquire(size_t bytes, void** out) { return arena_acquire(bytes, out); }
void device_block_release(void* ptr, size_t bytes) { arena_release(ptr, bytes); }
int record_error(int status, const char* msg) { return fail(status, msg); }
}  // namespace cav

struct cavity_plan_s {
  cav::Geo g{};
  cav::Trig trig{};
  cavity_opts opts{};
  // column data the Krylov kernels read: this plan's own (one cavity), or those of a
  // group of plans gathered for a group solve
  cav::Cols cols{};
  std::vector<double> group_h;       // aperture step of each right-hand side of a group solve
  Arena group_arena;                 // gathered column data of a group solve
  hipStream_t st = nullptr;
  int device = 0;                    // device current at plan creation (owns all its memory)
  bool layered = false;
  int nlayers = 1;
  double R = 0.0;
  Arena plan_arena, work_arena, sol_arena;
  // plan data
  zd *khat = nullptr, *rho_d = nullptr, *T = nullptr, *rho_n = nullptr;
  zd *pi_d = nullptr, *theta_d = nullptr, *pi_n = nullptr, *pinv = nullptr, *diag = nullptr;
  double *pivmin = nullptr, *dmin = nullptr;
  int* node_code = nullptr;
  zd *kappa2 = nullptr, *ratio = nullptr;
  double* hl = nullptr;   // grid step per layer
  cav::zf* khat_f = nullptr;   // single-precision spectrum for the mixed-precision inner solve
  double *pw1 = nullptr, *pw2 = nullptr;
  zd* ctmp = nullptr;
  zd* tbuf = nullptr;
  zd* r = nullptr;          // inspection scratch (max(3 NM, P1 P2))
  zd* dbg_out = nullptr;    // inspection scratch (3 NM)
  cav::Wave* dwave1 = nullptr;
  int synth_chunk = 1;
  // solve workspace (sized for nbwork right-hand sides)
  int nbwork = 0;
  zd *X = nullptr, *Y = nullptr, *S = nullptr;
  zd *V = nullptr, *w = nullptr, *bvec = nullptr;
  zd* zb = nullptr;          // preconditioned current basis vector P^{-1} v_j per rhs
  zd* rbuf = nullptr;        // residual at the start of a cycle, per rhs
  zd* dpart = nullptr;
  double* dnpart = nullptr;
  zd* h2 = nullptr;
  cav::Krylov kv{};
  cav::Wave* dwaves = nullptr;
  // solutions
  zd* xsol = nullptr;
  int nsol_cap = 0, nsol = 0;
  // pinned host staging
  int* hflags = nullptr;
  double* hn = nullptr;
  double* hratio = nullptr;   // pinned, host-mapped: per step and rhs, |g_{j+1}| / threshold
  int nblk_red = 128;                // blocks per rhs of the dot-product and norm passes
  cavity_info info{};
  // phase timers, resolved lazily: spectrum, elimination, preconditioner, rhs, krylov, synth
  hipEvent_t ev[12] = {};
  bool ev_used[6] = {};
  std::vector<hipEvent_t> poll_ev;   // one per Arnoldi step of a cycle (convergence polling)
  // Arnoldi steps captured as HIP graphs, keyed by (lockstep group size, step index); valid
  // while the solve workspace stays where it is.  Captured on a private stream.
  hipStream_t cap_st = nullptr;
  std::map<long long, hipGraphExec_t> step_graphs;
  // direct solve: (P A)^{-1} column-major and the row permutation, built on first use
  Arena dense_arena;
  Arena rcs_arena;                   // RCS queries and partial sums
  // spectral TBC operator: trial-function transforms (plan) and the P1 x P2 product
  // workspace per right-hand side and family (solve)
  Arena spec_arena;
  cav::SpecMats spec{};
  zd* U = nullptr;
  bool use_spec() const { return opts.tbc_operator == CAVITY_TBC_SPEC; }
  zd* dense_F = nullptr;
  int* dense_perm = nullptr;
  bool dense_now = false;            // the current solve call uses the direct solve

  long long nvec() const { return 3LL * g.NM; }
};

namespace cav {
int plan_view(cavity_plan p, PlanView* out) {
  if (!p || !out) return fail(CAVITY_EINVAL, "NULL argument");
  out->g = p->g;
  out->xsol = p->xsol;
  out->nvec = p->nvec();
  out->nsol = p->nsol;
  out->stream = p->st;
  out->device = p->device;
  out->rcs_blocks = rcs_blocks(p->g.NM);
  return CAVITY_OK;
}
int plan_set_stream(cavity_plan p, hipStream_t st) {
  if (!p) return fail(CAVITY_EINVAL, "NULL plan");
  p->st = st;
  p->opts.stream = st;
  return CAVITY_OK;
}
}  // namespace cav

namespace {

// Sizes of a plan's pinned host buffers: per-step convergence flags and residual ratios for
// up to 64 right-hand sides, and a few doubles for small read-backs.
size_t flag_bytes(int restart) { return (size_t)(restart + 2) * 64 * sizeof(int); }
size_t ratio_bytes(int restart) { return (size_t)(restart + 2) * 64 * sizeof(double); }
size_t norm_bytes() { return 64 * sizeof(double); }

void release(cavity_plan p) {
  if (!p) return;
  if (p->st) (void)hipStreamSynchronize(p->st);
  else (void)hipDeviceSynchronize();
  arena_release(p->plan_arena.ptr, p->plan_arena.bytes);
  arena_release(p->work_arena.ptr, p->work_arena.bytes);
  arena_release(p->sol_arena.ptr, p->sol_arena.bytes);
  arena_release(p->dense_arena.ptr, p->dense_arena.bytes);
  arena_release(p->rcs_arena.ptr, p->rcs_arena.bytes);
  arena_release(p->spec_arena.ptr, p->spec_arena.bytes);
  arena_release(p->group_arena.ptr, p->group_arena.bytes);
  pinned_put(p->hflags, flag_bytes(p->opts.restart));
  pinned_put(p->hn, norm_bytes());
  pinned_put(p->hratio, ratio_bytes(p->opts.restart));
  for (hipEvent_t e : p->ev) event_put(e, true);
  for (hipEvent_t e : p->poll_ev) event_put(e, false);
  for (auto& kv : p->step_graphs) (void)hipGraphExecDestroy(kv.second);
  if (p->cap_st) (void)hipStreamDestroy(p->cap_st);
  delete p;
}

// Wait for an event by polling it.  The waits of the Krylov loop last about one Arnoldi
// step; a blocking wait's wake-up can cost far more than that.
hipError_t poll_event(hipEvent_t ev) {
  hipError_t q;
  while ((q = hipEventQuery(ev)) == hipErrorNotReady) {
  }
  return q;
}

int mark(cavity_plan p, int phase, bool end) {
  HIPCHK(hipEventRecord(p->ev[2 * phase + (end ? 1 : 0)], p->st));
  if (end) p->ev_used[phase] = true;
  return CAVITY_OK;
}

void resolve_timers(cavity_plan p) {
  double* dst[6] = {&p->info.ms_spectrum, &p->info.ms_elimination, &p->info.ms_preconditioner,
                    &p->info.ms_rhs, &p->info.ms_krylov, &p->info.ms_synthesis};
  for (int i = 0; i < 6; ++i) {
    if (!p->ev_used[i]) continue;
    float ms = 0.f;
    if (hipEventSynchronize(p->ev[2 * i + 1]) == hipSuccess &&
        hipEventElapsedTime(&ms, p->ev[2 * i], p->ev[2 * i + 1]) == hipSuccess)
      *dst[i] = ms;
  }
}

// exp(-2 pi i t / n), t = 0 .. n-1, from extended-precision cos and sin.  Kept per length
// for the process: at n = 512 and 625 the extended-precision functions took about 0.8 ms
// per plan, most of a plan's set-up on a cached aperture.
const std::vector<zd>& twiddle_table(int n) {
  static std::mutex mu;
  static std::map<int, std::vector<zd>> tables;
  std::lock_guard<std::mutex> lk(mu);
  std::vector<zd>& out = tables[n];
  if ((int)out.size() != n) {
    out.resize(n);
    const long double two_pi = 6.283185307179586476925286766559L;
    for (int t = 0; t < n; ++t) {
      const long double ang = -two_pi * (long double)t / (long double)n;
      out[t] = cav::mk((double)cosl(ang), (double)sinl(ang));
    }
  }
  return out;
}

// Stage twiddle tables (double and single precision) of a plan's six transforms, kept on
// each device for the process and shared by the plans with the same transform lengths and
// radix choice: a plan then neither fills nor uploads them.  An entry is complete on the
// device before any other plan can find it.
struct StageTwiddles {
  const zd* tw = nullptr;
  const cav::zf* twf = nullptr;
};
int stage_twiddles(int device, const int* len, bool small_radices, const cav::FftPlan* plans,
                   int twn, hipStream_t st, StageTwiddles* out) {
  static std::mutex mu;
  static std::map<std::tuple<int, int, int, int, int, int, int, int>, StageTwiddles> cache;
  const auto key = std::make_tuple(device, len[0], len[1], len[2], len[3], len[4], len[5],
                                   small_radices ? 1 : 0);
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(key);
  if (it != cache.end()) {
    *out = it->second;
    return CAVITY_OK;
  }
  std::vector<zd> tw(twn);
  std::vector<cav::zf> twf(twn);
  int off = 0;
  for (int i = 0; i < 6; ++i) {
    cav::fill_stage_twiddles(plans[i], twiddle_table(len[i]).data(), tw.data() + off);
    off += std::max(1, plans[i].ntw);
  }
  for (int t = 0; t < twn; ++t) twf[t] = cav::cvt<float>(tw[t]);
  zd* dtw = nullptr;
  cav::zf* dtwf = nullptr;
  if (hipMalloc(&dtw, (size_t)twn * sizeof(zd)) != hipSuccess ||
      hipMalloc(&dtwf, (size_t)twn * sizeof(cav::zf)) != hipSuccess ||
      hipMemcpyAsync(dtw, tw.data(), (size_t)twn * sizeof(zd), hipMemcpyHostToDevice, st) !=
          hipSuccess ||
      hipMemcpyAsync(dtwf, twf.data(), (size_t)twn * sizeof(cav::zf), hipMemcpyHostToDevice,
                     st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    if (dtw) (void)hipFree(dtw);
    if (dtwf) (void)hipFree(dtwf);
    return fail(CAVITY_EDEVICE, "stage twiddle tables: device allocation or upload failed");
  }
  const StageTwiddles e{dtw, dtwf};
  cache.emplace(key, e);
  *out = e;
  return CAVITY_OK;
}

size_t plan_bytes(const cav::Geo& g, bool layered, int chunk, int nlayers) {
  Layout L;
  zd* z = nullptr;
  double* d = nullptr;
  int* i = nullptr;
  const size_t NM = g.NM;
  L.add(&z, (size_t)g.P1 * g.P2);
  L.add(&z, NM); L.add(&z, NM); L.add(&z, NM);
  L.add(&z, (size_t)(g.Nz + 1) * NM);
  L.add(&z, (size_t)(g.Nz + 1) * NM);
  if (layered) L.add(&z, (size_t)(g.Nz + 1) * NM);
  L.add(&z, 9 * NM); L.add(&z, 3 * NM);
  L.add(&d, NM); L.add(&d, 1);
  L.add(&i, g.Nz + 1); L.add(&z, nlayers); L.add(&z, nlayers); L.add(&d, nlayers);
  cav::zf* zf1 = nullptr;
  L.add(&zf1, (size_t)g.P1 * g.P2);
  L.add(&d, (size_t)2 * (g.M + 1) * g.P1); L.add(&d, (size_t)2 * g.P2 * (g.N + 1));
  L.add(&z, (size_t)2 * g.P1 * (g.N + 1));
  L.add(&z, (size_t)3 * chunk * (g.M + 1) * (g.ny + 1));
  L.add(&z, std::max<size_t>(3 * NM, (size_t)g.P1 * g.P2));
  L.add(&z, 3 * NM);
  L.add(&z, 8);
  return L.bytes;
}

size_t work_bytes(const cav::Geo& g, int restart, int nb, int nblk, bool spec) {
  const size_t n = 3ull * g.NM;
  const size_t z = sizeof(zd);
  return z * ((size_t)nb * 2 * 3 * (g.M + 1) * g.ldx + (size_t)nb * 3 * g.NM +
              (spec ? (size_t)nb * 3 * g.P1 * g.P2 + 2 * ((size_t)g.P1 * (g.M + 1) +
                                                         (size_t)g.P2 * (g.N + 1)) : 0) +
              (size_t)(restart + 1) * nb * n + 4ull * nb * n +
              (size_t)nblk * (restart + 1) * nb +
              (size_t)nb * (restart + 1) * 3 + (size_t)nb * restart * (restart + 4) + 64) +
         sizeof(double) * ((size_t)kNormBlocks * nb + 4 * nb) + sizeof(int) * 5 * nb + 64 * 256;
}

// Solve workspace for nb right-hand sides iterating together.
int ensure_work(cavity_plan p, int nb) {
  if (nb <= p->nbwork) return CAVITY_OK;
  const int R = p->opts.restart;
  const long long n = p->nvec();
  Layout L;
  L.add(&p->X, (size_t)nb * 3 * (p->g.M + 1) * p->g.ldx);
  L.add(&p->Y, (size_t)nb * 3 * (p->g.M + 1) * p->g.ldx);
  L.add(&p->S, (size_t)nb * 3 * p->g.NM);
  if (p->use_spec()) L.add(&p->U, (size_t)nb * 3 * p->g.P1 * p->g.P2);
  L.add(&p->V, (size_t)(R + 1) * nb * n);
  L.add(&p->w, (size_t)nb * n);
  L.add(&p->bvec, (size_t)nb * n);
  L.add(&p->zb, (size_t)nb * n);
  L.add(&p->rbuf, (size_t)nb * n);
  L.add(&p->dpart, (size_t)p->nblk_red * (R + 1) * nb);
  L.add(&p->dnpart, (size_t)kNormBlocks * nb);
  L.add(&p->h2, (size_t)nb * (R + 1));
  L.add(&p->kv.H, (size_t)nb * R * (R + 1));
  L.add(&p->kv.cs, (size_t)nb * R);
  L.add(&p->kv.sn, (size_t)nb * R);
  L.add(&p->kv.g, (size_t)nb * (R + 1));
  L.add(&p->kv.y, (size_t)nb * R);
  L.add(&p->kv.nrm2, (size_t)nb);
  L.add(&p->kv.bnorm, (size_t)nb);
  L.add(&p->kv.thr, (size_t)nb);
  L.add(&p->kv.relres, (size_t)nb);
  L.add(&p->kv.iters, (size_t)nb);
  L.add(&p->kv.active, (size_t)nb);
  L.add(&p->kv.incycle, (size_t)nb);
  L.add(&p->kv.jcount, (size_t)nb);
  L.add(&p->dwaves, (size_t)nb);
  if (p->st) HIPCHK(hipStreamSynchronize(p->st));
  else HIPCHK(hipDeviceSynchronize());
  for (auto& g : p->step_graphs) (void)hipGraphExecDestroy(g.second);
  p->step_graphs.clear();
  arena_release(p->work_arena.ptr, p->work_arena.bytes);
  p->work_arena = Arena();
  p->nbwork = 0;
  void* base = nullptr;
  int s = arena_acquire(L.bytes, &base);
  if (s) return s;
  p->work_arena = {base, L.bytes};
  L.bind(base);
  p->kv.restart = R;
  p->kv.tol = p->opts.tol;
  p->nbwork = nb;
  return CAVITY_OK;
}

int ensure_solutions(cavity_plan p, int count) {
  if (count <= p->nsol_cap) return CAVITY_OK;
  const size_t bytes = (size_t)count * p->nvec() * sizeof(zd);
  void* base = nullptr;
  int s = arena_acquire(bytes, &base);
  if (s) return s;
  if (p->xsol && p->nsol > 0)
    HIPCHK(hipMemcpyAsync(base, p->xsol, (size_t)p->nsol * p->nvec() * sizeof(zd),
                          hipMemcpyDeviceToDevice, p->st));
  if (p->st) HIPCHK(hipStreamSynchronize(p->st));
  else HIPCHK(hipDeviceSynchronize());
  arena_release(p->sol_arena.ptr, p->sol_arena.bytes);
  p->sol_arena = {base, bytes};
  p->xsol = static_cast<zd*>(base);
  p->nsol_cap = count;
  return CAVITY_OK;
}

// y = A v (or A P^{-1} v); low selects the single-precision convolutions.
int run_operator(cavity_plan p, int precond, int nb, const zd* v, zd* y, const int* active,
                 bool low = false, hipStream_t stream = nullptr) {
  const long long n = p->nvec();
  hipStream_t st = stream ? stream : p->st;
  if (p->use_spec()) {   // spectral operator: double precision in both precision modes
    HIPCHK(cav::launch_operator_spec(p->g, p->spec, p->khat, p->cols, precond, nb, v, n, p->X,
                                     p->Y, p->U, p->S, y, n, active, st));
    return CAVITY_OK;
  }
  if (low)
    HIPCHK(cav::launch_operator_f32(p->g, p->trig, p->khat_f, p->cols, precond, nb, v, n,
                                    reinterpret_cast<cav::zf*>(p->X),
                                    reinterpret_cast<cav::zf*>(p->Y), p->S, y, n, active, st));
  else
    HIPCHK(cav::launch_operator(p->g, p->trig, p->khat, p->cols, precond, nb, v, n, p->X, p->Y,
                                p->S, y, n, active, st));
  return CAVITY_OK;
}

// ---- autotuning of the TBC kernels' LDS batch ------------------------------------------
// The FFT kernels batch 2^lc transforms per block, sized from an LDS budget.  The best
// budget depends on the transform lengths and the precision (occupancy against strip width
// of the strided column accesses), so the first plan of each (P1, P2, s Nx, s Ny,
// precision) in a process times the operator apply of its Krylov iterations for a few
// budgets and keeps the fastest; later plans of the same shape reuse the choice.
// CAVITY_AUTOTUNE=0 turns this off (default budget), CAVITY_LDS_BUDGET fixes the budget.
struct TuneKey {
  int P1, P2, nq1, nq2, single, maxr;
  bool operator<(const TuneKey& o) const {
    return std::tie(P1, P2, nq1, nq2, single, maxr) <
           std::tie(o.P1, o.P2, o.nq1, o.nq2, o.single, o.maxr);
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, std::pair<int, int>> g_tune;   // (LDS budget, row passes in place)

int autotune_lds(cavity_plan p) {
  const char* e = std::getenv("CAVITY_AUTOTUNE");
  if ((e && std::atoi(e) == 0) || std::getenv("CAVITY_LDS_BUDGET") || p->use_spec())
    return CAVITY_OK;
  const bool single = p->opts.precision == CAVITY_MIXED;
  const TuneKey key{p->g.P1, p->g.P2, p->g.nq1, p->g.nq2, single ? 1 : 0, p->trig.maxr};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      p->g.lds_budget = it->second.first;
      p->g.rows_ip = it->second.second;
      p->info.lds_budget = p->g.lds_budget;
      p->info.tbc_rows_in_place = p->g.rows_ip;
      return CAVITY_OK;
    }
  }
  // timed with up to 8 right-hand sides in flight: with 2 the candidates were within the
  // timing noise of each other, and a choice that won there by a few per cent could lose by
  // a tenth at the 32 of a large batch (20 KB two-buffer rows against the default)
  const int nbt = std::min(8, p->opts.batch);
  int s = ensure_work(p, nbt);
  if (s) return s;
  const long long n = p->nvec();
  HIPCHK(hipMemsetAsync(p->zb, 0, (size_t)nbt * n * sizeof(zd), p->st));
  hipEvent_t t0 = nullptr, t1 = nullptr;
  HIPCHK(hipEventCreate(&t0));
  HIPCHK(hipEventCreate(&t1));
  // candidates: three LDS budgets x row passes in place or ping-pong; two sweeps, each
  // timing 4 applies after a warm-up; the fastest sweep of each candidate counts (guards
  // against a noisy first measurement)
  constexpr int kCand = 6;
  const int budgets[3] = {20000, 40000, 80000};
  float ms_best[kCand];
  for (float& v : ms_best) v = 1e30f;
  for (int sweep = 0; sweep < 2 && !s; ++sweep) {
    for (int ci = 0; ci < kCand && !s; ++ci) {
      p->g.lds_budget = budgets[ci % 3];
      p->g.rows_ip = ci / 3;
      if ((s = run_operator(p, 0, nbt, p->zb, p->w, nullptr, single))) break;   // warm-up
      if (hipEventRecord(t0, p->st) != hipSuccess) { s = CAVITY_EDEVICE; break; }
      for (int r = 0; r < 4 && !s; ++r) s = run_operator(p, 0, nbt, p->zb, p->w, nullptr, single);
      if (s) break;
      float ms = 0.f;
      if (hipEventRecord(t1, p->st) != hipSuccess || hipEventSynchronize(t1) != hipSuccess ||
          hipEventElapsedTime(&ms, t0, t1) != hipSuccess) {
        s = CAVITY_EDEVICE;
        break;
      }
      ms_best[ci] = std::min(ms_best[ci], ms);
    }
  }
  // the default (40000 bytes, in place) stays unless a candidate beats it by 3 %: candidates
  // closer than that are within the timing noise of these short runs, and the choice then
  // no longer flips between runs of the same workload
  constexpr int kDefault = 4;
  int best = kDefault;
  for (int ci = 0; ci < kCand; ++ci)
    if (ms_best[ci] < 0.97f * ms_best[kDefault] && ms_best[ci] < ms_best[best]) best = ci;
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if (s) return s;
  p->g.lds_budget = budgets[best % 3];
  p->g.rows_ip = best / 3;
  p->info.lds_budget = p->g.lds_budget;
  p->info.tbc_rows_in_place = p->g.rows_ip;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[key] = {p->g.lds_budget, p->g.rows_ip};
  return CAVITY_OK;
}

// Relative reduction a restart cycle of the mixed-precision solve aims for before the
// residual is recomputed with the double-precision operator (iterative refinement).
double mixed_inner_reduction() {
  static double v = -1.0;
  if (v < 0.0) {
    const char* e = std::getenv("CAVITY_MIXED_INNER");
    v = e ? std::atof(e) : 1e-5;
    if (!(v > 0.0 && v < 1.0)) v = 1e-5;
  }
  return v;
}

// Classical Gram-Schmidt passes of the mixed-precision inner cycles: one by default.  Their
// basis is stored in single precision (orthogonal to about 1e-7 whatever the passes), a
// cycle only has to reduce its residual by the inner factor, and every restart recomputes
// the residual with the double-precision operator, so the final accuracy does not rest on
// the inner basis; a second pass left the iteration counts unchanged (23 at 256^2 and on
// the layered batch, 27 at 512^2) for a third more basis traffic.  CAVITY_CGS_PASSES=2
// restores it.  Double-precision solves always take two passes.
int mixed_cgs_passes() {
  static const int v = [] {
    const char* e = std::getenv("CAVITY_CGS_PASSES");
    return e && std::atoi(e) == 2 ? 2 : 1;
  }();
  return v;
}

// Whether the preconditioned basis vector z = P^{-1} v (p->zb) is stored in single
// precision: in the mixed-precision inner cycles of the FFT operator, whose convolutions
// take their input in single precision anyway (the spectral operator's stay double).
bool z_single(cavity_plan p) { return p->opts.precision == CAVITY_MIXED && !p->use_spec(); }

// v_{j+1} = w / |w| into vn and z = P^{-1} v_{j+1} into p->zb (see launch_next_vector);
// w in single precision (WT = float) only in the mixed-precision inner steps.
template <typename VT, typename WT>
int next_vector(cavity_plan p, cav::Krylov& kv, int j, const double* npart, int nparts,
                const cav::cx<WT>* w, cav::cx<VT>* vn, int nb, hipStream_t st) {
  const long long n = p->nvec();
  if constexpr (sizeof(VT) == sizeof(float)) {
    if (z_single(p)) {
      HIPCHK(cav::launch_next_vector(p->g, kv, j, npart, nparts, w, vn, n, p->cols,
                                     reinterpret_cast<cav::zf*>(p->zb), nb, st));
      return CAVITY_OK;
    }
  }
  if constexpr (sizeof(WT) == sizeof(double)) {
    HIPCHK(cav::launch_next_vector(p->g, kv, j, npart, nparts, w, vn, n, p->cols, p->zb, nb, st));
    return CAVITY_OK;
  } else {
    return fail(CAVITY_ENOTIMPL, "single-precision w outside the mixed inner steps");
  }
}

// One Arnoldi step j for the lockstep group (kernels only, on stream st): w = A z_j,
// classical Gram-Schmidt twice (the second pass's coefficients added into H; once in the
// mixed-precision inner cycles, see mixed_cgs_passes), the Givens step of column j,
// v_{j+1} = w / |w| and z = P^{-1} v_{j+1} (in single precision in the mixed-precision
// inner cycles, see z_single).
template <typename VT>
int arnoldi_step(cavity_plan p, int nb, int j, cav::cx<VT>* V, hipStream_t st) {
  const long long n = p->nvec();
  const int R = p->opts.restart;
  const long long ldj = (long long)p->nbwork * n;
  const int nblk_u = (int)std::min<long long>(kNormBlocks, (n + 255) / 256);
  cav::Krylov& kv = p->kv;
  const bool mixed = p->opts.precision == CAVITY_MIXED;
  cav::cx<VT>* vn = V + (long long)(j + 1) * ldj;
  int s;
  const int nv = j + 1;
  zd* hcol = kv.H + (long long)j * (R + 1);
  const long long hstr = (long long)R * (R + 1);
  const bool fused = !p->use_spec() && nv <= kFusedGsMax;
  // the fused single-pass steps of the mixed-precision inner cycles keep w in single
  // precision too (updated in double, see k_update_norm)
  const bool w_single = sizeof(VT) == sizeof(float) && fused && z_single(p) &&
                        mixed_cgs_passes() == 1;
  cav::zf* wf = reinterpret_cast<cav::zf*>(p->w);
  if (fused) {
    // w = A z_j with the first dot products V^H w computed from the epilogue's registers
    if constexpr (sizeof(VT) == sizeof(float)) {
      cav::zf* Xf = reinterpret_cast<cav::zf*>(p->X);
      cav::zf* Yf = reinterpret_cast<cav::zf*>(p->Y);
      const cav::zf* zf = reinterpret_cast<const cav::zf*>(p->zb);
      if (w_single)
        HIPCHK(cav::launch_operator_dots_f32(p->g, p->trig, p->khat_f, p->cols, 0, nb, zf, n, Xf,
                                             Yf, p->S, wf, n, V, ldj, nv, R + 1, p->dpart,
                                             p->nblk_red, hcol, hstr, kv.active, st));
      else if (z_single(p))
        HIPCHK(cav::launch_operator_dots_f32(p->g, p->trig, p->khat_f, p->cols, 0, nb, zf, n, Xf,
                                             Yf, p->S, p->w, n, V, ldj, nv, R + 1, p->dpart,
                                             p->nblk_red, hcol, hstr, kv.active, st));
      else
        HIPCHK(cav::launch_operator_dots_f32(p->g, p->trig, p->khat_f, p->cols, 0, nb, p->zb, n,
                                             Xf, Yf, p->S, p->w, n, V, ldj, nv, R + 1, p->dpart,
                                             p->nblk_red, hcol, hstr, kv.active, st));
    } else {
      HIPCHK(cav::launch_operator_dots(p->g, p->trig, p->khat, p->cols, 0, nb, p->zb, n, p->X,
                                       p->Y, p->S, p->w, n, V, ldj, nv, R + 1, p->dpart,
                                       p->nblk_red, hcol, hstr, kv.active, st));
    }
  } else {
    if (z_single(p)) {
      HIPCHK(cav::launch_operator_f32(p->g, p->trig, p->khat_f, p->cols, 0, nb,
                                      reinterpret_cast<const cav::zf*>(p->zb), n,
                                      reinterpret_cast<cav::zf*>(p->X),
                                      reinterpret_cast<cav::zf*>(p->Y), p->S, p->w, n, kv.active,
                                      st));
    } else if ((s = run_operator(p, 0, nb, p->zb, p->w, kv.active, mixed, st))) {
      return s;
    }
    HIPCHK(cav::launch_dots(V, ldj, nv, R + 1, p->w, n, nb, p->dpart, p->nblk_red, hcol, hstr,
                            nullptr, 0, kv.active, st));
  }
  if (w_single) {   // one pass: update with hcol, then the norm
    if constexpr (sizeof(VT) == sizeof(float)) {
      HIPCHK(cav::launch_update_norm(V, ldj, nv, hcol, hstr, wf, n, nb, p->dnpart, nblk_u,
                                     kv.active, st));
      return next_vector(p, kv, j, p->dnpart, nblk_u, wf, vn, nb, st);
    }
  }
  if (mixed && mixed_cgs_passes() == 1) {   // one pass: update with hcol, then the norm
    HIPCHK(cav::launch_update_norm(V, ldj, nv, hcol, hstr, p->w, n, nb, p->dnpart, nblk_u,
                                   kv.active, st));
    if ((s = next_vector(p, kv, j, p->dnpart, nblk_u, p->w, vn, nb, st))) return s;
    return CAVITY_OK;
  }
  if (nv <= kFusedGsMax) {   // one pass: update with hcol, dot products of the updated w
    HIPCHK(cav::launch_update_dots(V, ldj, nv, R + 1, hcol, hstr, p->w, n, nb, p->dpart,
                                   p->nblk_red, p->h2, R + 1, hcol, hstr, kv.active, st));
  } else {
    HIPCHK(cav::launch_update(V, ldj, nv, hcol, hstr, p->w, n, nb, kv.active, st));
    HIPCHK(cav::launch_dots(V, ldj, nv, R + 1, p->w, n, nb, p->dpart, p->nblk_red, p->h2, R + 1,
                            hcol, hstr, kv.active, st));
  }
  HIPCHK(cav::launch_update_norm(V, ldj, nv, p->h2, R + 1, p->w, n, nb, p->dnpart, nblk_u,
                                 kv.active, st));
  return next_vector(p, kv, j, p->dnpart, nblk_u, p->w, vn, nb, st);
}

// Whether the Arnoldi steps run as captured graphs (one capture per step index and group
// size, replayed by later cycles, groups and solve calls): only with CAVITY_GRAPHS=1, and
// never while the kernel probe is watching (its events belong to individual launches).
// Off by default: the host queues launches far enough ahead that the GPU does not wait
// for them, and a graph launch measured 2-4 % slower than the step's direct launches.
bool use_step_graphs() {
  if (cav::g_probe_active()) return false;
  const char* e = std::getenv("CAVITY_GRAPHS");
  return e && std::atoi(e) == 1;
}

// The executable graph of step j for group size nb, captured on first use.
template <typename VT>
int step_graph(cavity_plan p, int nb, int j, cav::cx<VT>* V, hipGraphExec_t* out) {
  const long long key = ((long long)nb << 20) | j;
  auto it = p->step_graphs.find(key);
  if (it != p->step_graphs.end()) {
    *out = it->second;
    return CAVITY_OK;
  }
  if (!p->cap_st) HIPCHK(hipStreamCreateWithFlags(&p->cap_st, hipStreamNonBlocking));
  HIPCHK(hipStreamBeginCapture(p->cap_st, hipStreamCaptureModeThreadLocal));
  const int s = arnoldi_step<VT>(p, nb, j, V, p->cap_st);
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(p->cap_st, &graph);
  if (s) {
    if (graph) (void)hipGraphDestroy(graph);
    return s;
  }
  if (ec != hipSuccess) return fail(CAVITY_EDEVICE, std::string("graph capture: ") + hipGetErrorString(ec));
  hipGraphExec_t exec = nullptr;
  const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ei != hipSuccess)
    return fail(CAVITY_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(ei));
  p->step_graphs[key] = exec;
  *out = exec;
  return CAVITY_OK;
}

// Right-preconditioned restarted GMRES with classical Gram-Schmidt applied twice (once in
// the mixed-precision inner cycles), for nb
// right-hand sides b (p->bvec) iterating in lockstep; solutions in x (nb x n).  The
// Arnoldi step, the Givens rotations and the convergence test run on the device; the
// host looks at the convergence flags every few iterations and once per restart cycle.
// Mixed precision: the Arnoldi steps apply the operator with single-precision
// convolutions and a cycle ends once it has reduced its residual by the inner factor;
// every restart recomputes the residual b - A x with the double-precision operator, so
// the cycles are steps of iterative refinement and the final test is on that residual.
template <typename VT>
int gmres_batch_t(cavity_plan p, int nb, zd* x, std::vector<double>* relres_out,
                  std::vector<int>* iters_out, cav::cx<VT>* V) {
  const long long n = p->nvec();
  const int R = p->opts.restart;
  const bool mixed = p->opts.precision == CAVITY_MIXED;
  const double inner = mixed ? mixed_inner_reduction() : 0.0;
  const long long ldj = (long long)p->nbwork * n;
  cav::Krylov& kv = p->kv;
  // How many Arnoldi steps the host may run ahead of the last convergence flags it has seen.
  constexpr int kLag = 1;
  // one event per step, and one more for the waits at each cycle start and at the end
  if ((int)p->poll_ev.size() < R + 1) {
    const size_t old = p->poll_ev.size();
    p->poll_ev.resize(R + 1, nullptr);
    for (size_t i = old; i < p->poll_ev.size(); ++i)
      HIPCHK(event_get(&p->poll_ev[i], false));
  }
  int* hstat = p->hflags;   // pinned: [0, nb) active, [nb, 2 nb) iterations, then per step
  {
    int* dev = nullptr;
    double* devr = nullptr;
    HIPCHK(hipHostGetDevicePointer((void**)&dev, hstat, 0));
    HIPCHK(hipHostGetDevicePointer((void**)&devr, p->hratio, 0));
    kv.hflags = dev + 2 * nb;
    kv.hratio = devr;
    kv.nbh = nb;
  }
  HIPCHK(hipMemsetAsync(x, 0, (size_t)nb * n * sizeof(zd), p->st));
  HIPCHK(cav::launch_norm2(p->bvec, n, nb, p->dnpart, p->nblk_red, kv.nrm2, nullptr, p->st));
  HIPCHK(cav::launch_krylov_init(kv, nb, p->st));
  int s;
  bool first = true;
  while (true) {
    zd* r0 = p->rbuf;   // residual of rhs r at rbuf + r n
    if (first) {
      HIPCHK(hipMemcpyAsync(r0, p->bvec, (size_t)nb * n * sizeof(zd), hipMemcpyDeviceToDevice,
                            p->st));
    } else {
      // residual with the double-precision operator (the refinement step when mixed)
      if ((s = run_operator(p, 0, nb, x, p->w, nullptr))) return s;
      HIPCHK(cav::launch_sub(p->bvec, p->w, r0, (long long)nb * n, p->st));
    }
    first = false;
    HIPCHK(cav::launch_norm2(r0, n, nb, p->dnpart, p->nblk_red, kv.nrm2, nullptr, p->st));
    HIPCHK(cav::launch_cycle_start(kv, nb, p->opts.max_iter, inner, p->st));
    HIPCHK(hipMemcpyAsync(hstat, kv.active, nb * sizeof(int), hipMemcpyDeviceToHost, p->st));
    HIPCHK(hipMemcpyAsync(hstat + nb, kv.iters, nb * sizeof(int), hipMemcpyDeviceToHost, p->st));
    HIPCHK(hipEventRecord(p->poll_ev[R], p->st));
    HIPCHK(poll_event(p->poll_ev[R]));
    bool any = false;
    int budget = R;
    for (int r = 0; r < nb; ++r)
      if (hstat[r]) {
        any = true;
        budget = std::min(budget, std::max(1, p->opts.max_iter - hstat[nb + r]));
      }
    if (std::getenv("CAVITY_TRACE")) {
      std::vector<double> rr(nb);
      HIPCHK(hipMemcpy(rr.data(), kv.relres, nb * sizeof(double), hipMemcpyDeviceToHost));
      std::fprintf(stderr, "[gmres] nb=%d cycle start:", nb);
      for (int r = 0; r < nb; ++r)
        std::fprintf(stderr, " r%d it=%d res=%.3e", r, hstat[nb + r], rr[r]);
      std::fprintf(stderr, "\n");
    }
    if (!any) break;
    // per-step flag slots start at -1 ("not written yet"); the device writes 0 or 1
    for (size_t i = (size_t)2 * nb; i < (size_t)(2 + R) * nb; ++i) hstat[i] = -1;
    // v_0 = r / |r| and z = P^{-1} v_0 (norms already in kv.nrm2)
    if ((s = next_vector(p, kv, -1, nullptr, 0, r0, V, nb, p->st))) return s;
    int seen = 0;   // first step whose flags the host has not looked at
    const bool graphs = use_step_graphs();
    for (int j = 0; j < budget; ++j) {
      if (graphs) {
        hipGraphExec_t g = nullptr;
        if ((s = step_graph<VT>(p, nb, j, V, &g))) return s;
        HIPCHK(hipGraphLaunch(g, p->st));
      } else if ((s = arnoldi_step<VT>(p, nb, j, V, p->st))) {
        return s;
      }
      // the Givens step published this step's flags in host memory; the event marks them ready
      HIPCHK(hipEventRecord(p->poll_ev[j], p->st));
      bool stop = false;
      while (seen <= j && !stop) {
        // wait for a step when the host is kLag steps ahead of it, or when it is the step
        // just queued and the last two residual ratios predict that every rhs still
        // iterating converges in it (so no step is queued after convergence)
        bool wait = j - seen >= kLag;
        if (!wait && seen == j && j >= 2) {
          bool all = true;
          for (int r = 0; r < nb && all; ++r) {
            const volatile int* f1 = hstat + (size_t)(2 + j - 1) * nb;
            if (f1[r] != 1) continue;
            const volatile double* q1 = p->hratio + (size_t)(j - 1) * nb;
            const volatile double* q2 = p->hratio + (size_t)(j - 2) * nb;
            const double a1 = q1[r], a2 = q2[r];
            const double pred = a1 * (a1 / std::max(a2, 1e-300));
            all = pred <= 1.0;
          }
          wait = all;
        }
        if (wait) {
          HIPCHK(poll_event(p->poll_ev[seen]));
        } else {
          const hipError_t q = hipEventQuery(p->poll_ev[seen]);
          if (q == hipErrorNotReady) break;
          HIPCHK(q);
        }
        const volatile int* fl = hstat + (size_t)(2 + seen) * nb;
        bool still = false, written = true;
        for (int r = 0; r < nb; ++r) {
          still = still || fl[r] == 1;
          written = written && fl[r] >= 0;
        }
        if (!written) break;   // host view not updated yet: look again after the next step
        stop = !still;
        ++seen;
      }
      if (stop) break;
    }
    HIPCHK(cav::launch_solve_y(kv, nb, p->st));
    HIPCHK(cav::launch_combine(p->g, kv, V, ldj, p->cols, x, nb, p->st));
    HIPCHK(cav::launch_cycle_end(kv, nb, p->st));
  }
  std::vector<double> relres(nb);
  std::vector<int> iters(nb);
  HIPCHK(hipMemcpyAsync(p->hn, kv.relres, nb * sizeof(double), hipMemcpyDeviceToHost, p->st));
  HIPCHK(hipMemcpyAsync(hstat, kv.iters, nb * sizeof(int), hipMemcpyDeviceToHost, p->st));
  HIPCHK(hipEventRecord(p->poll_ev[R], p->st));
  HIPCHK(poll_event(p->poll_ev[R]));
  for (int r = 0; r < nb; ++r) {
    relres[r] = p->hn[r];
    iters[r] = hstat[r];
  }
  if (relres_out) *relres_out = relres;
  if (iters_out) *iters_out = iters;
  for (int r = 0; r < nb; ++r)
    if (relres[r] > p->opts.tol) return fail(CAVITY_ENOCONV, "GMRES did not reach the tolerance");
  return CAVITY_OK;
}

// The Krylov basis is stored in double precision, or in single precision for the
// mixed-precision solve (its cycles only need to reduce the residual by the inner factor;
// the refinement residuals stay double).
int gmres_batch(cavity_plan p, int nb, zd* x, std::vector<double>* relres_out,
                std::vector<int>* iters_out) {
  if (p->opts.precision == CAVITY_MIXED)
    return gmres_batch_t<float>(p, nb, x, relres_out, iters_out,
                                reinterpret_cast<cav::zf*>(p->V));
  return gmres_batch_t<double>(p, nb, x, relres_out, iters_out, p->V);
}

// RCS of n (stored solution, observation direction) pairs: one launch for all of them
// (queries and per-block partial sums in a plan-owned device buffer), one copy back, and
// the block sums reduced on the host in a fixed order.
//   L = (-E^2, E^1, 0);  sigma_theta = k^2/pi |phi^ . L|^2,  sigma_phi = k^2/pi |theta^ . L|^2
int rcs_queries(cavity_plan p, int n, const int* rhs, const double* th, const double* ph,
                double* sigma) {
  if (n == 0) return CAVITY_OK;
  const int nblk = rcs_blocks(p->g.NM);
  const size_t qbytes = ((size_t)n * sizeof(cav::RcsQuery) + 255) / 256 * 256;
  const size_t need = qbytes + (size_t)n * 2 * nblk * sizeof(zd);
  if (need > p->rcs_arena.bytes) {
    if (p->st) HIPCHK(hipStreamSynchronize(p->st));
    arena_release(p->rcs_arena.ptr, p->rcs_arena.bytes);
    p->rcs_arena = Arena();
    void* base = nullptr;
    const int s = arena_acquire(need, &base);
    if (s) return s;
    p->rcs_arena = {base, need};
  }
  auto* dq = static_cast<cav::RcsQuery*>(p->rcs_arena.ptr);
  zd* dpart = reinterpret_cast<zd*>(static_cast<char*>(p->rcs_arena.ptr) + qbytes);
  const double k = p->g.k;
  std::vector<cav::RcsQuery> q(n);
  for (int i = 0; i < n; ++i)
    q[i] = {rhs[i], k * std::sin(th[i]) * std::cos(ph[i]), k * std::sin(th[i]) * std::sin(ph[i])};
  std::vector<zd> part((size_t)n * 2 * nblk);
  HIPCHK(hipMemcpyAsync(dq, q.data(), n * sizeof(cav::RcsQuery), hipMemcpyHostToDevice, p->st));
  HIPCHK(cav::launch_rcs_partial(p->g, p->xsol, p->nvec(), dq, n, dpart, nblk, p->st));
  HIPCHK(hipMemcpyAsync(part.data(), dpart, part.size() * sizeof(zd), hipMemcpyDeviceToHost,
                        p->st));
  HIPCHK(hipStreamSynchronize(p->st));
  for (int i = 0; i < n; ++i) {
    std::complex<double> e1 = 0.0, e2 = 0.0;
    for (int b = 0; b < nblk; ++b) {
      const zd* pb = &part[2 * ((size_t)i * nblk + b)];
      e1 += std::complex<double>(pb[0].re, pb[0].im);
      e2 += std::complex<double>(pb[1].re, pb[1].im);
    }
    const double ct = std::cos(th[i]), sp = std::sin(ph[i]), cp = std::cos(ph[i]);
    const std::complex<double> L1 = -e2, L2 = e1;
    const std::complex<double> phiL = -sp * L1 + cp * L2;
    const std::complex<double> thL = ct * cp * L1 + ct * sp * L2;
    sigma[2 * i] = k * k / M_PI * std::norm(phiL);
    sigma[2 * i + 1] = k * k / M_PI * std::norm(thL);
  }
  return CAVITY_OK;
}

// Spectral TBC operator, plan part: the closed-form transforms of the trial functions on
// the kernel-spectrum lattice xi = 2 pi j / L (j centred at zero), host double precision,
//   F1[j1][m] = int_0^a cos or sin(mu_m x) e^{-i xi_j1 x} dx, F2 likewise along y,
// from E(w) = int_0^len e^{i w x} dx = len e^{i w len / 2} sin(w len / 2) / (w len / 2):
// cos -> (E(w+) + E(w-)) / 2, sin -> (E(w+) - E(w-)) / (2 i), w+- = -xi +- mu.
std::complex<double> exp_int(double w, double len) {
  const double t = 0.5 * w * len;
  const double sc = std::abs(t) < 1e-8 ? 1.0 - t * t / 6.0 : std::sin(t) / t;
  return len * sc * std::complex<double>(std::cos(t), std::sin(t));
}

void trial_transforms(int P, double L, int modes, double side, std::vector<zd>* fc,
                      std::vector<zd>* fs) {
  fc->resize((size_t)P * modes);
  fs->resize((size_t)P * modes);
  for (int j = 0; j < P; ++j) {
    const int js = j <= P / 2 ? j : j - P;
    const double alpha = -2.0 * M_PI * js / L;
    for (int m = 0; m < modes; ++m) {
      const double mu = M_PI * m / side;
      const std::complex<double> ep = exp_int(alpha + mu, side), em = exp_int(alpha - mu, side);
      const std::complex<double> c = 0.5 * (ep + em);
      const std::complex<double> sn = (ep - em) / std::complex<double>(0.0, 2.0);
      (*fc)[(size_t)j * modes + m] = cav::mk(c.real(), c.imag());
      (*fs)[(size_t)j * modes + m] = cav::mk(sn.real(), sn.imag());
    }
  }
}

int build_spec(cavity_plan p) {
  const cav::Geo& g = p->g;
  const int M1 = g.M + 1, N1 = g.N + 1;
  std::vector<zd> f1c, f1s, f2c, f2s;
  trial_transforms(g.P1, g.P1 * g.hq1, M1, g.a, &f1c, &f1s);
  trial_transforms(g.P2, g.P2 * g.hq2, N1, g.b, &f2c, &f2s);
  const size_t n1 = (size_t)g.P1 * M1, n2 = (size_t)g.P2 * N1;
  const size_t bytes = 2 * (n1 + n2) * sizeof(zd);
  void* base = nullptr;
  int s = arena_acquire(bytes, &base);
  if (s) return s;
  p->spec_arena = {base, bytes};
  zd* d = static_cast<zd*>(base);
  p->spec = {d, d + n1, d + 2 * n1, d + 2 * n1 + n2};
  HIPCHK(hipMemcpy(d, f1c.data(), n1 * sizeof(zd), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(d + n1, f1s.data(), n1 * sizeof(zd), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(d + 2 * n1, f2c.data(), n2 * sizeof(zd), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(d + 2 * n1 + n2, f2s.data(), n2 * sizeof(zd), hipMemcpyHostToDevice));
  // |F|^2 in the layouts of the preconditioner's diagonal contraction (pw1 [kind][m][j1],
  // pw2 [kind][j2][n], kind 0 cos, 1 sin): the exact diagonal of D_spec's S^f
  std::vector<double> w1(2 * n1), w2(2 * n2);
  for (int j = 0; j < g.P1; ++j)
    for (int m = 0; m < M1; ++m) {
      w1[(size_t)m * g.P1 + j] = cav::cabs2(f1c[(size_t)j * M1 + m]);
      w1[n1 + (size_t)m * g.P1 + j] = cav::cabs2(f1s[(size_t)j * M1 + m]);
    }
  for (int j = 0; j < g.P2; ++j)
    for (int n = 0; n < N1; ++n) {
      w2[(size_t)j * N1 + n] = cav::cabs2(f2c[(size_t)j * N1 + n]);
      w2[n2 + (size_t)j * N1 + n] = cav::cabs2(f2s[(size_t)j * N1 + n]);
    }
  HIPCHK(hipMemcpy(p->pw1, w1.data(), w1.size() * sizeof(double), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(p->pw2, w2.data(), w2.size() * sizeof(double), hipMemcpyHostToDevice));
  p->info.device_bytes += bytes;
  return CAVITY_OK;
}

// Direct solve, plan part (the paper's Steps 1 and 3, Section 6): the aperture matrix A is
// assembled column by column by applying the operator to unit vectors (the same TBC
// convolutions and local blocks GMRES applies, in double precision), the entries of absent
// modes get a unit diagonal, and Gauss-Jordan elimination with partial pivoting leaves
// (P A)^{-1} and the row permutation in the plan.
int dense_factor(cavity_plan p) {
  if (p->dense_F) return CAVITY_OK;
  const long long n = p->nvec();
  const size_t mat = (size_t)n * n * sizeof(zd);
  const size_t keep = mat + 2 * (size_t)n * sizeof(int) + 256;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  void* a = nullptr;
  void* b = nullptr;
  int s = arena_acquire(keep, &a);
  if (!s) s = arena_acquire(mat, &b);
  auto done = [&](int code) {
    if (b) arena_release(b, mat);
    if (code && a) arena_release(a, keep);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return code;
  };
  if (s) return done(s);
  zd* A = static_cast<zd*>(a);
  int* piv = reinterpret_cast<int*>(static_cast<char*>(a) + mat);
  int* perm = piv + n;
  if (hipEventRecord(e0, p->st) != hipSuccess) return done(fail(CAVITY_EDEVICE, "event"));
  for (long long k0 = 0; k0 < n; k0 += p->nbwork) {
    const int nb = (int)std::min<long long>(p->nbwork, n - k0);
    if (cav::launch_unit_vectors(n, k0, nb, p->rbuf, p->st) != hipSuccess)
      return done(fail(CAVITY_EDEVICE, "unit vectors"));
    if ((s = run_operator(p, 0, nb, p->rbuf, A + k0 * n, nullptr))) return done(s);
  }
  zd* F = nullptr;
  if (cav::launch_dense_fix(p->g, A, p->st) != hipSuccess ||
      cav::launch_gj_invert(A, static_cast<zd*>(b), n, piv, &F, p->st) != hipSuccess)
    return done(fail(CAVITY_EDEVICE, std::string("Gauss-Jordan: ") +
                                         hipGetErrorString(hipGetLastError())));
  if (F != A &&
      hipMemcpyAsync(A, F, mat, hipMemcpyDeviceToDevice, p->st) != hipSuccess)
    return done(fail(CAVITY_EDEVICE, "copy of the inverse"));
  std::vector<int> hp(n), hperm(n);
  if (hipMemcpyAsync(hp.data(), piv, n * sizeof(int), hipMemcpyDeviceToHost, p->st) !=
          hipSuccess ||
      hipEventRecord(e1, p->st) != hipSuccess || hipStreamSynchronize(p->st) != hipSuccess)
    return done(fail(CAVITY_EDEVICE, "pivot readback"));
  for (long long k = 0; k < n; ++k) hperm[k] = (int)k;
  for (long long k = 0; k < n; ++k) {
    if (hp[k] < k || hp[k] >= n)
      return done(fail(CAVITY_ERESONANT, "aperture matrix is singular (no pivot at column " +
                                             std::to_string(k) + ")"));
    std::swap(hperm[k], hperm[hp[k]]);
  }
  if (hipMemcpy(perm, hperm.data(), n * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
    return done(fail(CAVITY_EDEVICE, "permutation upload"));
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, e0, e1) == hipSuccess) p->info.ms_factor = ms;
  p->dense_arena = {a, keep};
  p->dense_F = A;
  p->dense_perm = perm;
  p->info.device_bytes += keep;
  return done(CAVITY_OK);
}

// Direct solve, per right-hand side: x = A^{-1} b for the nb right-hand sides in p->bvec,
// then the true residual b - A x with the operator; up to two refinement steps
// x += A^{-1} r while a residual is above the tolerance.
int dense_solve(cavity_plan p, int nb, zd* x, std::vector<double>* relres_out,
                std::vector<int>* iters_out) {
  const long long n = p->nvec();
  cav::Krylov& kv = p->kv;
  HIPCHK(cav::launch_dense_apply(p->dense_F, p->dense_perm, n, p->bvec, nb, p->zb, x, p->st));
  HIPCHK(cav::launch_norm2(p->bvec, n, nb, p->dnpart, p->nblk_red, kv.bnorm, nullptr, p->st));
  std::vector<double> b2(nb), r2(nb);
  HIPCHK(hipMemcpyAsync(b2.data(), kv.bnorm, nb * sizeof(double), hipMemcpyDeviceToHost, p->st));
  std::vector<double> rel(nb, 0.0);
  for (int pass = 0; pass < 3; ++pass) {
    int s;
    if ((s = run_operator(p, 0, nb, x, p->w, nullptr))) return s;
    HIPCHK(cav::launch_sub(p->bvec, p->w, p->rbuf, (long long)nb * n, p->st));
    HIPCHK(cav::launch_norm2(p->rbuf, n, nb, p->dnpart, p->nblk_red, kv.nrm2, nullptr, p->st));
    HIPCHK(hipMemcpyAsync(r2.data(), kv.nrm2, nb * sizeof(double), hipMemcpyDeviceToHost, p->st));
    HIPCHK(hipStreamSynchronize(p->st));
    bool ok = true;
    for (int r = 0; r < nb; ++r) {
      rel[r] = b2[r] > 0.0 ? std::sqrt(r2[r] / b2[r]) : 0.0;
      ok = ok && rel[r] <= p->opts.tol;
    }
    if (ok || pass == 2) break;
    HIPCHK(cav::launch_dense_apply(p->dense_F, p->dense_perm, n, p->rbuf, nb, p->zb, p->w,
                                   p->st));
    HIPCHK(cav::launch_add(x, p->w, (long long)nb * n, p->st));
  }
  *relres_out = rel;
  iters_out->assign(nb, 0);
  for (double v : rel)
    if (!(v <= p->opts.tol)) return CAVITY_ENOCONV;
  return CAVITY_OK;
}

void wave_setup(double k, double h, double theta, double phi, int pol, cav::Wave* wv) {
  const double st = std::sin(theta), ct = std::cos(theta), sp = std::sin(phi), cp = std::cos(phi);
  wv->h = h;
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

bool angles_ok(double theta, double phi, int pol) {
  return theta >= 0.0 && theta <= 0.5 * M_PI + 1e-12 && std::isfinite(phi) &&
         (pol == CAVITY_TM || pol == CAVITY_TE);
}

// Solve right-hand sides [i0, i0 + nb) of a batch into solution slots i0.., writing fields
// and packed aperture vectors when asked.
int solve_chunk(cavity_plan p, int i0, int nb, const double* theta, const double* phi,
                const int* pol, cavity_c128* E_out, cavity_c128* ap_out) {
  std::vector<cav::Wave> wv(nb);
  for (int r = 0; r < nb; ++r)
    wave_setup(p->g.k, p->cols.hs ? p->group_h[i0 + r] : p->g.h, theta[r], phi[r], pol[r],
               &wv[r]);
  HIPCHK(hipMemcpyAsync(p->dwaves, wv.data(), nb * sizeof(cav::Wave), hipMemcpyHostToDevice,
                        p->st));
  int s0;
  if ((s0 = mark(p, 3, false))) return s0;
  HIPCHK(cav::launch_rhs(p->g, p->dwaves, nb, p->bvec, p->st));
  if ((s0 = mark(p, 3, true))) return s0;
  zd* x = p->xsol + (long long)i0 * p->nvec();
  std::vector<double> relres;
  std::vector<int> iters;
  if ((s0 = mark(p, 4, false))) return s0;
  int status = p->dense_now ? dense_solve(p, nb, x, &relres, &iters)
                            : gmres_batch(p, nb, x, &relres, &iters);
  if (status != CAVITY_OK && status != CAVITY_ENOCONV) return status;
  if ((s0 = mark(p, 4, true))) return s0;
  p->info.last_iterations = *std::max_element(iters.begin(), iters.end());
  p->info.last_rel_residual = *std::max_element(relres.begin(), relres.end());
  const long long field = 3LL * (p->g.Nz + 1) * (p->g.ny + 1) * (p->g.nx + 1);
  if (E_out) {
    if ((s0 = mark(p, 5, false))) return s0;
    // the staging slab holds synth_chunk levels of one field: each launch pair takes up to
    // that many (field, level) pairs, all fields of the group together when they fit
    const int rg = std::min(nb, p->synth_chunk);
    const int jn = std::max(1, p->synth_chunk / rg);
    for (int r0 = 0; r0 < nb; r0 += rg) {
      const int nr = std::min(rg, nb - r0);
      for (int j0 = 0; j0 <= p->g.Nz; j0 += jn) {
        const int j1 = std::min(p->g.Nz + 1, j0 + jn);
        HIPCHK(cav::launch_synthesis(p->g, p->trig, p->pi_d, p->layered ? p->theta_d : nullptr,
                                     p->pi_n, x + (long long)r0 * p->nvec(), p->nvec(), nr, j0,
                                     j1, p->tbuf, reinterpret_cast<zd*>(E_out) + r0 * field,
                                     field, p->st));
      }
    }
    if ((s0 = mark(p, 5, true))) return s0;
  }
  if (ap_out)
    for (int r = 0; r < nb; ++r)
      HIPCHK(cav::launch_pack(p->g, x + (long long)r * p->nvec(),
                              reinterpret_cast<zd*>(ap_out) + r * p->info.n_ap, p->st));
  return status;
}

}  // namespace

namespace {

// ---- aperture cache ----------------------------------------------------------------
// The kernel spectrum (Section 5) and the exact diagonal of the three single-layer
// operators depend only on the aperture: a, b, k, Nx, Ny and the quadrature oversampling.
// Plans with an equal aperture (a served stream sees a handful of apertures for thousands
// of cavities) copy them from this process-wide cache instead of recomputing them.  Entries
// live in their own device blocks, filled asynchronously on the stream of the plan that
// computed them; a ready event orders every later copy after the fill.  Least recently
// used entries go when the cache exceeds its byte limit (CAVITY_APERTURE_CACHE_BYTES,
// default 1 GiB; 0 disables it); the device is synchronised before such a free because
// copies from the entry may still be queued on other streams.
struct ApertureEntry {
  double a, b, k;
  int nx, ny, s, method, dev;
  void* mem;
  size_t bytes;
  hipEvent_t ready;
  unsigned long long last_use;
};
std::mutex g_ap_mu;
std::vector<ApertureEntry> g_ap;
size_t g_ap_bytes = 0;
unsigned long long g_ap_clock = 0;

size_t aperture_cache_limit() {
  static long long v = -2;
  if (v == -2) {
    const char* e = std::getenv("CAVITY_APERTURE_CACHE_BYTES");
    v = e ? std::atoll(e) : (1LL << 30);
    if (v < 0) v = 0;
  }
  return (size_t)v;
}

size_t aperture_bytes(const cav::Geo& g) {
  return (size_t)g.P1 * g.P2 * (sizeof(zd) + sizeof(cav::zf)) + 3ull * g.NM * sizeof(zd);
}

bool aperture_match(const ApertureEntry& e, const cav::Geo& g, int s, int method, int dev) {
  return e.dev == dev && e.a == g.a && e.b == g.b && e.k == g.k && e.nx == g.nx &&
         e.ny == g.ny && e.s == s && e.method == method;
}

// On a hit, queue copies of the cached spectrum, its single-precision copy and the
// diagonal into the plan's arrays on stream st and return true.
bool aperture_lookup(const cav::Geo& g, int s, int method, zd* khat, cav::zf* khat_f, zd* diag,
                     hipStream_t st) {
  if (aperture_cache_limit() == 0) return false;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  std::lock_guard<std::mutex> lk(g_ap_mu);
  for (ApertureEntry& e : g_ap) {
    if (!aperture_match(e, g, s, method, dev)) continue;
    const size_t nk = (size_t)g.P1 * g.P2;
    char* base = static_cast<char*>(e.mem);
    if (hipStreamWaitEvent(st, e.ready, 0) != hipSuccess ||
        hipMemcpyAsync(khat, base, nk * sizeof(zd), hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpyAsync(khat_f, base + nk * sizeof(zd), nk * sizeof(cav::zf),
                       hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpyAsync(diag, base + nk * (sizeof(zd) + sizeof(cav::zf)),
                       3ull * g.NM * sizeof(zd), hipMemcpyDeviceToDevice, st) != hipSuccess)
      return false;
    e.last_use = ++g_ap_clock;
    return true;
  }
  return false;
}

// Store a freshly computed aperture (queued on st after its computation).  Best effort:
// any failure leaves the cache unchanged.
void aperture_insert(const cav::Geo& g, int s, int method, const zd* khat, const cav::zf* khat_f,
                     const zd* diag, hipStream_t st) {
  const size_t limit = aperture_cache_limit();
  const size_t bytes = aperture_bytes(g);
  if (limit == 0 || bytes > limit) return;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return;
  {
    std::lock_guard<std::mutex> lk(g_ap_mu);
    for (const ApertureEntry& e : g_ap)
      if (aperture_match(e, g, s, method, dev)) return;   // another plan stored it meanwhile
  }
  void* mem = nullptr;
  if (hipMalloc(&mem, bytes) != hipSuccess) return;
  hipEvent_t ev = nullptr;
  const size_t nk = (size_t)g.P1 * g.P2;
  char* base = static_cast<char*>(mem);
  if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess ||
      hipMemcpyAsync(base, khat, nk * sizeof(zd), hipMemcpyDeviceToDevice, st) != hipSuccess ||
      hipMemcpyAsync(base + nk * sizeof(zd), khat_f, nk * sizeof(cav::zf),
                     hipMemcpyDeviceToDevice, st) != hipSuccess ||
      hipMemcpyAsync(base + nk * (sizeof(zd) + sizeof(cav::zf)), diag, 3ull * g.NM * sizeof(zd),
                     hipMemcpyDeviceToDevice, st) != hipSuccess ||
      hipEventRecord(ev, st) != hipSuccess) {
    (void)hipStreamSynchronize(st);
    if (ev) (void)hipEventDestroy(ev);
    (void)hipFree(mem);
    return;
  }
  std::vector<ApertureEntry> evict;
  {
    std::lock_guard<std::mutex> lk(g_ap_mu);
    while (!g_ap.empty() && g_ap_bytes + bytes > limit) {
      size_t lru = 0;
      for (size_t i = 1; i < g_ap.size(); ++i)
        if (g_ap[i].last_use < g_ap[lru].last_use) lru = i;
      evict.push_back(g_ap[lru]);
      g_ap_bytes -= g_ap[lru].bytes;
      g_ap.erase(g_ap.begin() + lru);
    }
    g_ap.push_back({g.a, g.b, g.k, g.nx, g.ny, s, method, dev, mem, bytes, ev, ++g_ap_clock});
    g_ap_bytes += bytes;
  }
  if (!evict.empty()) {
    (void)hipDeviceSynchronize();
    for (ApertureEntry& e : evict) {
      (void)hipEventDestroy(e.ready);
      (void)hipFree(e.mem);
    }
  }
}

}  // namespace

namespace {

// Validated arguments and derived sizes of a plan.
struct PlanSpec {
  cav::Geo g{};
  cavity_opts o{};
  std::vector<int> lnz;
  std::vector<std::complex<double>> leps;
  std::vector<double> lh;   // grid step of each layer
  bool layered = false;
  double R = 0.0;
  int chunk = 1;
  int fft_len[6] = {};
  int twn = 0;
  size_t need = 0;     // device bytes of the plan with one right-hand side in flight
};

int prepare_plan(double a, double b, double c, int Nx, int Ny, int Nz, const cavity_eps* eps,
                 double k, const cavity_opts* opts, PlanSpec* ps) {
  if (!(a > 0 && b > 0 && c > 0 && k > 0) || !std::isfinite(a) || !std::isfinite(b) ||
      !std::isfinite(c) || !std::isfinite(k))
    return fail(CAVITY_EINVAL, "a, b, c, k must be positive and finite");
  if (Nx < 2 || Ny < 2 || Nz < 1) return fail(CAVITY_EINVAL, "need Nx, Ny >= 2 and Nz >= 1");
  cavity_opts o;
  cavity_opts_default(&o);
  if (opts) o = *opts;
  if (o.precision != CAVITY_FP64 && o.precision != CAVITY_MIXED)
    return fail(CAVITY_EINVAL, "precision must be CAVITY_FP64 or CAVITY_MIXED");
  if (o.tbc_oversample < 1 || o.tbc_oversample > 8)
    return fail(CAVITY_EINVAL, "tbc_oversample must be in 1..8");
  if (!(o.tol > 0 && o.tol < 1) || o.max_iter < 1 || o.restart < 1 || o.restart > 200)
    return fail(CAVITY_EINVAL, "tol in (0,1), max_iter >= 1, restart in 1..200");
  if (o.batch < 1 || o.batch > 64) return fail(CAVITY_EINVAL, "batch must be in 1..64");
  if (o.direct < -1 || o.direct > 1) return fail(CAVITY_EINVAL, "direct must be -1, 0 or 1");
  if (o.spectrum != CAVITY_SPECTRUM_EXACT && o.spectrum != CAVITY_SPECTRUM_ASYMPTOTIC)
    return fail(CAVITY_EINVAL,
                "spectrum must be CAVITY_SPECTRUM_EXACT or CAVITY_SPECTRUM_ASYMPTOTIC");
  if (o.tbc_operator != CAVITY_TBC_TRAP && o.tbc_operator != CAVITY_TBC_SPEC)
    return fail(CAVITY_EINVAL, "tbc_operator must be CAVITY_TBC_TRAP or CAVITY_TBC_SPEC");
  if (o.direct == 1 && 3LL * Nx * Ny > kDenseMax)
    return fail(CAVITY_EINVAL, "direct solve needs 3 Nx Ny <= " + std::to_string(kDenseMax));
  const int s = o.tbc_oversample;
  // the sine/cosine transforms run as FFTs of length 2 s Nx, 2 s Ny, 2 Nx and 2 Ny, built
  // from radices with the prime factors 2, 3, 5, 7, 11 and 13
  for (long long len : {2LL * s * Nx, 2LL * s * Ny, 2LL * Nx, 2LL * Ny})
    if (len > (1 << 20) || fft_plans((int)len).big.nst == 0)
      return fail(CAVITY_ENOTIMPL, "transform length " + std::to_string(len) +
                                       " has a prime factor above 13 (Nx, Ny and s*Nx, s*Ny "
                                       "need prime factors 2, 3, 5, 7, 11, 13)");
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
  // per-layer steps: common c / Nz unless the layer thicknesses are given
  std::vector<double> lh(lnz.size(), c / Nz);
  if (eps && eps->layer_depth) {
    double dsum = 0.0;
    for (size_t i = 0; i < lnz.size(); ++i) {
      const double d = eps->layer_depth[i];
      if (!(d > 0.0) || !std::isfinite(d))
        return fail(CAVITY_EINVAL, "layer thicknesses must be positive and finite");
      dsum += d;
      lh[i] = d / lnz[i];
    }
    if (std::fabs(dsum - c) > 1e-12 * c)
      return fail(CAVITY_EINVAL, "layer thicknesses must sum to c");
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
  g.h = lh.back();   // the aperture rows use the top layer's step
  g.k = k;
  g.hq1 = a / g.nq1;
  g.hq2 = b / g.nq2;
  g.pa = M_PI / a;
  g.pb = M_PI / b;
  g.iab = 1.0 / (a * b);
  g.rows_ip = 1;
  const double R = std::sqrt(2.0) * std::max(a, b);
  g.P1 = next_5smooth((long long)std::ceil((a + R) / g.hq1));
  g.P2 = next_5smooth((long long)std::ceil((b + R) / g.hq2));
  g.ldx = (g.P2 + 15) & ~15;

  if ((size_t)2 * std::max(g.P1, g.P2) * sizeof(zd) > (size_t)kMaxLdsPerBlock)
    return fail(CAVITY_EINVAL, "FFT box too large for one block's LDS");

  const bool layered = lnz.size() > 1;
  const size_t per_level = 3ull * (g.M + 1) * (g.ny + 1) * sizeof(zd);
  const size_t slab = kSynthStagingBytes * (size_t)std::min(4, std::max(1, o.batch / 8));
  int chunk = (int)std::max<size_t>(1, slab / per_level);
  chunk = (int)std::min<long long>(chunk, (long long)(Nz + 1) * o.batch);
  const int fft_len[6] = {2 * g.nq1, 2 * g.nq2, g.P1, g.P2, 2 * g.nx, 2 * g.ny};
  int twn = 0;   // entries of the stage twiddle tables of the six transform lengths
  const bool small_radices = small_radix_plans(fft_len, 6);
  for (int l : fft_len) twn += std::max(1, make_fft_plan(l, small_radices).ntw);
  const int nb0 = 1;
  const size_t need = plan_bytes(g, layered, chunk, (int)lnz.size()) +
                      work_bytes(g, o.restart, nb0, dot_blocks(3LL * g.NM),
                                 o.tbc_operator == CAVITY_TBC_SPEC) +
                      3ull * g.NM * sizeof(zd);
  ps->g = g;
  ps->o = o;
  ps->lnz = lnz;
  ps->leps = leps;
  ps->lh = lh;
  ps->layered = layered;
  ps->R = R;
  ps->chunk = chunk;
  for (int i = 0; i < 6; ++i) ps->fft_len[i] = fft_len[i];
  ps->twn = twn;
  ps->need = need;
  return CAVITY_OK;
}

}  // namespace

namespace cav {
int footprint_per_rhs(double a, double b, double c, int Nx, int Ny, int Nz, const cavity_eps* eps,
                      double k, const cavity_opts* opts, size_t* bytes) {
  PlanSpec ps;
  const int st = prepare_plan(a, b, c, Nx, Ny, Nz, eps, k, opts, &ps);
  if (st) return st;
  const bool spec = ps.o.tbc_operator == CAVITY_TBC_SPEC;
  const int nblk = dot_blocks(3LL * ps.g.NM);
  *bytes = work_bytes(ps.g, ps.o.restart, 2, nblk, spec) - work_bytes(ps.g, ps.o.restart, 1, nblk, spec) +
           15ull * ps.g.NM * sizeof(zd) + 2 * sizeof(double);
  return CAVITY_OK;
}
}  // namespace cav

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
  o->batch = 8;
  o->direct = 0;
  o->tbc_operator = CAVITY_TBC_TRAP;
  o->spectrum = CAVITY_SPECTRUM_EXACT;
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

int cavity_plan_footprint(double a, double b, double c, int Nx, int Ny, int Nz,
                          const cavity_eps* eps, double k, const cavity_opts* opts,
                          size_t* bytes) {
  if (!bytes) return fail(CAVITY_EINVAL, "NULL output");
  PlanSpec ps;
  const int st = prepare_plan(a, b, c, Nx, Ny, Nz, eps, k, opts, &ps);
  if (st) return st;
  *bytes = ps.need;
  return CAVITY_OK;
}

int cavity_plan_create(double a, double b, double c, int Nx, int Ny, int Nz,
                       const cavity_eps* eps, double k, const cavity_opts* opts,
                       cavity_plan* out) {
  if (!out) return fail(CAVITY_EINVAL, "NULL plan output");
  *out = nullptr;
  // CAVITY_TRACE: host time of the plan's set-up steps on stderr
  static const bool trace = std::getenv("CAVITY_TRACE") != nullptr;
  auto t_prev = std::chrono::steady_clock::now();
  auto lap = [&](const char* what) {
    if (!trace) return;
    const auto t = std::chrono::steady_clock::now();
    std::fprintf(stderr, "[plan] %s %.1f us\n", what,
                 std::chrono::duration<double, std::micro>(t - t_prev).count());
    t_prev = t;
  };
  PlanSpec ps;
  {
    const int st0 = prepare_plan(a, b, c, Nx, Ny, Nz, eps, k, opts, &ps);
    if (st0) return st0;
  }
  const cav::Geo& g = ps.g;
  const cavity_opts& o = ps.o;
  const std::vector<int>& lnz = ps.lnz;
  const std::vector<std::complex<double>>& leps = ps.leps;
  const bool layered = ps.layered;
  const double R = ps.R;
  const int chunk = ps.chunk;
  const int* fft_len = ps.fft_len;
  const int twn = ps.twn;
  const size_t need = ps.need;
  size_t budget = o.hbm_budget;
  if (budget == 0) {
    size_t fr = 0, tot = 0;
    HIPCHK(hipMemGetInfo(&fr, &tot));
    budget = (size_t)(0.9 * (double)(fr + g_cache_bytes));
  }
  if (need > budget)
    return fail(CAVITY_ENOMEM, "plan needs " + std::to_string(need) + " bytes, budget " +
                                   std::to_string(budget));

  lap("prepare + memory info");
  cavity_plan p = new cavity_plan_s();
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return fail(CAVITY_EDEVICE, "hipGetDevice failed");
  }
  p->g = g;
  p->opts = o;
  p->st = static_cast<hipStream_t>(o.stream);
  p->layered = layered;
  p->nlayers = (int)lnz.size();
  p->R = R;
  p->nblk_red = dot_blocks(p->nvec());
  p->synth_chunk = chunk;
  auto bail = [&](int code) {
    release(p);
    return code;
  };
  for (auto& e : p->ev)
    if (event_get(&e, true) != hipSuccess) return bail(fail(CAVITY_EDEVICE, "hipEventCreate failed"));
  if (pinned_get(flag_bytes(o.restart), (void**)&p->hflags) != hipSuccess ||
      pinned_get(ratio_bytes(o.restart), (void**)&p->hratio) != hipSuccess ||
      pinned_get(norm_bytes(), (void**)&p->hn) != hipSuccess)
    return bail(fail(CAVITY_EDEVICE, "hipHostMalloc failed"));
  lap("events + pinned flags");

  // one arena for all plan data
  const long long NM = g.NM;
  Layout L;
  L.add(&p->khat, (size_t)g.P1 * g.P2);
  L.add(&p->rho_d, NM);
  L.add(&p->T, NM);
  L.add(&p->rho_n, NM);
  L.add(&p->pi_d, (size_t)(Nz + 1) * NM);
  L.add(&p->pi_n, (size_t)(Nz + 1) * NM);
  if (layered) L.add(&p->theta_d, (size_t)(Nz + 1) * NM);
  L.add(&p->pinv, 9 * NM);
  L.add(&p->diag, 3 * NM);
  L.add(&p->pivmin, NM);
  L.add(&p->dmin, 1);
  L.add(&p->node_code, Nz + 1);
  L.add(&p->kappa2, lnz.size());
  L.add(&p->ratio, lnz.size());
  L.add(&p->hl, lnz.size());
  L.add(&p->khat_f, (size_t)g.P1 * g.P2);
  L.add(&p->pw1, (size_t)2 * (g.M + 1) * g.P1);
  L.add(&p->pw2, (size_t)2 * g.P2 * (g.N + 1));
  L.add(&p->ctmp, (size_t)2 * g.P1 * (g.N + 1));
  L.add(&p->tbuf, (size_t)3 * chunk * (g.M + 1) * (g.ny + 1));
  L.add(&p->r, std::max<size_t>(3 * NM, (size_t)g.P1 * g.P2));
  L.add(&p->dbg_out, 3 * NM);
  L.add(&p->dwave1, 8);
  {
    void* base = nullptr;
    int st0 = arena_acquire(L.bytes, &base);
    if (st0) return bail(st0);
    p->plan_arena = {base, L.bytes};
    L.bind(base);
  }
  lap("arena");

  // transform plans and their stage twiddles (shared device tables); host tables: node
  // codes, k^2 eps per layer, eps ratios per interface
  {
    cav::Fft* dst[6] = {&p->trig.ext1, &p->trig.ext2, &p->trig.box1, &p->trig.box2,
                        &p->trig.out1, &p->trig.out2};
    cav::FftPlan plans[6];
    p->trig.maxr = 1;
    const bool small_radices = small_radix_plans(fft_len, 6);
    for (int i = 0; i < 6; ++i) {
      plans[i] = make_fft_plan(fft_len[i], small_radices);
      p->trig.maxr = std::max(p->trig.maxr, plan_max_radix(plans[i]));
    }
    StageTwiddles stw;
    if (const int s0 = stage_twiddles(p->device, fft_len, small_radices, plans, twn, p->st, &stw))
      return bail(s0);
    int off = 0;
    for (int i = 0; i < 6; ++i) {
      dst[i]->p = plans[i];
      dst[i]->tw = stw.tw + off;
      dst[i]->twf = stw.twf + off;
      off += std::max(1, plans[i].ntw);
    }
    // CAVITY_FFT_MAXR=16: the same plans run by the kernels compiled for radices up to 16
    if (const char* e = std::getenv("CAVITY_FFT_MAXR"))
      if (std::atoi(e) == cav::kMaxRadix) p->trig.maxr = cav::kMaxRadix;
  }
  std::vector<int> code(Nz + 1, 0);
  std::vector<zd> kap(lnz.size()), rat(lnz.size(), cav::mk(1.0, 0.0));
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
  lap("host tables");
  auto chk = [&](hipError_t e, const char* what) {
    if (e != hipSuccess) {
      fail(CAVITY_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
      return false;
    }
    return true;
  };
  if (!chk(hipMemcpyAsync(p->node_code, code.data(), code.size() * sizeof(int),
                          hipMemcpyHostToDevice, p->st), "layer upload") ||
      !chk(hipMemcpyAsync(p->kappa2, kap.data(), kap.size() * sizeof(zd), hipMemcpyHostToDevice,
                          p->st), "layer upload") ||
      !chk(hipMemcpyAsync(p->ratio, rat.data(), rat.size() * sizeof(zd), hipMemcpyHostToDevice,
                          p->st), "layer upload") ||
      !chk(hipMemcpyAsync(p->hl, ps.lh.data(), ps.lh.size() * sizeof(double),
                          hipMemcpyHostToDevice, p->st), "layer upload"))
    return bail(CAVITY_EDEVICE);
  lap("uploads");

  // spectrum (scaled for the unnormalised inverse FFT and the grid cell)
  const double scale = 1.0 / (g.hq1 * g.hq2 * (double)g.P1 * (double)g.P2);
  int st = CAVITY_OK;
  if ((st = mark(p, 0, false))) return bail(st);
  const bool cached =
      aperture_lookup(g, o.tbc_oversample, o.spectrum, p->khat, p->khat_f, p->diag, p->st);
  if (!cached &&
      (!chk(cav::launch_spectrum(g, R, scale, o.spectrum, p->khat, p->st), "spectrum") ||
       !chk(cav::launch_to_f32(p->khat, p->khat_f, (long long)g.P1 * g.P2, p->st), "spectrum")))
    return bail(CAVITY_EDEVICE);
  if ((st = mark(p, 0, true))) return bail(st);
  cav::Layers ly{p->node_code, p->kappa2, p->ratio, p->hl, layered ? 1 : 0};
  if ((st = mark(p, 1, false))) return bail(st);
  if (!chk(cav::launch_elimination(g, ly, p->rho_d, p->T, p->rho_n, p->pi_d, p->theta_d, p->pi_n,
                                   p->pivmin, p->st), "elimination"))
    return bail(CAVITY_EDEVICE);
  if ((st = mark(p, 1, true))) return bail(st);
  if ((st = mark(p, 2, false))) return bail(st);
  if (p->use_spec()) {
    // the spectral operator's own diagonal (the cache holds the trapezoid one)
    if ((st = build_spec(p))) return bail(st);
    if (!chk(cav::launch_diag_contract(g, p->khat, p->pw1, p->pw2, p->ctmp, p->diag, p->st),
             "diagonal"))
      return bail(CAVITY_EDEVICE);
  } else {
    if (!cached &&
        (!chk(cav::launch_basis_power(g, p->trig, p->pw1, p->pw2, p->st), "basis power") ||
         !chk(cav::launch_diag_contract(g, p->khat, p->pw1, p->pw2, p->ctmp, p->diag, p->st),
              "diagonal")))
      return bail(CAVITY_EDEVICE);
    if (!cached)
      aperture_insert(g, o.tbc_oversample, o.spectrum, p->khat, p->khat_f, p->diag, p->st);
  }
  p->cols = cav::Cols{p->rho_d, p->T, p->rho_n, p->pinv, 0, nullptr};
  if (!chk(cav::launch_precond_build(g, p->rho_d, p->T, p->rho_n, p->diag, p->pinv, p->st),
           "preconditioner"))
    return bail(CAVITY_EDEVICE);
  if ((st = mark(p, 2, true))) return bail(st);
  lap("launches");
  if (!chk(cav::launch_min(p->pivmin, NM, p->dmin, p->st), "pivot minimum") ||
      !chk(hipMemcpyAsync(p->hn, p->dmin, sizeof(double), hipMemcpyDeviceToHost, p->st),
           "pivot copy") ||
      !chk(hipStreamSynchronize(p->st), "plan sync"))
    return bail(CAVITY_EDEVICE);
  p->info.min_pivot = p->hn[0];
  if (!(p->info.min_pivot > 1e-13))
    return bail(fail(CAVITY_ERESONANT, "z-elimination pivot below 1e-13"));
  lap("device work + sync");
  p->info.tbc_rows_in_place = p->g.rows_ip;
  if ((st = autotune_lds(p))) return bail(st);
  lap("tuning");
  // CAVITY_TBC_ROWS_IP=0 or 1 fixes the form of the TBC row passes (after any tuning)
  if (const char* e = std::getenv("CAVITY_TBC_ROWS_IP")) {
    p->g.rows_ip = std::atoi(e) != 0 ? 1 : 0;
    p->info.tbc_rows_in_place = p->g.rows_ip;
  }
  p->info.M = g.M;
  p->info.N = g.N;
  p->info.Nz = Nz;
  p->info.P1 = g.P1;
  p->info.P2 = g.P2;
  p->info.n_ap = (long long)(g.M + 1) * g.N + (long long)g.M * (g.N + 1) + (long long)g.M * g.N;
  p->info.unknowns = p->info.n_ap * Nz;
  *out = p;
  return CAVITY_OK;
}

void cavity_plan_destroy(cavity_plan p) { release(p); }

int cavity_plan_info(cavity_plan p, cavity_info* out) {
  if (!p || !out) return fail(CAVITY_EINVAL, "NULL argument");
  resolve_timers(p);
  p->info.device_bytes = p->plan_arena.bytes + p->work_arena.bytes + p->sol_arena.bytes +
                         p->dense_arena.bytes + p->rcs_arena.bytes + p->spec_arena.bytes +
                         p->group_arena.bytes;
  *out = p->info;
  return CAVITY_OK;
}

int cavity_solve(cavity_plan p, double theta, double phi, int pol, cavity_c128* E_out) {
  if (!p) return fail(CAVITY_EINVAL, "NULL plan");
  return cavity_solve_batch(p, 1, &theta, &phi, &pol, E_out, nullptr);
}

int cavity_solve_batch(cavity_plan p, int nrhs, const double* theta, const double* phi,
                       const int* pol, cavity_c128* E_out, cavity_c128* aperture_out) {
  if (!p || nrhs < 1 || !theta || !phi || !pol) return fail(CAVITY_EINVAL, "bad batch arguments");
  if (!cav::aligned16(E_out) || !cav::aligned16(aperture_out))
    return fail(CAVITY_EINVAL, "device outputs must be 16-byte aligned");
  for (int i = 0; i < nrhs; ++i)
    if (!angles_ok(theta[i], phi[i], pol[i]))
      return fail(CAVITY_EINVAL, "theta must lie in [0, pi/2], phi finite, pol TM or TE");
  // the stored solutions are those of this call only: indices 0..nrhs-1 once it succeeds
  p->nsol = 0;
  int s = ensure_solutions(p, nrhs);
  if (s) return s;
  const long long n = p->nvec();
  const int dm = p->opts.direct;
  p->dense_now = dm == 1 || (dm == 0 && n <= kDenseAuto &&
                             (p->dense_F != nullptr || nrhs >= kDenseAutoRhs));
  const int group = p->dense_now ? kDenseGroup : p->opts.batch;
  if ((s = ensure_work(p, std::min(nrhs, group)))) return s;
  if (p->dense_now && (s = dense_factor(p))) {
    // the automatic choice falls back to GMRES when the inverse does not fit in memory
    if (s != CAVITY_ENOMEM || p->opts.direct == 1) return s;
    p->dense_now = false;
    if ((s = ensure_work(p, std::min(nrhs, p->opts.batch)))) return s;
  }
  p->info.last_direct = p->dense_now ? 1 : 0;
  const long long field = 3LL * (p->g.Nz + 1) * (p->g.ny + 1) * (p->g.nx + 1);
  int worst = CAVITY_OK;
  int its = 0;
  double res = 0.0;
  for (int i0 = 0; i0 < nrhs; i0 += p->nbwork) {
    const int nb = std::min(p->nbwork, nrhs - i0);
    s = solve_chunk(p, i0, nb, theta + i0, phi + i0, pol + i0, E_out ? E_out + i0 * field : nullptr,
                    aperture_out ? aperture_out + i0 * p->info.n_ap : nullptr);
    if (s != CAVITY_OK && s != CAVITY_ENOCONV) return s;
    if (s == CAVITY_ENOCONV) worst = s;
    its = std::max(its, p->info.last_iterations);
    res = std::max(res, p->info.last_rel_residual);
    p->nsol = i0 + nb;
  }
  p->info.last_iterations = its;
  p->info.last_rel_residual = res;
  if (worst != CAVITY_OK)
    return fail(worst, p->dense_now ? "direct solve did not reach the tolerance"
                                    : "GMRES did not reach the tolerance");
  return CAVITY_OK;
}

int cavity_solve_group(int n, const cavity_plan* plans, const double* theta, const double* phi,
                       const int* pol, cavity_c128* const* E_out) {
  if (n < 1 || n > 64 || !plans || !theta || !phi || !pol)
    return fail(CAVITY_EINVAL, "group needs 1..64 plans and host angle arrays");
  cavity_plan lead = plans[0];
  if (!lead) return fail(CAVITY_EINVAL, "NULL plan in group");
  for (int r = 0; r < n; ++r) {
    const cavity_plan q = plans[r];
    if (!q) return fail(CAVITY_EINVAL, "NULL plan in group");
    for (int t = 0; t < r; ++t)
      if (plans[t] == q) return fail(CAVITY_EINVAL, "a plan appears twice in the group");
    if (!angles_ok(theta[r], phi[r], pol[r]))
      return fail(CAVITY_EINVAL, "theta must lie in [0, pi/2], phi finite, pol TM or TE");
    if (E_out && !cav::aligned16(E_out[r]))
      return fail(CAVITY_EINVAL, "device outputs must be 16-byte aligned");
    const cav::Geo &a = lead->g, &b = q->g;
    if (a.M != b.M || a.N != b.N || a.nq1 != b.nq1 || a.nq2 != b.nq2 || a.P1 != b.P1 ||
        a.P2 != b.P2 || a.a != b.a || a.b != b.b || a.k != b.k || q->device != lead->device ||
        q->opts.spectrum != lead->opts.spectrum || q->opts.precision != lead->opts.precision ||
        q->opts.tol != lead->opts.tol || q->opts.restart != lead->opts.restart ||
        q->opts.max_iter != lead->opts.max_iter)
      return fail(CAVITY_EINVAL, "group plans need one aperture (a, b, Nx, Ny, k, oversampling, "
                                 "spectrum) and the same precision, tol, restart and max_iter");
    if (q->use_spec()) return fail(CAVITY_ENOTIMPL, "group solves use the trapezoid operator");
  }
  for (int r = 1; r < n; ++r) {
    if (plans[r]->st) HIPCHK(hipStreamSynchronize(plans[r]->st));
    else HIPCHK(hipDeviceSynchronize());
  }
  int s;
  if ((s = ensure_work(lead, n)) || (s = ensure_solutions(lead, n))) return s;
  // gather each cavity's column data: [rho_d | T | rho_n | pinv] per right-hand side, then h
  const long long NM = lead->g.NM;
  const long long cs = 12 * NM;
  const size_t need = (size_t)n * cs * sizeof(zd) + (size_t)n * sizeof(double) + 256;
  if (need > lead->group_arena.bytes) {
    if (lead->st) HIPCHK(hipStreamSynchronize(lead->st));
    else HIPCHK(hipDeviceSynchronize());
    arena_release(lead->group_arena.ptr, lead->group_arena.bytes);
    lead->group_arena = Arena();
    void* base = nullptr;
    if ((s = arena_acquire(need, &base))) return s;
    lead->group_arena = {base, need};
  }
  zd* gc = static_cast<zd*>(lead->group_arena.ptr);
  double* gh = reinterpret_cast<double*>(gc + (size_t)n * cs);
  lead->group_h.assign(n, 0.0);
  for (int r = 0; r < n; ++r) {
    const cavity_plan q = plans[r];
    zd* dst = gc + (size_t)r * cs;
    HIPCHK(hipMemcpyAsync(dst, q->rho_d, NM * sizeof(zd), hipMemcpyDeviceToDevice, lead->st));
    HIPCHK(hipMemcpyAsync(dst + NM, q->T, NM * sizeof(zd), hipMemcpyDeviceToDevice, lead->st));
    HIPCHK(hipMemcpyAsync(dst + 2 * NM, q->rho_n, NM * sizeof(zd), hipMemcpyDeviceToDevice,
                          lead->st));
    HIPCHK(hipMemcpyAsync(dst + 3 * NM, q->pinv, 9 * NM * sizeof(zd), hipMemcpyDeviceToDevice,
                          lead->st));
    lead->group_h[r] = q->g.h;
  }
  HIPCHK(hipMemcpyAsync(gh, lead->group_h.data(), n * sizeof(double), hipMemcpyHostToDevice,
                        lead->st));
  const cav::Cols own = lead->cols;
  lead->cols = cav::Cols{gc, gc + NM, gc + 2 * NM, gc + 3 * NM, cs, gh};
  lead->dense_now = false;
  lead->nsol = 0;
  const int status = solve_chunk(lead, 0, n, theta, phi, pol, nullptr, nullptr);
  lead->cols = own;
  if (status != CAVITY_OK && status != CAVITY_ENOCONV) return status;
  // each plan keeps its own solution as index 0; fields from its own profiles
  const long long nv = lead->nvec();
  for (int r = 0; r < n; ++r) {
    const cavity_plan q = plans[r];
    if (r > 0) {
      q->nsol = 0;
      if ((s = ensure_solutions(q, 1))) return s;
      HIPCHK(hipMemcpyAsync(q->xsol, lead->xsol + (long long)r * nv, nv * sizeof(zd),
                            hipMemcpyDeviceToDevice, lead->st));
    }
    q->nsol = 1;
    q->info.last_iterations = lead->info.last_iterations;
    q->info.last_rel_residual = lead->info.last_rel_residual;
    q->info.last_direct = 0;
    if (E_out && E_out[r]) {
      for (int j0 = 0; j0 <= q->g.Nz; j0 += q->synth_chunk) {
        const int j1 = std::min(q->g.Nz + 1, j0 + q->synth_chunk);
        HIPCHK(cav::launch_synthesis(q->g, q->trig, q->pi_d, q->layered ? q->theta_d : nullptr,
                                     q->pi_n, q->xsol, nv, 1, j0, j1, q->tbuf,
                                     reinterpret_cast<zd*>(E_out[r]), 0, lead->st));
      }
    }
  }
  HIPCHK(hipStreamSynchronize(lead->st));
  if (status != CAVITY_OK) return fail(status, "GMRES did not reach the tolerance");
  return CAVITY_OK;
}

int cavity_aperture(cavity_plan p, int idx, cavity_c128* out_host) {
  if (!p || !out_host || idx < 0 || idx >= p->nsol) return fail(CAVITY_EINVAL, "no such solution");
  HIPCHK(cav::launch_pack(p->g, p->xsol + (long long)idx * p->nvec(), p->dbg_out, p->st));
  HIPCHK(hipMemcpyAsync(out_host, p->dbg_out, p->info.n_ap * sizeof(zd), hipMemcpyDeviceToHost,
                        p->st));
  HIPCHK(hipStreamSynchronize(p->st));
  return CAVITY_OK;
}

int cavity_rcs(cavity_plan p, int idx, int n_obs, const double* th, const double* ph,
               double* sigma) {
  if (!p || idx < 0 || idx >= p->nsol || n_obs < 0 || (n_obs > 0 && (!th || !ph || !sigma)))
    return fail(CAVITY_EINVAL, "bad rcs arguments");
  std::vector<int> rhs(n_obs, idx);
  return rcs_queries(p, n_obs, rhs.data(), th, ph, sigma);
}

int cavity_rcs_many(cavity_plan p, int n, const int* rhs_index, const double* th,
                    const double* ph, double* sigma) {
  if (!p || n < 0 || (n > 0 && (!rhs_index || !th || !ph || !sigma)))
    return fail(CAVITY_EINVAL, "bad rcs arguments");
  for (int i = 0; i < n; ++i)
    if (rhs_index[i] < 0 || rhs_index[i] >= p->nsol) return fail(CAVITY_EINVAL, "no such solution");
  return rcs_queries(p, n, rhs_index, th, ph, sigma);
}

int cavity_probe_kernel(int which, int capacity) {
  using cav::g_probe;
  for (hipEvent_t e : g_probe.pool) (void)hipEventDestroy(e);
  g_probe = cav::ProbeState();
  if (which < 0) return CAVITY_OK;
  if (which >= cav::K_COUNT || capacity < 1) return fail(CAVITY_EINVAL, "bad probe arguments");
  g_probe.pool.resize(2 * (size_t)capacity + 2);
  // timing only: no system-scope fence (cache writeback and invalidate) at each record,
  // which would slow the work around the probed launches
  for (auto& e : g_probe.pool)
    HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
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
  int s = ensure_work(p, 1);
  if (s) return s;
  HIPCHK(hipMemcpy(p->r, in, NM * sizeof(zd), hipMemcpyHostToDevice));
  if (p->use_spec())
    HIPCHK(cav::launch_spec_passes(p->g, p->spec, p->khat, nullptr, 0, family, 1, p->r, 0, p->X,
                                   p->Y, p->U, p->dbg_out, nullptr, p->st));
  else
    HIPCHK(cav::launch_single_family(p->g, p->trig, p->khat, family, p->r, p->X, p->Y,
                                     p->dbg_out, p->st));
  return copy_out(p, p->dbg_out, out, NM);
}

int cavity_debug_operator(cavity_plan p, const cavity_c128* in, cavity_c128* out) {
  if (!p || !in || !out) return fail(CAVITY_EINVAL, "NULL argument");
  const size_t n = 3 * (size_t)p->g.NM;
  int s = ensure_work(p, 1);
  if (s) return s;
  HIPCHK(hipMemcpy(p->r, in, n * sizeof(zd), hipMemcpyHostToDevice));
  if ((s = run_operator(p, 0, 1, p->r, p->dbg_out, nullptr))) return s;
  return copy_out(p, p->dbg_out, out, n);
}

int cavity_debug_rhs(cavity_plan p, double theta, double phi, int pol, cavity_c128* g1,
                     cavity_c128* g2) {
  if (!p || !g1 || !g2) return fail(CAVITY_EINVAL, "NULL argument");
  cav::Wave wv;
  wave_setup(p->g.k, p->g.h, theta, phi, pol, &wv);
  HIPCHK(hipMemcpy(p->dwave1, &wv, sizeof(wv), hipMemcpyHostToDevice));
  HIPCHK(cav::launch_rhs(p->g, p->dwave1, 1, p->r, p->st));
  int s;
  if ((s = copy_out(p, p->r, g1, p->g.NM)) || (s = copy_out(p, p->r + p->g.NM, g2, p->g.NM)))
    return s;
  return CAVITY_OK;
}

int cavity_debug_fft_plans(const int* len, int* radices, int* nst) {
  if (!len || !radices || !nst) return fail(CAVITY_EINVAL, "NULL argument");
  for (int i = 0; i < 6; ++i)
    if (len[i] < 1 || len[i] > (1 << 20)) return fail(CAVITY_EINVAL, "transform length out of range");
  const bool small_radices = small_radix_plans(len, 6);
  for (int i = 0; i < 6; ++i) {
    const cav::FftPlan pl = make_fft_plan(len[i], small_radices);
    nst[i] = pl.nst;
    for (int t = 0; t < 20; ++t) radices[20 * i + t] = t < pl.nst ? pl.radix[t] : 0;
  }
  return CAVITY_OK;
}

}  // extern "C"
