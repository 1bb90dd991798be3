// Request server: many cavities, each solved for one incidence, with several requests in
// flight on the GPU at once.  Worker threads each own a HIP stream; a free worker takes the
// oldest queued request whose device footprint fits in the budget left by the requests
// running and the resident plans, and the plan of a finished request stays resident for a
// later request on the same cavity.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "cavity.h"
#include "runtime.hpp"

namespace {

// A request passed over by later ones for longer than this is the only one admitted next.
constexpr double kMaxBypassMs = 25.0;
// Most requests solved together as one lockstep group.
constexpr int kMaxGroup = 8;

struct Pending {
  long long ticket;
  cavity_request req;
  std::vector<int> lnz;
  std::vector<cavity_c128> eps;
  std::string key;        // the cavity (geometry, grid, layers, k): equal keys share a plan
  std::string ap_key;     // the aperture (a, b, Nx, Ny, k): equal keys may share a group
  size_t plan_bytes;      // plan + workspace + solution (cavity_plan_footprint)
  size_t rhs_bytes;       // what one more right-hand side adds to a group leader's plan
  size_t field_bytes;     // temporary field buffer, 0 when the caller gave E_out
  double t_submit_ms;
};

struct Done {
  cavity_result res;
};

// A plan kept after its request, charged to the budget at its footprint.
struct Resident {
  std::string key;
  cavity_plan plan;
  size_t bytes;
  unsigned long long last_use;
  bool busy;
};

std::string cavity_key(const cavity_request& r, const std::vector<int>& lnz,
                       const std::vector<cavity_c128>& eps) {
  std::string k;
  auto put = [&](const void* p, size_t n) { k.append(static_cast<const char*>(p), n); };
  const double d[4] = {r.a, r.b, r.c, r.k};
  const int n[4] = {r.Nx, r.Ny, r.Nz, (int)lnz.size()};
  put(d, sizeof(d));
  put(n, sizeof(n));
  if (!lnz.empty()) put(lnz.data(), lnz.size() * sizeof(int));
  if (!eps.empty()) put(eps.data(), eps.size() * sizeof(cavity_c128));
  return k;
}

std::string aperture_key(const cavity_request& r) {
  std::string k;
  const double d[3] = {r.a, r.b, r.k};
  const int n[2] = {r.Nx, r.Ny};
  k.append(reinterpret_cast<const char*>(d), sizeof(d));
  k.append(reinterpret_cast<const char*>(n), sizeof(n));
  return k;
}

}  // namespace

struct cavity_server_s {
  cavity_server_opts opts{};
  int device = 0;
  size_t budget = 0;
  size_t in_use = 0;              // running requests and resident plans
  size_t plan_cache_limit = 0;
  size_t resident_bytes = 0;
  unsigned long long clock = 0;
  std::chrono::steady_clock::time_point t0;
  std::vector<std::thread> workers;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Pending> queue;
  std::vector<Resident> resident;
  std::map<long long, Done> done;
  std::set<long long> live;     // submitted and not yet released
  long long next_ticket = 1;
  int running = 0;
  int ready = 0;                // workers that have set up their stream
  bool stopping = false;
  bool trace = false;             // CAVITY_SERVER_TRACE=1: admissions on stderr

  double now_ms() const {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
        .count();
  }
  // Index of an idle resident plan for key, or -1 (caller holds mu).
  int idle_plan(const std::string& key) const {
    for (size_t i = 0; i < resident.size(); ++i)
      if (!resident[i].busy && resident[i].key == key) return (int)i;
    return -1;
  }
  // Bytes request pd needs on top of in_use, and bytes of idle resident plans it could
  // evict for them (caller holds mu).
  size_t need_of(const Pending& pd, int reuse) const {
    return reuse >= 0 ? pd.field_bytes : pd.plan_bytes + pd.field_bytes;
  }
  size_t evictable(int keep) const {
    size_t b = 0;
    for (size_t i = 0; i < resident.size(); ++i)
      if (!resident[i].busy && (int)i != keep) b += resident[i].bytes;
    return b;
  }
  bool fits(const Pending& pd) const {
    const int reuse = idle_plan(pd.key);
    return in_use + need_of(pd, reuse) <= budget + evictable(reuse);
  }
  // The queued request a free worker takes: the oldest that fits, unless the head has been
  // passed over for longer than kMaxBypassMs (then the head or nothing).  -1: none.
  int pick() const {
    for (size_t i = 0; i < queue.size(); ++i) {
      if (fits(queue[i])) return (int)i;
      if (i == 0 && now_ms() - queue[0].t_submit_ms > kMaxBypassMs) return -1;
    }
    return -1;
  }
  // Drop idle resident plans, least recently used first (never `keep`), until `extra` more
  // bytes fit in the budget and the resident total is within its limit.  The plans are
  // returned for destruction outside the lock (caller holds mu).
  std::vector<cavity_plan> evict_for(size_t extra, cavity_plan keep) {
    std::vector<cavity_plan> out;
    while (in_use + extra > budget || resident_bytes > plan_cache_limit) {
      int lru = -1;
      for (size_t i = 0; i < resident.size(); ++i)
        if (!resident[i].busy && resident[i].plan != keep &&
            (lru < 0 || resident[i].last_use < resident[lru].last_use))
          lru = (int)i;
      if (lru < 0) break;
      out.push_back(resident[lru].plan);
      in_use -= resident[lru].bytes;
      resident_bytes -= resident[lru].bytes;
      resident.erase(resident.begin() + lru);
    }
    return out;
  }
  bool has_resident(const std::string& key) const {
    for (const Resident& rp : resident)
      if (rp.key == key) return true;
    return false;
  }
  void work();
};

namespace {

size_t field_bytes_of(const cavity_request& r) {
  return 3ull * (size_t)(r.Nz + 1) * (size_t)(r.Ny + 1) * (size_t)(r.Nx + 1) *
         sizeof(cavity_c128);
}

void fill_eps(const Pending& pd, cavity_eps* e) {
  e->n_layers = (int)pd.lnz.size();
  e->layer_nz = pd.lnz.data();
  e->eps_r = pd.eps.data();
}

// One request on stream st: plan (given, or created into *plan), solve into the field
// buffer, backscatter RCS.
void run_request(const cavity_server_opts& so, hipStream_t st, const Pending& pd, void* field,
                 cavity_plan* plan, cavity_result* res) {
  const cavity_request& r = pd.req;
  int s = CAVITY_OK;
  if (*plan) {
    s = cav::plan_set_stream(*plan, st);
  } else {
    cavity_opts o;
    cavity_opts_default(&o);
    o.precision = so.precision;
    o.tol = so.tol;
    o.batch = 1;
    o.stream = st;
    o.hbm_budget = pd.plan_bytes + ((size_t)64 << 20);
    cavity_eps e{};
    fill_eps(pd, &e);
    s = cavity_plan_create(r.a, r.b, r.c, r.Nx, r.Ny, r.Nz, pd.lnz.empty() ? nullptr : &e, r.k,
                           &o, plan);
  }
  if (s == CAVITY_OK) {
    s = cavity_solve(*plan, r.theta, r.phi, r.pol, static_cast<cavity_c128*>(field));
    if (s == CAVITY_OK || s == CAVITY_ENOCONV) {
      const int s2 = cavity_rcs(*plan, 0, 1, &r.theta, &r.phi, res->sigma);
      if (s == CAVITY_OK) s = s2;
      cavity_info inf{};
      if (cavity_plan_info(*plan, &inf) == CAVITY_OK) {
        res->iterations = inf.last_iterations;
        res->rel_residual = inf.last_rel_residual;
        res->unknowns = inf.unknowns;
      }
    }
  }
  if (hipStreamSynchronize(st) != hipSuccess && s == CAVITY_OK) s = CAVITY_EDEVICE;
  res->status = s;
}

// Requests on cavities that share an aperture, solved as one lockstep group on stream st:
// a plan each (created here), one group solve, the backscatter RCS of each.  A request whose
// plan cannot be created fails alone; the others are still solved together.
void run_group(const cavity_server_opts& so, hipStream_t st, const std::vector<Pending>& grp,
               const std::vector<void*>& fields, std::vector<cavity_plan>* plans,
               std::vector<cavity_result>* res) {
  const int n = (int)grp.size();
  std::vector<cavity_plan> live;
  std::vector<int> idx;
  std::vector<double> th, ph;
  std::vector<int> po;
  std::vector<cavity_c128*> eo;
  for (int r = 0; r < n; ++r) {
    const Pending& pd = grp[r];
    const cavity_request& q = pd.req;
    cavity_opts o;
    cavity_opts_default(&o);
    o.precision = so.precision;
    o.tol = so.tol;
    o.batch = 1;
    o.stream = st;
    o.hbm_budget = pd.plan_bytes + (size_t)n * pd.rhs_bytes + ((size_t)64 << 20);
    cavity_eps e{};
    fill_eps(pd, &e);
    const int s = cavity_plan_create(q.a, q.b, q.c, q.Nx, q.Ny, q.Nz,
                                     pd.lnz.empty() ? nullptr : &e, q.k, &o, &(*plans)[r]);
    if (s != CAVITY_OK) {
      (*res)[r].status = s;
      continue;
    }
    live.push_back((*plans)[r]);
    idx.push_back(r);
    th.push_back(q.theta);
    ph.push_back(q.phi);
    po.push_back(q.pol);
    eo.push_back(static_cast<cavity_c128*>(fields[r]));
  }
  if (!live.empty()) {
    int s = cavity_solve_group((int)live.size(), live.data(), th.data(), ph.data(), po.data(),
                               eo.data());
    for (size_t i = 0; i < live.size(); ++i) {
      cavity_result& rr = (*res)[idx[i]];
      const cavity_request& q = grp[idx[i]].req;
      int si = s;
      if (s == CAVITY_OK || s == CAVITY_ENOCONV) {
        const int s2 = cavity_rcs(live[i], 0, 1, &q.theta, &q.phi, rr.sigma);
        if (si == CAVITY_OK) si = s2;
        cavity_info inf{};
        if (cavity_plan_info(live[i], &inf) == CAVITY_OK) {
          rr.iterations = inf.last_iterations;
          rr.rel_residual = inf.last_rel_residual;
          rr.unknowns = inf.unknowns;
        }
      }
      rr.status = si;
    }
  }
  if (hipStreamSynchronize(st) != hipSuccess)
    for (int r = 0; r < n; ++r)
      if ((*res)[r].status == CAVITY_OK) (*res)[r].status = CAVITY_EDEVICE;
}

}  // namespace

void cavity_server_s::work() {
  (void)hipSetDevice(device);
  hipStream_t st = nullptr;
  const bool have_stream = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
  {
    std::lock_guard<std::mutex> lk(mu);
    ++ready;
  }
  cv_done.notify_all();
  while (true) {
    std::vector<Pending> grp;
    cavity_plan reused = nullptr;
    size_t lead_extra = 0;     // group workspace the leader's plan adds
    std::vector<cavity_plan> drop;
    {
      std::unique_lock<std::mutex> lk(mu);
      int i = -1;
      cv_work.wait(lk, [&] {
        if (stopping && queue.empty()) return true;
        i = pick();
        if (trace && i < 0 && !queue.empty())
          std::fprintf(stderr, "[server] %.3f ms: worker waits, head %lld needs %zu, in use %zu of %zu, "
                       "%zu queued\n", now_ms(), queue[0].ticket,
                       queue[0].plan_bytes + queue[0].field_bytes, in_use, budget, queue.size());
        return i >= 0;
      });
      if (queue.empty()) break;
      grp.push_back(std::move(queue[i]));
      queue.erase(queue.begin() + i);
      const int reuse = idle_plan(grp[0].key);
      size_t total = need_of(grp[0], reuse);
      if (reuse >= 0) {
        resident[reuse].busy = true;
        resident[reuse].last_use = ++clock;
        reused = resident[reuse].plan;
      } else {
        // queued requests on the same aperture without a resident plan join the group
        for (size_t j = 0; j < queue.size() && (int)grp.size() < kMaxGroup;) {
          const Pending& q = queue[j];
          if (q.ap_key == grp[0].ap_key && idle_plan(q.key) < 0) {
            const size_t add = q.plan_bytes + q.field_bytes + grp[0].rhs_bytes;
            if (in_use + total + add <= budget + evictable(-1)) {
              total += add;
              lead_extra += grp[0].rhs_bytes;
              grp.push_back(std::move(queue[j]));
              queue.erase(queue.begin() + j);
              continue;
            }
          }
          ++j;
        }
      }
      drop = evict_for(total, reused);
      in_use += total;
      ++running;
      if (trace)
        std::fprintf(stderr, "[server] %.3f ms: ticket %lld starts (group %zu), in use %zu of %zu, "
                     "%zu queued\n", now_ms(), grp[0].ticket, grp.size(), in_use, budget,
                     queue.size());
    }
    for (cavity_plan q : drop) cavity_plan_destroy(q);
    cv_work.notify_all();
    const int n = (int)grp.size();
    std::vector<cavity_result> res(n);
    std::vector<void*> fields(n, nullptr);
    std::vector<cavity_plan> plans(n, nullptr);
    const double t_start = now_ms();
    int s = have_stream ? CAVITY_OK : CAVITY_EDEVICE;
    for (int r = 0; r < n; ++r) {
      std::memset(&res[r], 0, sizeof(res[r]));
      res[r].t_submit_ms = grp[r].t_submit_ms;
      res[r].t_start_ms = t_start;
      res[r].device_bytes = grp[r].plan_bytes + grp[r].field_bytes + (r == 0 ? lead_extra : 0);
      res[r].plan_reused = reused ? 1 : 0;
      res[r].group_size = n;
      fields[r] = grp[r].req.E_out;
      if (s == CAVITY_OK && !fields[r]) s = cav::device_block_acquire(grp[r].field_bytes, &fields[r]);
    }
    if (s != CAVITY_OK) {
      for (int r = 0; r < n; ++r) res[r].status = s;
    } else if (n == 1) {
      plans[0] = reused;
      run_request(opts, st, grp[0], fields[0], &plans[0], &res[0]);
    } else {
      run_group(opts, st, grp, fields, &plans, &res);
    }
    for (int r = 0; r < n; ++r)
      if (!grp[r].req.E_out && fields[r]) cav::device_block_release(fields[r], grp[r].field_bytes);
    const double t_done = now_ms();
    drop.clear();
    {
      std::lock_guard<std::mutex> lk(mu);
      for (int r = 0; r < n; ++r) {
        const Pending& pd = grp[r];
        cavity_plan plan = plans[r];
        in_use -= pd.field_bytes;
        if (reused) {
          for (Resident& rp : resident)
            if (rp.plan == plan) rp.busy = false;
        } else if (plan && res[r].status == CAVITY_OK && (n == 1 || r > 0) &&
                   pd.plan_bytes <= plan_cache_limit && !has_resident(pd.key)) {
          // keep the plan resident (its bytes stay in in_use); a group leader's plan holds
          // the group's workspace and is not kept
          resident.push_back({pd.key, plan, pd.plan_bytes, ++clock, false});
          resident_bytes += pd.plan_bytes;
          std::vector<cavity_plan> ev = evict_for(0, plan);
          drop.insert(drop.end(), ev.begin(), ev.end());
        } else {
          in_use -= pd.plan_bytes;
          if (plan) drop.push_back(plan);
        }
        res[r].t_done_ms = t_done;
        done[pd.ticket] = Done{res[r]};
      }
      in_use -= lead_extra;
      --running;
    }
    for (cavity_plan q : drop) cavity_plan_destroy(q);
    if (trace)
      std::fprintf(stderr, "[server] %.3f ms: ticket %lld done\n", now_ms(), grp[0].ticket);
    cv_done.notify_all();
    cv_work.notify_all();
  }
  if (st) (void)hipStreamDestroy(st);
}

extern "C" {

int cavity_server_opts_default(cavity_server_opts* o) {
  if (!o) return cav::record_error(CAVITY_EINVAL, "NULL opts");
  o->streams = 4;
  o->hbm_budget = 0;
  o->precision = CAVITY_MIXED;
  o->tol = 1e-12;
  o->plan_cache_bytes = SIZE_MAX;
  return CAVITY_OK;
}

int cavity_server_create(const cavity_server_opts* opts, cavity_server* out) {
  if (!out) return cav::record_error(CAVITY_EINVAL, "NULL server output");
  *out = nullptr;
  cavity_server_opts o;
  cavity_server_opts_default(&o);
  if (opts) o = *opts;
  if (o.streams < 1 || o.streams > 16)
    return cav::record_error(CAVITY_EINVAL, "streams must be in 1..16");
  if (o.precision != CAVITY_FP64 && o.precision != CAVITY_MIXED)
    return cav::record_error(CAVITY_EINVAL, "precision must be CAVITY_FP64 or CAVITY_MIXED");
  if (!(o.tol > 0 && o.tol < 1)) return cav::record_error(CAVITY_EINVAL, "tol in (0,1)");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess)
    return cav::record_error(CAVITY_EDEVICE, "no HIP device");
  size_t budget = o.hbm_budget;
  if (budget == 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess)
      return cav::record_error(CAVITY_EDEVICE, "hipMemGetInfo failed");
    budget = (size_t)(0.8 * (double)fr);
  }
  cavity_server srv = new cavity_server_s();
  srv->opts = o;
  srv->device = dev;
  srv->budget = budget;
  srv->plan_cache_limit = o.plan_cache_bytes == SIZE_MAX ? budget / 4
                                                         : std::min(o.plan_cache_bytes, budget);
  srv->t0 = std::chrono::steady_clock::now();
  if (const char* e = std::getenv("CAVITY_SERVER_TRACE")) srv->trace = std::atoi(e) != 0;
  for (int i = 0; i < o.streams; ++i) srv->workers.emplace_back([srv] { srv->work(); });
  {
    // every worker has its stream before the first request can arrive
    std::unique_lock<std::mutex> lk(srv->mu);
    srv->cv_done.wait(lk, [&] { return srv->ready == o.streams; });
  }
  *out = srv;
  return CAVITY_OK;
}

int cavity_server_submit(cavity_server srv, const cavity_request* r, long long* ticket) {
  if (!srv || !r || !ticket) return cav::record_error(CAVITY_EINVAL, "NULL argument");
  if (r->n_layers < 0 || (r->n_layers > 0 && (!r->layer_nz || !r->eps_r)))
    return cav::record_error(CAVITY_EINVAL, "layer stack needs both arrays");
  if (!(r->theta >= 0.0 && r->theta <= 0.5 * M_PI + 1e-12) || !std::isfinite(r->phi) ||
      (r->pol != CAVITY_TM && r->pol != CAVITY_TE))
    return cav::record_error(CAVITY_EINVAL, "theta in [0, pi/2], finite phi, pol TM or TE");
  if (!cav::aligned16(r->E_out))
    return cav::record_error(CAVITY_EINVAL, "E_out must be 16-byte aligned");
  Pending pd;
  pd.req = *r;
  pd.lnz.assign(r->layer_nz, r->layer_nz + r->n_layers);
  pd.eps.assign(r->eps_r, r->eps_r + r->n_layers);
  pd.req.layer_nz = nullptr;
  pd.req.eps_r = nullptr;
  cavity_opts o;
  cavity_opts_default(&o);
  o.precision = srv->opts.precision;
  o.tol = srv->opts.tol;
  o.batch = 1;
  cavity_eps e{};
  fill_eps(pd, &e);
  size_t plan_bytes = 0;
  const int s = cavity_plan_footprint(r->a, r->b, r->c, r->Nx, r->Ny, r->Nz,
                                      pd.lnz.empty() ? nullptr : &e, r->k, &o, &plan_bytes);
  if (s) return s;
  pd.field_bytes = r->E_out ? 0 : field_bytes_of(*r);
  pd.plan_bytes = plan_bytes;
  pd.key = cavity_key(*r, pd.lnz, pd.eps);
  pd.ap_key = aperture_key(*r);
  pd.rhs_bytes = 0;
  if (cav::footprint_per_rhs(r->a, r->b, r->c, r->Nx, r->Ny, r->Nz, pd.lnz.empty() ? nullptr : &e,
                             r->k, &o, &pd.rhs_bytes) != CAVITY_OK)
    return cav::record_error(CAVITY_EINVAL, "request arguments");
  const size_t footprint = plan_bytes + pd.field_bytes;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stopping) return cav::record_error(CAVITY_EINVAL, "server is shutting down");
    pd.ticket = srv->next_ticket++;
    pd.t_submit_ms = srv->now_ms();
    *ticket = pd.ticket;
    srv->live.insert(pd.ticket);
    if (footprint > srv->budget) {
      Done d;
      std::memset(&d.res, 0, sizeof(d.res));
      d.res.status = CAVITY_ENOMEM;
      d.res.device_bytes = footprint;
      d.res.t_submit_ms = d.res.t_start_ms = d.res.t_done_ms = pd.t_submit_ms;
      srv->done[pd.ticket] = d;
    } else {
      srv->queue.push_back(std::move(pd));
    }
  }
  srv->cv_work.notify_all();
  srv->cv_done.notify_all();
  return CAVITY_OK;
}

int cavity_server_wait(cavity_server srv, long long ticket, cavity_result* out) {
  if (!srv || !out) return cav::record_error(CAVITY_EINVAL, "NULL argument");
  std::unique_lock<std::mutex> lk(srv->mu);
  if (!srv->live.count(ticket)) return cav::record_error(CAVITY_EINVAL, "unknown ticket");
  srv->cv_done.wait(lk, [&] { return srv->done.count(ticket) > 0; });
  *out = srv->done[ticket].res;
  return CAVITY_OK;
}

int cavity_server_release(cavity_server srv, long long ticket) {
  if (!srv) return cav::record_error(CAVITY_EINVAL, "NULL server");
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->done.find(ticket);
  if (it == srv->done.end()) return cav::record_error(CAVITY_EINVAL, "no completed request");
  srv->done.erase(it);
  srv->live.erase(ticket);
  return CAVITY_OK;
}

double cavity_server_now_ms(cavity_server srv) { return srv ? srv->now_ms() : 0.0; }

void cavity_server_destroy(cavity_server srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stopping = true;
  }
  srv->cv_work.notify_all();
  for (std::thread& t : srv->workers) t.join();
  for (Resident& rp : srv->resident) cavity_plan_destroy(rp.plan);
  delete srv;
}

}  // extern "C"
