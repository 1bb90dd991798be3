// Request server: many cavities, each solved for one incidence, with several requests in
// flight on the GPU at once.  Worker threads each own a HIP stream; a request is admitted
// in arrival order when a worker is free and its device footprint fits in the budget left
// by the requests already running.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <condition_variable>
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

struct Pending {
  long long ticket;
  cavity_request req;
  std::vector<int> lnz;
  std::vector<cavity_c128> eps;
  size_t footprint;       // plan + workspace + solution (+ field when the server holds it)
  size_t field_bytes;     // temporary field buffer, 0 when the caller gave E_out
  double t_submit_ms;
};

struct Done {
  cavity_result res;
};

}  // namespace

struct cavity_server_s {
  cavity_server_opts opts{};
  int device = 0;
  size_t budget = 0;
  size_t in_use = 0;
  std::chrono::steady_clock::time_point t0;
  std::vector<std::thread> workers;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Pending> queue;
  std::map<long long, Done> done;
  std::set<long long> live;     // submitted and not yet released
  long long next_ticket = 1;
  int running = 0;
  bool stopping = false;

  double now_ms() const {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
        .count();
  }
  // The head of the queue may start (caller holds mu).
  bool head_fits() const {
    return !queue.empty() && in_use + queue.front().footprint <= budget;
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

// One request on stream st: plan, solve into the field buffer, backscatter RCS.
void run_request(const cavity_server_opts& so, hipStream_t st, const Pending& pd, void* field,
                 cavity_result* res) {
  cavity_opts o;
  cavity_opts_default(&o);
  o.precision = so.precision;
  o.tol = so.tol;
  o.batch = 1;
  o.stream = st;
  o.hbm_budget = pd.footprint + ((size_t)64 << 20);
  cavity_eps e{};
  fill_eps(pd, &e);
  const cavity_request& r = pd.req;
  cavity_plan plan = nullptr;
  int s = cavity_plan_create(r.a, r.b, r.c, r.Nx, r.Ny, r.Nz, pd.lnz.empty() ? nullptr : &e,
                             r.k, &o, &plan);
  if (s == CAVITY_OK) {
    s = cavity_solve(plan, r.theta, r.phi, r.pol, static_cast<cavity_c128*>(field));
    if (s == CAVITY_OK || s == CAVITY_ENOCONV) {
      const int s2 = cavity_rcs(plan, 0, 1, &r.theta, &r.phi, res->sigma);
      if (s == CAVITY_OK) s = s2;
      cavity_info inf{};
      if (cavity_plan_info(plan, &inf) == CAVITY_OK) {
        res->iterations = inf.last_iterations;
        res->rel_residual = inf.last_rel_residual;
        res->unknowns = inf.unknowns;
      }
    }
  }
  if (plan) cavity_plan_destroy(plan);
  if (hipStreamSynchronize(st) != hipSuccess && s == CAVITY_OK) s = CAVITY_EDEVICE;
  res->status = s;
}

}  // namespace

void cavity_server_s::work() {
  (void)hipSetDevice(device);
  hipStream_t st = nullptr;
  const bool have_stream = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
  while (true) {
    Pending pd;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_work.wait(lk, [&] { return (stopping && queue.empty()) || head_fits(); });
      if (queue.empty()) break;
      pd = std::move(queue.front());
      queue.pop_front();
      in_use += pd.footprint;
      ++running;
    }
    cv_work.notify_all();
    Done d;
    std::memset(&d.res, 0, sizeof(d.res));
    d.res.t_submit_ms = pd.t_submit_ms;
    d.res.t_start_ms = now_ms();
    d.res.device_bytes = pd.footprint;
    void* field = pd.req.E_out;
    int s = have_stream ? CAVITY_OK : CAVITY_EDEVICE;
    if (s == CAVITY_OK && !field) s = cav::device_block_acquire(pd.field_bytes, &field);
    if (s == CAVITY_OK) {
      run_request(opts, st, pd, field, &d.res);
    } else {
      d.res.status = s;
    }
    if (!pd.req.E_out && field) cav::device_block_release(field, pd.field_bytes);
    d.res.t_done_ms = now_ms();
    {
      std::lock_guard<std::mutex> lk(mu);
      in_use -= pd.footprint;
      --running;
      done[pd.ticket] = d;
    }
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
  srv->t0 = std::chrono::steady_clock::now();
  for (int i = 0; i < o.streams; ++i) srv->workers.emplace_back([srv] { srv->work(); });
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
  pd.footprint = plan_bytes + pd.field_bytes;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stopping) return cav::record_error(CAVITY_EINVAL, "server is shutting down");
    pd.ticket = srv->next_ticket++;
    pd.t_submit_ms = srv->now_ms();
    *ticket = pd.ticket;
    srv->live.insert(pd.ticket);
    if (pd.footprint > srv->budget) {
      Done d;
      std::memset(&d.res, 0, sizeof(d.res));
      d.res.status = CAVITY_ENOMEM;
      d.res.device_bytes = pd.footprint;
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
  delete srv;
}

}  // extern "C"
