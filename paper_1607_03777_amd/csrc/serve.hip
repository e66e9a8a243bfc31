// Request server: continuous admission of viscous and Stokes solves of
// different sizes and orders onto one GPU.
//
// Requests enter a FIFO queue with host copies of their inputs.  Worker
// threads (the slots), each with its own HIP stream, take the oldest request
// whose device memory (the problem's bytes with its element blocks counted
// from its viscosity, plus its input and output arrays) fits into what the budget has left, together with queued requests
// of the identical shape (mesh, options, kind, Dirichlet data present), up to
// max_batch of them, which then run as one batched problem.  A request that
// does not fit may be overtaken by later ones that do, at most `bypass`
// times; after that admission waits for it.  The solver state of a request
// (blocks, hierarchy, Krylov vectors) stays on the device from setup to the
// copy of its result; requests on different slots overlap on the device.
// With combine set, the CG iterations of all slots are launched together
// (the context's combiner): a request admitted into a free slot joins the
// running launches at its first iteration boundary, whatever its shape.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/sdg.h"
#include "admission.h"
#include "runtime.h"

namespace {

double wall_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

bool same_options(const sdg_options& a, const sdg_options& b) {
  return a.rtol == b.rtol && a.inner_rtol == b.inner_rtol && a.max_it == b.max_it &&
         a.inner_max_it == b.inner_max_it && a.restart == b.restart && a.smooth_dg == b.smooth_dg &&
         a.smooth_h == b.smooth_h && a.coarsest_n == b.coarsest_n && a.eig_steps == b.eig_steps &&
         a.cheb_lo == b.cheb_lo && a.cheb_hi == b.cheb_hi && a.prec_smoother == b.prec_smoother &&
         a.prec_apply == b.prec_apply && a.viscous_krylov == b.viscous_krylov && a.dedup == b.dedup &&
         a.seed == b.seed && a.refine == b.refine && a.outer_krylov == b.outer_krylov;
}

bool same_shape(const sdg_mesh& a, const sdg_mesh& b) {
  return a.nx == b.nx && a.ny == b.ny && a.k == b.k && a.lx == b.lx && a.ly == b.ly &&
         std::memcmp(a.bc, b.bc, sizeof(a.bc)) == 0;
}

}  // namespace

struct sdg_req {
  sdg_mesh mesh{};
  sdg_options opts{};
  int kind = 0;
  bool has_g = false;
  std::vector<double> eta, f, g, u, p;
  sdg_stats st{};
  int rc = 0;
  std::string err;  // message of a failed solve (set on the worker thread)
  int64_t nuniq = 0;  // distinct element blocks of this request after deduplication
  size_t bytes = 0;   // admission estimate for this request alone
  double t_submit = 0, t_start = 0, t_end = 0;
  int batch = 0;  // number of requests in the launch group it ran in
  bool done = false;
  bool user_freed = false;
  std::mutex mu;
  std::condition_variable cv;
};

struct sdg_server {
  sdg_ctx* ctx = nullptr;
  int device = 0;
  int slots = 1, max_batch = 1, bypass = 8;
  bool combine = false;  // CG iterations of the slots combined per launch
  size_t budget = 0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<sdg_req*> queue;
  sdg::Admission adm;
  bool stop = false;
  std::vector<std::thread> workers;
  int64_t completed = 0;
  size_t peak_bytes = 0;
  int peak_busy = 0;
};

namespace {

int64_t n_el(const sdg_mesh& m) { return (int64_t)m.nx * m.ny; }
int64_t n_u(const sdg_mesh& m) { return n_el(m) * 2 * (m.k + 1) * (m.k + 1); }
int64_t n_p(const sdg_mesh& m) { return n_el(m) * m.k * m.k; }
int64_t n_g(const sdg_mesh& m) { return (int64_t)(2 * m.nx + 2 * m.ny) * 2 * (m.k + 1); }

size_t io_bytes(const sdg_req& r, int nb) {
  return (size_t)nb * 8 *
         (n_el(r.mesh) + 2 * n_u(r.mesh) + (r.kind ? n_p(r.mesh) : 0) + (r.has_g ? n_g(r.mesh) : 0));
}

// Device bytes of a launch group of nb requests shaped like r whose
// distinct element blocks number nuniq in all (the sum over the requests:
// blocks shared across requests only lower it).
size_t group_bytes(const sdg_req& r, int nb, int64_t nuniq) {
  return sdg::required_bytes_blocks(&r.mesh, &r.opts, r.kind, nb, nuniq) + io_bytes(r, nb);
}

// Publishes a request's outcome.  The waiter is notified while the lock is
// held: once it is released the client may free the request at any time
// (sdg_wait then sdg_req_free), so after the unlock the worker touches the
// request only to delete it, and only when the client freed it before.
void finish(sdg_req* r, int rc, const sdg_stats* st, double t_end, int batch, const std::string& err) {
  bool del;
  {
    std::lock_guard<std::mutex> g(r->mu);
    r->rc = rc;
    r->err = err;
    if (st) r->st = *st;
    r->t_end = t_end;
    r->batch = batch;
    r->done = true;
    del = r->user_freed;
    r->cv.notify_all();
  }
  if (del) delete r;
}

// Runs one launch group (requests of one shape) as a batched problem on
// stream s.  Returns the group's rc; per-request results are stored.
void run_group(sdg_server* S, const std::vector<sdg_req*>& grp, hipStream_t s) {
  const sdg_req& r0 = *grp[0];
  const int nb = (int)grp.size();
  const int64_t ne = n_el(r0.mesh), nu = n_u(r0.mesh), np = n_p(r0.mesh), ng = n_g(r0.mesh);
  double *de = nullptr, *df = nullptr, *dg = nullptr, *du = nullptr, *dp = nullptr;
  int rc = SDG_OK;
  // staging arrays from the context's block cache (a group of the same
  // shape as an earlier one reuses its blocks)
  auto bytes_of = [](int64_t n) { return (size_t)std::max<int64_t>(n, 1) * sizeof(double); };
  auto al = [&](double** q, int64_t n) {
    if (rc < 0) return;
    *q = (double*)sdg::ctx_alloc(S->ctx, bytes_of(n));
    if (!*q) rc = SDG_ERR_NOMEM;
  };
  al(&de, nb * ne);
  al(&df, nb * nu);
  al(&du, nb * nu);
  if (r0.kind) al(&dp, nb * np);
  if (r0.has_g) al(&dg, nb * ng);
  for (int i = 0; i < nb && rc >= 0; ++i) {
    const sdg_req& r = *grp[i];
    if (hipMemcpyAsync(de + i * ne, r.eta.data(), ne * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(df + i * nu, r.f.data(), nu * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
        (r0.has_g && hipMemcpyAsync(dg + i * ng, r.g.data(), ng * 8, hipMemcpyHostToDevice, s) != hipSuccess))
      rc = SDG_ERR_DEVICE;
  }
  std::vector<sdg_stats> st(nb);
  sdg_problem* P = nullptr;
  if (rc >= 0) rc = sdg_problem_create_batch(S->ctx, &r0.mesh, &r0.opts, nb, de, s, &P);
  if (rc >= 0)
    rc = r0.kind ? sdg_solve_stokes_dev(P, df, dg, du, dp, st.data()) : sdg_solve_viscous_dev(P, df, dg, du, st.data());
  if (rc >= 0) {
    for (int i = 0; i < nb && rc >= 0; ++i) {
      sdg_req& r = *grp[i];
      r.u.resize(nu);
      if (r0.kind) r.p.resize(np);
      if (hipMemcpyAsync(r.u.data(), du + i * nu, nu * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
          (r0.kind && np > 0 &&
           hipMemcpyAsync(r.p.data(), dp + i * np, np * 8, hipMemcpyDeviceToHost, s) != hipSuccess))
        rc = SDG_ERR_DEVICE;
    }
    if (hipStreamSynchronize(s) != hipSuccess) rc = SDG_ERR_DEVICE;
  }
  sdg_problem_destroy(P);
  // no queued work uses the staging arrays any more: drain the stream (the
  // solve may have stopped on an error with work still queued)
  (void)hipStreamSynchronize(s);
  const int64_t ns[5] = {nb * ne, nb * nu, nb * ng, nb * nu, nb * np};
  double* qs[5] = {de, df, dg, du, dp};
  for (int i = 0; i < 5; ++i)
    if (qs[i]) sdg::ctx_release(S->ctx, qs[i], bytes_of(ns[i]));
  const double t = wall_ms();
  const std::string err = rc < 0 ? std::string(sdg_last_error()) : std::string();
  for (int i = 0; i < nb; ++i) {
    // a solve's soft outcome is per problem; errors apply to the whole group
    const int ri = rc < 0 ? rc : st[i].status;
    finish(grp[i], ri, rc < 0 ? nullptr : &st[i], t, nb, err);
  }
}

void worker(sdg_server* S) {
  if (hipSetDevice(S->device) != hipSuccess) return;
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return;
  while (true) {
    std::vector<sdg_req*> grp;
    size_t bytes = 0;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      int pick = -1;
      S->cv.wait(lk, [&] {
        if (S->queue.empty()) return S->stop;
        std::vector<size_t> need(S->queue.size());
        for (size_t i = 0; i < need.size(); ++i) need[i] = S->queue[i]->bytes;
        pick = S->adm.pick(need);
        return pick >= 0;
      });
      if (pick < 0) break;  // stopping and drained
      sdg_req* r = S->queue[pick];
      grp.push_back(r);
      S->queue.erase(S->queue.begin() + pick);
      bytes = r->bytes;
      int64_t nuniq = r->nuniq;
      // same-shape requests behind it join the launch group while they fit
      for (size_t i = 0; i < S->queue.size() && (int)grp.size() < S->max_batch;) {
        sdg_req* q = S->queue[i];
        const size_t nb2 = group_bytes(*r, (int)grp.size() + 1, nuniq + q->nuniq);
        if (q->kind == r->kind && q->has_g == r->has_g && same_shape(q->mesh, r->mesh) &&
            same_options(q->opts, r->opts) && S->adm.fits(nb2)) {
          grp.push_back(q);
          bytes = nb2;
          nuniq += q->nuniq;
          S->queue.erase(S->queue.begin() + i);
        } else {
          ++i;
        }
      }
      S->adm.start(bytes);
      S->peak_bytes = std::max(S->peak_bytes, S->adm.in_use());
      S->peak_busy = std::max(S->peak_busy, S->adm.busy());
    }
    const double t0 = wall_ms();
    for (sdg_req* r : grp) r->t_start = t0;
    run_group(S, grp, s);
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->adm.end(bytes);
      S->completed += (int64_t)grp.size();
    }
    S->cv.notify_all();
  }
  (void)hipStreamDestroy(s);
}

}  // namespace

extern "C" {

int sdg_server_create(sdg_ctx* ctx, const sdg_server_config* cfg, sdg_server** out) {
  if (!out || !ctx) {
    sdg::set_error("NULL context or output pointer");
    return SDG_ERR_INVALID;
  }
  *out = nullptr;
  sdg_server_config c{};
  if (cfg) c = *cfg;
  if (c.slots < 1 || c.slots > 64 || c.max_batch < 1 || c.max_batch > 4096 || c.bypass < 0 || c.combine < 0 ||
      c.combine > 1) {
    sdg_server_config d;
    sdg_server_config_default(&d);
    if (!cfg) c = d;
    else {
      sdg::set_error("server config out of range (slots 1..64, max_batch 1..4096, bypass >= 0, combine 0..1)");
      return SDG_ERR_INVALID;
    }
  }
  const int dev = sdg::ctx_device(ctx);
  if (hipSetDevice(dev) != hipSuccess) {
    (void)hipGetLastError();
    sdg::set_error("hipSetDevice failed");
    return SDG_ERR_DEVICE;
  }
  size_t budget = c.mem_budget;
  if (budget == 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
      (void)hipGetLastError();
      sdg::set_error("hipMemGetInfo failed");
      return SDG_ERR_DEVICE;
    }
    budget = fr / 10 * 9;
  }
  sdg_server* S = new sdg_server();
  S->ctx = ctx;
  S->device = dev;
  S->slots = c.slots;
  S->max_batch = c.max_batch;
  S->bypass = c.bypass;
  S->budget = budget;
  S->adm = sdg::Admission(budget, c.slots, c.bypass);
  S->combine = c.combine != 0;
  if (S->combine) sdg::ctx_combine(ctx, 1);
  for (int i = 0; i < c.slots; ++i) S->workers.emplace_back(worker, S);
  *out = S;
  return SDG_OK;
}

void sdg_server_config_default(sdg_server_config* c) {
  if (!c) return;
  std::memset(c, 0, sizeof(*c));
  c->slots = 4;
  c->max_batch = 16;
  c->bypass = 8;
  c->mem_budget = 0;
}

void sdg_server_destroy(sdg_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv.notify_all();
  for (auto& t : S->workers) t.join();
  if (S->combine) sdg::ctx_combine(S->ctx, 0);
  delete S;
}

int sdg_server_launch_stats(sdg_server* S, int64_t* launches, int64_t* combined, int* max_width, int64_t* graphs) {
  if (!S) {
    sdg::set_error("NULL server");
    return SDG_ERR_INVALID;
  }
  if (launches) *launches = 0;
  if (combined) *combined = 0;
  if (max_width) *max_width = 0;
  if (graphs) *graphs = 0;
  sdg::ctx_combine_stats(S->ctx, launches, combined, max_width, graphs);
  return SDG_OK;
}

int sdg_submit(sdg_server* S, const sdg_mesh* mesh, const sdg_options* opts, int kind, const double* eta,
               const double* f, const double* g, sdg_req** out) {
  if (!S || !mesh || !eta || !f || !out || (kind != SDG_VISCOUS && kind != SDG_STOKES)) {
    sdg::set_error("invalid argument");
    return SDG_ERR_INVALID;
  }
  *out = nullptr;
  sdg_req* r = new sdg_req();
  r->mesh = *mesh;
  if (opts) r->opts = *opts;
  else sdg_options_default(&r->opts);
  r->kind = kind;
  r->has_g = g != nullptr;
  const size_t b1 = sdg_required_bytes_batch(mesh, &r->opts, kind, 1);
  if (b1 == 0) {
    delete r;
    sdg::set_error("invalid mesh or options");
    return SDG_ERR_INVALID;
  }
  r->eta.assign(eta, eta + n_el(*mesh));
  r->f.assign(f, f + n_u(*mesh));
  if (g) r->g.assign(g, g + n_g(*mesh));
  r->nuniq = sdg::unique_blocks(*mesh, r->eta.data(), 1, r->opts.dedup != 0);
  r->bytes = group_bytes(*r, 1, r->nuniq);
  if (r->bytes > S->budget) {
    delete r;
    sdg::set_error("request needs more device memory than the server's budget");
    return SDG_ERR_NOMEM;
  }
  r->t_submit = wall_ms();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) {
      delete r;
      sdg::set_error("server is shutting down");
      return SDG_ERR_INVALID;
    }
    S->queue.push_back(r);
  }
  S->cv.notify_all();
  *out = r;
  return SDG_OK;
}

int sdg_poll(sdg_req* r, int* done) {
  if (!r || !done) {
    sdg::set_error("NULL argument");
    return SDG_ERR_INVALID;
  }
  std::lock_guard<std::mutex> g(r->mu);
  *done = r->done ? 1 : 0;
  return SDG_OK;
}

int sdg_wait(sdg_req* r, double* u, double* p, sdg_stats* st, sdg_req_info* info) {
  if (!r) {
    sdg::set_error("NULL request");
    return SDG_ERR_INVALID;
  }
  std::unique_lock<std::mutex> lk(r->mu);
  r->cv.wait(lk, [&] { return r->done; });
  if (r->rc >= 0) {
    if (u) std::copy(r->u.begin(), r->u.end(), u);
    if (p && r->kind) std::copy(r->p.begin(), r->p.end(), p);
  }
  if (st) *st = r->st;
  if (r->rc < 0) sdg::set_error(r->err.empty() ? std::string("request failed") : r->err);
  if (info) {
    info->submit_ms = r->t_submit;
    info->start_ms = r->t_start;
    info->end_ms = r->t_end;
    info->batch = r->batch;
    info->bytes = r->bytes;
  }
  return r->rc;
}

void sdg_req_free(sdg_req* r) {
  if (!r) return;
  bool del;
  {
    std::lock_guard<std::mutex> g(r->mu);
    r->user_freed = true;
    del = r->done;
  }
  if (del) delete r;  // else the worker deletes it when the solve ends
}

int sdg_server_stats(sdg_server* S, int64_t* completed, size_t* peak_bytes, int* peak_busy, size_t* budget) {
  if (!S) {
    sdg::set_error("NULL server");
    return SDG_ERR_INVALID;
  }
  std::lock_guard<std::mutex> lk(S->mu);
  if (completed) *completed = S->completed;
  if (peak_bytes) *peak_bytes = S->peak_bytes;
  if (peak_busy) *peak_busy = S->peak_busy;
  if (budget) *budget = S->budget;
  return SDG_OK;
}

int sdg_admission_simulate(int n, const double* arrival_ms, const double* service_ms, const size_t* bytes,
                           int slots, size_t budget, int bypass, double* start_ms) {
  if (n < 0 || (n > 0 && (!arrival_ms || !service_ms || !bytes || !start_ms)) || slots < 1 || bypass < 0) {
    sdg::set_error("invalid argument");
    return SDG_ERR_INVALID;
  }
  for (int i = 0; i < n; ++i)
    if (bytes[i] > budget) {
      sdg::set_error("a request needs more than the budget");
      return SDG_ERR_NOMEM;
    }
  return sdg::simulate_admission(n, arrival_ms, service_ms, bytes, slots, budget, bypass, start_ms);
}

}  // extern "C"
