// Serving runtime: requests to solve A x = b (FP64 right-hand sides, iterative
// refinement to a relative residual, the ACR factor of A as preconditioner)
// over a set of registered operators.  Factorisations stay resident in device
// memory under a byte budget; a request whose operator is not resident waits
// until its factor fits (least recently used idle factors are evicted) and
// is then factored together with every other operator admitted at the same
// moment (one batched factorisation).  Active requests advance together, one
// refinement step at a time: the residuals, norms, corrections M^{-1} r and
// updates of all of them are grouped launches, and requests that arrive
// while others run join at the next step (continuous batching).  A request's
// arithmetic never depends on the others (every grouped kernel computes a
// job exactly as it would alone), so its result is the same alone and in any
// mix.  One worker thread and one stream per server.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "factor.hpp"

namespace acr {

using Clock = std::chrono::steady_clock;

namespace {

struct OpEntry {
  acr_operator op{};            // arrays point into `arrays`
  DBuf<double> arrays;          // 5 N values: diag, west, east, south, north
  acr_options opt{};
  std::unique_ptr<FactorBase> factor;
  size_t bytes = 0;             // device bytes of the resident factor
  size_t est = 0;               // expected bytes (measured after the first factorisation)
  long long last_use = 0;
  int users = 0;                // active requests on this operator
  long long factorizations = 0;
};

struct Request {
  long long id = 0;
  int op = 0;
  const double* B = nullptr;
  double* X = nullptr;
  int nrhs = 0;
  hipEvent_t ready = nullptr;   // recorded on the submitter's stream
  Clock::time_point t0;
  DBuf<double> R, D, nrm;
  std::vector<double> hb;       // ||b_q||^2
  int iters = 0;
  double relres = INFINITY;
  bool active = false, done = false;
  acr_status status = ACR_OK;
  std::string err;
  double latency_ms = 0.0;
};

}  // namespace
}  // namespace acr

struct acr_server_s {
  acr_server_config cfg{};
  int device = 0;
  hipStream_t st = nullptr;
  std::thread worker;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stop = false;
  std::vector<std::unique_ptr<acr::OpEntry>> ops;
  std::deque<std::shared_ptr<acr::Request>> incoming;
  std::map<long long, std::shared_ptr<acr::Request>> reqs;
  long long next_id = 1;
  // worker-side state
  std::vector<std::shared_ptr<acr::Request>> pending, active;
  long long tick = 0;
  // statistics (under mu)
  std::vector<double> lat;
  long long rhs_done = 0, req_done = 0, evictions = 0, factorizations = 0, steps = 0;
  double busy_s = 0.0;
  acr::Clock::time_point t_first{}, t_last{};
  bool any = false;
  size_t resident = 0, peak_resident = 0;
};

namespace acr {
namespace {

size_t estimate_bytes(const acr_operator& op, const acr_options& opt) {
  // about three HODLR blocks per block row (X, E, F), leaves + U, V at rank ~8
  const int L = std::max(hodlr_depth(op.nx, opt.leaf), 0);
  const double b = (double)(op.nx >> L);
  const double per = (double)op.nx * (b + 2.0 * 8.0 * L);
  const double elem = opt.precision == ACR_FP64 ? 8.0 : 4.0;
  return (size_t)(3.0 * op.ny * per * elem);
}

template <typename T>
void solve_chunks(acr_server_s* S, const std::vector<Request*>& rs, hipStream_t st) {
  // corrections D = M^{-1} R in chunks of <= 8 columns (the fused solve path)
  std::vector<const Factor<T>*> fs;
  std::vector<const double*> bs;
  std::vector<double*> xs;
  std::vector<int> nr;
  for (Request* r : rs) {
    OpEntry& E = *S->ops[r->op];
    auto* f = static_cast<Factor<T>*>(E.factor.get());
    const size_t n = (size_t)E.op.nx * E.op.ny;
    if (!f->fused_ok(1)) {
      f->solve_gemm(r->R.get(), r->D.get(), r->nrhs, st);
      continue;
    }
    for (int q0 = 0; q0 < r->nrhs; q0 += 8) {
      fs.push_back(f);
      bs.push_back(r->R.get() + q0 * n);
      xs.push_back(r->D.get() + q0 * n);
      nr.push_back(std::min(8, r->nrhs - q0));
    }
  }
  if (!fs.empty()) solve_fused_many<T>(fs, bs, xs, nr, st);
}

void finish(acr_server_s* S, Request* r, acr_status status, const std::string& err) {
  const auto t = Clock::now();
  std::lock_guard<std::mutex> g(S->mu);
  r->status = status;
  r->err = err;
  r->done = true;
  r->latency_ms = std::chrono::duration<double, std::milli>(t - r->t0).count();
  if (status == ACR_OK || status == ACR_ERR_NOT_CONVERGED) {
    S->lat.push_back(r->latency_ms);
    S->rhs_done += r->nrhs;
    ++S->req_done;
    S->t_last = t;
  }
  S->cv_done.notify_all();
}

// Admit pending requests whose factor is (or can be made) resident.  Order of
// the operators to factor: those whose oldest request has waited longer than
// kStarveMs first (oldest first), then by the number of requests waiting for
// them.  A resident factor that pending requests wait for is evicted only to
// make room for a starving operator, so factors are reused by the requests
// they were made for instead of being recomputed.
constexpr double kStarveMs = 250.0;

void admit(acr_server_s* S) {
  hipStream_t st = S->st;
  const auto now = Clock::now();
  struct Need {
    int op;
    int count = 0;
    double wait_ms = 0.0;
  };
  std::vector<Need> need;
  std::vector<int> wanted(S->ops.size(), 0);
  for (auto& r : S->pending) {
    ++wanted[r->op];
    OpEntry& E = *S->ops[r->op];
    if (E.factor) continue;
    const double w = std::chrono::duration<double, std::milli>(now - r->t0).count();
    auto it = std::find_if(need.begin(), need.end(), [&](const Need& n) { return n.op == r->op; });
    if (it == need.end()) {
      need.push_back(Need{r->op, 1, w});
    } else {
      ++it->count;
      it->wait_ms = std::max(it->wait_ms, w);
    }
  }
  std::stable_sort(need.begin(), need.end(), [](const Need& a, const Need& b) {
    const bool sa = a.wait_ms > kStarveMs, sb = b.wait_ms > kStarveMs;
    if (sa != sb) return sa;
    if (sa) return a.wait_ms > b.wait_ms;
    return a.count > b.count;
  });
  std::vector<int> go;     // operators that fit now
  size_t planned = 0;
  const size_t budget = (size_t)S->cfg.memory_budget;
  for (const Need& nd : need) {
    OpEntry& E = *S->ops[nd.op];
    const size_t want = E.est;
    const bool starving = nd.wait_ms > kStarveMs;
    while (S->resident + planned + want > budget) {
      // least recently used idle factor; one that requests wait for only for a
      // starving operator.  Its memory goes back to this thread's pool for this
      // stream, so later work reuses it in stream order after the steps that read it.
      int victim = -1;
      for (size_t i = 0; i < S->ops.size(); ++i) {
        OpEntry& V = *S->ops[i];
        if (!V.factor || V.users > 0 || (wanted[i] && !starving)) continue;
        if (victim < 0 || V.last_use < S->ops[victim]->last_use) victim = (int)i;
      }
      if (victim < 0) break;
      OpEntry& V = *S->ops[victim];
      S->resident -= V.bytes;
      V.factor.reset();
      V.bytes = 0;
      std::lock_guard<std::mutex> g(S->mu);
      ++S->evictions;
    }
    if (S->resident + planned + want > budget && !(S->resident == 0 && planned == 0)) continue;
    go.push_back(nd.op);
    planned += want;
  }
  // one batched factorisation per distinct option set
  while (!go.empty()) {
    const acr_options o0 = S->ops[go[0]]->opt;
    std::vector<int> grp, rest;
    for (int o : go) {
      const acr_options& x = S->ops[o]->opt;
      const bool same = x.leaf == o0.leaf && x.eps == o0.eps && x.precision == o0.precision &&
                        x.max_rank == o0.max_rank && x.inner_eps == o0.inner_eps &&
                        x.stop_blocks == o0.stop_blocks;
      (same ? grp : rest).push_back(o);
    }
    std::vector<acr_operator> v;
    for (int o : grp) v.push_back(S->ops[o]->op);
    std::vector<std::unique_ptr<FactorBase>> fs;
    if (o0.precision == ACR_FP64) {
      auto f = factor_many<double>(v, o0, st);
      for (auto& x : f) fs.push_back(std::move(x));
    } else {
      auto f = factor_many<float>(v, o0, st);
      for (auto& x : f) fs.push_back(std::move(x));
    }
    for (size_t i = 0; i < grp.size(); ++i) {
      OpEntry& E = *S->ops[grp[i]];
      acr_info inf;
      fs[i]->info(&inf);
      E.factor = std::move(fs[i]);
      E.bytes = (size_t)inf.factor_bytes;
      E.est = E.bytes;
      ++E.factorizations;
      S->resident += E.bytes;
      S->peak_resident = std::max(S->peak_resident, S->resident);
      std::lock_guard<std::mutex> g(S->mu);
      ++S->factorizations;
    }
    go.swap(rest);
  }
  // activate the requests whose factor is resident, in arrival order
  std::vector<std::shared_ptr<Request>> still;
  for (auto& r : S->pending) {
    OpEntry& E = *S->ops[r->op];
    if (!E.factor) {
      still.push_back(r);
      continue;
    }
    const size_t n = (size_t)E.op.nx * E.op.ny;
    if (r->ready) ACR_HIP(hipStreamWaitEvent(st, r->ready, 0));
    r->R.resize(n * r->nrhs);
    r->D.resize(n * r->nrhs);
    r->nrm.resize(r->nrhs);
    memset_async(r->X, 0, n * r->nrhs * sizeof(double), st);
    copy_d2d_async(r->R.get(), r->B, n * r->nrhs * sizeof(double), st);
    r->active = true;
    ++E.users;
    S->active.push_back(r);
  }
  S->pending.swap(still);
}

// One refinement step of every active request.
void step(acr_server_s* S) {
  hipStream_t st = S->st;
  const double tol = S->cfg.tol;
  const int maxit = S->cfg.maxit;
  std::vector<RJob> res, nrm;
  for (auto& r : S->active) {
    OpEntry& E = *S->ops[r->op];
    RJob J;
    J.nx = E.op.nx; J.ny = E.op.ny; J.nrhs = r->nrhs;
    J.diag = E.op.diag; J.west = E.op.west; J.east = E.op.east; J.south = E.op.south; J.north = E.op.north;
    J.X = r->X; J.B = r->B; J.R = r->R.get(); J.out = r->nrm.get();
    if (r->iters > 0) res.push_back(J);   // the first residual is B itself
    nrm.push_back(J);
  }
  gresidual(st, res);
  gcol_sumsq(st, nrm);
  size_t tot = 0;
  for (auto& r : S->active) tot += r->nrhs;
  std::vector<double> hr(tot);
  {
    std::vector<HostCopy> cs;
    size_t o = 0;
    for (auto& r : S->active) {
      cs.push_back(HostCopy{hr.data() + o, r->nrm.get(), r->nrhs * sizeof(double)});
      o += r->nrhs;
    }
    read_many_to_host(cs, st);
  }
  std::vector<Request*> go32, go64;
  std::vector<std::shared_ptr<Request>> keep;
  size_t o = 0;
  ++S->tick;
  for (auto& r : S->active) {
    OpEntry& E = *S->ops[r->op];
    E.last_use = S->tick;
    if (r->iters == 0) r->hb.assign(hr.begin() + o, hr.begin() + o + r->nrhs);
    double rel = 0.0;
    for (int q = 0; q < r->nrhs; ++q) {
      const double v = r->hb[q] > 0 ? std::sqrt(hr[o + q] / r->hb[q]) : std::sqrt(hr[o + q]);
      rel = nan_max(rel, v);
    }
    o += r->nrhs;
    r->relres = rel;
    if (!(rel > tol) || r->iters >= maxit || !std::isfinite(rel)) {
      --E.users;
      r->R.reset();
      r->D.reset();
      r->nrm.reset();
      r->active = false;
      finish(S, r.get(), rel <= tol ? ACR_OK : ACR_ERR_NOT_CONVERGED,
             rel <= tol ? std::string() : "refinement stopped at relative residual " + std::to_string(rel));
      continue;
    }
    (E.opt.precision == ACR_FP64 ? go64 : go32).push_back(r.get());
    keep.push_back(r);
  }
  solve_chunks<double>(S, go64, st);
  solve_chunks<float>(S, go32, st);
  std::vector<RJob> ax;
  for (auto& r : keep) {
    OpEntry& E = *S->ops[r->op];
    RJob J;
    J.nx = E.op.nx; J.ny = E.op.ny; J.nrhs = r->nrhs;
    J.B = r->D.get(); J.R = r->X;
    ax.push_back(J);
    ++r->iters;
  }
  gaxpy(st, ax);
  queue_flush();
  S->active.swap(keep);
  std::lock_guard<std::mutex> g(S->mu);
  ++S->steps;
}

void fail_all(acr_server_s* S, acr_status code, const std::string& msg) {
  for (auto* v : {&S->active, &S->pending})
    for (auto& r : *v) {
      if (r->active) --S->ops[r->op]->users;
      r->active = false;
      finish(S, r.get(), code, msg);
    }
  S->active.clear();
  S->pending.clear();
}

void worker_main(acr_server_s* S) {
  (void)hipSetDevice(S->device);
  StreamScope ss(S->st);
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_work.wait(lk, [&] { return S->stop || !S->incoming.empty() || !S->active.empty() || !S->pending.empty(); });
      if (S->stop && S->incoming.empty() && S->active.empty() && S->pending.empty()) break;
      while (!S->incoming.empty()) {
        S->pending.push_back(S->incoming.front());
        S->incoming.pop_front();
      }
    }
    const auto t0 = Clock::now();
    try {
      // (with nothing active every resident factor is idle; a factor that
      // requests wait for is kept unless an operator starves, and waiting
      // requests start to starve after kStarveMs, so admission always makes
      // progress: a factor over the whole budget is admitted alone)
      if (!S->pending.empty()) admit(S);
      if (!S->active.empty()) step(S);
      queue_flush();
    } catch (const Error& e) {
      Queue::get().discard();
      fail_all(S, e.code, e.what());
    } catch (const std::exception& e) {
      Queue::get().discard();
      fail_all(S, ACR_ERR_INTERNAL, e.what());
    }
    std::lock_guard<std::mutex> g(S->mu);
    S->busy_s += std::chrono::duration<double>(Clock::now() - t0).count();
  }
  (void)hipStreamSynchronize(S->st);
}

double percentile(std::vector<double> v, double p) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const double x = p * (v.size() - 1);
  const size_t i = (size_t)x;
  const double f = x - i;
  return i + 1 < v.size() ? v[i] * (1 - f) + v[i + 1] * f : v[i];
}

}  // namespace
}  // namespace acr

using namespace acr;

extern "C" {

acr_status acr_server_create(const acr_server_config* cfg, acr_server* out) {
  return guard([&] {
    if (!cfg || !out) fail(ACR_ERR_INVALID_ARG, "NULL argument");
    if (cfg->memory_budget <= 0) fail(ACR_ERR_INVALID_ARG, "memory_budget must be > 0");
    if (!(cfg->tol > 0.0) || cfg->maxit < 0) fail(ACR_ERR_INVALID_ARG, "tol must be > 0 and maxit >= 0");
    auto S = std::make_unique<acr_server_s>();
    S->cfg = *cfg;
    ACR_HIP(hipGetDevice(&S->device));
    ACR_HIP(hipStreamCreateWithFlags(&S->st, hipStreamNonBlocking));
    acr_server_s* raw = S.get();
    S->worker = std::thread(worker_main, raw);
    *out = S.release();
  });
}

acr_status acr_server_add_operator(acr_server s, const acr_operator* op, const acr_options* opt, int32_t* op_id) {
  return guard([&] {
    if (!s || !op_id) fail(ACR_ERR_INVALID_ARG, "NULL argument");
    check_op(op);
    check_options(opt);
    if (hodlr_depth(op->nx, opt->leaf) < 0)
      fail(ACR_ERR_INVALID_ARG, "block size must be leaf' * 2^L (halving exact down to the leaf)");
    auto E = std::make_unique<OpEntry>();
    const size_t n = (size_t)op->nx * op->ny;
    ACR_HIP(hipDeviceSynchronize());   // the copy below is ordered after every stream's work
    E->arrays.resize(5 * n);
    const double* src[5] = {op->diag, op->west, op->east, op->south, op->north};
    for (int a = 0; a < 5; ++a)
      ACR_HIP(hipMemcpy(E->arrays.get() + a * n, src[a], n * sizeof(double), hipMemcpyDeviceToDevice));
    ACR_HIP(hipDeviceSynchronize());
    E->op = *op;
    E->op.diag = E->arrays.get();
    E->op.west = E->arrays.get() + n;
    E->op.east = E->arrays.get() + 2 * n;
    E->op.south = E->arrays.get() + 3 * n;
    E->op.north = E->arrays.get() + 4 * n;
    E->opt = *opt;
    E->est = estimate_bytes(*op, *opt);
    std::lock_guard<std::mutex> g(s->mu);
    *op_id = (int32_t)s->ops.size();
    s->ops.push_back(std::move(E));
  });
}

acr_status acr_server_submit(acr_server s, int32_t op_id, const double* B, double* X, int32_t nrhs, void* stream,
                             int64_t* request) {
  return guard([&] {
    if (!s || !B || !X || !request || nrhs < 1) fail(ACR_ERR_INVALID_ARG, "bad arguments");
    auto r = std::make_shared<Request>();
    {
      std::lock_guard<std::mutex> g(s->mu);
      if (op_id < 0 || op_id >= (int)s->ops.size()) fail(ACR_ERR_INVALID_ARG, "unknown operator id");
      const acr_operator& op = s->ops[op_id]->op;
      if (overlap2(X, (size_t)op.nx * op.ny * nrhs, B, (size_t)op.nx * op.ny * nrhs))
        fail(ACR_ERR_INVALID_ARG, "X must not overlap B");
    }
    ACR_HIP(hipEventCreateWithFlags(&r->ready, hipEventDisableTiming));
    ACR_HIP(hipEventRecord(r->ready, static_cast<hipStream_t>(stream)));
    r->op = op_id;
    r->B = B;
    r->X = X;
    r->nrhs = nrhs;
    r->t0 = Clock::now();
    std::lock_guard<std::mutex> g(s->mu);
    r->id = s->next_id++;
    if (!s->any) {
      s->any = true;
      s->t_first = r->t0;
    }
    s->reqs[r->id] = r;
    s->incoming.push_back(r);
    *request = r->id;
    s->cv_work.notify_one();
  });
}

acr_status acr_server_wait(acr_server s, int64_t request, int32_t* iters, double* relres, double* latency_ms) {
  std::shared_ptr<Request> r;
  acr_status st0 = guard([&] {
    if (!s) fail(ACR_ERR_INVALID_ARG, "NULL server");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(request);
    if (it == s->reqs.end()) fail(ACR_ERR_INVALID_ARG, "unknown request (or already waited for)");
    r = it->second;
    s->cv_done.wait(lk, [&] { return r->done; });
    s->reqs.erase(it);
  });
  if (st0 != ACR_OK) return st0;
  if (r->ready) (void)hipEventDestroy(r->ready);
  if (iters) *iters = r->iters;
  if (relres) *relres = r->relres;
  if (latency_ms) *latency_ms = r->latency_ms;
  if (r->status != ACR_OK) {
    set_last_error(r->err);
    return r->status;
  }
  return ACR_OK;
}

acr_status acr_server_stats(acr_server s, int32_t reset, acr_server_info* out) {
  return guard([&] {
    if (!s || !out) fail(ACR_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> g(s->mu);
    std::memset(out, 0, sizeof(*out));
    out->requests = s->req_done;
    out->rhs = s->rhs_done;
    out->steps = s->steps;
    out->factorizations = s->factorizations;
    out->evictions = s->evictions;
    out->resident_bytes = (int64_t)s->resident;
    out->peak_resident_bytes = (int64_t)s->peak_resident;
    const double span = s->any && s->req_done ? std::chrono::duration<double>(s->t_last - s->t_first).count() : 0.0;
    out->seconds = span;
    out->rhs_per_s = span > 0 ? s->rhs_done / span : 0.0;
    out->requests_per_s = span > 0 ? s->req_done / span : 0.0;
    out->latency_p50_ms = percentile(s->lat, 0.50);
    out->latency_p99_ms = percentile(s->lat, 0.99);
    out->latency_max_ms = s->lat.empty() ? 0.0 : *std::max_element(s->lat.begin(), s->lat.end());
    out->busy_s = s->busy_s;
    if (reset) {
      s->lat.clear();
      s->rhs_done = s->req_done = s->steps = 0;
      s->busy_s = 0.0;
      s->any = false;
      s->evictions = s->factorizations = 0;
      s->peak_resident = s->resident;
    }
  });
}

acr_status acr_server_destroy(acr_server s) {
  return guard([&] {
    if (!s) return;
    {
      std::lock_guard<std::mutex> g(s->mu);
      s->stop = true;
      s->cv_work.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    (void)hipDeviceSynchronize();
    {
      Pool::IdleScope idle;
      for (auto& kv : s->reqs)
        if (kv.second->ready) (void)hipEventDestroy(kv.second->ready);
      s->reqs.clear();
      s->ops.clear();
    }
    (void)hipStreamDestroy(s->st);
    delete s;
  });
}

}  // extern "C"
