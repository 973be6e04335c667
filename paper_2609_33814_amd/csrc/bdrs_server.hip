// Solve server: continuous batching of independent OT solves (bdrs_server_*).
//
// bdrs_server_submit validates a request and prepares its host image (points
// in Morton tile order, tile records) on the caller's thread, so the worker
// only uploads it.  A worker thread owns the GPU work.  Requests wait in a
// FIFO queue; at every block boundary the worker admits requests from the
// head of the queue while a slot is free and the pool can hold the request's
// workspace together with the batch engine's grown work lists (with the
// size-aware policy, requests above a work threshold run one at a time, in
// arrival order, and smaller ones may pass a waiting large one), runs one
// block of iterations of all running requests through the batch engine,
// reads every request's certificate, and retires the finished ones (their
// pool memory is reused by the next admissions).  A block whose set of
// running requests is the same as in the previous block is captured once as a
// graph and replayed until the set changes.  The per-request arithmetic is
// the single-problem one, so results do not depend on the mix.
#include "bdrs_host.h"
#include "bdrs_sched.h"

#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

using namespace bdrs_host;

namespace {

using bdrs_sched::PoolAlloc;

struct Request {
  uint64_t ticket = 0;
  bdrs_params prm{};
  HostImage img;          // prepared at submit; released when the request is done
  double tau = 0;
  int tau_relative = 1;
  int max_iters = 0;
  size_t bytes = 0, off = 0;
  double work = 0;  // implicit entries per sweep, m n
  bdrs_solver solver = nullptr;
  int iters = 0;
  bdrs_result res{};
};

}  // namespace

struct bdrs_server_ {
  char* pool = nullptr;
  int max_slots = 1, block_iters = 50, device = 0;
  double big_work = 0;  // > 0: requests with more entries per sweep run one at a time
  hipStream_t stream = nullptr;
  std::chrono::steady_clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stop = false;
  uint64_t next_ticket = 1;
  std::unique_ptr<PoolAlloc> alloc;
  std::deque<std::shared_ptr<Request>> queue;
  std::vector<std::shared_ptr<Request>> running;
  std::unordered_map<uint64_t, std::shared_ptr<Request>> all;
  std::thread worker;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  void run();
};

namespace {

void finish(bdrs_server_* sv, const std::shared_ptr<Request>& rq, int status) {
  // called with the lock held
  rq->res.state = 2;
  rq->res.status = status;
  rq->res.t_done = sv->now();
  if (rq->solver) {
    bdrs_destroy(rq->solver);
    rq->solver = nullptr;
  }
  if (rq->bytes) {
    sv->alloc->release(rq->off);
    rq->bytes = 0;
  }
  rq->img = HostImage();
}

// Puts a running request back at the head of the queue (its solver and
// workspace are given up; it restarts from iteration 0 when admitted again).
// Called with the lock held.
void requeue(bdrs_server_* sv, const std::shared_ptr<Request>& rq) {
  if (rq->solver) {
    bdrs_destroy(rq->solver);
    rq->solver = nullptr;
  }
  if (rq->bytes) {
    sv->alloc->release(rq->off);
    rq->bytes = 0;
  }
  rq->iters = 0;
  rq->res.state = 0;
  rq->res.cert = bdrs_cert{};
  rq->res.cert.repaired_cost = NAN;
  sv->queue.push_front(rq);
}

}  // namespace

void bdrs_server_::run() {
  const bool dev_ok = hipSetDevice(device) == hipSuccess;  // else every request fails with E_DEVICE
  BatchEngine eng;
  size_t eng_off = 0, eng_bytes = 0;
  bool eng_valid = false;  // the engine is bound to the current running set at eng_off
  bool stable = false;     // the running set is the same as in the previous block
  std::vector<double> rec;
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    // admission at the block boundary: in arrival order while a slot and memory
    // are free; with the size-aware policy a large request waits while another
    // large one runs and the requests behind it that are small may pass it
    bool changed = false;
    while (!stop && !queue.empty()) {
      std::vector<double> queued_work, running_work;
      for (auto& r : queue) queued_work.push_back(r->work);
      for (auto& r : running) running_work.push_back(r->work);
      const int pi = bdrs_sched::pick_admission(queued_work, running_work, max_slots, big_work);
      if (pi < 0) break;
      auto pick = queue.begin() + pi;
      std::shared_ptr<Request> rq = *pick;
      if (!dev_ok) {
        queue.erase(pick);
        finish(this, rq, BDRS_E_DEVICE);
        cv_done.notify_all();
        continue;
      }
      // the request's workspace and the engine's work lists for the grown
      // running set are placed together, so an admitted request always runs
      const Layout lay = make_layout(rq->prm.m, rq->prm.n, rq->prm.dim);
      std::vector<const Layout*> lays;
      for (auto& r : running) lays.push_back(&r->solver->L);
      lays.push_back(&lay);
      const size_t need = BatchEngine::bytes_for_layouts(lays);
      size_t off = 0;
      bool moved = false;
      const bool placed = bdrs_sched::place_with_engine(*alloc, lay.total, need, &off, &eng_off, &eng_bytes, &moved);
      if (moved) eng_valid = false;
      if (!placed) {
        if (running.empty()) {
          // it can never fit (e.g. the tuning table grew its layout since it was submitted)
          queue.erase(pick);
          finish(this, rq, BDRS_E_NOMEM);
          cv_done.notify_all();
          continue;
        }
        break;  // the candidate waits for memory; nothing passes it
      }
      queue.erase(pick);
      rq->off = off;
      rq->bytes = lay.total;
      rq->prm.workspace = pool + off;
      rq->prm.workspace_bytes = lay.total;
      rq->prm.stream = stream;
      lk.unlock();
      bdrs_solver s = nullptr;
      const bdrs_status st = create_from_image(&rq->prm, rq->img, &s);  // upload only
      lk.lock();
      if (st != BDRS_OK) {
        finish(this, rq, st);
        cv_done.notify_all();
        continue;
      }
      rq->solver = s;  // the host image stays until the request is done (a requeue re-uploads it)
      rq->res.state = 1;
      rq->res.t_admit = now();
      running.push_back(rq);
      changed = true;
    }
    if (running.empty()) {
      stable = false;
      if (stop) break;
      cv_work.wait(lk, [&] { return stop || !queue.empty(); });
      continue;
    }
    if (changed || !eng_valid) {
      std::vector<bdrs_solver> mem;
      for (auto& rq : running) mem.push_back(rq->solver);
      const size_t need = BatchEngine::bytes_for(mem);
      if (align_up(need) > eng_bytes) {
        // not reached: admission reserved the engine's room for this set.  If
        // it is, the newest request goes back to the head of the queue.
        auto rq = running.back();
        running.pop_back();
        requeue(this, rq);
        eng_valid = false;
        continue;
      }
      lk.unlock();
      // eager blocks until the set has stayed the same for one block
      const hipError_t e = eng.bind(mem, pool + eng_off, block_iters, false, stream);
      lk.lock();
      if (e != hipSuccess) {
        for (auto& rq : running) finish(this, rq, BDRS_E_DEVICE);
        running.clear();
        cv_done.notify_all();
        eng_valid = false;
        continue;
      }
      eng_valid = true;
      stable = false;
    }
    lk.unlock();
    hipError_t e = hipSuccess;
    if (stable && !eng.captured()) e = eng.capture();  // replayed until the set changes
    if (e == hipSuccess) e = eng.run_block();
    if (e == hipSuccess) e = eng.read_records(rec);
    lk.lock();
    if (e != hipSuccess) {
      for (auto& rq : running) finish(this, rq, BDRS_E_DEVICE);
      running.clear();
      eng_valid = false;
      cv_done.notify_all();
      continue;
    }
    std::vector<std::shared_ptr<Request>> still;
    for (size_t q = 0; q < running.size(); ++q) {
      auto& rq = running[q];
      rq->solver->k += block_iters;
      rq->iters += block_iters;
      const bdrs_status cs = cert_from_record(rq->solver, rec.data() + q * kCertSlots, false, &rq->res.cert);
      const bdrs_cert& ce = rq->res.cert;
      const double target = rq->tau_relative ? ce.rel_gap_best : (ce.U_best - ce.L_best);
      if (cs != BDRS_OK) finish(this, rq, cs);
      else if (target <= rq->tau) finish(this, rq, BDRS_OK);
      else if (rq->iters >= rq->max_iters) finish(this, rq, BDRS_NOT_CONVERGED);
      else still.push_back(rq);
    }
    stable = still.size() == running.size();
    if (!stable) {
      running.swap(still);
      eng_valid = false;
      cv_done.notify_all();
    }
    if (stop) {
      for (auto& rq : running) finish(this, rq, BDRS_E_STATE);
      running.clear();
      break;
    }
  }
  for (auto& rq : queue) finish(this, rq, BDRS_E_STATE);
  queue.clear();
  if (eng_bytes) alloc->release(eng_off);
  cv_done.notify_all();
}

extern "C" {

bdrs_status bdrs_server_create(void* pool, size_t pool_bytes, int32_t max_slots, int32_t block_iters,
                               bdrs_server* out) {
  if (!out) return fail(BDRS_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!pool || ((uintptr_t)pool) % kAlign) return fail(BDRS_E_INVALID, "pool must be non-NULL and 256-byte aligned");
  if (pool_bytes < kAlign) return fail(BDRS_E_INVALID, "pool_bytes too small");
  if (max_slots < 1) return fail(BDRS_E_INVALID, "max_slots must be >= 1");
  if (block_iters < 1) return fail(BDRS_E_INVALID, "block_iters must be >= 1");
  bdrs_status st = check_device();
  if (st != BDRS_OK) return st;
  auto* sv = new bdrs_server_();
  sv->pool = (char*)pool;
  sv->max_slots = max_slots;
  sv->block_iters = block_iters;
  sv->alloc.reset(new PoolAlloc(pool_bytes / kAlign * kAlign));
  sv->t0 = std::chrono::steady_clock::now();
  hipError_t e = hipGetDevice(&sv->device);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&sv->stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete sv;
    return fail(BDRS_E_DEVICE, "HIP error %s creating the server stream", hipGetErrorString(e));
  }
  sv->worker = std::thread([sv] { sv->run(); });
  *out = sv;
  return BDRS_OK;
}

bdrs_status bdrs_server_submit(bdrs_server sv, const bdrs_request* rq, uint64_t* ticket) {
  if (!sv) return fail(BDRS_E_INVALID, "server is NULL");
  if (!rq || !ticket) return fail(BDRS_E_INVALID, "request and ticket are required");
  const double t_call = sv->now();  // the host preparation below counts into the latency
  bdrs_params p{};
  p.m = rq->m;
  p.n = rq->n;
  p.dim = rq->dim;
  p.x = rq->x;
  p.y = rq->y;
  p.r = rq->r;
  p.c = rq->c;
  p.cost_scale = rq->cost_scale;
  p.eta = rq->eta;
  p.lambda = rq->lambda;
  p.omega = rq->omega;
  p.workspace = sv->pool;  // placeholder for the checks; the real slot is assigned at admission
  p.workspace_bytes = (size_t)-1;
  bdrs_status st = check_params(&p);
  if (st != BDRS_OK) return st;
  if (!(rq->tau >= 0 && std::isfinite(rq->tau))) return fail(BDRS_E_INVALID, "tau must be finite and >= 0");
  if (rq->max_iters < 1 || rq->max_iters % sv->block_iters)
    return fail(BDRS_E_INVALID, "max_iters must be a positive multiple of block_iters (%d)", sv->block_iters);
  auto r = std::make_shared<Request>();
  r->prm = p;
  const Layout lay = make_layout(p.m, p.n, p.dim);
  r->work = (double)p.m * (double)p.n;
  // its workspace and the batch engine's work lists for it alone must fit the pool
  const size_t alone = align_up(lay.total) + align_up(BatchEngine::bytes_for_layouts({&lay}));
  if (alone > sv->alloc->size())
    return fail(BDRS_E_NOMEM, "request needs %zu bytes with its work lists, the pool holds %zu", alone,
                sv->alloc->size());
  // contents validated and the host image built here, on the caller's thread
  if ((st = prepare_image(&p, rq->x, rq->y, rq->r, rq->c, r->img)) != BDRS_OK) return st;
  r->tau = rq->tau;
  r->tau_relative = rq->tau_relative;
  r->max_iters = rq->max_iters;
  std::lock_guard<std::mutex> g(sv->mu);
  if (sv->stop) return fail(BDRS_E_STATE, "server is stopping");
  r->ticket = sv->next_ticket++;
  r->res.state = 0;
  r->res.t_submit = t_call;
  r->res.cert.repaired_cost = NAN;
  sv->all[r->ticket] = r;
  sv->queue.push_back(r);
  *ticket = r->ticket;
  sv->cv_work.notify_all();
  return BDRS_OK;
}

bdrs_status bdrs_server_set_policy(bdrs_server sv, double big_work) {
  if (!sv) return fail(BDRS_E_INVALID, "server is NULL");
  if (!std::isfinite(big_work)) return fail(BDRS_E_INVALID, "big_work must be finite");
  std::lock_guard<std::mutex> g(sv->mu);
  sv->big_work = big_work > 0 ? big_work : 0.0;
  sv->cv_work.notify_all();
  return BDRS_OK;
}

bdrs_status bdrs_server_poll(bdrs_server sv, uint64_t ticket, bdrs_result* out) {
  if (!sv || !out) return fail(BDRS_E_INVALID, "server and out are required");
  std::lock_guard<std::mutex> g(sv->mu);
  auto it = sv->all.find(ticket);
  if (it == sv->all.end()) return fail(BDRS_E_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
  *out = it->second->res;
  return BDRS_OK;
}

bdrs_status bdrs_server_wait(bdrs_server sv, uint64_t ticket, bdrs_result* out) {
  if (!sv || !out) return fail(BDRS_E_INVALID, "server and out are required");
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->all.find(ticket);
  if (it == sv->all.end()) return fail(BDRS_E_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
  auto rq = it->second;
  sv->cv_done.wait(lk, [&] { return rq->res.state == 2; });
  *out = rq->res;
  return BDRS_OK;
}

bdrs_status bdrs_server_stats(bdrs_server sv, int32_t* running, int32_t* queued, size_t* pool_used) {
  if (!sv) return fail(BDRS_E_INVALID, "server is NULL");
  std::lock_guard<std::mutex> g(sv->mu);
  if (running) *running = (int32_t)sv->running.size();
  if (queued) *queued = (int32_t)sv->queue.size();
  if (pool_used) *pool_used = sv->alloc->used();
  return BDRS_OK;
}

bdrs_status bdrs_server_now(bdrs_server sv, double* t) {
  if (!sv || !t) return fail(BDRS_E_INVALID, "server and t are required");
  *t = sv->now();
  return BDRS_OK;
}

bdrs_status bdrs_server_destroy(bdrs_server sv) {
  if (!sv) return BDRS_OK;
  {
    std::lock_guard<std::mutex> g(sv->mu);
    sv->stop = true;
  }
  sv->cv_work.notify_all();
  if (sv->worker.joinable()) sv->worker.join();
  // teardown: the worker has drained the stream's work; nothing to report
  (void)hipStreamSynchronize(sv->stream);
  (void)hipStreamDestroy(sv->stream);
  delete sv;
  return BDRS_OK;
}

}  // extern "C"
