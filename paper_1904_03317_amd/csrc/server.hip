// Serving loop: many Poisson solves on different adaptive meshes resident in
// one HBM arena at once.  Host worker threads build each request's maps as
// it arrives; the scheduler thread admits ready requests whenever a slot and
// enough arena memory are free (first fit), binds them (upload and device
// set-up on the slot's stream), and then advances every resident solve by
// one CG iteration per tick.  The requests whose next iteration is due in a
// tick, grouped by dimension, degree, precision and smoother, run it as one
// batched iteration on the batch stream: every step of the V-cycle (each
// smoothing step, residual, restriction and prolongation of a level, the
// coarse solves) and of the rest of the CG iteration is one launch over all
// of them, so that a tick of K requests costs the launches of one iteration
// and fills the device with the blocks of all K.  The members of a batch are
// next checked together, once all of them finished, so that a group stays
// in step.  A request alone in its group (or with batching off) replays its
// V-cycle as a captured HIP graph on its own slot stream.  Requests leave
// when their residual reaches the tolerance and their memory and slot go to
// the next ones (continuous batching at CG iteration granularity).  All
// kernels are deterministic and a batched launch computes what the
// request's own launches would, so a result does not depend on what else
// was resident.  A finished solution is copied back into a pinned host
// buffer of the request on its slot stream; the scheduler keeps ticking the
// other requests and completes the copy on a later tick.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/gmg.h"
#include "host/forest.hpp"
#include "problem.hpp"

struct gmg_mesh_s {
  std::unique_ptr<gmg::Forest> f;
};

namespace gmg {

#define SRV_HIPCHECK(x)                                                                       \
  do {                                                                                        \
    hipError_t e_ = (x);                                                                      \
    if (e_ != hipSuccess) gmg::fail(GMG_E_HIP, std::string(#x ": ") + hipGetErrorString(e_)); \
  } while (0)

enum ReqState { kQueued = 0, kSetup = 1, kReady = 2, kBinding = 3, kRunning = 4, kDone = 5, kFailed = 6,
                kWaitRhs = 7 };

struct Request {
  uint64_t id = 0;
  int state = kQueued;
  int status = 0;
  std::string error;
  std::unique_ptr<Forest> mesh;
  gmg_options opt{};
  std::vector<double> coeff;
  // nodal right-hand side in canonical leaf DoF order; empty means f = 1
  std::vector<double> f_host;
  bool rhs_later = false;  // given by gmg_server_set_rhs (rhs_given once it was)
  bool rhs_given = false;
  int64_t n_dofs = -1;     // known after host set-up
  std::unique_ptr<Problem> P;
  size_t ws_bytes = 0, arena_off = 0;
  int slot = -1;
  double* d_f = nullptr;   // inside the workspace tail: f (nodal) and u
  double* d_u = nullptr;
  gmg_timing t{};
  double* u_pin = nullptr;        // pinned host copy of the solution
  hipEvent_t copied = nullptr;    // recorded after the copy-back
  bool copying = false;
  int iterations = 0;
  std::vector<double> hist;
  ~Request() {
    if (u_pin) (void)hipHostFree(u_pin);
    if (copied) (void)hipEventDestroy(copied);
  }
};

// first-fit allocator over the arena (offsets), 256-byte granularity
class Arena {
 public:
  explicit Arena(size_t bytes) : size_(bytes) { free_[0] = bytes; }
  bool alloc(size_t n, size_t* off) {
    n = (n + 255) & ~size_t(255);
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= n) {
        *off = it->first;
        size_t rest = it->second - n, start = it->first + n;
        free_.erase(it);
        if (rest) free_[start] = rest;
        used_ += n;
        peak_ = std::max(peak_, used_);
        return true;
      }
    return false;
  }
  void release(size_t off, size_t n) {
    n = (n + 255) & ~size_t(255);
    used_ -= n;
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }
  size_t size() const { return size_; }

 private:
  size_t size_, used_ = 0, peak_ = 0;
  std::map<size_t, size_t> free_;
};

struct Server {
  char* arena_base = nullptr;
  Arena arena;
  int max_slots = 1;
  int device = 0;
  std::vector<hipStream_t> streams;
  // batched V-cycles: launch tables at the front of the arena (table_bytes,
  // 0 = batching unavailable), uploaded through two pinned staging buffers
  // in turn, each reusable once its event (recorded after the upload) is done
  bool batching = true;
  std::atomic<bool> hold{false};  // resident solves not advanced while set
  hipStream_t bstream = nullptr;
  char* d_table = nullptr;
  size_t table_bytes = 0;
  char* h_stage[2] = {nullptr, nullptr};
  hipEvent_t ev_stage[2] = {nullptr, nullptr};
  hipEvent_t ev_batch = nullptr;
  int stage_next = 0;
  int64_t iterations = 0, batched_iterations = 0, batches = 0;
  // members of batched iterations still in flight: none of them is checked
  // before all of them have finished, so that a group stays in step and
  // its next V-cycles are batched again
  std::vector<std::vector<Request*>> inflight;
  std::vector<int> slot_free;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request*> setup_q;    // queued, waiting for a host worker
  std::deque<Request*> ready_q;    // maps built, waiting for admission
  std::deque<Request*> bind_q;     // admitted, waiting for device set-up
  std::vector<Request*> running;
  std::vector<Request*> copying;   // solution copy-back in flight
  std::map<uint64_t, std::unique_ptr<Request>> all;
  std::vector<std::thread> workers;
  int host_cpus = 1;               // host threads for map builds, shared by the workers
  std::atomic<int> building{0};    // map builds in progress
  std::thread sched;
  std::atomic<bool> stop{false};
  uint64_t next_id = 1;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  int64_t completed = 0, failed = 0;
  double dofs_done = 0.0;

  Server(char* base, size_t bytes, int slots) : arena_base(base), arena(bytes), max_slots(slots) {}
  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace {

size_t request_bytes(const Problem& P) { return P.ws_need + 2 * (size_t(P.maps->n_dofs) * 8 + 256); }

void fail_request(Server& S, Request* r, int code, const std::string& msg) {
  r->state = kFailed;
  r->status = code;
  r->error = msg;
  r->t.finished = S.now();
  ++S.failed;
}

// ready requests are admitted in arrival order
void push_ready(Server& S, Request* r) {
  r->state = kReady;
  auto it = S.ready_q.begin();
  while (it != S.ready_q.end() && (*it)->id < r->id) ++it;
  S.ready_q.insert(it, r);
}

// hand the arena range and slot of a request back once nothing of it is in
// flight on its slot stream (errors of that wait are not the request's any more)
void release_slot(Server& S, Request* r) {
  (void)hipStreamSynchronize(S.streams[r->slot]);
  (void)hipGetLastError();
  S.arena.release(r->arena_off, r->ws_bytes);
  S.slot_free.push_back(r->slot);
}

void worker_loop(Server* S) {
  SRV_HIPCHECK(hipSetDevice(S->device));
  while (true) {
    Request* r = nullptr;
    bool bind_job = false;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_work.wait(lk, [&] { return S->stop || !S->setup_q.empty() || !S->bind_q.empty(); });
      if (S->stop) return;
      if (!S->bind_q.empty()) {
        r = S->bind_q.front();
        S->bind_q.pop_front();
        bind_job = true;
      } else {
        r = S->setup_q.front();
        S->setup_q.pop_front();
        r->state = kSetup;
      }
    }
    try {
      if (!bind_job) {
        // host set-up: forest -> maps (no device work)
        auto P = std::make_unique<Problem>();
        P->opt = r->opt;
        P->kt = kernel_table(r->mesh->dim(), r->opt.degree);
        if (!P->kt) fail(GMG_E_INVAL, "no kernels for this dimension/degree");
        // the host threads are shared among the map builds in progress when
        // this one starts (the maps do not depend on the thread count)
        const int active = ++S->building;
        struct Done {
          std::atomic<int>& n;
          ~Done() { --n; }
        } done{S->building};
        P->maps = std::make_shared<const Maps>(build_maps(
            *r->mesh, r->opt.degree, r->coeff.empty() ? nullptr : r->coeff.data(), std::max(1, S->host_cpus / active)));
        const FE1D& fe = P->maps->fe;
        for (int i = 0; i < 25; ++i) {
          P->m64.M[i] = fe.M[i];
          P->m64.K[i] = fe.K[i];
          P->m32.M[i] = (float)fe.M[i];
          P->m32.K[i] = (float)fe.K[i];
        }
        for (int i = 0; i < 45; ++i) {
          P->m64.E[i] = fe.E[i];
          P->m32.E[i] = (float)fe.E[i];
        }
        P->ws_need = plan_workspace(*P, nullptr);
        std::lock_guard<std::mutex> lk(S->mu);
        r->P = std::move(P);
        r->mesh.reset();
        r->ws_bytes = request_bytes(*r->P);
        r->n_dofs = r->P->maps->n_dofs;
        r->t.setup_done = S->now();
        if (r->ws_bytes > S->arena.size()) {
          fail_request(*S, r, GMG_E_BUDGET, "request needs more device memory than the arena holds");
          S->cv_done.notify_all();
        } else if (!r->f_host.empty() && (int64_t)r->f_host.size() != r->n_dofs) {
          fail_request(*S, r, GMG_E_INVAL, "right-hand side length differs from the request's DoF count");
          S->cv_done.notify_all();
        } else if (r->rhs_later && !r->rhs_given) {
          r->state = kWaitRhs;  // gmg_server_set_rhs moves it on
          S->cv_done.notify_all();
        } else {
          push_ready(*S, r);
        }
      } else {
        // device set-up on the request's slot stream
        Problem& P = *r->P;
        hipStream_t s = S->streams[r->slot];
        char* base = S->arena_base + r->arena_off;
        bind_problem(P, base, P.ws_need, s);
        P.opt.use_graph = 1;
        const int64_t N = P.maps->n_dofs;
        size_t tail = (P.ws_need + 255) & ~size_t(255);
        r->d_f = reinterpret_cast<double*>(base + tail);
        r->d_u = reinterpret_cast<double*>(base + tail + ((size_t(N) * 8 + 255) & ~size_t(255)));
        if (r->f_host.empty())
          set_constant(r->d_f, N, 1.0, s);
        else
          SRV_HIPCHECK(hipMemcpyAsync(r->d_f, r->f_host.data(), size_t(N) * sizeof(double), hipMemcpyHostToDevice, s));
        if (!r->u_pin) SRV_HIPCHECK(hipHostMalloc((void**)&r->u_pin, std::max<size_t>(1, size_t(N)) * sizeof(double),
                                                  hipHostMallocDefault));
        if (!r->copied) SRV_HIPCHECK(hipEventCreateWithFlags(&r->copied, hipEventDisableTiming));
        apply_leaf(P, r->d_f, P.cb, true, s);
        cg_start(P, P.cb, r->d_u, s, false);
        std::lock_guard<std::mutex> lk(S->mu);
        r->t.bound = S->now();
        r->state = kRunning;
        S->running.push_back(r);
      }
    } catch (const Error& e) {
      std::lock_guard<std::mutex> lk(S->mu);
      if (bind_job) release_slot(*S, r);
      fail_request(*S, r, e.code, e.what());
      S->cv_done.notify_all();
    } catch (const std::exception& e) {
      std::lock_guard<std::mutex> lk(S->mu);
      if (bind_job) release_slot(*S, r);
      fail_request(*S, r, GMG_E_INVAL, e.what());
      S->cv_done.notify_all();
    }
  }
}

// The next CG iteration of each request of `due` (all of one group) as one
// batched iteration on the batch stream; requests whose iteration could not
// be enqueued are added to `failed` with their error.
void enqueue_batch(Server& S, const std::vector<Request*>& due,
                   std::vector<std::tuple<Request*, int, std::string>>& failed) {
  std::vector<Problem*> ps;
  for (Request* r : due) ps.push_back(r->P.get());
  size_t need = 0;
  try {
    cg_iteration_batch(ps, nullptr, 0, &need, nullptr, S.bstream);
    if (need > S.table_bytes) {
      // tables of the whole group do not fit: two halves in turn
      if (due.size() >= 2) {
        const size_t h = due.size() / 2;
        enqueue_batch(S, std::vector<Request*>(due.begin(), due.begin() + h), failed);
        enqueue_batch(S, std::vector<Request*>(due.begin() + h, due.end()), failed);
        return;
      }
      cg_enqueue_iteration(*due[0]->P);
      ++S.iterations;
      return;
    }
    const int k = S.stage_next;
    S.stage_next ^= 1;
    SRV_HIPCHECK(hipEventSynchronize(S.ev_stage[k]));  // the previous upload from this buffer has read it
    cg_iteration_batch(ps, S.d_table, S.table_bytes, &need, S.h_stage[k], S.bstream, S.ev_stage[k]);
  } catch (const Error& e) {
    // nothing of the failed requests may still run when their memory is
    // handed on
    (void)hipStreamSynchronize(S.bstream);
    (void)hipGetLastError();
    for (Request* r : due) failed.emplace_back(r, e.code, e.what());
    return;
  }
  ++S.batches;
  S.iterations += (int64_t)due.size();
  S.batched_iterations += (int64_t)due.size();
  S.inflight.push_back(due);
}

// requests of batched iterations whose batch has not finished yet (the
// others' batches are dropped from the in-flight list)
std::vector<Request*> gated(Server& S) {
  std::vector<Request*> out;
  for (size_t b = 0; b < S.inflight.size();) {
    bool all = true;
    for (Request* r : S.inflight[b])
      if (hipEventQuery(r->P->ev[4]) == hipErrorNotReady) {
        all = false;
        break;
      }
    if (all) {
      S.inflight.erase(S.inflight.begin() + b);
    } else {
      out.insert(out.end(), S.inflight[b].begin(), S.inflight[b].end());
      ++b;
    }
  }
  return out;
}

void scheduler_loop(Server* S) {
  SRV_HIPCHECK(hipSetDevice(S->device));
  while (!S->stop) {
    bool idle = true;
    {
      // admission: FIFO over ready requests, first fit in the arena
      std::lock_guard<std::mutex> lk(S->mu);
      for (auto it = S->ready_q.begin(); it != S->ready_q.end() && !S->slot_free.empty();) {
        Request* r = *it;
        size_t off;
        if (S->arena.alloc(r->ws_bytes, &off)) {
          r->arena_off = off;
          r->slot = S->slot_free.back();
          S->slot_free.pop_back();
          r->state = kBinding;
          r->t.admitted = S->now();
          S->bind_q.push_back(r);
          it = S->ready_q.erase(it);
          S->cv_work.notify_all();
          idle = false;
        } else {
          break;  // keep arrival order: wait for memory
        }
      }
    }
    std::vector<Request*> run, cop;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      if (!S->hold) run = S->running;
      cop = S->copying;
    }
    // copy-backs that have completed: the request is done, its memory and
    // slot go to the next ones
    for (Request* r : cop) {
      hipError_t e = hipEventQuery(r->copied);
      if (e == hipErrorNotReady) continue;
      idle = false;
      std::lock_guard<std::mutex> lk(S->mu);
      S->copying.erase(std::find(S->copying.begin(), S->copying.end(), r));
      release_slot(*S, r);
      r->t.finished = S->now();
      if (e != hipSuccess) {
        r->status = GMG_E_HIP;
        r->error = std::string("copying the solution back failed: ") + hipGetErrorString(e);
        r->state = kFailed;
        ++S->failed;
      } else {
        r->state = kDone;
        ++S->completed;
        S->dofs_done += (double)r->n_dofs;
      }
      r->P.reset();   // drop host maps and device views; the arena range is free
      S->cv_done.notify_all();
    }
    // requests whose solve finished (or failed), with status and error
    std::vector<std::tuple<Request*, int, std::string>> fin;
    // requests whose next iteration is due, by kernel set, precision,
    // Chebyshev degree and smoother
    std::map<std::tuple<const void*, int, int, int>, std::vector<Request*>> due;
    const std::vector<Request*> wait = gated(*S);
    for (Request* r : run) {
      if (std::find(wait.begin(), wait.end(), r) != wait.end()) continue;
      try {
        const int st = cg_check(*r->P, false);
        if (st == 0) continue;
        idle = false;
        if (st == 1) {
          fin.emplace_back(r, r->P->cg.status, std::string());
        } else {
          const gmg_options& o = r->P->opt;
          due[std::make_tuple((const void*)r->P->kt, o.mg_precision, o.cheb_degree, o.smoother)].push_back(r);
        }
      } catch (const Error& e) {
        idle = false;
        fin.emplace_back(r, e.code, e.what());
      }
    }
    for (auto& g : due) {
      if (S->batching && S->table_bytes && g.second.size() >= 2) {
        enqueue_batch(*S, g.second, fin);
        continue;
      }
      for (Request* r : g.second) {
        try {
          cg_enqueue_iteration(*r->P);
          ++S->iterations;
        } catch (const Error& e) {
          fin.emplace_back(r, e.code, e.what());
        }
      }
    }
    for (auto& f : fin) {
      Request* r = std::get<0>(f);
      int status = std::get<1>(f);
      std::string err = std::get<2>(f);
      Problem& P = *r->P;
      hipStream_t s = S->streams[r->slot];
      r->iterations = P.cg.it;
      r->hist.assign(P.cg.hist.begin(), P.cg.hist.begin() + P.cg.it + 1);
      if (status >= 0) {
        // enqueue the copy-back and finish the request on a later tick
        hipError_t e1 = hipMemcpyAsync(r->u_pin, r->d_u, P.maps->n_dofs * sizeof(double), hipMemcpyDeviceToHost, s);
        hipError_t e2 = e1 == hipSuccess ? hipEventRecord(r->copied, s) : e1;
        if (e2 == hipSuccess) {
          std::lock_guard<std::mutex> lk(S->mu);
          S->running.erase(std::find(S->running.begin(), S->running.end(), r));
          r->status = status;
          r->copying = true;
          S->copying.push_back(r);
          continue;
        }
        status = GMG_E_HIP;
        err = std::string("copying the solution back failed: ") + hipGetErrorString(e2);
      }
      std::lock_guard<std::mutex> lk(S->mu);
      S->running.erase(std::find(S->running.begin(), S->running.end(), r));
      release_slot(*S, r);
      r->t.finished = S->now();
      r->status = status;
      r->error = err;
      r->state = kFailed;
      ++S->failed;
      r->P.reset();
      S->cv_done.notify_all();
    }
    if (idle) std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
}

}  // namespace
}  // namespace gmg

using gmg::Server;

struct gmg_server_s {
  std::unique_ptr<Server> S;
};

namespace {
template <typename F>
int sguard(F&& f) {
  try {
    return f();
  } catch (const gmg::Error& e) {
    gmg::set_last_error(e.what());
    return e.code;
  } catch (const std::exception& e) {
    gmg::set_last_error(e.what());
    return GMG_E_INVAL;
  }
}
}  // namespace

extern "C" {

int gmg_server_create(void* d_arena, size_t arena_bytes, int32_t max_slots, int32_t host_threads,
                      gmg_server* out) {
  return sguard([&] {
    if (!d_arena || !out || max_slots < 1 || max_slots > 64 || host_threads < 1 || host_threads > 64)
      gmg::fail(GMG_E_INVAL, "invalid server arguments");
    if (reinterpret_cast<uintptr_t>(d_arena) & 255) gmg::fail(GMG_E_INVAL, "arena must be 256-byte aligned");
    // launch tables of the batched V-cycles at the front of the arena: 1/32
    // of it, at most 16 MiB (none for arenas under 2 MiB)
    const size_t tb = arena_bytes >= (size_t(2) << 20) ? std::min(arena_bytes / 32, size_t(16) << 20) & ~size_t(255) : 0;
    auto h = std::make_unique<gmg_server_s>();
    h->S = std::make_unique<Server>((char*)d_arena + tb, arena_bytes - tb, max_slots);
    Server& S = *h->S;
    S.d_table = (char*)d_arena;
    S.table_bytes = tb;
    SRV_HIPCHECK(hipGetDevice(&S.device));
    S.streams.resize(max_slots);
    for (int i = 0; i < max_slots; ++i) {
      SRV_HIPCHECK(hipStreamCreateWithFlags(&S.streams[i], hipStreamNonBlocking));
      S.slot_free.push_back(max_slots - 1 - i);
    }
    SRV_HIPCHECK(hipStreamCreateWithFlags(&S.bstream, hipStreamNonBlocking));
    SRV_HIPCHECK(hipEventCreateWithFlags(&S.ev_batch, hipEventDisableTiming));
    for (int i = 0; i < 2; ++i) {
      SRV_HIPCHECK(hipEventCreateWithFlags(&S.ev_stage[i], hipEventDisableTiming));
      if (tb) SRV_HIPCHECK(hipHostMalloc((void**)&S.h_stage[i], tb, hipHostMallocDefault));
    }
    S.host_cpus = std::max(1, (int)std::min(16u, std::thread::hardware_concurrency()));
    for (int i = 0; i < host_threads; ++i) S.workers.emplace_back(gmg::worker_loop, &S);
    S.sched = std::thread(gmg::scheduler_loop, &S);
    *out = h.release();
    return 0;
  });
}

int gmg_server_submit(gmg_server h, gmg_mesh mesh, const gmg_options* opts, const double* cell_coeff,
                      const double* f_nodal_host, int64_t n_f, uint64_t* request_id) {
  return sguard([&] {
    if (!h || !mesh || !opts || !request_id) gmg::fail(GMG_E_INVAL, "null argument");
    if (opts->degree < 1 || opts->degree > 4 || (opts->mg_precision != 32 && opts->mg_precision != 64) ||
        opts->cheb_degree < 1 || opts->max_iter < 1 || !(opts->rtol > 0) || opts->eig_iters < 1 ||
        !(opts->cheb_lo > 0) || !(opts->cheb_hi > opts->cheb_lo) ||
        (opts->smoother != GMG_SMOOTHER_CHEBYSHEV && opts->smoother != GMG_SMOOTHER_JACOBI) ||
        !(opts->relax > 0 && opts->relax <= 2))
      gmg::fail(GMG_E_INVAL, "invalid options");
    if (f_nodal_host ? n_f < 1 : (n_f != 0 && n_f != GMG_RHS_LATER))
      gmg::fail(GMG_E_INVAL, "right-hand side: an array with its length, or NULL with 0 or GMG_RHS_LATER");
    Server& S = *h->S;
    auto r = std::make_unique<gmg::Request>();
    r->opt = *opts;
    if (f_nodal_host) r->f_host.assign(f_nodal_host, f_nodal_host + n_f);
    r->rhs_later = !f_nodal_host && n_f == GMG_RHS_LATER;
    const int64_t nl = (int64_t)mesh->f->leaves().size();
    if (cell_coeff) r->coeff.assign(cell_coeff, cell_coeff + nl);
    r->mesh = std::move(mesh->f);
    delete mesh;
    std::lock_guard<std::mutex> lk(S.mu);
    r->id = S.next_id++;
    r->t.arrival = S.now();
    *request_id = r->id;
    S.setup_q.push_back(r.get());
    S.all[r->id] = std::move(r);
    S.cv_work.notify_all();
    return 0;
  });
}

int gmg_server_request_dofs(gmg_server h, uint64_t id, int64_t* n_dofs) {
  return sguard([&] {
    if (!h || !n_dofs) gmg::fail(GMG_E_INVAL, "null argument");
    Server& S = *h->S;
    std::lock_guard<std::mutex> lk(S.mu);
    auto it = S.all.find(id);
    if (it == S.all.end()) gmg::fail(GMG_E_INVAL, "unknown request id");
    if (it->second->n_dofs < 0) gmg::fail(GMG_E_STATE, "host set-up of the request not finished");
    *n_dofs = it->second->n_dofs;
    return 0;
  });
}

int gmg_server_set_rhs(gmg_server h, uint64_t id, const double* f_nodal_host, int64_t n_f) {
  return sguard([&] {
    if (!h || !f_nodal_host || n_f < 1) gmg::fail(GMG_E_INVAL, "invalid right-hand side");
    Server& S = *h->S;
    std::lock_guard<std::mutex> lk(S.mu);
    auto it = S.all.find(id);
    if (it == S.all.end()) gmg::fail(GMG_E_INVAL, "unknown request id");
    gmg::Request* r = it->second.get();
    if (!r->rhs_later || r->rhs_given) gmg::fail(GMG_E_STATE, "the request takes no (further) right-hand side");
    if (r->n_dofs >= 0 && n_f != r->n_dofs)
      gmg::fail(GMG_E_INVAL, "right-hand side length differs from the request's DoF count");
    r->f_host.assign(f_nodal_host, f_nodal_host + n_f);
    r->rhs_given = true;
    if (r->state == gmg::kWaitRhs) gmg::push_ready(S, r);
    return 0;
  });
}

int gmg_server_poll(gmg_server h, uint64_t id, int32_t* state, int32_t* status) {
  return sguard([&] {
    if (!h || !state || !status) gmg::fail(GMG_E_INVAL, "null argument");
    Server& S = *h->S;
    std::lock_guard<std::mutex> lk(S.mu);
    auto it = S.all.find(id);
    if (it == S.all.end()) gmg::fail(GMG_E_INVAL, "unknown request id");
    *state = it->second->state;
    *status = it->second->status;
    return 0;
  });
}

int gmg_server_wait(gmg_server h, uint64_t id, double timeout_s) {
  return sguard([&] {
    if (!h) gmg::fail(GMG_E_INVAL, "null argument");
    Server& S = *h->S;
    std::unique_lock<std::mutex> lk(S.mu);
    auto it = S.all.find(id);
    if (it == S.all.end()) gmg::fail(GMG_E_INVAL, "unknown request id");
    gmg::Request* r = it->second.get();
    bool ok = S.cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s),
                                 [&] { return r->state == gmg::kDone || r->state == gmg::kFailed; });
    if (!ok) gmg::fail(GMG_E_STATE, "timeout waiting for request");
    return 0;
  });
}

int gmg_server_result(gmg_server h, uint64_t id, double* u_host, int64_t* n_dofs, int32_t* iterations,
                      double* history, gmg_timing* t) {
  return sguard([&] {
    if (!h) gmg::fail(GMG_E_INVAL, "null argument");
    Server& S = *h->S;
    std::lock_guard<std::mutex> lk(S.mu);
    auto it = S.all.find(id);
    if (it == S.all.end()) gmg::fail(GMG_E_INVAL, "unknown request id");
    gmg::Request* r = it->second.get();
    if (r->state == gmg::kFailed) {
      gmg::set_last_error(r->error);
      if (t) *t = r->t;
      return r->status;
    }
    if (r->state != gmg::kDone) gmg::fail(GMG_E_STATE, "request not finished");
    if (n_dofs) *n_dofs = r->n_dofs;
    if (u_host && r->n_dofs > 0) std::memcpy(u_host, r->u_pin, size_t(r->n_dofs) * sizeof(double));
    if (iterations) *iterations = r->iterations;
    if (history) std::memcpy(history, r->hist.data(), r->hist.size() * sizeof(double));
    if (t) *t = r->t;
    return r->status;
  });
}

int gmg_server_release(gmg_server h, uint64_t id) {
  return sguard([&] {
    if (!h) gmg::fail(GMG_E_INVAL, "null argument");
    Server& S = *h->S;
    std::lock_guard<std::mutex> lk(S.mu);
    auto it = S.all.find(id);
    if (it == S.all.end()) gmg::fail(GMG_E_INVAL, "unknown request id");
    if (it->second->state != gmg::kDone && it->second->state != gmg::kFailed)
      gmg::fail(GMG_E_STATE, "request still in flight");
    S.all.erase(it);
    return 0;
  });
}

int gmg_server_stats(gmg_server h, gmg_server_stats_t* o) {
  return sguard([&] {
    if (!h || !o) gmg::fail(GMG_E_INVAL, "null argument");
    Server& S = *h->S;
    std::lock_guard<std::mutex> lk(S.mu);
    o->queued = (int64_t)(S.setup_q.size() + S.ready_q.size());
    o->running = (int64_t)(S.running.size() + S.bind_q.size() + S.copying.size());
    o->completed = S.completed;
    o->failed = S.failed;
    o->arena_used = S.arena.used();
    o->arena_peak = S.arena.peak();
    o->arena_bytes = S.arena.size();
    o->dofs_done = S.dofs_done;
    o->clock = S.now();
    o->iterations = S.iterations;
    o->batched_iterations = S.batched_iterations;
    o->batches = S.batches;
    return 0;
  });
}

int gmg_server_hold(gmg_server h, int hold) {
  return sguard([&] {
    if (!h) gmg::fail(GMG_E_INVAL, "null argument");
    h->S->hold = hold != 0;
    return 0;
  });
}

int gmg_server_set_batching(gmg_server h, int enable) {
  return sguard([&] {
    if (!h) gmg::fail(GMG_E_INVAL, "null argument");
    Server& S = *h->S;
    std::lock_guard<std::mutex> lk(S.mu);
    S.batching = enable != 0;
    return 0;
  });
}

int gmg_server_destroy(gmg_server h) {
  if (!h) return 0;
  Server& S = *h->S;
  {
    std::lock_guard<std::mutex> lk(S.mu);
    S.stop = true;
    S.cv_work.notify_all();
  }
  for (auto& t : S.workers) t.join();
  if (S.sched.joinable()) S.sched.join();
  for (auto s : S.streams) {
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
  }
  if (S.bstream) {
    (void)hipStreamSynchronize(S.bstream);
    (void)hipStreamDestroy(S.bstream);
  }
  if (S.ev_batch) (void)hipEventDestroy(S.ev_batch);
  for (int i = 0; i < 2; ++i) {
    if (S.ev_stage[i]) (void)hipEventDestroy(S.ev_stage[i]);
    if (S.h_stage[i]) (void)hipHostFree(S.h_stage[i]);
  }
  delete h;  // requests free their pinned buffers and events
  return 0;
}

}  // extern "C"
