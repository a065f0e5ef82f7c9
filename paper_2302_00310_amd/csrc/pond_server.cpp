// Serving loop of libpond.so: continuous batching of independent solves.
//
// A server thread owns a device arena and a stream.  Requests are queued by
// pond_submit (host copies of their inputs, no GPU work) and admitted first
// come, first served as soon as their footprint fits a first-fit free list
// over the arena and a batch slot is free.  Every iteration advances all
// resident solves together by K steps: per step, one batched step kernel per
// solve kind covers the tiles of the mixed-precision 2D solves (a device
// table maps blocks to solves), after each multiscale solve's switch and each
// walled solve's ghost layers; FP64, 1D and D2Q25 solves add their own step
// launches.  The K steps are captured once per change of the resident set
// into a HIP graph that is replayed while the set is unchanged.  Solves that reach
// their step count are retired: moments copied to host, status recorded
// (a non-physical state fails that solve only), arena released.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
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
#include <vector>

#include "../../include/pond.h"
#include "pond_internal.h"
#include "pond_state.h"

using namespace pond;

namespace {

using Clock = std::chrono::steady_clock;

constexpr int kChunk = 16;  // steps per iteration (fewer when a solve finishes earlier)

struct Job {
  uint64_t id = 0, tag = 0;
  pond_config cfg{};
  std::vector<double> rho, ux, uy, p;
  int nsteps = 0, remaining = 0;
  int status = POND_PENDING;
  double t_submit = 0.0, t_admit = -1.0, t_done = -1.0;
  size_t off = 0, bytes = 0;
  pond_state* st = nullptr;
  std::vector<double> out;  // rho, ux, uy, T planes after completion
};

// First-fit free list over [0, size), 256-byte granules.
class FreeList {
 public:
  void reset(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
  }
  bool take(size_t n, size_t* off) {
    n = (n + 255) & ~size_t(255);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      *off = it->first;
      const size_t rest = it->second - n, at = it->first + n;
      free_.erase(it);
      if (rest) free_[at] = rest;
      return true;
    }
    return false;
  }
  void give(size_t off, size_t n) {
    n = (n + 255) & ~size_t(255);
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

 private:
  std::map<size_t, size_t> free_;
};

}  // namespace

struct pond_server {
  char* arena = nullptr;
  size_t bytes = 0, usable = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int max_active = 0;
  BatchEntry* dev_tab = nullptr;
  BatchEntry* host_tab = nullptr;  // pinned
  FreeList alloc;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Job*> queue;
  std::vector<Job*> active;
  std::unordered_map<uint64_t, std::unique_ptr<Job>> jobs;
  std::thread th;
  std::atomic<bool> stop{false};
  uint64_t next_id = 1;
  Clock::time_point t0;
  // graph cache for the current resident set: key = (K, parity of the first step)
  std::map<std::pair<int, int>, hipGraphExec_t> graphs;
  int n_tab = 0, total_tiles = 0, phase = 0;
  unsigned tf_mask = 0;  // step-kernel kinds present in the resident set (bit per kind_of)
  // counters for pond_server_stats (written by the server thread under mu)
  double st_admit = 0.0, st_table = 0.0, st_capture = 0.0, st_retire = 0.0;
  double st_cell_updates = 0.0, st_chunks = 0.0, st_changes = 0.0, st_captures = 0.0;
  double st_gpu = 0.0;  // event-timed GPU seconds of the step chunks
  // chunks in flight: (start, end) events; finished ones are timed and recycled
  std::deque<std::pair<hipEvent_t, hipEvent_t>> inflight;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> spare;
  int device = 0;

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

namespace {

void drop_graphs(pond_server* S) {
  for (auto& kv : S->graphs) hipGraphExecDestroy(kv.second);
  S->graphs.clear();
}

// Mixed-precision 2D solves on the D2Q16 / D2Q9 / multiscale f-lattices
// share the batched step; the others (FP64, 1D, D2Q25) run their own step
// launches in the same graph.
bool batched(const pond_state* s) { return s->cfg.dim == 2 && !s->L.fp64 && !s->L.q25; }

int tiles_of(const pond_config& c) {
  return ((c.nx + kTX2 - 1) / kTX2) * ((c.ny + kTY2 - 1) / kTY2);
}

// Rebuild the device table of resident solves.
int upload_table(pond_server* S) {
  const double t = S->now();
  struct Acc {
    pond_server* S;
    double t;
    ~Acc() {
      std::lock_guard<std::mutex> lk(S->mu);
      S->st_table += S->now() - t;
      S->st_changes += 1.0;
    }
  } acc{S, t};
  drop_graphs(S);
  int tile = 0;
  for (size_t k = 0; k < S->active.size(); ++k) {
    pond_state* s = S->active[k]->st;
    BatchEntry& e = S->host_tab[k];
    for (int par = 0; par < 2; ++par) {
      const int in = par ? 1 - s->cur : s->cur;
      e.args[par] = s->args;
      e.args[par].n_in = s->n[in];
      e.args[par].n_out = s->n[1 - in];
      e.args[par].U_in = s->U[in];
      e.args[par].U_out = s->U[1 - in];
      e.args[par].lat_in = s->lat[in];
      e.args[par].lat_out = s->lat[1 - in];
      if (s->cfg.lattice == POND_D2Q9_D2Q16) {
        e.args[par].q16_in = s->q16 + in;
        e.args[par].q16_out = s->q16 + 1 - in;
      }
    }
    e.tile_begin = tile;
    e.tiles = batched(s) ? tiles_of(s->cfg) : 0;
    tile += e.tiles;
  }
  S->n_tab = int(S->active.size());
  S->total_tiles = tile;
  S->tf_mask = 0;
  for (Job* j : S->active) {
    if (!batched(j->st)) continue;
    S->tf_mask |= 1u << kind_of(j->cfg.transform, j->st->args.ms);
    // a multiscale step may run in the D2Q9 kernel (all cells on D2Q9)
    if (j->cfg.lattice == POND_D2Q9_D2Q16) S->tf_mask |= 1u << kind_of(POND_TF_GRAD, 3);
  }
  S->phase = 0;
  hipError_t err = hipMemcpyAsync(S->dev_tab, S->host_tab, sizeof(BatchEntry) * S->n_tab,
                                  hipMemcpyHostToDevice, S->stream);
  if (err == hipSuccess) err = hipStreamSynchronize(S->stream);
  return err == hipSuccess ? POND_OK : hip_fail(err, "batch table upload");
}

// K batched steps, captured into a graph on first use for this resident set.
int run_steps(pond_server* S, int K) {
  const int par0 = S->phase & 1;
  auto key = std::make_pair(K, par0);
  auto it = S->graphs.find(key);
  if (it == S->graphs.end()) {
    const double t = S->now();
    hipError_t err = hipStreamBeginCapture(S->stream, hipStreamCaptureModeThreadLocal);
    if (err != hipSuccess) return hip_fail(err, "hipStreamBeginCapture");
    int rc = POND_OK;
    for (int j = 0; j < K && rc == POND_OK; ++j) {
      const int par = (par0 + j) & 1;
      for (size_t k = 0; k < S->active.size() && rc == POND_OK; ++k) {
        pond_state* s = S->active[k]->st;
        const StepArgs& a = S->host_tab[k].args[par];
        const int in = a.n_in == s->n[1] ? 1 : 0;  // the buffer this step reads
        if (!batched(s)) {
          rc = step_launches(s, in, S->stream);
          continue;
        }
        // from the ledger at the start of the step: the f-lattice map of each
        // multiscale solve, the ghost layers of each walled one
        hipError_t e = hipSuccess;
        if (s->cfg.lattice == POND_D2Q9_D2Q16)
          e = launch_switch(a, a.U_in, s->cfg.ms_threshold, s->cfg.gamma, s->q16 + 1 - in,
                            s->theta, s->lat[1 - in], S->stream);
        if (e == hipSuccess && s->L.wall_bytes)
          e = launch_wall_ghosts(false, a, s->wU, s->wN, S->stream);
        if (e != hipSuccess) rc = hip_fail(e, "switch / wall-ghost launch");
      }
      if (rc == POND_OK && S->total_tiles > 0) {
        const hipError_t e = launch_step_batch(false, S->tf_mask, S->dev_tab, S->n_tab,
                                               S->total_tiles, par, S->stream);
        if (e != hipSuccess) rc = hip_fail(e, "batched step launch");
      }
    }
    hipGraph_t g = nullptr;
    err = hipStreamEndCapture(S->stream, &g);
    if (err == hipSuccess && rc != POND_OK) {
      hipGraphDestroy(g);
      return rc;
    }
    if (err != hipSuccess) return hip_fail(err, "hipStreamEndCapture");
    hipGraphExec_t ex = nullptr;
    err = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (err != hipSuccess) return hip_fail(err, "hipGraphInstantiate");
    it = S->graphs.emplace(key, ex).first;
    std::lock_guard<std::mutex> lk(S->mu);
    S->st_capture += S->now() - t;
    S->st_captures += 1.0;
  }
  std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
  if (!S->spare.empty()) {
    ev = S->spare.back();
    S->spare.pop_back();
  } else if (hipEventCreate(&ev.first) != hipSuccess || hipEventCreate(&ev.second) != hipSuccess) {
    return hip_fail(hipErrorOutOfMemory, "hipEventCreate");
  }
  hipEventRecord(ev.first, S->stream);
  hipError_t err = hipGraphLaunch(it->second, S->stream);
  if (err != hipSuccess) return hip_fail(err, "hipGraphLaunch");
  hipEventRecord(ev.second, S->stream);
  S->inflight.push_back(ev);
  S->phase += K;
  double cu = 0.0;
  for (Job* j : S->active) cu += double(j->cfg.nx) * j->cfg.ny * K;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->st_cell_updates += cu;
    S->st_chunks += 1.0;
  }
  for (Job* j : S->active) {
    j->remaining -= K;
    j->st->cur ^= (K & 1);
    j->st->nstep += K;
  }
  return POND_OK;
}

void finish(pond_server* S, Job* j, int status) {
  if (j->st) {
    pond_destroy(j->st);
    j->st = nullptr;
  }
  std::lock_guard<std::mutex> lk(S->mu);
  j->t_done = S->now();
  j->status = status;  // published under the lock: pond_poll reads it there
  S->alloc.give(j->off, j->bytes);
  S->cv.notify_all();
}

// Time the chunks that have finished (all of them when wait is set).
void harvest(pond_server* S, bool wait) {
  while (!S->inflight.empty()) {
    auto ev = S->inflight.front();
    if (wait) hipEventSynchronize(ev.second);
    else if (hipEventQuery(ev.second) != hipSuccess) break;
    float ms = 0.0f;
    hipEventElapsedTime(&ms, ev.first, ev.second);
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->st_gpu += 1e-3 * ms;
    }
    S->inflight.pop_front();
    S->spare.push_back(ev);
  }
}

void serve(pond_server* S) {
  hipSetDevice(S->device);
  std::vector<Job*> admit;
  bool changed = false;
  for (;;) {
    harvest(S, false);
    {
      std::unique_lock<std::mutex> lk(S->mu);
      while (!S->stop && !S->queue.empty() &&
             int(S->active.size() + admit.size()) < S->max_active) {
        Job* j = S->queue.front();
        size_t off = 0;
        if (!S->alloc.take(j->bytes, &off)) break;  // first come, first served: wait for memory
        j->off = off;
        S->queue.pop_front();
        admit.push_back(j);
      }
      if (S->active.empty() && admit.empty()) {
        if (S->stop) break;
        S->cv.wait_for(lk, std::chrono::milliseconds(2));
        continue;
      }
    }
    // admission: state in the job's arena region, comoving equilibrium on device
    const double t_adm = S->now();
    for (Job* j : admit) {
      pond_state* st = nullptr;
      int rc = pond_create(&j->cfg, S->arena + j->off, j->bytes, S->stream, &st);
      if (rc == POND_OK)
        rc = pond_init_fields(st, j->rho.data(), j->ux.data(), j->uy.data(), j->p.data());
      j->st = st;
      std::vector<double>().swap(j->rho);
      std::vector<double>().swap(j->ux);
      std::vector<double>().swap(j->uy);
      std::vector<double>().swap(j->p);
      if (rc != POND_OK) {
        finish(S, j, rc);
        continue;
      }
      j->t_admit = S->now();
      j->remaining = j->nsteps;
      if (j->remaining == 0) {
        j->out.assign(4 * size_t(j->cfg.nx) * j->cfg.ny, 0.0);
        const size_t n = size_t(j->cfg.nx) * j->cfg.ny;
        const int mrc = pond_moments(st, j->out.data(), j->out.data() + n, j->out.data() + 2 * n,
                                     j->out.data() + 3 * n);
        finish(S, j, mrc);
        continue;
      }
      S->active.push_back(j);
      changed = true;
    }
    if (!admit.empty()) {
      std::lock_guard<std::mutex> lk(S->mu);
      S->st_admit += S->now() - t_adm;
    }
    admit.clear();
    if (S->active.empty()) continue;
    if (changed) {
      if (upload_table(S) != POND_OK) {
        for (Job* j : S->active) finish(S, j, POND_ERR_DEVICE);
        S->active.clear();
        continue;
      }
      changed = false;
    }
    harvest(S, false);
    int K = kChunk;
    for (Job* j : S->active) K = std::min(K, j->remaining);
    if (run_steps(S, K) != POND_OK) {
      for (Job* j : S->active) finish(S, j, POND_ERR_DEVICE);
      S->active.clear();
      changed = true;
      continue;
    }
    // retire the solves that reached their step count
    bool any = false;
    for (Job* j : S->active) any |= j->remaining == 0;
    if (!any) continue;
    std::vector<Job*> keep;
    const double t_ret = S->now();
    for (Job* j : S->active) {
      if (j->remaining > 0) {
        keep.push_back(j);
        continue;
      }
      const size_t n = size_t(j->cfg.nx) * j->cfg.ny;
      j->out.assign(4 * n, 0.0);
      const int rc = pond_moments(j->st, j->out.data(), j->out.data() + n, j->out.data() + 2 * n,
                                  j->out.data() + 3 * n);
      finish(S, j, rc);
    }
    S->active.swap(keep);
    changed = true;
    std::lock_guard<std::mutex> lk(S->mu);
    S->st_retire += S->now() - t_ret;
  }
}

}  // namespace

extern "C" {

int pond_server_create(void* dev_arena, size_t bytes, void* hip_stream, int max_active,
                       pond_server** out) {
  if (!out) return fail(POND_ERR_INVALID, "null output handle");
  *out = nullptr;
  if (max_active < 1 || max_active > 4096) return fail(POND_ERR_INVALID, "max_active must lie in 1..4096");
  if (!dev_arena || (reinterpret_cast<uintptr_t>(dev_arena) & 255))
    return fail(POND_ERR_INVALID, "arena must be a 256-byte aligned device pointer");
  const size_t tab = (sizeof(BatchEntry) * size_t(max_active) + 255) & ~size_t(255);
  if (bytes <= tab) return fail(POND_ERR_NOMEM, "arena smaller than the batch table");
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::unique_ptr<pond_server> S(new pond_server());
  S->device = dev;
  S->arena = static_cast<char*>(dev_arena) + tab;
  S->bytes = bytes;
  S->usable = bytes - tab;
  S->dev_tab = static_cast<BatchEntry*>(dev_arena);
  S->max_active = max_active;
  // graph capture needs a stream other than the legacy default one
  if (hip_stream) {
    S->stream = static_cast<hipStream_t>(hip_stream);
  } else {
    e = hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "hipStreamCreateWithFlags");
    S->own_stream = true;
  }
  e = hipHostMalloc(reinterpret_cast<void**>(&S->host_tab), sizeof(BatchEntry) * size_t(max_active));
  if (e != hipSuccess) return hip_fail(e, "hipHostMalloc");
  S->alloc.reset(S->usable);
  S->t0 = Clock::now();
  pond_server* raw = S.release();
  raw->th = std::thread(serve, raw);
  *out = raw;
  return POND_OK;
}

int pond_submit(pond_server* S, const pond_request* req, uint64_t* id) {
  if (!S || !req || !id) return fail(POND_ERR_INVALID, "null argument");
  const pond_config& c = req->cfg;
  int rc = validate(&c);
  if (rc) return rc;
  if (req->nsteps < 0) return fail(POND_ERR_INVALID, "nsteps must be >= 0");
  if (!req->rho || !req->ux || !req->uy || !req->p) return fail(POND_ERR_INVALID, "null field");
  const size_t need = layout_of(&c).total;
  if (need > S->usable) return fail(POND_ERR_REJECTED, "solve footprint exceeds the whole arena");
  const size_t n = size_t(c.nx) * c.ny;
  std::unique_ptr<Job> j(new Job());
  j->cfg = c;
  j->tag = req->tag;
  j->nsteps = req->nsteps;
  j->bytes = need;
  j->rho.assign(req->rho, req->rho + n);
  j->ux.assign(req->ux, req->ux + n);
  j->uy.assign(req->uy, req->uy + n);
  j->p.assign(req->p, req->p + n);
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->stop) return fail(POND_ERR_INVALID, "server is stopping");
  j->id = S->next_id++;
  j->t_submit = S->now();
  *id = j->id;
  S->queue.push_back(j.get());
  S->jobs.emplace(j->id, std::move(j));
  S->cv.notify_all();
  return POND_OK;
}

int pond_poll(pond_server* S, uint64_t id, pond_result* res) {
  if (!S || !res) return fail(POND_ERR_INVALID, "null argument");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->jobs.find(id);
  if (it == S->jobs.end()) return fail(POND_ERR_INVALID, "unknown request id");
  Job* j = it->second.get();
  if (j->status == POND_PENDING) return POND_PENDING;
  res->status = j->status;
  res->t_submit = j->t_submit;
  res->t_admit = j->t_admit;
  res->t_done = j->t_done;
  res->tag = j->tag;
  const size_t n = size_t(j->cfg.nx) * j->cfg.ny;
  if (j->out.size() == 4 * n) {
    double* dst[4] = {res->rho, res->ux, res->uy, res->T};
    for (int q = 0; q < 4; ++q)
      if (dst[q]) std::memcpy(dst[q], j->out.data() + q * n, n * sizeof(double));
  }
  const int status = j->status;
  S->jobs.erase(it);
  return status;
}

int pond_server_stats(pond_server* S, double out[9]) {
  if (!S || !out) return fail(POND_ERR_INVALID, "null server or output");
  std::lock_guard<std::mutex> lk(S->mu);
  out[0] = S->now();
  out[1] = S->st_cell_updates;
  out[2] = S->st_chunks;
  out[3] = S->st_changes;
  out[4] = S->st_admit;
  out[5] = S->st_retire;
  out[6] = S->st_table;
  out[7] = S->st_capture;
  out[8] = S->st_gpu;
  return POND_OK;
}

int pond_server_destroy(pond_server* S) {
  if (!S) return POND_OK;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    // queued work is dropped; resident solves finish
    for (Job* j : S->queue) {
      j->status = POND_ERR_INVALID;
      j->t_done = S->now();
    }
    S->queue.clear();
    S->cv.notify_all();
  }
  if (S->th.joinable()) S->th.join();
  harvest(S, true);
  for (auto& ev : S->spare) {
    hipEventDestroy(ev.first);
    hipEventDestroy(ev.second);
  }
  drop_graphs(S);
  if (S->host_tab) hipHostFree(S->host_tab);
  hipStreamSynchronize(S->stream);
  if (S->own_stream) hipStreamDestroy(S->stream);
  delete S;
  return POND_OK;
}

}  // extern "C"
