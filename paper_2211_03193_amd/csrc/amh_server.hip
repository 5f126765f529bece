// amh_server.hip -- continuous-batching request loop for folding jobs (host code).
//
// Jobs (one protein each: a distogram table, a run configuration with its own
// Philox key, a target energy) are queued by amh_submit and admitted in arrival
// order while the device memory they need fits the budget and a slot is free.
// Every amh_server_step advances all admitted jobs together -- one batched launch
// (amh_batch_sweep) over jobs of different lengths -- then reads back each job's
// counters, retires the jobs that reached their target or their last sweep, and
// admits waiting ones into the freed memory.  Chain state stays resident on the
// device between steps.  A job's sweeps do not depend on which other jobs share
// its launches, so its result is the same alone and in the mix.
//
// The server is a client of the library's own C ABI (amh_init, amh_batch_*,
// amh_get_state); it adds no kernels.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <deque>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "amh.h"

#include "amh_error.h"

static_assert(sizeof(amh_server_opts) == 32, "amh_server_opts layout");
static_assert(sizeof(amh_job) == 144, "amh_job layout");
static_assert(sizeof(amh_job_trace) == 56, "amh_job_trace layout");
static_assert(sizeof(amh_job_status) == 72, "amh_job_status layout");

namespace {

using amh::sfail;

double now_s() {
  using clk = std::chrono::steady_clock;
  return std::chrono::duration<double>(clk::now().time_since_epoch()).count();
}

// Device bytes a context of this configuration holds: the padded table and its
// deviation copy (rows of n_bins + 2 floats rounded up to 16 bytes), and the chain
// state (torsions, best torsions, float64 atoms, energies, counters).
int64_t job_bytes(const amh_config& c) {
  const int64_t P = (int64_t)c.L * (c.L - 1) / 2;
  const int64_t stride = ((c.n_bins + 2) + 3) & ~3;
  const int64_t table = (2 * P + 1) * stride * 4;
  const int64_t state = (int64_t)c.n_chains * (2 * c.L * 8 * 2 + (int64_t)c.L * 12 * 8 + 2 * 8 + 4 * 8);
  return table + state;
}

struct Job {
  uint64_t id = 0;
  int64_t chunk = 1;           // sweeps per round
  amh_config cfg{};
  std::vector<float> y;        // host copy until admission
  double target = -INFINITY;
  amh_job_status st{};
  amh_ctx* ctx = nullptr;
  int64_t bytes = 0;
  std::vector<double> s_best;  // [C][2L] host copy at completion
  std::vector<double> v;       // [C][2]
  std::string error;
  bool traced = false;
  amh_job_trace trace{};
};

}  // namespace

struct amh_server {
  amh_server_opts o{};
  hipStream_t stream = nullptr;
  uint64_t next_id = 1;
  std::map<uint64_t, std::unique_ptr<Job>> jobs;
  std::deque<uint64_t> pending;
  std::vector<uint64_t> active;
  int64_t active_bytes = 0;
  amh_batch* batch = nullptr;
  std::vector<uint64_t> batch_members;   // job ids (a freed context's address can be reused)
  // read-back buffers (device and host) for counters and energies of active jobs
  int64_t* d_cnt = nullptr;
  double* d_v = nullptr;
  size_t cap_chains = 0;
  std::vector<int64_t> h_cnt;
  std::vector<double> h_v;
};

namespace {

#define SHIP(expr)                                                                   \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess) return sfail(AMH_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

amh_status lib_fail(amh_status st, const char* what) {
  const std::string msg = amh_last_error();
  return sfail(st, "%s: %s", what, msg.c_str());
}

void drop_batch(amh_server* s) {
  if (s->batch) (void)amh_batch_destroy(s->batch);
  s->batch = nullptr;
  s->batch_members.clear();
}

amh_status admit(amh_server* s, Job* j) {
  float* y_dev = nullptr;
  const size_t n = j->y.size();
  SHIP(hipMalloc(reinterpret_cast<void**>(&y_dev), sizeof(float) * (n ? n : 1)));
  hipError_t e = hipMemcpyAsync(y_dev, j->y.data(), sizeof(float) * n, hipMemcpyHostToDevice, s->stream);
  amh_status st = AMH_OK;
  if (e != hipSuccess) st = sfail(AMH_E_DEVICE, "table upload: %s", hipGetErrorString(e));
  if (st == AMH_OK) {
    st = amh_init(&j->cfg, y_dev, nullptr, s->stream, &j->ctx);   // synchronises the stream
    if (st != AMH_OK) j->error = amh_last_error();
  }
  (void)hipStreamSynchronize(s->stream);
  (void)hipFree(y_dev);
  if (st == AMH_OK && (st = amh_set_target(j->ctx, j->target)) != AMH_OK) j->error = amh_last_error();
  if (st == AMH_OK && j->traced &&
      (st = amh_set_trace(j->ctx, 1, &j->trace.chain, j->trace.dE_dev, j->trace.delta_dev,
                          j->trace.acc_dev, j->trace.capacity, j->trace.anchor_dev,
                          j->trace.anchor_capacity)) != AMH_OK)
    j->error = amh_last_error();
  if (st != AMH_OK) {
    if (j->ctx) (void)amh_destroy(j->ctx);
    j->ctx = nullptr;
    j->st.state = 3;
    j->st.t_done = now_s();
    return AMH_OK;   // the job failed, the server goes on
  }
  std::vector<float>().swap(j->y);
  j->st.state = 1;
  j->st.t_admit = now_s();
  s->active.push_back(j->id);
  s->active_bytes += j->bytes;
  return AMH_OK;
}

amh_status retire(amh_server* s, Job* j) {
  const size_t C = j->cfg.n_chains, n = 2 * (size_t)j->cfg.L;
  double* d_sb = nullptr;
  SHIP(hipMalloc(reinterpret_cast<void**>(&d_sb), sizeof(double) * C * n));
  amh_status st = amh_get_state(j->ctx, nullptr, d_sb, nullptr, nullptr, nullptr, nullptr);
  j->s_best.resize(C * n);
  if (st == AMH_OK) {
    hipError_t e = hipMemcpyAsync(j->s_best.data(), d_sb, sizeof(double) * C * n,
                                  hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) st = sfail(AMH_E_DEVICE, "best-state read-back: %s", hipGetErrorString(e));
  }
  (void)hipFree(d_sb);
  if (st != AMH_OK) return st;
  drop_batch(s);   // the batch borrows the context: never let it outlive it
  (void)amh_destroy(j->ctx);
  j->ctx = nullptr;
  j->st.state = 2;
  j->st.t_done = now_s();
  s->active_bytes -= j->bytes;
  return AMH_OK;
}

}  // namespace

extern "C" {

amh_status amh_server_create(const amh_server_opts* o, void* stream, amh_server** out) {
  if (!out) return sfail(AMH_E_INVAL, "out is NULL");
  *out = nullptr;
  if (!o) return sfail(AMH_E_INVAL, "opts is NULL");
  if (o->hbm_budget_bytes <= 0) return sfail(AMH_E_INVAL, "hbm_budget_bytes must be > 0");
  if (o->max_active < 1) return sfail(AMH_E_INVAL, "max_active=%d < 1", o->max_active);
  if (o->sweeps_per_round < 1) return sfail(AMH_E_INVAL, "sweeps_per_round=%d < 1", o->sweeps_per_round);
  if (o->plan < 0 || o->plan > 5) return sfail(AMH_E_INVAL, "plan=%d outside [0, 5]", o->plan);
  if (o->round_pairs < 0) return sfail(AMH_E_INVAL, "round_pairs < 0");
  amh_server* s = new amh_server;
  s->o = *o;
  s->stream = reinterpret_cast<hipStream_t>(stream);
  *out = s;
  return AMH_OK;
}

amh_status amh_submit(void* server, const void* job, uint64_t* job_id) {
  amh_server* s = static_cast<amh_server*>(server);
  const amh_job* jb = static_cast<const amh_job*>(job);
  if (!s || !jb || !job_id) return sfail(AMH_E_INVAL, "NULL argument");
  const amh_config& c = jb->cfg;
  if (c.L < 2 || c.L > 1024 || c.n_bins < 4 || c.n_bins > 64 || c.n_chains < 1)
    return sfail(AMH_E_INVAL, "job configuration out of range");
  if (!jb->y_host) return sfail(AMH_E_INVAL, "job table is NULL");
  if (std::isnan(jb->target)) return sfail(AMH_E_INVAL, "target is NaN");
  if (jb->trace) {
    const amh_job_trace& tr = *jb->trace;
    if (tr.chain < 0 || tr.chain >= c.n_chains) return sfail(AMH_E_INVAL, "trace chain out of range");
    if (!tr.dE_dev || !tr.delta_dev || !tr.acc_dev || tr.capacity < 1)
      return sfail(AMH_E_INVAL, "trace buffers missing or capacity < 1");
    if (tr.anchor_dev && tr.anchor_capacity < 1) return sfail(AMH_E_INVAL, "anchor capacity < 1");
  }
  auto j = std::make_unique<Job>();
  if (jb->trace) {
    j->traced = true;
    j->trace = *jb->trace;
  }
  j->id = s->next_id++;
  j->cfg = c;
  j->target = jb->target;
  j->bytes = job_bytes(c);
  j->st.bytes = j->bytes;
  j->chunk = s->o.sweeps_per_round;
  if (s->o.round_pairs > 0) {   // pair evaluations of R sweeps of all chains of this job
    const double L = c.L, h = c.window_d / 2;
    const int ge = c.global_every;
    const double fg = ge > 0 ? (double)(c.n_global < 1 ? 1 : c.n_global) / ge : 0.0;
    const double per_sweep = (L * L * L / 3.0 * fg + 2.0 * L * h * (h + 1) * (1.0 - fg)) * c.n_chains;
    const double k = std::floor((double)s->o.round_pairs / (per_sweep * s->o.sweeps_per_round));
    j->chunk *= (int64_t)std::min(64.0, std::max(1.0, k));
  }
  if (j->bytes > s->o.hbm_budget_bytes)
    return sfail(AMH_E_BUSY, "job needs %lld bytes, more than the whole budget (%lld)",
                 (long long)j->bytes, (long long)s->o.hbm_budget_bytes);
  const size_t P = (size_t)c.L * (c.L - 1) / 2;
  j->y.assign(jb->y_host, jb->y_host + P * c.n_bins);
  j->st.state = 0;
  j->st.sweeps_to_target = -1;
  j->st.best_V = INFINITY;
  j->st.t_submit = now_s();
  j->st.t_admit = j->st.t_done = j->st.t_target = -1.0;
  *job_id = j->id;
  s->pending.push_back(j->id);
  s->jobs[j->id] = std::move(j);
  return AMH_OK;
}

amh_status amh_server_step(amh_server* s, int32_t* n_active, int32_t* n_pending) {
  if (!s) return sfail(AMH_E_INVAL, "server is NULL");
  // admission: arrival order, while a slot is free and the memory fits
  while (!s->pending.empty() && (int)s->active.size() < s->o.max_active) {
    Job* j = s->jobs[s->pending.front()].get();
    if (s->active_bytes + j->bytes > s->o.hbm_budget_bytes) break;
    s->pending.pop_front();
    amh_status st = admit(s, j);
    if (st != AMH_OK) return st;
  }
  if (!s->active.empty()) {
    // every active job advances its own chunk of sweeps (fewer at the end of its run)
    std::vector<amh_ctx*> ctxs;
    std::vector<uint64_t> ids;
    std::vector<int64_t> nsw;
    std::vector<Job*> act;
    for (uint64_t id : s->active) {
      Job* j = s->jobs[id].get();
      act.push_back(j);
      ctxs.push_back(j->ctx);
      ids.push_back(id);
      const int64_t left = j->cfg.total_sweeps - j->st.sweeps;
      nsw.push_back(std::min(left, j->chunk));
    }
    if (ids != s->batch_members || !s->batch) {   // membership changed: regroup the launch
      drop_batch(s);
      if (amh_batch_create(ctxs.data(), (int32_t)ctxs.size(), &s->batch) != AMH_OK)
        return lib_fail(AMH_E_DEVICE, "amh_batch_create");
      s->batch_members = ids;
      if (amh_batch_set_plan(s->batch, s->o.plan) != AMH_OK) return lib_fail(AMH_E_DEVICE, "amh_batch_set_plan");
    }
    if (amh_batch_sweep_each(s->batch, nsw.data()) != AMH_OK) return lib_fail(AMH_E_DEVICE, "amh_batch_sweep_each");
    for (size_t q = 0; q < act.size(); ++q) act[q]->st.sweeps += nsw[q];
    // read back counters and energies of every active job
    size_t total = 0;
    for (Job* j : act) total += j->cfg.n_chains;
    if (total > s->cap_chains) {
      (void)hipFree(s->d_cnt);
      (void)hipFree(s->d_v);
      s->d_cnt = nullptr;
      s->d_v = nullptr;
      s->cap_chains = 0;
      SHIP(hipMalloc(reinterpret_cast<void**>(&s->d_cnt), sizeof(int64_t) * 4 * total));
      SHIP(hipMalloc(reinterpret_cast<void**>(&s->d_v), sizeof(double) * 2 * total));
      s->cap_chains = total;
    }
    s->h_cnt.resize(4 * total);
    s->h_v.resize(2 * total);
    size_t off = 0;
    for (Job* j : act) {
      if (amh_get_state(j->ctx, nullptr, nullptr, s->d_v + 2 * off, s->d_cnt + 4 * off, nullptr,
                        nullptr) != AMH_OK)
        return lib_fail(AMH_E_DEVICE, "amh_get_state");
      off += j->cfg.n_chains;
    }
    SHIP(hipMemcpyAsync(s->h_cnt.data(), s->d_cnt, sizeof(int64_t) * 4 * total, hipMemcpyDeviceToHost, s->stream));
    SHIP(hipMemcpyAsync(s->h_v.data(), s->d_v, sizeof(double) * 2 * total, hipMemcpyDeviceToHost, s->stream));
    SHIP(hipStreamSynchronize(s->stream));
    const double t_now = now_s();
    off = 0;
    std::vector<uint64_t> still;
    for (Job* j : act) {
      const int C = j->cfg.n_chains;
      int64_t ttt = -1;
      double best = INFINITY;
      for (int c = 0; c < C; ++c) {
        const int64_t q = s->h_cnt[4 * (off + c) + 2];
        if (q >= 0 && (ttt < 0 || q < ttt)) ttt = q;
        best = std::fmin(best, s->h_v[2 * (off + c) + 1]);
      }
      j->v.assign(s->h_v.begin() + 2 * off, s->h_v.begin() + 2 * (off + C));
      off += C;
      j->st.best_V = best;
      if (ttt >= 0 && j->st.sweeps_to_target < 0) {
        j->st.sweeps_to_target = ttt;
        j->st.reached = 1;
        j->st.t_target = t_now;
      }
      if (amh_poll(j->ctx) != AMH_OK) {
        j->error = amh_last_error();
        drop_batch(s);
        (void)amh_destroy(j->ctx);
        j->ctx = nullptr;
        j->st.state = 3;
        j->st.t_done = t_now;
        s->active_bytes -= j->bytes;
        continue;
      }
      if (j->st.reached || j->st.sweeps >= j->cfg.total_sweeps) {
        amh_status st = retire(s, j);
        if (st != AMH_OK) return st;
        continue;
      }
      still.push_back(j->id);
    }
    s->active.swap(still);
  }
  if (n_active) *n_active = (int32_t)s->active.size();
  if (n_pending) *n_pending = (int32_t)s->pending.size();
  return AMH_OK;
}

amh_status amh_server_job(amh_server* s, uint64_t job_id, amh_job_status* out, double* s_best_host,
                          double* v_host) {
  if (!s || !out) return sfail(AMH_E_INVAL, "NULL argument");
  auto it = s->jobs.find(job_id);
  if (it == s->jobs.end()) return sfail(AMH_E_INVAL, "unknown job %llu", (unsigned long long)job_id);
  const Job* j = it->second.get();
  *out = j->st;
  if (s_best_host) {
    if (j->st.state != 2) return sfail(AMH_E_BUSY, "job %llu has not finished", (unsigned long long)job_id);
    std::memcpy(s_best_host, j->s_best.data(), sizeof(double) * j->s_best.size());
  }
  if (v_host) {
    if (j->v.empty()) return sfail(AMH_E_BUSY, "job %llu has not run yet", (unsigned long long)job_id);
    std::memcpy(v_host, j->v.data(), sizeof(double) * j->v.size());
  }
  return AMH_OK;
}

amh_status amh_server_destroy(amh_server* s) {
  if (!s) return AMH_OK;
  (void)hipStreamSynchronize(s->stream);
  drop_batch(s);
  for (auto& kv : s->jobs)
    if (kv.second->ctx) (void)amh_destroy(kv.second->ctx);
  (void)hipFree(s->d_cnt);
  (void)hipFree(s->d_v);
  delete s;
  return AMH_OK;
}

}  // extern "C"
