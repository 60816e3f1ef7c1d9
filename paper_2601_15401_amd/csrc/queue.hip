// Work queue over job-table plans: FIFO admission by device memory, one
// plan per parameter set and launch, completion by HIP events.
#include <string.h>

#include <algorithm>
#include <deque>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "arena.h"
#include "internal.h"

using namespace mick;

namespace {

constexpr int kMaxSets = 16;
constexpr int kTableEntries = 65536;  // job-table entries of all running groups

struct Group {  // one launched plan
  hipEvent_t done = nullptr;
  std::vector<uint64_t> ids;
  std::vector<int*> status;                       // the jobs' status words (NULL: none)
  std::vector<std::pair<size_t, size_t>> blocks;  // workspace arena (offset, bytes)
  std::pair<size_t, size_t> table;                // table area (offset, bytes)
  mick_plan* plan = nullptr;                      // holds the source of the table copy
  ~Group() { mick_plan_destroy(plan); }
};

}  // namespace

struct mick_queue {
  std::vector<const mick_params*> prms;
  std::vector<const mick_keys*> keys;
  std::vector<int> set_order;  // sets by ring degree, smallest first
  Allocator alloc;
  char* base = nullptr;  // workspace arena, then the table area
  size_t capacity = 0;
  Arena arena{0};
  char* tables = nullptr;
  Arena tarena{0};
  std::deque<mick_qjob> pending;
  std::deque<std::unique_ptr<Group>> running;
  std::deque<uint64_t> done;  // completed, not yet reported
  int device = 0;
};

namespace {

size_t qjob_bytes(const mick_queue* q, const mick_qjob& jb) { return job_ws_bytes(q->prms[jb.set], jb.k, jb.level); }

// Moves completed groups to the done list and frees their blocks.  With
// `wait`, first waits for the oldest running group.
int reap(mick_queue* q, bool wait) {
  if (wait && !q->running.empty()) MICK_HIP(hipEventSynchronize(q->running.front()->done), "queue wait");
  for (auto it = q->running.begin(); it != q->running.end();) {
    const hipError_t e = hipEventQuery((*it)->done);
    if (e == hipErrorNotReady) {
      ++it;
      continue;
    }
    if (e != hipSuccess) return hip_error(e, "queue event");
    for (auto& b : (*it)->blocks) q->arena.give(b.first, b.second);
    q->tarena.give((*it)->table.first, (*it)->table.second);
    for (uint64_t id : (*it)->ids) q->done.push_back(id);
    for (int* st : (*it)->status)
      if (st) *st = MICK_OK;
    (void)hipEventDestroy((*it)->done);
    it = q->running.erase(it);
  }
  return MICK_OK;
}

}  // namespace

extern "C" {

int mick_queue_create(const mick_params* const* prms, const mick_keys* const* keys, int n_sets, size_t capacity,
                      mick_queue** out) {
  if (!out) return set_error(MICK_E_ARG, "NULL out");
  *out = nullptr;
  if (!prms || !keys) return set_error(MICK_E_ARG, "NULL argument");
  if (n_sets < 1 || n_sets > kMaxSets) return set_error(MICK_E_ARG, "n_sets must be in 1..16");
  if (capacity < 256) return set_error(MICK_E_ARG, "capacity below 256 bytes");
  std::unique_ptr<mick_queue> q(new mick_queue());
  for (int i = 0; i < n_sets; i++) {
    if (!prms[i] || !keys[i]) return set_error(MICK_E_ARG, "NULL parameter set or keys");
    if (keys[i]->prm != prms[i]) return set_error(MICK_E_ARG, "keys[i] belong to other params than prms[i]");
    q->prms.push_back(prms[i]);
    q->keys.push_back(keys[i]);
    q->set_order.push_back(i);
  }
  std::stable_sort(q->set_order.begin(), q->set_order.end(),
                   [&](int a, int b) { return q->prms[a]->log_n < q->prms[b]->log_n; });
  q->capacity = capacity / 256 * 256;
  q->alloc = current_allocator();
  MICK_HIP(hipGetDevice(&q->device), "hipGetDevice");
  const size_t tbytes = table_bytes(kTableEntries);
  void* base = nullptr;
  MICK_TRY(dev_alloc_bytes(q->alloc, &base, q->capacity + tbytes));
  q->base = (char*)base;
  q->arena = Arena(q->capacity);
  q->tables = q->base + q->capacity;
  q->tarena = Arena(tbytes);
  *out = q.release();
  return MICK_OK;
}

size_t mick_queue_job_bytes(const mick_queue* q, int set, int k, int level) {
  if (!q || set < 0 || set >= (int)q->prms.size()) return 0;
  const mick_params* prm = q->prms[set];
  if (k < 2 || k > kMaxK || level < k || level > prm->L) return 0;
  return job_ws_bytes(prm, k, level);
}

namespace {

int check_qjob(const mick_queue* q, const mick_qjob& jb) {
  if (jb.set < 0 || jb.set >= (int)q->prms.size()) return set_error(MICK_E_ARG, "job names an unknown set");
  mick_job one{};
  one.k = jb.k;
  one.level = jb.level;
  memcpy(one.cts, jb.cts, sizeof(one.cts));
  one.out = jb.out;
  MICK_TRY(check_job(q->prms[jb.set], q->keys[jb.set], one));
  if (qjob_bytes(q, jb) > q->capacity)
    return set_error(MICK_E_BUSY, "a job's workspace exceeds the queue's memory budget");
  return MICK_OK;
}

}  // namespace

int mick_queue_push(mick_queue* q, const mick_qjob* jobs, int n_jobs) {
  if (!q || !jobs) return set_error(MICK_E_ARG, "NULL argument");
  if (n_jobs < 0) return set_error(MICK_E_ARG, "n_jobs < 0");
  // all checks first: a refused job without a status word refuses the call
  std::vector<int> st(n_jobs);
  std::string first_error;
  for (int i = 0; i < n_jobs; i++) {
    st[i] = check_qjob(q, jobs[i]);
    if (st[i] != MICK_OK && !jobs[i].status) return st[i];
    if (st[i] != MICK_OK && first_error.empty()) first_error = mick_last_error();
  }
  for (int i = 0; i < n_jobs; i++) {
    if (jobs[i].status) *jobs[i].status = st[i] == MICK_OK ? MICK_PENDING : st[i];
    if (st[i] == MICK_OK) q->pending.push_back(jobs[i]);
  }
  if (!first_error.empty()) set_error(MICK_OK, first_error);  // detail of the first refused job
  return MICK_OK;
}

int mick_queue_cancel(mick_queue* q, uint64_t id) {
  if (!q) return set_error(MICK_E_ARG, "NULL queue");
  int removed = 0;
  for (auto it = q->pending.begin(); it != q->pending.end();) {
    if (it->id != id) {
      ++it;
      continue;
    }
    if (it->status) *it->status = MICK_E_CANCELLED;
    it = q->pending.erase(it);
    removed++;
  }
  if (removed) return MICK_OK;
  for (auto& g : q->running)
    for (uint64_t r : g->ids)
      if (r == id) return set_error(MICK_E_BUSY, "job already launched");
  return set_error(MICK_E_ARG, "no pending or running job with this id");
}

int mick_queue_run(mick_queue* q, void* stream) {
  if (!q) return set_error(MICK_E_ARG, "NULL queue");
  hipStream_t s = (hipStream_t)stream;
  MICK_TRY(reap(q, false));
  const int n_sets = (int)q->prms.size();
  // admission: FIFO while each job's workspace fits a free block
  std::vector<std::vector<mick_qjob>> jobs(n_sets);
  std::vector<std::vector<std::pair<size_t, size_t>>> blocks(n_sets);
  std::vector<std::pair<int, mick_qjob>> admitted;  // (set, job) in FIFO order
  while (!q->pending.empty()) {
    const mick_qjob& jb = q->pending.front();
    if ((int)jobs[jb.set].size() == kTableEntries) break;  // one plan holds at most this many
    const size_t bytes = qjob_bytes(q, jb);
    const size_t off = q->arena.take(bytes);
    if (off == SIZE_MAX) break;
    blocks[jb.set].push_back({off, bytes});
    jobs[jb.set].push_back(jb);
    admitted.push_back({jb.set, jb});
    q->pending.pop_front();
  }
  // one table per set; a set whose table finds no room goes back to the
  // front of the FIFO (all admitted jobs precede every pending one)
  std::vector<size_t> toff(n_sets, SIZE_MAX);
  std::vector<bool> back(n_sets, false);
  for (int set = 0; set < n_sets; set++) {
    if (jobs[set].empty()) continue;
    toff[set] = q->tarena.take(table_bytes((int)jobs[set].size()));
    if (toff[set] == SIZE_MAX) {
      back[set] = true;
      for (auto& b : blocks[set]) q->arena.give(b.first, b.second);
    }
  }
  for (auto it = admitted.rbegin(); it != admitted.rend(); ++it)
    if (back[it->first]) q->pending.push_front(it->second);
  int launched = 0;
  int status = MICK_OK;
  for (int set : q->set_order) {
    auto& js = jobs[set];
    if (js.empty() || back[set]) continue;
    const int n = (int)js.size();
    std::unique_ptr<Group> g(new Group());
    g->blocks = blocks[set];
    g->table = {toff[set], table_bytes(n)};
    std::vector<mick_job> mj(n);
    std::vector<uint32_t*> ws(n);
    for (int i = 0; i < n; i++) {
      mj[i].k = js[i].k;
      mj[i].level = js[i].level;
      memcpy(mj[i].cts, js[i].cts, sizeof(mj[i].cts));
      mj[i].out = js[i].out;
      ws[i] = (uint32_t*)(q->base + blocks[set][i].first);
      g->ids.push_back(js[i].id);
      g->status.push_back(js[i].status);
    }
    int st = plan_jobs(q->prms[set], q->keys[set], mj.data(), n, ws.data(), (JobDesc*)(q->tables + toff[set]), s,
                       &g->plan);
    if (st == MICK_OK) st = mick_plan_execute(g->plan, stream);
    if (st == MICK_OK) st = hip_error(hipEventCreateWithFlags(&g->done, hipEventDisableTiming), "queue event");
    if (st == MICK_OK) st = hip_error(hipEventRecord(g->done, s), "queue event record");
    if (st != MICK_OK) {
      // the group's memory may still be read by launches already queued:
      // wait for the stream before reusing it
      (void)hipStreamSynchronize(s);
      if (g->done) (void)hipEventDestroy(g->done);
      for (auto& b : g->blocks) q->arena.give(b.first, b.second);
      q->tarena.give(g->table.first, g->table.second);
      for (int* js_st : g->status)
        if (js_st) *js_st = st;
      status = st;
      continue;
    }
    launched += n;
    q->running.push_back(std::move(g));
  }
  return status != MICK_OK ? status : launched;
}

int mick_queue_poll(mick_queue* q, uint64_t* done_ids, int max) {
  if (!q || (!done_ids && max > 0)) return set_error(MICK_E_ARG, "NULL argument");
  MICK_TRY(reap(q, false));
  int n = 0;
  while (n < max && !q->done.empty()) {
    done_ids[n++] = q->done.front();
    q->done.pop_front();
  }
  return n;
}

int mick_queue_drain(mick_queue* q, void* stream) {
  if (!q) return set_error(MICK_E_ARG, "NULL queue");
  while (!q->pending.empty()) {
    const int n = mick_queue_run(q, stream);
    if (n < 0) return n;
    if (n == 0) {
      if (q->running.empty()) return set_error(MICK_E_NOMEM, "queue: the next job does not fit an empty arena");
      MICK_TRY(reap(q, true));
    }
  }
  while (!q->running.empty()) MICK_TRY(reap(q, true));
  q->done.clear();
  return MICK_OK;
}

int mick_queue_info(const mick_queue* q, int* pending, int* running, size_t* bytes_in_use) {
  if (!q) return set_error(MICK_E_ARG, "NULL queue");
  if (pending) *pending = (int)q->pending.size();
  if (running) {
    int r = 0;
    for (auto& g : q->running) r += (int)g->ids.size();
    *running = r;
  }
  if (bytes_in_use) *bytes_in_use = q->arena.used();
  return MICK_OK;
}

void mick_queue_destroy(mick_queue* q) {
  if (!q) return;
  for (auto& g : q->running) {
    (void)hipEventSynchronize(g->done);
    (void)hipEventDestroy(g->done);
  }
  dev_free(q->alloc, q->base);
  delete q;
}

}  // extern "C"
