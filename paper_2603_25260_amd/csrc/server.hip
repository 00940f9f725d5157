// Serving engine: continuous batching of encode / decode jobs from many
// sensors on one device.
//
// A fixed pool of slots runs concurrently; every slot owns a HIP stream and a
// context (its own workspace, where a frame's octree and features stay
// resident while it is processed).  Admission is by device memory: the
// workspace the slots' contexts hold counts as in use, and a job is admitted
// when the growth of its slot's workspace that it may need (an upper bound
// computed by the library's own carving code from the job's point count or
// its stream's depth counts) fits in the budget beside the slots' holdings
// and the growth granted to running jobs; each context is capped at what it
// was granted, so the workspace never exceeds the budget.  When a waiting job
// does not fit, idle slots release their workspace.  A free slot takes the
// oldest admissible job and up to max_batch - 1 queued jobs of the same model
// and kind, which then share every launch of the batched pipeline.  Jobs that arrive while
// others are on the device are admitted into slots as they free up, so work
// of different requests overlaps on the device.  Results are byte-identical
// to the isolated calls (the batched calls are).
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "lpcc_internal.h"

namespace {

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Pending {
  lpcc_job job;
  uint64_t ticket;
  int64_t t_arrival;
  int64_t points;            // encode: input points; decode: points in the stream header
  std::vector<int64_t> N;    // decode: node counts of every depth (header)
  int cl = 8;                // decode: chunk size of the stream
  bool host_in = false;      // encode: coordinates in host memory (staged)
  size_t need[3] = {0, 0, 0};  // workspace bound of the job alone (per arena)
};

}  // namespace

struct lpcc_server {
  int device = 0;
  std::vector<const lpcc_model*> models;
  std::vector<int> model_C;
  int max_batch = 1;
  size_t budget = 0;
  size_t held = 0;     // workspace the slots' contexts hold (as of their last job)
  size_t granted = 0;  // growth granted to running jobs
  size_t peak = 0;     // largest held + granted
  std::vector<size_t> slot_held;
  std::vector<bool> slot_busy;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Pending> queue;
  std::vector<lpcc_done> done;  // completed, not yet polled
  std::vector<double> lat_ms;   // all completed latencies
  int64_t pts_done = 0, first_arrival = -1, last_done = 0;
  int64_t admitted = 0, completed = 0, running = 0;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;
  std::vector<lpcc_ctx*> ctxs;
};

namespace {

// Workspace bound of a batch of jobs (per arena: octree, model, descriptors)
void bound_of(lpcc_server* S, const std::vector<const Pending*>& b, size_t need[3]) {
  const lpcc_model* m = S->models[b[0]->job.model];
  if (b[0]->job.kind == 0) {
    std::vector<int64_t> n;
    bool host = false;
    for (auto* p : b) {
      n.push_back(p->points);
      host = host || p->host_in;
    }
    lpcc::encode_workspace_bound(m, (int)b.size(), n.data(), b[0]->job.chunk_log2, host, need);
  } else {
    std::vector<const int64_t*> N;
    std::vector<int> cl;
    for (auto* p : b) {
      N.push_back(p->N.data());
      cl.push_back(p->cl);
    }
    lpcc::decode_workspace_bound(m, (int)b.size(), N.data(), cl.data(), need);
  }
}

// Growth of a slot's arenas up to the bound
size_t growth_of(lpcc_ctx* ctx, const size_t need[3]) {
  size_t caps[3];
  lpcc::ctx_caps(ctx, caps);
  size_t g = 0;
  for (int a = 0; a < 3; a++) g += need[a] > caps[a] ? need[a] - caps[a] : 0;
  return g;
}

bool same_kind(const Pending& a, const Pending& b) {
  return a.job.kind == b.job.kind && a.job.model == b.job.model &&
         (a.job.kind == 1 || a.job.chunk_log2 == b.job.chunk_log2);
}

void worker_main(lpcc_server* S, int slot) {
  (void)hipSetDevice(S->device);
  lpcc_ctx* ctx = S->ctxs[slot];
  for (;;) {
    std::vector<Pending> batch;
    size_t growth = 0;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      for (;;) {
        if (S->stop && S->queue.empty()) return;
        auto fits = [&](size_t g) { return S->held + S->granted + g <= S->budget; };
        // oldest job whose growth fits; once, idle slots give their
        // workspace back before the queue is scanned again
        auto pick = [&]() -> std::deque<Pending>::iterator {
          for (auto it = S->queue.begin(); it != S->queue.end(); ++it) {
            growth = growth_of(ctx, it->need);
            if (fits(growth)) return it;
          }
          return S->queue.end();
        };
        auto it = pick();
        if (it == S->queue.end() && !S->queue.empty()) {
          bool freed = false;
          for (size_t k = 0; k < S->ctxs.size(); k++)
            if (!S->slot_busy[k] && S->slot_held[k] > 0) {
              lpcc::ctx_trim(S->ctxs[k]);
              S->held -= S->slot_held[k];
              S->slot_held[k] = 0;
              freed = true;
            }
          if (freed) it = pick();
        }
        if (it == S->queue.end() && !S->queue.empty() && S->granted == 0 && S->running == 0) {
          // nothing runs and nothing else can free memory: the oldest job
          // gets what the budget leaves (it fails with LPCC_E_NOMEM if that
          // is too little)
          it = S->queue.begin();
          growth = S->budget > S->held ? S->budget - S->held : 0;
        }
        if (it != S->queue.end()) {
          batch.push_back(*it);
          S->queue.erase(it);
          // same-kind jobs of the same model, while the batch's growth fits
          for (auto jt = S->queue.begin(); jt != S->queue.end() && (int)batch.size() < S->max_batch;) {
            if (!same_kind(*jt, batch[0])) {
              ++jt;
              continue;
            }
            std::vector<const Pending*> v;
            for (auto& p : batch) v.push_back(&p);
            v.push_back(&*jt);
            size_t need[3];
            bound_of(S, v, need);
            const size_t g = growth_of(ctx, need);
            if (fits(g)) {
              growth = g;
              batch.push_back(*jt);
              jt = S->queue.erase(jt);
            } else {
              ++jt;
            }
          }
          S->granted += growth;
          S->peak = std::max(S->peak, S->held + S->granted);
          S->slot_busy[slot] = true;
          S->admitted += (int64_t)batch.size();
          S->running += (int64_t)batch.size();
          lpcc::ctx_set_budget(ctx, S->slot_held[slot] + growth);
          break;
        }
        S->cv_work.wait(lk);
      }
    }
    const int nb = (int)batch.size();
    const lpcc_model* m = S->models[batch[0].job.model];
    const int64_t t_start = now_ns();
    std::vector<int> status(nb, LPCC_OK);
    std::vector<size_t> out_len(nb, 0);
    std::vector<int64_t> n_out(nb, 0);
    if (batch[0].job.kind == 0) {
      std::vector<const int32_t*> xyz(nb);
      std::vector<int64_t> n(nb);
      std::vector<uint8_t*> out(nb);
      std::vector<size_t> cap(nb);
      for (int i = 0; i < nb; i++) {
        xyz[i] = (const int32_t*)batch[i].job.in;
        n[i] = batch[i].job.n_points;
        out[i] = (uint8_t*)batch[i].job.out;
        cap[i] = batch[i].job.out_cap;
      }
      int st = lpcc_encode_batch(ctx, m, nb, xyz.data(), n.data(), batch[0].job.chunk_log2, out.data(), cap.data(),
                                 out_len.data(), status.data());
      if (st == LPCC_E_DEVICE || st == LPCC_E_NOMEM || st == LPCC_E_INVAL)
        for (int i = 0; i < nb; i++)
          if (status[i] == LPCC_OK) status[i] = st;
    } else {
      std::vector<const uint8_t*> bs(nb);
      std::vector<size_t> len(nb);
      std::vector<int32_t*> out(nb);
      std::vector<int64_t> cap(nb);
      for (int i = 0; i < nb; i++) {
        bs[i] = (const uint8_t*)batch[i].job.in;
        len[i] = batch[i].job.in_len;
        out[i] = (int32_t*)batch[i].job.out;
        cap[i] = (int64_t)batch[i].job.out_cap;
      }
      int st = lpcc_decode_batch(ctx, m, nb, bs.data(), len.data(), out.data(), cap.data(), n_out.data(),
                                 status.data());
      if (st == LPCC_E_DEVICE || st == LPCC_E_NOMEM || st == LPCC_E_INVAL)
        for (int i = 0; i < nb; i++)
          if (status[i] == LPCC_OK) status[i] = st;
    }
    const int64_t t_done = now_ns();
    size_t caps[3];
    lpcc::ctx_caps(ctx, caps);
    {
      std::lock_guard<std::mutex> lk(S->mu);
      const size_t now_held = caps[0] + caps[1] + caps[2];
      S->held = S->held - S->slot_held[slot] + now_held;
      S->slot_held[slot] = now_held;
      S->granted -= growth;
      S->slot_busy[slot] = false;
      for (int i = 0; i < nb; i++) {
        lpcc_done d;
        memset(&d, 0, sizeof(d));
        d.ticket = batch[i].ticket;
        d.status = status[i];
        d.kind = batch[i].job.kind;
        d.out_len = batch[i].job.kind == 0 ? out_len[i] : (size_t)n_out[i];
        d.n_points = batch[i].points;
        d.t_arrival_ns = batch[i].t_arrival;
        d.t_start_ns = t_start;
        d.t_done_ns = t_done;
        d.batch = nb;
        S->done.push_back(d);
        S->lat_ms.push_back((double)(t_done - batch[i].t_arrival) / 1e6);
        if (status[i] == LPCC_OK) S->pts_done += batch[i].points;
        if (S->first_arrival < 0 || batch[i].t_arrival < S->first_arrival) S->first_arrival = batch[i].t_arrival;
        S->last_done = std::max(S->last_done, t_done);
      }
      S->completed += nb;
      S->running -= nb;
    }
    S->cv_done.notify_all();
    S->cv_work.notify_all();
  }
}

}  // namespace

extern "C" {

int lpcc_server_create(int device, const lpcc_model* const* models, int n_models, int n_slots, int max_batch,
                       size_t hbm_budget, lpcc_server** out) {
  if (!models || n_models <= 0 || n_slots <= 0 || max_batch <= 0 || !out) return LPCC_E_INVAL;
  *out = nullptr;
  if (hipSetDevice(device) != hipSuccess) return LPCC_E_DEVICE;
  lpcc_server* S = new lpcc_server();
  S->device = device;
  S->max_batch = max_batch;
  for (int i = 0; i < n_models; i++) {
    if (!models[i]) {
      delete S;
      return LPCC_E_INVAL;
    }
    int C = 0;
    lpcc_model_info(models[i], &C, nullptr, nullptr, nullptr);
    S->models.push_back(models[i]);
    S->model_C.push_back(C);
  }
  if (hbm_budget == 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
      delete S;
      return LPCC_E_DEVICE;
    }
    hbm_budget = fr - fr / 8;  // leave headroom for the caller
  }
  S->budget = hbm_budget;
  S->slot_held.assign(n_slots, 0);
  S->slot_busy.assign(n_slots, false);
  for (int k = 0; k < n_slots; k++) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      lpcc_server_free(S);
      return LPCC_E_DEVICE;
    }
    S->streams.push_back(st);
    lpcc_ctx* c = nullptr;
    int s = lpcc_ctx_create(device, st, 0, &c);
    if (s) {
      lpcc_server_free(S);
      return s;
    }
    S->ctxs.push_back(c);
  }
  for (int k = 0; k < n_slots; k++) S->workers.emplace_back(worker_main, S, k);
  *out = S;
  return LPCC_OK;
}

int lpcc_server_submit(lpcc_server* S, const lpcc_job* job, uint64_t* ticket) {
  if (!S || !job || !ticket || job->model < 0 || job->model >= (int)S->models.size()) return LPCC_E_INVAL;
  if (job->kind != 0 && job->kind != 1) return LPCC_E_INVAL;
  if (!job->in || !job->out) return LPCC_E_INVAL;
  Pending p;
  p.job = *job;
  p.t_arrival = job->t_arrival_ns > 0 ? job->t_arrival_ns : now_ns();
  hipPointerAttribute_t a;
  const bool dev = hipPointerGetAttributes(&a, job->in) == hipSuccess &&
                   (a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged);
  if (!dev) (void)hipGetLastError();
  if (job->kind == 0) {
    if (job->n_points < 0 || job->chunk_log2 < 4 || job->chunk_log2 > 14) return LPCC_E_INVAL;
    p.points = job->n_points;
    p.host_in = !dev;
  } else {
    // depth counts from the stream header (host streams directly, device
    // ones by copy): they bound the decode's workspace
    uint8_t h[16 + 4 * lpcc::kMaxD];
    if (job->in_len < 16) return LPCC_E_CORRUPT;
    const size_t nh = std::min(job->in_len, sizeof(h));
    if (dev) {
      (void)hipSetDevice(S->device);
      if (hipMemcpy(h, job->in, nh, hipMemcpyDeviceToHost) != hipSuccess) return LPCC_E_DEVICE;
    } else {
      memcpy(h, job->in, nh);
    }
    int D = 0;
    int64_t np = 0;
    int s = lpcc_peek_header(h, nh, &D, &np, nullptr);
    if (s) return s;
    int mD = 0;
    lpcc_model_info(S->models[job->model], nullptr, &mD, nullptr, nullptr);
    if (D != mD || nh < 16 + 4 * (size_t)D) return LPCC_E_CORRUPT;
    p.points = np;
    p.cl = h[7];
    if (p.cl < 4 || p.cl > 14) return LPCC_E_CORRUPT;
    p.N.assign(D + 1, 0);
    auto rd = [&](size_t o) {
      return (int64_t)((uint32_t)h[o] | ((uint32_t)h[o + 1] << 8) | ((uint32_t)h[o + 2] << 16) |
                       ((uint32_t)h[o + 3] << 24));
    };
    p.N[D] = rd(12);
    for (int d = 0; d < D; d++) p.N[d] = rd(16 + 4 * (size_t)d);
  }
  bound_of(S, {&p}, p.need);
  {
    std::lock_guard<std::mutex> lk(S->mu);
    p.ticket = S->next_ticket++;
    S->queue.push_back(p);
  }
  S->cv_work.notify_one();
  *ticket = p.ticket;
  return LPCC_OK;
}

int lpcc_server_poll(lpcc_server* S, lpcc_done* out, int max, int* n_done, int wait_ms) {
  if (!S || !out || max <= 0 || !n_done) return LPCC_E_INVAL;
  std::unique_lock<std::mutex> lk(S->mu);
  if (S->done.empty() && wait_ms > 0)
    S->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return !S->done.empty(); });
  const int k = std::min<int>(max, (int)S->done.size());
  for (int i = 0; i < k; i++) out[i] = S->done[i];
  S->done.erase(S->done.begin(), S->done.begin() + k);
  *n_done = k;
  return LPCC_OK;
}

int lpcc_server_drain(lpcc_server* S) {
  if (!S) return LPCC_E_INVAL;
  std::unique_lock<std::mutex> lk(S->mu);
  S->cv_done.wait(lk, [&] { return S->queue.empty() && S->running == 0; });
  return LPCC_OK;
}

int lpcc_server_stats(lpcc_server* S, lpcc_stats* st) {
  if (!S || !st) return LPCC_E_INVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  memset(st, 0, sizeof(*st));
  std::vector<double> v = S->lat_ms;
  if (!v.empty()) {
    std::sort(v.begin(), v.end());
    auto pct = [&](double q) {
      const double idx = q * (double)(v.size() - 1);
      const size_t lo = (size_t)idx;
      const size_t hi = std::min(lo + 1, v.size() - 1);
      return v[lo] + (v[hi] - v[lo]) * (idx - (double)lo);
    };
    st->p50_ms = pct(0.50);
    st->p99_ms = pct(0.99);
    double sum = 0;
    for (double x : v) sum += x;
    st->mean_ms = sum / (double)v.size();
  }
  if (S->first_arrival >= 0 && S->last_done > S->first_arrival)
    st->mpts_per_s = (double)S->pts_done / ((double)(S->last_done - S->first_arrival) / 1e9) / 1e6;
  st->completed = S->completed;
  st->admitted = S->admitted;
  st->queued = (int64_t)S->queue.size();
  st->running = S->running;
  st->bytes_in_use = S->held + S->granted;
  st->bytes_budget = S->budget;
  st->bytes_peak = S->peak;
  return LPCC_OK;
}

void lpcc_server_free(lpcc_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  for (auto& t : S->workers)
    if (t.joinable()) t.join();
  for (auto* c : S->ctxs) lpcc_ctx_free(c);
  for (auto st : S->streams) (void)hipStreamDestroy(st);
  delete S;
}

}  // extern "C"
