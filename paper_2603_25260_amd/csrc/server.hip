// Serving engine: continuous batching of encode / decode jobs from many
// sensors on one device.
//
// A fixed pool of slots runs concurrently; every slot owns a HIP stream and a
// context (its own workspace, where a frame's octree and features stay
// resident while it is processed).  A job is admitted as soon as a slot is
// free and its estimated device footprint fits in the memory budget next to
// the jobs already running; a free slot takes the oldest admissible job and
// up to max_batch - 1 queued jobs of the same model and kind, which then
// share every launch of the batched pipeline.  Jobs that arrive while
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
  int64_t points;  // encode: input points; decode: points in the stream header
  size_t est;      // estimated device bytes while it runs
};

}  // namespace

struct lpcc_server {
  int device = 0;
  std::vector<const lpcc_model*> models;
  std::vector<int> model_C;
  int max_batch = 1;
  size_t budget = 0;
  size_t in_use = 0;
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

size_t estimate_bytes(int C, int64_t points) {
  // octree arrays + features + neighbour tables + coder buffers, measured
  // at roughly (200 + 12 C) bytes per point, plus fixed tables
  return (size_t)std::max<int64_t>(points, 1) * (size_t)(200 + 12 * C) + ((size_t)8 << 20);
}

void worker_main(lpcc_server* S, int slot) {
  (void)hipSetDevice(S->device);
  lpcc_ctx* ctx = S->ctxs[slot];
  for (;;) {
    std::vector<Pending> batch;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      for (;;) {
        if (S->stop && S->queue.empty()) return;
        // oldest job that fits, then same-kind jobs of the same model
        auto it = S->queue.begin();
        for (; it != S->queue.end(); ++it)
          if (S->in_use + it->est <= S->budget || S->running == 0) break;
        if (it != S->queue.end()) {
          batch.push_back(*it);
          S->in_use += it->est;
          const Pending head = *it;
          S->queue.erase(it);
          for (auto jt = S->queue.begin(); jt != S->queue.end() && (int)batch.size() < S->max_batch;) {
            const bool same = jt->job.kind == head.job.kind && jt->job.model == head.job.model &&
                              (head.job.kind == 1 || jt->job.chunk_log2 == head.job.chunk_log2);
            if (same && S->in_use + jt->est <= S->budget) {
              S->in_use += jt->est;
              batch.push_back(*jt);
              jt = S->queue.erase(jt);
            } else {
              ++jt;
            }
          }
          S->admitted += (int64_t)batch.size();
          S->running += (int64_t)batch.size();
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
    {
      std::lock_guard<std::mutex> lk(S->mu);
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
        S->in_use -= batch[i].est;
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
  for (int k = 0; k < n_slots; k++) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      lpcc_server_free(S);
      return LPCC_E_DEVICE;
    }
    S->streams.push_back(st);
    lpcc_ctx* c = nullptr;
    int s = lpcc_ctx_create(device, st, &c);
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
  if (job->kind == 0) {
    if (job->n_points < 0 || job->chunk_log2 < 4 || job->chunk_log2 > 14) return LPCC_E_INVAL;
    p.points = job->n_points;
  } else {
    // points from the stream header (host streams directly, device ones by copy)
    uint8_t h[16];
    hipPointerAttribute_t a;
    bool dev = hipPointerGetAttributes(&a, job->in) == hipSuccess &&
               (a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged);
    if (!dev) (void)hipGetLastError();
    if (job->in_len < 16) return LPCC_E_CORRUPT;
    if (dev) {
      (void)hipSetDevice(S->device);
      if (hipMemcpy(h, job->in, 16, hipMemcpyDeviceToHost) != hipSuccess) return LPCC_E_DEVICE;
    } else {
      memcpy(h, job->in, 16);
    }
    int D = 0;
    int64_t np = 0;
    int s = lpcc_peek_header(h, 16, &D, &np);
    if (s) return s;
    p.points = np;
  }
  p.est = estimate_bytes(S->model_C[job->model], p.points);
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
  st->bytes_in_use = S->in_use;
  st->bytes_budget = S->budget;
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
