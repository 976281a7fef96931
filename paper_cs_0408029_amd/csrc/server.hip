// Serving engine: continuous batching of independent NNLS requests on one device.
//
// Submit copies a request into one pinned staging block (colptr | rowidx | val | b) taken
// from a size-class pool and queues it on one of two lanes, chosen by n alone:
//   - batched lane (n <= batch_max_n), stepped at pivot-iteration level: a lane thread
//     keeps a set of live problems whose state (dense A, Gram matrix, factor, (F, G) split,
//     x, y) stays in device memory.  Each step admits the queued requests that fit (up to
//     batch_max_count live), scatters their CSC into dense column-major blocks and forms
//     their Gram matrices, then advances every live problem by batch_step_iters pivot
//     iterations in one launch (one workgroup per problem) and retires the ones that
//     finished, so a short request leaves as soon as it converges and a new one joins at
//     the next step instead of waiting for a whole batch; several lanes step in turn;
//   - sparse lane: each worker owns a stream and a solver handle and runs one request at a
//     time through the full sparse path (Gram, tiled factor, triangular solves, residual,
//     dual), so several large requests overlap on the device.
// Admission is in arrival order per lane and bounded by the estimated device bytes of the
// running requests.  Neither lane lets one request's arithmetic depend on another's, so a
// result is the same alone and in the mix.
#include <algorithm>
#include <chrono>
#include <climits>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "nnls_internal.h"

using namespace nnls;

namespace {

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// Pinned host blocks in power-of-two size classes from 4 KiB, reused across requests so
// that submit does not pay for a page-locking allocation each time.
// Pinned host blocks in power-of-two size classes (4 KiB << c).  Blocks up to SLAB / 4
// are carved from SLAB-byte slabs, so that a growing backlog of requests costs one
// page-locking allocation per slab rather than one per request; larger blocks are
// allocated alone.  Blocks go back to their class's free list and are reused; everything
// is released when the pool ends.
class PinnedPool {
 public:
  ~PinnedPool() {
    for (void* p : slabs_) (void)hipHostFree(p);
    for (void* p : singles_) (void)hipHostFree(p);
  }
  void* get(size_t bytes, int* cls_out) {
    const int c = size_class(bytes);
    *cls_out = c;
    std::lock_guard<std::mutex> lk(mu_);
    if ((int)free_.size() <= c) free_.resize((size_t)c + 1);
    std::vector<void*>& fl = free_[(size_t)c];
    if (fl.empty()) {
      const size_t blk = (size_t)4096 << c;
      void* p = nullptr;
      if (blk <= SLAB / 4) {
        if (hipHostMalloc(&p, SLAB, hipHostMallocDefault) != hipSuccess) {
          (void)hipGetLastError();
          return nullptr;
        }
        slabs_.push_back(p);
        for (size_t o = blk; o + blk <= SLAB; o += blk) fl.push_back((char*)p + o);
        return p;
      }
      if (hipHostMalloc(&p, blk, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
      }
      singles_.push_back(p);
      return p;
    }
    void* p = fl.back();
    fl.pop_back();
    return p;
  }
  void put(void* p, int cls) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(mu_);
    if ((int)free_.size() <= cls) free_.resize((size_t)cls + 1);
    free_[(size_t)cls].push_back(p);
  }

 private:
  static constexpr size_t SLAB = (size_t)64 << 20;
  static int size_class(size_t bytes) {
    int c = 0;
    while (((size_t)4096 << c) < bytes) ++c;
    return c;
  }
  std::mutex mu_;
  std::vector<std::vector<void*>> free_;
  std::vector<void*> slabs_, singles_;
};

struct DevVec {
  void* p = nullptr;
  size_t bytes = 0;
  bool ensure(size_t need) {
    if (need == 0) need = 256;
    if (bytes >= need) return true;
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    if (hipMalloc(&p, need) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    bytes = need;
    return true;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
};

// Device blocks in power-of-two size classes (64 KiB << c), reused across requests of the
// batched lane; up to `keep` bytes of free blocks are cached, the rest go back at once.
class DevPool {
 public:
  explicit DevPool(size_t keep) : keep_(keep) {}
  ~DevPool() { release_all(); }
  void* get(size_t bytes, int* cls_out) {
    int c = 0;
    while (((size_t)65536 << c) < bytes) ++c;
    *cls_out = c;
    if ((int)free_.size() > c && !free_[(size_t)c].empty()) {
      void* p = free_[(size_t)c].back();
      free_[(size_t)c].pop_back();
      cached_ -= (size_t)65536 << c;
      return p;
    }
    void* p = nullptr;
    if (hipMalloc(&p, (size_t)65536 << c) != hipSuccess) {
      (void)hipGetLastError();
      release_all();   // give the cached blocks back and try once more
      if (hipMalloc(&p, (size_t)65536 << c) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
      }
    }
    return p;
  }
  void put(void* p, int cls) {
    if (!p) return;
    const size_t bytes = (size_t)65536 << cls;
    if (cached_ + bytes > keep_) {
      (void)hipFree(p);
      return;
    }
    if ((int)free_.size() <= cls) free_.resize((size_t)cls + 1);
    free_[(size_t)cls].push_back(p);
    cached_ += bytes;
  }
  void release_all() {
    for (std::vector<void*>& fl : free_)
      for (void* p : fl) (void)hipFree(p);
    free_.clear();
    cached_ = 0;
  }

 private:
  size_t keep_, cached_ = 0;
  std::vector<std::vector<void*>> free_;
};

struct PinnedVec {
  void* p = nullptr;
  size_t bytes = 0;
  bool ensure(size_t need) {
    if (need == 0) need = 256;
    if (bytes >= need) return true;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
    if (hipHostMalloc(&p, need, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    bytes = need;
    return true;
  }
  ~PinnedVec() {
    if (p) (void)hipHostFree(p);
  }
};

enum Lane { LANE_SPARSE = 0, LANE_BATCHED = 1 };

struct Request {
  uint64_t id = 0;
  int32_t m = 0, n = 0;
  int64_t nnz = 0;
  int lane = LANE_SPARSE;
  PackLayout L{};
  char* in = nullptr;   // pinned packed input
  int in_cls = 0;
  double* out = nullptr;  // pinned x | y
  int out_cls = 0;
  size_t footprint = 0;
  double t_submit = 0, t_start = 0, t_done = 0;
  nnls_info info{};
  bool done = false;
};

// Device bytes one request occupies while it runs, from its host CSC.
size_t sparse_footprint(int m, int n, int64_t nnz, const int32_t* rowidx) {
  std::vector<int64_t> rowlen((size_t)m, 0);
  for (int64_t e = 0; e < nnz; ++e) rowlen[(size_t)rowidx[e]] += 1;
  int64_t ub = 0;   // bound on the stored Gram entries (sum of squared row lengths)
  for (int i = 0; i < m; ++i) ub += rowlen[(size_t)i] * rowlen[(size_t)i];
  const int nb = (n + TILE - 1) / TILE;
  const size_t tiles = (size_t)tile_count(nb);
  size_t f = (size_t)pack_layout(m, n, nnz).total + (size_t)n * 16;          // input, x | y
  f += (size_t)(m + 1) * 4 + (size_t)nnz * 12 + (size_t)m * 4;                 // CSR copy
  f += (size_t)(n + 1) * 8 + (size_t)n * 8 + (size_t)ub * 24;                  // Gram + F-position lists
  f += (size_t)n * (8 + 8 + 1 + 4 + 4 + 4 + 4) + (size_t)m * 8;                // c, g, flags, F, pos, order, r
  f += (tiles + (size_t)nb) * TILE_ELEMS * 8 + tiles * 4 + (size_t)nb * (8 + 3 * TILE * 8);
  return f;
}

// Device block of one live request of the batched lane: packed input | dense A | x | y |
// workspace, each part 256-byte aligned.
struct LiveLayout {
  size_t dense, x, y, ws, total;
};
LiveLayout live_layout(int m, int n, int64_t nnz) {
  const auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
  LiveLayout L;
  L.dense = al((size_t)pack_layout(m, n, nnz).total);
  L.x = L.dense + al((size_t)m * n * 8);
  L.y = L.x + al((size_t)n * 8);
  L.ws = L.y + al((size_t)n * 8);
  L.total = L.ws + batched_workspace_bytes(m, n);
  return L;
}

size_t batched_footprint(int m, int n, int64_t nnz) {
  return live_layout(m, n, nnz).total + sizeof(ScatterDesc) + sizeof(BatchProblem) + sizeof(BatchInfo);
}

}  // namespace

struct nnls_server {
  int device = 0;
  nnls_options opts{};
  nnls_server_config cfg{};
  size_t budget = 0;
  size_t keep_bytes = 0;   // a sparse worker gives back workspaces above this after a request
  PinnedPool pool;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request*> queue[2];
  std::unordered_map<uint64_t, Request*> reqs;
  uint64_t next_id = 1;
  size_t committed = 0, peak_committed = 0;
  int running = 0, max_running = 0;
  bool stop = false;
  std::vector<std::thread> threads;
  int started = 0, failed_start = 0;
  // statistics since the last reset
  std::vector<double> latencies;
  int64_t submitted = 0, batches = 0;
  double first_submit = -1, last_done = 0;
};

namespace {

// Call with s->mu held.
bool admissible(const nnls_server* s, const Request* r) {
  return s->running == 0 || s->committed + r->footprint <= s->budget;
}

void admit(nnls_server* s, Request* r) {
  s->committed += r->footprint;
  s->peak_committed = std::max(s->peak_committed, s->committed);
  s->running += 1;
  s->max_running = std::max(s->max_running, s->running);
  r->t_start = now_ms();
}

// Mark requests finished (x, y and info already in place).  Call without s->mu.
void retire(nnls_server* s, Request* const* rs, size_t count) {
  const double t = now_ms();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    for (size_t i = 0; i < count; ++i) {
      Request* r = rs[i];
      r->t_done = t;
      r->info.setup_ms = r->t_start - r->t_submit;
      r->info.solve_ms = t - r->t_submit;
      r->done = true;
      s->committed -= r->footprint;
      s->running -= 1;
      s->latencies.push_back(t - r->t_submit);
    }
    s->last_done = std::max(s->last_done, t);
  }
  s->cv_done.notify_all();
  s->cv_work.notify_all();
}

void fail_all(nnls_server* s, std::vector<Request*>& rs, int st) {
  for (Request* r : rs) {
    std::memset(&r->info, 0, sizeof(r->info));
    r->info.status = st;
    r->info.failed_index = -1;
  }
  retire(s, rs.data(), rs.size());
}

void report_start(nnls_server* s, bool ok) {
  std::lock_guard<std::mutex> lk(s->mu);
  if (ok)
    s->started += 1;
  else
    s->failed_start += 1;
  s->cv_done.notify_all();
}

bool open_lane(nnls_server* s, hipStream_t* stream, nnls_handle** h) {
  if (hipSetDevice(s->device) != hipSuccess ||
      hipStreamCreateWithFlags(stream, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  if (nnls_create(h, s->device, (void*)*stream) != NNLS_OK) {
    (void)hipStreamDestroy(*stream);
    return false;
  }
  return true;
}

void sparse_worker(nnls_server* s) {
  hipStream_t stream = nullptr;
  nnls_handle* h = nullptr;
  const bool ok = open_lane(s, &stream, &h);
  report_start(s, ok);
  if (!ok) return;
  DevVec din, dout;
  std::deque<Request*>& q = s->queue[LANE_SPARSE];
  for (;;) {
    Request* r = nullptr;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait(lk, [&] { return s->stop || (!q.empty() && admissible(s, q.front())); });
      if (s->stop) break;
      r = q.front();
      q.pop_front();
      admit(s, r);
    }
    int st = NNLS_OK;
    const size_t in_bytes = (size_t)r->L.total, out_bytes = (size_t)r->n * 16;
    if (!din.ensure(in_bytes) || !dout.ensure(out_bytes)) st = NNLS_ERR_NO_MEMORY;
    if (st == NNLS_OK &&
        hipMemcpyAsync(din.p, r->in, in_bytes, hipMemcpyHostToDevice, stream) != hipSuccess) {
      (void)hipGetLastError();
      st = NNLS_ERR_DEVICE;
    }
    if (st == NNLS_OK) {
      const char* base = (const char*)din.p;
      double* x = (double*)dout.p;
      st = nnls_solve_csc(h, r->m, r->n, r->nnz, (const int32_t*)base, (const int32_t*)(base + r->L.rowidx),
                          (const double*)(base + r->L.val), (const double*)(base + r->L.b), x, x + r->n,
                          &s->opts, &r->info);
      if (hipMemcpyAsync(r->out, dout.p, out_bytes, hipMemcpyDeviceToHost, stream) != hipSuccess ||
          hipStreamSynchronize(stream) != hipSuccess) {
        (void)hipGetLastError();
        if (st == NNLS_OK) st = NNLS_ERR_DEVICE;
      }
    } else {
      std::memset(&r->info, 0, sizeof(r->info));
      r->info.failed_index = -1;
    }
    r->info.status = st;
    if (r->footprint > s->keep_bytes) {   // do not sit on a large workspace while idle
      release_workspace(h);
      din.release();
      dout.release();
    }
    retire(s, &r, 1);
  }
  din.release();
  dout.release();
  nnls_destroy(h);
  (void)hipStreamDestroy(stream);
}

void batch_lane(nnls_server* s) {
  hipStream_t stream = nullptr;
  nnls_handle* h = nullptr;
  const bool ok = open_lane(s, &stream, &h);
  report_start(s, ok);
  if (!ok) return;
  struct Live {
    Request* r;
    void* blk;
    int cls;
    int slot;
    BatchProblem desc;
  };
  const int cap = s->cfg.batch_max_count;
  DevPool blocks(s->keep_bytes);
  DevVec dinfo, ddesc, dscat;
  PinnedVec hinfo, hdesc, hscat;
  std::vector<Live> live, fresh, leaving;
  std::vector<int> free_slots;
  for (int i = cap - 1; i >= 0; --i) free_slots.push_back(i);
  std::vector<Request*> taken, finished;
  std::deque<Request*>& q = s->queue[LANE_BATCHED];
  if (!dinfo.ensure(sizeof(BatchInfo) * (size_t)cap) || !hinfo.ensure(sizeof(BatchInfo) * (size_t)cap) ||
      !ddesc.ensure(sizeof(BatchProblem) * (size_t)cap) || !hdesc.ensure(sizeof(BatchProblem) * (size_t)cap) ||
      !dscat.ensure(sizeof(ScatterDesc) * (size_t)cap) || !hscat.ensure(sizeof(ScatterDesc) * (size_t)cap)) {
    // cannot step at all: every request that reaches this lane fails
    for (;;) {
      taken.clear();
      {
        std::unique_lock<std::mutex> lk(s->mu);
        s->cv_work.wait(lk, [&] { return s->stop || (!q.empty() && admissible(s, q.front())); });
        if (s->stop) break;
        Request* r = q.front();
        q.pop_front();
        admit(s, r);
        taken.push_back(r);
      }
      fail_all(s, taken, NNLS_ERR_NO_MEMORY);
    }
    nnls_destroy(h);
    (void)hipStreamDestroy(stream);
    return;
  }
  BatchInfo* inf = (BatchInfo*)hinfo.p;
  BatchArgs ba;
  std::memset(&ba, 0, sizeof(ba));
  ba.tau = s->opts.tau;
  ba.p_max = s->opts.p_max;
  ba.max_iter = s->opts.max_iter;
  ba.fp32 = s->opts.precision != NNLS_FP64 ? 1 : 0;   // NNLS_BF16_IR: the batched float32 tier
  ba.ir_max_steps = s->opts.ir_max_steps;
  ba.ir_rtol = s->opts.ir_rtol;
  ba.gram_dual = (s->opts.flags & NNLS_FLAG_GRAM_DUAL) != 0 ? 1 : 0;
  const int step_iters = s->cfg.batch_step_iters;
  auto fail_live = [&](std::vector<Live>& v, int st) {
    taken.clear();
    for (Live& l : v) {
      taken.push_back(l.r);
      blocks.put(l.blk, l.cls);
      free_slots.push_back(l.slot);
    }
    v.clear();
    fail_all(s, taken, st);
  };
  for (;;) {
    // admission at the step boundary
    taken.clear();
    {
      std::unique_lock<std::mutex> lk(s->mu);
      if (live.empty())
        s->cv_work.wait(lk, [&] { return s->stop || (!q.empty() && admissible(s, q.front())); });
      if (s->stop && live.empty()) break;
      while (!s->stop && !q.empty() && (int)(live.size() + taken.size()) < cap && admissible(s, q.front())) {
        Request* r = q.front();
        q.pop_front();
        admit(s, r);
        taken.push_back(r);
      }
      s->batches += 1;
    }
    // new problems: device block, input copy, dense A, Gram matrix
    fresh.clear();
    std::vector<Request*> nomem;
    for (Request* r : taken) {
      const LiveLayout L = live_layout(r->m, r->n, r->nnz);
      Live l;
      l.r = r;
      l.blk = blocks.get(L.total, &l.cls);
      if (!l.blk) {
        nomem.push_back(r);
        continue;
      }
      l.slot = free_slots.back();
      free_slots.pop_back();
      char* base = (char*)l.blk;
      BatchProblem& d = l.desc;
      d.m = r->m;
      d.n = r->n;
      d.lda = r->m;
      d.pad = 0;
      d.A = (const double*)(base + L.dense);
      d.b = (const double*)(base + r->L.b);
      d.x = (double*)(base + L.x);
      d.y = (double*)(base + L.y);
      d.info = (BatchInfo*)dinfo.p + l.slot;
      d.ws = base + L.ws;
      fresh.push_back(l);
    }
    if (!nomem.empty()) fail_all(s, nomem, NNLS_ERR_NO_MEMORY);
    int st = NNLS_OK;
    if (!fresh.empty()) {
      ScatterDesc* sd = (ScatterDesc*)hscat.p;
      BatchProblem* bd = (BatchProblem*)hdesc.p;
      const char* origin = (const char*)fresh[0].blk;
      for (size_t i = 0; i < fresh.size(); ++i) {
        const Live& l = fresh[i];
        const LiveLayout L = live_layout(l.r->m, l.r->n, l.r->nnz);
        sd[i].m = l.r->m;
        sd[i].n = l.r->n;
        sd[i].nnz = l.r->nnz;
        sd[i].in_off = (int64_t)((const char*)l.blk - origin);
        sd[i].a_off = (int64_t)((const char*)l.blk + L.dense - origin) / 8;
        bd[i] = l.desc;
        if (hipMemcpyAsync(l.blk, l.r->in, (size_t)l.r->L.total, hipMemcpyHostToDevice, stream) != hipSuccess)
          st = NNLS_ERR_DEVICE;
      }
      if (st == NNLS_OK &&
          (hipMemcpyAsync(dscat.p, sd, sizeof(ScatterDesc) * fresh.size(), hipMemcpyHostToDevice, stream) !=
               hipSuccess ||
           hipMemcpyAsync(ddesc.p, bd, sizeof(BatchProblem) * fresh.size(), hipMemcpyHostToDevice, stream) !=
               hipSuccess))
        st = NNLS_ERR_DEVICE;
      if (st == NNLS_OK) {
        launch_csc_scatter(stream, (int)fresh.size(), (const ScatterDesc*)dscat.p, origin, (double*)origin);
        ba.count = (int)fresh.size();
        ba.probs = (const BatchProblem*)ddesc.p;
        ba.order = nullptr;
        launch_batched_gram(stream, ba, (int)fresh.size());
        if (hipGetLastError() != hipSuccess) st = NNLS_ERR_DEVICE;
      }
      // the host descriptor buffers are rewritten below: wait for the copies out of them
      if (st == NNLS_OK && hipStreamSynchronize(stream) != hipSuccess) st = NNLS_ERR_DEVICE;
      if (st != NNLS_OK) {
        (void)hipGetLastError();
        fail_live(fresh, st);
        fail_live(live, st);
        continue;
      }
      for (Live& l : fresh) live.push_back(l);
    }
    if (live.empty()) continue;
    // one step of every live problem
    BatchProblem* bd = (BatchProblem*)hdesc.p;
    int maxslot = 0;
    for (size_t i = 0; i < live.size(); ++i) {
      bd[i] = live[i].desc;
      maxslot = std::max(maxslot, live[i].slot + 1);
    }
    ba.count = (int)live.size();
    ba.probs = (const BatchProblem*)ddesc.p;
    ba.order = nullptr;
    ba.max_steps = step_iters;
    if (hipMemcpyAsync(ddesc.p, bd, sizeof(BatchProblem) * live.size(), hipMemcpyHostToDevice, stream) !=
        hipSuccess)
      st = NNLS_ERR_DEVICE;
    if (st == NNLS_OK) {
      launch_batched_steps(stream, ba, (int)live.size());
      if (hipGetLastError() != hipSuccess ||
          hipMemcpyAsync(inf, dinfo.p, sizeof(BatchInfo) * (size_t)maxslot, hipMemcpyDeviceToHost, stream) !=
              hipSuccess ||
          hipStreamSynchronize(stream) != hipSuccess)
        st = NNLS_ERR_DEVICE;
    }
    ba.max_steps = 0;
    if (st != NNLS_OK) {
      (void)hipGetLastError();
      fail_live(live, st);
      continue;
    }
    // retire the problems that finished in this step
    finished.clear();
    leaving.clear();
    size_t keep = 0;
    for (size_t i = 0; i < live.size(); ++i) {
      Live& l = live[i];
      const BatchInfo& qi = inf[l.slot];
      if (!qi.done) {
        live[keep++] = l;
        continue;
      }
      Request* r = l.r;
      if (hipMemcpyAsync(r->out, l.desc.x, (size_t)r->n * 8, hipMemcpyDeviceToHost, stream) != hipSuccess ||
          hipMemcpyAsync(r->out + r->n, l.desc.y, (size_t)r->n * 8, hipMemcpyDeviceToHost, stream) != hipSuccess) {
        (void)hipGetLastError();
        st = NNLS_ERR_DEVICE;
      }
      std::memset(&r->info, 0, sizeof(r->info));
      r->info.status = qi.status;
      r->info.iterations = qi.iterations;
      r->info.n_free = qi.n_free;
      r->info.last_ninf = qi.last_ninf;
      r->info.failed_index = qi.failed_index;
      r->info.ir_steps = qi.ir_steps;
      r->info.min_margin = qi.min_margin;
      r->info.est_rel_err = -1.0;
      finished.push_back(r);
      leaving.push_back(l);   // its block goes back to the pool after the copies out of it
    }
    live.resize(keep);
    if (!finished.empty()) {
      if (hipStreamSynchronize(stream) != hipSuccess) {
        (void)hipGetLastError();
        st = NNLS_ERR_DEVICE;
      }
      for (Live& l : leaving) {
        blocks.put(l.blk, l.cls);
        free_slots.push_back(l.slot);
      }
      if (st != NNLS_OK)
        for (Request* r : finished) r->info.status = st;
      retire(s, finished.data(), finished.size());
    }
  }
  ddesc.release();
  dinfo.release();
  dscat.release();
  blocks.release_all();
  nnls_destroy(h);
  (void)hipStreamDestroy(stream);
}

void free_request(nnls_server* s, Request* r) {
  s->pool.put(r->in, r->in_cls);
  s->pool.put(r->out, r->out_cls);
  delete r;
}

// Hand out a finished request and release its ticket.  Call with s->mu held.
int claim(nnls_server* s, Request* r, double* x, double* y, nnls_info* info) {
  if (x) std::memcpy(x, r->out, sizeof(double) * (size_t)r->n);
  if (y) std::memcpy(y, r->out + r->n, sizeof(double) * (size_t)r->n);
  if (info) *info = r->info;
  const int st = r->info.status;
  s->reqs.erase(r->id);
  free_request(s, r);
  return st;
}

void shutdown(nnls_server* s) {
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  for (std::thread& t : s->threads)
    if (t.joinable()) t.join();
  for (auto& kv : s->reqs) free_request(s, kv.second);
  s->reqs.clear();
}

}  // namespace

extern "C" {

int nnls_server_create(nnls_server** out, int device, const nnls_server_config* cfg,
                       const nnls_options* opts) {
  if (!out) return NNLS_ERR_INVALID_ARG;
  *out = nullptr;
  nnls_server_config c{};
  if (cfg) c = *cfg;
  if (c.workers == 0) c.workers = 16;
  if (c.batch_lanes == 0) c.batch_lanes = 2;
  if (c.batch_max_n == 0) c.batch_max_n = 256;
  if (c.batch_max_count == 0) c.batch_max_count = 1024;
  if (c.batch_step_iters == 0) c.batch_step_iters = 1;
  if (c.workers < 1 || c.workers > 64 || c.batch_lanes < 0 || c.batch_lanes > 16 || c.batch_max_count < 1)
    return NNLS_ERR_INVALID_ARG;
  if (c.batch_max_n < 0) c.batch_lanes = 0;
  if (c.batch_lanes == 0) c.batch_max_n = -1;
  nnls_options o;
  nnls_default_options(&o);
  if (opts) o = *opts;
  o.flags &= ~NNLS_FLAG_PROFILE;
  // several factorisations share the device: each takes a persistent grid of its own, and
  // 16 workers' grids of 96 fill the compute units about three times over
  if (o.max_workgroups == 0) o.max_workgroups = 96;
  if (!(o.tau >= 0.0) || o.p_max < 0 ||
      (o.precision != NNLS_FP64 && o.precision != NNLS_FP32_IR && o.precision != NNLS_BF16_IR) ||
      (o.precision != NNLS_FP64 && (o.ir_max_steps < 0 || !(o.ir_rtol > 0.0))))
    return NNLS_ERR_INVALID_ARG;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
    (void)hipGetLastError();
    return NNLS_ERR_DEVICE;
  }
  if (hipSetDevice(device) != hipSuccess) return NNLS_ERR_DEVICE;
  size_t budget = c.hbm_budget;
  if (budget == 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
      (void)hipGetLastError();
      return NNLS_ERR_DEVICE;
    }
    budget = fr / 10 * 9;
  }
  nnls_server* s = new (std::nothrow) nnls_server();
  if (!s) return NNLS_ERR_NO_MEMORY;
  s->device = device;
  s->opts = o;
  s->cfg = c;
  s->cfg.hbm_budget = budget;
  s->budget = budget;
  s->keep_bytes = std::max<size_t>(budget / (4 * (size_t)c.workers), 1);
  const int nthreads = c.workers + c.batch_lanes;
  try {
    for (int w = 0; w < c.workers; ++w) s->threads.emplace_back(sparse_worker, s);
    for (int w = 0; w < c.batch_lanes; ++w) s->threads.emplace_back(batch_lane, s);
  } catch (...) {
    shutdown(s);
    delete s;
    return NNLS_ERR_NO_MEMORY;
  }
  bool ok;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return s->started + s->failed_start == nthreads; });
    ok = s->failed_start == 0;
  }
  if (!ok) {
    shutdown(s);
    delete s;
    return NNLS_ERR_DEVICE;
  }
  *out = s;
  return NNLS_OK;
}

int nnls_server_submit_csc(nnls_server* s, int32_t m, int32_t n, int64_t nnz, const int32_t* colptr,
                           const int32_t* rowidx, const double* val, const double* b, uint64_t* ticket) {
  if (!s || !ticket || n < 1 || m < n || nnz < 0 || nnz > INT32_MAX || !colptr || !b ||
      (nnz > 0 && (!rowidx || !val)))
    return NNLS_ERR_INVALID_ARG;
  // structure check on the host, before anything indexes with it
  if (colptr[0] != 0 || colptr[n] != nnz) return NNLS_ERR_INVALID_ARG;
  for (int j = 0; j < n; ++j) {
    if (colptr[j + 1] < colptr[j] || colptr[j + 1] > nnz) return NNLS_ERR_INVALID_ARG;
    for (int32_t e = colptr[j]; e < colptr[j + 1]; ++e)
      if (rowidx[e] < 0 || rowidx[e] >= m || (e > colptr[j] && rowidx[e] <= rowidx[e - 1]))
        return NNLS_ERR_INVALID_ARG;
  }
  Request* r = new (std::nothrow) Request();
  if (!r) return NNLS_ERR_NO_MEMORY;
  r->m = m;
  r->n = n;
  r->nnz = nnz;
  r->lane = (s->cfg.batch_max_n >= 0 && n <= s->cfg.batch_max_n) ? LANE_BATCHED : LANE_SPARSE;
  r->L = pack_layout(m, n, nnz);
  r->in = (char*)s->pool.get((size_t)r->L.total, &r->in_cls);
  r->out = (double*)s->pool.get((size_t)n * 16, &r->out_cls);
  if (!r->in || !r->out) {
    free_request(s, r);
    return NNLS_ERR_NO_MEMORY;
  }
  std::memcpy(r->in, colptr, sizeof(int32_t) * ((size_t)n + 1));
  if (nnz > 0) {
    std::memcpy(r->in + r->L.rowidx, rowidx, sizeof(int32_t) * (size_t)nnz);
    std::memcpy(r->in + r->L.val, val, sizeof(double) * (size_t)nnz);
  }
  std::memcpy(r->in + r->L.b, b, sizeof(double) * (size_t)m);
  r->footprint = r->lane == LANE_BATCHED ? batched_footprint(m, n, nnz) : sparse_footprint(m, n, nnz, rowidx);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    r->id = s->next_id++;
    r->t_submit = now_ms();
    if (s->first_submit < 0) s->first_submit = r->t_submit;
    s->submitted += 1;
    s->reqs[r->id] = r;
    s->queue[r->lane].push_back(r);
    *ticket = r->id;
  }
  s->cv_work.notify_all();
  return NNLS_OK;
}

int nnls_server_poll(nnls_server* s, uint64_t ticket, int32_t* done, double* x, double* y, nnls_info* info) {
  if (!s || !done) return NNLS_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return NNLS_ERR_INVALID_ARG;
  *done = it->second->done ? 1 : 0;
  if (!*done) return NNLS_OK;
  return claim(s, it->second, x, y, info);
}

int nnls_server_wait(nnls_server* s, uint64_t ticket, double timeout_ms, double* x, double* y, nnls_info* info) {
  if (!s) return NNLS_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return NNLS_ERR_INVALID_ARG;
  Request* r = it->second;
  const auto finished = [&] { return r->done; };
  if (timeout_ms < 0) {
    s->cv_done.wait(lk, finished);
  } else if (!s->cv_done.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms), finished)) {
    return NNLS_ERR_TIMEOUT;
  }
  return claim(s, r, x, y, info);
}

int nnls_server_stats(nnls_server* s, nnls_serving_stats* out) {
  if (!s || !out) return NNLS_ERR_INVALID_ARG;
  std::vector<double> l;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    std::memset(out, 0, sizeof(*out));
    out->submitted = s->submitted;
    out->completed = (int64_t)s->latencies.size();
    out->pending = (int64_t)(s->queue[0].size() + s->queue[1].size());
    out->batches = s->batches;
    out->running = s->running;
    out->max_running = s->max_running;
    out->committed_bytes = (double)s->committed;
    out->peak_committed_bytes = (double)s->peak_committed;
    out->budget_bytes = (double)s->budget;
    l = s->latencies;
    const double span = s->last_done - s->first_submit;
    out->solves_per_s = (span > 0 && !l.empty()) ? 1e3 * (double)l.size() / span : 0.0;
  }
  if (!l.empty()) {
    std::sort(l.begin(), l.end());
    const auto pct = [&](double q) {   // linear interpolation between order statistics
      const double pos = q * (double)(l.size() - 1);
      const size_t lo = (size_t)pos, hi = std::min(lo + 1, l.size() - 1);
      return l[lo] + (l[hi] - l[lo]) * (pos - (double)lo);
    };
    out->p50_ms = pct(0.5);
    out->p99_ms = pct(0.99);
    out->max_ms = l.back();
    double sum = 0;
    for (double v : l) sum += v;
    out->mean_ms = sum / (double)l.size();
  }
  return NNLS_OK;
}

int nnls_server_reset_stats(nnls_server* s) {
  if (!s) return NNLS_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  s->latencies.clear();
  s->submitted = 0;
  s->batches = 0;
  s->first_submit = -1;
  s->last_done = 0;
  s->max_running = s->running;
  s->peak_committed = s->committed;
  return NNLS_OK;
}

int nnls_server_destroy(nnls_server* s) {
  if (!s) return NNLS_ERR_INVALID_ARG;
  shutdown(s);
  delete s;
  return NNLS_OK;
}

}  // extern "C"
