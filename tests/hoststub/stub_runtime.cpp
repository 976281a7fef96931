// Host-only stand-in for the HIP runtime calls the library's host code makes.  Device and
// pinned memory are host allocations (so the address sanitizer sees every access and every
// free); a stream is a worker thread that runs its enqueued copies and stub kernels in
// order, so host code that reads device results before synchronising, or frees memory a
// queued task still uses, shows up under the thread and address sanitizers.  hipFree waits
// for every stream first, as the HIP runtime's does.
#include <atomic>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "stub_runtime.h"

struct ihipStream_t {
  std::mutex mu;
  std::condition_variable cv, idle;
  std::deque<std::function<void()>> q;
  bool stop = false, busy = false;
  bool capturing = false;                        // tasks go to `captured` instead of q
  std::vector<std::function<void()>> captured;
  std::thread worker;
  ihipStream_t() { worker = std::thread([this] { run(); }); }
  ~ihipStream_t() {
    {
      std::lock_guard<std::mutex> lk(mu);
      stop = true;
    }
    cv.notify_all();
    worker.join();
  }
  void run() {
    for (;;) {
      std::function<void()> f;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] { return stop || !q.empty(); });
        if (q.empty()) return;
        f = std::move(q.front());
        q.pop_front();
        busy = true;
      }
      f();
      {
        std::lock_guard<std::mutex> lk(mu);
        busy = false;
      }
      idle.notify_all();
    }
  }
  void push(std::function<void()> f) {
    {
      std::lock_guard<std::mutex> lk(mu);
      if (capturing) {
        captured.push_back(std::move(f));
        return;
      }
      q.push_back(std::move(f));
    }
    cv.notify_one();
  }
  void sync() {
    std::unique_lock<std::mutex> lk(mu);
    idle.wait(lk, [&] { return q.empty() && !busy; });
  }
};

// An event is a flag that a task on the recording stream sets.
struct ihipEvent_t {
  std::mutex mu;
  std::condition_variable cv;
  bool done = true;
};
struct ihipGraph_t {
  std::vector<std::function<void()>> tasks;
};
struct ihipGraphExec_t {
  std::vector<std::function<void()>> tasks;
};

namespace {
// Live streams; a device-wide wait holds references, so a stream destroyed meanwhile
// lives until that wait is done with it.
std::mutex g_streams_mu;
std::map<ihipStream_t*, std::shared_ptr<ihipStream_t>> g_streams;

ihipStream_t* register_stream() {
  std::shared_ptr<ihipStream_t> st = std::make_shared<ihipStream_t>();
  std::lock_guard<std::mutex> lk(g_streams_mu);
  g_streams[st.get()] = st;
  return st.get();
}

ihipStream_t* default_stream() {
  static ihipStream_t* s = register_stream();
  return s;
}

ihipStream_t* resolve(hipStream_t s) { return s ? s : default_stream(); }

void sync_all() {
  std::vector<std::shared_ptr<ihipStream_t>> all;
  {
    std::lock_guard<std::mutex> lk(g_streams_mu);
    for (auto& kv : g_streams) all.push_back(kv.second);
  }
  for (auto& s : all) s->sync();
}
}  // namespace

void stub_enqueue(hipStream_t s, std::function<void()> task) { resolve(s)->push(std::move(task)); }

hipError_t hipGetDeviceCount(int* count) {
  *count = 1;
  return hipSuccess;
}
hipError_t hipSetDevice(int device) { return device == 0 ? hipSuccess : hipErrorInvalidValue; }
hipError_t hipDeviceGetAttribute(int* value, hipDeviceAttribute_t attr, int) {
  *value = attr == hipDeviceAttributeMultiprocessorCount ? 256 : 100000;
  return hipSuccess;
}
hipError_t hipGetLastError(void) { return hipSuccess; }
hipError_t hipMalloc(void** ptr, size_t bytes) {
  *ptr = std::aligned_alloc(256, (bytes + 255) / 256 * 256);
  return *ptr ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void* ptr) {
  sync_all();   // as the HIP runtime: the device is idle before the memory is released
  std::free(ptr);
  return hipSuccess;
}
hipError_t hipHostMalloc(void** ptr, size_t bytes, unsigned int) { return hipMalloc(ptr, bytes); }
hipError_t hipHostFree(void* ptr) { return hipFree(ptr); }
hipError_t hipMemGetInfo(size_t* free_bytes, size_t* total_bytes) {
  *free_bytes = (size_t)8 << 30;
  *total_bytes = (size_t)16 << 30;
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind, hipStream_t s) {
  if (kind == hipMemcpyHostToDevice) {
    // staged at the call, as a copy from pageable host memory is: the source may be reused
    std::vector<char> stage((const char*)src, (const char*)src + bytes);
    resolve(s)->push([dst, stage = std::move(stage)] { std::memcpy(dst, stage.data(), stage.size()); });
  } else {
    resolve(s)->push([dst, src, bytes] { std::memcpy(dst, src, bytes); });
  }
  return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int) {
  *s = register_stream();
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  if (!s) return hipErrorInvalidValue;
  s->sync();
  std::shared_ptr<ihipStream_t> last;
  {
    std::lock_guard<std::mutex> lk(g_streams_mu);
    auto it = g_streams.find(s);
    if (it == g_streams.end()) return hipErrorInvalidValue;
    last = std::move(it->second);
    g_streams.erase(it);
  }
  return hipSuccess;   // the worker ends when the last reference goes
}
hipError_t hipStreamSynchronize(hipStream_t s) {
  resolve(s)->sync();
  return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t* e) {
  *e = new ihipEvent_t();
  return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
  delete e;
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  {
    std::lock_guard<std::mutex> lk(e->mu);
    e->done = false;
  }
  resolve(s)->push([e] {
    std::lock_guard<std::mutex> lk(e->mu);   // notified under the lock: a waiter may destroy e at once
    e->done = true;
    e->cv.notify_all();
  });
  return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
  std::unique_lock<std::mutex> lk(e->mu);
  e->cv.wait(lk, [&] { return e->done; });
  return hipSuccess;
}
hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind) {
  sync_all();   // as the HIP runtime's blocking copy: after the work queued before it
  std::memcpy(dst, src, bytes);
  return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
  ihipStream_t* st = resolve(s);
  std::lock_guard<std::mutex> lk(st->mu);
  if (st->capturing) return hipErrorInvalidValue;
  st->capturing = true;
  st->captured.clear();
  return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g) {
  ihipStream_t* st = resolve(s);
  std::lock_guard<std::mutex> lk(st->mu);
  if (!st->capturing) return hipErrorInvalidValue;
  st->capturing = false;
  *g = new ihipGraph_t{std::move(st->captured)};
  st->captured.clear();
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
  *e = new ihipGraphExec_t{g->tasks};
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t s) {
  for (const auto& f : e->tasks) resolve(s)->push(f);
  return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t e) {
  delete e;
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
  delete g;
  return hipSuccess;
}
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
  *ms = 0.f;
  return hipSuccess;
}
hipError_t hipGetSymbolAddress(void** ptr, const void* symbol) {
  *ptr = const_cast<void*>(symbol);
  return hipSuccess;
}
