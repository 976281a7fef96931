// Concurrency driver of the host-only sanitizer build: a serving engine with many sparse
// workers and batched lanes under a small device budget (so workspaces are released and
// regrown between requests), fed by several submitting threads, while other threads create
// and destroy their own streams and solver handles and solve on them.  Exits 0 when every
// request and solve returned NNLS_OK with the stand-in kernels' values.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <random>
#include <thread>
#include <vector>

#include <hip/hip_runtime.h>

#include "nnls.h"

namespace {

struct Csc {
  int m, n;
  std::vector<int32_t> colptr, rowidx;
  std::vector<double> val, b;
};

Csc make_problem(std::mt19937& rng, int n) {
  Csc p;
  p.n = n;
  p.m = 3 * n;
  p.colptr.push_back(0);
  std::uniform_int_distribution<int> row(0, p.m - 1);
  std::normal_distribution<double> val(0.0, 1.0);
  for (int j = 0; j < n; ++j) {
    std::vector<int> rows = {j};
    for (int k = 0; k < 4; ++k) rows.push_back(row(rng));
    std::sort(rows.begin(), rows.end());
    rows.erase(std::unique(rows.begin(), rows.end()), rows.end());
    for (int r : rows) {
      p.rowidx.push_back(r);
      p.val.push_back(val(rng));
    }
    p.colptr.push_back((int32_t)p.rowidx.size());
  }
  for (int i = 0; i < p.m; ++i) p.b.push_back(val(rng));
  return p;
}

std::atomic<int> failures{0};

void fail(const char* what, int st) {
  std::fprintf(stderr, "FAIL %s: %d\n", what, st);
  failures += 1;
}

void submitter(nnls_server* s, int seed, int count) {
  std::mt19937 rng(seed);
  std::uniform_int_distribution<int> small(16, 256), large(300, 1400);
  std::vector<uint64_t> tickets;
  std::vector<int> ns;
  for (int r = 0; r < count; ++r) {
    const int n = (r % 3 == 0) ? large(rng) : small(rng);
    const Csc p = make_problem(rng, n);
    uint64_t t = 0;
    const int st = nnls_server_submit_csc(s, p.m, p.n, (int64_t)p.rowidx.size(), p.colptr.data(), p.rowidx.data(),
                                          p.val.data(), p.b.data(), &t);
    if (st != NNLS_OK) {
      fail("submit", st);
      continue;
    }
    tickets.push_back(t);
    ns.push_back(n);
    if (r % 4 == 3) {   // claim an early one without blocking, when it is done
      int32_t done = 0;
      std::vector<double> x((size_t)ns[0]), y((size_t)ns[0]);
      nnls_info info;
      const int ps = nnls_server_poll(s, tickets[0], &done, x.data(), y.data(), &info);
      if (done) {
        if (ps != NNLS_OK) fail("poll", ps);
        tickets.erase(tickets.begin());
        ns.erase(ns.begin());
      }
    }
  }
  for (size_t i = 0; i < tickets.size(); ++i) {
    std::vector<double> x((size_t)ns[i]), y((size_t)ns[i]);
    nnls_info info;
    const int st = nnls_server_wait(s, tickets[i], -1.0, x.data(), y.data(), &info);
    if (st != NNLS_OK) fail("wait", st);
    for (double v : x)
      if (!std::isfinite(v)) fail("x not finite", 0);
  }
}

void direct_solver(int seed, int rounds) {
  std::mt19937 rng(seed);
  std::uniform_int_distribution<int> size(100, 900);
  for (int r = 0; r < rounds; ++r) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      fail("stream", -1);
      return;
    }
    nnls_handle* h = nullptr;
    int rc = nnls_create(&h, 0, (void*)st);
    if (rc != NNLS_OK) {
      fail("create", rc);
      hipStreamDestroy(st);
      return;
    }
    for (int k = 0; k < 3; ++k) {
      const Csc p = make_problem(rng, size(rng));
      const int64_t nnz = (int64_t)p.rowidx.size();
      void *cp, *ri, *va, *b, *x, *y;
      hipMalloc(&cp, sizeof(int32_t) * (p.n + 1));
      hipMalloc(&ri, sizeof(int32_t) * nnz);
      hipMalloc(&va, sizeof(double) * nnz);
      hipMalloc(&b, sizeof(double) * p.m);
      hipMalloc(&x, sizeof(double) * p.n);
      hipMalloc(&y, sizeof(double) * p.n);
      hipMemcpyAsync(cp, p.colptr.data(), sizeof(int32_t) * (p.n + 1), hipMemcpyHostToDevice, st);
      hipMemcpyAsync(ri, p.rowidx.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice, st);
      hipMemcpyAsync(va, p.val.data(), sizeof(double) * nnz, hipMemcpyHostToDevice, st);
      hipMemcpyAsync(b, p.b.data(), sizeof(double) * p.m, hipMemcpyHostToDevice, st);
      nnls_options o;
      nnls_default_options(&o);
      o.precision = (k % 2) ? NNLS_FP32_IR : NNLS_FP64;
      if (k == 2) o.flags = NNLS_FLAG_REFINE_AUTO | NNLS_FLAG_PROFILE;
      nnls_info info;
      rc = nnls_solve_csc(h, p.m, p.n, nnz, (const int32_t*)cp, (const int32_t*)ri, (const double*)va,
                          (const double*)b, (double*)x, (double*)y, &o, &info);
      if (rc != NNLS_OK) fail("solve", rc);
      std::vector<double> xh((size_t)p.n);
      hipMemcpyAsync(xh.data(), x, sizeof(double) * p.n, hipMemcpyDeviceToHost, st);
      hipStreamSynchronize(st);
      for (double v : xh)
        if (!std::isfinite(v)) fail("direct x not finite", 0);
      for (void* q : {cp, ri, va, b, x, y}) hipFree(q);
    }
    nnls_destroy(h);
    hipStreamDestroy(st);
  }
}

// A prepared batch of dense problems replayed from its graph, on the thread's own stream
// and handle, while the server and the other threads run.
void plan_user(int seed, int rounds) {
  std::mt19937 rng(seed);
  std::uniform_int_distribution<int> size(8, 300);
  std::normal_distribution<double> val(0.0, 1.0);
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
    fail("plan stream", -1);
    return;
  }
  nnls_handle* h = nullptr;
  int rc = nnls_create(&h, 0, (void*)st);
  if (rc != NNLS_OK) {
    fail("plan create handle", rc);
    hipStreamDestroy(st);
    return;
  }
  for (int r = 0; r < rounds; ++r) {
    const int batch = 5;
    std::vector<int32_t> m(batch), n(batch), lda(batch);
    std::vector<const double*> A(batch), b(batch);
    std::vector<double*> x(batch), y(batch);
    std::vector<void*> owned;
    for (int i = 0; i < batch; ++i) {
      n[i] = size(rng);
      m[i] = lda[i] = 2 * n[i] + 3;
      std::vector<double> ha((size_t)m[i] * n[i]), hb((size_t)m[i]);
      for (double& v : ha) v = val(rng);
      for (double& v : hb) v = val(rng);
      void *da, *db, *dx, *dy;
      hipMalloc(&da, ha.size() * 8);
      hipMalloc(&db, hb.size() * 8);
      hipMalloc(&dx, (size_t)n[i] * 8);
      hipMalloc(&dy, (size_t)n[i] * 8);
      hipMemcpyAsync(da, ha.data(), ha.size() * 8, hipMemcpyHostToDevice, st);
      hipMemcpyAsync(db, hb.data(), hb.size() * 8, hipMemcpyHostToDevice, st);
      A[i] = (const double*)da;
      b[i] = (const double*)db;
      x[i] = (double*)dx;
      y[i] = (double*)dy;
      for (void* q : {da, db, dx, dy}) owned.push_back(q);
    }
    nnls_options o;
    nnls_default_options(&o);
    o.precision = (r % 2) ? NNLS_FP32_IR : NNLS_FP64;
    nnls_batch_plan* plan = nullptr;
    rc = nnls_batch_plan_create(h, batch, m.data(), n.data(), A.data(), lda.data(), b.data(), x.data(), y.data(),
                                &o, &plan);
    if (rc != NNLS_OK) {
      fail("plan create", rc);
    } else {
      std::vector<nnls_info> info((size_t)batch);
      for (int k = 0; k < 3; ++k) {
        rc = (k == 1) ? nnls_batch_plan_execute(plan, nullptr) : nnls_batch_plan_execute(plan, info.data());
        if (rc == NNLS_OK && k == 1) rc = nnls_batch_plan_info(plan, info.data());
        if (rc != NNLS_OK) fail("plan execute", rc);
      }
      int32_t shapes[9];
      if (nnls_batch_plan_tile_shapes(plan, shapes) != NNLS_OK) fail("plan shapes", -1);
      nnls_batch_plan_destroy(plan);
    }
    for (void* q : owned) hipFree(q);
  }
  nnls_destroy(h);
  hipStreamDestroy(st);
}

}  // namespace

int main() {
  nnls_server_config cfg;
  std::memset(&cfg, 0, sizeof(cfg));
  cfg.workers = 12;
  cfg.batch_lanes = 2;
  cfg.batch_max_n = 256;
  cfg.batch_max_count = 16;
  cfg.hbm_budget = (size_t)48 << 20;   // small: requests wait for admission, workspaces are given back
  nnls_options o;
  nnls_default_options(&o);
  o.precision = NNLS_FP32_IR;
  nnls_server* s = nullptr;
  int rc = nnls_server_create(&s, 0, &cfg, &o);
  if (rc != NNLS_OK) {
    std::fprintf(stderr, "server_create %d\n", rc);
    return 2;
  }
  std::vector<std::thread> th;
  for (int t = 0; t < 4; ++t) th.emplace_back(submitter, s, 100 + t, 36);
  for (int t = 0; t < 3; ++t) th.emplace_back(direct_solver, 200 + t, 4);
  th.emplace_back(plan_user, 300, 4);
  std::atomic<bool> stop{false};
  std::thread stats([&] {
    while (!stop) {
      nnls_serving_stats st;
      nnls_server_stats(s, &st);
      std::this_thread::sleep_for(std::chrono::milliseconds(2));
    }
  });
  for (std::thread& t : th) t.join();
  stop = true;
  stats.join();
  nnls_serving_stats st;
  nnls_server_stats(s, &st);
  nnls_server_reset_stats(s);
  nnls_server_destroy(s);

  // a server destroyed with requests still queued or running
  rc = nnls_server_create(&s, 0, &cfg, &o);
  if (rc != NNLS_OK) return 2;
  std::mt19937 rng(7);
  for (int r = 0; r < 24; ++r) {
    const Csc p = make_problem(rng, r % 2 ? 600 : 64);
    uint64_t t = 0;
    nnls_server_submit_csc(s, p.m, p.n, (int64_t)p.rowidx.size(), p.colptr.data(), p.rowidx.data(), p.val.data(),
                           p.b.data(), &t);
  }
  nnls_server_destroy(s);
  std::printf("completed %lld requests, %d failures\n", (long long)st.completed, failures.load());
  return failures.load() == 0 && st.completed == 4 * 36 ? 0 : 1;
}
