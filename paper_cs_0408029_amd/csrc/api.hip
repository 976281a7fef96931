// Host side of the C ABI: handle, device workspace, and the driver of the block principal
// pivoting loop (Sec. 2 algorithm box of the tsnnls paper).  Every arithmetic step runs
// in the kernels of k_setup / k_pivot / k_chol / k_spmv; the host only sizes launches
// and reads the device control block once per pivot iteration.
#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "nnls_internal.h"

using namespace nnls;

// Device memory of nnls_solve_dense_batched_noalloc: one fixed array per GPU, part of the
// code object.  In host code its name is only a stand-in for the symbol; the device
// address of each GPU's copy is looked up once per device (scratch_address) and used
// wherever host code hands this memory to a kernel or a copy.
static __device__ __align__(256) char scratch[NNLS_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};
bool g_scratch_looked_up[MAX_DEVICES] = {};

// Device address of `scratch` on `device` (current on the calling thread), looked up on
// the first call for that device and kept; nullptr if the lookup failed.
void* scratch_address(int device) {
  if (device < 0 || device >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_looked_up[device]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) {
      (void)hipGetLastError();
      ptr = nullptr;
    }
    g_scratch_ptr[device] = ptr;
    g_scratch_looked_up[device] = true;
  }
  return g_scratch_ptr[device];
}

}  // namespace

namespace {

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  uint64_t gen = 0;   // bumped by every (re)allocation: a new allocation may reuse the
                      // freed address, so only this tells whether the contents were kept
};

struct PendingEvent {
  int cls;
  hipEvent_t a, b;
  double work;
  bool ended;
  int64_t id;
};

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

// A prepared batch: device descriptors, statuses and workspace, and the captured graph of
// one batched solve (see nnls_batch_plan_create).
struct nnls_batch_plan {
  nnls_handle* h = nullptr;
  int batch = 0;
  void* d_probs = nullptr;
  void* d_order = nullptr;
  void* d_info = nullptr;
  void* d_ws = nullptr;
  void* h_info = nullptr;   // pinned copy of the statuses, written by the graph
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  double t0 = 0.0;
  uint8_t shapes[GS_NR + 1] = {};   // tile shape the autotuner chose per ceil(n / 32) (0: none)
};

struct nnls_handle {
  int device = 0;
  hipStream_t stream = nullptr;
  uint64_t wait_ticks = 0;
  int default_wgs = 0;        // factor grid cap when the options give none: the workgroups
                              // the device holds at once (launching one per tile costs
                              // more on large F-blocks)
  int max_wgs = 0;            // the grid cap of the current solve
  // workspace
  DevBuf err, ctrl, rowcnt, rowptr, colidx, valr, hptr, hcnt, hrow, hval, c, r, flags, Flist, pos;
  DevBuf Lt, Dinv, colcnt, dflag, tflag, z, xF, Hd, gF, rpart, spart;
  DevBuf upcnt, prow, pval, pcnt, Fold, zr;   // F-position Gram lists, order scratch, refinement z
  DevBuf wr, bw, bb;                   // sign-certificate bounds of the mixed path
  DevBuf rlo;                          // low part of the compensated refinement residual
  DevBuf Lbf;                          // bfloat16 copies of the factor tiles (NNLS_BF16_IR)
  DevBuf Mc;                           // coupling tiles of the triangular solves' walker
  DevBuf est, ev, exi;                         // condition estimate: state, probe vector, signs
  DevBuf bprobs, border, binfo, bws;   // batched dense problems
  DevBuf scan;                         // chunk sums of the setup prefix scans
  DevBuf slc, srp, sri, srv, sdp, sdi, sdv;   // sliced gathers: counts; residual and dual copies
  Ctrl* h_ctrl = nullptr;     // pinned
  int64_t* h_scalar = nullptr;  // pinned scratch for small reads
  int epoch = 0;
  bool slots_empty = false;   // every hand-over slot of the triangular solves is empty (a
                              // launch that stopped on an error may leave some filled)
  // precision of the factor tiles that belong to the current F order (and the forward-solve
  // blocks with them): 0 float64, 1 float32, -1 none; the next factor of the same
  // precision may keep their untouched leading columns
  int fact_prec = -1;
  // mixed path: the current split's x_F is only sign-certified (not refined to ir_rtol),
  // and the bound on the relative error of the last refined x_F
  bool certified_only = false;
  double err_rel = INFINITY;
  double err_xmax = 0.0;      // max|x_F| that err_rel is relative to
  std::vector<nnls_trace_row> trace;
  // profiling
  bool profiling = false;
  bool profile_always = false;   // nnls_set_profiling
  int64_t prof_launches[NNLS_PROFILE_CLASSES] = {};
  double prof_ms[NNLS_PROFILE_CLASSES] = {};
  double prof_work[NNLS_PROFILE_CLASSES] = {};
  std::vector<hipEvent_t> ev_pool;
  std::vector<PendingEvent> pending;
  int64_t next_event_id = 0;
  void* scratch = nullptr;    // this device's copy of the no-allocation scratch array
};

namespace {

int set_info_status(nnls_info* info, int st) {
  if (info) info->status = st;
  return st;
}

// Grow a device buffer to at least `bytes`.  Flag buffers are zero-filled when they grow.
int ensure(nnls_handle* h, DevBuf& b, size_t bytes, bool zero_i32 = false) {
  if (bytes == 0) bytes = 8;
  if (b.bytes >= bytes) return NNLS_OK;
  if (b.p) {
    if (hipStreamSynchronize(h->stream) != hipSuccess) return NNLS_ERR_DEVICE;
    (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
  }
  if (hipMalloc(&b.p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    return NNLS_ERR_NO_MEMORY;
  }
  b.bytes = bytes;
  b.gen += 1;
  if (zero_i32) launch_fill_i32(h->stream, (int32_t*)b.p, (int64_t)(bytes / 4), 0);
  return NNLS_OK;
}

#define TRY(expr)                  \
  do {                             \
    const int st_ = (expr);        \
    if (st_ != NNLS_OK) return st_; \
  } while (0)

#define HIP_TRY(expr)                                   \
  do {                                                  \
    if ((expr) != hipSuccess) {                         \
      (void)hipGetLastError();                          \
      return NNLS_ERR_DEVICE;                           \
    }                                                   \
  } while (0)

int64_t prof_begin(nnls_handle* h, int cls) {
  if (!h->profiling) return -1;
  PendingEvent pe;
  pe.cls = cls;
  pe.work = 0.0;
  pe.ended = false;
  for (hipEvent_t* e : {&pe.a, &pe.b}) {
    if (!h->ev_pool.empty()) {
      *e = h->ev_pool.back();
      h->ev_pool.pop_back();
    } else if (hipEventCreate(e) != hipSuccess) {
      return -1;
    }
  }
  (void)hipEventRecord(pe.a, h->stream);
  pe.id = h->next_event_id++;
  h->pending.push_back(pe);
  return pe.id;
}

void prof_end(nnls_handle* h, int64_t id, double work) {
  if (id < 0) return;
  for (PendingEvent& pe : h->pending) {
    if (pe.id != id) continue;
    (void)hipEventRecord(pe.b, h->stream);
    pe.work = work;
    pe.ended = true;
    return;
  }
}

// Call only after the stream has been synchronised.  Pairs whose end is not recorded yet
// (a phase that itself reads back from the device) stay pending, at their positions.
void prof_flush(nnls_handle* h) {
  size_t keep = 0;
  for (size_t i = 0; i < h->pending.size(); ++i) {
    PendingEvent& pe = h->pending[i];
    if (!pe.ended) {
      h->pending[keep++] = pe;
      continue;
    }
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, pe.a, pe.b) == hipSuccess) {
      h->prof_launches[pe.cls] += 1;
      h->prof_ms[pe.cls] += ms;
      h->prof_work[pe.cls] += pe.work;
    } else {
      (void)hipGetLastError();
    }
    h->ev_pool.push_back(pe.a);
    h->ev_pool.push_back(pe.b);
  }
  h->pending.resize(keep);
}

int sync_read(nnls_handle* h, void* dst, const void* src, size_t bytes) {
  HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  prof_flush(h);
  return NNLS_OK;
}

int check_options(const nnls_options& o) {
  if (!(o.tau >= 0.0) || !std::isfinite(o.tau)) return NNLS_ERR_INVALID_ARG;
  if (o.p_max < 0) return NNLS_ERR_INVALID_ARG;
  if (o.precision != NNLS_FP64 && o.precision != NNLS_FP32_IR && o.precision != NNLS_BF16_IR)
    return NNLS_ERR_INVALID_ARG;
  if (o.precision != NNLS_FP64 && (o.ir_max_steps < 0 || !(o.ir_rtol > 0.0))) return NNLS_ERR_INVALID_ARG;
  return NNLS_OK;
}

// Factor precisions, from the most accurate: 0 float64; 1 float32; 2 float32 with the
// left-looking updates on bfloat16 copies of the tiles.  Mixed solves start at their
// option's level and step towards 0 when a factor breaks down or refinement stalls.
enum { PREC_F64 = 0, PREC_F32 = 1, PREC_BF16 = 2 };
int prec_level(int precision) {
  return precision == NNLS_BF16_IR ? PREC_BF16 : precision == NNLS_FP32_IR ? PREC_F32 : PREC_F64;
}

// Problem description shared by the sparse and dense drivers.
struct Problem {
  bool sparse;
  int m, n;
  int64_t nnz;
  const int32_t* colptr;
  const int32_t* rowidx;
  const double* val;
  const double* A;
  int lda;
  const double* b;
};

int validate_device(nnls_handle* h, const Problem& P) {
  TRY(ensure(h, h->err, 16));
  launch_fill_i32(h->stream, (int32_t*)h->err.p, 4, 0);
  if (P.sparse)
    launch_validate_csc(h->stream, P.m, P.n, P.nnz, P.colptr, P.rowidx, P.val, P.b, (int32_t*)h->err.p);
  else
    launch_validate_dense(h->stream, P.m, P.n, P.A, P.lda, P.b, (int32_t*)h->err.p);
  int32_t e[4];
  TRY(sync_read(h, e, h->err.p, sizeof(e)));
  if (e[0]) return NNLS_ERR_INVALID_ARG;
  if (e[1]) return NNLS_ERR_INVALID_VALUE;
  return NNLS_OK;
}

int build_csr(nnls_handle* h, const Problem& P) {
  TRY(ensure(h, h->rowcnt, sizeof(int32_t) * (size_t)P.m));
  TRY(ensure(h, h->rowptr, sizeof(int32_t) * ((size_t)P.m + 1)));
  TRY(ensure(h, h->colidx, sizeof(int32_t) * (size_t)P.nnz));
  TRY(ensure(h, h->valr, sizeof(double) * (size_t)P.nnz));
  TRY(ensure(h, h->scan, sizeof(int64_t) * ((size_t)std::max(P.m, P.n) / 2048 + 1)));
  launch_build_csr(h->stream, P.m, P.n, P.nnz, P.colptr, P.rowidx, P.val, (int32_t*)h->rowcnt.p,
                   (int32_t*)h->rowptr.p, (int32_t*)h->colidx.p, (double*)h->valr.p, h->scan.p);
  return NNLS_OK;
}

GramLower gram_view(nnls_handle* h) {
  GramLower g;
  g.hptr = (const int64_t*)h->hptr.p;
  g.hcnt = (const int32_t*)h->hcnt.p;
  g.hrow = (const int32_t*)h->hrow.p;
  g.hval = (const double*)h->hval.p;
  return g;
}

GramPos gram_pos_view(nnls_handle* h) {
  GramPos g;
  g.pptr = (const int64_t*)h->hptr.p;
  g.pcnt = (const int32_t*)h->pcnt.p;
  g.prow = (const int32_t*)h->prow.p;
  g.pval = (const double*)h->pval.p;
  return g;
}

// Gram matrix (lower, padded CSC, then whole columns) and c = A^T b for a validated CSC
// problem.
int build_gram_sparse(nnls_handle* h, const Problem& P) {
  TRY(build_csr(h, P));
  TRY(ensure(h, h->hptr, sizeof(int64_t) * ((size_t)P.n + 1)));
  launch_gram_bound(h->stream, P.n, P.colptr, P.rowidx, (const int32_t*)h->rowptr.p, (int64_t*)h->hptr.p,
                    h->scan.p);
  int64_t ub = 0;
  TRY(sync_read(h, &ub, (int64_t*)h->hptr.p + P.n, sizeof(int64_t)));
  TRY(ensure(h, h->hcnt, sizeof(int32_t) * (size_t)P.n));
  TRY(ensure(h, h->hrow, sizeof(int32_t) * (size_t)ub));
  TRY(ensure(h, h->hval, sizeof(double) * (size_t)ub));
  launch_gram_lower(h->stream, P.n, P.colptr, P.rowidx, P.val, (const int32_t*)h->rowptr.p,
                    (const int32_t*)h->colidx.p, (const double*)h->valr.p, (const int64_t*)h->hptr.p,
                    (int32_t*)h->hcnt.p, (int32_t*)h->hrow.p, (double*)h->hval.p);
  // whole columns (upper entries appended) and room for the F-position lists
  TRY(ensure(h, h->upcnt, sizeof(int32_t) * (size_t)P.n));
  TRY(ensure(h, h->pcnt, sizeof(int32_t) * (size_t)P.n));
  TRY(ensure(h, h->prow, sizeof(int32_t) * (size_t)ub));
  TRY(ensure(h, h->pval, sizeof(double) * (size_t)ub));
  launch_fill_i32(h->stream, (int32_t*)h->upcnt.p, P.n, 0);
  launch_gram_mirror(h->stream, P.n, gram_view(h), (int32_t*)h->upcnt.p, (int32_t*)h->hrow.p, (double*)h->hval.p);
  TRY(ensure(h, h->c, sizeof(double) * (size_t)P.n));
  launch_spmvT_csc(h->stream, P.n, P.colptr, P.rowidx, P.val, P.b, (double*)h->c.p, 1.0);
  return NNLS_OK;
}

int build_gram_dense(nnls_handle* h, const Problem& P) {
  TRY(ensure(h, h->rpart, sizeof(double) * (size_t)dense_residual_chunks(P.m, P.n) * (size_t)P.m));
  TRY(ensure(h, h->Hd, sizeof(double) * (size_t)P.n * (size_t)P.n));
  launch_gram_dense(h->stream, P.m, P.n, P.A, P.lda, (double*)h->Hd.p, P.n);
  TRY(ensure(h, h->c, sizeof(double) * (size_t)P.n));
  launch_gemvT_dense(h->stream, P.m, P.n, P.A, P.lda, P.b, (double*)h->c.p, 1.0);
  return NNLS_OK;
}

// Factor-and-solve workspace for an F-block of order nF at precision level prec.  *lost
// (optional) is set when the tiles, inverted diagonal tiles, forward-solve blocks or
// (bfloat16 level) tile copies had to be reallocated.
int ensure_factor(nnls_handle* h, int nF, int prec, bool* lost = nullptr) {
  const int nb = (nF + TILE - 1) / TILE;
  const size_t w = prec >= PREC_F32 ? sizeof(float) : sizeof(double);
  const size_t ntiles = (size_t)tile_count(nb);
  const uint64_t before[5] = {h->Lt.gen, h->Dinv.gen, h->z.gen, h->Lbf.gen, h->Mc.gen};
  TRY(ensure(h, h->Lt, ntiles * TILE_ELEMS * w));
  if (prec == PREC_BF16) TRY(ensure(h, h->Lbf, ntiles * TILE_ELEMS * sizeof(uint16_t)));
  TRY(ensure(h, h->Dinv, (size_t)nb * TILE_ELEMS * w));
  TRY(ensure(h, h->Mc, walk_coupling_bytes(nb, prec >= PREC_F32)));
  TRY(ensure(h, h->colcnt, (size_t)nb * sizeof(int32_t), true));
  TRY(ensure(h, h->dflag, (size_t)nb * sizeof(int32_t), true));
  TRY(ensure(h, h->tflag, ntiles * sizeof(int32_t), true));
  TRY(ensure(h, h->z, (size_t)nb * TILE * sizeof(double)));
  TRY(ensure(h, h->zr, (size_t)nb * TILE * sizeof(double)));
  TRY(ensure(h, h->xF, (size_t)nb * TILE * sizeof(double)));
  const uint64_t slots_before = h->spart.gen;
  TRY(ensure(h, h->spart, 2 * (size_t)nb * TILE * sizeof(double)));
  if (h->spart.gen != slots_before) h->slots_empty = false;   // fresh memory: not emptied yet
  if (lost)
    *lost = before[0] != h->Lt.gen || before[1] != h->Dinv.gen || before[2] != h->z.gen ||
            (prec == PREC_BF16 && (before[3] != h->Lbf.gen || before[4] != h->Mc.gen));
  return NNLS_OK;
}

FactorArgs factor_args(nnls_handle* h, int nF, const int32_t* Flist, const double* dense, int64_t ldd,
                       bool sparse) {
  FactorArgs a;
  std::memset(&a, 0, sizeof(a));
  a.nF = nF;
  a.nb = (nF + TILE - 1) / TILE;
  a.j0 = 0;
  a.Flist = Flist;
  if (sparse) a.gpos = gram_pos_view(h);
  a.dense = dense;
  a.ldd = ldd;
  a.Ltiles = h->Lt.p;
  a.Mc = h->Mc.p;   // the walker's coupling tiles, formed after the factor
  a.Dinv = h->Dinv.p;
  a.colcnt = (int32_t*)h->colcnt.p;
  a.dflag = (int32_t*)h->dflag.p;
  a.tflag = (int32_t*)h->tflag.p;
  a.epoch = h->epoch;
  a.ctrl = (Ctrl*)h->ctrl.p;
  a.wait_ticks = h->wait_ticks;
  a.max_wgs = h->max_wgs;
  return a;
}

SolveArgs solve_args(nnls_handle* h, int nF, const int32_t* Flist, const double* rhs, double* out) {
  SolveArgs a;
  std::memset(&a, 0, sizeof(a));
  a.nF = nF;
  a.nb = (nF + TILE - 1) / TILE;
  a.Flist = Flist;
  a.Ltiles = h->Lt.p;
  a.Mc = h->Mc.p;
  a.Dinv = h->Dinv.p;
  a.rhs_full = rhs;
  a.rhs_dense = nullptr;
  a.z = (double*)h->z.p;
  a.xF = (double*)h->xF.p;
  a.out = out;
  a.epoch = h->epoch;
  a.ctrl = (Ctrl*)h->ctrl.p;
  a.wait_ticks = h->wait_ticks;
  a.part = (double*)h->spart.p;
  // a factor with bfloat16 updates also has bfloat16 copies of its off-diagonal tiles: the
  // solves read those (half the bytes of L; refinement absorbs the rounding)
  a.Lbf = h->fact_prec == PREC_BF16 ? h->Lbf.p : nullptr;
  if (!h->slots_empty) {   // each launch empties every slot it fills, unless it stopped early
    launch_fill_i32(h->stream, (int32_t*)h->spart.p, (int64_t)(h->spart.bytes / 4), SLOT_EMPTY_WORD);
    h->slots_empty = true;
  }
  return a;
}

// flops of a factor that keeps its leading p0 columns
double chol_flops_from(double nF, double p0) { return (nF * nF * nF - p0 * p0 * p0) / 3.0; }

// Eq. 5 for the refinement, compensated: r = A x - b, y_G = A_G^T r, gfree = A_F^T r.
int residual_dual_dd(nnls_handle* h, const Problem& P, const double* x, double* y, double* gfree) {
  TRY(ensure(h, h->rlo, sizeof(double) * (size_t)P.m));
  launch_residual_dual_dd(h->stream, P.m, P.n, P.nnz, (const int32_t*)h->rowptr.p, (const int32_t*)h->colidx.p,
                          (const double*)h->valr.p, P.colptr, P.rowidx, P.val, P.sparse ? nullptr : P.A, P.lda, x,
                          P.b, (const uint8_t*)h->flags.p, (double*)h->r.p, (double*)h->rlo.p, y, gfree);
  return NNLS_OK;
}

// Eq. 5: r = A x - b, then y_G = A_G^T r (y_F = 0); with gfree also A_F^T r on F.
void residual_dual(nnls_handle* h, const Problem& P, const double* x, double* y, double* gfree) {
  double* r = (double*)h->r.p;
  const uint8_t* flags = (const uint8_t*)h->flags.p;
  if (P.sparse) {
    launch_residual_csr(h->stream, P.m, P.nnz, (const int32_t*)h->rowptr.p, (const int32_t*)h->colidx.p,
                        (const double*)h->valr.p, x, P.b, r);
    launch_dual_csc(h->stream, P.n, P.colptr, P.rowidx, P.val, r, flags, y, gfree);
  } else {
    launch_residual_dense(h->stream, P.m, P.n, P.A, P.lda, x, P.b, r, (double*)h->rpart.p);
    launch_dual_dense(h->stream, P.m, P.n, P.A, P.lda, r, flags, y, gfree);
  }
}

// Float64 iterative refinement of x_F against the residual from A with the factor in the
// handle (float32 when fp32):  g_F = A_F^T (A x - b),  x_F <- x_F - (L L^T)^-1 g_F.
// It stops when the last correction is below ir_rtol max|x_F| (CONVERGE), or -- with certify, for the solve of an intermediate
// split -- as soon as every tested sign is certified by the error bounds of
// launch_ir_certify, since the pivot rule needs only correct signs of x_F and y_G (Sec. 3).
// It stops early when the corrections do not contract or the float32 factor breaks down.
// *outcome: REFINED (target reached; y_G was formed from the final x), CERTIFIED (signs
// certified; y_G was formed from the iterate before the last correction, x is the
// corrected one), STALLED (neither: redo or keep), or REPORT (the control block holds an
// error status for the next control step to report).  *err_rel: bound on the relative
// max-norm error of the final x_F (INF when not measured).
enum RefineOutcome { REFINED = 0, STALLED = 1, REPORT = 2, CERTIFIED = 3 };
int refine(nnls_handle* h, const Problem& P, int nF, double* x, double* y, const nnls_options& o,
           double spmv_bytes, bool fp32, double l_bytes, nnls_info* info, int* outcome, bool certify,
           double* err_rel, double* xmax_out = nullptr) {
  const int32_t* Flist = (const int32_t*)h->Flist.p;
  const uint8_t* flags = (const uint8_t*)h->flags.p;
  Ctrl* ctrl = (Ctrl*)h->ctrl.p;
  *outcome = STALLED;
  *err_rel = INFINITY;
  TRY(ensure(h, h->gF, sizeof(double) * (size_t)P.n));
  double* gF = (double*)h->gF.p;
  double gamma = 0.0;
  if (certify) {
    // per split: the sensitivity of y_G to an error in x_F and the rounding scale of y_G
    TRY(ensure(h, h->bw, sizeof(double) * (size_t)P.n));
    TRY(ensure(h, h->bb, sizeof(double) * (size_t)P.n));
    TRY(ensure(h, h->wr, sizeof(double) * (size_t)P.m));
    if (P.sparse)
      launch_sign_bounds_csr(h->stream, P.m, P.n, P.nnz, (const int32_t*)h->rowptr.p, (const int32_t*)h->colidx.p,
                             (const double*)h->valr.p, P.colptr, P.rowidx, P.val, flags, P.b,
                             (double*)h->wr.p, (double*)h->bw.p, (double*)h->bb.p);
    else
      launch_sign_bounds_dense(h->stream, P.m, P.n, P.A, P.lda, Flist, nF, flags, P.b, (double*)h->wr.p,
                               (double*)h->bw.p, (double*)h->bb.p);
    // 2 gamma_k^2, gamma_k = k u / (1 - k u) for compensated dot products of length
    // k <= m + n + 2 (both products of y_j = a_j^T (A_F x_F - b))
    const double ku = (double)(P.m + P.n + 2) * 1.1102230246251565e-16;
    gamma = 2.0 * (ku / (1.0 - ku)) * (ku / (1.0 - ku));
  }
  bool converged = false;
  double prev = INFINITY;
  for (int step = 0;; ++step) {
    int64_t pe = prof_begin(h, NNLS_PROF_RESIDUAL);
    TRY(residual_dual_dd(h, P, x, y, gF));
    prof_end(h, pe, spmv_bytes);
    if (converged) break;
    if (step >= o.ir_max_steps) break;
    pe = prof_begin(h, NNLS_PROF_REFINE);
    launch_reset_tickets(h->stream, ctrl);
    SolveArgs ca = solve_args(h, nF, Flist, gF, nullptr);
    ca.z = (double*)h->zr.p;   // the factor's own forward-solve blocks stay for the next factor
    launch_trsv(h->stream, ca, fp32, true);
    launch_ir_update(h->stream, nF, Flist, (const double*)h->xF.p, x, ctrl, step == 0 ? 1 : 0);
    if (certify)
      launch_ir_certify(h->stream, P.n, flags, x, y, (const double*)h->bw.p, (const double*)h->bb.p, o.tau, gamma,
                        ctrl);
    prof_end(h, pe, 2.0 * l_bytes);
    TRY(sync_read(h, h->h_ctrl, ctrl, sizeof(Ctrl)));
    if (h->h_ctrl->status == NNLS_ERR_NOT_PD && fp32) {   // float32 breakdown: the caller redoes it
      launch_ctrl_clear_breakdown(h->stream, ctrl);
      h->h_ctrl->status = 0;
      return NNLS_OK;
    }
    if (h->h_ctrl->status != 0) {                  // reported by the next control step
      *outcome = REPORT;
      return NNLS_OK;
    }
    if (info) info->ir_steps += 1;
    const double dmax = h->h_ctrl->ir_dmax, xmax = h->h_ctrl->ir_xmax;
    if (!(dmax < INFINITY) || !(xmax < INFINITY)) break;   // NaN or overflow: stalled
    // While the iteration contracts by 1/2 or better per step (checked on consecutive
    // corrections, rho = dmax / prev), the error left after a step is at most its
    // correction: stop once that is below the target.  (The ratio of consecutive
    // corrections can understate the contraction of the slowest error component, so it
    // only gates the iteration and does not shrink the bound.)
    const double rho = dmax / prev;                 // 0 on the first step
    const double scale = xmax > 0.0 ? xmax : 1.0;
    if (xmax_out) *xmax_out = scale;
    if (dmax <= o.ir_rtol * xmax) {
      converged = true;
      *err_rel = dmax / scale;
    } else if (rho > 0.5) {
      break;                                        // not contracting
    } else if (certify && h->h_ctrl->ir_uncert == 0) {
      *err_rel = h->h_ctrl->ir_err / scale;
      *outcome = CERTIFIED;
      return NNLS_OK;
    }
    prev = dmax;
  }
  *outcome = converged ? REFINED : STALLED;
  return NNLS_OK;
}

// Predicted relative error of the current split's normal-equations solution (the error
// control of Sec. 3): 0.1 * ||H_FF||_1 * est(||H_FF^-1||_1) * 2^-52, with the 1-norm of the
// inverse estimated by Hager's method with Higham's refinements (every solve uses the
// split's float64 factor).  Steps, on F-position vectors:
//   v = 1/n; y = H^-1 v; est = ||y||_1; xi = sign(y); z = H^-1 xi; j = argmax |z|;
//   repeat: y = H^-1 e_j; stop if sign(y) == xi or ||y||_1 <= est (est = the larger);
//           est = ||y||_1; xi = sign(y); z = H^-1 xi; stop if |z| peaks at j again or
//           after five rounds; j = argmax |z|;
//   finally est = max(est, 2 ||H^-1 v'||_1 / (3 n)) with v'_p = (-1)^p (1 + p / (n - 1)).
int estimate_rel_err(nnls_handle* h, const Problem& P, int nF, double* out) {
  const int32_t* Flist = (const int32_t*)h->Flist.p;
  TRY(ensure(h, h->est, sizeof(CondEst)));
  TRY(ensure(h, h->ev, sizeof(double) * (size_t)nF));
  TRY(ensure(h, h->exi, sizeof(double) * (size_t)nF));
  CondEst* est = (CondEst*)h->est.p;
  double* v = (double*)h->ev.p;
  double* xi = (double*)h->exi.p;
  const double* yv = (const double*)h->xF.p;
  Ctrl* ctrl = (Ctrl*)h->ctrl.p;
  CondEst init;
  std::memset(&init, 0, sizeof(init));
  init.j = -1;
  HIP_TRY(hipMemcpyAsync(est, &init, sizeof(init), hipMemcpyHostToDevice, h->stream));
  launch_block_onenorm(h->stream, nF, gram_view(h), (const int32_t*)h->upcnt.p, (const int32_t*)h->pos.p,
                       P.sparse ? nullptr : (const double*)h->Hd.p, P.n, Flist, est);
  // y = H^-1 rhs into xF, with the split's factor
  auto solve = [&](const double* rhs) {
    launch_reset_tickets(h->stream, ctrl);
    SolveArgs sa = solve_args(h, nF, Flist, nullptr, nullptr);
    sa.rhs_full = nullptr;
    sa.rhs_dense = rhs;
    sa.z = (double*)h->zr.p;
    launch_trsv(h->stream, sa, false, true);
  };
  CondEst st;
  auto read = [&]() { return sync_read(h, &st, est, sizeof(CondEst)); };
  double e = 0.0;
  if (nF == 1) {
    launch_est_vec(h->stream, EST_SET_UNIFORM, nF, v, yv, xi, est);
    solve(v);
    launch_est_vec(h->stream, EST_SIGNS, nF, v, yv, xi, est);
    TRY(read());
    e = st.ynorm;
  } else {
    launch_est_vec(h->stream, EST_SET_UNIFORM, nF, v, yv, xi, est);
    solve(v);
    launch_est_vec(h->stream, EST_SIGNS, nF, v, yv, xi, est);
    solve(xi);
    launch_est_vec(h->stream, EST_ARGMAX, nF, v, yv, xi, est);
    TRY(read());
    e = st.ynorm;
    for (int rounds = 2;;) {
      launch_est_vec(h->stream, EST_SET_UNIT, nF, v, yv, xi, est);
      solve(v);
      launch_est_vec(h->stream, EST_SIGNS, nF, v, yv, xi, est);
      TRY(read());
      if (!st.changed || st.ynorm <= e) {
        e = std::max(e, st.ynorm);
        break;
      }
      e = st.ynorm;
      solve(xi);
      launch_est_vec(h->stream, EST_ARGMAX, nF, v, yv, xi, est);
      TRY(read());
      ++rounds;
      if (st.zjlast == st.zmax || rounds > 5) break;
    }
    launch_est_vec(h->stream, EST_SET_ALT, nF, v, yv, xi, est);
    solve(v);
    launch_est_vec(h->stream, EST_SIGNS, nF, v, yv, xi, est);
    TRY(read());
    e = std::max(e, 2.0 * st.ynorm / (3.0 * nF));
  }
  if (!(e < INFINITY) || !(st.hnorm < INFINITY)) {
    *out = INFINITY;
    return NNLS_OK;
  }
  *out = 0.1 * st.hnorm * e * 2.220446049250313e-16;
  return NNLS_OK;
}

// x_F for the current split (Eq. 4 by the normal equations, Sec. 2.1): factor H_FF with
// the forward solve fused, then the backward solve scattered into x.  In the mixed
// precisions the factor is float32 (NNLS_BF16_IR: its updates from bfloat16 tile copies)
// and x_F is refined in float64 against the residual from A,
//   g_F = A_F^T (A x - b),  x_F <- x_F - (L L^T)^-1 g_F,
// until every tested sign is certified (certify: an intermediate split, Sec. 3) or the
// correction is below ir_rtol relative to x_F; if the factor breaks down, refinement stalls
// or the step cap is reached, the iteration is redone one precision level up (bfloat16
// updates -> float32 -> float64) and refined again.  force64 starts with the float64
// factor.  *y_done is set when the last refinement pass already left y_G (for the final
// x, or certified).
// j0: leading tile columns the control step kept from the previous factor (the first
// attempt may use them; *j0_used reports what it did).
int solve_free(nnls_handle* h, const Problem& P, int nF, int j0, double* x, double* y, const nnls_options& o,
               double spmv_bytes, bool* y_done, int* j0_used, nnls_info* info, bool certify, bool force64) {
  const int32_t* Flist = (const int32_t*)h->Flist.p;
  const bool mixed = o.precision != NNLS_FP64;
  int prec = force64 ? PREC_F64 : prec_level(o.precision);
  *y_done = false;
  *j0_used = 0;
  h->certified_only = false;
  h->err_rel = INFINITY;
  if (P.sparse)
    launch_gram_positions(h->stream, nF, gram_view(h), (const int32_t*)h->upcnt.p, Flist,
                          (const int32_t*)h->pos.p, (int32_t*)h->pcnt.p, (int32_t*)h->prow.p,
                          (double*)h->pval.p);
  for (int attempt = 0;; ++attempt) {
    const bool fp32 = prec >= PREC_F32;
    bool lost = false;
    TRY(ensure_factor(h, nF, prec, &lost));
    h->epoch += 1;
    if (attempt > 0 || force64) {
      // the control step zeroed the column counters and tickets for the first attempt
      // only: the first factor left its columns counted complete, and the refinement's
      // triangular solves used up the solve tickets
      launch_fill_i32(h->stream, (int32_t*)h->colcnt.p, (nF + TILE - 1) / TILE, 0);
      launch_reset_tickets(h->stream, (Ctrl*)h->ctrl.p);
    }
    FactorArgs fa = factor_args(h, nF, Flist, P.sparse ? nullptr : (const double*)h->Hd.p,
                                P.sparse ? 0 : P.n, P.sparse);
    fa.j0 = (attempt == 0 && !force64 && !lost && h->fact_prec == prec) ? std::min(j0, fa.nb - 1) : 0;
    if (attempt == 0) *j0_used = fa.j0;
    fa.rhs = (const double*)h->c.p;
    fa.z = (double*)h->z.p;
    fa.Lbf = prec == PREC_BF16 ? h->Lbf.p : nullptr;
    int64_t pe = prof_begin(h, NNLS_PROF_CHOLESKY);
    launch_cholesky(h->stream, fa, fp32);
    prof_end(h, pe, chol_flops_from(nF, (double)fa.j0 * TILE));
    h->fact_prec = prec;
    const double l_bytes = (fp32 ? 4.0 : 8.0) * (double)tile_count(fa.nb) * TILE_ELEMS;
    SolveArgs sa = solve_args(h, nF, Flist, (const double*)h->c.p, x);
    pe = prof_begin(h, NNLS_PROF_TRSV);
    launch_trsv(h->stream, sa, fp32, false);
    prof_end(h, pe, l_bytes);
    if (!mixed) return NNLS_OK;

    // refined against the residual from A; after a float64 redo as well, so that the mixed
    // path is never less accurate than the refined float64 solution
    int outcome = STALLED;
    double err = INFINITY;
    double xm = 0.0;
    TRY(refine(h, P, nF, x, y, o, spmv_bytes, fp32, l_bytes, info, &outcome, certify, &err, &xm));
    if (outcome == REPORT) return NNLS_OK;          // reported by the next control step
    if (outcome == REFINED || outcome == CERTIFIED) {
      *y_done = true;
      h->certified_only = outcome == CERTIFIED;
      h->err_rel = err;
      h->err_xmax = xm;
      return NNLS_OK;
    }
    if (prec == PREC_F64) return NNLS_OK;   // the float64 factor does not contract either: keep x_F
    prec -= 1;
  }
}

// The pivot loop on a problem whose Gram matrix and c are built.
int pivot_loop(nnls_handle* h, const Problem& P, double* x, double* y, const nnls_options& o,
               nnls_info* info) {
  const int n = P.n, m = P.m;
  TRY(ensure(h, h->flags, (size_t)n));
  TRY(ensure(h, h->Flist, sizeof(int32_t) * (size_t)n));
  TRY(ensure(h, h->pos, sizeof(int32_t) * (size_t)n));
  TRY(ensure(h, h->Fold, sizeof(int32_t) * (size_t)n));
  TRY(ensure(h, h->r, sizeof(double) * (size_t)m));
  TRY(ensure(h, h->ctrl, sizeof(Ctrl)));
  const int ncol = (n + TILE - 1) / TILE;
  h->fact_prec = -1;
  const int want_prec = prec_level(o.precision);
  const bool reuse = (o.flags & NNLS_FLAG_NO_FACTOR_REUSE) == 0;
  const bool gram_dual = (o.flags & NNLS_FLAG_GRAM_DUAL) != 0 && !P.sparse;   // Eq. 3 for y_G
  TRY(ensure(h, h->colcnt, sizeof(int32_t) * (size_t)ncol, true));
  TRY(ensure(h, h->dflag, sizeof(int32_t) * (size_t)ncol, true));
  const int max_iter = o.max_iter > 0 ? o.max_iter : 5 * n + 100;
  uint8_t* flags = (uint8_t*)h->flags.p;
  int32_t* Flist = (int32_t*)h->Flist.p;
  int32_t* pos = (int32_t*)h->pos.p;
  Ctrl* ctrl = (Ctrl*)h->ctrl.p;
  launch_pivot_init(h->stream, n, (const double*)h->c.p, x, y, flags, ctrl, o.p_max);

  // bytes moved by the classify / exchange sweep and by the residual + dual sweep
  const double ctrl_bytes = 2.0 * 17.0 * n;
  const double spmv_bytes = P.sparse ? (2.0 * 12.0 * (double)P.nnz + 32.0 * m + 24.0 * n)
                                     : (2.0 * 8.0 * (double)m * n + 32.0 * m + 24.0 * n);
  // NNLS_FLAG_REFINE_FINAL: once a split is feasible, refine its x_F in float64 against the
  // residual from A with the split's own factor, and classify the refined x and y again
  const bool auto_refine = (o.flags & NNLS_FLAG_REFINE_AUTO) != 0 && o.precision == NNLS_FP64;
  const bool final_refine = ((o.flags & NNLS_FLAG_REFINE_FINAL) != 0 || auto_refine) && o.precision == NNLS_FP64;
  const bool mixed = o.precision != NNLS_FP64;
  const bool certify = mixed && (o.flags & NNLS_FLAG_REFINE_ALL) == 0;   // intermediate splits
  bool refined = false;
  int last_nF = 0;
  h->certified_only = false;
  h->err_rel = INFINITY;
  for (;;) {
    int64_t pe = prof_begin(h, NNLS_PROF_CONTROL);
    // ordered F; the previous factor's untouched leading tiles are kept when its
    // precision is the one the next factor starts in
    launch_pivot_control(h->stream, n, x, y, flags, Flist, pos, ctrl, o.tau, o.p_max, max_iter,
                         (int32_t*)h->colcnt.p, ncol, (int32_t*)h->Fold.p,
                         reuse && h->fact_prec == want_prec ? 2 : 1);
    prof_end(h, pe, ctrl_bytes);
    TRY(sync_read(h, h->h_ctrl, ctrl, sizeof(Ctrl)));
    const Ctrl c = *h->h_ctrl;
    if (c.status != 0) break;
    if (c.done) {
      if (mixed && h->certified_only && !refined && last_nF > 0) {
        // the feasible split's x_F was refined only until its signs were certified:
        // refine it to ir_rtol with the split's factor, then classify again
        int outcome = STALLED;
        double err = INFINITY;
        const int ir_before = info ? info->ir_steps : 0;
        const bool f32 = h->fact_prec >= PREC_F32;
        const double l_bytes = (f32 ? 4.0 : 8.0) * (double)tile_count((last_nF + TILE - 1) / TILE) * TILE_ELEMS;
        double xm = 0.0;
        TRY(refine(h, P, last_nF, x, y, o, spmv_bytes, f32, l_bytes, info, &outcome, false, &err, &xm));
        refined = true;
        if (!h->trace.empty() && info) h->trace.back().ir_steps += info->ir_steps - ir_before;
        if (outcome == REPORT) continue;
        if (outcome == REFINED) {
          h->certified_only = false;
          h->err_rel = err;
          h->err_xmax = xm;
          continue;
        }
        // not contracting to the target: this split again with a float64 factor
        bool yd = false;
        int j0u = 0;
        const int ir_mid = info ? info->ir_steps : 0;
        TRY(solve_free(h, P, last_nF, 0, x, y, o, spmv_bytes, &yd, &j0u, info, false, true));
        if (!h->trace.empty() && info) h->trace.back().ir_steps += info->ir_steps - ir_mid;
        if (!yd) {
          pe = prof_begin(h, NNLS_PROF_RESIDUAL);
          residual_dual(h, P, x, y, nullptr);
          prof_end(h, pe, spmv_bytes);
        }
        continue;
      }
      if (!final_refine || refined || last_nF == 0) break;
      if (auto_refine && !(o.flags & NNLS_FLAG_REFINE_FINAL)) {
        // refine only when the split's predicted error misses the target
        double est_rel = INFINITY;
        const int64_t pe2 = prof_begin(h, NNLS_PROF_REFINE);
        TRY(estimate_rel_err(h, P, last_nF, &est_rel));
        prof_end(h, pe2, 0.0);
        if (info) info->est_rel_err = est_rel;
        if (est_rel <= o.ir_rtol) break;
      }
      int outcome = STALLED;
      const double l_bytes = 8.0 * (double)tile_count((last_nF + TILE - 1) / TILE) * TILE_ELEMS;
      double err_unused = INFINITY;
      TRY(refine(h, P, last_nF, x, y, o, spmv_bytes, false, l_bytes, info, &outcome, false, &err_unused));
      if (outcome == REPORT) {       // keep the split; the control step reports the status
        refined = true;
        continue;
      }
      if (outcome != REFINED) {
        pe = prof_begin(h, NNLS_PROF_RESIDUAL);
        residual_dual(h, P, x, y, nullptr);
        prof_end(h, pe, spmv_bytes);
      }
      refined = true;
      continue;
    }
    refined = false;
    nnls_trace_row row;
    row.k = c.k;
    row.branch = c.branch;
    row.N = c.N;
    row.p = c.p;
    row.n_free = c.n_free;
    row.n_reused = 0;
    const int ir_before = info ? info->ir_steps : 0;
    const int nF = c.n_free;
    last_nF = nF;
    bool y_done = false;
    int j0_used = 0;
    if (nF > 0) TRY(solve_free(h, P, nF, c.j0, x, y, o, spmv_bytes, &y_done, &j0_used, info, certify, false));
    row.n_reused = j0_used * TILE;
    row.ir_steps = info ? info->ir_steps - ir_before : 0;
    h->trace.push_back(row);
    if (!y_done && gram_dual) {
      pe = prof_begin(h, NNLS_PROF_DUAL);
      launch_dual_gram_dense(h->stream, n, (const double*)h->Hd.p, n, (const double*)h->c.p, flags, Flist, nF, x, y);
      prof_end(h, pe, 8.0 * (double)(n - nF) * nF + 8.0 * nF + 17.0 * n);
    } else if (!y_done) {
      pe = prof_begin(h, NNLS_PROF_RESIDUAL);
      residual_dual(h, P, x, y, nullptr);
      prof_end(h, pe, spmv_bytes);
    }
    if (hipGetLastError() != hipSuccess) return NNLS_ERR_DEVICE;
  }
  const Ctrl c = *h->h_ctrl;
  if (info) {
    info->iterations = c.iter;
    info->n_free = c.n_free;
    info->last_ninf = c.k;
    info->min_margin = c.min_margin;
    info->failed_index = -1;
    if (mixed) info->est_rel_err = -1.0;
    if (mixed && c.status == NNLS_OK) {
      if (last_nF == 0) {
        info->est_rel_err = 0.0;
      } else if (h->err_rel < INFINITY && !h->certified_only) {
        // the remaining correction plus the rounding of x_F itself (the compensated
        // residual leaves an error far below both)
        info->est_rel_err = h->err_rel + 2.220446049250313e-16;
      }
    }
  }
  if (c.status == NNLS_ERR_NOT_PD) {
    int32_t col = -1;
    if (c.failed_pos >= 0 && c.failed_pos < n)
      TRY(sync_read(h, &col, Flist + c.failed_pos, sizeof(int32_t)));
    if (info) info->failed_index = col;
  }
  return c.status;
}

int solve_common(nnls_handle* h, const Problem& P, double* x, double* y, const nnls_options* opts,
                 nnls_info* info) {
  const double t0 = now_ms();
  nnls_options o;
  nnls_default_options(&o);
  if (opts) o = *opts;
  nnls_info local;   // the loop records its counts (refinement steps per trace row) in info
  if (!info) info = &local;
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->failed_index = -1;
    info->est_rel_err = -1.0;
  }
  if (!h) return set_info_status(info, NNLS_ERR_INVALID_ARG);
  h->trace.clear();
  if (check_options(o) != NNLS_OK) return set_info_status(info, NNLS_ERR_INVALID_ARG);
  if (P.n < 1 || P.m < P.n || !P.b || !x || !y) return set_info_status(info, NNLS_ERR_INVALID_ARG);
  if (P.sparse) {
    if (P.nnz < 0 || P.nnz > INT32_MAX || !P.colptr || (P.nnz > 0 && (!P.rowidx || !P.val)))
      return set_info_status(info, NNLS_ERR_INVALID_ARG);
  } else {
    if (!P.A || P.lda < P.m) return set_info_status(info, NNLS_ERR_INVALID_ARG);
  }
  if (hipSetDevice(h->device) != hipSuccess) return set_info_status(info, NNLS_ERR_DEVICE);
  h->profiling = h->profile_always || (o.flags & NNLS_FLAG_PROFILE) != 0;
  h->max_wgs = o.max_workgroups > 0 ? (int)std::min<uint32_t>(o.max_workgroups, 1u << 20) : h->default_wgs;
  int st = validate_device(h, P);
  if (st != NNLS_OK) return set_info_status(info, st);
  const int64_t pe = prof_begin(h, NNLS_PROF_GRAM);
  st = P.sparse ? build_gram_sparse(h, P) : build_gram_dense(h, P);
  if (st != NNLS_OK) return set_info_status(info, st);
  prof_end(h, pe, P.sparse ? 12.0 * (double)P.nnz * 3.0 : 8.0 * (double)P.m * P.n);
  if (hipStreamSynchronize(h->stream) != hipSuccess) return set_info_status(info, NNLS_ERR_DEVICE);
  prof_flush(h);
  if (info) info->setup_ms = now_ms() - t0;
  st = pivot_loop(h, P, x, y, o, info);
  if (st != NNLS_OK) h->slots_empty = false;   // a solve may have stopped with slots filled
  if (info) info->solve_ms = now_ms() - t0;
  h->profiling = h->profile_always;
  return set_info_status(info, st);
}

}  // namespace

namespace nnls {

// Give back every device buffer of the handle (the next solve allocates them again).
void release_workspace(nnls_handle* h) {
  if (!h) return;
  (void)hipSetDevice(h->device);
  (void)hipStreamSynchronize(h->stream);
  h->fact_prec = -1;
  DevBuf* bufs[] = {&h->err, &h->ctrl, &h->rowcnt, &h->rowptr, &h->colidx, &h->valr, &h->hptr,
                    &h->hcnt, &h->hrow, &h->hval, &h->c, &h->r, &h->flags, &h->Flist, &h->pos,
                    &h->Lt, &h->Dinv, &h->colcnt, &h->dflag, &h->tflag, &h->z, &h->xF, &h->Hd, &h->gF, &h->rpart, &h->spart,
                    &h->upcnt, &h->prow, &h->pval, &h->pcnt, &h->Fold, &h->zr, &h->est, &h->ev, &h->exi,
                    &h->bprobs, &h->border, &h->binfo, &h->bws, &h->scan, &h->wr, &h->bw, &h->bb, &h->rlo, &h->Lbf,
                    &h->Mc, &h->slc, &h->srp, &h->sri, &h->srv, &h->sdp, &h->sdi, &h->sdv};
  for (DevBuf* b : bufs) {
    if (b->p) (void)hipFree(b->p);
    b->p = nullptr;
    b->bytes = 0;
  }
}

}  // namespace nnls

extern "C" {

const char* nnls_status_string(int status) {
  switch (status) {
    case NNLS_OK: return "NNLS_OK";
    case NNLS_ERR_INVALID_ARG: return "NNLS_ERR_INVALID_ARG";
    case NNLS_ERR_INVALID_VALUE: return "NNLS_ERR_INVALID_VALUE";
    case NNLS_ERR_NOT_PD: return "NNLS_ERR_NOT_PD";
    case NNLS_ERR_MAXITER: return "NNLS_ERR_MAXITER";
    case NNLS_ERR_NO_MEMORY: return "NNLS_ERR_NO_MEMORY";
    case NNLS_ERR_DEVICE: return "NNLS_ERR_DEVICE";
    case NNLS_ERR_REFINE: return "NNLS_ERR_REFINE";
    case NNLS_ERR_TIMEOUT: return "NNLS_ERR_TIMEOUT";
    case NNLS_ERR_TOO_LARGE: return "NNLS_ERR_TOO_LARGE";
    default: return "NNLS_ERR_UNKNOWN";
  }
}

void nnls_default_options(nnls_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->tau = 1e-12;
  o->p_max = 3;
  o->max_iter = 0;
  o->precision = NNLS_FP64;
  o->ir_max_steps = 10;
  o->ir_rtol = 1e-12;
  o->flags = 0;
}

int nnls_create(nnls_handle** out, int device, void* stream) {
  if (!out) return NNLS_ERR_INVALID_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
    (void)hipGetLastError();
    return NNLS_ERR_DEVICE;
  }
  if (hipSetDevice(device) != hipSuccess) return NNLS_ERR_DEVICE;
  nnls_handle* h = new (std::nothrow) nnls_handle();
  if (!h) return NNLS_ERR_NO_MEMORY;
  h->device = device;
  h->stream = (hipStream_t)stream;
  int rate_khz = 0;
  if (hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, device) != hipSuccess || rate_khz <= 0)
    rate_khz = 100000;
  h->wait_ticks = (uint64_t)rate_khz * 1000ull * 20ull;   // 20 s
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus <= 0)
    cus = 256;
  h->default_wgs = 2 * cus;

  if (hipHostMalloc((void**)&h->h_ctrl, sizeof(Ctrl), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&h->h_scalar, 64, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    nnls_destroy(h);
    return NNLS_ERR_NO_MEMORY;
  }
  std::memset(h->h_ctrl, 0, sizeof(Ctrl));
  // library set-up per device: the device address of the no-allocation scratch array
  // (looked up once per device; a failure is reported by the entry point that needs it)
  h->scratch = scratch_address(device);
  *out = h;
  return NNLS_OK;
}

int nnls_destroy(nnls_handle* h) {
  if (!h) return NNLS_ERR_INVALID_ARG;
  (void)hipSetDevice(h->device);
  (void)hipStreamSynchronize(h->stream);
  DevBuf* bufs[] = {&h->err, &h->ctrl, &h->rowcnt, &h->rowptr, &h->colidx, &h->valr, &h->hptr,
                    &h->hcnt, &h->hrow, &h->hval, &h->c, &h->r, &h->flags, &h->Flist, &h->pos,
                    &h->Lt, &h->Dinv, &h->colcnt, &h->dflag, &h->tflag, &h->z, &h->xF, &h->Hd, &h->gF, &h->rpart, &h->spart,
                    &h->upcnt, &h->prow, &h->pval, &h->pcnt, &h->Fold, &h->zr, &h->est, &h->ev, &h->exi,
                    &h->bprobs, &h->border, &h->binfo, &h->bws, &h->scan, &h->wr, &h->bw, &h->bb, &h->rlo, &h->Lbf,
                    &h->Mc, &h->slc, &h->srp, &h->sri, &h->srv, &h->sdp, &h->sdi, &h->sdv};
  for (DevBuf* b : bufs)
    if (b->p) (void)hipFree(b->p);
  for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
  for (PendingEvent& pe : h->pending) {
    (void)hipEventDestroy(pe.a);
    (void)hipEventDestroy(pe.b);
  }
  if (h->h_ctrl) (void)hipHostFree(h->h_ctrl);
  if (h->h_scalar) (void)hipHostFree(h->h_scalar);
  delete h;
  return NNLS_OK;
}

int nnls_solve_csc(nnls_handle* h, int32_t m, int32_t n, int64_t nnz, const int32_t* colptr,
                   const int32_t* rowidx, const double* val, const double* b, double* x, double* y,
                   const nnls_options* opts, nnls_info* info) {
  Problem P;
  std::memset(&P, 0, sizeof(P));
  P.sparse = true;
  P.m = m;
  P.n = n;
  P.nnz = nnz;
  P.colptr = colptr;
  P.rowidx = rowidx;
  P.val = val;
  P.b = b;
  return solve_common(h, P, x, y, opts, info);
}

int nnls_solve_dense(nnls_handle* h, int32_t m, int32_t n, const double* A, int32_t lda,
                     const double* b, double* x, double* y, const nnls_options* opts, nnls_info* info) {
  Problem P;
  std::memset(&P, 0, sizeof(P));
  P.sparse = false;
  P.m = m;
  P.n = n;
  P.A = A;
  P.lda = lda;
  P.b = b;
  return solve_common(h, P, x, y, opts, info);
}

int nnls_solve_dense_batched(nnls_handle* h, int32_t batch, const int32_t* m, const int32_t* n,
                             const double* const* A, const int32_t* lda, const double* const* b,
                             double* const* x, double* const* y, const nnls_options* opts,
                             nnls_info* info) {
  nnls_options o;
  nnls_default_options(&o);
  if (opts) o = *opts;
  if (!h || batch < 0 || (batch > 0 && (!m || !n || !A || !lda || !b || !x || !y)))
    return NNLS_ERR_INVALID_ARG;
  if (check_options(o) != NNLS_OK) return NNLS_ERR_INVALID_ARG;
  if (o.precision == NNLS_BF16_IR) o.precision = NNLS_FP32_IR;   // the batched path's float32 tier
  if (info)
    for (int i = 0; i < batch; ++i) {
      std::memset(&info[i], 0, sizeof(nnls_info));
      info[i].failed_index = -1;
      info[i].est_rel_err = -1.0;
    }
  if (batch == 0) return NNLS_OK;
  for (int i = 0; i < batch; ++i) {
    if (n[i] < 1 || m[i] < n[i] || lda[i] < m[i] || !A[i] || !b[i] || !x[i] || !y[i]) {
      if (info) info[i].status = NNLS_ERR_INVALID_ARG;
      return NNLS_ERR_INVALID_ARG;
    }
  }
  if (hipSetDevice(h->device) != hipSuccess) return NNLS_ERR_DEVICE;
  const double t0 = now_ms();
  std::vector<BatchProblem> probs((size_t)batch);
  std::vector<int32_t> order((size_t)batch);
  size_t total = 0;
  for (int i = 0; i < batch; ++i) {
    BatchProblem& bp = probs[(size_t)i];
    bp.m = m[i];
    bp.n = n[i];
    bp.lda = lda[i];
    bp.pad = 0;
    bp.A = A[i];
    bp.b = b[i];
    bp.x = x[i];
    bp.y = y[i];
    bp.info = nullptr;   // set below, once the device arrays exist
    bp.ws = (char*)(uintptr_t)total;
    total += batched_workspace_bytes(m[i], n[i]);
    order[(size_t)i] = i;
  }
  // largest work first, so the tail of the launch is made of small problems
  std::stable_sort(order.begin(), order.end(), [&](int a_, int b_) {
    const double wa = (double)n[a_] * n[a_] * (m[a_] + n[a_]);
    const double wb = (double)n[b_] * n[b_] * (m[b_] + n[b_]);
    return wa > wb;
  });
  TRY(ensure(h, h->bprobs, sizeof(BatchProblem) * (size_t)batch));
  TRY(ensure(h, h->border, sizeof(int32_t) * (size_t)batch));
  TRY(ensure(h, h->binfo, sizeof(BatchInfo) * (size_t)batch));
  TRY(ensure(h, h->bws, total));
  for (int i = 0; i < batch; ++i) {
    probs[(size_t)i].info = (BatchInfo*)h->binfo.p + i;
    probs[(size_t)i].ws = (char*)h->bws.p + (uintptr_t)probs[(size_t)i].ws;
  }
  HIP_TRY(hipMemcpyAsync(h->bprobs.p, probs.data(), sizeof(BatchProblem) * (size_t)batch,
                         hipMemcpyHostToDevice, h->stream));
  HIP_TRY(hipMemcpyAsync(h->border.p, order.data(), sizeof(int32_t) * (size_t)batch,
                         hipMemcpyHostToDevice, h->stream));
  BatchArgs ba;
  std::memset(&ba, 0, sizeof(ba));
  ba.count = batch;
  ba.probs = (const BatchProblem*)h->bprobs.p;
  ba.order = (const int32_t*)h->border.p;
  ba.tau = o.tau;
  ba.p_max = o.p_max;
  ba.max_iter = o.max_iter;
  ba.fp32 = o.precision == NNLS_FP32_IR ? 1 : 0;
  ba.ir_max_steps = o.ir_max_steps;
  ba.ir_rtol = o.ir_rtol;
  ba.gram_dual = (o.flags & NNLS_FLAG_GRAM_DUAL) != 0 ? 1 : 0;
  h->profiling = h->profile_always || (o.flags & NNLS_FLAG_PROFILE) != 0;
  double flops = 0.0;
  for (int i = 0; i < batch; ++i) flops += (double)n[i] * n[i] * m[i];
  const int64_t pg = prof_begin(h, NNLS_PROF_BATCHED_GRAM);
  launch_batched_gram(h->stream, ba, batch);
  prof_end(h, pg, flops);
  const int64_t pe = prof_begin(h, NNLS_PROF_BATCHED);
  launch_batched_steps(h->stream, ba, batch);   // max_steps 0: every problem to the end
  prof_end(h, pe, flops);
  std::vector<BatchInfo> bi((size_t)batch);
  const int st = sync_read(h, bi.data(), h->binfo.p, sizeof(BatchInfo) * (size_t)batch);
  h->profiling = h->profile_always;
  if (st != NNLS_OK) return st;
  if (hipGetLastError() != hipSuccess) return NNLS_ERR_DEVICE;
  const double el = now_ms() - t0;
  int worst = NNLS_OK;
  for (int i = 0; i < batch; ++i) {
    const BatchInfo& q = bi[(size_t)i];
    if (info) {
      info[i].status = q.status;
      info[i].iterations = q.iterations;
      info[i].n_free = q.n_free;
      info[i].last_ninf = q.last_ninf;
      info[i].failed_index = q.failed_index;
      info[i].ir_steps = q.ir_steps;
      info[i].min_margin = q.min_margin;
      info[i].solve_ms = el;
    }
    if (q.status != NNLS_OK && worst == NNLS_OK) worst = q.status;
  }
  return worst;
}

int nnls_solve_dense_batched_noalloc(nnls_handle* h, int32_t batch, const int32_t* m, const int32_t* n,
                                     const double* const* A, const int32_t* lda, const double* const* b,
                                     double* const* x, double* const* y, const nnls_options* opts,
                                     nnls_info* info) {
  nnls_options o;
  nnls_default_options(&o);
  if (opts) o = *opts;
  if (!h || batch < 0 || (batch > 0 && (!m || !n || !A || !lda || !b || !x || !y)))
    return NNLS_ERR_INVALID_ARG;
  if (check_options(o) != NNLS_OK) return NNLS_ERR_INVALID_ARG;
  if (o.precision == NNLS_BF16_IR) o.precision = NNLS_FP32_IR;   // the batched path's float32 tier
  if (info)
    for (int i = 0; i < batch; ++i) {
      std::memset(&info[i], 0, sizeof(nnls_info));
      info[i].failed_index = -1;
      info[i].est_rel_err = -1.0;
    }
  if (batch == 0) return NNLS_OK;
  // layout in the scratch array: descriptors | statuses | workspaces, each 256-byte aligned
  const auto align256 = [](size_t v) { return (v + 255) & ~(size_t)255; };
  const size_t probs_off = 0;
  const size_t info_off = align256(sizeof(BatchProblem) * (size_t)batch);
  const size_t ws_off = info_off + align256(sizeof(BatchInfo) * (size_t)batch);
  size_t total = ws_off;
  for (int i = 0; i < batch; ++i) {
    if (n[i] < 1 || m[i] < n[i] || lda[i] < m[i] || !A[i] || !b[i] || !x[i] || !y[i]) {
      if (info) info[i].status = NNLS_ERR_INVALID_ARG;
      return NNLS_ERR_INVALID_ARG;
    }
    total += batched_workspace_bytes(m[i], n[i]);
    if (total > NNLS_NOALLOC_SCRATCH_BYTES) return NNLS_ERR_TOO_LARGE;
  }
  if (hipSetDevice(h->device) != hipSuccess) return NNLS_ERR_DEVICE;
  char* base = (char*)h->scratch;
  if (!base) return NNLS_ERR_DEVICE;   // the symbol lookup at set-up failed
  const double t0 = now_ms();
  // descriptors: built on the host a chunk at a time and copied into the scratch array
  constexpr int CHUNK = 64;
  BatchProblem chunk[CHUNK];
  size_t ws = 0;
  for (int i0 = 0; i0 < batch; i0 += CHUNK) {
    const int cnt = std::min(CHUNK, batch - i0);
    for (int k = 0; k < cnt; ++k) {
      const int i = i0 + k;
      BatchProblem& bp = chunk[k];
      bp.m = m[i];
      bp.n = n[i];
      bp.lda = lda[i];
      bp.pad = 0;
      bp.A = A[i];
      bp.b = b[i];
      bp.x = x[i];
      bp.y = y[i];
      bp.info = (BatchInfo*)(base + info_off) + i;
      bp.ws = base + ws_off + ws;
      ws += batched_workspace_bytes(m[i], n[i]);
    }
    HIP_TRY(hipMemcpyAsync(base + probs_off + sizeof(BatchProblem) * (size_t)i0, chunk,
                           sizeof(BatchProblem) * (size_t)cnt, hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));   // the chunk buffer is reused
  }
  BatchArgs ba;
  std::memset(&ba, 0, sizeof(ba));
  ba.count = batch;
  ba.probs = (const BatchProblem*)(base + probs_off);
  ba.order = nullptr;
  ba.tau = o.tau;
  ba.p_max = o.p_max;
  ba.max_iter = o.max_iter;
  ba.fp32 = o.precision == NNLS_FP32_IR ? 1 : 0;
  ba.ir_max_steps = o.ir_max_steps;
  ba.ir_rtol = o.ir_rtol;
  ba.gram_dual = (o.flags & NNLS_FLAG_GRAM_DUAL) != 0 ? 1 : 0;
  launch_batched(h->stream, ba, batch);
  if (hipGetLastError() != hipSuccess) return NNLS_ERR_DEVICE;
  HIP_TRY(hipStreamSynchronize(h->stream));
  const double el = now_ms() - t0;
  int worst = NNLS_OK;
  BatchInfo bi[CHUNK];
  for (int i0 = 0; i0 < batch; i0 += CHUNK) {
    const int cnt = std::min(CHUNK, batch - i0);
    HIP_TRY(hipMemcpyAsync(bi, base + info_off + sizeof(BatchInfo) * (size_t)i0, sizeof(BatchInfo) * (size_t)cnt,
                           hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    for (int k = 0; k < cnt; ++k) {
      const BatchInfo& q = bi[k];
      if (info) {
        nnls_info& d = info[i0 + k];
        d.status = q.status;
        d.iterations = q.iterations;
        d.n_free = q.n_free;
        d.last_ninf = q.last_ninf;
        d.failed_index = q.failed_index;
        d.ir_steps = q.ir_steps;
        d.min_margin = q.min_margin;
        d.solve_ms = el;
      }
      if (q.status != NNLS_OK && worst == NNLS_OK) worst = q.status;
    }
  }
  return worst;
}

// ------------------------------------------------------------ prepared batches
int nnls_batch_plan_create(nnls_handle* h, int32_t batch, const int32_t* m, const int32_t* n,
                           const double* const* A, const int32_t* lda, const double* const* b,
                           double* const* x, double* const* y, const nnls_options* opts,
                           nnls_batch_plan** plan) {
  if (!plan) return NNLS_ERR_INVALID_ARG;
  *plan = nullptr;
  nnls_options o;
  nnls_default_options(&o);
  if (opts) o = *opts;
  if (!h || batch < 1 || !m || !n || !A || !lda || !b || !x || !y) return NNLS_ERR_INVALID_ARG;
  if (check_options(o) != NNLS_OK) return NNLS_ERR_INVALID_ARG;
  if (o.precision == NNLS_BF16_IR) o.precision = NNLS_FP32_IR;   // the batched path's float32 tier
  for (int i = 0; i < batch; ++i)
    if (n[i] < 1 || m[i] < n[i] || lda[i] < m[i] || !A[i] || !b[i] || !x[i] || !y[i]) return NNLS_ERR_INVALID_ARG;
  if (hipSetDevice(h->device) != hipSuccess) return NNLS_ERR_DEVICE;
  nnls_batch_plan* P = new (std::nothrow) nnls_batch_plan();
  if (!P) return NNLS_ERR_NO_MEMORY;
  P->h = h;
  P->batch = batch;
  std::vector<BatchProblem> probs((size_t)batch);
  std::vector<int32_t> order((size_t)batch);
  size_t total = 0;
  for (int i = 0; i < batch; ++i) {
    BatchProblem& bp = probs[(size_t)i];
    bp.m = m[i];
    bp.n = n[i];
    bp.lda = lda[i];
    bp.pad = 0;
    bp.A = A[i];
    bp.b = b[i];
    bp.x = x[i];
    bp.y = y[i];
    bp.ws = (char*)(uintptr_t)total;
    total += batched_workspace_bytes(m[i], n[i]);
    order[(size_t)i] = i;
  }
  std::stable_sort(order.begin(), order.end(), [&](int a_, int b_) {   // as nnls_solve_dense_batched
    const double wa = (double)n[a_] * n[a_] * (m[a_] + n[a_]);
    const double wb = (double)n[b_] * n[b_] * (m[b_] + n[b_]);
    return wa > wb;
  });
  auto fail = [&](int st) {
    (void)hipGetLastError();
    nnls_batch_plan_destroy(P);
    return st;
  };
  if (hipMalloc(&P->d_probs, sizeof(BatchProblem) * (size_t)batch) != hipSuccess ||
      hipMalloc(&P->d_order, sizeof(int32_t) * (size_t)batch) != hipSuccess ||
      hipMalloc(&P->d_info, sizeof(BatchInfo) * (size_t)batch) != hipSuccess ||
      hipMalloc(&P->d_ws, total) != hipSuccess ||
      hipHostMalloc(&P->h_info, sizeof(BatchInfo) * (size_t)batch, hipHostMallocDefault) != hipSuccess)
    return fail(NNLS_ERR_NO_MEMORY);
  for (int i = 0; i < batch; ++i) {
    probs[(size_t)i].info = (BatchInfo*)P->d_info + i;
    probs[(size_t)i].ws = (char*)P->d_ws + (uintptr_t)probs[(size_t)i].ws;
  }
  if (hipMemcpy(P->d_probs, probs.data(), sizeof(BatchProblem) * (size_t)batch, hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(P->d_order, order.data(), sizeof(int32_t) * (size_t)batch, hipMemcpyHostToDevice) != hipSuccess)
    return fail(NNLS_ERR_DEVICE);
  BatchArgs ba;
  std::memset(&ba, 0, sizeof(ba));
  ba.count = batch;
  ba.probs = (const BatchProblem*)P->d_probs;
  ba.order = (const int32_t*)P->d_order;
  ba.tau = o.tau;
  ba.p_max = o.p_max;
  ba.max_iter = o.max_iter;
  ba.fp32 = o.precision == NNLS_FP32_IR ? 1 : 0;
  ba.ir_max_steps = o.ir_max_steps;
  ba.ir_rtol = o.ir_rtol;
  ba.gram_dual = (o.flags & NNLS_FLAG_GRAM_DUAL) != 0 ? 1 : 0;
  ba.max_steps = 0;
  // Tile-shape autotuner of the Gram kernel: for each 32-column bucket of the batch
  // (problems with ceil(n / 32) = nr <= GS_NR), time the kernel on that bucket's problems
  // alone with each accumulator shape whose pass plan differs, and keep the fastest.  The
  // shapes sum every entry in the same order, so the choice changes no result.
  {
    std::vector<std::vector<int32_t>> bucket(GS_NR + 1);
    for (int i = 0; i < batch; ++i)
      if (n[i] <= 32 * GS_NR) bucket[(size_t)((n[i] + 31) / 32)].push_back(i);
    const int qv[2][GS_VARIANTS] = {{2, 3, 4}, {4, 6, 8}};   // rectangles per wave, as in the kernel
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return fail(NNLS_ERR_DEVICE);
    bool tune_ok = true;
    for (int nr = 1; nr <= GS_NR && tune_ok; ++nr) {
      const std::vector<int32_t>& bl = bucket[(size_t)nr];
      if (bl.empty()) continue;
      const int nrect = nr * (nr + 1) / 2;
      int plan_of[GS_VARIANTS];
      for (int k = 0; k < GS_VARIANTS; ++k) {
        const int q = qv[ba.fp32 ? 1 : 0][k];
        const int passes = (nrect + 8 * q - 1) / (8 * q), per = (nrect + passes - 1) / passes;
        plan_of[k] = passes * 64 + (per + 7) / 8;
      }
      tune_ok = hipMemcpy(P->d_order, bl.data(), sizeof(int32_t) * bl.size(), hipMemcpyHostToDevice) == hipSuccess;
      BatchArgs tb = ba;
      tb.order = (const int32_t*)P->d_order;
      int best = -1;
      float best_ms = 0.0f;
      for (int k = 0; k < GS_VARIANTS && tune_ok; ++k) {
        if (k != 1 && plan_of[k] == plan_of[1]) continue;   // the same code as the default
        tb.gram_variant[nr] = (uint8_t)(1 + k);
        float t = 0.0f;
        for (int rep = 0; rep < 3 && tune_ok; ++rep) {   // the first launch warms up
          tune_ok = hipEventRecord(e0, h->stream) == hipSuccess;
          launch_batched_gram(h->stream, tb, (int)bl.size());
          tune_ok = tune_ok && hipEventRecord(e1, h->stream) == hipSuccess &&
                    hipEventSynchronize(e1) == hipSuccess;
          float ms = 0.0f;
          if (tune_ok) tune_ok = hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
          if (rep == 1 || (rep == 2 && ms < t)) t = ms;
        }
        if (tune_ok && (best < 0 || t < best_ms)) {
          best = k;
          best_ms = t;
        }
      }
      if (best < 0) best = 1;
      ba.gram_variant[nr] = (uint8_t)(1 + best);
      P->shapes[nr] = (uint8_t)qv[ba.fp32 ? 1 : 0][best];
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!tune_ok ||
        hipMemcpy(P->d_order, order.data(), sizeof(int32_t) * (size_t)batch, hipMemcpyHostToDevice) != hipSuccess)
      return fail(NNLS_ERR_DEVICE);
  }
  // record: both kernels and the status copy, on a private stream (no memset nodes)
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return fail(NNLS_ERR_DEVICE);
  bool ok = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
  if (ok) {
    launch_batched_gram(cs, ba, batch);
    launch_batched_steps(cs, ba, batch);
    ok = hipMemcpyAsync(P->h_info, P->d_info, sizeof(BatchInfo) * (size_t)batch, hipMemcpyDeviceToHost, cs) ==
         hipSuccess;
    hipGraph_t g = nullptr;
    const bool ended = hipStreamEndCapture(cs, &g) == hipSuccess;
    ok = ok && ended && g;
    P->graph = g;
  }
  (void)hipStreamDestroy(cs);
  if (!ok || hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0) != hipSuccess) return fail(NNLS_ERR_DEVICE);
  *plan = P;
  return NNLS_OK;
}

int nnls_batch_plan_execute(nnls_batch_plan* plan, nnls_info* info) {
  if (!plan || !plan->exec) return NNLS_ERR_INVALID_ARG;
  if (hipSetDevice(plan->h->device) != hipSuccess) return NNLS_ERR_DEVICE;
  plan->t0 = now_ms();
  if (hipGraphLaunch(plan->exec, plan->h->stream) != hipSuccess) {
    (void)hipGetLastError();
    return NNLS_ERR_DEVICE;
  }
  return info ? nnls_batch_plan_info(plan, info) : NNLS_OK;
}

int nnls_batch_plan_info(nnls_batch_plan* plan, nnls_info* info) {
  if (!plan) return NNLS_ERR_INVALID_ARG;
  if (hipSetDevice(plan->h->device) != hipSuccess || hipStreamSynchronize(plan->h->stream) != hipSuccess) {
    (void)hipGetLastError();
    return NNLS_ERR_DEVICE;
  }
  const double el = now_ms() - plan->t0;
  const BatchInfo* bi = (const BatchInfo*)plan->h_info;
  int worst = NNLS_OK;
  for (int i = 0; i < plan->batch; ++i) {
    const BatchInfo& q = bi[i];
    if (info) {
      nnls_info& d = info[i];
      std::memset(&d, 0, sizeof(d));
      d.status = q.status;
      d.iterations = q.iterations;
      d.n_free = q.n_free;
      d.last_ninf = q.last_ninf;
      d.failed_index = q.failed_index;
      d.ir_steps = q.ir_steps;
      d.min_margin = q.min_margin;
      d.est_rel_err = -1.0;
      d.solve_ms = el;
    }
    if (q.status != NNLS_OK && worst == NNLS_OK) worst = q.status;
  }
  return worst;
}

int nnls_batch_plan_tile_shapes(const nnls_batch_plan* plan, int32_t* shapes) {
  if (!plan || !shapes) return NNLS_ERR_INVALID_ARG;
  for (int k = 0; k <= GS_NR; ++k) shapes[k] = plan->shapes[k];
  return NNLS_OK;
}

int nnls_batch_plan_destroy(nnls_batch_plan* plan) {
  if (!plan) return NNLS_OK;
  (void)hipSetDevice(plan->h->device);
  if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
  if (plan->graph) (void)hipGraphDestroy(plan->graph);
  for (void* p : {plan->d_probs, plan->d_order, plan->d_info, plan->d_ws})
    if (p) (void)hipFree(p);
  if (plan->h_info) (void)hipHostFree(plan->h_info);
  delete plan;
  return NNLS_OK;
}

int nnls_get_trace(nnls_handle* h, nnls_trace_row* rows, int cap) {
  if (!h) return NNLS_ERR_INVALID_ARG;
  const int cnt = (int)h->trace.size();
  if (rows && cap > 0) std::memcpy(rows, h->trace.data(), sizeof(nnls_trace_row) * (size_t)std::min(cap, cnt));
  return cnt;
}

int nnls_get_profile(nnls_handle* h, int64_t* launches, double* total_ms, double* work) {
  if (!h) return NNLS_ERR_INVALID_ARG;
  for (int c = 0; c < NNLS_PROFILE_CLASSES; ++c) {
    if (launches) launches[c] = h->prof_launches[c];
    if (total_ms) total_ms[c] = h->prof_ms[c];
    if (work) work[c] = h->prof_work[c];
  }
  return NNLS_OK;
}

int nnls_set_profiling(nnls_handle* h, int on) {
  if (!h) return NNLS_ERR_INVALID_ARG;
  h->profile_always = on != 0;
  h->profiling = h->profile_always;
  return NNLS_OK;
}

int nnls_reset_profile(nnls_handle* h) {
  if (!h) return NNLS_ERR_INVALID_ARG;
  for (int c = 0; c < NNLS_PROFILE_CLASSES; ++c) {
    h->prof_launches[c] = 0;
    h->prof_ms[c] = 0.0;
    h->prof_work[c] = 0.0;
  }
  return NNLS_OK;
}

int nnls_gram_csc(nnls_handle* h, int32_t m, int32_t n, int64_t nnz, const int32_t* colptr,
                  const int32_t* rowidx, const double* val, const double* b, double* H, int32_t ldh,
                  double* c) {
  if (!h || n < 1 || m < 1 || nnz < 0 || nnz > INT32_MAX || !colptr || !b || !H || !c || ldh < n ||
      (nnz > 0 && (!rowidx || !val)))
    return NNLS_ERR_INVALID_ARG;
  if (hipSetDevice(h->device) != hipSuccess) return NNLS_ERR_DEVICE;
  Problem P;
  std::memset(&P, 0, sizeof(P));
  P.sparse = true;
  P.m = m;
  P.n = n;
  P.nnz = nnz;
  P.colptr = colptr;
  P.rowidx = rowidx;
  P.val = val;
  P.b = b;
  TRY(validate_device(h, P));
  TRY(build_gram_sparse(h, P));
  launch_fill_2d(h->stream, n, n, H, ldh, 0.0);
  launch_lower_to_dense(h->stream, n, gram_view(h), H, ldh);
  HIP_TRY(hipMemcpyAsync(c, h->c.p, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return NNLS_OK;
}

int nnls_gram_dense(nnls_handle* h, int32_t m, int32_t n, const double* A, int32_t lda, const double* b,
                    double* H, int32_t ldh, double* c) {
  if (!h || n < 1 || m < 1 || !A || lda < m || !b || !H || !c || ldh < n) return NNLS_ERR_INVALID_ARG;
  if (hipSetDevice(h->device) != hipSuccess) return NNLS_ERR_DEVICE;
  launch_gram_dense(h->stream, m, n, A, lda, H, ldh);
  launch_gemvT_dense(h->stream, m, n, A, lda, b, c, 1.0);
  if (hipGetLastError() != hipSuccess) return NNLS_ERR_DEVICE;
  HIP_TRY(hipStreamSynchronize(h->stream));
  return NNLS_OK;
}

int nnls_cholesky(nnls_handle* h, int32_t n, const double* S, int32_t lds, double* L, int32_t ldl,
                  int32_t precision, int32_t* failed) {
  if (failed) *failed = -1;
  if (!h || n < 1 || !S || !L || lds < n || ldl < n ||
      (precision != NNLS_FP64 && precision != NNLS_FP32_IR && precision != NNLS_BF16_IR))
    return NNLS_ERR_INVALID_ARG;
  if (hipSetDevice(h->device) != hipSuccess) return NNLS_ERR_DEVICE;
  const int prec = prec_level(precision);
  const bool fp32 = prec >= PREC_F32;
  TRY(ensure(h, h->ctrl, sizeof(Ctrl)));
  TRY(ensure_factor(h, n, prec));
  launch_ctrl_set_state(h->stream, (Ctrl*)h->ctrl.p, INT32_MAX, 0, 0, 0);
  launch_fill_i32(h->stream, (int32_t*)h->colcnt.p, (n + TILE - 1) / TILE, 0);
  h->epoch += 1;
  h->max_wgs = h->default_wgs;
  h->fact_prec = -1;
  FactorArgs fa = factor_args(h, n, nullptr, S, lds, false);
  fa.Lbf = prec == PREC_BF16 ? h->Lbf.p : nullptr;
  fa.Mc = nullptr;   // no triangular solves follow
  launch_cholesky(h->stream, fa, fp32);
  launch_tiles_to_dense(h->stream, n, h->Lt.p, fp32, L, ldl);
  TRY(sync_read(h, h->h_ctrl, h->ctrl.p, sizeof(Ctrl)));
  const Ctrl c = *h->h_ctrl;
  if (c.status == NNLS_ERR_NOT_PD) {
    if (failed) *failed = c.failed_pos;
    return NNLS_ERR_NOT_PD;
  }
  return c.status;
}

int nnls_spd_solve(nnls_handle* h, int32_t n, const double* S, int32_t lds, const double* rhs, double* x,
                   int32_t* failed) {
  if (failed) *failed = -1;
  if (!h || n < 1 || !S || !rhs || !x || lds < n) return NNLS_ERR_INVALID_ARG;
  if (hipSetDevice(h->device) != hipSuccess) return NNLS_ERR_DEVICE;
  TRY(ensure(h, h->ctrl, sizeof(Ctrl)));
  TRY(ensure_factor(h, n, PREC_F64));
  launch_ctrl_set_state(h->stream, (Ctrl*)h->ctrl.p, INT32_MAX, 0, 0, 0);
  launch_fill_i32(h->stream, (int32_t*)h->colcnt.p, (n + TILE - 1) / TILE, 0);
  h->epoch += 1;
  h->max_wgs = h->default_wgs;
  h->fact_prec = -1;
  FactorArgs fa = factor_args(h, n, nullptr, S, lds, false);
  fa.rhs = rhs;
  fa.z = (double*)h->z.p;
  launch_cholesky(h->stream, fa, false);
  SolveArgs sa = solve_args(h, n, nullptr, rhs, x);
  launch_trsv(h->stream, sa, false, false);
  const int rs = sync_read(h, h->h_ctrl, h->ctrl.p, sizeof(Ctrl));
  if (rs != NNLS_OK || h->h_ctrl->status != NNLS_OK) h->slots_empty = false;
  TRY(rs);
  const Ctrl c = *h->h_ctrl;
  if (c.status == NNLS_ERR_NOT_PD && failed) *failed = c.failed_pos;
  return c.status;
}

int nnls_dual_csc(nnls_handle* h, int32_t m, int32_t n, int64_t nnz, const int32_t* colptr,
                  const int32_t* rowidx, const double* val, const double* b, const uint8_t* free_flags,
                  const double* x, double* r, double* y) {
  if (!h || n < 1 || m < 1 || nnz < 0 || nnz > INT32_MAX || !colptr || !b || !free_flags || !x || !y ||
      (nnz > 0 && (!rowidx || !val)))
    return NNLS_ERR_INVALID_ARG;
  if (hipSetDevice(h->device) != hipSuccess) return NNLS_ERR_DEVICE;
  Problem P;
  std::memset(&P, 0, sizeof(P));
  P.sparse = true;
  P.m = m;
  P.n = n;
  P.nnz = nnz;
  P.colptr = colptr;
  P.rowidx = rowidx;
  P.val = val;
  P.b = b;
  TRY(validate_device(h, P));
  TRY(build_csr(h, P));
  double* rr = r;
  if (!rr) {
    TRY(ensure(h, h->r, sizeof(double) * (size_t)m));
    rr = (double*)h->r.p;
  }
  // a gathered vector larger than an XCD's L2 is swept in slices (x for the residual,
  // r for the dual); the sliced copies of A are built before the products
  const bool slice_x = n > SLICE_MIN_LEN, slice_r = m > SLICE_MIN_LEN;
  const int nsx = slice_count(n), nsr = slice_count(m);
  if (slice_x || slice_r) {
    const int64_t slots = std::max(slice_x ? (int64_t)nsx * ((int64_t)m + 1) : 0,
                                   slice_r ? (int64_t)nsr * ((int64_t)n + 1) : 0);
    TRY(ensure(h, h->slc, sizeof(int32_t) * (size_t)slots));
    TRY(ensure(h, h->scan, sizeof(int32_t) * ((size_t)slots / 2048 + 1)));
  }
  if (slice_x) {
    TRY(ensure(h, h->srp, sizeof(int32_t) * ((size_t)nsx * ((size_t)m + 1) + 1)));
    TRY(ensure(h, h->sri, sizeof(int32_t) * (size_t)nnz));
    TRY(ensure(h, h->srv, sizeof(double) * (size_t)nnz));
    launch_slice_build(h->stream, m, nnz, (const int32_t*)h->rowptr.p, (const int32_t*)h->colidx.p,
                       (const double*)h->valr.p, nsx, (int32_t*)h->slc.p, (int32_t*)h->srp.p,
                       (int32_t*)h->sri.p, (double*)h->srv.p, (int32_t*)h->scan.p);
  }
  if (slice_r) {
    TRY(ensure(h, h->sdp, sizeof(int32_t) * ((size_t)nsr * ((size_t)n + 1) + 1)));
    TRY(ensure(h, h->sdi, sizeof(int32_t) * (size_t)nnz));
    TRY(ensure(h, h->sdv, sizeof(double) * (size_t)nnz));
    launch_slice_build(h->stream, n, nnz, colptr, rowidx, val, nsr, (int32_t*)h->slc.p, (int32_t*)h->sdp.p,
                       (int32_t*)h->sdi.p, (double*)h->sdv.p, (int32_t*)h->scan.p);
  }
  int64_t pe = prof_begin(h, NNLS_PROF_RESIDUAL);
  if (slice_x)
    launch_sliced_residual(h->stream, m, nsx, (const int32_t*)h->srp.p, (const int32_t*)h->sri.p,
                           (const double*)h->srv.p, x, b, rr);
  else
    launch_residual_csr(h->stream, m, nnz, (const int32_t*)h->rowptr.p, (const int32_t*)h->colidx.p,
                        (const double*)h->valr.p, x, b, rr);
  prof_end(h, pe, 12.0 * (double)nnz + 20.0 * m + 8.0 * n);
  pe = prof_begin(h, NNLS_PROF_DUAL);
  if (slice_r)
    launch_sliced_dual(h->stream, n, nsr, (const int32_t*)h->sdp.p, (const int32_t*)h->sdi.p,
                       (const double*)h->sdv.p, rr, free_flags, y);
  else
    launch_dual_csc(h->stream, n, colptr, rowidx, val, rr, free_flags, y);
  prof_end(h, pe, 12.0 * (double)nnz + 8.0 * m + 13.0 * n);
  HIP_TRY(hipStreamSynchronize(h->stream));
  prof_flush(h);
  return NNLS_OK;
}

int nnls_dual_dense(nnls_handle* h, int32_t m, int32_t n, const double* A, int32_t lda, const double* b,
                    const uint8_t* free_flags, const double* x, double* r, double* y) {
  if (!h || n < 1 || m < 1 || lda < m || !A || !b || !free_flags || !x || !y) return NNLS_ERR_INVALID_ARG;
  if (hipSetDevice(h->device) != hipSuccess) return NNLS_ERR_DEVICE;
  Problem P;
  std::memset(&P, 0, sizeof(P));
  P.sparse = false;
  P.m = m;
  P.n = n;
  P.A = A;
  P.lda = lda;
  P.b = b;
  TRY(validate_device(h, P));
  TRY(ensure(h, h->rpart, sizeof(double) * (size_t)dense_residual_chunks(m, n) * (size_t)m));
  double* rr = r;
  if (!rr) {
    TRY(ensure(h, h->r, sizeof(double) * (size_t)m));
    rr = (double*)h->r.p;
  }
  const double mn = (double)m * (double)n;
  int64_t pe = prof_begin(h, NNLS_PROF_RESIDUAL);
  launch_residual_dense(h->stream, m, n, A, lda, x, b, rr, (double*)h->rpart.p);
  prof_end(h, pe, 8.0 * mn + 8.0 * n + 16.0 * m);
  pe = prof_begin(h, NNLS_PROF_DUAL);
  launch_dual_dense(h->stream, m, n, A, lda, rr, free_flags, y);
  prof_end(h, pe, 8.0 * mn + 8.0 * m + 9.0 * n);
  HIP_TRY(hipStreamSynchronize(h->stream));
  prof_flush(h);
  return NNLS_OK;
}

int nnls_pivot_step(nnls_handle* h, int32_t n, double* x, double* y, uint8_t* free_flags, double tau,
                    int32_t p_max, int32_t* state, int32_t* out) {
  if (!h || n < 1 || !x || !y || !free_flags || !state || !out || !(tau >= 0.0) || p_max < 0)
    return NNLS_ERR_INVALID_ARG;
  if (hipSetDevice(h->device) != hipSuccess) return NNLS_ERR_DEVICE;
  TRY(ensure(h, h->ctrl, sizeof(Ctrl)));
  TRY(ensure(h, h->Flist, sizeof(int32_t) * (size_t)n));
  TRY(ensure(h, h->pos, sizeof(int32_t) * (size_t)n));
  const int N = state[0] < 0 ? INT32_MAX : state[0];
  launch_ctrl_set_state(h->stream, (Ctrl*)h->ctrl.p, N, state[1], 0, 0);
  TRY(ensure(h, h->colcnt, sizeof(int32_t) * (size_t)((n + TILE - 1) / TILE), true));
  h->fact_prec = -1;
  launch_pivot_control(h->stream, n, x, y, free_flags, (int32_t*)h->Flist.p, (int32_t*)h->pos.p,
                       (Ctrl*)h->ctrl.p, tau, p_max, INT32_MAX, (int32_t*)h->colcnt.p,
                       (n + TILE - 1) / TILE, nullptr, 0);
  TRY(sync_read(h, h->h_ctrl, h->ctrl.p, sizeof(Ctrl)));
  const Ctrl c = *h->h_ctrl;
  state[0] = c.N == INT32_MAX ? -1 : c.N;
  state[1] = c.p;
  out[0] = c.k;
  out[1] = c.branch;
  out[2] = c.rmax;
  out[3] = c.done ? -1 : c.n_free;
  return c.status;
}

}  // extern "C"
