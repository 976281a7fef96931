// Sparse products whose gathered vector is larger than an XCD's L2: the residual
// r = A x - b (gathers x[col] over the row-major copy) and the dual y_G = A_G^T r (gathers
// r[row] over the CSC input) of Eq. 5.  With uniformly scattered indices every 8-byte
// gather brings a whole cache line from the memory side, so the plain kernels move several
// times their algorithmic bytes.  Here the matrix is copied slice by slice: slice s holds,
// for every output in order, that output's entries whose gather index falls in
// [s W, (s + 1) W), W = 2^SLICE_SHIFT elements (2 MB of doubles).  Every wave sweeps the
// slices in order, so the waves of an XCD read the same slice of the vector at about the
// same time and their gathers hit the L2.
//
// A wave owns consecutive outputs.  Per slice their entries form one contiguous range
// of the copy, which the wave stages in windows: coalesced loads of indices and values,
// the gathers of v, all into LDS.  Each lane then adds the staged entries of its own
// outputs' runs in order.  An output's entries are thus added in slice order and in
// order within a slice, which is ascending gather-index order: every output is the
// sequential FMA chain of its entries, whatever the launch.
#include "nnls_internal.h"

namespace nnls {

namespace {

constexpr int WIN = 512;   // entries staged per window (eight per lane)

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// counts[s (N + 1) + o] = entries of output o in slice s (the indices of an output are
// ascending, so a slice's entries are one run); the padding slot o = N is 0, so that an
// exclusive scan of the whole array gives each slice's start in slot N of the one before.
__global__ __launch_bounds__(256) void k_slice_count(int N, const int32_t* __restrict__ ptr,
                                                     const int32_t* __restrict__ idx, int ns,
                                                     int32_t* __restrict__ counts) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o > N) return;
  const int64_t ld = (int64_t)N + 1;
  if (o == N) {
    for (int s = 0; s < ns; ++s) counts[s * ld + N] = 0;
    return;
  }
  int q = ptr[o];
  const int e = ptr[o + 1];
  for (int s = 0; s < ns; ++s) {
    const int p = q;
    while (q < e && (idx[q] >> SLICE_SHIFT) == s) ++q;
    counts[s * ld + o] = q - p;
  }
}

// Each output's entries go to its run in every slice, in their original order.
__global__ __launch_bounds__(256) void k_slice_scatter(int N, const int32_t* __restrict__ ptr,
                                                       const int32_t* __restrict__ idx,
                                                       const double* __restrict__ val,
                                                       const int32_t* __restrict__ sptr,
                                                       int32_t* __restrict__ sidx,
                                                       double* __restrict__ sval) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= N) return;
  const int64_t ld = (int64_t)N + 1;
  int cur = -1, pos = 0;
  const int e = ptr[o + 1];
  for (int q = ptr[o]; q < e; ++q) {
    const int i = idx[q];
    const int s = i >> SLICE_SHIFT;
    if (s != cur) {
      cur = s;
      pos = sptr[s * ld + o];
    }
    sidx[pos] = i;
    sval[pos] = val[q];
    ++pos;
  }
}

// One window of a slice's range: indices and values, coalesced.  Every load is made at an
// existing entry: past the range entry wb stands in (entry 0 when the range is empty; the
// copies hold at least one element), and the index is then replaced by 0, so the gather
// reads element 0 of v.  The stand-ins are never added.
template <int JL>
struct Window {
  int iv[JL];
  double av[JL];
};
template <int JL>
__device__ __forceinline__ Window<JL> load_window(const int32_t* __restrict__ sidx, const double* __restrict__ sval,
                                                  int wb, int r1, int lane) {
  Window<JL> w;
  const int nw = r1 - wb;
#pragma unroll
  for (int j = 0; j < JL; ++j) {
    const int c = j * 64 + lane;
    const bool in = c < nw;
    const int t = in ? wb + c : (nw > 0 ? wb : 0);
    const int i = __builtin_nontemporal_load(sidx + t);
    w.iv[j] = in ? i : 0;
    w.av[j] = __builtin_nontemporal_load(sval + t);
  }
  return w;
}

// Wave w of workgroup g owns outputs [ob, ob + 64 QL), ob = (4 g + w) 64 QL; lane l owns
// ob + l + 64 q, q < QL.  The grid is sized to stay resident (at most two workgroups per
// compute unit), so all waves sweep the slices in one generation and an XCD's waves work
// on neighbouring slices.  RESID: out = acc - b (the residual); otherwise the dual,
// out = 0 where flags is set (y_F) and acc elsewhere.  Only wave barriers are used, so a
// wave with no outputs leaves at once.
template <int QL, bool RESID>
__global__ __launch_bounds__(256) void k_sliced_gather(int N, int ns, const int32_t* __restrict__ sptr,
                                                       const int32_t* __restrict__ sidx,
                                                       const double* __restrict__ sval,
                                                       const double* __restrict__ v,
                                                       const double* __restrict__ b,
                                                       const uint8_t* __restrict__ flags,
                                                       double* __restrict__ out) {
  constexpr int GWQ = 64 * QL, JL = WIN / 64;
  __shared__ double s_a[4][WIN], s_g[4][WIN];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t ob = ((int64_t)blockIdx.x * 4 + w) * GWQ;
  if (ob >= N) return;
  const int ow = (int)((int64_t)N - ob < GWQ ? (int64_t)N - ob : GWQ);
  const int64_t ld = (int64_t)N + 1;
  double* sa = s_a[w];
  double* sg = s_g[w];
  bool on[QL];
  double acc[QL];
#pragma unroll
  for (int q = 0; q < QL; ++q) {
    const int lo = lane + 64 * q;
    on[q] = lo < ow && (RESID || flags[ob + lo] == 0);
    acc[q] = 0.0;
  }
  for (int s = 0; s < ns; ++s) {
    const int32_t* sp = sptr + s * ld + ob;
    int p[QL], e[QL];
#pragma unroll
    for (int q = 0; q < QL; ++q) {
      const int lo = lane + 64 * q;
      p[q] = lo < ow ? __builtin_nontemporal_load(sp + lo) : 0;
      e[q] = lo < ow ? __builtin_nontemporal_load(sp + lo + 1) : 0;
    }
    const int r0 = __builtin_nontemporal_load(sp), r1 = __builtin_nontemporal_load(sp + ow);
    for (int wb = r0; wb < r1; wb += WIN) {
      const Window<JL> wx = load_window<JL>(sidx, sval, wb, r1, lane);
      const int nw = r1 - wb < WIN ? r1 - wb : WIN;
#pragma unroll
      for (int j = 0; j < JL; ++j) {
        sa[j * 64 + lane] = wx.av[j];
        sg[j * 64 + lane] = v[wx.iv[j]];
      }
      wave_lds_sync();
#pragma unroll
      for (int q = 0; q < QL; ++q) {
        const int lo = p[q] > wb ? p[q] : wb;
        const int hi = e[q] < wb + nw ? e[q] : wb + nw;
        if (on[q])
          for (int t = lo; t < hi; ++t) acc[q] = fma(sa[t - wb], sg[t - wb], acc[q]);
      }
      wave_lds_sync();   // the next window overwrites the staged entries
    }
  }
#pragma unroll
  for (int q = 0; q < QL; ++q) {
    const int lo = lane + 64 * q;
    if (lo < ow) {
      const int64_t o = ob + lo;
      out[o] = RESID ? acc[q] - b[o] : (on[q] ? acc[q] : 0.0);
    }
  }
}

template <bool RESID>
void launch_gather(hipStream_t s, int N, int ns, const int32_t* sptr, const int32_t* sidx,
                   const double* sval, const double* v, const double* b, const uint8_t* flags,
                   double* out) {
  // outputs per lane: the fewest that keep the grid within two workgroups per compute unit
  // (512), so that every wave is resident from the start of the sweep
  int QL = 4;
  while (QL < 32 && ((int64_t)N + 256 * QL - 1) / (256 * QL) > 512) QL *= 2;
  const unsigned grid = (unsigned)(((int64_t)N + 256 * QL - 1) / (256 * QL));
  if (grid == 0) return;
  switch (QL) {
#define NNLS_GATHER_CASE(QQ)                                                                          \
  case QQ:                                                                                            \
    hipLaunchKernelGGL((k_sliced_gather<QQ, RESID>), dim3(grid), dim3(256), 0, s, N, ns, sptr, sidx, sval, v, \
                       b, flags, out);                                                                \
    break;
    NNLS_GATHER_CASE(4)
    NNLS_GATHER_CASE(8)
    NNLS_GATHER_CASE(16)
    default: NNLS_GATHER_CASE(32)
#undef NNLS_GATHER_CASE
  }
}

}  // namespace

void launch_slice_build(hipStream_t s, int N, int64_t nnz, const int32_t* ptr, const int32_t* idx,
                        const double* val, int ns, int32_t* counts, int32_t* sptr, int32_t* sidx,
                        double* sval, int32_t* scan_sums) {
  const int64_t slots = (int64_t)ns * ((int64_t)N + 1);
  hipLaunchKernelGGL(k_slice_count, dim3((unsigned)(((int64_t)N + 1 + 255) / 256)), dim3(256), 0, s, N, ptr,
                     idx, ns, counts);
  launch_scan_i32(s, slots, counts, sptr, scan_sums);
  if (nnz > 0 && N > 0)
    hipLaunchKernelGGL(k_slice_scatter, dim3((unsigned)(((int64_t)N + 255) / 256)), dim3(256), 0, s, N, ptr, idx,
                       val, (const int32_t*)sptr, sidx, sval);
}

void launch_sliced_residual(hipStream_t s, int m, int ns, const int32_t* sptr, const int32_t* sidx,
                            const double* sval, const double* x, const double* b, double* r) {
  launch_gather<true>(s, m, ns, sptr, sidx, sval, x, b, nullptr, r);
}

void launch_sliced_dual(hipStream_t s, int n, int ns, const int32_t* sptr, const int32_t* sidx,
                        const double* sval, const double* r, const uint8_t* flags, double* y) {
  launch_gather<false>(s, n, ns, sptr, sidx, sval, r, nullptr, flags, y);
}

}  // namespace nnls
