// Device building blocks shared by the tiled factorisation kernels: MFMA traits and
// lane layouts, agent-scope polling and publishing, and the in-LDS factorisation and
// inversion of one 64 x 64 diagonal tile.
#pragma once

#include "nnls_internal.h"

namespace nnls {

// Where a non-positive pivot is reported: positions base + (0..63) of the F-block,
// counted only below nF; the first one wins (atomicMin) and status becomes NOT_PD.
struct PivotReport {
  int base;
  int nF;
  int32_t* failed_pos;
  int32_t* status;
};

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T> struct MF;
template <> struct MF<double> {
  typedef d4 acc;
  static __device__ inline acc op(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // element v of lane l holds row (l / 16) + 4 v, column l % 16 of the 16 x 16 block
  static __device__ inline int row(int l, int v) { return (l >> 4) + 4 * v; }
};
template <> struct MF<float> {
  typedef f4 acc;
  static __device__ inline acc op(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // element v of lane l holds row 4 (l / 16) + v, column l % 16 of the 16 x 16 block
  static __device__ inline int row(int l, int v) { return 4 * (l >> 4) + v; }
};

constexpr int LDT = TILE + 1;    // LDS leading dimension of a column-major staged tile
// 16 bytes as a native vector (HIP's uint4 class type keeps arrays of it out of registers)
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ inline int32_t ld_relaxed(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void acquire_agent() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

__device__ inline void raise_abort(Ctrl* ctrl) {
  __hip_atomic_store(&ctrl->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  atomicCAS(&ctrl->status, 0, (int)NNLS_ERR_DEVICE);
}

// Spin with relaxed loads until *p >= target (or == target when exact).  No fence: the
// caller issues one acquire after it has learned all it can from the counters.
__device__ inline bool spin_until(const int32_t* p, int target, bool exact, Ctrl* ctrl,
                                  uint64_t wait_ticks) {
  int32_t v = ld_relaxed(p);
  if (exact ? v == target : v >= target) return true;
  const uint64_t t0 = wall_clock64();
  for (;;) {
    __builtin_amdgcn_s_sleep(1);
    v = ld_relaxed(p);
    if (exact ? v == target : v >= target) return true;
    if (ld_relaxed(&ctrl->abort)) return false;
    if (wall_clock64() - t0 > wait_ticks) {
      raise_abort(ctrl);
      return false;
    }
  }
}

// A hand-over slot whose value is its own ready flag: empty slots hold SLOT_EMPTY, a
// signalling NaN, which arithmetic never returns (it quiets NaN operands), so a computed
// value can never read as empty.  One agent-scope access carries both the data and the
// readiness, where a flag would need a second round trip through memory after it.
constexpr uint64_t SLOT_EMPTY = ((uint64_t)(uint32_t)SLOT_EMPTY_WORD << 32) | (uint32_t)SLOT_EMPTY_WORD;
__device__ inline void slot_put(double* p, double v) {
  __hip_atomic_store((uint64_t*)p, (uint64_t)__double_as_longlong(v), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
// Wait until the slot is filled, take its value and leave the slot empty again.  A wait
// beyond the bound raises NNLS_ERR_DEVICE and returns 0.
__device__ inline double slot_take(double* p, Ctrl* ctrl, uint64_t wait_ticks) {
  uint64_t* q = (uint64_t*)p;
  uint64_t v = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (v == SLOT_EMPTY) {
    const uint64_t t0 = wall_clock64();
    for (;;) {
      __builtin_amdgcn_s_sleep(1);
      v = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (v != SLOT_EMPTY) break;
      if (ld_relaxed(&ctrl->abort)) return 0.0;
      if (wall_clock64() - t0 > wait_ticks) {
        raise_abort(ctrl);
        return 0.0;
      }
    }
  }
  __hip_atomic_store(q, SLOT_EMPTY, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return __longlong_as_double((long long)v);
}

// Wait until the slot is filled and return its value, leaving it filled (for slots that
// several readers take the same value from).
__device__ inline double slot_wait(const double* p, Ctrl* ctrl, uint64_t wait_ticks) {
  const uint64_t* q = (const uint64_t*)p;
  uint64_t v = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (v == SLOT_EMPTY) {
    const uint64_t t0 = wall_clock64();
    for (;;) {
      __builtin_amdgcn_s_sleep(1);
      v = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (v != SLOT_EMPTY) break;
      if (ld_relaxed(&ctrl->abort)) return 0.0;
      if (wall_clock64() - t0 > wait_ticks) {
        raise_abort(ctrl);
        return 0.0;
      }
    }
  }
  return __longlong_as_double((long long)v);
}
__device__ inline void slot_clear(double* p) {
  __hip_atomic_store((uint64_t*)p, SLOT_EMPTY, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Make every thread's global stores visible at agent scope, then let thread 0 set a flag
// (and bump a counter).  The barrier completes the workgroup's stores into this XCD's L2
// (workgroup-scope release); thread 0's agent-scope release fence then writes that L2
// back once, and the flag writes after it need no ordering of their own.  (A full
// __threadfence in every thread would write the L2 back three times and also invalidate
// it, throwing away lines the other workgroups on this XCD are still reading.)
__device__ inline void publish_tile(int32_t* flag, int32_t* counter, int epoch) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_store(flag, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add(counter, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}
__device__ inline void publish_store(int32_t* flag, int value) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_store(flag, value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

__device__ inline double bcast_lane(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}
__device__ inline float bcast_lane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// 16 x 16 block product on MFMA for one wave: acc += sign * A * op(B), where A is the
// block of P at (pr, pc) and op(B) is the block of Q at (qr, qc), transposed when transB.
// Both operands are column-major with leading dimension LDT.
template <typename T>
__device__ inline typename MF<T>::acc mm16(typename MF<T>::acc acc, T sign, const T* P, int pr, int pc,
                                         const T* Q, int qr, int qc, bool transB) {
  const int lane = threadIdx.x & 63, lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int kk = 0; kk < 16; kk += 4) {
    const T av = sign * P[(pr + lr) + (pc + kk + lk) * LDT];
    const T bv = transB ? Q[(qr + lr) + (qc + kk + lk) * LDT] : Q[(qr + kk + lk) + (qc + lr) * LDT];
    acc = MF<T>::op(av, bv, acc);
  }
  return acc;
}

template <typename T>
__device__ inline typename MF<T>::acc load16(const T* X, int r0, int c0) {
  const int lane = threadIdx.x & 63, lr = lane & 15;
  typename MF<T>::acc v;
#pragma unroll
  for (int e = 0; e < 4; ++e) v[e] = X[(r0 + MF<T>::row(lane, e)) + (c0 + lr) * LDT];
  return v;
}

template <typename T>
__device__ inline void store16(T* X, int r0, int c0, typename MF<T>::acc v) {
  const int lane = threadIdx.x & 63, lr = lane & 15;
#pragma unroll
  for (int e = 0; e < 4; ++e) X[(r0 + MF<T>::row(lane, e)) + (c0 + lr) * LDT] = v[e];
}

__device__ inline double rsqrt_refined(double d) {
  const double y = __builtin_amdgcn_rsq(d);
  const double e = fma(-d, y * y, 1.0);
  return fma(y * e, fma(0.375, e, 0.5), y);
}
__device__ inline float rsqrt_refined(float d) {
  float y = __builtin_amdgcn_rsqf(d);
  y = y * fmaf(-0.5f * d, y * y, 1.5f);
  return y;
}

// Factor and invert the 16 x 16 diagonal block at offset o of S (one wave).  Lanes 0..15
// keep row i of the block in registers; lanes 16..31 start from column i of the identity
// and go through the very same updates, which turns them into column i of L^-1 (forward
// substitution, one column per lane, in step with the factorisation).  Pivots come from a
// reciprocal square root refined by one third-order step (the hardware estimate is good to
// about 2^-24; with e = 1 - d y^2 the step y (1 + e/2 + 3e^2/8) leaves about (5/16) e^3,
// under one ulp); a pivot that is not positive and finite is flagged and continues as 1
// without a branch.  Each step's column of L reaches every lane as wave-uniform values
// read from the factor lanes, so the pivot chain never touches LDS.
// L goes back into S, its inverse into W.
template <typename T>
__device__ inline void diag16(T* S, T* W, int o, const PivotReport& rep) {
  const int lane = threadIdx.x & 63, i = lane & 15;
  const bool inv = (lane >> 4) == 1;   // lanes 16..31 carry the inverse
  T r[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) r[j] = inv ? ((j == i) ? (T)1 : (T)0) : S[(o + i) + (o + j) * LDT];
  int firstbad = -1;                   // uniform: pivots are read from one lane
  T d = bcast_lane(r[0], 0);
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    const bool bad = !(d > (T)0) || !isfinite(d);
    if (bad && firstbad < 0) firstbad = c;
    const T dd = bad ? (T)1 : d;
    const T y = rsqrt_refined(dd);    // 1 / L_cc
    const T l = dd * y;               // L_cc
    // factor lanes: L_ic (L_cc on the diagonal); inverse lanes: (L^-1)_ci
    const T lic = (i == c && !inv) ? l : r[c] * y;
    r[c] = lic;
    if (c + 1 < 16) d = bcast_lane(fma(-lic, lic, r[c + 1]), c + 1);
    // column c of L below the pivot, as wave-uniform values read from the factor lanes
#pragma unroll
    for (int j = c + 1; j < 16; ++j) r[j] = fma(-lic, bcast_lane(lic, j), r[j]);
  }
  if (firstbad >= 0 && lane == 0 && rep.base + o + firstbad < rep.nF) {
    atomicMin(rep.failed_pos, rep.base + o + firstbad);
    atomicCAS(rep.status, 0, (int)NNLS_ERR_NOT_PD);
  }
  if (lane < 16) {
#pragma unroll
    for (int j = 0; j < 16; ++j) S[(o + i) + (o + j) * LDT] = (j <= i) ? r[j] : (T)0;
  } else if (inv) {
#pragma unroll
    for (int k = 0; k < 16; ++k) W[(o + k) + (o + i) * LDT] = (k >= i) ? r[k] : (T)0;
  }
}

// Waits until the workgroup-shared counter reaches `target`.  The other waves of the
// workgroup always post, so the wait ends; its bound only turns a broken invariant into a
// device error instead of a hang.
__device__ inline void lds_wait_count(const int* cnt, int target, const PivotReport& rep) {
  for (int guard = 0; guard < (1 << 22); ++guard) {
    if (__hip_atomic_load(cnt, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) >= target) return;
    __builtin_amdgcn_s_sleep(1);
  }
  if ((threadIdx.x & 63) == 0) atomicCAS(rep.status, 0, (int)NNLS_ERR_DEVICE);
}
__device__ inline void lds_post(int* cnt) {
  if ((threadIdx.x & 63) == 0) __hip_atomic_fetch_add(cnt, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// The 16 x 16 block operations of the tile factor, all by one wave.
template <typename T>
__device__ inline void blk_panel(T* S, const T* W, int p, int q) {   // L_pq = A_pq W_qq^T
  typename MF<T>::acc acc = {};
  acc = mm16<T>(acc, (T)1, S, 16 * p, 16 * q, W, 16 * q, 16 * q, true);
  store16<T>(S, 16 * p, 16 * q, acc);
}
template <typename T>
__device__ inline void blk_trail(T* S, int p, int r, int q) {       // A_pr -= L_pq L_rq^T
  typename MF<T>::acc acc = load16<T>(S, 16 * p, 16 * r);
  acc = mm16<T>(acc, (T)-1, S, 16 * p, 16 * q, S, 16 * r, 16 * q, true);
  store16<T>(S, 16 * p, 16 * r, acc);
}
// W_pq = -W_pp sum_{k=q}^{p-1} L_pk W_kq, the sum staged in the free upper block (0, sc) of S
template <typename T>
__device__ inline void blk_inverse(T* S, T* W, int p, int q, int sc) {
  typename MF<T>::acc t = {};
  for (int k = q; k < p; ++k) t = mm16<T>(t, (T)1, S, 16 * p, 16 * k, W, 16 * k, 16 * q, false);
  store16<T>(S, 0, 16 * sc, t);
  typename MF<T>::acc u = {};
  u = mm16<T>(u, (T)-1, W, 16 * p, 16 * p, S, 0, 16 * sc, false);
  store16<T>(W, 16 * p, 16 * q, u);
}

// Blocked Cholesky and inverse of the 64 x 64 tile in S (lower triangle) by the whole
// workgroup: 4 x 4 blocks of 16.  Wave 0 carries the chain: after diagonal block q it
// forms the panel block (q+1, q), applies its term to diagonal block q+1 and factors that
// block at once.  Meanwhile waves 1..3 form the other panel blocks of column q, wait (on a
// shared counter) for wave 0's panel block, apply the remaining trailing updates, and
// build the off-diagonal blocks of the inverse whose inputs are final.  Leaves L in the
// lower triangle of S and L^-1 in the lower triangle of W; the upper blocks of S are
// scratch.
template <typename T>
__device__ inline void factor_invert_tile(T* S, T* W, const PivotReport& rep) {
  __shared__ int cnt[3];
  const int w = threadIdx.x >> 6;
  if (threadIdx.x == 64) cnt[0] = cnt[1] = cnt[2] = 0;
  if (w == 0) diag16<T>(S, W, 0, rep);
  __syncthreads();
  // column 0: wave 0 -> (1,0), (1,1), diagonal 1; waves 1..3 -> (2,0), (3,0), then the
  // trailing blocks (2,1) (3,1) (2,2) (3,2) (3,3) once all three panel blocks are in
  if (w == 0) {
    blk_panel<T>(S, W, 1, 0);
    lds_post(&cnt[0]);
    blk_trail<T>(S, 1, 1, 0);
    diag16<T>(S, W, 16, rep);
  } else {
    if (w == 1) { blk_panel<T>(S, W, 2, 0); lds_post(&cnt[0]); }
    if (w == 2) { blk_panel<T>(S, W, 3, 0); lds_post(&cnt[0]); }
    lds_wait_count(&cnt[0], 3, rep);
    if (w == 1) { blk_trail<T>(S, 2, 1, 0); blk_trail<T>(S, 3, 2, 0); }
    if (w == 2) { blk_trail<T>(S, 3, 1, 0); blk_trail<T>(S, 3, 3, 0); }
    if (w == 3) blk_trail<T>(S, 2, 2, 0);
  }
  __syncthreads();
  // column 1: wave 0 -> (2,1), (2,2), diagonal 2; wave 1 -> (3,1), then W_10;
  // waves 2, 3 -> (3,2), (3,3) once (2,1) and (3,1) are in
  if (w == 0) {
    blk_panel<T>(S, W, 2, 1);
    lds_post(&cnt[1]);
    blk_trail<T>(S, 2, 2, 1);
    diag16<T>(S, W, 32, rep);
  } else if (w == 1) {
    blk_panel<T>(S, W, 3, 1);
    lds_post(&cnt[1]);
    blk_inverse<T>(S, W, 1, 0, 1);
  } else {
    lds_wait_count(&cnt[1], 2, rep);
    if (w == 2) blk_trail<T>(S, 3, 2, 1);
    else blk_trail<T>(S, 3, 3, 1);
  }
  __syncthreads();
  // column 2: wave 0 -> (3,2), (3,3), diagonal 3; waves 1, 2 -> W_21, W_20
  if (w == 0) {
    blk_panel<T>(S, W, 3, 2);
    blk_trail<T>(S, 3, 3, 2);
    diag16<T>(S, W, 48, rep);
  } else if (w == 1) {
    blk_inverse<T>(S, W, 2, 1, 1);
  } else if (w == 2) {
    blk_inverse<T>(S, W, 2, 0, 2);
  }
  __syncthreads();
  // last block row of the inverse: W_3q for q = 0, 1, 2
  if (w < 3) blk_inverse<T>(S, W, 3, w, w + 1);
  __syncthreads();
}


}  // namespace nnls
