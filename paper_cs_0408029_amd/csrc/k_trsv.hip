// Triangular solves of the normal equations with a factor of the F-block (Sec. 2.1 of the
// tsnnls paper: the forward and backward substitutions after the Cholesky factorisation),
// and the coupling tiles they read, formed once after each factor.
#include <type_traits>
#include <utility>

#include "tile_ops.h"

namespace nnls {

namespace {

// Triangular solves with a walker.  Forward: z_I = L_II^-1 (rhs_I - sum_{k<I} L_Ik z_k),
// blocks in ascending order; backward: x_I = L_II^-T (z_I - sum_{k>I} L_kI^T x_k), blocks in
// descending order.  Step s solves block I = blk(s).  Split the sum into the TD newest terms
// (the blocks of steps s-TD .. s-1) and the older ones:
//     x_I = y_I - sum_{j=1..TD} C_{I,j} x_{blk(s-j)},   y_I = D_I (rhs_I - older_I),
// with D_I = L_II^-1 (D_I^T backward) and the coupling tiles C_{I,j} = D_I L_{I,blk(s-j)}
// (backward D_I^T L_{blk(s-j),I}^T), which depend only on the factor and are formed once
// after it (k_walk_couplings).  Ticket 0 is the walker: it takes y_I and applies the TD
// newest terms, one product of TD tiles with its own last outputs (an LDS ring, in the
// factor's precision) and one barrier a step.  Ticket s+1 is the helper of step s: it accumulates every older term as
// the walker's outputs appear, forms y_I with D_I and the right-hand side, and hands it
// over.  Both directions go through slots whose values are their own ready flags: the
// walker writes each output block into output slots that the helpers read, and takes (and
// empties) each helper's slots; at its end it empties the output slots.
//
// The chain is bound by memory round trips, not arithmetic: a helper sees an output about
// one load latency after it is written, and its hand-over reaches the walker one more
// latency later.  TD newest terms give each helper TD walker steps for that round trip,
// and everything a walker step reads (its TD coupling tiles and the load of the helper's
// hand-over) is requested two steps ahead.  A helper's waves work independently: each
// polls the output slots of HP steps ahead and multiplies its 16 rows as they arrive.  A
// helper waits only for walker steps that precede its own, and the walker waits for
// helpers of steps it has reached, so every wait ends; each wait is also bounded in wall
// time.
//
// Thread layout of the walk: wave w takes rows 16 w .. 16 w + 15 of a 64-row block, four
// lanes a row (lane l: row 16 w + l / 4, columns 16 (l % 4) .. 16 (l % 4) + 15).

template <bool FWD>
__device__ inline int blk(int s, int nb) { return FWD ? s : nb - 1 - s; }

template <typename T, bool FWD>
__device__ inline void load_term_tile(const T* Lt, int I, int K, int r, int g, T (&v)[16]) {
  if (FWD) {   // L_IK, thread (r, g) takes row r, columns 16 g .. 16 g + 15
    const T* tl = Lt + tile_index(I, K) * TILE_ELEMS;
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = tl[(g * 16 + q) * TILE + r];
  } else {     // L_KI^T: thread (r, g) takes column r, rows 16 g .. 16 g + 15 of L_KI
    const T* tl = Lt + tile_index(K, I) * TILE_ELEMS;
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = tl[r * TILE + g * 16 + q];
  }
}

// A thread's 16 values of a term tile as loaded, converted only where they are used, so
// that a load issued steps ahead is not waited for by its conversion.
template <typename T, bool FWD, bool BF> struct TermRegs {
  T v[16];
  __device__ __forceinline__ void load(const void* L, int I, int K, int r, int g) {
    load_term_tile<T, FWD>((const T*)L, I, K, r, g, v);
  }
  __device__ __forceinline__ T at(int q) const { return v[q]; }
};
// From the bfloat16 row-major copy of the tile (element (r, c) at r TILE + c), forward: row
// r, columns 16 g .. 16 g + 15, 32 contiguous bytes.
template <> struct TermRegs<float, true, true> {
  u32x4 w0, w1;
  __device__ __forceinline__ void load(const void* L, int I, int K, int r, int g) {
    const u32x4* p = (const u32x4*)((const uint16_t*)L + tile_index(I, K) * TILE_ELEMS + r * TILE + g * 16);
    w0 = p[0];
    w1 = p[1];
  }
  __device__ __forceinline__ float at(int q) const {
    const uint32_t x = (q < 8 ? w0 : w1)[(q & 7) >> 1];
    return __uint_as_float((q & 1) ? (x & 0xFFFF0000u) : (x << 16));
  }
};
// backward: column r, rows 16 g .. 16 g + 15 of L_KI
template <> struct TermRegs<float, false, true> {
  uint32_t h[16];
  __device__ __forceinline__ void load(const void* L, int I, int K, int r, int g) {
    const uint16_t* tl = (const uint16_t*)L + tile_index(K, I) * TILE_ELEMS;
#pragma unroll
    for (int q = 0; q < 16; ++q) h[q] = tl[(g * 16 + q) * TILE + r];
  }
  __device__ __forceinline__ float at(int q) const { return __uint_as_float(h[q] << 16); }
};

template <typename T, bool FWD>
__device__ inline void load_dinv(const T* Dv, int I, int r, int g, T (&v)[16]) {
  const T* D = Dv + (int64_t)I * TILE_ELEMS;
#pragma unroll
  for (int q = 0; q < 16; ++q) v[q] = FWD ? D[(g * 16 + q) * TILE + r] : D[r * TILE + g * 16 + q];
}

// A lane's value from lane l ^ 1 (CTRL 0xB1) or l ^ 2 (CTRL 0x4E) of its quad.
template <int CTRL>
__device__ __forceinline__ double quad_swap(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
// Sum over the four lanes of a quad, (v0 + v1) + (v2 + v3): the same bits in all four lanes.
__device__ __forceinline__ double quad_sum(double v) {
  v += quad_swap<0xB1>(v);
  return v + quad_swap<0x4E>(v);
}
// Orders this wave's LDS accesses on either side for all of its lanes.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
__device__ __forceinline__ uint64_t slot_peek(const double* p) {
  return __hip_atomic_load((const uint64_t*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Every active lane's slot p, given the value an earlier load of it returned: waits until
// all of them are filled.  A wait beyond the bound raises NNLS_ERR_DEVICE.
__device__ inline uint64_t slot_fill_wait(const double* p, uint64_t v, Ctrl* ctrl, uint64_t wait_ticks) {
  if (__builtin_amdgcn_ballot_w64(v == SLOT_EMPTY) == 0) return v;
  const uint64_t t0 = wall_clock64();
  for (;;) {
    __builtin_amdgcn_s_sleep(1);
    if (v == SLOT_EMPTY) v = slot_peek(p);
    if (__builtin_amdgcn_ballot_w64(v == SLOT_EMPTY) == 0) return v;
    if (ld_relaxed(&ctrl->abort)) return 0;
    if (wall_clock64() - t0 > wait_ticks) {
      raise_abort(ctrl);
      return 0;
    }
  }
}

// f(integral_constant<int, 0>) .. f(integral_constant<int, N - 1>), written out
template <typename F, int... K>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, K...>) {
  (f(std::integral_constant<int, K>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) { static_for_impl(f, std::make_integer_sequence<int, N>{}); }

// A helper wave's steps in flight: HP steps of output loads and term tiles stay within the
// 63 loads the hardware counts in flight (a backward term tile of the bfloat16 copy is 16
// two-byte loads a thread: a column of a row-major tile).
template <typename T, bool FWD, bool BF> struct WalkHP { static constexpr int value = (!FWD && BF) ? 2 : 4; };
template <bool FWD, bool BF> struct WalkHP<double, FWD, BF> { static constexpr int value = 2; };

// Coupling tiles are stored in the order the walker's threads read them: the 16 entries
// C[r][16 g + q] of walk thread (r, g) (thread index 64 (r / 16) + 4 (r % 16) + g) go in
// 16-byte chunks, chunk k of every thread before chunk k + 1 of any, so that each load
// instruction of a wave reads 1 KB of consecutive bytes.  S is the stored type: the
// factor's precision, or bfloat16 (its bits) for a factor with bfloat16 updates, whose
// error already exceeds that rounding.
template <typename S> struct CouplingLayout {
  static constexpr int E = 16 / sizeof(S);   // entries per 16-byte chunk
  static __host__ __device__ int index(int r, int c) {
    const int thr = 64 * (r >> 4) + 4 * (r & 15) + (c >> 4), q = c & 15;
    return ((q / E) * 256 + thr) * E + q % E;
  }
};
template <typename S> struct RowRegs {   // a walk thread's 16 entries of a coupling tile
  S v[16];
  __device__ __forceinline__ void load(const S* tile, int tid) {
    constexpr int E = CouplingLayout<S>::E;
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = tile[((q / E) * 256 + tid) * E + q % E];
  }
  __device__ __forceinline__ S at(int q) const { return v[q]; }
};
template <> struct RowRegs<uint16_t> {
  u32x4 w[2];
  __device__ __forceinline__ void load(const uint16_t* tile, int tid) {
    const u32x4* p = (const u32x4*)tile;
    w[0] = p[tid];
    w[1] = p[256 + tid];
  }
  __device__ __forceinline__ float at(int q) const {
    const uint32_t x = w[q >> 3][(q & 7) >> 1];
    return __uint_as_float((q & 1) ? (x & 0xFFFF0000u) : (x << 16));
  }
};
template <typename S> __device__ inline S coupling_store(float v);
template <> __device__ inline float coupling_store<float>(float v) { return v; }
template <> __device__ inline uint16_t coupling_store<uint16_t>(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }
template <typename S> __device__ inline S coupling_store(double v) { return v; }

// Coupling tiles of the walker: forward C = D_I L_{I,I-j}, backward C = D_I^T L_{I+j,I}^T
// (D_I the inverted diagonal tile), j = 1 .. TD, formed in T and stored as S; one
// workgroup a tile, both operands staged in LDS, each thread 16 entries of one row.
template <typename T, typename S>
__global__ __launch_bounds__(256) void k_walk_couplings(int nb, const T* __restrict__ Lt, const T* __restrict__ Dv,
                                                         S* __restrict__ Mc) {
  constexpr int TD = WalkTD<T>::value;
  __shared__ T sD[TILE * LDT], sL[TILE * LDT];
  const int I = blockIdx.x, j = blockIdx.y + 1;
  const bool fwd = blockIdx.z == 0;
  const int K = fwd ? I - j : I + j;
  if (K < 0 || K >= nb) return;
  const T* D = Dv + (int64_t)I * TILE_ELEMS;
  const T* Lk = Lt + (fwd ? tile_index(I, K) : tile_index(K, I)) * TILE_ELEMS;
  const int tid = threadIdx.x;
  for (int e = tid; e < TILE_ELEMS; e += 256) {   // column-major sources, element (e % 64, e / 64)
    sD[(e >> 6) * LDT + (e & (TILE - 1))] = D[e];
    sL[(e >> 6) * LDT + (e & (TILE - 1))] = Lk[e];
  }
  __syncthreads();
  const int r = tid & (TILE - 1), c0 = (tid >> 6) * 16;
  T acc[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) acc[c] = (T)0;
  for (int k = 0; k < TILE; ++k) {
    const T dk = fwd ? sD[k * LDT + r] : sD[r * LDT + k];   // D[r][k], or D[k][r]
#pragma unroll
    for (int c = 0; c < 16; ++c)   // L[k][c0 + c], or L[c0 + c][k]
      acc[c] = fma(dk, fwd ? sL[(c0 + c) * LDT + k] : sL[k * LDT + c0 + c], acc[c]);
  }
  S* out = Mc + (((int64_t)blockIdx.z * nb + I) * TD + (j - 1)) * TILE_ELEMS;
#pragma unroll
  for (int c = 0; c < 16; ++c) out[CouplingLayout<S>::index(r, c0 + c)] = coupling_store<S>(acc[c]);
}

template <typename T, bool FWD, bool BF>
__global__ __launch_bounds__(256) void k_trsv_walk(SolveArgs a, uint64_t wait_ticks) {
  constexpr int TD = WalkTD<T>::value, HP = WalkHP<T, FWD, BF>::value;
  static_assert(HP == 2 || HP == 4, "the helper's pipeline is written out for two or four slots");
  typedef TermRegs<T, FWD, BF> Term;
  __shared__ T ring[TD + 1][TILE];   // the walker's outputs of its last TD + 1 steps, rounded to T
  __shared__ double ystage[TILE];
  __shared__ double xstage[4][HP][TILE];
  __shared__ int s_t;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int r = 16 * w + (lane >> 2), g = lane & 3;
  int32_t* ticket = FWD ? &a.ctrl->fwd_ticket : &a.ctrl->bwd_ticket;
  if (tid == 0) s_t = atomicAdd(ticket, 1) - 1;
  __syncthreads();
  const int t = s_t, nb = a.nb;
  if (t >= nb) return;   // also covers a counter that was not reset
  const void* L = BF ? a.Lbf : a.Ltiles;
  double* outv = FWD ? a.z : a.xF;
  double* xsl = a.part + (int64_t)nb * TILE;   // the walker's outputs, one slot per row
  int32_t* walked = FWD ? &a.ctrl->fwd_walked : &a.ctrl->bwd_walked;
  // a 16-term dot product with x[g * 16 ..] as four independent chains (fp64 FMA latency,
  // not issue, bounds a single chain)
  auto dot16 = [&](auto&& lhs, const double* x) __attribute__((always_inline)) -> double {
    double c[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < 16; ++q) c[q & 3] = fma((double)lhs(q), x[g * 16 + q], c[q & 3]);
    return (c[0] + c[1]) + (c[2] + c[3]);
  };

  if (t >= 0) {
    // helper of step t: every term from steps 0 .. t-TD-1, then y_I = D_I (rhs_I - older).
    // Each wave works on its own, with the output block (element `lane`) and the term tile
    // of HP steps in flight, in full groups of HP steps (the loads are unconditional, so
    // that no branch makes the compiler wait for the loads of later steps) and a short
    // tail.  An output that is not yet there when its step comes is waited for on the
    // walker's progress count first, sleeping longer the more walker steps remain before
    // this hand-over is needed: only the helpers next to the chain poll often, so the
    // newest output is not read by every helper at once.  The count is only a hint; every
    // output slot is checked when read.
    const int I = blk<FWD>(t, nb);
    const int last = t - TD;   // steps < last
    const int p = I * TILE + r;
    double rhs;
    if (FWD) rhs = p < a.nF ? (a.rhs_full ? a.rhs_full[a.Flist ? a.Flist[p] : p] : a.rhs_dense[p]) : 0.0;
    else rhs = a.z[p];
    T dv[16];
    load_dinv<T, FWD>((const T*)a.Dinv, I, r, g, dv);
    double hc[4] = {0.0, 0.0, 0.0, 0.0};   // row r, columns 16 g + q, q = k mod 4
    uint64_t xv[HP];
    Term tv[HP];
    double (*xw)[TILE] = xstage[w];
    auto wait_done = [&](int u) {   // until the walker has finished step u
      const uint64_t t0 = wall_clock64();
      for (;;) {
        if (ld_relaxed(walked) > u) return;
        // the walker needs this hand-over after at least last - u more steps, each about a
        // microsecond; a nap is 512 cycles
        int naps = (last - u) / 2 - 2;
        if (naps > 64) naps = 64;
        if (naps < 1) __builtin_amdgcn_s_sleep(1);
        for (int k = 0; k < naps; ++k) __builtin_amdgcn_s_sleep(8);
        if (ld_relaxed(&a.ctrl->abort)) return;
        if (wall_clock64() - t0 > wait_ticks) {
          raise_abort(a.ctrl);
          return;
        }
      }
    };
    auto issue = [&](auto slot, int u) __attribute__((always_inline)) {
      constexpr int d = decltype(slot)::value;
      const int K = blk<FWD>(u, nb);
      xv[d] = slot_peek(&xsl[(int64_t)K * TILE + lane]);
      tv[d].load(L, I, K, r, g);
    };
    auto term = [&](auto slot, auto next, int u) __attribute__((always_inline)) {
      constexpr int d = decltype(slot)::value;
      const double* xs = &xsl[(int64_t)blk<FWD>(u, nb) * TILE + lane];
      uint64_t v = xv[d];
      if (__builtin_amdgcn_ballot_w64(v == SLOT_EMPTY) != 0) {
        // far from the chain: sleep on the progress count first; next to it, poll the slot
        // itself (the count is stored after the output, one more round trip)
        if (last - u > 6) wait_done(u);
        v = slot_fill_wait(xs, v == SLOT_EMPTY ? slot_peek(xs) : v, a.ctrl, wait_ticks);
      }
      xw[d][lane] = __longlong_as_double((long long)v);
      wave_sync();
#pragma unroll
      for (int q = 0; q < 16; ++q) hc[q & 3] = fma((double)tv[d].at(q), xw[d][g * 16 + q], hc[q & 3]);
      if constexpr (decltype(next)::value) issue(slot, u + HP);
    };
    using N0 = std::false_type;
    using N1 = std::true_type;
    int u0 = 0;
    if (last >= HP) {
      issue(std::integral_constant<int, 0>{}, 0);
      issue(std::integral_constant<int, 1>{}, 1);
      if constexpr (HP == 4) {
        issue(std::integral_constant<int, 2>{}, 2);
        issue(std::integral_constant<int, 3>{}, 3);
      }
      for (; u0 + 2 * HP <= last; u0 += HP) {
        term(std::integral_constant<int, 0>{}, N1{}, u0);
        term(std::integral_constant<int, 1>{}, N1{}, u0 + 1);
        if constexpr (HP == 4) {
          term(std::integral_constant<int, 2>{}, N1{}, u0 + 2);
          term(std::integral_constant<int, 3>{}, N1{}, u0 + 3);
        }
      }
      term(std::integral_constant<int, 0>{}, N0{}, u0);
      term(std::integral_constant<int, 1>{}, N0{}, u0 + 1);
      if constexpr (HP == 4) {
        term(std::integral_constant<int, 2>{}, N0{}, u0 + 2);
        term(std::integral_constant<int, 3>{}, N0{}, u0 + 3);
      }
      u0 += HP;
    }
    for (; u0 < last; ++u0) {   // fewer than HP steps left
      issue(std::integral_constant<int, 0>{}, u0);
      term(std::integral_constant<int, 0>{}, N0{}, u0);
    }
    // y_I = D_I (rhs_I - older): the row's sum is in all four of its lanes, which write the
    // same entry
    ystage[r] = rhs - quad_sum((hc[0] + hc[1]) + (hc[2] + hc[3]));
    __syncthreads();
    const double y = quad_sum(dot16([&](int q) { return dv[q]; }, ystage));
    if (g == 0) slot_put(&a.part[(int64_t)p], y);
    return;
  }

  // the walker: x_I = y_I - sum_j C_{I,j} x_{blk(s-j)}.  Slot d of the operand registers
  // holds step s (s % PD == d): its TD coupling tile rows and the load of its hand-over,
  // requested at the end of step s - PD and used at step s.  Every lane issues the same
  // loads on every step (a step before step TD reads a tile it does not use), so that no
  // branch merges the compiler's count of loads in flight and a wait for one operand never
  // drains the next steps' requests.
  constexpr int PD = 2;   // three steps ahead: the hand-over's load comes too early and is polled again
  typedef std::conditional_t<BF, uint16_t, T> S;   // the coupling tiles' stored type
  const S* Mc = (const S*)a.Mc + (FWD ? 0 : (int64_t)nb * TD * TILE_ELEMS);
  RowRegs<S> td[PD][TD];
  uint64_t pv[PD];
  auto prefetch = [&](auto slot, int s1) __attribute__((always_inline)) {
    constexpr int d = decltype(slot)::value;
    const int In = blk<FWD>(min(s1, nb - 1), nb);
#pragma unroll
    for (int j = 0; j < TD; ++j) td[d][j].load(Mc + ((int64_t)In * TD + j) * TILE_ELEMS, tid);
    pv[d] = slot_peek(&a.part[(int64_t)In * TILE + r]);
  };
  auto step = [&](auto slot, int s) __attribute__((always_inline)) {
    constexpr int d = decltype(slot)::value;
    const int I = blk<FWD>(s, nb);
    // newest terms, nearest first, each a 16-term product in T (the coupling tiles are
    // rounded to T already) as four independent chains, summed in double
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < TD; ++j) {
      const int u = s - 1 - j;
      const T* xk = ring[u >= 0 ? u % (TD + 1) : 0] + g * 16;
      T c[4] = {(T)0, (T)0, (T)0, (T)0};
#pragma unroll
      for (int q = 0; q < 16; ++q) c[q & 3] = fma((T)td[d][j].at(q), xk[q], c[q & 3]);
      const double tj = (double)((c[0] + c[1]) + (c[2] + c[3]));
      acc += u >= 0 ? tj : 0.0;
    }
    acc = quad_sum(acc);
    double* pp = &a.part[(int64_t)I * TILE + r];
    const uint64_t v = slot_fill_wait(pp, pv[d], a.ctrl, wait_ticks);   // the row's four lanes
    // every lane consumes the loaded values: the row's four lanes write the same ring entry
    // (a value used on one side of a branch only would make the compiler wait for every
    // older load before it reuses that value's register)
    // (the row's four lanes store the same values, and every thread the same count: stores
    // under a branch would also break the compiler's count of memory operations in flight)
    const double x = __longlong_as_double((long long)v) - acc;
    ring[s % (TD + 1)][r] = (T)x;
    const int p = I * TILE + r;
    __hip_atomic_store((uint64_t*)pp, SLOT_EMPTY, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    outv[p] = x;
    slot_put(&xsl[p], x);
    prefetch(slot, s + PD);
    __syncthreads();   // the ring holds x_s (its slot was last read at step s - 1)
    __hip_atomic_store(walked, s + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  };
  static_for<PD>([&](auto k) { prefetch(k, decltype(k)::value); });
  int s0 = 0;
  for (; s0 + PD <= nb; s0 += PD)   // the loop body has no branch around a step
    static_for<PD>([&](auto k) { step(k, s0 + decltype(k)::value); });
  static_for<PD>([&](auto k) {
    if (s0 + decltype(k)::value < nb) step(k, s0 + decltype(k)::value);
  });
  // every helper has read its last output slot before handing over, and every hand-over
  // has been taken: the output slots can be emptied for the next launch
  for (int i = tid; i < nb * TILE; i += 256) slot_clear(&xsl[i]);
  // x into the caller's vector through the F list, off the chain (this workgroup wrote outv)
  if (!FWD && a.out) {
    __syncthreads();
    for (int p = tid; p < a.nF; p += 256) a.out[a.Flist ? a.Flist[p] : p] = outv[p];
  }
}

}  // namespace

void launch_walk_couplings(hipStream_t s, int nb, const void* Ltiles, const void* Dinv, void* Mc, bool fp32,
                           bool bf16) {
  if (nb <= 0 || !Mc) return;
  if (fp32 && bf16)
    hipLaunchKernelGGL((k_walk_couplings<float, uint16_t>), dim3(nb, WalkTD<float>::value, 2), dim3(256), 0, s, nb,
                       (const float*)Ltiles, (const float*)Dinv, (uint16_t*)Mc);
  else if (fp32)
    hipLaunchKernelGGL((k_walk_couplings<float, float>), dim3(nb, WalkTD<float>::value, 2), dim3(256), 0, s, nb,
                       (const float*)Ltiles, (const float*)Dinv, (float*)Mc);
  else
    hipLaunchKernelGGL((k_walk_couplings<double, double>), dim3(nb, WalkTD<double>::value, 2), dim3(256), 0, s, nb,
                       (const double*)Ltiles, (const double*)Dinv, (double*)Mc);
}

void launch_trsv(hipStream_t s, const SolveArgs& a, bool fp32, bool forward) {
  if (a.nb <= 0) return;
  const dim3 grid(a.nb + 1);   // the helpers and the walker
  if (fp32 && a.Lbf) {
    if (forward) hipLaunchKernelGGL((k_trsv_walk<float, true, true>), grid, dim3(256), 0, s, a, a.wait_ticks);
    hipLaunchKernelGGL((k_trsv_walk<float, false, true>), grid, dim3(256), 0, s, a, a.wait_ticks);
  } else if (fp32) {
    if (forward) hipLaunchKernelGGL((k_trsv_walk<float, true, false>), grid, dim3(256), 0, s, a, a.wait_ticks);
    hipLaunchKernelGGL((k_trsv_walk<float, false, false>), grid, dim3(256), 0, s, a, a.wait_ticks);
  } else {
    if (forward) hipLaunchKernelGGL((k_trsv_walk<double, true, false>), grid, dim3(256), 0, s, a, a.wait_ticks);
    hipLaunchKernelGGL((k_trsv_walk<double, false, false>), grid, dim3(256), 0, s, a, a.wait_ticks);
  }
}

}  // namespace nnls
