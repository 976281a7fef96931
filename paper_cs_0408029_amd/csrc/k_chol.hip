// Cholesky factor of the F-principal block of the cached Gram matrix, the first step of
// solving the normal equations (Sec. 2.1 and Sec. 3 of the tsnnls paper).
//
// Factorisation: one launch per pivot iteration.  The block is cut into 64 x 64 tiles and
// every lower tile (I, J) is one unit of work of a persistent grid.  A workgroup takes a
// ticket from a counter (tickets are handed out in column-major lower-tile order) and,
// for each ticket, gathers its tile of H_FF
// straight from the Gram matrix into LDS, then computes, left-looking,
//     S_IJ = H_IJ - sum_{k<J} L_Ik L_Jk^T        (MFMA, 16x16x4 blocks)
// A diagonal tile is then factored and inverted in LDS; an off-diagonal tile becomes
// L_IJ = S_IJ (L_JJ^-1)^T once the diagonal tile of its column is ready.
//
// Kept leading block: when the F order starts with j0 whole tile columns of the previous
// factor (same positions, same variables), the tiles (I, J) with I < j0 and the inverted
// diagonal tiles and forward-solve blocks of those columns are the previous launch's, and
// only the rows I >= j0 are computed (tiles of the kept columns are plain off-diagonal
// tiles; the walker starts at column j0).
//
// Dependencies: colcnt[J] counts the finished tiles of column J (complete at nb - J), and
// every finished tile also sets its own ready flag.  Every tile of column J+1 needs all of
// column J, so columns complete in order; each wave caches how many leading columns it
// knows to be complete and skips all checks below that frontier.  At the frontier it waits
// only for the two tiles the next step reads (relaxed polls, then one acquire fence).
// Every dependency of a tile has a smaller ticket, and tickets are only taken by running
// workgroups, so every wait ends; each wait is also bounded in wall time and raises
// NNLS_ERR_DEVICE instead of spinning forever.
//
// Forward solve z = L^-1 c_F: fused into the factorisation (the diagonal tile of column J
// emits z_J).  The stand-alone triangular solves, and the coupling tiles they read, which
// are formed after each factor, are in k_trsv.hip.
#include <climits>

#include <type_traits>
#include <utility>

#include "tile_ops.h"

namespace nnls {

namespace {

// Stage tile (I, J) of H_FF in LDS (column-major, leading dimension LDT).  Positions at or
// beyond nF are padding: identity on the diagonal, zero elsewhere.
// threadIdx.x as a value the compiler cannot carry from one loop iteration to the next
// (keeps the register footprint of the ticket loop at that of a single tile)
__device__ inline int fresh_tid() {
  int v = (int)threadIdx.x;
  asm volatile("" : "+v"(v));
  return v;
}

template <typename T>
__device__ inline void gather_tile(const FactorArgs& a, int tid, int I, int J, T* S) {
  const int r0 = I * TILE, c0 = J * TILE;
  if (a.dense) {
    for (int e = tid; e < TILE_ELEMS; e += 256) {
      const int r = e & (TILE - 1), c = e >> 6;
      const int p = r0 + r, q = c0 + c;
      double v;
      if (p < a.nF && q < a.nF) {
        const int64_t gi = a.Flist ? a.Flist[p] : p;
        const int64_t gj = a.Flist ? a.Flist[q] : q;
        v = a.dense[gi + gj * a.ldd];
      } else {
        v = (p == q) ? 1.0 : 0.0;
      }
      S[r + c * LDT] = (T)v;
    }
  } else {
    for (int e = tid; e < TILE_ELEMS; e += 256) S[(e & (TILE - 1)) + (e >> 6) * LDT] = (T)0;
    __syncthreads();
    // four lanes a column (a quad of one wave): position q's list holds the rows p >= q in
    // ascending order.  The quad narrows [L, R) to the first row >= r0 by a five-way search
    // (each lane probes one of the four interior points, and the count of probes below r0
    // picks the fifth), then scans the block's entries interleaved, lane k taking every
    // fourth from L + k.
    const int c = tid >> 2, k = tid & 3, q = c0 + c;
    if (q < a.nF && r0 < a.nF) {
      const int64_t s = a.gpos.pptr[a.Flist[q]], e = s + a.gpos.pcnt[q];
      int64_t L = s, R = e;
      while (R - L > 4) {   // the same trip count in the four lanes of the quad
        const int64_t step = (R - L) / 5;
        const int below = a.gpos.prow[L + (k + 1) * step] < r0 ? 1 : 0;
        int cnt = below + __shfl_xor(below, 1);
        cnt += __shfl_xor(cnt, 2);
        // the probes below r0 are a prefix (the rows ascend): cnt of them
        if (cnt < 4) R = L + (cnt + 1) * step;
        if (cnt > 0) L = L + cnt * step + 1;
      }
      for (int64_t t = L + k; t < e; t += 4) {
        const int p = a.gpos.prow[t];
        if (p >= r0 + TILE) break;
        if (p >= r0) S[(p - r0) + c * LDT] = (T)a.gpos.pval[t];
      }
    } else if (q >= a.nF && I == J && k == 0) {
      S[c + c * LDT] = (T)1;
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------- bfloat16 operand copies
// NNLS_BF16_IR: every finished off-diagonal tile is also stored rounded to bfloat16, row by
// row (element (r, c) at r * TILE + c, 8 KB a tile), and the left-looking updates read
// these copies: half the bytes of the float32 tiles, and v_mfma_f32_16x16x32_bf16 with
// float32 accumulation.  The diagonal chain (the walker's last term, the diagonal factor,
// the triangular solves with the inverted diagonal tiles) stays in float32.  Diagonal tiles
// never enter an update as operands, so they have no copy.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
constexpr int LDK = TILE + 8;   // LDS row stride (elements) of a staged bfloat16 tile

__device__ inline uint32_t pack_bf16x2(float lo, float hi) {
  return (uint32_t)__builtin_bit_cast(uint16_t, (__bf16)lo) |
         ((uint32_t)__builtin_bit_cast(uint16_t, (__bf16)hi) << 16);
}

// Row-major bfloat16 copy of an LDS tile (column-major float, leading dimension LDT):
// thread t writes row t / 4, columns 16 (t % 4) .. 16 (t % 4) + 15.
__device__ __forceinline__ void bf16_copy_to_global(uint16_t* __restrict__ g, const float* X, int tid) {
  const int r = tid >> 2, c0 = (tid & 3) * 16;
  uint32_t w[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) w[q] = pack_bf16x2(X[r + (c0 + 2 * q) * LDT], X[r + (c0 + 2 * q + 1) * LDT]);
  u32x4* dst = (u32x4*)(g + r * TILE + c0);
  dst[0] = u32x4{w[0], w[1], w[2], w[3]};
  dst[1] = u32x4{w[4], w[5], w[6], w[7]};
}

// One lower tile (I, J), I >= j0; S, W, s_part, s_rhs are the workgroup's LDS.
template <typename T, bool BF>
__device__ __forceinline__ void chol_tile(const FactorArgs& a, uint64_t wait_ticks, int tid, int I, int J,
                                          T* S, T* W, double (*s_part)[TILE]) {
  typedef MF<T> M;
  typedef typename M::acc Acc;
  const int lane = tid & 63, w = tid >> 6;
  const int nb = a.nb, j0 = a.j0;
  T* Lt = (T*)a.Ltiles;
  T* Dv = (T*)a.Dinv;

  gather_tile<T>(a, tid, I, J, S);

  const int qr = (w & 1) * 32, qc = (w >> 1) * 32;
  const int lr = lane & 15, lk = lane >> 4;
  Acc acc[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        acc[bi][bj][v] = S[(qr + 16 * bi + M::row(lane, v)) + (qc + 16 * bj + lr) * LDT];

  const bool skip = (I == J) && (qr < qc);   // upper quadrant of a diagonal tile
  // The diagonal tile stops one step short: the walker applies the last term, L_{J,J-1}
  // being its own output (except in the walker's first column j0).  The sub-diagonal tile
  // runs its whole update and leaves the triangular solve with L_JJ to the walker.  The
  // diagonal tile also runs the forward solve L z = c_F for its block up to its last step:
  // it streams every L_Jk anyway, and z_k is published before column k completes.  Tiles
  // of the kept columns (J < j0) read L_Jk and L_JJ^-1 from the previous launch.
  const bool partial = (I - J <= 1) && (J >= j0);
  const int kend = (I == J && J > j0) ? J - 1 : J;
  const bool needJ = (I != J) && (J >= j0);   // L_Jk is computed in this launch
  const bool fwd = (I == J) && (a.rhs != nullptr);
  double tacc = 0.0;                         // row `lane`, columns 16 w .. 16 w + 15
  // Software pipeline: the tiles of step k sit in LDS (S takes L_Ik, W takes L_Jk; neither
  // is needed during the update) while the loads of step k+1 are in flight in registers.
  // Step k+1 is prefetched only when its tiles are already known to be final; at the
  // frontier its loads wait until step k's products are issued.
  T* SA = S;
  T* SB = (I == J) ? S : W;
  T ra[BF ? 1 : TILE_ELEMS / 256], rb[BF ? 1 : TILE_ELEMS / 256];
  // bfloat16 operands: 16 values a thread (row tid / 4, columns 16 (tid % 4) ..), staged in
  // LDS row-major with row stride LDK
  uint16_t* HA = (uint16_t*)S;
  uint16_t* HB = (I == J) ? HA : (uint16_t*)W;
  const uint16_t* Lb = (const uint16_t*)a.Lbf;
  int known = 0;                             // leading columns this thread knows are complete
  // column k is complete when its nb - max(k, j0) computed tiles are
  auto ready = [&](int k1, bool block) -> bool {
    if (k1 < known) return true;
    if (ld_relaxed(&a.colcnt[k1]) >= nb - max(k1, j0)) {
      known = k1 + 1;
      while (known < J && ld_relaxed(&a.colcnt[known]) >= nb - max(known, j0)) ++known;
    } else if (!block) {
      if (ld_relaxed(&a.tflag[tile_index(I, k1)]) != a.epoch) return false;
      if (needJ && ld_relaxed(&a.tflag[tile_index(J, k1)]) != a.epoch) return false;
    } else {
      // at the frontier: wait only for the tiles this step reads
      spin_until(&a.tflag[tile_index(I, k1)], a.epoch, true, a.ctrl, wait_ticks);
      if (needJ) spin_until(&a.tflag[tile_index(J, k1)], a.epoch, true, a.ctrl, wait_ticks);
    }
    acquire_agent();
    return true;
  };
  auto load = [&](int k1) {
    const T* gi = Lt + tile_index(I, k1) * TILE_ELEMS;
#pragma unroll
    for (int q = 0; q < TILE_ELEMS / 256; ++q) ra[q] = gi[tid + q * 256];
    if (I != J) {
      const T* gj = Lt + tile_index(J, k1) * TILE_ELEMS;
#pragma unroll
      for (int q = 0; q < TILE_ELEMS / 256; ++q) rb[q] = gj[tid + q * 256];
    }
  };
  if constexpr (BF) {
    // Up to PD steps' operand copies in flight: step s is loaded into the registers of slot
    // s % PD as soon as its tiles are known final and its slot is free (step s - PD has
    // been staged), so the loads of later steps overlap the short bfloat16 MFMA steps.  A
    // step whose tiles were not final when its slot freed is loaded, waiting, at its turn.
    constexpr int PD = 4;
    u32x4 rg[PD][4];
    int held[PD];   // the step each slot holds (-1: none)
    auto fetch = [&](auto slot, int s1) __attribute__((always_inline)) {
      constexpr int d = decltype(slot)::value;
      const u32x4* gi = (const u32x4*)(Lb + tile_index(I, s1) * TILE_ELEMS) + 2 * tid;
      rg[d][0] = gi[0];
      rg[d][1] = gi[1];
      if (I != J) {
        const u32x4* gj = (const u32x4*)(Lb + tile_index(J, s1) * TILE_ELEMS) + 2 * tid;
        rg[d][2] = gj[0];
        rg[d][3] = gj[1];
      }
      held[d] = s1;
    };
    auto prime = [&](auto slot) __attribute__((always_inline)) {
      constexpr int d = decltype(slot)::value;
      held[d] = -1;
      if (d < kend && ready(d, d == 0)) fetch(slot, d);
    };
    prime(std::integral_constant<int, 0>{});
    prime(std::integral_constant<int, 1>{});
    prime(std::integral_constant<int, 2>{});
    prime(std::integral_constant<int, 3>{});
    auto step = [&](auto slot, int k) __attribute__((always_inline)) {
      constexpr int d = decltype(slot)::value;
      if (held[d] != k) {   // at the frontier: wait for this step's tiles
        ready(k, true);
        fetch(slot, k);
      }
      __syncthreads();   // the previous step's products (or the accumulator set-up) have read LDS
      {
        const int o = (tid >> 2) * LDK + (tid & 3) * 16;
        ((u32x4*)(HA + o))[0] = rg[d][0];
        ((u32x4*)(HA + o))[1] = rg[d][1];
        if (I != J) {
          ((u32x4*)(HB + o))[0] = rg[d][2];
          ((u32x4*)(HB + o))[1] = rg[d][3];
        }
      }
      __syncthreads();
      held[d] = -1;
      if (k + PD < kend && ready(k + PD, false)) fetch(slot, k + PD);
      if (fwd) {
        const double* zk = a.z + (int64_t)k * TILE;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int cc = w * 16 + q;
          tacc = fma((double)(float)__builtin_bit_cast(__bf16, HB[lane * LDK + cc]), zk[cc], tacc);
        }
      }
      if (!skip) {
        // lane l: row l % 16 of its 16 x 16 block, k = kh + 8 (l / 16) .. + 7, for both operands
#pragma unroll
        for (int kh = 0; kh < TILE; kh += 32) {
          const int kofs = kh + 8 * lk;
          u32x4 x0 = *(const u32x4*)(HA + (qr + lr) * LDK + kofs);
          u32x4 x1 = *(const u32x4*)(HA + (qr + 16 + lr) * LDK + kofs);
          const u32x4 y0 = *(const u32x4*)(HB + (qc + lr) * LDK + kofs);
          const u32x4 y1 = *(const u32x4*)(HB + (qc + 16 + lr) * LDK + kofs);
          const uint32_t neg = 0x80008000u;   // S -= L_Ik L_Jk^T: negate the L_Ik operand
          x0 ^= neg;
          x1 ^= neg;
          const bf16x8 a0 = __builtin_bit_cast(bf16x8, x0), a1 = __builtin_bit_cast(bf16x8, x1);
          const bf16x8 b0 = __builtin_bit_cast(bf16x8, y0), b1 = __builtin_bit_cast(bf16x8, y1);
          acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0, acc[0][0], 0, 0, 0);
          acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b1, acc[0][1], 0, 0, 0);
          acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b0, acc[1][0], 0, 0, 0);
          acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, acc[1][1], 0, 0, 0);
        }
      }
    };
    for (int k0 = 0; k0 < kend; k0 += PD) {
      step(std::integral_constant<int, 0>{}, k0);
      if (k0 + 1 < kend) step(std::integral_constant<int, 1>{}, k0 + 1);
      if (k0 + 2 < kend) step(std::integral_constant<int, 2>{}, k0 + 2);
      if (k0 + 3 < kend) step(std::integral_constant<int, 3>{}, k0 + 3);
    }
  } else {
    if (kend > 0) {
      ready(0, true);
      load(0);
    }
    for (int k = 0; k < kend; ++k) {
      __syncthreads();   // the previous step's products (or the accumulator set-up) have read LDS
#pragma unroll
      for (int q = 0; q < TILE_ELEMS / 256; ++q) {
        const int e = tid + q * 256, o = (e & (TILE - 1)) + (e >> 6) * LDT;
        SA[o] = ra[q];
        if (I != J) SB[o] = rb[q];
      }
      __syncthreads();
      bool pre = false;
      if (k + 1 < kend) {
        pre = ready(k + 1, false);
        if (pre) load(k + 1);
      }
      if (fwd) {
        const double* zk = a.z + (int64_t)k * TILE;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int cc = w * 16 + q;
          tacc = fma((double)SB[lane + cc * LDT], zk[cc], tacc);
        }
      }
      if (!skip) {
#pragma unroll
        for (int kk = 0; kk < TILE; kk += 4) {
          const int col = (kk + lk) * LDT;
          const T a0 = -SA[col + qr + lr], a1 = -SA[col + qr + 16 + lr];
          const T b0 = SB[col + qc + lr], b1 = SB[col + qc + 16 + lr];
          acc[0][0] = M::op(a0, b0, acc[0][0]);
          acc[0][1] = M::op(a0, b1, acc[0][1]);
          acc[1][0] = M::op(a1, b0, acc[1][0]);
          acc[1][1] = M::op(a1, b1, acc[1][1]);
        }
      }
      if (k + 1 < kend && !pre) {
        ready(k + 1, true);
        load(k + 1);
      }
    }
  }
  __syncthreads();   // the last products have read S and W

#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        S[(qr + 16 * bi + M::row(lane, v)) + (qc + 16 * bj + lr) * LDT] = acc[bi][bj][v];
  __syncthreads();

  const int64_t ti = tile_index(I, J);
  T* dst = Lt + ti * TILE_ELEMS;
  if (partial) {
    // hand the partial sum (and the diagonal's partial forward-solve sums) to the walker
    if (fwd) s_part[w][lane] = tacc;
    for (int e = tid; e < TILE_ELEMS; e += 256) dst[e] = S[(e & (TILE - 1)) + (e >> 6) * LDT];
    if (fwd) {
      __syncthreads();
      if (tid < TILE)
        a.z[(int64_t)J * TILE + tid] = ((s_part[0][tid] + s_part[1][tid]) + s_part[2][tid]) + s_part[3][tid];
    }
    publish_store(&a.tflag[ti], -a.epoch);
    return;
  }

  // off-diagonal: L_IJ = S_IJ (L_JJ^-1)^T once the diagonal tile of column J is ready
  if (J >= j0) {
    spin_until(&a.dflag[J], a.epoch, true, a.ctrl, wait_ticks);
    acquire_agent();
  }
  const T* D = Dv + (int64_t)J * TILE_ELEMS;
  Acc o[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) o[bi][bj][v] = (T)0;
#pragma unroll
  for (int kk = 0; kk < TILE; kk += 4) {
    const int kc = kk + lk;
    const T a0 = S[(qr + lr) + kc * LDT], a1 = S[(qr + 16 + lr) + kc * LDT];
    const T b0 = D[kc * TILE + qc + lr], b1 = D[kc * TILE + qc + 16 + lr];
    o[0][0] = M::op(a0, b0, o[0][0]);
    o[0][1] = M::op(a0, b1, o[0][1]);
    o[1][0] = M::op(a1, b0, o[1][0]);
    o[1][1] = M::op(a1, b1, o[1][1]);
  }
  __syncthreads();
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        S[(qr + 16 * bi + M::row(lane, v)) + (qc + 16 * bj + lr) * LDT] = o[bi][bj][v];
  __syncthreads();
  for (int e = tid; e < TILE_ELEMS; e += 256) dst[e] = S[(e & (TILE - 1)) + (e >> 6) * LDT];
  if constexpr (BF) bf16_copy_to_global((uint16_t*)a.Lbf + ti * TILE_ELEMS, (const float*)S, tid);
  publish_tile(&a.tflag[ti], &a.colcnt[J], a.epoch);
}

// A strip of cnt <= R off-diagonal tiles (I0 + r, J0 + c), r < cnt, c < C, of C = 1 or 2
// adjacent columns (bfloat16 updates).  Every step k < J0 stages the C tiles L_{J0+c,k} and
// the cnt tiles L_{I0+r,k} once, and the four waves each update their 32 x 32 quadrant of
// every tile of the strip: with C = 1 one pair of barriers and one L_Jk load serve R tiles
// (R + 1 tile loads for R outputs instead of 2 R), with C = 2 each L_Ik also serves both
// columns (R + 2 loads for 2 R outputs).  Two steps' operand copies are in flight in
// registers.  Column J0 is then finished as in chol_tile, L_IJ = S_IJ (L_JJ^-1)^T, stored,
// copied to bfloat16 and published; with C = 2 its new tiles (and the walker's
// L_{J0+1,J0}) give the last update term of column J0 + 1, which is finished after it.
// stage: (R + C) bfloat16 tiles with row stride LDK; S (a float tile) aliases it.
constexpr size_t STRIP_STAGE_BYTES =
    (size_t)(CHOL_STRIP + 1 > CHOL_PAIR + 2 ? CHOL_STRIP + 1 : CHOL_PAIR + 2) * TILE * LDK * 2;
// The row walkers of a kept block apply the ROW_TD newest terms from the forward coupling
// tiles (the same TD as the triangular solves'): a ring of ROW_TD + 1 outputs and ROW_TD
// staged couplings, bfloat16 row-major.
constexpr int ROW_TD = WalkTD<float>::value;
constexpr size_t ROW_STAGE_BYTES = (size_t)(2 * ROW_TD + 1) * TILE * LDK * sizeof(uint16_t);

// rw (one column of a kept block, with row walkers): the strip stops ROW_TD terms short and
// hands over Y = S L_JJ^-T, the partial tile of the row walker, in the float tile (flag
// -epoch, no bfloat16 copy, not counted in colcnt).
template <int R, int C>
__device__ __forceinline__ void chol_strip(const FactorArgs& a, uint64_t wait_ticks, int I0, int cnt, int J0,
                                           char* stage, bool rw = false) {
  typedef MF<float> M;
  typedef M::acc Acc;
  const int tid = fresh_tid(), lane = tid & 63, w = tid >> 6;
  const int nb = a.nb, j0 = a.j0;
  float* Lt = (float*)a.Ltiles;
  const float* Dv = (const float*)a.Dinv;
  const uint16_t* Lb = (const uint16_t*)a.Lbf;
  float* S = (float*)stage;
  uint16_t* HB = (uint16_t*)stage;                  // L_{J0+c,k} at HB + c TILE LDK
  uint16_t* HA0 = HB + C * TILE * LDK;              // L_{I0+r,k} at HA0 + r TILE LDK
  const int qr = (w & 1) * 32, qc = (w >> 1) * 32, lr = lane & 15, lk = lane >> 4;
  Acc acc[C][R][2][2];
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[c][r][bi][bj][v] = 0.0f;
      if (r < cnt) {
        gather_tile<float>(a, tid, I0 + r, J0 + c, S);
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int v = 0; v < 4; ++v)
              acc[c][r][bi][bj][v] = S[(qr + 16 * bi + M::row(lane, v)) + (qc + 16 * bj + lr) * LDT];
        __syncthreads();   // S is overwritten by the next gather or the first step's operands
      }
    }
  const bool needJ = J0 >= j0;   // the L_{J0+c,k} are computed in this launch (C = 2: both or neither)
  int known = 0;                 // leading columns this thread knows are complete
  auto ready = [&](int k1, bool block) -> bool {
    if (k1 < known) return true;
    if (ld_relaxed(&a.colcnt[k1]) >= nb - max(k1, j0)) {
      known = k1 + 1;
      while (known < J0 && ld_relaxed(&a.colcnt[known]) >= nb - max(known, j0)) ++known;
    } else if (!block) {
      for (int r = 0; r < cnt; ++r)
        if (ld_relaxed(&a.tflag[tile_index(I0 + r, k1)]) != a.epoch) return false;
      if (needJ)
        for (int c = 0; c < C; ++c)
          if (ld_relaxed(&a.tflag[tile_index(J0 + c, k1)]) != a.epoch) return false;
    } else {
      for (int r = 0; r < cnt; ++r) spin_until(&a.tflag[tile_index(I0 + r, k1)], a.epoch, true, a.ctrl, wait_ticks);
      if (needJ)
        for (int c = 0; c < C; ++c) spin_until(&a.tflag[tile_index(J0 + c, k1)], a.epoch, true, a.ctrl, wait_ticks);
    }
    acquire_agent();
    return true;
  };
  constexpr int PD = C == 1 ? 2 : 1;   // a pair's second step in flight would not fit the registers
  const int kend = rw ? max(J0 - ROW_TD, 0) : J0;   // update steps k < kend
  u32x4 rg[PD][R + C][2];
  int held[PD];
  auto fetch = [&](auto slot, int s1) __attribute__((always_inline)) {
    constexpr int d = decltype(slot)::value;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const u32x4* gj = (const u32x4*)(Lb + tile_index(J0 + c, s1) * TILE_ELEMS) + 2 * tid;
      rg[d][R + c][0] = gj[0];
      rg[d][R + c][1] = gj[1];
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (r < cnt) {
        const u32x4* gi = (const u32x4*)(Lb + tile_index(I0 + r, s1) * TILE_ELEMS) + 2 * tid;
        rg[d][r][0] = gi[0];
        rg[d][r][1] = gi[1];
      }
    held[d] = s1;
  };
  auto prime = [&](auto slot) __attribute__((always_inline)) {
    constexpr int d = decltype(slot)::value;
    held[d] = -1;
    if (d < kend && ready(d, d == 0)) fetch(slot, d);
  };
  // one update step from the staged operands: acc[c][r] -= L_{I0+r} L_{J0+c}^T over c < nc
  auto products = [&](int nc) __attribute__((always_inline)) {
#pragma unroll
    for (int kh = 0; kh < TILE; kh += 32) {
      const int kofs = kh + 8 * lk;
      bf16x8 b0[C], b1[C];
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const uint16_t* hb = HB + c * TILE * LDK;
        b0[c] = __builtin_bit_cast(bf16x8, *(const u32x4*)(hb + (qc + lr) * LDK + kofs));
        b1[c] = __builtin_bit_cast(bf16x8, *(const u32x4*)(hb + (qc + 16 + lr) * LDK + kofs));
      }
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (r < cnt) {
          const uint16_t* HA = HA0 + r * TILE * LDK;
          u32x4 x0 = *(const u32x4*)(HA + (qr + lr) * LDK + kofs);
          u32x4 x1 = *(const u32x4*)(HA + (qr + 16 + lr) * LDK + kofs);
          const uint32_t neg = 0x80008000u;   // S -= L_Ik L_Jk^T: negate the L_Ik operand
          x0 ^= neg;
          x1 ^= neg;
          const bf16x8 a0 = __builtin_bit_cast(bf16x8, x0), a1 = __builtin_bit_cast(bf16x8, x1);
#pragma unroll
          for (int c = 0; c < C; ++c)
            if (c >= C - nc) {
              acc[c][r][0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0[c], acc[c][r][0][0], 0, 0, 0);
              acc[c][r][0][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b1[c], acc[c][r][0][1], 0, 0, 0);
              acc[c][r][1][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b0[c], acc[c][r][1][0], 0, 0, 0);
              acc[c][r][1][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1[c], acc[c][r][1][1], 0, 0, 0);
            }
        }
    }
  };
  const int o16 = (tid >> 2) * LDK + (tid & 3) * 16;   // this thread's 16 staged values of a tile
  prime(std::integral_constant<int, 0>{});
  if constexpr (PD > 1) prime(std::integral_constant<int, PD - 1>{});
  auto step = [&](auto slot, int k) __attribute__((always_inline)) {
    constexpr int d = decltype(slot)::value;
    if (held[d] != k) {   // at the frontier: wait for this step's tiles
      ready(k, true);
      fetch(slot, k);
    }
    __syncthreads();   // the previous step's products have read the staged operands
#pragma unroll
    for (int c = 0; c < C; ++c) {
      uint16_t* hb = HB + c * TILE * LDK;
      ((u32x4*)(hb + o16))[0] = rg[d][R + c][0];
      ((u32x4*)(hb + o16))[1] = rg[d][R + c][1];
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (r < cnt) {
        uint16_t* HA = HA0 + r * TILE * LDK;
        ((u32x4*)(HA + o16))[0] = rg[d][r][0];
        ((u32x4*)(HA + o16))[1] = rg[d][r][1];
      }
    __syncthreads();
    held[d] = -1;
    if (k + PD < kend && ready(k + PD, false)) fetch(slot, k + PD);
    products(C);
  };
  for (int k0 = 0; k0 < kend; k0 += PD) {
    step(std::integral_constant<int, 0>{}, k0);
    if constexpr (PD > 1)
      if (k0 + 1 < kend) step(std::integral_constant<int, PD - 1>{}, k0 + 1);
  }
  __syncthreads();   // the last products have read the staged operands
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int J = J0 + c;
    if (c > 0) {
      // the last term of column J: L_{I,J-1} (finished above by this workgroup) times
      // L_{J,J-1} (the walker's sub-diagonal tile of column J-1, or a kept tile)
      if (needJ) {
        spin_until(&a.tflag[tile_index(J, J - 1)], a.epoch, true, a.ctrl, wait_ticks);
        acquire_agent();
      }
      {
        const u32x4* gj = (const u32x4*)(Lb + tile_index(J, J - 1) * TILE_ELEMS) + 2 * tid;
        const u32x4 j0v = gj[0], j1v = gj[1];
        u32x4 iv[R][2];
#pragma unroll
        for (int r = 0; r < R; ++r)
          if (r < cnt) {
            const u32x4* gi = (const u32x4*)(Lb + tile_index(I0 + r, J - 1) * TILE_ELEMS) + 2 * tid;
            iv[r][0] = gi[0];
            iv[r][1] = gi[1];
          }
        uint16_t* hb = HB + (C - 1) * TILE * LDK;   // products(1) reads column C-1's buffer
        ((u32x4*)(hb + o16))[0] = j0v;
        ((u32x4*)(hb + o16))[1] = j1v;
#pragma unroll
        for (int r = 0; r < R; ++r)
          if (r < cnt) {
            uint16_t* HA = HA0 + r * TILE * LDK;
            ((u32x4*)(HA + o16))[0] = iv[r][0];
            ((u32x4*)(HA + o16))[1] = iv[r][1];
          }
      }
      __syncthreads();
      products(1);
      __syncthreads();   // the products have read the staged operands (S aliases them)
    }
    if (needJ) {
      spin_until(&a.dflag[J], a.epoch, true, a.ctrl, wait_ticks);
      acquire_agent();
    }
    const float* D = Dv + (int64_t)J * TILE_ELEMS;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (r >= cnt) continue;
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            S[(qr + 16 * bi + M::row(lane, v)) + (qc + 16 * bj + lr) * LDT] = acc[c][r][bi][bj][v];
      __syncthreads();
      Acc o[2][2];
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
          for (int v = 0; v < 4; ++v) o[bi][bj][v] = 0.0f;
#pragma unroll
      for (int kk = 0; kk < TILE; kk += 4) {
        const int kc = kk + lk;
        const float a0 = S[(qr + lr) + kc * LDT], a1 = S[(qr + 16 + lr) + kc * LDT];
        const float b0 = D[kc * TILE + qc + lr], b1 = D[kc * TILE + qc + 16 + lr];
        o[0][0] = M::op(a0, b0, o[0][0]);
        o[0][1] = M::op(a0, b1, o[0][1]);
        o[1][0] = M::op(a1, b0, o[1][0]);
        o[1][1] = M::op(a1, b1, o[1][1]);
      }
      __syncthreads();
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            S[(qr + 16 * bi + M::row(lane, v)) + (qc + 16 * bj + lr) * LDT] = o[bi][bj][v];
      __syncthreads();
      const int64_t ti = tile_index(I0 + r, J);
      float* dst = Lt + ti * TILE_ELEMS;
      for (int e = tid; e < TILE_ELEMS; e += 256) dst[e] = S[(e & (TILE - 1)) + (e >> 6) * LDT];
      if (rw) {
        publish_store(&a.tflag[ti], -a.epoch);
      } else {
        bf16_copy_to_global((uint16_t*)a.Lbf + ti * TILE_ELEMS, S, tid);
        publish_tile(&a.tflag[ti], &a.colcnt[J], a.epoch);
      }
      __syncthreads();   // S is rewritten by the next tile
    }
  }
}

// Row walker of a kept block (bfloat16-update factor).  The tiles (I, J), J < j0, of a new
// tile row I >= j0 below the kept leading columns K solve X L_KK^T = H_IK, a chain along the
// row (Sec. 2.1: the factor of the new F-block reuses the kept one).  The strips of these
// tiles stop ROW_TD terms short and hand over Y_J = (H_IJ - sum_{k<J-TD} X_k L_Jk^T) L_JJ^-T;
// the walker finishes
//     X_J = Y_J - sum_{j=1..TD} X_{J-j} C_{J,j}^T,   C_{J,j} = L_JJ^-1 L_{J,J-j},
// with the forward coupling tiles the previous factor formed for the kept columns (unchanged,
// as the columns are), on bfloat16 MFMA from its own last TD outputs (an LDS ring), and
// publishes X_J as a finished tile (float and bfloat16 copy).  A link of the chain is then
// TD tile products in one workgroup instead of a publish, a poll and a tile load between two.
__device__ __forceinline__ void row_walker(const FactorArgs& a, uint64_t wait_ticks, int I, char* stage) {
  typedef MF<float> M;
  typedef M::acc Acc;
  constexpr int TD = ROW_TD;
  const int tid = fresh_tid(), lane = tid & 63, w = tid >> 6;
  const int j0 = a.j0;
  float* Lt = (float*)a.Ltiles;
  uint16_t* Lb = (uint16_t*)a.Lbf;
  const uint16_t* Mc = (const uint16_t*)a.Mc;    // forward couplings first: (J TD + j - 1) tiles
  uint16_t* ring = (uint16_t*)stage;              // X_J at slot J % (TD + 1), row-major, stride LDK
  uint16_t* cst = ring + (TD + 1) * TILE * LDK;   // C_{J,j} at slot j - 1, row-major, stride LDK
  const int qr = (w & 1) * 32, qc = (w >> 1) * 32, lr = lane & 15, lk = lane >> 4;
  // a coupling tile's 16 entries of walk thread tid (row tid / 4, columns 16 (tid % 4) ..)
  // are its 16-byte chunks tid and 256 + tid, staged at row tid / 4, column 16 (tid % 4)
  const int o16 = (tid >> 2) * LDK + (tid & 3) * 16;
  u32x4 cr[TD][2];
  auto fetch_c = [&](int J1) __attribute__((always_inline)) {   // column J1's couplings
#pragma unroll
    for (int j = 0; j < TD; ++j) {
      const u32x4* p = (const u32x4*)(Mc + ((int64_t)J1 * TD + j) * TILE_ELEMS);
      cr[j][0] = p[tid];
      cr[j][1] = p[256 + tid];
    }
  };
  fetch_c(0);
  for (int J = 0; J < j0; ++J) {
    const int64_t ti = tile_index(I, J);
    float* Y = Lt + ti * TILE_ELEMS;   // column-major; Y_J in, X_J out
    spin_until(&a.tflag[ti], -a.epoch, true, a.ctrl, wait_ticks);
    acquire_agent();
    Acc acc[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          acc[bi][bj][v] = Y[(qc + 16 * bj + lr) * TILE + qr + 16 * bi + M::row(lane, v)];
#pragma unroll
    for (int j = 0; j < TD; ++j) {
      ((u32x4*)(cst + j * TILE * LDK + o16))[0] = cr[j][0];
      ((u32x4*)(cst + j * TILE * LDK + o16))[1] = cr[j][1];
    }
    __syncthreads();   // couplings staged; the ring holds X_{J-1} .. X_{J-TD}
    fetch_c(min(J + 1, j0 - 1));
#pragma unroll
    for (int j = 1; j <= TD; ++j) {
      if (J - j < 0) break;
      const uint16_t* HA = ring + ((J - j) % (TD + 1)) * TILE * LDK;
      const uint16_t* HB = cst + (j - 1) * TILE * LDK;
#pragma unroll
      for (int kh = 0; kh < TILE; kh += 32) {
        const int kofs = kh + 8 * lk;
        u32x4 x0 = *(const u32x4*)(HA + (qr + lr) * LDK + kofs);
        u32x4 x1 = *(const u32x4*)(HA + (qr + 16 + lr) * LDK + kofs);
        const u32x4 y0 = *(const u32x4*)(HB + (qc + lr) * LDK + kofs);
        const u32x4 y1 = *(const u32x4*)(HB + (qc + 16 + lr) * LDK + kofs);
        const uint32_t neg = 0x80008000u;   // X_J -= X_{J-j} C^T: negate the X operand
        x0 ^= neg;
        x1 ^= neg;
        const bf16x8 a0 = __builtin_bit_cast(bf16x8, x0), a1 = __builtin_bit_cast(bf16x8, x1);
        const bf16x8 b0 = __builtin_bit_cast(bf16x8, y0), b1 = __builtin_bit_cast(bf16x8, y1);
        acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, acc[1][1], 0, 0, 0);
      }
    }
    // X_J into the ring (its slot held X_{J-TD-1}, last read at step J-1) and the float tile
    uint16_t* HX = ring + (J % (TD + 1)) * TILE * LDK;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int rr = qr + 16 * bi + M::row(lane, v), cc = qc + 16 * bj + lr;
          HX[rr * LDK + cc] = __builtin_bit_cast(uint16_t, (__bf16)acc[bi][bj][v]);
          Y[cc * TILE + rr] = acc[bi][bj][v];
        }
    __syncthreads();   // the ring slot is complete
    u32x4* dst = (u32x4*)(Lb + ti * TILE_ELEMS + (tid >> 2) * TILE + (tid & 3) * 16);   // bfloat16 copy
    dst[0] = ((const u32x4*)(HX + o16))[0];
    dst[1] = ((const u32x4*)(HX + o16))[1];
    publish_tile(&a.tflag[ti], &a.colcnt[J], a.epoch);
  }
}

// The walker's update of the ten lower 16 x 16 blocks of a diagonal tile, U -= X X^T,
// spread over four waves (three blocks for waves 0..2, one for wave 3).  A wave's blocks
// (I0, J0), (I1, J1), (I2, J2), the first NB of them, share the block rows of X they read.
template <typename T, int NB, int I0, int J0, int I1, int J1, int I2, int J2>
__device__ __forceinline__ void lower_update(typename MF<T>::acc (&acc)[3], const T* U, const T* X, int lane) {
  typedef MF<T> M;
  constexpr int BI[3] = {I0, I1, I2}, BJ[3] = {J0, J1, J2};
  const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int b = 0; b < NB; ++b) acc[b] = load16<T>(U, 16 * BI[b], 16 * BJ[b]);
#pragma unroll
  for (int kk = 0; kk < TILE; kk += 4) {
    const int kc = kk + lk;
    T x[4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
      bool used = false;
#pragma unroll
      for (int b = 0; b < NB; ++b) used = used || BI[b] == rb || BJ[b] == rb;
      x[rb] = used ? X[(16 * rb + lr) + kc * LDT] : (T)0;
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = M::op(-x[BI[b]], x[BJ[b]], acc[b]);
  }
}
template <typename T, int NB, int I0, int J0, int I1, int J1, int I2, int J2>
__device__ __forceinline__ void lower_store(const typename MF<T>::acc (&acc)[3], T* U) {
  constexpr int BI[3] = {I0, I1, I2}, BJ[3] = {J0, J1, J2};
#pragma unroll
  for (int b = 0; b < NB; ++b) store16<T>(U, 16 * BI[b], 16 * BJ[b], acc[b]);
}

// Copy a 64 x 64 tile (column-major, leading dimension TILE) from global memory into LDS
// (leading dimension LDT) with all sixteen loads of a thread in flight at once.
template <typename T>
__device__ __forceinline__ void tile_to_lds(const T* __restrict__ g, T* X, int tid) {
  T v[TILE_ELEMS / 256];
#pragma unroll
  for (int q = 0; q < TILE_ELEMS / 256; ++q) v[q] = g[tid + q * 256];
#pragma unroll
  for (int q = 0; q < TILE_ELEMS / 256; ++q) {
    const int e = tid + q * 256;
    X[(e & (TILE - 1)) + (e >> 6) * LDT] = v[q];
  }
}

// Store the lower triangle of an LDS tile (zeros above the diagonal) to global memory,
// all of a thread's LDS reads first.
template <typename T>
__device__ __forceinline__ void lower_to_global(T* __restrict__ g, const T* X, int tid) {
  T v[TILE_ELEMS / 256];
#pragma unroll
  for (int q = 0; q < TILE_ELEMS / 256; ++q) {
    const int e = tid + q * 256, r = e & (TILE - 1), c = e >> 6;
    v[q] = (r >= c) ? X[r + c * LDT] : (T)0;
  }
#pragma unroll
  for (int q = 0; q < TILE_ELEMS / 256; ++q) g[tid + q * 256] = v[q];
}

template <typename T>
__device__ __forceinline__ void tile_to_global(T* __restrict__ g, const T* X, int tid) {
  T v[TILE_ELEMS / 256];
#pragma unroll
  for (int q = 0; q < TILE_ELEMS / 256; ++q) {
    const int e = tid + q * 256;
    v[q] = X[(e & (TILE - 1)) + (e >> 6) * LDT];
  }
#pragma unroll
  for (int q = 0; q < TILE_ELEMS / 256; ++q) g[tid + q * 256] = v[q];
}

// The walker: one workgroup carries the column-to-column chain of the factorisation.  For
// each column J it takes the partial sum that the diagonal tile (J, J) published (every
// left-looking term except the one with L_{J,J-1}), applies that last term from LDS
// (L_{J,J-1} is its own previous output), factors and inverts the diagonal tile, emits
// z_J of the forward solve, publishes L_JJ^-1 for the other tiles of the column, and
// finishes the sub-diagonal tile L_{J+1,J} = S_{J+1,J} L_JJ^-T with the inverse still in
// LDS (S_{J+1,J} being fully updated by its own workgroup meanwhile).  It then prefetches
// the next diagonal partial sum into the buffer the inverse leaves free.  Per column the
// chain keeps one hand-over from another workgroup (S_{J+1,J}) instead of three.
template <typename T, bool BF>
__device__ __forceinline__ void walker(const FactorArgs& a, uint64_t wait_ticks, T* Pbuf, T* Qbuf,
                                       double (*s_part)[TILE], double* s_rhs, double* s_z, double* s_tp) {
  typedef MF<T> M;
  typedef typename M::acc Acc;
  const int nb = a.nb, j0 = a.j0;
  const bool fwd = a.rhs != nullptr;
  T* Lt = (T*)a.Ltiles;
  T* Dv = (T*)a.Dinv;
  T* X = Pbuf;   // L_{J,J-1} from the previous column (J > j0)
  T* U = Qbuf;   // partial sum of the diagonal tile (J, J)
  // column j0's diagonal tile, fully updated by its own workgroup
  {
    const int tid = fresh_tid();
    spin_until(&a.tflag[tile_index(j0, j0)], -a.epoch, true, a.ctrl, wait_ticks);
    acquire_agent();
    tile_to_lds<T>(Lt + tile_index(j0, j0) * TILE_ELEMS, U, tid);
    if (fwd && tid < TILE) s_tp[tid] = a.z[(int64_t)j0 * TILE + tid];
    __syncthreads();
  }
  for (int J = j0; J < nb; ++J) {
    const int tid = fresh_tid(), lane = tid & 63, w = tid >> 6;
    const int64_t td = tile_index(J, J);
    const bool sub = J + 1 < nb;
    const int64_t ts = sub ? tile_index(J + 1, J) : td;
    if (J > j0) {
      // last term of the diagonal tile, from LDS: the ten lower 16 x 16 blocks of
      // U -= X X^T (X = L_{J,J-1}), three blocks per wave at most
      Acc acc[3];
      switch (__builtin_amdgcn_readfirstlane(w)) {
        case 0: lower_update<T, 3, 0, 0, 3, 0, 3, 1>(acc, U, X, lane); break;
        case 1: lower_update<T, 3, 1, 0, 1, 1, 3, 2>(acc, U, X, lane); break;
        case 2: lower_update<T, 3, 2, 0, 2, 1, 3, 3>(acc, U, X, lane); break;
        default: lower_update<T, 1, 2, 2, 0, 0, 0, 0>(acc, U, X, lane); break;
      }
      if (fwd) {   // row `lane`, columns 16 w .. 16 w + 15 of L_{J,J-1} z_{J-1}
        double t2 = 0.0;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int cc = w * 16 + q;
          t2 = fma((double)X[lane + cc * LDT], s_z[cc], t2);
        }
        s_part[w][lane] = t2;
      }
      __syncthreads();   // U and X fully read
      switch (__builtin_amdgcn_readfirstlane(w)) {
        case 0: lower_store<T, 3, 0, 0, 3, 0, 3, 1>(acc, U); break;
        case 1: lower_store<T, 3, 1, 0, 1, 1, 3, 2>(acc, U); break;
        case 2: lower_store<T, 3, 2, 0, 2, 1, 3, 3>(acc, U); break;
        default: lower_store<T, 1, 2, 2, 0, 0, 0, 0>(acc, U); break;
      }
    }
    if (fwd && tid < TILE) {
      const int p = J * TILE + tid;
      double c = 0.0;
      if (p < a.nF) c = a.rhs[a.Flist ? a.Flist[p] : p];
      const double last = (J > j0) ? (((s_part[0][tid] + s_part[1][tid]) + s_part[2][tid]) + s_part[3][tid]) : 0.0;
      s_rhs[tid] = c - (s_tp[tid] + last);
    }
    __syncthreads();
    const PivotReport rep = {J * TILE, a.nF, &a.ctrl->failed_pos, &a.ctrl->status};
    factor_invert_tile<T>(U, X, rep);   // L_JJ in U, L_JJ^-1 in X (lower triangles)
    if (fwd) {
      double zz = 0.0;
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int c = w * 16 + q;
        if (c <= lane) zz = fma((double)X[lane + c * LDT], s_rhs[c], zz);
      }
      s_part[w][lane] = zz;
      __syncthreads();
      if (tid < TILE) {
        const double z = ((s_part[0][tid] + s_part[1][tid]) + s_part[2][tid]) + s_part[3][tid];
        a.z[(int64_t)J * TILE + tid] = z;
        s_z[tid] = z;
      }
    }
    // the inverse first: the rest of the column waits for it
    lower_to_global<T>(Dv + (int64_t)J * TILE_ELEMS, X, tid);
    publish_store(&a.dflag[J], a.epoch);
    lower_to_global<T>(Lt + td * TILE_ELEMS, U, tid);
    if (!sub) {
      publish_tile(&a.tflag[td], &a.colcnt[J], a.epoch);
      break;
    }
    // S_{J+1,J}, fully updated by its own workgroup, and the next diagonal partial sum
    T* dsub = Lt + ts * TILE_ELEMS;
    const int64_t tn = tile_index(J + 1, J + 1);
    spin_until(&a.tflag[ts], -a.epoch, true, a.ctrl, wait_ticks);
    spin_until(&a.tflag[tn], -a.epoch, true, a.ctrl, wait_ticks);
    acquire_agent();
    T vn[TILE_ELEMS / 256];   // next partial sum, parked in registers until X is free
    {
      const T* gn = Lt + tn * TILE_ELEMS;
#pragma unroll
      for (int q = 0; q < TILE_ELEMS / 256; ++q) vn[q] = gn[tid + q * 256];
    }
    const double tpn = (fwd && tid < TILE) ? a.z[(int64_t)(J + 1) * TILE + tid] : 0.0;
    __syncthreads();   // L_JJ stored from U
    tile_to_lds<T>(dsub, U, tid);
    __syncthreads();
    // L_{J+1,J} = S_{J+1,J} (L_JJ^-1)^T: wave w forms block row w; block column bj takes
    // the inverse's blocks (bj, kb) for kb <= bj only (the rest of its row is zero), which
    // spreads the 160 block products evenly over the four waves
    Acc o[4];
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) o[bj] = Acc{};
    {
      const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
      for (int kb = 0; kb < 4; ++kb)
#pragma unroll
        for (int kk = 0; kk < 16; kk += 4) {
          const int kc = 16 * kb + kk + lk;
          const T av = U[(16 * w + lr) + kc * LDT];
#pragma unroll
          for (int bj = kb; bj < 4; ++bj) o[bj] = M::op(av, X[(16 * bj + lr) + kc * LDT], o[bj]);
        }
    }
    __syncthreads();   // U and X fully read
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) store16<T>(U, 16 * w, 16 * bj, o[bj]);
    __syncthreads();
    tile_to_global<T>(dsub, U, tid);
    if constexpr (BF) bf16_copy_to_global((uint16_t*)a.Lbf + ts * TILE_ELEMS, (const float*)U, tid);
    // one release covers L_JJ and L_{J+1,J}
    __syncthreads();
    if (tid == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_store(&a.tflag[td], a.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&a.tflag[ts], a.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&a.colcnt[J], 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // the next diagonal partial sum into the buffer the inverse leaves free
#pragma unroll
    for (int q = 0; q < TILE_ELEMS / 256; ++q) {
      const int e = tid + q * 256;
      X[(e & (TILE - 1)) + (e >> 6) * LDT] = vn[q];
    }
    if (fwd && tid < TILE) s_tp[tid] = tpn;
    __syncthreads();
    // U holds L_{J+1,J}: the next column's X; X holds the next partial sum
    T* tmp = X;
    X = U;
    U = tmp;
  }
}

// A persistent grid: each workgroup takes tickets until none are left, so a launch holds
// at most gridDim.x workgroups however large the F-block is (the device's resident
// workgroups by default, fewer when concurrent solves share the device).  A workgroup
// holds one ticket at a time and only waits for smaller tickets, which running workgroups
// hold, so the lowest unfinished ticket always progresses.
template <typename T, bool BF>
__global__ __launch_bounds__(256, 2) void k_chol_tiles(FactorArgs a, uint64_t wait_ticks) {
  // two staged tiles (the walker's and a single tile's buffers), or a strip's operands
  constexpr size_t TWO = 2 * (size_t)TILE * LDT * sizeof(T);
  constexpr size_t BFSTAGE = STRIP_STAGE_BYTES > ROW_STAGE_BYTES ? STRIP_STAGE_BYTES : ROW_STAGE_BYTES;
  __shared__ __attribute__((aligned(16))) char smem[BF && BFSTAGE > TWO ? BFSTAGE : TWO];
  T* S = (T*)smem;
  T* W = S + TILE * LDT;
  __shared__ double s_part[4][TILE];
  __shared__ double s_rhs[TILE];
  __shared__ double s_z[TILE];
  __shared__ double s_tp[TILE];
  __shared__ int s_t, s_kind, s_I, s_J, s_cnt;
  const bool rw = BF && a.rowwalk;
  const UnitPlan plan = {a.nb, a.j0, BF ? CHOL_STRIP : 1, CHOL_PAIR, BF, rw};
  const int64_t nunits = unit_total(plan);
  const int nrw = rw ? a.nb - a.j0 : 0;   // row walkers: tickets 1 .. nrw
  for (;;) {
    const int tid = fresh_tid();
    if (tid == 0) {
      // ticket 0 is the walker, the next nrw the row walkers, then the units
      const int t = atomicAdd(&a.ctrl->chol_ticket, 1) - 1 - nrw;
      FactorUnit f = {UNIT_TILE, 0, 0, 1};
      if (t >= 0 && t < nunits) f = unit_at(t, plan);
      s_t = t;
      s_kind = f.kind;
      s_I = f.I;
      s_J = f.J;
      s_cnt = f.cnt;
    }
    __syncthreads();
    const int t = s_t, kind = s_kind, I = s_I, J = s_J, cnt = s_cnt;
    __syncthreads();   // every thread has its ticket before thread 0 may take the next
    if (t < -nrw) {
      walker<T, BF>(a, wait_ticks, S, W, s_part, s_rhs, s_z, s_tp);
      return;
    }
    if constexpr (BF) {
      if (t < 0) {
        row_walker(a, wait_ticks, a.j0 + nrw + t, smem);
        return;
      }
    }
    if (t >= nunits) return;
    if constexpr (BF) {
      if (kind == UNIT_STRIP) {
        chol_strip<CHOL_STRIP, 1>(a, wait_ticks, I, cnt, J, smem, rw && J < a.j0);
        __syncthreads();
        continue;
      }
      if (kind == UNIT_PAIR) {
        chol_strip<CHOL_PAIR, 2>(a, wait_ticks, I, cnt, J, smem);
        __syncthreads();
        continue;
      }
    }
    chol_tile<T, BF>(a, wait_ticks, tid, I, J, S, W, s_part);
    __syncthreads();   // LDS is reused by the next tile
  }
}

template <typename T>
__global__ void k_tiles_to_dense(int n, const T* __restrict__ Lt, double* __restrict__ L, int ldl) {
  const int64_t total = (int64_t)n * n;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int c = (int)(e / n), r = (int)(e - (int64_t)c * n);
    double v = 0.0;
    if (r >= c) v = (double)Lt[tile_index(r / TILE, c / TILE) * TILE_ELEMS + (c % TILE) * TILE + (r % TILE)];
    L[r + (int64_t)c * ldl] = v;
  }
}

}  // namespace

void launch_cholesky(hipStream_t s, const FactorArgs& args, bool fp32) {
  if (args.nb <= 0 || args.j0 < 0 || args.j0 >= args.nb) return;
  FactorArgs a = args;
  const bool bf = fp32 && a.Lbf;
  // Row walkers for the rows below a kept block: the bfloat16-update factor, whose previous
  // launch formed the kept columns' couplings (a kept block implies the same precision and
  // buffers), with a few rows and a grid that leaves workers beside the walkers.
  const int nrw = a.nb - a.j0;
  a.rowwalk = bf && a.Mc && a.j0 >= ROW_TD + 2 && nrw <= 32 && (a.max_wgs == 0 || a.max_wgs >= nrw + 9);
  const UnitPlan plan = {a.nb, a.j0, bf ? CHOL_STRIP : 1, CHOL_PAIR, bf, a.rowwalk != 0};
  int64_t grid = unit_total(plan) + 1 + (a.rowwalk ? nrw : 0);   // the units and the walkers
  if (a.max_wgs > 0 && grid > a.max_wgs) grid = a.max_wgs < 2 ? 2 : a.max_wgs;   // walkers + >= 1 worker
  if (fp32 && a.Lbf)
    hipLaunchKernelGGL((k_chol_tiles<float, true>), dim3((unsigned)grid), dim3(256), 0, s, a, a.wait_ticks);
  else if (fp32)
    hipLaunchKernelGGL((k_chol_tiles<float, false>), dim3((unsigned)grid), dim3(256), 0, s, a, a.wait_ticks);
  else
    hipLaunchKernelGGL((k_chol_tiles<double, false>), dim3((unsigned)grid), dim3(256), 0, s, a, a.wait_ticks);
  if (a.Mc) launch_walk_couplings(s, a.nb, a.Ltiles, a.Dinv, a.Mc, fp32, fp32 && a.Lbf);   // for the solves
}

void launch_tiles_to_dense(hipStream_t s, int n, const void* Ltiles, bool fp32, double* L, int ldl) {
  const int64_t total = (int64_t)n * n;
  int blocks = (int)((total + 255) / 256);
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  if (fp32)
    hipLaunchKernelGGL(k_tiles_to_dense<float>, dim3(blocks), dim3(256), 0, s, n, (const float*)Ltiles, L, ldl);
  else
    hipLaunchKernelGGL(k_tiles_to_dense<double>, dim3(blocks), dim3(256), 0, s, n, (const double*)Ltiles, L, ldl);
}

}  // namespace nnls
