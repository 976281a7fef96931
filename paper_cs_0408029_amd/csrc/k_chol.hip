// Cholesky factor of the F-principal block of the cached Gram matrix and the two
// triangular solves of the normal equations (Sec. 2.1 and Sec. 3 of the tsnnls paper).
//
// Factorisation: one launch per pivot iteration.  The block is cut into 64 x 64 tiles and
// every lower tile (I, J) is one workgroup.  A workgroup takes a ticket from a counter
// (tickets are handed out in column-major lower-tile order), gathers its tile of H_FF
// straight from the Gram matrix into LDS, then computes, left-looking,
//     S_IJ = H_IJ - sum_{k<J} L_Ik L_Jk^T        (MFMA, 16x16x4 blocks)
// waiting on the per-tile ready flags of L_Ik and L_Jk.  A diagonal tile is factored and
// inverted in LDS; an off-diagonal tile becomes L_IJ = S_IJ (L_JJ^-1)^T once the diagonal
// tile (J, J) is ready.  Each finished tile publishes its flag (epoch number of the launch).
// Every dependency of a tile has a smaller ticket, and a ticket is only taken by a running
// workgroup, so the waits always end; each wait is also bounded in wall time and raises
// NNLS_ERR_DEVICE instead of spinning forever.
//
// Triangular solves: the same scheme over 64-row blocks, one workgroup per block,
// z = L^-1 c_F forward and x_F = L^-T z backward, using the inverted diagonal tiles.
#include <climits>

#include "nnls_internal.h"

namespace nnls {

namespace {

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

constexpr int LDT = TILE + 1;   // LDS leading dimension of a staged tile

// Every wave polls the flag itself, so its later loads are ordered after its own acquire.
__device__ inline bool wait_epoch(const int32_t* flag, int epoch, Ctrl* ctrl, uint64_t wait_ticks) {
  if (__hip_atomic_load(flag, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == epoch) return true;
  const uint64_t t0 = wall_clock64();
  while (__hip_atomic_load(flag, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
    if (__hip_atomic_load(&ctrl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
    if (wall_clock64() - t0 > wait_ticks) {
      __hip_atomic_store(&ctrl->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      atomicCAS(&ctrl->status, 0, (int)NNLS_ERR_DEVICE);
      return false;
    }
    __builtin_amdgcn_s_sleep(2);
  }
  return true;
}

__device__ inline void publish(int32_t* flag, int epoch) {
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(flag, epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Stage tile (I, J) of H_FF in LDS (column-major, leading dimension LDT).  Positions at or
// beyond nF are padding: identity on the diagonal, zero elsewhere.
template <typename T>
__device__ inline void gather_tile(const FactorArgs& a, int I, int J, T* S) {
  const int tid = threadIdx.x;
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
    if (tid < TILE) {
      const int c = tid, q = c0 + c;
      const int phi = min(r0 + TILE, a.nF) - 1;
      if (q < a.nF && r0 <= phi) {
        const int j = a.Flist[q];
        const int lo = a.Flist[r0], hi = a.Flist[phi];
        const int64_t s = a.lower.hptr[j], e = s + a.lower.hcnt[j];
        int64_t L = s, R = e;
        while (L < R) {
          const int64_t M = (L + R) >> 1;
          if (a.lower.hrow[M] < lo) L = M + 1; else R = M;
        }
        for (int64_t t = L; t < e; ++t) {
          const int i = a.lower.hrow[t];
          if (i > hi) break;
          const int p = a.pos[i];
          if (p >= 0) S[(p - r0) + c * LDT] = (T)a.lower.hval[t];
        }
      } else if (q >= a.nF && I == J) {
        S[c + c * LDT] = (T)1;
      }
    }
  }
  __syncthreads();
}

// Unblocked right-looking Cholesky of the lower triangle of S in LDS.
template <typename T>
__device__ inline void potrf_lds(T* S, T* s_diag, int J, const FactorArgs& a) {
  const int tid = threadIdx.x;
  const int i = tid & (TILE - 1), g = tid >> 6;
  for (int c = 0; c < TILE; ++c) {
    const T d = S[c + c * LDT];
    const bool bad = !(d > (T)0) || !isfinite(d);
    const T l = bad ? (T)1 : (T)sqrt(d);
    const T inv = (T)1 / l;
    if (tid > c && tid < TILE) S[tid + c * LDT] *= inv;
    if (tid == 0) {
      s_diag[c] = l;
      if (bad && J * TILE + c < a.nF) {
        atomicMin(&a.ctrl->failed_pos, J * TILE + c);
        atomicCAS(&a.ctrl->status, 0, (int)NNLS_ERR_NOT_PD);
      }
    }
    __syncthreads();
    if (i > c) {
      const T lic = S[i + c * LDT];
      for (int j = c + 1 + g; j <= i; j += 4) S[i + j * LDT] -= lic * S[j + c * LDT];
    }
    __syncthreads();
  }
  if (tid < TILE) S[tid + tid * LDT] = s_diag[tid];
  __syncthreads();
}

// W = L^-1 for the lower-triangular L in S.  Four lanes of one wave own a column j and
// run forward substitution down it; the column never leaves its wave.
template <typename T>
__device__ inline void trtri_lds(const T* S, T* W) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int j = w * 16 + (lane >> 2);
  const int sub = lane & 3;
  for (int i = 0; i < TILE; ++i) {
    T s = (T)0;
    if (i > j)
      for (int k = j + sub; k < i; k += 4) s += S[i + k * LDT] * W[k + j * LDT];
    s += __shfl_xor(s, 1, 64);
    s += __shfl_xor(s, 2, 64);
    if (sub == 0) {
      const T dii = S[i + i * LDT];
      W[i + j * LDT] = (i < j) ? (T)0 : (i == j) ? (T)1 / dii : -s / dii;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(256) void k_chol_tiles(FactorArgs a, uint64_t wait_ticks) {
  typedef MF<T> M;
  typedef typename M::acc Acc;
  __shared__ T S[TILE * LDT];
  __shared__ T W[TILE * LDT];
  __shared__ T s_diag[TILE];
  __shared__ int s_t, s_I, s_J;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int nb = a.nb;
  if (tid == 0) {
    const int t = atomicAdd(&a.ctrl->chol_ticket, 1);
    int J = 0, start = 0;
    if (t < tile_count(nb)) {
      while (t >= start + (nb - J)) {
        start += nb - J;
        ++J;
      }
    }
    s_t = t;
    s_I = J + (t - start);
    s_J = J;
  }
  __syncthreads();
  const int t = s_t, I = s_I, J = s_J;
  if (t >= tile_count(nb)) return;   // counter not reset: do nothing rather than go out of range
  T* Lt = (T*)a.Ltiles;
  T* Dv = (T*)a.Dinv;

  gather_tile<T>(a, I, J, S);

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
  for (int k = 0; k < J; ++k) {
    wait_epoch(&a.tile_flags[tile_index(I, k, nb)], a.epoch, a.ctrl, wait_ticks);
    if (I != J) wait_epoch(&a.tile_flags[tile_index(J, k, nb)], a.epoch, a.ctrl, wait_ticks);
    if (skip) continue;
    const T* LI = Lt + tile_index(I, k, nb) * TILE_ELEMS;
    const T* LJ = Lt + tile_index(J, k, nb) * TILE_ELEMS;
#pragma unroll
    for (int kk = 0; kk < TILE; kk += 4) {
      const int col = (kk + lk) * TILE;
      const T a0 = -LI[col + qr + lr], a1 = -LI[col + qr + 16 + lr];
      const T b0 = LJ[col + qc + lr], b1 = LJ[col + qc + 16 + lr];
      acc[0][0] = M::op(a0, b0, acc[0][0]);
      acc[0][1] = M::op(a0, b1, acc[0][1]);
      acc[1][0] = M::op(a1, b0, acc[1][0]);
      acc[1][1] = M::op(a1, b1, acc[1][1]);
    }
  }

#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        S[(qr + 16 * bi + M::row(lane, v)) + (qc + 16 * bj + lr) * LDT] = acc[bi][bj][v];
  __syncthreads();

  T* dst = Lt + (int64_t)t * TILE_ELEMS;
  if (I == J) {
    potrf_lds<T>(S, s_diag, J, a);
    trtri_lds<T>(S, W);
    T* dinv = Dv + (int64_t)J * TILE_ELEMS;
    for (int e = tid; e < TILE_ELEMS; e += 256) {
      const int r = e & (TILE - 1), c = e >> 6;
      dst[e] = (r >= c) ? S[r + c * LDT] : (T)0;
      dinv[e] = (r >= c) ? W[r + c * LDT] : (T)0;
    }
  } else {
    wait_epoch(&a.tile_flags[tile_index(J, J, nb)], a.epoch, a.ctrl, wait_ticks);
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
  }
  publish(&a.tile_flags[t], a.epoch);
}

// z_I = L_II^-1 (rhs_I - sum_{k<I} L_Ik z_k)
template <typename T>
__global__ __launch_bounds__(256) void k_trsv_fwd(SolveArgs a, uint64_t wait_ticks) {
  __shared__ double part[4][TILE];
  __shared__ double srhs[TILE];
  __shared__ int s_I;
  const int tid = threadIdx.x, r = tid & (TILE - 1), g = tid >> 6;
  if (tid == 0) s_I = atomicAdd(&a.ctrl->fwd_ticket, 1);
  __syncthreads();
  const int I = s_I, nb = a.nb;
  if (I >= nb) return;
  const T* Lt = (const T*)a.Ltiles;
  const T* Dv = (const T*)a.Dinv;
  double acc = 0.0;
  for (int k = 0; k < I; ++k) {
    wait_epoch(&a.zflags[k], a.epoch, a.ctrl, wait_ticks);
    const T* tl = Lt + tile_index(I, k, nb) * TILE_ELEMS;
    const double* zk = a.z + (int64_t)k * TILE;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int cc = g * 16 + q;
      acc = fma((double)tl[cc * TILE + r], zk[cc], acc);
    }
  }
  part[g][r] = acc;
  __syncthreads();
  if (tid < TILE) {
    const int p = I * TILE + tid;
    double rhs = 0.0;
    if (p < a.nF) rhs = a.rhs_full ? a.rhs_full[a.Flist ? a.Flist[p] : p] : a.rhs_dense[p];
    srhs[tid] = rhs - (((part[0][tid] + part[1][tid]) + part[2][tid]) + part[3][tid]);
  }
  __syncthreads();
  const T* D = Dv + (int64_t)I * TILE_ELEMS;
  double zz = 0.0;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int c = g * 16 + q;
    zz = fma((double)D[c * TILE + r], srhs[c], zz);
  }
  part[g][r] = zz;
  __syncthreads();
  if (tid < TILE)
    a.z[(int64_t)I * TILE + tid] = ((part[0][tid] + part[1][tid]) + part[2][tid]) + part[3][tid];
  publish(&a.zflags[I], a.epoch);
}

// x_I = L_II^-T (z_I - sum_{k>I} L_kI^T x_k); scatter x_I through F
template <typename T>
__global__ __launch_bounds__(256) void k_trsv_bwd(SolveArgs a, uint64_t wait_ticks) {
  __shared__ double ssum[TILE];
  __shared__ double srhs[TILE];
  __shared__ double part[4][TILE];
  __shared__ int s_I;
  const int tid = threadIdx.x, r = tid & (TILE - 1), g = tid >> 6;
  if (tid == 0) s_I = a.nb - 1 - atomicAdd(&a.ctrl->bwd_ticket, 1);
  __syncthreads();
  const int I = s_I, nb = a.nb;
  if (I < 0) return;
  const T* Lt = (const T*)a.Ltiles;
  const T* Dv = (const T*)a.Dinv;
  double accl[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) accl[q] = 0.0;
  for (int k = nb - 1; k > I; --k) {
    wait_epoch(&a.xflags[k], a.epoch, a.ctrl, wait_ticks);
    const T* tl = Lt + tile_index(k, I, nb) * TILE_ELEMS;
    const double xr = a.xF[(int64_t)k * TILE + r];
#pragma unroll
    for (int q = 0; q < 16; ++q) accl[q] = fma((double)tl[(g * 16 + q) * TILE + r], xr, accl[q]);
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    double v = accl[q];
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    if (r == 0) ssum[g * 16 + q] = v;
  }
  __syncthreads();
  if (tid < TILE) srhs[tid] = a.z[(int64_t)I * TILE + tid] - ssum[tid];
  __syncthreads();
  const T* D = Dv + (int64_t)I * TILE_ELEMS;
  double xx = 0.0;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int c = g * 16 + q;
    xx = fma((double)D[r * TILE + c], srhs[c], xx);
  }
  part[g][r] = xx;
  __syncthreads();
  if (tid < TILE) {
    const double v = ((part[0][tid] + part[1][tid]) + part[2][tid]) + part[3][tid];
    const int p = I * TILE + tid;
    a.xF[p] = v;
    if (a.out && p < a.nF) a.out[a.Flist ? a.Flist[p] : p] = v;
  }
  publish(&a.xflags[I], a.epoch);
}

template <typename T>
__global__ void k_tiles_to_dense(int n, int nb, const T* __restrict__ Lt, double* __restrict__ L, int ldl) {
  const int64_t total = (int64_t)n * n;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int c = (int)(e / n), r = (int)(e - (int64_t)c * n);
    double v = 0.0;
    if (r >= c) v = (double)Lt[tile_index(r / TILE, c / TILE, nb) * TILE_ELEMS + (c % TILE) * TILE + (r % TILE)];
    L[r + (int64_t)c * ldl] = v;
  }
}

}  // namespace

void launch_cholesky(hipStream_t s, const FactorArgs& a, bool fp32) {
  const int64_t grid = tile_count(a.nb);
  if (grid <= 0) return;
  if (fp32)
    hipLaunchKernelGGL(k_chol_tiles<float>, dim3((unsigned)grid), dim3(256), 0, s, a, a.wait_ticks);
  else
    hipLaunchKernelGGL(k_chol_tiles<double>, dim3((unsigned)grid), dim3(256), 0, s, a, a.wait_ticks);
}

void launch_trsv(hipStream_t s, const SolveArgs& a, bool fp32) {
  if (a.nb <= 0) return;
  if (fp32) {
    hipLaunchKernelGGL(k_trsv_fwd<float>, dim3(a.nb), dim3(256), 0, s, a, a.wait_ticks);
    hipLaunchKernelGGL(k_trsv_bwd<float>, dim3(a.nb), dim3(256), 0, s, a, a.wait_ticks);
  } else {
    hipLaunchKernelGGL(k_trsv_fwd<double>, dim3(a.nb), dim3(256), 0, s, a, a.wait_ticks);
    hipLaunchKernelGGL(k_trsv_bwd<double>, dim3(a.nb), dim3(256), 0, s, a, a.wait_ticks);
  }
}

void launch_tiles_to_dense(hipStream_t s, int n, int nb, const void* Ltiles, bool fp32, double* L, int ldl) {
  const int64_t total = (int64_t)n * n;
  int blocks = (int)((total + 255) / 256);
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  if (fp32)
    hipLaunchKernelGGL(k_tiles_to_dense<float>, dim3(blocks), dim3(256), 0, s, n, nb, (const float*)Ltiles, L, ldl);
  else
    hipLaunchKernelGGL(k_tiles_to_dense<double>, dim3(blocks), dim3(256), 0, s, n, nb, (const double*)Ltiles, L, ldl);
}

}  // namespace nnls
