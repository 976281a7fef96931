// Batched dense NNLS: one launch solves many independent problems; each workgroup owns
// one problem and runs its whole block principal pivoting loop (Sec. 2 algorithm box of
// the tsnnls paper) on the device, with no host round trip per iteration:
//   Gram H = A^T A and c = A^T b (Sec. 3, Sec. 2.1), then per iteration the classify /
//   count / exchange step, the left-looking tiled Cholesky of H_FF on MFMA (one tile after
//   another inside the workgroup, with the same in-LDS diagonal factor as the large-problem
//   kernel), the two triangular solves, r = A_F x_F - b and y_G = A_G^T r (Eq. 5).
// The factor is float64, or float32 followed by float64 refinement of x_F against the
// residual from A.  A problem's arithmetic never depends on the other problems in the
// launch, so every result is the same alone or in any batch.
#include <climits>

#include "tile_ops.h"

namespace nnls {

namespace {

constexpr int BT = 256;   // threads per workgroup

// Workspace layout of one problem (byte offsets from its base).
struct WsLayout {
  size_t H, c, r, flags, Flist, Lt, Dv, z, xF, g, total;
};

__host__ __device__ inline WsLayout ws_layout(int m, int n) {
  const int nb = (n + TILE - 1) / TILE;
  const size_t nt = (size_t)nb * (nb + 1) / 2;
  WsLayout L;
  size_t o = 0;
  L.H = o;     o += ((size_t)n * n * 8 + 255) & ~(size_t)255;
  L.c = o;     o += ((size_t)n * 8 + 255) & ~(size_t)255;
  L.r = o;     o += ((size_t)m * 8 + 255) & ~(size_t)255;
  L.flags = o; o += ((size_t)n + 255) & ~(size_t)255;
  L.Flist = o; o += ((size_t)n * 4 + 255) & ~(size_t)255;
  L.Lt = o;    o += nt * TILE_ELEMS * 8;              // sized for float64 tiles
  L.Dv = o;    o += (size_t)nb * TILE_ELEMS * 8;
  L.z = o;     o += (size_t)nb * TILE * 8;
  L.xF = o;    o += (size_t)nb * TILE * 8;
  L.g = o;     o += (size_t)nb * TILE * 8;
  L.total = o;
  return L;
}

// ------------------------------------------------------------ workgroup reductions
__device__ inline double wg_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  return ((red[0] + red[1]) + red[2]) + red[3];
}
__device__ inline double wg_max(double v, double* red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int d = 32; d >= 1; d >>= 1) v = fmax(v, __shfl_xor(v, d, 64));
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  return fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}
__device__ inline double wg_min(double v, double* red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int d = 32; d >= 1; d >>= 1) v = fmin(v, __shfl_xor(v, d, 64));
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  return fmin(fmin(red[0], red[1]), fmin(red[2], red[3]));
}

// ------------------------------------------------------------ Gram matrix
// H = A^T A (full symmetric, column-major n x n) and c = A^T b.  Lower 64 x 64 tiles on
// MFMA float64; rows of A are staged in LDS 64 at a time (both column blocks of the tile),
// so every H_ij is summed over rows in a fixed order.
__device__ __noinline__ void wg_gram(const double* __restrict__ A, int lda, int m, int n, const double* __restrict__ b,
                        double* __restrict__ H, double* __restrict__ c, double* Sa, double* Sb) {
  typedef MF<double> M;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int qr = (w & 1) * 32, qc = (w >> 1) * 32, lr = lane & 15, lk = lane >> 4;
  const int nb = (n + TILE - 1) / TILE;
  for (int J = 0; J < nb; ++J)
    for (int I = J; I < nb; ++I) {
      M::acc acc[2][2];
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = (M::acc){0.0, 0.0, 0.0, 0.0};
      for (int r0 = 0; r0 < m; r0 += TILE) {
        // stage rows r0 .. r0+63 of column blocks I and J: Sa[row + col*LDT]
        __syncthreads();
        for (int e = tid; e < TILE_ELEMS; e += BT) {
          const int rr = e & (TILE - 1), cc = e >> 6;
          const int row = r0 + rr, ci = I * TILE + cc, cj = J * TILE + cc;
          Sa[rr + cc * LDT] = (row < m && ci < n) ? A[row + (int64_t)ci * lda] : 0.0;
          Sb[rr + cc * LDT] = (row < m && cj < n) ? A[row + (int64_t)cj * lda] : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < TILE; kk += 4) {
          const int k = kk + lk;
          const double a0 = Sa[k + (qr + lr) * LDT], a1 = Sa[k + (qr + 16 + lr) * LDT];
          const double b0 = Sb[k + (qc + lr) * LDT], b1 = Sb[k + (qc + 16 + lr) * LDT];
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
          for (int v = 0; v < 4; ++v) {
            const int i = I * TILE + qr + 16 * bi + M::row(lane, v);
            const int j = J * TILE + qc + 16 * bj + lr;
            if (i < n && j < n) {
              H[i + (int64_t)j * n] = acc[bi][bj][v];
              H[j + (int64_t)i * n] = acc[bi][bj][v];
            }
          }
    }
  // c_j = a_j^T b: one wave per column, lane-stride partials and a fixed tree
  for (int j = w; j < n; j += 4) {
    const double* col = A + (int64_t)j * lda;
    double s = 0.0;
    for (int q = lane; q < m; q += 64) s = fma(col[q], b[q], s);
    for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
    if (lane == 0) c[j] = s;
  }
  __syncthreads();
}

// ------------------------------------------------------------ factor and solves
// Out-of-line wrapper: the diagonal factor gets its own register allocation.
template <typename T>
__device__ __noinline__ void diag_tile(T* S, T* W, PivotReport rep) {
  factor_invert_tile<T>(S, W, rep);
}

// Left-looking tiled Cholesky of H_FF inside one workgroup (tiles one after another).
// Tiles (column-major packed) and inverted diagonal tiles go to the problem's workspace.
template <typename T>
__device__ __noinline__ void wg_factor(const double* __restrict__ H, int n, const int32_t* __restrict__ Flist, int nF,
                          T* Lt, T* Dv, T* S, T* W, const PivotReport& rep0) {
  typedef MF<T> M;
  typedef typename M::acc Acc;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int qr = (w & 1) * 32, qc = (w >> 1) * 32, lr = lane & 15, lk = lane >> 4;
  const int nb = (nF + TILE - 1) / TILE;
  for (int J = 0; J < nb; ++J)
    for (int I = J; I < nb; ++I) {
      // gather tile (I, J) of H_FF; positions past nF are identity padding
      __syncthreads();
      for (int e = tid; e < TILE_ELEMS; e += BT) {
        const int rr = e & (TILE - 1), cc = e >> 6;
        const int p = I * TILE + rr, q = J * TILE + cc;
        double v = (p == q) ? 1.0 : 0.0;
        if (p < nF && q < nF) v = H[Flist[p] + (int64_t)Flist[q] * n];
        S[rr + cc * LDT] = (T)v;
      }
      __syncthreads();
      Acc acc[2][2];
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            acc[bi][bj][v] = S[(qr + 16 * bi + M::row(lane, v)) + (qc + 16 * bj + lr) * LDT];
      const bool skip = (I == J) && (qr < qc);
      if (!skip)
        for (int k = 0; k < J; ++k) {
          const T* LI = Lt + tile_index(I, k) * TILE_ELEMS;
          const T* LJ = Lt + tile_index(J, k) * TILE_ELEMS;
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
      T* dst = Lt + tile_index(I, J) * TILE_ELEMS;
      if (I == J) {
        PivotReport rep = rep0;
        rep.base = J * TILE;
        diag_tile<T>(S, W, rep);
        T* dinv = Dv + (int64_t)J * TILE_ELEMS;
        for (int e = tid; e < TILE_ELEMS; e += BT) {
          const int rr = e & (TILE - 1), cc = e >> 6;
          dst[e] = (rr >= cc) ? S[rr + cc * LDT] : (T)0;
          dinv[e] = (rr >= cc) ? W[rr + cc * LDT] : (T)0;
        }
      } else {
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
        for (int e = tid; e < TILE_ELEMS; e += BT) dst[e] = S[(e & (TILE - 1)) + (e >> 6) * LDT];
      }
      __syncthreads();
    }
}

// (L L^T) u = rhs for the tiled factor: forward then backward, block by block, float64
// arithmetic.  rhs and u are indexed by F position; rhs may alias nothing else.
template <typename T>
__device__ __noinline__ void wg_solve(const T* Lt, const T* Dv, int nF, const double* rhs, double* z, double* u,
                         double* part, double* vec) {
  const int tid = threadIdx.x, r = tid & 63, g = tid >> 6;
  const int nb = (nF + TILE - 1) / TILE;
  for (int I = 0; I < nb; ++I) {
    double acc = 0.0;
    for (int k = 0; k < I; ++k) {
      const T* tl = Lt + tile_index(I, k) * TILE_ELEMS;
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int cc = g * 16 + q;
        acc = fma((double)tl[cc * TILE + r], z[k * TILE + cc], acc);
      }
    }
    part[g * TILE + r] = acc;
    __syncthreads();
    if (tid < TILE) {
      const int p = I * TILE + tid;
      vec[tid] = (p < nF ? rhs[p] : 0.0) - (((part[tid] + part[TILE + tid]) + part[2 * TILE + tid]) + part[3 * TILE + tid]);
    }
    __syncthreads();
    const T* D = Dv + (int64_t)I * TILE_ELEMS;
    double zz = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int cc = g * 16 + q;
      zz = fma((double)D[cc * TILE + r], vec[cc], zz);
    }
    part[g * TILE + r] = zz;
    __syncthreads();
    if (tid < TILE) z[I * TILE + tid] = ((part[tid] + part[TILE + tid]) + part[2 * TILE + tid]) + part[3 * TILE + tid];
    __syncthreads();
  }
  for (int I = nb - 1; I >= 0; --I) {
    double acc = 0.0;
    for (int k = nb - 1; k > I; --k) {
      const T* tl = Lt + tile_index(k, I) * TILE_ELEMS;
      // (L_kI^T u_k)[c] for c = tid & 63, rows split over the four waves
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int rr = g * 16 + q;
        acc = fma((double)tl[r * TILE + rr], u[k * TILE + rr], acc);
      }
    }
    part[g * TILE + r] = acc;
    __syncthreads();
    if (tid < TILE)
      vec[tid] = z[I * TILE + tid] - (((part[tid] + part[TILE + tid]) + part[2 * TILE + tid]) + part[3 * TILE + tid]);
    __syncthreads();
    const T* D = Dv + (int64_t)I * TILE_ELEMS;
    double xx = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int cc = g * 16 + q;
      xx = fma((double)D[r * TILE + cc], vec[cc], xx);
    }
    part[g * TILE + r] = xx;
    __syncthreads();
    if (tid < TILE) u[I * TILE + tid] = ((part[tid] + part[TILE + tid]) + part[2 * TILE + tid]) + part[3 * TILE + tid];
    __syncthreads();
  }
}

// r = A x - b over the free columns (ascending), then y_j = a_j^T r on G and, with g,
// g_p = a_{F[p]}^T r on F.
__device__ __noinline__ void wg_residual_dual(const double* __restrict__ A, int lda, int m, int n, const double* __restrict__ b,
                                 const uint8_t* flags, const int32_t* Flist, int nF, const double* x,
                                 double* r, double* y, double* g) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int i = tid; i < m; i += BT) {
    double s = 0.0;
    for (int p = 0; p < nF; ++p) {
      const int j = Flist[p];
      s = fma(A[i + (int64_t)j * lda], x[j], s);
    }
    r[i] = s - b[i];
  }
  __syncthreads();
  for (int j = w; j < n; j += 4) {
    const bool f = flags[j] != 0;
    if (f && !g) {
      if (lane == 0) y[j] = 0.0;
      continue;
    }
    const double* col = A + (int64_t)j * lda;
    double s = 0.0;
    for (int q = lane; q < m; q += 64) s = fma(col[q], r[q], s);
    for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
    if (lane == 0) y[j] = f ? 0.0 : s;
  }
  if (g) {
    __syncthreads();
    for (int p = tid; p < nF; p += BT) {
      // g is indexed by position: recompute from the column (cheap next to the sweep above)
      const int j = Flist[p];
      const double* col = A + (int64_t)j * lda;
      double s0 = 0.0, s1 = 0.0;
      int q = 0;
      for (; q + 1 < m; q += 2) {
        s0 = fma(col[q], r[q], s0);
        s1 = fma(col[q + 1], r[q + 1], s1);
      }
      if (q < m) s0 = fma(col[q], r[q], s0);
      g[p] = s0 + s1;
    }
  }
  __syncthreads();
}

// Eq. 3 on G: y_j = sum_p H[F_p, j] x[F_p] - c_j (H symmetric: column j), y_F = 0.
__device__ __noinline__ void wg_dual_gram(const double* __restrict__ H, int n, const double* __restrict__ c,
                                          const uint8_t* flags, const int32_t* Flist, int nF,
                                          const double* x, double* y) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int j = w; j < n; j += BT / 64) {
    if (flags[j]) {
      if (lane == 0) y[j] = 0.0;
      continue;
    }
    const double* col = H + (int64_t)j * n;
    double s = 0.0;
    for (int p = lane; p < nF; p += 64) {
      const int i = Flist[p];
      s = fma(col[i], x[i], s);
    }
    for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
    if (lane == 0) y[j] = s - c[j];
  }
  __syncthreads();
}

__global__ __launch_bounds__(BT, 2) void k_batched(BatchArgs a) {
  __shared__ double S64[TILE * LDT];
  __shared__ double W64[TILE * LDT];
  __shared__ double red[8];
  __shared__ double part[4 * TILE];
  __shared__ double vec[TILE];
  __shared__ int s_int[8];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int pi = a.order ? a.order[blockIdx.x] : (int)blockIdx.x;
  if (pi >= a.count) return;
  const BatchProblem P = a.probs[pi];
  const int m = P.m, n = P.n;
  const WsLayout Lw = ws_layout(m, n);
  char* base = a.ws + P.ws;
  double* H = (double*)(base + Lw.H);
  double* c = (double*)(base + Lw.c);
  double* r = (double*)(base + Lw.r);
  uint8_t* flags = (uint8_t*)(base + Lw.flags);
  int32_t* Flist = (int32_t*)(base + Lw.Flist);
  double* z = (double*)(base + Lw.z);
  double* xF = (double*)(base + Lw.xF);
  double* gpos = (double*)(base + Lw.g);
  double* x = P.x;
  double* y = P.y;
  BatchInfo* info = a.info + pi;
  int32_t* status = &info->status;
  int32_t* failed_pos = &info->failed_index;

  // validation: non-finite A or b
  double bad = 0.0;
  for (int64_t e = tid; e < (int64_t)m * n; e += BT) {
    const int64_t j = e / m, i = e - j * m;
    if (!isfinite(P.A[i + j * P.lda])) bad = 1.0;
  }
  for (int i = tid; i < m; i += BT)
    if (!isfinite(P.b[i])) bad = 1.0;
  if (wg_max(bad, red) > 0.0) {
    if (tid == 0) {   // every field: the status array may hold an earlier launch's values
      info->status = NNLS_ERR_INVALID_VALUE;
      info->iterations = 0;
      info->n_free = 0;
      info->last_ninf = 0;
      info->failed_index = -1;
      info->ir_steps = 0;
      info->min_margin = 0.0;
    }
    return;
  }

  wg_gram(P.A, P.lda, m, n, P.b, H, c, S64, W64);
  for (int i = tid; i < n; i += BT) {
    x[i] = 0.0;
    y[i] = -c[i];
    flags[i] = 0;
  }
  if (tid == 0) {
    info->status = 0;
    info->failed_index = INT32_MAX;
    info->ir_steps = 0;
  }
  __syncthreads();

  const int max_iter = a.max_iter > 0 ? a.max_iter : 5 * n + 100;
  int N = INT32_MAX, p = a.p_max, iter = 0, nF = 0, k = 0, result = 0;
  double margin = INFINITY;
  for (;;) {
    // classify: zero |v| < tau, count negatives, largest infeasible index; a tested
    // entry that is not finite ends the problem with NNLS_ERR_INVALID_VALUE
    double cnt = 0.0, rmx = -1.0, mar = INFINITY, nonfin = 0.0;
    for (int i = tid; i < n; i += BT) {
      const bool f = flags[i] != 0;
      const double v = f ? x[i] : y[i];
      if (!isfinite(v)) {
        nonfin = 1.0;
      } else if (fabs(v) < a.tau) {
        if (f) x[i] = 0.0; else y[i] = 0.0;
      } else {
        mar = fmin(mar, fabs(v));
        if (v < 0.0) {
          cnt += 1.0;
          rmx = (double)i;
        }
      }
    }
    k = (int)wg_sum(cnt, red);
    const int rmax = (int)wg_max(rmx, red);
    margin = wg_min(mar, red);
    if (wg_max(nonfin, red) > 0.0) {
      result = NNLS_ERR_INVALID_VALUE;
      break;
    }
    if (k == 0) break;
    if (iter >= max_iter) {
      result = NNLS_ERR_MAXITER;
      break;
    }
    int branch;
    if (k < N) {
      N = k;
      p = a.p_max;
      branch = 0;
    } else if (p > 0) {
      p -= 1;
      branch = 1;
    } else {
      branch = 2;
    }
    ++iter;
    for (int i = tid; i < n; i += BT) {
      const uint8_t f = flags[i];
      const double v = f ? x[i] : y[i];
      const bool flip = (branch == 2) ? (i == rmax) : (v < 0.0);
      if (flip) flags[i] = f ^ 1;
    }
    __syncthreads();
    // F list (ascending) by a scan over chunks of BT
    int off = 0;
    for (int i0 = 0; i0 < n; i0 += BT) {
      const int i = i0 + tid;
      const bool in = (i < n) && flags[i];
      const uint64_t bal = __ballot(in);
      const int below = __popcll(bal & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
      if (lane == 0) s_int[w] = __popcll(bal);
      __syncthreads();
      int pre = 0;
      for (int q = 0; q < w; ++q) pre += s_int[q];
      if (in) Flist[off + pre + below] = i;
      off += (s_int[0] + s_int[1]) + (s_int[2] + s_int[3]);
      __syncthreads();
    }
    nF = off;
    for (int i = tid; i < n; i += BT) {
      if (flags[i]) y[i] = 0.0; else x[i] = 0.0;
    }
    __syncthreads();

    bool y_done = false;
    if (nF > 0) {
      const PivotReport rep = {0, nF, failed_pos, status};
      bool use32 = a.fp32 != 0;
      for (int attempt = 0; attempt < 2 && !y_done; ++attempt) {
        if (use32) {
          wg_factor<float>(H, n, Flist, nF, (float*)(base + Lw.Lt), (float*)(base + Lw.Dv),
                           (float*)S64, (float*)W64, rep);
        } else {
          wg_factor<double>(H, n, Flist, nF, (double*)(base + Lw.Lt), (double*)(base + Lw.Dv), S64, W64, rep);
        }
        __syncthreads();
        if (use32 && *status == NNLS_ERR_NOT_PD) {   // float32 breakdown: float64 instead
          __syncthreads();
          if (tid == 0) {
            *status = 0;
            *failed_pos = INT32_MAX;
          }
          __syncthreads();
          use32 = false;
          continue;
        }
        if (*status != 0) break;
        // c_F by position into gpos, then x_F
        for (int q = tid; q < nF; q += BT) gpos[q] = c[Flist[q]];
        __syncthreads();
        if (use32)
          wg_solve<float>((float*)(base + Lw.Lt), (float*)(base + Lw.Dv), nF, gpos, z, xF, part, vec);
        else
          wg_solve<double>((double*)(base + Lw.Lt), (double*)(base + Lw.Dv), nF, gpos, z, xF, part, vec);
        for (int q = tid; q < nF; q += BT) x[Flist[q]] = xF[q];
        __syncthreads();
        if (!use32) break;
        // float64 refinement of x_F against the residual from A
        bool converged = false;
        double prev = INFINITY;
        for (int step = 0;; ++step) {
          wg_residual_dual(P.A, P.lda, m, n, P.b, flags, Flist, nF, x, r, y, gpos);
          if (converged) {
            y_done = true;
            break;
          }
          if (step >= a.ir_max_steps) break;
          wg_solve<float>((float*)(base + Lw.Lt), (float*)(base + Lw.Dv), nF, gpos, z, xF, part, vec);
          double dm = 0.0, xm = 0.0;
          for (int q = tid; q < nF; q += BT) {
            const int j = Flist[q];
            const double v = x[j] - xF[q];
            x[j] = v;
            dm = fmax(dm, fabs(xF[q]));
            xm = fmax(xm, fabs(v));
            if (!isfinite(xF[q]) || !isfinite(v)) dm = INFINITY;   // fmax drops NaN
          }
          dm = wg_max(dm, red);
          xm = wg_max(xm, red);
          if (tid == 0) info->ir_steps += 1;
          if (!(dm < INFINITY) || !(xm < INFINITY)) break;
          // as in the single-problem path: while the corrections contract by 1/2 or better,
          // the last one bounds the error left; stop once it is below the target
          const double rho = dm / prev;   // 0 on the first step
          if (dm <= a.ir_rtol * xm) converged = true;
          else if (rho > 0.5) break;
          prev = dm;
        }
        if (!y_done) use32 = false;   // not refined to the target: redo in float64
      }
      __syncthreads();
      if (*status != 0) {
        result = *status;
        break;
      }
    }
    if (!y_done) {
      if (a.gram_dual) wg_dual_gram(H, n, c, flags, Flist, nF, x, y);
      else wg_residual_dual(P.A, P.lda, m, n, P.b, flags, Flist, nF, x, r, y, nullptr);
    }
  }
  __syncthreads();
  if (tid == 0) {
    if (result == 0) result = *status;
    info->status = result;
    info->iterations = iter;
    info->n_free = nF;
    info->last_ninf = k;
    info->min_margin = margin;
    if (result == NNLS_ERR_NOT_PD) {
      const int fp = *failed_pos;
      info->failed_index = (fp >= 0 && fp < nF) ? Flist[fp] : -1;
    } else {
      info->failed_index = -1;
    }
  }
}

}  // namespace

size_t batched_workspace_bytes(int m, int n) { return ws_layout(m, n).total; }

void launch_batched(hipStream_t s, const BatchArgs& a, int grid) {
  if (grid <= 0) return;
  hipLaunchKernelGGL(k_batched, dim3(grid), dim3(BT), 0, s, a);
}

}  // namespace nnls
