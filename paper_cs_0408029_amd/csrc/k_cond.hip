// Condition estimate of the final F-block, for the error control of Sec. 3 of the tsnnls
// paper (it estimates the condition of A_F^T A_F from the Cholesky factor with LAPACK's
// dpocon and switches to a more accurate final solve when the predicted normal-equations
// error, about kappa^2 eps (Sec. 2.1), is too large).
//
// ||H_FF||_1 is computed exactly; ||H_FF^-1||_1 is estimated by Hager's method with
// Higham's refinements, whose solves use the split's cached factor (triangular-solve
// kernels) and whose vector steps are the single-workgroup kernel below.  The host drives
// the few rounds of the method and reads four scalars per round.
#include "nnls_internal.h"

namespace nnls {

namespace {

constexpr int EST_THREADS = 1024;

__device__ inline uint64_t dbits(double v) { return (uint64_t)__double_as_longlong(v); }

// ||H_FF||_1 = max over F columns of the sum of |H_{F_p F_q}| over the F rows: one wave
// per column, lane-strided partial sums and a fixed xor tree, then the maximum through the
// bits of non-negative doubles (ordered like the values), so the result is exact and does
// not depend on the launch.  Sparse source: the whole Gram column (lower entries, then the
// mirrored upper ones) restricted to F through pos; dense source: H column-major.
__global__ __launch_bounds__(256) void k_block_onenorm(int nF, GramLower g, const int32_t* __restrict__ upcnt,
                                                       const int32_t* __restrict__ pos,
                                                       const double* __restrict__ Hd, int64_t ldh,
                                                       const int32_t* __restrict__ Flist, CondEst* est) {
  const int lane = threadIdx.x & 63;
  const int q = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (q >= nF) return;
  const int j = Flist[q];
  double s = 0.0;
  if (Hd) {
    const double* col = Hd + (int64_t)j * ldh;
    for (int p = lane; p < nF; p += 64) s += fabs(col[Flist[p]]);
  } else {
    const int64_t b = g.hptr[j];
    const int cnt = g.hcnt[j] + upcnt[j];
    for (int t = lane; t < cnt; t += 64)
      if (pos[g.hrow[b + t]] >= 0) s += fabs(g.hval[b + t]);
  }
  for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
  if (lane == 0) atomicMax((unsigned long long*)&est->hnorm, (unsigned long long)dbits(s));
}

// Vector steps of the estimator on length-nF vectors in F-position order.
//   EST_SET_UNIFORM: v = 1/n;  EST_SET_UNIT: v = e_j (j from est);
//   EST_SET_ALT:     v_p = (-1)^p (1 + p / (n - 1));
//   EST_SIGNS:       est->ynorm = ||y||_1, est->changed = any sign(y_p) != xi_p, xi = sign(y)
//                    (sign: +1 for y >= 0, else -1);
//   EST_ARGMAX:      est->zjlast = |z_j| at the current j, then j = first index of max |z|,
//                    est->zmax = that maximum.
// Sums and the arg-max run in a fixed order (thread-strided, then by wave in turn).
__global__ __launch_bounds__(EST_THREADS) void k_est_vec(int mode, int nF, double* __restrict__ v,
                                                       const double* __restrict__ y,
                                                       double* __restrict__ xi, CondEst* est) {
  __shared__ double s_sum[EST_THREADS / 64];
  __shared__ double s_max[EST_THREADS / 64];
  __shared__ int s_idx[EST_THREADS / 64], s_chg[EST_THREADS / 64];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (mode == EST_SET_UNIFORM || mode == EST_SET_UNIT || mode == EST_SET_ALT) {
    const int jj = est->j;
    for (int p = tid; p < nF; p += EST_THREADS) {
      double val;
      if (mode == EST_SET_UNIFORM) val = 1.0 / nF;
      else if (mode == EST_SET_UNIT) val = (p == jj) ? 1.0 : 0.0;
      else val = ((p & 1) ? -1.0 : 1.0) * (1.0 + (double)p / (double)(nF - 1));
      v[p] = val;
    }
    return;
  }
  if (mode == EST_SIGNS) {
    double s = 0.0;
    int chg = 0;
    for (int p = tid; p < nF; p += EST_THREADS) {
      const double yy = y[p];
      const double sg = (yy >= 0.0) ? 1.0 : -1.0;
      s += fabs(yy);
      chg |= (sg != xi[p]);
      xi[p] = sg;
    }
    for (int d = 32; d >= 1; d >>= 1) {
      s += __shfl_xor(s, d, 64);
      chg |= __shfl_xor(chg, d, 64);
    }
    if (lane == 0) {
      s_sum[w] = s;
      s_chg[w] = chg;
    }
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      int c = 0;
      for (int q = 0; q < EST_THREADS / 64; ++q) {
        t += s_sum[q];
        c |= s_chg[q];
      }
      est->ynorm = t;
      est->changed = c;
    }
    return;
  }
  // EST_ARGMAX on z = y
  double m = -1.0;
  int idx = 0x7fffffff;
  for (int p = tid; p < nF; p += EST_THREADS) {
    const double a = fabs(y[p]);
    if (a > m) {   // p ascends per thread: the first maximum of this thread's entries
      m = a;
      idx = p;
    }
  }
  for (int d = 32; d >= 1; d >>= 1) {
    const double mo = __shfl_xor(m, d, 64);
    const int io = __shfl_xor(idx, d, 64);
    if (mo > m || (mo == m && io < idx)) {
      m = mo;
      idx = io;
    }
  }
  if (lane == 0) {
    s_max[w] = m;
    s_idx[w] = idx;
  }
  __syncthreads();
  if (tid == 0) {
    double bm = -1.0;
    int bi = 0x7fffffff;
    for (int q = 0; q < EST_THREADS / 64; ++q)
      if (s_max[q] > bm || (s_max[q] == bm && s_idx[q] < bi)) {
        bm = s_max[q];
        bi = s_idx[q];
      }
    const int jl = est->j;
    est->zjlast = (jl >= 0 && jl < nF) ? fabs(y[jl]) : -1.0;
    est->j = bi;
    est->zmax = bm;
  }
}

}  // namespace

void launch_block_onenorm(hipStream_t s, int nF, GramLower g, const int32_t* upcnt, const int32_t* pos,
                          const double* Hd, int64_t ldh, const int32_t* Flist, CondEst* est) {
  if (nF <= 0) return;
  hipLaunchKernelGGL(k_block_onenorm, dim3((nF + 3) / 4), dim3(256), 0, s, nF, g, upcnt, pos, Hd, ldh,
                     Flist, est);
}

void launch_est_vec(hipStream_t s, int mode, int nF, double* v, const double* y, double* xi, CondEst* est) {
  hipLaunchKernelGGL(k_est_vec, dim3(1), dim3(EST_THREADS), 0, s, mode, nF, v, y, xi, est);
}

}  // namespace nnls
