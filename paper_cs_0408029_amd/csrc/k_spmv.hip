// Residual and dual of a complementary basic solution (Eq. 5 of the tsnnls paper):
//   r   = A_F x_F - b      (x holds x_F on F and exact zeros on G)
//   y_G = A_G^T r,  y_F = 0
// Both are FP64 and memory bound.  r is a row sweep over the CSR copy of A (each row sum
// in ascending column order); y is a column sweep over the CSC input (ascending row
// order), so both results are independent of the launch configuration.
#include "nnls_internal.h"

namespace nnls {

namespace {

// One wave handles 64 consecutive rows, one row per lane.
// r = A x - b over the row-major copy, L lanes per row: each lane takes a fixed stride of
// the row's entries (consecutive lanes read consecutive entries, and consecutive rows are
// adjacent, so the loads coalesce), then a fixed xor tree combines the L partial sums.
template <int L>
__global__ __launch_bounds__(256) void k_residual_csr(int m, const int32_t* __restrict__ rowptr,
                                                      const int32_t* __restrict__ colidx,
                                                      const double* __restrict__ valr,
                                                      const double* __restrict__ x,
                                                      const double* __restrict__ b,
                                                      double* __restrict__ r) {
  const int sub = threadIdx.x & (L - 1);
  const int i = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / L);
  double s = 0.0;
  if (i < m) {
    const int e1 = rowptr[i + 1];
    for (int e = rowptr[i] + sub; e < e1; e += L) s = fma(valr[e], x[colidx[e]], s);
  }
#pragma unroll
  for (int d = L / 2; d >= 1; d >>= 1) s += __shfl_xor(s, d, L);
  if (i < m && sub == 0) r[i] = s - b[i];
}

// 16 lanes per column: each lane takes a fixed stride of the column's entries, then a
// fixed xor tree combines the 16 partial sums.  With gfree, the same product on the free
// columns (the normal-equations residual A_F^T r used by refinement) goes to gfree.
__global__ __launch_bounds__(256) void k_dual_csc(int n, const int32_t* __restrict__ colptr,
                                                  const int32_t* __restrict__ rowidx,
                                                  const double* __restrict__ val,
                                                  const double* __restrict__ r,
                                                  const uint8_t* __restrict__ flags,
                                                  double* __restrict__ y,
                                                  double* __restrict__ gfree) {
  const int sub = threadIdx.x & 15;
  const int j = (blockIdx.x * blockDim.x + threadIdx.x) >> 4;
  const bool active = j < n;
  double s = 0.0;
  const bool free_j = active ? (flags[j] != 0) : true;
  if (active && (!free_j || gfree)) {
    const int e1 = colptr[j + 1];
    for (int e = colptr[j] + sub; e < e1; e += 16) s = fma(val[e], r[rowidx[e]], s);
  }
  for (int d = 8; d >= 1; d >>= 1) s += __shfl_xor(s, d, 16);
  if (active && sub == 0) {
    y[j] = free_j ? 0.0 : s;
    if (gfree && free_j) gfree[j] = s;
  }
}

// ---------------------------------------------------------------- compensated (refinement)
// The refinement's residual and its products with A^T are summed with error-free
// transformations (Knuth's TwoSum, the FMA-based TwoProduct), so each is exact up to one
// final rounding plus a term of order (k u)^2: the refinement then converges to the
// normal-equations solution itself instead of stalling at the rounding error of an
// ordinary float64 residual (about kappa(A_F^T A_F) u).
// Contraction is off in these functions: a product fused with a following sum into one
// FMA would break the exactness of the transformations.
__device__ inline void two_sum(double a, double b, double* s, double* e) {
#pragma clang fp contract(off)
  const double t = a + b;
  const double bb = t - a;
  *e = (a - (t - bb)) + (b - bb);
  *s = t;
}
// (s, c) += a * v with the product's and the sum's rounding errors kept in c
__device__ inline void dd_acc(double a, double v, double* s, double* c) {
#pragma clang fp contract(off)
  const double p = a * v;
  const double pe = fma(a, v, -p);
  double t, e;
  two_sum(*s, p, &t, &e);
  *s = t;
  *c += e + pe;
}
__device__ inline void dd_add(double* s, double* c, double s2, double c2) {
#pragma clang fp contract(off)
  double t, e;
  two_sum(*s, s2, &t, &e);
  *s = t;
  *c += c2 + e;
}

// r = A x - b as an unevaluated pair r_hi + r_lo (CSR copy, L lanes per row).
template <int L>
__global__ __launch_bounds__(256) void k_residual_csr_dd(int m, const int32_t* __restrict__ rowptr,
                                                         const int32_t* __restrict__ colidx,
                                                         const double* __restrict__ valr,
                                                         const double* __restrict__ x,
                                                         const double* __restrict__ b,
                                                         double* __restrict__ rh, double* __restrict__ rl) {
  const int sub = threadIdx.x & (L - 1);
  const int i = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / L);
  double s = 0.0, c = 0.0;
  if (i < m) {
    const int e1 = rowptr[i + 1];
    for (int e = rowptr[i] + sub; e < e1; e += L) dd_acc(valr[e], x[colidx[e]], &s, &c);
  }
#pragma unroll
  for (int d = L / 2; d >= 1; d >>= 1) {
    const double s2 = __shfl_xor(s, d, L), c2 = __shfl_xor(c, d, L);
    dd_add(&s, &c, s2, c2);
  }
  if (i < m && sub == 0) {
    dd_add(&s, &c, -b[i], 0.0);
    const double hi = s + c;
    rh[i] = hi;
    rl[i] = c - (hi - s);
  }
}

// y_j = a_j^T (r_hi + r_lo) on G, gfree_j on F (16 lanes per column).
__global__ __launch_bounds__(256) void k_dual_csc_dd(int n, const int32_t* __restrict__ colptr,
                                                     const int32_t* __restrict__ rowidx,
                                                     const double* __restrict__ val,
                                                     const double* __restrict__ rh,
                                                     const double* __restrict__ rl,
                                                     const uint8_t* __restrict__ flags,
                                                     double* __restrict__ y, double* __restrict__ gfree) {
  const int sub = threadIdx.x & 15;
  const int j = (blockIdx.x * blockDim.x + threadIdx.x) >> 4;
  const bool active = j < n;
  double s = 0.0, c = 0.0;
  if (active) {
    const int e1 = colptr[j + 1];
    for (int e = colptr[j] + sub; e < e1; e += 16) {
      const int r = rowidx[e];
      const double a = val[e];
      dd_acc(a, rh[r], &s, &c);
      c = fma(a, rl[r], c);
    }
  }
  for (int d = 8; d >= 1; d >>= 1) {
    const double s2 = __shfl_xor(s, d, 16), c2 = __shfl_xor(c, d, 16);
    dd_add(&s, &c, s2, c2);
  }
  if (active && sub == 0) {
    const bool free_j = flags[j] != 0;
    const double v = s + c;
    y[j] = free_j ? 0.0 : v;
    if (free_j) gfree[j] = v;
  }
}

// Dense r = A x - b as r_hi + r_lo: one thread per row, ascending columns.
__global__ __launch_bounds__(256) void k_residual_dense_dd(int m, int n, const double* __restrict__ A, int lda,
                                                           const double* __restrict__ x,
                                                           const double* __restrict__ b,
                                                           double* __restrict__ rh, double* __restrict__ rl) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  double s = 0.0, c = 0.0;
  for (int j = 0; j < n; ++j) {
    const double xj = x[j];
    if (xj != 0.0) dd_acc(A[i + (int64_t)j * lda], xj, &s, &c);
  }
  dd_add(&s, &c, -b[i], 0.0);
  const double hi = s + c;
  rh[i] = hi;
  rl[i] = c - (hi - s);
}

// Dense y_j = a_j^T (r_hi + r_lo) on G, gfree_j on F: one wave per column.
__global__ __launch_bounds__(256) void k_dual_dense_dd(int m, int n, const double* __restrict__ A, int lda,
                                                       const double* __restrict__ rh,
                                                       const double* __restrict__ rl,
                                                       const uint8_t* __restrict__ flags,
                                                       double* __restrict__ y, double* __restrict__ gfree) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= n) return;
  const double* col = A + (int64_t)j * lda;
  double s = 0.0, c = 0.0;
  for (int q = lane; q < m; q += 64) {
    const double a = col[q];
    dd_acc(a, rh[q], &s, &c);
    c = fma(a, rl[q], c);
  }
  for (int d = 32; d >= 1; d >>= 1) {
    const double s2 = __shfl_xor(s, d, 64), c2 = __shfl_xor(c, d, 64);
    dd_add(&s, &c, s2, c2);
  }
  if (lane == 0) {
    const bool free_j = flags[j] != 0;
    const double v = s + c;
    y[j] = free_j ? 0.0 : v;
    if (free_j) gfree[j] = v;
  }
}

// Maximum that keeps a NaN operand (fmax drops it).
__device__ inline double max_nan(double a, double b) { return (a > b || a != a) ? a : b; }

// x[Flist[p]] -= d[p]; max |d| and max |x_F| by one workgroup (fixed reduction order).
// A NaN correction or iterate makes the reported maximum NaN, so the host sees it.
__global__ __launch_bounds__(1024) void k_ir_update(int nF, const int32_t* __restrict__ Flist,
                                                    const double* __restrict__ d,
                                                    double* __restrict__ x, Ctrl* ctrl, int first) {
  __shared__ double s_d[16], s_x[16];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  double dm = 0.0, xm = 0.0;
  for (int p = tid; p < nF; p += 1024) {
    const int i = Flist[p];
    const double v = x[i] - d[p];
    x[i] = v;
    dm = max_nan(dm, fabs(d[p]));
    xm = max_nan(xm, fabs(v));
  }
  for (int o = 32; o >= 1; o >>= 1) {
    dm = max_nan(dm, __shfl_xor(dm, o, 64));
    xm = max_nan(xm, __shfl_xor(xm, o, 64));
  }
  if (lane == 0) {
    s_d[w] = dm;
    s_x[w] = xm;
  }
  __syncthreads();
  if (tid == 0) {
    double a = 0.0, b = 0.0;
    for (int q = 0; q < 16; ++q) {
      a = max_nan(a, s_d[q]);
      b = max_nan(b, s_x[q]);
    }
    ctrl->ir_dprev = first ? INFINITY : ctrl->ir_dmax;
    ctrl->ir_dmax = a;
    ctrl->ir_xmax = b;
  }
}

// w_r = sum over the free columns j of row r of |a_rj| (CSR copy, L lanes per row as in
// the residual).
template <int L>
__global__ __launch_bounds__(256) void k_abs_rowsum_csr(int m, const int32_t* __restrict__ rowptr,
                                                        const int32_t* __restrict__ colidx,
                                                        const double* __restrict__ valr,
                                                        const uint8_t* __restrict__ flags,
                                                        double* __restrict__ w) {
  const int sub = threadIdx.x & (L - 1);
  const int i = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / L);
  double s = 0.0;
  if (i < m) {
    const int e1 = rowptr[i + 1];
    for (int e = rowptr[i] + sub; e < e1; e += L)
      if (flags[colidx[e]]) s += fabs(valr[e]);
  }
#pragma unroll
  for (int d = L / 2; d >= 1; d >>= 1) s += __shfl_xor(s, d, L);
  if (i < m && sub == 0) w[i] = s;
}

// bw_j = sum_r |a_rj| w_r and bb_j = sum_r |a_rj| |b_r| for j in G (0 on F); 16 lanes per
// column as in the dual.
__global__ __launch_bounds__(256) void k_abs_dual_csc(int n, const int32_t* __restrict__ colptr,
                                                      const int32_t* __restrict__ rowidx,
                                                      const double* __restrict__ val,
                                                      const double* __restrict__ w,
                                                      const double* __restrict__ b,
                                                      const uint8_t* __restrict__ flags,
                                                      double* __restrict__ bw, double* __restrict__ bb) {
  const int sub = threadIdx.x & 15;
  const int j = (blockIdx.x * blockDim.x + threadIdx.x) >> 4;
  const bool active = j < n;
  const bool want = active && flags[j] == 0;
  double sw = 0.0, sb = 0.0;
  if (want) {
    const int e1 = colptr[j + 1];
    for (int e = colptr[j] + sub; e < e1; e += 16) {
      const double a = fabs(val[e]);
      const int r = rowidx[e];
      sw = fma(a, w[r], sw);
      sb = fma(a, fabs(b[r]), sb);
    }
  }
  for (int d = 8; d >= 1; d >>= 1) {
    sw += __shfl_xor(sw, d, 16);
    sb += __shfl_xor(sb, d, 16);
  }
  if (active && sub == 0) {
    bw[j] = sw;
    bb[j] = sb;
  }
}

// Dense w_r = sum_{p < nF} |A(r, F_p)|: one thread per row.
__global__ __launch_bounds__(256) void k_abs_rowsum_dense(int m, const double* __restrict__ A, int lda,
                                                          const int32_t* __restrict__ Flist, int nF,
                                                          double* __restrict__ w) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  double s = 0.0;
  for (int p = 0; p < nF; ++p) s += fabs(A[i + (int64_t)Flist[p] * lda]);
  w[i] = s;
}

// Dense bw_j, bb_j for j in G (0 on F): one wave per column.
__global__ __launch_bounds__(256) void k_abs_dual_dense(int m, int n, const double* __restrict__ A, int lda,
                                                        const double* __restrict__ w,
                                                        const double* __restrict__ b,
                                                        const uint8_t* __restrict__ flags,
                                                        double* __restrict__ bw, double* __restrict__ bb) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= n) return;
  double sw = 0.0, sb = 0.0;
  if (!flags[j]) {
    const double* col = A + (int64_t)j * lda;
    for (int q = lane; q < m; q += 64) {
      const double a = fabs(col[q]);
      sw = fma(a, w[q], sw);
      sb = fma(a, fabs(b[q]), sb);
    }
  }
  for (int d = 32; d >= 1; d >>= 1) {
    sw += __shfl_xor(sw, d, 64);
    sb += __shfl_xor(sb, d, 64);
  }
  if (lane == 0) {
    bw[j] = sw;
    bb[j] = sb;
  }
}

// Sign certificates after a refinement step (one workgroup).  While the refinement
// contracts by 1/2 or better per step (rho = dmax / dprev, measured on consecutive
// corrections), the error left in x_F after a step is at most its correction, e_x = dmax,
// and that of the iterate the step's y_G came from at most e_y = 2 dmax (its distance to
// the corrected x plus e_x).  A tested entry v with |v| >= tau is certified when |v| minus
// its bound still exceeds tau:
//   on F (v = x_i after the step):  e_x plus the rounding of the update, 4 u |v|;
//   on G (v = y_i):  e_y bw_i (the error of x_F carried through |a_i|^T |A_F|) plus the
//                    rounding of the compensated y_i: 2 u |v| + gamma2 (xmax' bw_i + bb_i),
//                    gamma2 = 2 gamma_k^2, xmax' = xmax + dmax the largest entry of that
//                    iterate.
__global__ __launch_bounds__(1024) void k_ir_certify(int n, const uint8_t* __restrict__ flags,
                                                     const double* __restrict__ x,
                                                     const double* __restrict__ y,
                                                     const double* __restrict__ bw,
                                                     const double* __restrict__ bb, double tau,
                                                     double gamma2, Ctrl* ctrl) {
  __shared__ int s_cnt[16];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const double dmax = ctrl->ir_dmax, dprev = ctrl->ir_dprev, xmax = ctrl->ir_xmax;
  const double rho = dmax / dprev;
  const bool known = dprev < INFINITY && rho <= 0.5 && dmax < INFINITY && xmax < INFINITY;
  if (!known) {
    if (tid == 0) {
      ctrl->ir_err = INFINITY;
      ctrl->ir_uncert = -1;
    }
    return;
  }
  const double ex = dmax;
  const double ey = 2.0 * dmax;
  const double xm = xmax + dmax;
  int cnt = 0;
  for (int i = tid; i < n; i += 1024) {
    const bool f = flags[i] != 0;
    const double a = fabs(f ? x[i] : y[i]);
    if (!(a >= tau)) continue;   // zeroed by the next classify step
    const double e = f ? ex + 4.0 * 1.1102230246251565e-16 * a
                       : ey * bw[i] + 2.0 * 1.1102230246251565e-16 * a + gamma2 * (xm * bw[i] + bb[i]);
    if (!(a - e > tau)) ++cnt;
  }
  for (int o = 32; o >= 1; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
  if (lane == 0) s_cnt[w] = cnt;
  __syncthreads();
  if (tid == 0) {
    int t = 0;
    for (int q = 0; q < 16; ++q) t += s_cnt[q];
    ctrl->ir_err = ex;
    ctrl->ir_uncert = t;
  }
}

// Dense r = A x - b: one thread per row, ascending column order.
// Dense r = A x - b, one thread per row (column-major A: a wave reads 512 contiguous bytes
// per column).  With `part`, column chunk blockIdx.y of width `chunk` writes its partial
// sums to part[blockIdx.y * m + i] instead, so that tall-and-narrow grids still fill the
// device; k_residual_dense_combine then adds the chunks in order.
__global__ __launch_bounds__(256) void k_residual_dense(int m, int n, const double* __restrict__ A,
                                                        int lda, const double* __restrict__ x,
                                                        const double* __restrict__ b,
                                                        double* __restrict__ r, int chunk,
                                                        double* __restrict__ part) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int j0 = part ? blockIdx.y * chunk : 0;
  const int j1 = part ? min(n, j0 + chunk) : n;
  double s = 0.0;
  for (int j = j0; j < j1; ++j) s = fma(A[i + (int64_t)j * lda], x[j], s);
  if (part)
    part[(int64_t)blockIdx.y * m + i] = s;
  else
    r[i] = s - b[i];
}

__global__ __launch_bounds__(256) void k_residual_dense_combine(int m, int nchunk, const double* __restrict__ part,
                                                                const double* __restrict__ b,
                                                                double* __restrict__ r) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  double s = 0.0;
  for (int c = 0; c < nchunk; ++c) s += part[(int64_t)c * m + i];
  r[i] = s - b[i];
}

// Dense y_j = a_j^T r on G (and on F into gfree when given): one wave per column.
__global__ __launch_bounds__(256) void k_dual_dense(int m, int n, const double* __restrict__ A, int lda,
                                                    const double* __restrict__ r,
                                                    const uint8_t* __restrict__ flags,
                                                    double* __restrict__ y,
                                                    double* __restrict__ gfree) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= n) return;
  const bool free_j = flags[j] != 0;
  if (free_j && !gfree) {
    if (lane == 0) y[j] = 0.0;
    return;
  }
  const double* col = A + (int64_t)j * lda;
  double s = 0.0;
  for (int q = lane; q < m; q += 64) s = fma(col[q], r[q], s);
  for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
  if (lane == 0) {
    y[j] = free_j ? 0.0 : s;
    if (free_j) gfree[j] = s;
  }
}

// Eq. 3 on G: y_j = sum_p H[F_p, j] x[F_p] - c_j for j in G (H symmetric, so column j),
// y_j = 0 on F.  One wave per column, lane-strided over the F positions, fixed xor tree.
__global__ __launch_bounds__(256) void k_dual_gram_dense(int n, const double* __restrict__ H, int64_t ldh,
                                                         const double* __restrict__ c,
                                                         const uint8_t* __restrict__ flags,
                                                         const int32_t* __restrict__ Flist, int nF,
                                                         const double* __restrict__ x, double* __restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= n) return;
  if (flags[j]) {
    if (lane == 0) y[j] = 0.0;
    return;
  }
  const double* col = H + (int64_t)j * ldh;
  double s = 0.0;
  for (int p = lane; p < nF; p += 64) {
    const int i = Flist[p];
    s = fma(col[i], x[i], s);
  }
  for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
  if (lane == 0) y[j] = s - c[j];
}

}  // namespace

void launch_residual_csr(hipStream_t s, int m, int64_t nnz, const int32_t* rowptr, const int32_t* colidx,
                         const double* valr, const double* x, const double* b, double* r) {
  // lanes per row: the average row length rounded up to a power of two, at most 16
  const double avg = m > 0 ? (double)nnz / m : 0.0;
  const int L = avg > 8 ? 16 : avg > 4 ? 8 : avg > 2 ? 4 : avg > 1 ? 2 : 1;
  const unsigned grid = (unsigned)(((int64_t)m * L + 255) / 256);
  switch (L) {
    case 16: hipLaunchKernelGGL(k_residual_csr<16>, dim3(grid), dim3(256), 0, s, m, rowptr, colidx, valr, x, b, r); break;
    case 8: hipLaunchKernelGGL(k_residual_csr<8>, dim3(grid), dim3(256), 0, s, m, rowptr, colidx, valr, x, b, r); break;
    case 4: hipLaunchKernelGGL(k_residual_csr<4>, dim3(grid), dim3(256), 0, s, m, rowptr, colidx, valr, x, b, r); break;
    case 2: hipLaunchKernelGGL(k_residual_csr<2>, dim3(grid), dim3(256), 0, s, m, rowptr, colidx, valr, x, b, r); break;
    default: hipLaunchKernelGGL(k_residual_csr<1>, dim3(grid), dim3(256), 0, s, m, rowptr, colidx, valr, x, b, r); break;
  }
}

void launch_residual_dual_dd(hipStream_t s, int m, int n, int64_t nnz, const int32_t* rowptr,
                             const int32_t* colidx, const double* valr, const int32_t* colptr,
                             const int32_t* rowidx, const double* val, const double* A, int lda,
                             const double* x, const double* b, const uint8_t* flags, double* rh,
                             double* rl, double* y, double* gfree) {
  if (A) {
    hipLaunchKernelGGL(k_residual_dense_dd, dim3((m + 255) / 256), dim3(256), 0, s, m, n, A, lda, x, b, rh, rl);
    hipLaunchKernelGGL(k_dual_dense_dd, dim3((n + 3) / 4), dim3(256), 0, s, m, n, A, lda, (const double*)rh,
                       (const double*)rl, flags, y, gfree);
    return;
  }
  const double avg = m > 0 ? (double)nnz / m : 0.0;
  const int L = avg > 8 ? 16 : avg > 4 ? 8 : avg > 2 ? 4 : avg > 1 ? 2 : 1;
  const unsigned grid = (unsigned)(((int64_t)m * L + 255) / 256);
  switch (L) {
    case 16: hipLaunchKernelGGL(k_residual_csr_dd<16>, dim3(grid), dim3(256), 0, s, m, rowptr, colidx, valr, x, b, rh, rl); break;
    case 8: hipLaunchKernelGGL(k_residual_csr_dd<8>, dim3(grid), dim3(256), 0, s, m, rowptr, colidx, valr, x, b, rh, rl); break;
    case 4: hipLaunchKernelGGL(k_residual_csr_dd<4>, dim3(grid), dim3(256), 0, s, m, rowptr, colidx, valr, x, b, rh, rl); break;
    case 2: hipLaunchKernelGGL(k_residual_csr_dd<2>, dim3(grid), dim3(256), 0, s, m, rowptr, colidx, valr, x, b, rh, rl); break;
    default: hipLaunchKernelGGL(k_residual_csr_dd<1>, dim3(grid), dim3(256), 0, s, m, rowptr, colidx, valr, x, b, rh, rl); break;
  }
  const int64_t threads = (int64_t)n * 16;
  hipLaunchKernelGGL(k_dual_csc_dd, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, n, colptr, rowidx,
                     val, (const double*)rh, (const double*)rl, flags, y, gfree);
}

void launch_dual_csc(hipStream_t s, int n, const int32_t* colptr, const int32_t* rowidx,
                     const double* val, const double* r, const uint8_t* flags, double* y,
                     double* gfree) {
  const int64_t threads = (int64_t)n * 16;
  hipLaunchKernelGGL(k_dual_csc, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, n, colptr,
                     rowidx, val, r, flags, y, gfree);
}

void launch_ir_update(hipStream_t s, int nF, const int32_t* Flist, const double* d, double* x,
                      Ctrl* ctrl, int first) {
  hipLaunchKernelGGL(k_ir_update, dim3(1), dim3(1024), 0, s, nF, Flist, d, x, ctrl, first);
}

void launch_sign_bounds_csr(hipStream_t s, int m, int n, int64_t nnz, const int32_t* rowptr,
                            const int32_t* colidx, const double* valr, const int32_t* colptr,
                            const int32_t* rowidx, const double* val, const uint8_t* flags,
                            const double* b, double* w, double* bw, double* bb) {
  const double avg = m > 0 ? (double)nnz / m : 0.0;
  const int L = avg > 8 ? 16 : avg > 4 ? 8 : avg > 2 ? 4 : avg > 1 ? 2 : 1;
  const unsigned grid = (unsigned)(((int64_t)m * L + 255) / 256);
  switch (L) {
    case 16: hipLaunchKernelGGL(k_abs_rowsum_csr<16>, dim3(grid), dim3(256), 0, s, m, rowptr, colidx, valr, flags, w); break;
    case 8: hipLaunchKernelGGL(k_abs_rowsum_csr<8>, dim3(grid), dim3(256), 0, s, m, rowptr, colidx, valr, flags, w); break;
    case 4: hipLaunchKernelGGL(k_abs_rowsum_csr<4>, dim3(grid), dim3(256), 0, s, m, rowptr, colidx, valr, flags, w); break;
    case 2: hipLaunchKernelGGL(k_abs_rowsum_csr<2>, dim3(grid), dim3(256), 0, s, m, rowptr, colidx, valr, flags, w); break;
    default: hipLaunchKernelGGL(k_abs_rowsum_csr<1>, dim3(grid), dim3(256), 0, s, m, rowptr, colidx, valr, flags, w); break;
  }
  const int64_t threads = (int64_t)n * 16;
  hipLaunchKernelGGL(k_abs_dual_csc, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, n, colptr, rowidx,
                     val, (const double*)w, b, flags, bw, bb);
}

void launch_sign_bounds_dense(hipStream_t s, int m, int n, const double* A, int lda,
                              const int32_t* Flist, int nF, const uint8_t* flags, const double* b,
                              double* w, double* bw, double* bb) {
  hipLaunchKernelGGL(k_abs_rowsum_dense, dim3((m + 255) / 256), dim3(256), 0, s, m, A, lda, Flist, nF, w);
  hipLaunchKernelGGL(k_abs_dual_dense, dim3((n + 3) / 4), dim3(256), 0, s, m, n, A, lda, (const double*)w, b,
                     flags, bw, bb);
}

void launch_ir_certify(hipStream_t s, int n, const uint8_t* flags, const double* x, const double* y,
                       const double* bw, const double* bb, double tau, double gamma2, Ctrl* ctrl) {
  hipLaunchKernelGGL(k_ir_certify, dim3(1), dim3(1024), 0, s, n, flags, x, y, bw, bb, tau, gamma2, ctrl);
}

void launch_residual_dense(hipStream_t s, int m, int n, const double* A, int lda,
                           const double* x, const double* b, double* r, double* part) {
  const int rows = (m + 255) / 256;
  const int nchunk = dense_residual_chunks(m, n);
  if (nchunk <= 1 || !part) {
    hipLaunchKernelGGL(k_residual_dense, dim3(rows), dim3(256), 0, s, m, n, A, lda, x, b, r, n, (double*)nullptr);
    return;
  }
  const int chunk = (n + nchunk - 1) / nchunk;
  hipLaunchKernelGGL(k_residual_dense, dim3(rows, nchunk), dim3(256), 0, s, m, n, A, lda, x, b, r, chunk, part);
  hipLaunchKernelGGL(k_residual_dense_combine, dim3(rows), dim3(256), 0, s, m, nchunk, (const double*)part, b, r);
}

int dense_residual_chunks(int m, int n) {
  // enough workgroups for the device (about 1024), chunks of at least 64 columns
  const int rows = (m + 255) / 256;
  int c = (1024 + rows - 1) / rows;
  const int cmax = (n + 63) / 64;
  if (c > cmax) c = cmax;
  return c < 1 ? 1 : c;
}

void launch_dual_dense(hipStream_t s, int m, int n, const double* A, int lda, const double* r,
                       const uint8_t* flags, double* y, double* gfree) {
  hipLaunchKernelGGL(k_dual_dense, dim3((n + 3) / 4), dim3(256), 0, s, m, n, A, lda, r, flags, y, gfree);
}

void launch_dual_gram_dense(hipStream_t s, int n, const double* H, int64_t ldh, const double* c,
                            const uint8_t* flags, const int32_t* Flist, int nF, const double* x,
                            double* y) {
  hipLaunchKernelGGL(k_dual_gram_dense, dim3((n + 3) / 4), dim3(256), 0, s, n, H, ldh, c, flags, Flist, nF,
                     x, y);
}

}  // namespace nnls
