// Setup kernels, run once per problem: input validation, a row-major (CSR) copy of A,
// the cached Gram matrix H = A^T A from column dot products (Sec. 3 of the tsnnls paper)
// and the right-hand side c = A^T b of the normal equations (Sec. 2.1).
//
// H is kept as its lower triangle in a padded CSC layout: column j holds the rows i >= j
// with a structurally nonzero a_i^T a_j, ascending.  For the pivot loop each column's
// region is then completed with its rows i < j (copied from the lower triangle, unordered),
// and for every new F order the F-block is re-indexed into F-position space, each
// position keeping the entries at or below the diagonal in position order: the factor
// gathers its tiles from that.
#include "tile_ops.h"

namespace nnls {

namespace {

__global__ void k_validate_csc(int m, int n, int64_t nnz, const int32_t* __restrict__ colptr,
                               const int32_t* __restrict__ rowidx, const double* __restrict__ val,
                               const double* __restrict__ b, int32_t* err) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride) {
    const int64_t c0 = colptr[j], c1 = colptr[j + 1];
    if (j == 0 && c0 != 0) atomicOr(&err[0], 1);
    if (j == n - 1 && c1 != nnz) atomicOr(&err[0], 1);
    if (c0 < 0 || c1 < c0 || c1 > nnz) {
      atomicOr(&err[0], 1);
      continue;
    }
    int prev = -1;
    for (int64_t e = c0; e < c1; ++e) {
      const int r = rowidx[e];
      if (r <= prev || r >= m) {
        atomicOr(&err[0], 2);
        break;
      }
      prev = r;
      if (!isfinite(val[e])) atomicOr(&err[1], 1);
    }
  }
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride)
    if (!isfinite(b[i])) atomicOr(&err[1], 2);
}

__global__ void k_validate_dense(int m, int n, const double* __restrict__ A, int lda,
                                 const double* __restrict__ b, int32_t* err) {
  const int64_t total = (int64_t)m * n;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int64_t j = e / m, i = e - j * m;
    if (!isfinite(A[i + j * lda])) atomicOr(&err[1], 1);
  }
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride)
    if (!isfinite(b[i])) atomicOr(&err[1], 2);
}

__global__ void k_fill_f64(double* p, int64_t count, double v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = v;
}

__global__ void k_fill_i32(int32_t* p, int64_t count, int32_t v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = v;
}

__global__ void k_fill_2d(int rows, int cols, double* p, int ld, double v) {
  const int64_t total = (int64_t)rows * cols;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int64_t c = e / rows, r = e - c * rows;
    p[r + c * ld] = v;
  }
}

__global__ void k_row_count(int64_t nnz, const int32_t* __restrict__ rowidx, int32_t* rowcnt) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += stride)
    atomicAdd(&rowcnt[rowidx[e]], 1);
}

// Exclusive scan of count[0..n) into out[0..n], out[n] = total, in three launches over
// chunks of SCAN_CHUNK entries: the chunk sums; one workgroup scans those into chunk
// offsets; each chunk then stages its entries in LDS with coalesced loads, scans them
// (SCAN_PER consecutive entries per thread, then the thread totals across the workgroup)
// and stores the result coalesced.  A chunk is read whole before any of it is written and
// the sums are taken before any chunk is written, so count may alias out.
constexpr int SCAN_PER = 8;
constexpr int SCAN_CHUNK = 256 * SCAN_PER;

template <typename T>
__device__ inline T block_excl_scan256(T v, T* s_wave, T* total) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  T t = v;
  for (int d = 1; d < 64; d <<= 1) {
    const T o = __shfl_up(t, d, 64);
    if (lane >= d) t += o;
  }
  if (lane == 63) s_wave[w] = t;
  __syncthreads();
  const T before = (w > 0 ? s_wave[0] : 0) + (w > 1 ? s_wave[1] : 0) + (w > 2 ? s_wave[2] : 0);
  *total = s_wave[0] + s_wave[1] + s_wave[2] + s_wave[3];
  __syncthreads();
  return before + t - v;
}

template <typename Tin, typename Tout>
__global__ __launch_bounds__(256) void k_scan_sums(int64_t n, const Tin* count, Tout* sums) {
  __shared__ Tout s_wave[4];
  const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK;
  Tout v = 0;
#pragma unroll
  for (int q = 0; q < SCAN_PER; ++q) {
    const int64_t i = base + threadIdx.x + 256 * q;
    if (i < n) v += (Tout)count[i];
  }
  Tout total;
  block_excl_scan256<Tout>(v, s_wave, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// Exclusive scan of sums[0..nchunk) in place, one workgroup; *grand = the total.
template <typename Tout>
__global__ __launch_bounds__(256) void k_scan_top(int nchunk, Tout* sums, Tout* grand) {
  __shared__ Tout s_wave[4];
  Tout carry = 0;
  for (int c0 = 0; c0 < nchunk; c0 += 256) {
    const int c = c0 + threadIdx.x;
    const Tout v = (c < nchunk) ? sums[c] : (Tout)0;
    Tout total;
    const Tout ex = block_excl_scan256<Tout>(v, s_wave, &total);
    if (c < nchunk) sums[c] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) *grand = carry;
}

template <typename Tin, typename Tout>
__global__ __launch_bounds__(256) void k_scan_apply(int64_t n, const Tin* count, const Tout* offs, Tout* out) {
  __shared__ Tout s_val[SCAN_CHUNK];
  __shared__ Tout s_wave[4];
  const int tid = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK;
#pragma unroll
  for (int q = 0; q < SCAN_PER; ++q) {
    const int64_t i = base + tid + 256 * q;
    s_val[tid + 256 * q] = (i < n) ? (Tout)count[i] : (Tout)0;
  }
  __syncthreads();
  Tout v[SCAN_PER], local = 0;
#pragma unroll
  for (int q = 0; q < SCAN_PER; ++q) {
    v[q] = s_val[tid * SCAN_PER + q];
    local += v[q];
  }
  Tout total;
  Tout off = offs[blockIdx.x] + block_excl_scan256<Tout>(local, s_wave, &total);
#pragma unroll
  for (int q = 0; q < SCAN_PER; ++q) {
    s_val[tid * SCAN_PER + q] = off;
    off += v[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < SCAN_PER; ++q) {
    const int64_t i = base + tid + 256 * q;
    if (i < n) out[i] = s_val[tid + 256 * q];
  }
}

__global__ void k_csr_fill(int n, const int32_t* __restrict__ colptr, const int32_t* __restrict__ rowidx,
                           const double* __restrict__ val, const int32_t* __restrict__ rowptr,
                           int32_t* fill, int32_t* colidx, double* valr) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  for (int e = colptr[j]; e < colptr[j + 1]; ++e) {
    const int r = rowidx[e];
    const int slot = rowptr[r] + atomicAdd(&fill[r], 1);
    colidx[slot] = j;
    valr[slot] = val[e];
  }
}

// Sort each CSR row by column so that every later row sum has a fixed order.
__global__ void k_csr_sort(int m, const int32_t* __restrict__ rowptr, int32_t* colidx, double* valr) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= m) return;
  const int s = rowptr[r], e = rowptr[r + 1];
  for (int i = s + 1; i < e; ++i) {
    const int c = colidx[i];
    const double v = valr[i];
    int k = i - 1;
    while (k >= s && colidx[k] > c) {
      colidx[k + 1] = colidx[k];
      valr[k + 1] = valr[k];
      --k;
    }
    colidx[k + 1] = c;
    valr[k + 1] = v;
  }
}

// Upper bound of the entries of column j of lower(H): sum of the lengths of the rows
// that column j touches.
__global__ void k_gram_bound(int n, const int32_t* __restrict__ colptr, const int32_t* __restrict__ rowidx,
                             const int32_t* __restrict__ rowptr, int64_t* ub) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  int64_t s = 0;
  for (int e = colptr[j]; e < colptr[j + 1]; ++e) {
    const int r = rowidx[e];
    s += rowptr[r + 1] - rowptr[r];
  }
  ub[j] = s;
}

// H_ij = a_i^T a_j for i >= j.  One wave per column j, over windows of GRAM_WIN rows
// [base, base + GRAM_WIN) (one window unless n > GRAM_WIN).  Pass 1 marks in an LDS bitmap
// the rows i of the window that column j meets; a scan of the bitmap's popcounts gives each
// marked row its slot, in ascending i, which is also the output order.  Pass 2 sums
// a_rj a_ri into the slots (GRAM_SLOTS at a time).  The column's entries are fetched four
// at a time, one group of 16 lanes each, but applied one entry after the other in
// ascending r, and inside row r each i appears once: every H_ij is summed in ascending r,
// a fixed order independent of the launch.
constexpr int GRAM_WIN = 32768;
constexpr int GRAM_WORDS = GRAM_WIN / 32;
constexpr int GRAM_SLOTS = 1024;

__device__ inline int wave_excl_scan(int v, int lane, int* total) {
  int x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  *total = __shfl(x, 63, 64);
  return x - v;
}

__global__ __launch_bounds__(256) void k_gram_lower(
    int n, const int32_t* __restrict__ colptr, const int32_t* __restrict__ rowidx,
    const double* __restrict__ val, const int32_t* __restrict__ rowptr,
    const int32_t* __restrict__ colidx, const double* __restrict__ valr,
    const int64_t* __restrict__ hptr, int32_t* __restrict__ hcnt, int32_t* __restrict__ hrow,
    double* __restrict__ hval) {
  __shared__ uint32_t s_bits[4][GRAM_WORDS];
  __shared__ int32_t s_rank[4][GRAM_WORDS];
  __shared__ double s_acc[4][GRAM_SLOTS];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int j = blockIdx.x * 4 + w;
  if (j >= n) return;   // whole wave leaves; no workgroup barrier follows
  uint32_t* bits = s_bits[w];
  int32_t* rank = s_rank[w];
  double* acc = s_acc[w];
  const int grp = lane >> 4, gl = lane & 15;
  const int cs = colptr[j], ce = colptr[j + 1];
  const int64_t out = hptr[j];
  int count = 0;
  for (int base = j; base < n; base += GRAM_WIN) {
    const int span = min(GRAM_WIN, n - base);
    const int nwords = (span + 31) >> 5;
    for (int q = lane; q < nwords; q += 64) bits[q] = 0u;
    __builtin_amdgcn_wave_barrier();
    // pass 1: mark the rows met
    for (int e0 = cs; e0 < ce; e0 += 4) {
      const int e = e0 + grp;
      if (e < ce) {
        const int r = rowidx[e];
        const int rs = rowptr[r], re = rowptr[r + 1];
        for (int t = rs + gl; t < re; t += 16) {
          const int q = colidx[t] - base;
          if (q >= 0 && q < span) atomicOr(&bits[q >> 5], 1u << (q & 31));
        }
      }
    }
    __builtin_amdgcn_wave_barrier();
    // slots: exclusive prefix of the words' popcounts
    int total = 0;
    for (int q0 = 0; q0 < nwords; q0 += 64) {
      const int q = q0 + lane;
      const int c = (q < nwords) ? __popc(bits[q]) : 0;
      int chunk;
      const int ex = wave_excl_scan(c, lane, &chunk);
      if (q < nwords) rank[q] = total + ex;
      total += chunk;
    }
    __builtin_amdgcn_wave_barrier();
    // pass 2, GRAM_SLOTS slots at a time
    for (int s0 = 0; s0 < total; s0 += GRAM_SLOTS) {
      const int sn = min(GRAM_SLOTS, total - s0);
      for (int q = lane; q < sn; q += 64) acc[q] = 0.0;
      __builtin_amdgcn_wave_barrier();
      for (int e0 = cs; e0 < ce; e0 += 4) {
        const int e = e0 + grp;
        int r = 0, rs = 0, re = 0;
        double a = 0.0;
        if (e < ce) {
          r = rowidx[e];
          a = val[e];
          rs = rowptr[r];
          re = rowptr[r + 1];
        }
        // first 16 entries of each group's row, all in flight together
        int q1 = -1;
        double v1 = 0.0;
        if (rs + gl < re) {
          q1 = colidx[rs + gl] - base;
          v1 = valr[rs + gl];
        }
        // apply the four entries one after the other (ascending r)
        for (int k = 0; k < 4; ++k) {
          if (grp == k) {
            if (q1 >= 0 && q1 < span) {
              const int slot = rank[q1 >> 5] + __popc(bits[q1 >> 5] & ((1u << (q1 & 31)) - 1u)) - s0;
              if (slot >= 0 && slot < sn) acc[slot] = fma(a, v1, acc[slot]);
            }
            // the rest of a row longer than 16 entries
            for (int t = rs + 16 + gl; t < re; t += 16) {
              const int q = colidx[t] - base;
              if (q >= 0 && q < span) {
                const int slot = rank[q >> 5] + __popc(bits[q >> 5] & ((1u << (q & 31)) - 1u)) - s0;
                if (slot >= 0 && slot < sn) acc[slot] = fma(a, valr[t], acc[slot]);
              }
            }
          }
          __builtin_amdgcn_wave_barrier();
        }
      }
      __builtin_amdgcn_wave_barrier();
      // write the slots out: word q holds the rows base + 32 q + b of its set bits b
      for (int q = lane; q < nwords; q += 64) {
        uint32_t m = bits[q];
        int slot = rank[q];
        while (m) {
          const int b = __ffs(m) - 1;
          if (slot >= s0 && slot < s0 + sn) {
            hrow[out + count + slot] = base + 32 * q + b;
            hval[out + count + slot] = acc[slot - s0];
          }
          ++slot;
          m &= m - 1u;
        }
      }
      __builtin_amdgcn_wave_barrier();
    }
    count += total;
  }
  if (lane == 0) hcnt[j] = count;
}

// Column j's strictly lower entries (i > j) become the upper entries of column i, appended
// after its lower ones (slot from a counter per column, so in no particular order).  Every
// column's region holds its whole column: its size bounds the count of distinct rows.
__global__ __launch_bounds__(256) void k_gram_mirror(int n, GramLower g, int32_t* __restrict__ upcnt,
                                                     int32_t* __restrict__ hrow, double* __restrict__ hval) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= n) return;
  const int64_t s = g.hptr[j];
  const int cnt = g.hcnt[j];
  for (int q = lane; q < cnt; q += 64) {
    const int i = hrow[s + q];
    if (i == j) continue;
    const int slot = atomicAdd(&upcnt[i], 1);
    const int64_t o = g.hptr[i] + g.hcnt[i] + slot;
    hrow[o] = j;
    hval[o] = hval[s + q];
  }
}

// F-position lists: position q (column j = Flist[q]) keeps the entries p = pos[i] >= q of
// its whole column, written in ascending p.  One wave per position, over windows of
// GRAM_WIN positions: the entries' positions are marked in an LDS bitmap (each position
// occurs once in a column), a scan of the words' popcounts ranks them, and each entry is
// written at its rank.  The output is sorted by construction and does not depend on the
// launch.
__global__ __launch_bounds__(256) void k_gram_positions(int nF, GramLower g, const int32_t* __restrict__ upcnt,
                                                        const int32_t* __restrict__ Flist,
                                                        const int32_t* __restrict__ pos,
                                                        int32_t* __restrict__ pcnt, int32_t* __restrict__ prow,
                                                        double* __restrict__ pval) {
  __shared__ uint32_t s_bits[4][GRAM_WORDS];
  __shared__ int32_t s_rank[4][GRAM_WORDS];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int q = blockIdx.x * 4 + w;
  if (q >= nF) return;   // whole wave leaves; no workgroup barrier follows
  uint32_t* bits = s_bits[w];
  int32_t* rank = s_rank[w];
  const int j = Flist[q];
  const int64_t s = g.hptr[j];
  const int cnt = g.hcnt[j] + upcnt[j];
  // largest position in the column bounds the windows
  int pmax = q;
  for (int t = lane; t < cnt; t += 64) pmax = max(pmax, pos[g.hrow[s + t]]);
  for (int d = 32; d >= 1; d >>= 1) pmax = max(pmax, __shfl_xor(pmax, d, 64));
  int count = 0;
  for (int base = q; base <= pmax; base += GRAM_WIN) {
    const int span = min(GRAM_WIN, pmax + 1 - base);
    const int nwords = (span + 31) >> 5;
    for (int k = lane; k < nwords; k += 64) bits[k] = 0u;
    __builtin_amdgcn_wave_barrier();
    for (int t = lane; t < cnt; t += 64) {
      const int k = pos[g.hrow[s + t]] - base;
      if (k >= 0 && k < span) atomicOr(&bits[k >> 5], 1u << (k & 31));
    }
    __builtin_amdgcn_wave_barrier();
    int total = 0;
    for (int k0 = 0; k0 < nwords; k0 += 64) {
      const int k = k0 + lane;
      const int c = (k < nwords) ? __popc(bits[k]) : 0;
      int chunk;
      const int ex = wave_excl_scan(c, lane, &chunk);
      if (k < nwords) rank[k] = total + ex;
      total += chunk;
    }
    __builtin_amdgcn_wave_barrier();
    for (int t = lane; t < cnt; t += 64) {
      const int k = pos[g.hrow[s + t]] - base;
      if (k >= 0 && k < span) {
        const int slot = count + rank[k >> 5] + __popc(bits[k >> 5] & ((1u << (k & 31)) - 1u));
        prow[s + slot] = base + k;
        pval[s + slot] = g.hval[s + t];
      }
    }
    __builtin_amdgcn_wave_barrier();
    count += total;
  }
  if (lane == 0) pcnt[q] = count;
}

// out_j = scale * sum_r a_rj v_r  (ascending r), one thread per column.
__global__ void k_spmvT_csc(int n, const int32_t* __restrict__ colptr, const int32_t* __restrict__ rowidx,
                            const double* __restrict__ val, const double* __restrict__ v,
                            double* __restrict__ out, double scale) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double s = 0.0;
  for (int e = colptr[j]; e < colptr[j + 1]; ++e) s = fma(val[e], v[rowidx[e]], s);
  out[j] = scale * s;
}

__global__ void k_lower_to_dense(int n, GramLower g, double* H, int ldh) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int64_t s = g.hptr[j];
  for (int q = 0; q < g.hcnt[j]; ++q) {
    const int i = g.hrow[s + q];
    const double v = g.hval[s + q];
    H[i + (int64_t)j * ldh] = v;
    H[j + (int64_t)i * ldh] = v;
  }
}

// Dense H = A^T A on MFMA float64: one workgroup per 64 x 64 tile on or below the
// diagonal of H (tiles taken column by column).  Rows of A are staged in LDS 16 at a time
// for the tile's two column blocks (one block on the diagonal), double-buffered, with the
// next rows' loads in flight while the current ones are multiplied; each of the four waves
// accumulates a 32 x 32 quadrant as 2 x 2 blocks of 16.  Each H_ij is summed over the rows
// in a fixed order; the tile is written to both triangles (a diagonal tile from its lower
// half, so each entry has one writer).
constexpr int GD_KR = 16, GD_LD = 64 + 4;
__global__ __launch_bounds__(256) void k_gram_dense(int m, int n, const double* __restrict__ A, int lda,
                                                    double* __restrict__ H, int ldh) {
  typedef MF<double> M;
  __shared__ double Sa[2][GD_KR * GD_LD], Sb[2][GD_KR * GD_LD];
  const int nb = (n + 63) / 64;
  int t = blockIdx.x, J = 0;
  while (t >= nb - J) {
    t -= nb - J;
    ++J;
  }
  const int I = J + t;
  const bool diag = I == J;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, lr = lane & 15, lk = lane >> 4;
  const int qr = (w & 1) * 32, qc = (w >> 1) * 32;
  // staging: thread tid moves row srow of columns scol + 16 u (u < 4) of each block
  const int srow = tid & 15, scol = tid >> 4;
  const int ci0 = I * 64 + scol, cj0 = J * 64 + scol;
  double pa[4], pb[4];
  auto fetch = [&](int r0) __attribute__((always_inline)) {
    const double* rowp = A + min(r0 + srow, m - 1);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      pa[u] = rowp[(int64_t)min(ci0 + 16 * u, n - 1) * lda];
      pb[u] = rowp[(int64_t)min(cj0 + 16 * u, n - 1) * lda];   // on the diagonal, a copy of pa
    }
  };
  M::acc acc[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = (M::acc){0.0, 0.0, 0.0, 0.0};
  const int nch = (m + GD_KR - 1) / GD_KR;
  fetch(0);
  for (int ch = 0; ch < nch; ++ch) {
    double* sa = Sa[ch & 1];
    double* sb = diag ? sa : Sb[ch & 1];
    const bool rin = ch * GD_KR + srow < m;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      sa[srow * GD_LD + scol + 16 * u] = (rin && ci0 + 16 * u < n) ? pa[u] : 0.0;
      if (!diag) sb[srow * GD_LD + scol + 16 * u] = (rin && cj0 + 16 * u < n) ? pb[u] : 0.0;
    }
    __syncthreads();   // also: every wave is done with the buffer written next step
    if (ch + 1 < nch) fetch((ch + 1) * GD_KR);
#pragma unroll
    for (int kk = 0; kk < GD_KR; kk += 4) {
      const double* ra = sa + (kk + lk) * GD_LD + lr;
      const double* rb = sb + (kk + lk) * GD_LD + lr;
      const double a0 = ra[qr], a1 = ra[qr + 16], b0 = rb[qc], b1 = rb[qc + 16];
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
        const int i = I * 64 + qr + 16 * bi + M::row(lane, v), j = J * 64 + qc + 16 * bj + lr;
        if (i < n && j < n && (!diag || i >= j)) {
          H[i + (int64_t)j * ldh] = acc[bi][bj][v];
          H[j + (int64_t)i * ldh] = acc[bi][bj][v];
        }
      }
}

// out_j = scale * sum_r A_rj v_r: one wave per column, fixed lane-stride partial sums and
// a fixed shuffle tree.
__global__ __launch_bounds__(256) void k_gemvT_dense(int m, int n, const double* __restrict__ A, int lda,
                                                     const double* __restrict__ v, double* __restrict__ out,
                                                     double scale) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= n) return;
  const double* col = A + (int64_t)j * lda;
  double s = 0.0;
  for (int r = lane; r < m; r += 64) s = fma(col[r], v[r], s);
  for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
  if (lane == 0) out[j] = scale * s;
}

// One workgroup per packed request: the dense block is zeroed, then, one wave per column,
// dense[a_off + i + m j] = val for every stored entry (i, j).
__global__ void __launch_bounds__(256) k_csc_scatter(const ScatterDesc* __restrict__ desc,
                                                     const char* __restrict__ packed,
                                                     double* __restrict__ dense) {
  const ScatterDesc d = desc[blockIdx.x];
  const PackLayout L = pack_layout(d.m, d.n, d.nnz);
  const char* base = packed + d.in_off;
  const int32_t* colptr = (const int32_t*)base;
  const int32_t* rowidx = (const int32_t*)(base + L.rowidx);
  const double* val = (const double*)(base + L.val);
  double* A = dense + d.a_off;
  const int64_t total = (int64_t)d.m * d.n;
  for (int64_t e = threadIdx.x; e < total; e += blockDim.x) A[e] = 0.0;
  __syncthreads();   // the zeros land before the nonzeros
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int j = wave; j < d.n; j += 4) {
    const int e1 = colptr[j + 1];
    for (int e = colptr[j] + lane; e < e1; e += 64) A[(int64_t)j * d.m + rowidx[e]] = val[e];
  }
}

inline int blocks_for(int64_t n, int bs, int cap = 8192) {
  int64_t b = (n + bs - 1) / bs;
  if (b < 1) b = 1;
  return (int)(b > cap ? cap : b);
}

}  // namespace

void launch_fill(hipStream_t s, double* p, int64_t count, double v) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_fill_f64, dim3(blocks_for(count, 256)), dim3(256), 0, s, p, count, v);
}

void launch_fill_i32(hipStream_t s, int32_t* p, int64_t count, int32_t v) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(count, 256)), dim3(256), 0, s, p, count, v);
}

void launch_fill_2d(hipStream_t s, int rows, int cols, double* p, int ld, double v) {
  hipLaunchKernelGGL(k_fill_2d, dim3(blocks_for((int64_t)rows * cols, 256)), dim3(256), 0, s, rows, cols, p, ld, v);
}

void launch_validate_csc(hipStream_t s, int m, int n, int64_t nnz, const int32_t* colptr,
                         const int32_t* rowidx, const double* val, const double* b, int32_t* err) {
  hipLaunchKernelGGL(k_validate_csc, dim3(blocks_for(m > n ? m : n, 256, 2048)), dim3(256), 0, s,
                     m, n, nnz, colptr, rowidx, val, b, err);
}

void launch_validate_dense(hipStream_t s, int m, int n, const double* A, int lda, const double* b,
                           int32_t* err) {
  hipLaunchKernelGGL(k_validate_dense, dim3(blocks_for((int64_t)m * n, 256, 4096)), dim3(256), 0, s,
                     m, n, A, lda, b, err);
}

// sums: scratch of ceil(n / SCAN_CHUNK) entries
template <typename Tin, typename Tout>
static void launch_scan(hipStream_t s, int64_t n, const Tin* count, Tout* out, Tout* sums) {
  const int nchunk = (int)((n + SCAN_CHUNK - 1) / SCAN_CHUNK);
  if (nchunk > 0) hipLaunchKernelGGL((k_scan_sums<Tin, Tout>), dim3(nchunk), dim3(256), 0, s, n, count, sums);
  hipLaunchKernelGGL((k_scan_top<Tout>), dim3(1), dim3(256), 0, s, nchunk, sums, out + n);
  if (nchunk > 0)
    hipLaunchKernelGGL((k_scan_apply<Tin, Tout>), dim3(nchunk), dim3(256), 0, s, n, count, (const Tout*)sums, out);
}

void launch_scan_i32(hipStream_t s, int64_t n, const int32_t* count, int32_t* out, int32_t* sums) {
  launch_scan<int32_t, int32_t>(s, n, count, out, sums);
}

void launch_build_csr(hipStream_t s, int m, int n, int64_t nnz, const int32_t* colptr,
                      const int32_t* rowidx, const double* val, int32_t* rowcnt, int32_t* rowptr,
                      int32_t* colidx, double* valr, void* scan_scratch) {
  launch_fill_i32(s, rowcnt, m, 0);
  if (nnz > 0)
    hipLaunchKernelGGL(k_row_count, dim3(blocks_for(nnz, 256)), dim3(256), 0, s, nnz, rowidx, rowcnt);
  launch_scan<int32_t, int32_t>(s, (int64_t)m, (const int32_t*)rowcnt, rowptr, (int32_t*)scan_scratch);
  launch_fill_i32(s, rowcnt, m, 0);
  hipLaunchKernelGGL(k_csr_fill, dim3(blocks_for(n, 256, 1 << 30)), dim3(256), 0, s, n, colptr, rowidx,
                     val, (const int32_t*)rowptr, rowcnt, colidx, valr);
  hipLaunchKernelGGL(k_csr_sort, dim3(blocks_for(m, 256, 1 << 30)), dim3(256), 0, s, m,
                     (const int32_t*)rowptr, colidx, valr);
}

void launch_gram_bound(hipStream_t s, int n, const int32_t* colptr, const int32_t* rowidx,
                       const int32_t* rowptr, int64_t* hptr, void* scan_scratch) {
  // ub into hptr[0..n), then an in-place exclusive scan into hptr[0..n]
  hipLaunchKernelGGL(k_gram_bound, dim3(blocks_for(n, 256, 1 << 30)), dim3(256), 0, s, n, colptr,
                     rowidx, rowptr, hptr);
  launch_scan<int64_t, int64_t>(s, (int64_t)n, (const int64_t*)hptr, hptr, (int64_t*)scan_scratch);
}

void launch_gram_lower(hipStream_t s, int n, const int32_t* colptr, const int32_t* rowidx,
                       const double* val, const int32_t* rowptr, const int32_t* colidx,
                       const double* valr, const int64_t* hptr, int32_t* hcnt, int32_t* hrow,
                       double* hval) {
  hipLaunchKernelGGL(k_gram_lower, dim3((n + 3) / 4), dim3(256), 0, s, n, colptr, rowidx, val, rowptr,
                     colidx, valr, hptr, hcnt, hrow, hval);
}

void launch_gram_mirror(hipStream_t s, int n, GramLower g, int32_t* upcnt, int32_t* hrow, double* hval) {
  hipLaunchKernelGGL(k_gram_mirror, dim3((n + 3) / 4), dim3(256), 0, s, n, g, upcnt, hrow, hval);
}

void launch_gram_positions(hipStream_t s, int nF, GramLower g, const int32_t* upcnt,
                           const int32_t* Flist, const int32_t* pos, int32_t* pcnt, int32_t* prow,
                           double* pval) {
  if (nF <= 0) return;
  hipLaunchKernelGGL(k_gram_positions, dim3((nF + 3) / 4), dim3(256), 0, s, nF, g, upcnt, Flist, pos,
                     pcnt, prow, pval);
}

void launch_spmvT_csc(hipStream_t s, int n, const int32_t* colptr, const int32_t* rowidx,
                      const double* val, const double* v, double* out, double scale) {
  hipLaunchKernelGGL(k_spmvT_csc, dim3(blocks_for(n, 256, 1 << 30)), dim3(256), 0, s, n, colptr, rowidx,
                     val, v, out, scale);
}

void launch_lower_to_dense(hipStream_t s, int n, GramLower g, double* H, int ldh) {
  hipLaunchKernelGGL(k_lower_to_dense, dim3(blocks_for(n, 256, 1 << 30)), dim3(256), 0, s, n, g, H, ldh);
}

void launch_gram_dense(hipStream_t s, int m, int n, const double* A, int lda, double* H, int ldh) {
  const int nb = (n + 63) / 64;
  hipLaunchKernelGGL(k_gram_dense, dim3((unsigned)(nb * (nb + 1) / 2)), dim3(256), 0, s, m, n, A, lda, H, ldh);
}

void launch_gemvT_dense(hipStream_t s, int m, int n, const double* A, int lda, const double* v,
                        double* out, double scale) {
  hipLaunchKernelGGL(k_gemvT_dense, dim3((n + 3) / 4), dim3(256), 0, s, m, n, A, lda, v, out, scale);
}

void launch_csc_scatter(hipStream_t s, int count, const ScatterDesc* desc, const char* packed,
                        double* dense) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_csc_scatter, dim3(count), dim3(256), 0, s, desc, packed, dense);
}

}  // namespace nnls
