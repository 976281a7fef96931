// Pivot control: the classify / count / exchange part of the block principal pivoting
// loop (Sec. 2 algorithm box of the tsnnls paper), as one single-workgroup kernel.
//
// Per call:
//   1. For every variable take its tested entry v (x_i on F, y_i on G); if |v| < tau set
//      it to zero in place (the paper's degeneracy workaround), else it is infeasible iff
//      v < 0.  Count k with wavefront ballots; keep the largest infeasible index and the
//      smallest kept |v|.
//   2. k == 0: feasible, done.  Otherwise apply the counter rule: k < N -> N = k, p = p_max,
//      exchange all; else p > 0 -> p -= 1, exchange all; else exchange only the largest
//      infeasible index.
//   3. Flip the exchanged flags, rebuild the F list (the order in which the factor takes
//      F) and the position map, and zero x on the new G and y on the new F.
// The whole vector fits one workgroup's sweep for every size this library targets
// (n up to a few hundred thousand), so the step needs no grid-wide synchronisation.
//
// Order of F.  The paper's normal equations may take F in any order: H_FF and P H_FF P^T
// give the same x_F.  Inside the pivot loop the new order starts with the longest run of
// leading positions of the previous order that no exchange touched, cut to whole 64-wide
// tiles: the factor of that leading block (and the matching part of the forward solve) is
// exactly the previous one, so the factorisation starts after it.  The rest of the
// previous order follows, stably sorted by the binary exponent of x_F, largest first
// (variables with small x_F are the likely leavers of the next exchange, so they go
// last), then the variables that join F, ascending.
#include <climits>

#include "nnls_internal.h"

namespace nnls {

namespace {

constexpr int CTRL_THREADS = 1024;

__global__ void k_pivot_init(int n, const double* __restrict__ c, double* __restrict__ x,
                             double* __restrict__ y, uint8_t* __restrict__ flags, Ctrl* ctrl, int p_max) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    x[i] = 0.0;
    y[i] = -c[i];
    flags[i] = 0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    Ctrl z = {};
    z.N = INT32_MAX;
    z.p = p_max;
    z.branch = -1;
    z.rmax = -1;
    z.failed_pos = INT32_MAX;
    z.min_margin = INFINITY;
    *ctrl = z;
  }
}

__device__ inline double wave_min(double v) {
  for (int d = 32; d >= 1; d >>= 1) v = fmin(v, __shfl_xor(v, d, 64));
  return v;
}
__device__ inline int wave_max(int v) {
  for (int d = 32; d >= 1; d >>= 1) v = max(v, __shfl_xor(v, d, 64));
  return v;
}

constexpr int NBUCKET = 64;    // exponent classes of the reordered part of F
constexpr int CTRL_BATCH = 8;  // entries per thread fetched together by the classify and exchange

// Exponent class of x >= 0 relative to the largest exponent emax: 0 holds the largest
// values, NBUCKET - 1 holds zero, subnormals and anything NBUCKET - 2 binades below.
__device__ inline int order_bucket(double v, int emax) {
  const int e = (int)((__double_as_longlong(v) >> 52) & 0x7ff);
  if (!(v > 0.0) || e == 0) return NBUCKET - 1;
  return min(emax - e, NBUCKET - 2);
}

// mode 0: ascending F list; mode 1: ordered F, nothing kept from the previous factor;
// mode 2: ordered F, the untouched leading tiles of the previous factor are kept.
__global__ __launch_bounds__(CTRL_THREADS) void k_pivot_control(
    int n, double* __restrict__ x, double* __restrict__ y, uint8_t* __restrict__ flags,
    int32_t* __restrict__ Flist, int32_t* __restrict__ pos, Ctrl* ctrl, double tau, int p_max,
    int max_iter, int32_t* __restrict__ colcnt, int ncol, int32_t* __restrict__ Fold, int mode) {
  __shared__ int s_cnt[16], s_max[16], s_bad[16];
  __shared__ double s_mar[16];
  __shared__ int s_branch, s_rmax, s_done;
  __shared__ int s_off[16];
  __shared__ int s_hist[16][NBUCKET];
  __shared__ int s_tot[NBUCKET];
  __shared__ int s_p0[16], s_emax[16], s_add[16], s_rem[16];
  __shared__ int s_P, s_M, s_K, s_E, s_nold;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

  if (ctrl->status != 0) {          // a previous step failed: keep F as it was, stop
    if (tid == 0) ctrl->done = 1;
    return;
  }

  // the factorisation and solves of this iteration start from zeroed counters
  for (int i = tid; i < ncol; i += CTRL_THREADS) colcnt[i] = 0;

  // 1. classify + zero + count.  A tested entry that is not finite (an iterate that
  //    overflowed) is no sign test at all: the step stops with NNLS_ERR_INVALID_VALUE.
  int cnt = 0, rmax = -1;
  bool nonfinite = false;
  double mar = INFINITY;
  // CTRL_BATCH entries per thread are fetched together (flag, x and y alike, so no load
  // waits for another), then tested in the same order as one at a time
  for (int i0 = 0; i0 < n; i0 += CTRL_THREADS * CTRL_BATCH) {
    uint8_t fb[CTRL_BATCH];
    double xb[CTRL_BATCH], yb[CTRL_BATCH];
#pragma unroll
    for (int u = 0; u < CTRL_BATCH; ++u) {
      const int i = i0 + u * CTRL_THREADS + tid;
      fb[u] = (i < n) ? flags[i] : (uint8_t)0;
      xb[u] = (i < n) ? x[i] : 0.0;
      yb[u] = (i < n) ? y[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < CTRL_BATCH; ++u) {
      const int i = i0 + u * CTRL_THREADS + tid;
      bool bad = false;
      if (i < n) {
        const bool f = fb[u] != 0;
        const double v = f ? xb[u] : yb[u];
        if (!isfinite(v)) {
          nonfinite = true;
        } else if (fabs(v) < tau) {
          if (f) x[i] = 0.0; else y[i] = 0.0;
        } else {
          mar = fmin(mar, fabs(v));
          bad = v < 0.0;
        }
        if (bad) rmax = i;
      }
      cnt += __popcll(__ballot(bad));
    }
  }
  rmax = wave_max(rmax);
  mar = wave_min(mar);
  const bool wave_nonfinite = __ballot(nonfinite) != 0;
  if (lane == 0) {
    s_cnt[w] = cnt;
    s_max[w] = rmax;
    s_mar[w] = mar;
    s_bad[w] = wave_nonfinite ? 1 : 0;
  }
  __syncthreads();

  // 2. counter rule (one thread)
  if (tid == 0) {
    int k = 0, r = -1, nonfin = 0;
    double mm = INFINITY;
    for (int q = 0; q < CTRL_THREADS / 64; ++q) {
      k += s_cnt[q];
      r = max(r, s_max[q]);
      mm = fmin(mm, s_mar[q]);
      nonfin |= s_bad[q];
    }
    ctrl->k = k;
    ctrl->rmax = r;
    ctrl->min_margin = mm;
    int branch = -1, done = 0;
    if (nonfin) {
      done = 1;
      ctrl->status = NNLS_ERR_INVALID_VALUE;
    } else if (k == 0) {
      done = 1;
    } else if (ctrl->iter >= max_iter) {
      done = 1;
      ctrl->status = NNLS_ERR_MAXITER;
    } else {
      int N = ctrl->N, p = ctrl->p;
      if (k < N) {
        N = k;
        p = p_max;
        branch = 0;
      } else if (p > 0) {
        p -= 1;
        branch = 1;
      } else {
        branch = 2;
      }
      ctrl->N = N;
      ctrl->p = p;
      ctrl->iter += 1;
    }
    ctrl->branch = branch;
    ctrl->done = done;
    ctrl->chol_ticket = 0;
    ctrl->fwd_ticket = 0;
    ctrl->bwd_ticket = 0;
    ctrl->fwd_walked = 0;
    ctrl->bwd_walked = 0;
    s_branch = branch;
    s_rmax = r;
    s_done = done;
    s_nold = ctrl->n_free;
  }
  __syncthreads();
  if (s_done) return;

  // 3a. exchange (same element-to-thread map as step 1, so each thread re-reads its own
  //     zeroed entries).  In the ordered modes bit 1 of a flag keeps the old membership
  //     until the new order is built.
  const int branch = s_branch, rsel = s_rmax;
  int p0 = INT_MAX, emax = 0, nadd = 0, nrem = 0;
  for (int i0 = 0; i0 < n; i0 += CTRL_THREADS * CTRL_BATCH) {
    uint8_t fb[CTRL_BATCH];
    double xb[CTRL_BATCH], yb[CTRL_BATCH];
#pragma unroll
    for (int u = 0; u < CTRL_BATCH; ++u) {
      const int i = i0 + u * CTRL_THREADS + tid;
      fb[u] = (i < n) ? flags[i] : (uint8_t)0;
      xb[u] = (i < n) ? x[i] : 0.0;
      yb[u] = (i < n) ? y[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < CTRL_BATCH; ++u) {
      const int i = i0 + u * CTRL_THREADS + tid;
      bool add = false, rem = false;
      if (i < n) {
        const uint8_t f = fb[u];
        const double v = f ? xb[u] : yb[u];
        const bool flip = (branch == 2) ? (i == rsel) : (v < 0.0);
        if (mode == 0) {
          if (flip) flags[i] = f ^ 1;
        } else {
          flags[i] = (uint8_t)((f ^ (flip ? 1 : 0)) | (f << 1));
          add = flip && !f;
          rem = flip && f;
          if (rem && mode == 2) p0 = min(p0, pos[i]);
          if (f && !flip && v > 0.0) emax = max(emax, (int)((__double_as_longlong(v) >> 52) & 0x7ff));
        }
      }
      nadd += __popcll(__ballot(add));
      nrem += __popcll(__ballot(rem));
    }
  }
  if (mode != 0) {
    p0 = -wave_max(-p0);
    emax = wave_max(emax);
    if (lane == 0) {
      s_p0[w] = p0;
      s_emax[w] = emax;
      s_add[w] = nadd;
      s_rem[w] = nrem;
    }
  }
  __syncthreads();

  if (mode == 0) {
    // 3b. ascending F list by a block scan over contiguous segments
    const int seg = (n + CTRL_THREADS - 1) / CTRL_THREADS;
    const int s0 = min(n, tid * seg), s1 = min(n, s0 + seg);
    int local = 0;
    for (int i = s0; i < s1; ++i) local += flags[i];
    int v = local;
    for (int d = 1; d < 64; d <<= 1) {
      const int o = __shfl_up(v, d, 64);
      if (lane >= d) v += o;
    }
    if (lane == 63) s_off[w] = v;
    __syncthreads();
    if (tid == 0) {
      int run = 0;
      for (int q = 0; q < CTRL_THREADS / 64; ++q) {
        const int t = s_off[q];
        s_off[q] = run;
        run += t;
      }
      ctrl->n_free = run;
      ctrl->j0 = 0;
    }
    __syncthreads();
    int p = s_off[w] + v - local;
    for (int i = s0; i < s1; ++i) {
      if (flags[i]) {
        pos[i] = p;
        Flist[p] = i;
        y[i] = 0.0;
        ++p;
      } else {
        pos[i] = -1;
        x[i] = 0.0;
      }
    }
    return;
  }

  // 3c. the kept leading tiles, and the part of the previous order to reorder
  if (tid == 0) {
    int pm = INT_MAX, em = 0, na = 0, nr = 0;
    for (int q = 0; q < CTRL_THREADS / 64; ++q) {
      pm = min(pm, s_p0[q]);
      em = max(em, s_emax[q]);
      na += s_add[q];
      nr += s_rem[q];
    }
    const int nold = s_nold;
    const int nnew = nold - nr + na;
    int j0 = 0;
    if (mode == 2 && nnew > 0) {
      j0 = min(pm, nold) / TILE;
      j0 = min(j0, (nnew + TILE - 1) / TILE - 1);   // the last tile column is always refactored
      j0 = max(j0, 0);
    }
    s_P = j0 * TILE;
    s_M = nold - j0 * TILE;
    s_E = em;
    ctrl->j0 = j0;
    ctrl->n_free = nnew;
  }
  for (int b = tid; b < 16 * NBUCKET; b += CTRL_THREADS) s_hist[b / NBUCKET][b % NBUCKET] = 0;
  __syncthreads();
  const int P = s_P, M = s_M, E = s_E;
  for (int t = tid; t < M; t += CTRL_THREADS) Fold[t] = Flist[P + t];
  __syncthreads();

  // 3d. stable sort of the kept part of Fold[0, M) by exponent class: counts per wave and
  //     class, then offsets in (class, wave) order, then a scatter that keeps the order
  //     inside each wave's contiguous chunk (ranks among equal classes from ballots)
  const int chunk = (M + CTRL_THREADS / 64 - 1) / (CTRL_THREADS / 64);
  const int c0 = min(M, w * chunk), c1 = min(M, c0 + chunk);
  for (int t = c0 + lane; t < c1; t += 64) {
    const int i = Fold[t];
    if ((unsigned)i < (unsigned)n && (flags[i] & 1)) atomicAdd(&s_hist[w][order_bucket(x[i], E)], 1);
  }
  __syncthreads();
  if (tid < NBUCKET) {
    int run = 0;
    for (int q = 0; q < CTRL_THREADS / 64; ++q) {
      const int c = s_hist[q][tid];
      s_hist[q][tid] = run;
      run += c;
    }
    s_tot[tid] = run;
  }
  __syncthreads();
  if (tid == 0) {
    int run = P;
    for (int b = 0; b < NBUCKET; ++b) {
      const int c = s_tot[b];
      s_tot[b] = run;
      run += c;
    }
    s_K = run - P;
  }
  __syncthreads();
  if (tid < NBUCKET)
    for (int q = 0; q < CTRL_THREADS / 64; ++q) s_hist[q][tid] += s_tot[tid];
  __syncthreads();
  for (int t0 = c0; t0 < c1; t0 += 64) {
    const int t = t0 + lane;
    int i = -1, key = 0;
    bool keep = false;
    if (t < c1) {
      i = Fold[t];
      keep = (unsigned)i < (unsigned)n && (flags[i] & 1) != 0;
      if (keep) key = order_bucket(x[i], E);
    }
    uint64_t peers = __ballot(keep);
#pragma unroll
    for (int bit = 0; bit < 6; ++bit) {
      const uint64_t m = __ballot((key >> bit) & 1);
      peers &= ((key >> bit) & 1) ? m : ~m;
    }
    const int base = keep ? s_hist[w][key] : 0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (keep) {
      const int dest = base + __popcll(peers & lt_mask);
      Flist[dest] = i;
      pos[i] = dest;
      if ((peers & lt_mask) == 0) s_hist[w][key] = base + __popcll(peers);   // lowest lane of its class
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();

  // 3e. the joining variables after the kept ones, ascending (block scan over contiguous
  //     segments); new G: pos = -1, x = 0; new F: y = 0; flags back to 0 / 1
  const int seg = (n + CTRL_THREADS - 1) / CTRL_THREADS;
  const int s0 = min(n, tid * seg), s1 = min(n, s0 + seg);
  int local = 0;
  for (int i = s0; i < s1; ++i) local += (flags[i] == 1);
  int v = local;
  for (int d = 1; d < 64; d <<= 1) {
    const int o = __shfl_up(v, d, 64);
    if (lane >= d) v += o;
  }
  if (lane == 63) s_off[w] = v;
  __syncthreads();
  if (tid == 0) {
    int run = 0;
    for (int q = 0; q < CTRL_THREADS / 64; ++q) {
      const int t = s_off[q];
      s_off[q] = run;
      run += t;
    }
  }
  __syncthreads();
  int p = P + s_K + s_off[w] + v - local;
  for (int i = s0; i < s1; ++i) {
    const uint8_t f = flags[i];
    if (f & 1) {
      if (f == 1) {
        pos[i] = p;
        Flist[p] = i;
        ++p;
      }
      y[i] = 0.0;
    } else {
      pos[i] = -1;
      x[i] = 0.0;
    }
    flags[i] = f & 1;
  }
}

__global__ void k_reset_tickets(Ctrl* ctrl) {
  ctrl->chol_ticket = 0;
  ctrl->fwd_ticket = 0;
  ctrl->bwd_ticket = 0;
  ctrl->fwd_walked = 0;
  ctrl->bwd_walked = 0;
}

__global__ void k_ctrl_clear_breakdown(Ctrl* ctrl) {
  if (ctrl->status == NNLS_ERR_NOT_PD) {
    ctrl->status = 0;
    ctrl->failed_pos = INT32_MAX;
  }
}

__global__ void k_ctrl_set_state(Ctrl* ctrl, int N, int p, int iter) {
  Ctrl z = {};
  z.N = N;
  z.p = p;
  z.iter = iter;
  z.branch = -1;
  z.rmax = -1;
  z.failed_pos = INT32_MAX;
  z.min_margin = INFINITY;
  *ctrl = z;
}

}  // namespace

void launch_pivot_init(hipStream_t s, int n, const double* c, double* x, double* y,
                       uint8_t* flags, Ctrl* ctrl, int p_max) {
  int blocks = (n + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_pivot_init, dim3(blocks), dim3(256), 0, s, n, c, x, y, flags, ctrl, p_max);
}

void launch_pivot_control(hipStream_t s, int n, double* x, double* y, uint8_t* flags,
                          int32_t* Flist, int32_t* pos, Ctrl* ctrl, double tau, int p_max,
                          int max_iter, int32_t* colcnt, int ncol, int32_t* Fold, int mode) {
  hipLaunchKernelGGL(k_pivot_control, dim3(1), dim3(CTRL_THREADS), 0, s, n, x, y, flags, Flist, pos,
                     ctrl, tau, p_max, max_iter, colcnt, ncol, Fold, mode);
}

void launch_ctrl_set_state(hipStream_t s, Ctrl* ctrl, int N, int p, int iter, int /*unused*/) {
  hipLaunchKernelGGL(k_ctrl_set_state, dim3(1), dim3(1), 0, s, ctrl, N, p, iter);
}

void launch_ctrl_clear_breakdown(hipStream_t s, Ctrl* ctrl) {
  hipLaunchKernelGGL(k_ctrl_clear_breakdown, dim3(1), dim3(1), 0, s, ctrl);
}

void launch_reset_tickets(hipStream_t s, Ctrl* ctrl) {
  hipLaunchKernelGGL(k_reset_tickets, dim3(1), dim3(1), 0, s, ctrl);
}

}  // namespace nnls
