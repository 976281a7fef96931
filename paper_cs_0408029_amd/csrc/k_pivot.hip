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
//   3. Flip the exchanged flags, rebuild the ascending F list and the position map by a
//      block scan, and zero x on the new G and y on the new F.
// The whole vector fits one workgroup's sweep for every size this library targets
// (n up to a few hundred thousand), so the step needs no grid-wide synchronisation.
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

__global__ __launch_bounds__(CTRL_THREADS) void k_pivot_control(
    int n, double* __restrict__ x, double* __restrict__ y, uint8_t* __restrict__ flags,
    int32_t* __restrict__ Flist, int32_t* __restrict__ pos, Ctrl* ctrl, double tau, int p_max,
    int max_iter, int32_t* __restrict__ colcnt, int ncol) {
  __shared__ int s_cnt[16], s_max[16];
  __shared__ double s_mar[16];
  __shared__ int s_branch, s_rmax, s_done;
  __shared__ int s_off[16];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;

  if (ctrl->status != 0) {          // a previous step failed: keep F as it was, stop
    if (tid == 0) ctrl->done = 1;
    return;
  }

  // the factorisation and solves of this iteration start from zeroed counters
  for (int i = tid; i < ncol; i += CTRL_THREADS) colcnt[i] = 0;

  // 1. classify + zero + count
  int cnt = 0, rmax = -1;
  double mar = INFINITY;
  for (int i0 = 0; i0 < n; i0 += CTRL_THREADS) {
    const int i = i0 + tid;
    bool bad = false;
    if (i < n) {
      const bool f = flags[i] != 0;
      const double v = f ? x[i] : y[i];
      if (fabs(v) < tau) {
        if (f) x[i] = 0.0; else y[i] = 0.0;
      } else {
        mar = fmin(mar, fabs(v));
        bad = v < 0.0;
      }
      if (bad) rmax = i;
    }
    cnt += __popcll(__ballot(bad));
  }
  rmax = wave_max(rmax);
  mar = wave_min(mar);
  if (lane == 0) {
    s_cnt[w] = cnt;
    s_max[w] = rmax;
    s_mar[w] = mar;
  }
  __syncthreads();

  // 2. counter rule (one thread)
  if (tid == 0) {
    int k = 0, r = -1;
    double mm = INFINITY;
    for (int q = 0; q < CTRL_THREADS / 64; ++q) {
      k += s_cnt[q];
      r = max(r, s_max[q]);
      mm = fmin(mm, s_mar[q]);
    }
    ctrl->k = k;
    ctrl->rmax = r;
    ctrl->min_margin = mm;
    int branch = -1, done = 0;
    if (k == 0) {
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
    ctrl->fwd_done = 0;
    ctrl->bwd_done = 0;
    s_branch = branch;
    s_rmax = r;
    s_done = done;
  }
  __syncthreads();
  if (s_done) return;

  // 3a. exchange (same element-to-thread map as step 1, so each thread re-reads its own
  //     zeroed entries)
  const int branch = s_branch, rsel = s_rmax;
  for (int i = tid; i < n; i += CTRL_THREADS) {
    const uint8_t f = flags[i];
    const double v = f ? x[i] : y[i];
    const bool flip = (branch == 2) ? (i == rsel) : (v < 0.0);
    if (flip) flags[i] = f ^ 1;
  }
  __syncthreads();

  // 3b. F list by a block scan over contiguous segments
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
}

__global__ void k_reset_tickets(Ctrl* ctrl) {
  ctrl->chol_ticket = 0;
  ctrl->fwd_ticket = 0;
  ctrl->bwd_ticket = 0;
  ctrl->fwd_done = 0;
  ctrl->bwd_done = 0;
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
                          int max_iter, int32_t* colcnt, int ncol) {
  hipLaunchKernelGGL(k_pivot_control, dim3(1), dim3(CTRL_THREADS), 0, s, n, x, y, flags, Flist, pos,
                     ctrl, tau, p_max, max_iter, colcnt, ncol);
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
