// Batched dense NNLS: one launch solves many independent problems; each workgroup owns
// one problem and runs its whole block principal pivoting loop (Sec. 2 algorithm box of
// the tsnnls paper) on the device, with no host round trip per iteration:
//   one pass over A for c = A^T b and the finiteness check, the Gram matrix H = A^T A
//   (Sec. 3, Sec. 2.1) streamed through LDS on MFMA, then per iteration the classify /
//   count / exchange step, the left-looking tiled Cholesky of H_FF on MFMA (one tile after
//   another inside the workgroup, with the same in-LDS diagonal factor as the large-problem
//   kernel), the two triangular solves, r = A_F x_F - b and y_G = A_G^T r (Eq. 5).
// The factor is float64, or float32 (from a float32 Gram matrix) followed by float64
// refinement of x_F against the residual from A.  A problem's arithmetic never depends on
// the other problems in the launch, so every result is the same alone or in any batch.
#include <climits>

#include "tile_ops.h"

namespace nnls {

namespace {

constexpr int BT = 256;   // threads per workgroup

// Workspace layout of one problem (byte offsets from its base).
struct WsLayout {
  size_t state, H, c, r, flags, Flist, Glist, Lt, Dv, z, xF, g, total;
};

__host__ __device__ inline WsLayout ws_layout(int m, int n) {
  const int nb = (n + TILE - 1) / TILE;
  const size_t nt = (size_t)nb * (nb + 1) / 2;
  WsLayout L;
  size_t o = 0;
  L.state = o; o += 256;
  L.H = o;     o += ((size_t)n * n * 8 + 255) & ~(size_t)255;
  L.c = o;     o += ((size_t)n * 8 + 255) & ~(size_t)255;
  L.r = o;     o += ((size_t)m * 8 + 255) & ~(size_t)255;
  L.flags = o; o += ((size_t)n + 255) & ~(size_t)255;
  L.Flist = o; o += ((size_t)n * 4 + 255) & ~(size_t)255;
  L.Glist = o; o += ((size_t)n * 4 + 255) & ~(size_t)255;
  L.Lt = o;    o += nt * TILE_ELEMS * 8;              // sized for float64 tiles
  L.Dv = o;    o += (size_t)nb * TILE_ELEMS * 8;
  L.z = o;     o += (size_t)nb * TILE * 8;
  L.xF = o;    o += (size_t)nb * TILE * 8;
  L.g = o;     o += (size_t)nb * TILE * 8;
  L.total = o;
  return L;
}

// Pivot state of a problem between launches (a launch may stop after a number of pivot
// iterations and the next one resumes at the classify step): the Sec. 2 counters N and p,
// the iterations taken, |F| of the last exchange and the precision of the Gram matrix.
struct BatchState {
  int32_t started, N, p, iter, nF, h64, pad0, pad1;
};

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
// H = A^T A (full symmetric, column-major n x n) for n > GS_MAXN: lower 64 x 64 tiles on
// MFMA float64, one tile at a time; rows of A are staged in LDS 64 at a time (both column
// blocks of the tile), so every H_ij is summed over rows in a fixed order.
__device__ __noinline__ void wg_gram(const double* __restrict__ A, int lda, int m, int n,
                                     double* __restrict__ H, double* Sa, double* Sb) {
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
  __syncthreads();
}

// Problem data arrive through descriptors in memory, so the compiler cannot tell that
// their pointers are global: say so, so the loads are global loads (a flat load also
// counts as an LDS access, and every LDS wait would then wait for it too).
typedef const __attribute__((address_space(1))) double* gcdp;
__device__ inline gcdp gl(const double* p) { return (gcdp)p; }

// H = A^T A for n <= GS_MAXN, in T (float64, or float32 from float32-rounded A), streamed
// by a workgroup of GT threads (eight waves, two per SIMD): 16 rows of every column are
// staged in LDS per step (double-buffered, the next rows in registers while the MFMA work
// on the current ones runs).  H is cut into 32 x 32 rectangles on and below the diagonal;
// each wave keeps Q of them (2 x 2 MFMA blocks each, four products per four LDS reads) in
// its accumulators for a whole pass over the rows.  When the rectangles exceed 8 QMAX the
// rows are streamed again for the rest (spread evenly over the passes).  The first pass
// also forms c = A^T b in float64 from the staged values (each thread's rows, then a fixed
// tree over the 16 threads of a column) and checks every entry of A and b for finiteness.
// Every H_ij and c_j is summed over rows in a fixed order.  The code is specialised on
// NR = ceil(n / 32), so that every loop has a fixed trip count.
constexpr int GT = 512;                     // threads of the Gram workgroup
constexpr int GS_MAXN = 256;
constexpr int GS_KR = 16;                   // rows per step
constexpr int GS_CSTEP = GT / GS_KR;        // columns moved per thread step
// Accumulator tile shapes: the most rectangles a wave holds in one pass, by variant (an
// argument of the launch, chosen per NR by the autotuner of prepared batches; shape 1 is
// the default).  Every variant sums each H_ij and c_j in the same order, so the results do
// not depend on the choice.
template <typename T> struct GS;
template <> struct GS<double> { static constexpr int QV[GS_VARIANTS] = {2, 3, 4}; };
template <> struct GS<float> { static constexpr int QV[GS_VARIANTS] = {4, 6, 8}; };
template <typename T, int NR, int V> struct GSPlan {
  static constexpr int QMAX = GS<T>::QV[V];
  static constexpr int nrect = NR * (NR + 1) / 2;
  static constexpr int passes = (nrect + 8 * QMAX - 1) / (8 * QMAX);
  static constexpr int per = (nrect + passes - 1) / passes;   // rectangles per pass
  static constexpr int Q = (per + 7) / 8;                     // per wave
  static constexpr int EPT = 32 * NR / GS_CSTEP;              // staged values per thread
};
// LDS row stride (elements) of the staged rows: 16 columns of one row group start half a
// bank cycle apart from the next group's for 8-byte reads, a quarter for 4-byte reads
template <typename T> __host__ __device__ constexpr int gs_stride(int npad) {
  return sizeof(T) == 8 ? npad + ((16 - npad % 32) + 32) % 32 : npad + ((16 - npad % 64) + 64) % 64;
}
constexpr size_t GS_LDS_BYTES = 2 * GS_KR * (size_t)gs_stride<double>(GS_MAXN) * 8;

// One pass: wave w accumulates the rectangles t0 + w + 8 q (q < Q) below tend; slots past
// tend compute on rectangle (0, 0) and are not stored, so the MFMA sequence has no
// branches.  Staged values past m or n are read clamped into A and multiplied by zero, so
// the loads have no branches either.  Returns nonzero when the first pass met a value of
// A or b that is not finite (H and c are then not meaningful).
template <typename T, int NR, int V>
__device__ __noinline__ int gram_pass(const double* __restrict__ A, int lda, int m, int n,
                                      const double* __restrict__ b, T* __restrict__ H, double* __restrict__ c,
                                      T* St, int t0, int tend) {
  typedef MF<T> M;
  typedef typename M::acc Acc;
  typedef GSPlan<T, NR, V> PL;
  constexpr int KR = GS_KR, CSTEP = GS_CSTEP, EPT = PL::EPT, Q = PL::Q;
  constexpr int npad = 32 * NR, SR = gs_stride<T>(npad);
  static_assert(CSTEP * EPT == npad, "staging covers the padded columns");
  const int tid = threadIdx.x, lane = tid & 63, lr = lane & 15, lk = lane >> 4;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const bool first = t0 == 0;
  const int nch = (m + KR - 1) / KR;
  int ra[Q], rb[Q];   // first row and column of slot q's rectangle
  bool on[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    int t = t0 + w + 8 * q, cc = 0;
    on[q] = t < tend;
    if (!on[q]) t = 0;
    while (t >= NR - cc) {   // rectangles column by column: column cc holds rows cc .. NR-1
      t -= NR - cc;
      ++cc;
    }
    ra[q] = (cc + t) * 32;
    rb[q] = cc * 32;
  }
  Acc acc[Q][2][2];
#pragma unroll
  for (int q = 0; q < Q; ++q)
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[q][bi][bj][v] = (T)0;
  // staging: thread tid moves row srow of columns scol + CSTEP u
  const int srow = tid % KR, scol = tid / KR;
  const gcdp Ag = gl(A), bg = gl(b);
  double pre[EPT], bpre;   // raw loads: nothing waits for them before the next step's stores
  double cpart[EPT];
  bool bad = false;
#pragma unroll
  for (int u = 0; u < EPT; ++u) cpart[u] = 0.0;
  auto fetch = [&](int ch) __attribute__((always_inline)) {
    const int row = min(ch * KR + srow, m - 1);
    const gcdp src = Ag + row;
#pragma unroll
    for (int u = 0; u < EPT; ++u) pre[u] = src[(int64_t)min(scol + CSTEP * u, n - 1) * lda];
    bpre = bg[row];
  };
  fetch(0);
  for (int ch = 0; ch < nch; ++ch) {
    T* B = St + (ch & 1) * (KR * SR);
    T* dst = B + srow * SR + scol;
    const bool rin = ch * KR + srow < m;
    if (first) {
      const double bv = rin ? bpre : 0.0;
      bad |= !isfinite(bpre);
#pragma unroll
      for (int u = 0; u < EPT; ++u) {
        bad |= !isfinite(pre[u]);
        cpart[u] = fma(pre[u], bv, cpart[u]);   // bv = 0 past m; columns past n are not stored
      }
    }
#pragma unroll
    for (int u = 0; u < EPT; ++u)
      dst[CSTEP * u] = (T)(pre[u] * ((rin && scol + CSTEP * u < n) ? 1.0 : 0.0));
    __syncthreads();   // also: every wave is done with the buffer written next step
    if (ch + 1 < nch) fetch(ch + 1);
    // (k step, rectangle) pairs in order, the operands of the next pair read from LDS
    // while the four products of the current one run
    const T* rowp = B + lk * SR + lr;
    T op[2][4];
    constexpr int NS = (KR / 4) * Q;
    auto ld = [&](int st, T* o) __attribute__((always_inline)) {
      const T* pr = rowp + (st / Q) * 4 * SR;
      const int q = st % Q;
      o[0] = pr[ra[q]];
      o[1] = pr[ra[q] + 16];
      o[2] = pr[rb[q]];
      o[3] = pr[rb[q] + 16];
    };
    ld(0, op[0]);
#pragma unroll
    for (int st = 0; st < NS; ++st) {
      if (st + 1 < NS) ld(st + 1, op[(st + 1) & 1]);
      const int q = st % Q;
      const T* o = op[st & 1];
      acc[q][0][0] = M::op(o[0], o[2], acc[q][0][0]);
      acc[q][0][1] = M::op(o[0], o[3], acc[q][0][1]);
      acc[q][1][0] = M::op(o[1], o[2], acc[q][1][0]);
      acc[q][1][1] = M::op(o[1], o[3], acc[q][1][1]);
    }
  }
  if (first) {   // c_j: the 16 threads of column j are lanes 16 g .. 16 g + 15 of one wave
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      double v = cpart[u];
      for (int d = 1; d < 16; d <<= 1) v += __shfl_xor(v, d, 64);
      const int col = scol + CSTEP * u;
      if (srow == 0 && col < n) c[col] = v;
    }
  }
  const int any_bad = __syncthreads_or(bad ? 1 : 0);
#pragma unroll
  for (int q = 0; q < Q; ++q)
    if (on[q])
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int i = ra[q] + 16 * bi + M::row(lane, v), j = rb[q] + 16 * bj + lr;
            // on the diagonal only the lower half is stored, so each entry has one writer
            if (i < n && j < n && (ra[q] != rb[q] || i >= j)) {
              H[i + (int64_t)j * n] = acc[q][bi][bj][v];
              H[j + (int64_t)i * n] = acc[q][bi][bj][v];
            }
          }
  return any_bad;
}

template <typename T, int NR, int V>
__device__ inline int gram_passes(const double* A, int lda, int m, int n, const double* b, T* H, double* c, T* St) {
  typedef GSPlan<T, NR, V> PL;
  int bad = 0;
  for (int t0 = 0; t0 < PL::nrect && !bad; t0 += PL::per)
    bad = gram_pass<T, NR, V>(A, lda, m, n, b, H, c, St, t0, min(PL::nrect, t0 + PL::per));
  return bad;
}

template <typename T, int NR>
__device__ inline int gram_variant(int v, const double* A, int lda, int m, int n, const double* b, T* H, double* c,
                                   T* St) {
  switch (v) {
    case 0: return gram_passes<T, NR, 0>(A, lda, m, n, b, H, c, St);
    case 2: return gram_passes<T, NR, 2>(A, lda, m, n, b, H, c, St);
    default: return gram_passes<T, NR, 1>(A, lda, m, n, b, H, c, St);
  }
}

template <typename T>
__device__ int wg_gram_stream(const double* A, int lda, int m, int n, const double* b, T* H, double* c, T* St,
                              const uint8_t* variant) {
  const int nr = (n + 31) >> 5;
  const int v = variant[nr] == 0 ? 1 : variant[nr] - 1;   // 0: the default shape; 1 + k: shape k
  switch (nr) {
    case 1: return gram_variant<T, 1>(v, A, lda, m, n, b, H, c, St);
    case 2: return gram_variant<T, 2>(v, A, lda, m, n, b, H, c, St);
    case 3: return gram_variant<T, 3>(v, A, lda, m, n, b, H, c, St);
    case 4: return gram_variant<T, 4>(v, A, lda, m, n, b, H, c, St);
    case 5: return gram_variant<T, 5>(v, A, lda, m, n, b, H, c, St);
    case 6: return gram_variant<T, 6>(v, A, lda, m, n, b, H, c, St);
    case 7: return gram_variant<T, 7>(v, A, lda, m, n, b, H, c, St);
    default: return gram_variant<T, 8>(v, A, lda, m, n, b, H, c, St);
  }
}

// ------------------------------------------------------------ factor and solves
// Out-of-line wrapper: the diagonal factor gets its own register allocation.
template <typename T>
__device__ __noinline__ void diag_tile(T* S, T* W, PivotReport rep) {
  factor_invert_tile<T>(S, W, rep);
}

// Left-looking tiled Cholesky of H_FF inside one workgroup (tiles one after another), from
// a Gram matrix held in TH.  Tiles (column-major packed) and inverted diagonal tiles go to
// the problem's workspace.
template <typename T, typename TH>
__device__ __noinline__ void wg_factor(const TH* __restrict__ H, int n, const int32_t* __restrict__ Flist, int nF,
                          T* Lt, T* Dv, T* S, T* W, const PivotReport& rep0) {
  __shared__ int32_t sidx[2 * TILE];
  typedef MF<T> M;
  typedef typename M::acc Acc;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int qr = (w & 1) * 32, qc = (w >> 1) * 32, lr = lane & 15, lk = lane >> 4;
  const int nb = (nF + TILE - 1) / TILE;
  for (int J = 0; J < nb; ++J)
    for (int I = J; I < nb; ++I) {
      // gather tile (I, J) of H_FF (positions past nF are identity padding): the tile's
      // row and column indices staged in LDS, then every thread's 16 loads at once
      __syncthreads();
      if (tid < 2 * TILE) {
        const int p = (tid < TILE ? I : J) * TILE + (tid & (TILE - 1));
        sidx[tid] = p < nF ? Flist[p] : -1;
      }
      __syncthreads();
      constexpr int GH = TILE_ELEMS / BT / 2;   // loads in flight per thread
#pragma unroll
      for (int k0 = 0; k0 < TILE_ELEMS / BT; k0 += GH) {
        TH hv[GH];
#pragma unroll
        for (int k = 0; k < GH; ++k) {
          const int e = tid + BT * (k0 + k), rr = e & (TILE - 1), cc = e >> 6;
          const int fi = sidx[rr], fj = sidx[TILE + cc];
          hv[k] = H[(fi < 0 ? 0 : fi) + (int64_t)(fj < 0 ? 0 : fj) * n];
        }
#pragma unroll
        for (int k = 0; k < GH; ++k) {
          const int e = tid + BT * (k0 + k), rr = e & (TILE - 1), cc = e >> 6;
          const bool in = sidx[rr] >= 0 && sidx[TILE + cc] >= 0;
          S[rr + cc * LDT] = in ? (T)hv[k] : ((I * TILE + rr == J * TILE + cc) ? (T)1 : (T)0);
        }
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

// r = A_F x_F - b: thread t owns rows t + BT u (u < U); the free columns (ascending) and
// their x values are staged in LDS in chunks of CH, and K columns are loaded per step, so
// U K loads are in flight per thread.  Each r_i is summed over F positions in order.
constexpr int CH = 2048;
template <int U, int K>
__device__ __noinline__ void wg_resid_rows(const double* __restrict__ A, int lda, int m, const double* __restrict__ b,
                                           const int32_t* Flist, int nF, const double* x, double* r,
                                           int32_t* sF, double* sX) {
  const int tid = threadIdx.x;
  for (int i0 = 0; i0 < m; i0 += BT * U) {
    double acc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) acc[u] = 0.0;
    int rows[U];
#pragma unroll
    for (int u = 0; u < U; ++u) rows[u] = min(i0 + tid + BT * u, m - 1);   // in bounds; unused past m
    for (int p0 = 0; p0 < nF; p0 += CH) {
      const int cnt = min(CH, nF - p0);
      __syncthreads();
      for (int q = tid; q < cnt; q += BT) {
        const int j = Flist[p0 + q];
        sF[q] = j;
        sX[q] = x[j];
      }
      __syncthreads();
      int p = 0;
      for (; p + K <= cnt; p += K) {
        double v[K][U];
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const double* col = A + (int64_t)sF[p + k] * lda;
#pragma unroll
          for (int u = 0; u < U; ++u) v[k][u] = col[rows[u]];
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const double xv = sX[p + k];
#pragma unroll
          for (int u = 0; u < U; ++u) acc[u] = fma(v[k][u], xv, acc[u]);
        }
      }
      for (; p < cnt; ++p) {
        const double* col = A + (int64_t)sF[p] * lda;
        const double xv = sX[p];
#pragma unroll
        for (int u = 0; u < U; ++u) acc[u] = fma(col[rows[u]], xv, acc[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + tid + BT * u;
      if (i < m) r[i] = acc[u] - b[i];
    }
  }
  __syncthreads();
}

__device__ inline void wg_resid(const double* A, int lda, int m, const double* b, const int32_t* Flist, int nF,
                                const double* x, double* r, int32_t* sF, double* sX) {
  if (m <= BT) wg_resid_rows<1, 32>(A, lda, m, b, Flist, nF, x, r, sF, sX);
  else if (m <= 2 * BT) wg_resid_rows<2, 16>(A, lda, m, b, Flist, nF, x, r, sF, sX);
  else wg_resid_rows<4, 8>(A, lda, m, b, Flist, nF, x, r, sF, sX);
}

// Column dot products out_k = a_j^T v over a list of columns j = list[k] (k < cnt; the
// identity when list is null), one wave per CW columns at a time: lane l takes rows
// l + 64 t, and with m <= 64 RQ the lane's entries of v sit in registers and all RQ CW
// loads of a group are in flight at once; longer columns loop over rows.  With check, a
// non-finite entry of A or v is reported (return value 1).  Each dot product is summed
// in a fixed order (four interleaved partial sums, then a fixed tree).
__device__ inline double wave_tree(double s) {
  for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
  return s;
}

template <int RQ, int CW>
__device__ __noinline__ int wg_atr_reg(const double* __restrict__ A, int lda, int m, const double* v,
                                       const int32_t* list, int cnt, double* out, bool check) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const gcdp Ag = gl(A);
  double vr[RQ];
  int rows[RQ];
  bool bad = false;
#pragma unroll
  for (int t = 0; t < RQ; ++t) {
    const int q = lane + 64 * t;
    rows[t] = min(q, m - 1);
    vr[t] = q < m ? v[q] : 0.0;
    if (check && !isfinite(vr[t])) bad = true;
  }
  for (int k0 = w * CW; k0 < cnt; k0 += (BT / 64) * CW) {
    int js[CW];
#pragma unroll
    for (int c = 0; c < CW; ++c) {
      const int k = min(k0 + c, cnt - 1);   // past cnt: a repeat of the last column, not stored
      js[c] = list ? list[k] : k;
    }
    double a[CW][RQ];
#pragma unroll
    for (int c = 0; c < CW; ++c) {
      const gcdp col = Ag + (int64_t)js[c] * lda;
#pragma unroll
      for (int t = 0; t < RQ; ++t) a[c][t] = col[rows[t]];
    }
#pragma unroll
    for (int c = 0; c < CW; ++c) {
      double s[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int t = 0; t < RQ; ++t) {
        if (check && !isfinite(a[c][t])) bad = true;
        s[t & 3] = fma(a[c][t], vr[t], s[t & 3]);   // vr = 0 past m
      }
      const double tot = wave_tree((s[0] + s[1]) + (s[2] + s[3]));
      if (lane == 0 && k0 + c < cnt) out[k0 + c] = tot;
    }
  }
  __syncthreads();
  return bad ? 1 : 0;
}

__device__ __noinline__ int wg_atr_loop(const double* __restrict__ A, int lda, int m, const double* v,
                                        const int32_t* list, int cnt, double* out, bool check) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  bool bad = false;
  if (check)
    for (int q = threadIdx.x; q < m; q += BT)
      if (!isfinite(v[q])) bad = true;
  for (int k = w; k < cnt; k += BT / 64) {
    const double* col = A + (int64_t)(list ? list[k] : k) * lda;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    int q = lane;
    for (; q + 192 < m; q += 256) {
      double a[4], vv[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        a[t] = col[q + 64 * t];
        vv[t] = v[q + 64 * t];
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        if (check && !isfinite(a[t])) bad = true;
        s[t] = fma(a[t], vv[t], s[t]);
      }
    }
    for (; q < m; q += 64) {
      const double a = col[q];
      if (check && !isfinite(a)) bad = true;
      s[0] = fma(a, v[q], s[0]);
    }
    const double tot = wave_tree((s[0] + s[1]) + (s[2] + s[3]));
    if (lane == 0) out[k] = tot;
  }
  __syncthreads();
  return bad ? 1 : 0;
}

__device__ inline int wg_atr(const double* A, int lda, int m, const double* v, const int32_t* list, int cnt,
                             double* out, bool check) {
  if (m <= 256) return wg_atr_reg<4, 8>(A, lda, m, v, list, cnt, out, check);
  if (m <= 512) return wg_atr_reg<8, 4>(A, lda, m, v, list, cnt, out, check);
  if (m <= 1024) return wg_atr_reg<16, 2>(A, lda, m, v, list, cnt, out, check);
  return wg_atr_loop(A, lda, m, v, list, cnt, out, check);
}

// y_G = A_G^T r over the G list into gpos (by G position), then scattered to y; y_F = 0
__device__ inline void wg_dual(const double* A, int lda, int m, int n, const double* r, const uint8_t* flags,
                               const int32_t* Glist, int nF, double* gpos, double* y) {
  const int nG = n - nF;
  wg_atr(A, lda, m, r, Glist, nG, gpos, false);
  for (int k = threadIdx.x; k < nG; k += BT) y[Glist[k]] = gpos[k];
  for (int i = threadIdx.x; i < n; i += BT)
    if (flags[i]) y[i] = 0.0;
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

// First kernel of a batched solve, one workgroup of GT threads per problem: for
// n <= GS_MAXN the Gram matrix streamed on MFMA (float32 for the mixed path) with
// c = A^T b and the finiteness check of A and b in the same pass; the problem's status
// says whether it was rejected.  Larger problems only get their status cleared here: the
// pivoting kernel forms their c and Gram matrix itself.  On its own, so that the Gram
// passes run eight waves per CU with their own register budget while the pivoting kernel
// keeps two workgroups of four waves.
__global__ __launch_bounds__(GT, 1) void k_batched_gram(BatchArgs a) {
  __shared__ __attribute__((aligned(16))) char smem[GS_LDS_BYTES];
  const int tid = threadIdx.x;
  const int pi = a.order ? a.order[blockIdx.x] : (int)blockIdx.x;
  if (pi >= a.count) return;
  const BatchProblem P = a.probs[pi];
  const int m = P.m, n = P.n;
  const WsLayout Lw = ws_layout(m, n);
  char* base = P.ws;
  BatchInfo* info = P.info;
  int bad = 0;
  if (n <= GS_MAXN) {
    double* c = (double*)(base + Lw.c);
    if (a.fp32)
      bad = wg_gram_stream<float>(P.A, P.lda, m, n, P.b, (float*)(base + Lw.H), c, (float*)smem, a.gram_variant);
    else
      bad = wg_gram_stream<double>(P.A, P.lda, m, n, P.b, (double*)(base + Lw.H), c, (double*)smem, a.gram_variant);
  }
  if (tid == 0) {   // every field: the status array may hold an earlier launch's values
    info->status = bad ? NNLS_ERR_INVALID_VALUE : 0;
    info->iterations = 0;
    info->n_free = 0;
    info->last_ninf = 0;
    info->failed_index = bad ? -1 : INT32_MAX;
    info->ir_steps = 0;
    info->done = bad ? 1 : 0;
    info->min_margin = 0.0;
    ((BatchState*)(base + Lw.state))->started = 0;
  }
}

constexpr size_t SMEM_BYTES = 2 * TILE * LDT * 8;

__global__ __launch_bounds__(BT, 2) void k_batched(BatchArgs a) {
  // two staged 64 x 64 tiles, or the staged F columns and x values of the residual
  __shared__ __attribute__((aligned(16))) char smem[SMEM_BYTES];
  __shared__ double red[8];
  __shared__ double part[4 * TILE];
  __shared__ double vec[TILE];
  __shared__ int s_int[8];
  double* S64 = (double*)smem;
  double* W64 = S64 + TILE * LDT;
  int32_t* sF = (int32_t*)W64;
  double* sX = S64;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int pi = a.order ? a.order[blockIdx.x] : (int)blockIdx.x;
  if (pi >= a.count) return;
  const BatchProblem P = a.probs[pi];
  BatchInfo* info = P.info;
  if (info->done) return;   // finished in an earlier launch, or rejected by k_batched_gram
  const int m = P.m, n = P.n;
  const WsLayout Lw = ws_layout(m, n);
  char* base = P.ws;
  double* H = (double*)(base + Lw.H);
  double* c = (double*)(base + Lw.c);
  double* r = (double*)(base + Lw.r);
  uint8_t* flags = (uint8_t*)(base + Lw.flags);
  int32_t* Flist = (int32_t*)(base + Lw.Flist);
  int32_t* Glist = (int32_t*)(base + Lw.Glist);
  double* z = (double*)(base + Lw.z);
  double* xF = (double*)(base + Lw.xF);
  double* gpos = (double*)(base + Lw.g);
  BatchState* state = (BatchState*)(base + Lw.state);
  double* x = P.x;
  double* y = P.y;
  int32_t* status = &info->status;
  int32_t* failed_pos = &info->failed_index;

  const int max_iter = a.max_iter > 0 ? a.max_iter : 5 * n + 100;
  int N, p, iter, nF, k = 0, result = 0;
  bool h64;
  if (!state->started) {
    // for n <= GS_MAXN k_batched_gram has formed c and the Gram matrix (float32 for the
    // mixed path); larger problems do both here, the finiteness check too
    h64 = !(a.fp32 && n <= GS_MAXN);
    if (n > GS_MAXN) {
      const int bad = wg_atr(P.A, P.lda, m, P.b, nullptr, n, c, true);
      if (wg_max((double)bad, red) > 0.0) {
        if (tid == 0) {
          info->status = NNLS_ERR_INVALID_VALUE;
          info->failed_index = -1;
          info->done = 1;
        }
        return;
      }
      wg_gram(P.A, P.lda, m, n, H, S64, W64);
    }
    for (int i = tid; i < n; i += BT) {
      x[i] = 0.0;
      y[i] = -c[i];
      flags[i] = 0;
    }
    __syncthreads();
    N = INT32_MAX;
    p = a.p_max;
    iter = 0;
    nF = 0;
  } else {
    N = state->N;
    p = state->p;
    iter = state->iter;
    nF = state->nF;
    h64 = state->h64 != 0;
  }
  int steps = 0;
  bool finished = true;
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
    if (a.max_steps > 0 && steps >= a.max_steps) {   // suspend here; the next launch classifies again
      finished = false;
      break;
    }
    ++steps;
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
      else if (i < n) Glist[i - (off + pre + below)] = i;   // i minus the free indices below it
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
        if (!use32 && !h64) {   // float64 factor after a float32 failure: float64 Gram first
          wg_gram(P.A, P.lda, m, n, H, S64, W64);
          h64 = true;
        }
        if (use32 && h64)
          wg_factor<float, double>(H, n, Flist, nF, (float*)(base + Lw.Lt), (float*)(base + Lw.Dv),
                                   (float*)S64, (float*)W64, rep);
        else if (use32)
          wg_factor<float, float>((const float*)H, n, Flist, nF, (float*)(base + Lw.Lt), (float*)(base + Lw.Dv),
                                  (float*)S64, (float*)W64, rep);
        else
          wg_factor<double, double>(H, n, Flist, nF, (double*)(base + Lw.Lt), (double*)(base + Lw.Dv), S64, W64,
                                    rep);
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
        // float64 refinement of x_F against the residual from A: r = A_F x_F - b and
        // g = A_F^T r over the free columns only, the correction from the float32 factor
        bool converged = false;
        double prev = INFINITY;
        for (int step = 0; step < a.ir_max_steps; ++step) {
          wg_resid(P.A, P.lda, m, P.b, Flist, nF, x, r, sF, sX);
          wg_atr(P.A, P.lda, m, r, Flist, nF, gpos, false);
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
          if (dm <= a.ir_rtol * xm) {
            converged = true;
            break;
          }
          if (rho > 0.5) break;
          prev = dm;
        }
        if (converged) {   // y_G from the refined x (Eq. 5)
          wg_resid(P.A, P.lda, m, P.b, Flist, nF, x, r, sF, sX);
          wg_dual(P.A, P.lda, m, n, r, flags, Glist, nF, gpos, y);
          y_done = true;
        } else {
          use32 = false;   // not refined to the target: redo in float64
        }
      }
      __syncthreads();
      if (*status != 0) {
        result = *status;
        break;
      }
    }
    if (!y_done) {
      if (a.gram_dual) {   // H is float64 here: the mixed path reaches this only after a float64 factor
        wg_dual_gram(H, n, c, flags, Flist, nF, x, y);
      } else {
        wg_resid(P.A, P.lda, m, P.b, Flist, nF, x, r, sF, sX);
        wg_dual(P.A, P.lda, m, n, r, flags, Glist, nF, gpos, y);
      }
    }
  }
  __syncthreads();
  if (tid == 0) {
    if (!finished) {
      state->started = 1;
      state->N = N;
      state->p = p;
      state->iter = iter;
      state->nF = nF;
      state->h64 = h64 ? 1 : 0;
    } else {
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
      info->done = 1;
    }
  }
}

}  // namespace

size_t batched_workspace_bytes(int m, int n) { return ws_layout(m, n).total; }

void launch_batched_gram(hipStream_t s, const BatchArgs& a, int grid) {
  if (grid <= 0) return;
  hipLaunchKernelGGL(k_batched_gram, dim3(grid), dim3(GT), 0, s, a);
}

void launch_batched_steps(hipStream_t s, const BatchArgs& a, int grid) {
  if (grid <= 0) return;
  hipLaunchKernelGGL(k_batched, dim3(grid), dim3(BT), 0, s, a);
}

void launch_batched(hipStream_t s, const BatchArgs& a, int grid) {
  BatchArgs whole = a;
  whole.max_steps = 0;
  launch_batched_gram(s, whole, grid);
  launch_batched_steps(s, whole, grid);
}

}  // namespace nnls
