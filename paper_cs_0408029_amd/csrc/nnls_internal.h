// Internal declarations shared by the HIP translation units of the NNLS library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/nnls.h"

namespace nnls {

constexpr int TILE = 64;          // Cholesky / triangular-solve tile edge
constexpr int TILE_ELEMS = TILE * TILE;

// Device-resident control block of one solve.  Written by the pivot-control kernel and by
// the factorisation kernels; read back by the host once per pivot iteration.
struct Ctrl {
  int32_t k;           // infeasible count of the last classify step
  int32_t branch;      // exchange branch taken (-1 when k == 0)
  int32_t rmax;        // largest infeasible index
  int32_t N;           // best infeasible count so far (INT32_MAX = infinity)
  int32_t p;           // remaining non-improving block exchanges
  int32_t iter;        // pivot iterations done
  int32_t n_free;      // |F| after the exchange
  int32_t done;        // 1: feasible split reached, or stop
  int32_t status;      // nnls_status raised on the device (NOT_PD, DEVICE, MAXITER)
  int32_t failed_pos;  // first non-positive pivot position in F (INT32_MAX: none)
  int32_t abort;       // set when a device-side wait exceeds its bound
  int32_t chol_ticket; // work-queue counters of the dataflow kernels
  int32_t fwd_ticket;
  int32_t bwd_ticket;
  int32_t j0;          // leading tile columns of the previous factor that the new F order keeps
  int32_t fwd_walked;  // steps the forward-solve walker has finished (a hint for its helpers)
  double min_margin;   // smallest |v| over the tested entries that were not zeroed
  double ir_dmax;      // mixed precision: max |correction| of the last refinement step
  double ir_xmax;      //                  max |x_F| after it
  double ir_dprev;     //                  max |correction| of the step before (INF: none)
  double ir_err;       //                  bound on max |x_F - exact| after the last step
                       //                  (INF while the contraction is not measured)
  int32_t ir_uncert;   //                  tested entries whose sign the bounds do not
                       //                  certify (-1: no bound yet)
  int32_t bwd_walked;  // the same for the backward solve
};

// Lower-triangle Gram matrix in padded CSC: column j occupies
// [hptr[j], hptr[j] + hcnt[j]) of hrow / hval, rows ascending and >= j.  After the mirror
// step the same region continues with the upcnt[j] entries of rows < j, in no particular
// order, so that [hptr[j], hptr[j] + hcnt[j] + upcnt[j]) is the whole column.
struct GramLower {
  const int64_t* hptr;
  const int32_t* hcnt;
  const int32_t* hrow;
  const double* hval;
};

// The F-block of the Gram matrix in F-position space, rebuilt for every new F order:
// position q keeps the entries (p, H_{F_p F_q}) with p >= q, p ascending, at
// [pptr[F_q], pptr[F_q] + pcnt[q]) of prow / pval (the Gram column's own region size).
struct GramPos {
  const int64_t* pptr;
  const int32_t* pcnt;
  const int32_t* prow;
  const double* pval;
};

// Tile index of lower tile (I, J), I >= J, in row-major packed order.  The index does not
// depend on the number of tile rows, so the leading tiles of a factor stay in place when
// the F-block grows or shrinks behind them.
__host__ __device__ inline int64_t tile_index(int I, int J) { return (int64_t)I * (I + 1) / 2 + J; }
__host__ __device__ inline int64_t tile_count(int nb) { return (int64_t)nb * (nb + 1) / 2; }
// Tiles a factor with j0 reused leading tile columns computes: rows I >= max(J, j0).
__host__ __device__ inline int64_t tile_count_from(int nb, int j0) {
  return (int64_t)j0 * (nb - j0) + tile_count(nb - j0);
}
// Units of work of a factor launch.  The diagonal and sub-diagonal tiles of a computed
// column (the walker's inputs) are single units; the other off-diagonal tiles are taken in
// strips of RS rows of one column, or -- with pairs -- in strips of RP rows of two adjacent
// columns, whose second column is finished after the first.  Columns are grouped from the
// start of the kept (J < j0) and of the computed (J >= j0) range, two at a time with pairs
// (an odd last column alone).  A group's units, in ticket order:
//   computed single J:      (J, J), (J+1, J), strips of rows J+2 ..
//   computed pair (J, J+1): (J, J), (J+1, J), (J+2, J) alone, (J+1, J+1), (J+2, J+1),
//                           pair strips of rows J+3 ..
//   kept single or pair:    strips or pair strips of rows j0 ..
// Every unit waits only for units of earlier groups, earlier units of its own group and the
// walker (ticket 0), which are running or done.  RS = 1 without pairs is one tile per unit,
// in the column-major order of tile_count_from.
enum { UNIT_TILE = 0, UNIT_STRIP = 1, UNIT_PAIR = 2 };
struct FactorUnit {
  int kind, I, J, cnt;   // cnt rows I .. I + cnt - 1 of column J (and J + 1 for a pair)
};
struct UnitPlan {
  int nb, j0, RS, RP;
  bool pairs;
  bool kept_single = false;   // kept columns in one-column strips (the row walkers' partial tiles)
};
__host__ __device__ inline int strips_of(int rows, int R) { return rows > 0 ? (rows + R - 1) / R : 0; }
__host__ __device__ inline int group_span(int J, const UnitPlan& p) {
  const int end = J < p.j0 ? p.j0 : p.nb;
  return (p.pairs && J + 1 < end && !(J < p.j0 && p.kept_single)) ? 2 : 1;
}
__host__ __device__ inline int group_units(int J, int C, const UnitPlan& p) {
  if (J < p.j0) return strips_of(p.nb - p.j0, C == 2 ? p.RP : p.RS);
  if (C == 1) return 1 + (J + 1 < p.nb ? 1 : 0) + strips_of(p.nb - J - 2, p.RS);
  const int third = J + 2 < p.nb ? 1 : 0;
  return 3 + 2 * third + strips_of(p.nb - J - 3, p.RP);
}
__host__ __device__ inline int64_t unit_total(const UnitPlan& p) {
  int64_t u = 0;
  for (int J = 0; J < p.nb;) {
    const int C = group_span(J, p);
    u += group_units(J, C, p);
    J += C;
  }
  return u;
}
__host__ __device__ inline FactorUnit unit_at(int64_t t, const UnitPlan& p) {
  int J = 0, C = group_span(0, p);
  for (int64_t u = group_units(0, C, p); t >= u; u = group_units(J, C, p)) {
    t -= u;
    J += C;
    C = group_span(J, p);
  }
  FactorUnit f;
  f.J = J;
  f.cnt = 1;
  if (J < p.j0) {
    const int R = C == 2 ? p.RP : p.RS;
    f.kind = C == 2 ? UNIT_PAIR : UNIT_STRIP;
    f.I = p.j0 + (int)t * R;
    f.cnt = p.nb - f.I < R ? p.nb - f.I : R;
    return f;
  }
  f.kind = UNIT_TILE;
  if (C == 1) {
    if (t == 0) {
      f.I = J;
      return f;
    }
    if (t == 1 && J + 1 < p.nb) {
      f.I = J + 1;
      return f;
    }
    t -= J + 1 < p.nb ? 2 : 1;
    f.kind = UNIT_STRIP;
    f.I = J + 2 + (int)t * p.RS;
    f.cnt = p.nb - f.I < p.RS ? p.nb - f.I : p.RS;
    return f;
  }
  const bool third = J + 2 < p.nb;
  if (t < 2) {   // (J, J), (J+1, J)
    f.I = J + (int)t;
    return f;
  }
  t -= 2;
  if (third) {
    if (t == 0) {   // (J+2, J) alone: the next column's sub-diagonal tile reads it
      f.kind = UNIT_STRIP;
      f.I = J + 2;
      return f;
    }
    t -= 1;
  }
  if (t == 0) {   // (J+1, J+1)
    f.I = J + 1;
    f.J = J + 1;
    return f;
  }
  t -= 1;
  if (third) {
    if (t == 0) {   // (J+2, J+1)
      f.I = J + 2;
      f.J = J + 1;
      return f;
    }
    t -= 1;
  }
  f.kind = UNIT_PAIR;
  f.I = J + 3 + (int)t * p.RP;
  f.cnt = p.nb - f.I < p.RP ? p.nb - f.I : p.RP;
  return f;
}
constexpr int CHOL_STRIP = 4;   // rows per one-column strip of the bfloat16-update factor
constexpr int CHOL_PAIR = 3;    // rows per two-column strip

// ---------------------------------------------------------------- launchers
// setup (k_setup.hip)
void launch_validate_csc(hipStream_t s, int m, int n, int64_t nnz, const int32_t* colptr,
                         const int32_t* rowidx, const double* val, const double* b, int32_t* err);
void launch_validate_dense(hipStream_t s, int m, int n, const double* A, int lda, const double* b,
                           int32_t* err);
// scan_scratch: 8 * ceil(max(m, n) / 2048) bytes of device scratch for the prefix sums
void launch_build_csr(hipStream_t s, int m, int n, int64_t nnz, const int32_t* colptr,
                      const int32_t* rowidx, const double* val, int32_t* rowcnt, int32_t* rowptr,
                      int32_t* colidx, double* valr, void* scan_scratch);
void launch_gram_bound(hipStream_t s, int n, const int32_t* colptr, const int32_t* rowidx,
                       const int32_t* rowptr, int64_t* hptr, void* scan_scratch);
void launch_gram_lower(hipStream_t s, int n, const int32_t* colptr, const int32_t* rowidx,
                       const double* val, const int32_t* rowptr, const int32_t* colidx,
                       const double* valr, const int64_t* hptr, int32_t* hcnt, int32_t* hrow,
                       double* hval);
// append the strictly lower entries of every column as the upper entries of their row's
// column (upcnt zero on entry)
void launch_gram_mirror(hipStream_t s, int n, GramLower g, int32_t* upcnt, int32_t* hrow, double* hval);
// position-space lists of the F-block for the current F order (Flist, pos)
void launch_gram_positions(hipStream_t s, int nF, GramLower g, const int32_t* upcnt,
                           const int32_t* Flist, const int32_t* pos, int32_t* pcnt, int32_t* prow,
                           double* pval);
void launch_spmvT_csc(hipStream_t s, int n, const int32_t* colptr, const int32_t* rowidx,
                      const double* val, const double* v, double* out, double scale);
void launch_gram_dense(hipStream_t s, int m, int n, const double* A, int lda, double* H, int ldh);
void launch_gemvT_dense(hipStream_t s, int m, int n, const double* A, int lda, const double* v,
                        double* out, double scale);
void launch_lower_to_dense(hipStream_t s, int n, GramLower g, double* H, int ldh);
void launch_fill(hipStream_t s, double* p, int64_t count, double v);
void launch_fill_i32(hipStream_t s, int32_t* p, int64_t count, int32_t v);
void launch_fill_2d(hipStream_t s, int rows, int cols, double* p, int ld, double v);

// pivot control (k_pivot.hip)
void launch_pivot_init(hipStream_t s, int n, const double* c, double* x, double* y,
                       uint8_t* flags, Ctrl* ctrl, int p_max);
// reuse: the tiles of the factor of the current F order are valid for the next factor of
// the same precision; Fold: n ints of scratch
void launch_pivot_control(hipStream_t s, int n, double* x, double* y, uint8_t* flags,
                          int32_t* Flist, int32_t* pos, Ctrl* ctrl, double tau, int p_max,
                          int max_iter, int32_t* colcnt, int ncol, int32_t* Fold, int reuse);
void launch_ctrl_set_state(hipStream_t s, Ctrl* ctrl, int N, int p, int iter, int max_iter_flag);

// residual and dual (k_spmv.hip)
void launch_residual_csr(hipStream_t s, int m, int64_t nnz, const int32_t* rowptr, const int32_t* colidx,
                         const double* valr, const double* x, const double* b, double* r);
void launch_dual_csc(hipStream_t s, int n, const int32_t* colptr, const int32_t* rowidx,
                     const double* val, const double* r, const uint8_t* flags, double* y,
                     double* gfree = nullptr);
void launch_residual_dense(hipStream_t s, int m, int n, const double* A, int lda,
                           const double* x, const double* b, double* r, double* part = nullptr);
// column chunks the dense residual splits into (part needs chunks * m doubles; 1: no split)
int dense_residual_chunks(int m, int n);
void launch_dual_dense(hipStream_t s, int m, int n, const double* A, int lda, const double* r,
                       const uint8_t* flags, double* y, double* gfree = nullptr);
// y_G = H_GF x_F - c_G from a dense symmetric H (Eq. 3), y_F = 0
void launch_dual_gram_dense(hipStream_t s, int n, const double* H, int64_t ldh, const double* c,
                            const uint8_t* flags, const int32_t* Flist, int nF, const double* x,
                            double* y);
// Eq. 5 for the refinement, with compensated sums: r = A x - b kept as r_hi + r_lo, then
// y_j = a_j^T r on G and gfree_j = a_j^T r on F, each exact up to one rounding and an
// O((k u)^2) term.  Dense A when A != nullptr (lda), else the CSR copy and the CSC input.
void launch_residual_dual_dd(hipStream_t s, int m, int n, int64_t nnz, const int32_t* rowptr,
                             const int32_t* colidx, const double* valr, const int32_t* colptr,
                             const int32_t* rowidx, const double* val, const double* A, int lda,
                             const double* x, const double* b, const uint8_t* flags, double* rh,
                             double* rl, double* y, double* gfree);
// Gathers sliced for the L2 (k_slice.hip): slices of 2^SLICE_SHIFT elements (2 MB of
// doubles) of the gathered vector; used when that vector is longer than SLICE_MIN_LEN
// (larger than an XCD's 4 MB L2).
constexpr int SLICE_SHIFT = 18;
constexpr int SLICE_MIN_LEN = 1 << 19;
inline int slice_count(int len) { return (int)(((int64_t)len + (1 << SLICE_SHIFT) - 1) >> SLICE_SHIFT); }
// Copy a compressed matrix (N outputs, ptr[N + 1], ascending idx per output, values) slice
// by slice: sptr (ns (N + 1) + 1 ints) gives output o's run in slice s at
// [sptr[s (N + 1) + o], sptr[s (N + 1) + o + 1]); sidx, sval (nnz each) hold the runs.
// counts: ns (N + 1) ints of scratch; scan_sums: ceil(ns (N + 1) / 2048) ints.
void launch_slice_build(hipStream_t s, int N, int64_t nnz, const int32_t* ptr, const int32_t* idx,
                        const double* val, int ns, int32_t* counts, int32_t* sptr, int32_t* sidx,
                        double* sval, int32_t* scan_sums);
// r = A x - b over the row-major copy sliced by columns (ns slices of x)
void launch_sliced_residual(hipStream_t s, int m, int ns, const int32_t* sptr, const int32_t* sidx,
                            const double* sval, const double* x, const double* b, double* r);
// y_j = a_j^T r where flags[j] == 0, else 0, over the CSC sliced by rows (ns slices of r)
void launch_sliced_dual(hipStream_t s, int n, int ns, const int32_t* sptr, const int32_t* sidx,
                        const double* sval, const double* r, const uint8_t* flags, double* y);
// exclusive prefix sum of count[0..n) into out[0..n] (k_setup.hip); sums: ceil(n / 2048)
void launch_scan_i32(hipStream_t s, int64_t n, const int32_t* count, int32_t* out, int32_t* sums);
// x[Flist[p]] -= d[p] for p < nF; writes max |d| and max |x_F| into ctrl (one workgroup);
// first: the first step of a refinement (ir_dprev becomes INF, else the previous ir_dmax)
void launch_ir_update(hipStream_t s, int nF, const int32_t* Flist, const double* d, double* x,
                      Ctrl* ctrl, int first);
// Sign certificates of a refinement step (the Sec. 3 remark that intermediate solves need
// only correct signs).  Per pivot iteration, with w_r = sum_{j in F} |a_rj|:
//   bw_j = sum_r |a_rj| w_r  and  bb_j = sum_r |a_rj| |b_r|   for j in G
// (bounds of y_j's sensitivity to an error in x_F and of its rounding error).
void launch_sign_bounds_csr(hipStream_t s, int m, int n, int64_t nnz, const int32_t* rowptr,
                            const int32_t* colidx, const double* valr, const int32_t* colptr,
                            const int32_t* rowidx, const double* val, const uint8_t* flags,
                            const double* b, double* w, double* bw, double* bb);
void launch_sign_bounds_dense(hipStream_t s, int m, int n, const double* A, int lda,
                              const int32_t* Flist, int nF, const uint8_t* flags, const double* b,
                              double* w, double* bw, double* bb);

// After launch_ir_update: while the refinement contracts by 1/2 or better (rho =
// ir_dmax / ir_dprev, measured), the error of x_F is at most e = ir_dmax and that of the x
// the step's y_G was formed from at most 2 ir_dmax.  Counts the tested entries v (x_i on
// F, y_i on G) with |v| >= tau whose distance to the zeroing band does not exceed their
// bound: e (+ rounding) on F; 2 ir_dmax bw_j + 2 u |y_j| + gamma2 (xmax bw_j + bb_j) on G
// (the compensated y_j's rounding).
// Writes ctrl->ir_err and ctrl->ir_uncert (-1 when rho is unknown or above 1/2).
void launch_ir_certify(hipStream_t s, int n, const uint8_t* flags, const double* x, const double* y,
                       const double* bw, const double* bb, double tau, double gamma2, Ctrl* ctrl);

// condition estimate of the final F-block (k_cond.hip)
struct CondEst {
  double hnorm;    // ||H_FF||_1 (set to 0 before the norm kernel)
  double ynorm;    // ||y||_1 of the last EST_SIGNS step
  double zmax;     // max |z| of the last EST_ARGMAX step
  double zjlast;   // |z| at the index chosen before that step
  int32_t j;       // current index (-1: none yet)
  int32_t changed; // EST_SIGNS: some sign differed from the stored ones
};
enum { EST_SET_UNIFORM = 0, EST_SET_UNIT = 1, EST_SET_ALT = 2, EST_SIGNS = 3, EST_ARGMAX = 4 };
void launch_block_onenorm(hipStream_t s, int nF, GramLower g, const int32_t* upcnt, const int32_t* pos,
                          const double* Hd, int64_t ldh, const int32_t* Flist, CondEst* est);
void launch_est_vec(hipStream_t s, int mode, int nF, double* v, const double* y, double* xi, CondEst* est);

// factorisation and triangular solves (k_chol.hip)
struct FactorArgs {
  int nF;                 // order of the F-block
  int nb;                 // ceil(nF / TILE)
  const int32_t* Flist;   // F positions -> column numbers (nullptr: identity)
  GramPos gpos;           // sparse source (used when dense == nullptr)
  const double* dense;    // dense symmetric source, column-major
  int64_t ldd;
  int j0;                 // leading tile columns kept from the previous factor (rows < j0)
  void* Ltiles;           // tile storage, tile_count(nb) tiles of TILE_ELEMS
  void* Dinv;             // nb inverted diagonal tiles
  int32_t* colcnt;        // nb counters of finished tiles per column, zero at launch
  int32_t* tflag;         // tile_count(nb) flags: tile ready when == epoch
  int32_t* dflag;         // nb flags: diagonal tile of column J ready when == epoch
  int epoch;
  Ctrl* ctrl;
  uint64_t wait_ticks;    // bound of one device-side wait, in wall-clock ticks
  const double* rhs;      // optional: forward-solve L z = rhs_F during the factorisation
  double* z;              // nb * TILE, written when rhs != nullptr
  int max_wgs;            // cap on the persistent grid (0: one workgroup per tile and the walker)
  void* Lbf;              // float factor only: bfloat16 row-major copies of the off-diagonal
                          // tiles, which the left-looking updates then read (NNLS_BF16_IR);
                          // nullptr: the updates read the float tiles
  void* Mc;               // optional: the triangular solves' coupling tiles, formed after the
                          // factor (walk_coupling_bytes; nullptr: not formed)
  int rowwalk;            // set by launch_cholesky: the new tile rows below a kept block are
                          // finished by row walkers from the previous factor's coupling tiles
};
// Newest terms the walker of the triangular solves adds itself each step.  The factor's
// coupling tiles hold them premultiplied by the inverted diagonal tile, in the factor's
// precision and in the walker's thread order: forward D_I L_{I,I-j}, backward
// D_I^T L_{I+j,I}^T, j = 1 .. TD, at ((dir * nb + I) * TD + j - 1) * TILE_ELEMS (dir 0
// forward, 1 backward).
template <typename T> struct WalkTD { static constexpr int value = sizeof(T) == 4 ? 3 : 2; };
inline size_t walk_coupling_bytes(int nb, bool fp32) {
  return fp32 ? 2 * (size_t)WalkTD<float>::value * nb * TILE_ELEMS * sizeof(float)
              : 2 * (size_t)WalkTD<double>::value * nb * TILE_ELEMS * sizeof(double);
}
void launch_cholesky(hipStream_t s, const FactorArgs& a, bool fp32);
// z = L^-1 rhs (rhs gathered through Flist when gather != nullptr); x = L^-T z and
// scatter x through Flist into out (when out != nullptr) and into xF.
// Both 32-bit halves of an empty hand-over slot of the triangular solves (a signalling-NaN
// bit pattern, which no arithmetic result has); a buffer of slots is emptied by filling
// it with this word.
constexpr int32_t SLOT_EMPTY_WORD = 0x7FF4A5A5;

struct SolveArgs {
  int nF, nb;
  const int32_t* Flist;
  const void* Ltiles;
  const void* Dinv;
  const double* rhs_full;   // indexed by column number (through Flist) ...
  const double* rhs_dense;  // ... or by F position (used when rhs_full == nullptr)
  double* z;                // nb * TILE
  double* xF;               // nb * TILE
  double* out;              // optional scatter target, indexed by column number
  int epoch;
  Ctrl* ctrl;
  uint64_t wait_ticks;
  double* part;             // 2 * nb * TILE hand-over slots, empty (every 32-bit word
                            // SLOT_EMPTY_WORD) between launches: [0, nb * TILE) the helpers'
                            // partial sums, [nb * TILE, 2 nb * TILE) the walker's outputs
  const void* Lbf;          // float factor only: the bfloat16 copies of its off-diagonal tiles,
                            // read instead of the float tiles (nullptr: the float tiles)
  const void* Mc;           // the factor's coupling tiles (FactorArgs::Mc), formed after it
};
void launch_trsv(hipStream_t s, const SolveArgs& a, bool fp32, bool forward);
// The coupling tiles of a factor (FactorArgs::Mc), in bfloat16 for a factor with bfloat16
// updates; launch_cholesky calls it after the factor when Mc is set.
void launch_walk_couplings(hipStream_t s, int nb, const void* Ltiles, const void* Dinv, void* Mc, bool fp32,
                           bool bf16);
void launch_tiles_to_dense(hipStream_t s, int n, const void* Ltiles, bool fp32, double* L, int ldl);
void launch_reset_tickets(hipStream_t s, Ctrl* ctrl);

// batched dense problems (k_batched.hip): one workgroup per problem
struct BatchInfo {
  int32_t status, iterations, n_free, last_ninf, failed_index, ir_steps;
  int32_t done;           // finished (any status); 0 while the pivot loop is suspended
  int32_t pad;
  double min_margin;
};
struct BatchProblem {
  int32_t m, n, lda, pad;
  const double* A;
  const double* b;
  double* x;
  double* y;
  BatchInfo* info;        // the problem's result and status, kept across launches
  char* ws;               // the problem's workspace (batched_workspace_bytes), 256-byte aligned
};
constexpr int GS_NR = 8;         // the streamed Gram kernel takes n <= 32 GS_NR
constexpr int GS_VARIANTS = 3;   // its accumulator tile shapes (k = 0, 1, 2; 1 the default)
struct BatchArgs {
  int count;
  const BatchProblem* probs;
  const int32_t* order;   // launch order (workgroup b solves problem order[b]); may be null
  double tau;
  int p_max;
  int max_iter;           // <= 0: 5 n + 100 per problem
  int fp32;               // float32 factor + float64 refinement
  int ir_max_steps;
  double ir_rtol;
  int gram_dual;          // y_G from the cached Gram matrix (Eq. 3) instead of Eq. 5
  int max_steps;          // pivot iterations per launch of the pivoting kernel; <= 0: all
  uint8_t gram_variant[GS_NR + 1];   // Gram kernel tile shape by ceil(n / 32): 0 default, 1 + k shape k
};
size_t batched_workspace_bytes(int m, int n);
// Whole solves: the Gram kernel, then the pivoting kernel until every problem is done.
void launch_batched(hipStream_t s, const BatchArgs& a, int grid);
// The two kernels on their own: the Gram kernel starts problems (c, Gram matrix, status,
// fresh pivot state); the pivoting kernel runs up to a.max_steps pivot iterations of every
// problem that is not done yet and suspends the others at their next classify step.
void launch_batched_gram(hipStream_t s, const BatchArgs& a, int grid);
void launch_batched_steps(hipStream_t s, const BatchArgs& a, int grid);
void launch_ctrl_clear_breakdown(hipStream_t s, Ctrl* ctrl);   // NOT_PD -> 0 (mixed retry)

// One request packed into a single block (host staging and device copy share the layout):
// colptr int32[n+1] | rowidx int32[nnz] | val double[nnz] | b double[m], 8-byte aligned.
struct PackLayout {
  int64_t rowidx, val, b, total;
};
__host__ __device__ inline PackLayout pack_layout(int m, int n, int64_t nnz) {
  PackLayout L;
  L.rowidx = ((int64_t)(n + 1) * 4 + 7) / 8 * 8;
  L.val = (L.rowidx + nnz * 4 + 7) / 8 * 8;
  L.b = L.val + nnz * 8;
  L.total = (L.b + (int64_t)m * 8 + 255) / 256 * 256;
  return L;
}
// Scatter packed CSC requests into zero-filled dense column-major blocks (lda = m).
struct ScatterDesc {
  int32_t m, n;
  int64_t nnz;
  int64_t in_off;   // byte offset of the packed block
  int64_t a_off;    // element offset of the dense block
};
void release_workspace(::nnls_handle* h);   // api.hip: free the handle's device buffers
void launch_csc_scatter(hipStream_t s, int count, const ScatterDesc* desc, const char* packed,
                        double* dense);

}  // namespace nnls
