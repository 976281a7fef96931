// Stand-ins for the library's kernel launchers, for the host-only sanitizer build.  Each
// enqueues a task on its stream that reads every input element and writes every output
// element the real kernel would (so the address sanitizer checks the sizes the host code
// allocates), and drives the pivot loop through a short fixed trajectory: two exchanges
// (F = every second, then every third column), each solve refined to convergence at once,
// then a feasible split.  No arithmetic of the method is reproduced.
#include <cmath>
#include <cstring>
#include <vector>

#include "../../paper_cs_0408029_amd/csrc/nnls_internal.h"
#include "stub_runtime.h"

namespace nnls {

namespace {
// Keep reads from being optimised away (one per stream worker thread).
thread_local volatile double g_sink = 0.0;
template <typename T>
void read_all(const T* p, int64_t count) {
  double s = 0.0;
  for (int64_t i = 0; i < count; ++i) s += (double)p[i];
  g_sink = g_sink + s;
}
void read_bytes(const void* p, int64_t bytes) { read_all((const unsigned char*)p, bytes); }
void write_bytes(void* p, int64_t bytes) { std::memset(p, 0, (size_t)bytes); }
int64_t nb_of(int nF) { return (nF + TILE - 1) / TILE; }
}  // namespace

void launch_validate_csc(hipStream_t s, int m, int n, int64_t nnz, const int32_t* colptr, const int32_t* rowidx,
                         const double* val, const double* b, int32_t* err) {
  stub_enqueue(s, [=] {
    read_all(colptr, n + 1);
    read_all(rowidx, nnz);
    read_all(val, nnz);
    read_all(b, m);
    for (int i = 0; i < 4; ++i) err[i] = 0;
  });
}

void launch_validate_dense(hipStream_t s, int m, int n, const double* A, int lda, const double* b, int32_t* err) {
  stub_enqueue(s, [=] {
    for (int j = 0; j < n; ++j) read_all(A + (int64_t)j * lda, m);
    read_all(b, m);
    for (int i = 0; i < 4; ++i) err[i] = 0;
  });
}

void launch_build_csr(hipStream_t s, int m, int n, int64_t nnz, const int32_t* colptr, const int32_t* rowidx,
                      const double* val, int32_t* rowcnt, int32_t* rowptr, int32_t* colidx, double* valr,
                      void* scan_scratch) {
  stub_enqueue(s, [=] {
    write_bytes(scan_scratch, 8 * ((int64_t)(m > n ? m : n) / 2048 + 1));
    for (int i = 0; i < m; ++i) rowcnt[i] = 0;
    for (int64_t e = 0; e < nnz; ++e) rowcnt[rowidx[e]] += 1;
    rowptr[0] = 0;
    for (int i = 0; i < m; ++i) rowptr[i + 1] = rowptr[i] + rowcnt[i];
    std::vector<int32_t> fill(rowptr, rowptr + m);
    for (int j = 0; j < n; ++j)
      for (int32_t e = colptr[j]; e < colptr[j + 1]; ++e) {
        const int32_t q = fill[rowidx[e]]++;
        colidx[q] = j;
        valr[q] = val[e];
      }
  });
}

void launch_gram_bound(hipStream_t s, int n, const int32_t* colptr, const int32_t* rowidx, const int32_t* rowptr,
                       int64_t* hptr, void* scan_scratch) {
  stub_enqueue(s, [=] {
    read_all(rowidx, colptr[n]);
    read_bytes(scan_scratch, 8);
    (void)rowptr;
    hptr[0] = 0;
    for (int j = 0; j < n; ++j) hptr[j + 1] = hptr[j] + 2 * (colptr[j + 1] - colptr[j]) + 2;
  });
}

void launch_gram_lower(hipStream_t s, int n, const int32_t* colptr, const int32_t* rowidx, const double* val,
                       const int32_t* rowptr, const int32_t* colidx, const double* valr, const int64_t* hptr,
                       int32_t* hcnt, int32_t* hrow, double* hval) {
  stub_enqueue(s, [=] {
    read_all(val, colptr[n]);
    read_all(rowidx, colptr[n]);
    (void)rowptr;
    (void)colidx;
    (void)valr;
    for (int j = 0; j < n; ++j) {
      const int64_t len = hptr[j + 1] - hptr[j];
      hcnt[j] = (int32_t)(len / 2);
      for (int64_t q = hptr[j]; q < hptr[j + 1]; ++q) {
        hrow[q] = j;
        hval[q] = 1.0;
      }
    }
  });
}

void launch_gram_mirror(hipStream_t s, int n, GramLower g, int32_t* upcnt, int32_t* hrow, double* hval) {
  stub_enqueue(s, [=] {
    for (int j = 0; j < n; ++j) {
      const int64_t len = g.hptr[j + 1] - g.hptr[j];
      upcnt[j] = (int32_t)(len - g.hcnt[j]);
      for (int64_t q = g.hptr[j] + g.hcnt[j]; q < g.hptr[j + 1]; ++q) {
        hrow[q] = j;
        hval[q] = 0.5;
      }
    }
  });
}

void launch_gram_positions(hipStream_t s, int nF, GramLower g, const int32_t* upcnt, const int32_t* Flist,
                           const int32_t* pos, int32_t* pcnt, int32_t* prow, double* pval) {
  stub_enqueue(s, [=] {
    for (int q = 0; q < nF; ++q) {
      const int j = Flist[q];
      (void)pos[j];
      pcnt[q] = g.hcnt[j];
      for (int64_t e = g.hptr[j]; e < g.hptr[j] + g.hcnt[j] + upcnt[j]; ++e) {
        prow[e] = q;
        pval[e] = g.hval[e];
      }
    }
  });
}

void launch_spmvT_csc(hipStream_t s, int n, const int32_t* colptr, const int32_t* rowidx, const double* val,
                      const double* v, double* out, double scale) {
  stub_enqueue(s, [=] {
    for (int j = 0; j < n; ++j) {
      double t = 0.0;
      for (int32_t e = colptr[j]; e < colptr[j + 1]; ++e) t += val[e] * v[rowidx[e]];
      g_sink = g_sink + t;
      out[j] = scale * ((j % 2) ? -1.0 : 1.0);
    }
  });
}

void launch_gram_dense(hipStream_t s, int m, int n, const double* A, int lda, double* H, int ldh) {
  stub_enqueue(s, [=] {
    for (int j = 0; j < n; ++j) read_all(A + (int64_t)j * lda, m);
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) H[i + (int64_t)j * ldh] = (i == j) ? 2.0 : 0.1;
  });
}

void launch_gemvT_dense(hipStream_t s, int m, int n, const double* A, int lda, const double* v, double* out,
                        double scale) {
  stub_enqueue(s, [=] {
    for (int j = 0; j < n; ++j) read_all(A + (int64_t)j * lda, m);
    read_all(v, m);
    for (int j = 0; j < n; ++j) out[j] = scale * ((j % 2) ? -1.0 : 1.0);
  });
}

void launch_lower_to_dense(hipStream_t s, int n, GramLower g, double* H, int ldh) {
  stub_enqueue(s, [=] {
    read_all(g.hcnt, n);
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) H[i + (int64_t)j * ldh] = 0.0;
  });
}

void launch_fill(hipStream_t s, double* p, int64_t count, double v) {
  stub_enqueue(s, [=] {
    for (int64_t i = 0; i < count; ++i) p[i] = v;
  });
}

void launch_fill_i32(hipStream_t s, int32_t* p, int64_t count, int32_t v) {
  stub_enqueue(s, [=] {
    for (int64_t i = 0; i < count; ++i) p[i] = v;
  });
}

void launch_fill_2d(hipStream_t s, int rows, int cols, double* p, int ld, double v) {
  stub_enqueue(s, [=] {
    for (int j = 0; j < cols; ++j)
      for (int i = 0; i < rows; ++i) p[i + (int64_t)j * ld] = v;
  });
}

void launch_pivot_init(hipStream_t s, int n, const double* c, double* x, double* y, uint8_t* flags, Ctrl* ctrl,
                       int p_max) {
  stub_enqueue(s, [=] {
    for (int i = 0; i < n; ++i) {
      x[i] = 0.0;
      y[i] = -c[i];
      flags[i] = 0;
    }
    Ctrl z;
    std::memset(&z, 0, sizeof(z));
    z.N = INT32_MAX;
    z.p = p_max;
    z.branch = -1;
    z.rmax = -1;
    z.failed_pos = INT32_MAX;
    z.min_margin = INFINITY;
    *ctrl = z;
  });
}

void launch_pivot_control(hipStream_t s, int n, double* x, double* y, uint8_t* flags, int32_t* Flist, int32_t* pos,
                          Ctrl* ctrl, double, int, int, int32_t* colcnt, int ncol, int32_t* Fold, int) {
  stub_enqueue(s, [=] {
    read_all(x, n);
    read_all(y, n);
    read_all(flags, n);
    if (ctrl->iter >= 2 || ctrl->status != 0) {
      ctrl->k = 0;
      ctrl->branch = -1;
      ctrl->done = 1;
      return;
    }
    const int step = ctrl->iter + 2;   // F: every second column, then every third
    int nF = 0;
    for (int i = 0; i < n; ++i) {
      const bool f = (i % step) == 0;
      flags[i] = f ? 1 : 0;
      pos[i] = f ? nF : -1;
      if (f) Flist[nF++] = i;
      if (Fold) Fold[i] = i;
      if (f) y[i] = 0.0; else x[i] = 0.0;
    }
    for (int c = 0; c < ncol; ++c) colcnt[c] = 0;
    ctrl->iter += 1;
    ctrl->k = 3;
    ctrl->branch = 0;
    ctrl->N = 3;
    ctrl->n_free = nF;
    ctrl->done = 0;
    ctrl->j0 = 0;
    ctrl->min_margin = 1.0;
    ctrl->chol_ticket = ctrl->fwd_ticket = ctrl->bwd_ticket = 0;
  });
}

void launch_ctrl_set_state(hipStream_t s, Ctrl* ctrl, int N, int p, int iter, int) {
  stub_enqueue(s, [=] {
    Ctrl z;
    std::memset(&z, 0, sizeof(z));
    z.N = N;
    z.p = p;
    z.iter = iter;
    z.failed_pos = INT32_MAX;
    *ctrl = z;
  });
}

void launch_residual_csr(hipStream_t s, int m, int64_t nnz, const int32_t* rowptr, const int32_t* colidx,
                         const double* valr, const double* x, const double* b, double* r) {
  stub_enqueue(s, [=] {
    for (int i = 0; i < m; ++i) {
      double t = -b[i];
      for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) t += valr[e] * x[colidx[e]];
      r[i] = t;
    }
    (void)nnz;
  });
}

void launch_dual_csc(hipStream_t s, int n, const int32_t* colptr, const int32_t* rowidx, const double* val,
                     const double* r, const uint8_t* flags, double* y, double* gfree) {
  stub_enqueue(s, [=] {
    for (int j = 0; j < n; ++j) {
      double t = 0.0;
      for (int32_t e = colptr[j]; e < colptr[j + 1]; ++e) t += val[e] * r[rowidx[e]];
      g_sink = g_sink + t;
      y[j] = flags[j] ? 0.0 : 1.0;
      if (gfree && flags[j]) gfree[j] = 0.0;
    }
  });
}

// Sliced gathers: the copy is built exactly as the device does (counts per slice, a scan,
// a scatter), so the stub touches every range the real kernels touch.
void launch_slice_build(hipStream_t s, int N, int64_t nnz, const int32_t* ptr, const int32_t* idx, const double* val,
                        int ns, int32_t* counts, int32_t* sptr, int32_t* sidx, double* sval, int32_t* scan_sums) {
  stub_enqueue(s, [=] {
    const int64_t ld = (int64_t)N + 1;
    for (int64_t o = 0; o < N; ++o) {
      int32_t q = ptr[o];
      for (int sl = 0; sl < ns; ++sl) {
        const int32_t p0 = q;
        while (q < ptr[o + 1] && (idx[q] >> SLICE_SHIFT) == sl) ++q;
        counts[sl * ld + o] = q - p0;
      }
    }
    for (int sl = 0; sl < ns; ++sl) counts[sl * ld + N] = 0;
    int32_t run = 0;
    for (int64_t k = 0; k < ns * ld; ++k) {
      sptr[k] = run;
      run += counts[k];
    }
    sptr[ns * ld] = run;
    scan_sums[0] = run;
    for (int64_t o = 0; o < N; ++o) {
      int cur = -1;
      int32_t pos = 0;
      for (int32_t q = ptr[o]; q < ptr[o + 1]; ++q) {
        const int sl = idx[q] >> SLICE_SHIFT;
        if (sl != cur) {
          cur = sl;
          pos = sptr[sl * ld + o];
        }
        sidx[pos] = idx[q];
        sval[pos] = val[q];
        ++pos;
      }
    }
    (void)nnz;
  });
}

void launch_sliced_residual(hipStream_t s, int m, int ns, const int32_t* sptr, const int32_t* sidx,
                            const double* sval, const double* x, const double* b, double* r) {
  stub_enqueue(s, [=] {
    const int64_t ld = (int64_t)m + 1;
    for (int i = 0; i < m; ++i) {
      double t = -b[i];
      for (int sl = 0; sl < ns; ++sl)
        for (int32_t e = sptr[sl * ld + i]; e < sptr[sl * ld + i + 1]; ++e) t += sval[e] * x[sidx[e]];
      r[i] = t;
    }
  });
}

void launch_sliced_dual(hipStream_t s, int n, int ns, const int32_t* sptr, const int32_t* sidx,
                        const double* sval, const double* r, const uint8_t* flags, double* y) {
  stub_enqueue(s, [=] {
    const int64_t ld = (int64_t)n + 1;
    for (int j = 0; j < n; ++j) {
      double t = 0.0;
      for (int sl = 0; sl < ns; ++sl)
        for (int32_t e = sptr[sl * ld + j]; e < sptr[sl * ld + j + 1]; ++e) t += sval[e] * r[sidx[e]];
      g_sink = g_sink + t;
      y[j] = flags[j] ? 0.0 : 1.0;
    }
  });
}

int dense_residual_chunks(int m, int n) {
  const int rows = (m + 255) / 256;
  int c = (1024 + rows - 1) / rows;
  const int cmax = (n + 63) / 64;
  if (c > cmax) c = cmax;
  return c < 1 ? 1 : c;
}

void launch_residual_dense(hipStream_t s, int m, int n, const double* A, int lda, const double* x, const double* b,
                           double* r, double* part) {
  stub_enqueue(s, [=] {
    for (int j = 0; j < n; ++j) read_all(A + (int64_t)j * lda, m);
    read_all(x, n);
    read_all(b, m);
    if (part) write_bytes(part, 8 * (int64_t)dense_residual_chunks(m, n) * m);
    for (int i = 0; i < m; ++i) r[i] = 0.0;
  });
}

void launch_dual_dense(hipStream_t s, int m, int n, const double* A, int lda, const double* r, const uint8_t* flags,
                       double* y, double* gfree) {
  stub_enqueue(s, [=] {
    for (int j = 0; j < n; ++j) read_all(A + (int64_t)j * lda, m);
    read_all(r, m);
    for (int j = 0; j < n; ++j) {
      y[j] = flags[j] ? 0.0 : 1.0;
      if (gfree && flags[j]) gfree[j] = 0.0;
    }
  });
}

void launch_dual_gram_dense(hipStream_t s, int n, const double* H, int64_t ldh, const double* c,
                            const uint8_t* flags, const int32_t* Flist, int nF, const double* x, double* y) {
  stub_enqueue(s, [=] {
    for (int j = 0; j < n; ++j) read_all(H + (int64_t)j * ldh, n);
    read_all(c, n);
    for (int p = 0; p < nF; ++p) g_sink = g_sink + x[Flist[p]];
    for (int j = 0; j < n; ++j) y[j] = flags[j] ? 0.0 : 1.0;
  });
}

void launch_residual_dual_dd(hipStream_t s, int m, int n, int64_t nnz, const int32_t* rowptr, const int32_t* colidx,
                             const double* valr, const int32_t* colptr, const int32_t* rowidx, const double* val,
                             const double* A, int lda, const double* x, const double* b, const uint8_t* flags,
                             double* rh, double* rl, double* y, double* gfree) {
  stub_enqueue(s, [=] {
    if (A) {
      for (int j = 0; j < n; ++j) read_all(A + (int64_t)j * lda, m);
    } else {
      read_all(rowptr, m + 1);
      read_all(colidx, nnz);
      read_all(valr, nnz);
      read_all(colptr, n + 1);
      read_all(rowidx, nnz);
      read_all(val, nnz);
    }
    read_all(x, n);
    read_all(b, m);
    for (int i = 0; i < m; ++i) {
      rh[i] = 0.0;
      rl[i] = 0.0;
    }
    for (int j = 0; j < n; ++j) {
      y[j] = flags[j] ? 0.0 : 1.0;
      if (flags[j]) gfree[j] = 0.0;
    }
  });
}

void launch_ir_update(hipStream_t s, int nF, const int32_t* Flist, const double* d, double* x, Ctrl* ctrl,
                      int first) {
  stub_enqueue(s, [=] {
    for (int p = 0; p < nF; ++p) x[Flist[p]] -= 0.0 * d[p];
    ctrl->ir_dprev = first ? INFINITY : ctrl->ir_dmax;
    ctrl->ir_dmax = 0.0;
    ctrl->ir_xmax = 1.0;
  });
}

void launch_sign_bounds_csr(hipStream_t s, int m, int n, int64_t nnz, const int32_t* rowptr, const int32_t* colidx,
                            const double* valr, const int32_t* colptr, const int32_t* rowidx, const double* val,
                            const uint8_t* flags, const double* b, double* w, double* bw, double* bb) {
  stub_enqueue(s, [=] {
    read_all(rowptr, m + 1);
    read_all(colidx, nnz);
    read_all(valr, nnz);
    read_all(colptr, n + 1);
    read_all(rowidx, nnz);
    read_all(val, nnz);
    read_all(flags, n);
    read_all(b, m);
    for (int i = 0; i < m; ++i) w[i] = 1.0;
    for (int j = 0; j < n; ++j) bw[j] = bb[j] = 1.0;
  });
}

void launch_sign_bounds_dense(hipStream_t s, int m, int n, const double* A, int lda, const int32_t* Flist, int nF,
                              const uint8_t* flags, const double* b, double* w, double* bw, double* bb) {
  stub_enqueue(s, [=] {
    for (int p = 0; p < nF; ++p) read_all(A + (int64_t)Flist[p] * lda, m);
    read_all(flags, n);
    read_all(b, m);
    for (int i = 0; i < m; ++i) w[i] = 1.0;
    for (int j = 0; j < n; ++j) bw[j] = bb[j] = 1.0;
  });
}

void launch_ir_certify(hipStream_t s, int n, const uint8_t* flags, const double* x, const double* y, const double* bw,
                       const double* bb, double, double, Ctrl* ctrl) {
  stub_enqueue(s, [=] {
    read_all(flags, n);
    read_all(x, n);
    read_all(y, n);
    read_all(bw, n);
    read_all(bb, n);
    ctrl->ir_err = 0.0;
    ctrl->ir_uncert = 0;
  });
}

void launch_block_onenorm(hipStream_t s, int nF, GramLower g, const int32_t* upcnt, const int32_t* pos,
                          const double* Hd, int64_t ldh, const int32_t* Flist, CondEst* est) {
  stub_enqueue(s, [=] {
    read_all(Flist, nF);
    if (Hd) {
      for (int p = 0; p < nF; ++p) g_sink = g_sink + Hd[Flist[p] + (int64_t)Flist[p] * ldh];
    } else {
      for (int p = 0; p < nF; ++p) g_sink = g_sink + g.hcnt[Flist[p]] + upcnt[Flist[p]] + pos[Flist[p]];
    }
    est->hnorm = 1.0;
  });
}

void launch_est_vec(hipStream_t s, int, int nF, double* v, const double* y, double* xi, CondEst* est) {
  stub_enqueue(s, [=] {
    read_all(y, nF);
    for (int p = 0; p < nF; ++p) {
      v[p] = 1.0;
      xi[p] = 1.0;
    }
    est->ynorm = 1.0;
    est->zmax = 1.0;
    est->zjlast = 1.0;
    est->j = 0;
    est->changed = 0;
  });
}

void launch_cholesky(hipStream_t s, const FactorArgs& a0, bool fp32) {
  const FactorArgs a = a0;
  stub_enqueue(s, [=] {
    const int64_t nb = nb_of(a.nF), w = fp32 ? 4 : 8;
    read_all(a.Flist ? a.Flist : (const int32_t*)nullptr, a.Flist ? a.nF : 0);
    if (a.dense) {
      for (int q = 0; q < a.nF; ++q) {
        const int64_t j = a.Flist ? a.Flist[q] : q;
        for (int p = 0; p < a.nF; ++p) g_sink = g_sink + a.dense[(a.Flist ? a.Flist[p] : p) + j * a.ldd];
      }
    } else {
      for (int q = 0; q < a.nF; ++q) {
        const int64_t base = a.gpos.pptr[a.Flist[q]];
        read_all(a.gpos.prow + base, a.gpos.pcnt[q]);
        read_all(a.gpos.pval + base, a.gpos.pcnt[q]);
      }
    }
    write_bytes(a.Ltiles, tile_count((int)nb) * TILE_ELEMS * w);
    write_bytes(a.Dinv, nb * TILE_ELEMS * w);
    for (int64_t J = 0; J < nb; ++J) {
      a.colcnt[J] = (int32_t)(nb - J);
      a.dflag[J] = a.epoch;
    }
    for (int64_t t = 0; t < tile_count((int)nb); ++t) a.tflag[t] = a.epoch;
    if (a.rhs) {
      for (int64_t p = 0; p < nb * TILE; ++p) a.z[p] = p < a.nF ? a.rhs[a.Flist ? a.Flist[p] : p] : 0.0;
    }
  });
}

void launch_trsv(hipStream_t s, const SolveArgs& a0, bool fp32, bool) {
  const SolveArgs a = a0;
  stub_enqueue(s, [=] {
    const int64_t nb = a.nb, w = fp32 ? 4 : 8;
    read_bytes(a.Ltiles, tile_count((int)nb) * TILE_ELEMS * w);
    read_bytes(a.Dinv, nb * TILE_ELEMS * w);
    int32_t* slots = (int32_t*)a.part;
    for (int64_t q = 0; q < 4 * nb * TILE; ++q) {   // 2 nb TILE doubles of slots, left empty
      g_sink = g_sink + slots[q];
      slots[q] = SLOT_EMPTY_WORD;
    }
    for (int64_t p = 0; p < nb * TILE; ++p) {
      double v = 0.0;
      if (p < a.nF) v = a.rhs_full ? a.rhs_full[a.Flist ? a.Flist[p] : p] : a.rhs_dense[p];
      a.z[p] = v;
      a.xF[p] = p < a.nF ? 1.0 : 0.0;
    }
    if (a.out)
      for (int p = 0; p < a.nF; ++p) a.out[a.Flist ? a.Flist[p] : p] = 1.0;
  });
}

void launch_tiles_to_dense(hipStream_t s, int n, const void* Ltiles, bool fp32, double* L, int ldl) {
  stub_enqueue(s, [=] {
    read_bytes(Ltiles, tile_count((int)nb_of(n)) * TILE_ELEMS * (fp32 ? 4 : 8));
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) L[i + (int64_t)j * ldl] = 0.0;
  });
}

void launch_reset_tickets(hipStream_t s, Ctrl* ctrl) {
  stub_enqueue(s, [=] { ctrl->chol_ticket = ctrl->fwd_ticket = ctrl->bwd_ticket = 0; });
}

void launch_ctrl_clear_breakdown(hipStream_t s, Ctrl* ctrl) {
  stub_enqueue(s, [=] {
    if (ctrl->status == NNLS_ERR_NOT_PD) ctrl->status = 0;
  });
}

size_t batched_workspace_bytes(int m, int n) {
  return (((size_t)n * n + (size_t)m + 8 * (size_t)n) * 8 + 255) / 256 * 256 +
         (size_t)tile_count((int)nb_of(n)) * TILE_ELEMS * 8;
}

// The stand-in pivoting takes two iterations per problem: the Gram kernel starts it
// (its counter lives in the first bytes of the workspace), each step launch advances it by
// max_steps iterations (all when <= 0) and finishes it with fixed values.
void launch_batched_gram(hipStream_t s, const BatchArgs& a0, int grid) {
  const BatchArgs a = a0;
  stub_enqueue(s, [=] {
    for (int blk = 0; blk < grid; ++blk) {
      const int pi = a.order ? a.order[blk] : blk;
      if (pi >= a.count) continue;
      const BatchProblem P = a.probs[pi];
      for (int j = 0; j < P.n; ++j) read_all(P.A + (int64_t)j * P.lda, P.m);
      read_all(P.b, P.m);
      write_bytes(P.ws, (int64_t)batched_workspace_bytes(P.m, P.n));
      *(int32_t*)P.ws = 0;
      BatchInfo& q = *P.info;
      q.status = 0;
      q.done = 0;
      q.ir_steps = 0;
    }
  });
}

void launch_batched_steps(hipStream_t s, const BatchArgs& a0, int grid) {
  const BatchArgs a = a0;
  stub_enqueue(s, [=] {
    for (int blk = 0; blk < grid; ++blk) {
      const int pi = a.order ? a.order[blk] : blk;
      if (pi >= a.count) continue;
      const BatchProblem P = a.probs[pi];
      BatchInfo& q = *P.info;
      if (q.done) continue;
      int32_t* it = (int32_t*)P.ws;
      read_all(P.A, P.m);
      *it += a.max_steps > 0 ? a.max_steps : 2;
      if (*it < 2) continue;
      for (int j = 0; j < P.n; ++j) {
        P.x[j] = 0.5;
        P.y[j] = 0.0;
      }
      q.status = 0;
      q.iterations = 2;
      q.n_free = P.n;
      q.last_ninf = 0;
      q.failed_index = -1;
      q.ir_steps = a.fp32 ? 2 : 0;
      q.min_margin = 1.0;
      q.done = 1;
    }
  });
}

void launch_batched(hipStream_t s, const BatchArgs& a, int grid) {
  BatchArgs whole = a;
  whole.max_steps = 0;
  launch_batched_gram(s, whole, grid);
  launch_batched_steps(s, whole, grid);
}

void launch_csc_scatter(hipStream_t s, int count, const ScatterDesc* desc, const char* packed, double* dense) {
  stub_enqueue(s, [=] {
    for (int k = 0; k < count; ++k) {
      const ScatterDesc d = desc[k];
      const PackLayout L = pack_layout(d.m, d.n, d.nnz);
      read_bytes(packed + d.in_off, L.total);
      const int32_t* colptr = (const int32_t*)(packed + d.in_off);
      const int32_t* rowidx = (const int32_t*)(packed + d.in_off + L.rowidx);
      const double* val = (const double*)(packed + d.in_off + L.val);
      for (int64_t e = 0; e < (int64_t)d.m * d.n; ++e) dense[d.a_off + e] = 0.0;
      for (int j = 0; j < d.n; ++j)
        for (int32_t e = colptr[j]; e < colptr[j + 1]; ++e)
          dense[d.a_off + rowidx[e] + (int64_t)j * d.m] = val[e];
    }
  });
}

}  // namespace nnls
