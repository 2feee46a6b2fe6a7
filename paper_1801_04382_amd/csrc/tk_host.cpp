// Host side of libtrajkrotov: validation, operator packing, device memory,
// kernel launches and the Krotov iteration driver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <numeric>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "tk_host_internal.h"
#include "tk_internal.h"

using namespace tkh;

namespace {

// ---------------------------------------------------------------------------
// host sparse matrices
// ---------------------------------------------------------------------------

// dense-row accumulation helper (d is small enough for per-row scatter)
struct RowAcc {
  std::vector<cd> acc;
  std::vector<int32_t> cols;
  std::vector<char> used;
  explicit RowAcc(int64_t n) : acc(n), used(n, 0) {}
  void add(int32_t c, cd v) {
    if (!used[c]) {
      used[c] = 1;
      cols.push_back(c);
      acc[c] = 0;
    }
    acc[c] += v;
  }
  void flush(Csr &out) {
    std::sort(cols.begin(), cols.end());
    for (int32_t c : cols) {
      if (acc[c] != cd(0.0, 0.0)) {
        out.idx.push_back(c);
        out.val.push_back(acc[c]);
      }
      used[c] = 0;
    }
    cols.clear();
    out.ptr.push_back(out.nnz());
  }
};

Csr adjoint(const Csr &a) {
  Csr t;
  t.n = a.n;
  std::vector<int64_t> cnt(a.n + 1, 0);
  for (int32_t c : a.idx) cnt[c + 1]++;
  for (int64_t r = 0; r < a.n; ++r) cnt[r + 1] += cnt[r];
  t.ptr = cnt;
  t.idx.resize(a.nnz());
  t.val.resize(a.nnz());
  std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
  for (int64_t r = 0; r < a.n; ++r)
    for (int64_t p = a.ptr[r]; p < a.ptr[r + 1]; ++p) {
      const int32_t c = a.idx[p];
      t.idx[pos[c]] = static_cast<int32_t>(r);
      t.val[pos[c]] = std::conj(a.val[p]);
      pos[c]++;
    }
  return t;
}

// c = a + alpha * b
Csr axpy(const Csr &a, cd alpha, const Csr &b) {
  Csr c;
  c.n = a.n;
  c.ptr.push_back(0);
  RowAcc row(a.n);
  for (int64_t r = 0; r < a.n; ++r) {
    for (int64_t p = a.ptr[r]; p < a.ptr[r + 1]; ++p) row.add(a.idx[p], a.val[p]);
    for (int64_t p = b.ptr[r]; p < b.ptr[r + 1]; ++p) row.add(b.idx[p], alpha * b.val[p]);
    row.flush(c);
  }
  return c;
}

// c = a * b
Csr multiply(const Csr &a, const Csr &b) {
  Csr c;
  c.n = a.n;
  c.ptr.push_back(0);
  RowAcc row(a.n);
  for (int64_t r = 0; r < a.n; ++r) {
    for (int64_t p = a.ptr[r]; p < a.ptr[r + 1]; ++p) {
      const int32_t k = a.idx[p];
      for (int64_t q = b.ptr[k]; q < b.ptr[k + 1]; ++q) row.add(b.idx[q], a.val[p] * b.val[q]);
    }
    row.flush(c);
  }
  return c;
}


// ||A||_2 <= sqrt(||A||_1 ||A||_inf)
double norm2_bound(const Csr &a) {
  std::vector<double> col(a.n, 0.0);
  double rmax = 0.0;
  for (int64_t r = 0; r < a.n; ++r) {
    double rs = 0.0;
    for (int64_t p = a.ptr[r]; p < a.ptr[r + 1]; ++p) {
      rs += std::abs(a.val[p]);
      col[a.idx[p]] += std::abs(a.val[p]);
    }
    rmax = std::max(rmax, rs);
  }
  double cmax = 0.0;
  for (double v : col) cmax = std::max(cmax, v);
  return std::sqrt(rmax * cmax);
}

// y = A x (dense vector)
void spmv(const Csr &a, const std::vector<cd> &x, std::vector<cd> &y) {
  y.assign(a.n, cd(0.0, 0.0));
  for (int64_t r = 0; r < a.n; ++r) {
    cd s(0.0, 0.0);
    for (int64_t p = a.ptr[r]; p < a.ptr[r + 1]; ++p) s += a.val[p] * x[a.idx[p]];
    y[r] = s;
  }
}

// Estimate of ||A||_2 by power iteration on A^+ A (from below), inflated by 5%
// and never above the rigorous bound sqrt(||A||_1 ||A||_inf).
double norm2_estimate(const Csr &a) {
  const double rigorous = norm2_bound(a);
  if (a.nnz() == 0) return 0.0;
  const Csr ad = adjoint(a);
  std::vector<cd> x(a.n), y, z;
  for (int64_t i = 0; i < a.n; ++i) x[i] = cd(1.0 + 0.001 * (i % 7), 0.01 * (i % 3));
  double lam = 0.0;
  for (int it = 0; it < 300; ++it) {
    double nx = 0.0;
    for (const cd &v : x) nx += std::norm(v);
    nx = std::sqrt(nx);
    if (!(nx > 0.0)) break;
    for (cd &v : x) v /= nx;
    spmv(a, x, y);
    spmv(ad, y, z);
    double rq = 0.0;
    for (int64_t i = 0; i < a.n; ++i) rq += std::real(std::conj(x[i]) * z[i]);
    lam = std::sqrt(std::max(rq, 0.0));
    x.swap(z);
  }
  return std::min(1.05 * lam, rigorous);
}

double max_abs(const Csr &a) {
  double m = 0.0;
  for (const cd &v : a.val) m = std::max(m, std::abs(v));
  return m;
}

// ---------------------------------------------------------------------------
// device buffers
// ---------------------------------------------------------------------------

struct Ell {  // packed per-lane slices of one operator group
  std::vector<int32_t> col;
  std::vector<double> val;  // interleaved complex, FP64 (converted on upload)
};

}  // namespace


namespace tkh {

int fail(tk_ctx *c, int code, const std::string &msg) {
  if (c) c->err = msg;
  return code;
}

int hip_fail(tk_ctx *c, hipError_t e, const char *what) {
  return fail(c, e == hipErrorOutOfMemory ? TK_ENOMEM : TK_EHIP,
              std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace tkh

namespace {


int read_csr(tk_ctx *c, const tk_csr *m, int64_t d, const char *name, Csr &out) {
  if (!m) return fail(c, TK_EINVAL, std::string(name) + " is NULL");
  if (m->n_rows != d) return fail(c, TK_EDIM, std::string(name) + " has the wrong dimension");
  if (m->nnz < 0 || (m->nnz > 0 && (!m->indices || !m->values)) || !m->indptr)
    return fail(c, TK_EINVAL, std::string(name) + ": missing arrays");
  if (m->indptr[0] != 0 || m->indptr[d] != m->nnz)
    return fail(c, TK_EINVAL, std::string(name) + ": indptr does not span nnz");
  out.n = d;
  out.ptr.assign(m->indptr, m->indptr + d + 1);
  for (int64_t r = 0; r < d; ++r)
    if (out.ptr[r + 1] < out.ptr[r])
      return fail(c, TK_EINVAL, std::string(name) + ": indptr decreases");
  // merge duplicates / drop zeros through a row accumulator
  Csr clean;
  clean.n = d;
  clean.ptr.push_back(0);
  RowAcc row(d);
  for (int64_t r = 0; r < d; ++r) {
    for (int64_t p = out.ptr[r]; p < out.ptr[r + 1]; ++p) {
      const int32_t col = m->indices[p];
      const double re = m->values[2 * p], im = m->values[2 * p + 1];
      if (col < 0 || col >= d) return fail(c, TK_EINVAL, std::string(name) + ": column out of range");
      if (!std::isfinite(re) || !std::isfinite(im))
        return fail(c, TK_EINVAL, std::string(name) + ": non-finite value");
      row.add(col, cd(re, im));
    }
    row.flush(clean);
  }
  out = std::move(clean);
  return TK_OK;
}

bool hermitian(const Csr &h) {
  const Csr diff = axpy(h, cd(-1.0, 0.0), adjoint(h));
  return max_abs(diff) <= 1e-12 * std::max(max_abs(h), 1e-300);
}

// Per-lane slot layout of one operator `a` (may be null = all padding) in W
// slots starting at slot index `first` of an array laid out [slot][m][lane]
// (row r = lane + 64 m).  Each row's non-zeros are dealt to the slots; a slot
// a row does not use points at `dummy`, a zero element every lane may read at
// once (a broadcast).  Which non-zero goes to which slot is free, so for every
// slot and every 16-lane group the entries are chosen greedily to spread the
// gathered elements over the LDS bank groups (element c lies in group
// c mod n_bank_groups), which keeps the gathers of one instruction from
// colliding in the same banks.
// Row slots m >= 1 use only the first W_rest of the W slots (shapes whose
// basis order puts the rows with the most non-zeros in row slot 0).  With
// typed_real >= 0 (typed shapes), row slot 0's first typed_real slots take
// only real elements and the others only imaginary ones.  Returns false if a
// row has more non-zeros than its slots (of each type).
bool pack_group(const Csr *a, int W, int W_rest, int first, int R, int lanes, int n_bank_groups,
                int32_t dummy, std::vector<int32_t> &col, std::vector<double> &val,
                int typed_real = -1) {
  std::vector<std::vector<std::pair<int32_t, cd>>> left(static_cast<size_t>(R) * lanes);
  for (int m = 0; m < R; ++m)
    for (int lane = 0; lane < lanes; ++lane) {
      const int64_t row = lane + static_cast<int64_t>(lanes) * m;
      auto &l = left[static_cast<size_t>(m) * lanes + lane];
      if (a && row < a->n)
        for (int64_t p = a->ptr[row]; p < a->ptr[row + 1]; ++p) l.push_back({a->idx[p], a->val[p]});
    }
  std::vector<int> load(n_bank_groups);
  for (int w = 0; w < W; ++w)
    for (int m = 0; m < R; ++m)
      for (int g0 = 0; g0 < lanes; g0 += 16) {
        std::fill(load.begin(), load.end(), 0);
        bool dummy_used = false;
        for (int lane = g0; lane < g0 + 16; ++lane) {
          auto &l = left[static_cast<size_t>(m) * lanes + lane];
          const size_t slot = (static_cast<size_t>(first + w) * R + m) * lanes + lane;
          // the elements this slot may take (typed slots: real or imaginary ones)
          auto fits = [&](const std::pair<int32_t, cd> &e) {
            if (typed_real < 0 || m > 0) return true;
            return w < typed_real ? e.second.imag() == 0.0 : e.second.real() == 0.0;
          };
          size_t best = l.size();
          for (size_t q = 0; q < l.size(); ++q) {
            if (!fits(l[q])) continue;
            if (best == l.size()) {
              best = q;
              continue;
            }
            const int lb = load[l[best].first % n_bank_groups], lq = load[l[q].first % n_bank_groups];
            if (lq < lb || (lq == lb && l[q].first < l[best].first)) best = q;
          }
          if (best == l.size() || (m > 0 && w >= W_rest)) {
            col[slot] = dummy;
            val[2 * slot] = val[2 * slot + 1] = 0.0;
            if (!dummy_used) load[dummy % n_bank_groups]++;
            dummy_used = true;
            continue;
          }
          col[slot] = l[best].first;
          val[2 * slot] = l[best].second.real();
          val[2 * slot + 1] = l[best].second.imag();
          load[l[best].first % n_bank_groups]++;
          l.erase(l.begin() + static_cast<long>(best));
        }
      }
  for (const auto &l : left)
    if (!l.empty()) return false;
  return true;
}

// Operators ops[g], each in W slots: layout [g][w][m][lane], `lanes` lanes
// (64 G) per row slot m.
bool pack(const std::vector<const Csr *> &ops, int W, int R, int lanes, int n_bank_groups,
          Ell &out, int W_rest = -1, int typed_real = -1) {
  const size_t n = ops.size() * static_cast<size_t>(W) * R * lanes;
  out.col.assign(n, 0);
  out.val.assign(2 * n, 0.0);
  const int32_t dummy = R * lanes;
  bool ok = true;
  for (size_t g = 0; g < ops.size(); ++g)
    ok = pack_group(ops[g], W, W_rest < 0 ? W : W_rest, static_cast<int>(g) * W, R, lanes,
                    n_bank_groups, dummy, out.col, out.val, typed_real) &&
         ok;
  return ok;
}

// Control operators: slots c = i * wc .. i * wc + wc - 1 hold H_i; slots past
// n_ctrl * wc are padding.
bool pack_ctrl(const std::vector<Csr> &H, int wc, int NC, int R, int lanes, int n_bank_groups,
               Ell &out) {
  const size_t n = static_cast<size_t>(NC) * R * lanes;
  out.col.assign(n, 0);
  out.val.assign(2 * n, 0.0);
  const int32_t dummy = R * lanes;
  bool ok = true;
  for (int i = 0; i * wc < NC; ++i) {
    const Csr *a = i < static_cast<int>(H.size()) ? &H[i] : nullptr;
    const int w = std::min(wc, NC - i * wc);
    ok = pack_group(a, w, w, i * wc, R, lanes, n_bank_groups, dummy, out.col, out.val) && ok;
  }
  return ok;
}

// Rows and columns of a in device order: device row q is basis row perm[q]
// (inv is the inverse map).
Csr permute(const Csr &a, const std::vector<int32_t> &perm, const std::vector<int32_t> &inv) {
  Csr out;
  out.n = a.n;
  out.ptr.push_back(0);
  std::vector<std::pair<int32_t, cd>> row;
  for (int64_t q = 0; q < a.n; ++q) {
    const int64_t r = perm[q];
    row.clear();
    for (int64_t p = a.ptr[r]; p < a.ptr[r + 1]; ++p) row.push_back({inv[a.idx[p]], a.val[p]});
    std::sort(row.begin(), row.end(),
              [](const std::pair<int32_t, cd> &x, const std::pair<int32_t, cd> &y) {
                return x.first < y.first;
              });
    for (const auto &e : row) {
      out.idx.push_back(e.first);
      out.val.push_back(e.second);
    }
    out.ptr.push_back(static_cast<int64_t>(out.idx.size()));
  }
  return out;
}

// a without its diagonal; the diagonal goes to diag (length a.n)
Csr off_diagonal(const Csr &a, std::vector<cd> &diag) {
  Csr out;
  out.n = a.n;
  out.ptr.push_back(0);
  diag.assign(static_cast<size_t>(a.n), cd(0.0, 0.0));
  for (int64_t r = 0; r < a.n; ++r) {
    for (int64_t p = a.ptr[r]; p < a.ptr[r + 1]; ++p) {
      if (a.idx[p] == r) {
        diag[static_cast<size_t>(r)] = a.val[p];
      } else {
        out.idx.push_back(a.idx[p]);
        out.val.push_back(a.val[p]);
      }
    }
    out.ptr.push_back(static_cast<int64_t>(out.idx.size()));
  }
  return out;
}

}  // namespace

namespace tkh {

int upload(tk_ctx *c, DevBuf &buf, const void *src, size_t bytes) {
  TK_HIP(c, buf.ensure(bytes));
  if (bytes) TK_HIP(c, hipMemcpy(buf.p, src, bytes, hipMemcpyHostToDevice));
  return TK_OK;
}

}  // namespace tkh

namespace {

int upload_ell(tk_ctx *c, const Ell &e, DevBuf &col, DevBuf &val) {
  int rc = upload(c, col, e.col.data(), e.col.size() * sizeof(int32_t));
  if (rc) return rc;
  if (c->precision == TK_FP64) return upload(c, val, e.val.data(), e.val.size() * sizeof(double));
  std::vector<float> f(e.val.begin(), e.val.end());
  return upload(c, val, f.data(), f.size() * sizeof(float));
}

int upload_vec(tk_ctx *c, DevBuf &buf, const std::vector<double> &v) {
  if (c->precision == TK_FP64) return upload(c, buf, v.data(), v.size() * sizeof(double));
  std::vector<float> f(v.begin(), v.end());
  return upload(c, buf, f.data(), f.size() * sizeof(float));
}

// Remainder bound of the order-K Taylor polynomial of exp over ||A|| tau = x:
// x^(K+1)/(K+1)! e^x.
double remainder_bound(double x, int K) {
  double t = x;
  for (int n = 1; n <= K; ++n) t *= x / static_cast<double>(n + 1);
  return t * std::exp(x);
}

// ord_x[K] = the largest x whose order-K remainder bound is within tol (by
// bisection, keeping the side that meets it), made non-decreasing in K from
// above so that every entry stays a sufficient condition.
struct OrderTable {
  double x[tk::kMaxTaylor + 1];
  explicit OrderTable(double tol) {
    x[0] = 0.0;
    for (int K = 1; K <= tk::kMaxTaylor; ++K) {
      double lo = 0.0, hi = 1.0;
      while (remainder_bound(hi, K) <= tol) hi *= 2.0;
      for (int it = 0; it < 200 && hi - lo > 0.0; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        (remainder_bound(mid, K) <= tol ? lo : hi) = mid;
      }
      x[K] = lo;
    }
    for (int K = tk::kMaxTaylor - 1; K >= 1; --K) x[K] = std::min(x[K], x[K + 1]);
  }
};

const double *order_table(int precision) {
  // FP64: 1e-15 per step, the size of the step's own rounding (K = 9 at
  // ||H_eff|| dt = 0.14); FP32: 6e-8
  static const OrderTable t64(1e-15), t32(6e-8);
  return precision == TK_FP64 ? t64.x : t32.x;
}

// Taylor order of one step (the kernels' rule): the smallest K with
// x <= ord_x[K], else kmax.
int taylor_order_host(double x, const double *ord_x, int kmax) {
  for (int K = 1; K <= kmax; ++K)
    if (x <= ord_x[K]) return K;
  return kmax;
}

// Substeps and Taylor order of step j for pulses u (the kernels' rule without
// the term-buffer limit).
void plan_step_host(const tk_ctx *c, const std::vector<double> &u, int j, int *n_sub, int *K) {
  double b = c->b0;
  for (int i = 0; i < c->n_ctrl; ++i)
    b += std::fabs(u[static_cast<size_t>(i) * c->nt + j]) * c->bc[i];
  const double x = b * (c->T / c->nt);
  *n_sub = x > tk::kMaxStepNorm ? static_cast<int>(std::ceil(x / tk::kMaxStepNorm)) : 1;
  *K = taylor_order_host(x / *n_sub, order_table(c->precision), tk::kMaxTaylor);
}

}  // namespace

namespace tkh {

// Term vectors a pass needs: the largest order over its steps, plus one for
// the zeroth term (a step that ends in a jump keeps t_0 .. t_K) and `margin`
// for pulses that grow during a Krotov pass.
int plan_kbuf(const tk_ctx *c, const std::vector<double> &u, int margin) {
  int kmax = 1;
  for (int j = 0; j < c->nt; ++j) {
    int n_sub, K;
    plan_step_host(c, u, j, &n_sub, &K);
    kmax = std::max(kmax, K);
  }
  int kb = std::min(kmax + 1 + margin, tk::kMaxTaylor + 1);
  // at most what one team's LDS holds: a step that needs more terms is cut
  // into more substeps by the kernels (FP64 at d = 1296)
  while (kb > 3 && tk::block_lds_bytes(*c->var, 1, kb, 0) > tk::kLdsBytes) --kb;
  return kb;
}

// Term vectors of the gradient's reverse sweep: the kept terms t_0 .. t_Kg of
// a propagator unit, Kg the order for the bound ||H_eff|| + max_i ||H_i|| of
// Van Loan's block generator (at least the step's own order), plus two for
// the costate series.
int plan_kbuf_grad(const tk_ctx *c, const std::vector<double> &u, double bc_max) {
  int kg = 1;
  for (int j = 0; j < c->nt; ++j) {
    int n_sub, K;
    plan_step_host(c, u, j, &n_sub, &K);
    double b = c->b0;
    for (int i = 0; i < c->n_ctrl; ++i)
      b += std::fabs(u[static_cast<size_t>(i) * c->nt + j]) * c->bc[i];
    const double h = n_sub == 1 ? c->T / c->nt : (c->T / c->nt) / n_sub;
    const int Kg = taylor_order_host((b + bc_max) * h, order_table(c->precision), tk::kMaxTaylor);
    kg = std::max(kg, std::max(K, Kg));
  }
  return std::min(kg + 3, tk::kMaxTaylor + 1);
}

double pass_flops(const tk_ctx *c, const std::vector<double> &u, int M) {
  double f = 0.0;
  for (int j = 0; j < c->nt; ++j) {
    int n_sub, K;
    plan_step_host(c, u, j, &n_sub, &K);
    f += n_sub * (8.0 * K * c->nnz_heff + 8.0 * K * c->d + 4.0 * c->d);
  }
  return f * M;
}

}  // namespace tkh

namespace {

// Waves per block for a plain pass: as many as fit the LDS (at most 4).
// Teams per block for a plain pass: one G-wave team (G > 1), else as many
// one-wave teams as fit the LDS (at most 4).
int pass_waves(const tk_ctx *c, int kbuf) {
  if (c->var->G > 1) return tk::block_lds_bytes(*c->var, 1, kbuf, 0) <= tk::kLdsBytes ? 1 : 0;
  for (int w = tk::kWavesPerBlock; w >= 1; w /= 2)
    if (tk::block_lds_bytes(*c->var, w, kbuf, 0) <= tk::kLdsBytes) return w;
  return 0;
}

}  // namespace

namespace tkh {

tk::PassArgs base_args(tk_ctx *c, int M, uint64_t seed, uint64_t iteration, bool backward) {
  tk::PassArgs a;
  std::memset(&a, 0, sizeof(a));
  a.d = static_cast<int>(c->d);
  a.nt = c->nt;
  a.M = M;
  a.n_ctrl = c->n_ctrl;
  a.n_jump = c->n_jump;
  a.wc = c->wc;
  a.wl = c->wl;
  a.kmax = tk::kMaxTaylor;
  a.kbuf = plan_kbuf(c, c->u, 0);
  a.dt = c->T / c->nt;
  a.tol = c->precision == TK_FP64 ? 1e-15 : 6e-8;
  a.ftol = c->precision == TK_FP64 ? 4.0 * 0x1.0p-52 : 4.0 * 0x1.0p-23;
  a.b0 = c->b0;
  for (int i = 0; i < tk::kMaxCtrl; ++i) a.bc[i] = c->bc[i];
  a.inv_n[0] = 0.0;
  for (int n = 1; n <= tk::kMaxTaylor; ++n) a.inv_n[n] = 1.0 / n;
  std::memcpy(a.ord_x, order_table(c->precision), sizeof(a.ord_x));
  if (!backward) {
    a.scol = c->f_scol.as<int>();
    a.sval = c->f_sval.p;
    a.sdiag = c->f_sdiag.p;
    a.ccol = c->f_ccol.as<int>();
    a.cval = c->f_cval.p;
    a.psi_start = c->psi0_bulk.p;
  } else {
    a.scol = c->b_scol.as<int>();
    a.sval = c->b_sval.p;
    a.sdiag = c->b_sdiag.p;
    a.ccol = c->b_ccol.as<int>();
    a.cval = c->b_cval.p;
    a.psi_start = c->tgt_bulk.p;
  }
  a.lcol = c->lcol.as<int>();
  a.lval = c->lval.p;
  a.u = c->u_dev.as<double>();
  a.tgt = c->tgt64.as<double>();
  a.seed = seed;
  a.iteration = iteration;
  a.instance = 0;
  a.err = c->err_dev.as<int>();
  a.rec_count = c->rec_count.as<unsigned long long>();
  a.spin_limit = 1ll << 22;
  return a;
}

}  // namespace tkh

namespace {

int prepare_pass(tk_ctx *c, int M, int64_t cap) {
  if (!c->has_system) return fail(c, TK_ESTATE, "no system set");
  if (!c->has_states) return fail(c, TK_ESTATE, "no states set");
  if (!c->has_pulses) return fail(c, TK_ESTATE, "no pulses set");
  if (M < 1) return fail(c, TK_EINVAL, "M must be >= 1");
  if (cap < 0) return fail(c, TK_EINVAL, "negative record capacity");
  TK_HIP(c, c->err_dev.ensure(sizeof(int)));
  TK_HIP(c, c->rec_count.ensure(sizeof(unsigned long long)));
  TK_HIP(c, c->rec.ensure(std::max<int64_t>(cap, 1) * sizeof(tk_jump)));
  TK_HIP(c, c->tau.ensure(static_cast<size_t>(2) * M * sizeof(double)));
  TK_HIP(c, c->psiT.ensure(static_cast<size_t>(M) * c->d * c->bulk_cplx()));
  return TK_OK;
}

int reset_counters(tk_ctx *c) {
  TK_HIP(c, hipMemsetAsync(c->err_dev.p, 0, sizeof(int), c->stream));
  TK_HIP(c, hipMemsetAsync(c->rec_count.p, 0, sizeof(unsigned long long), c->stream));
  return TK_OK;
}

int check_kernel_errors(tk_ctx *c, const int *err_dev = nullptr) {
  int e = 0;
  TK_HIP(c, hipMemcpyAsync(&e, err_dev ? err_dev : c->err_dev.p, sizeof(int),
                           hipMemcpyDeviceToHost, c->stream));
  TK_HIP(c, hipStreamSynchronize(c->stream));
  if (e & tk::kErrSyncTimeout)
    return fail(c, TK_EHIP, "grid-wide step reduction timed out (blocks not co-resident)");
  if (e & tk::kErrNoJumpWeight)
    return fail(c, TK_ENUMERIC, "jump with all ||L_l psi||^2 = 0");
  if (e & tk::kErrTaylorOrder)
    return fail(c, TK_ENUMERIC, "time step too long for the polynomial propagator; raise nt");
  if (e & tk::kErrJumpLoop) return fail(c, TK_ENUMERIC, "too many jumps inside one time step");
  return TK_OK;
}

int fetch_records(tk_ctx *c, tk_jump *rec, int64_t cap, int64_t *n_rec) {
  unsigned long long n = 0;
  TK_HIP(c, hipMemcpy(&n, c->rec_count.p, sizeof(n), hipMemcpyDeviceToHost));
  if (n_rec) *n_rec = static_cast<int64_t>(n);
  const int64_t copy = std::min<int64_t>(static_cast<int64_t>(n), cap);
  if (rec && copy > 0)
    TK_HIP(c, hipMemcpy(rec, c->rec.p, copy * sizeof(tk_jump), hipMemcpyDeviceToHost));
  if (static_cast<int64_t>(n) > cap && (rec || cap > 0))
    return fail(c, TK_ERECCAP, "jump-record buffer too small");
  return TK_OK;
}

void to_host_cplx(const tk_ctx *c, const void *dev_copy, size_t n, double *out) {
  if (c->precision == TK_FP64) {
    std::memcpy(out, dev_copy, n * 16);
  } else {
    const float *f = static_cast<const float *>(dev_copy);
    for (size_t i = 0; i < 2 * n; ++i) out[i] = f[i];
  }
}

// n_states states of d complex values each, from the device basis order back
// to the basis order (in place)
void states_to_basis(const tk_ctx *c, double *x, size_t n_states) {
  if (c->perm.empty()) return;
  const size_t d = static_cast<size_t>(c->d);
  std::vector<double> tmp(2 * d);
  for (size_t k = 0; k < n_states; ++k) {
    double *v = x + 2 * d * k;
    std::copy(v, v + 2 * d, tmp.begin());
    for (size_t q = 0; q < d; ++q) {
      v[2 * static_cast<size_t>(c->perm[q])] = tmp[2 * q];
      v[2 * static_cast<size_t>(c->perm[q]) + 1] = tmp[2 * q + 1];
    }
  }
}

// the same from the basis order to the device order
void states_to_device(const tk_ctx *c, double *x, size_t n_states) {
  if (c->perm.empty()) return;
  const size_t d = static_cast<size_t>(c->d);
  std::vector<double> tmp(2 * d);
  for (size_t k = 0; k < n_states; ++k) {
    double *v = x + 2 * d * k;
    std::copy(v, v + 2 * d, tmp.begin());
    for (size_t q = 0; q < d; ++q) {
      v[2 * q] = tmp[2 * static_cast<size_t>(c->perm[q])];
      v[2 * q + 1] = tmp[2 * static_cast<size_t>(c->perm[q]) + 1];
    }
  }
}

struct TimedLaunch {
  tk_ctx *c;
  int kind;
  explicit TimedLaunch(tk_ctx *ctx, int k) : c(ctx), kind(k) {
    if (c->timing) (void)hipEventRecord(c->ev0, c->stream);
  }
  int finish(int64_t traj_steps, double flops, double bytes) {
    if (!c->timing) return TK_OK;
    TK_HIP(c, hipEventRecord(c->ev1, c->stream));
    TK_HIP(c, hipEventSynchronize(c->ev1));
    float ms = 0.f;
    TK_HIP(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
    tk_kernel_timing &t = c->tstat[kind];
    t.ms_total += ms;
    t.launches += 1;
    t.traj_steps += traj_steps;
    t.flops += flops;
    t.bytes += bytes;
    return TK_OK;
  }
};

// Plain forward pass.  `fixed` (no-allocation entry point) supplies the error
// bits, record counter and record slot, the overlaps' destination and no final
// states; otherwise the context's buffers are used.
struct FixedBuffers {
  int *err;
  unsigned long long *rec_count;
  tk_jump *rec;
  double *tau;
};

int run_forward(tk_ctx *c, int M, uint64_t seed, uint64_t iteration, int64_t cap,
                const FixedBuffers *fixed = nullptr) {
  tk::PassArgs a = base_args(c, M, seed, iteration, false);
  if (fixed) {
    a.err = fixed->err;
    a.rec_count = fixed->rec_count;
    a.rec = fixed->rec;
    a.rec_cap = 0;
    a.tau_out = fixed->tau;
    a.psiT = nullptr;
  } else {
    a.psiT = c->psiT.p;
    a.tau_out = c->tau.as<double>();
    a.rec = c->rec.as<tk_jump>();
    a.rec_cap = cap;
  }
  const int wpb = pass_waves(c, a.kbuf);
  if (!wpb) return fail(c, TK_EUNSUPPORTED, "the step's Taylor terms do not fit in LDS");
  const int blocks = (M + wpb - 1) / wpb;
  const size_t lds = tk::block_lds_bytes(*c->var, wpb, a.kbuf, 0);
  TK_HIP(c, hipFuncSetAttribute(c->var->k_forward, hipFuncAttributeMaxDynamicSharedMemorySize,
                                static_cast<int>(lds)));
  void *args[] = {&a};
  TimedLaunch tl(c, TK_KERNEL_FORWARD);
  TK_HIP(c, hipLaunchKernel(c->var->k_forward, dim3(blocks), dim3(tk::kWave * c->var->G * wpb), args, lds,
                            c->stream));
  int rc = tl.finish(static_cast<int64_t>(M) * c->nt, pass_flops(c, c->u, M),
                     static_cast<double>(M) * c->d * c->bulk_cplx());
  if (rc) return rc;
  if (!fixed) {
    c->tau_M = M;
    c->tau_seed = seed;
    c->tau_iter = static_cast<int64_t>(iteration);
  }
  return TK_OK;
}

// Costate pass.  unit_weights: every trajectory starts with weight 1 instead of
// its overlap tau_k (the backward states xi_k of the cross-trajectory update).
int run_backward(tk_ctx *c, int M, uint64_t seed, uint64_t iteration, int64_t cap,
                 bool unit_weights = false) {
  const size_t chi_bytes = static_cast<size_t>(c->nt) * M * c->d * c->bulk_cplx();
  c->chi_M = -1;
  TK_HIP(c, c->chi.ensure(chi_bytes));
  tk::PassArgs a = base_args(c, M, seed, iteration, true);
  a.tau_in = c->tau.as<double>();
  if (unit_weights) {
    if (c->ones_tau.bytes < 2 * static_cast<size_t>(M) * sizeof(double)) {
      std::vector<double> ones(2 * static_cast<size_t>(M), 0.0);
      for (int k = 0; k < M; ++k) ones[2 * k] = 1.0;
      int rc = upload(c, c->ones_tau, ones.data(), ones.size() * sizeof(double));
      if (rc) return rc;
    }
    a.tau_in = c->ones_tau.as<double>();
  }
  a.chi = c->chi.p;
  a.rec = c->rec.as<tk_jump>();
  a.rec_cap = cap;
  const int wpb = pass_waves(c, a.kbuf);
  if (!wpb) return fail(c, TK_EUNSUPPORTED, "the step's Taylor terms do not fit in LDS");
  const int blocks = (M + wpb - 1) / wpb;
  const size_t lds = tk::block_lds_bytes(*c->var, wpb, a.kbuf, 0);
  TK_HIP(c, hipFuncSetAttribute(c->var->k_backward, hipFuncAttributeMaxDynamicSharedMemorySize,
                                static_cast<int>(lds)));
  void *args[] = {&a};
  TimedLaunch tl(c, TK_KERNEL_BACKWARD);
  TK_HIP(c, hipLaunchKernel(c->var->k_backward, dim3(blocks), dim3(tk::kWave * c->var->G * wpb), args, lds,
                            c->stream));
  int rc = tl.finish(static_cast<int64_t>(M) * c->nt, pass_flops(c, c->u, M),
                     static_cast<double>(chi_bytes));
  if (rc) return rc;
  c->chi_M = M;
  return TK_OK;
}

// Gram matrices P_j = (1/M) sum_k |xi_k(t_j)><xi_k(t_j)| of the stored
// backward states, [nt][d][64 R] (cross-trajectory update).
int run_gram(tk_ctx *c, int M) {
  const int Rp = c->var->R * tk::kWave;
  TK_HIP(c, c->pmat.ensure(static_cast<size_t>(c->nt) * c->d * Rp * 16));
  const int nrb = (Rp + 31) / 32, ncb = static_cast<int>((c->d + 31) / 32);
  const int S = nrb * ncb;
  const int slots = ((c->nt + 7) / 8) * S;  // blocks of step j sit on XCD j % 8
  const void *chi = c->chi.p;
  int nt = c->nt, m = M, d = static_cast<int>(c->d), rp = Rp;
  double invM = 1.0 / M;
  void *P = c->pmat.p;
  void *args[] = {&chi, &nt, &m, &d, &rp, const_cast<int *>(&nrb), const_cast<int *>(&ncb), &invM,
                  &P};
  TimedLaunch tl(c, TK_KERNEL_CROSS_GRAM);
  TK_HIP(c, hipLaunchKernel(tk::cross_gram_kernel(c->precision), dim3(8 * slots), dim3(256), args,
                            0, c->stream));
  // algorithmic: d^2 complex products per trajectory and step (8 flops each);
  // the backward states are read once
  return tl.finish(static_cast<int64_t>(M) * c->nt,
                   8.0 * static_cast<double>(c->d) * c->d * M * c->nt,
                   static_cast<double>(c->nt) * M * c->d * c->bulk_cplx());
}

int run_krotov(tk_ctx *c, int M, uint64_t seed, uint64_t iteration, int64_t cap,
               bool cross = false) {
  if (c->chi_M != M) return fail(c, TK_ESTATE, "no costates stored for this M");
  const void *kern_lds = cross ? tk::cross_kernel(c->precision, c->var->R, c->var->ws_code,
                                                  c->var->NC, c->var->G)
                               : c->var->k_krotov;
  if (!kern_lds) return fail(c, TK_EUNSUPPORTED, "no cross-trajectory kernel for this variant");
  const void *kern = kern_lds;
  // pulses grow during the pass: one spare term vector; the kernel adds
  // substeps if a step would still need more terms
  const int kbuf = plan_kbuf(c, c->u, 1);
  auto lds_of = [&](int w, int t, bool in_lds) {
    return cross ? tk::cross_lds_bytes(*c->var, w, kbuf, t)
                 : tk::block_lds_bytes(*c->var, w, kbuf, t, in_lds);
  };
  // States in LDS where they fit; otherwise (the independent-trajectory
  // update only) in global memory, each team reading back its own rows.
  // TK_KROTOV_STATES=global takes the global-memory form at any M (tests
  // compare the two forms).
  const char *st_env = std::getenv("TK_KROTOV_STATES");
  const bool force_global = !cross && st_env && std::strcmp(st_env, "global") == 0;
  int tw = 0, wpb = 0, blocks = 0;
  size_t lds = 0;
  bool in_lds = true;
  for (int pass = force_global ? 1 : 0; pass < (cross ? 1 : 2) && !tw; ++pass) {
    in_lds = pass == 0;
    kern = in_lds ? kern_lds : c->var->k_krotov_gs;
    for (int t = 1; t <= 64 && !tw; ++t)
      for (int w = c->var->G > 1 ? 1 : tk::kWavesPerBlock; w >= 1; w /= 2) {
        const int b = (M + w * t - 1) / (w * t);
        const size_t l = lds_of(w, t, in_lds);
        if (b > tk::kMaxBlocks || l > tk::kLdsBytes) continue;
        TK_HIP(c, hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      static_cast<int>(l)));
        int occ = 0;
        TK_HIP(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(
                      &occ, kern, tk::kWave * c->var->G * w, l));
        if (occ > 0 && static_cast<int64_t>(occ) * c->n_cu >= b) {
          tw = t;
          wpb = w;
          blocks = b;
          lds = l;
          break;
        }
      }
  }
  if (!tw) return fail(c, TK_EUNSUPPORTED, "too many trajectories for one cooperative launch");
  if (!in_lds) {
    const size_t vec = static_cast<size_t>(c->var->R) * tk::kWave * c->var->G * c->bulk_cplx();
    TK_HIP(c, c->kstates.ensure(static_cast<size_t>(blocks) * wpb * tw * vec));
  }
  const int ncx = std::max(c->var->NC, 1);
  const size_t nslot = static_cast<size_t>(c->nt) * tk::kMaxBlocks * ncx;
  TK_HIP(c, c->slots.ensure(nslot * sizeof(unsigned long long)));
  TK_HIP(c, c->u_new_dev.ensure(static_cast<size_t>(tk::kMaxCtrl) * c->nt * sizeof(double)));
  {
    unsigned long long *sp = c->slots.as<unsigned long long>();
    long long n = static_cast<long long>(nslot);
    int nb = blocks, nc = ncx;
    void *fargs[] = {&sp, &n, &nb, &nc};
    TK_HIP(c, hipLaunchKernel(c->var->k_fill, dim3(256), dim3(256), fargs, 0, c->stream));
  }
  tk::PassArgs a = base_args(c, M, seed, iteration, false);
  a.psiT = c->psiT.p;
  a.tau_out = c->tau.as<double>();
  a.chi = c->chi.p;
  a.rec = c->rec.as<tk_jump>();
  a.rec_cap = cap;
  a.u_old = c->u_dev.as<double>();
  a.u_new = c->u_new_dev.as<double>();
  a.S = c->S_dev.as<double>();
  a.lam = c->lam_dev.as<double>();
  a.slots = c->slots.as<unsigned long long>();
  a.traj_per_wave = tw;
  a.kstates = in_lds ? nullptr : c->kstates.p;
  a.kbuf = kbuf;
  a.pmat = cross ? c->pmat.p : nullptr;
  void *args[] = {&a};
  c->last_wpb = wpb;
  c->last_tw = tw;
  c->last_blocks = blocks;
  TimedLaunch tl(c, TK_KERNEL_KROTOV);
  if (c->cooperative) {
    TK_HIP(c, hipLaunchCooperativeKernel(kern, dim3(blocks), dim3(tk::kWave * c->var->G * wpb),
                                         args, lds, c->stream));
  } else {  // occupancy was checked above; a stalled grid ends at the spin limit
    TK_HIP(c, hipLaunchKernel(kern, dim3(blocks), dim3(tk::kWave * c->var->G * wpb), args, lds,
                              c->stream));
  }
  // new pulses become the current ones
  std::vector<double> unew(c->u.size());
  if (!unew.empty()) {
    TK_HIP(c, hipMemcpyAsync(unew.data(), c->u_new_dev.p, unew.size() * sizeof(double),
                             hipMemcpyDeviceToHost, c->stream));
  }
  TK_HIP(c, hipStreamSynchronize(c->stream));
  int rc = tl.finish(static_cast<int64_t>(M) * c->nt, pass_flops(c, unew.empty() ? c->u : unew, M),
                     static_cast<double>(c->nt) * M * c->d * c->bulk_cplx());
  if (rc) return rc;
  rc = check_kernel_errors(c);
  if (rc) return rc;
  if (!unew.empty()) {
    c->u = unew;
    TK_HIP(c, hipMemcpyAsync(c->u_dev.p, c->u_new_dev.p, unew.size() * sizeof(double),
                             hipMemcpyDeviceToDevice, c->stream));
  }
  c->tau_M = M;
  c->tau_seed = seed;
  c->tau_iter = static_cast<int64_t>(iteration);
  c->chi_M = -1;  // costates belong to the pulses before the update
  return TK_OK;
}

// Jump paths of the pathwise gradient: forward records (direction 0) of
// trajectories k < M, ordered per trajectory by ordinal, as offsets + arrays.
int build_paths(tk_ctx *c, int M, const tk_jump *rec, int64_t n_rec, std::vector<int> &off,
                std::vector<int> &step, std::vector<double> &t, std::vector<int> &op) {
  if (n_rec < 0 || (n_rec > 0 && !rec)) return fail(c, TK_EINVAL, "bad jump-record array");
  std::vector<const tk_jump *> use;
  for (int64_t q = 0; q < n_rec; ++q) {
    const tk_jump &r = rec[q];
    if (r.direction != 0) continue;
    if (r.traj < 0 || r.traj >= M) return fail(c, TK_EINVAL, "jump record of a trajectory >= M");
    if (r.step < 0 || r.step >= c->nt) return fail(c, TK_EINVAL, "jump record outside the grid");
    if (r.op < 0 || r.op >= c->n_jump) return fail(c, TK_EINVAL, "jump record with a bad operator");
    const double dt = c->T / c->nt, slack = 1e-9 * dt;
    if (!std::isfinite(r.t) || r.t < r.step * dt - slack || r.t > (r.step + 1) * dt + slack)
      return fail(c, TK_EINVAL, "jump time outside its step");
    use.push_back(&r);
  }
  std::sort(use.begin(), use.end(), [](const tk_jump *x, const tk_jump *y) {
    return std::make_tuple(x->traj, x->ordinal) < std::make_tuple(y->traj, y->ordinal);
  });
  off.assign(M + 1, 0);
  step.clear();
  t.clear();
  op.clear();
  for (size_t q = 0; q < use.size(); ++q) {
    const tk_jump &r = *use[q];
    if (q > 0 && use[q - 1]->traj == r.traj) {
      const tk_jump &p = *use[q - 1];
      if (p.ordinal == r.ordinal) return fail(c, TK_EINVAL, "duplicate jump ordinal");
      if (r.step < p.step || r.t < p.t) return fail(c, TK_EINVAL, "jump records out of time order");
    }
    off[r.traj + 1]++;
    step.push_back(r.step);
    t.push_back(r.t);
    op.push_back(r.op);
  }
  for (int k = 0; k < M; ++k) off[k + 1] += off[k];
  return TK_OK;
}

int run_grad(tk_ctx *c, int M, const tk_jump *rec, int64_t n_rec) {
  std::vector<int> off, step, op;
  std::vector<double> t;
  int rc = build_paths(c, M, rec, n_rec, off, step, t, op);
  if (rc) return rc;
  if ((rc = upload(c, c->path_off, off.data(), off.size() * sizeof(int)))) return rc;
  if ((rc = upload(c, c->path_step, step.data(), step.size() * sizeof(int)))) return rc;
  if ((rc = upload(c, c->path_t, t.data(), t.size() * sizeof(double)))) return rc;
  if ((rc = upload(c, c->path_op, op.data(), op.size() * sizeof(int)))) return rc;
  const void *kern = c->var->k_grad;
  if (!kern) return fail(c, TK_EUNSUPPORTED, "no gradient kernel for this variant");
  tk::PassArgs a = base_args(c, M, 0, 0, false);
  a.bc_max = 0.0;
  for (int i = 0; i < c->n_ctrl; ++i) a.bc_max = std::max(a.bc_max, c->bc[i]);
  a.kbuf = plan_kbuf_grad(c, c->u, a.bc_max);
  int wpb = 0;
  for (int w = c->var->G > 1 ? 1 : tk::kWavesPerBlock; w >= 1 && !wpb; w /= 2)
    if (tk::grad_lds_bytes(*c->var, w, a.kbuf) <= tk::kLdsBytes) wpb = w;
  if (!wpb) return fail(c, TK_EUNSUPPORTED, "the gradient's term vectors do not fit in LDS");
  const int blocks = (M + wpb - 1) / wpb;
  const size_t lds = tk::grad_lds_bytes(*c->var, wpb, a.kbuf);
  const size_t vec = static_cast<size_t>(c->var->R) * tk::kWave * c->var->G * c->bulk_cplx();
  const int nseg = (c->nt + tk::kGradCheckpoint - 1) / tk::kGradCheckpoint;
  TK_HIP(c, c->ckpt.ensure(static_cast<size_t>(M) * nseg * vec));
  TK_HIP(c, c->stash.ensure(static_cast<size_t>(blocks) * wpb * tk::kGradCheckpoint * vec));
  const size_t ng = static_cast<size_t>(c->n_ctrl) * c->nt;
  TK_HIP(c, c->gk.ensure(std::max<size_t>(ng * M, 1) * sizeof(double)));
  TK_HIP(c, c->dJdu.ensure(std::max<size_t>(ng, 1) * sizeof(double)));
  a.tau_out = c->tau.as<double>();
  a.a_scol = c->b_scol.as<int>();
  a.a_sval = c->b_sval.p;
  a.a_sdiag = c->b_sdiag.p;
  a.a_ccol = c->b_ccol.as<int>();
  a.a_cval = c->b_cval.p;
  a.ldcol = c->ldcol.as<int>();
  a.ldval = c->ldval.p;
  a.wld = c->wld;
  a.path_off = c->path_off.as<int>();
  a.path_step = c->path_step.as<int>();
  a.path_t = c->path_t.as<double>();
  a.path_op = c->path_op.as<int>();
  a.ckpt = c->ckpt.p;
  a.stash = c->stash.p;
  a.gk = c->gk.as<double>();
  TK_HIP(c, hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                static_cast<int>(lds)));
  void *args[] = {&a};
  TimedLaunch tl(c, TK_KERNEL_GRAD);
  TK_HIP(c, hipLaunchKernel(kern, dim3(blocks), dim3(tk::kWave * c->var->G * wpb), args, lds,
                            c->stream));
  // replay, segment recompute, the units' kept forward series and the
  // costate series (4 plain passes; the pairs of the two series are not
  // counted); bytes: checkpoints and the stash, written and read once, and
  // the per-trajectory terms
  const double bytes = 2.0 * M * nseg * c->d * c->bulk_cplx() +
                       2.0 * M * c->nt * c->d * c->bulk_cplx() + 8.0 * ng * M;
  rc = tl.finish(static_cast<int64_t>(M) * c->nt, 4.0 * pass_flops(c, c->u, M), bytes);
  if (rc) return rc;
  if (ng > 0) {
    const double *gp = c->gk.as<double>();
    double *op_ = c->dJdu.as<double>();
    int m = M;
    void *rargs[] = {&gp, &m, &op_};
    TK_HIP(c, hipLaunchKernel(tk::grad_reduce_kernel(), dim3(static_cast<unsigned>(ng)),
                              dim3(tk::kWave), rargs, 0, c->stream));
  }
  return TK_OK;
}

// J_T = 1 - (1/M) sum_k |tau_k|^2 into the context's device scalar, reduced
// on the device in a fixed order
int functional_device(tk_ctx *c, int M) {
  TK_HIP(c, c->jt_dev.ensure(sizeof(double)));
  const double *tp = c->tau.as<double>();
  double *jp = c->jt_dev.as<double>();
  int m = M;
  void *args[] = {&tp, &m, &jp};
  TK_HIP(c, hipLaunchKernel(tk::functional_kernel(), dim3(1), dim3(256), args, 0, c->stream));
  return TK_OK;
}

// J_T to host memory (J) or to device memory (J_dev); one of them is set
int functional_out(tk_ctx *c, int M, double *J, double *J_dev) {
  int rc = functional_device(c, M);
  if (rc) return rc;
  if (J_dev) {
    TK_HIP(c, hipMemcpyAsync(J_dev, c->jt_dev.p, sizeof(double), hipMemcpyDeviceToDevice,
                             c->stream));
    return TK_OK;
  }
  TK_HIP(c, hipMemcpyAsync(J, c->jt_dev.p, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  TK_HIP(c, hipStreamSynchronize(c->stream));
  return TK_OK;
}

int functional_value(tk_ctx *c, int M, double *J) { return functional_out(c, M, J, nullptr); }

// The context's stream waits for the work queued so far on a caller's stream
// (join_in), and the caller's stream for the context's work (join_out).  A
// null handle is the device's null stream; the context's own stream needs
// nothing.
int join_in(tk_ctx *c, hipStream_t s) {
  if (s == c->stream) return TK_OK;
  TK_HIP(c, hipEventRecord(c->ev_join, s));
  TK_HIP(c, hipStreamWaitEvent(c->stream, c->ev_join, 0));
  return TK_OK;
}

int join_out(tk_ctx *c, hipStream_t s) {
  if (s == c->stream) return TK_OK;
  TK_HIP(c, hipEventRecord(c->ev_join, c->stream));
  TK_HIP(c, hipStreamWaitEvent(s, c->ev_join, 0));
  return TK_OK;
}

// Validated pulses into the context: host mirror (planning of the step order
// and substeps, tk_get_pulses) and the padded [kMaxCtrl][nt] device copies.
// With `dev`, u, S and lambda are device pointers and the device copies are
// made device to device.
int store_pulses(tk_ctx *c, int32_t nt, double T, const double *u, const double *S,
                 const double *lambda, bool dev) {
  if (!c->has_system) return fail(c, TK_ESTATE, "no system set");
  if (nt < 1) return fail(c, TK_EINVAL, "nt must be >= 1");
  if (!(T > 0.0) || !std::isfinite(T)) return fail(c, TK_EINVAL, "T must be positive");
  const size_t n = static_cast<size_t>(c->n_ctrl) * nt;
  if (n > 0 && !u) return fail(c, TK_EINVAL, "u is NULL");
  std::vector<double> uu(n), ss(n, 1.0), ll(c->n_ctrl, 1.0);
  if (dev) {
    if (n > 0)
      TK_HIP(c, hipMemcpyAsync(uu.data(), u, n * sizeof(double), hipMemcpyDeviceToHost,
                               c->stream));
    if (S && n > 0)
      TK_HIP(c, hipMemcpyAsync(ss.data(), S, n * sizeof(double), hipMemcpyDeviceToHost,
                               c->stream));
    if (lambda && c->n_ctrl > 0)
      TK_HIP(c, hipMemcpyAsync(ll.data(), lambda, c->n_ctrl * sizeof(double),
                               hipMemcpyDeviceToHost, c->stream));
    TK_HIP(c, hipStreamSynchronize(c->stream));
  } else {
    if (n > 0) uu.assign(u, u + n);
    if (S) ss.assign(S, S + n);
    if (lambda) ll.assign(lambda, lambda + c->n_ctrl);
  }
  for (double x : uu)
    if (!std::isfinite(x)) return fail(c, TK_EINVAL, "non-finite pulse value");
  for (double x : ss)
    if (!std::isfinite(x) || x < 0.0 || x > 1.0) return fail(c, TK_EINVAL, "S must be in [0, 1]");
  for (double x : ll)
    if (!(x > 0.0) || !std::isfinite(x)) return fail(c, TK_EINVAL, "lambda must be positive");
  c->nt = nt;
  c->T = T;
  c->u = uu;
  c->S = ss;
  c->lam = ll;
  // device copies have kMaxCtrl rows: zero pulses and shapes, lambda 1 past n_ctrl
  const size_t rows = static_cast<size_t>(tk::kMaxCtrl) * nt;
  std::vector<double> up(rows, 0.0), sp(rows, 0.0), lp(tk::kMaxCtrl, 1.0);
  std::copy(uu.begin(), uu.end(), up.begin());
  std::copy(ss.begin(), ss.end(), sp.begin());
  std::copy(ll.begin(), ll.end(), lp.begin());
  int rc = upload(c, c->u_dev, up.data(), up.size() * sizeof(double));
  if (rc) return rc;
  if ((rc = upload(c, c->S_dev, sp.data(), sp.size() * sizeof(double)))) return rc;
  if ((rc = upload(c, c->lam_dev, lp.data(), lp.size() * sizeof(double)))) return rc;
  if (dev && n > 0) {  // the caller's device values themselves, bit for bit
    TK_HIP(c, hipMemcpyAsync(c->u_dev.p, u, n * sizeof(double), hipMemcpyDeviceToDevice,
                             c->stream));
    if (S)
      TK_HIP(c, hipMemcpyAsync(c->S_dev.p, S, n * sizeof(double), hipMemcpyDeviceToDevice,
                               c->stream));
    if (lambda)
      TK_HIP(c, hipMemcpyAsync(c->lam_dev.p, lambda, c->n_ctrl * sizeof(double),
                               hipMemcpyDeviceToDevice, c->stream));
  }
  c->has_pulses = true;
  c->chi_M = c->tau_M = -1;
  return TK_OK;
}

// Krotov iterations (tk_krotov_iterate); J_T values go to host memory (J_out)
// or, with J_on_device, to device memory.
int krotov_iterate_impl(tk_ctx *c, int32_t M, uint64_t seed, uint64_t first_iteration,
                        int32_t n_iter, double *J_out, bool J_on_device, tk_jump *rec,
                        int64_t cap, int64_t *n_rec, bool cross = false) {
  if (!rec) cap = 0;
  if (n_iter < 0) return fail(c, TK_EINVAL, "n_iter must be >= 0");
  if (!J_out) return fail(c, TK_EINVAL, "J_T_out is NULL");
  const bool cont_ok = c->tau_M == M && c->tau_seed == seed &&
                       c->tau_iter == static_cast<int64_t>(first_iteration) - 1;
  int rc = prepare_pass(c, M, cap);
  if (rc) return rc;
  if ((rc = reset_counters(c))) return rc;
  int out = 0;
  uint64_t n = first_iteration;
  auto put_J = [&]() {
    double *dst = J_out + out++;
    return functional_out(c, M, J_on_device ? nullptr : dst, J_on_device ? dst : nullptr);
  };
  if (first_iteration == 0) {
    if ((rc = run_forward(c, M, seed, 0, cap))) return rc;
    if ((rc = check_kernel_errors(c))) return rc;
    if ((rc = put_J())) return rc;
    n = 1;
  } else if (!cont_ok) {
    return fail(c, TK_ESTATE, "no forward pass of the previous iteration with this M and seed");
  }
  const uint64_t last = (first_iteration == 0 ? 0 : first_iteration - 1) + n_iter;
  for (; n <= last; ++n) {
    if ((rc = run_backward(c, M, seed, n, cap, cross))) return rc;
    if ((rc = check_kernel_errors(c))) return rc;
    if (cross && (rc = run_gram(c, M))) return rc;
    if ((rc = run_krotov(c, M, seed, n, cap, cross))) return rc;
    if ((rc = put_J())) return rc;
  }
  return fetch_records(c, rec, cap, n_rec);
}

// Pathwise gradient (tk_grad_pathwise); outputs to host or device memory.
int grad_impl(tk_ctx *c, int32_t M, const tk_jump *rec, int64_t n_rec, double *J_T,
              double *tau_out, double *dJdu, bool dev) {
  if (!J_T || !dJdu) return fail(c, TK_EINVAL, "J_T or dJdu is NULL");
  int rc = prepare_pass(c, M, 0);
  if (rc) return rc;
  if ((rc = reset_counters(c))) return rc;
  if ((rc = run_grad(c, M, rec, n_rec))) return rc;
  if ((rc = check_kernel_errors(c))) return rc;
  if ((rc = functional_out(c, M, dev ? nullptr : J_T, dev ? J_T : nullptr))) return rc;
  const size_t ng = static_cast<size_t>(c->n_ctrl) * c->nt;
  const hipMemcpyKind kind = dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (ng > 0) TK_HIP(c, hipMemcpyAsync(dJdu, c->dJdu.p, ng * sizeof(double), kind, c->stream));
  if (tau_out)
    TK_HIP(c, hipMemcpyAsync(tau_out, c->tau.p, 2 * static_cast<size_t>(M) * sizeof(double),
                             kind, c->stream));
  if (!dev) TK_HIP(c, hipStreamSynchronize(c->stream));
  c->tau_M = -1;  // the overlaps now belong to the replay, not to a forward pass
  return TK_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char *tk_version(void) { return "trajkrotov 0.2 (gfx950)"; }

#ifndef TK_BUILD_ID
#define TK_BUILD_ID "unknown"
#endif
const char *tk_build_id(void) { return TK_BUILD_ID; }

const char *tk_last_error(const tk_ctx *ctx) {
  if (!ctx) return "no context";
  return ctx->err.c_str();
}

int tk_create(tk_ctx **out, int device, int precision) {
  if (!out) return TK_EINVAL;
  *out = nullptr;
  if (precision != TK_FP64 && precision != TK_FP32) return TK_EINVAL;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return TK_ENODEV;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return TK_ENODEV;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return TK_ENODEV;
  tk_ctx *c = new (std::nothrow) tk_ctx();
  if (!c) return TK_ENOMEM;
  c->device = device;
  c->precision = precision;
  const char *launch = std::getenv("TK_KROTOV_LAUNCH");
  c->cooperative = !(launch && std::strcmp(launch, "plain") == 0);
  c->n_cu = prop.multiProcessorCount;
  if (hipSetDevice(device) != hipSuccess || hipStreamCreate(&c->stream) != hipSuccess ||
      hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess ||
      tk::scratch_setup(device) != hipSuccess) {
    tk_destroy(c);
    return TK_EHIP;
  }
  *out = c;
  return TK_OK;
}

void tk_destroy(tk_ctx *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
  if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
  if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
  if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

int tk_set_system(tk_ctx *c, int64_t d, const tk_csr *H0, int32_t n_ctrl, const tk_csr *H_ctrl,
                  int32_t n_jump, const tk_csr *L_jump) {
  if (!c) return TK_EINVAL;
  TK_HIP(c, hipSetDevice(c->device));
  c->has_system = c->has_states = c->has_pulses = false;
  c->chi_M = c->tau_M = -1;
  if (d < 1 || d > (1 << 24)) return fail(c, TK_EINVAL, "d out of range");
  if (n_ctrl < 0 || n_ctrl > tk::kMaxCtrl) return fail(c, TK_EINVAL, "n_ctrl out of range (0..8)");
  if (n_jump < 0 || n_jump > tk::kMaxJump) return fail(c, TK_EINVAL, "n_jump out of range (0..8)");
  if ((n_ctrl > 0 && !H_ctrl) || (n_jump > 0 && !L_jump))
    return fail(c, TK_EINVAL, "operator array is NULL");
  Csr h0;
  int rc = read_csr(c, H0, d, "H0", h0);
  if (rc) return rc;
  std::vector<Csr> hc(n_ctrl), lj(n_jump);
  for (int i = 0; i < n_ctrl; ++i)
    if ((rc = read_csr(c, &H_ctrl[i], d, "H_ctrl", hc[i]))) return rc;
  for (int l = 0; l < n_jump; ++l)
    if ((rc = read_csr(c, &L_jump[l], d, "L_jump", lj[l]))) return rc;
  if (!hermitian(h0)) return fail(c, TK_ENOTHERM, "H0 is not Hermitian");
  for (int i = 0; i < n_ctrl; ++i)
    if (!hermitian(hc[i])) return fail(c, TK_ENOTHERM, "a control Hamiltonian is not Hermitian");

  // static part of H_eff: A = H0 - (i/2) sum_l L_l^+ L_l
  Csr A = h0;
  for (int l = 0; l < n_jump; ++l) A = axpy(A, cd(0.0, -0.5), multiply(adjoint(lj[l]), lj[l]));
  Csr Ad = adjoint(A);
  std::vector<Csr> hcd(n_ctrl);
  for (int i = 0; i < n_ctrl; ++i) hcd[i] = adjoint(hc[i]);

  // the static slots hold the off-diagonal elements (the diagonal multiplies
  // the lane's own element, with no gather)
  std::vector<cd> diag_unused;
  const Csr Aoff0 = off_diagonal(A, diag_unused), Adoff0 = off_diagonal(Ad, diag_unused);
  const int ws = std::max(Aoff0.max_row(), Adoff0.max_row());
  // static off-diagonal non-zeros of each basis row in the forward or the
  // costate operator, and the basis in decreasing order of them (stable):
  // shapes with fewer static slots in row slots m >= 1 take the first 64 G
  // rows of this order as row slot 0
  std::vector<int> cnt(static_cast<size_t>(d));
  for (int64_t r = 0; r < d; ++r)
    cnt[r] = static_cast<int>(
        std::max(Aoff0.ptr[r + 1] - Aoff0.ptr[r], Adoff0.ptr[r + 1] - Adoff0.ptr[r]));
  std::vector<int32_t> order(static_cast<size_t>(d));
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t x, int32_t y) { return cnt[x] > cnt[y]; });
  // the most static non-zeros of a row outside the first `lanes` rows of the order
  auto rest_width = [&](int64_t lanes) { return d > lanes ? cnt[order[lanes]] : 0; };
  // typed shapes: the rows of row slot 0 (the first `lanes` of the order) hold
  // at most n_re real and n_im imaginary off-diagonal elements, none complex
  auto typed_fit = [&](int64_t lanes, int n_re, int n_im) {
    for (int64_t q = 0; q < std::min<int64_t>(lanes, d); ++q) {
      const int64_t r = order[static_cast<size_t>(q)];
      for (const Csr *m : {&Aoff0, &Adoff0}) {
        int re = 0, im = 0;
        for (int64_t p = m->ptr[r]; p < m->ptr[r + 1]; ++p) {
          const cd v = m->val[p];
          if (v.imag() == 0.0)
            ++re;
          else if (v.real() == 0.0)
            ++im;
          else
            return false;
        }
        if (re > n_re || im > n_im) return false;
      }
    }
    return true;
  };
  int wc = 1;
  for (int i = 0; i < n_ctrl; ++i) wc = std::max({wc, hc[i].max_row(), hcd[i].max_row()});
  int wl = 1, wld = 1;
  std::vector<Csr> ljd(n_jump);
  for (int l = 0; l < n_jump; ++l) {
    ljd[l] = adjoint(lj[l]);
    wl = std::max(wl, lj[l].max_row());
    wld = std::max(wld, ljd[l].max_row());
  }
  const int nc = n_ctrl * wc;
  // shapes for real control elements (two-FMA control slots) need every H_i
  // element real
  bool ctrl_real = true;
  for (int i = 0; i < n_ctrl; ++i)
    for (const cd &v : hc[i].val) ctrl_real = ctrl_real && v.imag() == 0.0;
  // the compiled variant with the fewest rows 64 G R >= d; among those, FP64
  // shapes with 4 rows per lane come last (they spill registers), then one-wave
  // teams, then the fewest static slots per lane, then the narrowest.
  // TK_VARIANT=<name> picks one by name instead.
  const char *want = std::getenv("TK_VARIANT");
  int nv = 0;
  const tk::Variant *vs = tk::variants(&nv);
  const tk::Variant *best = nullptr;
  auto key = [](const tk::Variant &v) {
    const int spills = v.precision == TK_FP64 && v.R >= 4 ? 1 : 0;
    return std::make_tuple(v.R * v.G, spills, v.G, v.WS + (v.R - 1) * v.WSB, v.WS, v.NC);
  };
  for (int k = 0; k < nv; ++k) {
    const tk::Variant &v = vs[k];
    if (v.precision != c->precision || static_cast<int64_t>(v.R) * tk::kWave * v.G < d ||
        v.WS < ws || v.NC < nc || (v.R > 1 && v.WSB < rest_width(int64_t{tk::kWave} * v.G)) ||
        (v.real_ctrl && !ctrl_real) ||
        (v.typed_imag >= 0 && !typed_fit(int64_t{tk::kWave} * v.G, v.WS - v.typed_imag, v.typed_imag)))
      continue;
    if (want && *want) {
      if (std::strcmp(want, v.name) == 0) best = &v;
      continue;
    }
    if (!best || key(v) < key(*best)) best = &v;
  }
  if (!best)
    return fail(c, TK_EUNSUPPORTED,
                "no compiled kernel variant for d=" + std::to_string(d) + " static width " +
                    std::to_string(ws) + " control slots " + std::to_string(nc) +
                    (want && *want ? std::string(" named ") + want : std::string()));
  // norm bounds of the step plan, from the operators in the basis order (the
  // estimate's start vector is fixed in that order)
  const double b0 = norm2_estimate(A);
  double bc[tk::kMaxCtrl];
  for (int i = 0; i < tk::kMaxCtrl; ++i) bc[i] = i < n_ctrl ? norm2_estimate(hc[i]) : 0.0;
  // device basis order: the order above for shapes with fewer static slots in
  // row slots m >= 1, else the basis itself; operators and states are
  // permuted once here and in tk_set_states, states going out are put back
  c->perm.clear();
  c->inv_perm.clear();
  if (best->WSB < best->WS) {
    c->perm = order;
    c->inv_perm.assign(static_cast<size_t>(d), 0);
    for (int64_t q = 0; q < d; ++q) c->inv_perm[order[q]] = static_cast<int32_t>(q);
    A = permute(A, c->perm, c->inv_perm);
    Ad = permute(Ad, c->perm, c->inv_perm);
    for (int i = 0; i < n_ctrl; ++i) {
      hc[i] = permute(hc[i], c->perm, c->inv_perm);
      hcd[i] = permute(hcd[i], c->perm, c->inv_perm);
    }
    for (int l = 0; l < n_jump; ++l) {
      lj[l] = permute(lj[l], c->perm, c->inv_perm);
      ljd[l] = permute(ljd[l], c->perm, c->inv_perm);
    }
  }
  c->var = best;
  c->d = d;
  c->n_ctrl = n_ctrl;
  c->n_jump = n_jump;
  c->wc = wc;
  c->wl = wl;
  c->wld = wld;
  c->H_ctrl_host = hc;
  c->A_host = A;
  c->L_host = lj;
  c->rho_ready = false;

  const int R = best->R;
  const int lanes = tk::kWave * best->G;
  // LDS bank groups of one complex element (32 banks of 4 bytes)
  const int nbg = c->precision == TK_FP64 ? 8 : 16;
  Ell e;
  const char *packing = "a row has more non-zeros than its slots";
  {
    // static parts in device order: off-diagonal slots and the diagonal
    std::vector<cd> dg, ddg;
    const Csr Aoff = off_diagonal(A, dg), Adoff = off_diagonal(Ad, ddg);
    const int typed_real = best->typed_imag >= 0 ? best->WS - best->typed_imag : -1;
    if (!pack({&Aoff}, best->WS, R, lanes, nbg, e, best->WSB, typed_real))
      return fail(c, TK_EINVAL, packing);
    if ((rc = upload_ell(c, e, c->f_scol, c->f_sval))) return rc;
    if (!pack({&Adoff}, best->WS, R, lanes, nbg, e, best->WSB, typed_real))
      return fail(c, TK_EINVAL, packing);
    if ((rc = upload_ell(c, e, c->b_scol, c->b_sval))) return rc;
    std::vector<double> v(2 * static_cast<size_t>(R) * lanes, 0.0);
    for (int64_t q = 0; q < d; ++q) {
      v[2 * q] = dg[q].real();
      v[2 * q + 1] = dg[q].imag();
    }
    if ((rc = upload_vec(c, c->f_sdiag, v))) return rc;
    for (int64_t q = 0; q < d; ++q) {
      v[2 * q] = ddg[q].real();
      v[2 * q + 1] = ddg[q].imag();
    }
    if ((rc = upload_vec(c, c->b_sdiag, v))) return rc;
  }
  if (!pack_ctrl(hc, wc, best->NC, R, lanes, nbg, e)) return fail(c, TK_EINVAL, packing);
  if ((rc = upload_ell(c, e, c->f_ccol, c->f_cval))) return rc;
  if (!pack_ctrl(hcd, wc, best->NC, R, lanes, nbg, e)) return fail(c, TK_EINVAL, packing);
  if ((rc = upload_ell(c, e, c->b_ccol, c->b_cval))) return rc;
  std::vector<const Csr *> lp;
  for (int l = 0; l < n_jump; ++l) lp.push_back(&lj[l]);
  if (lp.empty()) lp.push_back(nullptr);
  if (!pack(lp, wl, R, lanes, nbg, e)) return fail(c, TK_EINVAL, packing);
  if ((rc = upload_ell(c, e, c->lcol, c->lval))) return rc;
  std::vector<const Csr *> ldp;
  for (int l = 0; l < n_jump; ++l) ldp.push_back(&ljd[l]);
  if (ldp.empty()) ldp.push_back(nullptr);
  if (!pack(ldp, wld, R, lanes, nbg, e)) return fail(c, TK_EINVAL, packing);
  if ((rc = upload_ell(c, e, c->ldcol, c->ldval))) return rc;

  c->b0 = b0;
  for (int i = 0; i < tk::kMaxCtrl; ++i) c->bc[i] = bc[i];
  // algorithmic non-zeros of H_eff: union of the static and control patterns
  Csr pat = A;
  for (int i = 0; i < n_ctrl; ++i) {
    Csr ones = hc[i];
    for (auto &v : ones.val) v = cd(1.0, 0.0);
    Csr absA = pat;
    for (auto &v : absA.val) v = cd(std::abs(v), 0.0);
    pat = axpy(absA, cd(1.0, 0.0), ones);
  }
  c->nnz_heff = pat.nnz();
  c->has_system = true;
  return TK_OK;
}

int tk_set_states(tk_ctx *c, const double *psi0, const double *psi_tgt) {
  if (!c) return TK_EINVAL;
  if (!c->has_system) return fail(c, TK_ESTATE, "no system set");
  if (!psi0 || !psi_tgt) return fail(c, TK_EINVAL, "state pointer is NULL");
  TK_HIP(c, hipSetDevice(c->device));
  const int64_t d = c->d;
  const int64_t dpad = static_cast<int64_t>(c->var->R) * tk::kWave * c->var->G;
  double n0 = 0.0, nt = 0.0;
  for (int64_t i = 0; i < 2 * d; ++i) {
    if (!std::isfinite(psi0[i]) || !std::isfinite(psi_tgt[i]))
      return fail(c, TK_EINVAL, "non-finite state entry");
    n0 += psi0[i] * psi0[i];
    nt += psi_tgt[i] * psi_tgt[i];
  }
  if (std::fabs(std::sqrt(n0) - 1.0) > 1e-10) return fail(c, TK_EINVAL, "psi0 is not normalised");
  if (!(nt > 0.0)) return fail(c, TK_EINVAL, "target is zero");
  const double inv = 1.0 / std::sqrt(nt);
  std::vector<double> p(2 * dpad, 0.0), t(2 * dpad, 0.0);
  for (int64_t q = 0; q < d; ++q) {
    const int64_t r = c->perm.empty() ? q : c->perm[q];  // device row q holds basis row r
    p[2 * q] = psi0[2 * r];
    p[2 * q + 1] = psi0[2 * r + 1];
    t[2 * q] = psi_tgt[2 * r] * inv;
    t[2 * q + 1] = psi_tgt[2 * r + 1] * inv;
  }
  int rc = upload_vec(c, c->psi0_bulk, p);
  if (rc) return rc;
  if ((rc = upload(c, c->psi0_64, p.data(), p.size() * sizeof(double)))) return rc;
  if ((rc = upload_vec(c, c->tgt_bulk, t))) return rc;
  if ((rc = upload(c, c->tgt64, t.data(), t.size() * sizeof(double)))) return rc;
  c->has_states = true;
  c->chi_M = c->tau_M = -1;
  return TK_OK;
}

int tk_set_pulses(tk_ctx *c, int32_t nt, double T, const double *u, const double *S,
                  const double *lambda) {
  if (!c) return TK_EINVAL;
  TK_HIP(c, hipSetDevice(c->device));
  return store_pulses(c, nt, T, u, S, lambda, false);
}

int tk_get_pulses(const tk_ctx *c, double *u_out) {
  if (!c) return TK_EINVAL;
  if (!c->has_pulses) return fail(const_cast<tk_ctx *>(c), TK_ESTATE, "no pulses set");
  if (!u_out) return fail(const_cast<tk_ctx *>(c), TK_EINVAL, "u_out is NULL");
  std::copy(c->u.begin(), c->u.end(), u_out);
  return TK_OK;
}

int tk_propagate_forward(tk_ctx *c, int32_t M, uint64_t seed, uint64_t iteration, double *psiT_out,
                         double *tau_out, tk_jump *rec, int64_t cap, int64_t *n_rec) {
  if (!c) return TK_EINVAL;
  TK_HIP(c, hipSetDevice(c->device));
  if (!rec) cap = 0;
  int rc = prepare_pass(c, M, cap);
  if (rc) return rc;
  if ((rc = reset_counters(c))) return rc;
  if ((rc = run_forward(c, M, seed, iteration, cap))) return rc;
  if ((rc = check_kernel_errors(c))) return rc;
  if (tau_out)
    TK_HIP(c, hipMemcpy(tau_out, c->tau.p, 2 * static_cast<size_t>(M) * sizeof(double),
                        hipMemcpyDeviceToHost));
  if (psiT_out) {
    std::vector<unsigned char> buf(static_cast<size_t>(M) * c->d * c->bulk_cplx());
    TK_HIP(c, hipMemcpy(buf.data(), c->psiT.p, buf.size(), hipMemcpyDeviceToHost));
    to_host_cplx(c, buf.data(), static_cast<size_t>(M) * c->d, psiT_out);
    states_to_basis(c, psiT_out, static_cast<size_t>(M));
  }
  return fetch_records(c, rec, cap, n_rec);
}

int tk_propagate_backward(tk_ctx *c, int32_t M, uint64_t seed, uint64_t iteration,
                          const double *tau, tk_jump *rec, int64_t cap, int64_t *n_rec) {
  if (!c) return TK_EINVAL;
  TK_HIP(c, hipSetDevice(c->device));
  if (!rec) cap = 0;
  const bool had_tau = (c->tau_M == M);
  int rc = prepare_pass(c, M, cap);
  if (rc) return rc;
  if (tau) {
    for (int64_t i = 0; i < 2 * static_cast<int64_t>(M); ++i)
      if (!std::isfinite(tau[i])) return fail(c, TK_EINVAL, "non-finite tau");
    TK_HIP(c, hipMemcpy(c->tau.p, tau, 2 * static_cast<size_t>(M) * sizeof(double),
                        hipMemcpyHostToDevice));
  } else if (!had_tau) {
    return fail(c, TK_ESTATE, "no overlaps kept for this M; pass tau");
  }
  if ((rc = reset_counters(c))) return rc;
  if ((rc = run_backward(c, M, seed, iteration, cap))) return rc;
  if ((rc = check_kernel_errors(c))) return rc;
  return fetch_records(c, rec, cap, n_rec);
}

int tk_get_costate(const tk_ctx *cc, int32_t j, double *chi_out) {
  tk_ctx *c = const_cast<tk_ctx *>(cc);
  if (!c) return TK_EINVAL;
  if (c->chi_M < 1) return fail(c, TK_ESTATE, "no costates stored");
  if (j < 0 || j >= c->nt) return fail(c, TK_EINVAL, "time index out of range");
  if (!chi_out) return fail(c, TK_EINVAL, "chi_out is NULL");
  TK_HIP(c, hipSetDevice(c->device));
  const size_t n = static_cast<size_t>(c->chi_M) * c->d;
  std::vector<unsigned char> buf(n * c->bulk_cplx());
  const unsigned char *src = c->chi.as<unsigned char>() + static_cast<size_t>(j) * buf.size();
  TK_HIP(c, hipMemcpy(buf.data(), src, buf.size(), hipMemcpyDeviceToHost));
  to_host_cplx(c, buf.data(), n, chi_out);
  states_to_basis(c, chi_out, static_cast<size_t>(c->chi_M));
  return TK_OK;
}

int tk_functional(tk_ctx *c, int32_t M, uint64_t seed, uint64_t iteration, double *J_T,
                  double *tau_out) {
  if (!c) return TK_EINVAL;
  TK_HIP(c, hipSetDevice(c->device));
  if (!J_T) return fail(c, TK_EINVAL, "J_T is NULL");
  int rc = prepare_pass(c, M, 0);
  if (rc) return rc;
  if ((rc = reset_counters(c))) return rc;
  if ((rc = run_forward(c, M, seed, iteration, 0))) return rc;
  if ((rc = check_kernel_errors(c))) return rc;
  if ((rc = functional_value(c, M, J_T))) return rc;
  if (tau_out)
    TK_HIP(c, hipMemcpy(tau_out, c->tau.p, 2 * static_cast<size_t>(M) * sizeof(double),
                        hipMemcpyDeviceToHost));
  return TK_OK;
}

int tk_grad_pathwise(tk_ctx *c, int32_t M, const tk_jump *rec, int64_t n_rec, double *J_T,
                     double *tau_out, double *dJdu) {
  if (!c) return TK_EINVAL;
  TK_HIP(c, hipSetDevice(c->device));
  return grad_impl(c, M, rec, n_rec, J_T, tau_out, dJdu, false);
}

int tk_krotov_iterate(tk_ctx *c, int32_t M, uint64_t seed, uint64_t first_iteration,
                      int32_t n_iter, double *J_T_out, tk_jump *rec, int64_t cap,
                      int64_t *n_rec) {
  if (!c) return TK_EINVAL;
  TK_HIP(c, hipSetDevice(c->device));
  return krotov_iterate_impl(c, M, seed, first_iteration, n_iter, J_T_out, false, rec, cap,
                             n_rec);
}

int tk_krotov_iterate_cross(tk_ctx *c, int32_t M, uint64_t seed, uint64_t first_iteration,
                            int32_t n_iter, double *J_T_out, tk_jump *rec, int64_t cap,
                            int64_t *n_rec) {
  if (!c) return TK_EINVAL;
  TK_HIP(c, hipSetDevice(c->device));
  if (c->has_system &&
      !tk::cross_kernel(c->precision, c->var->R, c->var->ws_code, c->var->NC, c->var->G))
    return fail(c, TK_EUNSUPPORTED,
                "the cross-trajectory update runs one-wave kernel shapes only (d <= 256)");
  return krotov_iterate_impl(c, M, seed, first_iteration, n_iter, J_T_out, false, rec, cap,
                             n_rec, true);
}

// ---- device-pointer variants ---------------------------------------------------

int tk_set_pulses_dev(tk_ctx *c, int32_t nt, double T, const double *u, const double *S,
                      const double *lambda, tk_stream_t stream) {
  if (!c) return TK_EINVAL;
  TK_HIP(c, hipSetDevice(c->device));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int rc = join_in(c, s);
  if (!rc) rc = store_pulses(c, nt, T, u, S, lambda, true);
  const int rc2 = join_out(c, s);
  return rc ? rc : rc2;
}

int tk_get_pulses_dev(const tk_ctx *cc, double *u_out, tk_stream_t stream) {
  if (!cc) return TK_EINVAL;
  tk_ctx *c = const_cast<tk_ctx *>(cc);
  TK_HIP(c, hipSetDevice(c->device));
  if (!c->has_pulses) return fail(c, TK_ESTATE, "no pulses set");
  if (!u_out) return fail(c, TK_EINVAL, "u_out is NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int rc = join_in(c, s);
  if (rc) return rc;
  const size_t n = static_cast<size_t>(c->n_ctrl) * c->nt;
  if (n > 0)
    TK_HIP(c, hipMemcpyAsync(u_out, c->u_dev.p, n * sizeof(double), hipMemcpyDeviceToDevice,
                             c->stream));
  return join_out(c, s);
}

int tk_functional_dev(tk_ctx *c, int32_t M, uint64_t seed, uint64_t iteration, double *J_T,
                      double *tau_out, tk_stream_t stream) {
  if (!c) return TK_EINVAL;
  TK_HIP(c, hipSetDevice(c->device));
  if (!J_T) return fail(c, TK_EINVAL, "J_T is NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int rc = join_in(c, s);
  if (!rc) rc = prepare_pass(c, M, 0);
  if (!rc) rc = reset_counters(c);
  if (!rc) rc = run_forward(c, M, seed, iteration, 0);
  if (!rc) rc = check_kernel_errors(c);
  if (!rc) rc = functional_out(c, M, nullptr, J_T);
  if (!rc && tau_out) {
    const hipError_t e = hipMemcpyAsync(tau_out, c->tau.p, 2 * static_cast<size_t>(M) * sizeof(double),
                                        hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) rc = hip_fail(c, e, "hipMemcpyAsync(tau)");
  }
  const int rc2 = join_out(c, s);
  return rc ? rc : rc2;
}

int tk_krotov_iterate_dev(tk_ctx *c, int32_t M, uint64_t seed, uint64_t first_iteration,
                          int32_t n_iter, double *J_T_out, tk_stream_t stream) {
  if (!c) return TK_EINVAL;
  TK_HIP(c, hipSetDevice(c->device));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int rc = join_in(c, s);
  if (!rc)
    rc = krotov_iterate_impl(c, M, seed, first_iteration, n_iter, J_T_out, true, nullptr, 0,
                             nullptr);
  const int rc2 = join_out(c, s);
  return rc ? rc : rc2;
}

int tk_grad_pathwise_dev(tk_ctx *c, int32_t M, const tk_jump *rec, int64_t n_rec, double *J_T,
                         double *tau_out, double *dJdu, tk_stream_t stream) {
  if (!c) return TK_EINVAL;
  TK_HIP(c, hipSetDevice(c->device));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int rc = join_in(c, s);
  if (!rc) rc = grad_impl(c, M, rec, n_rec, J_T, tau_out, dJdu, true);
  const int rc2 = join_out(c, s);
  return rc ? rc : rc2;
}

// ---- the entry point that allocates nothing --------------------------------------

int tk_functional_dev_noalloc(tk_ctx *c, int32_t M, uint64_t seed, uint64_t iteration,
                              double *J_T, double *tau_out, tk_stream_t stream) {
  if (!c) return TK_EINVAL;
  TK_HIP(c, hipSetDevice(c->device));
  if (!c->has_system) return fail(c, TK_ESTATE, "no system set");
  if (!c->has_states) return fail(c, TK_ESTATE, "no states set");
  if (!c->has_pulses) return fail(c, TK_ESTATE, "no pulses set");
  if (!J_T) return fail(c, TK_EINVAL, "J_T is NULL");
  if (M < 1) return fail(c, TK_EINVAL, "M must be >= 1");
  if (M > tk::kScratchMaxTraj)
    return fail(c, TK_EINVAL, "M exceeds the fixed scratch of the no-allocation call (at most " +
                                  std::to_string(tk::kScratchMaxTraj) + " trajectories)");
  unsigned char *base = static_cast<unsigned char *>(tk::scratch_base(c->device));
  if (!base) return fail(c, TK_EHIP, "device scratch not set up");
  FixedBuffers fb;
  fb.err = reinterpret_cast<int *>(base + tk::kScratchErrOffset);
  fb.rec_count = reinterpret_cast<unsigned long long *>(base + tk::kScratchCountOffset);
  fb.rec = reinterpret_cast<tk_jump *>(base + tk::kScratchRecOffset);
  fb.tau = reinterpret_cast<double *>(base + tk::kScratchTauOffset);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int rc = join_in(c, s);
  if (rc) return rc;
  TK_HIP(c, tk::scratch_clear(base, c->stream));
  if ((rc = run_forward(c, M, seed, iteration, 0, &fb))) return rc;
  {  // J_T = 1 - (1/M) sum |tau_k|^2 straight into the caller's memory
    const double *tp = fb.tau;
    double *jp = J_T;
    int m = M;
    void *args[] = {&tp, &m, &jp};
    TK_HIP(c, hipLaunchKernel(tk::functional_kernel(), dim3(1), dim3(256), args, 0, c->stream));
  }
  if (tau_out)
    TK_HIP(c, hipMemcpyAsync(tau_out, fb.tau, 2 * static_cast<size_t>(M) * sizeof(double),
                             hipMemcpyDeviceToDevice, c->stream));
  rc = check_kernel_errors(c, fb.err);
  const int rc2 = join_out(c, s);
  return rc ? rc : rc2;
}

// ---- pulse-noise measure (Sec. 3.4) ------------------------------------------------

int tk_pulse_noise(tk_ctx *c, int32_t n_ctrl, int32_t nt, double T, const double *u,
                   double *nu_out) {
  if (!c) return TK_EINVAL;
  TK_HIP(c, hipSetDevice(c->device));
  if (!nu_out) return fail(c, TK_EINVAL, "nu_out is NULL");
  const double *src = nullptr;
  if (!u) {  // the context's current pulses
    if (!c->has_pulses) return fail(c, TK_ESTATE, "no pulses set");
    n_ctrl = c->n_ctrl;
    nt = c->nt;
    T = c->T;
    src = c->u_dev.as<double>();
  }
  if (n_ctrl < 1 || n_ctrl > tk::kMaxCtrl) return fail(c, TK_EINVAL, "n_ctrl must be in [1, 8]");
  if (nt < 5) return fail(c, TK_EINVAL, "the five-point filter needs nt >= 5");
  if (!(T > 0.0) || !std::isfinite(T)) return fail(c, TK_EINVAL, "T must be positive");
  const size_t n = static_cast<size_t>(n_ctrl) * nt;
  if (u) {
    for (size_t q = 0; q < n; ++q)
      if (!std::isfinite(u[q])) return fail(c, TK_EINVAL, "non-finite pulse value");
    int rc = upload(c, c->noise_u, u, n * sizeof(double));
    if (rc) return rc;
    src = c->noise_u.as<double>();
  }
  TK_HIP(c, c->noise_nu.ensure(tk::kMaxCtrl * sizeof(double)));
  TK_HIP(c, tk::launch_pulse_noise(src, n_ctrl, nt, T / nt, c->noise_nu.as<double>(), c->stream));
  TK_HIP(c, hipMemcpyAsync(nu_out, c->noise_nu.p, n_ctrl * sizeof(double), hipMemcpyDeviceToHost,
                           c->stream));
  TK_HIP(c, hipStreamSynchronize(c->stream));
  return TK_OK;
}

// ---- dense matrix-core step against the sparse step ------------------------------

int tk_step_bench(tk_ctx *c, int32_t method, int32_t M, int32_t K, const double *x, double *y,
                  int32_t reps, double *ms_per_launch) {
  if (!c) return TK_EINVAL;
  TK_HIP(c, hipSetDevice(c->device));
  if (!c->has_system || !c->has_pulses) return fail(c, TK_ESTATE, "no system or pulses set");
  if (method != TK_STEP_SPARSE && method != TK_STEP_DENSE_MFMA)
    return fail(c, TK_EINVAL, "unknown step method");
  if (M < 1 || K < 1 || K > tk::kMaxTaylor || reps < 1 || !x)
    return fail(c, TK_EINVAL, "need M >= 1, 1 <= K <= 40, reps >= 1 and x");
  const int d = static_cast<int>(c->d);
  const size_t n = static_cast<size_t>(M) * d;
  for (size_t q = 0; q < 2 * n; ++q)
    if (!std::isfinite(x[q])) return fail(c, TK_EINVAL, "non-finite state");
  const bool fp64 = c->precision == TK_FP64;
  const size_t cb = c->bulk_cplx();
  {
    std::vector<double> xd(x, x + 2 * n);
    states_to_device(c, xd.data(), static_cast<size_t>(M));
    int rc;
    if (fp64) {
      rc = upload(c, c->bench_x, xd.data(), 2 * n * sizeof(double));
    } else {
      std::vector<float> xf(xd.begin(), xd.end());
      rc = upload(c, c->bench_x, xf.data(), 2 * n * sizeof(float));
    }
    if (rc) return rc;
  }
  TK_HIP(c, c->bench_y.ensure(n * cb));
  const void *kern = nullptr;
  dim3 grid, block;
  size_t lds = 0;
  std::vector<void *> args;
  tk::PassArgs a;
  int Kk = K, Dp = (d + 15) / 16 * 16, m = M, dd = d;
  double tau = c->T / c->nt;
  const void *xp = c->bench_x.p;
  void *yp = c->bench_y.p;
  const void *hp = nullptr;
  if (method == TK_STEP_SPARSE) {
    kern = tk::sparse_step_kernel(c->precision, c->var->R, c->var->ws_code, c->var->NC,
                                  c->var->G);
    if (!kern) return fail(c, TK_EUNSUPPORTED, "the sparse step runs one-wave kernel shapes only");
    a = base_args(c, M, 0, 0, false);
    a.kbuf = 2;
    lds = tk::block_lds_bytes(*c->var, tk::kWavesPerBlock, 2, 0);
    grid = dim3((M + tk::kWavesPerBlock - 1) / tk::kWavesPerBlock);
    block = dim3(tk::kWave * tk::kWavesPerBlock);
    args = {&a, &Kk, &xp, &yp};
  } else {
    if (Dp > 256) return fail(c, TK_EUNSUPPORTED, "the dense step takes d <= 256");
    // dense H_eff(u_0) = H0 - (i/2) sum L^+L + sum_i u_i0 H_i, padded to Dp
    std::vector<cd> Hd(static_cast<size_t>(Dp) * Dp, cd(0.0, 0.0));
    for (int64_t r = 0; r < c->A_host.n; ++r)
      for (int64_t p = c->A_host.ptr[r]; p < c->A_host.ptr[r + 1]; ++p)
        Hd[static_cast<size_t>(r) * Dp + c->A_host.idx[p]] += c->A_host.val[p];
    for (int i = 0; i < c->n_ctrl; ++i) {
      const tkh::Csr &h = c->H_ctrl_host[i];
      const double ui = c->u[static_cast<size_t>(i) * c->nt];
      for (int64_t r = 0; r < h.n; ++r)
        for (int64_t p = h.ptr[r]; p < h.ptr[r + 1]; ++p)
          Hd[static_cast<size_t>(r) * Dp + h.idx[p]] += ui * h.val[p];
    }
    int rc;
    if (fp64) {
      rc = upload(c, c->bench_h, Hd.data(), Hd.size() * sizeof(cd));
    } else {
      std::vector<float> hf(2 * Hd.size());
      for (size_t q = 0; q < Hd.size(); ++q) {
        hf[2 * q] = static_cast<float>(Hd[q].real());
        hf[2 * q + 1] = static_cast<float>(Hd[q].imag());
      }
      rc = upload(c, c->bench_h, hf.data(), hf.size() * sizeof(float));
    }
    if (rc) return rc;
    hp = c->bench_h.p;
    const int NT = fp64 ? (Dp <= 128 ? 2 : 1) : (Dp <= 128 ? 4 : 2);
    kern = tk::dense_step_kernel(c->precision, NT);
    lds = static_cast<size_t>(4) * Dp * 16 * NT * (fp64 ? 8 : 4);
    grid = dim3((M + 16 * NT - 1) / (16 * NT));
    block = dim3(256);
    args = {&hp, &dd, &Dp, &m, &Kk, &tau, &xp, &yp};
  }
  TK_HIP(c, hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                static_cast<int>(lds)));
  TK_HIP(c, hipLaunchKernel(kern, grid, block, args.data(), lds, c->stream));  // warm-up
  TK_HIP(c, hipEventRecord(c->ev0, c->stream));
  for (int r = 0; r < reps; ++r)
    TK_HIP(c, hipLaunchKernel(kern, grid, block, args.data(), lds, c->stream));
  TK_HIP(c, hipEventRecord(c->ev1, c->stream));
  TK_HIP(c, hipEventSynchronize(c->ev1));
  float ms = 0.f;
  TK_HIP(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
  if (ms_per_launch) *ms_per_launch = ms / reps;
  if (y) {
    std::vector<unsigned char> buf(n * cb);
    TK_HIP(c, hipMemcpy(buf.data(), c->bench_y.p, n * cb, hipMemcpyDeviceToHost));
    to_host_cplx(c, buf.data(), n, y);
    states_to_basis(c, y, static_cast<size_t>(M));
  }
  return TK_OK;
}

// ---- density-matrix passes (Sec. 2.2) ---------------------------------------------

}  // extern "C"

namespace {

// CSR copy of a host operator on the device (int row pointers, complex128 values)
int upload_csr(tk_ctx *c, const Csr &m, DevBuf *b) {
  std::vector<int> p(m.ptr.begin(), m.ptr.end());
  std::vector<int> ix(m.idx.begin(), m.idx.end());
  if (ix.empty()) ix.push_back(0);
  std::vector<cd> v(m.val.begin(), m.val.end());
  if (v.empty()) v.push_back(cd(0.0, 0.0));
  int rc = upload(c, b[0], p.data(), p.size() * sizeof(int));
  if (!rc) rc = upload(c, b[1], ix.data(), ix.size() * sizeof(int));
  if (!rc) rc = upload(c, b[2], v.data(), v.size() * sizeof(cd));
  return rc;
}

tk::RhoCsr csr_view(const DevBuf *b) {
  tk::RhoCsr r;
  r.ptr = b[0].as<int>();
  r.idx = b[1].as<int>();
  r.val = b[2].p;
  return r;
}

// Arguments of a density-matrix pass; the operators are uploaded once per
// system: three buffers each for A, A^+, H_0 .. H_7, L_0 .. L_7, L_0^+ .. L_7^+.
int rho_args(tk_ctx *c, bool backward, tk::RhoArgs &a) {
  if (!c->has_system || !c->has_states || !c->has_pulses)
    return fail(c, TK_ESTATE, "system, states and pulses must be set");
  std::memset(&a, 0, sizeof(a));
  const int d = static_cast<int>(c->d);
  auto slot = [&](int q) { return &c->rho_csr[3 * q]; };
  constexpr int kH = 2, kL = 2 + tk::kMaxCtrl, kLd = 2 + tk::kMaxCtrl + tk::kMaxJump;
  if (!c->rho_ready) {
    int rc = upload_csr(c, c->A_host, slot(0));
    if (!rc) rc = upload_csr(c, adjoint(c->A_host), slot(1));
    for (int i = 0; i < c->n_ctrl && !rc; ++i) rc = upload_csr(c, c->H_ctrl_host[i], slot(kH + i));
    for (int l = 0; l < c->n_jump && !rc; ++l) {
      rc = upload_csr(c, c->L_host[l], slot(kL + l));
      if (!rc) rc = upload_csr(c, adjoint(c->L_host[l]), slot(kLd + l));
    }
    if (rc) return rc;
    c->rho_bj = 0.0;
    for (int l = 0; l < c->n_jump; ++l) {
      const double nl = norm2_estimate(c->L_host[l]);
      c->rho_bj += nl * nl;
    }
    c->rho_ready = true;
  }
  const size_t n2 = static_cast<size_t>(d) * d;
  const int ny = std::max(c->n_jump, 1);
  TK_HIP(c, c->rho_work.ensure((4 + ny) * n2 * sizeof(cd)));
  cd *w = c->rho_work.as<cd>();
  a.d = d;
  a.nt = c->nt;
  a.n_ctrl = c->n_ctrl;
  a.n_jump = c->n_jump;
  a.dt = c->T / c->nt;
  a.B = csr_view(slot(backward ? 1 : 0));
  for (int i = 0; i < c->n_ctrl; ++i) a.H[i] = csr_view(slot(kH + i));
  for (int l = 0; l < c->n_jump; ++l) a.J[l] = csr_view(slot((backward ? kLd : kL) + l));
  a.s = backward ? 1.0 : -1.0;
  a.gen_b0 = 2.0 * c->b0;
  for (int i = 0; i < tk::kMaxCtrl; ++i) a.gen_bc[i] = 2.0 * c->bc[i];
  a.gen_bj = c->rho_bj;
  std::memcpy(a.ord_x, order_table(TK_FP64), sizeof(a.ord_x));
  a.kmax = tk::kMaxTaylor;
  a.u = c->u_dev.as<double>();
  a.Q0 = w;
  a.Q1 = w + n2;
  a.R = w + 2 * n2;
  a.X = w + 3 * n2;
  a.Y = w + 4 * n2;
  a.tgt = c->tgt64.p;
  a.start = backward ? c->tgt64.p : c->psi0_64.p;
  a.err = c->err_dev.as<int>();
  return TK_OK;
}

int rho_run(tk_ctx *c, const tk::RhoArgs &a, int dir) {
  TK_HIP(c, tk::launch_rho_pass(a, dir, c->stream));
  return check_kernel_errors(c);
}

}  // namespace

extern "C" {

int tk_density_functional(tk_ctx *c, double *J_T) {
  if (!c) return TK_EINVAL;
  TK_HIP(c, hipSetDevice(c->device));
  if (!J_T) return fail(c, TK_EINVAL, "J_T is NULL");
  TK_HIP(c, c->err_dev.ensure(sizeof(int)));
  TK_HIP(c, c->jt_dev.ensure(sizeof(double)));
  TK_HIP(c, hipMemsetAsync(c->err_dev.p, 0, sizeof(int), c->stream));
  tk::RhoArgs a;
  int rc = rho_args(c, false, a);
  if (rc) return rc;
  a.J_out = c->jt_dev.as<double>();
  if ((rc = rho_run(c, a, 0))) return rc;
  TK_HIP(c, hipMemcpy(J_T, c->jt_dev.p, sizeof(double), hipMemcpyDeviceToHost));
  return TK_OK;
}

int tk_density_krotov_iterate(tk_ctx *c, int32_t n_iter, double *J_T_out) {
  if (!c) return TK_EINVAL;
  TK_HIP(c, hipSetDevice(c->device));
  if (!J_T_out) return fail(c, TK_EINVAL, "J_T_out is NULL");
  if (n_iter < 0) return fail(c, TK_EINVAL, "n_iter must be >= 0");
  TK_HIP(c, c->err_dev.ensure(sizeof(int)));
  TK_HIP(c, c->jt_dev.ensure(sizeof(double)));
  TK_HIP(c, hipMemsetAsync(c->err_dev.p, 0, sizeof(int), c->stream));
  int rc = tk_density_functional(c, &J_T_out[0]);
  if (rc) return rc;
  const size_t n2 = static_cast<size_t>(c->d) * c->d;
  TK_HIP(c, c->rho_P.ensure(static_cast<size_t>(c->nt) * n2 * sizeof(cd)));
  TK_HIP(c, c->u_new_dev.ensure(static_cast<size_t>(tk::kMaxCtrl) * c->nt * sizeof(double)));
  for (int n = 1; n <= n_iter; ++n) {
    tk::RhoArgs b;
    if ((rc = rho_args(c, true, b))) return rc;
    b.store = c->rho_P.p;
    if ((rc = rho_run(c, b, 1))) return rc;
    tk::RhoArgs f;
    if ((rc = rho_args(c, false, f))) return rc;
    f.P = c->rho_P.p;
    f.u_old = c->u_dev.as<double>();
    f.S = c->S_dev.as<double>();
    f.lam = c->lam_dev.as<double>();
    f.u_new = c->u_new_dev.as<double>();
    f.J_out = c->jt_dev.as<double>();
    TK_HIP(c, hipMemcpyAsync(c->u_new_dev.p, c->u_dev.p,
                             static_cast<size_t>(tk::kMaxCtrl) * c->nt * sizeof(double),
                             hipMemcpyDeviceToDevice, c->stream));
    if ((rc = rho_run(c, f, 0))) return rc;
    TK_HIP(c, hipMemcpy(&J_T_out[n], c->jt_dev.p, sizeof(double), hipMemcpyDeviceToHost));
    // the updated pulses become the current ones (device and host mirror)
    TK_HIP(c, hipMemcpyAsync(c->u_dev.p, c->u_new_dev.p,
                             static_cast<size_t>(tk::kMaxCtrl) * c->nt * sizeof(double),
                             hipMemcpyDeviceToDevice, c->stream));
    if (!c->u.empty())
      TK_HIP(c, hipMemcpy(c->u.data(), c->u_new_dev.p, c->u.size() * sizeof(double),
                          hipMemcpyDeviceToHost));
    c->chi_M = c->tau_M = -1;
  }
  return TK_OK;
}

int tk_set_timing(tk_ctx *c, int enable) {
  if (!c) return TK_EINVAL;
  c->timing = enable != 0;
  return TK_OK;
}

int tk_get_timing(const tk_ctx *c, int kind, tk_kernel_timing *out) {
  if (!c || !out || kind < 0 || kind >= TK_KERNEL_COUNT) return TK_EINVAL;
  *out = c->tstat[kind];
  return TK_OK;
}

int tk_reset_timing(tk_ctx *c) {
  if (!c) return TK_EINVAL;
  for (auto &t : c->tstat) t = tk_kernel_timing{};
  return TK_OK;
}

int tk_get_launch_info(const tk_ctx *c, const char **variant, int32_t *waves_per_block,
                       int32_t *traj_per_wave, int32_t *blocks) {
  if (!c) return TK_EINVAL;
  if (variant) *variant = c->var ? c->var->name : "";
  if (waves_per_block) *waves_per_block = c->last_wpb;
  if (traj_per_wave) *traj_per_wave = c->last_tw;
  if (blocks) *blocks = c->last_blocks;
  return TK_OK;
}

}  // extern "C"
