// Host side of libtrajkrotov: validation, operator packing, device memory,
// kernel launches and the Krotov iteration driver.
#include <hip/hip_runtime.h>

#include <algorithm>
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
void pack_group(const Csr *a, int W, int first, int R, int lanes, int n_bank_groups,
                int32_t dummy, std::vector<int32_t> &col, std::vector<double> &val) {
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
          if (l.empty()) {
            col[slot] = dummy;
            val[2 * slot] = val[2 * slot + 1] = 0.0;
            if (!dummy_used) load[dummy % n_bank_groups]++;
            dummy_used = true;
            continue;
          }
          size_t best = 0;
          for (size_t q = 1; q < l.size(); ++q) {
            const int lb = load[l[best].first % n_bank_groups], lq = load[l[q].first % n_bank_groups];
            if (lq < lb || (lq == lb && l[q].first < l[best].first)) best = q;
          }
          col[slot] = l[best].first;
          val[2 * slot] = l[best].second.real();
          val[2 * slot + 1] = l[best].second.imag();
          load[l[best].first % n_bank_groups]++;
          l.erase(l.begin() + static_cast<long>(best));
        }
      }
}

// Operators ops[g], each in W slots: layout [g][w][m][lane], `lanes` lanes
// (64 G) per row slot m.
void pack(const std::vector<const Csr *> &ops, int W, int R, int lanes, int n_bank_groups,
          Ell &out) {
  const size_t n = ops.size() * static_cast<size_t>(W) * R * lanes;
  out.col.assign(n, 0);
  out.val.assign(2 * n, 0.0);
  const int32_t dummy = R * lanes;
  for (size_t g = 0; g < ops.size(); ++g)
    pack_group(ops[g], W, static_cast<int>(g) * W, R, lanes, n_bank_groups, dummy, out.col,
               out.val);
}

// Control operators: slots c = i * wc .. i * wc + wc - 1 hold H_i; slots past
// n_ctrl * wc are padding.
void pack_ctrl(const std::vector<Csr> &H, int wc, int NC, int R, int lanes, int n_bank_groups,
               Ell &out) {
  const size_t n = static_cast<size_t>(NC) * R * lanes;
  out.col.assign(n, 0);
  out.val.assign(2 * n, 0.0);
  const int32_t dummy = R * lanes;
  for (int i = 0; i * wc < NC; ++i) {
    const Csr *a = i < static_cast<int>(H.size()) ? &H[i] : nullptr;
    pack_group(a, std::min(wc, NC - i * wc), i * wc, R, lanes, n_bank_groups, dummy, out.col,
               out.val);
  }
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
  static const OrderTable t64(1e-16), t32(6e-8);
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
  return std::min(kmax + 1 + margin, tk::kMaxTaylor + 1);
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
  a.tol = c->precision == TK_FP64 ? 1e-16 : 6e-8;
  a.ftol = c->precision == TK_FP64 ? 4.0 * 0x1.0p-52 : 4.0 * 0x1.0p-23;
  a.b0 = c->b0;
  for (int i = 0; i < tk::kMaxCtrl; ++i) a.bc[i] = c->bc[i];
  a.inv_n[0] = 0.0;
  for (int n = 1; n <= tk::kMaxTaylor; ++n) a.inv_n[n] = 1.0 / n;
  std::memcpy(a.ord_x, order_table(c->precision), sizeof(a.ord_x));
  if (!backward) {
    a.scol = c->f_scol.as<int>();
    a.sval = c->f_sval.p;
    a.ccol = c->f_ccol.as<int>();
    a.cval = c->f_cval.p;
    a.psi_start = c->psi0_bulk.p;
  } else {
    a.scol = c->b_scol.as<int>();
    a.sval = c->b_sval.p;
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

int check_kernel_errors(tk_ctx *c) {
  int e = 0;
  TK_HIP(c, hipMemcpyAsync(&e, c->err_dev.p, sizeof(int), hipMemcpyDeviceToHost, c->stream));
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

int run_forward(tk_ctx *c, int M, uint64_t seed, uint64_t iteration, int64_t cap) {
  tk::PassArgs a = base_args(c, M, seed, iteration, false);
  a.psiT = c->psiT.p;
  a.tau_out = c->tau.as<double>();
  a.rec = c->rec.as<tk_jump>();
  a.rec_cap = cap;
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
  c->tau_M = M;
  c->tau_seed = seed;
  c->tau_iter = static_cast<int64_t>(iteration);
  return TK_OK;
}

int run_backward(tk_ctx *c, int M, uint64_t seed, uint64_t iteration, int64_t cap) {
  const size_t chi_bytes = static_cast<size_t>(c->nt) * M * c->d * c->bulk_cplx();
  c->chi_M = -1;
  TK_HIP(c, c->chi.ensure(chi_bytes));
  tk::PassArgs a = base_args(c, M, seed, iteration, true);
  a.tau_in = c->tau.as<double>();
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

int run_krotov(tk_ctx *c, int M, uint64_t seed, uint64_t iteration, int64_t cap) {
  if (c->chi_M != M) return fail(c, TK_ESTATE, "no costates stored for this M");
  // pulses grow during the pass: one spare term vector; the kernel adds
  // substeps if a step would still need more terms
  const int kbuf = plan_kbuf(c, c->u, 1);
  int tw = 0, wpb = 0, blocks = 0;
  size_t lds = 0;
  for (int t = 1; t <= 64 && !tw; ++t)
    for (int w = c->var->G > 1 ? 1 : tk::kWavesPerBlock; w >= 1; w /= 2) {
      const int b = (M + w * t - 1) / (w * t);
      const size_t l = tk::block_lds_bytes(*c->var, w, kbuf, t);
      if (b > tk::kMaxBlocks || l > tk::kLdsBytes) continue;
      TK_HIP(c, hipFuncSetAttribute(c->var->k_krotov, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    static_cast<int>(l)));
      int occ = 0;
      TK_HIP(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, c->var->k_krotov, tk::kWave * c->var->G * w,
                                                              l));
      if (occ > 0 && static_cast<int64_t>(occ) * c->n_cu >= b) {
        tw = t;
        wpb = w;
        blocks = b;
        lds = l;
        break;
      }
    }
  if (!tw) return fail(c, TK_EUNSUPPORTED, "too many trajectories for one cooperative launch");
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
  a.kbuf = kbuf;
  void *args[] = {&a};
  c->last_wpb = wpb;
  c->last_tw = tw;
  c->last_blocks = blocks;
  TimedLaunch tl(c, TK_KERNEL_KROTOV);
  if (c->cooperative) {
    TK_HIP(c, hipLaunchCooperativeKernel(c->var->k_krotov, dim3(blocks),
                                         dim3(tk::kWave * c->var->G * wpb), args, lds, c->stream));
  } else {  // occupancy was checked above; a stalled grid ends at the spin limit
    TK_HIP(c, hipLaunchKernel(c->var->k_krotov, dim3(blocks), dim3(tk::kWave * c->var->G * wpb), args, lds,
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
  a.a_ccol = c->b_ccol.as<int>();
  a.a_cval = c->b_cval.p;
  a.ldcol = c->ldcol.as<int>();
  a.ldval = c->ldval.p;
  a.wld = c->wld;
  a.bc_max = 0.0;
  for (int i = 0; i < c->n_ctrl; ++i) a.bc_max = std::max(a.bc_max, c->bc[i]);
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
  // replay, recompute and adjoint sweeps (3 plain passes) plus the augmented
  // series (1 + n_ctrl chains); bytes: checkpoints and the stash, written and
  // read once, and the per-trajectory terms
  const double bytes = 2.0 * M * nseg * c->d * c->bulk_cplx() +
                       2.0 * M * c->nt * c->d * c->bulk_cplx() + 8.0 * ng * M;
  rc = tl.finish(static_cast<int64_t>(M) * c->nt, (4.0 + c->n_ctrl) * pass_flops(c, c->u, M), bytes);
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

int functional_value(tk_ctx *c, int M, double *J) {
  // J_T = 1 - (1/M) sum_k |tau_k|^2, reduced on the device in a fixed order
  TK_HIP(c, c->jt_dev.ensure(sizeof(double)));
  const double *tp = c->tau.as<double>();
  double *jp = c->jt_dev.as<double>();
  int m = M;
  void *args[] = {&tp, &m, &jp};
  TK_HIP(c, hipLaunchKernel(tk::functional_kernel(), dim3(1), dim3(256), args, 0, c->stream));
  TK_HIP(c, hipMemcpyAsync(J, jp, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  TK_HIP(c, hipStreamSynchronize(c->stream));
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
      hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess) {
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
  const Csr Ad = adjoint(A);
  std::vector<Csr> hcd(n_ctrl);
  for (int i = 0; i < n_ctrl; ++i) hcd[i] = adjoint(hc[i]);

  const int ws = std::max(A.max_row(), Ad.max_row());
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
  // the compiled variant with the fewest rows 64 G R >= d; among those, FP64
  // shapes with 4 rows per lane come last (they spill registers), then one-wave
  // teams, then the narrowest slots.
  // TK_VARIANT=<name> picks one by name instead.
  const char *want = std::getenv("TK_VARIANT");
  int nv = 0;
  const tk::Variant *vs = tk::variants(&nv);
  const tk::Variant *best = nullptr;
  auto key = [](const tk::Variant &v) {
    const int spills = v.precision == TK_FP64 && v.R >= 4 ? 1 : 0;
    return std::make_tuple(v.R * v.G, spills, v.G, v.WS, v.NC);
  };
  for (int k = 0; k < nv; ++k) {
    const tk::Variant &v = vs[k];
    if (v.precision != c->precision || static_cast<int64_t>(v.R) * tk::kWave * v.G < d ||
        v.WS < ws || v.NC < nc)
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
  c->var = best;
  c->d = d;
  c->n_ctrl = n_ctrl;
  c->n_jump = n_jump;
  c->wc = wc;
  c->wl = wl;
  c->wld = wld;
  c->H_ctrl_host = hc;

  const int R = best->R;
  const int lanes = tk::kWave * best->G;
  // LDS bank groups of one complex element (32 banks of 4 bytes)
  const int nbg = c->precision == TK_FP64 ? 8 : 16;
  Ell e;
  pack({&A}, best->WS, R, lanes, nbg, e);
  if ((rc = upload_ell(c, e, c->f_scol, c->f_sval))) return rc;
  pack({&Ad}, best->WS, R, lanes, nbg, e);
  if ((rc = upload_ell(c, e, c->b_scol, c->b_sval))) return rc;
  pack_ctrl(hc, wc, best->NC, R, lanes, nbg, e);
  if ((rc = upload_ell(c, e, c->f_ccol, c->f_cval))) return rc;
  pack_ctrl(hcd, wc, best->NC, R, lanes, nbg, e);
  if ((rc = upload_ell(c, e, c->b_ccol, c->b_cval))) return rc;
  std::vector<const Csr *> lp;
  for (int l = 0; l < n_jump; ++l) lp.push_back(&lj[l]);
  if (lp.empty()) lp.push_back(nullptr);
  pack(lp, wl, R, lanes, nbg, e);
  if ((rc = upload_ell(c, e, c->lcol, c->lval))) return rc;
  std::vector<const Csr *> ldp;
  for (int l = 0; l < n_jump; ++l) ldp.push_back(&ljd[l]);
  if (ldp.empty()) ldp.push_back(nullptr);
  pack(ldp, wld, R, lanes, nbg, e);
  if ((rc = upload_ell(c, e, c->ldcol, c->ldval))) return rc;

  c->b0 = norm2_estimate(A);
  for (int i = 0; i < tk::kMaxCtrl; ++i) c->bc[i] = i < n_ctrl ? norm2_estimate(hc[i]) : 0.0;
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
  for (int64_t i = 0; i < 2 * d; ++i) {
    p[i] = psi0[i];
    t[i] = psi_tgt[i] * inv;
  }
  int rc = upload_vec(c, c->psi0_bulk, p);
  if (rc) return rc;
  if ((rc = upload_vec(c, c->tgt_bulk, t))) return rc;
  if ((rc = upload(c, c->tgt64, t.data(), t.size() * sizeof(double)))) return rc;
  c->has_states = true;
  c->chi_M = c->tau_M = -1;
  return TK_OK;
}

int tk_set_pulses(tk_ctx *c, int32_t nt, double T, const double *u, const double *S,
                  const double *lambda) {
  if (!c) return TK_EINVAL;
  if (!c->has_system) return fail(c, TK_ESTATE, "no system set");
  if (nt < 1) return fail(c, TK_EINVAL, "nt must be >= 1");
  if (!(T > 0.0) || !std::isfinite(T)) return fail(c, TK_EINVAL, "T must be positive");
  const size_t n = static_cast<size_t>(c->n_ctrl) * nt;
  if (n > 0 && !u) return fail(c, TK_EINVAL, "u is NULL");
  TK_HIP(c, hipSetDevice(c->device));
  std::vector<double> uu(u, u + n), ss(n, 1.0), ll(c->n_ctrl, 1.0);
  if (S) ss.assign(S, S + n);
  if (lambda) ll.assign(lambda, lambda + c->n_ctrl);
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
  std::vector<double> up(static_cast<size_t>(tk::kMaxCtrl) * nt, 0.0), sp(up.size(), 0.0),
      lp(tk::kMaxCtrl, 1.0);
  std::copy(uu.begin(), uu.end(), up.begin());
  std::copy(ss.begin(), ss.end(), sp.begin());
  std::copy(ll.begin(), ll.end(), lp.begin());
  int rc = upload(c, c->u_dev, up.data(), up.size() * sizeof(double));
  if (rc) return rc;
  if ((rc = upload(c, c->S_dev, sp.data(), sp.size() * sizeof(double)))) return rc;
  if ((rc = upload(c, c->lam_dev, lp.data(), lp.size() * sizeof(double)))) return rc;
  c->has_pulses = true;
  c->chi_M = c->tau_M = -1;
  return TK_OK;
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
  if (!J_T || !dJdu) return fail(c, TK_EINVAL, "J_T or dJdu is NULL");
  int rc = prepare_pass(c, M, 0);
  if (rc) return rc;
  if ((rc = reset_counters(c))) return rc;
  if ((rc = run_grad(c, M, rec, n_rec))) return rc;
  if ((rc = check_kernel_errors(c))) return rc;
  if ((rc = functional_value(c, M, J_T))) return rc;
  const size_t ng = static_cast<size_t>(c->n_ctrl) * c->nt;
  if (ng > 0) TK_HIP(c, hipMemcpy(dJdu, c->dJdu.p, ng * sizeof(double), hipMemcpyDeviceToHost));
  if (tau_out)
    TK_HIP(c, hipMemcpy(tau_out, c->tau.p, 2 * static_cast<size_t>(M) * sizeof(double),
                        hipMemcpyDeviceToHost));
  c->tau_M = -1;  // the overlaps now belong to the replay, not to a forward pass
  return TK_OK;
}

int tk_krotov_iterate(tk_ctx *c, int32_t M, uint64_t seed, uint64_t first_iteration,
                      int32_t n_iter, double *J_T_out, tk_jump *rec, int64_t cap,
                      int64_t *n_rec) {
  if (!c) return TK_EINVAL;
  TK_HIP(c, hipSetDevice(c->device));
  if (!rec) cap = 0;
  if (n_iter < 0) return fail(c, TK_EINVAL, "n_iter must be >= 0");
  if (!J_T_out) return fail(c, TK_EINVAL, "J_T_out is NULL");
  const bool cont_ok = c->tau_M == M && c->tau_seed == seed &&
                       c->tau_iter == static_cast<int64_t>(first_iteration) - 1;
  int rc = prepare_pass(c, M, cap);
  if (rc) return rc;
  if ((rc = reset_counters(c))) return rc;
  int out = 0;
  uint64_t n = first_iteration;
  if (first_iteration == 0) {
    if ((rc = run_forward(c, M, seed, 0, cap))) return rc;
    if ((rc = check_kernel_errors(c))) return rc;
    if ((rc = functional_value(c, M, &J_T_out[out++]))) return rc;
    n = 1;
  } else if (!cont_ok) {
    return fail(c, TK_ESTATE, "no forward pass of the previous iteration with this M and seed");
  }
  const uint64_t last = (first_iteration == 0 ? 0 : first_iteration - 1) + n_iter;
  for (; n <= last; ++n) {
    if ((rc = run_backward(c, M, seed, n, cap))) return rc;
    if ((rc = check_kernel_errors(c))) return rc;
    if ((rc = run_krotov(c, M, seed, n, cap))) return rc;
    if ((rc = functional_value(c, M, &J_T_out[out++]))) return rc;
  }
  return fetch_records(c, rec, cap, n_rec);
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
