// Host-side internals shared by the library's host sources: the context, its
// device buffers and the helpers the drivers of every pass use.
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "tk_internal.h"

namespace tkh {

using cd = std::complex<double>;

// host sparse matrix (CSR, complex128)
struct Csr {
  int64_t n = 0;
  std::vector<int64_t> ptr;
  std::vector<int32_t> idx;
  std::vector<cd> val;
  int64_t nnz() const { return static_cast<int64_t>(idx.size()); }
  int max_row() const {
    int64_t w = 0;
    for (int64_t r = 0; r < n; ++r) w = std::max(w, ptr[r + 1] - ptr[r]);
    return static_cast<int>(w);
  }
};

// owning device allocation that only grows
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  hipError_t ensure(size_t n) {
    if (n <= bytes && p) return hipSuccess;
    release();
    if (n == 0) n = 8;
    hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) {
      p = nullptr;
      return e;
    }
    bytes = n;
    return hipSuccess;
  }
  template <typename T>
  T *as() const {
    return static_cast<T *>(p);
  }
};

}  // namespace tkh

struct tk_ctx {
  int device = 0;
  int precision = TK_FP64;
  hipStream_t stream = nullptr;
  std::string err;
  int n_cu = 0;

  bool has_system = false, has_states = false, has_pulses = false;
  int64_t d = 0;
  int n_ctrl = 0, n_jump = 0;
  const tk::Variant *var = nullptr;
  int wc = 1, wl = 1;
  double b0 = 0.0;
  double bc[tk::kMaxCtrl] = {};
  int64_t nnz_heff = 0;
  std::vector<tkh::Csr> H_ctrl_host;
  tkh::Csr A_host;  // H0 - (i/2) sum_l L_l^+ L_l
  std::vector<tkh::Csr> L_host;  // jump operators

  tkh::DevBuf f_scol, f_sval, f_ccol, f_cval, b_scol, b_sval, b_ccol, b_cval, lcol, lval;
  tkh::DevBuf f_sdiag, b_sdiag;  // diagonals of the static parts, [m][team lane]
  tkh::DevBuf ldcol, ldval;  // L_l^+ (pathwise gradient)
  int wld = 1;
  tkh::DevBuf psi0_bulk, tgt_bulk, tgt64;

  int nt = 0;
  double T = 0.0;
  std::vector<double> u, S, lam;
  tkh::DevBuf u_dev, u_new_dev, S_dev, lam_dev;

  tkh::DevBuf chi, tau, psiT, slots, rec, rec_count, err_dev, jt_dev;
  tkh::DevBuf kstates;  // Krotov-pass states when they do not fit in LDS
  // device basis order (empty: the basis itself): device row q is basis row perm[q]
  std::vector<int32_t> perm, inv_perm;
  tkh::DevBuf path_off, path_step, path_t, path_op, ckpt, stash, gk, dJdu;
  tkh::DevBuf noise_u, noise_nu;  // pulse-noise measure
  tkh::DevBuf pmat, ones_tau;      // cross-trajectory update: Gram matrices, unit weights
  tkh::DevBuf bench_x, bench_y, bench_h;  // step comparison (tk_step_bench)
  // density-matrix passes: CSR copies (complex128) of A, A^+, H_i, L_l, L_l^+,
  // work matrices, the stored P(t_j) and psi0 in FP64
  bool rho_ready = false;
  tkh::DevBuf rho_csr[3 * (2 + tk::kMaxCtrl + 2 * tk::kMaxJump)];
  tkh::DevBuf rho_work, rho_P, psi0_64;
  double rho_bj = 0.0;
  int chi_M = -1;
  int tau_M = -1;
  uint64_t tau_seed = 0;
  int64_t tau_iter = -1;

  bool timing = false;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipEvent_t ev_join = nullptr;  // orders the context's stream with a caller's stream
  tk_kernel_timing tstat[TK_KERNEL_COUNT] = {};
  int last_wpb = 0, last_tw = 0, last_blocks = 0;
  bool cooperative = true;  // launch the Krotov pass with hipLaunchCooperativeKernel

  size_t bulk_cplx() const { return precision == TK_FP64 ? 16 : 8; }
};

namespace tkh {

int fail(tk_ctx *c, int code, const std::string &msg);
int hip_fail(tk_ctx *c, hipError_t e, const char *what);
int upload(tk_ctx *c, DevBuf &buf, const void *src, size_t bytes);
// arguments of a pass of M trajectories with the context's operator (forward)
// or its adjoint (backward), current pulses and term-buffer plan
tk::PassArgs base_args(tk_ctx *c, int M, uint64_t seed, uint64_t iteration, bool backward);
// term vectors a pass with pulses u needs (largest order + 1 + margin)
int plan_kbuf(const tk_ctx *c, const std::vector<double> &u, int margin);
// algorithmic flops of one pass of M trajectories with pulses u
double pass_flops(const tk_ctx *c, const std::vector<double> &u, int M);

}  // namespace tkh

#define TK_HIP(ctx, call)                                    \
  do {                                                       \
    hipError_t e_ = (call);                                  \
    if (e_ != hipSuccess) return tkh::hip_fail(ctx, e_, #call); \
  } while (0)
