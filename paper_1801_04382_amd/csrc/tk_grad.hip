// Pathwise gradient of the trajectory functional with the jump record fixed.
//
// A forward pass leaves, per trajectory, the times and operators of its jumps.
// Holding them fixed makes every trajectory a fixed chain of linear maps --
// propagator pieces exp(-i H_eff(u_j) tau) between consecutive jump times and
// jump operators L_l (their renormalisation is a positive constant, which the
// normalised final state does not see) -- and J_T = 1 - (1/M) sum_k F_k with
// F_k = |<tgt|phi_k>|^2 / <phi_k|phi_k> a smooth function of the pulses.
//
// One wave per trajectory:
//   1. Replay forward from psi0, storing the state every kGradCheckpoint steps.
//      At the end, tau_k and the adjoint seed lambda = dF/d<phi| =
//      (tau tgt - |tau|^2 phi_hat) / ||phi||.
//   2. Reverse sweep, one checkpoint segment at a time (last first): recompute
//      the segment's step-start states from its checkpoint into a per-wave
//      stash, then walk its steps backward.  For every propagator unit of a
//      step (a piece between jumps, cut into substeps no longer than the
//      MCWF step plan's), the state at the unit's start is recomputed from the
//      step's stashed start, and an augmented Taylor series gives both
//      X = exp(-i H tau) x and Y_i = d X / d u_i (the top-right block of
//      exp(tau [[-iH, -iH_i], [0, -iH]]), Van Loan 1978).  Then
//        lambda <- c L_l^+ lambda   for the jump that ends the piece
//                                   (c = 1 / ||L_l X||, as in the forward map),
//        g_ij   += Re <lambda|Y_i>,
//        lambda <- exp(+i H^+ tau) lambda.
//   3. dJ_T/du_ij = -(2/M) sum_k g_kij, summed over k in a fixed order.
#include <hip/hip_runtime.h>

// plain (not global-view) accesses: this kernel spills, and measured faster so
#define TK_GENERIC_ACCESS
#include "tk_device.h"
#include "tk_internal.h"

namespace tk {
namespace {

// the lane's rows of a state to / from a 64 G R-element vector in global memory
template <typename real, int R, int G>
__device__ __forceinline__ void put_rows(cx<real> *v, const cx<real> (&p)[R], const Team<G> &tm) {
#pragma unroll
  for (int m = 0; m < R; ++m) v[tm.gl + Team<G>::kLanes * m] = p[m];
}

template <typename real, int R, int G>
__device__ __forceinline__ void get_rows(const cx<real> *v, cx<real> (&p)[R], const Team<G> &tm) {
#pragma unroll
  for (int m = 0; m < R; ++m) p[m] = v[tm.gl + Team<G>::kLanes * m];
}

template <typename real, int R>
__device__ __forceinline__ void copy_state(const cx<real> (&in)[R], cx<real> (&out)[R]) {
#pragma unroll
  for (int m = 0; m < R; ++m) out[m] = in[m];
}

// psi <- exp(-i H_eff tau) psi in n = ceil(tau / h) equal substeps of order K
template <typename real, int R, int WS, int NC, int G>
__device__ void propagate_piece(const LaneOp<real, R, WS, NC, G> &op, const PassArgs &a,
                                const Terms<real, R, G> &T, cx<real> (&psi)[R], double tau,
                                const StepPlan &p, const Team<G> &tm) {
  if (!(tau > 0.0)) return;
  const int n = max(1, static_cast<int>(ceil(tau / p.h)));
  const double hs = tau / n;
  for (int s = 0; s < n; ++s) {
    cx<real> out[R];
    tm.sync();
    taylor_pingpong<real, R, WS, NC, G, -1, false>(op, a, T, psi, out, hs, p.K, tm);
    copy_state(out, psi);
  }
}

// psi <- L_l psi / ||L_l psi|| (the forward jump map); returns ||L_l psi||^2
template <typename real, int R, int G>
__device__ double jump_map(const PassArgs &a, const Terms<real, R, G> &T, int l, cx<real> (&psi)[R],
                           const Team<G> &tm) {
  tm.sync();
  store_lds(T[0], psi, tm);
  tm.sync();
  cx<real> y[R];
  apply_jump<real, R, G>(a, l, T[0], y, tm);
  const double w = norm2(y, tm);
  if (!(w > 0.0)) {
    if (tm.leader()) atomicOr(a.err, kErrNoJumpWeight);
    copy_state(y, psi);
    return w;
  }
  const real inv = static_cast<real>(1.0 / sqrt(w));
#pragma unroll
  for (int m = 0; m < R; ++m) psi[m] = cx<real>{y[m].x * inv, y[m].y * inv};
  return w;
}

// Jump times of a piece: piece q of step j (q < n_jumps) ends at the jump
// path_t[qs + q]; the last piece ends at t_{j+1}.
__device__ __forceinline__ double piece_end(const PassArgs &a, int j, int qs, int q, int nj) {
  return q < nj ? a.path_t[qs + q] : static_cast<double>(j + 1) * a.dt;
}

__device__ __forceinline__ double piece_start(const PassArgs &a, int j, int qs, int q) {
  return q > 0 ? a.path_t[qs + q - 1] : static_cast<double>(j) * a.dt;
}

// Replay of step j: pieces between the recorded jumps [qs, qs + nj).
template <typename real, int R, int WS, int NC, int G>
__device__ void replay_step(const LaneOp<real, R, WS, NC, G> &op, const PassArgs &a,
                            const Terms<real, R, G> &T, cx<real> (&psi)[R], int j, int qs, int nj,
                            const StepPlan &p, const Team<G> &tm) {
  for (int q = 0; q <= nj; ++q) {
    const double tau = fmax(piece_end(a, j, qs, q, nj) - piece_start(a, j, qs, q), 0.0);
    propagate_piece<real, R, WS, NC, G>(op, a, T, psi, tau, p, tm);
    if (q < nj) jump_map<real, R, G>(a, T, a.path_op[qs + q], psi, tm);
  }
}

// Augmented Taylor series over tau (forward direction):
//   x_n = (tau/n)(-i) H x_{n-1},  y_{i,n} = (tau/n)(-i)(H y_{i,n-1} + H_i x_{n-1}),
// X = sum x_n, Y_i = sum y_{i,n} for the controls i < n_ctrl.  Term vectors are
// double-buffered in LDS: buffer b holds x in T[b (1 + NCX)] and y_i in
// T[b (1 + NCX) + 1 + i].
template <typename real, int R, int WS, int NC, int G>
__device__ void taylor_aug(const LaneOp<real, R, WS, NC, G> &op, const PassArgs &a,
                           const Terms<real, R, G> &T, const cx<real> (&x0)[R], cx<real> (&X)[R],
                           cx<real> (&Y)[NC > 0 ? NC : 1][R], double tau, int K, const Team<G> &tm) {
  constexpr int NCX = NC > 0 ? NC : 1;
  const int nctl = a.n_ctrl;
  cx<real> incX[R];
#pragma unroll
  for (int m = 0; m < R; ++m) incX[m] = cx<real>{0, 0};
#pragma unroll
  for (int i = 0; i < NCX; ++i)
#pragma unroll
    for (int m = 0; m < R; ++m) Y[i][m] = cx<real>{0, 0};
  tm.sync();
  store_lds(T[0], x0, tm);
#pragma unroll
  for (int i = 0; i < NCX; ++i)
    if (i < nctl) store_lds(T[1 + i], Y[i], tm);
  int cur = 0;
  for (int n = 1; n <= K; ++n) {
    tm.sync();
    constexpr int kLen = Terms<real, R, G>::kLen;
    const int xshift = cur * (1 + NCX) * kLen;  // x_{n-1}: term vector cur (1 + NCX)
    // gathers of x_{n-1}: H x and the unscaled H_i x from the same loads.
    // Eight-wave teams (short of registers) gather the static slots, multiply
    // them, then gather the control slots; the others issue all gathers first.
    constexpr bool kHalves = G >= 4;
    cx<real> b[WS + NCX][R];
#pragma unroll
    for (int s = 0; s < WS; ++s)
#pragma unroll
      for (int m = 0; m < R; ++m) b[s][m] = op.sp[s][m][xshift];
    if constexpr (!kHalves) {
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int m = 0; m < R; ++m) b[WS + c][m] = op.cp[c][m][xshift];
    }
    __builtin_amdgcn_sched_barrier(0);
    cx<real> hx[R], hix[NCX][R];
#pragma unroll
    for (int m = 0; m < R; ++m) hx[m] = cx<real>{0, 0};
#pragma unroll
    for (int i = 0; i < NCX; ++i)
#pragma unroll
      for (int m = 0; m < R; ++m) hix[i][m] = cx<real>{0, 0};
#pragma unroll
    for (int s = 0; s < WS; ++s)
#pragma unroll
      for (int m = 0; m < R; ++m) cfma(hx[m], op.sval[s][m], b[s][m]);
    if constexpr (kHalves) {
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int m = 0; m < R; ++m) b[WS + c][m] = op.cp[c][m][xshift];
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      int i = 0;  // control of slot c: c / wc, by comparisons
#pragma unroll
      for (int ii = 1; ii < NC; ++ii)
        if (c >= ii * a.wc) i = ii;
#pragma unroll
      for (int m = 0; m < R; ++m) {
        cfma(hx[m], op.cv[c][m], b[WS + c][m]);
        const cx<real> q = op.cval_at(c, m);
#pragma unroll
        for (int ii = 0; ii < NCX; ++ii)
          if (ii == i) cfma(hix[ii][m], q, b[WS + c][m]);
      }
    }
    const real cf = static_cast<real>(tau * a.inv_n[n]);
    const int nxt = cur ^ 1;
    cx<real> t[R];
#pragma unroll
    for (int m = 0; m < R; ++m) {
      t[m] = cx<real>{cf * hx[m].y, -cf * hx[m].x};  // (tau/n)(-i) H x
      incX[m].x += t[m].x;
      incX[m].y += t[m].y;
    }
    // y_i terms (the gathers of y_{i,n-1} read the current buffer)
    cx<real> ty[NCX][R];
#pragma unroll
    for (int i = 0; i < NCX; ++i) {
      if (i < nctl) {
        cx<real> hy[R];
        op.apply_at((cur * (1 + NCX) + 1 + i) * kLen, hy);
#pragma unroll
        for (int m = 0; m < R; ++m) {
          const real sx = hy[m].x + hix[i][m].x, sy = hy[m].y + hix[i][m].y;
          ty[i][m] = cx<real>{cf * sy, -cf * sx};
          Y[i][m].x += ty[i][m].x;
          Y[i][m].y += ty[i][m].y;
        }
      }
    }
    store_lds(T[nxt * (1 + NCX)], t, tm);
#pragma unroll
    for (int i = 0; i < NCX; ++i)
      if (i < nctl) store_lds(T[nxt * (1 + NCX) + 1 + i], ty[i], tm);
    cur = nxt;
  }
#pragma unroll
  for (int m = 0; m < R; ++m) X[m] = cx<real>{x0[m].x + incX[m].x, x0[m].y + incX[m].y};
}

template <typename real, int R, int WS, int NC, int G>
__global__ __launch_bounds__(kWave *(G > kWavesPerBlock ? G : kWavesPerBlock)) void k_grad(
    PassArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double team_red[4 * G];
  constexpr int NCX = NC > 0 ? NC : 1;
  constexpr int kL = Team<G>::kLanes;
  constexpr int kLen = Terms<real, R, G>::kLen;
  const int team = __builtin_amdgcn_readfirstlane(threadIdx.x / kL);
  const int tpb = blockDim.x / kL;
  const Team<G> tm = make_team<G>(team_red);
  const int nbuf = max(a.kbuf, 2 * (1 + NCX));
  // LDS: per team nbuf term vectors; the unscaled control values of both
  // operators are read from global memory (they are small and cached)
  Terms<real, R, G> T;
  T.base = reinterpret_cast<cx<real> *>(smem_raw) + static_cast<size_t>(team) * nbuf * kLen;
  if (tm.gl < nbuf) T[tm.gl][R * kL] = cx<real>{0, 0};
  __syncthreads();
  // the forward operator stays in registers; the costate operator is loaded
  // where it is used (one series per substep of the reverse sweep), so the two
  // slices never hold registers at once
  LaneOp<real, R, WS, NC, G> opf;
  opf.load(a.scol, a.sval, a.ccol, static_cast<const cx<real> *>(a.cval), tm.gl);
  opf.bind(T[0]);

  const int nseg = (a.nt + kGradCheckpoint - 1) / kGradCheckpoint;
  const int wave = blockIdx.x * tpb + team;  // global team index
  const int nwaves = gridDim.x * tpb;
  const cx<real> *start = static_cast<const cx<real> *>(a.psi_start);
  cx<real> *stash = static_cast<cx<real> *>(a.stash) +
                    static_cast<size_t>(wave) * kGradCheckpoint * R * kL;

  for (int k = wave; k < a.M; k += nwaves) {
    cx<real> *ck = static_cast<cx<real> *>(a.ckpt) + static_cast<size_t>(k) * nseg * R * kL;
    const int q_first = a.path_off[k], q_last = a.path_off[k + 1];
    OrderHint khint;  // the previous step's order
    // ---- 1. forward replay with checkpoints ----
    cx<real> psi[R];
    get_rows(start, psi, tm);
    int q = q_first;
    for (int j = 0; j < a.nt; ++j) {
      if (j % kGradCheckpoint == 0) put_rows(ck + (j / kGradCheckpoint) * R * kL, psi, tm);
      int nj = 0;
      while (q + nj < q_last && a.path_step[q + nj] == j) ++nj;
      double uj[NCX];
#pragma unroll
      for (int i = 0; i < NCX; ++i) uj[i] = a.u[static_cast<size_t>(i) * a.nt + j];
      opf.set_pulses(uj, a.wc);
      const StepPlan p = plan_step(a, uj, khint);
      replay_step<real, R, WS, NC, G>(opf, a, T, psi, j, q, nj, p, tm);
      q += nj;
    }
    // ---- functional and adjoint seed ----
    const double nrm2 = norm2(psi, tm);
    const double inv = 1.0 / sqrt(nrm2);
    double tr = 0.0, ti = 0.0;
#pragma unroll
    for (int m = 0; m < R; ++m) {
      const int row = tm.gl + kL * m;
      const double px = psi[m].x * inv, py = psi[m].y * inv;
      const double gx = a.tgt[2 * row], gy = a.tgt[2 * row + 1];
      tr = fma(gx, px, fma(gy, py, tr));
      ti = fma(gx, py, fma(-gy, px, ti));
    }
    tr = tm.sum(tr);
    ti = tm.sum(ti);
    if (tm.leader()) {
      a.tau_out[2 * k] = tr;
      a.tau_out[2 * k + 1] = ti;
    }
    const double f = tr * tr + ti * ti;
    cx<real> lam[R];
#pragma unroll
    for (int m = 0; m < R; ++m) {
      const int row = tm.gl + kL * m;
      const double gx = a.tgt[2 * row], gy = a.tgt[2 * row + 1];
      const double px = psi[m].x * inv, py = psi[m].y * inv;
      lam[m] = cx<real>{static_cast<real>((tr * gx - ti * gy - f * px) * inv),
                        static_cast<real>((tr * gy + ti * gx - f * py) * inv)};
    }
    // ---- 2. reverse sweep over checkpoint segments ----
    int qe = q_last;  // end of the jumps of the step being processed
    for (int sg = nseg - 1; sg >= 0; --sg) {
      const int j0 = sg * kGradCheckpoint;
      const int j1 = min(a.nt, j0 + kGradCheckpoint);
      // recompute the segment's step-start states
      get_rows(ck + sg * R * kL, psi, tm);
      int qr = q_first;
      while (qr < q_last && a.path_step[qr] < j0) ++qr;
      for (int j = j0; j < j1; ++j) {
        put_rows(stash + (j - j0) * R * kL, psi, tm);
        if (j + 1 == j1) break;  // the last step's end state is not needed
        int nj = 0;
        while (qr + nj < q_last && a.path_step[qr + nj] == j) ++nj;
        double uj[NCX];
#pragma unroll
        for (int i = 0; i < NCX; ++i) uj[i] = a.u[static_cast<size_t>(i) * a.nt + j];
        opf.set_pulses(uj, a.wc);
        const StepPlan p = plan_step(a, uj, khint);
        replay_step<real, R, WS, NC, G>(opf, a, T, psi, j, qr, nj, p, tm);
        qr += nj;
      }
      for (int j = j1 - 1; j >= j0; --j) {
        int qs = qe;
        while (qs > q_first && a.path_step[qs - 1] == j) --qs;
        const int nj = qe - qs;
        double uj[NCX];
#pragma unroll
        for (int i = 0; i < NCX; ++i) uj[i] = a.u[static_cast<size_t>(i) * a.nt + j];
        opf.set_pulses(uj, a.wc);
        const StepPlan p = plan_step(a, uj, khint);
        double bnd = a.b0;
#pragma unroll
        for (int i = 0; i < NCX; ++i) bnd += fabs(uj[i]) * a.bc[i];
        int Kaug = taylor_order(a, (bnd + a.bc_max) * p.h, p.K);
        if (Kaug < 0) {
          if (tm.leader()) atomicOr(a.err, kErrTaylorOrder);
          Kaug = a.kmax;
        }
        double gl[NCX];  // lane partials of Re <lambda|Y_i> over the step's units
#pragma unroll
        for (int i = 0; i < NCX; ++i) gl[i] = 0.0;
        for (int pc = nj; pc >= 0; --pc) {
          const double tau = fmax(piece_end(a, j, qs, pc, nj) - piece_start(a, j, qs, pc), 0.0);
          // state at the start of piece pc
          cx<real> ps[R];
          get_rows(stash + (j - j0) * R * kL, ps, tm);
          for (int qq = 0; qq < pc; ++qq) {
            const double tq = fmax(piece_end(a, j, qs, qq, nj) - piece_start(a, j, qs, qq), 0.0);
            propagate_piece<real, R, WS, NC, G>(opf, a, T, ps, tq, p, tm);
            jump_map<real, R, G>(a, T, a.path_op[qs + qq], ps, tm);
          }
          if (!(tau > 0.0)) {
            // zero-length piece: only the jump that ends it (if any) acts
            if (pc < nj) {
              cx<real> y[R];
              tm.sync();
              store_lds(T[0], ps, tm);
              tm.sync();
              apply_jump<real, R, G>(a, a.path_op[qs + pc], T[0], y, tm);
              const double c = 1.0 / sqrt(norm2(y, tm));
              tm.sync();
              store_lds(T[0], lam, tm);
              tm.sync();
              apply_packed<real, R, G>(a.ldcol, a.ldval, a.wld, a.path_op[qs + pc], T[0], y, tm);
#pragma unroll
              for (int m = 0; m < R; ++m)
                lam[m] = cx<real>{static_cast<real>(c * y[m].x), static_cast<real>(c * y[m].y)};
            }
            continue;
          }
          const int n = max(1, static_cast<int>(ceil(tau / p.h)));
          const double hs = tau / n;
          for (int s = n - 1; s >= 0; --s) {
            // state at the start of substep s of this piece
            cx<real> xs[R];
            copy_state(ps, xs);
            for (int ss = 0; ss < s; ++ss) {
              cx<real> out[R];
              tm.sync();
              taylor_pingpong<real, R, WS, NC, G, -1, false>(opf, a, T, xs, out, hs, p.K, tm);
              copy_state(out, xs);
            }
            cx<real> X[R], Y[NCX][R];
            taylor_aug<real, R, WS, NC, G>(opf, a, T, xs, X, Y, hs, Kaug, tm);
            if (s == n - 1 && pc < nj) {
              // adjoint of the jump map that ends the piece: lambda <- c L^+ lambda
              cx<real> y[R];
              tm.sync();
              store_lds(T[0], X, tm);
              tm.sync();
              apply_jump<real, R, G>(a, a.path_op[qs + pc], T[0], y, tm);
              const double c = 1.0 / sqrt(norm2(y, tm));
              tm.sync();
              store_lds(T[0], lam, tm);
              tm.sync();
              apply_packed<real, R, G>(a.ldcol, a.ldval, a.wld, a.path_op[qs + pc], T[0], y, tm);
#pragma unroll
              for (int m = 0; m < R; ++m)
                lam[m] = cx<real>{static_cast<real>(c * y[m].x), static_cast<real>(c * y[m].y)};
            }
#pragma unroll
            for (int i = 0; i < NCX; ++i)
#pragma unroll
              for (int m = 0; m < R; ++m) {
                gl[i] = fma(static_cast<double>(lam[m].x), static_cast<double>(Y[i][m].x), gl[i]);
                gl[i] = fma(static_cast<double>(lam[m].y), static_cast<double>(Y[i][m].y), gl[i]);
              }
            // lambda <- exp(+i H^+ hs) lambda
            cx<real> out[R];
            {
              LaneOp<real, R, WS, NC, G> opb;
              opb.load(a.a_scol, a.a_sval, a.a_ccol, static_cast<const cx<real> *>(a.a_cval), tm.gl);
              opb.bind(T[0]);
              opb.set_pulses(uj, a.wc);
              tm.sync();
              taylor_pingpong<real, R, WS, NC, G, 1, false>(opb, a, T, lam, out, hs, p.K, tm);
            }
            copy_state(out, lam);
          }
        }
#pragma unroll
        for (int i = 0; i < NCX; ++i) {
          if (i < a.n_ctrl) {
            const double g = tm.sum(gl[i]);
            if (tm.leader()) a.gk[(static_cast<size_t>(i) * a.nt + j) * a.M + k] = g;
          }
        }
        qe = qs;
      }
    }
  }
}

// dJ_T/du_ij = -(2/M) sum_k g_kij, one wave per pulse value, fixed order
__global__ __launch_bounds__(kWave) void k_grad_reduce(const double *gk, int M, double *out) {
  const int row = blockIdx.x;
  const int lane = threadIdx.x;
  double s = 0.0;
  for (int k = lane; k < M; k += kWave) s += gk[static_cast<size_t>(row) * M + k];
  s = wave_sum(s);
  if (lane == 0) out[row] = -2.0 * s / static_cast<double>(M);
}

}  // namespace

const void *grad_kernel(int precision, int R, int WS, int NC, int G) {
#define TK_GRAD_CASE(real, r, ws, nc, g)                                                   \
  if (precision == (sizeof(real) == 8 ? TK_FP64 : TK_FP32) && R == r && WS == ws && NC == nc && \
      G == g)                                                                               \
    return reinterpret_cast<const void *>(&k_grad<real, r, ws, nc, g>);
  TK_GRAD_CASE(double, 1, 4, 2, 1)
  TK_GRAD_CASE(double, 2, 4, 2, 1)
  TK_GRAD_CASE(double, 4, 6, 3, 1)
  TK_GRAD_CASE(double, 4, 8, 4, 1)
  TK_GRAD_CASE(double, 1, 4, 2, 2)
  TK_GRAD_CASE(double, 2, 6, 3, 2)
  TK_GRAD_CASE(float, 1, 4, 2, 1)
  TK_GRAD_CASE(float, 2, 4, 2, 1)
  TK_GRAD_CASE(float, 4, 6, 3, 1)
  TK_GRAD_CASE(float, 4, 8, 4, 1)
  TK_GRAD_CASE(float, 1, 4, 2, 2)
  TK_GRAD_CASE(float, 2, 6, 3, 2)
  TK_GRAD_CASE(float, 3, 9, 4, 8)
#undef TK_GRAD_CASE
  return nullptr;
}

const void *grad_reduce_kernel() { return reinterpret_cast<const void *>(&k_grad_reduce); }

size_t grad_lds_bytes(const Variant &v, int teams, int kbuf) {
  const size_t cplx = v.precision == TK_FP64 ? 16 : 8;
  const size_t ncx = v.NC > 0 ? v.NC : 1;
  const size_t nbuf = std::max<size_t>(kbuf, 2 * (1 + ncx));
  return static_cast<size_t>(teams) * nbuf * (static_cast<size_t>(v.R) * kWave * v.G + 1) * cplx;
}

}  // namespace tk
