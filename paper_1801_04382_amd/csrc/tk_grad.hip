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
//      MCWF step plan's), the state x at the unit's start is recomputed from
//      the step's stashed start and the unit's series is run keeping its
//      terms s_k = (-i h H)^k x / k!.  Then
//        lambda <- c L_l^+ lambda   for the jump that ends the piece
//                                   (c = 1 / ||L_l X||, as in the forward map),
//      and the costate series t_m = (i h H^+)^m lambda / m! both advances
//      lambda <- exp(+i H^+ h) lambda and gives the unit's derivative: the
//      top-right block of exp(h [[-iH, -iH_i], [0, -iH]]) (Van Loan 1978),
//      expanded in powers of h, pairs the two series as
//        Re <lambda|dX/du_i> = h Im sum_{m+k<K} m! k! / (m+k+1)! <t_m|H_i|s_k>,
//      added to g_ij.  The forward and costate operators are loaded for the
//      phase that uses them, so only one of them holds registers at a time.
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
    taylor_pingpong<real, R, WS, NC, G, -1>(op, a, T, psi, out, hs, p.K, tm);
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

// Control of slot c (c / wc), by comparisons
template <int NC>
__device__ __forceinline__ int slot_ctrl(int c, int wc) {
  int i = 0;
#pragma unroll
  for (int ii = 1; ii < NC; ++ii)
    if (c >= ii * wc) i = ii;
  return i;
}

// v = sum_{k=0}^{Kg-1-m} beta_{m,k} s_k over the lane's rows, for the kept
// forward terms s_k at fown + k kLen; beta_{m,k} = m! k! / (m + k + 1)!, from
// beta_{m,0} = 1 / (m + 1) and beta_{m,k+1} = beta_{m,k} (k + 1) / (m + k + 2).
template <typename real, int R, int G>
__device__ __forceinline__ void pair_weights(const PassArgs &a, const cx<real> *fown, int m,
                                             int Kg, cx<real> (&v)[R]) {
  constexpr int kLen = Terms<real, R, G>::kLen;
  constexpr int kL = Team<G>::kLanes;
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] = cx<real>{0, 0};
  double beta = a.inv_n[m + 1];
#pragma unroll 2
  for (int k = 0; k + m < Kg; ++k) {
    const real bk = static_cast<real>(beta);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const cx<real> s = fown[k * kLen + kL * r];
      v[r] = cx<real>{fma(bk, s.x, v[r].x), fma(bk, s.y, v[r].y)};
    }
    beta *= static_cast<double>(k + 1) * a.inv_n[m + k + 2];
  }
}

// One term of the costate series together with the gradient pairs of its
// input: gathers t_m (the term vector at the bound addresses plus OFF),
// leaves t_{m+1} = (i h / (m + 1)) H^+ t_m in t (added to inc), and adds
// Im <H_i^+ t_m | v> over the lane's rows to gp[i].  op.cv holds the unscaled
// control elements (of H_i^+); us[c] is the pulse value of slot c.
template <typename real, int R, int WS, int NC, int G, int OFF>
__device__ __forceinline__ void costate_term(const LaneOp<real, R, WS, NC, G> &op,
                                             const real (&us)[NC > 0 ? NC : 1], int wc, real cf,
                                             const cx<real> (&v)[R], cx<real> (&t)[R],
                                             cx<real> (&inc)[R], real (&gp)[NC > 0 ? NC : 1]) {
  constexpr int NCX = NC > 0 ? NC : 1;
  constexpr int W0 = LaneOp<real, R, WS, NC, G>::W0;
  constexpr int H = (W0 + 1) / 2;
  cx<real> y[R];
#pragma unroll
  for (int m = 0; m < R; ++m) {  // the diagonal first, from t_m in registers
    y[m] = cx<real>{0, 0};
    cfma(y[m], op.dval[m], t[m]);
  }
  gather_fma<real, R, WS, NC, G, OFF, 0, H>(op, 0, y);
  if constexpr (H < W0) gather_fma<real, R, WS, NC, G, OFF, H, W0>(op, 0, y);
  if constexpr (NC > 0) {
    cx<real> b[NC][R];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int m = 0; m < R; ++m) b[c][m] = op.cp[c][m][OFF];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int i = slot_ctrl<NC>(c, wc);
#pragma unroll
      for (int m = 0; m < R; ++m) {
        const cx<real> q = op.cv[c][m];
        // (real control elements: q.y is zero)
        const cx<real> pr = LaneOp<real, R, WS, NC, G>::RC
                                ? cx<real>{q.x * b[c][m].x, q.x * b[c][m].y}
                                : cx<real>{q.x * b[c][m].x - q.y * b[c][m].y,
                                           q.x * b[c][m].y + q.y * b[c][m].x};
        y[m] = cx<real>{fma(us[c], pr.x, y[m].x), fma(us[c], pr.y, y[m].y)};
        const real im = pr.x * v[m].y - pr.y * v[m].x;  // Im(conj(pr) v)
#pragma unroll
        for (int ii = 0; ii < NCX; ++ii)
          if (ii == i) gp[ii] += im;
      }
    }
  }
#pragma unroll
  for (int m = 0; m < R; ++m) {
    t[m] = cx<real>{-cf * y[m].y, cf * y[m].x};
    inc[m].x += t[m].x;
    inc[m].y += t[m].y;
  }
}

// Costate series over one propagator unit of length h with the gradient of
// the unit.  With the forward terms s_k = (-i h H)^k x / k! of the unit kept
// in Tf[0 .. Kg] and the costate terms t_m = (i h H^+)^m lambda / m!, the
// derivative of the unit's propagator along H_i (the top-right block of Van
// Loan's block exponential, truncated at order Kg) satisfies
//   <lambda| dX/du_i = -i h sum_{m+k<=Kg-1} beta_{m,k} <t_m| H_i |s_k>,
// so Re <lambda|dX/du_i> = h Im(...), added to gl[i].  The costate advances
// as lambda <- sum_{m<=Kg} t_m = exp(+i H^+ h) lambda; its terms alternate
// between Tc[0] and Tc[1], where the gathers of op are bound.
template <typename real, int R, int WS, int NC, int G>
__device__ void costate_grad(const LaneOp<real, R, WS, NC, G> &op, const PassArgs &a,
                             const Terms<real, R, G> &Tc, const Terms<real, R, G> &Tf,
                             const real (&us)[NC > 0 ? NC : 1], cx<real> (&lam)[R], double h,
                             int Kg, double (&gl)[NC > 0 ? NC : 1], const Team<G> &tm) {
  constexpr int NCX = NC > 0 ? NC : 1;
  constexpr int kLen = Terms<real, R, G>::kLen;
  constexpr int kL = Team<G>::kLanes;
  cx<real> *own = Tc.base + tm.gl;
  const cx<real> *fown = Tf.base + tm.gl;
  cx<real> t[R], inc[R];
  real gp[NCX];
#pragma unroll
  for (int i = 0; i < NCX; ++i) gp[i] = 0;
  tm.sync();  // every gather of the previous use of Tc[0] is done
#pragma unroll
  for (int m = 0; m < R; ++m) {
    t[m] = lam[m];
    inc[m] = cx<real>{0, 0};
    own[kL * m] = t[m];
  }
  for (int n = 0; n < Kg; n += 2) {  // t_{n+1}, t_{n+2} from t_n (Tc[0]), t_{n+1} (Tc[1])
    cx<real> v[R];
    pair_weights<real, R, G>(a, fown, n, Kg, v);
    tm.sync();
    costate_term<real, R, WS, NC, G, 0>(op, us, a.wc, static_cast<real>(h * a.inv_n[n + 1]), v,
                                        t, inc, gp);
#pragma unroll
    for (int m = 0; m < R; ++m) own[kLen + kL * m] = t[m];
    if (n + 2 > Kg) break;
    pair_weights<real, R, G>(a, fown, n + 1, Kg, v);
    tm.sync();
    costate_term<real, R, WS, NC, G, kLen>(op, us, a.wc, static_cast<real>(h * a.inv_n[n + 2]),
                                           v, t, inc, gp);
#pragma unroll
    for (int m = 0; m < R; ++m) own[kL * m] = t[m];
  }
#pragma unroll
  for (int m = 0; m < R; ++m) lam[m] = cx<real>{lam[m].x + inc[m].x, lam[m].y + inc[m].y};
#pragma unroll
  for (int i = 0; i < NCX; ++i) gl[i] = fma(h, static_cast<double>(gp[i]), gl[i]);
}

// The forward operator (H_eff at the pulses uj) or the costate operator
// (H_eff^+, unit pulses: the costate series applies them itself), with its
// gathers bound to t0
template <typename real, int R, int WS, int NC, int G>
__device__ __forceinline__ void load_forward(LaneOp<real, R, WS, NC, G> &op, const PassArgs &a,
                                             const cx<real> *t0,
                                             const double (&uj)[NC > 0 ? NC : 1], int gl) {
  op.load(opaque(a.scol), opaque(static_cast<const cx<real> *>(a.sval)),
          opaque(static_cast<const cx<real> *>(a.sdiag)), opaque(a.ccol),
          opaque(static_cast<const cx<real> *>(a.cval)), gl);
  op.bind(t0);
  op.set_pulses(uj, a.wc);
}

template <typename real, int R, int WS, int NC, int G>
__device__ __forceinline__ void load_costate(LaneOp<real, R, WS, NC, G> &op, const PassArgs &a,
                                             const cx<real> *t0, int gl) {
  constexpr int NCX = NC > 0 ? NC : 1;
  double ones[NCX];
#pragma unroll
  for (int i = 0; i < NCX; ++i) ones[i] = 1.0;
  op.load(opaque(a.a_scol), opaque(static_cast<const cx<real> *>(a.a_sval)),
          opaque(static_cast<const cx<real> *>(a.a_sdiag)), opaque(a.a_ccol),
          opaque(static_cast<const cx<real> *>(a.a_cval)), gl);
  op.bind(t0);
  op.set_pulses(ones, a.wc);
}

// lambda <- c L_l^+ lambda with c = 1 / ||L_l x|| (the adjoint of the forward
// jump map at x); Tc[0] is scratch
template <typename real, int R, int G>
__device__ void jump_adjoint(const PassArgs &a, const Terms<real, R, G> &Tc, int l,
                             const cx<real> (&x)[R], cx<real> (&lam)[R], const Team<G> &tm) {
  cx<real> y[R];
  tm.sync();
  store_lds(Tc[0], x, tm);
  tm.sync();
  apply_jump<real, R, G>(a, l, Tc[0], y, tm);
  const double c = 1.0 / sqrt(norm2(y, tm));  // the team sum orders the gathers above
  store_lds(Tc[0], lam, tm);
  tm.sync();
  apply_packed<real, R, G>(a.ldcol, a.ldval, a.wld, l, Tc[0], y, tm);
#pragma unroll
  for (int m = 0; m < R; ++m)
    lam[m] = cx<real>{static_cast<real>(c * y[m].x), static_cast<real>(c * y[m].y)};
}

template <typename real, int R, int WS, int NC, int G>
__global__ __launch_bounds__(kWave *(G > kWavesPerBlock ? G : kWavesPerBlock)) void k_grad(
    PassArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double team_red[8 * G];
  constexpr int NCX = NC > 0 ? NC : 1;
  constexpr int kL = Team<G>::kLanes;
  constexpr int kLen = Terms<real, R, G>::kLen;
  const int team = __builtin_amdgcn_readfirstlane(threadIdx.x / kL);
  const int tpb = blockDim.x / kL;
  const Team<G> tm = make_team<G>(team_red);
  const int nbuf = a.kbuf;
  // LDS per team: nbuf term vectors.  The replay passes use vectors 0 and 1
  // (T); the reverse sweep keeps a unit's forward terms in vectors 2 ..
  // nbuf - 1 (Tf) and runs the costate series in vectors 0 and 1 (Tc).
  Terms<real, R, G> T;
  T.base = reinterpret_cast<cx<real> *>(smem_raw) + static_cast<size_t>(team) * nbuf * kLen;
  Terms<real, R, G> Tf;
  Tf.base = T.base + 2 * kLen;
  const Terms<real, R, G> &Tc = T;
  const int kg_max = nbuf - 3;  // largest order whose kept terms fit Tf
  if (tm.gl < nbuf) T[tm.gl][R * kL] = cx<real>{0, 0};
  __syncthreads();
  // Each phase loads the operator it uses (from global memory, where every
  // team reads the same slices) and drops it afterwards, so the forward and
  // costate operators never hold registers at the same time.

  double zeros[NCX];
#pragma unroll
  for (int i = 0; i < NCX; ++i) zeros[i] = 0.0;
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
    {
      LaneOp<real, R, WS, NC, G> opf;
      load_forward(opf, a, T[0], zeros, tm.gl);  // pulses set per step
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
      {
        LaneOp<real, R, WS, NC, G> opf;
        load_forward(opf, a, T[0], zeros, tm.gl);  // pulses set per step
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
      }
      for (int j = j1 - 1; j >= j0; --j) {
        int qs = qe;
        while (qs > q_first && a.path_step[qs - 1] == j) --qs;
        const int nj = qe - qs;
        double uj[NCX];
#pragma unroll
        for (int i = 0; i < NCX; ++i) uj[i] = a.u[static_cast<size_t>(i) * a.nt + j];
        const StepPlan p = plan_step(a, uj, khint);
        // order of the unit derivatives: the bound ||H_eff|| + max_i ||H_i||
        // of Van Loan's block generator
        double bnd = a.b0;
#pragma unroll
        for (int i = 0; i < NCX; ++i) bnd += fabs(uj[i]) * a.bc[i];
        int Kg = taylor_order(a, (bnd + a.bc_max) * p.h, p.K);
        if (Kg < 0 || Kg > kg_max) {
          if (tm.leader()) atomicOr(a.err, kErrTaylorOrder);
          Kg = kg_max;
        }
        real us[NCX];  // pulse value of each control slot
#pragma unroll
        for (int c = 0; c < NCX; ++c) {
          double u = uj[0];
#pragma unroll
          for (int i = 1; i < NCX; ++i)
            if (c >= i * a.wc) u = uj[i];
          us[c] = static_cast<real>(u);
        }
        double gl[NCX];  // lane partials of Re <lambda|dX/du_i> over the step's units
#pragma unroll
        for (int i = 0; i < NCX; ++i) gl[i] = 0.0;
        for (int pc = nj; pc >= 0; --pc) {
          const double tau = fmax(piece_end(a, j, qs, pc, nj) - piece_start(a, j, qs, pc), 0.0);
          const int n = tau > 0.0 ? max(1, static_cast<int>(ceil(tau / p.h))) : 1;
          const double hs = tau > 0.0 ? tau / n : 0.0;
          for (int s = n - 1; s >= 0; --s) {
            cx<real> X[R];  // the unit's end state
            {
              // forward: the state at the start of substep s of piece pc,
              // then the unit's series keeping its terms in Tf
              LaneOp<real, R, WS, NC, G> opf;
              load_forward(opf, a, Tf[0], uj, tm.gl);
              cx<real> xs[R];
              get_rows(stash + (j - j0) * R * kL, xs, tm);
              for (int qq = 0; qq < pc; ++qq) {
                const double tq =
                    fmax(piece_end(a, j, qs, qq, nj) - piece_start(a, j, qs, qq), 0.0);
                propagate_piece<real, R, WS, NC, G>(opf, a, Tf, xs, tq, p, tm);
                jump_map<real, R, G>(a, Tf, a.path_op[qs + qq], xs, tm);
              }
              if (!(tau > 0.0)) {
                copy_state(xs, X);  // zero-length piece: only its jump acts
              } else {
                for (int ss = 0; ss < s; ++ss) {
                  cx<real> out[R];
                  tm.sync();
                  taylor_pingpong<real, R, WS, NC, G, -1>(opf, a, Tf, xs, out, hs, p.K, tm);
                  copy_state(out, xs);
                }
                tm.sync();
                taylor_keep<real, R, WS, NC, G, -1>(opf, a, Tf, xs, X, hs, Kg, tm);
              }
            }
            if (s == n - 1 && pc < nj) jump_adjoint<real, R, G>(a, Tc, a.path_op[qs + pc], X, lam, tm);
            if (!(tau > 0.0)) continue;
            {
              // costate: lambda <- exp(+i H^+ hs) lambda with the unit's pairs
              LaneOp<real, R, WS, NC, G> opb;
              load_costate(opb, a, Tc[0], tm.gl);
              costate_grad<real, R, WS, NC, G>(opb, a, Tc, Tf, us, lam, hs, Kg, gl, tm);
            }
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

const void *grad_kernel(int precision, int R, int WS, int NC, int G) {  // WS: layout code
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
  TK_GRAD_CASE(double, 2, ws_code(3, 1, true, 1), 2, 1)
  TK_GRAD_CASE(double, 2, ws_code(5, 2, true, 2), 3, 2)
  TK_GRAD_CASE(float, 2, ws_code(3, 1, true, 1), 2, 1)
  TK_GRAD_CASE(float, 4, ws_code(5, 3, true, 2), 3, 1)
  TK_GRAD_CASE(float, 2, ws_code(5, 2, true, 2), 3, 2)
  TK_GRAD_CASE(float, 3, ws_code(8, 4, true, 4), 4, 8)
#undef TK_GRAD_CASE
  return nullptr;
}

const void *grad_reduce_kernel() { return reinterpret_cast<const void *>(&k_grad_reduce); }

size_t grad_lds_bytes(const Variant &v, int teams, int kbuf) {
  const size_t cplx = v.precision == TK_FP64 ? 16 : 8;
  return static_cast<size_t>(teams) * kbuf * (static_cast<size_t>(v.R) * kWave * v.G + 1) * cplx;
}

}  // namespace tk
