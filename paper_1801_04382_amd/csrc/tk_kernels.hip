// HIP kernels for gfx950: quantum-jump trajectories, costates and the
// sequential Krotov pass.
//
// Mapping.  One wavefront (64 lanes) advances one trajectory at a time; lane
// `l` owns the rows r = l + 64 m (m < R) of the state.  Each lane keeps its
// rows of the effective Hamiltonian in registers: the diagonal of
// H0 - (i/2) sum L^+L (one value per row, applied to the lane's own element
// without a gather), and as padded slots WS static slots (its off-diagonal
// elements) and NC control slots (H_i, scaled by u_ij once per step; the
// unscaled values sit in LDS, one copy per block).  Every Taylor
// term of a substep is written to its own per-wave LDS vector; the next term
// gathers from it (all gathers of a matrix-vector product are issued before
// the first multiply, so their latencies overlap).  A padding slot points at
// a trailing zero element that every lane may read at once.  Norms and
// overlaps are FP64 wavefront reductions in a fixed order (DPP within 16-lane
// rows, then the four row sums read as scalars), so every lane holds the
// identical sum.
//
// Step propagator.  exp(-i H_eff h) (forward) or exp(+i H_eff^+ h) (backward)
// applied as a Taylor polynomial.  The step is split into n_sub equal
// substeps so that ||H_eff|| h <= 1, and the order K of each substep is the
// smallest with truncation bound below `tol`; both follow from a norm bound of
// the step's H_eff and are uniform across the grid.
//
// Jumps (Sec. 2.1, MCWF steps 3-5 and the remark on precise jump times).  When
// the norm at the end of a (sub)step is below the threshold r, the crossing
// time is found by a safeguarded Newton iteration (bracketed, falling back to
// bisection) on f(s) = ||p(s)||^2 - r, where p(s) = sum_n s^n t_n is the
// substep's Taylor polynomial evaluated from the stored terms t_n (dense
// output: U(s tau) psi for s in [0, 1], to the same truncation error), so no
// step is propagated again.  The jump operator is then drawn with weights
// ||L_l psi||^2, applied, the state renormalised, and the rest of the substep
// propagated, so several jumps may fall in one step.
//
// Sequential Krotov pass (Sec. 2.2 "sequential", Sec. 2.3 update).  One
// cooperative persistent launch; waves own `traj_per_wave` trajectories
// whose states stay in LDS across steps.  Right after a trajectory advances
// to t_{j+1}, its share of sum_k Im <chi_k(t_{j+1})|H_i|psi_hat_k(t_{j+1})>
// is formed (the costate loads were issued before the advance, so their
// latency is hidden).  Each block sums its waves in a fixed order, publishes
// the FP64 partials into its own slot of a per-step array (initialised to a
// sentinel), and polls until every block's partial of that step is present;
// all blocks then sum the partials in block order, so they obtain the same
// u_ij bit for bit without a broadcast.
#include <hip/hip_runtime.h>

#include "tk_device.h"
#include "tk_internal.h"

namespace tk {
namespace {


// ---- plain forward / backward passes --------------------------------------
// Blocks hold kWavesPerBlock one-wave teams (G = 1) or one G-wave team.
template <typename real, int R, int WS, int NC, int G, int DIR>
__global__ __launch_bounds__(kWave *(G > kWavesPerBlock ? G : kWavesPerBlock)) void k_pass(
    PassArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double team_red[8 * G];
  constexpr int kL = Team<G>::kLanes;
  const int team = __builtin_amdgcn_readfirstlane(threadIdx.x / kL);
  const int tpb = blockDim.x / kL;
  const Team<G> tm = make_team<G>(team_red);
  LaneOp<real, R, WS, NC, G> op;
  const Terms<real, R, G> T = block_setup<real, R, WS, NC, G>(
      a, smem_raw, team, tm, terms_bytes<real, R, G>(a.kbuf), op);
  const int nteams = gridDim.x * tpb;
  for (int k = blockIdx.x * tpb + team; k < a.M; k += nteams)
    pass_trajectory<real, R, WS, NC, G, DIR>(op, a, T, k, make_stream(a, k, DIR), tm);
}

// ---- slot initialisation for the Krotov pass ---------------------------------
// slots[j][b][c]: the sentinel for the nblk live blocks, zero for the others.
__global__ void k_fill_slots(unsigned long long *slots, long long n, int nblk, int ncx) {
  const long long stride = static_cast<long long>(gridDim.x) * blockDim.x;
  for (long long i = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; i < n;
       i += stride) {
    const int b = static_cast<int>((i / ncx) % kMaxBlocks);
    slots[i] = b < nblk ? kSlotEmpty : 0ull;
  }
}

// ---- sequential Krotov forward pass (cooperative launch) ---------------------
// GS: the trajectories' states live in global memory (a.kstates), for more
// trajectories than the LDS holds; a separate instantiation, so that the LDS
// form keeps its own register allocation.
template <typename real, int R, int WS, int NC, int G, bool GS>
__global__ __launch_bounds__(kWave *(G > kWavesPerBlock ? G : kWavesPerBlock)) void k_krotov(
    PassArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  constexpr int NCX = NC > 0 ? NC : 1;
  constexpr int kL = Team<G>::kLanes;
  __shared__ double wpart[kWavesPerBlock][NCX];
  __shared__ double s_upd[NCX];
  __shared__ int s_abort;
  __shared__ double team_red[8 * G];
  const int lane = threadIdx.x & (kWave - 1);
  const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave-uniform
  const int team = __builtin_amdgcn_readfirstlane(threadIdx.x / kL);
  const int tpb = blockDim.x / kL;  // teams per block
  const Team<G> tm = make_team<G>(team_red);
  const int Tw = a.traj_per_wave;
  const int tglob = blockIdx.x * tpb + team;
  // LDS per team: term vectors, then Tw state vectors, then Tw bookkeeping
  // (the states and their bookkeeping live in global memory instead when
  // a.kstates is set: more trajectories per team than the LDS holds)
  // (the state vectors live in global memory instead with GS: more
  // trajectories per team than the LDS holds; each lane reads back only the
  // rows it wrote)
  constexpr bool states_in_lds = !GS;
  const size_t tb = terms_bytes<real, R, G>(a.kbuf);
  const size_t sb = states_in_lds ? static_cast<size_t>(Tw) * R * kL * sizeof(cx<real>) : 0;
  // (rounded to 16 bytes: every team's vectors keep the alignment of cx<real>)
  const size_t team_bytes = (tb + sb + static_cast<size_t>(Tw) * sizeof(TrajMeta) + 15) / 16 * 16;
  LaneOp<real, R, WS, NC, G> op;
  const Terms<real, R, G> T =
      block_setup<real, R, WS, NC, G>(a, smem_raw, team, tm, team_bytes, op);
  cx<real> *states_lds =
      reinterpret_cast<cx<real> *>(reinterpret_cast<unsigned char *>(T.base) + tb);
  cx<real> *states_glb =
      GS ? static_cast<cx<real> *>(a.kstates) + static_cast<size_t>(tglob) * Tw * R * kL : nullptr;
  TrajMeta *meta = reinterpret_cast<TrajMeta *>(reinterpret_cast<unsigned char *>(T.base) + tb + sb);
  auto load_state = [&](int t, cx<real>(&p)[R]) {
    if constexpr (states_in_lds) {
      load_lds(states_lds + static_cast<size_t>(t) * R * kL, p, tm);
    } else {
#pragma unroll
      for (int m = 0; m < R; ++m)
        p[m] = gld(states_glb, static_cast<size_t>(t) * R * kL + tm.gl + kL * m);
    }
  };
  auto store_state = [&](int t, const cx<real>(&p)[R]) {
    if constexpr (states_in_lds) {
      store_lds(states_lds + static_cast<size_t>(t) * R * kL, p, tm);
    } else {
#pragma unroll
      for (int m = 0; m < R; ++m)
        gst(states_glb, static_cast<size_t>(t) * R * kL + tm.gl + kL * m, p[m]);
    }
  };
  cx<real> *v = T[0];  // scratch vector for the update's gathers
  const cx<real> *start = static_cast<const cx<real> *>(a.psi_start);
  if (threadIdx.x == 0) s_abort = 0;
  if (threadIdx.x < NCX) s_upd[threadIdx.x] = 0.0;  // stays zero without controls

  // ---- start states and the first partial (t_0) ----
  double pc[NCX];
#pragma unroll
  for (int c = 0; c < NCX; ++c) pc[c] = 0.0;
  for (int t = 0; t < Tw; ++t) {
    const int k = tglob * Tw + t;
    cx<real> p[R];
#pragma unroll
    for (int m = 0; m < R; ++m) p[m] = start[tm.gl + kL * m];
    store_state(t, p);
    const double n = norm2(p, tm);
    TrajMeta st;
    st.nrm2 = n;
    st.ordinal = 0;
    st.pad = 0;
    st.r = 0.0;
    st.x = 0.0;
    if (k < a.M) make_stream(a, k, 0).draw(0, st);
    if (tm.leader()) meta[t] = st;
    if (k < a.M) {
      cx<real> ch[R];
      load_costate<real, R, G>(a, 0, k, tm, ch);
      store_lds(v, p, tm);
      tm.sync();
      krotov_share<real, R, WS, NC, G>(op, ch, 1.0 / sqrt(n), pc);
      tm.sync();
    }
  }

  // rows past n_ctrl of the pulse inputs are zero padding (lambda padded with
  // 1), so no guards are needed
  double inv_lm[NCX];
#pragma unroll
  for (int i = 0; i < NCX; ++i) inv_lm[i] = 1.0 / (a.lam[i] * a.M);
  double u_prev[NCX];  // block 0: the previous step's new pulse, stored with the next publish
  OrderHint khint;     // the previous step's order
  // One trajectory per team with its state in LDS: the state stays in term
  // vector 0 from its share to its next step, so the pulse-independent parts
  // of that step's first series term are formed while the grid exchanges the
  // step's partials, and the term itself needs no LDS round trip.  Shapes
  // with more rows per lane or multi-wave teams have no registers to spare
  // for the parts (they would spill) and take the gathered term.
  constexpr bool kFT = !GS && G == 1 && R <= 2;
  const bool use_ft = kFT && Tw == 1;
  cx<real> ft_ys[R], ft_bc[NCX][R];
  for (int j = 0; j < a.nt; ++j) {
    // pulse inputs of interval j, loaded now and used after the exchange
    double uo[NCX], so[NCX];
#pragma unroll
    for (int i = 0; i < NCX; ++i) {
      const size_t ij = static_cast<size_t>(i) * a.nt + j;
      uo[i] = a.u_old[ij];
      so[i] = a.S[ij];
    }
    // ---- reduce the partial of t_j: waves -> block (fixed order) -> publish ----
    tm.template sum_n<NC>(pc);
    if (tm.leader())
#pragma unroll
      for (int c = 0; c < NC; ++c) wpart[team][c] = pc[c];
    block_sync_lds();
    if (threadIdx.x < NCX) {  // control i's block partial (zero for padding controls)
      const int i = threadIdx.x;
      double s = 0.0;
      for (int w = 0; w < tpb; ++w)
        for (int c = i * a.wc; c < (i + 1) * a.wc && c < NC; ++c) s += wpart[w][c];
      __hip_atomic_store(&a.slots[(static_cast<size_t>(j) * kMaxBlocks + blockIdx.x) * NCX + i],
                         __double_as_longlong(s), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      // the new pulse of interval j - 1 leaves with this step's publish, so no
      // wave waits for its write on its own
      if (blockIdx.x == 0 && j > 0) a.u_new[static_cast<size_t>(i) * a.nt + j - 1] = pick(u_prev, i);
    }
    if constexpr (kFT)
      if (use_ft) {
        cx<real> own[R];
        load_lds(T[0], own, tm);
        first_term_parts(op, own, ft_ys, ft_bc);
      }
    // ---- wait for every block's partial of step j; sum in block order --------
    if (wib == 0 && a.n_ctrl > 0) {
      // every lane reads kPollPerLane blocks' slots in one batch of loads (slots of
      // blocks past the grid hold zero, so the sum over all kMaxBlocks is exact).
      // One batch is in flight at a time: when the loop ends no load is left
      // outstanding for later code to wait for.
      const unsigned long long *row = a.slots + static_cast<size_t>(j) * kMaxBlocks * NCX;
      double acc[NCX];
      long long spins = 0;
      bool abort = false;
      for (;;) {
        unsigned long long bits[kPollPerLane][NCX];
        poll_slots<NCX>(row, lane, bits);
        if (slots_complete<NCX>(bits, acc)) break;
        // another block's abort is looked for only now and then
        if (++spins > a.spin_limit ||
            ((spins & 255) == 0 &&
             (__hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &
              kErrSyncTimeout))) {
#pragma unroll
          for (int c = 0; c < NCX; ++c) acc[c] = 0.0;
          abort = true;
          break;
        }
      }
      wave_sum_n<NCX>(acc);
      if (lane == 0)
#pragma unroll
        for (int c = 0; c < NCX; ++c) s_upd[c] = acc[c];
      if (abort && lane == 0) {
        atomicOr(a.err, kErrSyncTimeout);
        s_abort = 1;
      }
    }
    block_sync_lds();
    if (s_abort) return;  // uniform across the block
    // ---- pulse update of interval j ---------------------------------------------
    double uj[NCX];
#pragma unroll
    for (int i = 0; i < NCX; ++i) {
      const double sf = so[i] * inv_lm[i];
      uj[i] = uo[i] + sf * s_upd[i];
      u_prev[i] = uj[i];
    }
    op.set_pulses(uj, a.wc);
    const StepPlan p = plan_step(a, uj, khint);
    // ---- advance every trajectory; form the partial of t_{j+1} ----------------
#pragma unroll
    for (int c = 0; c < NCX; ++c) pc[c] = 0.0;
    for (int t = 0; t < Tw; ++t) {
      const int k = tglob * Tw + t;
      if (k >= a.M) break;
      cx<real> ch[R];
      if (j + 1 < a.nt) load_costate<real, R, G>(a, j + 1, k, tm, ch);
      cx<real> psi[R];
      load_state(t, psi);
      TrajMeta st = meta[t];
      const Stream rng = make_stream(a, k, 0);
      cx<real> y1[R];
      if constexpr (kFT)
        if (use_ft) first_term_finish(op, ft_ys, ft_bc, y1);
      advance_step<real, R, WS, NC, G, 0, true, kFT>(op, a, T, psi, st, rng, j, p, k, tm, &y1,
                                                      use_ft);
      tm.sync();
      store_state(t, psi);
      if (tm.leader()) meta[t] = st;
      if (j + 1 < a.nt) {
        store_lds(v, psi, tm);
        tm.sync();
        krotov_share<real, R, WS, NC, G>(op, ch, 1.0 / sqrt(st.nrm2), pc);
      }
      tm.sync();
    }
  }
  if (blockIdx.x == 0 && threadIdx.x < NCX) a.u_new[static_cast<size_t>(threadIdx.x) * a.nt + a.nt - 1] = pick(u_prev, threadIdx.x);
  // ---- functional: tau_k = <tgt|psi_hat_k(T)> and the final states ----------
  cx<real> *psiT = static_cast<cx<real> *>(a.psiT);
  for (int t = 0; t < Tw; ++t) {
    const int k = tglob * Tw + t;
    if (k >= a.M) break;
    const double inv = 1.0 / sqrt(meta[t].nrm2);
    cx<real> ps[R];
    load_state(t, ps);
    double tr = 0.0, ti = 0.0;
#pragma unroll
    for (int m = 0; m < R; ++m) {
      const int row = tm.gl + kL * m;
      const cx<real> q = ps[m];
      const double px = q.x * inv, py = q.y * inv;
      const double gx = a.tgt[2 * row], gy = a.tgt[2 * row + 1];
      tr = fma(gx, px, fma(gy, py, tr));
      ti = fma(gx, py, fma(-gy, px, ti));
      if (psiT != nullptr && row < a.d)
        psiT[static_cast<size_t>(k) * a.d + row] =
            cx<real>{static_cast<real>(px), static_cast<real>(py)};
    }
    tr = tm.sum(tr);
    ti = tm.sum(ti);
    if (tm.leader() && a.tau_out != nullptr) {
      a.tau_out[2 * k] = tr;
      a.tau_out[2 * k + 1] = ti;
    }
  }
}

// J_T = 1 - (1/M) sum_k |tau_k|^2 (trajectory functional, Sec. 2.3); fixed order.
__global__ __launch_bounds__(256) void k_functional(const double *tau, int M, double *J) {
  __shared__ double part[256];
  double s = 0.0;
  for (int k = threadIdx.x; k < M; k += 256)
    s = fma(tau[2 * k], tau[2 * k], fma(tau[2 * k + 1], tau[2 * k + 1], s));
  part[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (static_cast<int>(threadIdx.x) < off) part[threadIdx.x] += part[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *J = 1.0 - part[0] / static_cast<double>(M);
}

template <typename real, int R, int WS, int NC, int G>
Variant make_variant(const char *name) {
  Variant v;
  v.name = name;
  v.precision = sizeof(real) == 8 ? TK_FP64 : TK_FP32;
  v.R = R;
  v.WS = ws_first(WS);
  v.WSB = ws_rest(WS);
  v.ws_code = WS;
  v.real_ctrl = ws_real_ctrl(WS);
  v.typed_imag = ws_typed(WS) ? ws_imag(WS) : -1;
  v.NC = NC;
  v.G = G;
  v.k_forward = reinterpret_cast<const void *>(&k_pass<real, R, WS, NC, G, 0>);
  v.k_backward = reinterpret_cast<const void *>(&k_pass<real, R, WS, NC, G, 1>);
  v.k_krotov = reinterpret_cast<const void *>(&k_krotov<real, R, WS, NC, G, false>);
  v.k_krotov_gs = reinterpret_cast<const void *>(&k_krotov<real, R, WS, NC, G, true>);
  v.k_fill = reinterpret_cast<const void *>(&k_fill_slots);
  v.k_grad = grad_kernel(v.precision, R, WS, NC, G);  // WS: the layout code
  return v;
}

}  // namespace

const Variant *variants(int *count) {
  static const Variant table[] = {
      make_variant<double, 1, 4, 2, 1>("fp64 R=1 WS=4 NC=2"),
      make_variant<double, 2, 4, 2, 1>("fp64 R=2 WS=4 NC=2"),
      make_variant<double, 4, 6, 3, 1>("fp64 R=4 WS=6 NC=3"),
      make_variant<double, 4, 8, 4, 1>("fp64 R=4 WS=8 NC=4"),
      make_variant<double, 1, 4, 2, 2>("fp64 R=1 WS=4 NC=2 G=2"),
      make_variant<double, 2, 6, 3, 2>("fp64 R=2 WS=6 NC=3 G=2"),
      make_variant<float, 1, 4, 2, 1>("fp32 R=1 WS=4 NC=2"),
      make_variant<float, 2, 4, 2, 1>("fp32 R=2 WS=4 NC=2"),
      make_variant<float, 4, 6, 3, 1>("fp32 R=4 WS=6 NC=3"),
      make_variant<float, 4, 8, 4, 1>("fp32 R=4 WS=8 NC=4"),
      make_variant<float, 1, 4, 2, 2>("fp32 R=1 WS=4 NC=2 G=2"),
      make_variant<float, 2, 6, 3, 2>("fp32 R=2 WS=6 NC=3 G=2"),
      make_variant<float, 3, 9, 4, 8>("fp32 R=3 WS=9 NC=4 G=8"),
      // heaviest rows in row slot 0, fewer static slots in the others
      make_variant<double, 2, ws_code(3, 1, true, 1), 2, 1>("fp64 R=2 WS=3/1 NC=2"),
      make_variant<double, 2, ws_code(5, 2, true, 2), 3, 2>("fp64 R=2 WS=5/2 NC=3 G=2"),
      make_variant<float, 2, ws_code(3, 1, true, 1), 2, 1>("fp32 R=2 WS=3/1 NC=2"),
      make_variant<float, 4, ws_code(5, 3, true, 2), 3, 1>("fp32 R=4 WS=5/3 NC=3"),
      make_variant<float, 2, ws_code(5, 2, true, 2), 3, 2>("fp32 R=2 WS=5/2 NC=3 G=2"),
      make_variant<float, 3, ws_code(8, 4, true, 4), 4, 8>("fp32 R=3 WS=8/4 NC=4 G=8"),
      // d = 1296 in FP64: one team's LDS holds five FP64 term vectors, so its
      // steps take substeps short enough for four-term series (several
      // times the work of the FP32 shape; it serves accuracy checks)
      make_variant<double, 3, ws_code(8, 4, true, 4), 4, 8>("fp64 R=3 WS=8/4 NC=4 G=8"),
  };
  *count = static_cast<int>(sizeof(table) / sizeof(table[0]));
  return table;
}

const void *functional_kernel() { return reinterpret_cast<const void *>(&k_functional); }

size_t block_lds_bytes(const Variant &v, int teams, int kbuf, int traj_per_wave,
                       bool states_in_lds) {
  const size_t cplx = v.precision == TK_FP64 ? 16 : 8;
  const size_t ncx = v.NC > 0 ? v.NC : 1;
  const size_t rows = static_cast<size_t>(v.R) * kWave * v.G;
  const size_t per_team = (static_cast<size_t>(kbuf) * (rows + 1) * cplx +
                           (states_in_lds ? static_cast<size_t>(traj_per_wave) * rows * cplx : 0) +
                           static_cast<size_t>(traj_per_wave) * sizeof(TrajMeta) + 15) / 16 * 16;
  // one-wave teams share a block copy of the control values; G-wave teams read them
  // from global memory
  return (v.G == 1 ? ncx * rows * cplx : 0) + static_cast<size_t>(teams) * per_team;
}

}  // namespace tk
