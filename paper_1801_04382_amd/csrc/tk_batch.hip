// Batched kernels: many independent optimisation instances in one launch.
//
// Every instance has its own system (operator slices), states, pulses,
// costates and random streams (the instance index is part of the Philox key),
// and its own kernel shape (rows per lane, slots).  Every shape has kernels of
// its own, compiled for that shape alone, so a small shape is not held to the
// registers of the largest one (more waves per SIMD); the instances of one
// shape are served by one launch, the shapes one after another.
//
// Plain passes (guess forward, costates): a list of (instance, trajectory)
// items of one shape, costliest first, dealt round-robin to the waves; an item
// is one trajectory over all of its instance's steps, computed by the same
// device code as the single-system passes.
//
// Sequential Krotov pass: each instance of the launch's shape owns a contiguous
// range of its blocks, all co-resident.  Trajectory states live in device memory between steps.
// After a trajectory reaches t_j its own FP64 share of
// s_ij = sum_k Im <chi_k(t_j)|H_i|psi_hat_k(t_j)> is published into a
// per-trajectory slot (initialised to a sentinel); every block of the instance
// waits for the M shares of step j, all its waves reading parts of them, and
// sums them in one fixed order (block_gather).  The update is therefore
// independent of how trajectories are split over waves and blocks:
// an instance gives bit-identical pulses whatever the tile shape chosen and
// whatever else runs in the batch.
//
// Instances whose shape needs a team of G > 1 waves per trajectory run in
// kernels of their own (k_batch_wide_*, one team per block, launched after the
// one-wave kernels of the same pass), with the same items, shares and gather.
// They do not store their costates: the backward pass keeps checkpoints every
// kSegment steps, and the Krotov pass recomputes each segment's costates from
// its checkpoint before the segment's first step.
#include <hip/hip_runtime.h>

#include "tk_device.h"
#include "tk_internal.h"

namespace tk {
namespace {

// One-wave kernel shapes of the batch: (index, R, WS layout code, NC).
#define TK_BATCH_SHAPES(X)   \
  X(0, 1, 4, 2)              \
  X(1, 2, 4, 2)              \
  X(2, 4, 6, 3)              \
  X(3, 4, 8, 4)              \
  X(4, 2, ws_code(3, 1, true, 1), 2)  \
  X(5, 4, ws_code(5, 3, true, 2), 3)

// ---- plain passes ------------------------------------------------------------
template <typename real, int R, int WS, int NC, int DIR>
__device__ void batch_pass_item(const PassArgs &a, int k, uint64_t it, unsigned char *wave_lds,
                                const Team<1> &tm) {
  const int lane = tm.lane;
  constexpr int NCX = NC > 0 ? NC : 1;
  cx<real> *cval_lds = reinterpret_cast<cx<real> *>(wave_lds);
  const cx<real> *cval_g = static_cast<const cx<real> *>(a.cval);
  wave_sync();  // the previous item's reads of this wave's LDS are done
  for (int i = lane; i < NCX * R * kWave; i += kWave) cval_lds[i] = cval_g[i];
  Terms<real, R, 1> T;
  T.base = cval_lds + NCX * R * kWave;
  if (lane < a.kbuf) T[lane][R * kWave] = cx<real>{0, 0};
  wave_sync();
  LaneOp<real, R, WS, NC, 1> op;
  op.load(a.scol, a.sval, a.sdiag, a.ccol, cval_lds, lane);
  op.bind(T[0]);
  pass_trajectory<real, R, WS, NC, 1, DIR>(op, a, T, k, make_stream(a, k, DIR, it), tm);
}

// Plain pass over the items of shape S (b.items holds only those).
template <typename real, int DIR, int S>
__global__ __launch_bounds__(kWave *kWavesPerBlock) void k_batch_pass(BatchArgs b) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const Team<1> tm = make_team<1>(nullptr);
  const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int wpb = blockDim.x / kWave;
  unsigned char *wl = smem_raw + static_cast<size_t>(wib) * b.wave_lds;
  const uint64_t it = *b.iteration;
  const int nwaves = gridDim.x * wpb;
  for (int q = blockIdx.x * wpb + wib; q < b.n_items; q += nwaves) {
    const int2 item = b.items[q];
    const BatchInstance &I = b.inst[__builtin_amdgcn_readfirstlane(item.x)];
    const PassArgs &a = DIR == 0 ? I.fw : I.bw;
    const int k = __builtin_amdgcn_readfirstlane(item.y);
    if (I.variant != S) continue;  // not an item of this launch (none are given)
#define TK_CASE(idx, R, WS, NC) \
  if constexpr (idx == S) batch_pass_item<real, R, WS, NC, DIR>(a, k, it, wl, tm);
    TK_BATCH_SHAPES(TK_CASE)
#undef TK_CASE
  }
}

// ---- sequential Krotov pass ------------------------------------------------------
// slots[(j M + k) NCX + i] <- the trajectory's share of control i (lane 0)
template <int NC>
__device__ __forceinline__ void publish_share(const PassArgs &a, unsigned long long *row, int k,
                                              const double (&pc)[NC > 0 ? NC : 1], int lane) {
  constexpr int NCX = NC > 0 ? NC : 1;
  double sc[NCX];
#pragma unroll
  for (int c = 0; c < NCX; ++c) sc[c] = c < NC ? pc[c] : 0.0;
  wave_sum_n<NC>(sc);  // two sums per exchange; the same bits as one at a time
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NCX; ++i) {
      double s = 0.0;  // control i owns slots i wc .. i wc + wc - 1
#pragma unroll
      for (int c = 0; c < NCX; ++c)
        if (c >= i * a.wc && c < (i + 1) * a.wc) s += sc[c];
      __hip_atomic_store(gmem(row) + (static_cast<size_t>(k) * NCX + i), __double_as_longlong(s),
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// Loads of the shares of trajectories lane + 64 (q0 + qq), qq < CH (0 past M).
template <int NCX, int CH>
__device__ __forceinline__ void load_shares(const unsigned long long *row, int M, int lane, int q0,
                                            unsigned long long (&v)[CH][NCX]) {
#pragma unroll
  for (int qq = 0; qq < CH; ++qq) {
    const int k = lane + kWave * (q0 + qq);
#pragma unroll
    for (int c = 0; c < NCX; ++c)
      v[qq][c] = k < M ? __hip_atomic_load(gmem(row) + (static_cast<size_t>(k) * NCX + c),
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                       : 0ull;
  }
}

// The M shares of one step are summed in a fixed order that does not depend on
// how trajectories, waves or blocks are split: the trajectories form groups of
// 64 CH (k = 64 (CH q + qq) + l, qq < CH), and group q belongs to part
// q mod kGatherParts.  Lane l sums its column of each part over the part's
// groups in increasing k; the parts' column sums are added in part order, then
// reduced over the lanes (wave tree).  Every wave of a block reads some of the
// parts (wave w takes parts w, w + waves, ...), so a block has up to
// kGatherParts groups of loads in flight instead of one.
constexpr int kGatherParts = 4;

// Column sums of part r (lane, control); waits for missing shares, reading a
// group again until it is complete while the part's next group is in flight.
// Returns false if the spin limit is reached or another block gave up.
template <int NCX>
__device__ bool gather_part(const unsigned long long *row, int M, int lane, int r,
                            long long spin_limit, int *err, double (&acc)[NCX]) {
  constexpr int CH = 4;
  constexpr int kStride = CH * kGatherParts;  // between a part's groups, in units of 64
#pragma unroll
  for (int c = 0; c < NCX; ++c) acc[c] = 0.0;
  if (r * CH * kWave >= M) return true;
  long long spins = 0;
  unsigned long long cur[CH][NCX], nxt[CH][NCX];
  load_shares<NCX, CH>(row, M, lane, r * CH, cur);
  for (int q0 = r * CH; q0 * kWave < M; q0 += kStride) {
    const bool more = (q0 + kStride) * kWave < M;
    if (more) load_shares<NCX, CH>(row, M, lane, q0 + kStride, nxt);
    __builtin_amdgcn_sched_barrier(0);
    for (;;) {
      int missing = 0;
#pragma unroll
      for (int qq = 0; qq < CH; ++qq)
#pragma unroll
        for (int c = 0; c < NCX; ++c) missing |= cur[qq][c] == kSlotEmpty;
      if (!__any(missing)) break;
      if (++spins > spin_limit ||
          ((spins & 255) == 0 &&
           (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kErrSyncTimeout)))
        return false;
      load_shares<NCX, CH>(row, M, lane, q0, cur);
    }
#pragma unroll
    for (int qq = 0; qq < CH; ++qq)
#pragma unroll
      for (int c = 0; c < NCX; ++c) acc[c] += __longlong_as_double(static_cast<long long>(cur[qq][c]));
    if (more) {
#pragma unroll
      for (int qq = 0; qq < CH; ++qq)
#pragma unroll
        for (int c = 0; c < NCX; ++c) cur[qq][c] = nxt[qq][c];
    }
  }
  return true;
}

// The update's sums s_upd[c] of one step (0 without controls), from the shares
// in `row`, by the block's `nwaves` waves.  On a timeout the block's abort flag
// is set.  Ends with the sums in s_upd for wave 0 only: the caller's block
// barrier publishes them.
template <int NCX>
__device__ __forceinline__ void block_gather(const unsigned long long *row, int M, bool active,
                                             const BatchArgs &b, int nwaves,
                                             double (&s_part)[kGatherParts][NCX][kWave],
                                             double *s_upd, int *s_abort) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  if (active) {
    bool ok = true;
    for (int r = wib; r < kGatherParts && ok; r += nwaves) {
      double acc[NCX];
      ok = gather_part<NCX>(row, M, lane, r, b.spin_limit, b.err, acc);
#pragma unroll
      for (int c = 0; c < NCX; ++c) s_part[r][c][lane] = acc[c];
    }
    if (!ok && lane == 0) {
      atomicOr(b.err, kErrSyncTimeout);
      *s_abort = 1;
    }
  }
  block_sync_lds();
  if (wib == 0) {
    double acc[NCX];
#pragma unroll
    for (int c = 0; c < NCX; ++c) acc[c] = 0.0;
    if (active)
#pragma unroll
      for (int r = 0; r < kGatherParts; ++r)
#pragma unroll
        for (int c = 0; c < NCX; ++c) acc[c] += s_part[r][c][lane];
    wave_sum_n<NCX>(acc);
    if (lane == 0)
#pragma unroll
      for (int c = 0; c < NCX; ++c) s_upd[c] = acc[c];
  }
}

template <typename real, int R, int WS, int NC>
__device__ void batch_krotov_instance(const BatchArgs &b, const BatchInstance &I, int lb,
                                      uint64_t it, unsigned char *smem, double *s_upd,
                                      int *s_abort) {
  constexpr int NCX = NC > 0 ? NC : 1;
  constexpr int kRows = R * kWave;
  const PassArgs &a = I.fw;
  const Team<1> tm = make_team<1>(nullptr);
  const int lane = tm.lane;
  const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int wpb = blockDim.x / kWave;
  __shared__ double s_part[kGatherParts][NCX][kWave];  // column sums of the gather's parts
  LaneOp<real, R, WS, NC, 1> op;
  const Terms<real, R, 1> T =
      block_setup<real, R, WS, NC, 1>(a, smem, wib, tm, terms_bytes<real, R, 1>(a.kbuf), op);
  const int nw = I.nblocks * wpb;
  const int w = lb * wpb + wib;
  cx<real> *psi_g = static_cast<cx<real> *>(I.psi);
  TrajMeta *meta_g = I.meta;
  cx<real> *v = T[0];  // scratch vector for the update's gathers
  const cx<real> *start = static_cast<const cx<real> *>(a.psi_start);
  const size_t row_len = static_cast<size_t>(a.M) * NCX;

  // ---- start states and their shares at t_0 ----
  for (int k = w; k < a.M; k += nw) {
    cx<real> p[R];
#pragma unroll
    for (int m = 0; m < R; ++m) {
      p[m] = gld(start, lane + kWave * m);
      gst(psi_g, static_cast<size_t>(k) * kRows + lane + kWave * m, p[m]);
    }
    const double n = norm2(p, tm);
    TrajMeta st;
    st.nrm2 = n;
    make_stream(a, k, 0, it).draw(0, st);
    st.ordinal = 0;
    st.pad = 0;
    if (lane == 0) gst(meta_g, k, st);
    cx<real> ch[R];
    load_costate<real, R, 1>(a, 0, k, tm, ch);
    double pc[NCX];
#pragma unroll
    for (int c = 0; c < NCX; ++c) pc[c] = 0.0;
    wave_sync();
    store_lds(v, p, tm);
    wave_sync();
    krotov_share<real, R, WS, NC, 1>(op, ch, 1.0 / sqrt(n), pc);
    publish_share<NC>(a, I.tslots, k, pc, lane);
  }

  double inv_lm[NCX];
#pragma unroll
  for (int i = 0; i < NCX; ++i) inv_lm[i] = 1.0 / (a.lam[i] * a.M);
  double u_prev[NCX];  // first block: the previous step's new pulse, written this step
  OrderHint khint;     // the previous step's order
  for (int j = 0; j < a.nt; ++j) {
    // pulse inputs of interval j, loaded now and used after the exchange
    double uo[NCX], so[NCX];
#pragma unroll
    for (int i = 0; i < NCX; ++i) {
      const size_t ij = static_cast<size_t>(i) * a.nt + j;
      uo[i] = gmem(a.u_old)[ij];
      so[i] = gmem(a.S)[ij];
    }
    block_sync_lds();  // every wave has used the previous step's s_upd
    if (lb == 0 && j > 0 && threadIdx.x < NCX)
      gmem(a.u_new)[static_cast<size_t>(threadIdx.x) * a.nt + j - 1] = pick(u_prev, threadIdx.x);
    block_gather<NCX>(I.tslots + static_cast<size_t>(j) * row_len, a.M, a.n_ctrl > 0, b, wpb,
                      s_part, s_upd, s_abort);
    block_sync_lds();
    if (*s_abort) return;  // uniform across the block
    double uj[NCX];
#pragma unroll
    for (int i = 0; i < NCX; ++i) {
      const double sf = so[i] * inv_lm[i];
      uj[i] = uo[i] + sf * s_upd[i];
      u_prev[i] = uj[i];
    }
    op.set_pulses(uj, a.wc);
    const StepPlan p = plan_step(a, uj, khint);
    // the wave's trajectories in turn; the state, clock and costate of the next
    // one are loaded while the current one advances
    cx<real> psi[R], ch[R];
    TrajMeta st;
    if (w < a.M) {
#pragma unroll
      for (int m = 0; m < R; ++m) psi[m] = gld(psi_g, static_cast<size_t>(w) * kRows + lane + kWave * m);
      st = gld(meta_g, w);
      if (j + 1 < a.nt) load_costate<real, R, 1>(a, j + 1, w, tm, ch);
    }
    for (int k = w; k < a.M; k += nw) {
      const int kn = k + nw;
      cx<real> psi_n[R], ch_n[R];
      TrajMeta st_n;
      if (kn < a.M) {
#pragma unroll
        for (int m = 0; m < R; ++m)
          psi_n[m] = gld(psi_g, static_cast<size_t>(kn) * kRows + lane + kWave * m);
        st_n = gld(meta_g, kn);
        if (j + 1 < a.nt) load_costate<real, R, 1>(a, j + 1, kn, tm, ch_n);
      }
      const Stream rng = make_stream(a, k, 0, it);
      advance_step<real, R, WS, NC, 1, 0, true>(op, a, T, psi, st, rng, j, p, k, tm);
#pragma unroll
      for (int m = 0; m < R; ++m) gst(psi_g, static_cast<size_t>(k) * kRows + lane + kWave * m, psi[m]);
      if (lane == 0) gst(meta_g, k, st);
      if (j + 1 < a.nt) {
        double pc[NCX];
#pragma unroll
        for (int c = 0; c < NCX; ++c) pc[c] = 0.0;
        wave_sync();
        store_lds(v, psi, tm);
        wave_sync();
        krotov_share<real, R, WS, NC, 1>(op, ch, 1.0 / sqrt(st.nrm2), pc);
        publish_share<NC>(a, I.tslots + static_cast<size_t>(j + 1) * row_len, k, pc, lane);
      }
      wave_sync();
      if (kn < a.M) {
#pragma unroll
        for (int m = 0; m < R; ++m) {
          psi[m] = psi_n[m];
          ch[m] = ch_n[m];
        }
        st = st_n;
      }
    }
  }
  if (lb == 0 && threadIdx.x < NCX)
    gmem(a.u_new)[static_cast<size_t>(threadIdx.x) * a.nt + a.nt - 1] = pick(u_prev, threadIdx.x);
  // ---- tau_k = <tgt|psi_hat_k(T)> ----
  for (int k = w; k < a.M; k += nw) {
    const double inv = 1.0 / sqrt(gmem(meta_g)[k].nrm2);
    double tr = 0.0, ti = 0.0;
#pragma unroll
    for (int m = 0; m < R; ++m) {
      const int row = lane + kWave * m;
      const cx<real> q = gld(psi_g, static_cast<size_t>(k) * kRows + row);
      const double px = q.x * inv, py = q.y * inv;
      const double gx = gmem(a.tgt)[2 * row], gy = gmem(a.tgt)[2 * row + 1];
      tr = fma(gx, px, fma(gy, py, tr));
      ti = fma(gx, py, fma(-gy, px, ti));
    }
    tr = wave_sum(tr);
    ti = wave_sum(ti);
    if (lane == 0) {
      gmem(a.tau_out)[2 * k] = tr;
      gmem(a.tau_out)[2 * k + 1] = ti;
    }
  }
}

// Krotov pass of the instances of shape S; b.block_inst maps this launch's
// blocks to them, and I.block0 is relative to the launch.
template <typename real, int S>
__global__ __launch_bounds__(kWave *kWavesPerBlock) void k_batch_krotov(BatchArgs b) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double s_upd[kMaxCtrl];
  __shared__ int s_abort;
  if (threadIdx.x == 0) {
    s_abort = 0;
    atomicMin(b.t_begin, static_cast<unsigned long long>(wall_clock64()));
  }
  const int i = __builtin_amdgcn_readfirstlane(b.block_inst[blockIdx.x]);
  const BatchInstance &I = b.inst[i];
  const int lb = blockIdx.x - I.block0;
  const uint64_t it = *b.iteration;
  if (I.variant == S) {  // uniform over the instance's blocks
#define TK_CASE(idx, R, WS, NC) \
  if constexpr (idx == S) batch_krotov_instance<real, R, WS, NC>(b, I, lb, it, smem_raw, s_upd, &s_abort);
    TK_BATCH_SHAPES(TK_CASE)
#undef TK_CASE
  }
  // the instance's finishing time, for the autotuner's block split
  __syncthreads();
  if (threadIdx.x == 0) atomicMax(&b.t_end[i], static_cast<unsigned long long>(wall_clock64()));
}

// ---- instances of multi-wave shapes (one G-wave team per block) --------------------
// Kernel shapes with G > 1 (indices continue those of TK_BATCH_SHAPES).  The
// eight-wave kernels serve the d = 1296 shape with fewer static slots past
// row slot 0 alone: a second eight-wave shape in the same kernel would set
// its register allocation and spill both.
#define TK_BATCH_WIDE_SHAPES(X)  \
  X(6, 1, 4, 2, 2)               \
  X(7, 2, 6, 3, 2)               \
  X(8, 2, ws_code(5, 2, true, 2), 3, 2)   \
  X(10, 3, ws_code(8, 4, true, 4), 4, 8)

// Term vectors of the block's team at the start of dynamic LDS, trailing
// zero elements set.
template <typename real, int R, int G>
__device__ __forceinline__ Terms<real, R, G> wide_terms(unsigned char *smem, int kbuf,
                                                         const Team<G> &tm) {
  Terms<real, R, G> T;
  T.base = reinterpret_cast<cx<real> *>(smem);
  block_sync_lds();  // earlier readers of these vectors are done
  if (tm.gl < kbuf) T[tm.gl][R * Team<G>::kLanes] = cx<real>{0, 0};
  block_sync_lds();
  return T;
}

template <typename real, int R, int WS, int NC, int G, int DIR>
__device__ void wide_pass_item(const PassArgs &a, int k, uint64_t it, unsigned char *smem,
                               const Team<G> &tm) {
  const Terms<real, R, G> T = wide_terms<real, R, G>(smem, a.kbuf, tm);
  LaneOp<real, R, WS, NC, G> op;
  op.load(a.scol, a.sval, a.sdiag, a.ccol, static_cast<const cx<real> *>(a.cval), tm.gl);
  op.bind(T[0]);
  pass_trajectory<real, R, WS, NC, G, DIR>(op, a, T, k, make_stream(a, k, DIR, it), tm);
}

template <typename real, int DIR, int G>
__global__ __launch_bounds__(kWave *G) void k_batch_wide_pass(BatchArgs b) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double team_red[8 * G];
  const Team<G> tm = make_team<G>(team_red);
  const uint64_t it = *b.iteration;
  for (int q = blockIdx.x; q < b.n_witems; q += gridDim.x) {
    const int2 item = b.witems[q];
    const BatchInstance &I = b.inst[__builtin_amdgcn_readfirstlane(item.x)];
    const PassArgs &a = DIR == 0 ? I.fw : I.bw;
    const int k = __builtin_amdgcn_readfirstlane(item.y);
    switch (I.variant) {
#define TK_CASE(idx, R, WS, NC, GG)                                             \
  case idx:                                                                     \
    if constexpr (GG == G) wide_pass_item<real, R, WS, NC, G, DIR>(a, k, it, smem_raw, tm); \
    break;
      TK_BATCH_WIDE_SHAPES(TK_CASE)
#undef TK_CASE
      default:
        break;
    }
  }
}

// The costates of segment s (chi(t_j), j0 = s kSegment <= j <= e = min(j0 +
// kSegment, nt), slot j - j0 of the instance's segment buffer) of the team's
// trajectories k = w, w + nteam, ..: the backward pass replayed from the
// checkpoint at t_e (from the target at t_nt for the last segment) with the
// same stream, pulses and device code, so every value equals the one the full
// backward pass computes.
template <typename real, int R, int WS, int NC, int G>
__device__ void wide_recompute(const BatchInstance &I, int w, int nteam, int s, uint64_t it,
                               const Terms<real, R, G> &T, const Team<G> &tm) {
  constexpr int kL = Team<G>::kLanes;
  constexpr int NCX = NC > 0 ? NC : 1;
  const PassArgs &ab = I.bw;
  const int nt = ab.nt, M = ab.M, d = ab.d;
  const int j0 = s * kSegment, e = min(j0 + kSegment, nt);
  LaneOp<real, R, WS, NC, G> opb;
  opb.load(ab.scol, ab.sval, ab.sdiag, ab.ccol, static_cast<const cx<real> *>(ab.cval), tm.gl);
  opb.bind(T[0]);
  cx<real> *seg = static_cast<cx<real> *>(I.fw.chi);
  const cx<real> *start = static_cast<const cx<real> *>(ab.psi_start);
  for (int k = w; k < M; k += nteam) {
    cx<real> psi[R];
    TrajMeta st;
    const Stream rng = make_stream(ab, k, 1, it);
    if (e == nt) {
#pragma unroll
      for (int m = 0; m < R; ++m) psi[m] = gld(start, tm.gl + kL * m);
      st.nrm2 = norm2(psi, tm);
      st.ordinal = 0;
      st.pad = 0;
      rng.draw(0, st);
    } else {
      const size_t c = static_cast<size_t>(s) * M + k;
      const cx<real> *ck = static_cast<const cx<real> *>(ab.ck_psi) + c * R * kL;
#pragma unroll
      for (int m = 0; m < R; ++m) psi[m] = gld(ck, tm.gl + kL * m);
      st = gld(ab.ck_meta, c);
    }
    const double tau_re = gmem(ab.tau_in)[2 * k], tau_im = gmem(ab.tau_in)[2 * k + 1];
    if (e < nt)
      store_costate<real, R, G>(seg + (static_cast<size_t>(e - j0) * M + k) * d, d, psi,
                                st.nrm2, tau_re, tau_im, tm);
    OrderHint hint;
    double un[NCX];  // pulses of the next step, loaded one step ahead
#pragma unroll
    for (int i = 0; i < NCX; ++i) un[i] = gmem(ab.u)[static_cast<size_t>(i) * nt + e - 1];
    for (int j = e - 1; j >= j0; --j) {
      double uj[NCX];
#pragma unroll
      for (int i = 0; i < NCX; ++i) uj[i] = un[i];
      if (j > j0)
#pragma unroll
        for (int i = 0; i < NCX; ++i) un[i] = gmem(ab.u)[static_cast<size_t>(i) * nt + j - 1];
      opb.set_pulses(uj, ab.wc);
      const StepPlan p = plan_step(ab, uj, hint);
      advance_step<real, R, WS, NC, G, 1>(opb, ab, T, psi, st, rng, j, p, k, tm);
      store_costate<real, R, G>(seg + (static_cast<size_t>(j - j0) * M + k) * d, d, psi,
                                st.nrm2, tau_re, tau_im, tm);
    }
    tm.sync();  // the term vectors are reused by the next trajectory
  }
}

// Share of one trajectory: pc summed over the team, then per control over its
// slots, into the trajectory's slot of the step (team leader).
template <int NC, int G>
__device__ __forceinline__ void publish_share_team(const PassArgs &a, unsigned long long *row,
                                                   int k, double (&pc)[NC > 0 ? NC : 1],
                                                   const Team<G> &tm) {
  constexpr int NCX = NC > 0 ? NC : 1;
  tm.template sum_n<NC>(pc);
  if (tm.leader()) {
#pragma unroll
    for (int i = 0; i < NCX; ++i) {
      double s = 0.0;  // control i owns slots i wc .. i wc + wc - 1
#pragma unroll
      for (int c = 0; c < NC; ++c)
        if (c >= i * a.wc && c < (i + 1) * a.wc) s += pc[c];
      __hip_atomic_store(gmem(row) + (static_cast<size_t>(k) * NCX + i), __double_as_longlong(s),
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// costate of trajectory k at slot q of the segment buffer (own rows; padding
// rows read row d - 1, see load_costate)
template <typename real, int R, int G>
__device__ __forceinline__ void load_seg_costate(const PassArgs &a, int q, int k, const Team<G> &tm,
                                                 cx<real> (&ch)[R]) {
  const cx<real> *chi = static_cast<const cx<real> *>(a.chi);
  const size_t base = (static_cast<size_t>(q) * a.M + k) * a.d;
#pragma unroll
  for (int m = 0; m < R; ++m) {
    const int row = tm.gl + Team<G>::kLanes * m;
    ch[m] = gld(chi, base + (row < a.d ? row : a.d - 1));
  }
}

// Sequential Krotov pass of one instance of a multi-wave shape; this block is
// team lb of the instance's I.nblocks.  The costates come segment by segment
// (wide_recompute) into one buffer; the shares, the fixed-order gather and the
// update are those of the one-wave instances.
template <typename real, int R, int WS, int NC, int G>
__device__ void wide_krotov_instance(const BatchArgs &b, const BatchInstance &I, int lb,
                                     uint64_t it, unsigned char *smem, double *s_upd,
                                     int *s_abort, const Team<G> &tm) {
  constexpr int NCX = NC > 0 ? NC : 1;
  constexpr int kL = Team<G>::kLanes;
  constexpr int kRows = R * kL;
  const PassArgs &a = I.fw;
  const int nt = a.nt, M = a.M;
  const int nteam = I.nblocks, w = lb;
  __shared__ double s_part[kGatherParts][NCX][kWave];  // column sums of the gather's parts
  const int kbuf = max(I.fw.kbuf, I.bw.kbuf);
  const Terms<real, R, G> T = wide_terms<real, R, G>(smem, kbuf, tm);
  cx<real> *psi_g = static_cast<cx<real> *>(I.psi);
  TrajMeta *meta_g = I.meta;
  const cx<real> *start = static_cast<const cx<real> *>(a.psi_start);
  const size_t row_len = static_cast<size_t>(M) * NCX;
  double inv_lm[NCX];
#pragma unroll
  for (int i = 0; i < NCX; ++i) inv_lm[i] = 1.0 / (a.lam[i] * M);
  double u_prev[NCX];  // first block: the previous step's new pulse, written this step
  const int nseg = (nt + kSegment - 1) / kSegment;
  for (int s = 0; s < nseg; ++s) {
    const int j0 = s * kSegment, j1 = min(j0 + kSegment, nt);
    wide_recompute<real, R, WS, NC, G>(I, w, nteam, s, it, T, tm);
    LaneOp<real, R, WS, NC, G> op;
    op.load(a.scol, a.sval, a.sdiag, a.ccol, static_cast<const cx<real> *>(a.cval), tm.gl);
    op.bind(T[0]);
    if (s == 0) {  // start states and their shares at t_0
      for (int k = w; k < M; k += nteam) {
        cx<real> p[R];
#pragma unroll
        for (int m = 0; m < R; ++m) {
          p[m] = gld(start, tm.gl + kL * m);
          gst(psi_g, static_cast<size_t>(k) * kRows + tm.gl + kL * m, p[m]);
        }
        const double n = norm2(p, tm);
        TrajMeta st;
        st.nrm2 = n;
        make_stream(a, k, 0, it).draw(0, st);
        st.ordinal = 0;
        st.pad = 0;
        if (tm.leader()) gst(meta_g, k, st);
        cx<real> ch[R];
        load_seg_costate<real, R, G>(a, 0, k, tm, ch);
        double pc[NCX];
#pragma unroll
        for (int c = 0; c < NCX; ++c) pc[c] = 0.0;
        tm.sync();
        store_lds(T[0], p, tm);
        tm.sync();
        krotov_share<real, R, WS, NC, G>(op, ch, 1.0 / sqrt(n), pc);
        publish_share_team<NC, G>(a, I.tslots, k, pc, tm);
      }
    }
    OrderHint khint;
    for (int j = j0; j < j1; ++j) {
      double uo[NCX], so[NCX];
#pragma unroll
      for (int i = 0; i < NCX; ++i) {
        const size_t ij = static_cast<size_t>(i) * nt + j;
        uo[i] = gmem(a.u_old)[ij];
        so[i] = gmem(a.S)[ij];
      }
      block_sync_lds();  // every wave has used the previous step's s_upd
      if (lb == 0 && j > 0 && threadIdx.x < NCX)
        gmem(a.u_new)[static_cast<size_t>(threadIdx.x) * nt + j - 1] = pick(u_prev, threadIdx.x);
      block_gather<NCX>(I.tslots + static_cast<size_t>(j) * row_len, M, a.n_ctrl > 0, b, G, s_part,
                        s_upd, s_abort);
      block_sync_lds();
      if (*s_abort) return;  // uniform across the block
      double uj[NCX];
#pragma unroll
      for (int i = 0; i < NCX; ++i) {
        const double sf = so[i] * inv_lm[i];
        uj[i] = uo[i] + sf * s_upd[i];
        u_prev[i] = uj[i];
      }
      op.set_pulses(uj, a.wc);
      const StepPlan p = plan_step(a, uj, khint);
      for (int k = w; k < M; k += nteam) {
        cx<real> psi[R], ch[R];
#pragma unroll
        for (int m = 0; m < R; ++m) psi[m] = gld(psi_g, static_cast<size_t>(k) * kRows + tm.gl + kL * m);
        TrajMeta st = gld(meta_g, k);
        if (j + 1 < nt) load_seg_costate<real, R, G>(a, j + 1 - j0, k, tm, ch);
        const Stream rng = make_stream(a, k, 0, it);
        // (the previous trajectory's reads of the term vectors ended before
        // the team sums that close its share or its advance)
        advance_step<real, R, WS, NC, G, 0, true>(op, a, T, psi, st, rng, j, p, k, tm);
#pragma unroll
        for (int m = 0; m < R; ++m) gst(psi_g, static_cast<size_t>(k) * kRows + tm.gl + kL * m, psi[m]);
        if (tm.leader()) gst(meta_g, k, st);
        if (j + 1 < nt) {
          double pc[NCX];
#pragma unroll
          for (int c = 0; c < NCX; ++c) pc[c] = 0.0;
          // the advance ended with a team sum, after every read of the term
          // vectors, so term vector 0 is free
          store_lds(T[0], psi, tm);
          tm.sync();
          krotov_share<real, R, WS, NC, G>(op, ch, 1.0 / sqrt(st.nrm2), pc);
          publish_share_team<NC, G>(a, I.tslots + static_cast<size_t>(j + 1) * row_len, k, pc, tm);
        }
      }
    }
  }
  if (lb == 0 && threadIdx.x < NCX)
    gmem(a.u_new)[static_cast<size_t>(threadIdx.x) * nt + nt - 1] = pick(u_prev, threadIdx.x);
  // ---- tau_k = <tgt|psi_hat_k(T)> ----
  for (int k = w; k < M; k += nteam) {
    const double inv = 1.0 / sqrt(gmem(meta_g)[k].nrm2);
    double tr = 0.0, ti = 0.0;
#pragma unroll
    for (int m = 0; m < R; ++m) {
      const int row = tm.gl + kL * m;
      const cx<real> q = gld(psi_g, static_cast<size_t>(k) * kRows + row);
      const double px = q.x * inv, py = q.y * inv;
      const double gx = gmem(a.tgt)[2 * row], gy = gmem(a.tgt)[2 * row + 1];
      tr = fma(gx, px, fma(gy, py, tr));
      ti = fma(gx, py, fma(-gy, px, ti));
    }
    tm.sum2(tr, ti);
    if (tm.leader()) {
      gmem(a.tau_out)[2 * k] = tr;
      gmem(a.tau_out)[2 * k + 1] = ti;
    }
  }
}

template <typename real, int G>
__global__ __launch_bounds__(kWave *G) void k_batch_wide_krotov(BatchArgs b) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double s_upd[kMaxCtrl];
  __shared__ int s_abort;
  __shared__ double team_red[8 * G];
  const Team<G> tm = make_team<G>(team_red);
  if (threadIdx.x == 0) {
    s_abort = 0;
    atomicMin(b.t_begin, static_cast<unsigned long long>(wall_clock64()));
  }
  const int i = __builtin_amdgcn_readfirstlane(b.wblock_inst[blockIdx.x]);
  const BatchInstance &I = b.inst[i];
  const int lb = blockIdx.x - I.block0;
  const uint64_t it = *b.iteration;
  switch (I.variant) {
#define TK_CASE(idx, R, WS, NC, GG)                                                          \
  case idx:                                                                                  \
    if constexpr (GG == G)                                                                   \
      wide_krotov_instance<real, R, WS, NC, G>(b, I, lb, it, smem_raw, s_upd, &s_abort, tm); \
    break;
    TK_BATCH_WIDE_SHAPES(TK_CASE)
#undef TK_CASE
    default:
      break;
  }
  __syncthreads();
  if (threadIdx.x == 0) atomicMax(&b.t_end[i], static_cast<unsigned long long>(wall_clock64()));
}

// ---- bookkeeping kernels ------------------------------------------------------------
// Per-trajectory slots of every instance <- sentinel (one block per instance).
__global__ __launch_bounds__(256) void k_batch_fill(BatchArgs b) {
  const BatchInstance &I = b.inst[blockIdx.x];
  const size_t n = static_cast<size_t>(I.fw.nt) * I.fw.M * I.ncx;
  for (size_t q = threadIdx.x; q < n; q += blockDim.x) I.tslots[q] = kSlotEmpty;
}

// J_T = 1 - (1/M) sum_k |tau_k|^2 of every instance (one block each, fixed
// order), kept in the history ring at the current iteration.
__global__ __launch_bounds__(256) void k_batch_functional(BatchArgs b) {
  __shared__ double part[256];
  const BatchInstance &I = b.inst[blockIdx.x];
  const double *tau = I.fw.tau_out;
  const int M = I.fw.M;
  double s = 0.0;
  for (int k = threadIdx.x; k < M; k += 256)
    s = fma(tau[2 * k], tau[2 * k], fma(tau[2 * k + 1], tau[2 * k + 1], s));
  part[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (static_cast<int>(threadIdx.x) < off) part[threadIdx.x] += part[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    b.J_hist[static_cast<size_t>(blockIdx.x) * kBatchHistory + (*b.iteration % kBatchHistory)] =
        1.0 - part[0] / static_cast<double>(M);
}

// End of an iteration: the updated pulses become the current ones (one block
// per instance); block 0 advances the iteration counter (read only by the next
// launches).
__global__ __launch_bounds__(256) void k_batch_finish(BatchArgs b, int copy_pulses) {
  const BatchInstance &I = b.inst[blockIdx.x];
  if (copy_pulses) {
    const size_t n = static_cast<size_t>(I.fw.n_ctrl) * I.fw.nt;
    double *u = const_cast<double *>(I.fw.u_old);
    for (size_t q = threadIdx.x; q < n; q += blockDim.x) u[q] = I.fw.u_new[q];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *b.iteration += 1;
}

}  // namespace

int batch_shape_index(int precision, int R, int wsc, int NC, int G) {
#define TK_CASE(idx, r, ws, nc) \
  if (G == 1 && R == r && wsc == (ws) && NC == nc) return idx;
  TK_BATCH_SHAPES(TK_CASE)
#undef TK_CASE
#define TK_CASE(idx, r, ws, nc, g) \
  if (G == g && R == r && wsc == (ws) && NC == nc) return idx;
  TK_BATCH_WIDE_SHAPES(TK_CASE)
#undef TK_CASE
  return -1;
}

BatchKernels batch_kernels(int precision) {
  BatchKernels k;
#define TK_CASE(idx, R, WS, NC)                                                               \
  if (precision == TK_FP64) {                                                                 \
    k.pass_fw[idx] = reinterpret_cast<const void *>(&k_batch_pass<double, 0, idx>);           \
    k.pass_bw[idx] = reinterpret_cast<const void *>(&k_batch_pass<double, 1, idx>);           \
    k.krotov[idx] = reinterpret_cast<const void *>(&k_batch_krotov<double, idx>);             \
  } else {                                                                                    \
    k.pass_fw[idx] = reinterpret_cast<const void *>(&k_batch_pass<float, 0, idx>);            \
    k.pass_bw[idx] = reinterpret_cast<const void *>(&k_batch_pass<float, 1, idx>);            \
    k.krotov[idx] = reinterpret_cast<const void *>(&k_batch_krotov<float, idx>);              \
  }
  TK_BATCH_SHAPES(TK_CASE)
#undef TK_CASE
  if (precision == TK_FP64) {
    k.wpass_fw = reinterpret_cast<const void *>(&k_batch_wide_pass<double, 0, 2>);
    k.wpass_bw = reinterpret_cast<const void *>(&k_batch_wide_pass<double, 1, 2>);
    k.wkrotov = reinterpret_cast<const void *>(&k_batch_wide_krotov<double, 2>);
    k.wpass_fw8 = reinterpret_cast<const void *>(&k_batch_wide_pass<double, 0, 8>);
    k.wpass_bw8 = reinterpret_cast<const void *>(&k_batch_wide_pass<double, 1, 8>);
    k.wkrotov8 = reinterpret_cast<const void *>(&k_batch_wide_krotov<double, 8>);
  } else {
    k.wpass_fw = reinterpret_cast<const void *>(&k_batch_wide_pass<float, 0, 2>);
    k.wpass_bw = reinterpret_cast<const void *>(&k_batch_wide_pass<float, 1, 2>);
    k.wkrotov = reinterpret_cast<const void *>(&k_batch_wide_krotov<float, 2>);
    k.wpass_fw8 = reinterpret_cast<const void *>(&k_batch_wide_pass<float, 0, 8>);
    k.wpass_bw8 = reinterpret_cast<const void *>(&k_batch_wide_pass<float, 1, 8>);
    k.wkrotov8 = reinterpret_cast<const void *>(&k_batch_wide_krotov<float, 8>);
  }
  k.fill = reinterpret_cast<const void *>(&k_batch_fill);
  k.functional = reinterpret_cast<const void *>(&k_batch_functional);
  k.finish = reinterpret_cast<const void *>(&k_batch_finish);
  return k;
}

}  // namespace tk
