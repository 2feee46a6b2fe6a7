// Cross-trajectory Krotov update (Sec. 2.3, eq. cross_traj_update):
//   Delta u_i(t_j) = S_ij / (M^2 lambda_i)
//                    sum_{k,k'} Im[<xi_k|H_i|Psi_k'> <Psi_k'|xi_k>]   (at t_j)
// with xi_k the normalised backward trajectories started from Psi_tgt.  The
// double sum over trajectories is regrouped around the Gram matrix of the
// backward states,
//   P_j = (1/M) sum_k |xi_k(t_j)><xi_k(t_j)|     (d x d, Hermitian),
//   sum_{k,k'} ... = M sum_k' Im <P_j Psi_k'| H_i |Psi_k'>,
// so that every forward trajectory contributes the share of the independent
// update with the costate chi'_k' = P_j Psi_hat_k' (work d^2 per trajectory
// instead of M d).
//
// k_cross_gram forms all P_j after the backward pass: per step a d x d
// product with the trajectory index as the inner dimension, on the FP64
// matrix cores (v_mfma_f64_16x16x4f64).  A block of four waves owns a 32 x 32
// piece of one P_j (each wave a 16 x 16 tile) and streams the backward states
// through LDS sixteen trajectories at a time; the blocks of one step are
// placed on one XCD (blocks are dealt to the eight XCDs round-robin), so the
// step's states are read from HBM about once and served to its blocks from
// that XCD's L2.  P_j is stored column-major with the rows padded to the
// forward kernel's 64 R rows: P[j][c][r].
//
// k_krotov_cross is the sequential pass of k_krotov (same exchange, update,
// step and jump handling) with the costate formed on the fly: after a step,
// the waves of a block share their normalised states through LDS, wave w
// multiplies the w-th quarter of P_j's columns into all of them (each column
// read once per block), and each trajectory sums the quarters in wave order.
#include <hip/hip_runtime.h>

#include "tk_device.h"
#include "tk_internal.h"

namespace tk {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kGramK = 16;  // trajectories staged per LDS round

template <typename real>
__global__ __launch_bounds__(256) void k_cross_gram(const cx<real> *chi, int nt, int M, int d,
                                                    int Rp, int nrb, int ncb, double invM,
                                                    cx<double> *P) {
  __shared__ double Ar[kGramK][32], Ai[kGramK][32], Br[kGramK][32], Bi[kGramK][32];
  const int S = nrb * ncb;
  const int b = blockIdx.x;
  const int xcd = b % 8, slot = b / 8;
  const int j = 8 * (slot / S) + xcd;  // every block of step j runs on XCD j % 8
  const int s = slot % S;
  if (j >= nt) return;  // uniform across the block
  const int r0 = 32 * (s / ncb), c0 = 32 * (s % ncb);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int tr = w >> 1, tc = w & 1;
  const cx<real> *X = chi + static_cast<size_t>(j) * M * d;
  v4d acc_re = {0.0, 0.0, 0.0, 0.0}, acc_im = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < M; k0 += kGramK) {
    // stage 16 trajectories x 32 rows (A) and x 32 columns (B); zero outside
    for (int e = threadIdx.x; e < kGramK * 32; e += 256) {
      const int kk = e / 32, q = e % 32;
      const int k = k0 + kk;
      double ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0;
      if (k < M) {
        if (r0 + q < d) {
          const cx<real> x = X[static_cast<size_t>(k) * d + r0 + q];
          ar = x.x;
          ai = x.y;
        }
        if (c0 + q < d) {
          const cx<real> x = X[static_cast<size_t>(k) * d + c0 + q];
          br = x.x;
          bi = x.y;
        }
      }
      Ar[kk][q] = ar;
      Ai[kk][q] = ai;
      Br[kk][q] = br;
      Bi[kk][q] = bi;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < kGramK / 4; ++ks) {
      const int kk = 4 * ks + (lane >> 4), i = lane & 15;
      const double ar = Ar[kk][16 * tr + i], ai = Ai[kk][16 * tr + i];
      const double br = Br[kk][16 * tc + i], bi = Bi[kk][16 * tc + i];
      // P~[r][c] = sum_k x_k[r] conj(x_k[c])
      acc_re = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, br, acc_re, 0, 0, 0);
      acc_re = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, bi, acc_re, 0, 0, 0);
      acc_im = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, br, acc_im, 0, 0, 0);
      acc_im = __builtin_amdgcn_mfma_f64_16x16x4f64(-ar, bi, acc_im, 0, 0, 0);
    }
    __syncthreads();
  }
  // result layout of the 16 x 16 x 4 FP64 product: lane l, register v holds
  // row (l / 16) + 4 v, column l % 16 of the tile
  const int col = c0 + 16 * tc + (lane & 15);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = r0 + 16 * tr + (lane >> 4) + 4 * v;
    if (row < Rp && col < d)
      P[(static_cast<size_t>(j) * d + col) * Rp + row] = cx<double>{acc_re[v] * invM,
                                                                  acc_im[v] * invM};
  }
}

// Cross-trajectory costate of every team's trajectory at step j:
// chi'_q = P_j psi_hat_q.  All waves of the block take part (uniform call).
// xhat [teams][Rp] and part [waves][teams][Rp] are LDS (FP64 complex).
template <typename real, int R>
__device__ __forceinline__ void cross_costate(const PassArgs &a, int j, const cx<real> (&psi)[R],
                                              double inv, bool active, int team, int tpb,
                                              cx<double> *xhat, cx<double> *part,
                                              cx<double> (&chi)[R]) {
  constexpr int kL = kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int Rp = R * kL;
#pragma unroll
  for (int m = 0; m < R; ++m)
    xhat[team * Rp + lane + kL * m] =
        active ? cx<double>{psi[m].x * inv, psi[m].y * inv} : cx<double>{0.0, 0.0};
  block_sync_lds();
  // this wave's columns: a contiguous quarter (or less) of 0 .. d-1
  const int per = (a.d + tpb - 1) / tpb;
  const int c_lo = team * per, c_hi = min(a.d, c_lo + per);
  cx<double> acc[kWavesPerBlock][R];
#pragma unroll
  for (int q = 0; q < kWavesPerBlock; ++q)
#pragma unroll
    for (int m = 0; m < R; ++m) acc[q][m] = cx<double>{0.0, 0.0};
  const cx<double> *Pj = static_cast<const cx<double> *>(a.pmat) + static_cast<size_t>(j) * a.d * Rp;
  // columns in groups of kCols: the group's loads are all issued before its
  // multiply-adds, so their latencies overlap (a column slice is read from L2)
  constexpr int kCols = R >= 4 ? 2 : 8 / R;
  int c = c_lo;
  for (; c + kCols <= c_hi; c += kCols) {
    cx<double> pc[kCols][R];
#pragma unroll
    for (int u = 0; u < kCols; ++u)
#pragma unroll
      for (int m = 0; m < R; ++m) pc[u][m] = gld(Pj, static_cast<size_t>(c + u) * Rp + lane + kL * m);
#pragma unroll
    for (int u = 0; u < kCols; ++u)
#pragma unroll
      for (int q = 0; q < kWavesPerBlock; ++q) {
        if (q < tpb) {
          const cx<double> x = xhat[q * Rp + c + u];
#pragma unroll
          for (int m = 0; m < R; ++m) cfma(acc[q][m], pc[u][m], x);
        }
      }
  }
  for (; c < c_hi; ++c) {
    cx<double> pc[R];
#pragma unroll
    for (int m = 0; m < R; ++m) pc[m] = gld(Pj, static_cast<size_t>(c) * Rp + lane + kL * m);
#pragma unroll
    for (int q = 0; q < kWavesPerBlock; ++q) {
      if (q < tpb) {
        const cx<double> x = xhat[q * Rp + c];
#pragma unroll
        for (int m = 0; m < R; ++m) cfma(acc[q][m], pc[m], x);
      }
    }
  }
#pragma unroll
  for (int q = 0; q < kWavesPerBlock; ++q)
    if (q < tpb)
#pragma unroll
      for (int m = 0; m < R; ++m) part[(team * tpb + q) * Rp + lane + kL * m] = acc[q][m];
  block_sync_lds();
#pragma unroll
  for (int m = 0; m < R; ++m) {
    cx<double> s{0.0, 0.0};
    for (int w = 0; w < tpb; ++w) {
      const cx<double> v = part[(w * tpb + team) * Rp + lane + kL * m];
      s.x += v.x;
      s.y += v.y;
    }
    chi[m] = s;
  }
}

// Share of Im <chi'|H_i|psi_hat> (FP64 costate) for every control slot c;
// the state is in term vector 0 where the gathers are bound, inv = 1/||psi||.
template <typename real, int R, int WS, int NC>
__device__ __forceinline__ void cross_share(const LaneOp<real, R, WS, NC, 1> &op,
                                            const cx<double> (&ch)[R], double inv, double *pc) {
#pragma unroll
  for (int m = 0; m < R; ++m) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const cx<real> q = op.cval_at(c, m);
      const cx<real> b = op.cp[c][m][0];
      const double hx = static_cast<double>(q.x) * b.x - static_cast<double>(q.y) * b.y;
      const double hy = static_cast<double>(q.x) * b.y + static_cast<double>(q.y) * b.x;
      pc[c] = fma(inv * ch[m].x, hy, pc[c]);
      pc[c] = fma(-inv * ch[m].y, hx, pc[c]);
    }
  }
}

// ---- sequential pass with the cross-trajectory update (cooperative launch) ----
// One-wave teams only.  Every wave runs the same number of trajectory slots
// (slots past M stay idle but join the block's barriers).
template <typename real, int R, int WS, int NC>
__global__ __launch_bounds__(kWave *kWavesPerBlock) void k_krotov_cross(PassArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  constexpr int NCX = NC > 0 ? NC : 1;
  constexpr int kL = kWave;
  constexpr int Rp = R * kL;
  __shared__ double wpart[kWavesPerBlock][NCX];
  __shared__ double s_upd[NCX];
  __shared__ int s_abort;
  __shared__ double team_red[4];
  const int lane = threadIdx.x & (kWave - 1);
  const int team = __builtin_amdgcn_readfirstlane(threadIdx.x / kL);
  const int tpb = blockDim.x / kL;
  const Team<1> tm = make_team<1>(team_red);
  const int Tw = a.traj_per_wave;
  const int tglob = blockIdx.x * tpb + team;
  const size_t tb = terms_bytes<real, R, 1>(a.kbuf);
  const size_t team_bytes = (tb + static_cast<size_t>(Tw) * R * kL * sizeof(cx<real>) +
                             static_cast<size_t>(Tw) * sizeof(TrajMeta) + 15) / 16 * 16;
  LaneOp<real, R, WS, NC, 1> op;
  const Terms<real, R, 1> T = block_setup<real, R, WS, NC, 1>(a, smem_raw, team, tm, team_bytes, op);
  cx<real> *states = reinterpret_cast<cx<real> *>(reinterpret_cast<unsigned char *>(T.base) + tb);
  TrajMeta *meta = reinterpret_cast<TrajMeta *>(states + static_cast<size_t>(Tw) * R * kL);
  // cross area after every team's share: xhat [tpb][Rp], part [tpb][tpb][Rp]
  const size_t cval_bytes = sizeof(cx<real>) * NCX * R * kL;
  cx<double> *xhat = reinterpret_cast<cx<double> *>(smem_raw + cval_bytes + tpb * team_bytes);
  cx<double> *part = xhat + static_cast<size_t>(tpb) * Rp;
  cx<real> *v = T[0];
  const cx<real> *start = static_cast<const cx<real> *>(a.psi_start);
  if (threadIdx.x == 0) s_abort = 0;
  if (threadIdx.x < NCX) s_upd[threadIdx.x] = 0.0;

  double pc[NCX];
#pragma unroll
  for (int c = 0; c < NCX; ++c) pc[c] = 0.0;
  for (int t = 0; t < Tw; ++t) {
    const int k = tglob * Tw + t;
    const bool active = k < a.M;
    cx<real> p[R];
#pragma unroll
    for (int m = 0; m < R; ++m) p[m] = start[lane + kL * m];
    store_lds(states + t * R * kL, p, tm);
    const double n = norm2(p, tm);
    TrajMeta st;
    st.nrm2 = n;
    st.ordinal = 0;
    st.pad = 0;
    st.r = 0.0;
    st.x = 0.0;
    if (active) make_stream(a, k, 0).draw(0, st);
    if (tm.leader()) meta[t] = st;
    cx<double> ch[R];
    const double inv = 1.0 / sqrt(n);
    cross_costate<real, R>(a, 0, p, inv, active, team, tpb, xhat, part, ch);
    if (active) {
      store_lds(v, p, tm);
      tm.sync();
      cross_share<real, R, WS, NC>(op, ch, inv, pc);
      tm.sync();
    }
    block_sync_lds();  // xhat / part are reused by the next slot
  }

  double inv_lm[NCX];
#pragma unroll
  for (int i = 0; i < NCX; ++i) inv_lm[i] = 1.0 / (a.lam[i] * a.M);
  double u_prev[NCX];
  OrderHint khint;
  for (int j = 0; j < a.nt; ++j) {
    double uo[NCX], so[NCX];
#pragma unroll
    for (int i = 0; i < NCX; ++i) {
      const size_t ij = static_cast<size_t>(i) * a.nt + j;
      uo[i] = a.u_old[ij];
      so[i] = a.S[ij];
    }
    tm.template sum_n<NC>(pc);
    if (tm.leader())
#pragma unroll
      for (int c = 0; c < NC; ++c) wpart[team][c] = pc[c];
    block_sync_lds();
    if (threadIdx.x < NCX) {
      const int i = threadIdx.x;
      double s = 0.0;
      for (int w = 0; w < tpb; ++w)
        for (int c = i * a.wc; c < (i + 1) * a.wc && c < NC; ++c) s += wpart[w][c];
      __hip_atomic_store(&a.slots[(static_cast<size_t>(j) * kMaxBlocks + blockIdx.x) * NCX + i],
                         __double_as_longlong(s), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (blockIdx.x == 0 && j > 0) a.u_new[static_cast<size_t>(i) * a.nt + j - 1] = pick(u_prev, i);
    }
    if (team == 0 && a.n_ctrl > 0) {
      const unsigned long long *row = a.slots + static_cast<size_t>(j) * kMaxBlocks * NCX;
      double acc[NCX];
      long long spins = 0;
      bool abort = false;
      for (;;) {
        unsigned long long bits[kPollPerLane][NCX];
        poll_slots<NCX>(row, lane, bits);
        if (slots_complete<NCX>(bits, acc)) break;
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
    if (s_abort) return;
    double uj[NCX];
#pragma unroll
    for (int i = 0; i < NCX; ++i) {
      uj[i] = uo[i] + so[i] * inv_lm[i] * s_upd[i];
      u_prev[i] = uj[i];
    }
    op.set_pulses(uj, a.wc);
    const StepPlan p = plan_step(a, uj, khint);
#pragma unroll
    for (int c = 0; c < NCX; ++c) pc[c] = 0.0;
    for (int t = 0; t < Tw; ++t) {
      const int k = tglob * Tw + t;
      const bool active = k < a.M;
      cx<real> *sv = states + t * R * kL;
      cx<real> psi[R];
      load_lds(sv, psi, tm);
      TrajMeta st = meta[t];
      if (active) {
        const Stream rng = make_stream(a, k, 0);
        advance_step<real, R, WS, NC, 1, 0, true>(op, a, T, psi, st, rng, j, p, k, tm);
        tm.sync();
        store_lds(sv, psi, tm);
        if (tm.leader()) meta[t] = st;
      }
      if (j + 1 < a.nt) {
        cx<double> ch[R];
        const double inv = 1.0 / sqrt(st.nrm2);
        cross_costate<real, R>(a, j + 1, psi, inv, active, team, tpb, xhat, part, ch);
        if (active) {
          tm.sync();
          store_lds(v, psi, tm);
          tm.sync();
          cross_share<real, R, WS, NC>(op, ch, inv, pc);
        }
        block_sync_lds();
      }
      tm.sync();
    }
  }
  if (blockIdx.x == 0 && threadIdx.x < NCX)
    a.u_new[static_cast<size_t>(threadIdx.x) * a.nt + a.nt - 1] = pick(u_prev, threadIdx.x);
  cx<real> *psiT = static_cast<cx<real> *>(a.psiT);
  for (int t = 0; t < Tw; ++t) {
    const int k = tglob * Tw + t;
    if (k >= a.M) break;
    const cx<real> *sv = states + t * R * kL;
    const double inv = 1.0 / sqrt(meta[t].nrm2);
    double tr = 0.0, ti = 0.0;
#pragma unroll
    for (int m = 0; m < R; ++m) {
      const int row = lane + kL * m;
      const cx<real> q = sv[row];
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

}  // namespace

const void *cross_kernel(int precision, int R, int WS, int NC, int G) {
  if (G != 1) return nullptr;
#define TK_CROSS(real, r, ws, nc) \
  if (R == r && WS == ws && NC == nc) return reinterpret_cast<const void *>(&k_krotov_cross<real, r, ws, nc>)
  if (precision == TK_FP64) {
    TK_CROSS(double, 1, 4, 2);
    TK_CROSS(double, 2, 4, 2);
    TK_CROSS(double, 4, 6, 3);
    TK_CROSS(double, 4, 8, 4);
    TK_CROSS(double, 2, ws_code(3, 1, true, 1), 2);
  } else {
    TK_CROSS(float, 1, 4, 2);
    TK_CROSS(float, 2, 4, 2);
    TK_CROSS(float, 4, 6, 3);
    TK_CROSS(float, 4, 8, 4);
    TK_CROSS(float, 2, ws_code(3, 1, true, 1), 2);
    TK_CROSS(float, 4, ws_code(5, 3, true, 2), 3);
  }
#undef TK_CROSS
  return nullptr;
}

const void *cross_gram_kernel(int precision) {
  return precision == TK_FP64 ? reinterpret_cast<const void *>(&k_cross_gram<double>)
                              : reinterpret_cast<const void *>(&k_cross_gram<float>);
}

size_t cross_lds_bytes(const Variant &v, int teams, int kbuf, int traj_per_wave) {
  const size_t rows = static_cast<size_t>(v.R) * kWave;
  return block_lds_bytes(v, teams, kbuf, traj_per_wave) +
         static_cast<size_t>(teams + teams * teams) * rows * 16;
}

}  // namespace tk
