// One step propagator exp(-i H_eff tau) ~ sum_{n<=K} (-i tau H_eff)^n / n!
// applied to M states in two ways, to decide on evidence whether the dense
// operator on the matrix cores beats the sparse per-lane product of the passes
// (the paper's fundamental operation is the matrix-vector product, Sec. 2.3):
//
// * k_step_sparse: the passes' own series (taylor_pingpong over the packed
//   per-lane slots of H_eff, one wave per trajectory).
// * k_step_dense: H_eff as a dense Dp x Dp matrix (Dp = d rounded up to 16) and
//   the states of 16 NT trajectories as the columns of a Dp x 16 NT block in
//   LDS; every term is a complex product on the matrix cores
//   (v_mfma_f64_16x16x4f64 / v_mfma_f32_16x16x4f32, four real products per
//   complex one): wave w computes the 16-row bands w, w + 4, ... for all NT
//   column tiles, reading its band of H_eff from L2 once per term.
//
// Both write the same result (up to rounding); the host times them.
#include <hip/hip_runtime.h>

#include "tk_device.h"
#include "tk_internal.h"

namespace tk {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename real>
struct Mfma;
// Operands of both products: lane l gives A[l % 16][l / 16] and B[l / 16][l % 16].
// Results differ: FP64 leaves D[(l / 16) + 4 v][l % 16] in register v, FP32
// D[4 (l / 16) + v][l % 16].
template <>
struct Mfma<double> {
  using acc = v4d;
  static __device__ __forceinline__ acc fma(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <>
struct Mfma<float> {
  using acc = v4f;
  static __device__ __forceinline__ acc fma(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

constexpr int kMaxBands = 4;  // 16-row bands per wave: Dp <= 256

template <typename real, int NT>
__global__ __launch_bounds__(256) void k_step_dense(const cx<real> *H, int d, int Dp, int M, int K,
                                                    double tau, const cx<real> *x, cx<real> *y) {
  using acc_t = typename Mfma<real>::acc;
  constexpr int W = 16 * NT;  // trajectories of the block
  extern __shared__ __align__(16) unsigned char smem_raw[];
  real *Xr[2], *Xi[2];
  Xr[0] = reinterpret_cast<real *>(smem_raw);
  Xi[0] = Xr[0] + Dp * W;
  Xr[1] = Xi[0] + Dp * W;
  Xi[1] = Xr[1] + Dp * W;
  const int k0 = blockIdx.x * W;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nb = Dp / 16;
  for (int e = threadIdx.x; e < Dp * W; e += 256) {
    const int row = e / W, col = e % W;
    const int k = k0 + col;
    cx<real> v{0, 0};
    if (row < d && k < M) v = x[static_cast<size_t>(k) * d + row];
    Xr[0][e] = v.x;
    Xi[0][e] = v.y;
  }
  __syncthreads();
  // running sum of the terms at this lane's output positions (starts with x)
  real Sr[kMaxBands][NT][4], Si[kMaxBands][NT][4];
#pragma unroll
  for (int q = 0; q < kMaxBands; ++q) {
    const int b = w + 4 * q;
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * b + Mfma<real>::row(lane, v), col = 16 * t + (lane & 15);
        Sr[q][t][v] = b < nb ? Xr[0][row * W + col] : real(0);
        Si[q][t][v] = b < nb ? Xi[0][row * W + col] : real(0);
      }
  }
  const int i = lane & 15, kq = lane >> 4;
  for (int n = 1; n <= K; ++n) {
    const real *cr = Xr[(n - 1) & 1], *ci = Xi[(n - 1) & 1];
    real *nr = Xr[n & 1], *ni = Xi[n & 1];
    const real c = static_cast<real>(tau / n);
#pragma unroll
    for (int q = 0; q < kMaxBands; ++q) {
      const int b = w + 4 * q;
      if (b >= nb) break;  // uniform across the wave
      acc_t ar[NT], ai[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        ar[t] = acc_t{0, 0, 0, 0};
        ai[t] = acc_t{0, 0, 0, 0};
      }
      const cx<real> *hrow = H + static_cast<size_t>(16 * b + i) * Dp;
      for (int kk0 = 0; kk0 < Dp; kk0 += 4) {
        const int kk = kk0 + kq;
        const cx<real> h = hrow[kk];  // A[i][k] = H[16 b + i][kk]
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const real xr = cr[kk * W + 16 * t + i], xi = ci[kk * W + 16 * t + i];  // B[k][j]
          ar[t] = Mfma<real>::fma(h.x, xr, ar[t]);
          ar[t] = Mfma<real>::fma(-h.y, xi, ar[t]);
          ai[t] = Mfma<real>::fma(h.x, xi, ai[t]);
          ai[t] = Mfma<real>::fma(h.y, xr, ai[t]);
        }
      }
      // t_n = (-i tau / n) H t_{n-1}
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = 16 * b + Mfma<real>::row(lane, v), col = 16 * t + (lane & 15);
          const real tr = c * ai[t][v], ti = -c * ar[t][v];
          nr[row * W + col] = tr;
          ni[row * W + col] = ti;
          Sr[q][t][v] += tr;
          Si[q][t][v] += ti;
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < kMaxBands; ++q) {
    const int b = w + 4 * q;
    if (b >= nb) break;
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * b + Mfma<real>::row(lane, v), k = k0 + 16 * t + (lane & 15);
        if (row < d && k < M) y[static_cast<size_t>(k) * d + row] = cx<real>{Sr[q][t][v], Si[q][t][v]};
      }
  }
}

// The passes' series on the packed slots (pulses of step 0), one wave per
// trajectory: y_k = sum_{n<=K} (-i tau H_eff)^n / n! x_k.
template <typename real, int R, int WS, int NC>
__global__ __launch_bounds__(kWave *kWavesPerBlock) void k_step_sparse(PassArgs a, int K,
                                                                        const cx<real> *x,
                                                                        cx<real> *y) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double team_red[4];
  constexpr int NCX = NC > 0 ? NC : 1;
  constexpr int kL = kWave;
  const int team = __builtin_amdgcn_readfirstlane(threadIdx.x / kL);
  const int tpb = blockDim.x / kL;
  const Team<1> tm = make_team<1>(team_red);
  LaneOp<real, R, WS, NC, 1> op;
  const Terms<real, R, 1> T =
      block_setup<real, R, WS, NC, 1>(a, smem_raw, team, tm, terms_bytes<real, R, 1>(a.kbuf), op);
  double uj[NCX];
#pragma unroll
  for (int q = 0; q < NCX; ++q) uj[q] = a.u[static_cast<size_t>(q) * a.nt];
  op.set_pulses(uj, a.wc);
  for (int k = blockIdx.x * tpb + team; k < a.M; k += gridDim.x * tpb) {
    cx<real> p[R], out[R];
#pragma unroll
    for (int m = 0; m < R; ++m) {
      const int row = tm.gl + kL * m;
      p[m] = row < a.d ? x[static_cast<size_t>(k) * a.d + row] : cx<real>{0, 0};
    }
    tm.sync();
    taylor_pingpong<real, R, WS, NC, 1, -1>(op, a, T, p, out, a.dt, K, tm);
#pragma unroll
    for (int m = 0; m < R; ++m) {
      const int row = tm.gl + kL * m;
      if (row < a.d) y[static_cast<size_t>(k) * a.d + row] = out[m];
    }
  }
}

}  // namespace

const void *dense_step_kernel(int precision, int NT) {
  if (precision == TK_FP64) {
    if (NT == 1) return reinterpret_cast<const void *>(&k_step_dense<double, 1>);
    if (NT == 2) return reinterpret_cast<const void *>(&k_step_dense<double, 2>);
    if (NT == 4) return reinterpret_cast<const void *>(&k_step_dense<double, 4>);
  } else {
    if (NT == 1) return reinterpret_cast<const void *>(&k_step_dense<float, 1>);
    if (NT == 2) return reinterpret_cast<const void *>(&k_step_dense<float, 2>);
    if (NT == 4) return reinterpret_cast<const void *>(&k_step_dense<float, 4>);
  }
  return nullptr;
}

const void *sparse_step_kernel(int precision, int R, int WS, int NC, int G) {
  if (G != 1) return nullptr;
#define TK_SPARSE(real, r, ws, nc) \
  if (R == r && WS == ws && NC == nc) return reinterpret_cast<const void *>(&k_step_sparse<real, r, ws, nc>)
  if (precision == TK_FP64) {
    TK_SPARSE(double, 1, 4, 2);
    TK_SPARSE(double, 2, 4, 2);
    TK_SPARSE(double, 4, 6, 3);
    TK_SPARSE(double, 4, 8, 4);
    TK_SPARSE(double, 2, ws_code(3, 1, true, 1), 2);
  } else {
    TK_SPARSE(float, 1, 4, 2);
    TK_SPARSE(float, 2, 4, 2);
    TK_SPARSE(float, 4, 6, 3);
    TK_SPARSE(float, 4, 8, 4);
    TK_SPARSE(float, 2, ws_code(3, 1, true, 1), 2);
    TK_SPARSE(float, 4, ws_code(5, 3, true, 2), 3);
  }
#undef TK_SPARSE
  return nullptr;
}

}  // namespace tk
