// Post-processing of optimised pulses: the noise measure of Sec. 3.4,
//   nu_i = int_0^T |Omega_i(t) - Omega_i^smooth(t)| dt,
// with Omega^smooth from a Savitzky-Golay five-point cubic filter.  Pulses are
// piecewise constant on nt intervals, so the integral is dt sum_j |u_ij - s_ij|.
// The filter value at a sample is the least-squares cubic of a five-sample
// window evaluated at that sample: the centred window in the interior, the
// first (last) five samples for the first (last) two.  Its weights are the
// rows of the hat matrix V (V^T V)^-1 V^T of the 5 x 4 Vandermonde matrix V,
// formed once on the host in FP64.
#include <hip/hip_runtime.h>

#include <cmath>

#include "tk_internal.h"

namespace tk {
namespace {

struct SgWeights {
  double w[5][5];  // w[p][q]: weight of window sample q for the value at position p
};

constexpr int kNoiseThreads = 256;

// one block per control: each thread sums |u_j - s_j| over its samples, then a
// fixed-order tree over the block
__global__ __launch_bounds__(kNoiseThreads) void k_pulse_noise(const double *u, int nt,
                                                               double dt, SgWeights W,
                                                               double *nu) {
  __shared__ double part[kNoiseThreads];
  const double *row = u + static_cast<size_t>(blockIdx.x) * nt;
  double acc = 0.0;
  for (int j = threadIdx.x; j < nt; j += kNoiseThreads) {
    const int s = j < 2 ? 0 : (j > nt - 3 ? nt - 5 : j - 2);  // window start
    const int p = j - s;                                         // position in the window
    double sm = 0.0;
#pragma unroll
    for (int q = 0; q < 5; ++q) sm = fma(W.w[p][q], row[s + q], sm);
    acc += fabs(row[j] - sm);
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int off = kNoiseThreads / 2; off > 0; off >>= 1) {
    if (static_cast<int>(threadIdx.x) < off) part[threadIdx.x] += part[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) nu[blockIdx.x] = dt * part[0];
}

// hat matrix of the least-squares cubic through positions -2 .. 2
SgWeights sg_weights() {
  double V[5][4];
  for (int p = 0; p < 5; ++p)
    for (int a = 0; a < 4; ++a) V[p][a] = std::pow(static_cast<double>(p - 2), a);
  // G = V^T V, then its inverse by Gauss-Jordan elimination with partial pivoting
  double G[4][8] = {};
  for (int a = 0; a < 4; ++a) {
    for (int b = 0; b < 4; ++b)
      for (int p = 0; p < 5; ++p) G[a][b] += V[p][a] * V[p][b];
    G[a][4 + a] = 1.0;
  }
  for (int c = 0; c < 4; ++c) {
    int piv = c;
    for (int r = c + 1; r < 4; ++r)
      if (std::fabs(G[r][c]) > std::fabs(G[piv][c])) piv = r;
    for (int k = 0; k < 8; ++k) std::swap(G[c][k], G[piv][k]);
    const double inv = 1.0 / G[c][c];
    for (int k = 0; k < 8; ++k) G[c][k] *= inv;
    for (int r = 0; r < 4; ++r) {
      if (r == c) continue;
      const double f = G[r][c];
      for (int k = 0; k < 8; ++k) G[r][k] -= f * G[c][k];
    }
  }
  SgWeights W;
  for (int p = 0; p < 5; ++p)
    for (int q = 0; q < 5; ++q) {
      double s = 0.0;
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) s += V[p][a] * G[a][4 + b] * V[q][b];
      W.w[p][q] = s;
    }
  return W;
}

}  // namespace

hipError_t launch_pulse_noise(const double *u_dev, int n_ctrl, int nt, double dt, double *nu_dev,
                              hipStream_t stream) {
  static const SgWeights W = sg_weights();
  SgWeights w = W;
  const double *up = u_dev;
  double *np_ = nu_dev;
  void *args[] = {&up, &nt, &dt, &w, &np_};
  return hipLaunchKernel(reinterpret_cast<const void *>(&k_pulse_noise), dim3(n_ctrl),
                         dim3(kNoiseThreads), args, 0, stream);
}

}  // namespace tk
