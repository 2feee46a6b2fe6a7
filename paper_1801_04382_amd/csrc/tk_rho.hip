// Density-matrix (Liouville-space) optimisation of Sec. 2.2, FP64:
//   forward   d rho/dt = L(rho) = -i (H_eff rho - rho H_eff^+) + sum_l L_l rho L_l^+
//   backward  d P/dt  = -L^+(P),  L^+(P) = +i (H_eff^+ P - P H_eff) + sum_l L_l^+ P L_l,
//             from P(T) = |tgt><tgt| (eqs. bwprop, krotov_boundary)
//   functional J_T = 1 - <tgt|rho(T)|tgt> (eq. functional)
//   update    u_ij = u_ij + S_ij / lambda_i Im <<P(t_j)| [H_i, rho(t_j)]>> (eq. krotovupdate,
//             sequential: rho carries the pulses already updated)
// with H_eff = H0 + sum_i u_i H_i - (i/2) sum_l L_l^+ L_l.
//
// Both generators have the form G(Q) = s i (X - X^+) + sum_l J_l (J_l Q)^+ on
// Hermitian Q, with X = B Q: forward s = -1, B = H_eff, J_l = L_l; backward
// s = +1, B = H_eff^+, J_l = L_l^+ (Q H^+ = (H Q)^+ for Hermitian Q, and
// J Q J^+ [i][j] = sum_m J[i][m] conj((J Q)[j][m])).  Every Taylor term of a
// step, t_n = (tau / n) G(t_{n-1}), is Hermitian like the state.
//
// One workgroup of 1024 threads runs a whole pass (the update is sequential
// in time and a d x d state is small): each Taylor term is two sweeps over the
// d^2 entries -- X and J_l Q by sparse rows, then the combination -- separated
// by workgroup barriers; the matrices live in device memory (L2-resident).
// Step order and substeps follow the same rule as the trajectory passes, from
// a bound on the generator's norm: 2 (||A|| + sum_i |u_i| ||H_i||) + sum_l ||L_l||^2.
#include <hip/hip_runtime.h>

#include "tk_device.h"
#include "tk_internal.h"

namespace tk {
namespace {

constexpr int kRhoThreads = 1024;

__device__ __forceinline__ cx<double> cmul(const cx<double> &a, const cx<double> &b) {
  return cx<double>{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__device__ __forceinline__ cx<double> conjc(const cx<double> &a) { return cx<double>{a.x, -a.y}; }

// Fixed-order sum over the workgroup (each thread's partial, then a tree);
// every thread receives the same value.
__device__ double block_sum(double v, double *red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int off = kRhoThreads / 2; off > 0; off >>= 1) {
    if (static_cast<int>(threadIdx.x) < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  const double s = red[0];
  __syncthreads();
  return s;
}

__device__ __forceinline__ const cx<double> *cv(const void *p) {
  return static_cast<const cx<double> *>(p);
}
__device__ __forceinline__ cx<double> *cv(void *p) { return static_cast<cx<double> *>(p); }

// y = sum over row i of M (CSR) of M[i][k] Q[k][j]
__device__ __forceinline__ cx<double> row_times(const RhoCsr &m, int i, const cx<double> *Q, int j,
                                                int d) {
  cx<double> y{0.0, 0.0};
  const cx<double> *val = cv(m.val);
  for (int p = m.ptr[i]; p < m.ptr[i + 1]; ++p) cfma(y, val[p], Q[static_cast<size_t>(m.idx[p]) * d + j]);
  return y;
}

// Advance R over one interval of length dt with pulses uj.
__device__ void rho_interval(const RhoArgs &a, const double *uj, int d) {
  const int n2 = d * d;
  double b = a.gen_b0 + a.gen_bj;
  for (int c = 0; c < a.n_ctrl; ++c) b += fabs(uj[c]) * a.gen_bc[c];
  const double x = b * a.dt;
  int n_sub = x > kMaxStepNorm ? static_cast<int>(ceil(x / kMaxStepNorm)) : 1;
  if (n_sub > kMaxSubsteps) {  // a generator far too large for the time step
    if (threadIdx.x == 0) atomicOr(a.err, kErrTaylorOrder);
    n_sub = kMaxSubsteps;
  }
  const double h = a.dt / n_sub;
  int K = 1;
  while (K < a.kmax && b * h > a.ord_x[K]) ++K;
  if (b * h > a.ord_x[K] && threadIdx.x == 0) atomicOr(a.err, kErrTaylorOrder);
  for (int sub = 0; sub < n_sub; ++sub) {
    // t_0 = R
    for (int e = threadIdx.x; e < n2; e += kRhoThreads) cv(a.Q0)[e] = cv(a.R)[e];
    __syncthreads();
    cx<double> *Qin = cv(a.Q0), *Qout = cv(a.Q1);
    for (int n = 1; n <= K; ++n) {
      // sweep 1: X = B Qin, Y_l = J_l Qin
      for (int e = threadIdx.x; e < n2; e += kRhoThreads) {
        const int i = e / d, j = e - i * d;
        cx<double> xv = row_times(a.B, i, Qin, j, d);
        for (int c = 0; c < a.n_ctrl; ++c) {
          const cx<double> hq = row_times(a.H[c], i, Qin, j, d);
          xv.x = fma(uj[c], hq.x, xv.x);
          xv.y = fma(uj[c], hq.y, xv.y);
        }
        cv(a.X)[e] = xv;
        for (int l = 0; l < a.n_jump; ++l) cv(a.Y)[static_cast<size_t>(l) * n2 + e] = row_times(a.J[l], i, Qin, j, d);
      }
      __syncthreads();
      // sweep 2: t_n = (h / n) [s i (X - X^+) + sum_l J_l Y_l^+], R += t_n
      const double cf = h / n;
      for (int e = threadIdx.x; e < n2; e += kRhoThreads) {
        const int i = e / d, j = e - i * d;
        const cx<double> xij = cv(a.X)[e], xji = cv(a.X)[static_cast<size_t>(j) * d + i];
        // s i (x_ij - conj(x_ji))
        const double dr = xij.x - xji.x, di = xij.y + xji.y;
        cx<double> g{-a.s * di, a.s * dr};
        for (int l = 0; l < a.n_jump; ++l) {
          const RhoCsr &J = a.J[l];
          const cx<double> *Yl = cv(a.Y) + static_cast<size_t>(l) * n2;
          const cx<double> *Jv = cv(J.val);
          for (int p = J.ptr[i]; p < J.ptr[i + 1]; ++p)
            cfma(g, Jv[p], conjc(Yl[static_cast<size_t>(j) * d + J.idx[p]]));
        }
        const cx<double> t{cf * g.x, cf * g.y};
        Qout[e] = t;
        cv(a.R)[e] = cx<double>{cv(a.R)[e].x + t.x, cv(a.R)[e].y + t.y};
      }
      __syncthreads();
      cx<double> *tmp = Qin;
      Qin = Qout;
      Qout = tmp;
    }
  }
}

// Plain forward (dir 0, J_T of rho(T)), backward (dir 1, storing P(t_j)), or
// the sequential forward pass with the update (dir 0 and a.P set).
__global__ __launch_bounds__(kRhoThreads) void k_rho_pass(RhoArgs a, int dir) {
  __shared__ double red[kRhoThreads];
  __shared__ double s_u[kMaxCtrl];
  const int d = a.d, n2 = d * d;
  for (int e = threadIdx.x; e < n2; e += kRhoThreads) {
    const int i = e / d, j = e - i * d;
    cv(a.R)[e] = cmul(cv(a.start)[i], conjc(cv(a.start)[j]));
  }
  __syncthreads();
  for (int jj = 0; jj < a.nt; ++jj) {
    const int j = dir == 0 ? jj : a.nt - 1 - jj;
    double uj[kMaxCtrl];
    if (dir == 0 && a.P != nullptr) {
      // Im <<P_j| [H_i, rho]>> = Im sum_ab conj(P_ab) (Z_ab - conj(Z_ba)), Z = H_i rho
      const cx<double> *Pj = cv(a.P) + static_cast<size_t>(j) * n2;
      for (int c = 0; c < a.n_ctrl; ++c) {
        for (int e = threadIdx.x; e < n2; e += kRhoThreads) {
          const int i = e / d, k = e - i * d;
          cv(a.X)[e] = row_times(a.H[c], i, cv(a.R), k, d);
        }
        __syncthreads();
        double part = 0.0;
        for (int e = threadIdx.x; e < n2; e += kRhoThreads) {
          const int i = e / d, k = e - i * d;
          const cx<double> z = cv(a.X)[e], zt = cv(a.X)[static_cast<size_t>(k) * d + i];
          const cx<double> comm{z.x - zt.x, z.y + zt.y};  // Z_ik - conj(Z_ki)
          const cx<double> p = Pj[e];
          part += p.x * comm.y - p.y * comm.x;  // Im(conj(p) comm)
        }
        const double sc = block_sum(part, red);
        if (threadIdx.x == 0) {
          const size_t ij = static_cast<size_t>(c) * a.nt + j;
          const double un = a.u_old[ij] + a.S[ij] / a.lam[c] * sc;
          a.u_new[ij] = un;
          s_u[c] = un;
        }
        __syncthreads();
      }
      for (int c = 0; c < a.n_ctrl; ++c) uj[c] = s_u[c];
    } else {
      for (int c = 0; c < a.n_ctrl; ++c) uj[c] = a.u[static_cast<size_t>(c) * a.nt + j];
    }
    rho_interval(a, uj, d);
    if (dir == 1 && a.store != nullptr) {
      cx<double> *out = cv(a.store) + static_cast<size_t>(j) * n2;
      for (int e = threadIdx.x; e < n2; e += kRhoThreads) out[e] = cv(a.R)[e];
      __syncthreads();
    }
  }
  if (dir == 0) {
    double part = 0.0;  // Re <tgt|rho|tgt>
    for (int e = threadIdx.x; e < n2; e += kRhoThreads) {
      const int i = e / d, k = e - i * d;
      const cx<double> v = cmul(cmul(conjc(cv(a.tgt)[i]), cv(a.R)[e]), cv(a.tgt)[k]);
      part += v.x;
    }
    const double f = block_sum(part, red);
    if (threadIdx.x == 0 && a.J_out != nullptr) *a.J_out = 1.0 - f;
  }
}

}  // namespace

hipError_t launch_rho_pass(const RhoArgs &a, int dir, hipStream_t stream) {
  RhoArgs arg = a;
  void *args[] = {&arg, &dir};
  return hipLaunchKernel(reinterpret_cast<const void *>(&k_rho_pass), dim3(1), dim3(kRhoThreads),
                         args, 0, stream);
}

}  // namespace tk
