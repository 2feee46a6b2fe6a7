// Device-side building blocks shared by the propagation kernels:
// complex helpers, wavefront reductions, Philox4x64-10, the per-lane
// operator slice, Taylor steps, dense output, jump handling and step
// planning.  Included by every kernel source (internal linkage).
#pragma once

#include <hip/hip_runtime.h>

#include "tk_internal.h"

namespace tk {
namespace {

// complex number of the bulk precision; aligned to its size so that one LDS
// access moves a whole element
template <typename real>
struct alignas(2 * sizeof(real)) cx {
  real x, y;
};

// Global-memory view of a pointer.  The batched kernels read their pointers
// from an instance table in device memory, whose address space the compiler
// cannot tell: it then emits flat instructions, which count against the LDS
// wait counter as well, so every LDS wait also waits for global loads and
// stores in flight.  Accesses through this view are global instructions.
// (Pointers from kernel arguments are global already; there it changes
// nothing.)  A translation unit that defines TK_GENERIC_ACCESS before this
// header keeps plain accesses: the gradient kernel, which spills, measured
// 5 % slower with the views.
#ifndef TK_GENERIC_ACCESS
#define TK_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ TK_GLOBAL T *gmem(T *p) {
  return (TK_GLOBAL T *)p;
}
template <typename T>
__device__ __forceinline__ const TK_GLOBAL T *gmem(const T *p) {
  return (const TK_GLOBAL T *)p;
}
// complex elements move through the view as two-element vectors (a struct's
// implicit assignment cannot take an object in the global address space)
template <typename real>
using vec2 = real __attribute__((ext_vector_type(2)));
template <typename real>
__device__ __forceinline__ cx<real> gld(const cx<real> *p, size_t i) {
  const vec2<real> v = ((const TK_GLOBAL vec2<real> *)p)[i];
  return cx<real>{v.x, v.y};
}
template <typename real>
__device__ __forceinline__ void gst(cx<real> *p, size_t i, const cx<real> &c) {
  ((TK_GLOBAL vec2<real> *)p)[i] = vec2<real>{c.x, c.y};
}
__device__ __forceinline__ TrajMeta gld(const TrajMeta *p, size_t i) {
  const TK_GLOBAL TrajMeta *q = gmem(p) + i;
  TrajMeta t;
  t.nrm2 = q->nrm2;
  t.r = q->r;
  t.x = q->x;
  t.ordinal = q->ordinal;
  t.pad = q->pad;
  return t;
}
__device__ __forceinline__ void gst(TrajMeta *p, size_t i, const TrajMeta &t) {
  TK_GLOBAL TrajMeta *q = gmem(p) + i;
  q->nrm2 = t.nrm2;
  q->r = t.r;
  q->x = t.x;
  q->ordinal = t.ordinal;
  q->pad = t.pad;
}
#else
template <typename T>
__device__ __forceinline__ T *gmem(T *p) {
  return p;
}
template <typename T>
__device__ __forceinline__ T gld(const T *p, size_t i) {
  return p[i];
}
template <typename T>
__device__ __forceinline__ void gst(T *p, size_t i, const T &v) {
  p[i] = v;
}
#endif

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int CTRL>
__device__ __forceinline__ double dpp_mov(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double read_lane(double x, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
  return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a full wave; every lane receives the same value.
// Within a 16-lane row: pairs (xor 1), pairs of pairs (xor 2), half-row
// mirror, row mirror -- each lane adds a partner holding a disjoint partial
// sum, and both partners add the same two operands.  Then the four row sums
// are combined as (row0 + row1) + (row2 + row3).
__device__ __forceinline__ double wave_sum(double x) {
  x += dpp_mov<0xB1>(x);   // quad_perm [1,0,3,2]
  x += dpp_mov<0x4E>(x);   // quad_perm [2,3,0,1]
  x += dpp_mov<0x141>(x);  // row_half_mirror
  x += dpp_mov<0x140>(x);  // row_mirror
  return (read_lane(x, 0) + read_lane(x, 16)) + (read_lane(x, 32) + read_lane(x, 48));
}

// Two wave sums at once (the DPP chains interleave); same order as wave_sum.
__device__ __forceinline__ void wave_sum2(double &x, double &y) {
  x += dpp_mov<0xB1>(x);
  y += dpp_mov<0xB1>(y);
  x += dpp_mov<0x4E>(x);
  y += dpp_mov<0x4E>(y);
  x += dpp_mov<0x141>(x);
  y += dpp_mov<0x141>(y);
  x += dpp_mov<0x140>(x);
  y += dpp_mov<0x140>(y);
  x = (read_lane(x, 0) + read_lane(x, 16)) + (read_lane(x, 32) + read_lane(x, 48));
  y = (read_lane(y, 0) + read_lane(y, 16)) + (read_lane(y, 32) + read_lane(y, 48));
}

// v[i] for a lane-dependent i < N, by comparisons (indexing a register array
// with a lane value would move the array to scratch memory).
template <int N>
__device__ __forceinline__ double pick(const double (&v)[N], int i) {
  double r = v[0];
#pragma unroll
  for (int q = 1; q < N; ++q)
    if (i == q) r = v[q];
  return r;
}

// Wave sums of the first N entries of v, two at a time.
template <int N, int L>
__device__ __forceinline__ void wave_sum_n(double (&v)[L]) {
#pragma unroll
  for (int c = 0; c + 1 < N; c += 2) wave_sum2(v[c], v[c + 1]);
  if (N % 2) v[N - 1] = wave_sum(v[N - 1]);
}

// The lanes that advance one trajectory together: G wavefronts (G = 1: one
// wavefront; G > 1: the G waves of a block, which then holds just this team).
// Row r of a state belongs to team lane r mod 64G as its slot m = r / 64G.
// Workgroup barrier that orders LDS traffic only: it waits for the wave's own
// LDS operations, not for its global loads and stores still in flight (which
// __syncthreads' release fence would wait for).  Every exchange between the
// waves of a block in these kernels goes through LDS.
__device__ __forceinline__ void block_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// sync() orders LDS traffic among the team; sum() is the team-wide FP64 sum
// in a fixed order (each wave's DPP tree, then the waves in index order, via a
// double-buffered LDS array), so every lane of the team holds the same bits.
template <int G>
struct Team {
  static constexpr int kLanes = kWave * G;
  int gl;            // lane within the team
  int lane;          // lane within the wave
  int g;             // wave within the team
  double *red;       // LDS [2][4 G] (G > 1)
  mutable int par;   // half of red the next sum writes
  __device__ __forceinline__ void sync() const {
    if (G == 1)
      wave_sync();
    else
      block_sync_lds();
  }
  __device__ __forceinline__ double sum(double x) const {
    x = wave_sum(x);
    if (G == 1) return x;
    double *r = red + par * 4 * G;
    if (lane == 0) r[g] = x;
    block_sync_lds();
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < G; ++q) s += r[q];
    par ^= 1;
    return s;
  }
  // two team sums with one exchange
  __device__ __forceinline__ void sum2(double &x, double &y) const {
    wave_sum2(x, y);
    if (G == 1) return;
    double *r = red + par * 4 * G;
    if (lane == 0) {
      r[g] = x;
      r[G + g] = y;
    }
    block_sync_lds();
    double sx = 0.0, sy = 0.0;
#pragma unroll
    for (int q = 0; q < G; ++q) {
      sx += r[q];
      sy += r[G + q];
    }
    par ^= 1;
    x = sx;
    y = sy;
  }
  // the first N entries of v summed over the team: wave sums two at a time,
  // then up to four values per exchange between the waves (each value with
  // the bits sum() gives it)
  template <int N, int L>
  __device__ __forceinline__ void sum_n(double (&v)[L]) const {
    wave_sum_n<N>(v);
    if (G == 1) return;
#pragma unroll
    for (int c0 = 0; c0 < N; c0 += 4) {
      constexpr int kQ = 4;
      double *r = red + par * 4 * G;
      if (lane == 0)
#pragma unroll
        for (int q = 0; q < kQ; ++q)
          if (c0 + q < N) r[q * G + g] = v[c0 + q];
      block_sync_lds();
#pragma unroll
      for (int q = 0; q < kQ; ++q) {
        if (c0 + q >= N) break;
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < G; ++w) s += r[q * G + w];
        v[c0 + q] = s;
      }
      par ^= 1;
    }
  }
  __device__ __forceinline__ bool leader() const { return gl == 0; }
};

template <int G>
__device__ __forceinline__ Team<G> make_team(double *red) {
  Team<G> t;
  t.gl = threadIdx.x % Team<G>::kLanes;
  t.lane = threadIdx.x & (kWave - 1);
  t.g = __builtin_amdgcn_readfirstlane(t.gl / kWave);
  t.red = red;
  t.par = 0;
  return t;
}

// ---- Philox4x64-10 (Salmon et al., SC'11) ---------------------------------
__device__ __forceinline__ void philox4x64(uint64_t c0, uint64_t c1, uint64_t c2,
                                           uint64_t c3, uint64_t k0, uint64_t k1,
                                           uint64_t &w0, uint64_t &w1) {
  constexpr uint64_t kMul0 = 0xD2E7470EE14C6C93ull;
  constexpr uint64_t kMul1 = 0xCA5A826395121157ull;
  constexpr uint64_t kWeyl0 = 0x9E3779B97F4A7C15ull;
  constexpr uint64_t kWeyl1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int rnd = 0; rnd < 10; ++rnd) {
    if (rnd) {
      k0 += kWeyl0;
      k1 += kWeyl1;
    }
    const uint64_t lo0 = kMul0 * c0, hi0 = __umul64hi(kMul0, c0);
    const uint64_t lo1 = kMul1 * c2, hi1 = __umul64hi(kMul1, c2);
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  w0 = c0;
  w1 = c1;
}

__device__ __forceinline__ double to_unit(uint64_t w) {
  return static_cast<double>(w >> 11) * 0x1.0p-53;
}

// A wave-uniform 64-bit value moved to scalar registers, so that arithmetic
// on it runs on the scalar unit (Philox's 64-bit products are far cheaper
// there than as quarter-rate vector multiplies).
__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v >> 32));
  return (static_cast<uint64_t>(hi) << 32) | lo;
}

// Counter-based stream of one trajectory.  Every argument is uniform across
// the team that advances the trajectory.
struct Stream {
  uint64_t k0, k1, iteration, direction;
  __device__ void block(uint64_t ordinal, double &thr, double &choice) const {
    uint64_t w0, w1;
    philox4x64(uniform64(ordinal), uniform64(iteration), uniform64(direction), 0, uniform64(k0),
               uniform64(k1), w0, w1);
    thr = to_unit(w0);
    choice = to_unit(w1);
  }
  // threshold and operator-choice number of jump `ordinal` (one block)
  __device__ void draw(uint64_t ordinal, TrajMeta &st) const { block(ordinal, st.r, st.x); }
};

// Stream of trajectory k: key [seed, (instance << 32) | k], counter
// [ordinal, iteration, direction, 0]
__device__ __forceinline__ Stream make_stream(const PassArgs &a, int k, int dir,
                                              uint64_t iteration) {
  Stream s;
  s.k0 = a.seed;
  s.k1 = (static_cast<uint64_t>(a.instance) << 32) | static_cast<uint32_t>(k);
  s.iteration = iteration;
  s.direction = static_cast<uint64_t>(dir);
  return s;
}

__device__ __forceinline__ Stream make_stream(const PassArgs &a, int k, int dir) {
  return make_stream(a, k, dir, a.iteration);
}

template <typename real>
__device__ __forceinline__ void cfma(cx<real> &y, const cx<real> &a, const cx<real> &b) {
  y.x = fma(a.x, b.x, y.x);
  y.x = fma(-a.y, b.y, y.x);
  y.y = fma(a.x, b.y, y.y);
  y.y = fma(a.y, b.x, y.y);
}

// y += a b for a control element a; RC: a is real (a.y is zero), two FMAs
template <bool RC, typename real>
__device__ __forceinline__ void cfma_ctrl(cx<real> &y, const cx<real> &a, const cx<real> &b) {
  if constexpr (RC) {
    y.x = fma(a.x, b.x, y.x);
    y.y = fma(a.x, b.y, y.y);
  } else {
    cfma(y, a, b);
  }
}

// Values the compiler cannot follow across this point.  A load whose address
// derives from one stays where it is written: the compiler neither hoists it
// out of an enclosing loop nor keeps its 64-bit address in registers from an
// earlier iteration (with one address per operator element, those held
// addresses alone can push a kernel into scratch spills).
template <typename T>
__device__ __forceinline__ const T *opaque(const T *p) {
  asm volatile("" : "+s"(p));
  return p;
}
__device__ __forceinline__ int opaque_lane(int gl) {
  asm volatile("" : "+v"(gl));
  return gl;
}

// ---- per-lane operator slice ------------------------------------------------
template <typename real, int R, int WS, int NC, int G>
struct LaneOp {
  static constexpr int kL = kWave * G;  // lanes of the team
  static constexpr int NCX = NC > 0 ? NC : 1;
  static constexpr int W0 = ws_first(WS);  // static slots of row slot 0 (the most)
  static constexpr bool RC = ws_real_ctrl(WS);  // real control elements
  static constexpr bool TY = ws_typed(WS);       // typed static slots in row slot 0
  static constexpr int WR = W0 - ws_imag(WS);    // (the real ones; the rest imaginary)
  // y += v b for static slot s of row slot m: typed slots hold a real element
  // (v.x) or an imaginary one (i v.y) and take two FMAs
  __device__ __forceinline__ static void sfma(cx<real> &y, const cx<real> &v, const cx<real> &b,
                                              int s, int m) {
    if (TY && m == 0) {
      if (s < WR) {
        y.x = fma(v.x, b.x, y.x);
        y.y = fma(v.x, b.y, y.y);
      } else {
        y.x = fma(-v.y, b.y, y.x);
        y.y = fma(v.y, b.x, y.y);
      }
    } else {
      cfma(y, v, b);
    }
  }
  // slot s of row slot m is used (unrolled loops fold this to a constant)
  static constexpr bool live(int s, int m) { return s < ws_at(WS, m); }
  int scol[W0][R];
  cx<real> sval[W0][R];  // off-diagonal elements of the static part
  cx<real> dval[R];      // its diagonal: multiplies the lane's own element, no gather
  int ccol[NCX][R];
  cx<real> cv[NCX][R];   // control matrix elements scaled by the current pulses
  const cx<real> *cval;  // unscaled control elements of this lane, [c][m][team lane]
  // LDS addresses of the gathered elements within term vector 0 (see bind);
  // term n lies n vector lengths further on, a constant offset
  const cx<real> *sp[W0][R];
  const cx<real> *cp[NCX][R];

  // static slots (scol_g, sval_g), the static diagonal (sdiag_g, [m][team
  // lane]) and control columns (ccol_g) from global memory; the unscaled
  // control values stay where cval_src points (LDS or global memory); gl is
  // the lane within the team
  __device__ void load(const int *scol_g, const void *sval_g, const void *sdiag_g,
                       const int *ccol_g, const cx<real> *cval_src, int gl) {
    gl = opaque_lane(gl);
    const cx<real> *sv = static_cast<const cx<real> *>(sval_g);
    const cx<real> *sd = static_cast<const cx<real> *>(sdiag_g);
#pragma unroll
    for (int m = 0; m < R; ++m) dval[m] = gld(sd, m * kL + gl);
#pragma unroll
    for (int s = 0; s < W0; ++s)
#pragma unroll
      for (int m = 0; m < R; ++m) {
        if (!live(s, m)) continue;
        const int idx = (s * R + m) * kL + gl;
        scol[s][m] = gmem(scol_g)[idx];
        sval[s][m] = gld(sv, idx);
      }
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int m = 0; m < R; ++m) {
        ccol[c][m] = gmem(ccol_g)[(c * R + m) * kL + gl];
        cv[c][m] = cx<real>{0, 0};
      }
    cval = cval_src + gl;
  }

  // addresses of the lane's gathers in the term vector t0 (once per team)
  __device__ void bind(const cx<real> *t0) {
#pragma unroll
    for (int s = 0; s < W0; ++s)
#pragma unroll
      for (int m = 0; m < R; ++m)
        if (live(s, m)) sp[s][m] = t0 + scol[s][m];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int m = 0; m < R; ++m) cp[c][m] = t0 + ccol[c][m];
  }

  // unscaled control element of slot c, row slot m (from the lane's elements at base)
  __device__ __forceinline__ cx<real> cval_at(int c, int m, const cx<real> *base) const {
    // one-wave teams read a copy in LDS, G-wave teams global memory
    if constexpr (G > 1)
      return gld(base, (c * R + m) * kL);
    else
      return base[(c * R + m) * kL];
  }
  __device__ __forceinline__ cx<real> cval_at(int c, int m) const { return cval_at(c, m, cval); }

  // cv = u_{c / wc} * cval for the pulse values uj[0 .. NCX) (zero past n_ctrl)
  __device__ void set_pulses(const double (&uj)[NCX], int wc) {
    const cx<real> *base = cval + opaque_lane(0);  // addresses formed here, per call
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      // control c / wc (< NC, hence a valid index), by comparisons: the slot
      // count is small and a division would cost more
      double u = uj[0];
#pragma unroll
      for (int i = 1; i < NC; ++i)
        if (c >= i * wc) u = uj[i];
      const real ui = static_cast<real>(u);
#pragma unroll
      for (int m = 0; m < R; ++m) {
        const cx<real> q = cval_at(c, m, base);
        cv[c][m] = cx<real>{ui * q.x, ui * q.y};
      }
    }
  }

  // y = Op v for the lane's rows, v the term vector `shift` elements past the
  // one the gathers are bound to, own = the lane's rows of v.  All gathers
  // first.
  // Eight-wave shapes (short of registers) gather and multiply the static
  // slots before gathering the control slots; the multiply-add order is the
  // same either way.
  __device__ void apply_at(int shift, const cx<real> (&own)[R], cx<real> (&y)[R]) const {
    constexpr bool kHalves = G >= 4;
    cx<real> b[W0 + NC][R];
#pragma unroll
    for (int s = 0; s < W0; ++s)
#pragma unroll
      for (int m = 0; m < R; ++m)
        if (live(s, m)) b[s][m] = sp[s][m][shift];
    if constexpr (!kHalves) {
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int m = 0; m < R; ++m) b[W0 + c][m] = cp[c][m][shift];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int m = 0; m < R; ++m) {
      y[m] = cx<real>{0, 0};
      cfma(y[m], dval[m], own[m]);
    }
#pragma unroll
    for (int s = 0; s < W0; ++s)
#pragma unroll
      for (int m = 0; m < R; ++m)
        if (live(s, m)) sfma(y[m], sval[s][m], b[s][m], s, m);
    if constexpr (kHalves) {
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int m = 0; m < R; ++m) b[W0 + c][m] = cp[c][m][shift];
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int m = 0; m < R; ++m) cfma_ctrl<RC>(y[m], cv[c][m], b[W0 + c][m]);
  }

};

template <typename real, int R, int G>
__device__ __forceinline__ double norm2(const cx<real> (&p)[R], const Team<G> &tm) {
  double s = 0.0;
#pragma unroll
  for (int m = 0; m < R; ++m) {
    const double x = p[m].x, y = p[m].y;
    s = fma(x, x, s);
    s = fma(y, y, s);
  }
  return tm.sum(s);
}

// the lane's rows of a team vector (LDS or global memory)
template <typename real, int R, int G>
__device__ __forceinline__ void store_lds(cx<real> *v, const cx<real> (&p)[R], const Team<G> &tm) {
#pragma unroll
  for (int m = 0; m < R; ++m) v[tm.gl + Team<G>::kLanes * m] = p[m];
}

template <typename real, int R, int G>
__device__ __forceinline__ void load_lds(const cx<real> *v, cx<real> (&p)[R], const Team<G> &tm) {
#pragma unroll
  for (int m = 0; m < R; ++m) p[m] = v[tm.gl + Team<G>::kLanes * m];
}

// Per-team LDS view: term vectors T_0 .. T_{kbuf-1}, each 64 G R + 1
// elements (element 64 G R is the zero read by padding slots).
template <typename real, int R, int G>
struct Terms {
  static constexpr int kLen = R * kWave * G + 1;
  cx<real> *base;
  __device__ cx<real> *operator[](int n) const { return base + n * kLen; }
};

// Smallest order K whose remainder bound x^(K+1)/(K+1)! e^x meets the step
// tolerance, read from the launch's threshold table (x <= ord_x[K]), or -1
// when kmax does not suffice.  The search starts at `hint` (a nearby order),
// so it costs one or two comparisons.
__device__ __forceinline__ int taylor_order(const PassArgs &a, double x, int hint) {
  int K = hint < 1 ? 1 : (hint > a.kmax ? a.kmax : hint);
  while (K < a.kmax && x > a.ord_x[K]) ++K;
  while (K > 1 && x <= a.ord_x[K - 1]) --K;
  return x <= a.ord_x[K] ? K : -1;
}

// The order found for the previous step with its interval ord_x[K-1] < x <=
// ord_x[K]: a step whose x falls in it (the usual case, pulses being smooth)
// needs no table read.  Starts empty.
struct OrderHint {
  int K = 1;
  double lo = 1.0, hi = 0.0;
  __device__ __forceinline__ int order(const PassArgs &a, double x) {
    if (x > lo && x <= hi) return K;
    const int k = taylor_order(a, x, K);
    if (k > 0) {
      K = k;
      lo = k > 1 ? a.ord_x[k - 1] : -1.0;
      hi = a.ord_x[k];
    }
    return k;
  }
};

// out = sum_{n=0..K} t_n with t_n = (s i tau Op)^n / n! in, s = -1 (forward)
// or +1 (backward); t_n is also left in T[n] for dense output.  The small
// increment sum_{n>=1} t_n is accumulated on its own and added to t_0 once, so
// the state is rounded once per substep rather than once per term.
template <typename real, int R, int WS, int NC, int G, int SGN>
__device__ void taylor(const LaneOp<real, R, WS, NC, G> &op, const PassArgs &a,
                       const Terms<real, R, G> &T, const cx<real> (&in)[R], cx<real> (&out)[R],
                       double tau, int K, const Team<G> &tm) {
  cx<real> t[R], inc[R];
#pragma unroll
  for (int m = 0; m < R; ++m) {
    t[m] = in[m];
    inc[m] = cx<real>{0, 0};
  }
  store_lds(T[0], t, tm);
  for (int n = 1; n <= K; ++n) {
    tm.sync();
    cx<real> y[R];
    op.apply_at((n - 1) * Terms<real, R, G>::kLen, t, y);
    const real c = static_cast<real>(tau * a.inv_n[n]);
#pragma unroll
    for (int m = 0; m < R; ++m) {
      if (SGN < 0)
        t[m] = cx<real>{c * y[m].y, -c * y[m].x};
      else
        t[m] = cx<real>{-c * y[m].y, c * y[m].x};
      inc[m].x += t[m].x;
      inc[m].y += t[m].y;
    }
    store_lds(T[n], t, tm);
  }
#pragma unroll
  for (int m = 0; m < R; ++m) out[m] = cx<real>{in[m].x + inc[m].x, in[m].y + inc[m].y};
}

// One term of the series from the term vector at the bound gather addresses
// plus OFF elements: t = (s i tau / n) Op t_prev for the lane's rows.
// `shift` (elements, uniform) moves every gather to a later term vector; a
// run of terms with the same shift shares its address arithmetic.
// Gathers and multiply-adds of slots [S0, S1) (static slots first, then the
// control slots) into y, all gathers of the range issued first.
template <typename real, int R, int WS, int NC, int G, int OFF, int S0, int S1>
__device__ __forceinline__ void gather_fma(const LaneOp<real, R, WS, NC, G> &op, int shift,
                                           cx<real> (&y)[R]) {
  constexpr int W0 = LaneOp<real, R, WS, NC, G>::W0;
  using Op = LaneOp<real, R, WS, NC, G>;
  cx<real> b[S1 - S0][R];
#pragma unroll
  for (int s = S0; s < S1; ++s)
#pragma unroll
    for (int m = 0; m < R; ++m) {
      if (s < W0 && !Op::live(s, m)) continue;
      b[s - S0][m] = s < W0 ? (op.sp[s < W0 ? s : 0][m] + shift)[OFF]
                            : (op.cp[s < W0 ? 0 : s - W0][m] + shift)[OFF];
    }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int s = S0; s < S1; ++s)
#pragma unroll
    for (int m = 0; m < R; ++m) {
      if (s < W0 && !Op::live(s, m)) continue;
      if (s < W0)
        Op::sfma(y[m], op.sval[s < W0 ? s : 0][m], b[s - S0][m], s, m);
      else
        cfma_ctrl<Op::RC>(y[m], op.cv[s < W0 ? 0 : s - W0][m], b[s - S0][m]);
    }
}

// One term of the series from the term vector at the bound gather addresses
// plus OFF elements: t = (s i tau / n) Op t_prev for the lane's rows.  Shapes
// with more than 16 gathers per lane issue them in two halves, so that half
// the gathered values need registers at a time (these shapes are the ones
// short of registers); the multiply-adds keep their order.  Measured: d = 1296
// passes 24 % faster, d = 216 Krotov iterations 1-4 %.  SPLIT = false keeps
// one batch (the gradient kernel, whose other live values make the halves
// slower there: its d = 1296 gradient 16 %).
template <typename real, int R, int WS, int NC, int G, int SGN, int OFF, bool SPLIT = true>
__device__ __forceinline__ void series_term(const LaneOp<real, R, WS, NC, G> &op, real cf,
                                            cx<real> (&t)[R], cx<real> (&inc)[R],
                                            int shift = 0) {
  constexpr int NS = LaneOp<real, R, WS, NC, G>::W0 + NC;
  constexpr int H = (SPLIT && NS * R > 16) ? (NS + 1) / 2 : NS;
  cx<real> y[R];
#pragma unroll
  for (int m = 0; m < R; ++m) {  // the diagonal first, from t_prev in registers
    y[m] = cx<real>{0, 0};
    cfma(y[m], op.dval[m], t[m]);
  }
  gather_fma<real, R, WS, NC, G, OFF, 0, H>(op, shift, y);
  if constexpr (H < NS) gather_fma<real, R, WS, NC, G, OFF, H, NS>(op, shift, y);
#pragma unroll
  for (int m = 0; m < R; ++m) {
    if (SGN < 0)
      t[m] = cx<real>{cf * y[m].y, -cf * y[m].x};
    else
      t[m] = cx<real>{-cf * y[m].y, cf * y[m].x};
    inc[m].x += t[m].x;
    inc[m].y += t[m].y;
  }
}

// The same series without keeping the terms: they alternate between T[0]
// and T[1], read through the addresses bound to T[0] (LaneOp::bind) plus a
// constant, so the loop does no address arithmetic.  Steps that end in a jump
// rebuild the stored terms with taylor() for the dense output.
template <typename real, int R, int WS, int NC, int G, int SGN, bool SPLIT = true>
__device__ void taylor_pingpong(const LaneOp<real, R, WS, NC, G> &op, const PassArgs &a,
                                const Terms<real, R, G> &T, const cx<real> (&in)[R],
                                cx<real> (&out)[R], double tau, int K, const Team<G> &tm,
                                double *d0 = nullptr) {
  constexpr int kLen = Terms<real, R, G>::kLen;
  constexpr int kL = Team<G>::kLanes;
  cx<real> *own = T.base + tm.gl;
  cx<real> t[R], inc[R];
#pragma unroll
  for (int m = 0; m < R; ++m) {
    t[m] = in[m];
    inc[m] = cx<real>{0, 0};
    own[kL * m] = t[m];
  }
  for (int n = 1; n <= K; n += 2) {
    tm.sync();
    series_term<real, R, WS, NC, G, SGN, 0, SPLIT>(op, static_cast<real>(tau * a.inv_n[n]), t, inc);
    if (d0 && n == 1) *d0 = re_dot(in, t);
#pragma unroll
    for (int m = 0; m < R; ++m) own[kLen + kL * m] = t[m];
    if (n + 1 > K) break;
    tm.sync();
    series_term<real, R, WS, NC, G, SGN, kLen, SPLIT>(op, static_cast<real>(tau * a.inv_n[n + 1]), t,
                                                inc);
#pragma unroll
    for (int m = 0; m < R; ++m) own[kL * m] = t[m];
  }
#pragma unroll
  for (int m = 0; m < R; ++m) out[m] = cx<real>{in[m].x + inc[m].x, in[m].y + inc[m].y};
}

// The series keeping every term t_n in T[n] (as taylor() does) at nearly the
// cost of the ping-pong form: terms go in runs of four, each run reading its
// gathers at the bound addresses moved once by the run's first vector plus
// constant offsets of 0 .. 3 vector lengths.
// Re <p|q> over the lane's rows (FP64 partial of a team sum)
template <typename real, int R>
__device__ __forceinline__ double re_dot(const cx<real> (&p)[R], const cx<real> (&q)[R]) {
  double s = 0.0;
#pragma unroll
  for (int m = 0; m < R; ++m) {
    s = fma(static_cast<double>(p[m].x), static_cast<double>(q[m].x), s);
    s = fma(static_cast<double>(p[m].y), static_cast<double>(q[m].y), s);
  }
  return s;
}

// FT: when use_y1 is set, the first term's product Op in comes ready in *y1
// (first_term_parts / first_term_finish: the same multiply-adds in the same
// order as the gathered term), so the first term takes no LDS round trip.
template <typename real, int R, int WS, int NC, int G, int SGN, bool FT = false>
__device__ void taylor_keep(const LaneOp<real, R, WS, NC, G> &op, const PassArgs &a,
                            const Terms<real, R, G> &T, const cx<real> (&in)[R],
                            cx<real> (&out)[R], double tau, int K, const Team<G> &tm,
                            double *d0 = nullptr, const cx<real> (*y1)[R] = nullptr,
                            bool use_y1 = false) {
  constexpr int kLen = Terms<real, R, G>::kLen;
  constexpr int kL = Team<G>::kLanes;
  cx<real> t[R], inc[R];
#pragma unroll
  for (int m = 0; m < R; ++m) {
    t[m] = in[m];
    inc[m] = cx<real>{0, 0};
    T.base[tm.gl + kL * m] = t[m];
  }
  for (int n0 = 0; n0 < K; n0 += 4) {  // terms n0 + 1 .. n0 + 4 from T[n0 .. n0 + 3]
    const int shift = n0 * kLen;
    cx<real> *own = T.base + shift + tm.gl;
    if (FT && n0 == 0 && use_y1) {
      const real cf = static_cast<real>(tau * a.inv_n[1]);
#pragma unroll
      for (int m = 0; m < R; ++m) {
        const cx<real> y = (*y1)[m];
        if (SGN < 0)
          t[m] = cx<real>{cf * y.y, -cf * y.x};
        else
          t[m] = cx<real>{-cf * y.y, cf * y.x};
        inc[m].x += t[m].x;
        inc[m].y += t[m].y;
      }
    } else {
      tm.sync();
      series_term<real, R, WS, NC, G, SGN, 0>(op, static_cast<real>(tau * a.inv_n[n0 + 1]), t,
                                              inc, shift);
    }
    if (d0 && n0 == 0) *d0 = re_dot(in, t);
#pragma unroll
    for (int m = 0; m < R; ++m) own[kLen + kL * m] = t[m];
    if (n0 + 2 > K) break;
    tm.sync();
    series_term<real, R, WS, NC, G, SGN, kLen>(op, static_cast<real>(tau * a.inv_n[n0 + 2]), t,
                                               inc, shift);
#pragma unroll
    for (int m = 0; m < R; ++m) own[2 * kLen + kL * m] = t[m];
    if (n0 + 3 > K) break;
    tm.sync();
    series_term<real, R, WS, NC, G, SGN, 2 * kLen>(op, static_cast<real>(tau * a.inv_n[n0 + 3]),
                                                   t, inc, shift);
#pragma unroll
    for (int m = 0; m < R; ++m) own[3 * kLen + kL * m] = t[m];
    if (n0 + 4 > K) break;
    tm.sync();
    series_term<real, R, WS, NC, G, SGN, 3 * kLen>(op, static_cast<real>(tau * a.inv_n[n0 + 4]),
                                                   t, inc, shift);
#pragma unroll
    for (int m = 0; m < R; ++m) own[4 * kLen + kL * m] = t[m];
  }
#pragma unroll
  for (int m = 0; m < R; ++m) out[m] = cx<real>{in[m].x + inc[m].x, in[m].y + inc[m].y};
}

// p(s) = sum_n s^n t_n and dp/ds from the stored terms (own rows only;
// Horner from t_K down).  The terms are read four at a time, so one LDS
// round trip serves four Horner steps.  (Issuing the next four before the
// current four's multiply-adds needs twice the registers, which the series
// kernels do not have to spare.)
template <typename real, int R, int G>
__device__ __forceinline__ void dense_output(const Terms<real, R, G> &T, int K, real s,
                                             cx<real> (&p)[R], cx<real> (&dp)[R], const Team<G> &tm) {
  load_lds(T[K], p, tm);
#pragma unroll
  for (int m = 0; m < R; ++m) dp[m] = cx<real>{0, 0};
  int n = K - 1;
  for (; n >= 3; n -= 4) {
    cx<real> tq[4][R];
#pragma unroll
    for (int q = 0; q < 4; ++q) load_lds(T[n - q], tq[q], tm);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int m = 0; m < R; ++m) {
        dp[m] = cx<real>{fma(dp[m].x, s, p[m].x), fma(dp[m].y, s, p[m].y)};
        p[m] = cx<real>{fma(p[m].x, s, tq[q][m].x), fma(p[m].y, s, tq[q][m].y)};
      }
  }
  for (; n >= 0; --n) {
    cx<real> tn[R];
    load_lds(T[n], tn, tm);
#pragma unroll
    for (int m = 0; m < R; ++m) {
      dp[m] = cx<real>{fma(dp[m].x, s, p[m].x), fma(dp[m].y, s, p[m].y)};
      p[m] = cx<real>{fma(p[m].x, s, tn[m].x), fma(p[m].y, s, tn[m].y)};
    }
  }
}

// y = L_l p for operator l of a group packed [l][w][m][lane] with wl slots per
// row (slices read from global memory; p in LDS v)
template <typename real, int R, int G>
__device__ void apply_packed(const int *lcol, const void *lval, int wl, int l,
                             const cx<real> *v, cx<real> (&y)[R], const Team<G> &tm) {
  const cx<real> *lv = static_cast<const cx<real> *>(lval);
#pragma unroll
  for (int m = 0; m < R; ++m) y[m] = cx<real>{0, 0};
  // two slots at a time: both slots' global loads, then both gathers, then
  // the multiply-adds in slot order (one global round trip per pair)
  for (int w0 = 0; w0 < wl; w0 += 2) {
    const bool two = w0 + 1 < wl;  // uniform
    int col[2][R];
    cx<real> val[2][R], b[2][R];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int m = 0; m < R; ++m) {
        const int idx = ((l * wl + (two ? w0 + q : w0)) * R + m) * Team<G>::kLanes + tm.gl;
        col[q][m] = gmem(lcol)[idx];
        val[q][m] = gld(lv, idx);
      }
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int m = 0; m < R; ++m) b[q][m] = v[col[q][m]];
#pragma unroll
    for (int m = 0; m < R; ++m) cfma(y[m], val[0][m], b[0][m]);
    if (two)
#pragma unroll
      for (int m = 0; m < R; ++m) cfma(y[m], val[1][m], b[1][m]);
  }
}

// y = L_l p for the jump operators of the pass
template <typename real, int R, int G>
__device__ __forceinline__ void apply_jump(const PassArgs &a, int l, const cx<real> *v,
                                           cx<real> (&y)[R], const Team<G> &tm) {
  apply_packed<real, R, G>(a.lcol, a.lval, a.wl, l, v, y, tm);
}

// Advance one trajectory across one substep of length h starting at time t0
// (MCWF with precise jump times).  DIR 0: forward, exp(-i H_eff tau), times
// t0 + elapsed; DIR 1: backward, exp(+i H_eff^+ tau), times t0 - elapsed.
// K is the order for the whole substep and bnd a bound on ||H_eff||; what is
// left of a substep after a jump takes the (lower) order its length needs.
// KEEP: every series keeps its terms (taylor_keep) so that a step ending in a jump
// goes straight to the root search; otherwise the series alternates two
// vectors (taylor_pingpong, a little cheaper) and a step that ends in a jump
// evaluates it again keeping the terms.  Passes whose step time is set by the
// slowest trajectory (the sequential Krotov pass) keep the terms.
// FT (with KEEP): *y1 is the first series term's product Op psi, formed ahead
// (taylor_keep); it serves the substep's first series only.
template <typename real, int R, int WS, int NC, int G, int DIR, bool KEEP = false, bool FT = false>
__device__ void advance(const LaneOp<real, R, WS, NC, G> &op, const PassArgs &a,
                        const Terms<real, R, G> &T, cx<real> (&psi)[R], TrajMeta &st,
                        const Stream &rng, int j, double t0, double h, int K, double bnd, int k,
                        const Team<G> &tm, const cx<real> (*y1)[R] = nullptr,
                        bool use_y1 = false) {
  static_assert(!FT || KEEP, "a first term formed ahead needs the kept-term series");
  // (one-wave teams with at most two rows per lane: the others are short of
  // registers, and there the extra live values cost more than they save)
  constexpr bool kSlope = G == 1 && R <= 2;
  constexpr int SGN = DIR == 0 ? -1 : 1;
  double tau_rem = h;
  int Kc = K;
  double n_s = st.nrm2;
  cx<real> ps[R];
#pragma unroll
  for (int m = 0; m < R; ++m) ps[m] = psi[m];
  constexpr double eps_real = sizeof(real) == 8 ? 0x1.0p-52 : 0x1.0p-23;
  for (int guard = 0;; ++guard) {
    cx<real> out[R];
    // g0 = Re <t_0|t_1> over the lane's rows: summed over the team only when
    // the substep ends below the threshold, it is half the slope of
    // ||p(s)||^2 at s = 0 for the root search's first point (kSlope shapes;
    // the others start from the secant).
    double g0 = 0.0;
    double *g0p = kSlope ? &g0 : nullptr;
    if (KEEP)
      taylor_keep<real, R, WS, NC, G, SGN, FT>(op, a, T, ps, out, tau_rem, Kc, tm, g0p, y1,
                                                       use_y1 && guard == 0);
    else
      taylor_pingpong<real, R, WS, NC, G, SGN>(op, a, T, ps, out, tau_rem, Kc, tm, g0p);
    const double n_end = norm2(out, tm);
    if (!(n_end < st.r)) {
#pragma unroll
      for (int m = 0; m < R; ++m) psi[m] = out[m];
      st.nrm2 = n_end;
      return;
    }
    if (guard >= 64) {  // pathological: give up on this step, keep the state
      if (tm.leader()) atomicOr(a.err, kErrJumpLoop);
#pragma unroll
      for (int m = 0; m < R; ++m) psi[m] = out[m];
      st.nrm2 = n_end;
      st.r = 0.0;
      return;
    }
    // the record's slot is claimed now; the atomic's round trip overlaps the
    // root search
    unsigned long long slot = 0;
    if (tm.leader()) slot = atomicAdd(a.rec_count, 1ull);
    // ---- jump time: root of f(s) = ||p(s)||^2 - r for s in (0, 1] (tau = s tau_rem) ----
    if (!KEEP) {  // the series again, now keeping every term for the dense output
      cx<real> again[R];
      tm.sync();
      taylor<real, R, WS, NC, G, SGN>(op, a, T, ps, again, tau_rem, Kc, tm);
    }
    tm.sync();
    double lo = 0.0, hi = 1.0;
    if constexpr (kSlope) {
      if (n_s < 0.0) {
        n_s = re_dot(ps, ps);
        tm.sum2(n_s, g0);
      } else {
        g0 = tm.sum(g0);
      }
    } else {
      if (n_s < 0.0) n_s = norm2(ps, tm);
    }
    const double flo = n_s - st.r, fhi = n_end - st.r;
    // first point: the root in (0, 1) of the quadratic through f(0), f'(0)
    // and f(1) (the crossing of the secant if that fails); the Newton
    // iteration's curvature estimate starts from the slope at s = 0
    const double fp0 = 2.0 * g0;
    double s = -1.0;
    if constexpr (kSlope) {
      const double c2 = fhi - flo - fp0;
      const double disc = fma(fp0, fp0, -4.0 * c2 * flo);
      s = 2.0 * flo / (-fp0 + sqrt(fmax(disc, 0.0)));
    }
    if (!(s > lo && s < hi)) s = flo / (flo - fhi);
    if (!(s > lo && s < hi)) s = 0.5;
    cx<real> pt[R], dp[R];
    double s_prev = kSlope ? 0.0 : -1.0, fp_prev = fp0;
    for (int it = 0; it < 64; ++it) {
      dense_output<real, R, G>(T, Kc, static_cast<real>(s), pt, dp, tm);
      double f = 0.0, g = 0.0;  // ||p||^2 and Re <p|dp/ds>, reduced together
#pragma unroll
      for (int m = 0; m < R; ++m) {
        const double px = pt[m].x, py = pt[m].y;
        f = fma(px, px, f);
        f = fma(py, py, f);
        g = fma(px, static_cast<double>(dp[m].x), g);
        g = fma(py, static_cast<double>(dp[m].y), g);
      }
      tm.sum2(f, g);
      f -= st.r;
      const double fp = 2.0 * g;
      if (f >= 0.0)
        lo = s;
      else
        hi = s;
      if (fabs(f) <= a.ftol * st.r || (hi - lo) <= 4.0 * eps_real) break;
      double sn = s - f / fp;
      const bool inside = sn > lo && sn < hi;
      if (!inside) sn = 0.5 * (lo + hi);
      // A Newton step from s leaves an error of about |f''/(2 f')| (sn - s)^2;
      // with f'' estimated from the derivatives at the last two points, the
      // step is taken without evaluating f again once that is below
      // kRootAccept (of the unit interval).
      bool accept = fabs(sn - s) <= 2.0 * eps_real;
      if (!accept && inside && s_prev >= 0.0 && s != s_prev && fp != 0.0) {
        const double c = fabs((fp - fp_prev) / (s - s_prev)) / (2.0 * fabs(fp));
        accept = c * (sn - s) * (sn - s) <= kRootAccept;
      }
      if (accept) {
        s = sn;
        dense_output<real, R, G>(T, Kc, static_cast<real>(s), pt, dp, tm);
        break;
      }
      s_prev = s;
      fp_prev = fp;
      s = sn;
    }
    const double tau = s * tau_rem;
    // ---- jump (MCWF step 4) ----
    tm.sync();
    store_lds(T[0], pt, tm);
    tm.sync();
    const double x = st.x;
    int lsel = -1;
    double wsel = 0.0;
    cx<real> y[R];
    if (a.n_jump == 1) {  // one operator: its weight only has to be non-zero
      apply_jump<real, R, G>(a, 0, T[0], y, tm);
      wsel = norm2(y, tm);
      if (wsel > 0.0) lsel = 0;
    } else {
      // weights ||L_l p||^2; pass 1 sums them, pass 2 walks the cumulative sum
      double total = 0.0;
      for (int l = 0; l < a.n_jump; ++l) {
        apply_jump<real, R, G>(a, l, T[0], y, tm);
        total += norm2(y, tm);
      }
      if (total > 0.0) {
        const double target = x * total;
        double acc = 0.0;
        for (int l = 0; l < a.n_jump; ++l) {
          apply_jump<real, R, G>(a, l, T[0], y, tm);
          wsel = norm2(y, tm);
          acc += wsel;
          if (target < acc) {
            lsel = l;
            break;
          }
        }
        if (lsel < 0) {  // rounding left target >= total: take the last operator
          lsel = a.n_jump - 1;
          apply_jump<real, R, G>(a, lsel, T[0], y, tm);
          wsel = norm2(y, tm);
        }
      }
    }
    if (lsel < 0) {
      if (tm.leader()) {
        atomicOr(a.err, kErrNoJumpWeight);
        if (static_cast<long long>(slot) < a.rec_cap) a.rec[slot].op = -1;  // no jump took place
      }
#pragma unroll
      for (int m = 0; m < R; ++m) psi[m] = pt[m];
      st.nrm2 = norm2(pt, tm);
      st.r = 0.0;
      tm.sync();
      return;
    }
    tm.sync();
    const real inv = static_cast<real>(1.0 / sqrt(wsel));
#pragma unroll
    for (int m = 0; m < R; ++m) ps[m] = cx<real>{y[m].x * inv, y[m].y * inv};
    const double elapsed = (h - tau_rem) + tau;
    if (tm.leader()) {
      if (static_cast<long long>(slot) < a.rec_cap) {
        tk_jump r;
        r.instance = static_cast<int32_t>(a.instance);
        r.traj = k;
        r.step = j;
        r.op = lsel;
        r.ordinal = st.ordinal;
        r.direction = DIR;
        r.iteration = static_cast<int32_t>(rng.iteration);
        r.reserved = 0;
        r.t = DIR == 0 ? t0 + elapsed : t0 - elapsed;
        a.rec[slot] = r;
      }
    }
    st.ordinal += 1;
    rng.draw(static_cast<uint64_t>(st.ordinal), st);
    n_s = -1.0;  // ||ps||^2 is reduced only if another jump falls in this substep
    tau_rem = tau_rem - tau;
    const int Kr = taylor_order(a, bnd * tau_rem, Kc);
    if (Kr >= 1 && Kr < Kc) Kc = Kr;
  }
}

struct StepPlan {
  int n_sub;   // substeps per step
  int K;       // Taylor order of a substep
  double h;    // substep length
  double bnd;  // bound on ||H_eff|| of the step
};

// Substeps and polynomial order of step j from the norm bound of its H_eff:
// enough substeps that ||H_eff|| h <= kMaxStepNorm and that the order fits the
// kbuf - 1 term vectors in LDS.  `hint` carries the previous step's order.
template <int N>
__device__ __forceinline__ StepPlan plan_step(const PassArgs &a, const double (&uj)[N],
                                              OrderHint &hint) {
  double b = a.b0;
#pragma unroll
  for (int i = 0; i < N; ++i) b += fabs(uj[i]) * a.bc[i];
  const double x = b * a.dt;
  StepPlan p;
  p.bnd = b;
  const int kfit = a.kbuf - 1;  // largest order whose terms fit the LDS
  p.n_sub = x > kMaxStepNorm ? static_cast<int>(ceil(x / kMaxStepNorm)) : 1;
  p.K = hint.order(a, p.n_sub == 1 ? x : x / static_cast<double>(p.n_sub));
  while ((p.K < 0 || p.K > kfit) && p.n_sub < kMaxSubsteps) {
    p.n_sub += 1;
    p.K = taylor_order(a, x / static_cast<double>(p.n_sub), kfit);
  }
  if (p.K < 0 || p.K > kfit) {
    atomicOr(a.err, kErrTaylorOrder);
    p.K = kfit;
  }
  p.h = p.n_sub == 1 ? a.dt : a.dt / static_cast<double>(p.n_sub);
  return p;
}

// Advance across the whole step j (its substeps).  FT: with use_y1 set, *y1
// is the first series term's product Op psi of the step's first substep.
template <typename real, int R, int WS, int NC, int G, int DIR, bool KEEP = false, bool FT = false>
__device__ __forceinline__ void advance_step(const LaneOp<real, R, WS, NC, G> &op,
                                             const PassArgs &a, const Terms<real, R, G> &T,
                                             cx<real> (&psi)[R], TrajMeta &st,
                                             const Stream &rng, int j, const StepPlan &p,
                                             int k, const Team<G> &tm,
                                             const cx<real> (*y1)[R] = nullptr,
                                             bool use_y1 = false) {
  for (int s = 0; s < p.n_sub; ++s) {
    const double t0 = DIR == 0 ? static_cast<double>(j) * a.dt + s * p.h
                               : static_cast<double>(j + 1) * a.dt - s * p.h;
    advance<real, R, WS, NC, G, DIR, KEEP, FT>(op, a, T, psi, st, rng, j, t0, p.h, p.K, p.bnd, k,
                                               tm, y1, use_y1 && s == 0);
  }
}

// Block prologue shared by the kernels: copy the unscaled control slots to LDS
// (one copy per block of one-wave teams; a G-wave team reads them from global
// memory, where they are few and cached, to leave its LDS to the term
// vectors), zero the trailing element of this team's term vectors, load the
// lane's operator slice.  `team` is the team's index in the block and
// team_bytes its share of LDS.  Returns the team's term vectors.
template <typename real, int R, int WS, int NC, int G>
__device__ __forceinline__ Terms<real, R, G> block_setup(const PassArgs &a, unsigned char *smem,
                                                         int team, const Team<G> &tm,
                                                         size_t team_bytes,
                                                         LaneOp<real, R, WS, NC, G> &op) {
  constexpr int NCX = NC > 0 ? NC : 1;
  constexpr int kL = Team<G>::kLanes;
  const cx<real> *cval_g = static_cast<const cx<real> *>(a.cval);
  const cx<real> *cval_src = cval_g;
  size_t cval_bytes = 0;
  if (G == 1) {
    cx<real> *cval_lds = reinterpret_cast<cx<real> *>(smem);
    for (int i = threadIdx.x; i < NCX * R * kL; i += blockDim.x) cval_lds[i] = cval_g[i];
    cval_src = cval_lds;
    cval_bytes = sizeof(cx<real>) * NCX * R * kL;
  }
  Terms<real, R, G> T;
  T.base = reinterpret_cast<cx<real> *>(smem + cval_bytes + static_cast<size_t>(team) * team_bytes);
  if (tm.gl < a.kbuf) T[tm.gl][R * kL] = cx<real>{0, 0};
  __syncthreads();
  op.load(a.scol, a.sval, a.sdiag, a.ccol, cval_src, tm.gl);
  op.bind(T[0]);
  return T;
}

template <typename real, int R, int G>
__device__ __forceinline__ size_t terms_bytes(int kbuf) {
  return static_cast<size_t>(kbuf) * Terms<real, R, G>::kLen * sizeof(cx<real>);
}

// One trajectory of a plain pass over all nt steps: DIR 0 forward from
// psi_start (final normalised state and tau_k = <tgt|psi_hat_k(T)>), DIR 1
// backward from the target, storing chi_k(t_j) = tau_k chi_hat_k(t_j).
// chi_k(t_j) = tau_k psi / ||psi|| for the rows < d (costate layout [M][d]
// at `out`, the trajectory's row).
template <typename real, int R, int G>
__device__ __forceinline__ void store_costate(cx<real> *out, int d, const cx<real> (&psi)[R],
                                              double nrm2, double tau_re, double tau_im,
                                              const Team<G> &tm) {
  const double inv = 1.0 / sqrt(nrm2);
#pragma unroll
  for (int m = 0; m < R; ++m) {
    const int row = tm.gl + Team<G>::kLanes * m;
    if (row < d) {
      const double px = psi[m].x * inv, py = psi[m].y * inv;
      gst(out, row, cx<real>{static_cast<real>(tau_re * px - tau_im * py),
                          static_cast<real>(tau_re * py + tau_im * px)});
    }
  }
}

template <typename real, int R, int WS, int NC, int G, int DIR>
__device__ void pass_trajectory(LaneOp<real, R, WS, NC, G> &op, const PassArgs &a,
                                const Terms<real, R, G> &T, int k, const Stream &rng, const Team<G> &tm) {
  const cx<real> *start = static_cast<const cx<real> *>(a.psi_start);
  cx<real> *chi = static_cast<cx<real> *>(a.chi);
  cx<real> psi[R];
#pragma unroll
  for (int m = 0; m < R; ++m) psi[m] = gld(start, tm.gl + Team<G>::kLanes * m);
  TrajMeta st;
  st.nrm2 = norm2(psi, tm);
  st.ordinal = 0;
  st.pad = 0;
  rng.draw(0, st);
  double tau_re = 0.0, tau_im = 0.0;
  if (DIR == 1) {
    tau_re = gmem(a.tau_in)[2 * k];
    tau_im = gmem(a.tau_in)[2 * k + 1];
  }
  constexpr int NCX = NC > 0 ? NC : 1;
  double un[NCX];  // pulses of the next step, loaded one step ahead (rows padded)
  {
    const int j0 = DIR == 0 ? 0 : a.nt - 1;
#pragma unroll
    for (int i = 0; i < NCX; ++i) un[i] = gmem(a.u)[static_cast<size_t>(i) * a.nt + j0];
  }
  OrderHint khint;
  for (int jj = 0; jj < a.nt; ++jj) {
    const int j = DIR == 0 ? jj : a.nt - 1 - jj;
    double uj[NCX];
#pragma unroll
    for (int i = 0; i < NCX; ++i) uj[i] = un[i];
    if (jj + 1 < a.nt) {
      const int jn = DIR == 0 ? j + 1 : j - 1;
#pragma unroll
      for (int i = 0; i < NCX; ++i) un[i] = gmem(a.u)[static_cast<size_t>(i) * a.nt + jn];
    }
    op.set_pulses(uj, a.wc);
    const StepPlan p = plan_step(a, uj, khint);
    advance_step<real, R, WS, NC, G, DIR>(op, a, T, psi, st, rng, j, p, k, tm);
    if (DIR == 1 && a.seg_len == 0)
      store_costate<real, R, G>(chi + (static_cast<size_t>(j) * a.M + k) * a.d, a.d, psi,
                                st.nrm2, tau_re, tau_im, tm);
    if (DIR == 1 && a.seg_len > 0 && j % a.seg_len == 0 && j > 0) {
      // checkpoint: the state at t_j, where segment j / seg_len - 1 ends
      const size_t c = static_cast<size_t>(j / a.seg_len - 1) * a.M + k;
      cx<real> *ck = static_cast<cx<real> *>(a.ck_psi) + c * R * Team<G>::kLanes;
#pragma unroll
      for (int m = 0; m < R; ++m) gst(ck, tm.gl + Team<G>::kLanes * m, psi[m]);
      if (tm.leader()) gst(a.ck_meta, c, st);
    }
  }
  if (DIR == 0) {
    const double inv = 1.0 / sqrt(st.nrm2);
    double tr = 0.0, ti = 0.0;
    cx<real> *psiT = static_cast<cx<real> *>(a.psiT);
#pragma unroll
    for (int m = 0; m < R; ++m) {
      const int row = tm.gl + Team<G>::kLanes * m;
      const double px = psi[m].x * inv, py = psi[m].y * inv;
      // tau_k = <tgt|psi_hat> = sum conj(tgt) psi_hat
      const double gx = gmem(a.tgt)[2 * row], gy = gmem(a.tgt)[2 * row + 1];
      tr = fma(gx, px, fma(gy, py, tr));
      ti = fma(gx, py, fma(-gy, px, ti));
      if (psiT != nullptr && row < a.d)
        gst(psiT, static_cast<size_t>(k) * a.d + row,
            cx<real>{static_cast<real>(px), static_cast<real>(py)});
    }
    tr = tm.sum(tr);
    ti = tm.sum(ti);
    if (tm.leader() && a.tau_out != nullptr) {
      gmem(a.tau_out)[2 * k] = tr;
      gmem(a.tau_out)[2 * k + 1] = ti;
    }
  }
}

// Per-lane share of Im <chi|H_i|psi_hat> for every control slot c, added to
// pc.  The (unnormalised) state is in term vector 0, where the gathers are
// bound; inv = 1/||psi||.
template <typename real, int R, int WS, int NC, int G>
__device__ __forceinline__ void krotov_share(const LaneOp<real, R, WS, NC, G> &op,
                                             const cx<real> (&ch)[R], double inv, double *pc) {
#pragma unroll
  for (int m = 0; m < R; ++m) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const cx<real> q = op.cval_at(c, m);
      const cx<real> b = op.cp[c][m][0];
      const double hx = static_cast<double>(q.x) * b.x - static_cast<double>(q.y) * b.y;
      const double hy = static_cast<double>(q.x) * b.y + static_cast<double>(q.y) * b.x;
      // Im(conj(chi) h) = chi.x h.y - chi.y h.x
      pc[c] = fma(inv * static_cast<double>(ch[m].x), hy, pc[c]);
      pc[c] = fma(-inv * static_cast<double>(ch[m].y), hx, pc[c]);
    }
  }
}

// The parts of the next step's first series term that do not depend on the
// pulses, from the state in term vector 0 (which the share has just gathered
// from; own = the lane's rows of it): ys = the diagonal's and the static
// slots' multiply-adds, in slot order; bc = the control
// slots' gathered elements.  first_term_finish adds the control slots'
// multiply-adds once the pulses are known: the same operations in the same
// order as series_term's gathered term, so the result is the same to the bit.
template <typename real, int R, int WS, int NC, int G>
__device__ __forceinline__ void first_term_parts(const LaneOp<real, R, WS, NC, G> &op,
                                                 const cx<real> (&own)[R], cx<real> (&ys)[R],
                                                 cx<real> (&bc)[NC > 0 ? NC : 1][R]) {
  using Op = LaneOp<real, R, WS, NC, G>;
  constexpr int W0 = Op::W0;
  cx<real> b[W0][R];
#pragma unroll
  for (int s = 0; s < W0; ++s)
#pragma unroll
    for (int m = 0; m < R; ++m)
      if (Op::live(s, m)) b[s][m] = op.sp[s][m][0];
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int m = 0; m < R; ++m) bc[c][m] = op.cp[c][m][0];
#pragma unroll
  for (int m = 0; m < R; ++m) {
    ys[m] = cx<real>{0, 0};
    cfma(ys[m], op.dval[m], own[m]);
  }
#pragma unroll
  for (int s = 0; s < W0; ++s)
#pragma unroll
    for (int m = 0; m < R; ++m)
      if (Op::live(s, m)) Op::sfma(ys[m], op.sval[s][m], b[s][m], s, m);
}

template <typename real, int R, int WS, int NC, int G>
__device__ __forceinline__ void first_term_finish(const LaneOp<real, R, WS, NC, G> &op,
                                                  const cx<real> (&ys)[R],
                                                  const cx<real> (&bc)[NC > 0 ? NC : 1][R],
                                                  cx<real> (&y)[R]) {
#pragma unroll
  for (int m = 0; m < R; ++m) y[m] = ys[m];
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int m = 0; m < R; ++m)
      cfma_ctrl<LaneOp<real, R, WS, NC, G>::RC>(y[m], op.cv[c][m], bc[c][m]);
}

// chi_k(t_j), own rows.  Padding rows (row >= d) read row d - 1 instead of a
// zero: they only ever multiply (H_i psi) rows that are exactly zero, and an
// unconditional load needs no wait for the previous step's loads into ch.
template <typename real, int R, int G>
__device__ __forceinline__ void load_costate(const PassArgs &a, int j, int k, const Team<G> &tm,
                                             cx<real> (&ch)[R]) {
  const cx<real> *chi = static_cast<const cx<real> *>(a.chi);
  const size_t base = (static_cast<size_t>(j) * a.M + k) * a.d;
#pragma unroll
  for (int m = 0; m < R; ++m) {
    const int row = tm.gl + Team<G>::kLanes * m;
    ch[m] = gld(chi, base + (row < a.d ? row : a.d - 1));
  }
}


// ---- grid-wide exchange of the sequential Krotov passes ----------------------
// One batch of agent-scope loads of the slots of blocks lane + 64 q.
template <int NCX>
__device__ __forceinline__ void poll_slots(const unsigned long long *row, int lane,
                                           unsigned long long (&bits)[kPollPerLane][NCX]) {
#pragma unroll
  for (int q = 0; q < kPollPerLane; ++q)
#pragma unroll
    for (int c = 0; c < NCX; ++c)
      bits[q][c] = __hip_atomic_load(&row[(lane + kWave * q) * NCX + c], __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT);
}

// True when every slot of a batch holds a partial; then acc = their sum per
// lane (in the batch's fixed order).
template <int NCX>
__device__ __forceinline__ bool slots_complete(const unsigned long long (&bits)[kPollPerLane][NCX],
                                               double (&acc)[NCX]) {
  int missing = 0;
#pragma unroll
  for (int q = 0; q < kPollPerLane; ++q)
#pragma unroll
    for (int c = 0; c < NCX; ++c) missing |= bits[q][c] == kSlotEmpty;
  if (__any(missing)) return false;
#pragma unroll
  for (int c = 0; c < NCX; ++c) {
    acc[c] = 0.0;
#pragma unroll
    for (int q = 0; q < kPollPerLane; ++q)
      acc[c] += __longlong_as_double(static_cast<long long>(bits[q][c]));
  }
  return true;
}


}  // namespace
}  // namespace tk
