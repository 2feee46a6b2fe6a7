// Host driver of the batched form: many independent optimisation instances,
// each a full problem (system, states, pulses, M, seed), advanced together.
//
// Every instance is held by a context of its own (operator packing, pulses and
// per-instance buffers come from the single-system code); the batch adds the
// buffers of the batched Krotov pass, the instance table the kernels read,
// the launch plan, an autotuner for the tile shapes and a HIP graph that
// replays one Krotov iteration of every instance.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "tk_host_internal.h"
#include "tk_internal.h"

using namespace tkh;

namespace {

struct Member {
  tk_ctx *c = nullptr;
  uint32_t id = 0;  // instance index in the random streams' key
  int M = 0;
  uint64_t seed = 0;
  int variant = -1;  // index among the kernel shapes of the precision
  int kbuf_fw = 0, kbuf_bw = 0;
  double step_cost = 0.0;  // model of one trajectory-step (relative units)
  int G = 1;               // waves per trajectory of its shape
  DevBuf psi, meta, tslots;
  DevBuf seg, ck_psi, ck_meta;  // multi-wave shapes: costate segment and checkpoints
  DevBuf tau_save;              // the overlaps the multi-wave Krotov pass starts from
  ~Member() {
    if (c) tk_destroy(c);
  }
};

struct LaunchPlan {
  int pass_wpb = 0, kro_wpb = 0;  // waves per block of the one-wave launches
  std::vector<int> nblocks;       // Krotov blocks per entry of narrow
};

// One-wave instances of one kernel shape: kernels of their own (compiled for
// that shape alone), launched one shape after another.
struct NarrowGroup {
  int S = 0;                   // shape index
  size_t q0 = 0, q1 = 0;       // their entries in narrow
  int item0 = 0, n_items = 0;  // their range of the one-wave work list
  int pass_blocks = 0, kro_blocks = 0, kro_block0 = 0;
  size_t pass_lds = 0, kro_lds = 0;
};

// Instances of one multi-wave team size: kernels of their own, one team per
// block, blocks split by the cost model.
struct WideClass {
  int G = 0;
  std::vector<int> idx;  // member indices
  const void *pass_fw = nullptr, *pass_bw = nullptr, *krotov = nullptr;
  DevBuf items_dev, block_inst_dev;
  int n_items = 0, pass_blocks = 0, kro_blocks = 0, kro_capacity = 0;
  size_t lds = 0;
  std::vector<int> nblocks;  // per entry of idx
};

}  // namespace

struct tk_batch {
  int device = 0;
  int precision = TK_FP64;
  hipStream_t stream = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  std::string err;
  int n_cu = 0;
  std::vector<std::unique_ptr<Member>> mem;
  std::vector<int> narrow;       // members of one-wave shapes, grouped by shape
  std::vector<NarrowGroup> groups;
  std::vector<std::unique_ptr<WideClass>> wide;  // members of multi-wave shapes, by team size
  tk::BatchKernels kern{};
  bool ready = false;
  uint64_t next_iter = 0;  // iteration the next call starts with
  LaunchPlan plan;
  bool tuned = false;
  DevBuf inst_dev, items_dev, block_inst_dev, iter_dev, J_hist_dev, err_dev, rec_dev, rec_count_dev;
  DevBuf t_begin_dev, t_end_dev;  // launch start and per-instance finish (constant clock)
  double clock_khz = 0.0;         // rate of that clock
  std::vector<tk::BatchInstance> inst;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  double last_iter_ms = 0.0, tuned_pass_ms = 0.0, tuned_krotov_ms = 0.0, tuned_wide_krotov_ms = 0.0;
  int64_t traj_steps = 0;
};

namespace {

int bfail(tk_batch *b, int code, const std::string &msg) {
  if (b) b->err = msg;
  return code;
}

int bhip(tk_batch *b, hipError_t e, const char *what) {
  return bfail(b, e == hipErrorOutOfMemory ? TK_ENOMEM : TK_EHIP,
               std::string(what) + ": " + hipGetErrorString(e));
}

#define TK_BHIP(b, call)                              \
  do {                                                \
    hipError_t e_ = (call);                           \
    if (e_ != hipSuccess) return bhip(b, e_, #call);  \
  } while (0)

int shape_index(const tk::Variant *v) {
  return tk::batch_shape_index(v->precision, v->R, v->ws_code, v->NC, v->G);
}

size_t cplx_bytes(int precision) { return precision == TK_FP64 ? 16 : 8; }

constexpr size_t kLaunchSlots = 16;  // start-time slots of the Krotov launches

// LDS bytes per wave of the batched plain passes for member m
size_t pass_wave_lds(const tk_batch *b, const Member &m) {
  const tk::Variant &v = *m.c->var;
  const size_t ncx = v.NC > 0 ? v.NC : 1;
  const size_t kb = std::max(m.kbuf_fw, m.kbuf_bw);
  const size_t bytes =
      (ncx * v.R * tk::kWave + kb * (v.R * tk::kWave + 1)) * cplx_bytes(b->precision);
  return (bytes + 15) / 16 * 16;
}

// Krotov blocks per instance of `idx`: every instance gets one, then blocks go
// one at a time to the instance with the longest estimated pass,
//   nt (ceil(M / (blocks * wpb)) cost + sync_cost),
// until `capacity` blocks are given out or the longest cannot gain.  `cost` is
// the time of one trajectory-step per member (measured), or null for the
// model m.step_cost.  Returns the blocks per entry of idx.
std::vector<int> split_blocks(const tk_batch *b, const std::vector<int> &idx, int capacity,
                              int wpb, double sync_cost, const std::vector<double> *cost) {
  const size_t n = idx.size();
  std::vector<int> nb(n, 1);
  auto est = [&](size_t q) {
    const Member &m = *b->mem[idx[q]];
    const double tw = std::ceil(static_cast<double>(m.M) / (static_cast<double>(nb[q]) * wpb));
    return m.c->nt * (tw * (cost ? (*cost)[idx[q]] : m.step_cost) + sync_cost);
  };
  int used = static_cast<int>(n);
  while (used < capacity && n > 0) {
    size_t worst = 0;
    for (size_t q = 1; q < n; ++q)
      if (est(q) > est(worst)) worst = q;
    const Member &m = *b->mem[idx[worst]];
    if (nb[worst] >= tk::kMaxBlocks || static_cast<int64_t>(nb[worst]) * wpb >= m.M) break;
    nb[worst]++;
    used++;
  }
  return nb;
}

// Block map of one Krotov launch: the blocks of member idx[q] are nb[q]
// consecutive blocks; sets block0 / nblocks of those members.
int upload_block_map(tk_batch *b, const std::vector<int> &idx, const std::vector<int> &nb,
                     DevBuf &dev, int *n_blocks) {
  std::vector<int> block_inst;
  for (size_t q = 0; q < idx.size(); ++q) {
    b->inst[idx[q]].block0 = static_cast<int>(block_inst.size());
    b->inst[idx[q]].nblocks = nb[q];
    for (int r = 0; r < nb[q]; ++r) block_inst.push_back(idx[q]);
  }
  *n_blocks = static_cast<int>(block_inst.size());
  if (block_inst.empty()) return TK_OK;
  TK_BHIP(b, dev.ensure(block_inst.size() * sizeof(int)));
  TK_BHIP(b, hipMemcpy(dev.p, block_inst.data(), block_inst.size() * sizeof(int),
                       hipMemcpyHostToDevice));
  return TK_OK;
}

// Instance table and the Krotov block maps of the current plans.
int upload_tables(tk_batch *b) {
  const size_t n = b->mem.size();
  if (b->plan.nblocks.size() == b->narrow.size()) {
    // one-wave instances: one launch per shape, block0 relative to the launch
    std::vector<int> block_inst;
    for (auto &g : b->groups) {
      g.kro_block0 = static_cast<int>(block_inst.size());
      for (size_t q = g.q0; q < g.q1; ++q) {
        const int i = b->narrow[q];
        b->inst[i].block0 = static_cast<int>(block_inst.size()) - g.kro_block0;
        b->inst[i].nblocks = b->plan.nblocks[q];
        for (int r = 0; r < b->plan.nblocks[q]; ++r) block_inst.push_back(i);
      }
      g.kro_blocks = static_cast<int>(block_inst.size()) - g.kro_block0;
    }
    if (!block_inst.empty()) {
      TK_BHIP(b, b->block_inst_dev.ensure(block_inst.size() * sizeof(int)));
      TK_BHIP(b, hipMemcpy(b->block_inst_dev.p, block_inst.data(),
                           block_inst.size() * sizeof(int), hipMemcpyHostToDevice));
    }
  }
  int rc = TK_OK;
  for (auto &w : b->wide)
    if ((rc = upload_block_map(b, w->idx, w->nblocks, w->block_inst_dev, &w->kro_blocks))) return rc;
  TK_BHIP(b, b->inst_dev.ensure(n * sizeof(tk::BatchInstance)));
  TK_BHIP(b, hipMemcpy(b->inst_dev.p, b->inst.data(), n * sizeof(tk::BatchInstance),
                       hipMemcpyHostToDevice));
  return TK_OK;
}

tk::BatchArgs batch_args(tk_batch *b) {
  tk::BatchArgs a;
  std::memset(&a, 0, sizeof(a));
  a.inst = b->inst_dev.as<tk::BatchInstance>();
  a.n_inst = static_cast<int>(b->mem.size());
  a.items = b->items_dev.as<int2>();
  a.block_inst = b->block_inst_dev.as<int>();
  a.iteration = b->iter_dev.as<uint64_t>();
  a.J_hist = b->J_hist_dev.as<double>();
  a.t_begin = b->t_begin_dev.as<unsigned long long>();
  a.t_end = b->t_end_dev.as<unsigned long long>();
  a.err = b->err_dev.as<int>();
  a.spin_limit = 1ll << 22;
  return a;
}

tk::BatchArgs wide_args(tk_batch *b, WideClass &w) {
  tk::BatchArgs a = batch_args(b);
  a.witems = w.items_dev.as<int2>();
  a.n_witems = w.n_items;
  a.wblock_inst = w.block_inst_dev.as<int>();
  return a;
}

// LDS bytes a kernel declares statically (beside its dynamic LDS).
size_t static_lds(const void *kernel) {
  hipFuncAttributes fa;
  if (hipFuncGetAttributes(&fa, kernel) != hipSuccess) return tk::kLdsBytes;
  return fa.sharedSizeBytes;
}

// Pass plan with `wpb` waves per block: per shape, as many blocks as are
// co-resident (the shapes' launches run one after another).
int plan_pass(tk_batch *b, int wpb) {
  for (auto &g : b->groups) {
    size_t wl = 0;
    for (size_t q = g.q0; q < g.q1; ++q) wl = std::max(wl, pass_wave_lds(b, *b->mem[b->narrow[q]]));
    const size_t lds = wl * wpb;
    if (lds > tk::kLdsBytes) return TK_EUNSUPPORTED;
    int occ = 1 << 30;
    for (const void *k : {b->kern.pass_fw[g.S], b->kern.pass_bw[g.S]}) {
      TK_BHIP(b, hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     static_cast<int>(lds)));
      int o = 0;
      TK_BHIP(b, hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, k, tk::kWave * wpb, lds));
      occ = std::min(occ, o);
    }
    if (occ < 1) return TK_EUNSUPPORTED;
    const int64_t blocks =
        std::min<int64_t>(static_cast<int64_t>(occ) * b->n_cu, (g.n_items + wpb - 1) / wpb);
    g.pass_lds = lds;
    g.pass_blocks = static_cast<int>(std::max<int64_t>(blocks, 1));
  }
  b->plan.pass_wpb = wpb;
  return TK_OK;
}

// Krotov plan with `wpb` waves per block and a fraction of the co-resident blocks.
// Per shape, the launch's co-resident blocks are split among its instances.
int plan_krotov(tk_batch *b, int wpb, double frac, double sync_cost,
                const std::vector<double> *cost = nullptr) {
  std::vector<int> nb(b->narrow.size(), 0);
  for (auto &g : b->groups) {
    size_t lds = 0;
    for (size_t q = g.q0; q < g.q1; ++q) {
      const Member &m = *b->mem[b->narrow[q]];
      lds = std::max(lds, tk::block_lds_bytes(*m.c->var, wpb, m.kbuf_fw, 0));
    }
    const void *k = b->kern.krotov[g.S];
    if (lds + static_lds(k) > tk::kLdsBytes) return TK_EUNSUPPORTED;
    TK_BHIP(b, hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   static_cast<int>(lds)));
    int occ = 0;
    TK_BHIP(b, hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k, tk::kWave * wpb, lds));
    const int capacity = static_cast<int>(frac * occ * b->n_cu);
    if (capacity < static_cast<int>(g.q1 - g.q0)) return TK_EUNSUPPORTED;
    g.kro_lds = lds;
    const std::vector<int> idx(b->narrow.begin() + g.q0, b->narrow.begin() + g.q1);
    const std::vector<int> part = split_blocks(b, idx, capacity, wpb, sync_cost, cost);
    std::copy(part.begin(), part.end(), nb.begin() + g.q0);
  }
  b->plan.kro_wpb = wpb;
  b->plan.nblocks = nb;
  return upload_tables(b);
}

// Plans of a multi-wave class: one team per block; the pass takes as many
// co-resident blocks as there is work, the Krotov pass splits the co-resident
// blocks by the cost model.
int plan_wide(tk_batch *b, WideClass &w) {
  size_t lds = 0;
  for (int i : w.idx) {
    const Member &m = *b->mem[i];
    lds = std::max(lds, tk::block_lds_bytes(*m.c->var, 1, std::max(m.kbuf_fw, m.kbuf_bw), 0));
  }
  if (lds + static_lds(w.krotov) > tk::kLdsBytes)
    return bfail(b, TK_EUNSUPPORTED, "team term vectors do not fit in LDS");
  w.lds = lds;
  int occ = tk::kLdsBytes;
  for (const void *k : {w.pass_fw, w.pass_bw, w.krotov}) {
    TK_BHIP(b, hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   static_cast<int>(lds)));
    int o = 0;
    TK_BHIP(b, hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, k, tk::kWave * w.G, lds));
    occ = std::min(occ, o);
  }
  if (occ < 1) return bfail(b, TK_EUNSUPPORTED, "team kernels do not fit a compute unit");
  const int capacity = occ * b->n_cu;
  if (capacity < static_cast<int>(w.idx.size()))
    return bfail(b, TK_EUNSUPPORTED, "instances do not fit one co-resident grid");
  w.pass_blocks = std::max(1, std::min(capacity, w.n_items));
  w.kro_capacity = capacity;
  w.nblocks = split_blocks(b, w.idx, capacity, 1, 0.0, nullptr);
  return TK_OK;
}

// which: 0 every instance, 1 one-wave instances only
int launch_pass(tk_batch *b, int dir, int which = 0) {
  for (const auto &g : b->groups) {
    tk::BatchArgs a = batch_args(b);
    a.items = b->items_dev.as<int2>() + g.item0;
    a.n_items = g.n_items;
    a.wave_lds = static_cast<int>(g.pass_lds / b->plan.pass_wpb);
    void *args[] = {&a};
    TK_BHIP(b, hipLaunchKernel(dir == 0 ? b->kern.pass_fw[g.S] : b->kern.pass_bw[g.S],
                               dim3(g.pass_blocks), dim3(tk::kWave * b->plan.pass_wpb), args,
                               g.pass_lds, b->stream));
  }
  for (auto &wp : b->wide) {
    if (which == 1) break;
    WideClass &w = *wp;
    tk::BatchArgs a = wide_args(b, w);
    void *args[] = {&a};
    TK_BHIP(b, hipLaunchKernel(dir == 0 ? w.pass_fw : w.pass_bw, dim3(w.pass_blocks),
                               dim3(tk::kWave * w.G), args, w.lds, b->stream));
  }
  return TK_OK;
}

// which: 0 every instance, 1 one-wave instances only, 2 multi-wave ones only
int launch_krotov(tk_batch *b, int which = 0) {
  tk::BatchArgs a = batch_args(b);
  void *args[] = {&a};
  TK_BHIP(b, hipLaunchKernel(b->kern.fill, dim3(static_cast<unsigned>(b->mem.size())), dim3(256),
                             args, 0, b->stream));
  // the blocks of each launch are co-resident by the occupancy check of the
  // plan; a block that waits past the spin limit aborts the pass with an error
  // instead of hanging.  Each launch takes its own start-time slot.
  unsigned long long *t_begin = b->t_begin_dev.as<unsigned long long>();
  for (size_t gi = 0; gi < b->groups.size() && which != 2; ++gi) {
    const NarrowGroup &g = b->groups[gi];
    tk::BatchArgs ga = batch_args(b);
    ga.block_inst = b->block_inst_dev.as<int>() + g.kro_block0;
    ga.t_begin = t_begin + gi;
    void *gargs[] = {&ga};
    TK_BHIP(b, hipLaunchKernel(b->kern.krotov[g.S], dim3(g.kro_blocks),
                               dim3(tk::kWave * b->plan.kro_wpb), gargs, g.kro_lds, b->stream));
  }
  for (size_t wi = 0; wi < b->wide.size(); ++wi) {
    if (which == 1) break;
    WideClass &w = *b->wide[wi];
    tk::BatchArgs wa = wide_args(b, w);
    wa.t_begin = t_begin + b->groups.size() + wi;
    void *wargs[] = {&wa};
    TK_BHIP(b, hipLaunchKernel(w.krotov, dim3(w.kro_blocks), dim3(tk::kWave * w.G), wargs, w.lds,
                               b->stream));
  }
  return TK_OK;
}

int launch_tail(tk_batch *b, int copy_pulses) {
  tk::BatchArgs a = batch_args(b);
  void *args[] = {&a};
  const dim3 grid(static_cast<unsigned>(b->mem.size()));
  TK_BHIP(b, hipLaunchKernel(b->kern.functional, grid, dim3(256), args, 0, b->stream));
  int cp = copy_pulses;
  void *fargs[] = {&a, &cp};
  TK_BHIP(b, hipLaunchKernel(b->kern.finish, grid, dim3(256), fargs, 0, b->stream));
  return TK_OK;
}

int check_errors(tk_batch *b) {
  int e = 0;
  TK_BHIP(b, hipMemcpyAsync(&e, b->err_dev.p, sizeof(int), hipMemcpyDeviceToHost, b->stream));
  TK_BHIP(b, hipStreamSynchronize(b->stream));
  if (e & tk::kErrSyncTimeout)
    return bfail(b, TK_EHIP, "per-step reduction timed out (blocks not co-resident)");
  if (e & tk::kErrNoJumpWeight) return bfail(b, TK_ENUMERIC, "jump with all ||L_l psi||^2 = 0");
  if (e & tk::kErrTaylorOrder)
    return bfail(b, TK_ENUMERIC, "time step too long for the polynomial propagator");
  if (e & tk::kErrJumpLoop) return bfail(b, TK_ENUMERIC, "too many jumps inside one time step");
  return TK_OK;
}

// Elapsed milliseconds of what `fn` enqueues on the batch stream.
template <typename F>
int timed(tk_batch *b, F fn, double *ms) {
  TK_BHIP(b, hipEventRecord(b->ev0, b->stream));
  int rc = fn();
  if (rc) return rc;
  TK_BHIP(b, hipEventRecord(b->ev1, b->stream));
  TK_BHIP(b, hipEventSynchronize(b->ev1));
  float f = 0.f;
  TK_BHIP(b, hipEventElapsedTime(&f, b->ev0, b->ev1));
  *ms = f;
  return TK_OK;
}

// Allocations, instance table and work list (first iteration call).
int finalize(tk_batch *b) {
  const size_t n = b->mem.size();
  if (n == 0) return bfail(b, TK_ESTATE, "batch has no instances");
  b->kern = tk::batch_kernels(b->precision);
  TK_BHIP(b, b->iter_dev.ensure(sizeof(uint64_t)));
  TK_BHIP(b, b->J_hist_dev.ensure(n * tk::kBatchHistory * sizeof(double)));
  TK_BHIP(b, b->err_dev.ensure(sizeof(int)));
  TK_BHIP(b, b->rec_dev.ensure(sizeof(tk_jump)));
  TK_BHIP(b, b->rec_count_dev.ensure(sizeof(unsigned long long)));
  // start-time slots: one per Krotov launch (one-wave shapes, then team sizes)
  TK_BHIP(b, b->t_begin_dev.ensure(kLaunchSlots * sizeof(unsigned long long)));
  TK_BHIP(b, b->t_end_dev.ensure(n * sizeof(unsigned long long)));
  {
    int khz = 0;
    TK_BHIP(b, hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, b->device));
    b->clock_khz = khz;
  }
  TK_BHIP(b, hipMemset(b->err_dev.p, 0, sizeof(int)));
  TK_BHIP(b, hipMemset(b->rec_count_dev.p, 0, sizeof(unsigned long long)));
  b->inst.assign(n, tk::BatchInstance{});
  b->traj_steps = 0;
  b->narrow.clear();
  b->groups.clear();
  b->wide.clear();
  std::vector<std::pair<double, int2>> items[tk::kBatchShapes];
  std::vector<std::vector<std::pair<double, int2>>> witems;
  for (size_t i = 0; i < n; ++i) {
    Member &m = *b->mem[i];
    tk_ctx *c = m.c;
    const tk::Variant &v = *c->var;
    m.G = v.G;
    const size_t cb = cplx_bytes(b->precision);
    const size_t vec = static_cast<size_t>(v.R) * tk::kWave * v.G * cb;
    const int ncx = v.NC > 0 ? v.NC : 1;
    size_t wc = 0;  // class of the member among the multi-wave ones
    if (v.G == 1) {
      b->narrow.push_back(static_cast<int>(i));
      // every costate of the pass is kept
      TK_BHIP(b, c->chi.ensure(static_cast<size_t>(c->nt) * m.M * c->d * cb));
    } else {
      while (wc < b->wide.size() && b->wide[wc]->G != v.G) ++wc;
      if (wc == b->wide.size()) {
        auto w = std::make_unique<WideClass>();
        w->G = v.G;
        w->pass_fw = v.G == 2 ? b->kern.wpass_fw : b->kern.wpass_fw8;
        w->pass_bw = v.G == 2 ? b->kern.wpass_bw : b->kern.wpass_bw8;
        w->krotov = v.G == 2 ? b->kern.wkrotov : b->kern.wkrotov8;
        if (!w->pass_fw || !w->pass_bw || !w->krotov)
          return bfail(b, TK_EUNSUPPORTED, "no batched kernels for this team size");
        b->wide.push_back(std::move(w));
        witems.emplace_back();
      }
      b->wide[wc]->idx.push_back(static_cast<int>(i));
      // one segment of costates, and the backward pass's checkpoints
      const int nseg = (c->nt + tk::kSegment - 1) / tk::kSegment;
      TK_BHIP(b, m.seg.ensure(static_cast<size_t>(tk::kSegment + 1) * m.M * c->d * cb));
      TK_BHIP(b, m.ck_psi.ensure(std::max(nseg - 1, 1) * static_cast<size_t>(m.M) * vec));
      TK_BHIP(b, m.ck_meta.ensure(std::max(nseg - 1, 1) * static_cast<size_t>(m.M) *
                                  sizeof(tk::TrajMeta)));
    }
    TK_BHIP(b, c->tau.ensure(static_cast<size_t>(2) * m.M * sizeof(double)));
    TK_BHIP(b, c->u_new_dev.ensure(static_cast<size_t>(tk::kMaxCtrl) * c->nt * sizeof(double)));
    TK_BHIP(b, hipMemset(c->u_new_dev.p, 0, static_cast<size_t>(tk::kMaxCtrl) * c->nt * sizeof(double)));
    TK_BHIP(b, m.psi.ensure(static_cast<size_t>(m.M) * vec));
    TK_BHIP(b, m.meta.ensure(static_cast<size_t>(m.M) * sizeof(tk::TrajMeta)));
    TK_BHIP(b, m.tslots.ensure(static_cast<size_t>(c->nt) * m.M * ncx * sizeof(uint64_t)));
    m.variant = shape_index(c->var);
    m.kbuf_fw = plan_kbuf(c, c->u, 1);
    m.kbuf_bw = plan_kbuf(c, c->u, 0);
    // relative cost of one trajectory-step: gathers per Taylor term times terms
    m.step_cost = static_cast<double>(m.kbuf_fw) * (v.WS + (v.R - 1) * v.WSB + v.R * v.NC);
    tk::BatchInstance &I = b->inst[i];
    I.fw = base_args(c, m.M, m.seed, 0, false);
    I.bw = base_args(c, m.M, m.seed, 0, true);
    for (tk::PassArgs *a : {&I.fw, &I.bw}) {
      a->instance = m.id;
      a->rec = b->rec_dev.as<tk_jump>();
      a->rec_cap = 0;
      a->rec_count = b->rec_count_dev.as<unsigned long long>();
      a->err = b->err_dev.as<int>();
      a->chi = v.G == 1 ? c->chi.p : m.seg.p;
      a->spin_limit = 1ll << 22;
    }
    if (v.G > 1) {
      I.bw.seg_len = tk::kSegment;
      I.bw.ck_psi = m.ck_psi.p;
      I.bw.ck_meta = m.ck_meta.as<tk::TrajMeta>();
    }
    I.fw.kbuf = m.kbuf_fw;
    I.bw.kbuf = m.kbuf_bw;
    I.fw.psiT = nullptr;
    I.fw.tau_out = c->tau.as<double>();
    I.fw.u_old = c->u_dev.as<double>();
    I.fw.u_new = c->u_new_dev.as<double>();
    I.fw.S = c->S_dev.as<double>();
    I.fw.lam = c->lam_dev.as<double>();
    I.bw.tau_in = c->tau.as<double>();
    I.variant = m.variant;
    I.G = v.G;
    I.ncx = ncx;
    I.psi = m.psi.p;
    I.meta = m.meta.as<tk::TrajMeta>();
    I.tslots = m.tslots.as<unsigned long long>();
    auto &list = v.G == 1 ? items[m.variant] : witems[wc];
    for (int k = 0; k < m.M; ++k)
      list.push_back({c->nt * m.step_cost, int2{static_cast<int>(i), k}});
    b->traj_steps += 2ll * m.M * c->nt;
  }
  // work lists, costliest first (per shape for the one-wave instances)
  auto costliest_first = [](std::vector<std::pair<double, int2>> &src) {
    std::stable_sort(src.begin(), src.end(),
                     [](const auto &x, const auto &y) { return x.first > y.first; });
  };
  auto upload_items = [&](const std::vector<std::pair<double, int2>> &src, DevBuf &dev) -> int {
    std::vector<int2> it(src.size());
    for (size_t q = 0; q < src.size(); ++q) it[q] = src[q].second;
    if (it.empty()) return TK_OK;
    TK_BHIP(b, dev.ensure(it.size() * sizeof(int2)));
    TK_BHIP(b, hipMemcpy(dev.p, it.data(), it.size() * sizeof(int2), hipMemcpyHostToDevice));
    return TK_OK;
  };
  // one-wave instances grouped by shape; one work list, a range per shape
  std::stable_sort(b->narrow.begin(), b->narrow.end(),
                   [&](int x, int y) { return b->mem[x]->variant < b->mem[y]->variant; });
  std::vector<std::pair<double, int2>> all_items;
  for (size_t q = 0; q < b->narrow.size();) {
    NarrowGroup g;
    g.S = b->mem[b->narrow[q]]->variant;
    g.q0 = q;
    while (q < b->narrow.size() && b->mem[b->narrow[q]]->variant == g.S) ++q;
    g.q1 = q;
    auto &src = items[g.S];
    costliest_first(src);
    g.item0 = static_cast<int>(all_items.size());
    g.n_items = static_cast<int>(src.size());
    all_items.insert(all_items.end(), src.begin(), src.end());
    b->groups.push_back(g);
  }
  if (b->groups.size() + b->wide.size() > kLaunchSlots)
    return bfail(b, TK_EUNSUPPORTED, "too many kernel shapes in one batch");
  int rc = upload_items(all_items, b->items_dev);
  if (rc) return rc;
  for (size_t q = 0; q < b->wide.size(); ++q) {
    b->wide[q]->n_items = static_cast<int>(witems[q].size());
    costliest_first(witems[q]);
    if ((rc = upload_items(witems[q], b->wide[q]->items_dev))) return rc;
    if ((rc = plan_wide(b, *b->wide[q]))) return rc;
  }
  if (!b->narrow.empty()) {
    rc = plan_pass(b, tk::kWavesPerBlock);
    if (rc == TK_EUNSUPPORTED) rc = plan_pass(b, 1);
    if (rc) return rc == TK_EUNSUPPORTED ? bfail(b, rc, "pass term vectors do not fit in LDS") : rc;
    const double sync_cost = 0.0;
    rc = plan_krotov(b, tk::kWavesPerBlock, 1.0, sync_cost);
    if (rc == TK_EUNSUPPORTED) rc = plan_krotov(b, 1, 1.0, sync_cost);
    if (rc)
      return rc == TK_EUNSUPPORTED ? bfail(b, rc, "instances do not fit one co-resident grid") : rc;
  } else if ((rc = upload_tables(b))) {
    return rc;
  }
  b->ready = true;
  return TK_OK;
}

// One Krotov pass with the current plan: its duration (ms) and, per instance,
// the time from the launch's first block start to the instance's last block end.
int time_krotov(tk_batch *b, double *ms, std::vector<double> *inst_us, int which = 1) {
  const size_t n = b->mem.size();
  std::vector<unsigned long long> t_begin(kLaunchSlots, ~0ull), t_end(n, 0ull);
  TK_BHIP(b, hipMemcpy(b->t_begin_dev.p, t_begin.data(), kLaunchSlots * sizeof(unsigned long long),
                       hipMemcpyHostToDevice));
  TK_BHIP(b, hipMemcpy(b->t_end_dev.p, t_end.data(), n * sizeof(unsigned long long),
                       hipMemcpyHostToDevice));
  int rc = timed(b, [&] { return launch_krotov(b, which); }, ms);
  if (rc) return rc;
  if ((rc = check_errors(b))) return rc;
  TK_BHIP(b, hipMemcpy(t_begin.data(), b->t_begin_dev.p, kLaunchSlots * sizeof(unsigned long long),
                       hipMemcpyDeviceToHost));
  TK_BHIP(b, hipMemcpy(t_end.data(), b->t_end_dev.p, n * sizeof(unsigned long long),
                       hipMemcpyDeviceToHost));
  // each instance's time counts from the start of its own launch
  std::vector<size_t> slot(n, 0);
  for (size_t gi = 0; gi < b->groups.size(); ++gi)
    for (size_t q = b->groups[gi].q0; q < b->groups[gi].q1; ++q) slot[b->narrow[q]] = gi;
  for (size_t wi = 0; wi < b->wide.size(); ++wi)
    for (int i : b->wide[wi]->idx) slot[i] = b->groups.size() + wi;
  inst_us->assign(n, 0.0);
  for (size_t i = 0; i < n; ++i) {
    const unsigned long long t0 = t_begin[slot[i]];
    (*inst_us)[i] = t_end[i] > t0 && t0 != ~0ull ? (t_end[i] - t0) * 1e3 / b->clock_khz : 0.0;
  }
  return TK_OK;
}

// Autotuner of the one-wave instances: times their costate pass for each
// waves-per-block choice, and their Krotov pass for each waves-per-block choice
// with two block splits -- one from the cost model, one from the per-instance
// times measured on the first run -- and keeps the fastest.  The passes are
// deterministic and independent of the tile shape, so the repeated runs leave
// the same results as one run.  The multi-wave classes (one team per block)
// keep the cost-model split.
int autotune(tk_batch *b) {
  if (b->narrow.empty()) {  // multi-wave classes keep their cost-model plans
    b->tuned = true;
    return TK_OK;
  }
  double best = 1e300;
  int best_wpb = 0;
  for (int wpb : {4, 2, 1}) {
    if (plan_pass(b, wpb)) continue;
    double ms = 0.0;
    int rc = timed(b, [&] { return launch_pass(b, 1, 1); }, &ms);
    if (rc) return rc;
    if (ms < best) {
      best = ms;
      best_wpb = wpb;
    }
  }
  if (!best_wpb) return bfail(b, TK_EUNSUPPORTED, "no batched pass shape fits");
  int rc = plan_pass(b, best_wpb);
  if (rc) return rc;
  b->tuned_pass_ms = best;
  // Krotov pass: for each waves-per-block choice, a split from the cost model,
  // then a split from the per-trajectory-step times measured on that run
  double kbest = 1e300;
  int kw = 0;
  std::vector<int> kblocks;
  double unit = 0.0;  // the cheapest instance's modelled step: scale of the exchange weight
  for (int i : b->narrow)
    unit = unit == 0.0 ? b->mem[i]->step_cost : std::min(unit, b->mem[i]->step_cost);
  for (int wpb : {4, 2, 1}) {
    std::vector<double> cost;
    for (int round = 0; round < 2; ++round) {
      if (plan_krotov(b, wpb, 1.0, round == 0 ? 2.0 * unit : 0.0, round == 0 ? nullptr : &cost))
        break;
      double ms = 0.0;
      std::vector<double> inst_us;
      if ((rc = time_krotov(b, &ms, &inst_us))) return rc;
      if (ms < kbest) {
        kbest = ms;
        kw = wpb;
        kblocks = b->plan.nblocks;
      }
      // measured time of one trajectory-step (with its share of the exchange)
      cost.assign(b->mem.size(), 0.0);
      for (size_t q = 0; q < b->narrow.size(); ++q) {
        const int i = b->narrow[q];
        const Member &m = *b->mem[i];
        const double tw = std::ceil(static_cast<double>(m.M) / (b->plan.nblocks[q] * wpb));
        cost[i] = inst_us[i] / (m.c->nt * tw);
      }
    }
  }
  if (!kw) return bfail(b, TK_EUNSUPPORTED, "no batched Krotov shape fits");
  if ((rc = plan_krotov(b, kw, 1.0, 0.0))) return rc;  // sets wpb and LDS
  b->plan.nblocks = kblocks;
  if ((rc = upload_tables(b))) return rc;
  b->tuned_krotov_ms = kbest;
  b->tuned = true;
  return TK_OK;
}

// Krotov pass of the multi-wave classes: run with the cost-model split, then
// with a split from the per-trajectory-step times that run measured; the
// faster plan is kept (the runs give identical results).  Their pass reads the
// overlaps tau_k of the previous forward pass (the costate weights of the
// segments it recomputes) and overwrites them at its end, so the second run
// starts from a saved copy.
int autotune_wide(tk_batch *b) {
  if (b->wide.empty()) return TK_OK;
  for (auto &wp : b->wide)
    for (int i : wp->idx) {
      Member &m = *b->mem[i];
      const size_t bytes = static_cast<size_t>(2) * m.M * sizeof(double);
      TK_BHIP(b, m.tau_save.ensure(bytes));
      TK_BHIP(b, hipMemcpyAsync(m.tau_save.p, m.c->tau.p, bytes, hipMemcpyDeviceToDevice,
                                b->stream));
    }
  double ms0 = 0.0;
  std::vector<double> inst_us;
  int rc = time_krotov(b, &ms0, &inst_us, 2);
  if (rc) return rc;
  for (auto &wp : b->wide)
    for (int i : wp->idx) {
      Member &m = *b->mem[i];
      TK_BHIP(b, hipMemcpyAsync(m.c->tau.p, m.tau_save.p, static_cast<size_t>(2) * m.M * sizeof(double),
                                hipMemcpyDeviceToDevice, b->stream));
    }
  std::vector<double> cost(b->mem.size(), 0.0);
  std::vector<std::vector<int>> old;
  for (auto &wp : b->wide) {
    WideClass &w = *wp;
    for (size_t q = 0; q < w.idx.size(); ++q) {
      const int i = w.idx[q];
      const Member &m = *b->mem[i];
      const double tw = std::ceil(static_cast<double>(m.M) / w.nblocks[q]);
      cost[i] = inst_us[i] / (m.c->nt * tw);
    }
    old.push_back(w.nblocks);
    w.nblocks = split_blocks(b, w.idx, w.kro_capacity, 1, 0.0, &cost);
  }
  if ((rc = upload_tables(b))) return rc;
  double ms1 = 0.0;
  if ((rc = time_krotov(b, &ms1, &inst_us, 2))) return rc;
  if (ms1 > ms0) {  // the model split was faster
    for (size_t q = 0; q < b->wide.size(); ++q) b->wide[q]->nblocks = old[q];
    if ((rc = upload_tables(b))) return rc;
  }
  b->tuned_wide_krotov_ms = std::min(ms0, ms1);
  return TK_OK;
}

int build_graph(tk_batch *b) {
  if (b->exec) {
    (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
  }
  if (b->graph) {
    (void)hipGraphDestroy(b->graph);
    b->graph = nullptr;
  }
  TK_BHIP(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  int rc = launch_pass(b, 1);
  if (!rc) rc = launch_krotov(b);
  if (!rc) rc = launch_tail(b, 1);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(b->stream, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return bhip(b, e, "hipStreamEndCapture");
  b->graph = g;
  TK_BHIP(b, hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
  return TK_OK;
}

}  // namespace

extern "C" {

int tk_batch_create(tk_batch **out, int device, int precision) {
  if (!out) return TK_EINVAL;
  *out = nullptr;
  if (precision != TK_FP64 && precision != TK_FP32) return TK_EINVAL;
  tk_ctx *probe = nullptr;
  int rc = tk_create(&probe, device, precision);  // device checks (gfx950)
  if (rc) return rc;
  tk_destroy(probe);
  tk_batch *b = new (std::nothrow) tk_batch();
  if (!b) return TK_ENOMEM;
  b->device = device;
  b->precision = precision;
  hipDeviceProp_t prop;
  if (hipSetDevice(device) != hipSuccess || hipGetDeviceProperties(&prop, device) != hipSuccess ||
      hipStreamCreate(&b->stream) != hipSuccess || hipEventCreate(&b->ev0) != hipSuccess ||
      hipEventCreate(&b->ev1) != hipSuccess) {
    tk_batch_destroy(b);
    return TK_EHIP;
  }
  b->n_cu = prop.multiProcessorCount;
  *out = b;
  return TK_OK;
}

void tk_batch_destroy(tk_batch *b) {
  if (!b) return;
  (void)hipSetDevice(b->device);
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->ev0) (void)hipEventDestroy(b->ev0);
  if (b->ev1) (void)hipEventDestroy(b->ev1);
  if (b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

const char *tk_batch_last_error(const tk_batch *b) { return b ? b->err.c_str() : "no batch"; }

int tk_batch_add(tk_batch *b, uint32_t instance_id, int64_t d, const tk_csr *H0, int32_t n_ctrl,
                 const tk_csr *H_ctrl, int32_t n_jump, const tk_csr *L_jump, const double *psi0,
                 const double *psi_tgt, int32_t nt, double T, const double *u, const double *S,
                 const double *lambda, int32_t M, uint64_t seed, int32_t *index_out) {
  if (!b) return TK_EINVAL;
  if (b->ready) return bfail(b, TK_ESTATE, "instances cannot be added after the first iteration");
  if (M < 1) return bfail(b, TK_EINVAL, "M must be >= 1");
  for (const auto &m : b->mem)
    if (m->id == instance_id) return bfail(b, TK_EINVAL, "duplicate instance id");
  auto m = std::make_unique<Member>();
  int rc = tk_create(&m->c, b->device, b->precision);
  if (rc) return bfail(b, rc, "context creation failed");
  if ((rc = tk_set_system(m->c, d, H0, n_ctrl, H_ctrl, n_jump, L_jump)) ||
      (rc = tk_set_states(m->c, psi0, psi_tgt)) ||
      (rc = tk_set_pulses(m->c, nt, T, u, S, lambda)))
    return bfail(b, rc, std::string("instance: ") + tk_last_error(m->c));
  {
    if (shape_index(m->c->var) < 0)
      return bfail(b, TK_EUNSUPPORTED, "kernel shape not available in the batched kernels");
  }
  m->id = instance_id;
  m->M = M;
  m->seed = seed;
  if (index_out) *index_out = static_cast<int32_t>(b->mem.size());
  b->mem.push_back(std::move(m));
  return TK_OK;
}

int tk_batch_krotov_iterate(tk_batch *b, uint64_t first_iteration, int32_t n_iter,
                            double *J_T_out) {
  if (!b) return TK_EINVAL;
  TK_BHIP(b, hipSetDevice(b->device));
  if (!J_T_out) return bfail(b, TK_EINVAL, "J_T_out is NULL");
  const int n_out = n_iter + (first_iteration == 0 ? 1 : 0);
  if (n_iter < 0 || n_out > tk::kBatchHistory)
    return bfail(b, TK_EINVAL, "n_iter out of range (at most 63 per call)");
  int rc;
  if (!b->ready && (rc = finalize(b))) return rc;
  if (first_iteration != 0 && first_iteration != b->next_iter)
    return bfail(b, TK_ESTATE, "first_iteration does not continue the last call");
  if (first_iteration == 0) {
    // guess pass: iteration 0 of every instance
    const uint64_t zero = 0;
    TK_BHIP(b, hipMemcpy(b->iter_dev.p, &zero, sizeof(zero), hipMemcpyHostToDevice));
    if ((rc = launch_pass(b, 0))) return rc;
    if ((rc = launch_tail(b, 0))) return rc;
    if ((rc = check_errors(b))) return rc;
  }
  const uint64_t first = first_iteration == 0 ? 1 : first_iteration;
  for (int32_t q = 0; q < n_iter; ++q) {
    double ms = 0.0;
    if (!b->tuned) {
      // the first iteration runs step by step while the autotuner picks tiles
      if ((rc = launch_pass(b, 1))) return rc;
      if ((rc = autotune(b))) return rc;  // runs the one-wave instances' Krotov pass
      if ((rc = autotune_wide(b))) return rc;  // runs the multi-wave instances' Krotov pass
      if ((rc = launch_tail(b, 1))) return rc;
      if ((rc = build_graph(b))) return rc;
    } else {
      rc = timed(b, [&]() -> int {
        TK_BHIP(b, hipGraphLaunch(b->exec, b->stream));
        return TK_OK;
      }, &ms);
      if (rc) return rc;
      b->last_iter_ms = ms;
    }
  }
  if ((rc = check_errors(b))) return rc;
  b->next_iter = first + n_iter;
  std::vector<double> hist(b->mem.size() * tk::kBatchHistory);
  TK_BHIP(b, hipMemcpy(hist.data(), b->J_hist_dev.p, hist.size() * sizeof(double),
                       hipMemcpyDeviceToHost));
  const uint64_t it0 = first_iteration == 0 ? 0 : first_iteration;
  for (size_t i = 0; i < b->mem.size(); ++i)
    for (int q = 0; q < n_out; ++q)
      J_T_out[i * n_out + q] = hist[i * tk::kBatchHistory + (it0 + q) % tk::kBatchHistory];
  return TK_OK;
}

int tk_batch_get_pulses(tk_batch *b, int32_t index, double *u_out) {
  if (!b) return TK_EINVAL;
  if (index < 0 || index >= static_cast<int32_t>(b->mem.size()))
    return bfail(b, TK_EINVAL, "instance index out of range");
  if (!u_out) return bfail(b, TK_EINVAL, "u_out is NULL");
  tk_ctx *c = b->mem[index]->c;
  TK_BHIP(b, hipSetDevice(b->device));
  TK_BHIP(b, hipStreamSynchronize(b->stream));
  TK_BHIP(b, hipMemcpy(u_out, c->u_dev.p, static_cast<size_t>(c->n_ctrl) * c->nt * sizeof(double),
                       hipMemcpyDeviceToHost));
  return TK_OK;
}

int tk_batch_get_info(const tk_batch *b, tk_batch_info *out) {
  if (!b || !out) return TK_EINVAL;
  out->n_instances = static_cast<int32_t>(b->mem.size());
  out->pass_waves_per_block = b->plan.pass_wpb;
  out->pass_blocks = 0;
  out->krotov_blocks = 0;
  for (const auto &g : b->groups) {
    out->pass_blocks += g.pass_blocks;
    out->krotov_blocks += g.kro_blocks;
  }
  out->krotov_waves_per_block = b->plan.kro_wpb;
  out->autotuned = b->tuned ? 1 : 0;
  out->last_iteration_ms = b->last_iter_ms;
  out->tuned_pass_ms = b->tuned_pass_ms;
  out->tuned_krotov_ms = b->tuned_krotov_ms;
  out->traj_steps_per_iteration = b->traj_steps;
  out->multiwave_instances = 0;
  out->multiwave_krotov_blocks = 0;
  for (const auto &w : b->wide) {
    out->multiwave_instances += static_cast<int32_t>(w->idx.size());
    out->multiwave_krotov_blocks += w->kro_blocks;
  }
  out->tuned_multiwave_krotov_ms = b->tuned_wide_krotov_ms;
  return TK_OK;
}

}  // extern "C"
