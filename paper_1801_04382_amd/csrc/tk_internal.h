// Internal definitions shared by the HIP kernels and the host library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "trajkrotov.h"

namespace tk {

constexpr int kWave = 64;          // lanes of a CDNA wavefront
constexpr int kMaxCtrl = 8;        // controls per system
constexpr int kMaxJump = 8;        // Lindblad operators per system
constexpr int kMaxTaylor = 40;     // largest polynomial order of a step
constexpr int kWavesPerBlock = 4;  // most waves per workgroup (fewer if LDS is short)
constexpr double kMaxStepNorm = 0.5;  // substeps keep ||H_eff|| h at most this
constexpr size_t kLdsBytes = 160 * 1024;  // LDS of one gfx950 compute unit
constexpr int kMaxSubsteps = 4096;    // substeps per time step before an error
constexpr int kPollPerLane = 4;       // blocks polled by one lane in the Krotov pass
constexpr int kMaxBlocks = kWave * kPollPerLane;  // blocks of one Krotov launch
constexpr int kGradCheckpoint = 64;   // steps between forward checkpoints (gradient)

// error bits a kernel may raise (device int, OR-ed)
// Static-slot layout of a kernel shape (slots for the off-diagonal elements of
// the static part).  The shape parameter WS holds the static slots of row slot
// 0 in its low four bits and, for shapes whose host orders the basis so that
// row slot 0 holds the rows with the most off-diagonal non-zeros, the fewer
// slots of row slots m >= 1 in the bits above (0: the same count).
// Bit 8 marks shapes for real control elements: their control slots multiply
// with two FMAs instead of four (the host picks them only when every H_i
// element is real).
constexpr int kRealCtrlBit = 1 << 8;
// Bit 13 marks shapes whose row slot 0 static slots are typed: the first
// ones hold real elements, the last ws_imag (bits 9..12) imaginary ones, each
// multiplied with two FMAs (the host picks them only when the rows of row
// slot 0 fit those counts).
constexpr int kTypedBit = 1 << 13;
constexpr int ws_first(int ws) { return ws & 15; }
constexpr int ws_rest(int ws) { return ((ws >> 4) & 15) != 0 ? ((ws >> 4) & 15) : (ws & 15); }
constexpr int ws_at(int ws, int m) { return m == 0 ? ws_first(ws) : ws_rest(ws); }
constexpr bool ws_real_ctrl(int ws) { return (ws & kRealCtrlBit) != 0; }
constexpr bool ws_typed(int ws) { return (ws & kTypedBit) != 0; }
constexpr int ws_imag(int ws) { return (ws >> 9) & 15; }
constexpr int ws_code(int first, int rest, bool real_ctrl = false, int typed_imag = -1) {
  return first | rest << 4 | (real_ctrl ? kRealCtrlBit : 0) |
         (typed_imag >= 0 ? (kTypedBit | typed_imag << 9) : 0);
}

// predicted error (fraction of the substep) below which the jump-time Newton
// iteration takes its last step without evaluating the norm again
constexpr double kRootAccept = 1e-15;
constexpr int kErrNoJumpWeight = 1;  // jump with all ||L_l psi||^2 == 0
constexpr int kErrTaylorOrder = 2;   // step too long for kMaxTaylor terms
constexpr int kErrSyncTimeout = 4;   // grid-wide step reduction did not complete
constexpr int kErrJumpLoop = 8;      // more jumps in one step than allowed

// Sentinel bit pattern of an unwritten reduction slot: a NaN whose payload
// floating-point arithmetic never creates from finite inputs.
constexpr uint64_t kSlotEmpty = 0xFFF7DEADBEEF5A5Aull;

// Per-trajectory bookkeeping of the MCWF clock (kept in LDS by the Krotov pass).
// Costate segment of the batched multi-wave instances: their backward pass
// keeps checkpoints every kSegment steps and the Krotov pass recomputes the
// costates of a segment from its checkpoint before it needs them.
constexpr int kSegment = 64;

// Fixed device scratch of the entry point that allocates nothing: error bits,
// record counter, a record slot and the overlaps of up to kScratchMaxTraj
// trajectories (tk_noalloc.hip).
constexpr size_t kScratchBytes = size_t(1) << 20;
constexpr size_t kScratchErrOffset = 0;
constexpr size_t kScratchCountOffset = 8;
constexpr size_t kScratchRecOffset = 64;
constexpr size_t kScratchTauOffset = 512;
constexpr int kScratchMaxTraj = static_cast<int>((kScratchBytes - kScratchTauOffset) / 16);

struct TrajMeta {
  double nrm2;  // squared norm of the unnormalised state
  double r;     // current threshold
  double x;     // operator-choice number of the next jump (drawn with r)
  int ordinal;  // jumps so far in this pass
  int pad;
};

// Arguments of every propagation kernel.  Operator slices use the per-lane
// padded layout [slot][m][lane]: row r = lane + 64 m of the Hilbert space;
// a complex value is two consecutive reals of the bulk precision.
struct PassArgs {
  int d;        // Hilbert dimension
  int nt;       // time steps
  int M;        // trajectories
  int n_ctrl;   // controls
  int n_jump;   // Lindblad operators
  int wc;       // control slots per control (slot c belongs to control c / wc)
  int wl;       // slots per row of each jump operator
  int kmax;     // largest Taylor order allowed
  int kbuf;     // LDS term buffers per wave: a substep uses at most kbuf - 1 terms
  double dt;    // T / nt
  double tol;   // truncation tolerance of one step (relative)
  double b0;    // bound on ||H0 - (i/2) sum L^+L||_2
  double bc[kMaxCtrl];  // bounds on ||H_i||_2
  double ftol;  // relative tolerance of the jump-time root
  double inv_n[kMaxTaylor + 1];  // 1/n for the Taylor recursion (entry 0 unused)
  // ord_x[K]: the largest x = ||H_eff|| tau for which order K keeps the remainder
  // bound x^(K+1)/(K+1)! e^x within tol; non-decreasing in K (entry 0 unused)
  double ord_x[kMaxTaylor + 1];
  // operator used by the pass: H_eff pieces (forward) or their adjoints
  const int *scol;
  const void *sval;   // static part's off-diagonal elements
  const void *sdiag;  // static part's diagonal, [m][team lane] (zero on padding rows)
  const int *ccol;
  const void *cval;
  // jump operators [l][w][m][lane]
  const int *lcol;
  const void *lval;
  // pulse-like arrays have kMaxCtrl rows; rows past n_ctrl are zero (lambda: 1)
  const double *u;          // [kMaxCtrl][nt] pulses propagated with (plain passes)
  const void *psi_start;    // [64 R] complex, bulk precision, zero padded
  const double *tgt;        // [64 R] complex128, normalised, zero padded
  uint64_t seed;
  uint64_t iteration;
  uint32_t instance;
  void *psiT;               // [M][d] normalised final states (bulk), may be null
  double *tau_out;          // [2M] overlaps <tgt|psi_hat(T)>, may be null
  const double *tau_in;     // [2M] costate weights (backward pass)
  void *chi;                // [nt][M][d] costates (bulk precision); in a batched
                            // multi-wave instance [kSegment + 1][M][d], one segment
  // costate checkpoints (backward pass of a batched multi-wave instance): the
  // unnormalised backward state and its clock at t_{(s+1) kSegment}, s < nseg - 1
  int seg_len;              // 0: the backward pass stores every chi(t_j); else kSegment
  void *ck_psi;             // [nseg - 1][M][64 G R] (bulk)
  TrajMeta *ck_meta;        // [nseg - 1][M]
  tk_jump *rec;             // [rec_cap] jump records
  unsigned long long *rec_count;
  long long rec_cap;
  int *err;                 // error bits
  // sequential Krotov pass
  const double *u_old;      // [kMaxCtrl][nt] pulses of the previous iteration
  double *u_new;            // [kMaxCtrl][nt] updated pulses (written by block 0)
  const double *S;          // [kMaxCtrl][nt] update shape
  const double *lam;        // [kMaxCtrl] lambda_i
  unsigned long long *slots;  // [nt][kMaxBlocks][NC] per-block partial sums
  int traj_per_wave;        // trajectories owned by one wave
  void *kstates;            // Krotov pass with its states in global memory (the
                            // k_krotov_gs kernels): [teams][traj_per_wave][64 G R] (bulk)
  const void *pmat;         // cross-trajectory update: P_j = (1/M) sum_k |xi_k><xi_k|,
                            // complex128 [nt][d][64 R] (column c, padded rows)
  long long spin_limit;     // polls before a step reduction gives up
  // pathwise gradient with the jump record fixed
  const int *a_scol;        // adjoint operator H_eff^+: static slots
  const void *a_sval;
  const void *a_sdiag;      // and its diagonal
  const int *a_ccol;        // adjoint control slots (H_i^+ = H_i)
  const void *a_cval;
  const int *ldcol;         // adjoint jump operators L_l^+ [l][w][m][lane]
  const void *ldval;
  int wld;                  // slots per row of each L_l^+
  double bc_max;            // max_i bc[i]
  const int *path_off;      // [M + 1] first jump of each trajectory
  const int *path_step;     // [n] step of each jump (time order per trajectory)
  const double *path_t;     // [n] jump time
  const int *path_op;       // [n] operator
  void *ckpt;               // [M][nseg][64 R] forward checkpoints (bulk)
  void *stash;              // [waves][kGradCheckpoint][64 R] step-start states (bulk)
  double *gk;               // [n_ctrl][nt][M] per-trajectory gradient terms
};

// One optimisation instance of a batch: its pass arguments and the buffers of
// the batched Krotov pass.
struct BatchInstance {
  PassArgs fw;        // forward passes (guess and sequential update)
  PassArgs bw;        // costate pass (adjoint operator, starts from the target)
  int variant;        // index of the kernel shape in the precision's table
  int block0;         // first block of the batched Krotov launch serving it
  int nblocks;        // blocks serving it
  int ncx;            // shares per trajectory and step: the shape's NC (at least 1)
  int G;              // waves per trajectory of the shape (1: one-wave kernels)
  void *psi;          // [M][64 G R] states between steps (bulk)
  TrajMeta *meta;     // [M] MCWF clocks between steps
  unsigned long long *tslots;  // [nt][M][NCX] per-trajectory partials s_ik (FP64 bits)
};

// Arguments of the batched kernels.
struct BatchArgs {
  const BatchInstance *inst;
  int n_inst;
  int wave_lds;          // LDS bytes per wave of the batched plain passes
  const int2 *items;     // (instance, trajectory) work of the plain passes (one-wave shapes)
  int n_items;
  const int *block_inst; // [blocks] instance of each block of a one-wave Krotov launch
  const int2 *witems;    // the same for the instances of multi-wave shapes (one team a block)
  int n_witems;
  const int *wblock_inst;
  uint64_t *iteration;   // iteration of the passes being run (device counter)
  double *J_hist;        // [n_inst][kBatchHistory] J_T by iteration
  unsigned long long *t_begin;  // earliest block start of one Krotov launch (constant clock)
  unsigned long long *t_end;    // [n_inst] latest block end of each instance
  int *err;
  long long spin_limit;
};
constexpr int kBatchHistory = 64;  // J_T values kept per instance (ring by iteration)

// One compiled kernel variant: bulk precision, rows per lane R, static slots
// per row WS, control slots per row NC, waves per trajectory G (a team; rows
// 64 G R).
struct Variant {
  const char *name;
  int precision;  // TK_FP64 / TK_FP32
  int R, WS, NC, G;  // WS: static slots of row slot 0
  int WSB;           // static slots of row slots m >= 1 (WSB < WS: heaviest rows first)
  int ws_code;       // the kernels' WS parameter (ws_first / ws_rest / ws_real_ctrl)
  bool real_ctrl;    // control elements must be real (two-FMA control slots)
  int typed_imag;    // typed row slot 0: its imaginary slots (-1: untyped)
  const void *k_forward;
  const void *k_backward;
  const void *k_krotov;
  const void *k_krotov_gs;  // the same with the states in global memory
  const void *k_fill;  // slot initialisation
  const void *k_grad;  // pathwise gradient (replay + reverse sweep)
};

// Table of compiled variants (defined in tk_kernels.hip).
const Variant *variants(int *count);

// Kernel reducing J_T = 1 - (1/M) sum |tau_k|^2 (one block of 256 threads).
const void *functional_kernel();

// Fixed device scratch of the no-allocation entry point (tk_noalloc.hip):
// scratch_setup looks the array's address up on `device` (once; at context
// creation), scratch_base returns it (null before setup), scratch_clear zeroes
// its error bits and record counter on `stream`.
hipError_t scratch_setup(int device);
void *scratch_base(int device);
hipError_t scratch_clear(void *base, hipStream_t stream);

// Cross-trajectory update (tk_cross.hip): the sequential pass of a one-wave
// variant (null for multi-wave ones), the kernel forming the Gram matrices
// P_j of the backward states, and the LDS bytes of a block of the pass.
const void *cross_kernel(int precision, int R, int WS, int NC, int G);
const void *cross_gram_kernel(int precision);
size_t cross_lds_bytes(const Variant &v, int teams, int kbuf, int traj_per_wave);

// One Taylor step of M states, dense on the matrix cores (NT = 1, 2 or 4
// tiles of 16 trajectories a block) or with the passes' sparse series
// (one-wave variants) -- tk_dense.hip.
const void *dense_step_kernel(int precision, int NT);
const void *sparse_step_kernel(int precision, int R, int WS, int NC, int G);

// Density-matrix passes (tk_rho.hip): one workgroup propagates a d x d
// matrix with the Liouvillian (forward) or its adjoint (backward).
struct RhoCsr {       // device CSR, complex128 values
  const int *ptr;     // [d + 1]
  const int *idx;
  const void *val;
};
struct RhoArgs {
  int d, nt, n_ctrl, n_jump;
  double dt;
  RhoCsr B;                 // A = H0 - (i/2) sum L^+L (forward) or A^+ (backward)
  RhoCsr H[kMaxCtrl];       // control Hamiltonians
  RhoCsr J[kMaxJump];       // L_l (forward) or L_l^+ (backward)
  double s;                 // -1 forward, +1 backward
  double gen_b0;            // 2 ||A||
  double gen_bc[kMaxCtrl];  // 2 ||H_i||
  double gen_bj;            // sum_l ||L_l||^2
  double ord_x[kMaxTaylor + 1];
  int kmax;
  const double *u;          // [kMaxCtrl][nt] pulses of a plain pass
  void *Q0, *Q1, *R, *X, *Y;  // complex128 work matrices d^2 each (Y: n_jump of them)
  void *store;              // backward: P(t_j), [nt][d][d]; may be null
  const void *P;            // forward with the update: P(t_j) [nt][d][d]; null: plain pass
  const double *u_old, *S, *lam;
  double *u_new;            // [kMaxCtrl][nt]
  const void *tgt;          // [d] complex128, normalised
  const void *start;        // [d]: the pass starts from |start><start|
  double *J_out;            // forward: 1 - <tgt|rho(T)|tgt>
  int *err;
};
hipError_t launch_rho_pass(const RhoArgs &a, int dir, hipStream_t stream);

// Noise measure of the pulses u_dev [n_ctrl][nt] (Sec. 3.4) into nu_dev
// [n_ctrl]: one block per control (tk_post.hip).
hipError_t launch_pulse_noise(const double *u_dev, int n_ctrl, int nt, double dt, double *nu_dev,
                              hipStream_t stream);

// Gradient kernel of a variant (defined in tk_grad.hip), and the kernel that
// reduces the per-trajectory terms: one 64-thread block per pulse value.
const void *grad_kernel(int precision, int R, int WS, int NC, int G);
const void *grad_reduce_kernel();

// Batched kernels of a precision (defined in tk_batch.hip).  The shape of an
// instance is selected inside the kernels by BatchInstance::variant, the index
// of (R, WS, NC) in variants() among those of the same precision.
constexpr int kBatchShapes = 6;  // one-wave kernel shapes of the batched kernels
// Index of a kernel shape among the batched kernels' shapes (one-wave shapes
// first, < kBatchShapes), or -1 when the batched kernels do not have it.
int batch_shape_index(int precision, int R, int wsc, int NC, int G);
struct BatchKernels {
  // one-wave shapes: per shape index
  const void *pass_fw[kBatchShapes], *pass_bw[kBatchShapes], *krotov[kBatchShapes];
  const void *fill, *functional, *finish;
  // multi-wave shapes, one team per block: two-wave teams, and eight-wave teams
  const void *wpass_fw, *wpass_bw, *wkrotov;
  const void *wpass_fw8 = nullptr, *wpass_bw8 = nullptr, *wkrotov8 = nullptr;
};
BatchKernels batch_kernels(int precision);

// LDS bytes of one block of the gradient kernel with `teams` teams.
size_t grad_lds_bytes(const Variant &v, int teams, int kbuf);

// LDS bytes of one block of `teams` teams (G waves each): the block's copy of
// the control slots (one-wave teams only), then per team `kbuf` term vectors of 64 G R + 1 elements
// and, for the Krotov pass, `traj_per_wave` state vectors (unless they are
// kept in global memory) and their bookkeeping.
size_t block_lds_bytes(const Variant &v, int teams, int kbuf, int traj_per_wave,
                       bool states_in_lds = true);

}  // namespace tk
