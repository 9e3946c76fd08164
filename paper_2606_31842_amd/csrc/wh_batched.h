// Device-side state of the batched solver: phases, per-problem descriptors and states, and
// the per-round work plan (shared by the solver's kernels and host code).
#pragma once
#include "wh_common.h"

namespace wh {

enum BPhase : int {
  BP_B_FIRST = 0, BP_B_STEP, BP_B_LAST,
  BP_INIT,
  BP_A_FIRST, BP_A_STEP, BP_A_LAST,
  BP_UPD1, BP_UPD2,
  BP_R_FIRST, BP_R_STEP, BP_R_LAST,
  BP_DONE
};

struct BDesc {
  int n, nt, ntx, nty, tile0, mixed, max_iters, max_outer, defect, x0;  // x0: start from x_0, A x_0 in q
  double a, tol, itol, om2dt2;   // om2dt2 = (omega dt)^2 of the fixed point
  double *x, *b, *r, *p, *q, *V;
  void* W[4];                 // FP64 (prev, cur) pairs 0 and 1; 8 bytes per node each
  void* W32[4];               // FP32 pairs (mixed only): four arrays, or (batches without
                              // forced FP32 steps) each pair one interleaved array of (W^n, D)
                              // at 8 bytes per node, slot 2k+1 its start, slot 2k 4 bytes further
  const double* kap64;
  const double* fs64;
  const float* kap32;
  const float* fs32;
  const double* w;            // trapezoid weights, N_t + 1
  const double* cosv;         // cos(omega_w t^n), N_t + 1
  double* partials;           // one per tile
};

struct BState {
  int phase, step, pair, iters, outer, status, stalls, force64, last_repl, restart, pad_[2];
  double r2, rhs2, nb2, alpha, beta, rel, itol, pq, prev_rel, it64;  // it64: FP64 inner iterations
};

// Stepping precision of a phase: 1 = FP32 (inner CG of a mixed problem that has not
// fallen back to FP64), 0 = FP64 (everything else, including element-wise phases).
__host__ __device__ inline int phase_prec(int ph, int mixed) {
  if (ph == BP_A_FIRST || ph == BP_A_STEP || ph == BP_A_LAST) return mixed ? 1 : 0;
  return 0;
}

// Tile of the work kernels: kBW wavefronts side by side, each a strip of 64 * kBC columns
// of which the inner 64 * kBC - 2K are written (the row-marching K-step pipeline), over
// kBSeg rows.  Element-wise phases cover the same tile with all 64 * kBW threads.
// Two-wave blocks: on the 256-problem batch (FP32, K = 8) the stepping launch takes 665 us
// against 698 us with four waves per block, and the batch 1.284 s against 1.346 s; one-wave
// blocks step faster still (658 us) but lengthen the other phases (batch 1.387 s).
constexpr int kBW = 2;
constexpr int kBC = 1;
constexpr int kBSeg = 32;
__host__ __device__ constexpr int batch_strip(int K) { return 64 * kBC - 2 * K; }
__host__ __device__ constexpr int batch_txo(int K) { return kBW * batch_strip(K); }
__host__ __device__ constexpr int batch_tyo() { return kBSeg; }

// Problems per batch (the work kernels search the plan's item offsets in LDS).
constexpr int kMaxBatch = 4096;

// Work plan of one round, per precision class (0: FP64 and element-wise phases, 1: FP32
// stepping phases): [active tiles, active problems, problem ids (nb), first item of each
// active problem (nb + 1)].
__host__ __device__ constexpr int plan_stride(int nb) { return 2 * nb + 3; }

}  // namespace wh
