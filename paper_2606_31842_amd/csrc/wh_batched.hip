// Batched WaveHoltz solves: many 2D problems of different sizes, frequencies and
// sources advanced together by device-side phase machines.
//
// Every problem runs the same method as wh_solve (the filter of eq. WaveHoltzDiscreteFPI
// applied by the leapfrog scheme with the trapezoid sum, and CG on A = I - S_h,
// Algorithm 3 without deflation; in mixed precision the CG recurrence applies the
// FP32-stepped operator and its residual is replaced by the true FP64 residual each
// time it has dropped tenfold).  Instead of host-driven loops, each problem keeps
// its phase, time-step counter and Krylov scalars in device memory:
//
//   B_FIRST -> B_STEP* -> B_LAST         b = Pi_h(0; f)                        (FP64)
//   INIT                                 r = p = b - A x_0, partial r.r
//   A_FIRST -> A_STEP* -> A_LAST         q = A p, partial sums of p.q          (CG precision)
//   UPD1                                 x += alpha p, r -= alpha q, partial r.r
//   R_FIRST -> R_STEP* -> R_LAST         r = b - A x, partial r.r              (FP64)
//   UPD2                                 p = r + beta p            -> A_FIRST
//
// One round = the FP32 work kernel (one block per tile of every problem, through a static
// block -> (problem, tile) table laid out so each XCD gets a contiguous run of tiles), beside
// it on a second stream the plan kernel and the FP64 work kernel (persistent blocks over the
// round's plan of FP64 and element-wise tiles), then the control kernel.  A
// block does the work of its problem's current phase on its tile, or returns.  The control
// kernel (one block per problem) reduces the tile partial sums in a fixed order, updates
// alpha/beta and the convergence state and advances the phase.  Rounds contain no host
// decisions, so the host captures several of them in one hipGraph and replays it, reading
// back one counter of unfinished problems per replay.
//
// In mixed batches whose FP32 steps are never forced (no defect form), each FP32 state pair
// is one interleaved array, (W, D) in 8 bytes per node; otherwise two arrays.
//
// Deflated problems (c = 1, n_defl sine modes W nearest omega^2) start from
// x_0 = W (W^T A W)^{-1} W^T b.  With exact eigenvectors this is the projection of the
// solution onto span W, W^T u = (omega^2 - lambda^2)^{-1} W^T f, and A x_0 =
// W diag(mu) W^T u: the set-up computes both from f before the batch (the host selects the
// modes and scales, the device projects and combines; x_0 into x, A x_0 into q) and INIT
// forms r_0 = b - A x_0.  r_0 is orthogonal to W, and CG
// continues without re-projection (Algorithm 3 with exact eigenvectors).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "wh_batched.h"
#include "wh_march2d.h"
#include "wh_reduce.h"

namespace wh {

__device__ __forceinline__ int xcd_tile_b(int bid, int nb) {
  const int xcd = bid & 7, idx = bid >> 3;
  const int q = nb >> 3, r = nb & 7;
  return xcd < r ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

// State slot k of a problem: pair k/2, k odd W^n, k even the other member.  Interleaved FP32
// pairs (W at 8 bytes per node, D 4 bytes after it) have their nodes 2 elements apart.
template <typename T>
__device__ __forceinline__ T* state_of(const BDesc& D, int k) {
  return sizeof(T) == 8 ? (T*)D.W[k] : (T*)D.W32[k];
}


template <typename T>
__device__ __forceinline__ const T* kap_of(const BDesc& D);
template <>
__device__ __forceinline__ const double* kap_of<double>(const BDesc& D) { return D.kap64; }
template <>
__device__ __forceinline__ const float* kap_of<float>(const BDesc& D) { return D.kap32; }
template <typename T>
__device__ __forceinline__ const T* fs_of(const BDesc& D);
template <>
__device__ __forceinline__ const double* fs_of<double>(const BDesc& D) { return D.fs64; }
template <>
__device__ __forceinline__ const float* fs_of<float>(const BDesc& D) { return D.fs32; }

// dt^2 L_h W at interior node p from a state array whose nodes are SS elements apart
// (global reads); DIFF sums the constant-c stencil as differences to the centre (FP32
// increment form).
template <typename T, bool VARC, bool DIFF, int SS>
__device__ __forceinline__ T lap_term(const T* c, const T* kap, int64_t p, int64_t P, T A) {
  const T cc = c[SS * p];
  const T cw = c[SS * (p - 1)], ce = c[SS * (p + 1)], cs = c[SS * (p - P)], cn = c[SS * (p + P)];
  if (VARC) {
    const T kc = kap[p];
    return (kc + kap[p - 1]) * (cw - cc) + (kc + kap[p + 1]) * (ce - cc) +
           ((kc + kap[p - P]) * (cs - cc) + (kc + kap[p + P]) * (cn - cc));
  }
  if (DIFF) return A * (((cw - cc) + (ce - cc)) + ((cs - cc) + (cn - cc)));
  return A * (((cw + ce) + (cs + cn)) - T(4) * cc);
}

// Fourth-order differences (c = 1), dt^2 L_h W at interior node (i, j) as A12 (sx + sy) with
// A12 = dt^2 / (12 h^2) and, per axis, 16 ((W_-1 - W) + (W_+1 - W)) - ((W_-2 - W) + (W_+2 - W)).
// The neighbour two points beyond the last interior point is the odd reflection -W (row or
// column -1 and n+1); the boundary rows and columns are zero (not read).  get(q) reads the
// interior node of flat index q.
template <typename T, typename Get>
__device__ __forceinline__ T lap4_at(Get get, int64_t p, int i, int j, int n, int64_t P, T A12) {
  const T cc = get(p);
  const T w1 = i > 1 ? get(p - 1) : T(0), e1 = i < n - 1 ? get(p + 1) : T(0);
  const T s1 = j > 1 ? get(p - P) : T(0), n1 = j < n - 1 ? get(p + P) : T(0);
  const T w2 = i == 1 ? -cc : (i == 2 ? T(0) : get(p - 2));
  const T e2 = i == n - 1 ? -cc : (i == n - 2 ? T(0) : get(p + 2));
  const T s2 = j == 1 ? -cc : (j == 2 ? T(0) : get(p - 2 * P));
  const T n2 = j == n - 1 ? -cc : (j == n - 2 ? T(0) : get(p + 2 * P));
  const T sx = T(16) * ((w1 - cc) + (e1 - cc)) - ((w2 - cc) + (e2 - cc));
  const T sy = T(16) * ((s1 - cc) + (n1 - cc)) - ((s2 - cc) + (n2 - cc));
  return A12 * (sx + sy);
}

// The work of one tile of problem sid in its current phase (lt: the tile within the problem).
// ORD: 2 (the five-point Laplacian, variable c allowed) or 4 (fourth-order differences for
// c == 1; the stepping launches advance K/2 steps, so that the halo, 2 points per step, and with
// it the tile geometry stay those of K second-order steps).  PAIR: the batch keeps each FP32
// state pair in one interleaved array (batches without forced FP32 steps; see prepare_batch).
template <typename T, int K, bool VARC, int ORD = 2, bool PAIR = false>
__device__ __forceinline__ void batch_tile(const BDesc* __restrict__ descs, const BState* __restrict__ states,
                                           int sid, int lt) {
  constexpr int TXO = batch_txo(K);
  constexpr int TYO = batch_tyo();
  constexpr int NT = 64 * kBW;
  // FP32 state pairs are (W^n, D^{n-1/2} = W^n - W^{n-1}), stepped in the increment form
  // D += dt^2 (L_h W - f cos), W += D; FP64 pairs are (W^n, W^{n-1}).
  constexpr bool INC = sizeof(T) == 4;
  static_assert(ORD == 2 || (ORD == 4 && !VARC && K % 2 == 0), "fourth order: c == 1, even K");
  constexpr int KS = ORD == 4 ? K / 2 : K;   // steps per stepping launch
  constexpr bool PR = PAIR && INC;             // interleaved FP32 pairs
  constexpr int SS = PR ? 2 : 1;
  const BDesc& D = descs[sid];
  const int ph = states[sid].phase;
  const int n = D.n;
  const int64_t P = (int64_t)n + 1;
  const int x0 = 1 + (lt % D.ntx) * TXO;
  const int y0 = 1 + (lt / D.ntx) * TYO;
  const int tid = threadIdx.y * 64 + threadIdx.x;
  const BState& S = states[sid];
  double acc = 0.0;
  bool reduce = false;
  const T A = (T)D.a;

  // element-wise loop over the tile's interior nodes
#define TILE_FOR(p)                                                                  \
  for (int e = tid; e < TXO * TYO; e += NT)                                          \
    if (x0 + e % TXO <= n - 1 && y0 + e / TXO <= n - 1)                              \
      for (int64_t p = (int64_t)(y0 + e / TXO) * P + (x0 + e % TXO), _o = 0; _o < 1; ++_o)

  switch (ph) {
    case BP_INIT: {
      // r_0 = p_0 = b - A x_0 (deflated start) or b (x = 0; a restart clears x first)
      reduce = true;
      const bool clear = S.restart != 0;
      TILE_FOR(p) {
        const double v = D.x0 ? D.b[p] - D.q[p] : D.b[p];
        if (clear) D.x[p] = 0.0;
        D.r[p] = v;
        D.p[p] = v;
        acc += v * v;
      }
      break;
    }
    case BP_UPD1: {
      double* y = D.x;
      const double al = S.alpha;
      reduce = true;
      TILE_FOR(p) {
        y[p] += al * D.p[p];
        const double rv = D.r[p] - al * D.q[p];
        D.r[p] = rv;
        acc += rv * rv;
      }
      break;
    }
    case BP_UPD2: {
      const double be = S.beta;
      TILE_FOR(p) { D.p[p] = D.r[p] + be * D.p[p]; }
      break;
    }
    case BP_A_FIRST:
      if (ORD == 2 && sizeof(T) == 4 && D.defect) {
        // FP32 inner operator in the defect form A p = Pi_h(0; H p): forcing
        // fs = -dt^2 H p, W^0 = 0, W^1 = -fs/2, V = w1 W^1
        T* w0o = state_of<T>(D, 0);
        T* w1o = state_of<T>(D, 1);
        T* fso = (T*)D.fs32;
        TILE_FOR(p) {
          const int i = (int)(p % P), j = (int)(p / P);
          const double pc = D.p[p];
          const double nbv[4] = {i > 1 ? D.p[p - 1] : 0.0, i < n - 1 ? D.p[p + 1] : 0.0,
                                 j > 1 ? D.p[p - P] : 0.0, j < n - 1 ? D.p[p + P] : 0.0};
          const int64_t nbi[4] = {p - 1, p + 1, p - P, p + P};
          double lap = 0.0;
          for (int t = 0; t < 4; ++t)
            lap += (VARC ? D.kap64[p] + D.kap64[nbi[t]] : D.a) * (nbv[t] - pc);
          const T fsv = (T)(-(lap + D.om2dt2 * pc));
          fso[p] = fsv;
          const T w1 = T(-0.5) * fsv;
          w0o[SS * p] = w1;           // FP32 pair: D^{1/2} = W^1 - W^0 = W^1
          w1o[SS * p] = w1;
          D.V[p] = D.w[1] * (double)w1;
        }
        break;
      }
      [[fallthrough]];
    case BP_B_FIRST:
    case BP_R_FIRST: {
      // W^0 = src (B: zero), W^1 = W^0 + dt^2/2 (L_h W^0 - f), V = w0 W^0 + w1 W^1
      const double* src = ph == BP_A_FIRST ? D.p : (ph == BP_R_FIRST ? D.x : nullptr);
      const bool force = ph == BP_B_FIRST;
      T* w0o = state_of<T>(D, 0);
      T* w1o = state_of<T>(D, 1);
      const T* kap = kap_of<T>(D);
      const T* fs = fs_of<T>(D);
      TILE_FOR(p) {
        T c = T(0), lap = T(0);
        if (src && ORD == 4) {
          const int i = (int)(p % P), j = (int)(p / P);
          c = (T)src[p];
          lap = lap4_at<T>([&](int64_t q) { return (T)src[q]; }, p, i, j, n, P, (T)(D.a / 12.0));
        } else if (src) {
          const int i = (int)(p % P), j = (int)(p / P);
          c = (T)src[p];
          const T wv = i > 1 ? (T)src[p - 1] : T(0);
          const T ev = i < n - 1 ? (T)src[p + 1] : T(0);
          const T sv = j > 1 ? (T)src[p - P] : T(0);
          const T nv = j < n - 1 ? (T)src[p + P] : T(0);
          if (VARC) {
            const T kc = kap[p];
            lap = (kc + kap[p - 1]) * (wv - c) + (kc + kap[p + 1]) * (ev - c) +
                  ((kc + kap[p - P]) * (sv - c) + (kc + kap[p + P]) * (nv - c));
          } else if (INC) {
            lap = A * (((wv - c) + (ev - c)) + ((sv - c) + (nv - c)));
          } else {
            lap = A * (((wv + ev) + (sv + nv)) - T(4) * c);
          }
        }
        if (force) lap -= (T)D.cosv[0] * fs[p];
        if (INC) {               // FP32 pair (W^1, D^{1/2})
          const T d = T(0.5) * lap;
          const T w1 = c + d;
          w0o[SS * p] = d;
          w1o[SS * p] = w1;
          D.V[p] = D.w[0] * (src ? src[p] : 0.0) + D.w[1] * (double)w1;
        } else {
          const T w1 = c + T(0.5) * lap;
          w0o[SS * p] = c;
          w1o[SS * p] = w1;
          D.V[p] = D.w[0] * (src ? src[p] : 0.0) + D.w[1] * (double)w1;
        }
      }
      break;
    }
    case BP_B_LAST:
    case BP_A_LAST:
    case BP_R_LAST: {
      const int pr = S.pair;
      const T* cur = state_of<T>(D, 2 * pr + 1);
      const T* prv = state_of<T>(D, 2 * pr);
      const T* kap = kap_of<T>(D);
      const T* fs = fs_of<T>(D);
      const int k = D.nt - 1;
      const double wn = D.w[k + 1];
      const T cn = (T)D.cosv[k];
      const bool defect = sizeof(T) == 4 && D.defect && ph == BP_A_LAST;
      reduce = true;
      TILE_FOR(p) {
        T nw;
        if (ORD == 4) {
          const T lap = lap4_at<T>([&](int64_t q) { return cur[SS * q]; }, p, (int)(p % P), (int)(p / P), n, P,
                                   (T)(D.a / 12.0));
          if (INC) {
            nw = cur[SS * p] + (prv[SS * p] + (ph == BP_B_LAST ? lap - cn * fs[p] : lap));
          } else {
            nw = (cur[SS * p] + cur[SS * p]) - prv[SS * p] + lap;
            if (ph == BP_B_LAST) nw -= cn * fs[p];
          }
        } else if (INC) {
          T lap = lap_term<T, VARC, true, SS>(cur, kap, p, P, A);
          if (ph == BP_B_LAST || defect) lap -= cn * fs[p];
          nw = cur[SS * p] + (prv[SS * p] + lap);
        } else {
          nw = (cur[SS * p] + cur[SS * p]) - prv[SS * p] + lap_term<T, VARC, false, SS>(cur, kap, p, P, A);
          if (ph == BP_B_LAST || defect) nw -= cn * fs[p];
        }
        const double vf = D.V[p] + wn * (double)nw;
        if (ph == BP_B_LAST) {
          D.b[p] = vf;
          acc += vf * vf;
        } else if (ph == BP_A_LAST) {
          const double pv = D.p[p];
          const double qv = defect ? -vf : pv - vf;
          D.q[p] = qv;
          acc += pv * qv;
        } else {
          // true residual b - A x replaces r (FP64 batches take it once, at the end)
          const double rv = D.b[p] - (D.x[p] - vf);
          D.r[p] = rv;
          acc += rv * rv;
        }
      }
      break;
    }
    case BP_B_STEP:
    case BP_A_STEP:
    case BP_R_STEP: {
      // K' <= K steps by the row-marching pipeline, one strip per wavefront
      const int pr = S.pair;
      MarchIO<T> io;
      io.cin = state_of<T>(D, 2 * pr + 1);
      io.pin = state_of<T>(D, 2 * pr);
      io.cout = state_of<T>(D, 2 * (pr ^ 1) + 1);
      io.pout = state_of<T>(D, 2 * (pr ^ 1));
      io.V = D.V;
      io.kap = kap_of<T>(D);
      io.fs = fs_of<T>(D);
      io.w = D.w + S.step;
      io.cs = D.cosv + S.step;
      io.A = ORD == 4 ? (T)(D.a / 12.0) : A;
      io.n = n;
      io.Kp = min(KS, D.nt - 1 - S.step);
      io.force = ph == BP_B_STEP || (sizeof(T) == 4 && D.defect && ph == BP_A_STEP);
      const int xs = x0 + (int)threadIdx.y * batch_strip(K);
      const bool up = ((lt / D.ntx) & 1) != 0;
      if (xs <= n - 1) {
        if constexpr (ORD == 4) march2d<T, KS, kBC, false, 2, PR>(io, xs, y0, min(y0 + TYO, n), up);
        else march2d<T, K, kBC, VARC, 1, PR>(io, xs, y0, min(y0 + TYO, n), up);
      }
      break;
    }
    default:
      break;
  }
#undef TILE_FOR
  if (reduce) {
    const double sres = block_sum<kBW>(acc, tid);
    if (tid == 0) D.partials[lt] = sres;
  }
}

// Occupancy bound of the work kernels (waves per SIMD): what the row-marching pipeline's
// registers allow without spilling.
template <typename T, int K, bool VARC, int ORD = 2>
constexpr int batch_waves_per_eu() {
  // fourth order: the radius-2 pipeline keeps 8 rows per level
  if (ORD == 4) return sizeof(T) == 4 ? (K <= 4 ? 4 : 3) : (K <= 2 ? 4 : (K <= 4 ? 3 : 2));
  if (sizeof(T) == 4) return VARC ? (K <= 2 ? 4 : (K <= 4 ? 3 : 2)) : (K <= 2 ? 6 : (K <= 4 ? 4 : 3));
  return VARC ? (K <= 2 ? 4 : (K <= 4 ? 3 : 2)) : (K <= 2 ? 6 : (K <= 4 ? 4 : 2));
}

// One work kernel: persistent blocks take the active tiles of their class that the plan lists.
// The item range is cut into 8 contiguous chunks, one per XCD (blocks are dispatched
// round-robin over the XCDs), so that neighbouring tiles of a problem share an L2; a block
// takes items of its XCD's chunk from that chunk's counter, then helps with the other chunks.
// The plan kernel resets the counters.  TAG only separates the measurement launches of
// wh_time_batch_kernel (TAG = 1) from the solver's in profiles; the code is the same.
// The occupancy bound keeps the register budget of the one-tile-per-block form
// (batch_waves_per_eu: the waves per SIMD that the row pipeline's registers allow).
template <typename T, int K, bool VARC, int TAG = 0, int ORD = 2>
__global__ __launch_bounds__(64 * kBW, (batch_waves_per_eu<T, K, VARC, ORD>()))
void k_batch_work(const BDesc* __restrict__ descs,
                                                        const BState* __restrict__ states,
                                                        int* __restrict__ plan, int nb, int want) {
  constexpr int kCache = kMaxBatch;   // item offsets of the active problems, searched in LDS
  const int* pl = plan + want * plan_stride(nb);
  int* ctr = plan + 2 * plan_stride(nb) + 8 * want;
  const int total = pl[0], nact = pl[1];
  if (total == 0) return;
  const int* pid = pl + 2;
  const int* start = pl + 2 + nb;
  const int tid = threadIdx.y * 64 + threadIdx.x;
  __shared__ int s_start[kCache + 1];
  __shared__ int s_item;
  for (int k = tid; k <= nact; k += 64 * kBW) s_start[k] = start[k];
  const int xcd = blockIdx.x & 7;
  int q = 0, c = xcd;
  int c0 = (int)((int64_t)total * c / 8), c1 = (int)((int64_t)total * (c + 1) / 8);
  if (tid == 0) s_item = c0 + atomicAdd(&ctr[c], 1);
  __syncthreads();
  while (true) {
    const int it = s_item;
    __syncthreads();
    if (it >= c1) {
      // this chunk is done: help with the next XCD's chunk
      if (++q == 8) break;
      c = (xcd + q) & 7;
      c0 = (int)((int64_t)total * c / 8);
      c1 = (int)((int64_t)total * (c + 1) / 8);
      if (tid == 0) s_item = c0 + atomicAdd(&ctr[c], 1);
      __syncthreads();
      continue;
    }
    // the next item's index is requested now and stored after this item's work, so the
    // atomic's latency overlaps the tile
    int nxt = 0;
    if (tid == 0) nxt = atomicAdd(&ctr[c], 1);
    // the active problem holding item it: start[k] <= it < start[k + 1]
    int lo = 0, hi = nact - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (s_start[mid] <= it) lo = mid;
      else hi = mid - 1;
    }
    const int k0 = s_start[lo];
    batch_tile<T, K, VARC, ORD>(descs, states, pid[lo], it - k0);
    if (tid == 0) s_item = c0 + nxt;
    __syncthreads();
  }
}

// The same work, one tile per block over every tile of every problem (block -> tile through
// the static tile table, in XCD-contiguous order); blocks whose problem is not in class `want`
// return at once.  Used for the class that holds most of the tiles (the FP32 stepping of a
// mixed batch, everything in an FP64 batch), where the hardware's block dispatch balances the
// work best.
template <typename T, int K, bool VARC, int TAG = 0, int ORD = 2, bool PAIR = false>
__global__ __launch_bounds__(64 * kBW, (batch_waves_per_eu<T, K, VARC, ORD>()))
void k_batch_tile(const BDesc* __restrict__ descs, const BState* __restrict__ states,
                  const int* __restrict__ tile_solve, int ntiles, int want) {
  const int gt = xcd_tile_b(blockIdx.x, ntiles);
  const int sid = tile_solve[gt];
  const BDesc& D = descs[sid];
  const BState& S = states[sid];
  const int ph = S.phase;
  if (ph == BP_DONE) return;
  const bool stepping = ph != BP_INIT && ph != BP_UPD1 && ph != BP_UPD2;
  const int cls = (stepping && phase_prec(ph, D.mixed && !S.force64) == 1) ? 1 : 0;
  if (cls != want) return;
  batch_tile<T, K, VARC, ORD, PAIR>(descs, states, sid, gt - D.tile0);
}

// The plan of the next round from the problems' phases (one block; problems in index order,
// so that the tiles of a problem stay consecutive).
__global__ __launch_bounds__(256) void k_batch_plan(const BDesc* __restrict__ descs,
                                                    const BState* __restrict__ states, int nb, int* plan) {
  __shared__ int sc[4][256];
  __shared__ int base[4];   // tiles class 0, problems class 0, tiles class 1, problems class 1
  const int tid = threadIdx.x;
  if (tid < 4) base[tid] = 0;
  __syncthreads();
  for (int c0 = 0; c0 < nb; c0 += 256) {
    const int i = c0 + tid;
    int cls = -1, nt = 0;
    if (i < nb) {
      const int ph = states[i].phase;
      if (ph != BP_DONE) {
        const int prec = phase_prec(ph, descs[i].mixed && !states[i].force64);
        const bool stepping = ph != BP_INIT && ph != BP_UPD1 && ph != BP_UPD2;
        cls = (stepping && prec == 1) ? 1 : 0;
        nt = descs[i].ntx * descs[i].nty;
      }
    }
    int v[4] = {cls == 0 ? nt : 0, cls == 0 ? 1 : 0, cls == 1 ? nt : 0, cls == 1 ? 1 : 0};
    // inclusive scans (Hillis-Steele) of the four values
    for (int q = 0; q < 4; ++q) sc[q][tid] = v[q];
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
      int t[4];
      for (int q = 0; q < 4; ++q) t[q] = tid >= o ? sc[q][tid - o] : 0;
      __syncthreads();
      for (int q = 0; q < 4; ++q) sc[q][tid] += t[q];
      __syncthreads();
    }
    if (cls >= 0) {
      int* pl = plan + cls * plan_stride(nb);
      const int k = base[2 * cls + 1] + sc[2 * cls + 1][tid] - 1;        // position among the active
      pl[2 + k] = i;
      pl[2 + nb + k] = base[2 * cls] + sc[2 * cls][tid] - nt;          // first item of problem i
    }
    __syncthreads();
    if (tid == 0)
      for (int q = 0; q < 4; ++q) base[q] += sc[q][255];
    __syncthreads();
  }
  if (tid < 2) {
    int* pl = plan + tid * plan_stride(nb);
    pl[0] = base[2 * tid];
    pl[1] = base[2 * tid + 1];
    pl[2 + nb + base[2 * tid + 1]] = base[2 * tid];
  }
  if (tid < 16) plan[2 * plan_stride(nb) + tid] = 0;   // the work kernels' item counters
}

// One block per problem: reduce the tile partials in order and advance the phase.
__global__ __launch_bounds__(256) void k_batch_control(const BDesc* __restrict__ descs,
                                                       BState* __restrict__ states, int K) {
  const int sid = blockIdx.x;
  const BDesc& D = descs[sid];
  BState& S = states[sid];
  const int ph = S.phase;
  if (ph == BP_DONE) return;
  const bool red = ph == BP_B_LAST || ph == BP_INIT || ph == BP_A_LAST || ph == BP_R_LAST || ph == BP_UPD1;
  double sum = 0.0;
  if (red) {
    double acc = 0.0;
    const int nt = D.ntx * D.nty;
    for (int t = threadIdx.x; t < nt; t += 256) acc += D.partials[t];
    sum = block_sum256(acc, threadIdx.x);
  }
  if (threadIdx.x != 0) return;
  auto after_first = [&](int step_phase, int last_phase) {
    S.step = 1;
    S.pair = 0;
    S.phase = (D.nt - 1 == 1) ? last_phase : step_phase;
  };
  auto after_step = [&](int last_phase) {
    const int Kp = min(K, D.nt - 1 - S.step);
    S.step += Kp;
    S.pair ^= 1;
    if (S.step >= D.nt - 1) S.phase = last_phase;
  };
  switch (ph) {
    case BP_B_FIRST: after_first(BP_B_STEP, BP_B_LAST); break;
    case BP_A_FIRST: after_first(BP_A_STEP, BP_A_LAST); break;
    case BP_R_FIRST: after_first(BP_R_STEP, BP_R_LAST); break;
    case BP_B_STEP: after_step(BP_B_LAST); break;
    case BP_A_STEP: after_step(BP_A_LAST); break;
    case BP_R_STEP: after_step(BP_R_LAST); break;
    case BP_B_LAST:
      S.nb2 = sum;
      S.prev_rel = 1.0;
      if (!(sum > 0)) {         // f = 0: u = 0 is the solution
        S.rel = 0.0;
        S.status = WH_OK;
        S.phase = BP_DONE;
      } else if (!isfinite(sum)) {
        S.status = WH_EUNSTABLE;
        S.phase = BP_DONE;
      } else {
        S.rhs2 = sum;
        S.rel = 1.0;
        S.phase = BP_INIT;
      }
      break;
    case BP_INIT: {
      // r_0 = b (no start vector) or b - A x_0 (deflated start), both exact in FP64
      S.restart = 0;
      if (!(S.nb2 > 0)) {
        // b = 0: the solution is 0, and x is 0 here (no start, or the start from a zero f)
        S.r2 = 0.0;
        S.rel = 0.0;
        S.prev_rel = 0.0;
        S.status = WH_OK;
        S.phase = BP_DONE;
        break;
      }
      const double rel = sqrt(sum / S.nb2);
      S.r2 = sum;
      S.rel = rel;
      S.prev_rel = rel;       // relative true residual at the last replacement
      if (!isfinite(rel)) {
        S.status = WH_EUNSTABLE;
        S.phase = BP_DONE;
      } else if (rel <= D.tol) {
        // the start already meets the tolerance: report its true residual
        S.status = WH_OK;
        S.pq = sum;
        S.phase = BP_R_FIRST;
      } else {
        S.phase = BP_A_FIRST;
      }
      break;
    }
    case BP_A_LAST:
      S.pq = sum;
      if (!isfinite(sum)) {
        S.status = WH_EUNSTABLE;
        S.phase = BP_DONE;
      } else if (sum == 0.0) {
        S.status = WH_EBREAKDOWN;
        S.phase = BP_DONE;
      } else {
        S.alpha = S.r2 / sum;
        S.phase = BP_UPD1;
      }
      break;
    case BP_UPD1: {
      const double r2_old = S.r2;
      S.beta = sum / r2_old;
      S.r2 = sum;
      S.iters++;
      if (D.mixed && S.force64) S.it64 += 1.0;
      const double rel = sqrt(sum / S.nb2);
      const bool cap = S.iters >= D.max_iters;
      S.rel = rel;
      if (!isfinite(rel)) {
        S.status = WH_EUNSTABLE;
        S.phase = BP_DONE;
      } else if (!D.mixed) {
        if (rel <= D.tol || cap) {
          S.status = rel <= D.tol ? WH_OK : WH_ENOCONV;
          S.phase = BP_R_FIRST;        // true FP64 residual for the report
        } else {
          S.phase = BP_UPD2;
        }
      } else if (S.force64 ? (rel <= D.tol || cap)
                           : (rel <= D.itol * S.prev_rel || rel >= 10.0 * S.prev_rel || rel <= D.tol || cap ||
                              S.iters - S.last_repl >= 500)) {
        // FP32 operator: the recursive residual is replaced by the true one whenever it has
        // fallen by itol (or grown tenfold, or 500 iterations passed).  After the fallback to
        // FP64 the recurrence runs as plain CG and the true residual is formed only when the
        // recursive one meets the tolerance (a replacement then continues the iteration)
        S.pq = r2_old;                 // kept for beta after the replacement
        S.phase = BP_R_FIRST;
      } else {
        S.phase = BP_UPD2;
      }
      break;
    }
    case BP_UPD2: S.phase = BP_A_FIRST; break;
    case BP_R_LAST: {
      const double rel = sqrt(sum / S.nb2);
      S.outer++;
      if (!D.mixed) {
        S.pq = rel;                    // true residual (status already set)
        S.phase = BP_DONE;
        break;
      }
      // residual replacement: beta from the true residual, the recurrence continues
      S.beta = sum / S.pq;
      S.r2 = sum;
      S.rel = rel;
      S.stalls = rel > 0.5 * S.prev_rel ? S.stalls + 1 : 0;
      S.last_repl = S.iters;
      if (S.stalls >= 2 && !S.force64) {
        // the FP32 operator error dominates: continue in FP64.  A problem without a
        // deflated start begins again from x = 0 as plain FP64 CG (the iterate the FP32
        // operator left can hold large components along near-singular, possibly negative
        // modes of A, from which CG need not recover); a deflated one continues from the
        // true residual (p = r)
        S.force64 = 1;
        S.beta = 0.0;
        if (!D.x0) {
          S.restart = 1;
          S.prev_rel = 1.0;
          S.phase = BP_INIT;
          break;
        }
      }
      S.prev_rel = rel;
      if (!isfinite(rel)) {
        S.status = WH_EUNSTABLE;
        S.phase = BP_DONE;
      } else if (rel <= D.tol) {
        S.status = WH_OK;
        S.phase = BP_DONE;
      } else if (S.iters >= D.max_iters) {
        S.status = WH_ENOCONV;
        S.phase = BP_DONE;
      } else {
        S.phase = BP_UPD2;
      }
      break;
    }
    default: break;
  }
}

__global__ void k_batch_count(const BState* states, int nb, int* remaining) {
  int c = 0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) c += states[i].phase != BP_DONE;
  __shared__ int sm[256];
  sm[threadIdx.x] = c;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sm[threadIdx.x] += sm[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) remaining[0] = sm[0];
}

// ------------------------------------------------------------------ host side

static bool batch_k_ok(int K) { return K == 2 || K == 4 || K == 8; }

// Second stream of a round: the FP64 work kernel runs beside the FP32 one.  Every problem
// is in one phase, and the plan gives each problem's tiles to exactly one of the two kernels,
// so the two write disjoint data; both only read the states, which the control kernel updates
// after both have finished.
struct RoundFork {
  hipStream_t s2 = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};

// Persistent grid of a work kernel: the blocks that fit on the device at once (a multiple of
// 8, one share per XCD).
template <typename T, int K, bool VARC, int TAG>
static int work_grid() {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_batch_work<T, K, VARC, TAG>, 64 * kBW, 0) !=
          hipSuccess)
    return 512;
  const int g = (std::max(1, cus * per) / 8) * 8;
  return std::max(8, g);
}

struct BatchGrids {
  int g64 = 512;   // persistent blocks of the FP64 work kernel (mixed batches)
};

template <int K, bool VARC>
static BatchGrids batch_grids_k() {
  return BatchGrids{work_grid<double, K, VARC, 0>()};
}

static BatchGrids batch_grids(int K, bool varc) {
  switch (K) {
    case 2: return varc ? batch_grids_k<2, true>() : batch_grids_k<2, false>();
    case 4: return varc ? batch_grids_k<4, true>() : batch_grids_k<4, false>();
    default: return varc ? batch_grids_k<8, true>() : batch_grids_k<8, false>();
  }
}

// What the launches of a round need.
struct RoundArgs {
  const BDesc* descs;
  BState* states;
  int* plan;
  const int* tiles;
  int ntiles, nb;
  bool mixed;
  BatchGrids grids;
  bool ord4;   // fourth-order differences (c == 1): K/2 steps per stepping launch
  bool pair;   // interleaved FP32 state pairs
};

template <int K, bool VARC, int ORD>
static void launch_round_ko(const RoundArgs& a, hipStream_t s, const RoundFork* rf) {
  const dim3 b(64, kBW);
  const BState* st = a.states;
  if (!a.mixed) {
    // FP64 batch: every phase is FP64, one tile per block
    hipLaunchKernelGGL((k_batch_tile<double, K, VARC, 0, ORD>), dim3(a.ntiles), b, 0, s, a.descs, st, a.tiles,
                       a.ntiles, 0);
    return;
  }
  // mixed batch: the FP32 stepping tiles one per block, and beside them the plan of the round
  // and the few FP64 and element-wise tiles by persistent blocks over it.  The FP32 kernel,
  // which holds most rounds' critical path, is issued first (in a captured graph the kernel
  // issued second starts about 9 us later) and does not wait for the plan (it finds its tiles
  // through the static table; plan and FP32 kernel only read the states).
  hipStream_t s64 = s;
  if (rf) (void)hipEventRecord(rf->fork, s);
  if (!VARC && a.pair)
    hipLaunchKernelGGL((k_batch_tile<float, K, VARC, 0, ORD, true>), dim3(a.ntiles), b, 0, s, a.descs, st, a.tiles,
                       a.ntiles, 1);
  else
    hipLaunchKernelGGL((k_batch_tile<float, K, VARC, 0, ORD>), dim3(a.ntiles), b, 0, s, a.descs, st, a.tiles,
                       a.ntiles, 1);
  if (rf) {
    (void)hipStreamWaitEvent(rf->s2, rf->fork, 0);
    s64 = rf->s2;
  }
  hipLaunchKernelGGL(k_batch_plan, dim3(1), dim3(256), 0, s64, a.descs, st, a.nb, a.plan);
  hipLaunchKernelGGL((k_batch_work<double, K, VARC, 0, ORD>), dim3(a.grids.g64), b, 0, s64, a.descs, st, a.plan,
                     a.nb, 0);
  if (rf) {
    (void)hipEventRecord(rf->join, rf->s2);
    (void)hipStreamWaitEvent(s, rf->join, 0);
  }
}

template <int K, bool VARC>
static void launch_round_k(const RoundArgs& a, hipStream_t s, const RoundFork* rf) {
  if constexpr (!VARC) {
    if (a.ord4) return launch_round_ko<K, false, 4>(a, s, rf);
  }
  launch_round_ko<K, VARC, 2>(a, s, rf);
}

// Time steps of one stepping launch.
static int batch_steps(int K, bool ord4) { return ord4 ? K / 2 : K; }

// One round: the work kernels (in mixed batches after the round's plan, which runs beside the
// FP32 kernel) and the control kernel (phases advance).
static void launch_round(int K, bool varc, const RoundArgs& a, hipStream_t s, const RoundFork* rf = nullptr) {
  switch (K) {
    case 2: varc ? launch_round_k<2, true>(a, s, rf) : launch_round_k<2, false>(a, s, rf); break;
    case 4: varc ? launch_round_k<4, true>(a, s, rf) : launch_round_k<4, false>(a, s, rf); break;
    default: varc ? launch_round_k<8, true>(a, s, rf) : launch_round_k<8, false>(a, s, rf); break;
  }
  hipLaunchKernelGGL(k_batch_control, dim3(a.nb), dim3(256), 0, s, a.descs, a.states, batch_steps(K, a.ord4));
}

// The FP32 stepping kernel alone, under its measurement tag (wh_time_batch_kernel).
template <int K, bool VARC>
static void launch_work_tagged(const RoundArgs& a, hipStream_t s) {
  if (!VARC && a.pair)
    hipLaunchKernelGGL((k_batch_tile<float, K, VARC, 1, 2, true>), dim3(a.ntiles), dim3(64, kBW), 0, s, a.descs,
                       (const BState*)a.states, a.tiles, a.ntiles, 1);
  else
    hipLaunchKernelGGL((k_batch_tile<float, K, VARC, 1>), dim3(a.ntiles), dim3(64, kBW), 0, s, a.descs,
                       (const BState*)a.states, a.tiles, a.ntiles, 1);
}

static void launch_work_timing(int K, bool varc, const RoundArgs& a, hipStream_t s) {
  switch (K) {
    case 2: varc ? launch_work_tagged<2, true>(a, s) : launch_work_tagged<2, false>(a, s); break;
    case 4: varc ? launch_work_tagged<4, true>(a, s) : launch_work_tagged<4, false>(a, s); break;
    default: varc ? launch_work_tagged<8, true>(a, s) : launch_work_tagged<8, false>(a, s); break;
  }
}

static int tile_dim(int n, int K, int axis) {
  const int t = axis == 0 ? batch_txo(K) : batch_tyo();
  return (n - 1 + t - 1) / t;
}

struct BatchLayout {
  size_t total = 0;
  std::vector<size_t> off;  // per problem base offsets
  std::vector<size_t> bytes;
  size_t descs = 0, states = 0, tiles = 0, remaining = 0;
  int ntiles = 0;
};

// per problem: 4 state arrays + V, b, r, p, q (8N each), FP32 states (4 x 4N or 2 x 8N, mixed), kap64/fs64 (8N),
// kap32/fs32 (4N, mixed), partials (tiles).  The weight tables (2(N_t+1) doubles per problem) sit
// in one region after all problems.
static size_t problem_bytes(int n, int K, bool mixed, bool varc) {
  const size_t N = (size_t)(n + 1) * (n + 1);
  size_t b = 0;
  auto add = [&](size_t x) { b += (x + 255) & ~(size_t)255; };
  for (int i = 0; i < 4; ++i) add(8 * N);
  if (mixed) for (int i = 0; i < 4; ++i) add(4 * N);   // covers 2 x 8N as well
  for (int i = 0; i < 5; ++i) add(8 * N);
  if (varc) add(8 * N);
  add(8 * N);
  if (mixed) { if (varc) add(4 * N); add(4 * N); }
  add(8 * (size_t)tile_dim(n, K, 0) * tile_dim(n, K, 1));
  return b;
}

// Scratch of the deflated start of one problem (each deflated problem has its own, so the
// starts of all problems run without host synchronisation): sine tables, projection partials
// and the two coefficient sets.  The mode numbers and scales of all problems sit in two shared
// upload regions (2 n_defl ints and 2 n_defl doubles per problem).
static size_t defl_scratch_bytes(int n, int nd) {
  if (nd <= 0) return 0;
  Defl dl;
  dl.kind = WH_DEFL_SINE;
  dl.nd = nd;
  dl.dim = 2;
  dl.n = n;
  size_t b = 0;
  auto add = [&](size_t x) { b += (x + 255) & ~(size_t)255; };
  add(8 * (size_t)nd * 2 * (n + 1));
  add(8 * (size_t)defl_partial_blocks(dl) * nd);
  add(8 * (size_t)nd * 2);
  return b;
}

}  // namespace wh

using namespace wh;

namespace {

#define WHB_FAIL(ctx, code, ...)                                  \
  do {                                                            \
    char _b[512];                                                 \
    snprintf(_b, sizeof(_b), __VA_ARGS__);                        \
    if (ctx) (ctx)->err = _b;                                     \
    return (code);                                                \
  } while (0)

#define HIPB(ctx, call)                                                           \
  do {                                                                            \
    hipError_t _e = (call);                                                       \
    if (_e != hipSuccess)                                                         \
      WHB_FAIL(ctx, WH_EHIP, "%s failed: %s", #call, hipGetErrorString(_e));     \
  } while (0)

struct Prepared {
  std::vector<TimeParams> tp;
  std::vector<double> cmax;
};

wh_status batch_validate(wh_ctx* ctx, int32_t nb, const wh_problem* probs, const wh_params* P) {
  if (nb < 1 || !probs || !P) WHB_FAIL(ctx, WH_EINVAL, "need nb >= 1 problems and params");
  if (nb > kMaxBatch) WHB_FAIL(ctx, WH_EINVAL, "at most %d problems per batch", kMaxBatch);
  if (P->precision != WH_F64 && P->precision != WH_MIXED) WHB_FAIL(ctx, WH_EINVAL, "bad precision");
  if (P->solver != WH_CG && P->solver != WH_DCG)
    WHB_FAIL(ctx, WH_EUNSUPPORTED, "batched solves use CG or DCG");
  if (!(P->tol > 0)) WHB_FAIL(ctx, WH_EINVAL, "tol must be > 0");
  const bool varc0 = probs[0].c2 != nullptr;
  for (int i = 0; i < nb; ++i) {
    const wh_problem& q = probs[i];
    if (q.grid.dim != 2) WHB_FAIL(ctx, WH_EUNSUPPORTED, "batched solves are 2D (problem %d)", i);
    if (q.grid.order != 2 && q.grid.order != 4)
      WHB_FAIL(ctx, WH_EUNSUPPORTED, "order must be 2 or 4 (problem %d)", i);
    if (q.grid.order != probs[0].grid.order)
      WHB_FAIL(ctx, WH_EUNSUPPORTED, "all problems of a batch must have one order (problem %d)", i);
    if (q.grid.order == 4 && q.c2)
      WHB_FAIL(ctx, WH_EUNSUPPORTED, "fourth-order differences need c == 1 (problem %d)", i);
    // the work kernels address each node array with 32-bit byte offsets
    if (q.grid.n < 4 || q.grid.n > 16000) WHB_FAIL(ctx, WH_EINVAL, "n must lie in [4, 16000] (problem %d)", i);
    if (!(q.omega > 0)) WHB_FAIL(ctx, WH_EINVAL, "omega must be > 0 (problem %d)", i);
    if (!q.f || !q.u) WHB_FAIL(ctx, WH_EINVAL, "f / u is NULL (problem %d)", i);
    if ((q.c2 != nullptr) != varc0)
      WHB_FAIL(ctx, WH_EUNSUPPORTED, "all problems of a batch must have c2 or none");
    if (q.n_defl < 0 || (int64_t)q.n_defl > (int64_t)(q.grid.n - 1) * (q.grid.n - 1))
      WHB_FAIL(ctx, WH_EINVAL, "bad n_defl (problem %d)", i);
    if (q.n_defl > 0 && P->solver != WH_DCG)
      WHB_FAIL(ctx, WH_EINVAL, "n_defl > 0 needs solver WH_DCG (problem %d)", i);
    if (q.n_defl > 0 && q.c2)
      WHB_FAIL(ctx, WH_EUNSUPPORTED, "sine-mode deflation needs c == 1 (problem %d)", i);
  }
  if (varc0 && !(P->c_max > 0))
    WHB_FAIL(ctx, WH_EINVAL, "batched solves with variable c need params->c_max > 0");
  return WH_OK;
}

int batch_K(const wh_params* P) { return batch_k_ok(P->k_fuse) ? P->k_fuse : 4; }

// Copy host data to the device through the context's pinned block (synchronous).
wh_status stage_to_device(wh_ctx* ctx, void* dev, const void* host, size_t bytes, hipStream_t s) {
  const size_t chunk = sizeof(double) * (size_t)ctx->hbuf_len;
  for (size_t o = 0; o < bytes; o += chunk) {
    const size_t cnt = std::min(bytes - o, chunk);
    HIPB(ctx, hipStreamSynchronize(s));
    std::memcpy(ctx->hbuf, (const char*)host + o, cnt);
    HIPB(ctx, hipMemcpyAsync((char*)dev + o, ctx->hbuf, cnt, hipMemcpyHostToDevice, s));
  }
  HIPB(ctx, hipStreamSynchronize(s));
  return WH_OK;
}

// Deflated start of one c = 1 problem: with the n_defl sine modes phi_k nearest
// omega^2 (eigenvectors of L_h, L_h phi_k = -lambda_k^2 phi_k, and of A with
// mu_k = 1 - beta_h(lambda_k^2)), the fixed point's coefficients are
// c_k = phi_k^T f / (omega_fp^2 - lambda_k^2); x = sum c_k phi_k, q = A x = sum mu_k c_k phi_k.
// Host part: the modes (2 nd ints) and the two scale vectors (2 nd doubles: -1/den, -mu/den;
// launch_defl_combine subtracts sum_k slot_k phi_k, so the coefficients are stored negated).
wh_status deflated_start_host(wh_ctx* ctx, const wh_problem& pr, const TimeParams& tp, int32_t* modes,
                              double* sc) {
  const int n = pr.grid.n, nd = pr.n_defl;
  std::vector<double> lam2(nd);
  if (wh_select_sine_modes(2, n, pr.grid.order, pr.omega, nd, modes, lam2.data()) != WH_OK)
    WHB_FAIL(ctx, WH_EINVAL, "sine mode selection failed (n = %d, n_defl = %d)", n, nd);
  // the frequency whose Helmholtz problem the fixed point solves: (2/dt) sin(omega_w dt / 2)
  const double sh = std::sin(0.5 * tp.omega_w * tp.dt);
  const double om2 = 4.0 * sh * sh / (tp.dt * tp.dt);
  for (int k = 0; k < nd; ++k) {
    const double den = om2 - lam2[k];
    if (den == 0.0) WHB_FAIL(ctx, WH_EBREAKDOWN, "sine mode %d is at resonance", k);
    const double mu = 1.0 - transfer(tp, lam2[k]);
    sc[k] = -1.0 / den;
    sc[nd + k] = -mu / den;
  }
  return WH_OK;
}

// Device part, from the uploaded modes and scales, in the problem's own scratch (no host
// synchronisation): the sine tables, the projections of f, the coefficients, x and q = A x.
// x and q must be zero on entry.
struct DeflScratch {
  double* tab = nullptr;
  double* partials = nullptr;
  double* coef = nullptr;
  int32_t* modes = nullptr;   // in the shared upload region
  double* scales = nullptr;
};

void deflated_start_launch(const wh_problem& pr, BDesc& d, const DeflScratch& w, hipStream_t s) {
  const int n = pr.grid.n, nd = pr.n_defl;
  const int64_t N = (int64_t)(n + 1) * (n + 1);
  Defl dl;
  dl.kind = WH_DEFL_SINE;
  dl.nd = nd;
  dl.dim = 2;
  dl.n = n;
  const int blocks = defl_partial_blocks(dl);
  launch_sine_tables(w.tab, w.modes, nd, 2, n, s);
  dl.tab = w.tab;
  launch_defl_project(dl, pr.f, w.partials, s);
  launch_defl_reduce(w.partials, blocks, nd, w.coef, 0, w.scales, s);
  launch_defl_reduce(w.partials, blocks, nd, w.coef, nd, w.scales + nd, s);
  launch_defl_combine(dl, d.x, 1.0, nullptr, 0.0, w.coef, 0, N, s);
  launch_defl_combine(dl, d.q, 1.0, nullptr, 0.0, w.coef, nd, N, s);
  d.x0 = 1;
}

// Extra streams of the set-up (default priority), released when it ends: the deflated starts
// are short launches bound by launch latency, so problems alternate over these streams.
struct AuxStreams {
  static constexpr int kMax = 4;
  hipStream_t st[kMax] = {};
  hipEvent_t join[kMax] = {};
  hipEvent_t fork = nullptr;
  int m = 0;
  AuxStreams() {
    if (hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess) {
      fork = nullptr;
      return;
    }
    while (m < kMax && hipStreamCreateWithFlags(&st[m], hipStreamNonBlocking) == hipSuccess) {
      if (hipEventCreateWithFlags(&join[m], hipEventDisableTiming) != hipSuccess) {
        (void)hipStreamDestroy(st[m]);
        st[m] = nullptr;
        join[m] = nullptr;
        break;
      }
      ++m;
    }
  }
  ~AuxStreams() {
    for (int k = 0; k < m; ++k) {
      (void)hipEventDestroy(join[k]);
      (void)hipStreamDestroy(st[k]);
    }
    if (fork) (void)hipEventDestroy(fork);
  }
};

// Validation, workspace carving, coefficient arrays, zeroed states, weight tables, deflated
// starts, and the descriptors, tile table and initial states on the device: everything a
// batched solve (or a timing of its work kernel) needs before the first round.
struct BatchSetup {
  std::vector<TimeParams> tps;
  std::vector<BDesc> D;
  int ntiles = 0, K = 4;
  bool mixed = false, varc = false, ord4 = false, pair = false;
  BDesc* ddesc = nullptr;
  BState* dstate = nullptr;
  int* dplan = nullptr;      // the two class plans of the next round (plan_stride(nb) ints each)
  int* dtiles = nullptr;     // block -> problem of every tile (one-tile-per-block kernels)
  int* dremain = nullptr;
  BatchGrids grids;
};

wh_status prepare_batch(wh_ctx* ctx, int32_t nb, const wh_problem* probs, const wh_params* params,
                        void* ws, size_t ws_bytes, BatchSetup& B) {
  wh_status vs = batch_validate(ctx, nb, probs, params);
  if (vs != WH_OK) return vs;
  const size_t need = wh_workspace_bytes_batched(nb, probs, params);
  if (!ws || ((uintptr_t)ws & 255)) WHB_FAIL(ctx, WH_EWORKSPACE, "workspace NULL or misaligned");
  if (ws_bytes < need) WHB_FAIL(ctx, WH_EWORKSPACE, "workspace too small: %zu < %zu", ws_bytes, need);
  HIPB(ctx, hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  const bool mixed = params->precision == WH_MIXED;
  const bool varc = probs[0].c2 != nullptr;
  char* base = (char*)ws;
  size_t cur_off = 0;
  auto take = [&](size_t bytes) {
    size_t o = cur_off;
    cur_off += (bytes + 255) & ~(size_t)255;
    return (void*)(base + o);
  };
  // time parameters (c = 1, or the caller's c_max bound for variable c)
  double* red = (double*)take(16 * (size_t)kReduceBlocks);
  (void)red;
  std::vector<TimeParams> tps(nb);
  for (int i = 0; i < nb; ++i) {
    const double cmax = params->c_max > 0 ? params->c_max : 1.0;
    wh_params p = *params;
    p.omega = probs[i].omega;
    wh_status st = make_time_params(ctx, 2, probs[i].grid.n, p, cmax, tps[i], probs[i].grid.order);
    if (st != WH_OK) return st;
  }
  const int K = batch_K(params);
  // FP32 A-apply: the defect form for undeflated problems (near-resonant modes present), direct
  // stepping when the near-resonant modes are deflated (second order only, as in the single
  // solves).  A batch whose FP32 steps are never forced keeps each FP32 state pair in one
  // interleaved array (one 8-byte access per node and row: 724 -> 696 us per launch on the
  // 256-problem batch); with forced steps the interleaved form ran slower (1013 -> 1118 us),
  // so such batches keep two arrays.
  auto defect_of = [&](int i) {
    return probs[i].grid.order == 2 &&
           (params->mixed_form == 0 || (params->mixed_form < 0 && probs[i].n_defl == 0));
  };
  bool pair = mixed && !varc;
  for (int i = 0; i < nb && pair; ++i) pair = !defect_of(i);
  // pass 1: carve the workspace (no device writes until the layout is known to fit)
  std::vector<BDesc> D(nb);
  std::vector<int> tile_solve;
  const size_t probs_begin = cur_off;   // the problems' arrays, zeroed by one fill
  for (int i = 0; i < nb; ++i) {
    const int n = probs[i].grid.n;
    const size_t N = (size_t)(n + 1) * (n + 1);
    BDesc& d = D[i];
    std::memset(&d, 0, sizeof(d));
    d.n = n;
    d.nt = tps[i].nt;
    d.ntx = tile_dim(n, K, 0);
    d.nty = tile_dim(n, K, 1);
    d.tile0 = (int)tile_solve.size();
    for (int t = 0; t < d.ntx * d.nty; ++t) tile_solve.push_back(i);
    d.mixed = mixed;
    d.max_iters = params->max_iters > 0 ? params->max_iters : 10000;
    d.max_outer = params->max_outer > 0 ? params->max_outer : 30;
    const double h = 1.0 / n;
    d.a = tps[i].dt * tps[i].dt / (h * h);
    d.tol = params->tol;
    // deflated problems tolerate long FP32 stretches: 1e-4 per replacement needs 2 residual
    // replacements (FP64 wave solves) per problem where 1e-3 needs 3 (256-problem batch: 512
    // instead of 768 besides the 256 right-hand sides, same iterations)
    d.itol = (params->inner_tol > 0 && params->inner_tol < 1) ? params->inner_tol
                                                              : (probs[i].n_defl > 0 ? 1e-4 : 0.1);
    d.defect = defect_of(i);
    d.om2dt2 = 4.0 * std::sin(0.5 * tps[i].omega_w * tps[i].dt) * std::sin(0.5 * tps[i].omega_w * tps[i].dt);
    for (int k = 0; k < 4; ++k) d.W[k] = take(8 * N);
    if (mixed && pair) {
      for (int k = 0; k < 2; ++k) {
        // interleaved FP32 pair k: W^n (slot 2k+1) at 8 bytes per node, D (slot 2k) 4 after
        char* pk = (char*)take(8 * N);
        d.W32[2 * k + 1] = pk;
        d.W32[2 * k] = pk + 4;
      }
    } else if (mixed) {
      for (int k = 0; k < 4; ++k) d.W32[k] = take(4 * N);
    }
    d.V = (double*)take(8 * N);
    d.b = (double*)take(8 * N);
    d.r = (double*)take(8 * N);
    d.p = (double*)take(8 * N);
    d.q = (double*)take(8 * N);
    d.x = probs[i].u;
    double* kap64 = varc ? (double*)take(8 * N) : nullptr;
    double* fs64 = (double*)take(8 * N);
    float* kap32 = (mixed && varc) ? (float*)take(4 * N) : nullptr;
    float* fs32 = mixed ? (float*)take(4 * N) : nullptr;
    d.kap64 = kap64;
    d.fs64 = fs64;
    d.kap32 = kap32;
    d.fs32 = fs32;
    d.partials = (double*)take(8 * (size_t)d.ntx * d.nty);
  }
  const size_t probs_end = cur_off;
  // weight tables of all problems (w then cos, N_t + 1 each), uploaded in one copy
  size_t wtot = 0;
  for (int i = 0; i < nb; ++i) wtot += 2 * (size_t)(D[i].nt + 1);
  double* wall = (double*)take(8 * wtot);
  {
    size_t o = 0;
    for (int i = 0; i < nb; ++i) {
      D[i].w = wall + o;
      D[i].cosv = wall + o + D[i].nt + 1;
      o += 2 * (size_t)(D[i].nt + 1);
    }
  }
  // deflated starts: per-problem scratch, and the shared upload regions of modes and scales
  std::vector<DeflScratch> dsc(nb);
  size_t ndt = 0;
  for (int i = 0; i < nb; ++i) {
    const int nd = probs[i].n_defl, n = probs[i].grid.n;
    if (nd <= 0) continue;
    Defl dl;
    dl.kind = WH_DEFL_SINE;
    dl.nd = nd;
    dl.dim = 2;
    dl.n = n;
    dsc[i].tab = (double*)take(8 * (size_t)nd * 2 * (n + 1));
    dsc[i].partials = (double*)take(8 * (size_t)defl_partial_blocks(dl) * nd);
    dsc[i].coef = (double*)take(8 * (size_t)nd * 2);
    ndt += 2 * (size_t)nd;
  }
  int32_t* modes_all = (int32_t*)take(4 * ndt);
  double* scales_all = (double*)take(8 * ndt);
  {
    size_t o = 0;
    for (int i = 0; i < nb; ++i) {
      if (probs[i].n_defl <= 0) continue;
      dsc[i].modes = modes_all + o;
      dsc[i].scales = scales_all + o;
      o += 2 * (size_t)probs[i].n_defl;
    }
  }
  const int ntiles = (int)tile_solve.size();
  BDesc* ddesc = (BDesc*)take(sizeof(BDesc) * nb);
  BState* dstate = (BState*)take(sizeof(BState) * nb);
  int* dplan = (int*)take(4 * (2 * (size_t)plan_stride(nb) + 16));
  int* dtiles = (int*)take(4 * (size_t)ntiles);
  int* dremain = (int*)take(256);
  if (cur_off > ws_bytes) WHB_FAIL(ctx, WH_EWORKSPACE, "workspace too small (layout %zu)", cur_off);
  // host part of the deflated starts (mode selection can fail: before any device write)
  std::vector<int32_t> hmodes(ndt);
  std::vector<double> hscales(ndt);
  {
    size_t o = 0;
    for (int i = 0; i < nb; ++i) {
      if (probs[i].n_defl <= 0) continue;
      wh_status ds = deflated_start_host(ctx, probs[i], tps[i], hmodes.data() + o, hscales.data() + o);
      if (ds != WH_OK) return ds;
      o += 2 * (size_t)probs[i].n_defl;
    }
  }
  // pass 2 (stream-ordered, no host synchronisation until the end): zeroed states, coefficient
  // arrays, the weight tables, the deflated starts
  HIPB(ctx, hipMemsetAsync(base + probs_begin, 0, probs_end - probs_begin, s));
  for (int i = 0; i < nb; ++i) {
    const int n = probs[i].grid.n;
    const size_t N = (size_t)(n + 1) * (n + 1);
    const double h = 1.0 / n;
    BDesc& d = D[i];
    const double dt2 = tps[i].dt * tps[i].dt;
    const double ks = dt2 / (2.0 * h * h);
    launch_prep_coeffs(probs[i].c2, probs[i].f, (double*)d.kap64, (double*)d.fs64, false, ks, dt2, (int64_t)N, n, 2,
                       s);
    if (mixed)
      launch_prep_coeffs(probs[i].c2, probs[i].f, (float*)d.kap32, (float*)d.fs32, true, ks, dt2, (int64_t)N, n, 2,
                         s);
    HIPB(ctx, hipMemsetAsync(d.x, 0, 8 * N, s));   // batched solves start from zero
  }
  // (copies from pageable host memory return once the data is staged)
  std::vector<double> tab(wtot);
  {
    size_t o = 0;
    for (int i = 0; i < nb; ++i) {
      const int nt = D[i].nt;
      for (int k = 0; k <= nt; ++k) {
        tab[o + k] = tps[i].w[k];
        tab[o + nt + 1 + k] = tps[i].cosv[k];
      }
      o += 2 * (size_t)(nt + 1);
    }
  }
  HIPB(ctx, hipMemcpyAsync(wall, tab.data(), 8 * wtot, hipMemcpyHostToDevice, s));
  if (ndt) {
    HIPB(ctx, hipMemcpyAsync(modes_all, hmodes.data(), 4 * ndt, hipMemcpyHostToDevice, s));
    HIPB(ctx, hipMemcpyAsync(scales_all, hscales.data(), 8 * ndt, hipMemcpyHostToDevice, s));
  }
  if (ndt) {
    // the deflated starts on the extra streams (each problem has its own scratch), joined back
    // into the set-up stream
    AuxStreams aux;
    if (aux.m > 0) {
      HIPB(ctx, hipEventRecord(aux.fork, s));
      for (int k = 0; k < aux.m; ++k) HIPB(ctx, hipStreamWaitEvent(aux.st[k], aux.fork, 0));
    }
    int q = 0;
    for (int i = 0; i < nb; ++i)
      if (probs[i].n_defl > 0) deflated_start_launch(probs[i], D[i], dsc[i], aux.m > 0 ? aux.st[q++ % aux.m] : s);
    for (int k = 0; k < aux.m; ++k) {
      HIPB(ctx, hipEventRecord(aux.join[k], aux.st[k]));
      HIPB(ctx, hipStreamWaitEvent(s, aux.join[k], 0));
    }
    HIPB(ctx, hipStreamSynchronize(s));
  }
  // upload descriptors, tile table and the initial states (synchronous copies from host memory)
  HIPB(ctx, hipMemcpyAsync(ddesc, D.data(), sizeof(BDesc) * nb, hipMemcpyHostToDevice, s));
  HIPB(ctx, hipMemcpyAsync(dtiles, tile_solve.data(), 4 * (size_t)ntiles, hipMemcpyHostToDevice, s));
  std::vector<BState> S0(nb);
  std::memset(S0.data(), 0, sizeof(BState) * nb);
  for (auto& st : S0) st.phase = BP_B_FIRST;
  HIPB(ctx, hipMemcpyAsync(dstate, S0.data(), sizeof(BState) * nb, hipMemcpyHostToDevice, s));
  // the plan of the first round
  hipLaunchKernelGGL(k_batch_plan, dim3(1), dim3(256), 0, s, (const BDesc*)ddesc, (const BState*)dstate, nb, dplan);
  HIPB(ctx, hipStreamSynchronize(s));
  HIPB(ctx, hipGetLastError());
  B.tps = std::move(tps);
  B.D = std::move(D);
  B.ntiles = ntiles;
  B.K = K;
  B.mixed = mixed;
  B.varc = varc;
  B.ord4 = probs[0].grid.order == 4;
  B.pair = pair;
  B.ddesc = ddesc;
  B.dstate = dstate;
  B.dplan = dplan;
  B.dtiles = dtiles;
  B.grids = batch_grids(K, varc);
  B.dremain = dremain;
  return WH_OK;
}

}  // namespace

extern "C" {

size_t wh_workspace_bytes_batched(int32_t nb, const wh_problem* probs, const wh_params* params) {
  return guard_size([&]() -> size_t {
  if (batch_validate(nullptr, nb, probs, params) != WH_OK) return 0;
  const bool mixed = params->precision == WH_MIXED;
  const bool varc = probs[0].c2 != nullptr;
  const int K = batch_K(params);
  const double cmax = params->c_max > 0 ? params->c_max : 1.0;
  size_t total = 0, wtot = 0;
  for (int i = 0; i < nb; ++i) {
    wh_params p = *params;
    p.omega = probs[i].omega;
    TimeParams tp;
    if (make_time_params(nullptr, 2, probs[i].grid.n, p, cmax, tp, probs[i].grid.order) != WH_OK) return 0;
    total += problem_bytes(probs[i].grid.n, K, mixed, varc);
    wtot += 2 * (size_t)(tp.nt + 1);
  }
  total += (8 * wtot + 255) & ~(size_t)255;
  size_t ndt = 0;
  for (int i = 0; i < nb; ++i) {
    total += defl_scratch_bytes(probs[i].grid.n, probs[i].n_defl);
    ndt += 2 * (size_t)std::max(0, probs[i].n_defl);
  }
  total += ((4 * ndt + 255) & ~(size_t)255) + ((8 * ndt + 255) & ~(size_t)255);
  total += 16 * (size_t)kReduceBlocks;  // c_max reductions (multiple of 256)
  total += ((sizeof(BDesc) * nb + 255) & ~(size_t)255) + ((sizeof(BState) * nb + 255) & ~(size_t)255);
  total += ((4 * (2 * (size_t)plan_stride(nb) + 16) + 255) & ~(size_t)255) + 256;
  size_t ntl = 0;
  for (int i = 0; i < nb; ++i) ntl += (size_t)tile_dim(probs[i].grid.n, K, 0) * tile_dim(probs[i].grid.n, K, 1);
  total += (4 * ntl + 255) & ~(size_t)255;
  return total;
  });
}

wh_status wh_solve_batched(wh_ctx* ctx, int32_t nb, const wh_problem* probs,
                           const wh_params* params, void* ws, size_t ws_bytes, wh_info* infos) {
  return guard(ctx, [&]() -> wh_status {
  if (!ctx) return WH_EINVAL;
  const auto t0 = std::chrono::steady_clock::now();
  BatchSetup B;
  {
    const wh_status ps = prepare_batch(ctx, nb, probs, params, ws, ws_bytes, B);
    if (ps != WH_OK) return ps;
  }
  hipStream_t s = ctx->stream;
  const bool mixed = B.mixed;
  const bool varc = B.varc;
  const int K = B.K;
  std::vector<BDesc>& D = B.D;
  std::vector<TimeParams>& tps = B.tps;
  BDesc* ddesc = B.ddesc;
  BState* dstate = B.dstate;
  int* dplan = B.dplan;
  int* dremain = B.dremain;

  // Capture G rounds + the counter in a graph on a private stream, twice (two
  // executables whose counters go to different slots).  Replays alternate between
  // them and the host keeps one replay queued ahead: it reads the counter of replay
  // k while replay k+1 runs, so the GPU does not wait for the host between replays.
  // Rounds of finished problems return at once, so the replay that runs past the
  // end costs little.
  const int G = 32;
  hipStream_t cs;
  HIPB(ctx, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  RoundFork rf;
  bool use_fork = hipStreamCreateWithFlags(&rf.s2, hipStreamNonBlocking) == hipSuccess;
  use_fork = use_fork && hipEventCreateWithFlags(&rf.fork, hipEventDisableTiming) == hipSuccess;
  use_fork = use_fork && hipEventCreateWithFlags(&rf.join, hipEventDisableTiming) == hipSuccess;
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  hipEvent_t ev[2] = {nullptr, nullptr};
  int* dcount[2] = {dremain, dremain + 32};
  hipError_t e = hipSuccess;
  for (int gi = 0; gi < 2 && e == hipSuccess; ++gi) {
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      for (int g = 0; g < G; ++g)
        launch_round(K, varc, RoundArgs{ddesc, dstate, dplan, B.dtiles, B.ntiles, nb, mixed, B.grids, B.ord4, B.pair}, cs,
                     use_fork ? &rf : nullptr);
      hipLaunchKernelGGL(k_batch_count, dim3(1), dim3(256), 0, cs, (const BState*)dstate, nb, dcount[gi]);
      e = hipStreamEndCapture(cs, &graph[gi]);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&exec[gi], graph[gi], nullptr, nullptr, 0);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev[gi], hipEventDisableTiming);
  }
  auto release = [&]() {
    for (int gi = 0; gi < 2; ++gi) {
      if (exec[gi]) (void)hipGraphExecDestroy(exec[gi]);
      if (graph[gi]) (void)hipGraphDestroy(graph[gi]);
      if (ev[gi]) (void)hipEventDestroy(ev[gi]);
    }
    if (rf.fork) (void)hipEventDestroy(rf.fork);
    if (rf.join) (void)hipEventDestroy(rf.join);
    if (rf.s2) (void)hipStreamDestroy(rf.s2);
    (void)hipStreamDestroy(cs);
  };
  if (e != hipSuccess) {
    release();
    WHB_FAIL(ctx, WH_EHIP, "graph capture failed: %s", hipGetErrorString(e));
  }
  // bound on replays: every problem needs at most max_iters iterations of
  // (N_t/K + 6) rounds plus its outer sweeps
  long long max_rounds = 0;
  for (int i = 0; i < nb; ++i) {
    const int ks = batch_steps(K, B.ord4);
    const long long per_it = (D[i].nt + ks - 1) / ks + 6;
    // an iteration is at most one A wave solve plus one residual replacement
    max_rounds = std::max(max_rounds, (long long)D[i].max_iters * 2 * per_it + 2 * per_it + 8);
  }
  const long long max_replays = max_rounds / G + 2;
  // host slots for the two counters in the pinned block
  int* hcount[2] = {(int*)ctx->hbuf, (int*)(ctx->hbuf + 8)};
  auto enqueue = [&](long long r) -> hipError_t {
    const int k = (int)(r & 1);
    hipError_t er = hipGraphLaunch(exec[k], s);
    if (er == hipSuccess) er = hipMemcpyAsync(hcount[k], dcount[k], sizeof(int), hipMemcpyDeviceToHost, s);
    if (er == hipSuccess) er = hipEventRecord(ev[k], s);
    return er;
  };
  long long launched = 0, checked = 0;
  int remaining = nb;
  wh_status st = WH_OK;
  e = enqueue(launched++);
  while (e == hipSuccess && checked < launched) {
    // keep the next replay queued before waiting for the current one
    if (launched < max_replays) {
      e = enqueue(launched++);
      if (e != hipSuccess) break;
    }
    const int k = (int)(checked & 1);
    e = hipEventSynchronize(ev[k]);
    if (e != hipSuccess) break;
    std::memcpy(&remaining, hcount[k], sizeof(int));
    ++checked;
    if (remaining == 0) break;
  }
  // the replay queued past the end (if any) must finish before the states are read
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  release();
  if (e != hipSuccess) WHB_FAIL(ctx, WH_EHIP, "batched replay failed: %s", hipGetErrorString(e));
  // results
  std::vector<BState> SF(nb);
  HIPB(ctx, hipMemcpyAsync(SF.data(), dstate, sizeof(BState) * nb, hipMemcpyDeviceToHost, s));
  HIPB(ctx, hipStreamSynchronize(s));
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  for (int i = 0; i < nb; ++i) {
    int status = SF[i].phase == BP_DONE ? SF[i].status : WH_ENOCONV;
    if (status < 0 && st >= 0) st = (wh_status)status;
    else if (status == WH_ENOCONV && st == WH_OK) st = WH_ENOCONV;
    if (infos) {
      wh_info& in = infos[i];
      std::memset(&in, 0, sizeof(in));
      in.status = status;
      in.iters = SF[i].iters;
      in.outer = mixed ? SF[i].outer : 0;
      const int wsol = SF[i].iters + SF[i].outer + 1;  // A applies + residual solves + b
      const int it64 = (int)SF[i].it64;
      in.wave_solves = mixed ? SF[i].outer + 1 + it64 : wsol;
      in.wave_solves_f32 = mixed ? SF[i].iters - it64 : 0;
      in.nt = tps[i].nt;
      in.m = tps[i].m;
      in.k_fuse = K;
      in.k_rows = kBSeg;
      in.k_waves = kBW;
      in.rel_res = SF[i].rel;
      in.true_rel_res = mixed ? SF[i].rel : SF[i].pq;
      in.omega_tilde = tps[i].omega_w;
      in.dt = tps[i].dt;
      in.c_max = tps[i].c_max;
      in.ms = ms;
    }
  }
  if (st == WH_ENOCONV) ctx->err = "some batched problems did not reach the tolerance";
  return st;
  });
}

wh_status wh_time_batch_kernel(wh_ctx* ctx, int32_t nb, const wh_problem* probs, const wh_params* params,
                               int32_t reps, void* ws, size_t ws_bytes, double* us_per_launch, int64_t* points) {
  return guard(ctx, [&]() -> wh_status {
  if (!ctx) return WH_EINVAL;
  if (reps < 1 || !us_per_launch) WHB_FAIL(ctx, WH_EINVAL, "reps must be >= 1 and us_per_launch set");
  if (!params || params->precision != WH_MIXED)
    WHB_FAIL(ctx, WH_EINVAL, "the FP32 work kernel is timed with params->precision = WH_MIXED");
  if (nb >= 1 && probs && probs[0].grid.order != 2)
    WHB_FAIL(ctx, WH_EUNSUPPORTED, "the work kernel is timed for second-order batches");
  BatchSetup B;
  {
    const wh_status ps = prepare_batch(ctx, nb, probs, params, ws, ws_bytes, B);
    if (ps != WH_OK) return ps;
  }
  hipStream_t s = ctx->stream;
  int64_t pts = 0;
  for (int i = 0; i < nb; ++i) {
    if (B.D[i].nt - 2 < B.K)
      WHB_FAIL(ctx, WH_EINVAL, "problem %d has fewer than K + 2 time steps (N_t = %d)", i, B.D[i].nt);
    pts += (int64_t)(B.D[i].n - 1) * (B.D[i].n - 1);
  }
  // every problem in the FP32 time-stepping phase of an A-apply, K steps per launch
  std::vector<BState> S(nb);
  std::memset(S.data(), 0, sizeof(BState) * nb);
  for (auto& st : S) {
    st.phase = BP_A_STEP;
    st.step = 1;
  }
  HIPB(ctx, hipMemcpyAsync(B.dstate, S.data(), sizeof(BState) * nb, hipMemcpyHostToDevice, s));
  const RoundArgs ra{B.ddesc, B.dstate, B.dplan, B.dtiles, B.ntiles, nb, true, B.grids, false, B.pair};
  auto one = [&]() { launch_work_timing(B.K, B.varc, ra, s); };
  HIPB(ctx, hipStreamSynchronize(s));
  one();
  hipEvent_t e0, e1;
  HIPB(ctx, hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    WHB_FAIL(ctx, WH_EHIP, "hipEventCreate failed");
  }
  (void)hipEventRecord(e0, s);
  for (int r = 0; r < reps; ++r) one();
  (void)hipEventRecord(e1, s);
  hipError_t e = hipEventSynchronize(e1);
  float ms = 0;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) WHB_FAIL(ctx, WH_EHIP, "event timing failed: %s", hipGetErrorString(e));
  *us_per_launch = 1e3 * (double)ms / reps;
  if (points) *points = pts;
  return WH_OK;
  });
}

}  // extern "C"
