// Temporally blocked 2D leapfrog + filter: K time steps per launch.
//
// Same scheme as the streaming kernels (Section 2.2, eq. discreteWaveExplicit with
// the trapezoid sum of eq. quadrature folded in), but each block of NW wavefronts
// keeps a 64-column x NW*R-row region of (W^n, W^{n-1}) in registers and advances
// it K steps before writing back.  Lane l of wave w owns column x0-K+l and rows
// y0-K+wR .. y0-K+wR+R-1.  Per step:
//   * x-neighbours come from the adjacent lanes (DPP wavefront shift, a VALU move),
//   * y-neighbours come from the thread's own rows, except the first/last row of
//     each wave, which are exchanged through a small double-buffered LDS array,
//   * points outside the open domain are held at zero (Dirichlet data).
// The valid region shrinks by one point per step on every side, so the block
// writes the inner (64-2K) x (NW*R-2K) tile: W^{n+K}, W^{n+K-1} and
// V + sum_s w_s W^{n+s}.  V is loaded together with the state, before the steps,
// so that its latency overlaps the other loads.
// HBM traffic per point and launch is 8 (state in) + 8 (state out) + 16 (V) bytes in
// FP32, i.e. 32/K bytes per point-step against 28 for the streaming kernel.
//
// Block shapes (R, NW): more waves per block and fewer rows per thread raise the
// number of resident waves (latency hiding); taller regions waste less halo.  The
// autotuner picks K and the shape per grid.
//
// FP32 pairs are (W^n, D^{n-1/2} = W^n - W^{n-1}) and step in the increment form
// D += dt^2 (L_h W - f cos), W += D, with the Laplacian summed as differences to the
// centre; FP64 pairs are (W^n, W^{n-1}).
//
// Inputs and outputs are distinct buffers (neighbouring blocks read the halo).
//
// The kernel is instantiated per phase of a wave solve: kPhaseFirst starts from the
// input W^0 with the half step, kPhaseMid carries the state through, kPhaseLast ends
// in the epilogue.  Each phase is compiled in its own translation unit.
#pragma once
#include "wh_common.h"
#include "wh_reduce.h"

namespace wh {

enum { kPhaseMid = 0, kPhaseFirst = 1, kPhaseLast = 2 };

struct FusedDev {
  const void* cur;
  const void* prev;
  void* cur_out;
  void* prev_out;
  double* V;
  const void* kap;
  const void* fs;
  double a;
  int n;
  int gx, gy;          // tile grid
  double w[16];        // w_{n+1..n+K}
  double cs[16];       // cos(omega_w t^{n..n+K-1})
  // first launch of a wave solve: W^0 = vin (FP64; NULL: 0), the first step is the half
  // step of D_0t W^0 = 0, and V starts as w0 W^0 (no state or V is read)
  const double* vin;
  double w0;
  // last launch: the final step ends in an epilogue instead of storing the state
  // (M_LAST_V: V; M_LAST_AQ: out = x - V; M_LAST_EQ: out = -V; M_LAST_FPI: out = V),
  // with per-block partial sums of x.out (AQ, EQ) or (out - x)^2 (FPI)
  int last;            // StepMode; M_MID for none
  const double* x;
  double* out;
  double* partials;
  // first launch, when dr is set: W^0 = dr + beta dp (beta = dslots[S_BETA]) instead of vin,
  // i.e. the CG direction update fused into the load; dout receives it over the interior
  const double* dr;
  const double* dp;
  const double* dslots;
  double* dout;
};

// Tile order that gives each XCD a contiguous run of tiles (blocks are dispatched
// round-robin over the 8 XCDs), so horizontally adjacent tiles share an L2.
__device__ __forceinline__ int xcd_tile(int bid, int nb) {
  const int xcd = bid & 7, idx = bid >> 3;
  const int q = nb >> 3, r = nb & 7;
  return xcd < r ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

template <typename T, int K, int R, int NW, bool VARC, bool FORCE, int PH>
__global__ __launch_bounds__(64 * NW) void k_fused2d(const FusedDev a) {
  constexpr int TXO = 64 - 2 * K;
  constexpr int TYO = NW * R - 2 * K;
  static_assert(TXO > 0 && TYO > 0, "tile too small for K");
  const int n = a.n;
  const int64_t P = (int64_t)n + 1;
  const int lane = threadIdx.x;
  const int wv = threadIdx.y;
  const int nb = a.gx * a.gy;
  const int t = xcd_tile(blockIdx.x, nb);
  const int tx = t % a.gx, ty = t / a.gx;
  const int x0 = 1 + tx * TXO;
  const int y0 = 1 + ty * TYO;
  const int xg = x0 - K + lane;
  const int yb = y0 - K + wv * R;
  const bool xin = xg >= 1 && xg <= n - 1;
  // lanes and rows of the inner tile (written back)
  const bool xout = lane >= K && lane < 64 - K && xin;

  const T* __restrict__ cin = (const T*)a.cur;
  const T* __restrict__ pin = (const T*)a.prev;
  const T* __restrict__ kap = (const T*)a.kap;
  const T* __restrict__ fsv = (const T*)a.fs;

  T cur[R], prv[R];
  double acc[R];
  T cw[VARC ? R : 1], ce[VARC ? R : 1], cu[VARC ? R : 1], cd[VARC ? R : 1];
  T frc[FORCE ? R : 1];
  uint32_t mask = 0, omask = 0;
  const double* __restrict__ Vin = a.V;
  constexpr bool first = PH == kPhaseFirst;
  // first launch: W^0 as loaded (FP64); converted only after every row's load has been
  // issued, so that the loads overlap instead of waiting one by one
  // (rows outside the domain load a valid interior node of the tile and discard it, so
  // the loads carry no branches)
  double v0[first ? R : 1];
  const bool dirupd = first && a.dr != nullptr;
  const double beta = dirupd ? a.dslots[S_BETA] : 0.0;
  const int64_t p_in = (int64_t)y0 * P + x0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int y = yb + r;
    const bool in = xin && y >= 1 && y <= n - 1;
    const int64_t p = (int64_t)y * P + xg;
    // boundary nodes hold the Dirichlet value 0: read interior nodes only
    if (!first) {
      cur[r] = in ? cin[p] : T(0);
      prv[r] = in ? pin[p] : T(0);
    }
    if (in) mask |= 1u << r;
    const int ry = wv * R + r;
    const bool o = in && xout && ry >= K && ry < NW * R - K;
    if (o) omask |= 1u << r;
    acc[r] = (o && !first) ? Vin[p] : 0.0;
    if (VARC) {
      T kc = T(0), kw = T(0), ke = T(0), ku = T(0), kd = T(0);
      if (in) {
        kc = kap[p];
        kw = kap[p - 1];
        ke = kap[p + 1];
        ku = kap[p - P];
        kd = kap[p + P];
      }
      cw[VARC ? r : 0] = kc + kw;
      ce[VARC ? r : 0] = kc + ke;
      cu[VARC ? r : 0] = kc + ku;
      cd[VARC ? r : 0] = kc + kd;
    }
    if (FORCE) frc[FORCE ? r : 0] = in ? fsv[p] : T(0);
  }
  if constexpr (first) {
    // one uniform branch around straight-line loads: every row's loads are issued before
    // the first is used
    if (dirupd) {
      double rv[R], pv[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int64_t ps = ((mask >> r) & 1u) ? (int64_t)(yb + r) * P + xg : p_in;
        rv[r] = a.dr[ps];
        pv[r] = a.dp[ps];
      }
#pragma unroll
      for (int r = 0; r < R; ++r) v0[r] = ((mask >> r) & 1u) ? rv[r] + beta * pv[r] : 0.0;
#pragma unroll
      for (int r = 0; r < R; ++r)
        if ((omask >> r) & 1u) a.dout[(int64_t)(yb + r) * P + xg] = v0[r];
    } else if (a.vin) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int64_t ps = ((mask >> r) & 1u) ? (int64_t)(yb + r) * P + xg : p_in;
        v0[r] = a.vin[ps];
      }
#pragma unroll
      for (int r = 0; r < R; ++r) v0[r] = ((mask >> r) & 1u) ? v0[r] : 0.0;
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r) v0[r] = 0.0;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      cur[r] = (T)v0[r];
      prv[r] = T(0);
      acc[r] = ((omask >> r) & 1u) ? a.w0 * v0[r] : 0.0;
    }
  }

  __shared__ T edge[2][NW][2][64];
  const T A = (T)a.a;
#pragma unroll
  for (int s = 0; s < K; ++s) {
    const int b = s & 1;
    edge[b][wv][0][lane] = cur[0];
    edge[b][wv][1][lane] = cur[R - 1];
    __syncthreads();
    const T up_e = wv > 0 ? edge[b][wv - 1][1][lane] : T(0);
    const T dn_e = wv < NW - 1 ? edge[b][wv + 1][0][lane] : T(0);
    const T cn = (T)a.cs[s];
    const double ws = a.w[s];
    if constexpr (sizeof(T) == 4) {
      // FP32 pair (W, D = W^n - W^{n-1}): D += dt^2 (L_h W - f cos), W += D.  Row r-1
      // is overwritten before row r reads it, so its old value is carried in uo.
      T uo = up_e;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const T c = cur[r];
        const T d = r < R - 1 ? cur[r + 1] : dn_e;
        const T w = from_prev_lane(c);
        const T e = from_next_lane(c);
        T lap;
        if (VARC) {
          const int q = VARC ? r : 0;
          lap = (cw[q] * (w - c) + ce[q] * (e - c)) + (cu[q] * (uo - c) + cd[q] * (d - c));
        } else {
          lap = A * (((w - c) + (e - c)) + ((uo - c) + (d - c)));
        }
        if (FORCE) lap -= cn * frc[FORCE ? r : 0];
        // first step of a wave solve: D^{1/2} = dt^2/2 (L_h W^0 - f)
        const T dsum = (first && s == 0) ? T(0.5) * lap : prv[r] + lap;
        // points outside the open domain keep W = D = 0: masking D suffices (W = 0 + 0),
        // and a bitwise AND keeps the update branch-free
        const T dn = __int_as_float(__float_as_int(dsum) & (int)(0u - ((mask >> r) & 1u)));
        const T nw = c + dn;
        prv[r] = dn;
        uo = c;
        cur[r] = nw;
        acc[r] += ws * (double)nw;
      }
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const T c = cur[r];
        const T u = r > 0 ? cur[r - 1] : up_e;
        const T d = r < R - 1 ? cur[r + 1] : dn_e;
        const T w = from_prev_lane(c);
        const T e = from_next_lane(c);
        T nw;
        if (first && s == 0) {
          // first step of a wave solve: W^1 = W^0 + dt^2/2 (L_h W^0 - f)
          T lap;
          if (VARC) {
            const int q = VARC ? r : 0;
            lap = (cw[q] * (w - c) + ce[q] * (e - c) + (cu[q] * (u - c) + cd[q] * (d - c)));
          } else {
            lap = A * (((w + e) + (u + d)) - T(4) * c);
          }
          if (FORCE) lap -= cn * frc[FORCE ? r : 0];
          nw = c + T(0.5) * lap;
        } else {
          if (VARC) {
            const int q = VARC ? r : 0;
            nw = (c + c) - prv[r] + (cw[q] * (w - c) + ce[q] * (e - c) + (cu[q] * (u - c) + cd[q] * (d - c)));
          } else {
            nw = (c + c) - prv[r] + A * (((w + e) + (u + d)) - T(4) * c);
          }
          if (FORCE) nw -= cn * frc[FORCE ? r : 0];
        }
        nw = ((mask >> r) & 1u) ? nw : T(0);
        prv[r] = nw;   // rows r+1.. still read the old cur[r]
        acc[r] += ws * (double)nw;
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const T tmp = cur[r];
        cur[r] = prv[r];
        prv[r] = tmp;
      }
    }
  }

  // boundary nodes of the result (V from the first launch on, out in the last) hold the
  // Dirichlet value 0; every block writes the ones it covers (repeated writes of 0)
  if constexpr (PH != kPhaseMid) {
    double* __restrict__ dst = (PH == kPhaseFirst || a.last == M_LAST_V) ? a.V : a.out;
    if (xg >= 0 && xg <= n) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int y = yb + r;
        if (y >= 0 && y <= n && (xg == 0 || xg == n || y == 0 || y == n)) dst[(int64_t)y * P + xg] = 0.0;
      }
    }
  }
  // write the inner tile (acc holds V + sum_s w_s W^{n+s})
  // the row addresses are formed again below rather than kept from the loads through the
  // time loop (an opaque copy of the row index stops the compiler from reusing them):
  // R 64-bit addresses per array held across the steps cost more registers than the
  // few instructions that recompute them
  int ys = yb;
  asm volatile("" : "+v"(ys));
  if constexpr (PH != kPhaseLast) {
    T* __restrict__ cout = (T*)a.cur_out;
    T* __restrict__ pout = (T*)a.prev_out;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if ((omask >> r) & 1u) {
        const int64_t p = (int64_t)(ys + r) * P + xg;
        cout[p] = cur[r];
        pout[p] = prv[r];
        a.V[p] = acc[r];
      }
    }
  } else {
    // last launch: epilogue of the wave solve on V = acc.  Every x value is loaded (rows
    // outside the tile read a valid in-grid node) before any is used, and every result is
    // formed before any store, so the block waits once for its loads.  With M_LAST_FPI x
    // and out may alias; each block reads x only where it writes out, before writing.
    double part = 0.0;
    double res[R];
    if (a.last == M_LAST_V) {
#pragma unroll
      for (int r = 0; r < R; ++r) res[r] = acc[r];
    } else {
      double xr[R];
      const int64_t p0 = (int64_t)y0 * P + x0;   // a node of this block's tile
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int64_t p = ((omask >> r) & 1u) ? (int64_t)(ys + r) * P + xg : p0;
        xr[r] = a.x[p];
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const bool o = (omask >> r) & 1u;
        const double vf = acc[r];
        const double xv = o ? xr[r] : 0.0;
        if (a.last == M_LAST_AQ) {
          res[r] = xv - vf;
          part += xv * res[r];
        } else if (a.last == M_LAST_EQ) {
          res[r] = -vf;
          part += xv * res[r];
        } else {   // M_LAST_FPI
          const double d = vf - xv;
          res[r] = vf;
          part += o ? d * d : 0.0;
        }
      }
    }
    double* __restrict__ dst = a.last == M_LAST_V ? a.V : a.out;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if ((omask >> r) & 1u) dst[(int64_t)(ys + r) * P + xg] = res[r];
    }
    if (a.last != M_LAST_V) {
      const double sum = block_sum<NW>(part, wv * 64 + lane);
      if (wv == 0 && lane == 0) a.partials[blockIdx.x] = sum;
    }
  }
}

template <typename T, int K, int R, int NW, int PH>
static void launch_krw(bool varc, bool force, FusedDev& d, hipStream_t s) {
  static_assert(NW * R - 2 * K > 0, "tile too small for K");
  const int n = d.n;
  d.gx = (n - 1 + (64 - 2 * K) - 1) / (64 - 2 * K);
  d.gy = (n - 1 + (NW * R - 2 * K) - 1) / (NW * R - 2 * K);
  dim3 g(d.gx * d.gy), b(64, NW);
  if (varc) {
    if (force) hipLaunchKernelGGL((k_fused2d<T, K, R, NW, true, true, PH>), g, b, 0, s, d);
    else hipLaunchKernelGGL((k_fused2d<T, K, R, NW, true, false, PH>), g, b, 0, s, d);
  } else {
    if (force) hipLaunchKernelGGL((k_fused2d<T, K, R, NW, false, true, PH>), g, b, 0, s, d);
    else hipLaunchKernelGGL((k_fused2d<T, K, R, NW, false, false, PH>), g, b, 0, s, d);
  }
}

template <typename T, int K, int PH>
static void launch_shape(int shape, bool varc, bool force, FusedDev& d, hipStream_t s) {
  if constexpr (sizeof(T) == 4) {
    // (rows per thread, waves per block) as listed by fused2d_shape_dims
    constexpr int R1 = K == 9 ? 9 : 8;
    if (shape == 0) launch_krw<T, K, 16, 4, PH>(varc, force, d, s);
    else if (shape == 1) launch_krw<T, K, R1, 8, PH>(varc, force, d, s);
    else launch_krw<T, K, 8, 4, PH>(varc, force, d, s);
  } else {
    if (shape == 0) launch_krw<T, K, 8, 4, PH>(varc, force, d, s);
    else if (shape == 1) launch_krw<T, K, 4, 8, PH>(varc, force, d, s);
    else launch_krw<T, K, 4, 16, PH>(varc, force, d, s);
  }
}

template <typename T, int PH>
static void launch_k(int k, int shape, bool varc, bool force, FusedDev& d, hipStream_t s) {
  switch (k) {
    case 2: launch_shape<T, 2, PH>(shape, varc, force, d, s); break;
    case 3: launch_shape<T, 3, PH>(shape, varc, force, d, s); break;
    case 4: launch_shape<T, 4, PH>(shape, varc, force, d, s); break;
    case 6: launch_shape<T, 6, PH>(shape, varc, force, d, s); break;
    case 8: launch_shape<T, 8, PH>(shape, varc, force, d, s); break;
    case 9:
      if constexpr (sizeof(T) == 4) launch_shape<T, 9, PH>(shape, varc, force, d, s);
      break;
    default: break;
  }
}

// entry of one phase's translation unit
template <int PH>
void launch_fused2d_phase(bool f32, int k, int shape, bool varc, bool force, FusedDev& d, hipStream_t s) {
  if (f32) launch_k<float, PH>(k, shape, varc, force, d, s);
  else launch_k<double, PH>(k, shape, varc, force, d, s);
}

void launch_fused2d_mid(bool f32, int k, int shape, bool varc, bool force, FusedDev& d, hipStream_t s);
void launch_fused2d_first(bool f32, int k, int shape, bool varc, bool force, FusedDev& d, hipStream_t s);
void launch_fused2d_last(bool f32, int k, int shape, bool varc, bool force, FusedDev& d, hipStream_t s);

}  // namespace wh
