// Temporally blocked 2D leapfrog + filter: K time steps per launch.
//
// Same scheme as the streaming kernels (Section 2.2, eq. discreteWaveExplicit with
// the trapezoid sum of eq. quadrature folded in), but each 256-thread block keeps
// a 64-column x 4R-row region of (W^n, W^{n-1}) in registers and advances it K
// steps before writing back.  Lane l of wave w owns column x0-K+l and rows
// y0-K+wR .. y0-K+wR+R-1.  Per step:
//   * x-neighbours come from the adjacent lanes (cross-lane shuffle),
//   * y-neighbours come from the thread's own rows, except the first/last row of
//     each wave, which are exchanged through a small double-buffered LDS array,
//   * points outside the open domain are held at zero (Dirichlet data).
// The valid region shrinks by one point per step on every side, so the block
// writes the inner (64-2K) x (4R-2K) tile: W^{n+K}, W^{n+K-1} and V += sum_s w_s W^{n+s}.
// HBM traffic per point and launch is 8 (state in) + 8 (state out) + 16 (V) bytes in
// FP32, i.e. 32/K bytes per point-step against 28 for the streaming kernel.
//
// Inputs and outputs are distinct buffers (neighbouring blocks read the halo).
#include "wh_common.h"

namespace wh {

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
};

// Tile order that gives each XCD a contiguous run of tiles (blocks are dispatched
// round-robin over the 8 XCDs), so horizontally adjacent tiles share an L2.
__device__ __forceinline__ int xcd_tile(int bid, int nb) {
  const int xcd = bid & 7, idx = bid >> 3;
  const int q = nb >> 3, r = nb & 7;
  return xcd < r ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

template <typename T>
__device__ __forceinline__ T lane_up(T v) { return __shfl_up(v, 1, 64); }
template <typename T>
__device__ __forceinline__ T lane_down(T v) { return __shfl_down(v, 1, 64); }

template <typename T, int K, int R, bool VARC, bool FORCE>
__global__ __launch_bounds__(256) void k_fused2d(const FusedDev a) {
  constexpr int TXO = 64 - 2 * K;
  constexpr int TYO = 4 * R - 2 * K;
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
  const bool xok = xg >= 0 && xg <= n;

  const T* __restrict__ cin = (const T*)a.cur;
  const T* __restrict__ pin = (const T*)a.prev;
  const T* __restrict__ kap = (const T*)a.kap;
  const T* __restrict__ fsv = (const T*)a.fs;

  T cur[R], prv[R];
  double acc[R];
  T cw[VARC ? R : 1], ce[VARC ? R : 1], cu[VARC ? R : 1], cd[VARC ? R : 1];
  T frc[FORCE ? R : 1];
  uint32_t mask = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int y = yb + r;
    const bool in = xin && y >= 1 && y <= n - 1;
    const bool ok = xok && y >= 0 && y <= n;
    const int64_t p = (int64_t)y * P + xg;
    // boundary nodes hold the Dirichlet value 0: read interior nodes only
    cur[r] = in ? cin[p] : T(0);
    prv[r] = in ? pin[p] : T(0);
    (void)ok;
    acc[r] = 0.0;
    if (in) mask |= 1u << r;
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

  __shared__ T edge[2][4][2][64];
  const T A = (T)a.a;
#pragma unroll
  for (int s = 0; s < K; ++s) {
    const int b = s & 1;
    edge[b][wv][0][lane] = cur[0];
    edge[b][wv][1][lane] = cur[R - 1];
    __syncthreads();
    const T up_e = wv > 0 ? edge[b][wv - 1][1][lane] : T(0);
    const T dn_e = wv < 3 ? edge[b][wv + 1][0][lane] : T(0);
    const T cn = (T)a.cs[s];
    const double ws = a.w[s];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const T c = cur[r];
      const T u = r > 0 ? cur[r - 1] : up_e;
      const T d = r < R - 1 ? cur[r + 1] : dn_e;
      const T w = lane_up(c);
      const T e = lane_down(c);
      T nw;
      if (VARC) {
        const int q = VARC ? r : 0;
        nw = (c + c) - prv[r] + (cw[q] * (w - c) + ce[q] * (e - c) + (cu[q] * (u - c) + cd[q] * (d - c)));
      } else {
        nw = (c + c) - prv[r] + A * (((w + e) + (u + d)) - T(4) * c);
      }
      if (FORCE) nw -= cn * frc[FORCE ? r : 0];
      nw = ((mask >> r) & 1u) ? nw : T(0);
      prv[r] = nw;
      acc[r] += ws * (double)nw;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const T tmp = cur[r];
      cur[r] = prv[r];
      prv[r] = tmp;
    }
  }

  // write the inner tile
  if (lane >= K && lane < 64 - K && xin) {
    T* __restrict__ cout = (T*)a.cur_out;
    T* __restrict__ pout = (T*)a.prev_out;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int ry = wv * R + r;
      if (ry >= K && ry < 4 * R - K && ((mask >> r) & 1u)) {
        const int64_t p = (int64_t)(yb + r) * P + xg;
        cout[p] = cur[r];
        pout[p] = prv[r];
        a.V[p] += acc[r];
      }
    }
  }
}

template <typename T, int K, int R>
static void launch_kr(bool varc, bool force, const FusedDev& d, hipStream_t s) {
  dim3 g(d.gx * d.gy), b(64, 4);
  if (varc) {
    if (force) hipLaunchKernelGGL((k_fused2d<T, K, R, true, true>), g, b, 0, s, d);
    else hipLaunchKernelGGL((k_fused2d<T, K, R, true, false>), g, b, 0, s, d);
  } else {
    if (force) hipLaunchKernelGGL((k_fused2d<T, K, R, false, true>), g, b, 0, s, d);
    else hipLaunchKernelGGL((k_fused2d<T, K, R, false, false>), g, b, 0, s, d);
  }
}

// Supported (K, R) pairs: rows per thread R = 16 (FP32) / 8 (FP64).
bool fused2d_supported(bool f32, int k) {
  (void)f32;
  return k == 2 || k == 3 || k == 4 || k == 6 || k == 8;
}

template <typename T, int R>
static void launch_k(int k, bool varc, bool force, FusedDev& d, hipStream_t s) {
  const int n = d.n;
  auto grid = [&](int K) {
    d.gx = (n - 1 + (64 - 2 * K) - 1) / (64 - 2 * K);
    d.gy = (n - 1 + (4 * R - 2 * K) - 1) / (4 * R - 2 * K);
  };
  switch (k) {
    case 2: grid(2); launch_kr<T, 2, R>(varc, force, d, s); break;
    case 3: grid(3); launch_kr<T, 3, R>(varc, force, d, s); break;
    case 4: grid(4); launch_kr<T, 4, R>(varc, force, d, s); break;
    case 6: grid(6); launch_kr<T, 6, R>(varc, force, d, s); break;
    case 8: grid(8); launch_kr<T, 8, R>(varc, force, d, s); break;
    default: break;
  }
}

void launch_fused2d(bool f32, bool varc, bool force, const FusedArgs& fa, hipStream_t s) {
  FusedDev d{};
  d.cur = fa.cur;
  d.prev = fa.prev;
  d.cur_out = fa.cur_out;
  d.prev_out = fa.prev_out;
  d.V = fa.V;
  d.kap = fa.kap;
  d.fs = fa.fs;
  d.a = fa.a;
  d.n = fa.n;
  for (int j = 0; j < fa.k && j < 16; ++j) {
    d.w[j] = fa.wts[j];
    d.cs[j] = fa.cosv[j];
  }
  if (f32) launch_k<float, 16>(fa.k, varc, force, d, s);
  else launch_k<double, 8>(fa.k, varc, force, d, s);
}

}  // namespace wh
