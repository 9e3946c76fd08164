// Temporally blocked fourth-order 2D stepping for single solves (c == 1): K steps per launch by
// the row-marching pipeline of wh_march2d.h with the radius-2 stencil of the fourth-order
// difference (odd reflection at the Dirichlet boundary, as the single-step kernel k_step4).
// A wave solve runs its first and last steps in k_step4 (the half step from the input, the
// epilogue) and the steps between in these launches.
//
// Tiles of a launch: kM4W strips of 64 - 4K columns side by side by kM4Seg rows, one
// wavefront per strip; odd tile rows march upwards (shared halo rows meet in L2).
#include "wh_common.h"
#include "wh_march2d.h"

namespace wh {

constexpr int kM4W = 4;
constexpr int kM4Seg = 32;

int march4_strip(int K) { return 64 - 4 * K; }
int march4_tiles_x(int n, int K) { return (n - 1 + kM4W * march4_strip(K) - 1) / (kM4W * march4_strip(K)); }
int march4_tiles_y(int n) { return (n - 1 + kM4Seg - 1) / kM4Seg; }

__device__ __forceinline__ int xcd_tile_m4(int bid, int nb) {
  const int xcd = bid & 7, idx = bid >> 3;
  const int q = nb >> 3, r = nb & 7;
  return xcd < r ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

template <typename T, int K>
__global__ __launch_bounds__(64 * kM4W, sizeof(T) == 4 ? 3 : 2) void k_march4(const March4Args a) {
  const int strip = 64 - 4 * K;
  const int ntx = (a.n - 1 + kM4W * strip - 1) / (kM4W * strip);
  const int nty = (a.n - 1 + kM4Seg - 1) / kM4Seg;
  const int tile = xcd_tile_m4(blockIdx.x, ntx * nty);
  const int tx = tile % ntx, ty = tile / ntx;
  const int xs = 1 + (tx * kM4W + (int)threadIdx.y) * strip;
  const int ys = 1 + ty * kM4Seg;
  if (xs > a.n - 1) return;
  MarchIO<T> io;
  io.cin = (const T*)a.cur;
  io.pin = (const T*)a.prev;
  io.cout = (T*)a.cur_out;
  io.pout = (T*)a.prev_out;
  io.V = a.V;
  io.kap = nullptr;
  io.fs = (const T*)a.fs;
  io.w = a.w;
  io.cs = a.cs;
  io.A = (T)a.a12;
  io.n = a.n;
  io.Kp = a.kp;
  io.force = a.fs != nullptr;
  march2d<T, K, 1, false, 2>(io, xs, ys, min(ys + kM4Seg, a.n), (ty & 1) != 0);
}

template <typename T, int K>
static void launch_m4(const March4Args& a, hipStream_t s) {
  const int nb = march4_tiles_x(a.n, K) * march4_tiles_y(a.n);
  hipLaunchKernelGGL((k_march4<T, K>), dim3(nb), dim3(64, kM4W), 0, s, a);
}

bool march4_supported(int K) { return K == 2 || K == 4; }

void launch_march4(bool f32, int K, const March4Args& a, hipStream_t s) {
  if (f32) {
    if (K == 4) launch_m4<float, 4>(a, s);
    else launch_m4<float, 2>(a, s);
  } else {
    if (K == 4) launch_m4<double, 4>(a, s);
    else launch_m4<double, 2>(a, s);
  }
}

}  // namespace wh
