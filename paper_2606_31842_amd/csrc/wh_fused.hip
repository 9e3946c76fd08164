// Temporally blocked 2D kernel: host side and the instantiations of the middle phase
// (the kernel itself is in wh_fused_kernel.h).
#include "wh_fused_kernel.h"

namespace wh {

void launch_fused2d_mid(bool f32, int k, int shape, bool varc, bool force, FusedDev& d, hipStream_t s) {
  launch_fused2d_phase<kPhaseMid>(f32, k, shape, varc, force, d, s);
}

bool fused2d_supported(bool f32, int k) {
  // FP32 also K = 9: a wave solve of N_t = 8m + 1 steps is then 8s, one 9 and a last 8
  // instead of ending in a 6 and a 3
  return k == 2 || k == 3 || k == 4 || k == 6 || k == 8 || (f32 && k == 9);
}

// Shapes (rows per thread R, waves per block NW).  FP32: (16,4) (8,8) (8,4);
// FP64: (8,4) (4,8) (4,16).  Measured on 1024^2: FP32 (8,8) and FP64 (4,16) are the
// fastest; on 512^2 and below the 4-wave shapes are.
int fused2d_default_shape(bool f32, int n) {
  if (f32) return n >= 768 ? 1 : 2;
  return n >= 768 ? 2 : 1;
}

void fused2d_shape_dims(bool f32, int k, int shape, int* rows, int* waves) {
  static const int r32[kFusedShapes] = {16, 8, 8}, w32[kFusedShapes] = {4, 8, 4};
  static const int r64[kFusedShapes] = {8, 4, 4}, w64[kFusedShapes] = {4, 8, 16};
  const int s = shape < 0 || shape >= kFusedShapes ? 0 : shape;
  *rows = f32 ? r32[s] : r64[s];
  *waves = f32 ? w32[s] : w64[s];
  // FP32 K = 9 with 8 waves takes 9 rows per thread: a 64 x 72 region, whose 46 x 54 inner
  // tiles keep a 1024^2 launch within two blocks per CU (64 x 64 would need 529 blocks)
  if (f32 && k == 9 && s == 1) *rows = 9;
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
  d.vin = fa.vin;
  d.w0 = fa.w0;
  d.last = fa.last;
  d.x = fa.x;
  d.out = fa.out;
  d.partials = fa.partials;
  d.dr = fa.dr;
  d.dp = fa.dp;
  d.dslots = fa.dslots;
  d.dout = fa.dout;
  const int shape = fa.shape < 0 || fa.shape >= kFusedShapes ? 0 : fa.shape;
  if (fa.first) launch_fused2d_first(f32, fa.k, shape, varc, force, d, s);
  else if (fa.last != M_MID) launch_fused2d_last(f32, fa.k, shape, varc, force, d, s);
  else launch_fused2d_mid(f32, fa.k, shape, varc, force, d, s);
}

int fused2d_blocks(bool f32, int k, int shape, int n) {
  int rows, waves;
  fused2d_shape_dims(f32, k, shape, &rows, &waves);
  const int tx = 64 - 2 * k, ty = waves * rows - 2 * k;
  return ((n - 1 + tx - 1) / tx) * ((n - 1 + ty - 1) / ty);
}

}  // namespace wh
