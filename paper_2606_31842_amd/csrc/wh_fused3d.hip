// Temporally blocked 3D leapfrog + filter: K time steps per launch on a z-marching
// register pipeline.
//
// Same scheme as the streaming 3D kernel (Section 2.2, eq. discreteWaveExplicit with the
// trapezoid sum of eq. quadrature folded in; 7-point stencil, variable c through the
// face average of c^2).  A block of NW wavefronts owns a 64 x NW*R column tile (lane l:
// x = x0-K+l; wave w: rows y0-K+wR .. +R-1) and marches through a run of ZS output
// planes plus K planes of lead-in and lead-out.  At every z-position t it loads plane t
// (level 0) and advances each level s = 1..K by one plane: level s is computed at plane
// t-s from level s-1 at planes t-s-1, t-s, t-s+1, which the thread keeps in registers
// (three planes per level).  x-neighbours come from adjacent lanes (DPP), y-neighbours
// from the thread's own rows, except at wave edges: level-0 edges are read from memory
// with the plane, edges of computed levels are exchanged through a double-buffered LDS
// array (one barrier per plane).  The valid tile shrinks by one point per level in x and
// y, so the block writes the inner (64-2K) x (NW*R-2K) x ZS box: W^{n+K}, the second
// state and V + sum_s w_s W^{n+s}.
//
// All levels step in the increment form D += dt^2 (L_h W - f cos), W += D.  FP32 pairs
// are (W, D) already; FP64 pairs (W^n, W^{n-1}) are converted on load (D = W^n - W^{n-1})
// and on store (W^{n+K-1} = W^{n+K} - D).
//
// HBM traffic per output point and launch: state pair in + out, V in + out, kap and the
// forcing in, i.e. (4 + 4 + 4 + 4 + 8 + 8 [+4 +4]) bytes in FP32 for K steps.
#include "wh_common.h"

namespace wh {

__device__ __forceinline__ int xcd_tile3(int bid, int nb) {
  const int xcd = bid & 7, idx = bid >> 3;
  const int q = nb >> 3, r = nb & 7;
  return xcd < r ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

template <typename T, int K, int R, int NW, bool VARC, bool FORCE>
__global__ __launch_bounds__(64 * NW) void k_fused3d(const Fused3Dev a) {
  constexpr bool INC = sizeof(T) == 4;   // FP32 pairs are stored as (W, D)
  constexpr int TXO = 64 - 2 * K;
  constexpr int TYO = NW * R - 2 * K;
  static_assert(TXO > 0 && TYO > 0, "tile too small for K");
  const int n = a.n;
  const int64_t P = (int64_t)n + 1;
  const int64_t P2 = P * P;
  const int lane = threadIdx.x;
  const int wv = threadIdx.y;
  const int nb = a.gx * a.gy * a.gz;
  const int t3 = xcd_tile3(blockIdx.x, nb);
  const int tx = t3 % a.gx, ty = (t3 / a.gx) % a.gy, tz = t3 / (a.gx * a.gy);
  const int x0 = 1 + tx * TXO;
  const int y0 = 1 + ty * TYO;
  const int z0 = 1 + tz * a.zs;
  const int xg = x0 - K + lane;
  const int yb = y0 - K + wv * R;
  const bool xin = xg >= 1 && xg <= n - 1;
  const bool xout = lane >= K && lane < 64 - K && xin;
  // ymask: open domain (state), kmask: any node incl. the boundary (kap, whose boundary
  // values enter the face averages of the boundary faces)
  const bool xok = xg >= 0 && xg <= n;
  uint32_t ymask = 0, omask = 0, kmask = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int y = yb + r;
    const int ry = wv * R + r;
    if (xin && y >= 1 && y <= n - 1) ymask |= 1u << r;
    if (xok && y >= 0 && y <= n) kmask |= 1u << r;
    if (xout && y >= 1 && y <= n - 1 && ry >= K && ry < NW * R - K) omask |= 1u << r;
  }
  const bool yup_in = xin && yb - 1 >= 1 && yb - 1 <= n - 1;       // row above row 0
  const bool ydn_in = xin && yb + R >= 1 && yb + R <= n - 1;       // row below row R-1
  const bool yup_ok = xok && yb - 1 >= 0 && yb - 1 <= n;
  const bool ydn_ok = xok && yb + R >= 0 && yb + R <= n;

  const T* __restrict__ cin = (const T*)a.cur;
  const T* __restrict__ pin = (const T*)a.prev;
  const T* __restrict__ kap = (const T*)a.kap;
  const T* __restrict__ fsv = (const T*)a.fs;
  T* __restrict__ cout = (T*)a.cur_out;
  T* __restrict__ pout = (T*)a.prev_out;
  const T A = (T)a.a;

  // registers (static indices; rings shift by explicit moves)
  T Wr[K][3][R];          // level s at planes (t-s-2, t-s-1, t-s)
  T Dr[K][2][R];          // level s increments at planes (t-s-1, t-s)
  T E0[2][2];             // level-0 rows above/below the thread's rows at planes (t-1, t)
  T KP[VARC ? K + 2 : 1][R];   // kap at planes t-K-1 .. t
  T KE[VARC ? K + 2 : 1][2];   // kap above/below at the same planes
  T FS[FORCE ? K + 1 : 1][R];  // forcing at planes t-K .. t
  double AC[K + 1][R];    // V accumulators at planes t-K .. t
#pragma unroll
  for (int s = 0; s < K; ++s)
#pragma unroll
    for (int r = 0; r < R; ++r) {
      Wr[s][0][r] = Wr[s][1][r] = Wr[s][2][r] = T(0);
      Dr[s][0][r] = Dr[s][1][r] = T(0);
    }
  E0[0][0] = E0[0][1] = E0[1][0] = E0[1][1] = T(0);
#pragma unroll
  for (int q = 0; q < (VARC ? K + 2 : 1); ++q) {
    KE[q][0] = KE[q][1] = T(0);
#pragma unroll
    for (int r = 0; r < R; ++r) KP[q][r] = T(0);
  }
#pragma unroll
  for (int q = 0; q < (FORCE ? K + 1 : 1); ++q)
#pragma unroll
    for (int r = 0; r < R; ++r) FS[q][r] = T(0);
#pragma unroll
  for (int q = 0; q <= K; ++q)
#pragma unroll
    for (int r = 0; r < R; ++r) AC[q][r] = 0.0;

  __shared__ T edge[2][K > 1 ? K - 1 : 1][NW][2][64];
  const int zlast = min(z0 + a.zs - 1, n - 1);   // last output plane
  // FP32: plane loads run one z-step ahead (the values of plane t+1 are requested before
  // the levels are computed at plane t, so their latency overlaps that arithmetic).  FP64
  // loads plane t where it is used: its staging registers would spill.
  constexpr bool PF = sizeof(T) == 4;
  T sw[R], sd[R], sk[VARC ? R : 1], sf[FORCE ? R : 1], seu, sed, sku = T(0), skd = T(0);
  double sv[R];
  auto load_plane = [&](int tt) {
    const bool zin = tt >= 1 && tt <= n - 1;
    const bool zok = tt >= 0 && tt <= n;
    const int64_t pz = (int64_t)(zok ? tt : 0) * P2;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const bool in = zin && ((ymask >> r) & 1u);
      const int64_t p = pz + (int64_t)(yb + r) * P + xg;
      T w0 = T(0), d0 = T(0);
      if (in) {
        w0 = cin[p];
        d0 = INC ? pin[p] : w0 - pin[p];
      }
      sw[r] = w0;
      sd[r] = d0;
      if (VARC) sk[VARC ? r : 0] = (zok && ((kmask >> r) & 1u)) ? kap[p] : T(0);
      if (FORCE) sf[FORCE ? r : 0] = in ? fsv[p] : T(0);
      // V of plane tt for the inner tile, added to as the levels pass this plane
      sv[r] = (zin && tt >= z0 && tt <= zlast && ((omask >> r) & 1u)) ? a.V[p] : 0.0;
    }
    const int64_t pu = pz + (int64_t)(yb - 1) * P + xg;
    const int64_t pd = pz + (int64_t)(yb + R) * P + xg;
    seu = (zin && yup_in) ? cin[pu] : T(0);
    sed = (zin && ydn_in) ? cin[pd] : T(0);
    if (VARC) {
      sku = (zok && yup_ok) ? kap[pu] : T(0);
      skd = (zok && ydn_ok) ? kap[pd] : T(0);
    }
  };
  if constexpr (PF) load_plane(z0 - K);
  for (int t = z0 - K; t <= zlast + K; ++t) {
    const int b = t & 1;
    // (a) edges of levels 1..K-1 at their centre planes, written one plane ago
    T eu[K > 1 ? K - 1 : 1], ed[K > 1 ? K - 1 : 1];
#pragma unroll
    for (int s = 1; s < K; ++s) {
      eu[s - 1] = wv > 0 ? edge[b ^ 1][s - 1][wv - 1][1][lane] : T(0);
      ed[s - 1] = wv < NW - 1 ? edge[b ^ 1][s - 1][wv + 1][0][lane] : T(0);
    }
    // (b) shift the rings and take plane t (zero outside the open domain)
    if constexpr (!PF) load_plane(t);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      Wr[0][0][r] = Wr[0][1][r];
      Wr[0][1][r] = Wr[0][2][r];
      Dr[0][0][r] = Dr[0][1][r];
    }
    E0[0][0] = E0[1][0];
    E0[0][1] = E0[1][1];
    if (VARC) {
#pragma unroll
      for (int q = 0; q < (VARC ? K + 1 : 0); ++q) {
        KE[q][0] = KE[q + 1][0];
        KE[q][1] = KE[q + 1][1];
#pragma unroll
        for (int r = 0; r < R; ++r) KP[q][r] = KP[q + 1][r];
      }
    }
    if (FORCE) {
#pragma unroll
      for (int q = 0; q < (FORCE ? K : 0); ++q)
#pragma unroll
        for (int r = 0; r < R; ++r) FS[q][r] = FS[q + 1][r];
    }
#pragma unroll
    for (int q = 0; q < K; ++q)
#pragma unroll
      for (int r = 0; r < R; ++r) AC[q][r] = AC[q + 1][r];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      Wr[0][2][r] = sw[r];
      Dr[0][1][r] = sd[r];
      if (VARC) KP[VARC ? K + 1 : 0][r] = sk[VARC ? r : 0];
      if (FORCE) FS[FORCE ? K : 0][r] = sf[FORCE ? r : 0];
      AC[K][r] = sv[r];
    }
    E0[1][0] = seu;
    E0[1][1] = sed;
    if (VARC) {
      KE[VARC ? K + 1 : 0][0] = sku;
      KE[VARC ? K + 1 : 0][1] = skd;
    }
    if constexpr (PF) {
      if (t < zlast + K) load_plane(t + 1);
    }
    // (c) levels s = 1..K at planes q = t - s
#pragma unroll
    for (int s = 1; s <= K; ++s) {
      const int q = t - s;
      const bool qin = q >= 1 && q <= n - 1;
      const T up_e = s == 1 ? E0[0][0] : eu[s > 1 ? s - 2 : 0];
      const T dn_e = s == 1 ? E0[0][1] : ed[s > 1 ? s - 2 : 0];
      const T cn = FORCE ? (T)a.cs[s - 1] : T(0);
      const double ws = a.w[s - 1];
      T nwv[R], dnv[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const T c = Wr[s - 1][1][r];
        const T zm = Wr[s - 1][0][r];
        const T zp = Wr[s - 1][2][r];
        const T ym = r > 0 ? Wr[s - 1][1][r - 1] : up_e;
        const T yp = r < R - 1 ? Wr[s - 1][1][r + 1] : dn_e;
        const T xm = from_prev_lane(c);
        const T xp = from_next_lane(c);
        T lap;
        if (VARC) {
          const int ic = VARC ? K + 1 - s : 0;
          const T kc = KP[ic][r];
          const T kxm = from_prev_lane(kc);
          const T kxp = from_next_lane(kc);
          const T kym = r > 0 ? KP[ic][r - 1] : KE[ic][0];
          const T kyp = r < R - 1 ? KP[ic][r + 1] : KE[ic][1];
          const T kzm = KP[VARC ? ic - 1 : 0][r];
          const T kzp = KP[VARC ? ic + 1 : 0][r];
          lap = ((kc + kxm) * (xm - c) + (kc + kxp) * (xp - c)) +
                ((kc + kym) * (ym - c) + (kc + kyp) * (yp - c)) +
                ((kc + kzm) * (zm - c) + (kc + kzp) * (zp - c));
        } else {
          lap = A * ((((xm - c) + (xp - c)) + ((ym - c) + (yp - c))) + ((zm - c) + (zp - c)));
        }
        if (FORCE) lap -= cn * FS[FORCE ? K - s : 0][r];
        // outside the open domain W = D = 0 at every level, so masking D suffices
        const bool m = qin && ((ymask >> r) & 1u);
        T dn;
        if constexpr (sizeof(T) == 4) {
          dn = __int_as_float(__float_as_int(Dr[s - 1][0][r] + lap) & (int)(0u - (uint32_t)m));
        } else {
          dn = m ? Dr[s - 1][0][r] + lap : T(0);
        }
        const T nw = c + dn;
        nwv[r] = nw;
        dnv[r] = dn;
        AC[K - s][r] += ws * (double)nw;
      }
      if (s < K) {
        // append plane q of level s to its rings; publish its edge rows
#pragma unroll
        for (int r = 0; r < R; ++r) {
          Wr[s < K ? s : 0][0][r] = Wr[s < K ? s : 0][1][r];
          Wr[s < K ? s : 0][1][r] = Wr[s < K ? s : 0][2][r];
          Wr[s < K ? s : 0][2][r] = nwv[r];
          Dr[s < K ? s : 0][0][r] = Dr[s < K ? s : 0][1][r];
          Dr[s < K ? s : 0][1][r] = dnv[r];
        }
        edge[b][s < K ? s - 1 : 0][wv][0][lane] = nwv[0];
        edge[b][s < K ? s - 1 : 0][wv][1][lane] = nwv[R - 1];
      } else if (q >= z0 && q <= zlast) {
        // level K at plane q = t - K is complete: write the inner tile
        const int64_t pq = (int64_t)q * P2;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if ((omask >> r) & 1u) {
            const int64_t p = pq + (int64_t)(yb + r) * P + xg;
            cout[p] = nwv[r];
            pout[p] = INC ? dnv[r] : nwv[r] - dnv[r];
            a.V[p] = AC[0][r];
          }
        }
      }
    }
    __syncthreads();
  }
}

// Output planes per block when the shape leaves it open (zs = 0): every block marches its
// run plus 2K lead planes, and blocks run in rounds of (CUs x resident blocks per CU), so
// the launch takes about rounds x (zs + 2K) plane steps; take the z-split that minimises it,
// with runs of at least 2K planes (the lead planes at most double the loads).
static int balanced_zs(int n, int K, int tiles_xy, int slots) {
  int best_zs = n - 1;
  long best = -1;
  for (int gz = 1; gz <= n - 1; ++gz) {
    const int zs = (n - 1 + gz - 1) / gz;
    if ((n - 1 + zs - 1) / zs != gz) continue;   // the same run length as a smaller gz
    if (zs < 2 * K && gz > 1) break;
    const long rounds = ((long)tiles_xy * gz + slots - 1) / slots;
    const long cost = rounds * (zs + 2 * K);
    if (best < 0 || cost < best) {
      best = cost;
      best_zs = zs;
    }
  }
  return best_zs;
}

template <typename T, int K, int R, int NW, bool VARC, bool FORCE>
static int resident_slots() {
  static int slots = 0;   // per kernel: CUs x resident blocks per CU (of the first device used)
  if (slots == 0) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_fused3d<T, K, R, NW, VARC, FORCE>, 64 * NW, 0) !=
            hipSuccess)
      return 256;
    slots = std::max(1, cus * std::max(1, per));
  }
  return slots;
}

template <typename T, int K, int R, int NW>
static void launch_3d(bool varc, bool force, Fused3Dev& d, hipStream_t s) {
  const int n = d.n;
  d.gx = (n - 1 + (64 - 2 * K) - 1) / (64 - 2 * K);
  d.gy = (n - 1 + (NW * R - 2 * K) - 1) / (NW * R - 2 * K);
  if (d.zs <= 0) {
    int slots;
    if (varc) slots = force ? resident_slots<T, K, R, NW, true, true>() : resident_slots<T, K, R, NW, true, false>();
    else slots = force ? resident_slots<T, K, R, NW, false, true>() : resident_slots<T, K, R, NW, false, false>();
    d.zs = balanced_zs(n, K, d.gx * d.gy, slots);
  }
  d.gz = (n - 1 + d.zs - 1) / d.zs;
  dim3 g(d.gx * d.gy * d.gz), b(64, NW);
  if (varc) {
    if (force) hipLaunchKernelGGL((k_fused3d<T, K, R, NW, true, true>), g, b, 0, s, d);
    else hipLaunchKernelGGL((k_fused3d<T, K, R, NW, true, false>), g, b, 0, s, d);
  } else {
    if (force) hipLaunchKernelGGL((k_fused3d<T, K, R, NW, false, true>), g, b, 0, s, d);
    else hipLaunchKernelGGL((k_fused3d<T, K, R, NW, false, false>), g, b, 0, s, d);
  }
}

bool fused3d_supported(bool f32, int k) {
  (void)f32;
  return k == 2 || k == 3;
}

// Shapes (rows per thread R, waves per block NW, output planes per block ZS; 0: balanced
// over the resident blocks, see balanced_zs):
// FP32 (4,8,0) (4,8,16) (2,16,0); FP64 (2,16,0) (2,16,16) (4,8,0).
void fused3d_shape_dims(bool f32, int shape, int* rows, int* waves, int* zs) {
  static const int r32[kFusedShapes] = {4, 4, 2}, w32[kFusedShapes] = {8, 8, 16}, z32[kFusedShapes] = {0, 16, 0};
  static const int r64[kFusedShapes] = {2, 2, 4}, w64[kFusedShapes] = {16, 16, 8}, z64[kFusedShapes] = {0, 16, 0};
  const int sh = shape < 0 || shape >= kFusedShapes ? 0 : shape;
  *rows = f32 ? r32[sh] : r64[sh];
  *waves = f32 ? w32[sh] : w64[sh];
  *zs = f32 ? z32[sh] : z64[sh];
}

template <typename T, int K>
static void launch_3d_shape(int shape, bool varc, bool force, Fused3Dev& d, hipStream_t s) {
  int rows, waves, zs;
  fused3d_shape_dims(sizeof(T) == 4, shape, &rows, &waves, &zs);
  d.zs = zs;
  if (rows == 4 && waves == 8) launch_3d<T, K, 4, 8>(varc, force, d, s);
  else launch_3d<T, K, 2, 16>(varc, force, d, s);
}

void launch_fused3d(bool f32, bool varc, bool force, const FusedArgs& fa, hipStream_t s) {
  Fused3Dev d{};
  d.cur = fa.cur;
  d.prev = fa.prev;
  d.cur_out = fa.cur_out;
  d.prev_out = fa.prev_out;
  d.V = fa.V;
  d.kap = fa.kap;
  d.fs = fa.fs;
  d.a = fa.a;
  d.n = fa.n;
  for (int j = 0; j < fa.k && j < 8; ++j) {
    d.w[j] = fa.wts[j];
    d.cs[j] = fa.cosv[j];
  }
  const int shape = fa.shape < 0 || fa.shape >= kFusedShapes ? 0 : fa.shape;
  if (f32) {
    if (fa.k == 2) launch_3d_shape<float, 2>(shape, varc, force, d, s);
    else if (fa.k == 3) launch_3d_shape<float, 3>(shape, varc, force, d, s);
  } else {
    if (fa.k == 2) launch_3d_shape<double, 2>(shape, varc, force, d, s);
    else if (fa.k == 3) launch_3d_shape<double, 3>(shape, varc, force, d, s);
  }
}

}  // namespace wh
