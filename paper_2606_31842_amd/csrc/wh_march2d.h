// K leapfrog steps of the 2D wave equation with the filter sum, as a row-marching pipeline
// run by one wavefront on its own (no LDS, no barriers).
//
// The scheme is that of eq. discreteWaveExplicit with the trapezoid sum of eq. quadrature
// folded in (Section 2.2).  A wavefront owns a strip of 64*C columns (lane l holds columns
// xs - K + C l .. + C - 1) and marches over the rows of its tile.  When row t of the input
// state (time level 0) arrives, level 1 can be formed on row t-1, level 2 on row t-2, ...,
// level K on row t-K: each level s+1 needs level s on three consecutive rows and nothing
// else, so every level keeps a ring of its last rows in registers.  x-neighbours come from
// the adjacent columns of the lane and, at the lane's edge, from the adjacent lane (DPP
// wavefront shift).  The strip's K outermost columns on each side are halo: their values
// go stale by one column per level, so the inner 64*C - 2K columns are written.  Along y
// the pipeline starts K rows before the tile and ends K rows after it, which costs 2K rows
// of loads and work per tile (the tile is much taller than K).
//
// HBM traffic per written point is the state pair in and out and V read and written once
// per launch (FP32: 8 + 8 + 16 bytes), with the halo columns read again by the neighbour
// strip (mostly from L2).
//
// Rings: with the loop over rows unrolled U times (U a multiple of 4 and of K), every ring
// slot is a compile-time index, so the rings stay in registers:
//   W level s (s < K): 4 rows (3 needed), slot = (row - tstart) & 3
//   FP32 increment D (one register per row in flight: D_s(r) becomes D_{s+1}(r)),
//     the forcing, and the FP64 sum of V: K rows, slot = (row - tstart) % K
//   FP64 previous level -1: 2 rows.
// Rows of the next input are loaded PF iterations ahead.
//
// Points outside the open domain are held at zero (Dirichlet data).  When the launch
// advances Kp < K steps (the last launch of a wave solve), the levels above Kp are still
// formed but carry no filter weight, and the output is level Kp on row t - Kp.
//
// The unrolled body has no branches, so that the compiler can interleave the level chains
// of consecutive rows (level s+1 of row t-s needs level s of rows t-s-1 .. t-s+1 only):
// every load and store is a buffer access whose offset is moved out of the buffer's range
// when the point is masked (the hardware returns 0 for such a load and drops such a store),
// and masked results are selected, not branched around.
#pragma once
#include "wh_common.h"

namespace wh {

template <typename T>
struct MarchIO {
  const T* cin;        // W^n
  const T* pin;        // FP32: D^{n-1/2}; FP64: W^{n-1}
  T* cout;             // W^{n+Kp}
  T* pout;             // FP32: D^{n+Kp-1/2}; FP64: W^{n+Kp-1}
  double* V;           // filter sum, += sum_s w_s W^{n+s}
  const T* kap;        // VARC: c2 dt^2 / (2 h^2) per node
  const T* fs;         // forcing dt^2 f (used when force)
  const double* w;     // w[s] = weight of W^{n+s}, s = 1..Kp (w[0] unused)
  const double* cs;    // cs[s] = cos(omega t^{n+s}), s = 0..Kp-1
  T A;                 // constant c: dt^2 / h^2
  int n;
  int Kp;
  bool force;
};

// Raw buffer accesses (offsets in bytes); an offset at or beyond the buffer's size reads 0
// and writes nothing.
constexpr int kBufOff = 0x7ffffff0;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* p, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, int off);
template <>
__device__ __forceinline__ float buf_load<float>(__amdgpu_buffer_rsrc_t r, int off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
template <>
__device__ __forceinline__ double buf_load<double>(__amdgpu_buffer_rsrc_t r, int off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ void buf_store(float v, __amdgpu_buffer_rsrc_t r, int off) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, 0);
}
__device__ __forceinline__ void buf_store(double v, __amdgpu_buffer_rsrc_t r, int off) {
  using u2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, off, 0, 0);
}
// An interleaved FP32 pair (a at off, b at off + 4) in one 8-byte access.  The loaded vector is
// reinterpreted as a whole before its halves are taken: reading the halves of the integer
// vector the builtin returns got compiled into a single 4-byte load whose value served as both.
typedef float wh_float2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void buf_load_pair(__amdgpu_buffer_rsrc_t r, int off, float& a, float& b) {
  const wh_float2v f = __builtin_bit_cast(wh_float2v, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
  a = f.x;
  b = f.y;
}
__device__ __forceinline__ void buf_store_pair(float a, float b, __amdgpu_buffer_rsrc_t r, int off) {
  using u2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
  wh_float2v f;
  f.x = a;
  f.y = b;
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, f), r, off, 0, 0);
}

// Node arrays must hold (n+1)^2 elements of at most 2^31 bytes.
// FULL: the launch advances K steps (Kp == K), so the output is fixed at level K and the
// body stays free of branches; otherwise the store of level Kp is a uniform branch.
// RAD: stencil radius, 1 (second-order differences, variable c allowed) or 2 (fourth-order
// differences for c == 1, closed at the Dirichlet boundary by odd reflection: the neighbour
// two points beyond the last interior point is minus that point).  Level s+1 is formed on
// the row RAD rows behind level s, and the halo is RAD * K points on each side.
// PAIR (FP32 only): the state pair is one interleaved array, (W, D) in 8 bytes per node, at
// cin / cout (pin and pout unused), so that each row of the state is one access per lane.
template <typename T, int K, int C, int RAD, bool VARC, bool FORCE, bool FULL, bool UP, bool PAIR>
__device__ __forceinline__ void march2d_body(const MarchIO<T>& io, int xs, int ys, int ye) {
  constexpr bool INC = sizeof(T) == 4;
  constexpr int H = RAD * K;                 // halo points per side, rows before and after
  constexpr int WR = RAD == 1 ? 4 : 8;       // rows kept per level (>= 2 RAD + 1)
  constexpr int RK = RAD * K;                // rows in flight for D, the forcing and V
  constexpr int U = RK > WR ? RK : WR;
  static_assert(U % WR == 0 && U % RK == 0, "unroll must be a multiple of the ring sizes");
  static_assert(RAD == 1 || (C == 1 && !VARC), "fourth order: one column per lane, c == 1");
  static_assert(!PAIR || sizeof(T) == 4, "interleaved pairs are FP32");
  constexpr int PF = 2;
  constexpr int DK = INC ? RK : 1;
  constexpr int PK = INC ? 1 : (RAD == 1 ? 2 : 4);
  constexpr int TS = (int)sizeof(T);
  const int n = io.n;
  const int P = n + 1;
  const int64_t NN = (int64_t)P * P;
  const int Kp = io.Kp;
  const int lane = threadIdx.x;
  const int xb = xs - H + C * lane;
  constexpr int SB = PAIR ? 2 * TS : TS;   // bytes per node of a state array
  const __amdgpu_buffer_rsrc_t rc = buf_rsrc(io.cin, NN * SB), rp = buf_rsrc(PAIR ? io.cin : io.pin, NN * SB);
  const __amdgpu_buffer_rsrc_t rco = buf_rsrc(io.cout, NN * SB), rpo = buf_rsrc(PAIR ? io.cout : io.pout, NN * SB);
  const __amdgpu_buffer_rsrc_t rv = buf_rsrc(io.V, NN * 8);
  const __amdgpu_buffer_rsrc_t rk = buf_rsrc(VARC ? (const void*)io.kap : (const void*)io.cin, NN * TS);
  const __amdgpu_buffer_rsrc_t rf = buf_rsrc(FORCE ? (const void*)io.fs : (const void*)io.cin, NN * TS);

  constexpr int CR = RAD == 2 ? C : 1;
  bool colin[C], colout[C], refl_w[CR], refl_e[CR];
  int colm[C];   // all ones inside the open domain, else 0
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int col = xb + c;
    colin[c] = col >= 1 && col <= n - 1;
    const int lc = C * lane + c;
    colout[c] = colin[c] && lc >= H && lc < 64 * C - H;
    if constexpr (RAD == 2) {
      refl_w[c] = col == 1;       // its west neighbour at distance 2 is the reflection
      refl_e[c] = col == n - 1;
    }
    colm[c] = colin[c] ? -1 : 0;
    // opaque to the optimiser, which would otherwise turn the masking below back into a
    // select and then into a branch around the stencil
    asm("" : "+v"(colm[c]));
  }
  double wts[K + 1];
  T cn[K];
#pragma unroll
  for (int s = 0; s < K; ++s) {
    wts[s + 1] = s < Kp ? io.w[s + 1] : 0.0;
    cn[s] = (FORCE && s < Kp) ? (T)io.cs[s] : T(0);
  }

  constexpr int FK = FORCE ? RK : 1;
  T Wr[K][WR][C];
  T Dr[DK][C];
  T Pr[PK][C];
  T Fr[FK][C];   // forcing of the rows in flight (same slots as D)
  double acc[RK][C];
#pragma unroll
  for (int s = 0; s < RK; ++s)
#pragma unroll
    for (int c = 0; c < C; ++c) {
      if (s < K) {
#pragma unroll
        for (int q = 0; q < WR; ++q) Wr[s < K ? s : 0][q][c] = T(0);
      }
      acc[s][c] = 0.0;
    }
#pragma unroll
  for (int c = 0; c < C; ++c) {
#pragma unroll
    for (int q = 0; q < DK; ++q) Dr[q][c] = T(0);
#pragma unroll
    for (int q = 0; q < PK; ++q) Pr[q][c] = T(0);
#pragma unroll
    for (int q = 0; q < FK; ++q) Fr[q][c] = T(0);
  }

  const int tstart = ys - H;
  const int tlast = ye + H - 1;   // last input row the pipeline needs
  // pipeline row t is grid row rb + sg * t: downwards from row ys - H, or upwards from row
  // ye + H - 1 (the stencil is symmetric in y, so only the addresses change)
  const int rb = UP ? ys + ye - 1 : 0;
  constexpr int sg = UP ? -1 : 1;
  const int nit = ((ye - ys + 2 * H) + U - 1) / U * U;

  T sW[PF][C], sP[PF][C], sF[PF][C];
  double sV[PF][C];
#define WH_MARCH_LOAD(y_, q_)                                                    \
  {                                                                             \
    const int y = (y_);                                                         \
    const int ya = rb + sg * y;                                                 \
    const bool rin = ya >= 1 && ya <= n - 1 && y <= tlast;                      \
    const bool rout = ya >= ys && ya < ye;                                      \
    _Pragma("unroll") for (int c = 0; c < C; ++c) {                             \
      const int p = ya * P + xb + c;                                            \
      const bool in_ = rin && colin[c];                                         \
      if constexpr (PAIR) {                                                     \
        buf_load_pair(rc, in_ ? p * SB : kBufOff, sW[q_][c], sP[q_][c]);        \
      } else {                                                                  \
        sW[q_][c] = buf_load<T>(rc, in_ ? p * TS : kBufOff);                    \
        sP[q_][c] = buf_load<T>(rp, in_ ? p * TS : kBufOff);                    \
      }                                                                         \
      if (FORCE) sF[q_][c] = buf_load<T>(rf, in_ ? p * TS : kBufOff);           \
      sV[q_][c] = buf_load<double>(rv, (rout && colout[c]) ? p * 8 : kBufOff);  \
    }                                                                           \
  }
#pragma unroll
  for (int q = 0; q < PF; ++q) WH_MARCH_LOAD(tstart + q, q)

  for (int i0 = 0; i0 < nit; i0 += U) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = tstart + i0 + u;
      // row t of level 0 (and of level -1 in FP64) enters the rings
      T newD[C], newF[C];
      double newV[C];
#pragma unroll
      for (int c = 0; c < C; ++c) {
        Wr[0][u & (WR - 1)][c] = sW[u % PF][c];
        if constexpr (INC) newD[c] = sP[u % PF][c];
        else Pr[u & (PK - 1)][c] = sP[u % PF][c];
        if constexpr (FORCE) newF[c] = sF[u % PF][c];
        newV[c] = sV[u % PF][c];
      }
      WH_MARCH_LOAD(t + PF, u % PF)
#pragma unroll
      for (int s = 0; s < K; ++s) {
        // level s+1 on row r from level s on rows r-RAD .. r+RAD
        const int o = u - RAD * (s + 1);   // slot offset of row r
        const int r = rb + sg * (t - RAD * (s + 1));   // its grid row
        const bool rowok = r >= 1 && r <= n - 1;
        const int rowm = ~(((r - 1) | (n - 1 - r)) >> 31);   // all ones for 1 <= r <= n-1
        const bool rowout = r >= ys && r < ye;
        const int qc = o & (WR - 1), qu = (o - 1) & (WR - 1), qd = (o + 1) & (WR - 1);
        const int qk = (o % RK + RK) % RK;
        T wv[C];
#pragma unroll
        for (int c = 0; c < C; ++c) wv[c] = Wr[s][qc][c];
        const T wl = from_prev_lane(wv[C - 1]);
        const T er = from_next_lane(wv[0]);
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const T cc = wv[c];
          const T we = c > 0 ? wv[c - 1] : wl;
          const T ea = c < C - 1 ? wv[c + 1] : er;
          const T up = Wr[s][qu][c];
          const T dn = Wr[s][qd][c];
          const bool ok = rowok && colin[c];
          const int p = r * P + xb + c;
          T lap;
          if constexpr (RAD == 2) {
            // the rows two away in the pipeline are grid rows r -/+ 2 sg; a grid row -1 or
            // n+1 (beyond the boundary) is the odd reflection -W(r)
            const int ru2 = r - 2 * sg, rd2 = r + 2 * sg;
            const T up2 = (ru2 == -1 || ru2 == n + 1) ? -cc : Wr[s][(o - 2) & (WR - 1)][c];
            const T dn2 = (rd2 == -1 || rd2 == n + 1) ? -cc : Wr[s][(o + 2) & (WR - 1)][c];
            const T we2 = refl_w[c] ? -cc : from_prev_lane(wl);
            const T ea2 = refl_e[c] ? -cc : from_next_lane(er);
            const T sx = T(16) * ((we - cc) + (ea - cc)) - ((we2 - cc) + (ea2 - cc));
            const T sy = T(16) * ((up - cc) + (dn - cc)) - ((up2 - cc) + (dn2 - cc));
            lap = io.A * (sx + sy);
          } else if constexpr (VARC) {
            const T kc = buf_load<T>(rk, ok ? p * TS : kBufOff);
            const T kw = buf_load<T>(rk, ok ? (p - 1) * TS : kBufOff);
            const T ke = buf_load<T>(rk, ok ? (p + 1) * TS : kBufOff);
            // the pipeline's previous row is grid row r - sg
            const T ku = buf_load<T>(rk, ok ? (p - sg * P) * TS : kBufOff);
            const T kd = buf_load<T>(rk, ok ? (p + sg * P) * TS : kBufOff);
            lap = ((kc + kw) * (we - cc) + (kc + ke) * (ea - cc)) + ((kc + ku) * (up - cc) + (kc + kd) * (dn - cc));
          } else if constexpr (INC) {
            lap = io.A * (((we - cc) + (ea - cc)) + ((up - cc) + (dn - cc)));
          } else {
            lap = io.A * (((we + ea) + (up + dn)) - T(4) * cc);
          }
          if constexpr (FORCE) lap -= cn[s] * Fr[qk][c];
          const int m = colm[c] & rowm;
          T nw, pn;
          if constexpr (INC) {
            const T d = __int_as_float(__float_as_int(Dr[qk][c] + lap) & m);
            Dr[qk][c] = d;
            nw = cc + d;
            pn = d;
          } else {
            const T pv = s == 0 ? Pr[(u - RAD) & (PK - 1)][c] : Wr[s - 1][qc][c];
            nw = __longlong_as_double(__double_as_longlong((cc + cc) - pv + lap) & (long long)m);
            pn = cc;
          }
          if (s + 1 < K) Wr[s + 1][qc][c] = nw;
          const double a = acc[qk][c] + wts[s + 1] * (double)nw;
          acc[qk][c] = a;
          if (FULL ? s == K - 1 : s + 1 == Kp) {
            // level Kp on an output row and column is written (a masked store is dropped)
            const bool ob = rowout && colout[c];
            if constexpr (PAIR) {
              buf_store_pair(nw, pn, rco, ob ? p * SB : kBufOff);
            } else {
              buf_store(nw, rco, ob ? p * TS : kBufOff);
              buf_store(pn, rpo, ob ? p * TS : kBufOff);
            }
            buf_store(a, rv, ob ? p * 8 : kBufOff);
          }
        }
      }
      // row t starts its D and its filter sum (the slots of row t - RK, finished above)
#pragma unroll
      for (int c = 0; c < C; ++c) {
        if constexpr (INC) Dr[u % RK][c] = newD[c];
        if constexpr (FORCE) Fr[u % RK][c] = newF[c];
        acc[u % RK][c] = newV[c];
      }
      // FP64: keep the scheduler from overlapping consecutive rows, whose live rings would
      // otherwise cost more registers than the overlap gains
      if constexpr (!INC) __builtin_amdgcn_sched_barrier(0);
    }
  }
#undef WH_MARCH_LOAD
}

// up: march from the tile's last row towards its first.  Vertically adjacent tiles march in
// opposite directions, so the halo rows two tiles share are read by both at about the same
// time (both at the start or both at the end of their marches) and the second read finds them
// in L2.
template <typename T, int K, int C, int RAD, bool VARC, bool UP, bool PAIR>
__device__ __forceinline__ void march2d_dir(const MarchIO<T>& io, int xs, int ys, int ye) {
  if (io.force) {
    if (io.Kp == K) march2d_body<T, K, C, RAD, VARC, true, true, UP, PAIR>(io, xs, ys, ye);
    else march2d_body<T, K, C, RAD, VARC, true, false, UP, PAIR>(io, xs, ys, ye);
  } else {
    if (io.Kp == K) march2d_body<T, K, C, RAD, VARC, false, true, UP, PAIR>(io, xs, ys, ye);
    else march2d_body<T, K, C, RAD, VARC, false, false, UP, PAIR>(io, xs, ys, ye);
  }
}

template <typename T, int K, int C, bool VARC, int RAD = 1, bool PAIR = false>
__device__ __forceinline__ void march2d(const MarchIO<T>& io, int xs, int ys, int ye, bool up) {
  if (up) march2d_dir<T, K, C, RAD, VARC, true, PAIR>(io, xs, ys, ye);
  else march2d_dir<T, K, C, RAD, VARC, false, PAIR>(io, xs, ys, ye);
}

}  // namespace wh
