// Leapfrog time steps of the wave equation with the trapezoid filter folded in.
//
// Scheme (Section 2.2, eq. discreteWaveExplicit and eq. quadrature):
//   W^{n+1} = 2 W^n - W^{n-1} + dt^2 (L_h W^n - f cos(omega_w t^n)),
//   W^1     = W^0 + dt^2/2 (L_h W^0 - f)             (D_0t W^0 = 0),
//   V       = sum_n w_n W^n.
// dt^2 L_h is applied as  a * (sum of neighbours - 2 dim W)  for c == 1 with
// a = dt^2/h^2, and as  sum_faces (kap_p + kap_q)(W_q - W_p)  with
// kap = c2 dt^2 / (2 h^2) for variable c (face average of c2).  The forcing array
// holds f dt^2.  The state type T is double (FP64 path) or float (mixed path);
// the accumulator V is always double.
//
// FP32 state pairs are (W^n, D^{n-1/2}) with D = W^n - W^{n-1} (the increment form of
// the same recurrence, which keeps FP32 rounding out of the low-frequency modes), and
// the Laplacian is summed as differences to the centre; FP64 pairs are (W^n, W^{n-1}).
//
// Streaming kernels: one thread per (x[, y]) column of interior nodes, marching
// RB rows (2D) or planes (3D) so that the neighbours along the marching axis are
// reused from registers; x/y neighbours come through the L1/L2 caches.
#include "wh_common.h"
#include "wh_reduce.h"

namespace wh {

constexpr int RB2 = 4;   // rows per thread (2D)
constexpr int RB3 = 8;   // planes per thread (3D)

template <typename T, int MODE>
__device__ __forceinline__ void step_epilogue(const StepArgs& a, size_t p, T nw, T* prev,
                                              double& acc) {
  if (MODE == M_MID) {
    prev[p] = nw;
    a.V[p] += a.wn * (double)nw;
  } else if (MODE == M_LAST_V) {
    a.V[p] += a.wn * (double)nw;
  } else if (MODE == M_LAST_AQ) {
    double vf = a.V[p] + a.wn * (double)nw;
    double xv = a.x[p];
    double q = xv - vf;
    a.out[p] = q;
    acc += xv * q;
  } else if (MODE == M_LAST_EQ) {
    const double q = -(a.V[p] + a.wn * (double)nw);
    a.out[p] = q;
    acc += a.x[p] * q;
  } else if (MODE == M_LAST_FPI) {
    // x and out may be the same array: read x before writing out
    double vf = a.V[p] + a.wn * (double)nw;
    double d = vf - a.x[p];
    a.out[p] = vf;
    acc += d * d;
  }
}

// --------------------------------------------------------------------- 2D
template <typename T, int MODE, bool VARC, bool FORCE>
__global__ __launch_bounds__(256) void k_step2d(StepArgs a) {
  constexpr bool INC = sizeof(T) == 4;   // increment form for FP32 pairs
  const int n = a.n;
  const size_t P = (size_t)n + 1;
  const int tid = threadIdx.y * 64 + threadIdx.x;
  const int i = 1 + blockIdx.x * 64 + threadIdx.x;
  const int j0 = 1 + (blockIdx.y * 4 + threadIdx.y) * RB2;
  const T* __restrict__ cur = (const T*)a.cur;
  T* __restrict__ prev = (T*)a.prev;
  const T* __restrict__ kap = (const T*)a.kap;
  const T* __restrict__ fs = (const T*)a.fs;
  const T A = (T)a.a;
  const T cn = (T)a.cosn;
  double acc = 0.0;
  if (i < n && j0 < n) {
    const int jend = min(j0 + RB2, n);
    size_t p = (size_t)j0 * P + i;
    T up = cur[p - P];
    T c = cur[p];
    T kup = T(0), kc = T(0);
    if (VARC) { kup = kap[p - P]; kc = kap[p]; }
    for (int j = j0; j < jend; ++j, p += P) {
      const T dn = cur[p + P];
      const T w = cur[p - 1];
      const T e = cur[p + 1];
      const T pv = prev[p];
      T nw;
      if (INC) {
        T lap;
        if (VARC) {
          const T kdn = kap[p + P];
          lap = (kc + kap[p - 1]) * (w - c) + (kc + kap[p + 1]) * (e - c) +
                ((kc + kup) * (up - c) + (kc + kdn) * (dn - c));
          kup = kc;
          kc = kdn;
        } else {
          lap = A * (((w - c) + (e - c)) + ((up - c) + (dn - c)));
        }
        if (FORCE) lap -= cn * fs[p];
        const T dnew = pv + lap;
        nw = c + dnew;
        if (MODE == M_MID) {
          prev[p] = dnew;
          ((T*)a.cur_next)[p] = nw;
          a.V[p] += a.wn * (double)nw;
        } else {
          step_epilogue<T, MODE>(a, p, nw, prev, acc);
        }
      } else {
        if (VARC) {
          const T kdn = kap[p + P];
          const T lap = (kc + kap[p - 1]) * (w - c) + (kc + kap[p + 1]) * (e - c) +
                        (kc + kup) * (up - c) + (kc + kdn) * (dn - c);
          nw = (c + c) - pv + lap;
          kup = kc;
          kc = kdn;
        } else {
          nw = (c + c) - pv + A * (((w + e) + (up + dn)) - T(4) * c);
        }
        if (FORCE) nw -= cn * fs[p];
        step_epilogue<T, MODE>(a, p, nw, prev, acc);
      }
      up = c;
      c = dn;
    }
  }
  if (MODE == M_LAST_AQ || MODE == M_LAST_FPI || MODE == M_LAST_EQ) {
    double s = block_sum256(acc, tid);
    if (tid == 0) a.partials[blockIdx.y * gridDim.x + blockIdx.x] = s;
  }
}

// --------------------------------------------------------------------- 3D
template <typename T, int MODE, bool VARC, bool FORCE>
__global__ __launch_bounds__(256) void k_step3d(StepArgs a) {
  constexpr bool INC = sizeof(T) == 4;   // increment form for FP32 pairs
  const int n = a.n;
  const size_t P = (size_t)n + 1;
  const size_t P2 = P * P;
  const int tid = threadIdx.y * 64 + threadIdx.x;
  const int i = 1 + blockIdx.x * 64 + threadIdx.x;
  const int j = 1 + blockIdx.y * 4 + threadIdx.y;
  const int k0 = 1 + blockIdx.z * RB3;
  const T* __restrict__ cur = (const T*)a.cur;
  T* __restrict__ prev = (T*)a.prev;
  const T* __restrict__ kap = (const T*)a.kap;
  const T* __restrict__ fs = (const T*)a.fs;
  const T A = (T)a.a;
  const T cn = (T)a.cosn;
  double acc = 0.0;
  if (i < n && j < n && k0 < n) {
    const int kend = min(k0 + RB3, n);
    size_t p = (size_t)k0 * P2 + (size_t)j * P + i;
    T bk = cur[p - P2];
    T c = cur[p];
    T kbk = T(0), kc = T(0);
    if (VARC) { kbk = kap[p - P2]; kc = kap[p]; }
    for (int k = k0; k < kend; ++k, p += P2) {
      const T fw = cur[p + P2];
      const T w = cur[p - 1], e = cur[p + 1];
      const T s = cur[p - P], nn = cur[p + P];
      const T pv = prev[p];
      T nw;
      if (INC) {
        T lap;
        if (VARC) {
          const T kfw = kap[p + P2];
          lap = ((kc + kap[p - 1]) * (w - c) + (kc + kap[p + 1]) * (e - c)) +
                ((kc + kap[p - P]) * (s - c) + (kc + kap[p + P]) * (nn - c)) +
                ((kc + kbk) * (bk - c) + (kc + kfw) * (fw - c));
          kbk = kc;
          kc = kfw;
        } else {
          lap = A * ((((w - c) + (e - c)) + ((s - c) + (nn - c))) + ((bk - c) + (fw - c)));
        }
        if (FORCE) lap -= cn * fs[p];
        const T dnew = pv + lap;
        nw = c + dnew;
        if (MODE == M_MID) {
          prev[p] = dnew;
          ((T*)a.cur_next)[p] = nw;
          a.V[p] += a.wn * (double)nw;
        } else {
          step_epilogue<T, MODE>(a, p, nw, prev, acc);
        }
      } else {
        if (VARC) {
          const T kfw = kap[p + P2];
          const T lap = (kc + kap[p - 1]) * (w - c) + (kc + kap[p + 1]) * (e - c) +
                        (kc + kap[p - P]) * (s - c) + (kc + kap[p + P]) * (nn - c) +
                        (kc + kbk) * (bk - c) + (kc + kfw) * (fw - c);
          nw = (c + c) - pv + lap;
          kbk = kc;
          kc = kfw;
        } else {
          nw = (c + c) - pv + A * ((((w + e) + (s + nn)) + (bk + fw)) - T(6) * c);
        }
        if (FORCE) nw -= cn * fs[p];
        step_epilogue<T, MODE>(a, p, nw, prev, acc);
      }
      bk = c;
      c = fw;
    }
  }
  if (MODE == M_LAST_AQ || MODE == M_LAST_FPI || MODE == M_LAST_EQ) {
    double s = block_sum256(acc, tid);
    if (tid == 0)
      a.partials[(blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = s;
  }
}

// --------------------------------------------------------------------- first step
// Covers every node: boundary nodes get zero state and zero accumulator; interior
// nodes take W^0 = v (boundary neighbours of v read as 0).
template <typename T, int DIM, bool VARC, bool FORCE>
__global__ __launch_bounds__(256) void k_first(StepArgs a) {
  const int n = a.n;
  const size_t P = (size_t)n + 1;
  const size_t N = DIM == 2 ? P * P : P * P * P;
  const size_t p = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= N) return;
  T* __restrict__ w0o = (T*)a.prev;
  T* __restrict__ w1o = (T*)a.cur_out;
  const int i = (int)(p % P);
  const int j = (int)((p / P) % P);
  const int k = DIM == 3 ? (int)(p / (P * P)) : 1;
  const bool interior = i > 0 && i < n && j > 0 && j < n && (DIM == 2 || (k > 0 && k < n));
  if (!interior) {
    w0o[p] = T(0);
    w1o[p] = T(0);
    if (a.zb0) ((T*)a.zb0)[p] = T(0);
    if (a.zb1) ((T*)a.zb1)[p] = T(0);
    a.V[p] = 0.0;
    return;
  }
  constexpr bool INC = sizeof(T) == 4;   // FP32 pair: (W^1, D^{1/2} = W^1 - W^0)
  const double* __restrict__ v = a.vin;
  const T* __restrict__ kap = (const T*)a.kap;
  if (!v) {  // W^0 = 0
    const T w1 = FORCE ? T(-0.5) * (T)a.cosn * ((const T*)a.fs)[p] : T(0);
    w0o[p] = INC ? w1 : T(0);
    w1o[p] = w1;
    a.V[p] = a.wn * (double)w1;
    return;
  }
  const T c = (T)v[p];
  const T w = i > 1 ? (T)v[p - 1] : T(0);
  const T e = i < n - 1 ? (T)v[p + 1] : T(0);
  const T s = j > 1 ? (T)v[p - P] : T(0);
  const T nn = j < n - 1 ? (T)v[p + P] : T(0);
  T bk = T(0), fw = T(0);
  if (DIM == 3) {
    bk = k > 1 ? (T)v[p - P * P] : T(0);
    fw = k < n - 1 ? (T)v[p + P * P] : T(0);
  }
  T lap;
  if (VARC) {
    const T kc = kap[p];
    lap = (kc + kap[p - 1]) * (w - c) + (kc + kap[p + 1]) * (e - c) + (kc + kap[p - P]) * (s - c) +
          (kc + kap[p + P]) * (nn - c);
    if (DIM == 3) lap += (kc + kap[p - P * P]) * (bk - c) + (kc + kap[p + P * P]) * (fw - c);
  } else if (INC) {
    T sum = ((w - c) + (e - c)) + ((s - c) + (nn - c));
    if (DIM == 3) sum += (bk - c) + (fw - c);
    lap = (T)a.a * sum;
  } else {
    T sum = (w + e) + (s + nn);
    if (DIM == 3) sum += bk + fw;
    lap = (T)a.a * (sum - T(2 * DIM) * c);
  }
  if (FORCE) lap -= (T)a.cosn * ((const T*)a.fs)[p];
  if (INC) {
    const T d = T(0.5) * lap;
    const T w1 = c + d;
    w0o[p] = d;
    w1o[p] = w1;
    a.V[p] = a.w0 * v[p] + a.wn * (double)w1;
  } else {
    const T w1 = c + T(0.5) * lap;
    w0o[p] = c;
    w1o[p] = w1;
    a.V[p] = a.w0 * v[p] + a.wn * (double)w1;
  }
}

// --------------------------------------------------------------------- fourth order
// c == 1: per axis h^-2 (-W_{i-2} + 16 W_{i-1} - 30 W_i + 16 W_{i+1} - W_{i+2}) / 12, the
// Dirichlet boundary closed by odd reflection (W_{-1} = -W_1, W_{n+1} = -W_{n-1}), which
// keeps the operator symmetric with the sine vectors as eigenvectors.  One thread per node;
// the scheme, the state pairs (increment form in FP32) and the epilogues are those of the
// second-order kernels, M_FIRST included.

// value at axis offset d (|d| <= 2) of the node at axis coordinate c (1 <= c <= n-1)
template <typename S>
__device__ __forceinline__ double nb4(const S* u, int64_t p, int c, int d, int n, int64_t st) {
  const int q = c + d;
  if (q >= 1 && q <= n - 1) return (double)u[p + d * st];
  if (q == -1) return -(double)u[p + (d + 2) * st];      // reflected node 1
  if (q == n + 1) return -(double)u[p + (d - 2) * st];   // reflected node n-1
  return 0.0;                                            // boundary node
}

// sum over axes of (-W_{-2} + 16 W_{-1} + 16 W_{+1} - W_{+2}) - 30 dim W, as differences to
// the centre (c0 = W at the node)
template <int DIM, typename S, typename T>
__device__ __forceinline__ T lap4_sum(const S* u, int64_t p, const int* crd, int n, int64_t P, T c0) {
  T sum = T(0);
  int64_t st = 1;
#pragma unroll
  for (int ax = 0; ax < DIM; ++ax) {
    const T m2 = (T)nb4(u, p, crd[ax], -2, n, st), m1 = (T)nb4(u, p, crd[ax], -1, n, st);
    const T p1 = (T)nb4(u, p, crd[ax], 1, n, st), p2 = (T)nb4(u, p, crd[ax], 2, n, st);
    sum += (T(16) * ((m1 - c0) + (p1 - c0))) - ((m2 - c0) + (p2 - c0));
    st *= P;
  }
  return sum;
}

template <typename T, int DIM, int MODE, bool FORCE>
__global__ __launch_bounds__(256) void k_step4(StepArgs a) {
  constexpr bool INC = sizeof(T) == 4;
  const int n = a.n;
  const int64_t P = (int64_t)n + 1;
  const int64_t N = DIM == 2 ? P * P : P * P * P;
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const T A12 = (T)(a.a / 12.0);
  double acc = 0.0;
  if (p < N) {
    const int crd[3] = {(int)(p % P), (int)((p / P) % P), DIM == 3 ? (int)(p / (P * P)) : 1};
    const bool interior = crd[0] > 0 && crd[0] < n && crd[1] > 0 && crd[1] < n &&
                          (DIM == 2 || (crd[2] > 0 && crd[2] < n));
    if (MODE == M_FIRST) {
      T* __restrict__ w0o = (T*)a.prev;
      T* __restrict__ w1o = (T*)a.cur_out;
      if (!interior) {
        w0o[p] = T(0);
        w1o[p] = T(0);
        if (a.zb0) ((T*)a.zb0)[p] = T(0);
        if (a.zb1) ((T*)a.zb1)[p] = T(0);
        a.V[p] = 0.0;
      } else {
        const double v0 = a.vin ? a.vin[p] : 0.0;
        const T c = (T)v0;
        T lap = a.vin ? A12 * lap4_sum<DIM>(a.vin, p, crd, n, P, c) : T(0);
        if (FORCE) lap -= (T)a.cosn * ((const T*)a.fs)[p];
        const T d = T(0.5) * lap;
        const T w1 = c + d;
        w0o[p] = INC ? d : c;
        w1o[p] = w1;
        a.V[p] = a.w0 * v0 + a.wn * (double)w1;
      }
    } else if (interior) {
      const T* __restrict__ cur = (const T*)a.cur;
      T* __restrict__ prev = (T*)a.prev;
      const T c = cur[p];
      T lap = A12 * lap4_sum<DIM>(cur, p, crd, n, P, c);
      if (FORCE) lap -= (T)a.cosn * ((const T*)a.fs)[p];
      if (INC) {
        const T dnew = prev[p] + lap;
        const T nw = c + dnew;
        if (MODE == M_MID) {
          prev[p] = dnew;
          ((T*)a.cur_next)[p] = nw;
          a.V[p] += a.wn * (double)nw;
        } else {
          step_epilogue<T, MODE>(a, (size_t)p, nw, prev, acc);
        }
      } else {
        const T nw = (c + c) - prev[p] + lap;
        step_epilogue<T, MODE>(a, (size_t)p, nw, prev, acc);
      }
    }
  }
  if (MODE == M_LAST_AQ || MODE == M_LAST_FPI || MODE == M_LAST_EQ) {
    const double sm = block_sum256(acc, threadIdx.x);
    if (threadIdx.x == 0) a.partials[blockIdx.x] = sm;
  }
}

template <typename T, int DIM, bool FORCE>
static void step4_mode(StepMode mode, dim3 g, const StepArgs& a, hipStream_t s) {
  switch (mode) {
    case M_FIRST: hipLaunchKernelGGL((k_step4<T, DIM, M_FIRST, FORCE>), g, dim3(256), 0, s, a); break;
    case M_MID: hipLaunchKernelGGL((k_step4<T, DIM, M_MID, FORCE>), g, dim3(256), 0, s, a); break;
    case M_LAST_V: hipLaunchKernelGGL((k_step4<T, DIM, M_LAST_V, FORCE>), g, dim3(256), 0, s, a); break;
    case M_LAST_AQ: hipLaunchKernelGGL((k_step4<T, DIM, M_LAST_AQ, FORCE>), g, dim3(256), 0, s, a); break;
    case M_LAST_FPI: hipLaunchKernelGGL((k_step4<T, DIM, M_LAST_FPI, FORCE>), g, dim3(256), 0, s, a); break;
    case M_LAST_EQ: hipLaunchKernelGGL((k_step4<T, DIM, M_LAST_EQ, FORCE>), g, dim3(256), 0, s, a); break;
    default: break;
  }
}

int step4_blocks(int dim, int n) {
  const int64_t P = (int64_t)n + 1;
  return (int)(((dim == 2 ? P * P : P * P * P) + 255) / 256);
}

int launch_step4(int dim, bool f32, bool force, StepMode mode, const StepArgs& a, hipStream_t s) {
  const int nb = step4_blocks(dim, a.n);
  const dim3 g((unsigned)nb);
  if (f32) {
    if (dim == 2) force ? step4_mode<float, 2, true>(mode, g, a, s) : step4_mode<float, 2, false>(mode, g, a, s);
    else force ? step4_mode<float, 3, true>(mode, g, a, s) : step4_mode<float, 3, false>(mode, g, a, s);
  } else {
    if (dim == 2) force ? step4_mode<double, 2, true>(mode, g, a, s) : step4_mode<double, 2, false>(mode, g, a, s);
    else force ? step4_mode<double, 3, true>(mode, g, a, s) : step4_mode<double, 3, false>(mode, g, a, s);
  }
  return nb;
}

// --------------------------------------------------------------------- dispatch
template <typename T, bool VARC, bool FORCE>
static void dispatch_dim(int dim, StepMode mode, const StepArgs& a, hipStream_t s) {
  const int n = a.n;
  if (mode == M_FIRST) {
    size_t P = (size_t)n + 1;
    size_t N = dim == 2 ? P * P : P * P * P;
    dim3 g((unsigned)((N + 255) / 256));
    if (dim == 2)
      hipLaunchKernelGGL((k_first<T, 2, VARC, FORCE>), g, dim3(256), 0, s, a);
    else
      hipLaunchKernelGGL((k_first<T, 3, VARC, FORCE>), g, dim3(256), 0, s, a);
    return;
  }
  dim3 b(64, 4);
  if (dim == 2) {
    dim3 g((n - 1 + 63) / 64, (n - 1 + 4 * RB2 - 1) / (4 * RB2));
    switch (mode) {
      case M_MID: hipLaunchKernelGGL((k_step2d<T, M_MID, VARC, FORCE>), g, b, 0, s, a); break;
      case M_LAST_V: hipLaunchKernelGGL((k_step2d<T, M_LAST_V, VARC, FORCE>), g, b, 0, s, a); break;
      case M_LAST_AQ: hipLaunchKernelGGL((k_step2d<T, M_LAST_AQ, VARC, FORCE>), g, b, 0, s, a); break;
      case M_LAST_FPI: hipLaunchKernelGGL((k_step2d<T, M_LAST_FPI, VARC, FORCE>), g, b, 0, s, a); break;
      case M_LAST_EQ: hipLaunchKernelGGL((k_step2d<T, M_LAST_EQ, VARC, FORCE>), g, b, 0, s, a); break;
      default: break;
    }
  } else {
    dim3 g((n - 1 + 63) / 64, (n - 1 + 3) / 4, (n - 1 + RB3 - 1) / RB3);
    switch (mode) {
      case M_MID: hipLaunchKernelGGL((k_step3d<T, M_MID, VARC, FORCE>), g, b, 0, s, a); break;
      case M_LAST_V: hipLaunchKernelGGL((k_step3d<T, M_LAST_V, VARC, FORCE>), g, b, 0, s, a); break;
      case M_LAST_AQ: hipLaunchKernelGGL((k_step3d<T, M_LAST_AQ, VARC, FORCE>), g, b, 0, s, a); break;
      case M_LAST_FPI: hipLaunchKernelGGL((k_step3d<T, M_LAST_FPI, VARC, FORCE>), g, b, 0, s, a); break;
      case M_LAST_EQ: hipLaunchKernelGGL((k_step3d<T, M_LAST_EQ, VARC, FORCE>), g, b, 0, s, a); break;
      default: break;
    }
  }
}

int step_partial_blocks(int dim, int n) {
  if (dim == 2) return ((n - 1 + 63) / 64) * ((n - 1 + 4 * RB2 - 1) / (4 * RB2));
  return ((n - 1 + 63) / 64) * ((n - 1 + 3) / 4) * ((n - 1 + RB3 - 1) / RB3);
}

template <typename T>
static void dispatch_flags(int dim, bool varc, bool force, StepMode mode, const StepArgs& a,
                           hipStream_t s) {
  if (varc) {
    if (force) dispatch_dim<T, true, true>(dim, mode, a, s);
    else dispatch_dim<T, true, false>(dim, mode, a, s);
  } else {
    if (force) dispatch_dim<T, false, true>(dim, mode, a, s);
    else dispatch_dim<T, false, false>(dim, mode, a, s);
  }
}

int launch_step(int dim, bool f32, bool varc, bool force, StepMode mode, const StepArgs& a,
                hipStream_t s) {
  if (f32) dispatch_flags<float>(dim, varc, force, mode, a, s);
  else dispatch_flags<double>(dim, varc, force, mode, a, s);
  return step_partial_blocks(dim, a.n);
}

}  // namespace wh
