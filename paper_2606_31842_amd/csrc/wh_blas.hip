// Vector kernels of the Krylov solvers (Section 3): FP64 reductions, CG updates,
// Gram-Schmidt steps and the deflation projections W^T r / W c.
//
// Reductions are two-pass and deterministic: a fixed grid writes one partial sum
// per block (wave64 shuffle tree, then the four waves in order), and a single
// block adds the partials in index order.  No floating-point atomics are used.
#include "wh_common.h"
#include "wh_reduce.h"

namespace wh {

#define GRID_STRIDE(idx, N) \
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < (N); \
       idx += (int64_t)gridDim.x * blockDim.x)

static inline unsigned grid_for(int64_t N) {
  int64_t b = (N + kBlock - 1) / kBlock;
  return (unsigned)(b < 1 ? 1 : (b > kReduceBlocks ? kReduceBlocks : b));
}

// ----------------------------------------------------------------- coefficients
template <typename T>
__global__ void k_prep(const double* c2, const double* f, T* kap, T* fs, double ks, double fsc,
                       int64_t N, int n, int dim) {
  const int64_t P = n + 1;
  GRID_STRIDE(p, N) {
    if (c2) kap[p] = (T)(c2[p] * ks);
    if (f) {
      int i = (int)(p % P), j = (int)((p / P) % P), k = dim == 3 ? (int)(p / (P * P)) : 1;
      bool in = i > 0 && i < n && j > 0 && j < n && (dim == 2 || (k > 0 && k < n));
      fs[p] = in ? (T)(f[p] * fsc) : T(0);
    }
  }
}

void launch_prep_coeffs(const double* c2, const double* f, void* kap, void* fs, bool f32,
                        double ks, double fsc, int64_t N, int n, int dim, hipStream_t s) {
  if (f32)
    hipLaunchKernelGGL(k_prep<float>, dim3(grid_for(N)), dim3(kBlock), 0, s, c2, f, (float*)kap,
                       (float*)fs, ks, fsc, N, n, dim);
  else
    hipLaunchKernelGGL(k_prep<double>, dim3(grid_for(N)), dim3(kBlock), 0, s, c2, f,
                       (double*)kap, (double*)fs, ks, fsc, N, n, dim);
}

__global__ void k_zero_boundary(double* u, int n, int dim, int64_t N) {
  const int64_t P = n + 1;
  GRID_STRIDE(p, N) {
    int i = (int)(p % P), j = (int)((p / P) % P), k = dim == 3 ? (int)(p / (P * P)) : 1;
    bool in = i > 0 && i < n && j > 0 && j < n && (dim == 2 || (k > 0 && k < n));
    if (!in) u[p] = 0.0;
  }
}

void launch_zero_boundary(double* u, int n, int dim, hipStream_t s) {
  int64_t P = n + 1, N = dim == 2 ? P * P : P * P * P;
  hipLaunchKernelGGL(k_zero_boundary, dim3(grid_for(N)), dim3(kBlock), 0, s, u, n, dim, N);
}

// Defect forcing for the A-apply in the form A v = Pi_h(0; (L_h + omega^2) v): the
// scaled forcing array fs = f dt^2 with f = -(L_h + omega^2) v.
template <typename T>
__global__ void k_defect(const double* v, const double* kap, double a, double om2dt2, T* fs, int n,
                         int dim, int64_t N) {
  const int64_t P = n + 1;
  GRID_STRIDE(p, N) {
    int i = (int)(p % P), j = (int)((p / P) % P), k = dim == 3 ? (int)(p / (P * P)) : 1;
    bool in = i > 0 && i < n && j > 0 && j < n && (dim == 2 || (k > 0 && k < n));
    if (!in) continue;
    const int64_t nb[6] = {p - 1, p + 1, p - P, p + P, p - P * P, p + P * P};
    const bool ins[6] = {i > 1, i < n - 1, j > 1, j < n - 1, k > 1, k < n - 1};
    const double vc = v[p];
    double lap = 0.0;
    for (int t = 0; t < 2 * dim; ++t) {
      const double vq = ins[t] ? v[nb[t]] : 0.0;
      lap += (kap ? kap[p] + kap[nb[t]] : a) * (vq - vc);
    }
    fs[p] = (T)(-(lap + om2dt2 * vc));
  }
}

void launch_defect_forcing(const double* v, const double* kap64, double a, double om2dt2, void* fs,
                           bool f32, int n, int dim, hipStream_t s) {
  int64_t P = n + 1, N = dim == 2 ? P * P : P * P * P;
  if (f32)
    hipLaunchKernelGGL(k_defect<float>, dim3(grid_for(N)), dim3(kBlock), 0, s, v, kap64, a, om2dt2,
                       (float*)fs, n, dim, N);
  else
    hipLaunchKernelGGL(k_defect<double>, dim3(grid_for(N)), dim3(kBlock), 0, s, v, kap64, a, om2dt2,
                       (double*)fs, n, dim, N);
}

// ----------------------------------------------------------------- reductions
// max of a (or of -a); a NaN counts as +infinity in both, so that it reaches the result
// (fmax alone would drop it)
__global__ void k_max_partials(const double* a, int64_t N, double* partials, bool neg) {
  double m = -1.0e308;
  GRID_STRIDE(p, N) {
    const double v = a[p];
    m = fmax(m, v == v ? (neg ? -v : v) : HUGE_VAL);
  }
  double r = block_max256(m, threadIdx.x);
  if (threadIdx.x == 0) partials[blockIdx.x] = r;
}

void launch_max_partials(const double* a, int64_t N, double* partials, bool neg, hipStream_t s) {
  hipLaunchKernelGGL(k_max_partials, dim3(kReduceBlocks), dim3(kBlock), 0, s, a, N, partials, neg);
}

__global__ void k_max_finalize(const double* partials, int count, double* out) {
  double m = -1.0e308;
  for (int i = threadIdx.x; i < count; i += blockDim.x) m = fmax(m, partials[i]);
  double r = block_max256(m, threadIdx.x);
  if (threadIdx.x == 0) out[0] = r;
}

void launch_max_finalize(const double* partials, int count, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_max_finalize, dim3(1), dim3(kBlock), 0, s, partials, count, out);
}

__global__ void k_dot_partials(const double* a, const double* b, int64_t N, double* partials) {
  double acc = 0.0;
  GRID_STRIDE(p, N) acc += a[p] * b[p];
  double r = block_sum256(acc, threadIdx.x);
  if (threadIdx.x == 0) partials[blockIdx.x] = r;
}

void launch_dot_partials(const double* a, const double* b, int64_t N, double* partials,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_dot_partials, dim3(kReduceBlocks), dim3(kBlock), 0, s, a, b, N, partials);
}

__global__ void k_reduce(const double* partials, int count, double* slots, int dst, int mode) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < count; i += blockDim.x) acc += partials[i];
  double s = block_sum256(acc, threadIdx.x);
  if (threadIdx.x == 0) {
    if (mode == 0) {
      slots[dst] = s;
    } else if (mode == 1) {        // p^T q -> alpha
      slots[S_PQ] = s;
      slots[S_ALPHA] = slots[S_R2] / s;
    } else if (mode == 2) {        // r^T r -> beta
      slots[S_BETA] = s / slots[S_R2];
      slots[S_R2] = s;
    }
  }
}

void launch_reduce(const double* partials, int count, double* slots, int dst, int mode,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kBlock), 0, s, partials, count, slots, dst, mode);
}

// After a residual replacement: beta = slots[src] / r2_old, slots[R2] = slots[src].
__global__ void k_set_beta(double* slots, int src, double r2_old) {
  if (threadIdx.x == 0) {
    slots[S_BETA] = slots[src] / r2_old;
    slots[S_R2] = slots[src];
  }
}

void launch_set_beta(double* slots, int src, double r2_old, hipStream_t s) {
  hipLaunchKernelGGL(k_set_beta, dim3(1), dim3(64), 0, s, slots, src, r2_old);
}

// ----------------------------------------------------------------- CG updates
// x += alpha p, r -= alpha q, partial sums of r.r.  With pq_parts, every block first
// forms p^T q from the A-apply's pq_count partial sums (the same order as k_reduce, so the
// same value) and alpha = r^T r / p^T q itself; block 0 stores both in the slots.
__global__ void k_cg_update1(double* x, double* r, const double* p, const double* q,
                             double* slots, int64_t N, double* partials, const double* pq_parts,
                             int pq_count) {
  double alpha;
  if (pq_parts) {
    __shared__ double sh_alpha;
    double a = 0.0;
    for (int i = threadIdx.x; i < pq_count; i += blockDim.x) a += pq_parts[i];
    const double pq = block_sum256(a, threadIdx.x);
    if (threadIdx.x == 0) {
      sh_alpha = slots[S_R2] / pq;
      if (blockIdx.x == 0) {
        slots[S_PQ] = pq;
        slots[S_ALPHA] = sh_alpha;
      }
    }
    __syncthreads();
    alpha = sh_alpha;
  } else {
    alpha = slots[S_ALPHA];
  }
  double acc = 0.0;
  GRID_STRIDE(i, N) {
    x[i] += alpha * p[i];
    double rv = r[i] - alpha * q[i];
    r[i] = rv;
    acc += rv * rv;
  }
  double s = block_sum256(acc, threadIdx.x);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

void launch_cg_update1(double* x, double* r, const double* p, const double* q, double* slots,
                       int64_t N, double* partials, hipStream_t s, const double* pq_parts,
                       int pq_count) {
  hipLaunchKernelGGL(k_cg_update1, dim3(kReduceBlocks), dim3(kBlock), 0, s, x, r, p, q, slots, N,
                     partials, pq_parts, pq_count);
}

__global__ void k_cg_update2(double* p, const double* r, const double* slots, int64_t N) {
  const double beta = slots[S_BETA];
  GRID_STRIDE(i, N) p[i] = r[i] + beta * p[i];
}

void launch_cg_update2(double* p, const double* r, const double* slots, int64_t N, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_update2, dim3(grid_for(N)), dim3(kBlock), 0, s, p, r, slots, N);
}

__global__ void k_cg_update2_to(double* pn, const double* r, const double* p, const double* slots,
                                int64_t N) {
  const double beta = slots[S_BETA];
  GRID_STRIDE(i, N) pn[i] = r[i] + beta * p[i];
}

void launch_cg_update2_to(double* pn, const double* r, const double* p, const double* slots,
                          int64_t N, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_update2_to, dim3(grid_for(N)), dim3(kBlock), 0, s, pn, r, p, slots, N);
}

__global__ void k_axpy_slot(double* y, const double* x, const double* slots, int slot,
                            double sign, int64_t N) {
  const double a = sign * slots[slot];
  GRID_STRIDE(i, N) y[i] += a * x[i];
}

void launch_axpy_slot(double* y, const double* x, const double* slots, int slot, double sign,
                      int64_t N, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy_slot, dim3(grid_for(N)), dim3(kBlock), 0, s, y, x, slots, slot, sign, N);
}

__global__ void k_axpy(double* y, const double* x, double a, int64_t N) {
  GRID_STRIDE(i, N) y[i] += a * x[i];
}

void launch_axpy(double* y, const double* x, double a, int64_t N, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy, dim3(grid_for(N)), dim3(kBlock), 0, s, y, x, a, N);
}

// y = a x1 + b x2 + c x3 (element-wise; y may alias any input; a null x3 counts as 0)
__global__ void k_lincomb3(double* y, double a, const double* x1, double b, const double* x2,
                           double c, const double* x3, int64_t N) {
  GRID_STRIDE(i, N) {
    double v = a * x1[i] + b * x2[i];
    if (x3) v += c * x3[i];
    y[i] = v;
  }
}

void launch_lincomb3(double* y, double a, const double* x1, double b, const double* x2, double c,
                     const double* x3, int64_t N, hipStream_t s) {
  hipLaunchKernelGGL(k_lincomb3, dim3(grid_for(N)), dim3(kBlock), 0, s, y, a, x1, b, x2, c, x3, N);
}

__global__ void k_scale_copy(double* y, const double* x, const double* slots, int slot, int64_t N) {
  const double inv = 1.0 / sqrt(slots[slot]);
  GRID_STRIDE(i, N) y[i] = x[i] * inv;
}

void launch_scale_copy(double* y, const double* x, const double* slots, int slot, int64_t N,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_scale_copy, dim3(grid_for(N)), dim3(kBlock), 0, s, y, x, slots, slot, N);
}

__global__ void k_sub(double* y, const double* a, const double* b, int64_t N) {
  GRID_STRIDE(i, N) y[i] = a[i] - b[i];
}

void launch_sub(double* y, const double* a, const double* b, int64_t N, hipStream_t s) {
  hipLaunchKernelGGL(k_sub, dim3(grid_for(N)), dim3(kBlock), 0, s, y, a, b, N);
}

__global__ void k_copy(double* y, const double* x, int64_t N) {
  GRID_STRIDE(i, N) y[i] = x[i];
}

void launch_copy(double* y, const double* x, int64_t N, hipStream_t s) {
  hipLaunchKernelGGL(k_copy, dim3(grid_for(N)), dim3(kBlock), 0, s, y, x, N);
}

// x += sum_{c<k} y[c] V[:, c]
__global__ void k_gemv_acc(double* x, const double* V, int64_t ldv, int k, const double* y,
                           int64_t N) {
  GRID_STRIDE(i, N) {
    double acc = 0.0;
    for (int c = 0; c < k; ++c) acc += y[c] * V[(int64_t)c * ldv + i];
    x[i] += acc;
  }
}

void launch_gemv_acc(double* x, const double* V, int64_t ldv, int k, const double* y, int64_t N,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_gemv_acc, dim3(grid_for(N)), dim3(kBlock), 0, s, x, V, ldv, k, y, N);
}

// ----------------------------------------------------------------- Helmholtz residual
// value at axis offset d of node coordinate c for the fourth-order residual (odd reflection)
__device__ __forceinline__ double res_nb4(const double* u, int64_t p, int c, int d, int n, int64_t st) {
  const int q = c + d;
  if (q >= 1 && q <= n - 1) return u[p + d * st];
  if (q == -1) return -u[p + (d + 2) * st];
  if (q == n + 1) return -u[p + (d - 2) * st];
  return 0.0;
}

__global__ void k_helm_res(const double* c2, const double* f, const double* u, double om2,
                           double ih2, int n, int dim, int order, double* pr, double* pf) {
  const int64_t P = n + 1;
  const int64_t N = dim == 2 ? P * P : P * P * P;
  double ar = 0.0, af = 0.0;
  GRID_STRIDE(p, N) {
    int i = (int)(p % P), j = (int)((p / P) % P), k = dim == 3 ? (int)(p / (P * P)) : 1;
    bool in = i > 0 && i < n && j > 0 && j < n && (dim == 2 || (k > 0 && k < n));
    if (!in) continue;
    auto U = [&](int64_t q, bool inside) { return inside ? u[q] : 0.0; };
    const double uc = u[p];
    int64_t nb[6] = {p - 1, p + 1, p - P, p + P, p - P * P, p + P * P};
    bool ins[6] = {i > 1, i < n - 1, j > 1, j < n - 1, k > 1, k < n - 1};
    double lap = 0.0;
    if (order == 4) {   // c == 1
      const int crd[3] = {i, j, k};
      int64_t st = 1;
      for (int ax = 0; ax < dim; ++ax, st *= P)
        lap += (16.0 * (res_nb4(u, p, crd[ax], -1, n, st) + res_nb4(u, p, crd[ax], 1, n, st)) -
                (res_nb4(u, p, crd[ax], -2, n, st) + res_nb4(u, p, crd[ax], 2, n, st)) - 30.0 * uc) / 12.0;
    } else {
      for (int t = 0; t < 2 * dim; ++t) {
        double cf = c2 ? 0.5 * (c2[p] + c2[nb[t]]) : 1.0;
        lap += cf * (U(nb[t], ins[t]) - uc);
      }
    }
    double r = f[p] - (lap * ih2 + om2 * uc);
    ar += r * r;
    af += f[p] * f[p];
  }
  double sr = block_sum256(ar, threadIdx.x);
  double sf = block_sum256(af, threadIdx.x);
  if (threadIdx.x == 0) {
    pr[blockIdx.x] = sr;
    pf[blockIdx.x] = sf;
  }
}

int helmholtz_partial_blocks(int, int) { return kReduceBlocks; }

void launch_helmholtz_residual(const double* c2, const double* f, const double* u, double om2,
                               double ih2, int n, int dim, int order, double* pr, double* pf,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_helm_res, dim3(kReduceBlocks), dim3(kBlock), 0, s, c2, f, u, om2, ih2, n, dim,
                     order, pr, pf);
}

// ----------------------------------------------------------------- deflation
// Analytic sine modes: tab[(k*dim + axis)*(n+1) + i] = sqrt(2/n) sin(pi m_{k,axis} i / n).
__global__ void k_sine_tables(double* tab, const int32_t* modes, int nd, int dim, int n) {
  const int P = n + 1;
  const int total = nd * dim * P;
  const double nrm = sqrt(2.0 / n);
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < total; t += gridDim.x * blockDim.x) {
    int i = t % P;
    int ka = t / P;  // k*dim + axis
    long m = modes[ka];
    long r = (m * (long)i) % (2L * n);
    tab[t] = nrm * sinpi((double)r / (double)n);
  }
}

void launch_sine_tables(double* tab, const int32_t* modes_dev, int nd, int dim, int n,
                        hipStream_t s) {
  int total = nd * dim * (n + 1);
  hipLaunchKernelGGL(k_sine_tables, dim3((total + 255) / 256), dim3(256), 0, s, tab, modes_dev, nd,
                     dim, n);
}

constexpr int kDChunk = 32;   // modes per register pass

// Multi-value block sum: vals[c] summed over the 256 threads (4 waves), out[c] written by
// thread c.  C is a power of two <= 32.  Within a wave the value set is halved at every
// exchange: at lane distance o the lane keeps the half selected by bit o of its index and
// adds the partner's copy of that half (log2 C steps, C - 1 shuffles in all), after which
// each lane holds one value summed over 64 / C lanes; plain exchanges finish the sum over
// the wave.  The four wave sums are added in a fixed order, so results are reproducible.
// one halving step at lane distance O: keep H of the 2H live values (compile-time indices)
template <int C, int H, int O>
__device__ __forceinline__ void halve_values(double (&vals)[C], int lane, int& idx) {
  if constexpr (H >= 1) {
    const bool up = (lane & O) != 0;
#pragma unroll
    for (int i = 0; i < H; ++i) {
      const double give = up ? vals[i] : vals[i + H];
      const double keep = up ? vals[i + H] : vals[i];
      vals[i] = keep + __shfl_xor(give, O, 64);
    }
    if (up) idx += H;
    halve_values<C, H / 2, O / 2>(vals, lane, idx);
  }
}

template <int C>
__device__ __forceinline__ void block_sum_multi(double (&vals)[C], double* out, int tid) {
  static_assert(C >= 1 && C <= 32 && (C & (C - 1)) == 0, "power of two <= 32");
  __shared__ double sw[4][C];
  const int wv = tid >> 6, lane = tid & 63;
  int idx = 0;
  halve_values<C, C / 2, 32>(vals, lane, idx);
#pragma unroll
  for (int o = 32 / C; o >= 1; o >>= 1) vals[0] += __shfl_xor(vals[0], o, 64);
  if ((lane & (64 / C - 1)) == 0) sw[wv][idx] = vals[0];
  __syncthreads();
  if (tid < C) out[tid] = (sw[0][tid] + sw[1][tid]) + (sw[2][tid] + sw[3][tid]);
  __syncthreads();
}

// Sine modes, W^T r.  Rows of length P run along x; the mode factor of a row,
// prod_{axis>=1} tab[k][axis][coord], is the same for the whole row.  A block covers 64
// columns (one per lane) and 32 rows (8 per wave).  Per chunk of 32 modes the block first
// stages the 32 x 32 row factors in LDS (four per thread) and every thread issues its 32
// column-factor loads at once; then acc_k = sx_k(i) sum_t r(i, t) fy_k(t).  Partials
// layout [block][nd].
constexpr int kSineCols = 64, kSineRows = 32, kSineRowsPerWave = 8;

__global__ __launch_bounds__(256) void k_sine_project(const double* tab, int nd, int dim, int n,
                                                      const double* r, double* partials) {
  const int P = n + 1;
  const int rows = dim == 2 ? P : P * P;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int i = blockIdx.x * kSineCols + lane;
  const int rb = blockIdx.y * kSineRows;
  const int blk = blockIdx.y * gridDim.x + blockIdx.x;
  const bool col_ok = i < P;
  double rv[kSineRowsPerWave];
#pragma unroll
  for (int t = 0; t < kSineRowsPerWave; ++t) {
    const int row = rb + wv * kSineRowsPerWave + t;
    rv[t] = (col_ok && row < rows) ? r[(int64_t)row * P + i] : 0.0;
  }
  __shared__ double fy[kDChunk][kSineRows + 1];
  __shared__ double red[kDChunk];
  for (int k0 = 0; k0 < nd; k0 += kDChunk) {
    for (int e = tid; e < kDChunk * kSineRows; e += 256) {
      const int c = e / kSineRows, t = e % kSineRows, k = k0 + c;
      const int row = min(rb + t, rows - 1);
      double fv = 0.0;
      if (k < nd) {
        fv = tab[(int64_t)(k * dim + 1) * P + row % P];
        if (dim == 3) fv *= tab[(int64_t)(k * dim + 2) * P + row / P];
      }
      fy[c][t] = fv;
    }
    double sx[kDChunk];
#pragma unroll
    for (int c = 0; c < kDChunk; ++c)
      sx[c] = (col_ok && k0 + c < nd) ? tab[(int64_t)((k0 + c) * dim) * P + i] : 0.0;
    __syncthreads();
    double acc[kDChunk];
#pragma unroll
    for (int c = 0; c < kDChunk; ++c) {
      double a = 0.0;
#pragma unroll
      for (int t = 0; t < kSineRowsPerWave; ++t) a += rv[t] * fy[c][wv * kSineRowsPerWave + t];
      acc[c] = a * sx[c];
    }
    block_sum_multi<kDChunk>(acc, red, tid);   // ends with a barrier: fy may be rewritten
    if (tid < kDChunk && k0 + tid < nd) partials[(int64_t)blk * nd + k0 + tid] = red[tid];
  }
}

// Columns of a dense block V (column stride ldv): partials[bx][c] = sum over the block's
// points of V_c . r.  blockIdx.y picks a chunk of KC columns, so every column is read once
// and r once per chunk; all KC loads of a point are issued before the products.
template <int KC>
__global__ __launch_bounds__(256) void k_cols_project(const double* V, int64_t ldv, int ncols,
                                                      int64_t N, const double* r, double* partials) {
  const int tid = threadIdx.x;
  const int c0 = blockIdx.y * KC;
  const int nc = min(KC, ncols - c0);
  double acc[KC];
#pragma unroll
  for (int i = 0; i < KC; ++i) acc[i] = 0.0;
  GRID_STRIDE(p, N) {
    double v[KC];
#pragma unroll
    for (int i = 0; i < KC; ++i) v[i] = i < nc ? V[(int64_t)(c0 + i) * ldv + p] : 0.0;
    const double rv = r[p];
#pragma unroll
    for (int i = 0; i < KC; ++i) acc[i] += v[i] * rv;
  }
  __shared__ double red[KC];
  block_sum_multi<KC>(acc, red, tid);
  if (tid < nc) partials[(int64_t)blockIdx.x * ncols + c0 + tid] = red[tid];
}

static void launch_cols_project(const double* V, int64_t ldv, int ncols, int64_t N, const double* r,
                                double* partials, hipStream_t s) {
  const int kc = ncols <= 8 ? 8 : ncols <= 16 ? 16 : 32;
  const dim3 g(kReduceBlocks, (unsigned)((ncols + kc - 1) / kc)), b(256);
  if (kc == 8) hipLaunchKernelGGL(k_cols_project<8>, g, b, 0, s, V, ldv, ncols, N, r, partials);
  else if (kc == 16) hipLaunchKernelGGL(k_cols_project<16>, g, b, 0, s, V, ldv, ncols, N, r, partials);
  else hipLaunchKernelGGL(k_cols_project<32>, g, b, 0, s, V, ldv, ncols, N, r, partials);
}

static dim3 sine_grid(const Defl& d) {
  int P = d.n + 1;
  int64_t rows = d.dim == 2 ? (int64_t)P : (int64_t)P * P;
  return dim3((P + kSineCols - 1) / kSineCols, (unsigned)((rows + kSineRows - 1) / kSineRows));
}

int defl_partial_blocks(const Defl& d) {
  if (d.kind == WH_DEFL_SINE || d.kind == WH_DEFL_FACTORED) {
    dim3 g = sine_grid(d);
    return (int)(g.x * g.y);
  }
  return kReduceBlocks;
}

void launch_defl_project(const Defl& d, const double* r, double* partials, hipStream_t s) {
  if (d.kind == WH_DEFL_SINE || d.kind == WH_DEFL_FACTORED) {
    // factored modes: the same tiled kernel over the separable terms
    const int nk = d.kind == WH_DEFL_FACTORED ? d.nt : d.nd;
    hipLaunchKernelGGL(k_sine_project, sine_grid(d), dim3(256), 0, s, d.tab, nk, d.dim, d.n, r,
                       partials);
  } else {
    int64_t P = d.n + 1, N = d.dim == 2 ? P * P : P * P * P;
    launch_cols_project(d.V, d.ldv, d.nd, N, r, partials, s);
  }
}

__global__ void k_defl_reduce(const double* partials, int count, int nd, double* slots, int dst,
                              const double* scale) {
  const int k = blockIdx.x;
  double acc = 0.0;
  for (int b = threadIdx.x; b < count; b += blockDim.x) acc += partials[(int64_t)b * nd + k];
  double s = block_sum256(acc, threadIdx.x);
  if (threadIdx.x == 0) slots[dst + k] = scale ? s * scale[k] : s;
}

void launch_defl_reduce(const double* partials, int count, int nd, double* slots, int dst,
                        const double* scale_dev, hipStream_t s) {
  hipLaunchKernelGGL(k_defl_reduce, dim3(nd), dim3(256), 0, s, partials, count, nd, slots, dst,
                     scale_dev);
}

// factored modes: slots[dst + k] = sum of the projections of mode k's terms (* scale[k]),
// in term order
__global__ void k_terms_to_modes(const double* tsum, const int* toff, int nd, double* slots, int dst,
                                 const double* scale) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nd) return;
  double acc = 0.0;
  for (int t = toff[k]; t < toff[k + 1]; ++t) acc += tsum[t];
  slots[dst + k] = scale ? acc * scale[k] : acc;
}

// factored modes: per-term coefficients tcoef[t] = coef[tmap[t]]
__global__ void k_modes_to_terms(const double* coef, const int* tmap, int nt, double* tcoef) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nt) tcoef[t] = coef[tmap[t]];
}

void launch_defl_reduce_set(const Defl& d, const double* partials, double* slots, int dst,
                            const double* scale_dev, hipStream_t s) {
  if (d.kind == WH_DEFL_FACTORED) {
    hipLaunchKernelGGL(k_defl_reduce, dim3(d.nt), dim3(256), 0, s, partials, defl_partial_blocks(d), d.nt,
                       d.tsum, 0, (const double*)nullptr);
    hipLaunchKernelGGL(k_terms_to_modes, dim3((d.nd + 255) / 256), dim3(256), 0, s, (const double*)d.tsum,
                       d.toff, d.nd, slots, dst, scale_dev);
  } else {
    launch_defl_reduce(partials, defl_partial_blocks(d), d.nd, slots, dst, scale_dev, s);
  }
}

// y = alpha*y + beta*r - sum_k c_k W_k ; alpha taken from *aptr if aptr is set.
// Same tiling as the projection: per chunk of 32 modes the row factors times c_k are staged
// in LDS and the column factors loaded at once.
__global__ __launch_bounds__(256) void k_sine_combine(const double* tab, int nd, int dim, int n,
                                                      double* y, double alpha, const double* aptr,
                                                      const double* r, double beta,
                                                      const double* coef) {
  const int P = n + 1;
  const int rows = dim == 2 ? P : P * P;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int i = blockIdx.x * kSineCols + lane;
  const int rb = blockIdx.y * kSineRows;
  const bool col_ok = i < P;
  const double al = aptr ? *aptr : alpha;
  double sum[kSineRowsPerWave];
#pragma unroll
  for (int t = 0; t < kSineRowsPerWave; ++t) sum[t] = 0.0;
  __shared__ double fy[kDChunk][kSineRows + 1];
  for (int k0 = 0; k0 < nd; k0 += kDChunk) {
    for (int e = tid; e < kDChunk * kSineRows; e += 256) {
      const int c = e / kSineRows, t = e % kSineRows, k = k0 + c;
      const int row = min(rb + t, rows - 1);
      double fv = 0.0;
      if (k < nd) {
        fv = coef[k] * tab[(int64_t)(k * dim + 1) * P + row % P];
        if (dim == 3) fv *= tab[(int64_t)(k * dim + 2) * P + row / P];
      }
      fy[c][t] = fv;
    }
    double sx[kDChunk];
#pragma unroll
    for (int c = 0; c < kDChunk; ++c)
      sx[c] = (col_ok && k0 + c < nd) ? tab[(int64_t)((k0 + c) * dim) * P + i] : 0.0;
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kDChunk; ++c)
#pragma unroll
      for (int t = 0; t < kSineRowsPerWave; ++t) sum[t] += sx[c] * fy[c][wv * kSineRowsPerWave + t];
    __syncthreads();   // fy is rewritten by the next chunk
  }
  if (!col_ok) return;
#pragma unroll
  for (int t = 0; t < kSineRowsPerWave; ++t) {
    const int row = rb + wv * kSineRowsPerWave + t;
    if (row >= rows) break;
    const int64_t p = (int64_t)row * P + i;
    double v = (al == 0.0 ? 0.0 : al * y[p]) - sum[t];
    if (r) v += beta * r[p];
    y[p] = v;
  }
}

// s = sum_k c_k V_k in column order, 16 columns' loads issued at a time
__device__ __forceinline__ double cols_sum(const double* V, int64_t ldv, int nd, const double* c,
                                           int64_t p) {
  double sacc = 0.0;
  for (int k0 = 0; k0 < nd; k0 += 16) {
    double v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = k0 + i < nd ? V[(int64_t)(k0 + i) * ldv + p] : 0.0;
#pragma unroll
    for (int i = 0; i < 16; ++i)
      if (k0 + i < nd) sacc += c[k0 + i] * v[i];
  }
  return sacc;
}

__global__ __launch_bounds__(256) void k_dense_combine(const double* V, int64_t ldv, int nd, int64_t N,
                                                       double* y, double alpha, int aslot,
                                                       const double* r, double beta,
                                                       const double* slots, int src) {
  const double al = aslot >= 0 ? slots[aslot] : alpha;
  GRID_STRIDE(p, N) {
    const double sacc = cols_sum(V, ldv, nd, slots + src, p);
    double v = (al == 0.0 ? 0.0 : al * y[p]) - sacc;
    if (r) v += beta * r[p];
    y[p] = v;
  }
}

// w -= V h, h = slots[hsrc ..], subtracted column by column (bases wider than one register chunk)
__global__ __launch_bounds__(256) void k_gs_sub(const double* V, int64_t N, int nv, const double* slots,
                                                int hsrc, double* w) {
  GRID_STRIDE(p, N) {
    double wp = w[p];
    for (int k0 = 0; k0 < nv; k0 += 16) {
      double v[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) v[i] = k0 + i < nv ? V[(int64_t)(k0 + i) * N + p] : 0.0;
#pragma unroll
      for (int i = 0; i < 16; ++i)
        if (k0 + i < nv) wp -= slots[hsrc + k0 + i] * v[i];
    }
    w[p] = wp;
  }
}

// ---- classical Gram-Schmidt against an Arnoldi basis (column stride N)
// h = V^T w over the first nv columns: partials [kReduceBlocks][nv] (the dense projection).
void launch_gs_project(const double* V, int64_t N, int nv, const double* w, double* partials,
                       hipStream_t s) {
  launch_cols_project(V, N, nv, N, w, partials, s);
}

// w <- w - V h (h = slots[hsrc ..], subtracted in column order), then in the same pass either
// the projection V^T w and ||w||^2 of the updated w (PROJ; partials [block][nv + 1], the norm
// last) or ||w||^2 alone (partials [block]).  One read of the nv columns per point, kept in
// registers between the two uses.
template <int KC, bool PROJ>
__global__ __launch_bounds__(256) void k_gs_update(const double* V, int64_t N, int nv,
                                                   const double* slots, int hsrc, double* w,
                                                   double* partials) {
  const int tid = threadIdx.x;
  double h[KC];
#pragma unroll
  for (int i = 0; i < KC; ++i) h[i] = i < nv ? slots[hsrc + i] : 0.0;
  double acc[PROJ ? KC : 1];   // projections of the updated w
#pragma unroll
  for (int i = 0; i < (PROJ ? KC : 1); ++i) acc[i] = 0.0;
  double nrm = 0.0;
  GRID_STRIDE(p, N) {
    double v[KC];
#pragma unroll
    for (int i = 0; i < KC; ++i) v[i] = i < nv ? V[(int64_t)i * N + p] : 0.0;
    double wp = w[p];
#pragma unroll
    for (int i = 0; i < KC; ++i) wp -= h[i] * v[i];
    w[p] = wp;
    if constexpr (PROJ) {
#pragma unroll
      for (int i = 0; i < KC; ++i) acc[i] += v[i] * wp;
    }
    nrm += wp * wp;
  }
  const double t = block_sum256(nrm, tid);
  if constexpr (PROJ) {
    __shared__ double red[KC];
    block_sum_multi<KC>(acc, red, tid);
    if (tid < nv) partials[(int64_t)blockIdx.x * (nv + 1) + tid] = red[tid];
    if (tid == 0) partials[(int64_t)blockIdx.x * (nv + 1) + nv] = t;
  } else {
    if (tid == 0) partials[blockIdx.x] = t;
  }
}

template <bool PROJ>
static void gs_update_kc(int kc, const double* V, int64_t N, int nv, const double* slots, int hsrc,
                         double* w, double* partials, hipStream_t s) {
  const dim3 g(kReduceBlocks), b(256);
  if (kc == 8) hipLaunchKernelGGL((k_gs_update<8, PROJ>), g, b, 0, s, V, N, nv, slots, hsrc, w, partials);
  else if (kc == 16) hipLaunchKernelGGL((k_gs_update<16, PROJ>), g, b, 0, s, V, N, nv, slots, hsrc, w, partials);
  else hipLaunchKernelGGL((k_gs_update<32, PROJ>), g, b, 0, s, V, N, nv, slots, hsrc, w, partials);
}

void launch_gs_update(const double* V, int64_t N, int nv, const double* slots, int hsrc, double* w,
                      bool proj, double* partials, hipStream_t s) {
  if (nv <= 32) {
    const int kc = nv <= 8 ? 8 : nv <= 16 ? 16 : 32;
    if (proj) gs_update_kc<true>(kc, V, N, nv, slots, hsrc, w, partials, s);
    else gs_update_kc<false>(kc, V, N, nv, slots, hsrc, w, partials, s);
    return;
  }
  // wider bases: subtract, then project (w is the next column of the basis array, so the
  // projection on nv + 1 columns ends with ||w||^2) or take the norm in a second pass
  hipLaunchKernelGGL(k_gs_sub, dim3(grid_for(N)), dim3(256), 0, s, V, N, nv, slots, hsrc, w);
  if (proj) launch_cols_project(V, N, nv + 1, N, w, partials, s);
  else launch_dot_partials(w, w, N, partials, s);
}

static void combine_impl(const Defl& d, double* y, double alpha, int aslot, const double* r,
                         double beta, const double* slots, int src, int64_t N, hipStream_t s) {
  const double* aptr = aslot >= 0 ? slots + aslot : nullptr;
  if (d.kind == WH_DEFL_SINE) {
    hipLaunchKernelGGL(k_sine_combine, sine_grid(d), dim3(256), 0, s, d.tab, d.nd, d.dim, d.n, y,
                       alpha, aptr, r, beta, slots + src);
  } else if (d.kind == WH_DEFL_FACTORED) {
    hipLaunchKernelGGL(k_modes_to_terms, dim3((d.nt + 255) / 256), dim3(256), 0, s, slots + src, d.tmap,
                       d.nt, d.tcoef);
    hipLaunchKernelGGL(k_sine_combine, sine_grid(d), dim3(256), 0, s, d.tab, d.nt, d.dim, d.n, y,
                       alpha, aptr, r, beta, (const double*)d.tcoef);
  } else
    hipLaunchKernelGGL(k_dense_combine, dim3(grid_for(N)), dim3(256), 0, s, d.V, d.ldv, d.nd, N, y,
                       alpha, aslot, r, beta, slots, src);
}

void launch_defl_combine(const Defl& d, double* y, double alpha, const double* r, double beta,
                         const double* slots, int src, int64_t N, hipStream_t s) {
  combine_impl(d, y, alpha, -1, r, beta, slots, src, N, s);
}

void launch_dcg_update2(const Defl& d, double* p, const double* r, const double* slots, int src,
                        int64_t N, hipStream_t s) {
  combine_impl(d, p, 0.0, S_BETA, r, 1.0, slots, src, N, s);
}

// slots[dst + k] = scale * sum_j M[k][j] slots[src + j], k < nd (M row-major nd x nd; the two
// slot ranges do not overlap).  One block; the right-hand side is staged in LDS.
__global__ __launch_bounds__(256) void k_small_matvec(const double* M, int nd, double* slots, int src, int dst,
                                                      double scale) {
  __shared__ double v[1024];
  for (int j = threadIdx.x; j < nd; j += blockDim.x) v[j] = slots[src + j];
  __syncthreads();
  for (int k = threadIdx.x; k < nd; k += blockDim.x) {
    double acc = 0.0;
    for (int j = 0; j < nd; ++j) acc += M[(int64_t)k * nd + j] * v[j];
    slots[dst + k] = scale * acc;
  }
}

void launch_small_matvec(const double* M, int nd, double* slots, int src, int dst, double scale, hipStream_t s) {
  hipLaunchKernelGGL(k_small_matvec, dim3(1), dim3(256), 0, s, M, nd, slots, src, dst, scale);
}

}  // namespace wh
