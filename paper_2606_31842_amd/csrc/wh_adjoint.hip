// Kernels of the misfit gradient dJ/dc2 (2D).
//
// At the fixed point u = Pi_h(u; c2) (Section 2.1; discrete form eq. WaveHoltzDiscreteFPI),
// dJ/dc2 = (dPi_h/dc2)^T z with z = A^{-1} dJ/du (A = I - S_h is symmetric).  The
// vector-Jacobian product runs the leapfrog recurrence of eq. discreteWaveExplicit
// backwards (its transpose, L_h being symmetric) with the trapezoid weights as the
// source:
//   Lam^{N} = w_N z,  Lam^{n} = 2 Lam^{n+1} + dt^2 L_h Lam^{n+1} - Lam^{n+2} + w_n z,
// and collects, for every step n >= 1 of the forward trajectory W^n of Pi_h(u; f),
//   grad_k += -(dt^2 / (2 h^2)) sum_{faces (k,q)} (Lam^{n+1}_k - Lam^{n+1}_q)(W^n_k - W^n_q),
// plus half that term for the first (half) step with Lam^1 and W^0.  Each face's
// coefficient c2_f = (c2_k + c2_q)/2 splits its derivative evenly between its two nodes.
#include "wh_common.h"
#include "wh_reduce.h"

namespace wh {

// out = 2 cur - prev + dt^2 (L_h cur - f cos_n)  (first = true: out = cur + dt^2/2 (L_h cur - f))
// at interior nodes; kap = c2 dt^2 / (2 h^2) (FP64), fs = f dt^2 or NULL.
__global__ void k_fwd_out2d(const double* __restrict__ cur, const double* __restrict__ prev,
                            double* __restrict__ out, const double* __restrict__ kap,
                            const double* __restrict__ fs, double cosn, int first, int n) {
  const int64_t P = (int64_t)n + 1;
  const int i = 1 + blockIdx.x * 64 + threadIdx.x;
  const int j = 1 + blockIdx.y * 4 + threadIdx.y;
  if (i >= n || j >= n) return;
  const int64_t p = (int64_t)j * P + i;
  const double c = cur[p];
  const double kc = kap[p];
  double lap = (kc + kap[p - 1]) * (cur[p - 1] - c) + (kc + kap[p + 1]) * (cur[p + 1] - c) +
               ((kc + kap[p - P]) * (cur[p - P] - c) + (kc + kap[p + P]) * (cur[p + P] - c));
  if (fs) lap -= cosn * fs[p];
  out[p] = first ? c + 0.5 * lap : (c + c) - prev[p] + lap;
}

// One reverse step over all nodes: interior nodes update lam_out = Lam^n from
// lam1 = Lam^{n+1}, lam2 = Lam^{n+2}; every node accumulates the face terms of
// (lam1, W) into grad with factor gscale.  do_lam = 0 skips the Lam update.
__global__ void k_adj_step2d(const double* __restrict__ lam1, const double* __restrict__ lam2,
                             double* __restrict__ lam_out, const double* __restrict__ W,
                             const double* __restrict__ kap, const double* __restrict__ z,
                             double wn, double gscale, double* __restrict__ grad, int do_lam,
                             int n) {
  const int64_t P = (int64_t)n + 1;
  const int i = blockIdx.x * 64 + threadIdx.x;
  const int j = blockIdx.y * 4 + threadIdx.y;
  if (i > n || j > n) return;
  const int64_t p = (int64_t)j * P + i;
  const double lc = lam1[p], wc = W[p];
  double g = 0.0;
  if (i > 0) g += (lc - lam1[p - 1]) * (wc - W[p - 1]);
  if (i < n) g += (lc - lam1[p + 1]) * (wc - W[p + 1]);
  if (j > 0) g += (lc - lam1[p - P]) * (wc - W[p - P]);
  if (j < n) g += (lc - lam1[p + P]) * (wc - W[p + P]);
  grad[p] += gscale * g;
  if (do_lam && i > 0 && i < n && j > 0 && j < n) {
    const double kc = kap[p];
    const double lap = (kc + kap[p - 1]) * (lam1[p - 1] - lc) + (kc + kap[p + 1]) * (lam1[p + 1] - lc) +
                       ((kc + kap[p - P]) * (lam1[p - P] - lc) + (kc + kap[p + P]) * (lam1[p + P] - lc));
    lam_out[p] = (lc + lc) - lam2[p] + lap + wn * z[p];
  }
}

// Receiver misfit: res_k = u[idx_k] - d_k, J += 1/2 sum res_k^2 (into out[0]), and
// g = R^T res (g zeroed by the caller).  One block; receivers are visited in order so
// repeated indices accumulate deterministically.
__global__ void k_misfit(const double* u, const int64_t* idx, const double* d, int nrec, double* g,
                         double* out) {
  double acc = 0.0;
  for (int k = threadIdx.x; k < nrec; k += blockDim.x) {
    const double r = u[idx[k]] - d[k];
    acc += r * r;
  }
  const double s = block_sum256(acc, threadIdx.x);
  if (threadIdx.x == 0) {
    out[0] = 0.5 * s;
    for (int k = 0; k < nrec; ++k) g[idx[k]] += u[idx[k]] - d[k];
  }
}

// Receivers must be interior nodes (bad[0] = 1 otherwise); checked before any read.
__global__ void k_check_idx(const int64_t* idx, int nrec, int n, int* bad) {
  const int64_t P = (int64_t)n + 1;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nrec; k += gridDim.x * blockDim.x) {
    const int64_t q = idx[k];
    const bool ok = q >= 0 && q < P * P && q % P >= 1 && q % P <= n - 1 && q / P >= 1 && q / P <= n - 1;
    if (!ok) bad[0] = 1;
  }
}

void launch_fwd_out2d(const double* cur, const double* prev, double* out, const double* kap,
                      const double* fs, double cosn, bool first, int n, hipStream_t s) {
  dim3 b(64, 4), g((n - 1 + 63) / 64, (n - 1 + 3) / 4);
  hipLaunchKernelGGL(k_fwd_out2d, g, b, 0, s, cur, prev, out, kap, fs, cosn, (int)first, n);
}

void launch_adj_step2d(const double* lam1, const double* lam2, double* lam_out, const double* W,
                       const double* kap, const double* z, double wn, double gscale, double* grad,
                       bool do_lam, int n, hipStream_t s) {
  dim3 b(64, 4), g((n + 1 + 63) / 64, (n + 1 + 3) / 4);
  hipLaunchKernelGGL(k_adj_step2d, g, b, 0, s, lam1, lam2, lam_out, W, kap, z, wn, gscale, grad,
                     (int)do_lam, n);
}

void launch_misfit(const double* u, const int64_t* idx, const double* d, int nrec, double* g,
                   double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_misfit, dim3(1), dim3(256), 0, s, u, idx, d, nrec, g, out);
}

void launch_check_idx(const int64_t* idx, int nrec, int n, int* bad, hipStream_t s) {
  hipLaunchKernelGGL(k_check_idx, dim3((nrec + 255) / 256), dim3(256), 0, s, idx, nrec, n, bad);
}

}  // namespace wh
