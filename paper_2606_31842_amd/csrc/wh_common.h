// Internal declarations shared by the libwaveholtz translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <exception>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/waveholtz.h"

struct wh_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  double* hbuf = nullptr;  // pinned host scalars
  int hbuf_len = 0;
  hipEvent_t rb_event = nullptr;   // marks the end of an asynchronous scalar read-back
  double* dred = nullptr;          // device: kReduceBlocks + 8 doubles for the context's own reductions
  // (dim, n, f32, varc, force) -> steps per launch K | (block shape << 8)
  std::map<std::tuple<int, int, int, int, int>, int> ktune;
};

namespace wh {

// Error message of a failure with no context to hold it (thread-local; wh_last_error(NULL)).
void set_thread_error(const char* msg);

// Entry-point guard: runs body() and turns any C++ exception into WH_EHOST with the
// message in the context (or the thread-local slot), so nothing throws across the ABI.
template <typename F>
wh_status guard(wh_ctx* ctx, F&& body) noexcept {
  const char* what = nullptr;
  try {
    return body();
  } catch (const std::exception& e) {
    what = e.what();
  } catch (...) {
    what = "unknown exception";
  }
  try {
    std::string m = std::string("internal host failure: ") + (what ? what : "");
    if (ctx) ctx->err = m;
    else set_thread_error(m.c_str());
  } catch (...) {
  }
  return WH_EHOST;
}

// The same for entry points that return a size (0 signals failure).
template <typename F>
size_t guard_size(F&& body) noexcept {
  try {
    return body();
  } catch (...) {
    set_thread_error("internal host failure while sizing the workspace");
    return 0;
  }
}

// Time discretisation of one wave solve (host, FP64).
struct TimeParams {
  int m = 0, nt = 0;
  double dt = 0, omega_w = 0, tbar = 0, c_max = 0;
  std::vector<double> w, cosv;
};
wh_status make_time_params(wh_ctx* ctx, int dim, int n, const wh_params& P, double c_max,
                           TimeParams& tp, int order = 2);
double transfer(const TimeParams& tp, double lam2);

// ----------------------------------------------------------------- device scalars
// Slots of the per-solve FP64 scalar block in the workspace.
enum Slot : int {
  S_R2 = 0,      // r^T r of the current residual
  S_PQ = 1,      // p^T A p
  S_ALPHA = 2,   // CG step length
  S_BETA = 3,    // CG direction update
  S_TMP = 4,     // scratch reduction target
  S_NB = 5,      // ||b||^2
  S_TMP2 = 6,
  S_NSLOTS_FIXED = 8,
  S_H = 8        // GMRES: Hessenberg column h_{0..m}, then deflation coefficients
};

constexpr int kBlock = 256;          // threads per block for 1D kernels
constexpr int kMaxTerms = 4096;       // separable terms of a factored deflation set
constexpr int kReduceBlocks = 1024;  // partial-sum slots for grid-stride 1D reductions

// ----------------------------------------------------------------- stencil launch
enum StepMode : int {
  M_FIRST = 0,   // W^1 from W^0 = v (D_0t W^0 = 0), V = w0 W^0 + w1 W^1, writes both states
  M_MID = 1,     // W^{n+1} = 2W^n - W^{n-1} + ...,  V += w W^{n+1}
  M_LAST_V = 2,  // last step, V += w W^{N_t}, state not stored
  M_LAST_AQ = 3, // last step, q = x - (V + w W^{N_t}); partial sums of x.q
  M_LAST_FPI = 4,// last step, out = V + w W^{N_t}; partial sums of (out - x)^2
  M_LAST_EQ = 5  // last step of the defect form: out = -(V + w W^{N_t}); partial sums of x.out
};

struct StepArgs {
  const void* cur;        // W^n (state type)
  void* prev;             // in: W^{n-1}; out: W^{n+1}  (M_FIRST: out W^0)
  void* cur_out;          // M_FIRST: out W^1
  const double* vin;      // M_FIRST: W^0 in FP64 (nodal; boundary read as 0)
  double* V;              // filter accumulator (FP64 nodal)
  const void* kap;        // variable c: c2 dt^2 / (2 h^2) nodal (state type)
  const void* fs;         // forcing: f dt^2 nodal, zero boundary (state type)
  double a;               // constant c: dt^2 / h^2
  double cosn;            // cos(omega_w t^n) for the forcing at step n
  double w0;              // M_FIRST: w_0
  double wn;              // weight of the new state (w_{n+1})
  const double* x;        // M_LAST_AQ / M_LAST_FPI: the vector being filtered
  double* out;            // M_LAST_AQ: q ; M_LAST_FPI: Pi x
  double* partials;       // per-block partial sums
  void* zb0;              // M_FIRST: second state pair whose boundary ring is zeroed
  void* zb1;
  void* cur_next;         // FP32 M_MID: out W^{n+1} (see below)
  int n;
};
// FP32 state pairs hold (W^n, D^{n-1/2} = W^n - W^{n-1}) instead of (W^n, W^{n-1}): the
// step is D^{n+1/2} = D^{n-1/2} + dt^2 (L_h W^n - f cos), W^{n+1} = W^n + D^{n+1/2}
// (the same recurrence; rounding no longer enters the low-frequency modes with the
// 1/(lambda dt) gain of the three-level form).  The "prev" buffer of a pair holds D.
// FP64 pairs keep (W^n, W^{n-1}).

// Launch one time step of a d-dimensional wave solve. T: float or double.
// Returns the number of blocks that wrote partial sums.
// Fourth-order (c == 1) single step, every mode; one block per 256 nodes.  Returns the
// number of blocks (= partial sums of the epilogue reductions).
int launch_step4(int dim, bool f32, bool force, StepMode mode, const StepArgs& a, hipStream_t s);
int step4_blocks(int dim, int n);
int launch_step(int dim, bool f32, bool varc, bool force, StepMode mode, const StepArgs& a,
                hipStream_t s);
int step_partial_blocks(int dim, int n);

// Fused k-step 2D launch (temporal blocking).  Advances (cur, prev) by k steps and
// accumulates sum_{j=1..k} w[j-1] W^{n+j} into V.  Returns false if unsupported.
struct FusedArgs {
  const void* cur;   // W^n
  const void* prev;  // W^{n-1}
  void* cur_out;     // W^{n+k}
  void* prev_out;    // W^{n+k-1}
  double* V;
  const void* kap;
  const void* fs;
  double a;
  const double* wts;     // host: w_{n+1..n+k}
  const double* cosv;    // host: cos(omega_w t^{n..n+k-1})
  int n;
  int k;
  int shape;             // block shape index, 0 .. kFusedShapes-1
  // 2D only: first launch of a wave solve (W^0 = vin, half step, V = w0 W^0 + ...) and
  // last launch (final step ends in the epilogue `last` instead of storing the state)
  int first = 0;
  const double* vin = nullptr;
  double w0 = 0;
  int last = M_MID;
  const double* x = nullptr;
  double* out = nullptr;
  double* partials = nullptr;
  // first launch only, instead of vin: W^0 = dr + beta dp with beta = dslots[S_BETA] (the
  // CG direction update), also written to dout over the interior
  const double* dr = nullptr;
  const double* dp = nullptr;
  const double* dslots = nullptr;
  double* dout = nullptr;
};
constexpr int kFusedShapes = 3;
bool fused2d_supported(bool f32, int k);
// Default block shape for a grid when no timing is available.
int fused2d_default_shape(bool f32, int n);
// Register rows per thread and wavefronts per block of a block shape.
void fused2d_shape_dims(bool f32, int k, int shape, int* rows, int* waves);
void launch_fused2d(bool f32, bool varc, bool force, const FusedArgs& a, hipStream_t s);

// Kernel arguments of the K-step 3D launch (wh_fused3d.hip): the state pair in and out, V, the
// coefficients, the tile grid (gx x gy x gz blocks, zs output planes per block) and the weights
// and cosines of the launch's steps.
struct Fused3Dev {
  const void* cur;
  const void* prev;
  void* cur_out;
  void* prev_out;
  double* V;
  const void* kap;
  const void* fs;
  double a;
  int n;
  int gx, gy, gz, zs;
  double w[8];    // w_{n+1..n+K}
  double cs[8];   // cos(omega_w t^{n..n+K-1})
};

// K (2 or 4) fourth-order steps of a 2D single solve (c == 1) by the row-marching pipeline
// (wh_march4.hip).  The state pair is read from (cur, prev) and written to (cur_out, prev_out)
// with the conventions of the other stepping kernels (FP32: W, D; FP64: W^n, W^{n-1}).
struct March4Args {
  const void* cur;
  const void* prev;
  void* cur_out;
  void* prev_out;
  double* V;
  const void* fs;     // dt^2 f in the state type, or NULL (no forcing)
  double a12;         // dt^2 / (12 h^2)
  double w[5];        // w[s] = filter weight of W^{n+s}, s = 1..K
  double cs[4];       // cs[s] = cos(omega t^{n+s}), s = 0..K-1
  int n;
  int kp;             // steps of this launch (<= K)
};
bool march4_supported(int K);
int march4_strip(int K);
int march4_tiles_x(int n, int K);
int march4_tiles_y(int n);
void launch_march4(bool f32, int K, const March4Args& a, hipStream_t s);
// Blocks (= partial sums) of a 2D blocked launch with this K and shape.
int fused2d_blocks(bool f32, int k, int shape, int n);
// 3D: K in {2, 3}; shapes give rows per thread, waves per block and output planes per block.
bool fused3d_supported(bool f32, int k);
void fused3d_shape_dims(bool f32, int shape, int* rows, int* waves, int* zs);
void launch_fused3d(bool f32, bool varc, bool force, const FusedArgs& a, hipStream_t s);

// ----------------------------------------------------------------- lane shifts
// Whole-wavefront shifts by one lane through DPP (wave_shr:1 / wave_shl:1): lane l
// receives lane l-1 (from_prev_lane) or lane l+1 (from_next_lane); the lane with no
// source receives 0 (bound_ctrl).  These are VALU moves the compiler can fold into
// the consuming instruction, unlike ds_bpermute shuffles.
__device__ __forceinline__ float from_prev_lane(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float from_next_lane(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ double from_prev_lane(double v) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)b, 0x138, 0xf, 0xf, true);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), 0x138, 0xf, 0xf, true);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
__device__ __forceinline__ double from_next_lane(double v) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)b, 0x130, 0xf, 0xf, true);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), 0x130, 0xf, 0xf, true);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}


// ----------------------------------------------------------------- BLAS-like kernels
void launch_prep_coeffs(const double* c2, const double* f, void* kap, void* fs, bool f32,
                        double kap_scale, double f_scale, int64_t N, int n, int dim,
                        hipStream_t s);
void launch_zero_boundary(double* u, int n, int dim, hipStream_t s);
// fs = -(dt^2 L_h + omega^2 dt^2) v at interior nodes (state type); boundary untouched.
// kap64: c2 dt^2/(2h^2) or NULL (then a = dt^2/h^2 is used).
void launch_defect_forcing(const double* v, const double* kap64, double a, double om2dt2, void* fs,
                           bool f32, int n, int dim, hipStream_t s);
void launch_max_partials(const double* a, int64_t N, double* partials, bool neg, hipStream_t s);
void launch_max_finalize(const double* partials, int count, double* out, hipStream_t s);
void launch_dot_partials(const double* a, const double* b, int64_t N, double* partials,
                         hipStream_t s);
// Classical Gram-Schmidt against the first nv columns of an Arnoldi basis V (column stride
// N).  project: partials [kReduceBlocks][nv] of V^T w.  update: w <- w - V h with
// h = slots[hsrc .. hsrc+nv), then partials of (V^T w, ||w||^2) (proj, [kReduceBlocks][nv+1];
// w must be column nv of the basis array) or of ||w||^2 ([kReduceBlocks]) for the updated w.
void launch_gs_project(const double* V, int64_t N, int nv, const double* w, double* partials,
                       hipStream_t s);
void launch_gs_update(const double* V, int64_t N, int nv, const double* slots, int hsrc, double* w,
                      bool proj, double* partials, hipStream_t s);
// slot[dst] = sum(partials[0..count)); mode 0 plain, 1: alpha = slot[R2]/sum (sum -> PQ),
// 2: beta = sum/slot[R2], slot[R2] = sum
void launch_reduce(const double* partials, int count, double* slots, int dst, int mode,
                   hipStream_t s);
void launch_set_beta(double* slots, int src, double r2_old, hipStream_t s);
// x += alpha p, r -= alpha q, partial sums of r.r into partials.  With pq_parts set, alpha
// (and slots[S_PQ], slots[S_ALPHA]) is formed from the pq_count partial sums of p.q in the
// same kernel, in place of a preceding launch_reduce(..., S_PQ, 1).
void launch_cg_update1(double* x, double* r, const double* p, const double* q, double* slots,
                       int64_t N, double* partials, hipStream_t s, const double* pq_parts = nullptr,
                       int pq_count = 0);
void launch_cg_update2(double* p, const double* r, const double* slots, int64_t N,
                       hipStream_t s);
// pn = r + beta p (beta from the slots), into a separate buffer
void launch_cg_update2_to(double* pn, const double* r, const double* p, const double* slots,
                          int64_t N, hipStream_t s);
void launch_axpy_slot(double* y, const double* x, const double* slots, int slot, double sign,
                      int64_t N, hipStream_t s);
void launch_axpy(double* y, const double* x, double alpha, int64_t N, hipStream_t s);
void launch_scale_copy(double* y, const double* x, const double* slots, int slot, int64_t N,
                       hipStream_t s);  // y = x / sqrt(slot)
void launch_sub(double* y, const double* a, const double* b, int64_t N, hipStream_t s);  // y=a-b
void launch_copy(double* y, const double* x, int64_t N, hipStream_t s);
// y = a x1 + b x2 + c x3 (y may alias an input; x3 may be NULL)
void launch_lincomb3(double* y, double a, const double* x1, double b, const double* x2, double c,
                     const double* x3, int64_t N, hipStream_t s);
void launch_gemv_acc(double* x, const double* V, int64_t ldv, int k, const double* y_dev,
                     int64_t N, hipStream_t s);  // x += V[:, :k] y
void launch_helmholtz_residual(const double* c2, const double* f, const double* u, double omega2,
                               double ih2, int n, int dim, int order, double* pr, double* pf,
                               hipStream_t s);
int helmholtz_partial_blocks(int n, int dim);

// ----------------------------------------------------------------- adjoint (2D)
void launch_fwd_out2d(const double* cur, const double* prev, double* out, const double* kap,
                      const double* fs, double cosn, bool first, int n, hipStream_t s);
void launch_adj_step2d(const double* lam1, const double* lam2, double* lam_out, const double* W,
                       const double* kap, const double* z, double wn, double gscale, double* grad,
                       bool do_lam, int n, hipStream_t s);
void launch_misfit(const double* u, const int64_t* idx, const double* d, int nrec, double* g,
                   double* out, hipStream_t s);
void launch_check_idx(const int64_t* idx, int nrec, int n, int* bad, hipStream_t s);

// Deflation: W^T r into slots[dst..dst+nd) and y -= W c (c from slots[src..]).
struct Defl {
  int kind = WH_DEFL_NONE;
  int nd = 0;
  int dim = 2;
  int n = 0;
  const double* tab = nullptr;  // sine: nd x dim x (n+1) table, [k][axis][i]; factored: nt x 2 x (n+1)
  const double* V = nullptr;    // dense
  int64_t ldv = 0;
  // factored (2D): nt separable terms, mode k owning terms toff[k] .. toff[k+1]-1
  int nt = 0;
  const int* tmap = nullptr;    // mode of each term
  const int* toff = nullptr;    // nd + 1 offsets
  double* tsum = nullptr;       // nt scratch: per-term projections
  double* tcoef = nullptr;      // nt scratch: per-term combination coefficients
};
int defl_partial_blocks(const Defl& d);
void launch_defl_project(const Defl& d, const double* r, double* partials, hipStream_t s);
// reduce nd columns of partials (count rows) into slots[dst + k]; scale by scale_dev[k] if set
void launch_defl_reduce(const double* partials, int count, int nd, double* slots, int dst,
                        const double* scale_dev, hipStream_t s);
// the partials of launch_defl_project for this set -> slots[dst + k] = (W^T r)_k (* scale_dev[k])
void launch_defl_reduce_set(const Defl& d, const double* partials, double* slots, int dst,
                            const double* scale_dev, hipStream_t s);
// y = alpha*y + beta*r - sum_k slots[src+k] W_k     (r may be null)
void launch_defl_combine(const Defl& d, double* y, double alpha, const double* r, double beta,
                         const double* slots, int src, int64_t N, hipStream_t s);
// p = beta_slot * p + r - W c  for CG with deflation
void launch_dcg_update2(const Defl& d, double* p, const double* r, const double* slots, int src,
                        int64_t N, hipStream_t s);
void launch_sine_tables(double* tab, const int32_t* modes_dev, int nd, int dim, int n,
                        hipStream_t s);
// slots[dst + k] = scale * (M slots[src ..])_k for a row-major nd x nd matrix M (nd <= 1024)
void launch_small_matvec(const double* M, int nd, double* slots, int src, int dst, double scale, hipStream_t s);

}  // namespace wh
