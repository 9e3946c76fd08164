// Host side of libwaveholtz: argument validation, time parameters, the wave-solve
// driver (one application of Pi_h) and the Krylov drivers.  All device work is
// enqueued on the context stream; scalars live in a small device block inside the
// caller's workspace and are read back through pinned host memory only where a
// host decision is needed (convergence tests, Givens rotations).
#include <algorithm>
#include <chrono>
#include <map>
#include <mutex>
#include <tuple>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "wh_common.h"

using namespace wh;


namespace {

constexpr int kHostScalars = 4096;

// ----------------------------------------------------------------- errors
#define WH_FAIL(ctx, code, ...)                                   \
  do {                                                            \
    char _b[512];                                                 \
    snprintf(_b, sizeof(_b), __VA_ARGS__);                        \
    if (ctx) (ctx)->err = _b;                                     \
    else wh::set_thread_error(_b);                                \
    return (code);                                                \
  } while (0)

#define HIPCHK(ctx, call)                                                         \
  do {                                                                            \
    hipError_t _e = (call);                                                       \
    if (_e != hipSuccess)                                                         \
      WH_FAIL(ctx, WH_EHIP, "%s failed: %s", #call, hipGetErrorString(_e));      \
  } while (0)

#define WHCHK(call)                 \
  do {                              \
    wh_status _s = (call);          \
    if (_s < 0) return _s;          \
  } while (0)

// ----------------------------------------------------------------- time parameters

}  // namespace

namespace wh {
// Section 2.2: dt from the CFL bound, m whole steps per period, the adjusted
// frequency omega_tilde = (2 pi/m)/dt with dt = 2 sin(pi/m)/omega (so that the
// leapfrog dispersion relation maps omega_tilde to omega), trapezoid weights
// w_n = (2/Tbar) eta_n dt (cos(omega_tilde t^n) - 1/4).
// Leapfrog stability: dt^2 max eig(-L_h) < 4.  Second order: max eig = 4 dim / h^2, so
// c dt / h < 1/sqrt(dim); fourth order: 16 dim / (3 h^2), so c dt / h < sqrt(3 / (4 dim)).
// 1D Dirichlet eigenvalue lambda_k^2 of the second- or fourth-order difference (the sine
// vectors are eigenvectors of both; the fourth-order boundary is closed by odd reflection)
double lam2_1d(int k, int n, int order) {
  const double h = 1.0 / n;
  if (order == 4) {
    const double t = M_PI * k * h;
    return (30.0 - 32.0 * std::cos(t) + 2.0 * std::cos(2.0 * t)) / (12.0 * h * h);
  }
  const double sv = std::sin(M_PI * k * h / 2.0);
  return 4.0 / (h * h) * sv * sv;
}

double cfl_limit(int dim, int order) {
  return order == 4 ? std::sqrt(3.0 / (4.0 * dim)) : 1.0 / std::sqrt((double)dim);
}

wh_status make_time_params(wh_ctx* ctx, int dim, int n, const wh_params& P, double c_max,
                           TimeParams& tp, int order) {
  const double h = 1.0 / n;
  if (!(c_max > 0) || !std::isfinite(c_max)) WH_FAIL(ctx, WH_EINVAL, "c_max must be > 0");
  int m = P.steps_per_period;
  if (m <= 0) {
    const double dt_cfl = P.cfl * h / c_max;
    m = std::max(3, (int)std::ceil(2.0 * M_PI / (P.omega * dt_cfl) - 1e-12));
  }
  if (m < 3) WH_FAIL(ctx, WH_EINVAL, "steps_per_period must be >= 3");
  const double theta = 2.0 * M_PI / m;
  double dt, omw;
  if (P.freq_correction) {
    dt = 2.0 * std::sin(theta / 2.0) / P.omega;
    omw = theta / dt;
  } else {
    dt = theta / P.omega;
    omw = P.omega;
  }
  const double cfl_eff = c_max * dt / h;
  if (cfl_eff >= cfl_limit(dim, order))
    WH_FAIL(ctx, WH_EINVAL, "time step violates the leapfrog stability bound (c dt/h = %g)", cfl_eff);
  tp.m = m;
  tp.nt = P.n_periods * m;
  tp.dt = dt;
  tp.omega_w = omw;
  tp.tbar = tp.nt * dt;
  tp.c_max = c_max;
  tp.w.resize(tp.nt + 1);
  tp.cosv.resize(tp.nt + 1);
  for (int k = 0; k <= tp.nt; ++k) {
    // cos(omega_w k dt) = cos(k theta) exactly under either reading; reduce k mod m first
    const double c = P.freq_correction ? std::cos(theta * (k % m)) : std::cos(omw * dt * k);
    const double eta = (k == 0 || k == tp.nt) ? 0.5 : 1.0;
    tp.cosv[k] = c;
    tp.w[k] = (2.0 / tp.tbar) * eta * dt * (c - 0.25);
  }
  return WH_OK;
}

// beta_h(lambda2) = sum_n w_n T_n(1 - lambda2 dt^2 / 2)
double transfer(const TimeParams& tp, double lam2) {
  const double x = 1.0 - 0.5 * lam2 * tp.dt * tp.dt;
  double t0 = 1.0, t1 = x;
  double s = tp.w[0] * t0 + tp.w[1] * t1;
  for (int k = 1; k < tp.nt; ++k) {
    double t2 = 2.0 * x * t1 - t0;
    s += tp.w[k + 1] * t2;
    t0 = t1;
    t1 = t2;
  }
  return s;
}

}  // namespace wh

namespace {

// ----------------------------------------------------------------- workspace layout
struct Layout {
  size_t total = 0;
  size_t Wa = 0, Wb = 0, Wc = 0, Wd = 0, V = 0, kap64 = 0, fs64 = 0, kap32 = 0, fs32 = 0;
  size_t b = 0, r = 0, p = 0, q = 0, ro = 0, d = 0, basis = 0, p2 = 0;
  bool has_p2 = false;   // CG/DCG: second direction buffer for the look-ahead
  size_t partials = 0, partials2 = 0, slots = 0, tab = 0, modes = 0, invmu = 0, ones = 0, tsum = 0;
  size_t aw = 0, einv = 0;   // general deflation vectors: A W (N x n_d) and (W^T A W)^{-1}
  int64_t N = 0;
  int nslots = 0, npart = 0;
};

size_t take(Layout& L, size_t bytes) {
  size_t off = L.total;
  L.total += (bytes + 255) & ~(size_t)255;
  return off;
}

int64_t nodal_count(int dim, int n) {
  int64_t P = n + 1;
  return dim == 2 ? P * P : P * P * P;
}

int defl_n(const wh_deflation* d) { return (d && d->kind != WH_DEFL_NONE) ? d->n_d : 0; }

// rows of the projection table: modes, or the separable terms of factored modes
int defl_rows(const wh_deflation* d) {
  const int nd = defl_n(d);
  if (nd && d->kind == WH_DEFL_FACTORED) return std::max(nd, std::min(d->n_terms, kMaxTerms));
  return nd;
}

Layout make_layout(const wh_grid& g, const wh_params& P, const wh_deflation* defl) {
  Layout L;
  const int64_t N = nodal_count(g.dim, g.n);
  L.N = N;
  const int nd = defl_n(defl);
  const bool mixed = P.precision == WH_MIXED;
  const int restart = std::max(1, P.restart);
  L.Wa = take(L, 8 * N);
  L.Wb = take(L, 8 * N);
  L.Wc = take(L, 8 * N);
  L.Wd = take(L, 8 * N);
  L.V = take(L, 8 * N);
  L.kap64 = take(L, 8 * N);
  L.fs64 = take(L, 8 * N);
  if (mixed) {
    L.kap32 = take(L, 4 * N);
    L.fs32 = take(L, 4 * N);
  }
  L.b = take(L, 8 * N);
  L.r = take(L, 8 * N);
  L.p = take(L, 8 * N);
  L.q = take(L, 8 * N);
  if (P.solver == WH_CG || P.solver == WH_DCG) {
    L.p2 = take(L, 8 * N);
    L.has_p2 = true;
  }
  if (mixed) {
    L.ro = take(L, 8 * N);
    L.d = take(L, 8 * N);
  }
  if (P.solver == WH_GMRES) L.basis = take(L, 8 * N * (size_t)(restart + 1));
  if (P.solver == WH_BICGSTAB) L.basis = take(L, 8 * N * 4);   // shadow residual, s, t, kept x
  Defl dd;
  dd.kind = nd ? defl->kind : WH_DEFL_NONE;
  dd.nd = nd;
  dd.dim = g.dim;
  dd.n = g.n;
  int np = std::max(kReduceBlocks, step_partial_blocks(g.dim, g.n));
  // 2D blocked launches end with one partial per block: room for the most blocks any
  // supported (precision, K, shape) launches on this grid
  if (g.dim == 2)
    for (int f = 0; f < 2; ++f)
      for (int k = 2; k <= 9; ++k)
        if (fused2d_supported(f == 1, k))
          for (int sh = 0; sh < kFusedShapes; ++sh) np = std::max(np, fused2d_blocks(f == 1, k, sh, g.n));
  if (g.order == 4) np = std::max(np, step4_blocks(g.dim, g.n));
  const int nrow = defl_rows(defl);
  if (nd) np = std::max(np, defl_partial_blocks(dd) * nrow);
  // Gram-Schmidt partials of GMRES: [kReduceBlocks][restart + 1]
  if (P.solver == WH_GMRES) np = std::max(np, kReduceBlocks * (restart + 2));
  L.npart = np;
  L.partials = take(L, 8 * (size_t)np);
  L.partials2 = take(L, 8 * (size_t)kReduceBlocks);
  L.nslots = S_H + restart + 2 + 2 * nd + 2 * (restart + 2) + 16;
  L.slots = take(L, 8 * (size_t)L.nslots);
  if (nd) {
    L.tab = take(L, 8 * (size_t)nrow * g.dim * (g.n + 1));
    // sine: mode numbers; factored: term -> mode map and mode offsets
    L.modes = take(L, 4 * (size_t)std::max(nd * g.dim, nrow + nd + 1));
    L.invmu = take(L, 8 * (size_t)nd);
    L.ones = take(L, 8 * (size_t)nd);
    L.tsum = take(L, 8 * 2 * (size_t)nrow);   // factored: per-term sums and coefficients
    if (dd.kind == WH_DEFL_DENSE) {
      L.aw = take(L, 8 * (size_t)N * nd);
      L.einv = take(L, 8 * (size_t)nd * nd);
    }
  }
  return L;
}

// The buffers one wave solve needs when its accumulator is the caller's output: the two
// state pairs, the scaled coefficients in each stepping precision, partial sums and scalars.
Layout make_filter_layout(const wh_grid& g, const wh_params& P) {
  Layout L;
  const int64_t N = nodal_count(g.dim, g.n);
  L.N = N;
  L.Wa = take(L, 8 * N);
  L.Wb = take(L, 8 * N);
  L.Wc = take(L, 8 * N);
  L.Wd = take(L, 8 * N);
  L.kap64 = take(L, 8 * N);
  L.fs64 = take(L, 8 * N);
  if (P.precision == WH_MIXED) {
    L.kap32 = take(L, 4 * N);
    L.fs32 = take(L, 4 * N);
  }
  L.npart = kReduceBlocks;
  L.partials = take(L, 8 * (size_t)kReduceBlocks);
  L.partials2 = take(L, 8 * (size_t)kReduceBlocks);
  L.nslots = S_NSLOTS_FIXED;
  L.slots = take(L, 8 * (size_t)L.nslots);
  return L;
}

template <typename T>
T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

// ----------------------------------------------------------------- validation
wh_status check_grid(wh_ctx* ctx, const wh_grid* g) {
  if (!g) WH_FAIL(ctx, WH_EINVAL, "grid is NULL");
  if (g->dim != 2 && g->dim != 3) WH_FAIL(ctx, WH_EUNSUPPORTED, "dim must be 2 or 3");
  if (g->order != 2 && g->order != 4) WH_FAIL(ctx, WH_EUNSUPPORTED, "order must be 2 or 4");
  if (g->n < 4) WH_FAIL(ctx, WH_EINVAL, "n must be >= 4");
  if (g->dim == 2 && g->n > 46340) WH_FAIL(ctx, WH_EINVAL, "n too large");
  if (g->dim == 3 && g->n > 1290) WH_FAIL(ctx, WH_EINVAL, "n too large");
  return WH_OK;
}

wh_status check_params(wh_ctx* ctx, const wh_grid* g, const wh_params* P) {
  if (!P) WH_FAIL(ctx, WH_EINVAL, "params is NULL");
  if (!(P->omega > 0) || !std::isfinite(P->omega)) WH_FAIL(ctx, WH_EINVAL, "omega must be > 0");
  if (P->n_periods < 1) WH_FAIL(ctx, WH_EINVAL, "n_periods must be >= 1");
  if (P->steps_per_period == 0 && !(P->cfl > 0 && P->cfl <= cfl_limit(g->dim, g->order)))
    WH_FAIL(ctx, WH_EINVAL, "cfl must lie in (0, %g] for this dim and order", cfl_limit(g->dim, g->order));
  if (P->steps_per_period < 0 || (P->steps_per_period > 0 && P->steps_per_period < 3))
    WH_FAIL(ctx, WH_EINVAL, "steps_per_period must be 0 or >= 3");
  if (P->precision != WH_F64 && P->precision != WH_MIXED) WH_FAIL(ctx, WH_EINVAL, "bad precision");
  if (P->c_max < 0) WH_FAIL(ctx, WH_EINVAL, "c_max must be >= 0");
  if (P->k_fuse < 0 || P->k_fuse > 64) WH_FAIL(ctx, WH_EINVAL, "k_fuse must be in [0, 64]");
  if (P->k_shape < -1 || P->k_shape >= kFusedShapes)
    WH_FAIL(ctx, WH_EINVAL, "k_shape must be -1 or in [0, %d)", kFusedShapes);
  return WH_OK;
}

wh_status check_defl(wh_ctx* ctx, const wh_grid* g, const wh_deflation* d, bool varc) {
  if (!d || d->kind == WH_DEFL_NONE) return WH_OK;
  if (d->n_d < 0 || d->n_d > 256) WH_FAIL(ctx, WH_EINVAL, "n_d must be in [0, 256]");
  if (d->n_d == 0) return WH_OK;
  if (d->kind == WH_DEFL_SINE) {
    if (varc) WH_FAIL(ctx, WH_EUNSUPPORTED, "analytic sine modes need c == 1 (c2 == NULL)");
    if (!d->modes) WH_FAIL(ctx, WH_EINVAL, "deflation modes is NULL");
    for (int k = 0; k < d->n_d * g->dim; ++k)
      if (d->modes[k] < 1 || d->modes[k] > g->n - 1) WH_FAIL(ctx, WH_EINVAL, "mode number out of range");
  } else if (d->kind == WH_DEFL_DENSE_EXACT) {
    if (!d->V || !d->lambda2) WH_FAIL(ctx, WH_EINVAL, "dense deflation needs V and lambda2");
    if (d->ldv < nodal_count(g->dim, g->n)) WH_FAIL(ctx, WH_EINVAL, "ldv too small");
  } else if (d->kind == WH_DEFL_DENSE) {
    if (!d->V) WH_FAIL(ctx, WH_EINVAL, "dense deflation needs V");
    if (d->ldv < nodal_count(g->dim, g->n)) WH_FAIL(ctx, WH_EINVAL, "ldv too small");
  } else if (d->kind == WH_DEFL_FACTORED) {
    if (g->dim != 2) WH_FAIL(ctx, WH_EUNSUPPORTED, "factored deflation vectors are 2D");
    if (!d->fx || !d->fy || !d->lambda2 || !d->term_mode)
      WH_FAIL(ctx, WH_EINVAL, "factored deflation needs fx, fy, term_mode and lambda2");
    if (d->n_terms < d->n_d || d->n_terms > kMaxTerms)
      WH_FAIL(ctx, WH_EINVAL, "n_terms must be in [n_d, %d]", kMaxTerms);
    int prev = -1;
    for (int t = 0; t < d->n_terms; ++t) {
      const int k = d->term_mode[t];
      if (k < prev || k > prev + 1 || k >= d->n_d)
        WH_FAIL(ctx, WH_EINVAL, "term_mode must be nondecreasing and cover modes 0..n_d-1");
      prev = k;
    }
    if (prev != d->n_d - 1) WH_FAIL(ctx, WH_EINVAL, "term_mode must cover modes 0..n_d-1");
  } else {
    WH_FAIL(ctx, WH_EINVAL, "bad deflation kind");
  }
  return WH_OK;
}

wh_status check_ws(wh_ctx* ctx, void* ws, size_t ws_bytes, size_t need) {
  if (!ws) WH_FAIL(ctx, WH_EWORKSPACE, "workspace is NULL (need %zu bytes)", need);
  if (((uintptr_t)ws) & 255) WH_FAIL(ctx, WH_EWORKSPACE, "workspace must be 256-byte aligned");
  if (ws_bytes < need) WH_FAIL(ctx, WH_EWORKSPACE, "workspace too small: %zu < %zu", ws_bytes, need);
  return WH_OK;
}

// ----------------------------------------------------------------- host read-back
wh_status readback(wh_ctx* ctx, const double* dev, int count) {
  if (count > ctx->hbuf_len) WH_FAIL(ctx, WH_EINVAL, "read-back too large");
  HIPCHK(ctx, hipMemcpyAsync(ctx->hbuf, dev, sizeof(double) * count, hipMemcpyDeviceToHost,
                             ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  return WH_OK;
}

// Read-back in two halves: the copy is queued (and an event after it), work queued
// next keeps the GPU busy, and readback_wait blocks until the copy alone has finished.
wh_status readback_async(wh_ctx* ctx, const double* dev, int count) {
  if (count > ctx->hbuf_len) WH_FAIL(ctx, WH_EINVAL, "read-back too large");
  HIPCHK(ctx, hipMemcpyAsync(ctx->hbuf, dev, sizeof(double) * count, hipMemcpyDeviceToHost,
                             ctx->stream));
  HIPCHK(ctx, hipEventRecord(ctx->rb_event, ctx->stream));
  return WH_OK;
}

wh_status readback_wait(wh_ctx* ctx) {
  HIPCHK(ctx, hipEventSynchronize(ctx->rb_event));
  return WH_OK;
}

wh_status upload(wh_ctx* ctx, double* dev, const double* host, int count) {
  if (count > ctx->hbuf_len) WH_FAIL(ctx, WH_EINVAL, "upload too large");
  // stage through pinned memory; the copy is complete before this returns
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  std::memcpy(ctx->hbuf, host, sizeof(double) * count);
  HIPCHK(ctx, hipMemcpyAsync(dev, ctx->hbuf, sizeof(double) * count, hipMemcpyHostToDevice,
                             ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  return WH_OK;
}

// ----------------------------------------------------------------- wave solve
struct WaveOp {
  int dim = 2, n = 0;
  bool varc = false, f32 = false;
  void* Wa = nullptr;
  void* Wb = nullptr;
  void* Wc = nullptr;   // second state pair for the temporally blocked kernel
  void* Wd = nullptr;
  double* V = nullptr;
  const void* kap = nullptr;
  const void* fs = nullptr;
  double a = 0;  // dt^2/h^2
  const TimeParams* tp = nullptr;
  double* partials = nullptr;
  int k_fuse = 1;
  int k_shape = 0;   // block shape of the temporally blocked kernel
  int order = 2;     // 4: the fourth-order single-step kernel (c == 1)
};

// The temporally blocked kernels: 2D (register tiles) and 3D (z-marching pipeline).
bool fused_supported(int dim, bool f32, int k) {
  return dim == 2 ? fused2d_supported(f32, k) : fused3d_supported(f32, k);
}
void launch_fused(int dim, bool f32, bool varc, bool force, const FusedArgs& fa, hipStream_t s) {
  if (dim == 2) launch_fused2d(f32, varc, force, fa, s);
  else launch_fused3d(f32, varc, force, fa, s);
}
void fused_shape_dims(int dim, bool f32, int k, int shape, int* rows, int* waves) {
  if (dim == 2) {
    fused2d_shape_dims(f32, k, shape, rows, waves);
  } else {
    int zs = 0;
    fused3d_shape_dims(f32, shape, rows, waves, &zs);
  }
}

// One wave solve from W^0 = vin.  last = M_LAST_V: V holds Pi_h(vin);
// M_LAST_AQ: out = x - Pi_h(vin) with partial sums of x.out (x == vin);
// M_LAST_FPI: out = Pi_h(vin) with partial sums of (out - x)^2.
// Split N_t steps into blocked launches of supported sizes (K where possible).
std::vector<int> plan_launches(int nt, int K, bool f32) {
  std::vector<int> parts;
  auto ok = [&](int k) { return k >= 2 && fused2d_supported(f32, k); };
  // decompose r (>= 2) into supported sizes <= K, largest first (r <= 2K + 1)
  auto split = [&](int r) {
    std::vector<int> best;
    for (int a = std::min(K, r); a >= 2; --a) {
      if (!ok(a)) continue;
      if (a == r) return std::vector<int>{a};
      for (int b = std::min(a, r - a); b >= 2; --b) {
        if (!ok(b)) continue;
        if (a + b == r) return std::vector<int>{a, b};
        for (int c = std::min(b, r - a - b); c >= 2; --c)
          if (ok(c) && a + b + c == r) best = {a, b, c};
      }
      if (!best.empty()) return best;
    }
    return best;
  };
  int full = nt / K, rem = nt % K;
  if (rem == 1 && full > 1 && ok(K + 1)) {
    // one launch of K + 1 takes the odd step; it is the one before the last, so that the
    // last launch (the epilogue) keeps the size of the others
    for (int i = 0; i < full - 2; ++i) parts.push_back(K);
    parts.push_back(K + 1);
    parts.push_back(K);
    return parts;
  }
  if (rem == 1 && full > 0) {
    --full;
    rem += K;
  }
  for (int i = 0; i < full; ++i) parts.push_back(K);
  if (rem > 0) {
    std::vector<int> tail = split(rem);
    if (tail.empty()) return {};
    parts.insert(parts.end(), tail.begin(), tail.end());
  }
  return parts;
}

// one single-step launch of the operator's order
int step_any(const WaveOp& op, bool force, StepMode mode, const StepArgs& a, hipStream_t s) {
  if (op.order == 4) return launch_step4(op.dim, op.f32, force, mode, a, s);
  return launch_step(op.dim, op.f32, op.varc, force, mode, a, s);
}

// A CG direction update p' = r + beta p (beta = slots[S_BETA]) that a wave solve forms as
// its input; out receives p' (distinct from r and p).
struct DirUpd {
  const double* r;
  const double* p;
  const double* slots;
  double* out;
};

// One wave solve from vin (or from the direction update du, whose result is also the
// epilogue's x when x == du->out).  Returns the number of partial sums the epilogue wrote.
int wave_solve(const WaveOp& op, const double* vin, bool force, StepMode last, const double* x,
               double* out, hipStream_t s, const DirUpd* du = nullptr) {
  const TimeParams& tp = *op.tp;
  const bool fused2d = op.order == 2 && op.dim == 2 && op.k_fuse > 1 && fused2d_supported(op.f32, op.k_fuse);
  const std::vector<int> parts = fused2d ? plan_launches(tp.nt, op.k_fuse, op.f32) : std::vector<int>{};
  if (du && parts.size() < 2) {
    // no blocked first launch to fuse the update into: form p' on its own
    launch_cg_update2_to(du->out, du->r, du->p, du->slots, nodal_count(op.dim, op.n), s);
    vin = du->out;
    du = nullptr;
  }
  if (fused2d) {
    // 2D: every step in blocked launches; the first starts from vin with the half step,
    // the last ends in the epilogue (no streaming kernels)
    // at least two launches: vin (read with halo by the first) may alias out (written by
    // the last), as in the fixed-point update x <- Pi x
    if (parts.size() >= 2) {
      FusedArgs fa{};
      fa.V = op.V;
      fa.kap = op.kap;
      fa.fs = force ? op.fs : nullptr;
      fa.a = op.a;
      fa.n = op.n;
      fa.shape = op.k_shape;
      fa.vin = vin;
      fa.w0 = tp.w[0];
      fa.x = x;
      fa.out = out;
      fa.partials = op.partials;
      void* cur = op.Wb;
      void* prev = op.Wa;
      void* oc = op.Wc;
      void* op_ = op.Wd;
      int nn = 0;
      for (size_t i = 0; i < parts.size(); ++i) {
        fa.k = parts[i];
        fa.cur = cur;
        fa.prev = prev;
        fa.cur_out = oc;
        fa.prev_out = op_;
        fa.wts = &tp.w[nn + 1];
        fa.cosv = &tp.cosv[nn];
        fa.first = i == 0;
        fa.last = i + 1 == parts.size() ? last : M_MID;
        if (du && i == 0) {
          fa.dr = du->r;
          fa.dp = du->p;
          fa.dslots = du->slots;
          fa.dout = du->out;
        } else {
          fa.dr = fa.dp = fa.dslots = nullptr;
          fa.dout = nullptr;
        }
        launch_fused2d(op.f32, op.varc, force, fa, s);
        std::swap(cur, oc);
        std::swap(prev, op_);
        nn += parts[i];
      }
      return last == M_LAST_V ? 0 : fused2d_blocks(op.f32, parts.back(), op.k_shape, op.n);
    }
  }
  StepArgs a{};
  a.n = op.n;
  a.kap = op.kap;
  a.fs = force ? op.fs : nullptr;
  a.a = op.a;
  a.vin = vin;
  a.prev = op.Wa;
  a.cur_out = op.Wb;
  a.V = op.V;
  a.w0 = tp.w[0];
  a.wn = tp.w[1];
  a.cosn = tp.cosv[0];
  a.zb0 = op.Wc;
  a.zb1 = op.Wd;
  step_any(op, force, M_FIRST, a, s);
  a.zb0 = a.zb1 = nullptr;
  void* cur = op.Wb;
  void* prev = op.Wa;
  void* oc = op.Wc;
  void* op_ = op.Wd;
  int nn = 1;  // cur holds W^nn
  if (op.order == 4 && op.dim == 2 && op.k_fuse > 1) {
    // fourth order: the steps between the first and the last by the row-marching launches
    // (the largest supported K that still leaves the last step to the epilogue)
    int Kc = op.k_fuse;
    while (true) {
      while (Kc > 1 && (nn + Kc > tp.nt - 1 || !march4_supported(Kc))) --Kc;
      if (Kc <= 1) break;
      March4Args m{};
      m.cur = cur;
      m.prev = prev;
      m.cur_out = oc;
      m.prev_out = op_;
      m.V = op.V;
      m.fs = force ? op.fs : nullptr;
      m.a12 = op.a / 12.0;
      for (int j = 1; j <= Kc; ++j) m.w[j] = tp.w[nn + j];
      for (int j = 0; j < Kc; ++j) m.cs[j] = tp.cosv[nn + j];
      m.n = op.n;
      m.kp = Kc;
      launch_march4(op.f32, Kc, m, s);
      std::swap(cur, oc);
      std::swap(prev, op_);
      nn += Kc;
    }
  }
  const int K = op.order == 2 ? op.k_fuse : 1;
  if (K > 1 && fused_supported(op.dim, op.f32, K)) {
    FusedArgs fa{};
    fa.V = op.V;
    fa.kap = op.kap;
    fa.fs = force ? op.fs : nullptr;
    fa.a = op.a;
    fa.n = op.n;
    fa.k = K;
    fa.shape = op.k_shape;
    // the last step stays with the streaming kernel (it carries the epilogue); the
    // remainder is covered by the largest supported K that still fits
    int Kc = K;
    while (true) {
      while (Kc > 1 && (nn + Kc > tp.nt - 1 || !fused_supported(op.dim, op.f32, Kc))) --Kc;
      if (Kc <= 1) break;
      fa.k = Kc;
      fa.cur = cur;
      fa.prev = prev;
      fa.cur_out = oc;
      fa.prev_out = op_;
      fa.wts = &tp.w[nn + 1];
      fa.cosv = &tp.cosv[nn];
      launch_fused(op.dim, op.f32, op.varc, force, fa, s);
      std::swap(cur, oc);
      std::swap(prev, op_);
      nn += Kc;
    }
  }
  int nblk = 0;
  for (int k = nn; k < tp.nt; ++k) {
    a.cur = cur;
    a.prev = prev;
    a.cur_next = oc;   // FP32: W^{n+1} goes to a free buffer, D is updated in place
    a.cosn = tp.cosv[k];
    a.wn = tp.w[k + 1];
    a.x = x;
    a.out = out;
    a.partials = op.partials;
    const StepMode md = (k == tp.nt - 1) ? last : M_MID;
    nblk = step_any(op, force, md, a, s);
    if (op.f32) std::swap(cur, oc);
    else std::swap(cur, prev);
  }
  return nblk;
}

// ----------------------------------------------------------------- autotuner
// Steps per launch and block shape of the temporally blocked 2D kernel: time every
// supported (K, shape) on this grid (after one warm-up launch) and keep the fastest
// per-step time; K = 1 is the streaming kernel.  Candidates within 3% of the fastest
// count as equal and the largest K among them wins (then the earlier shape), so that
// timing noise does not flip the choice from one context to the next.  k_fixed > 0
// restricts the search to that K.  The state buffers and V serve as scratch; every
// caller initialises them afterwards.  Returns K | (shape << 8), cached per context.
int autotune_k(wh_ctx* ctx, const WaveOp& op, bool force, int k_fixed = 0) {
  const auto key = std::make_tuple(op.dim, op.n, (int)op.f32, (int)op.varc, (int)force + 2 * k_fixed);
  auto it = ctx->ktune.find(key);
  if (it != ctx->ktune.end()) return it->second;
  const TimeParams& tp = *op.tp;
  const int fallback = k_fixed > 1 ? (k_fixed | ((op.dim == 2 ? fused2d_default_shape(op.f32, op.n) : 0) << 8))
                                   : (op.dim == 2 ? 4 : 1);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return fallback;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fallback;
  }
  int best = k_fixed == 1 ? 1 : fallback;
  float best_t = 1e30f;
  int tried_code[64];
  float tried_t[64];
  int n_tried = 0;
  const int cands[] = {1, 2, 3, 4, 6, 8};
  for (int K : cands) {
    if (k_fixed > 0 && K != k_fixed) continue;
    if (K > 1 && (!fused_supported(op.dim, op.f32, K) || K + 2 > tp.nt)) continue;
    for (int shape = 0; shape < (K == 1 ? 1 : kFusedShapes); ++shape) {
      auto run = [&]() {
        if (K == 1) {
          StepArgs a{};
          a.n = op.n;
          a.kap = op.kap;
          a.fs = force ? op.fs : nullptr;
          a.a = op.a;
          a.cur = op.Wb;
          a.prev = op.Wa;
          a.cur_next = op.Wc;
          a.V = op.V;
          a.cosn = tp.cosv[1];
          a.wn = tp.w[2];
          launch_step(op.dim, op.f32, op.varc, force, M_MID, a, ctx->stream);
        } else {
          FusedArgs fa{};
          fa.V = op.V;
          fa.kap = op.kap;
          fa.fs = force ? op.fs : nullptr;
          fa.a = op.a;
          fa.n = op.n;
          fa.k = K;
          fa.shape = shape;
          fa.cur = op.Wb;
          fa.prev = op.Wa;
          fa.cur_out = op.Wc;
          fa.prev_out = op.Wd;
          fa.wts = &tp.w[2];
          fa.cosv = &tp.cosv[1];
          launch_fused(op.dim, op.f32, op.varc, force, fa, ctx->stream);
        }
      };
      run();
      const int reps = 5;
      (void)hipEventRecord(e0, ctx->stream);
      for (int r = 0; r < reps; ++r) run();
      (void)hipEventRecord(e1, ctx->stream);
      if (hipEventSynchronize(e1) != hipSuccess) break;
      float ms = 0;
      (void)hipEventElapsedTime(&ms, e0, e1);
      const float per_step = ms / (reps * K);
      if (n_tried < 64) {
        tried_code[n_tried] = K | (shape << 8);
        tried_t[n_tried++] = per_step;
      }
      best_t = std::min(best_t, per_step);
    }
  }
  // candidates are visited by increasing K, then shape: the last one within the
  // tolerance has the largest K and, for that K, the first such shape
  int best_k = 0;
  for (int i = 0; i < n_tried; ++i) {
    const int K = tried_code[i] & 0xff;
    if (tried_t[i] <= 1.03f * best_t && K > best_k) {
      best_k = K;
      best = tried_code[i];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  ctx->ktune[key] = best;
  return best;
}

// Steps per launch and shape without timing anything: the autotuner's cached choice for
// this grid if there is one, else K (8 by default) with the default block shape.
int untuned_k(wh_ctx* ctx, const WaveOp& op, int k_fixed) {
  auto it = ctx->ktune.find(std::make_tuple(op.dim, op.n, (int)op.f32, (int)op.varc, 2 * k_fixed));
  if (it != ctx->ktune.end()) return it->second;
  const int K = k_fixed > 1 ? k_fixed : (op.dim == 2 ? 8 : 3);
  if (!fused_supported(op.dim, op.f32, K)) return 1;
  return K | ((op.dim == 2 ? fused2d_default_shape(op.f32, op.n) : 0) << 8);
}

// ----------------------------------------------------------------- solver state
struct Solver {
  wh_ctx* ctx;
  hipStream_t s;
  int64_t N;
  WaveOp op64, op32;
  double* slots;
  double* partials;
  double* partials2;
  Defl defl;
  const double* invmu = nullptr;   // 1/mu_k (device)
  const double* negmu = nullptr;   // -1/mu_k (device) for the deflated start
  double* p2 = nullptr;            // CG: spare direction buffer (look-ahead); nullptr: none
  int ws64 = 0, ws32 = 0;          // wave-solve counters
  int iters = 0;
  bool defect = true;              // FP32 A-applies in the defect form
  double om2dt2 = 0;               // omega^2 dt^2
  double reliable_drop = 0.1;  // mixed CG: residual reduction between FP64 replacements
  std::vector<double> mu;          // mu_k = 1 - beta_h(lambda_k^2) of the deflation set (host)
  // general deflation vectors (not eigenvectors): A W and (W^T A W)^{-1}, row-major (device)
  bool general = false;
  Defl defl_aw;
  const double* einv = nullptr;
};

// q = A x (x nonzero).  Leaves partial sums of x.q in op.partials.
// FP32 stepping uses the defect form A x = Pi_h(0; (L_h + omega^2) x): the state that is
// stepped (and rounded) is W^n - cos(omega_w t^n) x, which is small for the components
// of x near resonance, where A's eigenvalues are small.
int applyA(Solver& S, bool f32, const double* x, double* q) {
  const WaveOp& op = f32 ? S.op32 : S.op64;
  (f32 ? S.ws32 : S.ws64)++;
  if (f32 && S.defect) {
    launch_defect_forcing(x, op.varc ? (const double*)S.op64.kap : nullptr, op.a, S.om2dt2,
                          (void*)op.fs, true, op.n, op.dim, S.s);
    return wave_solve(op, nullptr, true, M_LAST_EQ, x, q, S.s);
  }
  return wave_solve(op, x, false, M_LAST_AQ, x, q, S.s);
}

// pn = r + beta p, then q = A pn; in the blocked 2D form the update is part of the wave
// solve's first launch.  Same values as launch_cg_update2_to followed by applyA.
int applyA_dir(Solver& S, bool f32, const double* r, const double* p, double* pn, double* q) {
  if (f32 && S.defect) {
    launch_cg_update2_to(pn, r, p, S.slots, S.N, S.s);
    return applyA(S, f32, pn, q);
  }
  const WaveOp& op = f32 ? S.op32 : S.op64;
  (f32 ? S.ws32 : S.ws64)++;
  const DirUpd du{r, p, S.slots, pn};
  return wave_solve(op, nullptr, false, M_LAST_AQ, pn, q, S.s, &du);
}

// slots[dst] = a . b
void dot(Solver& S, const double* a, const double* b, int dst) {
  launch_dot_partials(a, b, S.N, S.partials2, S.s);
  launch_reduce(S.partials2, kReduceBlocks, S.slots, dst, 0, S.s);
}

struct KrylovResult {
  double rel = 0;
  int iters = 0;
  wh_status st = WH_OK;
  bool diverged = false;   // residual grew past 1e3 x the right-hand side (abandoned)
  int replacements = 0;    // reliable-update residual replacements (FP64 wave solves)
};

// CG / DCG (Algorithm 3) for A x = rhs with A applied in the requested precision.
// x holds the initial guess (x_nonzero says whether it can be nonzero).  Stops on
// ||r|| <= tol * ||rhs||.  Uses S.partials for step partials.
//
// reliable = true (mixed precision): the recurrence applies the FP32-stepped operator,
// and whenever the recursive residual has fallen by the factor S.reliable_drop since
// the last replacement, has grown tenfold, or looks converged, it is replaced by the
// true residual rhs - A x computed with an FP64 wave solve, beta being formed from the
// replaced residual.  The CG recurrence itself is never restarted.  If two
// consecutive replacements do not halve the true residual, the FP32 operator error
// is too large for this problem and the remaining iterations apply the FP64 operator.

// The filter's eigenvalues beta_h lie in [-1/2, 1] when the leapfrog scheme is stable (Section 2.3),
// so A = I - S_h has |p^T A p| <= 1.5 |p|^2.  Where p = r (CG's first iteration without
// deflation, the start of a BiCGStab run), |p^T A p| > 6 r^T r shows a growing wave solve (a
// c_max below the largest c, or a time step beyond the CFL bound) rather than a solvable system.
wh_status check_stable_filter(wh_ctx* ctx, int k, int nd, double pq, double r2_first) {
  if (k != 0 || nd != 0 || !(r2_first > 0)) return WH_OK;
  if (std::fabs(pq) > 6.0 * r2_first)
    WH_FAIL(ctx, WH_EUNSTABLE, "|p^T A p| = %.3g |p|^2 exceeds the bound 1.5 of a stable filter: the wave "
            "solve is unstable (c_max below the largest c, or the time step above the CFL bound)",
            std::fabs(pq) / r2_first);
  return WH_OK;
}

wh_status cg_solve(Solver& S, bool f32, const double* rhs, double* x, bool x_nonzero, double* r,
                   double* p, double* q, double tol, int maxit, bool use_defl, bool reproject,
                   int check_every, KrylovResult& res, bool stop_on_divergence = false,
                   bool reliable = false) {
  wh_ctx* ctx = S.ctx;
  const int64_t N = S.N;
  const int nd = use_defl ? S.defl.nd : 0;
  // true residuals are always formed with the FP64 operator in reliable mode
  const bool f32_true = reliable ? false : f32;
  // ||rhs||^2
  dot(S, rhs, rhs, S_NB);
  // r_{-1}
  if (x_nonzero) {
    applyA(S, f32_true, x, q);
    launch_sub(r, rhs, q, N, S.s);
  } else {
    launch_copy(r, rhs, N, S.s);
  }
  if (nd && S.general) {
    // general vectors: x_0 = x_{-1} + W (W^T A W)^{-1} W^T r_{-1}; r_0 = rhs - A x_0;
    // mu_0 = (W^T A W)^{-1} (A W)^T r_0 (A symmetric); p_0 = r_0 - W mu_0.  The coefficients
    // are formed in slots [S_H + nd, S_H + 2 nd) from the projections in [S_H, S_H + nd).
    launch_defl_project(S.defl, r, S.partials, S.s);
    launch_defl_reduce_set(S.defl, S.partials, S.slots, S_H, nullptr, S.s);
    launch_small_matvec(S.einv, nd, S.slots, S_H, S_H + nd, -1.0, S.s);
    launch_defl_combine(S.defl, x, 1.0, nullptr, 0.0, S.slots, S_H + nd, N, S.s);
    applyA(S, f32_true, x, q);
    launch_sub(r, rhs, q, N, S.s);
    launch_defl_project(S.defl_aw, r, S.partials, S.s);
    launch_defl_reduce_set(S.defl_aw, S.partials, S.slots, S_H, nullptr, S.s);
    launch_small_matvec(S.einv, nd, S.slots, S_H, S_H + nd, 1.0, S.s);
    launch_defl_combine(S.defl, p, 0.0, r, 1.0, S.slots, S_H + nd, N, S.s);
  } else if (nd) {
    // x_0 = x_{-1} + W (W^T A W)^{-1} W^T r_{-1}
    launch_defl_project(S.defl, r, S.partials, S.s);
    launch_defl_reduce_set(S.defl, S.partials, S.slots, S_H, S.negmu, S.s);
    launch_defl_combine(S.defl, x, 1.0, nullptr, 0.0, S.slots, S_H, N, S.s);
    // r_0 = rhs - A x_0
    applyA(S, f32_true, x, q);
    launch_sub(r, rhs, q, N, S.s);
    // mu_0 = (W^T A W)^{-1} (A W)^T r_0 = W^T r_0 for eigenvectors; p_0 = r_0 - W mu_0
    launch_defl_project(S.defl, r, S.partials, S.s);
    launch_defl_reduce_set(S.defl, S.partials, S.slots, S_H, nullptr, S.s);
    launch_defl_combine(S.defl, p, 0.0, r, 1.0, S.slots, S_H, N, S.s);
  } else {
    launch_copy(p, r, N, S.s);
  }
  dot(S, r, r, S_R2);
  WHCHK(readback(ctx, S.slots, S_NSLOTS_FIXED));
  const double nb2 = ctx->hbuf[S_NB];
  double r2 = ctx->hbuf[S_R2];
  if (!(nb2 > 0)) {
    res.rel = 0;
    res.iters = 0;
    res.st = WH_OK;
    return WH_OK;
  }
  double rel = std::sqrt(r2 / nb2);
  if (!std::isfinite(rel)) WH_FAIL(ctx, WH_EUNSTABLE, "non-finite residual (unstable wave solve?)");
  int k = 0;
  const int ce = reliable ? 1 : std::max(1, check_every);
  bool op32 = f32;
  double anchor = rel;        // relative true residual at the last replacement
  int stalls = 0, last_repl = 0;
  res.replacements = 0;
  // Look-ahead: while the host waits for an iteration's scalars, the GPU already forms
  // the next direction p' = r + beta p in the spare buffer and applies A to it, as if the
  // iteration went on unchanged.  When it does not (a residual replacement, convergence,
  // a stop), that A-apply is discarded: its result is overwritten before use and it is not
  // counted as a wave solve.  Needs S.p2 and the plain direction update (no re-projection).
  double* pc = p;                 // this iteration's direction
  int nb_ahead = -1;              // >= 0: A pc is already queued (its partial-sum count)
  bool ahead_f32 = false;
  const bool can_ahead = S.p2 != nullptr && !(nd && (reproject || S.general));
  auto discard_ahead = [&]() {
    if (nb_ahead >= 0) (ahead_f32 ? S.ws32 : S.ws64)--;
    nb_ahead = -1;
  };
  while (rel > tol && k < maxit) {
    const double r2_old = r2;
    const int nb = nb_ahead >= 0 ? nb_ahead : applyA(S, op32, pc, q);
    nb_ahead = -1;
    // alpha from the A-apply's partial sums: inside the update kernel when they are few
    // (each of its blocks sums them), else by a reduction launch of its own
    if (nb <= 4096) {
      launch_cg_update1(x, r, pc, q, S.slots, N, S.partials2, S.s, S.partials, nb);
    } else {
      launch_reduce(S.partials, nb, S.slots, S_PQ, 1, S.s);
      launch_cg_update1(x, r, pc, q, S.slots, N, S.partials2, S.s);
    }
    launch_reduce(S.partials2, kReduceBlocks, S.slots, S_R2, 2, S.s);
    // the first iteration always reads back, so that an unstable wave solve is caught at once
    const bool sync = reliable || k == 0 || (k + 1) % ce == 0 || k + 1 == maxit;
    double* pn = nullptr;
    if (sync) {
      WHCHK(readback_async(ctx, S.slots, S_NSLOTS_FIXED));
      if (can_ahead && k + 1 < maxit) {
        pn = pc == p ? S.p2 : p;
        ahead_f32 = op32;
        nb_ahead = applyA_dir(S, op32, r, pc, pn, q);
      }
      WHCHK(readback_wait(ctx));
    }
    if (reliable) {
      const double pq = ctx->hbuf[S_PQ];
      r2 = ctx->hbuf[S_R2];
      if (!std::isfinite(pq) || !std::isfinite(r2))
        WH_FAIL(ctx, WH_EUNSTABLE, "non-finite p^T A p or residual at iteration %d", k + 1);
      WHCHK(check_stable_filter(ctx, k, nd, pq, r2_old));
      if (pq == 0.0) WH_FAIL(ctx, WH_EBREAKDOWN, "CG breakdown: p^T A p = 0 at iteration %d", k + 1);
      rel = std::sqrt(r2 / nb2);
      if (rel <= S.reliable_drop * anchor || rel >= 10.0 * anchor || rel <= tol ||
          k + 1 - last_repl >= 500) {
        discard_ahead();
        applyA(S, false, x, q);
        launch_sub(r, rhs, q, N, S.s);
        dot(S, r, r, S_TMP);
        launch_set_beta(S.slots, S_TMP, r2_old, S.s);
        WHCHK(readback(ctx, S.slots, S_NSLOTS_FIXED));
        r2 = ctx->hbuf[S_TMP];
        rel = std::sqrt(r2 / nb2);
        res.replacements++;
        if (!std::isfinite(rel)) WH_FAIL(ctx, WH_EUNSTABLE, "non-finite true residual");
        stalls = (rel > 0.5 * anchor) ? stalls + 1 : 0;
        last_repl = k + 1;
        if (stalls >= 2 && op32) {
          // the FP32 operator error dominates: continue in FP64 from the true residual
          op32 = false;
          launch_set_beta(S.slots, S_TMP, HUGE_VAL, S.s);   // beta = 0: p = r
        }
        anchor = rel;
        if (rel <= tol) {
          ++k;
          break;
        }
      }
    }
    if (nb_ahead >= 0) {
      pc = pn;   // the look-ahead direction stands
    } else if (nd && S.general) {
      // Algorithm 3: eta = (A W)^T r, mu = (W^T A W)^{-1} eta, p = beta p + r - W mu
      launch_defl_project(S.defl_aw, r, S.partials, S.s);
      launch_defl_reduce_set(S.defl_aw, S.partials, S.slots, S_H, nullptr, S.s);
      launch_small_matvec(S.einv, nd, S.slots, S_H, S_H + nd, 1.0, S.s);
      launch_dcg_update2(S.defl, pc, r, S.slots, S_H + nd, N, S.s);
    } else if (nd && reproject) {
      launch_defl_project(S.defl, r, S.partials, S.s);
      launch_defl_reduce_set(S.defl, S.partials, S.slots, S_H, nullptr, S.s);
      launch_dcg_update2(S.defl, pc, r, S.slots, S_H, N, S.s);
    } else {
      launch_cg_update2(pc, r, S.slots, N, S.s);
    }
    ++k;
    if (!reliable && sync) {
      const double pq = ctx->hbuf[S_PQ];
      r2 = ctx->hbuf[S_R2];
      if (!std::isfinite(pq) || !std::isfinite(r2))
        WH_FAIL(ctx, WH_EUNSTABLE, "non-finite p^T A p or residual at iteration %d", k);
      WHCHK(check_stable_filter(ctx, k - 1, nd, pq, r2_old));
      if (pq == 0.0) WH_FAIL(ctx, WH_EBREAKDOWN, "CG breakdown: p^T A p = 0 at iteration %d", k);
      rel = std::sqrt(r2 / nb2);
      if (stop_on_divergence && rel > 1e3) {
        discard_ahead();
        res.rel = rel;
        res.iters = k;
        res.st = WH_ENOCONV;
        res.diverged = true;
        return WH_OK;
      }
      if (rel <= tol) discard_ahead();
    }
  }
  discard_ahead();
  res.rel = rel;
  res.iters = k;
  res.st = rel <= tol ? WH_OK : WH_ENOCONV;
  return WH_OK;
}

// Restarted GMRES(m), Algorithm 4: classical Gram-Schmidt (second pass when needed) on the device, Givens
// rotations and the triangular solve on the host.  With use_defl the Krylov space is
// augmented by the deflation set W (exact eigenvectors, A W = W diag(mu)): the QR of A W
// is W diag(mu), so W itself heads the basis, the restart vector is (I - W W^T) r, every
// new Arnoldi vector is orthogonalised against W first (h_{W,k} = W^T A v_k, by the
// table kernels), and the least-squares solution splits into the Krylov part y_K (back
// substitution on the rotated rows) and y_W = (W^T r - H_{W,K} y_K) / mu; x += W y_W + V y_K.
wh_status gmres_solve(Solver& S, bool f32, const double* rhs, double* x, bool x_nonzero,
                      double* r, double* basis, int m, double tol, int maxit, KrylovResult& res,
                      bool use_defl = false) {
  wh_ctx* ctx = S.ctx;
  const int64_t N = S.N;
  const int nd = use_defl ? S.defl.nd : 0;
  const int SW = S_H + m + 2;   // slots for the W coefficients
  const int SH2 = SW + nd;      // Gram-Schmidt coefficients (m + 1 slots)
  dot(S, rhs, rhs, S_NB);
  WHCHK(readback(ctx, S.slots, S_NSLOTS_FIXED));
  const double nb = std::sqrt(ctx->hbuf[S_NB]);
  if (!(nb > 0)) {
    res = KrylovResult{};
    return WH_OK;
  }
  std::vector<double> H((size_t)(m + 1) * m, 0.0), g(m + 1), cs(m), sn(m), y(m);
  std::vector<double> gW(nd), HW((size_t)nd * m, 0.0), yW(nd);
  auto Hc = [&](int i, int j) -> double& { return H[(size_t)j * (m + 1) + i]; };
  int its = 0;
  bool first = true;
  double rel = 1.0;
  while (true) {
    if (first && !x_nonzero) {
      launch_copy(r, rhs, N, S.s);
    } else {
      applyA(S, f32, x, basis);  // basis[0] as scratch for A x
      launch_sub(r, rhs, basis, N, S.s);
    }
    first = false;
    if (nd) {
      // g_W = W^T r; r <- (I - W W^T) r
      launch_defl_project(S.defl, r, S.partials, S.s);
      launch_defl_reduce_set(S.defl, S.partials, S.slots, SW, nullptr, S.s);
      launch_defl_combine(S.defl, r, 1.0, nullptr, 0.0, S.slots, SW, N, S.s);
    }
    dot(S, r, r, S_TMP);
    WHCHK(readback(ctx, S.slots, nd ? SW + nd : S_NSLOTS_FIXED));
    double r2 = ctx->hbuf[S_TMP];
    const double beta0 = std::sqrt(r2);
    for (int i = 0; i < nd; ++i) {
      gW[i] = ctx->hbuf[SW + i];
      r2 += gW[i] * gW[i];
    }
    if (!std::isfinite(r2)) WH_FAIL(ctx, WH_EUNSTABLE, "non-finite residual in GMRES");
    rel = std::sqrt(r2) / nb;
    if (rel <= tol || its >= maxit) break;
    std::fill(g.begin(), g.end(), 0.0);
    std::fill(HW.begin(), HW.end(), 0.0);
    g[0] = beta0;
    int kk = 0;
    bool done = false;
    if (beta0 > 0) {
      launch_scale_copy(basis, r, S.slots, S_TMP, N, S.s);
      for (int k = 0; k < m; ++k) {
        double* vk = basis + (size_t)k * N;
        double* w = basis + (size_t)(k + 1) * N;
        applyA(S, f32, vk, w);
        if (nd) {
          // h_{W,k} = W^T w; w <- w - W h_{W,k}
          launch_defl_project(S.defl, w, S.partials, S.s);
          launch_defl_reduce_set(S.defl, S.partials, S.slots, SW, nullptr, S.s);
          launch_defl_combine(S.defl, w, 1.0, nullptr, 0.0, S.slots, SW, N, S.s);
        }
        // classical Gram-Schmidt applied twice (CGS2), three passes over the basis and one
        // read-back per step: h1 = V^T w; w -= V h1 with h2 = V^T w in the same pass;
        // w -= V h2 with ||w||^2.  Column k of H is h1 + h2.  (For this operator the first
        // pass nearly always cancels most of w, so the second is needed anyway.)
        const int nv = k + 1;
        launch_gs_project(basis, N, nv, w, S.partials, S.s);
        launch_defl_reduce(S.partials, kReduceBlocks, nv, S.slots, SH2, nullptr, S.s);
        launch_gs_update(basis, N, nv, S.slots, SH2, w, true, S.partials, S.s);
        // partials [block][nv + 1]: h2, then an intermediate norm that lands in the slot the
        // final norm overwrites
        launch_defl_reduce(S.partials, kReduceBlocks, nv + 1, S.slots, S_H, nullptr, S.s);
        launch_gs_update(basis, N, nv, S.slots, S_H, w, false, S.partials2, S.s);
        launch_reduce(S.partials2, kReduceBlocks, S.slots, S_H + k + 1, 0, S.s);
        WHCHK(readback(ctx, S.slots, SH2 + nv));
        for (int i = 0; i <= k; ++i) Hc(i, k) = ctx->hbuf[SH2 + i] + ctx->hbuf[S_H + i];
        for (int i = 0; i < nd; ++i) HW[(size_t)k * nd + i] = ctx->hbuf[SW + i];
        const double hn2 = ctx->hbuf[S_H + k + 1];
        if (!std::isfinite(hn2)) WH_FAIL(ctx, WH_EUNSTABLE, "non-finite Arnoldi vector");
        {
          // ||A v_k||^2 of the unit vector v_k: at most 1.5^2 for a stable wave solve
          double c2n = hn2;
          for (int i = 0; i <= k; ++i) c2n += Hc(i, k) * Hc(i, k);
          for (int i = 0; i < nd; ++i) c2n += HW[(size_t)k * nd + i] * HW[(size_t)k * nd + i];
          if (c2n > 36.0)
            WH_FAIL(ctx, WH_EUNSTABLE, "|A v| = %.3g |v| exceeds the bound 1.5 of a stable filter: the wave "
                    "solve is unstable (c_max below the largest c, or the time step above the CFL bound)",
                    std::sqrt(c2n));
        }
        Hc(k + 1, k) = std::sqrt(std::max(hn2, 0.0));
        if (Hc(k + 1, k) > 0) launch_scale_copy(w, w, S.slots, S_H + k + 1, N, S.s);
        for (int i = 0; i < k; ++i) {
          const double t = cs[i] * Hc(i, k) + sn[i] * Hc(i + 1, k);
          Hc(i + 1, k) = -sn[i] * Hc(i, k) + cs[i] * Hc(i + 1, k);
          Hc(i, k) = t;
        }
        const double a = Hc(k, k), b = Hc(k + 1, k);
        const double dd = std::hypot(a, b);
        cs[k] = dd == 0 ? 1.0 : a / dd;
        sn[k] = dd == 0 ? 0.0 : b / dd;
        Hc(k, k) = dd;
        Hc(k + 1, k) = 0.0;
        g[k + 1] = -sn[k] * g[k];
        g[k] = cs[k] * g[k];
        ++its;
        kk = k + 1;
        if (std::fabs(g[k + 1]) < tol * nb || its >= maxit) {
          done = true;
          break;
        }
        if (dd == 0.0) WH_FAIL(ctx, WH_EBREAKDOWN, "GMRES breakdown (singular Hessenberg)");
        if (b == 0.0) {  // lucky breakdown: exact solution in the space
          done = true;
          break;
        }
      }
    } else {
      done = true;       // r lies in span W: the W part below is the whole correction
    }
    for (int i = kk - 1; i >= 0; --i) {
      double sacc = g[i];
      for (int j = i + 1; j < kk; ++j) sacc -= Hc(i, j) * y[j];
      y[i] = sacc / Hc(i, i);
    }
    if (kk > 0) {
      WHCHK(upload(ctx, S.slots + S_H, y.data(), kk));
      launch_gemv_acc(x, basis, N, kk, S.slots + S_H, N, S.s);
    }
    if (nd) {
      // y_W = (g_W - H_{W,K} y_K) / mu; x += W y_W (the combine kernel subtracts: store -y_W)
      for (int i = 0; i < nd; ++i) {
        double sacc = gW[i];
        for (int j = 0; j < kk; ++j) sacc -= HW[(size_t)j * nd + i] * y[j];
        yW[i] = -sacc / S.mu[i];
      }
      WHCHK(upload(ctx, S.slots + SW, yW.data(), nd));
      launch_defl_combine(S.defl, x, 1.0, nullptr, 0.0, S.slots, SW, N, S.s);
    }
    if (done && (its >= maxit || nd)) {
      // the true residual decides (with W the W part was solved exactly; check it)
      applyA(S, f32, x, basis);
      launch_sub(r, rhs, basis, N, S.s);
      dot(S, r, r, S_TMP);
      WHCHK(readback(ctx, S.slots, S_NSLOTS_FIXED));
      rel = std::sqrt(ctx->hbuf[S_TMP]) / nb;
      if (rel <= tol || its >= maxit) break;
      x_nonzero = true;
      first = true;
      continue;
    }
  }
  res.rel = rel;
  res.iters = its;
  res.st = rel <= tol ? WH_OK : WH_ENOCONV;
  return WH_OK;
}

// BiCGStab, Algorithm 5.  With use_defl the deflation set W (exact eigenvectors) plays
// the part of the recycled space: the thin QR of A W is W diag(mu), so every A-product
// is projected off W (e = W^T v, v -= W e), the W-coordinates xi gather -W^T r0 and
// alpha e1 + omega e2 per step, and x -= W diag(mu)^{-1} xi recovers the W part at the
// end of a run.  Scalars are formed on the host from FP64 device reductions (three
// read-backs per step).  A run ends on the recursive residual; the true residual
// b - A x then decides, and a further run restarts from it (new shadow residual).
// BiCGStab's residual is not monotone: the iterate with the smallest recursive residual
// is kept, and a run whose residual grows 1e3-fold past that minimum is abandoned for a
// restart from it (after three such restarts the solve stops, res.diverged set, x the
// kept iterate).  work: four vectors (shadow residual, s, t, kept x); r, p, v are the
// caller's.
wh_status bicgstab_solve(Solver& S, bool f32, const double* rhs, double* x, bool x_nonzero,
                         double* r, double* p, double* v, double* work, double tol, int maxit,
                         KrylovResult& res, bool use_defl = false) {
  wh_ctx* ctx = S.ctx;
  const int64_t N = S.N;
  const int nd = use_defl ? S.defl.nd : 0;
  const int SE1 = S_H, SE2 = S_H + nd;   // W-projections of v and t
  double* rt = work;
  double* sv = work + N;
  double* tv = work + 2 * N;
  double* xb = work + 3 * N;   // kept iterate (W part applied)
  dot(S, rhs, rhs, S_NB);
  WHCHK(readback(ctx, S.slots, S_NSLOTS_FIXED));
  const double nb = std::sqrt(ctx->hbuf[S_NB]);
  res = KrylovResult{};
  if (!(nb > 0)) return WH_OK;
  std::vector<double> xi(nd, 0.0), e1(nd, 0.0), cW(nd, 0.0), xib(nd, 0.0);
  bool xib_live = false;   // the kept iterate still lacks its W part (taken inside a run)
  // e = W^T y into slots[dst]; y -= W e
  auto project_off = [&](double* y, int dst) {
    launch_defl_project(S.defl, y, S.partials, S.s);
    launch_defl_reduce_set(S.defl, S.partials, S.slots, dst, nullptr, S.s);
    launch_defl_combine(S.defl, y, 1.0, nullptr, 0.0, S.slots, dst, N, S.s);
  };
  int its = 0, its_at_start = -1, blowups = 0;
  double rel = 1.0, best = HUGE_VAL;
  bool nonzero = x_nonzero;
  while (true) {
    // (re)start from the residual of the current x
    if (nonzero) {
      applyA(S, f32, x, v);
      launch_sub(r, rhs, v, N, S.s);
    } else {
      launch_copy(r, rhs, N, S.s);
    }
    if (nd) project_off(r, SE1);
    launch_copy(rt, r, N, S.s);
    dot(S, r, r, S_R2);
    WHCHK(readback(ctx, S.slots, nd ? SE1 + nd : S_NSLOTS_FIXED));
    for (int i = 0; i < nd; ++i) xi[i] = -ctx->hbuf[SE1 + i];
    double rho = ctx->hbuf[S_R2];   // rt^T r with rt = r
    rel = std::sqrt(rho) / nb;
    if (!std::isfinite(rel)) WH_FAIL(ctx, WH_EUNSTABLE, "non-finite residual in BiCGStab");
    if (rel < best) {          // the run starts from the best iterate so far
      best = rel;
      launch_copy(xb, x, N, S.s);
      xib_live = false;
    }
    if (rel <= tol || its >= maxit || res.diverged) {
      res.rel = rel;
      break;
    }
    if (its == its_at_start) WH_FAIL(ctx, WH_EBREAKDOWN, "BiCGStab breakdown at iteration %d", its);
    its_at_start = its;
    double rho_old = 1.0, alpha = 1.0, om = 1.0;
    bool first = true, blew_up = false;
    while (its < maxit) {
      if (rho == 0.0) break;   // breakdown of the shadow residual: restart
      const bool p_is_r = first;   // p = r = rt, orthogonal to W: rt^T v = r^T A r
      if (first) {
        launch_copy(p, r, N, S.s);
      } else {
        const double beta = (rho / rho_old) * (alpha / om);
        launch_lincomb3(p, 1.0, r, beta, p, -beta * om, v, N, S.s);
      }
      first = false;
      applyA(S, f32, p, v);
      if (nd) project_off(v, SE1);
      dot(S, rt, v, S_TMP);
      WHCHK(readback(ctx, S.slots, nd ? SE1 + nd : S_NSLOTS_FIXED));
      const double rtv = ctx->hbuf[S_TMP];
      for (int i = 0; i < nd; ++i) e1[i] = ctx->hbuf[SE1 + i];
      if (!std::isfinite(rtv)) WH_FAIL(ctx, WH_EUNSTABLE, "non-finite BiCGStab scalar");
      if (p_is_r) WHCHK(check_stable_filter(ctx, 0, 0, rtv, rho));
      if (rtv == 0.0) break;   // restart
      alpha = rho / rtv;
      launch_lincomb3(sv, 1.0, r, -alpha, v, 0.0, nullptr, N, S.s);
      dot(S, sv, sv, S_TMP2);
      WHCHK(readback(ctx, S.slots, S_NSLOTS_FIXED));
      if (std::sqrt(ctx->hbuf[S_TMP2]) <= tol * nb) {
        launch_axpy(x, p, alpha, N, S.s);
        launch_copy(r, sv, N, S.s);
        for (int i = 0; i < nd; ++i) xi[i] += alpha * e1[i];
        ++its;
        rel = std::sqrt(ctx->hbuf[S_TMP2]) / nb;
        break;
      }
      applyA(S, f32, sv, tv);
      if (nd) project_off(tv, SE2);
      dot(S, tv, sv, S_TMP);
      dot(S, tv, tv, S_PQ);
      WHCHK(readback(ctx, S.slots, nd ? SE2 + nd : S_NSLOTS_FIXED));
      const double ts = ctx->hbuf[S_TMP], tt = ctx->hbuf[S_PQ];
      if (!std::isfinite(ts) || !std::isfinite(tt)) WH_FAIL(ctx, WH_EUNSTABLE, "non-finite BiCGStab scalar");
      om = tt > 0 ? ts / tt : 0.0;
      for (int i = 0; i < nd; ++i) xi[i] += alpha * e1[i] + om * ctx->hbuf[SE2 + i];
      launch_lincomb3(x, 1.0, x, alpha, p, om, sv, N, S.s);
      launch_lincomb3(r, 1.0, sv, -om, tv, 0.0, nullptr, N, S.s);
      rho_old = rho;
      ++its;
      dot(S, r, r, S_R2);
      dot(S, rt, r, S_TMP);
      WHCHK(readback(ctx, S.slots, S_NSLOTS_FIXED));
      rel = std::sqrt(ctx->hbuf[S_R2]) / nb;
      rho = ctx->hbuf[S_TMP];
      if (!std::isfinite(rel)) WH_FAIL(ctx, WH_EUNSTABLE, "non-finite residual in BiCGStab");
      if (rel <= tol) break;
      if (rel < best) {
        best = rel;
        launch_copy(xb, x, N, S.s);
        xib = xi;
        xib_live = true;
      } else if (rel > 1e3 * best) {   // abandon the run, restart from the kept iterate
        blew_up = true;
        break;
      }
      if (om == 0.0) break;    // stagnation of the stabilising step: restart
    }
    bool add_w = nd > 0;
    if (blew_up) {
      launch_copy(x, xb, N, S.s);
      add_w = nd > 0 && xib_live;
      xi = xib;
      if (++blowups >= 3) res.diverged = true;
    }
    if (add_w) {
      // x -= W diag(mu)^{-1} xi (the combine kernel subtracts sum_k c_k W_k)
      for (int i = 0; i < nd; ++i) cW[i] = xi[i] / S.mu[i];
      WHCHK(upload(ctx, S.slots + SE1, cW.data(), nd));
      launch_defl_combine(S.defl, x, 1.0, nullptr, 0.0, S.slots, SE1, N, S.s);
    }
    if (blew_up) {
      // the kept iterate is complete now: keep it so for a further blow-up
      launch_copy(xb, x, N, S.s);
      xib_live = false;
    }
    nonzero = true;
    // the next pass through the loop head forms the true residual b - A x and stops there
    // if it meets tol or the iterations are spent; a pass that made no step is a breakdown
  }
  res.iters = its;
  res.rel = rel;
  res.st = rel <= tol ? WH_OK : WH_ENOCONV;
  return WH_OK;
}

// Fixed-point iteration (Algorithm 1): x <- Pi_h(x; f) until ||Pi x - x|| <= tol ||b||.
// deflate_iterates (Algorithm 2 with deflated iterates): after every step
// x <- x - W W^T x; the update norm is then ||(I - W W^T)(Pi x - x)||, computed as
// ||Pi x - x||^2 - ||W^T Pi x||^2 (x itself is deflated).
wh_status fpi_solve(Solver& S, double* x, double tol, int maxit, int check_every,
                    KrylovResult& res, bool deflate_iterates = false) {
  wh_ctx* ctx = S.ctx;
  // ||b||^2 (b = Pi_h(0; f)) is expected in slots[S_NB]
  double nb2 = 0;
  res = KrylovResult{};
  int k = 0;
  double rel = 1.0;
  const int ce = std::max(1, check_every);
  const int nd = deflate_iterates ? S.defl.nd : 0;
  while (k < maxit) {
    int nb = wave_solve(S.op64, x, true, M_LAST_FPI, x, x, S.s);
    S.ws64++;
    launch_reduce(S.partials, nb, S.slots, S_TMP, 0, S.s);
    if (nd) {
      // (S.partials is free again: the update-norm partials were reduced above)
      launch_defl_project(S.defl, x, S.partials, S.s);
      launch_defl_reduce_set(S.defl, S.partials, S.slots, S_H, nullptr, S.s);
      launch_defl_combine(S.defl, x, 1.0, nullptr, 0.0, S.slots, S_H, S.N, S.s);
    }
    ++k;
    if (k % ce == 0 || k == maxit) {
      WHCHK(readback(ctx, S.slots, S_NSLOTS_FIXED + nd));
      nb2 = ctx->hbuf[S_NB];
      double d2 = ctx->hbuf[S_TMP];
      for (int j = 0; j < nd; ++j) d2 -= ctx->hbuf[S_H + j] * ctx->hbuf[S_H + j];
      rel = nb2 > 0 ? std::sqrt(std::max(d2, 0.0) / nb2) : 0.0;
      if (!std::isfinite(rel)) WH_FAIL(ctx, WH_EUNSTABLE, "non-finite FPI update");
      if (rel <= tol) break;
    }
  }
  res.rel = rel;
  res.iters = k;
  res.st = rel <= tol ? WH_OK : WH_ENOCONV;
  return WH_OK;
}

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// Steps per launch of a fourth-order solve: the row-marching launches take 2 or 4 (2D only);
// 0 asks for 4, 1 keeps one step per launch, other values take the largest supported below.
int order4_k(int dim, int k_fuse) {
  if (dim != 2 || k_fuse == 1) return 1;
  if (k_fuse == 0 || k_fuse >= 4) return 4;
  return k_fuse >= 2 ? 2 : 1;
}

// Common setup for wh_apply_filter / wh_solve: c_max, time parameters, coefficient
// arrays in the stepping precisions.
wh_status setup_ops(wh_ctx* ctx, const wh_grid& g, const wh_params& P, const double* c2,
                    const double* f, void* ws, const Layout& L, TimeParams& tp, Solver& S,
                    bool may_tune = true) {
  hipStream_t s = ctx->stream;
  const bool varc = c2 != nullptr;
  const bool mixed = P.precision == WH_MIXED;
  double c_max = P.c_max;
  if (c_max == 0) {
    if (varc) {
      double* part = at<double>(ws, L.partials2);
      double* slots = at<double>(ws, L.slots);
      launch_max_partials(c2, L.N, part, false, s);
      launch_max_finalize(part, kReduceBlocks, slots + S_TMP2, s);
      launch_max_partials(c2, L.N, part, true, s);
      launch_max_finalize(part, kReduceBlocks, slots + S_TMP, s);
      WHCHK(readback(ctx, slots, S_NSLOTS_FIXED));
      const double m = ctx->hbuf[S_TMP2];
      const double negmin = ctx->hbuf[S_TMP];
      if (!(m > 0) || !std::isfinite(m) || !(negmin < 0))
        WH_FAIL(ctx, WH_EINVAL, "c2 must be positive and finite at every node");
      c_max = std::sqrt(m);
    } else {
      c_max = 1.0;
    }
  }
  if (g.order == 4 && varc)
    WH_FAIL(ctx, WH_EUNSUPPORTED, "fourth-order differences are built for c == 1 (c2 == NULL)");
  WHCHK(make_time_params(ctx, g.dim, g.n, P, c_max, tp, g.order));
  const double h = 1.0 / g.n;
  const double dt2 = tp.dt * tp.dt;
  const double ks = dt2 / (2.0 * h * h);
  launch_prep_coeffs(c2, f, at<void>(ws, L.kap64), at<void>(ws, L.fs64), false, ks, dt2, L.N, g.n,
                     g.dim, s);
  if (mixed)
    launch_prep_coeffs(c2, f, at<void>(ws, L.kap32), at<void>(ws, L.fs32), true, ks, dt2, L.N, g.n,
                       g.dim, s);
  S.ctx = ctx;
  S.s = s;
  S.N = L.N;
  S.slots = at<double>(ws, L.slots);
  S.partials = at<double>(ws, L.partials);
  S.partials2 = at<double>(ws, L.partials2);
  WaveOp base;
  base.dim = g.dim;
  base.n = g.n;
  base.varc = varc;
  base.Wa = at<void>(ws, L.Wa);
  base.Wb = at<void>(ws, L.Wb);
  base.Wc = at<void>(ws, L.Wc);
  base.Wd = at<void>(ws, L.Wd);
  base.k_fuse = 1;
  base.order = g.order;
  base.V = at<double>(ws, L.V);
  base.a = dt2 / (h * h);
  base.tp = &tp;
  base.partials = S.partials;
  S.op64 = base;
  S.op64.f32 = false;
  S.op64.kap = at<void>(ws, L.kap64);
  S.op64.fs = at<void>(ws, L.fs64);
  // (omega_fp dt)^2 with omega_fp the frequency the fixed point solves for:
  // (2/dt) sin(omega_w dt / 2) (= omega under the corrected frequency)
  S.om2dt2 = 4.0 * std::sin(0.5 * tp.omega_w * tp.dt) * std::sin(0.5 * tp.omega_w * tp.dt);
  // defect form by default for CG/GMRES; DCG has removed the near-resonant modes, where
  // the defect form gains, so it steps W directly (one stencil pass less per iteration)
  S.defect = (P.mixed_form == 0 || (P.mixed_form < 0 && P.solver != WH_DCG)) && g.order == 2;
  // exact deflation removes the near-resonant modes whose FP32 error would slow CG, so
  // DCG can go longer between FP64 residual replacements
  S.reliable_drop = (P.inner_tol > 0 && P.inner_tol < 1) ? P.inner_tol : (P.solver == WH_DCG ? 1e-3 : 0.1);
  S.op32 = base;
  S.op32.f32 = true;
  if (mixed) {
    S.op32.kap = at<void>(ws, L.kap32);
    S.op32.fs = at<void>(ws, L.fs32);
  }
  // steps per launch: fixed by the caller, else autotuned (cached per context).  The
  // operator without forcing dominates every solve, so it sets K for both precisions.
  auto pick = [&](WaveOp& op) {
    int code = 1;
    if (g.order == 4) code = order4_k(g.dim, P.k_fuse);
    else if (P.k_fuse == 1 || (P.k_fuse > 1 && !fused_supported(g.dim, op.f32, P.k_fuse))) code = 1;
    else if (P.k_fuse > 1 && P.k_shape >= 0) code = P.k_fuse | (P.k_shape << 8);
    else if (may_tune) code = autotune_k(ctx, op, false, P.k_fuse);
    else code = untuned_k(ctx, op, P.k_fuse);
    op.k_fuse = code & 0xff;
    op.k_shape = code >> 8;
  };
  pick(S.op64);
  if (mixed) pick(S.op32);
  HIPCHK(ctx, hipGetLastError());
  return WH_OK;
}

// Inverse of a small dense matrix (row-major, n x n) by Gauss-Jordan elimination with partial
// pivoting; false if a pivot vanishes.
bool invert_small(std::vector<double> a, int n, std::vector<double>& inv) {
  inv.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(a[(size_t)r * n + c]) > std::fabs(a[(size_t)piv * n + c])) piv = r;
    const double pv = a[(size_t)piv * n + c];
    if (!(std::fabs(pv) > 0) || !std::isfinite(pv)) return false;
    if (piv != c)
      for (int j = 0; j < n; ++j) {
        std::swap(a[(size_t)piv * n + j], a[(size_t)c * n + j]);
        std::swap(inv[(size_t)piv * n + j], inv[(size_t)c * n + j]);
      }
    const double d = 1.0 / pv;
    for (int j = 0; j < n; ++j) {
      a[(size_t)c * n + j] *= d;
      inv[(size_t)c * n + j] *= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double m = a[(size_t)r * n + c];
      if (m == 0.0) continue;
      for (int j = 0; j < n; ++j) {
        a[(size_t)r * n + j] -= m * a[(size_t)c * n + j];
        inv[(size_t)r * n + j] -= m * inv[(size_t)c * n + j];
      }
    }
  }
  return true;
}

// Algorithm 3 with any l2-orthonormal deflation vectors W (not eigenvectors): A W by n_d FP64
// wave solves (the start-up cost of Section 5.1), E = W^T A W by projections, and E^{-1} formed
// on the host (E symmetrised, A being symmetric) for the per-iteration mu = E^{-1} (A W)^T r.
wh_status setup_general_deflation(Solver& S, void* ws, const Layout& L, const double* V, int64_t ldv, int nd) {
  wh_ctx* ctx = S.ctx;
  hipStream_t s = S.s;
  const int64_t N = S.N;
  double* aw = at<double>(ws, L.aw);
  for (int k = 0; k < nd; ++k) applyA(S, false, V + (size_t)k * ldv, aw + (size_t)k * N);
  double* E = at<double>(ws, L.einv);   // E first, then its inverse
  for (int k = 0; k < nd; ++k) {
    launch_defl_project(S.defl, aw + (size_t)k * N, S.partials, s);
    launch_defl_reduce(S.partials, defl_partial_blocks(S.defl), nd, E, k * nd, nullptr, s);  // E[k][i] = w_i^T A w_k
  }
  std::vector<double> eh((size_t)nd * nd), es((size_t)nd * nd), inv;
  HIPCHK(ctx, hipMemcpyAsync(eh.data(), E, 8 * eh.size(), hipMemcpyDeviceToHost, s));
  HIPCHK(ctx, hipStreamSynchronize(s));
  for (int i = 0; i < nd; ++i)
    for (int j = 0; j < nd; ++j) es[(size_t)i * nd + j] = 0.5 * (eh[(size_t)i * nd + j] + eh[(size_t)j * nd + i]);
  if (!invert_small(es, nd, inv)) WH_FAIL(ctx, WH_EBREAKDOWN, "W^T A W is singular");
  HIPCHK(ctx, hipMemcpyAsync(E, inv.data(), 8 * inv.size(), hipMemcpyHostToDevice, s));
  HIPCHK(ctx, hipStreamSynchronize(s));
  S.general = true;
  S.defl_aw.kind = WH_DEFL_DENSE;
  S.defl_aw.nd = nd;
  S.defl_aw.dim = S.defl.dim;
  S.defl_aw.n = S.defl.n;
  S.defl_aw.V = aw;
  S.defl_aw.ldv = N;
  S.einv = E;
  return WH_OK;
}

void fill_info(wh_info* info, const TimeParams& tp, int k_fuse, const WaveOp* op = nullptr) {
  if (!info) return;
  info->nt = tp.nt;
  info->m = tp.m;
  info->dt = tp.dt;
  info->omega_tilde = tp.omega_w;
  info->c_max = tp.c_max;
  info->k_fuse = k_fuse;
  info->k_rows = info->k_waves = 0;
  if (op && k_fuse > 1 && op->order == 4) {
    info->k_rows = 32;
    info->k_waves = 4;
  } else if (op && k_fuse > 1) {
    fused_shape_dims(op->dim, op->f32, k_fuse, op->k_shape, &info->k_rows, &info->k_waves);
  }
}

}  // namespace

// =================================================================== C ABI
// Message of the last failure on this thread of a call with no context to hold it
// (wh_create, the host helpers, workspace sizing).
namespace {
thread_local std::string g_create_err;

// Fixed device scratch of wh_apply_filter_noalloc (one copy per GPU, held until the process
// ends).  Host code never uses the name itself: wh_create looks up its device address once
// per device (with that device current) and every use goes through that address.
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
void* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;
}  // namespace

namespace wh {
void set_thread_error(const char* msg) { g_create_err = msg ? msg : ""; }
}  // namespace wh

extern "C" {

void wh_params_default(wh_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->omega = 1.0;
  p->n_periods = 1;
  p->cfl = 0.5;
  p->steps_per_period = 0;
  p->freq_correction = 1;
  p->c_max = 0.0;
  p->precision = WH_F64;
  p->solver = WH_CG;
  p->restart = 40;
  p->tol = 1e-8;
  p->max_iters = 10000;
  p->inner_tol = 0.0;
  p->max_outer = 30;
  p->k_fuse = 0;
  p->reproject = -1;
  p->check_every = 1;
  p->mixed_form = -1;
  p->devd = 0;
  p->k_shape = -1;
}

const char* wh_status_string(wh_status s) {
  switch (s) {
    case WH_OK: return "ok";
    case WH_ENOCONV: return "tolerance not reached";
    case WH_EINVAL: return "invalid argument";
    case WH_EUNSUPPORTED: return "unsupported";
    case WH_EHIP: return "HIP runtime error";
    case WH_EWORKSPACE: return "workspace missing or too small";
    case WH_EUNSTABLE: return "unstable wave solve";
    case WH_EBREAKDOWN: return "Krylov breakdown";
    case WH_EHOST: return "host-side failure inside the library";
  }
  return "unknown status";
}


wh_status wh_create(wh_ctx** out, int device, void* stream) {
  return guard(nullptr, [&]() -> wh_status {
  if (!out) return WH_EINVAL;
  *out = nullptr;
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || device < 0 || device >= count) {
    g_create_err = std::string("no such device (hipGetDeviceCount: ") + hipGetErrorString(e) + ")";
    return WH_EHIP;
  }
  e = hipSetDevice(device);
  if (e != hipSuccess) {
    g_create_err = std::string("hipSetDevice: ") + hipGetErrorString(e);
    return WH_EHIP;
  }
  if (device >= kMaxDevices) {
    g_create_err = "device index too large";
    return WH_EINVAL;
  }
  {
    // address of this device's copy of the no-allocation scratch array
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
      void* ptr = nullptr;
      e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !ptr) {
        g_create_err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
        return WH_EHIP;
      }
      g_scratch_ptr[device] = ptr;
    }
  }
  wh_ctx* c = new wh_ctx();
  c->device = device;
  c->stream = (hipStream_t)stream;
  e = hipHostMalloc((void**)&c->hbuf, sizeof(double) * kHostScalars, hipHostMallocDefault);
  if (e != hipSuccess) {
    g_create_err = std::string("hipHostMalloc: ") + hipGetErrorString(e);
    delete c;
    return WH_EHIP;
  }
  c->hbuf_len = kHostScalars;
  e = hipEventCreateWithFlags(&c->rb_event, hipEventDisableTiming);
  if (e != hipSuccess) {
    g_create_err = std::string("hipEventCreateWithFlags: ") + hipGetErrorString(e);
    (void)hipHostFree(c->hbuf);
    delete c;
    return WH_EHIP;
  }
  e = hipMalloc((void**)&c->dred, sizeof(double) * (kReduceBlocks + 8));
  if (e != hipSuccess) {
    g_create_err = std::string("hipMalloc: ") + hipGetErrorString(e);
    (void)hipEventDestroy(c->rb_event);
    (void)hipHostFree(c->hbuf);
    delete c;
    return WH_EHIP;
  }
  *out = c;
  return WH_OK;
  });
}

wh_status wh_destroy(wh_ctx* ctx) {
  if (!ctx) return WH_EINVAL;
  if (ctx->rb_event) (void)hipEventDestroy(ctx->rb_event);
  if (ctx->hbuf) (void)hipHostFree(ctx->hbuf);
  if (ctx->dred) (void)hipFree(ctx->dred);
  delete ctx;
  return WH_OK;
}

wh_status wh_set_stream(wh_ctx* ctx, void* stream) {
  if (!ctx) return WH_EINVAL;
  ctx->stream = (hipStream_t)stream;
  return WH_OK;
}

wh_status wh_coeff_bound(wh_ctx* ctx, const wh_grid* grid, const double* c2, double* c_max) {
  return guard(ctx, [&]() -> wh_status {
  if (!ctx) return WH_EINVAL;
  if (!grid || !c_max) WH_FAIL(ctx, WH_EINVAL, "NULL argument");
  WHCHK(check_grid(ctx, grid));
  *c_max = 0;
  if (!c2) {
    *c_max = 1.0;
    return WH_OK;
  }
  HIPCHK(ctx, hipSetDevice(ctx->device));
  const int64_t N = nodal_count(grid->dim, grid->n);
  double* part = ctx->dred;
  double* res = ctx->dred + kReduceBlocks;
  launch_max_partials(c2, N, part, false, ctx->stream);
  launch_max_finalize(part, kReduceBlocks, res, ctx->stream);
  launch_max_partials(c2, N, part, true, ctx->stream);
  launch_max_finalize(part, kReduceBlocks, res + 1, ctx->stream);
  WHCHK(readback(ctx, res, 2));
  const double m = ctx->hbuf[0], negmin = ctx->hbuf[1];
  if (!(m > 0) || !std::isfinite(m) || !(negmin < 0))
    WH_FAIL(ctx, WH_EINVAL, "c2 must be positive and finite at every node");
  *c_max = std::sqrt(m);
  return WH_OK;
  });
}

const char* wh_last_error(const wh_ctx* ctx) { return ctx ? ctx->err.c_str() : g_create_err.c_str(); }

wh_status wh_time_params(const wh_grid* grid, const wh_params* params, double c_max, int32_t* m,
                         int32_t* nt, double* dt, double* omega_tilde) {
  return guard(nullptr, [&]() -> wh_status {
  WHCHK(check_grid(nullptr, grid));
  WHCHK(check_params(nullptr, grid, params));
  TimeParams tp;
  WHCHK(make_time_params(nullptr, grid->dim, grid->n, *params, c_max > 0 ? c_max : 1.0, tp, grid->order));
  if (m) *m = tp.m;
  if (nt) *nt = tp.nt;
  if (dt) *dt = tp.dt;
  if (omega_tilde) *omega_tilde = tp.omega_w;
  return WH_OK;
  });
}

wh_status wh_transfer(const wh_grid* grid, const wh_params* params, double c_max, int32_t count,
                      const double* lambda2, double* beta) {
  return guard(nullptr, [&]() -> wh_status {
  WHCHK(check_grid(nullptr, grid));
  WHCHK(check_params(nullptr, grid, params));
  if (count < 0 || (count > 0 && (!lambda2 || !beta))) return WH_EINVAL;
  TimeParams tp;
  WHCHK(make_time_params(nullptr, grid->dim, grid->n, *params, c_max > 0 ? c_max : 1.0, tp, grid->order));
  for (int i = 0; i < count; ++i) beta[i] = transfer(tp, lambda2[i]);
  return WH_OK;
  });
}

wh_status wh_select_sine_modes(int32_t dim, int32_t n, int32_t order, double omega, int32_t n_d,
                               int32_t* modes, double* lambda2) {
  return guard(nullptr, [&]() -> wh_status {
  if ((dim != 2 && dim != 3) || n < 4 || n_d < 0 || !(omega > 0) || (n_d > 0 && !modes) ||
      (order != 2 && order != 4))
    return WH_EINVAL;
  const int K = n - 1;
  if ((int64_t)K * K * (dim == 3 ? K : 1) < n_d) return WH_EINVAL;
  std::vector<double> e(n);   // e[k] = lambda_k^2 of the 1D Dirichlet operator, increasing in k
  for (int k = 1; k < n; ++k) e[k] = lam2_1d(k, n, order);
  const double om2 = omega * omega;
  // The n_d modes with the smallest |lambda^2 - omega^2|, the distance taken on a grid of
  // 1e-9 omega^2 so that modes whose lambda^2 agree up to rounding (degenerate sets
  // summed in different orders) tie; ties in lexicographic order of the mode numbers.
  // For fixed leading mode numbers the distance grows monotonically
  // as the last mode number moves away from the crossing point of omega^2, so each
  // leading tuple gives two sorted streams (downwards and upwards from the crossing);
  // a heap merges the streams in (distance, mode numbers) order.
  struct Item {
    double dist;
    int k[3];
    int dir;  // -1: last mode number decreasing, +1: increasing
  };
  auto later = [&](const Item& a, const Item& b) {   // heap order: smallest key on top
    if (a.dist != b.dist) return a.dist > b.dist;
    for (int t = 0; t < dim; ++t)
      if (a.k[t] != b.k[t]) return a.k[t] > b.k[t];
    return false;
  };
  const double quantum = 1e-9 * om2;
  auto dist_of = [&](const int* k) {
    double l2 = e[k[0]] + e[k[1]];
    if (dim == 3) l2 += e[k[2]];
    return std::floor(std::fabs(l2 - om2) / quantum + 0.5);
  };
  std::vector<Item> heap;
  auto push_streams = [&](int a, int b) {   // leading mode numbers (a) or (a, b)
    double lead = e[a] + (dim == 3 ? e[b] : 0.0);
    const double t = om2 - lead;
    // first last-mode number with e >= t
    const int j = (int)(std::lower_bound(e.begin() + 1, e.end(), t) - e.begin());
    const int last = dim - 1;
    if (j - 1 >= 1) {
      Item it{};
      it.k[0] = a;
      if (dim == 3) it.k[1] = b;
      it.k[last] = j - 1;
      it.dir = -1;
      it.dist = dist_of(it.k);
      heap.push_back(it);
      std::push_heap(heap.begin(), heap.end(), later);
    }
    if (j <= K) {
      Item it{};
      it.k[0] = a;
      if (dim == 3) it.k[1] = b;
      it.k[last] = j;
      it.dir = 1;
      it.dist = dist_of(it.k);
      heap.push_back(it);
      std::push_heap(heap.begin(), heap.end(), later);
    }
  };
  if (dim == 2) {
    for (int a = 1; a <= K; ++a) push_streams(a, 0);
  } else {
    for (int a = 1; a <= K; ++a)
      for (int b = 1; b <= K; ++b) push_streams(a, b);
  }
  const int last = dim - 1;
  for (int i = 0; i < n_d; ++i) {
    std::pop_heap(heap.begin(), heap.end(), later);
    Item it = heap.back();
    heap.pop_back();
    for (int a = 0; a < dim; ++a) modes[i * dim + a] = it.k[a];
    if (lambda2) {
      double l2 = e[it.k[0]] + e[it.k[1]];
      if (dim == 3) l2 += e[it.k[2]];
      lambda2[i] = l2;
    }
    const int nxt = it.k[last] + it.dir;
    if (nxt >= 1 && nxt <= K) {
      it.k[last] = nxt;
      it.dist = dist_of(it.k);
      heap.push_back(it);
      std::push_heap(heap.begin(), heap.end(), later);
    }
  }
  return WH_OK;
  });
}

size_t wh_workspace_bytes(const wh_grid* grid, const wh_params* params, const wh_deflation* defl) {
  return guard_size([&]() -> size_t {
  if (!grid || !params || check_grid(nullptr, grid) != WH_OK) return 0;
  return make_layout(*grid, *params, defl).total;
  });
}

wh_status wh_apply_filter(wh_ctx* ctx, const wh_grid* grid, const double* c2, const double* f,
                          const double* v_in, double* v_out, const wh_params* params, void* ws,
                          size_t ws_bytes, wh_info* info) {
  return guard(ctx, [&]() -> wh_status {
  if (!ctx) return WH_EINVAL;
  const double t0 = now_ms();
  WHCHK(check_grid(ctx, grid));
  WHCHK(check_params(ctx, grid, params));
  if (!v_in || !v_out) WH_FAIL(ctx, WH_EINVAL, "v_in / v_out is NULL");
  const Layout L = make_layout(*grid, *params, nullptr);
  WHCHK(check_ws(ctx, ws, ws_bytes, L.total));
  HIPCHK(ctx, hipSetDevice(ctx->device));
  TimeParams tp;
  Solver S{};
  WHCHK(setup_ops(ctx, *grid, *params, c2, f, ws, L, tp, S));
  WaveOp op = params->precision == WH_MIXED ? S.op32 : S.op64;
  op.V = v_out;  // accumulate straight into the output
  wave_solve(op, v_in, f != nullptr, M_LAST_V, nullptr, nullptr, ctx->stream);
  HIPCHK(ctx, hipGetLastError());
  if (info) {
    std::memset(info, 0, sizeof(*info));
    fill_info(info, tp, params->precision == WH_MIXED ? S.op32.k_fuse : S.op64.k_fuse,
              params->precision == WH_MIXED ? &S.op32 : &S.op64);
    info->wave_solves = params->precision == WH_MIXED ? 0 : 1;
    info->wave_solves_f32 = params->precision == WH_MIXED ? 1 : 0;
    info->ms = now_ms() - t0;
  }
  return WH_OK;
  });
}

wh_status wh_apply_filter_noalloc(wh_ctx* ctx, const wh_grid* grid, const double* c2, const double* f,
                                  const double* v_in, double* v_out, const wh_params* params,
                                  wh_info* info) {
  return guard(ctx, [&]() -> wh_status {
  if (!ctx) return WH_EINVAL;
  const double t0 = now_ms();
  WHCHK(check_grid(ctx, grid));
  WHCHK(check_params(ctx, grid, params));
  if (!v_in || !v_out) WH_FAIL(ctx, WH_EINVAL, "v_in / v_out is NULL");
  if (v_in == v_out) WH_FAIL(ctx, WH_EINVAL, "v_in and v_out must not overlap");
  const Layout L = make_filter_layout(*grid, *params);
  if (L.total > kScratchBytes)
    WH_FAIL(ctx, WH_EWORKSPACE,
            "grid too large for the fixed scratch of wh_apply_filter_noalloc: needs %zu bytes, "
            "the scratch holds %zu (use wh_apply_filter with a workspace)", L.total, kScratchBytes);
  void* ws = g_scratch_ptr[ctx->device];
  if (!ws) WH_FAIL(ctx, WH_EHIP, "no scratch address for device %d", ctx->device);
  HIPCHK(ctx, hipSetDevice(ctx->device));
  TimeParams tp;
  Solver S{};
  WHCHK(setup_ops(ctx, *grid, *params, c2, f, ws, L, tp, S, false));
  WaveOp op = params->precision == WH_MIXED ? S.op32 : S.op64;
  op.V = v_out;
  wave_solve(op, v_in, f != nullptr, M_LAST_V, nullptr, nullptr, ctx->stream);
  HIPCHK(ctx, hipGetLastError());
  if (info) {
    std::memset(info, 0, sizeof(*info));
    fill_info(info, tp, op.k_fuse, &op);
    info->wave_solves = params->precision == WH_MIXED ? 0 : 1;
    info->wave_solves_f32 = params->precision == WH_MIXED ? 1 : 0;
    info->ms = now_ms() - t0;
  }
  return WH_OK;
  });
}

wh_status wh_solve(wh_ctx* ctx, const wh_grid* grid, const double* c2, const double* f,
                   const wh_deflation* defl, const wh_params* params, double* u, void* ws,
                   size_t ws_bytes, wh_info* info) {
  return guard(ctx, [&]() -> wh_status {
  if (!ctx) return WH_EINVAL;
  const double t0 = now_ms();
  if (info) std::memset(info, 0, sizeof(*info));
  WHCHK(check_grid(ctx, grid));
  WHCHK(check_params(ctx, grid, params));
  if (!f || !u) WH_FAIL(ctx, WH_EINVAL, "f / u is NULL");
  const wh_params& P = *params;
  if (P.solver < WH_FPI || P.solver > WH_BICGSTAB) WH_FAIL(ctx, WH_EINVAL, "bad solver");
  if (!(P.tol > 0)) WH_FAIL(ctx, WH_EINVAL, "tol must be > 0");
  if (P.max_iters < 0) WH_FAIL(ctx, WH_EINVAL, "max_iters must be >= 0");
  if (P.solver == WH_GMRES && (P.restart < 1 || P.restart > 1000))
    WH_FAIL(ctx, WH_EINVAL, "restart must be in [1, 1000]");
  WHCHK(check_defl(ctx, grid, defl, c2 != nullptr));
  const int nd = defl_n(defl);
  if (P.solver == WH_DCG && nd == 0) WH_FAIL(ctx, WH_EINVAL, "DCG needs a deflation set");
  if (P.devd < 0 || P.devd > 2) WH_FAIL(ctx, WH_EINVAL, "devd must be 0, 1 or 2");
  const bool devd = P.devd > 0;
  if (devd && (nd == 0 || P.solver == WH_DCG))
    WH_FAIL(ctx, WH_EINVAL, "devd needs a deflation set and solver FPI, CG, GMRES or BiCGStab");
  if (P.devd == 2 && P.solver != WH_FPI) WH_FAIL(ctx, WH_EINVAL, "devd = 2 (deflated iterates) is for FPI");
  if (!devd && (P.solver == WH_FPI || P.solver == WH_CG) && nd > 0)
    WH_FAIL(ctx, WH_EUNSUPPORTED, "a deflation set is used by DCG, augmented GMRES / BiCGStab or devd");
  if (nd > 0 && defl->kind == WH_DEFL_DENSE && P.solver != WH_DCG)
    WH_FAIL(ctx, WH_EUNSUPPORTED, "general deflation vectors (WH_DEFL_DENSE) are used by DCG");
  // GMRES / BiCGStab with a deflation set (and no devd) are the augmented methods of
  // Algorithms 4 and 5
  const bool agmres = (P.solver == WH_GMRES || P.solver == WH_BICGSTAB) && nd > 0 && !devd;
  const bool outer_refined = P.solver == WH_GMRES || P.solver == WH_BICGSTAB;
  const bool mixed = P.precision == WH_MIXED;
  if (mixed && P.solver == WH_FPI) WH_FAIL(ctx, WH_EUNSUPPORTED, "FPI runs in FP64 only");
  const Layout L = make_layout(*grid, P, defl);
  WHCHK(check_ws(ctx, ws, ws_bytes, L.total));
  HIPCHK(ctx, hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  TimeParams tp;
  Solver S{};
  WHCHK(setup_ops(ctx, *grid, P, c2, f, ws, L, tp, S));
  const int64_t N = L.N;
  launch_zero_boundary(u, grid->n, grid->dim, s);
  double* b = at<double>(ws, L.b);
  double* r = at<double>(ws, L.r);
  double* p = at<double>(ws, L.p);
  double* q = at<double>(ws, L.q);
  HIPCHK(ctx, hipMemsetAsync(r, 0, 8 * N, s));
  HIPCHK(ctx, hipMemsetAsync(p, 0, 8 * N, s));
  HIPCHK(ctx, hipMemsetAsync(q, 0, 8 * N, s));
  if (L.has_p2) {
    S.p2 = at<double>(ws, L.p2);
    HIPCHK(ctx, hipMemsetAsync(S.p2, 0, 8 * N, s));
  }
  HIPCHK(ctx, hipMemsetAsync(S.slots, 0, 8 * (size_t)L.nslots, s));
  // the stencil epilogues write interior nodes only: Krylov vectors keep a zero boundary
  if (P.solver == WH_GMRES)
    HIPCHK(ctx, hipMemsetAsync(at<double>(ws, L.basis), 0, 8 * (size_t)N * (std::max(1, P.restart) + 1), s));
  if (P.solver == WH_BICGSTAB) HIPCHK(ctx, hipMemsetAsync(at<double>(ws, L.basis), 0, 8 * (size_t)N * 4, s));
  if (mixed) {
    HIPCHK(ctx, hipMemsetAsync(at<double>(ws, L.ro), 0, 8 * N, s));
    HIPCHK(ctx, hipMemsetAsync(at<double>(ws, L.d), 0, 8 * N, s));
  }
  // deflation set
  // Algorithm 3 may skip the per-iteration A-orthogonalisation with exact eigenvectors;
  // every deflation kind built here is exact (for the FP64 operator), so auto = off.
  bool reproject = P.reproject == 1;
  if (nd) {
    S.defl.kind = defl->kind;
    S.defl.nd = nd;
    S.defl.dim = grid->dim;
    S.defl.n = grid->n;
    std::vector<double> lam2(nd);
    if (defl->kind == WH_DEFL_SINE) {
      for (int k = 0; k < nd; ++k) {
        double l2 = 0;
        for (int a = 0; a < grid->dim; ++a) l2 += lam2_1d(defl->modes[k * grid->dim + a], grid->n, grid->order);
        lam2[k] = l2;
      }
      // mode numbers to the device (through the pinned block as doubles -> ints)
      std::vector<int32_t> md(defl->modes, defl->modes + nd * grid->dim);
      HIPCHK(ctx, hipStreamSynchronize(s));
      std::memcpy(ctx->hbuf, md.data(), md.size() * sizeof(int32_t));
      HIPCHK(ctx, hipMemcpyAsync(at<int32_t>(ws, L.modes), ctx->hbuf, md.size() * sizeof(int32_t),
                                 hipMemcpyHostToDevice, s));
      HIPCHK(ctx, hipStreamSynchronize(s));
      launch_sine_tables(at<double>(ws, L.tab), at<int32_t>(ws, L.modes), nd, grid->dim, grid->n, s);
      S.defl.tab = at<double>(ws, L.tab);
    } else if (defl->kind == WH_DEFL_FACTORED) {
      for (int k = 0; k < nd; ++k) lam2[k] = defl->lambda2[k];
      // table [t][axis][i]: x-factor then y-factor of every term
      const int T = defl->n_terms;
      const size_t P1 = (size_t)grid->n + 1;
      double* tab = at<double>(ws, L.tab);
      HIPCHK(ctx, hipMemcpy2DAsync(tab, 2 * P1 * 8, defl->fx, P1 * 8, P1 * 8, T, hipMemcpyDeviceToDevice, s));
      HIPCHK(ctx, hipMemcpy2DAsync(tab + P1, 2 * P1 * 8, defl->fy, P1 * 8, P1 * 8, T, hipMemcpyDeviceToDevice, s));
      std::vector<int32_t> mp(T + nd + 1);
      for (int t = 0; t < T; ++t) mp[t] = defl->term_mode[t];
      for (int k = 0, t = 0; k <= nd; ++k) {
        while (t < T && defl->term_mode[t] < k) ++t;
        mp[T + k] = t;
      }
      HIPCHK(ctx, hipStreamSynchronize(s));
      std::memcpy(ctx->hbuf, mp.data(), mp.size() * sizeof(int32_t));
      int32_t* mdev = at<int32_t>(ws, L.modes);
      HIPCHK(ctx, hipMemcpyAsync(mdev, ctx->hbuf, mp.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
      HIPCHK(ctx, hipStreamSynchronize(s));
      S.defl.tab = tab;
      S.defl.nt = T;
      S.defl.tmap = mdev;
      S.defl.toff = mdev + T;
      S.defl.tsum = at<double>(ws, L.tsum);
      S.defl.tcoef = at<double>(ws, L.tsum) + T;
    } else if (defl->kind == WH_DEFL_DENSE) {
      S.defl.V = defl->V;
      S.defl.ldv = defl->ldv;
      WHCHK(setup_general_deflation(S, ws, L, defl->V, defl->ldv, nd));
    } else {
      for (int k = 0; k < nd; ++k) lam2[k] = defl->lambda2[k];
      S.defl.V = defl->V;
      S.defl.ldv = defl->ldv;
    }
    std::vector<double> inv(nd), neg(nd);
    S.mu.assign(nd, 0.0);
    for (int k = 0; k < nd && !S.general; ++k) {
      const double mu = 1.0 - transfer(tp, lam2[k]);
      S.mu[k] = mu;
      if (mu == 0.0) WH_FAIL(ctx, WH_EBREAKDOWN, "deflation vector %d is at resonance (mu = 0)", k);
      inv[k] = 1.0 / mu;
      neg[k] = -1.0 / mu;
    }
    if (!S.general) {
      WHCHK(upload(ctx, at<double>(ws, L.invmu), inv.data(), nd));
      WHCHK(upload(ctx, at<double>(ws, L.ones), neg.data(), nd));
      S.invmu = at<double>(ws, L.invmu);
      S.negmu = at<double>(ws, L.ones);
    }
    if (devd) {
      // Algorithm 2: f_d = f - W W^T f (into r, then the forcing arrays are rebuilt from it);
      // ones <- -(phi_k^T f) / (omega_fp^2 - lambda_k^2), added to the solution at the end
      const double sh = std::sin(0.5 * tp.omega_w * tp.dt);
      const double om2 = 4.0 * sh * sh / (tp.dt * tp.dt);
      std::vector<double> sc(nd);
      for (int k = 0; k < nd; ++k) {
        const double den = om2 - lam2[k];
        if (den == 0.0) WH_FAIL(ctx, WH_EBREAKDOWN, "deflation vector %d is at resonance", k);
        sc[k] = -1.0 / den;
      }
      WHCHK(upload(ctx, at<double>(ws, L.invmu), sc.data(), nd));
      launch_defl_project(S.defl, f, S.partials, s);
      launch_defl_reduce_set(S.defl, S.partials, S.slots, S_H, nullptr, s);
      launch_defl_reduce_set(S.defl, S.partials, at<double>(ws, L.ones), 0, at<double>(ws, L.invmu), s);
      launch_defl_combine(S.defl, r, 0.0, f, 1.0, S.slots, S_H, N, s);
      const double h = 1.0 / grid->n;
      const double dt2 = tp.dt * tp.dt;
      const double ks = dt2 / (2.0 * h * h);
      launch_prep_coeffs(c2, r, at<void>(ws, L.kap64), at<void>(ws, L.fs64), false, ks, dt2, N, grid->n,
                         grid->dim, s);
      if (mixed)
        launch_prep_coeffs(c2, r, at<void>(ws, L.kap32), at<void>(ws, L.fs32), true, ks, dt2, N, grid->n,
                           grid->dim, s);
      HIPCHK(ctx, hipMemsetAsync(r, 0, 8 * N, s));
    }
  }
  // b = Pi_h(0; f) in FP64: one wave solve from zero, accumulated into b
  {
    WaveOp ob = S.op64;
    ob.V = b;
    HIPCHK(ctx, hipMemsetAsync(q, 0, 8 * N, s));
    wave_solve(ob, q, true, M_LAST_V, nullptr, nullptr, s);
    S.ws64++;
  }
  // is the initial guess nonzero?  Is b zero (then so is the solution: A is nonsingular,
  // and no relative stopping test is defined)?
  dot(S, u, u, S_TMP2);
  dot(S, b, b, S_NB);
  WHCHK(readback(ctx, S.slots, S_NSLOTS_FIXED));
  const bool b_zero = !(ctx->hbuf[S_NB] > 0);
  if (b_zero) HIPCHK(ctx, hipMemsetAsync(u, 0, 8 * N, s));
  const bool u_nonzero = !b_zero && ctx->hbuf[S_TMP2] > 0;
  wh_status st = WH_OK;
  KrylovResult kr;
  int outer = 0;
  double true_rel = -1.0;
  const int restart = std::max(1, P.restart);
  if (b_zero) {
    // u = 0 is the solution (set above); no iteration
    kr = KrylovResult{};
    st = WH_OK;
    S.iters = 0;
    true_rel = 0.0;
  } else if (!mixed) {
    if (P.solver == WH_FPI) {
      // FPI: x <- Pi x with the forcing on; ||b||^2 for the relative update
      dot(S, b, b, S_NB);
      WHCHK(fpi_solve(S, u, P.tol, P.max_iters, P.check_every, kr, P.devd == 2));
    } else if (P.solver == WH_GMRES) {
      WHCHK(gmres_solve(S, false, b, u, u_nonzero, r, at<double>(ws, L.basis), restart, P.tol,
                        P.max_iters, kr, agmres));
    } else if (P.solver == WH_BICGSTAB) {
      WHCHK(bicgstab_solve(S, false, b, u, u_nonzero, r, p, q, at<double>(ws, L.basis), P.tol,
                           P.max_iters, kr, agmres));
    } else {
      WHCHK(cg_solve(S, false, b, u, u_nonzero, r, p, q, P.tol, P.max_iters, P.solver == WH_DCG,
                     reproject, P.check_every, kr));
    }
    st = kr.st;
    S.iters = kr.iters;
    // true FP64 residual at exit
    applyA(S, false, u, q);
    launch_sub(r, b, q, N, s);
    dot(S, r, r, S_TMP);
    dot(S, b, b, S_NB);
    WHCHK(readback(ctx, S.slots, S_NSLOTS_FIXED));
    true_rel = ctx->hbuf[S_NB] > 0 ? std::sqrt(ctx->hbuf[S_TMP] / ctx->hbuf[S_NB]) : 0.0;
  } else if (!outer_refined) {
    // CG / DCG with FP32 stepping and reliable updates (true FP64 residuals)
    WHCHK(cg_solve(S, true, b, u, u_nonzero, r, p, q, P.tol, P.max_iters, P.solver == WH_DCG,
                   reproject, 1, kr, false, true));
    st = kr.st;
    S.iters = kr.iters;
    outer = kr.replacements;
    true_rel = kr.rel;
  } else {
    // GMRES / BiCGStab: FP64 outer residual, FP32 inner solves
    double* ro = at<double>(ws, L.ro);
    double* dv = at<double>(ws, L.d);
    dot(S, b, b, S_NB);
    WHCHK(readback(ctx, S.slots, S_NSLOTS_FIXED));
    const double nb = std::sqrt(ctx->hbuf[S_NB]);
    const int max_outer = P.max_outer > 0 ? P.max_outer : 30;
    const double itol = P.inner_tol > 0 ? P.inner_tol : 1e-3;
    bool nonzero = u_nonzero;
    int inner_total = 0;
    st = WH_ENOCONV;
    double rel = 1.0, prev_rel = 1.0;
    bool inner_f32 = true;   // cleared when FP32 refinement stops contracting
    for (outer = 0; outer <= max_outer; ++outer) {
      if (nonzero) {
        applyA(S, false, u, q);
        launch_sub(ro, b, q, N, s);
      } else {
        launch_copy(ro, b, N, s);
      }
      dot(S, ro, ro, S_TMP);
      WHCHK(readback(ctx, S.slots, S_NSLOTS_FIXED));
      rel = nb > 0 ? std::sqrt(ctx->hbuf[S_TMP]) / nb : 0.0;
      if (!std::isfinite(rel)) WH_FAIL(ctx, WH_EUNSTABLE, "non-finite outer residual");
      if (rel <= P.tol) {
        st = WH_OK;
        break;
      }
      if (outer == max_outer || inner_total >= P.max_iters) break;
      // refinement must contract; if a sweep did not halve the true residual the FP32
      // operator error is too large for this problem and the inner solves go to FP64
      if (outer >= 2 && rel > 0.5 * prev_rel) inner_f32 = false;
      prev_rel = rel;
      // inner: A d = ro to a relative tolerance (never tighter than needed)
      const double t_in = inner_f32 ? std::max(itol, 0.3 * P.tol / rel) : 0.3 * P.tol / rel;
      HIPCHK(ctx, hipMemsetAsync(dv, 0, 8 * N, s));
      KrylovResult ir;
      if (P.solver == WH_GMRES) {
        WHCHK(gmres_solve(S, inner_f32, ro, dv, false, r, at<double>(ws, L.basis), restart, t_in,
                          P.max_iters - inner_total, ir, agmres));
      } else if (P.solver == WH_BICGSTAB) {
        WHCHK(bicgstab_solve(S, inner_f32, ro, dv, false, r, p, q, at<double>(ws, L.basis), t_in,
                             P.max_iters - inner_total, ir, agmres));
      } else {
        WHCHK(cg_solve(S, inner_f32, ro, dv, false, r, p, q, t_in, P.max_iters - inner_total,
                       P.solver == WH_DCG, reproject, P.check_every, ir, inner_f32));
      }
      inner_total += ir.iters;
      if (ir.diverged) {       // discard the sweep and redo it in FP64
        inner_f32 = false;
        continue;
      }
      launch_axpy(u, dv, 1.0, N, s);
      nonzero = true;
    }
    S.iters = inner_total;
    kr.rel = rel;
    true_rel = rel;
  }
  if (devd) {
    // Algorithm 2, inflation: u += sum_k (phi_k^T f) / (omega_fp^2 - lambda_k^2) phi_k
    // (the coefficients were stored negated in the workspace before the solve)
    launch_defl_combine(S.defl, u, 1.0, nullptr, 0.0, at<double>(ws, L.ones), 0, N, s);
  }
  HIPCHK(ctx, hipGetLastError());
  HIPCHK(ctx, hipStreamSynchronize(s));
  if (info) {
    fill_info(info, tp, params->precision == WH_MIXED ? S.op32.k_fuse : S.op64.k_fuse,
              params->precision == WH_MIXED ? &S.op32 : &S.op64);
    info->status = st;
    info->iters = S.iters;
    info->wave_solves = S.ws64;
    info->wave_solves_f32 = S.ws32;
    info->outer = outer;
    info->rel_res = kr.rel;
    info->true_rel_res = true_rel;
    info->ms = now_ms() - t0;
  }
  if (st == WH_ENOCONV) ctx->err = "tolerance not reached";
  return st;
  });
}

wh_status wh_helmholtz_residual(wh_ctx* ctx, const wh_grid* grid, const double* c2,
                                const double* f, double omega, const double* u, void* ws,
                                size_t ws_bytes, double* rel) {
  return guard(ctx, [&]() -> wh_status {
  if (!ctx) return WH_EINVAL;
  WHCHK(check_grid(ctx, grid));
  if (!f || !u || !rel) WH_FAIL(ctx, WH_EINVAL, "NULL argument");
  const size_t need = 16 * (size_t)kReduceBlocks + 256;
  WHCHK(check_ws(ctx, ws, ws_bytes, need));
  HIPCHK(ctx, hipSetDevice(ctx->device));
  double* pr = at<double>(ws, 0);
  double* pf = pr + kReduceBlocks;
  double* out = at<double>(ws, 16 * (size_t)kReduceBlocks);
  const double ih2 = (double)grid->n * grid->n;
  if (grid->order == 4 && c2)
    WH_FAIL(ctx, WH_EUNSUPPORTED, "fourth-order differences are built for c == 1 (c2 == NULL)");
  launch_helmholtz_residual(c2, f, u, omega * omega, ih2, grid->n, grid->dim, grid->order, pr, pf,
                            ctx->stream);
  launch_reduce(pr, kReduceBlocks, out, 0, 0, ctx->stream);
  launch_reduce(pf, kReduceBlocks, out, 1, 0, ctx->stream);
  HIPCHK(ctx, hipGetLastError());
  WHCHK(readback(ctx, out, 2));
  *rel = ctx->hbuf[1] > 0 ? std::sqrt(ctx->hbuf[0] / ctx->hbuf[1]) : 0.0;
  return WH_OK;
  });
}

wh_status wh_time_step_kernel(wh_ctx* ctx, const wh_grid* grid, const double* c2,
                              const wh_params* params, int32_t reps, void* ws, size_t ws_bytes,
                              double* us_per_launch, int32_t* k_used, int32_t* rows,
                              int32_t* waves) {
  return guard(ctx, [&]() -> wh_status {
  if (!ctx) return WH_EINVAL;
  WHCHK(check_grid(ctx, grid));
  WHCHK(check_params(ctx, grid, params));
  if (reps < 1 || !us_per_launch) WH_FAIL(ctx, WH_EINVAL, "reps must be >= 1 and us_per_launch set");
  const Layout L = make_layout(*grid, *params, nullptr);
  WHCHK(check_ws(ctx, ws, ws_bytes, L.total));
  HIPCHK(ctx, hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  TimeParams tp;
  Solver S{};
  WHCHK(setup_ops(ctx, *grid, *params, c2, nullptr, ws, L, tp, S));
  const WaveOp& op = params->precision == WH_MIXED ? S.op32 : S.op64;
  for (size_t off : {L.Wa, L.Wb, L.Wc, L.Wd, L.V})
    HIPCHK(ctx, hipMemsetAsync(at<void>(ws, off), 0, 8 * (size_t)L.N, s));
  const int K = op.k_fuse;
  if (K > 1 && K + 2 > tp.nt) WH_FAIL(ctx, WH_EINVAL, "K larger than the wave solve");
  auto run = [&](int r) {
    if (K > 1 && op.order == 4) {
      March4Args m{};
      m.cur = (r & 1) ? op.Wc : op.Wb;
      m.prev = (r & 1) ? op.Wd : op.Wa;
      m.cur_out = (r & 1) ? op.Wb : op.Wc;
      m.prev_out = (r & 1) ? op.Wa : op.Wd;
      m.V = op.V;
      m.fs = nullptr;
      m.a12 = op.a / 12.0;
      for (int j = 1; j <= K; ++j) m.w[j] = tp.w[j + 1];
      for (int j = 0; j < K; ++j) m.cs[j] = tp.cosv[j + 1];
      m.n = op.n;
      m.kp = K;
      launch_march4(op.f32, K, m, s);
    } else if (K <= 1) {
      StepArgs a{};
      a.n = op.n;
      a.kap = op.kap;
      a.a = op.a;
      a.cur = (r & 1) ? op.Wa : op.Wb;
      a.prev = (r & 1) ? op.Wb : op.Wa;
      a.cur_next = op.Wc;
      a.V = op.V;
      a.cosn = tp.cosv[1];
      a.wn = tp.w[2];
      step_any(op, false, M_MID, a, s);
    } else {
      FusedArgs fa{};
      fa.V = op.V;
      fa.kap = op.kap;
      fa.a = op.a;
      fa.n = op.n;
      fa.k = K;
      fa.shape = op.k_shape;
      fa.cur = (r & 1) ? op.Wc : op.Wb;
      fa.prev = (r & 1) ? op.Wd : op.Wa;
      fa.cur_out = (r & 1) ? op.Wb : op.Wc;
      fa.prev_out = (r & 1) ? op.Wa : op.Wd;
      fa.wts = &tp.w[1];
      fa.cosv = &tp.cosv[1];
      launch_fused(op.dim, op.f32, op.varc, false, fa, s);
    }
  };
  run(0);
  hipEvent_t e0, e1;
  HIPCHK(ctx, hipEventCreate(&e0));
  HIPCHK(ctx, hipEventCreate(&e1));
  (void)hipEventRecord(e0, s);
  for (int r = 0; r < reps; ++r) run(r + 1);
  (void)hipEventRecord(e1, s);
  hipError_t e = hipEventSynchronize(e1);
  float ms = 0;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) WH_FAIL(ctx, WH_EHIP, "event timing failed: %s", hipGetErrorString(e));
  *us_per_launch = 1e3 * (double)ms / reps;
  if (k_used) *k_used = K;
  int rr = 0, wv = 0;
  if (K > 1 && op.order == 4) {
    rr = 32;   // rows per tile of the row-marching launch
    wv = 4;    // strips (wavefronts) per block
  } else if (K > 1) {
    fused_shape_dims(op.dim, op.f32, K, op.k_shape, &rr, &wv);
  }
  if (rows) *rows = rr;
  if (waves) *waves = wv;
  return WH_OK;
  });
}

// ------------------------------------------------------------------ adjoint
}  // extern "C"

namespace {

struct VjpLayout {
  Layout L;           // solver part (CG on A)
  size_t ck = 0, seg = 0, lam = 0, z = 0, g = 0, u = 0, misc = 0, total = 0;
  int nseg = 0, K = 16, nt = 0;
};

VjpLayout make_vjp_layout(const wh_grid& g, const wh_params& P0, int ckpt, int nt) {
  wh_params P = P0;
  if (P.solver != WH_CG) P.solver = WH_CG;
  VjpLayout V;
  V.L = make_layout(g, P, nullptr);
  V.K = ckpt > 0 ? ckpt : 16;
  V.nt = nt;
  V.nseg = (nt + V.K - 1) / V.K;
  const size_t N = (size_t)V.L.N;
  size_t off = V.L.total;
  auto take2 = [&](size_t bytes) {
    size_t o = off;
    off += (bytes + 255) & ~(size_t)255;
    return o;
  };
  V.ck = take2(8 * N * 2 * (size_t)V.nseg);
  V.seg = take2(8 * N * (size_t)(V.K + 1));
  V.lam = take2(8 * N * 3);
  V.z = take2(8 * N);
  V.g = take2(8 * N);
  V.u = take2(8 * N);
  V.misc = take2(4096);
  V.total = off;
  return V;
}

// grad += (dPi_h/dc2)^T A^{-1} g at the fixed point u of Pi_h(.; f) (2D, c2 given).
// g must have a zero boundary; u too.  Uses the solver part of the workspace for
// the CG solve of A z = g.
wh_status vjp_core(wh_ctx* ctx, const wh_grid& G, const double* c2, const double* f,
                   const double* u, double* g, const wh_params& P, void* ws,
                   const VjpLayout& V, double* grad, wh_info* info) {
  hipStream_t s = ctx->stream;
  TimeParams tp;
  Solver S{};
  WHCHK(setup_ops(ctx, G, P, c2, f, ws, V.L, tp, S));
  if (tp.nt != V.nt) WH_FAIL(ctx, WH_EINVAL, "time steps changed between sizing and use");
  const int64_t N = V.L.N;
  const int n = G.n;
  double* z = at<double>(ws, V.z);
  double* r = at<double>(ws, V.L.r);
  double* p = at<double>(ws, V.L.p);
  double* q = at<double>(ws, V.L.q);
  HIPCHK(ctx, hipMemsetAsync(z, 0, 8 * N, s));
  for (double* v : {r, p, q}) HIPCHK(ctx, hipMemsetAsync(v, 0, 8 * N, s));
  if (V.L.has_p2) {
    S.p2 = at<double>(ws, V.L.p2);
    HIPCHK(ctx, hipMemsetAsync(S.p2, 0, 8 * N, s));
  }
  HIPCHK(ctx, hipMemsetAsync(S.slots, 0, 8 * (size_t)V.L.nslots, s));
  // z = A^{-1} g (A symmetric)
  KrylovResult kr;
  const bool mixed = P.precision == WH_MIXED;
  WHCHK(cg_solve(S, mixed, g, z, false, r, p, q, P.tol, P.max_iters, false, false,
                 P.check_every, kr, false, mixed));
  if (info) {
    info->iters += kr.iters;
    info->rel_res = std::max(info->rel_res, kr.rel);
  }
  const double* kap = (const double*)S.op64.kap;   // c2 dt^2 / (2 h^2), FP64
  const double* fs = (const double*)S.op64.fs;     // f dt^2
  double* ck = at<double>(ws, V.ck);
  double* seg = at<double>(ws, V.seg);
  double* lamb = at<double>(ws, V.lam);
  for (size_t o : {V.seg, V.lam}) HIPCHK(ctx, hipMemsetAsync(at<void>(ws, o), 0,
                                                           8 * (size_t)N * (o == V.seg ? V.K + 1 : 3), s));
  HIPCHK(ctx, hipMemsetAsync(ck, 0, 8 * (size_t)N * 2 * V.nseg, s));
  const int K = V.K, NT = tp.nt;
  auto CK = [&](int j, int w) { return ck + ((size_t)2 * j + w) * N; };
  auto SEG = [&](int m) { return seg + (size_t)m * N; };
  // forward pass from W^0 = u with the forcing, keeping (W^{jK}, W^{jK+1})
  {
    // three rotating slots of the segment buffer (K >= 2): bufs[m % 3] holds W^m
    double* bufs[3] = {SEG(0), SEG(1), SEG(2)};
    HIPCHK(ctx, hipMemcpyAsync(bufs[0], u, 8 * N, hipMemcpyDeviceToDevice, s));
    launch_fwd_out2d(bufs[0], nullptr, bufs[1], kap, fs, tp.cosv[0], true, n, s);
    for (int m = 0; m < NT; ++m) {
      if (m >= 2) launch_fwd_out2d(bufs[(m - 1) % 3], bufs[(m - 2) % 3], bufs[m % 3], kap, fs,
                                   tp.cosv[m - 1], false, n, s);
      if (m % K == 0)
        HIPCHK(ctx, hipMemcpyAsync(CK(m / K, 0), bufs[m % 3], 8 * N, hipMemcpyDeviceToDevice, s));
      if (m % K == 1)
        HIPCHK(ctx, hipMemcpyAsync(CK(m / K, 1), bufs[m % 3], 8 * N, hipMemcpyDeviceToDevice, s));
    }
  }
  // reverse sweep
  double* L0 = lamb;          // Lam^n (output)
  double* L1 = lamb + N;      // Lam^{n+1}
  double* L2 = lamb + 2 * N;  // Lam^{n+2}
  HIPCHK(ctx, hipMemsetAsync(lamb, 0, 8 * (size_t)N * 3, s));
  launch_axpy(L1, z, tp.w[NT], N, s);  // Lam^N = w_N z
  const double h = 1.0 / n;
  const double gscale = -tp.dt * tp.dt / (2.0 * h * h);
  for (int j = V.nseg - 1; j >= 0; --j) {
    const int n0 = j * K, n1 = std::min(n0 + K, NT);
    HIPCHK(ctx, hipMemcpyAsync(SEG(0), CK(j, 0), 8 * N, hipMemcpyDeviceToDevice, s));
    if (n1 - n0 >= 2)
      HIPCHK(ctx, hipMemcpyAsync(SEG(1), CK(j, 1), 8 * N, hipMemcpyDeviceToDevice, s));
    for (int m = 2; m < n1 - n0; ++m)
      launch_fwd_out2d(SEG(m - 1), SEG(m - 2), SEG(m), kap, fs, tp.cosv[n0 + m - 1], false, n, s);
    for (int nn = n1 - 1; nn >= n0; --nn) {
      const double* W = SEG(nn - n0);
      if (nn >= 1) {
        launch_adj_step2d(L1, L2, L0, W, kap, z, tp.w[nn], gscale, grad, true, n, s);
        double* t = L2;
        L2 = L1;
        L1 = L0;
        L0 = t;
      } else {
        launch_adj_step2d(L1, L2, L0, W, kap, z, 0.0, 0.5 * gscale, grad, false, n, s);
      }
    }
  }
  HIPCHK(ctx, hipGetLastError());
  if (info) {
    fill_info(info, tp, 1);
    info->wave_solves += S.ws64 + 3;
    info->wave_solves_f32 += S.ws32;
  }
  return WH_OK;
}

wh_status adjoint_validate(wh_ctx* ctx, const wh_grid* grid, const double* c2, const wh_params* P,
                           int ckpt) {
  WHCHK(check_grid(ctx, grid));
  WHCHK(check_params(ctx, grid, P));
  if (grid->dim != 2 || grid->order != 2)
    WH_FAIL(ctx, WH_EUNSUPPORTED, "the adjoint gradient is built for 2D second-order grids");
  if (!c2) WH_FAIL(ctx, WH_EINVAL, "c2 is required (the gradient is taken with respect to it)");
  if (ckpt < 0 || ckpt == 1 || ckpt > 4096)
    WH_FAIL(ctx, WH_EINVAL, "ckpt_every must be 0 (default 16) or in [2, 4096]");
  if (!(P->tol > 0)) WH_FAIL(ctx, WH_EINVAL, "tol must be > 0");
  return WH_OK;
}

// N_t needs c_max: the caller's bound, else computed on the device from c2.
wh_status adjoint_nt(wh_ctx* ctx, const wh_grid& G, const double* c2, const wh_params& P,
                     void* ws, int* nt) {
  double cmax = P.c_max;
  if (!(cmax > 0)) {
    if (!ctx || !ws) return WH_EINVAL;
    const int64_t N = nodal_count(G.dim, G.n);
    double* part = at<double>(ws, 0);
    launch_max_partials(c2, N, part, false, ctx->stream);
    launch_max_finalize(part, kReduceBlocks, part + kReduceBlocks, ctx->stream);
    WHCHK(readback(ctx, part + kReduceBlocks, 1));
    cmax = std::sqrt(ctx->hbuf[0]);
  }
  TimeParams tp;
  WHCHK(make_time_params(ctx, G.dim, G.n, P, cmax, tp));
  *nt = tp.nt;
  return WH_OK;
}

}  // namespace

extern "C" {

size_t wh_workspace_bytes_adjoint(const wh_grid* grid, const wh_params* params, int32_t ckpt_every) {
  return guard_size([&]() -> size_t {
  if (!grid || !params || check_grid(nullptr, grid) != WH_OK || grid->dim != 2 || grid->order != 2) return 0;
  if (!(params->c_max > 0)) return 0;
  TimeParams tp;
  if (make_time_params(nullptr, 2, grid->n, *params, params->c_max, tp) != WH_OK) return 0;
  return make_vjp_layout(*grid, *params, ckpt_every, tp.nt).total;
  });
}

wh_status wh_solve_vjp(wh_ctx* ctx, const wh_grid* grid, const double* c2, const double* f,
                       const double* u, const double* grad_u, const wh_params* params,
                       int32_t ckpt_every, double* grad_c2, void* ws, size_t ws_bytes,
                       wh_info* info) {
  return guard(ctx, [&]() -> wh_status {
  if (!ctx) return WH_EINVAL;
  const double t0 = now_ms();
  if (info) std::memset(info, 0, sizeof(*info));
  WHCHK(adjoint_validate(ctx, grid, c2, params, ckpt_every));
  if (!f || !u || !grad_u || !grad_c2) WH_FAIL(ctx, WH_EINVAL, "NULL argument");
  if (!(params->c_max > 0)) WH_FAIL(ctx, WH_EINVAL, "params->c_max must bound c (sizes the workspace)");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  int nt = 0;
  WHCHK(adjoint_nt(ctx, *grid, c2, *params, nullptr, &nt));
  const VjpLayout V = make_vjp_layout(*grid, *params, ckpt_every, nt);
  WHCHK(check_ws(ctx, ws, ws_bytes, V.total));
  const int64_t N = V.L.N;
  double* g = at<double>(ws, V.g);
  double* uu = at<double>(ws, V.u);
  HIPCHK(ctx, hipMemcpyAsync(g, grad_u, 8 * N, hipMemcpyDeviceToDevice, ctx->stream));
  HIPCHK(ctx, hipMemcpyAsync(uu, u, 8 * N, hipMemcpyDeviceToDevice, ctx->stream));
  launch_zero_boundary(g, grid->n, 2, ctx->stream);
  launch_zero_boundary(uu, grid->n, 2, ctx->stream);
  WHCHK(vjp_core(ctx, *grid, c2, f, uu, g, *params, ws, V, grad_c2, info));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  if (info) info->ms = now_ms() - t0;
  return WH_OK;
  });
}

wh_status wh_adjoint_grad(wh_ctx* ctx, const wh_grid* grid, const double* c2, int32_t n_src,
                          const double* const* f, int32_t n_rec, const int64_t* rec_idx,
                          const double* d, const wh_params* params, int32_t ckpt_every,
                          double* grad_c2, double* J, void* ws, size_t ws_bytes, wh_info* info) {
  return guard(ctx, [&]() -> wh_status {
  if (!ctx) return WH_EINVAL;
  const double t0 = now_ms();
  if (info) std::memset(info, 0, sizeof(*info));
  WHCHK(adjoint_validate(ctx, grid, c2, params, ckpt_every));
  if (n_src < 1 || !f || n_rec < 1 || !rec_idx || !d || !J)
    WH_FAIL(ctx, WH_EINVAL, "need n_src >= 1 sources, n_rec >= 1 receivers and outputs");
  for (int s_ = 0; s_ < n_src; ++s_)
    if (!f[s_]) WH_FAIL(ctx, WH_EINVAL, "source %d is NULL", s_);
  if (!(params->c_max > 0)) WH_FAIL(ctx, WH_EINVAL, "params->c_max must bound c (sizes the workspace)");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  int nt = 0;
  WHCHK(adjoint_nt(ctx, *grid, c2, *params, nullptr, &nt));
  const VjpLayout V = make_vjp_layout(*grid, *params, ckpt_every, nt);
  WHCHK(check_ws(ctx, ws, ws_bytes, V.total));
  const int64_t N = V.L.N;
  // receivers: interior nodes only, checked before any read through them
  int* bad = at<int>(ws, V.misc);
  HIPCHK(ctx, hipMemsetAsync(bad, 0, 4, s));
  launch_check_idx(rec_idx, n_rec, grid->n, bad, s);
  HIPCHK(ctx, hipMemcpyAsync(ctx->hbuf, bad, 4, hipMemcpyDeviceToHost, s));
  HIPCHK(ctx, hipStreamSynchronize(s));
  int badv = 0;
  std::memcpy(&badv, ctx->hbuf, 4);
  if (badv) WH_FAIL(ctx, WH_EINVAL, "receiver indices must be interior nodes of the grid");
  if (grad_c2) HIPCHK(ctx, hipMemsetAsync(grad_c2, 0, 8 * N, s));
  double* u = at<double>(ws, V.u);
  double* g = at<double>(ws, V.g);
  double* jslot = at<double>(ws, V.misc) + 8;
  wh_params P = *params;
  P.solver = WH_CG;
  double Jsum = 0.0;
  wh_status worst = WH_OK;
  for (int si = 0; si < n_src; ++si) {
    wh_info in{};
    HIPCHK(ctx, hipMemsetAsync(u, 0, 8 * N, s));
    wh_status st = wh_solve(ctx, grid, c2, f[si], nullptr, &P, u, ws, V.L.total, &in);
    if (st < 0) return st;
    if (st == WH_ENOCONV) worst = WH_ENOCONV;
    HIPCHK(ctx, hipMemsetAsync(g, 0, 8 * N, s));
    launch_misfit(u, rec_idx, d + (size_t)si * n_rec, n_rec, g, jslot, s);
    WHCHK(readback(ctx, jslot, 1));
    Jsum += ctx->hbuf[0];
    wh_info vi{};
    if (grad_c2) WHCHK(vjp_core(ctx, *grid, c2, f[si], u, g, P, ws, V, grad_c2, &vi));
    if (info) {
      info->iters += in.iters + vi.iters;
      info->wave_solves += in.wave_solves + vi.wave_solves;
      info->wave_solves_f32 += in.wave_solves_f32 + vi.wave_solves_f32;
      info->true_rel_res = std::max(info->true_rel_res, in.true_rel_res);
      info->rel_res = std::max(info->rel_res, vi.rel_res);
      info->nt = in.nt;
      info->m = in.m;
      info->dt = in.dt;
      info->omega_tilde = in.omega_tilde;
      info->c_max = in.c_max;
    }
  }
  HIPCHK(ctx, hipStreamSynchronize(s));
  *J = Jsum;
  if (info) {
    info->status = worst;
    info->ms = now_ms() - t0;
  }
  return worst;
  });
}

}  // extern "C"
