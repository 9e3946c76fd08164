// Drives every libwaveholtz entry point through the C ABI with the host-only build and
// the stand-in runtime of hip_stub.hip (see there).  Each "device" buffer is a host
// allocation of exactly the size the Python binding would pass, registered with the
// stand-in so that every launch and copy is checked against it; the workspace is exactly
// wh_workspace_bytes*() long.  Usage: hostcheck <group> [seed]; groups: vjp, solve,
// filter, batched, all.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/waveholtz.h"

extern "C" {
void hostcheck_register(const void* p, size_t bytes, const char* name);
void hostcheck_unregister(const void* p);
void hostcheck_seed(unsigned s);
void hostcheck_report(void);
void hostcheck_restart_residual(void);
}

namespace {

struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
  Buf(size_t b, const char* name) : bytes(b) {
    const size_t cap = (b + 255) / 256 * 256;
    p = aligned_alloc(256, cap ? cap : 256);
    std::memset(p, 0, cap ? cap : 256);
    hostcheck_register(p, b, name);
  }
  ~Buf() {
    hostcheck_unregister(p);
    free(p);
  }
  Buf(const Buf&) = delete;
  Buf& operator=(const Buf&) = delete;
  double* d() { return (double*)p; }
};

int g_fail = 0;
wh_ctx* g_ctx = nullptr;

void expect(bool ok, const char* what, int st) {
  if (!ok) {
    fprintf(stderr, "unexpected status %d (%s) in %s: %s\n", st, wh_status_string((wh_status)st), what,
            wh_last_error(g_ctx));
    ++g_fail;
  }
}

size_t nodal(int dim, int n) {
  size_t P = (size_t)n + 1;
  return dim == 2 ? P * P : P * P * P;
}

void fill_field(double* a, int dim, int n, double base, double amp, unsigned seed) {
  const size_t N = nodal(dim, n);
  unsigned s = seed * 2654435761u + 12345u;
  for (size_t i = 0; i < N; ++i) {
    s = s * 1664525u + 1013904223u;
    a[i] = base + amp * ((double)(s >> 8) / (double)(1u << 24) - 0.5);
  }
}

wh_params params(double omega) {
  hostcheck_restart_residual();
  wh_params p;
  wh_params_default(&p);
  p.omega = omega;
  return p;
}

// ------------------------------------------------------------------ adjoint
void vjp_case(int n, int ckpt, double omega, unsigned seed) {
  const wh_grid g{2, n, 2};
  const size_t N = nodal(2, n);
  Buf c2(8 * N, "c2"), f(8 * N, "f"), u(8 * N, "u"), gu(8 * N, "grad_u"), out(8 * N, "grad_c2");
  fill_field(c2.d(), 2, n, 1.1, 0.2, seed);
  fill_field(f.d(), 2, n, 0.0, 1.0, seed + 1);
  fill_field(u.d(), 2, n, 0.0, 1.0, seed + 2);
  fill_field(gu.d(), 2, n, 0.0, 1.0, seed + 3);
  double cmax2 = 0;
  for (size_t i = 0; i < N; ++i) cmax2 = std::max(cmax2, c2.d()[i]);
  wh_params p = params(omega);
  p.tol = 1e-13;
  p.c_max = std::sqrt(cmax2);
  p.max_iters = 5000;
  const size_t need = wh_workspace_bytes_adjoint(&g, &p, ckpt);
  expect(need > 0, "wh_workspace_bytes_adjoint", 0);
  Buf ws(need, "adjoint workspace");
  wh_info info;
  int st = wh_solve_vjp(g_ctx, &g, c2.d(), f.d(), u.d(), gu.d(), &p, ckpt, out.d(), ws.p, need, &info);
  expect(st >= 0, "wh_solve_vjp", st);
  printf("vjp n=%d ckpt=%d status=%d iters=%d nt=%d\n", n, ckpt, st, info.iters, info.nt);
}

void adjoint_case(int n, int n_src, double omega, int ckpt, unsigned seed) {
  const wh_grid g{2, n, 2};
  const size_t N = nodal(2, n);
  Buf c2(8 * N, "c2"), grad(8 * N, "grad");
  fill_field(c2.d(), 2, n, 1.1, 0.2, seed);
  std::vector<Buf*> srcs;
  std::vector<const double*> fp;
  for (int s = 0; s < n_src; ++s) {
    srcs.push_back(new Buf(8 * N, "source"));
    fill_field(srcs.back()->d(), 2, n, 0.0, 1.0, seed + 10 + s);
    fp.push_back(srcs.back()->d());
  }
  std::vector<int64_t> idx;
  for (int k = 1; k < n; k += 3) idx.push_back((int64_t)(n / 4) * (n + 1) + k);
  for (int k = 1; k < n; k += 3) idx.push_back((int64_t)k * (n + 1) + 3 * n / 4);
  const int nrec = (int)idx.size();
  Buf ridx(8 * nrec, "rec_idx"), d(8 * (size_t)nrec * n_src, "data");
  std::memcpy(ridx.p, idx.data(), 8 * nrec);
  double cmax2 = 0;
  for (size_t i = 0; i < N; ++i) cmax2 = std::max(cmax2, c2.d()[i]);
  wh_params p = params(omega);
  p.tol = 1e-12;
  p.c_max = std::sqrt(cmax2);
  p.max_iters = 5000;
  const size_t need = wh_workspace_bytes_adjoint(&g, &p, ckpt);
  Buf ws(need, "adjoint workspace");
  double J = 0;
  wh_info info;
  int st = wh_adjoint_grad(g_ctx, &g, c2.d(), n_src, fp.data(), nrec, (const int64_t*)ridx.p, d.d(), &p, ckpt,
                           grad.d(), &J, ws.p, need, &info);
  expect(st >= 0, "wh_adjoint_grad", st);
  printf("adjoint n=%d n_src=%d status=%d\n", n, n_src, st);
  for (Buf* b : srcs) delete b;
}

// ------------------------------------------------------------------ solves
void select_modes(int dim, int n, double omega, int nd, std::vector<int32_t>& modes, std::vector<double>& l2) {
  modes.assign((size_t)nd * dim, 0);
  l2.assign(nd, 0.0);
  int st = wh_select_sine_modes(dim, n, 2, omega, nd, modes.data(), l2.data());
  expect(st == 0, "wh_select_sine_modes", st);
}

void solve_case(int dim, int n, int solver, int precision, bool varc, int k_fuse, int k_shape, int nd,
                int defl_kind, unsigned seed, int devd = 0, int restart = 40) {
  const wh_grid g{dim, n, 2};
  const size_t N = nodal(dim, n);
  Buf f(8 * N, "f"), u(8 * N, "u");
  Buf* c2 = varc ? new Buf(8 * N, "c2") : nullptr;
  if (c2) fill_field(c2->d(), dim, n, 1.1, 0.2, seed);
  fill_field(f.d(), dim, n, 0.0, 1.0, seed + 1);
  const double omega = 0.37 * n + 1.3;
  wh_params p = params(omega);
  p.solver = solver;
  p.precision = precision;
  p.k_fuse = k_fuse;
  p.k_shape = k_shape;
  p.devd = devd;
  p.restart = restart;
  p.max_iters = 60;
  p.tol = 1e-9;
  if (c2) {
    double m = 0;
    for (size_t i = 0; i < N; ++i) m = std::max(m, c2->d()[i]);
    p.c_max = std::sqrt(m);
  }
  wh_deflation d{};
  std::vector<int32_t> modes;
  std::vector<double> l2;
  Buf* V = nullptr;
  Buf* fx = nullptr;
  Buf* fy = nullptr;
  std::vector<int32_t> tm;
  if (nd > 0) {
    select_modes(dim, n, omega, nd, modes, l2);
    d.kind = defl_kind;
    d.n_d = nd;
    if (defl_kind == WH_DEFL_SINE) {
      d.modes = modes.data();
    } else if (defl_kind == WH_DEFL_DENSE) {
      V = new Buf(8 * N * nd, "deflation columns");
      fill_field(V->d(), dim, n, 0.0, 0.1, seed + 7);
      d.V = V->d();
      d.ldv = (int64_t)N;
    } else if (defl_kind == WH_DEFL_DENSE_EXACT) {
      V = new Buf(8 * N * nd, "deflation columns");
      fill_field(V->d(), dim, n, 0.0, 0.1, seed + 7);
      d.V = V->d();
      d.ldv = (int64_t)N;
      d.lambda2 = l2.data();
    } else if (defl_kind == WH_DEFL_FACTORED) {
      const int T = 2 * nd;
      fx = new Buf(8 * (size_t)T * (n + 1), "fx");
      fy = new Buf(8 * (size_t)T * (n + 1), "fy");
      for (int t = 0; t < T; ++t) tm.push_back(t / 2);
      d.n_terms = T;
      d.term_mode = tm.data();
      d.fx = fx->d();
      d.fy = fy->d();
      d.lambda2 = l2.data();
    }
  }
  const size_t need = wh_workspace_bytes(&g, &p, nd ? &d : nullptr);
  Buf ws(need, "workspace");
  wh_info info;
  int st = wh_solve(g_ctx, &g, c2 ? c2->d() : nullptr, f.d(), nd ? &d : nullptr, &p, u.d(), ws.p, need, &info);
  expect(st >= 0 || st == WH_EUNSTABLE || st == WH_EBREAKDOWN, "wh_solve", st);
  printf("solve dim=%d n=%d solver=%d prec=%d varc=%d K=%d shape=%d nd=%d kind=%d devd=%d -> %d (K used %d)\n", dim,
         n, solver, precision, (int)varc, k_fuse, k_shape, nd, defl_kind, devd, st, info.k_fuse);
  // Helmholtz residual of the result
  Buf hws(16 * 1024 + 4096, "residual workspace");
  double rel = 0;
  st = wh_helmholtz_residual(g_ctx, &g, c2 ? c2->d() : nullptr, f.d(), omega, u.d(), hws.p, hws.bytes, &rel);
  expect(st == 0, "wh_helmholtz_residual", st);
  delete c2;
  delete V;
  delete fx;
  delete fy;
}

void filter_case(int dim, int n, int order, bool varc, bool force, int precision, int k_fuse, unsigned seed) {
  const wh_grid g{dim, n, order};
  const size_t N = nodal(dim, n);
  Buf v(8 * N, "v_in"), out(8 * N, "v_out"), f(8 * N, "f");
  Buf* c2 = varc ? new Buf(8 * N, "c2") : nullptr;
  if (c2) fill_field(c2->d(), dim, n, 1.1, 0.2, seed);
  fill_field(v.d(), dim, n, 0.0, 1.0, seed + 1);
  fill_field(f.d(), dim, n, 0.0, 1.0, seed + 2);
  wh_params p = params(0.3 * n + 2.1);
  p.precision = precision;
  p.k_fuse = k_fuse;
  if (c2) p.c_max = 0;   // computed on the device
  const size_t need = wh_workspace_bytes(&g, &p, nullptr);
  Buf ws(need, "workspace");
  wh_info info;
  int st = wh_apply_filter(g_ctx, &g, c2 ? c2->d() : nullptr, force ? f.d() : nullptr, v.d(), out.d(), &p, ws.p,
                           need, &info);
  // a device-computed c_max reads a synthetic maximum; only argument errors are unexpected
  expect(st >= 0 || (varc && st == WH_EINVAL), "wh_apply_filter", st);
  if (dim == 2 && !varc) {
    double us = 0;
    int32_t k = 0, rows = 0, waves = 0;
    st = wh_time_step_kernel(g_ctx, &g, nullptr, &p, 3, ws.p, need, &us, &k, &rows, &waves);
    expect(st == 0, "wh_time_step_kernel", st);
  }
  delete c2;
}

// the allocation-free filter: two calls in a row (the second on a smaller grid), and a grid
// beyond its fixed scratch, which must be rejected with WH_EWORKSPACE
void noalloc_case(int dim, int n, int precision, bool varc, unsigned seed) {
  const wh_grid g{dim, n, 2};
  const size_t N = nodal(dim, n);
  Buf v(8 * N, "v_in"), out(8 * N, "v_out"), f(8 * N, "f");
  Buf* c2 = varc ? new Buf(8 * N, "c2") : nullptr;
  if (c2) fill_field(c2->d(), dim, n, 1.1, 0.2, seed);
  fill_field(v.d(), dim, n, 0.0, 1.0, seed + 1);
  fill_field(f.d(), dim, n, 0.0, 1.0, seed + 2);
  wh_params p = params(0.3 * n + 2.1);
  p.precision = precision;
  if (c2) {
    double m = 0;
    for (size_t i = 0; i < N; ++i) m = std::max(m, c2->d()[i]);
    p.c_max = std::sqrt(m);
  }
  wh_info info;
  int st = wh_apply_filter_noalloc(g_ctx, &g, c2 ? c2->d() : nullptr, f.d(), v.d(), out.d(), &p, &info);
  const bool fits = dim == 2 ? n <= 1024 : n <= 96;
  expect(fits ? st == 0 : st == WH_EWORKSPACE, "wh_apply_filter_noalloc", st);
  printf("noalloc dim=%d n=%d prec=%d varc=%d -> %d (K %d)\n", dim, n, precision, (int)varc, st, info.k_fuse);
  delete c2;
}

void batched_case(int precision, int solver, bool deflate, unsigned seed, int order = 2, int k_fuse = 0) {
  const int ns[] = {8, 16, 24, 33, order == 4 ? 200 : 12};
  const int nb = 5;
  std::vector<Buf*> keep;
  std::vector<wh_problem> probs(nb);
  for (int i = 0; i < nb; ++i) {
    const int n = ns[i];
    const size_t N = nodal(2, n);
    Buf* f = new Buf(8 * N, "f");
    Buf* u = new Buf(8 * N, "u");
    fill_field(f->d(), 2, n, 0.0, 1.0, seed + i);
    keep.push_back(f);
    keep.push_back(u);
    probs[i].grid = wh_grid{2, n, order};
    probs[i].c2 = nullptr;
    probs[i].f = f->d();
    probs[i].omega = 0.31 * n + 1.7;
    probs[i].u = u->d();
    probs[i].n_defl = deflate ? 1 + i % 3 : 0;
  }
  wh_params p = params(1.0);
  p.precision = precision;
  p.solver = solver;
  p.max_iters = 40;
  p.k_fuse = k_fuse;
  const size_t need = wh_workspace_bytes_batched(nb, probs.data(), &p);
  expect(need > 0, "wh_workspace_bytes_batched", 0);
  Buf ws(need, "batched workspace");
  std::vector<wh_info> infos(nb);
  int st = wh_solve_batched(g_ctx, nb, probs.data(), &p, ws.p, need, infos.data());
  expect(st >= 0, "wh_solve_batched", st);
  printf("batched prec=%d solver=%d defl=%d order=%d k=%d -> %d\n", precision, solver, (int)deflate, order,
         k_fuse, st);
  if (precision == WH_MIXED) {
    double us = 0;
    int64_t pts = 0;
    st = wh_time_batch_kernel(g_ctx, nb, probs.data(), &p, 3, ws.p, need, &us, &pts);
    expect(order == 2 ? st == 0 : st == WH_EUNSUPPORTED, "wh_time_batch_kernel", st);
  }
  for (Buf* b : keep) delete b;
}

}  // namespace

int main(int argc, char** argv) {
  const std::string group = argc > 1 ? argv[1] : "all";
  const unsigned seed = argc > 2 ? (unsigned)atoi(argv[2]) : 1;
  hostcheck_seed(seed);
  int st = wh_create(&g_ctx, 0, nullptr);
  if (st != 0) {
    fprintf(stderr, "wh_create failed: %s\n", wh_last_error(nullptr));
    return 2;
  }
  const bool all = group == "all";
  if (all || group == "vjp") {
    // the GPU adjoint tests' arguments: n = 24 with checkpoints every 2, 5, 16 steps;
    // the gradient with 3 sources on 32^2 and 2 on 40^2
    for (int ck : {2, 5, 16}) vjp_case(24, ck, 9.7, seed);
    vjp_case(24, 0, 9.7, seed);
    vjp_case(5, 2, 3.1, seed);
    adjoint_case(32, 3, 9.7, 16, seed);
    adjoint_case(40, 2, 9.7, 16, seed);
    adjoint_case(17, 1, 6.3, 3, seed);
  }
  if (all || group == "solve") {
    for (int n : {5, 7, 16, 24, 33, 64, 97})
      for (int prec : {0, 1})
        for (int solver : {WH_CG, WH_GMRES, WH_BICGSTAB}) {
          solve_case(2, n, solver, prec, false, 0, -1, 0, 0, seed, 0, solver == WH_GMRES ? 7 : 40);
          solve_case(2, n, solver, prec, true, 0, -1, 0, 0, seed);
        }
    for (int n : {7, 24, 64}) {
      solve_case(2, n, WH_FPI, 0, false, 0, -1, 0, 0, seed);
      for (int prec : {0, 1}) {
        solve_case(2, n, WH_DCG, prec, false, 0, -1, 3, WH_DEFL_SINE, seed);
        solve_case(2, n, WH_DCG, prec, false, 0, -1, 3, WH_DEFL_DENSE_EXACT, seed);
        solve_case(2, n, WH_DCG, prec, false, 0, -1, 3, WH_DEFL_FACTORED, seed);
        solve_case(2, n, WH_DCG, prec, true, 0, -1, 4, WH_DEFL_DENSE, seed);
        solve_case(3, n / 4 + 4, WH_DCG, prec, true, 0, -1, 3, WH_DEFL_DENSE, seed);
        solve_case(2, n, WH_GMRES, prec, false, 0, -1, 3, WH_DEFL_SINE, seed, 0, 5);
        solve_case(2, n, WH_BICGSTAB, prec, false, 0, -1, 3, WH_DEFL_SINE, seed);
        solve_case(2, n, WH_CG, prec, false, 0, -1, 3, WH_DEFL_SINE, seed, 1);
      }
      solve_case(2, n, WH_FPI, 0, false, 0, -1, 3, WH_DEFL_SINE, seed, 2);
    }
    // every fixed (K, shape) of the 2D blocked kernel on small and ragged grids
    for (int n : {5, 9, 24, 50, 130})
      for (int K : {2, 3, 4, 6, 8, 9})
        for (int sh = 0; sh < 3; ++sh)
          for (int prec : {0, 1}) {
            solve_case(2, n, WH_CG, prec, false, K, sh, 0, 0, seed);
            solve_case(2, n, WH_CG, prec, true, K, sh, 0, 0, seed);
          }
    for (int n : {6, 12}) {
      solve_case(3, n, WH_CG, 0, true, 0, -1, 0, 0, seed);
      solve_case(3, n, WH_GMRES, 1, true, 0, -1, 0, 0, seed, 0, 5);
    }
  }
  if (all || group == "filter") {
    for (int n : {4, 5, 24, 40, 129})
      for (int prec : {0, 1})
        for (bool varc : {false, true})
          for (bool force : {false, true}) {
            filter_case(2, n, 2, varc, force, prec, 0, seed);
            filter_case(2, n, 2, varc, force, prec, 1, seed);
          }
    for (int n : {6, 10}) {
      filter_case(3, n, 2, false, true, 0, 0, seed);
      filter_case(3, n, 4, false, true, 1, 0, seed);
    }
    // fourth order in 2D: the blocked launches (K = 4 by default, 2 on request) and one step
    // per launch
    for (int n : {6, 10, 40, 129})
      for (int prec : {0, 1})
        for (int k : {0, 2, 3, 1})
          filter_case(2, n, 4, false, n != 40, prec, k, seed);
  }
  if (all || group == "filter") {
    for (int prec : {0, 1})
      for (bool varc : {false, true}) {
        noalloc_case(2, 96, prec, varc, seed);
        noalloc_case(2, 40, prec, varc, seed);
        noalloc_case(2, 5, prec, varc, seed);
        noalloc_case(3, 20, prec, varc, seed);
      }
    noalloc_case(2, 1024, 1, false, seed);
    noalloc_case(2, 1100, 1, false, seed);
    noalloc_case(3, 120, 0, false, seed);
  }
  if (all || group == "batched") {
    for (int prec : {0, 1}) {
      batched_case(prec, WH_CG, false, seed);
      batched_case(prec, WH_DCG, true, seed);
      // fourth order (a 200^2 problem spans two tile columns); K = 8, 4, 2 steps of halo
      for (int k : {0, 8, 2}) batched_case(prec, k == 2 ? WH_CG : WH_DCG, k != 2, seed, 4, k);
    }
  }
  wh_destroy(g_ctx);
  hostcheck_report();
  if (g_fail) {
    fprintf(stderr, "%d unexpected statuses\n", g_fail);
    return 1;
  }
  printf("HOSTCHECK OK\n");
  return 0;
}
