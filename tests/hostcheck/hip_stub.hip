// Host-only stand-in for the HIP runtime, for checking libwaveholtz's host code on a
// machine without a GPU.  The library's sources are compiled host-only (no device code)
// with AddressSanitizer and UBSan and linked against this file instead of libamdhip64.
//
// "Device" memory is ordinary host memory that the driver program allocates and
// registers (hostcheck_register); copies and fills really run (memcpy / memset, so the
// sanitizer checks both ranges).  Kernels do not run.  Instead every launch is checked:
// for the kernels modelled below, the exact index range each thread of the launch would
// touch through every pointer argument is computed with the kernel's own index formulas
// and must lie inside one registered allocation; the launch geometry must match what the
// kernel assumes (tile grids, partial-sum counts).  A violation prints the launch and
// aborts the program, so the calling test fails with the message.
//
// Scalar read-backs into the pinned block return synthetic values that let the Krylov
// drivers run through several iterations (a residual that shrinks by a fixed factor per
// read-back), so that their loops, look-ahead and replacement logic are exercised too.
#include <cxxabi.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../paper_2606_31842_amd/csrc/wh_batched.h"
#include "../../paper_2606_31842_amd/csrc/wh_fused_kernel.h"

using namespace wh;

namespace {

struct Alloc {
  size_t bytes;
  std::string name;
};
std::map<uintptr_t, Alloc>& allocs() {
  static std::map<uintptr_t, Alloc> m;
  return m;
}
std::map<const void*, void*>& vars() {
  static std::map<const void*, void*> m;
  return m;
}
std::map<const void*, std::string>& kernels() {
  static std::map<const void*, std::string> m;
  return m;
}
uintptr_t g_pinned = 0;
size_t g_pinned_bytes = 0;
long g_launches = 0, g_modelled = 0, g_readbacks = 0, g_timings = 0, g_rb_base = 0;
std::map<std::string, long> g_unmodelled;
unsigned g_seed = 1;
std::string g_current;   // name of the launch being checked

[[noreturn]] void fail(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  fprintf(stderr, "HOSTCHECK FAILURE in %s: ", g_current.c_str());
  vfprintf(stderr, fmt, ap);
  fprintf(stderr, "\n");
  va_end(ap);
  fflush(stderr);
  abort();
}

// the registered allocation containing [p, p + bytes), or fail
void check_range(const void* p, int64_t lo_bytes, int64_t hi_bytes, const char* what) {
  if (hi_bytes <= lo_bytes) return;
  const uintptr_t a = (uintptr_t)p + lo_bytes, b = (uintptr_t)p + hi_bytes;
  if (!p) fail("%s: null pointer accessed at bytes [%lld, %lld)", what, (long long)lo_bytes, (long long)hi_bytes);
  auto& m = allocs();
  auto it = m.upper_bound(a);
  if (it != m.begin()) {
    --it;
    if (a >= it->first && b <= it->first + it->second.bytes) return;
    fail("%s: bytes [%lld, %lld) from %p leave allocation '%s' (%zu bytes at offset %lld)", what,
         (long long)lo_bytes, (long long)hi_bytes, p, it->second.name.c_str(), it->second.bytes,
         (long long)((uintptr_t)p - it->first));
  }
  fail("%s: bytes [%lld, %lld) from %p are in no registered allocation", what, (long long)lo_bytes,
       (long long)hi_bytes, p);
}

// element index range [lo, hi] touched through one pointer
struct Span {
  const void* p = nullptr;
  size_t esz = 8;
  int64_t lo = INT64_MAX, hi = INT64_MIN;
  const char* what = "";
  void touch(int64_t i) {
    if (i < lo) lo = i;
    if (i > hi) hi = i;
  }
  void check() const {
    if (hi < lo) return;
    check_range(p, lo * (int64_t)esz, (hi + 1) * (int64_t)esz, what);
  }
};

template <typename T>
T arg(void** args, int i) {
  T v;
  std::memcpy(&v, args[i], sizeof(T));
  return v;
}

// ------------------------------------------------------------------ name parsing
std::string demangle(const std::string& m) {
  int st = 0;
  char* d = abi::__cxa_demangle(m.c_str(), nullptr, nullptr, &st);
  std::string r = st == 0 && d ? d : m;
  free(d);
  return r;
}
// "void wh::k_fused2d<double, 8, 4, 16, true, false, 0>(wh::FusedDev)" -> base, template args
void parse(const std::string& dm, std::string& base, std::vector<std::string>& targs) {
  size_t s = dm.find("wh::");
  s = s == std::string::npos ? 0 : s + 4;
  size_t e = dm.find_first_of("<(", s);
  base = dm.substr(s, e - s);
  targs.clear();
  if (e != std::string::npos && dm[e] == '<') {
    size_t c = dm.find('>', e);
    std::string in = dm.substr(e + 1, c - e - 1);
    size_t q = 0;
    while (q <= in.size()) {
      size_t k = in.find(',', q);
      if (k == std::string::npos) k = in.size();
      std::string t = in.substr(q, k - q);
      while (!t.empty() && t[0] == ' ') t.erase(0, 1);
      targs.push_back(t);
      q = k + 1;
    }
  }
}
int ti(const std::vector<std::string>& t, size_t i) {
  if (i >= t.size()) fail("missing template argument %zu", i);
  if (t[i] == "true") return 1;
  if (t[i] == "false") return 0;
  return atoi(t[i].c_str());
}
size_t tsize(const std::vector<std::string>& t, size_t i) {
  if (i >= t.size()) fail("missing template argument %zu", i);
  return t[i] == "float" ? 4 : 8;
}

// ------------------------------------------------------------------ kernel models
int xcd_tile_host(int bid, int nb) {
  const int xcd = bid & 7, idx = bid >> 3;
  const int q = nb >> 3, r = nb & 7;
  return xcd < r ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

void model_fused2d(const std::vector<std::string>& t, dim3 g, dim3 b, void** args) {
  const size_t TS = tsize(t, 0);
  const int K = ti(t, 1), R = ti(t, 2), NW = ti(t, 3), VARC = ti(t, 4), FORCE = ti(t, 5), PH = ti(t, 6);
  const FusedDev a = arg<FusedDev>(args, 0);
  const int n = a.n;
  const int64_t P = (int64_t)n + 1;
  const int TXO = 64 - 2 * K, TYO = NW * R - 2 * K;
  if (TXO <= 0 || TYO <= 0) fail("tile too small");
  if ((int)b.x != 64 || (int)b.y != NW || b.z != 1) fail("block (%u,%u,%u) != (64,%d,1)", b.x, b.y, b.z, NW);
  if (a.gx != (n - 1 + TXO - 1) / TXO || a.gy != (n - 1 + TYO - 1) / TYO) fail("tile grid %d x %d wrong", a.gx, a.gy);
  const int nb = a.gx * a.gy;
  if ((int)g.x != nb || g.y != 1 || g.z != 1) fail("grid %u != %d tiles", g.x, nb);
  if (K > 16) fail("K = %d exceeds the weight arrays", K);
  const bool first = PH == kPhaseFirst, lastp = PH == kPhaseLast;
  const bool dirupd = first && a.dr != nullptr;
  Span cur{a.cur, TS}, prv{a.prev, TS}, kap{a.kap, TS}, fs{a.fs, TS}, V{a.V, 8}, vin{a.vin, 8};
  Span dr{a.dr, 8}, dp{a.dp, 8}, dsl{a.dslots, 8}, dout{a.dout, 8}, co{a.cur_out, TS}, po{a.prev_out, TS};
  Span x{a.x, 8}, out{a.out, 8}, part{a.partials, 8};
  cur.what = "cur"; prv.what = "prev"; kap.what = "kap"; fs.what = "fs"; V.what = "V"; vin.what = "vin";
  dr.what = "dr"; dp.what = "dp"; dsl.what = "dslots"; dout.what = "dout"; co.what = "cur_out";
  po.what = "prev_out"; x.what = "x"; out.what = "out"; part.what = "partials";
  std::vector<char> seen(nb, 0);
  if (dirupd) dsl.touch(S_BETA);
  for (int bid = 0; bid < nb; ++bid) {
    const int tt = xcd_tile_host(bid, nb);
    if (tt < 0 || tt >= nb || seen[tt]) fail("XCD tile map is not a permutation (block %d -> %d)", bid, tt);
    seen[tt] = 1;
    const int tx = tt % a.gx, ty = tt / a.gx;
    const int x0 = 1 + tx * TXO, y0 = 1 + ty * TYO;
    const int64_t p_in = (int64_t)y0 * P + x0;
    for (int wv = 0; wv < NW; ++wv)
      for (int lane = 0; lane < 64; ++lane) {
        const int xg = x0 - K + lane, yb = y0 - K + wv * R;
        const bool xin = xg >= 1 && xg <= n - 1;
        const bool xout = lane >= K && lane < 64 - K && xin;
        for (int r = 0; r < R; ++r) {
          const int y = yb + r;
          const bool in = xin && y >= 1 && y <= n - 1;
          const int64_t p = (int64_t)y * P + xg;
          const int ry = wv * R + r;
          const bool o = in && xout && ry >= K && ry < NW * R - K;
          if (!first && in) { cur.touch(p); prv.touch(p); }
          if (o && !first) V.touch(p);
          if (VARC && in) { kap.touch(p); kap.touch(p - 1); kap.touch(p + 1); kap.touch(p - P); kap.touch(p + P); }
          if (FORCE && in) fs.touch(p);
          if (first) {
            const int64_t ps = in ? p : p_in;
            if (dirupd) { dr.touch(ps); dp.touch(ps); if (o) dout.touch(p); }
            else if (a.vin) vin.touch(ps);
          }
          if (PH != kPhaseMid && xg >= 0 && xg <= n && y >= 0 && y <= n && (xg == 0 || xg == n || y == 0 || y == n)) {
            if (first || a.last == M_LAST_V) V.touch(p); else out.touch(p);
          }
          if (!lastp) {
            if (o) { co.touch(p); po.touch(p); V.touch(p); }
          } else {
            if (a.last != M_LAST_V) x.touch(o ? p : p_in);
            if (o) { if (a.last == M_LAST_V) V.touch(p); else out.touch(p); }
          }
        }
        if (lastp && a.last != M_LAST_V && wv == 0 && lane == 0) part.touch(bid);
      }
  }
  for (Span* s : {&cur, &prv, &kap, &fs, &V, &vin, &dr, &dp, &dsl, &dout, &co, &po, &x, &out, &part}) s->check();
}

void model_step2d(const std::vector<std::string>& t, dim3 g, dim3 b, void** args) {
  const size_t TS = tsize(t, 0);
  const int MODE = ti(t, 1), VARC = ti(t, 2), FORCE = ti(t, 3);
  const bool INC = TS == 4;
  const StepArgs a = arg<StepArgs>(args, 0);
  const int n = a.n;
  const int64_t P = (int64_t)n + 1;
  if (b.x != 64 || b.y != 4) fail("block shape");
  if ((int)g.x != (n - 1 + 63) / 64 || (int)g.y != (n - 1 + 15) / 16) fail("grid (%u,%u)", g.x, g.y);
  Span cur{a.cur, TS}, prv{a.prev, TS}, kap{a.kap, TS}, fs{a.fs, TS}, V{a.V, 8}, x{a.x, 8}, out{a.out, 8};
  Span cn{a.cur_next, TS}, part{a.partials, 8};
  cur.what = "cur"; prv.what = "prev"; kap.what = "kap"; fs.what = "fs"; V.what = "V"; x.what = "x";
  out.what = "out"; cn.what = "cur_next"; part.what = "partials";
  for (unsigned by = 0; by < g.y; ++by)
    for (unsigned bx = 0; bx < g.x; ++bx) {
      for (int ty = 0; ty < 4; ++ty)
        for (int tx = 0; tx < 64; ++tx) {
          const int i = 1 + bx * 64 + tx;
          const int j0 = 1 + (by * 4 + ty) * 4;
          if (!(i < n && j0 < n)) continue;
          const int jend = std::min(j0 + 4, n);
          int64_t p = (int64_t)j0 * P + i;
          cur.touch(p - P); cur.touch(p);
          if (VARC) { kap.touch(p - P); kap.touch(p); }
          for (int j = j0; j < jend; ++j, p += P) {
            cur.touch(p + P); cur.touch(p - 1); cur.touch(p + 1); prv.touch(p);
            if (VARC) { kap.touch(p + P); kap.touch(p - 1); kap.touch(p + 1); }
            if (FORCE) fs.touch(p);
            if (INC && MODE == M_MID) { prv.touch(p); cn.touch(p); V.touch(p); continue; }
            switch (MODE) {
              case M_MID: prv.touch(p); V.touch(p); break;
              case M_LAST_V: V.touch(p); break;
              case M_LAST_AQ: case M_LAST_EQ: case M_LAST_FPI: V.touch(p); x.touch(p); out.touch(p); break;
              default: fail("mode %d", MODE);
            }
          }
        }
      if (MODE == M_LAST_AQ || MODE == M_LAST_FPI || MODE == M_LAST_EQ) part.touch(by * g.x + bx);
    }
  for (Span* s : {&cur, &prv, &kap, &fs, &V, &x, &out, &cn, &part}) s->check();
}

// 3D streaming step: (64, 4) threads per block over (x, y), 8 planes per thread in z
void model_step3d(const std::vector<std::string>& t, dim3 g, dim3 b, void** args) {
  const size_t TS = tsize(t, 0);
  const int MODE = ti(t, 1), VARC = ti(t, 2), FORCE = ti(t, 3);
  const bool INC = TS == 4;
  const StepArgs a = arg<StepArgs>(args, 0);
  const int n = a.n;
  const int64_t P = (int64_t)n + 1, P2 = P * P;
  constexpr int RB = 8;
  if (b.x != 64 || b.y != 4) fail("block shape");
  if ((int)g.x != (n - 1 + 63) / 64 || (int)g.y != (n - 1 + 3) / 4 || (int)g.z != (n - 1 + RB - 1) / RB)
    fail("grid (%u,%u,%u) for n = %d", g.x, g.y, g.z, n);
  Span cur{a.cur, TS}, prv{a.prev, TS}, kap{a.kap, TS}, fs{a.fs, TS}, V{a.V, 8}, x{a.x, 8}, out{a.out, 8};
  Span cn{a.cur_next, TS}, part{a.partials, 8};
  cur.what = "cur"; prv.what = "prev"; kap.what = "kap"; fs.what = "fs"; V.what = "V"; x.what = "x";
  out.what = "out"; cn.what = "cur_next"; part.what = "partials";
  for (unsigned bz = 0; bz < g.z; ++bz)
    for (unsigned by = 0; by < g.y; ++by)
      for (unsigned bx = 0; bx < g.x; ++bx) {
        for (int ty = 0; ty < 4; ++ty)
          for (int tx = 0; tx < 64; ++tx) {
            const int i = 1 + bx * 64 + tx, j = 1 + by * 4 + ty, k0 = 1 + bz * RB;
            if (!(i < n && j < n && k0 < n)) continue;
            const int kend = std::min(k0 + RB, n);
            for (int k = k0; k < kend; ++k) {
              const int64_t p = (int64_t)k * P2 + (int64_t)j * P + i;
              for (int64_t o : {-P2, -P, (int64_t)-1, (int64_t)0, (int64_t)1, P, P2}) {
                cur.touch(p + o);
                if (VARC) kap.touch(p + o);
              }
              prv.touch(p);
              if (FORCE) fs.touch(p);
              V.touch(p);
              if (MODE == M_MID) {
                if (INC) cn.touch(p);
              } else if (MODE == M_LAST_AQ || MODE == M_LAST_EQ || MODE == M_LAST_FPI) {
                x.touch(p); out.touch(p);
              } else if (MODE != M_LAST_V) {
                fail("mode %d", MODE);
              }
            }
          }
        if (MODE == M_LAST_AQ || MODE == M_LAST_FPI || MODE == M_LAST_EQ) part.touch((bz * g.y + by) * g.x + bx);
      }
  for (Span* sp : {&cur, &prv, &kap, &fs, &V, &x, &out, &cn, &part}) sp->check();
}

void model_first(const std::vector<std::string>& t, dim3 g, dim3, void** args) {
  const size_t TS = tsize(t, 0);
  const int DIM = ti(t, 1), VARC = ti(t, 2), FORCE = ti(t, 3);
  const StepArgs a = arg<StepArgs>(args, 0);
  const int n = a.n;
  const int64_t P = (int64_t)n + 1, N = DIM == 2 ? P * P : P * P * P;
  if ((int64_t)g.x * 256 < N) fail("grid covers %lld of %lld nodes", (long long)g.x * 256, (long long)N);
  Span w0{a.prev, TS}, w1{a.cur_out, TS}, z0{a.zb0, TS}, z1{a.zb1, TS}, V{a.V, 8}, v{a.vin, 8}, kap{a.kap, TS},
      fs{a.fs, TS};
  w0.what = "prev"; w1.what = "cur_out"; z0.what = "zb0"; z1.what = "zb1"; V.what = "V"; v.what = "vin";
  kap.what = "kap"; fs.what = "fs";
  for (int64_t p = 0; p < N; ++p) {
    const int i = (int)(p % P), j = (int)((p / P) % P), k = DIM == 3 ? (int)(p / (P * P)) : 1;
    const bool interior = i > 0 && i < n && j > 0 && j < n && (DIM == 2 || (k > 0 && k < n));
    w0.touch(p); w1.touch(p); V.touch(p);
    if (!interior) { if (a.zb0) z0.touch(p); if (a.zb1) z1.touch(p); continue; }
    if (FORCE) fs.touch(p);
    if (!a.vin) continue;
    v.touch(p);
    if (i > 1) v.touch(p - 1);
    if (i < n - 1) v.touch(p + 1);
    if (j > 1) v.touch(p - P);
    if (j < n - 1) v.touch(p + P);
    if (DIM == 3) { if (k > 1) v.touch(p - P * P); if (k < n - 1) v.touch(p + P * P); }
    if (VARC) {
      kap.touch(p); kap.touch(p - 1); kap.touch(p + 1); kap.touch(p - P); kap.touch(p + P);
      if (DIM == 3) { kap.touch(p - P * P); kap.touch(p + P * P); }
    }
  }
  for (Span* s : {&w0, &w1, &z0, &z1, &V, &v, &kap, &fs}) s->check();
}

void model_fwd_out2d(dim3 g, dim3 b, void** args) {
  const double* cur = arg<const double*>(args, 0);
  const double* prev = arg<const double*>(args, 1);
  double* out = arg<double*>(args, 2);
  const double* kap = arg<const double*>(args, 3);
  const double* fs = arg<const double*>(args, 4);
  const int first = arg<int>(args, 6), n = arg<int>(args, 7);
  const int64_t P = (int64_t)n + 1;
  Span C{cur, 8, INT64_MAX, INT64_MIN, "cur"}, Pv{prev, 8, INT64_MAX, INT64_MIN, "prev"},
      O{out, 8, INT64_MAX, INT64_MIN, "out"}, Kp{kap, 8, INT64_MAX, INT64_MIN, "kap"},
      F{fs, 8, INT64_MAX, INT64_MIN, "fs"};
  if (b.x != 64 || b.y != 4) fail("block shape");
  for (unsigned by = 0; by < g.y; ++by)
    for (unsigned bx = 0; bx < g.x; ++bx)
      for (int ty = 0; ty < 4; ++ty)
        for (int tx = 0; tx < 64; ++tx) {
          const int i = 1 + bx * 64 + tx, j = 1 + by * 4 + ty;
          if (i >= n || j >= n) continue;
          const int64_t p = (int64_t)j * P + i;
          for (int64_t q : {p, p - 1, p + 1, p - P, p + P}) { C.touch(q); Kp.touch(q); }
          if (fs) F.touch(p);
          if (!first) Pv.touch(p);
          O.touch(p);
        }
  if ((int)g.x * 64 < n - 1 || (int)g.y * 4 < n - 1) fail("grid does not cover the interior");
  for (Span* s : {&C, &Pv, &O, &Kp, &F}) s->check();
}

void model_adj_step2d(dim3 g, dim3 b, void** args) {
  const double* lam1 = arg<const double*>(args, 0);
  const double* lam2 = arg<const double*>(args, 1);
  double* lout = arg<double*>(args, 2);
  const double* W = arg<const double*>(args, 3);
  const double* kap = arg<const double*>(args, 4);
  const double* z = arg<const double*>(args, 5);
  double* grad = arg<double*>(args, 8);
  const int do_lam = arg<int>(args, 9), n = arg<int>(args, 10);
  const int64_t P = (int64_t)n + 1;
  Span L1{lam1, 8, INT64_MAX, INT64_MIN, "lam1"}, L2{lam2, 8, INT64_MAX, INT64_MIN, "lam2"},
      LO{lout, 8, INT64_MAX, INT64_MIN, "lam_out"}, WW{W, 8, INT64_MAX, INT64_MIN, "W"},
      Kp{kap, 8, INT64_MAX, INT64_MIN, "kap"}, Z{z, 8, INT64_MAX, INT64_MIN, "z"},
      G{grad, 8, INT64_MAX, INT64_MIN, "grad"};
  if (b.x != 64 || b.y != 4) fail("block shape");
  for (unsigned by = 0; by < g.y; ++by)
    for (unsigned bx = 0; bx < g.x; ++bx)
      for (int ty = 0; ty < 4; ++ty)
        for (int tx = 0; tx < 64; ++tx) {
          const int i = bx * 64 + tx, j = by * 4 + ty;
          if (i > n || j > n) continue;
          const int64_t p = (int64_t)j * P + i;
          L1.touch(p); WW.touch(p); G.touch(p);
          if (i > 0) { L1.touch(p - 1); WW.touch(p - 1); }
          if (i < n) { L1.touch(p + 1); WW.touch(p + 1); }
          if (j > 0) { L1.touch(p - P); WW.touch(p - P); }
          if (j < n) { L1.touch(p + P); WW.touch(p + P); }
          if (do_lam && i > 0 && i < n && j > 0 && j < n) {
            for (int64_t q : {p, p - 1, p + 1, p - P, p + P}) Kp.touch(q);
            L2.touch(p); Z.touch(p); LO.touch(p);
          }
        }
  if ((int)g.x * 64 < n + 1 || (int)g.y * 4 < n + 1) fail("grid does not cover the grid");
  for (Span* s : {&L1, &L2, &LO, &WW, &Kp, &Z, &G}) s->check();
}


// ---- batched solver: the plan kernel is emulated (so that the work kernels see a real plan)
// and every work item's tile is checked against its problem's arrays
int batch_class(const BDesc& d, const BState& st) {
  if (st.phase == BP_DONE) return -1;
  const int prec = phase_prec(st.phase, d.mixed && !st.force64);
  const bool stepping = st.phase != BP_INIT && st.phase != BP_UPD1 && st.phase != BP_UPD2;
  return (stepping && prec == 1) ? 1 : 0;
}

// control: one block per problem reduces that problem's tile partials and updates its state
void model_batch_control(dim3 g, dim3 b, void** args) {
  const BDesc* descs = arg<const BDesc*>(args, 0);
  const BState* states = arg<const BState*>(args, 1);
  const int K = arg<int>(args, 2);
  const int nb = (int)g.x;
  if (b.x != 256 || g.y != 1) fail("control launch shape");
  if (K < 1 || K > 8) fail("steps per launch %d", K);
  check_range(descs, 0, (int64_t)sizeof(BDesc) * nb, "descs");
  check_range(states, 0, (int64_t)sizeof(BState) * nb, "states");
  for (int i = 0; i < nb; ++i)
    check_range(descs[i].partials, 0, 8LL * descs[i].ntx * descs[i].nty, "tile partials");
}

// count of unfinished problems (one block)
void model_batch_count(dim3 g, dim3 b, void** args) {
  const int nb = arg<int>(args, 1);
  if (g.x != 1 || b.x != 256) fail("count launch shape");
  check_range(arg<const BState*>(args, 0), 0, (int64_t)sizeof(BState) * nb, "states");
  check_range(arg<int*>(args, 2), 0, 4, "counter");
}

void model_batch_plan(dim3 g, dim3 b, void** args) {
  const BDesc* descs = arg<const BDesc*>(args, 0);
  const BState* states = arg<const BState*>(args, 1);
  const int nb = arg<int>(args, 2);
  int* plan = arg<int*>(args, 3);
  if (g.x != 1 || b.x != 256) fail("plan launch shape");
  check_range(descs, 0, (int64_t)sizeof(BDesc) * nb, "descs");
  check_range(states, 0, (int64_t)sizeof(BState) * nb, "states");
  check_range(plan, 0, 4LL * (2 * plan_stride(nb) + 16), "plan");
  int tiles[2] = {0, 0}, act[2] = {0, 0};
  for (int i = 0; i < nb; ++i) {
    const int c = batch_class(descs[i], states[i]);
    if (c < 0) continue;
    int* pl = plan + c * plan_stride(nb);
    pl[2 + act[c]] = i;
    pl[2 + nb + act[c]] = tiles[c];
    act[c]++;
    tiles[c] += descs[i].ntx * descs[i].nty;
  }
  for (int c = 0; c < 2; ++c) {
    int* pl = plan + c * plan_stride(nb);
    pl[0] = tiles[c];
    pl[1] = act[c];
    pl[2 + nb + act[c]] = tiles[c];
  }
  for (int k = 0; k < 16; ++k) plan[2 * plan_stride(nb) + k] = 0;
}

void check_batch_item(const BDesc* descs, const BState* states, int nb, int sid, int lt, int want, int K,
                      int VARC, int it) {
  const int TXO = batch_txo(K), TYO = batch_tyo();
      if (sid < 0 || sid >= nb) fail("item %d maps to problem %d", it, sid);
      const BDesc& d = descs[sid];
      const BState& st = states[sid];
      if (batch_class(d, st) != want) fail("item %d of problem %d is in the other class", it, sid);
      if (lt < 0 || lt >= d.ntx * d.nty) fail("item %d: tile %d of problem %d out of %d", it, lt, sid, d.ntx * d.nty);
      const int n = d.n;
      const int64_t P = (int64_t)n + 1, N = P * P;
      const int x0 = 1 + (lt % d.ntx) * TXO, y0 = 1 + (lt / d.ntx) * TYO;
      if (x0 > n - 1 || y0 > n - 1) fail("tile origin (%d, %d) outside the grid n = %d", x0, y0, n);
      // nodes the phase can touch: the tile with its K-point halo (the strips' halo columns,
      // the pipeline's rows before and after the tile) clipped to the interior, and their
      // neighbours
      const int ya = std::max(1, y0 - K), yb = std::min(n - 1, y0 + TYO + K - 1);
      const int xa = std::max(1, x0 - K), xb = std::min(n - 1, x0 + TXO + K - 1);
      const int64_t lo_i = (int64_t)(ya - 1) * P + xa - 1, hi_i = (int64_t)(yb + 1) * P + xb + 1;
      if (lo_i < 0 || hi_i >= N) fail("tile node range [%lld, %lld] outside 0..%lld", (long long)lo_i,
                                      (long long)hi_i, (long long)N - 1);
      const size_t TS = want == 1 ? 4 : 8;
      auto arr = [&](const void* ptr, size_t esz, const char* what) {
        if (ptr) check_range(ptr, lo_i * (int64_t)esz, (hi_i + 1) * (int64_t)esz, what);
      };
      arr(d.x, 8, "x"); arr(d.b, 8, "b"); arr(d.r, 8, "r"); arr(d.p, 8, "p"); arr(d.q, 8, "q"); arr(d.V, 8, "V");
      if (TS == 8) {
        for (int k = 0; k < 4; ++k) arr(d.W[k], 8, "state");
      } else {
        // FP32 pairs: interleaved (slot 2k+1 starts the pair's array, slot 2k is 4 bytes further,
        // node i of either slot at 8 i; only where no FP32 step is forced) or four arrays
        for (int k = 0; k < 2; ++k) {
          if ((const char*)d.W32[2 * k] == (const char*)d.W32[2 * k + 1] + 4) {
            if (d.defect) fail("FP32 pair %d interleaved in a batch with forced steps", k);
            check_range(d.W32[2 * k + 1], lo_i * 8, (hi_i + 1) * 8, "state pair");
          } else {
            arr(d.W32[2 * k], 4, "state"); arr(d.W32[2 * k + 1], 4, "state");
          }
        }
      }
      if (VARC) arr(TS == 8 ? (const void*)d.kap64 : (const void*)d.kap32, TS, "kap");
      arr(TS == 8 ? (const void*)d.fs64 : (const void*)d.fs32, TS, "fs");
      check_range(d.partials, 8LL * lt, 8LL * (lt + 1), "partials");
      check_range(d.w, 0, 8LL * (d.nt + 1), "weights");
      check_range(d.cosv, 0, 8LL * (d.nt + 1), "cosines");
      if (st.phase == BP_A_STEP || st.phase == BP_B_STEP || st.phase == BP_R_STEP) {
        const int Kp = std::min(K, d.nt - 1 - st.step);
        if (Kp < 1 || st.step + Kp > d.nt) fail("step %d + %d beyond N_t = %d", st.step, Kp, d.nt);
      }
}

void model_batch_work(const std::vector<std::string>& t, dim3 g, dim3 b, void** args) {
  const int K = ti(t, 1), VARC = ti(t, 2), NW = kBW;
  const BDesc* descs = arg<const BDesc*>(args, 0);
  const BState* states = arg<const BState*>(args, 1);
  const int* plan = arg<const int*>(args, 2);
  const int nb = arg<int>(args, 3), want = arg<int>(args, 4);
  if (g.x % 8 != 0 || g.x == 0) fail("persistent grid %u is not a positive multiple of 8", g.x);
  (void)g;
  if ((int)b.x != 64 || (int)b.y != NW) fail("block shape");
  const int* pl = plan + want * plan_stride(nb);
  const int total = pl[0], nact = pl[1];
  if (nact < 0 || nact > nb || total < 0) fail("plan header (%d tiles, %d problems)", total, nact);
  const int* pid = pl + 2;
  const int* start = pl + 2 + nb;
  std::vector<int> hit(total, 0);
  check_range(plan + 2 * plan_stride(nb) + 8 * want, 0, 32, "item counters");
  // items are taken dynamically from the 8 chunk counters; every item of [0, total) is taken once
  for (int c = 0; c < 8; ++c) {
    const int c0 = (int)((int64_t)total * c / 8), c1 = (int)((int64_t)total * (c + 1) / 8);
    for (int it = c0; it < c1; ++it) {
      int lo = 0, hi = nact - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= it) lo = mid;
        else hi = mid - 1;
      }
      hit[it]++;
      check_batch_item(descs, states, nb, pid[lo], it - start[lo], want, K, VARC, it);
    }
  }
  for (int i = 0; i < total; ++i)
    if (hit[i] != 1) fail("work item %d visited %d times", i, hit[i]);
}

void model_batch_tile(const std::vector<std::string>& t, dim3 g, dim3 b, void** args) {
  const int K = ti(t, 1), VARC = ti(t, 2), NW = kBW;
  const BDesc* descs = arg<const BDesc*>(args, 0);
  const BState* states = arg<const BState*>(args, 1);
  const int* tiles = arg<const int*>(args, 2);
  const int ntiles = arg<int>(args, 3), want = arg<int>(args, 4);
  if ((int)g.x != ntiles) fail("grid %u != %d tiles", g.x, ntiles);
  if ((int)b.x != 64 || (int)b.y != NW) fail("block shape");
  check_range(tiles, 0, 4LL * ntiles, "tile table");
  std::vector<char> seen(ntiles, 0);
  int nb = 0;
  for (int i = 0; i < ntiles; ++i) nb = std::max(nb, tiles[i] + 1);
  for (int bid = 0; bid < ntiles; ++bid) {
    const int gt = xcd_tile_host(bid, ntiles);
    if (gt < 0 || gt >= ntiles || seen[gt]) fail("XCD tile map is not a permutation");
    seen[gt] = 1;
    const int sid = tiles[gt];
    const BDesc& d = descs[sid];
    const BState& st = states[sid];
    if (batch_class(d, st) != want) continue;
    if (gt < d.tile0 || gt >= d.tile0 + d.ntx * d.nty) fail("tile %d outside problem %d's range", gt, sid);
    check_batch_item(descs, states, nb, sid, gt - d.tile0, want, K, VARC, gt);
  }
}

void vec(const void* p, int64_t count, size_t esz, const char* what) {
  if (p && count > 0) check_range(p, 0, count * (int64_t)esz, what);
}

bool model_generic(const std::string& base, const std::vector<std::string>& t, dim3 g, dim3, void** args) {
  const int64_t G = g.x;
  if (base == "k_prep") {
    const size_t TS = tsize(t, 0);
    const int64_t N = arg<int64_t>(args, 6);
    const double* c2 = arg<const double*>(args, 0);
    const double* f = arg<const double*>(args, 1);
    vec(c2, N, 8, "c2"); vec(f, N, 8, "f");
    if (c2) vec(arg<void*>(args, 2), N, TS, "kap");
    if (f) vec(arg<void*>(args, 3), N, TS, "fs");
  } else if (base == "k_zero_boundary") {
    vec(arg<void*>(args, 0), arg<int64_t>(args, 3), 8, "u");
  } else if (base == "k_defect") {
    const int64_t N = arg<int64_t>(args, 7);
    vec(arg<void*>(args, 0), N, 8, "v"); vec(arg<void*>(args, 1), N, 8, "kap");
    vec(arg<void*>(args, 4), N, tsize(t, 0), "fs");
  } else if (base == "k_max_partials") {
    vec(arg<void*>(args, 0), arg<int64_t>(args, 1), 8, "a"); vec(arg<void*>(args, 2), G, 8, "partials");
  } else if (base == "k_max_finalize") {
    vec(arg<void*>(args, 0), arg<int>(args, 1), 8, "partials"); vec(arg<void*>(args, 2), 1, 8, "out");
  } else if (base == "k_dot_partials") {
    const int64_t N = arg<int64_t>(args, 2);
    vec(arg<void*>(args, 0), N, 8, "a"); vec(arg<void*>(args, 1), N, 8, "b");
    vec(arg<void*>(args, 3), G, 8, "partials");
  } else if (base == "k_reduce") {
    vec(arg<void*>(args, 0), arg<int>(args, 1), 8, "partials");
    const int dst = arg<int>(args, 3), mode = arg<int>(args, 4);
    vec(arg<void*>(args, 2), mode == 0 ? dst + 1 : 4, 8, "slots");
  } else if (base == "k_set_beta") {
    vec(arg<void*>(args, 0), std::max(arg<int>(args, 1), 3) + 1, 8, "slots");
  } else if (base == "k_cg_update1") {
    const int64_t N = arg<int64_t>(args, 5);
    for (int i = 0; i < 4; ++i) vec(arg<void*>(args, i), N, 8, "vector");
    vec(arg<void*>(args, 4), 4, 8, "slots"); vec(arg<void*>(args, 6), G, 8, "partials");
    vec(arg<void*>(args, 7), arg<int>(args, 8), 8, "pq_parts");
  } else if (base == "k_cg_update2") {
    const int64_t N = arg<int64_t>(args, 3);
    vec(arg<void*>(args, 0), N, 8, "p"); vec(arg<void*>(args, 1), N, 8, "r"); vec(arg<void*>(args, 2), 4, 8, "slots");
  } else if (base == "k_cg_update2_to") {
    const int64_t N = arg<int64_t>(args, 4);
    for (int i = 0; i < 3; ++i) vec(arg<void*>(args, i), N, 8, "vector");
    vec(arg<void*>(args, 3), 4, 8, "slots");
  } else if (base == "k_axpy_slot") {
    const int64_t N = arg<int64_t>(args, 5);
    vec(arg<void*>(args, 0), N, 8, "y"); vec(arg<void*>(args, 1), N, 8, "x");
    vec(arg<void*>(args, 2), arg<int>(args, 3) + 1, 8, "slots");
  } else if (base == "k_axpy") {
    const int64_t N = arg<int64_t>(args, 3);
    vec(arg<void*>(args, 0), N, 8, "y"); vec(arg<void*>(args, 1), N, 8, "x");
  } else if (base == "k_lincomb3") {
    const int64_t N = arg<int64_t>(args, 7);
    for (int i : {0, 2, 4, 6}) vec(arg<void*>(args, i), N, 8, "vector");
  } else if (base == "k_scale_copy") {
    const int64_t N = arg<int64_t>(args, 4);
    vec(arg<void*>(args, 0), N, 8, "y"); vec(arg<void*>(args, 1), N, 8, "x");
    vec(arg<void*>(args, 2), arg<int>(args, 3) + 1, 8, "slots");
  } else if (base == "k_sub") {
    const int64_t N = arg<int64_t>(args, 3);
    for (int i = 0; i < 3; ++i) vec(arg<void*>(args, i), N, 8, "vector");
  } else if (base == "k_copy") {
    const int64_t N = arg<int64_t>(args, 2);
    for (int i = 0; i < 2; ++i) vec(arg<void*>(args, i), N, 8, "vector");
  } else if (base == "k_gemv_acc") {
    const int64_t ldv = arg<int64_t>(args, 2), N = arg<int64_t>(args, 5);
    const int k = arg<int>(args, 3);
    vec(arg<void*>(args, 0), N, 8, "x");
    if (k > 0) vec(arg<void*>(args, 1), (k - 1) * ldv + N, 8, "V");
    vec(arg<void*>(args, 4), k, 8, "y");
  } else if (base == "k_helm_res") {
    const int n = arg<int>(args, 5), dim = arg<int>(args, 6);
    const int64_t P = n + 1, N = dim == 2 ? P * P : P * P * P;
    for (int i = 0; i < 3; ++i) vec(arg<void*>(args, i), N, 8, "vector");
    vec(arg<void*>(args, 8), G, 8, "pr"); vec(arg<void*>(args, 9), G, 8, "pf");
  } else if (base == "k_misfit") {
    const int64_t* idx = arg<const int64_t*>(args, 1);
    const int nrec = arg<int>(args, 3);
    vec(idx, nrec, 8, "rec_idx"); vec(arg<void*>(args, 2), nrec, 8, "d");
    vec(arg<void*>(args, 5), 1, 8, "out");
    Span u{arg<const double*>(args, 0), 8, INT64_MAX, INT64_MIN, "u"}, gg{arg<double*>(args, 4), 8, INT64_MAX, INT64_MIN, "g"};
    for (int k = 0; k < nrec; ++k) { u.touch(idx[k]); gg.touch(idx[k]); }
    u.check(); gg.check();
  } else if (base == "k_small_matvec") {
    const int nd = arg<int>(args, 1), src = arg<int>(args, 3), dst = arg<int>(args, 4);
    if (nd > 1024) fail("n_d = %d beyond the staging array", nd);
    if (!(src + nd <= dst || dst + nd <= src)) fail("source and destination slot ranges overlap");
    vec(arg<void*>(args, 0), (int64_t)nd * nd, 8, "matrix");
    vec(arg<void*>(args, 2), std::max(src, dst) + nd, 8, "slots");
  } else if (base == "k_cols_project") {
    // columns c0 .. c0+KC-1 of V (stride ldv) against r over N points; partials [block][ncols]
    const int KC = ti(t, 0);
    const int64_t ldv = arg<int64_t>(args, 1), N = arg<int64_t>(args, 3);
    const int ncols = arg<int>(args, 2);
    if (ncols < 1 || (int)g.y != (ncols + KC - 1) / KC) fail("%d columns in %u chunks of %d", ncols, g.y, KC);
    if (ldv < N) fail("column stride %lld below N = %lld", (long long)ldv, (long long)N);
    vec(arg<void*>(args, 0), (int64_t)(ncols - 1) * ldv + N, 8, "V");
    vec(arg<void*>(args, 4), N, 8, "r");
    vec(arg<void*>(args, 5), (int64_t)g.x * ncols, 8, "partials");
  } else if (base == "k_dense_combine") {
    const int64_t ldv = arg<int64_t>(args, 1), N = arg<int64_t>(args, 3);
    const int nd = arg<int>(args, 2), aslot = arg<int>(args, 6), src = arg<int>(args, 10);
    if (nd > 0) vec(arg<void*>(args, 0), (int64_t)(nd - 1) * ldv + N, 8, "V");
    vec(arg<void*>(args, 4), N, 8, "y");
    vec(arg<void*>(args, 7), N, 8, "r");
    const double* slots = arg<const double*>(args, 9);
    if (nd > 0) check_range(slots, 8LL * src, 8LL * (src + nd), "coefficient slots");
    if (aslot >= 0) check_range(slots, 8LL * aslot, 8LL * (aslot + 1), "alpha slot");
  } else if (base == "k_gs_sub" || base == "k_gs_update") {
    // w -= V h over the first nv columns (stride N); k_gs_update holds h in KC registers
    const int64_t N = arg<int64_t>(args, 1);
    const int nv = arg<int>(args, 2), hsrc = arg<int>(args, 4);
    if (base == "k_gs_update" && nv > ti(t, 0)) fail("%d columns beyond the %d registers", nv, ti(t, 0));
    vec(arg<void*>(args, 0), (int64_t)nv * N, 8, "basis");
    check_range(arg<const double*>(args, 3), 8LL * hsrc, 8LL * (hsrc + nv), "h slots");
    vec(arg<void*>(args, 5), N, 8, "w");
    if (base == "k_gs_update") {
      const bool proj = ti(t, 1) != 0;
      vec(arg<void*>(args, 6), (int64_t)g.x * (proj ? nv + 1 : 1), 8, "partials");
    }
  } else if (base == "k_terms_to_modes") {
    const int* toff = arg<const int*>(args, 1);
    const int nd = arg<int>(args, 2), dst = arg<int>(args, 4);
    vec(toff, nd + 1, 4, "term offsets");
    for (int k = 0; k < nd; ++k)
      if (toff[k + 1] < toff[k]) fail("term offsets decrease at %d", k);
    vec(arg<void*>(args, 0), toff[nd], 8, "term sums");
    check_range(arg<const double*>(args, 3), 8LL * dst, 8LL * (dst + nd), "slots");
    vec(arg<void*>(args, 5), nd, 8, "scale");
  } else if (base == "k_modes_to_terms") {
    const int* tmap = arg<const int*>(args, 1);
    const int nt = arg<int>(args, 2);
    vec(tmap, nt, 4, "term map");
    int mx = -1;
    for (int q = 0; q < nt; ++q) mx = std::max(mx, tmap[q]);
    vec(arg<void*>(args, 0), mx + 1, 8, "mode coefficients");
    vec(arg<void*>(args, 3), nt, 8, "term coefficients");
  } else if (base == "k_sine_tables") {
    // tab[(k dim + axis)(n + 1) + i] for every k < nd, axis < dim, i <= n; modes[k dim + axis]
    const int nd = arg<int>(args, 2), dim = arg<int>(args, 3), n = arg<int>(args, 4);
    const int64_t total = (int64_t)nd * dim * (n + 1);
    if (nd < 1 || (dim != 2 && dim != 3) || n < 2) fail("nd %d dim %d n %d", nd, dim, n);
    vec(arg<void*>(args, 0), total, 8, "tab");
    vec(arg<void*>(args, 1), (int64_t)nd * dim, 4, "modes");
  } else if (base == "k_sine_project" || base == "k_sine_combine") {
    // 64 columns x 32 rows per block over the rows of length n + 1 (2D: n + 1 rows, 3D: (n + 1)^2)
    const int nd = arg<int>(args, 1), dim = arg<int>(args, 2), n = arg<int>(args, 3);
    const int64_t P = n + 1, rows = dim == 2 ? P : P * P;
    if ((int64_t)g.x != (P + 63) / 64 || (int64_t)g.y != (rows + 31) / 32 || g.z != 1)
      fail("grid (%u, %u) for n = %d, dim = %d", g.x, g.y, n, dim);
    if (nd < 1) fail("nd = %d", nd);
    vec(arg<void*>(args, 0), (int64_t)nd * dim * P, 8, "tab");
    if (base == "k_sine_project") {
      vec(arg<void*>(args, 4), rows * P, 8, "r");
      vec(arg<void*>(args, 5), (int64_t)g.x * g.y * nd, 8, "partials");
    } else {
      vec(arg<void*>(args, 4), rows * P, 8, "y");
      vec(arg<void*>(args, 6), 1, 8, "alpha slot");
      vec(arg<void*>(args, 7), rows * P, 8, "r");
      vec(arg<void*>(args, 9), nd, 8, "coef");
    }
  } else if (base == "k_defl_reduce") {
    const int count = arg<int>(args, 1), nd = arg<int>(args, 2), dst = arg<int>(args, 4);
    if ((int)g.x != nd) fail("grid %u for %d slots", g.x, nd);
    vec(arg<void*>(args, 0), (int64_t)count * nd, 8, "partials");
    double* slots = arg<double*>(args, 3);
    if (slots) check_range(slots, 8LL * dst, 8LL * (dst + nd), "slots");
    vec(arg<void*>(args, 5), nd, 8, "scale");
  } else if (base == "k_check_idx") {
    vec(arg<void*>(args, 0), arg<int>(args, 1), 8, "rec_idx"); vec(arg<void*>(args, 3), 1, 4, "bad");
  } else {
    return false;
  }
  return true;
}

// Fourth-order single step: one thread per node of the (n+1)^dim grid (p < N guard), so every
// array the mode uses must hold N elements; partial sums one per block in the epilogues.
void model_step4(const std::vector<std::string>& t, dim3 g, dim3 b, void** args) {
  const size_t TS = tsize(t, 0);
  const int DIM = ti(t, 1), MODE = ti(t, 2), FORCE = ti(t, 3);
  const StepArgs a = arg<StepArgs>(args, 0);
  const int64_t P = (int64_t)a.n + 1, N = DIM == 2 ? P * P : P * P * P;
  if (b.x != 256 || b.y != 1) fail("block shape (%u,%u)", b.x, b.y);
  if ((int64_t)g.x != (N + 255) / 256) fail("grid %u for %lld nodes", g.x, (long long)N);
  if (a.n < 4) fail("n = %d", a.n);
  if (FORCE) vec(a.fs, N, TS, "fs");
  vec(a.V, N, 8, "V");
  if (MODE == M_FIRST) {
    vec(a.prev, N, TS, "prev"); vec(a.cur_out, N, TS, "cur_out");
    vec(a.zb0, N, TS, "zb0"); vec(a.zb1, N, TS, "zb1"); vec(a.vin, N, 8, "vin");
    return;
  }
  vec(a.cur, N, TS, "cur"); vec(a.prev, N, TS, "prev");
  if (MODE == M_MID) {
    if (TS == 4) vec(a.cur_next, N, TS, "cur_next");
    return;
  }
  if (MODE == M_LAST_AQ || MODE == M_LAST_FPI || MODE == M_LAST_EQ) {
    vec(a.x, N, 8, "x"); vec(a.out, N, 8, "out");
    if (!a.partials) fail("no partials");
    vec(a.partials, g.x, 8, "partials");
  }
}

// K-step 3D launch: a block of NW wavefronts owns a 64 x NW R column tile of a z-run of zs planes
// with a K-point halo; every access is guarded to the (n+1)^3 grid, so the model checks the tile
// grid against the Fused3Dev fields and that each array holds the grid.
void model_fused3d(const std::vector<std::string>& t, dim3 g, dim3 b, void** args) {
  const size_t TS = tsize(t, 0);
  const int K = ti(t, 1), R = ti(t, 2), NW = ti(t, 3), VARC = ti(t, 4), FORCE = ti(t, 5);
  const Fused3Dev d = arg<Fused3Dev>(args, 0);
  const int n = d.n;
  if ((int)b.x != 64 || (int)b.y != NW) fail("block (%u,%u) for %d waves", b.x, b.y, NW);
  if (K < 2 || K > 3) fail("K = %d", K);
  const int txo = 64 - 2 * K, tyo = NW * R - 2 * K;
  if (d.gx != (n - 1 + txo - 1) / txo || d.gy != (n - 1 + tyo - 1) / tyo) fail("tile grid %d x %d", d.gx, d.gy);
  if (d.zs < 1 || d.gz != (n - 1 + d.zs - 1) / d.zs) fail("z-runs: %d of %d planes", d.gz, d.zs);
  if ((int64_t)g.x != (int64_t)d.gx * d.gy * d.gz || g.y != 1) fail("grid %u for %d tiles", g.x, d.gx * d.gy * d.gz);
  const int64_t P = (int64_t)n + 1, N = P * P * P;
  vec(d.cur, N, TS, "cur"); vec(d.prev, N, TS, "prev");
  vec(d.cur_out, N, TS, "cur_out"); vec(d.prev_out, N, TS, "prev_out");
  vec(d.V, N, 8, "V");
  if (VARC) vec(d.kap, N, TS, "kap");
  if (FORCE) vec(d.fs, N, TS, "fs");
  if (d.cur_out == d.cur || d.prev_out == d.prev) fail("the launch writes a state array that it reads");
}

// Blocked fourth-order launch: K steps of a 2D single solve by the row-marching pipeline.
// Every access goes through a buffer resource sized to the (n+1)^2 grid, so the model checks
// that each pointer holds the whole grid, and that the grid and block match the tiling.
void model_march4(const std::vector<std::string>& t, dim3 g, dim3 b, void** args) {
  const size_t TS = t.at(0) == "float" ? 4 : 8;
  const int K = ti(t, 1);
  const March4Args a = arg<March4Args>(args, 0);
  if (!march4_supported(K)) fail("K = %d has no blocked fourth-order kernel", K);
  if (a.kp < 1 || a.kp > K) fail("steps per launch %d outside 1..%d", a.kp, K);
  if (a.n < 2) fail("n = %d", a.n);
  const int nt = march4_tiles_x(a.n, K) * march4_tiles_y(a.n);
  if ((int)g.x != nt || g.y != 1) fail("grid %u != %d tiles", g.x, nt);
  if ((int)b.x != 64 || (int)b.y != 4) fail("block shape (%u,%u)", b.x, b.y);
  // the strips of the last tile column start inside the grid or return at once; every
  // interior column is covered by exactly one strip
  const int strip = march4_strip(K);
  if ((int64_t)march4_tiles_x(a.n, K) * 4 * strip < a.n - 1) fail("strips do not cover the columns");
  if ((int64_t)march4_tiles_y(a.n) * 32 < a.n - 1) fail("tiles do not cover the rows");
  const int64_t N = (int64_t)(a.n + 1) * (a.n + 1);
  vec(a.cur, N, TS, "cur"); vec(a.prev, N, TS, "prev");
  vec(a.cur_out, N, TS, "cur_out"); vec(a.prev_out, N, TS, "prev_out");
  vec(a.V, N, 8, "V");
  if (a.fs) vec(a.fs, N, TS, "fs");
  if (a.cur_out == a.cur || a.prev_out == a.prev || a.cur_out == a.prev || a.prev_out == a.cur)
    fail("the launch writes a state array that it reads");
}

void check_launch(const void* fn, dim3 g, dim3 b, void** args) {
  ++g_launches;
  auto it = kernels().find(fn);
  if (it == kernels().end()) fail("launch of an unregistered kernel handle %p", fn);
  g_current = demangle(it->second);
  if (g.x == 0 || g.y == 0 || g.z == 0) fail("empty grid (%u,%u,%u)", g.x, g.y, g.z);
  if ((uint64_t)b.x * b.y * b.z > 1024 || b.x == 0) fail("block (%u,%u,%u)", b.x, b.y, b.z);
  std::string base;
  std::vector<std::string> t;
  parse(g_current, base, t);
  bool done = true;
  if (base == "k_fused2d") model_fused2d(t, g, b, args);
  else if (base == "k_step2d") model_step2d(t, g, b, args);
  else if (base == "k_step3d") model_step3d(t, g, b, args);
  else if (base == "k_fused3d") model_fused3d(t, g, b, args);
  else if (base == "k_first") model_first(t, g, b, args);
  else if (base == "k_fwd_out2d") model_fwd_out2d(g, b, args);
  else if (base == "k_adj_step2d") model_adj_step2d(g, b, args);
  else if (base == "k_batch_plan") model_batch_plan(g, b, args);
  else if (base == "k_batch_control") model_batch_control(g, b, args);
  else if (base == "k_batch_count") model_batch_count(g, b, args);
  else if (base == "k_batch_work") model_batch_work(t, g, b, args);
  else if (base == "k_batch_tile") model_batch_tile(t, g, b, args);
  else if (base == "k_march4") model_march4(t, g, b, args);
  else if (base == "k_step4") model_step4(t, g, b, args);
  else done = model_generic(base, t, g, b, args);
  if (done) ++g_modelled;
  else ++g_unmodelled[base];
  g_current.clear();
}

// ------------------------------------------------------------------ launch configuration
struct Cfg {
  dim3 g, b;
  size_t sh;
  hipStream_t s;
};
std::vector<Cfg>& cfgs() {
  static std::vector<Cfg> v;
  return v;
}

double synth(int i, long k) {
  // slots: 0 r.r, 1 p.Ap, 2 alpha, 3 beta, 4 scratch (true residual), 5 ||b||^2, 6 scratch
  const double d = std::pow(0.35, (double)k);
  switch (i) {
    case 0: case 1: case 4: return d;   // p.Ap within the stable-filter bound of r.r
    case 2: case 5: case 6: return 1.0;
    case 3: return 0.5;
    default: return 0.1 * d + 1e-3 * (i % 7);
  }
}

struct Ev {
  int dummy;
};

}  // namespace

// ---------------------------------------------------------------------- program interface
extern "C" {
void hostcheck_register(const void* p, size_t bytes, const char* name) {
  allocs()[(uintptr_t)p] = Alloc{bytes, name ? name : "?"};
}
void hostcheck_unregister(const void* p) { allocs().erase((uintptr_t)p); }
void hostcheck_seed(unsigned s) { g_seed = s; }
// the synthetic residual starts again from 1 (call before each solve)
void hostcheck_restart_residual(void) { g_rb_base = g_readbacks; }
void hostcheck_report(void) {
  fprintf(stdout, "hostcheck: %ld launches, %ld checked by a model, %ld read-backs, %ld timings\n", g_launches,
          g_modelled, g_readbacks, g_timings);
  for (auto& kv : g_unmodelled) fprintf(stdout, "hostcheck: not modelled: %s x%ld\n", kv.first.c_str(), kv.second);
}
}

// ---------------------------------------------------------------------- HIP runtime stand-in
extern "C" {
void** __hipRegisterFatBinary(const void*) {
  static void* h = nullptr;
  return &h;
}
void __hipRegisterFunction(void**, const void* hostFunction, char* deviceFunction, const char*, unsigned int,
                           uint3*, uint3*, dim3*, dim3*, int*) {
  kernels()[hostFunction] = deviceFunction;
}
void __hipUnregisterFatBinary(void**) {}
void __hipRegisterVar(void**, void* var, char*, char* deviceVar, int, size_t size, int, int) {
  // a device variable: its "device copy" is a host block of the same size, registered under
  // its name, returned by hipGetSymbolAddress
  void* p = aligned_alloc(256, (size + 255) / 256 * 256);
  std::memset(p, 0, size);
  vars()[var] = p;
  hostcheck_register(p, size, deviceVar);
}
}

hipError_t __hipPushCallConfiguration(dim3 g, dim3 b, size_t sh, hipStream_t s) {
  cfgs().push_back(Cfg{g, b, sh, s});
  return hipSuccess;
}
hipError_t __hipPopCallConfiguration(dim3* g, dim3* b, size_t* sh, hipStream_t* s) {
  if (cfgs().empty()) fail("pop without push");
  const Cfg c = cfgs().back();
  cfgs().pop_back();
  *g = c.g;
  *b = c.b;
  *sh = c.sh;
  *s = c.s;
  return hipSuccess;
}
hipError_t hipLaunchKernel(const void* f, dim3 g, dim3 b, void** args, size_t, hipStream_t) {
  check_launch(f, g, b, args);
  return hipSuccess;
}

hipError_t hipGetSymbolAddress(void** p, const void* symbol) {
  auto it = vars().find(symbol);
  if (it == vars().end()) return hipErrorInvalidSymbol;
  *p = it->second;
  return hipSuccess;
}
hipError_t hipGetDeviceCount(int* c) {
  *c = 1;
  return hipSuccess;
}
hipError_t hipSetDevice(int d) { return d == 0 ? hipSuccess : hipErrorInvalidDevice; }
hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t a, int) {
  *v = a == hipDeviceAttributeMultiprocessorCount ? 256 : 1;
  return hipSuccess;
}
hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* n, const void*, int, size_t) {
  *n = 2;
  return hipSuccess;
}
hipError_t hipHostMalloc(void** p, size_t bytes, unsigned int) {
  *p = malloc(bytes);
  if (!*p) return hipErrorOutOfMemory;
  g_pinned = (uintptr_t)*p;
  g_pinned_bytes = bytes;
  hostcheck_register(*p, bytes, "pinned host block");
  return hipSuccess;
}
hipError_t hipHostFree(void* p) {
  hostcheck_unregister(p);
  free(p);
  return hipSuccess;
}
hipError_t hipMalloc(void** p, size_t bytes) {
  *p = malloc(bytes);
  if (!*p) return hipErrorOutOfMemory;
  hostcheck_register(*p, bytes, "library device buffer");
  return hipSuccess;
}
hipError_t hipFree(void* p) {
  hostcheck_unregister(p);
  free(p);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind, hipStream_t) {
  if (!bytes) return hipSuccess;
  g_current = "hipMemcpyAsync";
  // device-side ends only: host ends (pageable vectors) are checked by the sanitizer
  if (kind != hipMemcpyDeviceToHost) check_range(dst, 0, (int64_t)bytes, "copy destination");
  if (kind != hipMemcpyHostToDevice) check_range(src, 0, (int64_t)bytes, "copy source");
  g_current.clear();
  std::memcpy(dst, src, bytes);
  if (kind == hipMemcpyDeviceToHost && (uintptr_t)dst == g_pinned && bytes % 8 == 0) {
    ++g_readbacks;
    double* h = (double*)dst;
    for (size_t i = 0; i < bytes / 8; ++i) h[i] = synth((int)i, g_readbacks - g_rb_base);
  }
  return hipSuccess;
}
hipError_t hipMemcpy2DAsync(void* dst, size_t dpitch, const void* src, size_t spitch, size_t width, size_t height,
                            hipMemcpyKind, hipStream_t) {
  g_current = "hipMemcpy2DAsync";
  for (size_t r = 0; r < height; ++r) {
    check_range((char*)dst + r * dpitch, 0, (int64_t)width, "2D copy destination");
    check_range((const char*)src + r * spitch, 0, (int64_t)width, "2D copy source");
    std::memcpy((char*)dst + r * dpitch, (const char*)src + r * spitch, width);
  }
  g_current.clear();
  return hipSuccess;
}
hipError_t hipMemsetAsync(void* dst, int v, size_t bytes, hipStream_t) {
  if (!bytes) return hipSuccess;
  g_current = "hipMemsetAsync";
  check_range(dst, 0, (int64_t)bytes, "fill destination");
  g_current.clear();
  std::memset(dst, v, bytes);
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipGetLastError(void) { return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "stub"; }
hipError_t hipEventCreate(hipEvent_t* e) {
  *e = (hipEvent_t) new Ev{0};
  return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) {
  delete (Ev*)e;
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
  // deterministic, seed-dependent "timings" so that the autotuner's choices vary by seed
  ++g_timings;
  const unsigned h = (unsigned)(g_timings * 2654435761u) ^ (g_seed * 40503u);
  *ms = 0.5f + (float)(h % 1000u) / 1000.0f;
  return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
  *s = (hipStream_t) new Ev{1};
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  delete (Ev*)s;
  return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipSuccess; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t* g) {
  *g = (hipGraph_t) new Ev{2};
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t, hipGraphNode_t*, char*, size_t) {
  *e = (hipGraphExec_t) new Ev{3};
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipSuccess; }
hipError_t hipGraphExecDestroy(hipGraphExec_t e) {
  delete (Ev*)e;
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
  delete (Ev*)g;
  return hipSuccess;
}
