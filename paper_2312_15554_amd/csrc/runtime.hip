// Host runtime behind the C ABI: argument checks, per-cell plans (twiddle and
// symbol tables computed in FP64), workspace, the graph-replayed iteration
// loops and the read-out transforms.
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <stdlib.h>

#include <chrono>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/acm.h"
#include "acm_internal.hpp"
#include "fft_core.hpp"

namespace acm {

// ------------------------------------------------------------------ errors
static thread_local std::string g_err;

static acm_status fail(acm_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(e_ == hipErrorOutOfMemory ? ACM_E_NOMEM : ACM_E_HIP,                 \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                  \
  } while (0)

// ------------------------------------------------------------------- plans
struct CellPlan {
  Geom g;
  int prec;  // bytes per real
  int device;
  void* ctab = nullptr;
  void* rtab = nullptr;
  TableOffsets off{};
  int green_blocks = 0;  // largest green-pass grid over the tile variants
  int local_blocks = 0;
  int green_var = -1;    // tile variant picked by the autotuner (-1: not yet)
  int deriv = 0;         // derivative symbols (acm_opts.derivative)
  ~CellPlan() {
    if (ctab) (void)hipFree(ctab);
    if (rtab) (void)hipFree(rtab);
  }
};

static std::mutex g_mu;
static std::map<std::tuple<int, int, int, int, int, int, int>, std::unique_ptr<CellPlan>> g_plans;

static bool make_geom(const acm_grid* grid, Geom* g, const char** why) {
  if (!grid) {
    *why = "grid is NULL";
    return false;
  }
  if (grid->dim != 2 && grid->dim != 3) {
    *why = "dim must be 2 or 3";
    return false;
  }
  g->dim = grid->dim;
  g->nx = grid->n[0];
  g->ny = grid->n[1];
  g->nz = grid->dim == 3 ? grid->n[2] : 1;
  if (grid->dim == 2 && grid->n[2] != 1) {
    *why = "n[2] must be 1 when dim = 2";
    return false;
  }
  g->xh = g->nx / 2 + 1;
  g->ntot = (int64_t)g->nx * g->ny * g->nz;
  g->nrows = (int64_t)g->ny * g->nz;
  g->nspec = (int64_t)g->nz * g->ny * g->xh;
  g->last_n = g->dim == 3 ? g->nz : g->ny;
  g->plane = g->dim == 3 ? (int64_t)g->ny * g->xh : g->xh;
  return true;
}

static const char* const kUnsupportedSizeMsg =
    "grid lengths must be in {8,16,24,32,48,64,96,128,192,256,512,1024}";

static bool size_supported(const Geom& g) {
  auto ok = [](int n) { return fft_length_supported(n); };
  if (!ok(g.nx) || !ok(g.ny)) return false;
  if (g.dim == 3 && !ok(g.nz)) return false;
  return true;
}

static void push_twiddles(std::vector<double>& c, int L) {
  RadixPlan p = make_plan(L);
  for (int s = 0; s < p.nst; ++s) {
    const int R = p.r[s], NS = p.ns[s];
    for (int k = 0; k < NS; ++k)
      for (int r = 1; r < R; ++r) {
        const double ang = -2.0 * M_PI * (double)(k * r) / (double)(NS * R);
        c.push_back(cos(ang));
        c.push_back(sin(ang));
      }
  }
}

// Per-axis symbols on the unit cell (h = 1/n) for bins k < count: kind 0 the
// central difference sin(2 pi k/n)/h and the compact Laplacian
// 4 sin^2(pi k/n)/h^2 (eq. fft_app); kind 1 the exact 2 pi m and (2 pi m)^2
// with m the signed wavenumber.  The first derivative vanishes at Nyquist.
static void push_symbols(std::vector<double>& rv, int n, int count, int kind, int* s_off,
                         int* l_off) {
  *s_off = (int)rv.size();
  for (int k = 0; k < count; ++k) {
    const int m = 2 * k <= n ? k : k - n;
    double v;
    if (2 * k == n || n == 1) v = 0.0;
    else v = kind == 1 ? 2.0 * M_PI * m : sin(2.0 * M_PI * k / n) * n;
    rv.push_back(v);
  }
  *l_off = (int)rv.size();
  for (int k = 0; k < count; ++k) {
    const int m = 2 * k <= n ? k : k - n;
    const double sn = sin(M_PI * k / n);
    double l = 0.0;
    if (n != 1) l = kind == 1 ? (2.0 * M_PI * m) * (2.0 * M_PI * m) : 4.0 * sn * sn * n * n;
    rv.push_back(l);
  }
}

template <typename T>
static hipError_t upload(const std::vector<double>& v, void** dst) {
  std::vector<T> tmp(v.size());
  for (size_t i = 0; i < v.size(); ++i) tmp[i] = (T)v[i];
  size_t bytes = std::max<size_t>(tmp.size(), 2) * sizeof(T);
  hipError_t e = hipMalloc(dst, bytes);
  if (e != hipSuccess) return e;
  if (!tmp.empty()) e = hipMemcpy(*dst, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice);
  return e;
}

static acm_status get_plan(const acm_grid* grid, int precision, CellPlan** out, int deriv = 0) {
  Geom g;
  const char* why = nullptr;
  if (!make_geom(grid, &g, &why)) return fail(ACM_E_INVALID, why);
  if (!size_supported(g)) return fail(ACM_E_UNSUPPORTED_SIZE, kUnsupportedSizeMsg);
  if (precision != ACM_FP32 && precision != ACM_FP64)
    return fail(ACM_E_INVALID, "precision must be ACM_FP32 or ACM_FP64");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  if (deriv != 0 && deriv != 1) return fail(ACM_E_INVALID, "derivative must be 0 or 1");
  auto key = std::make_tuple(dev, precision, g.dim, g.nx, g.ny, g.nz, deriv);
  auto it = g_plans.find(key);
  if (it != g_plans.end()) {
    *out = it->second.get();
    return ACM_OK;
  }
  auto p = std::make_unique<CellPlan>();
  p->g = g;
  p->prec = precision == ACM_FP64 ? 8 : 4;
  p->device = dev;
  p->deriv = deriv;
  std::vector<double> c, r;
  p->off.tw_x = 0;
  push_twiddles(c, g.nx / 2);
  p->off.tw_y = (int)(c.size() / 2);
  push_twiddles(c, g.ny);
  p->off.tw_z = (int)(c.size() / 2);
  if (g.dim == 3) push_twiddles(c, g.nz);
  p->off.rtw = (int)(c.size() / 2);
  for (int k = 0; k <= g.nx / 2; ++k) {
    const double ang = -2.0 * M_PI * k / g.nx;
    c.push_back(cos(ang));
    c.push_back(sin(ang));
  }
  p->off.ncomplex = (int)(c.size() / 2);
  push_symbols(r, g.nx, g.xh, deriv, &p->off.sx, &p->off.lx);
  push_symbols(r, g.ny, g.ny, deriv, &p->off.sy, &p->off.ly);
  push_symbols(r, g.nz, g.nz, deriv, &p->off.sz, &p->off.lz);
  p->off.nreal = (int)r.size();
  hipError_t e;
  if (precision == ACM_FP64) {
    e = upload<double>(c, &p->ctab);
    if (e == hipSuccess) e = upload<double>(r, &p->rtab);
  } else {
    e = upload<float>(c, &p->ctab);
    if (e == hipSuccess) e = upload<float>(r, &p->rtab);
  }
  if (e != hipSuccess) return fail(ACM_E_HIP, std::string("table upload: ") + hipGetErrorString(e));
  p->green_blocks = 0;
  for (int v = 0; v < kGreenVariants; ++v)
    p->green_blocks = std::max(p->green_blocks, stokes_green_blocks(g, p->prec, v));
  p->local_blocks = stokes_local_blocks(g, p->prec);
  *out = p.get();
  g_plans[key] = std::move(p);
  return ACM_OK;
}

template <typename T>
static DevTables<T> tables_of(const CellPlan* p) {
  DevTables<T> tb;
  tb.ctab = p->ctab;
  tb.rtab = reinterpret_cast<const T*>(p->rtab);
  tb.off = p->off;
  return tb;
}

// A scoped device allocation.
struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

// Timing of eager launches with HIP events, per kernel kind.
LaunchEvents& launch_events() {
  static thread_local LaunchEvents e;
  return e;
}

// Per-kind kernel times of the profiling mode.  begin() arms launch_events()
// with a fresh event pair, so the next ACM_LAUNCH times its own kernel; end()
// keeps the pair if that launch consumed it.
struct Profiler {
  bool on = false;
  hipStream_t s = nullptr;
  double ms[KK_COUNT] = {0};
  int64_t calls[KK_COUNT] = {0};
  std::vector<std::tuple<int, hipEvent_t, hipEvent_t>> ev;
  hipEvent_t armed_stop = nullptr;
  void begin(int kind, hipEvent_t* a) {
    (void)kind;
    *a = nullptr;
    if (!on) return;
    hipEvent_t b = nullptr;
    if (hipEventCreate(a) != hipSuccess) return;
    if (hipEventCreate(&b) != hipSuccess) {
      (void)hipEventDestroy(*a);
      *a = nullptr;
      return;
    }
    armed_stop = b;
    launch_events() = LaunchEvents{*a, b};
  }
  void end(int kind, hipEvent_t a) {
    if (!on || !a) return;
    LaunchEvents& le = launch_events();
    if (le.start == a) {  // not consumed: the launch did not go through ACM_LAUNCH
      (void)hipEventDestroy(le.start);
      (void)hipEventDestroy(le.stop);
      le = LaunchEvents{};
      return;
    }
    ev.emplace_back(kind, a, armed_stop);
  }
  void collect() {
    for (auto& x : ev) {
      float t = 0.f;
      (void)hipEventSynchronize(std::get<2>(x));
      (void)hipEventElapsedTime(&t, std::get<1>(x), std::get<2>(x));
      ms[std::get<0>(x)] += t;
      calls[std::get<0>(x)] += 1;
      (void)hipEventDestroy(std::get<1>(x));
      (void)hipEventDestroy(std::get<2>(x));
    }
    ev.clear();
  }
};

// Streams owned by the library (default priority), one per device.
static hipStream_t work_stream(int dev) {
  static std::mutex mu;
  static std::map<int, hipStream_t> streams;
  std::lock_guard<std::mutex> lk(mu);
  auto it = streams.find(dev);
  if (it != streams.end()) return it->second;
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return nullptr;
  streams[dev] = s;
  return s;
}

// Order `ws` after the caller's stream.
static hipError_t join_from(hipStream_t caller, hipStream_t ws) {
  hipEvent_t e;
  hipError_t r = hipEventCreateWithFlags(&e, hipEventDisableTiming);
  if (r != hipSuccess) return r;
  r = hipEventRecord(e, caller);
  if (r == hipSuccess) r = hipStreamWaitEvent(ws, e, 0);
  (void)hipEventDestroy(e);
  return r;
}

// ------------------------------------------------------------------ Stokes
// One Stokes cell of a (possibly batched) call.
struct StokesCellIn {
  const uint8_t* H;
  double g[3];
  void* u;
  void* q;
};

// Extra default-priority streams used as graph branches (one per size class).
static std::vector<hipStream_t> branch_streams(int dev, int n) {
  static std::mutex mu;
  static std::map<int, std::vector<hipStream_t>> pool;
  std::lock_guard<std::mutex> lk(mu);
  auto& v = pool[dev];
  while ((int)v.size() < n) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) break;
    v.push_back(st);
  }
  return std::vector<hipStream_t>(v.begin(), v.begin() + std::min<int>(n, (int)v.size()));
}

// The state slot written last (the one with more completed iterations).
static const StokesState& latest_state(const StokesCtl& c) {
  return c.st[1].iter > c.st[0].iter ? c.st[1] : c.st[0];
}
static const TransportState& latest_tstate(const TransportCtl& c) {
  if (c.st[0].total_iter != c.st[1].total_iter)
    return c.st[1].total_iter > c.st[0].total_iter ? c.st[1] : c.st[0];
  return c.st[1].done ? c.st[1] : c.st[0];
}

// Cells sharing one plan (same grid and precision) are launched together.
template <typename T>
struct StokesGroup {
  CellPlan* pl = nullptr;
  std::vector<int> cells;  // indices into the call's cell list
  bool slab = false;
  bool fused = false;    // slab local + rhs in one launch (single resident cell)
  bool s4 = false;       // Step 4 in the green pass after the first iterations (single slab cell)
  bool rows5 = false;    // row-step pass structure (single cell, pass mode 5)
  int green_var = 0;     // tile variant of the green pass
  int ngreen = 0;        // green workgroups per cell for that variant
  int ngreen_max = 0;    // partial-buffer capacity (largest variant)
  int nlocal = 0;
  size_t spec_b = 0, one_b = 0, a_b = 0, part_b = 0, cell_b = 0;
  DevBuf ws;
  DevBuf dargs_buf, dcols_buf;
  std::vector<StokesCellArgs> hargs;
  std::vector<ColCellArgs> hcols;
  int par = 0;           // parity of the next iteration (state slot its passes read)
  const StokesCellArgs* dargs() const { return (const StokesCellArgs*)dargs_buf.p; }
  const ColCellArgs* dcols() const { return (const ColCellArgs*)dcols_buf.p; }
};

static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// IT_RHS: Step 4 in the rhs pass (slab) or the local pass (rows).
// IT_STEP4: slab passes whose iteration ends with the one-workgroup Step 4
// kernel instead of the rhs pass (the local pass has formed r with the b of
// the iteration; a Step 4 that changes b sets the hold word).
enum { IT_RHS = 0, IT_STEP4 = 1 };

template <typename T>
static hipError_t enqueue_iteration(StokesGroup<T>& G, hipStream_t s, Profiler* prof,
                                    int mode = IT_RHS) {
  const Geom& g = G.pl->g;
  DevTables<T> tb = tables_of<T>(G.pl);
  const int n = (int)G.cells.size();
  const StokesCellArgs& one = G.hargs[0];
  const StokesCellArgs* many = n > 1 ? G.dargs() : nullptr;
  const int d = g.dim;
  hipError_t e;
  hipEvent_t ev0 = nullptr;
  auto cols = [&](int sign, int kind) -> hipError_t {
    prof->begin(kind, &ev0);
    hipError_t r = n > 1 ? launch_cols_batched<T>(g, tb, 1, sign, d, G.dcols(), n, s)
                         : launch_cols<T>(g, tb, 1, sign, d, one.spec, s, &one.ctl->st[0].done,
                                          &one.ctl->st[1].done);
    prof->end(kind, ev0);
    return r;
  };
  const int par = G.par;
  G.par ^= 1;
  if (prof->on) {
    // an empty kernel timed the same way: the per-launch overhead of the
    // event timestamps (reported as its own kind)
    prof->begin(KK_OTHER, &ev0);
    e = launch_noop(s);
    if (e != hipSuccess) return e;
    prof->end(KK_OTHER, ev0);
  }
  prof->begin(KK_GREEN, &ev0);
  e = launch_stokes_green<T>(g, tb, one, many, n, par, G.green_var, nullptr, s);
  if (e != hipSuccess) return e;
  prof->end(KK_GREEN, ev0);
  if (G.rows5) {
    if (d == 3 && (e = cols(+1, KK_YINV)) != hipSuccess) return e;
    prof->begin(KK_LOCAL, &ev0);
    e = launch_rows_step<T>(g, tb, one, par, G.ngreen, s);
    if (e != hipSuccess) return e;
    prof->end(KK_LOCAL, ev0);
    prof->begin(KK_RHS, &ev0);
    e = launch_step4_nohold(g, one, par, rows_step_blocks(g, (int)sizeof(T)), s);
    if (e != hipSuccess) return e;
    prof->end(KK_RHS, ev0);
    prof->begin(KK_RHS, &ev0);
    e = launch_rows_rhs_cond<T>(g, tb, one, par, s);
    if (e != hipSuccess) return e;
    prof->end(KK_RHS, ev0);
    if (d == 3 && (e = cols(-1, KK_YFWD)) != hipSuccess) return e;
    return hipSuccess;
  }
  if (mode == IT_STEP4) {
    prof->begin(KK_LOCAL, &ev0);
    e = launch_slab_local<T>(g, tb, one, many, n, par, G.ngreen, s);
    if (e != hipSuccess) return e;
    prof->end(KK_LOCAL, ev0);
    prof->begin(KK_RHS, &ev0);
    e = launch_slab_step4<T>(g, one, par, slab_local_blocks<T>(g), s);
    if (e != hipSuccess) return e;
    prof->end(KK_RHS, ev0);
    return hipSuccess;
  }
  if (G.fused) {
    prof->begin(KK_LOCAL, &ev0);
    e = launch_slab_fused<T>(g, tb, one, par, G.ngreen, s);
    if (e != hipSuccess) return e;
    prof->end(KK_LOCAL, ev0);
    return hipSuccess;
  }
  if (G.slab) {
    prof->begin(KK_LOCAL, &ev0);
    e = launch_slab_local<T>(g, tb, one, many, n, par, G.ngreen, s);
    if (e != hipSuccess) return e;
    prof->end(KK_LOCAL, ev0);
    prof->begin(KK_RHS, &ev0);
    e = launch_slab_rhs<T>(g, tb, one, many, n, par, 1, G.ngreen, s);
    if (e != hipSuccess) return e;
    prof->end(KK_RHS, ev0);
    return hipSuccess;
  }
  if (d == 3 && (e = cols(+1, KK_YINV)) != hipSuccess) return e;
  prof->begin(KK_LOCAL, &ev0);
  e = launch_stokes_local<T>(g, tb, one, many, n, par, G.ngreen, s);
  if (e != hipSuccess) return e;
  prof->end(KK_LOCAL, ev0);
  prof->begin(KK_RHS, &ev0);
  e = launch_stokes_rhs<T>(g, tb, one, many, n, par ^ 1, s);
  if (e != hipSuccess) return e;
  prof->end(KK_RHS, ev0);
  if (d == 3 && (e = cols(-1, KK_YFWD)) != hipSuccess) return e;
  return hipSuccess;
}

template <typename T>
static acm_status stokes_run(const std::vector<CellPlan*>& plans,
                             const std::vector<StokesCellIn>& cells, double nu,
                             const acm_penalty& pen, const acm_opts& o, acm_stats* stats,
                             double* history, hipStream_t caller) {
  const int ncell = (int)cells.size();
  const int dev = plans[0]->device;
  hipStream_t s = work_stream(dev);
  if (!s) return fail(ACM_E_HIP, "cannot create work stream");
  HIP_TRY(join_from(caller, s));

  // ---- group cells by plan
  std::vector<std::unique_ptr<StokesGroup<T>>> groups;
  for (int i = 0; i < ncell; ++i) {
    StokesGroup<T>* G = nullptr;
    for (auto& gp : groups)
      if (gp->pl == plans[i]) G = gp.get();
    if (!G) {
      groups.emplace_back(new StokesGroup<T>());
      G = groups.back().get();
      G->pl = plans[i];
    }
    G->cells.push_back(i);
  }
  const int hist_cap = (ncell == 1 && o.history_cap > 0) ? o.history_cap : 0;
  DevBuf ctl_buf, hist_buf;
  HIP_TRY(hipMalloc(&ctl_buf.p, sizeof(StokesCtl) * ncell));
  StokesCtl* dctl = (StokesCtl*)ctl_buf.p;
  if (hist_cap > 0) HIP_TRY(hipMalloc(&hist_buf.p, sizeof(double) * kHistDoubles * hist_cap));

  for (auto& Gp : groups) {
    StokesGroup<T>& G = *Gp;
    const Geom& g = G.pl->g;
    const int d = g.dim;
    const size_t cb = sizeof(T) * 2;
    G.spec_b = cb * (size_t)g.nspec * d;
    G.one_b = cb * (size_t)g.nspec;
    G.a_b = sizeof(T) * (size_t)g.ntot * d;
    G.ngreen_max = G.pl->green_blocks;
    G.green_var = G.pl->green_var >= 0 ? G.pl->green_var : 0;
    G.ngreen = stokes_green_blocks(g, G.pl->prec, G.green_var);
    bool aligned = true;
    for (int i : G.cells)
      aligned = aligned && ((uintptr_t)cells[i].u % 32 == 0) && ((uintptr_t)cells[i].H % 16 == 0);
    const bool one_cell = groups.size() == 1 && G.cells.size() == 1;
    if (o.pass_mode == 2 || o.pass_mode == 3 || o.pass_mode == 4) {
      if (!(slab_supported<T>(g) && aligned))
        return fail(ACM_E_INVALID,
                    "fused xy passes need a 3D cell with nx == ny <= 128 and aligned u, H");
      if (o.pass_mode == 4 && !one_cell)
        return fail(ACM_E_INVALID, "the Step 4 kernel form needs a single cell");
      G.s4 = o.pass_mode == 4;
      if (o.pass_mode == 3 && !(one_cell && slab_fused_capacity<T>(g) >= g.nz * g.dim))
        return fail(ACM_E_INVALID,
                    "the single-launch slab pass needs one cell whose nz * 3 workgroups are all "
                    "resident on the device at once");
      G.slab = true;
      G.fused = o.pass_mode == 3;
    } else if (o.pass_mode == 5) {
      if (!one_cell) return fail(ACM_E_INVALID, "the row-step pass structure needs a single cell");
      if (!aligned) return fail(ACM_E_INVALID, "the row-step passes need 32-byte aligned u and 16-byte aligned H");
      G.rows5 = true;
    } else if (o.pass_mode == 0) {
      // the single-launch structure is not chosen automatically: its
      // device-wide gate has measured slower than the launch boundary; the
      // Step 4 kernel form is (one cell); a single 3D cell whose slab does
      // not fit takes the row-step structure
      G.slab = slab_supported<T>(g) && aligned;
      G.s4 = G.slab && one_cell;
      G.rows5 = !G.slab && one_cell && aligned && g.dim == 3;
    }
    G.nlocal = std::max(std::max(G.pl->local_blocks, slab_local_blocks<T>(g)),
                        rows_step_blocks(g, (int)sizeof(T)));
    G.part_b = sizeof(double) * (size_t)(3 * G.ngreen_max + 7 * G.nlocal);
    G.cell_b = al256(G.spec_b) + 2 * al256(G.one_b) + al256(G.a_b) + al256(G.part_b);
    HIP_TRY(hipMalloc(&G.ws.p, G.cell_b * G.cells.size()));
    for (size_t k = 0; k < G.cells.size(); ++k) {
      const int i = G.cells[k];
      char* base = (char*)G.ws.p + k * G.cell_b;
      StokesCellArgs A;
      A.spec = base;
      A.qhat = base + al256(G.spec_b);
      A.dhat = (char*)A.qhat + al256(G.one_b);
      A.a = (char*)A.dhat + al256(G.one_b);
      A.part = (double*)((char*)A.a + al256(G.a_b));
      A.lpart = A.part + 3 * (size_t)G.ngreen_max;
      A.u = cells[i].u;
      A.H = cells[i].H;
      A.ctl = dctl + i;
      A.hist = hist_cap > 0 ? (double*)hist_buf.p : nullptr;
      G.hargs.push_back(A);
      G.hcols.push_back(ColCellArgs{A.spec, &A.ctl->st[0].done, &A.ctl->st[1].done});
    }
    if (G.cells.size() > 1) {
      HIP_TRY(hipMalloc(&G.dargs_buf.p, sizeof(StokesCellArgs) * G.cells.size()));
      HIP_TRY(hipMalloc(&G.dcols_buf.p, sizeof(ColCellArgs) * G.cells.size()));
      HIP_TRY(hipMemcpyAsync(G.dargs_buf.p, G.hargs.data(), sizeof(StokesCellArgs) * G.cells.size(),
                             hipMemcpyHostToDevice, s));
      HIP_TRY(hipMemcpyAsync(G.dcols_buf.p, G.hcols.data(), sizeof(ColCellArgs) * G.cells.size(),
                             hipMemcpyHostToDevice, s));
    }
    // zero start: spectra, q-hat, div-hat, a and partials of every cell
    if (!o.warm_start) {
      HIP_TRY(hipMemsetAsync(G.ws.p, 0, G.cell_b * G.cells.size(), s));
      for (int i : G.cells) HIP_TRY(hipMemsetAsync(cells[i].u, 0, G.a_b, s));
    } else {
      for (const auto& A : G.hargs) HIP_TRY(hipMemsetAsync(A.part, 0, G.part_b, s));
    }
  }

  // ---- control blocks
  std::vector<StokesCtl> hc(ncell);
  for (int i = 0; i < ncell; ++i) {
    const Geom& g = plans[i]->g;
    const int d = g.dim;
    StokesCtl& c = hc[i];
    memset(&c, 0, sizeof(c));
    const double p0 = nu * (double)std::max(g.nx, std::max(g.ny, g.nz));
    StokesState& s0 = c.st[0];
    s0.psi[0] = pen.alpha > 0 ? pen.alpha : p0;
    s0.psi[1] = pen.beta > 0 ? pen.beta : p0;
    s0.psi[2] = pen.b > 0 ? pen.b : p0;
    for (int k = 0; k < 3; ++k) {
      c.phi[k] = pen.phi[k];
      c.tau[k] = pen.tau[k];
      c.psi_min[k] = pen.psi_min[k] > 0 ? pen.psi_min[k] : 1e-3 * s0.psi[k];
      c.g[k] = k < d ? cells[i].g[k] : 0.0;
    }
    s0.c_prev = 0.0;
    s0.s_min = INFINITY;
    s0.iter = 0;
    s0.done = 0;
    s0.status = 1;
    c.st[1] = s0;
    c.eps = o.eps;
    c.sqrt_n[0] = sqrt((double)d * (double)g.ntot);
    c.sqrt_n[1] = sqrt((double)g.ntot);
    c.sqrt_n[2] = c.sqrt_n[0];
    c.nu = nu;
    c.max_iter = o.max_iter;
    c.adaptive = pen.adaptive;
    c.hist_cap = hist_cap;
  }
  // Step 1 in increment form: the two-launch slab passes form X in their
  // local pass (automatic for FP32 there; FP64 keeps the paper's form)
  for (auto& Gp : groups) {
    const bool can = (Gp->slab && !Gp->fused) || Gp->rows5;
    const int form = o.step1_form != 0 ? o.step1_form : (can && sizeof(T) == 4 ? 2 : 1);
    if (form == 2 && !can)
      return fail(ACM_E_INVALID,
                  "the increment form of Step 1 needs the two-launch xy-slab passes or the "
                  "row-step passes (pass mode 2, 4 or 5)");
    for (int i : Gp->cells) hc[i].incr_enabled = form == 2 ? 1 : 0;
  }
  HIP_TRY(hipMemcpyAsync(dctl, hc.data(), sizeof(StokesCtl) * ncell, hipMemcpyHostToDevice, s));

  // ---- warm start: u0 = (1-H) u_in, q0 = q_in, a0 = lambda0 = H (g - grad q0 +
  // nu Delta u0); q-hat0 = FFT(q0), div-hat0 = FFT(div u0); the Step-1
  // right-hand side from the rhs pass (c_prev = 0: u0 vanishes in the solid).
  if (o.warm_start) {
    for (auto& Gp : groups) {
      StokesGroup<T>& G = *Gp;
      const Geom& g = G.pl->g;
      DevTables<T> tb = tables_of<T>(G.pl);
      for (size_t k = 0; k < G.cells.size(); ++k) {
        const StokesCellArgs& A = G.hargs[k];
        const StokesCellIn& C = cells[G.cells[k]];
        T* divbuf = (T*)A.spec;  // scratch: the spectra are rebuilt below
        hipError_t e = launch_warm_init<T>(g, (const T*)A.u, (const T*)C.q, A.H, (T*)A.a, divbuf,
                                           nu, hc[G.cells[k]].g, s);
        if (e == hipSuccess) e = launch_rows_r2c<T>(g, tb, 1, divbuf, A.dhat, s);
        if (e == hipSuccess) e = launch_cols<T>(g, tb, 1, -1, 1, A.dhat, s);
        if (e == hipSuccess && g.dim == 3) e = launch_cols<T>(g, tb, 2, -1, 1, A.dhat, s);
        if (e == hipSuccess) {
          if (C.q) {
            e = launch_rows_r2c<T>(g, tb, 1, (const T*)C.q, A.qhat, s);
            if (e == hipSuccess) e = launch_cols<T>(g, tb, 1, -1, 1, A.qhat, s);
            if (e == hipSuccess && g.dim == 3) e = launch_cols<T>(g, tb, 2, -1, 1, A.qhat, s);
          } else {
            e = hipMemsetAsync(A.qhat, 0, G.one_b, s);
          }
        }
        if (e == hipSuccess) {
          if (G.slab) {
            e = launch_slab_rhs<T>(g, tb, A, nullptr, 1, 0, 0, 0, s);
          } else {
            e = launch_stokes_rhs<T>(g, tb, A, nullptr, 1, 0, s);
            if (e == hipSuccess && g.dim == 3) e = launch_cols<T>(g, tb, 1, -1, g.dim, A.spec, s);
          }
        }
        if (e != hipSuccess) return fail(ACM_E_HIP, std::string("warm start: ") + hipGetErrorString(e));
      }
    }
  }

  Profiler prof;
  prof.on = o.profile != 0;
  prof.s = s;

  int K = o.check_every;
  if (K <= 0) {
    double work = 0.0;
    for (int i = 0; i < ncell; ++i) work += (double)plans[i]->g.ntot * plans[i]->g.dim;
    K = (int)std::min(200.0, std::max(8.0, 3.0e8 / work));
  }
  if (o.max_iter < K) K = (int)std::max<int64_t>(1, o.max_iter);
  // even, so that every replay of the captured iterations starts on the same
  // state slot (the passes alternate between the two slots)
  K += K & 1;

  StokesCtl* hctl = nullptr;
  HIP_TRY(hipHostMalloc((void**)&hctl, sizeof(StokesCtl) * ncell, hipHostMallocDefault));
  struct HostFree {
    void* p;
    ~HostFree() {
      if (p) (void)hipHostFree(p);
    }
  } hf{hctl};

  // ---- autotuning of the green pass: the first iterations of the first solve
  // of a plan run eagerly, one kernel variant at a time (tile widths of the
  // LDS-staged kernel, then of the register-resident one), with HIP events
  // around whole iterations; the fastest variant is kept for this plan.  The
  // variants are timed in interleaved rounds and each keeps its best round:
  // an iteration whose Step 4 changes b runs the full rhs pass, and a single
  // round would charge such an iteration to whichever variant it fell on.
  // The variants apply the same arithmetic in the same order (up to the
  // compiler's contraction choices), so the choice changes iterates only at
  // the rounding level.
  {
    for (auto& Gp : groups) {
      StokesGroup<T>& G = *Gp;
      const Geom& g = G.pl->g;
      if (o.green_variant > 0) {
        G.green_var = o.green_variant - 1;
      } else if (G.pl->green_var < 0 && g.ntot >= (int64_t)64 * 64 * 64 &&
                 o.max_iter >= 2 * kTuneRounds * kGreenVariants * 5) {
        float vbest[kGreenVariants];
        for (int v = 0; v < kGreenVariants; ++v) vbest[v] = 1e30f;
        hipEvent_t e0, e1;
        HIP_TRY(hipEventCreate(&e0));
        HIP_TRY(hipEventCreate(&e1));
        Profiler off;
        for (int tv = 0; tv < kTuneRounds * kGreenVariants; ++tv) {
          const int v = tv % kGreenVariants;
          G.green_var = v;
          G.ngreen = stokes_green_blocks(g, G.pl->prec, v);
          // one warm-up iteration, then 4 timed iterations back to back
          hipError_t e = enqueue_iteration<T>(G, s, &off);
          if (e == hipSuccess) e = hipEventRecord(e0, s);
          for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) e = enqueue_iteration<T>(G, s, &off);
          if (e == hipSuccess) e = hipEventRecord(e1, s);
          if (e == hipSuccess) e = hipEventSynchronize(e1);
          float ms = 0.f;
          if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
          if (e != hipSuccess) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            return fail(ACM_E_HIP, std::string("autotune: ") + hipGetErrorString(e));
          }
          vbest[v] = std::min(vbest[v], ms);
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        int bestv = 0;
        for (int v = 1; v < kGreenVariants; ++v)
          if (vbest[v] < vbest[bestv]) bestv = v;
        G.pl->green_var = bestv;
        G.green_var = bestv;
      } else if (G.pl->green_var >= 0) {
        G.green_var = G.pl->green_var;
      }
      G.ngreen = stokes_green_blocks(g, G.pl->prec, G.green_var);
    }
  }

  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  std::vector<hipEvent_t> evs;
  struct EvFree {
    std::vector<hipEvent_t>* v;
    ~EvFree() {
      for (auto e : *v) (void)hipEventDestroy(e);
    }
  } evf{&evs};
  const bool use_graph = o.use_graph && !prof.on;
  // Step 4 in its own kernel: a single slab cell after its first iterations
  // (in which Step 4 changes b often); graph_b holds those iterations
  StokesGroup<T>* s4g = (groups.size() == 1 && groups[0]->s4) ? groups[0].get() : nullptr;
  // profiled solves check every other iteration, so that the launches that
  // skip behind a hold (counted by the profiler) stay at most one iteration
  if (s4g && prof.on) K = std::min(K, 2);
  hipGraph_t graph_b = nullptr;
  hipGraphExec_t exec_b = nullptr;
  struct GraphFreeB {
    hipGraph_t* g;
    hipGraphExec_t* x;
    ~GraphFreeB() {
      if (*x) (void)hipGraphExecDestroy(*x);
      if (*g) (void)hipGraphDestroy(*g);
    }
  } gfb{&graph_b, &exec_b};
  const int start_par = groups[0]->par;  // state slot every replay starts from
  if (use_graph) {
    std::vector<hipStream_t> br;
    if (groups.size() > 1) {
      br = branch_streams(dev, (int)groups.size());
      if (br.size() < groups.size()) return fail(ACM_E_HIP, "cannot create branch streams");
      for (size_t i = 0; i < 2 * groups.size(); ++i) {
        hipEvent_t e;
        HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        evs.push_back(e);
      }
    }
    if (s4g) {
      // the iterations ending with the Step 4 kernel, captured from the same
      // state slot as the others
      HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      hipError_t e = hipSuccess;
      for (int k = 0; k < K && e == hipSuccess; ++k)
        e = enqueue_iteration<T>(*s4g, s, &prof, IT_STEP4);
      hipError_t e2 = hipStreamEndCapture(s, &graph_b);
      if (e != hipSuccess) {
        if (graph_b) (void)hipGraphDestroy(graph_b);
        graph_b = nullptr;
        return fail(ACM_E_HIP, std::string("kernel launch during capture: ") + hipGetErrorString(e));
      }
      HIP_TRY(e2);
      HIP_TRY(hipGraphInstantiate(&exec_b, graph_b, nullptr, nullptr, 0));
    }
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    if (groups.size() == 1) {
      for (int k = 0; k < K && e == hipSuccess; ++k) e = enqueue_iteration<T>(*groups[0], s, &prof);
    } else {
      for (size_t gi = 0; gi < groups.size() && e == hipSuccess; ++gi) {
        e = hipEventRecord(evs[2 * gi], s);
        if (e == hipSuccess) e = hipStreamWaitEvent(br[gi], evs[2 * gi], 0);
        for (int k = 0; k < K && e == hipSuccess; ++k)
          e = enqueue_iteration<T>(*groups[gi], br[gi], &prof);
        if (e == hipSuccess) e = hipEventRecord(evs[2 * gi + 1], br[gi]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, evs[2 * gi + 1], 0);
      }
    }
    hipError_t e2 = hipStreamEndCapture(s, &graph);
    if (e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return fail(ACM_E_HIP, std::string("kernel launch during capture: ") + hipGetErrorString(e));
    }
    HIP_TRY(e2);
    HIP_TRY(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
  }
  struct GraphFree {
    hipGraph_t g;
    hipGraphExec_t x;
    ~GraphFree() {
      if (x) (void)hipGraphExecDestroy(x);
      if (g) (void)hipGraphDestroy(g);
    }
  } gf{graph, exec};

  auto t0 = std::chrono::steady_clock::now();
  std::vector<double> t_done(ncell, -1.0);
  int64_t launched = 0;
  bool step4_kernel = false;  // the iterations now end with the Step 4 kernel
  int64_t it_prev = -1;
  for (;;) {
    if (use_graph) {
      HIP_TRY(hipGraphLaunch(step4_kernel ? exec_b : exec, s));
    } else {
      for (int k = 0; k < K; ++k)
        for (auto& Gp : groups) {
          hipError_t e = enqueue_iteration<T>(*Gp, s, &prof, step4_kernel ? IT_STEP4 : IT_RHS);
          if (e != hipSuccess) return fail(ACM_E_HIP, std::string("launch: ") + hipGetErrorString(e));
        }
    }
    launched += K;
    HIP_TRY(hipMemcpyAsync(hctl, dctl, sizeof(StokesCtl) * ncell, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    prof.collect();
    bool all = true;
    const double now = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int i = 0; i < ncell; ++i) {
      const bool done = stokes_done(&hctl[i]);
      if (done && t_done[i] < 0) t_done[i] = now;
      all = all && done;
    }
    if (all) break;
    // safety net (the device caps the iterations itself): launches that no
    // longer advance any cell; iterations skipped behind a hold do not count
    int64_t it_now = 0;
    for (int i = 0; i < ncell; ++i) it_now = std::max(it_now, latest_state(hctl[i]).iter);
    const bool held = s4g && step4_kernel && hctl[0].hold;
    if (!held && launched > o.max_iter + 2LL * K && it_now == it_prev) break;
    it_prev = it_now;
    if (s4g && !step4_kernel && launched >= kRhsStep4Iters) {
      // from here Step 4 runs in its own kernel (Step 4 of the last iteration
      // was formed by its rhs pass: nothing else to do)
      step4_kernel = true;
    } else if (s4g && step4_kernel && hctl[0].hold) {
      // A Step 4 kernel found that b changed, stored the new state in slot
      // hold - 1 and stopped the iterations after it.  r is formed again from
      // u, a and H with the new b; then, if needed, one iteration brings the
      // next state slot back to the one the captured iterations start from.
      StokesGroup<T>& G = *s4g;
      const Geom& g = G.pl->g;
      DevTables<T> tb = tables_of<T>(G.pl);
      const int slot = hctl[0].hold - 1;
      HIP_TRY(hipMemsetAsync(&dctl[0].hold, 0, sizeof(int32_t), s));
      hipEvent_t ev0 = nullptr;
      prof.begin(KK_RHS, &ev0);
      hipError_t e = launch_slab_rhs<T>(g, tb, G.hargs[0], nullptr, 1, slot, 0, 0, s);
      prof.end(KK_RHS, ev0);
      G.par = slot;
      if (e == hipSuccess && G.par != start_par) {
        e = enqueue_iteration<T>(G, s, &prof, IT_STEP4);
        launched += 1;
      }
      if (e != hipSuccess) return fail(ACM_E_HIP, std::string("launch: ") + hipGetErrorString(e));
    }
  }
  auto t1 = std::chrono::steady_clock::now();

  // ---- read-out of q: inverse transform of q-hat
  for (auto& Gp : groups) {
    StokesGroup<T>& G = *Gp;
    const Geom& g = G.pl->g;
    DevTables<T> tb = tables_of<T>(G.pl);
    for (size_t k = 0; k < G.cells.size(); ++k) {
      const StokesCellIn& C = cells[G.cells[k]];
      if (!C.q) continue;
      const StokesCellArgs& A = G.hargs[k];
      HIP_TRY(hipMemcpyAsync(A.spec, A.qhat, G.one_b, hipMemcpyDeviceToDevice, s));
      hipError_t e = hipSuccess;
      if (g.dim == 3) e = launch_cols<T>(g, tb, 2, +1, 1, A.spec, s);
      if (e == hipSuccess) e = launch_cols<T>(g, tb, 1, +1, 1, A.spec, s);
      if (e == hipSuccess) e = launch_rows_c2r<T>(g, tb, 1, A.spec, (T*)C.q, 1.0 / (double)g.ntot, s);
      if (e != hipSuccess) return fail(ACM_E_HIP, hipGetErrorString(e));
    }
  }
  if (history && hist_cap > 0) {
    std::vector<double> h((size_t)hist_cap * kHistDoubles);
    HIP_TRY(hipMemcpyAsync(h.data(), hist_buf.p, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const int64_t n = latest_state(hctl[0]).iter;
    const int64_t keep = std::min<int64_t>(n, hist_cap);
    for (int64_t i = 0; i < keep; ++i) {
      const int64_t it = n - keep + i;
      memcpy(history + i * kHistDoubles, h.data() + (it % hist_cap) * kHistDoubles,
             sizeof(double) * kHistDoubles);
    }
  }
  HIP_TRY(hipStreamSynchronize(s));
  const double total_s = std::chrono::duration<double>(t1 - t0).count();
  for (int i = 0; i < ncell; ++i)
    if (hctl[i].fault)
      return fail(ACM_E_HIP, "the single-launch slab pass gave up waiting at its device-wide gate "
                             "(its workgroups were not all resident)");
  int worst = 0;
  for (int i = 0; i < ncell; ++i) {
    const StokesState& c = latest_state(hctl[i]);
    if (c.status == -5) worst = -5;
    else if (c.status != 0 && worst == 0) worst = 1;
    if (!stats) continue;
    acm_stats* st = stats + i;
    memset(st, 0, sizeof(*st));
    st->iters = c.iter;
    for (int k = 0; k < 3; ++k) {
      st->r_p[k] = c.rp[k];
      st->r_d[k] = c.rd[k];
      st->tol_p[k] = c.tp[k];
      st->tol_d[k] = c.td[k];
      st->psi[k] = c.psi[k];
    }
    st->seconds = ncell == 1 ? total_s : (t_done[i] >= 0 ? t_done[i] : total_s);
    st->converged = c.status == 0;
    st->status = c.status;
    if (i == 0)
      for (int k = 0; k < KK_COUNT; ++k) {
        st->kernel_ms[k] = prof.ms[k];
        st->kernel_calls[k] = prof.calls[k];
      }
  }
  if (worst == -5)
    return fail(ACM_E_DIVERGED, "a residual became non-finite or grew a millionfold over its minimum");
  return worst == 0 ? ACM_OK : ACM_NOT_CONVERGED;
}

// Argument checks shared by the single and batched Stokes entry points.
static acm_status check_stokes_cell(const acm_grid* grid, const uint8_t* H, const double* g_p,
                                    void* u, int precision, int deriv, hipStream_t cs,
                                    CellPlan** pl, bool* all_solid) {
  if (!H || !g_p || !u) return fail(ACM_E_INVALID, "H, g_p and u must be non-NULL");
  acm_status r = get_plan(grid, precision, pl, deriv);
  if (r != ACM_OK) return r;
  for (int k = 0; k < grid->dim; ++k)
    if (!isfinite(g_p[k])) return fail(ACM_E_INVALID, "g_p must be finite");
  // H must contain a solid voxel: with no solid the mean of a grows without
  // bound under a body force and no steady flow exists.
  std::vector<uint8_t> hh((size_t)(*pl)->g.ntot);
  hipError_t e = hipMemcpyAsync(hh.data(), H, hh.size(), hipMemcpyDeviceToHost, cs);
  if (e == hipSuccess) e = hipStreamSynchronize(cs);
  if (e != hipSuccess) return fail(ACM_E_HIP, std::string("reading H: ") + hipGetErrorString(e));
  bool any = false, all = true;
  for (uint8_t v : hh) {
    if (v > 1) return fail(ACM_E_INVALID, "H must hold 0 or 1");
    any |= v == 1;
    all &= v == 1;
  }
  if (!any) return fail(ACM_E_INVALID, "H has no solid voxel: no steady flow under a body force");
  *all_solid = all;
  return ACM_OK;
}

// An all-solid cell: the flow is zero (u = 0 in the solid) and so is the
// multiplier q; no iteration runs.
static acm_status stokes_all_solid(const CellPlan* pl, void* u, void* q, acm_stats* st,
                                   hipStream_t cs) {
  const Geom& g = pl->g;
  HIP_TRY(hipMemsetAsync(u, 0, (size_t)pl->prec * g.dim * (size_t)g.ntot, cs));
  if (q) HIP_TRY(hipMemsetAsync(q, 0, (size_t)pl->prec * (size_t)g.ntot, cs));
  HIP_TRY(hipStreamSynchronize(cs));
  if (st) {
    memset(st, 0, sizeof(*st));
    st->converged = 1;
    st->status = 0;
  }
  return ACM_OK;
}

static acm_status check_penalty_opts(const acm_penalty& P, const acm_opts& O, double nu) {
  if (!(nu > 0.0) || !isfinite(nu)) return fail(ACM_E_INVALID, "nu must be positive");
  if (!(O.eps >= 0.0) || O.max_iter < 1) return fail(ACM_E_INVALID, "eps >= 0 and max_iter >= 1 required");
  if (O.pass_mode < 0 || O.pass_mode > 5) return fail(ACM_E_INVALID, "pass_mode must be 0 to 5");
  if (O.derivative != 0 && O.derivative != 1) return fail(ACM_E_INVALID, "derivative must be 0 or 1");
  if (O.step1_form < 0 || O.step1_form > 2) return fail(ACM_E_INVALID, "step1_form must be 0, 1 or 2");
  if (O.derivative == 1 && O.warm_start)
    return fail(ACM_E_INVALID, "the warm start forms its state with central differences: derivative 0");
  if (O.green_variant < 0 || O.green_variant > kGreenVariants)
    return fail(ACM_E_INVALID, "green_variant must be in [0, " + std::to_string(kGreenVariants) + "]");
  for (int k = 0; k < 3; ++k)
    if (!(P.phi[k] >= 1.0) || !(P.tau[k] > 0.0))
      return fail(ACM_E_INVALID, "phi >= 1 and tau > 0 required");
  return ACM_OK;
}

// --------------------------------------------------------------- reductions
// Run a partial-sum kernel and add the block partials on the host in order.
template <typename Launch>
static acm_status reduce_on_host(const Geom& g, hipStream_t s, std::vector<double>* out,
                                 Launch&& launch) {
  const int nb = reduction_blocks(g);
  DevBuf part;
  HIP_TRY(hipMalloc(&part.p, sizeof(double) * 16 * (size_t)nb));
  int ns = 0;
  HIP_TRY(launch((double*)part.p, &ns));
  std::vector<double> h((size_t)nb * ns);
  HIP_TRY(hipMemcpyAsync(h.data(), part.p, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  out->assign(ns, 0.0);
  for (int b = 0; b < nb; ++b)
    for (int k = 0; k < ns; ++k) (*out)[k] += h[(size_t)b * ns + k];
  return ACM_OK;
}

// --------------------------------------------------------------- transport
template <typename T>
static acm_status transport_impl(CellPlan* pl, const uint8_t* H, const T* u, const double* gchi,
                                 double Pe, double diff, double eta, double A0, const double* B0,
                                 double dt, int n_steps, const acm_opts& o, T* chi,
                                 acm_stats* st, hipStream_t caller) {
  const Geom& g = pl->g;
  const int d = g.dim;
  DevTables<T> tb = tables_of<T>(pl);
  hipStream_t s = work_stream(pl->device);
  if (!s) return fail(ACM_E_HIP, "cannot create work stream");
  HIP_TRY(join_from(caller, s));

  // pore-averaged velocity (Section 2) for calF = Pe (1-H) ubar . g
  std::vector<double> fs;
  acm_status r = reduce_on_host(g, s, &fs, [&](double* part, int* ns) {
    return launch_flow_sums<T>(g, u, H, part, ns, s);
  });
  if (r != ACM_OK) return r;
  if (!(fs[0] > 0.0)) return fail(ACM_E_INVALID, "H has no pore voxel");
  double ubar_g = 0.0;
  for (int c = 0; c < d; ++c) ubar_g += (fs[1 + c] / fs[0]) * gchi[c];

  // 3D cubes that fit take the slab form of the local pass (no separate y
  // passes; f arrives as d partial spectra)
  // (the slab form folds the x and y divergence in as central differences, so
  // the exact symbols take the row form)
  // The flux form (face fluxes with harmonic-mean diffusivity) takes the row
  // form: its green pass returns the central gradient and the forward
  // difference (2 d fields).
  const bool flux = o.transport_form == 1;
  if (flux && pl->deriv != 0)
    return fail(ACM_E_INVALID, "the flux form is built on differences: derivative must be 0");
  const bool tslab = !flux && d == 3 && pl->deriv == 0 && slab_supported<T>(g) &&
                     ((uintptr_t)u % 16 == 0) && ((uintptr_t)H % 4 == 0);
  const size_t cb = sizeof(T) * 2;
  // slab form: a fifth field holds f_z (see k_transport_slab)
  const size_t spec_b = cb * (size_t)g.nspec * (flux ? 2 * d : d + (tslab ? 2 : 1));
  const size_t one_b = cb * (size_t)g.nspec;
  const int ngreen = std::max(std::max(transport_green_blocks(g, pl->prec, false),
                                       transport_green_blocks(g, pl->prec, tslab)),
                              transport_green_blocks(g, pl->prec, false, flux));
  const size_t part_b = sizeof(double) * 2 * (size_t)ngreen;
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  DevBuf ws;
  HIP_TRY(hipMalloc(&ws.p, al(spec_b) + 2 * al(one_b) + al(part_b) + al(sizeof(TransportCtl))));
  char* cur = (char*)ws.p;
  auto take = [&](size_t b) {
    void* p = cur;
    cur += al(b);
    return p;
  };
  void* spec = take(spec_b);
  void* chat = take(one_b);
  void* chat_m = take(one_b);
  double* part = (double*)take(part_b);
  TransportCtl* dctl = (TransportCtl*)take(sizeof(TransportCtl));

  const bool steady = !isfinite(dt);
  TransportCtl c{};
  c.eps = o.eps;
  c.sqrt_n1 = sqrt((double)g.ntot);
  c.sqrt_n2 = sqrt((double)d * (double)g.ntot);
  c.inv_dt = steady ? 0.0 : 1.0 / dt;
  c.A0 = A0;
  for (int k = 0; k < 3; ++k) {
    c.B0[k] = k < d ? B0[k] : 0.0;
    c.g[k] = k < d ? gchi[k] : 0.0;
  }
  c.Pe = Pe;
  c.eta = eta;
  c.diff = diff;
  c.calF = Pe * ubar_g;
  c.max_iter = o.max_iter;
  c.steady = steady ? 1 : 0;
  c.flux = flux ? 1 : 0;
  c.st[0].status = 1;
  c.st[1] = c.st[0];
  HIP_TRY(hipMemcpyAsync(dctl, &c, sizeof(c), hipMemcpyHostToDevice, s));

  // chi-hat^0 = FFT(chi^0); grad chi-hat^0 in the layout the local pass reads
  {
    hipError_t e = launch_rows_r2c<T>(g, tb, 1, chi, chat, s);
    if (e == hipSuccess) e = launch_cols<T>(g, tb, 1, -1, 1, chat, s);
    if (e == hipSuccess && d == 3) e = launch_cols<T>(g, tb, 2, -1, 1, chat, s);
    if (e == hipSuccess)
      e = launch_transport_green<T>(g, tb, 1, spec, chat, chat_m, part, dctl, 0, 0, 1, s, flux);
    if (e != hipSuccess) return fail(ACM_E_HIP, std::string("set-up: ") + hipGetErrorString(e));
  }

  Profiler prof;
  prof.on = o.profile != 0;
  prof.s = s;
  // Iterations alternate between the two state slots (see TransportState);
  // a captured graph holds an even number of them, so every replay starts on
  // slot 0.  On the slab path the stop test of iteration n is formed by the
  // slab pass of iteration n + 1 (no cross-workgroup traffic in the green pass).
  int tpar = 0;
  auto one_iter = [&]() -> hipError_t {
    hipError_t e;
    hipEvent_t ev0 = nullptr;
    const int par = tpar;
    tpar ^= 1;
    if (tslab) {
      prof.begin(KK_T_LOCAL, &ev0);
      e = launch_transport_slab<T>(g, tb, spec, u, H, dctl, part,
                                   transport_green_blocks(g, pl->prec, true), par, s);
      if (e != hipSuccess) return e;
      prof.end(KK_T_LOCAL, ev0);
      prof.begin(KK_T_GREEN, &ev0);
      e = launch_transport_green<T>(g, tb, 0, spec, chat, chat_m, part, dctl, 1, par ^ 1, 0, s);
      if (e != hipSuccess) return e;
      prof.end(KK_T_GREEN, ev0);
      return hipSuccess;
    }
    if (d == 3) {
      prof.begin(KK_YINV, &ev0);
      e = launch_cols<T>(g, tb, 1, +1, flux ? 2 * d : d, spec, s, &dctl->st[0].done,
                         &dctl->st[1].done);
      if (e != hipSuccess) return e;
      prof.end(KK_YINV, ev0);
    }
    prof.begin(KK_T_LOCAL, &ev0);
    e = launch_transport_local<T>(g, tb, spec, u, H, dctl, s, flux);
    if (e != hipSuccess) return e;
    prof.end(KK_T_LOCAL, ev0);
    if (d == 3) {
      prof.begin(KK_YFWD, &ev0);
      e = launch_cols<T>(g, tb, 1, -1, d + 1, spec, s, &dctl->st[0].done, &dctl->st[1].done);
      if (e != hipSuccess) return e;
      prof.end(KK_YFWD, ev0);
    }
    prof.begin(KK_T_GREEN, &ev0);
    e = launch_transport_green<T>(g, tb, 0, spec, chat, chat_m, part, dctl, 0, par, 1, s, flux);
    if (e != hipSuccess) return e;
    prof.end(KK_T_GREEN, ev0);
    return hipSuccess;
  };

  int K = o.check_every;
  if (K <= 0) K = 16;
  if (o.max_iter < K) K = (int)std::max<int64_t>(1, o.max_iter);
  K += K & 1;  // even: see one_iter
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  const bool use_graph = o.use_graph && !prof.on;
  if (use_graph) {
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int k = 0; k < K && e == hipSuccess; ++k) e = one_iter();
    hipError_t e2 = hipStreamEndCapture(s, &graph);
    if (e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return fail(ACM_E_HIP, std::string("kernel launch during capture: ") + hipGetErrorString(e));
    }
    HIP_TRY(e2);
    HIP_TRY(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
  }
  struct GraphFree {
    hipGraph_t g;
    hipGraphExec_t x;
    ~GraphFree() {
      if (x) (void)hipGraphExecDestroy(x);
      if (g) (void)hipGraphDestroy(g);
    }
  } gf{graph, exec};
  TransportCtl* hctl = nullptr;
  HIP_TRY(hipHostMalloc((void**)&hctl, sizeof(TransportCtl), hipHostMallocDefault));
  struct HostFree {
    void* p;
    ~HostFree() {
      if (p) (void)hipHostFree(p);
    }
  } hf{hctl};

  auto t0 = std::chrono::steady_clock::now();
  int64_t total = 0;
  int status = 0;
  for (int step = 0; step < n_steps; ++step) {
    if (!steady) HIP_TRY(hipMemcpyAsync(chat_m, chat, one_b, hipMemcpyDeviceToDevice, s));
    TransportState s0{};
    s0.iter = 0;
    s0.total_iter = total;
    s0.r1_min = INFINITY;
    s0.done = 0;
    s0.status = 1;
    s0.pend = 0;
    c.st[0] = s0;
    c.st[1] = s0;
    c.counter = 0;
    tpar = 0;
    HIP_TRY(hipMemcpyAsync(dctl, &c, sizeof(c), hipMemcpyHostToDevice, s));
    int64_t launched = 0;
    for (;;) {
      if (use_graph) {
        HIP_TRY(hipGraphLaunch(exec, s));
      } else {
        for (int k = 0; k < K; ++k) {
          hipError_t e = one_iter();
          if (e != hipSuccess) return fail(ACM_E_HIP, std::string("launch: ") + hipGetErrorString(e));
        }
      }
      launched += K;
      HIP_TRY(hipMemcpyAsync(hctl, dctl, sizeof(TransportCtl), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      prof.collect();
      if (transport_done(hctl)) break;
      if (launched > o.max_iter + 2LL * K) break;
    }
    const TransportState& ls = latest_tstate(*hctl);
    total = ls.total_iter;
    if (ls.status == -5) {
      status = -5;
      break;
    }
    if (ls.status != 0) status = 1;
  }
  auto t1 = std::chrono::steady_clock::now();
  if (status == -5) return fail(ACM_E_DIVERGED, "a transport residual became non-finite");
  // read-out: chi = inverse FFT of chi-hat
  HIP_TRY(hipMemcpyAsync(spec, chat, one_b, hipMemcpyDeviceToDevice, s));
  {
    hipError_t e = hipSuccess;
    if (d == 3) e = launch_cols<T>(g, tb, 2, +1, 1, spec, s);
    if (e == hipSuccess) e = launch_cols<T>(g, tb, 1, +1, 1, spec, s);
    if (e == hipSuccess) e = launch_rows_c2r<T>(g, tb, 1, spec, chi, 1.0 / (double)g.ntot, s);
    if (e != hipSuccess) return fail(ACM_E_HIP, hipGetErrorString(e));
  }
  HIP_TRY(hipStreamSynchronize(s));
  if (st) {
    memset(st, 0, sizeof(*st));
    st->iters = total;
    st->r_p[0] = latest_tstate(*hctl).r1;
    st->r_p[1] = latest_tstate(*hctl).r2;
    st->tol_p[0] = c.sqrt_n1 * o.eps;
    st->tol_p[1] = c.sqrt_n2 * o.eps;
    st->seconds = std::chrono::duration<double>(t1 - t0).count();
    st->converged = status == 0;
    st->status = status;
    for (int k = 0; k < KK_COUNT; ++k) {
      st->kernel_ms[k] = prof.ms[k];
      st->kernel_calls[k] = prof.calls[k];
    }
  }
  return status == 0 ? ACM_OK : ACM_NOT_CONVERGED;
}

// --------------------------------------------------------------- properties
// eq. K and eq. D from the FP64 totals of the reductions:
//   flow[i] = k_flow_sums totals of flow i (for K),
//   tr      = k_flow_sums totals of u_transport (pore volume and pore sums of u),
//   chi[j]  = k_chi_sums totals of chi^j.
// Host arithmetic only; both properties entry points call it.
static acm_status props_from_totals(const Geom& g, int n_flow, const double* const* flow,
                                    const double* tr, int n_chi, const double* const* chi,
                                    double nu, double Pe, double* K, double* D, double* mass) {
  const int d = g.dim;
  const double N = (double)g.ntot;
  if (K)
    for (int i = 0; i < n_flow; ++i)
      for (int j = 0; j < d; ++j) K[i * d + j] = flow[i][1 + d + j] / (N * nu);
  if (n_chi > 0 && (D || mass)) {
    const double npore = tr[0];
    if (!(npore > 0.0)) return fail(ACM_E_INVALID, "H has no pore voxel");
    double ubar[3] = {0.0, 0.0, 0.0};
    for (int c = 0; c < d; ++c) ubar[c] = tr[1 + c] / npore;
    const double por = npore / N;
    for (int j = 0; j < n_chi; ++j) {
      const double* cs = chi[j];
      if (mass) mass[j] = cs[0] / N;
      if (D)
        for (int i = 0; i < d; ++i)
          D[i * n_chi + j] = (i == j ? por : 0.0) + Pe * (ubar[i] * cs[1] - cs[2 + i]) / N +
                             cs[2 + d + i] / N;
    }
  }
  return ACM_OK;
}

template <typename T>
static acm_status props_impl(CellPlan* pl, const uint8_t* H, int n_flow, const void* const* u,
                             int n_chi, const void* const* chi, const void* u_tr, double nu,
                             double Pe, double* K, double* D, double* mass, hipStream_t caller) {
  const Geom& g = pl->g;
  hipStream_t s = work_stream(pl->device);
  if (!s) return fail(ACM_E_HIP, "cannot create work stream");
  HIP_TRY(join_from(caller, s));
  std::vector<std::vector<double>> fl(K ? n_flow : 0), cs;
  std::vector<double> tr;
  for (size_t i = 0; i < fl.size(); ++i) {
    acm_status r = reduce_on_host(g, s, &fl[i], [&](double* part, int* ns) {
      return launch_flow_sums<T>(g, (const T*)u[i], H, part, ns, s);
    });
    if (r != ACM_OK) return r;
  }
  const bool want_chi = n_chi > 0 && (D || mass);
  if (want_chi) {
    acm_status r = reduce_on_host(g, s, &tr, [&](double* part, int* ns) {
      return launch_flow_sums<T>(g, (const T*)u_tr, H, part, ns, s);
    });
    if (r != ACM_OK) return r;
    cs.resize(n_chi);
    for (int j = 0; j < n_chi; ++j) {
      r = reduce_on_host(g, s, &cs[j], [&](double* part, int* ns) {
        return launch_chi_sums<T>(g, (const T*)chi[j], (const T*)u_tr, H, part, ns, s);
      });
      if (r != ACM_OK) return r;
    }
  }
  HIP_TRY(hipStreamSynchronize(s));
  std::vector<const double*> flp, csp;
  for (auto& v : fl) flp.push_back(v.data());
  for (auto& v : cs) csp.push_back(v.data());
  return props_from_totals(g, (int)fl.size(), flp.data(), tr.data(), want_chi ? n_chi : 0,
                           csp.data(), nu, Pe, K, D, mass);
}

// ------------------------------------------------- allocation-free properties
// acm_effective_props_noalloc keeps its partial sums in this file-scope array,
// which every GPU holds for the life of the process:
//   [0, kNaPart)               per-block records of the reduction in flight
//                              (every reduction of a call reuses them, in
//                              stream order);
//   [kNaPart, kNaPart + kNaTot) one record of totals per reduction.
// Every kernel writes all of the records it owns before they are read, so
// nothing needs clearing between calls.  Calls that overlap on one GPU share
// the array and race.
constexpr int kNaMaxReductions = 33;  // n_flow <= 16, plus u_transport and n_chi <= 16
constexpr int kNaPart = kReductionBlocksMax * kReductionSumsMax;
constexpr int kNaTot = kNaMaxReductions * kReductionSumsMax;
constexpr int kNaMaxDevices = 64;
static __device__ __align__(256) double scratch[kNaPart + kNaTot];

static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kNaMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device (the name itself is a host-side stand-in, not a device address).
static acm_status scratch_address(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(ACM_E_HIP, hipGetErrorString(e));
  if (dev < 0 || dev >= kNaMaxDevices)
    return fail(ACM_E_INVALID, "device index above the allocation-free table (64 devices)");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return fail(ACM_E_HIP, "hipGetSymbolAddress(scratch) failed");
    g_scratch_ptr[dev] = (double*)p;
  }
  *out = g_scratch_ptr[dev];
  return ACM_OK;
}

template <typename T>
static acm_status props_noalloc_impl(const Geom& g, double* sc, const uint8_t* H, int n_flow,
                                     const void* const* u, int n_chi, const void* const* chi,
                                     const void* u_tr, double nu, double Pe, double* K, double* D,
                                     double* mass, hipStream_t s) {
  double* part = sc;
  double* tot = sc + kNaPart;
  const int nb = reduction_blocks(g);
  const int nf = K ? n_flow : 0;
  const int nc = (n_chi > 0 && (D || mass)) ? n_chi : 0;
  const int nred = nf + (nc > 0 ? 1 + nc : 0);
  int ns = 0;
  hipError_t e = hipSuccess;
  for (int r = 0; r < nred && e == hipSuccess; ++r) {
    if (r < nf)
      e = launch_flow_sums<T>(g, (const T*)u[r], H, part, &ns, s);
    else if (r == nf)
      e = launch_flow_sums<T>(g, (const T*)u_tr, H, part, &ns, s);
    else
      e = launch_chi_sums<T>(g, (const T*)chi[r - nf - 1], (const T*)u_tr, H, part, &ns, s);
    if (e == hipSuccess) e = launch_sum_partials(part, nb, ns, tot + r * kReductionSumsMax, s);
  }
  if (e != hipSuccess) return fail(ACM_E_HIP, hipGetErrorString(e));
  double host[kNaTot];
  if (nred > 0) {
    e = hipMemcpyAsync(host, tot, sizeof(double) * kReductionSumsMax * nred,
                       hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(ACM_E_HIP, hipGetErrorString(e));
  }
  const double* flp[16];
  const double* csp[16];
  for (int i = 0; i < nf; ++i) flp[i] = host + i * kReductionSumsMax;
  for (int j = 0; j < nc; ++j) csp[j] = host + (nf + 1 + j) * kReductionSumsMax;
  return props_from_totals(g, nf, flp, host + nf * kReductionSumsMax, nc, csp, nu, Pe, K, D,
                           mass);
}

// --------------------------------------------------------------------- FFT
template <typename T>
static acm_status fft_impl(CellPlan* pl, int nfields, const void* in, void* out, bool forward,
                           hipStream_t caller) {
  const Geom& g = pl->g;
  DevTables<T> tb = tables_of<T>(pl);
  hipStream_t s = work_stream(pl->device);
  if (!s) return fail(ACM_E_HIP, "cannot create work stream");
  HIP_TRY(join_from(caller, s));
  hipError_t e;
  if (forward) {
    e = launch_rows_r2c<T>(g, tb, nfields, (const T*)in, out, s);
    if (e == hipSuccess) e = launch_cols<T>(g, tb, 1, -1, nfields, out, s);
    if (e == hipSuccess && g.dim == 3) e = launch_cols<T>(g, tb, 2, -1, nfields, out, s);
    if (e != hipSuccess) return fail(ACM_E_HIP, hipGetErrorString(e));
  } else {
    DevBuf tmp;
    const size_t b = sizeof(T) * 2 * (size_t)g.nspec * nfields;
    HIP_TRY(hipMalloc(&tmp.p, b));
    HIP_TRY(hipMemcpyAsync(tmp.p, in, b, hipMemcpyDeviceToDevice, s));
    e = hipSuccess;
    if (g.dim == 3) e = launch_cols<T>(g, tb, 2, +1, nfields, tmp.p, s);
    if (e == hipSuccess) e = launch_cols<T>(g, tb, 1, +1, nfields, tmp.p, s);
    if (e == hipSuccess) e = launch_rows_c2r<T>(g, tb, nfields, tmp.p, (T*)out, 1.0 / (double)g.ntot, s);
    if (e != hipSuccess) return fail(ACM_E_HIP, hipGetErrorString(e));
    HIP_TRY(hipStreamSynchronize(s));
  }
  HIP_TRY(hipStreamSynchronize(s));
  return ACM_OK;
}


// --------------------------------------------------------------------- FNO
// Parameter layout (FP32 master / BF16 copy, complex weights as (re, im)):
//   Pw[C] Pb[C] | per layer: R[nm][C][C] complex, W[C][C], b[C] | Q1[Cp][C]
//   c1[Cp] Q2[4][Cp] c2[4],  nm = (2m)^2 m kept modes.
struct FnoLayout {
  int C, Cp, m, L, nm;
  int64_t Pw, Pb, R[16], W[16], b[16], Q1, c1, Q2, c2, total;
};

static bool fno_layout(const acm_fno_shape* sh, FnoLayout* f) {
  if (!sh) return false;
  f->C = sh->channels;
  f->Cp = sh->hidden;
  f->m = sh->modes;
  f->L = sh->layers;
  if (!(f->C == 4 || f->C == 8 || f->C == 16 || f->C == 32)) return false;
  if (f->Cp < 1 || f->Cp * f->C > 4096 || f->Cp > 1024) return false;
  if (f->m < 1 || f->L < 1 || f->L > 16) return false;
  f->nm = (2 * f->m) * (2 * f->m) * f->m;
  int64_t o = 0;
  f->Pw = o;
  o += f->C;
  f->Pb = o;
  o += f->C;
  for (int l = 0; l < f->L; ++l) {
    f->R[l] = o;
    o += 2LL * f->nm * f->C * f->C;
    f->W[l] = o;
    o += (int64_t)f->C * f->C;
    f->b[l] = o;
    o += f->C;
  }
  f->Q1 = o;
  o += (int64_t)f->Cp * f->C;
  f->c1 = o;
  o += f->Cp;
  f->Q2 = o;
  o += 4LL * f->Cp;
  f->c2 = o;
  o += 4;
  f->total = o;
  return true;
}

// Workspace carve-up (train = 1 keeps every layer's activations for backward).
struct FnoWs {
  float* vs[17];
  float* pre[16];
  float2* Xm[16];
  float2* spec;
  float* kbuf;
  float* dv;
  float* dvdir;
  float* dpre;
  float* h;
  float* dh;
  float2* Fm;
  float* part;
  int* midx;
  float* mw;
  int64_t bytes;
};

static int64_t fno_ws_plan(const FnoLayout& f, const Geom& g, int B, int train, char* base, FnoWs* w) {
  const int64_t nv = g.ntot;
  const int64_t act = (int64_t)B * f.C * nv * 4;
  const int64_t xm = (int64_t)B * f.C * f.nm * 8;
  int64_t o = 0;
  auto take = [&](int64_t b) {
    char* p = base ? base + o : nullptr;
    o += (b + 255) & ~(int64_t)255;
    return p;
  };
  const int nact = train ? f.L + 1 : 2;
  for (int l = 0; l < nact; ++l) w->vs[l] = (float*)take(act);
  if (train)
    for (int l = 0; l < f.L; ++l) w->pre[l] = (float*)take(act);
  for (int l = 0; l < (train ? f.L : 1); ++l) w->Xm[l] = (float2*)take(xm);
  w->spec = (float2*)take((int64_t)B * f.C * g.nspec * 8);
  w->kbuf = (float*)take(act);
  w->midx = (int*)take(4LL * f.nm);
  w->mw = (float*)take(4LL * f.nm);
  if (train) {
    w->dv = (float*)take(act);
    w->dvdir = (float*)take(act);
    w->dpre = (float*)take(act);
    w->h = (float*)take((int64_t)B * f.Cp * nv * 4);
    w->dh = (float*)take((int64_t)B * f.Cp * nv * 4);
    w->Fm = (float2*)take(xm);
    w->part = (float*)take(4LL * fno_outer_blocks(nv, B) * 4096);
  }
  w->bytes = o;
  return o;
}

static acm_status fno_check(const acm_fno_shape* sh, const acm_grid* grid, int B, CellPlan** pl,
                            FnoLayout* f) {
  if (!fno_layout(sh, f))
    return fail(ACM_E_INVALID, "fno shape: channels in {4,8,16,32}, hidden*channels <= 4096, modes >= 1, 1 <= layers <= 16");
  acm_status r = get_plan(grid, ACM_FP32, pl);
  if (r != ACM_OK) return r;
  const Geom& g = (*pl)->g;
  if (g.dim != 3 || g.nx != g.ny || g.ny != g.nz) return fail(ACM_E_INVALID, "fno needs a cubic 3D grid");
  if (2 * f->m > g.nx) return fail(ACM_E_INVALID, "fno modes must satisfy 2*modes <= n");
  if (B < 1) return fail(ACM_E_INVALID, "batch >= 1 required");
  return ACM_OK;
}

static hipError_t fno_mode_tables(const FnoLayout& f, const Geom& g, FnoWs& w, hipStream_t s) {
  std::vector<int> mi(f.nm);
  std::vector<float> mw(f.nm);
  std::vector<int> idx;
  for (int k = 0; k < f.m; ++k) idx.push_back(k);
  for (int k = g.nx - f.m; k < g.nx; ++k) idx.push_back(k);
  int j = 0;
  for (int kz : idx)
    for (int ky : idx)
      for (int kx = 0; kx < f.m; ++kx, ++j) {
        mi[j] = (kz * g.ny + ky) * g.xh + kx;
        mw[j] = (kx == 0 || 2 * kx == g.nx) ? 1.f : 2.f;
      }
  hipError_t e = hipMemcpyAsync(w.midx, mi.data(), 4 * mi.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(w.mw, mw.data(), 4 * mw.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);  // host vectors go out of scope
  return e;
}

// Forward real FFT of nf fields (in) into spec; inverse (spec -> out, normalised).
static hipError_t fno_fft_fwd(const Geom& g, const DevTables<float>& tb, int nf, const float* in,
                              void* spec, hipStream_t s) {
  hipError_t e = launch_rows_r2c<float>(g, tb, nf, in, spec, s);
  if (e == hipSuccess) e = launch_cols<float>(g, tb, 1, -1, nf, spec, s);
  if (e == hipSuccess) e = launch_cols<float>(g, tb, 2, -1, nf, spec, s);
  return e;
}
static hipError_t fno_fft_inv(const Geom& g, const DevTables<float>& tb, int nf, void* spec,
                              float* out, hipStream_t s) {
  hipError_t e = launch_cols<float>(g, tb, 2, +1, nf, spec, s);
  if (e == hipSuccess) e = launch_cols<float>(g, tb, 1, +1, nf, spec, s);
  if (e == hipSuccess) e = launch_rows_c2r<float>(g, tb, nf, spec, out, 1.0 / (double)g.ntot, s);
  return e;
}

#define FNO_TRY(expr)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) return fail(ACM_E_HIP, std::string("fno: ") + #expr + ": " +    \
                                                     hipGetErrorString(e_));             \
  } while (0)

static acm_status fno_forward_impl(const FnoLayout& f, CellPlan* pl, int B, const uint16_t* P,
                                   const uint8_t* H, float* out, FnoWs& w, int train,
                                   hipStream_t s) {
  const Geom& g = pl->g;
  DevTables<float> tb = tables_of<float>(pl);
  const int64_t nv = g.ntot;
  const int nf = B * f.C;
  FNO_TRY(fno_mode_tables(f, g, w, s));
  FNO_TRY(fno_lift(H, P + f.Pw, P + f.Pb, w.vs[0], f.C, nv, B, s));
  for (int l = 0; l < f.L; ++l) {
    float* vin = train ? w.vs[l] : w.vs[l & 1];
    float* vout = train ? w.vs[l + 1] : w.vs[(l + 1) & 1];
    float2* Xm = train ? w.Xm[l] : w.Xm[0];
    FNO_TRY(fno_fft_fwd(g, tb, nf, vin, w.spec, s));
    FNO_TRY(fno_gather(w.spec, Xm, w.midx, f.nm, g.nspec, nf, s));
    FNO_TRY(hipMemsetAsync(w.spec, 0, (size_t)nf * g.nspec * 8, s));
    FNO_TRY(fno_mix(Xm, P + f.R[l], w.spec, w.midx, f.nm, f.C, B, g.nspec, false, s));
    FNO_TRY(fno_fft_inv(g, tb, nf, w.spec, w.kbuf, s));
    FNO_TRY(fno_pointwise(f.C, vin, w.kbuf, P + f.W[l], P + f.b[l], train ? w.pre[l] : nullptr,
                          vout, nv, B, l < f.L - 1 ? 1 : 0, s));
  }
  float* vl = train ? w.vs[f.L] : w.vs[f.L & 1];
  FNO_TRY(fno_project(f.C, vl, P + f.Q1, P + f.c1, P + f.Q2, P + f.c2, out, f.Cp, nv, B, s));
  return ACM_OK;
}

static acm_status fno_backward_impl(const FnoLayout& f, CellPlan* pl, int B, const uint16_t* P,
                                    const uint8_t* H, const float* dout, float* grad, FnoWs& w,
                                    hipStream_t s) {
  const Geom& g = pl->g;
  DevTables<float> tb = tables_of<float>(pl);
  const int64_t nv = g.ntot;
  const int nf = B * f.C;
  const int64_t nact = (int64_t)nf * nv;
  // projection
  FNO_TRY(fno_project_bwd(f.C, w.vs[f.L], dout, P + f.Q1, P + f.c1, P + f.Q2, w.h, w.dh, w.dv,
                          f.Cp, nv, B, s));
  FNO_TRY(fno_outer(w.dh, w.vs[f.L], nullptr, f.Cp, f.C, nv, B, w.part, grad + f.Q1, s));
  FNO_TRY(fno_outer(w.dh, nullptr, nullptr, f.Cp, 1, nv, B, w.part, grad + f.c1, s));
  FNO_TRY(fno_outer(dout, w.h, nullptr, 4, f.Cp, nv, B, w.part, grad + f.Q2, s));
  FNO_TRY(fno_outer(dout, nullptr, nullptr, 4, 1, nv, B, w.part, grad + f.c2, s));
  for (int l = f.L - 1; l >= 0; --l) {
    FNO_TRY(fno_pointwise_bwd(f.C, w.dv, w.pre[l], P + f.W[l], w.dpre, w.dvdir, nv, B,
                              l < f.L - 1 ? 1 : 0, s));
    FNO_TRY(fno_outer(w.dpre, w.vs[l], nullptr, f.C, f.C, nv, B, w.part, grad + f.W[l], s));
    FNO_TRY(fno_outer(w.dpre, nullptr, nullptr, f.C, 1, nv, B, w.part, grad + f.b[l], s));
    // spectral path: F = FFT(dpre); dR = sum_b (w/N) F conj(X); dv_spec = iFFT(R^H F)
    FNO_TRY(fno_fft_fwd(g, tb, nf, w.dpre, w.spec, s));
    FNO_TRY(fno_gather(w.spec, w.Fm, w.midx, f.nm, g.nspec, nf, s));
    FNO_TRY(fno_dR(w.Fm, w.Xm[l], w.mw, grad + f.R[l], f.nm, f.C, B, (float)(1.0 / (double)nv), s));
    FNO_TRY(hipMemsetAsync(w.spec, 0, (size_t)nf * g.nspec * 8, s));
    FNO_TRY(fno_mix(w.Fm, P + f.R[l], w.spec, w.midx, f.nm, f.C, B, g.nspec, true, s));
    FNO_TRY(fno_fft_inv(g, tb, nf, w.spec, w.dv, s));
    FNO_TRY(fno_add(w.dv, w.dvdir, nact, s));
  }
  FNO_TRY(fno_outer(w.dv, nullptr, H, f.C, 1, nv, B, w.part, grad + f.Pw, s));
  FNO_TRY(fno_outer(w.dv, nullptr, nullptr, f.C, 1, nv, B, w.part, grad + f.Pb, s));
  return ACM_OK;
}

}  // namespace acm

// ===================================================================== C ABI
using namespace acm;

extern "C" {

void acm_default_penalty(acm_penalty* p) {
  if (!p) return;
  memset(p, 0, sizeof(*p));
  for (int k = 0; k < 3; ++k) p->phi[k] = 1.1;
  p->tau[0] = 5.0;
  p->tau[1] = 10.0;
  p->tau[2] = 5.0;
  p->adaptive = 1;
}

void acm_default_opts(acm_opts* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->eps = 1e-6;
  o->max_iter = 1000000;
  o->precision = ACM_FP32;
  o->use_graph = 1;
}

const char* acm_last_error(void) { return g_err.c_str(); }

int32_t acm_version(void) { return 6; }

acm_status acm_stokes_solve(const acm_grid* grid, const uint8_t* H, const double* g_p, double nu,
                            const acm_penalty* pen, const acm_opts* opts, void* u, void* q,
                            acm_stats* stats, double* history, void* stream) {
  g_err.clear();
  acm_penalty P;
  acm_opts O;
  acm_default_penalty(&P);
  acm_default_opts(&O);
  if (pen) P = *pen;
  if (opts) O = *opts;
  acm_status r = check_penalty_opts(P, O, nu);
  if (r != ACM_OK) return r;
  CellPlan* pl = nullptr;
  bool solid = false;
  r = check_stokes_cell(grid, H, g_p, u, O.precision, O.derivative, (hipStream_t)stream, &pl,
                        &solid);
  if (r != ACM_OK) return r;
  if (solid) return stokes_all_solid(pl, u, q, stats, (hipStream_t)stream);
  StokesCellIn c{H, {0, 0, 0}, u, q};
  for (int k = 0; k < grid->dim; ++k) c.g[k] = g_p[k];
  std::vector<CellPlan*> plans{pl};
  std::vector<StokesCellIn> cells{c};
  if (O.precision == ACM_FP64)
    return stokes_run<double>(plans, cells, nu, P, O, stats, history, (hipStream_t)stream);
  return stokes_run<float>(plans, cells, nu, P, O, stats, history, (hipStream_t)stream);
}

acm_status acm_stokes_solve_batched(int32_t ncell, const acm_grid* grids, const uint8_t* const* H,
                                    const double* g_p, double nu, const acm_penalty* pen,
                                    const acm_opts* opts, void* const* u, void* const* q,
                                    acm_stats* stats, void* stream) {
  g_err.clear();
  if (ncell < 1 || !grids || !H || !g_p || !u) return fail(ACM_E_INVALID, "ncell >= 1 and non-NULL arrays required");
  acm_penalty P;
  acm_opts O;
  acm_default_penalty(&P);
  acm_default_opts(&O);
  if (pen) P = *pen;
  if (opts) O = *opts;
  acm_status r = check_penalty_opts(P, O, nu);
  if (r != ACM_OK) return r;
  // all-solid cells are answered at once (u = 0, q = 0); the others run
  std::vector<CellPlan*> plans;
  std::vector<StokesCellIn> cells;
  std::vector<int> active;
  std::vector<CellPlan*> solid_plan(ncell, nullptr);
  for (int i = 0; i < ncell; ++i) {
    CellPlan* pl = nullptr;
    bool solid = false;
    r = check_stokes_cell(grids + i, H[i], g_p + 3 * i, u[i], O.precision, O.derivative,
                          (hipStream_t)stream, &pl, &solid);
    if (r != ACM_OK) return fail(r, "cell " + std::to_string(i) + ": " + g_err);
    if (solid) {
      solid_plan[i] = pl;
      continue;
    }
    active.push_back(i);
    plans.push_back(pl);
    cells.push_back(StokesCellIn{H[i], {g_p[3 * i], g_p[3 * i + 1], g_p[3 * i + 2]}, u[i],
                                 q ? q[i] : nullptr});
  }
  for (int i = 0; i < ncell; ++i)
    if (solid_plan[i]) {
      r = stokes_all_solid(solid_plan[i], u[i], q ? q[i] : nullptr, stats ? stats + i : nullptr,
                           (hipStream_t)stream);
      if (r != ACM_OK) return r;
    }
  if (active.empty()) return ACM_OK;
  std::vector<acm_stats> st(active.size());
  r = O.precision == ACM_FP64
          ? stokes_run<double>(plans, cells, nu, P, O, stats ? st.data() : nullptr, nullptr,
                               (hipStream_t)stream)
          : stokes_run<float>(plans, cells, nu, P, O, stats ? st.data() : nullptr, nullptr,
                              (hipStream_t)stream);
  if (stats && r >= 0)
    for (size_t k = 0; k < active.size(); ++k) stats[active[k]] = st[k];
  return r;
}

acm_status acm_fft_r2c(const acm_grid* grid, int32_t precision, int32_t nfields, const void* in,
                       void* out, void* stream) {
  g_err.clear();
  if (!in || !out || nfields < 1) return fail(ACM_E_INVALID, "in/out non-NULL and nfields >= 1 required");
  CellPlan* pl = nullptr;
  acm_status r = get_plan(grid, precision, &pl);
  if (r != ACM_OK) return r;
  if (precision == ACM_FP64) return fft_impl<double>(pl, nfields, in, out, true, (hipStream_t)stream);
  return fft_impl<float>(pl, nfields, in, out, true, (hipStream_t)stream);
}

acm_status acm_fft_c2r(const acm_grid* grid, int32_t precision, int32_t nfields, const void* in,
                       void* out, void* stream) {
  g_err.clear();
  if (!in || !out || nfields < 1) return fail(ACM_E_INVALID, "in/out non-NULL and nfields >= 1 required");
  CellPlan* pl = nullptr;
  acm_status r = get_plan(grid, precision, &pl);
  if (r != ACM_OK) return r;
  if (precision == ACM_FP64) return fft_impl<double>(pl, nfields, in, out, false, (hipStream_t)stream);
  return fft_impl<float>(pl, nfields, in, out, false, (hipStream_t)stream);
}

acm_status acm_transport_step(const acm_grid* grid, const uint8_t* H, const void* u,
                              const double* g_chi, double Pe, double diffusivity, double eta,
                              double A0, const double* B0, double dt, int32_t n_steps,
                              const acm_opts* opts, void* chi, acm_stats* stats, void* stream) {
  g_err.clear();
  acm_opts O;
  acm_default_opts(&O);
  if (opts) O = *opts;
  if (!H || !u || !g_chi || !B0 || !chi) return fail(ACM_E_INVALID, "H, u, g_chi, B0, chi must be non-NULL");
  if (!(A0 > 0.0) || !isfinite(A0)) return fail(ACM_E_INVALID, "A0 must be positive");
  if (!(eta > 0.0) || !(diffusivity > 0.0)) return fail(ACM_E_INVALID, "eta and diffusivity must be positive");
  if (!isfinite(Pe)) return fail(ACM_E_INVALID, "Pe must be finite");
  if (n_steps < 1) return fail(ACM_E_INVALID, "n_steps >= 1 required");
  if (isfinite(dt) ? !(dt > 0.0) : !(dt > 0.0)) return fail(ACM_E_INVALID, "dt must be > 0 or +INFINITY");
  if (!isfinite(dt) && n_steps != 1) return fail(ACM_E_INVALID, "the steady problem takes n_steps = 1");
  if (!(O.eps >= 0.0) || O.max_iter < 1) return fail(ACM_E_INVALID, "eps >= 0 and max_iter >= 1 required");
  if (O.transport_form != 0 && O.transport_form != 1)
    return fail(ACM_E_INVALID, "transport_form must be 0 or 1");
  CellPlan* pl = nullptr;
  acm_status r = get_plan(grid, O.precision, &pl, O.derivative);
  if (r != ACM_OK) return r;
  for (int k = 0; k < grid->dim; ++k)
    if (!isfinite(g_chi[k]) || !isfinite(B0[k])) return fail(ACM_E_INVALID, "g_chi, B0 must be finite");
  if (O.precision == ACM_FP64)
    return transport_impl<double>(pl, H, (const double*)u, g_chi, Pe, diffusivity, eta, A0, B0, dt,
                                  n_steps, O, (double*)chi, stats, (hipStream_t)stream);
  return transport_impl<float>(pl, H, (const float*)u, g_chi, Pe, diffusivity, eta, A0, B0, dt,
                               n_steps, O, (float*)chi, stats, (hipStream_t)stream);
}

acm_status acm_effective_props(const acm_grid* grid, int32_t precision, const uint8_t* H,
                               int32_t n_flow, const void* const* u, int32_t n_chi,
                               const void* const* chi, const void* u_transport, double nu,
                               double Pe, double* K, double* D, double* mass, void* stream) {
  g_err.clear();
  if (!H) return fail(ACM_E_INVALID, "H must be non-NULL");
  if (n_flow < 0 || n_chi < 0) return fail(ACM_E_INVALID, "counts must be >= 0");
  if (K && n_flow > 0 && !u) return fail(ACM_E_INVALID, "u must be non-NULL when K is requested");
  if (n_chi > 0 && (D || mass) && (!chi || !u_transport))
    return fail(ACM_E_INVALID, "chi and u_transport must be non-NULL when D or mass is requested");
  if (K && !(nu > 0.0)) return fail(ACM_E_INVALID, "nu must be positive");
  CellPlan* pl = nullptr;
  acm_status r = get_plan(grid, precision, &pl);
  if (r != ACM_OK) return r;
  if (K)
    for (int i = 0; i < n_flow; ++i)
      if (!u[i]) return fail(ACM_E_INVALID, "null flow field");
  if (n_chi > 0 && (D || mass))
    for (int j = 0; j < n_chi; ++j)
      if (!chi[j]) return fail(ACM_E_INVALID, "null chi field");
  if (precision == ACM_FP64)
    return props_impl<double>(pl, H, n_flow, u, n_chi, chi, u_transport, nu, Pe, K, D, mass,
                              (hipStream_t)stream);
  return props_impl<float>(pl, H, n_flow, u, n_chi, chi, u_transport, nu, Pe, K, D, mass,
                           (hipStream_t)stream);
}

acm_status acm_effective_props_noalloc(const acm_grid* grid, int32_t precision,
                                       const uint8_t* H, int32_t n_flow, const void* const* u,
                                       int32_t n_chi, const void* const* chi,
                                       const void* u_transport, double nu, double Pe, double* K,
                                       double* D, double* mass, void* stream) {
  if (!H) return fail(ACM_E_INVALID, "H must be non-NULL");
  if (n_flow < 0 || n_chi < 0) return fail(ACM_E_INVALID, "counts must be >= 0");
  if (n_flow > 16 || n_chi > 16)
    return fail(ACM_E_INVALID, "allocation-free properties take at most 16 flows and 16 chi fields");
  if (K && n_flow > 0 && !u) return fail(ACM_E_INVALID, "u must be non-NULL when K is requested");
  if (n_chi > 0 && (D || mass) && (!chi || !u_transport))
    return fail(ACM_E_INVALID, "chi and u_transport must be non-NULL when D or mass is requested");
  if (K && !(nu > 0.0)) return fail(ACM_E_INVALID, "nu must be positive");
  if (precision != ACM_FP32 && precision != ACM_FP64)
    return fail(ACM_E_INVALID, "precision must be ACM_FP32 or ACM_FP64");
  Geom g;
  const char* why = nullptr;
  if (!make_geom(grid, &g, &why)) return fail(ACM_E_INVALID, why);
  if (!size_supported(g)) return fail(ACM_E_UNSUPPORTED_SIZE, kUnsupportedSizeMsg);
  if (K)
    for (int i = 0; i < n_flow; ++i)
      if (!u[i]) return fail(ACM_E_INVALID, "null flow field");
  if (n_chi > 0 && (D || mass))
    for (int j = 0; j < n_chi; ++j)
      if (!chi[j]) return fail(ACM_E_INVALID, "null chi field");
  double* sc = nullptr;
  acm_status r = scratch_address(&sc);
  if (r != ACM_OK) return r;
  if (precision == ACM_FP64)
    return props_noalloc_impl<double>(g, sc, H, n_flow, u, n_chi, chi, u_transport, nu, Pe, K, D,
                                      mass, (hipStream_t)stream);
  return props_noalloc_impl<float>(g, sc, H, n_flow, u, n_chi, chi, u_transport, nu, Pe, K, D,
                                   mass, (hipStream_t)stream);
}

int64_t acm_fno_param_count(const acm_fno_shape* shape) {
  FnoLayout f;
  if (!fno_layout(shape, &f)) return -1;
  return f.total;
}

int64_t acm_fno_workspace_bytes(const acm_fno_shape* shape, const acm_grid* grid, int32_t batch,
                                int32_t train) {
  g_err.clear();
  FnoLayout f;
  CellPlan* pl = nullptr;
  if (fno_check(shape, grid, batch, &pl, &f) != ACM_OK) return -1;
  FnoWs w;
  return fno_ws_plan(f, pl->g, batch, train, nullptr, &w);
}

acm_status acm_fno_forward(const acm_fno_shape* shape, const acm_grid* grid, int32_t batch,
                           const uint16_t* params_bf16, const uint8_t* H, float* out,
                           void* workspace, int64_t workspace_bytes, int32_t train,
                           void* stream) {
  g_err.clear();
  if (!params_bf16 || !H || !out || !workspace) return fail(ACM_E_INVALID, "null argument");
  if ((uintptr_t)params_bf16 % 4 != 0) return fail(ACM_E_INVALID, "params_bf16 must be 4-byte aligned");
  FnoLayout f;
  CellPlan* pl = nullptr;
  acm_status r = fno_check(shape, grid, batch, &pl, &f);
  if (r != ACM_OK) return r;
  FnoWs w;
  if (fno_ws_plan(f, pl->g, batch, train, (char*)workspace, &w) > workspace_bytes)
    return fail(ACM_E_INVALID, "workspace too small (see acm_fno_workspace_bytes)");
  hipStream_t s = work_stream(pl->device);
  if (!s) return fail(ACM_E_HIP, "cannot create work stream");
  HIP_TRY(join_from((hipStream_t)stream, s));
  r = fno_forward_impl(f, pl, batch, params_bf16, H, out, w, train ? 1 : 0, s);
  if (r != ACM_OK) return r;
  HIP_TRY(hipStreamSynchronize(s));
  return ACM_OK;
}

acm_status acm_fno_backward(const acm_fno_shape* shape, const acm_grid* grid, int32_t batch,
                            const uint16_t* params_bf16, const uint8_t* H, const float* dout,
                            float* grad, void* workspace, int64_t workspace_bytes, void* stream) {
  g_err.clear();
  if (!params_bf16 || !H || !dout || !grad || !workspace) return fail(ACM_E_INVALID, "null argument");
  if ((uintptr_t)params_bf16 % 4 != 0) return fail(ACM_E_INVALID, "params_bf16 must be 4-byte aligned");
  FnoLayout f;
  CellPlan* pl = nullptr;
  acm_status r = fno_check(shape, grid, batch, &pl, &f);
  if (r != ACM_OK) return r;
  FnoWs w;
  if (fno_ws_plan(f, pl->g, batch, 1, (char*)workspace, &w) > workspace_bytes)
    return fail(ACM_E_INVALID, "workspace too small (see acm_fno_workspace_bytes with train = 1)");
  hipStream_t s = work_stream(pl->device);
  if (!s) return fail(ACM_E_HIP, "cannot create work stream");
  HIP_TRY(join_from((hipStream_t)stream, s));
  r = fno_backward_impl(f, pl, batch, params_bf16, H, dout, grad, w, s);
  if (r != ACM_OK) return r;
  HIP_TRY(hipStreamSynchronize(s));
  return ACM_OK;
}

acm_status acm_fno_adam(int64_t n, float* params, uint16_t* params_bf16, const float* grad,
                        float* m, float* v, int64_t step, double lr, double beta1, double beta2,
                        double eps, void* stream) {
  g_err.clear();
  if (n < 1 || !params || !params_bf16 || !grad || !m || !v || step < 1)
    return fail(ACM_E_INVALID, "bad Adam arguments");
  hipStream_t s = (hipStream_t)stream;
  const double c1 = 1.0 - pow(beta1, (double)step), c2 = 1.0 - pow(beta2, (double)step);
  HIP_TRY(fno_adam(params, params_bf16, grad, m, v, n, (float)lr, (float)beta1, (float)beta2,
                   (float)eps, (float)c1, (float)c2, s));
  HIP_TRY(hipStreamSynchronize(s));
  return ACM_OK;
}

acm_status acm_fno_to_bf16(int64_t n, const float* params, uint16_t* params_bf16, void* stream) {
  g_err.clear();
  if (n < 1 || !params || !params_bf16) return fail(ACM_E_INVALID, "bad arguments");
  HIP_TRY(fno_to_bf16(params, params_bf16, n, (hipStream_t)stream));
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  return ACM_OK;
}

acm_status acm_fno_mse(int64_t n, const float* out, const float* target, float* dout,
                       double* loss, void* stream) {
  g_err.clear();
  if (n < 1 || !out || !target || !dout) return fail(ACM_E_INVALID, "bad arguments");
  hipStream_t s = (hipStream_t)stream;
  const int nb = 256;
  DevBuf part;
  HIP_TRY(hipMalloc(&part.p, sizeof(double) * nb));
  HIP_TRY(fno_mse(out, target, dout, n, 1.0 / (double)n, (double*)part.p, nb, s));
  std::vector<double> h(nb);
  HIP_TRY(hipMemcpyAsync(h.data(), part.p, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  double t = 0.0;
  for (double x : h) t += x;
  if (loss) *loss = t;
  return ACM_OK;
}

}  // extern "C"
