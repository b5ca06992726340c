// C ABI: operator creation, apply, GMRES solve (host orchestration).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <string>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>
#include <vector>

#include "ls.h"
#include "ls_host.h"
#include "ls_kernels.hpp"
#include "ls_setup.hpp"

using lsx::cd;

namespace {
thread_local std::string g_err;
ls_status fail(ls_status s, const std::string& msg) {
  g_err = msg;
  return s;
}
#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) return fail(LS_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

struct Fp32c { float x, y; };
struct Fp64c { double x, y; };
}  // namespace

struct ls_host_op {
  lsx::HostOp h;
};

// Device scratch of ls_apply_noalloc: a file-scope array (each device that
// loads the library holds its own copy until the process ends).  Host code
// never passes the array's name to a kernel: it is a host-side stand-in;
// the per-device address comes from hipGetSymbolAddress at set-up.
constexpr size_t LS_NOALLOC_SCRATCH_BYTES = size_t(96) << 20;
static __device__ __align__(256) unsigned char scratch[LS_NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;     // device -> address of its scratch copy

// called with `device` current (ls_create); once per device
hipError_t init_scratch(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr.count(device)) return hipSuccess;
  void* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
  if (e == hipSuccess && ptr) g_scratch_ptr[device] = ptr;
  return e;
}

void* scratch_of(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(device);
  return it == g_scratch_ptr.end() ? nullptr : it->second;
}
}  // namespace

using GraphKey = std::tuple<bool, bool, int, int, int, uintptr_t, int64_t>;

struct ls_op {
  int device = 0;
  int64_t N = 0;
  std::vector<double> xy;
  std::vector<int32_t> key;
  // device blocks the op holds, with their sizes (for the allocator's release)
  std::vector<std::pair<void*, size_t>> allocs;
  size_t resident = 0;
  ls_allocator alloc{};           // alloc.alloc == nullptr: hipMalloc / hipFree
  // the fork / join sequence of an apply on the op's side stream and events
  // (and graph capture, which records it) is taken under this lock
  std::recursive_mutex apply_mu;
  // solves run one at a time (they share the Givens buffers and events)
  std::mutex solve_mu;
  lsx::DevView<double> d64;
  lsx::DevView<float> d32;
  double kappa = 0;
  int64_t stats[15] = {0};
  // solver scratch (ls_solve without a caller workspace)
  void* gm = nullptr;
  size_t gm_bytes = 0;
  void* gm_last = nullptr;        // workspace base the last solve used (captured graphs point into it)
  std::complex<double>* pinned = nullptr;
  size_t pinned_n = 0;
  hipEvent_t gm_ev[2] = {nullptr, nullptr};
  // captured Arnoldi steps: (single precision, CGS2, nrhs, restart, step,
  // solver buffer, N) -> executable graph; capture runs on cap_stream
  std::map<GraphKey, hipGraphExec_t> graphs;
  hipStream_t cap_stream = nullptr;
  // host data kept for evaluating the field off the scatterer
  struct {
    std::vector<double> cw;                         // plain quadrature weights c_j
    std::vector<int32_t> cell_map, cell_start, cell_nint, cell_nb;
    std::vector<lsx::cd> Bp;                        // cell Dirichlet fit
    int L = 0, nfb = 0, F = 0;
    int64_t c_lo = 0;
    double H = 0, shape_a = 0;
    int shape_k = 0;
  } ext;
};

struct ls_targets {
  int64_t n = 0;
  std::vector<std::pair<void*, size_t>> allocs;
  ls_allocator alloc{};
  lsx::TargetView view;
};

namespace {

// device memory through the op's allocator (or hipMalloc)
void* dev_alloc(const ls_allocator& a, size_t bytes) {
  if (bytes == 0) bytes = 1;
  if (a.alloc) return a.alloc(bytes, a.ctx);
  void* p = nullptr;
  return hipMalloc(&p, bytes) == hipSuccess ? p : nullptr;
}
void dev_free(const ls_allocator& a, void* p, size_t bytes) {
  if (!p) return;
  if (a.alloc) {
    if (a.release) a.release(p, bytes, a.ctx);
  } else {
    (void)hipFree(p);
  }
}

template <typename X>
ls_status upload(ls_op* op, const X* src, size_t count, void** dst) {
  *dst = nullptr;
  if (count == 0) return LS_OK;
  void* p = dev_alloc(op->alloc, count * sizeof(X));
  if (!p) return fail(LS_ENOMEM, "device allocation failed");
  op->allocs.emplace_back(p, count * sizeof(X));
  op->resident += count * sizeof(X);
  if (hipMemcpy(p, src, count * sizeof(X), hipMemcpyHostToDevice) != hipSuccess)
    return fail(LS_EDEVICE, "hipMemcpy H2D failed");
  *dst = p;
  return LS_OK;
}

// upload a complex double array and/or its single-precision rounding
ls_status upload_c(ls_op* op, const std::vector<cd>& v, const void** d64, const void** d32) {
  if (d64) {
    void* a = nullptr;
    ls_status s = upload(op, v.data(), v.size(), &a);
    if (s) return s;
    *d64 = a;
  }
  if (!d32) return LS_OK;
  ls_status s;
  std::vector<Fp32c> f(v.size());
  for (size_t i = 0; i < v.size(); ++i) f[i] = {(float)v[i].real(), (float)v[i].imag()};
  void* b = nullptr;
  s = upload(op, f.data(), f.size(), &b);
  if (s) return s;
  *d32 = b;
  return LS_OK;
}

template <typename X>
ls_status upload_i(ls_op* op, const std::vector<X>& v, const X** dst) {
  void* a = nullptr;
  ls_status s = upload(op, v.data(), v.size(), &a);
  *dst = (const X*)a;
  return s;
}

lsx::FftPlan make_plan(int n) {
  lsx::FftPlan p{};
  p.n = n;
  int r = n;
  p.npass = 0;
  // fewest passes: the largest supported radix (<= 16, in-register DFT)
  // that divides what is left
  static const int rad[] = {16, 15, 12, 10, 9, 8, 6, 5, 4, 3, 2};
  while (r > 1) {
    int pick = 0;
    for (int R : rad)
      if (r % R == 0) {
        pick = R;
        break;
      }
    if (!pick) break;       // next_smooth sizes only have factors 2, 3, 5
    p.radix[p.npass++] = (int8_t)pick;
    r /= pick;
  }
  return p;
}

void clear_graphs(ls_op* op) {
  for (auto& kv : op->graphs) (void)hipGraphExecDestroy(kv.second);
  op->graphs.clear();
}

void release(ls_op* op) {
  // a caching allocator hands blocks out again at once: let every kernel
  // that may still read them finish first (hipFree waits by itself)
  if (op->alloc.alloc) (void)hipDeviceSynchronize();
  for (auto& pb : op->allocs) dev_free(op->alloc, pb.first, pb.second);
  op->allocs.clear();
  dev_free(op->alloc, op->gm, op->gm_bytes);
  op->gm = nullptr;
  op->gm_bytes = 0;
  if (op->pinned) (void)hipHostFree(op->pinned);
  op->pinned = nullptr;
  for (auto& e : op->gm_ev) {
    if (e) (void)hipEventDestroy(e);
    e = nullptr;
  }
  clear_graphs(op);
  if (op->cap_stream) (void)hipStreamDestroy(op->cap_stream);
  op->cap_stream = nullptr;
  for (hipEvent_t* e : {&op->d64.ev_fork, &op->d64.ev_join, &op->d32.ev_fork, &op->d32.ev_join}) {
    if (*e) (void)hipEventDestroy(*e);
    *e = nullptr;
  }
  if (op->d64.side) (void)hipStreamDestroy(op->d64.side);
  op->d64.side = op->d32.side = nullptr;
}

size_t ws_bytes(const ls_op* op, int nrhs, ls_prec prec) {
  size_t c = prec == LS_C128 ? 16 : 8;
  const auto& d = op->d64;
  size_t Gw = (size_t)d.gw;
  // projections, lattices, interior grid, near-field buffer of the
  // concurrent near field, and with Fourier refinement the rows' input x
  // and the band lines
  const size_t rfe = d.ldx > d.N ? (size_t)nrhs * ((size_t)d.ldx + (size_t)d.rf_lines * d.rf_n1) : 0;
  const size_t rfie = d.rfi > 1 ? (size_t)nrhs * Gw * Gw : 0;   // spectra of the psi grids
  return c * ((size_t)nrhs * d.ncell * d.U + (size_t)nrhs * 4 * d.Pa * d.Pb + (size_t)nrhs * Gw * Gw +
              (size_t)nrhs * op->N + rfe + rfie) + 256;
}

}  // namespace

namespace lsx {
FftPlan make_fft_plan(int n) { return make_plan(n); }
}  // namespace lsx

extern "C" {

// Field off the scatterer (see ls.h): targets sorted by cell of the lattice
// box, one Dirichlet-fit row and one row of adjacent-cell sources each.
ls_status ls_targets_create(ls_op* op, int64_t n, const double* xy, ls_targets** out) {
  if (!op || !out || n < 1 || !xy) return fail(LS_EINVAL, "bad argument");
  *out = nullptr;
  const auto& x = op->ext;
  const double H = x.H, kappa = op->kappa;
  const int L = x.L, F = x.F;
  std::vector<int64_t> cell(n);
  for (int64_t i = 0; i < n; ++i) {
    const double px = xy[2 * i], py = xy[2 * i + 1];
    const double rr = std::hypot(px, py), th = std::atan2(py, px);
    const double R = 1.0 + x.shape_a * std::cos(x.shape_k * th);
    if (!(rr > R * (1.0 + 1e-12))) return fail(LS_EINVAL, "target inside or on the scatterer");
    const int64_t cx = (int64_t)std::floor(px / H) - x.c_lo, cy = (int64_t)std::floor(py / H) - x.c_lo;
    if (cx < 0 || cy < 0 || cx >= L || cy >= L) return fail(LS_EINVAL, "target outside the operator's cell box");
    cell[i] = cy * L + cx;
  }
  std::vector<int32_t> order(n);
  for (int64_t i = 0; i < n; ++i) order[i] = (int32_t)i;
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return cell[a] < cell[b]; });
  std::vector<int32_t> cxy, start;
  for (int64_t k = 0; k < n; ++k) {
    if (k == 0 || cell[order[k]] != cell[order[k - 1]]) {
      cxy.push_back((int32_t)(cell[order[k]] % L));
      cxy.push_back((int32_t)(cell[order[k]] / L));
      start.push_back((int32_t)k);
    }
  }
  start.push_back((int32_t)n);
  // fit rows and adjacent-cell sources, per target (in sorted order)
  std::vector<lsx::cd> fit((size_t)n * F);
  std::vector<std::vector<int32_t>> rc(n);
  std::vector<std::vector<lsx::cd>> rv(n);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t k = 0; k < n; ++k) {
    const int64_t i = order[k];
    const int cx = (int)(cell[i] % L), cy = (int)(cell[i] / L);
    const double rel[2] = {xy[2 * i] - (cx + x.c_lo) * H, xy[2 * i + 1] - (cy + x.c_lo) * H};
    lsx::fit_row(x.Bp, x.nfb, F, kappa, H, rel, &fit[(size_t)k * F]);
    for (int oy = -1; oy <= 1; ++oy)
      for (int ox = -1; ox <= 1; ++ox) {
        const int nx = cx + ox, ny = cy + oy;
        if (nx < 0 || ny < 0 || nx >= L || ny >= L) continue;
        const int c = x.cell_map[(size_t)ny * L + nx];
        if (c < 0) continue;
        const int64_t j0 = x.cell_start[c], j1 = j0 + x.cell_nint[c] + x.cell_nb[c];
        for (int64_t j = j0; j < j1; ++j) {
          const double d = std::hypot(xy[2 * i] - op->xy[2 * j], xy[2 * i + 1] - op->xy[2 * j + 1]);
          rc[k].push_back((int32_t)j);
          rv[k].push_back(lsx::green2d(kappa, d) * x.cw[j]);
        }
      }
  }
  std::vector<int64_t> rowptr(n + 1, 0);
  for (int64_t k = 0; k < n; ++k) rowptr[k + 1] = rowptr[k] + (int64_t)rc[k].size();
  std::vector<int32_t> cols((size_t)std::max<int64_t>(rowptr[n], 1), 0);
  std::vector<lsx::cd> vals((size_t)std::max<int64_t>(rowptr[n], 1), 0.0);
  for (int64_t k = 0; k < n; ++k) {
    std::copy(rc[k].begin(), rc[k].end(), cols.begin() + rowptr[k]);
    std::copy(rv[k].begin(), rv[k].end(), vals.begin() + rowptr[k]);
  }
  auto* tg = new (std::nothrow) ls_targets();
  if (!tg) return fail(LS_ENOMEM, "host allocation");
  tg->alloc = op->alloc;
  auto put = [&](const void* src, size_t bytes, const void** dst) -> bool {
    void* p = dev_alloc(tg->alloc, bytes);
    if (!p) return false;
    tg->allocs.emplace_back(p, bytes);
    *dst = p;
    return hipMemcpy(p, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
  };
  lsx::TargetView& v = tg->view;
  v.n = n;
  v.ncell = (int)(start.size() - 1);
  const void *a1, *a2, *a3, *a5, *a6;
  bool ok = put(cxy.data(), cxy.size() * 4, &a1) && put(start.data(), start.size() * 4, &a2) &&
            put(order.data(), order.size() * 4, &a3) && put(fit.data(), fit.size() * 16, &v.fit) &&
            put(rowptr.data(), rowptr.size() * 8, &a5) && put(cols.data(), cols.size() * 4, &a6) &&
            put(vals.data(), vals.size() * 16, &v.vals);
  if (!ok) {
    ls_targets_destroy(tg);
    return fail(LS_ENOMEM, "target upload");
  }
  v.cell_xy = (const int32_t*)a1;
  v.start = (const int32_t*)a2;
  v.orig = (const int32_t*)a3;
  v.rowptr = (const int64_t*)a5;
  v.cols = (const int32_t*)a6;
  tg->n = n;
  *out = tg;
  return LS_OK;
}

void ls_targets_destroy(ls_targets* tg) {
  if (!tg) return;
  for (auto& pb : tg->allocs) dev_free(tg->alloc, pb.first, pb.second);
  delete tg;
}

ls_status ls_scattered_field(ls_op* op, const ls_targets* tg, const void* u_tot, int nrhs, void* us, void* ws,
                             size_t ws_bytes_, void* stream) {
  if (!op || !tg || !u_tot || !us || !ws || nrhs < 1) return fail(LS_EINVAL, "bad argument");
  if (ws_bytes_ < ws_bytes(op, nrhs, LS_C128)) return fail(LS_EINVAL, "workspace too small");
  std::lock_guard<std::recursive_mutex> lk(op->apply_mu);
  hipError_t e = lsx::launch_targets(op->d64, tg->view, u_tot, us, nrhs, ws, (hipStream_t)stream);
  if (e != hipSuccess) return fail(LS_EDEVICE, std::string("scattered field launch: ") + hipGetErrorString(e));
  return LS_OK;
}

const char* ls_status_str(ls_status s) {
  switch (s) {
    case LS_OK: return "ok";
    case LS_EINVAL: return "invalid argument";
    case LS_ENOMEM: return "out of memory";
    case LS_EDEVICE: return "device error";
    case LS_ENOCONV: return "not converged";
    case LS_EBUDGET: return "over memory budget";
    case LS_ENOTREADY: return "not ready";
    case LS_ENUMERIC: return "non-finite value";
  }
  return "unknown status";
}

const char* ls_last_error(void) { return g_err.c_str(); }

ls_status ls_host_build(const ls_geometry* g, ls_n2_fn n2, void* ctx, double kappa, const ls_params* p,
                        ls_host_op** out) {
  if (!g || !n2 || !p || !out) return fail(LS_EINVAL, "null argument");
  *out = nullptr;
  ls_host_op* h = new (std::nothrow) ls_host_op();
  if (!h) return fail(LS_ENOMEM, "host allocation");
  std::string err;
  ls_status s;
  try {
    s = lsx::build_host_op(g, n2, ctx, kappa, p, h->h, err);
  } catch (const std::bad_alloc&) {
    s = LS_ENOMEM;
    err = "host allocation during set-up";
  }
  if (s != LS_OK) {
    delete h;
    return fail(s, err);
  }
  *out = h;
  return LS_OK;
}

void ls_host_destroy(ls_host_op* h) { delete h; }

ls_status ls_host_num_points(const ls_host_op* h, int64_t* N) {
  if (!h || !N) return fail(LS_EINVAL, "null argument");
  *N = h->h.N;
  return LS_OK;
}

ls_status ls_host_points(const ls_host_op* h, double* xy, int32_t* key) {
  if (!h || !xy) return fail(LS_EINVAL, "null argument");
  std::memcpy(xy, h->h.xy.data(), h->h.xy.size() * sizeof(double));
  if (key) std::memcpy(key, h->h.key.data(), h->h.key.size() * sizeof(int32_t));
  return LS_OK;
}

ls_status ls_host_stats(const ls_host_op* h, int64_t* out, int nout) {
  if (!h || !out) return fail(LS_EINVAL, "null argument");
  const auto& o = h->h;
  int64_t v[12] = {o.N, o.n_band, o.ncell, o.L, (int64_t)o.rows.size(), (int64_t)o.cols.size(),
                   o.Pa, o.Pb, o.U, o.F, o.S, o.Wn};
  for (int i = 0; i < nout && i < 12; ++i) out[i] = v[i];
  return LS_OK;
}

ls_status ls_host_near_row(const ls_host_op* h, int64_t i, int64_t cap, int32_t* cols, double* vals,
                           int64_t* count) {
  if (!h || !count) return fail(LS_EINVAL, "null argument");
  const auto& o = h->h;
  const int64_t nsr = (int64_t)o.sr_rows.size();
  if (i < 0 || i >= o.N + nsr) return fail(LS_EINVAL, "row out of range");
  std::vector<std::pair<int32_t, cd>> ent;
  if (i >= o.N) {
    // off-grid shortcut: the boundary rule of grid node i - N (its s column
    // is sr_rows[i - N])
    const int64_t r = i - o.N;
    for (int64_t k = o.sr_rowptr[r]; k < o.sr_rowptr[r + 1]; ++k) ent.emplace_back(o.sr_cols[k], o.sr_vals[k]);
    *count = (int64_t)ent.size();
    if (cols && vals)
      for (int64_t k = 0; k < (int64_t)ent.size() && k < cap; ++k) {
        cols[k] = ent[k].first;
        vals[2 * k] = ent[k].second.real();
        vals[2 * k + 1] = ent[k].second.imag();
      }
    return LS_OK;
  }
  if (o.key[3 * i] == 0) {
    // shared window part: interior sources in the 5x5 cells around i's cell
    int c = -1, slot = -1;
    for (int cc = 0; cc < o.ncell && c < 0; ++cc)
      for (int a = 0; a < o.S; ++a)
        if (o.slot_map[(size_t)cc * o.S + a] == i) { c = cc; slot = a; break; }
    const int ch = o.p.cell_h, Wn = o.Wn;
    const int cx = o.cell_xy[2 * c], cy = o.cell_xy[2 * c + 1];
    for (int wy = 0; wy < Wn; ++wy)
      for (int wx = 0; wx < Wn; ++wx) {
        int nx = cx + wx / ch - 2, ny = cy + wy / ch - 2;
        if (nx < 0 || ny < 0 || nx >= o.L || ny >= o.L) continue;
        int cn = o.cell_map[ny * o.L + nx];
        if (cn < 0) continue;
        int j = o.slot_map[(size_t)cn * o.S + (wy % ch) * ch + (wx % ch)];
        if (j < 0) continue;
        cd w = o.Wsh[(size_t)slot * Wn * Wn + (size_t)wy * Wn + wx] * o.dw[j];
        if (w != 0.0) ent.emplace_back(j, w);
      }
    // interior refinement: the windows of the shifted psi grids, on the
    // refined-grid columns (grid position cell * cell_h + window offset)
    for (int s = 1; s < o.rfi * o.rfi; ++s)
      for (int wy = 0; wy < Wn; ++wy)
        for (int wx = 0; wx < Wn; ++wx) {
          const cd w = o.Wsh[((size_t)s * o.S + slot) * Wn * Wn + (size_t)wy * Wn + wx];
          if (w == 0.0) continue;
          const int64_t gx = (int64_t)cx * ch + wx, gy = (int64_t)cy * ch + wy;
          ent.emplace_back((int32_t)(o.N + o.rf_ioff + ((int64_t)(s - 1) * o.M + gy) * o.M + gx), w);
        }
  }
  auto it = std::lower_bound(o.rows.begin(), o.rows.end(), (int32_t)i);
  if (it != o.rows.end() && *it == i) {
    size_t r = it - o.rows.begin();
    for (int64_t k = o.rowptr[r]; k < o.rowptr[r + 1]; ++k) ent.emplace_back(o.cols[k], o.vals[k]);
  }
  *count = (int64_t)ent.size();
  if (cols && vals) {
    for (int64_t k = 0; k < (int64_t)ent.size() && k < cap; ++k) {
      cols[k] = ent[k].first;
      vals[2 * k] = ent[k].second.real();
      vals[2 * k + 1] = ent[k].second.imag();
    }
  }
  return LS_OK;
}

ls_status ls_create(const ls_geometry* g, ls_n2_fn n2, void* ctx, double kappa, const ls_params* p,
                    const ls_allocator* alloc, ls_op** out) {
  if (!out) return fail(LS_EINVAL, "null argument");
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return fail(LS_EDEVICE, "no HIP device");
  ls_host_op* hb = nullptr;
  ls_status s = ls_host_build(g, n2, ctx, kappa, p, &hb);
  if (s) return s;
  lsx::HostOp& h = hb->h;
  ls_op* op = new (std::nothrow) ls_op();
  if (!op) { ls_host_destroy(hb); return fail(LS_ENOMEM, "host allocation"); }
  (void)hipGetDevice(&op->device);
  {
    // address of this device's copy of the no-allocation scratch
    hipError_t e = init_scratch(op->device);
    if (e != hipSuccess) {
      ls_host_destroy(hb);
      delete op;
      return fail(LS_EDEVICE, std::string("scratch symbol address: ") + hipGetErrorString(e));
    }
  }
  if (alloc) {
    if (!alloc->alloc || !alloc->release) {
      ls_host_destroy(hb);
      delete op;
      return fail(LS_EINVAL, "allocator without alloc or release");
    }
    op->alloc = *alloc;
  }
  op->N = h.N;
  op->kappa = kappa;
  op->xy = h.xy;
  op->key = h.key;
  (void)ls_host_stats(hb, op->stats, 12);

  auto cleanup = [&](ls_status st) {
    release(op);
    delete op;
    ls_host_destroy(hb);
    return st;
  };
  // LDS needed by the FFT kernels
  int lds_max = 0;
  (void)hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, op->device);
  // columns per workgroup of the column transforms: default 128-byte row
  // segments (8 double / 16 float columns), at most what 150 KB of LDS holds
  // beside the staged twiddles (Pa values); ls_autotune may pick another
  // value up to that limit.  The FFT kernels may use all 160 KB.
  const size_t lds_cap = 150 * 1024;
  if ((size_t)h.Pa * 16 * 3 > lds_cap || 2 * (size_t)h.Pb * 16 > 160 * 1024) {
    ls_host_destroy(hb);
    delete op;
    return fail(LS_EINVAL, "FFT line too long for one workgroup's LDS");
  }
  const int tc = std::max(1, std::min(8, (int)((lds_cap - (size_t)h.Pa * 16) / (2 * (size_t)h.Pa * 16))));
  const int tc32 = std::max(1, std::min(16, (int)((lds_cap - (size_t)h.Pa * 8) / (2 * (size_t)h.Pa * 8))));
  {
    hipError_t e = lsx::set_fft_lds_limits(160 * 1024);
    if (e != hipSuccess) return cleanup(fail(LS_EDEVICE, std::string("LDS attribute: ") + hipGetErrorString(e)));
  }
  (void)lds_max;

  lsx::DevView<double>& a = op->d64;
  lsx::DevView<float>& b = op->d32;
  a.N = b.N = h.N;
  a.ncell = b.ncell = h.ncell;
  a.S = b.S = h.S;
  a.U = b.U = h.U;
  a.F = b.F = h.F;
  a.q = b.q = h.q;
  a.L = b.L = h.L;
  a.na = b.na = h.na;
  a.nb = b.nb = h.nb;
  a.Pa = b.Pa = h.Pa;
  a.Pb = b.Pb = h.Pb;
  a.ch = b.ch = h.p.cell_h;
  // psi grid side: the cells plus two on each side, or the interior
  // refinement's period
  a.gw = b.gw = h.rfi > 1 ? h.M : (h.L + 4) * h.p.cell_h;
  a.tc = tc;
  b.tc = tc32;
  a.kappa = b.kappa = kappa;
  // the near field's own stream (default priority, non-blocking) and the
  // fork / join events of the concurrent apply
  {
    hipStream_t side = nullptr;
    if (hipStreamCreateWithFlags(&side, hipStreamNonBlocking) != hipSuccess)
      return cleanup(fail(LS_EDEVICE, "side stream"));
    a.side = b.side = side;
    for (hipEvent_t* e : {&a.ev_fork, &a.ev_join, &b.ev_fork, &b.ev_join})
      if (hipEventCreateWithFlags(e, hipEventDisableTiming) != hipSuccess)
        return cleanup(fail(LS_EDEVICE, "fork / join events"));
  }
  a.nrows = b.nrows = (int)h.rows.size();
  a.csr_f64 = true;
  b.csr_f64 = false;
  int max_nb = 0;
  std::vector<int32_t> icells, bcells;
  for (int c = 0; c < h.ncell; ++c) {
    max_nb = std::max(max_nb, h.cell_nb[c]);
    if (h.cell_nint[c] > 0) icells.push_back(c);
    if (h.cell_nb[c] > 0) bcells.push_back(c);
  }
  a.nbcell = b.nbcell = (int)bcells.size();
  // the band projection kernel stages a cell's nodes for 16 right-hand
  // sides in LDS
  if ((size_t)(max_nb + 96) * 16 * 16 > 150 * 1024) a.proj_mfma = b.proj_mfma = false;
  a.max_nb = b.max_nb = max_nb;
  a.nicell = b.nicell = (int)icells.size();
  a.pa = b.pa = make_plan(h.Pa);
  a.pb = b.pb = make_plan(h.Pb);

#define UP(expr)              \
  do {                        \
    ls_status s_ = (expr);    \
    if (s_) return cleanup(s_); \
  } while (0)
  UP(upload_c(op, h.Psh, &a.Psh, nullptr));
  UP(upload_c(op, h.Pbd, &a.Pbd, nullptr));
  UP(upload_c(op, h.Psh32, nullptr, &b.Psh));
  {
    // slot projection transposed to [S][U] (the kernel's 96 output lanes read consecutive words)
    std::vector<cd> t64((size_t)h.S * h.U), t32((size_t)h.S * h.U);
    for (int t = 0; t < h.U; ++t)
      for (int a2 = 0; a2 < h.S; ++a2) {
        t64[(size_t)a2 * h.U + t] = h.Psh[(size_t)t * h.S + a2];
        t32[(size_t)a2 * h.U + t] = h.Psh32[(size_t)t * h.S + a2];
      }
    UP(upload_c(op, t64, &a.PshT, nullptr));
    UP(upload_c(op, t32, nullptr, &b.PshT));
  }
  UP(upload_c(op, h.Pbd32, nullptr, &b.Pbd));
  {
    // transposed layouts for coalesced reads in the interpolation kernel
    std::vector<cd> IshT((size_t)h.F * h.S);
    for (int a2 = 0; a2 < h.S; ++a2)
      for (int t = 0; t < h.F; ++t) IshT[(size_t)t * h.S + a2] = h.Ish[(size_t)a2 * h.F + t];
    UP(upload_c(op, IshT, &a.Ish, &b.Ish));
  }
  {
    // band fit rows transposed to [F][n_band] (lanes of the interpolation
    // kernel take consecutive nodes)
    std::vector<cd> IbdT((size_t)h.F * h.n_band);
    for (int64_t bb = 0; bb < h.n_band; ++bb)
      for (int t = 0; t < h.F; ++t) IbdT[(size_t)t * h.n_band + bb] = h.Ibd[(size_t)bb * h.F + t];
    UP(upload_c(op, IbdT, &a.Ibd, &b.Ibd));
    a.nband = b.nband = h.n_band;
  }
  {
    std::vector<cd> ToffT((size_t)9 * h.U * h.F);
    for (int o = 0; o < 9; ++o)
      for (int t = 0; t < h.F; ++t)
        for (int u2 = 0; u2 < h.U; ++u2)
          ToffT[((size_t)o * h.U + u2) * h.F + t] = h.Toff[((size_t)o * h.F + t) * h.U + u2];
    UP(upload_c(op, ToffT, &a.Toff, &b.Toff));
  }
  {
    // shared window with the adjacent far-field subtraction of each
    // precision folded in
    std::vector<cd> w64(h.Wsh), w32(h.Wsh);
    for (size_t i = 0; i < h.Wadj.size(); ++i) {     // (the window of shift 0)
      w64[i] += h.Wadj[i];
      w32[i] += h.Wadj32[i];
    }
    UP(upload_c(op, w64, &a.Wsh, nullptr));
    UP(upload_c(op, w32, nullptr, &b.Wsh));
  }
  // near-field rows stored padded to a multiple of four entries (zero
  // weights, column offset 0), so a lane can take four at a time
  const size_t nrow = h.rows.size();
  std::vector<int64_t> prow(nrow + 1, 0);
  for (size_t r = 0; r < nrow; ++r) prow[r + 1] = prow[r] + ((h.rowptr[r + 1] - h.rowptr[r] + 3) & ~int64_t(3));
  {
    std::vector<cd> pv((size_t)prow[nrow], cd(0.0, 0.0));
    for (size_t r = 0; r < nrow; ++r)
      std::copy(h.vals.begin() + h.rowptr[r], h.vals.begin() + h.rowptr[r + 1], pv.begin() + prow[r]);
    UP(upload_c(op, pv, &a.vals, &b.vals));
  }
  {
    std::vector<float> f(h.cw.begin(), h.cw.end()), g2(h.dw.begin(), h.dw.end());
    UP(upload_i(op, h.cw, &a.cw));
    UP(upload_i(op, f, &b.cw));
    UP(upload_i(op, h.dw, &a.dw));
    UP(upload_i(op, g2, &b.dw));
  }
  UP(upload_i(op, h.slot_map, &a.slot_map));
  UP(upload_i(op, h.cell_start, &a.cell_start));
  UP(upload_i(op, h.cell_nint, &a.cell_nint));
  UP(upload_i(op, h.cell_nb, &a.cell_nb));
  UP(upload_i(op, h.cell_boff, &a.cell_boff));
  UP(upload_i(op, h.cell_xy, &a.cell_xy));
  UP(upload_i(op, h.cell_map, &a.cell_map));
  UP(upload_i(op, icells, &a.icells));
  if (!bcells.empty()) UP(upload_i(op, bcells, &a.bcells));
  UP(upload_i(op, h.rows, &a.rows));
  {
    // columns as 16-bit offsets from the row's smallest column (a row spans
    // at most a few cell rows of the cell-sorted order)
    const size_t nr = h.rows.size();
    std::vector<int32_t> cbase(nr);
    bool narrow = true;
    for (size_t r = 0; r < nr; ++r) {
      int32_t lo = INT32_MAX, hi = INT32_MIN;
      for (int64_t k = h.rowptr[r]; k < h.rowptr[r + 1]; ++k) {
        lo = std::min(lo, h.cols[k]);
        hi = std::max(hi, h.cols[k]);
      }
      if (h.rowptr[r + 1] == h.rowptr[r]) lo = hi = 0;
      if (hi - lo > 65535) narrow = false;
      cbase[r] = lo;
    }
    UP(upload_i(op, cbase, &a.colbase));
    if (narrow) {
      std::vector<uint16_t> coff((size_t)prow[nr], 0);
      for (size_t r = 0; r < nr; ++r)
        for (int64_t k = h.rowptr[r]; k < h.rowptr[r + 1]; ++k)
          coff[prow[r] + (k - h.rowptr[r])] = (uint16_t)(h.cols[k] - cbase[r]);
      UP(upload_i(op, coff, &a.coloff));
    } else {
      std::vector<int32_t> c32((size_t)prow[nr], 0);
      for (size_t r = 0; r < nr; ++r)
        for (int64_t k = h.rowptr[r]; k < h.rowptr[r + 1]; ++k)
          c32[prow[r] + (k - h.rowptr[r])] = h.cols[k] - cbase[r];
      UP(upload_i(op, c32, &a.cols32));
    }
  }
  UP(upload_i(op, prow, &a.rowptr));
  if (!h.sr_rows.empty()) {
    // off-grid shortcut: the boundary rule at the patch's grid nodes as rows
    // writing s into x (32-bit column offsets from each row's first column)
    const int n1 = h.g.N1, nlines = h.g.N2 + 1;
    a.rf_n1 = b.rf_n1 = n1;
    a.rf_lines = b.rf_lines = nlines;
    if (h.rf == 1) a.ldx = b.ldx = h.N + h.sc_off + (int64_t)nlines * n1;
    a.nsr = b.nsr = (int)h.sr_rows.size();
    a.sc_off = b.sc_off = h.sc_off;
    const size_t ns = h.sr_rows.size();
    std::vector<int32_t> cb(ns), c32(h.sr_cols.size());
    for (size_t r = 0; r < ns; ++r) {
      cb[r] = h.sr_cols[h.sr_rowptr[r]];     // sorted: the smallest column
      for (int64_t k = h.sr_rowptr[r]; k < h.sr_rowptr[r + 1]; ++k) c32[k] = h.sr_cols[k] - cb[r];
    }
    UP(upload_i(op, h.sr_rowptr, &a.sr_rowptr));
    UP(upload_i(op, h.sr_rows, &a.sr_rows));
    UP(upload_i(op, cb, &a.sr_colbase));
    UP(upload_i(op, c32, &a.sr_cols32));
    UP(upload_c(op, h.sr_vals, &a.sr_vals, &b.sr_vals));
    b.sr_rowptr = a.sr_rowptr;
    b.sr_rows = a.sr_rows;
    b.sr_colbase = a.sr_colbase;
    b.sr_cols32 = a.sr_cols32;
  }
  if (h.rf > 1) {
    // Fourier refinement of the band's t1 lines: line maps, phase ramps of
    // the shifts s / rf (with the inverse transform's 1 / N1; the Nyquist
    // term, even N1, split between +-N1/2: cos(pi s / rf)), twiddles
    const int n1 = h.g.N1, nlines = h.g.N2 + 1, rf = h.rf;
    a.rf = b.rf = rf;
    a.rf_n1 = b.rf_n1 = n1;
    a.rf_lines = b.rf_lines = nlines;
    a.ldx = b.ldx = h.N + (int64_t)(rf - 1) * nlines * n1 + (int64_t)(h.rfi * h.rfi - 1) * h.M * h.M +
                    (h.sr_rows.empty() ? 0 : (int64_t)rf * nlines * n1);
    a.rf_ioff = b.rf_ioff = h.rf_ioff;
    a.rf_plan = b.rf_plan = make_plan(n1);
    std::vector<cd> ph((size_t)(rf - 1) * n1), tw(n1);
    for (int s = 1; s < rf; ++s)
      for (int k = 0; k < n1; ++k) {
        cd z;
        if (n1 % 2 == 0 && 2 * k == n1) {
          z = cd(std::cos(M_PI * s / rf), 0.0);
        } else {
          const int f = 2 * k < n1 ? k : k - n1;
          z = std::polar(1.0, 2.0 * M_PI * (double)f * s / ((double)rf * n1));
        }
        ph[(size_t)(s - 1) * n1 + k] = z / (double)n1;
      }
    for (int k = 0; k < n1; ++k) tw[k] = std::polar(1.0, -2.0 * M_PI * (double)k / n1);
    UP(upload_c(op, ph, &a.rf_ph, &b.rf_ph));
    UP(upload_c(op, tw, &a.rf_tw, &b.rf_tw));
    UP(upload_i(op, h.rf_idx, &a.rf_idx));
    b.rf_idx = a.rf_idx;
    std::vector<float> df(h.rf_dens.begin(), h.rf_dens.end());
    UP(upload_i(op, h.rf_dens, &a.rf_dens));
    UP(upload_i(op, df, &b.rf_dens));
    if (h.rfi > 1) {
      // interior: phase ramps [s][k] of the shifts s / rf on the M-point axis
      // (1 / M included, Nyquist split as above), twiddles
      const int M = h.M;
      a.rfi = b.rfi = rf;
      a.rf_iplan = b.rf_iplan = make_plan(M);
      std::vector<cd> iph((size_t)rf * M), itw(M);
      for (int s = 0; s < rf; ++s)
        for (int k = 0; k < M; ++k) {
          cd z;
          if (M % 2 == 0 && 2 * k == M) z = cd(std::cos(M_PI * s / rf), 0.0);
          else z = std::polar(1.0, 2.0 * M_PI * (double)(2 * k < M ? k : k - M) * s / ((double)rf * M));
          iph[(size_t)s * M + k] = z / (double)M;
        }
      for (int k = 0; k < M; ++k) itw[k] = std::polar(1.0, -2.0 * M_PI * (double)k / M);
      UP(upload_c(op, iph, &a.rf_iph, &b.rf_iph));
      UP(upload_c(op, itw, &a.rf_itw, &b.rf_itw));
    }
  }
  {
    // the same columns as runs of consecutive indices (padding: a final run
    // at column 0); not used when some row needs more than 256 runs
    const size_t nr = h.rows.size();
    std::vector<int32_t> rptr(nr + 1, 0), rcs, rpre;
    bool fits = true;
    int rmax = 0;
    for (size_t r = 0; r < nr && fits; ++r) {
      const int64_t b0 = h.rowptr[r], len = h.rowptr[r + 1] - b0;
      for (int64_t k = 0; k < len; ++k)
        if (k == 0 || h.cols[b0 + k] != h.cols[b0 + k - 1] + 1) {
          rcs.push_back(h.cols[b0 + k]);
          rpre.push_back((int32_t)k);
        }
      if (prow[r + 1] - prow[r] > len) {
        rcs.push_back(0);
        rpre.push_back((int32_t)len);
      }
      rptr[r + 1] = (int32_t)rcs.size();
      rmax = std::max(rmax, rptr[r + 1] - rptr[r]);
      if (rptr[r + 1] - rptr[r] > 256) fits = false;
    }
    if (fits && !rcs.empty()) {
      op->stats[12] = (int64_t)rcs.size();
      a.run_max = rmax;
      UP(upload_i(op, rptr, &a.run_ptr));
      UP(upload_i(op, rcs, &a.run_cs));
      UP(upload_i(op, rpre, &a.run_pre));
    }
  }
  // adjacent far-field subtraction folded into the stored row weights (both
  // precisions); the single-precision weights then come back for the tiles
  // (no tiles with Fourier refinement: their columns would include the
  // refined values)
  const bool tiles = !p->skip_tiles && h.rf == 1 && h.sr_rows.empty();
  std::vector<Fp32c> vals32(tiles ? (size_t)prow[nrow] : 0);
  std::vector<Fp64c> vals64(tiles ? (size_t)prow[nrow] : 0);
  {
    // entries the fold visits: those at unknowns (a row's refined columns,
    // at N and beyond, come last in its sorted columns)
    std::vector<int64_t> olen(nrow);
    for (size_t r = 0; r < nrow; ++r) {
      int64_t k = h.rowptr[r];
      while (k < h.rowptr[r + 1] && h.cols[k] < h.N) ++k;
      olen[r] = k - h.rowptr[r];
    }
    std::vector<int32_t> pt_cell((size_t)h.N, -1), pt_idx((size_t)h.N, 0);
    for (int c = 0; c < h.ncell; ++c) {
      for (int a2 = 0; a2 < h.S; ++a2) {
        const int32_t j = h.slot_map[(size_t)c * h.S + a2];
        if (j >= 0) {
          pt_cell[j] = c;
          pt_idx[j] = a2;
        }
      }
      for (int t = 0; t < h.cell_nb[c]; ++t) {
        const int32_t j = h.cell_start[c] + h.cell_nint[c] + t;
        pt_cell[j] = c;
        pt_idx[j] = -(h.cell_boff[c] + t + 1);
      }
    }
    for (int64_t j = 0; j < h.N; ++j)
      if (pt_cell[(size_t)j] < 0) return cleanup(fail(LS_EINVAL, "a node outside every cell"));
    const size_t b_olen = 8 * std::max<size_t>(1, nrow), b_pt = 4 * (size_t)h.N;
    void* d_olen = dev_alloc(op->alloc, b_olen);
    void* d_cell = d_olen ? dev_alloc(op->alloc, b_pt) : nullptr;
    void* d_idx = d_cell ? dev_alloc(op->alloc, b_pt) : nullptr;
    if (!d_idx) {
      dev_free(op->alloc, d_olen, b_olen);
      dev_free(op->alloc, d_cell, b_pt);
      return cleanup(fail(LS_ENOMEM, "device allocation failed (near-field fold)"));
    }
    bool ok = true;
    ok = ok && hipMemcpy(d_olen, olen.data(), 8 * nrow, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(d_cell, pt_cell.data(), 4 * (size_t)h.N, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(d_idx, pt_idx.data(), 4 * (size_t)h.N, hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && lsx::launch_fold_rows(a, b, (const int64_t*)d_olen, (const int32_t*)d_cell, (const int32_t*)d_idx,
                                     0) == hipSuccess;
    ok = ok && hipDeviceSynchronize() == hipSuccess;
    ok = ok && (vals32.empty() ||
                hipMemcpy(vals32.data(), b.vals, 8 * vals32.size(), hipMemcpyDeviceToHost) == hipSuccess);
    ok = ok && (vals64.empty() ||
                hipMemcpy(vals64.data(), a.vals, 16 * vals64.size(), hipMemcpyDeviceToHost) == hipSuccess);
    dev_free(op->alloc, d_olen, b_olen);
    dev_free(op->alloc, d_cell, b_pt);
    dev_free(op->alloc, d_idx, b_pt);
    if (!ok) return cleanup(fail(LS_EDEVICE, "near-field fold failed"));
  }
  if (tiles) {
    // Single precision, batched use: the rows as dense tiles of 16 rows of
    // one cell and kind.  A tile's columns are the points of the 3 x 3
    // adjacent cells that all its rows couple to (every point for
    // boundary-patch targets, the boundary-patch points for interior
    // targets), followed by the union of its rows' other columns.
    const int64_t N = h.N;
    std::vector<int32_t> cell_of((size_t)N, -1);
    for (int c = 0; c < h.ncell; ++c)
      for (int64_t j = h.cell_start[c]; j < (int64_t)h.cell_start[c] + h.cell_nint[c] + h.cell_nb[c]; ++j)
        cell_of[(size_t)j] = c;
    std::vector<int32_t> bt_rows, bt_info, bt_cols, adjcols, extra;
    std::vector<int64_t> bt_woff;
    std::vector<Fp32c> bt_w;
    std::vector<Fp64c> bt_w64;   // the same tiles in double precision
    int64_t n_extra = 0;
    std::vector<int32_t> pos((size_t)h.ncell, -1);   // column of an adjacent cell's first point
    const size_t nr = h.rows.size();
    auto is_band = [&](int32_t i) { return h.key[3 * (size_t)i] >= 1; };
    size_t r = 0;
    while (r < nr) {
      const int c = cell_of[(size_t)h.rows[r]];
      const bool tb = is_band(h.rows[r]);
      size_t r1 = r;
      while (r1 < nr && cell_of[(size_t)h.rows[r1]] == c && is_band(h.rows[r1]) == tb) ++r1;
      std::vector<int> adj;
      const int cx = h.cell_xy[2 * c], cy = h.cell_xy[2 * c + 1];
      for (int oy = -1; oy <= 1; ++oy)
        for (int ox = -1; ox <= 1; ++ox) {
          const int x = cx + ox, y = cy + oy;
          if (x < 0 || y < 0 || x >= h.L || y >= h.L) continue;
          const int cc = h.cell_map[(size_t)y * h.L + x];
          if (cc >= 0) adj.push_back(cc);
        }
      std::sort(adj.begin(), adj.end());
      auto first = [&](int cc) { return h.cell_start[cc] + (tb ? 0 : h.cell_nint[cc]); };
      adjcols.clear();
      for (int cc : adj) {
        pos[cc] = (int32_t)adjcols.size();
        for (int32_t j = first(cc); j < h.cell_start[cc] + h.cell_nint[cc] + h.cell_nb[cc]; ++j) adjcols.push_back(j);
      }
      auto in_adj = [&](int32_t j) { const int cj = cell_of[(size_t)j]; return pos[cj] >= 0 && j >= first(cj); };
      const int Ka = (int)adjcols.size();
      for (size_t t0 = r; t0 < r1; t0 += 16) {
        const size_t t1 = std::min(r1, t0 + 16);
        extra.clear();
        for (size_t rr = t0; rr < t1; ++rr)
          for (int64_t k = h.rowptr[rr]; k < h.rowptr[rr + 1]; ++k)
            if (!in_adj(h.cols[k])) extra.push_back(h.cols[k]);
        std::sort(extra.begin(), extra.end());
        extra.erase(std::unique(extra.begin(), extra.end()), extra.end());
        const int K = Ka + (int)extra.size(), Kp = (K + 3) & ~3;
        const int32_t coff = (int32_t)bt_cols.size();
        bt_cols.insert(bt_cols.end(), adjcols.begin(), adjcols.end());
        bt_cols.insert(bt_cols.end(), extra.begin(), extra.end());
        for (int k = K; k < Kp; ++k) bt_cols.push_back(bt_cols[coff]);
        const int64_t woff = (int64_t)bt_w.size();
        bt_w.resize(bt_w.size() + (size_t)Kp * 16, Fp32c{0.f, 0.f});
        bt_w64.resize(bt_w.size(), Fp64c{0.0, 0.0});
        bt_woff.push_back(woff);
        bt_info.push_back(Kp);
        bt_info.push_back(coff);
        n_extra += (int64_t)(Kp - Ka) * 16;
        for (int q = 0; q < 16; ++q) {
          const size_t rr = t0 + q;
          bt_rows.push_back(rr < t1 ? h.rows[rr] : -1);
          if (rr >= t1) continue;
          for (int64_t k = h.rowptr[rr]; k < h.rowptr[rr + 1]; ++k) {
            const int32_t j = h.cols[k];
            const int kk = in_adj(j) ? pos[cell_of[(size_t)j]] + (j - first(cell_of[(size_t)j]))
                                     : Ka + (int)(std::lower_bound(extra.begin(), extra.end(), j) - extra.begin());
            const size_t at = (size_t)woff + (size_t)(kk / 4) * 64 + (kk % 4) * 16 + q;
            const size_t from = (size_t)(prow[rr] + (k - h.rowptr[rr]));
            bt_w[at].x += vals32[from].x;
            bt_w[at].y += vals32[from].y;
            bt_w64[at].x += vals64[from].x;
            bt_w64[at].y += vals64[from].y;
          }
        }
      }
      for (int cc : adj) pos[cc] = -1;
      r = r1;
    }
    if (!bt_woff.empty()) {
      void* wd = nullptr;
      UP(upload(op, bt_w.data(), bt_w.size(), &wd));
      b.bt_w = wd;
      UP(upload_i(op, bt_rows, &b.bt_rows));
      UP(upload_i(op, bt_info, &b.bt_info));
      UP(upload_i(op, bt_cols, &b.bt_cols));
      UP(upload_i(op, bt_woff, &b.bt_woff));
      b.bt_ntiles = (int)bt_woff.size();
      void* wd64 = nullptr;
      UP(upload(op, bt_w64.data(), bt_w64.size(), &wd64));
      a.bt_w = wd64;
      a.bt_rows = b.bt_rows;
      a.bt_info = b.bt_info;
      a.bt_cols = b.bt_cols;
      a.bt_woff = b.bt_woff;
      a.bt_ntiles = b.bt_ntiles;
      op->stats[13] = (int64_t)bt_w.size();
      op->stats[14] = n_extra;
    }
  }
  b.slot_map = a.slot_map;
  b.cell_start = a.cell_start;
  b.cell_nint = a.cell_nint;
  b.cell_nb = a.cell_nb;
  b.cell_boff = a.cell_boff;
  b.cell_xy = a.cell_xy;
  b.cell_map = a.cell_map;
  b.icells = a.icells;
  b.bcells = a.bcells;
  b.rows = a.rows;
  b.colbase = a.colbase;
  b.coloff = a.coloff;
  b.cols32 = a.cols32;
  b.rowptr = a.rowptr;
  b.run_ptr = a.run_ptr;
  b.run_cs = a.run_cs;
  b.run_pre = a.run_pre;
  b.run_max = a.run_max;
  // twiddles exp(-2 pi i k / n), computed in double
  for (int which = 0; which < 2; ++which) {
    int n = which == 0 ? h.Pa : h.Pb;
    std::vector<cd> tw(n);
    for (int k = 0; k < n; ++k) tw[k] = std::polar(1.0, -2.0 * M_PI * (double)k / n);
    if (which == 0) UP(upload_c(op, tw, &a.twa, &b.twa));
    else UP(upload_c(op, tw, &a.twb, &b.twb));
  }
  // Green's function spectra: forward FFT (double) of the padded lattices
  {
    void* kd = nullptr;
    UP(upload(op, h.kern.data(), h.kern.size(), &kd));
    // rows a >= na are not all zero here (negative offsets wrap), so transform every row
    lsx::DevView<double> full = a;
    full.na = h.Pa;
    hipError_t e = lsx::launch_fft_kernels_forward(full, kd, 4, 0);
    if (e != hipSuccess) return cleanup(fail(LS_EDEVICE, std::string("kernel FFT: ") + hipGetErrorString(e)));
    if (hipDeviceSynchronize() != hipSuccess) return cleanup(fail(LS_EDEVICE, "kernel FFT failed"));
    a.khat = kd;
    std::vector<cd> kh(h.kern.size());
    if (hipMemcpy(kh.data(), kd, kh.size() * sizeof(cd), hipMemcpyDeviceToHost) != hipSuccess)
      return cleanup(fail(LS_EDEVICE, "copy of spectra"));
    std::vector<Fp32c> kf(kh.size());
    for (size_t i = 0; i < kh.size(); ++i) kf[i] = {(float)kh[i].real(), (float)kh[i].imag()};
    void* kf_d = nullptr;
    UP(upload(op, kf.data(), kf.size(), &kf_d));
    b.khat = kf_d;
  }
#undef UP
  op->ext.cw = h.cw;
  op->ext.cell_map = h.cell_map;
  op->ext.cell_start = h.cell_start;
  op->ext.cell_nint = h.cell_nint;
  op->ext.cell_nb = h.cell_nb;
  op->ext.Bp = h.Bp;
  op->ext.L = h.L;
  op->ext.nfb = h.p.n_fb;
  op->ext.F = h.F;
  op->ext.c_lo = h.c_lo;
  op->ext.H = h.H;
  op->ext.shape_a = h.g.shape_a;
  op->ext.shape_k = h.g.shape_k;
  ls_host_destroy(hb);
  *out = op;
  return LS_OK;
}

void ls_destroy(ls_op* op) {
  if (!op) return;
  release(op);
  delete op;
}

ls_status ls_num_points(const ls_op* op, int64_t* N) {
  if (!op || !N) return fail(LS_EINVAL, "null argument");
  *N = op->N;
  return LS_OK;
}

ls_status ls_points(const ls_op* op, double* xy, int32_t* key) {
  if (!op || !xy) return fail(LS_EINVAL, "null argument");
  std::memcpy(xy, op->xy.data(), op->xy.size() * sizeof(double));
  if (key) std::memcpy(key, op->key.data(), op->key.size() * sizeof(int32_t));
  return LS_OK;
}

size_t ls_resident_bytes(const ls_op* op) { return op ? op->resident : 0; }

ls_status ls_op_stats(const ls_op* op, int64_t* out, int nout) {
  if (!op || !out) return fail(LS_EINVAL, "null argument");
  for (int i = 0; i < nout && i < 15; ++i) out[i] = op->stats[i];
  return LS_OK;
}

ls_status ls_workspace_size(const ls_op* op, int nrhs, ls_prec prec, size_t* bytes) {
  if (!op || !bytes || nrhs < 1 || (prec != LS_C128 && prec != LS_C64)) return fail(LS_EINVAL, "bad argument");
  *bytes = ws_bytes(op, nrhs, prec);
  return LS_OK;
}

ls_status ls_apply(ls_op* op, const void* u, void* v, int nrhs, ls_prec prec, void* ws, size_t wsb,
                   void* stream) {
  if (!op || !u || !v || !ws || nrhs < 1) return fail(LS_EINVAL, "null argument or nrhs < 1");
  if (prec != LS_C128 && prec != LS_C64) return fail(LS_EINVAL, "unknown precision");
  if (wsb < ws_bytes(op, nrhs, prec)) return fail(LS_EINVAL, "workspace too small");
  size_t vb = (size_t)nrhs * op->N * (prec == LS_C128 ? 16 : 8);
  const char* uc = (const char*)u;
  const char* vc = (const char*)v;
  if (uc < vc + vb && vc < uc + vb) return fail(LS_EINVAL, "u and v overlap");
  hipStream_t st = (hipStream_t)stream;
  std::lock_guard<std::recursive_mutex> lk(op->apply_mu);
  hipError_t e = prec == LS_C128 ? lsx::launch_apply<double>(op->d64, u, v, nrhs, ws, st)
                                 : lsx::launch_apply<float>(op->d32, u, v, nrhs, ws, st);
  if (e != hipSuccess) return fail(LS_EDEVICE, std::string("apply launch: ") + hipGetErrorString(e));
  return LS_OK;
}

ls_status ls_apply_noalloc(ls_op* op, const void* u, void* v, int nrhs, ls_prec prec, void* stream) {
  if (!op || !u || !v || nrhs < 1) return fail(LS_EINVAL, "null argument or nrhs < 1");
  if (prec != LS_C128 && prec != LS_C64) return fail(LS_EINVAL, "unknown precision");
  const size_t need = ws_bytes(op, nrhs, prec);
  if (need > LS_NOALLOC_SCRATCH_BYTES)
    return fail(LS_EINVAL, "apply needs " + std::to_string(need) + " bytes of scratch; the static scratch holds " +
                               std::to_string(LS_NOALLOC_SCRATCH_BYTES));
  const size_t vb = (size_t)nrhs * op->N * (prec == LS_C128 ? 16 : 8);
  const char* uc = (const char*)u;
  const char* vc = (const char*)v;
  if (uc < vc + vb && vc < uc + vb) return fail(LS_EINVAL, "u and v overlap");
  void* ws = scratch_of(op->device);
  if (!ws) return fail(LS_EDEVICE, "no scratch address for the op's device");
  hipStream_t st = (hipStream_t)stream;
  std::lock_guard<std::recursive_mutex> lk(op->apply_mu);
  hipError_t e = prec == LS_C128 ? lsx::launch_apply<double>(op->d64, u, v, nrhs, ws, st)
                                 : lsx::launch_apply<float>(op->d32, u, v, nrhs, ws, st);
  if (e != hipSuccess) return fail(LS_EDEVICE, std::string("apply launch: ") + hipGetErrorString(e));
  return LS_OK;
}

ls_status ls_noalloc_scratch_bytes(size_t* bytes) {
  if (!bytes) return fail(LS_EINVAL, "null argument");
  *bytes = LS_NOALLOC_SCRATCH_BYTES;
  return LS_OK;
}

ls_status ls_apply_profile(ls_op* op, const void* u, void* v, int nrhs, ls_prec prec, void* ws, size_t wsb,
                           void* stream, double* stage_ms, int nstage) {
  if (!op || !u || !v || !ws || nrhs < 1 || !stage_ms || nstage < 1) return fail(LS_EINVAL, "bad argument");
  if (prec != LS_C128 && prec != LS_C64) return fail(LS_EINVAL, "unknown precision");
  if (wsb < ws_bytes(op, nrhs, prec)) return fail(LS_EINVAL, "workspace too small");
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t ev[9];
  for (int i = 0; i < 9; ++i) HIPCHK(hipEventCreate(&ev[i]));
  std::lock_guard<std::recursive_mutex> lk(op->apply_mu);
  hipError_t e = prec == LS_C128 ? lsx::launch_apply<double>(op->d64, u, v, nrhs, ws, st, ev)
                                 : lsx::launch_apply<float>(op->d32, u, v, nrhs, ws, st, ev);
  ls_status out = LS_OK;
  if (e != hipSuccess) out = fail(LS_EDEVICE, std::string("apply launch: ") + hipGetErrorString(e));
  if (out == LS_OK && hipEventSynchronize(ev[8]) != hipSuccess) out = fail(LS_EDEVICE, "apply failed");
  for (int i = 0; i < 8 && i < nstage && out == LS_OK; ++i) {
    float ms = 0;
    (void)hipEventElapsedTime(&ms, ev[i], ev[i + 1]);
    stage_ms[i] = ms;
  }
  for (int i = 0; i < 9; ++i) (void)hipEventDestroy(ev[i]);
  return out;
}

extern "C++" {
namespace {
// stage times of one apply (HIP events between the stages)
template <typename T>
ls_status timed_apply(ls_op* op, lsx::DevView<T>& d, const void* u, void* v, int nrhs, void* ws, hipStream_t st,
                      hipEvent_t* ev, double* ms8) {
  hipError_t e = lsx::launch_apply<T>(d, u, v, nrhs, ws, st, ev);
  if (e != hipSuccess) return fail(LS_EDEVICE, std::string("apply launch: ") + hipGetErrorString(e));
  if (hipEventSynchronize(ev[8]) != hipSuccess) return fail(LS_EDEVICE, "apply failed");
  for (int i = 0; i < 8; ++i) {
    float ms = 0;
    (void)hipEventElapsedTime(&ms, ev[i], ev[i + 1]);
    ms8[i] = ms;
  }
  (void)op;
  return LS_OK;
}

template <typename T>
ls_status autotune_view(ls_op* op, lsx::DevView<T>& d, int nrhs, const void* u, void* v, void* ws, hipStream_t st,
                        hipEvent_t* ev, ls_tune_result* res) {
  constexpr int reps = 3;
  double ms8[8];
  // LS_TUNE_LOG=1 prints every candidate's time to stderr
  const char* lg = std::getenv("LS_TUNE_LOG");
  const bool logc = lg && lg[0] == '1';
  auto log = [&](const char* what, int a, int b, double t) {
    if (logc) std::fprintf(stderr, "ls_autotune nrhs=%d %s %d %d: %.4f ms\n", nrhs, what, a, b, t);
  };
  // best (smallest) of reps applies for the stages [s0, s1]
  auto measure = [&](int s0, int s1, double* best) -> ls_status {
    *best = 1e30;
    for (int r = 0; r < reps; ++r) {
      ls_status s = timed_apply<T>(op, d, u, v, nrhs, ws, st, ev, ms8);
      if (s) return s;
      double t = 0;
      for (int i = s0; i <= s1; ++i) t += ms8[i];
      *best = std::min(*best, t);
    }
    return LS_OK;
  };
  // column tile of the transforms (stages 2-4: forward, spectral, inverse)
  // (separate kernels: two buffers of tc columns; fused: two of 2 tc)
  int best_tc = d.tc, best_fv = d.fft_variant, best_cn = d.cols_nth;
  double best = 1e30;
  for (int fv = 0; fv < 2; ++fv) {
    const int tmax = (int)((150 * 1024 - d.Pa * sizeof(T) * 2) / (2 * (size_t)d.Pa * sizeof(T) * 2 * (fv + 1)));
    for (int tc : {1, 2, 4, 8, 16, 32}) {
      if (tc > tmax) break;
      for (int cn : {256, 512}) {
        if (fv == 0 && cn != 256) continue;   // threads only tuned for the fused kernel
        d.tc = tc;
        d.fft_variant = fv;
        d.cols_nth = cn;
        double t;
        ls_status s = measure(2, 4, &t);
        if (s) return s;
        log("fft variant/tile", fv, tc * 10000 + cn, t);
        if (t < best) {
          best = t;
          best_tc = tc;
          best_fv = fv;
          best_cn = cn;
        }
      }
    }
  }
  d.tc = best_tc;
  d.fft_variant = best_fv;
  d.cols_nth = best_cn;
  // threads per row transform (a few hundred rows of a few thousand points:
  // more threads per row keep more waves resident)
  int best_nth = d.rows_nth;
  for (int nth : {256, 512, 1024}) {
    d.rows_nth = nth;
    double t;
    ls_status s = measure(2, 4, &t);
    if (s) return s;
    log("fft row threads", nth, 0, t);
    if (t < best) {
      best = t;
      best_nth = nth;
    }
  }
  d.rows_nth = best_nth;
  res->fft_col_tile = best_tc;
  res->fft_variant = best_fv;
  res->fft_row_threads = best_nth;
  res->fft_rows_inplace = d.rows_ip;
  res->near_rows_first = d.rows_first;
  res->fft_col_threads = d.cols_nth;
  res->fft_ms = best;
  // interior contraction variant (stage 6) and near-field rows variant (stage 7)
  const int nnear = std::is_same<T, float>::value ? 5 : 1;
  int bv = 0;
  best = 1e30;
  for (int var = 0; var < nnear; ++var) {
    d.near_variant = var;
    double t;
    ls_status s = measure(6, 6, &t);
    if (s) return s;
    log("near variant", var, 0, t);
    if (t < best) {
      best = t;
      bv = var;
    }
  }
  d.near_variant = bv;
  res->near_variant = bv;
  res->near_ms = best;
  bv = 0;
  best = 1e30;
  std::vector<int> csr_cands{0};
  if (std::is_same<T, float>::value) {
    csr_cands.push_back(1);
    if (d.run_ptr) csr_cands.push_back(2);
    if (d.bt_ntiles > 0 && nrhs % 16 == 0) {
      csr_cands.push_back(3);
      csr_cands.push_back(4);
    }
  } else if (d.bt_ntiles > 0 && nrhs % 16 == 0) {
    csr_cands.push_back(3);
  }
  for (int var : csr_cands) {
    d.csr_variant = var;
    double t;
    ls_status s = measure(7, 7, &t);
    if (s) return s;
    log("csr variant", var, 0, t);
    if (t < best) {
      best = t;
      bv = var;
    }
  }
  d.csr_variant = bv;
  res->csr_variant = bv;
  res->csr_ms = best;
  double t;
  ls_status s = measure(0, 7, &t);
  if (s) return s;
  res->apply_ms = t;
  // With the near field forked onto the side stream the stages share the
  // chip, and a schedule that is faster alone can be slower beside the others
  // (512-thread row transforms: faster alone, 0.714 against 0.681 ms per
  // concurrent apply with 256).  Coordinate descent over the transform
  // threads and tile and the interior contraction variant, timed on whole
  // concurrent applies.
  if (d.side) {
    // best of 3 runs of 6 back-to-back applies (as a solve issues them),
    // per apply
    auto conc = [&](double* best_t) -> ls_status {
      constexpr int K = 6;
      *best_t = 1e30;
      for (int rep = 0; rep < 3; ++rep) {
        HIPCHK(hipEventRecord(ev[0], st));
        for (int k = 0; k < K; ++k) {
          hipError_t e = lsx::launch_apply<T>(d, u, v, nrhs, ws, st);
          if (e != hipSuccess) return fail(LS_EDEVICE, std::string("apply launch: ") + hipGetErrorString(e));
        }
        HIPCHK(hipEventRecord(ev[8], st));
        HIPCHK(hipEventSynchronize(ev[8]));
        float ms = 0;
        (void)hipEventElapsedTime(&ms, ev[0], ev[8]);
        *best_t = std::min(*best_t, (double)ms / K);
      }
      return LS_OK;
    };
    double cur;
    s = conc(&cur);
    if (s) return s;
    log("concurrent apply (staged choices)", 0, 0, cur);
    // try one field at a time; keep a change only if the whole apply is faster
    auto trial = [&](int* field, int value, const char* what) -> ls_status {
      const int keep = *field;
      if (value == keep) return LS_OK;
      *field = value;
      double t2;
      ls_status s2 = conc(&t2);
      if (s2) return s2;
      log(what, value, 0, t2);
      if (t2 < cur) cur = t2;
      else *field = keep;
      return LS_OK;
    };
    for (int nth : {256, 512, 1024})
      if ((s = trial(&d.rows_nth, nth, "concurrent: fft row threads"))) return s;
    if (d.pb.n <= lsx::kRowIpMax)
      for (int ip : {1, 0})
        if ((s = trial(&d.rows_ip, ip, "concurrent: one-buffer row transforms"))) return s;
    if (d.fft_variant == 1)
      for (int cn : {256, 512})
        if ((s = trial(&d.cols_nth, cn, "concurrent: fft column threads"))) return s;
    {
      const int tmax = (int)((150 * 1024 - d.Pa * sizeof(T) * 2) /
                             (2 * (size_t)d.Pa * sizeof(T) * 2 * (d.fft_variant + 1)));
      const int t0 = d.tc;
      for (int tc : {t0 / 2, t0 * 2})
        if (tc >= 1 && tc <= tmax && (s = trial(&d.tc, tc, "concurrent: fft column tile"))) return s;
    }
    for (int var = 0; var < nnear; ++var)
      if ((s = trial(&d.near_variant, var, "concurrent: near variant"))) return s;
    for (int rf : {1, 0})
      if ((s = trial(&d.rows_first, rf, "concurrent: rows before the interior contraction"))) return s;
    res->fft_col_tile = d.tc;
    res->fft_row_threads = d.rows_nth;
    res->fft_col_threads = d.cols_nth;
    res->fft_rows_inplace = d.rows_ip;
    res->near_rows_first = d.rows_first;
    res->near_variant = d.near_variant;
    res->apply_ms = cur;
  }
  return LS_OK;
}
}  // namespace
}  // extern "C++"

ls_status ls_autotune(ls_op* op, int nrhs, ls_prec prec, void* stream, ls_tune_result* result) {
  if (!op || nrhs < 1 || !result) return fail(LS_EINVAL, "bad argument");
  if (prec != LS_C128 && prec != LS_C64) return fail(LS_EINVAL, "unknown precision");
  hipStream_t st = (hipStream_t)stream;
  const size_t c = prec == LS_C128 ? 16 : 8;
  const size_t vb = c * (size_t)op->N * nrhs, wsb = ws_bytes(op, nrhs, prec);
  std::lock_guard<std::recursive_mutex> lk(op->apply_mu);
  void* u = dev_alloc(op->alloc, vb);
  void* v = u ? dev_alloc(op->alloc, vb) : nullptr;
  void* ws = v ? dev_alloc(op->alloc, wsb) : nullptr;
  if (!ws) {
    dev_free(op->alloc, u, vb);
    dev_free(op->alloc, v, vb);
    return fail(LS_ENOMEM, "autotune buffers");
  }
  ls_status out = LS_OK;
  hipEvent_t ev[9] = {};
  for (int i = 0; i < 9 && out == LS_OK; ++i)
    if (hipEventCreate(&ev[i]) != hipSuccess) out = fail(LS_EDEVICE, "hipEventCreate");
  // a fixed nonzero input (byte pattern 0x3f: about 0.75 in float, 4.8e-4 in double)
  if (out == LS_OK && hipMemsetAsync(u, 0x3f, vb, st) != hipSuccess) out = fail(LS_EDEVICE, "memset");
  *result = ls_tune_result{};
  if (out == LS_OK)
    out = prec == LS_C128 ? autotune_view<double>(op, op->d64, nrhs, u, v, ws, st, ev, result)
                          : autotune_view<float>(op, op->d32, nrhs, u, v, ws, st, ev, result);
  (void)hipStreamSynchronize(st);
  for (int i = 0; i < 9; ++i)
    if (ev[i]) (void)hipEventDestroy(ev[i]);
  dev_free(op->alloc, u, vb);
  dev_free(op->alloc, v, vb);
  dev_free(op->alloc, ws, wsb);
  return out;
}

extern "C++" {
namespace {
template <typename T>
ls_status set_schedule_view(const ls_op* op, lsx::DevView<T>& d, const ls_tune_result* r) {
  const bool f32 = std::is_same<T, float>::value;
  const int fv = r->fft_variant;
  if (fv != 0 && fv != 1) return fail(LS_EINVAL, "fft_variant must be 0 or 1");
  const int tmax = (int)((150 * 1024 - d.Pa * sizeof(T) * 2) / (2 * (size_t)d.Pa * sizeof(T) * 2 * (fv + 1)));
  if (r->fft_col_tile < 1 || r->fft_col_tile > tmax)
    return fail(LS_EINVAL, "fft_col_tile outside 1 .. " + std::to_string(tmax));
  if (r->fft_row_threads != 256 && r->fft_row_threads != 512 && r->fft_row_threads != 1024)
    return fail(LS_EINVAL, "fft_row_threads must be 256, 512 or 1024");
  if (r->fft_col_threads != 256 && r->fft_col_threads != 512)
    return fail(LS_EINVAL, "fft_col_threads must be 256 or 512");
  if (r->near_variant < 0 || r->near_variant > (f32 ? 4 : 0)) return fail(LS_EINVAL, "near_variant out of range");
  if (r->csr_variant < 0 || r->csr_variant > 4 || (!f32 && r->csr_variant != 0 && r->csr_variant != 3))
    return fail(LS_EINVAL, "csr_variant out of range");
  if (r->csr_variant == 2 && !d.run_ptr) return fail(LS_EINVAL, "csr_variant 2: the op keeps no run-length columns");
  if (r->csr_variant >= 3 && d.bt_ntiles == 0) return fail(LS_EINVAL, "csr_variant 3 / 4: the op keeps no dense tiles");
  if (r->fft_rows_inplace != 0 && r->fft_rows_inplace != 1) return fail(LS_EINVAL, "fft_rows_inplace must be 0 or 1");
  if (r->fft_rows_inplace && d.pb.n > lsx::kRowIpMax) return fail(LS_EINVAL, "fft_rows_inplace: rows longer than 4096");
  if (r->near_rows_first != 0 && r->near_rows_first != 1) return fail(LS_EINVAL, "near_rows_first must be 0 or 1");
  (void)op;
  d.rows_ip = r->fft_rows_inplace;
  d.rows_first = r->near_rows_first;
  d.fft_variant = fv;
  d.tc = r->fft_col_tile;
  d.rows_nth = r->fft_row_threads;
  d.cols_nth = r->fft_col_threads;
  d.near_variant = r->near_variant;
  d.csr_variant = r->csr_variant;
  return LS_OK;
}
template <typename T>
void get_schedule_view(const lsx::DevView<T>& d, ls_tune_result* r) {
  *r = ls_tune_result{};
  r->fft_col_tile = d.tc;
  r->near_variant = d.near_variant;
  r->csr_variant = d.csr_variant;
  r->fft_variant = d.fft_variant;
  r->fft_row_threads = d.rows_nth;
  r->fft_col_threads = d.cols_nth;
  r->fft_rows_inplace = d.rows_ip;
  r->near_rows_first = d.rows_first;
}
}  // namespace
}  // extern "C++"

ls_status ls_set_schedule(ls_op* op, ls_prec prec, const ls_tune_result* sched) {
  if (!op || !sched) return fail(LS_EINVAL, "null argument");
  if (prec != LS_C128 && prec != LS_C64) return fail(LS_EINVAL, "unknown precision");
  std::lock_guard<std::recursive_mutex> lk(op->apply_mu);
  return prec == LS_C128 ? set_schedule_view<double>(op, op->d64, sched) : set_schedule_view<float>(op, op->d32, sched);
}

ls_status ls_get_schedule(const ls_op* op, ls_prec prec, ls_tune_result* sched) {
  if (!op || !sched) return fail(LS_EINVAL, "null argument");
  if (prec != LS_C128 && prec != LS_C64) return fail(LS_EINVAL, "unknown precision");
  if (prec == LS_C128) get_schedule_view<double>(op->d64, sched);
  else get_schedule_view<float>(op->d32, sched);
  return LS_OK;
}

// ---------------------------------------------------------------------------
// GMRES (Sec. 2: matrix-free GMRES in complex arithmetic).  All right-hand
// sides advance together; CGS2 Arnoldi in double precision on the device;
// the small Hessenberg least-squares problems (Givens rotations) on the host.
// ---------------------------------------------------------------------------
namespace {

struct Gm {
  ls_op* op;
  int nrhs, m;
  int64_t N;
  hipStream_t st;
  double2 *V, *w, *r, *tmp64, *rout, *e, *hdev, *partial;
  double2* hdev2[2];                       // per-step h1 | h2 | |w|^2, two slots (steps alternate)
  void *ws, *u32, *v32;
  double* sdev;
  size_t wsb;
  int nparts;
  bool cgs2 = true;
  bool use_graph = false;
  ls_prec inner_prec = LS_C128;            // apply precision of the double-basis GMRES
  char* base = nullptr;                    // workspace the buffers are carved from
  double apply_s = 0;
  int applies = 0;
  std::complex<double>* pinned[2] = {nullptr, nullptr};   // host copies of the two slots
  hipEvent_t ev[2] = {nullptr, nullptr};
  // per-stage device time (opts->profile): events in stream order, each
  // tagged with the stage of the interval that ends at it
  bool profile = false;
  std::vector<hipEvent_t> marks;
  std::vector<int> tags;
};

// record a profiling event closing an interval of stage `tag` (-1: start)
ls_status prof(Gm& g, int tag) {
  if (!g.profile) return LS_OK;
  hipEvent_t e = nullptr;
  HIPCHK(hipEventCreate(&e));
  g.marks.push_back(e);
  g.tags.push_back(tag);
  HIPCHK(hipEventRecord(e, g.st));
  return LS_OK;
}

void prof_collect(Gm& g, double* us4) {
  for (size_t i = 1; i < g.marks.size(); ++i) {
    float ms = 0;
    if (g.tags[i] >= 0 && hipEventElapsedTime(&ms, g.marks[i - 1], g.marks[i]) == hipSuccess)
      us4[g.tags[i]] += 1e3 * ms;
  }
  for (hipEvent_t e : g.marks) (void)hipEventDestroy(e);
  g.marks.clear();
  g.tags.clear();
}

size_t gm_slot(int nrhs, int m) { return (size_t)(m + 2) * nrhs * 2 + nrhs; }

size_t gm_need(const ls_op* op, int nrhs, int m) {
  size_t N = op->N;
  size_t v = 16 * N * nrhs;
  size_t b = v * (m + 1) + 5 * v + 16 * (size_t)(m + 2) * nrhs * 2 + 2 * 16 * gm_slot(nrhs, m) +
             16 * 1024 * (size_t)(m + 2) * nrhs + 8 * nrhs + ws_bytes(op, nrhs, LS_C128) + 2 * 8 * N * nrhs +
             16384;
  return b;
}

// carve the solver buffers from `ws` (caller's) or from the op's own scratch
ls_status gm_setup(Gm& g, void* ws, size_t ws_size) {
  size_t need = gm_need(g.op, g.nrhs, g.m);
  char* p = nullptr;
  if (ws) {
    if (ws_size < need) return fail(LS_EINVAL, "solver workspace too small");
    p = (char*)ws;
  } else {
    if (g.op->gm_bytes < need) {
      dev_free(g.op->alloc, g.op->gm, g.op->gm_bytes);
      g.op->gm = nullptr;
      g.op->gm_bytes = 0;
      g.op->gm = dev_alloc(g.op->alloc, need);
      if (!g.op->gm) return fail(LS_ENOMEM, "solver workspace");
      g.op->gm_bytes = need;
    }
    p = (char*)g.op->gm;
  }
  if (p != g.op->gm_last) {
    clear_graphs(g.op);     // captured steps point into the previous workspace
    g.op->gm_last = p;
  }
  g.base = p;
  if (g.use_graph && !g.op->cap_stream &&
      hipStreamCreateWithFlags(&g.op->cap_stream, hipStreamNonBlocking) != hipSuccess)
    return fail(LS_EDEVICE, "capture stream");
  auto take = [&](size_t bytes) {
    char* q = p;
    p += (bytes + 255) & ~size_t(255);
    return q;
  };
  size_t vb = 16 * (size_t)g.N * g.nrhs;
  g.V = (double2*)take(vb * (g.m + 1));    // complex double basis, or complex float basis in its first half
  g.w = (double2*)take(vb);
  g.r = (double2*)take(vb);
  g.tmp64 = (double2*)take(vb);
  g.rout = (double2*)take(vb);
  g.e = (double2*)take(vb);
  g.hdev = (double2*)take(16 * (size_t)(g.m + 2) * g.nrhs * 2);
  const size_t slot = gm_slot(g.nrhs, g.m);
  g.hdev2[0] = (double2*)take(16 * slot);
  g.hdev2[1] = (double2*)take(16 * slot);
  // workgroups of the reduction passes: about two elements per thread, at most 1024
  g.nparts = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (g.N + 511) / 512));
  g.partial = (double2*)take(16 * 1024 * (size_t)(g.m + 2) * g.nrhs);
  g.sdev = (double*)take(8 * g.nrhs);
  g.wsb = ws_bytes(g.op, g.nrhs, LS_C128);
  g.ws = take(g.wsb);
  g.u32 = take(8 * (size_t)g.N * g.nrhs);
  g.v32 = take(8 * (size_t)g.N * g.nrhs);
  if (!g.op->pinned || g.op->pinned_n < 2 * slot) {
    clear_graphs(g.op);     // captured steps copy into the old pinned slots
    if (g.op->pinned) (void)hipHostFree(g.op->pinned);
    g.op->pinned = nullptr;
    g.op->pinned_n = 2 * slot;
    if (hipHostMalloc((void**)&g.op->pinned, 16 * g.op->pinned_n) != hipSuccess) {
      g.op->pinned = nullptr;
      g.op->pinned_n = 0;
      return fail(LS_ENOMEM, "pinned host buffer");
    }
  }
  g.pinned[0] = g.op->pinned;
  g.pinned[1] = g.op->pinned + slot;
  for (int i = 0; i < 2; ++i) {
    if (!g.op->gm_ev[i] && hipEventCreateWithFlags(&g.op->gm_ev[i], hipEventDisableTiming) != hipSuccess)
      return fail(LS_EDEVICE, "hipEventCreate");
    g.ev[i] = g.op->gm_ev[i];
  }
  return LS_OK;
}

// y = A x between double vectors, the apply in precision prec (single: the
// input rounded, the output widened)
ls_status gm_apply(Gm& g, const double2* x, double2* y, ls_prec prec) {
  auto t0 = std::chrono::steady_clock::now();
  int64_t n = g.N * g.nrhs;
  ls_status s = prof(g, 3);
  if (s) return s;
  {
    std::lock_guard<std::recursive_mutex> lk(g.op->apply_mu);
    if (prec == LS_C128) {
      hipError_t e = lsx::launch_apply<double>(g.op->d64, x, y, g.nrhs, g.ws, g.st);
      if (e != hipSuccess) return fail(LS_EDEVICE, hipGetErrorString(e));
    } else {
      HIPCHK(lsx::gm_to_f32(x, g.u32, n, g.st));
      hipError_t e = lsx::launch_apply<float>(g.op->d32, g.u32, g.v32, g.nrhs, g.ws, g.st);
      if (e != hipSuccess) return fail(LS_EDEVICE, hipGetErrorString(e));
      HIPCHK(lsx::gm_to_f64(g.v32, y, n, g.st));
    }
  }
  s = prof(g, prec == LS_C128 ? 0 : 1);
  if (s) return s;
  g.apply_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  g.applies++;
  return LS_OK;
}

// single-precision apply between single-precision vectors
ls_status gm_apply32(Gm& g, const void* x, void* y) {
  auto t0 = std::chrono::steady_clock::now();
  ls_status s = prof(g, 3);
  if (s) return s;
  {
    std::lock_guard<std::recursive_mutex> lk(g.op->apply_mu);
    hipError_t e = lsx::launch_apply<float>(g.op->d32, x, y, g.nrhs, g.ws, g.st);
    if (e != hipSuccess) return fail(LS_EDEVICE, hipGetErrorString(e));
  }
  s = prof(g, 1);
  if (s) return s;
  g.apply_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  g.applies++;
  return LS_OK;
}

// d[r][j] = <V_j, w>_r for j < nvec (vstride between basis vectors)
ls_status gm_dots_host(Gm& g, const double2* Vb, const double2* w, int nvec, int64_t vstride,
                       std::vector<std::complex<double>>& out) {
  HIPCHK(lsx::gm_dots(Vb, w, g.partial, g.hdev, nvec, g.N, g.nrhs, vstride, g.nparts, g.st));
  out.resize((size_t)nvec * g.nrhs);
  HIPCHK(hipMemcpyAsync(out.data(), g.hdev, out.size() * 16, hipMemcpyDeviceToHost, g.st));
  HIPCHK(hipStreamSynchronize(g.st));
  return LS_OK;
}

bool finite_c(const std::complex<double>& z) { return std::isfinite(z.real()) && std::isfinite(z.imag()); }

// Hessenberg matrix of one restart cycle per right-hand side (column-major
// (m+1) x m), reduced to triangular form by Givens rotations as columns arrive.
struct Hessenberg {
  int R = 0, m = 0;
  std::vector<std::complex<double>> H, cs, sn, gv;
  std::vector<int> kdone;     // Krylov dimension at which each rhs met its tolerance (-1: not yet)

  void reset(int R_, int m_, const std::vector<double>& beta, const std::vector<double>& relres,
             const std::vector<double>& tol, const std::vector<char>& frozen) {
    R = R_;
    m = m_;
    H.assign((size_t)R * (m + 1) * m, 0.0);
    cs.assign((size_t)R * m, 0.0);
    sn.assign((size_t)R * m, 0.0);
    gv.assign((size_t)R * (m + 1), 0.0);
    kdone.assign(R, -1);
    for (int r = 0; r < R; ++r) {
      gv[(size_t)r * (m + 1)] = beta[r];
      if (frozen[r] || relres[r] <= tol[r]) kdone[r] = 0;
    }
  }

  // column k of rhs r: h_j = h1_j + h2_j (h2 may be null), h_{k+1} = hn.
  // Returns |residual| estimate after the rotation.
  double column(int r, int k, const std::complex<double>* h1, const std::complex<double>* h2, double hn) {
    std::complex<double>* col = &H[((size_t)r * m + k) * (m + 1)];
    for (int j = 0; j <= k; ++j) col[j] = h2 ? h1[j] + h2[j] : h1[j];
    col[k + 1] = hn;
    std::complex<double>* c = &cs[(size_t)r * m];
    std::complex<double>* sv = &sn[(size_t)r * m];
    for (int j = 0; j < k; ++j) {
      std::complex<double> t = c[j] * col[j] + sv[j] * col[j + 1];
      col[j + 1] = -std::conj(sv[j]) * col[j] + std::conj(c[j]) * col[j + 1];
      col[j] = t;
    }
    double den = std::sqrt(std::norm(col[k]) + std::norm(col[k + 1]));
    c[k] = den > 0 ? std::conj(col[k]) / den : 1.0;
    sv[k] = den > 0 ? std::conj(col[k + 1]) / den : 0.0;
    col[k] = den;
    col[k + 1] = 0.0;
    std::complex<double>* gg = &gv[(size_t)r * (m + 1)];
    gg[k + 1] = -std::conj(sv[k]) * gg[k];
    gg[k] = c[k] * gg[k];
    return std::abs(gg[k + 1]);
  }

  // coefficients y[r][0..k) of the cycle's update (each rhs uses its own
  // dimension; a zero diagonal, an exact breakdown, ends that rhs's sum)
  std::vector<std::complex<double>> solve(int k) const {
    std::vector<std::complex<double>> y((size_t)R * std::max(k, 1), 0.0);
    for (int r = 0; r < R; ++r) {
      int kk = kdone[r] >= 0 ? kdone[r] : k;
      const std::complex<double>* Hr = &H[(size_t)r * m * (m + 1)];
      const std::complex<double>* gg = &gv[(size_t)r * (m + 1)];
      while (kk > 0 && Hr[(size_t)(kk - 1) * (m + 1) + kk - 1] == 0.0) --kk;
      std::complex<double>* yr = &y[(size_t)r * k];
      for (int i = kk - 1; i >= 0; --i) {
        std::complex<double> sacc = gg[i];
        for (int j = i + 1; j < kk; ++j) sacc -= Hr[(size_t)j * (m + 1) + i] * yr[j];
        yr[i] = sacc / Hr[(size_t)i * (m + 1) + i];
      }
    }
    return y;
  }
};

// Per right-hand side outcome flags of a solve
enum : char { RHS_OK = 0, RHS_NUMERIC = 1, RHS_STAGNANT = 2 };

// Solve A x = f (x holds the initial guess; f and x complex double) to
// relative residual tol.  F32: Krylov basis, work vector and operator apply
// in single precision (reductions and the update of x in double); otherwise
// basis and Arnoldi in double with the apply in g.inner_prec.  The
// orthogonalisation is classical Gram–Schmidt, applied twice when g.cgs2.
// Step k+1 is queued on the stream before the host waits for the Hessenberg
// column of step k, so the device never waits for the host inside a cycle;
// when step k meets the tolerance the queued step is discarded.
// flag[r]: a non-finite norm or Hessenberg entry freezes the right-hand side
// at its last finite step (RHS_NUMERIC); a restart cycle that leaves its
// residual unchanged (to 1e-12 relative) freezes it as RHS_STAGNANT: the
// next cycle would build the same Krylov space again.
extern "C++" {
template <bool F32>
ls_status gmres(Gm& g, const double2* f, double2* x, bool x_zero, const std::vector<double>& tol, int max_iter,
                int* iters, std::vector<double>& relres, std::vector<char>& flag) {
  const int R = g.nrhs, m = g.m;
  const int64_t N = g.N;
  const int64_t vstride = N * R;          // distance between basis vectors (elements)
  float2* V32 = (float2*)g.V;
  float2* w32 = (float2*)g.w;
  std::vector<std::complex<double>> dd;
  std::vector<double> fnorm(R), prev_beta(R, -1.0);
  ls_status s = gm_dots_host(g, f, f, 1, 0, dd);
  if (s) return s;
  for (int r = 0; r < R; ++r) {
    fnorm[r] = std::sqrt(std::max(0.0, dd[r].real()));
    if (!std::isfinite(dd[r].real())) flag[r] = RHS_NUMERIC;
  }
  relres.assign(R, 1.0);
  Hessenberg hs;
  int it = 0;
  bool first = true;

  // one Arnoldi step: w = A V_k, orthogonalise against V_0..V_k, V_{k+1} = w / |w|,
  // then h1 | h2 | |w|^2 to the host slot (k & 1)
  auto step = [&](int k) -> ls_status {
    const int nv = k + 1;
    const size_t nh = (size_t)nv * R;
    double2* d1 = g.hdev2[k & 1];
    double2* d2 = d1 + nh;
    double2* dn = d1 + 2 * nh;
    ls_status st;
    if (F32) {
      st = gm_apply32(g, V32 + (size_t)k * vstride, w32);
      if (st) return st;
      float2* vnext = V32 + (size_t)(k + 1) * vstride;
      HIPCHK(lsx::gm32_dots(V32, w32, g.partial, d1, nv, nv, N, R, vstride, g.nparts, g.st));
      if (g.cgs2) {
        HIPCHK(lsx::gm32_update(V32, w32, w32, d1, nv, N, R, vstride, g.nparts, g.partial, nullptr, g.st));
        HIPCHK(lsx::gm32_dots(V32, w32, g.partial, d2, nv, nv, N, R, vstride, g.nparts, g.st));
        HIPCHK(lsx::gm32_update(V32, w32, vnext, d2, nv, N, R, vstride, g.nparts, g.partial, dn, g.st));
      } else {
        HIPCHK(lsx::gm32_update(V32, w32, vnext, d1, nv, N, R, vstride, g.nparts, g.partial, dn, g.st));
      }
      HIPCHK(lsx::gm_inv_norm(dn, g.sdev, R, g.st));
      HIPCHK(lsx::gm32_scale(vnext, g.sdev, N, R, g.st));
    } else {
      st = gm_apply(g, g.V + (size_t)k * vstride, g.w, g.inner_prec);
      if (st) return st;
      HIPCHK(lsx::gm_cgs(g.V, g.w, nullptr, g.partial, d1, nv, N, R, vstride, g.nparts, 0, g.st));
      if (g.cgs2) HIPCHK(lsx::gm_cgs(g.V, g.w, d1, g.partial, d2, nv, N, R, vstride, g.nparts, 1, g.st));
      HIPCHK(lsx::gm_cgs(g.V, g.w, g.cgs2 ? d2 : d1, g.partial, dn, nv, N, R, vstride, g.nparts, 2, g.st));
      HIPCHK(lsx::gm_inv_norm(dn, g.sdev, R, g.st));
      HIPCHK(lsx::gm_scale_copy(g.w, g.V + (size_t)(k + 1) * vstride, g.sdev, N, R, g.st));
    }
    st = prof(g, 2);
    if (st) return st;
    HIPCHK(hipMemcpyAsync(g.pinned[k & 1], d1, 16 * (2 * nh + R), hipMemcpyDeviceToHost, g.st));
    return LS_OK;
  };
  // one step, replayed from a captured graph when g.use_graph (captured on
  // first use for this step index and kept with the op), then the event the
  // host waits on
  auto launch_step = [&](int k) -> ls_status {
    if (g.use_graph) {
      const GraphKey key{F32, g.cgs2, R, m, k, (uintptr_t)g.base, N * 4 + (int64_t)g.inner_prec};
      auto it = g.op->graphs.find(key);
      if (it == g.op->graphs.end()) {
        std::lock_guard<std::recursive_mutex> lk(g.op->apply_mu);
        hipStream_t user = g.st;
        g.st = g.op->cap_stream;
        HIPCHK(hipStreamBeginCapture(g.st, hipStreamCaptureModeRelaxed));
        ls_status st2 = step(k);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(g.st, &graph);
        g.st = user;
        if (st2) {
          if (graph) (void)hipGraphDestroy(graph);
          return st2;
        }
        if (e != hipSuccess) return fail(LS_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return fail(LS_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
        it = g.op->graphs.emplace(key, exec).first;
      }
      HIPCHK(hipGraphLaunch(it->second, g.st));
    } else {
      ls_status st2 = step(k);
      if (st2) return st2;
    }
    HIPCHK(hipEventRecord(g.ev[k & 1], g.st));
    return LS_OK;
  };

  while (true) {
    // r = f - A x, V_0 = r / |r|
    std::vector<double> beta(R);
    if (F32) {
      const float2* ax = nullptr;
      if (!(x_zero && first)) {
        HIPCHK(lsx::gm_to_f32(x, g.u32, N * R, g.st));
        s = gm_apply32(g, g.u32, w32);
        if (s) return s;
        ax = w32;
      }
      HIPCHK(lsx::gm32_resid(f, ax, V32, N, R, g.nparts, g.partial, g.hdev, g.st));
      dd.resize(R);
      HIPCHK(hipMemcpyAsync(dd.data(), g.hdev, 16 * R, hipMemcpyDeviceToHost, g.st));
      HIPCHK(hipStreamSynchronize(g.st));
    } else {
      if (x_zero && first) {
        HIPCHK(hipMemcpyAsync(g.r, f, 16 * (size_t)N * R, hipMemcpyDeviceToDevice, g.st));
      } else {
        s = gm_apply(g, x, g.w, g.inner_prec);
        if (s) return s;
        HIPCHK(lsx::gm_sub(f, g.w, g.r, N * R, g.st));
      }
      s = gm_dots_host(g, g.r, g.r, 1, 0, dd);
      if (s) return s;
    }
    first = false;
    bool all = true;
    for (int r = 0; r < R; ++r) {
      beta[r] = std::sqrt(std::max(0.0, dd[r].real()));
      if (!std::isfinite(dd[r].real())) flag[r] = RHS_NUMERIC;
      relres[r] = fnorm[r] > 0 ? beta[r] / fnorm[r] : 0.0;
      if (!flag[r] && prev_beta[r] >= 0 && relres[r] > tol[r] && beta[r] >= prev_beta[r] * (1.0 - 1e-12))
        flag[r] = RHS_STAGNANT;
      prev_beta[r] = beta[r];
      if (!flag[r] && relres[r] > tol[r]) all = false;
    }
    if (all || it >= max_iter) break;
    std::vector<double> inv(R);
    for (int r = 0; r < R; ++r) inv[r] = (beta[r] > 0 && !flag[r]) ? 1.0 / beta[r] : 0.0;
    HIPCHK(hipMemcpyAsync(g.sdev, inv.data(), 8 * R, hipMemcpyHostToDevice, g.st));
    if (F32)
      HIPCHK(lsx::gm32_scale(V32, g.sdev, N, R, g.st));
    else
      HIPCHK(lsx::gm_scale_copy(g.r, g.V, g.sdev, N, R, g.st));
    hs.reset(R, m, beta, relres, tol, flag);
    int k = 0;
    s = launch_step(0);
    if (s) return s;
    for (; k < m && it < max_iter; ++k) {
      if (k + 1 < m && it + 1 < max_iter) {
        s = launch_step(k + 1);
        if (s) return s;
      }
      HIPCHK(hipEventSynchronize(g.ev[k & 1]));
      ++it;
      const size_t nh = (size_t)(k + 1) * R;
      const std::complex<double>* h1 = g.pinned[k & 1];
      const std::complex<double>* h2 = g.cgs2 ? h1 + nh : nullptr;
      const std::complex<double>* dn = h1 + 2 * nh;
      bool all_done = true;
      for (int r = 0; r < R; ++r) {
        if (hs.kdone[r] >= 0) continue;
        const std::complex<double>* c1 = h1 + (size_t)r * (k + 1);
        const std::complex<double>* c2 = h2 ? h2 + (size_t)r * (k + 1) : nullptr;
        bool fin = std::isfinite(dn[r].real());
        for (int j = 0; j <= k && fin; ++j) fin = finite_c(c1[j]) && (!c2 || finite_c(c2[j]));
        if (!fin) {
          // keep the k finite columns of this cycle; freeze the rhs
          flag[r] = RHS_NUMERIC;
          hs.kdone[r] = k;
          continue;
        }
        double hn = std::sqrt(std::max(0.0, dn[r].real()));
        double est = hs.column(r, k, c1, c2, hn);
        est = fnorm[r] > 0 ? est / fnorm[r] : 0.0;
        if (est <= tol[r] || hn == 0.0) hs.kdone[r] = k + 1;
        if (hs.kdone[r] < 0) all_done = false;
      }
      if (all_done) { ++k; break; }
    }
    // x += V y
    std::vector<std::complex<double>> yk = hs.solve(k);
    HIPCHK(hipMemcpyAsync(g.hdev, yk.data(), 16 * yk.size(), hipMemcpyHostToDevice, g.st));
    if (k > 0) {
      if (F32)
        HIPCHK(lsx::gm32_axpy_combo(x, V32, g.hdev, k, N, R, vstride, g.st));
      else
        HIPCHK(lsx::gm_axpy_combo(x, g.V, g.hdev, k, N, R, vstride, g.st));
    }
  }
  *iters = it;
  return LS_OK;
}
}  // extern "C++"

}  // namespace

ls_status ls_solve_workspace_size(const ls_op* op, int nrhs, const ls_solve_opts* opts, size_t* bytes) {
  if (!op || !opts || !bytes || nrhs < 1 || opts->restart < 1) return fail(LS_EINVAL, "bad argument");
  *bytes = gm_need(op, nrhs, opts->restart);
  return LS_OK;
}

extern "C++" {
namespace {
ls_status solve_locked(ls_op* op, const void* u_inc, void* u_tot, int nrhs, const ls_solve_opts* opts,
                       ls_solve_stats* stats, void* ws, size_t ws_size, hipStream_t stream) {
  auto t0 = std::chrono::steady_clock::now();
  Gm g{};
  g.op = op;
  g.nrhs = nrhs;
  g.m = opts->restart;
  g.N = op->N;
  g.st = stream;
  g.cgs2 = opts->ortho != LS_ORTHO_CGS1;
  g.use_graph = opts->graph != 0;
  g.profile = opts->profile != 0 && !g.use_graph;
  ls_status s = gm_setup(g, ws, ws_size);
  if (s) return s;
  double us4[4] = {0, 0, 0, 0};
  struct ProfGuard {
    Gm& g;
    double* us;
    ~ProfGuard() {
      if (!g.marks.empty()) {
        (void)hipEventSynchronize(g.marks.back());
        prof_collect(g, us);
      }
    }
  } guard{g, us4};
  s = prof(g, -1);
  if (s) return s;
  const double2* f = (const double2*)u_inc;
  double2* x = (double2*)u_tot;
  const int64_t n = op->N * nrhs;
  if (!opts->use_x0) HIPCHK(hipMemsetAsync(x, 0, 16 * (size_t)n, g.st));
  int iters = 0, outer = 0;
  std::vector<double> rel;
  std::vector<char> flag(nrhs, RHS_OK);
  bool have_r = false;   // g.r holds f - A x of the final iterate
  if (opts->mode == LS_SOLVE_FP64) {
    s = gmres<false>(g, f, x, !opts->use_x0, std::vector<double>(nrhs, opts->tol), opts->max_iter, &iters, rel,
                     flag);
    if (s) return s;
  } else {
    // FP64 residual, FP32 inner solves, x += e.  Each inner solve stops at
    // the looser of inner_tol and half the reduction its right-hand side
    // still needs to reach tol, so the last correction is no longer than
    // necessary.  A refinement step that no longer reduces a right-hand
    // side's residual (to 1e-12 relative) freezes it as stagnant.
    int total = 0;
    bool xzero = !opts->use_x0;
    std::vector<double> prev(nrhs, -1.0);
    for (outer = 0;; ++outer) {
      if (xzero) {
        HIPCHK(hipMemcpyAsync(g.rout, f, 16 * (size_t)n, hipMemcpyDeviceToDevice, g.st));
      } else {
        s = gm_apply(g, x, g.w, LS_C128);
        if (s) return s;
        HIPCHK(lsx::gm_sub(f, g.w, g.rout, n, g.st));
      }
      std::vector<std::complex<double>> dr, df;
      s = gm_dots_host(g, g.rout, g.rout, 1, 0, dr);
      if (s) return s;
      s = gm_dots_host(g, f, f, 1, 0, df);
      if (s) return s;
      bool all = true;
      std::vector<char> done(nrhs, 0);
      for (int k = 0; k < nrhs; ++k) {
        const double rn = std::sqrt(std::max(0.0, dr[k].real())), fn = std::sqrt(std::max(0.0, df[k].real()));
        if (!std::isfinite(dr[k].real()) || !std::isfinite(df[k].real())) flag[k] = RHS_NUMERIC;
        if (!flag[k] && prev[k] >= 0 && rn > opts->tol * fn && rn >= prev[k] * (1.0 - 1e-12)) flag[k] = RHS_STAGNANT;
        prev[k] = rn;
        done[k] = flag[k] || rn <= opts->tol * fn;
        if (!done[k]) all = false;
      }
      if (all || total >= opts->max_iter || outer >= std::max(1, opts->max_outer)) {
        HIPCHK(hipMemcpyAsync(g.r, g.rout, 16 * (size_t)n, hipMemcpyDeviceToDevice, g.st));
        have_r = true;
        break;
      }
      std::vector<double> itol(nrhs);
      for (int k = 0; k < nrhs; ++k) {
        const double rn = std::sqrt(std::max(0.0, dr[k].real())), fn = std::sqrt(std::max(0.0, df[k].real()));
        itol[k] = rn > 0 ? std::min(0.5, std::max(opts->inner_tol, 0.5 * opts->tol * fn / rn)) : opts->inner_tol;
      }
      // right-hand sides that are done get no further correction, so each
      // one ends exactly where its own solve would
      for (int k = 0; k < nrhs; ++k)
        if (done[k]) HIPCHK(hipMemsetAsync(g.rout + (size_t)k * op->N, 0, 16 * (size_t)op->N, g.st));
      HIPCHK(hipMemsetAsync(g.e, 0, 16 * (size_t)n, g.st));
      int it = 0;
      std::vector<double> rr;
      std::vector<char> iflag(nrhs, RHS_OK);
      if (opts->inner_f64_basis) {
        g.inner_prec = LS_C64;
        s = gmres<false>(g, g.rout, g.e, true, itol, opts->max_iter - total, &it, rr, iflag);
        g.inner_prec = LS_C128;
      } else {
        s = gmres<true>(g, g.rout, g.e, true, itol, opts->max_iter - total, &it, rr, iflag);
      }
      if (s) return s;
      for (int k = 0; k < nrhs; ++k)
        if (iflag[k] == RHS_NUMERIC) flag[k] = RHS_NUMERIC;
      total += it;
      HIPCHK(lsx::gm_add(x, g.e, n, g.st));
      xzero = false;
    }
    iters = total;
  }
  // true FP64 residual (the refinement loop ends with it in g.r)
  if (!have_r) {
    s = gm_apply(g, x, g.w, LS_C128);
    if (s) return s;
    HIPCHK(lsx::gm_sub(f, g.w, g.r, n, g.st));
  }
  std::vector<std::complex<double>> dr, df;
  s = gm_dots_host(g, g.r, g.r, 1, 0, dr);
  if (s) return s;
  s = gm_dots_host(g, f, f, 1, 0, df);
  if (s) return s;
  s = prof(g, 3);
  if (s) return s;
  HIPCHK(hipStreamSynchronize(g.st));
  double worst = 0;
  int conv = 0;
  bool numeric = false;
  for (int k = 0; k < nrhs; ++k) {
    const bool fin = std::isfinite(dr[k].real()) && std::isfinite(df[k].real());
    double rr = !fin ? std::numeric_limits<double>::quiet_NaN()
                     : df[k].real() > 0 ? std::sqrt(dr[k].real() / df[k].real()) : 0.0;
    if (!fin) flag[k] = RHS_NUMERIC;
    if (flag[k] == RHS_NUMERIC) {
      numeric = true;
      worst = std::numeric_limits<double>::quiet_NaN();
      continue;
    }
    if (!std::isnan(worst)) worst = std::max(worst, rr);
    if (rr <= opts->tol) ++conv;
  }
  if (stats) {
    stats->iterations = iters;
    stats->outer = outer;
    stats->converged = conv;
    stats->rel_residual = worst;
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    stats->apply_seconds = g.apply_s;
    prof_collect(g, us4);
    for (int i = 0; i < 4; ++i) stats->stage_us[i] = us4[i];
  }
  if (numeric) return fail(LS_ENUMERIC, "non-finite value in the right-hand side or the iteration");
  return conv == nrhs ? LS_OK : fail(LS_ENOCONV, "tolerance not reached");
}
}  // namespace
}  // extern "C++"

ls_status ls_solve(ls_op* op, const void* u_inc, void* u_tot, int nrhs, const ls_solve_opts* opts,
                   ls_solve_stats* stats, void* ws, size_t ws_size, void* stream) {
  if (!op || !u_inc || !u_tot || !opts || nrhs < 1) return fail(LS_EINVAL, "null argument");
  if (opts->restart < 1 || opts->max_iter < 1 || !(opts->tol > 0)) return fail(LS_EINVAL, "bad solver options");
  if (opts->mode != LS_SOLVE_FP64 && opts->mode != LS_SOLVE_FP32_REFINE) return fail(LS_EINVAL, "unknown mode");
  if (stats) *stats = ls_solve_stats{};
  std::lock_guard<std::mutex> lk(op->solve_mu);
  return solve_locked(op, u_inc, u_tot, nrhs, opts, stats, ws, ws_size, (hipStream_t)stream);
}

}  // extern "C"
