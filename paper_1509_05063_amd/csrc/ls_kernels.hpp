// Device-side views and launchers (internal header).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace lsx {

struct FftPlan {
  int n;
  int npass;
  int8_t radix[28];
};

// Everything one apply needs, for one precision T (double or float).
// longest row the one-buffer row transform takes
constexpr int kRowIpMax = 4096;

template <typename T>
struct DevView {
  int64_t N = 0;
  int ncell = 0, nicell = 0, S = 0, U = 0, F = 0, q = 0, L = 0, na = 0, nb = 0, Pa = 0, Pb = 0, ch = 0;
  int max_nb = 0, tc = 1, nrows = 0;
  int64_t nband = 0;   // boundary-patch nodes (Ibd is stored as [F][nband])
  // kernel variants chosen by ls_autotune: near_variant 0 = double-buffered
  // interior contraction, 16 cells per workgroup (single precision), 1 =
  // single-buffered, 2 / 3 = double-buffered with 32 / 64 cells; csr_variant
  // 0 = four entries per lane (single precision, 16-bit offsets), 1 = one,
  // 2 = four entries per lane with run-length columns, 3 = dense tiles on
  // the matrix cores (right-hand-side-major input; used when nrhs is a
  // multiple of 16, else as 2)
  int near_variant = 0, csr_variant = 0;
  // nonzero: row transforms with one LDS buffer (rows of at most kRowIpMax
  // points)
  int rows_ip = 0;
  // concurrent apply: nonzero runs the boundary-patch rows before the
  // interior contraction on the side stream
  int rows_first = 0;
  // fft_variant 0 = separate column transforms and spectral product, 1 =
  // fused per column tile
  int fft_variant = 0;
  int rows_nth = 256;   // threads per workgroup of the row transforms (256, 512, 1024)
  int cols_nth = 256;   // threads per workgroup of the fused column kernel (256, 512)
  bool csr_f64 = true;
  double kappa = 0;
  const void *Psh = nullptr, *PshT = nullptr, *Pbd = nullptr, *Ish = nullptr, *Ibd = nullptr, *Toff = nullptr, *Wsh = nullptr;
  const void *khat = nullptr, *twa = nullptr, *twb = nullptr, *vals = nullptr;
  const T *cw = nullptr, *dw = nullptr;
  const int32_t *slot_map = nullptr, *cell_start = nullptr, *cell_nint = nullptr, *cell_nb = nullptr;
  const int32_t *cell_boff = nullptr, *cell_xy = nullptr, *cell_map = nullptr, *icells = nullptr;
  // cells holding boundary-patch nodes, and whether the projection runs on
  // the matrix cores (k_project_int + k_project_band; else the older
  // per-cell kernels)
  const int32_t* bcells = nullptr;
  int nbcell = 0;
  bool proj_mfma = true;
  const int32_t *rows = nullptr, *colbase = nullptr;
  const uint16_t* coloff = nullptr;   // column = colbase[row] + coloff[k] (16-bit form)
  const int32_t* cols32 = nullptr;    // column = colbase[row] + cols32[k] (when a row spans > 65535)
  const int64_t* rowptr = nullptr;
  // the same columns as runs of consecutive indices: run r of row i is
  // run_ptr[i] + r, covering the row's entries from run_pre on at columns
  // run_cs, run_cs + 1, ... (null when some row has more than 256 runs);
  // run_max: the largest number of runs of a row
  const int32_t *run_ptr = nullptr, *run_cs = nullptr, *run_pre = nullptr;
  int run_max = 0;
  // Single precision only: the same rows as dense tiles of 16 rows of one
  // cell and kind (boundary-patch or interior targets).  Tile t: target rows
  // bt_rows[16 t ..] (-1 = padding), K = bt_info[2 t] (multiple of 4)
  // columns listed at bt_cols + bt_info[2 t + 1] (the points of the 3 x 3
  // adjacent cells the rows all couple to, then the union of the rows'
  // other columns), weights at bt_w + bt_woff[t] as [K / 4][4 columns][16
  // rows], zero where a row has no entry.
  int bt_ntiles = 0;
  const int32_t *bt_rows = nullptr, *bt_info = nullptr, *bt_cols = nullptr;
  const int64_t* bt_woff = nullptr;
  const void* bt_w = nullptr;
  // Concurrent near field: when set, an apply that is not being profiled
  // runs the near-field kernels on `side` (forked from the caller's stream
  // at ev_fork, accumulating into a workspace buffer) while the far field
  // runs on the caller's stream, and joins at ev_join before adding the
  // buffer into v.
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  FftPlan pa{}, pb{};
  // Fourier refinement of the band's t1 lines (rf = 1: none): rf_lines
  // lines of rf_n1 points, op index and density weight of each grid node at
  // rf_idx / rf_dens [line][v]; rf_ph [(rf - 1)][rf_n1] the phase ramps of
  // the shifts s / rf divided by rf_n1 (complex T), rf_tw the line
  // transform's twiddles.  The rows then read x = [u ; refined values], ldx
  // entries per right-hand side (the refined value at t1 = v + s / rf of
  // line l at N + ((s - 1) rf_lines + l) rf_n1 + v).
  int rf = 1, rf_n1 = 0, rf_lines = 0;
  int64_t ldx = 0;
  // psi grid side (the lattice box of the cells plus two cells per side, or
  // with interior refinement its period M, prime factors 2, 3, 5); interior
  // refinement (rfi = rf, else 1): the refined psi grid of shift s = s2 rf +
  // s1 > 0 at x + N + rf_ioff + (s - 1) gw^2 (stride gw), window s at Wsh +
  // s S Wn^2; rf_iph [rf][gw] the phase ramps / gw, rf_itw the twiddles
  int gw = 0, rfi = 1;
  int64_t rf_ioff = 0;
  // off-grid shortcut (nsr > 0): nsr rows of the boundary rule at the
  // patch's grid nodes (output column sr_rows in x, CSR with 32-bit column
  // offsets from sr_colbase, weights complex T); their values s at x + N +
  // sc_off + u N1 + v, the refined s lines after them
  int nsr = 0;
  int64_t sc_off = 0;
  const int64_t* sr_rowptr = nullptr;
  const int32_t *sr_rows = nullptr, *sr_colbase = nullptr, *sr_cols32 = nullptr;
  const void* sr_vals = nullptr;
  const void *rf_iph = nullptr, *rf_itw = nullptr;
  FftPlan rf_iplan{};
  const int32_t* rf_idx = nullptr;
  const T* rf_dens = nullptr;
  const void *rf_ph = nullptr, *rf_tw = nullptr;
  FftPlan rf_plan{};
};

// lattice_only: stop after the inverse transforms (workspace holds the
// strengths and the face-lattice field; v is not touched)
template <typename T>
hipError_t launch_apply(const DevView<T>& d, const void* u, void* v, int nrhs, void* ws, hipStream_t st,
                        hipEvent_t* ev = nullptr, bool lattice_only = false);

// Targets off the scatterer, sorted by their cell of the lattice box.
struct TargetView {
  int64_t n = 0;                 // targets
  int ncell = 0;                 // target cells
  const int32_t *cell_xy = nullptr, *start = nullptr, *orig = nullptr;   // [ncell][2], [ncell+1], [n]
  const void* fit = nullptr;     // [n][F] complex double: face values -> field at the target
  const int64_t* rowptr = nullptr;
  // the same columns as runs of consecutive indices: run r of row i is
  // run_ptr[i] + r, covering the row's entries from run_pre on at columns
  // run_cs, run_cs + 1, ... (null when some row has more than 256 runs)
  const int32_t *run_ptr = nullptr, *run_cs = nullptr, *run_pre = nullptr;   // [n+1] adjacent-cell sources
  const int32_t* cols = nullptr;
  const void* vals = nullptr;    // complex double G(|x - y_j|) c_j
};
// out[r][n] = scattered field at the targets for the totals u [nrhs][N]
hipError_t launch_targets(const DevView<double>& d, const TargetView& tg, const void* u, void* out, int nrhs,
                          void* ws, hipStream_t st);
hipError_t launch_fft_kernels_forward(const DevView<double>& d, void* data, int nbatch, hipStream_t st);
// Set-up: adds the adjacent far-field subtraction to the stored weights of
// the rows touching the boundary patch, both precisions (olen: entries per
// row before padding; pt_cell: cell of each point; pt_idx: slot of an
// interior point, -(boundary ordinal + 1) of a boundary-patch point).
hipError_t launch_fold_rows(const DevView<double>& a, const DevView<float>& b, const int64_t* olen,
                            const int32_t* pt_cell, const int32_t* pt_idx, hipStream_t st);
// One-axis transforms of multi-dimensional arrays (3-D face lattices).
int fft_lines_per_group(bool dbl, int n);
hipError_t launch_fft_lines(bool dbl, int dir, const void* src, void* dst, const void* tw, const FftPlan& plan,
                            int nlines, int64_t s_line, int64_t s_batch, int64_t s_z, int64_t d_line, int64_t d_batch,
                            int64_t d_z, int nbatch, int nz, int nload, int nstore, hipStream_t st);
hipError_t launch_fft_strided(bool dbl, int dir, void* data, const void* tw, const FftPlan& plan, int ncols, int TC,
                              int64_t batch_stride, int nbatch, int nload, int nstore, int64_t zstride, int nz,
                              hipStream_t st);
// Fused transform along the normal axis of 3-D face lattices, spectral
// product with octant-stored kernel spectra khs [2][Pa/2+1][Pb/2+1][Pc/2+1]
// and inverse transform, single precision: nsets sets of [2 kinds][Pa][Pb][Pc]
// (planes rstride >= Pb Pc apart, vol per kind); rows < na are read and, in
// kind 0, written back
hipError_t launch_fft_conv_octant(void* data, const void* tw, const void* khs, const FftPlan& plan, int Pb, int Pc,
                                  int TC, int nth, int64_t rstride, int64_t vol, int na, int nsets, hipStream_t st);
FftPlan make_fft_plan(int n);
hipError_t set_fft_lds_limits(size_t bytes);

// GMRES building blocks (double complex)
hipError_t gm_dots(const void* Vb, const void* w, void* partial, void* out, int nvec, int64_t N, int nrhs,
                   int64_t vstride, int nparts, hipStream_t st);
hipError_t gm_cgs(const void* Vb, void* w, const void* h, void* partial, void* out, int nvec, int64_t N,
                  int nrhs, int64_t vstride, int nparts, int mode, hipStream_t st);
hipError_t gm_inv_norm(const void* dd, double* s, int nrhs, hipStream_t st);
hipError_t gm_update(const void* Vb, void* w, const void* h, int nvec, int64_t N, int nrhs, int64_t vstride,
                     hipStream_t st);
hipError_t gm_scale_copy(const void* src, void* dst, const double* s, int64_t N, int nrhs, hipStream_t st);
hipError_t gm_axpy_combo(void* x, const void* Vb, const void* y, int nvec, int64_t N, int nrhs, int64_t vstride,
                         hipStream_t st);
hipError_t gm_sub(const void* a, const void* b, void* out, int64_t n, hipStream_t st);
hipError_t gm_add(void* x, const void* e, int64_t n, hipStream_t st);
hipError_t gm_to_f32(const void* a, void* b, int64_t n, hipStream_t st);
hipError_t gm_to_f64(const void* a, void* b, int64_t n, hipStream_t st);

// GMRES building blocks with a single-precision basis (complex float
// vectors, reductions in double).  dots: out[r * ldo + j] = <V_j, w_r>.
// update: dst = src - sum_j h[r * nvec + j] V_j, |dst|^2 to norm_out[r] when
// norm_out != nullptr.  resid: dst = f - a (a may be null), |f - a|^2.
hipError_t gm32_dots(const void* Vb, const void* w, void* partial, void* out, int nvec, int ldo, int64_t N,
                     int nrhs, int64_t vstride, int nparts, hipStream_t st);
hipError_t gm32_update(const void* Vb, const void* src, void* dst, const void* h, int nvec, int64_t N, int nrhs,
                       int64_t vstride, int nparts, void* partial, void* norm_out, hipStream_t st);
hipError_t gm32_resid(const void* f, const void* a, void* dst, int64_t N, int nrhs, int nparts, void* partial,
                      void* norm_out, hipStream_t st);
hipError_t gm32_scale(void* v, const double* s, int64_t N, int nrhs, hipStream_t st);
hipError_t gm32_axpy_combo(void* x, const void* Vb, const void* y, int nvec, int64_t N, int nrhs, int64_t vstride,
                           hipStream_t st);

}  // namespace lsx
