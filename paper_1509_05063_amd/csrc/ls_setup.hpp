// Host-side set-up of the 2-D operator (internal header).
//
// Everything here is double precision and runs once per operator in
// ls_create; the device side only sees the flat arrays of HostOp.
#pragma once
#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "ls.h"

namespace lsx {

using cd = std::complex<double>;

struct HostOp {
  ls_geometry g{};
  ls_params p{};
  double kappa = 0;

  // ---- Nystrom nodes in operator order (sorted by cell) -----------------
  int64_t N = 0;
  std::vector<double> xy;       // 2N
  std::vector<int32_t> key;     // 3N: (patch, i1, i2)
  std::vector<double> cw;       // plain quadrature weight c_j = w |J| omega m
  std::vector<double> dw;       // interior nodes: m omega (density of the
                                // interior singular rule); boundary nodes: 0

  // ---- cells (side H = cell_h h, aligned with the interior lattice) ------
  double H = 0;
  int S = 0;                    // cell_h^2 interior slots per cell
  int L = 0;                    // cells per axis
  int64_t c_lo = 0;             // cell(x) = floor(x / H) - c_lo
  int ncell = 0;                // occupied cells
  std::vector<int32_t> cell_xy;     // 2 per occupied cell
  std::vector<int32_t> cell_map;    // L*L -> occupied index or -1
  std::vector<int32_t> cell_start;  // first op index of the cell
  std::vector<int32_t> cell_nint;   // interior nodes (first in the cell)
  std::vector<int32_t> cell_nb;     // boundary-patch nodes (after them)
  std::vector<int32_t> cell_boff;   // ordinal of the cell's first boundary node
  std::vector<int32_t> slot_map;    // ncell*S -> op index or -1
  int64_t n_band = 0;

  // ---- accelerator --------------------------------------------------------
  int q = 0, U = 0, F = 0, nfb = 0;
  std::vector<cd> Psh;          // [U][S]  projection of interior slots
  std::vector<cd> Pbd;          // [n_band][U] projection column per boundary node
  std::vector<cd> Psh32, Pbd32; // the same from a more strongly truncated fit,
                                // for the single-precision apply
  std::vector<cd> Ish;          // [S][F]  face values -> interior slots
  std::vector<cd> Ibd;          // [n_band][F] face values -> boundary node
  std::vector<cd> Toff;         // [9][F][U] adjacent equivalent-source fields
  std::vector<cd> Bp;           // [nf][F] Dirichlet fit: face values -> Fourier–Bessel coefficients
  int na = 0, nb = 0, Pa = 0, Pb = 0;
  std::vector<cd> kern;         // [2 sets][2 kinds][Pa*Pb] kernel / (Pa Pb)

  // ---- near field ----------------------------------------------------------
  int Wn = 0;                   // window side in lattice nodes (5 cell_h)
  std::vector<cd> Wsh;          // [S][Wn*Wn]
  std::vector<cd> Wadj, Wadj32; // [S][Wn*Wn] adjacent far-field subtraction
                                // (double / single precision projection)
  std::vector<int64_t> rowptr;  // CSR over `rows`
  std::vector<int32_t> rows, cols;
  std::vector<cd> vals;
  // Fourier refinement of the band's t1 lines (rf = 1: none).  Columns
  // N + ((s - 1) (N2 + 1) + u) N1 + v of the rows are refined values at
  // t1 = v + s / rf on line u; rf_idx / rf_dens: [N2 + 1][N1] op index
  // (-1: none) and density weight of grid node (v, u)
  int rf = 1;
  std::vector<int32_t> rf_idx;
  std::vector<double> rf_dens;
  // Fourier refinement of the interior lattice as well (rfi = rf, else 1):
  // psi grids of side M (the period); the refined grid of shift s = s2 rf +
  // s1 > 0 at columns N + rf_ioff + ((s - 1) M + gy) M + gx, lattice node
  // (gx, gy) + (c_lo - 2) cell_h; Wsh holds rfi^2 windows
  int rfi = 1, M = 0;
  int64_t rf_ioff = 0;
  // off-grid shortcut: the boundary rule's value s at grid node (v, u) of
  // the patch at column N + sc_off + u N1 + v (the refined s lines follow,
  // (rf - 1) (N2 + 1) N1 values laid out as the densities'); sr_*: those
  // rules as rows (output column in sr_rows, CSR over sr_rowptr)
  int64_t sc_off = 0;
  std::vector<int64_t> sr_rowptr;
  std::vector<int32_t> sr_rows, sr_cols;
  std::vector<cd> sr_vals;
};

// Returns LS_OK or an error code with a message in err.
ls_status build_host_op(const ls_geometry* g, ls_n2_fn n2, void* ctx, double kappa,
                        const ls_params* p, HostOp& op, std::string& err);

// Cell Dirichlet fit (Sec. 3.2, eq:-PWE read as Fourier–Bessel modes
// |n| <= nfb about the cell centre, normalised at the half diagonal):
// basis values at rel (relative to the cell origin), and the row of weights
// that maps the cell's F face values to the field at rel.
void fb_basis(int nfb, double kappa, double H, const double* rel, cd* out);
void fit_row(const std::vector<cd>& Bp, int nfb, int F, double kappa, double H, const double* rel, cd* out);

// ---- numerical helpers shared by the set-up (ls_math.cpp) ----------------
cd green2d(double kappa, double r);                    // (i/4) H0(kappa r)
cd green2d_dipole(double kappa, const double d[2], int axis);   // d/dy_axis G(|x-y|), d = x - y
void gauss_legendre01(int n, std::vector<double>& x, std::vector<double>& w);
std::vector<double> newton_cotes(int Q);               // closed rule on 0..Q-1
double smooth_step(double z);
double chi(double s, double c0);
void lagrange(double pos, int64_t base, int P, double* w);
int64_t centered_base(double pos, int P);
// Minimum-norm least-squares pseudo-inverse of a complex m x n matrix (row
// major), singular values below rcond * sigma_max dropped.  Result n x m.
std::vector<cd> pinv(const std::vector<cd>& A, int m, int n, double rcond);
int next_smooth(int n);                                 // >= n, of the form 2^a 3^b 5^c
// Householder QR with column pivoting of a complex m x n matrix (row major),
// truncated at the first |R_kk| <= rcond |R_00|; solve gives the basic
// least-squares solution of the truncated problem (backward stable).
struct QRCP {
  int m = 0, n = 0, r = 0;
  std::vector<cd> QR, v;
  std::vector<double> vn;
  std::vector<int> perm;
};
QRCP qrcp(const std::vector<cd>& A, int m, int n, double rcond);
void qrcp_solve(const QRCP& f, const cd* b, cd* x);

}  // namespace lsx
