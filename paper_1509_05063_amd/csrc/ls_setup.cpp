// Host set-up of the 2-D discrete operator: Nystrom nodes, cells, near-field
// quadratures, equivalent-source and Dirichlet-fit matrices, Green's
// function lattices.  Independent of any test code.
#include <omp.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <numeric>
#include <tuple>

#include "ls_setup.hpp"

namespace lsx {

namespace {

struct Geo {
  double a;
  int k;
  double s_in, s_a, s_b;
  int N1, N2;
  int P = 1;              // boundary patches (1: one periodic band)
  double overlap = 0;     // half-overlap of neighbouring patches (radians), P >= 2
  double R(double th) const { return 1.0 + a * std::cos(k * th); }
  // theta at t1 = 0 and the theta span of boundary patch p
  double th0(int p) const { return P == 1 ? 0.0 : 2.0 * M_PI * p / P - (M_PI / P + overlap); }
  double span() const { return P == 1 ? 2.0 * M_PI : 2.0 * (M_PI / P + overlap); }
  // angle difference wrapped to (-pi, pi]
  static double wrap(double d) {
    double m = std::fmod(M_PI - d, 2.0 * M_PI);
    if (m < 0) m += 2.0 * M_PI;
    return M_PI - m;
  }
  // tangential partition of unity of patch p at angle th: normalised bumps
  // that vanish to all orders at their patch's ends (Sec. 2, patches with a
  // partition of unity; the formula is a reading)
  double tan_pou(double th, int p) const {
    if (P == 1) return 1.0;
    const double D = M_PI / P + overlap;
    double bp = 0, sum = 0;
    for (int q = 0; q < P; ++q) {
      const double b = smooth_step((D - std::fabs(wrap(th - 2.0 * M_PI * q / P))) / (2.0 * overlap));
      sum += b;
      if (q == p) bp = b;
    }
    return sum > 0 ? bp / sum : 0.0;
  }
  // boundary-patch map xi(t1, t2) of patch p (Sec. 2: t2 = 0 is the interface)
  void map(double t1, double t2, double* x, int p = 0) const {
    double th = th0(p) + span() * t1;
    double s = 1.0 - (1.0 - s_in) * t2;
    double r = s * R(th);
    x[0] = r * std::cos(th);
    x[1] = r * std::sin(th);
  }
  double jac(double t1, double t2, int p = 0) const {
    double th = th0(p) + span() * t1;
    double s = 1.0 - (1.0 - s_in) * t2;
    double r = R(th);
    return span() * (1.0 - s_in) * s * r * r;
  }
  double omega_band(double s) const { return smooth_step((s - s_a) / (s_b - s_a)); }
  double srad(const double* x) const {
    double th = std::atan2(x[1], x[0]);
    return std::hypot(x[0], x[1]) / R(th);
  }
  // grid coordinates in patch p (v = t1 N1, u = t2 N2) of any point; u
  // within 1e-9 of a grid line is put on it.  Returns whether the point is
  // in the closed patch.
  bool coords(const double* x, double& v, double& u, int p = 0) const {
    double th = std::atan2(x[1], x[0]);
    bool vin = true;
    if (P == 1) {
      double t1 = std::fmod(th / (2.0 * M_PI), 1.0);
      if (t1 < 0) t1 += 1.0;
      v = t1 * N1;
      if (v >= N1) v -= N1;
    } else {
      const double half = 0.5 * span();
      v = (wrap(th - th0(p) - half) + half) / span() * N1;
      vin = v >= 0.0 && v <= (double)N1;
    }
    double s = std::hypot(x[0], x[1]) / R(th);
    u = (1.0 - s) / (1.0 - s_in) * N2;
    double ur = std::nearbyint(u);
    if (std::fabs(u - ur) < 1e-9) u = ur;
    return vin && u >= 0.0 && u <= (double)N2;
  }
};

int64_t floordiv(int64_t a, int64_t b) { return (a >= 0) ? a / b : -((-a + b - 1) / b); }

// ----------------------------------------------------------------------------
// 1-D pieces of the singular rules
// ----------------------------------------------------------------------------

// radial nodes on [0, r] (graded Gauss on [0, c0 r], Gauss on [c0 r, r]);
// weights include chi(rho / r)
void polar_rule(const ls_params& p, std::vector<double>& rho, std::vector<double>& w) {
  double r = p.r_int, a = p.chi_c0 * r;
  std::vector<double> s, ws, t, wt;
  gauss_legendre01(p.polar_n_in, s, ws);
  gauss_legendre01(p.polar_n_out, t, wt);
  rho.clear();
  w.clear();
  for (int i = 0; i < p.polar_n_in; ++i) {
    rho.push_back(a * std::pow(s[i], p.polar_grade));
    w.push_back(a * p.polar_grade * std::pow(s[i], p.polar_grade - 1) * ws[i]);
  }
  for (int i = 0; i < p.polar_n_out; ++i) {
    double x = a + (r - a) * t[i];
    rho.push_back(x);
    w.push_back((r - a) * wt[i] * chi(x / r, p.chi_c0));
  }
}

// t1 offsets (grid units) and weights on [-r1, r1] incl. chi
void varrho_rule(const ls_params& p, std::vector<double>& d, std::vector<double>& w) {
  double r1 = p.r1, a = p.chi_c0 * r1;
  int M = p.band_M;
  std::vector<double> s, ws, t, wt;
  gauss_legendre01(p.band_n_in, s, ws);
  gauss_legendre01(p.band_n_out, t, wt);
  std::vector<double> dd, ww;
  for (int i = 0; i < p.band_n_in; ++i) {
    dd.push_back(a * std::pow(s[i], M + 1));
    ww.push_back(a * (M + 1) * std::pow(s[i], M) * ws[i]);
  }
  for (int i = 0; i < p.band_n_out; ++i) {
    double x = a + (r1 - a) * t[i];
    dd.push_back(x);
    ww.push_back((r1 - a) * wt[i] * chi(x / r1, p.chi_c0));
  }
  d.clear();
  w.clear();
  for (size_t i = 0; i < dd.size(); ++i) {
    d.push_back(-dd[i]);
    w.push_back(ww[i]);
    d.push_back(dd[i]);
    w.push_back(ww[i]);
  }
}

// Transverse rule anchored at ux (multi-split composite Newton–Cotes,
// Sec. 3.1.2): full panels of Q-1 intervals away from ux, then single
// intervals each carrying a Q-point rule, then the remaining piece to the
// patch edge; weights include chi(|u - ux| / r2).
void multisplit(double ux, int N2, int Q, double r2, double c0, const std::vector<double>& nc,
                std::vector<double>& pos, std::vector<double>& wts) {
  std::vector<std::pair<double, double>> pw;
  auto panel = [&](double a, double b) {
    double hh = (b - a) / (Q - 1);
    for (int k = 0; k < Q; ++k) pw.emplace_back(a + k * hh, nc[k] * hh);
  };
  for (int sd = -1; sd <= 1; sd += 2) {
    double side = sd;
    double span = sd < 0 ? ux : N2 - ux;
    int Lp = (int)std::floor(span / (Q - 1));
    for (int l = 1; l <= Lp; ++l) {
      if ((double)(l - 1) * (Q - 1) >= r2) break;
      double a = ux + side * (l - 1) * (Q - 1), b = ux + side * l * (Q - 1);
      panel(std::min(a, b), std::max(a, b));
    }
    double rem = span - (double)Lp * (Q - 1);
    int I = (int)std::floor(rem);
    double base = (double)Lp * (Q - 1);
    for (int i = 1; i <= I; ++i) {
      if (base + i - 1 >= r2) break;
      double a = ux + side * (base + i - 1), b = ux + side * (base + i);
      panel(std::min(a, b), std::max(a, b));
    }
    double wrest = rem - I;
    if (wrest > 0.0 && base + I < r2) {
      double a = ux + side * (base + I), b = ux + side * span;
      panel(std::min(a, b), std::max(a, b));
    }
  }
  for (auto& e : pw) e.second *= chi(std::fabs(e.first - ux) / r2, c0);
  std::sort(pw.begin(), pw.end());
  pos.clear();
  wts.clear();
  for (auto& e : pw) {
    if (e.second == 0.0) continue;
    if (!pos.empty() && std::fabs(e.first - pos.back()) < 1e-9) {
      wts.back() += e.second;
    } else {
      pos.push_back(e.first);
      wts.push_back(e.second);
    }
  }
}

// Interior polar rule around (base + frac) h: offsets relative to base and
// weights on the lattice (density m*omega*u).
struct Stencil {
  int R = 0;                // offsets in [-R, R]
  std::vector<cd> w;        // (2R+1)^2
  cd at(int d1, int d2) const {
    if (std::abs(d1) > R || std::abs(d2) > R) return 0.0;
    return w[(d1 + R) * (2 * R + 1) + (d2 + R)];
  }
};

// rf > 1: the Lagrange stencils sit on the rf-fold refined lattice and the
// offsets are in refined units
Stencil interior_stencil(double f1, double f2, const std::vector<double>& rho,
                         const std::vector<double>& wr, const ls_params& p, double h, double kappa, int rf = 1) {
  Stencil st;
  st.R = rf * (int)std::ceil(p.r_int / h) + p.P + 2 + (rf > 1 ? rf : 0);
  int side = 2 * st.R + 1;
  st.w.assign((size_t)side * side, 0.0);
  int nth = p.polar_n_theta;
  int P = p.P;
  double L1[32], L2[32];
  for (size_t k = 0; k < rho.size(); ++k) {
    cd wk = wr[k] * rho[k] * green2d(kappa, rho[k]) * (2.0 * M_PI / nth);
    for (int b = 0; b < nth; ++b) {
      double th = 2.0 * M_PI * b / nth;
      double p1 = rf * (f1 + (rho[k] * std::cos(th)) / h);
      double p2 = rf * (f2 + (rho[k] * std::sin(th)) / h);
      int64_t b1 = centered_base(p1, P), b2 = centered_base(p2, P);
      lagrange(p1, b1, P, L1);
      lagrange(p2, b2, P, L2);
      for (int i = 0; i < P; ++i) {
        cd wi = wk * L1[i];
        int o1 = (int)(b1 + i) + st.R;
        for (int j = 0; j < P; ++j) {
          int o2 = (int)(b2 + j) + st.R;
          st.w[(size_t)o1 * side + o2] += wi * L2[j];
        }
      }
    }
  }
  return st;
}

}  // namespace

// ============================================================================
void fb_basis(int nfb, double kappa, double H, const double* rel, cd* out) {
  const double Rc = H / std::sqrt(2.0);
  const double dx = rel[0] - 0.5 * H, dy = rel[1] - 0.5 * H;
  const double rr = std::hypot(dx, dy), th = std::atan2(dy, dx);
  for (int n = -nfb; n <= nfb; ++n) {
    const int an = std::abs(n);
    double jn = std::cyl_bessel_j((double)an, kappa * rr) / std::cyl_bessel_j((double)an, kappa * Rc);
    if (n < 0 && (an & 1)) jn = -jn;
    out[n + nfb] = jn * std::exp(cd(0.0, n * th));
  }
}

void fit_row(const std::vector<cd>& Bp, int nfb, int F, double kappa, double H, const double* rel, cd* out) {
  const int nf = 2 * nfb + 1;
  std::vector<cd> e(nf);
  fb_basis(nfb, kappa, H, rel, e.data());
  for (int t = 0; t < F; ++t) {
    cd acc = 0;
    for (int n = 0; n < nf; ++n) acc += e[n] * Bp[(size_t)n * F + t];
    out[t] = acc;
  }
}

ls_status build_host_op(const ls_geometry* gp, ls_n2_fn n2fn, void* ctx, double kappa,
                        const ls_params* pp, HostOp& op, std::string& err) {
  const ls_geometry& g = *gp;
  const ls_params& p = *pp;
  op.g = g;
  op.p = p;
  op.kappa = kappa;
  if (g.dim != 2) { err = "only dim = 2 is supported"; return LS_EINVAL; }
  if (!(kappa > 0) || !(g.h > 0)) { err = "kappa and h must be positive"; return LS_EINVAL; }
  if (!(g.s_in <= g.s_a && g.s_a < g.s_b && g.s_b < 1.0 && g.s_in > 0)) {
    err = "need 0 < s_in <= s_a < s_b < 1"; return LS_EINVAL;
  }
  if (p.Q < 2 || g.N2 % (p.Q - 1) != 0) { err = "N2 must be a multiple of Q-1"; return LS_EINVAL; }
  if (p.P < 4 || p.P % 2 || p.P > 16 || g.N2 + 1 < p.P || g.N1 < 2 * p.P) {
    err = "P must be even in [4,16] and fit the boundary grid"; return LS_EINVAL;
  }
  if (p.cell_h < 2 || p.q < 2 || p.n_fb < 1 || p.coll_factor < 1) { err = "bad accelerator sizes"; return LS_EINVAL; }
  const double h = g.h;
  const int ch = p.cell_h;
  const double H = ch * h;
  if (kappa * H >= M_PI * std::sqrt(2.0)) { err = "cells resonate: kappa H >= pi sqrt(2)"; return LS_EINVAL; }
  if (p.r_int + (p.P / 2) * h > 2 * H * (1 + 1e-12)) { err = "interior cut-off reaches beyond two cells"; return LS_EINVAL; }
  if (4 * p.q < 2 * p.n_fb + 1) { err = "need 4q >= 2 n_fb + 1 face values"; return LS_EINVAL; }
  if (p.r1 <= 0 || p.r2 <= 0 || p.r_int <= 0 || p.r1 > g.N1 / 2 - p.P) { err = "bad cut-off radii"; return LS_EINVAL; }

  const int NP = g.n_patches < 1 ? 1 : g.n_patches;
  if (NP > 1 && !(g.overlap > 0.0 && g.overlap < M_PI / NP)) {
    err = "several boundary patches need 0 < overlap < pi / n_patches"; return LS_EINVAL;
  }
  if (NP > 64) { err = "at most 64 boundary patches"; return LS_EINVAL; }
  // Fourier refinement of the band's t1 lines (Sec. 3.1): line transforms of
  // N1 points with radices 2, 3, 5 in one workgroup's LDS
  const int rf = p.fft_refine > 1 ? p.fft_refine : 1;
  if (rf > 1) {
    int rest = g.N1;
    for (int f : {2, 3, 5})
      while (rest % f == 0) rest /= f;
    if (NP > 1) { err = "fft_refine needs the single periodic band"; return LS_EINVAL; }
    if (rf > 8 || g.N1 > 4096 || rest != 1) {
      err = "fft_refine: r <= 8, N1 <= 4096 with prime factors 2, 3, 5"; return LS_EINVAL;
    }
  }
  op.rf = rf;
  if (p.offgrid_shortcut && NP > 1) { err = "offgrid_shortcut needs the single periodic band"; return LS_EINVAL; }
  if (p.fft_refine_interior) {
    if (rf < 2) { err = "fft_refine_interior needs fft_refine >= 2"; return LS_EINVAL; }
    if (p.cell_h != 8) { err = "fft_refine_interior needs cell_h = 8"; return LS_EINVAL; }
  }
  Geo G{g.shape_a, g.shape_k, g.s_in, g.s_a, g.s_b, g.N1, g.N2, NP, NP > 1 ? g.overlap : 0.0};
  const int N1 = g.N1, N2 = g.N2;
  const bool periodic = NP == 1;
  const int n1g = periodic ? N1 : N1 + 1;      // t1 grid nodes per patch

  // ---------------------------------------------------------------- nodes
  struct Node { int chart; int64_t i1, i2; double x, y, w, om, J; };
  std::vector<Node> nodes;
  const int64_t imax = (int64_t)std::ceil(g.s_b * (1.0 + std::fabs(g.shape_a)) / h) + 1;
  for (int64_t i1 = -imax; i1 <= imax; ++i1)
    for (int64_t i2 = -imax; i2 <= imax; ++i2) {
      double x[2] = {i1 * h, i2 * h};
      double om = 1.0 - G.omega_band(G.srad(x));
      if (om > 0.0) nodes.push_back({0, i1, i2, x[0], x[1], h * h, om, 1.0});
    }
  const int64_t n_int = (int64_t)nodes.size();
  std::vector<double> nc = newton_cotes(p.Q);
  std::vector<double> ncw(N2 + 1, 0.0);
  for (int pnl = 0; pnl < N2 / (p.Q - 1); ++pnl)
    for (int k = 0; k < p.Q; ++k) ncw[pnl * (p.Q - 1) + k] += nc[k];
  // boundary patches: trapezoid in t1 (non-periodic patches: the end nodes
  // carry a zero partition of unity and are not unknowns) x composite
  // Newton–Cotes in t2; the node's partition of unity is the transverse one
  // times the tangential one
  for (int pp = 0; pp < NP; ++pp)
    for (int j1 = 0; j1 < n1g; ++j1) {
      const double t1 = (double)j1 / N1;
      const double omt = G.tan_pou(G.th0(pp) + G.span() * t1, pp);
      if (!(omt > 0.0)) continue;
      for (int j2 = 0; j2 <= N2; ++j2) {
        double t2 = (double)j2 / N2;
        double x[2];
        G.map(t1, t2, x, pp);
        double s = 1.0 - (1.0 - g.s_in) * t2;
        double J = G.jac(t1, t2, pp);
        nodes.push_back({1 + pp, j1, j2, x[0], x[1], ncw[j2] * J / ((double)N1 * N2), G.omega_band(s) * omt, J});
      }
    }
  const int64_t N = (int64_t)nodes.size();
  op.N = N;
  op.n_band = N - n_int;

  // refractive index through the callback (interior limit on the interface)
  std::vector<double> xy0(2 * N), n2v(N);
  std::vector<int32_t> onb(N);
  for (int64_t i = 0; i < N; ++i) {
    xy0[2 * i] = nodes[i].x;
    xy0[2 * i + 1] = nodes[i].y;
    onb[i] = (nodes[i].chart >= 1 && nodes[i].i2 == 0) ? 1 : 0;
  }
  n2fn(N, xy0.data(), onb.data(), n2v.data(), ctx);

  // ---------------------------------------------------------------- cells
  auto cell_of = [&](const Node& nd, int64_t& cx, int64_t& cy) {
    if (nd.chart == 0) { cx = floordiv(nd.i1, ch); cy = floordiv(nd.i2, ch); }
    else { cx = (int64_t)std::floor(nd.x / H); cy = (int64_t)std::floor(nd.y / H); }
  };
  int64_t lo = INT64_MAX, hi = INT64_MIN;
  std::vector<int64_t> ncx(N), ncy(N);
  for (int64_t i = 0; i < N; ++i) {
    cell_of(nodes[i], ncx[i], ncy[i]);
    lo = std::min({lo, ncx[i], ncy[i]});
    hi = std::max({hi, ncx[i], ncy[i]});
  }
  const int L = (int)(hi - lo + 1);
  op.H = H;
  op.S = ch * ch;
  op.L = L;
  op.c_lo = lo;
  if (p.fft_refine_interior) {
    // period of the interior refinement: the lattice box of the cells plus
    // two cells on each side, rounded up to prime factors 2, 3, 5
    int M = (L + 4) * ch;
    for (;; ++M) {
      int rest = M;
      for (int f : {2, 3, 5})
        while (rest % f == 0) rest /= f;
      if (rest == 1) break;
    }
    if (M > 4096) { err = "fft_refine_interior: lattice period above 4096"; return LS_EINVAL; }
    op.rfi = rf;
    op.M = M;
  }
  std::vector<int64_t> lin(N);
  for (int64_t i = 0; i < N; ++i) lin[i] = (ncy[i] - lo) * L + (ncx[i] - lo);
  std::vector<int64_t> order(N);
  std::iota(order.begin(), order.end(), 0);
  auto slot_of = [&](const Node& nd) -> int64_t {
    int64_t sx = nd.i1 - ch * floordiv(nd.i1, ch), sy = nd.i2 - ch * floordiv(nd.i2, ch);
    return sy * ch + sx;
  };
  std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
    if (lin[a] != lin[b]) return lin[a] < lin[b];
    const Node &A = nodes[a], &B = nodes[b];
    if (A.chart != B.chart) return A.chart < B.chart;
    if (A.chart == 0) return slot_of(A) < slot_of(B);
    return std::make_pair(A.i1, A.i2) < std::make_pair(B.i1, B.i2);
  });
  std::vector<int64_t> opos(N);   // original index -> op index
  for (int64_t k = 0; k < N; ++k) opos[order[k]] = k;

  op.xy.resize(2 * N);
  op.key.resize(3 * N);
  op.cw.resize(N);
  op.dw.resize(N);
  std::vector<double> dens(N), mv(N);      // density weight of the singular rules
  for (int64_t k = 0; k < N; ++k) {
    const Node& nd = nodes[order[k]];
    double m = 1.0 - n2v[order[k]];
    mv[k] = m;
    op.xy[2 * k] = nd.x;
    op.xy[2 * k + 1] = nd.y;
    op.key[3 * k] = nd.chart;
    op.key[3 * k + 1] = (int32_t)nd.i1;
    op.key[3 * k + 2] = (int32_t)nd.i2;
    op.cw[k] = nd.w * nd.om * m;
    dens[k] = (nd.chart == 0) ? m * nd.om : m * nd.om * nd.J;
    op.dw[k] = (nd.chart == 0) ? m * nd.om : 0.0;
  }
  op.cell_map.assign((size_t)L * L, -1);
  op.cell_xy.clear();
  op.cell_start.clear();
  op.cell_nint.clear();
  op.cell_nb.clear();
  op.cell_boff.clear();
  std::vector<int32_t> cell_of_op(N);
  int32_t band_ord = 0;
  for (int64_t k = 0; k < N;) {
    int64_t l0 = lin[order[k]];
    int64_t e = k;
    int32_t ni = 0, nbd = 0;
    while (e < N && lin[order[e]] == l0) {
      if (nodes[order[e]].chart == 0) ++ni; else ++nbd;
      ++e;
    }
    int32_t ci = (int32_t)op.cell_xy.size() / 2;
    op.cell_map[l0] = ci;
    op.cell_xy.push_back((int32_t)(l0 % L));
    op.cell_xy.push_back((int32_t)(l0 / L));
    op.cell_start.push_back((int32_t)k);
    op.cell_nint.push_back(ni);
    op.cell_nb.push_back(nbd);
    op.cell_boff.push_back(band_ord);
    band_ord += nbd;
    for (int64_t t = k; t < e; ++t) cell_of_op[t] = ci;
    k = e;
  }
  const int ncell = (int)op.cell_start.size();
  op.ncell = ncell;
  const int S = op.S;
  op.slot_map.assign((size_t)ncell * S, -1);
  for (int c = 0; c < ncell; ++c)
    for (int t = 0; t < op.cell_nint[c]; ++t) {
      int64_t k = op.cell_start[c] + t;
      op.slot_map[(size_t)c * S + slot_of(nodes[order[k]])] = (int32_t)k;
    }
  auto cell_at = [&](int64_t cx, int64_t cy) -> int {
    if (cx < 0 || cy < 0 || cx >= L || cy >= L) return -1;
    return op.cell_map[cy * L + cx];
  };

  // lattice (i1, i2) -> op index; boundary grid (j1, j2) -> op index
  const int64_t lside = 2 * imax + 1;
  std::vector<int32_t> lat(lside * lside, -1);
  // boundary grids: patch p, (j1, j2) -> op index (-1: not an unknown)
  std::vector<int32_t> bgrid((size_t)NP * n1g * (N2 + 1), -1);
  auto bg = [&](int pp, int64_t j1, int64_t j2) -> int32_t& {
    return bgrid[((size_t)pp * n1g + j1) * (N2 + 1) + j2];
  };
  for (int64_t k = 0; k < N; ++k) {
    int32_t c = op.key[3 * k], i1 = op.key[3 * k + 1], i2 = op.key[3 * k + 2];
    if (c == 0) lat[(i1 + imax) * lside + (i2 + imax)] = (int32_t)k;
    else bg(c - 1, i1, i2) = (int32_t)k;
  }
  auto lat_at = [&](int64_t i1, int64_t i2) -> int32_t {
    if (i1 < -imax || i1 > imax || i2 < -imax || i2 > imax) return -1;
    return lat[(i1 + imax) * lside + (i2 + imax)];
  };
  // refined band values past the N unknowns, then the refined psi grids
  op.rf_ioff = rf > 1 ? (int64_t)(rf - 1) * (N2 + 1) * N1 : 0;
  if (rf > 1) {
    // the band's t2 lines for the refinement: op index and density weight
    // of grid node (v, u) at [u][v]
    op.rf_idx.assign((size_t)(N2 + 1) * N1, -1);
    op.rf_dens.assign((size_t)(N2 + 1) * N1, 0.0);
    for (int64_t u = 0; u <= N2; ++u)
      for (int64_t v = 0; v < N1; ++v) {
        const int32_t j = bg(0, v, u);
        op.rf_idx[(size_t)u * N1 + v] = j;
        if (j >= 0) op.rf_dens[(size_t)u * N1 + v] = dens[j];
      }
  }

  // ------------------------------------------------------ singular rules
  std::vector<double> prho, pw;
  polar_rule(p, prho, pw);
  std::vector<double> d1, w1;
  varrho_rule(p, d1, w1);
  const int rfi = op.rfi;
  Stencil Ton = interior_stencil(0.0, 0.0, prho, pw, p, h, kappa, rfi);

  // boundary singular row at (vt, ut) for target point xt -> (op index, coeff)
  // On a non-periodic patch the t1 rule's nodes beyond the patch ends are
  // dropped (the partition of unity makes the density vanish there) and the
  // t1 stencils are shifted one-sided at the ends.  With Fourier refinement
  // (rf > 1, periodic band) the t1 stencils sit on the rf-fold refined grid:
  // refined node rf v0 + s is grid node v0 for s = 0 (an unknown, weight
  // times its density factor) and otherwise refined column
  // N + ((s - 1) (N2 + 1) + u) N1 + v0, whose value the apply computes from
  // the line's density by FFT.
  auto band_sing = [&](const double* xt, double vt, double ut, int pp, std::vector<std::pair<int32_t, cd>>& out) {
    std::vector<double> lines, w2;
    multisplit(ut, N2, p.Q, p.r2, p.chi_c0, nc, lines, w2);
    if (lines.empty()) return;
    const int P = p.P;
    const int nk = (int)d1.size();
    int64_t vlo = centered_base(rf * (vt - p.r1), P) - 1, vhi = centered_base(rf * (vt + p.r1), P) + P + 1;
    if (!periodic) {
      vlo = std::max<int64_t>(vlo, 0);
      vhi = std::min<int64_t>(vhi, N1);
    }
    int nvw = (int)(vhi - vlo + 1);
    int64_t ulo = 0, uhi = N2;
    int nuw = (int)(uhi - ulo + 1);
    std::vector<cd> win((size_t)nvw * nuw, 0.0), Rv(nvw);
    std::vector<double> Lv((size_t)nk * P);
    std::vector<int64_t> bv(nk);
    std::vector<char> use(nk, 1);
    for (int k = 0; k < nk; ++k) {
      double V = vt + d1[k];
      if (!periodic && (V < 0.0 || V > (double)N1)) {
        use[k] = 0;
        continue;
      }
      bv[k] = centered_base(rf * V, P);
      if (!periodic) bv[k] = std::min<int64_t>(std::max<int64_t>(bv[k], 0), N1 - P + 1);
      lagrange(rf * V, bv[k], P, &Lv[(size_t)k * P]);
    }
    double Lu[32];
    for (size_t l = 0; l < lines.size(); ++l) {
      std::fill(Rv.begin(), Rv.end(), cd(0.0));
      double T2 = lines[l] / N2;
      for (int k = 0; k < nk; ++k) {
        if (!use[k]) continue;
        double V = vt + d1[k];
        double y[2];
        G.map(V / N1, T2, y, pp);
        double r = std::hypot(y[0] - xt[0], y[1] - xt[1]);
        if (!(r > 0.0)) continue;
        cd W = (w2[l] / N2) * (w1[k] / N1) * green2d(kappa, r);
        for (int a = 0; a < P; ++a) Rv[bv[k] + a - vlo] += W * Lv[(size_t)k * P + a];
      }
      int64_t bu = std::min<int64_t>(std::max<int64_t>(centered_base(lines[l], P), 0), N2 - P + 1);
      lagrange(lines[l], bu, P, Lu);
      for (int b = 0; b < P; ++b) {
        cd* rowp = &win[(size_t)(bu + b - ulo) * nvw];
        for (int v = 0; v < nvw; ++v) rowp[v] += Lu[b] * Rv[v];
      }
    }
    for (int u = 0; u < nuw; ++u)
      for (int v = 0; v < nvw; ++v) {
        cd c = win[(size_t)u * nvw + v];
        if (c == 0.0) continue;
        if (rf > 1) {
          const int64_t nr = (int64_t)rf * N1, vr = ((vlo + v) % nr + nr) % nr, v0 = vr / rf, s = vr % rf;
          if (s > 0) {
            out.emplace_back((int32_t)(N + ((s - 1) * (N2 + 1) + ulo + u) * N1 + v0), c);
            continue;
          }
          const int32_t j = bg(pp, v0, ulo + u);
          if (j >= 0) out.emplace_back(j, c * dens[j]);
          continue;
        }
        int64_t vv = periodic ? ((vlo + v) % N1 + N1) % N1 : vlo + v;
        int32_t j = bg(pp, vv, ulo + u);
        if (j >= 0) out.emplace_back(j, c * dens[j]);
      }
  };

  // -------------------------------------------------- shared near window
  // With interior refinement one window per refined shift s = s2 rf + s1
  // (the values at lattice node + (s1, s2) / rf); the plain terms sit in
  // the window of s = 0.
  const int Wn = 5 * ch;
  op.Wn = Wn;
  op.Wsh.assign((size_t)rfi * rfi * S * Wn * Wn, 0.0);
#pragma omp parallel for schedule(dynamic)
  for (int a = 0; a < S; ++a) {
    int ax = a % ch, ay = a / ch;
    for (int wy = 0; wy < Wn; ++wy)
      for (int wx = 0; wx < Wn; ++wx) {
        int dx = wx - 2 * ch - ax, dy = wy - 2 * ch - ay;
        int ocx = wx / ch - 2, ocy = wy / ch - 2;
        bool adj = std::abs(ocx) <= 1 && std::abs(ocy) <= 1;
        cd val = Ton.at(rfi * dx, rfi * dy);
        if (dx != 0 || dy != 0) {
          double d = std::hypot((double)dx * h, (double)dy * h);
          double eta = chi(d / p.r_int, p.chi_c0);
          double f = adj ? 1.0 - eta : -eta;
          if (f != 0.0) val += h * h * f * green2d(kappa, d);
        }
        op.Wsh[(size_t)a * Wn * Wn + (size_t)wy * Wn + wx] = val;
        for (int s = 1; s < rfi * rfi; ++s)
          op.Wsh[((size_t)s * S + a) * Wn * Wn + (size_t)wy * Wn + wx] =
              Ton.at(rfi * dx + s % rfi, rfi * dy + s / rfi);
      }
  }

  // ------------------------------------------------------ CSR rows
  // Rows: every boundary-patch target (all sources) and every interior
  // target with boundary-patch sources (adjacent, cut-off or singular rule).
  // every point's grid coordinates in every boundary patch (inp: whether it
  // lies in that patch); t2 (tu) is the same in all patches
  std::vector<char> inp((size_t)NP * N, 0);
  std::vector<double> tvp((size_t)NP * N), tu(N);
  for (int64_t k = 0; k < N; ++k) {
    const int ck = op.key[3 * k];
    for (int pp = 0; pp < NP; ++pp) {
      double v, u;
      bool in = G.coords(&op.xy[2 * k], v, u, pp);
      if (ck == 1 + pp) {     // a node of this patch: exact grid coordinates
        in = true;
        v = op.key[3 * k + 1];
        u = op.key[3 * k + 2];
      }
      inp[(size_t)pp * N + k] = in ? 1 : 0;
      tvp[(size_t)pp * N + k] = v;
      tu[k] = u;
    }
  }
  auto eta_band = [&](double vt, double ut, double vs, double us) {
    double dv = std::fabs(vs - vt);
    if (periodic) dv = std::min(dv, N1 - dv);
    return chi(dv / p.r1, p.chi_c0) * chi(std::fabs(us - ut) / p.r2, p.chi_c0);
  };
  // off-grid shortcut: boundary rule values s at the patch's grid nodes in
  // x at N + sc_off + u N1 + v (then the refined s lines, as the densities')
  const bool sc = p.offgrid_shortcut != 0;
  op.sc_off = op.rf_ioff + (int64_t)(op.rfi * op.rfi - 1) * op.M * op.M;
  std::vector<std::vector<std::pair<int32_t, cd>>> rowdata(N);
  std::vector<char> has_row(N, 0);
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < N; ++i) {
    const bool tb = op.key[3 * i] >= 1;
    const double* xi = &op.xy[2 * i];
    const int ci = cell_of_op[i];
    const int cx = op.cell_xy[2 * ci], cy = op.cell_xy[2 * ci + 1];
    std::vector<std::pair<int32_t, cd>> ent;
    auto adjacent = [&](int32_t j) {
      int cj = cell_of_op[j];
      return std::abs(op.cell_xy[2 * cj] - cx) <= 1 && std::abs(op.cell_xy[2 * cj + 1] - cy) <= 1;
    };
    // plain adjacent pairs
    for (int oy = -1; oy <= 1; ++oy)
      for (int ox = -1; ox <= 1; ++ox) {
        int c = cell_at(cx + ox, cy + oy);
        if (c < 0) continue;
        int64_t j0 = op.cell_start[c], j1e = j0 + op.cell_nint[c] + op.cell_nb[c];
        int64_t jb = tb ? j0 : j0 + op.cell_nint[c];      // interior targets: boundary sources only
        for (int64_t j = jb; j < j1e; ++j) {
          // every adjacent source gets an entry (zero where the plain rule
          // gives none): the adjacent equivalent-source fields are folded
          // into these rows after the projections are known
          if (j == i) {
            ent.emplace_back((int32_t)j, cd(0.0, 0.0));
            continue;
          }
          double eta;
          const int cj = op.key[3 * j];
          if (cj == 0) {
            double d = std::hypot(op.xy[2 * j] - xi[0], op.xy[2 * j + 1] - xi[1]);
            eta = chi(d / p.r_int, p.chi_c0);
          } else {
            // the localisation of the source's own patch, centred at the
            // target's coordinates in that patch (0 if the target is not in it)
            const size_t o = (size_t)(cj - 1) * N;
            eta = inp[o + i] ? eta_band(tvp[o + i], tu[i], tvp[o + j], tu[j]) : 0.0;
          }
          double f = 1.0 - eta;
          if (f == 0.0) {
            ent.emplace_back((int32_t)j, cd(0.0, 0.0));
            continue;
          }
          double d = std::hypot(op.xy[2 * j] - xi[0], op.xy[2 * j + 1] - xi[1]);
          ent.emplace_back((int32_t)j, f * green2d(kappa, d) * op.cw[j]);
        }
      }
    // cut-off tails on non-adjacent sources: -eta G c
    if (tb) {
      int64_t r = (int64_t)std::ceil(p.r_int / h) + 1;
      int64_t g1 = (int64_t)std::floor(xi[0] / h), g2 = (int64_t)std::floor(xi[1] / h);
      for (int64_t a1 = g1 - r; a1 <= g1 + r + 1; ++a1)
        for (int64_t a2 = g2 - r; a2 <= g2 + r + 1; ++a2) {
          int32_t j = lat_at(a1, a2);
          if (j < 0 || adjacent(j)) continue;
          double d = std::hypot(op.xy[2 * j] - xi[0], op.xy[2 * j + 1] - xi[1]);
          double eta = chi(d / p.r_int, p.chi_c0);
          if (eta != 0.0) ent.emplace_back(j, -eta * green2d(kappa, d) * op.cw[j]);
        }
    }
    for (int pp = 0; pp < NP; ++pp) {
      const size_t o = (size_t)pp * N;
      if (!inp[o + i]) continue;
      const double tvi = tvp[o + i];
      int64_t v0 = (int64_t)std::floor(tvi - p.r1) - 1, v1 = (int64_t)std::ceil(tvi + p.r1) + 1;
      if (!periodic) {
        v0 = std::max<int64_t>(v0, 0);
        v1 = std::min<int64_t>(v1, N1);
      }
      int64_t u0 = std::max<int64_t>(0, (int64_t)std::floor(tu[i] - p.r2) - 1);
      int64_t u1 = std::min<int64_t>(N2, (int64_t)std::ceil(tu[i] + p.r2) + 1);
      for (int64_t v = v0; v <= v1; ++v)
        for (int64_t u = u0; u <= u1; ++u) {
          int64_t vv = periodic ? ((v % N1) + N1) % N1 : v;
          int32_t j = bg(pp, vv, u);
          if (j < 0 || j == i || adjacent(j)) continue;
          double eta = eta_band(tvi, tu[i], tvp[o + j], tu[j]);
          if (eta == 0.0) continue;
          double d = std::hypot(op.xy[2 * j] - xi[0], op.xy[2 * j + 1] - xi[1]);
          ent.emplace_back(j, -eta * green2d(kappa, d) * op.cw[j]);
        }
      if (sc) {
        // off-grid shortcut: a grid node of the patch reads its own boundary
        // rule value s from x; an interior lattice node inside the patch
        // interpolates the node values (t2 Lagrange, t1 Lagrange on the
        // refined lines)
        if (tb) {
          ent.emplace_back((int32_t)(N + op.sc_off + (int64_t)op.key[3 * i + 2] * N1 + op.key[3 * i + 1]), cd(1.0, 0.0));
        } else {
          const int P = p.P;
          double Lu[32], Lv[32];
          const int64_t bu = std::min<int64_t>(std::max<int64_t>(centered_base(tu[i], P), 0), N2 - P + 1);
          lagrange(tu[i], bu, P, Lu);
          const int64_t bv = centered_base(rf * tvi, P);
          lagrange(rf * tvi, bv, P, Lv);
          const int64_t nr = (int64_t)rf * N1;
          for (int a = 0; a < P; ++a)
            for (int c = 0; c < P; ++c) {
              const int64_t vr = ((bv + c) % nr + nr) % nr, v0 = vr / rf, s = vr % rf, u = bu + a;
              const int64_t col = s == 0 ? N + op.sc_off + u * N1 + v0
                                         : N + op.sc_off + (int64_t)(N2 + 1) * N1 + ((s - 1) * (N2 + 1) + u) * N1 + v0;
              ent.emplace_back((int32_t)col, cd(Lu[a] * Lv[c], 0.0));
            }
        }
        continue;
      }
      band_sing(xi, tvi, tu[i], pp, ent);
    }
    if (tb) {
      // interior polar rule centred off the lattice
      double g1 = xi[0] / h, g2 = xi[1] / h;
      int64_t b1 = (int64_t)std::floor(g1), b2 = (int64_t)std::floor(g2);
      Stencil st = interior_stencil(g1 - b1, g2 - b2, prho, pw, p, h, kappa, rfi);
      int side = 2 * st.R + 1;
      for (int o1 = 0; o1 < side; ++o1)
        for (int o2 = 0; o2 < side; ++o2) {
          cd c = st.w[(size_t)o1 * side + o2];
          if (c == 0.0) continue;
          if (rfi > 1) {
            // refined offset -> lattice node and shift; a shifted value is
            // read from the refined psi grid of its shift
            const int64_t r1 = o1 - st.R, r2 = o2 - st.R;
            const int64_t d1 = floordiv(r1, rfi), d2 = floordiv(r2, rfi);
            const int64_t s = (r2 - rfi * d2) * rfi + (r1 - rfi * d1);
            if (s > 0) {
              const int64_t gx = b1 + d1 - (op.c_lo - 2) * ch, gy = b2 + d2 - (op.c_lo - 2) * ch;
              if (gx < 0 || gy < 0 || gx >= op.M || gy >= op.M) continue;   // outside the box: zero density
              ent.emplace_back((int32_t)(N + op.rf_ioff + ((s - 1) * op.M + gy) * op.M + gx), c);
              continue;
            }
            const int32_t j = lat_at(b1 + d1, b2 + d2);
            if (j >= 0) ent.emplace_back(j, c * dens[j]);
            continue;
          }
          int32_t j = lat_at(b1 + o1 - st.R, b2 + o2 - st.R);
          if (j >= 0) ent.emplace_back(j, c * dens[j]);
        }
    }
    if (ent.empty()) continue;
    std::sort(ent.begin(), ent.end(), [](const std::pair<int32_t, cd>& a, const std::pair<int32_t, cd>& b) {
      return a.first < b.first;
    });
    std::vector<std::pair<int32_t, cd>> merged;
    merged.reserve(ent.size());
    for (auto& e : ent) {
      if (!merged.empty() && merged.back().first == e.first) merged.back().second += e.second;
      else merged.push_back(e);
    }
    rowdata[i].swap(merged);
    has_row[i] = 1;
  }
  op.rowptr.assign(1, 0);
  op.rows.clear();
  int64_t nnz = 0;
  for (int64_t i = 0; i < N; ++i)
    if (has_row[i]) { op.rows.push_back((int32_t)i); nnz += rowdata[i].size(); op.rowptr.push_back(nnz); }
  op.cols.resize(nnz);
  op.vals.resize(nnz);
  {
    int64_t r = 0;
    for (int64_t i = 0; i < N; ++i) {
      if (!has_row[i]) continue;
      int64_t o = op.rowptr[r];
      for (auto& e : rowdata[i]) { op.cols[o] = e.first; op.vals[o] = e.second; ++o; }
      std::vector<std::pair<int32_t, cd>>().swap(rowdata[i]);
      ++r;
    }
  }
  if (sc) {
    // the boundary rule at every grid node of the patch, as rows whose
    // output is the node's s entry in x
    const int64_t nl = (int64_t)(N2 + 1) * N1;
    std::vector<std::vector<std::pair<int32_t, cd>>> srow(nl);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t g = 0; g < nl; ++g) {
      const int64_t u = g / N1, v = g % N1;
      const int32_t j = bg(0, v, u);
      if (j < 0) continue;
      std::vector<std::pair<int32_t, cd>> ent;
      band_sing(&op.xy[2 * j], (double)v, (double)u, 0, ent);
      std::sort(ent.begin(), ent.end(), [](const std::pair<int32_t, cd>& a, const std::pair<int32_t, cd>& b) {
        return a.first < b.first;
      });
      for (auto& e : ent) {
        if (!srow[g].empty() && srow[g].back().first == e.first) srow[g].back().second += e.second;
        else srow[g].push_back(e);
      }
    }
    op.sr_rowptr.assign(1, 0);
    op.sr_rows.clear();
    op.sr_cols.clear();
    op.sr_vals.clear();
    for (int64_t g = 0; g < nl; ++g) {
      if (srow[g].empty()) continue;
      op.sr_rows.push_back((int32_t)(N + op.sc_off + g));
      for (auto& e : srow[g]) {
        op.sr_cols.push_back(e.first);
        op.sr_vals.push_back(e.second);
      }
      op.sr_rowptr.push_back((int64_t)op.sr_cols.size());
    }
  }

  // ------------------------------------------------ equivalent sources
  const int q = p.q;
  op.q = q;
  op.U = 8 * q;
  op.F = 4 * q;
  op.nfb = p.n_fb;
  const int U = op.U, F = op.F, U1 = 4 * q;
  auto node_pos = [&](int s, int f, int j, double* x) {   // set s, face f, index j
    x[s] = f * H;
    x[1 - s] = (j + 0.5) * H / q;
  };
  const int ncol = p.coll_factor * U1;
  std::vector<double> coll(2 * ncol);
  for (int k = 0; k < ncol; ++k) {
    double t = (k + 0.5) * 12.0 * H / ncol;
    int side = std::min(3, (int)std::floor(t / (3 * H)));
    double u = t - side * 3 * H;
    double* c = &coll[2 * k];
    if (side == 0) { c[0] = -H + u; c[1] = -H; }
    else if (side == 1) { c[0] = 2 * H; c[1] = -H + u; }
    else if (side == 2) { c[0] = 2 * H - u; c[1] = 2 * H; }
    else { c[0] = -H; c[1] = 2 * H - u; }
  }
  // least squares per set: QR with column pivoting, numerical rank at
  // 1e-14 (double-precision apply) and 1e-8 (single precision: smaller
  // strengths, so rounding in the projection is not amplified)
  QRCP fac[2][2];
  for (int s = 0; s < 2; ++s) {
    std::vector<cd> A((size_t)ncol * U1);
    for (int k = 0; k < ncol; ++k)
      for (int f = 0; f < 2; ++f)
        for (int j = 0; j < q; ++j) {
          double x[2];
          node_pos(s, f, j, x);
          double d[2] = {coll[2 * k] - x[0], coll[2 * k + 1] - x[1]};
          int col = f * q + j;
          A[(size_t)k * U1 + col] = green2d(kappa, std::hypot(d[0], d[1]));
          A[(size_t)k * U1 + 2 * q + col] = green2d_dipole(kappa, d, s);
        }
    fac[0][s] = qrcp(A, ncol, U1, 1e-14);
    fac[1][s] = qrcp(A, ncol, U1, 1e-8);
  }
  // projection of a source at rel (relative to the cell origin) -> U values
  auto project_col = [&](const double* rel, cd* out, int which) {
    std::vector<cd> gcol(ncol);
    for (int k = 0; k < ncol; ++k)
      gcol[k] = green2d(kappa, std::hypot(coll[2 * k] - rel[0], coll[2 * k + 1] - rel[1]));
    for (int s = 0; s < 2; ++s) qrcp_solve(fac[which][s], gcol.data(), out + s * U1);
  };
  // Dirichlet fit: Fourier–Bessel modes |n| <= n_fb about the cell centre
  const int nf = 2 * p.n_fb + 1;
  std::vector<cd> B((size_t)F * nf);
  for (int s = 0; s < 2; ++s)
    for (int f = 0; f < 2; ++f)
      for (int j = 0; j < q; ++j) {
        double x[2];
        node_pos(s, f, j, x);
        fb_basis(p.n_fb, kappa, H, x, &B[(size_t)(s * 2 * q + f * q + j) * nf]);
      }
  op.Bp = pinv(B, F, nf, 1e-14);   // nf x F
  auto interp_row = [&](const double* rel, cd* out) { fit_row(op.Bp, p.n_fb, F, kappa, H, rel, out); };
  op.Psh.assign((size_t)U * S, 0.0);
  op.Psh32.assign((size_t)U * S, 0.0);
  op.Ish.assign((size_t)S * F, 0.0);
  for (int a = 0; a < S; ++a) {
    double rel[2] = {(a % ch) * h, (a / ch) * h};
    std::vector<cd> col(U), col32(U);
    project_col(rel, col.data(), 0);
    project_col(rel, col32.data(), 1);
    for (int t = 0; t < U; ++t) {
      op.Psh[(size_t)t * S + a] = col[t];
      op.Psh32[(size_t)t * S + a] = col32[t];
    }
    interp_row(rel, &op.Ish[(size_t)a * F]);
  }
  op.Pbd.assign((size_t)op.n_band * U, 0.0);
  op.Pbd32.assign((size_t)op.n_band * U, 0.0);
  op.Ibd.assign((size_t)op.n_band * F, 0.0);
#pragma omp parallel for schedule(dynamic, 4)
  for (int c = 0; c < ncell; ++c) {
    double ox = (op.cell_xy[2 * c] + lo) * H, oy = (op.cell_xy[2 * c + 1] + lo) * H;
    for (int t = 0; t < op.cell_nb[c]; ++t) {
      int64_t k = op.cell_start[c] + op.cell_nint[c] + t;
      double rel[2] = {op.xy[2 * k] - ox, op.xy[2 * k + 1] - oy};
      int64_t b = op.cell_boff[c] + t;
      project_col(rel, &op.Pbd[(size_t)b * U], 0);
      project_col(rel, &op.Pbd32[(size_t)b * U], 1);
      interp_row(rel, &op.Ibd[(size_t)b * F]);
    }
  }
  // adjacent equivalent-source fields: target face node (s,f,j) of cell 0,
  // source unknowns of the same set in cell `off`
  op.Toff.assign((size_t)9 * F * U, 0.0);
  for (int oy = -1; oy <= 1; ++oy)
    for (int ox = -1; ox <= 1; ++ox) {
      int o = (oy + 1) * 3 + (ox + 1);
      for (int s = 0; s < 2; ++s)
        for (int f = 0; f < 2; ++f)
          for (int j = 0; j < q; ++j) {
            double xt[2];
            node_pos(s, f, j, xt);
            int row = s * 2 * q + f * q + j;
            for (int f2 = 0; f2 < 2; ++f2)
              for (int j2 = 0; j2 < q; ++j2) {
                double xs[2];
                node_pos(s, f2, j2, xs);
                xs[0] += ox * H;
                xs[1] += oy * H;
                double d[2] = {xt[0] - xs[0], xt[1] - xs[1]};
                if (std::hypot(d[0], d[1]) < 1e-9 * H) continue;   // K(0) = 0
                int col = f2 * q + j2;
                cd* T = &op.Toff[((size_t)o * F + row) * U];
                T[s * U1 + col] = green2d(kappa, std::hypot(d[0], d[1]));
                T[s * U1 + 2 * q + col] = green2d_dipole(kappa, d, s);
              }
          }
    }
  // The far field at a cell's targets leaves out its 3 x 3 adjacent cells'
  // equivalent sources: -I T_off P applied to those cells' weighted
  // densities c u.  For interior slot sources seen from interior slot
  // targets this is the same for every cell, a window term like Wsh (in
  // terms of psi = m omega u: c = h^2 psi there), once per precision with
  // that precision's projection.  Rows touching the boundary patch take it
  // on the device (ls_create).
  {
    const int Wn = op.Wn;
    for (int prec = 0; prec < 2; ++prec) {
      const std::vector<cd>& Ps = prec == 0 ? op.Psh : op.Psh32;
      std::vector<cd>& Wt = prec == 0 ? op.Wadj : op.Wadj32;
      Wt.assign((size_t)S * Wn * Wn, 0.0);
      std::vector<cd> TP((size_t)F * S);
      for (int o = 0; o < 9; ++o) {
        const int ox = o % 3 - 1, oy = o / 3 - 1;
        std::fill(TP.begin(), TP.end(), cd(0.0, 0.0));
        for (int t = 0; t < F; ++t)
          for (int u2 = 0; u2 < U; ++u2) {
            const cd tv2 = op.Toff[((size_t)o * F + t) * U + u2];
            if (tv2 == 0.0) continue;
            for (int s2 = 0; s2 < S; ++s2) TP[(size_t)t * S + s2] += tv2 * Ps[(size_t)u2 * S + s2];
          }
        for (int a = 0; a < S; ++a)
          for (int s2 = 0; s2 < S; ++s2) {
            cd acc = 0.0;
            for (int t = 0; t < F; ++t) acc += op.Ish[(size_t)a * F + t] * TP[(size_t)t * S + s2];
            const int wx = (ox + 2) * ch + s2 % ch, wy = (oy + 2) * ch + s2 / ch;
            Wt[(size_t)a * Wn * Wn + (size_t)wy * Wn + wx] -= h * h * acc;
          }
      }
    }
  }
  // Green's function on the face lattices, zero padded for linear
  // convolution: set s, normal offset da (units H), tangential db (H/q)
  op.na = L + 1;
  op.nb = L * q;
  op.Pa = next_smooth(2 * op.na - 1);
  op.Pb = next_smooth(2 * op.nb - 1);
  const int Pa = op.Pa, Pb = op.Pb;
  op.kern.assign((size_t)4 * Pa * Pb, 0.0);
  const double scale = 1.0 / ((double)Pa * Pb);
#pragma omp parallel for schedule(static)
  for (int ia = 0; ia < Pa; ++ia) {
    int da = ia < op.na ? ia : ia - Pa;
    if (da <= -op.na || da >= op.na) continue;
    for (int ib = 0; ib < Pb; ++ib) {
      int db = ib < op.nb ? ib : ib - Pb;
      if (db <= -op.nb || db >= op.nb) continue;
      if (da == 0 && db == 0) continue;
      for (int s = 0; s < 2; ++s) {
        double d[2];
        d[s] = da * H;
        d[1 - s] = db * H / q;
        double r = std::hypot(d[0], d[1]);
        op.kern[((size_t)(s * 2 + 0) * Pa + ia) * Pb + ib] = green2d(kappa, r) * scale;
        op.kern[((size_t)(s * 2 + 1) * Pa + ia) * Pb + ib] = green2d_dipole(kappa, d, s) * scale;
      }
    }
  }
  return LS_OK;
}

}  // namespace lsx
