// Numerical helpers of the host set-up: Green's function, 1-D rules,
// cut-offs, Lagrange weights and a complex pseudo-inverse.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "ls_setup.hpp"

namespace lsx {

// G(r) = (i/4) H0^(1)(kappa r) with H0 = J0 + i Y0 (Sec. 1, eq:-G); Bessel
// functions from the C library.
cd green2d(double kappa, double r) {
  double z = kappa * r;
  return cd(-0.25 * ::y0(z), 0.25 * ::j0(z));
}

// d/dy_a of G(|x - y|) at d = x - y: dG/dr = -(i kappa / 4) H1(kappa r) and
// dr/dy_a = -d_a / r, so the derivative is (i kappa / 4) H1(kappa r) d_a / r.
cd green2d_dipole(double kappa, const double d[2], int axis) {
  double r = std::hypot(d[0], d[1]);
  double z = kappa * r;
  cd h1(::j1(z), ::y1(z));
  return cd(0.0, 0.25 * kappa) * h1 * (d[axis] / r);
}

// Gauss–Legendre on [0,1]: Newton iteration on P_n from the Chebyshev-like
// initial guess, P_n and P_n' from the three-term recurrence.
void gauss_legendre01(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < (n + 1) / 2; ++i) {
    long double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    long double pp = 0;
    for (int it = 0; it < 100; ++it) {
      long double p0 = 1, p1 = z;
      for (int k = 2; k <= n; ++k) {
        long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = z; p0 = 1; }
      pp = n * (z * p1 - p0) / (z * z - 1);
      long double dz = p1 / pp;
      z -= dz;
      if (std::fabs((double)dz) < 1e-19) break;
    }
    // recompute derivative at the converged root
    long double p0 = 1, p1 = z;
    for (int k = 2; k <= n; ++k) {
      long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    pp = n * (z * p1 - p0) / (z * z - 1);
    long double wt = 2.0L / ((1 - z * z) * pp * pp);
    // nodes in increasing order on [0,1]
    x[i] = (double)(0.5L * (1 - z));
    x[n - 1 - i] = (double)(0.5L * (1 + z));
    w[i] = w[n - 1 - i] = (double)(0.5L * wt);
  }
}

// Closed Newton–Cotes weights on the nodes 0..Q-1: the interpolatory rule,
// i.e. the solution of sum_k w_k k^p = (Q-1)^(p+1)/(p+1), p < Q, solved in
// extended precision.
std::vector<double> newton_cotes(int Q) {
  std::vector<long double> A(Q * Q), b(Q);
  for (int p = 0; p < Q; ++p) {
    for (int k = 0; k < Q; ++k) A[p * Q + k] = std::pow((long double)k, p);
    b[p] = std::pow((long double)(Q - 1), p + 1) / (p + 1);
  }
  for (int c = 0; c < Q; ++c) {
    int piv = c;
    for (int r = c + 1; r < Q; ++r)
      if (std::fabs((double)A[r * Q + c]) > std::fabs((double)A[piv * Q + c])) piv = r;
    for (int k = 0; k < Q; ++k) std::swap(A[c * Q + k], A[piv * Q + k]);
    std::swap(b[c], b[piv]);
    for (int r = c + 1; r < Q; ++r) {
      long double f = A[r * Q + c] / A[c * Q + c];
      for (int k = c; k < Q; ++k) A[r * Q + k] -= f * A[c * Q + k];
      b[r] -= f * b[c];
    }
  }
  std::vector<long double> x(Q);
  for (int r = Q - 1; r >= 0; --r) {
    long double s = b[r];
    for (int k = r + 1; k < Q; ++k) s -= A[r * Q + k] * x[k];
    x[r] = s / A[r * Q + r];
  }
  return std::vector<double>(x.begin(), x.end());
}

// C-infinity step built on erfc: 0 below 0, 1 above 1.
double smooth_step(double z) {
  if (z <= 0.0) return 0.0;
  if (z >= 1.0) return 1.0;
  const double beta = 3.0;
  return 0.5 * std::erfc(beta * (1.0 - 2.0 * z) / (2.0 * std::sqrt(z * (1.0 - z))));
}

double chi(double s, double c0) { return 1.0 - smooth_step((std::fabs(s) - c0) / (1.0 - c0)); }

int64_t centered_base(double pos, int P) { return (int64_t)std::floor(pos) - (P / 2 - 1); }

// Lagrange weights of the nodes base..base+P-1 at pos (product form).
void lagrange(double pos, int64_t base, int P, double* w) {
  double d[32];
  for (int m = 0; m < P; ++m) d[m] = pos - (double)(base + m);
  for (int k = 0; k < P; ++k) {
    double v = 1.0;
    for (int m = 0; m < P; ++m)
      if (m != k) v *= d[m] / (double)(k - m);
    w[k] = v;
  }
}

// One-sided (Hestenes) Jacobi SVD of a complex m x n matrix (m >= n) in
// extended precision (the matrices are small and their smallest singular
// directions matter), after scaling the columns to unit norm; then
// V diag(1/sigma) U^H with singular values below rcond * sigma_max dropped.
std::vector<cd> pinv(const std::vector<cd>& Ain, int m, int n, double rcond) {
  using ld = long double;
  using cl = std::complex<ld>;
  std::vector<cl> A((size_t)m * n);
  std::vector<ld> dsc(n);
  for (int j = 0; j < n; ++j) {
    ld nn = 0;
    for (int r = 0; r < m; ++r) nn += std::norm(cl(Ain[(size_t)r * n + j]));
    dsc[j] = nn > 0 ? 1.0L / std::sqrt(nn) : 1.0L;
    for (int r = 0; r < m; ++r) A[(size_t)r * n + j] = cl(Ain[(size_t)r * n + j]) * dsc[j];
  }
  std::vector<cl> V((size_t)n * n, cl(0));
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1;
  auto col_dot = [&](int a, int b) {  // a^H b
    cl s = 0;
    for (int r = 0; r < m; ++r) s += std::conj(A[(size_t)r * n + a]) * A[(size_t)r * n + b];
    return s;
  };
  const ld tol = 1e-19L;
  for (int sweep = 0; sweep < 100; ++sweep) {
    ld off = 0;
    for (int p = 0; p < n - 1; ++p)
      for (int qq = p + 1; qq < n; ++qq) {
        ld al = std::real(col_dot(p, p));
        ld be = std::real(col_dot(qq, qq));
        cl ga = col_dot(p, qq);
        ld ag = std::abs(ga);
        if (ag == 0 || al == 0 || be == 0) continue;
        off = std::max(off, ag / std::sqrt(al * be));
        if (ag <= tol * std::sqrt(al * be)) continue;
        cl ph = ga / ag;
        ld zeta = (be - al) / (2 * ag);
        ld t = (zeta >= 0 ? 1 : -1) / (std::fabs(zeta) + std::sqrt(1 + zeta * zeta));
        ld c = 1 / std::sqrt(1 + t * t), s = c * t;
        // [a_p, a_q] <- [a_p, a_q] [[c, s e^{i phi}], [-s e^{-i phi}, c]]
        for (int r = 0; r < m; ++r) {
          cl ap = A[(size_t)r * n + p], aq = A[(size_t)r * n + qq];
          A[(size_t)r * n + p] = c * ap - s * std::conj(ph) * aq;
          A[(size_t)r * n + qq] = s * ph * ap + c * aq;
        }
        for (int r = 0; r < n; ++r) {
          cl vp = V[(size_t)r * n + p], vq = V[(size_t)r * n + qq];
          V[(size_t)r * n + p] = c * vp - s * std::conj(ph) * vq;
          V[(size_t)r * n + qq] = s * ph * vp + c * vq;
        }
      }
    if (off < tol) break;
  }
  std::vector<ld> sig(n);
  ld smax = 0;
  for (int i = 0; i < n; ++i) {
    sig[i] = std::sqrt(std::real(col_dot(i, i)));
    smax = std::max(smax, sig[i]);
  }
  std::vector<cl> acc((size_t)n * m, cl(0));
  for (int i = 0; i < n; ++i) {
    if (sig[i] <= rcond * smax) continue;
    ld inv2 = 1 / (sig[i] * sig[i]);   // u_i = a_i / sigma_i
    for (int j = 0; j < n; ++j) {
      cl vj = V[(size_t)j * n + i] * inv2;
      for (int k = 0; k < m; ++k) acc[(size_t)j * m + k] += vj * std::conj(A[(size_t)k * n + i]);
    }
  }
  std::vector<cd> out((size_t)n * m);
  for (int j = 0; j < n; ++j)
    for (int k = 0; k < m; ++k) out[(size_t)j * m + k] = cd(acc[(size_t)j * m + k] * dsc[j]);
  return out;
}

// Householder QR with column pivoting (numerical rank at rcond |R_00|).
QRCP qrcp(const std::vector<cd>& A, int m, int n, double rcond) {
  QRCP f;
  f.m = m;
  f.n = n;
  f.QR = A;
  f.perm.resize(n);
  std::iota(f.perm.begin(), f.perm.end(), 0);
  f.v.assign((size_t)n * m, 0.0);
  f.vn.assign(n, 0.0);
  f.r = 0;
  double r00 = 0;
  for (int k = 0; k < n && k < m; ++k) {
    // pivot: remaining column of largest norm
    int best = k;
    double bn = -1;
    for (int j = k; j < n; ++j) {
      double nn = 0;
      for (int i = k; i < m; ++i) nn += std::norm(f.QR[(size_t)i * n + j]);
      if (nn > bn) { bn = nn; best = j; }
    }
    if (best != k) {
      for (int i = 0; i < m; ++i) std::swap(f.QR[(size_t)i * n + k], f.QR[(size_t)i * n + best]);
      std::swap(f.perm[k], f.perm[best]);
    }
    double xn = std::sqrt(bn);
    if (k == 0) r00 = xn;
    if (xn <= rcond * r00 || xn == 0.0) break;
    cd x0 = f.QR[(size_t)k * n + k];
    cd alpha = -(std::abs(x0) > 0 ? x0 / std::abs(x0) : cd(1.0)) * xn;
    cd* v = &f.v[(size_t)k * m];
    for (int i = k; i < m; ++i) v[i] = f.QR[(size_t)i * n + k];
    v[k] -= alpha;
    double vn = 0;
    for (int i = k; i < m; ++i) vn += std::norm(v[i]);
    f.vn[k] = vn;
    // apply H = I - 2 v v^H / (v^H v) to the remaining columns
    for (int j = k + 1; j < n; ++j) {
      cd dot = 0;
      for (int i = k; i < m; ++i) dot += std::conj(v[i]) * f.QR[(size_t)i * n + j];
      cd fct = 2.0 * dot / vn;
      for (int i = k; i < m; ++i) f.QR[(size_t)i * n + j] -= fct * v[i];
    }
    f.QR[(size_t)k * n + k] = alpha;
    for (int i = k + 1; i < m; ++i) f.QR[(size_t)i * n + k] = 0.0;
    f.r = k + 1;
  }
  return f;
}

// Basic least-squares solution of the rank-r truncated problem:
// x = P [R11^{-1} (Q^H b)_{1..r}; 0].
void qrcp_solve(const QRCP& f, const cd* b, cd* x) {
  const int m = f.m, n = f.n, r = f.r;
  std::vector<cd> y(b, b + m);
  for (int k = 0; k < r; ++k) {
    const cd* v = &f.v[(size_t)k * m];
    cd dot = 0;
    for (int i = k; i < m; ++i) dot += std::conj(v[i]) * y[i];
    cd fct = 2.0 * dot / f.vn[k];
    for (int i = k; i < m; ++i) y[i] -= fct * v[i];
  }
  std::vector<cd> z(r);
  for (int i = r - 1; i >= 0; --i) {
    cd s = y[i];
    for (int j = i + 1; j < r; ++j) s -= f.QR[(size_t)i * n + j] * z[j];
    z[i] = s / f.QR[(size_t)i * n + i];
  }
  for (int j = 0; j < n; ++j) x[j] = 0.0;
  for (int i = 0; i < r; ++i) x[f.perm[i]] = z[i];
}

int next_smooth(int n) {
  for (int m = std::max(n, 1);; ++m) {
    int r = m;
    for (int f : {2, 3, 5})
      while (r % f == 0) r /= f;
    if (r == 1) return m;
  }
}

}  // namespace lsx
