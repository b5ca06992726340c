// Numerical helpers of the host set-up: Green's function, 1-D rules,
// cut-offs, Lagrange weights and a complex pseudo-inverse.
#include <algorithm>
#include <cmath>

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

// One-sided (Hestenes) Jacobi SVD of a complex m x n matrix (m >= n), then
// V diag(1/sigma) U^H with small singular values dropped.
std::vector<cd> pinv(const std::vector<cd>& Ain, int m, int n, double rcond) {
  std::vector<cd> A(Ain);          // columns are orthogonalised in place
  std::vector<cd> V(n * n, 0.0);
  for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
  auto col_dot = [&](int a, int b) {  // a^H b
    cd s = 0;
    for (int r = 0; r < m; ++r) s += std::conj(A[r * n + a]) * A[r * n + b];
    return s;
  };
  for (int sweep = 0; sweep < 80; ++sweep) {
    double off = 0;
    for (int p = 0; p < n - 1; ++p)
      for (int qq = p + 1; qq < n; ++qq) {
        double al = std::real(col_dot(p, p));
        double be = std::real(col_dot(qq, qq));
        cd ga = col_dot(p, qq);
        double ag = std::abs(ga);
        if (ag == 0.0 || al == 0.0 || be == 0.0) continue;
        off = std::max(off, ag / std::sqrt(al * be));
        if (ag <= 1e-16 * std::sqrt(al * be)) continue;
        cd ph = ga / ag;
        double zeta = (be - al) / (2.0 * ag);
        double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        double c = 1.0 / std::sqrt(1.0 + t * t), s = c * t;
        // [a_p, a_q] <- [a_p, a_q] [[c, s e^{i phi}], [-s e^{-i phi}, c]]
        for (int r = 0; r < m; ++r) {
          cd ap = A[r * n + p], aq = A[r * n + qq];
          A[r * n + p] = c * ap - s * std::conj(ph) * aq;
          A[r * n + qq] = s * ph * ap + c * aq;
        }
        for (int r = 0; r < n; ++r) {
          cd vp = V[r * n + p], vq = V[r * n + qq];
          V[r * n + p] = c * vp - s * std::conj(ph) * vq;
          V[r * n + qq] = s * ph * vp + c * vq;
        }
      }
    if (off < 1e-15) break;
  }
  std::vector<double> sig(n);
  double smax = 0;
  for (int i = 0; i < n; ++i) {
    sig[i] = std::sqrt(std::real(col_dot(i, i)));
    smax = std::max(smax, sig[i]);
  }
  std::vector<cd> out(n * m, 0.0);
  for (int i = 0; i < n; ++i) {
    if (sig[i] <= rcond * smax) continue;
    double inv2 = 1.0 / (sig[i] * sig[i]);   // u_i = a_i / sigma_i
    for (int j = 0; j < n; ++j) {
      cd vj = V[j * n + i] * inv2;
      for (int k = 0; k < m; ++k) out[j * m + k] += vj * std::conj(A[k * n + i]);
    }
  }
  return out;
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
