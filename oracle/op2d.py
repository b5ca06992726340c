"""The discrete 2-D Lippmann–Schwinger operator A = I + kappa^2 K_h (oracle).

Test infrastructure only (see oracle/__init__.py).

K_h[u](x_i) = sum_j (1 - eta_ij) G(x_i - x_j) c_j u_j          (plain part)
            + sum_{patches k with x_i in P_k} K_k^sing[u](x_i)   (eta parts)

* c_j = w_j |J_j| omega_j m_j is the plain quadrature weight (Sec. 3:
  trapezoid on the interior patch, trapezoid x composite Newton–Cotes on the
  boundary patch; eq:-disctete-conv for the far part).
* eta_ij is the localisation of the patch that owns node j, centred at the
  target (eq:-VolInt-Adj-NonAdj-I); it is zero when x_i is not in that patch.
  With several boundary patches each one contributes its own eta and its own
  singular part at every target it contains.
  The terms with eta_ij = 1 (including j = i) drop out.
* The split of K_h into adjacent and non-adjacent cells (eq:-VolInt-Adj-NonAdj)
  only reorganises this sum; the oracle sums every pair directly (the
  non-accelerated O(N^2) evaluation of the paper's efficiency study).
"""
import numpy as np

from .geom2d import band_index, discretize, lattice_index
from .near2d import (band_sing_row, eta_band, eta_interior, green2d,
                     interior_sing_row, polar_radial_rule, varrho_rule)


class Setup2D:
    def __init__(self, cfg, n2_fn):
        self.cfg = cfg
        self.kappa = cfg["kappa"]
        self.pts = discretize(cfg, n2_fn)
        self.N = self.pts["x"].shape[0]
        self.lat = lattice_index(self.pts)
        self.bidx = band_index(self.pts, cfg)
        self.polar_rule = polar_radial_rule(cfg)
        self.t1_rule = varrho_rule(cfg)
        self._cache = {}

    # ------------------------------------------------------------------ rows
    def plain_row(self, i):
        p, cfg = self.pts, self.cfg
        x = p["x"]
        eta = np.zeros(self.N)
        n_int = p["n_int"]
        eta[:n_int] = eta_interior(x[i], x[:n_int], cfg)
        # sources of boundary patch k: eta centred at the target's own
        # coordinates in patch k when it lies in patch k, else 0
        for k in range(p["vp"].shape[0]):
            if p["inp"][k, i]:
                own = np.nonzero(p["chart"] == 1 + k)[0]
                eta[own] = eta_band(p["vp"][k, i], p["u"][i], p["vp"][k, own], p["u"][own], cfg)
        f = 1.0 - eta
        row = np.zeros(self.N, complex)
        nz = f != 0.0
        r = np.hypot(x[nz, 0] - x[i, 0], x[nz, 1] - x[i, 1])
        row[nz] = f[nz] * green2d(self.kappa, r) * p["c"][nz]
        return row

    def sing_row(self, i):
        """Dense row of the eta parts (already multiplied by the density
        weights m omega (interior) / m omega J (boundary patch))."""
        p, cfg = self.pts, self.cfg
        row = np.zeros(self.N, complex)
        j, w = interior_sing_row(p["x"][i], p, self.lat, cfg, self.kappa, self.polar_rule,
                                 self._cache)
        np.add.at(row, j, w * p["dens"][j])
        for k in range(p["vp"].shape[0]):
            if p["inp"][k, i]:
                j, w = band_sing_row(p["x"][i], p["vp"][k, i], p["u"][i], p, self.bidx, cfg,
                                     self.kappa, self.t1_rule, patch=k)
                np.add.at(row, j, w * p["dens"][j])
        return row

    def K_row(self, i):
        return self.plain_row(i) + self.sing_row(i)

    def K_rows(self, rows):
        return np.stack([self.K_row(int(i)) for i in rows])

    def dense_K(self):
        return self.K_rows(range(self.N))

    # ----------------------------------------------------------- operators
    def A_rows(self, rows):
        K = self.K_rows(rows)
        A = (self.kappa ** 2) * K
        A[np.arange(len(rows)), np.asarray(rows)] += 1.0
        return A

    def dense_A(self):
        return self.A_rows(np.arange(self.N))
