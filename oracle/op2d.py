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
* cfg["offgrid_shortcut"]: at an interior lattice node inside the boundary
  patch the patch's eta part is interpolated from its values at the patch's
  grid nodes (the remark after eq:-VolInt-Adj-Sing-MultiSplit; shortcut_weights).
* The split of K_h into adjacent and non-adjacent cells (eq:-VolInt-Adj-NonAdj)
  only reorganises this sum; the oracle sums every pair directly (the
  non-accelerated O(N^2) evaluation of the paper's efficiency study).
"""
import numpy as np

from .geom2d import band_index, discretize, lattice_index
from .near2d import (band_sing_row, eta_band, eta_interior, green2d,
                     interior_sing_row, polar_radial_rule, varrho_rule)
from .quad import centered_base, lagrange_weights, trig_interp_weights


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
        weights m omega (interior) / m omega J (boundary patch)).  With
        cfg["offgrid_shortcut"] the boundary patch's part at an interior
        lattice node inside the patch comes from band_sing_shortcut."""
        p, cfg = self.pts, self.cfg
        row = np.zeros(self.N, complex)
        j, w = interior_sing_row(p["x"][i], p, self.lat, cfg, self.kappa, self.polar_rule,
                                 self._cache)
        np.add.at(row, j, w * p["dens"][j])
        for k in range(p["vp"].shape[0]):
            if p["inp"][k, i]:
                if cfg.get("offgrid_shortcut", 0) and p["chart"][i] == 0:
                    row += self.band_sing_shortcut(i) * p["dens"]
                    continue
                j, w = band_sing_row(p["x"][i], p["vp"][k, i], p["u"][i], p, self.bidx, cfg,
                                     self.kappa, self.t1_rule, patch=k)
                np.add.at(row, j, w * p["dens"][j])
        return row

    def _node_sing(self, j):
        """Boundary rule at band grid node j (its own grid coordinates)."""
        c = self._cache.setdefault("node_sing", {})
        if j not in c:
            p = self.pts
            c[j] = band_sing_row(p["x"][j], float(p["key"][j, 1]), float(p["key"][j, 2]), p, self.bidx,
                                 self.cfg, self.kappa, self.t1_rule, patch=0)
        return c[j]

    def band_sing_shortcut(self, i):
        """The paper's shortcut for a target off the patch's grid lines (remark
        after eq:-VolInt-Adj-Sing-MultiSplit): the boundary rule's value at the
        patch's grid nodes, interpolated to the target's patch coordinates
        (vt, ut) by P-point Lagrange stencils in t2 (one-sided at the ends)
        and, in t1, on the fft_refine-fold refined grid of each t2 line
        (trigonometric interpolation of the line's node values, as for the
        densities).  Single periodic band only.  Returns the weights of
        (m omega J)_j u_j as a dense row."""
        p = self.pts
        acc = np.zeros(self.N, complex)
        for (v, u), w in shortcut_weights(float(p["vp"][0, i]), float(p["u"][i]), self.cfg).items():
            jj, ww = self._node_sing(int(self.bidx[0][v, u]))
            np.add.at(acc, jj, w * ww)
        return acc


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

def shortcut_weights(vt, ut, cfg):
    """Interpolation weights of the off-grid shortcut: {(v, u): weight} over
    the band grid nodes for the value at patch coordinates (vt, ut) (grid
    units): P-point Lagrange in t2 (stencil shifted one-sided at the ends),
    in t1 P-point Lagrange on the fft_refine-fold refined grid whose values
    are the trigonometric interpolant of the line (periodic; plain Lagrange
    with wrap-around when fft_refine = 1)."""
    b = cfg["band"]
    if b.get("patches", 1) != 1:
        raise ValueError("the off-grid shortcut needs the single periodic band")
    N1, N2, P = b["N1"], b["N2"], cfg["P"]
    rf = int(cfg.get("fft_refine", 1))
    bu = int(np.clip(centered_base(np.array([ut]), P)[0], 0, N2 - P + 1))
    Lu = lagrange_weights(np.array([ut]), np.array([bu]), P)[0]
    bv = int(centered_base(np.array([rf * vt]), P)[0])
    Lv = lagrange_weights(np.array([rf * vt]), np.array([bv]), P)[0]
    if rf > 1:
        Wv = Lv @ trig_interp_weights((bv + np.arange(P)) / rf, N1)
    else:
        Wv = np.zeros(N1)
        np.add.at(Wv, np.mod(bv + np.arange(P), N1), Lv)
    out = {}
    for a in range(P):
        for v in np.nonzero(Wv)[0]:
            out[(int(v), bu + a)] = out.get((int(v), bu + a), 0.0) + Lu[a] * Wv[v]
    return out
