"""Kernel, localisation and singular quadratures of the 2-D method (oracle).

Test infrastructure only (see oracle/__init__.py).

* Green's function G(x,y) = (i/4) H_0^(1)(kappa |x-y|)  (Sec. 1, eq:-G),
  evaluated with the library Bessel routines J0, Y0.
* Localisation eta (Sec. 3, eq:-VolInt-B-III):
  interior patch: eta = chi(|y - x| / r_int) (circular support, Sec. 3.1.1);
  boundary patch: eta = chi(|t1-t1^x|/r1) chi(|t2-t2^x|/r2) (rectangular
  support, Sec. 3.1.2; separate radii per parametric axis are a reading).
* Interior singular rule (Sec. 3.1.1, eq:-K-Int-Sing-Polar): polar
  coordinates around the target.  The paper's claim that |rho| G is smooth
  does not hold in 2-D (rho log rho term), so the radial integral is split at
  the radius where chi stops being 1: graded Gauss–Legendre rho = a s^g on
  [0, a], Gauss–Legendre on [a, r]; trapezoid in theta (reading).
* Boundary singular rule (Sec. 3.1.2): t1 = t1^x + varrho(tau),
  varrho = tau^(M+1) applied on the inner part [0, a] of the cut-off and a
  Gauss–Legendre rule on the cut-off transition (reading of eq:-I-inTau);
  the t2 integral uses the multi-split composite Newton–Cotes rule
  (eq:-VolInt-Adj-Sing-MultiSplit) anchored at t2^x.
* Off-grid values of the patch densities come from tensor Lagrange
  interpolation with P nodes per axis.  With cfg["fft_refine"] = r > 1 the
  boundary rule uses the Fourier refined polynomial interpolation of Sec. 3.1
  along the periodic t1 axis of the single band: each t2 line of the density
  is first refined r-fold by trigonometric interpolation (zero-padded
  spectrum), and the P-point Lagrange stencils then sit on the refined grid
  (spacing 1/r).  The t2 axis (the interface end is not periodic) keeps
  plain Lagrange stencils (reading).  With cfg["fft_refine_interior"] set as
  well, the interior polar rule's stencils sit on the r-fold refined lattice:
  the refined values are the two-dimensional trigonometric interpolant of
  the interior density (m omega u, compactly supported inside the lattice)
  with the period M of interior_refine_period in both axes.
"""
import numpy as np
from scipy import special

from .quad import (centered_base, chi, gauss_legendre01, lagrange_weights,
                   newton_cotes_closed, trig_interp_weights)


def green2d(kappa, r):
    """(i/4) H0^(1)(kappa r) = (i/4) (J0 + i Y0)."""
    z = kappa * np.asarray(r, dtype=np.float64)
    return 0.25j * special.j0(z) - 0.25 * special.y0(z)


# ----------------------------------------------------------------------------
# localisation functions
# ----------------------------------------------------------------------------

def eta_interior(xt, xs, cfg):
    """eta for a source on the interior patch: chi(|x_s - x_t| / r_int)."""
    d = np.hypot(xs[..., 0] - xt[..., 0], xs[..., 1] - xt[..., 1])
    return chi(d / cfg["r_int"], cfg["chi_c0"])


def eta_band(vt, ut, vs, us, cfg):
    """eta for a source on a boundary patch (grid units of that patch; t1
    periodic for the single periodic band)."""
    N1 = cfg["band"]["N1"]
    dv = np.abs(vs - vt)
    if cfg["band"].get("patches", 1) == 1:
        dv = np.minimum(dv, N1 - dv)
    return chi(dv / cfg["r1"], cfg["chi_c0"]) * chi(np.abs(us - ut) / cfg["r2"], cfg["chi_c0"])


# ----------------------------------------------------------------------------
# one-dimensional pieces of the singular rules
# ----------------------------------------------------------------------------

def polar_radial_rule(cfg):
    """Radial nodes and weights on [0, r_int] (physical units); the weights
    include chi(rho/r) but neither rho nor G."""
    p = cfg["polar"]
    r = cfg["r_int"]
    a = cfg["chi_c0"] * r
    s, ws = gauss_legendre01(p["n_in"])
    g = p["grade"]
    rho_in = a * s ** g
    w_in = a * g * s ** (g - 1) * ws
    t, wt = gauss_legendre01(p["n_out"])
    rho_out = a + (r - a) * t
    w_out = (r - a) * wt * chi(rho_out / r, cfg["chi_c0"])
    return np.concatenate([rho_in, rho_out]), np.concatenate([w_in, w_out])


def varrho_rule(cfg):
    """Offsets (t1 grid units) and weights of the boundary-patch t1 rule on
    [-r1, r1]; the weights include chi(|offset| / r1)."""
    br = cfg["band_rule"]
    r1 = cfg["r1"]
    a = cfg["chi_c0"] * r1
    M = br["M"]
    s, ws = gauss_legendre01(br["n_in"])
    d_in = a * s ** (M + 1)
    w_in = a * (M + 1) * s ** M * ws
    t, wt = gauss_legendre01(br["n_out"])
    d_out = a + (r1 - a) * t
    w_out = (r1 - a) * wt * chi(d_out / r1, cfg["chi_c0"])
    d = np.concatenate([d_in, d_out])
    w = np.concatenate([w_in, w_out])
    return np.concatenate([-d[::-1], d]), np.concatenate([w[::-1], w])


def multisplit_rule(ux, N2, Q, r2, c0):
    """Transverse rule for int_0^{N2} f(u) chi(|u-ux|/r2) du (grid units).

    Eq. eq:-VolInt-Adj-Sing-MultiSplit, read with floor brackets: on each side
    of ux, L full panels of Q-1 unit intervals anchored at ux, then I single
    unit intervals (each with a Q-point rule on Q-1 sub-intervals), then the
    remaining piece up to the patch edge (empty when ux is a grid line),
    also with one Q-point rule.  Returns (positions, weights incl. chi)."""
    nc = newton_cotes_closed(Q)
    pos, wts = [], []

    def panel(a, b):
        hh = (b - a) / (Q - 1)
        for k in range(Q):
            pos.append(a + k * hh)
            wts.append(nc[k] * hh)

    for side in (-1.0, 1.0):
        span = ux if side < 0 else N2 - ux
        L = int(np.floor(span / (Q - 1)))
        for l in range(1, L + 1):
            if (l - 1) * (Q - 1) >= r2:
                break
            a, b = ux + side * (l - 1) * (Q - 1), ux + side * l * (Q - 1)
            panel(min(a, b), max(a, b))
        rem = span - L * (Q - 1)
        I = int(np.floor(rem))
        base = L * (Q - 1)
        for i in range(1, I + 1):
            if base + i - 1 >= r2:
                break
            a, b = ux + side * (base + i - 1), ux + side * (base + i)
            panel(min(a, b), max(a, b))
        w = rem - I
        if w > 0.0 and base + I < r2:
            a, b = ux + side * (base + I), ux + side * span
            panel(min(a, b), max(a, b))
    pos = np.array(pos)
    wts = np.array(wts) * chi(np.abs(pos - ux) / r2, c0)
    keep = wts != 0.0
    pos, wts = pos[keep], wts[keep]
    # merge coincident panel end points
    key = np.round(pos * 2.0 ** 30)
    uk, inv = np.unique(key, return_inverse=True)
    wsum = np.zeros(uk.shape[0])
    np.add.at(wsum, inv, wts)
    psum = np.zeros(uk.shape[0])
    psum[inv] = pos
    return psum, wsum


# ----------------------------------------------------------------------------
# singular (eta) parts as sparse rows
# ----------------------------------------------------------------------------

def interior_refine_period(pts, cfg):
    """Period (lattice points per axis) of the interior refinement: the
    side of the box of the cells of side cell_h h that hold every node
    (interior nodes by their lattice index, boundary-patch nodes by their
    position), plus two cells on each side, rounded up to the next integer
    whose only prime factors are 2, 3 and 5 (reading: the paper names no
    period; the density vanishes well inside this box)."""
    ch = cfg["cell_h"]
    H = ch * cfg["h"]
    key, x = pts["key"], pts["x"]
    interior = key[:, 0] == 0
    c = np.where(interior[:, None], np.floor_divide(key[:, 1:], ch), np.floor(x / H).astype(np.int64))
    L = int(c.max() - c.min() + 1)
    M = (L + 4) * ch
    while True:
        r = M
        for f in (2, 3, 5):
            while r % f == 0:
                r //= f
        if r == 1:
            return M
        M += 1


def interior_stencil(frac1, frac2, rule, cfg, kappa, rf=1):
    """Polar rule around a target at (base + frac) h, base integer:
    returns lattice offsets (d1, d2) relative to base and complex weights such
    that K_sing = sum w * (m omega u)[base + d].  Quadrature nodes
    y = x + rho (cos th, sin th), th = 2 pi b / n_theta (trapezoid); values at
    y from the P x P Lagrange stencil around y.  rf > 1: the stencils sit on
    the rf-fold refined lattice and the offsets are in refined units
    (refined node rf (base + d) + s is lattice node base + d for s = 0)."""
    rho, wr = rule
    h = cfg["h"]
    P = cfg["P"]
    nth = cfg["polar"]["n_theta"]
    th = 2.0 * np.pi * np.arange(nth) / nth
    wrad = wr * rho * green2d(kappa, rho) * (2.0 * np.pi / nth)
    p1 = (rf * (frac1 + np.multiply.outer(rho, np.cos(th)) / h)).ravel()
    p2 = (rf * (frac2 + np.multiply.outer(rho, np.sin(th)) / h)).ravel()
    Wq = np.repeat(wrad, nth)
    b1 = centered_base(p1, P)
    b2 = centered_base(p2, P)
    L1 = lagrange_weights(p1, b1, P) * Wq[:, None]
    L2 = lagrange_weights(p2, b2, P)
    lo1, lo2 = b1.min(), b2.min()
    n1 = b1.max() + P - lo1
    n2 = b2.max() + P - lo2
    i1 = (b1 - lo1)[:, None, None] + np.arange(P)[None, :, None]
    i2 = (b2 - lo2)[:, None, None] + np.arange(P)[None, None, :]
    flat = (i1 * n2 + i2).ravel()
    W = (L1[:, :, None] * L2[:, None, :]).ravel()
    acc = np.bincount(flat, W.real, n1 * n2) + 1j * np.bincount(flat, W.imag, n1 * n2)
    nz = np.nonzero(acc)[0]
    return nz // n2 + lo1, nz % n2 + lo2, acc[nz]


def interior_sing_row(xt, pts, lat_idx, cfg, kappa, rule=None, cache=None):
    """Row of the interior-patch singular part at target xt: returns
    (point indices, weights) such that K_sing = sum_j wt_j * (m omega)_j u_j.
    Lattice nodes that are not unknowns carry zero density and are dropped.
    On-lattice targets all share one stencil (the patch is Cartesian and G
    depends on x - y only); it is computed once and shifted.  With interior
    Fourier refinement a refined node between lattice nodes carries the
    two-dimensional trigonometric interpolant (period M) of the lattice
    density, which spreads its weight over the whole lattice."""
    if rule is None:
        rule = polar_radial_rule(cfg)
    rf = int(cfg.get("fft_refine", 1)) if cfg.get("fft_refine_interior", 0) else 1
    h = cfg["h"]
    g = xt / h
    gi = np.round(g)
    if np.all(np.abs(g - gi) < 1e-12):
        base = gi.astype(np.int64)
        if cache is not None and "onlattice" in cache:
            d1, d2, w = cache["onlattice"]
        else:
            d1, d2, w = interior_stencil(0.0, 0.0, rule, cfg, kappa, rf)
            if cache is not None:
                cache["onlattice"] = (d1, d2, w)
    else:
        base = np.floor(g).astype(np.int64)
        d1, d2, w = interior_stencil(g[0] - base[0], g[1] - base[1], rule, cfg, kappa, rf)
    imax = pts["imax"]
    n = 2 * imax + 1
    if rf > 1:
        s1, s2 = np.mod(d1, rf), np.mod(d2, rf)
        on = (s1 == 0) & (s2 == 0)
        # refined node positions in lattice index units, off the lattice
        X1 = base[0] + d1[~on] / rf
        X2 = base[1] + d2[~on] / rf
        wo = w[~on]
        d1, d2, w = d1[on] // rf, d2[on] // rf, w[on]
    I1 = base[0] + d1 + imax
    I2 = base[1] + d2 + imax
    ok = (I1 >= 0) & (I1 < n) & (I2 >= 0) & (I2 < n)
    j = lat_idx[I1[ok], I2[ok]]
    sel = j >= 0
    jj, ww = j[sel], w[ok][sel]
    if rf == 1 or wo.size == 0:
        return jj, ww
    # sum_n wo_n D(X1_n - i1) D(X2_n - i2) over lattice (i1, i2), grouped by
    # the distinct X1 (sample k of the period box is lattice index k - imax)
    M = cache["period"] if cache is not None and "period" in cache else interior_refine_period(pts, cfg)
    if cache is not None:
        cache["period"] = M
    ux, inv = np.unique(np.round(X1 * rf).astype(np.int64), return_inverse=True)
    D2 = trig_interp_weights(X2 + imax, M)[:, :n] * wo[:, None]            # (n_off, n)
    G2 = np.zeros((ux.size, n), complex)
    np.add.at(G2, inv, D2)
    D1 = trig_interp_weights(ux / rf + imax, M)[:, :n]                     # (n_ux, n)
    R = D1.T @ G2                                                          # (n, n) over (I1, I2)
    J = lat_idx
    m = J >= 0
    jj = np.concatenate([jj, J[m]])
    ww = np.concatenate([ww, R[m]])
    return jj, ww


def band_sing_row(xt, vt, ut, pts, band_idx, cfg, kappa, t1rule=None, patch=0):
    """Row of boundary patch `patch`'s singular part at a target with patch
    coordinates (vt, ut) (grid units): K_sing = sum_j wt_j (m omega J)_j u_j.
    On a non-periodic patch the t1 rule's nodes beyond the patch ends are
    dropped (the partition of unity makes the density vanish there) and the
    t1 interpolation stencils are shifted one-sided at the ends, like the t2
    stencils at the interface.  With cfg["fft_refine"] = r > 1 (single
    periodic band only) the t1 stencils sit on the r-fold refined grid; a
    refined node between grid nodes carries the trigonometric interpolant of
    its t2 line, which spreads its weight over the whole line."""
    from .geom2d import band_map
    b = cfg["band"]
    N1, N2 = b["N1"], b["N2"]
    P = cfg["P"]
    periodic = b.get("patches", 1) == 1
    rf = int(cfg.get("fft_refine", 1))
    if rf > 1 and not periodic:
        raise ValueError("fft_refine needs the single periodic band")
    if t1rule is None:
        t1rule = varrho_rule(cfg)
    d1, w1 = t1rule
    lines, w2 = multisplit_rule(ut, N2, cfg["Q"], cfg["r2"], cfg["chi_c0"])
    if lines.size == 0:
        return np.zeros(0, np.int64), np.zeros(0, complex)
    V = vt + d1                        # (n1,)
    if not periodic:
        keep = (V >= 0.0) & (V <= N1)
        V, w1 = V[keep], w1[keep]
        if V.size == 0:
            return np.zeros(0, np.int64), np.zeros(0, complex)
    T1 = np.broadcast_to(V[None, :] / N1, (lines.size, V.size))
    T2 = np.broadcast_to((lines / N2)[:, None], (lines.size, V.size))
    Y = band_map(T1, T2, cfg, patch)
    r = np.hypot(Y[..., 0] - xt[0], Y[..., 1] - xt[1])
    # a node that rounds onto the target itself has zero measure: drop it
    Gr = np.where(r > 0.0, green2d(kappa, np.where(r > 0.0, r, 1.0)), 0.0)
    Wq = (w2[:, None] / N2) * (w1[None, :] / N1) * Gr                    # (nl, n1)
    # t1 stencils in units of the (refined) grid spacing 1/rf
    bv = centered_base(rf * V, P)
    if not periodic:
        bv = np.clip(bv, 0, N1 - P + 1)
    Lv = lagrange_weights(rf * V, bv, P)                                   # (n1,P)
    bu = np.clip(centered_base(lines, P), 0, N2 - P + 1)
    Lu = lagrange_weights(lines, bu, P)                                    # (nl,P)
    # tangential scatter: R[l, v] = sum_k Wq[l,k] Lv[k,a] at v = bv[k]+a
    lo_v = bv.min()
    nv = bv.max() + P - lo_v
    vflat = ((bv - lo_v)[:, None] + np.arange(P)[None, :]).ravel()     # (n1*P,)
    Sv = np.zeros((V.size * P, nv))
    Sv[np.arange(V.size * P), vflat] = 1.0
    Rv = (Wq[:, :, None] * Lv[None, :, :]).reshape(lines.size, -1) @ Sv   # (nl, nv)
    # transverse scatter: row[u, v] = sum_l Lu[l,b] R[l, v] at u = bu[l]+b
    lo_u = bu.min()
    nu = bu.max() + P - lo_u
    Su = np.zeros((nu, lines.size))
    for bb in range(P):
        Su[bu - lo_u + bb, np.arange(lines.size)] += Lu[:, bb]
    win = Su @ Rv                                                          # (nu, nv)
    if rf > 1:
        # refined node (v0 + s/rf) of line u: the trigonometric interpolant
        # of the line's N1 grid values; s = 0 is the grid node itself
        vr = np.arange(nv) + lo_v
        T = trig_interp_weights(vr / rf, N1)                               # (nv, N1)
        win = win @ T                                                      # (nu, N1)
        lo_v = 0
    iu, iv = np.nonzero(win)
    vv = np.mod(iv + lo_v, N1) if periodic else iv + lo_v
    j = band_idx[patch][vv, iu + lo_u]
    wt = win[iu, iv]
    # grid nodes that are not unknowns (zero partition of unity) carry no density
    wt, j = wt[j >= 0], j[j >= 0]
    # several window columns can wrap onto one periodic index
    uj, inv = np.unique(j, return_inverse=True)
    acc = np.zeros(uj.shape[0], complex)
    np.add.at(acc, inv, wt)
    return uj, acc
