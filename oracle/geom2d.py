"""Two-dimensional Nyström discretisation used by the oracle.

Test infrastructure only (see oracle/__init__.py).

The scatterer is the star domain  s(x) = |x| / R(theta) < 1  with
R(theta) = 1 + a cos(k theta)  (a = 0: the unit disc).  It is covered by two
overlapping patches (Sec. 2):

* an interior patch: the Cartesian lattice x = h (i1, i2), whose partition of
  unity function vanishes to all orders before the boundary, so that the
  trapezoidal rule (weight h^2) applies (Sec. 3, regular quadratures);
* a boundary patch (the band s_in <= s <= 1): t1 in [0,1) periodic
  (theta = 2 pi t1), t2 in [0,1] transverse with the boundary at t2 = 0
  (remark at the end of Sec. 2), x = s R(theta) (cos theta, sin theta),
  s = 1 - (1 - s_in) t2, nodes (i1/N1, i2/N2), 0 <= i1 < N1, 0 <= i2 <= N2.
  Quadrature: trapezoid in t1 times composite Newton–Cotes in t2.

Partition of unity (not given in the paper; a reading):
omega_b(x) = smooth_step((s - s_a)/(s_b - s_a)), omega_int = 1 - omega_b.
Interior lattice nodes with omega_int = 0 are not unknowns.

Several boundary patches (Sec. 2: the boundary is covered by overlapping
patches with a partition of unity; the paper's layouts use two).  With
cfg["band"]["patches"] = P >= 2 the band is covered by P non-periodic
patches: patch p spans theta in [theta_p - D, theta_p + D] with
theta_p = 2 pi p / P and D = pi / P + delta (delta = cfg["band"]["overlap"]),
t1 in [0, 1] maps linearly onto that range, nodes t1 = i1 / N1 with
0 <= i1 <= N1.  Tangential partition of unity: bumps
b_p = smooth_step((D - |theta - theta_p|) / (2 delta)), which vanish to all
orders at their patch's ends, normalised, omega_p = b_p / sum_q b_q; a node's
weight carries omega_band(s) omega_p(theta).  The integrand then vanishes to
all orders at both t1 ends, so the trapezoid rule in t1 stays spectrally
accurate (Sec. 3, regular quadratures); nodes with omega = 0 (the end nodes)
are not unknowns.  P = 1 is the single periodic band.
"""
import numpy as np

from .quad import composite_newton_cotes, smooth_step


def radius(theta, shape):
    return 1.0 + shape["a"] * np.cos(shape["k"] * theta)


def n_patches(cfg):
    return int(cfg["band"].get("patches", 1))


def patch_frame(cfg, p):
    """(theta at t1 = 0, theta span) of boundary patch p."""
    P = n_patches(cfg)
    if P == 1:
        return 0.0, 2.0 * np.pi
    D = np.pi / P + cfg["band"]["overlap"]
    return 2.0 * np.pi * p / P - D, 2.0 * D


def _wrap(a):
    """Angle difference wrapped to (-pi, pi]."""
    return np.pi - np.mod(np.pi - a, 2.0 * np.pi)


def tangential_pou(theta, cfg, p):
    """omega_p(theta) of the tangential partition of unity (1 for P = 1)."""
    P = n_patches(cfg)
    if P == 1:
        return np.ones_like(np.asarray(theta, dtype=np.float64))
    delta = cfg["band"]["overlap"]
    D = np.pi / P + delta
    bumps = [smooth_step((D - np.abs(_wrap(theta - 2.0 * np.pi * q / P))) / (2.0 * delta)) for q in range(P)]
    return bumps[p] / np.sum(bumps, axis=0)


def band_map(t1, t2, cfg, p=0):
    """Boundary-patch parametrisation xi(t1, t2) -> physical point."""
    b = cfg["band"]
    th0, span = patch_frame(cfg, p)
    th = th0 + span * t1
    s = 1.0 - (1.0 - b["s_in"]) * t2
    R = radius(th, cfg["shape"])
    return np.stack([s * R * np.cos(th), s * R * np.sin(th)], axis=-1)


def band_jacobian(t1, t2, cfg, p=0):
    """|det d xi / d(t1,t2)| = span (1 - s_in) s R(theta)^2 with span = 2 pi
    for the periodic band (the R'(theta) term drops out of the cross
    product)."""
    b = cfg["band"]
    th0, span = patch_frame(cfg, p)
    th = th0 + span * t1
    s = 1.0 - (1.0 - b["s_in"]) * t2
    R = radius(th, cfg["shape"])
    return span * (1.0 - b["s_in"]) * s * R * R


def normalized_radius(x, shape):
    th = np.arctan2(x[..., 1], x[..., 0])
    return np.hypot(x[..., 0], x[..., 1]) / radius(th, shape), th


def omega_band(s, pou):
    return smooth_step((s - pou["s_a"]) / (pou["s_b"] - pou["s_a"]))


def band_coords(x, cfg, p=0):
    """Parameters of arbitrary points in boundary patch p, in grid units
    (v = t1 N1, u = t2 N2), and whether the point lies in the closed patch
    (s_in <= s <= 1 and, for P >= 2, inside the patch's theta range).  A
    transverse coordinate within 1e-9 grid units of a grid line is snapped
    onto it (reading of the multi-split rule for targets on grid lines)."""
    b = cfg["band"]
    s, th = normalized_radius(x, cfg["shape"])
    th0, span = patch_frame(cfg, p)
    if n_patches(cfg) == 1:
        v = np.mod(th / (2.0 * np.pi), 1.0) * b["N1"]
        v = np.where(v >= b["N1"], v - b["N1"], v)
        vin = np.ones(v.shape, bool)
    else:
        v = (_wrap(th - th0 - 0.5 * span) + 0.5 * span) / span * b["N1"]
        vin = (v >= 0.0) & (v <= b["N1"])
    u = (1.0 - s) / (1.0 - b["s_in"]) * b["N2"]
    ur = np.round(u)
    u = np.where(np.abs(u - ur) < 1e-9, ur, u)
    inside = (u >= 0.0) & (u <= b["N2"]) & vin
    return v, u, inside


def discretize(cfg, n2_fn):
    """All Nystrom nodes with their weights.

    n2_fn(x (n,2), on_boundary (n,) bool) -> n^2 (n,); at boundary nodes it
    returns the interior limit.
    Returns a dict of arrays; 'key' = (chart, i1, i2) identifies each node
    (chart 0: interior lattice, chart 1 + p: boundary patch p).  'vp', 'inp'
    (P x N): every point's t1 grid coordinate in each boundary patch and
    whether it lies in that patch; 'u': its t2 grid coordinate (the same in
    every patch); 'in_band': in any boundary patch.
    """
    h = cfg["h"]
    shape, b, pou = cfg["shape"], cfg["band"], cfg["pou"]
    if not (b["s_in"] <= pou["s_a"] < pou["s_b"] < 1.0):
        raise ValueError("need s_in <= s_a < s_b < 1")
    P = n_patches(cfg)
    Rmax = 1.0 + abs(shape["a"])
    imax = int(np.ceil(pou["s_b"] * Rmax / h)) + 1
    ii = np.arange(-imax, imax + 1)
    I1, I2 = np.meshgrid(ii, ii, indexing="ij")
    I1, I2 = I1.ravel(), I2.ravel()
    xi = np.stack([I1 * h, I2 * h], axis=-1)
    s_i, _ = normalized_radius(xi, shape)
    om_i = 1.0 - omega_band(s_i, pou)
    keep = om_i > 0.0
    I1, I2, xi, om_i = I1[keep], I2[keep], xi[keep], om_i[keep]
    n_int = xi.shape[0]

    N1, N2 = b["N1"], b["N2"]
    nc_all = composite_newton_cotes(N2, cfg["Q"])
    parts = []
    for p in range(P):
        n1 = N1 if P == 1 else N1 + 1             # periodic: i1 = N1 is i1 = 0
        J1, J2 = np.meshgrid(np.arange(n1), np.arange(N2 + 1), indexing="ij")
        J1, J2 = J1.ravel(), J2.ravel()
        t1, t2 = J1 / N1, J2 / N2
        th0, span = patch_frame(cfg, p)
        om_t = tangential_pou(th0 + span * t1, cfg, p)
        sb = 1.0 - (1.0 - b["s_in"]) * t2
        om = omega_band(sb, pou) * om_t
        kp = om_t > 0.0
        J1, J2, t1, t2, om = J1[kp], J2[kp], t1[kp], t2[kp], om[kp]
        parts.append(dict(p=p, J1=J1, J2=J2, x=band_map(t1, t2, cfg, p), om=om,
                          jac=band_jacobian(t1, t2, cfg, p), nc=nc_all[J2]))
    xb = np.concatenate([q["x"] for q in parts])
    J1 = np.concatenate([q["J1"] for q in parts])
    J2 = np.concatenate([q["J2"] for q in parts])
    om_b = np.concatenate([q["om"] for q in parts])
    jac = np.concatenate([q["jac"] for q in parts])
    nc = np.concatenate([q["nc"] for q in parts])
    pb = np.concatenate([np.full(q["J1"].size, q["p"]) for q in parts])
    nb = xb.shape[0]

    x = np.concatenate([xi, xb])
    on_bdry = np.concatenate([np.zeros(n_int, bool), J2 == 0])
    m = 1.0 - n2_fn(x, on_bdry)
    chart = np.concatenate([np.zeros(n_int, np.int64), 1 + pb])
    key = np.stack([chart, np.concatenate([I1, J1]), np.concatenate([I2, J2])], axis=-1)
    omega = np.concatenate([om_i, om_b])
    # plain quadrature weight (physical area element): trapezoid x composite
    # Newton-Cotes in the patch parameters (the end nodes of non-periodic
    # patches carry omega = 0 and are not unknowns, so every kept node has
    # the interior trapezoid weight 1/N1)
    w = np.concatenate([np.full(n_int, h * h), nc * jac / (N1 * N2)])
    # weight turning u_j into the density that the singular rules interpolate:
    # interior patch (physical polar rule): m*omega ; boundary patch
    # (parametric rule): m*omega*J
    dens = np.concatenate([m[:n_int] * om_i, m[n_int:] * om_b * jac])
    vp = np.empty((P, x.shape[0]))
    inp = np.empty((P, x.shape[0]), bool)
    u = None
    for p in range(P):
        v, u, inb = band_coords(x, cfg, p)
        own = np.concatenate([np.zeros(n_int, bool), pb == p])
        # boundary-patch nodes carry their exact grid coordinates
        v[own] = J1[pb == p]
        inb[own] = True
        vp[p], inp[p] = v, inb
    u = u.copy()
    u[n_int:] = J2
    return {
        "key": key, "x": x, "chart": chart, "omega": omega, "m": m, "w": w,
        "c": w * omega * m, "dens": dens, "v": vp[0], "vp": vp, "u": u, "inp": inp,
        "in_band": inp.any(axis=0), "n_int": n_int, "imax": imax, "n_band": nb,
    }


def lattice_index(pts):
    """Dense map lattice (i1, i2) -> point index (-1 where no node)."""
    imax = pts["imax"]
    n = 2 * imax + 1
    idx = -np.ones((n, n), np.int64)
    k = pts["key"][: pts["n_int"]]
    idx[k[:, 1] + imax, k[:, 2] + imax] = np.arange(pts["n_int"])
    return idx


def band_index(pts, cfg):
    """Per boundary patch, the map grid (i1, i2) -> point index (-1 for grid
    nodes that are not unknowns)."""
    b = cfg["band"]
    P = n_patches(cfg)
    out = []
    n1 = b["N1"] if P == 1 else b["N1"] + 1
    for p in range(P):
        sel = np.nonzero(pts["chart"] == 1 + p)[0]
        k = pts["key"][sel]
        idx = -np.ones((n1, b["N2"] + 1), np.int64)
        idx[k[:, 1], k[:, 2]] = sel
        out.append(idx)
    return out
