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

Partition of unity (not given in the paper; reading recorded in the design doc):
omega_b(x) = smooth_step((s - s_a)/(s_b - s_a)), omega_int = 1 - omega_b.
Interior lattice nodes with omega_int = 0 are not unknowns.
"""
import numpy as np

from .quad import composite_newton_cotes, smooth_step


def radius(theta, shape):
    return 1.0 + shape["a"] * np.cos(shape["k"] * theta)


def band_map(t1, t2, cfg):
    """Boundary-patch parametrisation xi(t1, t2) -> physical point."""
    b = cfg["band"]
    th = 2.0 * np.pi * t1
    s = 1.0 - (1.0 - b["s_in"]) * t2
    R = radius(th, cfg["shape"])
    return np.stack([s * R * np.cos(th), s * R * np.sin(th)], axis=-1)


def band_jacobian(t1, t2, cfg):
    """|det d xi / d(t1,t2)| = 2 pi (1 - s_in) s R(theta)^2 (the R'(theta)
    term drops out of the cross product)."""
    b = cfg["band"]
    th = 2.0 * np.pi * t1
    s = 1.0 - (1.0 - b["s_in"]) * t2
    R = radius(th, cfg["shape"])
    return 2.0 * np.pi * (1.0 - b["s_in"]) * s * R * R


def normalized_radius(x, shape):
    th = np.arctan2(x[..., 1], x[..., 0])
    return np.hypot(x[..., 0], x[..., 1]) / radius(th, shape), th


def omega_band(s, pou):
    return smooth_step((s - pou["s_a"]) / (pou["s_b"] - pou["s_a"]))


def band_coords(x, cfg):
    """Boundary-patch parameters of arbitrary points, in grid units
    (v = t1 N1 in [0, N1), u = t2 N2), and whether the point lies in the
    closed patch (s_in <= s <= 1).  A transverse coordinate within 1e-9 grid
    units of a grid line is snapped onto it (reading of the multi-split rule
    for targets on grid lines)."""
    b = cfg["band"]
    s, th = normalized_radius(x, cfg["shape"])
    v = np.mod(th / (2.0 * np.pi), 1.0) * b["N1"]
    v = np.where(v >= b["N1"], v - b["N1"], v)
    u = (1.0 - s) / (1.0 - b["s_in"]) * b["N2"]
    ur = np.round(u)
    u = np.where(np.abs(u - ur) < 1e-9, ur, u)
    inside = (u >= 0.0) & (u <= b["N2"])
    return v, u, inside


def discretize(cfg, n2_fn):
    """All Nyström nodes with their weights.

    n2_fn(x (n,2), on_boundary (n,) bool) -> n^2 (n,); at boundary nodes it
    returns the interior limit.
    Returns a dict of arrays; 'key' = (chart, i1, i2) identifies each node.
    """
    h = cfg["h"]
    shape, b, pou = cfg["shape"], cfg["band"], cfg["pou"]
    if not (b["s_in"] <= pou["s_a"] < pou["s_b"] < 1.0):
        raise ValueError("need s_in <= s_a < s_b < 1")
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
    J1, J2 = np.meshgrid(np.arange(N1), np.arange(N2 + 1), indexing="ij")
    J1, J2 = J1.ravel(), J2.ravel()
    t1, t2 = J1 / N1, J2 / N2
    xb = band_map(t1, t2, cfg)
    sb = 1.0 - (1.0 - b["s_in"]) * t2
    om_b = omega_band(sb, pou)
    jac = band_jacobian(t1, t2, cfg)
    nc = composite_newton_cotes(N2, cfg["Q"])[J2]

    x = np.concatenate([xi, xb])
    on_bdry = np.concatenate([np.zeros(n_int, bool), J2 == 0])
    m = 1.0 - n2_fn(x, on_bdry)
    chart = np.concatenate([np.zeros(n_int, np.int64), np.ones(N1 * (N2 + 1), np.int64)])
    key = np.stack([chart, np.concatenate([I1, J1]), np.concatenate([I2, J2])], axis=-1)
    omega = np.concatenate([om_i, om_b])
    # plain quadrature weight (physical area element)
    w = np.concatenate([np.full(n_int, h * h), nc * jac / (N1 * N2)])
    # weight turning u_j into the density that the singular rules interpolate:
    # interior patch (physical polar rule): m*omega ; boundary patch
    # (parametric rule): m*omega*J
    dens = np.concatenate([m[:n_int] * om_i, m[n_int:] * om_b * jac])
    v, u, inb = band_coords(x, cfg)
    # boundary-patch nodes carry their exact grid coordinates
    v[n_int:] = J1
    u[n_int:] = J2
    inb[n_int:] = True
    return {
        "key": key, "x": x, "chart": chart, "omega": omega, "m": m, "w": w,
        "c": w * omega * m, "dens": dens, "v": v, "u": u, "in_band": inb,
        "n_int": n_int, "imax": imax,
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
    """Map boundary-patch grid (i1, i2) -> point index."""
    b = cfg["band"]
    k = pts["key"][pts["n_int"]:]
    idx = -np.ones((b["N1"], b["N2"] + 1), np.int64)
    idx[k[:, 1], k[:, 2]] = pts["n_int"] + np.arange(k.shape[0])
    return idx
