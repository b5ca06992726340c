"""Closed forms used to pin the oracle (test infrastructure only).

* Mie (separation of variables) series for a plane wave scattered by a disc /
  ball of constant refractive index n (the exact solution the paper compares
  with in its disc and sphere examples).  Derived from continuity of u and
  du/dr at r = R; Bessel routines from scipy.
* Volume potential of a constant density over a disc / ball:
  v(x) = int_{|y|<R} G(x - y) dy solves (Delta + kappa^2) v = -1 inside,
  radiates outside and is C^1, which gives
  2-D: v = (i pi R / (2 kappa)) H1(kappa R) J0(kappa |x|) - 1/kappa^2,
  3-D: v = i R^2 h1(kappa R) j0(kappa |x|) - 1/kappa^2      (|x| < R).
"""
import numpy as np
from scipy import special


def volume_potential_disc(kappa, R, x):
    r = np.hypot(x[..., 0], x[..., 1])
    return (1j * np.pi * R / (2 * kappa)) * special.hankel1(1, kappa * R) * special.j0(kappa * r) \
        - 1.0 / kappa ** 2


def _sph_h1(n, z, derivative=False):
    return special.spherical_jn(n, z, derivative) + 1j * special.spherical_yn(n, z, derivative)


def volume_potential_ball(kappa, R, x):
    r = np.sqrt(np.sum(x * x, axis=-1))
    return 1j * R ** 2 * _sph_h1(1, kappa * R) * special.spherical_jn(0, kappa * r) - 1.0 / kappa ** 2


def mie2d_coeffs(kappa, n, R, mmax):
    """Interior a_m and exterior b_m for the incident field
    exp(i kappa r cos(theta - alpha)) = sum_m i^m J_m(kappa r) e^{i m (theta - alpha)}."""
    m = np.arange(-mmax, mmax + 1)
    k1 = kappa * n
    J1 = special.jv(m, k1 * R)
    J1p = special.jvp(m, k1 * R)
    J0 = special.jv(m, kappa * R)
    H = special.hankel1(m, kappa * R)
    Hp = special.h1vp(m, kappa * R)
    im = 1j ** (m % 4)
    a = im * (2j / (np.pi * kappa * R)) / (J1 * Hp - n * J1p * H)
    b = (a * J1 - im * J0) / H
    return m, a, b


def mie2d_total(kappa, n, R, x, alpha=0.0, mmax=None):
    """Total field at points x (..., 2) for incidence direction angle alpha."""
    if mmax is None:
        mmax = int(kappa * max(n, 1.0) * R + 40)
    m, a, b = mie2d_coeffs(kappa, n, R, mmax)
    r = np.hypot(x[..., 0], x[..., 1])
    th = np.arctan2(x[..., 1], x[..., 0])
    ph = np.exp(1j * np.multiply.outer(th - alpha, m))
    inside = r < R
    out = np.zeros(r.shape, complex)
    ri = r[inside]
    out[inside] = np.sum(a * special.jv(m, kappa * n * ri[..., None]) * ph[inside], axis=-1)
    ro = r[~inside]
    inc = np.exp(1j * kappa * (x[~inside][..., 0] * np.cos(alpha) + x[~inside][..., 1] * np.sin(alpha)))
    out[~inside] = inc + np.sum(b * special.hankel1(m, kappa * ro[..., None]) * ph[~inside], axis=-1)
    return out


def mie3d_coeffs(kappa, n, R, lmax):
    """Interior a_l for incidence exp(i kappa z) = sum (2l+1) i^l j_l P_l(cos)."""
    l = np.arange(lmax + 1)
    k1 = kappa * n
    j1 = special.spherical_jn(l, k1 * R)
    j1p = special.spherical_jn(l, k1 * R, True)
    j0 = special.spherical_jn(l, kappa * R)
    j0p = special.spherical_jn(l, kappa * R, True)
    h = _sph_h1(l, kappa * R)
    hp = _sph_h1(l, kappa * R, True)
    c = (2 * l + 1) * 1j ** (l % 4)
    # continuity of u and du/dr:  a j1 = c j0 + b h ;  a k1 j1' = c kappa j0' + b kappa h'
    a = c * (j0p * h - j0 * hp) * kappa / (k1 * j1p * h - kappa * j1 * hp)
    b = (a * j1 - c * j0) / h
    return l, a, b


def mie3d_total(kappa, n, R, x, lmax=None):
    if lmax is None:
        lmax = int(kappa * max(n, 1.0) * R + 40)
    l, a, b = mie3d_coeffs(kappa, n, R, lmax)
    r = np.sqrt(np.sum(x * x, axis=-1))
    ct = np.where(r > 0, x[..., 2] / np.where(r > 0, r, 1.0), 1.0)
    Pl = np.stack([special.eval_legendre(k, ct) for k in l], axis=-1)
    inside = r < R
    out = np.zeros(r.shape, complex)
    out[inside] = np.sum(a * special.spherical_jn(l, kappa * n * r[inside][..., None]) * Pl[inside], -1)
    ro = r[~inside]
    out[~inside] = np.exp(1j * kappa * x[~inside][..., 2]) + np.sum(
        b * _sph_h1(l, kappa * ro[..., None]) * Pl[~inside], -1)
    return out
