"""Pins of the 3-D face-lattice convolution oracle (oracle/conv3d.py) on the
CPU: the kernels against independent definitions (spherical Hankel
function, finite differences, the Helmholtz equation), the lattice sum
against an explicit loop, and the symmetries a transposed axis or a wrong
sign would break."""
import numpy as np
from scipy import special

from oracle.conv3d import conv3d, conv3d_at, dipole3d, green3d

KAPPA = 7.3


def test_green3d_is_the_spherical_hankel_form():
    r = np.linspace(0.05, 3.0, 37)
    h0 = special.spherical_jn(0, KAPPA * r) + 1j * special.spherical_yn(0, KAPPA * r)
    ref = 1j * KAPPA / (4 * np.pi) * h0
    assert np.abs(green3d(KAPPA, r) - ref).max() / np.abs(ref).max() < 1e-13


def test_green3d_solves_helmholtz_away_from_the_source():
    x0, h = np.array([0.7, -0.4, 0.9]), 1e-3
    f = lambda p: green3d(KAPPA, np.linalg.norm(p))
    lap = sum(f(x0 + h * e) + f(x0 - h * e) - 2 * f(x0) for e in np.eye(3)) / h ** 2
    assert abs(lap + KAPPA ** 2 * f(x0)) < 1e-4 * abs(KAPPA ** 2 * f(x0))


def test_dipole_is_the_source_derivative():
    x, y, h = np.array([0.3, 0.8, -0.2]), np.array([-0.1, 0.2, 0.4]), 1e-5
    e = np.array([1.0, 0.0, 0.0])
    fd = (green3d(KAPPA, np.linalg.norm(x - y - h * e)) - green3d(KAPPA, np.linalg.norm(x - y + h * e))) / (2 * h)
    d = x - y
    assert abs(dipole3d(KAPPA, d[0], np.linalg.norm(d)) - fd) < 1e-7 * abs(fd)


def test_lattice_sum_against_explicit_loop():
    rng = np.random.default_rng(11)
    na, nb, nc, hn, ht = 2, 3, 2, 0.25, 0.0625
    sm = rng.standard_normal((na, nb, nc)) + 1j * rng.standard_normal((na, nb, nc))
    sd = rng.standard_normal((na, nb, nc)) + 1j * rng.standard_normal((na, nb, nc))
    F = conv3d(sm, sd, hn, ht, KAPPA)
    for a in range(na):
        for b in range(nb):
            for c in range(nc):
                acc = 0j
                for a2 in range(na):
                    for b2 in range(nb):
                        for c2 in range(nc):
                            if (a, b, c) == (a2, b2, c2):
                                continue
                            dn, d1, d2 = (a - a2) * hn, (b - b2) * ht, (c - c2) * ht
                            r = (dn * dn + d1 * d1 + d2 * d2) ** 0.5
                            g = np.exp(1j * KAPPA * r) / (4 * np.pi * r)
                            gp = g * (1j * KAPPA * r - 1) / r          # dG/dr
                            acc += g * sm[a2, b2, c2] - gp * dn / r * sd[a2, b2, c2]
                assert abs(F[a, b, c] - acc) < 1e-12 * abs(acc)


def test_reciprocity_and_dipole_antisymmetry():
    na, nb, nc, hn, ht = 3, 4, 5, 0.3, 0.1
    z = np.zeros((na, nb, nc), complex)
    p, q = (0, 1, 3), (2, 3, 0)
    dp, dq = z.copy(), z.copy()
    dp[p], dq[q] = 1.0, 1.0
    # monopole: the response at q to a unit source at p equals the reverse
    assert abs(conv3d_at(dp, z, hn, ht, KAPPA, [q])[0] - conv3d_at(dq, z, hn, ht, KAPPA, [p])[0]) < 1e-15
    # dipole along the normal axis: odd under exchange; zero within a normal plane
    a = conv3d_at(z, dp, hn, ht, KAPPA, [q])[0]
    b = conv3d_at(z, dq, hn, ht, KAPPA, [p])[0]
    assert abs(a + b) < 1e-14 * abs(a) and abs(a) > 0
    s = (0, 3, 1)
    assert abs(conv3d_at(z, dp, hn, ht, KAPPA, [s])[0]) < 1e-15


def test_translation_invariance():
    rng = np.random.default_rng(3)
    na, nb, nc, hn, ht = 3, 6, 5, 0.2, 0.05
    sm = np.zeros((na, nb, nc), complex)
    sd = np.zeros((na, nb, nc), complex)
    sm[0, 1:3, 1:3] = rng.standard_normal((2, 2))
    sd[0, 1:3, 1:3] = rng.standard_normal((2, 2))
    sm2, sd2 = np.roll(sm, (1, 2, 1), axis=(0, 1, 2)), np.roll(sd, (1, 2, 1), axis=(0, 1, 2))
    f1 = conv3d_at(sm, sd, hn, ht, KAPPA, [(1, 2, 2)])[0]
    f2 = conv3d_at(sm2, sd2, hn, ht, KAPPA, [(2, 4, 3)])[0]
    assert abs(f1 - f2) < 1e-14 * abs(f1)
