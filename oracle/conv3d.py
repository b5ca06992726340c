"""Three-dimensional face-lattice convolution by direct summation.  TEST
INFRASTRUCTURE ONLY: used by tests/ alone, never by the library.

In three dimensions the accelerated far field (Sec. 3.2, equiv-conv-loc)
places the equivalent sources of every cell on the faces normal to one axis
per source set, so each set lives on a regular lattice: spacing hn along the
set's normal axis, ht along the two tangential axes.  The convolution step
of the method then computes, at every lattice node x,

    F(x) = sum over nodes y != x of  G(x - y) sigma_m(y) + D(x - y) sigma_d(y)

with the free-space Helmholtz Green's function G(r) = exp(i kappa r) / (4 pi r)
and the dipole kernel D = dG(|x - y|)/dy_n along the set's normal axis
(Delta = 0 excluded, the K(0) = 0 convention of the method).  The oracle sums
every pair directly; the library does the same convolution by zero-padded
FFTs.  Arrays are indexed [a][b][c] = (normal, tangential 1, tangential 2).
"""
import numpy as np


def green3d(kappa, r):
    """exp(i kappa r) / (4 pi r), r > 0."""
    return np.exp(1j * kappa * r) / (4 * np.pi * r)


def dipole3d(kappa, dn, r):
    """d/dy_n G(|x - y|) for d = x - y with normal component dn, r = |d| > 0:
    G'(r) * (-dn / r), G'(r) = exp(i kappa r) (i kappa r - 1) / (4 pi r^2)."""
    gp = np.exp(1j * kappa * r) * (1j * kappa * r - 1) / (4 * np.pi * r * r)
    return -gp * dn / r


def node_coords(na, nb, nc, hn, ht):
    a, b, c = np.meshgrid(np.arange(na), np.arange(nb), np.arange(nc), indexing="ij")
    return np.stack([a * hn, b * ht, c * ht], axis=-1).reshape(-1, 3)


def conv3d_at(sig_m, sig_d, hn, ht, kappa, targets):
    """F at the lattice nodes `targets` (array of (a, b, c) index triples)."""
    na, nb, nc = sig_m.shape
    y = node_coords(na, nb, nc, hn, ht)
    sm, sd = sig_m.reshape(-1), sig_d.reshape(-1)
    out = np.empty(len(targets), complex)
    for k, (a, b, c) in enumerate(targets):
        d = np.array([a * hn, b * ht, c * ht]) - y
        r = np.sqrt((d * d).sum(axis=1))
        m = r > 0
        out[k] = (green3d(kappa, r[m]) * sm[m]).sum() + (dipole3d(kappa, d[m, 0], r[m]) * sd[m]).sum()
    return out


def conv3d(sig_m, sig_d, hn, ht, kappa):
    """F at every node of the lattice (direct sum; small lattices only)."""
    na, nb, nc = sig_m.shape
    idx = np.stack(np.meshgrid(np.arange(na), np.arange(nb), np.arange(nc), indexing="ij"), axis=-1).reshape(-1, 3)
    return conv3d_at(sig_m, sig_d, hn, ht, kappa, idx).reshape(na, nb, nc)
