"""CPU checks of two facts the transform kernels rely on.

1. Division by a run-time divisor d as q = floor(x m / 2^32) with
   m = floor((2^32 - 1) / d) + 1 is exact whenever x d < 2^32 (the FFT
   kernels' index arithmetic: x < 2^20, d < 2^12).  Checked at the worst
   cases of every divisor (x just below multiples of d, the largest x in
   range) and on random samples.
2. The spectra of the 3-D face-lattice kernels, laid out with wrapped
   offsets in the padded box, are even in every frequency axis for the
   monopole G and odd along the normal axis (even along the other two) for
   the dipole dG/dy_n, so one octant of each determines the rest (the fused
   normal-axis pass reads only that octant).  Built from the oracle's own
   kernel functions and numpy's FFT on small ragged lattices, odd and even
   padded sizes.
"""
import numpy as np

from oracle.conv3d import dipole3d, green3d


def _fastdiv(x, d):
    m = (0xFFFFFFFF // d) + 1
    return (x * m) >> 32


def test_multiply_high_division_is_exact_in_range():
    rng = np.random.default_rng(11)
    for d in range(1, 4096):
        xmax = min((1 << 20) - 1, ((1 << 32) - 1) // d)
        xs = {0, 1, d - 1, d, xmax, xmax - 1}
        k = xmax // d
        xs.update({k * d - 1, k * d, (k // 2) * d - 1 if k > 1 else 0})
        xs.update(int(v) for v in rng.integers(0, xmax + 1, 8))
        for x in xs:
            if x < 0:
                continue
            assert _fastdiv(x, d) == x // d, (x, d)


def test_multiply_high_division_fails_outside_range():
    # the bound matters: past it quotients go wrong (d = 7, m d - 2^32 = 3:
    # the first errors sit just above x = 2^32 / 3, far beyond x d = 2^32)
    d = 7
    x0 = (1 << 32) // 3
    bad = [x for x in range(x0, x0 + 1000) if _fastdiv(x, d) != x // d]
    assert bad and all(x * d >= (1 << 32) for x in bad)


def _kernel_lattices(na, nb, nc, hn, ht, kappa):
    Pa, Pb, Pc = 2 * na - 1 + 1, 2 * nb - 1, 2 * nc - 1 + 2   # even, odd, odd + 2 padded lengths
    G = np.zeros((Pa, Pb, Pc), complex)
    D = np.zeros((Pa, Pb, Pc), complex)
    for ia in range(Pa):
        da = ia if ia < na else ia - Pa
        if not -na < da < na:
            continue
        for ib in range(Pb):
            db = ib if ib < nb else ib - Pb
            if not -nb < db < nb:
                continue
            for ic in range(Pc):
                dc = ic if ic < nc else ic - Pc
                if not -nc < dc < nc or (da == 0 and db == 0 and dc == 0):
                    continue
                dn, d1, d2 = da * hn, db * ht, dc * ht
                r = np.sqrt(dn * dn + d1 * d1 + d2 * d2)
                G[ia, ib, ic] = green3d(kappa, r)
                D[ia, ib, ic] = dipole3d(kappa, dn, r)
    return G, D


def test_kernel_spectra_octant_symmetry():
    for na, nb, nc, hn, ht, kappa in [(3, 4, 5, 0.25, 0.0625, 8.0), (4, 3, 2, 0.1, 0.05, 20.0)]:
        G, D = _kernel_lattices(na, nb, nc, hn, ht, kappa)
        Gh, Dh = np.fft.fftn(G), np.fft.fftn(D)
        Pa, Pb, Pc = G.shape
        ka, kb, kc = np.meshgrid(np.arange(Pa), np.arange(Pb), np.arange(Pc), indexing="ij")
        ma, mb, mc = np.minimum(ka, Pa - ka), np.minimum(kb, Pb - kb), np.minimum(kc, Pc - kc)
        sign = np.where(ka > Pa - ka, -1.0, 1.0)
        scale = np.abs(Gh).max()
        assert np.abs(Gh - Gh[ma, mb, mc]).max() < 1e-12 * scale
        assert np.abs(Dh - sign * Dh[ma, mb, mc]).max() < 1e-12 * np.abs(Dh).max()
        # the dipole really is odd along the normal axis (not trivially even)
        assert np.abs(Dh - Dh[ma, mb, mc]).max() > 1e-3 * np.abs(Dh).max()
