"""CPU checks of three facts the transform kernels rely on.

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
3. The index map of the register-first two-pass transforms (radix R1 then
   radix R2, intermediate rows j R1 + m, twiddles W^(j m)) is the DFT, for
   the 16 x 16 and 12 x 6 splits the kernels instantiate and the reverse
   order.
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


def _two_pass(x, R1, R2, sign):
    """The index map of the register-first two-pass kernels: pass 1
    (radix R1) butterfly j < R2 takes rows j + m R2 and leaves its outputs at
    intermediate rows j R1 + m; pass 2 (radix R2) butterfly j < R1 takes
    rows j + m R1, multiplies entry m by W_n^(j m), and writes rows
    j + m R1 of the result."""
    n = R1 * R2
    w = np.exp(sign * 2j * np.pi * np.arange(n) / n)
    mid = np.empty(n, complex)
    for j in range(R2):
        v = x[[j + m * R2 for m in range(R1)]]
        f = np.array([sum(v[a] * np.exp(sign * 2j * np.pi * a * b / R1) for a in range(R1)) for b in range(R1)])
        mid[[j * R1 + m for m in range(R1)]] = f
    out = np.empty(n, complex)
    for j in range(R1):
        v = mid[[j + m * R1 for m in range(R2)]] * w[[j * m for m in range(R2)]]
        f = np.array([sum(v[a] * np.exp(sign * 2j * np.pi * a * b / R2) for a in range(R2)) for b in range(R2)])
        out[[j + m * R1 for m in range(R2)]] = f
    return out


def test_two_pass_index_map_is_the_dft():
    rng = np.random.default_rng(5)
    for R1, R2 in [(16, 16), (12, 6), (6, 12)]:
        x = rng.standard_normal(R1 * R2) + 1j * rng.standard_normal(R1 * R2)
        assert np.abs(_two_pass(x, R1, R2, -1) - np.fft.fft(x)).max() < 1e-9
        assert np.abs(_two_pass(x, R1, R2, 1) - np.fft.ifft(x) * x.size).max() < 1e-9
