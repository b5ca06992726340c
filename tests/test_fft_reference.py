"""The double-precision reference of the dense 3-D FFT's GPU test, numpy's
fftn, against the definition of the 3-D DFT summed term by term on tiny
ragged arrays (a wrong sign, axis or normalisation fails it)."""
import numpy as np


def _dft3(a, sign):
    out = np.zeros(a.shape, complex)
    for k in np.ndindex(a.shape):
        acc = 0j
        for x in np.ndindex(a.shape):
            acc += a[x] * np.exp(sign * 2j * np.pi * sum(k[d] * x[d] / a.shape[d] for d in range(3)))
        out[k] = acc
    return out


def test_numpy_fftn_is_the_dft_sum():
    rng = np.random.default_rng(3)
    for shape in [(2, 3, 5), (1, 4, 3), (3, 1, 2)]:
        a = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
        assert np.abs(np.fft.fftn(a) - _dft3(a, -1)).max() < 1e-12
        assert np.abs(np.fft.ifftn(a) * a.size - _dft3(a, 1)).max() < 1e-12
