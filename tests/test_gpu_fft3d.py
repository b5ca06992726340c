"""GPU parity of the dense 3-D complex FFT (ls_fft3d_*): ragged smooth sizes
against numpy's FFT in double precision (pinned to the DFT sum in
test_fft_reference.py), the 256^3 cube of the sphere workload's
equivalent-source grid, the round trip, and argument checks."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _cplx(rng, shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2)


def _run(f, a, direction):
    import torch
    t = torch.tensor(a, dtype=torch.complex64, device="cuda")
    f.exec(t, direction)
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(complex)


@pytest.mark.parametrize("shape", [(4, 6, 10), (16, 9, 25), (1, 1, 9), (8, 250, 3), (45, 2, 96), (3, 5, 2048)])
def test_forward_and_inverse_against_numpy(shape):
    from paper_1509_05063_amd import binding
    rng = np.random.default_rng(sum(shape))
    a = _cplx(rng, shape)
    f = binding.FFT3D(*shape)
    try:
        fw = _run(f, a, 1)
        inv = _run(f, a, -1)
    finally:
        f.close()
    ref = np.fft.fftn(a)
    ref_inv = np.fft.ifftn(a) * a.size
    e1 = np.linalg.norm(fw - ref) / np.linalg.norm(ref)
    e2 = np.linalg.norm(inv - ref_inv) / np.linalg.norm(ref_inv)
    print(f"{shape}: forward rel err {e1:.2e}, inverse {e2:.2e}", flush=True)
    assert e1 < 2e-6 and e2 < 2e-6


def test_cube_256():
    import torch
    from paper_1509_05063_amd import binding
    rng = np.random.default_rng(256)
    a = _cplx(rng, (256, 256, 256)).astype(np.complex64)
    f = binding.FFT3D(256, 256, 256)
    try:
        t = torch.tensor(a, device="cuda")
        f.exec(t, 1)
        torch.cuda.synchronize()
        fw = t.cpu().numpy().astype(complex)
        f.exec(t, -1)
        torch.cuda.synchronize()
        back = t.cpu().numpy().astype(complex) / a.size
    finally:
        f.close()
    ref = np.fft.fftn(a.astype(complex))
    e1 = np.linalg.norm(fw - ref) / np.linalg.norm(ref)
    e2 = np.linalg.norm(back - a) / np.linalg.norm(a)
    print(f"256^3: forward rel err {e1:.2e}, round trip {e2:.2e}", flush=True)
    assert e1 < 2e-6 and e2 < 2e-6


def test_bad_arguments():
    from paper_1509_05063_amd import binding
    for shape in [(0, 4, 4), (7, 4, 4), (4, 4, 4096), (4, 2000, 4), (1024, 4, 4)]:
        with pytest.raises(binding.LSError):
            binding.FFT3D(*shape)
    import torch
    f = binding.FFT3D(4, 4, 4)
    try:
        t = torch.zeros((4, 4, 4), dtype=torch.complex64, device="cuda")
        with pytest.raises(binding.LSError):
            f.exec(t, 0)
    finally:
        f.close()
