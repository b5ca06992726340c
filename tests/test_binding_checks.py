"""The Python binding validates every device vector before it crosses the C
ABI (the library cannot see a tensor's length or dtype, so a wrong one would
make the kernels read or write past the allocation).  CPU only: the checks
run before any device call."""
import pytest
import torch

from paper_1509_05063_amd.binding import check_vectors

N = 10
C128, C64 = (torch.complex128,), (torch.complex128, torch.complex64)


def test_accepts_matching_shapes_up_to_the_device_check():
    for t in (torch.zeros(N, dtype=torch.complex128), torch.zeros(3, N, dtype=torch.complex64)):
        with pytest.raises(ValueError, match="device"):
            check_vectors(t, N, C64, "u")


@pytest.mark.parametrize("t,dtypes,nrhs,msg", [
    (torch.zeros(N, dtype=torch.complex64), C128, None, "dtype"),          # solve takes complex128 only
    (torch.zeros(N, dtype=torch.float64), C64, None, "dtype"),             # real data
    (torch.zeros(2 * N, dtype=torch.float32).view(torch.complex64)[:N // 2], C64, None, "shape"),
    (torch.zeros(N + 1, dtype=torch.complex128), C64, None, "shape"),      # one value too many
    (torch.zeros(N, 3, dtype=torch.complex128).t(), C64, None, "contiguous"),
    (torch.zeros(2, N, dtype=torch.complex128), C64, 3, "vectors"),         # v with fewer vectors than u
    (torch.zeros(1, 1, N, dtype=torch.complex128), C64, None, "shape"),
    ("not a tensor", C64, None, "tensor"),
])
def test_rejects_bad_vectors(t, dtypes, nrhs, msg):
    with pytest.raises(ValueError, match=msg):
        check_vectors(t, N, dtypes, "u", nrhs)
