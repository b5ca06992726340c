"""ls_apply_noalloc (the apply that takes its workspace from the library's
static device scratch instead of a caller buffer) against ls_apply, through
the C ABI, on two calls in a row, the second with a smaller input; and the
rejection of an apply that needs more scratch than the array holds."""
import ctypes as C

import numpy as np
import pytest

from paper_1509_05063_amd.inputs import config, n2_function, plane_wave, random_density

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def disc_op():
    import torch
    from paper_1509_05063_amd import binding
    assert torch.cuda.is_available()
    cfg = config("disc_k2pi")
    op = binding.Operator(cfg, n2_function(cfg))
    yield cfg, op
    op.close()


@pytest.mark.parametrize("cdt", ["complex128", "complex64"])
def test_noalloc_apply_equals_apply_twice_second_smaller(disc_op, cdt):
    import torch
    cfg, op = disc_op
    dt = getattr(torch, cdt)
    xy, key = op.points()
    for nrhs in (5, 2):                    # the second call smaller than the first
        U = torch.tensor(np.stack([random_density(key, seed=40 + r) for r in range(nrhs)]), dtype=dt,
                         device="cuda")
        V_ref, V_na = torch.full_like(U, float("nan")), torch.full_like(U, float("nan"))
        op.apply(U, V_ref)
        op.apply_noalloc(U, V_na)
        torch.cuda.synchronize()
        print(f"{cdt} nrhs {nrhs}: max |diff| {(V_ref - V_na).abs().max().item():.3e}", flush=True)
        assert torch.equal(V_ref, V_na), nrhs


def test_noalloc_apply_single_vector_plane_wave(disc_op):
    import torch
    cfg, op = disc_op
    xy, _ = op.points()
    u = torch.tensor(plane_wave(cfg, xy, 0.9), dtype=torch.complex128, device="cuda")
    v0, v1 = torch.empty_like(u), torch.empty_like(u)
    op.apply(u, v0)
    op.apply_noalloc(u, v1)
    torch.cuda.synchronize()
    assert torch.equal(v0, v1)


def test_noalloc_rejects_more_than_the_scratch(disc_op):
    import torch
    from paper_1509_05063_amd import binding
    cfg, op = disc_op
    cap = C.c_size_t()
    binding._check(binding.lib().ls_noalloc_scratch_bytes(C.byref(cap)), "ls_noalloc_scratch_bytes")
    per = op.workspace_bytes(1, binding.LS_C128)
    nrhs = cap.value // per + 2
    assert op.workspace_bytes(nrhs, binding.LS_C128) > cap.value
    U = torch.zeros((nrhs, op.N), dtype=torch.complex128, device="cuda")
    V = torch.empty_like(U)
    with pytest.raises(binding.LSError) as ei:
        op.apply_noalloc(U, V)
    assert ei.value.status == binding.LS_EINVAL and "scratch" in str(ei.value)
