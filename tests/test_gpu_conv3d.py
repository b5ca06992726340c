"""GPU parity of the 3-D face-lattice convolution (ls_conv3d_*, the FFT step
of the 3-D method) against the oracle's direct sum: every node of small
ragged lattices (default schedule), sampled nodes at the sphere workload's
lattice shape (33 x 128 x 128 per set, three sets) under the autotuned
schedule and under every candidate schedule, and the edge cases."""
import numpy as np
import pytest

from oracle.conv3d import conv3d, conv3d_at

pytestmark = pytest.mark.gpu


def _sigma(rng, nsets, na, nb, nc):
    return (rng.standard_normal((nsets, 2, na, nb, nc)) + 1j * rng.standard_normal((nsets, 2, na, nb, nc))) / np.sqrt(2)


def _run(c, sig):
    import torch
    sd = torch.tensor(sig, dtype=torch.complex64, device="cuda")
    fd = torch.empty(sig.shape[:1] + sig.shape[2:], dtype=torch.complex64, device="cuda")
    c.apply(sd, fd)
    torch.cuda.synchronize()
    return fd.cpu().numpy().astype(complex)


@pytest.mark.parametrize("na,nb,nc,hn,ht,kappa", [(4, 9, 7, 0.25, 0.0625, 8.0), (1, 5, 3, 0.5, 0.1, 3.0),
                                                  (6, 4, 11, 0.1, 0.05, 25.0), (2, 5, 300, 0.3, 0.01, 10.0)])
def test_every_node_against_direct_sum(na, nb, nc, hn, ht, kappa):
    from paper_1509_05063_amd import binding
    rng = np.random.default_rng(1509 + na * 100 + nb)
    nsets = 2
    sig = _sigma(rng, nsets, na, nb, nc)
    c = binding.Conv3D(na, nb, nc, hn, ht, kappa, nsets)
    try:
        F = _run(c, sig)
    finally:
        c.close()
    for s in range(nsets):
        ref = conv3d(sig[s, 0], sig[s, 1], hn, ht, kappa)
        err = np.abs(F[s] - ref).max() / np.abs(ref).max()
        print(f"{na}x{nb}x{nc} set {s}: max rel err {err:.2e}", flush=True)
        assert err < 2e-5


def test_sphere_lattice_shape_sampled_nodes():
    """Sphere workload (kappa = 8 pi, h = 1/64, cells H = 4h, q = 4 nodes per
    face edge): set lattices of 33 x 128 x 128 nodes, hn = H, ht = H / 4."""
    from paper_1509_05063_amd import binding
    H = 4 / 64
    na, nb, nc, hn, ht, kappa = 33, 128, 128, H, H / 4, 8 * np.pi
    rng = np.random.default_rng(2025)
    sig = _sigma(rng, 3, na, nb, nc)
    c = binding.Conv3D(na, nb, nc, hn, ht, kappa, 3)
    try:
        assert c.padded == (72, 256, 256)
        sched = c.autotune()
        print(f"sphere lattice schedule {sched}", flush=True)
        F = _run(c, sig)
    finally:
        c.close()
    pick = [(0, 0, 0), (na - 1, nb - 1, nc - 1), (16, 64, 64), (0, 127, 3), (32, 5, 120), (7, 77, 31)]
    for s in range(3):
        ref = conv3d_at(sig[s, 0], sig[s, 1], hn, ht, kappa, pick)
        got = np.array([F[s][p] for p in pick])
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        print(f"sphere lattice set {s}: sampled rel err {err:.2e}", flush=True)
        assert err < 1e-4


def test_every_schedule_sphere_lattice():
    """Every candidate schedule (tiles that leave partial last tiles, both
    thread counts, product entries past the prefetched ones) gives the
    oracle's values at sampled nodes of the sphere lattices."""
    from paper_1509_05063_amd import binding
    H = 4 / 64
    na, nb, nc, hn, ht, kappa = 33, 128, 128, H, H / 4, 8 * np.pi
    rng = np.random.default_rng(77)
    sig = _sigma(rng, 3, na, nb, nc)
    pick = [(0, 0, 0), (na - 1, nb - 1, nc - 1), (16, 64, 64), (3, 100, 7)]
    ref = [conv3d_at(sig[s, 0], sig[s, 1], hn, ht, kappa, pick) for s in range(3)]
    c = binding.Conv3D(na, nb, nc, hn, ht, kappa, 3)
    try:
        for ta in (3, 4, 8, 16, 32, 64):
            for nth in (256, 512):
                for tb, sk in ((4, 0), (8, 32), (16, 512), (8, 7)):
                    c.set_schedule(ta, nth, tb, sk)
                    F = _run(c, sig)
                    err = max(np.linalg.norm(np.array([F[s][p] for p in pick]) - ref[s]) / np.linalg.norm(ref[s])
                              for s in range(3))
                    assert err < 1e-4, (ta, nth, tb, sk, err)
        print(f"every schedule: last sampled rel err {err:.2e}", flush=True)
        for bad in [(0, 256, 8), (16, 128, 8), (16, 256, 0), (128, 256, 8), (16, 256, 32), (16, 256, 8, -1),
                    (16, 256, 8, 513)]:
            with pytest.raises(binding.LSError):
                c.set_schedule(*bad)
    finally:
        c.close()


def test_zero_input_and_bad_arguments():
    from paper_1509_05063_amd import binding
    c = binding.Conv3D(3, 8, 8, 0.2, 0.05, 5.0, 1)
    try:
        F = _run(c, np.zeros((1, 2, 3, 8, 8), complex))
        assert not np.any(F)
    finally:
        c.close()
    for args in [(0, 8, 8, 0.2, 0.05, 5.0, 1), (3, 8, 8, -0.2, 0.05, 5.0, 1), (3, 8, 8, 0.2, 0.05, 0.0, 1),
                 (3, 400, 8, 0.2, 0.05, 5.0, 1), (3, 8, 8, 0.2, 0.05, 5.0, 2000)]:
        with pytest.raises(binding.LSError):
            binding.Conv3D(*args)
