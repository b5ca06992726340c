"""GPU parity through the C ABI: the device apply and solve against the CPU
oracle on the same seeded inputs (disc workload, every row)."""
import math

import numpy as np
import pytest

from paper_1509_05063_amd.inputs import config, match_keys, n2_function, plane_wave, random_density

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def disc():
    import torch
    from oracle.op2d import Setup2D
    from paper_1509_05063_amd import binding
    assert torch.cuda.is_available()
    cfg = config("disc_k2pi")
    n2 = n2_function(cfg)
    op = binding.Operator(cfg, n2)
    orc = Setup2D(cfg, n2)
    xy, key = op.points()
    p = match_keys(orc.pts["key"], key)       # oracle index -> library index
    A = orc.dense_A()
    return cfg, op, orc, A, p, xy, key


def _to_lib(x_or, p, N):
    out = np.empty(N, complex)
    out[p] = x_or
    return out


def test_apply_fp64_matches_oracle_every_row(disc):
    import torch
    cfg, op, orc, A, p, xy, key = disc
    for name, u_or in [("random", random_density(orc.pts["key"])),
                       ("plane", plane_wave(cfg, orc.pts["x"], 0.0))]:
        v_or = A @ u_or
        u = torch.tensor(_to_lib(u_or, p, op.N), dtype=torch.complex128, device="cuda")
        v = torch.empty_like(u)
        op.apply(u, v)
        torch.cuda.synchronize()
        v_lib = v.cpu().numpy()[p]
        err = np.linalg.norm(v_lib - v_or) / np.linalg.norm(v_or)
        emax = np.abs(v_lib - v_or).max() / np.abs(v_or).max()
        print(f"apply fp64 {name}: rel2 {err:.3e} relmax {emax:.3e}", flush=True)
        assert err < 1e-8 and emax < 1e-8


def test_apply_fp32_close_to_oracle(disc):
    import torch
    cfg, op, orc, A, p, xy, key = disc
    u_or = random_density(orc.pts["key"])
    v_or = A @ u_or
    u = torch.tensor(_to_lib(u_or, p, op.N), dtype=torch.complex64, device="cuda")
    v = torch.empty_like(u)
    op.apply(u, v)
    torch.cuda.synchronize()
    v_lib = v.cpu().numpy().astype(complex)[p]
    err = np.linalg.norm(v_lib - v_or) / np.linalg.norm(v_or)
    print(f"apply fp32: rel2 {err:.3e}", flush=True)
    assert err < 1e-4


def test_multi_rhs_equals_single(disc):
    import torch
    cfg, op, orc, A, p, xy, key = disc
    U = torch.stack([torch.tensor(_to_lib(random_density(orc.pts["key"], seed=s), p, op.N),
                                  dtype=torch.complex128) for s in range(3)]).cuda()
    V = torch.empty_like(U)
    op.apply(U, V)
    for k in range(3):
        v1 = torch.empty_like(U[k])
        op.apply(U[k].contiguous(), v1)
        torch.cuda.synchronize()
        assert torch.equal(v1, V[k])


@pytest.mark.parametrize("cdt", ["complex128", "complex64"])
def test_batched_kernels_equal_single_applies(disc, cdt):
    """17 right-hand sides: the first 16 take the batched projection and
    interpolation kernels (16 right-hand sides per workgroup), the 17th a
    group of one; each result is bitwise that of its own single apply."""
    import torch
    cfg, op, orc, A, p, xy, key = disc
    dt = getattr(torch, cdt)
    U = torch.stack([torch.tensor(_to_lib(random_density(orc.pts["key"], seed=s), p, op.N), dtype=dt)
                     for s in range(17)]).cuda()
    V = torch.empty_like(U)
    op.apply(U, V)
    for k in (0, 7, 15, 16):
        v1 = torch.empty_like(U[k])
        op.apply(U[k].contiguous(), v1)
        torch.cuda.synchronize()
        assert torch.equal(v1, V[k]), k


def test_operator_without_tiles(disc):
    """skip_tiles: no dense tiles are kept (less device memory), the tuner
    does not offer them for batches, and applies are unchanged."""
    import torch
    from paper_1509_05063_amd import binding
    cfg, op, orc, A, p, xy, key = disc
    cfg2 = dict(cfg, skip_tiles=1)
    op2 = binding.Operator(cfg2, n2_function(cfg2))
    try:
        assert op2.stats()["tile_weights"] == 0 and op.stats()["tile_weights"] > 0
        assert op2.resident_bytes() < op.resident_bytes()
        ch = op2.autotune(16, binding.LS_C64)
        assert ch["csr_variant"] != 3
        U = torch.stack([torch.tensor(_to_lib(random_density(orc.pts["key"], seed=s), p, op.N),
                                      dtype=torch.complex128) for s in range(2)]).cuda()
        V1, V2 = torch.empty_like(U), torch.empty_like(U)
        op.apply(U, V1)
        op2.apply(U, V2)
        torch.cuda.synchronize()
        assert (torch.linalg.norm(V1 - V2) / torch.linalg.norm(V1)).item() < 1e-13
    finally:
        op2.close()


def test_apply_is_deterministic(disc):
    import torch
    cfg, op, orc, A, p, xy, key = disc
    u = torch.tensor(_to_lib(random_density(orc.pts["key"]), p, op.N), dtype=torch.complex128, device="cuda")
    v1, v2 = torch.empty_like(u), torch.empty_like(u)
    op.apply(u, v1)
    op.apply(u, v2)
    torch.cuda.synchronize()
    assert torch.equal(v1, v2)


@pytest.mark.parametrize("mode,ortho,restart", [(0, 0, 100), (1, 0, 100), (0, 1, 100), (1, 1, 100), (0, 0, 7),
                                                (1, 0, 7)])
def test_solve_matches_oracle_lu(disc, mode, ortho, restart):
    import torch
    from oracle.mie import mie2d_total
    cfg, op, orc, A, p, xy, key = disc
    f_or = plane_wave(cfg, orc.pts["x"], 0.0)
    u_or = np.linalg.solve(A, f_or)
    f = torch.tensor(_to_lib(f_or, p, op.N), dtype=torch.complex128, device="cuda")
    x = torch.empty_like(f)
    st = op.solve(f, x, tol=1e-10, restart=restart, max_iter=2000, mode=mode, inner_tol=1e-5, ortho=ortho)
    u = x.cpu().numpy()[p]
    err = np.linalg.norm(u - u_or) / np.linalg.norm(u_or)
    mie = mie2d_total(cfg["kappa"], 1.5, 1.0, orc.pts["x"] * (1 - 1e-15))
    emie = np.linalg.norm(u - mie) / np.linalg.norm(mie)
    print(f"solve mode {mode} ortho {ortho} restart {restart}: {st} vs LU {err:.3e} vs Mie {emie:.3e}", flush=True)
    assert err < 1e-8
    assert emie < 5e-3


def test_autotune_keeps_the_operator(disc):
    """The tuned schedules apply the same operator: every row still matches
    the oracle (FP64 to 1e-8, FP32 to 1e-4), and the choices are in range."""
    import torch
    from paper_1509_05063_amd import binding
    cfg, op, orc, A, p, xy, key = disc
    x_or = random_density(orc.pts["key"], seed=7)
    y_or = A @ x_or
    for prec, dt, tol in ((binding.LS_C128, torch.complex128, 1e-8), (binding.LS_C64, torch.complex64, 1e-4)):
        ch = op.autotune(nrhs=1, prec=prec)
        print(f"autotune prec {prec}: {ch}", flush=True)
        assert ch["fft_col_tile"] in (1, 2, 4, 8, 16, 32) and ch["near_variant"] in (0, 1, 2, 3) and ch["csr_variant"] in (0, 1, 2, 3)
        u = torch.tensor(_to_lib(x_or, p, op.N), dtype=dt, device="cuda")
        v = torch.empty_like(u)
        op.apply(u, v)
        torch.cuda.synchronize()
        y = v.cpu().numpy().astype(complex)[p]
        err = np.linalg.norm(y - y_or) / np.linalg.norm(y_or)
        assert err < tol, (prec, err)


def test_variable_index_medium_matches_oracle():
    """Smooth variable index n = sin(pi x1) cos(pi x2) (m = 1 - n^2 between 0
    and 1, n vanishing on lines through the star): the device apply matches
    the oracle on every row and both solve forms match the oracle's dense LU
    solve."""
    import torch
    from oracle.op2d import Setup2D
    from paper_1509_05063_amd import binding
    cfg = config("star_sincos_k2")
    n2 = n2_function(cfg)
    op = binding.Operator(cfg, n2)
    orc = Setup2D(cfg, n2)
    xy, key = op.points()
    p = match_keys(orc.pts["key"], key)
    A = orc.dense_A()
    x_or = random_density(orc.pts["key"], seed=11)
    y_or = A @ x_or
    u = torch.tensor(_to_lib(x_or, p, op.N), dtype=torch.complex128, device="cuda")
    v = torch.empty_like(u)
    op.apply(u, v)
    torch.cuda.synchronize()
    y = v.cpu().numpy()[p]
    err = np.linalg.norm(y - y_or) / np.linalg.norm(y_or)
    assert err < 1e-8, err
    f_or = plane_wave(cfg, orc.pts["x"], 0.0)
    u_or = np.linalg.solve(A, f_or)
    f = torch.tensor(_to_lib(f_or, p, op.N), dtype=torch.complex128, device="cuda")
    for mode in (binding.LS_SOLVE_FP64, binding.LS_SOLVE_FP32_REFINE):
        x = torch.empty_like(f)
        st = op.solve(f, x, tol=1e-10, restart=100, max_iter=2000, mode=mode, inner_tol=1e-5)
        e = np.linalg.norm(x.cpu().numpy()[p] - u_or) / np.linalg.norm(u_or)
        print(f"sin cos medium, N={op.N}, mode {mode}: {st} vs LU {e:.2e}, apply {err:.2e}", flush=True)
        assert st["converged"] == 1 and e < 1e-8, e
    op.close()


def test_scattered_field_off_the_disc(disc):
    """The device scattered field at points outside the disc (inside its cell
    box) equals the oracle's direct sum over the same solution, and the Mie
    scattered field to the discretisation's accuracy."""
    import torch
    from oracle.exterior import scattered_field
    from oracle.mie import mie2d_total
    from paper_1509_05063_amd import binding
    cfg, op, orc, A, p, xy, key = disc
    f_or = plane_wave(cfg, orc.pts["x"], 0.0)
    f = torch.tensor(_to_lib(f_or, p, op.N), dtype=torch.complex128, device="cuda")
    x = torch.empty_like(f)
    op.solve(f, x, tol=1e-12, restart=100, max_iter=500, mode=binding.LS_SOLVE_FP64)
    rng = np.random.default_rng(5)
    pts = rng.uniform(-0.999, 0.999, (4000, 2))
    rad = np.hypot(pts[:, 0], pts[:, 1])
    far = pts[rad > 1.12][:200]                      # a few grid spacings off the interface
    near = pts[(rad > 1.0 + 1e-6) & (rad < 1.03)][:50]
    xt = np.concatenate([far, near])
    us = op.scattered_field(x, xt).cpu().numpy()
    u_or = x.cpu().numpy()[p]
    ref = scattered_field(orc, u_or, xt)
    err = np.linalg.norm(us - ref) / np.linalg.norm(ref)
    ex = mie2d_total(cfg["kappa"], 1.5, 1.0, far) - np.exp(1j * cfg["kappa"] * far[:, 0])
    emie = np.linalg.norm(us[:len(far)] - ex) / np.linalg.norm(ex)
    print(f"scattered field: {len(xt)} targets, vs direct sum {err:.2e}, vs Mie {emie:.2e}", flush=True)
    assert err < 1e-9, err
    assert emie < 5e-3, emie
    with pytest.raises(binding.LSError):
        op.scattered_field(x, np.array([[0.1, 0.2]]))    # inside the scatterer
