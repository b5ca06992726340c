"""GPU parity through the C ABI: the device apply and solve against the CPU
oracle on the same seeded inputs (disc workload, every row)."""
import math

import numpy as np
import pytest

from gpu_helpers import fused_tile_max, schedule_cases
from paper_1509_05063_amd.inputs import config, match_keys, n2_function, plane_wave, random_density

pytestmark = pytest.mark.gpu

# FP32 apply against the FP64 oracle: rounding of about 800 products per row
# in single precision (unit roundoff 6e-8) on values of mixed sign; measured
# 6.6e-7 on the disc
F32_TOL = 1e-5


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
    assert err < F32_TOL


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
        assert ch["csr_variant"] not in (3, 4)
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
    the oracle (FP64 to 1e-8, FP32 to F32_TOL), and the choices are in range."""
    import torch
    from paper_1509_05063_amd import binding
    cfg, op, orc, A, p, xy, key = disc
    x_or = random_density(orc.pts["key"], seed=7)
    y_or = A @ x_or
    for prec, dt, tol in ((binding.LS_C128, torch.complex128, 1e-8), (binding.LS_C64, torch.complex64, F32_TOL)):
        ch = op.autotune(nrhs=1, prec=prec)
        print(f"autotune prec {prec}: {ch}", flush=True)
        assert ch["fft_col_tile"] in (1, 2, 4, 8, 16, 32) and ch["near_variant"] in (0, 1, 2, 3, 4) and ch["csr_variant"] in (0, 1, 2, 3, 4)
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


@pytest.mark.parametrize("prec_name", ["c128", "c64"])
def test_forced_schedules_match_oracle_every_row(disc, prec_name):
    """Every kernel variant the tuner can choose, forced through
    ls_set_schedule, applies the oracle's operator on every row of the disc
    (FP64 to 1e-8, FP32 to F32_TOL)."""
    import torch
    from paper_1509_05063_amd import binding
    cfg, op, orc, A, p, xy, key = disc
    prec = binding.LS_C128 if prec_name == "c128" else binding.LS_C64
    dt, tol = (torch.complex128, 1e-8) if prec == binding.LS_C128 else (torch.complex64, F32_TOL)
    saved = op.get_schedule(prec)
    x_or = random_density(orc.pts["key"], seed=21)
    y_or = A @ x_or
    u = torch.tensor(_to_lib(x_or, p, op.N), dtype=dt, device="cuda")
    try:
        for name, fields in schedule_cases(prec, fused_tile_max(op, prec)):
            op.set_schedule(prec, **saved)
            sch = op.set_schedule(prec, **fields)
            v = torch.empty_like(u)
            op.apply(u, v)
            torch.cuda.synchronize()
            y = v.cpu().numpy().astype(complex)[p]
            err = np.linalg.norm(y - y_or) / np.linalg.norm(y_or)
            emax = np.abs(y - y_or).max() / np.abs(y_or).max()
            print(f"{prec_name} schedule {name} {sch}: rel2 {err:.2e} relmax {emax:.2e}", flush=True)
            assert err < tol and emax < 10 * tol, (name, err, emax)
    finally:
        op.set_schedule(prec, **saved)


@pytest.mark.parametrize("nrhs", [16, 32])
def test_dense_tile_rows_double_precision_match_oracle(disc, nrhs):
    """The dense-tile rows in double precision (csr_variant 3 of the LS_C128
    schedule, on the matrix cores in FP64) against the oracle on every row of
    every right-hand side, and against the row kernel."""
    import torch
    from paper_1509_05063_amd import binding
    cfg, op, orc, A, p, xy, key = disc
    saved = op.get_schedule(binding.LS_C128)
    X = np.stack([random_density(orc.pts["key"], seed=200 + r) for r in range(nrhs)])
    Y = X @ A.T
    U = torch.tensor(np.stack([_to_lib(x, p, op.N) for x in X]), dtype=torch.complex128, device="cuda")
    try:
        op.set_schedule(binding.LS_C128, csr_variant=3)
        V = torch.empty_like(U)
        op.apply(U, V)
        op.set_schedule(binding.LS_C128, csr_variant=0)
        V2 = torch.empty_like(U)
        op.apply(U, V2)
        torch.cuda.synchronize()
    finally:
        op.set_schedule(binding.LS_C128, **saved)
    Vn = V.cpu().numpy()[:, p]
    err = (np.linalg.norm(Vn - Y, axis=1) / np.linalg.norm(Y, axis=1)).max()
    dif = (torch.linalg.norm(V - V2, dim=1) / torch.linalg.norm(V2, dim=1)).max().item()
    print(f"double-precision dense tiles, {nrhs} right-hand sides: vs oracle {err:.2e}, vs rows {dif:.2e}",
          flush=True)
    assert err < 1e-8 and dif < 1e-12


def test_schedule_setter_rejects_out_of_range(disc):
    from paper_1509_05063_amd import binding
    cfg, op, orc, A, p, xy, key = disc
    saved = op.get_schedule(binding.LS_C64)
    for bad in (dict(csr_variant=5), dict(near_variant=5), dict(near_variant=-1), dict(fft_variant=2), dict(fft_row_threads=128), dict(fft_rows_inplace=2), dict(near_rows_first=2),
                dict(fft_col_threads=1024), dict(fft_col_tile=0), dict(fft_col_tile=100000)):
        with pytest.raises(binding.LSError):
            op.set_schedule(binding.LS_C64, **bad)
        assert op.get_schedule(binding.LS_C64) == saved
    with pytest.raises(binding.LSError):
        op.set_schedule(binding.LS_C128, csr_variant=2)      # double precision has one row kernel


@pytest.mark.parametrize("nrhs,variant", [(16, 3), (32, 3), (16, 4), (32, 4)])
def test_dense_tile_rows_match_oracle(disc, nrhs, variant):
    """The dense-tile row kernel on the matrix cores (csr_variant 3, taken for
    multiples of 16 right-hand sides; 4: three real products per complex
    product) against the oracle on every row of every right-hand side, and
    against the single-right-hand-side run-length rows."""
    import torch
    from paper_1509_05063_amd import binding
    cfg, op, orc, A, p, xy, key = disc
    saved = op.get_schedule(binding.LS_C64)
    X = np.stack([random_density(orc.pts["key"], seed=100 + r) for r in range(nrhs)])
    Y = X @ A.T
    U = torch.tensor(np.stack([_to_lib(x, p, op.N) for x in X]), dtype=torch.complex64, device="cuda")
    try:
        op.set_schedule(binding.LS_C64, csr_variant=variant)
        V = torch.empty_like(U)
        op.apply(U, V)
        op.set_schedule(binding.LS_C64, csr_variant=2)
        V2 = torch.empty_like(U)
        op.apply(U, V2)
        torch.cuda.synchronize()
    finally:
        op.set_schedule(binding.LS_C64, **saved)
    Vn = V.cpu().numpy().astype(complex)[:, p]
    err = (np.linalg.norm(Vn - Y, axis=1) / np.linalg.norm(Y, axis=1)).max()
    dif = (torch.linalg.norm(V - V2, dim=1) / torch.linalg.norm(V2, dim=1)).max().item()
    print(f"dense tiles (variant {variant}), {nrhs} right-hand sides: vs oracle {err:.2e}, "
          f"vs run-length rows {dif:.2e}", flush=True)
    assert err < F32_TOL and dif < F32_TOL


def test_solve_inner_f64_basis_and_profile(disc):
    """FP32 apply inside a complex-double inner Arnoldi (inner_f64_basis)
    reaches the oracle's LU solution like the other forms; with profile set
    the stage times are positive and bounded by the wall time."""
    import torch
    from paper_1509_05063_amd import binding
    cfg, op, orc, A, p, xy, key = disc
    f_or = plane_wave(cfg, orc.pts["x"], 0.0)
    u_or = np.linalg.solve(A, f_or)
    f = torch.tensor(_to_lib(f_or, p, op.N), dtype=torch.complex128, device="cuda")
    for basis64 in (True, False):
        x = torch.empty_like(f)
        st = op.solve(f, x, tol=1e-10, restart=100, max_iter=2000, mode=binding.LS_SOLVE_FP32_REFINE,
                      inner_tol=1e-5, inner_f64_basis=basis64, profile=True)
        err = np.linalg.norm(x.cpu().numpy()[p] - u_or) / np.linalg.norm(u_or)
        us = st["stage_us"]
        print(f"inner f64 basis {basis64}: {st} vs LU {err:.2e}", flush=True)
        assert st["converged"] == 1 and err < 1e-8
        assert us["apply_fp32"] > 0 and us["apply_fp64"] > 0 and us["arnoldi"] > 0
        assert sum(us.values()) < 1e6 * st["seconds"]


def test_solve_with_caller_workspace_equals_own_scratch(disc):
    import torch
    from paper_1509_05063_amd import binding
    cfg, op, orc, A, p, xy, key = disc
    f = torch.tensor(plane_wave(cfg, xy, 0.3), dtype=torch.complex128, device="cuda")
    kw = dict(tol=1e-10, restart=30, max_iter=2000, mode=binding.LS_SOLVE_FP32_REFINE, inner_tol=1e-5)
    x0, x1 = torch.empty_like(f), torch.empty_like(f)
    op.solve(f, x0, **kw)
    nb = op.solve_workspace_bytes(1, restart=30)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    op.solve(f, x1, workspace=ws, **kw)
    torch.cuda.synchronize()
    assert torch.equal(x0, x1)
    with pytest.raises(binding.LSError):
        op.solve(f, x1, workspace=ws[: nb // 2], **kw)      # too small


def test_nan_input_reports_numeric_status(disc):
    """A non-finite right-hand side is reported (LS_ENUMERIC) at once in both
    modes, without running to max_iter; in a batch the finite right-hand
    sides still converge to their own solutions."""
    import torch
    from paper_1509_05063_amd import binding
    cfg, op, orc, A, p, xy, key = disc
    F = torch.tensor(np.stack([plane_wave(cfg, xy, a) for a in (0.0, 0.5, 1.0)]), dtype=torch.complex128,
                     device="cuda")
    F[1, 17] = float("nan")
    for mode in (binding.LS_SOLVE_FP64, binding.LS_SOLVE_FP32_REFINE):
        X = torch.empty_like(F)
        st = op.solve(F, X, tol=1e-10, restart=100, max_iter=2000, mode=mode, inner_tol=1e-5,
                      raise_on_noconv=False)
        print(f"NaN right-hand side, mode {mode}: {st}", flush=True)
        assert st["status"] == binding.LS_ENUMERIC
        assert st["converged"] == 2 and st["iterations"] < 400
        for k in (0, 2):
            x1 = torch.empty_like(F[k])
            op.solve(F[k].contiguous(), x1, tol=1e-10, restart=100, max_iter=2000, mode=mode, inner_tol=1e-5)
            assert torch.isfinite(X[k]).all()
            assert (torch.linalg.norm(X[k] - x1) / torch.linalg.norm(x1)).item() < 1e-8


def test_stagnation_stops_early(disc):
    """A tolerance below what double precision can reach stops once a
    restart cycle no longer reduces the residual (LS_ENOCONV with the best
    iterate), long before max_iter."""
    import torch
    from paper_1509_05063_amd import binding
    cfg, op, orc, A, p, xy, key = disc
    f = torch.tensor(plane_wave(cfg, xy, 0.0), dtype=torch.complex128, device="cuda")
    x = torch.empty_like(f)
    st = op.solve(f, x, tol=1e-30, restart=20, max_iter=100000, mode=binding.LS_SOLVE_FP64, raise_on_noconv=False)
    print(f"tol 1e-30: {st}", flush=True)
    assert st["status"] == binding.LS_ENOCONV and st["iterations"] < 5000 and st["rel_residual"] < 1e-12


def test_torch_allocator_and_failing_allocator():
    """Operator memory from PyTorch's caching allocator: the same applies as
    with hipMalloc, the bytes show up in torch's accounting and go back at
    destroy.  An allocator that fails on its k-th call makes ls_create return
    LS_ENOMEM with every block it handed out released."""
    import ctypes as C
    import torch
    from paper_1509_05063_amd import binding
    cfg = config("disc_k2pi")
    n2 = n2_function(cfg)
    ref = binding.Operator(cfg, n2)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    op = binding.Operator(cfg, n2, allocator="torch")
    try:
        assert torch.cuda.memory_allocated() - before >= op.resident_bytes()
        xy, _ = op.points()
        u = torch.tensor(plane_wave(cfg, xy, 0.2), dtype=torch.complex128, device="cuda")
        v0, v1 = torch.empty_like(u), torch.empty_like(u)
        ref.apply(u, v0)
        op.apply(u, v1)
        x0, x1 = torch.empty_like(u), torch.empty_like(u)
        ref.solve(u, x0, tol=1e-10, restart=50)
        op.solve(u, x1, tol=1e-10, restart=50)
        torch.cuda.synchronize()
        assert torch.equal(v0, v1) and torch.equal(x0, x1)
    finally:
        op.close()
        ref.close()
    del u, v0, v1, x0, x1
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() <= before

    for fail_at in (1, 5, 40):
        live = {}
        calls = [0]

        def _alloc(nbytes, ctx):
            calls[0] += 1
            if calls[0] >= fail_at:
                return None
            t = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
            live[t.data_ptr()] = t
            return t.data_ptr()

        def _release(ptr, nbytes, ctx):
            live.pop(ptr)

        al = binding.Allocator(binding.ALLOCFN(_alloc), binding.RELEASEFN(_release), None)
        with pytest.raises(binding.LSError) as ei:
            binding.Operator(cfg, n2, allocator=al)
        assert ei.value.status == binding.LS_ENOMEM
        assert calls[0] == fail_at and not live, (fail_at, calls[0], len(live))


@pytest.mark.parametrize("name", ["disc_k2pi_p2", "star_sincos_k2_p3"])
def test_several_boundary_patches_match_oracle(name):
    """Boundary covered by two / three overlapping patches with a tangential
    partition of unity: both precisions' applies against the oracle on every
    row, and both solve forms against the oracle's dense LU solution."""
    import torch
    from oracle.op2d import Setup2D
    from paper_1509_05063_amd import binding
    cfg = config(name)
    n2 = n2_function(cfg)
    op = binding.Operator(cfg, n2)
    orc = Setup2D(cfg, n2)
    xy, key = op.points()
    p = match_keys(orc.pts["key"], key)
    A = orc.dense_A()
    x_or = random_density(orc.pts["key"], seed=13)
    y_or = A @ x_or
    for dt, tol in ((torch.complex128, 1e-8), (torch.complex64, F32_TOL)):
        u = torch.tensor(_to_lib(x_or, p, op.N), dtype=dt, device="cuda")
        v = torch.empty_like(u)
        op.apply(u, v)
        torch.cuda.synchronize()
        y = v.cpu().numpy().astype(complex)[p]
        err = np.linalg.norm(y - y_or) / np.linalg.norm(y_or)
        print(f"{name} N={op.N} apply {dt}: {err:.2e}", flush=True)
        assert err < tol, (dt, err)
    f_or = plane_wave(cfg, orc.pts["x"], 0.4)
    u_or = np.linalg.solve(A, f_or)
    f = torch.tensor(_to_lib(f_or, p, op.N), dtype=torch.complex128, device="cuda")
    for mode in (binding.LS_SOLVE_FP64, binding.LS_SOLVE_FP32_REFINE):
        x = torch.empty_like(f)
        st = op.solve(f, x, tol=1e-10, restart=100, max_iter=2000, mode=mode, inner_tol=1e-5)
        e = np.linalg.norm(x.cpu().numpy()[p] - u_or) / np.linalg.norm(u_or)
        print(f"{name} solve mode {mode}: {st} vs LU {e:.2e}", flush=True)
        assert st["converged"] == 1 and e < 1e-8, e
    op.close()


@pytest.mark.parametrize("r", [2, 3])
def test_fft_refined_interpolation_matches_oracle(r):
    """Fourier refined interpolation along the band's t1 lines (ls_params
    fft_refine = r): the device refines the density lines by FFT every
    apply and the rows read the refined values.  Both precisions against the
    oracle's refined operator on every row, under each row-kernel schedule;
    a batch of three right-hand sides equals three single applies; the
    refined solve matches the oracle's dense LU solution."""
    import torch
    from oracle.op2d import Setup2D
    from paper_1509_05063_amd import binding
    from paper_1509_05063_amd.inputs import scaled
    cfg = scaled(config("disc_k2pi"), fft_refine=r)
    n2 = n2_function(cfg)
    op = binding.Operator(cfg, n2)
    orc = Setup2D(cfg, n2)
    xy, key = op.points()
    p = match_keys(orc.pts["key"], key)
    A = orc.dense_A()
    with pytest.raises(binding.LSError):         # no dense tiles with refinement
        op.set_schedule(binding.LS_C128, csr_variant=3)
    x_or = random_density(orc.pts["key"], seed=31)
    y_or = A @ x_or
    for prec, dt, tol, variants in ((binding.LS_C128, torch.complex128, 1e-8, (0,)),
                                    (binding.LS_C64, torch.complex64, F32_TOL, (0, 1, 2))):
        saved = op.get_schedule(prec)
        u = torch.tensor(_to_lib(x_or, p, op.N), dtype=dt, device="cuda")
        try:
            for cv in variants:
                op.set_schedule(prec, **dict(saved, csr_variant=cv))
                v = torch.empty_like(u)
                op.apply(u, v)
                torch.cuda.synchronize()
                y = v.cpu().numpy().astype(complex)[p]
                err = np.linalg.norm(y - y_or) / np.linalg.norm(y_or)
                emax = np.abs(y - y_or).max() / np.abs(y_or).max()
                print(f"refine {r} {dt} csr {cv}: rel2 {err:.2e} relmax {emax:.2e}", flush=True)
                assert err < tol and emax < 10 * tol, (cv, err, emax)
            U = torch.stack([torch.tensor(_to_lib(random_density(orc.pts["key"], seed=40 + s), p, op.N), dtype=dt)
                             for s in range(3)]).cuda()
            V = torch.empty_like(U)
            op.apply(U, V)
            for k in range(3):
                vk = torch.empty_like(U[k])
                op.apply(U[k].contiguous(), vk)
                torch.cuda.synchronize()
                d = (torch.linalg.norm(V[k] - vk) / torch.linalg.norm(vk)).item()
                assert d < (1e-13 if dt == torch.complex128 else 1e-6), (k, d)
        finally:
            op.set_schedule(prec, **saved)
    f_or = plane_wave(cfg, orc.pts["x"], 0.3)
    u_or = np.linalg.solve(A, f_or)
    f = torch.tensor(_to_lib(f_or, p, op.N), dtype=torch.complex128, device="cuda")
    x = torch.empty_like(f)
    st = op.solve(f, x, tol=1e-10, restart=100, max_iter=2000, mode=binding.LS_SOLVE_FP32_REFINE, inner_tol=1e-5)
    e = np.linalg.norm(x.cpu().numpy()[p] - u_or) / np.linalg.norm(u_or)
    print(f"refine {r} solve: {st} vs LU {e:.2e}", flush=True)
    assert st["converged"] == 1 and e < 1e-8, e
    op.close()


def test_fft_refined_interior_matches_oracle():
    """Fourier refinement of the interior lattice as well (fft_refine = 2,
    fft_refine_interior = 1): the device transforms the interior psi grids
    every apply, forms the three shifted grids and contracts one window per
    shift.  Both precisions against the oracle's rows (every boundary-patch
    row and 600 interior rows) under each interior-contraction and row
    kernel schedule; a batch of three equals three single applies; the
    refined solve satisfies the oracle's rows."""
    import torch
    from oracle.op2d import Setup2D
    from paper_1509_05063_amd import binding
    from paper_1509_05063_amd.inputs import scaled
    cfg = scaled(config("disc_k2pi"), fft_refine=2, fft_refine_interior=1)
    n2 = n2_function(cfg)
    op = binding.Operator(cfg, n2)
    orc = Setup2D(cfg, n2)
    xy, key = op.points()
    p = match_keys(orc.pts["key"], key)
    rng = np.random.default_rng(3)
    n_int = orc.pts["n_int"]
    rows = np.concatenate([np.sort(rng.choice(n_int, 600, replace=False)), np.arange(n_int, orc.N)])
    A = orc.A_rows(rows)
    x_or = random_density(orc.pts["key"], seed=33)
    y_or = A @ x_or
    cases = {binding.LS_C128: (torch.complex128, 1e-8, [{}]),
             binding.LS_C64: (torch.complex64, F32_TOL,
                              [dict(near_variant=v) for v in range(5)] + [dict(csr_variant=v) for v in (0, 1, 2)])}
    for prec, (dt, tol, scheds) in cases.items():
        saved = op.get_schedule(prec)
        u = torch.tensor(_to_lib(x_or, p, op.N), dtype=dt, device="cuda")
        try:
            for sch in scheds:
                op.set_schedule(prec, **dict(saved, **sch))
                v = torch.empty_like(u)
                op.apply(u, v)
                torch.cuda.synchronize()
                y = v.cpu().numpy().astype(complex)[p][rows]
                err = np.linalg.norm(y - y_or) / np.linalg.norm(y_or)
                emax = np.abs(y - y_or).max() / np.abs(y_or).max()
                print(f"refined interior {dt} {sch}: rel2 {err:.2e} relmax {emax:.2e}", flush=True)
                assert err < tol and emax < 10 * tol, (sch, err, emax)
            U = torch.stack([torch.tensor(_to_lib(random_density(orc.pts["key"], seed=50 + s), p, op.N), dtype=dt)
                             for s in range(3)]).cuda()
            V = torch.empty_like(U)
            op.apply(U, V)
            for k in range(3):
                vk = torch.empty_like(U[k])
                op.apply(U[k].contiguous(), vk)
                torch.cuda.synchronize()
                d = (torch.linalg.norm(V[k] - vk) / torch.linalg.norm(vk)).item()
                assert d < (1e-13 if dt == torch.complex128 else 1e-6), (k, d)
        finally:
            op.set_schedule(prec, **saved)
    f_or = plane_wave(cfg, orc.pts["x"], 0.3)
    f = torch.tensor(_to_lib(f_or, p, op.N), dtype=torch.complex128, device="cuda")
    x = torch.empty_like(f)
    st = op.solve(f, x, tol=1e-10, restart=100, max_iter=2000, mode=binding.LS_SOLVE_FP32_REFINE, inner_tol=1e-5)
    xo = x.cpu().numpy()[p]
    res = np.linalg.norm(A @ xo - f_or[rows]) / np.linalg.norm(f_or[rows])
    print(f"refined interior solve: {st} oracle-row residual {res:.2e}", flush=True)
    assert st["converged"] == 1 and res < 1e-8, res
    op.close()


@pytest.mark.parametrize("r", [1, 2])
def test_offgrid_shortcut_matches_oracle(r):
    """The paper's off-grid shortcut (offgrid_shortcut; with r = 2 its s lines
    refined along t1): every apply first evaluates the boundary rule at the
    patch's grid nodes into the workspace, then the rows read those values.
    Both precisions against the oracle on every row of the disc, under each
    row-kernel schedule; a batch of three equals three single applies; the
    solve matches the oracle's dense LU solution."""
    import torch
    from oracle.op2d import Setup2D
    from paper_1509_05063_amd import binding
    from paper_1509_05063_amd.inputs import scaled
    cfg = scaled(config("disc_k2pi"), fft_refine=r, offgrid_shortcut=1)
    n2 = n2_function(cfg)
    op = binding.Operator(cfg, n2)
    orc = Setup2D(cfg, n2)
    xy, key = op.points()
    p = match_keys(orc.pts["key"], key)
    A = orc.dense_A()
    x_or = random_density(orc.pts["key"], seed=35)
    y_or = A @ x_or
    for prec, dt, tol, variants in ((binding.LS_C128, torch.complex128, 1e-8, (0,)),
                                    (binding.LS_C64, torch.complex64, F32_TOL, (0, 1, 2))):
        saved = op.get_schedule(prec)
        u = torch.tensor(_to_lib(x_or, p, op.N), dtype=dt, device="cuda")
        try:
            for cv in variants:
                op.set_schedule(prec, **dict(saved, csr_variant=cv))
                v = torch.empty_like(u)
                op.apply(u, v)
                torch.cuda.synchronize()
                y = v.cpu().numpy().astype(complex)[p]
                err = np.linalg.norm(y - y_or) / np.linalg.norm(y_or)
                emax = np.abs(y - y_or).max() / np.abs(y_or).max()
                print(f"shortcut r={r} {dt} csr {cv}: rel2 {err:.2e} relmax {emax:.2e}", flush=True)
                assert err < tol and emax < 10 * tol, (cv, err, emax)
            U = torch.stack([torch.tensor(_to_lib(random_density(orc.pts["key"], seed=60 + s), p, op.N), dtype=dt)
                             for s in range(3)]).cuda()
            V = torch.empty_like(U)
            op.apply(U, V)
            for k in range(3):
                vk = torch.empty_like(U[k])
                op.apply(U[k].contiguous(), vk)
                torch.cuda.synchronize()
                d = (torch.linalg.norm(V[k] - vk) / torch.linalg.norm(vk)).item()
                assert d < (1e-13 if dt == torch.complex128 else 1e-6), (k, d)
        finally:
            op.set_schedule(prec, **saved)
    f_or = plane_wave(cfg, orc.pts["x"], 0.3)
    u_or = np.linalg.solve(A, f_or)
    f = torch.tensor(_to_lib(f_or, p, op.N), dtype=torch.complex128, device="cuda")
    x = torch.empty_like(f)
    st = op.solve(f, x, tol=1e-10, restart=100, max_iter=2000, mode=binding.LS_SOLVE_FP32_REFINE, inner_tol=1e-5)
    e = np.linalg.norm(x.cpu().numpy()[p] - u_or) / np.linalg.norm(u_or)
    print(f"shortcut r={r} solve: {st} vs LU {e:.2e}", flush=True)
    assert st["converged"] == 1 and e < 1e-8, e
    op.close()


def test_fft_refined_odd_line_length_matches_oracle():
    """Fourier refinement on band lines of odd length (N1 = 75 = 3 x 5^2:
    no Nyquist term, mixed-radix line transforms) with r = 3, the interior
    refined as well (eight shifted grids): both precisions against the
    oracle on 300 boundary-patch and 300 interior rows of the disc."""
    import torch
    from oracle.op2d import Setup2D
    from paper_1509_05063_amd import binding
    from paper_1509_05063_amd.inputs import scaled
    cfg = scaled(config("disc_k2pi"), band={"N1": 75}, fft_refine=3, fft_refine_interior=1)
    n2 = n2_function(cfg)
    op = binding.Operator(cfg, n2)
    orc = Setup2D(cfg, n2)
    xy, key = op.points()
    p = match_keys(orc.pts["key"], key)
    n_int = orc.pts["n_int"]
    rng = np.random.default_rng(5)
    rows = np.concatenate([np.sort(rng.choice(n_int, 300, replace=False)),
                           n_int + np.sort(rng.choice(orc.N - n_int, 300, replace=False))])
    A = orc.A_rows(rows)
    x_or = random_density(orc.pts["key"], seed=37)
    y_or = A @ x_or
    for dt, tol in ((torch.complex128, 1e-8), (torch.complex64, F32_TOL)):
        u = torch.tensor(_to_lib(x_or, p, op.N), dtype=dt, device="cuda")
        v = torch.empty_like(u)
        op.apply(u, v)
        torch.cuda.synchronize()
        y = v.cpu().numpy().astype(complex)[p][rows]
        err = np.linalg.norm(y - y_or) / np.linalg.norm(y_or)
        print(f"odd N1 refine 3 {dt}: rel2 {err:.2e}", flush=True)
        assert err < tol, (dt, err)
    op.close()
