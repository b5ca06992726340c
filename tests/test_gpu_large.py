"""GPU parity at the benchmark size (sampled rows, the oracle computes them
one by one), multi-right-hand-side batching and edge cases, through the C ABI."""
import math

import numpy as np
import pytest

from paper_1509_05063_amd.inputs import (config, match_keys, n2_function, plane_wave, random_density,
                                         scaled)

pytestmark = pytest.mark.gpu

F32_TOL = 1e-5      # single-precision apply against the FP64 oracle (measured about 2e-6 here)


def _op(cfg):
    from paper_1509_05063_amd import binding
    return binding.Operator(cfg, n2_function(cfg))


@pytest.fixture(scope="module")
def star32():
    from oracle.op2d import Setup2D
    cfg = config("star_k32pi")
    op = _op(cfg)
    orc = Setup2D(cfg, n2_function(cfg))
    _, key = op.points()
    p = match_keys(orc.pts["key"], key)
    return cfg, op, orc, p


def _sampled_rows(orc, nrows, seed=1509):
    rng = np.random.default_rng(seed)
    n_int = orc.pts["n_int"]
    # half the rows on the boundary patch (they carry the interface rules)
    a = rng.choice(n_int, nrows // 2, replace=False)
    b = n_int + rng.choice(orc.N - n_int, nrows - nrows // 2, replace=False)
    return np.concatenate([a, b])


def classified_rows(orc, per_class=43, seed=1509):
    """Rows that exercise every rule of the near field: boundary-patch nodes
    on the interface (t2 = 0), boundary-patch nodes in the partition-of-unity
    transition, interior-lattice nodes inside the boundary patch (off-grid
    targets of its rule) with and without the transition, other
    boundary-patch nodes, deep interior nodes.  Returns (rows, class names)."""
    rng = np.random.default_rng(seed)
    pt = orc.pts
    chart, key, om, inb = pt["chart"], pt["key"], pt["omega"], pt["in_band"]
    classes = {
        "interface": (chart == 1) & (key[:, 2] == 0),
        "band_pou": (chart == 1) & (om > 0) & (om < 1),
        "offgrid_pou": (chart == 0) & inb & (om > 0) & (om < 1),
        "offgrid": (chart == 0) & inb & (om == 1),
        "band": (chart == 1) & (key[:, 2] > 0),
        "interior": (chart == 0) & ~inb,
    }
    rows, names = [], []
    for name, mask in classes.items():
        idx = np.nonzero(mask)[0]
        assert idx.size >= per_class, name
        rows.append(rng.choice(idx, per_class, replace=False))
        names += [name] * per_class
    return np.concatenate(rows), np.array(names)


def oracle_rows_times(orc, rows, U, chunk=16):
    """A_rows(rows) @ U without keeping the dense rows (U: (N, k))."""
    out = []
    for c in range(0, len(rows), chunk):
        out.append(orc.A_rows(rows[c:c + chunk]) @ U)
    return np.concatenate(out)


@pytest.fixture(scope="module")
def star32_rows(star32):
    cfg, op, orc, p = star32
    rows, names = classified_rows(orc)
    U = np.stack([random_density(orc.pts["key"]), plane_wave(cfg, orc.pts["x"], cfg["incidence"][0])], 1)
    return rows, names, U, oracle_rows_times(orc, rows, U)


def test_benchmark_size_apply_sampled_rows(star32, star32_rows):
    """258 oracle rows in six classes (interface, partition-of-unity
    transition, off-grid targets of the boundary patch, ...) against both
    precisions' applies with the default kernels, for a random density and
    the incident plane wave."""
    import torch
    cfg, op, orc, p = star32
    rows, names, U, V_or = star32_rows
    for dt, tol in [(torch.complex128, 1e-8), (torch.complex64, F32_TOL)]:
        for k in range(U.shape[1]):
            u = np.empty(op.N, complex)
            u[p] = U[:, k]
            ud = torch.tensor(u, dtype=dt, device="cuda")
            vd = torch.empty_like(ud)
            op.apply(ud, vd)
            torch.cuda.synchronize()
            v = vd.cpu().numpy().astype(complex)[p][rows]
            err = np.abs(v - V_or[:, k]) / np.abs(V_or[:, k]).max()
            for cl in np.unique(names):
                print(f"star_k32pi {dt} input {k} {cl}: max rel err {err[names == cl].max():.3e}", flush=True)
            assert err.max() < tol


def test_benchmark_schedules_match_oracle_rows(star32, star32_rows):
    """Every kernel variant the tuner can choose at the benchmark size,
    forced through ls_set_schedule (one field at a time, and the combination
    the tuner picks), against the oracle's rows."""
    import torch
    from paper_1509_05063_amd import binding
    from gpu_helpers import fused_tile_max, schedule_cases
    cfg, op, orc, p = star32
    rows, names, U, V_or = star32_rows
    u = np.empty(op.N, complex)
    u[p] = U[:, 0]
    for prec, dt, tol in ((binding.LS_C64, torch.complex64, F32_TOL), (binding.LS_C128, torch.complex128, 1e-8)):
        saved = op.get_schedule(prec)
        ud = torch.tensor(u, dtype=dt, device="cuda")
        try:
            for name, fields in schedule_cases(prec, fused_tile_max(op, prec)):
                op.set_schedule(prec, **saved)
                sch = op.set_schedule(prec, **fields)
                vd = torch.empty_like(ud)
                op.apply(ud, vd)
                torch.cuda.synchronize()
                v = vd.cpu().numpy().astype(complex)[p][rows]
                err = (np.abs(v - V_or[:, 0]) / np.abs(V_or[:, 0]).max()).max()
                print(f"star_k32pi prec {prec} schedule {name} {sch}: max rel err {err:.3e}", flush=True)
                assert err < tol, (name, err)
        finally:
            op.set_schedule(prec, **saved)


@pytest.mark.parametrize("interior,shortcut", [(False, False), (True, False), (False, True)])
def test_benchmark_size_fft_refined_rows(star32, interior, shortcut):
    """Fourier refined interpolation (fft_refine = 2) at the benchmark size:
    4096-point line transforms of the band's 33 t2 lines in both
    precisions, the rows' 32-bit columns reaching the refined values past
    the N unknowns; with the interior refinement also the 2-D transforms of
    the interior psi grids (1350 x 1350) and one interior contraction per
    shift.  Oracle rows of every class (its refined rules) against both
    precisions' applies; the apply times are printed beside the unrefined
    operator's.  With the off-grid shortcut (unrefined): the boundary rule at
    the 135,168 grid nodes first, then the rows reading those values."""
    import copy
    import time
    import torch
    cfg0, op0, orc0, p = star32
    # (the off-grid shortcut unrefined here: the oracle's refined shortcut
    # spreads over whole 4096-point lines of node rules)
    cfg = scaled(cfg0, fft_refine=1 if shortcut else 2, fft_refine_interior=int(interior),
                 offgrid_shortcut=int(shortcut))
    t0 = time.perf_counter()
    op = _op(cfg)
    t_setup = time.perf_counter() - t0
    orc = copy.copy(orc0)           # same nodes; its rows follow the refined rule
    orc.cfg = cfg
    orc._cache = {}
    rows, names = classified_rows(orc, per_class=10 if interior else 20, seed=7)
    U = random_density(orc.pts["key"], seed=5)[:, None]
    V_or = oracle_rows_times(orc, rows, U)[:, 0]
    u = np.empty(op.N, complex)
    u[p] = U[:, 0]
    for dt, tol in [(torch.complex128, 1e-8), (torch.complex64, F32_TOL)]:
        ud = torch.tensor(u, dtype=dt, device="cuda")
        times = []
        for o in (op0, op):
            vd = torch.empty_like(ud)
            o.apply(ud, vd)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(20):
                o.apply(ud, vd)
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t0) / 20 * 1e3)
        v = vd.cpu().numpy().astype(complex)[p][rows]
        err = np.abs(v - V_or) / np.abs(V_or).max()
        for cl in np.unique(names):
            print(f"refined star_k32pi (interior {interior}, shortcut {shortcut}) {dt} {cl}: max rel err "
                  f"{err[names == cl].max():.3e}", flush=True)
        print(f"refined star_k32pi (interior {interior}, shortcut {shortcut}) {dt}: apply {times[1]:.3f} ms (unrefined {times[0]:.3f} ms), "
              f"set-up {t_setup:.1f} s, resident {op.resident_bytes() / 1e9:.2f} GB", flush=True)
        assert err.max() < tol
    op.close()


@pytest.mark.parametrize("double,variant", [(False, 3), (False, 4), (True, 3)])
def test_benchmark_size_dense_tiles_match_oracle_rows(star32, star32_rows, double, variant):
    """The dense-tile row kernel (16 right-hand sides, csr_variant 3; 4: three
    real products per complex product; in single and double precision) at
    the benchmark size against the oracle's rows (each right-hand side a
    phase-shifted copy of the random density)."""
    import torch
    from paper_1509_05063_amd import binding
    cfg, op, orc, p = star32
    rows, names, U, V_or = star32_rows
    prec, dt, tol = (binding.LS_C128, torch.complex128, 1e-8) if double else (binding.LS_C64, torch.complex64, F32_TOL)
    ph = np.exp(2j * np.pi * np.arange(16) / 16)
    X = np.empty((16, op.N), complex)
    X[:, p] = ph[:, None] * U[:, 0][None, :]
    saved = op.get_schedule(prec)
    try:
        op.set_schedule(prec, csr_variant=variant)
        Xd = torch.tensor(X, dtype=dt, device="cuda")
        Vd = torch.empty_like(Xd)
        op.apply(Xd, Vd)
        torch.cuda.synchronize()
    finally:
        op.set_schedule(prec, **saved)
    V = Vd.cpu().numpy().astype(complex)[:, p][:, rows]
    ref = ph[:, None] * V_or[:, 0][None, :]
    err = (np.abs(V - ref) / np.abs(ref).max()).max()
    print(f"star_k32pi dense tiles ({'double' if double else 'single'} precision, variant {variant}), "
          f"16 right-hand sides: max rel err {err:.3e}", flush=True)
    assert err < tol


def test_benchmark_size_solve_modes_agree(star32):
    import torch
    from paper_1509_05063_amd import binding
    cfg, op, orc, p = star32
    xy, _ = op.points()
    f = torch.tensor(plane_wave(cfg, xy, cfg["incidence"][0]), dtype=torch.complex128, device="cuda")
    x64, x32 = torch.empty_like(f), torch.empty_like(f)
    s64 = op.solve(f, x64, tol=1e-10, restart=60, max_iter=3000, mode=binding.LS_SOLVE_FP64)
    s32 = op.solve(f, x32, tol=1e-8, restart=60, max_iter=3000, mode=binding.LS_SOLVE_FP32_REFINE, inner_tol=1e-4)
    err = (torch.linalg.norm(x32 - x64) / torch.linalg.norm(x64)).item()
    print(f"star_k32pi solves: fp64 {s64} fp32+refine {s32} diff {err:.3e}", flush=True)
    assert s64["converged"] == 1 and s32["converged"] == 1
    assert err < 1e-6
    # the solution satisfies the oracle's equation on sampled rows
    rows = _sampled_rows(orc, 8, seed=7)
    x_or = x64.cpu().numpy()[p]
    r = orc.A_rows(rows) @ x_or - plane_wave(cfg, orc.pts["x"][rows], cfg["incidence"][0])
    assert np.abs(r).max() < 1e-7, np.abs(r).max()
    # longer restart cycles (more than 64 basis vectors: chunked passes) and
    # single Gram-Schmidt reach the same solution
    for restart, ortho in ((80, binding.LS_ORTHO_CGS2), (60, binding.LS_ORTHO_CGS1)):
        for mode in (binding.LS_SOLVE_FP64, binding.LS_SOLVE_FP32_REFINE):
            xo = torch.empty_like(f)
            so = op.solve(f, xo, tol=1e-8, restart=restart, max_iter=3000, mode=mode, inner_tol=1e-4, ortho=ortho)
            e = (torch.linalg.norm(xo - x64) / torch.linalg.norm(x64)).item()
            print(f"restart {restart} ortho {ortho} mode {mode}: {so} diff {e:.3e}", flush=True)
            assert so["converged"] == 1 and e < 1e-6


def test_multi_rhs_batch_matches_single_and_oracle():
    import torch
    from oracle.op2d import Setup2D
    cfg = config("star_k16pi")
    op = _op(cfg)
    xy, key = op.points()
    R = 8
    dirs = cfg["incidence"][:: len(cfg["incidence"]) // R][:R]
    U = torch.tensor(np.stack([plane_wave(cfg, xy, a) for a in dirs]), dtype=torch.complex128, device="cuda")
    V = torch.empty_like(U)
    op.apply(U, V)
    for k in (0, R - 1):
        v1 = torch.empty_like(U[k])
        op.apply(U[k].contiguous(), v1)
        torch.cuda.synchronize()
        assert torch.equal(v1, V[k])
    orc = Setup2D(cfg, n2_function(cfg))
    p = match_keys(orc.pts["key"], key)
    rows = _sampled_rows(orc, 8)
    A = orc.A_rows(rows)
    for k in (0, 5):
        v_or = A @ plane_wave(cfg, orc.pts["x"], dirs[k])
        v = V[k].cpu().numpy()[p][rows]
        assert np.abs(v - v_or).max() / np.abs(v_or).max() < 1e-8
    # batched solve: every right-hand side converges and matches its own solve
    X = torch.empty_like(U)
    st = op.solve(U[:4].contiguous(), X[:4], tol=1e-8, restart=60, max_iter=3000, mode=1, inner_tol=1e-4)
    assert st["converged"] == 4
    x1 = torch.empty_like(U[0])
    op.solve(U[2].contiguous(), x1, tol=1e-8, restart=60, max_iter=3000, mode=1, inner_tol=1e-4)
    assert (torch.linalg.norm(x1 - X[2]) / torch.linalg.norm(x1)).item() < 1e-6


def test_large_batch_projection_matches_oracle():
    """64 right-hand sides in single precision on the kappa = 16 pi star take
    the batch projection kernels (the interior part as a walking kernel, the
    boundary-patch nodes on the matrix cores): sampled rows of every sixth
    right-hand side against the oracle, and every right-hand side against its
    own single apply (smaller launches use other kernels, so to rounding)."""
    import torch
    from oracle.op2d import Setup2D
    from paper_1509_05063_amd import binding
    cfg = config("star_k16pi")
    op = _op(cfg)
    xy, key = op.points()
    R = 64
    dirs = [2 * np.pi * r / R for r in range(R)]
    U = torch.tensor(np.stack([plane_wave(cfg, xy, a) for a in dirs]), dtype=torch.complex64, device="cuda")
    saved = op.get_schedule(binding.LS_C64)
    try:
        op.set_schedule(binding.LS_C64, csr_variant=2)     # rows as for one right-hand side
        V = torch.empty_like(U)
        op.apply(U, V)
        V1 = torch.empty_like(U)
        for k in range(R):
            op.apply(U[k].contiguous(), V1[k])
        torch.cuda.synchronize()
    finally:
        op.set_schedule(binding.LS_C64, **saved)
    dif = (torch.linalg.norm(V - V1, dim=1) / torch.linalg.norm(V1, dim=1)).max().item()
    orc = Setup2D(cfg, n2_function(cfg))
    p = match_keys(orc.pts["key"], key)
    rows = _sampled_rows(orc, 8)
    A = orc.A_rows(rows)
    err = 0.0
    for k in range(0, R, 6):
        v_or = A @ plane_wave(cfg, orc.pts["x"], dirs[k])
        v = V[k].cpu().numpy().astype(complex)[p][rows]
        err = max(err, np.abs(v - v_or).max() / np.abs(v_or).max())
    print(f"64 right-hand sides: vs single applies {dif:.2e}, vs oracle rows {err:.2e}", flush=True)
    assert dif < F32_TOL and err < F32_TOL


def test_edge_cases_tiny_grid_zero_input_and_errors():
    import torch
    from oracle.op2d import Setup2D
    from paper_1509_05063_amd import binding
    # the smallest admissible grid: N2 = Q-1 intervals would not fit the
    # 8-node stencil, so N2 = 8; lattice h = 1/16
    cfg = scaled(config("disc_k2pi"), h=1 / 16, band={"N1": 32, "N2": 8}, r_int=6 / 16, r1=6.0, r2=4.0)
    op = _op(cfg)
    orc = Setup2D(cfg, n2_function(cfg))
    _, key = op.points()
    p = match_keys(orc.pts["key"], key)
    u_or = random_density(orc.pts["key"], seed=3)
    v_or = orc.dense_A() @ u_or
    u = np.empty(op.N, complex)
    u[p] = u_or
    ud = torch.tensor(u, dtype=torch.complex128, device="cuda")
    vd = torch.empty_like(ud)
    op.apply(ud, vd)
    torch.cuda.synchronize()
    v = vd.cpu().numpy()[p]
    assert np.linalg.norm(v - v_or) / np.linalg.norm(v_or) < 1e-8
    # zero in, zero out (exactly)
    z = torch.zeros_like(ud)
    vz = torch.ones_like(ud)
    op.apply(z, vz)
    torch.cuda.synchronize()
    assert torch.count_nonzero(vz).item() == 0
    # invalid calls are reported, not executed
    with pytest.raises(binding.LSError):
        op.apply(ud, ud)                      # u and v overlap
    with pytest.raises(ValueError):
        op.apply(ud[:10], vd[:10])            # wrong length


def test_batched_schedules_apply_the_same_operator():
    """After tuning for 32 right-hand sides (the batched row kernel and the
    wide interior contraction are candidates), a 32-vector single-precision
    apply matches the double-precision apply of every vector to FP32
    accuracy."""
    import torch
    from paper_1509_05063_amd import binding
    cfg = config("star_k16pi")
    op = _op(cfg)
    ch = op.autotune(32, binding.LS_C64)
    print(f"tuned for 32 right-hand sides: {ch}", flush=True)
    xy, _ = op.points()
    U = torch.tensor(np.stack([plane_wave(cfg, xy, 2 * np.pi * r / 32) for r in range(32)]), dtype=torch.complex128,
                     device="cuda")
    V64 = torch.empty_like(U)
    op.apply(U, V64)
    U32 = U.to(torch.complex64)
    V32 = torch.empty_like(U32)
    op.apply(U32, V32)
    torch.cuda.synchronize()
    err = (torch.linalg.norm(V32.to(torch.complex128) - V64, dim=1) / torch.linalg.norm(V64, dim=1)).max().item()
    assert err < F32_TOL, err
    op.close()
