"""Graph-captured Arnoldi steps: a solve that replays captured HIP graphs
gives bitwise the result of the same solve launched eagerly, on every replay,
with eager solves and host synchronisations in between."""
import time

import numpy as np
import pytest

from paper_1509_05063_amd.inputs import config, n2_function, plane_wave, serving_pool

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def disc_op():
    import torch
    from paper_1509_05063_amd import binding
    assert torch.cuda.is_available()
    cfg = config("disc_k2pi")
    op = binding.Operator(cfg, n2_function(cfg))
    xy, _ = op.points()
    return cfg, op, xy


@pytest.mark.parametrize("mode,ortho,restart,nrhs", [(0, 0, 100, 1), (1, 0, 100, 1), (1, 1, 100, 1), (1, 0, 7, 1),
                                                     (0, 1, 7, 3), (1, 0, 30, 3)])
def test_graph_solve_equals_eager(disc_op, mode, ortho, restart, nrhs):
    import torch
    cfg, op, xy = disc_op
    F = torch.tensor(np.stack([plane_wave(cfg, xy, 0.4 * k) for k in range(nrhs)]), dtype=torch.complex128,
                     device="cuda")
    kw = dict(tol=1e-10, restart=restart, max_iter=3000, mode=mode, inner_tol=1e-5, ortho=ortho)
    x_eager = torch.empty_like(F)
    s_eager = op.solve(F, x_eager, graph=False, **kw)
    for rep in range(3):
        x_graph = torch.empty_like(F)
        s_graph = op.solve(F, x_graph, graph=True, **kw)
        torch.cuda.synchronize()
        assert s_graph["iterations"] == s_eager["iterations"] and s_graph["converged"] == nrhs, (s_graph, s_eager)
        assert torch.equal(x_graph, x_eager), f"replay {rep}"
        # eager work between replays
        x_again = torch.empty_like(F)
        op.solve(F, x_again, graph=False, **kw)
        assert torch.equal(x_again, x_eager)


def test_graph_solve_small_operator_timing():
    """Serving-size operator: eager and graph-replayed solves agree bitwise;
    prints both times (launch overhead dominates at this size)."""
    import torch
    from paper_1509_05063_amd import binding
    cfg = [c for c in serving_pool() if 1 / c["h"] <= 64][0]
    op = binding.Operator(cfg, n2_function(cfg))
    xy, _ = op.points()
    f = torch.tensor(plane_wave(cfg, xy, 0.3), dtype=torch.complex128, device="cuda")
    kw = dict(tol=1e-7, restart=60, max_iter=3000, mode=binding.LS_SOLVE_FP32_REFINE, inner_tol=1e-4,
              ortho=binding.LS_ORTHO_CGS1)
    xs = {}
    times = {}
    for graph in (False, True, False, True):
        x = torch.empty_like(f)
        op.solve(f, x, graph=graph, **kw)         # warm (captures on the first graph solve)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = op.solve(f, x, graph=graph, **kw)
        times[graph] = time.perf_counter() - t0
        xs.setdefault(graph, x)
        assert torch.equal(x, xs[graph])
    assert torch.equal(xs[True], xs[False])
    print(f"N={op.N} iterations {st['iterations']}: eager {times[False] * 1e3:.1f} ms, "
          f"graph {times[True] * 1e3:.1f} ms", flush=True)
    op.close()


def test_graph_solve_refined_operator_equals_eager():
    """The Fourier refined operator (its line refinement runs inside every
    apply): graph-replayed solves equal the eager solve bitwise, on every
    replay, with eager work in between; the allocation-free apply equals
    the workspace apply bitwise."""
    import torch
    from paper_1509_05063_amd import binding
    from paper_1509_05063_amd.inputs import scaled
    cfg = scaled(config("disc_k2pi"), fft_refine=2)
    op = binding.Operator(cfg, n2_function(cfg))
    xy, _ = op.points()
    F = torch.tensor(np.stack([plane_wave(cfg, xy, 0.5 * k) for k in range(2)]), dtype=torch.complex128,
                     device="cuda")
    kw = dict(tol=1e-10, restart=40, max_iter=3000, mode=binding.LS_SOLVE_FP32_REFINE, inner_tol=1e-5)
    x_eager = torch.empty_like(F)
    s_eager = op.solve(F, x_eager, graph=False, **kw)
    assert s_eager["converged"] == 2
    for rep in range(3):
        x_graph = torch.empty_like(F)
        s_graph = op.solve(F, x_graph, graph=True, **kw)
        torch.cuda.synchronize()
        assert s_graph["iterations"] == s_eager["iterations"], (s_graph, s_eager)
        assert torch.equal(x_graph, x_eager), f"replay {rep}"
        x_again = torch.empty_like(F)
        op.solve(F, x_again, graph=False, **kw)
        assert torch.equal(x_again, x_eager)
    for dt in (torch.complex64, torch.complex128):
        u = F.to(dt)
        v1, v2 = torch.empty_like(u), torch.empty_like(u)
        op.apply(u, v1)
        op.apply_noalloc(u, v2)
        torch.cuda.synchronize()
        assert torch.equal(v1, v2), dt
    op.close()
