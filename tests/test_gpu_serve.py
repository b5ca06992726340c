"""Serving loop on the GPU (ls_server_* through the Python face):
continuous batching over resident operators under an HBM budget; each result
is the same alone and in the mix."""
import numpy as np
import pytest

from paper_1509_05063_amd.inputs import plane_wave, serving_pool, serving_trace

pytestmark = pytest.mark.gpu


def _one_op_budget(pool):
    """A budget that holds any one of the pool's operators with a solve of
    four right-hand sides but not two operators with a solve of one."""
    from paper_1509_05063_amd import binding
    from paper_1509_05063_amd.inputs import n2_function
    need = []
    for c in pool:
        op = binding.Operator(dict(c, skip_tiles=1), n2_function(c))
        need.append((op.resident_bytes(), op.solve_workspace_bytes(1, restart=60) + 32 * op.N,
                     op.solve_workspace_bytes(4, restart=60) + 128 * op.N))
        op.close()
    budget = max(a + c for a, _, c in need)
    print(f"pool sizes (operator, solve of 1, solve of 4): {need}, budget {budget}", flush=True)
    assert 2 * min(a for a, _, _ in need) + min(b for _, b, _ in need) > budget
    return budget


@pytest.mark.parametrize("budget_gb,workers", [(40, 3), (None, 2)])
def test_serving_mix_equals_solo(budget_gb, workers):
    from paper_1509_05063_amd.serve import Server, latency_stats, replay
    pool = [c for c in serving_pool() if 1 / c["h"] <= 64]      # the small scatterers (~17k unknowns)
    trace = serving_trace(pool, 40, rate=50.0)
    if budget_gb is None:
        budget_gb = _one_op_budget(pool) / 1e9
    srv = Server(budget_bytes=budget_gb * 1e9, max_batch=8, workers=workers)
    try:
        reqs, wall = replay(srv, trace)
        st = latency_stats(reqs)
        print(f"budget {budget_gb} GB: {st} wall {wall:.2f}s server {srv.info()}", flush=True)
        bad = [(r.key, r.stats) for r in reqs if r.stats["converged"] != r.batch]
        assert not bad, bad[:3]
        assert st["mean_batch"] > 1.0            # requests that arrived during a solve were batched
        if budget_gb < 1:
            assert srv.evictions > 0             # only one operator fits: they are evicted and rebuilt
        # the same requests again, one at a time on an idle server
        checked = 0
        for r in reqs:
            if r.batch > 1 and checked < 6:
                t = srv.submit(r.key, r.cfg, r.alpha)
                srv.drain()
                alone = srv.tickets[t]
                assert alone.batch == 1
                if budget_gb >= 1:
                    assert np.array_equal(alone.result, r.result), np.abs(alone.result - r.result).max()
                else:      # the operator may have been evicted and rebuilt in between
                    assert np.allclose(alone.result, r.result, rtol=0, atol=1e-12 * np.abs(r.result).max())
                checked += 1
        assert checked > 0
    finally:
        srv.close()


def test_server_results_solve_the_scatterer():
    """A served request's total field equals the oracle's dense LU solution
    of the same plane wave (nodes matched by key) and the operator solve in
    the library's point order."""
    import torch
    from oracle.op2d import Setup2D
    from paper_1509_05063_amd import binding
    from paper_1509_05063_amd.inputs import config, match_keys, n2_function
    from paper_1509_05063_amd.serve import Server
    cfg = config("disc_k2pi")
    srv = Server(budget_bytes=10e9, max_batch=4, workers=1, tol=1e-10, inner_tol=1e-5)
    try:
        tickets = [srv.submit("disc", cfg, a) for a in (0.0, 0.7, 1.9)]
        srv.drain()
        xy = srv.points("disc")
        op = binding.Operator(cfg, n2_function(cfg))
        xo, key = op.points()
        assert np.array_equal(xy, xo)
        orc = Setup2D(cfg, n2_function(cfg))
        p = match_keys(orc.pts["key"], key)
        A = orc.dense_A()
        for t in tickets:
            r = srv.tickets[t]
            assert r.status == binding.LS_OK and r.stats["converged"] == r.batch
            u_or = np.linalg.solve(A, plane_wave(cfg, orc.pts["x"], r.alpha))
            e_or = np.linalg.norm(r.result[p] - u_or) / np.linalg.norm(u_or)
            f = torch.tensor(plane_wave(cfg, xo, r.alpha), dtype=torch.complex128, device="cuda")
            x = torch.empty_like(f)
            op.solve(f, x, tol=1e-10, restart=60, max_iter=4000, mode=binding.LS_SOLVE_FP64)
            ref = x.cpu().numpy()
            err = np.linalg.norm(r.result - ref) / np.linalg.norm(ref)
            print(f"served alpha {r.alpha}: batch {r.batch}, vs oracle LU {e_or:.2e}, vs op solve {err:.2e}",
                  flush=True)
            assert e_or < 1e-8, e_or
            assert err < 1e-8, err
        op.close()
    finally:
        srv.close()


def test_server_rejects_an_operator_over_budget():
    """An operator whose data and one-right-hand-side solve alone exceed the
    budget is not run: its requests finish with LS_EBUDGET, and a scatterer
    that fits is still served."""
    from paper_1509_05063_amd import binding
    from paper_1509_05063_amd.inputs import config, scaled
    from paper_1509_05063_amd.serve import Server
    small = scaled(config("disc_k2pi"), h=1 / 16, band={"N1": 32, "N2": 8}, r_int=6 / 16, r1=6.0, r2=4.0)
    big = config("star_k16pi")
    # 300 MB: the small operator (about 1k unknowns) and its solve fit; the
    # 270k-unknown star (estimated at 8 kB per unknown before it is built)
    # does not, so it is never built
    srv = Server(budget_bytes=300e6, max_batch=2, workers=1, tol=1e-8)
    try:
        tb = srv.submit("big", big, 0.0)
        ts = srv.submit("small", small, 0.0)
        srv.drain()
        rb, rs = srv.tickets[tb], srv.tickets[ts]
        print(f"over budget: {rb.status}, fitting: {rs.status} {rs.stats}", flush=True)
        assert rb.status == binding.LS_EBUDGET
        assert rs.status == binding.LS_OK
    finally:
        srv.close()
