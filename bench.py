"""Benchmark of the FFT-accelerated Lippmann–Schwinger solve on one MI355X.

A step is one full pass of the hot path on the workload: a GMRES solve of
(I + kappa^2 K_h) u = u^i whose every iteration runs the whole operator
apply (projection, FFT convolution, cell interpolation, near-field
correction with the adjacency subtraction folded in, combine) in single
precision inside double-precision iterative refinement (FP64 residual and
Arnoldi).

Prints one JSON line (rank 0):  metric / value = solves per second at
<= 1e-6 relative error against the double-precision reference solve, plus
matvec rates, solve latency percentiles, the roofline of the dominant kernel
(timed with HIP events on the apply's stream) and the CPU oracle timed on a
bounded sample of rows.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def stage_bytes(st, N, n_int, s, s_w, csr_variant=0):
    """Algorithmic bytes per apply of each stage for one right-hand side
    (what the method has to move; s bytes per complex value of the data,
    s_w per stored complex weight).  The near-field rows' column information
    is what the chosen row format stores: a 16-bit offset per entry, or
    8 bytes (start column, first entry) per run of consecutive columns."""
    Pa, Pb, ncell, U, F, S, Wn = st["Pa"], st["Pb"], st["ncell"], st["U"], st["F"], st["S"], st["Wn"]
    nb = st["n_band"]
    na = st["L"] + 1
    plane = Pa * Pb
    r = s // 2            # real bytes
    return {
        "project": N * (s + r) + nb * U * s_w + U * S * s_w + ncell * U * s,
        "fill": ncell * U * s + 4 * plane * s,
        "fft_fwd": 4 * (na * Pb + plane) * 2 * s,
        "spectral": 2 * (2 + 2 + 1) * plane * s,
        "fft_inv": 2 * (plane + na * Pb) * 2 * s,
        "interp": ncell * F * s + nb * F * s_w + S * F * s_w + 2 * N * s,
        "near_shared": S * Wn * Wn * s_w + n_int * (s + r) + 2 * n_int * s,
        "near_csr": (st["csr_nnz"] * (s_w + 2) + st["csr_rows"] * (8 + 4 + 4 + 2 * s) + N * s
                     if csr_variant not in (2, 3, 4) else
                     st["csr_nnz"] * s_w + st["csr_runs"] * 8 + st["csr_rows"] * (8 + 4 + 4 + 2 * s) + N * s),
    }


# single-precision kernel of each one-kernel stage (the FFT stages run several)
STAGE_KERNEL = {"project": "k_project_int<float,true>", "fill": "k_fill<float>", "spectral": "k_spectral<float>",
                "interp": "k_interp_mfma<float,16>", "near_shared": "k_near_shared_mfma_db<1,false>",
                "near_csr": "k_near_csr4"}


def counter_traffic(kernel, summary=os.path.join(ROOT, "profiles", "apply_star_k32pi.md")):
    """HBM bytes per dispatch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel calibration),
    or None when the summary is missing or was taken on a different kernel
    source than the one built here."""
    import hashlib
    src = os.path.join(ROOT, "paper_1509_05063_amd", "csrc", "ls_kernels.hip")
    try:
        text = open(summary).read()
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    if f"ls_kernels.hip sha256: {digest}" not in text:
        return None
    for line in text.splitlines():
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) == 4 and cells[0] == kernel:
            return int(round((float(cells[1]) + float(cells[2])) * 2 ** 20))
    return None


def host_cpu():
    """Host CPU model and the threads the oracle legs use."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, max(1, min(16, os.cpu_count() or 1))


def cpu_oracle_rate(cfg, n2, budget_s=15.0, x_ref=None, f_ref=None, key_lib=None):
    """Oracle rows per second on a bounded sample of targets, the rows
    spread over the host's cores (numpy releases the interpreter lock inside
    its array kernels, so threads run the rows side by side).  With the
    double-precision reference solution x_ref (library order, keys key_lib)
    and its right-hand side f_ref, the same rows also give the oracle's
    residual A x_ref - f on them (relative to max |f|)."""
    from concurrent.futures import ThreadPoolExecutor

    from oracle.op2d import Setup2D
    from paper_1509_05063_amd.inputs import match_keys
    t0 = time.time()
    orc = Setup2D(cfg, n2)
    log(f"oracle discretisation {time.time() - t0:.1f}s, N={orc.N}")
    x_or = f_or = None
    if x_ref is not None:
        p = match_keys(orc.pts["key"], key_lib)
        x_or, f_or = x_ref[p], f_ref[p]
    rng = np.random.default_rng(1509)
    rows = rng.choice(orc.N, 4096, replace=False)
    _, nth = host_cpu()
    deadline = time.time() + budget_s
    res = {}

    def work(chunk):
        out = []
        for i in chunk:
            if time.time() > deadline:
                break
            row = orc.A_rows([int(i)])[0]
            out.append((int(i), row @ x_or - f_or[i] if x_or is not None else row.sum()))
        return out

    t0 = time.time()
    with ThreadPoolExecutor(nth) as ex:
        for part in ex.map(work, np.array_split(rows, nth)):
            res.update(part)
    dt = time.time() - t0
    resid = None
    if x_or is not None and res:
        resid = max(abs(v) for v in res.values()) / np.abs(f_or).max()
    return len(res) / dt, len(res), orc.N, nth, resid


def cpu_disc_oracle():
    """The oracle on the 4k-unknown disc: the dense operator built row by
    row (one thread: these short rows are interpreter-bound, threads slow
    them down), one matvec with it (ZGEMV, BLAS threads) and the dense LU
    solve."""
    from oracle.op2d import Setup2D
    from paper_1509_05063_amd.inputs import config, n2_function, plane_wave
    cfg = config("disc_k2pi")
    orc = Setup2D(cfg, n2_function(cfg))
    _, nth = host_cpu()
    t0 = time.time()
    A = orc.dense_A()
    t_build = time.time() - t0
    f = plane_wave(cfg, orc.pts["x"], 0.0)
    t0 = time.time()
    for _ in range(5):
        A @ f
    t_mv = (time.time() - t0) / 5
    t0 = time.time()
    np.linalg.solve(A, f)
    t_lu = time.time() - t0
    return {"workload": f"disc_k2pi, N={orc.N}", "blas_threads": nth, "dense_rows_s": round(t_build, 2),
            "matvecs_per_s_dense": round(1 / t_mv, 1), "lu_solve_s": round(t_lu, 2),
            "solves_per_s_incl_rows": round(1 / (t_build + t_lu), 4)}


def multi_rhs_profile(nrhs, reps):
    """Profiling run: the kappa = 16 pi star's batched single-precision apply
    (tuned for nrhs right-hand sides), reps staged applies."""
    import torch
    from paper_1509_05063_amd import binding
    from paper_1509_05063_amd.inputs import config, n2_function, plane_wave
    cfg = config("star_k16pi")
    op = binding.Operator(cfg, n2_function(cfg))
    try:
        tune = op.autotune(nrhs, binding.LS_C64)
        xy, _ = op.points()
        F = torch.tensor(np.stack([plane_wave(cfg, xy, 2 * math.pi * r / nrhs) for r in range(nrhs)]),
                         dtype=torch.complex64, device="cuda")
        V = torch.empty_like(F)
        acc = None
        for _ in range(reps):
            p = op.apply_profile(F, V)
            acc = p if acc is None else {k: acc[k] + p[k] for k in p}
        torch.cuda.synchronize()
        return {"schedule": tune, "stage_ms": {k: v / reps for k, v in acc.items()}}
    finally:
        op.close()


def multi_rhs_run(nrhs, ortho, autotune):
    """Batched solves on the kappa = 16 pi star: nrhs equispaced incident
    directions as the right-hand sides of one solve (FP64 reference, then the
    single-precision + refinement form), RHS-solves/s and the worst error."""
    import torch
    from paper_1509_05063_amd import binding
    from paper_1509_05063_amd.inputs import config, n2_function, plane_wave
    cfg = config("star_k16pi")
    op = binding.Operator(cfg, n2_function(cfg))
    try:
        if autotune:
            op.autotune(nrhs, binding.LS_C64)
            op.autotune(nrhs, binding.LS_C128)
        xy, _ = op.points()
        F = torch.tensor(np.stack([plane_wave(cfg, xy, 2 * math.pi * r / nrhs) for r in range(nrhs)]),
                         dtype=torch.complex128, device="cuda")
        g = cfg["gmres"]
        # stage times of one batched single-precision apply (HIP events)
        F32 = F.to(torch.complex64)
        V32 = torch.empty_like(F32)
        op.apply_profile(F32, V32)
        stages = op.apply_profile(F32, V32)
        apply_ms = sum(stages.values())
        del F32, V32
        X64, X32 = torch.empty_like(F), torch.empty_like(F)
        t0 = time.perf_counter()
        s64 = op.solve(F, X64, tol=1e-10, restart=g["restart"], max_iter=3000, mode=binding.LS_SOLVE_FP64)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t0
        t0 = time.perf_counter()
        s32 = op.solve(F, X32, tol=1e-7, restart=g["restart"], max_iter=3000, mode=binding.LS_SOLVE_FP32_REFINE,
                       inner_tol=1e-4, max_outer=30, ortho=ortho)
        torch.cuda.synchronize()
        t32 = time.perf_counter() - t0
        err = ((torch.linalg.norm(X32 - X64, dim=1) / torch.linalg.norm(X64, dim=1)).max()).item()
        # the plain double-precision form at the same tolerance as the timed one
        Xp = torch.empty_like(F)
        t0 = time.perf_counter()
        sp = op.solve(F, Xp, tol=1e-7, restart=g["restart"], max_iter=3000, mode=binding.LS_SOLVE_FP64)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
        errp = ((torch.linalg.norm(Xp - X64, dim=1) / torch.linalg.norm(X64, dim=1)).max()).item()
        return {"workload": f"star_k16pi, N={op.N}, {nrhs} incident directions", "nrhs": nrhs,
                "rhs_solves_per_s": nrhs / t32, "seconds": t32, "iterations": s32["iterations"],
                "max_err_vs_fp64_ref": err, "fp64_tol1e-7_rhs_solves_per_s": nrhs / tp,
                "fp64_tol1e-7_err": errp, "fp64_tol1e-7_iterations": sp["iterations"],
                "fp64_ref_tol1e-10_rhs_solves_per_s": nrhs / t64,
                "fp64_ref_iterations": s64["iterations"], "all_converged": s32["converged"] == nrhs,
                "fp32_apply_ms": apply_ms, "fp32_apply_stage_ms": stages}
    finally:
        op.close()


def serving_run(n_requests, rate=50.0, ortho=None, restart=60, wide=True):
    """Poisson stream of solves over a warm pool of resident operators
    (continuous batching per operator, concurrent solves across operators).
    wide: the 2-D part of the mixed stream (8 stars, N log-uniform in 16k-1M,
    kappa up to 32 pi); else six small stars.  When the offered rate exceeds
    what the server completes, requests queue: reported as the backlog (time
    from the last arrival to the last completion) and the sustained rate."""
    from paper_1509_05063_amd.inputs import serving_pool, serving_pool_wide, serving_trace
    from paper_1509_05063_amd.serve import Server, latency_stats, replay
    pool = serving_pool_wide() if wide else serving_pool()
    from paper_1509_05063_amd import binding
    srv = Server(budget_bytes=200e9, max_batch=16, workers=4, keep_results=False, restart=restart,
                 ortho=binding.LS_ORTHO_CGS1 if ortho is None else ortho)
    try:
        t0 = time.time()
        for c in pool:                      # warm: build every operator once
            srv.submit(c["name"], c, 0.0)
        srv.drain()
        warm = time.time() - t0
        warm_stats = {r.key: (r.N, r.stats["iterations"], round(r.latency * 1e3, 1)) for r in srv.tickets.values()}
        srv.tickets.clear()
        trace = serving_trace(pool, n_requests, rate=rate)
        reqs, wall = replay(srv, trace)
        st = latency_stats(reqs)
        conv = sum(1 for r in reqs if r.stats["converged"] == r.batch)
        iters, lat_by = {}, {}
        for r in reqs:
            iters[r.key] = max(iters.get(r.key, 0), r.stats["iterations"])
            lat_by.setdefault(r.key, []).append((r.done - r.arrival) * 1e3)
        t_first = min(r.arrival for r in reqs)
        last_arrival = max(r.arrival for r in reqs) - t_first
        last_done = max(r.done for r in reqs) - t_first
        return {"requests": len(reqs), "rate_per_s": rate, "operators": len(pool),
                "N_range": [min(r.N for r in reqs), max(r.N for r in reqs)],
                "kappa_over_pi_range": [round(min(c["kappa"] for c in pool) / math.pi, 2),
                                        round(max(c["kappa"] for c in pool) / math.pi, 2)],
                "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"], "mean_batch": st["mean_batch"],
                "solves_per_s": len(reqs) / wall, "sustained_solves_per_s": len(reqs) / last_done,
                "backlog_s": last_done - last_arrival, "all_converged": conv == len(reqs), "warmup_s": warm,
                "solo_N_iterations_ms": warm_stats, "max_iterations": iters,
                "median_latency_ms_by_scatterer": {k: round(float(np.median(v)), 1) for k, v in lat_by.items()}}
    finally:
        srv.close()


SPHERE_LATTICE = dict(na=33, nb=128, nc=128, hn=4 / 64, ht=1 / 64, kappa=8 * math.pi, nsets=3)


def conv3d_textbook_bytes(Pa, Pb, Pc, nsets):
    """Textbook pencil count of the FFT convolution (complex float): per set
    three full transforms (two forward, one inverse) of three passes, each
    reading and writing the padded volume, plus the two kernel spectra."""
    P = Pa * Pb * Pc
    return 8 * nsets * (3 * 3 * 2 * P + 2 * P)


def conv3d_pass_bytes(na, nb, nc, Pa, Pb, Pc, nsets):
    """Bytes the implemented passes have to move (complex float): padding
    rows are neither read nor written.  Per array (2 nsets: both kinds of
    every set) lines along c read straight from the compact strengths, then
    columns along b; per set the fused pass along a (both kinds' na rows and
    the one stored octant of each of the two kernel spectra in, kind 0's na
    rows out), then columns along b and lines along c written straight into
    the compact field (kind 0)."""
    e = 8
    octant = (Pa // 2 + 1) * (Pb // 2 + 1) * (Pc // 2 + 1)
    fwd = (na * nb * nc + na * nb * Pc) + (na * nb * Pc + na * Pb * Pc)
    conv = 2 * na * Pb * Pc + 2 * octant + na * Pb * Pc
    inv = (na * Pb * Pc + na * nb * Pc) + (na * nb * Pc + na * nb * nc)
    return e * (2 * nsets * fwd + nsets * (conv + inv))


def conv3d_run(reps):
    """The 3-D method's FFT convolution step (monopole + dipole face-lattice
    sums, Sec. 3.2) on the face lattices of the unit-sphere workload
    (kappa = 8 pi, h = 1/64, cells of 4 h, 4 nodes per face edge): three
    sets of 33 x 128 x 128 nodes.  Timed with HIP events on the stream the
    library launches on (torch's current stream)."""
    import torch
    from paper_1509_05063_amd import binding
    L = SPHERE_LATTICE
    c = binding.Conv3D(L["na"], L["nb"], L["nc"], L["hn"], L["ht"], L["kappa"], L["nsets"])
    Pa, Pb, Pc = c.padded
    sched = c.autotune()
    g = torch.Generator(device="cuda").manual_seed(1509)
    sig = torch.randn(L["nsets"], 2, L["na"], L["nb"], L["nc"], dtype=torch.complex64, device="cuda", generator=g)
    fld = torch.empty(L["nsets"], L["na"], L["nb"], L["nc"], dtype=torch.complex64, device="cuda")
    st = torch.cuda.current_stream()
    for _ in range(reps):       # untimed: a cold GPU's clocks ramp up over the first milliseconds
        c.apply(sig, fld)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        c.apply(sig, fld)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    byts = conv3d_textbook_bytes(Pa, Pb, Pc, L["nsets"])
    pbyts = conv3d_pass_bytes(L["na"], L["nb"], L["nc"], Pa, Pb, Pc, L["nsets"])
    gbs, pgbs = byts / (ms * 1e-3) / 1e9, pbyts / (ms * 1e-3) / 1e9
    # achieved / frac: the bytes the implemented passes must move (a lower
    # bound on their HBM traffic); textbook_*: the pencil count of three
    # unfused padded transforms per set, for comparison with that design
    out = {"stage": "fft3d", "bound": "hbm", "achieved": round(pgbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
           "frac": round(pgbs / PEAK_HBM_GBS, 4), "algorithmic_bytes": int(pbyts), "avg_ms": round(ms, 4),
           "textbook_bytes": int(byts), "textbook_gbs": round(gbs, 1), "textbook_frac": round(gbs / PEAK_HBM_GBS, 4),
           "lattice": f"{L['nsets']} sets x {L['na']}x{L['nb']}x{L['nc']} padded to {Pa}x{Pb}x{Pc}",
           "workspace_gb": c.ws_bytes / 1e9,
           "schedule": {"normal_tile": sched[0], "normal_threads": sched[1], "second_tile": sched[2],
                        "plane_skew": sched[3]}}
    c.close()
    return out


def fft256_run(reps):
    """The dense 3-D complex FFT of the sphere workload's 256^3 equivalent-
    source grid (complex float, in place): forward and inverse transforms
    timed with HIP events on torch's current stream.  Textbook bytes per
    transform: three one-axis passes, each reading and writing the cube."""
    import torch
    from paper_1509_05063_amd import binding
    n = 256
    f = binding.FFT3D(n, n, n)
    g = torch.Generator(device="cuda").manual_seed(256)
    a = torch.randn(n, n, n, dtype=torch.complex64, device="cuda", generator=g)
    st = torch.cuda.current_stream()
    for _ in range(reps):       # untimed: a cold GPU's clocks ramp up over the first milliseconds
        f.exec(a, 1)
        f.exec(a, -1)
        a.mul_(1.0 / n ** 3)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        f.exec(a, 1)
        f.exec(a, -1)
        a.mul_(1.0 / n ** 3)    # keep the values bounded (a scaling kernel, timed apart below)
    e1.record(st)
    torch.cuda.synchronize()
    tot = e0.elapsed_time(e1)
    e0.record(st)
    for _ in range(reps):
        a.mul_(1.0)
    e1.record(st)
    torch.cuda.synchronize()
    ms = (tot - e0.elapsed_time(e1)) / (2 * reps)
    byts = 3 * 2 * n ** 3 * 8
    gbs = byts / (ms * 1e-3) / 1e9
    f.close()
    return {"stage": "fft256", "bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(gbs / PEAK_HBM_GBS, 4), "algorithmic_bytes": byts, "avg_ms": round(ms, 4),
            "grid": "256^3 complex float, in place, one transform (forward and inverse averaged)"}


def refined_run(cfg, n2, f, x_ref, r, ortho, autotune, interior=False, shortcut=False):
    """The same workload with Fourier refined interpolation along the band's
    t1 lines (fft_refine = r), and with interior=True of the interior lattice
    too: set-up, tuned applies, per-stage times of the single-precision apply
    (the band refinement runs inside the rows stage, the interior one inside
    the interior contraction's) and the timed solve form; with shortcut=True
    the interior lattice nodes inside the boundary patch interpolate the
    boundary rule's values at the patch's grid nodes (computed first in the
    rows stage) instead of evaluating it.  Its solution
    against the unrefined FP64 reference (the change the refinement makes to
    the discretisation)."""
    import torch
    from paper_1509_05063_amd import binding
    from paper_1509_05063_amd.inputs import scaled
    c = scaled(cfg, fft_refine=r, fft_refine_interior=int(interior), offgrid_shortcut=int(shortcut))
    t0 = time.time()
    op = binding.Operator(c, n2)
    setup_s = time.time() - t0
    st = op.stats()
    out = {"fft_refine": r, "interior": interior, "offgrid_shortcut": shortcut, "setup_s": round(setup_s, 1), "resident_gb": op.resident_bytes() / 1e9,
           "csr_nnz": int(st["csr_nnz"])}
    try:
        if autotune:
            out["autotune"] = {"fp32": op.autotune(1, binding.LS_C64), "fp64": op.autotune(1, binding.LS_C128)}
        for name, dt in [("fp64", torch.complex128), ("fp32", torch.complex64)]:
            u = f.to(dt)
            v = torch.empty_like(u)
            op.apply(u, v)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(20):
                op.apply(u, v)
            torch.cuda.synchronize()
            out[f"matvecs_per_s_{name}"] = 20 / (time.perf_counter() - t1)
        u = f.to(torch.complex64)
        v = torch.empty_like(u)
        acc = None
        for _ in range(10):
            p = op.apply_profile(u, v)
            acc = p if acc is None else {k: acc[k] + p[k] for k in p}
        out["stage_ms_fp32"] = {k: acc[k] / 10 for k in acc}
        g = c["gmres"]
        x = torch.empty_like(f)
        ts = []
        for _ in range(3):
            t1 = time.perf_counter()
            info = op.solve(f, x, tol=1e-7, restart=g["restart"], max_iter=3000, mode=binding.LS_SOLVE_FP32_REFINE,
                            inner_tol=1e-4, max_outer=30, ortho=ortho)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t1)
        out["solves_per_s"] = 1.0 / min(ts)
        out["iterations"] = info["iterations"]
        out["converged"] = info["converged"]
        out["diff_vs_unrefined_fp64_ref"] = (torch.linalg.norm(x - x_ref) / torch.linalg.norm(x_ref)).item()
    finally:
        op.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="star_k32pi")
    ap.add_argument("--matvec-reps", type=int, default=20)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-disc-oracle", action="store_true",
                    help="skip the dense oracle timing on the 4k-unknown disc in the CPU baseline")
    ap.add_argument("--serving-requests", type=int, default=300,
                    help="requests in the serving measurement (0 skips it)")
    ap.add_argument("--serving-rate", type=float, default=50.0, help="mean Poisson arrival rate (requests/s)")
    ap.add_argument("--serving-small", action="store_true",
                    help="serve the six small stars (16.7k-230k unknowns) instead of the wide 2-D mix")
    ap.add_argument("--serving-only", action="store_true", help="run only the serving measurement")
    ap.add_argument("--ortho", choices=["cgs1", "cgs2"], default="cgs1",
                    help="Gram-Schmidt passes per Arnoldi step of the single-precision inner solves")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default kernel schedules")
    ap.add_argument("--fft-refine", type=int, default=1,
                    help="profiling runs: build the main operator with this Fourier refinement factor")
    ap.add_argument("--fft-refine-interior", action="store_true",
                    help="profiling runs: refine the interior lattice as well")
    ap.add_argument("--offgrid-shortcut", action="store_true",
                    help="profiling runs: the off-grid shortcut for the boundary patch's interior lattice nodes")
    ap.add_argument("--refine", type=int, default=2,
                    help="refinement factor of the Fourier refined interpolation measured on the same workload "
                         "(0 skips it)")
    ap.add_argument("--multi-rhs", type=int, default=256,
                    help="right-hand sides of the batched measurement on the kappa = 16 pi star (0 skips it)")
    ap.add_argument("--profile-solve", action="store_true",
                    help="profiling run: one single-precision-with-refinement solve only")
    ap.add_argument("--profile-applies", type=int, default=0,
                    help="profiling run: only this many staged applies per precision plus a 512 MiB "
                         "device copy (the calibration kernel for HBM byte counters)")
    ap.add_argument("--fft3d-reps", type=int, default=20,
                    help="applies of the 3-D face-lattice convolution in its measurement (0 skips it)")
    ap.add_argument("--profile-multi", type=int, default=0,
                    help="profiling run: only this many batched single-precision applies on the kappa = 16 pi star "
                         "(--multi-rhs right-hand sides)")
    ap.add_argument("--profile-fft3d", type=int, default=0,
                    help="profiling run: only this many 3-D face-lattice convolutions")
    ap.add_argument("--fft256-reps", type=int, default=20,
                    help="forward + inverse pairs of the 256^3 transform in its measurement (0 skips it)")
    ap.add_argument("--profile-fft256", type=int, default=0,
                    help="profiling run: only this many forward + inverse pairs of the 256^3 transform")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the solve is not sharded across GPUs",
              file=sys.stderr)
        sys.exit(2)

    if args.profile_fft3d:
        log(f"profile fft3d {conv3d_run(args.profile_fft3d)}")
        import torch
        a = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)          # the calibration kernel for HBM byte counters
        torch.cuda.synchronize()
        return
    if args.profile_multi:
        log(f"profile multi {multi_rhs_profile(args.multi_rhs, args.profile_multi)}")
        return
    if args.profile_fft256:
        log(f"profile fft256 {fft256_run(args.profile_fft256)}")
        return
    if args.serving_only:
        log(f"serving {serving_run(args.serving_requests, rate=args.serving_rate, wide=not args.serving_small)}")
        return

    import torch
    from paper_1509_05063_amd import binding
    from paper_1509_05063_amd.inputs import config, n2_function, plane_wave

    cfg = config(args.config)
    if args.fft_refine > 1:
        if not (args.profile_applies or args.profile_solve):
            print("--fft-refine is for the profiling runs; the full run measures the refined operator itself "
                  "(--refine)", file=sys.stderr)
            sys.exit(2)
        from paper_1509_05063_amd.inputs import scaled
        cfg = scaled(cfg, fft_refine=args.fft_refine, fft_refine_interior=int(args.fft_refine_interior),
                     offgrid_shortcut=int(args.offgrid_shortcut))
    n2 = n2_function(cfg)
    log(f"create {args.config}")
    t0 = time.time()
    op = binding.Operator(cfg, n2)
    setup_s = time.time() - t0
    st = op.stats()
    log(f"setup {setup_s:.1f}s stats {st}")
    xy, key = op.points()
    N = op.N
    n_int = int((key[:, 0] == 0).sum())
    f = torch.tensor(plane_wave(cfg, xy, cfg["incidence"][0]), dtype=torch.complex128, device="cuda")
    tune = None
    if not args.no_autotune:
        t0 = time.time()
        tune = {"fp32": op.autotune(1, binding.LS_C64), "fp64": op.autotune(1, binding.LS_C128)}
        log(f"autotune {time.time() - t0:.1f}s {tune}")
    if args.profile_applies:
        # the staged apply (stages in order on one stream, as the roofline
        # figures are timed), not the concurrent one the solves use
        for dt in (torch.complex64, torch.complex128):
            u = f.to(dt)
            v = torch.empty_like(u)
            for _ in range(args.profile_applies):
                op.apply_profile(u, v)
            torch.cuda.synchronize()
        a = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"profile run done: {args.profile_applies} applies per precision, copy of {a.numel()} bytes")
        return
    g = cfg["gmres"]
    ortho = binding.LS_ORTHO_CGS1 if args.ortho == "cgs1" else binding.LS_ORTHO_CGS2
    if args.profile_solve:
        x = torch.empty_like(f)
        info = op.solve(f, x, tol=1e-7, restart=g["restart"], max_iter=3000,
                        mode=binding.LS_SOLVE_FP32_REFINE, inner_tol=1e-4, max_outer=30, ortho=ortho)
        log(f"profile solve {info}")
        return
    x_ref = torch.empty_like(f)
    t0 = time.time()
    ref = op.solve(f, x_ref, tol=1e-10, restart=g["restart"], max_iter=3000, mode=binding.LS_SOLVE_FP64)
    log(f"FP64 reference solve {time.time() - t0:.2f}s {ref}")

    def step(x):
        return op.solve(f, x, tol=1e-7, restart=g["restart"], max_iter=3000,
                        mode=binding.LS_SOLVE_FP32_REFINE, inner_tol=1e-4, max_outer=30, ortho=ortho)

    x = torch.empty_like(f)
    for w in range(args.warmup):
        info = step(x)
        log(f"warmup {w}: {info}")
    torch.cuda.synchronize()
    lat = []
    t_start = time.perf_counter()
    for k in range(args.steps):
        t1 = time.perf_counter()
        info = step(x)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t1)
        log(f"step {k}: {lat[-1] * 1e3:.1f} ms {info}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    err = (torch.linalg.norm(x - x_ref) / torch.linalg.norm(x_ref)).item()
    log(f"error vs FP64 reference solve {err:.3e}")

    # the same single-precision apply inside a complex-double inner Arnoldi
    # (the precision split north of the bulk work: FP64 basis and
    # orthogonalisation, FP32 operator)
    xa = torch.empty_like(f)
    ta = []
    for _ in range(max(1, min(args.steps, 3))):
        t1 = time.perf_counter()
        info_a = op.solve(f, xa, tol=1e-7, restart=g["restart"], max_iter=3000, mode=binding.LS_SOLVE_FP32_REFINE,
                          inner_tol=1e-4, max_outer=30, ortho=ortho, inner_f64_basis=True)
        torch.cuda.synchronize()
        ta.append(time.perf_counter() - t1)
    err_a = (torch.linalg.norm(xa - x_ref) / torch.linalg.norm(x_ref)).item()
    log(f"FP32 apply + FP64 Arnoldi solve {min(ta) * 1e3:.1f} ms err {err_a:.3e} {info_a}")
    # one profiled solve of the timed form: device time per stage
    xp = torch.empty_like(f)
    info_p = op.solve(f, xp, tol=1e-7, restart=g["restart"], max_iter=3000, mode=binding.LS_SOLVE_FP32_REFINE,
                      inner_tol=1e-4, max_outer=30, ortho=ortho, profile=True)
    log(f"profiled solve stage us {info_p['stage_us']}")

    # plain FP64 GMRES form for comparison (same tolerance on the error)
    xf = torch.empty_like(f)
    t1 = time.perf_counter()
    info64 = op.solve(f, xf, tol=1e-7, restart=g["restart"], max_iter=3000, mode=binding.LS_SOLVE_FP64)
    torch.cuda.synchronize()
    t64 = time.perf_counter() - t1
    err64 = (torch.linalg.norm(xf - x_ref) / torch.linalg.norm(x_ref)).item()
    log(f"FP64 plain solve {t64 * 1e3:.1f} ms err {err64:.3e} {info64}")

    # matvec rates
    rates = {}
    for name, dt in [("fp64", torch.complex128), ("fp32", torch.complex64)]:
        u = f.to(dt)
        v = torch.empty_like(u)
        op.apply(u, v)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.matvec_reps):
            op.apply(u, v)
        torch.cuda.synchronize()
        rates[name] = args.matvec_reps / (time.perf_counter() - t1)
        log(f"matvecs/s {name}: {rates[name]:.1f}")

    # per-stage times (HIP events on the apply's stream), single precision
    # (the form the timed solves spend their applies in) and double
    prof = {}
    for name, dt, s, s_w in [("fp32", torch.complex64, 8, 8), ("fp64", torch.complex128, 16, 16)]:
        u = f.to(dt)
        v = torch.empty_like(u)
        acc = None
        reps = 10
        for _ in range(reps):
            p = op.apply_profile(u, v)
            acc = p if acc is None else {k: acc[k] + p[k] for k in p}
        prof[name] = {k: acc[k] / reps for k in acc}
        log(f"stage ms {name}: " + " ".join(f"{k}={v:.3f}" for k, v in prof[name].items()))
    p32 = prof["fp32"]
    dom = max(p32, key=p32.get)
    byts = stage_bytes(st, N, n_int, 8, 8, tune["fp32"]["csr_variant"] if tune else 0)
    achieved = byts[dom] / (p32[dom] * 1e-3) / 1e9
    kname = STAGE_KERNEL.get(dom, dom)
    if tune and dom == "near_csr":
        # (3 and 4, the dense tiles, fall back to the run-length rows for one
        # right-hand side)
        kname = {0: "k_near_csr4", 1: "k_near_csr<float,float2,unsigned short>", 2: "k_near_csr4r", 3: "k_near_csr4r",
                 4: "k_near_csr4r"}[tune["fp32"]["csr_variant"]]
    if tune and dom == "near_shared":
        nv = tune["fp32"]["near_variant"]
        kname = "k_near_shared_mfma<float,2>" if nv == 1 else "k_near_shared_mfma_db<" + {
            0: "1,false", 2: "2,false", 3: "4,false", 4: "4,true"}[nv] + ">"
    alg = byts[dom]
    if dom == "near_csr":
        # per-unit bytes of stored near-field rows (the roofline figure): a weight
        # (8 B, complex float) and a 4-byte column index per stored entry;
        # the run-length kernel moves fewer bytes (kernel_bytes: weights,
        # one 8-byte entry per column run, row data, the input vector)
        alg = st["csr_nnz"] * (8 + 4)
        achieved = alg / (p32[dom] * 1e-3) / 1e9
    roof = {"kernel": kname, "stage": dom, "bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
            "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": counter_traffic(kname),
            "algorithmic_bytes": int(alg), "avg_ms": round(p32[dom], 4),
            "kernel_bytes": int(byts[dom]),
            "kernel_frac": round(byts[dom] / (p32[dom] * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}
    # the FFT convolution stage as a whole (row and column transforms, spectral
    # product): textbook pencil count of its bytes over the three stages' time
    fft_b = byts["fft_fwd"] + byts["spectral"] + byts["fft_inv"]
    fft_ms = p32["fft_fwd"] + p32["spectral"] + p32["fft_inv"]
    fft_gbs = fft_b / (fft_ms * 1e-3) / 1e9
    roof_fft = {"stage": "fft", "bound": "hbm", "achieved": round(fft_gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(fft_gbs / PEAK_HBM_GBS, 4), "algorithmic_bytes": int(fft_b), "avg_ms": round(fft_ms, 4),
                "note": "2-D face lattices (2 sets x 2 kinds x Pa x Pb complex float) fit in the 256 MB MALL"}

    refined = refined_int = refined_sc = None
    if args.refine > 1:
        refined = refined_run(cfg, n2, f, x_ref, args.refine, ortho, not args.no_autotune)
        log(f"refined {refined}")
        refined_int = refined_run(cfg, n2, f, x_ref, args.refine, ortho, not args.no_autotune, interior=True)
        log(f"refined with the interior {refined_int}")
        refined_sc = refined_run(cfg, n2, f, x_ref, args.refine, ortho, not args.no_autotune, shortcut=True)
        log(f"refined with the off-grid shortcut {refined_sc}")

    fft3d = None
    if args.fft3d_reps:
        fft3d = conv3d_run(args.fft3d_reps)
        log(f"fft3d {fft3d}")

    fft256 = None
    if args.fft256_reps:
        fft256 = fft256_run(args.fft256_reps)
        log(f"fft256 {fft256}")

    multi = None
    if args.multi_rhs:
        multi = multi_rhs_run(args.multi_rhs, ortho, not args.no_autotune)
        log(f"multi-rhs {multi}")

    serving = None
    if args.serving_requests:
        serving = serving_run(args.serving_requests, rate=args.serving_rate, ortho=ortho, wide=not args.serving_small)
        log(f"serving {serving}")

    cpu = None
    if not args.no_cpu_baseline:
        model, _ = host_cpu()
        rows_s, nrows, N_or, nth, resid = cpu_oracle_rate(cfg, n2, args.cpu_budget, x_ref=x_ref.cpu().numpy(),
                                                          f_ref=f.cpu().numpy(), key_lib=key)
        mv = rows_s / N_or
        applies_per_solve = info["iterations"] + info["outer"] + 1
        cpu = {"value": mv / max(applies_per_solve, 1), "unit": "solves/s", "cores": nth, "kind": "oracle",
               "cpu_model": model,
               "sample": f"{nrows} direct-sum rows of N={N_or} on {nth} threads ({rows_s:.2f} rows/s = "
                         f"{mv:.3e} matvecs/s), scaled by {applies_per_solve} applies per solve",
               "fp64_ref_oracle_row_residual": None if resid is None else float(resid),
               "fp64_ref_residual_rows": nrows}
        if not args.no_disc_oracle:
            cpu["disc_oracle"] = cpu_disc_oracle()
        log(f"cpu baseline {cpu}")

    out = {
        "metric": "LS solves/s at 1e-6 err vs FP64 reference (FP32 GMRES + FP64 refinement)",
        "value": args.steps / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 apply + c64 inner Arnoldi (f64 block reductions) + c128 residual",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: star R=1+0.3cos5t, kappa=32pi, n^2=1+0.8exp(-4|x|^2), "
                               f"plane wave at 30deg, N={N}", "N": N, "nrhs": 1,
                   "solver": f"GMRES({g['restart']}), inner {args.ortho} tol 1e-4, outer FP64 residual tol 1e-7"},
        "err_vs_fp64_ref": err,
        "solve_p50_ms": float(np.percentile(np.array(lat) * 1e3, 50)),
        "solve_p99_ms": float(np.percentile(np.array(lat) * 1e3, 99)),
        "iterations": info["iterations"],
        "outer": info["outer"],
        "fp32_apply_f64_arnoldi_solves_per_s": 1.0 / min(ta),
        "fp32_apply_f64_arnoldi_err": err_a,
        "fp32_apply_f64_arnoldi_iterations": info_a["iterations"],
        "solve_stage_us": info_p["stage_us"],
        "fp64_plain_solves_per_s": 1.0 / t64,
        "fp64_plain_err": err64,
        "fp64_plain_iterations": info64["iterations"],
        "matvecs_per_s_fp64": rates["fp64"],
        "matvecs_per_s_fp32": rates["fp32"],
        "stage_ms": prof,
        "setup_s": setup_s,
        "resident_gb": op.resident_bytes() / 1e9,
        "roofline": roof,
        "roofline_fft": roof_fft,
        "roofline_fft3d": fft3d,
        "roofline_fft256": fft256,
        "autotune": tune,
        "multi_rhs": multi,
        "fft_refined": refined,
        "fft_refined_interior": refined_int,
        "fft_refined_shortcut": refined_sc,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
