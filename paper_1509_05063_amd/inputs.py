"""Seeded synthetic inputs shared by the tests, the smoke check and the
benchmark.

This module holds problem descriptions (geometry, wavenumber, refractive
index, discretisation parameters) and random vectors only; it contains none
of the method's arithmetic.  Both the GPU library and the CPU oracle receive
the same numbers from here.

Parameter names follow the paper: h interior spacing, (N1, N2) boundary-patch
intervals, Q Newton–Cotes points, P interpolation nodes per axis, chi_c0 and
the cut-off radii r_int (physical), r1 / r2 (boundary-patch grid units), the
polar and varrho rule sizes, cell size H = cell_h * h, q equivalent sources
per cell face, n_fb Fourier–Bessel modes of the cell Dirichlet fit.
"""
import copy
import math

import numpy as np

TWO_PI = 2.0 * math.pi


def _base(kappa, h, a, k, s_in, N1, N2, s_a, s_b):
    return {
        "dim": 2,
        "kappa": kappa,
        "shape": {"a": a, "k": k},
        "h": h,
        "band": {"s_in": s_in, "N1": N1, "N2": N2},
        "pou": {"s_a": s_a, "s_b": s_b},
        "Q": 5,
        "P": 8,
        "chi_c0": 0.1,
        "r_int": 12 * h,
        "r1": 12.0,
        "r2": 8.0,
        "polar": {"n_in": 16, "grade": 3, "n_out": 32, "n_theta": 48},
        "band_rule": {"M": 4, "n_in": 24, "n_out": 32},
        # accelerator (library only; the oracle sums every pair directly)
        "cell_h": 8,
        "q": 12,
        "n_fb": 20,
        "coll_factor": 4,
    }


def config(name):
    """Named workloads.

    disc_k2pi   unit disc, n = 1.5, kappa = 2 pi, h = 1/32, annulus 0.8 < r < 1
                with 64 x 16 intervals (about 4k points)
    star_k32pi  star R = 1 + 0.3 cos 5 theta, n^2 = 1 + 0.8 exp(-4|x|^2),
                kappa = 32 pi, h = 1/512, band 0.9 < s < 1 with 4096 x 32
                intervals (about 950k points)
    star_k16pi  the same star at kappa = 16 pi, h = 1/256, band 2048 x 32
                (about 270k points; 256 incident directions)
    star_sincos_k2  the same star at kappa = 2 with the smooth variable index
                n = sin(pi x1) cos(pi x2) (vanishing on lines through the
                scatterer), h = 1/32, band 0.8 < s < 1 with 128 x 16 intervals
    disc_k2pi_p2    disc_k2pi with the band covered by two overlapping
                boundary patches (half-overlap 0.35 rad) with a tangential
                partition of unity, 40 x 16 intervals each (about the
                periodic band's t1 spacing)
    star_sincos_k2_p3  star_sincos_k2 with three boundary patches
                (half-overlap 0.3 rad), 56 x 16 intervals each
    """
    if name == "disc_k2pi":
        c = _base(TWO_PI, 1.0 / 32, 0.0, 0, 0.8, 64, 16, 0.8, 0.95)
        c["n2"] = {"kind": "const", "value": 2.25}
        c["incidence"] = [0.0]
        c["gmres"] = {"tol": 1e-10, "restart": 100}
    elif name == "star_k32pi":
        c = _base(32 * math.pi, 1.0 / 512, 0.3, 5, 0.9, 4096, 32, 0.9, 0.975)
        c["n2"] = {"kind": "gauss", "base": 1.0, "amp": 0.8, "decay": 4.0}
        c["incidence"] = [math.pi / 6]
        c["gmres"] = {"tol": 1e-8, "restart": 100}
    elif name == "star_k16pi":
        c = _base(16 * math.pi, 1.0 / 256, 0.3, 5, 0.9, 2048, 32, 0.9, 0.975)
        c["n2"] = {"kind": "gauss", "base": 1.0, "amp": 0.8, "decay": 4.0}
        c["incidence"] = [TWO_PI * r / 256 for r in range(256)]
        c["gmres"] = {"tol": 1e-8, "restart": 60}
    elif name == "star_sincos_k2":
        c = _base(2.0, 1.0 / 32, 0.3, 5, 0.8, 128, 16, 0.8, 0.95)
        c["n2"] = {"kind": "sincos"}
        c["incidence"] = [0.0]
        c["gmres"] = {"tol": 1e-10, "restart": 100}
    elif name == "disc_k2pi_p2":
        c = config("disc_k2pi")
        c["band"].update({"N1": 40, "patches": 2, "overlap": 0.35})
    elif name == "star_sincos_k2_p3":
        c = config("star_sincos_k2")
        c["band"].update({"N1": 56, "patches": 3, "overlap": 0.3})
    else:
        raise KeyError(name)
    c["name"] = name
    return c


def scaled(cfg, **over):
    """Copy of a configuration with some entries replaced (nested dicts are
    updated, not replaced)."""
    c = copy.deepcopy(cfg)
    for k, v in over.items():
        if isinstance(v, dict) and isinstance(c.get(k), dict):
            c[k].update(v)
        else:
            c[k] = v
    return c


def n2_function(cfg):
    """n^2 at points x (n, 2); on_boundary flags the nodes on the interface,
    where the interior limit is returned (every profile here is smooth inside
    the scatterer, so that limit is the formula itself)."""
    spec = cfg["n2"]
    if spec["kind"] == "const":
        val = float(spec["value"])
        return lambda x, on_b: np.full(x.shape[0], val)
    if spec["kind"] == "gauss":
        b, a, d = float(spec["base"]), float(spec["amp"]), float(spec["decay"])
        return lambda x, on_b: b + a * np.exp(-d * (x[:, 0] ** 2 + x[:, 1] ** 2))
    if spec["kind"] == "sincos":
        return lambda x, on_b: (np.sin(math.pi * x[:, 0]) * np.cos(math.pi * x[:, 1])) ** 2
    if spec["kind"] == "zero":
        return lambda x, on_b: np.zeros(x.shape[0])
    raise KeyError(spec["kind"])


def plane_wave(cfg, x, alpha):
    """Incident field exp(i kappa d . x), d = (cos alpha, sin alpha)."""
    k = cfg["kappa"]
    return np.exp(1j * k * (x[:, 0] * math.cos(alpha) + x[:, 1] * math.sin(alpha)))


def random_density(keys, seed=1509):
    """Complex Gaussian (g1 + i g2)/sqrt(2) assigned to nodes by their key
    (chart, i1, i2), so that both sides see the same value at the same node
    whatever order they store the nodes in."""
    keys = np.asarray(keys, dtype=np.int64)
    order = np.lexsort((keys[:, 2], keys[:, 1], keys[:, 0]))
    rng = np.random.default_rng(seed)
    g = (rng.standard_normal(keys.shape[0]) + 1j * rng.standard_normal(keys.shape[0])) / math.sqrt(2)
    out = np.empty(keys.shape[0], complex)
    out[order] = g
    return out


def match_keys(keys_a, keys_b):
    """Permutation p with keys_b[p] == keys_a (raises if the sets differ)."""
    ka = np.asarray(keys_a, np.int64)
    kb = np.asarray(keys_b, np.int64)
    if ka.shape != kb.shape:
        raise ValueError(f"node counts differ: {ka.shape[0]} vs {kb.shape[0]}")
    def code(k):
        return (k[:, 0] << 42) + ((k[:, 1] + (1 << 20)) << 21) + (k[:, 2] + (1 << 20))
    ca, cb = code(ka), code(kb)
    ob = np.argsort(cb)
    pos = np.searchsorted(cb[ob], ca)
    pos = np.clip(pos, 0, len(ob) - 1)
    p = ob[pos]
    if not np.array_equal(cb[p], ca):
        raise ValueError("node sets differ")
    return p


def serving_pool(n_ops=6, seed=20509, n_range=(1.05, 1.25), kappa_range=(4 * math.pi, 20 * math.pi)):
    """A pool of 2-D star scatterers R = 1 + a cos(k theta), a ~ U[0, 0.3],
    k ~ U{3..7}, constant n ~ U[n_range], kappa ~ U[kappa_range]; the lattice
    spacing keeps about 12 points per interior wavelength (1/h a power of two
    in 64..256) and the cells below resonance (kappa H < pi sqrt 2)."""
    rng = np.random.default_rng(seed)
    pool = []
    for i in range(n_ops):
        a = float(rng.uniform(0.0, 0.3))
        k = int(rng.integers(3, 8))
        n = float(rng.uniform(*n_range))
        kappa = float(rng.uniform(*kappa_range))
        level = 64
        while level < 256 and (kappa * n / level > 2 * math.pi / 12 or kappa * 8 / level >= math.pi * math.sqrt(2)):
            level *= 2
        kappa = min(kappa, 0.95 * math.pi * math.sqrt(2) * level / 8)
        N2 = max(8, 4 * round(level / 64))
        c = _base(kappa, 1.0 / level, a, k, 0.9, 8 * level, N2, 0.9, 0.975)
        c["n2"] = {"kind": "const", "value": n * n}
        c["name"] = f"pool{i}"
        pool.append(c)
    return pool


def serving_pool_wide(n_ops=8, seed=20509, N_range=(16e3, 1e6), kappa_range=(4 * math.pi, 32 * math.pi),
                      n_range=(1.05, 1.25)):
    """The 2-D part of the mixed serving stream: star scatterers
    R = 1 + a cos(k theta), a ~ U[0, 0.3], k ~ U{3..7}, unknowns log-uniform
    in N_range (lattice 1/h the power of two in 64..512 nearest to it on a log
    scale: about 3.6 / h^2 unknowns), kappa ~ U[kappa_range] lowered where
    needed to keep at least 10 points per interior wavelength and the cells
    below resonance (kappa H < pi sqrt 2), constant n ~ U[n_range]."""
    rng = np.random.default_rng(seed)
    pool = []
    for i in range(n_ops):
        a = float(rng.uniform(0.0, 0.3))
        k = int(rng.integers(3, 8))
        n = float(rng.uniform(*n_range))
        target = math.exp(rng.uniform(math.log(N_range[0]), math.log(N_range[1])))
        level = min((64, 128, 256, 512), key=lambda L: abs(math.log(3.6 * L * L / target)))
        kappa = float(rng.uniform(*kappa_range))
        kappa = min(kappa, 2 * math.pi * level / (10 * n), 0.95 * math.pi * math.sqrt(2) * level / 8)
        N2 = max(8, 4 * round(level / 64))
        c = _base(kappa, 1.0 / level, a, k, 0.9, 8 * level, N2, 0.9, 0.975)
        c["n2"] = {"kind": "const", "value": n * n}
        c["name"] = f"wide{i}"
        pool.append(c)
    return pool


def serving_trace(pool, n_requests, rate=50.0, seed=20509):
    """Poisson arrivals (mean `rate` per second) of solves on a scatterer drawn
    uniformly from `pool`, incidence angle uniform in [0, 2 pi).
    Returns [(arrival_s, key, cfg, alpha)]."""
    rng = np.random.default_rng(seed + 1)
    t = 0.0
    out = []
    for _ in range(n_requests):
        t += float(rng.exponential(1.0 / rate))
        c = pool[int(rng.integers(len(pool)))]
        out.append((t, c["name"], c, float(rng.uniform(0.0, 2 * math.pi))))
    return out
