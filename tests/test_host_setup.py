"""The library's host set-up (C++, independent code) against the oracle, on
the CPU: same nodes, same weights, and near-field rows that complete the
oracle's rows once the plain far sum of non-adjacent cells is added."""
import math

import numpy as np
import pytest
from scipy import special

from oracle.op2d import Setup2D
from paper_1509_05063_amd.inputs import config, match_keys, n2_function, scaled

binding = pytest.importorskip("paper_1509_05063_amd.binding")


@pytest.fixture(scope="module")
def disc():
    cfg = config("disc_k2pi")
    n2 = n2_function(cfg)
    host = binding.HostOperator(cfg, n2)
    orc = Setup2D(cfg, n2)
    return cfg, host, orc


def test_library_exports_every_symbol():
    import re
    L = binding.lib()
    names = set()
    for h in ("include/ls.h", "include/ls_host.h"):
        txt = open(h).read()
        names |= set(re.findall(r"\b(ls_[a-z0-9_]+)\s*\(", txt))
    names -= {"ls_n2_fn"}
    missing = [n for n in sorted(names) if not hasattr(L, n)]
    assert not missing, missing


def test_same_nodes(disc):
    cfg, host, orc = disc
    xy, key = host.points()
    p = match_keys(orc.pts["key"], key)       # oracle order -> library index
    assert np.abs(xy[p] - orc.pts["x"]).max() < 1e-14


def _cells(cfg, key, xy):
    ch, h = cfg["cell_h"], cfg["h"]
    H = ch * h
    c = np.where(key[:, :1] == 0, np.floor_divide(key[:, 1:], ch), np.floor(xy / H).astype(np.int64))
    return c


@pytest.fixture(scope="module", params=["disc_k2pi_p2", "star_sincos_k2_p3"])
def patches(request):
    cfg = config(request.param)
    n2 = n2_function(cfg)
    return cfg, binding.HostOperator(cfg, n2), Setup2D(cfg, n2)


def test_several_patches_same_nodes_and_weights(patches):
    """Several boundary patches: the library and the oracle build the same
    nodes and plain quadrature weights, the partition of unity sums to one
    at every node, and the weights integrate the area of the scatterer."""
    cfg, host, orc = patches
    xy, key = host.points()
    p = match_keys(orc.pts["key"], key)
    assert np.abs(xy[p] - orc.pts["x"]).max() < 1e-14
    assert set(np.unique(key[:, 0])) == set(range(cfg["band"]["patches"] + 1))
    a = cfg["shape"]["a"]
    assert abs(np.sum(orc.pts["w"] * orc.pts["omega"]) - math.pi * (1 + a * a / 2)) < 5e-4


@pytest.mark.parametrize("which", ["interior", "band", "interior_in_band", "overlap"])
def test_near_rows_complete_oracle_rows_several_patches(patches, which):
    _check_rows(patches, which)


@pytest.mark.parametrize("which", ["interior", "band", "interior_in_band"])
def test_near_rows_complete_oracle_rows(disc, which):
    _check_rows(disc, which)


def _check_rows(setup, which):
    cfg, host, orc = setup
    xy, key = host.points()
    p = match_keys(orc.pts["key"], key)       # p[i_oracle] = library index
    inv = np.empty_like(p)
    inv[p] = np.arange(p.size)                # library index -> oracle index
    cells = _cells(cfg, key, xy)
    s = np.hypot(xy[:, 0], xy[:, 1])
    if which == "interior":
        cand = np.where((key[:, 0] == 0) & (s < 0.5))[0]
    elif which == "band":
        cand = np.where(key[:, 0] >= 1)[0]
    elif which == "overlap":
        # points of a boundary patch that also lie in another patch
        inp = orc.pts["inp"][:, inv]
        cand = np.where((key[:, 0] >= 1) & (inp.sum(axis=0) >= 2))[0]
    else:
        cand = np.where((key[:, 0] == 0) & (s > 0.82))[0]
    rng = np.random.default_rng(7)
    for i in rng.choice(cand, 4, replace=False):
        cols, vals = host.near_row(i)
        lib_row = np.zeros(host.N, complex)
        np.add.at(lib_row, cols, vals)
        orow = orc.K_row(inv[i])[p]            # oracle row in library order... as function of library col
        # oracle row indexed by oracle col; reorder to library col
        orow = np.zeros(host.N, complex)
        orow[p] = orc.K_row(inv[i])
        adj = np.all(np.abs(cells - cells[i]) <= 1, axis=1)
        d = np.hypot(*(xy - xy[i]).T)
        c = np.zeros(host.N)
        c[p] = orc.pts["c"]
        far = np.where(adj | (d == 0), 0.0, 0.25j * special.hankel1(0, cfg["kappa"] * np.where(d > 0, d, 1)) * c)
        scale = np.abs(orow).max()
        err = np.abs(lib_row + far - orow).max() / scale
        assert err < 1e-11, (which, i, err)


def _zero_pad_refine(N1, r):
    """Refinement of a periodic line of N1 samples to N1 r points by numpy's
    FFT with a zero-padded spectrum (the Nyquist bin of even N1 split evenly
    between +-N1/2): returns the (r N1, N1) matrix whose row r v + s gives
    the value at v + s / r."""
    X = np.fft.fft(np.eye(N1), axis=0)
    Y = np.zeros((r * N1, N1), complex)
    h = (N1 + 1) // 2                         # frequencies 0 .. h-1 and -(h-1) .. -1
    Y[:h] = X[:h]
    Y[r * N1 - (N1 - h):] = X[h:]
    if N1 % 2 == 0:
        Y[N1 // 2] = X[N1 // 2] / 2
        Y[r * N1 - N1 // 2] = X[N1 // 2] / 2
    return np.fft.ifft(Y, axis=0) * r


@pytest.mark.parametrize("r,N1", [(2, 64), (3, 64), (3, 75)])
def test_refined_rows_complete_oracle_rows(r, N1):
    """Fourier refinement along the band's t1 lines: a library row's
    refined columns (values at t1 = v + s / r of line u of the density
    (m omega J) u) expanded over the line's unknowns with an independent
    zero-padded FFT refinement, plus its other columns and the plain far
    sum, give the oracle's row (boundary-patch targets and interior targets
    inside the patch)."""
    cfg = scaled(config("disc_k2pi"), fft_refine=r, band={"N1": N1})
    n2 = n2_function(cfg)
    host, orc = binding.HostOperator(cfg, n2), Setup2D(cfg, n2)
    xy, key = host.points()
    N = host.N
    N2 = cfg["band"]["N2"]
    p = match_keys(orc.pts["key"], key)
    inv = np.empty_like(p)
    inv[p] = np.arange(p.size)
    dens = np.zeros(N)
    dens[p] = orc.pts["dens"]
    grid = -np.ones((N1, N2 + 1), np.int64)
    b = key[:, 0] == 1
    grid[key[b, 1], key[b, 2]] = np.nonzero(b)[0]
    R = _zero_pad_refine(N1, r)
    cells = _cells(cfg, key, xy)
    s_ = np.hypot(xy[:, 0], xy[:, 1])
    rng = np.random.default_rng(11)
    picks = list(rng.choice(np.where(key[:, 0] == 1)[0], 4, replace=False))
    picks += list(rng.choice(np.where((key[:, 0] == 0) & (s_ > 0.82))[0], 3, replace=False))
    n_ext = 0
    for i in picks:
        cols, vals = host.near_row(i)
        assert cols.max() < N + (r - 1) * (N2 + 1) * N1
        lib_row = np.zeros(N, complex)
        own = cols < N
        np.add.at(lib_row, cols[own], vals[own])
        for c, w in zip(cols[~own], vals[~own]):
            t = int(c) - N
            s, rem = divmod(t, (N2 + 1) * N1)
            u, v0 = divmod(rem, N1)
            j = grid[:, u]
            lib_row[j] += w * R[r * v0 + s + 1] * dens[j]
        n_ext += int((~own).sum())
        orow = np.zeros(N, complex)
        orow[p] = orc.K_row(inv[i])
        adj = np.all(np.abs(cells - cells[i]) <= 1, axis=1)
        d = np.hypot(*(xy - xy[i]).T)
        cw = np.zeros(N)
        cw[p] = orc.pts["c"]
        far = np.where(adj | (d == 0), 0.0, 0.25j * special.hankel1(0, cfg["kappa"] * np.where(d > 0, d, 1)) * cw)
        err = np.abs(lib_row + far - orow).max() / np.abs(orow).max()
        assert err < 1e-11, (i, err)
    assert n_ext > 0


def test_refined_interior_rows_complete_oracle_rows():
    """Fourier refinement of the interior lattice as well (fft_refine = 2,
    fft_refine_interior): a library row's refined-grid columns (the shifted
    psi grids) expanded over the interior unknowns with an independent
    zero-padded FFT refinement along each axis (period M: the cell box plus
    two cells per side, rounded up to factors 2, 3, 5), its refined band
    columns likewise, plus its other columns and the plain far sum, give the
    oracle's row, for interior, boundary-patch and in-patch interior targets."""
    from oracle.near2d import interior_refine_period
    r = 2
    cfg = scaled(config("disc_k2pi"), fft_refine=r, fft_refine_interior=1)
    n2 = n2_function(cfg)
    host, orc = binding.HostOperator(cfg, n2), Setup2D(cfg, n2)
    xy, key = host.points()
    N = host.N
    N1, N2, ch = cfg["band"]["N1"], cfg["band"]["N2"], cfg["cell_h"]
    H = ch * cfg["h"]
    p = match_keys(orc.pts["key"], key)
    inv = np.empty_like(p)
    inv[p] = np.arange(p.size)
    dens = np.zeros(N)
    dens[p] = orc.pts["dens"]
    grid = -np.ones((N1, N2 + 1), np.int64)
    b = key[:, 0] == 1
    grid[key[b, 1], key[b, 2]] = np.nonzero(b)[0]
    it = np.nonzero(key[:, 0] == 0)[0]
    cells = np.where(key[:, :1] == 0, np.floor_divide(key[:, 1:], ch), np.floor(xy / H).astype(np.int64))
    lo = cells.min()
    M = interior_refine_period(orc.pts, cfg)
    gxi, gyi = key[it, 1] - (lo - 2) * ch, key[it, 2] - (lo - 2) * ch     # grid positions of the interior nodes
    Rb, Ri = _zero_pad_refine(N1, r), _zero_pad_refine(M, r)
    ext_b = (r - 1) * (N2 + 1) * N1
    rng = np.random.default_rng(17)
    s_ = np.hypot(xy[:, 0], xy[:, 1])
    picks = list(rng.choice(np.where((key[:, 0] == 0) & (s_ < 0.5))[0], 2, replace=False))
    picks += list(rng.choice(np.where(key[:, 0] == 1)[0], 2, replace=False))
    picks += list(rng.choice(np.where((key[:, 0] == 0) & (s_ > 0.82))[0], 2, replace=False))
    n_int_ext = 0
    for i in picks:
        cols, vals = host.near_row(i)
        lib_row = np.zeros(N, complex)
        own = cols < N
        np.add.at(lib_row, cols[own], vals[own])
        for c, w in zip(cols[~own], vals[~own]):
            t = int(c) - N
            if t < ext_b:
                s, rem = divmod(t, (N2 + 1) * N1)
                u, v0 = divmod(rem, N1)
                j = grid[:, u]
                lib_row[j] += w * Rb[r * v0 + s + 1] * dens[j]
            else:
                s, rem = divmod(t - ext_b, M * M)
                gy, gx = divmod(rem, M)
                s1, s2 = (s + 1) % r, (s + 1) // r
                lib_row[it] += w * Ri[r * gx + s1, gxi] * Ri[r * gy + s2, gyi] * dens[it]
                n_int_ext += 1
        orow = np.zeros(N, complex)
        orow[p] = orc.K_row(inv[i])
        adj = np.all(np.abs(cells - cells[i]) <= 1, axis=1)
        d = np.hypot(*(xy - xy[i]).T)
        cw = np.zeros(N)
        cw[p] = orc.pts["c"]
        far = np.where(adj | (d == 0), 0.0, 0.25j * special.hankel1(0, cfg["kappa"] * np.where(d > 0, d, 1)) * cw)
        err = np.abs(lib_row + far - orow).max() / np.abs(orow).max()
        assert err < 1e-11, (i, err)
    assert n_int_ext > 0


@pytest.mark.parametrize("r", [1, 2])
def test_offgrid_shortcut_rows_complete_oracle_rows(r):
    """The paper's off-grid shortcut (offgrid_shortcut, with and without the
    t1 refinement): a library row's s columns (the boundary rule at the
    patch's grid nodes, read back through ls_host_near_row's rows N ..) and
    refined s columns (expanded with an independent zero-padded FFT
    refinement of the s lines), plus its other columns and the plain far
    sum, give the oracle's row, for grid-node and in-patch interior targets."""
    cfg = scaled(config("disc_k2pi"), fft_refine=r, offgrid_shortcut=1)
    n2 = n2_function(cfg)
    host, orc = binding.HostOperator(cfg, n2), Setup2D(cfg, n2)
    xy, key = host.points()
    N = host.N
    N1, N2 = cfg["band"]["N1"], cfg["band"]["N2"]
    nl = (N2 + 1) * N1
    p = match_keys(orc.pts["key"], key)
    inv = np.empty_like(p)
    inv[p] = np.arange(p.size)
    dens = np.zeros(N)
    dens[p] = orc.pts["dens"]
    grid = -np.ones((N1, N2 + 1), np.int64)
    b = key[:, 0] == 1
    grid[key[b, 1], key[b, 2]] = np.nonzero(b)[0]
    assert np.all(grid >= 0)
    R = _zero_pad_refine(N1, r) if r > 1 else None
    ext_b = (r - 1) * nl                       # refined band densities, then s, then refined s
    node_rows = {}

    def expand(cols, vals, out, scale=1.0):
        for c, w in zip(cols, vals):
            c = int(c)
            if c < N:
                out[c] += scale * w
                continue
            t = c - N
            if t < ext_b:                       # refined band density
                s, rem = divmod(t, nl)
                u, v0 = divmod(rem, N1)
                j = grid[:, u]
                out[j] += scale * w * R[r * v0 + s + 1] * dens[j]
            elif t < ext_b + nl:                # s at grid node g
                g = t - ext_b
                if g not in node_rows:
                    node_rows[g] = host.near_row(N + g)
                expand(*node_rows[g], out, scale * w)
            else:                               # refined s line
                s, rem = divmod(t - ext_b - nl, nl)
                u, v0 = divmod(rem, N1)
                for v in range(N1):
                    g = u * N1 + v
                    if g not in node_rows:
                        node_rows[g] = host.near_row(N + g)
                    expand(*node_rows[g], out, scale * w * R[r * v0 + s + 1, v])

    cells = _cells(cfg, key, xy)
    s_ = np.hypot(xy[:, 0], xy[:, 1])
    rng = np.random.default_rng(23)
    picks = list(rng.choice(np.where((key[:, 0] == 0) & (s_ > 0.82))[0], 3, replace=False))
    picks += list(rng.choice(np.where(key[:, 0] == 1)[0], 2, replace=False))
    for i in picks:
        lib_row = np.zeros(N, complex)
        expand(*host.near_row(i), lib_row)
        orow = np.zeros(N, complex)
        orow[p] = orc.K_row(inv[i])
        adj = np.all(np.abs(cells - cells[i]) <= 1, axis=1)
        d = np.hypot(*(xy - xy[i]).T)
        cw = np.zeros(N)
        cw[p] = orc.pts["c"]
        far = np.where(adj | (d == 0), 0.0, 0.25j * special.hankel1(0, cfg["kappa"] * np.where(d > 0, d, 1)) * cw)
        err = np.abs(lib_row + far - orow).max() / np.abs(orow).max()
        assert err < 1e-11, (i, err)


def test_fft_refine_parameter_checks():
    for over, msg in [({"band": {"patches": 2, "overlap": 0.3, "N1": 40}}, "single periodic band"),
                      ({"band": {"N1": 56}}, "prime factors"),
                      ({"fft_refine": 1, "fft_refine_interior": 1}, "needs fft_refine >= 2")]:
        cfg = scaled(config("disc_k2pi"), **dict({"fft_refine": 2}, **over))
        with pytest.raises(binding.LSError) as e:
            binding.HostOperator(cfg, n2_function(cfg))
        assert msg in str(e.value)


@pytest.mark.parametrize("over,msg", [
    ({"kappa": 40.0}, "resonate"),                    # kappa H >= pi sqrt(2)
    ({"band": {"N2": 18}}, "multiple of Q-1"),
    ({"r_int": 20 / 32}, "two cells"),
    ({"P": 7}, "P must be even"),
    ({"pou": {"s_b": 1.0}}, "s_in <= s_a < s_b < 1"),
])
def test_invalid_parameters_rejected(over, msg):
    cfg = scaled(config("disc_k2pi"), **over)
    with pytest.raises(binding.LSError) as e:
        binding.HostOperator(cfg, n2_function(cfg))
    assert msg in str(e.value)
