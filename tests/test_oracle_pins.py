"""Pins of the CPU oracle against facts that do not come from the oracle:
textbook rule properties, closed forms (volume potential, Mie series),
brute force on tiny inputs.  CPU only."""
import math

import numpy as np
import pytest
from scipy import integrate, special

from oracle import quad
from oracle.geom2d import discretize, omega_band, normalized_radius
from oracle.mie import mie2d_coeffs, mie2d_total, volume_potential_disc
from oracle.near2d import (green2d, interior_stencil, multisplit_rule,
                           polar_radial_rule, varrho_rule)
from oracle.op2d import Setup2D
from oracle.solve import gmres
from paper_1509_05063_amd.inputs import config, n2_function, scaled

ZERO_N2 = {"kind": "zero"}


# ----------------------------------------------------------------- 1-D rules

def test_boole_weights_textbook():
    # Boole's rule: (2/45) [7, 32, 12, 32, 7] on unit spacing
    w = quad.newton_cotes_closed(5)
    assert np.allclose(w, np.array([7, 32, 12, 32, 7]) * 2 / 45, rtol=0, atol=1e-15)
    w3 = quad.newton_cotes_closed(3)          # Simpson
    assert np.allclose(w3, [1 / 3, 4 / 3, 1 / 3], atol=1e-15)


@pytest.mark.parametrize("Q", [3, 5, 7])
def test_composite_newton_cotes_exact_on_polynomials(Q):
    N = 4 * (Q - 1)
    w = quad.composite_newton_cotes(N, Q)
    x = np.arange(N + 1.0)
    deg = Q if Q % 2 else Q - 1
    for p in range(deg + 1):
        assert abs(np.dot(w, x ** p) - N ** (p + 1) / (p + 1)) <= 1e-12 * N ** (p + 1)


def test_trapezoid_spectral_on_periodic_bump():
    f = lambda t: np.exp(np.cos(2 * np.pi * t))
    exact = special.i0(1.0)
    for n in (16, 32):
        t = np.arange(n) / n
        assert abs(f(t).mean() - exact) < 1e-13


def test_lagrange_reproduces_polynomials():
    P = 8
    pos = np.array([0.3, 4.7, -2.25, 10.0])
    base = quad.centered_base(pos, P)
    W = quad.lagrange_weights(pos, base, P)
    nodes = base[:, None] + np.arange(P)
    for d in range(P):
        assert np.allclose((W * nodes ** d).sum(1), pos ** d, rtol=1e-12, atol=1e-9)
    # exact delta on nodes
    W2 = quad.lagrange_weights(np.array([5.0]), np.array([2]), P)
    assert np.array_equal(W2[0], np.eye(P)[3])


def test_smooth_step_and_chi():
    z = np.linspace(-0.5, 1.5, 2001)
    S = quad.smooth_step(z)
    assert np.all(np.diff(S) >= 0)
    assert np.all(S[z <= 0] == 0) and np.all(S[z >= 1] == 1)
    assert np.allclose(S + quad.smooth_step(1 - z), 1.0, atol=1e-15)
    c = quad.chi(np.array([0.0, 0.05, 0.1, 1.0, 2.0]), 0.1)
    assert np.array_equal(c, [1, 1, 1, 0, 0])


def test_gauss_legendre_exact():
    x, w = quad.gauss_legendre01(10)
    for p in range(20):
        assert abs(np.dot(w, x ** p) - 1 / (p + 1)) < 1e-14


# ------------------------------------------------------- singular 1-D rules

def test_polar_radial_rule_log_singularity():
    cfg = config("disc_k2pi")
    kappa = cfg["kappa"]
    rho, w = polar_radial_rule(cfg)
    r = cfg["r_int"]
    f = lambda t: t * green2d(kappa, t) * quad.chi(t / r, cfg["chi_c0"])
    num = np.sum(w * rho * green2d(kappa, rho))
    a = cfg["chi_c0"] * r
    ref = 0
    for part in (np.real, np.imag):
        g = lambda t: part(f(np.array([t]))[0])
        ref_p = integrate.quad(g, 0, a, limit=200, epsabs=1e-16, epsrel=1e-14)[0] + \
            integrate.quad(g, a, r, limit=200, epsabs=1e-16, epsrel=1e-14)[0]
        ref = ref + (ref_p if part is np.real else 1j * ref_p)
    assert abs(num - ref) < 1e-11 * abs(ref)


def test_varrho_rule_log_singularity():
    cfg = config("disc_k2pi")
    d, w = varrho_rule(cfg)
    r1, c0 = cfg["r1"], cfg["chi_c0"]
    f = lambda t: np.log(abs(t)) * math.cos(0.3 * t)
    num = np.sum(w * np.log(np.abs(d)) * np.cos(0.3 * d))
    g = lambda t: f(t) * quad.chi(np.array([abs(t) / r1]), c0)[0]
    ref = sum(integrate.quad(g, a, b, limit=200, epsabs=1e-15, epsrel=1e-14)[0]
              for a, b in [(-r1, -c0 * r1), (-c0 * r1, 0), (0, c0 * r1), (c0 * r1, r1)])
    assert abs(num - ref) < 1e-10 * abs(ref)


@pytest.mark.parametrize("ux", [0.0, 3.0, 6.0, 2.4, 7.77, 16.0])
def test_multisplit_rule_piecewise_polynomials(ux):
    """With chi == 1 (huge radius) the rule integrates exactly any function
    that is a polynomial of degree <= Q on each side of ux (a kink at ux is
    what the split is for)."""
    N2, Q = 16, 5
    pos, w = multisplit_rule(ux, N2, Q, 1e9, 0.1)
    assert np.all(pos >= -1e-12) and np.all(pos <= N2 + 1e-12)
    assert abs(w.sum() - N2) < 1e-12
    for p in range(1, Q + 1):
        f = np.where(pos < ux, (ux - pos) ** p, 2.0 * (pos - ux) ** p)
        exact = ux ** (p + 1) / (p + 1) + 2.0 * (N2 - ux) ** (p + 1) / (p + 1)
        assert abs(np.dot(w, f) - exact) < 1e-10 * max(1.0, exact)


def test_multisplit_grid_line_uses_grid_nodes_only_away_from_edges():
    pos, w = multisplit_rule(8.0, 16, 5, 6.0, 0.1)
    assert np.allclose(pos, np.round(pos))


# ------------------------------------------------------------- geometry

@pytest.mark.parametrize("a,N1", [(0.0, 64), (0.3, 128)])
def test_partition_of_unity_and_area(a, N1):
    """sum_k omega_k = 1 at every node, and sum_j w_j omega_j (the quadrature
    of the partition of unity) tends to the exact area pi (1 + a^2/2) of the
    star R = 1 + a cos 5 theta under refinement."""
    errs = []
    for lev in range(3):
        f = 2 ** lev
        cfg = scaled(config("disc_k2pi"), shape={"a": a, "k": 5}, h=1 / (32 * f),
                     band={"N1": N1 * f, "N2": 16 * f}, n2=ZERO_N2)
        pts = discretize(cfg, n2_function(cfg))
        s, _ = normalized_radius(pts["x"], cfg["shape"])
        ob = omega_band(s, cfg["pou"])
        om_int = np.where(s < 1, 1 - ob, 0)
        assert np.allclose(np.where(pts["chart"] == 0, pts["omega"], om_int) +
                           np.where(pts["chart"] == 1, pts["omega"], ob), 1.0)
        errs.append(abs(np.sum(pts["w"] * pts["omega"]) - math.pi * (1 + a * a / 2)))
    assert errs[0] < 5e-4 and errs[2] < 1e-8
    assert errs[1] < errs[0] / 50 and errs[2] < errs[1] / 50


# ------------------------------------------------------ closed-form pins

def _mode_exact(kappa, m, k, x, R=1.0):
    """int_{|y|<R} G(x-y) J_m(k|y|) e^{i m arg y} dy: particular solution
    J_m(k r)e^{im th}/(k^2-kappa^2) plus A J_m(kappa r) e^{im th} inside and
    B H_m(kappa r) e^{im th} outside, C^1 at r = R."""
    r = np.hypot(x[:, 0], x[:, 1])
    th = np.arctan2(x[:, 1], x[:, 0])
    d = k * k - kappa * kappa
    M = np.array([[special.jv(m, kappa * R), -special.hankel1(m, kappa * R)],
                  [kappa * special.jvp(m, kappa * R), -kappa * special.h1vp(m, kappa * R)]])
    A, _ = np.linalg.solve(M, np.array([-special.jv(m, k * R) / d, -k * special.jvp(m, k * R) / d]))
    return (special.jv(m, k * r) / d + A * special.jv(m, kappa * r)) * np.exp(1j * m * th)


def test_mode_closed_form_matches_volume_potential():
    # k -> 0, m = 0 reduces the mode potential to the constant-density one
    x = np.array([[0.2, 0.1], [0.0, 0.9]])
    kappa = 2 * math.pi
    a = _mode_exact(kappa, 0, 1e-4, x) * special.jv(0, 0) / 1.0
    b = volume_potential_disc(kappa, 1.0, x)
    assert np.allclose(a, b, rtol=1e-6)


def _ladder_errors(levels, modes, nrows=200):
    out = []
    for (h, N1, N2) in levels:
        cfg = scaled(config("disc_k2pi"), h=h, band={"N1": N1, "N2": N2}, r_int=12 * h,
                     r1=12.0 * N1 / 128, r2=8.0 * N2 / 16, n2=ZERO_N2)
        S = Setup2D(cfg, n2_function(cfg))
        x = S.pts["x"]
        idx = np.linspace(0, S.N - 1, nrows).astype(int)
        K = S.K_rows(idx)
        r = np.hypot(x[:, 0], x[:, 1])
        th = np.arctan2(x[:, 1], x[:, 0])
        errs = []
        for (m, k) in modes:
            u = special.jv(m, k * r) * np.exp(1j * m * th)
            ex = _mode_exact(cfg["kappa"], m, k, x[idx] * (1 - 1e-15))
            errs.append(np.abs(K @ u - ex).max() / np.abs(ex).max())
        out.append(errs)
    return np.array(out)


@pytest.mark.slow
def test_operator_closed_form_convergence():
    """K_h applied to densities with a closed-form volume potential
    (constant, and Bessel modes J_m(k r) e^{i m th}) converges to it under
    refinement (patch geometry, partition of unity and cut-off radii fixed in
    physical units)."""
    e = _ladder_errors([(1 / 32, 128, 16), (1 / 64, 256, 32)], [(0, 1e-3), (3, 9.4), (8, 9.4)])
    assert np.all(e[0] < 3e-3)
    assert np.all(e[1] < 6e-4)
    order = np.log2(e[0] / e[1])
    assert np.all(order > 2.0), order


def test_mie2d_series_pins():
    kappa, n, R = 2 * math.pi, 1.5, 1.0
    # Jacobi–Anger expansion of the incident wave
    m = np.arange(-60, 61)
    r, th = 0.7, 0.3
    assert abs(np.sum(1j ** (m % 4) * special.jv(m, kappa * r) * np.exp(1j * m * th)) -
               np.exp(1j * kappa * r * math.cos(th))) < 1e-13
    # continuity of u and du/dr across r = R
    th = np.linspace(0, 2 * np.pi, 7)
    eps = 1e-6
    xin = np.stack([(R - eps) * np.cos(th), (R - eps) * np.sin(th)], -1)
    xout = np.stack([(R + eps) * np.cos(th), (R + eps) * np.sin(th)], -1)
    uin, uout = mie2d_total(kappa, n, R, xin), mie2d_total(kappa, n, R, xout)
    assert np.abs(uin - uout).max() < 1e-4
    x2in = np.stack([(R - 3 * eps) * np.cos(th), (R - 3 * eps) * np.sin(th)], -1)
    x2out = np.stack([(R + 3 * eps) * np.cos(th), (R + 3 * eps) * np.sin(th)], -1)
    din = (uin - mie2d_total(kappa, n, R, x2in)) / (2 * eps)
    dout = (mie2d_total(kappa, n, R, x2out) - uout) / (2 * eps)
    assert np.abs(din - dout).max() < 1e-3 * np.abs(din).max()
    # n = 1: no scatterer
    mm, a, b = mie2d_coeffs(kappa, 1.0, R, 20)
    assert np.allclose(a, 1j ** (mm % 4), atol=1e-12) and np.allclose(b, 0, atol=1e-12)


# ------------------------------------------------------------- solves

@pytest.fixture(scope="module")
def disc_setup():
    cfg = config("disc_k2pi")
    return cfg, Setup2D(cfg, n2_function(cfg))


def test_disc_solve_against_mie_and_gmres_against_lu(disc_setup):
    cfg, S = disc_setup
    A = S.dense_A()
    x = S.pts["x"]
    f = np.exp(1j * cfg["kappa"] * x[:, 0])
    u = np.linalg.solve(A, f)
    ex = mie2d_total(cfg["kappa"], 1.5, 1.0, x * (1 - 1e-15))
    e2 = np.linalg.norm(u - ex) / np.linalg.norm(ex)
    assert e2 < 5e-3, e2
    ug, info = gmres(lambda z: A @ z, f, tol=1e-10, restart=100)
    assert info["converged"]
    assert np.linalg.norm(ug - u) / np.linalg.norm(u) < 1e-8
    # the scattered field off the disc, from the discrete solution, against
    # the Mie series' scattered part (total minus incident)
    from oracle.exterior import scattered_field
    rng = np.random.default_rng(3)
    rad = rng.uniform(1.15, 2.5, 64)
    th = rng.uniform(0, 2 * np.pi, 64)
    xt = np.stack([rad * np.cos(th), rad * np.sin(th)], axis=1)
    us = scattered_field(S, u, xt)
    ex_s = mie2d_total(cfg["kappa"], 1.5, 1.0, xt) - np.exp(1j * cfg["kappa"] * xt[:, 0])
    es = np.linalg.norm(us - ex_s) / np.linalg.norm(ex_s)
    assert es < 5e-3, es


def test_interior_stencil_constant_density(disc_setup):
    """For a constant density the interior eta part is the radial integral
    2 pi int_0^r rho G(kappa rho) chi(rho/r) d rho, on and off the lattice."""
    cfg, S = disc_setup
    kappa, r, c0 = cfg["kappa"], cfg["r_int"], cfg["chi_c0"]
    ref = 0
    for part in (np.real, np.imag):
        g = lambda t: part(t * green2d(kappa, np.array([t]))[0] * quad.chi(np.array([t / r]), c0)[0])
        v = sum(integrate.quad(g, a, b, limit=200, epsabs=1e-16, epsrel=1e-13)[0]
                for a, b in [(0, c0 * r), (c0 * r, r)])
        ref = ref + (v if part is np.real else 1j * v)
    ref *= 2 * np.pi
    for frac in [(0.0, 0.0), (0.31, 0.77)]:
        d1, d2, w = interior_stencil(frac[0], frac[1], S.polar_rule, cfg, kappa)
        assert abs(w.sum() - ref) < 1e-10 * abs(ref)


def test_rows_brute_force_tiny(disc_setup):
    """The plain part of a row is the direct pair sum: recompute one entry by
    hand from the node data."""
    cfg, S = disc_setup
    p = S.pts
    i, j = 100, S.N - 5
    row = S.plain_row(i)
    d = np.hypot(*(p["x"][i] - p["x"][j]))
    tv, tu = p["v"][i], p["u"][i]
    eta = 0.0
    if p["in_band"][i]:
        dv = min(abs(p["v"][j] - tv), cfg["band"]["N1"] - abs(p["v"][j] - tv))
        eta = quad.chi(np.array([dv / cfg["r1"]]), cfg["chi_c0"])[0] * \
            quad.chi(np.array([abs(p["u"][j] - tu) / cfg["r2"]]), cfg["chi_c0"])[0]
    exp = (1 - eta) * (0.25j * special.hankel1(0, cfg["kappa"] * d)) * p["c"][j]
    assert abs(row[j] - exp) < 1e-14 * max(abs(exp), 1e-30) + 1e-300
