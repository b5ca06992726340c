"""One-dimensional rules used by the oracle: Newton–Cotes, Gauss–Legendre,
Lagrange interpolation weights and the smooth cut-off functions.

Test infrastructure only (see oracle/__init__.py).  Everything is FP64.
"""
from fractions import Fraction

import numpy as np


def newton_cotes_closed(Q):
    """Closed Q-point Newton–Cotes weights on the nodes 0, 1, ..., Q-1.

    Each weight is the exact integral over [0, Q-1] of a Lagrange basis
    polynomial (the definition of an interpolatory rule), evaluated in rational
    arithmetic so that no rounding enters the table.  Used for the transverse
    integration on boundary patches (Sec. 3, regular quadratures; Sec. 3.1.2,
    multi-split rule).
    """
    if Q < 2:
        raise ValueError("Q must be >= 2")
    out = []
    for k in range(Q):
        poly = [Fraction(1)]          # ascending coefficients
        denom = Fraction(1)
        for m in range(Q):
            if m == k:
                continue
            nxt = [Fraction(0)] * (len(poly) + 1)
            for i, c in enumerate(poly):
                nxt[i] -= m * c
                nxt[i + 1] += c
            poly = nxt
            denom *= (k - m)
        b = Fraction(Q - 1)
        integral = sum(c * b ** (i + 1) / (i + 1) for i, c in enumerate(poly))
        out.append(integral / denom)
    return np.array([float(w) for w in out])


def composite_newton_cotes(N, Q):
    """Composite closed Q-point rule on nodes 0..N (unit spacing).

    N must be a multiple of Q-1; panels start at node 0, i.e. at the
    physical boundary t_d = 0 of a boundary patch (Sec. 2, remark on the
    transverse parameter; Sec. 3 regular quadrature in t_2)."""
    if N % (Q - 1):
        raise ValueError("N must be divisible by Q-1")
    base = newton_cotes_closed(Q)
    w = np.zeros(N + 1)
    for p in range(N // (Q - 1)):
        w[p * (Q - 1):p * (Q - 1) + Q] += base
    return w


def gauss_legendre01(n):
    """n-point Gauss–Legendre nodes and weights on [0, 1] (library routine)."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def lagrange_weights(pos, base, P):
    """Lagrange interpolation weights.

    pos  : (n,) positions in grid units
    base : (n,) integer index of the first stencil node
    P    : number of stencil nodes (degree P-1)
    returns (n, P): weight of node base+k for the value at pos.
    The textbook product form prod_{m!=k} (pos - x_m)/(x_k - x_m); a position
    that coincides with a node gives exactly 1 there and 0 elsewhere.
    """
    pos = np.asarray(pos, dtype=np.float64)
    base = np.asarray(base)
    d = pos[:, None] - (base[:, None] + np.arange(P)[None, :])
    W = np.ones((pos.shape[0], P))
    for k in range(P):
        for m in range(P):
            if m != k:
                W[:, k] *= d[:, m] / (k - m)
    return W


def centered_base(pos, P):
    """First node of the P-point stencil around pos: floor(pos) - (P//2 - 1)."""
    return np.floor(pos).astype(np.int64) - (P // 2 - 1)


def smooth_step(z, beta=3.0):
    """C-infinity step: 0 for z <= 0, 1 for z >= 1 and
    erfc(beta (1 - 2z) / (2 sqrt(z (1 - z)))) / 2 in between.  All
    derivatives vanish at both ends (the argument tends to -/+ infinity like
    1/sqrt(z)), and its Fourier transform decays fast, which keeps the
    trapezoid / Newton–Cotes rules accurate on integrands that carry it.
    Used for the partition of unity and the cut-off chi (the paper gives
    neither formula; this one is a reading)."""
    from scipy import special
    z = np.asarray(z, dtype=np.float64)
    out = np.where(z >= 1.0, 1.0, 0.0)
    inside = (z > 0.0) & (z < 1.0)
    zi = z[inside]
    out[inside] = 0.5 * special.erfc(beta * (1.0 - 2.0 * zi) / (2.0 * np.sqrt(zi * (1.0 - zi))))
    return out


def chi(s, c0):
    """Cut-off chi of Sec. 3.1: identically 1 on [0, c0], 0 for s >= 1,
    smooth in between: chi(s) = 1 - smooth_step((s - c0)/(1 - c0))."""
    s = np.abs(np.asarray(s, dtype=np.float64))
    return 1.0 - smooth_step((s - c0) / (1.0 - c0))


def trig_interp_direct(x, N):
    """Weights of N periodic samples f(0), ..., f(N-1) (unit spacing) for the
    value at x of their trigonometric interpolant, from the definition: the
    discrete Fourier coefficients c_k = (1/N) sum_v f(v) e^{-2 pi i k v / N}
    summed back as sum_k c_k e^{2 pi i k x / N} over |k| < N/2, plus for even
    N the Nyquist coefficient split evenly between k = +-N/2, i.e.
    c_{N/2} cos(pi x).  This is the interpolant that zero-padding the
    spectrum produces (the FFT refinement of Sec. 3.1).  O(N) per weight:
    small N only.  Returns (len(x), N) real weights."""
    x = np.asarray(x, dtype=np.float64)
    v = np.arange(N)
    y = x[:, None] - v[None, :]
    K = (N - 1) // 2                               # |k| <= K strictly below N/2
    W = np.ones_like(y)
    for k in range(1, K + 1):
        W += 2.0 * np.cos(2.0 * np.pi * k * y / N)
    if N % 2 == 0:
        W += np.cos(np.pi * y)
    return W / N


def trig_interp_weights(x, N):
    """The same weights in closed form (the geometric sums of
    trig_interp_direct done analytically): D(y) = sin(pi y) / (N tan(pi y/N))
    for even N, sin(pi y) / (N sin(pi y / N)) for odd N, and 1 where y is a
    multiple of N.  Returns (len(x), N)."""
    x = np.asarray(x, dtype=np.float64)
    y = x[:, None] - np.arange(N)[None, :]
    yr = y - N * np.round(y / N)                   # same value, |yr| <= N/2
    on = np.abs(yr) < 1e-14
    node = np.abs(yr - np.round(yr)) < 1e-14       # at a sample: 1 or exactly 0
    ys = np.where(node, 0.5, yr)
    den = N * (np.tan(np.pi * ys / N) if N % 2 == 0 else np.sin(np.pi * ys / N))
    # numerator and denominator both from the reduced y: their ratio is the
    # same as for y (both change sign together for odd N)
    W = np.sin(np.pi * ys) / den
    return np.where(on, 1.0, np.where(node, 0.0, W))
