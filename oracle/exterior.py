"""Scattered field at points off the scatterer.  TEST INFRASTRUCTURE ONLY:
used by tests/ alone, never by the library.

Outside the scatterer the Lippmann–Schwinger equation (Sec. 1,
eq:-Lippmann) gives the scattered field directly as the volume potential of
the solution, u^s(x) = u(x) - u^i(x) = -kappa^2 int G(x - y) m(y) u(y) dy,
with an integrand that is smooth in y when x lies outside.  The oracle
evaluates it with the discretisation's own plain quadrature (the weights
c_j = w_j |J_j| omega_j m_j of the Nystrom nodes, Sec. 2), summing every node
directly:  u^s(x) = -kappa^2 sum_j G(|x - y_j|) c_j u_j.
"""
import numpy as np

from .near2d import green2d


def scattered_field(setup, u, xt, chunk=64):
    """u: solution at the setup's nodes (oracle order); xt: (M, 2) targets
    outside the scatterer.  Returns u^s at xt."""
    p = setup.pts
    x, c = p["x"], p["c"]
    cu = c * u
    out = np.empty(xt.shape[0], complex)
    for s in range(0, xt.shape[0], chunk):
        t = xt[s:s + chunk]
        r = np.hypot(t[:, None, 0] - x[None, :, 0], t[:, None, 1] - x[None, :, 1])
        out[s:s + chunk] = green2d(setup.kappa, r) @ cu
    return -(setup.kappa ** 2) * out
