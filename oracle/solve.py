"""Linear solvers of the oracle (test infrastructure only).

* gmres: restarted GMRES (Saad & Schultz) in complex arithmetic, as used by the
  paper for the Nyström system (Sec. 2): Arnoldi with modified Gram–Schmidt,
  Givens rotations on the Hessenberg matrix, x0 = 0 unless given.
* dense_solve: LU with partial pivoting (library routine) for tiny systems.
"""
import numpy as np


def gmres(matvec, b, tol=1e-10, restart=100, max_iter=2000, x0=None):
    """Solve A x = b.  Returns (x, info) with info = dict(iterations,
    rel_residual, converged, history)."""
    n = b.shape[0]
    x = np.zeros(n, complex) if x0 is None else np.array(x0, complex)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return x, {"iterations": 0, "rel_residual": 0.0, "converged": True, "history": []}
    hist = []
    it = 0
    while True:
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        hist.append(beta / bnorm)
        if beta / bnorm <= tol or it >= max_iter:
            return x, {"iterations": it, "rel_residual": beta / bnorm,
                       "converged": beta / bnorm <= tol, "history": hist}
        m = restart
        V = np.zeros((n, m + 1), complex)
        Hm = np.zeros((m + 1, m), complex)
        cs = np.zeros(m, complex)
        sn = np.zeros(m, complex)
        g = np.zeros(m + 1, complex)
        g[0] = beta
        V[:, 0] = r / beta
        k_done = 0
        for k in range(m):
            w = matvec(V[:, k])
            for j in range(k + 1):
                Hm[j, k] = np.vdot(V[:, j], w)
                w = w - Hm[j, k] * V[:, j]
            Hm[k + 1, k] = np.linalg.norm(w)
            if Hm[k + 1, k] != 0.0:
                V[:, k + 1] = w / Hm[k + 1, k]
            for j in range(k):
                t = cs[j] * Hm[j, k] + sn[j] * Hm[j + 1, k]
                Hm[j + 1, k] = -np.conj(sn[j]) * Hm[j, k] + np.conj(cs[j]) * Hm[j + 1, k]
                Hm[j, k] = t
            a, bb = Hm[k, k], Hm[k + 1, k]
            den = np.sqrt(abs(a) ** 2 + abs(bb) ** 2)
            cs[k] = np.conj(a) / den if den != 0 else 1.0
            sn[k] = np.conj(bb) / den if den != 0 else 0.0
            Hm[k, k] = den
            Hm[k + 1, k] = 0.0
            g[k + 1] = -np.conj(sn[k]) * g[k]
            g[k] = cs[k] * g[k]
            it += 1
            k_done = k + 1
            hist.append(abs(g[k + 1]) / bnorm)
            if abs(g[k + 1]) / bnorm <= tol or it >= max_iter:
                break
        y = np.linalg.solve(np.triu(Hm[:k_done, :k_done]), g[:k_done])
        x = x + V[:, :k_done] @ y


def dense_solve(A, b):
    return np.linalg.solve(A, b)
