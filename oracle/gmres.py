"""Restarted right-preconditioned GMRES (oracle; test infrastructure).

The paper (Section 3.3) solves with GMRES at a relative tolerance; it gives
no restart length, side or counting rule.  Readings: right preconditioning
x = P y; restart 30; tolerance on the relative residual ||g - A x|| / ||g||;
Arnoldi by modified Gram-Schmidt with Givens rotations (Saad & Schultz 1986);
at the end of a cycle x += P(V y), then the true residual is recomputed and
the solve stops if it meets the tolerance, else a new cycle starts from x.
The iteration count is the total number of Arnoldi steps.
"""
import numpy as np


class GmresResult:
    def __init__(self, x, iters, relres, history, converged):
        self.x, self.iters, self.relres = x, iters, relres
        self.history, self.converged = history, converged


def gmres(apply_A, apply_P, g, tol=1e-8, restart=30, max_iters=1000):
    g = np.asarray(g, dtype=np.complex128)
    gnorm = np.linalg.norm(g)
    x = np.zeros_like(g)
    if gnorm == 0.0:
        return GmresResult(x, 0, 0.0, [], True)
    r = g.copy()
    beta = np.linalg.norm(r)
    iters = 0
    history = []
    while True:
        if beta <= tol * gnorm:
            return GmresResult(x, iters, beta / gnorm, history, True)
        if iters >= max_iters:
            return GmresResult(x, iters, beta / gnorm, history, False)
        V = np.zeros((restart + 1, g.size), dtype=np.complex128)
        H = np.zeros((restart + 1, restart), dtype=np.complex128)
        cs = np.zeros(restart, dtype=np.complex128)
        sn = np.zeros(restart, dtype=np.complex128)
        gam = np.zeros(restart + 1, dtype=np.complex128)
        V[0] = r / beta
        gam[0] = beta
        k_used = 0
        for k in range(restart):
            w = apply_A(apply_P(V[k]))
            for i in range(k + 1):                      # modified Gram-Schmidt
                H[i, k] = np.vdot(V[i], w)
                w = w - H[i, k] * V[i]
            H[k + 1, k] = np.linalg.norm(w)
            if H[k + 1, k] != 0.0:
                V[k + 1] = w / H[k + 1, k]
            for i in range(k):                          # previous rotations
                t = cs[i] * H[i, k] + sn[i] * H[i + 1, k]
                H[i + 1, k] = -np.conj(sn[i]) * H[i, k] + np.conj(cs[i]) * H[i + 1, k]
                H[i, k] = t
            a, bb = H[k, k], H[k + 1, k]
            den = np.sqrt(abs(a) ** 2 + abs(bb) ** 2)
            if den == 0.0:
                cs[k], sn[k] = 1.0, 0.0
            elif abs(a) == 0.0:
                cs[k], sn[k] = 0.0, 1.0
            else:
                cs[k] = abs(a) / den
                sn[k] = (a / abs(a)) * np.conj(bb) / den
            H[k, k] = cs[k] * a + sn[k] * bb
            H[k + 1, k] = 0.0
            gam[k + 1] = -np.conj(sn[k]) * gam[k]
            gam[k] = cs[k] * gam[k]
            iters += 1
            k_used = k + 1
            history.append(abs(gam[k + 1]) / gnorm)
            if abs(gam[k + 1]) <= tol * gnorm or iters >= max_iters:
                break
        y = np.linalg.solve(np.triu(H[:k_used, :k_used]), gam[:k_used])
        x = x + apply_P(V[:k_used].T @ y)
        r = g - apply_A(x)
        beta = np.linalg.norm(r)
