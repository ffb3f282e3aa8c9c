"""CPU Davidson for CIS and TDHF built on the matrix-free product of Eqs. 8-9.

GPU-implementation subsection of the paper: A and B are never formed; the
lowest roots come from a Davidson iteration that only needs products of the
matrices with subspace vectors.  The batched outline in that subsection, for
one molecule: start from orthonormal vectors; form the products; project and
diagonalise; build Ritz vectors and residuals; precondition the unconverged
residuals with the diagonal; orthonormalise them against the basis, append,
repeat.

Readings where the paper is silent:
  * guess: unit vectors e_ia at the min(nov, 2K) smallest gaps
    eps_a - eps_i (ties by flat index i*v + a);
  * TDHF: one orthonormal basis V for both X+Y and X-Y (symmetric and
    antisymmetric subspace method): M+ = V^T (A+B) V, M- = V^T (A-B) V,
    M- = L L^T, (L^T M+ L) w = omega^2 w, t = L w, u = M+ t / omega, scaled so
    that t^T u = 1 (that is X^T X - Y^T Y = 1);
  * residuals r_T = (A+B) T - omega U, r_U = (A-B) U - omega T; a root is
    converged when sqrt(|r_T|^2 + |r_U|^2) <= tol (CIS: |A X - omega X|);
  * preconditioner: CIS r / (omega - d); TDHF adds (r_T + r_U)/(omega - d) and
    (r_T - r_U)/(-omega - d), d = eps_a - eps_i, denominators kept >= 1e-8 in
    magnitude;
  * orthonormalisation: classical Gram-Schmidt applied twice; a new vector
    whose norm drops below 1e-10 is discarded;
  * optional subspace cap `max_sub`: when the basis would exceed it, it is
    replaced by the orthonormalised current Ritz vectors (X+Y and X-Y for TDHF,
    the 2K lowest for CIS) -- the restart from the current best estimates the
    paper describes when memory runs out (Results section).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import excited as X
from . import integrals as I


@dataclass
class DavidsonResult:
    omega: np.ndarray
    X: np.ndarray
    Y: np.ndarray
    iterations: int
    n_sigma: int
    residuals: np.ndarray
    history: list = field(default_factory=list)   # per iteration: (n_sigma, omegas)


def _guard(d):
    return np.where(np.abs(d) < 1e-8, np.where(d < 0, -1e-8, 1e-8), d)


def _orthonormalise(V: np.ndarray, W: np.ndarray) -> np.ndarray:
    """Rows of W orthonormalised against the rows of V and each other.

    Classical Gram-Schmidt applied twice: every projection coefficient against
    V is taken from the vector before that pass (done for the whole block at
    once), then the block is orthonormalised row by row the same way."""
    W = np.array(W, dtype=np.float64, copy=True)
    if V.shape[0]:
        for _ in range(2):
            W -= (W @ V.T) @ V
    out = []
    for w in W:
        for _ in range(2):
            for u in out:
                w = w - u * (u @ w)
        nrm = np.linalg.norm(w)
        if nrm > 1e-10:
            out.append(w / nrm)
    return np.array(out).reshape(len(out), V.shape[1])


class _Rows:
    """Growable row storage (amortised doubling) without per-iteration copies of the whole basis."""

    def __init__(self, ncol: int):
        self.a = np.empty((64, ncol))
        self.n = 0

    def append(self, rows: np.ndarray):
        need = self.n + rows.shape[0]
        if need > self.a.shape[0]:
            b = np.empty((max(need, 2 * self.a.shape[0]), self.a.shape[1]))
            b[:self.n] = self.a[:self.n]
            self.a = b
        self.a[self.n:need] = rows
        self.n = need

    @property
    def v(self) -> np.ndarray:
        return self.a[:self.n]


def solve(ints: I.Integrals, eps: np.ndarray, C: np.ndarray, nocc: int, nroots: int,
          theory: str = "tdhf", tol: float = 1e-7, max_iter: int = 200,
          guess: np.ndarray | None = None, max_sub: int | None = None) -> DavidsonResult:
    o = nocc
    v = C.shape[1] - nocc
    nov = o * v
    d = (eps[None, nocc:] - eps[:o, None]).reshape(-1)
    if guess is None:
        ng = min(nov, 2 * nroots)
        idx = np.argsort(d, kind="stable")[:ng]
        V = np.zeros((ng, nov))
        V[np.arange(ng), idx] = 1.0
    else:
        V = _orthonormalise(np.zeros((0, nov)), guess.reshape(guess.shape[0], -1))
    tdhf = theory == "tdhf"
    Vs, SPs, SMs = _Rows(nov), _Rows(nov), _Rows(nov)   # basis, (A+B) V (CIS: A V), (A-B) V
    Mp = np.zeros((0, 0))
    Mm = np.zeros((0, 0))
    new = V
    n_sigma = 0
    hist = []

    def grow(M, Vall, S_new, s0):
        # projected matrix V^T S V: new columns from the new products, rows by symmetry
        n1 = Vall.shape[0]
        out = np.zeros((n1, n1))
        out[:s0, :s0] = M
        col = Vall @ S_new.T                    # [n1, k]
        out[:, s0:] = col
        out[s0:, :s0] = col[:s0].T
        out[s0:, s0:] = 0.5 * (col[s0:] + col[s0:].T)
        return out

    for it in range(1, max_iter + 1):
        AV, BV = X.sigma(ints, eps, C, nocc, new.reshape(-1, o, v))
        AV, BV = AV.reshape(-1, nov), BV.reshape(-1, nov)
        n_sigma += new.shape[0]
        s0 = Vs.n
        Vs.append(new)
        V = Vs.v
        if tdhf:
            SPs.append(AV + BV)
            SMs.append(AV - BV)
            SP, SM = SPs.v, SMs.v
            Mp = grow(Mp, V, SP[s0:], s0)
            Mm = grow(Mm, V, SM[s0:], s0)
            L = np.linalg.cholesky(Mm)
            w2, W = np.linalg.eigh(L.T @ Mp @ L)
            om = np.sqrt(w2[:nroots])
            t = (L @ W[:, :nroots]) / np.sqrt(om)[None, :]
            u = (Mp @ t) / om[None, :]
            T, U = t.T @ V, u.T @ V
            rT = t.T @ SP - om[:, None] * U
            rU = u.T @ SM - om[:, None] * T
            res = np.sqrt(np.sum(rT * rT, axis=1) + np.sum(rU * rU, axis=1))
        else:
            SPs.append(AV)
            SP = SPs.v
            Mp = grow(Mp, V, SP[s0:], s0)
            w, W = np.linalg.eigh(Mp)
            om = w[:nroots]
            x = W[:, :nroots]
            T = x.T @ V
            r = x.T @ SP - om[:, None] * T
            res = np.linalg.norm(r, axis=1)
        hist.append((n_sigma, om.copy()))
        if np.all(res <= tol):
            break
        cand = []
        for k in np.nonzero(res > tol)[0]:
            if tdhf:
                cand.append((rT[k] + rU[k]) / _guard(om[k] - d))
                cand.append((rT[k] - rU[k]) / _guard(-om[k] - d))
            else:
                cand.append(r[k] / _guard(om[k] - d))
        if max_sub is not None and Vs.n + len(cand) > max_sub:
            # restart from the current best estimates (paper, Results: collapse of the subspace)
            base = np.vstack([T, U]) if tdhf else W[:, :min(2 * nroots, W.shape[1])].T @ V
            Vn = _orthonormalise(np.zeros((0, nov)), base)
            G = Vn @ V.T                      # new basis expressed in the old orthonormal one
            Vs, SPs = _Rows(nov), _Rows(nov)
            Vs.append(Vn)
            SPs.append(G @ SP)
            Mp = G @ Mp @ G.T
            if tdhf:
                SMs = _Rows(nov)
                SMs.append(G @ SM)
                Mm = G @ Mm @ G.T
            V = Vs.v
        new = _orthonormalise(V, np.array(cand))
        if new.shape[0] == 0:
            break
    else:
        raise RuntimeError("Davidson did not converge")
    if tdhf:
        Xs = ((T + U) / 2).reshape(nroots, o, v)
        Ys = ((T - U) / 2).reshape(nroots, o, v)
    else:
        Xs = T.reshape(nroots, o, v)
        Ys = np.zeros_like(Xs)
    flat = Xs.reshape(nroots, -1)
    for k in range(nroots):
        j = int(np.argmax(np.abs(flat[k])))
        if flat[k, j] < 0:
            Xs[k] *= -1.0
            Ys[k] *= -1.0
    return DavidsonResult(om, Xs, Ys, it, n_sigma, res, hist)
