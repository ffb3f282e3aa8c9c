"""Learned Davidson guess: per-pair features, the 3-layer network, its loss and gradients.

TEST INFRASTRUCTURE ONLY (like all of oracle/): plain FP64 NumPy, used by the
tests, by smoke() and by bench.py's CPU baseline, never by the library.

The paper's outlook proposes machine-learned starting points for the excited
state solver; the construction here (features, target, network, loss) is the
reading stated in the design notes, written out directly:

Features of the single excitation i -> a (i occupied, a virtual; C[mu, p],
eps ascending, atoms A with AO sets, g_A = (s_A s_A | s_A s_A)):
  q_A   = sum_{mu in A} C[mu, i] C[mu, a]          transition charge on atom A
  p_A^x = sum_{mu in A} C[mu, x]^2                 orbital population on atom A
  r_x   = sum_A p_A^x R_A                          orbital centroid (bohr)
  f0  = eps_a - eps_i
  f1  = eps_HOMO - eps_i
  f2  = eps_a - eps_LUMO
  f3  = sum_A q_A^2
  f4..f7 = the four largest |q_A|, descending (zero when fewer atoms)
  f8  = sum_A g_A q_A^2                            one-centre exchange estimate
  f9  = sum_A g_A p_A^i p_A^a                      one-centre Coulomb estimate
  f10 = |r_i - r_a|
  f11 = f0 + 2 f8 - f9                             corrected gap
All are unchanged when an orbital changes sign.

Network (features standardised with fixed mean mu and scale sd):
  h1 = silu(x W1 + b1)   (F -> 128),  h2 = silu(h1 W2 + b2)  (128 -> 128),
  z  = h2 w3 + b3        (128 -> 1),   silu(t) = t / (1 + exp(-t)).
Target of a molecule with K converged roots X^n: w_ia = (1/K) sum_n (X^n_ia)^2
(a distribution over the pairs, invariant to root signs and to rotations among
degenerate roots).  Loss of one molecule: softmax cross-entropy
  L = -sum_ia w_ia log softmax(z)_ia,
and a batch loss is the mean over its molecules.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

NFEAT = 12
WIDTH = 128


def features(sys, C: np.ndarray, eps: np.ndarray, nocc: int) -> np.ndarray:
    """[nocc * nvirt, NFEAT] in the pair order i * nvirt + a (hartree, bohr)."""
    n = C.shape[0]
    o, v = nocc, n - nocc
    natoms = sys.natoms
    g = np.array([sys.el(A).gss for A in range(natoms)])
    # atom x AO membership
    Mat = np.zeros((natoms, n))
    Mat[sys.ao_atom, np.arange(n)] = 1.0
    pop = Mat @ (C ** 2)                      # [natoms, n] populations p_A^x
    cent = pop.T @ sys.R                      # [n, 3] centroids
    Co, Cv = C[:, :o], C[:, o:]
    feats = np.zeros((o, v, NFEAT))
    # q[A, i, a] = sum_{mu in A} C[mu, i] C[mu, a]
    q = np.einsum("Am,mi,ma->Aia", Mat, Co, Cv)
    de = eps[o:][None, :] - eps[:o][:, None]
    feats[:, :, 0] = de
    feats[:, :, 1] = (eps[o - 1] - eps[:o])[:, None]
    feats[:, :, 2] = (eps[o:] - eps[o])[None, :]
    feats[:, :, 3] = np.sum(q ** 2, axis=0)
    top = -np.sort(-np.abs(q), axis=0)        # descending along atoms
    for t in range(4):
        if t < natoms:
            feats[:, :, 4 + t] = top[t]
    feats[:, :, 8] = np.einsum("A,Aia->ia", g, q ** 2)
    feats[:, :, 9] = np.einsum("A,Ai,Aa->ia", g, pop[:, :o], pop[:, o:])
    feats[:, :, 10] = np.linalg.norm(cent[:o][:, None, :] - cent[o:][None, :, :], axis=2)
    feats[:, :, 11] = feats[:, :, 0] + 2 * feats[:, :, 8] - feats[:, :, 9]
    return feats.reshape(o * v, NFEAT)


def target(X: np.ndarray) -> np.ndarray:
    """w_ia = (1/K) sum_n X[n, i, a]^2 for K roots X [K, o, v] (each normalised)."""
    K = X.shape[0]
    return np.sum(X.reshape(K, -1) ** 2, axis=0) / K


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even) and return as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


@dataclass
class Params:
    W1: np.ndarray   # [F, 128]
    b1: np.ndarray   # [128]
    W2: np.ndarray   # [128, 128]
    b2: np.ndarray   # [128]
    w3: np.ndarray   # [128]
    b3: float
    mu: np.ndarray   # [F] feature means
    sd: np.ndarray   # [F] feature scales

    def flat(self) -> np.ndarray:
        return np.concatenate([self.W1.ravel(), self.b1, self.W2.ravel(), self.b2, self.w3, [self.b3]])


def silu(t):
    return t / (1.0 + np.exp(-t))


def dsilu(t):
    s = 1.0 / (1.0 + np.exp(-t))
    return s * (1.0 + t * (1.0 - s))


def forward(p: Params, F: np.ndarray):
    """Scores z [npairs] and the intermediates the backward pass needs."""
    x = (F - p.mu) / p.sd
    a1 = x @ p.W1 + p.b1
    h1 = silu(a1)
    a2 = h1 @ p.W2 + p.b2
    h2 = silu(a2)
    z = h2 @ p.w3 + p.b3
    return z, (x, a1, h1, a2, h2)


def loss(z: np.ndarray, w: np.ndarray, seg: np.ndarray):
    """Mean over molecules of the softmax cross-entropy; seg = pair offsets per molecule."""
    nmol = len(seg) - 1
    L = 0.0
    dz = np.zeros_like(z)
    for m in range(nmol):
        s = slice(seg[m], seg[m + 1])
        zm = z[s]
        mx = zm.max()
        lse = mx + np.log(np.sum(np.exp(zm - mx)))
        L += -np.sum(w[s] * (zm - lse))
        dz[s] = (np.exp(zm - lse) * np.sum(w[s]) - w[s]) / nmol
    return L / nmol, dz


def backward(p: Params, cache, dz: np.ndarray) -> dict:
    """Gradients of the loss w.r.t. every parameter (chain rule through the layers)."""
    x, a1, h1, a2, h2 = cache
    g = {}
    g["w3"] = h2.T @ dz
    g["b3"] = float(np.sum(dz))
    d2 = np.outer(dz, p.w3) * dsilu(a2)
    g["W2"] = h1.T @ d2
    g["b2"] = d2.sum(axis=0)
    d1 = (d2 @ p.W2.T) * dsilu(a1)
    g["W1"] = x.T @ d1
    g["b1"] = d1.sum(axis=0)
    return g


def loss_and_grad(p: Params, F: np.ndarray, w: np.ndarray, seg: np.ndarray):
    z, cache = forward(p, F)
    L, dz = loss(z, w, seg)
    return L, backward(p, cache, dz), z


def init_params(seed: int, mu: np.ndarray, sd: np.ndarray) -> Params:
    """Seeded initial weights (uniform, fan-in scaled), FP64."""
    rng = np.random.default_rng(seed)
    lim1, lim2 = np.sqrt(6.0 / NFEAT), np.sqrt(6.0 / WIDTH)
    return Params(rng.uniform(-lim1, lim1, (NFEAT, WIDTH)), np.zeros(WIDTH),
                  rng.uniform(-lim2, lim2, (WIDTH, WIDTH)), np.zeros(WIDTH),
                  rng.uniform(-lim2, lim2, WIDTH), 0.0, mu.copy(), sd.copy())


def pspace_guess(z: np.ndarray, M: int) -> np.ndarray:
    """Flat pair indices of the M largest scores (ties: lower index first), ascending index order."""
    order = np.lexsort((np.arange(z.size), -z))
    return np.sort(order[:M])
