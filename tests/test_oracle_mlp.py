"""Pins of the oracle's learned-guess pieces (no GPU): closed forms of the
features on H2, invariances, the loss on uniform scores, bfloat16 rounding on
known values, and the backward pass against central finite differences."""
import numpy as np
import pytest

from oracle import excited, integrals, mlp, model, scf
from synthetic import molecules, params

PR = params.load()


def _ground(mol):
    sy = model.make_system(mol.Z, mol.xyz, PR)
    ints = integrals.build(sy)
    res = scf.run(sy, ints)
    return sy, ints, res


def test_features_h2_closed_forms():
    """H2: C = [[1, 1], [1, -1]] / sqrt(2) up to signs, so q_A = +-1/2 on both atoms,
    populations 1/2, both centroids at the bond midpoint."""
    sy, _, res = _ground(molecules.h2(0.74))
    F = mlp.features(sy, res.C, res.eps, 1)
    assert F.shape == (1, mlp.NFEAT)
    g = sy.el(0).gss
    f = F[0]
    assert abs(f[0] - (res.eps[1] - res.eps[0])) < 1e-14
    assert abs(f[1]) < 1e-14 and abs(f[2]) < 1e-14
    assert abs(f[3] - 0.5) < 1e-12
    assert np.allclose(f[4:6], 0.5, atol=1e-12) and np.allclose(f[6:8], 0.0)
    assert abs(f[8] - g / 2) < 1e-12 and abs(f[9] - g / 2) < 1e-12
    assert abs(f[10]) < 1e-12
    assert abs(f[11] - (f[0] + g / 2)) < 1e-12


def test_features_sign_invariant_and_charges_sum_to_zero():
    sy, _, res = _ground(molecules.add_noise(molecules.polyene(6), 0.02, np.random.default_rng(3)))
    o = res.nocc
    F = mlp.features(sy, res.C, res.eps, o)
    rng = np.random.default_rng(1)
    flip = np.where(rng.random(sy.nao) < 0.5, -1.0, 1.0)
    F2 = mlp.features(sy, res.C * flip[None, :], res.eps, o)
    assert np.abs(F - F2).max() < 1e-13
    # transition charges of orthonormal MOs sum to zero over atoms: check through f3 bound and a direct sum
    Mat = np.zeros((sy.natoms, sy.nao))
    Mat[sy.ao_atom, np.arange(sy.nao)] = 1.0
    q = np.einsum("Am,mi,ma->Aia", Mat, res.C[:, :o], res.C[:, o:])
    assert np.abs(q.sum(axis=0)).max() < 1e-12
    assert (F[:, 3] <= 1.0 + 1e-12).all() and (F[:, 4] >= F[:, 5]).all() and (F[:, 6] >= F[:, 7]).all()


def test_target_is_a_distribution():
    sy, ints, res = _ground(molecules.ethylene())
    o, v = res.nocc, sy.nao - res.nocc
    A, _ = excited.build_AB(ints, res.eps, res.C, o)
    ex = excited.cis_dense(A, 4, o, v)
    w = mlp.target(ex.X)
    assert abs(w.sum() - 1.0) < 1e-12 and (w >= 0).all()


def test_loss_of_uniform_scores():
    rng = np.random.default_rng(0)
    seg = np.array([0, 7, 20])
    w = rng.random(20)
    w[:7] /= w[:7].sum()
    w[7:] /= w[7:].sum()
    z = np.full(20, 0.3)
    L, dz = mlp.loss(z, w, seg)
    assert abs(L - 0.5 * (np.log(7) + np.log(13))) < 1e-13
    assert np.allclose(dz[:7], (1 / 7 - w[:7]) / 2) and np.allclose(dz[7:], (1 / 13 - w[7:]) / 2)


def test_bf16_rounding_known_values():
    vals = np.array([1.0, 1.0 + 2.0 ** -9, 1.0 + 3 * 2.0 ** -9, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -2.5, 0.0])
    ref = np.array([1.0, 1.0, 1.0078125, 1.0, 1.015625, -2.5, 0.0])
    assert np.array_equal(mlp.bf16_round(vals), ref)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(5)
    nf = mlp.NFEAT
    F = rng.normal(size=(40, nf))
    seg = np.array([0, 15, 40])
    w = rng.random(40)
    w[:15] /= w[:15].sum()
    w[15:] /= w[15:].sum()
    p = mlp.init_params(11, F.mean(axis=0), F.std(axis=0))
    p.b1 = rng.normal(size=mlp.WIDTH) * 0.1
    p.b2 = rng.normal(size=mlp.WIDTH) * 0.1
    L, g, _ = mlp.loss_and_grad(p, F, w, seg)
    h = 1e-6
    checks = [("W1", (3, 17)), ("W1", (11, 100)), ("b1", (5,)), ("W2", (0, 0)), ("W2", (77, 3)),
              ("W2", (127, 127)), ("b2", (64,)), ("w3", (9,)), ("w3", (120,))]
    for name, idx in checks:
        arr = getattr(p, name)
        old = arr[idx]
        arr[idx] = old + h
        Lp, _, _ = mlp.loss_and_grad(p, F, w, seg)
        arr[idx] = old - h
        Lm, _, _ = mlp.loss_and_grad(p, F, w, seg)
        arr[idx] = old
        fd = (Lp - Lm) / (2 * h)
        an = g[name][idx]
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)) + 1e-9, (name, idx, fd, an)


def test_pspace_selection_ties_and_order():
    z = np.array([0.1, 0.9, 0.5, 0.9, -1.0, 0.5])
    assert list(mlp.pspace_guess(z, 3)) == [1, 2, 3]
    assert list(mlp.pspace_guess(z, 4)) == [1, 2, 3, 5]
