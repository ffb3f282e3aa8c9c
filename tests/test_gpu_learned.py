"""Learned starting space on the GPU against the oracle (oracle/mlp.py).

Bars:
  * features: FP32 storage of values formed in FP64, so 2e-6 relative (plus
    1e-9 absolute for the orbital differences of two independent SCFs);
  * scores and gradients: the network uses bfloat16-valued weights (the oracle
    is given the same rounded weights); activations enter the bfloat16 layer as
    hi + lo pairs (about 16 significant bits) and everything else is FP32, so
    1e-4 relative, as the learned-guess bar states;
  * guesses change iteration counts, never the roots: 1e-6 eV against the gap
    guess in FP64.
"""
import os
import tempfile

import numpy as np
import pytest

from oracle import excited, integrals, mlp, model, scf
from paper_2505_24807_amd import seqx
from synthetic import molecules, params

pytestmark = pytest.mark.gpu
PR = params.load()
MOLS = {
    "C2H4": molecules.ethylene(),
    "C10H12n": molecules.add_noise(molecules.polyene(10), 0.02, np.random.default_rng(10)),
    "H2O12": molecules.water_cluster(12, 5),
}


@pytest.fixture(scope="module")
def ctx():
    c = seqx.Context(0)
    c.set_params(*seqx.params_table(PR))
    yield c
    c.close()


def _oracle_ground(mol):
    sy = model.make_system(mol.Z, mol.xyz, PR)
    ints = integrals.build(sy)
    res = scf.run(sy, ints)
    return sy, ints, res


def _rounded(p: mlp.Params) -> mlp.Params:
    return mlp.Params(mlp.bf16_round(p.W1), p.b1.astype(np.float32).astype(np.float64), mlp.bf16_round(p.W2),
                      p.b2.astype(np.float32).astype(np.float64), mlp.bf16_round(p.w3),
                      float(np.float32(p.b3)), p.mu.astype(np.float32).astype(np.float64),
                      p.sd.astype(np.float32).astype(np.float64))


def _flat(p: mlp.Params) -> np.ndarray:
    return np.concatenate([p.flat(), p.mu, p.sd]).astype(np.float32)


def _params(seed, mu, sd):
    p = mlp.init_params(seed, mu, sd)
    rng = np.random.default_rng(seed + 1)
    p.b1 = rng.normal(size=mlp.WIDTH) * 0.1
    p.b2 = rng.normal(size=mlp.WIDTH) * 0.1
    p.b3 = 0.25
    return p


@pytest.mark.parametrize("name", list(MOLS))
def test_features_match_oracle(ctx, name):
    sy, _, res = _oracle_ground(MOLS[name])
    Fo = mlp.features(sy, res.C, res.eps, res.nocc)
    job = ctx.prepare([MOLS[name].natoms], MOLS[name].Z, MOLS[name].xyz)
    Fl = job.features().astype(np.float64)
    job.free()
    assert Fl.shape == Fo.shape
    err = np.abs(Fl - Fo) / (np.abs(Fo) + 1e-3)
    print(f"[gpu] {name}: max rel feature error {err.max():.2e}", flush=True)
    assert (np.abs(Fl - Fo) <= 2e-6 * np.abs(Fo) + 1e-9 + 1e-6 * np.abs(Fo).max(axis=0)).all()


def test_scores_and_gradients_match_oracle(ctx):
    mol = MOLS["H2O12"]
    job = ctx.prepare([mol.natoms], mol.Z, mol.xyz)
    F = job.features().astype(np.float64)
    p = _params(3, F.mean(axis=0), F.std(axis=0))
    ctx.mlp_set_params(_flat(p))
    z = job.mlp_scores().astype(np.float64)
    job.free()
    pr = _rounded(p)
    zo, _ = mlp.forward(pr, F.astype(np.float32).astype(np.float64))
    assert np.abs(z - zo).max() <= 1e-4 * (1.0 + np.abs(zo).max())
    # gradient on two molecules' worth of pairs with random targets
    rng = np.random.default_rng(4)
    n1 = F.shape[0] // 3
    seg = np.array([0, n1, F.shape[0]])
    w = rng.random(F.shape[0])
    w[:n1] /= w[:n1].sum()
    w[n1:] /= w[n1:].sum()
    w32 = w.astype(np.float32)
    L, g = ctx.mlp_loss_grad(F.astype(np.float32), w32, seg)
    Lo, go, _ = mlp.loss_and_grad(pr, F.astype(np.float32).astype(np.float64), w32.astype(np.float64), seg)
    assert abs(L - Lo) <= 1e-5 * abs(Lo)
    blocks = {"W1": (0, 1536), "b1": (1536, 1664), "W2": (1664, 18048), "b2": (18048, 18176), "w3": (18176, 18304)}
    for name, (a, b) in blocks.items():
        ref = np.asarray(go[name]).ravel()
        rel = np.linalg.norm(g[a:b] - ref) / np.linalg.norm(ref)
        el = np.abs(g[a:b] - ref).max() / np.abs(ref).max()
        print(f"[gpu] grad {name}: rel err {rel:.2e}, largest element error / largest element {el:.2e}",
              flush=True)
        assert rel <= 1e-4, name
        # element by element: within 1e-4 of the element plus 1e-4 of the block's largest
        assert np.all(np.abs(g[a:b] - ref) <= 1e-4 * np.abs(ref) + 1e-4 * np.abs(ref).max()), name
    assert abs(g[18304] - go["b3"]) <= 1e-5


def test_params_save_load_roundtrip(ctx):
    p = _params(9, np.zeros(12), np.ones(12))
    flat = _flat(p)
    ctx.mlp_set_params(flat)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "net.bin")
        ctx.mlp_save(path)
        ctx.mlp_set_params(flat * 0.5 + np.concatenate([np.zeros(flat.size - 12), np.ones(12, np.float32) * 0.5]))
        ctx.mlp_load(path)
    assert np.array_equal(ctx.mlp_get_params(), flat)


def test_training_lowers_loss_and_guesses_keep_roots(ctx):
    rng = np.random.default_rng(77)
    train = [molecules.add_noise(molecules.polyene(int(n)), 0.02, rng) for n in rng.choice([4, 6, 8, 10], 12)]
    train += [molecules.water_cluster(int(m), int(rng.integers(1 << 30))) for m in rng.choice([4, 5, 6], 12)]
    natoms, Z, xyz = molecules.concat(train)
    job = ctx.prepare(list(natoms), Z, xyz)
    job.solve(theory=seqx.CIS, nroots=5, tol=1e-6, max_iter=200, precision=seqx.FP64, batched=True)
    log = job.mlp_train(epochs=15, batch=8, lr=3e-3, seed=5, init=True)
    job.free()
    print(f"[gpu] training loss {log['loss'][0]:.4f} -> {log['loss'][-1]:.4f} in {log['seconds']:.2f} s", flush=True)
    assert log["loss"][-1] < 0.9 * log["loss"][0]
    held = molecules.add_noise(molecules.polyene(14), 0.02, np.random.default_rng(123))
    roots = {}
    for guess in (seqx.GUESS_GAP, seqx.GUESS_GAP_PSPACE, seqx.GUESS_LEARNED):
        j = ctx.prepare([held.natoms], held.Z, held.xyz)
        j.solve(theory=seqx.CIS, nroots=5, tol=1e-7, max_iter=200, guess=guess)
        roots[guess] = (j.results().omega_eV, j.stats().dav_iterations)
        j.free()
    print(f"[gpu] iterations gap/gap-P/learned-P: {[roots[g][1] for g in roots]}", flush=True)
    for g in (seqx.GUESS_GAP_PSPACE, seqx.GUESS_LEARNED):
        assert np.abs(roots[g][0] - roots[seqx.GUESS_GAP][0]).max() < 1e-6


def test_learned_guess_needs_a_network():
    c = seqx.Context(0)
    c.set_params(*seqx.params_table(PR))
    job = c.prepare([MOLS["C2H4"].natoms], MOLS["C2H4"].Z, MOLS["C2H4"].xyz)
    with pytest.raises(seqx.SeqxError) as e:
        job.solve(theory=seqx.CIS, nroots=2, guess=seqx.GUESS_LEARNED)
    assert e.value.name == "E_STATE"
    job.free()
    c.close()


def test_packaged_network_saves_iterations():
    """The packaged network (guess_net.bin) on the first five held-out
    evaluation molecules (seeds 100000-100004, 207-579 atoms, CIS, 10 roots):
    fewer Davidson iterations in total than the gap guess and than the
    gap-ranked P-space of the same size, with the same roots."""
    from paper_2505_24807_amd.train_guess import evaluate

    c = seqx.Context(0)
    c.set_params(*seqx.params_table(PR))
    c.mlp_load(os.path.join(os.path.dirname(seqx.__file__), "guess_net.bin"))
    rows = evaluate(c, list(range(100000, 100005)), log=lambda *a, **k: None)
    c.close()
    keys = ("gap", "gap_pspace", "learned_pspace")
    tot = {key: sum(r[key]["iterations"] for r in rows) for key in keys}
    print(f"[gpu] summed iterations {tot}", flush=True)
    assert tot["learned_pspace"] < tot["gap"] and tot["learned_pspace"] < tot["gap_pspace"]
    assert max(r[key]["max_abs_dev_eV"] for r in rows for key in keys) < 1e-6
