"""The selector's HIP kernels against the binary64 CPU oracle of the network,
and the single-scene features against values recomputed from the oracle's state."""
import math

import numpy as np
import pytest

import synth
from oracle import mlp, model

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nnc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_18314_amd as p
    from paper_2606_18314_amd import binding
    p.load()
    return binding


def _batch(g, B):
    X = g.standard_normal((B, 6)).astype(np.float32)
    y = g.integers(0, 2, B).astype(np.int32)
    w = (g.random(B) + 0.1).astype(np.float32)
    return X, y, w


def test_forward_matches_oracle(nnc):
    g = np.random.default_rng(1)
    p = (mlp.init_params(g) + 0.1 * g.standard_normal(mlp.NPARAMS)).astype(np.float32)
    X, _, _ = _batch(g, 777)
    got = nnc.mlp_forward(torch.from_numpy(p).cuda(), torch.from_numpy(X).cuda()).cpu().numpy()
    want, _ = mlp.forward(p.astype(np.float64), X.astype(np.float64))
    assert np.allclose(got, want, rtol=1e-4, atol=1e-4)


@pytest.mark.parametrize("B", [1, 100, 1024])
def test_gradient_and_loss_match_oracle(nnc, B):
    g = np.random.default_rng(B)
    p = (mlp.init_params(g) + 0.05 * g.standard_normal(mlp.NPARAMS)).astype(np.float32)
    X, y, w = _batch(g, B)
    loss, gr = nnc.mlp_grad(torch.from_numpy(p).cuda(), torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda(),
                            torch.from_numpy(w).cuda())
    want_g = mlp.grad(p.astype(np.float64), X.astype(np.float64), y, w.astype(np.float64))
    want_l = mlp.loss(p.astype(np.float64), X.astype(np.float64), y, w.astype(np.float64))
    assert abs(float(loss.item()) - want_l) <= 1e-5 * max(1.0, abs(want_l))
    got = gr.cpu().numpy()
    scale = np.max(np.abs(want_g))
    assert np.max(np.abs(got - want_g)) <= 2e-5 * scale + 1e-7


def test_adam_matches_oracle(nnc):
    g = np.random.default_rng(7)
    p = g.standard_normal(mlp.NPARAMS).astype(np.float32)
    m = (0.01 * g.standard_normal(mlp.NPARAMS)).astype(np.float32)
    v = (0.01 * g.random(mlp.NPARAMS)).astype(np.float32)
    gr = g.standard_normal(mlp.NPARAMS).astype(np.float32)
    pd, md, vd = (torch.from_numpy(a.copy()).cuda() for a in (p, m, v))
    nnc.mlp_adam(pd, md, vd, torch.from_numpy(gr).cuda(), 3, lr=1e-2)
    wp, wm, wv = mlp.adam(p.astype(np.float64), m.astype(np.float64), v.astype(np.float64),
                          gr.astype(np.float64), 3, lr=1e-2)
    assert np.allclose(pd.cpu().numpy(), wp, rtol=1e-5, atol=1e-6)
    assert np.allclose(md.cpu().numpy(), wm, rtol=1e-5, atol=1e-7)
    assert np.allclose(vd.cpu().numpy(), wv, rtol=1e-5, atol=1e-7)


def test_training_learns_a_separable_rule(nnc):
    from paper_2606_18314_amd import selector
    g = np.random.default_rng(3)
    X = g.random((8192, 6)).astype(np.float32)
    t_rep = 1.0 + 2.0 * X[:, 0]
    t_reb = np.full(8192, 2.0)
    y, w = selector.labels(t_rep, t_reb)
    params = selector.train(X, y, w, epochs=25, seed=1)
    ch = selector.decide(params, X)
    assert np.mean(ch == y) > 0.95
    assert selector.regret(ch, t_rep, t_reb) < 0.02


def _host_features(sc, res, S_prev):
    """The six features from the oracle's state (same power-of-two median rule)."""
    n = sc.n
    H, m, C, F = sc.frontier_entropy(model.CANDIDATES, res.candidates)
    r = sc.e[:1024] - S_prev
    r = r[(r > 0) & np.isfinite(r)]
    h = np.zeros(64, int)
    if r.size:
        ex = np.frexp(r)[1] - 1          # ilogb
        np.add.at(h, np.clip(ex + 48, 0, 63), 1)
    V = h.sum()
    radius = 0.0
    if V:
        b = int(np.searchsorted(np.cumsum(h) * 2 >= V, True))
        radius = 1.5 * 2.0 ** (b - 48)
    return np.array([F / n, H, math.log(n), sc.d, m / sc.G ** sc.d,
                     float(res.eps) / radius if radius > 0 else 0.0])


def test_single_scene_features(nnc):
    import paper_2606_18314_amd as p
    tr = synth.make_trajectory("clustered_drift", 5000, 3, 5, 5e-4, 9)
    ctx = p.NNCert(5000, 3, grid_g=12)
    sc = model.OracleScene(d=3, n=5000, G=12)
    ctx.init_certificates(torch.from_numpy(tr.frames[0]).cuda())
    sc.init_certificates(tr.frames[0])
    for t in range(1, 6):
        S_prev = sc.S
        e_prev = sc.e.copy()
        ctx.step(torch.from_numpy(tr.frames[t]).cuda(), tr.eps)
        res = sc.step(tr.frames[t])
        f = ctx.features().cpu().numpy()
        sc.e = e_prev                      # features use the keys of the pending step
        want = _host_features(sc, res, S_prev)
        assert np.allclose(f, want, rtol=1e-5, atol=1e-7), (t, f, want)
        ctx.repair()
        sc.repair()
    ctx.close()


def test_batch_cost_accounting_and_snapshots(nnc):
    """Per-scene wall-clock accounting of the batched step (NNC_BATCH_TIMING): every
    scene with queries reports query time, a grid build time exactly where a grid was
    built; a batch snapshot restores the state bit for bit (the same step run twice
    from it gives the same arrays)."""
    import synth
    from paper_2606_18314_amd import selector
    specs = selector.scene_specs(12, seed=7400, n_hi=6000)
    trajs = [synth.make_trajectory(sp["family"], sp["n"], sp["d"], 3, sp["eps"], tuple(sp["seed"])) for sp in specs]
    frames = [torch.from_numpy(synth.concat_frame(trajs, t)).cuda() for t in range(4)]
    b = nnc.NNCBatch([t.n for t in trajs], [t.d for t in trajs], timing=True, features=True)
    b.init(frames[0])
    b.step(frames[1], nnc.POLICY_REPAIR)
    snap = b.snapshot()
    b.step(frames[2], nnc.POLICY_REBUILD)
    st = b.stats()
    assert all(x["t_grid_us"] > 0 and x["t_query_us"] > 0 and x["t_filter_us"] > 0 for x in st)
    first = {k: v.clone() for k, v in b.state().items()}
    b.restore(snap)
    b.step(frames[2], nnc.POLICY_REBUILD)
    again = b.state()
    for k in first:
        assert torch.equal(first[k], again[k]), k
    b.restore(snap)
    b.step(frames[2], nnc.POLICY_REPAIR)
    st = b.stats()
    for x in st:
        assert x["t_query_us"] > 0 if x["n_cand"] > 0 else x["t_query_us"] >= 0
    b.close()


def test_trained_selector_beats_always_repair_on_held_out_transitions(nnc):
    """The committed network (trained on transitions labelled inside the batched step)
    against always repairing, on held-out scenes of other seeds with step sizes over a
    decade: its time regret, with the learned policy's feature and inference cost added
    to every transition inside its band (where it computes features), is lower.  The
    held-out batch has the training batches' size (128 scenes; a scene's labels depend
    on the batch it runs in) and 40 steps per scene."""
    from paper_2606_18314_amd import selector
    params, meta = selector.load_params()
    assert params is not None
    specs = selector.scene_specs(128, seed=9900)
    data = selector.collect_batched(specs, 40)
    X, tr, tb = data["X"], data["t_repair"], data["t_rebuild"]
    c_inf = float(meta.get("inference_wave_us_per_scene_step", 0.0))
    lo, hi = meta.get("band", [0.0, 2.0])
    ch, band = selector.band_choice(X, selector.decide(params, X), lo, hi)
    r_net = selector.regret(ch, tr, tb, np.where(band, c_inf, 0.0))
    r_rep = selector.regret(np.zeros(len(X), np.int32), tr, tb)
    print(f"held-out regret: learned {r_net:.4f} (inference {c_inf:.2f} wave-us on {band.mean():.3f} of the "
          f"transitions), always repair {r_rep:.4f}")
    assert r_net < r_rep
