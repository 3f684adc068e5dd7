"""GPU parity of the batched step: every scene of a batch against its own oracle.

The batch chooses a strategy per scene and step (fixed, by the size threshold,
or by the selector network); the oracle of each scene replays the chosen
strategy, and every state array of the scene must match bit for bit.
"""
import numpy as np
import pytest

import synth
from oracle import model

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

H_TOL = 1e-12


@pytest.fixture(scope="module")
def nnc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_18314_amd as p
    p.load()
    return p


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def bits(a):
    return np.ascontiguousarray(a).view(np.uint32 if a.dtype == np.float32 else np.uint64)


def make_scenes(seed, count, nmax=6000, steps=10):
    g = np.random.default_rng(seed)
    trajs, grids = [], []
    sizes = [0, 1, 2, 3, 40, 300] + list(np.exp(g.uniform(np.log(100), np.log(nmax), count)).astype(int))
    for s, n in enumerate(sizes):
        d = int(g.integers(2, 4))
        fam = synth.FAMILIES[int(g.integers(0, len(synth.FAMILIES)))]
        tr = synth.make_trajectory(fam, int(n), d, steps, 5e-4, (seed, s))
        trajs.append(tr)
        # a deliberately wide range of resolutions, including fine grids that widen often
        grids.append(int(g.choice([1, 3, 7, 15, 30])) if n < 500 else int(g.choice([8, 15, 25, 40])))
    return trajs, grids


def localized_scene(seed, d, n, steps, radius=0.15):
    """Points of the unit box of which only those within `radius` of one centre move."""
    g = np.random.default_rng(seed)
    p = g.random((d, n))
    c = np.full((d, 1), 0.4)
    frames = [p.copy()]
    for _ in range(steps):
        movers = np.linalg.norm(p - c, axis=0) < radius
        p = p + np.where(movers, g.standard_normal((d, n)) * 3e-4, 0.0)
        frames.append(p.copy())
    return synth.Trajectory("custom", d, n, -1.0, np.array(frames, dtype=np.float32))


def run_batch(nnc, trajs, grids, policy, tau=0.5, params=None, lanes=0, budget=False):
    ns = [t.n for t in trajs]
    ds = [t.d for t in trajs]
    b = nnc.NNCBatch(ns, ds, grids=grids, lanes=lanes, features=True, budget=budget)
    rule = "budget" if budget else "clock"
    oracles = [model.OracleScene(d=t.d, n=t.n, G=G, rule=rule) for t, G in zip(trajs, grids)]
    steps = trajs[0].steps
    frames = [dev(synth.concat_frame(trajs, t)) for t in range(steps + 1)]
    if params is not None:
        b.selector_load(params)
    b.init(frames[0])
    for o, tr in zip(oracles, trajs):
        o.init_certificates(tr.frames[0])
    chosen = []
    for t in range(1, steps + 1):
        b.step(frames[t], policy, tau)
        stats = b.stats()
        st = {k: v.cpu().numpy() for k, v in b.state().items()}
        for s, (o, tr) in enumerate(zip(oracles, trajs)):
            res = o.step(tr.frames[t])
            assert stats[s]["err"] == 0
            assert stats[s]["n_cand"] == res.candidates.size, (s, t)
            assert stats[s]["eps"] == float(res.eps) and stats[s]["S"] == res.S
            H, m, C, F = o.frontier_entropy(model.CANDIDATES, res.candidates)
            assert (stats[s]["m_cand"], stats[s]["C"]) == (m, C), (s, t)
            assert abs(stats[s]["H_cand"] - H) <= H_TOL * max(1.0, abs(H))
            if stats[s]["strategy"] == 1:
                o.rebuild()
            else:
                o.repair()
            chosen.append(stats[s]["strategy"])
            a, z = int(b.point_off[s]), int(b.point_off[s + 1])
            assert np.array_equal(st["nn"][a:z], o.nn), (s, t)
            assert np.array_equal(bits(st["d1"][a:z]), bits(o.d1)), (s, t)
            assert np.array_equal(bits(st["d2"][a:z]), bits(o.d2)), (s, t)
            assert np.array_equal(bits(st["e"][a:z]), bits(o.e)), (s, t)
            assert np.array_equal(st["cell"][a:z], o.cell), (s, t)
            assert np.array_equal(st["fail"][a:z].astype(bool), o.fail), (s, t)
            H, m, C, F = o.frontier_entropy(model.FAILED)
            assert stats[s]["n_fail"] == F
            assert abs(stats[s]["H_fail"] - H) <= H_TOL * max(1.0, abs(H))
            f = stats[s]["features"]
            assert f[0] == pytest.approx(res.candidates.size / tr.n if tr.n else 0.0, rel=1e-6)
            assert f[3] == tr.d
        # no scene misses a failure: state nn equals brute force at the new positions
        for s, (o, tr) in enumerate(zip(oracles, trajs)):
            a, z = int(b.point_off[s]), int(b.point_off[s + 1])
            assert np.array_equal(st["nn"][a:z], model.top2(tr.frames[t])[0])
    b.close()
    return chosen


@pytest.mark.parametrize("dims", ["plane", "cube", "empty_plane"])
def test_batch_one_dimension_and_an_empty_chain(nnc, dims):
    """Batches whose scenes all share one dimension (the step's kernels in one chain),
    and a mixed batch whose plane scenes are all empty (the plane's chain of kernels
    has no ingest tile), under the repair and the rebuild policy."""
    spec = {"plane": [(2, 500), (2, 3000), (2, 1200)],
            "cube": [(3, 800), (3, 2500), (3, 40)],
            "empty_plane": [(2, 0), (3, 1500), (2, 0), (3, 700)]}[dims]
    trajs, grids = [], []
    for k, (d, n) in enumerate(spec):
        fam = synth.FAMILIES[k % len(synth.FAMILIES)]
        trajs.append(synth.make_trajectory(fam, n, d, 6, 5e-4, (71, k)))
        grids.append(15 if n < 1000 else 25)
    for policy in (0, 1):
        run_batch(nnc, trajs, grids, policy)


@pytest.mark.parametrize("policy", [0, 1, 2])
def test_batch_policies_match_per_scene_oracles(nnc, policy):
    trajs, grids = make_scenes(11 + policy, 10)
    chosen = run_batch(nnc, trajs, grids, policy, tau=0.45)
    if policy == 0:
        assert set(chosen) == {0}
    if policy == 1:
        assert set(chosen) == {1}


@pytest.mark.parametrize("policy", [0, 2])
def test_batch_budget_matches_per_scene_oracles(nnc, policy):
    """The per-point motion budget in every scene (NNC_BATCH_BUDGET): candidates,
    moved keys and certificates of each scene against its oracle under the budget
    rule, with two scenes whose motion is confined to one ball (the block-local test
    keeps the still blocks' certificates there)."""
    trajs, grids = make_scenes(61 + policy, 8)
    steps = trajs[0].steps
    for k, d in enumerate((2, 3)):
        trajs.append(localized_scene(70 + k, d, 6000 if d == 2 else 5000, steps))
        grids.append(60 if d == 2 else 15)
    run_batch(nnc, trajs, grids, policy, tau=0.45, budget=True)


@pytest.mark.parametrize("lanes", [1, 8, 16, 32, 64])
def test_batch_lane_widths(nnc, lanes):
    trajs, grids = make_scenes(21, 6, nmax=4000, steps=6)
    run_batch(nnc, trajs, grids, 2, tau=0.5, lanes=lanes)


def test_batch_equals_single_scene_contexts(nnc):
    trajs, grids = make_scenes(41, 5, steps=6)
    ns = [t.n for t in trajs]
    ds = [t.d for t in trajs]
    b = nnc.NNCBatch(ns, ds, grids=grids)
    frames = [dev(synth.concat_frame(trajs, t)) for t in range(7)]
    b.init(frames[0])
    ctxs = []
    for tr, G in zip(trajs, grids):
        c = nnc.NNCert(tr.n, tr.d, grid_g=G)
        c.init_certificates(dev(tr.frames[0]))
        ctxs.append(c)
    for t in range(1, 7):
        b.step(frames[t], 0)
        for c, tr in zip(ctxs, trajs):
            c.step(dev(tr.frames[t]))
            c.repair()
    bs = b.state()
    for s, c in enumerate(ctxs):
        a, z = int(b.point_off[s]), int(b.point_off[s + 1])
        cs = c.state()
        for k in ("nn", "d1", "d2", "e", "cell", "fail"):
            assert torch.equal(bs[k][a:z], cs[k]), (s, k)
        c.close()
    b.close()
