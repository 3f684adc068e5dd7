"""Learned repair/rebuild selector: labelled transitions, training, evaluation.

Transitions are produced by the method itself on seeded synthetic scenes: each
step's six features come from the library (nnc_features), and both strategies
are timed on the same pending step with HIP events (the state is restored
between them), the label being the faster one.  The network (6-64-64-2, ReLU)
is trained by the library's own forward/backward and Adam kernels on a
cost-weighted cross-entropy (weight |T_repair - T_rebuild| / min(T_repair,
T_rebuild), clipped), with feature standardisation folded into the first layer
afterwards, so that the batched step can evaluate the raw features directly.

Its error is judged by the time regret on held-out transitions:
    regret = sum_t T(choice_t) / sum_t min(T_repair_t, T_rebuild_t) - 1.
The plain size-threshold rule (rebuild iff |F|/N >= tau, tau fitted on the
training set) is the fallback and the baseline.
"""
from __future__ import annotations

import json
import math
import os
import time

import numpy as np
import torch

from . import binding

HERE = os.path.dirname(os.path.abspath(__file__))
PARAMS_PATH = os.path.join(HERE, "selector_params.npy")

NF, NH = 6, 64
SHAPES = [(NH, NF), (NH,), (NH, NH), (NH,), (2, NH), (2,)]


def scene_specs(count: int, seed: int, n_lo: int = 500, n_hi: int = 20000):
    """Scenes like the batched workload (log-uniform N, d in {2,3}, the five families),
    with the step size spread over a decade so that both strategies get to win."""
    import synth
    g = synth.rng(seed)
    specs = []
    for s in range(count):
        n = int(round(math.exp(g.uniform(math.log(n_lo), math.log(n_hi)))))
        d = 2 if g.random() < 0.5 else 3
        fam = synth.FAMILIES[int(g.integers(0, len(synth.FAMILIES)))]
        eps = float(np.exp(g.uniform(np.log(1e-4), np.log(5e-3))))
        specs.append({"family": fam, "n": n, "d": d, "eps": eps, "seed": [seed, s]})
    return specs


def collect(specs, steps: int, reps: int = 2, lanes: int = 16, log=None):
    """Features and timed strategies of every step of every scene.

    Returns a dict of numpy arrays: X [M,6], t_repair [M], t_rebuild [M] (ms)."""
    import synth
    X, trep, treb = [], [], []
    s = torch.cuda.Stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    t0 = time.time()
    for k, sp in enumerate(specs):
        tr = synth.make_trajectory(sp["family"], sp["n"], sp["d"], steps, sp["eps"], tuple(sp["seed"]))
        frames = torch.from_numpy(tr.frames).cuda()
        with torch.cuda.stream(s):
            ctx = binding.NNCert(sp["n"], sp["d"], stream=s.cuda_stream, lanes=lanes)
            ctx.init_certificates(frames[0])
        for t in range(1, steps + 1):
            with torch.cuda.stream(s):
                ctx.step(frames[t], sp["eps"])
            f = ctx.features().cpu().numpy()
            snap = ctx.snapshot(into=snap) if t > 1 else ctx.snapshot()
            best_rep, best_reb = math.inf, math.inf
            for _ in range(reps):
                for strat in (0, 1):
                    with torch.cuda.stream(s):
                        ctx.restore(snap)
                    ev[0].record(s)
                    with torch.cuda.stream(s):
                        ctx.repair() if strat == 0 else ctx.rebuild()
                    ev[1].record(s)
                    ev[1].synchronize()
                    ms = ev[0].elapsed_time(ev[1])
                    if strat == 0:
                        best_rep = min(best_rep, ms)
                    else:
                        best_reb = min(best_reb, ms)
            with torch.cuda.stream(s):
                ctx.restore(snap)
                ctx.repair()
            X.append(f)
            trep.append(best_rep)
            treb.append(best_reb)
        del snap
        ctx.close()
        if log and (k + 1) % 50 == 0:
            log(f"collected {k + 1}/{len(specs)} scenes, {len(X)} transitions, {time.time() - t0:.0f} s")
    return {"X": np.array(X, np.float32), "t_repair": np.array(trep), "t_rebuild": np.array(treb)}


WAVES_PER_WORKGROUP = 16   # the batched filter and grid build run 1024-thread workgroups


def scene_cost(st: dict) -> float:
    """A scene-step's strategy-dependent cost inside the batched step, in wave-microseconds:
    its grid build's workgroup time (16 waves) plus the summed time of the query waves
    that worked on it (the filter's work is the same for both strategies)."""
    return WAVES_PER_WORKGROUP * st["t_grid_us"] + st["t_query_us"]


def collect_batched(specs, steps: int, batch_size: int = 128, lanes: int = 0, log=None):
    """Features and the in-batch costs of both strategies of every scene-step.

    Scenes are advanced in batches with the deployment's grids (the batch tuner's
    rule); at each step the batch state is saved, the step is run with every scene
    repaired and again with every scene rebuilt (per-scene wall-clock accounting,
    NNC_BATCH_TIMING), and the batch continues from the repaired step.  Returns X
    [M,6], t_repair [M], t_rebuild [M] (wave-microseconds, see scene_cost)."""
    import synth
    from . import autotune
    X, trep, treb = [], [], []
    s = torch.cuda.Stream()
    t0 = time.time()
    for b0 in range(0, len(specs), batch_size):
        chunk = specs[b0:b0 + batch_size]
        trajs = [synth.make_trajectory(sp["family"], sp["n"], sp["d"], steps, sp["eps"], tuple(sp["seed"]))
                 for sp in chunk]
        ns = [t.n for t in trajs]
        ds = [t.d for t in trajs]
        frames = [torch.from_numpy(synth.concat_frame(trajs, t)).cuda() for t in range(steps + 1)]
        grids = autotune.batch_grids(frames[0], ns, ds, lanes=lanes, factor=1.5, cells_per_point=8)
        with torch.cuda.stream(s):
            b = binding.NNCBatch(ns, ds, grids=grids, lanes=lanes, stream=s.cuda_stream, features=True,
                                 timing=True, eager=True)
            b.init(frames[0])
        snap = None
        for t in range(1, steps + 1):
            with torch.cuda.stream(s):
                snap = b.snapshot(into=snap)
                b.step(frames[t], binding.POLICY_REPAIR)
            st_rep = b.stats()
            with torch.cuda.stream(s):
                b.restore(snap)
                b.step(frames[t], binding.POLICY_REBUILD)
            st_reb = b.stats()
            with torch.cuda.stream(s):
                b.restore(snap)
                b.step(frames[t], binding.POLICY_REPAIR)
            for a, r in zip(st_rep, st_reb):
                X.append(a["features"])
                trep.append(scene_cost(a))
                treb.append(scene_cost(r))
        del snap
        b.close()
        if log:
            log(f"collected {min(b0 + batch_size, len(specs))}/{len(specs)} scenes, {len(X)} transitions, "
                f"{time.time() - t0:.0f} s")
    return {"X": np.array(X, np.float32), "t_repair": np.array(trep), "t_rebuild": np.array(treb)}


def inference_cost(specs, steps: int, params: np.ndarray, tau: float, lanes: int = 0, reps: int = 5):
    """Per scene-step cost of the learned policy's features and network inside the batched
    step, in the labels' unit (wave-microseconds).  The same step is run from the same
    state under the size rule set to always repair and under the learned policy with a
    network whose output always says repair (the trained weights with the output bias
    shifted), so both make the same decisions and differ only by the features and the
    network; the wall-clock difference (median of reps) is converted to wave-microseconds
    with the step's own ratio of summed scene costs to wall time, and shared over the
    scenes."""
    import synth
    from . import autotune
    trajs = [synth.make_trajectory(sp["family"], sp["n"], sp["d"], steps, sp["eps"], tuple(sp["seed"]))
             for sp in specs]
    ns = [t.n for t in trajs]
    ds = [t.d for t in trajs]
    frames = [torch.from_numpy(synth.concat_frame(trajs, t)).cuda() for t in range(steps + 1)]
    grids = autotune.batch_grids(frames[0], ns, ds, lanes=lanes, factor=1.5, cells_per_point=8)
    repair_only = params.astype(np.float32).copy()
    repair_only[-2], repair_only[-1] = 1e6, -1e6          # b3: the repair logit always wins
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b = binding.NNCBatch(ns, ds, grids=grids, lanes=lanes, stream=s.cuda_stream, timing=True, eager=True)
        b.selector_load(torch.from_numpy(repair_only).cuda())
        b.init(frames[0])
    snap = None
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    per_scene = []
    for t in range(1, steps + 1):
        with torch.cuda.stream(s):
            snap = b.snapshot(into=snap)
        wall = {}
        for pol, tv in ((binding.POLICY_THRESHOLD, 2.0), (binding.POLICY_LEARNED, tau)):
            times = []
            for _ in range(reps):
                with torch.cuda.stream(s):
                    b.restore(snap)
                    ev[0].record(s)
                    b.step(frames[t], pol, tv)
                    ev[1].record(s)
                ev[1].synchronize()
                times.append(ev[0].elapsed_time(ev[1]) * 1e3)
            wall[pol] = float(np.median(times))
        st = b.stats()
        busy = sum(scene_cost(x) for x in st)
        ratio = busy / wall[binding.POLICY_THRESHOLD]           # wave-microseconds per wall microsecond
        dwall = wall[binding.POLICY_LEARNED] - wall[binding.POLICY_THRESHOLD]
        per_scene.append(dwall * ratio / len(specs))
        with torch.cuda.stream(s):
            b.restore(snap)
            b.step(frames[t], binding.POLICY_REPAIR)
    b.close()
    return max(0.0, float(np.median(per_scene)))


def fit_band(X, t_rep, t_reb, choice, c_inf: float):
    """Band [lo, hi) of candidate fractions in which the network decides (outside it:
    repair below lo, rebuild from hi on), minimising the regret with the features' and
    network's cost c_inf charged to the transitions inside the band."""
    f0 = X[:, 0]
    qs = np.unique(np.concatenate([[0.0, 2.0], np.quantile(f0, np.linspace(0.0, 1.0, 41))]))
    best = (math.inf, 0.0, 2.0)
    for lo in qs:
        for hi in qs:
            if hi < lo:
                continue
            band = (f0 >= lo) & (f0 < hi)
            ch = np.where(band, choice, (f0 >= hi).astype(np.int32))
            r = regret(ch, t_rep, t_reb, np.where(band, c_inf, 0.0))
            if r < best[0]:
                best = (r, float(lo), float(hi))
    return best[1], best[2]


def band_choice(X, choice, lo: float, hi: float):
    f0 = X[:, 0]
    band = (f0 >= lo) & (f0 < hi)
    return np.where(band, choice, (f0 >= hi).astype(np.int32)), band


def labels(t_rep, t_reb, clip: float = 10.0, floor: float = 0.05):
    y = (t_reb < t_rep).astype(np.int32)
    w = np.abs(t_rep - t_reb) / np.minimum(t_rep, t_reb)
    return y, np.clip(w, floor, clip).astype(np.float32)


def he_init(seed: int) -> np.ndarray:
    g = np.random.default_rng(seed)
    parts = []
    for shape in SHAPES:
        parts.append(g.standard_normal(shape) * np.sqrt(2.0 / shape[1]) if len(shape) == 2 else np.zeros(shape))
    return np.concatenate([p.reshape(-1) for p in parts]).astype(np.float32)


def fold_standardisation(params: np.ndarray, mu: np.ndarray, sd: np.ndarray) -> np.ndarray:
    """Parameters acting on raw features from ones trained on (x - mu) / sd."""
    p = params.astype(np.float64).copy()
    W1 = p[:NH * NF].reshape(NH, NF)
    b1 = p[NH * NF:NH * NF + NH]
    W1n = W1 / sd
    b1n = b1 - W1n @ mu
    p[:NH * NF] = W1n.reshape(-1)
    p[NH * NF:NH * NF + NH] = b1n
    return p.astype(np.float32)


def train(X, y, w, epochs: int = 30, batch: int = 1024, lr: float = 1e-3, seed: int = 0, log=None):
    """Train on the GPU kernels; returns raw-feature parameters (numpy float32)."""
    mu = X.mean(0).astype(np.float64)
    sd = X.std(0).astype(np.float64)
    sd[sd < 1e-6] = 1.0
    Xs = ((X - mu) / sd).astype(np.float32)
    dev = torch.device("cuda")
    Xd = torch.from_numpy(Xs).to(dev)
    yd = torch.from_numpy(y.astype(np.int32)).to(dev)
    wd = torch.from_numpy(w.astype(np.float32)).to(dev)
    p = torch.from_numpy(he_init(seed)).to(dev)
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    ws = torch.empty(binding.load().nnc_mlp_workspace_bytes(batch) // 4 + 1, dtype=torch.float32, device=dev)
    g = np.random.default_rng(seed)
    step = 0
    M = X.shape[0]
    for ep in range(epochs):
        order = torch.from_numpy(g.permutation(M)).to(dev)
        tot = 0.0
        nb = 0
        for b0 in range(0, M - batch + 1, batch):
            idx = order[b0:b0 + batch]
            xb = Xd.index_select(0, idx).contiguous()
            yb = yd.index_select(0, idx).contiguous()
            wb = wd.index_select(0, idx).contiguous()
            loss, gr = binding.mlp_grad(p, xb, yb, wb, ws)
            step += 1
            binding.mlp_adam(p, m, v, gr, step, lr=lr)
            tot += float(loss.item()) if (nb % 20 == 0) else 0.0
            nb += 1
        if log and (ep % 5 == 0 or ep == epochs - 1):
            log(f"epoch {ep}: sampled loss {tot / max(1, (nb + 19) // 20):.4f}")
    return fold_standardisation(p.cpu().numpy(), mu, sd)


def decide(params: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Network decisions (1 = rebuild) by the library's inference kernel."""
    p = torch.from_numpy(params.astype(np.float32)).cuda()
    logits = binding.mlp_forward(p, torch.from_numpy(X.astype(np.float32)).cuda()).cpu().numpy()
    return (logits[:, 1] > logits[:, 0]).astype(np.int32)


def regret(choice, t_rep, t_reb, extra: float = 0.0) -> float:
    """Time regret against the per-step best strategy, sum T(choice) / sum min - 1; extra
    is a per-transition cost of making the choice (features and inference)."""
    cost = np.where(choice == 1, t_reb, t_rep) + extra
    return float(cost.sum() / np.minimum(t_rep, t_reb).sum() - 1.0)


def fit_threshold(X, t_rep, t_reb):
    """tau minimising the time regret of 'rebuild iff |F|/N >= tau' on the given set."""
    best = (math.inf, 1.0)
    for tau in np.linspace(0.0, 1.01, 203):
        r = regret((X[:, 0] >= tau).astype(np.int32), t_rep, t_reb)
        if r < best[0]:
            best = (r, float(tau))
    return best[1], best[0]


def save(params: np.ndarray, meta: dict, path: str = PARAMS_PATH):
    np.save(path, params.astype(np.float32), allow_pickle=False)
    with open(os.path.splitext(path)[0] + ".json", "w") as f:
        json.dump(meta, f, indent=1)


def load_params(path: str = PARAMS_PATH):
    if not os.path.exists(path):
        return None, None
    p = np.load(path, allow_pickle=False)
    meta_path = os.path.splitext(path)[0] + ".json"
    meta = json.load(open(meta_path)) if os.path.exists(meta_path) else {}
    return p, meta


def main_batched(args, log):
    """Labels timed inside the batched step (collect_batched), training on the GPU
    kernels, the threshold fitted on the same set, and on held-out scenes (other seeds)
    the regrets with the learned policy's feature and inference cost included."""
    train_specs = scene_specs(args.scenes, args.seed)
    test_specs = scene_specs(max(args.scenes // 4, 32), args.seed + 4000)
    t0 = time.time()
    tr = collect_batched(train_specs, args.steps, log=log)
    te = collect_batched(test_specs, args.steps, log=log)
    log(f"{len(tr['X'])} training and {len(te['X'])} held-out transitions in {time.time() - t0:.0f} s; rebuild "
        f"cheaper in {np.mean(tr['t_rebuild'] < tr['t_repair']):.3f} of the training ones")
    Xtr, rtr, btr = tr["X"], tr["t_repair"], tr["t_rebuild"]
    Xte, rte, bte = te["X"], te["t_repair"], te["t_rebuild"]
    y, w = labels(rtr, btr)
    t1 = time.time()
    params = train(Xtr, y, w, epochs=args.epochs, seed=args.seed, log=log)
    train_s = time.time() - t1
    tau, _ = fit_threshold(Xtr, rtr, btr)
    c_inf = inference_cost(test_specs[:64], 12, params, tau)
    lo, hi = fit_band(Xtr, rtr, btr, decide(params, Xtr), c_inf)
    ch_net, band = band_choice(Xte, decide(params, Xte), lo, hi)
    res = {
        "labels": "timed inside the batched step (per-scene wall-clock accounting, wave-microseconds)",
        "transitions": int(len(Xtr) + len(Xte)), "train": int(len(Xtr)), "held_out": int(len(Xte)),
        "train_seconds": train_s,
        "rebuild_wins_fraction": float(np.mean(btr < rtr)),
        "inference_wave_us_per_scene_step": c_inf,
        "band": [lo, hi], "held_out_fraction_in_band": float(band.mean()),
        "mean_best_wave_us_per_scene_step": float(np.minimum(rte, bte).mean()),
        "regret_learned": regret(ch_net, rte, bte, np.where(band, c_inf, 0.0)),
        "regret_learned_without_inference": regret(ch_net, rte, bte),
        "regret_network_everywhere": regret(decide(params, Xte), rte, bte, c_inf),
        "regret_threshold": regret((Xte[:, 0] >= tau).astype(np.int32), rte, bte),
        "regret_always_repair": regret(np.zeros(len(Xte), np.int32), rte, bte),
        "regret_always_rebuild": regret(np.ones(len(Xte), np.int32), rte, bte),
        "tau": tau, "accuracy_learned": float(np.mean(ch_net == (bte < rte))),
        "specs_seed": args.seed, "held_out_seed": args.seed + 4000, "steps_per_scene": args.steps,
        "scenes": args.scenes,
    }
    log(json.dumps(res))
    save(params, res, args.out)


def main():
    import argparse
    ap = argparse.ArgumentParser(description="collect labelled transitions and train the selector")
    ap.add_argument("--scenes", type=int, default=1000)
    ap.add_argument("--steps", type=int, default=110)
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--seed", type=int, default=5000)
    ap.add_argument("--holdout", type=float, default=0.2)
    ap.add_argument("--out", default=PARAMS_PATH)
    ap.add_argument("--single-scene", action="store_true",
                    help="label with isolated single-scene timing instead of inside the batched step")
    args = ap.parse_args()

    def log(msg):
        print(msg, flush=True)

    if not args.single_scene:
        main_batched(args, log)
        return

    specs = scene_specs(args.scenes, args.seed)
    n_train = int(round(len(specs) * (1 - args.holdout)))
    t0 = time.time()
    data = collect(specs, args.steps, args.reps, log=log)
    per_scene = args.steps
    cut = n_train * per_scene
    Xtr, Xte = data["X"][:cut], data["X"][cut:]
    rtr, rte = data["t_repair"][:cut], data["t_repair"][cut:]
    btr, bte = data["t_rebuild"][:cut], data["t_rebuild"][cut:]
    log(f"{len(data['X'])} transitions ({len(Xtr)} train, {len(Xte)} held out) in {time.time() - t0:.0f} s; "
        f"rebuild faster in {np.mean(data['t_rebuild'] < data['t_repair']):.3f} of them")
    y, w = labels(rtr, btr)
    t1 = time.time()
    params = train(Xtr, y, w, epochs=args.epochs, seed=args.seed, log=log)
    train_s = time.time() - t1
    tau, r_tau_train = fit_threshold(Xtr, rtr, btr)
    ch_net = decide(params, Xte)
    res = {
        "transitions": int(len(data["X"])), "train": int(len(Xtr)), "held_out": int(len(Xte)),
        "train_seconds": train_s,
        "rebuild_wins_fraction": float(np.mean(data["t_rebuild"] < data["t_repair"])),
        "regret_learned": regret(ch_net, rte, bte),
        "regret_threshold": regret((Xte[:, 0] >= tau).astype(np.int32), rte, bte),
        "regret_always_repair": regret(np.zeros(len(Xte), np.int32), rte, bte),
        "regret_always_rebuild": regret(np.ones(len(Xte), np.int32), rte, bte),
        "tau": tau, "accuracy_learned": float(np.mean(ch_net == (bte < rte))),
        "specs_seed": args.seed, "steps_per_scene": args.steps, "scenes": args.scenes,
    }
    log(json.dumps(res))
    save(params, res, args.out)


if __name__ == "__main__":
    main()
