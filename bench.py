#!/usr/bin/env python3
"""Benchmark of the certificate-maintenance step on one MI355X.

Workload (the headline configuration): N = 16000 points in the unit cube,
d = 3, the five motion families (uniform Brownian, ring rotation, adversarial
crossing, clustered drift, shear band), eps = 5e-4, seeded synthetic
trajectories resident in HBM before timing.  One bench step advances all five
scenes by one transition through the whole maintenance path: ingest
(eps_t, cells), safety filter and ordered compaction, grid repair of the
candidates (with the amortised grid refresh) and the failure-entropy reduction.

Legs (--legs):
  repair    the method (Algorithm 1 with the clock), captured once in a HIP graph
            and replayed, the five scenes as parallel branches: the headline
            value; also one stream, eager launches, and per-kernel HIP events;
  rebuild   the O(N) grid rebuild competitor in place of the repair;
  allpairs  the exact all-pairs top-2 competitor (VALU roofline);
  sweep     N = 2^20 planar scene, candidate fractions 0.1 % to 50 %, localized
            and diffuse motion: repair against rebuild, and H of the frontier;
  batched   512 scenes of uneven N advanced together under four strategy
            policies (repair, rebuild, size threshold, the learned selector),
            against one context per scene; selector regret on fresh scenes;
  scaling   the step, repair and rebuild kernels from N = 2^16 to 2^26 with
            achieved bandwidth;
  audit     the certificate-failure audit of Table 1 on the ten families
            (d = 2 and 3, three step scales, N = 16000): failure fraction,
            misses of the safety rule and its over-flagging, and the local
            predictor rho's recall and false flags;
  queue     candidate detection by the expiry calendar against the scan of
            all keys, N = 2^20 to 2^24 at low pressure;
plus a certification pass (every timed step of the repair and rebuild legs
audited by the GPU all-pairs oracle: zero missed failures and bitwise-equal
fresh certificates), HBM traffic of the dominant kernel from committed
rocprofv3 counters, and the CPU oracle timed on a bounded sample.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "certified point-steps/s (N=16k, d=3): repair vs rebuild vs batched; % roofline"
N, D, EPS = 16000, 3, 5e-4
HBM_PEAK_GBS = 8000.0
# FP32 VALU issue rate without FMA and without packed FP32:
# 256 CUs x 64 lanes x 2.4 GHz = 39.3e12 operations/s.
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
FP32_PUBLISHED_TFLOPS = 157.3


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=190)
    ap.add_argument("--branches", type=int, default=5, help="streams (graph branches) the five headline scenes use")
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--legs", default="repair,rebuild,allpairs,batched,sweep,scaling,audit,queue")
    ap.add_argument("--queue-exps", default="20,22,24", help="log2 N of the queue leg's scenes")
    ap.add_argument("--sweep-reps", type=int, default=3)
    ap.add_argument("--repeats", type=int, default=5, help="timed replays per leg (the median is reported)")
    ap.add_argument("--scaling-lanes", type=int, default=4, help="lanes per query of the scaling leg's queries")
    ap.add_argument("--scaling-exps", default="16,18,20,22,24,26",
                    help="log2 N of the scaling leg's scenes")
    ap.add_argument("--scenes", type=int, default=512)
    ap.add_argument("--batch-steps", type=int, default=100)
    ap.add_argument("--batch-tune", type=int, default=1,
                    help="1: time the batch tuner's choices; 0: use its usual choice without timing")
    ap.add_argument("--batch-policies", default="repair,rebuild,threshold,learned,repair_budget",
                    help="policies of the batched leg")
    ap.add_argument("--batch-loops", type=int, default=1,
                    help="1: also time the one-context-per-scene baselines")
    ap.add_argument("--regret-scenes", type=int, default=100)
    ap.add_argument("--regret-steps", type=int, default=40)
    ap.add_argument("--grid", default="table",
                    help="'table' (the committed tuning table, paper_2606_18314_amd/tuned_cube16k.json), "
                         "'auto' (tuned per family now) or an integer G for all")
    ap.add_argument("--grid-json", default="", help='fixed {"family": [G, lanes], ...} instead of tuning')
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-certify", action="store_true")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    return ap.parse_args()


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), for the CPU baseline's record."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def progress(msg):
    """One line on stderr per finished piece of work (long runs stay visibly alive)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def src_hash(*names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2606_18314_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic(kernel_tag, current_hash):
    """HBM bytes per dispatch from a committed rocprofv3 --pmc summary, or None when
    the summary is missing or was taken from a different kernel source."""
    path = os.path.join(ROOT, "profiles", f"pmc_{kernel_tag}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_hash") != current_hash:
        return None
    try:
        return float(vals["hbm_bytes_per_dispatch"])
    except (KeyError, ValueError):
        return None


def batched_leg(args, nnc, synth, autotune, torch):
    """Batched workload: 512 scenes advanced together per launch, under each strategy policy,
    against the same scenes advanced one by one (one context per scene)."""
    from paper_2606_18314_amd import selector
    t0 = time.time()
    spec = synth.batch_spec(args.scenes, seed=4000)
    steps = args.batch_steps
    trajs = synth.batch_trajectories(spec, steps + 1, eps=5e-4, seed=4000)
    ns = [int(v) for v in spec.n]
    ds = [int(v) for v in spec.d]
    frames = [torch.from_numpy(synth.concat_frame(trajs, t)).cuda() for t in range(steps + 2)]
    torch.cuda.synchronize()
    gen_s = time.time() - t0
    s = torch.cuda.Stream()
    if args.batch_tune:
        grids, lanes, table = autotune.tune_batch(frames, ns, ds, eps_steps=8, stream=s)
    else:   # the tuner's usual choice, without its timing sweep
        lanes, table = 0, {}   # the library's default: 4 lanes per plane query, 8 per cube query
        grids = autotune.batch_grids(frames[0], ns, ds, lanes=0, factor=1.5, cells_per_point=8)
    params, meta = selector.load_params()
    tau = float(meta.get("tau", 0.5)) if meta else 0.5
    total = sum(ns)
    res = {"scenes": len(ns), "points": total, "steps": steps, "lanes": lanes, "tuning_ms": table,
           "generator_seconds": round(gen_s, 1), "tau": tau}

    def ev():
        return torch.cuda.Event(enable_timing=True)

    # the paper's rule under each policy, then repair with the per-point motion budget
    policies = [("repair", 0, False), ("rebuild", 1, False), ("threshold", 2, False)]
    if params is not None:
        policies.append(("learned", 3, False))
    policies.append(("repair_budget", 0, True))
    wanted = set(args.batch_policies.split(","))
    policies = [p for p in policies if p[0] in wanted]
    pdev = torch.from_numpy(params).cuda() if params is not None else None
    for name, pol, budget in policies:
        with torch.cuda.stream(s):
            b = nnc.NNCBatch(ns, ds, grids=grids, lanes=lanes, stream=s.cuda_stream, budget=budget)
            if pdev is not None:
                b.selector_load(pdev)
                band = meta.get("band", [0.0, 2.0])
                b.selector_band(band[0], band[1])
            b.init(frames[0])
            b.step(frames[1], pol, tau)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            for t in range(2, steps + 2):
                b.step(frames[t], pol, tau)
        torch.cuda.synchronize()
        e0, e1 = ev(), ev()
        e0.record(s)
        with torch.cuda.stream(s):
            g.replay()
        e1.record(s)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        st = b.stats()
        rebuilt = sum(x["strategy"] for x in st) / len(st)
        nbytes = batched_step_bytes(ns, ds, grids, st, budget)
        gbs = nbytes / (ms / steps * 1e-3) / 1e9
        progress(f"batched {name}: {ms / steps:.4f} ms/step, {gbs:.0f} GB/s algorithmic")
        res[name] = {"value": total * steps / (ms / 1e3), "ms_per_step": ms / steps,
                     "last_step_rebuild_fraction": rebuilt,
                     "errors": sum(1 for x in st if x["err"] != 0),
                     "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                  "frac": gbs / HBM_PEAK_GBS, "bytes_per_step": nbytes}}
        del g
        b.close()
    if not args.batch_loops:
        return res

    def scene_lanes(d):
        """The batch's lanes per query for a scene of dimension d (its default: 4 / 8)."""
        return (4 if d == 2 else 8) if lanes == 0 else lanes
    # the same scenes, one context per scene, advanced one after another (graph-captured)
    per = min(steps, 10)
    tr_frames = [[torch.from_numpy(tr.frames[t]).cuda() for t in range(per + 2)] for tr in trajs]
    ctxs = []
    with torch.cuda.stream(s):
        for k, tr in enumerate(trajs):
            c = nnc.NNCert(ns[k], ds[k], grid_g=grids[k], stream=s.cuda_stream, lanes=scene_lanes(ds[k]))
            c.init_certificates(tr_frames[k][0])
            c.step(tr_frames[k][1], 5e-4)
            c.repair()
            ctxs.append(c)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        for t in range(2, per + 2):
            for k, c in enumerate(ctxs):
                c.step(tr_frames[k][t], 5e-4)
                c.repair()
    torch.cuda.synchronize()
    e0, e1 = ev(), ev()
    e0.record(s)
    with torch.cuda.stream(s):
        g.replay()
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    res["per_scene_loop"] = {"value": total * per / (ms / 1e3), "ms_per_step": ms / per, "steps": per,
                             "form": "one context per scene, one stream, one graph"}
    del g
    for c in ctxs:
        c.close()
    # the fairer per-scene baseline: the contexts spread over several streams that run as
    # parallel branches of one graph (as the headline runs its five scenes)
    nstreams = 8
    bstreams = [torch.cuda.Stream() for _ in range(nstreams)]
    ctxs = []
    for k, tr in enumerate(trajs):
        st_k = bstreams[k % nstreams]
        with torch.cuda.stream(st_k):
            c = nnc.NNCert(ns[k], ds[k], grid_g=grids[k], stream=st_k.cuda_stream, lanes=scene_lanes(ds[k]))
            c.init_certificates(tr_frames[k][0])
            c.step(tr_frames[k][1], 5e-4)
            c.repair()
            ctxs.append(c)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        for st_k in bstreams:
            st_k.wait_stream(s)
        for t in range(2, per + 2):
            for k, c in enumerate(ctxs):
                with torch.cuda.stream(bstreams[k % nstreams]):
                    c.step(tr_frames[k][t], 5e-4)
                    c.repair()
        for st_k in bstreams:
            s.wait_stream(st_k)
    torch.cuda.synchronize()
    e0, e1 = ev(), ev()
    e0.record(s)
    with torch.cuda.stream(s):
        g.replay()
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    res["per_scene_branches"] = {"value": total * per / (ms / 1e3), "ms_per_step": ms / per, "steps": per,
                                 "form": f"one context per scene on {nstreams} streams, parallel branches of one graph"}
    del g
    for c in ctxs:
        c.close()
    res["speedup_batched_repair_over_branches"] = res["repair"]["value"] / res["per_scene_branches"]["value"]
    res["speedup_batched_repair_over_loop"] = res["repair"]["value"] / res["per_scene_loop"]["value"]
    if "learned" in res:
        res["speedup_learned_over_loop"] = res["learned"]["value"] / res["per_scene_loop"]["value"]
    # selector error on freshly generated held-out transitions (seeds unseen in training),
    # both strategies timed inside the batched step; the learned policy's feature and
    # network cost is charged to every transition inside its band
    if params is not None and args.regret_scenes > 0:
        specs = selector.scene_specs(args.regret_scenes, seed=9500)
        data = selector.collect_batched(specs, args.regret_steps)
        X, tr_, tb_ = data["X"], data["t_repair"], data["t_rebuild"]
        lo, hi = meta.get("band", [0.0, 2.0])
        c_inf = float(meta.get("inference_wave_us_per_scene_step", 0.0))
        ch, inb = selector.band_choice(X, selector.decide(params, X), lo, hi)
        res["selector"] = {
            "transitions": int(len(X)), "labels": "timed inside the batched step (wave-microseconds)",
            "regret_learned": selector.regret(ch, tr_, tb_, np.where(inb, c_inf, 0.0)),
            "regret_learned_without_inference": selector.regret(ch, tr_, tb_),
            "fraction_in_band": float(inb.mean()),
            "regret_threshold": selector.regret((X[:, 0] >= tau).astype(np.int32), tr_, tb_),
            "regret_always_repair": selector.regret(np.zeros(len(X), np.int32), tr_, tb_),
            "regret_always_rebuild": selector.regret(np.ones(len(X), np.int32), tr_, tb_),
            "training": meta,
        }
        # the batched step on these mixed-step scenes under each policy (the selector's
        # deployment workload: step sizes over a decade)
        res["mixed_eps_batch"] = mixed_eps_batch(nnc, synth, autotune, selector, torch, params, meta, tau)
    return res


def mixed_eps_batch(nnc, synth, autotune, selector, torch, params, meta, tau, scenes=256, steps=40):
    """The selector's workload as one batch (N log-uniform in [500, 20000], both d, the
    five families, eps log-uniform in [1e-4, 5e-3]): ms per step under each policy,
    graph-captured like the 512-scene leg."""
    specs = selector.scene_specs(scenes, seed=9700)
    trajs = [synth.make_trajectory(sp["family"], sp["n"], sp["d"], steps + 1, sp["eps"], tuple(sp["seed"]))
             for sp in specs]
    ns = [t.n for t in trajs]
    ds = [t.d for t in trajs]
    frames = [torch.from_numpy(synth.concat_frame(trajs, t)).cuda() for t in range(steps + 2)]
    grids = autotune.batch_grids(frames[0], ns, ds, lanes=0, factor=1.5, cells_per_point=8)
    s = torch.cuda.Stream()
    pdev = torch.from_numpy(params).cuda()
    out = {"scenes": scenes, "points": sum(ns), "steps": steps}
    for name, pol in (("repair", 0), ("rebuild", 1), ("threshold", 2), ("learned", 3)):
        with torch.cuda.stream(s):
            b = nnc.NNCBatch(ns, ds, grids=grids, lanes=0, stream=s.cuda_stream)
            b.selector_load(pdev)
            band = meta.get("band", [0.0, 2.0])
            b.selector_band(band[0], band[1])
            b.init(frames[0])
            b.step(frames[1], pol, tau)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            for t in range(2, steps + 2):
                b.step(frames[t], pol, tau)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        with torch.cuda.stream(s):
            g.replay()
        e1.record(s)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        st = b.stats()
        out[name] = {"ms_per_step": ms / steps, "value": sum(ns) * steps / (ms / 1e3),
                     "last_step_rebuild_fraction": sum(x["strategy"] for x in st) / len(st)}
        progress(f"mixed-eps batch {name}: {ms / steps:.4f} ms/step")
        del g
        b.close()
    return out


def batched_step_bytes(ns, ds, grids, stats, budget=False):
    """Algorithmic bytes of one batched step from the last step's per-scene counts:
    ingest (new coordinates, rank, the slot record read and rewritten, cell), filter
    (key, fail flag; candidate list), queries (each query's coordinates and list entry,
    its certificate written; every slot record of the scene read once; the cell-start
    table), and for a rebuilt scene its grid build (counts, scan, scatter); with the
    per-point budget, its pass reads every key once (the expired points' further
    reads are not counted: a lower bound)."""
    tot = 0
    for n, d, G, st in zip(ns, ds, grids, stats):
        if budget:
            tot += 8 * n
        cells = G ** d
        q = n if st["strategy"] == 1 else st["n_cand"]
        tot += n * (4 * d + 4 + 16 + 16 + 4) + n * 9 + 4 * st["n_cand"]
        tot += q * (4 * d + 4 + 25) + 16 * n + 4 * (cells + 1)
        if st["strategy"] == 1:
            tot += 12 * cells + n * (8 * d + 12)
    return tot


def sweep_leg(args, nnc, synth, torch):
    """Frontier sweep: N = 2^20 uniform points in the plane; for each target candidate fraction
    f, one transition with eps = c_(ceil(fN))/4 applied to a disc (localized) or to
    the same number of random points (diffuse); both strategies timed on the same
    pending step from the same state, and forced frontiers of equal size (nearest the
    disc centre vs uniform) repaired to isolate the entropy axis."""
    n, d, G = 1 << 20, 2, 512
    p0 = synth.sweep_start(n)
    s = torch.cuda.Stream()
    P0 = torch.from_numpy(p0).cuda()
    reps = args.sweep_reps

    def ev():
        return torch.cuda.Event(enable_timing=True)

    # lanes per query: the fastest of 1, 4, 8 and 16 on repair + rebuild of a 5% diffuse transition
    lanes_table = {}
    c = None
    for L in (1, 4, 8, 16):
        with torch.cuda.stream(s):
            ctx = nnc.NNCert(n, d, grid_g=G, stream=s.cuda_stream, lanes=L)
            ctx.init_certificates(P0)
        torch.cuda.synchronize()
        if c is None:
            st = ctx.state()
            c = np.sort((st["d2"] - st["d1"]).cpu().numpy())
        P1 = torch.from_numpy(synth.sweep_motion(p0, float(c[int(0.05 * n)]) / 4.0, "diffuse")).cuda()
        with torch.cuda.stream(s):
            ctx.step(P1, -1.0)
        sn = ctx.snapshot()
        best = math.inf
        for _ in range(max(reps, 2)):
            e0, e1 = ev(), ev()
            with torch.cuda.stream(s):
                ctx.restore(sn)
                e0.record(s)
                ctx.repair()
                ctx.restore(sn)
                ctx.rebuild()
                e1.record(s)
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1))
        lanes_table[L] = best
        del sn
        ctx.close()
    lanes = min(lanes_table, key=lanes_table.get)
    with torch.cuda.stream(s):
        ctx = nnc.NNCert(n, d, grid_g=G, stream=s.cuda_stream, lanes=lanes)
        ctx.init_certificates(P0)
    torch.cuda.synchronize()
    fresh = ctx.snapshot()

    def timed(fn):
        best = math.inf
        for _ in range(reps):
            with torch.cuda.stream(s):
                ctx.restore(snap)
            e0, e1 = ev(), ev()
            e0.record(s)
            with torch.cuda.stream(s):
                fn()
            e1.record(s)
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1))
        return best

    rows = []
    # kernel-level timing of the queries at this size (HBM roofline)
    kern = {}
    for f in (0.001, 0.01, 0.05, 0.2, 0.5):
        k = max(1, int(math.ceil(f * n)))
        eps = float(c[k - 1]) / 4.0
        for mode in ("localized", "diffuse"):
            P1 = torch.from_numpy(synth.sweep_motion(p0, eps, mode)).cuda()
            with torch.cuda.stream(s):
                ctx.restore(fresh)
                ctx.profile_enable(True)
                ctx.step(P1, -1.0)
            prof_step = ctx.profile_read()
            ctx.profile_enable(False)
            snap = ctx.snapshot()
            hc = ctx.frontier_entropy(nnc.NNC_CANDIDATES)
            t_rep = timed(lambda: ctx.repair())
            t_reb = timed(lambda: ctx.rebuild())
            with torch.cuda.stream(s):
                ctx.restore(snap)
                ctx.profile_enable(True)
                ctx.repair()
            prof_rep = ctx.profile_read()
            with torch.cuda.stream(s):
                ctx.restore(snap)
                ctx.rebuild()
            prof_reb = ctx.profile_read()
            ctx.profile_enable(False)
            hf = ctx.frontier_entropy(nnc.NNC_FAILED)
            rows.append({"target_fraction": f, "mode": mode, "eps": eps, "candidates": hc["count"],
                         "candidate_fraction": hc["count"] / n, "H_candidates": hc["H"], "m_candidates": hc["m"],
                         "failures": hf["count"], "H_fail": hf["H"], "m_fail": hf["m"], "C": hf["C"],
                         "repair_ms": t_rep, "rebuild_ms": t_reb,
                         "step_kernels_us": (prof_step["ingest"][0] + prof_step["filter"][0]) * 1e3,
                         "repair_query_us": prof_rep["query"][0] * 1e3,
                         "rebuild_query_us": prof_reb["query"][0] * 1e3,
                         "rebuild_grid_us": prof_reb["grid"][0] * 1e3})
            del snap
        # forced frontiers of equal size: localized vs diffuse
        local, diffuse = synth.sweep_lists(p0, k)
        with torch.cuda.stream(s):
            ctx.restore(fresh)
            ctx.step(P0, -1.0)
        snap = ctx.snapshot()
        cnt = torch.tensor([k], dtype=torch.int32, device="cuda")
        out = {}
        for name, lst in (("localized", local), ("diffuse", diffuse)):
            L = torch.from_numpy(lst).cuda()
            out[name] = timed(lambda: ctx.repair(L, cnt))
        rows.append({"target_fraction": f, "mode": "forced", "count": k, "forced_localized_ms": out["localized"],
                     "forced_diffuse_ms": out["diffuse"]})
        del snap
    # the per-point motion budget: the candidate set now depends on where the points
    # moved (stationary points need twice the clearance of moving ones), so localized
    # and diffuse motion of the same size give different frontiers
    with torch.cuda.stream(s):
        bctx = nnc.NNCert(n, d, grid_g=G, stream=s.cuda_stream, lanes=lanes, budget=True)
        bctx.init_certificates(P0)
    torch.cuda.synchronize()
    bfresh = bctx.snapshot()
    budget_rows = []
    gq = torch.Generator(device="cuda")
    gq.manual_seed(3500)
    qidx = torch.sort(torch.randperm(n, generator=gq, device="cuda")[:4096]).values.to(torch.int32)
    for f in (0.001, 0.01, 0.05, 0.2, 0.5):
        k = max(1, int(math.ceil(f * n)))
        eps = float(c[k - 1]) / 4.0
        for mode in ("localized", "diffuse"):
            P1 = torch.from_numpy(synth.sweep_motion(p0, eps, mode)).cuda()
            with torch.cuda.stream(s):
                bctx.restore(bfresh)
                bctx.step(P1, -1.0)
            bsnap = bctx.snapshot()
            hc = bctx.frontier_entropy(nnc.NNC_CANDIDATES)
            best = math.inf
            for _ in range(reps):
                e0, e1 = ev(), ev()
                with torch.cuda.stream(s):
                    bctx.restore(bsnap)
                    e0.record(s)
                    bctx.repair()
                    e1.record(s)
                e1.synchronize()
                best = min(best, e0.elapsed_time(e1))
            hf = bctx.frontier_entropy(nnc.NNC_FAILED)
            nn_s, _, _ = nnc.allpairs_top2(P1, qidx)
            bad = int((bctx.state()["nn"][qidx.long()] != nn_s).sum())
            budget_rows.append({"target_fraction": f, "mode": mode, "eps": eps, "candidates": hc["count"],
                                "candidate_fraction": hc["count"] / n, "H_candidates": hc["H"],
                                "m_candidates": hc["m"], "failures": hf["count"], "H_fail": hf["H"],
                                "repair_ms": best, "sampled_missed": bad})
            del bsnap
    del bfresh
    bctx.close()
    # HBM roofline of the rebuild's all-point query at this size
    reb = [r for r in rows if r.get("mode") == "diffuse"]
    q_us = sum(r["rebuild_query_us"] for r in reb) / len(reb)
    C_mean = sum(r["C"] for r in reb) / len(reb)
    qbytes = n * (8 * d + 29) + 4 * (C_mean + 1)
    rep50 = [r for r in rows if r.get("mode") == "diffuse" and r["target_fraction"] == 0.5][0]
    rbytes = rep50["candidates"] * (4 * d + 4 + 25) + n * (4 * d + 4) + 4 * (rep50["C"] + 1)
    ctx.close()
    return {"n": n, "d": d, "G": G, "lanes": lanes, "lanes_table_ms": lanes_table, "rows": rows,
            "budget_rows": budget_rows,
            "roofline_rebuild_query": {"bound": "hbm", "achieved": qbytes / (q_us * 1e-6) / 1e9,
                                       "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                       "frac": qbytes / (q_us * 1e-6) / 1e9 / HBM_PEAK_GBS,
                                       "avg_launch_us": q_us, "bytes_per_launch": qbytes},
            "roofline_repair_query_f50": {"bound": "hbm",
                                          "achieved": rbytes / (rep50["repair_query_us"] * 1e-6) / 1e9,
                                          "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                          "frac": rbytes / (rep50["repair_query_us"] * 1e-6) / 1e9 / HBM_PEAK_GBS,
                                          "avg_launch_us": rep50["repair_query_us"], "bytes_per_launch": rbytes}}


def audit_leg(args, nnc, synth, torch):
    """Table 1's certificate-failure audit on the ten families: N = 16000, d = 2 and 3,
    eps in {5e-4, 2e-3, 8e-3}, 24 repaired steps each; every step checked by the
    exact all-pairs oracle.  Per family, pooled: the mean fraction of certificates
    that fail per step, the safety rule's misses (must be 0) and the fraction of
    still-valid certificates it flags, and the local predictor rho_i > 1/2's recall
    (flagged failures / failures) and false flags (flagged valid / valid)."""
    n, steps = 16000, 24
    table = {}
    for fi, fam in enumerate(synth.FAMILIES + synth.EXTRA_FAMILIES):
        acc = dict(steps=0, fail=0, valid=0, missed=0, cand_false=0, rho_hit=0, rho_false=0, frac=0.0)
        for d in (2, 3):
            for k, eps in enumerate((5e-4, 2e-3, 8e-3)):
                tr = synth.make_trajectory(fam, n, d, steps, eps, (6000 + fi, d, k))
                frames = [torch.from_numpy(f).cuda() for f in tr.frames]
                ctx = nnc.NNCert(n, d)
                ctx.init_certificates(frames[0])
                for t in range(1, steps + 1):
                    ctx.step(frames[t], -1.0)  # no declared bound: the measured eps_t drives the audit
                    ctx.rho_predict()
                    ctx.repair()
                    a = ctx.oracle_verify()
                    f = a["n_true_fail"]
                    acc["steps"] += 1
                    acc["fail"] += f
                    acc["valid"] += n - f
                    acc["frac"] += f / n
                    acc["missed"] += a["n_missed"]
                    acc["cand_false"] += a["n_false"]
                    acc["rho_hit"] += a["rho_hit"]
                    acc["rho_false"] += a["rho_flagged"] - a["rho_hit"]
                ctx.close()
        table[fam] = {"invalid": acc["frac"] / acc["steps"], "miss_safe": acc["missed"],
                      "false_safe": acc["cand_false"] / max(acc["valid"], 1),
                      "recall_rho": acc["rho_hit"] / max(acc["fail"], 1),
                      "false_rho": acc["rho_false"] / max(acc["valid"], 1), "steps": acc["steps"]}
        progress(f"audit {fam}: " + ", ".join(f"{k} {v:.3f}" for k, v in table[fam].items() if k != "steps"))
    return {"n": n, "steps_per_run": steps, "eps": [5e-4, 2e-3, 8e-3], "d": [2, 3], "families": table}


def queue_leg(args, nnc, synth, torch):
    """Candidate detection by the expiry calendar (NNC_QUEUE) against the scan of all
    keys, at low pressure (eps for about 0.1 % and 1 % of the points per step) and
    N = 2^20 to 2^24 in the plane: per step the detection kernels' time (the scan, or
    the calendar's pop plus the filing of the repaired keys) and the calendar's
    entries read, from HIP events; both runs' candidate sets are compared."""
    rows = []
    d = 2
    for e in [int(v) for v in args.queue_exps.split(",") if v]:
        n = 1 << e
        for frac in (0.001, 0.01):
            p0 = synth.device_uniform(n, d, seed=8000 + e)
            ctxs = {"scan": nnc.NNCert(n, d, lanes=16), "queue": nnc.NNCert(n, d, lanes=16, queue=True)}
            for c in ctxs.values():
                c.init_certificates(p0)
            st = ctxs["scan"].state()
            cs = (st["d2"] - st["d1"]).float()
            eps = float(torch.kthvalue(cs, max(1, int(frac * n))).values) / 4.0
            del st, cs
            frames = [p0]
            for t in range(1, 9):
                frames.append(synth.device_brownian_step(frames[-1], eps, seed=8100 + 10 * e + t))
            res = {}
            same = True
            for t in range(1, 9):
                lists = {}
                for name, c in ctxs.items():
                    if t == 3:
                        c.profile_enable(True)
                    c.step(frames[t], -1.0)
                    lists[name] = c.frontier_indices()
                    c.repair()
                same = same and torch.equal(torch.sort(lists["queue"]).values, lists["scan"])
                cand = lists["scan"].numel()
            for name, c in ctxs.items():
                prof = c.profile_read()
                ms, cnt = prof["filter"]
                res[name] = ms / 6 * 1e3          # six profiled steps
            qs = ctxs["queue"].queue_stats()
            for c in ctxs.values():
                c.close()
            row = {"n": n, "target_fraction": frac, "eps": eps, "candidates_last_step": cand,
                   "scan_detect_us_per_step": round(res["scan"], 2), "queue_detect_us_per_step": round(res["queue"], 2),
                   "queue_entries_read_per_pop": round(qs["entries_read"] / max(qs["pops"], 1), 1),
                   "queue_counters": qs, "same_candidate_sets": bool(same)}
            progress(f"queue N=2^{e} f={frac}: scan {row['scan_detect_us_per_step']} us, queue "
                     f"{row['queue_detect_us_per_step']} us, read {row['queue_entries_read_per_pop']}")
            rows.append(row)
            del frames
            torch.cuda.empty_cache()
    return {"d": d, "rows": rows}


def scaling_leg(args, nnc, synth, torch):
    """The step, repair and rebuild kernels from N = 2^16 to 2^26 (d = 2, uniform,
    Brownian steps, eps set so that about 5 % of the points are candidates): mean
    kernel times from HIP events and achieved bandwidth against 8 TB/s with the
    algorithmic bytes of each kernel; each size certified on 4096 sampled points by
    the exact all-pairs kernel."""
    rows = []
    d = 2
    for e in [int(v) for v in args.scaling_exps.split(",") if v]:
        n = 1 << e
        p0 = synth.device_uniform(n, d, seed=7000 + e)
        ctx = nnc.NNCert(n, d, lanes=args.scaling_lanes)
        G = ctx.grid_g
        ctx.init_certificates(p0)
        st = ctx.state()
        c = (st["d2"] - st["d1"]).float()
        k = max(1, int(0.05 * n))
        eps = float(torch.kthvalue(c, k).values) / 4.0
        del st, c
        frames = [p0]
        for t in range(1, 7):
            frames.append(synth.device_brownian_step(frames[-1], eps, seed=7100 + 10 * e + t))
        torch.cuda.synchronize()
        prof = {}
        nf = C = 0
        for t in range(1, 7):
            strategy = "repair" if t <= 4 else "rebuild"
            if t == 2 or t == 5:
                ctx.profile_enable(True)
            ctx.step(frames[t], -1.0)
            if t == 4:  # candidates and occupied cells of a profiled step
                ctx.profile_enable(False)
                F = ctx.frontier_entropy(nnc.NNC_CANDIDATES)
                nf, C = F["count"], F["C"]
                ctx.profile_enable(True)
            ctx.repair() if strategy == "repair" else ctx.rebuild()
            if t == 4 or t == 6:
                for name, (ms, cnt) in ctx.profile_read().items():
                    prof[(strategy, name)] = (ms / cnt * 1e3) if cnt else 0.0
                ctx.profile_enable(False)
        g = torch.Generator(device="cuda")
        g.manual_seed(7200 + e)
        qidx = torch.sort(torch.randperm(n, generator=g, device="cuda")[:4096]).values.to(torch.int32)
        nn, d1, d2 = nnc.allpairs_top2(frames[6], qidx)
        stt = ctx.state()
        ql = qidx.long()
        bad = int((stt["nn"][ql] != nn).sum()) + int((stt["d1"][ql].view(torch.int32) != d1.view(torch.int32)).sum())
        ctx.close()
        occ = n / G ** d
        nbytes = {
            "ingest": n * (12 * d + 8),
            "filter": n * 9 + 4 * nf,
            "repair_query": nf * (4 * d + 4 + 25) + min(n, 9 * occ * nf) * (4 * d + 4) + 4 * (C + 1),
            "grid": 12 * G ** d + n * (8 * d + 12),
            "rebuild_query": n * (8 * d + 29) + 4 * (C + 1),
        }
        times = {"ingest": prof[("repair", "ingest")], "filter": prof[("repair", "filter")],
                 "repair_query": prof[("repair", "query")], "grid": prof[("rebuild", "grid")],
                 "rebuild_query": prof[("rebuild", "query")]}
        # reference: a plain random-permutation scatter of the same coordinates (torch's
        # index_copy_), the pattern that moving points into slot order costs
        perm = torch.randperm(n, generator=g, device="cuda")
        src = frames[6].reshape(-1)
        dst = torch.empty_like(src)
        idx = torch.cat([perm + k * n for k in range(d)])
        dst.index_copy_(0, idx, src)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(3):
            dst.index_copy_(0, idx, src)
        e1.record()
        torch.cuda.synchronize()
        scatter_us = e0.elapsed_time(e1) * 1e3 / 3
        del perm, dst, idx
        row = {"n": n, "G": G, "eps": eps, "candidates": nf, "sampled_mismatches": bad,
               "reference_scatter_us": round(scatter_us, 2)}
        for kname, us in times.items():
            gbs = nbytes[kname] / (us * 1e-6) / 1e9 if us > 0 else 0.0
            row[kname] = {"us": round(us, 2), "bytes": int(nbytes[kname]), "GB_s": round(gbs, 1),
                          "frac": round(gbs / HBM_PEAK_GBS, 4)}
        progress(f"scaling N=2^{e}: " + ", ".join(f"{k} {v['us']} us {v['frac']:.3f}" for k, v in row.items()
                                                   if isinstance(v, dict)))
        rows.append(row)
        del frames
        torch.cuda.empty_cache()
    return {"d": d, "rows": rows}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the certificate-maintenance "
              f"path of this library runs on a single GPU.", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    import paper_2606_18314_amd as nnc
    from paper_2606_18314_amd import autotune

    nnc.load()
    W, K = args.warmup, args.steps
    T = W + K
    dev = torch.device("cuda:0")
    fams = list(synth.FAMILIES)
    t_gen = time.time()
    trajs = {f: synth.cube_16k(f, n=N, steps=T) for f in fams}
    frames = {f: torch.from_numpy(trajs[f].frames).to(dev) for f in fams}   # resident in HBM
    torch.cuda.synchronize()
    gen_s = time.time() - t_gen
    stream = torch.cuda.Stream()
    s_ptr = stream.cuda_stream

    tuning = {}
    lanes = {}
    table_path = os.path.join(ROOT, "paper_2606_18314_amd", "tuned_cube16k.json")
    if not args.grid_json and args.grid == "table":
        if os.path.exists(table_path):
            tab = json.load(open(table_path))["scenes"]
            args.grid_json = json.dumps({f: [tab[f]["G"], tab[f]["lanes"]] for f in fams})
        else:
            args.grid = "auto"
    grid_source = "table" if args.grid == "table" else ("fixed" if args.grid_json else args.grid)
    if args.grid_json:
        fixed = json.loads(args.grid_json)
        grids = {f: int(fixed[f][0]) for f in fams}
        lanes = {f: int(fixed[f][1]) for f in fams}
    elif args.grid == "auto":
        grids = {}
        for f in fams:   # tuned on the first warm-up frames, outside every timed region
            (grids[f], lanes[f]), tuning[f] = autotune.tune_grid(
                [frames[f][t] for t in range(min(T, 8) + 1)], D, EPS, steps=min(T, 8))
    else:
        grids = {f: int(args.grid) for f in fams}
        lanes = {f: 0 for f in fams}

    # one stream per scene: the five scenes are independent, so their step chains
    # may run side by side (the graph holds one branch per scene); with --branches k < 5
    # the scenes share k streams, the longest first onto the least loaded (the tuning
    # table's step times as weights)
    nbr = max(1, min(args.branches, len(fams)))
    if nbr >= len(fams):
        fstreams = {f: torch.cuda.Stream() for f in fams}
    else:
        weight = {f: 1.0 for f in fams}
        if os.path.exists(table_path):
            tabw = json.load(open(table_path))["scenes"]
            weight = {f: float(tabw[f]["ms_per_step"]) for f in fams}
        pool = [torch.cuda.Stream() for _ in range(nbr)]
        load = [0.0] * nbr
        fstreams = {}
        for f in sorted(fams, key=lambda f: -weight[f]):
            k = min(range(nbr), key=lambda j: load[j])
            fstreams[f] = pool[k]
            load[k] += weight[f]

    def make_ctxs(per_scene_streams):
        ctxs = {}
        for f in fams:
            st = fstreams[f] if per_scene_streams else stream
            with torch.cuda.stream(st):
                c = nnc.NNCert(N, D, grid_g=grids[f], stream=st.cuda_stream, lanes=lanes[f])
                c.init_certificates(frames[f][0])
            ctxs[f] = (c, st)
        torch.cuda.synchronize()
        return ctxs

    def run_steps(ctxs, t0, t1, strategy):
        for t in range(t0, t1):
            for f in fams:
                c, st = ctxs[f]
                with torch.cuda.stream(st):
                    c.step(frames[f][t], EPS)
                    if strategy == "repair":
                        c.repair()
                    else:
                        c.rebuild()

    def fork(ctxs):
        for f in fams:
            ctxs[f][1].wait_stream(stream)

    def join(ctxs):
        for f in fams:
            stream.wait_stream(ctxs[f][1])

    def ev():
        return torch.cuda.Event(enable_timing=True)

    def timed(fn):
        torch.cuda.synchronize()
        e0, e1 = ev(), ev()
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    out = {"metric": METRIC, "unit": "point-steps/s", "n_gpus": 1, "steps": K, "warmup": W,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic"}
    legs = {}
    legs_req = set(args.legs.split(","))
    pts_per_step = N * len(fams)

    # ---- repair and rebuild: graph replays (per-scene streams and one stream), eager,
    # kernel timing, certification ------------------------------------------------------
    kernel_avg = {}
    audits = {}
    end_hash = {}
    for strategy in ("repair", "rebuild"):
        if strategy not in legs_req:
            continue
        leg = {}
        for mode in ("streams", "serial"):
            ctxs = make_ctxs(mode == "streams")
            fork(ctxs)
            run_steps(ctxs, 1, W + 1, strategy)
            join(ctxs)
            torch.cuda.synchronize()
            snaps = {f: ctxs[f][0].snapshot() for f in fams}
            torch.cuda.synchronize()

            def eager():
                fork(ctxs)
                run_steps(ctxs, W + 1, T + 1, strategy)
                join(ctxs)
            eager_ms = timed(eager)
            for f in fams:
                ctxs[f][0].restore(snaps[f])
            torch.cuda.synchronize()
            # capture records the K steps without running them: afterwards the device
            # state is still that of step W while the host side has advanced to step T;
            # the replay brings the device to step T as well
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=stream):
                fork(ctxs)
                run_steps(ctxs, W + 1, T + 1, strategy)
                join(ctxs)
            torch.cuda.synchronize()

            def replay():
                with torch.cuda.stream(stream):
                    g.replay()
            # several replays of the same K steps from the same state; the median is reported.
            # The first replay follows the capture, which left the contexts' host-side step
            # bookkeeping at step T, so its end state is audited against the step-T positions;
            # a restore rewinds that bookkeeping to step W while a replay still advances the
            # device to step T, so the later replays are compared with the first by their
            # neighbour arrays (plain copies: no heavy kernel between the timed replays), and
            # the audit runs at the end on the first replay's end state, restored with its
            # bookkeeping.
            runs = []
            replays_identical = True
            for r in range(args.repeats):
                if r:
                    for f in fams:
                        ctxs[f][0].restore(snaps[f])
                    torch.cuda.synchronize()
                runs.append(timed(replay))
                if r == 0:
                    first_nn = {f: ctxs[f][0].state()["nn"] for f in fams}
                    snaps_T = {f: ctxs[f][0].snapshot() for f in fams}  # state and bookkeeping at T
                else:
                    replays_identical &= all(torch.equal(ctxs[f][0].state()["nn"], first_nn[f]) for f in fams)
            graph_ms = sorted(runs)[len(runs) // 2]
            for f in fams:
                ctxs[f][0].restore(snaps_T[f])
            torch.cuda.synchronize()
            end_audit = {f: ctxs[f][0].oracle_verify() for f in fams}
            end_hash[(strategy, mode)] = {f: end_audit[f]["nn_hash"] for f in fams}
            progress(f"{strategy} {mode}: {graph_ms / K:.4f} ms/step (median of {len(runs)})")
            leg[mode] = {"value": pts_per_step * K / (graph_ms / 1e3), "ms_per_step": graph_ms / K,
                         "replay_ms": [round(v, 4) for v in runs],
                         "eager_value": pts_per_step * K / (eager_ms / 1e3), "eager_ms_per_step": eager_ms / K,
                         "end_state_missed": sum(a["n_missed"] for a in end_audit.values()),
                         "end_state_value_mismatch": sum(a["n_value_mismatch"] for a in end_audit.values()),
                         "replays_identical": replays_identical}
            del g
            if mode == "serial":
                # kernel timing pass (eager, HIP events on the library stream)
                for f in fams:
                    ctxs[f][0].restore(snaps[f])
                    ctxs[f][0].profile_enable(True)
                run_steps(ctxs, W + 1, T + 1, strategy)
                prof = {}
                fam_q = {}
                for f in fams:
                    for name, (ms, cnt) in ctxs[f][0].profile_read().items():
                        acc = prof.setdefault(name, [0.0, 0])
                        acc[0] += ms
                        acc[1] += cnt
                        if name == "query" and cnt:
                            fam_q[f] = round(ms * 1e3 / cnt, 2)
                    ctxs[f][0].profile_enable(False)
                kernel_avg[strategy] = {k: (v[0] / v[1] if v[1] else 0.0, v[1]) for k, v in prof.items()}
                leg["kernels_avg_us"] = {k: round(v[0] * 1e3, 3) for k, v in kernel_avg[strategy].items()}
                leg["kernel_launches"] = {k: v[1] for k, v in kernel_avg[strategy].items()}
                leg["query_avg_us_per_family"] = fam_q
                # certification pass: every step audited by the exact GPU all-pairs oracle
                cert = None
                if not args.no_certify:
                    for f in fams:
                        ctxs[f][0].restore(snaps[f])
                    tot = {"steps": 0, "n_missed": 0, "n_value_mismatch": 0, "n_detect": 0, "n_true_fail": 0,
                           "H_fail_sum": 0.0, "H_cand_sum": 0.0, "C_sum": 0}
                    last_hash = {}
                    for t in range(W + 1, T + 1):
                        for f in fams:
                            c, st = ctxs[f]
                            with torch.cuda.stream(st):
                                c.step(frames[f][t], EPS)
                            hc = c.frontier_entropy(nnc.NNC_CANDIDATES)
                            with torch.cuda.stream(st):
                                c.repair() if strategy == "repair" else c.rebuild()
                            hf = c.frontier_entropy(nnc.NNC_FAILED)
                            a = c.oracle_verify()
                            tot["steps"] += 1
                            tot["n_missed"] += a["n_missed"]
                            tot["n_value_mismatch"] += a["n_value_mismatch"]
                            tot["n_detect"] += a["n_detect"]
                            tot["n_true_fail"] += a["n_true_fail"]
                            tot["H_fail_sum"] += hf["H"]
                            tot["H_cand_sum"] += hc["H"]
                            tot["C_sum"] += hf["C"]
                            last_hash[f] = a["nn_hash"]
                    cert = {"scene_steps": tot["steps"], "n_missed": tot["n_missed"],
                            "n_value_mismatch": tot["n_value_mismatch"],
                            "candidate_fraction": tot["n_detect"] / (tot["steps"] * N),
                            "failure_fraction": tot["n_true_fail"] / (tot["steps"] * N),
                            "mean_H_fail": tot["H_fail_sum"] / tot["steps"],
                            "mean_H_candidates": tot["H_cand_sum"] / tot["steps"],
                            "mean_occupied_cells": tot["C_sum"] / tot["steps"],
                            # the audited run and the timed graph replays end in the same state
                            "end_hash_equals_timed_runs": all(end_hash[(strategy, m)] == last_hash
                                                              for m in ("streams", "serial"))}
                progress(f"{strategy} certification done")
                audits[strategy] = cert
                leg["certification"] = cert
            for f in fams:
                ctxs[f][0].close()
        leg["value"] = leg["streams"]["value"]
        leg["ms_per_step"] = leg["streams"]["ms_per_step"]
        legs[strategy] = leg

    # ---- all-pairs competitor -----------------------------------------------------------
    if "allpairs" in legs_req:
        ksteps = min(K, 40)
        with torch.cuda.stream(stream):
            for t in range(1, 3):
                for f in fams:
                    nnc.allpairs_top2(frames[f][t])
        torch.cuda.synchronize()
        e0, e1 = ev(), ev()
        e0.record(stream)
        with torch.cuda.stream(stream):
            for t in range(W + 1, W + 1 + ksteps):
                for f in fams:
                    nnc.allpairs_top2(frames[f][t])
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        launch_us = ms * 1e3 / (ksteps * len(fams))
        ops = (3 * D) * N * (N - 1)           # 3d-1 distance operations + 1 comparison per pair
        dist_ops = (3 * D - 1) * N * (N - 1)
        progress(f"allpairs: {ms / ksteps:.4f} ms/step")
        legs["allpairs"] = {"value": pts_per_step * ksteps / (ms / 1e3), "ms_per_step": ms / ksteps,
                            "steps": ksteps, "pairs_per_s": N * (N - 1) * ksteps * len(fams) / (ms / 1e3),
                            "kernel_avg_us": launch_us,
                            "roofline": {"bound": "alu", "achieved": ops / (launch_us * 1e-6) / 1e12,
                                         "peak": VALU_PEAK_TOPS, "unit": "TFLOP/s",
                                         "frac": ops / (launch_us * 1e-6) / 1e12 / VALU_PEAK_TOPS,
                                         "traffic": None,
                                         # the same work against the published FP32 vector peak (packed
                                         # FMA counted as four operations), distance operations only
                                         "published_peak": FP32_PUBLISHED_TFLOPS,
                                         "frac_of_published": dist_ops / (launch_us * 1e-6) / 1e12
                                         / FP32_PUBLISHED_TFLOPS}}

    # ---- frontier-fraction sweep at N = 2^20 -----------------------------------------------
    if "sweep" in legs_req:
        legs["sweep"] = sweep_leg(args, nnc, synth, torch)
        progress("sweep done")
    if "scaling" in legs_req:
        legs["scaling"] = scaling_leg(args, nnc, synth, torch)
    if "audit" in legs_req:
        legs["audit"] = audit_leg(args, nnc, synth, torch)
    if "queue" in legs_req:
        legs["queue"] = queue_leg(args, nnc, synth, torch)

    # ---- batched scenes (512 scenes, log-uniform N, mixed d and families) ------------------
    if "batched" in legs_req:
        legs["batched"] = batched_leg(args, nnc, synth, autotune, torch)
        progress("batched done")

    # ---- headline ------------------------------------------------------------------------
    head = legs.get("repair")
    if head is not None:
        out["value"] = head["value"]
        out["ms_per_step"] = head["ms_per_step"]
        q_us, q_cnt = kernel_avg["repair"]["query"]
        q_us *= 1e3
        cand = audits["repair"]["candidate_fraction"] if audits.get("repair") else None
        occ_cells = audits["repair"]["mean_occupied_cells"] if audits.get("repair") else 0.0
        G = grids
        # algorithmic bytes of one repair query launch (per scene): each candidate reads its
        # coordinates and list entry and writes its certificate (nn, d1, d2, stamp 4 B each,
        # expiry 8 B, fail flag 1 B); every point of the visited blocks is read once
        # (coordinates + grid slot); one cell-start entry per occupied cell.
        if cand is not None:
            per_launch = cand * N * (4 * D + 4 + 25) + N * (4 * D + 4) + 4 * (occ_cells + 1)
        else:
            per_launch = None
        roof = None
        if per_launch is not None and q_us > 0:
            achieved = per_launch / (q_us * 1e-6) / 1e9
            roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS,
                    "traffic": read_traffic("query_repair_cube_16k", src_hash("grid.hip", "device_common.hpp", "kernels_common.hpp")),
                    "kernel": "k_query (repair of the candidates)", "avg_launch_us": q_us,
                    "bytes_per_launch": per_launch}
        out["roofline"] = roof
    out["config"] = {"workload": "cube_16k: N=16000 points, d=3, five motion families, eps=5e-4, "
                                 f"{K} timed steps after {W} warm-up steps; the five independent scenes "
                                 "advance on their own streams as branches of one HIP graph",
                     "families": fams, "grid_g": grids, "lanes_per_query": lanes, "grid_tuning_ms": tuning,
                     "grid_source": grid_source, "strategy": "repair",
                     "generator_seconds": round(gen_s, 2)}
    out["strategies"] = legs

    if "repair" in legs and audits.get("repair"):
        a = audits["repair"]
        out["certified"] = (a["n_missed"] == 0 and a["n_value_mismatch"] == 0 and a["end_hash_equals_timed_runs"]
                            and all(legs["repair"][m]["end_state_missed"] == 0
                                    and legs["repair"][m]["replays_identical"] for m in ("streams", "serial")))

    # ---- counter calibration copy ----------------------------------------------------------
    if args.copy_mib:
        nbytes = args.copy_mib * 2 ** 20
        a = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = nbytes

    # ---- CPU oracle baseline -------------------------------------------------------------
    if not args.no_cpu_baseline:
        from oracle import model

        def oracle_run(seconds):
            done, spent, last = 0, 0.0, 0
            scenes = {}
            for f in fams:
                sc = model.OracleScene(d=D, n=N, G=grids[f])
                sc.init_certificates(trajs[f].frames[0])
                scenes[f] = sc
            t = 1
            while spent < seconds and t <= T:
                for f in fams:     # the same step of every family, round robin
                    t0 = time.perf_counter()
                    scenes[f].step(trajs[f].frames[t])
                    scenes[f].repair()
                    spent += time.perf_counter() - t0
                    done += 1
                last = t
                t += 1
            return done, spent, last

        all_cores = model.threads()
        done, spent, last = oracle_run(args.cpu_seconds)
        progress(f"cpu baseline ({all_cores} threads): {done} scene-steps in {spent:.1f} s")
        model.set_threads(1)
        done1, spent1, last1 = oracle_run(args.cpu_seconds / 3)
        model.set_threads(all_cores)
        progress(f"cpu baseline (1 thread): {done1} scene-steps in {spent1:.1f} s")
        out["cpu_baseline"] = {"value": done * N / spent, "unit": "point-steps/s", "cores": all_cores,
                               "kind": "oracle", "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
                               "single_thread_value": done1 * N / spent1,
                               "sample": f"oracle step + repair (brute-force certificates of the candidates) of the "
                                         f"first {last} steps of each of the five N=16000 five-family scenes, "
                                         f"{spent:.1f} s of CPU time on {all_cores} threads; single thread: first "
                                         f"{last1} steps, {spent1:.1f} s"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
