"""Transition dataset in the layout of the paper's released data (Section 6).

Each row is one transition of one seeded synthetic scene, advanced by the
library (the repair strategy carries the state forward), with

* motion parameters: family, eps (the generator's step bound), seed, n, d, frame;
* frontier descriptors of the failed set F_t (Definition 2):
  clearance_pressure = |F_t|/N, frontier_entropy = H(F_t), frontier_cells = m
  (occupied cells F_t meets), occupied_cells = C, gyration (radius of gyration of
  F_t at the new positions) and compactness = |F_t| / m (failures per touched
  cell) -- the paper names the last two without defining them; these are the
  readings used here;
* the certificate-failure audit: eps_t, n_detect_safe (candidates of the safety
  rule), n_missed_safe, n_false_safe (candidates that did not fail), n_fail (true
  failures), n_flag_rho and n_hit_rho (the local predictor's flagged points and
  flagged failures);
* per-strategy times on this GPU, each the fastest of ``reps`` runs from the same
  restored state: gpu_grid_repair_s (grid repair of the candidates), gpu_frontier_s
  (exact brute force over the candidates), gpu_grid_s (O(N) grid rebuild),
  gpu_full_s (exact brute force over all points); the host strategies of the
  paper's second machine are not measured (t_m4_local_s and t_m4_hybrid_s are
  null) and no host-device transfer happens inside a step (transfer_s = 0);
* best_strategy (the fastest of the four, Section 3's label) and its speedups
  over the full brute force and over the grid rebuild.

Every value comes from the library's kernels; this module only sequences the
calls and writes JSONL (and Parquet when pyarrow is present).
"""
from __future__ import annotations

import json
import math

import torch

from . import binding

STRATEGIES = ("gpu_grid_repair", "gpu_frontier", "gpu_grid", "gpu_full")

FIELDS = ("family", "eps", "seed", "n", "d", "frame",
          "clearance_pressure", "frontier_entropy", "compactness", "gyration", "frontier_cells", "occupied_cells",
          "eps_t", "n_detect_safe", "n_missed_safe", "n_false_safe", "n_fail", "n_flag_rho", "n_hit_rho",
          "t_m4_local_s", "t_m4_hybrid_s", "gpu_grid_repair_s", "gpu_frontier_s", "gpu_grid_s", "gpu_full_s",
          "transfer_s", "best_strategy", "speedup_over_gpu_full", "speedup_over_gpu_grid")


def scene_transitions(spec: dict, steps: int, reps: int = 3, lanes: int = 16, grid_g: int = 0):
    """Rows of every transition of one scene (spec: family, n, d, eps, seed)."""
    import synth
    tr = synth.make_trajectory(spec["family"], spec["n"], spec["d"], steps, spec["eps"], tuple(spec["seed"]))
    frames = torch.from_numpy(tr.frames).cuda()
    s = torch.cuda.Stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    rows = []
    with torch.cuda.stream(s):
        ctx = binding.NNCert(tr.n, tr.d, grid_g=grid_g, stream=s.cuda_stream, lanes=lanes)
        ctx.init_certificates(frames[0])
    snap = None
    for t in range(1, steps + 1):
        with torch.cuda.stream(s):
            ctx.step(frames[t], spec["eps"])
        cand = ctx.frontier_entropy(binding.NNC_CANDIDATES)
        with torch.cuda.stream(s):
            snap = ctx.snapshot(into=snap) if snap is not None else ctx.snapshot()
        qidx = ctx.frontier_indices()
        times = {k: math.inf for k in STRATEGIES}
        for _ in range(reps):
            for name in STRATEGIES:
                with torch.cuda.stream(s):
                    if name in ("gpu_grid_repair", "gpu_grid"):
                        ctx.restore(snap)
                    ev[0].record(s)
                    if name == "gpu_grid_repair":
                        ctx.repair()
                    elif name == "gpu_grid":
                        ctx.rebuild()
                    elif name == "gpu_frontier":
                        if qidx.numel():
                            binding.allpairs_top2(frames[t], qidx)
                    else:
                        binding.allpairs_top2(frames[t])
                    ev[1].record(s)
                ev[1].synchronize()
                times[name] = min(times[name], ev[0].elapsed_time(ev[1]) / 1e3)
        with torch.cuda.stream(s):
            ctx.restore(snap)
            ctx.rho_predict()        # the predictor's flags are not part of a snapshot
            ctx.repair()
        audit = ctx.oracle_verify()
        ent = ctx.frontier_entropy(binding.NNC_FAILED)
        gyr, _ = ctx.frontier_gyration(binding.NNC_FAILED)
        best = min(STRATEGIES, key=lambda k: times[k])
        F, m = ent["count"], ent["m"]
        rows.append({
            "family": spec["family"], "eps": spec["eps"], "seed": list(spec["seed"]), "n": tr.n, "d": tr.d,
            "frame": t,
            "clearance_pressure": F / tr.n if tr.n else 0.0, "frontier_entropy": ent["H"],
            "compactness": F / m if m else 0.0, "gyration": gyr, "frontier_cells": m, "occupied_cells": ent["C"],
            "eps_t": cand["eps"], "n_detect_safe": cand["count"], "n_missed_safe": audit["n_missed"],
            "n_false_safe": audit["n_false"], "n_fail": audit["n_true_fail"],
            "n_flag_rho": audit["rho_flagged"], "n_hit_rho": audit["rho_hit"],
            "t_m4_local_s": None, "t_m4_hybrid_s": None,
            **{f"{k}_s": times[k] for k in STRATEGIES},
            "transfer_s": 0.0, "best_strategy": best,
            "speedup_over_gpu_full": times["gpu_full"] / times[best],
            "speedup_over_gpu_grid": times["gpu_grid"] / times[best],
        })
    ctx.close()
    return rows


def write_jsonl(rows, path: str) -> None:
    with open(path, "w") as f:
        for r in rows:
            f.write(json.dumps({k: r[k] for k in FIELDS}) + "\n")


def write_parquet(rows, path: str) -> bool:
    """Parquet copy of the rows (False when pyarrow is not importable)."""
    try:
        import pyarrow as pa
        import pyarrow.parquet as pq
    except ImportError:
        return False
    cols = {k: [r[k] for r in rows] for k in FIELDS}
    cols["seed"] = [json.dumps(v) for v in cols["seed"]]
    pq.write_table(pa.table(cols), path)
    return True


def main():
    import argparse
    from . import selector
    ap = argparse.ArgumentParser(description="write labelled transitions in the released dataset's layout")
    ap.add_argument("--scenes", type=int, default=20)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--seed", type=int, default=6000)
    ap.add_argument("--out", default="transitions.jsonl")
    ap.add_argument("--parquet", default="")
    args = ap.parse_args()
    rows = []
    for spec in selector.scene_specs(args.scenes, seed=args.seed):
        rows += scene_transitions(spec, args.steps)
    write_jsonl(rows, args.out)
    if args.parquet:
        write_parquet(rows, args.parquet)
    best = {k: sum(r["best_strategy"] == k for r in rows) for k in STRATEGIES}
    print(json.dumps({"rows": len(rows), "best_strategy_counts": best}))


if __name__ == "__main__":
    main()
