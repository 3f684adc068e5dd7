"""Autotuner for the grid resolution (cells per axis) of a scene.

The uniform grid of Section 2 is sized for a small constant mean occupancy; for
clustered or thin (ring) point sets the occupancy of the occupied cells is far
from the mean over the box, so the resolution is chosen from the data:

* ``pick_grid``  the smallest G whose occupied cells hold at most ``target``
                 points on average (C from the library's occupancy count);
* ``tune_grid``  times a few maintenance steps at each candidate G and number of
                 lanes per query with HIP events and keeps the fastest.

Both run the library's kernels only; results never depend on G (every
certificate is exact at any resolution), only the time does.
"""
from __future__ import annotations

import math

import torch

from . import binding

MAX_CELLS = 1 << 22


def default_grid(n: int, d: int) -> int:
    if n <= 0:
        return 1
    w = 2.0 / math.sqrt(n) if d == 2 else (4.0 / n) ** (1.0 / 3.0)
    return max(1, int(math.floor(1.0 / w)))


def candidates(n: int, d: int):
    g0 = default_grid(n, d)
    out = []
    for f in (0.75, 1.0, 1.25, 1.5, 2.0, 2.5, 3.0, 4.0, 6.0, 8.0, 12.0):
        g = max(1, int(round(g0 * f)))
        if g ** d <= MAX_CELLS and g not in out:
            out.append(g)
    return out


def occupied_cells(pos: torch.Tensor, d: int, G: int) -> int:
    n = pos.shape[1]
    ctx = binding.NNCert(n, d, grid_g=G)
    ctx.init_certificates(pos)
    c = ctx.frontier_entropy(binding.NNC_CANDIDATES)["C"]
    ctx.close()
    return int(c)


def pick_grid(pos: torch.Tensor, d: int, target: float = 3.0) -> int:
    """Smallest candidate G with mean occupancy of occupied cells <= target."""
    n = pos.shape[1]
    best = None
    for G in candidates(n, d):
        C = occupied_cells(pos, d, G)
        best = G
        if C > 0 and n / C <= target:
            break
    return best


def tune_grid(frames, d: int, eps: float, steps: int = 6, grids=None, lanes=(1, 8, 16, 32, 64),
              stream=None) -> tuple[tuple[int, int], dict]:
    """Fastest (G, lanes per query) over a short run of step + repair on frames[0..steps];
    returns ((G, L), {"G/L": ms per step})."""
    n = frames[0].shape[1]
    grids = grids or candidates(n, d)
    s = stream or torch.cuda.Stream()
    times = {}
    for G, L in [(g, l) for g in grids for l in lanes]:
        with torch.cuda.stream(s):
            ctx = binding.NNCert(n, d, grid_g=G, stream=s.cuda_stream, lanes=L)
            ctx.init_certificates(frames[0])
            ctx.step(frames[1], eps)
            ctx.repair()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s)
        with torch.cuda.stream(s):
            for t in range(2, steps + 1):
                ctx.step(frames[t], eps)
                ctx.repair()
        e1.record(s)
        torch.cuda.synchronize()
        times[(G, L)] = e0.elapsed_time(e1) / max(1, steps - 1)
        ctx.close()
    best = min(times, key=times.get)
    return best, {f"{g}/{l}": round(v, 5) for (g, l), v in times.items()}


def batch_grids(frame0: torch.Tensor, ns, ds, target: float = 4.0, lanes: int = 16, factor: float = 1.0,
                cells_per_point: int = 8):
    """Per-scene cells per axis for a batch: start from the occupancy rule, read each
    scene's occupied-cell count C from the library, and refine G so that the occupied
    cells hold about ``target`` points (capped at 8x the rule and 2^22 cells)."""
    b = binding.NNCBatch(ns, ds, lanes=lanes, features=True)
    b.init(frame0)
    b.step(frame0, 0)            # a zero-motion step fills the per-scene statistics
    st = b.stats()
    b.close()
    grids = []
    for s, (n, d) in enumerate(zip(ns, ds)):
        g0 = default_grid(int(n), int(d))
        C = max(1, st[s]["C"])
        occ = n / C
        scale = min(8.0, max(1.0, (occ / target) ** (1.0 / d)))
        g = max(1, int(round(g0 * scale * factor)))
        # at most cells_per_point cells per point: a scene's grid is built by one workgroup
        while g > 1 and (g ** d > MAX_CELLS or g ** d > cells_per_point * max(int(n), 1)):
            g -= 1
        grids.append(g)
    return grids


def tune_batch(frames, ns, ds, eps_steps: int = 4, factors=(1.25, 1.5, 2.0), caps=(8, 16), lanes=(0, 8, 16),
               policy: int = 0, stream=None):
    """Fastest (grid factor, cells-per-point cap, lanes) for a batch over a few steps;
    returns (grids, lanes, table)."""
    s = stream or torch.cuda.Stream()
    table = {}
    best = None
    for L in lanes:
        for cap in caps:
            for f in factors:
                grids = batch_grids(frames[0], ns, ds, lanes=L, factor=f, cells_per_point=cap)
                with torch.cuda.stream(s):
                    b = binding.NNCBatch(ns, ds, grids=grids, lanes=L, stream=s.cuda_stream)
                    b.init(frames[0])
                    b.step(frames[1], policy)
                torch.cuda.synchronize()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(s)
                with torch.cuda.stream(s):
                    for t in range(2, eps_steps + 2):
                        b.step(frames[t], policy)
                e1.record(s)
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / eps_steps
                b.close()
                table[f"{f}/{cap}/{L}"] = round(ms, 4)
                if best is None or ms < best[0]:
                    best = (ms, grids, L)
    return best[1], best[2], table


def tune_table(frames_by_scene: dict, d: int, eps: float, steps: int = 30, rounds: int = 3) -> dict:
    """(G, lanes) per scene: the smallest median step time over ``rounds`` runs of
    ``tune_grid`` on the scene's first ``steps`` transitions."""
    out = {}
    for name, frames in frames_by_scene.items():
        runs = [tune_grid(frames, d, eps, steps=steps)[1] for _ in range(rounds)]
        med = {k: sorted(r[k] for r in runs)[len(runs) // 2] for k in runs[0]}
        best = min(med, key=med.get)
        g, lanes = (int(v) for v in best.split("/"))
        out[name] = {"G": g, "lanes": lanes, "ms_per_step": med[best], "median_ms": med}
    return out


def main():
    """Tune the five-family N = 16000, d = 3 scenes and write the table bench.py uses."""
    import argparse
    import json
    import os
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import synth
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--rounds", type=int, default=3)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_cube16k.json"))
    args = ap.parse_args()
    binding.load()
    frames = {}
    for f in synth.FAMILIES:
        tr = synth.cube_16k(f, steps=args.steps + 1)
        fr = torch.from_numpy(tr.frames).cuda()
        frames[f] = [fr[t] for t in range(args.steps + 1)]
    table = tune_table(frames, 3, 5e-4, steps=args.steps, rounds=args.rounds)
    meta = {"device": torch.cuda.get_device_name(0), "steps": args.steps, "rounds": args.rounds,
            "workload": "cube_16k: N = 16000, d = 3, eps = 5e-4, the five families"}
    with open(args.out, "w") as fh:
        json.dump({"meta": meta, "scenes": table}, fh, indent=1)
    print(json.dumps({k: (v["G"], v["lanes"], v["ms_per_step"]) for k, v in table.items()}))


if __name__ == "__main__":
    main()
