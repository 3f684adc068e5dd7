"""GPU: the transition dataset (Section 6's layout) against the CPU oracle.

Every descriptor and audit count of every row equals what the oracle computes
for the same transition (entropy and gyration within 1e-12 relative); the label
is the fastest measured strategy; JSONL and Parquet round-trip the rows."""
import json

import numpy as np
import pytest

import synth
from oracle import model

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dataset():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_18314_amd import binding, dataset
    binding.load()
    return dataset


@pytest.mark.parametrize("spec", [
    {"family": "adversarial_crossing", "n": 3000, "d": 3, "eps": 2e-3, "seed": [6100, 0]},
    {"family": "clustered_drift", "n": 5000, "d": 2, "eps": 1e-3, "seed": [6100, 1]},
    {"family": "split_merge", "n": 2500, "d": 3, "eps": 4e-3, "seed": [6100, 2]},
])
def test_rows_match_the_oracle(dataset, spec, tmp_path):
    from paper_2606_18314_amd import autotune
    steps = 5
    rows = dataset.scene_transitions(spec, steps, reps=2)
    assert len(rows) == steps
    tr = synth.make_trajectory(spec["family"], spec["n"], spec["d"], steps, spec["eps"], tuple(spec["seed"]))
    G = autotune.default_grid(spec["n"], spec["d"])
    sc = model.OracleScene(d=spec["d"], n=spec["n"], G=G)
    sc.init_certificates(tr.frames[0])
    for t, row in enumerate(rows, start=1):
        assert set(dataset.FIELDS) <= set(row)
        res = sc.step(tr.frames[t])
        flags = sc.rho_flags()
        sc.repair()
        H, m, C, F = sc.frontier_entropy(model.FAILED)
        g, _ = model.gyration(tr.frames[t], sc.fail)
        assert row["frame"] == t and row["eps_t"] == float(res.eps)
        assert row["n_detect_safe"] == res.candidates.size
        assert row["n_fail"] == F == int(sc.fail.sum())
        assert row["n_missed_safe"] == 0
        assert row["n_false_safe"] == res.candidates.size - F
        assert row["n_flag_rho"] == int(flags.sum()) and row["n_hit_rho"] == int((flags & sc.fail).sum())
        assert (row["frontier_cells"], row["occupied_cells"]) == (m, C)
        assert row["clearance_pressure"] == F / spec["n"]
        assert row["compactness"] == (F / m if m else 0.0)
        assert abs(row["frontier_entropy"] - H) <= 1e-12 * max(1.0, abs(H))
        assert abs(row["gyration"] - g) <= 1e-12 * max(1.0, g)
        times = {k: row[f"{k}_s"] for k in dataset.STRATEGIES}
        assert all(v > 0 for v in times.values())
        assert row["best_strategy"] == min(times, key=times.get)
        assert row["speedup_over_gpu_full"] >= 1.0 and row["t_m4_local_s"] is None
    path = tmp_path / "rows.jsonl"
    dataset.write_jsonl(rows, str(path))
    back = [json.loads(line) for line in open(path)]
    assert [list(r) for r in back] == [list(dataset.FIELDS)] * steps
    assert back[2]["gyration"] == rows[2]["gyration"]
    if dataset.write_parquet(rows, str(tmp_path / "rows.parquet")):
        import pyarrow.parquet as pq
        tab = pq.read_table(str(tmp_path / "rows.parquet"))
        assert tab.num_rows == steps and tab.column_names == list(dataset.FIELDS)


def test_gyration_of_candidates_and_failures(dataset):
    """nnc_frontier_gyration of the candidate list and of the failed set against the
    oracle, on a step with both sets large."""
    from paper_2606_18314_amd import binding
    tr = synth.make_trajectory("uniform_brownian", 20000, 3, 2, 2e-3, 6200)
    ctx = binding.NNCert(tr.n, 3, grid_g=20)
    sc = model.OracleScene(d=3, n=tr.n, G=20)
    ctx.init_certificates(torch.from_numpy(tr.frames[0]).cuda())
    sc.init_certificates(tr.frames[0])
    for t in (1, 2):
        ctx.step(torch.from_numpy(tr.frames[t]).cuda())
        res = sc.step(tr.frames[t])
        g, c = ctx.frontier_gyration(binding.NNC_CANDIDATES)
        wg, wc = model.gyration(tr.frames[t], res.candidates)
        assert abs(g - wg) <= 1e-12 * wg and np.allclose(c, wc, rtol=1e-12, atol=1e-15)
        ctx.repair()
        sc.repair()
        g, c = ctx.frontier_gyration(binding.NNC_FAILED)
        wg, wc = model.gyration(tr.frames[t], sc.fail)
        assert sc.fail.sum() > 10
        assert abs(g - wg) <= 1e-12 * wg and np.allclose(c, wc, rtol=1e-12, atol=1e-15)
    ctx.close()
