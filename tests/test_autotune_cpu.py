"""Host logic of the launch-schedule autotuner: the cache keys of the
benchmark workloads are stable functions of their shapes, the committed cache
holds a valid entry for each, and the library validates a schedule before any
device work (argument errors only; no GPU needed)."""
import json
import os

from paper_2604_07644_amd import autotune, workloads as W


def test_batch_key_depends_on_shapes_only():
    a = W.uneven_batch(count=16)
    b = W.uneven_batch(count=16)
    assert autotune.batch_key(a) == autotune.batch_key(b)
    c = W.uneven_batch(count=16, first_instance=1000)
    assert autotune.batch_key(c) != autotune.batch_key(a)        # other horizons and shapes
    assert autotune.batch_key(a).startswith("batch:16:")


def test_committed_cache_covers_the_benchmark_workloads():
    with open(autotune.CACHE) as f:
        cache = json.load(f)
    entries = cache["entries"]
    key = autotune.batch_key(W.uneven_batch(count=512))
    e = entries[key]
    assert e["kind"] == "batch"
    assert 1 <= e["gang"] <= 32 and e["park_share"] > 0
    assert all(c["ok"] for c in e["candidates"] if c["gang"] == e["gang"] and c["park_share"] == e["park_share"])
    # the winner is the best valid candidate by the score it reports
    best = min((c for c in e["candidates"] if c["ok"]), key=lambda c: c["score"])
    assert (best["gang"], best["park_share"]) == (e["gang"], e["park_share"])
    from paper_2604_07644_amd import gsls
    for wl in ("quadruped", "humanoid"):
        p = {"quadruped": W.quadruped_qp, "humanoid": W.humanoid_qp}[wl](0)
        q = entries[autotune.qp_key(p, gsls.MIXED)]
        assert q["kind"] == "qp" and q["chunks_iter"] >= 0 and q["chunks_epoch"] >= 0


def test_lookup_of_unknown_key_is_none(tmp_path):
    path = os.path.join(tmp_path, "t.json")
    assert autotune.lookup("batch:1:0", path) is None
    with open(path, "w") as f:
        json.dump({"version": 1, "entries": {"k": {"kind": "batch", "gang": 8, "park_share": 1.0}}}, f)
    assert autotune.lookup("k", path)["gang"] == 8
