"""Host logic of the launch-shape autotuner (no GPU: a fake timer stands in
for the device)."""
import json

import numpy as np

from paper_2305_07030_amd import dr
from paper_2305_07030_amd import inputs as I
from paper_2305_07030_amd import tune as T


def test_buckets_cover_every_size_once():
    rng = np.random.default_rng(0)
    sizes = np.exp(rng.uniform(np.log(200), np.log(33000), 500)).round().astype(int)
    bs = T.buckets(sizes)
    seen = np.concatenate([idx for _, _, idx in bs])
    assert sorted(seen.tolist()) == list(range(len(sizes)))
    lo_prev = 0
    for lo, hi, idx in bs:
        assert lo > lo_prev and lo <= hi
        assert ((sizes[idx] >= lo) & (sizes[idx] <= hi)).all()
        lo_prev = hi
    assert bs[-1][1] == sizes.max()
    # the bounds are contiguous (empty buckets fold into the next one's range)
    assert all(bs[k + 1][0] > bs[k][1] for k in range(len(bs) - 1))


def test_sample_keeps_largest_and_spreads():
    sizes = np.arange(1000, 2000)
    idx = np.arange(1000)
    s = T.sample(sizes, idx, 16)
    assert len(s) == 16 and sizes[s].max() == 1999 and sizes[s].min() == 1000
    assert (np.diff(sizes[s]) > 0).all()
    assert np.array_equal(T.sample(sizes, idx[:5], 16), idx[:5])


def test_candidates():
    c = T.candidates(300)
    assert all(p.block <= 1024 for p in c)
    assert {p.block for p in c} == {256, 512}  # 1024 lanes for 300 nodes is skipped
    assert {p.placement for p in c} == {dr.DR_PLACE_LDS, dr.DR_PLACE_GLOBAL}
    assert {p.block for p in T.candidates(20000)} == {256, 512, 1024}


def test_tuner_picks_fastest_and_caches(tmp_path):
    batch = I.small_batch(12, 40, 700, 0.01, seed=4)
    calls = []

    def fake_timer(sub, plan, *, passes, precision, reps):
        calls.append((len(sub), plan))
        n = max(x.n_nodes for x in sub.nets)
        if plan.placement == dr.DR_PLACE_LDS and plan.block * 8 < n:
            return None  # rejected, as the library would
        # prefer 512 lanes and chunks of 2 in LDS
        return 1.0 + (plan.block != 512) + 0.5 * (plan.chunk != 2) + (plan.placement != dr.DR_PLACE_LDS)

    path = tmp_path / "tune.json"
    tu = T.Tuner(edges=(256, 512), passes=100, sample_size=4, cache_path=str(path),
                 timer=fake_timer, key=lambda prec: f"fake|prec{prec}")
    plans = tu.tune(batch)
    sizes = np.array([n.n_nodes for n in batch.nets])
    assert [p["n_hi"] for p in plans] == [b[1] for b in T.buckets(sizes, (256, 512))]
    for p, (lo, hi, idx) in zip(plans, T.buckets(sizes, (256, 512))):
        blk = 512 if any(c.block == 512 for c in T.candidates(int(sizes[idx].max()))) else 256
        assert (p["block"], p["chunk"], p["placement"]) == (blk, 2, dr.DR_PLACE_LDS)
    assert any(p["block"] == 512 for p in plans)
    assert all(n <= 4 for n, _ in calls)
    n_calls = len(calls)
    # second tuner reads the cache file and times nothing
    tu2 = T.Tuner(edges=(256, 512), passes=100, sample_size=4, cache_path=str(path),
                  timer=fake_timer, key=lambda prec: f"fake|prec{prec}")
    assert [{k: p[k] for k in ("n_hi", "block", "chunk", "placement")} for p in tu2.tune(batch)] == \
        [{k: p[k] for k in ("n_hi", "block", "chunk", "placement")} for p in plans]
    assert len(calls) == n_calls
    assert all(k.startswith("fake|prec0|") for k in json.loads(path.read_text()))
    # another precision is another key
    tu2.tune(batch, precision=dr.DR_FP32)
    assert len(calls) > n_calls
