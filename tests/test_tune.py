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


def test_candidates():
    c = T.candidates(300)
    assert all(p.block <= 1024 for p in c)
    assert {p.block for p in c} == {256, 512}  # 1024 lanes for 300 nodes is skipped
    assert {p.placement for p in c} == {dr.DR_PLACE_LDS, dr.DR_PLACE_GLOBAL}
    assert {p.block for p in T.candidates(20000)} == {256, 512, 1024}
    # global placement with 256 lanes: chunks of 1 only
    assert {p.chunk for p in c if p.block == 256 and p.placement == dr.DR_PLACE_GLOBAL} == {1}


class FakeTimer:
    """Stands in for the device: a launch costs the sum of the buckets' costs
    (they share the device); 512 lanes, chunks of 2, LDS placement are
    cheapest; one shape is 'broken' and changes the pass counts."""

    def __init__(self, batch, precision):
        self.sizes = np.array([n.n_nodes for n in batch.nets])
        self.calls = 0
        self.closed = False

    def __call__(self, plans, passes):
        self.calls += 1
        cost, iters = 0.0, np.full(len(self.sizes), 100)
        if not plans:  # the library's default split
            return 1.3 * 1.5 * float(self.sizes.sum()) * passes, iters
        lo = 1
        for p in plans:
            n = int(self.sizes[(self.sizes >= lo) & (self.sizes <= p["n_hi"])].sum())
            if p["placement"] == dr.DR_PLACE_LDS and p["block"] and p["block"] * 8 < n / 4:
                return None  # rejected, as the library would
            if p["block"] == 1024 and p["chunk"] == 4:
                iters = iters + 1  # a broken shape
            f = (1.0 if p["block"] == 512 else 1.5) * (1.0 if p["chunk"] == 2 else 1.2) * \
                (1.0 if p["placement"] == dr.DR_PLACE_LDS else 1.3)
            cost += f * n
            lo = p["n_hi"] + 1
        return cost * passes, iters

    def close(self):
        self.closed = True


def test_tuner_whole_batch_greedy_and_cache(tmp_path):
    batch = I.small_batch(12, 40, 700, 0.01, seed=4)
    made = []

    def factory(b, prec):
        t = FakeTimer(b, prec)
        made.append(t)
        return t

    path = tmp_path / "tune.json"
    tu = T.Tuner(edges=(256, 512), passes=100, cache_path=str(path), timer_factory=factory,
                 key=lambda prec: f"fake|prec{prec}")
    plans = tu.tune(batch)
    sizes = np.array([n.n_nodes for n in batch.nets])
    assert [p["n_hi"] for p in plans] == [b[1] for b in T.buckets(sizes, (256, 512))]
    assert made[0].closed
    # the bucket that sets the launch time gets the cheapest valid shape; the
    # broken shape (1024 lanes, chunks of 4) is never chosen
    big = plans[-1]
    assert (big["block"], big["chunk"], big["placement"]) == (512, 2, dr.DR_PLACE_LDS)
    assert not any(p["block"] == 1024 and p["chunk"] == 4 for p in plans)
    n_calls = made[0].calls
    # a second tuner reads the cache file and times nothing
    tu2 = T.Tuner(edges=(256, 512), passes=100, cache_path=str(path), timer_factory=factory,
                  key=lambda prec: f"fake|prec{prec}")
    assert tu2.tune(batch) == plans
    assert len(made) == 1 and made[0].calls == n_calls
    assert all(k.startswith("fake|prec0|K100/1000|") for k in json.loads(path.read_text()))
    # another precision is another key
    tu2.tune(batch, precision=dr.DR_FP32)
    assert len(made) == 2
