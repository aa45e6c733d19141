"""CPU tests of the autotuner's keying, candidates and cache (no GPU: a
cached key returns before any device work)."""
import json

import pytest


def test_candidates_are_valid_parameter_sets(hqr_lib):
    import paper_1110_1553_amd as h
    from paper_1110_1553_amd import tune

    cands = tune.candidates()
    assert len(cands) == len(tune.TILES) * len(tune.TREES)
    assert len({json.dumps(c, sort_keys=True) for c in cands}) == len(cands)
    for c in cands:
        p = h.make_params(**c)
        mt = -(-5000 // c["nb"])
        nt = -(-700 // c["nb"])
        st = h.dag_stats(mt, nt, p)
        # every candidate expands to the same total weight (Section II): it changes speed only
        assert st["weight"] == 6 * mt * nt * nt - 2 * nt ** 3


def test_keys_are_shape_buckets_independent_of_order():
    from paper_1110_1553_amd import tune

    k = tune.Autotuner.batch_key
    assert k([(1000, 300), (500, 40)], [1, 1]) == k([(500, 40), (1000, 300)], [1, 1])
    # shapes inside one 64 x 64 bucket share a key; the next bucket does not
    assert k([(1000, 300)], [1]) == k([(961, 257)], [1])
    assert k([(1000, 300)], [1]) != k([(1025, 300)], [1])
    # the number of right-hand sides is part of the key
    assert k([(1000, 300)], [1]) != k([(1000, 300)], [2])


def test_cache_persists_and_answers_without_the_device(tmp_path):
    from paper_1110_1553_amd import tune

    path = str(tmp_path / "tune.json")
    t = tune.Autotuner(path=path)
    shapes, nrhs = [(2000, 300), (800, 64)], [1, 1]
    key = t.batch_key(shapes, nrhs)
    t.cache[key] = {"params": {"nb": 128, "a": 4, "low": "greedy", "high": "greedy"}, "times": {"x": 1.0}}
    t.cache["factor:%dx%d" % tune._bucket(4000, 500)] = {"params": {"nb": 256, "a": 1, "low": "greedy"},
                                                          "times": {"y": 2.0}}
    t._save()
    t2 = tune.Autotuner(path=path)
    # a cached key is answered before any GPU work ("cpu" would fail on the first device call)
    params, times = t2.tune_batch(list(reversed(shapes)), list(reversed(nrhs)), device="cpu")
    assert params == {"nb": 128, "a": 4, "low": "greedy", "high": "greedy"} and times == {"x": 1.0}
    params, _ = t2.tune_factor(3990, 470, device="cpu")
    assert params["nb"] == 256


def test_uncached_key_needs_the_device(tmp_path):
    import torch

    from paper_1110_1553_amd import tune

    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    t = tune.Autotuner(path=str(tmp_path / "t.json"))
    with pytest.raises(Exception):
        t.tune_factor(512, 256, device="cpu", cands=[dict(nb=64, a=1, low="greedy")])
