"""The seeded workload recipes (CPU): sizes and ranges the documentation
states, and determinism, so a change of a recipe is caught."""
import numpy as np

from paper_2411_03040_amd import synth


def test_batch_recipe():
    spec = synth.batch_spec()
    assert len(spec) == 256
    n = np.array([d["npoints"] for d in spec])
    lev = np.array([d["nlev"] for d in spec])
    rays = np.array([12 if d["nside"] == 1 else 48 for d in spec])
    assert n.sum() == 5_910_428
    assert 1000 <= n.min() and n.max() <= 100_000
    assert lev.min() >= 2 and lev.max() <= 20
    assert set(rays) == {12, 48}
    upd = (n * rays * (lev - 1) * 31).sum()
    assert upd == 56_083_891_800
    assert synth.batch_spec() == spec
    # the seeded subset checked against the oracle
    idx = sorted(int(i) for i in np.random.default_rng(8).choice(256, 8, replace=False))
    assert idx == [44, 58, 80, 81, 163, 179, 201, 248]


def test_serve_recipe():
    spec = synth.serve_spec(8)
    assert [(d["npoints"], d["nlev"]) for d in spec] == [
        (177906, 15), (346962, 19), (35970, 7), (891389, 13),
        (25641, 17), (10915, 20), (93354, 17), (21722, 11)]
    assert all(d["nside"] == 1 and d["nbins"] == 31 for d in spec)


def test_small_batch_models_are_valid():
    for m in synth.batch_models(count=256, subset=[163]):
        m.validate()
        assert m.npoints == 2708 and m.nlev == 3
