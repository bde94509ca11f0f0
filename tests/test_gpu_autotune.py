"""The autotuner: tuned bin edges and splat partition change no integer
result and no height beyond FP32 summation order."""
import numpy as np
import pytest

import oracle
from paper_2511_02852_amd import autotune, scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield


def rel_rms(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.sqrt(np.mean((a - b) ** 2)) / max(np.sqrt(np.mean(b ** 2)), 1e-300))


def canon(P):
    return P[np.lexsort(P.T[::-1])] if P.shape[0] else P


def test_tuned_and_default_settings_agree(tmp_path):
    from paper_2511_02852_amd import hwo
    s = scenes.c2()
    cache = str(tmp_path / "tune.json")
    tuned = autotune.tune(s, preroll=150, cache=cache, reps=2, frames=5, log=print)
    print("tuned", tuned["bins"], tuned["plan"], tuned["frame_ms"], tuned["default_frame_ms"], flush=True)
    assert not tuned["cached"]
    again = autotune.tune(s, preroll=150, cache=cache)
    assert again["cached"] and again["bins"] == tuned["bins"] and again["plan"] == tuned["plan"]
    ga = hwo.Ocean(s, compact=True, batched=True)
    gb = hwo.Ocean(s.replace(bins=tuned["bins"]), compact=True, batched=True)
    autotune.apply(gb, tuned)
    assert gb.get_plan() == tuned["plan"]
    oa, ob = oracle.Oracle(s), oracle.Oracle(s, bins=tuned["bins"])
    for g in (ga, gb):
        g.step(240)
    for o in (oa, ob):
        o.step(240)
    assert np.array_equal(ga.counts(0)[:, :5], gb.counts(0)[:, :5])
    assert np.array_equal(gb.counts(0)[:, :5], ob.counts(0))
    assert np.array_equal(canon(ga.particles()), canon(gb.particles()))
    assert np.array_equal(canon(gb.particles()), canon(ob.particles()))
    for b in range(ob.nb):
        assert np.array_equal(gb.tiles(0, b), ob.tiles(0, b))
        assert np.array_equal(ga.tiles(0, b), oa.tiles(0, b))
    H = ob.background()
    raw, bl = ob.patch_maps(0, H)
    assert rel_rms(gb.patch_map(0, 1), raw) <= 1e-4
    assert rel_rms(gb.patch_map(0, 0), bl) <= 1e-4
    assert rel_rms(ga.patch_map(0, 1), gb.patch_map(0, 1)) <= 1e-5
    ga.close()
    gb.close()
