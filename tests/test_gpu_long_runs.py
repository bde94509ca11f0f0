"""Full-length integer parity of the multi-patch scenes against stored
oracle digests.

The batched scene (32 patches, 1000 steps), the precision scene (600
steps, 50 km from the origin) and the stress scene (64 patches, 16
buckets, 1000 steps) run their whole stated length on the GPU.  At the
middle and the end of the run the per-bucket counts, every bin histogram
and the particle multiset of every patch must equal the FP64 oracle's
bit for bit.  The oracle's values were written by
``tests/golden/make_long_runs.py`` (oracle only) into
``tests/golden/long_runs.json``; ring particles of every source reach
their split ages (a few hundred steps) well inside these runs, so
subdivision is compared on every multi-source scene.
"""
import json
import os
import sys

import numpy as np
import pytest

from paper_2511_02852_amd import scenes

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
from digest import state_digest  # noqa: E402

pytestmark = pytest.mark.gpu

with open(os.path.join(HERE, "golden", "long_runs.json")) as _f:
    GOLDEN = json.load(_f)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_2511_02852_amd import hwo
    hwo.lib()
    yield


def say(*a):
    print(*a, flush=True)


FORMS = {"production": dict(compact=True, batched=True),
         "plain": dict(compact=False, batched=False),
         "scene": {}}


@pytest.mark.parametrize("name,form", [("c3", "production"), ("c3", "plain"), ("c4", "scene"),
                                       ("c5", "production"), ("c5", "plain")])
def test_full_length_integer_state(name, form):
    from paper_2511_02852_amd import hwo
    s = scenes.get(name)
    want = GOLDEN[name]
    assert want["steps"] == s.steps
    npch, nb = len(s.patches), s.spectrum.n_buckets
    say(f"{name} {form}: {npch} patches, {s.steps} steps")
    g = hwo.Ocean(s, **FORMS[form])
    done = 0
    for key in sorted(want["checkpoints"], key=int):
        n = int(key)
        while done < n:
            k = min(100, n - done)
            g.step(k)
            done += k
        g.sync()
        got = state_digest(g, npch, nb)
        ref = want["checkpoints"][key]
        say(f"  n={n} live={got['n_particles']} (oracle {ref['n_particles']})")
        for p in range(npch):
            assert got["counts"][p] == ref["counts"][p], f"n={n} patch {p} counts\n{got['counts'][p]}\n{ref['counts'][p]}"
            assert np.all(np.asarray(g.counts(p))[:, 5] == 0), f"n={n} patch {p} dropped particles"
            assert got["hist_sha"][p] == ref["hist_sha"][p], f"n={n} patch {p} bin histograms"
            assert got["particles_sha"][p] == ref["particles_sha"][p], f"n={n} patch {p} particle multiset"
        assert got["n_particles"] == ref["n_particles"]
        subdivided = sum(int(np.asarray(ref["counts"][p])[:, 3].sum()) for p in range(npch))
        say(f"  n={n}: integer state bit-exact, {subdivided} subdivisions so far")
    g.close()
