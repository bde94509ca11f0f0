"""Write ``long_runs.json``: the oracle's integer state of the batched
scenes at the middle and the end of their stated runs.

    python tests/golden/make_long_runs.py [c3 c4 c5]

Calls only the FP64 oracle (``oracle/``) on the seeded scenes of
``paper_2511_02852_amd.scenes``; the stored values are digests of the
oracle's counts, bin histograms and particle multisets (``digest.py``).
The GPU tests compare the library's state at the same steps against them.
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

import oracle  # noqa: E402
from digest import state_digest  # noqa: E402
from paper_2511_02852_amd import scenes  # noqa: E402

OUT = os.path.join(HERE, "long_runs.json")
# checkpoints: the middle and the end of each scene's stated run
CHECKPOINTS = {"c3": (500, 1000), "c4": (300, 600), "c5": (500, 1000)}


def run(name: str) -> dict:
    s = scenes.get(name)
    o = oracle.Oracle(s)
    res = {"scene": s.name, "steps": s.steps, "checkpoints": {}}
    t0 = time.time()
    for n in CHECKPOINTS[name]:
        o.step(n - o.n)
        d = state_digest(o, len(s.patches), s.spectrum.n_buckets)
        res["checkpoints"][str(n)] = d
        print(f"{name} n={n} live={d['n_particles']} ({time.time() - t0:.0f} s)", flush=True)
    o.close()
    return res


def main(names):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    data.setdefault("source", "FP64 oracle (oracle/oracle.c) via tests/golden/make_long_runs.py")
    for name in names:
        data[name] = run(name)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(CHECKPOINTS))
