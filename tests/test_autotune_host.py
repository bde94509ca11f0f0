"""Host logic of the autotuner (no GPU): cache keys and bin candidates."""
import dataclasses

from paper_2511_02852_amd import autotune, scenes


def test_signature_ignores_name_length_and_bins():
    s = scenes.c2()
    a = autotune.scene_signature(s)
    assert a == autotune.scene_signature(s.replace(name="other", steps=5, bins=[32] * 8))
    assert a != autotune.scene_signature(s.replace(seed=7))
    sp = dataclasses.replace(s.spectrum, U10=14.0)
    assert a != autotune.scene_signature(s.replace(spectrum=sp))
    assert a != autotune.scene_signature(s.replace(compact=not s.compact))


def test_bin_candidates_fit_the_library_limits():
    # radii in cells of the stress scene's buckets (0.59 .. 108 cells)
    r = [2 ** ((2 * i + 1) / 4) / 2 for i in range(16)]
    base = scenes.c5().bins
    cands = autotune.bin_candidates(base, r)
    assert cands[0] == base
    assert 2 <= len(cands) <= 3
    for c in cands:
        assert len(c) == 16
        for e, rc in zip(c, r):
            assert autotune.bins_fit(e, rc), (e, rc)
            # the library's own test of a bucket's bin edge
            assert (63 + 4 * rc) / e + 2 <= 32


def test_bins_fit_rejects_what_the_library_rejects():
    assert not autotune.bins_fit(4, 108.0)
    assert autotune.bins_fit(32, 108.0)
    assert not autotune.bins_fit(2, 0.5)      # below the least edge
    assert not autotune.bins_fit(128, 0.5)    # above the largest edge


def test_shipped_tuned_settings_are_valid():
    """The settings shipped with the package (tuned on the target device for
    the benchmark scenes) name usable bin edges and a partition inside the
    library's limits, for the scene signatures of the benchmark scenes."""
    import json
    import os
    if not os.path.exists(autotune.TUNED_PATH):
        return
    store = json.load(open(autotune.TUNED_PATH))
    sigs = {}
    for name in ("c1", "c2", "c3", "c4", "c5", "p0"):
        for kernel in (0, 1):
            s = scenes.get(name).replace(kernel=kernel)
            sigs[autotune.scene_signature(s)] = s
    assert store
    for key, e in store.items():
        dev, sig, pre = key.split("|")[:-2], key.split("|")[-2], key.split("|")[-1]
        assert dev and int(pre) >= 0
        assert sig in sigs, key
        s = sigs[sig]
        assert len(e["bins"]) == s.spectrum.n_buckets
        assert all(autotune.MIN_BIN <= b <= autotune.MAX_BIN for b in e["bins"])
        p = e["plan"]
        assert 64 <= p["chunk_load"] <= 1 << 24 and 0 <= p["items_target"] <= 8192
        assert 0 <= p["splat_grid"] <= 65535 and p["splat_kernel"] in (0, 1, 2)
