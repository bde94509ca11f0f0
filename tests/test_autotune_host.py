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
