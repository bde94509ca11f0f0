"""The paper-default scene against the parameters the paper prints (Sec 5),
and the oracle's particle budget against the direction of the trends in
Table 2 (CPU only).  Fixture: tests/golden/paper_defaults.json."""
import dataclasses
import json
import os

import pytest

import oracle
from paper_2511_02852_amd import scenes

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_defaults.json")))


def test_paper_default_scene_uses_the_printed_parameters():
    d = GOLD["defaults"]
    s = scenes.p0()
    sp = s.spectrum
    assert sp.n_buckets == d["n_omega"] and sp.eta == d["n_theta"]
    assert sp.U10 == d["U10"] and sp.fetch == d["fetch"]
    assert s.fft_n == d["res"] and s.fft_L == d["fft_ocean_size_m"]
    (p,) = s.patches
    assert p.nx == p.ny == d["res"]
    assert p.nx * p.dx == pytest.approx(d["wp_region_size_m"], rel=1e-15)
    # the paper's sampling: equal-energy buckets, a group of N_theta directions
    assert sp.bucket_mode == 1 and sp.dir_mode == 1


def injection_per_step(U10, n):
    """Particles injected per step into the default patch (Eq 17/18 summed
    over the buckets and both side pairs), from the oracle's 32.32 rates."""
    base = scenes.p0()
    sp = dataclasses.replace(base.spectrum, U10=U10, n_buckets=n, eta=float(n))
    o = oracle.Oracle(base.replace(spectrum=sp, bins=[32] * n))
    tot = sum(o.patch_bucket(0, i)["Rx"] + o.patch_bucket(0, i)["Ry"] for i in range(n)) / 2.0 ** 32
    o.close()
    return tot


def test_particle_budget_follows_the_table2_trends():
    """Table 2: frame rate rises with U10 and falls as (N_omega, N_theta)
    grows.  The particle budget that drives the cost moves the opposite way:
    fewer particles per step at higher wind (the spectrum moves to longer
    waves and N_i grows as w_i^3), more with finer sampling."""
    rows = GOLD["table2_hybrid"]
    by_u = sorted((r["U10"], r["fps"]) for r in rows if r["n_omega"] == 16 and r["res"] == 512)
    by_n = sorted((r["n_omega"], r["fps"]) for r in rows if r["U10"] == 5.0 and r["res"] == 512)
    assert [f for _, f in by_u] == sorted(f for _, f in by_u)          # fps rises with U10
    assert [f for _, f in by_n] == sorted((f for _, f in by_n), reverse=True)   # falls with N
    rate_u = [injection_per_step(u, 16) for u, _ in by_u]
    rate_n = [injection_per_step(5.0, n) for n, _ in by_n]
    assert rate_u == sorted(rate_u, reverse=True)
    assert rate_n == sorted(rate_n)
