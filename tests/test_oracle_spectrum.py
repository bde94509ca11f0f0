"""Pins of the oracle's spectral model, buckets and RNG (CPU only).

Each test checks the oracle against something other than itself: a closed
form, an invariant of the paper's equations, or an independent library
implementation.
"""
import dataclasses
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
from paper_2511_02852_amd import scenes


def make(scene=None, **sp):
    s = scene or scenes.c1()
    if sp:
        s = s.replace(spectrum=scenes.Spectrum(**{**s.spectrum.__dict__, **sp}))
    return oracle.Oracle(s)


# ---------------------------------------------------------------- Philox
@pytest.mark.parametrize("ctr,key", [
    ((1, 0, 0, 0), (0, 0)),
    ((5, 7, 11, 13), (0x1234, 0xABCD)),
    ((2**64 - 1, 3, 2**63, 17), (2**64 - 1, 2**64 - 1)),
    ((0, 1, 2, 3), (0, 1)),
])
def test_philox_matches_numpy(ctr, key):
    """Philox4x64-10 against numpy's independent implementation.

    numpy increments the counter before each block, so its state counter
    c - 1 yields the block for counter c."""
    c = list(ctr)
    prev = [(c[0] - 1) % 2**64] + c[1:]
    if c[0] == 0:
        # borrow into the next word
        prev = [2**64 - 1, (c[1] - 1) % 2**64] + c[2:]
    bg = np.random.Philox(counter=np.array(prev, dtype=np.uint64),
                          key=np.array(key, dtype=np.uint64))
    want = bg.random_raw(4)
    got = oracle.philox4x64(c, key)
    assert np.array_equal(got, want)


# ---------------------------------------------------------------- JONSWAP
def test_jonswap_gamma1_closed_form_integral():
    """Eq 2 with gamma = 1: int_0^inf S_J dw = alpha g^2 / (5 wp^4)
    (substitute u = (wp/w)^4)."""
    o = make(gamma=1.0)
    k = o.spectrum_consts()
    g = o.scene.g
    val, err = integrate.quad(o.jonswap, 0.0, np.inf, limit=500, epsabs=0, epsrel=1e-12)
    want = k["alpha"] * g * g / (5.0 * k["wp"] ** 4)
    assert abs(val - want) <= 1e-9 * want


def test_jonswap_peak_location_and_enhancement():
    """gamma = 1 peaks exactly at wp; gamma enters only as gamma^r with
    r = 1 at wp and r = e^{-1/2} one sigma away (sigma 0.07 below, 0.09 above)."""
    o1 = make(gamma=1.0)
    o3 = make(gamma=3.3)
    wp = o1.spectrum_consts()["wp"]
    s0 = o1.jonswap(wp)
    for e in (1e-3, 1e-2):
        assert o1.jonswap(wp * (1 + e)) < s0
        assert o1.jonswap(wp * (1 - e)) < s0
    assert o3.jonswap(wp) / o1.jonswap(wp) == pytest.approx(3.3, rel=1e-13)
    for sig, w in ((0.09, wp * 1.09), (0.07, wp * 0.93)):
        ratio = o3.jonswap(w) / o1.jonswap(w)
        assert ratio == pytest.approx(3.3 ** math.exp(-0.5), rel=1e-12)
    # far from the peak the enhancement vanishes
    assert o3.jonswap(5 * wp) / o1.jonswap(5 * wp) == pytest.approx(1.0, rel=1e-12)


def test_eq4_dimensionless_groups():
    """Eq 4: alpha and gamma depend on U^2/(F g) only and wp U / g likewise,
    so scaling U by 2 and F by 4 leaves alpha, gamma and halves wp."""
    a = make(U10=10.0, fetch=100e3, gamma=-1.0).spectrum_consts()
    b = make(U10=20.0, fetch=400e3, gamma=-1.0).spectrum_consts()
    assert b["alpha"] == pytest.approx(a["alpha"], rel=1e-14)
    assert b["gamma"] == pytest.approx(a["gamma"], rel=1e-14)
    assert b["wp"] == pytest.approx(a["wp"] / 2.0, rel=1e-14)
    # the fetch-limited gamma of Eq 4 lies in the usual 1..7 range
    assert 1.0 < a["gamma"] < 7.0


# ---------------------------------------------------------------- spreading
@pytest.mark.parametrize("s", [0.5, 1.0, 2.0, 4.0, 8.0, 13.7])
def test_dir_normalised(s):
    """Eq 5: int_{-pi}^{pi} Dir = 1."""
    o = make(spread_s=s)
    val, _ = integrate.quad(lambda th: o.dir(1.0, th), -math.pi, math.pi, epsabs=0, epsrel=1e-12,
                            limit=200)
    assert val == pytest.approx(1.0, abs=1e-11)


def test_dir_s1_closed_form():
    """s = 1: Gamma(2)/(2 sqrt(pi) Gamma(3/2)) cos^2(th/2) = (1 + cos th) / (2 pi)."""
    o = make(spread_s=1.0)
    for th in np.linspace(-math.pi, math.pi, 17):
        assert o.dir(1.0, th) == pytest.approx((1 + math.cos(th)) / (2 * math.pi), rel=1e-13,
                                               abs=1e-16)


def test_mitsuyasu_eq6():
    """Eq 6: s(wp) = 16 from both sides, s = 16 (w/wp)^5 below, 16 (w/wp)^-2.5 above."""
    o = make(spread_s=-1.0)
    wp = o.spectrum_consts()["wp"]
    assert o.spread(wp) == pytest.approx(16.0, rel=1e-15)
    assert o.spread(wp * 0.5) == pytest.approx(16.0 / 32.0, rel=1e-13)
    assert o.spread(wp * 2.0) == pytest.approx(16.0 * 2 ** -2.5, rel=1e-13)


def test_direction_table_integer_cdf():
    """Midpoint weights of Dir over 64 bins: exact quadrature of a degree-s
    trig polynomial for integer s < 64, so the integer weights total 2^30 up
    to per-bin rounding; the CDF is their running sum."""
    o = make()
    for i in range(o.nb):
        q, cdf, codes = o.dir_table(i)
        assert np.all(q >= 0)
        assert abs(int(q.sum()) - 2 ** 30) <= 32
        assert np.array_equal(np.cumsum(q), cdf)
        # bin b points at angle -pi + (b + 1/2) 2pi/64 from the wind
        ang = codes * 2 * math.pi / oracle.NCODE
        want = -math.pi + (np.arange(64) + 0.5) * 2 * math.pi / 64
        d = np.angle(np.exp(1j * (ang - want)))
        assert np.max(np.abs(d)) < 1e-12
        # symmetric about the wind
        assert np.array_equal(q, q[::-1])


# ---------------------------------------------------------------- buckets
@pytest.mark.parametrize("name", ["c1", "c2", "c5"])
def test_bucket_kinematics(name):
    """Sec 3.2: k = w^2/g, lambda = 2 pi g / w^2, r = lambda / 2, c = g / w;
    log-spaced wavelength edges cover [lambda_min, lambda_max]."""
    o = oracle.Oracle(scenes.get(name))
    sp = o.scene.spectrum
    g = o.scene.g
    tot = 0.0
    prev = None
    for i in range(o.nb):
        b = o.bucket(i)
        k = b["w"] ** 2 / g
        assert b["lam"] == pytest.approx(2 * math.pi / k, rel=1e-14)
        assert b["r"] == pytest.approx(b["lam"] / 2, rel=1e-14)
        assert b["c"] == pytest.approx(b["w"] / k, rel=1e-14)
        assert sp.lambda_min < b["lam"] < sp.lambda_max
        if prev is not None:
            assert b["lam"] > prev
        prev = b["lam"]
        tot += b["dw"]
    want = math.sqrt(2 * math.pi * g / sp.lambda_min) - math.sqrt(2 * math.pi * g / sp.lambda_max)
    assert tot == pytest.approx(want, rel=1e-13)


def test_velocity_table_fixed_point():
    """Per-step displacement table: |V - c dt u 2^32| <= 1/2 unit."""
    o = oracle.Oracle(scenes.c2())
    dt = o.scene.dt
    for i in (0, 3, 7):
        c = o.bucket(i)["c"]
        for code in (0, 1, 81, 2592, 5184, 7777, 10367):
            ang = 2 * math.pi * code / oracle.NCODE
            vx, vy = o.velocity(i, code)
            assert abs(vx - c * dt * math.cos(ang) * 2 ** 32) <= 0.5 + 1e-6
            assert abs(vy - c * dt * math.sin(ang) * 2 ** 32) <= 0.5 + 1e-6


def test_injection_energy_identity():
    """Eq 12 = N_i x group energy (Eq 15): with importance
    sampling each of the eta particles of a group carries A^2 = 2 S_J dw / eta,
    so for a square patch N_i * eta * (1/8 rho g A^2 pi r^2) must equal
    2 rho g L dt (g / w) S_J(w) dw (the direction integral of Dir is 1)."""
    s = scenes.c1()
    o = oracle.Oracle(s)
    p = s.patches[0]
    L = p.nx * p.dx
    g, dt, rho = s.g, s.dt, 1025.0
    for i in range(o.nb):
        b = o.bucket(i)
        pb = o.patch_bucket(0, i)
        eta = pb["eta"]
        groups = (pb["Rx"] + pb["Ry"]) / 2 ** 32 / eta  # both pairs
        e_group = eta * 0.125 * rho * g * pb["A"] ** 2 * math.pi * b["r"] ** 2
        e_in = 2 * rho * g * L * dt * (g / b["w"]) * o.jonswap(b["w"]) * b["dw"]
        assert groups * e_group == pytest.approx(e_in, rel=1e-9)


def test_injection_rate_scales_with_w_cubed_and_side():
    """Eq 18: the rate per pair is proportional to w_i^3 and to the
    length of the sides of that pair."""
    s = scenes.c1()
    s.patches[0].nx = 96  # rectangle 48 m x 32 m
    o = oracle.Oracle(s)
    b0 = o.bucket(0)
    p0 = o.patch_bucket(0, 0)
    assert p0["Ry"] / p0["Rx"] == pytest.approx(96 / 64, rel=1e-9)
    for i in range(1, o.nb):
        bi = o.bucket(i)
        pi = o.patch_bucket(0, i)
        assert pi["Rx"] / p0["Rx"] == pytest.approx((bi["w"] / b0["w"]) ** 3, rel=1e-9)


def test_injection_counts_telescope():
    """Deterministic fractional counts: sum_{n<=T} cnt(n) = floor(T R / 2^32)
    and each cnt is floor or ceil of R / 2^32."""
    o = oracle.Oracle(scenes.c2())
    for i in range(o.nb):
        R = o.patch_bucket(0, i)["Rx"]
        tot = 0
        for n in range(1, 200):
            c = o.inject_count(0, i, 0, n)
            assert c in (R >> 32, (R >> 32) + 1)
            tot += c
            assert tot == (n * R) >> 32


def test_source_volume_identity():
    """Ring emission: crest volume of one emission sum_j |A_j| r^2 equals the
    volume swept by the disc since the previous emission, 2 R |v| E dt draft."""
    s = scenes.c2()
    o = oracle.Oracle(s)
    src = s.sources[0]
    si = o.source_info(0)
    r = o.bucket(si["bucket"])["r"]
    speed = math.hypot(src.vx, src.vy)
    assert si["B"] * si["sum_abs"] * r * r == pytest.approx(
        2 * src.radius * speed * si["E"] * s.dt * src.draft, rel=1e-12)
    # closest-radius bucket
    rs = [o.bucket(i)["r"] for i in range(o.nb)]
    assert si["bucket"] == int(np.argmin([abs(x - src.radius) for x in rs]))
    # emission cadence: the disc moves at most half a radius between rings
    assert si["E"] * speed * s.dt <= 0.5 * r + 1e-12
    assert (si["E"] + 1) * speed * s.dt > 0.5 * r


def test_subdivision_ages_closed_form():
    """Split age T_L is the first age at which the ring spacing
    alpha_L (R + c dt age) exceeds subdiv_frac * r (alpha_L = 2 pi / (n 3^L))."""
    s = scenes.c2()
    o = oracle.Oracle(s)
    si = o.source_info(0)
    b = o.bucket(si["bucket"])
    R = s.sources[0].radius
    n = s.sources[0].ring_n
    for L in range(4):
        T = si["T"][L]
        alpha = 2 * math.pi / (n * 3 ** L)
        sp = lambda age: alpha * (R + b["c"] * s.dt * age)
        assert sp(T) > 0.5 * b["r"]
        if T > 0:
            assert sp(T - 1) <= 0.5 * b["r"]


def test_equal_energy_buckets():
    """Sec 3.3: the sampling band [0.5 w_p, 2.5 w_p] is cut into N_omega
    buckets of equal energy.  The edges are rebuilt from each bucket's w_i
    (geometric mean of its edges) and dw_i; they must tile the band exactly,
    and every bucket must hold 1/N of the band's integral of S_J, measured with
    an independent adaptive quadrature."""
    s = scenes.p0()
    o = oracle.Oracle(s)
    wp = o.spectrum_consts()["wp"]
    nb = s.spectrum.n_buckets
    edges = []
    for i in range(nb):
        b = o.bucket(i)
        hi = 0.5 * (b["dw"] + math.sqrt(b["dw"] ** 2 + 4.0 * b["w"] ** 2))
        edges.append((hi - b["dw"], hi))
    # bucket 0 holds the highest frequencies (shortest waves); buckets are contiguous
    for i in range(nb - 1):
        assert edges[i][0] == pytest.approx(edges[i + 1][1], rel=1e-12)
        assert o.bucket(i)["w"] > o.bucket(i + 1)["w"]
    assert edges[0][1] == pytest.approx(2.5 * wp, rel=1e-12)
    assert edges[-1][0] == pytest.approx(0.5 * wp, rel=1e-12)
    opts = dict(epsabs=0.0, epsrel=1e-12, limit=200)
    total = integrate.quad(o.jonswap, 0.5 * wp, 2.5 * wp, points=[wp], **opts)[0]
    for lo, hi in edges:
        e = integrate.quad(o.jonswap, lo, hi, points=[wp] if lo < wp < hi else None, **opts)[0]
        assert e == pytest.approx(total / nb, rel=1e-7), (lo, hi)
    # equal energy with the importance-sampled amplitude: A^2 ~ S_J(w_i) dw_i
    # differs between buckets only by how well S_J(w_i) dw_i approximates the
    # bucket integral, which is tight away from the steep low-frequency edge
    A = [o.patch_bucket(0, i)["A"] for i in range(nb - 1)]
    assert max(A) / min(A) < 1.05


def test_bucket_mode_validation():
    s = scenes.p0()
    bad = s.replace(spectrum=dataclasses.replace(s.spectrum, bucket_mode=2))
    with pytest.raises(oracle.OracleError):
        oracle.Oracle(bad)
