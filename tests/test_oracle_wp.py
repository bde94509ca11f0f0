"""Pins of the oracle's wave-particle branch and blend (CPU only)."""
import dataclasses
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from paper_2511_02852_amd import scenes

UNIT = 2 ** 20


def pin_scene(nx=64, dx=0.25, lam=(1.0, 4.0), band=0.0):
    """One bucket with lambda_i = sqrt(1 * 4) = 2 m, so r = 1 m = 4 cells."""
    sp = scenes.Spectrum(U10=10.0, n_buckets=1, lambda_min=lam[0], lambda_max=lam[1], eta=4.0)
    return scenes.Scene(name="pin", fft_n=64, fft_L=256.0, seed=3, steps=0, spectrum=sp,
                        patches=[scenes.Patch(anchor_x=0.0, anchor_y=0.0, nx=nx, ny=nx, dx=dx,
                                              blend_band=band)],
                        bins=[8])


def rec(x_u, y_u, code, bucket=0, birth=0, kind=0, level=0, src=-1, slot=0, patch=0):
    return [patch, bucket, kind, level, code, birth, x_u, y_u, src, slot]


# ---------------------------------------------------------------- splat
@pytest.mark.parametrize("axis", ["x", "y"])
def test_pair_lattice_sums_to_cosine(axis):
    """Fig 1: particles at spacing lambda along their direction and r across
    compose a wave.  With the raised cosine w (a partition of unity at spacing
    r) and each particle a crest/trough pair r apart, the lattice sums to
    exactly A cos(k (x - x0)), k = 2 pi / lambda."""
    s = pin_scene()
    o = oracle.Oracle(s)
    r = o.bucket(0)["r"]
    lam = o.bucket(0)["lam"]
    A = o.patch_bucket(0, 0)["A"]
    x0 = 3.3
    recs = []
    code = 0 if axis == "x" else oracle.NCODE // 4
    for m in range(-3, 12):
        for n in range(-3, 24):
            a = x0 + m * lam   # along the direction
            b = 0.1 + n * r    # across
            xu, yu = (a, b) if axis == "x" else (b, a)
            recs.append(rec(int(round(xu * UNIT)), int(round(yu * UNIT)), code))
    recs = np.array(recs)
    # exact positions after rounding to units
    h = o.splat(0, recs)
    p = s.patches[0]
    xc = (np.arange(p.nx) + 0.5) * p.dx
    X, Y = np.meshgrid(xc, xc)
    along = X if axis == "x" else Y
    x0u = round(x0 * UNIT) / UNIT
    want = A * np.cos(math.pi * (along - x0u) / r)
    # lattice rounding to 2^-20 m is below 1e-6 of a radius
    assert np.max(np.abs(h - want)) <= 1e-5 * A


def test_single_pair_moments():
    """Crest volume of the raised-cosine product is A (r/dx)^2 per cell area
    when 2r/dx is an integer; the pair has zero volume and first moment
    A (r/dx)^2 r along its direction (trough one radius behind)."""
    s = pin_scene()
    o = oracle.Oracle(s)
    r = o.bucket(0)["r"]
    A = o.patch_bucket(0, 0)["A"]
    p = s.patches[0]
    xc = (np.arange(p.nx) + 0.5) * p.dx
    X, Y = np.meshgrid(xc, xc)
    for code, ux, uy in ((0, 1, 0), (oracle.NCODE // 4, 0, 1), (oracle.NCODE // 2, -1, 0)):
        px, py = 8.13, 7.71
        h = o.splat(0, np.array([rec(int(px * UNIT), int(py * UNIT), code)]))
        vol = (r / p.dx) ** 2 * A
        assert abs(h.sum()) <= 1e-12 * vol
        mx = (h * X).sum()
        my = (h * Y).sum()
        assert mx == pytest.approx(vol * r * ux, abs=1e-9 * vol)
        assert my == pytest.approx(vol * r * uy, abs=1e-9 * vol)
        # positive lobe of the crest alone equals the crest volume when the
        # trough does not overlap: check the crest peak value
        i = np.unravel_index(np.argmax(h), h.shape)
        assert h[i] <= A + 1e-15


def test_single_particle_closed_form():
    """One particle at direction theta: h = A [w(dx) w(dy) - w(dx + r cos) w(dy + r sin)]."""
    s = pin_scene()
    o = oracle.Oracle(s)
    r = o.bucket(0)["r"]
    A = o.patch_bucket(0, 0)["A"]
    p = s.patches[0]
    code = 1234
    th = 2 * math.pi * code / oracle.NCODE
    xu, yu = 8_000_001, 8_400_003
    h = o.splat(0, np.array([rec(xu, yu, code)]))
    xc = (np.arange(p.nx) + 0.5) * p.dx
    X, Y = np.meshgrid(xc, xc)

    def w(d):
        return np.where(np.abs(d) < r, 0.5 * (1 + np.cos(np.pi * d / r)), 0.0)

    dx_, dy_ = X - xu / UNIT, Y - yu / UNIT
    want = A * (w(dx_) * w(dy_) - w(dx_ + r * math.cos(th)) * w(dy_ + r * math.sin(th)))
    assert np.max(np.abs(h - want)) <= 1e-14


def radial_scene():
    """One bucket with lambda = 4 m, r = 2 m = 8 cells of 0.25 m, radial kernel."""
    return pin_scene(lam=(2.0, 8.0)).replace(kernel=1)


def test_radial_kernel_depends_on_distance_only():
    """Fig 1 profile taken as a radial W(|d|): in front of a crest moving
    along +x the trough (one radius behind) contributes nothing, so every
    cell at the same distance from the crest holds the same value -- here the
    lattice points at distance 5 cells: (3, 4), (4, 3), (5, 0), (0, 5) and
    their mirror images in y.  The separable product gives w(3)w(4) != w(5)w(0)."""
    s = radial_scene()
    o = oracle.Oracle(s)
    assert o.bucket(0)["r"] == pytest.approx(2.0)
    A = o.patch_bucket(0, 0)["A"]
    dxu = int(0.25 * UNIT)
    i0, j0 = 30, 31
    h = o.splat(0, np.array([rec(i0 * dxu + dxu // 2, j0 * dxu + dxu // 2, 0)]))
    vals = [h[j0 + dy, i0 + dx] for dx, dy in ((3, 4), (4, 3), (5, 0), (0, 5), (3, -4), (4, -3), (0, -5))]
    assert min(vals) > 0.05 * A
    assert max(vals) - min(vals) <= 1e-14 * A
    sep = oracle.Oracle(pin_scene(lam=(2.0, 8.0)))
    hs = sep.splat(0, np.array([rec(i0 * dxu + dxu // 2, j0 * dxu + dxu // 2, 0)]))
    assert abs(hs[j0 + 4, i0 + 3] - hs[j0, i0 + 5]) > 0.02 * A   # 0.346 A vs 0.309 A


def test_radial_kernel_volume_and_moment():
    """The pair has zero volume (crest and trough sample the kernel at the
    same sub-cell offsets when r is a whole number of cells along an axis) and
    first moment A V r along its direction, where V is the crest's volume in
    cells; V tends to the integral of the raised cosine over the disc,
    r^2 (pi/2 - 2/pi), within 5e-4 at r = 8 cells (midpoint rule)."""
    s = radial_scene()
    o = oracle.Oracle(s)
    r = o.bucket(0)["r"]
    A = o.patch_bucket(0, 0)["A"]
    p = s.patches[0]
    rc = r / p.dx
    xc = (np.arange(p.nx) + 0.5) * p.dx
    X, Y = np.meshgrid(xc, xc)
    disc = rc * rc * (math.pi / 2 - 2 / math.pi)
    for code, ux, uy in ((0, 1, 0), (oracle.NCODE // 4, 0, 1), (oracle.NCODE // 2, -1, 0)):
        px, py = 8.13, 7.71
        h = o.splat(0, np.array([rec(int(px * UNIT), int(py * UNIT), code)]))
        assert abs(h.sum()) <= 1e-12 * A * disc
        V = ((h * X).sum() * ux + (h * Y).sum() * uy) / (A * r)
        assert V == pytest.approx(disc, rel=5e-4)
        assert abs(V - rc * rc) > 0.05 * rc * rc   # not the separable kernel's (r/dx)^2


def test_radial_kernel_validation():
    s = radial_scene()
    for bad in (s.replace(kernel=2), s.replace(synth=1)):
        with pytest.raises(oracle.OracleError):
            oracle.Oracle(bad)


# ---------------------------------------------------------------- blend
def test_blend_limits_and_bilinear():
    """Sec 3.1 local replacement: a vanishing blend band gives the pure WP map
    inside the patch; an unbounded band gives the background sampled by
    bilinear interpolation at the cell's world position (exact for a field
    linear in the grid index, away from the periodic wrap)."""
    H = np.zeros((64, 64))
    jy, jx = np.mgrid[0:64, 0:64]
    H[:] = 0.01 * jx - 0.02 * jy + 0.3
    s = scenes.c1()
    s.patches[0].blend_band = 1e-9
    o = oracle.Oracle(s)
    o.step(3)
    raw, bl = o.patch_maps(0, H)
    assert np.array_equal(raw, bl)
    s = scenes.c1()
    s.patches[0].blend_band = 1e12
    o = oracle.Oracle(s)
    o.step(3)
    raw, bl = o.patch_maps(0, H)
    p = s.patches[0]
    dxf = s.fft_L / s.fft_n
    X = p.anchor_x + (np.arange(p.nx) + 0.5) * p.dx
    Y = p.anchor_y + (np.arange(p.ny) + 0.5) * p.dx
    XX, YY = np.meshgrid(X, Y)
    want = 0.01 * XX / dxf - 0.02 * YY / dxf + 0.3
    assert np.max(np.abs(bl - want)) <= 1e-12


def test_blend_profile():
    """Default band: weight 1 (pure WP) at depth >= band, smooth rise from
    ~0 at the border, monotone in depth."""
    s = scenes.c1()
    o = oracle.Oracle(s)
    o.step(0)
    H = np.ones((64, 64))
    raw, bl = o.patch_maps(0, H)   # no particles: raw = 0, blended = 1 - w
    p = s.patches[0]
    band = o.patch_bucket(0, 0)["band"]
    i = np.arange(p.nx)
    d = np.minimum(i + 0.5, p.nx - i - 0.5) * p.dx
    row = bl[p.ny // 2]            # depth along x only in the middle row
    deep = d >= band
    assert np.all(row[deep] == 0.0)
    sh = ~deep
    assert np.all(row[sh] > 0) and np.all(row[sh] < 1)
    # outermost cell: 1 - w >= 1 - 3 (dx / 2 band)^2
    assert row[0] >= 1 - 3 * (0.5 * p.dx / band) ** 2
    half = row[: p.nx // 2]
    assert np.all(np.diff(half) <= 0)


# ---------------------------------------------------------------- kinematics
def positions(o, P, n):
    out = np.zeros((P.shape[0], 2), dtype=np.int64)
    for k, q in enumerate(P):
        vx, vy = o.velocity(int(q[1]), int(q[4]))
        age = n - q[5]
        out[k, 0] = q[6] + ((age * vx) >> 12)
        out[k, 1] = q[7] + ((age * vy) >> 12)
    return out


def test_propagation_and_survival_window():
    """Positions advance at the bucket phase speed c_i = g / w_i (Sec 3.2) to
    within the fixed-point rounding, and every live particle lies inside its
    window expanded by 2 r."""
    s = scenes.c2()
    o = oracle.Oracle(s)
    o.step(120)
    P = o.particles()
    assert P.shape[0] > 10000
    n = o.n
    pos = positions(o, P, n)
    wx, wy = o.window(0)
    dxu = int(s.patches[0].dx * UNIT)
    sel = np.random.default_rng(0).choice(P.shape[0], 3000, replace=False)
    for k in sel:
        q = P[k]
        b = o.bucket(int(q[1]))
        age = n - q[5]
        th = 2 * math.pi * q[4] / oracle.NCODE
        ex = q[6] + age * b["c"] * s.dt * math.cos(th) * UNIT
        ey = q[7] + age * b["c"] * s.dt * math.sin(th) * UNIT
        assert abs(pos[k, 0] - ex) <= 1 + age * 0.5 / 4096
        assert abs(pos[k, 1] - ey) <= 1 + age * 0.5 / 4096
        m = b["margin_u"]
        assert wx * dxu - m <= pos[k, 0] <= (wx + s.patches[0].nx) * dxu + m
        assert wy * dxu - m <= pos[k, 1] <= (wy + s.patches[0].ny) * dxu + m


def test_entry_side_matches_direction():
    """Boundary particles enter through the side they travel away from."""
    s = scenes.c1()
    o = oracle.Oracle(s)
    o.step(5)
    P = o.particles()
    new = P[(P[:, 5] == 5) & (P[:, 2] == 0)]
    assert new.shape[0] > 50
    dxu = int(s.patches[0].dx * UNIT)
    W = s.patches[0].nx * dxu
    for q in new:
        vx, vy = o.velocity(int(q[1]), int(q[4]))
        on_l, on_r = q[6] == 0, q[6] == W
        on_b, on_t = q[7] == 0, q[7] == W
        assert on_l or on_r or on_b or on_t
        if on_l:
            assert vx > 0 or on_b or on_t
        if on_r:
            assert vx <= 0 or on_b or on_t
        if on_b:
            assert vy > 0 or on_l or on_r
        if on_t:
            assert vy <= 0 or on_l or on_r


def test_inverse_cdf_direction_frequencies():
    """Directions are drawn from Dir (Sec 4.2): chi-square of the bin
    frequencies of freshly injected particles against q / Q."""
    s = scenes.c1()
    s.spectrum.eta = 1000.0
    o = oracle.Oracle(s)
    q, cdf, codes = o.dir_table(0)
    counts = np.zeros(64)
    code_to_bin = {int(c): b for b, c in enumerate(codes)}
    for n in range(1, 9):
        o.step(1)
        P = o.particles()
        new = P[(P[:, 5] == n) & (P[:, 1] == 0)]
        for c in new[:, 4]:
            counts[code_to_bin[int(c)]] += 1
    tot = counts.sum()
    assert tot > 20000
    exp = tot * q / q.sum()
    keep = exp >= 5
    obs = np.append(counts[keep], counts[~keep].sum())
    ex = np.append(exp[keep], exp[~keep].sum())
    chi2 = ((obs - ex) ** 2 / ex).sum()
    dof = obs.size - 1
    assert stats.chi2.sf(chi2, dof) > 1e-4
    assert counts[~(q > 0)].sum() == 0


def test_count_conservation_and_histogram():
    """Per bucket: live = injected + emitted + 2 x subdivided - died, and the
    bin histogram sums to the live count on the stated bin grid."""
    s = scenes.c2()
    o = oracle.Oracle(s)
    o.step(400)
    c = o.counts(0)
    live = c[:, 0]
    assert np.array_equal(live, c[:, 1] + c[:, 2] + 2 * c[:, 3] - c[:, 4])
    assert c[:, 3].sum() > 0   # splits happened
    P = o.particles()
    for b in range(o.nb):
        assert (P[:, 1] == b).sum() == live[b]
        binw, nbx, nby = o.tile_dims(0, b)
        m = o.bucket(b)["margin_u"]
        dxu = int(s.patches[0].dx * UNIT)
        assert nbx == (s.patches[0].nx * dxu + 2 * m) // (binw * dxu) + 1
        assert o.tiles(0, b).sum() == live[b]


def test_emission_count():
    """A source emits a ring of n_e particles every E steps, from step 1."""
    s = scenes.c2()
    o = oracle.Oracle(s)
    E = o.source_info(0)["E"]
    o.step(100)
    b = o.source_info(0)["bucket"]
    assert o.counts(0)[b, 2] == 64 * math.ceil(100 / E)


def test_subdivision_conserves_amplitude():
    """A split replaces a particle of amplitude B m 3^-L by three of
    B m 3^-(L+1) at codes c and c +- a0 / 3^(L+1): each complete family (one
    ring slot of one emission) keeps total amplitude B m and a code set
    symmetric about the slot direction."""
    s = scenes.c2()
    o = oracle.Oracle(s)
    si = o.source_info(0)
    o.step(si["T"][0] + 40)
    P = o.particles()
    src = P[P[:, 2] == 1]
    assert (src[:, 3] >= 1).any()
    fam = {}
    for q in src:
        fam.setdefault((int(q[5]), int(q[9])), []).append(q)
    a0 = si["a0"]
    checked = 0
    for (birth, slot), qs in fam.items():
        levels = {int(q[3]) for q in qs}
        assert len(levels) == 1
        L = levels.pop()
        if len(qs) != 3 ** L:
            continue  # part of the family has left the window
        tot = sum(3.0 ** -int(q[3]) for q in qs)
        assert tot == pytest.approx(1.0, rel=1e-14)
        offs = sorted(((int(q[4]) - slot * a0 + oracle.NCODE // 2) % oracle.NCODE) - oracle.NCODE // 2
                      for q in qs)
        assert offs == sorted(-x for x in offs)
        step = a0 // 3 ** L if L else a0
        if L:
            assert all(x % step == 0 for x in offs)
        checked += 1
    assert checked > 10


def test_seek_splat_and_blend_reproduce_patch_maps():
    """Evaluating a stepped oracle's own particles through seek + splat + blend
    in a fresh oracle gives the stepped oracle's maps (windows, ages and the
    blend depend only on the step index)."""
    s = scenes.c1()
    a = oracle.Oracle(s)
    a.step(12)
    H = a.background()
    raw, bl = a.patch_maps(0, H)
    b = oracle.Oracle(s)
    b.seek(12)
    assert b.window(0) == a.window(0)
    raw2 = b.splat(0, a.particles())
    assert np.allclose(raw2, raw, rtol=0, atol=1e-12 * max(1.0, np.abs(raw).max()))
    assert np.allclose(b.blend(0, H, raw2), bl, rtol=0, atol=1e-12 * max(1.0, np.abs(bl).max()))
    with pytest.raises(oracle.OracleError):
        a.seek(20)   # holds particles


# ---------------------------------------------------------------- stratified directions
def strat_scene(wind_dir, spread_s=-1.0, eta=16.0, nx=64):
    """Two equal-energy buckets of the paper's default spectrum with Mitsuyasu
    spreading (a different s per bucket), stratified directions."""
    sp = scenes.Spectrum(U10=5.0, fetch=10e3, gamma=0.0, spread_s=spread_s, wind_dir=wind_dir,
                         n_buckets=2, eta=eta, bucket_mode=1, dir_mode=1)
    return scenes.Scene(name="strat", fft_n=64, fft_L=256.0, seed=5, steps=0, spectrum=sp,
                        patches=[scenes.Patch(anchor_x=0.0, anchor_y=0.0, nx=nx, ny=nx,
                                              dx=100.0 / 512)],
                        bins=[16, 16])


def wind_code(wind_dir):
    return int(round(wind_dir * oracle.NCODE / (2 * math.pi))) % oracle.NCODE


def test_stratified_groups_cover_every_sector():
    """Sec 3.3: a group holds N_theta particles spanning all directions with
    dtheta = 2 pi / N_theta.  The injected stream of each (bucket, side pair)
    visits the N_theta sectors round robin, so over any run each sector holds
    floor or ceil of M / N_theta of that stream's M particles; inside its
    sector a direction is uniform."""
    wd = 0.7
    s = strat_scene(wd, eta=16.0, nx=512)
    o = oracle.Oracle(s)
    nsteps = 40
    o.step(nsteps)
    P = o.particles()
    c = o.counts(0)
    nth = 16
    frac = []
    for b in range(o.nb):
        M = [sum(o.inject_count(0, b, pair, n) for n in range(1, nsteps + 1)) for pair in (0, 1)]
        assert c[b, 1] == sum(M) and sum(M) > 10 * nth
        died = int(c[b, 4])
        rel = (P[P[:, 1] == b, 4] - wind_code(wd) - oracle.NCODE // 2) % oracle.NCODE
        sector = rel * nth // oracle.NCODE
        per = np.bincount(sector, minlength=nth)
        lo = sum(m // nth for m in M) - died
        hi = sum(-(-m // nth) for m in M)
        assert per.min() >= lo and per.max() <= hi, (b, per, M, died)
        lo_code = sector * oracle.NCODE // nth
        hi_code = (sector + 1) * oracle.NCODE // nth
        frac.append((rel - lo_code) / (hi_code - lo_code))
    frac = np.concatenate(frac)
    assert frac.min() >= 0.0 and frac.max() < 1.0
    assert stats.kstest(frac, "uniform").pvalue > 1e-4


def test_stratified_amplitude_follows_directional_spectrum():
    """Eq 7 with dtheta = 2 pi / N_theta: relative to the equal-amplitude
    particle of the inverse-CDF mode, a particle heading theta carries
    sqrt(2 pi Dir(theta - wind)).  Pinned by single-particle splats against
    what Dir must satisfy: it integrates to one over a turn (so the squared
    factor averages to one over the directions), it peaks along the wind, it
    is even about the wind and it vanishes against it (cos-2s, Eq 5)."""
    k0 = 1008
    wd = 2 * math.pi * k0 / oracle.NCODE
    s1 = strat_scene(wd)
    s0 = s1.replace(spectrum=dataclasses.replace(s1.spectrum, dir_mode=0))
    o1, o0 = oracle.Oracle(s1), oracle.Oracle(s0)
    c = (0.5 * 64 * 100.0 / 512) * UNIT
    stride = 16
    codes = np.arange(0, oracle.NCODE, stride)
    def factor(b, q):
        one = np.array([rec(int(c), int(c), int(q), bucket=b)])
        ref = o0.splat(0, one)
        j = np.unravel_index(np.argmax(np.abs(ref)), ref.shape)
        return o1.splat(0, one)[j] / ref[j]

    for b in range(2):
        ratio = np.array([factor(b, q) for q in codes])
        assert np.all(ratio >= 0.0)
        # periodic trapezoid rule over a smooth periodic integrand
        assert np.mean(ratio ** 2) == pytest.approx(1.0, abs=1e-9)
        assert codes[np.argmax(ratio)] == k0
        opp = (k0 + oracle.NCODE // 2) % oracle.NCODE
        assert ratio[codes == opp][0] == pytest.approx(0.0, abs=1e-12)
        for d in (stride, 7 * stride, 100 * stride):
            a = ratio[codes == (k0 + d) % oracle.NCODE][0]
            bb = ratio[codes == (k0 - d) % oracle.NCODE][0]
            assert a == pytest.approx(bb, rel=1e-9)
    # the Mitsuyasu exponent differs between the buckets (s peaks at w_p)
    assert o1.spread(o1.bucket(0)["w"]) != o1.spread(o1.bucket(1)["w"])


def test_stratified_needs_whole_group():
    s = strat_scene(0.0, eta=16.5)
    with pytest.raises(oracle.OracleError):
        oracle.Oracle(s)
    s = strat_scene(0.0, eta=16.0)
    s.patches[0].eta = 3.25
    with pytest.raises(oracle.OracleError):
        oracle.Oracle(s)


# ---------------------------------------------------------------- obliquity-weighted injection
def live_inside(o, scene):
    """Per-bucket number of live particles whose current position lies inside
    the patch proper (positions from origin, birth step and velocity)."""
    p = scene.patches[0]
    wx, wy = o.window(0)
    dxu = int(round(p.dx * UNIT))
    P = o.particles()
    keys = {(int(b), int(c)) for b, c in zip(P[:, 1], P[:, 4])}
    V = {k: o.velocity(*k) for k in keys}
    v = np.array([V[(int(b), int(c))] for b, c in zip(P[:, 1], P[:, 4])], dtype=np.int64).reshape(-1, 2)
    age = o.n - P[:, 5]
    px = P[:, 6] + (age * v[:, 0]) // 4096
    py = P[:, 7] + (age * v[:, 1]) // 4096
    inside = ((px >= wx * dxu) & (px < (wx + p.nx) * dxu) & (py >= wy * dxu) & (py < (wy + p.ny) * dxu))
    return np.array([np.sum(inside & (P[:, 1] == b)) for b in range(o.nb)])


def test_obliquity_weighted_injection_reaches_spectral_density():
    """With obliquity weighting the inflow of direction theta through a side
    is c |n . u| times the density, so the steady state holds a uniform
    density of eta 4 w^4 / (pi^3 g^2) particles per square metre in each
    bucket (Eq 13 and Eq 9: the energy density rho g S_J(w_i) dw_i).  The
    paper-literal count of Eq 18 overfills the same square: at oblique
    incidence a side pair's share is not reduced by |cos|."""
    base = scenes.c1()
    L = base.patches[0].nx * base.patches[0].dx
    for fm in (1, 0):
        s = base.replace(spectrum=dataclasses.replace(base.spectrum, flux_mode=fm, wind_dir=0.4))
        o = oracle.Oracle(s)
        # the longest chord of the square, L sqrt 2, takes 30 s at the slowest c
        o.step(2000)
        acc = np.zeros(o.nb)
        for _ in range(6):
            o.step(25)
            acc += live_inside(o, s)
        acc /= 6
        for b in range(o.nb):
            w = o.bucket(b)["w"]
            want = s.spectrum.eta * 4.0 * L * L * w ** 4 / (math.pi ** 3 * s.g ** 2)
            if fm == 1:
                assert abs(acc[b] - want) <= 4.0 * math.sqrt(want), (b, acc[b], want)
            else:
                assert acc[b] > 1.3 * want, (b, acc[b], want)


def test_obliquity_factor_and_direction_weights():
    """kappa, the factor on a side pair's count, is the mean of |cos| (x
    sides) or |sin| (y sides) of the direction under Dir: 2/pi for both pairs
    when s = 1 and the wind is along an axis (Dir = (1 + cos theta) / 2 pi),
    and the quadrature of the integral otherwise (64-bin midpoint rule, whose
    error at the two kinks of |cos| is below 3e-3)."""
    from scipy import integrate
    for spread, wd in ((1.0, 0.0), (8.0, 0.4), (2.0, 2.5)):
        s0 = scenes.c1()
        s0 = s0.replace(spectrum=dataclasses.replace(s0.spectrum, spread_s=spread, wind_dir=wd))
        s1 = s0.replace(spectrum=dataclasses.replace(s0.spectrum, flux_mode=1))
        o0, o1 = oracle.Oracle(s0), oracle.Oracle(s1)
        for b in range(o0.nb):
            w = o0.bucket(b)["w"]
            p0, p1 = o0.patch_bucket(0, b), o1.patch_bucket(0, b)
            for key, f in (("Rx", lambda t: abs(math.cos(t))), ("Ry", lambda t: abs(math.sin(t)))):
                want = integrate.quad(lambda t: f(t) * o0.dir(w, t - wd), -math.pi, math.pi,
                                      points=[-math.pi / 2, 0.0, math.pi / 2], limit=200)[0]
                if spread == 1.0 and wd == 0.0:
                    assert want == pytest.approx(2.0 / math.pi, rel=1e-9)
                assert p1[key] / p0[key] == pytest.approx(want, rel=3e-3), (spread, wd, b, key)
            # the literal mode shares one table between the pairs
            assert np.array_equal(o0.dir_table(b, 0)[0], o0.dir_table(b, 1)[0])


def test_flux_mode_validation():
    s = scenes.c1()
    for kw in (dict(flux_mode=2), dict(flux_mode=1, dir_mode=1)):
        bad = s.replace(spectrum=dataclasses.replace(s.spectrum, **kw))
        with pytest.raises(oracle.OracleError):
            oracle.Oracle(bad)


# ---------------------------------------------------------------- texel-layer synthesis
def texel_pair(s, synth, x_u, y_u, code, bucket=0):
    o = oracle.Oracle(s.replace(synth=synth))
    return o.splat(0, np.array([rec(x_u, y_u, code, bucket=bucket)]))


def test_texel_layers_equal_exact_splat_at_cell_centres():
    """Sec 4.2 synthesis (deposit into a bucket layer, then a pass along x and
    one along y): a crest and trough sitting on cell centres deposit into one
    texel each, and the separable passes then evaluate the raised cosine at
    exact cell offsets, so the layer map equals the exact-position splat."""
    s = pin_scene()
    dxu = int(s.patches[0].dx * UNIT)
    for code in (0, oracle.NCODE // 4, oracle.NCODE // 2):
        for (i, j) in ((20, 31), (1, 2), (63, 0)):
            xu, yu = i * dxu + dxu // 2, j * dxu + dxu // 2
            h0 = texel_pair(s, 0, xu, yu, code)
            h1 = texel_pair(s, 1, xu, yu, code)
            assert np.max(np.abs(h0)) > 0.1 * o_amp(s)
            assert np.max(np.abs(h1 - h0)) <= 1e-12 * o_amp(s)


def o_amp(s):
    return oracle.Oracle(s).patch_bucket(0, 0)["A"]


def test_texel_layers_second_order_in_cell_size():
    """Bilinear deposit makes the layer map the bilinear interpolant, in the
    particle position, of the exact kernel: per point the error is at most
    A dx^2 max|w''| / 4 = A dx^2 pi^2 / (8 r^2), and it falls by 4 when dx
    halves.  Particles up to a radius outside the patch count too."""
    rng = np.random.default_rng(7)
    errs = []
    for nx, dx in ((64, 0.25), (128, 0.125)):
        s = pin_scene(nx=nx, dx=dx)
        A = o_amp(s)
        r = 1.0
        bound = 2 * A * dx * dx * math.pi ** 2 / (8 * r * r)
        L = nx * dx
        worst = 0.0
        for _ in range(12):
            x, y = rng.uniform(-r, L + r, size=2)
            code = int(rng.integers(0, oracle.NCODE))
            xu, yu = int(round(x * UNIT)), int(round(y * UNIT))
            d = np.max(np.abs(texel_pair(s, 1, xu, yu, code) - texel_pair(s, 0, xu, yu, code)))
            assert d <= bound * (1 + 1e-9), (nx, x, y, code, d, bound)
            worst = max(worst, d / A)
        errs.append(worst)
    assert errs[0] / errs[1] > 3.0


def test_texel_layers_sum_buckets_and_blend():
    """Layers are summed: a scene's texel map is the sum of its particles'
    maps; the mode changes the splat only (same particles, same blend)."""
    s = scenes.c1().replace(synth=1)
    o = oracle.Oracle(s)
    o.step(6)
    P = o.particles()
    raw, bl = o.patch_maps(0)
    parts = sum(o.splat(0, P[P[:, 1] == b]) for b in range(o.nb))
    assert np.max(np.abs(raw - parts)) <= 1e-12 * max(np.max(np.abs(raw)), 1.0)
    s0 = scenes.c1()
    o0 = oracle.Oracle(s0)
    o0.step(6)
    assert np.array_equal(o0.particles(), P)
    raw0, _ = o0.patch_maps(0)
    assert np.sqrt(np.mean((raw - raw0) ** 2)) < 0.05 * np.sqrt(np.mean(raw0 ** 2))


# ---------------------------------------------------------------- normals
def test_normals_exact_for_planes_and_closed_form_for_cosines():
    """Sec 4.2 normals by finite differences.  Central (and the one-sided
    edge) differences are exact for a plane h = a x + b y, giving the normal
    (-a, -b, 1) / sqrt(1 + a^2 + b^2) everywhere.  For h = A cos(k x) the
    interior central difference is -A sin(k x) sin(k dx) / dx exactly, which
    tends to the analytic slope -A k sin(k x) as dx^2."""
    s = pin_scene(nx=64, dx=0.25)
    o = oracle.Oracle(s)
    p = s.patches[0]
    xc = (np.arange(p.nx) + 0.5) * p.dx
    X, Y = np.meshgrid(xc, xc)
    a, b = 0.3, -0.7
    n = o.normals(0, a * X + b * Y)
    want = np.array([-a, -b, 1.0]) / math.sqrt(1 + a * a + b * b)
    assert np.max(np.abs(n - want[:, None, None])) <= 1e-12
    A, k = 0.4, 2 * math.pi / 3.0
    n = o.normals(0, A * np.cos(k * X))
    sx = -A * np.sin(k * X[:, 1:-1]) * math.sin(k * p.dx) / p.dx
    inv = 1.0 / np.sqrt(1 + sx * sx)
    assert np.max(np.abs(n[0][:, 1:-1] - (-sx * inv))) <= 1e-12
    assert np.max(np.abs(n[2][:, 1:-1] - inv)) <= 1e-12
    assert np.max(np.abs(n[1])) <= 1e-12
    assert np.allclose(np.sum(n * n, axis=0), 1.0, atol=1e-12)
    # second order: the gap to the analytic normal falls by 4 when dx halves
    errs = []
    for nx, dx in ((64, 0.25), (128, 0.125)):
        s2 = pin_scene(nx=nx, dx=dx)
        o2 = oracle.Oracle(s2)
        xc = (np.arange(nx) + 0.5) * dx
        X2, _ = np.meshgrid(xc, xc)
        n2 = o2.normals(0, A * np.cos(k * X2))
        ex = A * k * np.sin(k * X2)   # -dh/dx
        errs.append(np.max(np.abs(n2[0][:, 1:-1] - ex[:, 1:-1] / np.sqrt(1 + ex[:, 1:-1] ** 2))))
    assert 3.5 < errs[0] / errs[1] < 4.5


# ---------------------------------------------------------------- probes
def test_probe_sampling_exact_for_planes_and_grid_points():
    """Object-receives-water sampling (Sec 4.3): inside a patch the probe
    reads the bilinear interpolant of the blended map and a normal from
    interpolated finite-difference slopes, both exact for a plane; outside
    every patch it reads the periodic background, and at a background grid
    point it returns the grid value and the central-difference slope, here
    checked on one Fourier mode against its closed form."""
    s = pin_scene(nx=64, dx=0.25)
    o = oracle.Oracle(s)
    o.step(1)
    p = s.patches[0]
    wx, wy = o.window(0)
    N, L = s.fft_n, s.fft_L
    dxf = L / N
    # plane on the patch, background elsewhere
    xc = p.anchor_x + (wx + np.arange(p.nx) + 0.5) * p.dx
    yc = p.anchor_y + (wy + np.arange(p.ny) + 0.5) * p.dx
    X, Y = np.meshgrid(xc, yc)
    a, b, c0 = 0.2, -0.35, 1.5
    plane = a * X + b * Y + c0
    k = 2 * math.pi / L * 3
    gx = np.arange(N) * dxf
    GX, GY = np.meshgrid(gx, gx)
    H = np.cos(k * GX)
    rng = np.random.default_rng(3)
    inside = np.column_stack([rng.uniform(xc[0], xc[-1], 40), rng.uniform(yc[0], yc[-1], 40)])
    out = o.sample_probes(inside, H=H, blended=[plane])
    assert np.max(np.abs(out[:, 0] - (a * inside[:, 0] + b * inside[:, 1] + c0))) <= 1e-12
    want = np.array([-a, -b, 1.0]) / math.sqrt(1 + a * a + b * b)
    assert np.max(np.abs(out[:, 1:] - want)) <= 1e-12
    # grid points of the background away from the patch
    jx = np.array([40, 41, 50, 63]); jy = np.array([5, 60, 33, 47])
    pts = np.column_stack([jx * dxf, jy * dxf])
    assert not np.any((pts[:, 0] >= xc[0]) & (pts[:, 0] <= xc[-1]) & (pts[:, 1] >= yc[0]) & (pts[:, 1] <= yc[-1]))
    out = o.sample_probes(pts, H=H, blended=[plane])
    assert np.max(np.abs(out[:, 0] - np.cos(k * jx * dxf))) <= 1e-12
    sx = -np.sin(k * jx * dxf) * math.sin(k * dxf) / dxf
    assert np.max(np.abs(out[:, 1] - (-sx / np.sqrt(1 + sx * sx)))) <= 1e-12
    assert np.max(np.abs(out[:, 2])) <= 1e-12


# ---------------------------------------------------------------- bins and windows
def crest_positions(o, P, n):
    """Crest positions origin + floor(age V / 4096), V from the (separately
    pinned) velocity table, vectorised over the particle set."""
    key = P[:, 1] * oracle.NCODE + P[:, 4]
    uk, inv = np.unique(key, return_inverse=True)
    V = np.array([o.velocity(int(k // oracle.NCODE), int(k % oracle.NCODE)) for k in uk],
                 dtype=np.int64).reshape(-1, 2)
    age = n - P[:, 5]
    px = P[:, 6] + np.floor_divide(age * V[inv, 0], 4096)
    py = P[:, 7] + np.floor_divide(age * V[inv, 1], 4096)
    return px, py


@pytest.mark.parametrize("name,steps", [("c2", 400), ("c1", 16)])
def test_bin_histogram_is_histogram2d_of_crests(name, steps):
    """The per-(patch, bucket) bin histogram (the counting-sort key of the
    binning step) equals numpy.histogram2d of the crest positions -- not the
    troughs -- over bins of the stated edge, anchored at the window origin
    minus the bucket margin 2 r, with nbx = floor((nx dx + 2 m) / edge) + 1
    bins per row.  c2 has a window that follows its source (400 steps, splits
    included); c1's patch is static."""
    s = scenes.get(name)
    o = oracle.Oracle(s)
    o.step(steps)
    n = o.n
    P = o.particles()
    pt = s.patches[0]
    dxu = int(round(pt.dx * UNIT))
    wx, wy = o.window(0)
    px, py = crest_positions(o, P, n)
    checked = 0
    for b in range(o.nb):
        sel = P[:, 1] == b
        m = int(math.ceil(2.0 * o.bucket(b)["r"] * UNIT))
        assert m == o.bucket(b)["margin_u"]
        edge = s.bins[b] * dxu
        lox, loy = wx * dxu - m, wy * dxu - m
        nbx = (pt.nx * dxu + 2 * m) // edge + 1
        nby = (pt.ny * dxu + 2 * m) // edge + 1
        assert o.tile_dims(0, b) == (s.bins[b], nbx, nby)
        ex = lox + edge * np.arange(nbx + 1, dtype=np.float64)
        ey = loy + edge * np.arange(nby + 1, dtype=np.float64)
        want, _, _ = np.histogram2d(py[sel].astype(np.float64), px[sel].astype(np.float64), bins=[ey, ex])
        assert want.sum() == sel.sum(), "a crest fell outside the expanded window"
        assert np.array_equal(o.tiles(0, b), want.astype(np.int64)), f"bucket {b}"
        checked += int(sel.sum())
    assert checked == P.shape[0] and checked > 1000


@pytest.mark.parametrize("name,steps", [("c2", 600), ("p0", 600)])
def test_window_follows_source_within_half_cell(name, steps):
    """A patch that follows its source recentres in whole cells every step:
    the window centre anchor + (W + n/2) dx stays within half a cell of the
    source position x0 + v n dt, and moves by at most one cell per step at
    these speeds (below one cell per step).  Stepped one step at a time with
    one particle per group (the windows do not depend on the particles)."""
    s = scenes.get(name)
    s = s.replace(spectrum=dataclasses.replace(s.spectrum, eta=1.0))
    o = oracle.Oracle(s)
    pt, src = s.patches[0], s.sources[0]
    assert pt.follow == 0
    prev = None
    for n in range(1, steps + 1):
        o.step(1)
        wx, wy = o.window(0)
        cx = pt.anchor_x + (wx + pt.nx / 2) * pt.dx
        cy = pt.anchor_y + (wy + pt.ny / 2) * pt.dx
        xs = src.x0 + src.vx * n * s.dt
        ys = src.y0 + src.vy * n * s.dt
        assert abs(cx - xs) <= 0.5 * pt.dx + 1e-9, (n, cx, xs)
        assert abs(cy - ys) <= 0.5 * pt.dx + 1e-9, (n, cy, ys)
        if prev is not None:
            assert abs(wx - prev[0]) <= 1 and abs(wy - prev[1]) <= 1
        prev = (wx, wy)
    # the window really moved
    assert abs(prev[0]) + abs(prev[1]) > 10


def test_ring_origin_is_source_position():
    """Ring particles start on a circle of radius R around the source's
    position at their birth step, x0 + v n dt (anchor-relative, 2^-20 m):
    origin - R (cos, sin)(2 pi j / n_e) is within one unit of it."""
    s = scenes.c2()
    o = oracle.Oracle(s)
    o.step(100)
    P = o.particles()
    ring = P[P[:, 2] == 1]
    pt, src = s.patches[0], s.sources[0]
    assert ring.shape[0] > 64
    for q in ring[::7]:
        n, j = int(q[5]), int(q[9])
        phi = 2 * math.pi * j / src.ring_n
        ex = (src.x0 + src.vx * n * s.dt - pt.anchor_x) * UNIT + src.radius * math.cos(phi) * UNIT
        ey = (src.y0 + src.vy * n * s.dt - pt.anchor_y) * UNIT + src.radius * math.sin(phi) * UNIT
        assert abs(q[6] - ex) <= 1.0 and abs(q[7] - ey) <= 1.0, (q, ex, ey)


def test_loaded_state_continues_like_the_original():
    """A state taken out after step n and loaded into a fresh oracle as the
    state after step n continues exactly as the original: the same
    particles, windows and bin histograms after more steps (c2 with a
    moving window and splits), and the histogram of the loaded step itself
    equals the original's."""
    s = scenes.c2()
    a = oracle.Oracle(s)
    a.step(320)
    b = oracle.Oracle(s)
    b.load(a.n, a.particles())
    assert b.n == a.n and b.window(0) == a.window(0)
    for i in range(a.nb):
        assert np.array_equal(b.tiles(0, i), a.tiles(0, i))
    a.step(25)
    b.step(25)
    key = lambda P: P[np.lexsort(P.T[::-1])]
    assert np.array_equal(key(a.particles()), key(b.particles()))
    for i in range(a.nb):
        assert np.array_equal(b.tiles(0, i), a.tiles(0, i))
    ca, cb = a.counts(0), b.counts(0)
    assert np.array_equal(ca[:, 0], cb[:, 0])
    bad = a.particles()[:1].copy()
    bad[0, 1] = a.nb
    with pytest.raises(oracle.OracleError):
        b.load(b.n, bad)


# ---------------------------------------------------------------- vertical motion (Sec 4.3)
def heave_scene(a=0.1, T=1.5, R=2.0, vx=0.0):
    """One bucket with r = 1 m = 4 cells (lambda 1-4 m), a 32 m patch and a
    disc of radius R at its centre heaving as a sin(2 pi t / T)."""
    sp = scenes.Spectrum(U10=10.0, n_buckets=1, lambda_min=1.0, lambda_max=4.0, eta=1e-6)
    p = scenes.Patch(anchor_x=0.0, anchor_y=0.0, nx=128, ny=128, dx=0.25)
    src = scenes.Source(x0=16.0, y0=16.0, vx=vx, vy=0.0, radius=R, draft=1.0, ring_n=64, patch=0,
                        heave_amp=a, heave_period=T)
    return scenes.Scene(name="heave", fft_n=64, fft_L=256.0, seed=3, steps=0, spectrum=sp,
                        patches=[p], sources=[src], bins=[8])


def test_heave_ring_volume_equals_displaced_volume():
    """Every ring a heaving disc emits carries, in its crests, the volume the
    disc pushed out since the previous ring: sum_j crest volume =
    pi R^2 (z(t - Eh dt) - z(t)).  Each crest volume is measured from the
    particle's own splat through its first moment (crest volume times r
    along its direction, pinned for single pairs), so the identity checks the
    amplitudes against the disc's motion, not against their formula.  (The
    moment is exact when the trough sits a whole number of cells from the
    crest, so each particle is measured with its direction turned to +x,
    which leaves its amplitude unchanged.)"""
    s = heave_scene()
    o = oracle.Oracle(s)
    si = o.source_info(0)
    r = o.bucket(0)["r"]
    c = o.bucket(0)["c"]
    Eh = si["Eh"]
    # cadence: a ring leaves each time the previous one has run half a radius
    assert Eh * c * s.dt <= 0.5 * r < (Eh + 1) * c * s.dt
    src, p = s.sources[0], s.patches[0]
    xc = (np.arange(p.nx) + 0.5) * p.dx
    X, Y = np.meshgrid(xc, xc)
    z = lambda n: src.heave_amp * math.sin(2 * math.pi * n * s.dt / src.heave_period)
    checked = 0
    for k in range(6):
        n = 1 + k * Eh
        o.step(n - o.n)
        P = o.particles()
        ring = P[(P[:, 2] == 2) & (P[:, 5] == n)]
        assert ring.shape[0] == src.ring_n
        vol = 0.0
        for q in ring:
            qx = q.copy()
            qx[4] = 0   # direction +x: the trough r = 4 cells behind the crest along x
            h = o.splat(0, qx[None, :])
            vol += (h * X).sum() * p.dx * p.dx / r
        want = math.pi * src.radius ** 2 * (z(n - Eh) - z(n))
        assert vol == pytest.approx(want, rel=1e-9, abs=1e-12)
        checked += 1
    # only vertical rings from a disc at rest: n_e per emission, ceil(n / Eh) emissions
    assert int(o.counts(0)[0, 2]) == src.ring_n * (1 + (o.n - 1) // Eh)
    assert checked == 6


def test_heave_ring_is_isotropic():
    """A vertical-motion ring is the same in every direction: its field is
    symmetric under the diagonal reflection and both axis reflections about
    the disc centre (a horizontal-motion ring, signed by the heading, is
    not)."""
    s = heave_scene()
    o = oracle.Oracle(s)
    Eh = o.source_info(0)["Eh"]
    o.step(1 + 2 * Eh)
    P = o.particles()
    ring = P[(P[:, 2] == 2) & (P[:, 5] == o.n)]
    h = o.splat(0, ring)
    scale = np.abs(h).max()
    assert scale > 0
    for g in (h.T, h[::-1, :], h[:, ::-1]):
        assert np.max(np.abs(h - g)) <= 1e-9 * scale
    # the horizontal-motion ring of a moving disc is antisymmetric along its heading
    sm = heave_scene(a=0.0, vx=4.0)
    om = oracle.Oracle(sm)
    om.step(1)
    Pm = om.particles()
    hm = om.splat(0, Pm[Pm[:, 2] == 1])
    assert np.max(np.abs(hm - hm[:, ::-1])) > 0.1 * np.abs(hm).max()


def test_heave_rings_subdivide_and_keep_amplitude():
    """Vertical-motion ring particles split like horizontal ones (same ages,
    codes c and c +- a0/3^(L+1)); a complete family's amplitudes sum to the
    parent's (measured through single-particle splats, as above)."""
    s = heave_scene()
    o = oracle.Oracle(s)
    si = o.source_info(0)
    T0 = si["T"][0]
    o.step(T0 + 1)
    P = o.particles()
    kids = P[(P[:, 2] == 2) & (P[:, 5] == 1)]
    assert kids.shape[0] == 3 * 64 and np.all(kids[:, 3] == 1)
    off = si["a0"] // 3
    for j in range(64):
        fam = kids[kids[:, 9] == j]
        assert sorted(int(x) for x in fam[:, 4]) == sorted([(j * si["a0"] + d) % oracle.NCODE for d in (-off, 0, off)])
    # amplitudes of a family: three equal thirds of the parent's, via the splat's peak of an isolated copy
    o2 = oracle.Oracle(s)
    o2.step(1)
    parent = o2.particles()
    parent = parent[(parent[:, 2] == 2) & (parent[:, 9] == 5)][0].copy()
    o3 = oracle.Oracle(s)
    o3.seek(o2.n)
    hp = o3.splat(0, parent[None, :])
    child = parent.copy()
    child[3] = 1
    hc = o3.splat(0, child[None, :])
    assert np.allclose(hc, hp / 3.0, rtol=0, atol=1e-15 * np.abs(hp).max())
