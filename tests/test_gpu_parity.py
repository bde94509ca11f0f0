"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Integer state (per-bucket counts, per-bin histograms and the multiset of
particle records) must be bit-exact; heights within 1e-4 relative RMS,
reported separately for the background, the raw wave-particle map and the
blended map.
"""
import functools
import sys

import numpy as np
import pytest

import oracle
from paper_2511_02852_amd import scenes

pytestmark = pytest.mark.gpu
TOL = 1e-4


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
    sys.stdout.flush()


def rel_rms(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.sqrt(np.mean((a - b) ** 2)) / max(np.sqrt(np.mean(b ** 2)), 1e-300))


def canon(P):
    if P.shape[0] == 0:
        return P
    return P[np.lexsort(P.T[::-1])]


def check_integer_state(g, o, scene):
    for p in range(len(scene.patches)):
        gc = g.counts(p)
        oc = o.counts(p)
        assert np.array_equal(gc[:, :5], oc), f"patch {p} counts\n{gc}\n{oc}"
        assert np.all(gc[:, 5] == 0)
        for b in range(o.nb):
            assert g.tile_dims(p, b) == o.tile_dims(p, b)
            assert np.array_equal(g.tiles(p, b), o.tiles(p, b)), f"patch {p} bucket {b} tiles"
    gp, op = canon(g.particles()), canon(o.particles())
    assert gp.shape == op.shape, (gp.shape, op.shape)
    assert np.array_equal(gp, op), "particle multisets differ"


def check_heights(g, o, scene, patches=None, tol=TOL):
    H = o.background()
    e_bg = rel_rms(g.background(), H)
    out = {"bg": e_bg}
    assert e_bg <= tol, f"background rel rms {e_bg}"
    for p in (range(len(scene.patches)) if patches is None else patches):
        raw, bl = o.patch_maps(p, H)
        e_raw = rel_rms(g.patch_map(p, 1), raw)
        e_bl = rel_rms(g.patch_map(p, 0), bl)
        out[p] = (e_raw, e_bl)
        assert e_raw <= tol, f"patch {p} raw rel rms {e_raw}"
        assert e_bl <= tol, f"patch {p} blended rel rms {e_bl}"
    return out


def make(scene, **kw):
    from paper_2511_02852_amd import hwo
    return hwo.Ocean(scene, **kw), oracle.Oracle(scene)


# ---------------------------------------------------------------- background
@pytest.mark.parametrize("N,L", [(16, 64.0), (64, 256.0), (256, 500.0), (512, 1000.0), (1024, 2000.0),
                                 (2048, 4000.0), (4096, 8000.0)])
def test_background_matches_oracle(N, L):
    s = scenes.Scene(name="bg", fft_n=N, fft_L=L, seed=5, spectrum=scenes.Spectrum(U10=15.0))
    say(f"background N={N}")
    g, o = make(s, torch_memory=True)
    for steps in (1, 36):
        g.step(steps)
        o.step(steps)
        e = rel_rms(g.background(), o.background())
        say(f"  n={o.n} rel_rms={e:.3e}")
        assert e <= TOL


@pytest.mark.parametrize("N,L", [(16, 64.0), (64, 256.0), (512, 1000.0), (2048, 4000.0), (4096, 8000.0)])
def test_background_slope_and_choppy_fields(N, L):
    """The derived background fields (dH/dx, dH/dy, choppy displacement x
    and y) from the same two FFT passes, against the oracle's fields."""
    s = scenes.Scene(name="bgf", fft_n=N, fft_L=L, seed=6, spectrum=scenes.Spectrum(U10=12.0))
    say(f"background fields N={N}")
    from paper_2511_02852_amd import hwo
    g, o = hwo.Ocean(s, bg_fields=True), oracle.Oracle(s)
    g.step(7)
    o.step(7)
    assert rel_rms(g.background(0), o.background()) <= TOL
    for f in (1, 2, 3, 4):
        e = rel_rms(g.background(f), o.background_field(f))
        say(f"  field {f} rel_rms={e:.3e}")
        assert e <= TOL


def test_background_unit_modulus_and_mitsuyasu():
    sp = scenes.Spectrum(U10=7.0, fetch=30e3, gamma=-1.0, spread_s=-1.0, h0_mode=1, wind_dir=0.6)
    s = scenes.Scene(name="bg2", fft_n=256, fft_L=300.0, seed=9, spectrum=sp)
    g, o = make(s)
    g.step(17)
    o.step(17)
    assert rel_rms(g.background(), o.background()) <= TOL


# ---------------------------------------------------------------- c1
def test_c1_every_step():
    s = scenes.c1()
    g, o = make(s)
    for n in range(1, s.steps + 1):
        g.step(1)
        o.step(1)
        check_integer_state(g, o, s)
        e = check_heights(g, o, s)
        say(f"c1 n={n} live={int(g.counts(0)[:, 0].sum())} err={e}")


# ---------------------------------------------------------------- c2 forms
@pytest.mark.parametrize("form", ["plain", "compact", "batched"])
def test_c2_forms(form):
    s = scenes.c2()
    kw = dict(plain=dict(compact=False, batched=False), compact=dict(compact=True, batched=False),
              batched=dict(compact=True, batched=True))[form]
    g, o = make(s, **kw)
    done = 0
    for target in (60, 300, 600):
        g.step(target - done)
        o.step(target - done)
        done = target
        say(f"c2 {form} n={target}")
        check_integer_state(g, o, s)
        if target in (60, 600):
            e = check_heights(g, o, s)
            say(f"  live={int(g.counts(0)[:, 0].sum())} err={e}")


def test_c2_subdivision_happens():
    s = scenes.c2()
    g, o = make(s, compact=True)
    g.step(330)
    o.step(330)
    c = g.counts(0)
    assert c[:, 3].sum() > 0
    check_integer_state(g, o, s)


# ---------------------------------------------------------------- large scenes, short runs
@pytest.mark.parametrize("name,steps", [("c3", 12), ("c5", 6)])
def test_batched_scenes_short(name, steps):
    s = scenes.get(name)
    say(f"{name}: {len(s.patches)} patches, {steps} steps")
    g, o = make(s)
    g.step(steps)
    o.step(steps)
    check_integer_state(g, o, s)
    e = check_heights(g, o, s, patches=[0, 1, len(s.patches) - 1])
    say(f"  err={e}")


def test_paper_default_scene_short():
    """The paper's default parameters with equal-energy buckets (every bucket
    on the matrix-core path, radii 4.7-50 cells), Mitsuyasu spreading and
    fetch-dependent gamma: 40 steps, integer state bit-exact, heights."""
    s = scenes.p0()
    g, o = make(s, compact=True, batched=True)
    # the library's FP64 bucket table equals the oracle's bit for bit
    want = np.array([[o.bucket(i)[k] for k in ("w", "dw", "r", "c")] for i in range(o.nb)])
    assert np.array_equal(g.buckets(), want)
    g.step(40)
    o.step(40)
    check_integer_state(g, o, s)
    e = check_heights(g, o, s)
    say(f"p0 err={e}")


@pytest.mark.parametrize("name,steps,form", [("c1", 30, "plain"), ("c2", 60, "plain"),
                                             ("c2", 60, "batched"), ("p0", 40, "batched")])
def test_stratified_directions(name, steps, form):
    """Stratified boundary directions (a group of N_theta = eta particles
    visits every sector, amplitude from S(w, theta)): integer state bit-exact
    and heights, in the wide and the compact record forms."""
    import dataclasses
    s = scenes.get(name)
    s = s.replace(spectrum=dataclasses.replace(s.spectrum, dir_mode=1, wind_dir=0.7))
    kw = dict(compact=True, batched=True) if form == "batched" else {}
    say(f"stratified {name} {form} {steps} steps")
    g, o = make(s, **kw)
    g.step(steps)
    o.step(steps)
    check_integer_state(g, o, s)
    e = check_heights(g, o, s)
    say(f"stratified {name} {form} err={e}")


@pytest.mark.parametrize("name,steps,form", [("c1", 30, "plain"), ("c2", 60, "plain"),
                                             ("c2", 60, "batched"), ("p0", 40, "batched")])
def test_obliquity_weighted_injection(name, steps, form):
    """Obliquity-weighted boundary injection (per side pair direction tables
    and counts scaled by the mean crossing |cos|): integer state bit-exact and
    heights."""
    import dataclasses
    s = scenes.get(name)
    # obliquity weighting draws directions by inverse CDF (dir_mode 0)
    s = s.replace(spectrum=dataclasses.replace(s.spectrum, flux_mode=1, dir_mode=0, wind_dir=0.4))
    kw = dict(compact=True, batched=True) if form == "batched" else {}
    say(f"obliquity {name} {form} {steps} steps")
    g, o = make(s, **kw)
    g.step(steps)
    o.step(steps)
    check_integer_state(g, o, s)
    e = check_heights(g, o, s)
    say(f"obliquity {name} {form} err={e}")


def test_c4_far_anchor():
    s = scenes.c4()
    g, o = make(s)
    g.step(90)
    o.step(90)
    check_integer_state(g, o, s)
    e = check_heights(g, o, s)
    say(f"c4 err={e}")


@pytest.mark.parametrize("name,frames", [("c3", 900), ("c5", 900), ("p0", 1200)])
def test_full_size_state(name, frames):
    """The benchmark's state: frame 900 of the batched scenes in the timed
    launch configuration (16-byte records, one launch per stage, graph
    replay).  Identities that hold at any size are checked exactly; heights of
    sampled patches against the oracle evaluated on the GPU's own particles at
    that step, and the whole background."""
    from paper_2511_02852_amd import hwo
    s = scenes.get(name)
    npch, nb = len(s.patches), s.spectrum.n_buckets
    say(f"{name}: {npch} patches, {frames} frames (batched, 16-byte records, graph)")
    g = hwo.Ocean(s, compact=True, batched=True)
    done = 0
    while done < frames:
        k = min(100, frames - done)
        g.step(k)
        done += k
    g.sync()
    P = g.particles()
    say(f"  {P.shape[0]} live particles")
    live = np.zeros((npch, nb), dtype=np.int64)
    for p in range(npch):
        c = g.counts(p)
        assert np.all(c[:, 5] == 0), f"patch {p}: dropped particles"
        # every subdivision replaces one particle by three
        assert np.array_equal(c[:, 0], c[:, 1] + c[:, 2] + 2 * c[:, 3] - c[:, 4]), f"patch {p} conservation"
        for b in range(nb):
            assert int(g.tiles(p, b).sum()) == int(c[b, 0]), f"patch {p} bucket {b} histogram"
        live[p] = c[:, 0]
    # the particle records: multiplicity per (patch, bucket) and field ranges
    assert np.array_equal(np.bincount(P[:, 0] * nb + P[:, 1], minlength=npch * nb).reshape(npch, nb), live)
    kind, level, code, birth, src = P[:, 2], P[:, 3], P[:, 4], P[:, 5], P[:, 8]
    assert np.all((kind == 0) | (kind == 1))
    assert np.all((code >= 0) & (code < 10368))
    assert np.all((birth >= 1) & (birth <= frames))
    assert np.all(level[kind == 0] == 0) and np.all(src[kind == 0] == -1)
    assert np.all((level[kind == 1] <= s.spectrum.max_level) & (src[kind == 1] >= 0))
    # heights
    o = oracle.Oracle(s)
    o.seek(frames)
    H = o.background()
    e_bg = rel_rms(g.background(), H)
    assert e_bg <= TOL, f"background rel rms {e_bg}"
    errs = {}
    for p in sorted({0, npch // 2, npch - 1}):
        raw = o.splat(p, P[P[:, 0] == p])
        e_raw = rel_rms(g.patch_map(p, 1), raw)
        e_bl = rel_rms(g.patch_map(p, 0), o.blend(p, H, raw))
        errs[p] = (e_raw, e_bl)
        assert e_raw <= TOL, f"patch {p} raw rel rms {e_raw}"
        assert e_bl <= TOL, f"patch {p} blended rel rms {e_bl}"
    say(f"  bg={e_bg:.2e} patches={errs}")


# ---------------------------------------------------------------- splat pins on the GPU
def pin_scene():
    sp = scenes.Spectrum(U10=10.0, n_buckets=1, lambda_min=1.0, lambda_max=4.0, eta=4.0)
    return scenes.Scene(name="pin", fft_n=64, fft_L=256.0, seed=3, spectrum=sp,
                        patches=[scenes.Patch(anchor_x=0.0, anchor_y=0.0, nx=96, ny=80, dx=0.25)],
                        bins=[8])


@pytest.mark.parametrize("compact", [False, True])
def test_gpu_pair_lattice_cosine(compact):
    """Particles at spacing lambda along +x and r across sum to A cos(k(x - x0))."""
    from paper_2511_02852_amd import hwo
    s = pin_scene()
    g = hwo.Ocean(s, compact=compact)
    o = oracle.Oracle(s)
    g.step(1)
    r, lam = o.bucket(0)["r"], o.bucket(0)["lam"]
    A = o.patch_bucket(0, 0)["A"]
    x0 = 3.3
    recs = []
    for m in range(-3, 16):
        for k in range(-3, 28):
            recs.append([0, 0, 0, 0, 0, 1, int(round((x0 + m * lam) * 2 ** 20)), int(round((0.1 + k * r) * 2 ** 20)),
                         -1, 0])
    h = g.test_splat(0, np.array(recs))
    p = s.patches[0]
    X = (np.arange(p.nx) + 0.5) * p.dx
    want = A * np.cos(np.pi * (X - round(x0 * 2 ** 20) / 2 ** 20) / r)
    err = np.max(np.abs(h - want[None, :]))
    assert err <= 2e-5 * A, err


def use_schedule(g, splat_kernel):
    """Select the splat schedule (0 batches per wavefront, 1 a quadrant per
    wavefront, 2 the hybrid default) on a built ocean."""
    p = g.get_plan()
    p["splat_kernel"] = splat_kernel
    g.set_plan(**p)


@pytest.mark.parametrize("compact,splat_kernel", [(False, 2), (True, 0), (True, 1), (True, 2)])
def test_gpu_splat_random_particles(compact, splat_kernel):
    """Hand-placed boundary and ring particles of every bucket, c2 geometry,
    through both splat schedules."""
    from paper_2511_02852_amd import hwo
    s = scenes.c2()
    g = hwo.Ocean(s, compact=compact)
    o = oracle.Oracle(s)
    g.step(1)
    o.step(1)
    use_schedule(g, splat_kernel)
    wx, wy = o.window(0)
    rng = np.random.default_rng(4)
    dxu = int(0.25 * 2 ** 20)
    recs = []
    for k in range(3000):
        b = int(rng.integers(0, 8))
        kind = int(rng.random() < 0.3)
        si = o.source_info(0)
        if kind:
            b = si["bucket"]
        level = int(rng.integers(0, 3)) if kind else 0
        x = int((wx + rng.uniform(-10, 266)) * dxu)
        y = int((wy + rng.uniform(-10, 266)) * dxu)
        code = int(rng.integers(0, 10368))
        birth = int(rng.integers(0, 2))
        recs.append([0, b, kind, level, code, birth, x, y, 0 if kind else -1, int(rng.integers(0, 64)) if kind else 0])
    recs = np.array(recs)
    h = g.test_splat(0, recs)
    ref = o.splat(0, recs)
    e = rel_rms(h, ref)
    say(f"splat random rel rms {e:.2e}")
    assert e <= 1e-5


@functools.lru_cache(maxsize=1)
def _subcell_case():
    """Records and the oracle's raw map of patch 0 after one step of the
    64-patch stress scene (shared by the three schedules)."""
    s = scenes.c5()
    o = oracle.Oracle(s)
    o.step(1)
    wx, wy = o.window(0)
    pt = s.patches[0]
    rng = np.random.default_rng(11)
    dxu = int(pt.dx * 2 ** 20)
    recs = []
    for k in range(4000):
        # most particles in the four smallest buckets, the rest anywhere
        b = int(rng.integers(0, 4)) if rng.random() < 0.6 else int(rng.integers(0, 16))
        x = int((wx + rng.uniform(-10, pt.nx + 10)) * dxu)
        y = int((wy + rng.uniform(-10, pt.ny + 10)) * dxu)
        code = int(rng.integers(0, 10368))
        birth = int(rng.integers(0, 2))
        recs.append([0, b, 0, 0, code, birth, x, y, -1, 0])
    recs = np.array(recs)
    return s, recs, o.splat(0, recs)


@pytest.mark.parametrize("splat_kernel", [0, 1, 2])
def test_gpu_splat_random_particles_subcell_radii(splat_kernel):
    """Boundary particles of every bucket of the 64-patch stress geometry,
    whose two smallest buckets have radii under one cell (footprints of at
    most two cells per axis: the short loops of the small-footprint path),
    hand-placed over one patch and its margins, through the three splat
    schedules."""
    from paper_2511_02852_amd import hwo
    s, recs, ref = _subcell_case()
    g = hwo.Ocean(s, compact=True)
    g.step(1)
    use_schedule(g, splat_kernel)
    h = g.test_splat(0, recs)
    e = rel_rms(h, ref)
    say(f"splat sub-cell radii (schedule {splat_kernel}) rel rms {e:.2e}")
    assert e <= 1e-5


@pytest.mark.parametrize("synth,splat_kernel", [(0, 0), (0, 1), (0, 2), (1, 2)])
def test_splat_of_no_records_is_zero(synth, splat_kernel):
    """An empty record list splats to an all-zero map, in every splat
    schedule and through the texel layers."""
    from paper_2511_02852_amd import hwo
    s = scenes.c2().replace(synth=synth)
    g = hwo.Ocean(s, compact=True)
    g.step(1)
    use_schedule(g, splat_kernel)
    h = g.test_splat(0, np.zeros((0, 10), dtype=np.int64))
    assert h.shape == (s.patches[0].ny, s.patches[0].nx)
    assert not np.any(h)


@pytest.mark.parametrize("compact", [False, True])
def test_gpu_texel_layers_random_particles(compact):
    """The texel-layer synthesis through the test hook: hand-placed boundary
    and ring particles of every bucket (inside and up to 10 cells outside the
    patch), c2 geometry, against the oracle's layer synthesis."""
    from paper_2511_02852_amd import hwo
    s = scenes.c2().replace(synth=1)
    g = hwo.Ocean(s, compact=compact)
    o = oracle.Oracle(s)
    g.step(1)
    o.step(1)
    wx, wy = o.window(0)
    rng = np.random.default_rng(5)
    dxu = int(0.25 * 2 ** 20)
    si = o.source_info(0)
    recs = []
    for k in range(3000):
        kind = int(rng.random() < 0.3)
        b = si["bucket"] if kind else int(rng.integers(0, 8))
        level = int(rng.integers(0, 3)) if kind else 0
        x = int((wx + rng.uniform(-10, 266)) * dxu)
        y = int((wy + rng.uniform(-10, 266)) * dxu)
        code = int(rng.integers(0, 10368))
        birth = int(rng.integers(0, 2))
        recs.append([0, b, kind, level, code, birth, x, y, 0 if kind else -1, int(rng.integers(0, 64)) if kind else 0])
    recs = np.array(recs)
    say(f"texel layers random particles compact={compact}")
    h = g.test_splat(0, recs)
    ref = o.splat(0, recs)
    e = rel_rms(h, ref)
    say(f"texel random rel rms {e:.2e}")
    assert e <= 1e-5


@pytest.mark.parametrize("compact,splat_kernel", [(False, 2), (True, 0), (True, 1), (True, 2)])
def test_gpu_radial_kernel_random_particles(compact, splat_kernel):
    """The radial kernel W(|d|) through the test hook: hand-placed boundary
    and ring particles of every bucket (small footprints one point per lane,
    large ones one point per wavefront), c2 geometry, against the oracle,
    through both splat schedules."""
    from paper_2511_02852_amd import hwo
    s = scenes.c2().replace(kernel=1)
    g = hwo.Ocean(s, compact=compact)
    o = oracle.Oracle(s)
    g.step(1)
    o.step(1)
    use_schedule(g, splat_kernel)
    wx, wy = o.window(0)
    rng = np.random.default_rng(6)
    dxu = int(0.25 * 2 ** 20)
    si = o.source_info(0)
    recs = []
    for k in range(3000):
        kind = int(rng.random() < 0.3)
        b = si["bucket"] if kind else int(rng.integers(0, 8))
        level = int(rng.integers(0, 3)) if kind else 0
        x = int((wx + rng.uniform(-10, 266)) * dxu)
        y = int((wy + rng.uniform(-10, 266)) * dxu)
        code = int(rng.integers(0, 10368))
        birth = int(rng.integers(0, 2))
        recs.append([0, b, kind, level, code, birth, x, y, 0 if kind else -1, int(rng.integers(0, 64)) if kind else 0])
    recs = np.array(recs)
    say(f"radial kernel random particles compact={compact}")
    h = g.test_splat(0, recs)
    ref = o.splat(0, recs)
    e = rel_rms(h, ref)
    say(f"radial random rel rms {e:.2e}")
    assert e <= 1e-5


@pytest.mark.parametrize("name,steps,kernel,schedule", [("c2", 60, 0, 0), ("p0", 40, 0, 0), ("c3", 12, 0, 0),
                                                        ("c5", 6, 0, 0), ("c2", 60, 1, 0), ("c2", 60, 0, 1),
                                                        ("p0", 40, 0, 1), ("c3", 12, 0, 1), ("c2", 60, 1, 1),
                                                        ("p0", 40, 1, 1)])
def test_other_schedule_scenes(name, steps, kernel, schedule):
    """The batch-per-wavefront splat schedule (0) and the quadrant-per-
    wavefront one (1) in the batched form (both crest/trough kernels):
    integer state bit-exact and heights against the oracle, as for the
    default hybrid schedule (2) that every other test runs."""
    s = scenes.get(name).replace(kernel=kernel)
    say(f"schedule {schedule} {name} kernel={kernel} {steps} steps")
    g, o = make(s, compact=True, batched=True)
    use_schedule(g, schedule)
    g.step(steps)
    o.step(steps)
    check_integer_state(g, o, s)
    e = check_heights(g, o, s, patches=[0, 1, len(s.patches) - 1] if len(s.patches) > 3 else None)
    say(f"schedule {schedule} {name} kernel={kernel} err={e}")


@pytest.mark.parametrize("name,steps,form", [("c1", 30, "plain"), ("c2", 60, "batched"),
                                             ("p0", 40, "batched"), ("c3", 12, "batched")])
def test_radial_kernel_scenes(name, steps, form):
    """Scenes with the radial kernel: integer state bit-exact (the kernel
    shape touches heights only) and heights against the oracle."""
    s = scenes.get(name).replace(kernel=1)
    kw = dict(compact=True, batched=True) if form == "batched" else {}
    say(f"radial kernel {name} {form} {steps} steps")
    g, o = make(s, **kw)
    g.step(steps)
    o.step(steps)
    check_integer_state(g, o, s)
    e = check_heights(g, o, s)
    say(f"radial kernel {name} {form} err={e}")


@pytest.mark.parametrize("name,steps,form", [("c1", 30, "plain"), ("c2", 60, "plain"),
                                             ("c2", 60, "batched"), ("p0", 40, "batched"),
                                             ("c3", 12, "batched"), ("c3", 12, "plain")])
def test_texel_layer_synthesis(name, steps, form):
    """Scenes through the texel layers (deposit, x pass, y pass, layer sum,
    blend): integer state bit-exact and heights against the oracle's layer
    synthesis."""
    s = scenes.get(name).replace(synth=1)
    kw = dict(compact=True, batched=True) if form == "batched" else {}
    say(f"texel layers {name} {form} {steps} steps")
    g, o = make(s, **kw)
    g.step(steps)
    o.step(steps)
    check_integer_state(g, o, s)
    e = check_heights(g, o, s)
    say(f"texel layers {name} {form} err={e}")


@pytest.mark.parametrize("name,steps,form,synth", [("c1", 20, "plain", 0), ("c2", 60, "batched", 0),
                                                   ("p0", 40, "batched", 1), ("c3", 12, "batched", 0)])
def test_finite_difference_normals(name, steps, form, synth):
    """Normals of the blended maps by finite differences (Sec 4.2), computed
    on the GPU every frame, against the oracle's normals of its own blended
    map: x and y components within the height tolerance (relative RMS), z
    likewise, every normal of unit length."""
    from paper_2511_02852_amd import hwo
    s = scenes.get(name).replace(synth=synth)
    kw = dict(compact=True, batched=True) if form == "batched" else {}
    say(f"normals {name} {form} synth={synth}")
    g = hwo.Ocean(s, normals=True, **kw)
    o = oracle.Oracle(s)
    g.step(steps)
    o.step(steps)
    H = o.background()
    for p in range(len(s.patches)):
        _, bl = o.patch_maps(p, H)
        want = o.normals(p, bl)
        got = g.normals(p)
        errs = [rel_rms(got[c], want[c]) for c in range(3)]
        say(f"normals {name} patch {p} rel rms {errs}")
        assert max(errs) <= TOL
        assert np.max(np.abs(np.sum(got.astype(np.float64) ** 2, axis=0) - 1.0)) <= 1e-5


@pytest.mark.parametrize("name,steps,form,synth", [("c2", 60, "batched", 0), ("c3", 12, "batched", 0),
                                                   ("p0", 40, "batched", 1)])
def test_probe_sampling(name, steps, form, synth):
    """Object-receives-water sampling at probe points: inside patches (the
    blended map) and outside (the background), against the oracle sampling
    its own maps; heights and normals within the height tolerance."""
    from paper_2511_02852_amd import hwo
    s = scenes.get(name).replace(synth=synth)
    g = hwo.Ocean(s, compact=True, batched=True)
    o = oracle.Oracle(s)
    g.step(steps)
    o.step(steps)
    rng = np.random.default_rng(9)
    pts = []
    for p, P in enumerate(s.patches[:4]):
        wx, wy = o.window(p)
        x0, y0 = P.anchor_x + wx * P.dx, P.anchor_y + wy * P.dx
        pts.append(np.column_stack([rng.uniform(x0 - 5, x0 + P.nx * P.dx + 5, 200),
                                    rng.uniform(y0 - 5, y0 + P.ny * P.dx + 5, 200)]))
    pts.append(rng.uniform(0, s.fft_L, (200, 2)))
    pts = np.concatenate(pts)
    say(f"probes {name}: {pts.shape[0]} points")
    got = g.sample_probes(pts)
    want = o.sample_probes(pts)
    for c in range(4):
        e = rel_rms(got[:, c], want[:, c])
        say(f"  component {c} rel rms {e:.2e}")
        assert e <= TOL


@pytest.mark.parametrize("name,form,synth", [("c2", "batched", 0), ("c3", "plain", 0), ("p0", "batched", 1)])
def test_snapshot_and_resume(name, form, synth):
    """Checkpoint / resume: k steps, snapshot, n - k more steps must equal a
    fresh handle restored from the snapshot and stepped n - k times, and the
    original handle restored and stepped again: integer state bit for bit,
    heights up to FP32 summation order.  A snapshot of another scene is
    refused."""
    from paper_2511_02852_amd import hwo
    s = scenes.get(name).replace(synth=synth)
    kw = dict(compact=True, batched=True) if form == "batched" else dict(compact=False, batched=False)
    say(f"snapshot {name} {form} synth={synth}")
    a = hwo.Ocean(s, **kw)
    a.step(40)
    img = a.snapshot()
    a.step(25)
    a.sync()
    want_c = [a.counts(p) for p in range(len(s.patches))]
    want_p = canon(a.particles())
    want_h = [a.patch_map(p, 0) for p in range(len(s.patches))]
    want_bg = a.background()
    for g in (hwo.Ocean(s, **kw), a):
        g.restore(img)
        assert g.n == 40
        g.step(25)
        g.sync()
        for p in range(len(s.patches)):
            assert np.array_equal(g.counts(p), want_c[p])
            assert rel_rms(g.patch_map(p, 0), want_h[p]) <= 1e-6
        assert np.array_equal(canon(g.particles()), want_p)
        assert np.array_equal(g.background(), want_bg)
    other = hwo.Ocean(scenes.c1(), **kw)
    other.step(1)
    with pytest.raises(hwo.HwoError):
        other.restore(img)


def test_restore_sets_the_windows_of_the_restored_step():
    """A fresh handle restored from a snapshot of a moving-window scene (c2)
    evaluates test splats in the windows of the restored step before any
    further step: the same records splat to the same map as on the handle
    the snapshot was taken from."""
    from paper_2511_02852_amd import hwo
    s = scenes.c2()
    a = hwo.Ocean(s, compact=True, batched=True)
    a.step(40)
    img = a.snapshot()
    P = a.particles()
    recs = P[np.random.default_rng(5).choice(P.shape[0], 2000, replace=False)]
    want = a.test_splat(0, recs)
    b = hwo.Ocean(s, compact=True, batched=True)
    b.restore(img)
    got = b.test_splat(0, recs)
    assert np.abs(want).max() > 0
    assert rel_rms(got, want) <= 1e-6


@pytest.mark.parametrize("name,synth", [("c2", 0), ("c3", 0), ("p0", 1)])
def test_repeated_runs_agree(name, synth):
    """Race check: LDS atomics, wavefront-aggregated counters and the
    timing-driven splat partition change the order of work between runs, so
    two identical runs must agree bit for bit on every integer (counts, bins,
    particle records) and on heights up to FP32 summation order."""
    from paper_2511_02852_amd import hwo
    s = scenes.get(name).replace(synth=synth)
    runs = []
    for _ in range(2):
        g = hwo.Ocean(s, compact=True, batched=True)
        g.step(50)
        g.sync()
        runs.append((g, canon(g.particles())))
    (g0, p0), (g1, p1) = runs
    assert np.array_equal(p0, p1)
    for p in range(len(s.patches)):
        assert np.array_equal(g0.counts(p), g1.counts(p))
        for b in range(s.spectrum.n_buckets):
            assert np.array_equal(g0.tiles(p, b), g1.tiles(p, b))
        assert rel_rms(g0.patch_map(p, 0), g1.patch_map(p, 0)) <= 1e-6
    assert np.array_equal(g0.background(), g1.background())


# ---------------------------------------------------------------- edge cases
def test_capacity_overflow_reported():
    """More live particles than capacity: records beyond it are dropped,
    the drop is counted and reported, nothing is written out of bounds."""
    from paper_2511_02852_amd import hwo
    s = scenes.c1()
    g = hwo.Ocean(s, max_particles=500)
    g.step(16)
    with pytest.raises(hwo.HwoError) as ei:
        g.counts(0)
    assert ei.value.code == hwo.HWO_EOVERFLOW
    c = g.counts(0, allow_overflow=True)
    assert c[0, 5] > 0
    assert g.particles().shape[0] == 500
    # the first step fits, so its counts are exact
    g1, o1 = make(s)
    g1.step(1)
    o1.step(1)
    check_integer_state(g1, o1, s)


def test_patch_plus_margin_beyond_32_bit_offsets_rejected():
    """The splat forms a particle's offset from its tile in 32 bits, which is
    exact while a patch side plus a bucket's survival margin stays below 2^31
    position units; a scene beyond that (a 1280 m patch with 700-900 m waves)
    is rejected at its first step, and a slightly smaller patch is not."""
    from paper_2511_02852_amd import hwo
    sp = scenes.Spectrum(U10=15.0, n_buckets=1, lambda_min=700.0, lambda_max=900.0)
    big = scenes.Scene(name="wide", fft_n=16, fft_L=4096.0, dt=0.01, spectrum=sp,
                       patches=[scenes.Patch(anchor_x=0.0, anchor_y=0.0, nx=4096, ny=64, dx=0.3125)],
                       bins=[2048])
    with pytest.raises(hwo.HwoError) as ei:
        g = hwo.Ocean(big)
        g.step(1)
    assert ei.value.code == hwo.HWO_EINVAL
    ok = big.replace(patches=[scenes.Patch(anchor_x=0.0, anchor_y=0.0, nx=3072, ny=64, dx=0.3125)])
    g = hwo.Ocean(ok)
    g.step(1)
    g.close()


def test_empty_scene_and_zero_steps():
    from paper_2511_02852_amd import hwo
    s = scenes.Scene(name="empty", fft_n=32, fft_L=100.0, seed=1, spectrum=scenes.Spectrum(n_buckets=2))
    g = hwo.Ocean(s)
    g.step(0)
    assert g.particles().shape[0] == 0
    g.step(3)
    o = oracle.Oracle(s)
    o.step(3)
    assert rel_rms(g.background(), o.background()) <= TOL
    # batched form without patches: the graph, stage timing and the derived
    # background fields still work (no particle or splat launch is made)
    gb = hwo.Ocean(s, compact=True, batched=True, bg_fields=True)
    gb.step(3)
    for stage in ("fft_a", "fft_b", "splat", "splat_plan", "splat_reduce"):
        assert gb.time_stage(stage, 2) >= 0.0
    assert rel_rms(gb.background(), o.background()) <= TOL
    assert rel_rms(gb.background(3), o.background_field(3)) <= TOL


def test_static_source_outside_patch_emits_dead_particles():
    """A ring emitted outside its patch window dies at once (counted)."""
    s = scenes.c1()
    s.sources = [scenes.Source(x0=300.0, y0=300.0, vx=3.0, vy=0.0, radius=1.0, ring_n=32, patch=0)]
    g, o = make(s)
    g.step(10)
    o.step(10)
    check_integer_state(g, o, s)
    assert o.counts(0)[:, 4].sum() > 0


def test_splat_profile_accounts_every_bucket():
    """The splat's per-bucket profile: every live particle's crest and
    trough are visited by at least one tile (points >= 2 x live per bucket),
    buckets with particles take time, and profiling changes no integer
    state (the oracle's after the same steps)."""
    from paper_2511_02852_amd import hwo
    s = scenes.c2()
    g, o = make(s, compact=True, batched=True)
    g.step(100)
    live0 = g.counts(0)[:, 0]
    g.set_splat_profile(True)
    g.step(20)
    g.sync()
    prof = g.splat_profile()
    g.set_splat_profile(False)
    o.step(120)
    check_integer_state(g, o, s)
    live = g.counts(0)[:, 0]
    say(f"profile points={prof['points'].tolist()} live={live.tolist()}")
    # each of the 20 frames visits every live particle at least once (live
    # counts move by a few percent over 20 frames)
    assert np.all(prof["points"] >= 2 * 20 * np.minimum(live0, live) * 0.95)
    assert np.all(prof["bucket"][live > 0] > 0)
    assert prof["decode"] > 0 and prof["setup"] > 0 and prof["epilogue"] > 0
    # off: nothing more accumulates
    before = g.splat_profile()
    g.step(3)
    g.sync()
    after = g.splat_profile()
    assert np.array_equal(before["points"], after["points"])


# ---------------------------------------------------------------- vertical motion (Sec 4.3)
def heave_scene_gpu():
    """Two patches: one follows a disc that moves and heaves (horizontal and
    vertical rings), one holds a disc at rest that only heaves."""
    s = scenes.c2()
    src0 = scenes.Source(x0=500.0, y0=500.0, vx=5.0, vy=2.0, radius=4.0, draft=1.0, ring_n=64, patch=0,
                         heave_amp=0.3, heave_period=2.5)
    src1 = scenes.Source(x0=700.0, y0=520.0, vx=0.0, vy=0.0, radius=3.0, draft=1.0, ring_n=32, patch=1,
                         heave_amp=0.5, heave_period=1.7)
    p0 = scenes.Patch(anchor_x=500.0, anchor_y=500.0, nx=192, ny=160, dx=0.25, follow=0)
    p1 = scenes.Patch(anchor_x=680.0, anchor_y=500.0, nx=160, ny=160, dx=0.25, follow=-1)
    return s.replace(name="heave", patches=[p0, p1], sources=[src0, src1], steps=400)


@pytest.mark.parametrize("form", ["plain", "compact", "batched"])
def test_vertical_motion_rings(form):
    """Rings of heaving discs (isotropic, amplitude from the displaced
    volume) and their subdivisions: integer state bit-exact and heights
    against the oracle over 400 steps, past the first split ages."""
    s = heave_scene_gpu()
    kw = dict(plain=dict(compact=False, batched=False), compact=dict(compact=True, batched=False),
              batched=dict(compact=True, batched=True))[form]
    g, o = make(s, **kw)
    done = 0
    for target in (37, 400):
        g.step(target - done)
        o.step(target - done)
        done = target
        check_integer_state(g, o, s)
        e = check_heights(g, o, s)
        P = o.particles()
        say(f"heave {form} n={target} heave particles={int((P[:, 2] == 2).sum())} "
            f"split={int((P[(P[:, 2] == 2), 3] > 0).sum())} err={e}")
    P = o.particles()
    assert (P[:, 2] == 2).sum() > 0 and (P[(P[:, 2] == 2), 3] > 0).sum() > 0


@pytest.mark.parametrize("N,L", [(1024, 2000.0), (2048, 4000.0), (4096, 8000.0)])
def test_background_radix16_matrix_core_stage(N, L):
    """The optional radix-16 first FFT stage on the matrix cores (split bf16
    operands, FP32 accumulation): the background within the height tolerance
    of the oracle (its error is reported next to that of the FP32 stages),
    and both passes timed back to back for the keep/drop comparison."""
    from paper_2511_02852_amd import hwo
    s = scenes.Scene(name="bg16", fft_n=N, fft_L=L, seed=5, spectrum=scenes.Spectrum(U10=15.0))
    o = oracle.Oracle(s)
    res = {}
    for m16 in (False, True):
        g = hwo.Ocean(s, fft_mfma16=m16)
        g.step(23)
        if m16:
            o.step(23)
        H = o.background() if m16 else None
        res[m16] = (g.background(), g.time_stage("fft_a", 20), g.time_stage("fft_b", 20))
        g.close()
    H = o.background()
    e32, e16 = rel_rms(res[False][0], H), rel_rms(res[True][0], H)
    say(f"N={N}: FP32 stages err {e32:.2e} pass A {res[False][1] * 1e3:.1f} us pass B {res[False][2] * 1e3:.1f} us; "
        f"matrix-core radix 16 err {e16:.2e} pass A {res[True][1] * 1e3:.1f} us pass B {res[True][2] * 1e3:.1f} us")
    assert e32 <= TOL and e16 <= TOL
