"""Seeded synthetic scenes for the hybrid ocean (inputs only).

This module draws the *inputs* of a run -- spectrum parameters, patch
geometry, moving sources -- and nothing else.  It holds none of the
method's arithmetic: no spectrum, no bucket table, no injection rate and no
particle state is computed here.  Both the GPU library binding and the CPU
oracle wrapper consume the same :class:`Scene` object, so the two always see
identical inputs.

The paper evaluates in a Unity scene with assets that are not available; it
uses no public dataset.  The five scenes below stand in for its workloads at
the sizes named in the measurement plan: FFT background grids from 64^2 to
4096^2, one to 64 wave-particle patches of 64^2 to 1024^2 cells, 4 to 16
frequency buckets, and moving disc sources (ship-like) that the patches
follow.  Scene randomness (patch sizes, headings, speeds, per-patch particle
density) is drawn from ``numpy.random.default_rng(seed)``; the method's own
random draws (boundary injection, h0 noise) use Philox4x64-10 on each side.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


@dataclass
class Spectrum:
    """Spectral parameters shared by the FFT background and the particles.

    U10, fetch: wind speed at 10 m (m/s) and fetch (m) of the JONSWAP model.
    gamma: peak enhancement; <= 0 selects the fetch-dependent parameterisation.
    spread_s: cos-2s spreading exponent; < 0 selects the Mitsuyasu s(omega).
    wind_dir: wind direction in radians from +x.
    n_buckets, lambda_min, lambda_max: log-spaced wavelength buckets (m).
    eta: particles per injected group (the paper's N_theta, may be fractional).
    max_level: maximum subdivision level of source particles (<= 4).
    subdiv_frac: split when neighbour spacing exceeds subdiv_frac * radius.
    h0_mode: 0 Gaussian h0 amplitudes, 1 unit-modulus (deterministic variance).
    bucket_mode: 0 log-spaced wavelength buckets over [lambda_min, lambda_max];
      1 equal-energy buckets over [0.5 w_p, 2.5 w_p] (the lambda range is unused).
    dir_mode: 0 directions by inverse CDF of Dir, equal amplitudes; 1 stratified
      groups of eta (= N_theta, a whole number) directions, amplitude from S(w, theta).
    flux_mode: 0 each side pair injects the group count of Eq 18; 1 obliquity-weighted:
      the count is scaled by the mean |cos| of the crossing angle and directions are
      drawn from Dir |cos| (needs dir_mode 0).
    """
    U10: float = 10.0
    fetch: float = 100e3
    gamma: float = 3.3
    spread_s: float = 8.0
    wind_dir: float = 0.0
    n_buckets: int = 4
    lambda_min: float = 1.0
    lambda_max: float = 16.0
    eta: float = 16.0
    max_level: int = 4
    subdiv_frac: float = 0.5
    h0_mode: int = 0
    bucket_mode: int = 0
    dir_mode: int = 0
    flux_mode: int = 0


@dataclass
class Patch:
    """A rectangular wave-particle patch of nx*ny cells of size dx (m).

    anchor_x/anchor_y: world position (m, FP64) of the patch frame origin.
    follow: index of the source whose position recentres the window each
    step, or -1 for a static window.  eta <= 0 inherits the spectrum's eta;
    blend_band <= 0 selects the default blend band.
    """
    anchor_x: float
    anchor_y: float
    nx: int
    ny: int
    dx: float
    eta: float = 0.0
    blend_band: float = 0.0
    follow: int = -1


@dataclass
class Source:
    """A moving disc (ship-like) that emits rings of wave particles.

    (x0, y0): world start position (m); (vx, vy): constant velocity (m/s);
    radius, draft: disc radius and draft (m); ring_n particles per ring;
    patch: index of the patch that receives the emitted particles;
    heave_amp, heave_period: vertical motion z(t) = heave_amp sin(2 pi t /
    heave_period) (m, s); 0 amplitude: no vertical motion.
    """
    x0: float
    y0: float
    vx: float
    vy: float
    radius: float = 5.0
    draft: float = 1.0
    ring_n: int = 64
    patch: int = 0
    heave_amp: float = 0.0
    heave_period: float = 0.0


@dataclass
class Scene:
    name: str
    fft_n: int
    fft_L: float
    g: float = 9.81
    dt: float = 1.0 / 60.0
    seed: int = 0
    steps: int = 16
    spectrum: Spectrum = field(default_factory=Spectrum)
    patches: List[Patch] = field(default_factory=list)
    sources: List[Source] = field(default_factory=list)
    # per-bucket particle bin edge in cells (None: the library's choice)
    bins: Optional[List[int]] = None
    # record form and launch form
    compact: bool = False
    batched: bool = False
    # height synthesis: 0 exact-position splat, 1 texel layers + separable passes
    synth: int = 0
    # crest/trough kernel shape: 0 separable w(dx) w(dy), 1 radial W(|d|) (synth 0 only)
    kernel: int = 0

    def replace(self, **kw) -> "Scene":
        return dataclasses.replace(self, **kw)

    def with_steps(self, steps: int) -> "Scene":
        return dataclasses.replace(self, steps=int(steps))


def default_bins(n_buckets: int, lambda_min: float, lambda_max: float, dx: float) -> List[int]:
    """A geometric bin-edge guess per bucket (cells), larger for long waves.

    Only a partition of the patch for counting and gathering; it changes no
    height and no count other than the per-bin histogram.
    """
    out = []
    for i in range(n_buckets):
        lam = lambda_min * (lambda_max / lambda_min) ** ((i + 0.5) / n_buckets)
        cells = lam / dx  # roughly two radii
        b = 8
        while b < cells and b < 32:
            b *= 2
        out.append(b)
    return out


# --------------------------------------------------------------------------
# The five workloads.

def c1() -> Scene:
    """Plain method, tiny: FFT 64^2 over 256 m, one static 64^2 patch."""
    sp = Spectrum(U10=10.0, fetch=100e3, gamma=3.3, spread_s=8.0, wind_dir=0.0,
                  n_buckets=4, lambda_min=1.0, lambda_max=16.0, eta=16.0)
    return Scene(name="c1-tiny", fft_n=64, fft_L=256.0, seed=0, steps=16, spectrum=sp,
                 patches=[Patch(anchor_x=112.0, anchor_y=112.0, nx=64, ny=64, dx=0.5)],
                 sources=[], bins=[8, 8, 16, 16])


def c2() -> Scene:
    """Single 256^2 patch at 0.25 m following one ship-like source, FFT 512^2.

    eta = 34 particles per group keeps about 200k live particles at frame 600
    (the window moves at 8 m/s, so slow short waves leave it early)."""
    sp = Spectrum(U10=15.0, fetch=100e3, gamma=3.3, spread_s=8.0, wind_dir=0.0,
                  n_buckets=8, lambda_min=0.5, lambda_max=32.0, eta=34.0)
    h = math.radians(45.0)
    src = Source(x0=500.0, y0=500.0, vx=8.0 * math.cos(h), vy=8.0 * math.sin(h),
                 radius=5.0, draft=1.0, ring_n=64, patch=0)
    p = Patch(anchor_x=500.0, anchor_y=500.0, nx=256, ny=256, dx=0.25, follow=0)
    return Scene(name="c2-single-patch", fft_n=512, fft_L=1000.0, seed=0, steps=600,
                 spectrum=sp, patches=[p], sources=[src],
                 bins=default_bins(8, 0.5, 32.0, 0.25))


def _grid_patches(rng, n_patches, cols, pitch, side_lo, side_hi, dx, eta0, ref_side,
                  speed_lo, speed_hi, origin):
    """Patches on a cols x rows grid, each following its own source."""
    patches, sources = [], []
    ratio = side_hi / side_lo
    for k in range(n_patches):
        u = rng.random()
        side = int(round(side_lo * ratio ** u / 16.0)) * 16
        side = max(side_lo, min(side_hi, side))
        z = rng.standard_normal()
        heading = rng.uniform(-math.pi, math.pi)
        speed = rng.uniform(speed_lo, speed_hi)
        ax = origin[0] + (k % cols + 0.5) * pitch
        ay = origin[1] + (k // cols + 0.5) * pitch
        # log-normal density, scaled by 1/side so that counts do not grow
        # with patch perimeter (recipe stated in the design notes)
        eta = eta0 * math.exp(z) * (ref_side / side)
        radius = min(5.0, side * dx / 8.0)
        patches.append(Patch(anchor_x=ax, anchor_y=ay, nx=side, ny=side, dx=dx,
                             eta=eta, follow=k))
        sources.append(Source(x0=ax, y0=ay, vx=speed * math.cos(heading),
                              vy=speed * math.sin(heading), radius=radius, draft=1.0,
                              ring_n=64, patch=k))
    return patches, sources


def c3() -> Scene:
    """Batching: 32 patches of 64^2..512^2 cells, FFT 1024^2 over 2 km.

    eta0 = 6.4 gives a median of about 50k and a total of about 4M live
    particles at frame 1000."""
    rng = np.random.default_rng(1)
    sp = Spectrum(U10=15.0, fetch=100e3, gamma=3.3, spread_s=8.0, wind_dir=0.0,
                  n_buckets=8, lambda_min=0.5, lambda_max=32.0, eta=8.0)
    patches, sources = _grid_patches(rng, 32, 8, 250.0, 64, 512, 0.25, eta0=6.4,
                                     ref_side=256, speed_lo=2.0, speed_hi=12.0,
                                     origin=(0.0, 0.0))
    return Scene(name="c3-batched", fft_n=1024, fft_L=2000.0, seed=1, steps=1000,
                 spectrum=sp, patches=patches, sources=sources,
                 bins=default_bins(8, 0.5, 32.0, 0.25), compact=True, batched=True)


def c4() -> Scene:
    """The c2 scene, 16-byte records, anchored ~50 km from the origin, FFT 2048^2."""
    s = c2()
    d = 50e3 / math.sqrt(2.0)
    ax = round(d, 1)
    p = dataclasses.replace(s.patches[0], anchor_x=ax, anchor_y=ax)
    src = dataclasses.replace(s.sources[0], x0=ax, y0=ax)
    return s.replace(name="c4-precision", fft_n=2048, fft_L=4000.0, patches=[p],
                     sources=[src], compact=True)


def c5() -> Scene:
    """Stress: FFT 4096^2 over 8 km, 64 patches of 128^2..1024^2, 16 buckets.

    eta0 = 1.2 gives about 16M live particles at frame 1000."""
    rng = np.random.default_rng(2)
    sp = Spectrum(U10=20.0, fetch=100e3, gamma=3.3, spread_s=4.0, wind_dir=0.0,
                  n_buckets=16, lambda_min=0.25, lambda_max=64.0, eta=0.74)
    patches, sources = _grid_patches(rng, 64, 8, 1000.0, 128, 1024, 0.25, eta0=1.2,
                                     ref_side=512, speed_lo=2.0, speed_hi=15.0,
                                     origin=(0.0, 0.0))
    return Scene(name="c5-stress", fft_n=4096, fft_L=8000.0, seed=2, steps=1000,
                 spectrum=sp, patches=patches, sources=sources,
                 bins=default_bins(16, 0.25, 64.0, 0.25), compact=True, batched=True)


def p0() -> Scene:
    """The paper's default parameters (Sec 5): U10 = 5 m/s, fetch 10 km,
    N_omega = N_theta = 16, a 100 m wave-particle region at 512^2 cells and a
    500 m FFT ocean at 512^2.  Buckets are the paper's equal-energy partition
    of [0.5 w_p, 2.5 w_p], spreading is Mitsuyasu's s(w), gamma follows from
    the fetch, and each injected group holds N_theta stratified directions
    with amplitudes from S(w, theta); the group count per side pair is the
    paper's (no obliquity weighting).  The region follows a small moving
    source (a boat).
    About 0.54M particles are live after the ~3600 steps that the slowest
    waves need to cross the region.  Bin edges (cells) are chosen for this
    spectrum's bucket wavelengths (about 1.8-19.7 m, i.e. 9-101 cells)."""
    sp = Spectrum(U10=5.0, fetch=10e3, gamma=0.0, spread_s=-1.0, wind_dir=0.0,
                  n_buckets=16, lambda_min=1.0, lambda_max=2.0, eta=16.0, bucket_mode=1,
                  dir_mode=1)
    h = math.radians(30.0)
    src = Source(x0=250.0, y0=250.0, vx=3.0 * math.cos(h), vy=3.0 * math.sin(h),
                 radius=2.5, draft=0.5, ring_n=64, patch=0)
    p = Patch(anchor_x=250.0, anchor_y=250.0, nx=512, ny=512, dx=100.0 / 512, follow=0)
    return Scene(name="p0-paper-default", fft_n=512, fft_L=500.0, seed=0, steps=3600,
                 spectrum=sp, patches=[p], sources=[src], bins=[16, 16] + [32] * 14)


SCENES = {"c1": c1, "c2": c2, "c3": c3, "c4": c4, "c5": c5, "p0": p0}


def get(name: str) -> Scene:
    return SCENES[name]()
