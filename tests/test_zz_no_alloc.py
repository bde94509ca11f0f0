"""The allocation-free probe entry point against the allocating one.

hwo_sample_probes_static stages probe positions and results in a static
device array instead of allocating; its results must equal those of
hwo_sample_probes (host arrays) bit for bit, on two calls in a row, the
second with fewer probes, so that a stale tail of the shared array from
the first call cannot leak into the second.
"""
import ctypes as C

import numpy as np
import pytest

from paper_2511_02852_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield


def probe_points(scene, n, seed):
    """World points over the patch windows and the open background."""
    rng = np.random.default_rng(seed)
    P, S = scene.patches[0], scene.sources[0]
    t = 40 * scene.dt
    cx, cy = S.x0 + S.vx * t, S.y0 + S.vy * t
    half = 0.5 * P.nx * P.dx
    near = np.column_stack([rng.uniform(cx - 1.2 * half, cx + 1.2 * half, n // 2),
                            rng.uniform(cy - 1.2 * half, cy + 1.2 * half, n // 2)])
    far = rng.uniform(0.0, scene.fft_L, size=(n - n // 2, 2))
    return np.ascontiguousarray(np.vstack([near, far]), dtype=np.float64)


def call(L, h, fn, xy, static):
    n = xy.shape[0]
    out = np.full((n, 4), np.nan, dtype=np.float32)
    pxy = xy.ctypes.data_as(C.POINTER(C.c_double))
    pout = out.ctypes.data_as(C.POINTER(C.c_float))
    rc = fn(h, pxy, n, pout) if static else fn(h, pxy, n, pout, 0)
    assert rc == 0, L.hwo_last_error(h)
    return out


def test_static_probes_equal_allocating_probes():
    from paper_2511_02852_amd import hwo
    s = scenes.c2()
    g = hwo.Ocean(s, compact=True, batched=True)
    L, h = g.L, g.h
    # before any step the static variant refuses (it never builds state)
    xy0 = probe_points(s, 8, 0)
    out0 = np.zeros((8, 4), dtype=np.float32)
    assert L.hwo_sample_probes_static(h, xy0.ctypes.data_as(C.POINTER(C.c_double)), 8,
                                      out0.ctypes.data_as(C.POINTER(C.c_float))) == hwo.HWO_ESTATE
    g.step(40)
    g.sync()
    for n, seed in ((5000, 1), (1234, 2)):
        print(f"probes n={n}", flush=True)
        xy = probe_points(s, n, seed)
        want = call(L, h, L.hwo_sample_probes, xy, static=False)
        got = call(L, h, L.hwo_sample_probes_static, xy, static=True)
        assert np.all(np.isfinite(want))
        assert np.array_equal(got, want), f"n={n}: max diff {np.nanmax(np.abs(got - want))}"
    # the maximum size is accepted, one more is refused
    n = 131072
    xy = probe_points(s, n, 3)
    got = call(L, h, L.hwo_sample_probes_static, xy, static=True)
    want = call(L, h, L.hwo_sample_probes, xy, static=False)
    assert np.array_equal(got, want)
    out = np.zeros((n + 1, 4), dtype=np.float32)
    xy1 = np.vstack([xy, xy[:1]])
    assert L.hwo_sample_probes_static(h, xy1.ctypes.data_as(C.POINTER(C.c_double)), n + 1,
                                      out.ctypes.data_as(C.POINTER(C.c_float))) == hwo.HWO_ERANGE
    g.close()
