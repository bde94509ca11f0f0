"""ctypes front end of the FP64 CPU oracle (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library and its Python binding
never do.  The oracle is plain C compiled with gcc (``build()``); it shares no
code with the GPU path and takes its inputs from the same seeded
:class:`paper_2511_02852_amd.scenes.Scene` objects.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_OUT_DIR = os.path.join(_HERE, "_build")
_LIB_PATH = os.path.join(_OUT_DIR, "liboracle.so")

NCODE = 10368
NDIR = 64
C_LIVE, C_INJ, C_EMIT, C_SUB, C_DIED = range(5)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP contraction off, no fast-math)."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    os.makedirs(_OUT_DIR, exist_ok=True)
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wno-unused-function", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True, cwd=_HERE)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    L = C.CDLL(_LIB_PATH)
    vp, i32, i64, u64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double
    P = C.POINTER
    sig = {
        "orc_create": (vp, [i32, dbl, dbl, dbl, u64]),
        "orc_destroy": (None, [vp]),
        "orc_error": (C.c_char_p, [vp]),
        "orc_set_spectrum": (C.c_int, [vp, dbl, dbl, dbl, dbl, dbl, i32, dbl, dbl, dbl, i32, dbl, i32, i32, i32, i32]),
        "orc_add_patch": (C.c_int, [vp, dbl, dbl, i32, i32, dbl, dbl, dbl, i32]),
        "orc_add_source": (C.c_int, [vp, dbl, dbl, dbl, dbl, dbl, dbl, i32, i32, dbl, dbl]),
        "orc_set_bins": (C.c_int, [vp, P(i32)]),
        "orc_set_synthesis": (C.c_int, [vp, i32, i32]),
        "orc_normals": (C.c_int, [vp, i32, P(dbl), P(dbl)]),
        "orc_background_field": (C.c_int, [vp, i32, dbl, P(dbl)]),
        "orc_sample_probes": (C.c_int, [vp, P(dbl), P(dbl), P(dbl), i64, P(dbl)]),
        "orc_step": (C.c_int, [vp, i32]),
        "orc_step_index": (i64, [vp]),
        "orc_background": (C.c_int, [vp, P(dbl)]),
        "orc_background_at": (C.c_int, [vp, dbl, P(dbl)]),
        "orc_patch_maps": (C.c_int, [vp, i32, P(dbl), P(dbl), P(dbl)]),
        "orc_counts": (C.c_int, [vp, i32, P(i64)]),
        "orc_tile_dims": (C.c_int, [vp, i32, i32, P(i64)]),
        "orc_tiles": (C.c_int, [vp, i32, i32, P(i64), i64]),
        "orc_num_particles": (i64, [vp]),
        "orc_particles": (i64, [vp, P(i64), i64]),
        "orc_window": (C.c_int, [vp, i32, P(i64)]),
        "orc_jonswap": (dbl, [vp, dbl]),
        "orc_dir": (dbl, [vp, dbl, dbl]),
        "orc_spread": (dbl, [vp, dbl]),
        "orc_spectrum_consts": (C.c_int, [vp, P(dbl)]),
        "orc_bucket": (C.c_int, [vp, i32, P(dbl)]),
        "orc_patch_bucket": (C.c_int, [vp, i32, i32, P(dbl)]),
        "orc_dir_table": (C.c_int, [vp, i32, i32, P(i64), P(i64), P(i64)]),
        "orc_velocity": (C.c_int, [vp, i32, i32, P(i64)]),
        "orc_source_info": (C.c_int, [vp, i32, P(dbl)]),
        "orc_inject_count": (i64, [vp, i32, i32, i32, i64]),
        "orc_philox4x64": (None, [P(u64), P(u64), P(u64)]),
        "orc_fft_inverse": (None, [P(dbl), P(dbl), i32]),
        "orc_fft2_inverse": (None, [P(dbl), P(dbl), i32]),
        "orc_dft2_inverse": (None, [P(dbl), P(dbl), P(dbl), P(dbl), i32]),
        "orc_h0": (C.c_int, [vp, P(dbl), P(dbl)]),
        "orc_set_h0": (C.c_int, [vp, P(dbl), P(dbl)]),
        "orc_splat": (C.c_int, [vp, i32, P(i64), i64, P(dbl)]),
        "orc_seek": (C.c_int, [vp, i64]),
        "orc_load": (C.c_int, [vp, i64, P(i64), i64]),
        "orc_blend": (C.c_int, [vp, i32, P(dbl), P(dbl), P(dbl)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def philox4x64(ctr, key):
    out = np.zeros(4, dtype=np.uint64)
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    lib().orc_philox4x64(_p(c, C.c_uint64), _p(k, C.c_uint64), _p(out, C.c_uint64))
    return out


def fft2_inverse(z: np.ndarray) -> np.ndarray:
    n = z.shape[0]
    re = np.ascontiguousarray(z.real, dtype=np.float64).copy()
    im = np.ascontiguousarray(z.imag, dtype=np.float64).copy()
    lib().orc_fft2_inverse(_p(re, C.c_double), _p(im, C.c_double), n)
    return re + 1j * im


def fft_inverse(z: np.ndarray) -> np.ndarray:
    n = z.shape[0]
    re = np.ascontiguousarray(z.real, dtype=np.float64).copy()
    im = np.ascontiguousarray(z.imag, dtype=np.float64).copy()
    lib().orc_fft_inverse(_p(re, C.c_double), _p(im, C.c_double), n)
    return re + 1j * im


def dft2_inverse(z: np.ndarray) -> np.ndarray:
    n = z.shape[0]
    re = np.ascontiguousarray(z.real, dtype=np.float64)
    im = np.ascontiguousarray(z.imag, dtype=np.float64)
    ore = np.zeros_like(re)
    oim = np.zeros_like(im)
    lib().orc_dft2_inverse(_p(re, C.c_double), _p(im, C.c_double), _p(ore, C.c_double),
                           _p(oim, C.c_double), n)
    return ore + 1j * oim


class OracleError(RuntimeError):
    pass


class Oracle:
    """One oracle ocean built from a Scene (same inputs as the GPU library)."""

    def __init__(self, scene, bins=None, spectrum_overrides=None):
        self.L = lib()
        self.scene = scene
        h = self.L.orc_create(scene.fft_n, scene.fft_L, scene.g, scene.dt, scene.seed)
        if not h:
            raise OracleError("orc_create rejected the configuration")
        self.h = h
        sp = scene.spectrum
        if spectrum_overrides:
            import dataclasses
            sp = dataclasses.replace(sp, **spectrum_overrides)
        self._check(self.L.orc_set_spectrum(h, sp.U10, sp.fetch, sp.gamma, sp.spread_s, sp.wind_dir,
                                            sp.n_buckets, sp.lambda_min, sp.lambda_max, sp.eta,
                                            sp.max_level, sp.subdiv_frac, sp.h0_mode,
                                            sp.bucket_mode, sp.dir_mode, sp.flux_mode))
        self.nb = sp.n_buckets
        for p in scene.patches:
            self._check(self.L.orc_add_patch(h, p.anchor_x, p.anchor_y, p.nx, p.ny, p.dx, p.eta,
                                             p.blend_band, p.follow))
        for s in scene.sources:
            self._check(self.L.orc_add_source(h, s.x0, s.y0, s.vx, s.vy, s.radius, s.draft,
                                              s.ring_n, s.patch, float(getattr(s, "heave_amp", 0.0)),
                                              float(getattr(s, "heave_period", 0.0))))
        self._check(self.L.orc_set_synthesis(h, int(getattr(scene, "synth", 0)), int(getattr(scene, "kernel", 0))))
        b = bins if bins is not None else scene.bins
        if b is not None:
            arr = np.ascontiguousarray(b, dtype=np.int32)
            self._check(self.L.orc_set_bins(h, _p(arr, C.c_int32)))

    def _check(self, rc):
        if rc != 0:
            raise OracleError(self.L.orc_error(self.h).decode())

    def close(self):
        if self.h:
            self.L.orc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # stepping / state
    def step(self, n: int):
        self._check(self.L.orc_step(self.h, int(n)))

    @property
    def n(self) -> int:
        return int(self.L.orc_step_index(self.h))

    def background(self, t=None) -> np.ndarray:
        N = self.scene.fft_n
        H = np.zeros((N, N), dtype=np.float64)
        if t is None:
            self._check(self.L.orc_background(self.h, _p(H, C.c_double)))
        else:
            self._check(self.L.orc_background_at(self.h, float(t), _p(H, C.c_double)))
        return H

    def background_field(self, field: int, t=None) -> np.ndarray:
        """Background field (N, N): 0 height, 1 dH/dx, 2 dH/dy, 3/4 choppy displacement x/y."""
        N = self.scene.fft_n
        out = np.zeros((N, N), dtype=np.float64)
        tt = self.n * self.scene.dt if t is None else float(t)
        self._check(self.L.orc_background_field(self.h, int(field), tt, _p(out, C.c_double)))
        return out

    def sample_probes(self, xy, H=None, blended=None) -> np.ndarray:
        """Height and unit normal (n, 4) at world points xy (n, 2) from the
        background H and the patches' blended maps (own maps when None)."""
        if H is None:
            H = self.background()
        if blended is None:
            blended = [self.patch_maps(p, H)[1] for p in range(len(self.scene.patches))]
        B = np.ascontiguousarray(np.concatenate([np.ravel(b) for b in blended]) if blended else np.zeros(1))
        H = np.ascontiguousarray(H, dtype=np.float64)
        xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
        out = np.zeros((xy.shape[0], 4))
        self._check(self.L.orc_sample_probes(self.h, _p(H, C.c_double), _p(B, C.c_double), _p(xy, C.c_double),
                                             xy.shape[0], _p(out, C.c_double)))
        return out

    def patch_maps(self, p: int, H=None, blended=True):
        pt = self.scene.patches[p]
        raw = np.zeros((pt.ny, pt.nx), dtype=np.float64)
        bl = np.zeros((pt.ny, pt.nx), dtype=np.float64) if blended else None
        Hp = None
        if H is not None:
            H = np.ascontiguousarray(H, dtype=np.float64)
            Hp = _p(H, C.c_double)
        self._check(self.L.orc_patch_maps(self.h, p, Hp, _p(raw, C.c_double),
                                          _p(bl, C.c_double) if bl is not None else None))
        return raw, bl

    def counts(self, p: int) -> np.ndarray:
        out = np.zeros((self.nb, 5), dtype=np.int64)
        self._check(self.L.orc_counts(self.h, p, _p(out, C.c_int64)))
        return out

    def tile_dims(self, p: int, b: int):
        d = np.zeros(3, dtype=np.int64)
        self._check(self.L.orc_tile_dims(self.h, p, b, _p(d, C.c_int64)))
        return int(d[0]), int(d[1]), int(d[2])

    def tiles(self, p: int, b: int) -> np.ndarray:
        _, nbx, nby = self.tile_dims(p, b)
        out = np.zeros((nby, nbx), dtype=np.int64)
        self._check(self.L.orc_tiles(self.h, p, b, _p(out, C.c_int64), out.size))
        return out

    def particles(self) -> np.ndarray:
        n = int(self.L.orc_num_particles(self.h))
        out = np.zeros((n, 10), dtype=np.int64)
        if n:
            self.L.orc_particles(self.h, _p(out, C.c_int64), n)
        return out

    def window(self, p: int):
        w = np.zeros(2, dtype=np.int64)
        self._check(self.L.orc_window(self.h, p, _p(w, C.c_int64)))
        return int(w[0]), int(w[1])

    # tables
    def jonswap(self, w: float) -> float:
        return float(self.L.orc_jonswap(self.h, float(w)))

    def dir(self, w: float, theta: float) -> float:
        return float(self.L.orc_dir(self.h, float(w), float(theta)))

    def spread(self, w: float) -> float:
        return float(self.L.orc_spread(self.h, float(w)))

    def spectrum_consts(self):
        out = np.zeros(4)
        self._check(self.L.orc_spectrum_consts(self.h, _p(out, C.c_double)))
        return dict(alpha=out[0], wp=out[1], gamma=out[2], wind_code=int(out[3]))

    def bucket(self, i: int):
        out = np.zeros(6)
        self._check(self.L.orc_bucket(self.h, i, _p(out, C.c_double)))
        return dict(w=out[0], dw=out[1], r=out[2], c=out[3], lam=out[4], margin_u=int(out[5]))

    def patch_bucket(self, p: int, i: int):
        out = np.zeros(5)
        self._check(self.L.orc_patch_bucket(self.h, p, i, _p(out, C.c_double)))
        return dict(A=out[0], Rx=int(out[1]), Ry=int(out[2]), band=out[3], eta=out[4])

    def dir_table(self, i: int, pair: int = 0):
        q = np.zeros(NDIR, dtype=np.int64)
        cdf = np.zeros(NDIR, dtype=np.int64)
        codes = np.zeros(NDIR, dtype=np.int64)
        self._check(self.L.orc_dir_table(self.h, i, pair, _p(q, C.c_int64), _p(cdf, C.c_int64),
                                         _p(codes, C.c_int64)))
        return q, cdf, codes

    def velocity(self, i: int, code: int):
        v = np.zeros(2, dtype=np.int64)
        self._check(self.L.orc_velocity(self.h, i, code, _p(v, C.c_int64)))
        return int(v[0]), int(v[1])

    def source_info(self, s: int):
        out = np.zeros(12)
        self._check(self.L.orc_source_info(self.h, s, _p(out, C.c_double)))
        return dict(bucket=int(out[0]), E=int(out[1]), B=out[2], heading=out[3], sum_abs=out[4],
                    T=[int(x) for x in out[5:9]], a0=int(out[9]), Eh=int(out[10]), Bh=out[11])

    def inject_count(self, p, i, pair, n) -> int:
        return int(self.L.orc_inject_count(self.h, p, i, pair, n))

    def h0(self) -> np.ndarray:
        N = self.scene.fft_n
        re = np.zeros((N, N))
        im = np.zeros((N, N))
        self._check(self.L.orc_h0(self.h, _p(re, C.c_double), _p(im, C.c_double)))
        return re + 1j * im

    def set_h0(self, z: np.ndarray):
        re = np.ascontiguousarray(z.real, dtype=np.float64)
        im = np.ascontiguousarray(z.imag, dtype=np.float64)
        self._check(self.L.orc_set_h0(self.h, _p(re, C.c_double), _p(im, C.c_double)))

    def seek(self, n: int):
        """Step index n (with its windows) for evaluating caller-supplied
        particles and maps; only for an oracle that holds no particles."""
        self._check(self.L.orc_seek(self.h, int(n)))

    def load(self, n: int, recs: np.ndarray):
        """Take caller-supplied particle records (the ten-column layout of
        ``particles()``) as the state after step n; the next ``step``
        continues from there.  Used to time one full frame of a large scene
        without re-running its history."""
        r = np.ascontiguousarray(recs, dtype=np.int64).reshape(-1, 10)
        self._check(self.L.orc_load(self.h, int(n), _p(r, C.c_int64), r.shape[0]))

    def blend(self, p: int, H: np.ndarray, raw: np.ndarray) -> np.ndarray:
        H = np.ascontiguousarray(H, dtype=np.float64)
        raw = np.ascontiguousarray(raw, dtype=np.float64)
        out = np.zeros_like(raw)
        self._check(self.L.orc_blend(self.h, p, _p(H, C.c_double), _p(raw, C.c_double), _p(out, C.c_double)))
        return out

    def normals(self, p: int, h: np.ndarray) -> np.ndarray:
        """Unit normals (3, ny, nx) of patch p's map h by finite differences."""
        pt = self.scene.patches[p]
        h = np.ascontiguousarray(h, dtype=np.float64)
        out = np.zeros((3, pt.ny, pt.nx))
        self._check(self.L.orc_normals(self.h, p, _p(h, C.c_double), _p(out, C.c_double)))
        return out

    def splat(self, p: int, recs: np.ndarray) -> np.ndarray:
        pt = self.scene.patches[p]
        raw = np.zeros((pt.ny, pt.nx))
        r = np.ascontiguousarray(recs, dtype=np.int64).reshape(-1, 10)
        self._check(self.L.orc_splat(self.h, p, _p(r, C.c_int64), r.shape[0], _p(raw, C.c_double)))
        return raw
