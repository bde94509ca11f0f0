"""ctypes binding of the gfx950 hybrid-ocean library (``include/hwo.h``).

Argument marshalling only: every step of the path runs in the HIP kernels of
``_build/libhwo.so``.  PyTorch supplies device memory (through the
allocator hooks) and the stream.  There is no CPU fallback: if the library
is not built, or no GPU is present, the calls fail loudly.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "libhwo.so")

HWO_OK, HWO_EINVAL, HWO_ESTATE, HWO_ENOMEM, HWO_EDEVICE, HWO_ERANGE, HWO_EOVERFLOW = 0, -1, -2, -3, -4, -5, -6
STAGES = ["params", "fft_a", "fft_b", "count", "scan", "scatter", "splat", "splat_plan", "splat_reduce",
          "bin_plan", "deposit_x", "filter_y", "layer_sum", "normals"]
EXPORTS = ["hwo_create_ocean", "hwo_destroy_ocean", "hwo_last_error", "hwo_set_spectrum", "hwo_add_patch",
           "hwo_add_source", "hwo_set_bins", "hwo_step", "hwo_sync", "hwo_step_index", "hwo_read_heightmaps",
           "hwo_read_counts", "hwo_read_buckets", "hwo_tile_dims", "hwo_read_tiles", "hwo_read_particles", "hwo_test_splat",
           "hwo_set_timing", "hwo_stage_times", "hwo_time_stage", "hwo_record_bytes", "hwo_sample_probes",
           "hwo_sample_probes_static", "hwo_set_splat_profile", "hwo_read_splat_profile", "hwo_get_plan",
           "hwo_set_plan", "hwo_autotune", "hwo_snapshot_size", "hwo_snapshot", "hwo_restore"]

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class HwoConfig(C.Structure):
    _fields_ = [("fft_n", C.c_int32), ("fft_L", C.c_double), ("g", C.c_double), ("dt", C.c_double),
                ("seed", C.c_uint64), ("compact", C.c_int32), ("batched", C.c_int32), ("stream", C.c_void_p),
                ("dev_alloc", ALLOC_FN), ("dev_free", FREE_FN), ("alloc_ctx", C.c_void_p),
                ("max_particles", C.c_int64), ("synth", C.c_int32), ("normals", C.c_int32),
                ("bg_fields", C.c_int32), ("kernel", C.c_int32), ("fft_mfma16", C.c_int32)]


class HwoSpectrum(C.Structure):
    _fields_ = [("U10", C.c_double), ("fetch", C.c_double), ("gamma", C.c_double), ("spread_s", C.c_double),
                ("wind_dir", C.c_double), ("n_buckets", C.c_int32), ("lambda_min", C.c_double),
                ("lambda_max", C.c_double), ("eta", C.c_double), ("max_level", C.c_int32),
                ("subdiv_frac", C.c_double), ("h0_mode", C.c_int32),
                ("bucket_mode", C.c_int32), ("dir_mode", C.c_int32),
                ("flux_mode", C.c_int32)]


class HwoPatch(C.Structure):
    _fields_ = [("anchor_x", C.c_double), ("anchor_y", C.c_double), ("nx", C.c_int32), ("ny", C.c_int32),
                ("dx", C.c_double), ("eta", C.c_double), ("blend_band", C.c_double), ("follow", C.c_int32)]


class HwoPlan(C.Structure):
    _fields_ = [("chunk_load", C.c_int32), ("items_target", C.c_int32), ("splat_grid", C.c_int32),
                ("splat_kernel", C.c_int32)]


class HwoSource(C.Structure):
    _fields_ = [("x0", C.c_double), ("y0", C.c_double), ("vx", C.c_double), ("vy", C.c_double),
                ("radius", C.c_double), ("draft", C.c_double), ("ring_n", C.c_int32), ("patch", C.c_int32),
                ("heave_amp", C.c_double), ("heave_period", C.c_double)]


class HwoError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"hwo error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load the built library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise HwoError(HWO_EDEVICE, f"{LIB_PATH} is missing: run __graft_entry__.build() first")
    # PyTorch ships its own HIP runtime under the same soname; load it first so
    # the library binds to that runtime and shares torch's streams and memory.
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, P = C.c_void_p, C.c_int32, C.c_int64, C.POINTER
    sig = {
        "hwo_create_ocean": (C.c_int, [P(HwoConfig), P(vp)]),
        "hwo_destroy_ocean": (None, [vp]),
        "hwo_last_error": (C.c_char_p, [vp]),
        "hwo_set_spectrum": (C.c_int, [vp, P(HwoSpectrum)]),
        "hwo_add_patch": (C.c_int, [vp, P(HwoPatch), P(i32)]),
        "hwo_add_source": (C.c_int, [vp, P(HwoSource), P(i32)]),
        "hwo_set_bins": (C.c_int, [vp, P(i32), i32]),
        "hwo_step": (C.c_int, [vp, i32]),
        "hwo_sync": (C.c_int, [vp]),
        "hwo_step_index": (i64, [vp]),
        "hwo_read_heightmaps": (C.c_int, [vp, i32, i32, vp, i64, i32]),
        "hwo_read_counts": (C.c_int, [vp, i32, P(i64), i64]),
        "hwo_read_buckets": (C.c_int, [vp, P(C.c_double), i32]),
        "hwo_tile_dims": (C.c_int, [vp, i32, i32, P(i64)]),
        "hwo_read_tiles": (C.c_int, [vp, i32, i32, P(i64), i64]),
        "hwo_read_particles": (C.c_int, [vp, P(i64), i64, P(i64)]),
        "hwo_test_splat": (C.c_int, [vp, i32, P(i64), i64, P(C.c_float), i64]),
        "hwo_set_timing": (C.c_int, [vp, i32]),
        "hwo_stage_times": (C.c_int, [vp, P(C.c_double), P(i64), i32]),
        "hwo_time_stage": (C.c_int, [vp, i32, i32, P(C.c_double)]),
        "hwo_record_bytes": (i32, [vp]),
        "hwo_get_plan": (C.c_int, [vp, P(HwoPlan)]),
        "hwo_set_plan": (C.c_int, [vp, P(HwoPlan)]),
        "hwo_autotune": (C.c_int, [vp, i32, P(HwoPlan), P(C.c_double), P(C.c_double)]),
        "hwo_sample_probes": (C.c_int, [vp, P(C.c_double), i64, P(C.c_float), i32]),
        "hwo_sample_probes_static": (C.c_int, [vp, P(C.c_double), i64, P(C.c_float)]),
        "hwo_set_splat_profile": (C.c_int, [vp, i32]),
        "hwo_read_splat_profile": (C.c_int, [vp, P(C.c_double), i32]),
        "hwo_snapshot_size": (C.c_int, [vp, P(i64)]),
        "hwo_snapshot": (C.c_int, [vp, vp, i64]),
        "hwo_restore": (C.c_int, [vp, vp, i64]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


class _TorchAllocator:
    """Device memory from PyTorch's caching allocator, kept alive by pointer.

    Blocks are allocated with the library's stream current, so the caching
    allocator associates them with that stream: a block is only handed out
    again to allocations on the same stream, which are ordered after every
    library kernel that used it."""

    def __init__(self, stream):
        import torch
        self.torch = torch
        self.stream = stream
        self.live = {}
        self.alloc_cb = ALLOC_FN(self._alloc)
        self.free_cb = FREE_FN(self._free)

    def _alloc(self, nbytes, ctx):
        try:
            with self.torch.cuda.stream(self.stream):
                t = self.torch.empty(int(nbytes), dtype=self.torch.uint8, device="cuda")
        except Exception:
            return None
        ptr = t.data_ptr()
        self.live[ptr] = t
        return ptr

    def _free(self, ptr, ctx):
        self.live.pop(ptr, None)


class Ocean:
    """One hybrid ocean on the GPU, built from a :class:`scenes.Scene`."""

    def __init__(self, scene, *, compact=None, batched=None, bins=None, max_particles=0,
                 torch_memory=True, stream=None, normals=False, bg_fields=False, fft_mfma16=False):
        self.L = lib()
        self.scene = scene
        self.h = C.c_void_p()
        cfg = HwoConfig()
        cfg.fft_n = scene.fft_n
        cfg.fft_L = scene.fft_L
        cfg.g = scene.g
        cfg.dt = scene.dt
        cfg.seed = scene.seed
        cfg.compact = int(scene.compact if compact is None else compact)
        cfg.batched = int(scene.batched if batched is None else batched)
        self._alloc = None
        self._stream = None
        if torch_memory or stream is not None:
            import torch
            if stream is None:
                stream = torch.cuda.Stream()
            self._stream = stream
            cfg.stream = C.c_void_p(stream.cuda_stream)
        if torch_memory:
            self._alloc = _TorchAllocator(self._stream)
            cfg.dev_alloc = self._alloc.alloc_cb
            cfg.dev_free = self._alloc.free_cb
        cfg.max_particles = int(max_particles)
        cfg.synth = int(getattr(scene, "synth", 0))
        cfg.kernel = int(getattr(scene, "kernel", 0))
        cfg.normals = int(bool(normals))
        cfg.bg_fields = int(bool(bg_fields))
        cfg.fft_mfma16 = int(bool(fft_mfma16))
        self._cfg = cfg
        self._check(self.L.hwo_create_ocean(C.byref(cfg), C.byref(self.h)))
        sp = scene.spectrum
        hs = HwoSpectrum(sp.U10, sp.fetch, sp.gamma, sp.spread_s, sp.wind_dir, sp.n_buckets, sp.lambda_min,
                         sp.lambda_max, sp.eta, sp.max_level, sp.subdiv_frac, sp.h0_mode,
                         sp.bucket_mode, sp.dir_mode, sp.flux_mode)
        self._check(self.L.hwo_set_spectrum(self.h, C.byref(hs)))
        self.nb = sp.n_buckets
        pid = C.c_int32()
        for p in scene.patches:
            hp = HwoPatch(p.anchor_x, p.anchor_y, p.nx, p.ny, p.dx, p.eta, p.blend_band, p.follow)
            self._check(self.L.hwo_add_patch(self.h, C.byref(hp), C.byref(pid)))
        for s in scene.sources:
            hs_ = HwoSource(s.x0, s.y0, s.vx, s.vy, s.radius, s.draft, s.ring_n, s.patch,
                            float(getattr(s, "heave_amp", 0.0)), float(getattr(s, "heave_period", 0.0)))
            self._check(self.L.hwo_add_source(self.h, C.byref(hs_), C.byref(pid)))
        b = bins if bins is not None else scene.bins
        if b is not None:
            arr = np.ascontiguousarray(b, dtype=np.int32)
            self._check(self.L.hwo_set_bins(self.h, _p(arr, C.c_int32), arr.size))

    def _check(self, rc, allow=()):
        if rc != HWO_OK and rc not in allow:
            msg = self.L.hwo_last_error(self.h).decode() if self.h else "create failed"
            raise HwoError(rc, msg)
        return rc

    def close(self):
        if self.h:
            self.L.hwo_destroy_ocean(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- stepping
    def step(self, n: int = 1):
        self._check(self.L.hwo_step(self.h, int(n)))

    def sync(self):
        self._check(self.L.hwo_sync(self.h))

    @property
    def n(self) -> int:
        return int(self.L.hwo_step_index(self.h))

    # -- outputs
    def background(self, field: int = 0) -> np.ndarray:
        """Background field: 0 height, 1 dH/dx, 2 dH/dy, 3/4 choppy displacement (needs bg_fields)."""
        N = self.scene.fft_n
        out = np.zeros((N, N), dtype=np.float32)
        self._check(self.L.hwo_read_heightmaps(self.h, -1, int(field), out.ctypes.data, out.size, 0))
        return out

    def patch_map(self, p: int, layer: int = 0) -> np.ndarray:
        pt = self.scene.patches[p]
        out = np.zeros((pt.ny, pt.nx), dtype=np.float32)
        self._check(self.L.hwo_read_heightmaps(self.h, p, layer, out.ctypes.data, out.size, 0))
        return out

    def normals(self, p: int) -> np.ndarray:
        """Unit normals (3, ny, nx) of patch p's blended map (needs normals=True)."""
        return np.stack([self.patch_map(p, layer) for layer in (2, 3, 4)])

    def snapshot(self) -> bytes:
        """Host image of the state at the current step boundary."""
        n = C.c_int64()
        self._check(self.L.hwo_snapshot_size(self.h, C.byref(n)))
        buf = (C.c_char * n.value)()
        self._check(self.L.hwo_snapshot(self.h, buf, n.value))
        return bytes(buf)

    def restore(self, image: bytes):
        """Continue from a snapshot of the same scene."""
        buf = C.create_string_buffer(image, len(image))
        self._check(self.L.hwo_restore(self.h, buf, len(image)))

    def sample_probes(self, xy) -> np.ndarray:
        """Height and unit normal (n, 4) of the current frame at world points xy (n, 2)."""
        xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
        out = np.zeros((xy.shape[0], 4), dtype=np.float32)
        self._check(self.L.hwo_sample_probes(self.h, _p(xy, C.c_double), xy.shape[0], _p(out, C.c_float), 0))
        return out

    def read_into(self, which: int, layer: int, tensor):
        """Device-to-device copy of a height map into a CUDA tensor (float32)."""
        self._check(self.L.hwo_read_heightmaps(self.h, which, layer, C.c_void_p(tensor.data_ptr()),
                                               tensor.numel(), 1))

    def counts(self, p: int, allow_overflow=False) -> np.ndarray:
        out = np.zeros((self.nb, 6), dtype=np.int64)
        allow = (HWO_EOVERFLOW,) if allow_overflow else ()
        self._check(self.L.hwo_read_counts(self.h, p, _p(out, C.c_int64), out.size), allow)
        return out

    def tile_dims(self, p: int, b: int):
        d = np.zeros(3, dtype=np.int64)
        self._check(self.L.hwo_tile_dims(self.h, p, b, _p(d, C.c_int64)))
        return int(d[0]), int(d[1]), int(d[2])

    def buckets(self) -> np.ndarray:
        """Per bucket: w_i, dw_i, radius r_i (m), phase speed c_i (m/s)."""
        out = np.zeros((self.nb, 4))
        self._check(self.L.hwo_read_buckets(self.h, _p(out, C.c_double), out.size))
        return out

    def tiles(self, p: int, b: int) -> np.ndarray:
        _, nbx, nby = self.tile_dims(p, b)
        out = np.zeros((nby, nbx), dtype=np.int64)
        self._check(self.L.hwo_read_tiles(self.h, p, b, _p(out, C.c_int64), out.size))
        return out

    def particles(self) -> np.ndarray:
        n = C.c_int64()
        self._check(self.L.hwo_read_particles(self.h, None, 0, C.byref(n)))
        out = np.zeros((n.value, 10), dtype=np.int64)
        if n.value:
            self._check(self.L.hwo_read_particles(self.h, _p(out, C.c_int64), n.value, C.byref(n)))
        return out

    def test_splat(self, p: int, recs) -> np.ndarray:
        pt = self.scene.patches[p]
        r = np.ascontiguousarray(recs, dtype=np.int64).reshape(-1, 10)
        out = np.zeros((pt.ny, pt.nx), dtype=np.float32)
        self._check(self.L.hwo_test_splat(self.h, p, _p(r, C.c_int64), r.shape[0], _p(out, C.c_float),
                                          out.size))
        return out

    # -- timing
    def set_timing(self, on: bool):
        self._check(self.L.hwo_set_timing(self.h, 1 if on else 0))

    def stage_times(self):
        ms = np.zeros(len(STAGES))
        n = np.zeros(len(STAGES), dtype=np.int64)
        self._check(self.L.hwo_stage_times(self.h, _p(ms, C.c_double), _p(n, C.c_int64), len(STAGES)))
        return {s: (float(ms[i]), int(n[i])) for i, s in enumerate(STAGES)}

    def set_splat_profile(self, on: bool):
        """Start (clearing the accumulators) or stop the splat's per-bucket profile."""
        self._check(self.L.hwo_set_splat_profile(self.h, 1 if on else 0))

    def splat_profile(self):
        """Accumulated splat profile: wavefront ticks per category (set-up,
        decode, wait, epilogue and one per bucket) and points visited per bucket."""
        v = np.zeros(36)
        self._check(self.L.hwo_read_splat_profile(self.h, _p(v, C.c_double), 36))
        nb = self.scene.spectrum.n_buckets
        return {"setup": v[0], "decode": v[1], "wait": v[2], "epilogue": v[3],
                "bucket": v[4:4 + nb].copy(), "points": v[20:20 + nb].copy()}

    def get_plan(self) -> dict:
        """Current work partition of the splat (chunk_load, items_target,
        splat_grid, splat_kernel)."""
        p = HwoPlan()
        self._check(self.L.hwo_get_plan(self.h, C.byref(p)))
        return {"chunk_load": p.chunk_load, "items_target": p.items_target, "splat_grid": p.splat_grid,
                "splat_kernel": p.splat_kernel}

    def set_plan(self, chunk_load: int, items_target: int, splat_grid: int = 0, splat_kernel: int = 2):
        p = HwoPlan(int(chunk_load), int(items_target), int(splat_grid), int(splat_kernel))
        self._check(self.L.hwo_set_plan(self.h, C.byref(p)))

    def autotune(self, reps: int = 5):
        """Search the splat partition on the current frame; returns (plan,
        ms per plan + splat + reduce of the chosen plan, of the starting one)."""
        p = HwoPlan()
        best, start = C.c_double(), C.c_double()
        self._check(self.L.hwo_autotune(self.h, int(reps), C.byref(p), C.byref(best), C.byref(start)))
        return ({"chunk_load": p.chunk_load, "items_target": p.items_target, "splat_grid": p.splat_grid,
                 "splat_kernel": p.splat_kernel},
                float(best.value), float(start.value))

    def time_stage(self, stage: str, reps: int = 20) -> float:
        """Mean ms per back-to-back launch of a repeatable stage on the finished frame."""
        ms = C.c_double(0.0)
        self._check(self.L.hwo_time_stage(self.h, STAGES.index(stage), int(reps), C.byref(ms)))
        return float(ms.value)

    @property
    def record_bytes(self) -> int:
        return int(self.L.hwo_record_bytes(self.h))
