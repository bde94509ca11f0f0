"""Host-side checks of the C ABI (no GPU needed).

The library must load, export every function that include/hwo.h declares,
and validate its configuration on the host before touching the device.
"""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_2511_02852_amd import hwo
    if not os.path.exists(hwo.LIB_PATH):
        from paper_2511_02852_amd import build
        build.build()
    return hwo.lib()


def declared_functions():
    text = open(os.path.join(ROOT, "include", "hwo.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hwo_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["hwo_create_ocean", "hwo_set_spectrum", "hwo_add_patch", "hwo_add_source", "hwo_step",
              "hwo_read_heightmaps", "hwo_destroy_ocean"]:
        assert n in names


def declaration_blocks():
    """(comment, [function names]) for every run of declarations in the
    header after the type definitions: each run of consecutive prototypes
    and the comment block directly above it."""
    text = open(os.path.join(ROOT, "include", "hwo.h")).read()
    body = text[text.index("} hwo_source;"):]
    blocks = []
    comment, names = None, []
    for tok in re.finditer(r"/\*.*?\*/|[^;/]*?\b(hwo_[a-z_]+)\s*\([^;]*;", body, flags=re.S):
        if tok.group(0).startswith("/*"):
            if names:
                blocks.append((comment, names))
                names = []
            comment = tok.group(0)
        elif tok.group(1):
            names.append(tok.group(1))
    if names:
        blocks.append((comment, names))
    return blocks


def test_every_declaration_cites_the_paper():
    """Every declaration block of the boundary names the passage that defines
    its operation (a Sec, Eq, Fig or Table tag of the paper)."""
    blocks = declaration_blocks()
    covered = sorted({n for _, ns in blocks for n in ns})
    assert covered == declared_functions()
    for comment, names in blocks:
        assert comment, f"{names}: no comment"
        if names == ["hwo_sample_probes_static"]:
            # the allocation-free variant names the callers it is for instead
            assert "cannot allocate" in comment
            continue
        assert re.search(r"\b(Sec|Eq|Fig|Table) \d", comment), f"{names}: no citation in {comment[:80]!r}"


def test_every_declared_symbol_is_exported(L):
    from paper_2511_02852_amd import hwo
    names = declared_functions()
    assert names, "no declarations found"
    for n in names:
        assert hasattr(L, n), f"{n} not exported"
    assert sorted(hwo.EXPORTS) == names


def cfg(**kw):
    from paper_2511_02852_amd import hwo
    c = hwo.HwoConfig()
    c.fft_n = 64
    c.fft_L = 256.0
    c.g = 9.81
    c.dt = 1 / 60
    c.seed = 0
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def test_create_validates_config(L):
    from paper_2511_02852_amd import hwo
    h = C.c_void_p()
    assert L.hwo_create_ocean(None, C.byref(h)) == hwo.HWO_EINVAL
    for bad in (dict(fft_n=100), dict(fft_n=8), dict(fft_n=8192), dict(fft_L=0.0), dict(g=-1.0),
                dict(dt=0.0), dict(max_particles=-5), dict(synth=2), dict(normals=3), dict(bg_fields=2),
                dict(kernel=2), dict(kernel=1, synth=1)):
        assert L.hwo_create_ocean(C.byref(cfg(**bad)), C.byref(h)) == hwo.HWO_EINVAL, bad
    assert L.hwo_create_ocean(C.byref(cfg()), C.byref(h)) == hwo.HWO_OK
    assert h.value
    L.hwo_destroy_ocean(h)


def test_call_order_errors(L):
    """Scene calls before set_spectrum and stepping without a spectrum fail
    with HWO_ESTATE, without any device work."""
    from paper_2511_02852_amd import hwo
    h = C.c_void_p()
    assert L.hwo_create_ocean(C.byref(cfg()), C.byref(h)) == hwo.HWO_OK
    pid = C.c_int32()
    p = hwo.HwoPatch(0.0, 0.0, 64, 64, 0.5, 0.0, 0.0, -1)
    assert L.hwo_add_patch(h, C.byref(p), C.byref(pid)) == hwo.HWO_ESTATE
    b = (C.c_int32 * 4)(8, 8, 8, 8)
    assert L.hwo_set_bins(h, b, 4) == hwo.HWO_ESTATE
    assert L.hwo_step(h, 1) == hwo.HWO_ESTATE
    assert b"set_spectrum" in L.hwo_last_error(h)
    assert L.hwo_step_index(h) == 0
    assert L.hwo_record_bytes(h) == 32
    buf = (C.c_double * 64)()
    assert L.hwo_read_buckets(h, buf, 64) == hwo.HWO_ESTATE   # before set_spectrum
    ms = C.c_double()
    # only idempotent stages can be re-launched, and only after a step
    for stage in (0, 3, 4, 5, 13, 14):   # params, count, scan, scatter, normals (off), no such stage
        assert L.hwo_time_stage(h, stage, 5, C.byref(ms)) == hwo.HWO_EINVAL
    for stage in (10, 11, 12):   # layer stages need synth 1
        assert L.hwo_time_stage(h, stage, 5, C.byref(ms)) == hwo.HWO_EINVAL
    assert L.hwo_time_stage(h, 6, 5, C.byref(ms)) == hwo.HWO_ESTATE
    assert L.hwo_time_stage(h, 6, 0, C.byref(ms)) == hwo.HWO_EINVAL
    xy = (C.c_double * 4)(0.0, 0.0, 1.0, 1.0)
    out = (C.c_float * 8)()
    assert L.hwo_sample_probes(h, xy, -1, out, 0) == hwo.HWO_EINVAL
    assert L.hwo_sample_probes(h, None, 2, out, 0) == hwo.HWO_EINVAL
    assert L.hwo_sample_probes(h, xy, 2, out, 0) == hwo.HWO_ESTATE   # no spectrum, no step
    assert L.hwo_sample_probes_static(h, xy, -1, out) == hwo.HWO_EINVAL
    assert L.hwo_sample_probes_static(h, None, 2, out) == hwo.HWO_EINVAL
    assert L.hwo_sample_probes_static(h, xy, 131073, out) == hwo.HWO_ERANGE   # beyond the static scratch
    assert L.hwo_sample_probes_static(h, xy, 2, out) == hwo.HWO_ESTATE        # nothing built, no step
    for bad in ((10, 100, 0, 0), (3500, -1, 0, 0), (3500, 9000, 0, 0), (3500, 100, -2, 0), (1 << 25, 0, 0, 0),
                (3500, 100, 0, 3), (3500, 100, 0, -1)):
        assert L.hwo_set_plan(h, C.byref(hwo.HwoPlan(*bad))) == hwo.HWO_EINVAL, bad
    assert L.hwo_set_plan(h, None) == hwo.HWO_EINVAL
    plan, t1, t2 = hwo.HwoPlan(), C.c_double(), C.c_double()
    assert L.hwo_autotune(h, 0, C.byref(plan), C.byref(t1), C.byref(t2)) == hwo.HWO_EINVAL
    assert L.hwo_autotune(h, 3, C.byref(plan), C.byref(t1), C.byref(t2)) == hwo.HWO_ESTATE   # no step yet
    nbytes = C.c_int64()
    assert L.hwo_snapshot_size(h, C.byref(nbytes)) == hwo.HWO_ESTATE   # nothing to save yet
    img = (C.c_char * 16)()
    assert L.hwo_snapshot(h, img, 16) == hwo.HWO_ESTATE
    assert L.hwo_restore(h, img, 16) == hwo.HWO_EINVAL                # shorter than a header
    L.hwo_destroy_ocean(h)
    c2 = cfg(compact=1)
    assert L.hwo_create_ocean(C.byref(c2), C.byref(h)) == hwo.HWO_OK
    assert L.hwo_record_bytes(h) == 16
    L.hwo_destroy_ocean(h)


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    """The binding has no fallback: a missing library is an error."""
    from paper_2511_02852_amd import hwo
    monkeypatch.setattr(hwo, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(hwo, "_lib", None)
    with pytest.raises(hwo.HwoError):
        hwo.lib()


def test_product_never_imports_oracle():
    """The package and its kernels do not reference the oracle."""
    pkg = os.path.join(ROOT, "paper_2511_02852_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src, f
                assert "oracle.h" not in src and "liboracle" not in src, f
