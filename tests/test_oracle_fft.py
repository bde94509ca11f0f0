"""Pins of the oracle's FFT background (CPU only)."""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
from paper_2511_02852_amd import scenes


def rand_c(n, seed):
    r = np.random.default_rng(seed)
    return r.standard_normal((n, n)) + 1j * r.standard_normal((n, n))


@pytest.mark.parametrize("n", [2, 4, 8, 16])
def test_fft_matches_naive_dft(n):
    """Radix-2 FFT against the O(N^4) definition, e^{+i} kernel, no 1/N^2."""
    z = rand_c(n, n)
    a = oracle.fft2_inverse(z)
    b = oracle.dft2_inverse(z)
    assert np.max(np.abs(a - b)) <= 1e-12 * max(1.0, np.max(np.abs(b)))


@pytest.mark.parametrize("n", [32, 64, 256, 1024])
def test_fft_matches_numpy(n):
    """Against numpy.fft (pocketfft): ifft2 scaled by N^2."""
    z = rand_c(n, 100 + n)
    a = oracle.fft2_inverse(z)
    b = np.fft.ifft2(z) * (n * n)
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))


def test_parseval():
    n = 128
    z = rand_c(n, 7)
    a = oracle.fft2_inverse(z)
    assert np.sum(np.abs(a) ** 2) == pytest.approx(n * n * np.sum(np.abs(z) ** 2), rel=1e-12)


def test_h0_hermitian_real_background():
    """h~(-k) = conj(h~(k)) by construction, so the inverse transform of the
    evolved spectrum is real: the oracle's H equals the real part and the
    imaginary part of the full transform vanishes."""
    s = scenes.c1()
    o = oracle.Oracle(s)
    N = s.fft_n
    h0 = o.h0()
    assert h0[0, 0] == 0
    t = 0.37
    dk = 2 * math.pi / s.fft_L
    m = np.fft.fftfreq(N, 1.0 / N)
    kx, ky = np.meshgrid(dk * m, dk * m)
    w = np.sqrt(s.g * np.hypot(kx, ky))
    neg = np.roll(np.flip(h0, (0, 1)), 1, (0, 1))  # h0(-k)
    ht = h0 * np.exp(-1j * w * t) + np.conj(neg) * np.exp(1j * w * t)
    full = oracle.fft2_inverse(ht)
    H = o.background(t)
    assert np.max(np.abs(full.imag)) <= 1e-12 * np.max(np.abs(full.real))
    assert np.max(np.abs(full.real - H)) <= 1e-12 * np.max(np.abs(H))


@pytest.mark.parametrize("mode", [(3, 0), (0, 5), (-4, 7), (11, -2)])
def test_single_mode_phase_speed(mode):
    """One spectral mode h0(k0) = a e^{i phi}: H(x, t) = 2 a cos(k0.x - w t + phi)
    with w = sqrt(g |k0|), i.e. a plane wave at the deep-water phase speed
    sqrt(g / k) (Sec 3.2: w^2 = g k)."""
    s = scenes.c1()
    o = oracle.Oracle(s)
    N, L, g = s.fft_n, s.fft_L, s.g
    mx, my = mode
    z = np.zeros((N, N), dtype=complex)
    a, phi = 0.3, 0.7
    z[my % N, mx % N] = a * np.exp(1j * phi)
    o.set_h0(z)
    k0 = 2 * math.pi / L * np.array([mx, my])
    w = math.sqrt(g * np.linalg.norm(k0))
    x = np.arange(N) * L / N
    X, Y = np.meshgrid(x, x)
    for t in (0.0, 0.5, 3.25, 17.0):
        H = o.background(t)
        want = 2 * a * np.cos(k0[0] * X + k0[1] * Y - w * t + phi)
        assert np.max(np.abs(H - want)) <= 1e-11
    # phase speed: a crest moves a distance (w / |k|) t along k
    assert w / np.linalg.norm(k0) == pytest.approx(math.sqrt(g / np.linalg.norm(k0)), rel=1e-14)


def test_background_variance_matches_spectrum():
    """Unit-modulus h0: the time-averaged variance of H is sum_k S_k dk^2,
    which approximates m0 = int S_J dw (Dir integrates to 1) over the band the
    grid resolves.  c1: 64^2 over 256 m resolves k in [2pi/256, pi/4]."""
    s = scenes.c1()
    s.spectrum.h0_mode = 1
    o = oracle.Oracle(s)
    ts = np.linspace(0, 200, 41)
    var = np.mean([np.var(o.background(t)) for t in ts])
    g = s.g
    kmin = 2 * math.pi / s.fft_L
    kmax = math.pi * s.fft_n / s.fft_L
    wlo, whi = math.sqrt(g * kmin), math.sqrt(g * kmax)
    m0, _ = integrate.quad(o.jonswap, wlo, whi, limit=400)
    # grid quadrature of a peaked spectrum with 4 m cells: a few percent
    assert var == pytest.approx(m0, rel=0.05)
    # Gaussian amplitudes have the same expected power per mode: the ratio
    # |h0_gauss|^2 / |h0_unit|^2 = rho^2 / 2 with rho^2 ~ Exp(mean 2)
    s2 = scenes.c1()
    og = oracle.Oracle(s2)
    pg = np.abs(og.h0()) ** 2
    pu = np.abs(o.h0()) ** 2
    ok = pu > 0
    ratio = pg[ok] / pu[ok]
    assert ratio.size > 4000
    assert ratio.mean() == pytest.approx(1.0, abs=4.0 / math.sqrt(ratio.size))
    assert ratio.var() == pytest.approx(1.0, abs=0.15)


@pytest.mark.parametrize("mode", [(3, 0), (0, 5), (-4, 7), (11, -2)])
def test_slope_and_choppy_fields_of_a_single_mode(mode):
    """Derived background fields of one spectral mode h0(k0) = a e^{i phi},
    H = 2a cos(theta) with theta = k0.x - w t + phi: the slopes are the exact
    derivatives -2a k0x sin(theta), -2a k0y sin(theta), and the choppy
    displacement sum -i (k/|k|) h~ e^{ik.x} is (k0 / |k0|) 2a sin(theta)."""
    s = scenes.c1()
    o = oracle.Oracle(s)
    N, L, g = s.fft_n, s.fft_L, s.g
    mx, my = mode
    z = np.zeros((N, N), dtype=complex)
    a, phi = 0.3, 0.7
    z[my % N, mx % N] = a * np.exp(1j * phi)
    o.set_h0(z)
    k0 = 2 * math.pi / L * np.array([mx, my])
    kn = np.linalg.norm(k0)
    w = math.sqrt(g * kn)
    x = np.arange(N) * L / N
    X, Y = np.meshgrid(x, x)
    for t in (0.0, 3.25):
        th = k0[0] * X + k0[1] * Y - w * t + phi
        want = {1: -2 * a * k0[0] * np.sin(th), 2: -2 * a * k0[1] * np.sin(th),
                3: 2 * a * k0[0] / kn * np.sin(th), 4: 2 * a * k0[1] / kn * np.sin(th)}
        for f, v in want.items():
            assert np.max(np.abs(o.background_field(f, t) - v)) <= 1e-11, (f, t)


def test_derived_fields_are_spectral_derivatives_of_the_height():
    """On a full spectrum the derived fields are the spectral derivative and
    the Riesz transform of the oracle's own height field: numpy's FFT of H,
    times i kx, i ky or -i k/|k| (Nyquist rows and columns and k = 0
    dropped), transformed back, reproduces fields 1-4.  This ties the derived
    transforms to the height transform through an independent FFT."""
    s = scenes.c1()
    s.spectrum.h0_mode = 1
    o = oracle.Oracle(s)
    N, L = s.fft_n, s.fft_L
    t = 1.5
    Hk = np.fft.fft2(o.background(t))
    m = np.fft.fftfreq(N, 1.0 / N)
    KX, KY = np.meshgrid(2 * math.pi / L * m, 2 * math.pi / L * m)
    keep = (np.abs(np.meshgrid(m, m)[0]) != N // 2) & (np.abs(np.meshgrid(m, m)[1]) != N // 2)
    kk = np.hypot(KX, KY)
    inv = np.where(kk > 0, 1.0 / np.where(kk > 0, kk, 1.0), 0.0)
    mult = {1: 1j * KX, 2: 1j * KY, 3: -1j * KX * inv, 4: -1j * KY * inv}
    for f, mk in mult.items():
        want = np.fft.ifft2(Hk * mk * keep)
        got = o.background_field(f, t)
        assert np.max(np.abs(want.imag)) <= 1e-12 * np.max(np.abs(want.real))
        assert np.max(np.abs(got - want.real)) <= 1e-10 * np.max(np.abs(want.real)), f
