"""Pins of the oracle's power-spectrum estimator (no GPU).

The estimator (objective.power_spectrum) takes the half spectrum of a real
field with Hermitian weights; the pins compare it with a brute-force sum over
every mode of the full complex spectrum, with single Fourier modes of known
amplitude, with Parseval's identity and with the flat spectrum of white noise.
P is defined through <delta(k) delta(k')> = V P(k) (Sec. 2.1, eq. Plin), so a
field with unit-variance white noise has P = V / N_c per mode.
"""
import numpy as np
import pytest

from oracle import objective
from paper_2211_09815_amd import inputs


def _brute_force_spectrum(delta, box):
    """Every mode of the full complex FFT, no Hermitian symmetry used: shell
    b = round(|m|) for b = 1..n/2, P = mean of |delta(k) V / N_c|^2 / V."""
    n = delta.shape[0]
    V = box ** 3
    dk = np.fft.fftn(delta) * (V / delta.size)
    m = np.fft.fftfreq(n) * n
    cnt = np.zeros(n // 2)
    ps = np.zeros(n // 2)
    ks = np.zeros(n // 2)
    for idx in np.ndindex(delta.shape):
        mag = np.sqrt(m[idx[0]] ** 2 + m[idx[1]] ** 2 + m[idx[2]] ** 2)
        b = int(np.floor(mag + 0.5))
        if 1 <= b <= n // 2:
            cnt[b - 1] += 1
            ps[b - 1] += abs(dk[idx]) ** 2 / V
            ks[b - 1] += mag
    return ks / cnt * (2 * np.pi / box), ps / cnt, cnt


def _spectrum_error(estimator, delta, box):
    k, P, c = estimator(delta, box)
    kb, Pb, cb = _brute_force_spectrum(delta, box)
    return max(np.abs(c - cb).max(), np.abs(k - kb).max() / kb.max(), np.abs(P - Pb).max() / Pb.max())


def _cosine(n, m, amp=1.0):
    g = np.stack(np.meshgrid(*[np.arange(n, dtype=float)] * 3, indexing="ij"))
    return amp * np.cos(2 * np.pi * (m[0] * g[0] + m[1] * g[1] + m[2] * g[2]) / n + 0.4)


def _single_mode_error(estimator, n=16, box=50.0):
    """A cosine of amplitude A has mean square A^2/2 (A^2 at the Nyquist
    frequency, where cos(pi z + phase) = cos(phase) (-1)^z), all of it in the
    shell round(|m|): P cnt = V A^2 / 2 there and zero elsewhere."""
    V = box ** 3
    err = 0.0
    for m in ((3, 0, 0), (0, 0, 3), (1, 2, 2), (2, 2, 0), (0, 5, 1), (0, 0, n // 2)):
        amp = 0.7
        delta = _cosine(n, m, amp)
        _, P, c = estimator(delta, box)
        tot = np.nan_to_num(P * c)
        b = int(np.floor(np.sqrt(sum(x * x for x in m)) + 0.5))
        want = V * np.mean(delta ** 2)
        err = max(err, abs(tot[b - 1] - want) / want, np.abs(np.delete(tot, b - 1)).max() / want)
    return err


def test_power_spectrum_matches_full_spectrum_brute_force():
    for n, seed in ((8, 11), (12, 12)):
        delta = inputs.normal((n, n, n), seed)
        assert _spectrum_error(objective.power_spectrum, delta, 37.0) < 1e-12


def test_power_spectrum_single_modes():
    assert _single_mode_error(objective.power_spectrum) < 1e-12


def test_power_spectrum_parseval_and_white_noise():
    # sum_b P_b cnt_b = V mean(delta^2) for a field whose modes all lie in
    # shells 1..n/2; white noise of variance sigma^2 has P = V sigma^2 / N_c
    n, box = 32, 100.0
    m = np.fft.fftfreq(n) * n
    MX, MY, MZ = np.meshgrid(m, m, np.fft.rfftfreq(n) * n, indexing="ij")
    band = (np.sqrt(MX ** 2 + MY ** 2 + MZ ** 2) < n // 2 - 0.5) & ((MX != 0) | (MY != 0) | (MZ != 0))
    delta = np.fft.irfftn(np.where(band, np.fft.rfftn(inputs.normal((n, n, n), 13)), 0), s=(n, n, n), axes=(0, 1, 2))
    _, P, c = objective.power_spectrum(delta, box)
    assert np.nansum(P * c) == pytest.approx(box ** 3 * np.mean(delta ** 2), rel=1e-12)
    sigma = 1.7
    _, P, c = objective.power_spectrum(inputs.normal((n, n, n), 14, scale=sigma), box)
    flat = box ** 3 * sigma ** 2 / n ** 3
    assert np.sum(P * c) / np.sum(c) == pytest.approx(flat, rel=0.01)
    assert np.all(np.abs(P[3:] / flat - 1) < 5 / np.sqrt(c[3:]))


def test_power_spectrum_pins_catch_planted_mistakes():
    def variant(weight_two=True, rounding=True, norm=1.0):
        def est(delta, box):
            n = delta.shape[0]
            V = box ** 3
            dk = np.fft.rfftn(delta) * (V / delta.size) * norm
            m = np.fft.fftfreq(n) * n
            MX, MY, MZ = np.meshgrid(m, m, np.fft.rfftfreq(n) * n, indexing="ij")
            kmag = np.sqrt(MX ** 2 + MY ** 2 + MZ ** 2)
            w = np.full(MZ.shape, 2.0 if weight_two else 1.0)
            w[..., 0] = 1.0
            w[..., -1] = 1.0
            b = np.floor(kmag + (0.5 if rounding else 0.0)).astype(int)
            sel = (b >= 1) & (b <= n // 2)
            cnt = np.bincount(b[sel], weights=w[sel], minlength=n // 2 + 1)[1:]
            ps = np.bincount(b[sel], weights=(w * np.abs(dk) ** 2 / V)[sel], minlength=n // 2 + 1)[1:]
            ks = np.bincount(b[sel], weights=(w * kmag)[sel], minlength=n // 2 + 1)[1:]
            with np.errstate(invalid="ignore", divide="ignore"):
                return ks / cnt * (2 * np.pi / box), ps / cnt, cnt
        return est

    good = variant()
    delta = inputs.normal((8, 8, 8), 11)
    assert _spectrum_error(good, delta, 37.0) < 1e-12
    for bad in (variant(weight_two=False), variant(rounding=False), variant(norm=np.sqrt(8.0))):
        assert _spectrum_error(bad, delta, 37.0) > 1e-3
        assert _single_mode_error(bad) > 1e-3
