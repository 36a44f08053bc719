"""Host planner (single-rate bank -> multi-rate bank, §2.2), checked with the
FP64 oracle: the assignment rule by brute force, exact identities, the
response at each filter's resonance per band, and the match (normalised
correlation, the fraction of SNR kept) of the whole planned bank."""
import numpy as np
import pytest

import oracle
from paper_1702_02256_amd import planner as PL
from paper_1702_02256_amd import workloads as W

R = 4096


def _bank(seed=3, M=64, fmax=700.0):
    rng = np.random.default_rng(seed)
    f = rng.uniform(5, fmax, M) * rng.choice([-1, 1], M)
    r = rng.uniform(0.995, 0.9995, M)
    a1 = r * np.exp(2j * np.pi * f / R)
    b0 = (rng.standard_normal(M) + 1j * rng.standard_normal(M)) * 1e-3
    d = rng.integers(0, 2048, M).astype(np.int32)
    return W.BankTables(base_rate=R, n_filters=np.array([[M]], np.int32), a1=a1, b0=b0, delay=d)


def test_assignment_rule_brute_force():
    tb = _bank(seed=11, M=400, fmax=1500)
    H = 6
    got = PL.assign_bands(tb.a1, R, H, tb.delay)
    for a, d, g in zip(tb.a1, tb.delay, got):
        edge = abs(np.angle(a)) * R / (2 * np.pi) + 3.0 * (1 - abs(a)) * R / np.pi
        want = 0
        for h in range(1, H):
            if edge <= 0.35 * R / 2 ** h and d >= 31 * (2 ** h - 1):
                want = h
        assert g == want
    assert len(set(got.tolist())) >= 4  # the draw spreads over several bands


def test_band_zero_is_identity_and_short_delays_are_refused():
    tb = _bank()
    a, b, d = PL.to_band(tb.a1, tb.b0, tb.delay, 0, 32, 32)
    assert np.array_equal(a, tb.a1) and np.array_equal(b, tb.b0) and np.array_equal(d, tb.delay)
    with pytest.raises(ValueError):
        PL.to_band(np.array([0.99 + 0j]), np.array([1e-3 + 0j]), np.array([10]), 2, 32, 32)
    assert PL.path_delay(3, 32, 32) == 31 * 7


@pytest.mark.parametrize("h", [1, 2, 3, 4])
def test_tone_at_resonance_matches_single_rate(h):
    # one filter moved to band h, driven by a tone at its resonance: the band path
    # reproduces the single-rate response to the passband ripple of the 2h
    # resampling stages (about 1e-3 each for 32-tap, 60 dB filters)
    worst = 0.0
    for f, r, d in ((10.0, 0.999, 1500), (-0.3 * R / 2 ** h, 0.9995, 1900), (40.0, 0.999, 900)):
        a1 = np.array([r * np.exp(2j * np.pi * f / R)])
        b0 = np.array([1e-3 - 2e-4j])
        tb = W.BankTables(base_rate=R, n_filters=np.array([[1]], np.int32), a1=a1, b0=b0,
                          delay=np.array([d], np.int32))
        ah, bh, dh = PL.to_band(a1, b0, np.array([d]), h, 32, 32)
        nf = np.zeros((1, 5), np.int32)
        nf[0, h] = 1
        pl = W.BankTables(base_rate=R, n_filters=nf, a1=ah, b0=bh, delay=dh.astype(np.int32),
                          h_down=W.down_taps(32), h_up=W.up_taps(32))
        x = np.cos(2 * np.pi * f * np.arange(8 * R) / R)
        z1, z2 = oracle.run_stream(tb, x), oracle.run_stream(pl, x)
        sl = slice(6 * R, None)
        worst = max(worst, np.abs(z1[0, sl] - z2[0, sl]).max() / np.abs(z1[0, sl]).max())
    assert worst <= 1e-2, worst


def test_planned_bank_keeps_the_snr():
    tb = _bank()
    pl = PL.plan_multirate(tb, 5)
    assert pl.n_filters.sum() == tb.n_filters.sum()
    saved = PL.filter_samples_saved(tb, pl, 4096)
    assert saved > 0.4  # most filters run at lower rates
    rng = np.random.default_rng(7)
    n = 8 * R
    x = rng.standard_normal(n)
    X = np.fft.rfft(x)
    X[np.fft.rfftfreq(n, 1 / R) > 800] = 0
    x = np.fft.irfft(X, n)
    z1, z2 = oracle.run_stream(tb, x)[0, 3 * R:], oracle.run_stream(pl, x)[0, 3 * R:]
    match = abs(np.vdot(z1, z2)) / np.linalg.norm(z1) / np.linalg.norm(z2)
    assert match >= 0.995, match


def test_pow2_padding_changes_nothing():
    tb = W.BankTables(base_rate=R, n_filters=np.array([[64], [64]], np.int32),
                      a1=np.concatenate([_bank(1).a1, _bank(2).a1]),
                      b0=np.concatenate([_bank(1).b0, _bank(2).b0]),
                      delay=np.concatenate([_bank(1).delay, _bank(2).delay]))
    a = PL.plan_multirate(tb, 5)
    b = PL.plan_multirate(tb, 5, pad_pow2=True)
    nz = b.n_filters[b.n_filters > 0]
    assert np.all((nz & (nz - 1)) == 0) and np.all(b.n_filters >= a.n_filters)
    x = W.noise_stream(5, 2 * R)
    assert np.array_equal(oracle.run_stream(a, x), oracle.run_stream(b, x))
