"""Host planner: turn a single-rate SPIIR bank into a multi-rate one (§2.2).

The paper assigns each filter to a sampling rate by its a1 coefficient: a1's
phase places the filter's passband, so it fixes the Nyquist rate the filter
needs, and the filter runs at the lowest available rate (base / 2^h) at or
above it.  This module makes that assignment and converts every filter to the
rate of its band, so that the multi-rate path (downsample, filter, upsample and
add) reproduces the single-rate output for signals inside the filter's band.

Readings (the paper gives the rule, not the formulas):

* A filter's band edge is |f_c| + width * f_w with f_c = arg(a1) R / 2pi (phase
  taken in (-pi, pi]) and f_w = (1 - |a1|) R / pi, the half-power half-width
  of a first-order resonance.  Band h is usable up to guard * R_h, R_h =
  R / 2^h, below its Nyquist rate because the 2x resampling filters have a
  transition band (guard = 0.35 for the default 32-tap, 60 dB filters).
* The resampling path of band h delays its signal by G_h base samples (below),
  which the filter's own delay must absorb: a filter only moves to band h if
  d >= G_h, else the start of its response would be lost (causality).
* Converting a filter to band h (D = 2^h): the band sees x delayed by the
  down path and its output is delayed again by the up path, G = ((T_d - 1) +
  (T_u - 1)) / 2 * (D - 1) base samples for linear-phase taps; the filter's
  own delay d absorbs that: d_h = ceil((d - G) / D).  At the lower rate the
  filter's pole is a1^D.  Its gain is set so that the band path's response to
  a tone at the filter's resonance (omega = arg a1) equals the single-rate
  filter's: with s = D d_h - (d - G) the remaining shift and r = |a1|,
  b0 -> b0 e^{i arg(a1) s} (1 - r^D) / (1 - r), i.e. D b0 a1^s up to
  O(D (1 - r)).  Away from resonance the first-order low-rate filter cannot
  match exactly: the error spectrum is roughly flat at |b0| D / 2, small
  against the resonance peak |b0| / (1 - r).
* Optional zero padding of every (template, band) filter count to a power of
  two, as the paper's bank configuration does (Table 5); zero filters add
  nothing to z.
"""
from __future__ import annotations

import numpy as np

from .workloads import BankTables, down_taps, up_taps

DEFAULT_GUARD = 0.35
DEFAULT_WIDTH = 3.0


def band_edge_hz(a1: np.ndarray, base_rate: float, width: float = DEFAULT_WIDTH) -> np.ndarray:
    """Upper edge of each filter's passband in Hz: |f_c| + width * f_w."""
    a1 = np.asarray(a1, np.complex128)
    fc = np.abs(np.angle(a1)) * base_rate / (2 * np.pi)
    fw = np.clip(1.0 - np.abs(a1), 0.0, None) * base_rate / np.pi
    return fc + width * fw


def assign_bands(a1: np.ndarray, base_rate: float, n_bands: int, delay=None, n_taps_down: int = 32,
                 n_taps_up: int = 32, guard: float = DEFAULT_GUARD,
                 width: float = DEFAULT_WIDTH) -> np.ndarray:
    """Band of each filter: the largest h < n_bands with edge <= guard * base_rate / 2^h and, when
    delays are given, d >= the band's path delay (0 if no lower band qualifies)."""
    edge = band_edge_hz(a1, base_rate, width)
    d = None if delay is None else np.asarray(delay, np.float64)
    h = np.zeros(edge.shape, np.int64)
    for b in range(1, n_bands):
        ok = edge <= guard * base_rate / (1 << b)
        if d is not None:
            ok &= d >= path_delay(b, n_taps_down, n_taps_up)
        h[ok] = b
    return h


def path_delay(h: int, n_taps_down: int, n_taps_up: int) -> float:
    """Base-rate group delay of band h's down and up resampling path (linear-phase taps)."""
    return ((n_taps_down - 1) + (n_taps_up - 1)) / 2.0 * ((1 << h) - 1)


def to_band(a1, b0, d, h: int, n_taps_down: int, n_taps_up: int):
    """Coefficients of filters moved from the base rate to band h: (a1_h, b0_h, d_h).
    Requires d >= the band's path delay (assign_bands guarantees it)."""
    a1 = np.asarray(a1, np.complex128)
    b0 = np.asarray(b0, np.complex128)
    d = np.asarray(d, np.float64)
    D = 1 << h
    if D == 1:
        return a1.copy(), b0.copy(), d.astype(np.int64)
    G = path_delay(h, n_taps_down, n_taps_up)
    if np.any(d < G):
        raise ValueError("a filter's delay is shorter than the band's resampling delay")
    dh = np.ceil((d - G) / D - 1e-9).astype(np.int64)
    s = D * dh - (d - G)
    r = np.abs(a1)
    # sum_{j<D} r^j: the gain of D base-rate steps at resonance
    gsum = np.where(np.abs(1.0 - r) > 1e-12, (1.0 - r ** D) / np.where(r == 1.0, 1.0, 1.0 - r), D)
    b_h = b0 * np.exp(1j * np.angle(a1) * s) * gsum
    return a1 ** D, b_h, dh


def plan_multirate(tables: BankTables, n_bands: int, n_taps_down: int = 32, n_taps_up: int = 32,
                   atten_down: float = 60.0, atten_up: float = 60.0, guard: float = DEFAULT_GUARD,
                   width: float = DEFAULT_WIDTH, pad_pow2: bool = False) -> BankTables:
    """Multi-rate tables from single-rate ones (n_bands == 1 on input)."""
    if tables.n_bands != 1:
        raise ValueError("plan_multirate takes a single-rate bank")
    if n_bands < 1:
        raise ValueError("n_bands must be >= 1")
    T = tables.n_templates
    off = tables.offsets()[:, 0]
    nf = np.zeros((T, n_bands), np.int32)
    a_out, b_out, d_out = [], [], []
    band = assign_bands(tables.a1, tables.base_rate, n_bands, tables.delay, n_taps_down, n_taps_up,
                        guard, width)
    for t in range(T):
        sl = slice(int(off[t]), int(off[t]) + int(tables.n_filters[t, 0]))
        for h in range(n_bands):
            sel = np.nonzero(band[sl] == h)[0] + sl.start
            a_h, b_h, d_h = to_band(tables.a1[sel], tables.b0[sel], tables.delay[sel], h,
                                    n_taps_down, n_taps_up)
            m = len(sel)
            if pad_pow2 and m > 0:
                m2 = 1 << int(np.ceil(np.log2(m)))
                pad = m2 - m
                a_h = np.concatenate([a_h, np.zeros(pad, np.complex128)])
                b_h = np.concatenate([b_h, np.zeros(pad, np.complex128)])
                d_h = np.concatenate([d_h, np.zeros(pad, np.int64)])
                m = m2
            nf[t, h] = m
            a_out.append(a_h)
            b_out.append(b_h)
            d_out.append(d_h)
    cat = lambda xs, dt: np.concatenate(xs).astype(dt) if xs else np.zeros(0, dt)
    return BankTables(
        base_rate=tables.base_rate,
        n_filters=nf,
        a1=cat(a_out, np.complex128),
        b0=cat(b_out, np.complex128),
        delay=cat(d_out, np.int32),
        h_down=down_taps(n_taps_down, atten_down) if n_bands > 1 else np.ones(1),
        h_up=up_taps(n_taps_up, atten_up) if n_bands > 1 else np.ones(1),
    )


def filter_samples_saved(tables: BankTables, planned: BankTables, n: int) -> float:
    """Fraction of filter-samples per block the multi-rate bank saves (the paper's cost model)."""
    return 1.0 - planned.filter_samples_per_block(n) / tables.filter_samples_per_block(n)


__all__ = ["band_edge_hz", "assign_bands", "path_delay", "to_band", "plan_multirate",
           "filter_samples_saved", "DEFAULT_GUARD", "DEFAULT_WIDTH"]
