"""Seeded synthetic inputs with the shapes of the paper's SPIIR workloads.

This module only *generates inputs*: filter tables (a1, b0, d), resampling taps and
white-noise streams.  It holds none of the filtering arithmetic, so both the FP64
oracle (test infrastructure) and the HIP library can take their inputs from it
without sharing any of the method's computation.

Stand-ins for data the paper used but that is not available here:

* whitened detector strain (paper §2.1, Eq. 2: whitening makes the noise white)
  -> i.i.d. N(0, 1) samples;
* SPIIR filter tables built from CBC templates (§2.1, the construction is only
  referenced, not given) -> random first-order filters a1 = r e^{i theta},
  complex-normal b0 scaled by 1e-3 and uniform integer delays;
* gstreamer's Kaiser resampling filters (§2.2, Eq. 9 and the text after it)
  -> our own Kaiser-windowed sinc design (Kaiser's published window and beta
  formula), causal, 2x polyphase.

Every table for template t is drawn from ``numpy.random.default_rng([seed, t])``
so any subset of templates can be regenerated exactly without drawing the rest.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# --------------------------------------------------------------------------
# Resampling taps (inputs to both sides; parity does not depend on their values)
# --------------------------------------------------------------------------


def kaiser_beta(atten_db: float) -> float:
    """Kaiser's empirical beta for a stop-band attenuation in dB."""
    a = float(atten_db)
    if a > 50.0:
        return 0.1102 * (a - 8.7)
    if a >= 21.0:
        return 0.5842 * (a - 21.0) ** 0.4 + 0.07886 * (a - 21.0)
    return 0.0


def kaiser_lowpass(n_taps: int, cutoff: float, atten_db: float = 60.0) -> np.ndarray:
    """Kaiser-windowed sinc low-pass, causal, ``n_taps`` long, unit DC gain.

    ``cutoff`` is relative to the Nyquist frequency of the rate the filter runs
    at (0.5 = half-band, the 2x resampling case).  The design matches
    ``scipy.signal.firwin(n_taps, cutoff, window=('kaiser', beta))``.
    """
    n = np.arange(n_taps, dtype=np.float64)
    centre = (n_taps - 1) / 2.0
    ideal = cutoff * np.sinc(cutoff * (n - centre))
    h = ideal * np.kaiser(n_taps, kaiser_beta(atten_db))
    return h / h.sum()


def down_taps(n_taps: int = 32, atten_db: float = 60.0) -> np.ndarray:
    """Anti-alias taps for one /2 stage: half-band low-pass, sum = 1 (DC gain 1)."""
    return kaiser_lowpass(n_taps, 0.5, atten_db)


def up_taps(n_taps: int = 32, atten_db: float = 60.0) -> np.ndarray:
    """Interpolation taps for one x2 stage applied to the zero-stuffed signal.

    Each polyphase branch (even taps, odd taps) is normalised to sum to 1, so a
    constant input at the low rate gives the same constant at the high rate and
    the total gain is 2, compensating for the inserted zeros.
    """
    h = kaiser_lowpass(n_taps, 0.5, atten_db) * 2.0
    for phase in (0, 1):
        s = h[phase::2].sum()
        h[phase::2] /= s
    return h


# --------------------------------------------------------------------------
# Filter banks
# --------------------------------------------------------------------------


@dataclass
class BankTables:
    """Per-template, per-band SPIIR tables in (template, band, filter) order.

    This is the layout the C ABI's ``spiir_bank_desc`` reads and the oracle
    consumes: ``n_filters[t, h]`` filters for template t at band h (rate
    ``base_rate / 2**h``), followed by their complex a1, complex b0 and integer
    delay (in samples at the band's own rate).
    """

    base_rate: int
    n_filters: np.ndarray  # int32 [T, H]
    a1: np.ndarray  # complex128 [sum(n_filters)]
    b0: np.ndarray  # complex128 [sum(n_filters)]
    delay: np.ndarray  # int32 [sum(n_filters)]
    h_down: np.ndarray = field(default_factory=lambda: np.ones(1))
    h_up: np.ndarray = field(default_factory=lambda: np.ones(1))

    @property
    def n_templates(self) -> int:
        return int(self.n_filters.shape[0])

    @property
    def n_bands(self) -> int:
        return int(self.n_filters.shape[1])

    @property
    def total_filters(self) -> int:
        return int(self.n_filters.sum())

    def offsets(self) -> np.ndarray:
        """Start index of each (t, h) segment in the flat filter arrays, [T, H]."""
        flat = self.n_filters.reshape(-1).astype(np.int64)
        off = np.concatenate([[0], np.cumsum(flat)[:-1]])
        return off.reshape(self.n_filters.shape)

    def subset(self, templates) -> "BankTables":
        """Tables restricted to the listed templates (kept in the given order)."""
        templates = np.asarray(templates, dtype=np.int64)
        off = self.offsets()
        idx = []
        for t in templates:
            for h in range(self.n_bands):
                o = off[t, h]
                idx.append(np.arange(o, o + self.n_filters[t, h], dtype=np.int64))
        idx = np.concatenate(idx) if idx else np.zeros(0, np.int64)
        return BankTables(
            base_rate=self.base_rate,
            n_filters=self.n_filters[templates].copy(),
            a1=self.a1[idx].copy(),
            b0=self.b0[idx].copy(),
            delay=self.delay[idx].copy(),
            h_down=self.h_down.copy(),
            h_up=self.h_up.copy(),
        )

    def rounded_coefficients(self) -> "BankTables":
        """Copy with a1 and b0 rounded to complex64 and widened back (the
        tables as an FP32 device holds them), for splitting error sources."""
        return BankTables(
            base_rate=self.base_rate,
            n_filters=self.n_filters.copy(),
            a1=self.a1.astype(np.complex64).astype(np.complex128),
            b0=self.b0.astype(np.complex64).astype(np.complex128),
            delay=self.delay.copy(),
            h_down=self.h_down.copy(),
            h_up=self.h_up.copy(),
        )

    def filter_samples_per_block(self, n: int) -> int:
        """Sum over (t, h) of M_{t,h} * n / 2**h: filter-samples for an n-sample block."""
        per_band = self.n_filters.sum(axis=0).astype(np.int64)
        return int(sum(int(per_band[h]) * (n >> h) for h in range(self.n_bands)))


def _draw_filters(rng: np.random.Generator, m: int, d_max: int):
    """Draw m filters in the fixed order r, theta, b0.re, b0.im, d."""
    r = rng.uniform(0.9, 0.9999, m)
    theta = rng.uniform(0.0, 2.0 * np.pi, m)
    b_re = rng.standard_normal(m) * 1e-3
    b_im = rng.standard_normal(m) * 1e-3
    d = rng.integers(0, d_max + 1, m)
    a1 = r * np.exp(1j * theta)
    return a1, b_re + 1j * b_im, d.astype(np.int32)


def random_bank(
    seed: int,
    n_filters: np.ndarray,
    base_rate: int,
    d_max_per_band,
    n_taps_down: int = 32,
    n_taps_up: int = 32,
) -> BankTables:
    """Tables with the given per-(template, band) filter counts.

    ``d_max_per_band[h]`` is the largest delay drawn for band h.  Each template
    t draws from ``default_rng([seed, t])``, band by band.
    """
    n_filters = np.asarray(n_filters, dtype=np.int32)
    T, H = n_filters.shape
    a_parts, b_parts, d_parts = [], [], []
    for t in range(T):
        rng = np.random.default_rng([seed, t])
        for h in range(H):
            a, b, d = _draw_filters(rng, int(n_filters[t, h]), int(d_max_per_band[h]))
            a_parts.append(a)
            b_parts.append(b)
            d_parts.append(d)
    cat = lambda p, dt: np.concatenate(p).astype(dt) if p else np.zeros(0, dt)
    return BankTables(
        base_rate=base_rate,
        n_filters=n_filters,
        a1=cat(a_parts, np.complex128),
        b0=cat(b_parts, np.complex128),
        delay=cat(d_parts, np.int32),
        h_down=down_taps(n_taps_down) if H > 1 else np.ones(1),
        h_up=up_taps(n_taps_up) if H > 1 else np.ones(1),
    )


def noise_stream(seed: int, n: int, stream: int = 0) -> np.ndarray:
    """White N(0, 1) float64 samples standing in for whitened strain."""
    rng = np.random.default_rng([seed, 1_000_000 + stream])
    return rng.standard_normal(n)


# --------------------------------------------------------------------------
# The five workload shapes
# --------------------------------------------------------------------------

SEED_BASE = 1000


@dataclass
class Workload:
    name: str
    bank: BankTables
    block: int  # samples per block at the base rate
    n_blocks: int
    seed: int

    @property
    def n_samples(self) -> int:
        return self.block * self.n_blocks

    def stream(self, stream: int = 0) -> np.ndarray:
        return noise_stream(self.seed, self.n_samples, stream)


def config1(seed: int = SEED_BASE + 1) -> Workload:
    """Plain SPIIR, single rate: 1 template x 128 filters, 4096 Hz, d <= 2047, 1 s."""
    nf = np.full((1, 1), 128, np.int32)
    bank = random_bank(seed, nf, 4096, [2047])
    return Workload("cfg1-single-rate-1x128", bank, 4096, 1, seed)


def config2(seed: int = SEED_BASE + 2, n_templates: int = 1024, n_blocks: int = 16,
            templates=None) -> Workload:
    """Single rate: n_templates x 512 filters, 2048 Hz, d <= 4095, 1 s blocks."""
    nf = np.full((n_templates, 1), 512, np.int32)
    bank = random_bank(seed, nf, 2048, [4095])
    if templates is not None:
        bank = bank.subset(templates)
    return Workload(f"cfg2-single-rate-{n_templates}x512", bank, 2048, n_blocks, seed)


MULTIRATE_BANDS = 7


def multirate_counts(seed: int, n_templates: int, n_bands: int = MULTIRATE_BANDS,
                     lo: int = 40, hi: int = 300) -> np.ndarray:
    """Filters per (template, band): uniform integers in [lo, hi]."""
    rng = np.random.default_rng([seed, 2_000_000])
    return rng.integers(lo, hi + 1, size=(n_templates, n_bands)).astype(np.int32)


def multirate_dmax(base_rate: int, n_bands: int) -> list:
    """Delays span half a second at each band's own rate: d <= R_h/2 - 1."""
    return [max((base_rate >> h) // 2 - 1, 0) for h in range(n_bands)]


def config3(seed: int = SEED_BASE + 3, n_templates: int = 4096, n_blocks: int = 64,
            block: int = 4096, templates=None) -> Workload:
    """Multi-rate: 7 bands 4096..64 Hz, U{40..300} filters per band, 32/32 taps."""
    nf = multirate_counts(seed, n_templates)
    if templates is not None:
        templates = np.asarray(templates)
        nf_sel = nf[templates]
    rate = 4096
    dmax = multirate_dmax(rate, MULTIRATE_BANDS)
    if templates is None:
        bank = random_bank(seed, nf, rate, dmax)
    else:
        bank = _random_bank_rows(seed, nf_sel, templates, rate, dmax)
    return Workload(f"cfg3-multirate-{n_templates}x7band", bank, block, n_blocks, seed)


def _random_bank_rows(seed, nf_rows, template_ids, rate, dmax):
    """Like random_bank, but row i is drawn as template ``template_ids[i]``."""
    a_parts, b_parts, d_parts = [], [], []
    for i, t in enumerate(template_ids):
        rng = np.random.default_rng([seed, int(t)])
        for h in range(nf_rows.shape[1]):
            a, b, d = _draw_filters(rng, int(nf_rows[i, h]), int(dmax[h]))
            a_parts.append(a)
            b_parts.append(b)
            d_parts.append(d)
    return BankTables(
        base_rate=rate,
        n_filters=np.asarray(nf_rows, np.int32),
        a1=np.concatenate(a_parts),
        b0=np.concatenate(b_parts),
        delay=np.concatenate(d_parts).astype(np.int32),
        h_down=down_taps(32),
        h_up=up_taps(32),
    )


def uneven_counts(seed: int, n_templates: int, n_bands: int = MULTIRATE_BANDS,
                  lo: int = 16, hi: int = 1024) -> np.ndarray:
    """Uneven banks: total M log-uniform in [lo, hi]; 1..n_bands active bands.

    The top band is always active, B-1 other bands are picked at random, and M
    is split multinomially over the active bands with at least one each.
    """
    rng = np.random.default_rng([seed, 3_000_000])
    out = np.zeros((n_templates, n_bands), np.int32)
    for t in range(n_templates):
        m = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        nb = int(rng.integers(1, n_bands + 1))
        others = rng.permutation(np.arange(1, n_bands))[: nb - 1]
        bands = np.concatenate([[0], np.sort(others)]).astype(np.int64)
        nb = len(bands)
        m = max(m, nb)
        split = rng.multinomial(m - nb, np.full(nb, 1.0 / nb)) + 1
        out[t, bands] = split
    return out


def config4(seed: int = SEED_BASE + 4, n_templates: int = 8192, n_blocks: int = 64,
            block: int = 4096, templates=None) -> Workload:
    """Batched uneven banks: M log-U[16, 1024] over 1..7 active bands."""
    nf = uneven_counts(seed, n_templates)
    rate = 4096
    dmax = multirate_dmax(rate, MULTIRATE_BANDS)
    if templates is None:
        bank = random_bank(seed, nf, rate, dmax)
    else:
        templates = np.asarray(templates)
        bank = _random_bank_rows(seed, nf[templates], templates, rate, dmax)
    return Workload(f"cfg4-uneven-{n_templates}", bank, block, n_blocks, seed)


def serving_banks(seed: int = SEED_BASE + 5, n_templates: int = 16384, n_streams: int = 3):
    """Serving: config-3-shaped templates split evenly over one bank per stream."""
    sizes = [n_templates // n_streams + (1 if s < n_templates % n_streams else 0)
             for s in range(n_streams)]
    banks = []
    for s, sz in enumerate(sizes):
        banks.append(config3(seed=seed * 10 + s, n_templates=sz, n_blocks=1).bank)
    return banks


def serving_arrivals(seed: int, n_streams: int, duration_s: float, rate_hz: int = 4096,
                     speed: float = 1.0, min_s: float = 0.125, max_s: float = 1.0):
    """Per-stream block lengths (multiples of 1/64 s in [min_s, max_s]) and
    Poisson arrival times, with mean arrival rate matching real time x speed."""
    out = []
    q = rate_hz // 64
    lo, hi = int(round(min_s * 64)), int(round(max_s * 64))
    for s in range(n_streams):
        rng = np.random.default_rng([seed, 4_000_000 + s])
        lens, times = [], []
        total, t = 0, 0.0
        mean_dur = (lo + hi) / 2.0 / 64.0
        while total < duration_s * rate_hz:
            n = int(rng.integers(lo, hi + 1)) * q
            t += rng.exponential(mean_dur / speed)
            lens.append(n)
            times.append(t)
            total += n
        out.append((np.asarray(lens, np.int64), np.asarray(times)))
    return out


# --------------------------------------------------------------------------
# Algorithmic work (what throughput and roofline figures are priced in)
# --------------------------------------------------------------------------

FLOPS_PER_FILTER_SAMPLE = 12  # complex multiply-add with real input plus the sum (§2.2)


def algorithmic_flops(bank: BankTables, n: int, n_taps_down=None, n_taps_up=None) -> dict:
    """Algorithmic flops of one n-sample block: filtering, resampling, up-add.

    Filtering counts 12 flops per filter-sample (§2.2).  The downsample cascade
    counts 2 flops per tap per output per stream; the upsample-and-add counts a
    complex (2 real) multiply-add per polyphase tap plus the complex add, per
    template and output sample.  Padding lanes, the carry correction and
    compensation terms are not counted.
    """
    H = bank.n_bands
    td = len(bank.h_down) if n_taps_down is None else n_taps_down
    tu = len(bank.h_up) if n_taps_up is None else n_taps_up
    filt = FLOPS_PER_FILTER_SAMPLE * bank.filter_samples_per_block(n)
    down = sum(2 * td * (n >> h) for h in range(1, H))
    up_per_t = sum((4 * ((tu + 1) // 2) + 2) * (n >> h) for h in range(0, H - 1))
    up = up_per_t * bank.n_templates
    return {"filter": filt, "down": down, "up": up, "total": filt + down + up}
