"""The pins have teeth: plausible mistakes planted in a copy of the oracle fail them.

Each case edits one line of ``oracle/spiir_oracle.c`` the way a slip would (a
conjugated or dropped coefficient, an index off by one, the wrong polyphase
parity, a reversed tap order, a lost carry between blocks), builds the copy
with gcc on the CPU, swaps it in for the real oracle and runs the pins of
``test_oracle_pins.py``; at least one of them must fail.  The real oracle is
restored afterwards.
"""
import os
import subprocess

import pytest

import oracle
import test_oracle_pins as P

SRC = os.path.join(os.path.dirname(oracle.__file__), "spiir_oracle.c")

# (name, original text, planted text): each original occurs exactly once
MUTANTS = [
    ("conjugated pole", "y = a1 * y + b0 * xk;", "y = conj(a1) * y + b0 * xk;"),
    ("dropped input gain", "y = a1 * y + b0 * xk;", "y = a1 * y + xk;"),
    ("delay off by one", "int64_t i = k0 + k - d;", "int64_t i = k0 + k - d - 1;"),
    ("output before update", "y = a1 * y + b0 * xk;\n        acc[k] += y;",
     "acc[k] += y;\n        y = a1 * y + b0 * xk;"),
    ("decimation keeps odd samples", "int64_t i = 2 * (m0 + m) - j;", "int64_t i = 2 * (m0 + m) + 1 - j;"),
    ("reversed decimator taps", "if (i >= 0) s += hd[j] * in[i];", "if (i >= 0) s += hd[td - 1 - j] * in[i];"),
    ("zero-stuffing parity", "if (m % 2 != 0) continue;", "if (m % 2 == 0) continue;"),
    ("reversed interpolator taps", "if (e >= 0) s += hu[j] * ext[e];", "if (e >= 0) s += hu[tu - 1 - j] * ext[e];"),
    ("band output not added", "cplx s = z[k];", "cplx s = 0.0;"),
    ("filter state not carried", "b->y[f] = filter_run(", "(void)filter_run("),
    ("up-chain history not carried", "for (int i = 0; i < b->hu_len; ++i) hist[i] = ext[cnt_lo + i];", ""),
]


def _pins():
    """The pins as (name, callable) pairs, parametrised cases spelled out."""
    out = [(f"impulse d={d} k0={k0}", lambda d=d, k0=k0: P.test_impulse_response_closed_form(d, k0))
           for d, k0 in [(0, 0), (5, 0), (3, 11), (17, 4)]]
    out += [
        ("complex exponential", P.test_complex_exponential_closed_form),
        ("cosine", P.test_cosine_through_bank_path),
        ("lfilter", P.test_bank_matches_lfilter),
        ("brute force", P.test_bank_matches_bruteforce_convolution),
        ("time shift", P.test_time_shift),
        ("downsample", lambda: P.test_downsample_matches_upfirdn("asymmetric")),
        ("upsample", lambda: P.test_upsample_add_matches_upfirdn("asymmetric")),
        ("multirate", lambda: P.test_multirate_matches_scipy_composition([[3, 4, 2]])),
        ("pure delay", P.test_pure_delay_taps_reduce_to_decimation_and_zero_stuffing),
        ("block split", lambda: P.test_block_split_invariance(64)),
    ]
    return out


def _build(tmp_path, old, new):
    text = open(SRC).read()
    assert text.count(old) == 1, old
    path = tmp_path / "spiir_oracle_mutant.c"
    path.write_text(text.replace(old, new))
    so = tmp_path / "liboracle_mutant.so"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=gnu11", "-o", str(so), str(path),
                    "-lm"], check=True)
    return str(so)


def test_the_real_oracle_passes_every_pin():
    for name, pin in _pins():
        pin()


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_a_planted_mistake_fails_a_pin(tmp_path, monkeypatch, name, old, new):
    so = _build(tmp_path, old, new)
    monkeypatch.setattr(oracle, "_LIB", so)
    monkeypatch.setattr(oracle, "_lib", None)
    failed = []
    for pin_name, pin in _pins():
        try:
            pin()
        except (AssertionError, ValueError):
            failed.append(pin_name)
    monkeypatch.setattr(oracle, "_lib", None)  # the real library is loaded again after the test
    assert failed, f"no pin catches: {name}"
