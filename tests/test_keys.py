"""The library's key expansion and range check (host code, no GPU) against
the oracle: the same splitmix64 draws in the same order, the same rejections
(Eq. (1) key range with kappa of Table "parameters"), for ordinary seeds and
for seeds that force a rejected or a largest-admissible candidate."""
from __future__ import annotations

import numpy as np
import pytest

import oracle_pins
from paper_1609_09840_amd import pmp

SEEDS = (0, 1, 2, 7, 12345, 2**64 - 1)


@pytest.mark.parametrize("wide", [False, True], ids=["pm32", "pm64"])
def test_expand_keys_matches_oracle(orc, wide):
    forced = [f[0] for f in oracle_pins.reject_seeds(wide)]
    for seed in SEEDS + tuple(forced):
        got = pmp.pmp_expand_keys64(seed) if wide else pmp.pmp_expand_keys32(seed)
        want = orc.expand_keys64(seed) if wide else orc.expand_keys32(seed)
        assert got.dtype == want.dtype and got.shape == (1032,)
        assert np.array_equal(got, want), (wide, hex(seed), int(np.nonzero(got != want)[0][0]))
        check = pmp.pmp_check_keys64 if wide else pmp.pmp_check_keys32
        assert check(got) == pmp.PMP_OK


@pytest.mark.parametrize("wide", [False, True], ids=["pm32", "pm64"])
def test_forced_rejection_changes_the_table(orc, wide):
    """A seed whose draw d is out of range: the library skips it, so a_d is
    the next draw, exactly as in the oracle's table."""
    amax = oracle_pins.AMAX64 if wide else oracle_pins.AMAX32
    shift = 0 if wide else 32
    for seed, draw, cand, ok in oracle_pins.reject_seeds(wide):
        got = pmp.pmp_expand_keys64(seed) if wide else pmp.pmp_expand_keys32(seed)
        stream = [int(v) >> shift for v in orc.splitmix64_stream(seed, draw + 2)]
        if ok:
            assert int(got[draw]) == amax
        else:
            assert int(got[draw]) == stream[draw + 1]


@pytest.mark.parametrize("wide", [False, True], ids=["pm32", "pm64"])
def test_check_keys_range(wide):
    amax = oracle_pins.AMAX64 if wide else oracle_pins.AMAX32
    k = pmp.pmp_expand_keys64(3) if wide else pmp.pmp_expand_keys32(3)
    check = pmp.pmp_check_keys64 if wide else pmp.pmp_check_keys32
    for idx in (0, 127, 128, 1023):
        kk = k.copy()
        kk[idx] = amax
        assert check(kk) == pmp.PMP_OK
        kk[idx] = amax + 1
        assert check(kk) == pmp.PMP_E_KEY_RANGE
    kk = k.copy()
    kk[1024:] = np.iinfo(kk.dtype).max  # b is unrestricted
    assert check(kk) == pmp.PMP_OK
