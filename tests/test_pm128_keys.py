"""PM+128 key expansion of the library (host code) equals the oracle's, and
the range check; no GPU needed."""
from __future__ import annotations

import numpy as np

from oracle import pm128 as O
from paper_1609_09840_amd import pmp


def test_expand_keys128_matches_oracle():
    for seed in (0, 1, 2, 77):
        got = pmp.pmp_expand_keys128(seed)
        a, b = O.expand_keys128(seed)
        assert np.array_equal(got, O.key_table_u64(a, b))
        assert pmp.pmp_check_keys128(got) == pmp.PMP_OK


def test_check_keys128_range():
    k = pmp.pmp_expand_keys128(3)
    k[2 * 5] = np.uint64(2**64 - 49)  # a_{1,5} = 2^128 - 49: one above the range
    k[2 * 5 + 1] = np.uint64(2**64 - 1)
    assert pmp.pmp_check_keys128(k) == pmp.PMP_E_KEY_RANGE
    k[2 * 5] = np.uint64(2**64 - 50)  # 2^128 - 50: the largest admissible key
    assert pmp.pmp_check_keys128(k) == pmp.PMP_OK
