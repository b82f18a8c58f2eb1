"""The oracle against facts fixed by the paper and by mathematics (CPU only)."""
import pytest

import oracle_pins


@pytest.mark.parametrize("pin", oracle_pins.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(orc, pin):
    pin(orc)


def test_batch_matches_single(orc):
    """The threaded batch entry gives the same values as one-string calls."""
    import numpy as np

    from paper_1609_09840_amd import workloads as W

    rng = np.random.default_rng(3)
    lengths = rng.integers(0, 3000, size=200)
    lengths[:5] = [0, 1, 511, 512, 1024]
    for wide in (False, True):
        rg = W.from_lengths(lengths, 7, wide, lead=3)
        keys = orc.expand_keys64(9) if wide else orc.expand_keys32(9)
        for mode in (0, 1, 2):
            got = orc.batch(wide, rg.buf, rg.offsets, keys, mode, nthreads=4)
            for i in range(0, rg.count, 17):
                want = (orc.pm64 if wide else orc.pm32)(rg.string(i), keys, mode)[0]
                g = got[i]
                g = int(g[0]) | (int(g[1]) << 64) if (wide and mode == 2) else int(g)
                assert g == want
