"""Plants plausible mistakes in copies of the CPU oracle and checks that the
pins of ``oracle_pins.py`` catch every one of them (CPU only; the planted
copies are built in a temporary directory and never touch the GPU path)."""
import os
import tempfile

import pytest

import oracle
import oracle_pins

# (name, text in pmp_oracle.c, replacement)
MUTANTS = [
    ("big_endian_words", "v |= byte << (8 * t);", "v |= byte << (8 * (W - 1 - t));"),
    ("pad_byte_0x80", "(pos == len ? 1u : 0u)", "(pos == len ? 0x80u : 0u)"),
    ("no_pad_byte", "(pos == len ? 1u : 0u)", "0u"),
    ("while_not_do_while", "  do {\n    if (j >= lmax)", "  while (len > 1) {\n    if (j >= lmax)"),
    ("level_keys_swapped", "akeys)[(uint64_t)j * m + i]", "akeys)[(uint64_t)(j ^ 1) * m + i]"),
    ("level_b_swapped", "bkeys)[j]", "bkeys)[j ^ 1]"),
    ("last_term_dropped", "for (int i = 0; i < m; ++i) {", "for (int i = 0; i < m - 1; ++i) {"),
    ("keys_reversed", "akeys)[(uint64_t)j * m + i]", "akeys)[(uint64_t)j * m + (m - 1 - i)]"),
    ("no_constant_term", "u128 acc = b % p;", "u128 acc = 0;"),
    ("wrong_prime32", "((u128)1 << 32) + 15", "((u128)1 << 32) + 17"),
    ("wrong_prime64", "((u128)1 << 64) + 13", "((u128)1 << 64) + 15"),
    ("truncate_level_values", "next[c] = acc;", "next[c] = wide ? (uint64_t)acc : (uint32_t)acc;"),
    ("sum_mod_2_2n", "acc = (acc + (a * s) % p) % p;", "acc = (uint64_t)(acc + a * s) % p;"),
    ("mix32_shift", "z = z ^ (z >> 13);", "z = z ^ (z >> 12);"),
    ("mix64_mult", "z = z * 0xc4ceb9fe1a85ec53ULL;", "z = z * 0xc4ceb9fe1a85ec55ULL;"),
    ("keys32_low_half", "do { c = sm64_next(&s) >> 32; }", "do { c = sm64_next(&s) & 0xffffffffULL; }"),
    ("splitmix_gamma", "0x9e3779b97f4a7c15ULL", "0x9e3779b97f4a7c17ULL"),
    ("block_127", "tree_generic(sig, n, 128, 8, p, p - 28 - 1", "tree_generic(sig, n, 127, 8, p, p - 28 - 1"),
    ("kappa_off", "p - 24 - 1, keys", "p - 23 - 1, keys"),
    ("raw_not_mod_2n", "else if (mode == OR_RAW) out[0] = low;\n  else out[0] = oracle_mix32(low);",
     "else if (mode == OR_RAW) out[0] = (uint64_t)h;\n  else out[0] = oracle_mix32(low);"),
    ("pad_block_reuses_value", "u128 s = idx < len ? cur[idx] : 0;", "u128 s = idx < len ? cur[idx] : cur[len - 1];"),
]


@pytest.fixture(scope="module")
def src():
    with open(oracle.SRC) as f:
        return f.read()


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(src, name, old, new):
    assert old in src, f"mutation site for {name} not found"
    # every occurrence is replaced, so a constant written twice changes everywhere
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "m.c")
        with open(path, "w") as f:
            f.write(src.replace(old, new))
        so = oracle.build(path, os.path.join(d, "libm.so"))
        o = oracle.load(so)
        failed = []
        for pin in oracle_pins.ALL_PINS:
            try:
                pin(o)
            except (AssertionError, oracle.OracleError):
                failed.append(pin.__name__)
        assert failed, f"mutant {name} passed every pin"


# the property pins of Lemma 9 / Lemma 8 must catch these on their own
PROPERTY_MUTANTS = ["wrong_prime32", "wrong_prime64", "keys_reversed", "level_keys_swapped"]


@pytest.mark.parametrize("name", PROPERTY_MUTANTS)
def test_property_pins_bite(src, name):
    old, new = next((m[1], m[2]) for m in MUTANTS if m[0] == name)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "m.c")
        with open(path, "w") as f:
            f.write(src.replace(old, new))
        o = oracle.load(oracle.build(path, os.path.join(d, "libm.so")))
        for pin in (oracle_pins.pin_regularity, oracle_pins.pin_single_key_collisions):
            with pytest.raises((AssertionError, oracle.OracleError)):
                pin(o)
