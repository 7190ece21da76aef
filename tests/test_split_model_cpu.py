"""CPU checks of the test-side model of the split-bf16 digit scheme."""
import numpy as np


def test_split_model_digits_are_exact_and_bounded():
    # the split scheme's digits: balanced, integer, exact in bf16 (|d| <= 256),
    # and S digits reproduce each entry to 2^(e - 8S - 1)
    from tests import split_model

    rng = np.random.default_rng(61)
    X = rng.standard_normal((7, 50)) * np.exp(rng.uniform(-20, 20, size=(7, 1)))
    for S in (3, 4):
        D, e = split_model.digits(X, S)
        assert np.all(np.abs(D[0]) <= 256) and all(np.all(np.abs(d) <= 128) for d in D[1:])
        assert all(np.array_equal(d, np.rint(d)) for d in D)
        rec = sum(np.ldexp(d, e[:, None] - 8 * (p + 1)) for p, d in enumerate(D))
        assert np.all(np.abs(rec - X) <= np.ldexp(1.0, e - 8 * S - 1)[:, None])


def test_split_model_chunk_exponents_reconstruct_within_the_chunk_bound():
    # per-(row, chunk) exponents: each chunk reconstructs to 2^(e_chunk - 8S - 1),
    # never worse than the row bound
    from tests import split_model

    rng = np.random.default_rng(62)
    X = rng.standard_normal((5, 300)) * np.exp(rng.uniform(-6, 6, size=(5, 300)))
    for S in (3, 4):
        D, e = split_model.digits(X, S, chunk=128)
        _, er = split_model.digits(X, S)
        assert e.shape == (5, 3) and np.all(e <= er[:, None])
        ek = np.repeat(e, 128, axis=1)[:, :300]
        rec = sum(np.ldexp(d, ek - 8 * (p + 1)) for p, d in enumerate(D))
        assert np.all(np.abs(rec - X) <= np.ldexp(1.0, ek - 8 * S - 1))
        assert all(np.all(np.abs(d) <= 256) for d in D)


def test_split_model_bf16_rounding_matches_float32_then_bf16_on_exact_cases():
    # values with at most 24 significant bits round through float32 exactly, and
    # bf16 rounding of a float32 is round-to-nearest-even on its top 16 bits
    from tests import split_model

    rng = np.random.default_rng(63)
    x32 = (rng.standard_normal(4000) * np.exp(rng.uniform(-30, 30, 4000))).astype(np.float32)
    bits = x32.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    rounded = ((bits + 0x7FFF + lsb) >> 16) << 16
    want = rounded.astype(np.uint32).view(np.float32).astype(np.float64)
    assert np.array_equal(split_model.bf16_rne(x32.astype(np.float64)), want)
    # ties go to even: 1 + 2^-8 lies halfway between 1 and 1 + 2^-7
    assert split_model.bf16_rne(1.0 + 2.0 ** -8) == 1.0
    assert split_model.bf16_rne(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6


def test_split_model_hi_lo_bound():
    # hi + lo reproduces x to 2^-16 |x| (two roundings to 8 significant bits)
    from tests import split_model

    rng = np.random.default_rng(64)
    X = rng.standard_normal((9, 70)) * np.exp(rng.uniform(-20, 20, size=(9, 70)))
    hi, lo = split_model.hi_lo(X)
    assert np.array_equal(split_model.bf16_rne(hi), hi) and np.array_equal(split_model.bf16_rne(lo), lo)
    assert np.all(np.abs(X - hi) <= 2.0 ** -8 * np.abs(X))
    assert np.all(np.abs(X - hi - lo) <= 2.0 ** -16 * np.abs(X))
