"""CPU checks of the test-side model of the split-bf16 digit scheme."""
import numpy as np


def test_split_model_digits_are_exact_and_bounded():
    # the split scheme's digits: balanced, integer, exact in bf16 (|d| <= 256),
    # and S digits reproduce each entry to 2^(e - 8S - 1)
    from tests import split_model

    rng = np.random.default_rng(61)
    X = rng.standard_normal((7, 50)) * np.exp(rng.uniform(-20, 20, size=(7, 1)))
    for S in (2, 3, 4):
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
    for S in (2, 4):
        D, e = split_model.digits(X, S, chunk=128)
        _, er = split_model.digits(X, S)
        assert e.shape == (5, 3) and np.all(e <= er[:, None])
        ek = np.repeat(e, 128, axis=1)[:, :300]
        rec = sum(np.ldexp(d, ek - 8 * (p + 1)) for p, d in enumerate(D))
        assert np.all(np.abs(rec - X) <= np.ldexp(1.0, ek - 8 * S - 1))
        assert all(np.all(np.abs(d) <= 256) for d in D)
