"""The pair-symmetric adjoint's half-written W block, checked on the CPU against
the float64 oracle (host-side check of the reading and of the K ranges, not of
the kernels).

With t and lam pair-symmetric (x[j,i,d,c] = x[i,j,c,d]) the adjoint block
W[a,c,b,d] = sum_ij lam[i,j,a,b] t[i,j,c,d] satisfies W[b,d,a,c] = W[a,c,b,d].
The library forms only Wh, its b >= a half with the diagonal a == b halved, so
that W = Wh + Wh^T, and gets both dL terms of W from two products of Wh:

    dL[x,a,c] += 2 sum_{b>=a,d} Wh[a,c,b,d] L[x,b,d]       (first term, K from b = a)
    dL[x,b,d] += 2 sum_{a<=b,c} L[x,a,c] Wh[a,c,b,d]       (second term, K up to a = b)

The products run over whole tiles and whole K-steps, so a tile's K range starts
at (ends after) the virtual of its first (last) column, rounded out to a K-step:
the model below repeats that tiling with the unwritten part of Wh poisoned with
NaN, except the band of rows b in [a - s, a) that the library zeroes, and so
shows that the band is wide enough."""
import numpy as np
import pytest

import oracle
from paper_2310_04559_amd.inputs import make_inputs

BN_DIRECT, BN_STAGED = 256, 128  # tile columns of the direct and register-staged kernels
BK_F64, BK_F32 = 16, 32          # K-steps (float64, float32)


def band_rows(v):
    # rows below the diagonal the rounded K ranges can reach (widest tile, deepest step)
    return -(-(BN_DIRECT - 1) // v) + -(-(32 - 1) // v)


def model_dL(L, t, lam, nblocks, bn, bk):
    P, v, _ = L.shape
    o = t.shape[0]
    L2 = L.reshape(P, v * v)
    dL = np.zeros((P, v * v))
    s = band_rows(v)
    bounds = np.linspace(0, v, nblocks + 1).round().astype(int)
    for a0, a1 in zip(bounds[:-1], bounds[1:]):
        na = a1 - a0
        if na == 0:
            continue
        Wh = np.full((na, v, v, v), np.nan)  # stale contents of the scratch block
        for al in range(na):
            a = a0 + al
            Wh[al, :, max(0, a - s):a, :] = 0.0
            for b in range(a, v):
                w = 0.5 if a == b else 1.0
                Wh[al, :, b, :] = w * np.einsum("ij,ijcd->cd", lam[:, :, a, b], t)
        Wr = Wh.reshape(na * v, v * v)
        # first term: columns (a - a0, c), K = (b, d) from the tile's smallest a
        K = v * v
        for n0 in range(0, na * v, bn):
            n1 = min(n0 + bn, na * v)
            k0 = ((a0 + n0 // v) * v) // bk * bk
            dL[:, a0 * v + n0:a0 * v + n1] += 2.0 * (L2[:, k0:] @ Wr[n0:n1, k0:].T)
        # second term: columns (b - a0, d) for b >= a0, K rows (a - a0, c) up to the tile's largest b
        N, K2 = (v - a0) * v, na * v
        B = Wr[:, a0 * v:]
        for n0 in range(0, N, bn):
            n1 = min(n0 + bn, N)
            kend = min(K2, ((n1 - 1) // v + 1) * v)
            k1 = min(K2, -(-kend // bk) * bk)
            dL[:, a0 * v + n0:a0 * v + n1] += 2.0 * (L2[:, a0 * v:a0 * v + k1] @ B[:k1, n0:n1])
    return dL.reshape(P, v, v)


@pytest.mark.parametrize("o,v,P,nblocks,bn,bk", [
    (2, 5, 4, 1, BN_DIRECT, BK_F64),
    (2, 7, 5, 2, BN_STAGED, BK_F32),
    (3, 18, 7, 3, BN_DIRECT, BK_F32),
    (2, 33, 6, 4, BN_STAGED, BK_F64),
    (2, 40, 5, 1, BN_DIRECT, BK_F32),
])
def test_half_block_adjoint_matches_oracle(o, v, P, nblocks, bn, bk):
    inp = make_inputs(o, v, P, 97 + v, with_lambda=True)
    dL_ref, _ = oracle.ladder_backward(inp.L_vv, inp.t, inp.lam)
    dL = model_dL(inp.L_vv, inp.t, inp.lam, nblocks, bn, bk)
    assert np.all(np.isfinite(dL)), "a K range reached an unwritten row of the half block"
    assert np.max(np.abs(dL - dL_ref)) < 1e-13 * np.max(np.abs(dL_ref))


def test_half_block_needs_the_band():
    # without the zeroed band a rounded K range reads the stale rows below the diagonal
    inp = make_inputs(2, 18, 5, 7, with_lambda=True)
    global band_rows
    saved = band_rows
    try:
        band_rows = lambda v: 0  # noqa: E731
        dL = model_dL(inp.L_vv, inp.t, inp.lam, 2, BN_DIRECT, BK_F32)
    finally:
        band_rows = saved
    assert not np.all(np.isfinite(dL))


def pair_row(q, v):
    """Largest a with sum_{a' < a} (v - a') <= q, as the device epilogues decode it:
    the smaller root of a^2 - (2v+1) a + 2q = 0 in float64, floored, then one
    correction step each way."""
    prefix = lambda a: a * v - a * (a - 1) // 2  # noqa: E731
    b = 2.0 * v + 1.0
    a = int((b - np.sqrt(b * b - 8.0 * float(q))) * 0.5)
    a = min(max(a, 0), v - 1)
    if a + 1 < v and prefix(a + 1) <= q:
        a += 1
    if a > 0 and prefix(a) > q:
        a -= 1
    return a


def test_pair_row_decode():
    # every packed index of small v, and the indices around every row start of the
    # largest v the planner accepts (46340)
    for v in list(range(1, 70)) + [300, 361]:
        q = 0
        for a in range(v):
            for _ in range(a, v):
                assert pair_row(q, v) == a
                q += 1
    v = 46340
    rng = np.random.default_rng(5)
    for a in list(range(0, 40)) + list(rng.integers(0, v, 400)) + list(range(v - 40, v)):
        a = int(a)
        start = a * v - a * (a - 1) // 2
        assert pair_row(start, v) == a
        if a > 0:
            assert pair_row(start - 1, v) == a - 1
        if a + 1 < v:
            assert pair_row(start + (v - a) - 1, v) == a


def test_general_adjoint_one_block_symmetric_part():
    # general t, lam, L: with W'[(a,c)][(b,d)] = sum_ij lam[i,j,a,b] t[i,j,c,d] held
    # whole, both dL terms are one product with its symmetric part,
    # dL[x][p] = sum_q L[x][q] (W'[p][q] + W'[q][p])
    from paper_2310_04559_amd.inputs import random_general

    L, t, lam = random_general(3, 7, 5, 61)
    P, v, _ = L.shape
    W = np.einsum("ijab,ijcd->acbd", lam, t).reshape(v * v, v * v)
    dL = (L.reshape(P, v * v) @ (W + W.T).T).reshape(P, v, v)
    ref, _ = oracle.ladder_backward(L, t, lam)
    assert np.max(np.abs(dL - ref)) < 1e-13 * np.max(np.abs(ref))
