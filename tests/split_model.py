"""NumPy model of the split-bf16 arithmetic (test-side reference for the
scheme, not for the ladder).

Three or four slices: exponents per row (the integral build) or per (row,
chunk of contracted indices) (the amplitude contraction), balanced
base-256 digits, slice products (p, q) kept when p + q <= S + D (1-based),
exact integer sums per chunk.

Two slices: the per-element split hi = bf16(x), lo = bf16(x - hi), both
rounded to nearest even, and the products hi*hi, hi*lo, lo*hi (D = 2 adds
lo*lo), summed here in float64.

Used to check that the GPU kernels implement exactly this scheme; the
scheme's own error is measured against the float64 oracle."""
import numpy as np


def chunk_len(S):
    """Contracted indices per exponent of the contraction's rows (and per
    exact float32 chunk): 128 for three slices, 256 otherwise."""
    return 128 if S == 3 else 256


def digits(X, S, chunk=0):
    """Rows of X along axis 1 -> (list of S digit arrays, exponents): one
    exponent per row, or with ``chunk`` one per (row, chunk) as ``e[row][c]``."""
    if chunk:
        R, K = X.shape
        nc = (K + chunk - 1) // chunk
        Xp = np.zeros((R, nc * chunk))
        Xp[:, :K] = X
        m = np.max(np.abs(Xp.reshape(R, nc, chunk)), axis=2)
        e = np.where(m > 0, np.frexp(m)[1], 0)
        y = np.ldexp(Xp.reshape(R, nc, chunk), -e[:, :, None]).reshape(R, nc * chunk)[:, :K]
        D = []
        for _ in range(S):
            y = y * 256.0
            q = np.rint(y)
            y = y - q
            D.append(q)
        return D, e
    m = np.max(np.abs(X), axis=1)
    e = np.where(m > 0, np.frexp(m)[1], 0)
    y = np.ldexp(X, -e[:, None])
    D = []
    for _ in range(S):
        y = y * 256.0
        q = np.rint(y)
        y = y - q
        D.append(q)
    return D, e


def bf16_rne(x):
    """x rounded to the nearest bf16 value (8 significant bits, ties to even),
    for finite values inside bf16's normal range."""
    m, e = np.frexp(np.asarray(x, dtype=np.float64))   # x = m 2^e, 1/2 <= |m| < 1
    return np.ldexp(np.rint(np.ldexp(m, 8)), e - 8)


def hi_lo(X):
    hi = bf16_rne(X)
    return hi, bf16_rne(X - hi)


def product(A, B, S, depth, chunk=0):
    """C = A @ B.T through the split scheme (integer digit sums are exact in
    float64; the hi/lo products are exact in float64 and summed there)."""
    if S == 2:
        Ah, Al = hi_lo(A)
        Bh, Bl = hi_lo(B)
        C = Ah @ Bh.T + Ah @ Bl.T + Al @ Bh.T
        return C + Al @ Bl.T if depth >= 2 else C
    Da, ea = digits(A, S, chunk)
    Db, eb = digits(B, S, chunk)
    C = np.zeros((A.shape[0], B.shape[0]))
    if chunk:
        K = A.shape[1]
        for c in range((K + chunk - 1) // chunk):
            sl = slice(c * chunk, min(K, (c + 1) * chunk))
            Cc = np.zeros_like(C)
            for p in range(S):
                for q in range(S):
                    if (p + 1) + (q + 1) <= S + depth:
                        Cc += (Da[p][:, sl] @ Db[q][:, sl].T) * 2.0 ** (-8 * (p + q + 2))
            C += Cc * np.ldexp(1.0, ea[:, c][:, None] + eb[:, c][None, :])
        return C
    for p in range(S):
        for q in range(S):
            if (p + 1) + (q + 1) <= S + depth:
                C += (Da[p] @ Db[q].T) * 2.0 ** (-8 * (p + q + 2))
    return np.ldexp(C, ea[:, None] + eb[None, :])


def ladder(L, t, S, depth):
    """Ladder term through the scheme: build V, re-cut its (a,b) rows, contract."""
    P, v, _ = L.shape
    o = t.shape[0]
    Lr = L.reshape(P, v * v).T                           # rows (p,q) along x
    V = product(Lr, Lr, S, depth)                         # [(a,c)][(b,d)]
    V = V.reshape(v, v, v, v).transpose(0, 2, 1, 3).reshape(v * v, v * v)  # [(a,b)][(c,d)]
    R = product(t.reshape(o * o, v * v), V, S, depth, chunk_len(S))  # [(i,j)][(a,b)]
    return R.reshape(o, o, v, v)


def default_depth(S):
    return 2 if S == 4 else 1


# ---------------------------------------------------------------------------
# int8 digits (the split-int8 form)
# ---------------------------------------------------------------------------

I8_CHUNK = 16384


def digits_i8(X, S, chunk=I8_CHUNK):
    """Rows of X along axis 1 -> (list of S int8 digit arrays as float64,
    exponents e[row][c] per chunk of ``chunk`` indices).  With m the chunk's
    largest |x|, e is the smallest integer with m < 2^e * 127/128; the value
    x 2^(7 + 8(S-1) - e) is rounded to the nearest integer X (ties to even) and
    written X = sum_p d_p 2^(8(S-1-p)) with balanced digits d_p in [-128, 127]
    taken from the lowest one up (the leading one is then within [-127, 127])."""
    R, K = X.shape
    nc = max(1, (K + chunk - 1) // chunk)
    Xp = np.zeros((R, nc * chunk))
    Xp[:, :K] = X
    m = np.max(np.abs(Xp.reshape(R, nc, chunk)), axis=2)
    e = np.where(m > 0, np.frexp(m)[1], 0)
    e = e + (m >= np.ldexp(127.0 / 128.0, e)).astype(e.dtype)
    ek = np.repeat(e, chunk, axis=1)[:, :K]
    Xi = np.rint(np.ldexp(X, 7 + 8 * (S - 1) - ek)).astype(np.int64)
    D = []
    for _ in range(S - 1):
        d = ((Xi + 128) % 256) - 128
        D.append(d)
        Xi = (Xi - d) // 256
    D.append(Xi)
    return [d.astype(np.float64) for d in D[::-1]], e


def product_i8(A, B, S, depth, chunk=I8_CHUNK):
    """C = A @ B.T through the int8 digit scheme: per chunk, the digit products
    (p, q) with p + q <= S + depth (1-based) summed exactly (float64 holds the
    integer sums), scaled by 2^(eA + eB - 14 - 8(p+q)) (0-based p, q)."""
    Da, ea = digits_i8(A, S, chunk)
    Db, eb = digits_i8(B, S, chunk)
    K = A.shape[1]
    C = np.zeros((A.shape[0], B.shape[0]))
    for c in range(max(1, (K + chunk - 1) // chunk)):
        sl = slice(c * chunk, min(K, (c + 1) * chunk))
        Cc = np.zeros_like(C)
        for p in range(S):
            for q in range(S):
                if (p + 1) + (q + 1) <= S + depth:
                    Cc += (Da[p][:, sl] @ Db[q][:, sl].T) * 2.0 ** (-14 - 8 * (p + q))
        C += Cc * np.ldexp(1.0, ea[:, c][:, None] + eb[:, c][None, :])
    return C


def ladder_i8(L, t, S, depth, chunk=I8_CHUNK):
    """Ladder term through the int8 scheme: build V, re-cut its (a,b) rows, contract."""
    P, v, _ = L.shape
    o = t.shape[0]
    Lr = L.reshape(P, v * v).T
    V = product_i8(Lr, Lr, S, depth, chunk)
    V = V.reshape(v, v, v, v).transpose(0, 2, 1, 3).reshape(v * v, v * v)
    R = product_i8(t.reshape(o * o, v * v), V, S, depth, chunk)
    return R.reshape(o, o, v, v)
