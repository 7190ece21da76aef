"""NumPy model of the split-bf16 digit arithmetic (test-side reference for the
scheme, not for the ladder): per-row exponents, balanced base-256 digits,
slice products (p, q) kept when p + q <= S + D (1-based), exact integer sums.
Used to check that the GPU kernels implement exactly this scheme; the scheme's
own error is measured against the float64 oracle."""
import numpy as np


def digits(X, S):
    """Rows of X along axis 1 -> (list of S digit arrays, row exponents)."""
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


def product(A, B, S, depth):
    """C = A @ B.T through the digit scheme (integer digit sums are exact in float64)."""
    Da, ea = digits(A, S)
    Db, eb = digits(B, S)
    C = np.zeros((A.shape[0], B.shape[0]))
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
    R = product(t.reshape(o * o, v * v), V, S, depth)     # [(i,j)][(a,b)]
    return R.reshape(o, o, v, v)


def default_depth(S):
    return 2 if S == 4 else 1
