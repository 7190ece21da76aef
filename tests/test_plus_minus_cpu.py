"""The symmetric/antisymmetric decomposition the PLUS_MINUS forward uses,
checked on the CPU against the float64 oracle (host-side check of the
reading, not of the kernels): with pair-symmetric t and any Cholesky vectors,

    R+[ij][ab] = R[i,j,a,b] + R[i,j,b,a] = sum_{c<=d} V+[ab][cd] t+[ij][cd]
    R-[ij][ab] = R[i,j,a,b] - R[i,j,b,a] = sum_{c<d}  V-[ab][cd] t-[ij][cd]

with V+- = (ac|bd) +- (ad|bc) (2(ac|bc) on c = d) and t+- = t_ijcd +- t_ijdc
(t_ijcc on c = d), over rows i <= j (i < j for R-) and columns a <= b (a < b),
scattered to the four (i,j)/(a,b) mirrors with half weight."""
import numpy as np

import oracle
from paper_2310_04559_amd.inputs import make_inputs, random_general


def plus_minus_ladder(L, t):
    P, v, _ = L.shape
    o = t.shape[0]
    V = np.einsum("xac,xbd->acbd", L, L)          # V[a,c,b,d] = (ac|bd)
    cu, du = np.triu_indices(v)
    cs, ds = np.triu_indices(v, 1)
    iu, ju = np.triu_indices(o)
    is_, js = np.triu_indices(o, 1)
    tp = t[:, :, cu, du] + t[:, :, du, cu]
    tp[:, :, cu == du] *= 0.5
    tp = tp[iu, ju]
    tm = (t[:, :, cs, ds] - t[:, :, ds, cs])[is_, js]
    Vp = np.stack([V[a, cu, b, du] + V[a, du, b, cu] for a, b in zip(cu, du)])
    Vm = np.stack([V[a, cs, b, ds] - V[a, ds, b, cs] for a, b in zip(cs, ds)]).reshape(-1, len(cs))
    Rp = tp @ Vp.T
    Rm = tm @ Vm.T
    R = np.zeros_like(t)
    for m, (i, j) in enumerate(zip(iu, ju)):
        for n, (a, b) in enumerate(zip(cu, du)):
            for x in {(i, j, a, b), (i, j, b, a), (j, i, b, a), (j, i, a, b)}:
                R[x] += 0.5 * Rp[m, n]
    for m, (i, j) in enumerate(zip(is_, js)):
        for n, (a, b) in enumerate(zip(cs, ds)):
            w = 0.5 * Rm[m, n]
            R[i, j, a, b] += w
            R[j, i, b, a] += w
            R[i, j, b, a] -= w
            R[j, i, a, b] -= w
    return R


def test_plus_minus_decomposition_general_vectors():
    L, t, _ = random_general(4, 6, 5, 31)
    t = 0.5 * (t + t.transpose(1, 0, 3, 2))
    ref = oracle.ladder_forward(L, t)
    assert np.max(np.abs(plus_minus_ladder(L, t) - ref)) < 1e-14 * np.max(np.abs(ref))


def test_plus_minus_decomposition_workload_and_exchange():
    inp = make_inputs(3, 7, 9, 32)
    ref = oracle.ladder_forward(inp.L_vv, inp.t)
    assert np.max(np.abs(plus_minus_ladder(inp.L_vv, inp.t) - ref)) < 1e-14 * np.max(np.abs(ref))
    # the exchange partner is the ladder of t with c, d swapped: t+ unchanged, t- negated
    tx = np.ascontiguousarray(inp.t.transpose(0, 1, 3, 2))
    refx = oracle.exchange_forward(inp.L_vv, inp.t)
    assert np.max(np.abs(plus_minus_ladder(inp.L_vv, tx) - refx)) < 1e-14 * np.max(np.abs(refx))


def test_plus_minus_needs_pair_symmetric_amplitudes():
    # without pair symmetry the rows i > j are not recovered from i <= j
    L, t, _ = random_general(3, 5, 4, 33)
    ref = oracle.ladder_forward(L, t)
    assert np.max(np.abs(plus_minus_ladder(L, t) - ref)) > 1e-6 * np.max(np.abs(ref))


def _pp(a, v):
    # packed pairs (a', c) with a' < a, a' <= c: the first packed index of row a
    return a * v - a * (a - 1) // 2


def gathered_block(L, a0, na):
    """V+ and V- of the block's rows (a, b), a in [a0, a0 + na), b >= a, as the
    symmetric-vector path forms them: the whole pair-pair integral
    G[p][q] = sum_x Lp[x][p] Lp[x][q] over unordered pairs p = {a, c}, then each
    X_ab[c][d] = (ac|bd) read from G in the orientation the gather uses for its
    element class (d >= b: row {a,c}, column {b,d}; d < b and c >= a: row {b,d},
    column {a,c}; c < a and d < b: row {c,a}, column {d,b})."""
    P, v, _ = L.shape
    iu = np.triu_indices(v)
    Lp = L[:, iu[0], iu[1]]                       # Lp[x][pair(a, c)], a <= c
    G = Lp.T @ Lp
    pp = lambda a: _pp(a, v)                      # noqa: E731
    plus, minus = [], []
    for a in range(a0, a0 + na):
        for b in range(a, v):
            X = np.empty((v, v))
            for c in range(v):
                for d in range(v):
                    if d >= b:
                        pac = pp(a) + c - a if a <= c else pp(c) + a - c
                        X[c, d] = G[pac, pp(b) + d - b]
                    elif c >= a:
                        X[c, d] = G[pp(d) + b - d, pp(a) + c - a]
                    else:
                        X[c, d] = G[pp(c) + a - c, pp(d) + b - d]
            cu, du = np.triu_indices(v)
            xp = X[cu, du] + X[du, cu]
            xp[cu == du] = 2.0 * X[cu, cu][cu == du]
            plus.append(xp)
            if a < b:
                cs, ds = np.triu_indices(v, 1)
                minus.append(X[cs, ds] - X[ds, cs])
    return np.array(plus), np.array(minus)


def test_symmetric_vector_gather():
    # the workload's vectors are symmetric: V+- gathered from the pair-pair
    # integral equal V+- of the definition, (ac|bd) +- (ad|bc), for every block
    inp = make_inputs(2, 9, 7, 34)
    L = inp.L_vv
    assert np.array_equal(L, L.transpose(0, 2, 1))
    V = np.einsum("xac,xbd->abcd", L, L)           # V[a,b,c,d] = (ac|bd)
    v = L.shape[1]
    cu, du = np.triu_indices(v)
    cs, ds = np.triu_indices(v, 1)
    for a0, na in ((0, 3), (3, 4), (7, 2)):
        plus, minus = gathered_block(L, a0, na)
        rows = [(a, b) for a in range(a0, a0 + na) for b in range(a, v)]
        want_p = np.array([V[a, b, cu, du] + V[a, b, du, cu] for a, b in rows])
        want_m = np.array([V[a, b, cs, ds] - V[a, b, ds, cs] for a, b in rows if a < b])
        scale = np.max(np.abs(want_p))
        assert np.max(np.abs(plus - want_p)) < 1e-14 * scale
        assert np.max(np.abs(minus - want_m)) < 1e-14 * scale


def test_symmetric_vector_gather_needs_symmetric_vectors():
    # general vectors: G built from the upper triangles misses (ac|bd) for c < a
    L, _, _ = random_general(2, 6, 5, 35)
    V = np.einsum("xac,xbd->abcd", L, L)
    v = L.shape[1]
    cu, du = np.triu_indices(v)
    plus, _ = gathered_block(L, 0, v)
    want = np.array([V[a, b, cu, du] + V[a, b, du, cu] for a in range(v) for b in range(a, v)])
    assert np.max(np.abs(plus - want)) > 1e-3 * np.max(np.abs(want))
