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
