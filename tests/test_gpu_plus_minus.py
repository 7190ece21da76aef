"""GPU parity of the symmetric/antisymmetric (t+, t-) forward against the
float64 oracle, through the C ABI.

With pair-symmetric amplitudes the library contracts V+ = (ac|bd) + (ad|bc)
with t+ over the pairs c <= d, and V- with t- over c < d, for rows i <= j
(i < j) and columns a <= b (a < b), and scatters half of each result to the
four (i,j)/(a,b) mirrors.  Any Cholesky vectors (the scheme uses only the
pair exchange (pq|rs) = (rs|pq)); ragged shapes across the 32-wide pair
tiles of the combination pass, the 128/160-row and 64-row remainder tiles of
the contraction, and blocks of several sizes.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2310_04559_amd.inputs import CONFIGS, integer_inputs, make_inputs, random_general, seed_for
from tests.gpu_common import TOL, announce, dev, host, rel_fro

pytestmark = pytest.mark.gpu


def _pair_symmetric(t):
    return 0.5 * (t + t.transpose(1, 0, 3, 2))


def run(native, L, t, R0, precision, **kw):
    R = dev(R0)
    native.cc_ladder_residual(dev(L), dev(t), R, precision,
                              opts=native.make_opts(pair_symmetric=True, plus_minus=True, **kw))
    torch.cuda.synchronize()
    return host(R)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("o,v,P,a_block", [(5, 20, 75, 0), (9, 37, 101, 7), (4, 44, 131, 13),
                                           (3, 130, 17, 40), (2, 3, 2, 0), (16, 64, 200, 1),
                                           (1, 33, 9, 0), (7, 1, 4, 0), (23, 65, 50, 30)])
def test_plus_minus_general_vectors(gpu_lib, o, v, P, a_block, precision):
    announce("forward-pm", o, v, P, "a_block", a_block, "precision", precision)
    L, t, _ = random_general(o, v, P, 1300 + o + v)
    t = _pair_symmetric(t)
    R0 = np.random.default_rng(10).standard_normal(t.shape)
    inc = oracle.ladder_forward(L, t)
    got = run(gpu_lib, L, t, R0, precision, a_block=a_block)
    err = rel_fro(got - R0, inc)
    print(f"CASE forward-pm error {err:.2e}", flush=True)
    assert err < TOL[precision]


@pytest.mark.parametrize("precision", [0, 1])
def test_plus_minus_integer_exact(gpu_lib, precision):
    # integer vectors and pair-symmetric integer amplitudes: every sum, the
    # halves and the mirrored additions are exact
    announce("forward-pm-int", precision)
    L, t = integer_inputs(4, 11, 5, 79)
    t = t + t.transpose(1, 0, 3, 2)
    ref = oracle.ladder_forward(L, t)
    got = run(gpu_lib, L, t, np.zeros_like(t), precision, a_block=4)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("precision", [0, 1])
def test_plus_minus_exchange(gpu_lib, precision):
    # the exchange partner's amplitudes combine to t+ and -t-
    announce("forward-pm-exchange", precision)
    L, t, _ = random_general(9, 37, 101, 45)
    t = _pair_symmetric(t)
    inc = oracle.exchange_forward(L, t)
    got = run(gpu_lib, L, t, np.zeros_like(t), precision, a_block=7, exchange=True)
    assert rel_fro(got, inc) < TOL[precision]


def test_plus_minus_c2_workload_whole_tensor(gpu_lib):
    name = "o20_v180_P600"
    o, v, P = CONFIGS[name]
    announce("forward-pm", name)
    inp = make_inputs(o, v, P, seed_for(name))
    ref = oracle.ladder_forward(inp.L_vv, inp.t)
    for precision in (0, 1):
        got = run(gpu_lib, inp.L_vv, inp.t, np.zeros_like(inp.t), precision)
        err = rel_fro(got, ref)
        print(f"CASE forward-pm {name} precision {precision} error {err:.2e}", flush=True)
        assert err < TOL[precision]


def _symmetric_vectors(L):
    return 0.5 * (L + L.transpose(0, 2, 1))


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("o,v,P,a_block", [(5, 20, 75, 0), (9, 37, 101, 7), (4, 44, 131, 13),
                                           (3, 130, 17, 40), (2, 3, 2, 0), (16, 64, 200, 1),
                                           (1, 33, 9, 0), (7, 1, 4, 0), (23, 65, 50, 30)])
def test_symmetric_vectors(gpu_lib, o, v, P, a_block, precision):
    # symmetric Cholesky vectors: V+- gathered from the whole pair-pair integral
    # (ragged 32-wide pair tiles, pair counts that are not multiples of the
    # 128 x 128 / 128 x 256 tiles of its upper-triangle grid, blocks of several sizes)
    announce("forward-pm-symv", o, v, P, "a_block", a_block, "precision", precision)
    L, t, _ = random_general(o, v, P, 1500 + o + v)
    L, t = _symmetric_vectors(L), _pair_symmetric(t)
    kw = dict(a_block=a_block, pair_symmetric=True, plus_minus=True)
    with_g = gpu_lib.cc_ladder_workspace_query(o, v, P, precision,
                                               opts=gpu_lib.make_opts(symmetric_vectors=True, **kw))
    without = gpu_lib.cc_ladder_workspace_query(o, v, P, precision, opts=gpu_lib.make_opts(**kw))
    if v >= 8:  # (a few virtuals: the two footprints can coincide)
        assert with_g != without  # the whole-integral plan is the one taken
    R0 = np.random.default_rng(11).standard_normal(t.shape)
    inc = oracle.ladder_forward(L, t)
    got = run(gpu_lib, L, t, R0, precision, a_block=a_block, symmetric_vectors=True)
    err = rel_fro(got - R0, inc)
    print(f"CASE forward-pm-symv error {err:.2e}", flush=True)
    assert err < TOL[precision]


@pytest.mark.parametrize("precision", [0, 1])
def test_symmetric_vectors_integer_exact_and_exchange(gpu_lib, precision):
    # integer symmetric vectors and pair-symmetric integer amplitudes: exact;
    # the exchange partner from the same integral within tolerance
    announce("forward-pm-symv-int", precision)
    L, t = integer_inputs(4, 11, 5, 81)
    L, t = L + L.transpose(0, 2, 1), t + t.transpose(1, 0, 3, 2)
    got = run(gpu_lib, L, t, np.zeros_like(t), precision, a_block=4, symmetric_vectors=True)
    assert np.array_equal(got, oracle.ladder_forward(L, t))
    L, t, _ = random_general(9, 37, 101, 47)
    L, t = _symmetric_vectors(L), _pair_symmetric(t)
    got = run(gpu_lib, L, t, np.zeros_like(t), precision, a_block=7, exchange=True,
              symmetric_vectors=True)
    assert rel_fro(got, oracle.exchange_forward(L, t)) < TOL[precision]


def test_symmetric_vectors_checks_and_fallback(gpu_lib):
    announce("forward-pm-symv-checks")
    o, v, P = 4, 29, 13
    L, t, _ = random_general(o, v, P, 48)
    t = _pair_symmetric(t)
    Ls = _symmetric_vectors(L)
    kw = dict(pair_symmetric=True, plus_minus=True, symmetric_vectors=True)
    # the symmetry check rejects general vectors with the outputs untouched, and
    # passes symmetric ones
    R = torch.zeros(t.shape, dtype=torch.float64, device="cuda")
    with pytest.raises(gpu_lib.LadderError) as e:
        gpu_lib.cc_ladder_residual(dev(L), dev(t), R, 0,
                                   opts=gpu_lib.make_opts(check_symmetry=True, **kw))
    assert e.value.code == gpu_lib.CC_LADDER_EINVAL
    torch.cuda.synchronize()
    assert float(R.abs().max()) == 0.0
    ref = oracle.ladder_forward(Ls, t)
    got = run(gpu_lib, Ls, t, np.zeros_like(t), 0, check_symmetry=True, symmetric_vectors=True)
    assert rel_fro(got, ref) < TOL[0]
    # without PAIR_SYMMETRIC the flag is rejected
    with pytest.raises(gpu_lib.LadderError) as e:
        gpu_lib.cc_ladder_residual(dev(Ls), dev(t), R, 0,
                                   opts=gpu_lib.make_opts(symmetric_vectors=True))
    assert e.value.code == gpu_lib.CC_LADDER_EINVAL
    # a budget the whole integral does not fit: the packed blocks, same result
    ldg = (v * (v + 1) // 2 + 3) // 4 * 4
    got = run(gpu_lib, Ls, t, np.zeros_like(t), 0, hbm_budget=ldg * ldg * 8, symmetric_vectors=True)
    assert rel_fro(got, ref) < TOL[0]


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("exchange", [False, True])
@pytest.mark.parametrize("o,v,P,a_block", [(5, 20, 75, 0), (9, 37, 101, 7), (3, 130, 17, 40),
                                           (2, 3, 2, 0), (7, 1, 4, 0), (23, 65, 50, 30)])
def test_symmetric_vectors_packed_rows(gpu_lib, o, v, P, a_block, precision, exchange):
    # the pair-symmetric forward without the combinations: packed rows (a,b),
    # a <= b, gathered whole from the pair-pair integral, then the mirrored contraction
    announce("forward-pairsym-symv", o, v, P, "a_block", a_block, "precision", precision, exchange)
    L, t, _ = random_general(o, v, P, 1600 + o + v)
    L, t = _symmetric_vectors(L), _pair_symmetric(t)
    R0 = np.random.default_rng(12).standard_normal(t.shape)
    inc = oracle.exchange_forward(L, t) if exchange else oracle.ladder_forward(L, t)
    R = dev(R0)
    gpu_lib.cc_ladder_residual(dev(L), dev(t), R, precision,
                               opts=gpu_lib.make_opts(a_block=a_block, pair_symmetric=True,
                                                      symmetric_vectors=True, exchange=exchange))
    torch.cuda.synchronize()
    err = rel_fro(host(R) - R0, inc)
    print(f"CASE forward-pairsym-symv error {err:.2e}", flush=True)
    assert err < TOL[precision]


def test_plus_minus_rejections(gpu_lib):
    announce("forward-pm-rejections")
    L, t, _ = random_general(3, 10, 4, 46)
    R = torch.zeros(t.shape, dtype=torch.float64, device="cuda")
    with pytest.raises(gpu_lib.LadderError) as e:
        gpu_lib.cc_ladder_residual(dev(L), dev(t), R, 0, opts=gpu_lib.make_opts(plus_minus=True))
    assert e.value.code == gpu_lib.CC_LADDER_EINVAL
    with pytest.raises(gpu_lib.LadderError) as e:
        gpu_lib.cc_ladder_residual(dev(L), dev(_pair_symmetric(t)), R, 2,
                                   opts=gpu_lib.make_opts(pair_symmetric=True, plus_minus=True))
    assert e.value.code == gpu_lib.CC_LADDER_EUNSUPPORTED
    torch.cuda.synchronize()
    assert float(R.abs().max()) == 0.0


@pytest.mark.parametrize("precision,slices,pm", [(0, 0, False), (0, 0, True), (1, 0, True),
                                                 (2, 4, False), (3, 5, False)])
def test_pair_balanced_blocks(gpu_lib, precision, slices, pm):
    # a budget that forces several blocks of about equal pair counts (no a_block
    # given): the same result as one block, bit for bit in float64, and the
    # oracle's within tolerance
    o, v, P = 6, 53, 40
    announce("pair-balanced-blocks", precision, slices, pm)
    L, t, _ = random_general(o, v, P, 1400 + precision)
    t = _pair_symmetric(t)
    kw = dict(split_slices=slices, pair_symmetric=True, plus_minus=pm)
    one, blk1 = gpu_lib.cc_ladder_workspace_query(o, v, P, precision, opts=gpu_lib.make_opts(**kw))
    assert blk1 == v
    budget = one // 3
    nbytes, blk = gpu_lib.cc_ladder_workspace_query(o, v, P, precision, hbm_budget=budget,
                                                    opts=gpu_lib.make_opts(**kw))
    assert nbytes <= budget and blk < v
    R1 = dev(np.zeros_like(t))
    gpu_lib.cc_ladder_residual(dev(L), dev(t), R1, precision, opts=gpu_lib.make_opts(**kw))
    Rb = dev(np.zeros_like(t))
    gpu_lib.cc_ladder_residual(dev(L), dev(t), Rb, precision,
                               opts=gpu_lib.make_opts(hbm_budget=budget, **kw))
    torch.cuda.synchronize()
    if precision == 0:
        assert torch.equal(R1, Rb)
    ref = oracle.ladder_forward(L, t)
    tol = {0: TOL[0], 1: TOL[1], 2: 2e-9, 3: 1e-9}[precision]
    assert rel_fro(host(Rb), ref) < tol
