"""GPU parity of the ladder forward against the float64 oracle, through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
from paper_2310_04559_amd.inputs import (CONFIGS, integer_inputs, make_inputs, random_general,
                                         seed_for)
from tests.gpu_common import TOL, TOL_SPLIT, TOL_SPLIT_WORKLOAD, announce, dev, host, rel_fro

pytestmark = pytest.mark.gpu

# (o, v, P): ragged against the 128x128 tiles and the 16/32-deep K steps, odd v
# (unaligned rows), single vectors, more than one tile in every dimension.
SHAPES = [(5, 20, 75), (9, 37, 101), (12, 44, 131), (16, 64, 200), (1, 3, 1), (3, 130, 17),
          (2, 1, 3)]


def run_forward(native, L, t, R0, precision, **kw):
    R = dev(R0)
    native.cc_ladder_residual(dev(L), dev(t), R, precision, opts=native.make_opts(**kw))
    torch.cuda.synchronize()
    return host(R)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("o,v,P", SHAPES)
@pytest.mark.parametrize("a_block", [0, 7])
def test_forward_general_inputs(gpu_lib, o, v, P, a_block, precision):
    announce("forward", o, v, P, "a_block", a_block, "precision", precision)
    L, t, _ = random_general(o, v, P, 100 + o + v + P)
    R0 = np.random.default_rng(7).standard_normal(t.shape)
    inc_ref = oracle.ladder_forward(L, t)
    got = run_forward(gpu_lib, L, t, R0, precision, a_block=a_block)
    assert rel_fro(got - R0, inc_ref) < TOL[precision]


@pytest.mark.parametrize("precision", [0, 1])
def test_forward_integer_inputs_exact(gpu_lib, precision):
    # integer L and t with every partial sum below 2**24: exact in both forms
    announce("forward-int", precision)
    L, t = integer_inputs(3, 10, 5, 77)
    ref = oracle.ladder_forward(L, t)
    got = run_forward(gpu_lib, L, t, np.zeros_like(t), precision)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("precision", [0, 1])
def test_forward_c1_workload(gpu_lib, precision):
    o, v, P = CONFIGS["o5_v20_P75"]
    announce("forward-o5-v20-P75", precision)
    inp = make_inputs(o, v, P, seed_for("o5_v20_P75"))
    ref = oracle.ladder_forward(inp.L_vv, inp.t)
    got = run_forward(gpu_lib, inp.L_vv, inp.t, np.zeros_like(inp.t), precision)
    assert rel_fro(got, ref) < TOL[precision]
    # pair symmetry of the result (t is pair-symmetric, L symmetric)
    assert rel_fro(got.transpose(1, 0, 3, 2), got) < 10 * TOL[precision]


@pytest.mark.parametrize("precision", [0, 1])
def test_forward_tall_and_remainder_tiles(gpu_lib, precision):
    # o^2 = 1600 amplitude rows: for a 64-virtual block of v = 80 (20 tile
    # columns) 128-row tiles need two rounds of the 256 CUs, so float64 takes
    # 160-row tiles (one round) and float32 128-row tiles over 1536 rows plus a
    # 64-row launch over the last 64; the last block (16 virtuals, 5 columns)
    # takes plain 128-row tiles.  Whole tensor against the oracle, and integer
    # inputs exactly.
    o, v, P = 40, 80, 30
    announce("forward-tall-remainder", o, v, P, "precision", precision)
    L, t, _ = random_general(o, v, P, 4242)
    R0 = np.random.default_rng(11).standard_normal(t.shape)
    got = run_forward(gpu_lib, L, t, R0, precision, a_block=64)
    assert rel_fro(got - R0, oracle.ladder_forward(L, t)) < TOL[precision]
    Li, ti = integer_inputs(o, v, P, 4243)
    got = run_forward(gpu_lib, Li, ti, np.zeros_like(ti), precision, a_block=64)
    assert np.array_equal(got, oracle.ladder_forward(Li, ti))


def test_forward_bitwise_independent_of_block_size(gpu_lib):
    # every output's K-sum lives in one tile with the same step order, whatever
    # the integral block size
    announce("forward-determinism")
    L, t, _ = random_general(12, 44, 131, 5)
    z = np.zeros_like(t)
    ref = run_forward(gpu_lib, L, t, z, 0)
    for a_block in (1, 5, 13, 44):
        assert np.array_equal(run_forward(gpu_lib, L, t, z, 0, a_block=a_block), ref)
    assert np.array_equal(run_forward(gpu_lib, L, t, z, 0), ref)


def test_forward_caller_workspace(gpu_lib):
    announce("forward-workspace")
    L, t, _ = random_general(6, 30, 40, 8)
    nbytes, n_a = gpu_lib.cc_ladder_workspace_query(6, 30, 40, 0, opts=gpu_lib.make_opts(a_block=8))
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    ref = oracle.ladder_forward(L, t)
    R = dev(np.zeros_like(t))
    gpu_lib.cc_ladder_residual(dev(L), dev(t), R, 0, opts=gpu_lib.make_opts(a_block=8, workspace=ws))
    torch.cuda.synchronize()
    assert rel_fro(host(R), ref) < 1e-12
    small = ws[: nbytes // 2]
    with pytest.raises(gpu_lib.LadderError) as e:
        gpu_lib.cc_ladder_residual(dev(L), dev(t), R, 0,
                                   opts=gpu_lib.make_opts(a_block=8, workspace=small))
    assert e.value.code == gpu_lib.CC_LADDER_ENOMEM


def test_forward_on_side_stream(gpu_lib):
    announce("forward-stream")
    L, t, _ = random_general(4, 26, 30, 9)
    ref = oracle.ladder_forward(L, t)
    s = torch.cuda.Stream()
    Ld, td = dev(L), dev(t)
    R = torch.zeros_like(td)
    torch.cuda.synchronize()
    gpu_lib.cc_ladder_residual(Ld, td, R, 0, stream=s)
    s.synchronize()
    assert rel_fro(host(R), ref) < 1e-12


def _sampled_pairs(v, n, seed):
    rng = np.random.default_rng(seed)
    pairs = {(0, 0), (v - 1, v - 1), (0, v - 1), (v - 1, 0)}
    while len(pairs) < n:
        pairs.add((int(rng.integers(0, v)), int(rng.integers(0, v))))
    return sorted(pairs)


def test_reduce_matches_oracle(gpu_lib):
    announce("reduce")
    rng = np.random.default_rng(11)
    for o, v in ((1, 1), (3, 7), (20, 45)):
        x = rng.standard_normal((o, o, v, v))
        y = rng.standard_normal((o, o, v, v))
        out = host(gpu_lib.cc_ladder_reduce(dev(x), dev(y)))
        torch.cuda.synchronize()
        sxy, syy = oracle.reduce_dot(x, y)
        assert abs(out[0] - sxy) <= 1e-13 * np.sum(np.abs(x * y))
        assert abs(out[1] - syy) <= 1e-13 * syy


def _pair_symmetric(t):
    return 0.5 * (t + t.transpose(1, 0, 3, 2))


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("o,v,P,a_block", [(5, 20, 75, 0), (9, 37, 101, 7), (4, 44, 131, 13),
                                           (3, 130, 17, 40), (2, 3, 2, 0), (16, 64, 200, 1)])
def test_forward_pair_symmetric_path(gpu_lib, o, v, P, a_block, precision):
    # packed integral rows a <= b and mirrored results; any L, pair-symmetric t
    announce("forward-pairsym", o, v, P, "a_block", a_block, "precision", precision)
    L, t, _ = random_general(o, v, P, 700 + o + v)
    t = _pair_symmetric(t)
    R0 = np.random.default_rng(8).standard_normal(t.shape)
    inc = oracle.ladder_forward(L, t)
    got = run_forward(gpu_lib, L, t, R0, precision, a_block=a_block, pair_symmetric=True)
    assert rel_fro(got - R0, inc) < TOL[precision]


@pytest.mark.parametrize("precision", [0, 1, 2])
@pytest.mark.parametrize("o,v,P,a_block", [(5, 20, 75, 0), (9, 37, 101, 7), (3, 130, 17, 40),
                                           (2, 1, 3, 0), (12, 44, 131, 13)])
def test_forward_exchange(gpu_lib, o, v, P, a_block, precision):
    # exchange partner (eq. vfunction2) on unsymmetric inputs: (ad|bc) differs
    # from (ac|bd) and nothing cancels; ragged v spans several 32-wide swap tiles
    announce("forward-exchange", o, v, P, "a_block", a_block, "precision", precision)
    L, t, _ = random_general(o, v, P, 900 + o + v)
    R0 = np.random.default_rng(9).standard_normal(t.shape)
    inc = oracle.exchange_forward(L, t)
    got = run_forward(gpu_lib, L, t, R0, precision, a_block=a_block, exchange=True)
    tol = TOL_SPLIT[4] if precision == 2 else TOL[precision]
    assert rel_fro(got - R0, inc) < tol


def test_forward_exchange_integer_exact(gpu_lib):
    announce("forward-exchange-int")
    L, t = integer_inputs(3, 10, 5, 78)
    ref = oracle.exchange_forward(L, t)
    for precision in (0, 1, 2):
        got = run_forward(gpu_lib, L, t, np.zeros_like(t), precision, exchange=True)
        assert np.array_equal(got, ref), precision


@pytest.mark.parametrize("precision", [0, 1])
def test_forward_exchange_pair_symmetric(gpu_lib, precision):
    # swapping c and d keeps pair symmetry, so both flags combine
    announce("forward-exchange-pairsym", precision)
    L, t, _ = random_general(9, 37, 101, 44)
    t = _pair_symmetric(t)
    inc = oracle.exchange_forward(L, t)
    got = run_forward(gpu_lib, L, t, np.zeros_like(t), precision, a_block=7, exchange=True,
                      pair_symmetric=True)
    assert rel_fro(got, inc) < TOL[precision]


def test_forward_exchange_full_size_sampled(gpu_lib):
    # the exchange partner at the 40/360/1200 workload, default options; the
    # oracle's columns come from the ladder of the swapped amplitudes, whose
    # identity with the exchange term is pinned on the CPU
    o, v, P = CONFIGS["o40_v360_P1200"]
    announce("forward-exchange-full", "o40_v360_P1200")
    inp = make_inputs(o, v, P, seed_for("o40_v360_P1200"), device="cuda")
    Ld, td = dev(inp.L_vv), dev(inp.t)
    pairs = _sampled_pairs(v, 16, 4)
    ref = oracle.ladder_pairs(inp.L_vv, np.ascontiguousarray(inp.t.transpose(0, 1, 3, 2)), pairs)
    ia = torch.tensor([a for a, _ in pairs], device="cuda")
    ib = torch.tensor([b for _, b in pairs], device="cuda")
    for precision in (0, 1, 2):
        R = torch.zeros_like(td)
        gpu_lib.cc_ladder_residual(Ld, td, R, precision, opts=gpu_lib.make_opts(exchange=True))
        torch.cuda.synchronize()
        tol = TOL_SPLIT_WORKLOAD[4] if precision == 2 else TOL[precision]
        assert rel_fro(host(R[:, :, ia, ib].permute(2, 0, 1)), ref) < tol, precision
        del R


def test_trace_hook_and_budget(gpu_lib):
    # the phase hook sees each phase of each integral block, in order, and a
    # budget that forces several blocks gives the planner's block count
    announce("forward-trace-budget")
    o, v, P = 6, 40, 50
    L, t, _ = random_general(o, v, P, 21)
    budget = 9 * v ** 3 * 4 + 4 * (P * v * v + o * o * v * v) + (1 << 16)
    nbytes, n_a = gpu_lib.cc_ladder_workspace_query(o, v, P, 1, hbm_budget=budget)
    assert 1 < n_a < v
    seen = []

    def hook(user, phase, block, end, stream):
        seen.append((phase, block, end))

    fn = gpu_lib.TRACE_FN(hook)
    R = dev(np.zeros_like(t))
    gpu_lib.cc_ladder_residual(dev(L), dev(t), R, 1, opts=gpu_lib.make_opts(hbm_budget=budget, trace=fn))
    torch.cuda.synchronize()
    assert rel_fro(host(R), oracle.ladder_forward(L, t)) < TOL[1]
    nb = -(-v // n_a)
    PREP, BUILD, CONTRACT = 0, 1, 2
    want = [(PREP, 0, 0), (PREP, 0, 1)]
    for b in range(nb):
        want += [(BUILD, b, 0), (BUILD, b, 1), (CONTRACT, b, 0), (CONTRACT, b, 1)]
    assert seen == want


def test_misaligned_workspace_is_rejected(gpu_lib):
    announce("forward-workspace-align")
    L, t, _ = random_general(3, 12, 10, 22)
    nbytes, _ = gpu_lib.cc_ladder_workspace_query(3, 12, 10, 0)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    R = dev(np.zeros_like(t))
    with pytest.raises(gpu_lib.LadderError) as e:
        gpu_lib.cc_ladder_residual(dev(L), dev(t), R, 0, opts=gpu_lib.make_opts(workspace=ws[8:]))
    assert e.value.code == gpu_lib.CC_LADDER_EINVAL
    torch.cuda.synchronize()
    assert not torch.any(R)  # nothing enqueued
