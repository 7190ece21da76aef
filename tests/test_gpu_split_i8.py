"""GPU parity of the split-int8 form (int8 digits on exponents per chunk of
16384 contracted indices, exact int32 sums on the integer MFMA, float64
drains) against the float64 oracle and the NumPy model of the digit scheme."""
import numpy as np
import pytest
import torch

import oracle
from paper_2310_04559_amd.inputs import (CONFIGS, integer_inputs, make_inputs, random_general,
                                         seed_for)
from tests import split_model
from tests.gpu_common import announce, dev, host, rel_fro

pytestmark = pytest.mark.gpu
I8 = 3

# Kernel against the NumPy model of the scheme: the digit products and their
# int32 chunk sums are exact on both sides, so only the float64 rounding of the
# drains (and a digit of the re-cut integral block flipping at a rounding
# boundary, at most 2^-39 of its row's maximum) separates them.
TOL_MODEL = 1e-12
# Against the oracle: five digits keep 39 bits below each chunk's maximum
# (about 2e-11 measured on unstructured inputs, 7e-11 on the workloads);
# four digits with the next anti-diagonal 31 bits (1.3e-9 and 2e-9).
TOL = {(5, 1): 1e-9, (4, 2): 1e-8, (4, 1): 4e-8}


def run_i8(native, L, t, R0, slices=0, depth=0, **kw):
    R = dev(R0)
    native.cc_ladder_residual(dev(L), dev(t), R, I8,
                              opts=native.make_opts(split_slices=slices, split_depth=depth, **kw))
    torch.cuda.synchronize()
    return host(R)


@pytest.mark.parametrize("slices,depth", [(4, 1), (4, 2), (5, 1)])
@pytest.mark.parametrize("o,v,P", [(5, 20, 75), (9, 37, 101), (3, 44, 131)])
def test_i8_kernel_implements_the_digit_scheme(gpu_lib, o, v, P, slices, depth):
    announce("i8-model", o, v, P, slices, depth)
    L, t, _ = random_general(o, v, P, 600 + o + v)
    model = split_model.ladder_i8(L, t, slices, depth)
    got = run_i8(gpu_lib, L, t, np.zeros_like(t), slices, depth, a_block=7)
    err = rel_fro(got, model)
    print(f"CASE i8-model error {err:.3e}", flush=True)
    assert err < TOL_MODEL


def test_i8_integer_inputs_exact(gpu_lib):
    # integers need one digit each: every product and chunk sum is exact
    announce("i8-int")
    L, t = integer_inputs(3, 10, 5, 77)
    ref = oracle.ladder_forward(L, t)
    for slices in (4, 5):
        assert np.array_equal(run_i8(gpu_lib, L, t, np.zeros_like(t), slices), ref), slices


@pytest.mark.parametrize("o,v,P,a_block", [(5, 20, 75, 0), (9, 37, 101, 7), (12, 44, 131, 0),
                                           (3, 130, 17, 40), (1, 3, 1, 0), (16, 64, 200, 9),
                                           (2, 20, 16400, 0)])
def test_i8_general_inputs(gpu_lib, o, v, P, a_block):
    # (3, 130, 17): 16900 contracted indices, two exponent chunks and two drains
    # of the contraction; (2, 20, 16400): two chunks of the integral build
    announce("i8", o, v, P, "a_block", a_block)
    L, t, _ = random_general(o, v, P, 610 + o + v)
    R0 = np.random.default_rng(11).standard_normal(t.shape)
    inc = oracle.ladder_forward(L, t)
    for slices, depth in ((5, 1), (4, 2)):
        got = run_i8(gpu_lib, L, t, R0, slices, depth, a_block=a_block)
        err = rel_fro(got - R0, inc)
        print(f"CASE i8 {o} {v} {P} slices {slices} error {err:.2e}", flush=True)
        assert err < TOL[(slices, depth)], (slices, err)


def test_i8_two_build_chunks_match_the_model(gpu_lib):
    # the build's second chunk adds to the stored first one
    announce("i8-model-two-build-chunks")
    L, t, _ = random_general(2, 12, 16500, 620)
    model = split_model.ladder_i8(L, t, 5, 1)
    got = run_i8(gpu_lib, L, t, np.zeros_like(t), 5, 1)
    assert rel_fro(got, model) < TOL_MODEL


@pytest.mark.parametrize("o,v,P,a_block", [(5, 20, 75, 0), (9, 37, 101, 7), (3, 130, 17, 40)])
def test_i8_pair_symmetric_and_exchange(gpu_lib, o, v, P, a_block):
    announce("i8-pairsym-exchange", o, v, P, a_block)
    L, t, _ = random_general(o, v, P, 630 + o + v)
    t = 0.5 * (t + t.transpose(1, 0, 3, 2))
    ref = oracle.ladder_forward(L, t)
    got = run_i8(gpu_lib, L, t, np.zeros_like(t), a_block=a_block, pair_symmetric=True)
    assert rel_fro(got, ref) < TOL[(5, 1)]
    ref_x = oracle.exchange_forward(L, t)
    got = run_i8(gpu_lib, L, t, np.zeros_like(t), a_block=a_block, exchange=True)
    assert rel_fro(got, ref_x) < TOL[(5, 1)]
    got = run_i8(gpu_lib, L, t, np.zeros_like(t), a_block=a_block, exchange=True,
                 pair_symmetric=True)
    assert rel_fro(got, ref_x) < TOL[(5, 1)]


@pytest.mark.parametrize("o,v,P,a_block,exchange", [
    (5, 20, 75, 0, False), (9, 37, 101, 7, False), (4, 44, 131, 13, True), (3, 130, 17, 40, False),
    (2, 3, 2, 0, False), (1, 1, 3, 0, False), (2, 12, 16500, 5, False)])
def test_i8_symmetric_vectors(gpu_lib, o, v, P, a_block, exchange):
    # symmetric vectors: the pair-pair integral G from the packed vectors' digits,
    # then the block's packed rows gathered from it.  A column {a,c} of the packed
    # vectors carries the digits and exponent of column (a,c) of L, so every
    # element of G is the packed build's element bit for bit, and so is R;
    # (2, 12, 16500): two exponent chunks of G's product (stored, then added)
    announce("i8-symv", o, v, P, "a_block", a_block, "exchange", exchange)
    L, t, _ = random_general(o, v, P, 650 + o + v)
    L = 0.5 * (L + L.transpose(0, 2, 1))
    t = 0.5 * (t + t.transpose(1, 0, 3, 2))
    R0 = np.random.default_rng(13).standard_normal(t.shape)
    kw = dict(a_block=a_block, pair_symmetric=True, exchange=exchange)
    packed = run_i8(gpu_lib, L, t, R0, **kw)
    got = run_i8(gpu_lib, L, t, R0, symmetric_vectors=True, **kw)
    assert np.array_equal(got, packed)
    ref = oracle.exchange_forward(L, t) if exchange else oracle.ladder_forward(L, t)
    err = rel_fro(got - R0, ref)
    print(f"CASE i8-symv error {err:.2e}", flush=True)
    assert err < TOL[(5, 1)]


def test_i8_symmetric_vectors_footprint(gpu_lib):
    # G replaces the per-block packed build: the plan holds G and the packed
    # vectors, and falls back to the packed build when they do not fit
    o, v, P = 4, 60, 50
    q = lambda **kw: gpu_lib.cc_ladder_workspace_query(  # noqa: E731
        o, v, P, I8, opts=gpu_lib.make_opts(pair_symmetric=True, **kw))
    plain, _ = q()
    symv, _ = q(symmetric_vectors=True)
    npv = v * (v + 1) // 2
    assert symv >= plain + npv * npv * 8 - 3 * npv * 128 * 8
    L, t, _ = random_general(o, v, P, 660)
    L = 0.5 * (L + L.transpose(0, 2, 1))
    t = 0.5 * (t + t.transpose(1, 0, 3, 2))
    packed = run_i8(gpu_lib, L, t, np.zeros_like(t), pair_symmetric=True)
    # a budget of G's own size: the symmetric-vector plan cannot fit, the packed one does
    small = run_i8(gpu_lib, L, t, np.zeros_like(t), pair_symmetric=True, symmetric_vectors=True,
                   hbm_budget=npv * npv * 8)
    assert np.array_equal(small, packed)


def test_i8_c1_workload(gpu_lib):
    o, v, P = CONFIGS["o5_v20_P75"]
    announce("i8-o5-v20-P75")
    inp = make_inputs(o, v, P, seed_for("o5_v20_P75"))
    ref = oracle.ladder_forward(inp.L_vv, inp.t)
    err = rel_fro(run_i8(gpu_lib, inp.L_vv, inp.t, np.zeros_like(inp.t)), ref)
    print(f"CASE i8 o5_v20_P75 error {err:.2e}", flush=True)
    assert err < TOL[(5, 1)]


def test_i8_rejections(gpu_lib):
    announce("i8-rejections")
    L, t, lam = random_general(3, 10, 4, 640)
    Ld, td = dev(L), dev(t)
    with pytest.raises(gpu_lib.LadderError) as e:
        gpu_lib.cc_ladder_backward(Ld, td, dev(lam), torch.zeros_like(Ld), torch.zeros_like(td), I8)
    assert e.value.code == gpu_lib.CC_LADDER_EUNSUPPORTED
    with pytest.raises(gpu_lib.LadderError) as e:
        gpu_lib.cc_ladder_residual(Ld, td, torch.zeros_like(td), I8,
                                   opts=gpu_lib.make_opts(pair_symmetric=True, plus_minus=True))
    assert e.value.code == gpu_lib.CC_LADDER_EUNSUPPORTED
