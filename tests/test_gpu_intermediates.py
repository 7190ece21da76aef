"""GPU parity of the occupied intermediates (eqs. vfunction3 and vfunction4)
and of the hole-hole ladder against the float64 oracle, through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
from paper_2310_04559_amd.inputs import (CONFIGS, integer_inputs, integer_ov, make_inputs,
                                         random_general, random_ov, seed_for)
from tests.gpu_common import TOL, announce, dev, host, rel_fro

pytestmark = pytest.mark.gpu

# (o, v, P): ragged against the tiles, odd v (unaligned rows), o = 1, v = 1,
# several tiles in every dimension
SHAPES = [(5, 20, 75), (9, 37, 101), (3, 130, 17), (1, 3, 1), (2, 1, 3), (13, 44, 131),
          (16, 64, 200)]


def run(native, which, L, Lov, t, Z0, precision, **kw):
    Z = dev(Z0)
    opts = native.make_opts(**kw)
    if which == "ijkl":
        native.cc_intermediate_ijkl(dev(Lov), dev(t), Z, precision, opts=opts)
    else:
        native.cc_intermediate_ijbk(dev(L), dev(Lov), dev(t), Z, precision, opts=opts)
    torch.cuda.synchronize()
    return host(Z)


def reference(which, L, Lov, t):
    if which == "ijkl":
        return oracle.intermediate_ijkl(Lov, t)
    return oracle.intermediate_ijbk(L, Lov, t)


def out_shape(which, o, v):
    return (o, o, o, o) if which == "ijkl" else (o, o, v, o)


@pytest.mark.parametrize("which", ["ijkl", "ijbk"])
@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("o,v,P", SHAPES)
@pytest.mark.parametrize("block", [0, 2])
def test_intermediate_general_inputs(gpu_lib, which, o, v, P, block, precision):
    announce("intermediate", which, o, v, P, "block", block, "precision", precision)
    L, t, _ = random_general(o, v, P, 400 + o + v)
    Lov = random_ov(o, v, P, 500 + o + v)
    Z0 = np.random.default_rng(6).standard_normal(out_shape(which, o, v))
    inc = reference(which, L, Lov, t)
    got = run(gpu_lib, which, L, Lov, t, Z0, precision, a_block=block)
    assert rel_fro(got - Z0, inc) < TOL[precision]


@pytest.mark.parametrize("which", ["ijkl", "ijbk"])
def test_intermediate_integer_inputs_exact(gpu_lib, which):
    announce("intermediate-int", which)
    L, t = integer_inputs(3, 10, 5, 87)
    Lov = integer_ov(3, 10, 5, 88)
    ref = reference(which, L, Lov, t)
    for precision in (0, 1):
        got = run(gpu_lib, which, L, Lov, t, np.zeros(out_shape(which, 3, 10)), precision)
        assert np.array_equal(got, ref), precision


@pytest.mark.parametrize("which", ["ijkl", "ijbk"])
@pytest.mark.parametrize("o,v,P", [(9, 37, 101), (16, 64, 200)])
def test_intermediate_bitwise_independent_of_block_size(gpu_lib, which, o, v, P):
    # (16, 64, 200) splits the contraction's K into ranges; the ranges depend on
    # the whole output, not on the block, so every block sums in one order
    announce("intermediate-determinism", which, o, v, P)
    L, t, _ = random_general(o, v, P, 12)
    Lov = random_ov(o, v, P, 13)
    z = np.zeros(out_shape(which, o, v))
    for precision in (0, 1):
        ref = run(gpu_lib, which, L, Lov, t, z, precision)
        for block in (1, 4, 7):
            got = run(gpu_lib, which, L, Lov, t, z, precision, a_block=block)
            assert np.array_equal(got, ref), (precision, block)


@pytest.mark.parametrize("which", ["ijkl", "ijbk"])
@pytest.mark.parametrize("name", ["o5_v20_P75", "o20_v180_P600"])
def test_intermediate_workloads(gpu_lib, which, name):
    # the generator's own vectors: L_ov is the occupied-virtual block of the
    # same symmetric Cholesky vectors, t the MP2-like amplitudes
    o, v, P = CONFIGS[name]
    announce("intermediate-workload", which, name)
    inp = make_inputs(o, v, P, seed_for(name))
    ref = reference(which, inp.L_vv, inp.L_ov, inp.t)
    for precision in (0, 1):
        got = run(gpu_lib, which, inp.L_vv, inp.L_ov, inp.t, np.zeros_like(ref), precision)
        assert rel_fro(got, ref) < TOL[precision], precision
    if which == "ijkl":
        # (kc|ld) = (ld|kc) and pair-symmetric t: X[i,j,k,l] = X[j,i,l,k]
        assert rel_fro(got.transpose(1, 0, 3, 2), got) < 10 * TOL[1]


@pytest.mark.parametrize("which", ["ijkl", "ijbk"])
def test_intermediate_full_size_sampled(gpu_lib, which):
    # the 40/360/1200 workload with default options; the oracle computes whole
    # slices X[:, :, k, :] or Y[:, :, b, :] for a few first indices
    o, v, P = CONFIGS["o40_v360_P1200"]
    announce("intermediate-full", which)
    inp = make_inputs(o, v, P, seed_for("o40_v360_P1200"), device="cuda")
    firsts = [0, o // 2, o - 1] if which == "ijkl" else [0, 17, v // 2, v - 1]
    ref = np.zeros(out_shape(which, o, v))
    for p in firsts:
        if which == "ijkl":
            oracle.intermediate_ijkl(inp.L_ov, inp.t, ref, p, p + 1)
        else:
            oracle.intermediate_ijbk(inp.L_vv, inp.L_ov, inp.t, ref, p, p + 1)
    Ld, Lovd, td = dev(inp.L_vv), dev(inp.L_ov), dev(inp.t)
    for precision in (0, 1):
        Z = torch.zeros(out_shape(which, o, v), dtype=torch.float64, device="cuda")
        if which == "ijkl":
            gpu_lib.cc_intermediate_ijkl(Lovd, td, Z, precision)
        else:
            gpu_lib.cc_intermediate_ijbk(Ld, Lovd, td, Z, precision)
        torch.cuda.synchronize()
        got = host(Z)
        assert rel_fro(got[:, :, firsts, :], ref[:, :, firsts, :]) < TOL[precision], precision


def test_intermediate_caller_workspace_and_unsupported(gpu_lib):
    announce("intermediate-workspace")
    o, v, P = 4, 26, 30
    L, t, _ = random_general(o, v, P, 14)
    Lov = random_ov(o, v, P, 15)
    nbytes, _ = gpu_lib.cc_intermediate_workspace_query("ijbk", o, v, P, 0,
                                                         opts=gpu_lib.make_opts(a_block=v))
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    Y = torch.zeros((o, o, v, o), dtype=torch.float64, device="cuda")
    gpu_lib.cc_intermediate_ijbk(dev(L), dev(Lov), dev(t), Y, 0,
                                 opts=gpu_lib.make_opts(workspace=ws, a_block=v))
    torch.cuda.synchronize()
    assert rel_fro(host(Y), oracle.intermediate_ijbk(L, Lov, t)) < TOL[0]
    # a fixed block that does not fit the workspace; without one, the planner
    # shrinks the block to what the workspace holds
    half = ws[: nbytes // 2]
    with pytest.raises(gpu_lib.LadderError) as e:
        gpu_lib.cc_intermediate_ijbk(dev(L), dev(Lov), dev(t), Y, 0,
                                     opts=gpu_lib.make_opts(workspace=half, a_block=v))
    assert e.value.code == gpu_lib.CC_LADDER_ENOMEM
    Y.zero_()
    gpu_lib.cc_intermediate_ijbk(dev(L), dev(Lov), dev(t), Y, 0, opts=gpu_lib.make_opts(workspace=half))
    torch.cuda.synchronize()
    assert rel_fro(host(Y), oracle.intermediate_ijbk(L, Lov, t)) < TOL[0]
    X = torch.zeros((o, o, o, o), dtype=torch.float64, device="cuda")
    with pytest.raises(gpu_lib.LadderError) as e:
        gpu_lib.cc_intermediate_ijkl(dev(Lov), dev(t), X, 2)
    assert e.value.code == gpu_lib.CC_LADDER_EUNSUPPORTED


def random_oo(o, P, seed):
    return np.random.default_rng(seed).standard_normal((P, o, o)) / np.sqrt(o)


def run_hole(native, Loo, t, R0, precision, **kw):
    R = dev(R0)
    native.cc_hole_ladder(dev(Loo), dev(t), R, precision, opts=native.make_opts(**kw))
    torch.cuda.synchronize()
    return host(R)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("o,v,P", SHAPES + [(37, 9, 40), (130, 3, 7)])
@pytest.mark.parametrize("block", [0, 3])
def test_hole_ladder_general_inputs(gpu_lib, o, v, P, block, precision):
    # unsymmetric L_oo and t; o up to 130 spans several tiles of the (i,k) rows
    announce("hole", o, v, P, "block", block, "precision", precision)
    _, t, _ = random_general(o, v, P, 800 + o + v)
    Loo = random_oo(o, P, 810 + o)
    R0 = np.random.default_rng(7).standard_normal(t.shape)
    inc = oracle.hole_ladder(Loo, t)
    got = run_hole(gpu_lib, Loo, t, R0, precision, a_block=block)
    assert rel_fro(got - R0, inc) < TOL[precision]


def test_hole_ladder_integer_exact_and_deterministic(gpu_lib):
    announce("hole-int")
    _, t = integer_inputs(7, 6, 5, 89)
    Loo = np.random.default_rng(90).integers(-2, 3, size=(5, 7, 7)).astype(np.float64)
    ref = oracle.hole_ladder(Loo, t)
    for precision in (0, 1):
        assert np.array_equal(run_hole(gpu_lib, Loo, t, np.zeros_like(t), precision), ref)
    _, t, _ = random_general(13, 44, 131, 91)
    Loo = random_oo(13, 131, 92)
    z = np.zeros_like(t)
    base = run_hole(gpu_lib, Loo, t, z, 0)
    for block in (1, 5):
        assert np.array_equal(run_hole(gpu_lib, Loo, t, z, 0, a_block=block), base)


@pytest.mark.parametrize("name", ["o5_v20_P75", "o20_v180_P600", "o40_v360_P1200"])
def test_hole_ladder_workloads(gpu_lib, name):
    # the generator's own occupied-occupied vectors; at 40/360/1200 the oracle
    # computes the rows of a few occupied i
    o, v, P = CONFIGS[name]
    announce("hole-workload", name)
    inp = make_inputs(o, v, P, seed_for(name), device="cuda" if name == "o40_v360_P1200" else None)
    rows = list(range(o)) if name != "o40_v360_P1200" else [0, o // 2, o - 1]
    ref = np.zeros_like(inp.t)
    for i in rows:
        oracle.hole_ladder(inp.L_oo, inp.t, ref, i, i + 1)
    Ld, td = dev(inp.L_oo), dev(inp.t)
    for precision in (0, 1):
        R = torch.zeros_like(td)
        gpu_lib.cc_hole_ladder(Ld, td, R, precision)
        torch.cuda.synchronize()
        got = host(R)
        assert rel_fro(got[rows], ref[rows]) < TOL[precision], precision
        # (ik|jl) = (jl|ik) with pair-symmetric t: R[i,j,a,b] = R[j,i,b,a]
        assert rel_fro(got.transpose(1, 0, 3, 2), got) < 10 * TOL[precision]
        del R
