"""GPU parity of the hand-written adjoint against the float64 oracle, and the
autograd wrapper, through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
from paper_2310_04559_amd.inputs import CONFIGS, integer_inputs, make_inputs, random_general, seed_for
from tests.gpu_common import announce, dev, host, rel_fro

pytestmark = pytest.mark.gpu

TOL_BWD = {0: 1e-12, 1: 1e-6}


def run_backward(native, L, t, lam, precision, dL0=None, dt0=None, **kw):
    dL = dev(np.zeros_like(L) if dL0 is None else dL0)
    dt = dev(np.zeros_like(t) if dt0 is None else dt0)
    native.cc_ladder_backward(dev(L), dev(t), dev(lam), dL, dt, precision,
                              opts=native.make_opts(**kw))
    torch.cuda.synchronize()
    return host(dL), host(dt)


@pytest.mark.parametrize("precision", [0, 1])
def test_backward_oracle_gradient_small(gpu_lib, precision):
    # the gradient workload's oracle size: o=4, v=12, P=40
    announce("backward-small", precision)
    inp = make_inputs(4, 12, 40, seed_for("o30_v300_P900"), with_lambda=True)
    dL_ref, dt_ref = oracle.ladder_backward(inp.L_vv, inp.t, inp.lam)
    dL, dt = run_backward(gpu_lib, inp.L_vv, inp.t, inp.lam, precision)
    assert rel_fro(dL, dL_ref) < TOL_BWD[precision]
    assert rel_fro(dt, dt_ref) < TOL_BWD[precision]


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("o,v,P,a_block", [(5, 23, 37, 5), (9, 37, 101, 0), (3, 130, 17, 40),
                                           (12, 44, 70, 1)])
def test_backward_general_inputs(gpu_lib, o, v, P, a_block, precision):
    # unsymmetric L, t and lam: the two dL terms differ, nothing cancels
    announce("backward", o, v, P, "a_block", a_block, "precision", precision)
    L, t, lam = random_general(o, v, P, 200 + o + v)
    dL0 = np.random.default_rng(1).standard_normal(L.shape)
    dt0 = np.random.default_rng(2).standard_normal(t.shape)
    dL_ref, dt_ref = oracle.ladder_backward(L, t, lam)
    dL, dt = run_backward(gpu_lib, L, t, lam, precision, dL0, dt0, a_block=a_block)
    assert rel_fro(dL - dL0, dL_ref) < TOL_BWD[precision]
    assert rel_fro(dt - dt0, dt_ref) < TOL_BWD[precision]


def test_autograd_function(gpu_lib):
    announce("autograd")
    from paper_2310_04559_amd.ladder import ladder

    L, t, lam = random_general(4, 18, 25, 31)
    Ld = dev(L).requires_grad_(True)
    td = dev(t).requires_grad_(True)
    R = ladder(Ld, td)
    loss = (R * dev(lam)).sum()
    gL, gt = torch.autograd.grad(loss, (Ld, td))
    dL_ref, dt_ref = oracle.ladder_backward(L, t, lam)
    assert rel_fro(host(R), oracle.ladder_forward(L, t)) < 1e-12
    assert rel_fro(host(gL), dL_ref) < 1e-12
    assert rel_fro(host(gt), dt_ref) < 1e-12


def test_central_differences_gradient_workload(gpu_lib):
    # the gradient workload (o=30, v=300, P=900): Loss = sum lam*R evaluated by
    # the GPU forward; central differences with h = 1e-6 are exact up to rounding
    # (Loss is quadratic in L and linear in t).  L entries are drawn among the
    # leading vectors, where the gradient stands above the rounding floor.
    o, v, P = CONFIGS["o30_v300_P900"]
    announce("backward-fd", o, v, P)
    inp = make_inputs(o, v, P, seed_for("o30_v300_P900"), with_lambda=True, device="cuda")
    Ld, td, lamd = dev(inp.L_vv), dev(inp.t), dev(inp.lam)
    dL = torch.zeros_like(Ld)
    dt = torch.zeros_like(td)
    gpu_lib.cc_ladder_backward(Ld, td, lamd, dL, dt, 0)
    torch.cuda.synchronize()
    rng = np.random.default_rng(seed_for("o30_v300_P900") + 1)
    h = 1e-6
    R = torch.empty_like(td)
    out = torch.empty(2, dtype=torch.float64, device="cuda")

    def loss(Lx, tx):
        R.zero_()
        gpu_lib.cc_ladder_residual(Lx, tx, R, 0)
        gpu_lib.cc_ladder_reduce(lamd, R, out)
        return float(out[0])

    gLmax = float(dL.abs().max())
    gtmax = float(dt.abs().max())
    for k in range(10):
        x, p, q = int(rng.integers(0, 100)), int(rng.integers(0, v)), int(rng.integers(0, v))
        keep = float(Ld[x, p, q])
        Ld[x, p, q] = keep + h
        fp = loss(Ld, td)
        Ld[x, p, q] = keep - h
        fm = loss(Ld, td)
        Ld[x, p, q] = keep
        fd = (fp - fm) / (2 * h)
        g = float(dL[x, p, q])
        assert abs(fd - g) <= 1e-6 * abs(g) + 1e-9 * gLmax, (k, x, p, q, fd, g)
    for k in range(10):
        idx = tuple(int(rng.integers(0, s)) for s in inp.t.shape)
        keep = float(td[idx])
        td[idx] = keep + h
        fp = loss(Ld, td)
        td[idx] = keep - h
        fm = loss(Ld, td)
        td[idx] = keep
        fd = (fp - fm) / (2 * h)
        g = float(dt[idx])
        assert abs(fd - g) <= 1e-6 * abs(g) + 1e-9 * gtmax, (k, idx, fd, g)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("o,v,P,a_block", [(5, 23, 37, 5), (3, 130, 17, 40), (9, 37, 101, 0)])
def test_backward_exchange(gpu_lib, o, v, P, a_block, precision):
    # adjoint of the exchange partner (eq. vfunction2), accumulated onto given
    # dL and dt, against the oracle's gradients of that term
    announce("backward-exchange", o, v, P, "a_block", a_block, "precision", precision)
    L, t, lam = random_general(o, v, P, 600 + o + v)
    dL0 = np.random.default_rng(3).standard_normal(L.shape)
    dt0 = np.random.default_rng(4).standard_normal(t.shape)
    dL_ref, dt_ref = oracle.exchange_backward(L, t, lam)
    dL, dt = run_backward(gpu_lib, L, t, lam, precision, dL0, dt0, a_block=a_block, exchange=True)
    assert rel_fro(dL - dL0, dL_ref) < TOL_BWD[precision]
    assert rel_fro(dt - dt0, dt_ref) < TOL_BWD[precision]


def test_backward_exchange_integer_exact(gpu_lib):
    announce("backward-exchange-int")
    L, t = integer_inputs(3, 10, 5, 79)
    lam = integer_inputs(3, 10, 5, 80)[1]
    dL_ref, dt_ref = oracle.exchange_backward(L, t, lam)
    for precision in (0, 1):
        dL, dt = run_backward(gpu_lib, L, t, lam, precision, exchange=True)
        assert np.array_equal(dL, dL_ref) and np.array_equal(dt, dt_ref), precision


def test_autograd_function_exchange(gpu_lib):
    announce("autograd-exchange")
    from paper_2310_04559_amd.ladder import ladder

    L, t, lam = random_general(4, 18, 25, 32)
    Ld = dev(L).requires_grad_(True)
    td = dev(t).requires_grad_(True)
    R = ladder(Ld, td, opts=gpu_lib.make_opts(exchange=True))
    gL, gt = torch.autograd.grad((R * dev(lam)).sum(), (Ld, td))
    dL_ref, dt_ref = oracle.exchange_backward(L, t, lam)
    assert rel_fro(host(R), oracle.exchange_forward(L, t)) < 1e-12
    assert rel_fro(host(gL), dL_ref) < 1e-12
    assert rel_fro(host(gt), dt_ref) < 1e-12


def _pair_symmetric(x):
    return 0.5 * (x + x.transpose(1, 0, 3, 2))


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("exchange,symv", [(False, False), (True, False), (False, True),
                                           (True, True)])
@pytest.mark.parametrize("o,v,P,a_block", [(5, 23, 37, 5), (9, 37, 101, 0), (3, 130, 17, 40)])
def test_backward_pair_symmetric(gpu_lib, o, v, P, a_block, precision, exchange, symv):
    # t and lam pair-symmetric: the half-written W block gives both dL terms;
    # with symmetric vectors the packed integral rows come from the pair-pair integral
    announce("backward-pairsym", o, v, P, "a_block", a_block, "precision", precision, exchange,
             "symv", symv)
    L, t, lam = random_general(o, v, P, 650 + o + v)
    t, lam = _pair_symmetric(t), _pair_symmetric(lam)
    if symv:
        L = 0.5 * (L + L.transpose(0, 2, 1))
    dL0 = np.random.default_rng(5).standard_normal(L.shape)
    dt0 = np.random.default_rng(6).standard_normal(t.shape)
    ref = oracle.exchange_backward(L, t, lam) if exchange else oracle.ladder_backward(L, t, lam)
    dL, dt = run_backward(gpu_lib, L, t, lam, precision, dL0, dt0, a_block=a_block,
                          pair_symmetric=True, exchange=exchange, symmetric_vectors=symv)
    assert rel_fro(dL - dL0, ref[0]) < TOL_BWD[precision]
    assert rel_fro(dt - dt0, ref[1]) < TOL_BWD[precision]


@pytest.mark.parametrize("precision,a_block,symv", [(0, 0, False), (0, 64, False), (1, 64, False),
                                                    (0, 0, True), (1, 0, True)])
def test_backward_pair_symmetric_gradient_workload(gpu_lib, precision, a_block, symv):
    # the gradient workload's lam and t are pair-symmetric: the symmetric adjoint
    # against the general one over the whole tensors (one block, or five blocks of
    # 64 virtuals whose half-written W blocks start past the first virtual)
    o, v, P = CONFIGS["o30_v300_P900"]
    announce("backward-pairsym-o30-v300-P900", "precision", precision, "a_block", a_block,
             "symv", symv)
    inp = make_inputs(o, v, P, seed_for("o30_v300_P900"), with_lambda=True, device="cuda")
    Ld, td, lamd = dev(inp.L_vv), dev(inp.t), dev(inp.lam)
    out = {}
    for sym in (False, True):
        dL = torch.zeros_like(Ld)
        dt = torch.zeros_like(td)
        gpu_lib.cc_ladder_backward(Ld, td, lamd, dL, dt, precision,
                                   opts=gpu_lib.make_opts(pair_symmetric=sym, a_block=a_block,
                                                          symmetric_vectors=sym and symv))
        torch.cuda.synchronize()
        out[sym] = (dL, dt)
    for k in (0, 1):
        den = float(torch.linalg.vector_norm(out[False][k]))
        # float64: both orders of summation agree to rounding; float32: each side
        # is within its own float32 bound of the float64 result
        assert float(torch.linalg.vector_norm(out[True][k] - out[False][k])) / den < (
            1e-12 if precision == 0 else 2 * TOL_BWD[1])


def test_autograd_clears_pair_symmetry_for_the_backward(gpu_lib):
    # a pair-symmetric forward with an unsymmetric upstream gradient
    announce("autograd-pairsym")
    from paper_2310_04559_amd.ladder import ladder

    L, t, lam = random_general(4, 18, 25, 33)
    t = _pair_symmetric(t)
    Ld = dev(L).requires_grad_(True)
    td = dev(t).requires_grad_(True)
    R = ladder(Ld, td, opts=gpu_lib.make_opts(pair_symmetric=True))
    gL, gt = torch.autograd.grad((R * dev(lam)).sum(), (Ld, td))
    dL_ref, dt_ref = oracle.ladder_backward(L, t, lam)
    assert rel_fro(host(gL), dL_ref) < 1e-12
    assert rel_fro(host(gt), dt_ref) < 1e-12


def test_autograd_inline_workspace_is_kept_and_not_reused_by_the_backward(gpu_lib):
    # a workspace made inline in the options call: the options keep it alive for
    # the forward, and the backward plans and allocates its own scratch
    announce("autograd-inline-workspace")
    from paper_2310_04559_amd.ladder import ladder

    o, v, P = 4, 18, 25
    L, t, lam = random_general(o, v, P, 34)
    nbytes, _ = gpu_lib.cc_ladder_workspace_query(o, v, P, 0)
    Ld = dev(L).requires_grad_(True)
    td = dev(t).requires_grad_(True)
    opts = gpu_lib.make_opts(workspace=torch.empty(nbytes, dtype=torch.uint8, device="cuda"))
    R = ladder(Ld, td, opts=opts)
    # allocations after the forward may not land in the workspace
    junk = [torch.full((nbytes // 8 + 1,), 7.0, dtype=torch.float64, device="cuda") for _ in range(3)]
    gL, gt = torch.autograd.grad((R * dev(lam)).sum(), (Ld, td))
    del junk
    dL_ref, dt_ref = oracle.ladder_backward(L, t, lam)
    assert rel_fro(host(R), oracle.ladder_forward(L, t)) < 1e-12
    assert rel_fro(host(gL), dL_ref) < 1e-12
    assert rel_fro(host(gt), dt_ref) < 1e-12


@pytest.mark.parametrize("precision", [0, 1])
def test_symmetry_check_flag(gpu_lib, precision):
    # with the check flag a false pair-symmetry assertion is an EINVAL that
    # leaves the outputs untouched; a true one runs as without the check
    announce("symmetry-check", precision)
    o, v, P = 5, 23, 37
    L, t, lam = random_general(o, v, P, 35)
    ts, lams = _pair_symmetric(t), _pair_symmetric(lam)
    R0 = np.random.default_rng(36).standard_normal(t.shape)
    kw = dict(pair_symmetric=True, check_symmetry=True)
    nudged = ts.copy()
    nudged[0, 1, 2, 3] += 1e-9 * np.abs(ts).max()  # one entry off its mirror
    for bad_t in (t, nudged):
        R = dev(R0)
        with pytest.raises(gpu_lib.LadderError) as e:
            gpu_lib.cc_ladder_residual(dev(L), dev(bad_t), R, precision, opts=gpu_lib.make_opts(**kw))
        assert e.value.code == gpu_lib.CC_LADDER_EINVAL
        torch.cuda.synchronize()
        assert np.array_equal(host(R), R0)
    R = dev(R0)
    gpu_lib.cc_ladder_residual(dev(L), dev(ts), R, precision, opts=gpu_lib.make_opts(**kw))
    R1 = dev(R0)
    gpu_lib.cc_ladder_residual(dev(L), dev(ts), R1, precision,
                               opts=gpu_lib.make_opts(pair_symmetric=True))
    torch.cuda.synchronize()
    assert torch.equal(R, R1)
    # the adjoint checks lam as well
    dL, dt = dev(np.zeros_like(L)), dev(np.zeros_like(t))
    with pytest.raises(gpu_lib.LadderError) as e:
        gpu_lib.cc_ladder_backward(dev(L), dev(ts), dev(lam), dL, dt, precision,
                                   opts=gpu_lib.make_opts(**kw))
    assert e.value.code == gpu_lib.CC_LADDER_EINVAL
    torch.cuda.synchronize()
    assert float(torch.count_nonzero(dL)) == 0 and float(torch.count_nonzero(dt)) == 0
    dL_ref, dt_ref = oracle.ladder_backward(L, ts, lams)
    gpu_lib.cc_ladder_backward(dev(L), dev(ts), dev(lams), dL, dt, precision,
                               opts=gpu_lib.make_opts(**kw))
    torch.cuda.synchronize()
    assert rel_fro(host(dL), dL_ref) < TOL_BWD[precision]
    assert rel_fro(host(dt), dt_ref) < TOL_BWD[precision]
