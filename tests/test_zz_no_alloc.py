"""The no-allocation forward (cc_ladder_residual_noalloc, static device scratch)
against the allocating entry point, through the C ABI.

Two calls in a row on the static array, the second with a smaller input, in
every arithmetic form and with the pair-symmetric and exchange flags.  Given
the same block size the two entry points run the same kernels on the same
plan, so their results agree bit for bit; with its own plan (blocks sized to
the static array) the float64 result is held to the float64 tolerance against
the allocating call and against the oracle.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2310_04559_amd.inputs import make_inputs, random_general
from tests.gpu_common import TOL, announce, dev, host, rel_fro

pytestmark = pytest.mark.gpu

# (o, v, P): first call, then a smaller one (ragged tiles in both)
SHAPES = [(9, 70, 130), (5, 33, 41)]


def _pair(native, Ld, td, precision, **kw):
    """(allocating result, static-scratch result) on zeroed outputs."""
    opts = native.make_opts(**kw)
    R1 = torch.zeros_like(td)
    native.cc_ladder_residual(Ld, td, R1, precision, opts=opts)
    R2 = torch.zeros_like(td)
    native.cc_ladder_residual_noalloc(Ld, td, R2, precision, opts=native.make_opts(**kw))
    torch.cuda.synchronize()
    return R1, R2


@pytest.mark.parametrize("precision,slices", [(0, 0), (1, 0), (2, 4), (2, 2)])
@pytest.mark.parametrize("flag", ["plain", "pairsym", "exchange"])
def test_noalloc_matches_allocating_entry_point(gpu_lib, precision, slices, flag):
    for k, (o, v, P) in enumerate(SHAPES):
        announce("noalloc", "call", k, "o", o, "v", v, "P", P, "precision", precision,
                 "slices", slices, flag)
        inp = make_inputs(o, v, P, seed=700 + k)
        Ld, td = dev(inp.L_vv), dev(inp.t)
        # the same block size on both sides: the same plan and kernels
        n_a = 16 if k == 0 else 7
        R1, R2 = _pair(gpu_lib, Ld, td, precision, a_block=n_a, split_slices=slices,
                       pair_symmetric=flag == "pairsym", exchange=flag == "exchange")
        assert torch.equal(R1, R2), (k, precision, slices, flag)
        ref = oracle.exchange_forward(inp.L_vv, inp.t) if flag == "exchange" else \
            oracle.ladder_forward(inp.L_vv, inp.t)
        err = rel_fro(host(R2), ref)
        tol = TOL[precision] if precision != 2 else (1e-9 if slices == 4 else 2e-5)
        print(f"CASE noalloc call {k} rel. error vs oracle {err:.2e}", flush=True)
        assert err < tol, (k, err)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("symv", [False, True])
def test_noalloc_plus_minus_paths(gpu_lib, precision, symv):
    # the +- combinations, with the packed build or gathered from the whole
    # pair-pair integral of the workload's symmetric vectors (it fits the static array)
    for k, (o, v, P) in enumerate(SHAPES):
        announce("noalloc-pm", "call", k, "o", o, "v", v, "P", P, "precision", precision,
                 "symv", symv)
        inp = make_inputs(o, v, P, seed=720 + k)
        Ld, td = dev(inp.L_vv), dev(inp.t)
        R1, R2 = _pair(gpu_lib, Ld, td, precision, a_block=16 if k == 0 else 7,
                       pair_symmetric=True, plus_minus=True, symmetric_vectors=symv)
        assert torch.equal(R1, R2), (k, precision, symv)
        err = rel_fro(host(R2), oracle.ladder_forward(inp.L_vv, inp.t))
        print(f"CASE noalloc-pm call {k} rel. error vs oracle {err:.2e}", flush=True)
        assert err < TOL[precision], (k, err)


def test_noalloc_own_plan_and_accumulation(gpu_lib):
    # blocks sized by the library to the static array; R accumulates (+=)
    for k, (o, v, P) in enumerate([(20, 180, 600), (6, 50, 64)]):
        announce("noalloc-own-plan", "call", k, "o", o, "v", v, "P", P)
        inp = make_inputs(o, v, P, seed=710 + k)
        Ld, td = dev(inp.L_vv), dev(inp.t)
        nbytes, n_a = gpu_lib.cc_ladder_workspace_query(
            o, v, P, 0, hbm_budget=gpu_lib.CC_LADDER_NOALLOC_SCRATCH_BYTES)
        assert nbytes <= gpu_lib.CC_LADDER_NOALLOC_SCRATCH_BYTES
        R0 = dev(np.linspace(-1.0, 1.0, o * o * v * v).reshape(o, o, v, v))
        R1 = R0.clone()
        gpu_lib.cc_ladder_residual(Ld, td, R1, 0)
        R2 = R0.clone()
        gpu_lib.cc_ladder_residual_noalloc(Ld, td, R2, 0)
        torch.cuda.synchronize()
        d = rel_fro(host(R2 - R0), host(R1 - R0))
        err = rel_fro(host(R2 - R0), oracle.ladder_forward(inp.L_vv, inp.t))
        print(f"CASE noalloc own plan n_a {n_a}: vs allocating {d:.2e}, vs oracle {err:.2e}",
              flush=True)
        assert d < TOL[0] and err < TOL[0], (k, d, err)


def test_noalloc_rejections(gpu_lib):
    announce("noalloc-rejections")
    lib = gpu_lib.load()
    Lg, tg, _ = random_general(3, 24, 10, seed=720)
    Ld, td = dev(Lg), dev(tg)
    R = torch.zeros_like(td)
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    bad = [gpu_lib.make_opts(workspace=ws),
           gpu_lib.make_opts(pair_symmetric=True, check_symmetry=True)]
    for opts in bad:
        rc = lib.cc_ladder_residual_noalloc(3, 24, 10, Ld.data_ptr(), td.data_ptr(), R.data_ptr(),
                                            0, None, gpu_lib._opts_ref(opts))
        assert rc == gpu_lib.CC_LADDER_EINVAL
    # one float64 virtual of v = 330 needs 330^3 * 8 bytes > 256 MiB
    big = torch.zeros(1, 1, 330, 330, dtype=torch.float64, device="cuda")
    Lb = torch.zeros(2, 330, 330, dtype=torch.float64, device="cuda")
    Rb = torch.zeros_like(big)
    rc = lib.cc_ladder_residual_noalloc(1, 330, 2, Lb.data_ptr(), big.data_ptr(), Rb.data_ptr(),
                                        0, None, None)
    assert rc == gpu_lib.CC_LADDER_ENOMEM
    torch.cuda.synchronize()
    assert float(Rb.abs().max()) == 0.0 and float(R.abs().max()) == 0.0
