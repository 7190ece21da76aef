"""Whole-tensor parity at the workloads' real shapes, in the launch
configuration the benchmark times (default options, library-planned blocks).

The oracle evaluates the complete R of the 20/180/600 and 40/360/1200
workloads once (about 2 and 100 seconds of host BLAS) and every arithmetic form
is held to its relative Frobenius tolerance over the whole tensor.  On the
30/300/900 gradient workload the adjoint is held to the whole-tensor
identities of the quadratic loss (Euler's theorem for the parts linear in t
and quadratic in L) and to self-adjointness: with symmetric Cholesky vectors
the integral satisfies V[c,a,d,b] = V[a,c,b,d], so dt equals the ladder
evaluated on lam, which the oracle computes whole.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2310_04559_amd.inputs import CONFIGS, make_inputs, seed_for
from tests.gpu_common import TOL, TOL_SPLIT_WORKLOAD, announce, dev, host, rel_fro

pytestmark = pytest.mark.gpu

# (precision, split slices, pair-symmetric) -> tolerance over the whole tensor
# ("pm": the symmetric/antisymmetric combinations over i <= j, a <= b, c <= d;
# "pmv": the same gathered from the whole pair-pair integral of the workload's
# symmetric Cholesky vectors; "sv": the packed rows gathered from it)
FORMS = [(0, 0, False, TOL[0]), (1, 0, False, TOL[1]), (2, 4, False, TOL_SPLIT_WORKLOAD[4]),
         (2, 2, False, TOL_SPLIT_WORKLOAD[2]), (0, 0, True, TOL[0]), (1, 0, True, TOL[1]),
         (2, 4, True, TOL_SPLIT_WORKLOAD[4]), (0, 0, "pm", TOL[0]), (1, 0, "pm", TOL[1]),
         (0, 0, "pmv", TOL[0]), (1, 0, "pmv", TOL[1]), (0, 0, "sv", TOL[0]), (1, 0, "sv", TOL[1]),
         (3, 5, False, TOL[2]), (3, 5, True, TOL[2]), (3, 5, "sv", TOL[2]),
         (2, 4, "sv", TOL_SPLIT_WORKLOAD[4])]


def _check_forms(native, name, Ld, td, ref):
    nref = np.linalg.norm(ref)
    for precision, slices, sym, tol in FORMS:
        announce("whole", name, "precision", precision, "slices", slices, "pairsym", sym)
        R = torch.zeros_like(td)
        native.cc_ladder_residual(Ld, td, R, precision,
                                  opts=native.make_opts(split_slices=slices, pair_symmetric=bool(sym),
                                                        plus_minus=sym in ("pm", "pmv"),
                                                        symmetric_vectors=sym in ("pmv", "sv")))
        torch.cuda.synchronize()
        if sym:
            # entries a != b are stored twice from one computed value: exact mirrors
            v = R.shape[2]
            off = ~torch.eye(v, dtype=torch.bool, device=R.device)[None, None]
            assert torch.equal(torch.where(off, R, 0.0), torch.where(off, R.permute(1, 0, 3, 2), 0.0))
        got = host(R)
        del R
        err = float(np.linalg.norm(got - ref) / nref)
        print(f"CASE whole {name} precision {precision} slices {slices} pairsym {sym} "
              f"rel. Frobenius error {err:.3e} (tolerance {tol:.1e})", flush=True)
        assert err < tol, (name, precision, slices, sym, err)


def test_whole_tensor_o20_v180_P600(gpu_lib):
    name = "o20_v180_P600"
    o, v, P = CONFIGS[name]
    announce("whole-oracle", name)
    inp = make_inputs(o, v, P, seed_for(name))
    ref = oracle.ladder_forward(inp.L_vv, inp.t)
    Ld, td = dev(inp.L_vv), dev(inp.t)
    _check_forms(gpu_lib, name, Ld, td, ref)
    # the exchange partner (eq. vfunction2) over the whole tensor
    ref_x = oracle.exchange_forward(inp.L_vv, inp.t)
    for precision, slices, tol in ((0, 0, TOL[0]), (1, 0, TOL[1]), (2, 4, TOL_SPLIT_WORKLOAD[4])):
        announce("whole-exchange", name, precision)
        R = torch.zeros_like(td)
        gpu_lib.cc_ladder_residual(Ld, td, R, precision,
                                   opts=gpu_lib.make_opts(split_slices=slices, exchange=True))
        torch.cuda.synchronize()
        err = rel_fro(host(R), ref_x)
        print(f"CASE whole-exchange {name} precision {precision} error {err:.3e}", flush=True)
        assert err < tol, (precision, err)


@pytest.mark.timeout(900)
def test_whole_tensor_o40_v360_P1200(gpu_lib):
    name = "o40_v360_P1200"
    o, v, P = CONFIGS[name]
    announce("whole-oracle", name, "(host oracle, about 100 s)")
    inp = make_inputs(o, v, P, seed_for(name), device="cuda")
    ref = oracle.ladder_forward(inp.L_vv, inp.t)
    print("CASE whole-oracle done", flush=True)
    _check_forms(gpu_lib, name, dev(inp.L_vv), dev(inp.t), ref)


@pytest.mark.timeout(600)
def test_whole_tensor_adjoint_o30_v300_P900(gpu_lib):
    name = "o30_v300_P900"
    o, v, P = CONFIGS[name]
    announce("whole-adjoint", name)
    inp = make_inputs(o, v, P, seed_for(name), with_lambda=True, device="cuda")
    Ld, td, lamd = dev(inp.L_vv), dev(inp.t), dev(inp.lam)
    # dt = Ladder(lam) for symmetric vectors (pinned on the CPU), whole tensor
    dt_ref = oracle.ladder_forward(inp.L_vv, inp.lam)
    R = torch.zeros_like(td)
    gpu_lib.cc_ladder_residual(Ld, td, R, 0)
    Rl = torch.zeros_like(td)
    gpu_lib.cc_ladder_residual(Ld, lamd, Rl, 0)
    torch.cuda.synchronize()
    loss = float(torch.sum(lamd * R))
    for precision in (0, 1):
        for sym in (False, True):
            announce("whole-adjoint", name, "precision", precision, "pairsym", sym)
            dL = torch.zeros_like(Ld)
            dt = torch.zeros_like(td)
            gpu_lib.cc_ladder_backward(Ld, td, lamd, dL, dt, precision,
                                       opts=gpu_lib.make_opts(pair_symmetric=sym))
            torch.cuda.synchronize()
            tol = TOL[precision]
            err_dt = rel_fro(host(dt), dt_ref)
            # self-adjointness against the library's own forward of lam
            err_self = float(torch.linalg.vector_norm(dt - Rl) / torch.linalg.vector_norm(Rl))
            # Euler: <dt, t> = Loss (linear in t), <dL, L> = 2 Loss (quadratic in L).
            # The scalars are held relative to |dt||t| and |dL||L|: by Cauchy-Schwarz
            # |<dt - dt_exact, t>| <= |dt - dt_exact| |t|, so a gradient within its
            # relative Frobenius tolerance meets the identity within that tolerance
            # of |dt||t|, while Loss itself (a sum against zero-mean lam) cancels down
            # to a few times less than |dt||t|.
            nrm = lambda x: float(torch.linalg.vector_norm(x))
            e_t = abs(float(torch.sum(dt * td)) - loss) / (nrm(dt) * nrm(td))
            e_L = abs(float(torch.sum(dL * Ld)) - 2.0 * loss) / (nrm(dL) * nrm(Ld))
            print(f"CASE whole-adjoint precision {precision} pairsym {sym}: dt vs oracle "
                  f"{err_dt:.3e}, dt vs ladder(lam) {err_self:.3e}, Euler t {e_t:.3e}, "
                  f"Euler L {e_L:.3e}", flush=True)
            assert err_dt < tol and err_self < tol, (precision, sym, err_dt, err_self)
            assert e_t < tol and e_L < tol, (precision, sym, e_t, e_L)
            del dL, dt
