"""Helpers shared by the GPU parity tests (no arithmetic of the method here)."""
import sys

import numpy as np


def announce(*parts):
    """Names the case before any device work, so a failure that ends the run is attributable."""
    print("CASE", *parts, flush=True)
    sys.stdout.flush()


def dev(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def host(x):
    return x.detach().cpu().numpy()


def rel_fro(x, ref):
    den = np.linalg.norm(np.ravel(ref))
    return float(np.linalg.norm(np.ravel(x - ref)) / (den if den > 0 else 1.0))


# Relative Frobenius tolerances of each arithmetic form against the float64 oracle.
TOL = {0: 1e-12, 1: 1e-6, 2: 1e-9}
# split-bf16 at S slices, default product sets.  S = 3, 4: exponent-aligned
# digits, each operand keeping 8S bits below its row (or chunk) maximum; on
# unstructured N(0,1) inputs a row's maximum is about four times its rms, and
# the representation errors of the four operands of the two products add, so
# S = 4 is held to 2e-9 there and to the precision form's 1e-9 on the MP2-like
# workloads; S = 3 to 16 * 2^-24.  S = 2: the per-element hi/lo split, each
# operand within 2^-16 of itself plus the dropped lo*lo product and float32
# sums: 16 * 2^-16 on unstructured inputs, 2e-5 on the workloads (about 6e-6
# measured).  S = 2 cannot meet the 1e-9 target and is reported with its error.
TOL_SPLIT = {2: 16 * 2.0 ** -16, 3: 16 * 2.0 ** -24, 4: 2e-9}
TOL_SPLIT_WORKLOAD = {2: 2e-5, 3: 16 * 2.0 ** -24, 4: 1e-9}
