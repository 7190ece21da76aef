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
TOL = {0: 1e-12, 1: 1e-6}
