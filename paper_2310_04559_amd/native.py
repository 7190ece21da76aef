"""ctypes binding of libccladder.so: argument marshalling only.

Every function here has the name of the C entry point it calls and takes
torch tensors (device memory and streams come from PyTorch); all arithmetic
happens in the library's HIP kernels.  The library is required: when it is
not built, ``load()`` raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import torch  # loaded first so the library binds to the HIP runtime torch uses

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libccladder.so")

CC_LADDER_FP64 = 0
CC_LADDER_FP32 = 1
CC_LADDER_SPLIT_BF16 = 2
CC_LADDER_SPLIT_INT8 = 3
PRECISIONS = {"fp64": CC_LADDER_FP64, "fp32": CC_LADDER_FP32, "split_bf16": CC_LADDER_SPLIT_BF16,
              "split_int8": CC_LADDER_SPLIT_INT8}

CC_LADDER_OK = 0
# static scratch of cc_ladder_residual_noalloc, bytes per device
CC_LADDER_NOALLOC_SCRATCH_BYTES = 256 << 20
CC_LADDER_EINVAL = -1
CC_LADDER_ENOMEM = -2
CC_LADDER_ENODEV = -3
CC_LADDER_EHIP = -4
CC_LADDER_EUNSUPPORTED = -5

EXPORTS = ("cc_ladder_residual", "cc_ladder_residual_noalloc", "cc_ladder_backward", "cc_ladder_reduce",
           "cc_ladder_workspace_query", "cc_ladder_strerror", "cc_intermediate_ijkl",
           "cc_intermediate_ijbk", "cc_intermediate_workspace_query", "cc_hole_ladder")


class CcLadderOpts(ctypes.Structure):
    _fields_ = [
        ("a_block", ctypes.c_int),
        ("split_slices", ctypes.c_int),
        ("k_chunk", ctypes.c_int),
        ("split_depth", ctypes.c_int),
        ("hbm_budget", ctypes.c_size_t),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
        ("trace", ctypes.c_void_p),
        ("trace_user", ctypes.c_void_p),
        ("flags", ctypes.c_uint),
        ("reserved", ctypes.c_int),
    ]


CC_LADDER_PAIR_SYMMETRIC = 1
CC_LADDER_EXCHANGE = 2
CC_LADDER_CHECK_SYMMETRY = 4
CC_LADDER_PLUS_MINUS = 8
CC_LADDER_SYMMETRIC_VECTORS = 16
CC_INTERMEDIATE_IJKL = 0
CC_INTERMEDIATE_IJBK = 1
CC_HOLE_LADDER = 2
INTERMEDIATES = {"ijkl": CC_INTERMEDIATE_IJKL, "ijbk": CC_INTERMEDIATE_IJBK, "hole": CC_HOLE_LADDER}


TRACE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                            ctypes.c_void_p)
PHASES = {0: "prep", 1: "build", 2: "contract", 3: "dt", 4: "W", 5: "dL", 6: "slice"}


class LadderError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} (code {code})")


_lib = None


def load():
    """Loads the library (once).  Raises ImportError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    i, p, st = ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t
    opts_p = ctypes.POINTER(CcLadderOpts)
    lib.cc_ladder_residual.argtypes = [i, i, i, p, p, p, i, p, opts_p]
    lib.cc_ladder_residual.restype = i
    lib.cc_ladder_residual_noalloc.argtypes = [i, i, i, p, p, p, i, p, opts_p]
    lib.cc_ladder_residual_noalloc.restype = i
    lib.cc_ladder_backward.argtypes = [i, i, i, p, p, p, p, p, i, p, opts_p]
    lib.cc_ladder_backward.restype = i
    lib.cc_ladder_reduce.argtypes = [i, i, p, p, p, p]
    lib.cc_ladder_reduce.restype = i
    lib.cc_ladder_workspace_query.argtypes = [i, i, i, i, i, st, opts_p,
                                              ctypes.POINTER(st), ctypes.POINTER(i)]
    lib.cc_ladder_workspace_query.restype = i
    lib.cc_intermediate_ijkl.argtypes = [i, i, i, p, p, p, i, p, opts_p]
    lib.cc_intermediate_ijkl.restype = i
    lib.cc_intermediate_ijbk.argtypes = [i, i, i, p, p, p, p, i, p, opts_p]
    lib.cc_intermediate_ijbk.restype = i
    lib.cc_hole_ladder.argtypes = [i, i, i, p, p, p, i, p, opts_p]
    lib.cc_hole_ladder.restype = i
    lib.cc_intermediate_workspace_query.argtypes = [i, i, i, i, i, st, opts_p,
                                                    ctypes.POINTER(st), ctypes.POINTER(i)]
    lib.cc_intermediate_workspace_query.restype = i
    lib.cc_ladder_strerror.argtypes = [i]
    lib.cc_ladder_strerror.restype = ctypes.c_char_p
    _lib = lib
    return lib


def strerror(code: int) -> str:
    return load().cc_ladder_strerror(int(code)).decode()


def make_opts(a_block: int = 0, split_slices: int = 0, k_chunk: int = 0, hbm_budget: int = 0,
              workspace: Optional[torch.Tensor] = None, trace=None,
              split_depth: int = 0, pair_symmetric: bool = False,
              exchange: bool = False, check_symmetry: bool = False,
              plus_minus: bool = False, symmetric_vectors: bool = False) -> CcLadderOpts:
    """``trace`` is a TRACE_FN.  The options keep references to the workspace
    tensor and the trace callback, so neither is freed while they are in use."""
    o = CcLadderOpts()
    o.a_block = int(a_block)
    o.split_slices = int(split_slices)
    o.k_chunk = int(k_chunk)
    o.split_depth = int(split_depth)
    o.flags = ((CC_LADDER_PAIR_SYMMETRIC if pair_symmetric else 0)
               | (CC_LADDER_EXCHANGE if exchange else 0)
               | (CC_LADDER_CHECK_SYMMETRY if check_symmetry else 0)
               | (CC_LADDER_PLUS_MINUS if plus_minus else 0)
               | (CC_LADDER_SYMMETRIC_VECTORS if symmetric_vectors else 0))
    o.reserved = 0
    o.hbm_budget = int(hbm_budget)
    o._workspace_ref = None
    o._trace_ref = None
    if workspace is not None:
        if workspace.device.type != "cuda" or not workspace.is_contiguous():
            raise TypeError("workspace must be a contiguous device tensor")
        o.workspace = workspace.data_ptr()
        o.workspace_bytes = workspace.numel() * workspace.element_size()
        o._workspace_ref = workspace
    if trace is not None:
        o.trace = ctypes.cast(trace, ctypes.c_void_p)
        o._trace_ref = trace
    return o


def copy_opts(opts: CcLadderOpts, **changes) -> CcLadderOpts:
    """A copy of ``opts`` (with its references) with fields replaced; passing
    ``workspace=None`` drops the workspace and its reference."""
    o = CcLadderOpts.from_buffer_copy(opts)
    o._workspace_ref = getattr(opts, "_workspace_ref", None)
    o._trace_ref = getattr(opts, "_trace_ref", None)
    for k, val in changes.items():
        if k == "workspace":
            if val is None:
                o.workspace, o.workspace_bytes, o._workspace_ref = None, 0, None
            else:
                o.workspace = val.data_ptr()
                o.workspace_bytes = val.numel() * val.element_size()
                o._workspace_ref = val
        else:
            setattr(o, k, val)
    return o


def _prec(precision) -> int:
    if isinstance(precision, str):
        return PRECISIONS[precision]
    return int(precision)


def _dev_f64(x: torch.Tensor, name: str, shape=None) -> int:
    if not isinstance(x, torch.Tensor) or x.device.type != "cuda":
        raise TypeError(f"{name} must be a device tensor")
    if x.dtype != torch.float64 or not x.is_contiguous():
        raise TypeError(f"{name} must be contiguous float64")
    if shape is not None and tuple(x.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(x.shape)}, expected {tuple(shape)}")
    return x.data_ptr()


def _stream(dev, stream) -> int:
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    return s.cuda_stream


def _opts_ref(opts):
    return ctypes.byref(opts) if opts is not None else None


def _check(rc: int, where: str):
    if rc != CC_LADDER_OK:
        raise LadderError(rc, where)


def cc_ladder_residual(L: torch.Tensor, t: torch.Tensor, R: torch.Tensor, precision=0,
                       stream=None, opts: Optional[CcLadderOpts] = None) -> torch.Tensor:
    """R[i,j,a,b] += sum_cd (sum_x L[x,a,c] L[x,b,d]) t[i,j,c,d]; returns R."""
    lib = load()
    P, v, _ = L.shape
    o = t.shape[0]
    pL = _dev_f64(L, "L", (P, v, v))
    pt = _dev_f64(t, "t", (o, o, v, v))
    pR = _dev_f64(R, "R", (o, o, v, v))
    with torch.cuda.device(R.device):
        rc = lib.cc_ladder_residual(o, v, P, pL, pt, pR, _prec(precision),
                                    _stream(R.device, stream), _opts_ref(opts))
    _check(rc, "cc_ladder_residual")
    return R


def cc_ladder_residual_noalloc(L: torch.Tensor, t: torch.Tensor, R: torch.Tensor, precision=0,
                               stream=None, opts: Optional[CcLadderOpts] = None) -> torch.Tensor:
    """cc_ladder_residual with the library's static scratch (no device allocation); returns R."""
    lib = load()
    P, v, _ = L.shape
    o = t.shape[0]
    pL = _dev_f64(L, "L", (P, v, v))
    pt = _dev_f64(t, "t", (o, o, v, v))
    pR = _dev_f64(R, "R", (o, o, v, v))
    with torch.cuda.device(R.device):
        rc = lib.cc_ladder_residual_noalloc(o, v, P, pL, pt, pR, _prec(precision),
                                            _stream(R.device, stream), _opts_ref(opts))
    _check(rc, "cc_ladder_residual_noalloc")
    return R


def cc_ladder_backward(L: torch.Tensor, t: torch.Tensor, lam: torch.Tensor, dL: torch.Tensor,
                       dt: torch.Tensor, precision=0, stream=None,
                       opts: Optional[CcLadderOpts] = None):
    """dL += dLoss/dL and dt += dLoss/dt for Loss = sum lam * R; returns (dL, dt)."""
    lib = load()
    P, v, _ = L.shape
    o = t.shape[0]
    args = (_dev_f64(L, "L", (P, v, v)), _dev_f64(t, "t", (o, o, v, v)),
            _dev_f64(lam, "lam", (o, o, v, v)), _dev_f64(dL, "dL", (P, v, v)),
            _dev_f64(dt, "dt", (o, o, v, v)))
    with torch.cuda.device(dt.device):
        rc = lib.cc_ladder_backward(o, v, P, *args, _prec(precision),
                                    _stream(dt.device, stream), _opts_ref(opts))
    _check(rc, "cc_ladder_backward")
    return dL, dt


def cc_ladder_reduce(x: torch.Tensor, y: torch.Tensor, out: Optional[torch.Tensor] = None,
                     stream=None) -> torch.Tensor:
    """out = [sum x*y, sum y*y] (device float64[2])."""
    lib = load()
    if x.dim() != 4 or x.shape[0] != x.shape[1] or x.shape[2] != x.shape[3]:
        raise ValueError("x must be [o][o][v][v]")
    o, v = x.shape[0], x.shape[2]
    px = _dev_f64(x, "x")
    py = _dev_f64(y, "y", x.shape)
    if out is None:
        out = torch.empty(2, dtype=torch.float64, device=x.device)
    pout = _dev_f64(out, "out", (2,))
    with torch.cuda.device(x.device):
        rc = lib.cc_ladder_reduce(o, v, px, py, pout, _stream(x.device, stream))
    _check(rc, "cc_ladder_reduce")
    return out


def cc_ladder_workspace_query(o: int, v: int, P: int, precision=0, backward: bool = False,
                              hbm_budget: int = 0, opts: Optional[CcLadderOpts] = None):
    """(scratch bytes, virtuals per block) the planner picks; needs no device."""
    lib = load()
    nbytes = ctypes.c_size_t(0)
    a_block = ctypes.c_int(0)
    rc = lib.cc_ladder_workspace_query(int(o), int(v), int(P), _prec(precision), int(bool(backward)),
                                       int(hbm_budget), _opts_ref(opts), ctypes.byref(nbytes),
                                       ctypes.byref(a_block))
    _check(rc, "cc_ladder_workspace_query")
    return nbytes.value, a_block.value


def cc_intermediate_ijkl(L_ov: torch.Tensor, t: torch.Tensor, X: torch.Tensor, precision=0,
                         stream=None, opts: Optional[CcLadderOpts] = None) -> torch.Tensor:
    """X[i,j,k,l] += sum_cd (sum_x L_ov[x,k,c] L_ov[x,l,d]) t[i,j,c,d]; returns X."""
    lib = load()
    P, o, v = L_ov.shape
    args = (_dev_f64(L_ov, "L_ov", (P, o, v)), _dev_f64(t, "t", (o, o, v, v)),
            _dev_f64(X, "X", (o, o, o, o)))
    with torch.cuda.device(X.device):
        rc = lib.cc_intermediate_ijkl(o, v, P, *args, _prec(precision),
                                      _stream(X.device, stream), _opts_ref(opts))
    _check(rc, "cc_intermediate_ijkl")
    return X


def cc_intermediate_ijbk(L: torch.Tensor, L_ov: torch.Tensor, t: torch.Tensor, Y: torch.Tensor,
                         precision=0, stream=None,
                         opts: Optional[CcLadderOpts] = None) -> torch.Tensor:
    """Y[i,j,b,k] += sum_cd (sum_x L[x,b,d] L_ov[x,k,c]) t[i,j,c,d]; returns Y."""
    lib = load()
    P, o, v = L_ov.shape
    args = (_dev_f64(L, "L", (P, v, v)), _dev_f64(L_ov, "L_ov", (P, o, v)),
            _dev_f64(t, "t", (o, o, v, v)), _dev_f64(Y, "Y", (o, o, v, o)))
    with torch.cuda.device(Y.device):
        rc = lib.cc_intermediate_ijbk(o, v, P, *args, _prec(precision),
                                      _stream(Y.device, stream), _opts_ref(opts))
    _check(rc, "cc_intermediate_ijbk")
    return Y


def cc_hole_ladder(L_oo: torch.Tensor, t: torch.Tensor, R: torch.Tensor, precision=0, stream=None,
                   opts: Optional[CcLadderOpts] = None) -> torch.Tensor:
    """R[i,j,a,b] += sum_kl (sum_x L_oo[x,i,k] L_oo[x,j,l]) t[k,l,a,b]; returns R."""
    lib = load()
    P, o, _ = L_oo.shape
    v = t.shape[2]
    args = (_dev_f64(L_oo, "L_oo", (P, o, o)), _dev_f64(t, "t", (o, o, v, v)),
            _dev_f64(R, "R", (o, o, v, v)))
    with torch.cuda.device(R.device):
        rc = lib.cc_hole_ladder(o, v, P, *args, _prec(precision), _stream(R.device, stream),
                                _opts_ref(opts))
    _check(rc, "cc_hole_ladder")
    return R


def cc_intermediate_workspace_query(which, o: int, v: int, P: int, precision=0,
                                    hbm_budget: int = 0, opts: Optional[CcLadderOpts] = None):
    """(scratch bytes, first indices per block) for an intermediate; needs no device."""
    lib = load()
    w = INTERMEDIATES[which] if isinstance(which, str) else int(which)
    nbytes = ctypes.c_size_t(0)
    block = ctypes.c_int(0)
    rc = lib.cc_intermediate_workspace_query(w, int(o), int(v), int(P), _prec(precision),
                                             int(hbm_budget), _opts_ref(opts), ctypes.byref(nbytes),
                                             ctypes.byref(block))
    _check(rc, "cc_intermediate_workspace_query")
    return nbytes.value, block.value


def cc_ladder_strerror(code: int) -> str:
    return strerror(code)
