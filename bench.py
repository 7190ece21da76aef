#!/usr/bin/env python3
"""Throughput of the particle-particle ladder residual on one MI355X.

A step is one pass of the forward hot path over the throughput workload
(o=40 occupied, v=360 virtual, P=1200 Cholesky vectors; synthetic MP2-like
amplitudes, see paper_2310_04559_amd/inputs.py): planning, operand
preparation, integral-block builds, amplitude contractions with float64
accumulation into R, and the float64 reductions sum t*R and |R|^2.  Inputs
are resident in HBM before timing starts.  The headline ``value`` is the
nominal 2(P+o^2)v^4 flops of a step over its time, in TFLOP/s, for the
float64 form; the float32 and split-bf16 forms are timed the same way and
reported with their error against the float64 oracle.

Also reported: the dominant kernel's roofline (HIP events recorded around its
launches through the library's trace hook), the exchange partner, the
occupied intermediates X[i,j,k,l] and Y[i,j,b,k] and the hole-hole ladder on the same workload's
vectors, the adjoint's throughput on the gradient workload (o=30, v=300,
P=900), and the oracle timed on the host's cores over a bounded sample of the
same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp64]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ladder-residual TFLOP/s at o=40,v=360,P=1200: FP64 vs FP32/split-BF16 at rel err"
# form -> (precision enum name, digit slices, pair-symmetric amplitudes asserted,
# exchange partner).  split_bf16 is the 4-slice form (13 slice products); the
# *_pairsym forms use the packed a <= b integral rows, valid because the
# workload's amplitudes are pair-symmetric (t[i,j,c,d] = t[j,i,d,c]); the
# *_exchange forms evaluate the exchange partner sum_cd (ad|bc) t[i,j,c,d]
# (eq. vfunction2) with the same nominal flops.
# The *_pm forms contract the symmetric and antisymmetric combinations t+- with
# V+- = (ac|bd) +- (ad|bc) over i <= j, a <= b, c <= d (pair-symmetric amplitudes);
# the *_symv forms gather the packed rows (*_pairsym_symv) or V+- (*_pm_symv)
# from the whole pair-pair integral of the workload's symmetric Cholesky vectors
# (built over its upper triangle; in the split forms from the packed vectors' digits).
FORMS = {"fp64": ("fp64", 0, False, False), "fp32": ("fp32", 0, False, False),
         "split_bf16": ("split_bf16", 4, False, False),
         "split_bf16_s2": ("split_bf16", 2, False, False),
         "split_bf16_s3": ("split_bf16", 3, False, False),
         "fp64_pairsym": ("fp64", 0, True, False), "fp32_pairsym": ("fp32", 0, True, False),
         "split_bf16_pairsym": ("split_bf16", 4, True, False),
         "split_bf16_pairsym_symv": ("split_bf16", 4, "sv", False),
         "fp64_pm": ("fp64", 0, "pm", False), "fp32_pm": ("fp32", 0, "pm", False),
         "fp64_pm_symv": ("fp64", 0, "pmv", False), "fp32_pm_symv": ("fp32", 0, "pmv", False),
         "fp64_pairsym_symv": ("fp64", 0, "sv", False), "fp32_pairsym_symv": ("fp32", 0, "sv", False),
         "fp64_exchange": ("fp64", 0, False, True), "fp32_exchange": ("fp32", 0, False, True),
         "split_bf16_exchange": ("split_bf16", 4, False, True),
         "split_int8": ("split_int8", 5, False, False),
         "split_int8_pairsym": ("split_int8", 5, True, False),
         "split_int8_pairsym_symv": ("split_int8", 5, "sv", False)}
_PEAK = {"fp64": 78.6, "fp32": 157.3, "split_bf16": 2500.0,
         "split_int8": 5000.0}  # dense MFMA, TFLOP/s (int8: TOP/s)
_DTYPE = {"fp64": "f64", "fp32": "f32", "split_bf16": "bf16", "split_int8": "i8"}
# Target relative Frobenius errors against the float64 oracle per arithmetic
# (every split form is held to the precision form's 1e-9), and the bound each
# slice count can reach by construction (S = 2: the per-element hi/lo split,
# about 16 significant bits per operand; S = 3: 24 bits; S = 4: 33 bits).
_TARGET = {"fp64": 1e-12, "fp32": 1e-6, "split_bf16": 1e-9, "split_int8": 1e-9}
_SPLIT_BOUND = {2: 2e-5, 3: 16 * 2.0 ** -24, 4: 1e-9, 5: 1e-9}
PEAK_TFLOPS = {f: _PEAK[p[0]] for f, p in FORMS.items()}
DTYPE = {f: _DTYPE[p[0]] for f, p in FORMS.items()}
TOL = {f: _TARGET[p[0]] for f, p in FORMS.items()}
DESIGN_BOUND = {f: (_SPLIT_BOUND[p[1]] if p[1] else _TARGET[p[0]]) for f, p in FORMS.items()}


def mfma_products(form):
    """Slice products per nominal product (executed MFMA work multiplier): the
    S(S+1)/2 triangle (hi*hi, hi*lo, lo*hi for S = 2), plus S-1 for the bf16
    4-slice form's extra anti-diagonal; the int8 form keeps the triangle."""
    s = FORMS[form][1]
    if not s:
        return 1
    if FORMS[form][0] == "split_int8":
        return s * (s + 1) // 2
    return s * (s + 1) // 2 + (s - 1 if s == 4 else 0)


def executed_flops(form, o, v, P):
    """(build, contraction) flops a form executes per forward: 2 P v^4 and
    2 o^2 v^4 in general; packed rows a <= b halve both (the build's (v+1)/(2v));
    the +- combinations contract o(o+1)/2 rows with the v(v+1)/2 pairs c <= d
    and o(o-1)/2 rows with the v(v-1)/2 pairs c < d; with symmetric vectors the
    build is the upper triangle of the pair-pair integral, P n(n+1) for
    n = v(v+1)/2 pairs."""
    v4 = float(v) ** 4
    sym = FORMS[form][2]
    if not sym:
        return 2.0 * P * v4, 2.0 * o * o * v4
    npk = v * (v + 1) / 2.0
    build = 2.0 * P * v * v * npk
    if sym in ("pmv", "sv"):
        build = P * npk * (npk + 1)  # the pair-pair integral's upper triangle
    if sym in ("pm", "pmv"):
        nm = v * (v - 1) / 2.0
        return build, 2.0 * (o * (o + 1) / 2.0 * npk * npk + o * (o - 1) / 2.0 * nm * nm)
    return build, 2.0 * o * o * v * v * npk


def executed_fraction(form, v, o=1, P=1):
    """Share of the nominal flops a form executes per forward."""
    b, c = executed_flops(form, o, v, P)
    return (b + c) / (2.0 * (P + o * o) * float(v) ** 4)
KERNEL_SRC = [os.path.join(ROOT, "paper_2310_04559_amd", "csrc", f)
              for f in ("gemm.hpp", "gemm_direct.hpp", "ccladder.hip", "split.hip", "split.hpp",
                        "split_i8.hip", "plan.cpp", "plan.h")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_src_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SRC:
        if os.path.exists(p):
            h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def read_traffic(kernel: str, form: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when it is absent or was taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_c3_{form}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.lstrip().startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_src_sha256_16") != kernel_src_hash():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def read_mfma_busy(kernel: str, form: str):
    """MFMA-busy fraction (SQ_VALU_MFMA_BUSY_CYCLES over the SIMDs' active cycles)
    of a kernel from the committed rocprofv3 summary, or None when absent or
    taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", "mfma_busy_c3.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.lstrip().startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_src_sha256_16") != kernel_src_hash():
        return None
    try:
        return float(kv[f"{kernel}_{form}"])
    except (KeyError, ValueError):
        return None


class PhaseTimer:
    """Records a HIP event pair on the call's stream around each traced phase."""

    def __init__(self, native, stream):
        import torch

        self.torch = torch
        self.stream = stream
        self.open = {}
        self.spans = []  # (phase name, block, start event, end event)
        self.fn = native.TRACE_FN(self._hook)
        self.phases = native.PHASES

    def _hook(self, user, phase, block, end, stream):
        ev = self.torch.cuda.Event(enable_timing=True)
        ev.record(self.stream)
        if not end:
            self.open[(phase, block)] = ev
        else:
            self.spans.append((self.phases[phase], block, self.open.pop((phase, block)), ev))

    def reset(self):
        self.spans = []

    def summary(self):
        out = {}
        for name, _, a, b in self.spans:
            d = out.setdefault(name, [0.0, 0])
            d[0] += a.elapsed_time(b)
            d[1] += 1
        return {k: {"ms_total": v[0], "launches": v[1], "ms_avg": v[0] / v[1]} for k, v in out.items()}


def sampled_pairs(v, n, seed):
    import numpy as np

    rng = np.random.default_rng(seed)
    pairs = {(0, 0), (v - 1, v - 1), (0, v - 1), (v - 1, 0)}
    while len(pairs) < n:
        pairs.add((int(rng.integers(0, v)), int(rng.integers(0, v))))
    return sorted(pairs)


def form_opts(native, form, **kw):
    """The library options of a form (plus workspace, trace, ... in kw)."""
    slices, sym, exchange = FORMS[form][1:]
    return native.make_opts(split_slices=slices, pair_symmetric=bool(sym), exchange=exchange,
                            plus_minus=sym in ("pm", "pmv"),
                            symmetric_vectors=sym in ("pmv", "sv"), **kw)


def bench_form(native, form, L, t, R, out, ws_bytes, steps, warmup, o, v, P):
    import torch

    prec = native.PRECISIONS[FORMS[form][0]]
    stream = torch.cuda.current_stream()
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    nbytes, n_a = native.cc_ladder_workspace_query(o, v, P, prec, hbm_budget=ws_bytes,
                                                   opts=form_opts(native, form))
    timer = PhaseTimer(native, stream)
    opts = form_opts(native, form, workspace=ws, trace=timer.fn)

    def step():
        native.cc_ladder_residual(L, t, R, prec, opts=opts)
        native.cc_ladder_reduce(t, R, out)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    timer.reset()
    # one event between consecutive steps on the call's stream: per-step times
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    w0 = time.perf_counter()
    evs[0].record(stream)
    for k in range(steps):
        step()
        evs[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = evs[0].elapsed_time(evs[-1]) / steps
    per = [evs[k].elapsed_time(evs[k + 1]) for k in range(steps)]
    phases = timer.summary()
    del ws
    return {"ms_per_step": ms, "ms_std": statistics.pstdev(per), "ms_min": min(per),
            "wall_s": wall, "a_block": n_a, "workspace_bytes": nbytes, "phases": phases}


def rel_err_form(native, form, L, t, ref, idx_a, idx_b, ws_bytes):
    import numpy as np
    import torch

    R = torch.zeros_like(t)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    native.cc_ladder_residual(L, t, R, native.PRECISIONS[FORMS[form][0]],
                              opts=form_opts(native, form, workspace=ws))
    torch.cuda.synchronize()
    got = R[:, :, idx_a, idx_b].permute(2, 0, 1).cpu().numpy()
    del R, ws
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo), or "unknown"."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(inp, target_s=15.0):
    """The oracle (NumPy/SciPy, float64 BLAS) over the first k values of its
    explicit sum over the contracted index c, k sized to roughly target_s
    seconds of host work, scaled to the whole forward."""
    import oracle

    try:
        from threadpoolctl import threadpool_info

        cores = max([d.get("num_threads", 0) for d in threadpool_info()
                     if d.get("user_api") == "blas"] or [os.cpu_count()])
    except Exception:  # threadpoolctl missing: report the visible cores
        cores = os.cpu_count()
    o, v, P = inp.o, inp.v, inp.P
    t0 = time.perf_counter()
    R = oracle.ladder_forward(inp.L_vv, inp.t, c_begin=0, c_end=1)
    one = time.perf_counter() - t0
    k = int(max(1, min(v - 1, target_s / max(one, 1e-3))))
    t0 = time.perf_counter()
    oracle.ladder_forward(inp.L_vv, inp.t, R=R, c_begin=1, c_end=1 + k)
    dt = time.perf_counter() - t0
    flops = 2.0 * (P + o * o) * float(v) ** 3 * k
    return {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": int(cores), "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"oracle forward over c in [1,{1 + k}) of the o={o},v={v},P={P} workload "
                      f"({k}/{v} of its flops, {dt:.1f} s)"}


def adjoint_executed_flops(o, v, P, sym, symv, n_a):
    """Flops the adjoint executes: build 2 P v^4, dt and W 2 o^2 v^4 each, and the
    two dL terms 2 P v^4 each, or one product of 2 P v^4 when one block holds
    all of W (its symmetric part gives both terms).  Pair-symmetric: every
    product over the packed pairs, n = v(v+1)/2 rows instead of v^2 (the dL
    terms over the half-written W, K ranges b >= a); with symmetric vectors the
    build is the pair-pair integral's upper triangle, P n(n+1)."""
    v4 = float(v) ** 4
    if not sym:
        dl = 2.0 if n_a == v else 4.0
        return (2.0 * P + 4.0 * o * o + dl * P) * v4
    n = v * (v + 1) / 2.0
    build = P * n * (n + 1) if symv else 2.0 * P * v * v * n
    return build + (4.0 * o * o + 4.0 * P) * v * v * n


def bench_adjoint(native, steps, forms=("fp64", "fp32", "fp64_pairsym", "fp32_pairsym",
                                        "fp64_pairsym_symv", "fp32_pairsym_symv")):
    """The adjoint on the gradient workload (o=30, v=300, P=900); its lam and t
    are pair-symmetric, so the *_pairsym forms (the half-written W block) apply
    and report effective TFLOP/s on the same nominal count; its vectors are
    symmetric, so the *_symv forms gather the packed rows from the pair-pair
    integral."""
    import numpy as np
    import torch

    from paper_2310_04559_amd.inputs import CONFIGS, make_inputs, seed_for

    o, v, P = CONFIGS["o30_v300_P900"]
    inp = make_inputs(o, v, P, seed_for("o30_v300_P900"), with_lambda=True, device="cuda")
    L = torch.from_numpy(inp.L_vv).cuda()
    t = torch.from_numpy(inp.t).cuda()
    lam = torch.from_numpy(inp.lam).cuda()
    del inp
    flops = (6.0 * P + 4.0 * o * o) * float(v) ** 4
    res = {"workload": f"o={o},v={v},P={P}", "nominal_tflop": flops / 1e12}
    ref = None
    stream = torch.cuda.current_stream()
    free, _ = torch.cuda.mem_get_info()
    budget = int(min(free // 2, 128 << 30))
    for form in forms:
        prec = native.PRECISIONS[form.split("_")[0]]
        sym = "_pairsym" in form
        symv = form.endswith("_symv")
        timer = PhaseTimer(native, stream)
        # the caller's workspace, allocated once outside the timed calls
        nbytes, n_a = native.cc_ladder_workspace_query(
            o, v, P, prec, backward=True, hbm_budget=budget,
            opts=native.make_opts(pair_symmetric=sym, symmetric_vectors=symv))
        ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        opts = native.make_opts(trace=timer.fn, pair_symmetric=sym, symmetric_vectors=symv,
                                workspace=ws)
        dL = torch.zeros_like(L)
        dt = torch.zeros_like(t)
        native.cc_ladder_backward(L, t, lam, dL, dt, prec, opts=opts)  # warm-up, also the result
        torch.cuda.synchronize()
        if ref is None:
            ref = (dL.clone(), dt.clone())
            err = None
        else:
            err = max(float(torch.linalg.vector_norm(dL - ref[0]) / torch.linalg.vector_norm(ref[0])),
                      float(torch.linalg.vector_norm(dt - ref[1]) / torch.linalg.vector_norm(ref[1])))
        timer.reset()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            native.cc_ladder_backward(L, t, lam, dL, dt, prec, opts=opts)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        executed = adjoint_executed_flops(o, v, P, sym, symv, n_a)
        res[form] = {"ms_per_step": ms, "tflops": flops / (ms * 1e-3) / 1e12,
                     "tflops_executed": executed / (ms * 1e-3) / 1e12, "a_block": n_a,
                     "rel_err_vs_fp64_gpu": err,
                     "phases_ms_per_step": {k: d["ms_total"] / steps for k, d in timer.summary().items()}}
        log(f"adjoint {form}: {ms:.1f} ms {res[form]['tflops']:.1f} TFLOP/s "
            f"({res[form]['tflops_executed']:.1f} executed) "
            f"phases {json.dumps(res[form]['phases_ms_per_step'])}")
        del ws, opts, timer
        del dL, dt
    return res


def bench_large(native, forms=("fp64", "split_int8", "split_bf16"), budget_names=("default", "device"),
                adjoint=True):
    """The large single-GPU workload (o=60, v=600, P=1800) under two scratch
    budgets, each a caller workspace allocated once: the default (half the free
    memory, at most 128 GiB, as the library plans by default) and one sized to the device (the free memory left
    with every array of the call resident, less 8 GiB).  Per budget and form: a
    warm-up call, then one timed call (HIP events on the call's stream) with
    per-phase times; the float32 adjoint is timed the same way.  Errors: the
    forwards against the oracle on sampled (a,b) columns."""
    import numpy as np
    import torch

    import oracle
    from paper_2310_04559_amd.inputs import CONFIGS, make_inputs, seed_for

    o, v, P = CONFIGS["o60_v600_P1800"]
    inp = make_inputs(o, v, P, seed_for("o60_v600_P1800"), with_lambda=True, device="cuda")
    pairs = sampled_pairs(v, 8, 5)
    ref = oracle.ladder_pairs(inp.L_vv, inp.t, pairs)
    L = torch.from_numpy(inp.L_vv).cuda()
    t = torch.from_numpy(inp.t).cuda()
    lam = torch.from_numpy(inp.lam).cuda()
    del inp
    ia = torch.tensor([a for a, _ in pairs], device="cuda")
    ib = torch.tensor([b for _, b in pairs], device="cuda")
    fwd = 2.0 * (P + o * o) * float(v) ** 4
    bwd = (6.0 * P + 4.0 * o * o) * float(v) ** 4
    res = {"workload": f"o={o},v={v},P={P}", "nominal_tflop_forward": fwd / 1e12,
           "nominal_tflop_adjoint": bwd / 1e12}
    stream = torch.cuda.current_stream()
    R = torch.zeros_like(t)
    torch.cuda.empty_cache()
    free, total = torch.cuda.mem_get_info()
    # the adjoint's dL and dt are allocated later: keep their room out of the large budget
    extra = t.numel() * 8 + L.numel() * 8
    budgets = {"default": int(min(free // 2, 128 << 30)),
               "device": int(free - extra - (8 << 30))}
    res["device_total_bytes"] = int(total)
    res["budgets_bytes"] = budgets

    def timed(call, timer, after_warmup=None):
        call()  # warm-up (also plans nothing new: the workspace is the caller's)
        torch.cuda.synchronize()
        if after_warmup is not None:
            after_warmup()
        timer.reset()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        call()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    for bname, budget in budgets.items():
        if bname not in budget_names:
            continue
        for form in forms:
            prec, slices = native.PRECISIONS[FORMS[form][0]], FORMS[form][1]
            nbytes, n_a = native.cc_ladder_workspace_query(
                o, v, P, prec, hbm_budget=budget, opts=native.make_opts(split_slices=slices))
            ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
            timer = PhaseTimer(native, stream)
            opts = native.make_opts(workspace=ws, trace=timer.fn, split_slices=slices)
            R.zero_()
            got = []

            def check():
                # the warm-up call's R (one forward onto zeros), then zeros again
                got.append(R[:, :, ia, ib].permute(2, 0, 1).cpu().numpy())
                R.zero_()
                torch.cuda.synchronize()

            ms = timed(lambda: native.cc_ladder_residual(L, t, R, prec, opts=opts), timer, check)
            got = got[0]
            phases = {k: d["ms_total"] for k, d in timer.summary().items()}
            # release the workspace (the options hold a reference) before the next plan
            del ws, opts, timer
            torch.cuda.empty_cache()
            r = {"ms": ms, "tflops": fwd / (ms * 1e-3) / 1e12, "a_block": n_a,
                 "workspace_bytes": nbytes,
                 "rel_err_vs_oracle_sampled": float(np.linalg.norm(got - ref) / np.linalg.norm(ref)),
                 "phases_ms": phases}
            res[f"{form}_{bname}"] = r
            log(f"large {form} budget {bname} ({budget / 2**30:.0f} GiB, a_block {n_a}): "
                f"{ms:.0f} ms {r['tflops']:.1f} TFLOP/s phases {json.dumps(r['phases_ms'])}")
    del R
    torch.cuda.empty_cache()
    if not adjoint:
        return res
    dL = torch.zeros_like(L)
    dt = torch.zeros_like(t)
    nbytes, n_a = native.cc_ladder_workspace_query(o, v, P, native.CC_LADDER_FP32, backward=True,
                                                   hbm_budget=budgets["device"])
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    timer = PhaseTimer(native, stream)
    opts = native.make_opts(workspace=ws, trace=timer.fn)
    ms = timed(lambda: native.cc_ladder_backward(L, t, lam, dL, dt, native.CC_LADDER_FP32,
                                                 opts=opts), timer)
    res["adjoint_fp32_device"] = {"ms": ms, "tflops": bwd / (ms * 1e-3) / 1e12, "a_block": n_a,
                                  "phases_ms": {k: d["ms_total"] for k, d in timer.summary().items()}}
    log(f"large adjoint fp32 (a_block {n_a}): {ms:.0f} ms "
        f"{res['adjoint_fp32_device']['tflops']:.1f} TFLOP/s")
    return res


def bench_intermediates(native, inp, steps, warmup, ws_bytes):
    """The occupied intermediates (eqs. vfunction3/vfunction4) and the
    hole-hole ladder on the throughput workload's own L_ov, L_oo, L_vv and t:
    time per call with HIP events on the call's stream, nominal TFLOP/s, and
    the error of sampled first-index slices against the oracle."""
    import numpy as np
    import torch

    import oracle

    o, v, P = inp.o, inp.v, inp.P
    Ld = torch.from_numpy(inp.L_vv).cuda()
    Lovd = torch.from_numpy(inp.L_ov).cuda()
    Lood = torch.from_numpy(inp.L_oo).cuda()
    td = torch.from_numpy(inp.t).cuda()
    stream = torch.cuda.current_stream()
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    res = {}
    shapes = {"ijkl": (o, o, o, o), "ijbk": (o, o, v, o), "hole": (o, o, v, v)}
    for which in ("ijkl", "ijbk", "hole"):
        shape = shapes[which]
        # sampled first indices: X[:, :, k, :], Y[:, :, b, :]; rows R[i] of the hole ladder
        firsts = [0, v // 2, v - 1] if which == "ijbk" else [0, o - 1]
        ref = np.zeros(shape)
        for p in firsts:
            if which == "ijkl":
                oracle.intermediate_ijkl(inp.L_ov, inp.t, ref, p, p + 1)
            elif which == "ijbk":
                oracle.intermediate_ijbk(inp.L_vv, inp.L_ov, inp.t, ref, p, p + 1)
            else:
                oracle.hole_ladder(inp.L_oo, inp.t, ref, p, p + 1)
        pick = (lambda a: a[firsts]) if which == "hole" else (lambda a: a[:, :, firsts, :])
        flops = {"ijkl": oracle.nominal_flops_ijkl, "ijbk": oracle.nominal_flops_ijbk,
                 "hole": oracle.nominal_flops_hole}[which](o, v, P)
        Z = torch.zeros(shape, dtype=torch.float64, device="cuda")
        for prec_name in ("fp64", "fp32"):
            prec = native.PRECISIONS[prec_name]
            timer = PhaseTimer(native, stream)
            opts = native.make_opts(workspace=ws, trace=timer.fn)
            _, block = native.cc_intermediate_workspace_query(which, o, v, P, prec, hbm_budget=ws_bytes)

            def call():
                if which == "ijkl":
                    native.cc_intermediate_ijkl(Lovd, td, Z, prec, opts=opts)
                elif which == "ijbk":
                    native.cc_intermediate_ijbk(Ld, Lovd, td, Z, prec, opts=opts)
                else:
                    native.cc_hole_ladder(Lood, td, Z, prec, opts=opts)

            Z.zero_()
            call()
            torch.cuda.synchronize()
            got = pick(Z.cpu().numpy())
            err = float(np.linalg.norm(got - pick(ref)) / np.linalg.norm(pick(ref)))
            for _ in range(warmup):
                call()
            torch.cuda.synchronize()
            timer.reset()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(steps):
                call()
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            r = {"ms_per_call": ms, "tflops": flops / (ms * 1e-3) / 1e12, "block": block,
                 "nominal_tflop": flops / 1e12, "rel_err_vs_oracle_sampled": err,
                 "within_tolerance": err < TOL[prec_name],
                 "phases_ms_avg": {k: d["ms_avg"] for k, d in timer.summary().items()}}
            res[f"{which}_{prec_name}"] = r
            log(f"intermediate {which} {prec_name}: {ms:.2f} ms {r['tflops']:.1f} TFLOP/s "
                f"err {err:.2e} block {block} phases {json.dumps(r['phases_ms_avg'])}")
        del Z
    del ws, Ld, Lovd, Lood, td
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp64", choices=list(FORMS))
    ap.add_argument("--forms", default="fp64,fp32,split_bf16,split_int8,split_bf16_s2,fp64_pairsym,"
                                       "fp64_pairsym_symv,fp64_pm,fp32_pm,fp64_pm_symv,fp32_pm_symv,"
                                       "split_bf16_pairsym,split_bf16_pairsym_symv,"
                                       "split_int8_pairsym,split_int8_pairsym_symv,fp64_exchange")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--budget-gib", type=float, default=128.0,
                    help="scratch budget of the timed forms: at most this many GiB, and at most "
                         "half the free device memory")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-intermediates", action="store_true")
    ap.add_argument("--large", action="store_true",
                    help="also run the o=60, v=600, P=1800 workload (about five minutes)")
    ap.add_argument("--only-large", action="store_true",
                    help="run only the o=60, v=600, P=1800 workload and print its JSON")
    ap.add_argument("--large-forms", default="fp64,split_int8,split_bf16",
                    help="forms of the large workload")
    ap.add_argument("--large-budgets", default="default,device",
                    help="scratch budgets of the large workload: default and/or device")
    ap.add_argument("--no-large-adjoint", action="store_true")
    ap.add_argument("--only-adjoint", action="store_true",
                    help="run only the adjoint on the o=30, v=300, P=900 workload and print its JSON")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run one plain device copy of this many MiB (a known-size "
                         "reference for HBM byte counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        msg = ("bench.py measures one GPU only: the ladder library runs on a single MI355X and "
               "the library has no multi-GPU path (--gpus must be 1).")
        print(json.dumps({"error": msg, "n_gpus": args.gpus}), flush=True)
        log(msg)
        sys.exit(2)

    import numpy as np
    import torch

    import oracle
    from paper_2310_04559_amd import native
    from paper_2310_04559_amd.inputs import CONFIGS, make_inputs, seed_for

    native.load()
    if not torch.cuda.is_available():
        log("no GPU visible")
        sys.exit(1)
    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {args.copy_calibration_mib} MiB read + written")
        del src, dst
    if args.only_large:
        print(json.dumps({"large": bench_large(native, tuple(args.large_forms.split(",")),
                                               tuple(args.large_budgets.split(",")),
                                               not args.no_large_adjoint)}), flush=True)
        return
    if args.only_adjoint:
        print(json.dumps({"adjoint": bench_adjoint(native, max(1, min(args.steps, 2)))}), flush=True)
        return
    o, v, P = CONFIGS["o40_v360_P1200"]
    t0 = time.perf_counter()
    inp = make_inputs(o, v, P, seed_for("o40_v360_P1200"), device="cuda")
    log(f"inputs o={o} v={v} P={P} drawn in {time.perf_counter() - t0:.1f} s")
    L = torch.from_numpy(inp.L_vv).cuda()
    t = torch.from_numpy(inp.t).cuda()
    R = torch.zeros_like(t)
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    free, _ = torch.cuda.mem_get_info()
    ws_bytes = int(min(free // 2, args.budget_gib * (1 << 30)))
    flops = 2.0 * (P + o * o) * float(v) ** 4

    pairs = sampled_pairs(v, 24, 3)
    ref = oracle.ladder_pairs(inp.L_vv, inp.t, pairs)
    # exchange partner: the ladder of the amplitudes with c and d swapped
    ref_x = oracle.ladder_pairs(inp.L_vv, np.ascontiguousarray(inp.t.transpose(0, 1, 3, 2)), pairs)
    idx_a = torch.tensor([a for a, _ in pairs], device="cuda")
    idx_b = torch.tensor([b for _, b in pairs], device="cuda")

    forms = {}
    for form in [f for f in args.forms.split(",") if f]:
        try:
            err = rel_err_form(native, form, L, t, ref_x if FORMS[form][3] else ref, idx_a, idx_b,
                               ws_bytes)
        except native.LadderError as e:
            forms[form] = {"status": "unsupported", "detail": str(e)}
            log(f"{form}: {e}")
            continue
        r = bench_form(native, form, L, t, R, out, ws_bytes, args.steps, args.warmup, o, v, P)
        r["tflops"] = flops / (r["ms_per_step"] * 1e-3) / 1e12
        r["executed_tflops"] = r["tflops"] * executed_fraction(form, v, o, P)
        r["rel_err_vs_oracle"] = err
        r["tolerance"] = TOL[form]
        r["within_tolerance"] = err < TOL[form]
        r["design_bound"] = DESIGN_BOUND[form]
        n_a = r["a_block"]
        # dominant kernel: the amplitude contraction, 2 o^2 (n_a v) v^2 flops per full-block launch
        c = r["phases"].get("contract")
        if c:
            per_step = c["launches"] / args.steps  # launches of the kernel in one step
            launch_flops = executed_flops(form, o, v, P)[1] / per_step
            # executed MFMA flops: the split forms run S(S+1)/2 slice products per product
            achieved = mfma_products(form) * launch_flops / (c["ms_avg"] * 1e-3) / 1e12
            r["roofline"] = {"kernel": "contract", "bound": "mfma", "achieved": achieved,
                             "peak": PEAK_TFLOPS[form],
                             "unit": "TOP/s" if FORMS[form][0] == "split_int8" else "TFLOP/s",
                             "frac": achieved / PEAK_TFLOPS[form],
                             "traffic": read_traffic("contract", form),
                             "mfma_busy_counter": read_mfma_busy("contract", form),
                             "flops_per_launch": mfma_products(form) * launch_flops,
                             "nominal_tflops": launch_flops / (c["ms_avg"] * 1e-3) / 1e12}
        b = r["phases"].get("build")
        if b:
            bflops = executed_flops(form, o, v, P)[0] / (b["launches"] / args.steps)
            r["build_tflops"] = bflops / (b["ms_avg"] * 1e-3) / 1e12
        forms[form] = r
        log(f"{form}: {r['ms_per_step']:.1f} +- {r['ms_std']:.1f} (min {r['ms_min']:.1f}) ms/step "
            f"{r['tflops']:.2f} TFLOP/s err {err:.2e} "
            f"a_block {n_a} phases {json.dumps(r['phases'])}")
        R.zero_()

    head = forms.get(args.precision)
    if not head or "ms_per_step" not in head:
        log(f"headline form {args.precision} did not run")
        sys.exit(1)
    line = {
        "metric": METRIC,
        "value": head["tflops"],
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "ms_per_step_std": head["ms_std"],
        "ms_per_step_min": head["ms_min"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.precision],
        "data": "synthetic",
        "config": {"workload": "ladder residual o=40 v=360 P=1200 (MP2-like amplitudes)",
                   "o": o, "v": v, "P": P, "a_block": head["a_block"],
                   "nominal_tflop_per_step": flops / 1e12, "precision": args.precision},
        "roofline": head.get("roofline"),
        "rel_err_vs_oracle": head["rel_err_vs_oracle"],
        "forms": {k: {kk: vv for kk, vv in f.items() if kk != "phases"} | (
            {"phases_ms_avg": {p: d["ms_avg"] for p, d in f["phases"].items()}} if "phases" in f else {})
                  for k, f in forms.items()},
    }
    del L, t, R
    torch.cuda.empty_cache()
    if not args.no_intermediates:
        log("intermediates ...")
        line["intermediates"] = bench_intermediates(native, inp, args.steps, args.warmup, ws_bytes)
        torch.cuda.empty_cache()
    if not args.no_adjoint:
        log("adjoint ...")
        line["adjoint"] = bench_adjoint(native, max(1, min(args.steps, 2)))
    if args.large:
        log("large workload ...")
        line["large"] = bench_large(native)
    if not args.no_cpu_baseline:
        log("cpu baseline ...")
        line["cpu_baseline"] = cpu_baseline(inp)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
