"""Host-side checks of the C ABI: the library loads, exports what the header
declares, plans blocks and rejects bad arguments without touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ccladder.h")


@pytest.fixture(scope="module")
def native():
    from paper_2310_04559_amd import native as nat

    nat.load()
    return nat


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cc_(?:ladder|intermediate|hole)_\w+)\s*\(", text)))


def test_exports_every_declared_symbol(native):
    names = declared_functions()
    assert set(names) == set(native.EXPORTS)
    lib = native.load()
    for n in names:
        assert hasattr(lib, n), n


def test_opts_struct_layout(native):
    # int a_block, split_slices, k_chunk, split_depth; size_t budget; void* ws; size_t ws_bytes;
    # trace hook and its user pointer; unsigned flags, int reserved
    assert ctypes.sizeof(native.CcLadderOpts) == 4 * 4 + 8 * 5 + 8


def test_strerror(native):
    for code in (0, -1, -2, -3, -4, -5):
        assert native.cc_ladder_strerror(code)
    assert "unknown" in native.cc_ladder_strerror(7)


def test_planner_whole_range_without_budget(native):
    nbytes, n_a = native.cc_ladder_workspace_query(40, 360, 1200, "fp64")
    assert n_a == 360
    assert nbytes == 360 ** 4 * 8  # one float64 integral block of all virtuals


def test_planner_shrinks_to_budget(native):
    per_a = 360 ** 3 * 8
    nbytes, n_a = native.cc_ladder_workspace_query(40, 360, 1200, "fp64", hbm_budget=32 * per_a)
    assert nbytes <= 32 * per_a
    # equalised blocks: ceil(360/32) = 12 blocks of 30
    assert n_a == 30
    nbytes, n_a = native.cc_ladder_workspace_query(20, 180, 600, "fp64", hbm_budget=32 * 180 ** 3 * 8)
    assert n_a == 30  # 6 blocks of 30 rather than 5x32 + 20


def test_planner_backward_and_fp32_footprints(native):
    v, o, P = 30, 4, 50
    b64, n = native.cc_ladder_workspace_query(o, v, P, "fp64", backward=True)
    assert n == v and b64 >= 2 * v ** 4 * 8
    b32, n = native.cc_ladder_workspace_query(o, v, P, "fp32")
    assert n == v and b32 >= (P * v * v + o * o * v * v + v ** 4) * 4


def test_planner_split_footprint(native):
    # digit buffers: S slices of L (rows v^2, K = P padded to 64), of t and of
    # one integral block, plus the float64 block itself
    o, v, P = 4, 30, 50
    b4, n = native.cc_ladder_workspace_query(o, v, P, "split_bf16")
    b2, _ = native.cc_ladder_workspace_query(o, v, P, "split_bf16", opts=native.make_opts(split_slices=2))
    assert n == v and b4 > b2 >= v ** 4 * 8
    with pytest.raises(native.LadderError) as e:
        native.cc_ladder_workspace_query(o, v, P, "split_bf16", backward=True)
    assert e.value.code == native.CC_LADDER_EUNSUPPORTED


def test_planner_pair_symmetric_footprint(native):
    # packed rows a <= b: v(v+1)/2 integral rows instead of v^2 for one block
    o, v, P = 4, 30, 50
    full, n = native.cc_ladder_workspace_query(o, v, P, "fp64")
    half, n2 = native.cc_ladder_workspace_query(o, v, P, "fp64", opts=native.make_opts(pair_symmetric=True))
    assert n == n2 == v
    rnd = lambda b: (b + 255) // 256 * 256  # buffers are 256-byte aligned
    tiles_m = (v * v + 127) // 128             # plus the compact build grid's row table
    assert half == rnd((v * (v + 1) // 2) * v * v * 8) + rnd((tiles_m + 1) * 4)
    assert full == rnd(v ** 4 * 8)
    # the split form: packed float64 block and packed digit rows, row table of
    # its 64-row tiles
    sfull, _ = native.cc_ladder_workspace_query(o, v, P, "split_bf16")
    shalf, n3 = native.cc_ladder_workspace_query(o, v, P, "split_bf16",
                                                 opts=native.make_opts(pair_symmetric=True))
    assert n3 == v and shalf < sfull
    rows_pad = lambda r: (r + 127) // 128 * 128 + 128
    kp, npk = (v * v + 63) // 64 * 64, v * (v + 1) // 2
    chunks = (kp + 255) // 256  # one exponent per 256 contracted indices with four slices
    packed = (rnd(npk * v * v * 8) + rnd(4 * rows_pad(npk) * kp * 2) + rnd(rows_pad(npk) * chunks * 4)
              + rnd(((v * v + 63) // 64 + 1) * 4))
    dense = rnd(v ** 4 * 8) + rnd(4 * rows_pad(v * v) * kp * 2) + rnd(rows_pad(v * v) * chunks * 4)
    assert sfull - shalf == dense - packed


def test_planner_exchange_footprint(native):
    # the swapped amplitudes (float64; the float32 form swaps into its own copy)
    # and, for the adjoint, dt in swapped order
    o, v, P = 4, 30, 50
    rnd = lambda b: (b + 255) // 256 * 256
    t64 = rnd(o * o * v * v * 8)
    ex = native.make_opts(exchange=True)
    for prec, bwd, extra in (("fp64", False, t64), ("fp64", True, 2 * t64), ("fp32", False, 0),
                             ("fp32", True, t64), ("split_bf16", False, t64)):
        plain, n = native.cc_ladder_workspace_query(o, v, P, prec, backward=bwd)
        swapped, n2 = native.cc_ladder_workspace_query(o, v, P, prec, backward=bwd, opts=ex)
        assert n == n2 == v and swapped == plain + extra, (prec, bwd)
    both = native.make_opts(exchange=True, pair_symmetric=True)
    ps, _ = native.cc_ladder_workspace_query(o, v, P, "fp64", opts=native.make_opts(pair_symmetric=True))
    assert native.cc_ladder_workspace_query(o, v, P, "fp64", opts=both)[0] == ps + t64


def test_planner_intermediate_footprints(native):
    # integral block [n_p][o][v][v] over first indices p (occupied k for ijkl,
    # virtual b for ijbk); ijbk also holds the swapped amplitudes (float64)
    o, v, P = 4, 30, 50
    rnd = lambda b: (b + 255) // 256 * 256
    b, n = native.cc_intermediate_workspace_query("ijkl", o, v, P, "fp64")
    assert n == o and b == rnd(o * o * v * v * 8)
    b, n = native.cc_intermediate_workspace_query("ijbk", o, v, P, "fp64")
    assert n == v and b == rnd(o * o * v * v * 8) + rnd(v * o * v * v * 8)
    b, n = native.cc_intermediate_workspace_query("ijkl", o, v, P, "fp32")
    assert n == o and b == rnd(P * o * v * 4) + rnd(o * o * v * v * 4) + rnd(o * o * v * v * 4)
    b, n = native.cc_intermediate_workspace_query("ijbk", o, v, P, "fp32")
    assert n == v and b == (rnd(P * o * v * 4) + rnd(P * v * v * 4) + rnd(o * o * v * v * 4)
                            + rnd(v * o * v * v * 4))
    # budget: 7 virtuals' blocks fit, equalised to ceil(30 / ceil(30/7)) = 6
    per_b = o * v * v * 8
    b, n = native.cc_intermediate_workspace_query("ijbk", o, v, P, "fp64",
                                                   hbm_budget=rnd(o * o * v * v * 8) + 7 * per_b)
    assert n == 6
    b, n = native.cc_intermediate_workspace_query("ijkl", o, v, P, "fp64", opts=native.make_opts(a_block=3))
    assert n == 3 and b == rnd(3 * o * v * v * 8)
    for kw, prec in ((dict(), "split_bf16"), (dict(exchange=True), "fp64"),
                     (dict(pair_symmetric=True), "fp32")):
        with pytest.raises(native.LadderError) as e:
            native.cc_intermediate_workspace_query("ijkl", o, v, P, prec, opts=native.make_opts(**kw))
        assert e.value.code == native.CC_LADDER_EUNSUPPORTED
    with pytest.raises(native.LadderError) as e:
        native.cc_intermediate_workspace_query(3, o, v, P, "fp64")
    assert e.value.code == native.CC_LADDER_EINVAL


def _waves_per_work(tiles, s, cus=256):
    return -(-tiles * s // cus) / s


@pytest.mark.parametrize("o,v,P,which,prec", [(40, 360, 1200, "ijkl", "fp64"),
                                              (20, 180, 600, "ijkl", "fp32"),
                                              (16, 64, 200, "ijbk", "fp64"),
                                              (40, 360, 1200, "ijbk", "fp64")])
def test_planner_intermediate_split_partials(native, o, v, P, which, prec):
    # the contraction's 128 x 256 tile grid over o^2 x (n_first*o); when it alone
    # leaves the 256 compute units idle, K = v^2 is cut into S ranges (at least
    # 64 K-steps each) that minimise waves per unit of work, with float64
    # partials [S][o^2][n_p*o] in scratch
    rnd = lambda b: (b + 255) // 256 * 256
    n_first = o if which == "ijkl" else v
    tiles = -(-o * o // 128) * -(-n_first * o // 256)
    nk = -(-v * v // (16 if prec == "fp64" else 32))
    S, best = 1, 1.0
    if tiles < 256:
        for s in range(2, 17):
            if nk // s < 64:
                break
            if _waves_per_work(tiles, s) < best * 0.999:
                S, best = s, _waves_per_work(tiles, s)
    b, n = native.cc_intermediate_workspace_query(which, o, v, P, prec)
    base, _ = native.cc_intermediate_workspace_query(which, o, v, P, prec,
                                                      opts=native.make_opts(a_block=n))
    assert b == base
    esz = 8 if prec == "fp64" else 4
    ops = (rnd(P * o * v * 4) + (rnd(P * v * v * 4) if which == "ijbk" else 0) + rnd(o * o * v * v * 4)
           if prec == "fp32" else (rnd(o * o * v * v * 8) if which == "ijbk" else 0))
    part = rnd(S * o * o * n * o * 8) if S > 1 else 0
    assert b == ops + rnd(n * o * v * v * esz) + part
    if (o, v, which) == (40, 360, "ijkl"):
        assert S == 14  # 91 tiles: 14 ranges give 1274 workgroups in 5 waves


def test_planner_hole_ladder_footprint(native):
    # (ik|jl) for a block of occupied i: [n_p][o][o][o]; the float32 form adds
    # its copies of L_oo and t
    o, v, P = 6, 30, 50
    rnd = lambda b: (b + 255) // 256 * 256
    b, n = native.cc_intermediate_workspace_query("hole", o, v, P, "fp64")
    assert n == o and b == rnd(o ** 4 * 8)
    b, n = native.cc_intermediate_workspace_query("hole", o, v, P, "fp32")
    assert n == o and b == rnd(P * o * o * 4) + rnd(o * o * v * v * 4) + rnd(o ** 4 * 4)
    b, n = native.cc_intermediate_workspace_query("hole", o, v, P, "fp64", hbm_budget=rnd(2 * o ** 3 * 8))
    assert n == 2 and b == rnd(2 * o ** 3 * 8)


def test_planner_explicit_block_and_enomem(native):
    opts = native.make_opts(a_block=7)
    nbytes, n_a = native.cc_ladder_workspace_query(5, 20, 75, "fp64", opts=opts)
    assert n_a == 7 and nbytes >= 7 * 20 ** 3 * 8
    with pytest.raises(native.LadderError) as e:
        native.cc_ladder_workspace_query(5, 20, 75, "fp64", hbm_budget=1000)
    assert e.value.code == native.CC_LADDER_ENOMEM
    with pytest.raises(native.LadderError) as e:
        native.cc_ladder_workspace_query(5, 20, 75, "fp64", hbm_budget=3 * 20 ** 3 * 8, opts=opts)
    assert e.value.code == native.CC_LADDER_ENOMEM


@pytest.mark.parametrize("o,v,P,prec", [(0, 4, 4, 0), (2, 0, 4, 0), (2, 4, -1, 0), (2, 4, 4, 4),
                                        (2, 4, 4, -1), (50000, 4, 4, 0)])
def test_planner_rejects_bad_arguments(native, o, v, P, prec):
    with pytest.raises(native.LadderError) as e:
        native.cc_ladder_workspace_query(o, v, P, prec)
    assert e.value.code == native.CC_LADDER_EINVAL


def test_bad_options_rejected(native):
    for kw in (dict(split_slices=1), dict(split_slices=5), dict(k_chunk=100), dict(a_block=-2),
               dict(split_depth=3), dict(split_depth=-1)):
        with pytest.raises(native.LadderError) as e:
            native.cc_ladder_workspace_query(3, 8, 10, "fp32", opts=native.make_opts(**kw))
        assert e.value.code == native.CC_LADDER_EINVAL
    for flags, reserved in ((8, 0), (1 << 31, 0), (0, 1)):
        o = native.make_opts()
        o.flags, o.reserved = flags, reserved
        with pytest.raises(native.LadderError) as e:
            native.cc_ladder_workspace_query(3, 8, 10, "fp64", opts=o)
        assert e.value.code == native.CC_LADDER_EINVAL


def test_argument_checks_precede_device_checks(native):
    lib = native.load()
    # null pointers and aliasing are rejected on the host, device or not
    assert lib.cc_ladder_residual(2, 4, 2, None, None, None, 0, None, None) == native.CC_LADDER_EINVAL
    R = 1 << 20
    assert lib.cc_ladder_residual(2, 4, 2, 1 << 24, R + 8, R, 0, None, None) == native.CC_LADDER_EINVAL
    assert lib.cc_ladder_backward(2, 4, 2, 1 << 24, 1 << 26, 1 << 28, 1 << 30, 1 << 30, 0, None,
                                  None) == native.CC_LADDER_EINVAL
    assert lib.cc_ladder_reduce(2, 4, None, 1 << 20, 1 << 24, None) == native.CC_LADDER_EINVAL


def test_intermediate_argument_checks_precede_device_checks(native):
    lib = native.load()
    # null pointers and an output overlapping an input are host-side errors
    assert lib.cc_intermediate_ijkl(2, 4, 2, None, 1 << 24, 1 << 26, 0, None, None) == native.CC_LADDER_EINVAL
    t = 1 << 24
    assert lib.cc_intermediate_ijkl(2, 4, 2, 1 << 28, t, t + 64, 0, None, None) == native.CC_LADDER_EINVAL
    assert lib.cc_intermediate_ijbk(2, 4, 2, 1 << 28, 1 << 30, t, t - 8, 0, None,
                                    None) == native.CC_LADDER_EINVAL
    assert lib.cc_intermediate_ijbk(0, 4, 2, 1 << 28, 1 << 30, t, 1 << 32, 0, None,
                                    None) == native.CC_LADDER_EINVAL
    assert lib.cc_hole_ladder(2, 4, 2, 1 << 28, t, t + 128, 0, None, None) == native.CC_LADDER_EINVAL
    assert lib.cc_hole_ladder(2, 4, 2, None, t, 1 << 30, 0, None, None) == native.CC_LADDER_EINVAL


def test_no_device_is_reported(native):
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    lib = native.load()
    rc = lib.cc_ladder_residual(2, 4, 2, 1 << 24, 1 << 26, 1 << 28, 0, None, None)
    assert rc == native.CC_LADDER_ENODEV
    assert lib.cc_ladder_reduce(2, 4, 1 << 24, 1 << 26, 1 << 28, None) == native.CC_LADDER_ENODEV
    assert lib.cc_intermediate_ijkl(2, 4, 2, 1 << 24, 1 << 26, 1 << 28, 0, None,
                                    None) == native.CC_LADDER_ENODEV
    assert lib.cc_intermediate_ijbk(2, 4, 2, 1 << 24, 1 << 26, 1 << 28, 1 << 30, 1, None,
                                    None) == native.CC_LADDER_ENODEV
    assert lib.cc_hole_ladder(2, 4, 2, 1 << 24, 1 << 26, 1 << 28, 0, None, None) == native.CC_LADDER_ENODEV


def test_symmetry_check_flag_plan(native):
    # the check needs one 256-byte slot, and only with the pair-symmetric flag
    for backward in (False, True):
        base, _ = native.cc_ladder_workspace_query(
            3, 20, 30, "fp64", backward=backward, opts=native.make_opts(pair_symmetric=True))
        chk, _ = native.cc_ladder_workspace_query(
            3, 20, 30, "fp64", backward=backward,
            opts=native.make_opts(pair_symmetric=True, check_symmetry=True))
        assert chk == base + 256
        plain, _ = native.cc_ladder_workspace_query(3, 20, 30, "fp64", backward=backward)
        alone, _ = native.cc_ladder_workspace_query(3, 20, 30, "fp64", backward=backward,
                                                    opts=native.make_opts(check_symmetry=True))
        assert alone == plain


def _opts_at(native, addr, nbytes):
    o = native.make_opts()
    o.workspace, o.workspace_bytes = addr, nbytes
    return o


def test_workspace_overlapping_an_array_is_rejected_on_the_host(native):
    # host-side: the plan (sized to the workspace) and the overlap of the bytes
    # it uses with every array argument are checked before any device call
    lib = native.load()
    o, v, P = 2, 8, 4
    planned, _ = native.cc_ladder_workspace_query(o, v, P, "fp64", hbm_budget=1 << 30)
    nt, nL = o * o * v * v * 8, P * v * v * 8
    L, t, R = 1 << 24, 1 << 26, 1 << 28
    big = 1 << 30
    ref = ctypes.byref
    for ws in (L, t + 256, R + nt - 256, t - 256 * ((planned + 255) // 256) + 256):
        opts = _opts_at(native, ws, big)
        assert lib.cc_ladder_residual(o, v, P, L, t, R, 0, None, ref(opts)) == native.CC_LADDER_EINVAL, ws
    # the adjoint: every one of its five arrays counts
    lam, dL, dt = 1 << 29, 1 << 31, 1 << 32
    planned_b, _ = native.cc_ladder_workspace_query(o, v, P, "fp64", backward=True,
                                                    hbm_budget=1 << 30)
    for ws in (L, t, lam + 512, dL, dt + nt - 256):
        opts = _opts_at(native, ws, big)
        assert lib.cc_ladder_backward(o, v, P, L, t, lam, dL, dt, 0, None,
                                      ref(opts)) == native.CC_LADDER_EINVAL, ws
    # an occupied-index term
    Lov, X = 1 << 24, 1 << 28
    opts = _opts_at(native, X, big)
    assert lib.cc_intermediate_ijkl(o, v, P, Lov, t, X, 0, None, ref(opts)) == native.CC_LADDER_EINVAL


def test_workspace_overlap_counts_only_the_planned_bytes(native):
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    lib = native.load()
    o, v, P = 2, 8, 4
    planned, _ = native.cc_ladder_workspace_query(o, v, P, "fp64", hbm_budget=1 << 30)
    L, t, R = 1 << 24, 1 << 26, 1 << 28
    # a workspace ending inside t, but whose planned part ends before t: accepted
    # by the host checks, so the call proceeds to the device check
    ws = t - ((planned + 255) // 256) * 256
    opts = _opts_at(native, ws, (t - ws) + 4096)
    rc = lib.cc_ladder_residual(o, v, P, L, t, R, 0, None, ctypes.byref(opts))
    assert rc == native.CC_LADDER_ENODEV
    # clear of every array: the device check is reached as well
    opts = _opts_at(native, 1 << 34, 1 << 30)
    assert lib.cc_ladder_residual(o, v, P, L, t, R, 0, None, ctypes.byref(opts)) == native.CC_LADDER_ENODEV


def test_make_opts_keeps_its_tensors(native):
    import torch

    ws = torch.empty(512, dtype=torch.uint8)
    with pytest.raises(TypeError):
        native.make_opts(workspace=ws)  # host memory is not a device workspace
    o = native.make_opts(pair_symmetric=True, check_symmetry=True)
    assert o.flags == native.CC_LADDER_PAIR_SYMMETRIC | native.CC_LADDER_CHECK_SYMMETRY
    c = native.copy_opts(o, a_block=3)
    assert c.a_block == 3 and c.flags == o.flags and o.a_block == 0


def test_planner_plus_minus_footprint(native):
    # t+ / t- over the pairs i <= j, i < j and c <= d, c < d (row strides rounded
    # to 4 elements), V+ / V- over the block's pairs a <= b, a < b, the packed
    # integral block, and the packed build's tile offsets
    def r256(x):
        return (x + 255) // 256 * 256

    o, v, P, n_a = 5, 21, 30, 6
    for prec, es in (("fp64", 8), ("fp32", 4)):
        nbytes, blk = native.cc_ladder_workspace_query(
            o, v, P, prec, opts=native.make_opts(a_block=n_a, pair_symmetric=True, plus_minus=True))
        assert blk == n_a
        kp, km = v * (v + 1) // 2, v * (v - 1) // 2
        ldp, ldm = (kp + 3) // 4 * 4, (km + 3) // 4 * 4
        npk = n_a * v - n_a * (n_a - 1) // 2
        want = (r256(o * (o + 1) // 2 * ldp * es) + r256(o * (o - 1) // 2 * ldm * es)
                + r256(npk * ldp * es) + r256((npk - n_a) * ldm * es))
        if prec == "fp32":
            want += r256(P * v * v * 4)
        want += r256(npk * v * v * es)
        tiles_m = (n_a * v + 127) // 128
        want += r256((tiles_m + 1) * 4)
        assert nbytes == want, (prec, nbytes, want)


def test_planner_symmetric_vectors_footprint(native):
    # t+- and V+- as above, then the packed vectors [P][ldg] and the whole
    # pair-pair integral [ldg][ldg] (ldg = v(v+1)/2 rounded to 4) in place of the
    # packed block (and of the float32 copy of L), and the tile offsets of its
    # upper-triangle grid
    def r256(x):
        return (x + 255) // 256 * 256

    o, v, P, n_a = 5, 21, 30, 6
    for prec, es in (("fp64", 8), ("fp32", 4)):
        opts = native.make_opts(a_block=n_a, pair_symmetric=True, plus_minus=True,
                                symmetric_vectors=True)
        nbytes, blk = native.cc_ladder_workspace_query(o, v, P, prec, opts=opts)
        assert blk == n_a
        kp, km = v * (v + 1) // 2, v * (v - 1) // 2
        ldp, ldm = (kp + 3) // 4 * 4, (km + 3) // 4 * 4
        npk = n_a * v - n_a * (n_a - 1) // 2
        want = (r256(o * (o + 1) // 2 * ldp * es) + r256(o * (o - 1) // 2 * ldm * es)
                + r256(npk * ldp * es) + r256((npk - n_a) * ldm * es))
        want += r256(P * ldp * es) + r256(ldp * ldp * es)
        want += r256(((ldp + 127) // 128 + 1) * 4)
        assert nbytes == want, (prec, nbytes, want)
        # a budget that the whole integral alone fills: the packed blocks of one
        # virtual, as without the flag
        small = ldp * ldp * es
        one = dict(a_block=1, pair_symmetric=True, plus_minus=True)
        a = native.cc_ladder_workspace_query(
            o, v, P, prec, hbm_budget=small, opts=native.make_opts(symmetric_vectors=True, **one))
        b = native.cc_ladder_workspace_query(o, v, P, prec, hbm_budget=small,
                                             opts=native.make_opts(**one))
        assert a == b and a[0] <= small


def test_symmetric_vectors_footprint_packed_forward_and_adjoint(native):
    # the packed forward and the pair-symmetric adjoint keep their buffers and add
    # the packed vectors and the pair-pair integral (the float32 forward drops its
    # float32 copy of L); the split forwards add both in float64 and cut their
    # digits from the packed vectors' v(v+1)/2 columns instead of L's v^2
    def r256(x):
        return (x + 255) // 256 * 256

    o, v, P, n_a = 4, 19, 11, 5
    ldg = (v * (v + 1) // 2 + 3) // 4 * 4
    tiles_old = r256(((n_a * v + 127) // 128 + 1) * 4)
    tiles_new = r256(((ldg + 127) // 128 + 1) * 4)
    for prec, es in (("fp64", 8), ("fp32", 4)):
        for backward in (False, True):
            kw = dict(a_block=n_a, pair_symmetric=True)
            a, _ = native.cc_ladder_workspace_query(
                o, v, P, prec, backward=backward, opts=native.make_opts(symmetric_vectors=True, **kw))
            b, _ = native.cc_ladder_workspace_query(o, v, P, prec, backward=backward,
                                                    opts=native.make_opts(**kw))
            want = b + r256(P * ldg * es) + r256(ldg * ldg * es) - tiles_old + tiles_new
            if prec == "fp32" and not backward:
                want -= r256(P * v * v * 4)
            assert a == want, (prec, backward, a, want)
    kw = dict(a_block=n_a, pair_symmetric=True)
    a, _ = native.cc_ladder_workspace_query(o, v, P, "split_int8",
                                            opts=native.make_opts(symmetric_vectors=True, **kw))
    b, _ = native.cc_ladder_workspace_query(o, v, P, "split_int8", opts=native.make_opts(**kw))

    def digits(rows, nbytes):  # digit bytes per entry; rows padded past the last tile, K to 64
        rows_pad = (rows + 127) // 128 * 128 + 128
        return r256(nbytes * rows_pad * ((P + 63) // 64 * 64)) + r256(rows_pad * 4)

    want = (b - digits(v * v, 5) + digits(ldg, 5) + r256(P * ldg * 8) + r256(ldg * ldg * 8)
            - tiles_old + tiles_new)
    assert a == want, ("split_int8", a, want)
    # split-bf16: four bf16 digits, one exponent per row; its compact grid's rows are 64 high
    a, _ = native.cc_ladder_workspace_query(o, v, P, "split_bf16",
                                            opts=native.make_opts(symmetric_vectors=True, **kw))
    b, _ = native.cc_ladder_workspace_query(o, v, P, "split_bf16", opts=native.make_opts(**kw))
    tiles64_old = r256(((n_a * v + 63) // 64 + 1) * 4)
    tiles64_new = r256(((ldg + 63) // 64 + 1) * 4)
    want = (b - digits(v * v, 8) + digits(ldg, 8) + r256(P * ldg * 8) + r256(ldg * ldg * 8)
            - tiles64_old + tiles64_new)
    assert a == want, ("split_bf16", a, want)


def test_symmetric_vectors_needs_pair_symmetry(native):
    with pytest.raises(native.LadderError) as e:
        native.cc_ladder_workspace_query(3, 10, 5, "fp64",
                                         opts=native.make_opts(symmetric_vectors=True))
    assert e.value.code == native.CC_LADDER_EINVAL
    native.cc_ladder_workspace_query(
        3, 10, 5, "fp64", opts=native.make_opts(pair_symmetric=True, symmetric_vectors=True))


def test_plus_minus_needs_pair_symmetry(native):
    with pytest.raises(native.LadderError) as e:
        native.cc_ladder_workspace_query(3, 10, 5, "fp64", opts=native.make_opts(plus_minus=True))
    assert e.value.code == native.CC_LADDER_EINVAL
    with pytest.raises(native.LadderError) as e:
        native.cc_ladder_workspace_query(3, 10, 5, "split_bf16",
                                         opts=native.make_opts(pair_symmetric=True, plus_minus=True))
    assert e.value.code == native.CC_LADDER_EUNSUPPORTED
    # the adjoint plans as with pair symmetry alone
    a = native.cc_ladder_workspace_query(3, 10, 5, "fp64", backward=True,
                                         opts=native.make_opts(pair_symmetric=True, plus_minus=True))
    b = native.cc_ladder_workspace_query(3, 10, 5, "fp64", backward=True,
                                         opts=native.make_opts(pair_symmetric=True))
    assert a == b


def test_planner_split_int8_footprint(native):
    # int8 digit buffers (one byte per digit) of L (rows v^2, K = P padded to
    # 64), t and one integral block, exponents per (row, chunk of 16384), and
    # the float64 block
    def r256(x):
        return (x + 255) // 256 * 256

    rows_pad = lambda r: (r + 127) // 128 * 128 + 128
    o, v, P = 4, 30, 50
    for S in (0, 4, 5):
        nbytes, n = native.cc_ladder_workspace_query(o, v, P, "split_int8",
                                                     opts=native.make_opts(split_slices=S))
        s = S or 5
        kL, kt = (P + 63) // 64 * 64, (v * v + 63) // 64 * 64
        ch = lambda k: max(1, (k + 16383) // 16384)
        want = (r256(s * rows_pad(v * v) * kL) + r256(rows_pad(v * v) * ch(kL) * 4)
                + r256(s * rows_pad(o * o) * kt) + r256(rows_pad(o * o) * ch(kt) * 4)
                + r256(v ** 4 * 8) + r256(s * rows_pad(v * v) * kt) + r256(rows_pad(v * v) * ch(kt) * 4))
        assert n == v and nbytes == want, (S, nbytes, want)
    for bad in (2, 3, 6):
        with pytest.raises(native.LadderError) as e:
            native.cc_ladder_workspace_query(o, v, P, "split_int8",
                                             opts=native.make_opts(split_slices=bad))
        assert e.value.code == native.CC_LADDER_EINVAL
    # five digits keep the triangle only (five int32 sums per output)
    with pytest.raises(native.LadderError) as e:
        native.cc_ladder_workspace_query(o, v, P, "split_int8",
                                         opts=native.make_opts(split_slices=5, split_depth=2))
    assert e.value.code == native.CC_LADDER_EUNSUPPORTED
    with pytest.raises(native.LadderError) as e:
        native.cc_ladder_workspace_query(o, v, P, "split_int8", backward=True)
    assert e.value.code == native.CC_LADDER_EUNSUPPORTED


def test_noalloc_host_checks(native):
    import torch

    lib = native.load()
    # one float64 virtual at v = 330 needs 330^3 * 8 bytes, beyond the static
    # scratch: rejected before any device call
    assert lib.cc_ladder_residual_noalloc(1, 330, 2, 1 << 24, 1 << 34, 1 << 36, 0, None,
                                          None) == native.CC_LADDER_ENOMEM
    nbytes, _ = native.cc_ladder_workspace_query(
        1, 322, 2, "fp64", hbm_budget=native.CC_LADDER_NOALLOC_SCRATCH_BYTES)
    assert nbytes <= native.CC_LADDER_NOALLOC_SCRATCH_BYTES
    # a caller workspace, or the symmetry check's read-back, is not accepted
    o = _opts_at(native, 1 << 40, 1 << 20)
    assert lib.cc_ladder_residual_noalloc(2, 4, 2, 1 << 24, 1 << 26, 1 << 28, 0, None,
                                          ctypes.byref(o)) == native.CC_LADDER_EINVAL
    o = native.make_opts(pair_symmetric=True, check_symmetry=True)
    assert lib.cc_ladder_residual_noalloc(2, 4, 2, 1 << 24, 1 << 26, 1 << 28, 0, None,
                                          ctypes.byref(o)) == native.CC_LADDER_EINVAL
    # argument checks as the allocating entry point
    assert lib.cc_ladder_residual_noalloc(2, 4, 2, None, 1 << 26, 1 << 28, 0, None,
                                          None) == native.CC_LADDER_EINVAL
    R = 1 << 20
    assert lib.cc_ladder_residual_noalloc(2, 4, 2, 1 << 24, R + 8, R, 0, None,
                                          None) == native.CC_LADDER_EINVAL
    if not torch.cuda.is_available():
        assert lib.cc_ladder_residual_noalloc(2, 4, 2, 1 << 24, 1 << 26, 1 << 28, 0, None,
                                              None) == native.CC_LADDER_ENODEV
