// Host-only planner: buffer layout and block-size selection.
#include "plan.h"

#include "split.hpp"

#include <cstdint>

namespace ccl {

namespace {

constexpr size_t kAlign = 256;

size_t round_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Appends a buffer of `bytes` at the end of the layout and returns its offset.
size_t take(size_t* cursor, size_t bytes) {
  size_t off = *cursor;
  *cursor = round_up(off + bytes);
  return off;
}

}  // namespace

int check_dims(int o, int v, int P) {
  if (o <= 0 || v <= 0 || P <= 0) return CC_LADDER_EINVAL;
  // o^2 and v^2 are GEMM extents held in 32-bit ints.
  if (o > 46340 || v > 46340 || P > (1 << 24)) return CC_LADDER_EINVAL;
  // element counts of the arrays (o^2 v^2, P v^2, P o v) stay far inside size_t
  // byte counts: at most 2^52 elements each
  const unsigned long long o2 = static_cast<unsigned long long>(o) * o;
  const unsigned long long v2 = static_cast<unsigned long long>(v) * v;
  constexpr unsigned long long kMaxElems = 1ull << 52;
  if (o2 * v2 > kMaxElems || static_cast<unsigned long long>(P) * v2 > kMaxElems ||
      static_cast<unsigned long long>(P) * o * v > kMaxElems)
    return CC_LADDER_EINVAL;
  return CC_LADDER_OK;
}

int check_precision_opts(int precision, const cc_ladder_opts* opts) {
  if (precision != CC_LADDER_FP64 && precision != CC_LADDER_FP32 &&
      precision != CC_LADDER_SPLIT_BF16 && precision != CC_LADDER_SPLIT_INT8)
    return CC_LADDER_EINVAL;
  if (!opts) return CC_LADDER_OK;
  if (opts->a_block < 0 || opts->split_depth < 0 || opts->split_depth > 2) return CC_LADDER_EINVAL;
  if ((opts->flags & ~(CC_LADDER_PAIR_SYMMETRIC | CC_LADDER_EXCHANGE | CC_LADDER_CHECK_SYMMETRY |
                       CC_LADDER_PLUS_MINUS | CC_LADDER_SYMMETRIC_VECTORS)) != 0 ||
      opts->reserved != 0)
    return CC_LADDER_EINVAL;
  // the symmetric/antisymmetric combinations and the whole pair-pair integral
  // serve the pair-symmetric paths
  if ((opts->flags & (CC_LADDER_PLUS_MINUS | CC_LADDER_SYMMETRIC_VECTORS)) &&
      !(opts->flags & CC_LADDER_PAIR_SYMMETRIC))
    return CC_LADDER_EINVAL;
  if (opts->split_slices != 0) {
    const int lo = precision == CC_LADDER_SPLIT_INT8 ? 4 : 2;
    const int hi = precision == CC_LADDER_SPLIT_INT8 ? 5 : 4;
    if (opts->split_slices < lo || opts->split_slices > hi) return CC_LADDER_EINVAL;
  }
  if (opts->k_chunk < 0 || opts->k_chunk % 64 != 0) return CC_LADDER_EINVAL;
  if (opts->workspace && (reinterpret_cast<uintptr_t>(opts->workspace) % kAlign) != 0)
    return CC_LADDER_EINVAL;
  return CC_LADDER_OK;
}

bool overlaps(const void* a, size_t abytes, const void* b, size_t bbytes) {
  if (!abytes || !bbytes) return false;
  const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
  return x < y + bbytes && y < x + abytes;
}

int check_residual_args(int o, int v, int P, const double* L, const double* t, const double* R,
                        int precision, const cc_ladder_opts* opts, Operand ops[3]) {
  int rc = check_dims(o, v, P);
  if (rc) return rc;
  rc = check_precision_opts(precision, opts);
  if (rc) return rc;
  if (!L || !t || !R) return CC_LADDER_EINVAL;
  const size_t nt = static_cast<size_t>(o) * o * v * v * sizeof(double);
  const size_t nL = static_cast<size_t>(P) * v * v * sizeof(double);
  ops[0] = {L, nL};
  ops[1] = {t, nt};
  ops[2] = {R, nt};
  if (overlaps(R, nt, t, nt) || overlaps(R, nt, L, nL)) return CC_LADDER_EINVAL;
  return CC_LADDER_OK;
}

int check_backward_args(int o, int v, int P, const double* L, const double* t, const double* lam,
                        const double* dL, const double* dt, int precision,
                        const cc_ladder_opts* opts, Operand ops[5]) {
  int rc = check_dims(o, v, P);
  if (rc) return rc;
  rc = check_precision_opts(precision, opts);
  if (rc) return rc;
  if (!L || !t || !lam || !dL || !dt) return CC_LADDER_EINVAL;
  const size_t nt = static_cast<size_t>(o) * o * v * v * sizeof(double);
  const size_t nL = static_cast<size_t>(P) * v * v * sizeof(double);
  ops[0] = {L, nL};
  ops[1] = {t, nt};
  ops[2] = {lam, nt};
  ops[3] = {dL, nL};
  ops[4] = {dt, nt};
  if (overlaps(dt, nt, t, nt) || overlaps(dt, nt, lam, nt) || overlaps(dt, nt, L, nL) ||
      overlaps(dL, nL, L, nL) || overlaps(dL, nL, t, nt) || overlaps(dL, nL, lam, nt) ||
      overlaps(dL, nL, dt, nt))
    return CC_LADDER_EINVAL;
  return CC_LADDER_OK;
}

int check_workspace(const cc_ladder_opts* opts, size_t plan_bytes, const Operand* ops, int n) {
  if (!opts || !opts->workspace) return CC_LADDER_OK;
  for (int i = 0; i < n; ++i)
    if (overlaps(opts->workspace, plan_bytes, ops[i].p, ops[i].bytes)) return CC_LADDER_EINVAL;
  return CC_LADDER_OK;
}

int pair_block_start(int v, int nb, int k) {
  if (k <= 0) return 0;
  if (k >= nb) return v;
  const long long target = (long long)k * ((long long)v * (v + 1) / 2);
  int lo = 0, hi = v;  // smallest a with pair_prefix(a) * nb >= target
  while (lo < hi) {
    const int mid = lo + (hi - lo) / 2;
    if (pair_prefix(mid, v) * nb >= target) hi = mid; else lo = mid + 1;
  }
  return lo;
}

void block_range(const Plan& pl, int blk, int* a0, int* na) {
  if (pl.balanced) {
    *a0 = pair_block_start(pl.v, pl.nblocks, blk);
    *na = pair_block_start(pl.v, pl.nblocks, blk + 1) - *a0;
    return;
  }
  *a0 = blk * pl.n_a;
  *na = (pl.v - *a0) < pl.n_a ? (pl.v - *a0) : pl.n_a;
}

int layout_plan(int o, int v, int P, int precision, int backward, int n_a,
                int slices, int depth, int k_chunk, unsigned flags, Plan* plan, int nb) {
  const int pairsym = (flags & CC_LADDER_PAIR_SYMMETRIC) ? 1 : 0;
  Plan p;
  // packed forward in pair-balanced blocks: the widest block sizes the tile
  // table, the block with the most pairs (a <= b, and a < b) the buffers
  size_t npk_max = 0, nstrict_max = 0;
  if (nb > 0 && pairsym && !backward) {
    if (nb > v) return CC_LADDER_EINVAL;
    p.balanced = 1;
    n_a = 0;
    for (int k = 0; k < nb; ++k) {
      const int a0 = pair_block_start(v, nb, k), a1 = pair_block_start(v, nb, k + 1);
      const size_t np = static_cast<size_t>(pair_prefix(a1, v) - pair_prefix(a0, v));
      n_a = (a1 - a0) > n_a ? (a1 - a0) : n_a;
      npk_max = np > npk_max ? np : npk_max;
      const size_t ns = np - static_cast<size_t>(a1 - a0);
      nstrict_max = ns > nstrict_max ? ns : nstrict_max;
    }
  }
  if (n_a < 1 || n_a > v) return CC_LADDER_EINVAL;
  p.o = o; p.v = v; p.P = P;
  p.precision = precision;
  p.backward = backward ? 1 : 0;
  p.n_a = n_a;
  p.nblocks = p.balanced ? nb : (v + n_a - 1) / n_a;
  const size_t v2 = static_cast<size_t>(v) * v;
  const size_t o2 = static_cast<size_t>(o) * o;
  p.pairsym = (pairsym && !backward) ? 1 : 0;
  p.pairsym_adj = (pairsym && backward) ? 1 : 0;
  // entries of one integral block: n_a*v rows (a,b); packed rows a <= b when the
  // amplitudes are pair-symmetric (with equal virtual counts the first block
  // holds the most).  The adjoint's W block always has n_a*v rows.
  const size_t npk = p.balanced ? npk_max : static_cast<size_t>(pair_prefix(n_a, v));
  p.npk = p.pairsym ? static_cast<long long>(npk) : 0;
  const size_t npk_ld = (npk + 3) / 4 * 4;  // row stride of the adjoint's gathered lam
  const size_t rows = (p.pairsym || p.pairsym_adj) ? npk : static_cast<size_t>(n_a) * v;
  const size_t blk = rows * v2;
  const size_t blk_w = static_cast<size_t>(n_a) * v * v2;
  size_t cur = 0;
  p.exchange = (flags & CC_LADDER_EXCHANGE) ? 1 : 0;
  p.pm = (p.pairsym && (flags & CC_LADDER_PLUS_MINUS)) ? 1 : 0;
  // symmetric vectors: the whole pair-pair integral G [ldg][ldg] and the packed
  // vectors [P][ldg] (side v(v+1)/2 rounded to 4, pads zero) replace the packed
  // build in the FP64 and FP32 pair-symmetric paths and in the split
  // pair-symmetric forwards (there G is float64, built from digits of the packed
  // vectors)
  const size_t es_g = precision == CC_LADDER_FP32 ? sizeof(float) : sizeof(double);
  p.gsym = ((flags & CC_LADDER_SYMMETRIC_VECTORS) &&
            (((p.pairsym || p.pairsym_adj) &&
              (precision == CC_LADDER_FP64 || precision == CC_LADDER_FP32)) ||
             (p.pairsym && !p.backward &&
              (precision == CC_LADDER_SPLIT_INT8 || precision == CC_LADDER_SPLIT_BF16)))) ? 1 : 0;
  if (p.gsym) p.ldg = static_cast<long long>((static_cast<size_t>(v) * (v + 1) / 2 + 3) / 4 * 4);
  if (p.exchange) {
    // the float32 form swaps while converting into its own operand copy; the
    // combinations t+- of swapped amplitudes are t+ and -t-, made without a copy
    if (precision != CC_LADDER_FP32 && !p.pm) p.off_tx = take(&cur, o2 * v2 * sizeof(double));
    if (p.backward) p.off_dtx = take(&cur, o2 * v2 * sizeof(double));
  }
  if (p.pm) {
    if (precision == CC_LADDER_SPLIT_BF16 || precision == CC_LADDER_SPLIT_INT8)
      return CC_LADDER_EUNSUPPORTED;
    // operand rows over the pairs c <= d (t+, V+) and c < d (t-, V-), strides
    // rounded to 16-byte multiples of either element size
    const size_t es = precision == CC_LADDER_FP64 ? sizeof(double) : sizeof(float);
    const size_t kp = static_cast<size_t>(v) * (v + 1) / 2, km = static_cast<size_t>(v) * (v - 1) / 2;
    p.ldp = static_cast<long long>((kp + 3) / 4 * 4);
    p.ldm = static_cast<long long>((km + 3) / 4 * 4);
    const size_t mp = static_cast<size_t>(o) * (o + 1) / 2, mm = static_cast<size_t>(o) * (o - 1) / 2;
    // packed rows of the largest block: a <= b, and a < b
    const size_t np = npk, nm = p.balanced ? nstrict_max : npk - static_cast<size_t>(n_a);
    p.off_Tp = take(&cur, mp * p.ldp * es);
    p.off_Tm = take(&cur, mm * p.ldm * es);
    p.off_Vp = take(&cur, np * p.ldp * es);
    p.off_Vm = take(&cur, nm * p.ldm * es);
    if (precision == CC_LADDER_FP32) p.k_chunk = k_chunk ? k_chunk : 512;
    if (p.gsym) {
      // no packed block: V+- are gathered from G
      p.off_Lp = take(&cur, static_cast<size_t>(P) * p.ldg * es);
      p.off_G = take(&cur, static_cast<size_t>(p.ldg) * p.ldg * es);
    } else {
      if (precision == CC_LADDER_FP32)
        p.off_L = take(&cur, static_cast<size_t>(P) * v2 * sizeof(float));
      p.off_V = take(&cur, blk * es);
    }
  } else {
  switch (precision) {
    case CC_LADDER_FP64:
      p.off_V = take(&cur, blk * sizeof(double));
      if (p.backward) p.off_W = take(&cur, blk_w * sizeof(double));
      if (p.pairsym_adj) p.off_lamP = take(&cur, o2 * npk_ld * sizeof(double));
      break;
    case CC_LADDER_FP32:
      p.k_chunk = k_chunk ? k_chunk : 512;
      // the forward over G needs no float32 copy of L (the adjoint's dL does)
      if (!p.gsym || p.backward) p.off_L = take(&cur, static_cast<size_t>(P) * v2 * sizeof(float));
      p.off_t = take(&cur, o2 * v2 * sizeof(float));
      if (p.backward) p.off_lam = take(&cur, o2 * v2 * sizeof(float));
      p.off_V = take(&cur, blk * sizeof(float));
      if (p.backward) p.off_W = take(&cur, blk_w * sizeof(float));
      if (p.pairsym_adj) p.off_lamP = take(&cur, o2 * npk_ld * sizeof(float));
      break;
    case CC_LADDER_SPLIT_BF16: {
      if (p.backward) return CC_LADDER_EUNSUPPORTED;
      p.slices = slices ? slices : 4;
      // automatic depth: the 4-slice form keeps the triangle's next anti-diagonal
      p.split_depth = depth ? depth : (p.slices == 4 ? 2 : 1);
      const size_t s = static_cast<size_t>(p.slices);
      // digits of L's columns (a,c), or of the packed vectors' columns {a,c}
      const SliceDims dL = slice_dims(p.gsym ? p.ldg : static_cast<long long>(v2), P);
      const SliceDims dt = slice_dims(static_cast<long long>(o2), static_cast<int>(v2));
      const SliceDims dV = slice_dims(static_cast<long long>(rows), static_cast<int>(v2));
      p.off_L = take(&cur, s * dL.rows_pad * dL.k_pad * 2);
      p.off_Lexp = take(&cur, static_cast<size_t>(dL.rows_pad) * sizeof(int));
      p.off_t = take(&cur, s * dt.rows_pad * dt.k_pad * 2);
      p.off_texp = take(&cur, static_cast<size_t>(dt.rows_pad) * exp_chunks(dt.k_pad, p.slices) * sizeof(int));
      p.off_V = take(&cur, blk * sizeof(double));
      p.off_Vs = take(&cur, s * dV.rows_pad * dV.k_pad * 2);
      p.off_Vexp = take(&cur, static_cast<size_t>(dV.rows_pad) * exp_chunks(dV.k_pad, p.slices) * sizeof(int));
      break;
    }
    case CC_LADDER_SPLIT_INT8: {
      if (p.backward) return CC_LADDER_EUNSUPPORTED;
      p.slices = slices ? slices : 5;
      p.split_depth = depth ? depth : 1;
      // the kernels hold S + depth - 1 int32 sums per output: 5 at most
      if (p.slices + p.split_depth - 1 > 5) return CC_LADDER_EUNSUPPORTED;
      const size_t s = static_cast<size_t>(p.slices);  // one byte per digit
      // digits of the vectors' columns (a,c), or with symmetric vectors of the
      // packed vectors' columns {a,c}, a <= c
      const SliceDims dL = slice_dims(p.gsym ? p.ldg : static_cast<long long>(v2), P);
      const SliceDims dt = slice_dims(static_cast<long long>(o2), static_cast<int>(v2));
      const SliceDims dV = slice_dims(static_cast<long long>(rows), static_cast<int>(v2));
      p.off_L = take(&cur, s * dL.rows_pad * dL.k_pad);
      p.off_Lexp = take(&cur, static_cast<size_t>(dL.rows_pad) * i8_chunks(dL.k_pad) * sizeof(int));
      p.off_t = take(&cur, s * dt.rows_pad * dt.k_pad);
      p.off_texp = take(&cur, static_cast<size_t>(dt.rows_pad) * i8_chunks(dt.k_pad) * sizeof(int));
      p.off_V = take(&cur, blk * sizeof(double));
      p.off_Vs = take(&cur, s * dV.rows_pad * dV.k_pad);
      p.off_Vexp = take(&cur, static_cast<size_t>(dV.rows_pad) * i8_chunks(dV.k_pad) * sizeof(int));
      break;
    }
    default:
      return CC_LADDER_EINVAL;
  }
  }
  if (p.pairsym_adj) {
    // the adjoint's dt accumulates B[(ij)][(cd)] over packed rows; dt += B + mirror(B)
    p.off_B = take(&cur, o2 * v2 * sizeof(double));
  }
  if (p.gsym && !p.pm) {
    p.off_Lp = take(&cur, static_cast<size_t>(P) * p.ldg * es_g);
    p.off_G = take(&cur, static_cast<size_t>(p.ldg) * p.ldg * es_g);
  }
  if ((p.pairsym || p.pairsym_adj) && (flags & CC_LADDER_CHECK_SYMMETRY)) {
    // two maxima of the pair-symmetry check (bit patterns of non-negative doubles)
    p.check_sym = 1;
    p.off_check = take(&cur, 2 * sizeof(unsigned long long));
  }
  if (p.pairsym || p.pairsym_adj) {
    // tile-row offsets of the packed build's compact grid (128-row tiles; 64 rows
    // in the split form), or of the upper-triangle grid of the pair-pair integral
    const size_t bm = precision == CC_LADDER_SPLIT_BF16 ? 64 : 128;
    const size_t rows_m = p.gsym ? static_cast<size_t>(p.ldg) : static_cast<size_t>(n_a) * v;
    const size_t tiles_m = (rows_m + bm - 1) / bm;
    p.off_tiles = take(&cur, (tiles_m + 1) * sizeof(int));
  }
  p.bytes = cur;
  *plan = p;
  return CC_LADDER_OK;
}

namespace {

// Largest block of first indices (1..n_max) whose layout fits `budget`
// (0 = unlimited), then equalised: the same block count with the smallest
// block that achieves it.  `fixed` > 0 takes that block size as given.
template <class Layout>
int search_block(int n_max, size_t budget, int fixed, Layout layout, Plan* plan) {
  int rc;
  if (fixed > 0) {
    rc = layout(fixed < n_max ? fixed : n_max, plan);
    if (rc) return rc;
    return (budget && plan->bytes > budget) ? CC_LADDER_ENOMEM : CC_LADDER_OK;
  }
  // the footprint grows monotonically with the block size
  Plan best;
  rc = layout(1, &best);
  if (rc) return rc;
  if (budget && best.bytes > budget) return CC_LADDER_ENOMEM;
  int lo = 1, hi = n_max;
  while (lo < hi) {
    const int mid = lo + (hi - lo + 1) / 2;
    Plan trial;
    rc = layout(mid, &trial);
    if (rc) return rc;
    if (!budget || trial.bytes <= budget) {
      lo = mid;
      best = trial;
    } else {
      hi = mid - 1;
    }
  }
  const int nb = (n_max + best.n_a - 1) / best.n_a;
  const int n_eq = (n_max + nb - 1) / nb;
  if (n_eq != best.n_a) {
    rc = layout(n_eq, &best);
    if (rc) return rc;
  }
  *plan = best;
  return CC_LADDER_OK;
}

}  // namespace

namespace {

int make_plan_flags(int o, int v, int P, int precision, int backward, size_t budget,
                    const cc_ladder_opts* opts, unsigned flags, Plan* plan) {
  const int slices = opts ? opts->split_slices : 0;
  const int depth = opts ? opts->split_depth : 0;
  const int k_chunk = opts ? opts->k_chunk : 0;
  const int fixed = opts ? opts->a_block : 0;
  if ((flags & CC_LADDER_PAIR_SYMMETRIC) && !backward && fixed == 0) {
    // packed forward: blocks of about equal pair counts (equal virtual counts
    // would leave the last blocks, whose virtuals pair with few others, a
    // small fraction of the first one's work); the fewest blocks that fit
    auto fits = [&](int nb, Plan* p) {
      const int rc = layout_plan(o, v, P, precision, backward, 0, slices, depth, k_chunk, flags, p,
                                 nb);
      if (rc) return rc;
      return (budget && p->bytes > budget) ? CC_LADDER_ENOMEM : CC_LADDER_OK;
    };
    Plan best;
    int rc = fits(v, &best);
    if (rc) return rc;
    int lo = 1, hi = v;
    while (lo < hi) {
      const int mid = lo + (hi - lo) / 2;
      Plan trial;
      rc = fits(mid, &trial);
      if (rc == CC_LADDER_OK) {
        hi = mid;
        best = trial;
      } else if (rc == CC_LADDER_ENOMEM) {
        lo = mid + 1;
      } else {
        return rc;
      }
    }
    if (best.nblocks != lo) {
      rc = fits(lo, &best);
      if (rc) return rc;
    }
    *plan = best;
    return CC_LADDER_OK;
  }
  return search_block(v, budget, fixed, [&](int n_a, Plan* p) {
    return layout_plan(o, v, P, precision, backward, n_a, slices, depth, k_chunk, flags, p);
  }, plan);
}

}  // namespace

int make_plan(int o, int v, int P, int precision, int backward, size_t budget,
              const cc_ladder_opts* opts, Plan* plan) {
  int rc = check_dims(o, v, P);
  if (rc) return rc;
  rc = check_precision_opts(precision, opts);
  if (rc) return rc;
  const unsigned flags = opts ? opts->flags : 0u;
  rc = make_plan_flags(o, v, P, precision, backward, budget, opts, flags, plan);
  // the whole pair-pair integral does not fit: the packed blocks instead
  if (rc == CC_LADDER_ENOMEM && (flags & CC_LADDER_SYMMETRIC_VECTORS))
    rc = make_plan_flags(o, v, P, precision, backward, budget, opts,
                         flags & ~CC_LADDER_SYMMETRIC_VECTORS, plan);
  return rc;
}

int choose_kc_tiling(long long M, long long N, bool tall, bool split, long long* main_rows) {
  constexpr long long kCUs = 256;  // compute units of one MI355X
  constexpr long long kTN = 256;   // the K-contiguous kernel's tile width
  const long long tn = (N + kTN - 1) / kTN;
  // one workgroup per CU at a time: a launch lasts about (rounds of its grid
  // over the CUs) x (one tile's time, proportional to its height)
  auto span = [&](long long rows, long long bm) {
    const long long tiles = (rows + bm - 1) / bm * tn;
    return (tiles + kCUs - 1) / kCUs * bm;
  };
  const long long rem = M % 128;
  long long best = span(M, 128);
  int choice = 128;
  if (tall && span(M, 160) < best) {
    best = span(M, 160);
    choice = 160;
  }
  if (split && M > 128 && rem > 0 && rem <= 64 && span(M - rem, 128) + span(rem, 64) < best) {
    best = span(M - rem, 128) + span(rem, 64);
    choice = 64;
  }
  *main_rows = choice == 64 ? M - rem : M;
  return choice;
}

int choose_k_splits(long long M, long long N, long long K, int bk) {
  constexpr long long kCUs = 256;           // compute units of one MI355X
  constexpr long long kTM = 128, kTN = 256;  // the K-contiguous kernel's tile
  const long long tiles = ((M + kTM - 1) / kTM) * ((N + kTN - 1) / kTN);
  const long long nk = (K + bk - 1) / bk;
  if (tiles <= 0 || tiles >= kCUs) return 1;
  int best = 1;
  double best_cost = 1.0;  // waves per unit of work without a split
  for (int s = 2; s <= 16; ++s) {
    if (nk / s < 64) break;
    const double cost = static_cast<double>((tiles * s + kCUs - 1) / kCUs) / s;
    if (cost < best_cost * 0.999) {
      best = s;
      best_cost = cost;
    }
  }
  return best;
}

int layout_intermediate(int which, int o, int v, int P, int precision, int n_p, int k_chunk,
                        Plan* plan) {
  const int n_first = which == CC_INTERMEDIATE_IJBK ? v : o;
  if (n_p < 1 || n_p > n_first) return CC_LADDER_EINVAL;
  Plan p;
  p.o = o; p.v = v; p.P = P;
  p.precision = precision;
  p.op = which == CC_INTERMEDIATE_IJKL ? kOpIjkl : which == CC_INTERMEDIATE_IJBK ? kOpIjbk : kOpHole;
  p.n_a = n_p;
  p.nblocks = (n_first + n_p - 1) / n_p;
  const size_t v2 = static_cast<size_t>(v) * v;
  const size_t o2 = static_cast<size_t>(o) * o;
  const size_t ov = static_cast<size_t>(o) * v;
  // integral block: [n_p][o][v][v] for the intermediates, (ik|jl) as [n_p][o][o][o]
  // for the hole-hole ladder
  const size_t blk = p.op == kOpHole ? static_cast<size_t>(n_p) * o * o2
                                     : static_cast<size_t>(n_p) * o * v2;
  size_t cur = 0;
  switch (precision) {
    case CC_LADDER_FP64:
      // (bd|kc) is built with its last two indices in (d, c) order and met by
      // the amplitudes with c, d swapped
      if (p.op == kOpIjbk) p.off_tx = take(&cur, o2 * v2 * sizeof(double));
      p.off_V = take(&cur, blk * sizeof(double));
      break;
    case CC_LADDER_FP32:
      p.k_chunk = k_chunk ? k_chunk : 512;
      // L_ov (L_oo for the hole-hole ladder)
      p.off_L = take(&cur, static_cast<size_t>(P) * (p.op == kOpHole ? o2 : ov) * sizeof(float));
      if (p.op == kOpIjbk) p.off_L2 = take(&cur, static_cast<size_t>(P) * v2 * sizeof(float));
      p.off_t = take(&cur, o2 * v2 * sizeof(float));
      p.off_V = take(&cur, blk * sizeof(float));
      break;
    case CC_LADDER_SPLIT_BF16:
    case CC_LADDER_SPLIT_INT8:
      return CC_LADDER_EUNSUPPORTED;
    default:
      return CC_LADDER_EINVAL;
  }
  if (p.op != kOpHole) {
    // split K from the whole output's tile count, so every block sums in the
    // same order whatever n_p is
    p.k_splits = choose_k_splits(static_cast<long long>(o2), static_cast<long long>(n_first) * o,
                                 static_cast<long long>(v2), precision == CC_LADDER_FP64 ? 16 : 32);
    if (p.k_splits > 1)
      p.off_part = take(&cur, static_cast<size_t>(p.k_splits) * o2 * n_p * o * sizeof(double));
  }
  p.bytes = cur;
  *plan = p;
  return CC_LADDER_OK;
}

int make_plan_intermediate(int which, int o, int v, int P, int precision, size_t budget,
                           const cc_ladder_opts* opts, Plan* plan) {
  if (which != CC_INTERMEDIATE_IJKL && which != CC_INTERMEDIATE_IJBK && which != CC_HOLE_LADDER)
    return CC_LADDER_EINVAL;
  int rc = check_dims(o, v, P);
  if (rc) return rc;
  rc = check_precision_opts(precision, opts);
  if (rc) return rc;
  // the packed and exchange variants belong to the ladder term only
  if (opts && opts->flags) return CC_LADDER_EUNSUPPORTED;
  const int k_chunk = opts ? opts->k_chunk : 0;
  const int n_first = which == CC_INTERMEDIATE_IJBK ? v : o;
  return search_block(n_first, budget, opts ? opts->a_block : 0, [&](int n_p, Plan* p) {
    return layout_intermediate(which, o, v, P, precision, n_p, k_chunk, p);
  }, plan);
}

}  // namespace ccl
