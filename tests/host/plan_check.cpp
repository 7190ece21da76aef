// Host-only checker of the planner and the argument validation, built by the
// CPU test suite with g++ under AddressSanitizer and UndefinedBehaviorSanitizer
// (no device code is involved: plan.cpp is plain host C++).  Exercises the
// entry points' host checks and the planner over a sweep of dimensions, forms,
// flags and budgets, and checks the invariants the kernels rely on.  Prints
// "plan_check OK" and returns 0 when every check holds.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "plan.h"

using namespace ccl;

static int g_fail = 0;
#define CHECK(cond)                                                          \
  do {                                                                       \
    if (!(cond)) {                                                           \
      std::fprintf(stderr, "FAILED %s:%d: %s\n", __FILE__, __LINE__, #cond); \
      ++g_fail;                                                              \
    }                                                                        \
  } while (0)

static const double* P_(uintptr_t a) { return reinterpret_cast<const double*>(a); }

static void argument_checks() {
  Operand ops[5];
  const uintptr_t L = 1ull << 24, t = 1ull << 30, R = 1ull << 36;
  CHECK(check_residual_args(2, 8, 4, P_(L), P_(t), P_(R), 0, nullptr, ops) == CC_LADDER_OK);
  CHECK(ops[1].bytes == 2 * 2 * 8 * 8 * sizeof(double) && ops[0].bytes == 4 * 8 * 8 * sizeof(double));
  CHECK(check_residual_args(2, 8, 4, nullptr, P_(t), P_(R), 0, nullptr, ops) == CC_LADDER_EINVAL);
  CHECK(check_residual_args(2, 8, 4, P_(L), P_(t), P_(t + 8), 0, nullptr, ops) == CC_LADDER_EINVAL);
  CHECK(check_residual_args(2, 8, 4, P_(L), P_(t), P_(L + 2040), 0, nullptr, ops) == CC_LADDER_EINVAL);
  CHECK(check_residual_args(2, 8, 4, P_(L), P_(t), P_(R), 4, nullptr, ops) == CC_LADDER_EINVAL);
  // dimensions whose byte counts would not fit comfortably in size_t
  CHECK(check_residual_args(46340, 46340, 1, P_(L), P_(t), P_(R), 0, nullptr, ops) == CC_LADDER_EINVAL);
  CHECK(check_residual_args(1, 46340, 1 << 24, P_(L), P_(t), P_(R), 0, nullptr, ops) ==
        CC_LADDER_EINVAL);
  CHECK(check_residual_args(0, 8, 4, P_(L), P_(t), P_(R), 0, nullptr, ops) == CC_LADDER_EINVAL);
  const uintptr_t lam = 1ull << 38, dL = 1ull << 40, dt = 1ull << 42;
  CHECK(check_backward_args(2, 8, 4, P_(L), P_(t), P_(lam), P_(dL), P_(dt), 1, nullptr, ops) ==
        CC_LADDER_OK);
  CHECK(check_backward_args(2, 8, 4, P_(L), P_(t), P_(lam), P_(dL), P_(lam), 1, nullptr, ops) ==
        CC_LADDER_EINVAL);
  CHECK(check_backward_args(2, 8, 4, P_(L), P_(t), P_(lam), P_(dt + 64), P_(dt), 1, nullptr, ops) ==
        CC_LADDER_EINVAL);
  CHECK(check_backward_args(2, 8, 4, P_(L), P_(t), P_(lam), P_(L), P_(dt), 1, nullptr, ops) ==
        CC_LADDER_EINVAL);
  // options
  cc_ladder_opts o{};
  o.flags = CC_LADDER_PAIR_SYMMETRIC | CC_LADDER_EXCHANGE | CC_LADDER_CHECK_SYMMETRY;
  CHECK(check_precision_opts(0, &o) == CC_LADDER_OK);
  o.flags = 32;  // no such flag
  CHECK(check_precision_opts(0, &o) == CC_LADDER_EINVAL);
  o.flags = CC_LADDER_SYMMETRIC_VECTORS;  // needs PAIR_SYMMETRIC
  CHECK(check_precision_opts(0, &o) == CC_LADDER_EINVAL);
  o.flags |= CC_LADDER_PAIR_SYMMETRIC;
  CHECK(check_precision_opts(0, &o) == CC_LADDER_OK);
  o = cc_ladder_opts{};
  o.workspace = reinterpret_cast<void*>(uintptr_t(4096 + 128));
  CHECK(check_precision_opts(0, &o) == CC_LADDER_EINVAL);  // misaligned workspace
  o = cc_ladder_opts{};
  o.k_chunk = 96;
  CHECK(check_precision_opts(1, &o) == CC_LADDER_EINVAL);
}

static void workspace_checks() {
  Operand ops[3];
  const uintptr_t L = 1ull << 24, t = 1ull << 30, R = 1ull << 36;
  CHECK(check_residual_args(3, 16, 5, P_(L), P_(t), P_(R), 0, nullptr, ops) == CC_LADDER_OK);
  cc_ladder_opts o{};
  CHECK(check_workspace(&o, 1 << 20, ops, 3) == CC_LADDER_OK);  // no workspace
  CHECK(check_workspace(nullptr, 1 << 20, ops, 3) == CC_LADDER_OK);
  const uintptr_t spots[] = {L, t, R, t + ops[1].bytes - 256, L - 256 + 1 * 0};
  for (uintptr_t w : spots) {
    o.workspace = reinterpret_cast<void*>(w);
    o.workspace_bytes = 1 << 20;
    CHECK(check_workspace(&o, 512, ops, 3) == CC_LADDER_EINVAL || w == L - 256);
  }
  // ends exactly where t begins: no shared byte
  o.workspace = reinterpret_cast<void*>(t - 4096);
  CHECK(check_workspace(&o, 4096, ops, 3) == CC_LADDER_OK);
  CHECK(check_workspace(&o, 4097, ops, 3) == CC_LADDER_EINVAL);
  CHECK(!overlaps(reinterpret_cast<void*>(t), 0, reinterpret_cast<void*>(t), 64));
}

static void plan_invariants(const Plan& p, int backward, size_t budget) {
  CHECK(p.n_a >= 1 && p.n_a <= p.v);
  if (p.balanced) {
    // pair-balanced blocks tile [0, v) and none exceeds the buffers' sizes
    CHECK(p.pairsym && !backward && p.nblocks >= 1 && p.nblocks <= p.v);
    int next = 0;
    for (int k = 0; k < p.nblocks; ++k) {
      int a0, na;
      block_range(p, k, &a0, &na);
      CHECK(a0 == next && na >= 0 && na <= p.n_a);
      CHECK(pair_prefix(a0 + na, p.v) - pair_prefix(a0, p.v) <= p.npk);
      next = a0 + na;
    }
    CHECK(next == p.v);
  } else {
    CHECK(p.nblocks == (p.v + p.n_a - 1) / p.n_a);
  }
  CHECK(p.bytes % 256 == 0);
  CHECK(budget == 0 || p.bytes <= budget);
  const size_t offs[] = {p.off_lamP, p.off_B, p.off_check, p.off_tx, p.off_dtx, p.off_L, p.off_t,
                         p.off_lam, p.off_L2, p.off_part, p.off_Lexp, p.off_texp, p.off_V, p.off_W,
                         p.off_Vs, p.off_Vexp, p.off_tiles, p.off_Tp, p.off_Tm, p.off_Vp,
                         p.off_Vm, p.off_Lp, p.off_G};
  for (size_t off : offs) {
    CHECK(off % 256 == 0);
    CHECK(off == 0 || off < p.bytes);
  }
  if (backward) CHECK(p.off_W > p.off_V);
  if (p.pm) {
    // row strides of the pair operands: whole 16-byte chunks of either element size
    CHECK(p.ldp % 4 == 0 && p.ldm % 4 == 0);
    CHECK(p.ldp >= static_cast<long long>(p.v) * (p.v + 1) / 2);
    CHECK(p.ldm >= static_cast<long long>(p.v) * (p.v - 1) / 2);
    CHECK(p.pairsym && !backward && p.off_Vp > p.off_Tp);
    if (p.gsym) {
      // the whole pair-pair integral instead of a packed block
      CHECK(p.ldg == p.ldp && p.off_G > p.off_Lp && p.off_Lp >= p.off_Vm && p.off_V == 0);
    } else {
      CHECK(p.off_V > 0 && p.off_G == 0);
    }
  }
  if (p.gsym) {
    // FP64/FP32 pair-symmetric paths and the split pair-symmetric forwards;
    // the compact grid's tile offsets come after G
    CHECK(p.pairsym || p.pairsym_adj);
    CHECK(p.precision == CC_LADDER_FP64 || p.precision == CC_LADDER_FP32 ||
          ((p.precision == CC_LADDER_SPLIT_INT8 || p.precision == CC_LADDER_SPLIT_BF16) &&
           p.pairsym && !backward));
    CHECK(p.ldg % 4 == 0 && p.ldg >= static_cast<long long>(p.v) * (p.v + 1) / 2);
    CHECK(p.off_G > p.off_Lp && p.off_tiles > p.off_G);
  } else {
    CHECK(p.off_G == 0 && p.off_Lp == 0);
  }
}

static void planner_sweep() {
  std::mt19937_64 rng(1234);
  int plans = 0;
  for (int it = 0; it < 4000; ++it) {
    const int o = 1 + static_cast<int>(rng() % 64);
    const int v = 1 + static_cast<int>(rng() % 700);
    const int P = 1 + static_cast<int>(rng() % 2500);
    const int precision = static_cast<int>(rng() % 4);
    const int backward = static_cast<int>(rng() % 2);
    const bool split = precision == CC_LADDER_SPLIT_BF16 || precision == CC_LADDER_SPLIT_INT8;
    cc_ladder_opts opts{};
    opts.flags = static_cast<unsigned>(rng() % 32);
    if (precision == CC_LADDER_SPLIT_INT8)
      opts.split_slices = (rng() % 3 == 0) ? 0 : 4 + static_cast<int>(rng() % 2);
    else
      opts.split_slices = (rng() % 3 == 0) ? 0 : 2 + static_cast<int>(rng() % 3);
    opts.split_depth = static_cast<int>(rng() % 3);
    opts.a_block = (rng() % 4 == 0) ? 1 + static_cast<int>(rng() % v) : 0;
    const size_t budget = (rng() % 5 == 0) ? 0 : (size_t(1) << (20 + rng() % 20));
    Plan p;
    const int rc = make_plan(o, v, P, precision, backward, budget, &opts, &p);
    const bool pm = (opts.flags & CC_LADDER_PLUS_MINUS) != 0;
    if ((opts.flags & (CC_LADDER_PLUS_MINUS | CC_LADDER_SYMMETRIC_VECTORS)) &&
        !(opts.flags & CC_LADDER_PAIR_SYMMETRIC)) {
      CHECK(rc == CC_LADDER_EINVAL);
      continue;
    }
    const int i8_slices = opts.split_slices ? opts.split_slices : 5;
    const int i8_depth = opts.split_depth ? opts.split_depth : 1;
    if ((split && backward) || (split && pm) ||
        (precision == CC_LADDER_SPLIT_INT8 && i8_slices + i8_depth - 1 > 5)) {
      CHECK(rc == CC_LADDER_EUNSUPPORTED);
      continue;
    }
    CHECK(rc == CC_LADDER_OK || rc == CC_LADDER_ENOMEM);
    if (rc) continue;
    ++plans;
    plan_invariants(p, backward, budget);
    // the footprint grows with the block size (the search relies on it); for
    // pair-balanced blocks it shrinks as their count grows
    if (p.balanced) {
      if (p.nblocks > 1) {
        Plan q;
        const int rc2 = layout_plan(o, v, P, precision, backward, 0, opts.split_slices,
                                    opts.split_depth, opts.k_chunk, opts.flags, &q, p.nblocks - 1);
        CHECK(rc2 == CC_LADDER_OK && q.bytes >= p.bytes);
      }
    } else if (p.n_a < v) {
      Plan q;
      const int rc2 = layout_plan(o, v, P, precision, backward, p.n_a + 1, opts.split_slices,
                                  opts.split_depth, opts.k_chunk, opts.flags, &q);
      CHECK(rc2 == CC_LADDER_OK && q.bytes >= p.bytes);
    }
  }
  CHECK(plans > 600);
  // occupied-index terms
  for (int it = 0; it < 2000; ++it) {
    const int which = static_cast<int>(rng() % 3);
    const int o = 1 + static_cast<int>(rng() % 80);
    const int v = 1 + static_cast<int>(rng() % 500);
    const int P = 1 + static_cast<int>(rng() % 2000);
    const int precision = static_cast<int>(rng() % 2);
    const size_t budget = (rng() % 4 == 0) ? 0 : (size_t(1) << (18 + rng() % 22));
    Plan p;
    const int rc = make_plan_intermediate(which, o, v, P, precision, budget, nullptr, &p);
    CHECK(rc == CC_LADDER_OK || rc == CC_LADDER_ENOMEM);
    if (!rc) {
      CHECK(p.bytes % 256 == 0 && (budget == 0 || p.bytes <= budget));
      CHECK(p.k_splits >= 1 && p.k_splits <= 16);
    }
  }
  Plan p;
  CHECK(make_plan_intermediate(3, 2, 2, 2, 0, 0, nullptr, &p) == CC_LADDER_EINVAL);
  CHECK(make_plan_intermediate(0, 2, 2, 2, 2, 0, nullptr, &p) == CC_LADDER_EUNSUPPORTED);
}

static void tiling_sweep() {
  std::mt19937_64 rng(99);
  for (int it = 0; it < 20000; ++it) {
    const long long M = 1 + static_cast<long long>(rng() % 20000);
    const long long N = 1 + static_cast<long long>(rng() % 400000);
    const bool tall = rng() % 2, split = rng() % 2;
    long long main_rows = -1;
    const int bm = choose_kc_tiling(M, N, tall, split, &main_rows);
    CHECK(bm == 128 || (bm == 160 && tall) || (bm == 64 && split));
    if (bm == 64)
      CHECK(main_rows > 0 && main_rows < M && main_rows % 128 == 0 && M - main_rows <= 64);
    else
      CHECK(main_rows == M);
    const int s = choose_k_splits(M, N, 1 + static_cast<long long>(rng() % 200000), 16);
    CHECK(s >= 1 && s <= 16);
  }
}

int main() {
  argument_checks();
  workspace_checks();
  planner_sweep();
  tiling_sweep();
  if (g_fail) {
    std::fprintf(stderr, "plan_check: %d failures\n", g_fail);
    return 1;
  }
  std::printf("plan_check OK\n");
  return 0;
}
