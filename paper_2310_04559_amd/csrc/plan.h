// Host-side planning of the virtual-index blocking (no device calls).
//
// The integral V[a,c,b,d] is rebuilt for a block of n_a first-virtual indices
// at a time.  Like the paper's batch-wise scheme (Sec. "CuPy and batch-wise
// computations"), the element counts of every buffer are multiplied by their
// element sizes and the block is shrunk until everything fits the budget;
// here the inputs are already resident, so only the scratch is planned.
#pragma once
#include <cstddef>

#include "ccladder.h"

namespace ccl {

// Operation a plan is made for.
enum { kOpLadder = 0, kOpIjkl = 1, kOpIjbk = 2, kOpHole = 3 };

// Scratch buffers of one call, as byte offsets into a single workspace.
struct Plan {
  int op = kOpLadder;
  int o = 0, v = 0, P = 0;
  int precision = 0;
  int backward = 0;
  int n_a = 0;          // first indices per integral block (virtuals; occupied for ijkl)
  int nblocks = 0;      // ceil(v / n_a) (ceil(o / n_a) for ijkl)
  int slices = 0;       // split-bf16 slice count (0 for the other forms)
  int split_depth = 0;  // split-bf16 anti-diagonals kept beyond the slice triangle (1 or 2)
  int pairsym = 0;      // forward over packed integral rows a <= b (pair-symmetric amplitudes)
  int pairsym_adj = 0;  // adjoint with pair-symmetric t and lam: packed integral rows for dt,
                        // one dL term added twice
  size_t off_lamP = 0;  // pair-symmetric adjoint: lam at the block's packed pairs, weighted
  size_t off_B = 0;     // pair-symmetric adjoint: float64 B[(ij)][(cd)], dt += B + mirror(B)
  int check_sym = 0;    // verify the pair-symmetry assertion before any other work
  size_t off_check = 0; // its result: max |x - pair transpose of x|, max |x| (as uint64 bits)
  int exchange = 0;     // exchange partner: amplitudes (and dt) with c,d swapped
  size_t off_tx = 0;    // exchange: t with its last two indices swapped (float64; not in FP32)
  size_t off_dtx = 0;   // exchange adjoint: dt of the swapped amplitudes (float64)
  int pm = 0;           // forward over the symmetric/antisymmetric combinations (PLUS_MINUS)
  long long ldp = 0, ldm = 0;  // PLUS_MINUS: row strides of the c <= d and c < d operands
  size_t off_Tp = 0, off_Tm = 0;  // PLUS_MINUS: t+ [o(o+1)/2][ldp], t- [o(o-1)/2][ldm]
  size_t off_Vp = 0, off_Vm = 0;  // PLUS_MINUS: V+ [pairs a <= b][ldp], V- [pairs a < b][ldm]
  int gsym = 0;         // PLUS_MINUS with symmetric vectors: whole pair-pair integral G
  long long ldg = 0;    // its side: v(v+1)/2 rounded up to a multiple of 4
  size_t off_Lp = 0;    // packed vectors Lp[x][pair(a,c)], a <= c ([P][ldg], pads zero)
  size_t off_G = 0;     // G[ldg][ldg], symmetric
  int k_chunk = 0;      // float32 drain interval along the contracted index
  // operand copies made once per call (float32 / bf16 slice forms)
  size_t off_L = 0, off_t = 0, off_lam = 0;
  size_t off_L2 = 0;    // intermediate ijbk, FP32: the virtual-virtual vectors (off_L: L_ov)
  int k_splits = 1;     // intermediates: K ranges of the contraction (split K when its tile
                        // grid alone leaves compute units idle)
  size_t off_part = 0;  // float64 partials of the split contraction [k_splits][o^2][n_a*o]
  size_t off_Lexp = 0, off_texp = 0;
  // per-block buffers
  size_t off_V = 0;     // float64 or float32 integral block [n_a][v][v][v] (or packed rows)
  size_t off_W = 0;     // adjoint block W'[n_a][v][v][v] (backward)
  size_t off_Vs = 0;    // bf16 slices of the integral block
  size_t off_Vexp = 0;  // exponents of the integral block's digit rows, per (row, chunk)
  size_t off_tiles = 0; // packed build: first tile of every tile row (int32, tiles_m + 1)
  int balanced = 0;     // packed forward: nblocks blocks of about equal pair counts (n_a is
                        // then the widest block's virtual count)
  long long npk = 0;    // packed forward: packed rows (a,b) of the block that has the most
  size_t bytes = 0;     // total scratch
};

// Fills `plan` for a block size of n_a (1 <= n_a <= v), or, when nb > 0 and the
// plan is a packed (pair-symmetric) forward, for nb pair-balanced blocks (n_a
// ignored).  Returns 0, CC_LADDER_EINVAL or CC_LADDER_EUNSUPPORTED.
int layout_plan(int o, int v, int P, int precision, int backward, int n_a,
                int slices, int depth, int k_chunk, unsigned flags, Plan* plan, int nb = 0);

// Packed integral rows (a,b), a <= b, ordered by a then b: rows of virtuals
// [0, a) come first.  pair_prefix(a, v) = sum_{a' < a} (v - a').
inline long long pair_prefix(long long a, long long v) { return a * v - a * (a - 1) / 2; }

// First virtual of block k of nb blocks with about equal pair counts: the
// smallest a with pair_prefix(a, v) * nb >= k * v(v+1)/2 (0 for k = 0, v for k = nb).
int pair_block_start(int v, int nb, int k);

// Virtual range [*a0, *a0 + *na) of block `blk` of a plan: equal virtual
// counts (n_a, the last block the remainder), or equal pair counts for a
// balanced plan.  *na may be 0 for a balanced plan (an empty block).
void block_range(const Plan& pl, int blk, int* a0, int* na);

// Picks n_a (honouring opts->a_block when set) so that plan.bytes <= budget
// (budget 0 = unlimited).  Returns 0, CC_LADDER_EINVAL or CC_LADDER_ENOMEM.
int make_plan(int o, int v, int P, int precision, int backward, size_t budget,
              const cc_ladder_opts* opts, Plan* plan);

// The occupied intermediates (eqs. vfunction3/vfunction4) and the hole-hole
// ladder: blocks of n_p first indices (occupied k for ijkl, virtual b for ijbk,
// occupied i for the hole-hole ladder), integral block [n_p][o][v][v]
// ([n_p][o][o][o] for the hole-hole ladder).  Same search and return codes as
// make_plan; flags are CC_LADDER_EUNSUPPORTED, SPLIT_BF16 too.
// Tiling of the K-contiguous product C[M][N] (tiles 256 columns wide) that
// finishes first on the device's compute units: 128-row tiles; 160-row tiles
// (when `tall` is allowed); or 128-row tiles over the first *main_rows rows and
// one launch of 64-row tiles over the rest (when `split` is allowed and the
// last 128-row tile row would be at most half full).  Returns 128, 160 or 64
// (the split); *main_rows is M unless split.
int choose_kc_tiling(long long M, long long N, bool tall, bool split, long long* main_rows);

// K ranges for a K-contiguous product of M x N (tiles of 128 x 256) over K
// elements in steps of `bk`: 1 when the tiles fill the chip, otherwise the count
// that minimises the waves per unit of work (at least 64 K-steps per range).
int choose_k_splits(long long M, long long N, long long K, int bk);

int layout_intermediate(int which, int o, int v, int P, int precision, int n_p, int k_chunk,
                        Plan* plan);
int make_plan_intermediate(int which, int o, int v, int P, int precision, size_t budget,
                           const cc_ladder_opts* opts, Plan* plan);

// Forwards phase boundaries to the caller's optional trace hook.
struct Tracer {
  cc_ladder_trace_fn fn = nullptr;
  void* user = nullptr;
  hipStream_t stream = nullptr;
  Tracer(const cc_ladder_opts* o, hipStream_t s)
      : fn(o ? o->trace : nullptr), user(o ? o->trace_user : nullptr), stream(s) {}
  void operator()(int phase, int block, int end) const {
    if (fn) fn(user, phase, block, end, stream);
  }
};

// Argument checks shared by every entry point (dimensions, precision, options).
int check_dims(int o, int v, int P);
int check_precision_opts(int precision, const cc_ladder_opts* opts);

// One array argument of a call: its first byte and its size in bytes.
struct Operand {
  const void* p;
  size_t bytes;
};

// True when [a, a + abytes) and [b, b + bbytes) share a byte.
bool overlaps(const void* a, size_t abytes, const void* b, size_t bbytes);

// Host-only argument validation of the ladder entry points, in the order the
// entry points apply it: dimensions, precision and options, null pointers, then
// outputs overlapping inputs (or each other).  Returns 0 or CC_LADDER_EINVAL.
// The array sizes these checks use are filled into ops[] (inputs then outputs:
// forward L, t, R; adjoint L, t, lam, dL, dt) for the workspace check below.
int check_residual_args(int o, int v, int P, const double* L, const double* t, const double* R,
                        int precision, const cc_ladder_opts* opts, Operand ops[3]);
int check_backward_args(int o, int v, int P, const double* L, const double* t, const double* lam,
                        const double* dL, const double* dt, int precision,
                        const cc_ladder_opts* opts, Operand ops[5]);

// A caller workspace must not overlap any array of the call over the bytes the
// plan uses: CC_LADDER_EINVAL when [workspace, workspace + plan_bytes) meets
// ops[i] for some i < n, else 0 (also when there is no caller workspace).
int check_workspace(const cc_ladder_opts* opts, size_t plan_bytes, const Operand* ops, int n);

// The ladder forward once its plan is made and its scratch (`base`, at least
// pl.bytes, 256-byte aligned) is settled: the optional pair-symmetry check,
// operand preparation and the block loop, enqueued on `stream`.
int ladder_forward_planned(const Plan& pl, const double* L, const double* t, double* R,
                           int precision, char* base, const cc_ladder_opts* opts,
                           hipStream_t stream);

// CC_LADDER_OK when the current device is a gfx950, else CC_LADDER_ENODEV.
int device_ok();

}  // namespace ccl
