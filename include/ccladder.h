/*
 * ccladder.h -- C ABI of the MI355X (gfx950) particle-particle ladder library.
 *
 * The library evaluates the bottleneck term of the Cholesky-vector CCD/CCSD
 * doubles vector function of arXiv 2310.04559:
 *
 *   (ac|bd) = V[a,c,b,d] = sum_x L[x,a,c] L[x,b,d]          (eq. cholesky)
 *   R[i,j,a,b] += sum_{c,d} V[a,c,b,d] t[i,j,c,d]           (eq. vfunction)
 *
 * The four-index integral is never stored whole: it is rebuilt in blocks of
 * the first virtual index a (the paper's loop over one virtual index,
 * Sec. "tensordot", generalised to blocks sized to device memory as in
 * Sec. "CuPy and batch-wise computations").
 *
 * The same build-then-contract scheme gives the exchange partner of the
 * ladder (eq. vfunction2, an option flag) and the two occupied intermediates
 * that share one contraction pattern (eqs. vfunction3 and vfunction4), which
 * take the occupied-virtual block of the Cholesky vectors as well.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Tensor pointers are DEVICE pointers to float64, C-contiguous:
 *     L   [P][v][v]      virtual-virtual block of the Cholesky vectors
 *     t   [o][o][v][v]   t[i][j][c][d]
 *     R   [o][o][v][v]   R[i][j][a][b]
 *     L_ov [P][o][v]     occupied-virtual block of the Cholesky vectors, L_ov[x][k][c]
 *     L_oo [P][o][o]     occupied-occupied block of the Cholesky vectors, L_oo[x][i][k]
 *     X   [o][o][o][o]   X[i][j][k][l]  (eq. vfunction3)
 *     Y   [o][o][v][o]   Y[i][j][b][k]  (eq. vfunction4)
 *   The caller owns all of them; the library never frees caller memory.
 * - Results are ACCUMULATED (+=) into R, dL, dt, X and Y; zero them for the bare term.
 * - Calls enqueue work on `stream` (NULL = the legacy default stream) and
 *   return without a host synchronisation.  Kernel faults surface at the
 *   caller's next synchronisation of that stream.
 * - Return value: 0 on success, else one of the negative CC_LADDER_E* codes.
 *   Nothing throws across the ABI.  Argument, planning, device and scratch
 *   allocation errors are found before any kernel is enqueued: the outputs are
 *   then untouched.  A kernel launch the runtime rejects part-way (CC_LADDER_EHIP)
 *   can leave the outputs partly updated.
 * - Internal scratch: taken from opts->workspace when given, otherwise
 *   allocated with hipMallocAsync on `stream` and released with hipFreeAsync
 *   on the same stream before return.
 */
#ifndef CCLADDER_H
#define CCLADDER_H

#include <stddef.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Error codes. */
#define CC_LADDER_OK            0
#define CC_LADDER_EINVAL       -1   /* bad dimension, null/aliased pointer, unknown precision or option */
#define CC_LADDER_ENOMEM       -2   /* not even a one-virtual block fits the budget / workspace too small */
#define CC_LADDER_ENODEV       -3   /* no gfx950 device is current */
#define CC_LADDER_EHIP         -4   /* a HIP runtime call failed */
#define CC_LADDER_EUNSUPPORTED -5   /* valid request the library does not implement */

/* Arithmetic of the two contractions.  Sources and results are always float64. */
typedef enum {
  CC_LADDER_FP64 = 0,        /* float64 MFMA throughout */
  CC_LADDER_FP32 = 1,        /* float32 operands and MFMA, float32 partial sums drained to float64 */
  CC_LADDER_SPLIT_BF16 = 2,  /* operands cut into bf16 slices, slice products on bf16 MFMA, summed
                                in float32 over chunks of 256 indices (128 with 3 slices) and
                                drained to float64.
                                3 or 4 slices (default 4): digits on shared exponents (per row for
                                the integral build, per row and chunk for the contraction),
                                summed exactly, except that with 4 slices the products scaled
                                by 2^-16 or less share one rounded sum.
                                2 slices: the per-element split hi = bf16(x), lo = bf16(x - hi)
                                (round to nearest even) with the products hi*hi, hi*lo, lo*hi,
                                about 16 significant bits per operand */
  CC_LADDER_SPLIT_INT8 = 3   /* the digit scheme on the integer matrix cores: each operand row
                                gets an exponent per chunk of 16384 contracted indices and
                                every value S balanced int8 digits (default and most 5: 39 bits
                                below the chunk's maximum; 4 also accepted), digit products on
                                the int8 MFMA summed exactly in int32 over each chunk (products
                                (p,q) with p+q <= S+depth, 1-based; depth 1, the triangle of
                                S(S+1)/2 products, or 2 with 4 digits), drained to float64.
                                Forward only. */
} cc_ladder_precision;

/* opts.flags bits */
#define CC_LADDER_PAIR_SYMMETRIC 1u  /* caller asserts t[i][j][c][d] == t[j][i][d][c] (true of CC
                                        doubles amplitudes).  The integral then enters only through
                                        its rows (a,b) with a <= b, stored packed, and each result
                                        is added at both R[i][j][a][b] and R[j][i][b][a]: half the
                                        build and half the contraction.  Forward, every form.  In
                                        the adjoint the caller asserts that lam is pair-symmetric
                                        too; the two dL terms are then equal and one is computed
                                        and added twice (one product fewer of five). */

#define CC_LADDER_EXCHANGE 2u        /* evaluate the exchange partner instead (eq. vfunction2):
                                        R[i][j][a][b] += sum_{c,d} (ad|bc) t[i][j][c][d], i.e. the
                                        ladder of t with its last two indices swapped.  The swapped
                                        copy lives in scratch (o^2 v^2 float64; the FP32 form swaps
                                        into its float32 copy instead), and the adjoint accumulates
                                        dt in swapped order in another o^2 v^2 float64 buffer before
                                        swapping it back; the adjoint returns the exchange term's
                                        gradients.  Combines with PAIR_SYMMETRIC and every form. */

#define CC_LADDER_CHECK_SYMMETRY 4u  /* with PAIR_SYMMETRIC: verify the assertion before any other
                                        work.  A kernel compares t (and, in the adjoint, lam) with
                                        its pair transpose; the call then synchronises `stream` to
                                        read the result and returns CC_LADDER_EINVAL, with the
                                        outputs untouched, when some |x[i][j][c][d] - x[j][i][d][c]|
                                        exceeds 2^-40 max|x|.  Ignored without PAIR_SYMMETRIC. */

#define CC_LADDER_PLUS_MINUS 8u      /* with PAIR_SYMMETRIC, FP64 and FP32 forward: contract the
                                        symmetric and antisymmetric combinations of the integral
                                        with its exchange partner (eqs. vfunction and vfunction2;
                                        the permutational symmetry of the integrals, Sec. "The CC
                                        ansatz") instead of packed rows.  With t+[ij][cd] = t[i][j][c][d] + t[i][j][d][c]
                                        (c < d; t[i][j][c][c] for c = d), t-[ij][cd] = t[i][j][c][d]
                                        - t[i][j][d][c] (c < d) and the integrals
                                        V+-[ab][cd] = (ac|bd) +- (ad|bc), the sums
                                        R+[ij][ab] = R[i][j][a][b] + R[i][j][b][a] =
                                        sum_{c<=d} V+[ab][cd] t+[ij][cd] and R- (the same with -,
                                        over c < d) are symmetric (antisymmetric) in a,b and in
                                        i,j, so rows i <= j, columns a <= b and the contracted pairs
                                        c <= d suffice: a quarter of the general contraction (half of
                                        the packed-row form), the build as with PAIR_SYMMETRIC, plus
                                        one pass forming V+- from each built block.  R[i][j][a][b]
                                        = (R+ + R-)/2 and R[i][j][b][a] = (R+ - R-)/2, added with
                                        their (j,i) mirrors.  Holds for any Cholesky vectors (it
                                        uses (pq|rs) = (rs|pq) only).  EINVAL without
                                        PAIR_SYMMETRIC; EUNSUPPORTED in the split forms; the
                                        adjoint ignores it. */

#define CC_LADDER_SYMMETRIC_VECTORS 16u /* with PAIR_SYMMETRIC: the caller asserts L[x][a][c] ==
                                        L[x][c][a] (real orbitals give one symmetric Cholesky
                                        factor for both pair indices, Sec. "The CC ansatz",
                                        eq. cholesky).  The integral is then the symmetric matrix
                                        G[{a,c}][{b,d}] = sum_x L[x][a][c] L[x][b][d] over the
                                        v(v+1)/2 unordered pairs, built once per call over its
                                        upper triangle (the 8-fold permutational symmetry: a
                                        quarter of the packed build's flops), and each block's
                                        packed rows (a,b), a <= b (or, with PLUS_MINUS, its V+-)
                                        are gathered from it.  FP64 and FP32, forward and
                                        adjoint, and the split forwards (G in float64 from the
                                        digits of the packed vectors: split-int8 equal bit for
                                        bit to the packed build, split-bf16 up to the order of
                                        its rounded low-order sums).  G is kept whole in
                                        scratch, a square of v(v+1)/2 (rounded up to a multiple
                                        of 4) elements of the form's type (float64 for the split
                                        forms; 34 GB in float64 at v = 360)
                                        plus the packed vectors; when it does not fit the
                                        budget the flag changes nothing.  With CHECK_SYMMETRY, L
                                        is checked as well: EINVAL when some |L[x][a][c] -
                                        L[x][c][a]| exceeds 2^-40 max|L|.  EINVAL without
                                        PAIR_SYMMETRIC. */

/* Kernel phases reported to an optional trace hook. */
typedef enum {
  CC_LADDER_PHASE_PREP = 0,      /* operand conversion / slicing of L, t, lam; the exchange swaps
                                    (block 1: the adjoint's final swap of dt) */
  CC_LADDER_PHASE_BUILD = 1,     /* integral block V_A (eq. cholesky) */
  CC_LADDER_PHASE_CONTRACT = 2,  /* R += t . V_A (eq. vfunction) */
  CC_LADDER_PHASE_DT = 3,        /* adjoint: dt += lam . V_A */
  CC_LADDER_PHASE_W = 4,         /* adjoint: W_A = lam^T t */
  CC_LADDER_PHASE_DL = 5,        /* adjoint: both dL terms */
  CC_LADDER_PHASE_SLICE = 6      /* split-bf16: slicing of the integral block */
} cc_ladder_phase;

/* Called on the host right before (end = 0) and right after (end = 1) the
 * kernels of one phase of integral block `block` are enqueued on `stream`, so
 * the caller can record events there.  Must not call back into the library. */
typedef void (*cc_ladder_trace_fn)(void* user, int phase, int block, int end, hipStream_t stream);

/* Optional controls; a zero-initialised struct (or NULL) selects everything automatically. */
typedef struct {
  int    a_block;          /* virtuals per integral block; 0 = largest that fits hbm_budget */
  int    split_slices;     /* SPLIT_BF16 slices S in [2, 4]; 0 = 4 (2 = the hi/lo split);
                              SPLIT_INT8 digits in [4, 5]; 0 = 5 */
  int    k_chunk;          /* FP32 drain interval along the contracted index (multiple of 64); 0 = 512 */
  int    split_depth;      /* SPLIT_BF16 slice products (p,q), 1-based, kept when p+q <= S+depth,
                              depth in [1, 2]; 0 = 2 for S = 4 (13 products), 1 otherwise
                              (S = 2: hi*hi, hi*lo, lo*hi; S = 3: 6 products) */
  size_t hbm_budget;       /* bytes the library may use for scratch; 0 = half the free device
                              memory, at most 128 GiB */
  void*  workspace;        /* caller scratch (device, 256-byte aligned) or NULL; the part the
                              plan uses, [workspace, workspace + planned bytes), must not
                              overlap any tensor argument (CC_LADDER_EINVAL) */
  size_t workspace_bytes;  /* its size; the plan must fit in it */
  cc_ladder_trace_fn trace;  /* optional per-phase hook, NULL = none */
  void*  trace_user;       /* passed back to `trace` */
  unsigned flags;          /* CC_LADDER_PAIR_SYMMETRIC | CC_LADDER_EXCHANGE |
                              CC_LADDER_CHECK_SYMMETRY | CC_LADDER_PLUS_MINUS |
                              CC_LADDER_SYMMETRIC_VECTORS, or 0 */
  int    reserved;         /* must be 0 */
} cc_ladder_opts;

/*
 * Ladder term (eq. vfunction with eq. cholesky):
 *   R[i][j][a][b] += sum_{c,d} ( sum_x L[x][a][c] L[x][b][d] ) t[i][j][c][d]
 * o, v, P > 0.  R must not overlap L or t.
 */
int cc_ladder_residual(int o, int v, int P,
                       const double* L, const double* t, double* R,
                       int precision, hipStream_t stream, const cc_ladder_opts* opts);

/* Size of the static scratch of cc_ladder_residual_noalloc (bytes per device). */
#define CC_LADDER_NOALLOC_SCRATCH_BYTES (256ull << 20)

/*
 * cc_ladder_residual for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation.  Same arguments, result and kernels as cc_ladder_residual, but
 * the scratch is a static device array of CC_LADDER_NOALLOC_SCRATCH_BYTES
 * (256 MiB) that every device the library runs on holds until the process
 * ends; the call makes no hipMalloc/hipFree and no other allocating call.
 * Its device address is looked up once per device, on the first call there.
 * - The plan is sized to that array (or to opts->hbm_budget when smaller):
 *   CC_LADDER_ENOMEM when not even a one-virtual block fits it (for float64,
 *   v^3 * 8 bytes must be below 256 MiB, i.e. v <= 322; query beforehand with
 *   cc_ladder_workspace_query(..., hbm_budget = CC_LADDER_NOALLOC_SCRATCH_BYTES)).
 * - opts->workspace must be NULL and workspace_bytes 0, and the
 *   CC_LADDER_CHECK_SYMMETRY flag (which reads a result back to the host) is
 *   not accepted: CC_LADDER_EINVAL.
 * - Every call on one device shares that device's array and leaves its
 *   contents behind; each call rewrites what it reads, so no state carries
 *   over.  Calls that overlap in time on one device (different streams, or
 *   host threads enqueueing concurrently) race on the array: serialise them.
 */
int cc_ladder_residual_noalloc(int o, int v, int P,
                               const double* L, const double* t, double* R,
                               int precision, hipStream_t stream, const cc_ladder_opts* opts);

/*
 * Adjoint of the ladder term for Loss = sum lam[i][j][a][b] R[i][j][a][b]
 * (lam = dLoss/dR, any values, pair symmetry not assumed):
 *   dt[i][j][c][d] += sum_{a,b} lam[i][j][a][b] V[a,c,b,d]
 *   dL[x][p][q]    += sum_{b,d} W[p,b,q,d] L[x][b][d] + sum_{a,c} W[a,p,c,q] L[x][a][c]
 *   with W[a,b,c,d] = sum_{i,j} lam[i][j][a][b] t[i][j][c][d].
 * dL is the entrywise gradient (each entry of L independent).  Integral
 * blocks are rebuilt, not stored.  dL/dt must not overlap any input.
 */
int cc_ladder_backward(int o, int v, int P,
                       const double* L, const double* t, const double* lam,
                       double* dL, double* dt,
                       int precision, hipStream_t stream, const cc_ladder_opts* opts);

/*
 * float64 reductions over n = o*o*v*v entries: the energy-like functional and
 * the residual norm that a CC iteration evaluates once per vector function (the
 * per-iteration quantities of the paper's timings, Table tbl:dye):
 *   out_dev[0] = sum x*y,  out_dev[1] = sum y*y        (out_dev: device, 2 doubles)
 * x, y: device [o][o][v][v] float64.  out_dev must not overlap x or y
 * (CC_LADDER_EINVAL).  Deterministic for a given device and size.  Scratch for
 * the partial sums (16 KB) is allocated and freed stream-ordered.
 */
int cc_ladder_reduce(int o, int v, const double* x, const double* y, double* out_dev,
                     hipStream_t stream);

/*
 * Host-only planner query (needs no device): the scratch bytes and the
 * integral block (virtuals per block) that cc_ladder_residual (backward = 0)
 * or cc_ladder_backward (backward = 1) would use under `hbm_budget` bytes
 * (0 = no limit, i.e. the whole virtual range in one block).  This is the
 * paper's memory-fit rule for its batches (Sec. "CuPy and batch-wise
 * computations": element counts times element sizes, blocks shrunk until they
 * fit), applied to device-resident data.  `opts` may be NULL; every field that
 * shapes the plan is honoured (a_block, split_slices, split_depth, k_chunk,
 * flags), its budget and workspace fields are not.  *bytes and *a_block are
 * written on success only.
 */
int cc_ladder_workspace_query(int o, int v, int P, int precision, int backward,
                              size_t hbm_budget, const cc_ladder_opts* opts,
                              size_t* bytes, int* a_block);

/* Which occupied-index term (planner query): the intermediates of eqs.
 * vfunction3 and vfunction4, and the hole-hole ladder. */
typedef enum {
  CC_INTERMEDIATE_IJKL = 0,  /* X[i][j][k][l] += sum_{c,d} (kc|ld) t[i][j][c][d] */
  CC_INTERMEDIATE_IJBK = 1,  /* Y[i][j][b][k] += sum_{c,d} (bd|kc) t[i][j][c][d] */
  CC_HOLE_LADDER = 2         /* R[i][j][a][b] += sum_{k,l} (ik|jl) t[k][l][a][b] */
} cc_intermediate_kind;

/*
 * Occupied-occupied intermediate (eq. vfunction3):
 *   X[i][j][k][l] += sum_{c,d} ( sum_x L_ov[x][k][c] L_ov[x][l][d] ) t[i][j][c][d]
 * The integrals (kc|ld) are rebuilt for blocks of the occupied index k
 * (opts->a_block counts occupied indices here).  FP64 and FP32 forms;
 * SPLIT_BF16 and every opts->flags bit return CC_LADDER_EUNSUPPORTED.
 * o, v, P > 0.  X must not overlap L_ov or t.
 */
int cc_intermediate_ijkl(int o, int v, int P,
                         const double* L_ov, const double* t, double* X,
                         int precision, hipStream_t stream, const cc_ladder_opts* opts);

/*
 * Intermediate with one virtual and one occupied output index (eq. vfunction4):
 *   Y[i][j][b][k] += sum_{c,d} ( sum_x L[x][b][d] L_ov[x][k][c] ) t[i][j][c][d]
 * The integrals (bd|kc) are rebuilt for blocks of the virtual index b; the
 * amplitudes are met with c and d swapped (a copy in scratch, or inside the
 * FP32 form's float32 copy).  Forms and flags as cc_intermediate_ijkl.
 * Y must not overlap L, L_ov or t.
 */
int cc_intermediate_ijbk(int o, int v, int P,
                         const double* L, const double* L_ov, const double* t, double* Y,
                         int precision, hipStream_t stream, const cc_ladder_opts* opts);

/*
 * Hole-hole ladder, the o^4 v^2 term the paper's pCCD-LCCSD vector function
 * offloads beside the ladder (Sec. "Comparison between CPU and
 * GPU-accelerated implementations"; the paper gives its contraction pattern,
 * whose Cholesky operand expands as for eq. cholesky):
 *   R[i][j][a][b] += sum_{k,l} ( sum_x L_oo[x][i][k] L_oo[x][j][l] ) t[k][l][a][b]
 * The integrals (ik|jl) are rebuilt for blocks of the occupied index i
 * (opts->a_block counts occupied indices).  Forms and flags as
 * cc_intermediate_ijkl.  R must not overlap L_oo or t.
 */
int cc_hole_ladder(int o, int v, int P,
                   const double* L_oo, const double* t, double* R,
                   int precision, hipStream_t stream, const cc_ladder_opts* opts);

/*
 * Host-only planner query for the occupied-index terms (`which` a cc_intermediate_kind):
 * scratch bytes and first indices per integral block under `hbm_budget`
 * (0 = no limit), as cc_ladder_workspace_query.
 */
int cc_intermediate_workspace_query(int which, int o, int v, int P, int precision,
                                    size_t hbm_budget, const cc_ladder_opts* opts,
                                    size_t* bytes, int* block);

/* Static description of an error code (never NULL). */
const char* cc_ladder_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* CCLADDER_H */
