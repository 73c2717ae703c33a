/*
 * fftc -- batched one-dimensional complex FFTs on AMD Instinct MI355X (gfx950).
 *
 * The operation (paper, Section II): for each transform of length N,
 *     y = DFT_N x,   DFT_N[m, n] = w_N^{m n},   w_N = exp(-2 pi i / N),
 * computed by the Cooley-Tukey factorisation of Eq. 2,
 *     DFT_N = (DFT_K (x) I_M) D^N_M (I_K (x) DFT_M) Pi^N_K,   N = M K,
 * applied recursively in Stockham order (no separate bit-reversal pass).
 * The inverse direction uses w_N^{-1} and is not scaled (inverse(forward(x))
 * = N x); the paper defines only the forward transform.
 *
 * Conventions shared by every entry point:
 *  - Layout: interleaved complex (re, im), transforms contiguous and
 *    batch-major: element (b, j) of a plan with length N is at index b N + j.
 *    complex64 = two floats (8 bytes, 8-byte aligned), complex128 = two
 *    doubles (16 bytes, 16-byte aligned).
 *  - Device pointers are HIP device allocations on the current device; the
 *    caller owns them.  `stream` is a hipStream_t passed as void* (NULL = the
 *    default stream).
 *  - Every call returns an fftc_status; no call aborts, exits or throws.
 *    A non-OK status leaves a human-readable message for the calling thread
 *    in fftc_last_error().
 *  - Supported lengths: 1 <= N <= 2^20 whose prime factors are all <= 7.
 */
#ifndef FFTC_H
#define FFTC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FFTC_OK = 0,
    FFTC_ERR_INVALID_ARG = 1,      /* null / misaligned pointer, bad enum, batch < 1 ... */
    FFTC_ERR_UNSUPPORTED_SIZE = 2, /* N < 1, N > 2^20, or a prime factor > 7 */
    FFTC_ERR_OUT_OF_MEMORY = 3,    /* a device or host allocation failed */
    FFTC_ERR_TOO_LARGE = 4,        /* request larger than the server's memory budget */
    FFTC_ERR_HIP = 5,              /* a HIP runtime call failed (text in fftc_last_error) */
    FFTC_ERR_SHUTDOWN = 6,         /* server not running / stopped before completion */
    FFTC_ERR_INTERNAL = 7
} fftc_status;

/* Sign of the exponent. */
enum { FFTC_FORWARD = -1, FFTC_INVERSE = +1 };

/* Element type and arithmetic of a plan. */
enum {
    FFTC_C64 = 0,  /* complex64 in and out, fp32 arithmetic, twiddles made in fp64 */
    FFTC_C128 = 1, /* complex128 in and out, fp64 arithmetic */
    /* complex64 in and out; every DFT_16 stage is a dense 16 x 16 complex
     * product on the matrix cores with split low-precision operands and fp32
     * accumulation (x = x_hi + 2^-s x_lo, products hi*hi + 2^-s (hi*lo +
     * lo*hi)); twiddles and any radix-2/4/8 stage in fp32.  Lengths 256,
     * 512, 1024, 2048, 4096, 8192, 16384.  Intermediate values must stay
     * within the fp16 range for the fp16 modes (|y| < 65504). */
    FFTC_C64_SPLIT_F16 = 2,   /* fp16 hi + lo, s = 11 */
    FFTC_C64_SPLIT_BF16 = 3,  /* bf16 hi + lo, s = 8 */
    FFTC_C64_SPLIT3_BF16 = 4, /* bf16 hi + mid + lo, three-term products */
    FFTC_C64_F16 = 5          /* fp16 operands without split (reference) */
};

/* Plan variants reported by fftc_plan_describe. */
enum {
    FFTC_VARIANT_SINGLE_SPECIALISED = 0, /* one kernel compiled for this N and radix list */
    FFTC_VARIANT_SINGLE_GENERIC = 1,     /* one kernel, runtime N and radix list */
    FFTC_VARIANT_TWO_PASS = 2,           /* Eq. 2 four-step in two kernels + scratch */
    FFTC_VARIANT_MIXED_PERSISTENT = 3,   /* mixed lengths, one persistent launch in a hipGraph */
    FFTC_VARIANT_SPLIT_MFMA = 4,         /* DFT_16 stages on the matrix cores (split precision) */
    FFTC_VARIANT_FORMULA = 5,            /* a Kronecker-product formula (fftc_plan_formula) */
    FFTC_VARIANT_ORDER = 6               /* an alternative factorisation order (fftc_plan_order) */
};

typedef struct fftc_plan_s *fftc_plan_t;

/*
 * Create a plan for `batch` transforms of length `n`.
 *   direction: FFTC_FORWARD or FFTC_INVERSE;  dtype: one of FFTC_C64,
 *   FFTC_C128 or the split-precision complex64 modes above.
 * The radix list comes from the tuning database when it holds an entry for
 * (n, dtype), else from the built-in heuristic.  Allocates the plan's twiddle
 * tables (generated in fp64 on the GPU of the current device) and, for
 * two-pass plans, its scratch buffer; synchronises once before returning.
 * On success *plan_out owns these until fftc_destroy_plan.
 */
fftc_status fftc_plan(int64_t n, int64_t batch, int direction, int dtype, fftc_plan_t *plan_out);

/*
 * As fftc_plan with an explicit Stockham radix list r[0..count) whose
 * product is n; every radix must be one of 2, 3, 4, 5, 7, 8, 16.  Only
 * single-kernel lengths (see fftc_max_single_n) are accepted; for the wide
 * lengths only their compiled lists (fftc_compiled_entry).
 */
fftc_status fftc_plan_radices(int64_t n, int64_t batch, int direction, int dtype,
                              const int *radices, int count, fftc_plan_t *plan_out);

/*
 * Enqueue the plan's transforms on `stream`: in and out are device arrays of
 * batch * n elements.  in == out (in place) is allowed; other overlaps are
 * not.  Asynchronous: returns after the launch.  A plan may be executed on
 * several streams at once, except a two-pass plan, whose calls must be
 * ordered (they share the plan's scratch).
 */
fftc_status fftc_execute(fftc_plan_t plan, const void *in, void *out, void *stream);

/* As fftc_execute for the first `batch` transforms only (1 <= batch <= the
 * plan's batch); in and out hold batch * n elements.  Not for mixed plans. */
fftc_status fftc_execute_batch(fftc_plan_t plan, const void *in, void *out, int64_t batch, void *stream);

/*
 * For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc): plan and
 * run `batch` transforms of length n in one call, as fftc_plan (without a
 * recorded alternative order or an explicit radix list) followed by
 * fftc_execute, with no hipMalloc, hipFree or other device allocation.
 *   dtype: FFTC_C64 or FFTC_C128 only; n, batch, direction, in, out, stream
 *   as for fftc_plan / fftc_execute (in == out allowed, other overlaps not).
 * The twiddle tables (made in fp64 on the GPU by a kernel enqueued on
 * `stream`) and, for an in-place call of a two-pass length, the intermediate
 * live in one static device array of fftc_static_scratch_bytes() bytes (64
 * MiB) that each GPU the library runs on holds until the process ends: 2 MiB
 * for tables, the rest for the intermediate, which an in-place call fills a
 * chunk of transforms at a time.  Lengths whose tables exceed 2 MiB give
 * FFTC_ERR_TOO_LARGE (none of the supported lengths does).  Asynchronous;
 * results equal fftc_plan + fftc_execute's bit for bit.  Every call on one
 * GPU shares that GPU's array: calls that overlap in time on one GPU (other
 * streams, other threads) race and give wrong results; calls ordered on one
 * stream are safe.
 */
fftc_status fftc_execute_static(int64_t n, int64_t batch, int direction, int dtype, const void *in, void *out,
                                void *stream);

/* Size in bytes of fftc_execute_static's static device array. */
size_t fftc_static_scratch_bytes(void);

/* ---------------------------------------------------------------------------
 * Data layouts (planar and strided).  The DSL of the paper's Section IV-A
 * builds its complex input from separate real and imaginary arrays
 * (createComplex of Listing 1); libraries also transform data that is not
 * contiguous.  A layout says where element j of transform b is:
 *     interleaved:  ptr[b dist + j stride]            (complex elements)
 *     planar:       re[b dist + j stride], im[b dist + j stride]   (reals)
 * stride >= 1, dist >= 1, in elements.  The transforms of a layout must not
 * share elements: either dist >= (n - 1) stride + 1 (one block per
 * transform) or stride >= batch dist (transforms interleaved element by
 * element, e.g. the columns of a row-major array).  The layout is applied in
 * the first stage's loads and the last stage's stores of the same Stockham
 * kernels (no extra pass over HBM).
 * ------------------------------------------------------------------------- */
typedef struct {
    int64_t stride;  /* elements between consecutive points of one transform */
    int64_t dist;    /* elements between the first points of consecutive transforms */
    int planar;      /* 0: interleaved complex; 1: separate real and imaginary arrays */
} fftc_layout;

/*
 * Plan for `batch` transforms of length n reading the `in` layout and
 * writing the `out` layout (NULL = interleaved, stride 1, dist n).
 * complex64 or complex128, single-kernel lengths (fftc_max_single_n) that
 * have a compiled kernel (every length of fftc_compiled_entry).  Column-like
 * layouts (dist < stride on either side) of lengths above 2048 (complex64)
 * or 1024 (complex128), and of any 7-smooth length n = m k up to 2^20 with
 * both factors <= 1024 compiled as two-pass column lengths, run as two
 * passes of Eq. 2 through a plan-owned scratch buffer of batch * n elements
 * (executions of such a plan must be ordered); other layout plans allocate
 * only their twiddles.  UNSUPPORTED_SIZE otherwise, INVALID_ARG for a bad or
 * self-overlapping layout.
 */
fftc_status fftc_plan_layout(int64_t n, int64_t batch, int direction, int dtype, const fftc_layout *in,
                             const fftc_layout *out, fftc_plan_t *plan_out);

/*
 * Execute a layout plan.  Interleaved sides pass the complex array as *_re
 * and NULL as *_im; planar sides pass both arrays (each aligned to its real
 * type).  In place is allowed when both layouts are equal and the pointers
 * are the same; other overlaps are not.  fftc_execute also runs layout plans
 * whose two sides are interleaved.
 */
fftc_status fftc_execute_layout(fftc_plan_t plan, const void *in_re, const void *in_im, void *out_re,
                                void *out_im, void *stream);

/* Free the plan's device memory.  NULL is a no-op.  The caller must ensure
 * no execution of the plan is still in flight. */
fftc_status fftc_destroy_plan(fftc_plan_t plan);

/* What a plan runs.  radices[] holds the Stockham radix list (for two-pass
 * plans: the list of the first pass, then of the second). */
typedef struct {
    int64_t n, batch;
    int direction, dtype;
    int variant;          /* FFTC_VARIANT_* */
    int nradices;
    int radices[16];
    int threads_per_transform;
    int transforms_per_group;
    int64_t split_m, split_k;  /* two-pass: n = m k; else 0 */
    size_t twiddle_bytes, scratch_bytes;
    /* mixed plans: transforms, total elements, distinct lengths, work items,
     * persistent workgroups */
    int64_t mixed_transforms, mixed_elements;
    int mixed_classes, mixed_items, persistent_groups;
    /* formula plans: passes after lowering (0 when folded), 1 if the formula
     * folded to I(p) (x) DFT(n) and runs as p batched transforms of the
     * ordinary plan for n (then fold_n, fold_p), 1 if all passes run in one
     * LDS-resident kernel, kernels launched per execution (0 when folded) */
    int formula_passes, formula_folded, formula_lds;
    int64_t formula_fold_n, formula_fold_p;
    int formula_kernels;
    /* layout plans: the in and out layouts (interleaved contiguous otherwise) */
    int has_layout;
    fftc_layout layout_in, layout_out;
    /* order plans: FFTC_ORDER_* and the radix */
    int order, order_radix;
} fftc_plan_desc;

fftc_status fftc_plan_describe(fftc_plan_t plan, fftc_plan_desc *desc);

/* ---------------------------------------------------------------------------
 * Formula plans (Section IV-A: the DSL of Listing 1, grammar of Listing 2).
 * A formula is a text such as
 *     (DFT(2) (x) I(2)) . twiddle(4,2) . (I(2) (x) DFT(2)) . Permute(4,2)
 * built from DFT(n), I(n), twiddle(N, M) = D^N_M and Permute(N, K) = Pi^N_K
 * of Eq. 2, with (Pi^N_K x)[i M + j] = x[j K + i] (M = N / K) and D^N_M the
 * diagonal w_N^{i j} at position i M + j.  Kronecker product: U+2297, "(x)"
 * or "kron"; matrix product: U+00B7, ".", "*" or "@"; both group to the right at
 * equal precedence (parentheses as needed); keywords are case-insensitive; a
 * trailing identifier after a final product (the vector operand) is ignored.
 * Sizes obey the shape rule (a Kronecker product multiplies them, a matrix
 * product needs equal ones) and the whole formula is at most 2^24.
 *
 * The plan applies the formula's matrix F to `batch` contiguous vectors of
 * length dim (batch * dim < 2^31): y = F x for FFTC_FORWARD and
 * y = conj(F) x (for a DFT formula: the unscaled inverse) for FFTC_INVERSE.
 * dtype: FFTC_C64 or FFTC_C128.  Unless FFTC_FORMULA_NO_FOLD is given, every
 * four-factor window equal to Eq. 2 (or its transpose) folds back to DFT(N),
 * and a formula that folds to I(p) (x) DFT(n) runs as the ordinary plan of
 * n with p times the batch.  Everything else lowers to passes: DFT codelets,
 * Stockham stages (or with FFTC_FORMULA_EQ2 the Eq. 2 factors themselves),
 * direct sums for DFT sizes with prime factors > 7 (each such factor at most
 * 16384), diagonals and permutations; with vectors of at most
 * fftc_formula_max_lds_dim(dtype) elements they run in one kernel.  Longer
 * vectors run in as few kernels as the passes allow: consecutive passes
 * I_p (x) E (x) I_q whose common factors P0 | p, Q0 | q leave sub-vectors of
 * dim / (P0 Q0) <= that limit run together in LDS; a pass that touches more
 * elements runs alone over HBM.  FFTC_FORMULA_HBM_PASSES runs every pass as
 * its own HBM kernel.  Plans of more than one kernel own a scratch buffer
 * of batch * dim elements (their executions must be ordered).  INVALID_ARG for a syntax or shape error or bad flags,
 * UNSUPPORTED_SIZE when a factor cannot be lowered; the message names the
 * place.
 * ------------------------------------------------------------------------- */
enum {
    FFTC_FORMULA_NO_FOLD = 1,    /* keep the formula's own factors (no Eq. 2 folding) */
    FFTC_FORMULA_EQ2 = 2,        /* DFT(n) factors lower to Eq. 2 (Pi, D, smaller DFTs) */
    FFTC_FORMULA_HBM_PASSES = 4  /* one kernel per pass even when a vector fits LDS */
};

fftc_status fftc_plan_formula(const char *formula, int64_t batch, int direction, int dtype, int flags,
                              fftc_plan_t *plan_out);

/* Host-only: check and lower a formula without a GPU.  *dim = its size;
 * text (capacity text_len, may be NULL) receives the folded formula and the
 * pass list, one line each, NUL-terminated and truncated to fit. */
fftc_status fftc_formula_lower(const char *formula, int flags, int dtype, int64_t *dim, char *text,
                               size_t text_len);

/* Largest vector length a formula plan runs in one LDS-resident kernel. */
int64_t fftc_formula_max_lds_dim(int dtype);

/*
 * Host-only: the radix list fftc_plan would choose for (n, dtype), without a
 * GPU.  Writes at most max_count radices and the count.  For two-pass
 * lengths, the list covers the first pass then the second (see split_m).
 */
fftc_status fftc_factorize(int64_t n, int dtype, int *radices, int max_count, int *count,
                           int64_t *split_m);

/*
 * Host-only: the candidate Stockham radix lists for single-kernel length n,
 * in the planner's preference order (the autotuner times these; for a wide
 * length it times the compiled lists instead).  List i is
 * radices[i * 16 .. i * 16 + lens[i]); at most max_lists lists are written,
 * *nlists is how many there are (up to 12).
 */
fftc_status fftc_candidates(int64_t n, int *radices, int *lens, int max_lists, int *nlists);

/*
 * Host-only: the radix lists compiled as specialised kernels for dtype,
 * the wide lengths' lists (see fftc_max_single_n) last.
 * Entry i (0 <= i < fftc_compiled_count(dtype)) has length *n and list
 * radices[0..*count); max_count is the capacity of radices (>= 8).
 */
int fftc_compiled_count(int dtype);
fftc_status fftc_compiled_entry(int dtype, int i, int64_t *n, int *radices, int max_count, int *count);

/*
 * Host-only: every supported n up to this value (complex64 16384,
 * complex128 8192) runs as one kernel for dtype.  Above it, the wide lengths
 * complex64 32768 and complex128 16384 also run as one kernel (one transform
 * per 1024-thread workgroup, its stages exchanging real and imaginary parts
 * in turn through 139 KB of LDS, from their compiled lists only); every other
 * n runs as the two passes of Eq. 2.
 */
int64_t fftc_max_single_n(int dtype);

/*
 * Bandwidth reference (not an operation of the method): copy `bytes` from
 * device memory `in` to device memory `out` in the transforms' own access
 * form, one 16-byte nontemporal load and store per thread, asynchronously on
 * `stream` (hipStream_t, NULL = default).  Both pointers 16-byte aligned and
 * bytes a multiple of 16, the ranges disjoint; otherwise
 * FFTC_ERR_INVALID_ARG and nothing is launched.  bytes = 0 does nothing.
 * The caller owns both buffers.  The benchmark times it beside the
 * transforms: what a plain stream of the same bytes reaches on the device.
 */
fftc_status fftc_copy(const void *in, void *out, size_t bytes, void *stream);

/*
 * Mixed-length plan: `count` transforms of lengths n[0..count), packed back to
 * back in that order (transform i starts at element n[0] + ... + n[i-1]) in
 * both in and out.  Every length must satisfy 1 <= n[i] <= 4096 with prime
 * factors <= 7.  The uneven batch runs as one persistent launch: equal lengths
 * form classes with their own radix list (tuning database or heuristic), and
 * the plan assigns the work items, longest first, each to the resident
 * workgroup with the least work so far; a workgroup fetches its next item's
 * descriptor while it runs the current one.  The
 * launch is recorded in a hipGraph at plan time; fftc_execute replays it on
 * the caller's stream (updating the graph's pointer arguments when in/out
 * change), or launches the kernel directly (fftc_plan_mixed_set_launch).  Executions of one mixed plan on different streams must not
 * overlap: they share the plan's one instantiated graph, whose pointer
 * arguments a call with other in/out updates.
 */
fftc_status fftc_plan_mixed(const int64_t *n, int64_t count, int direction, int dtype,
                            fftc_plan_t *plan_out);

/*
 * How fftc_execute runs a mixed plan's persistent launch:
 * FFTC_MIXED_LAUNCH_GRAPH (the default) replays the plan's instantiated
 * hipGraph; FFTC_MIXED_LAUNCH_DIRECT launches the same kernel with the same
 * arguments on the stream (a caller can still capture that launch into a
 * graph of its own).  Results are identical.  Measured on MI355X, a replay
 * leaves the GPU idle about 8 us before the kernel starts, where back-to-back
 * direct launches leave no gap.  FFTC_ERR_INVALID_ARG for a NULL or non-mixed
 * plan or another mode.  Host-only; not while an execution is being enqueued
 * on the plan from another thread.
 */
enum { FFTC_MIXED_LAUNCH_GRAPH = 0, FFTC_MIXED_LAUNCH_DIRECT = 1 };
fftc_status fftc_plan_mixed_set_launch(fftc_plan_t plan, int mode);

/*
 * Autotuner (the planner the paper names as missing, Section VI; different
 * factorisations suit different hardware, Section I).  Times every
 * candidate Stockham radix list for single-kernel length n (for a wide
 * length, each of its compiled lists), forward, on an
 * internal stream, at the HBM-bound shape: max(batch, 2^24 / n) transforms
 * per launch, launches rotating over four input/output pairs that it
 * allocates and frees (1 GiB for complex64 at 2^24 elements), each launch
 * timed by its own events.  A candidate's time is the median of `reps`
 * launches (1 <= reps <= 100000; use 20 or more).  Every candidate whose
 * median is within the tie window of the fastest -- twice the larger
 * relative interquartile range of the two candidates' launches, and at least
 * 3% -- counts as equally fast, and among those the list with fewer stages,
 * then the one earlier in the planner's order, wins; picking from the whole
 * tied set keeps the choice the same from run to run.  The winner is recorded
 * in the process's tuning database, which later plans for (n, dtype) use.
 * Returns the chosen list in radices[0..*count) and its median time per
 * launch in microseconds.  Synchronous.
 */
fftc_status fftc_autotune(int64_t n, int64_t batch, int dtype, int reps, int *radices,
                          int max_count, int *count, double *best_us);

/* ---------------------------------------------------------------------------
 * Alternative factorisation orders (Sections I-II: the factorisation that
 * suits the hardware is an open choice -- Stockham, Pease, or the recursive
 * Cooley-Tukey form the paper runs).  For N = radix^t (N = 64, 256, 1024,
 * 4096 with the radices listed by fftc_order_entry), one LDS-resident kernel
 * per order:
 *   FFTC_ORDER_CT     Eq. 2 unrolled: explicit digit reversal of the input
 *                     (the product of the recursion's Pi factors), then t
 *                     in-place radix-R stages (decimation in time);
 *   FFTC_ORDER_PEASE  constant geometry: every stage reads x[j + r N/R] and
 *                     writes y[j R + r]; explicit digit reversal on output;
 *   FFTC_ORDER_WAVE   N = 256 only (radix 16): Stockham with the stride
 *                     permutation between its two radix-16 stages done inside
 *                     the wave -- a 16 x 16 transpose across the 16 lanes of a
 *                     transform by DPP quad permutes and ds_swizzle, no LDS
 *                     and no barrier (the wavefront-shuffle exchange);
 *   FFTC_ORDER_FOURSTEP  Eq. 2 applied once (the block form): N = K M with
 *                     M = R^ceil(t/2), K = R^floor(t/2); Pi^N_K on load, DFT_M
 *                     on the K rows, D^N_M, DFT_K on the M columns (radix-R
 *                     Stockham stages for both), natural-order store.
 * Same conventions and results as fftc_plan (up to rounding).
 * ------------------------------------------------------------------------- */
enum { FFTC_ORDER_STOCKHAM = 0, FFTC_ORDER_CT = 1, FFTC_ORDER_PEASE = 2, FFTC_ORDER_FOURSTEP = 3,
       FFTC_ORDER_WAVE = 4 };

fftc_status fftc_plan_order(int64_t n, int64_t batch, int direction, int dtype, int order, int radix,
                            fftc_plan_t *plan_out);

/* Host-only: the compiled (n, order, radix) triples for dtype. */
int fftc_order_count(int dtype);
fftc_status fftc_order_entry(int dtype, int i, int64_t *n, int *order, int *radix);

/*
 * Order autotuner: times the Stockham plan (its tuned or preferred list) and
 * every compiled (order, radix) for n, like fftc_autotune (median of `reps`
 * launches at the HBM-bound shape, rotating internal buffers).  Writes up to
 * `max` results (orders[i], radices[i] -- 0 for Stockham -- and us[i]), the
 * count, and the index of the pick: Stockham unless it is outside the tie
 * window (as for fftc_autotune) of the fastest candidate, else the first
 * compiled order within that window of the fastest.  The winner is recorded in the tuning database, and
 * fftc_plan then uses that order for (n, dtype).
 */
fftc_status fftc_autotune_orders(int64_t n, int64_t batch, int dtype, int reps, int *orders, int *radices,
                                 double *us, int max, int *count, int *best);

/* Tuning database persistence (the planner's memory of what was fastest,
 * Section VI; FFTW's wisdom is the model the paper cites, Section III).
 * Text, one line per entry:
 *   <arch> <toolchain> <c64|c128> <n> [<order>:]<r1,r2,...> <ms>
 * keyed on the device architecture and the HIP version the library's kernels
 * were compiled with (fftc_tune_key(), e.g. "gfx950 hip7.2.53211"); lines
 * with another key or in another format are skipped.  The database is read
 * once from the file named by the FFTC_TUNE_DB environment variable, if set,
 * and from fftc_server_config.tune_db when a server starts.
 * fftc_tune_load merges the file's entries (*entries = lines accepted). */
fftc_status fftc_tune_load(const char *path, int *entries);
fftc_status fftc_tune_save(const char *path, int *entries);
fftc_status fftc_tune_clear(void);
/* "<arch> <toolchain>" of this build (static storage). */
const char *fftc_tune_key(void);

/* ---------------------------------------------------------------------------
 * Serving.  One process-global server takes FFT requests of any supported
 * length and batch as they arrive and runs them with continuous batching:
 * requests are admitted in arrival order as device memory (a budget arena
 * for outputs) and in-flight slots free up, each admitted request is launched
 * at once on a stream of a pool so it overlaps with work already on the GPU,
 * and plans with their twiddle tables stay resident between requests (the
 * paper's point that an FFT is compiled once and run many times, Section
 * VI; the just-in-time flexibility of its JIT mode over a fixed-size AOT
 * build, Section IV-B, comes from the plan cache: any supported n is served).
 *
 * Failure hooks (environment): FFTC_FAULT=k makes the k-th device or arena
 * allocation from then on fail with FFTC_ERR_OUT_OF_MEMORY before any HIP
 * call (a failed arena allocation fails that request only; the server keeps
 * serving), FFTC_LOG=1 logs plans, server start/stop and injected faults to
 * stderr, FFTC_ROCTX=1 adds roctx ranges (fftc_plan, fftc_execute,
 * fftc_execute_batch, fftc_server_round) for rocprofv3 --marker-trace,
 * loading the ROCm profiler's roctx library at run time.  fftc_fault_set(k)
 * sets the fault counter from code (k <= 0: off).
 * ------------------------------------------------------------------------- */
fftc_status fftc_fault_set(int64_t k);
/* Allocations counted since the last fftc_fault_set (or FFTC_FAULT). */
int64_t fftc_fault_count(void);

enum { FFTC_EXECUTOR_GPU = 0, FFTC_EXECUTOR_MOCK = 1 };

typedef struct {
    size_t budget_bytes;   /* device memory for request outputs */
    int n_streams;         /* HIP streams the requests are spread over (>= 1) */
    int max_inflight;      /* requests on the GPU at once (>= 1) */
    int executor;          /* FFTC_EXECUTOR_GPU, or FFTC_EXECUTOR_MOCK: no device
                              use and no computation, for testing the admission
                              and scheduling logic on a host without a GPU */
    int64_t mock_ns_per_mb;/* mock executor: simulated time per MiB of output */
    int fuse;              /* 1: requests admitted together that share (n, direction,
                              dtype) run as one launch (up to 16 per launch) when the
                              length has a several-requests kernel (powers of two with
                              the preferred radix list); 0: one launch per request */
    const char *tune_db;   /* tuning database file merged into the process's database
                              before any plan is made (NULL or "": none; a file that
                              cannot be read fails the start with FFTC_ERR_INVALID_ARG) */
    int hold_at;           /* 0: an admitted request launches at once; k > 0: requests
                              admitted while k or more are on the GPU wait, holding their
                              slots and outputs, and launch together as soon as fewer
                              than k are (larger rounds for fuse under load; nothing
                              waits below k) */
} fftc_server_config;

typedef struct {
    int64_t n, batch;      /* batch transforms of length n */
    int direction, dtype;
    const void *in;        /* device input, batch * n elements; must stay valid
                              until the request's completion is polled */
    uint64_t tag;          /* returned in the completion */
    int64_t arrival_ns;    /* caller's arrival time on fftc_now_ns's clock */
} fftc_request;

typedef struct {
    uint64_t tag;
    fftc_status status;    /* FFTC_OK, FFTC_ERR_SHUTDOWN (cancelled) or a launch error */
    void *out;             /* device output (batch * n elements) owned by the
                              caller until fftc_release; NULL unless OK */
    int64_t arrival_ns, admit_ns, start_ns, done_ns;  /* done: completion observed */
    int64_t n, batch;
} fftc_completion;

typedef struct {
    int64_t submitted, admitted, completed, rejected, cancelled, failed;
    size_t budget_bytes, bytes_in_use, peak_bytes;
    int pending, inflight, max_inflight_seen;
    int64_t fused_launches, fused_requests;  /* several-requests launches and the requests they ran */
    size_t plan_bytes;     /* device memory of the resident plans (twiddle tables), on
                              top of the budget: at most 16 bytes per element of each
                              distinct (n, direction, dtype) served */
} fftc_server_stats;

/* Monotonic clock (ns) used for all server timestamps. */
int64_t fftc_now_ns(void);

/* Start the server on the current device: allocates the budget arena (and
 * writes it once, so requests never meet untouched memory), the streams and
 * events.  Fails if a server is already running. */
fftc_status fftc_server_start(const fftc_server_config *cfg);

/* Build (and keep) the plan for (n, direction, dtype) able to run batches up
 * to max_batch, and run it once on a scratch buffer of its own (with the
 * several-requests kernel too when fusing), so the first request of that
 * shape pays neither planning nor kernel loading.  Synchronous. */
fftc_status fftc_server_prepare(int64_t n, int direction, int dtype, int64_t max_batch);

/* Queue a request (copied); returns at once.  FFTC_ERR_TOO_LARGE if its
 * output alone exceeds the budget; a full arena only delays admission. */
fftc_status fftc_submit(const fftc_request *req);

/* Take up to max finished requests (non-blocking); *n_out = how many. */
fftc_status fftc_poll(fftc_completion *out, int max, int *n_out);

/* Return a completion's output to the arena. */
fftc_status fftc_release(void *out);

fftc_status fftc_server_stats_get(fftc_server_stats *stats);

/* Stop: drain != 0 runs everything queued first (outputs still have to be
 * released by the caller if memory is short), else queued requests complete
 * with FFTC_ERR_SHUTDOWN.  Waits for GPU work, then frees plans, arena and
 * streams (outputs not yet released become invalid). */
fftc_status fftc_server_stop(int drain);

/* Text of a status code (static storage). */
const char *fftc_status_string(fftc_status s);

/* Detail of the last failure on the calling thread ("" if none). */
const char *fftc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FFTC_H */
