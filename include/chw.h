/*
 * chw.h -- C ABI of libchw, the Cascading Haar Wavelet (CHW) computation of
 * the dyadic-ordered (Paley) Walsh-Hadamard transform on AMD Instinct MI355X
 * (gfx950).
 *
 * What is computed.  For every signal i of a batch, with n_i = 2^{m_i}:
 *
 *   orthonormal mode   y_i = H_{m_i} x_i
 *   unnormalized mode  y_i = H'_{m_i} x_i,   H'_m = 2^{m/2} H_m  (entries +-1)
 *
 * where H_m is the Hadamard matrix with columns in dyadic (Paley) order of
 * eq. (1) of the paper (H_0 = 1, H_{k+1} = 2^{-1/2}[H_k (x) (1 1); H_k (x)
 * (1 -1)]).  It is evaluated by the CHW algorithm of Sec. 2 / Theorem 1
 * (eq. 3): a full-size Haar transform Psi_m (eq. 2) followed by the m-1
 * block-diagonal factors I_{r-1} (x) diag(I_{m-r}, Psi_{m-r}), with the
 * identity blocks not performed, m*2^m additions in all (Theorem 2).  The
 * backward call applies H_m^T as the transposed factors in reverse order.
 * H_m is symmetric, so forward and backward give the same numbers.
 *
 * Memory.  All data pointers are DEVICE pointers (hipMalloc, or a torch
 * CUDA/HIP tensor's data_ptr()).  Host pointers are named as such below.
 * The caller owns x, y, the workspace and the stream; the plan owns copies
 * of the sizes and offsets, its device-side work tables and any captured
 * graph.
 *
 * Errors.  Every entry point returns a chw_status.  Arguments are checked
 * before any device work is enqueued; on error nothing is written.  No entry
 * point aborts, throws or prints (except with CHW_LOG set).  A detail string
 * for the last failure of the calling thread is kept by chw_last_error().
 * Calls enqueue work asynchronously on the given stream and return; device
 * faults surface at the caller's next synchronizing HIP call.
 */
#ifndef CHW_H
#define CHW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Opaque plan handle. */
typedef struct chw_plan_s *chw_plan_t;

/* Element type of x and y.  BF16 and F16 are stored as 16-bit values and
 * computed in FP32 inside every pass (the intermediate between HBM passes is
 * FP32); the result is rounded to nearest even.  F64 is for verification and
 * gradient checks. */
typedef enum {
    CHW_F32 = 0,
    CHW_BF16 = 1,
    CHW_F16 = 2,
    CHW_I32 = 3,
    CHW_F64 = 4,
    /* Range markers (not types): they make every int32 value a valid
       chw_dtype, so that a caller's out-of-range value reaches the argument
       check (CHW_ERR_INVALID_ARGUMENT) instead of being undefined. */
    CHW_DTYPE_MIN_ = -2147483647 - 1,
    CHW_DTYPE_MAX_ = 2147483647
} chw_dtype;

/* CHW_ORTHONORMAL: y = H_m x (float types only).
 * CHW_UNNORMALIZED: y = H'_m x, every 1/sqrt(2) of eqs. (1)-(2) dropped.
 * The integer type supports only CHW_UNNORMALIZED: int32 arithmetic wraps
 * modulo 2^32, so the result is exact whenever it fits in int32 (always the
 * case for |x| <= 128 and n <= 2^22). */
typedef enum {
    CHW_ORTHONORMAL = 0,
    CHW_UNNORMALIZED = 1,
    CHW_NORM_MIN_ = -2147483647 - 1, /* range markers, as for chw_dtype */
    CHW_NORM_MAX_ = 2147483647
} chw_norm;

typedef enum {
    CHW_OK = 0,
    CHW_ERR_INVALID_ARGUMENT = 1, /* NULL/negative/out-of-range/overlapping */
    CHW_ERR_UNSUPPORTED = 2,      /* valid request the library cannot serve */
    CHW_ERR_MISALIGNED = 3,       /* pointer or offset not 16-byte aligned  */
    CHW_ERR_OUT_OF_MEMORY = 4,    /* host/device allocation or size overflow */
    CHW_ERR_NO_DEVICE = 5,        /* no usable gfx950 device in this process */
    CHW_ERR_HIP = 6,              /* a HIP runtime call failed              */
    CHW_ERR_DEVICE = 7            /* a kernel reported an error flag        */
} chw_status;

/* Plan flags. */
enum {
    CHW_FLAG_GRAPH = 1u << 0,        /* capture the launches of a call in a
                                        hipGraph and replay it               */
    CHW_FLAG_NO_AUTOTUNE = 1u << 1,  /* neither start from nor record into the
                                        tuning cache (see chw_tuning_load)    */
    CHW_FLAG_PERSISTENT = 1u << 2,   /* one persistent launch (exec 2)        */
    CHW_FLAG_MULTI_LAUNCH = 1u << 3, /* one launch per HBM pass              */
    /* Coefficient order of the output of chw_forward (and of the input of
       chw_backward).  Default: dyadic (Paley) order of eq. (1).  The other
       orders permute the same coefficients (same bits):
         SEQUENCY: Walsh order, row s of the matrix has s sign changes
                   (output s = dyadic coefficient gray(s), gray(s) = s ^ s>>1);
         NATURAL:  Sylvester (Kronecker) order, output k = dyadic coefficient
                   bitrev_m(k).
       Exclusive with each other and with CHW_FLAG_PERSISTENT; plans with an
       order other than dyadic run their adjoint one workgroup per tile (no
       prefetching), one launch per round of a signed call, and need the
       workspace in out-of-place forward calls too (their last pass stores
       outside the blocks it loads). */
    CHW_FLAG_ORDER_SEQUENCY = 1u << 4,
    CHW_FLAG_ORDER_NATURAL = 1u << 5,
    /* Run signals of 2^20 elements or more in the three HBM passes that
       signals above 2^25 always take (see chw_workspace_size): the same
       numbers, more traffic.  It exists to check that form at sizes an
       oracle runs in seconds.  Dyadic order only; exclusive with
       CHW_FLAG_PERSISTENT. */
    CHW_FLAG_THREE_PASS = 1u << 6
};

/* Largest supported log2 signal size (all dtypes except F64).  Signals above
 * 2^15 elements run in two HBM passes, signals above 2^25 in three (dyadic
 * order; the other orders take two passes up to 2^27 and stop there). */
#define CHW_MAX_LOG2 30
/* Largest supported log2 signal size for CHW_F64. */
#define CHW_MAX_LOG2_F64 20
/* Largest number of rounds of a signed call (chw_forward_signed). */
#define CHW_MAX_ROUNDS 64

/* Layout of the random-sign diagonals of chw_forward_signed. */
typedef enum {
    CHW_SIGNS_PER_ELEMENT = 0,  /* bit e of a round's words is the sign of
                                   element e of the buffers (e counts from
                                   element 0, gaps included)                */
    CHW_SIGNS_SHARED = 1,       /* bit j is the sign of element j of every
                                   signal (one diagonal shared by all
                                   signals; a signal of 2^m elements uses
                                   bits 0 .. 2^m - 1)                       */
    CHW_SIGN_MODE_MIN_ = -2147483647 - 1, /* range markers, as for chw_dtype */
    CHW_SIGN_MODE_MAX_ = 2147483647
} chw_sign_mode;

/*
 * chw_plan -- validate a batch description and build a plan.
 *
 *   plan        out: the new plan (host pointer to a handle).
 *   batch       number of signals, >= 0 (0 gives a plan whose calls do
 *               nothing).
 *   log2_sizes  host array [batch]: m_i, 0 <= m_i <= CHW_MAX_LOG2
 *               (CHW_MAX_LOG2_F64 for CHW_F64).  m_i = 0 is a copy (H_0 = 1).
 *   offsets     host array [batch + 1] of int64 ELEMENT offsets, or NULL for
 *               signals packed back to back from element 0.  Signal i
 *               occupies [offsets[i], offsets[i] + 2^{m_i}); offsets must be
 *               non-negative, ascending and non-overlapping:
 *               offsets[i] + 2^{m_i} <= offsets[i + 1].  offsets[batch] is the
 *               extent of the buffers in elements.  Elements in gaps are never
 *               read or written.  Signals whose byte size is >= 16 must start
 *               on a 16-byte boundary (offsets[i] * sizeof(element) % 16 == 0)
 *               or CHW_ERR_MISALIGNED is returned.
 *   dtype, norm see the enums.  I32 requires CHW_UNNORMALIZED.
 *   flags       CHW_FLAG_* bits.
 *
 * The plan is immutable after creation (tuning aside) and may be used from
 * several host threads at once provided each call uses its own workspace.
 * Planning itself needs no device; device tables are uploaded at first use
 * on the device that is current at that time.
 */
chw_status chw_plan(chw_plan_t *plan, int64_t batch, const int32_t *log2_sizes,
                    const int64_t *offsets, chw_dtype dtype, chw_norm norm,
                    uint32_t flags);

/*
 * chw_plan_haar_walsh -- plan the Haar-Walsh transform of eq. (4) for `batch`
 * signals of 2^m elements packed back to back (signal i at element i 2^m):
 *     y = diag(1, H_0, H_1, ..., H_{m-1}) w,
 * the matrix eq. (4) equates with H_m Psi_m^T.  w holds Haar coefficients in
 * the order of eq. (2) (scaling coefficient, then the detail blocks of 2^k
 * coefficients, coarsest first); coefficient block [2^k, 2^{k+1}) of every
 * signal is transformed by H_k and w_0 is copied, so H_m x = (this
 * transform)(Psi_m x).  The result is an ordinary plan over the ragged batch
 * of those blocks: chw_forward applies the transform, chw_backward its
 * transpose, with every rule of chw_plan.  0 <= m <= CHW_MAX_LOG2
 * (CHW_MAX_LOG2_F64); other arguments as chw_plan.
 */
chw_status chw_plan_haar_walsh(chw_plan_t *plan, int64_t batch, int32_t m, chw_dtype dtype,
                               chw_norm norm, uint32_t flags);

/* Bytes of device workspace a call may need: the FP32 (FP64 for CHW_F64)
 * intermediate between HBM passes of every signal larger than 2^12 elements,
 * twice over for the signals that take three passes (above 2^25, or 2^20 and
 * above with CHW_FLAG_THREE_PASS), which keep two intermediates.
 * The figure does not depend on tuning or options, so a buffer sized from it
 * stays large enough after chw_autotune / chw_plan_set_option.  Calls whose
 * signals all run in one pass, and out-of-place forward F32/I32/F64 calls of
 * dyadic-order plans without three-pass signals (which route the intermediate
 * through y), accept NULL.  A workspace must not be shared by concurrent
 * calls. */
chw_status chw_workspace_size(chw_plan_t plan, size_t *bytes);

/*
 * chw_forward -- y_i = H_{m_i} x_i (or H'_{m_i} x_i) for every signal.
 *
 *   x, y       device buffers of plan's dtype, each of extent offsets[batch]
 *              elements; 16-byte aligned.  y == x (in place) is allowed;
 *              partial overlap is CHW_ERR_INVALID_ARGUMENT.
 *   workspace  device buffer of chw_workspace_size() bytes, or NULL when that
 *              is 0 (see chw_workspace_size for out-of-place calls).
 *   stream     a hipStream_t, or NULL for the default stream.
 */
chw_status chw_forward(chw_plan_t plan, const void *x, void *y, void *workspace,
                       void *stream);

/*
 * chw_forward_noalloc -- chw_forward for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same result, bit for bit, as chw_forward on the same
 * plan; the intermediate between the two HBM passes lives in a static device
 * array of the library (64 MiB per device, held from the first call on a
 * device until the process ends) instead of a workspace argument.  The call
 * performs no hipMalloc, hipFree, graph capture or event creation.
 *
 *   x, y     as chw_forward (device buffers owned by the caller).
 *   stream   as chw_forward.
 * Errors (as chw_forward, plus):
 *   CHW_ERR_UNSUPPORTED  the plan's intermediate (4 bytes per element of its
 *                        two-pass signals, 8 for CHW_F64) exceeds 64 MiB, i.e.
 *                        more than 2^24 such elements (2^23 for CHW_F64);
 *                        or the plan's work tables have not been uploaded to
 *                        the current device yet (one chw_forward or
 *                        chw_backward call on that device does it); or option
 *                        "timing" is on.
 * A plan with CHW_FLAG_GRAPH launches directly here (no replay).  Every call
 * on one device shares that device's array: calls that overlap in time on
 * one device (on different streams, or from several host threads without
 * ordering) race on it and give wrong results.  The array's contents are
 * whatever the last call left; each call writes every intermediate element
 * before it reads it, so nothing needs clearing.
 */
chw_status chw_forward_noalloc(chw_plan_t plan, const void *x, void *y, void *stream);

/* chw_backward -- y_i = H_{m_i}^T g_i: the adjoint of eq. (3), the transposed
 * factors in reverse order (Haar synthesis).  In the dyadic order H_m is
 * symmetric and the synthesis cascade adds the same pairs in the same order
 * as the forward one (on positions relabelled by the bit reversal), so by
 * default a dyadic-order plan runs the forward launches, which give the same
 * bits faster; option "adjoint" = 1 runs the synthesis kernels instead.
 * Plans of the other orders always run the synthesis kernels.  Same
 * arguments and rules as chw_forward. */
chw_status chw_backward(chw_plan_t plan, const void *g, void *y, void *workspace,
                        void *stream);

/*
 * chw_forward_signed -- randomized Hadamard transform with the random-sign
 * diagonals fused into the tile kernels (not part of the paper: the step
 * that usually precedes the transform in sketching and Hadamard rotations):
 *     y_i = H D_k ... H D_2 H D_1 x_i          (k = rounds, H = H_{m_i})
 * where D_r = diag(d_r), d_r[j] = -1 where the sign bit is set, else +1.
 * Round r's diagonal multiplies the vector the round reads: x for r = 1, the
 * dyadic-ordered output of round r - 1 otherwise.  Each round is one complete
 * transform (orthonormal or not as the plan says) whose output is stored in
 * y in the plan's dtype; rounds after the first run in place on y.
 *
 *   signs   device array of rounds * W uint32 words, 4-byte aligned, W =
 *           chw_sign_words(plan, mode); round r (0-based) uses words
 *           [r W, (r + 1) W).  Bit b of the round is bit (b % 32) of word
 *           b / 32; b is chosen by `mode`.  Read only.
 *   mode    CHW_SIGNS_PER_ELEMENT or CHW_SIGNS_SHARED.
 *   rounds  1 .. CHW_MAX_ROUNDS.  rounds > 1 with signals above 2^12
 *           elements needs a workspace (the later rounds run in place).
 * Other arguments and errors as chw_forward; signs = NULL or a misaligned
 * signs pointer gives CHW_ERR_INVALID_ARGUMENT / CHW_ERR_MISALIGNED.  The
 * sign flips are exact, so with d = +1 everywhere and rounds = 1 the result
 * equals chw_forward bit for bit.
 */
chw_status chw_forward_signed(chw_plan_t plan, const void *x, void *y, void *workspace,
                              const uint32_t *signs, chw_sign_mode mode, int rounds,
                              void *stream);

/*
 * chw_haar_forward -- the Haar wavelet transform alone, y_i = Psi_{m_i} x_i
 * (eq. 2; the first factor of Theorem 1, "computed for free" by the
 * cascade): output in the order of eq. (2), scaling coefficient first, then
 * the detail blocks of 2^k coefficients, coarsest first.  Orthonormal or
 * unnormalized as the plan says (the unnormalized form drops every
 * 1/sqrt(2)).  x and y must be distinct (no in-place call); signals above
 * 2^12 elements need a workspace of chw_workspace_size() bytes (their tile
 * sums between level passes).  Otherwise as chw_forward.
 */
chw_status chw_haar_forward(chw_plan_t plan, const void *x, void *y, void *workspace,
                            void *stream);

/* chw_haar_backward -- Psi^T g (Haar synthesis, the adjoint and, in the
 * orthonormal form, the inverse of chw_haar_forward).  Same rules. */
chw_status chw_haar_backward(chw_plan_t plan, const void *g, void *y, void *workspace,
                             void *stream);

/*
 * chw_nodes_forward -- y_i = H_m x_i evaluated factor by factor, the way the
 * parallel scheme of Sec. 4 distributes the cascade over processing nodes:
 * one launch ("node") per factor of eq. (3), node 0 applying Psi_m (eq. 2) to
 * every signal and node r (1 <= r <= m - 1) applying F_r = I_{r-1} (x)
 * diag(I_{m-r}, Psi_{m-r}) -- the Haar transforms of size 2^{m-r} on the
 * upper halves -- while passing the rest of the stream through.  Every Haar
 * level scales by fl(2^{-1/2}) as eq. (2) writes it, so results equal
 * chw_forward's up to rounding.  Each node reads and writes the whole
 * vector: this entry point exists to measure the paper's decomposition
 * against the stage-grouped kernels of chw_forward, which it does not
 * replace.
 *
 *   plan       orthonormal, dyadic CHW_F32 plan of equal sizes 2^m,
 *              1 <= m <= 24, packed back to back (offsets NULL or i 2^m);
 *              other plans give CHW_ERR_UNSUPPORTED.
 *   x, y       distinct, non-overlapping device buffers of batch 2^m floats,
 *              4-byte aligned.
 *   workspace  chw_nodes_workspace_size() bytes (the stream between nodes
 *              and the chunk sums of the large Haar transforms), 4-byte
 *              aligned, not overlapping x or y.
 *   chunk      0: every node runs over the whole batch before the next one;
 *              c > 0: the batch runs c signals at a time, all m nodes on one
 *              chunk before the next, so a node reads its predecessor's output
 *              while it is still cached (the streaming between nodes).
 *   stream     as chw_forward.
 */
chw_status chw_nodes_forward(chw_plan_t plan, const void *x, void *y, void *workspace,
                             int64_t chunk, void *stream);

/* Workspace bytes of chw_nodes_forward for any chunk: 4 (batch 2^m +
 * batch 2^{m-12}) (the second term for m > 12 only). */
chw_status chw_nodes_workspace_size(chw_plan_t plan, size_t *bytes);

/* chw_backward_signed -- the adjoint of chw_forward_signed:
 *     y_i = D_1 H^T D_2 H^T ... D_k H^T g_i
 * (rounds in reverse order, each diagonal applied to its round's output as
 * it is stored).  A dyadic-order plan runs its two-pass signals through the
 * forward launches (H^T = H with the same bits, see chw_backward) in one-round
 * calls, and in multi-round calls where it uses round-boundary tiles: round 1
 * without a diagonal, D_k .. D_2 at the boundaries, D_1 at the last pass's
 * store; option "adjoint" = 1 runs the synthesis kernels instead.  Same
 * arguments and rules as chw_forward_signed. */
chw_status chw_backward_signed(chw_plan_t plan, const void *g, void *y, void *workspace,
                               const uint32_t *signs, chw_sign_mode mode, int rounds,
                               void *stream);

/* Words per round W of the sign arrays of this plan: ceil(2^{max m_i} / 32)
 * for CHW_SIGNS_SHARED, ceil(offsets[batch] / 32) for CHW_SIGNS_PER_ELEMENT. */
chw_status chw_sign_words(chw_plan_t plan, chw_sign_mode mode, size_t *words);

/*
 * chw_philox_signs -- generate the sign arrays of chw_forward_signed /
 * chw_backward_signed on the device from the Philox4x64-10 counter-based
 * generator (J. Salmon et al., "Parallel random numbers: as easy as 1, 2,
 * 3", SC 2011; each sign is +1 or -1 with probability 1/2):
 *     word w of round r (0-based) = 32-bit word (w mod 8) of the Philox4x64-10
 *     block with counter (floor(w / 8), r, 0, 0) and key (seed, 0), where the
 *     block's 64-bit outputs o_0..o_3 give words 2i (low half of o_i) and
 *     2i + 1 (high half).
 * The words depend only on (seed, r, w), so any thread, call or host can
 * regenerate any sign.
 *
 *   seed    the generator key.
 *   rounds  1 .. CHW_MAX_ROUNDS.
 *   signs   device array of rounds * W uint32 words (W = chw_sign_words(plan,
 *           mode)), 4-byte aligned, owned by the caller; round r is written at
 *           words [r W, (r + 1) W), the bits past the last element included.
 *   stream  as chw_forward.
 * Errors: plan or signs NULL, bad mode or rounds -> CHW_ERR_INVALID_ARGUMENT;
 * signs misaligned -> CHW_ERR_MISALIGNED; no GPU -> CHW_ERR_NO_DEVICE.
 */
chw_status chw_philox_signs(chw_plan_t plan, chw_sign_mode mode, uint64_t seed, int rounds,
                            uint32_t *signs, void *stream);

/* Release a plan and its device tables and graphs.  NULL is a no-op.  The
 * caller must have synchronized every stream the plan was used on. */
chw_status chw_plan_destroy(chw_plan_t plan);

/* Override a planner choice before first use.  Keys (value):
 *   "split_l1"  levels of the first HBM pass of multi-pass signals (-1 = auto)
 *   "lr12"      5 or 6: log2 registers per thread of the 2^12-element tiles
 *               (0, the default: 5 in single-pass launches, 6 in the others)
 *   "lr15"      5 or 6: log2 registers per thread of the 2^15-element tiles
 *   "single15"  1: signals of 2^13..2^15 in one pass; 0: two passes
 *   "chunk"     elements of multi-pass signals per first/last pass pair
 *               (0 = the whole batch in one pair of launches)
 *   "exec"      0 = one launch per pass; 2 = one persistent launch in which a
 *               workgroup runs both passes of a multi-pass signal (also set by
 *               CHW_FLAG_PERSISTENT).  1 (a dependency-counter work queue) is
 *               disabled: it gives CHW_ERR_UNSUPPORTED.
 *   "ptile"     tile size of the persistent launch: 12 (2^12-element tiles,
 *               several workgroups per CU, signals up to 2^21), 15
 *               (2^15-element tiles, one workgroup per CU, signals up to 2^23;
 *               not FP64) or 0 (default: 15, and 12 for FP64).
 *   "pipeline"  1 (with "chunk" > 0): launch j runs the last pass of chunk
 *               j - 1 together with the first pass of chunk j, both in
 *               2^15-element tiles, and the chunks' intermediates alternate
 *               between two workspace slots (0: passes of a chunk in separate
 *               launches).
 *   "stream"    2: a launch (exec 0) of 2^15-element tiles that are all
 *               full and of one kind runs as a loop over its items, fetching
 *               the next tile's vectors while the current tile runs;
 *               1 (default): the same, except that a launch of single-pass
 *               tiles prefetches only when it has at least 1024 of them;
 *               0: one workgroup per tile.  (The adjoint of the sequency and
 *               natural orders always runs one workgroup per tile.)
 *   "turn"      1 (default): signed calls of several rounds join round r's
 *               last pass and round r + 1's first pass (forward; the other
 *               way round for the adjoint) in one launch of round-boundary
 *               tiles, where the plan qualifies (FP32 / int32, dyadic order,
 *               first passes in 2^15-element tiles); 0: one launch pair per
 *               round.
 *   "spread"    1 (default): a launch of single-pass 2^15-element tiles that
 *               would fill fewer than 256 tiles puts its signals one or a few
 *               per tile (partly filled tiles, more CUs busy); 0: packed.
 *   "adjoint"   0 (default): chw_backward of a dyadic-order plan, and the
 *               two-pass signals of a multi-round chw_backward_signed with
 *               round-boundary tiles, run the forward launches (same bits,
 *               see chw_backward); 1: the Haar synthesis kernels.
 *   "occupancy" 0 (default): the looping launches (the persistent kernel,
 *               the prefetching kernels) run as many workgroups as can be
 *               resident; 1 .. 32: at most that many per CU (grid = min(items,
 *               occupancy x CUs)).  A tuning choice of the persistent form.
 *   "timing"    1: record a HIP event around every launch (instrumentation;
 *               may be toggled at any time; disables graph replay)
 * Unknown keys or values give CHW_ERR_INVALID_ARGUMENT; so does changing a
 * planner choice on a plan that has been used (plans are immutable once used).
 * No choice changes the numbers: every configuration runs the same stages on
 * the same operands in the same order. */
chw_status chw_plan_set_option(chw_plan_t plan, const char *key, int64_t value);

/* With option "timing" on: durations in milliseconds of the kernel launches of
 * the plan's last call, measured by HIP events on that call's stream.  *n in:
 * capacity of ms (host array); out: number of launches of that call.  Waits
 * for the last call to finish. */
chw_status chw_launch_times(chw_plan_t plan, float *ms, int *n);

/* Host-only check of the plan's work tables: every element of every signal is
 * covered exactly once per pass (one single-pass tile, or one first-pass and
 * one last-pass tile), no tile leaves its signal or the workspace, launches of
 * the two passes are ordered, persistent whole-signal items fit the tile
 * sizes, prefetching launches hold only full 2^15-element tiles of one kind, and the
 * round-boundary tiles of signed multi-round calls cover every two-pass
 * signal exactly once.  CHW_OK, or
 * CHW_ERR_UNSUPPORTED with the reason in chw_last_error(). */
chw_status chw_plan_check(chw_plan_t plan);

/* Write a NUL-terminated JSON description of the plan (passes, level split,
 * tile sizes, work items, workspace) into the host buffer buf of len bytes. */
chw_status chw_plan_describe(chw_plan_t plan, char *buf, size_t len);

/* Time the candidate configurations of this plan on the given buffers (y and
 * workspace are overwritten; x is read only unless x == y) and keep the
 * fastest.  `iters` timed repetitions per candidate.  The candidates vary the
 * level split of the two HBM passes, the registers per thread of both tile
 * sizes, one or two passes for 2^13..2^15 signals, the prefetching form,
 * pipelined chunks, and the persistent launch with its workgroups per CU
 * (option "occupancy"); a launch form fixed by the plan's flags
 * (CHW_FLAG_PERSISTENT, CHW_FLAG_MULTI_LAUNCH) is kept.  The plan's own
 * configuration is timed first, and another replaces the best so far only
 * when it is more than 1% faster.  Candidates the planner cannot build are
 * skipped.  Every candidate computes bitwise-identical results.  Unless the
 * plan has CHW_FLAG_NO_AUTOTUNE, the winner is recorded in the tuning cache
 * under the plan's key (chw_plan_describe reports it as "tuning_key"). */
chw_status chw_autotune(chw_plan_t plan, const void *x, void *y, void *workspace,
                        void *stream, int iters);

/*
 * Tuning cache.  The process keeps the configurations chw_autotune found,
 * keyed by the dtype, the coefficient order, the launch form fixed by the
 * flags and the size mix of the batch (each log2 size present, with the bit
 * length of its signal count).  chw_plan starts a plan from the entry of its
 * key unless it is given CHW_FLAG_NO_AUTOTUNE (chw_plan_describe reports
 * "tuned": 1 then); chw_plan_set_option overrides single choices as usual.
 * An entry never changes the numbers, only which kernels compute them.
 *
 * chw_tuning_save writes every entry to the text file `path` (host string),
 * one line per key: the key, then name=value for each tuned option (lr12,
 * lr15, single15, split_l1, exec, ptile, chunk, stream, pipeline, spread,
 * occupancy); `comment` (may be NULL) is written first as '#' lines.
 * chw_tuning_load merges such a file into the cache: CHW_ERR_INVALID_ARGUMENT
 * (nothing merged, the line in chw_last_error) when it cannot be read or a
 * line is malformed (unknown or repeated option, value out of range, missing
 * option).  chw_tuning_clear empties the cache; chw_tuning_count gives the
 * number of entries.  All four are host-only and thread-safe.
 */
chw_status chw_tuning_save(const char *path, const char *comment);
chw_status chw_tuning_load(const char *path);
chw_status chw_tuning_clear(void);
chw_status chw_tuning_count(size_t *n);

/* Host-only consistency check of the tile kernels' index maps (no device
 * needed): runs the kernels' own layout formulas on the CPU for every compiled
 * tile shape and checks that each load/round/store phase is a bijection onto
 * the tile, stays inside the LDS allocation, and that the per-thread base plus
 * compile-time offset split equals the intended address.  Writes a JSON
 * report (including worst LDS bank multiplicities per phase) into the host
 * buffer report[len] (truncated if short; may be NULL).  Returns CHW_OK, or
 * CHW_ERR_UNSUPPORTED when a map is inconsistent. */
chw_status chw_layout_selfcheck(char *report, size_t len);

/* Human-readable name of a status code (static storage). */
const char *chw_status_string(chw_status s);

/* Detail of the calling thread's last failed call (static or thread-local
 * storage; "" when none). */
const char *chw_last_error(void);

/* Library version string. */
const char *chw_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CHW_H */
