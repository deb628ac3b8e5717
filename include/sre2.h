/*
 * sre2.h - C ABI of libsre2: exact second-order stabilizer Renyi entropy M2 of
 * an N-qubit state vector on an AMD Instinct MI355X (gfx950), by the XOR-FWHT
 * algorithm of Huang, Li, Lee and Zhong (arXiv:2512.24685).
 *
 * What is computed (paper, Eq. 1 with alpha = 2, Eq. Pauli_expect, Eq. final1,
 * Algorithm 1):
 *
 *   W_x(z) = sum_k (-1)^{popcount(z & k)} conj(psi[k ^ x]) psi[k]
 *          = <psi| X^x Z^z |psi>                 (every Pauli string, up to phase)
 *   S_x    = sum_z |W_x(z)|^4                     (one Walsh-Hadamard transform)
 *   S      = sum_x S_x                            (all 4^N Pauli strings)
 *   n      = sum_k |psi[k]|^2
 *   M2     = -log2( S / (2^N n^4) )
 *
 * For a normalised state (n = 1) M2 is the paper's -log2(S / d), d = 2^N.  The
 * division by n^4 makes the result invariant under psi -> c psi.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - psi is a caller-owned DEVICE buffer of 2^N complex amplitudes, interleaved
 *    (re, im): SRE2_C64 = 2 x float32 per amplitude, SRE2_C128 = 2 x float64.
 *    Index k is the integer encoding of the computational basis bit string
 *    (qubit j = bit j).  M2 does not depend on the qubit order.
 *  - Output buffers are caller-owned DEVICE memory.  The library never frees
 *    caller memory.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream) and
 *    is stream-ordered like any HIP call: inputs must stay valid and outputs
 *    must not be read until the stream work completes.
 *  - Argument errors are detected on the host and returned before any work is
 *    enqueued.  Errors raised by the HIP runtime while enqueuing are returned as
 *    SRE2_EHIP.  Properties of the input VALUES (zero norm, NaN, Inf) are only
 *    known on the device: they are reported through the status slot of the
 *    output (see sre2_m2), never by the return code.
 *  - A context owns lazily grown device workspace and is NOT safe for
 *    concurrent use: calls that share a context must be ordered on one stream
 *    (or one host thread).  Use one context per stream.
 *  - All sums are fixed-shape FP64 reductions: for a given (psi bytes, N,
 *    dtype, form) the results are bitwise reproducible run to run.
 */
#ifndef SRE2_H
#define SRE2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes (every function returns one; 0 = success) ------------- */
#define SRE2_OK 0
#define SRE2_EINVAL (-1)     /* null pointer, N outside [1, SRE2_MAX_N], bad count/range */
#define SRE2_EDTYPE (-2)     /* dtype not SRE2_C64 / SRE2_C128 */
#define SRE2_EFORM (-3)      /* unknown or unsupported form for this N */
#define SRE2_ENORM (-4)      /* reserved for host-side input checks (serving) */
#define SRE2_ENOMEM (-5)     /* device workspace could not be allocated */
#define SRE2_EHIP (-6)       /* HIP runtime / launch error (no GPU, bad stream...) */
#define SRE2_EBUSY (-7)      /* serving: no free slot or HBM budget right now */
#define SRE2_ECANCELLED (-8) /* serving: request was cancelled */
#define SRE2_ENOTFOUND (-9)  /* serving: unknown ticket */
#define SRE2_ESCRATCH (-10)  /* allocation-free call: problem larger than its fixed scratch */

/* ---- element types ----------------------------------------------------- */
#define SRE2_C64 0  /* complex64: float32 (re, im) */
#define SRE2_C128 1 /* complex128: float64 (re, im) */

/* ---- arithmetic forms -------------------------------------------------- */
/* FP32: f_x and every butterfly in float32; |W|^2 in float32, squared and
 * accumulated in float64 (complex128 input is rounded to complex64 first). */
#define SRE2_FORM_FP32 0
/* SPLIT_F16: the FP32 form with every group of four butterfly stages replaced
 * by one H_16 = H_2^{(x)4} Kronecker factor on the matrix cores: each FP32
 * value, pre-scaled by an exact power of two so that all values stay below
 * 2^14, is split into FP16 hi + lo halves, and v_mfma_f32_16x16x32_f16 applies
 * the exact +-1 matrix to both with FP32 accumulation (the scale is removed in
 * FP64 at the end).  Stages left over (N mod 4) use FP32 butterflies; N < 5
 * uses the FP32 kernel. */
#define SRE2_FORM_SPLIT_F16 1
/* SPLIT_BF16: the same factors on v_mfma_f32_16x16x32_bf16 with BF16 hi + lo
 * halves (16 significant bits per value instead of 22; BF16 has FP32's
 * exponent range).  Same plans, scale and tolerance bar as SPLIT_F16. */
#define SRE2_FORM_SPLIT_BF16 2
/* FP64: everything in float64 (complex64 input is widened exactly). */
#define SRE2_FORM_FP64 3
/* Hermitian-pair forms: same arithmetic precision as FP32 / FP64 and the same
 * result up to rounding, at half the work.  For x != 0, f_x(k ^ x) equals
 * conj f_x(k) (from Eq. Pauli_expect), so with j the top set bit of x the
 * transform of f_x restricted to the half-space k_j = 0 gives every W_x(z):
 * W_x(z) = 2 Re or 2i Im of it, and S_x = 16 sum (Re^4 + Im^4).  Shift 0 (and,
 * for N >= 15 in FP32 / 14 in FP64, the shifts below 2^12 / 2^11) use the plain
 * kernels. */
#define SRE2_FORM_FP32_HERM 4
#define SRE2_FORM_FP64_HERM 5

#define SRE2_MAX_N 26

/* Layout of the 4-double result written by sre2_m2 / sre2_m2_batched. */
#define SRE2_OUT_M2 0     /* M2 (NaN when status != 0)                        */
#define SRE2_OUT_S 1      /* S = sum over all 4^N Pauli strings of |<P>|^4      */
#define SRE2_OUT_NORM 2   /* n = sum_k |psi[k]|^2 of the arithmetic's input     */
#define SRE2_OUT_STATUS 3 /* 0 = ok; 1 = n == 0 or a non-finite amplitude       */
#define SRE2_OUT_LEN 4

typedef struct sre2_ctx sre2_ctx;

/* Library version, e.g. 100 for 0.1.0. */
int sre2_version(void);

/* Static, never NULL, description of a status code. */
const char* sre2_strerror(int status);

/* Create a context bound to HIP device `hip_device`.  No device work happens
 * here; the device is first touched by the first compute call.
 * Errors: SRE2_EINVAL (out == NULL or hip_device < 0), SRE2_ENOMEM (host). */
int sre2_create(sre2_ctx** out, int hip_device);

/* Free the context and its device workspace (waits for the device).  NULL is
 * accepted. */
int sre2_destroy(sre2_ctx* ctx);

/* Upper bound for the two-pass scratch slab (N >= 15 in FP32, N >= 14 in
 * FP64); shifts are processed in chunks that fit it (at most 2^L shifts per
 * chunk, L = sre2_row_bits).  Default 32 GiB: larger chunks keep both passes
 * closer to the memory rate.  Values below one shift's slab are raised to one
 * slab.  When the device cannot allocate a call's slab, that call halves its
 * chunks until the slab fits (down to one shift per chunk); results never
 * depend on the chunk size. */
int sre2_set_scratch_limit(sre2_ctx* ctx, size_t bytes);

/* Row pairs of the plain and split forms (default on).  Pass 1 of the
 * two-pass path (N >= 15 in FP32, N >= 14 in FP64) transforms the rows of a
 * shift's 2^L x 2^(N-L) slab over their low L bits (Algorithm 1's transform
 * split into rows and columns).  Because f_x(k XOR x) = conj f_x(k) (the
 * summand of Eq. 3 at k and k XOR x), row r XOR (x >> L) of that slab is
 * row r with its L-bit input XOR-permuted and conjugated; for x >= 2^L the
 * library stores only the half of the rows whose bit j is clear (j a set bit
 * of x >> L) and pass 2 rebuilds the other half by sign flips, which halves
 * the memory traffic and the pass-1 work of those shifts.  In the plain
 * FP32 / FP64 forms the rebuilt rows equal those of the full slab bit for
 * bit, so every S_x, S and M2 is identical either way; in the split forms
 * (whose H_16 products on the matrix cores sum in an order the permutation
 * does not preserve) they are the exact images of the computed stored rows,
 * so results differ from the full slab's by rounding only, within the same
 * error bound.  enable = 0 keeps the full slab (for comparison).  The general
 * index and the spectrum (sre2_sre, sre2_pauli_spectrum) always take the
 * full slab.  Errors: SRE2_EINVAL (ctx == NULL). */
int sre2_set_row_pairs(sre2_ctx* ctx, int enable);

/* First shift x of an N-qubit evaluation that takes a half slab in the
 * two-pass path with the default settings (Hermitian pair; row pairs, which
 * start at 2^L, or in the plain forms where x >> L has a register row bit
 * of the pass-2 tile when that tile is a half-LDS one: 2^(L + 5) at N = 22
 * and 24 in FP32);
 * shifts below it take the full slab.  2^N when N uses the fused kernel.
 * Host-only.  Returns -1 for invalid arguments. */
int64_t sre2_half_slab_first_shift(int N, int form);

/* Device workspace (bytes) a call with these arguments grows the context to,
 * with the current default scratch limit.  0 for invalid arguments. */
size_t sre2_workspace_bytes(int N, int dtype, int form);

/* M2 of one state (Algorithm 1 over all 2^N shifts).
 *   psi       device, 2^N amplitudes of `dtype`
 *   out       device, SRE2_OUT_LEN doubles: M2, S, n, status
 *   partials  device, NULL or 2^N doubles: partials[x] = S_x (natural x order)
 * Errors: SRE2_EINVAL, SRE2_EDTYPE, SRE2_EFORM, SRE2_ENOMEM, SRE2_EHIP. */
int sre2_m2(sre2_ctx* ctx, const void* psi, int N, int dtype, int form, void* stream,
            double* out, double* partials);

/* Moments of the input as given (the state written in the computational
 * basis, main text): out[0] = n = sum_t |psi_t|^2, out[1] = sum_t |psi_t|^4
 * (the inverse participation ratio times n^2; by Parseval on the x = 0
 * transform, f_0 = |psi|^2, sum_z |W_0(z)|^2 = 2^N out[1]), out[2] = number
 * of non-finite amplitudes.  FP64 over the input's own element type, fixed
 * summation order (bitwise reproducible).  Stream-ordered, no host sync.
 *   psi  device, 2^N amplitudes of `dtype`;  out  device, 3 doubles
 * Errors: SRE2_EINVAL (null pointer, N outside [1, SRE2_MAX_N]), SRE2_EDTYPE,
 * SRE2_ENOMEM, SRE2_EHIP. */
int sre2_moments(sre2_ctx* ctx, const void* psi, int N, int dtype, void* stream, double* out);

/* Stabilizer Renyi entropy of any index alpha > 0 (Eq. 1):
 *   M_alpha = log2( sum_P |<P>|^(2 alpha) / 2^N ) / (1 - alpha),
 * and for alpha = 1 its limit M_1 = -sum_P Xi_P log2 Xi_P - N with
 * Xi_P = |<P>|^2 / 2^N (using sum_P |<P>|^2 = 2^N for a pure state).  The
 * same shift transforms as sre2_m2 feed sum w^alpha (or sum w log2 w),
 * w = |W_x(z)|^2, each term evaluated in the form's precision and summed in
 * FP64; the input need not be normalised (<P> = W / n).
 *   out  device, SRE2_OUT_LEN doubles: M_alpha, the Pauli sum (of w^alpha,
 *        or of w log2 w at alpha = 1, before normalisation), n, status
 * alpha = 2 runs exactly sre2_m2 (bitwise equal results).  The split form
 * supports alpha = 2 only.
 * Errors: as sre2_m2; SRE2_EINVAL for alpha not positive and finite;
 * SRE2_EFORM for the split form with alpha != 2. */
int sre2_sre(sre2_ctx* ctx, const void* psi, int N, int dtype, int form, double alpha,
             void* stream, double* out);

/* Pauli spectrum: histogram of q_P = |<P>|^2 over all 4^N Pauli strings.
 * String P goes to bin round(-log2 q_P) clamped to [0, nbins - 1]; q_P = 0
 * goes to the last bin, which thus holds everything below 2^-(nbins - 1.5).
 * Bin edges sit halfway (in log2) between powers of two, so the values
 * 2^-k of stabilizer and |T>-product states land at bin centres.  Values
 * within rounding of an edge may fall on either side; below the form's
 * precision floor (FP32: q ~ 1e-12) bins hold rounding noise.
 *   nbins   2 .. 64
 *   counts  device, nbins uint64 counters (cleared by the call)
 *   out     device, SRE2_OUT_LEN doubles: NaN, 0, n, status
 * Errors: as sre2_m2; SRE2_EINVAL for a bad nbins or null pointers;
 * SRE2_EFORM for the split form. */
int sre2_pauli_spectrum(sre2_ctx* ctx, const void* psi, int N, int dtype, int form, int nbins,
                        void* stream, uint64_t* counts, double* out);

/* Per-shift sums S_x for x in [x_begin, x_begin + x_count) only: the body of
 * Algorithm 1's loop over shifts for a sub-range of x.  The main text notes
 * that the shifts are independent of each other, so a range is the unit a
 * multi-GPU shard computes (each GPU takes a range and the totals add), and
 * the unit a checkpointed evaluation stores (sre2_m2_from_partials finishes
 * it).
 *   partials  device, x_count doubles: S_x in order of x
 * Errors: as sre2_m2, plus SRE2_EINVAL for a range outside [0, 2^N). */
int sre2_partials(sre2_ctx* ctx, const void* psi, int N, int dtype, int form, int64_t x_begin,
                  int64_t x_count, void* stream, double* partials);

/* M2 from per-shift sums computed earlier: the end of Algorithm 1 (the sum
 * over shifts and the logarithm) on S_x that the caller gathered, e.g. from
 * sre2_partials over shift ranges that were checkpointed and resumed, or
 * computed on several GPUs (the shifts are independent, main text).  The
 * norm n is computed from psi as in sre2_m2, and the sum over x runs in the
 * same fixed order, so S_x equal to those of sre2_m2 give a bitwise equal
 * result.
 *   psi       device, 2^N values of dtype (the state the S_x belong to)
 *   form      the form the S_x were computed in (it fixes the precision of
 *             the staged input and so of n)
 *   partials  device, 2^N doubles: S_x for x = 0 .. 2^N - 1, read only
 *   out       device, SRE2_OUT_LEN doubles: M2, S, n, status (as sre2_m2)
 * Errors: as sre2_m2; SRE2_EINVAL for null partials or out. */
int sre2_m2_from_partials(sre2_ctx* ctx, const void* psi, int N, int dtype, int form,
                          const double* partials, void* stream, double* out);

/* M2 of `count` states, each with its own N (mixed N allowed): Algorithm 1
 * applied to every state, the states sharing launches where they can.
 *   psi_list  HOST array of `count` device pointers
 *   N_list    HOST array of `count` qubit counts
 *   out       device, SRE2_OUT_LEN * count doubles (state i at out + 4 i)
 * States with the same N <= 14 (FP32 forms) / 13 (FP64 forms) are packed, up
 * to 64 per launch, into shared launches of the same kernels (the grid's y
 * index selects the state); larger N run one after another.  Each state's
 * result is bitwise identical to a single sre2_m2 call. */
int sre2_m2_batched(sre2_ctx* ctx, const void* const* psi_list, const int* N_list, int count,
                    int dtype, int form, void* stream, double* out);

/* ---- allocation-free evaluation ----------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 *
 * sre2_m2 without a context: the same launch sequence and kernels (results
 * bitwise equal to sre2_m2 on the same psi, N, dtype and form), with every
 * intermediate buffer carved out of one fixed device array of
 * SRE2_NOALLOC_SCRATCH_BYTES that the library holds on each device it runs
 * on until the process ends.  The call never allocates or frees device
 * memory (no hipMalloc, hipFree or allocating library routine).  The array's
 * device address is looked up once per device, on the first call there
 * (with that device current).
 *   hip_device  device to run on (made current for the call)
 *   psi, N, dtype, form, stream, out, partials: as sre2_m2
 * Two-pass shapes (N >= 15 in FP32 forms, 14 in FP64 forms) run in chunks
 * of as many shifts as the array holds, so large N is slower than sre2_m2.
 * Limit: the call is accepted when the input copy (dtype != the form's
 * precision), S_x (when partials == NULL), the reduction buffers and one
 * shift's slab fit the array - N <= 20 in the FP32 forms and N <= 19 in
 * the FP64 forms for complex64 input without a partials buffer; larger
 * problems return SRE2_ESCRATCH before any work is enqueued.
 * Every call on one device shares that device's array: calls that overlap
 * on one device (two host threads, or two streams whose work overlaps)
 * race and corrupt each other's results.  No part of the array needs to
 * start at zero (each kernel writes every entry it later reads).
 * Errors: SRE2_EINVAL (hip_device < 0, null psi or out, N out of range),
 * SRE2_EDTYPE, SRE2_EFORM, SRE2_ESCRATCH, SRE2_EHIP. */
#define SRE2_NOALLOC_SCRATCH_BYTES (32u << 20)
int sre2_m2_noalloc(int hip_device, const void* psi, int N, int dtype, int form, void* stream,
                    double* out, double* partials);

/* ---- measurement ------------------------------------------------------- */
/* Kernel classes for per-launch timing. */
#define SRE2_KIND_SHIFT 0 /* k_tiny / k_fused: whole transforms, N <= 14 (FP32), 13 (FP64) */
#define SRE2_KIND_PASS1 1 /* two-pass row transform (writes the scratch slab)          */
#define SRE2_KIND_PASS2 2 /* two-pass column transform + |W|^4 (reads the slab)        */
#define SRE2_KIND_AUX 3   /* conversion, norm, reductions, logarithm                    */
#define SRE2_KIND_COUNT 4

/* Enable (1) or disable (0) per-launch timing on this context: every later
 * launch is bracketed by a pair of HIP events recorded on the caller's stream.
 * Clears previously recorded pairs.  Errors: SRE2_EINVAL (ctx == NULL). */
int sre2_set_timing(sre2_ctx* ctx, int enable);

/* Wait for the recorded launches, then return per kernel class the summed
 * elapsed milliseconds ms[SRE2_KIND_COUNT] and launch counts
 * launches[SRE2_KIND_COUNT] (host arrays) since the last read; clears them.
 * Errors: SRE2_EINVAL, SRE2_EHIP. */
int sre2_timing_read(sre2_ctx* ctx, double* ms, int64_t* launches);

/* Two-pass geometry of a full evaluation with this context's scratch limit
 * and row-pair setting: shifts per chunk of the shifts x >= 2^L (most of an
 * evaluation; half slabs in the Hermitian-pair forms and, with row pairs, in
 * the plain and split forms; 0 when N uses the fused kernel) and column
 * groups per shift in pass 2.  Host-only.  Errors: SRE2_EINVAL. */
int sre2_chunking(sre2_ctx* ctx, int N, int form, int64_t* shifts_per_chunk, int* groups);

/* Row bits L of pass 1 for (N, form): the slab of NS = N bits (N - 1 in the
 * Hermitian-pair forms) is transformed as 2^(NS - L) rows of 2^L values, then
 * by columns; 0 when N is evaluated by the fused kernel, -1 for invalid
 * arguments. */
int sre2_row_bits(int N, int form);

/* ---- serving loop (continuous batching) ------------------------------- */
/* The paper's shift loop consists of independent units (main text: the
 * computation parallelises over shifts x), so evaluations of different
 * states can share the device in any interleaving without changing a result.
 * A server owns a worker thread, two HIP streams, a device arena of
 * hbm_budget_bytes and max_slots request slots.  Requests wait in one of two
 * FIFO lanes, small (N <= 14 in FP32 forms / 13 in FP64 forms) and large,
 * and each lane admits in order while a slot is free and the state fits the
 * arena (admission by HBM footprint; a full arena is backpressure).  Newly
 * admitted requests are enqueued at once, without waiting for running work:
 * small requests admitted together are packed by N into shared launches on
 * one stream; large ones run on a second stream, at most two enqueued at a
 * time, so a backlog of large requests waits in its lane and never delays a
 * small one.  A request's result is bitwise identical to a single sre2_m2
 * call on the same state and form. */
typedef struct sre2_server sre2_server;

#define SRE2_REQ_QUEUED 0    /* waiting for a slot / memory            */
#define SRE2_REQ_RUNNING 1   /* admitted, work enqueued on the device  */
#define SRE2_REQ_DONE 2      /* result available                       */
#define SRE2_REQ_CANCELLED 3 /* cancelled; result undefined            */
#define SRE2_REQ_FAILED 4    /* a HIP error hit its work               */

#define SRE2_SERVER_STAT_SUBMITTED 0
#define SRE2_SERVER_STAT_ADMITTED 1
#define SRE2_SERVER_STAT_COMPLETED 2
#define SRE2_SERVER_STAT_CANCELLED 3
#define SRE2_SERVER_STAT_PACKS 4         /* packed launches (small N)        */
#define SRE2_SERVER_STAT_PACKED_STATES 5 /* states that went through packs    */
#define SRE2_SERVER_STAT_SINGLES 6       /* single-state launches (large N)  */
#define SRE2_SERVER_STAT_PEAK_BYTES 7    /* peak arena bytes in use          */
#define SRE2_SERVER_STAT_PEAK_INFLIGHT 8 /* peak admitted, unfinished requests */
#define SRE2_SERVER_STAT_COUNT 9

/* Create a server on `hip_device` for one arithmetic form.
 * Errors: SRE2_EINVAL (null out, device < 0, max_slots < 1, budget < 1 MiB),
 * SRE2_EFORM, SRE2_ENOMEM (arena or result buffers), SRE2_EHIP. */
int sre2_server_create(sre2_server** out, int hip_device, int form, size_t hbm_budget_bytes,
                       int max_slots);

/* Submit one state of 2^N amplitudes of `dtype`; returns at once with a
 * ticket.  psi_on_device = 0: psi is host memory, copied before return (a
 * non-finite amplitude is rejected with SRE2_ENORM); 1: psi is device memory
 * whose producing work is already complete (the server copies it on its own
 * streams) and that stays valid until the request is done.
 * Errors: SRE2_EINVAL, SRE2_EDTYPE, SRE2_EFORM, SRE2_ENORM, SRE2_ENOMEM (the
 * state can never fit the arena), SRE2_EBUSY (server stopping). */
int sre2_server_submit(sre2_server* s, const void* psi, int N, int dtype, int psi_on_device,
                       uint64_t* ticket);

/* Non-blocking: *state = SRE2_REQ_*.  When the state is final (DONE,
 * CANCELLED, FAILED) the result (host, SRE2_OUT_LEN doubles: M2, S, n,
 * status; may be NULL) and the latency from submit to completion (seconds, may
 * be NULL) are returned and the ticket is released.
 * Errors: SRE2_EINVAL, SRE2_ENOTFOUND (unknown or released ticket). */
int sre2_server_poll(sre2_server* s, uint64_t ticket, int* state, double* result,
                     double* latency_s);

/* Cancel a request: a queued request is dropped before admission, a running
 * one finishes but reports SRE2_REQ_CANCELLED.  Errors: SRE2_EINVAL,
 * SRE2_ENOTFOUND. */
int sre2_server_cancel(sre2_server* s, uint64_t ticket);

/* Block until no request is queued or running, or the timeout passes
 * (SRE2_EBUSY).  Returns SRE2_EHIP if device work failed. */
int sre2_server_drain(sre2_server* s, double timeout_s);

/* Counters SRE2_SERVER_STAT_* (host array of `count` int64). */
int sre2_server_stats(sre2_server* s, int64_t* stats, int count);

/* Stop admitting, finish queued and running work, free everything.  NULL is
 * accepted.  Returns SRE2_EHIP if device work failed. */
int sre2_server_destroy(sre2_server* s);

/* ---- quench-dynamics simulator and snapshot pipeline ------------------
 * A complex128 state vector of N qubits (2 <= N <= 26) on one device, with
 * its own HIP stream, for the paper's two quench examples.  Qubit i is bit i
 * of the basis index, |0> = spin up (Z = +1).  All calls are asynchronous on
 * the simulator's stream except sre2_sim_state and the pipeline runs. */
typedef struct sre2_sim sre2_sim;

/* Creates the simulator in |0...0>.  Errors: SRE2_EINVAL, SRE2_ENOMEM,
 * SRE2_EHIP. */
int sre2_sim_create(sre2_sim** out, int hip_device, int N);
int sre2_sim_destroy(sre2_sim* s);

/* psi = prod_i (cos(theta_i/2)|0> + e^{i phi_i} sin(theta_i/2)|1>), the random
 * product initial state of the Hamiltonian-quench example.  theta, phi: host,
 * N doubles each.  Errors: SRE2_EINVAL (null or non-finite), SRE2_EHIP. */
int sre2_sim_product_state(sre2_sim* s, const double* theta, const double* phi);

/* Applies `count` two-qubit gates in order (the brickwork random-circuit
 * example).  gates: host, count x 16 complex (row-major 4x4 U[i][j],
 * interleaved re, im); the gate acts on the index j = bit(q0) + 2 bit(q1) of
 * its pair.  pairs: host, count x 2 distinct qubits (q0, q1).
 * Errors: SRE2_EINVAL (null, bad qubits), SRE2_EHIP. */
int sre2_sim_apply_gates(sre2_sim* s, const double* gates, const int* pairs, int count);

/* psi <- exp(-i H dt) psi for the TFIM with a longitudinal field on an open
 * chain, H = -J sum_{i=0}^{N-2} Z_i Z_{i+1} - hx sum_i X_i - hz sum_i Z_i,
 * by a Chebyshev expansion of the propagator cut below 1e-17 (FP64).
 * Errors: SRE2_EINVAL (non-finite parameters), SRE2_EHIP. */
int sre2_sim_tfim_step(sre2_sim* s, double J, double hx, double hz, double dt);

/* Copies the current state to dst (device, 2^N values of dtype; complex64 is
 * rounded from complex128) and waits for the simulator's stream. */
int sre2_sim_state(sre2_sim* s, int dtype, void* dst);

/* Snapshot pipelines: evolve `steps` steps and evaluate M2 (the server's
 * form) of the state before the first step and after every step, each
 * snapshot streamed to `srv` as a device input while the next step runs.
 * results: host, (steps + 1) x SRE2_OUT_LEN doubles, snapshot t at 4 t.
 * Blocks until every result is in.  The server must be owned by the caller
 * and be on the simulator's device.
 * Errors: SRE2_EINVAL, SRE2_ENOMEM, SRE2_EHIP, and any server error. */
int sre2_sim_run_tfim(sre2_sim* s, sre2_server* srv, double J, double hx, double hz, double dt,
                      int steps, int dtype, double* results);
/* gates: host, steps x gates_per_step x 16 complex (step t uses block t - 1);
 * pairs: host, gates_per_step x 2, the same bonds every step. */
int sre2_sim_run_circuit(sre2_sim* s, sre2_server* srv, const double* gates, const int* pairs,
                         int gates_per_step, int steps, int dtype, double* results);

#ifdef __cplusplus
}
#endif

#endif /* SRE2_H */
