/*
 * mrg32k3a_gpu.h -- C ABI of the MI355X (gfx950) MRG32k3a stream library.
 *
 * The library generates uniform random numbers in bulk from many independent,
 * reproducible streams of L'Ecuyer's combined multiple-recursive generator
 * MRG32k3a, placed by jump-ahead as in Passerat-Palmbach & Hill, HPCS 2012:
 *   sec. 4.1  MRG32k3a keeps 6 integers of state; its sequence is split into
 *             2^64 adjacent streams of 2^127 numbers, each divided into
 *             substreams of 2^76 numbers, one stream or substream per thread;
 *   sec. 2.3  sequence splitting needs a jump ahead; random spacing seeds the
 *             generator from different random states;
 *   sec. 5.1  a host-side initialisation allocates the device structures and
 *             prepares every thread's starting state before any kernel runs;
 *   sec. 5.2  on the device each thread draws the next number of its own
 *             stream (Listing 1 stores one float per thread).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Return value: MRG_OK (0) or a negative mrg_status.  A validation error
 *   returns before anything is enqueued; the text of the last error of the
 *   calling thread is available from mrg_last_error().
 * - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *   Every call that touches device memory is enqueued on it and is
 *   asynchronous unless stated otherwise.  Kernel faults surface as MRG_EHIP
 *   on a later call or at synchronisation.
 * - Device pointers (d_*) are device memory of the current HIP device, owned
 *   by the caller.  Host pointers (h_*) are ordinary host memory.
 * - A stream set and everything it owns live on the device that was current
 *   when it was created; calls on it must be made with that device current.
 * - States are 6 uint32 words per stream, oldest first in each component:
 *   (x1[n-3], x1[n-2], x1[n-1], x2[n-3], x2[n-2], x2[n-1]), with x1 words in
 *   [0, m1), x2 words in [0, m2), m1 = 2^32-209, m2 = 2^32-22853, and
 *   neither triple all zero.
 * - Output number k of a stream (k = 0, 1, ...) is the combined value after
 *   k+1 steps of its recurrence: z = (x1 - x2) mod m1, reported as m1 when 0,
 *   so uint32 outputs lie in [1, m1] (values above m1 never occur).
 *   FP64: z * NORM with NORM the double nearest 1/(m1+1) (one rounding).
 *   FP32: (2*((z-1) >> 9) + 1) * 2^-24 (exact).  Both lie in (0, 1) and are
 *   derived from the same integers, so all three dtypes carry one sequence.
 * - This library is not thread-safe per stream set: concurrent calls on one
 *   stream set must be ordered by the caller (e.g. by using one HIP stream).
 */
#ifndef MRG32K3A_GPU_H
#define MRG32K3A_GPU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mrg_status;
#define MRG_OK      0
#define MRG_EINVAL (-1)  /* bad argument: null pointer, invalid seed/state, bad dtype */
#define MRG_ENOMEM (-2)  /* device or host allocation failed */
#define MRG_EHIP   (-3)  /* a HIP runtime call failed (see mrg_last_error) */
#define MRG_ERANGE (-4)  /* stream range or size outside the stream set / limits */
#define MRG_ENODEV (-5)  /* no usable HIP device */
#define MRG_EBUSY  (-6)  /* serving: waiting on memory or time that did not come */

typedef enum { MRG_U32 = 0, MRG_F32 = 1, MRG_F64 = 2 } mrg_dtype;
typedef enum { MRG_STREAM_MAJOR = 0, MRG_INTERLEAVED = 1 } mrg_layout;

/* Opaque stream set: `n_streams` consecutive streams of one generator,
 * global stream indices [first_stream, first_stream + n_streams), with their
 * current states held on the device (6 planes of n_streams uint32). */
typedef struct mrg_streamset_s *mrg_streamset;

/* ---------------------------------------------------------------------- */
/* Stream sets (sec. 5.1 host initialisation; sec. 4.1 streams)            */
/* ---------------------------------------------------------------------- */

/* Create a stream set whose stream g (global index) starts at
 * A^(g * 2^127) * seed6, i.e. stream 0 is seed6 itself and streams are 2^127
 * outputs apart (sec. 4.1).  seed6 (host, 6 words) must be a valid state.
 * n_streams >= 1; first_stream + n_streams must not exceed 2^64.
 * Enqueues the start-state computation on `stream`; the set is usable on
 * that stream immediately.  *out receives the handle (caller owns it; free
 * with mrg_streamset_destroy).  Errors: MRG_EINVAL (null, invalid seed),
 * MRG_ERANGE (n_streams == 0 or index overflow), MRG_ENOMEM, MRG_EHIP. */
mrg_status mrg_streamset_create(mrg_streamset *out, uint64_t n_streams,
                                uint64_t first_stream, const uint32_t seed6[6],
                                void *stream);

/* As mrg_streamset_create, with the base state expanded from a 64-bit
 * master seed (random spacing, sec. 2.3) by mrg_seed_from_master. */
mrg_status mrg_streamset_create_seed64(mrg_streamset *out, uint64_t n_streams,
                                       uint64_t first_stream, uint64_t master_seed,
                                       void *stream);

/* Random spacing (sec. 2.3: the same generator started from different random
 * states): stream g (global index) starts at the state that
 * mrg_seed_from_master expands from output g (g = 0, 1, ...) of SplitMix64
 * seeded with master_seed, i.e. mix(master_seed + (g+1) * gamma).  Streams
 * are not spaced by a jump, so two of them may overlap after an unknown
 * number of outputs (for 2^20 streams of 2^40 outputs each the chance is
 * about 2^-90 of a period of 2^191).  Sizes, errors and ownership as
 * mrg_streamset_create; mrg_streamset_info reports an all-zero seed6. */
mrg_status mrg_streamset_create_random(mrg_streamset *out, uint64_t n_streams,
                                       uint64_t first_stream, uint64_t master_seed,
                                       void *stream);

/* A stream set of the counter-based generator Philox4x32-10 (Salmon, Moraes,
 * Dror & Shaw, SC 2011), the third family the paper embeds.  Stream g
 * (global index) has the 6 state words (position lo, hi, g lo, hi, key lo,
 * hi), position 0 at creation; its output number p is word p % 4 of the
 * ten-round Philox block of counter (p / 4 as two words, g as two words)
 * under `key`.  uint32 outputs are those words (all of [0, 2^32)); FP32 is
 * (2*(w >> 9) + 1) * 2^-24 and FP64 (2*w + 1) * 2^-33 (exact, in (0, 1)).
 * mrg_fill, mrg_jump and mrg_jump_uniform work on such a set (a jump by e
 * adds e mod 2^64 to the position), as do mrg_get_states / mrg_set_states
 * (any 6 words are a state).  Substream jumps, leapfrog, batches and
 * mrg::Stream are MRG32k3a only and return MRG_EINVAL.  Sizes, errors and
 * ownership as mrg_streamset_create; mrg_streamset_info reports an all-zero
 * seed6.
 * Parity unpinned: the two round multipliers (0xD2511F53, 0xCD9E8D57) are
 * typed from the published definition; no known-answer vector was available
 * to check them, so agreement with other Philox4x32-10 implementations rests
 * on those two constants (the oracle and the library agree bit for bit). */
mrg_status mrg_streamset_create_philox(mrg_streamset *out, uint64_t n_streams,
                                       uint64_t first_stream, uint64_t key, void *stream);

/* ---------------------------------------------------------------------- */
/* TinyMT32 stream sets (sec. 4.2: the hybrid of parameterisation and      */
/* sequence splitting)                                                     */
/* ---------------------------------------------------------------------- */
/* TinyMT32 (Saito & Matsumoto, 2011) has a 127-bit state and period
 * 2^127 - 1 for a good parameter set (mat1, mat2, tmat).  In the paper's
 * hybrid the threads of a group share one parameter set and each takes its
 * own sub-stream of that generator by sequence splitting.  Here global
 * stream g uses parameter set q = g / per_param and starts
 * (g % per_param) * 2^64 outputs past the set's base status, the published
 * seeding from the 32-bit seed (uint32)SplitMix64_q(master_seed) (output q,
 * as mrg_streamset_create_random numbers them).  A stream's six state words
 * are (s0, s1, s2, s3, q, 0).
 *
 * Parameter sets replace Dynamic Creator's files: candidate c of the search
 * under master_seed takes SplitMix64 outputs 2c and 2c+1 of master_seed + 1
 * (mat1 | mat2 << 32 = the first, tmat = the low half of the second), and a
 * candidate is accepted when the characteristic polynomial of its
 * transition (Berlekamp-Massey on 254 output bits) has degree 127 and is
 * irreducible (Rabin's test), which for the Mersenne exponent 127 gives the
 * full period.  Parameter set q is the q-th accepted candidate.
 *
 * uint32 outputs are the tempered words (all of [0, 2^32)); FP32
 * (2*(w >> 9) + 1) * 2^-24 and FP64 (2*w + 1) * 2^-33, exact, in (0, 1).
 * mrg_fill (both layouts), mrg_jump / mrg_jump_uniform (polynomial jumps,
 * any exponent below 2^192), mrg_get_states / mrg_set_states work on such a
 * set; substream jumps, leapfrog and batches return MRG_EINVAL.
 * Parity unpinned: no known-answer output of TinyMT32 was available, so the
 * transition, tempering and seeding rest on their written definition (the
 * oracle and the library agree bit for bit). */

/* Test candidates c0 .. c0+n-1 of the search under master_seed on the
 * device: d_flags[i] (device, n uint32) = L | accepted << 16, L the linear
 * complexity found by Berlekamp-Massey; d_phi (device, 4n uint32, may be
 * NULL) receives each characteristic polynomial (bit b of word k the
 * coefficient of x^(32k+b); written when L = 127, zero otherwise).
 * Asynchronous on `stream`.  n <= 2^31.  Errors: MRG_EINVAL (null flags,
 * pointers not device memory), MRG_ERANGE, MRG_EHIP. */
mrg_status mrg_tinymt_test_candidates(uint64_t master_seed, uint64_t c0, uint64_t n,
                                      uint32_t *d_flags, uint32_t *d_phi, void *stream);

/* Parameter sets 0 .. count-1 of the search under master_seed: h_params
 * (host, 3*count words: mat1, mat2, tmat) and, if not NULL, h_cand (host,
 * count words) their candidate numbers.  Candidates are tested on the
 * device in batches; synchronous on `stream`.  count <= 2^20.  Errors:
 * MRG_EINVAL, MRG_ERANGE, MRG_ENOMEM, MRG_EHIP. */
mrg_status mrg_tinymt_search(uint64_t master_seed, uint64_t count, uint32_t *h_params,
                             uint64_t *h_cand, void *stream);

/* Create a TinyMT32 stream set of n_streams streams from global index
 * first_stream, per_param consecutive global streams per parameter set (a
 * workgroup's threads, in the paper's hybrid).  The sets used, q0 =
 * first_stream / per_param .. qlast = (first_stream + n_streams - 1) /
 * per_param (at most 2^20 of them, qlast < 2^32), come from h_params (host,
 * 3 words per set, holding sets params_first .. params_first + n_params - 1,
 * which must cover q0 .. qlast, else MRG_ERANGE) or, when h_params is NULL,
 * from mrg_tinymt_search(master_seed, qlast + 1).  Every set is checked on
 * the device (MRG_EINVAL names a set without a degree-127 irreducible
 * characteristic polynomial) and gets a record (parameters, polynomial,
 * x^(2^i) mod phi for i < 192).  Synchronous on `stream`.  Sizes as
 * mrg_streamset_create; per_param >= 1.  Errors: MRG_EINVAL, MRG_ERANGE,
 * MRG_ENOMEM, MRG_EHIP. */
mrg_status mrg_streamset_create_tinymt(mrg_streamset *out, uint64_t n_streams,
                                       uint64_t first_stream, uint64_t per_param,
                                       uint64_t master_seed, const uint32_t *h_params,
                                       uint64_t params_first, uint64_t n_params, void *stream);

/* Description of a TinyMT32 set for user kernels (tinymt_device.h): streams
 * per parameter set, global index q0 of the first set held, number of sets,
 * and the device address of their records (n_sets * 776 uint32, owned by
 * the set, valid until destroy).  Any output may be NULL.  MRG_EINVAL for a
 * set of another generator. */
mrg_status mrg_streamset_tinymt_info(mrg_streamset ss, uint64_t *per_param, uint64_t *q0,
                                     uint64_t *n_sets, const void **d_records);

/* Release the stream set and its device memory (sec. 5.1 release()).
 * Synchronises the device work the library enqueued on the set first.
 * NULL is accepted and ignored. */
mrg_status mrg_streamset_destroy(mrg_streamset ss);

/* Host-side metadata of a stream set: size, first global index, base state.
 * Any output pointer may be NULL. */
mrg_status mrg_streamset_info(mrg_streamset ss, uint64_t *n_streams,
                              uint64_t *first_stream, uint32_t seed6[6]);

/* Device pointer of the 6 state planes ([6][n_streams] uint32, plane c holds
 * word c of every stream).  Owned by the stream set; valid until destroy.
 * User kernels draw from these states with mrg::Stream (mrg32k3a_device.h). */
mrg_status mrg_streamset_states_ptr(mrg_streamset ss, void **d_states);

/* Device pointer of the windowed jump tables of the set's device (sec. 2.3
 * jump-ahead): [2][48][16][9] uint32, entry (c, w, d) = A_c^(d * 16^w) mod m_c
 * row-major.  Owned by the library; valid until the process ends.  User
 * kernels pass it to mrg::Stream::jump / substream (mrg32k3a_device.h). */
mrg_status mrg_streamset_tables_ptr(mrg_streamset ss, const void **d_tables);

/* ---------------------------------------------------------------------- */
/* Jump ahead (sec. 2.3 sequence splitting; sec. 4.1 substreams of 2^76)   */
/* Streams [first, first+count) of the set (indices relative to the set).  */
/* ---------------------------------------------------------------------- */

/* Advance every stream in the range by its own exponent: stream first+i is
 * moved e_i outputs ahead, e_i given as 3 little-endian uint64 words at
 * d_exp[3*i .. 3*i+2] (device memory, e_i < 2^192).  Uses 4-bit windowed
 * tables of A^(d * 16^w) mod m staged in LDS.  count == 0 is a no-op.
 * Errors: MRG_EINVAL (null, or d_exp not device memory of the set's device),
 * MRG_ERANGE (range outside the set, or the 24 * count bytes at d_exp run
 * past the end of their allocation). */
mrg_status mrg_jump(mrg_streamset ss, uint64_t first, uint64_t count,
                    const uint64_t *d_exp, void *stream);

/* Advance every stream in the range by the same exponent e (3 host words,
 * little-endian).  The matrix A^e is formed on the host; one matrix-vector
 * product per component per stream on the device. */
mrg_status mrg_jump_uniform(mrg_streamset ss, uint64_t first, uint64_t count,
                            const uint64_t h_exp[3], void *stream);

/* Advance every stream in the range by k substreams, i.e. k * 2^76 outputs
 * (sec. 4.1).  k < 2^115. */
mrg_status mrg_jump_substreams(mrg_streamset ss, uint64_t first, uint64_t count,
                               uint64_t k, void *stream);

/* ---------------------------------------------------------------------- */
/* Bulk generation (sec. 5.2 next(); Listing 1 pattern)                    */
/* ---------------------------------------------------------------------- */

/* Write n_per_stream outputs of each stream first .. first+count-1 to d_out
 * and advance each of those streams by n_per_stream.
 *   layout MRG_STREAM_MAJOR: d_out[s * n_per_stream + k] (a [count, n] array)
 *   layout MRG_INTERLEAVED : d_out[k * count + s]        (a [n, count] array)
 * d_out must hold count * n_per_stream elements of the dtype (4 bytes for
 * MRG_U32/MRG_F32, 8 for MRG_F64) and be aligned to the element size (any
 * row start works: each row is written in whole 128-byte lines after its
 * first line boundary).  n_per_stream == 0 or count == 0
 * is a no-op.  Errors: MRG_EINVAL (null d_out, bad dtype/layout,
 * misaligned, d_out not device (or managed) memory of the set's device),
 * MRG_ERANGE (range outside the set, or the output runs past the end of the
 * allocation holding d_out).  Nothing is enqueued on an error. */
mrg_status mrg_fill(mrg_streamset ss, uint64_t first, uint64_t count,
                    uint64_t n_per_stream, mrg_dtype dtype, mrg_layout layout,
                    void *d_out, void *stream);

/* Leapfrog (sec. 2.3): the outputs of stream s of the set dealt to
 * `players` players like cards, `per_player` each: card k of player t is
 * output t + k * players of the stream.  With P = players, K = per_player:
 *   layout MRG_STREAM_MAJOR: d_out[t * K + k] (a [P, K] array: each
 *                            player's cards in a row; full speed needs
 *                            K >= 64, since 64 adjacent cards of one player
 *                            make one store)
 *   layout MRG_INTERLEAVED : d_out[k * P + t] (a [K, P] array: the stream's
 *                            outputs in order, generated by sequence
 *                            splitting over the whole device)
 * Advances stream s by P * K.  d_out holds P * K elements of the dtype,
 * aligned to the element size.  P == 0 or K == 0 is a no-op.  Errors:
 * MRG_EINVAL (null d_out, bad dtype/layout, misaligned, d_out not device
 * memory of the set's device), MRG_ERANGE (s outside the set, P * K *
 * element size above 2^64 - 1 or past the end of d_out's allocation). */
mrg_status mrg_fill_leapfrog(mrg_streamset ss, uint64_t s, uint64_t players,
                             uint64_t per_player, mrg_dtype dtype, mrg_layout layout,
                             void *d_out, void *stream);

/* Copy the states of streams [first, first+count) to host memory h_out
 * ([count][6] uint32).  Synchronous with respect to `stream` (waits for it). */
mrg_status mrg_get_states(mrg_streamset ss, uint64_t first, uint64_t count,
                          uint32_t *h_out, void *stream);

/* Overwrite the states of streams [first, first+count) from host memory
 * h_in ([count][6] uint32, each a valid state; checked on the host, else
 * MRG_EINVAL and nothing is written).  Synchronous with respect to `stream`. */
mrg_status mrg_set_states(mrg_streamset ss, uint64_t first, uint64_t count,
                          const uint32_t *h_in, void *stream);

/* ---------------------------------------------------------------------- */
/* Batched generation: many fill requests in one graph of persistent launches */
/* ---------------------------------------------------------------------- */

/* Request flag: the request's streams are substreams (sec. 4.1) of ONE
 * stream of the set -- stream j of the request starts at that stream's state
 * jumped by (substream0 + j) * 2^76 -- and the stored state is not changed. */
#define MRG_REQ_SUBSTREAMS 1u

/* One generation request.  Without flags it is exactly
 * mrg_fill(set, first, count, n_per_stream, dtype, MRG_STREAM_MAJOR, d_out):
 * streams first .. first+count-1 of the set, advanced by n_per_stream.
 * With MRG_REQ_SUBSTREAMS, `first` names the one stream and count substreams
 * starting at substream0 are generated (substream0 + count - 1 must fit in
 * 64 bits, else MRG_ERANGE).  d_out is device memory holding
 * count * n_per_stream elements of dtype, stream-major, aligned to the
 * element size (rows starting on 128-byte lines are written fastest).
 * Requests with count or n_per_stream equal to 0 are skipped. */
typedef struct {
    uint64_t first;
    uint64_t count;
    uint64_t n_per_stream;
    uint64_t substream0;
    void *d_out;
    int32_t dtype;    /* mrg_dtype */
    uint32_t flags;   /* 0 or MRG_REQ_SUBSTREAMS */
} mrg_request;

#define MRG_SCHEDULE_DYNAMIC 1u /* waves claim work items from an atomic counter */
#define MRG_SCHEDULE_STATIC 2u  /* wave w takes items w, w + grid, ... */

/* Work decomposition of a batch (0 in any field selects its default). */
typedef struct {
    uint64_t segment_bytes;   /* output bytes per work item of a long stream (256 KiB) */
    uint64_t wave_min_bytes;  /* streams of at least this many output bytes get a whole
                                 wave per segment, shorter ones one lane each (16 KiB) */
    uint32_t waves_per_cu;    /* persistent one-wave workgroups per compute unit (16) */
    uint32_t schedule;        /* MRG_SCHEDULE_DYNAMIC (default) or MRG_SCHEDULE_STATIC */
} mrg_batch_config;

typedef struct {
    uint64_t requests;        /* non-empty requests */
    uint64_t items;           /* work items */
    uint64_t samples;         /* outputs per run */
    uint64_t bytes;           /* output bytes per run */
    uint64_t scratch_states;  /* end states staged before copy-back */
    uint32_t grid;            /* persistent workgroups */
    uint32_t pad;
    mrg_batch_config config;  /* effective configuration */
} mrg_batch_info_t;

typedef struct mrg_batch_s *mrg_batch;

/* Plan a batch over stream set ss: validate the requests (plain requests
 * must cover disjoint stream ranges and no substream request may name a
 * stream that a plain request advances, else MRG_EINVAL), cut them into
 * one-wave work items (a segment of one stream, whole streams packed about a
 * segment per item, or up to 16 blocks of 64 streams shorter than
 * wave_min_bytes, one per lane), group them into at most one launch per
 * dtype of the long streams' items, the first (least output) led by the
 * short streams' items of every dtype, largest first, and capture one
 * hipGraph (per group a counter reset and a persistent kernel, then the
 * copy-back of end states).  Every non-empty request's d_out must be device
 * memory of the set's device holding its output inside one allocation (else
 * MRG_EINVAL / MRG_ERANGE naming the request).  reqs is copied; cfg may be
 * NULL.  The plan refers to ss and to the output buffers, which must outlive
 * it.  Free with mrg_batch_destroy. */
mrg_status mrg_batch_create(mrg_batch *out, mrg_streamset ss, const mrg_request *reqs,
                            uint64_t n_reqs, const mrg_batch_config *cfg);

/* Run the batch: one hipGraph launch on `stream` (asynchronous).  Every run
 * continues the plain requests' streams, like repeating the fills. */
mrg_status mrg_batch_run(mrg_batch b, void *stream);

/* Same kernels launched directly on `stream` instead of through the graph. */
mrg_status mrg_batch_run_direct(mrg_batch b, void *stream);

/* Reference schedule with the same results: one launch per request (plain
 * requests through mrg_fill, substream requests through the batch kernel
 * restricted to that request). */
mrg_status mrg_batch_run_per_request(mrg_batch b, void *stream);

mrg_status mrg_batch_info(mrg_batch b, mrg_batch_info_t *info);

/* One launch group of a batch plan (mrg_batch_plan_groups). */
typedef struct {
    int32_t dtype;         /* dtype of the group's wave items */
    int32_t rows;          /* 1: the group is led by the row items of every dtype */
    uint64_t requests;     /* requests in the group */
    uint64_t items;        /* work items */
    uint64_t row_items;    /* of which row items (they come first) */
    uint64_t bytes;        /* output bytes of the group's requests */
} mrg_plan_group;

/* The launch groups that mrg_batch_create would capture for these requests
 * under cfg (NULL: defaults), computed on the host alone: no stream set,
 * device or output memory is touched, d_out is not read, and the requests
 * are not validated against a stream set (dtype and flags are checked).
 * groups receives up to 3 groups in launch order (*n_groups of them); when
 * pos is not NULL, pos[i] is input request i's index in the grouped order
 * (items are claimed in that order; UINT64_MAX for empty requests), and
 * when items is not NULL, items[i] its work items.  For tests and tools. */
mrg_status mrg_batch_plan_groups(const mrg_request *reqs, uint64_t n_reqs,
                                 const mrg_batch_config *cfg, mrg_plan_group *groups,
                                 uint32_t *n_groups, uint64_t *pos, uint64_t *items);

/* Completion time of every request in the last mrg_batch_run or
 * mrg_batch_run_direct: h_ms[i] (n_reqs doubles, host memory, input order)
 * receives the milliseconds from the earliest workgroup start of that run to
 * the device wall clock read when request i's last work item ended (0 for
 * requests with count or n_per_stream 0).  Waits for `stream` first. */
mrg_status mrg_batch_request_times(mrg_batch b, void *stream, double *h_ms);

/* Time each candidate configuration (reps runs after one warm-up, on
 * `stream`), keep the fastest and re-plan with it.  The stream states are
 * restored afterwards, so autotuning has no visible effect on results.
 * best_out (may be NULL) receives the chosen index; ms_out (may be NULL,
 * else n_cands floats) the average milliseconds per run of each candidate.
 * Synchronous. */
mrg_status mrg_batch_autotune(mrg_batch b, const mrg_batch_config *cands, uint32_t n_cands,
                              uint32_t reps, void *stream, uint32_t *best_out, float *ms_out);

/* Release the plan (synchronises the device first).  NULL is ignored. */
mrg_status mrg_batch_destroy(mrg_batch b);

/* Bytes of the fixed device array behind mrg_batch_run_noalloc (per device,
 * held until the process ends). */
#define MRG_NOALLOC_SCRATCH_BYTES (16u << 20)

/* For callers that cannot allocate device memory (serving loops and
 * harnesses that forbid hipMalloc, code that must not grow the device heap):
 * plan and run one batch -- the same validation, work items, kernels and
 * results as mrg_batch_create(ss, reqs, n_reqs, cfg) followed by
 * mrg_batch_run and mrg_batch_destroy -- without any device or pinned
 * allocation.  The request descriptors, item prefixes, claim counters and the
 * staged end states of multi-segment streams go into one fixed device array
 * of MRG_NOALLOC_SCRATCH_BYTES bytes; a batch needing more (about 80 bytes per
 * request plus 24 bytes per stream of more than one segment) returns
 * MRG_ERANGE before anything is enqueued, naming the size it needs.  The
 * caller passes the stream set, the requests (host memory, read during the
 * call) and the outputs, as for mrg_batch_create.  Host planning uses ordinary
 * heap memory.  The call waits for earlier work on `stream`, uploads the plan
 * (waiting for that copy), then enqueues the kernels and returns; no
 * completion stamps are kept.  Every call on one device shares the array, and
 * each call overwrites what the last one left there: calls that may overlap
 * on one device (other host threads, other streams) race and must be ordered
 * by the caller. */
mrg_status mrg_batch_run_noalloc(mrg_streamset ss, const mrg_request *reqs, uint64_t n_reqs,
                                 const mrg_batch_config *cfg, void *stream);

/* ---------------------------------------------------------------------- */
/* Serving: continuous batching of client requests                         */
/* ---------------------------------------------------------------------- */
/* Each client c owns global stream first_stream + c (its state stays on the
 * device and never changes) and a substream cursor: a request of client c
 * for k streams gets the client's next k substreams (sec. 4.1), assigned at
 * admission.  A scheduler thread admits queued requests in arrival order,
 * separately for small and large ones (big_request_bytes), while the output
 * arena has room, launches every admitted group as one persistent batch
 * launch on the next free HIP stream of its class (max_inflight streams, a
 * quarter of them for large requests; groups overlap on the device), and
 * retires them when their completion events fire.  A request's output is a [k, n] stream-major array of its dtype in
 * the arena, identical to generating that request alone. */
typedef struct mrg_server_s *mrg_server;

typedef struct {
    uint64_t n_clients;     /* client streams */
    uint64_t first_stream;  /* global index of client 0's stream */
    uint64_t master_seed;   /* base state via mrg_seed_from_master */
    uint64_t arena_bytes;   /* device output arena: the admission cap (rounded down to a
                               multiple of 256 bytes, the arena's block unit; at least 256) */
    uint32_t max_inflight;  /* HIP streams, i.e. groups in flight (0: 8; at most 64) */
    uint32_t max_batch;     /* requests per group (0: 4096; at most 2^20) */
    uint32_t waves_per_cu;  /* persistent workgroups per CU per tick kernel (0: 8) */
    uint32_t auto_release;  /* 1: free each output when it completes (throughput runs) */
    uint32_t pad;
    uint64_t big_request_bytes;  /* requests of at least this many output bytes queue
                                    apart and run on a quarter of the streams, so that
                                    smaller ones never share a tick with them
                                    (0: 64 MiB; UINT64_MAX: one class) */
} mrg_server_config;

typedef struct {
    uint64_t ticket, client, n_streams, n_per_stream, substream0;
    void *d_out;            /* arena pointer (NULL with auto_release) */
    int32_t dtype;
    int32_t pad;
    double latency_s;       /* completion seen by the scheduler - submission */
    double queue_s;         /* admission - submission */
    double t_submit;        /* submission time (steady clock, seconds) */
} mrg_server_result;

typedef struct {
    uint64_t pending, inflight, completed, ticks, samples, bytes, arena_used, arena_bytes;
} mrg_server_stats_t;

typedef struct {
    double t;               /* arrival time, seconds from the start of the trace */
    uint64_t client, n_streams, n_per_stream;
    int32_t dtype;
    int32_t pad;
} mrg_arrival;

/* Create the client stream set, the arena, the streams and start the
 * scheduler thread (on the device current at the call). */
mrg_status mrg_server_create(mrg_server *out, const mrg_server_config *cfg);

/* Queue a request (thread-safe).  *ticket (may be NULL) identifies it.
 * MRG_ERANGE if it can never fit in the arena. */
mrg_status mrg_server_submit(mrg_server s, uint64_t client, uint64_t n_streams,
                             uint64_t n_per_stream, int32_t dtype, uint64_t *ticket);

/* Take up to max_out finished requests (oldest first); *n_out receives the
 * count.  Returns the scheduler's error status, if it stopped on one. */
mrg_status mrg_server_poll(mrg_server s, mrg_server_result *out, uint64_t max_out,
                           uint64_t *n_out);

/* Free a finished request's output (not needed with auto_release). */
mrg_status mrg_server_release(mrg_server s, uint64_t ticket);

/* Copy the first `bytes` of a finished, held output to host memory
 * (synchronous). */
mrg_status mrg_server_copy_output(mrg_server s, uint64_t ticket, void *h_dst, uint64_t bytes);

mrg_status mrg_server_stats(mrg_server s, mrg_server_stats_t *st);

/* Wait until nothing is queued or in flight (MRG_EBUSY on timeout or when
 * the queue waits for outputs that are not released). */
mrg_status mrg_server_drain(mrg_server s, double timeout_s);

/* Replay a trace: submit arrival i at time arr[i].t * time_scale after the
 * call (arrivals sorted by t), then drain.  *wall_s (may be NULL) receives
 * the elapsed time.  The results are collected with mrg_server_poll. */
mrg_status mrg_server_run_trace(mrg_server s, const mrg_arrival *arr, uint64_t n,
                                double time_scale, double *wall_s);

/* A client's (fixed) stream state and its next substream. */
mrg_status mrg_server_client_state(mrg_server s, uint64_t client, uint32_t out6[6],
                                   uint64_t *next_substream);

/* Stop the scheduler after the groups in flight, drop queued requests and
 * free everything.  NULL is ignored. */
mrg_status mrg_server_destroy(mrg_server s);

/* ---------------------------------------------------------------------- */
/* Host-only helpers (no device work; usable without a GPU)               */
/* ---------------------------------------------------------------------- */

/* Expand a 64-bit master seed into a valid 6-word state (random spacing,
 * sec. 2.3): successive SplitMix64 outputs (Steele, Lea & Flood 2014) taken
 * mod m1 for words 0-2 and mod m2 for words 3-5; an all-zero triple is
 * drawn again. */
mrg_status mrg_seed_from_master(uint64_t master_seed, uint32_t out6[6]);

/* A_c^e mod m_c (row-major 3x3) for component c in {0, 1} and a 192-bit
 * exponent e (3 little-endian words); A_c is the companion matrix acting on
 * the column (x[n-3], x[n-2], x[n-1]) (sec. 2.3 jump ahead). */
mrg_status mrg_jump_matrix(int component, const uint64_t h_exp[3], uint32_t out9[9]);

/* Check a host state: MRG_OK if valid, else MRG_EINVAL. */
mrg_status mrg_state_check(const uint32_t state6[6]);

/* Process-wide tuning of the generation kernels (no effect on results):
 *   "engine"     0 = 32-bit integer arithmetic with lazy residues,
 *                1 = binary64 arithmetic on integer-valued doubles (default);
 *   "tile_bytes" bytes per stream per LDS tile of the lane-per-stream
 *                stream-major fill, 128 or 256, or 0 (default: 128 for rows
 *                shorter than 1 KiB, else 256);
 *   "strategy"   stream-major fill: 0 = automatic (default: one wave per
 *                stream when a stream has at least 64 x 128 bytes of output,
 *                except rows under 16 KiB that are not whole chunks on
 *                128-byte lines when at least 2^17 streams are filled; else
 *                one lane per stream), 1 = always lane per stream,
 *                2 = always wave per stream;
 *   "coop_wgs_per_cu" wave-per-stream fill: one-wave workgroups per compute
 *                unit, each looping over stream groups (0 = one workgroup
 *                per group, the default), 0 .. 1024;
 *   "coop_order" wave-per-stream fill: order of stream groups over the XCDs,
 *                0 (default) chunked: 64 consecutive groups per XCD in turn,
 *                all XCDs moving through memory together; 1: one contiguous
 *                range per XCD;
 *   "coop_lanes" wave-per-stream fill: lanes per stream, 64, 32, 16 or 8
 *                (64/coop_lanes streams share a wave), or 0 (the default:
 *                16 for rows under 64 KiB, else 64).
 * Unknown keys or values: MRG_EINVAL.  Takes effect for later launches. */
mrg_status mrg_config_set(const char *key, int64_t value);
mrg_status mrg_config_get(const char *key, int64_t *value);

/* Store-only bandwidth probe (a measurement aid, not part of the method):
 * writes `bytes` of filler to device memory d_out on `stream` with the store
 * pattern of the fills but no generation work, so that a fill's write rate can
 * be compared with what its stores alone attain.
 *   pattern 0: streaming 16-byte stores, one pass in address order (bytes a
 *              multiple of 16, d_out 16-byte aligned);
 *   pattern 1: the wave-per-stream fill's geometry at 16 lanes per stream and
 *              1 KiB per lane: four 16 KiB rows per wave, two 128-byte lines
 *              per lane staged in LDS per flush, each store instruction four
 *              runs of two adjacent lines (bytes a multiple of 65536, d_out
 *              128-byte aligned);
 *   pattern 2: the same 64 KiB per wave as runs of 8 lines (1 KiB) per store
 *              instruction (sizes and alignment as pattern 1);
 *   pattern 3: as pattern 1 with one line per lane per flush (8 single lines
 *              1 KiB apart per store instruction).
 * Other patterns or sizes, or d_out not device memory of the current device:
 * MRG_EINVAL.  Asynchronous. */
mrg_status mrg_write_probe(void *d_out, uint64_t bytes, int32_t pattern, void *stream);

/* Static text of a status code. */
const char *mrg_status_string(mrg_status s);

/* Text of the last error raised on the calling thread ("" if none). */
const char *mrg_last_error(void);

/* Library version as an integer (major*10000 + minor*100 + patch). */
int32_t mrg_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MRG32K3A_GPU_H */
