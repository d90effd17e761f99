/*
 * prng.h - C ABI of libprng, bulk uniform pseudo-random number generation on
 * AMD Instinct MI355X (gfx950) for the six generators studied in
 * V. Demchik, "Pseudo-random number generators for Monte Carlo simulations on
 * Graphics Processing Units", arXiv:1003.1898, and two more members of the
 * linear congruential family it describes (DRAND48, RANNYU).
 *
 * Model (Section 3.1, "General implementation scheme"): every generator
 * instance owns its own lag table in GPU memory and produces an independent
 * sequence; a kernel loads the table once (initialisation), produces numbers
 * (generation) and writes the table back (finalisation).  Here one
 * generator object holds N such streams; `prng_generate` produces the next
 * `count` numbers of every stream.
 *
 * Conventions for every entry point:
 *  - Return value: PRNG_OK (0) or a negative PRNG_E* code; a thread-local
 *    message is available from prng_last_error().  No C++ exception crosses
 *    this boundary.
 *  - Device memory (state buffers, outputs, sums, histograms) is owned by the
 *    caller and passed as plain device pointers.  The library owns only host
 *    metadata; it never frees caller memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the legacy default
 *    stream).  Work is enqueued asynchronously on it unless stated otherwise.
 *    Calls that share a generator object must be ordered by the caller
 *    (same stream or events); concurrent calls on one object race.
 *  - Asynchronous device faults surface as PRNG_EHIP from a later call that
 *    synchronises.
 *
 * Native integer draw u of each generator and its bit width b:
 *   GGL 31 bits, u in [1, 2^31-2];  XOR128 32;  RANECU 31, u in [1, 2147483562];
 *   RANMAR 24;  RANLUX 24;  MT19937 32;  DRAND48 and RANNYU 32, the top 32
 *   bits X >> 16 of the 48-bit state X.
 * Output element types:
 *   PRNG_U32  u itself (RANMAR/RANLUX values are < 2^24).
 *   PRNG_F32  (u >> (b-24)) * 2^-24, exact, in [0, 1).
 *   PRNG_F64  two consecutive draws u1, u2 per element (Section 3.1 asks for
 *             several single draws per double rather than a widening
 *             conversion): ((u1 >> (b-27)) 2^26 + (u2 >> (b-26))) 2^-53 for
 *             b >= 27 (53 random bits), (u1 2^24 + u2) 2^-48 for b = 24.
 *   PRNG_F32_PAPER  float, each generator's own scaling as the paper's kernels
 *             write it, evaluated in fp32 (the integer rounded to nearest):
 *             GGL x / 2147483647.0 (Section 3.2), XOR128 w / 4294967295.0
 *             (3.3), RANECU Z * 2^-31 (3.4), RANMAR and RANLUX X * 2^-24 (3.5,
 *             3.6), MT19937 (y + 0.5) / 4294967296.0 (3.7).  Values can be 1.0
 *             (GGL, XOR128, MT19937).  prng_generate and prng_generate_packed4
 *             only (the table and the server reject it); DRAND48 and RANNYU
 *             have no such rule (PRNG_EUNSUPPORTED).
 * Outputs are stream-major: element i of stream s is out[s*count + i].
 */
#ifndef PRNG_H
#define PRNG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Generator kinds (Section 3.2-3.7; definitions in Appendix A). */
typedef enum {
  PRNG_GGL = 1,     /* MLCG x <- 16807 x mod (2^31-1), Appendix A.1            */
  PRNG_XOR128 = 2,  /* Marsaglia xorshift on 4 x 32 bits, Appendix A.4.2       */
  PRNG_RANECU = 3,  /* L'Ecuyer combination of two MLCGs, Appendix A.4.1       */
  PRNG_RANMAR = 4,  /* LFG(97,33,-) mod 2^24 combined with C_n, Appendix A.4.4  */
  PRNG_RANLUX = 5,  /* SWB(24,10) mod 2^24 with luxury skip p, Appendix A.4.5-6 */
  PRNG_MT19937 = 6, /* Mersenne twister, Appendix A.4.3                        */
  PRNG_DRAND48 = 7, /* LCG x <- 25214903917 x + 11 mod 2^48, Appendix A.1 (eq. DRAND48) */
  PRNG_RANNYU = 8   /* MLCG x <- 31167285 x mod 2^48, Section 2 (Chroma's generator)   */
} prng_kind;

typedef enum { PRNG_U32 = 1, PRNG_F32 = 2, PRNG_F64 = 3, PRNG_F32_PAPER = 4 } prng_dtype;

enum {
  PRNG_OK = 0,
  PRNG_EINVAL = -1,      /* bad argument (null pointer, unknown kind, too small buffer) */
  PRNG_ERANGE = -2,      /* a seed word outside the generator's valid range            */
  PRNG_ENOMEM = -3,      /* host allocation failed                                      */
  PRNG_EHIP = -4,        /* a HIP runtime call failed (message names it)                */
  PRNG_ESTATE = -5,      /* malformed or mismatched state blob                          */
  PRNG_EUNSUPPORTED = -6 /* valid request the library does not support                  */
};

typedef struct prng_gen prng_gen; /* opaque; created by prng_create, freed by prng_destroy */

/* Thread-local text of the last error raised on this thread ("" if none). */
const char *prng_last_error(void);

/* Number of uint64 words in one stream's seed tuple: GGL 1 (x0), XOR128 4
 * (x, y, z, w), RANECU 2 (s1, s2), RANMAR 2 (ij, kl), RANLUX 1 (v), MT19937 1
 * (s), DRAND48 and RANNYU 1 (X_0).  Negative for an unknown kind. */
int prng_seed_tuple_words(int kind);

/* Number of uint32 words of one stream's canonical state (the layout of the
 * state blob): GGL 1, XOR128 4, RANECU 2, RANMAR 98 (97 lags oldest first,
 * then C), RANLUX 26 (24 lags oldest first, borrow, kept-in-block count),
 * MT19937 625 (mt[624], index), DRAND48 and RANNYU 2 (X mod 2^32, X >> 32).
 * Negative for an unknown kind. */
int prng_state_words(int kind);

/* Host-only helper: per-stream seed tuples for n_streams streams derived from
 * one master seed with SplitMix64 and mapped into the generator's valid seed
 * range (valid ranges: GGL x0 in [1, 2^31-2]; XOR128 four 32-bit words, not
 * all zero; RANECU s1 in [1, 2147483562], s2 in [1, 2147483398]; RANMAR
 * ij in [0, 31328], kl in [0, 30081] (Section 3.5); RANLUX v in
 * [1, 2147483562]; MT19937 s in [0, 2^32); DRAND48 X_0 in [0, 2^48); RANNYU
 * X_0 odd in [1, 2^48)).  Tuples are distinct within one
 * call.  `out` is a host array of n_streams * prng_seed_tuple_words(kind)
 * words, written stream by stream. */
int prng_seed_words(int kind, uint64_t master, uint64_t n_streams, uint64_t *out);

/* Device bytes the caller must provide as `d_state` to prng_create for
 * n_streams streams of this kind: the internal state layout plus a staging
 * area for the seed tuples read by the initialisation kernel (for RANLUX also
 * a state snapshot and the jump tables of its luxury, about 75 KB; for XOR128
 * a state snapshot and 64 KB of jump matrices).  0 for an unknown kind. */
size_t prng_state_bytes(int kind, uint64_t n_streams);

/* Create a generator object with n_streams independent streams.
 *   kind          one of prng_kind.
 *   p             RANLUX luxury: values produced per block of 24 kept ones
 *                 (24, 48, 97, 223, 389 are the luxury levels 0-4 of
 *                 Appendix A.4.6; any p >= 24 is accepted).  Ignored (pass 0)
 *                 for the other kinds.
 *   h_seed_words  host array, n_streams * prng_seed_tuple_words(kind) words,
 *                 checked against the ranges above (PRNG_ERANGE otherwise).
 *   d_state       caller-owned device buffer of at least
 *                 prng_state_bytes(kind, n_streams) bytes, 256-byte aligned;
 *                 it must stay allocated until prng_destroy.
 * The initialisation kernel (RMARIN for RANMAR, the LCG fill for RANLUX,
 * init_genrand for MT19937, a copy for the others) runs on `stream`; the call
 * synchronises `stream` before it returns (the host seed array may be freed
 * at once).  On success *g receives the new object. */
int prng_create(prng_gen **g, int kind, uint32_t p, uint64_t n_streams, const uint64_t *h_seed_words,
                void *d_state, size_t d_state_bytes, void *stream);

/* Release the object's host metadata.  Never touches caller memory. */
void prng_destroy(prng_gen *g);

/* Generator properties (0 on a NULL object). */
int prng_kind_of(const prng_gen *g);
uint32_t prng_luxury_of(const prng_gen *g);
uint64_t prng_n_streams(const prng_gen *g);

/* Produce the next `count` elements of every stream (Section 3.1, the
 * generation phase), element type `dtype`, into the caller's device buffer
 * d_out of at least n_streams * count * sizeof(element) bytes (out_bytes),
 * stream-major, and advance every stream.  count = 0 is a no-op.  Successive
 * calls continue the streams: generate(a) then generate(b) writes exactly the
 * elements generate(a + b) would.  dtype PRNG_U32, PRNG_F32, PRNG_F64 or
 * PRNG_F32_PAPER.
 * RANLUX and XOR128 objects cut long requests into segments started from
 * jumped-ahead states (same output), so that several wavefronts per SIMD
 * run: the call copies the state into the object's scratch area on `stream`
 * first and takes the jumps from tables written by prng_create, so it stays
 * asynchronous and can be captured into a graph. */
int prng_generate(prng_gen *g, uint64_t count, int dtype, void *d_out, size_t out_bytes, void *stream);

/* prng_generate for callers that cannot allocate device memory or take an
 * allocation of theirs for scratch (code under stream capture, serving loops
 * that forbid allocation).  Same arguments, outputs and stream advance as
 * prng_generate; it calls no allocating routine.  Scratch: the only kernels
 * of prng_generate that use scratch memory are those of RANLUX and XOR128 (a
 * copy of the state taken before the launch, read by the jumped segments);
 * this call keeps that copy in a static device array of 8 MiB that the
 * library holds on every GPU it runs on until the process ends, instead of in
 * the object's buffer.  RANLUX objects therefore need at most
 * 8 MiB / 104 B = 80659 streams, XOR128 objects 8 MiB / 16 B = 524288
 * (PRNG_EINVAL beyond).  Every call on one GPU shares that GPU's array:
 * RANLUX calls that overlap on one GPU (different streams without ordering
 * between them) race; calls ordered on one stream do not.  The array's
 * contents are fully rewritten by every call that uses them. */
int prng_generate_noalloc(prng_gen *g, uint64_t count, int dtype, void *d_out, size_t out_bytes, void *stream);

/* prng_generate with the streams interleaved four by four, the layout of the
 * paper's kernels, where one thread runs four sequences in the four
 * components of a register and stores them as one 16-byte vector (Section
 * 3.1; GGL, RANECU and RANMAR, Sections 3.2, 3.4, 3.5): element i of stream s
 * is out[((s / 4) * count + i) * 4 + s % 4].  dtype PRNG_U32, PRNG_F32 or
 * PRNG_F32_PAPER; any lane-per-stream kind (not MT19937: PRNG_EUNSUPPORTED);
 * n_streams a multiple of 4 and d_out 16-byte aligned (PRNG_EINVAL
 * otherwise).  Advances every stream by `count`, as prng_generate does. */
int prng_generate_packed4(prng_gen *g, uint64_t count, int dtype, void *d_out, size_t out_bytes, void *stream);

/* Where the RANLUX lag table lives during generation: the paper compares
 * three implementations of the same generator (Section 3.6, Table 3).
 * PRNG_LAG_REGISTERS is its planar scheme taken to the register file (the
 * path prng_generate runs); PRNG_LAG_LDS keeps the 24 lags in an indexed
 * array (the temporary-array scheme, here in LDS); PRNG_LAG_HBM reads and
 * writes them in the stream's state words in device memory at every step
 * (the direct translation through the global buffer).  All three produce the
 * same numbers. */
enum { PRNG_LAG_REGISTERS = 0, PRNG_LAG_LDS = 1, PRNG_LAG_HBM = 2 };

/* prng_generate for a RANLUX object with the lag table placed by `variant`
 * (PRNG_LAG_*); same arguments, outputs and stream advance.  PRNG_EINVAL for
 * an object of another kind, an unknown variant or PRNG_F32_PAPER. */
int prng_ranlux_generate_variant(prng_gen *g, int variant, uint64_t count, int dtype, void *d_out,
                                 size_t out_bytes, void *stream);

/* In-kernel consumer (Section 3.1: numbers used where they are produced and
 * never stored).  Draws `draws` single-precision uniforms from every stream and
 * reduces them in the kernel: d_sum[s] = exact sum of the 24-bit mantissas
 * k = u >> (b-24) (the float sum is d_sum[s] * 2^-24), and
 * d_hist[s*64 + j] = number of draws with k >> 18 == j, i.e. in [j/64, (j+1)/64).
 * d_sum: n_streams uint64 words; d_hist: n_streams * 64 uint32 words (device,
 * caller-owned; both fully overwritten).  Advances every stream by `draws`.
 * RANLUX objects of at most 65536 streams cut runs of at least 5760 draws into
 * jumped segments, one wavefront per stream, with the same state copy as
 * prng_generate (asynchronous too). */
int prng_fused_sum_hist(prng_gen *g, uint64_t draws, uint64_t *d_sum, uint32_t *d_hist, void *stream);

/* Size in bytes of the canonical state blob of this object:
 * a 32-byte header (magic "PRNG", version 1, kind, p, n_streams, words per
 * stream) followed by n_streams * prng_state_words(kind) uint32 words,
 * stream by stream, in the canonical layout described at prng_state_words. */
size_t prng_blob_bytes(const prng_gen *g);

/* Copy every stream's state into the host buffer h_blob (canonical blob,
 * `bytes` >= prng_blob_bytes).  Synchronises `stream` (the finalisation
 * phase of Section 3.1: state stored for the next run). */
int prng_get_state(const prng_gen *g, void *h_blob, size_t bytes, void *stream);

/* Replace every stream's state from a canonical blob made by prng_get_state
 * for an object of the same kind, p and n_streams (PRNG_ESTATE when the header
 * does not match or a stream's words are not a valid state).  Synchronises
 * `stream`. */
int prng_set_state(prng_gen *g, const void *h_blob, size_t bytes, void *stream);

/* ------------------------------------------------------------------ stream table
 * Batched generation of many streams of mixed kinds and uneven lengths in one
 * submission.  The paper runs every instance the same length in one kernel
 * (Section 3.1); a table generalises that launch to arbitrary rows.  A row is
 * one stream of one generator object; every run of the table produces the
 * next `count` elements of each row's stream into that row's buffer,
 * exactly as prng_generate would for that stream alone (bit-identical), and
 * advances the stream.  Rows are planned into wave-sized tasks (64 segments of
 * one kind, luxury and dtype; one task per MT19937 stream), ordered longest
 * first, and executed by two persistent kernels that pull tasks from a
 * counter; a run is optionally captured into a HIP graph and replayed. */
typedef struct prng_table prng_table;

typedef struct {
  uint32_t gen;    /* index into the generator array passed to prng_table_create */
  uint32_t dtype;  /* PRNG_U32, PRNG_F32 or PRNG_F64                               */
  uint64_t stream; /* stream index inside that generator object                  */
  uint64_t count;  /* elements per run (0: the row is ignored); f64 rows use two
                      draws per element; at most 2^30 draws per row              */
  void *d_out;     /* device buffer of `count` elements, aligned to the element  */
} prng_table_row;

/* Segment length: rows of the lane-per-stream kinds longer than one segment
 * are cut into segments of that many positions, each started from a state
 * jumped ahead to its first position (GGL/RANECU: a^J mod m; XOR128: the
 * GF(2) matrix T^J; RANMAR: x^J modulo the lag polynomial and C_n in closed
 * form; RANLUX: the equivalent LCG modulo 2^576 - 2^240 + 1; MT19937: x^J
 * modulo the characteristic polynomial of its state transition), so that
 * several lanes or workgroups work on one long stream; the output is
 * unchanged.  PRNG_SEG_AUTO picks lengths from the table's total work (MT19937
 * rows, worked by a whole workgroup, are cut only when far longer than their
 * share); PRNG_SEG_NEVER disables cutting; any other value is rounded up to a
 * multiple of 384 (for MT19937 to a multiple of 624, at least 1248).  RANLUX
 * segments are the lane length divided by RANLUX's cost per draw relative to
 * the other lane kinds (1.5 at p = 24, plus 0.35 per 24 discarded values:
 * 4.4 at p = 223), rounded up to a multiple of 384, so that its tasks take
 * about as long as theirs. */
#define PRNG_SEG_AUTO 0u
#define PRNG_SEG_NEVER 0xFFFFFFFFu

/* Device workspace bytes prng_table_create needs for these rows and this
 * segment length (task lists, segment descriptors, state snapshots, jump
 * data, counters); 0 on invalid rows (see prng_last_error). */
size_t prng_table_work_bytes(prng_gen *const *gens, int n_gens, const prng_table_row *rows, uint64_t n_rows,
                             uint32_t seg_len);

/* Plan a table.  gens: n_gens generator objects (they must outlive the table);
 * rows: host array; a stream may appear in at most one row (PRNG_EINVAL).
 * d_work: caller-owned device workspace of prng_table_work_bytes(...) bytes
 * for the same arguments, 256-byte aligned, kept until prng_table_destroy.
 * Synchronises `stream` after uploading the plan.  A shape tuned earlier in
 * the process (same task counts and draw totals) starts from the cached
 * setting. */
int prng_table_create(prng_table **t, prng_gen *const *gens, int n_gens, const prng_table_row *rows,
                      uint64_t n_rows, uint32_t seg_len, void *d_work, size_t work_bytes, void *stream);

/* Segment lengths per class of kind, for prng_table_create_ex: each 0
 * (automatic, as PRNG_SEG_AUTO), PRNG_SEG_NEVER or a length, rounded as for
 * prng_table_create (MT19937 to a multiple of 624, at least 1248).  The
 * automatic RANMAR length is four automatic lane lengths (its jump costs
 * about 2 x 97^2 operations per segment). */
typedef struct {
  uint32_t lane;   /* GGL, XOR128, RANECU, RANLUX, DRAND48, RANNYU */
  uint32_t ranmar; /* RANMAR */
  uint32_t mt;     /* MT19937 */
} prng_seg_lengths;

/* prng_table_work_bytes and prng_table_create with a length per class (seg
 * NULL: all automatic). */
size_t prng_table_work_bytes_ex(prng_gen *const *gens, int n_gens, const prng_table_row *rows, uint64_t n_rows,
                                const prng_seg_lengths *seg);
int prng_table_create_ex(prng_table **t, prng_gen *const *gens, int n_gens, const prng_table_row *rows,
                         uint64_t n_rows, const prng_seg_lengths *seg, void *d_work, size_t work_bytes, void *stream);
/* The lengths a table cuts its rows at, per class (0: not cut; a row that
 * would exceed 4096 segments is cut into 4096 longer ones). */
int prng_table_seg_lengths(const prng_table *t, prng_seg_lengths *out);

/* Segment-length tuner, the numbers each lane (or MT19937 workgroup) works
 * on: starting from the automatic lengths A it tries A / 2 and 2 A for the
 * lane kinds, then for RANMAR, then for MT19937, keeping a change when the
 * tuned table (prng_table_autotune on each candidate) runs faster.  Each
 * candidate is planned into the caller's workspace d_work of work_bytes
 * (prng_table_tune_work_bytes covers every candidate; a candidate that does
 * not fit is skipped).  Restores all referenced stream states; output buffers
 * are overwritten.  best: the lengths to pass to prng_table_create_ex; best_ms
 * (may be NULL): the time of one tuned run with them.  Synchronises `stream`. */
int prng_table_tune_segments(prng_gen *const *gens, int n_gens, const prng_table_row *rows, uint64_t n_rows,
                             int repeats, void *d_work, size_t work_bytes, void *stream, prng_seg_lengths *best,
                             float *best_ms);
size_t prng_table_tune_work_bytes(prng_gen *const *gens, int n_gens, const prng_table_row *rows, uint64_t n_rows);

/* One run of the table on `stream`.  use_graph != 0: the first call captures
 * the run (one kernel clearing the counters and copying the cut streams'
 * starting states, the MT19937 jump kernel, then the persistent kernels of
 * the two lane-per-stream classes -- GGL, XOR128, RANECU, DRAND48, RANNYU
 * and RANLUX; RANMAR -- and of MT19937, placed on streams by the concurrency
 * setting) into a HIP graph and every call launches that graph;
 * use_graph == 0 enqueues the kernels directly. */
int prng_table_run(prng_table *t, int use_graph, void *stream);

/* Autotuner: times every candidate (lane-per-stream classes on half, three
 * quarters or all of the chip, MT grid 128..2048 blocks, concurrency 0..3)
 * on the real rows as replays of its captured graph: one untimed replay,
 * then `repeats` timed replays back to back (the median counts), after which
 * all referenced stream states are restored; keeps the fastest, and caches
 * it for tables of the same shape.  Output buffers are overwritten by the
 * trials.  Synchronises `stream`. */
int prng_table_autotune(prng_table *t, int repeats, void *stream);

/* Current setting (grids in 256-thread blocks of four wavefronts; lane_grid
 * counts blocks of RANMAR's class, one per CU, 256 filling the chip; the
 * other lane class runs twice as many; an MT19937 block works on one segment
 * at a time).  concurrent: 0 runs the kernels
 * one after the other; 1 runs MT19937's beside the lane classes, which follow
 * one another; 2 gives MT19937 and every lane class a stream of its own, the
 * classes sharing the chip; 3 is 2 with the lane classes started before the
 * MT19937 jump kernel, which then runs on MT19937's stream. */
int prng_table_get_config(const prng_table *t, int *lane_grid, int *mt_grid, int *concurrent);
/* Override the setting (drops a captured graph); PRNG_EINVAL for grids
 * outside [1, 65536] or concurrent outside 0..3. */
int prng_table_set_config(prng_table *t, int lane_grid, int mt_grid, int concurrent);
/* Plan statistics: tasks per class, total and largest draws per row, number
 * of segments (rows after cutting). */
int prng_table_info(const prng_table *t, uint32_t *n_lane_tasks, uint32_t *n_mt_tasks, uint64_t *total_draws,
                    uint64_t *max_draws, uint64_t *n_segments);
/* Release the table (graph, internal streams and events).  Never touches
 * caller memory. */
void prng_table_destroy(prng_table *t);

/* ------------------------------------------------------------ serving loop
 * Not in the paper (it generates fixed-size blocks only).  A server keeps the
 * generator objects' stream states resident on the device and answers
 * requests (generator index, stream, count, dtype) with the next `count`
 * elements of that stream, in per-stream arrival order, bit-identical to what
 * prng_generate / prng_table_run would give for the same stream positions.
 * A worker thread admits arrived requests in arrival order while the output
 * memory they need fits into the caller's device pool (a request that does not
 * fit waits, and so does everything behind it: nothing is over-allocated),
 * packs up to max_batch admitted requests of one class of kinds (GGL, XOR128,
 * RANECU, DRAND48, RANNYU, RANLUX; RANMAR; MT19937), and at most
 * 1/max_inflight of the pool's output room, into one stream-table launch (rows
 * longer than the segment length are cut and started from jumped-ahead
 * states), and keeps up to max_inflight such batches in flight, each slot on
 * a HIP stream of its own (a class takes any free slot except those that
 * other classes with arrived requests and no batch in flight still need; with
 * max_inflight = 1 one batch runs at a time), so that batches, of one class
 * or of several, run side by side and requests arriving while others run are
 * admitted as memory and slots free up (continuous batching).  A request
 * whose stream has an earlier request waiting or in flight waits for it.
 * While a server exists, the generator objects it holds must not be used by
 * any other call.  Times are nanoseconds on the host's steady clock since
 * prng_server_create. */
typedef struct prng_server prng_server;

/* gens: n_gens generator objects (they must outlive the server).
 * d_pool: caller-owned device memory, 256-byte aligned, pool_bytes long, kept
 * until prng_server_destroy; the server places its jump tables at the front
 * and serves outputs and batch workspaces from the rest (the memory budget).
 * max_inflight in [1, 16] batches; max_batch >= 1 requests per batch.
 * seg_len: a base length L, PRNG_SEG_AUTO (L = 384) or a length rounded up
 * to a multiple of 384; segments are 2 L positions for GGL, RANECU, DRAND48
 * and RANNYU, 4 L for XOR128, L / 2 for RANLUX (at least 384, a multiple of 384: its
 * draws cost about four of the others', and a batch lasts as long as its
 * longest task), 4 L for RANMAR and 512 L for MT19937 (a multiple of 624);
 * PRNG_SEG_NEVER: one lane or workgroup per request, as a plain per-stream
 * kernel.  max_request_draws: the largest request in draws (two per fp64
 * element), at most 2^30 and at most 32768 segments.  Synchronous; starts the
 * worker thread. */
int prng_server_create(prng_server **s, prng_gen *const *gens, int n_gens, void *d_pool, size_t pool_bytes,
                       int max_inflight, int max_batch, uint32_t seg_len, uint64_t max_request_draws);
/* Queue n requests (host arrays).  arrive_ns: scheduled arrival of each (an
 * open-loop schedule; a negative value or a NULL array means now); arrivals
 * must be non-decreasing, also across calls while earlier ones wait.  keep = 0
 * frees each output as soon as its batch completes (timing runs); keep != 0
 * holds it until prng_server_release.  tickets[i] receives request i's id.
 * Thread-safe; never blocks on the device. */
int prng_server_submit_many(prng_server *s, uint64_t n, const uint32_t *gen, const uint64_t *stream,
                            const uint64_t *count, const int *dtype, const int64_t *arrive_ns, int keep,
                            uint64_t *tickets);
/* One request, arriving now, kept until released. */
int prng_server_submit(prng_server *s, uint32_t gen, uint64_t stream, uint64_t count, int dtype, uint64_t *ticket);
/* Wait up to timeout_ms (0: poll, < 0: forever) for a kept request.  Returns 1
 * and its device output (inside the pool, valid until released) when done, 0
 * if not done yet, or a negative code: the request's batch failed on the
 * device (no output is returned for it, ever), the server was stopped by a
 * device or planning error before running it, or the ticket is unknown or
 * released.  A failed request's memory is already back in the pool;
 * prng_server_release on it only retires the ticket. */
int prng_server_result(prng_server *s, uint64_t ticket, int timeout_ms, void **d_out, size_t *bytes);
/* Return a completed kept request's output memory to the pool. */
int prng_server_release(prng_server *s, uint64_t ticket);
/* Arrival, admission and completion times of n tickets (-1 while pending);
 * any output array may be NULL. */
int prng_server_times(const prng_server *s, uint64_t n, const uint64_t *tickets, int64_t *arrive_ns,
                      int64_t *admit_ns, int64_t *done_ns);
/* Counters; pool_in_use counts output and workspace bytes held right now. */
int prng_server_stats(const prng_server *s, uint64_t *submitted, uint64_t *completed, uint64_t *batches,
                      size_t *pool_in_use);
/* Host time spent planning and enqueuing batches, and the sum of the
 * batches' durations on the device (from the start of their upload to
 * their completion, overlapping batches counted each). */
int prng_server_timing(const prng_server *s, int64_t *host_plan_ns, double *device_ms);
/* The server's clock (ns since creation). */
int64_t prng_server_now_ns(const prng_server *s);
/* Stop the worker, wait for batches in flight, free host objects.  Requests
 * not yet admitted are dropped; caller memory is never touched. */
void prng_server_destroy(prng_server *s);

#ifdef __cplusplus
}
#endif

#endif /* PRNG_H */
