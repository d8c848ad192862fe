/*
 * ga.h -- C ABI of the MI355X guided extension aligner.
 *
 * The library computes, for a batch of (target, query) pairs, the banded
 * two-piece affine-gap extension alignment with per-anti-diagonal maximum
 * tracking and z-drop termination of AGAThA (PPoPP'24, arXiv 2403.06478),
 * Section 2.1: the score table of Eq. 1-3 (generalised to two gap pieces)
 * restricted to a diagonal band (k-banding), and the termination condition
 * of Eq. 4-7. Every result is exact int32.
 *
 * Definition (0-based; i indexes the target T, j the query Q):
 *   S(x,y) = -ambig if x or y is N, +a if x == y, else -b.
 *   A gap run of length l costs min(q + l*e, q2 + l*e2).
 *   Lattice point (i,j), i,j >= -1, is usable iff w < 0 or |i-j| <= w.
 *   H(i,j) = best score of an alignment path from (-1,-1) to (i,j) through
 *            usable points, each maximal gap run charged as above.
 *   Anti-diagonal r = i+j, r = 0..n+m-2: M_r = max H over its in-band cells,
 *   (mi,mj) the cell with the smallest i attaining it. Starting from
 *   G = 0 at (-1,-1): if M_r > G the maximum moves to (M_r,mi,mj); else if
 *   Z >= 0, mi > gi, mj > gj and G - M_r > Z + e2*|(mi-gi)-(mj-gj)| the pair
 *   is z-dropped at r and the sweep stops. end_* is (M_r,mi,mj) of the last
 *   anti-diagonal examined. Empty sequences give (0,-1,-1,0,-1,-1,0).
 *
 * Conventions: every pointer named *_dev is device memory owned by the
 * caller; the library never frees caller memory. Calls returning an int give
 * GA_OK (0) or a negative GA_E* code; validation happens on the host before
 * any launch. Work is enqueued on `stream` (a hipStream_t, NULL = default
 * stream) and is asynchronous: results are valid once the stream has
 * completed. Errors found on the device (a pair longer than the declared
 * bound, offsets outside the packed streams) are latched in the context and
 * reported by ga_context_check().
 *
 * A context serves one call at a time: its workspace (planning counters
 * and work lists, the error latch) is reused by every ga_pack and
 * ga_align_batch on it, so calls on one context must be ordered on the
 * device (issued on one stream, or with the caller's synchronisation
 * between streams) and made from one host thread at a time. Work that
 * should overlap uses one context per stream.
 */
#ifndef GA_H
#define GA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GA_OK 0
#define GA_EINVAL (-1)       /* null pointer, negative size or parameter, range guard */
#define GA_ENOMEM (-2)       /* device workspace allocation failed */
#define GA_EHIP (-3)         /* HIP launch or runtime error */
#define GA_EUNSUPPORTED (-4) /* parameters outside what the kernels implement */
#define GA_EDEVICE (-5)      /* a device-side check failed (see ga_context_check) */

/* Scoring (Section 2.1): match +a, mismatch -b, N against anything -ambig,
 * gap run of length l costs min(q + l*e, q2 + l*e2). Every field >= 0.
 * The kernels hold S + q + 2e in signed bytes: they take a + q + 2e <= 127,
 * q + 2e - b >= -128 and q + 2e - ambig >= -128 (else GA_EUNSUPPORTED). */
typedef struct {
    int32_t a, b, q, e, q2, e2, ambig;
} ga_scoring_t;

/* Per-pair result, 28 bytes, 0-based indices; -1 means "the origin". */
typedef struct {
    int32_t max_score, max_i, max_j; /* global maximum G and its cell */
    int32_t end_score, end_i, end_j; /* anti-diagonal maximum where the sweep ended */
    int32_t zdropped;                /* 1 if the z-drop condition fired */
} ga_result_t;

/* A packed batch (input packing, Section 2.2): bases as 2-bit codes A=0 C=1
 * G=2 T=3, 16 per uint32; base k of a sequence starting at word `off` sits at
 * bits 2*(k%16) of word off + k/16. The optional N bitmap holds one bit per
 * base position of the 2-bit stream: base k of that sequence is N iff bit
 * (16*off + k) % 32 of word (16*off + k) / 32 is set; NULL means no N. */
typedef struct {
    int64_t n_pairs;
    const uint32_t *t_words_dev; /* target 2-bit stream */
    int64_t t_nwords;            /* its length in words (may exceed the packed words) */
    const uint32_t *q_words_dev; /* query 2-bit stream */
    int64_t q_nwords;
    const int64_t *t_off_dev;    /* [n_pairs] first word of each target */
    const int64_t *q_off_dev;    /* [n_pairs] first word of each query */
    const int32_t *t_len_dev;    /* [n_pairs] target lengths in bases */
    const int32_t *q_len_dev;    /* [n_pairs] query lengths in bases */
    const uint32_t *t_nmask_dev; /* N bitmap of the target stream, or NULL */
    const uint32_t *q_nmask_dev; /* N bitmap of the query stream, or NULL */
    int32_t max_len;             /* caller's bound on every t_len and q_len */
} ga_batch_t;

typedef struct ga_context ga_context_t;

/* Create a context on HIP device `device`; it owns the device workspace
 * (work lists, counters: about 1 MiB plus 8 bytes per pair). Returns GA_EINVAL for a bad device. */
int ga_context_create(ga_context_t **ctx, int device);

/* Release the context and its workspace (synchronises the device). */
int ga_context_destroy(ga_context_t *ctx);

/* Wait for `stream`, then report and clear the device-side error latch:
 * GA_OK, or GA_EDEVICE if any pair violated the batch's declared bounds
 * (such pairs get the result {0,-1,-1,0,-1,-1,-1}). */
int ga_context_check(ga_context_t *ctx, void *stream);

/* The device address of pinned host memory (allocated with hipHostMalloc,
 * or as a pinned torch tensor), for callers that let the kernels read their
 * inputs and write their results in place (zero-copy staging): every *_dev
 * pointer of this interface may be such an address. GA_EINVAL (and NULL)
 * if `host` is not pinned host memory. */
int ga_host_device_pointer(void *host, void **dev);

/* Human-readable text for a GA_* code (static storage). */
const char *ga_strerror(int code);

/* Number of uint32 words ga_pack writes for sequences of the given lengths
 * (host array), i.e. the sum of ceil(len/16). */
int64_t ga_pack_words(const int32_t *len_host, int64_t n);

/* On-device input packing (Section 2.2, input packing): `ascii_dev` holds
 * n sequences, sequence p at byte offset off_dev[p] with length len_dev[p].
 * Writes word_off_dev[p] (exclusive prefix sum of ceil(len/16)), the 2-bit
 * stream words_dev[0 .. ga_pack_words) and the N bitmap
 * nmask_dev[0 .. (ga_pack_words+1)/2). Any byte outside ACGTacgt becomes N
 * (2-bit code 0 plus its N bit). `nwords` is the capacity of words_dev in
 * words, at least ga_pack_words(len); words past the packed ones are left
 * as they are (a caller may declare fixed capacities, e.g. to replay one
 * captured graph over batches of different sizes). */
int ga_pack(ga_context_t *ctx, const uint8_t *ascii_dev, const int64_t *off_dev,
            const int32_t *len_dev, int64_t n, int64_t nwords, uint32_t *words_dev,
            int64_t *word_off_dev, uint32_t *nmask_dev, void *stream);

/* Align every pair of `batch` (Section 2.1, Eq. 1-7) with band half-width w
 * (w < 0: no band) and z-drop threshold Z (Z < 0: never drop), writing
 * out_dev[p] for each pair. Range guard (GA_EINVAL otherwise):
 * (2*max_len + 2) * (max(a, b, ambig, q+e, q2+e2) + a + e + e2) + max(Z,0) < 2^29.
 * Band widths with 2*min(w, max_len) + 1 > 8180 return GA_EUNSUPPORTED. */
int ga_align_batch(ga_context_t *ctx, const ga_batch_t *batch, const ga_scoring_t *sc,
                   int32_t w, int32_t Z, ga_result_t *out_dev, void *stream);
/* Graph capture: under GA_SCHED_PERSISTENT (and GA_SCHED_UNORDERED) with
 * timing off, ga_pack and ga_align_batch only enqueue kernels on `stream`
 * (no host waits, no memset nodes), so both may be captured into a HIP graph
 * once the context's workspace has grown to the batch's size: run the same
 * shapes once before capturing. The graph then holds the pointers, sizes
 * and parameters of the captured call; pairs of length 0 finish at once. */

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): as
 * ga_align_batch, with the same arguments and results, but the call's
 * planning workspace is a fixed device array inside the library (about
 * 9 MiB, one copy per GPU, held until the process ends) instead of the
 * context's workspace, and the call allocates nothing. It takes at most
 * GA_NOALLOC_MAX_PAIRS pairs (GA_EINVAL above that) and the persistent or
 * unordered schedule (GA_EUNSUPPORTED under GA_SCHED_BUCKETED, which waits
 * for the host). Every such call on one GPU, from any context, uses that
 * GPU's one array: calls that overlap on the device race, so order them
 * (one stream, or the caller's synchronisation). Each call clears what it
 * needs first. Its launches spread over the context's streams (see
 * ga_context_set_lanes) only if an earlier ga_align_batch on the context
 * made them; otherwise they all run on `stream`. GA_EHIP if the array could not be located on the device when
 * the context was created. */
#define GA_NOALLOC_MAX_PAIRS (1 << 20)
int ga_align_batch_noalloc(ga_context_t *ctx, const ga_batch_t *batch, const ga_scoring_t *sc,
                           int32_t w, int32_t Z, ga_result_t *out_dev, void *stream);

/* A whole ga_align_batch call captured into a HIP graph (the batched
 * offline path's launches -- planning, the fork of the context's streams,
 * every kernel class's persistent launch, the join -- replayed by one
 * hipGraphLaunch). ga_graph_capture first grows the context's workspace to
 * the batch and makes its side streams, then captures the call on `stream`
 * (not NULL) and instantiates the graph; nothing runs on the device. The
 * graph holds the batch's pointers, sizes, scoring, w and Z and the
 * context's workspace: ga_graph_launch(graph, stream) then aligns that
 * batch again (into out_dev) as ga_align_batch would, with the same
 * results, while the context and every buffer stay alive and no other call
 * uses the context's workspace in between. Timing must be off and the
 * schedule persistent or unordered (else GA_EINVAL). */
typedef struct ga_graph ga_graph_t;
int ga_graph_capture(ga_context_t *ctx, const ga_batch_t *batch, const ga_scoring_t *sc, int32_t w,
                     int32_t Z, ga_result_t *out_dev, void *stream, ga_graph_t **graph);
int ga_graph_launch(ga_graph_t *graph, void *stream);
int ga_graph_destroy(ga_graph_t *graph);

/* Work schedules of ga_align_batch (results are identical under both):
 * GA_SCHED_PERSISTENT (the default): every pair goes to the cheapest kernel
 * class that runs it, ordered longest first within the class, and each
 * class runs as one persistent launch of resident workgroups pulling pairs
 * through an atomic head (Section 4.4's load balancing, in this form).
 * GA_SCHED_BUCKETED: the plain baseline kept for comparison -- pairs are
 * bucketed by the power of two above max(n, m), and each bucket runs as one
 * fixed-shape launch (the fixed class holding the bucket's longest band)
 * with one workgroup per pair; the host waits for the bucket sizes. */
#define GA_SCHED_PERSISTENT 0
#define GA_SCHED_BUCKETED 1
/* GA_SCHED_UNORDERED: as GA_SCHED_PERSISTENT, but the pairs of a class run in
 * batch order instead of longest first (the ordering's own effect, for the
 * long-pair ratio study of Section 5.6, Fig. 12). */
#define GA_SCHED_UNORDERED 2

/* Select the schedule of later ga_align_batch calls on this context;
 * GA_EINVAL for an unknown schedule. */
int ga_context_set_schedule(ga_context_t *ctx, int schedule);

/* Streams the persistent launches of one ga_align_batch call spread over
 * (1..4; default 4): the caller's stream plus up to three streams the
 * context owns, forked from and joined back into the caller's stream, so the
 * call stays ordered on `stream` while the launches of different kernel
 * classes overlap on the device. The class holding the band's full width
 * (where a batch's longest pairs land) launches first, on the caller's
 * stream, so its longest pairs start at once. 1 keeps every launch on
 * `stream` (e.g. where many contexts share the GPU's few hardware queues).
 * GA_EINVAL outside 1..4. */
int ga_context_set_lanes(ga_context_t *ctx, int lanes);

/* Restrict the kernel classes (bit c = class c, see ga_context_timing) that
 * later ga_align_batch calls on this context may use; the default is all
 * fifteen. Each pair takes the cheapest allowed class that runs it in the
 * shape the cheapest-first rule gives that class (a sliding class only for a
 * band wider than its window, a class of W waves only for a band that
 * reaches its last wave: more than 64*K*(W-1) diagonals). A pair that no
 * allowed class runs gets the result {0,-1,-1,0,-1,-1,-1} and latches
 * GA_EDEVICE (see ga_context_check). For sensitivity studies of the kernel
 * shapes (the slice width of Section 5.5 and the subwarp size of Section 5.7 have
 * their counterparts in the slots per lane and the waves per pair). Returns
 * GA_EINVAL for an empty mask or bits above class 14. */
int ga_context_set_classes(ga_context_t *ctx, uint32_t mask);

/* Autotuner (the context's autotune table): runs a synthetic probe batch
 * through every kernel class on this context's device -- random pairs with
 * about one substitution in 16, in the shape the cheapest-first rule gives
 * each class (the band filling 7/8 of its slots; short-by-long pairs for the
 * sliding classes), enough pairs for two rounds of resident workgroups --
 * and times each class's launch. ns_per_step[c] (c < n, n <= 15) receives
 * the measured cost of class c in nanoseconds per pair and anti-diagonal at
 * full occupancy. Later ga_align_batch calls on this context then try the
 * classes cheapest first: each pair takes the cheapest allowed class that
 * runs it (results do not depend on the class). This is where the shape
 * choices of Sections 5.5 and 5.7 (slice width, subwarp size) are made by
 * measurement. It also times each class on a batch of 64 such pairs, each
 * alone on its CU: one pair's time per anti-diagonal (its latency, see
 * ga_context_class_latency). Calls of at most 2 x (compute units) pairs
 * then use the classes in that order instead: such a batch does not fill
 * the GPU and takes as long as its longest sweep, so a band spread over
 * more waves (shorter steps, classes 12-14) can end it sooner even though
 * it costs more per pair at full occupancy. Allocates temporary device
 * memory and synchronises `stream`; on an error the default order is in
 * force (and no latency order). */
int ga_context_autotune(ga_context_t *ctx, float *ns_per_step, int n, void *stream);

/* The latency the autotuner measured per class (ns per anti-diagonal of one
 * pair in a batch of 64), into ns_per_step[c] for c < n; GA_EINVAL if the
 * context was not autotuned. */
int ga_context_class_latency(const ga_context_t *ctx, float *ns_per_step, int n);

/* Calls of at most n_pairs pairs plan with the latency order (0: never);
 * the autotuner sets 2 x (compute units). GA_EINVAL if the context was not
 * autotuned or n_pairs < 0. */
int ga_context_set_latency_pairs(ga_context_t *ctx, int32_t n_pairs);

/* The class a call of n_pairs pairs on this context picks for a pair of
 * lengths n, m at band w (the latency or throughput order, see
 * ga_context_autotune); -1 if none. */
int ga_context_batch_class(const ga_context_t *ctx, int32_t n, int32_t m, int32_t w, int64_t n_pairs);

/* The class ga_align_batch on this context picks for a pair of lengths
 * n, m at band w (its class mask and autotuned order); -1 if none. */
int ga_context_pair_class(const ga_context_t *ctx, int32_t n, int32_t m, int32_t w);

/* Stage timing for benchmarking: while enabled, ga_align_batch records HIP
 * events on its stream around its stages. */
int ga_context_set_timing(ga_context_t *ctx, int enable);

/* Milliseconds spent by the stages of the last timed ga_align_batch on this
 * context (waits for those events): ms[0] = planning kernels,
 * ms[1+c] = the alignment launches of class c (summed over buckets under
 * GA_SCHED_BUCKETED), for c < n-1 and c < 15. Class
 * c runs K slots per lane and W waves per pair: classes 0-4, (K, W) = (4,1)
 * (8,1) (16,1) (24,1) (32,1), hold bands of up to 64*K diagonals; classes
 * 5, 6 and 11, (8,1) (16,1) (4,1) with a sliding window, run pairs whose
 * shorter sequence s has 2s + 11 + K <= 64K whatever the band; classes
 * 7-10, (24,2) (32,2) (32,3) (32,4), and 12-14, (8,2) (4,2) (4,4), hold
 * bands of up to
 * 64*K + (W-1)*(64*K - 4) diagonals (3068, 4092, 6136, 8180: neighbouring
 * waves share 4 diagonals). Classes 3 and 2 run the start and end
 * triangles of a band (while an anti-diagonal's finite cells fit) with 16
 * and 8 slots per lane inside the same launch.
 * GA_EINVAL if timing was off for that call. */
int ga_context_timing(ga_context_t *ctx, float *ms, int n);

/* Class (0..14, see ga_context_timing) that ga_align_batch uses for a pair
 * of lengths n, m at band w: the cheapest whose kernel holds the band's
 * min(w, n) + min(w, m) + 1 diagonals (all n + m + 1 when w < 0), or, for a
 * sliding class, the pair's 2 min(n, m) + 11 + K; -1 for an empty pair or
 * a band wider than the kernels hold. Cheapest means fewest slots per lane
 * (4, sliding 4, 8, sliding 8, 16, sliding 16, 24, 32), then the multi-wave
 * classes.
 * Host function, for attributing work to the per-class kernels. */
int ga_pair_class(int32_t n, int32_t m, int32_t w);

/* As ga_pair_class, among the classes of `mask` only (the choice
 * ga_align_batch makes after ga_context_set_classes(ctx, mask)). */
int ga_pair_class_in(int32_t n, int32_t m, int32_t w, uint32_t mask);

/* Measured integer VALU peak of the context's device, for rooflines: a
 * probe kernel of independent v_max3_i32 / v_add_u32 chains (8 waves per
 * SIMD on every CU) is timed with HIP events on `stream`; *lane_ops_per_s
 * receives int32 lane-operations per second. Synchronises `stream`. */
int ga_calibrate_valu(ga_context_t *ctx, double *lane_ops_per_s, void *stream);

/* Algorithmic work of one pair: the number of in-band cells (i,j),
 * 0 <= i < n, 0 <= j < m, on anti-diagonals 0..r_end (r_end = end_i+end_j);
 * 0 when n or m is 0. Host function: sums the band's cell count of each
 * anti-diagonal, which is an interval of rows with closed-form ends. */
int64_t ga_count_cells(int32_t n, int32_t m, int32_t w, int32_t r_end);

/* ---------------------------------------------------------------------
 * Native continuous-batching server (host runtime over the calls above).
 *
 * Requests (one target/query pair each) arrive over time. Each lane (short
 * requests, and requests of more than long_bases bases) keeps a request
 * ring in pinned host memory that the packing kernel reads in place; a
 * request is admitted when its bytes fit (admission by memory footprint),
 * in groups of at most a batch, and waits in the lane's FIFO until then.
 * Each lane has its own execution slots; a slot owns a context (one stream
 * for all its launches), a HIP stream, pinned tables and device streams
 * sized for its capacity and, with `graphs`, one captured HIP graph of the
 * capacity-shaped ga_pack + ga_pack + ga_align_batch, replayed per batch
 * (unused pair entries are empty pairs). Whenever a slot is free, the
 * admitted requests waiting in its lane form its next batch, up to
 * max_batch_pairs pairs and max_batch_bases bases (long lane: long_*). A
 * server is driven from one host thread; calls that touch the device make
 * the server's device current for their duration and restore the caller's. */
typedef struct {
    int32_t slots, long_slots;              /* execution slots per lane (1 .. GA_SERVER_MAX_SLOTS) */
    int32_t max_batch_pairs, long_batch_pairs; /* 1 .. GA_SERVER_MAX_BATCH_PAIRS */
    int64_t max_batch_bases, long_batch_bases;
    int32_t long_bases;                     /* requests with more bases go to the long lane */
    int32_t ring_factor;                    /* ring bytes = ring_factor x the lane's batch bases
                                               (at most GA_SERVER_MAX_RING_BYTES) */
    int32_t graphs;                         /* 1: replay a captured graph per batch */
    double replay_timeout_s;                /* ga_server_replay gives up after this long with
                                               requests in flight and no batch finished;
                                               0: GA_SERVER_REPLAY_TIMEOUT_S */
} ga_server_config_t;

#define GA_SERVER_MAX_SLOTS 16
#define GA_SERVER_MAX_BATCH_PAIRS (1 << 20)
#define GA_SERVER_MAX_RING_BYTES ((int64_t)1 << 33)
#define GA_SERVER_REPLAY_TIMEOUT_S 60.0

typedef struct ga_server ga_server_t;

/* Create a server on `device` for one scoring, band and threshold (see
 * ga_align_batch). Allocates every buffer and captures the graphs now.
 * GA_EINVAL for a bad configuration (checked before any device work: counts
 * below 1 or above the GA_SERVER_MAX_* limits, a negative timeout),
 * GA_ENOMEM, GA_EHIP. */
int ga_server_create(ga_server_t **srv, int device, const ga_scoring_t *sc, int32_t w, int32_t Z,
                     const ga_server_config_t *cfg);

/* Release the server (waits for its batches). */
int ga_server_destroy(ga_server_t *srv);

/* Queue one request (bytes are copied; any byte outside ACGTacgt is N).
 * `tag` is returned with its result; t_arrival is its arrival time in
 * seconds on the steady clock (negative: now). GA_EUNSUPPORTED for a
 * request larger than its lane's ring or longer than 2^20 bases. */
int ga_server_submit(ga_server_t *srv, int64_t tag, const uint8_t *target, int32_t n, const uint8_t *query,
                     int32_t m, double t_arrival);

/* Make progress without waiting: collect finished batches (writing up to
 * max_done (tag, result, completion time) triples; a batch is collected
 * only when all of it fits), admit waiting requests, start batches on free
 * slots. max_done is 0 (collect nothing) or at least the larger of
 * max_batch_pairs and long_batch_pairs (else GA_EINVAL). Returns the number
 * of results written. Errors never cost results: an error found while
 * results are handed back (GA_EDEVICE for a collected batch with pairs
 * outside the declared bounds, which got the sentinel result; GA_EHIP for a
 * batch whose completion cannot be queried, which stays in its slot; a
 * failed launch, whose requests wait again) is latched, and the next poll
 * that writes no results returns it (and clears it). */
int ga_server_poll(ga_server_t *srv, int64_t *tags, ga_result_t *results, double *t_done, int max_done);

/* Requests submitted and not yet collected; batches launched so far. */
int64_t ga_server_pending(const ga_server_t *srv);
int64_t ga_server_batches(const ga_server_t *srv);

/* Replay an arrival trace natively (the serving benchmark): request k --
 * target bytes t_ascii[t_off[k] .. +t_len[k]), query likewise -- arrives
 * arrival_s[k] seconds (non-decreasing) after the start; the call submits
 * each at its time, polls until all are done and writes results[k] and
 * latency_s[k] (arrival to collection), and the wall time. Returns GA_EHIP
 * if requests stay in flight for the configured timeout with no batch
 * finishing, or the first error a poll returns. */
int ga_server_replay(ga_server_t *srv, const uint8_t *t_ascii, const int64_t *t_off, const int32_t *t_len,
                     const uint8_t *q_ascii, const int64_t *q_off, const int32_t *q_len, const double *arrival_s,
                     int64_t n, ga_result_t *results, double *latency_s, double *wall_s);

#ifdef __cplusplus
}
#endif

#endif /* GA_H */
