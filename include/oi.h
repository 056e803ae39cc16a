/*
 * oi.h -- C ABI of the MI355X (gfx950) outward-influence estimator.
 *
 * Implements, on one GPU, the data-parallel hot path of SOIEA / SIEA from
 * Nguyen, Dinh, Thai, "Outward Influence and Cascade Size Estimation in
 * Billion-scale Networks": Importance IC Polling samples (Sec. 3.1, Alg. 1)
 * under the Independent Cascade model (Sec. 2.1), driven by the RSA stopping
 * rule (Sec. 4, Algs. 2 and 3), for one seed set (Alg. 4 / Alg. 5) or many,
 * plus a score-function backward of the fixed-count estimate.
 *
 * Conventions for every call:
 *   - Every function returns oi_status; OI_OK = 0.  On failure
 *     oi_last_error() returns a message for the calling thread.  No
 *     exception crosses this boundary.
 *   - "host" pointers are CPU memory, "device" pointers are memory of the
 *     GPU the graph lives on.  Inputs are only read and stay owned by the
 *     caller; the library copies what it keeps.  Outputs go to caller-owned
 *     buffers of the stated size.
 *   - All GPU work of a graph is issued on the HIP stream given at creation
 *     (or oi_set_stream); every call returns after that work has completed.
 *     Calls on one graph are not thread-safe; distinct graphs are.
 *   - Samples are keyed, not scheduled: the i-th sample of a stream of a
 *     query is a pure function of (graph, seed set, query_id, run_seed,
 *     stream, i).  Randomness is Philox4x32-10 with key (query_id, run_seed)
 *     and counter (lo32(idx), hi32(idx), lo32(i), kind<<28 | stream<<27 |
 *     hi32(i)); the coin of CSR edge e is word e%4 of the block with
 *     idx = e/4, kind 0, and is live iff word < floor(p_e * 2^32); Stage-1
 *     entry j uses kind 2 the same way with floor(P_{S,v_j} * 2^32); the
 *     selection uniform is kind 1, idx 0, U = ((w0>>5)*2^26 + (w1>>6))*2^-53.
 */
#ifndef OI_H
#define OI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct oi_graph oi_graph;

typedef enum {
  OI_OK = 0,
  OI_EINVAL = -1, /* invalid argument (sizes, ranges, null pointers) */
  OI_ERANGE = -2, /* value outside the supported range (ids, sample counts) */
  OI_ENOMEM = -3, /* device or host allocation failed */
  OI_EHIP = -4,   /* a HIP runtime call failed */
  OI_ESTATE = -5  /* internal consistency check failed (reported by a kernel) */
} oi_status;

/* SOIEA estimates OI(S) with X = Y (Alg. 4); SIEA estimates IS(S) with
 * X = Z = beta_0 * Y + |S| (Eq. z_s, Alg. 5).  SIEA_LT (Sec. 5.3 and the LT
 * experiment of Sec. 6) estimates IS(S) under the LT model: RSA on the
 * sizes X = |S| + Y of LT cascades (oi_sample_lt) over [|S|, n], the edge
 * probabilities being the LT weights.  All report OI and IS = OI + |S|. */
typedef enum { OI_MODE_SOIEA = 0, OI_MODE_SIEA = 1, OI_MODE_SIEA_LT = 2 } oi_mode;

/* Gradient with respect to p_e, or to theta_e where p_e = sigmoid(theta_e). */
typedef enum { OI_PARAM_P = 0, OI_PARAM_THETA = 1 } oi_param;

typedef struct {
  double oi;          /* estimate of the outward influence OI(S) = I(S) - |S| */
  double is;          /* estimate of the influence spread IS(S) = OI(S) + |S| */
  double beta0;       /* probability of a non-trivial cascade (Eq. zerop) */
  double mu;          /* estimate of E[X] returned by RSA (or GSRA) */
  double mu1;         /* step-1 rough estimate of RSA */
  uint64_t T1, h1;    /* step 1: samples until the stopping rule, and their sum of Y */
  uint64_t nsigma;    /* step 2: number of pairs of X' */
  uint64_t D_lo, D_hi;/* step 2: 128-bit sum of squared paired differences of Y' */
  uint64_t T, hT;     /* step 3: samples used for the estimate, and their sum of Y */
  uint64_t samples_x, samples_xp; /* samples generated on the X and X' streams */
  uint64_t sum_y;     /* sum of Y over all generated samples */
  uint64_t edges_examined; /* sum over generated samples of (Stage-1 entries after
                              the selected one) + (out-degree of every activated node) */
  int64_t k;          /* |S| after removing duplicate seeds */
  int64_t l;          /* |N^out_S|, the size of the Stage-1 table */
  int32_t gsra_only;  /* 1 if eps >= 1/4 (RSA reduces to GSRA, Alg. 3) */
  int32_t early;      /* 1 if the first GSRA returned its lower bound without sampling */
  int32_t status;     /* per-query oi_status (batch calls) */
  int32_t rounds;     /* sampling launches used */
} oi_result;

/*
 * Create a graph.  CSR: row_ptr[n+1] (int64, row_ptr[0] = 0, non-decreasing,
 * row_ptr[n] = m), col[m] (int32 targets in [0, n)), p[m] (fp32 IC
 * probabilities in [0, 1], Sec. 2.1: edge (u, v) is live with probability
 * w(u, v)).  Edge ids are CSR positions.  If device_ptrs is nonzero the three
 * arrays are device pointers, else host pointers.  hip_stream is a
 * hipStream_t (NULL = default stream).  Limits: n < 2^31, m <= 2^32 - 16,
 * out-degree < 2^29.
 * Errors: OI_EINVAL for malformed CSR or p outside [0, 1] (NaN included).
 */
oi_status oi_graph_create(int64_t n, int64_t m, const int64_t* row_ptr, const int32_t* col, const float* p,
                          int device_ptrs, void* hip_stream, oi_graph** out);

/* Replace all m edge probabilities (same topology).  p as in oi_graph_create. */
oi_status oi_graph_set_probs(oi_graph* g, const float* p, int device_ptr);

/* Set p_e = sigmoid(theta_e) for all m edges (evaluated in fp64 on the GPU,
 * rounded to fp32); theta: float[m], device pointer if device_ptr != 0,
 * else host.  Used with OI_PARAM_THETA gradients. */
oi_status oi_graph_set_theta(oi_graph* g, const float* theta, int device_ptr);

/* Copy the m edge probabilities the library currently uses to host p_out. */
oi_status oi_graph_get_probs(oi_graph* g, float* p_out);

/* Change the HIP stream used for the graph's work. */
oi_status oi_set_stream(oi_graph* g, void* hip_stream);

void oi_graph_destroy(oi_graph* g);

/*
 * Stage-1 table of a seed set (Sec. 3.1): N^out_S sorted by node id, P_{S,v}
 * (Eq. psv, product over the edges from S into v in ascending edge id),
 * CDF_j = sum_{i<=j} Pr[A_i] (Eq. pai) and beta_0 = CDF_l (Eq. zerop), as the
 * sampler uses them.  seeds: host int32[k]; duplicates are removed.  Outputs
 * (host, any may be NULL, filled only if l <= cap): v[l], P[l], cdf[l+1]
 * (cdf[0] = 0), thr[l] = floor(P * 2^32).  *l_out and *beta0 always set.
 */
oi_status oi_stage1_table(oi_graph* g, const int32_t* seeds, int64_t k, int64_t cap, int64_t* l_out,
                          double* beta0, int32_t* v, double* P, double* cdf, uint64_t* thr);

/*
 * Fixed-count IICP sampling (Alg. 1): samples first .. first+count-1 of
 * stream `stream` (0 = X, 1 = X') of the query (query_id, seeds).
 * y_out: device uint32[count] (or NULL) receives Y per sample;
 * e_out: device uint64[count] (or NULL) receives the examined-edge count per
 * sample.  sums (host, may be NULL): sum_y, edges_examined, beta0, k, l, and
 * the fixed-count estimate of Lemma 2 over these samples: mu = mean(Y),
 * oi = beta_0 * mu, is = oi + |S| (T = count, hT = sum_y).
 * If beta_0 = 0 nothing is sampled, y_out is left untouched and oi = 0,
 * is = |S|.
 */
oi_status oi_sample_fixed(oi_graph* g, uint32_t query_id, const int32_t* seeds, int64_t k, int stream,
                          uint64_t first, uint64_t count, uint32_t run_seed, uint32_t* y_out, uint64_t* e_out,
                          oi_result* sums);

/*
 * Classic IC Monte-Carlo cascades M^(S) (Sec. 2.3; the MC_N estimators the
 * paper compares against, Sec. 6.1): samples first .. first+count-1 of stream
 * `stream`.  Every node of S is active from the start and each out-edge of
 * each active node is examined once with its coin; a sample shares its edge
 * coins with the IICP sample of the same key (query_id, run_seed, stream,
 * index).  y_out: device uint32[count] (or NULL) receives M - |S|, the nodes
 * outside S that end active (zero allowed); e_out: device uint64[count] (or
 * NULL) the out-degree summed over every node expanded, S included.  sums
 * (host, may be NULL): sum_y = sum of M - |S|, edges_examined, k, l, beta0
 * (of the Stage-1 table, for comparison), and the MC_N estimates over these
 * samples: is = |S| + mean(M - |S|), oi = is - |S| (mu = oi, T = count).
 * Samples are drawn even when beta_0 = 0 (they are then all zero).
 */
oi_status oi_sample_mc(oi_graph* g, uint32_t query_id, const int32_t* seeds, int64_t k, int stream, uint64_t first,
                       uint64_t count, uint32_t run_seed, uint32_t* y_out, uint64_t* e_out, oi_result* sums);

/*
 * LT-model cascades (the model of Kempe et al. that Sec. 5.3 and the LT
 * experiment of Sec. 6 use with SIEA_LT), samples first .. first+count-1
 * of stream `stream`, the edge probabilities read as LT weights w(u, v) (the
 * in-weights of every node must sum to at most 1; up to 1e-6 of rounding
 * is taken as 1, more gives OI_EINVAL).  Live-edge form: every node v keeps
 * at most one in-edge, (u, v) with probability w(u, v); its choice is the
 * word W_v = word (v mod 4) of the Philox block kind 4, idx v div 4, and its
 * in-edges in ascending edge id own consecutive intervals [t_{k-1}, t_k),
 * t_k = floor(min(c_k, 1) * 2^32), c_k the fp64 running sum of their
 * weights; edge (u, v) is live iff W_v lies in its interval.  A sample is
 * the set reachable from S over live edges.  y_out, e_out and sums as in
 * oi_sample_mc (Y = |cascade| - |S|; is = |S| + mean(Y), oi = mean(Y)).
 * The per-edge intervals (8 bytes per edge) are made on the first LT call
 * and kept until the probabilities change.
 */
oi_status oi_sample_lt(oi_graph* g, uint32_t query_id, const int32_t* seeds, int64_t k, int stream, uint64_t first,
                       uint64_t count, uint32_t run_seed, uint32_t* y_out, uint64_t* e_out, oi_result* sums);

/*
 * oi_sample_fixed for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same samples, outputs and sums as oi_sample_fixed, with no hipMalloc,
 * hipFree or other allocating library call.  Its working memory (Stage-1
 * table, launch control block, hand-over lists, the large-cascade kernel's
 * bitmaps and queues) is one static device array of 64 MiB, which every GPU
 * the library runs on holds until the process ends.  y_out (device
 * uint32[count]) is required; e_out (device uint64[count]) may be NULL.
 * Limits: n <= 2^22 nodes, a Stage-1 table of at most 2^18 entries, at most
 * 2^16 distinct seeds, else OI_ERANGE; the graph's device must be current,
 * else OI_EINVAL.  Samples are drawn in launches of up to 2^19.  The array is
 * shared by every call on a GPU and keeps the last call's contents (the call
 * clears what must start empty): calls that overlap on one GPU, from any
 * graph or thread, race and must not be made.
 */
oi_status oi_sample_fixed_noalloc(oi_graph* g, uint32_t query_id, const int32_t* seeds, int64_t k, int stream,
                                  uint64_t first, uint64_t count, uint32_t run_seed, uint32_t* y_out,
                                  uint64_t* e_out, oi_result* sums);

/*
 * (eps, delta)-estimate of OI(S) and IS(S) = OI(S) + |S| (Sec. 2, estimation
 * problems) by SOIEA (Alg. 4) or SIEA (Alg. 5) with RSA (Alg. 3).
 * Requires 0 < eps < 1 and 0 < delta < 1/2.  beta_0 = 0 gives OI = 0,
 * IS = |S| without sampling.  out: host oi_result.
 */
oi_status oi_estimate(oi_graph* g, uint32_t query_id, const int32_t* seeds, int64_t k, double eps, double delta,
                      oi_mode mode, uint32_t run_seed, oi_result* out);

/*
 * Many seed sets at once: set q is seeds[seed_off[q] .. seed_off[q+1]) with
 * query id query_ids[q] (host arrays; seed_off has nq+1 entries).  Every set
 * keeps its own RSA state; each sampling round serves all unfinished sets in
 * one launch.  Per-set results are identical to oi_estimate with the same
 * query id.  out: host oi_result[nq]; out[q].status holds the set's status.
 */
oi_status oi_estimate_batch(oi_graph* g, int32_t nq, const int64_t* seed_off, const int32_t* seeds,
                            const uint32_t* query_ids, double eps, double delta, oi_mode mode,
                            uint32_t run_seed, oi_result* out);

/*
 * Score-function gradient of the fixed-count estimate beta_0 * mean(Y) of
 * OI(S) over samples first .. first+count-1 of stream X, with respect to
 * every edge probability (OI_PARAM_P) or to theta with p = sigmoid(theta)
 * (OI_PARAM_THETA), multiplied by grad_scale.  Each sample is recomputed from
 * its Philox key; y_in (device uint32[count], the forward's Y) may be NULL,
 * in which case the forward is run first.  Accumulation is exact (64-bit
 * integer sums of Y: per edge over the samples in which it is live, per node
 * over the samples that expand it, the dead sum of an edge being the
 * difference), finished in fp64 and written as fp32 to grad_out (device
 * float[m]; every entry is written).  The estimator is unbiased for edges
 * with 0 < p_e < 1.  The sums take 8 bytes per edge plus 8 bytes and one
 * bit per node of device memory, allocated on the first call and kept by the
 * graph until oi_graph_destroy.
 */
oi_status oi_backward(oi_graph* g, uint32_t query_id, const int32_t* seeds, int64_t k, uint64_t first,
                      uint64_t count, uint32_t run_seed, const uint32_t* y_in, oi_param param, double grad_scale,
                      float* grad_out);

/* Kernel timing collected with HIP events on the graph's stream.  Every
 * sampling launch runs three kernels: tiny (one sample per lane), small
 * (several samples per wavefront) and large (one block per sample); a sample
 * that outgrows one kernel is restarted from its key by the next. */
typedef struct {
  double tiny_ms, small_ms, large_ms; /* summed kernel times */
  uint64_t launches;                  /* sampling launches */
  uint64_t samples;                   /* samples produced */
  uint64_t handed_small;              /* samples passed from tiny to small */
  uint64_t handed_large;              /* samples passed from small to large */
  uint64_t tiny_y, tiny_edges;        /* sum of Y and examined edges of the samples each kernel finished */
  uint64_t small_y, small_edges;
  uint64_t large_y, large_edges;      /* (the large kernel's figures include its full-queue pass) */
  uint64_t handed_full;               /* samples passed to the large kernel's full-queue pass */
  uint64_t left_soft;                 /* ... of which left the main pool at the soft cap */
} oi_timing;

/* enable != 0 turns event timing on (and resets the counters). */
oi_status oi_timing_enable(oi_graph* g, int enable);
oi_status oi_timing_get(oi_graph* g, oi_timing* out);

/* Tuning.  variant: small-kernel variant (see oi_variant_info); chunk:
 * samples the small kernel takes per work-counter increment; tiny: 1 to run
 * the one-sample-per-lane kernel first (default), 0 to start every sample in
 * the small kernel; tiny_chunk: samples the tiny kernel takes per increment
 * (0 = automatic, the default; negative keeps the current setting);
 * round_max: samples per sampling launch (multiple of 4096, at most 2^31; the
 * default, set at graph creation, is the largest power of two up to 2^30 whose
 * round buffers, 36 bytes per sample, fit in a quarter of the free device
 * memory).  Negative (or
 * zero) values keep the current setting.  Results do not depend on any of
 * these. */
oi_status oi_set_tuning(oi_graph* g, int variant, int chunk, int tiny, int tiny_chunk, int64_t round_max);
/* Routing of large samples.  small_direct: 0 (default) lets the small
 * kernel forward the samples the tiny kernel hands over straight to the
 * large kernel when there are at most 128 of them per large-kernel block; 1
 * always forwards them (the small kernel does no sampling); 2 never does;
 * -1 keeps the setting.  The large kernel's main pool has queues of
 * min(n, 2^20) entries per block; a sample that activates more nodes than
 * that is finished by a second pass with n-entry queues and 1024-thread
 * blocks.  By default (large_qcap = 0) a soft cap adapts: after a launch in
 * which only a few samples (at most four per block of the second pass)
 * activated more than min(2^17, queue entries / 8) nodes, such samples of
 * the next launches leave the main pool once they pass that mark (at most
 * two per second-pass block per launch; later ones go on in the main pool),
 * so rare giant samples finish side by side in the second pass instead of
 * keeping one 256-thread block busy long after the rest of the launch;
 * after a launch with more of them the soft cap is lifted.  large_qcap > 0
 * fixes the queues at that many entries, with no soft cap.  Changing
 * large_qcap reallocates the pool.  Results do not depend on either
 * setting.  Errors: OI_EINVAL for a null graph or small_direct > 2. */
oi_status oi_set_routing(oi_graph* g, int small_direct, int64_t large_qcap);
/* First-level passes of the one-sample-per-lane kernel (a tuning and testing
 * aid; results never depend on it).  In a pass the kernel tests 64 new
 * samples of a segment at once for whether they end at their first
 * activated node (Alg. 1: no later Stage-1 entry and no out-edge of that
 * node into a node outside S live) and finishes those; the rest run the
 * cascade.  mode -1 (default): per launch, the instantiation with passes
 * over single-entry tables when at least 70% of the launch's samples are
 * expected to end so in them, else the one with passes over tables of up to
 * 16 entries when 70% do in all, else none; in either, only tables where
 * at least 20% are expected to end so take passes.  0: no passes.  1 / 2:
 * that instantiation for every launch, and passes for every table it
 * takes.  Applies to calls made after it; another mode gives OI_EINVAL. */
oi_status oi_set_first_level(oi_graph* g, int mode);
/* Queued RSA rounds.  In steps 2 and 3 of the RSA estimator (Alg. 3) the
 * number of samples is fixed when the step starts, so a round that neither
 * starts nor ends a step determines the next one.  mode 1 (the default):
 * the next round is queued on the stream before this one's sums are read
 * back, and the GPU does not wait for the host between them; 2: as 1, and
 * every round (table uploads, sampling kernels, reductions, read-back) is
 * captured as one graph and launched with one call (while event timing is
 * on, rounds are issued as in mode 1); 0: every round is read back before
 * the next is planned.  Results
 * do not depend on the mode.  Errors: OI_EINVAL for a null graph or a mode
 * outside 0..2. */
oi_status oi_set_pipeline(oi_graph* g, int mode);
/* Stage-1 skip sampling (part of the sampling specification; results depend
 * on it).  A Stage-1 table of l >= max(min_l, 65) entries (default min_l =
 * 4096) that passes the density test of oi_set_stage1_skip_cost is sampled
 * after the selection i (Alg. 1, Stage 1) without one coin per entry:
 * entries with P_j >= 1/2 keep their coins (kind 2); entries with
 * 0 < P_j < 1/2 are found by one walk per segment of 256 table indices.  In
 * segment m (indices [256m, 256m + 256)) R_j is the product of (1 - P_k) over
 * its entries k <= j with 0 < P_k < 1/2 (fp64, ascending k).  A walk stands
 * at pos = i if i lies in the segment, else at 256m - 1 with R = 1; it draws
 * U' = 1 - U with U the 53-bit uniform of Philox (kind 3, idx = pos, or
 * 2^40 + m at the segment's start), and the next live entry is the smallest
 * j > pos in the segment with R_j < U' * R_pos; the walk moves to j (idx = j)
 * and draws again, and ends when no such j exists.  Every later entry is
 * then live independently with probability P_j, as with one coin each, while
 * a sample draws about (l - i)/256 + sum_j P_j numbers instead of l - i.  The
 * examined-edge count still includes the l - 1 - i entries after i.
 * Applies to calls made after it; min_l < 1 gives OI_EINVAL. */
oi_status oi_set_stage1_skip(oi_graph* g, int64_t min_l);
/* The density test of Stage-1 skip sampling (part of the sampling
 * specification).  A walk step (a Philox draw whose counter is the walk's
 * last position, then a search) costs several coin blocks, so a long table is
 * skip-sampled only when W * cost <= l / 4, where W = ceil(l / 256) plus the
 * sum of P_j over its entries with 0 < P_j < 1/2 (fp64, the count first,
 * then ascending j) is the walks' expected number of draws from i = 0 and
 * l / 4 the number of coin blocks.  Default cost 8 (one walk step measured
 * at about 6.5 coin blocks on the 1M-node graph); cost 0 drops the test.
 * Applies to calls made after it; a negative or non-finite cost gives
 * OI_EINVAL. */
oi_status oi_set_stage1_skip_cost(oi_graph* g, double cost);

/* What oi_autotune chose and measured. */
typedef struct {
  int32_t variant;      /* small-kernel variant */
  int32_t tiny;         /* 1: the tiny kernel runs first */
  int32_t small_direct; /* as in oi_set_routing */
  int32_t candidates;   /* configurations timed */
  int32_t seed_sets;    /* pilot seed sets (beta_0 > 0) */
  int32_t pad;
  double best_ms;       /* pilot launch time of the chosen configuration */
  double default_ms;    /* ... of the default (tiny first, variant 0, automatic routing) */
} oi_autotune_result;

/* Sampler-schedule autotuner (a tuning aid; results never depend on it).
 * Times one sampling launch of `pilot` samples (stream X, samples
 * 0..pilot-1) of up to four of the nq seed sets (spread over the list, those
 * with beta_0 = 0 skipped), best of two runs after an untimed one, under
 * every combination of: the tiny kernel first
 * or not, each small-kernel variant, and automatic or always-direct routing
 * of hand-overs to the large kernel; then applies the fastest to the graph
 * (as oi_set_tuning / oi_set_routing would).  Seed sets are given as in
 * oi_estimate_batch.  pilot in [4096, round_max], else OI_ERANGE.  With no
 * seed set of positive beta_0 nothing is timed or changed (candidates = 0).
 * Uses the graph's Y workspace; blocks until done. */
oi_status oi_autotune(oi_graph* g, int32_t nq, const int64_t* seed_off, const int32_t* seeds,
                      const uint32_t* query_ids, uint64_t pilot, uint32_t run_seed, oi_autotune_result* out);
int oi_num_variants(void);
oi_status oi_variant_info(int variant, int* slots_per_wave, int* hash_cap, int* ring_cap, int* rounds_per_pass);

/* Measurement aid, outside the method: the random-gather bandwidth that the
 * samplers' Stage-2 reads (Alg. 1, the BFS over out-edges) are bound by, on
 * this graph.  For `count` nodes u, each the target of a uniformly random
 * edge h(seed, i) (a choice in proportion to in-degree, the law by which
 * cascades reach nodes), one GPU lane reads row_ptr[u], row_ptr[u+1] and
 * then u's out-edge targets and probabilities in the same 32-byte groups of
 * four edges that the samplers read; there are no coins, queues or visited
 * sets.  Outputs: useful_bytes = 16 * count + 8 * edges (the samplers'
 * algorithmic bytes per activated node and per examined edge), edges = the
 * out-edges read, ms = kernel time (HIP events on the graph's stream).  The
 * node list (4 * count bytes) is allocated and freed inside the call.
 * count in [1, 2^31], else OI_ERANGE; a graph with m = 0 gives OI_EINVAL. */
oi_status oi_gather_probe(oi_graph* g, uint64_t count, uint32_t seed, uint64_t* useful_bytes, uint64_t* edges,
                          double* ms);

/* Measurement aid, outside the method: the rate at which this GPU produces
 * the samplers' coins (Alg. 1 draws one uniform word per Stage-1 entry and
 * per probed edge; here one Philox4x32-10 draw of four words per edge group,
 * keyed and counted exactly as the samplers' edge coins: key (qid, seed),
 * kind 0, stream 0, sample s, group g).  Draws every group g in
 * [0, groups_per_sample) of every sample s in [0, samples) and compares its
 * four words with the fixed thresholds 0x19999999, 0x028F5C28, 0x00418937 and
 * 0x80000000 (word b against threshold b), with no loads, queues or visited
 * sets.  Outputs: live = words below their threshold (a checksum of the
 * draws), ms = kernel time (HIP events on the graph's stream).  samples in
 * [1, 2^40] and groups_per_sample in [1, 4096], else OI_ERANGE. */
oi_status oi_coin_probe(oi_graph* g, uint64_t samples, uint32_t groups_per_sample, uint32_t seed, uint32_t qid,
                        uint64_t* live, double* ms);

const char* oi_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* OI_H */
