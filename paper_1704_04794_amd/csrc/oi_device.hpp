// Device-side data layout shared by the HIP kernels and the host library code.
// Internal to the library: the public boundary is include/oi.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace oi {

// Out-edges in groups of four consecutive CSR edge ids (edge e lives in group
// e/4, lane e%4).  One group is 32 bytes, so a sampler lane reads the targets
// and coin thresholds of four edges with two 16-byte loads from one 64-byte
// line, and the four coins of a group come from one Philox block.  The
// threshold of an edge with probability p (fp32) is floor(p * 2^32) for
// p < 1 (at most 2^32 - 256) and 0xFFFFFFFF for p = 1, which is thereby
// unambiguous: the edge is live iff its coin word is below the threshold or
// the threshold is 0xFFFFFFFF.  Padding entries past m have v = 0, thr = 0
// and are never inside a row range.  The fp32 p themselves sit in a plain
// array of their own (read by the backward only).
struct alignas(32) EdgeGroup {
  int32_t v[4];
  uint32_t thr[4];
};

constexpr uint32_t kThrAlways = 0xFFFFFFFFu;

// The threshold of probability p in [0, 1] (fp32 arithmetic, exact: p * 2^32
// only shifts the exponent, and the conversion truncates).
__host__ __device__ inline uint32_t coin_threshold(float p) {
  return p >= 1.0f ? kThrAlways : (uint32_t)(p * 4294967296.0f);
}

// Stage-1 table entries in groups of four (entry j in group j/4): the
// neighbour v_j and its coin threshold floor(P_{S,v_j} * 2^32), which may be
// 2^32 when P = 1.  48 bytes per group.
struct alignas(16) TabGroup {
  int32_t v[4];
  uint64_t thr[4];
};

// One seed set's read-only data.
struct QueryDev {
  const double* cdf;     // l+1 values, cdf[0] = 0, cdf[l] = beta_0
  const TabGroup* tab;   // ceil(l/4) groups
  const int32_t* shash;  // open-addressing set of S (capacity smask+1), -1 = empty
  int64_t l;
  uint32_t smask;
  int32_t k;             // |S| after removing duplicates
  int32_t s0;            // the seed when k == 1
  uint32_t qid;          // Philox key word 0
  double beta0;
  // 1: the samples are classic IC Monte-Carlo cascades M^(S) (Sec. 2.3):
  // no Stage 1, every node of S active from the start, Y = the nodes
  // outside S that end active (zero allowed); 0: IICP samples (Alg. 1)
  int32_t mc;
  // 1 (with mc = 1): the cascades follow the LT model in its live-edge form:
  // node v keeps the in-edge whose interval of v's cumulative in-weights
  // holds v's choice word (Philox kind 4, idx v/4, word v%4)
  int32_t lt;
  // 1: Stage 1 after the selection by skip sampling (long tables): entries
  // with P >= 1/2 ("heavy", listed in `heavy`) by their own coins, the
  // others by one walk per kSkipSeg-entry segment over `skipR`, the product
  // of (1 - P_k) over the light entries of the segment up to each index
  int32_t skip;
  const double* skipR;   // l values (skip only)
  const int32_t* heavy;  // nheavy table indices, ascending (skip only)
  int64_t nheavy;
  // 1: the tiny kernel's first-level passes are worth running for this query
  // (tables of at most 16 entries; a decision of speed, not of results)
  int32_t p1;
};

// LT model: edge e is live iff lo <= W_v <= last for its target v's choice
// word W_v; an empty interval is stored as lo = 1, last = 0
struct LtEdge {
  uint32_t lo;
  uint32_t last;
};

constexpr int64_t kSkipSeg = 256;       // entries per skip-sampling segment
constexpr int64_t kSkipMinFloor = 65;   // shorter tables never use skip sampling

// A contiguous range of samples of one query's stream.  Samples of all
// segments of a launch are numbered by one flat index f; segment i covers
// f in [flat0, flat0 + count), sample index s = first + (f - flat0), output
// slot out_off + (f - flat0).
struct Segment {
  uint32_t q;
  uint32_t stream;
  uint64_t first;
  uint64_t count;
  uint64_t out_off;
  uint64_t flat0;
};

// One sampling launch.  Samples pass through up to three kernels, each of
// which either finishes a sample or hands it (by flat index) to the next:
//   tiny  (one sample per lane, <= TINY_CAP visited nodes)  -> list1
//   small (several samples per wavefront, LDS visited sets) -> list2
//   large (one block per sample, global bitmap)
struct SampleLaunch {
  int64_t n;
  const int64_t* row_ptr;
  const EdgeGroup* eg;
  const QueryDev* qs;
  const Segment* segs;
  int32_t nseg;
  uint64_t total;
  uint32_t seed;
  uint32_t* y_out;                 // per sample Y (null: only the per-segment sums are wanted)
  uint64_t* e_out;                 // per sample E (optional)
  unsigned long long* seg_sums;    // 2 per segment: sum Y, sum E
  unsigned long long* tier_sums;   // 2 per kernel (tiny, small, large): sum Y, sum E it finished
  unsigned long long* counter;     // flat work counter of the first kernel
  unsigned long long* counter1;    // work counter of the small kernel over list1
  unsigned long long* counter2;    // work counter of the large kernel over list2
  unsigned long long* list1;       // flat indices handed from tiny to small
  unsigned int* nlist1;
  unsigned long long* list2;       // flat indices handed from small to large
  unsigned int* nlist2;
  int32_t small_from_list1;        // 1 if the tiny kernel ran before the small one
  uint32_t small_direct_max;       // at most this many handed samples go straight to the large kernel
  unsigned int* err;               // nonzero on an internal inconsistency
  uint32_t chunk;                  // samples the small kernel takes per counter increment
  uint32_t tiny_chunk;             // samples the tiny kernel takes per counter increment
  // large-cascade kernel workspace: per block a visited bitmap and a queue
  // of qcap entries (queue_stride apart); a sample that activates more than
  // qcap nodes is abandoned and its flat index appended to list3, for a
  // second pass with blocks whose queues hold n entries
  uint32_t* bits;
  int32_t* queue;
  int64_t bits_words;
  uint32_t qcap;
  int64_t queue_stride;
  unsigned long long* list3;       // null in that second pass
  unsigned int* nlist3;
  // backward accumulators (null in the forward)
  const uint32_t* y_in;            // per-sample Y from the forward
  unsigned long long* acc_live;    // per edge: sum of Y over samples where the edge is revealed live
  // per node u: sum of Y over samples that expand u.  Every out-edge of an
  // expanded node is revealed unless its target is in S, so an edge's
  // "revealed dead" sum is acc_node[u] - acc_live[e]: one atomic per
  // expanded node instead of one per dead edge
  unsigned long long* acc_node;
  unsigned long long* acc_tab;     // per Stage-1 entry: sum of Y over samples with x_j = 1
  // backward: S as an n-bit bitmap (one load per membership test instead
  // of a probe of the seed-set hash), or null
  const uint32_t* sbits;
  // the large kernel counts the samples it finishes with more than big_mark
  // activations (null: no count); the host sets the next launch's soft cap
  // from it
  unsigned int* nbig;
  uint32_t big_mark;
  // forward large kernel: a sample that activates more than soft_cap (<=
  // qcap) nodes leaves for the full-queue pass if fewer than soft_budget
  // samples of the launch have left that way (counted in nsoft), and
  // otherwise continues up to qcap; soft_cap == qcap turns this off
  uint32_t soft_cap;
  uint32_t soft_budget;
  unsigned int* nsoft;
  // 1: every query of the launch draws classic Monte-Carlo cascades
  // (QueryDev::mc), which the tiny kernel runs in an instantiation of its own
  int32_t mc;
  // 1: every query of the launch draws LT-model cascades (QueryDev::lt); the
  // tiny kernel does not run, the small kernel forwards every sample and the
  // large kernel runs an instantiation of its own
  int32_t lt;
  const LtEdge* lt_iv;             // per edge (LT launches)
  // the tiny kernel's instantiation (chosen on the host from how often the
  // launch's samples are expected to end at their first activated node): 0
  // without first-level passes, 1 with passes over single-entry Stage-1
  // tables, 2 with passes over tables of up to 16 entries
  int32_t p1;
};

// Hash used for the per-query seed set table (built on the host, probed on the device).
__host__ __device__ inline uint32_t mix32(uint32_t v) {
  v ^= v >> 16;
  v *= 0x7feb352du;
  v ^= v >> 15;
  v *= 0x846ca68bu;
  v ^= v >> 16;
  return v;
}

constexpr int KIND_EDGE = 0;
constexpr int KIND_SELECT = 1;
constexpr int KIND_STAGE1 = 2;
constexpr int KIND_SKIP = 3;
constexpr int KIND_LT = 4;

}  // namespace oi
