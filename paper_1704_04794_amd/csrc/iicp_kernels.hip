// HIP kernels for IICP sampling (Alg. 1), its score-function backward, and the
// integer reductions the stopping rules need (Algs. 2 and 3).
//
// Sampling is split over two kernels:
//   * tiny_kernel: persistent; every lane runs one sample as a small state
//     machine (start / Stage-1 group / edge group / pop), with its visited
//     list in LDS; each loop iteration costs one Philox block per lane.  A
//     sample that would visit more than TINY_CAP nodes (or whose Stage-1
//     table is long) is handed to small_kernel.
//   * small_kernel: persistent; every wavefront runs K samples at once, each
//     with a visited set in LDS (open addressing) and a shared LDS ring of
//     pending expansion items.  Each pass the wave gathers up to 64 items,
//     load-balances their edge groups over its 64 lanes (prefix sum +
//     binary search), draws one Philox block per group of four edges, and
//     inserts the live, unvisited, non-seed targets.  A sample whose visited
//     set would exceed the LDS capacity is abandoned and handed over by its
//     flat index.
//   * large_kernel: one 256-thread block per handed-over sample; it restarts
//     the sample from its counter key with a global visited bitmap and a
//     global queue.
// Both produce the same visited set as the sequential algorithm, because
// every coin is a pure function of (query, stream, sample, edge id): the set
// of activated nodes is the closure of the Stage-1 set under live edges,
// whatever order the edges are examined in.
#include <type_traits>
#include "oi_device.hpp"

namespace oi {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and the coin conventions
// ---------------------------------------------------------------------------
struct Words {
  uint32_t w[4];
};

// a ^ b ^ c in one instruction (gfx950's three-input bitwise operation;
// 0x96 is the truth table of the three-way exclusive or)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ Words philox_draw(uint32_t k0, uint32_t k1, uint32_t kind, uint32_t stream,
                                             uint64_t s, uint64_t idx) {
  uint32_t c0 = (uint32_t)idx, c1 = (uint32_t)(idx >> 32), c2 = (uint32_t)s;
  uint32_t c3 = (kind << 28) | (stream << 27) | ((uint32_t)(s >> 32) & 0x07FFFFFFu);
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t a = (uint64_t)0xD2511F53u * (uint64_t)c0;
    const uint64_t b = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    const uint32_t n0 = xor3((uint32_t)(b >> 32), c1, k0);
    const uint32_t n2 = xor3((uint32_t)(a >> 32), c3, k1);
    c1 = (uint32_t)b;
    c3 = (uint32_t)a;
    c0 = n0;
    c2 = n2;
  }
  Words o;
  o.w[0] = c0;
  o.w[1] = c1;
  o.w[2] = c2;
  o.w[3] = c3;
  return o;
}

// Pointers read out of device structures are generic; these casts let the
// compiler issue global (not flat) loads through them.
#define OI_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ const OI_GLOBAL T* gptr(const T* p) {
  return (const OI_GLOBAL T*)p;
}
// Launch-invariant data (segments, query descriptors) read through the
// constant address space: wave-uniform loads from it become scalar loads.
#define OI_CONST __attribute__((address_space(4)))
template <typename T>
__device__ __forceinline__ const OI_CONST T* cptr(const T* p) {
  return (const OI_CONST T*)p;
}

typedef int v4i32 __attribute__((ext_vector_type(4)));
// the same, for 16-byte loads at 8-byte aligned addresses (a row_ptr pair)
typedef int v4i32_a8 __attribute__((ext_vector_type(4), aligned(8)));
typedef unsigned long long v2u64 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ TabGroup load_tab(const TabGroup* base, int64_t g) {
  const OI_GLOBAL char* p = (const OI_GLOBAL char*)(gptr(base) + g);
  const v4i32 v = *(const OI_GLOBAL v4i32*)p;
  const v2u64 t0 = *(const OI_GLOBAL v2u64*)(p + 16);
  const v2u64 t1 = *(const OI_GLOBAL v2u64*)(p + 32);
  TabGroup T;
  T.v[0] = v.x;
  T.v[1] = v.y;
  T.v[2] = v.z;
  T.v[3] = v.w;
  T.thr[0] = t0.x;
  T.thr[1] = t0.y;
  T.thr[2] = t1.x;
  T.thr[3] = t1.y;
  return T;
}

// v of Stage-1 entry j
__device__ __forceinline__ int32_t tab_v(const TabGroup* base, int64_t j) {
  const OI_GLOBAL char* p = (const OI_GLOBAL char*)(gptr(base) + (j >> 2));
  return *(const OI_GLOBAL int32_t*)(p + 4 * (j & 3));
}

// coin threshold of Stage-1 entry j
__device__ __forceinline__ uint64_t tab_thr(const TabGroup* base, int64_t j) {
  const OI_GLOBAL char* p = (const OI_GLOBAL char*)(gptr(base) + (j >> 2));
  return *(const OI_GLOBAL uint64_t*)(p + 16 + 8 * (j & 3));
}

// word k (0..3) of a Philox block, k chosen at run time
__device__ __forceinline__ uint32_t word_at(const Words& d, int64_t k) {
  return k == 0 ? d.w[0] : k == 1 ? d.w[1] : k == 2 ? d.w[2] : d.w[3];
}

// Live iff word < floor(p * 2^32); p = 1 (threshold kThrAlways) is always
// live.  See coin_threshold.
__device__ __forceinline__ bool edge_live(uint32_t word, uint32_t thr) {
  return word < thr || thr == kThrAlways;
}

// Alg. 1, Stage 1 selection: t = U * beta_0, i = min{j : CDF_j > t}; if no
// entry qualifies, the last entry with Pr[A_j] > 0.
__device__ int64_t select_entry(const QueryDev& Q, uint32_t seed, uint32_t stream, uint64_t s) {
  const Words d = philox_draw(Q.qid, seed, KIND_SELECT, stream, s, 0);
  const uint64_t a = d.w[0] >> 5, b = d.w[1] >> 6;
  const double U = (double)(a * 67108864ull + b) * (1.0 / 9007199254740992.0);
  const double t = U * Q.beta0;
  const OI_GLOBAL double* cdf = gptr(Q.cdf);
  int64_t lo = 0, hi = Q.l;
  while (lo < hi) {
    const int64_t mid = lo + ((hi - lo) >> 1);
    if (cdf[mid + 1] > t)
      hi = mid;
    else
      lo = mid + 1;
  }
  if (lo < Q.l) return lo;
  for (int64_t j = Q.l - 1; j >= 0; --j)
    if (cdf[j + 1] > cdf[j]) return j;
  return -1;
}

__device__ __forceinline__ bool in_seed_set(const QueryDev& Q, int32_t v) {
  if (Q.k == 1) return v == Q.s0;
  uint32_t h = mix32((uint32_t)v) & Q.smask;
  while (true) {
    const int32_t c = gptr(Q.shash)[h];
    if (c == v) return true;
    if (c < 0) return false;
    h = (h + 1) & Q.smask;
  }
}

// membership in the backward's bitmap of S
__device__ __forceinline__ bool seed_bit(const uint32_t* sbits, int32_t v) {
  return (gptr(sbits)[(uint32_t)v >> 5] >> ((uint32_t)v & 31u)) & 1u;
}

__device__ __forceinline__ bool in_seed_fields(int32_t k, int32_t s0, uint32_t smask, const int32_t* shash,
                                               int32_t v) {
  if (k == 1) return v == s0;
  uint32_t h = mix32((uint32_t)v) & smask;
  while (true) {
    const int32_t c = gptr(shash)[h];
    if (c == v) return true;
    if (c < 0) return false;
    h = (h + 1) & smask;
  }
}

// find_segment for a wave-uniform flat index (scalar loads)
__device__ __forceinline__ uint32_t find_segment_uniform(const SampleLaunch& A, uint64_t f) {
  const OI_CONST Segment* segs = cptr(A.segs);
  int32_t lo = 0, hi = A.nseg - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (segs[mid].flat0 <= f)
      lo = mid;
    else
      hi = mid - 1;
  }
  return (uint32_t)lo;
}

__device__ __forceinline__ uint32_t find_segment(const SampleLaunch& A, uint64_t f) {
  int32_t lo = 0, hi = A.nseg - 1;  // last segment with flat0 <= f
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (A.segs[mid].flat0 <= f)
      lo = mid;
    else
      hi = mid - 1;
  }
  return (uint32_t)lo;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t lane_prefix(unsigned long long mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

template <typename T>
__device__ __forceinline__ T uniform(T v) {
  return (T)__builtin_amdgcn_readfirstlane((int)v);
}
__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  return x;
}

// Sum of a 64-bit value over the 64 lanes of the wave (every lane gets it).
__device__ __forceinline__ unsigned long long wave_sum64(unsigned long long x) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) x += __shfl_xor(x, d, 64);
  return x;
}

// Add the per-lane (segment, Y sum, E sum) accumulators of the lanes with
// `pred` to seg_sums and to the tier's two totals, one atomic per distinct
// segment in the wave rather than one per lane: same-address atomics from
// every lane of every wave serialise at the memory side.  Must be reached by
// the whole wave.
__device__ __forceinline__ void wave_flush(bool pred, uint32_t seg, unsigned long long y, unsigned long long e,
                                           unsigned long long* seg_sums, unsigned long long* tier, int lane) {
  unsigned long long todo = __ballot(pred);
  while (todo) {
    const int leader = __builtin_ctzll(todo);
    const uint32_t sq = uniform((uint32_t)__shfl((int)seg, leader, 64));
    const bool mine = pred && seg == sq;
    const unsigned long long sy = wave_sum64(mine ? y : 0ull);
    const unsigned long long se = wave_sum64(mine ? e : 0ull);
    if (lane == leader) {
      atomicAdd(&seg_sums[2 * sq], sy);
      atomicAdd(&seg_sums[2 * sq + 1], se);
      atomicAdd(&tier[0], sy);
      atomicAdd(&tier[1], se);
    }
    todo &= ~__ballot(mine);
  }
}

// ---------------------------------------------------------------------------
// tiny_kernel: one sample per lane
// ---------------------------------------------------------------------------
constexpr uint32_t TINY_LMAX = 64;  // longest Stage-1 table the tiny kernel takes
constexpr uint32_t P1_MAXG = 16;    // first-level passes: v_0's row spans at most this many edge groups
constexpr uint32_t P1_PEND = 256;   // first-level passes: pending samples per wave (a power of two)
constexpr uint32_t P1L_MAXL = 16;   // first-level passes: longest Stage-1 table they take
constexpr uint32_t P1_DIRG = 8;     // single-entry passes hand their coins on for rows of at most this many groups
enum : uint32_t { T_IDLE = 0, T_START = 1, T_STAGE1 = 2, T_EXPAND = 3, T_POP = 4 };

// Append the flat indices of the lanes with `pred` to a hand-over list.
// Must be reached by the whole wave.
__device__ __forceinline__ void hand_over(bool pred, uint64_t f, unsigned long long* list, unsigned int* nlist,
                                          int lane) {
  const unsigned long long m = __ballot(pred);
  if (m) {
    unsigned int base = 0;
    if (lane == 0) base = atomicAdd(nlist, (unsigned int)__popcll(m));
    base = (unsigned int)__builtin_amdgcn_readfirstlane((int)__shfl(base, 0, 64));
    if (pred) list[base + lane_prefix(m)] = f;
  }
}

// Wave-uniform state of the tiny kernel's first-level passes: whether the
// current segment takes them (and whether its table has several entries),
// for a single entry v_0 its edge groups (count, first), counted slots and
// out-degree, the samples the passes finished in the segment with their E
// sum, and the pending list's bounds [head, tail).
struct FirstLevel {
  bool on, gen;  // passes in this segment; a table of 2..P1L_MAXL entries
  uint32_t ng, g0;
  unsigned long long mask, deg, n, e;  // e: the E sum of the samples finished by passes
  uint32_t head, tail;
};
struct NoFirstLevel {};

// MC: the launch's samples are classic Monte-Carlo cascades (Sec. 2.3), a
// separate instantiation so that the IICP loop carries none of their
// bookkeeping.  PASS: the forward IICP instantiation with first-level passes,
// over single-entry tables only (1) or over tables of up to P1L_MAXL entries (2).
// Each instantiation is given the occupancy it is held to: five waves per
// SIMD for the single-entry pass variant and four for the general one (they
// need more registers; the former spills ten values for its fifth wave), six
// for the forward without passes (a few spilled values), five for the
// backward.
template <int CAP, bool BWD, bool MC, int PASS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PASS == 1 ? 5 : (PASS ? 4 : (BWD ? 5 : 6))))) tiny_kernel(SampleLaunch A) {
  __shared__ int32_t vis_all[4][CAP * 64];
  // the current segment's CDF and table nodes (tables of 2..TINY_LMAX
  // entries): the samples a wave starts in an iteration all come from that
  // segment, and select their first entry in the same iteration
  __shared__ double cdf_all[4][TINY_LMAX + 1];
  __shared__ int32_t tv_all[4][TINY_LMAX];
  const int lane = threadIdx.x & 63;
  int32_t* vis = &vis_all[threadIdx.x >> 6][lane];  // entry c of this lane at vis[64 * c]
  double* wcdf = cdf_all[threadIdx.x >> 6];
  int32_t* wtv = tv_all[threadIdx.x >> 6];

  // lane state; the query's fields are copied into registers when a sample
  // starts, so no iteration re-reads shared structures
  uint32_t st = T_IDLE;
  uint64_t f = 0, s = 0, oidx = 0;
  uint32_t sg = 0, stream = 0, cnt = 0, qh = 0, y = 0, g = 0, gend = 0;
  uint32_t qid = 0, smask = 0;
  int32_t qk = 0, s0 = 0;
  int64_t ql = 0;
  const TabGroup* tab = nullptr;
  const int32_t* shash = nullptr;
  unsigned long long E = 0;
  uint32_t lo_e = 0, hi_e = 0;  // edge ids (m < 2^32) or Stage-1 entry indices
  // the wave's current work chunk [cur, cend) and the segment of cur
  // (wave-uniform); every refill hands out samples of one segment only, so
  // the segment and its query are read with scalar loads, once per refill
  uint64_t cur = 0, cend = 0, cseg_end = 0;
  uint32_t cseg = 0;
  // the current segment and its query (wave-uniform, refreshed when cur
  // crosses a segment boundary)
  uint64_t c_first = 0, c_flat0 = 0, c_out = 0;
  uint32_t c_stream = 0, c_qid = 0, c_smask = 0;
  int32_t c_k = 0, c_s0 = 0;
  int64_t c_l = 0;
  const TabGroup* c_tab = nullptr;
  const int32_t* c_shash = nullptr;
  // when the segment's Stage-1 table has a single entry, that entry v_0 and
  // its row bounds: every sample of the segment starts by popping v_0
  int32_t c_v0 = 0, c_v0v = 0;
  int64_t c_rb0 = 0, c_re0 = 0;
  // first-level passes (the forward IICP kernel; segments whose Stage-1 table
  // has a single entry v_0 with at most P1_MAXG edge groups): the wave tests
  // 64 new samples at a time for a live out-edge of v_0, finishes those
  // without one, and queues the others in a per-wave list of P1_PEND
  // segment-relative indices, from which its lanes start the cascades.
  // Everything here is wave-uniform.
  constexpr bool P1 = PASS != 0 && !BWD && !MC;
  constexpr bool P1GEN = P1 && PASS == 2;  // passes also over tables of several entries
  constexpr bool P1DIR = P1 && PASS == 1;  // pending samples start from their pass's live out-edges of v_0
  __shared__ uint32_t p1thr_all[4][P1 ? 4 * P1_MAXG : 1];
  __shared__ uint32_t pend_all[4][P1 ? P1_PEND : 1];
  // single-entry tables with v_0's row within P1_DIRG groups: the targets of
  // v_0's counted slots, and for each pending sample its live counted slots
  // (its cascade then starts from them instead of drawing v_0's coins again)
  __shared__ int32_t p1tgt_all[4][P1DIR ? 4 * P1_DIRG : 1];
  __shared__ uint32_t pmask_all[4][P1DIR ? P1_PEND : 1];
  // tables of 2..P1L_MAXL entries: each entry's Stage-1 coin threshold and
  // its node's row bounds
  __shared__ uint64_t p1sthr_all[4][P1GEN ? P1L_MAXL : 1];
  __shared__ uint32_t p1rb_all[4][P1GEN ? P1L_MAXL : 1];
  __shared__ uint32_t p1re_all[4][P1GEN ? P1L_MAXL : 1];
  uint32_t* wp1thr = p1thr_all[threadIdx.x >> 6];
  uint32_t* wpend = pend_all[threadIdx.x >> 6];
  int32_t* wp1tgt = p1tgt_all[threadIdx.x >> 6];
  uint32_t* wpmask = pmask_all[threadIdx.x >> 6];
  uint32_t pmask = 0;  // a pending sample's live counted slots of v_0 (0: none handed on)
  uint64_t* wsthr = p1sthr_all[threadIdx.x >> 6];
  uint32_t* wrb = p1rb_all[threadIdx.x >> 6];
  uint32_t* wre = p1re_all[threadIdx.x >> 6];
  std::conditional_t<P1, FirstLevel, NoFirstLevel> pw{};
  // which per-sample outputs the launch wants, in one scalar word
  const uint32_t outs = __builtin_amdgcn_readfirstlane((A.y_out ? 1u : 0u) | (A.e_out ? 2u : 0u));
  bool exhausted = false;
  uint32_t acc_seg = 0xFFFFFFFFu;
  unsigned long long acc_y = 0, acc_e = 0;

  while (true) {
    // the output flags, tested where the outputs are written; the empty asm
    // makes them look new each iteration, so the tests are not turned into
    // lane masks kept (and spilled) across the loop
    uint32_t o = outs;
    asm volatile("" : "+s"(o));
    // (0) lanes whose queue is drained finish their sample.  A lane whose
    // sample belongs to another segment than its running sums flushes them
    // first; lanes reach segment ends at different times, so these atomics
    // rarely meet on one address (the final flush, where they would, is
    // wave-cooperative)
    if (st == T_POP && qh == cnt) {
      if (MC) --cnt;  // a Monte-Carlo sample does not count its seed
      if (BWD) {
        if (cnt != y) atomicOr(A.err, 2u);
      } else {
        if (o & 1u) A.y_out[oidx] = cnt;
        if (o & 2u) A.e_out[oidx] = E;
      }
      if (sg != acc_seg) {
        if (acc_seg != 0xFFFFFFFFu) {
          atomicAdd(&A.seg_sums[2 * acc_seg], acc_y);
          atomicAdd(&A.seg_sums[2 * acc_seg + 1], acc_e);
          atomicAdd(&A.tier_sums[0], acc_y);
          atomicAdd(&A.tier_sums[1], acc_e);
        }
        acc_seg = sg;
        acc_y = 0;
        acc_e = 0;
      }
      acc_y += cnt;
      acc_e += E;
      st = T_IDLE;
    }
    const unsigned long long idle = __ballot(st == T_IDLE);
    bool started = false;
    if constexpr (P1) {
      // (1) idle lanes take new samples, all from the segment of `cur`: in a
      // segment that takes first-level passes (below), samples that a pass
      // found to need the cascade; otherwise the next samples of the chunk
      if (idle && !(exhausted && pw.head == pw.tail)) {
        const uint32_t nidle = (uint32_t)__popcll(idle);
        // a segment's pending samples are started before the wave moves on
        if ((cur >= cend || cur >= cseg_end) && !exhausted && !(P1 && pw.head != pw.tail)) {
          if (cur >= cend) {
            unsigned long long c = 0;
            if (lane == 0) c = atomicAdd(A.counter, (unsigned long long)A.tiny_chunk);
            c = uniform64(__shfl(c, 0, 64));
            if (c >= A.total) {
              exhausted = true;
            } else {
              cur = c;
              cend = c + A.tiny_chunk < A.total ? c + A.tiny_chunk : A.total;
            }
          }
          if (!exhausted && cur >= cseg_end) {
            if (P1 && pw.n) {
              // the samples the first-level passes finished in the old segment
              if (lane == 0) {
                atomicAdd(&A.seg_sums[2 * cseg], pw.n);
                atomicAdd(&A.seg_sums[2 * cseg + 1], pw.e);
                atomicAdd(&A.tier_sums[0], pw.n);
                atomicAdd(&A.tier_sums[1], pw.e);
              }
              pw.n = 0;
              pw.e = 0;
            }
            cseg = uniform(find_segment_uniform(A, cur));
            const OI_CONST Segment* Sp = cptr(A.segs) + cseg;
            c_flat0 = Sp->flat0;
            c_first = Sp->first;
            c_out = Sp->out_off;
            c_stream = Sp->stream;
            cseg_end = c_flat0 + Sp->count;
            const OI_CONST QueryDev* Qp = cptr(A.qs) + Sp->q;
            c_qid = Qp->qid;
            c_l = Qp->l;
            c_k = Qp->k;
            c_s0 = Qp->s0;
            c_smask = Qp->smask;
            c_shash = Qp->shash;
            c_tab = Qp->tab;
            if (!MC && c_l > 1 && c_l <= (int64_t)TINY_LMAX) {
              const OI_GLOBAL double* qc = gptr(Qp->cdf);
              for (int64_t x = lane; x <= c_l; x += 64) wcdf[x] = qc[x];
              if (lane < c_l) wtv[lane] = tab_v(c_tab, lane);
              wave_sync();
            }
            pw.on = false;
            pw.gen = false;
            if (P1GEN && c_l > 1 && c_l <= (int64_t)P1L_MAXL && Qp->p1) {
              // (the entries' nodes are in wtv already)
              if (lane < c_l) {
                wsthr[lane] = tab_thr(c_tab, lane);
                const int32_t v = wtv[lane];
                wrb[lane] = (uint32_t)cptr(A.row_ptr)[v];
                wre[lane] = (uint32_t)cptr(A.row_ptr)[v + 1];
              }
              wave_sync();
              pw.on = true;
              pw.gen = true;
            }
            if (!MC && c_l == 1) {
              c_v0 = cptr(c_tab)->v[0];
              c_rb0 = cptr(A.row_ptr)[c_v0];
              c_re0 = cptr(A.row_ptr)[c_v0 + 1];
              // v_0 is only ever stored to LDS: kept in a vector register
              // (the empty asm places it there) it costs no scalar register
              // across the loop and no move at each start
              c_v0v = c_v0;
              asm volatile("" : "+v"(c_v0v));
              const int64_t ng = c_re0 > c_rb0 ? ((c_re0 + 3) >> 2) - (c_rb0 >> 2) : 0;
              if (P1 && ng <= (int64_t)P1_MAXG) {
                // v_0's edges, read once per segment: slot x (= lane) of the
                // row's groups counts iff it is one of v_0's out-edges and its
                // target lies outside S (an edge into S activates nothing).
                // Passes are taken when the host found that samples often end
                // at v_0
                bool counted = false;
                uint32_t thr = 0;
                int32_t tgt = -1;
                const int64_t e = 4 * (c_rb0 >> 2) + lane;
                if (lane < 4 * ng && e >= c_rb0 && e < c_re0) {
                  const OI_GLOBAL EdgeGroup* grp = gptr(A.eg) + (e >> 2);
                  tgt = grp->v[e & 3];
                  thr = grp->thr[e & 3];
                  counted = !in_seed_fields(c_k, c_s0, c_smask, c_shash, tgt);
                }
                wp1thr[lane] = thr;
                if (P1DIR && lane < 4 * P1_DIRG) wp1tgt[lane] = tgt;
                pw.on = Qp->p1 != 0;
                pw.ng = (uint32_t)ng;
                pw.g0 = (uint32_t)(c_rb0 >> 2);
                pw.deg = (unsigned long long)(c_re0 - c_rb0);
                pw.mask = __ballot(counted);
                wave_sync();
              }
            }
          }
        }
        while (P1 && pw.on && pw.tail - pw.head < nidle && cur < (cend < cseg_end ? cend : cseg_end)) {
          // a first-level pass over the next (up to) 64 samples, one per lane:
          // v_0 is activated (the single entry is selected whatever U is, and
          // no entry follows), and its out-edges' coins are drawn; a sample in
          // which none of them is live into a node outside S is finished here
          // (Y = 1, E = deg(v_0)), the others are queued for the cascade
          {
            const uint64_t lim = cend < cseg_end ? cend : cseg_end;
            const uint32_t take = lim - cur < 64ull ? (uint32_t)(lim - cur) : 64u;
            const bool valid = (uint32_t)lane < take;
            const uint64_t off = cur - c_flat0 + (uint64_t)lane;
            const uint64_t ps = c_first + off;
            uint32_t pseed = A.seed;
            asm volatile("" : "+s"(pseed));
            bool need = false;           // the sample needs the cascade
            unsigned long long eo = 0;   // its E if it ends at its first node
            uint32_t lm = 0;             // its live counted slots (rows within P1_DIRG groups)
            if (!P1GEN || !pw.gen) {
  #pragma unroll 1
              for (uint32_t gi = 0; gi < pw.ng; ++gi) {
                const Words d = philox_draw(c_qid, pseed, KIND_EDGE, c_stream, ps, (uint64_t)(pw.g0 + gi));
  #pragma unroll
                for (int b = 0; b < 4; ++b) {
                  const uint32_t slot = 4 * gi + (uint32_t)b;
                  if (((pw.mask >> slot) & 1ull) && edge_live(d.w[b], wp1thr[slot])) {
                    need = true;
                    if (P1DIR && slot < 32u) lm |= 1u << slot;
                  }
                }
              }
              if (pw.ng > P1_DIRG) lm = 0;
              eo = pw.deg;
            } else if constexpr (P1GEN) {
              // Alg. 1 for a table of several entries: the selection i (as the
              // state machine makes it; its rare fallback is left to it), the
              // coins of the later entries, then the coins of v_i's out-edges
              const Words dsel = philox_draw(c_qid, pseed, KIND_SELECT, c_stream, ps, 0ull);
              const uint64_t ua = dsel.w[0] >> 5, ub = dsel.w[1] >> 6;
              const double U = (double)(ua * 67108864ull + ub) * (1.0 / 9007199254740992.0);
              const double t = U * wcdf[c_l];
              int64_t lo = 0, hi = c_l;
              while (lo < hi) {
                const int64_t mid = lo + ((hi - lo) >> 1);
                if (wcdf[mid + 1] > t)
                  hi = mid;
                else
                  lo = mid + 1;
              }
              need = lo >= c_l;
              const int64_t i = need ? 0 : lo;
              for (int64_t g = (i + 1) >> 2; !need && 4 * g < c_l; ++g) {
                const Words d = philox_draw(c_qid, pseed, KIND_STAGE1, c_stream, ps, (uint64_t)g);
  #pragma unroll
                for (int b = 0; b < 4; ++b) {
                  const int64_t j = 4 * g + b;
                  if (j > i && j < c_l && (uint64_t)d.w[b] < wsthr[j]) need = true;
                }
              }
              const uint32_t rb = wrb[i], re = wre[i];
              const uint32_t g0 = rb >> 2, ng = re > rb ? ((re + 3) >> 2) - g0 : 0u;
              if (ng > P1_MAXG) need = true;
              for (uint32_t gi = 0; !need && gi < ng; ++gi) {
                const Words d = philox_draw(c_qid, pseed, KIND_EDGE, c_stream, ps, (uint64_t)(g0 + gi));
                const OI_GLOBAL char* q = (const OI_GLOBAL char*)(gptr(A.eg) + g0 + gi);
                const v4i32 tv = *(const OI_GLOBAL v4i32*)q;
                const v4i32 tp = *(const OI_GLOBAL v4i32*)(q + 16);
  #pragma unroll
                for (int b = 0; b < 4; ++b) {
                  const uint32_t e = 4 * (g0 + gi) + (uint32_t)b;
                  if (e >= rb && e < re && edge_live(d.w[b], (uint32_t)tp[b]) &&
                      !in_seed_fields(c_k, c_s0, c_smask, c_shash, tv[b]))
                    need = true;
                }
              }
              eo = (unsigned long long)(c_l - 1 - i) + (re - rb);
            }
            const bool done = valid && !need;
            const bool more = valid && need;
            if (done) {
              if (o & 1u) A.y_out[c_out + off] = 1u;
              if (o & 2u) A.e_out[c_out + off] = eo;
            }
            const unsigned long long dm = __ballot(done), mm = __ballot(more);
            pw.n += (unsigned long long)__popcll(dm);
            if (P1GEN && pw.gen)
              pw.e += uniform64(wave_sum64(done ? eo : 0ull));
            else
              pw.e += (unsigned long long)__popcll(dm) * pw.deg;
            if (more) {
              const uint32_t slot = (pw.tail + lane_prefix(mm)) & (P1_PEND - 1);
              wpend[slot] = (uint32_t)off;
              if (P1DIR) wpmask[slot] = lm;
            }
            pw.tail += (uint32_t)__popcll(mm);
            wave_sync();
            cur += take;
          }
        }
        if (P1 && pw.head != pw.tail) {
          // pending samples of the current segment go to idle lanes
          const uint32_t npend = pw.tail - pw.head;
          const uint32_t take = npend < nidle ? npend : nidle;
          const uint32_t rank = lane_prefix(idle);
          if (st == T_IDLE && rank < take) {
            const uint32_t slot = (pw.head + rank) & (P1_PEND - 1);
            f = c_flat0 + wpend[slot];
            if (P1DIR) pmask = wpmask[slot];
            st = T_START;
            started = true;
          }
          pw.head += take;
        } else if (!exhausted && !(P1 && pw.on)) {
          const uint64_t lim = cend < cseg_end ? cend : cseg_end;
          const uint64_t room = lim - cur;
          const uint32_t take = room < (uint64_t)nidle ? (uint32_t)room : nidle;
          const uint32_t rank = lane_prefix(idle);
          if (st == T_IDLE && rank < take) {
            f = cur + rank;
            pmask = 0;
            st = T_START;
            started = true;
          }
          cur += take;
        }
      }
    } else {
      // (1) idle lanes take the next samples of the wave's chunk, all from the
      // segment of `cur`
      if (idle && !exhausted) {
        if (cur >= cend) {
          unsigned long long c = 0;
          if (lane == 0) c = atomicAdd(A.counter, (unsigned long long)A.tiny_chunk);
          c = uniform64(__shfl(c, 0, 64));
          if (c >= A.total) {
            exhausted = true;
          } else {
            cur = c;
            cend = c + A.tiny_chunk < A.total ? c + A.tiny_chunk : A.total;
          }
        }
        if (!exhausted) {
          if (cur >= cseg_end) {
            cseg = uniform(find_segment_uniform(A, cur));
            const OI_CONST Segment* Sp = cptr(A.segs) + cseg;
            c_flat0 = Sp->flat0;
            c_first = Sp->first;
            c_out = Sp->out_off;
            c_stream = Sp->stream;
            cseg_end = c_flat0 + Sp->count;
            const OI_CONST QueryDev* Qp = cptr(A.qs) + Sp->q;
            c_qid = Qp->qid;
            c_l = Qp->l;
            c_k = Qp->k;
            c_s0 = Qp->s0;
            c_smask = Qp->smask;
            c_shash = Qp->shash;
            c_tab = Qp->tab;
            if (!MC && c_l > 1 && c_l <= (int64_t)TINY_LMAX) {
              const OI_GLOBAL double* qc = gptr(Qp->cdf);
              for (int64_t x = lane; x <= c_l; x += 64) wcdf[x] = qc[x];
              if (lane < c_l) wtv[lane] = tab_v(c_tab, lane);
              wave_sync();
            }
            if (!MC && c_l == 1) {
              c_v0 = cptr(c_tab)->v[0];
              c_rb0 = cptr(A.row_ptr)[c_v0];
              c_re0 = cptr(A.row_ptr)[c_v0 + 1];
              // v_0 is only ever stored to LDS: kept in a vector register
              // (the empty asm places it there) it costs no scalar register
              // across the loop and no move at each start
              c_v0v = c_v0;
              asm volatile("" : "+v"(c_v0v));
            }
          }
          const uint64_t lim = cend < cseg_end ? cend : cseg_end;
          const uint64_t room = lim - cur;
          const uint32_t want = (uint32_t)__popcll(idle);
          const uint32_t take = room < (uint64_t)want ? (uint32_t)room : want;
          const uint32_t rank = lane_prefix(idle);
          if (st == T_IDLE && rank < take) {
            f = cur + rank;
            st = T_START;
            started = true;
          }
          cur += take;
        }
      }
    }
    if constexpr (!P1) {
      if (__ballot(st != T_IDLE) == 0ull) {
        if (exhausted) break;
        continue;
      }
    }
    // (with first-level passes an idle wave skips the sampling step rather
    // than restarting the loop: one back-edge keeps the lanes' registers
    // from being copied between two)
    const bool busy = P1 ? __ballot(st != T_IDLE) != 0ull : true;
    if constexpr (P1) {
      if (!busy && exhausted && pw.head == pw.tail) break;
    }
    if (busy) {
    // (2) new samples copy their (common) segment's and query's fields.  Long
    // Stage-1 tables (and, in the backward, samples known to be large) go
    // straight to the small kernel.
    bool pass_on = false;
    if (started) {
      sg = cseg;
      stream = c_stream;
      s = c_first + (f - c_flat0);
      oidx = c_out + (f - c_flat0);
      qid = c_qid;
      ql = c_l;
      qk = c_k;
      s0 = c_s0;
      smask = c_smask;
      shash = c_shash;
      tab = c_tab;
      // a Monte-Carlo sample starts from its seed set, which this kernel
      // takes only when it is one node (its output is then the visited
      // count minus that seed)
      pass_on = MC ? c_k != 1 : ql > (int64_t)TINY_LMAX;
      if (BWD) {
        y = A.y_in[oidx];
        pass_on |= y > (uint32_t)CAP;
      }
      if (pass_on) {
        st = T_IDLE;
      } else if (MC) {
        // Sec. 2.3: the seed is active and is expanded first, as any node
        vis[0] = c_s0;
        cnt = 1;
        qh = 0;
        E = 0;
        st = T_POP;
      } else if (c_l == 1) {
        // Stage 1 with a single table entry (the selection of Alg. 1 picks it
        // whatever U is, and no entry follows): v_0 is activated and, with
        // its row bounds read once per segment, popped at once, so the
        // sample examines its first edge group in this very iteration.
        vis[0] = c_v0v;
        cnt = 1;
        qh = 1;
        E = (unsigned long long)(c_re0 - c_rb0);
        if (BWD) atomicAdd(&A.acc_tab[0], (unsigned long long)y);
        if (BWD && c_re0 > c_rb0) atomicAdd(&A.acc_node[c_v0], (unsigned long long)y);
        if (P1DIR && pmask) {
          // a pending sample whose pass drew v_0's coins: v_0's live
          // out-edges into nodes outside S (a non-empty set) are expanded
          // here, in slot order, as the edge-group steps would have done
          bool overflow = false;
          for (uint32_t mk = pmask; mk; mk &= mk - 1u) {
            const int32_t v = wp1tgt[__builtin_ctz(mk)];
            bool dup = false;
            for (uint32_t c = 0; c < cnt; ++c) dup |= vis[64 * c] == v;
            if (!dup) {
              if (cnt >= (uint32_t)CAP) {
                overflow = true;
              } else {
                vis[64 * cnt] = v;
                ++cnt;
              }
            }
          }
          pass_on = overflow;
          st = overflow ? T_IDLE : T_POP;
        } else if (c_re0 > c_rb0) {
          lo_e = (uint32_t)c_rb0;
          hi_e = (uint32_t)c_re0;
          g = (uint32_t)(c_rb0 >> 2);
          gend = (uint32_t)((c_re0 + 3) >> 2);
          st = T_EXPAND;
        } else {
          st = T_POP;
        }
      }
    }
    hand_over(pass_on, f, A.list1, A.nlist1, lane);
    pass_on = false;
    // (3) one round of independent loads: popping lanes fetch the next
    // node's row bounds (16 bytes), expanding lanes their group of four edges
    // (32 bytes) or table entries (48 bytes).  Every lane issues the same
    // three 16-byte loads from addresses chosen per state (lanes with
    // nothing to read point at row_ptr[0..1]), with no branch between them,
    // so the three kinds of load are in flight together instead of one after
    // another; the Philox block below overlaps their latency.
    const OI_GLOBAL char* la = (const OI_GLOBAL char*)gptr(A.row_ptr);
    const OI_GLOBAL char* lb = la;
    const OI_GLOBAL char* lc = la;
    if (st == T_POP && qh < cnt) {
      const int32_t u = vis[64 * qh];
      la = (const OI_GLOBAL char*)(gptr(A.row_ptr) + u);
    } else if (st == T_EXPAND) {
      la = (const OI_GLOBAL char*)(gptr(A.eg) + g);
      lb = la + 16;
    } else if (st == T_STAGE1) {
      la = (const OI_GLOBAL char*)(gptr(tab) + g);
      lb = la + 16;
      lc = la + 32;
    }
    const v4i32 ra = *(const OI_GLOBAL v4i32_a8*)la;
    const v4i32 rb = *(const OI_GLOBAL v4i32*)lb;
    const v4i32 rc = *(const OI_GLOBAL v4i32*)lc;
    Words d;
    d.w[0] = d.w[1] = d.w[2] = d.w[3] = 0;
    // the run seed (key word 1) stays a scalar: the empty asm makes it look
    // new each iteration, so its ten round keys are formed with scalar adds
    // here instead of being kept across the loop (where they would spill
    // to vector lanes and each cost a vector read per round)
    uint32_t seed = A.seed;
    asm volatile("" : "+s"(seed));
    if (st == T_START || st == T_STAGE1 || st == T_EXPAND) {
      const uint32_t kind = st == T_START ? KIND_SELECT : (st == T_STAGE1 ? KIND_STAGE1 : KIND_EDGE);
      d = philox_draw(qid, seed, kind, stream, s, st == T_START ? 0ull : (uint64_t)g);
    }
    // (4) consume
    const int32_t tv[4] = {ra.x, ra.y, ra.z, ra.w};
    const uint32_t tp[4] = {(uint32_t)rb.x, (uint32_t)rb.y, (uint32_t)rb.z, (uint32_t)rb.w};
    const uint64_t tt[4] = {(uint64_t)(uint32_t)rb.x | ((uint64_t)(uint32_t)rb.y << 32),
                            (uint64_t)(uint32_t)rb.z | ((uint64_t)(uint32_t)rb.w << 32),
                            (uint64_t)(uint32_t)rc.x | ((uint64_t)(uint32_t)rc.y << 32),
                            (uint64_t)(uint32_t)rc.z | ((uint64_t)(uint32_t)rc.w << 32)};
    const int64_t peb = (int64_t)((uint64_t)(uint32_t)ra.x | ((uint64_t)(uint32_t)ra.y << 32));
    const int64_t pee = (int64_t)((uint64_t)(uint32_t)ra.z | ((uint64_t)(uint32_t)ra.w << 32));
    if (st == T_POP) {
      // a lane that entered T_POP with its queue drained during this
      // iteration (a single-entry start whose node has no out-edges) read
      // nothing; the next iteration finishes it
      if (qh < cnt) {
        if (BWD && pee > peb) atomicAdd(&A.acc_node[vis[64 * qh]], (unsigned long long)y);
        ++qh;
        E += (unsigned long long)(pee - peb);
        if (pee > peb) {
          lo_e = (uint32_t)peb;
          hi_e = (uint32_t)pee;
          g = (uint32_t)(peb >> 2);
          gend = (uint32_t)((pee + 3) >> 2);
          st = T_EXPAND;
        }
      }
    } else if (st == T_START) {
      // Alg. 1, Stage 1: select and activate the first entry (a single entry is selected whatever U is)
      // (the lanes in this state started in this iteration, from the
      // segment whose CDF and nodes the wave holds in LDS; a one-entry table
      // never comes here)
      int64_t i = 0;
      if (ql > 1) {
        const uint64_t a = d.w[0] >> 5, b = d.w[1] >> 6;
        const double U = (double)(a * 67108864ull + b) * (1.0 / 9007199254740992.0);
        const double t = U * wcdf[ql];  // beta_0 = CDF_l (Eq. zerop)
        int64_t lo = 0, hi = ql;
        while (lo < hi) {
          const int64_t mid = lo + ((hi - lo) >> 1);
          if (wcdf[mid + 1] > t)
            hi = mid;
          else
            lo = mid + 1;
        }
        i = lo;
        if (lo >= ql) {
          i = -1;
          for (int64_t j = ql - 1; j >= 0; --j)
            if (wcdf[j + 1] > wcdf[j]) {
              i = j;
              break;
            }
          if (i < 0) {
            atomicOr(A.err, 1u);
            i = 0;
          }
        }
      }
      const int32_t vi = ql > 1 ? wtv[i] : tab_v(tab, i);
      vis[0] = vi;
      cnt = 1;
      qh = 0;
      E = (unsigned long long)(ql - 1 - i);
      if (BWD) atomicAdd(&A.acc_tab[i], (unsigned long long)y);
      if (i + 1 < ql) {
        lo_e = (uint32_t)(i + 1);
        hi_e = (uint32_t)ql;
        g = (uint32_t)((i + 1) >> 2);
        gend = (uint32_t)((ql + 3) >> 2);
        st = T_STAGE1;
      } else {
        st = T_POP;
      }
    } else if (st == T_STAGE1 || st == T_EXPAND) {
      // Alg. 1: Stage-1 coins of a table group, or Stage-2 coins of an edge group
      uint32_t live = 0;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const uint32_t x = 4 * g + b;
        if (x >= lo_e && x < hi_e) {
          if (st == T_STAGE1) {
            if ((uint64_t)d.w[b] < tt[b]) {
              live |= 1u << b;
              if (BWD) atomicAdd(&A.acc_tab[x], (unsigned long long)y);
            }
          } else {
            const bool lv = edge_live(d.w[b], tp[b]);
            if (lv) {
              bool ins = tv[b] == s0;
              if (BWD && A.sbits) {
                ins = seed_bit(A.sbits, tv[b]);
              } else if (qk != 1) {
                uint32_t h = mix32((uint32_t)tv[b]) & smask;
                while (true) {
                  const int32_t c = gptr(shash)[h];
                  if (c == tv[b]) {
                    ins = true;
                    break;
                  }
                  if (c < 0) {
                    ins = false;
                    break;
                  }
                  h = (h + 1) & smask;
                }
              }
              if (!ins) {
                if (BWD) atomicAdd(&A.acc_live[x], (unsigned long long)y);
                live |= 1u << b;
              }
            }
          }
        }
      }
      bool overflow = false;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        if ((live >> b) & 1u) {
          const int32_t v = tv[b];
          bool dup = false;
          for (uint32_t c = 0; c < cnt; ++c) dup |= vis[64 * c] == v;
          if (!dup) {
            if (cnt >= (uint32_t)CAP) {
              overflow = true;
            } else {
              vis[64 * cnt] = v;
              ++cnt;
            }
          }
        }
      }
      if (overflow) {
        if (BWD) atomicOr(A.err, 8u);  // y_in said the sample fits
        pass_on = !BWD;
        st = T_IDLE;
      } else if (++g >= gend) {
        st = T_POP;
      }
    }
    hand_over(pass_on, f, A.list1, A.nlist1, lane);
    }
  }
  wave_flush(acc_seg != 0xFFFFFFFFu, acc_seg, acc_y, acc_e, A.seg_sums, A.tier_sums, lane);
  if constexpr (P1) {
    if (pw.n && lane == 0) {
      atomicAdd(&A.seg_sums[2 * cseg], pw.n);
      atomicAdd(&A.seg_sums[2 * cseg + 1], pw.e);
      atomicAdd(&A.tier_sums[0], pw.n);
      atomicAdd(&A.tier_sums[1], pw.e);
    }
  }
}

// ---------------------------------------------------------------------------
// small_kernel
// ---------------------------------------------------------------------------
// Ring items (64 bits): a = node id (node item) or next Stage-1 entry index
// (Stage-1 item) in bits 0..31; group offset from the row's first group in
// bits 32..58 (node items); kind in bits 59..60; slot in bits 61..63.
constexpr uint32_t ITEM_NODE = 0;
constexpr uint32_t ITEM_STAGE1 = 1;

__device__ __forceinline__ uint64_t mk_item(uint32_t slot, uint32_t kind, uint32_t off, uint32_t a) {
  return ((uint64_t)slot << 61) | ((uint64_t)kind << 59) | ((uint64_t)off << 32) | (uint64_t)a;
}
__device__ __forceinline__ uint32_t item_slot(uint64_t it) { return (uint32_t)(it >> 61); }
__device__ __forceinline__ uint32_t item_kind(uint64_t it) { return (uint32_t)(it >> 59) & 3u; }
__device__ __forceinline__ uint32_t item_off(uint64_t it) { return (uint32_t)(it >> 32) & 0x07FFFFFFu; }
__device__ __forceinline__ uint32_t item_a(uint64_t it) { return (uint32_t)it; }

template <int K, int HCAP, int RCAP>
struct SmallLds {
  int32_t hash[K][HCAP];
  uint64_t ring[RCAP];
  uint64_t it_item[64];
  int64_t it_eb[64];
  int64_t it_ee[64];
  uint32_t it_g0[64];
  uint32_t it_scan[64];
  uint64_t s_f[K];
  uint64_t s_s[K];
  unsigned long long s_E[K];
  uint32_t s_q[K];
  uint32_t s_seg[K];
  uint32_t s_stream[K];
  uint32_t s_cnt[K];
  uint32_t s_pend[K];
  uint32_t s_new[K];
  uint32_t s_active[K];
  uint32_t s_y[K];
  int32_t s_vi[K];
  uint32_t s_i[K];
  uint32_t s_mc[K];  // 1: a classic Monte-Carlo sample (its seed is counted in s_cnt)
  // the slot's query, copied when the sample starts
  uint32_t s_full;  // slots whose LDS set overflowed (backward consistency check)
  const TabGroup* s_tab[K];
  const int32_t* s_shash[K];
  int64_t s_l[K];
  uint32_t s_qid[K];
  uint32_t s_smask[K];
  int32_t s_k[K];
  int32_t s_s0[K];
  uint32_t head, tail;
};

template <int HCAP>
__device__ __forceinline__ uint32_t hslot(int32_t v) {
  constexpr int LOG = __builtin_ctz(HCAP);
  return ((uint32_t)v * 0x9E3779B1u) >> (32 - LOG);
}

// Open addressing with linear probing; every probe loop is bounded by the
// table size, so a full table can never make a lane spin.
template <int HCAP>
__device__ __forceinline__ bool hash_contains(const int32_t* h, int32_t v) {
  uint32_t p = hslot<HCAP>(v);
  for (int n = 0; n < HCAP; ++n) {
    const int32_t c = h[p];
    if (c == v) return true;
    if (c < 0) return false;
    p = (p + 1) & (HCAP - 1);
  }
  return false;
}

// 1: inserted, 0: already present, -1: table full
template <int HCAP>
__device__ __forceinline__ int hash_insert(int32_t* h, int32_t v) {
  uint32_t p = hslot<HCAP>(v);
  for (int n = 0; n < HCAP; ++n) {
    int32_t c = h[p];
    if (c == v) return 0;
    if (c < 0) {
      c = atomicCAS(&h[p], -1, v);
      if (c < 0) return 1;
      if (c == v) return 0;
    }
    p = (p + 1) & (HCAP - 1);
  }
  return -1;
}

// Remove, in order, the ring items of the slots in `mask` (stable compaction
// of [head, tail)).  Must be reached by the whole wave.
template <int RCAP>
__device__ void drop_ring_items(uint64_t* ring, uint32_t* head, uint32_t* tail, uint32_t mask, int lane) {
  const uint32_t h0 = uniform(*head), n0 = uniform(*tail) - h0;
  uint32_t w = h0;
  for (uint32_t i0 = 0; i0 < n0; i0 += 64) {
    const uint32_t i = i0 + lane;
    const bool valid = i < n0;
    const uint64_t it = valid ? ring[(h0 + i) & (RCAP - 1)] : 0ull;
    const bool keep = valid && !((mask >> item_slot(it)) & 1u);
    const unsigned long long bal = __ballot(keep);
    wave_sync();
    if (keep) ring[(w + lane_prefix(bal)) & (RCAP - 1)] = it;
    w += (uint32_t)__popcll(bal);
    wave_sync();
  }
  if (lane == 0) *tail = w;
}

template <int K, int HCAP, int RCAP, int R, bool BWD>
__global__ void __launch_bounds__(256) small_kernel(SampleLaunch A) {
  constexpr int WPB = 4;
  constexpr uint32_t CMAX = RCAP / K - 1;  // visited nodes one slot may hold
  static_assert(2 * CMAX <= HCAP, "LDS hash load factor must stay <= 1/2");
  static_assert(K <= 8, "slot field is 3 bits");
  constexpr uint32_t B = 64u * R;          // edge groups per pass
  __shared__ SmallLds<K, HCAP, RCAP> lds_all[WPB];
  SmallLds<K, HCAP, RCAP>& W = lds_all[threadIdx.x >> 6];
  const int lane = threadIdx.x & 63;

  if (lane < K) {
    W.s_active[lane] = 0;
    W.s_new[lane] = 0;
  }
  if (lane == 0) {
    W.head = 0;
    W.tail = 0;
    W.s_full = 0;
  }
  wave_sync();

  uint64_t cur = 0, cend = 0;
  bool exhausted = false;
  uint32_t acc_seg = 0xFFFFFFFFu;
  unsigned long long acc_y = 0, acc_e = 0;
  const bool from_list = A.small_from_list1 != 0;
  const uint64_t total = from_list ? (uint64_t)*A.nlist1 : A.total;
  unsigned long long* const counter = from_list ? A.counter1 : A.counter;
  if (from_list && total <= A.small_direct_max) {
    // Few samples were handed over: one block per sample in the large
    // kernel finishes them sooner than a wave working through its slots, so
    // block 0 forwards the list unchanged and every block leaves.
    __shared__ unsigned int s_base;
    if (blockIdx.x == 0) {
      if (threadIdx.x == 0 && total) s_base = atomicAdd(A.nlist2, (unsigned int)total);
      __syncthreads();
      for (uint32_t t = threadIdx.x; t < (uint32_t)total; t += blockDim.x) A.list2[s_base + t] = A.list1[t];
    }
    return;
  }

  while (true) {
    // ---- refill free slots from the work counter ----------------------
    uint32_t newmask = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (uniform(W.s_active[k]) == 0u) {
        if (cur >= cend && !exhausted) {
          unsigned long long c = 0;
          if (lane == 0) c = atomicAdd(counter, (unsigned long long)A.chunk);
          c = uniform64(__shfl(c, 0, 64));
          if (c >= total) {
            exhausted = true;
          } else {
            cur = c;
            cend = c + A.chunk < total ? c + A.chunk : total;
          }
        }
        if (cur < cend) {
          if (lane == 0) W.s_f[k] = from_list ? A.list1[cur] : cur;
          ++cur;
          newmask |= 1u << k;
        }
      }
    }
    wave_sync();
    if (newmask) {
      // lanes 0..K-1 start their slot's sample: the Stage-1 selection of Alg. 1
      if (lane < K && ((newmask >> lane) & 1u)) {
        const uint64_t f = W.s_f[lane];
        const uint32_t sg = find_segment(A, f);
        const Segment S = A.segs[sg];
        const QueryDev& Q = A.qs[S.q];
        const uint64_t s = S.first + (f - S.flat0);
        uint32_t y = 0;
        bool start = true;
        const bool mc = Q.mc != 0;
        if (BWD) {
          y = A.y_in[S.out_off + (f - S.flat0)];
          // known too large for LDS, or a table sampled by skip sampling
          // (the large kernel's): straight to the large kernel
          if (y > CMAX || Q.skip) {
            const unsigned int pos = atomicAdd(A.nlist2, 1u);
            A.list2[pos] = f;
            start = false;
          }
        } else if (Q.lt || (mc ? Q.k != 1 : Q.skip != 0)) {
          // an LT cascade, a Monte-Carlo sample from several seeds (the large
          // kernel queues the whole seed set), or a long table's skip-sampled
          // Stage 1
          const unsigned int pos = atomicAdd(A.nlist2, 1u);
          A.list2[pos] = f;
          start = false;
        }
        if (start) {
          int64_t i = 0;
          int32_t vi = Q.s0;  // a Monte-Carlo sample starts by expanding its seed (Sec. 2.3)
          if (!mc) {
            i = select_entry(Q, A.seed, S.stream, s);
            if (i < 0) {
              atomicOr(A.err, 1u);
              i = 0;
            }
            vi = tab_v(Q.tab, i);
          }
          W.s_tab[lane] = Q.tab;
          W.s_shash[lane] = Q.shash;
          W.s_l[lane] = Q.l;
          W.s_qid[lane] = Q.qid;
          W.s_smask[lane] = Q.smask;
          W.s_k[lane] = Q.k;
          W.s_s0[lane] = Q.s0;
          W.s_s[lane] = s;
          W.s_q[lane] = S.q;
          W.s_seg[lane] = sg;
          W.s_stream[lane] = S.stream;
          W.s_E[lane] = mc ? 0ull : (unsigned long long)(Q.l - 1 - i);
          W.s_cnt[lane] = 1;
          W.s_pend[lane] = (!mc && i + 1 < Q.l) ? 2u : 1u;
          W.s_new[lane] = 0;
          W.s_y[lane] = y;
          W.s_vi[lane] = vi;
          W.s_i[lane] = (uint32_t)i;
          W.s_mc[lane] = mc ? 1u : 0u;
          W.s_active[lane] = 1;
          if (BWD) atomicAdd(&A.acc_tab[i], (unsigned long long)y);
        } else {
          W.s_active[lane] = 0;
        }
      }
      wave_sync();
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if ((newmask >> k) & 1u) {
          for (int h = lane; h < HCAP; h += 64) W.hash[k][h] = -1;
        }
      }
      wave_sync();
      if (lane < K && ((newmask >> lane) & 1u) && W.s_active[lane]) {
        const int32_t vi = W.s_vi[lane];
        W.hash[lane][hslot<HCAP>(vi)] = vi;
        const uint32_t i = W.s_i[lane];
        const bool more = !W.s_mc[lane] && (int64_t)i + 1 < W.s_l[lane];
        const uint32_t pos = atomicAdd(&W.tail, more ? 2u : 1u);
        W.ring[pos & (RCAP - 1)] = mk_item(lane, ITEM_NODE, 0, (uint32_t)vi);
        if (more) W.ring[(pos + 1) & (RCAP - 1)] = mk_item(lane, ITEM_STAGE1, 0, i + 1);
      }
      wave_sync();
    }
    uint32_t anyactive = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) anyactive |= uniform(W.s_active[k]);
    if (!anyactive) {
      if (exhausted) break;
      continue;
    }

    // ---- gather up to 64 items and cut them to B edge groups -------------
    const uint32_t head = uniform(W.head), tail = uniform(W.tail);
    const uint32_t avail = tail - head;
    const uint32_t nit = avail < 64u ? avail : 64u;
    if (nit == 0) {  // active slots always have queued items; never spin if not
      if (lane == 0) atomicOr(A.err, 4u);
      if (lane < K) W.s_active[lane] = 0;
      wave_sync();
      continue;
    }
    uint64_t item = 0;
    uint32_t ntask = 0, kind = 0, slot = 0, off = 0, a = 0, g0 = 0;
    int64_t eb = 0, ee = 0;
    if ((uint32_t)lane < nit) {
      item = W.ring[(head + lane) & (RCAP - 1)];
      kind = item_kind(item);
      slot = item_slot(item);
      off = item_off(item);
      a = item_a(item);
      if (kind == ITEM_NODE) {
        eb = A.row_ptr[a];
        ee = A.row_ptr[a + 1];
        if (ee > eb) {
          g0 = (uint32_t)(eb >> 2) + off;
          ntask = (uint32_t)((ee + 3) >> 2) - g0;
        }
      } else {
        const int64_t l = W.s_l[slot];
        eb = a;
        ee = l;
        g0 = a >> 2;
        ntask = (uint32_t)((l + 3) >> 2) - g0;
      }
    }
    const uint32_t sc = wave_incl_scan(ntask, lane);
    const uint32_t total = uniform(__shfl(sc, nit ? (int)nit - 1 : 0, 64));
    uint32_t take = ntask;
    bool consumed = (uint32_t)lane < nit;
    uint32_t cut = nit;
    if (total > B) {
      const unsigned long long m = __ballot((uint32_t)lane < nit && sc > B);
      cut = (uint32_t)__ffsll((long long)m) - 1u;
      if ((uint32_t)lane == cut) {
        take = B - (sc - ntask);
        consumed = false;
      } else if ((uint32_t)lane > cut) {
        take = 0;
        consumed = false;
      }
    }
    if ((uint32_t)lane < nit) {
      if (kind == ITEM_NODE && off == 0 && (consumed || take > 0)) {
        atomicAdd(&W.s_E[slot], (unsigned long long)(ee - eb));
        if (BWD && ee > eb) atomicAdd(&A.acc_node[a], (unsigned long long)W.s_y[slot]);
      }
      if (consumed) atomicSub(&W.s_pend[slot], 1u);
      if ((uint32_t)lane == cut) {
        // the remainder starts at the first group not taken; a Stage-1 item
        // keeps its exact first entry while none of its groups was taken
        const uint64_t rem = kind == ITEM_NODE ? mk_item(slot, ITEM_NODE, off + take, a)
                                               : mk_item(slot, ITEM_STAGE1, 0, take ? (g0 + take) * 4u : a);
        W.ring[(head + cut) & (RCAP - 1)] = rem;
      }
    }
    W.it_item[lane] = item;
    W.it_eb[lane] = eb;
    W.it_ee[lane] = ee;
    W.it_g0[lane] = g0;
    W.it_scan[lane] = sc < B ? sc : B;
    if (lane == 0) W.head = head + cut;
    wave_sync();
    const uint32_t ntot = total < B ? total : B;

    // ---- phase A: coins for every task, count new live targets -----------
    uint32_t mask[R];
    int32_t tv[R][4];
    uint32_t tslot[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      mask[r] = 0;
      tslot[r] = 0;
      const uint32_t t = (uint32_t)(r * 64 + lane);
      if (t < ntot) {
        int lo = 0, hi = (int)nit - 1;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (W.it_scan[mid] > t)
            hi = mid;
          else
            lo = mid + 1;
        }
        const uint64_t it = W.it_item[lo];
        const uint32_t sl = item_slot(it);
        const uint32_t kd = item_kind(it);
        const uint32_t base = lo ? W.it_scan[lo - 1] : 0u;
        const uint32_t g = W.it_g0[lo] + (t - base);
        const int64_t lo_e = W.it_eb[lo], hi_e = W.it_ee[lo];
        const uint32_t qid = W.s_qid[sl];
        const int32_t qk = W.s_k[sl], qs0 = W.s_s0[sl];
        const uint32_t qmask = W.s_smask[sl];
        const int32_t* qhash = W.s_shash[sl];
        const uint64_t s = W.s_s[sl];
        const uint32_t stream = W.s_stream[sl];
        const int32_t* hs = W.hash[sl];
        tslot[r] = sl;
        uint32_t mk = 0;
        if (kd == ITEM_NODE) {
          const Words d = philox_draw(qid, A.seed, KIND_EDGE, stream, s, g);
          const int4 vv = *reinterpret_cast<const int4*>(&A.eg[g].v[0]);
          const uint4 pp = *reinterpret_cast<const uint4*>(&A.eg[g].thr[0]);
          const int32_t va[4] = {vv.x, vv.y, vv.z, vv.w};
          const uint32_t pa[4] = {pp.x, pp.y, pp.z, pp.w};
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const int64_t e = 4 * (int64_t)g + b;
            tv[r][b] = va[b];
            if (e >= lo_e && e < hi_e) {
              const bool live = edge_live(d.w[b], pa[b]);
              if (BWD) {
                if (live && !(A.sbits ? seed_bit(A.sbits, va[b]) : in_seed_fields(qk, qs0, qmask, qhash, va[b]))) {
                  atomicAdd(&A.acc_live[e], (unsigned long long)W.s_y[sl]);
                  if (!hash_contains<HCAP>(hs, va[b])) mk |= 1u << b;
                }
              } else if (live && !in_seed_fields(qk, qs0, qmask, qhash, va[b]) &&
                         !hash_contains<HCAP>(hs, va[b])) {
                mk |= 1u << b;
              }
            }
          }
        } else {
          const Words d = philox_draw(qid, A.seed, KIND_STAGE1, stream, s, g);
          const TabGroup T = load_tab(W.s_tab[sl], g);
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const int64_t j = 4 * (int64_t)g + b;
            tv[r][b] = T.v[b];
            if (j >= lo_e && j < hi_e && (uint64_t)d.w[b] < T.thr[b]) {
              if (BWD) atomicAdd(&A.acc_tab[j], (unsigned long long)W.s_y[sl]);
              if (!hash_contains<HCAP>(hs, T.v[b])) mk |= 1u << b;
            }
          }
        }
        mask[r] = mk;
        if (mk) atomicAdd(&W.s_new[sl], (uint32_t)__popc(mk));
      }
    }
    wave_sync();

    // ---- hand over samples that would outgrow the LDS set ----------------
    // (forward only: in the backward every started sample is known to fit)
    uint32_t defmask = 0;
    if (!BWD) {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (uniform(W.s_active[k]) && uniform(W.s_cnt[k]) + uniform(W.s_new[k]) > CMAX) defmask |= 1u << k;
      }
      if (defmask) {
        if (lane == 0) {
          for (int k = 0; k < K; ++k) {
            if ((defmask >> k) & 1u) {
              const unsigned int pos = atomicAdd(A.nlist2, 1u);
              A.list2[pos] = W.s_f[k];
              W.s_active[k] = 0;
            }
          }
        }
        drop_ring_items<RCAP>(W.ring, &W.head, &W.tail, defmask, lane);
      }
    }
    if (lane < K) W.s_new[lane] = 0;
    wave_sync();

    // ---- phase B: insert new targets and queue them ----------------------
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (mask[r] && !((defmask >> tslot[r]) & 1u)) {
        const uint32_t sl = tslot[r];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          if ((mask[r] >> b) & 1u) {
            const int32_t v = tv[r][b];
            const int ins = hash_insert<HCAP>(W.hash[sl], v);
            if (ins > 0) {
              atomicAdd(&W.s_cnt[sl], 1u);
              atomicAdd(&W.s_pend[sl], 1u);
              const uint32_t pos = atomicAdd(&W.tail, 1u);
              W.ring[pos & (RCAP - 1)] = mk_item(sl, ITEM_NODE, 0, (uint32_t)v);
            } else if (ins < 0) {
              atomicOr(&W.s_full, 1u << sl);
            }
          }
        }
      }
    }
    wave_sync();

    // ---- a full set can only mean that y_in disagrees with the recomputed
    // sample (backward): flag it and drop the sample
    {
      const uint32_t full = uniform(W.s_full);
      if (full) {
        if (lane == 0) {
          atomicOr(A.err, 8u);
          for (int k = 0; k < K; ++k)
            if ((full >> k) & 1u) W.s_active[k] = 0;
          W.s_full = 0;
        }
        drop_ring_items<RCAP>(W.ring, &W.head, &W.tail, full, lane);
        wave_sync();
      }
    }

    // ---- finished samples --------------------------------------------------
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (uniform(W.s_active[k]) && uniform(W.s_pend[k]) == 0u) {
        const uint32_t cnt = uniform(W.s_cnt[k]) - uniform(W.s_mc[k]);
        const uint64_t E = uniform64(W.s_E[k]);
        const uint32_t sg = uniform(W.s_seg[k]);
        if (lane == 0) {
          const Segment& S = A.segs[sg];
          const uint64_t idx = S.out_off + (W.s_f[k] - S.flat0);
          if (BWD) {
            if (cnt != W.s_y[k]) atomicOr(A.err, 2u);
          } else {
            if (A.y_out) A.y_out[idx] = cnt;
            if (A.e_out) A.e_out[idx] = E;
          }
          W.s_active[k] = 0;
        }
        if (sg != acc_seg) {
          if (lane == 0 && acc_seg != 0xFFFFFFFFu) {
            atomicAdd(&A.seg_sums[2 * acc_seg], acc_y);
            atomicAdd(&A.seg_sums[2 * acc_seg + 1], acc_e);
            atomicAdd(&A.tier_sums[2], acc_y);
            atomicAdd(&A.tier_sums[3], acc_e);
          }
          acc_seg = sg;
          acc_y = 0;
          acc_e = 0;
        }
        acc_y += cnt;
        acc_e += E;
      }
    }
    wave_sync();
  }
  if (lane == 0 && acc_seg != 0xFFFFFFFFu) {
    atomicAdd(&A.seg_sums[2 * acc_seg], acc_y);
    atomicAdd(&A.seg_sums[2 * acc_seg + 1], acc_e);
    atomicAdd(&A.tier_sums[2], acc_y);
    atomicAdd(&A.tier_sums[3], acc_e);
  }
}

// ---------------------------------------------------------------------------
// large_kernel: one block per handed-over sample, global bitmap + queue
// ---------------------------------------------------------------------------
// A block of LB threads runs one sample at a time, taking samples from a
// work counter; as many blocks run as fit on the GPU (within the workspace
// budget), so many samples are in flight at once.  The visited set is a bitmap of n bits and the queue an array
// of n node ids, both owned by the block; the seed set is marked in the
// bitmap while the sample runs, so an edge into S is never pushed.  Stage 2
// expands the queue in batches of up to LB * LBN nodes: each thread reads
// LBN nodes' row bounds, a block scan lays the batch's edge groups out in one
// index space, and thread t takes groups t, t + LB, ... of it.  After the
// sample the bits it set (the queue and S) are cleared again, or the whole
// bitmap when the sample was dense.
constexpr int LB = 256;        // threads of a main-pool block
constexpr int LB_FULL = 1024;  // threads of a block of the full-queue pass (few, very large samples)
constexpr int LBN = 4;         // queued nodes per thread per expansion batch

template <int NT>
__device__ __forceinline__ uint32_t block_incl_scan(uint32_t x, uint32_t* wtot, int tid, uint32_t* total) {
  const int lane = tid & 63, wid = tid >> 6;
  x = wave_incl_scan(x, lane);
  if (lane == 63) wtot[wid] = x;
  __syncthreads();
  uint32_t add = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) {
    const uint32_t v = wtot[w];
    if (w < wid) add += v;
    tot += v;
  }
  *total = tot;
  __syncthreads();
  return x + add;
}

// Sets (set = true) or clears the bits of the seed set in a block's bitmap.
template <int NT>
__device__ __forceinline__ void mark_seed_set(const QueryDev& Q, uint32_t* bits, bool set, int tid) {
  if (Q.k == 1) {
    if (tid == 0) {
      if (set)
        atomicOr(&bits[Q.s0 >> 5], 1u << (Q.s0 & 31));
      else
        atomicAnd(&bits[Q.s0 >> 5], ~(1u << (Q.s0 & 31)));
    }
    return;
  }
  for (uint32_t h = tid; h <= Q.smask; h += NT) {
    const int32_t v = gptr(Q.shash)[h];
    if (v >= 0) {
      if (set)
        atomicOr(&bits[v >> 5], 1u << (v & 31));
      else
        atomicAnd(&bits[v >> 5], ~(1u << (v & 31)));
    }
  }
}

// Marks v visited; true if this call was the first to do so.
__device__ __forceinline__ bool claim(uint32_t* bits, int32_t v) {
  const uint32_t bit = 1u << (v & 31);
  return !(atomicOr(&bits[v >> 5], bit) & bit);
}

// Appends v to a block's queue of capacity qcap.  The tail keeps counting
// past the capacity, which is how the block notices that the sample has
// outgrown its queue.
__device__ __forceinline__ void push(int32_t* queue, uint32_t* tail, uint32_t qcap, int32_t v) {
  const uint32_t pos = atomicAdd(tail, 1u);
  if (pos < qcap) queue[pos] = v;
}

// LT: the launch's samples are LT-model cascades (forward only).  The kernel
// waits on memory most of the time, so it is held to 64 vector registers
// (eight waves per SIMD, a few values spilled) rather than the 69 that would
// leave room for seven.
template <bool BWD, int NT, bool LT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(8))) large_kernel(SampleLaunch A) {
  __shared__ uint32_t s_tail;
  __shared__ unsigned long long s_E;
  __shared__ uint32_t wtot[NT / 64];
  __shared__ uint32_t it_scan[NT * LBN];
  __shared__ uint32_t it_eb[NT * LBN];
  __shared__ uint32_t it_ee[NT * LBN];
  __shared__ int64_t s_i;
  __shared__ uint32_t s_di;
  __shared__ uint32_t s_go;
  const int tid = threadIdx.x;
  uint32_t* bits = A.bits + (int64_t)blockIdx.x * A.bits_words;
  int32_t* queue = A.queue + (int64_t)blockIdx.x * A.queue_stride;
  const uint32_t nd = *A.nlist2;
  // a block past the list's length could never take a sample: it leaves
  // without touching the shared counter (most launches have few or none)
  if (blockIdx.x >= nd) return;
  while (true) {
    if (tid == 0) s_di = (uint32_t)atomicAdd(A.counter2, 1ull);
    __syncthreads();
    const uint32_t di = s_di;
    if (di >= nd) break;
    const uint64_t f = A.list2[di];
    const uint32_t sg = find_segment(A, f);
    const Segment S = A.segs[sg];
    const QueryDev& Q = A.qs[S.q];
    const uint64_t s = S.first + (f - S.flat0);
    const uint64_t oidx = S.out_off + (f - S.flat0);
    const unsigned long long y = BWD ? A.y_in[oidx] : 0ull;
    if (BWD && y > A.qcap) {
      // known too large for this pass's queues (the backward must not start
      // a sample it cannot finish: its accumulations cannot be undone)
      if (tid == 0) {
        if (A.list3)
          A.list3[atomicAdd(A.nlist3, 1u)] = f;
        else
          atomicOr(A.err, 16u);
      }
      __syncthreads();
      continue;
    }
    mark_seed_set<NT>(Q, bits, true, tid);
    __syncthreads();
    const bool mc = !BWD && Q.mc != 0;
    if (tid == 0) {
      if (mc) {
        // Sec. 2.3: a Monte-Carlo cascade starts with all of S active (its
        // bits are set above); a single seed is queued here
        s_tail = 0;
        if (Q.k == 1) {
          queue[0] = Q.s0;
          s_tail = 1;
        }
        s_E = 0;
        s_i = Q.l;
      } else {
        int64_t i = select_entry(Q, A.seed, S.stream, s);
        if (i < 0) {
          atomicOr(A.err, 1u);
          i = 0;
        }
        const int32_t vi = tab_v(Q.tab, i);
        queue[0] = vi;
        atomicOr(&bits[vi >> 5], 1u << (vi & 31));
        s_tail = 1;
        s_E = (unsigned long long)(Q.l - 1 - i);
        s_i = i;
        if (BWD) atomicAdd(&A.acc_tab[i], y);
      }
    }
    __syncthreads();
    if (mc && Q.k != 1) {
      // several seeds: every one goes into the queue (from the seed-set table)
      for (uint32_t h = tid; h <= Q.smask; h += NT) {
        const int32_t v = gptr(Q.shash)[h];
        if (v >= 0) push(queue, &s_tail, A.qcap, v);
      }
      __syncthreads();
    }
    const int64_t i = s_i;
    const bool skip = !mc && Q.skip != 0;
    if (skip) {
      // Alg. 1, Stage 1 by skip sampling (long tables).  Heavy entries
      // (P >= 1/2) after i: their own coins, one thread each
      const OI_GLOBAL int32_t* hv = gptr(Q.heavy);
      int64_t lo = 0, hi = Q.nheavy;  // first heavy entry after i
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)hv[mid] > i)
          hi = mid;
        else
          lo = mid + 1;
      }
      for (int64_t h = lo + tid; h < Q.nheavy; h += NT) {
        const int64_t j = hv[h];
        const Words d = philox_draw(Q.qid, A.seed, KIND_STAGE1, S.stream, s, (uint64_t)(j >> 2));
        if ((uint64_t)word_at(d, j & 3) < tab_thr(Q.tab, j)) {
          if (BWD) atomicAdd(&A.acc_tab[j], y);
          const int32_t v = tab_v(Q.tab, j);
          if (claim(bits, v)) push(queue, &s_tail, A.qcap, v);
        }
      }
      // light entries: one walk per segment reaching past i, one thread each.
      // Standing at pos, the next live entry is the first j > pos of the
      // segment with R_j < U' R_pos (U' = 1 - U, U a 53-bit uniform).
      const OI_GLOBAL double* R = gptr(Q.skipR);
      for (int64_t m = (i + 1) / kSkipSeg + tid; m * kSkipSeg < Q.l; m += NT) {
        const int64_t a = m * kSkipSeg, b = a + kSkipSeg < Q.l ? a + kSkipSeg : Q.l;
        int64_t pos = i >= a ? i : a - 1;
        double Rpos = pos >= a ? R[pos] : 1.0;
        uint64_t idx = pos >= a ? (uint64_t)pos : (1ull << 40) + (uint64_t)m;
        while (true) {
          const Words d = philox_draw(Q.qid, A.seed, KIND_SKIP, S.stream, s, idx);
          const uint64_t ua = d.w[0] >> 5, ub = d.w[1] >> 6;
          const double U = (double)(ua * 67108864ull + ub) * (1.0 / 9007199254740992.0);
          const double thr = (1.0 - U) * Rpos;
          int64_t jl = pos + 1, jh = b;  // first j in (pos, b) with R_j < thr
          while (jl < jh) {
            const int64_t mid = (jl + jh) >> 1;
            if (R[mid] < thr)
              jh = mid;
            else
              jl = mid + 1;
          }
          if (jl >= b) break;
          if (BWD) atomicAdd(&A.acc_tab[jl], y);
          const int32_t v = tab_v(Q.tab, jl);
          if (claim(bits, v)) push(queue, &s_tail, A.qcap, v);
          pos = jl;
          Rpos = R[jl];
          idx = (uint64_t)jl;
        }
      }
    }
    // Alg. 1, Stage 1: one coin for each later table entry (none for a
    // Monte-Carlo sample or a skip-sampled table)
    const int64_t gend = (mc || skip) ? 0 : (Q.l + 3) >> 2;
    for (int64_t g = ((i + 1) >> 2) + tid; g < gend; g += NT) {
      const Words d = philox_draw(Q.qid, A.seed, KIND_STAGE1, S.stream, s, (uint64_t)g);
      const TabGroup T = load_tab(Q.tab, g);
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int64_t j = 4 * g + b;
        if (j > i && j < Q.l && (uint64_t)d.w[b] < T.thr[b]) {
          if (BWD) atomicAdd(&A.acc_tab[j], y);
          if (claim(bits, T.v[b])) push(queue, &s_tail, A.qcap, T.v[b]);
        }
      }
    }
    __syncthreads();
    // Alg. 1, Stage 2: expand the queue in batches of up to NT * LBN
    // nodes, LBN consecutive queue entries per thread (their row reads are
    // independent, so they are in flight together)
    uint32_t head = 0;
    // the soft cap (block-uniform): a forward sample that grows past it
    // leaves for the full-queue pass while this launch's budget of such
    // departures lasts, and otherwise goes on up to the queue's size
    uint32_t cap = BWD ? A.qcap : A.soft_cap;
    bool leave = false;
    while (true) {
      const uint32_t tail = s_tail;
      __syncthreads();
      if (!BWD && tail > cap && cap < A.qcap) {
        if (tid == 0) s_go = atomicAdd(A.nsoft, 1u) < A.soft_budget ? 1u : 0u;
        __syncthreads();
        if (s_go) {
          leave = true;
          break;
        }
        cap = A.qcap;
      }
      if (head >= tail || tail > A.qcap) break;
      const uint32_t nb = tail - head < (uint32_t)(NT * LBN) ? tail - head : (uint32_t)(NT * LBN);
      uint32_t rb[LBN], re[LBN], part[LBN];
      uint32_t mine = 0;
      unsigned long long eloc = 0;
#pragma unroll
      for (int k = 0; k < LBN; ++k) {
        const uint32_t j = (uint32_t)(LBN * tid + k);
        rb[k] = re[k] = 0;
        if (j < nb) {
          const int32_t u = queue[head + j];
          rb[k] = (uint32_t)A.row_ptr[u];
          re[k] = (uint32_t)A.row_ptr[u + 1];
          if (BWD && re[k] > rb[k]) atomicAdd(&A.acc_node[u], y);
        }
      }
#pragma unroll
      for (int k = 0; k < LBN; ++k) {
        eloc += re[k] - rb[k];
        mine += re[k] > rb[k] ? ((re[k] + 3) >> 2) - (rb[k] >> 2) : 0u;
        part[k] = mine;  // inclusive over this thread's entries
      }
      if (eloc) atomicAdd(&s_E, eloc);
      uint32_t total;
      const uint32_t base = block_incl_scan<NT>(mine, wtot, tid, &total) - mine;
#pragma unroll
      for (int k = 0; k < LBN; ++k) {
        const uint32_t j = (uint32_t)(LBN * tid + k);
        it_scan[j] = base + part[k];
        it_eb[j] = rb[k];
        it_ee[j] = re[k];
      }
      __syncthreads();
      // two groups per thread per step, so that their loads and coin
      // blocks are in flight together
      for (uint32_t t0 = tid; t0 < total; t0 += 2 * NT) {
        uint32_t gg[2], lo_e[2], hi_e[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const uint32_t t = t0 + (uint32_t)u * NT;
          gg[u] = 0;
          lo_e[u] = hi_e[u] = 0;  // no edge of group 0 is in [0, 0)
          if (t < total) {
            int lo = 0, hi = (int)nb - 1;  // first entry whose groups end after t
            while (lo < hi) {
              const int mid = (lo + hi) >> 1;
              if (it_scan[mid] > t)
                hi = mid;
              else
                lo = mid + 1;
            }
            const uint32_t before = lo ? it_scan[lo - 1] : 0u;
            lo_e[u] = it_eb[lo];
            hi_e[u] = it_ee[lo];
            gg[u] = (lo_e[u] >> 2) + (t - before);
          }
        }
        Words d[2];
        v4i32 va[2], pa[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const OI_GLOBAL char* q = (const OI_GLOBAL char*)(gptr(A.eg) + gg[u]);
          va[u] = *(const OI_GLOBAL v4i32*)q;
          pa[u] = *(const OI_GLOBAL v4i32*)(q + 16);
        }
        if (!LT) {
#pragma unroll
          for (int u = 0; u < 2; ++u) d[u] = philox_draw(Q.qid, A.seed, KIND_EDGE, S.stream, s, gg[u]);
        }
        if constexpr (!LT) {
          // the claims of the two groups' live edges are issued together (the
          // atomics are in flight at once rather than one round trip each),
          // then the thread's new nodes take one queue reservation
          // the live edges' targets (-1: none), selected outside any branch
          // so that the groups' loads are waited for once, before the claims
          int32_t tg[8];
#pragma unroll
          for (int u = 0; u < 2; ++u) {
#pragma unroll
            for (int b = 0; b < 4; ++b) {
              const uint32_t e = 4 * gg[u] + b;
              bool live = e >= lo_e[u] && e < hi_e[u] && edge_live(d[u].w[b], (uint32_t)pa[u][b]);
              // the backward: an edge into S is never revealed (its target is
              // not outside S), and a revealed one adds Y to its live sum
              if (BWD && live) live = !(A.sbits ? seed_bit(A.sbits, va[u][b]) : in_seed_set(Q, va[u][b]));
              tg[4 * u + b] = live ? va[u][b] : -1;
            }
          }
          if constexpr (BWD) {
#pragma unroll
            for (int k = 0; k < 8; ++k)
              if (tg[k] >= 0) atomicAdd(&A.acc_live[4 * gg[k >> 2] + (k & 3)], y);
          }
          // all eight targets are ready before the first claim (the empty asm
          // takes them), so that no wait for the second group's loads falls
          // between claims; the no-claim value is opaque, so that no test of
          // a claim's result is folded into its branch (which would wait on
          // that claim at once).  S is marked in the bitmap, so a live edge
          // into S claims nothing
          asm volatile("" ::"v"(tg[0]), "v"(tg[1]), "v"(tg[2]), "v"(tg[3]), "v"(tg[4]), "v"(tg[5]), "v"(tg[6]),
                       "v"(tg[7]));
          uint32_t none = 0xFFFFFFFFu;
          asm volatile("" : "+v"(none));
          uint32_t old[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            old[k] = none;
            if (tg[k] >= 0) old[k] = atomicOr(&bits[tg[k] >> 5], 1u << (tg[k] & 31));
          }
          uint32_t won = 0;
#pragma unroll
          for (int k = 0; k < 8; ++k)
            if (tg[k] >= 0 && !((old[k] >> (tg[k] & 31)) & 1u)) won |= 1u << k;
          if (won) {
            // the tail keeps counting past the capacity, as in push
            uint32_t pos = atomicAdd(&s_tail, (uint32_t)__popc(won));
#pragma unroll
            for (int k = 0; k < 8; ++k) {
              if ((won >> k) & 1u) {
                if (pos < A.qcap) queue[pos] = tg[k];
                ++pos;
              }
            }
          }
        }
        if constexpr (LT) {
#pragma unroll
          for (int u = 0; u < 2; ++u) {
#pragma unroll
            for (int b = 0; b < 4; ++b) {
              const uint32_t e = 4 * gg[u] + b;
              if (e >= lo_e[u] && e < hi_e[u]) {
                // the LT model: v activates through e iff v's choice word
                // falls in e's interval (S is marked, so an edge into S and a
                // node already active draw nothing)
                const int32_t v = va[u][b];
                if (!((gptr(bits)[(uint32_t)v >> 5] >> ((uint32_t)v & 31u)) & 1u)) {
                  const Words dv = philox_draw(Q.qid, A.seed, KIND_LT, S.stream, s, (uint64_t)((uint32_t)v >> 2));
                  const uint32_t W = word_at(dv, v & 3);
                  const OI_GLOBAL LtEdge* iv = gptr(A.lt_iv) + e;
                  if (W >= iv->lo && W <= iv->last && claim(bits, v)) push(queue, &s_tail, A.qcap, v);
                }
              }
            }
          }
        }
      }
      head += nb;
      __syncthreads();
    }
    const uint32_t Y = s_tail;
    if (leave || Y > A.qcap) {
      // outgrew the queue (or left at the soft cap): nothing of the sample
      // was recorded; it goes to the pass with full-size queues, and the
      // whole bitmap is cleared (bits may be set for nodes the queue could
      // not hold)
      if (tid == 0) {
        if (!BWD && A.list3)
          A.list3[atomicAdd(A.nlist3, 1u)] = f;
        else
          atomicOr(A.err, 16u);
      }
      for (int64_t w = tid; w < A.bits_words; w += NT) bits[w] = 0u;
      __syncthreads();
      continue;
    }
    if (tid == 0) {
      // a Monte-Carlo sample's output leaves out the seeds it started with
      const uint32_t Yo = mc ? Y - (uint32_t)Q.k : Y;
      if (BWD) {
        if (Y != y) atomicOr(A.err, 2u);
      } else {
        if (A.y_out) A.y_out[oidx] = Yo;
        if (A.e_out) A.e_out[oidx] = s_E;
        if (A.nbig && Y > A.big_mark) atomicAdd(A.nbig, 1u);
      }
      atomicAdd(&A.seg_sums[2 * sg], (unsigned long long)Yo);
      atomicAdd(&A.seg_sums[2 * sg + 1], s_E);
      atomicAdd(&A.tier_sums[4], (unsigned long long)Yo);
      atomicAdd(&A.tier_sums[5], s_E);
    }
    if ((int64_t)Y * 32 >= A.bits_words) {
      // a dense sample (at least one activation per 1024 nodes): clearing
      // the whole bitmap with coalesced full-line stores costs less than a
      // read-modify-write of one random line per activated node
      for (int64_t w = tid; w < A.bits_words; w += NT) bits[w] = 0u;
      __syncthreads();
    } else {
      for (uint32_t t = tid; t < Y; t += NT) bits[queue[t] >> 5] = 0u;
      __syncthreads();
      mark_seed_set<NT>(Q, bits, false, tid);
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// reductions for the stopping rules
// ---------------------------------------------------------------------------
// Sum of each chunk of `ch` consecutive Y values.
__global__ void __launch_bounds__(256) chunk_sums_kernel(const uint32_t* y, uint64_t count, uint32_t ch,
                                                         unsigned long long* out) {
  __shared__ unsigned long long part[4];
  const uint64_t c = blockIdx.x;
  const uint64_t b = c * ch;
  const uint64_t e = b + ch < count ? b + ch : count;
  unsigned long long s = 0;
  // 16-byte loads, four in flight per thread (b is a multiple of ch, which
  // is a multiple of 4), then the ragged tail one value at a time
  const uint64_t nv = (e - b) >> 2;
  const uint4* v = reinterpret_cast<const uint4*>(y + b);
  for (uint64_t k0 = threadIdx.x; k0 < nv; k0 += 4 * 256) {
    uint4 r[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint64_t k = k0 + (uint64_t)u * 256;
      r[u] = k < nv ? v[k] : make_uint4(0u, 0u, 0u, 0u);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) s += (unsigned long long)r[u].x + r[u].y + r[u].z + r[u].w;
  }
  for (uint64_t i = b + 4 * nv + threadIdx.x; i < e; i += 256) s += y[i];
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) s += __shfl_down(s, d, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[c] = part[0] + part[1] + part[2] + part[3];
}

constexpr uint64_t kPairsPerBlock = 16384;  // pair kernel: 128 KB of Y per block

// 128-bit sums of (y[2i] - y[2i+1])^2 per pair segment.  Each term is below
// 2^62; partial sums are carried as (lo, hi) pairs.  A segment's accumulator
// is two words (w0, w1) with sum = w0 + w1 * 2^32: an update adds the low 32
// bits of a partial sum to w0 and the rest to w1, so its two atomics need
// no returned value (w0 stays below 2^32 times the number of updates).
struct PairSeg {
  uint64_t out_off;  // first Y of the segment in y
  uint64_t npairs;
  uint64_t flat0;    // prefix over segments, in pairs
  uint32_t acc;      // accumulator index (2 words each)
  uint32_t pad;
};

__device__ __forceinline__ void add128(unsigned long long& lo, unsigned long long& hi, unsigned long long xlo,
                                       unsigned long long xhi) {
  const unsigned long long n = lo + xlo;
  hi += xhi + (n < lo ? 1ull : 0ull);
  lo = n;
}

__device__ __forceinline__ void flush128(unsigned long long* acc, unsigned long long lo, unsigned long long hi) {
  const unsigned long long old = atomicAdd(&acc[0], lo);
  atomicAdd(&acc[1], hi + (old + lo < old ? 1ull : 0ull));
}

// Pair segment holding flat pair index x (flat0 strictly increases: every
// pair segment has at least one pair).
__device__ __forceinline__ int32_t pair_segment(const PairSeg* ps, int32_t nps, uint64_t x) {
  int32_t a = 0, b = nps - 1;
  while (a < b) {
    const int32_t mid = (a + b + 1) >> 1;
    if (ps[mid].flat0 <= x)
      a = mid;
    else
      b = mid - 1;
  }
  return a;
}

__device__ __forceinline__ void add_limbs(unsigned long long* acc, unsigned long long L, unsigned long long H) {
  // a partial sum below 2^96 (at most 2^31 pairs of terms below 2^62), so
  // H * 2^32 fits in 64 bits
  if (L | H) {
    atomicAdd(&acc[0], L & 0xFFFFFFFFull);
    atomicAdd(&acc[1], (L >> 32) | (H << 32));
  }
}

// One pass per block over a contiguous range of pairs; partial sums are
// reduced across the block.  The block's first segment run goes to its
// own slot of `part` (no atomics: a launch over one segment would otherwise
// serialise on one address), later runs (past a segment boundary, rare) to
// the segment's accumulator.
__global__ void __launch_bounds__(256) pair_sq_kernel(const uint32_t* y, const PairSeg* ps, int32_t nps,
                                                      uint64_t total, uint64_t per_block, unsigned long long* acc,
                                                      unsigned long long* part) {
  __shared__ unsigned long long red_lo[4], red_hi[4];
  const uint64_t b0 = (uint64_t)blockIdx.x * per_block;
  const uint64_t b1 = b0 + per_block < total ? b0 + per_block : total;
  if (b0 >= b1) return;
  // segment of the block's first pair; blocks are small next to segments,
  // so a block crosses few segment boundaries
  int32_t seg = pair_segment(ps, nps, b0);
  bool first = true;
  uint64_t lo_pair = b0;
  while (lo_pair < b1 && seg < nps) {
    const PairSeg P = ps[seg];
    const uint64_t seg_end = P.flat0 + P.npairs;
    const uint64_t hi_pair = seg_end < b1 ? seg_end : b1;
    if (hi_pair <= lo_pair) {  // empty segment
      ++seg;
      continue;
    }
    unsigned long long lo = 0, hi = 0;
    // local pair indices [a, b) of this segment; pairs 2k and 2k + 1 sit in
    // one 16-byte-aligned group of four Y values (out_off is 4096-aligned)
    uint64_t a = lo_pair - P.flat0;
    const uint64_t b = hi_pair - P.flat0;
    const uint32_t* yb = y + P.out_off;
    if ((a & 1) && a < b) {  // a leading odd pair
      if (threadIdx.x == 0) {
        const uint2 v = *reinterpret_cast<const uint2*>(&yb[2 * a]);
        const unsigned long long d = v.x > v.y ? (unsigned long long)(v.x - v.y) : (unsigned long long)(v.y - v.x);
        add128(lo, hi, d * d, 0);
      }
      ++a;
    }
    const uint64_t q0 = a >> 1, q1 = b >> 1;  // whole groups of two pairs
    for (uint64_t q = q0 + threadIdx.x; q < q1; q += 8 * 256) {
      uint4 v[8];  // eight 16-byte loads in flight per thread
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const uint64_t qq = q + (uint64_t)u * 256;
        v[u] = make_uint4(0u, 0u, 0u, 0u);
        if (qq < q1) v[u] = *reinterpret_cast<const uint4*>(&yb[4 * qq]);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const unsigned long long d0 =
            v[u].x > v[u].y ? (unsigned long long)(v[u].x - v[u].y) : (unsigned long long)(v[u].y - v[u].x);
        const unsigned long long d1 =
            v[u].z > v[u].w ? (unsigned long long)(v[u].z - v[u].w) : (unsigned long long)(v[u].w - v[u].z);
        add128(lo, hi, d0 * d0, 0);
        add128(lo, hi, d1 * d1, 0);
      }
    }
    if ((b & 1) && 2 * q1 >= a && threadIdx.x == 0) {  // a trailing odd pair
      const uint2 v = *reinterpret_cast<const uint2*>(&yb[2 * (b - 1)]);
      const unsigned long long d = v.x > v.y ? (unsigned long long)(v.x - v.y) : (unsigned long long)(v.y - v.x);
      add128(lo, hi, d * d, 0);
    }
#pragma unroll
    for (int sh = 32; sh > 0; sh >>= 1) {
      const unsigned long long olo = __shfl_down(lo, sh, 64), ohi = __shfl_down(hi, sh, 64);
      add128(lo, hi, olo, ohi);
    }
    if ((threadIdx.x & 63) == 0) {
      red_lo[threadIdx.x >> 6] = lo;
      red_hi[threadIdx.x >> 6] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long L = 0, H = 0;
      for (int w = 0; w < 4; ++w) add128(L, H, red_lo[w], red_hi[w]);
      if (first) {
        part[2 * blockIdx.x] = L;
        part[2 * blockIdx.x + 1] = H;
      } else {
        add_limbs(&acc[2 * P.acc], L, H);
      }
    }
    first = false;
    __syncthreads();
    lo_pair = hi_pair;
    ++seg;
  }
}

// Adds each pair_sq block's first-run partial to its segment's accumulator:
// one block; thread t takes blocks t, t + 256, ... (independent loads) and
// makes one update per change of segment.
__global__ void __launch_bounds__(256) pair_reduce_kernel(const PairSeg* ps, int32_t nps, uint64_t nblocks,
                                                          uint64_t per_block, const unsigned long long* part,
                                                          unsigned long long* acc) {
  int32_t cur = -1;
  unsigned long long L = 0, H = 0;
#pragma unroll 4
  for (uint64_t k = threadIdx.x; k < nblocks; k += 256) {
    const int32_t j = nps == 1 ? 0 : pair_segment(ps, nps, k * per_block);
    if (j != cur) {
      if (cur >= 0) add_limbs(&acc[2 * ps[cur].acc], L, H);
      cur = j;
      L = H = 0;
    }
    add128(L, H, part[2 * k], part[2 * k + 1]);
  }
  if (cur >= 0) add_limbs(&acc[2 * ps[cur].acc], L, H);
}

// ---------------------------------------------------------------------------
// backward finishing: integer Y-sums -> fp32 gradient
// ---------------------------------------------------------------------------
// edges per run of the finishing pass (one block per run at a time), and
// the longest slice of row_ptr a run stages in LDS
constexpr int64_t kBwdRun = 2048;
constexpr int64_t kBwdRows = 2048;

// src[r] = the source of run r's first edge (r < runs), src[runs] = the
// source of the last edge: the first u with row_ptr[u + 1] > e, one search
// per thread
__global__ void __launch_bounds__(256) bwd_run_sources_kernel(const int64_t* row_ptr, int64_t n, int64_t m,
                                                              int64_t runs, int64_t* src) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r <= runs; r += stride) {
    const int64_t e = r < runs ? r * kBwdRun : m - 1;
    int64_t lo = 0, hi = n - 1;
    while (lo < hi) {
      const int64_t mid = lo + ((hi - lo) >> 1);
      if (row_ptr[mid + 1] > e)
        hi = mid;
      else
        lo = mid + 1;
    }
    src[r] = lo;
  }
}

// Stage-2 edges: g_p = scale * (L/p - D/(1-p)), g_theta = scale * (L(1-p) - D p),
// with D = N_u - L for an edge (u, v), v outside S (N_u: the Y-sum of the
// samples that expand u), and L = D = 0 for an edge into S.  One thread per
// edge, which keeps a hub's row spread over many threads; its source u is
// the row with row_ptr[u] <= e < row_ptr[u + 1].  A block takes runs of
// kBwdRun consecutive edges: run r's sources lie in [src[r], src[r + 1]],
// whose slice of row_ptr is staged in LDS when it fits (else the search
// reads row_ptr itself).  Every edge's gradient is written.  The live sums
// read are cleared, so that the array is all zero again for the next
// backward.
__global__ void __launch_bounds__(256) bwd_edges_kernel(const int64_t* row_ptr, const EdgeGroup* eg, int64_t n,
                                                        int64_t m, const float* pe_arr, unsigned long long* acc_live,
                                                        const unsigned long long* acc_node, const uint32_t* sbits,
                                                        const int64_t* src, double scale, int theta, float* grad) {
  __shared__ int64_t s_rp[kBwdRows + 1];
  const int64_t runs = (m + kBwdRun - 1) / kBwdRun;
  for (int64_t r = blockIdx.x; r < runs; r += gridDim.x) {
    const int64_t first = r * kBwdRun;
    const int64_t last = (first + kBwdRun < m ? first + kBwdRun : m) - 1;
    const int64_t u0 = src[r], u1 = src[r + 1];
    // row_ptr[u0 + 1 .. u1 + 1]: the bounds the search compares against
    const int64_t nr = u1 - u0 + 1;
    const bool staged = nr <= kBwdRows + 1;
    if (staged)
      for (int64_t x = threadIdx.x; x < nr; x += blockDim.x) s_rp[x] = row_ptr[u0 + 1 + x];
    __syncthreads();
    for (int64_t e = first + threadIdx.x; e <= last; e += blockDim.x) {
      int64_t lo = u0, hi = u1;  // e's source lies between src[r] and src[r + 1]
      while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if ((staged ? s_rp[mid - u0] : row_ptr[mid + 1]) > e)
          hi = mid;
        else
          lo = mid + 1;
      }
      const unsigned long long N = acc_node[lo];
      double g = 0.0;
      if (N == 0) {
        // no sample expanded the source: L = D = 0 (a live sum only grows
        // with its source's expansion sum)
        g = scale * 0.0;
      } else {
        const double p = (double)pe_arr[e];
        const unsigned long long L = acc_live[e];
        if (L) acc_live[e] = 0ull;  // left cleared for the next backward
        const unsigned long long D = seed_bit(sbits, eg[e >> 2].v[e & 3]) ? 0ull : N - L;
        if (theta) {
          g = scale * ((double)L * (1.0 - p) - (double)D * p);
        } else {
          double a = 0.0, b = 0.0;
          if (L) a = (double)L / p;
          if (D) b = (double)D / (1.0 - p);
          g = scale * (a - b);
        }
      }
      grad[e] = (float)g;
    }
    __syncthreads();  // s_rp is rewritten by the next run
  }
}

// S-edges into Stage-1 entry j: x_j = 1 contributes A_j * prod_{f != e}(1 - p_f) / P_j,
// x_j = 0 contributes -B_j / (1 - p_e), B_j = sumY - A_j.
__global__ void __launch_bounds__(256) bwd_stage1_kernel(const float* pe_arr, const int64_t* se_off,
                                                         const int64_t* se, const double* P, int64_t l,
                                                         const unsigned long long* acc_tab,
                                                         unsigned long long sumY, double scale, int theta,
                                                         float* grad) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < l; j += stride) {
    const unsigned long long Aj = acc_tab[j], Bj = sumY - Aj;
    const int64_t b0 = se_off[j], b1 = se_off[j + 1];
    for (int64_t a = b0; a < b1; ++a) {
      const int64_t e = se[a];
      const double pe = (double)pe_arr[e];
      double live = 0.0, dead = 0.0;
      if (Aj) {
        double prod = 1.0;
        for (int64_t c = b0; c < b1; ++c)
          if (c != a) {
            const int64_t f = se[c];
            prod = prod * (1.0 - (double)pe_arr[f]);
          }
        live = (double)Aj * prod / P[j];
      }
      double g;
      if (theta) {
        if (Bj) dead = (double)Bj * pe;
        g = scale * (live * pe * (1.0 - pe) - dead);
      } else {
        if (Bj) dead = (double)Bj / (1.0 - pe);
        g = scale * (live - dead);
      }
      grad[e] = (float)g;
    }
  }
}

// p_e = sigmoid(theta_e) in fp64, rounded to fp32, written into the plain
// fp32 array and, as coin thresholds, into the edge groups.
__global__ void __launch_bounds__(256) theta_to_p_kernel(const float* theta, int64_t m, EdgeGroup* eg, float* p_out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += stride) {
    const double t = (double)theta[e];
    const float p = (float)(1.0 / (1.0 + exp(-t)));
    eg[e >> 2].thr[e & 3] = coin_threshold(p);
    p_out[e] = p;
  }
}

// ---------------------------------------------------------------------------
// gather probe: the samplers' memory accesses without coins, queues or
// visited sets, to measure the random-read bandwidth they are bound by
// ---------------------------------------------------------------------------

// nodes[i] = target of edge h(seed, i) mod m: nodes drawn in proportion to
// their in-degree, the law by which a cascade reaches them.
__global__ void __launch_bounds__(256) probe_nodes_kernel(const EdgeGroup* eg, int64_t m, uint64_t count,
                                                          uint32_t seed, int32_t* nodes) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
    const uint32_t a = mix32((uint32_t)i ^ seed);
    const uint32_t b = mix32((uint32_t)(i >> 32) ^ a ^ 0x85EBCA6Bu);
    const uint64_t h = ((((uint64_t)b) << 32) | a) % (uint64_t)m;
    nodes[i] = eg[h >> 2].v[h & 3];
  }
}

// A wave takes 64 nodes, one per lane: each lane reads its node's row_ptr
// pair, then the wave reads the edge groups of all 64 rows together, lane t
// taking group t of the concatenated rows (so long rows are read by many
// lanes and short ones do not leave lanes idle).  This reads exactly the
// bytes the samplers read for those nodes, as fast as a wave can.
// out[0] += edges read (inside the rows), out[1] ^= a fold of everything
// read (keeps the loads live).
__global__ void __launch_bounds__(256) gather_probe_kernel(const int64_t* row_ptr, const EdgeGroup* eg,
                                                           const int32_t* nodes, uint64_t count,
                                                           unsigned long long* out) {
  __shared__ int64_t s_b[4][64], s_e[4][64];
  __shared__ uint32_t s_end[4][64];
  __shared__ unsigned long long red[4];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint64_t nwaves = (uint64_t)gridDim.x * 4;
  uint64_t edges = 0;
  uint32_t fold = 0;
  for (uint64_t base = ((uint64_t)blockIdx.x * 4 + w) * 64; base < count; base += nwaves * 64) {
    const uint64_t i = base + lane;
    int64_t b = 0, e = 0;
    if (i < count) {
      const int32_t u = nodes[i];
      b = row_ptr[u];
      e = row_ptr[u + 1];
    }
    edges += (uint64_t)(e - b);
    const uint32_t ng = e > b ? (uint32_t)(((e + 3) >> 2) - (b >> 2)) : 0u;
    const uint32_t incl = wave_incl_scan(ng, lane);
    s_b[w][lane] = b;
    s_e[w][lane] = e;
    s_end[w][lane] = incl;
    wave_sync();
    const uint32_t total = uniform((uint32_t)__shfl((int)incl, 63, 64));
    for (uint32_t t = lane; t < total; t += 64) {
      int lo = 0, hi = 63;  // first lane whose rows end after group t
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (s_end[w][mid] > t)
          hi = mid;
        else
          lo = mid + 1;
      }
      const uint32_t start = lo ? s_end[w][lo - 1] : 0u;
      const int64_t rb = s_b[w][lo], re = s_e[w][lo];
      const int64_t g = (rb >> 2) + (int64_t)(t - start);
      const OI_GLOBAL char* q = (const OI_GLOBAL char*)(gptr(eg) + g);
      const v4i32 vv = *(const OI_GLOBAL v4i32*)q;
      const v4i32 pp = *(const OI_GLOBAL v4i32*)(q + 16);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int64_t x = 4 * g + k;
        if (x >= rb && x < re) fold ^= (uint32_t)vv[k] ^ (uint32_t)pp[k];
      }
    }
    wave_sync();
  }
  const unsigned long long se = wave_sum64(edges);
  unsigned long long sf = fold;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) sf ^= __shfl_xor(sf, d, 64);
  if (lane == 0) red[w] = se;
  __syncthreads();
  if (threadIdx.x == 0) {
    atomicAdd(&out[0], red[0] + red[1] + red[2] + red[3]);
    atomicXor(&out[1], sf);
  }
}

// coin probe: the samplers' coin draws (Philox4x32-10 with the edge-coin key
// and counter layout) and threshold compares alone, without loads, queues or
// visited sets, to measure the rate at which this chip can produce coins
// ---------------------------------------------------------------------------

// Lane t draws the coins of samples s = t, t + stride, ...: for each, edge
// groups 0..groups_per_sample-1 (one draw of four coin words each), every
// word compared with one of four fixed thresholds.  out[0] += words below
// their threshold.
__global__ void __launch_bounds__(256) coin_probe_kernel(uint64_t samples, uint32_t groups_per_sample, uint32_t seed,
                                                         uint32_t qid, unsigned long long* out) {
  __shared__ unsigned long long red[4];
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint32_t thr[4] = {0x19999999u, 0x028F5C28u, 0x00418937u, 0x80000000u};
  uint32_t live = 0;
  for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < samples; s += stride) {
    for (uint32_t g = 0; g < groups_per_sample; ++g) {
      const Words w = philox_draw(qid, seed, KIND_EDGE, 0, s, g);
#pragma unroll
      for (int b = 0; b < 4; ++b) live += w.w[b] < thr[b] ? 1u : 0u;
    }
  }
  const unsigned long long sum = wave_sum64(live);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sum;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(&out[0], red[0] + red[1] + red[2] + red[3]);
}

// ---------------------------------------------------------------------------
// host-callable launchers
// ---------------------------------------------------------------------------
struct SmallVariant {
  const void* fwd;
  const void* bwd;
  int k, hcap, rcap, r;
};

#define OI_VARIANT(K, H, RC, R) \
  {reinterpret_cast<const void*>(&small_kernel<K, H, RC, R, false>), \
   reinterpret_cast<const void*>(&small_kernel<K, H, RC, R, true>), K, H, RC, R}

static const SmallVariant kVariants[] = {
    OI_VARIANT(4, 256, 512, 2),
    OI_VARIANT(8, 128, 512, 2),
    OI_VARIANT(2, 512, 512, 2),
    OI_VARIANT(4, 256, 512, 1),
    OI_VARIANT(4, 256, 512, 4),
    OI_VARIANT(8, 256, 1024, 2),
};

int num_small_variants() { return (int)(sizeof(kVariants) / sizeof(kVariants[0])); }

void small_variant_info(int v, int* k, int* hcap, int* rcap, int* r) {
  const SmallVariant& s = kVariants[v];
  *k = s.k;
  *hcap = s.hcap;
  *rcap = s.rcap;
  *r = s.r;
}

hipError_t small_occupancy(int v, bool bwd, int* blocks_per_cu) {
  const SmallVariant& s = kVariants[v];
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, bwd ? s.bwd : s.fwd, 256, 0);
}

hipError_t launch_small(int v, bool bwd, const SampleLaunch& A, int blocks, hipStream_t st) {
  const SmallVariant& s = kVariants[v];
  void* args[] = {const_cast<SampleLaunch*>(&A)};
  return hipLaunchKernel(bwd ? s.bwd : s.fwd, dim3(blocks), dim3(256), args, 0, st);
}

constexpr int TINY_CAP = 16;

int tiny_cap() { return TINY_CAP; }

// the instantiation a launch runs: the backward, Monte-Carlo cascades, or
// IICP samples with or without first-level passes
static const void* tiny_fn(bool bwd, const SampleLaunch& A) {
  if (bwd) return reinterpret_cast<const void*>(&tiny_kernel<TINY_CAP, true, false, 0>);
  if (A.mc) return reinterpret_cast<const void*>(&tiny_kernel<TINY_CAP, false, true, 0>);
  if (A.p1 == 1) return reinterpret_cast<const void*>(&tiny_kernel<TINY_CAP, false, false, 1>);
  if (A.p1 == 2) return reinterpret_cast<const void*>(&tiny_kernel<TINY_CAP, false, false, 2>);
  return reinterpret_cast<const void*>(&tiny_kernel<TINY_CAP, false, false, 0>);
}

hipError_t tiny_occupancy(bool bwd, const SampleLaunch& A, int* blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, tiny_fn(bwd, A), 256, 0);
}

hipError_t launch_tiny(bool bwd, const SampleLaunch& A, int blocks, hipStream_t st) {
  void* args[] = {const_cast<SampleLaunch*>(&A)};
  return hipLaunchKernel(tiny_fn(bwd, A), dim3(blocks), dim3(256), args, 0, st);
}

hipError_t large_occupancy(bool bwd, int* blocks_per_cu) {
  // the pool is sized for the most demanding instantiation of the main pool
  int a = 0, b = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &a,
      bwd ? reinterpret_cast<const void*>(&large_kernel<true, LB, false>)
          : reinterpret_cast<const void*>(&large_kernel<false, LB, false>),
      LB, 0);
  if (e == hipSuccess && !bwd)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, reinterpret_cast<const void*>(&large_kernel<false, LB, true>),
                                                     LB, 0);
  *blocks_per_cu = bwd ? a : (a > b ? a : b);
  return e;
}

// Resident 1024-thread blocks per CU of the full-queue pass (the most of its
// three instantiations).
hipError_t large_full_occupancy(int* blocks_per_cu) {
  int a = 0, b = 0, c = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &a, reinterpret_cast<const void*>(&large_kernel<false, LB_FULL, false>), LB_FULL, 0);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &b, reinterpret_cast<const void*>(&large_kernel<false, LB_FULL, true>), LB_FULL, 0);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &c, reinterpret_cast<const void*>(&large_kernel<true, LB_FULL, false>), LB_FULL, 0);
  int m = a > b ? a : b;
  *blocks_per_cu = m > c ? m : c;
  return e;
}

hipError_t launch_large(bool bwd, const SampleLaunch& A, int blocks, hipStream_t st) {
  if (bwd)
    hipLaunchKernelGGL((large_kernel<true, LB, false>), dim3(blocks), dim3(LB), 0, st, A);
  else if (A.lt)
    hipLaunchKernelGGL((large_kernel<false, LB, true>), dim3(blocks), dim3(LB), 0, st, A);
  else
    hipLaunchKernelGGL((large_kernel<false, LB, false>), dim3(blocks), dim3(LB), 0, st, A);
  return hipGetLastError();
}

hipError_t launch_large_full(bool bwd, const SampleLaunch& A, int blocks, hipStream_t st) {
  if (bwd)
    hipLaunchKernelGGL((large_kernel<true, LB_FULL, false>), dim3(blocks), dim3(LB_FULL), 0, st, A);
  else if (A.lt)
    hipLaunchKernelGGL((large_kernel<false, LB_FULL, true>), dim3(blocks), dim3(LB_FULL), 0, st, A);
  else
    hipLaunchKernelGGL((large_kernel<false, LB_FULL, false>), dim3(blocks), dim3(LB_FULL), 0, st, A);
  return hipGetLastError();
}

hipError_t launch_chunk_sums(const uint32_t* y, uint64_t count, uint32_t ch, unsigned long long* out,
                             hipStream_t st) {
  const uint64_t nc = (count + ch - 1) / ch;
  if (nc == 0) return hipSuccess;
  if (ch % 4) return hipErrorInvalidValue;  // chunks start 16-byte aligned
  hipLaunchKernelGGL(chunk_sums_kernel, dim3((unsigned)nc), dim3(256), 0, st, y, count, ch, out);
  return hipGetLastError();
}

// Sets the bit of every seed found in an open-addressing seed-set table of
// cap entries (empty slots hold -1).
__global__ void __launch_bounds__(256) seed_bits_kernel(const int32_t* shash, uint32_t cap, uint32_t* sbits) {
  for (uint32_t h = blockIdx.x * 256u + threadIdx.x; h < cap; h += gridDim.x * 256u) {
    const int32_t v = shash[h];
    if (v >= 0) atomicOr(&sbits[(uint32_t)v >> 5], 1u << ((uint32_t)v & 31u));
  }
}

hipError_t launch_seed_bits(const int32_t* shash, uint32_t cap, uint32_t* sbits, hipStream_t st) {
  const uint32_t want = (cap + 255u) / 256u, blocks = want < 64u ? want : 64u;
  hipLaunchKernelGGL(seed_bits_kernel, dim3(blocks ? blocks : 1u), dim3(256), 0, st, shash, cap, sbits);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256) clear_u64_kernel(unsigned long long* p, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) p[i] = 0ull;
}

hipError_t launch_clear_u64(unsigned long long* p, uint64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const uint64_t want = (n + 255) / 256, blocks = want < 1024 ? want : 1024;
  hipLaunchKernelGGL(clear_u64_kernel, dim3((unsigned)blocks), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

uint64_t pair_sq_blocks(uint64_t total) { return (total + kPairsPerBlock - 1) / kPairsPerBlock; }

// part: 2 words per block (pair_sq_blocks(total) blocks)
hipError_t launch_pair_sq(const uint32_t* y, const void* ps, int32_t nps, uint64_t total, unsigned long long* acc,
                          unsigned long long* part, hipStream_t st) {
  if (total == 0) return hipSuccess;
  const uint64_t blocks = pair_sq_blocks(total);
  const PairSeg* p = reinterpret_cast<const PairSeg*>(ps);
  hipLaunchKernelGGL(pair_sq_kernel, dim3((unsigned)blocks), dim3(256), 0, st, y, p, nps, total, kPairsPerBlock,
                     acc, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(pair_reduce_kernel, dim3(1), dim3(256), 0, st, p, nps, blocks, kPairsPerBlock, part, acc);
  return hipGetLastError();
}

size_t pair_seg_size() { return sizeof(PairSeg); }

hipError_t launch_theta_to_p(const float* theta, int64_t m, EdgeGroup* eg, float* p_out, hipStream_t st) {
  if (m == 0) return hipSuccess;
  int64_t blocks = (m + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(theta_to_p_kernel, dim3((unsigned)blocks), dim3(256), 0, st, theta, m, eg, p_out);
  return hipGetLastError();
}

size_t bwd_run_count(int64_t m) { return m > 0 ? (size_t)((m + kBwdRun - 1) / kBwdRun) : 0; }

// src: bwd_run_count(m) + 1 entries of workspace
hipError_t launch_bwd_edges(const int64_t* row_ptr, const EdgeGroup* eg, int64_t n, int64_t m, const float* pe,
                            unsigned long long* L, const unsigned long long* N, const uint32_t* sbits,
                            int64_t* src, double scale, int theta, float* grad, hipStream_t st) {
  if (m == 0) return hipSuccess;
  const int64_t runs = (int64_t)bwd_run_count(m);
  int64_t sb = (runs + 1 + 255) / 256;
  if (sb > 65536) sb = 65536;
  hipLaunchKernelGGL(bwd_run_sources_kernel, dim3((unsigned)sb), dim3(256), 0, st, row_ptr, n, m, runs, src);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  int64_t blocks = runs;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(bwd_edges_kernel, dim3((unsigned)blocks), dim3(256), 0, st, row_ptr, eg, n, m, pe, L, N, sbits,
                     src, scale, theta, grad);
  return hipGetLastError();
}

hipError_t launch_bwd_stage1(const float* pe, const int64_t* se_off, const int64_t* se, const double* P,
                             int64_t l, const unsigned long long* acc_tab, unsigned long long sumY, double scale,
                             int theta, float* grad, hipStream_t st) {
  if (l == 0) return hipSuccess;
  int64_t blocks = (l + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(bwd_stage1_kernel, dim3((unsigned)blocks), dim3(256), 0, st, pe, se_off, se, P, l, acc_tab,
                     sumY, scale, theta, grad);
  return hipGetLastError();
}

hipError_t launch_probe_nodes(const EdgeGroup* eg, int64_t m, uint64_t count, uint32_t seed, int32_t* nodes,
                              hipStream_t st) {
  if (count == 0 || m == 0) return hipSuccess;
  uint64_t blocks = (count + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(probe_nodes_kernel, dim3((unsigned)blocks), dim3(256), 0, st, eg, m, count, seed, nodes);
  return hipGetLastError();
}

hipError_t launch_gather_probe(const int64_t* row_ptr, const EdgeGroup* eg, const int32_t* nodes, uint64_t count,
                               unsigned long long* out, int cus, hipStream_t st) {
  if (count == 0) return hipSuccess;
  int bpc = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &bpc, reinterpret_cast<const void*>(&gather_probe_kernel), 256, 0);
  if (e != hipSuccess) return e;
  if (bpc < 1) bpc = 1;
  uint64_t blocks = (uint64_t)bpc * (uint64_t)cus;
  const uint64_t need = (count + 255) / 256;
  if (blocks > need) blocks = need;
  hipLaunchKernelGGL(gather_probe_kernel, dim3((unsigned)blocks), dim3(256), 0, st, row_ptr, eg, nodes, count, out);
  return hipGetLastError();
}

hipError_t launch_coin_probe(uint64_t samples, uint32_t groups_per_sample, uint32_t seed, uint32_t qid,
                             unsigned long long* out, int cus, hipStream_t st) {
  if (samples == 0 || groups_per_sample == 0) return hipSuccess;
  int bpc = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &bpc, reinterpret_cast<const void*>(&coin_probe_kernel), 256, 0);
  if (e != hipSuccess) return e;
  if (bpc < 1) bpc = 1;
  uint64_t blocks = (uint64_t)bpc * (uint64_t)cus * 4;
  const uint64_t need = (samples + 255) / 256;
  if (blocks > need) blocks = need;
  hipLaunchKernelGGL(coin_probe_kernel, dim3((unsigned)blocks), dim3(256), 0, st, samples, groups_per_sample, seed,
                     qid, out);
  return hipGetLastError();
}

}  // namespace oi
