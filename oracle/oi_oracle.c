/*
 * CPU oracle for outward-influence estimation with IICP samples and RSA.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link,
 * load or call this file.  Only tests/, the smoke check in __graft_entry__.py
 * and the `cpu_baseline` leg of bench.py use it.  It shares no code, header,
 * table or helper with the HIP library: it implements the same written
 * specification independently, in plain sequential C (fp64, no FMA: build
 * with -ffp-contract=off), so that the two can be compared bit for bit.
 *
 * What it computes (paper: Nguyen, Dinh, Thai, "Outward Influence and
 * Cascade Size Estimation in Billion-scale Networks"):
 *   - the exact outward influence Ext(S) and its gradient by enumerating all
 *     live-edge graphs (Sec. 2, the sample-graph definition of I(S) and the
 *     enumeration form of Ext(S) used in the proof of Lemma 1);
 *   - the Stage-1 quantities P_{S,v}, Pr[A_i] and beta_0 (Sec. 3.1,
 *     Eqs. psv, pai, pal, zerop);
 *   - one IICP sample (Alg. 1), and one classic IC Monte-Carlo sample M^(S)
 *     (Sec. 2.3) for comparison;
 *   - GSRA (Alg. 2) and RSA (Alg. 3) over abstract integer streams;
 *   - SOIEA (Alg. 4) and SIEA (Alg. 5, the Z transform of Sec. 5.2);
 *   - a score-function gradient of the fixed-count estimate (not in the
 *     paper; see oo_backward).
 *
 * Readings of points the paper leaves open (each is a choice both
 * implementations make identically):
 *   R1 N^out_S is ordered by ascending node id ("assume an order", Sec. 3.1).
 *   R2 P_{S,v} = 1 - prod (1 - w(u,v)) with the product taken over the edges
 *      from S into v in ascending edge id, left to right, in fp64.  P_{S,v}=1
 *      is allowed; S is never modified.
 *   R3 Pr[A_j] is formed as Q_{j-1} * P_j with Q_0 = 1, Q_j = Q_{j-1}(1-P_j);
 *      CDF_j = CDF_{j-1} + Pr[A_j]; beta_0 = CDF_l (Eqs. pai, zerop).
 *   R4 Randomness is Philox4x32-10 (Salmon et al., SC'11) keyed by
 *      (query id, run seed); counter = (lo32(idx), hi32(idx), lo32(s),
 *      kind<<28 | stream<<27 | hi32(s)), s = sample index in its stream.
 *      Edge coin of edge e: word (e mod 4) of the block with idx = e div 4,
 *      kind 0.  Stage-1 coin of table entry j (0-based): word (j mod 4) of
 *      idx = j div 4, kind 2.  Selection uniform: kind 1, idx 0,
 *      U = ((w0>>5)*2^26 + (w1>>6)) * 2^-53.
 *   R5 A coin with probability p is live iff word < floor(p * 2^32)
 *      (exact for p in [0,1]; p=0 never, p=1 always live).
 *   R6 Selection: t = U*beta_0, i = min{j : CDF_j > t}; if none, the largest
 *      j with Pr[A_j] > 0.
 *   R7 Nodes v_1..v_{i-1} are not marked by Stage 1 and may be activated in
 *      Stage 2; S is marked (Alg. 1 as written).
 *   R8 Stopping-rule constants: c(eps',delta) uses eps' in its (2 + 2/3 .)
 *      factor (Table 1 as printed); expression order is fixed (see upsilon()).
 *   R9 GSRA returns h/T (the unbiased form of Alg. 2).
 *   R10 RSA step 2 uses consecutive disjoint pairs (X'_{2i-1}, X'_{2i}),
 *       i = 1..N_sigma (as in the proof of Theorem 4); N_sigma and T are
 *       rounded up and floored at 1; step 3 sums exactly X_1..X_T of the
 *       same stream as step 1; Upsilon_2 uses Upsilon(eps, delta) with the
 *       final eps, delta and the same (a, b).
 *   R11 For SIEA the running sum of Z = beta_0 Y + |S| is formed from the
 *       integer sum of Y: sum Z = beta_0 * sumY + |S| * T (one expression), and
 *       the paired squared differences of Z' are beta_0^2 times the integer
 *       sum of squared differences of Y'.
 *   R12 beta_0 = 0 (S has no out-neighbour outside S): OI = 0, IS = |S|, no
 *       samples are drawn.
 *   R17 The LT model (Sec. 5.3, and SIEA_LT in the experiments) in its
 *       live-edge form (Kempe et al.): every node v keeps at most one of its
 *       in-edges, edge (u, v) with probability w(u, v) and none with
 *       probability 1 - sum_u w(u, v) (which must be >= 0; sums up to
 *       1 + 1e-6 are taken as 1).  v's choice is the word W_v = word (v mod 4)
 *       of the Philox block kind 4, idx = v div 4; v's in-edges, in ascending
 *       edge id, own consecutive intervals [t_{k-1}, t_k) of the 2^32 words,
 *       t_k = floor(min(c_k, 1) * 2^32) with c_k the fp64 running sum of their
 *       weights (left to right), and an edge is live iff W_v falls in its
 *       interval.  An LT sample is the set reachable from S over live edges;
 *       SIEA_LT runs RSA on its size X = |S| + Y over [a, b] = [|S|, n].
 *   R16 Stage-1 skip sampling (a different consumption of randomness for the
 *       same law, used when l >= max(skip_min_l, 65), skip_min_l = 4096
 *       unless set, and the table is sparse enough for the walks to pay:
 *       W * skip_cost <= l / 4, where W = ceil(l / 256) plus the sum of P_j
 *       over the light entries (fp64, the count first, then ascending j) is
 *       the walks' expected number of draws from i = 0, l / 4 the coins'
 *       Philox blocks, and skip_cost = 8 unless set (0: no density test), the
 *       measured cost of one walk step in coin blocks rounded up to a power
 *       of two): after the selection i, entries with P_j >= 1/2 ("heavy") are
 *       flipped with their own coins as in R4; entries with 0 < P_j < 1/2
 *       ("light") are visited by one walk per segment of 256 table indices.
 *       Within segment m (indices [256m, 256m + 256)) R_j is the product of
 *       (1 - P_k) over the light k in [256m, j].  A walk stands at pos = i if
 *       i lies in the segment, else at 256m - 1 (R = 1 there), draws
 *       U' = 1 - U (U as for the selection, kind 3, idx = pos, or 2^40 + m at
 *       the segment's start), and the next live entry is the smallest j > pos
 *       in the segment with R_j < U' R_pos (none: the walk ends); the walk
 *       moves to j and draws again.  Given the walk at pos, no entry of
 *       (pos, j] is live with probability R_j / R_pos, so every light entry
 *       after i is live independently with probability P_j, while the draws
 *       number about (l - i) / 256 + sum of P_j instead of l - i.  The
 *       examined-edge count keeps the l - 1 - i Stage-1 entries of R15.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 oo_u128;

enum { OO_OK = 0, OO_EINVAL = -1, OO_ERANGE = -2, OO_ENOMEM = -3 };
enum { KIND_EDGE = 0, KIND_SELECT = 1, KIND_STAGE1 = 2, KIND_SKIP = 3, KIND_LT = 4 };

/* R16: the spec's constants, the table size from which skip sampling is
 * used, and the draw-cost ratio of its density test */
enum { SKIP_SEG = 256, SKIP_LMIN_FLOOR = 65 };
static int64_t g_skip_min_l = 4096;
static double g_skip_cost = 8.0;
void oo_set_stage1_skip(int64_t min_l) { g_skip_min_l = min_l; }
void oo_set_stage1_skip_cost(double cost) { g_skip_cost = cost; }

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from the published description (multiply-xor rounds with  */
/* the Weyl key schedule).                                                  */
/* ------------------------------------------------------------------------ */
void oo_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t a = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t b = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(a >> 32), lo0 = (uint32_t)a;
        uint32_t hi1 = (uint32_t)(b >> 32), lo1 = (uint32_t)b;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

static void draw(uint32_t qid, uint32_t seed, uint32_t kind, uint32_t stream,
                 uint64_t s, uint64_t idx, uint32_t out[4])
{
    uint32_t ctr[4], key[2];
    ctr[0] = (uint32_t)idx;
    ctr[1] = (uint32_t)(idx >> 32);
    ctr[2] = (uint32_t)s;
    ctr[3] = (kind << 28) | (stream << 27) | ((uint32_t)(s >> 32) & 0x07FFFFFFu);
    key[0] = qid;
    key[1] = seed;
    oo_philox(ctr, key, out);
}

/* R5 */
static uint64_t coin_threshold(double prob) { return (uint64_t)(prob * 4294967296.0); }

/* ------------------------------------------------------------------------ */
/* Graph and Stage-1 table                                                  */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t n, m;
    const int64_t *row_ptr;
    const int32_t *col;
    const float *p;
} oo_graph;

typedef struct {
    int64_t k;          /* |S| after removing duplicates */
    int32_t *S;         /* sorted seeds */
    uint8_t *inS;       /* n flags */
    int64_t l;          /* |N^out_S| */
    int32_t *v;         /* v_1..v_l (0-based j) */
    double *P;          /* P_{S,v_j} */
    double *cdf;        /* l+1 entries, cdf[0] = 0, cdf[j+1] = CDF after entry j */
    uint64_t *thr;      /* floor(P_j * 2^32) */
    double beta0;
    int64_t *se_off;    /* l+1: S-edges into v_j are se[se_off[j]..se_off[j+1]) */
    int64_t *se;        /* edge ids, ascending inside each entry */
    int skip;           /* R16: Stage 1 by skip sampling */
    double *R;          /* R16: survival products of light entries, per segment */
    int64_t *heavy;     /* R16: entries with P_j >= 1/2, ascending */
    int64_t nheavy;
} oo_table;

void oo_table_free(oo_table *t)
{
    if (!t) return;
    free(t->S); free(t->inS); free(t->v); free(t->P); free(t->cdf);
    free(t->thr); free(t->se_off); free(t->se); free(t->R); free(t->heavy);
    memset(t, 0, sizeof(*t));
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

typedef struct { int64_t v, e; } vedge;
static int cmp_vedge(const void *a, const void *b)
{
    const vedge *x = a, *y = b;
    if (x->v != y->v) return (x->v > y->v) - (x->v < y->v);
    return (x->e > y->e) - (x->e < y->e);
}

/* Sec. 3.1: N^out_S, P_{S,v} (Eq. psv), Pr[A_i] (Eq. pai), beta_0 (Eq. zerop). */
int oo_table_build(const oo_graph *g, const int32_t *seeds, int64_t k, oo_table *t)
{
    memset(t, 0, sizeof(*t));
    if (k <= 0) return OO_EINVAL;
    for (int64_t i = 0; i < k; ++i)
        if (seeds[i] < 0 || seeds[i] >= g->n) return OO_ERANGE;
    int32_t *S = malloc(sizeof(int32_t) * (size_t)k);
    uint8_t *inS = calloc((size_t)g->n, 1);
    if (!S || !inS) { free(S); free(inS); return OO_ENOMEM; }
    memcpy(S, seeds, sizeof(int32_t) * (size_t)k);
    qsort(S, (size_t)k, sizeof(int32_t), cmp_i32);
    int64_t kk = 0;
    for (int64_t i = 0; i < k; ++i)
        if (kk == 0 || S[kk - 1] != S[i]) S[kk++] = S[i];
    for (int64_t i = 0; i < kk; ++i) inS[S[i]] = 1;
    t->k = kk; t->S = S; t->inS = inS;

    int64_t cnt = 0;
    for (int64_t i = 0; i < kk; ++i) {
        int32_t u = S[i];
        for (int64_t e = g->row_ptr[u]; e < g->row_ptr[u + 1]; ++e)
            if (!inS[g->col[e]]) ++cnt;
    }
    vedge *ve = malloc(sizeof(vedge) * (size_t)(cnt ? cnt : 1));
    if (!ve) { oo_table_free(t); return OO_ENOMEM; }
    int64_t c = 0;
    for (int64_t i = 0; i < kk; ++i) {
        int32_t u = S[i];
        for (int64_t e = g->row_ptr[u]; e < g->row_ptr[u + 1]; ++e)
            if (!inS[g->col[e]]) { ve[c].v = g->col[e]; ve[c].e = e; ++c; }
    }
    qsort(ve, (size_t)cnt, sizeof(vedge), cmp_vedge);
    int64_t l = 0;
    for (int64_t i = 0; i < cnt; ++i)
        if (i == 0 || ve[i].v != ve[i - 1].v) ++l;
    t->l = l;
    t->v = malloc(sizeof(int32_t) * (size_t)(l ? l : 1));
    t->P = malloc(sizeof(double) * (size_t)(l ? l : 1));
    t->cdf = malloc(sizeof(double) * (size_t)(l + 1));
    t->thr = malloc(sizeof(uint64_t) * (size_t)(l ? l : 1));
    t->se_off = malloc(sizeof(int64_t) * (size_t)(l + 1));
    t->se = malloc(sizeof(int64_t) * (size_t)(cnt ? cnt : 1));
    if (!t->v || !t->P || !t->cdf || !t->thr || !t->se_off || !t->se) {
        free(ve); oo_table_free(t); return OO_ENOMEM;
    }
    int64_t j = -1;
    for (int64_t i = 0; i < cnt; ++i) {
        if (i == 0 || ve[i].v != ve[i - 1].v) {
            ++j;
            t->v[j] = (int32_t)ve[i].v;
            t->se_off[j] = i;
        }
        t->se[i] = ve[i].e;
    }
    t->se_off[l] = cnt;
    free(ve);
    /* Eq. psv with R2 */
    for (j = 0; j < l; ++j) {
        double prod = 1.0;
        for (int64_t q = t->se_off[j]; q < t->se_off[j + 1]; ++q)
            prod = prod * (1.0 - (double)g->p[t->se[q]]);
        t->P[j] = 1.0 - prod;
        t->thr[j] = coin_threshold(t->P[j]);
    }
    /* Eqs. pai and zerop with R3 */
    double Q = 1.0;
    t->cdf[0] = 0.0;
    for (j = 0; j < l; ++j) {
        double pa = Q * t->P[j];
        t->cdf[j + 1] = t->cdf[j] + pa;
        Q = Q * (1.0 - t->P[j]);
    }
    t->beta0 = t->cdf[l];
    /* R16 */
    t->skip = l >= (g_skip_min_l > SKIP_LMIN_FLOOR ? g_skip_min_l : SKIP_LMIN_FLOOR);
    if (t->skip && g_skip_cost > 0.0) {
        /* the walks' expected draws against the coins' blocks */
        double W = (double)((l + SKIP_SEG - 1) / SKIP_SEG);
        for (j = 0; j < l; ++j)
            if (t->P[j] > 0.0 && t->P[j] < 0.5) W = W + t->P[j];
        t->skip = W * g_skip_cost <= (double)l / 4.0;
    }
    if (t->skip) {
        t->R = malloc(sizeof(double) * (size_t)l);
        t->heavy = malloc(sizeof(int64_t) * (size_t)l);
        if (!t->R || !t->heavy) { oo_table_free(t); return OO_ENOMEM; }
        double R = 1.0;
        for (j = 0; j < l; ++j) {
            if (j % SKIP_SEG == 0) R = 1.0;
            if (t->P[j] >= 0.5) t->heavy[t->nheavy++] = j;
            else if (t->P[j] > 0.0) R = R * (1.0 - t->P[j]);
            t->R[j] = R;
        }
    }
    return OO_OK;
}

/* ------------------------------------------------------------------------ */
/* IICP (Alg. 1)                                                            */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint8_t *vis;     /* n flags, all zero between samples */
    int32_t *queue;   /* n entries */
    uint8_t *live;    /* Stage-1 live flags of the last sample (table size) */
    int64_t nlive;
} oo_scratch;

static int scratch_init(oo_scratch *w, int64_t n)
{
    w->vis = calloc((size_t)n, 1);
    w->queue = malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    w->live = NULL;
    w->nlive = 0;
    if (!w->vis || !w->queue) { free(w->vis); free(w->queue); return OO_ENOMEM; }
    return OO_OK;
}
static void scratch_free(oo_scratch *w) { free(w->vis); free(w->queue); free(w->live); }

/* R6: Alg. 1, Stage 1: the first activated table entry */
static int64_t select_first(const oo_table *t, double U)
{
    double x = U * t->beta0;
    int64_t lo = 0, hi = t->l;       /* find min j with cdf[j+1] > x */
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (t->cdf[mid + 1] > x) hi = mid; else lo = mid + 1;
    }
    if (lo < t->l) return lo;
    for (int64_t j = t->l - 1; j >= 0; --j)
        if (t->cdf[j + 1] > t->cdf[j]) return j;
    return -1;
}

static double uniform53(const uint32_t r[4])
{
    uint64_t a = r[0] >> 5, b = r[1] >> 6;
    return (double)(a * 67108864ull + b) * (1.0 / 9007199254740992.0);
}

static double selection_uniform(uint32_t qid, uint32_t seed, uint32_t stream, uint64_t s)
{
    uint32_t r[4];
    draw(qid, seed, KIND_SELECT, stream, s, 0, r);
    return uniform53(r);
}

static int stage1_coin(uint32_t qid, uint32_t seed, uint32_t stream, uint64_t s,
                       const oo_table *t, int64_t j)
{
    uint32_t r[4];
    draw(qid, seed, KIND_STAGE1, stream, s, (uint64_t)j >> 2, r);
    return (uint64_t)r[j & 3] < t->thr[j];
}

static int edge_coin(uint32_t qid, uint32_t seed, uint32_t stream, uint64_t s,
                     const oo_graph *g, int64_t e)
{
    uint32_t r[4];
    draw(qid, seed, KIND_EDGE, stream, s, (uint64_t)e >> 2, r);
    return (uint64_t)r[e & 3] < coin_threshold((double)g->p[e]);
}

/* Alg. 1, Stage 1 after the selection of entry i: which later entries are
 * live, each with probability P_j (R4, or R16 for long tables).  live[j] is
 * set to 1 for every live j > i (live has l entries, zero on entry for
 * j > i). */
static void stage1_later(const oo_table *t, uint32_t qid, uint32_t seed, uint32_t stream, uint64_t s,
                         int64_t i, uint8_t *live)
{
    if (!t->skip) {
        for (int64_t j = i + 1; j < t->l; ++j)
            if (stage1_coin(qid, seed, stream, s, t, j)) live[j] = 1;
        return;
    }
    /* heavy entries: their own coins */
    for (int64_t h = 0; h < t->nheavy; ++h) {
        int64_t j = t->heavy[h];
        if (j > i && stage1_coin(qid, seed, stream, s, t, j)) live[j] = 1;
    }
    /* light entries: one walk per segment that reaches past i */
    for (int64_t m = (i + 1) / SKIP_SEG; m * SKIP_SEG < t->l; ++m) {
        int64_t a = m * SKIP_SEG, b = a + SKIP_SEG < t->l ? a + SKIP_SEG : t->l;
        int64_t pos = i >= a ? i : a - 1;
        double Rpos = pos >= a ? t->R[pos] : 1.0;
        uint64_t idx = pos >= a ? (uint64_t)pos : (1ull << 40) + (uint64_t)m;
        for (;;) {
            uint32_t r[4];
            draw(qid, seed, KIND_SKIP, stream, s, idx, r);
            double thr = (1.0 - uniform53(r)) * Rpos;
            int64_t lo = pos + 1, hi = b;      /* first j in (pos, b) with R_j < thr */
            while (lo < hi) {
                int64_t mid = lo + (hi - lo) / 2;
                if (t->R[mid] < thr) hi = mid; else lo = mid + 1;
            }
            if (lo >= b) break;
            live[lo] = 1;
            pos = lo;
            Rpos = t->R[lo];
            idx = (uint64_t)lo;
        }
    }
}

/*
 * One IICP sample (Alg. 1).  Returns Y (the outer size).  *E_out receives the
 * number of coins the sample examined in the sense used for GTEPS:
 * (l - i) Stage-1 entries after the selected one (0-based l-1-i) plus the
 * full out-degree of every activated node.  On return, w->queue[0..Y) holds
 * the activated nodes in the order Alg. 1 activates them, *sel the selected
 * 0-based index i.  The visited flags are cleared before returning.
 */
static uint32_t iicp_sample(const oo_graph *g, const oo_table *t, uint32_t qid,
                            uint32_t seed, uint32_t stream, uint64_t s,
                            uint64_t *E_out, int64_t *sel, oo_scratch *w)
{
    const uint8_t *inS = t->inS;
    /* Stage 1: select the first activated entry i */
    int64_t i = select_first(t, selection_uniform(qid, seed, stream, s));
    /* R <- {v_i}, Y = 1, mark v_i (S is marked through inS) */
    int64_t head = 0, tail = 0;
    uint32_t Y = 1;
    uint64_t E = (uint64_t)(t->l - 1 - i);
    w->queue[tail++] = t->v[i];
    w->vis[t->v[i]] = 1;
    /* Stage 1: each later entry j > i live with probability P_j */
    if (w->nlive < t->l) {
        free(w->live);
        w->live = malloc((size_t)t->l);
        if (!w->live) abort();   /* a test tool: fail loudly rather than sample wrongly */
        w->nlive = t->l;
    }
    memset(w->live, 0, (size_t)t->l);
    stage1_later(t, qid, seed, stream, s, i, w->live);
    for (int64_t j = i + 1; j < t->l; ++j) {
        if (w->live[j]) {
            w->queue[tail++] = t->v[j];
            w->vis[t->v[j]] = 1;
            ++Y;
        }
    }
    /* Stage 2: FIFO BFS over unvisited out-neighbours */
    while (head < tail) {
        int32_t u = w->queue[head++];
        int64_t b = g->row_ptr[u], e1 = g->row_ptr[u + 1];
        E += (uint64_t)(e1 - b);
        for (int64_t e = b; e < e1; ++e) {
            int32_t v = g->col[e];
            if (inS[v] || w->vis[v]) continue;
            if (edge_coin(qid, seed, stream, s, g, e)) {
                w->vis[v] = 1;
                w->queue[tail++] = v;
                ++Y;
            }
        }
    }
    for (int64_t h = 0; h < tail; ++h) w->vis[w->queue[h]] = 0;
    if (E_out) *E_out = E;
    if (sel) *sel = i;
    return Y;
}

/* ------------------------------------------------------------------------ */
/* Fixed-count sampling, split over threads by contiguous sample ranges.    */
/* The sums are integers, so they do not depend on the number of threads.   */
/* ------------------------------------------------------------------------ */
typedef struct {
    const oo_graph *g; const oo_table *t;
    uint32_t qid, seed, stream;
    uint64_t first, count;
    uint32_t *y_out; uint64_t *e_out;
    uint64_t sumY, sumE;
    int rc;
} fixed_job;

static void *fixed_worker(void *arg)
{
    fixed_job *j = arg;
    oo_scratch w;
    if (scratch_init(&w, j->g->n)) { j->rc = OO_ENOMEM; return NULL; }
    uint64_t sy = 0, se = 0;
    for (uint64_t q = 0; q < j->count; ++q) {
        uint64_t E;
        uint32_t Y = iicp_sample(j->g, j->t, j->qid, j->seed, j->stream, j->first + q, &E, NULL, &w);
        if (j->y_out) j->y_out[q] = Y;
        if (j->e_out) j->e_out[q] = E;
        sy += Y;
        se += E;
    }
    scratch_free(&w);
    j->sumY = sy;
    j->sumE = se;
    j->rc = OO_OK;
    return NULL;
}

/* Oracle entry: count samples of stream `stream` starting at index `first`. */
int oo_sample_fixed(int64_t n, int64_t m, const int64_t *row_ptr, const int32_t *col,
                    const float *p, const int32_t *seeds, int64_t k, uint32_t qid,
                    uint32_t seed, uint32_t stream, uint64_t first, uint64_t count,
                    uint32_t *y_out, uint64_t *e_out, uint64_t *sums /* [sumY, sumE] */,
                    double *beta0_out, int nthreads)
{
    oo_graph g = {n, m, row_ptr, col, p};
    oo_table t;
    int rc = oo_table_build(&g, seeds, k, &t);
    if (rc) return rc;
    if (beta0_out) *beta0_out = t.beta0;
    sums[0] = sums[1] = 0;
    if (t.beta0 == 0.0 || count == 0) { oo_table_free(&t); return OO_OK; }
    if (nthreads < 1) nthreads = 1;
    if ((uint64_t)nthreads > count) nthreads = (int)count;
    fixed_job *jobs = calloc((size_t)nthreads, sizeof(fixed_job));
    pthread_t *th = calloc((size_t)nthreads, sizeof(pthread_t));
    uint64_t per = count / (uint64_t)nthreads, rem = count % (uint64_t)nthreads, off = 0;
    for (int i = 0; i < nthreads; ++i) {
        uint64_t c = per + ((uint64_t)i < rem ? 1 : 0);
        jobs[i] = (fixed_job){&g, &t, qid, seed, stream, first + off, c,
                              y_out ? y_out + off : NULL, e_out ? e_out + off : NULL, 0, 0, 0};
        off += c;
        if (nthreads == 1) fixed_worker(&jobs[i]);
        else pthread_create(&th[i], NULL, fixed_worker, &jobs[i]);
    }
    rc = OO_OK;
    for (int i = 0; i < nthreads; ++i) {
        if (nthreads > 1) pthread_join(th[i], NULL);
        if (jobs[i].rc) rc = jobs[i].rc;
        sums[0] += jobs[i].sumY;
        sums[1] += jobs[i].sumE;
    }
    free(jobs); free(th);
    oo_table_free(&t);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Classic IC Monte-Carlo sample M^(S) (Sec. 2.3, Lemma 3)                  */
/* ------------------------------------------------------------------------ */
/*
 * One plain IC cascade from S: every node of S is active from the start, and
 * a FIFO BFS examines each out-edge (u, v) of each active node once, with
 * its coin (R4/R5: the same edge coin as an IICP sample with this key uses
 * in Stage 2).  Returns M - |S|, the number of nodes outside S that end
 * active (zero allowed); *E_out receives the out-degree summed over every
 * node expanded, S included.  The visited flags are cleared before
 * returning.
 */
static uint32_t mc_sample(const oo_graph *g, const oo_table *t, uint32_t qid, uint32_t seed,
                          uint32_t stream, uint64_t s, uint64_t *E_out, oo_scratch *w)
{
    int64_t head = 0, tail = 0;
    uint64_t E = 0;
    for (int64_t i = 0; i < t->k; ++i) {
        w->queue[tail++] = t->S[i];
        w->vis[t->S[i]] = 1;
    }
    while (head < tail) {
        int32_t u = w->queue[head++];
        int64_t b = g->row_ptr[u], e1 = g->row_ptr[u + 1];
        E += (uint64_t)(e1 - b);
        for (int64_t e = b; e < e1; ++e) {
            int32_t v = g->col[e];
            if (w->vis[v]) continue;
            if (edge_coin(qid, seed, stream, s, g, e)) {
                w->vis[v] = 1;
                w->queue[tail++] = v;
            }
        }
    }
    for (int64_t h = 0; h < tail; ++h) w->vis[w->queue[h]] = 0;
    if (E_out) *E_out = E;
    return (uint32_t)(tail - t->k);
}

typedef struct {
    const oo_graph *g; const oo_table *t;
    uint32_t qid, seed, stream;
    uint64_t first, count;
    uint32_t *y_out; uint64_t *e_out;
    uint64_t sumY, sumE;
    int rc;
} mc_job;

static void *mc_worker(void *arg)
{
    mc_job *j = arg;
    oo_scratch w;
    if (scratch_init(&w, j->g->n)) { j->rc = OO_ENOMEM; return NULL; }
    uint64_t sy = 0, se = 0;
    for (uint64_t q = 0; q < j->count; ++q) {
        uint64_t E;
        uint32_t Y = mc_sample(j->g, j->t, j->qid, j->seed, j->stream, j->first + q, &E, &w);
        if (j->y_out) j->y_out[q] = Y;
        if (j->e_out) j->e_out[q] = E;
        sy += Y;
        se += E;
    }
    scratch_free(&w);
    j->sumY = sy;
    j->sumE = se;
    j->rc = OO_OK;
    return NULL;
}

/* Oracle entry: `count` classic Monte-Carlo samples M^(S) - |S| of stream
 * `stream` from index `first`; sums = [sum of M - |S|, sum of E].  The mean of
 * M over N samples is the MC_N estimate of I(S) (Sec. 6.1). */
int oo_mc_fixed(int64_t n, int64_t m, const int64_t *row_ptr, const int32_t *col,
                const float *p, const int32_t *seeds, int64_t k, uint32_t qid,
                uint32_t seed, uint32_t stream, uint64_t first, uint64_t count,
                uint32_t *y_out, uint64_t *e_out, uint64_t *sums, int64_t *k_out, int nthreads)
{
    oo_graph g = {n, m, row_ptr, col, p};
    oo_table t;
    int rc = oo_table_build(&g, seeds, k, &t);
    if (rc) return rc;
    if (k_out) *k_out = t.k;
    sums[0] = sums[1] = 0;
    if (count == 0) { oo_table_free(&t); return OO_OK; }
    if (nthreads < 1) nthreads = 1;
    if ((uint64_t)nthreads > count) nthreads = (int)count;
    mc_job *jobs = calloc((size_t)nthreads, sizeof(mc_job));
    pthread_t *th = calloc((size_t)nthreads, sizeof(pthread_t));
    uint64_t per = count / (uint64_t)nthreads, rem = count % (uint64_t)nthreads, off = 0;
    for (int i = 0; i < nthreads; ++i) {
        uint64_t c = per + ((uint64_t)i < rem ? 1 : 0);
        jobs[i] = (mc_job){&g, &t, qid, seed, stream, first + off, c,
                           y_out ? y_out + off : NULL, e_out ? e_out + off : NULL, 0, 0, 0};
        off += c;
        if (nthreads == 1) mc_worker(&jobs[i]);
        else pthread_create(&th[i], NULL, mc_worker, &jobs[i]);
    }
    rc = OO_OK;
    for (int i = 0; i < nthreads; ++i) {
        if (nthreads > 1) pthread_join(th[i], NULL);
        if (jobs[i].rc) rc = jobs[i].rc;
        sums[0] += jobs[i].sumY;
        sums[1] += jobs[i].sumE;
    }
    free(jobs); free(th);
    oo_table_free(&t);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* LT model cascades (R17)                                                   */
/* ------------------------------------------------------------------------ */
/* Per-edge selection intervals [lo[e], hi[e]) of the 2^32 words (R17). */
static int lt_intervals(const oo_graph *g, uint64_t *lo, uint64_t *hi)
{
    int64_t n = g->n, m = g->m;
    int64_t *cnt = calloc((size_t)n + 1, sizeof(int64_t));
    int64_t *ord = malloc(sizeof(int64_t) * (size_t)(m ? m : 1));
    if (!cnt || !ord) { free(cnt); free(ord); return OO_ENOMEM; }
    for (int64_t e = 0; e < m; ++e) cnt[g->col[e] + 1]++;
    for (int64_t v = 0; v < n; ++v) cnt[v + 1] += cnt[v];
    int64_t *pos = malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
    if (!pos) { free(cnt); free(ord); return OO_ENOMEM; }
    for (int64_t v = 0; v < n; ++v) pos[v] = cnt[v];
    for (int64_t e = 0; e < m; ++e) ord[pos[g->col[e]]++] = e;   /* ascending e per target */
    int rc = OO_OK;
    for (int64_t v = 0; v < n && rc == OO_OK; ++v) {
        double c = 0.0;
        uint64_t prev = 0;
        for (int64_t q = cnt[v]; q < cnt[v + 1]; ++q) {
            int64_t e = ord[q];
            c = c + (double)g->p[e];
            if (c > 1.0 + 1e-6) { rc = OO_EINVAL; break; }
            uint64_t t = (uint64_t)((c < 1.0 ? c : 1.0) * 4294967296.0);
            lo[e] = prev;
            hi[e] = t;
            prev = t;
        }
    }
    free(cnt); free(ord); free(pos);
    return rc;
}

static uint32_t lt_word(uint32_t qid, uint32_t seed, uint32_t stream, uint64_t s, int32_t v)
{
    uint32_t r[4];
    draw(qid, seed, KIND_LT, stream, s, (uint64_t)v >> 2, r);
    return r[v & 3];
}

/* One LT cascade from S (R17): returns Y, the nodes outside S reached;
 * *E_out = out-degree summed over the nodes expanded, S included. */
static uint32_t lt_sample(const oo_graph *g, const oo_table *t, const uint64_t *lo, const uint64_t *hi,
                          uint32_t qid, uint32_t seed, uint32_t stream, uint64_t s, uint64_t *E_out,
                          oo_scratch *w)
{
    int64_t head = 0, tail = 0;
    uint64_t E = 0;
    for (int64_t i = 0; i < t->k; ++i) {
        w->queue[tail++] = t->S[i];
        w->vis[t->S[i]] = 1;
    }
    while (head < tail) {
        int32_t u = w->queue[head++];
        int64_t b = g->row_ptr[u], e1 = g->row_ptr[u + 1];
        E += (uint64_t)(e1 - b);
        for (int64_t e = b; e < e1; ++e) {
            int32_t v = g->col[e];
            if (w->vis[v]) continue;
            uint64_t W = lt_word(qid, seed, stream, s, v);
            if (lo[e] <= W && W < hi[e]) {
                w->vis[v] = 1;
                w->queue[tail++] = v;
            }
        }
    }
    for (int64_t h = 0; h < tail; ++h) w->vis[w->queue[h]] = 0;
    if (E_out) *E_out = E;
    return (uint32_t)(tail - t->k);
}

typedef struct {
    const oo_graph *g; const oo_table *t; const uint64_t *lo, *hi;
    uint32_t qid, seed, stream;
    uint64_t first, count;
    uint32_t *y_out; uint64_t *e_out;
    uint64_t sumY, sumE;
    int rc;
} lt_job;

static void *lt_worker(void *arg)
{
    lt_job *j = arg;
    oo_scratch w;
    if (scratch_init(&w, j->g->n)) { j->rc = OO_ENOMEM; return NULL; }
    uint64_t sy = 0, se = 0;
    for (uint64_t q = 0; q < j->count; ++q) {
        uint64_t E;
        uint32_t Y = lt_sample(j->g, j->t, j->lo, j->hi, j->qid, j->seed, j->stream, j->first + q, &E, &w);
        if (j->y_out) j->y_out[q] = Y;
        if (j->e_out) j->e_out[q] = E;
        sy += Y;
        se += E;
    }
    scratch_free(&w);
    j->sumY = sy;
    j->sumE = se;
    j->rc = OO_OK;
    return NULL;
}

/* Oracle entry: `count` LT cascades (R17) of stream `stream` from index
 * `first`: per-sample Y = |cascade| - |S| and E; sums = [sum Y, sum E]. */
int oo_lt_fixed(int64_t n, int64_t m, const int64_t *row_ptr, const int32_t *col,
                const float *p, const int32_t *seeds, int64_t k, uint32_t qid,
                uint32_t seed, uint32_t stream, uint64_t first, uint64_t count,
                uint32_t *y_out, uint64_t *e_out, uint64_t *sums, int64_t *k_out, int nthreads)
{
    oo_graph g = {n, m, row_ptr, col, p};
    oo_table t;
    int rc = oo_table_build(&g, seeds, k, &t);
    if (rc) return rc;
    if (k_out) *k_out = t.k;
    sums[0] = sums[1] = 0;
    uint64_t *lo = malloc(sizeof(uint64_t) * (size_t)(m ? m : 1));
    uint64_t *hi = malloc(sizeof(uint64_t) * (size_t)(m ? m : 1));
    if (!lo || !hi) { free(lo); free(hi); oo_table_free(&t); return OO_ENOMEM; }
    rc = lt_intervals(&g, lo, hi);
    if (rc || count == 0) { free(lo); free(hi); oo_table_free(&t); return rc; }
    if (nthreads < 1) nthreads = 1;
    if ((uint64_t)nthreads > count) nthreads = (int)count;
    lt_job *jobs = calloc((size_t)nthreads, sizeof(lt_job));
    pthread_t *th = calloc((size_t)nthreads, sizeof(pthread_t));
    uint64_t per = count / (uint64_t)nthreads, rem = count % (uint64_t)nthreads, off = 0;
    for (int i = 0; i < nthreads; ++i) {
        uint64_t c = per + ((uint64_t)i < rem ? 1 : 0);
        jobs[i] = (lt_job){&g, &t, lo, hi, qid, seed, stream, first + off, c,
                           y_out ? y_out + off : NULL, e_out ? e_out + off : NULL, 0, 0, 0};
        off += c;
        if (nthreads == 1) lt_worker(&jobs[i]);
        else pthread_create(&th[i], NULL, lt_worker, &jobs[i]);
    }
    rc = OO_OK;
    for (int i = 0; i < nthreads; ++i) {
        if (nthreads > 1) pthread_join(th[i], NULL);
        if (jobs[i].rc) rc = jobs[i].rc;
        sums[0] += jobs[i].sumY;
        sums[1] += jobs[i].sumE;
    }
    free(jobs); free(th); free(lo); free(hi);
    oo_table_free(&t);
    return rc;
}

/* Stage-1 table export for tests: copies l entries into caller arrays (any may
 * be NULL), returns l through *l_out and beta_0 through *beta0. */
int oo_stage1(int64_t n, int64_t m, const int64_t *row_ptr, const int32_t *col, const float *p,
              const int32_t *seeds, int64_t k, int64_t cap, int64_t *l_out, double *beta0,
              int32_t *v, double *P, double *cdf, uint64_t *thr, int64_t *k_out)
{
    oo_graph g = {n, m, row_ptr, col, p};
    oo_table t;
    int rc = oo_table_build(&g, seeds, k, &t);
    if (rc) return rc;
    *l_out = t.l;
    *beta0 = t.beta0;
    if (k_out) *k_out = t.k;
    if (t.l <= cap) {
        for (int64_t j = 0; j < t.l; ++j) {
            if (v) v[j] = t.v[j];
            if (P) P[j] = t.P[j];
            if (thr) thr[j] = t.thr[j];
        }
        if (cdf) for (int64_t j = 0; j <= t.l; ++j) cdf[j] = t.cdf[j];
    }
    oo_table_free(&t);
    return OO_OK;
}

/* Per-sample selection index (for distribution tests of Stage 1). */
int oo_selection(int64_t n, int64_t m, const int64_t *row_ptr, const int32_t *col, const float *p,
                 const int32_t *seeds, int64_t k, uint32_t qid, uint32_t seed, uint32_t stream,
                 uint64_t first, uint64_t count, int64_t *sel_out)
{
    oo_graph g = {n, m, row_ptr, col, p};
    oo_table t;
    int rc = oo_table_build(&g, seeds, k, &t);
    if (rc) return rc;
    for (uint64_t q = 0; q < count; ++q)
        sel_out[q] = t.beta0 > 0.0 ? select_first(&t, selection_uniform(qid, seed, stream, first + q)) : -1;
    oo_table_free(&t);
    return OO_OK;
}

/* ------------------------------------------------------------------------ */
/* GSRA (Alg. 2) and RSA (Alg. 3) over integer streams X = scale*Y + offset */
/* ------------------------------------------------------------------------ */
typedef uint32_t (*oo_next_fn)(void *ctx, uint32_t stream, uint64_t index);

typedef struct {
    double mu;          /* returned estimate of E[X] */
    double mu1;         /* step-1 rough estimate (RSA) */
    double ups;         /* Upsilon(eps, delta) of the final call */
    double ups1;        /* Upsilon of the step-1 GSRA */
    double ups2;        /* Upsilon_2 */
    uint64_t T1, h1;    /* step-1 sample count and sum of Y */
    uint64_t nsigma;
    uint64_t D_lo, D_hi; /* sum of squared paired differences of Y' (128-bit) */
    uint64_t T, hT;     /* step-3 sample count and sum of Y over X_1..X_T */
    uint64_t drawn_x, drawn_xp; /* samples consumed from X and X' */
    int32_t gsra_only;  /* eps >= 1/4 */
    int32_t early;      /* the (first) GSRA returned a without sampling */
} oo_rsa_result;

/* Upsilon of Alg. 2, with c(eps', delta) from Table 1 (R8). */
static double upsilon(double eps, double delta, double a, double b)
{
    double L = log(2.0 / delta);
    double epsp = eps * (1.0 - (eps * b) / ((2.0 + (2.0 / 3.0) * eps) * L * (b - a)));
    double c = (2.0 + (2.0 / 3.0) * epsp) * L / (epsp * epsp);
    return (1.0 + eps) * c * (b - a);
}

static double sumx(double scale, double offset, uint64_t h, uint64_t T)
{
    return scale * (double)h + offset * (double)T;   /* R11 */
}

/* Alg. 2.  Draws X_1, X_2, ... from stream 0 starting at index 0. */
static void gsra(oo_next_fn next, void *ctx, double eps, double delta, double a, double b,
                 double scale, double offset, double *mu, uint64_t *T_out, uint64_t *h_out,
                 double *ups_out, int32_t *early)
{
    if (b - a < eps * b) {           /* the early exit of Alg. 2 */
        *mu = a; *T_out = 0; *h_out = 0; *ups_out = 0.0; *early = 1;
        return;
    }
    double ups = upsilon(eps, delta, a, b);   /* the threshold */
    uint64_t h = 0, T = 0;
    while (sumx(scale, offset, h, T) < ups) { /* draw until the sum reaches it */
        h += next(ctx, 0, T);
        ++T;
    }
    *mu = sumx(scale, offset, h, T) / (double)T;   /* R9 */
    *T_out = T; *h_out = h; *ups_out = ups; *early = 0;
}

/* Alg. 3, step 2: the number of pairs of X' from step 1's estimate mu' (R10). */
static int rsa_nsigma(double eps, double delta, double a, double b, double mu1,
                      double *ups_out, double *ups2_out, uint64_t *nsigma)
{
    double se = sqrt(eps);
    double L = log(2.0 / delta);
    double ups = upsilon(eps, delta, a, b);
    double ups2 = 2.0 * (1.0 + se) / (1.0 - se) * (1.0 + log(1.5) / L) * ups;
    double ns = ceil(ups2 * eps / mu1);
    if (!(ns < 4.0e18)) return OO_ERANGE;
    *nsigma = ns < 1.0 ? 1 : (uint64_t)ns;
    if (ups_out) *ups_out = ups;
    *ups2_out = ups2;
    return OO_OK;
}

/* Alg. 3, step 3: the number of samples T from mu', the 128-bit sum D of
 * squared paired differences of the integer stream Y', N_sigma and Upsilon_2
 * (R10, R11: the differences of X' = scale * Y' + offset are scale times
 * those of Y'). */
static int rsa_steps3(double eps, double a, double b, double scale, double mu1, double ups2,
                      uint64_t nsigma, oo_u128 D, uint64_t *T)
{
    double Delta = scale * scale * (double)D / 2.0;
    double rho1 = Delta / (double)nsigma;
    double rho2 = eps * mu1 * (b - a);
    double rho = rho1 > rho2 ? rho1 : rho2;
    double tt = ceil(ups2 * rho / (mu1 * mu1 * (b - a)));
    if (!(tt < 4.0e18)) return OO_ERANGE;
    *T = tt < 1.0 ? 1 : (uint64_t)tt;
    return OO_OK;
}

/* Alg. 3 (RSA) with readings R10, R11. */
int oo_rsa(oo_next_fn next, void *ctx, double eps, double delta, double a, double b,
           double scale, double offset, oo_rsa_result *r)
{
    memset(r, 0, sizeof(*r));
    if (!(eps > 0.0 && eps < 1.0) || !(delta > 0.0 && delta < 0.5) || !(b > a) || !(a >= 0.0))
        return OO_EINVAL;
    if (eps >= 0.25) {                                   /* Alg. 3 reduces to GSRA */
        r->gsra_only = 1;
        gsra(next, ctx, eps, delta, a, b, scale, offset, &r->mu, &r->T1, &r->h1, &r->ups1, &r->early);
        r->T = r->T1; r->hT = r->h1; r->drawn_x = r->T1;
        return OO_OK;
    }
    double se = sqrt(eps);
    /* step 1 */
    gsra(next, ctx, se, delta / 3.0, a, b, scale, offset, &r->mu1, &r->T1, &r->h1, &r->ups1, &r->early);
    /* step 2 */
    int rc = rsa_nsigma(eps, delta, a, b, r->mu1, &r->ups, &r->ups2, &r->nsigma);
    if (rc) return rc;
    oo_u128 D = 0;
    for (uint64_t i = 0; i < r->nsigma; ++i) {
        uint32_t y0 = next(ctx, 1, 2 * i), y1 = next(ctx, 1, 2 * i + 1);
        uint64_t d = y0 > y1 ? (uint64_t)(y0 - y1) : (uint64_t)(y1 - y0);
        D += (oo_u128)(d * d);
    }
    r->D_lo = (uint64_t)D;
    r->D_hi = (uint64_t)(D >> 64);
    /* step 3 */
    rc = rsa_steps3(eps, a, b, scale, r->mu1, r->ups2, r->nsigma, D, &r->T);
    if (rc) return rc;
    uint64_t h = 0;
    for (uint64_t i = 0; i < r->T; ++i) h += next(ctx, 0, i);
    r->hT = h;
    r->mu = sumx(scale, offset, h, r->T) / (double)r->T;
    r->drawn_x = r->T > r->T1 ? r->T : r->T1;
    r->drawn_xp = 2 * r->nsigma;
    return OO_OK;
}

/*
 * The decisions of RSA (Alg. 3, eps < 1/4) as functions of the integer sums
 * it observes, through the same code as oo_rsa: for each of the `count`
 * cases, step 1 ended after T1[i] samples whose Y summed to h1[i] (mu' =
 * (scale * h1 + offset * T1) / T1, R11), giving nsigma_out[i]; if D_lo is not
 * NULL, step 2's sum of squared paired differences of Y' was D_hi[i] * 2^64 +
 * D_lo[i], giving T_out[i].  thr_out (may be NULL) receives the step-1 GSRA
 * threshold, Upsilon(eps, delta) and Upsilon_2.  For tests that evaluate
 * Theorem 4 exactly.
 */
int oo_rsa_plan(double eps, double delta, double a, double b, double scale, double offset,
                uint64_t count, const uint64_t *h1, const uint64_t *T1, const uint64_t *D_lo,
                const uint64_t *D_hi, uint64_t *nsigma_out, uint64_t *T_out, double *thr_out)
{
    if (!(eps > 0.0 && eps < 0.25) || !(delta > 0.0 && delta < 0.5) || !(b > a) || !(a >= 0.0))
        return OO_EINVAL;
    double se = sqrt(eps);
    if (thr_out) {
        thr_out[0] = upsilon(se, delta / 3.0, a, b);
        thr_out[1] = upsilon(eps, delta, a, b);
    }
    for (uint64_t i = 0; i < count; ++i) {
        if (T1[i] == 0) return OO_EINVAL;
        double mu1 = sumx(scale, offset, h1[i], T1[i]) / (double)T1[i];
        double ups, ups2;
        int rc = rsa_nsigma(eps, delta, a, b, mu1, &ups, &ups2, &nsigma_out[i]);
        if (rc) return rc;
        if (thr_out) thr_out[2] = ups2;
        if (D_lo) {
            oo_u128 D = ((oo_u128)D_hi[i] << 64) | (oo_u128)D_lo[i];
            rc = rsa_steps3(eps, a, b, scale, mu1, ups2, nsigma_out[i], D, &T_out[i]);
            if (rc) return rc;
        }
    }
    return OO_OK;
}

/* Stream source backed by two caller arrays (for tests of the stopping rules). */
/* Array streams for tests.  Past its end a stream is marked overrun (the
 * call then reports OO_ERANGE) and yields UINT32_MAX, so that every
 * stopping loop still ends: a stream of zeros would never reach a threshold. */
typedef struct { const uint32_t *x; uint64_t nx; const uint32_t *xp; uint64_t nxp; int overrun; } arr_ctx;
static uint32_t arr_next(void *c, uint32_t stream, uint64_t i)
{
    arr_ctx *a = c;
    if (stream == 0) { if (i < a->nx) return a->x[i]; a->overrun = 1; return UINT32_MAX; }
    if (i < a->nxp) return a->xp[i];
    a->overrun = 1;
    return UINT32_MAX;
}

int oo_rsa_arrays(const uint32_t *x, uint64_t nx, const uint32_t *xp, uint64_t nxp,
                  double eps, double delta, double a, double b, double scale, double offset,
                  oo_rsa_result *r)
{
    arr_ctx c = {x, nx, xp, nxp, 0};
    int rc = oo_rsa(arr_next, &c, eps, delta, a, b, scale, offset, r);
    if (rc) return rc;
    return c.overrun ? OO_ERANGE : OO_OK;
}

/* GSRA alone over an array stream (Alg. 2), for tests. */
int oo_gsra_array(const uint32_t *x, uint64_t nx, double eps, double delta, double a, double b,
                  double scale, double offset, double *mu, uint64_t *T, uint64_t *h, double *ups)
{
    arr_ctx c = {x, nx, NULL, 0, 0};
    int32_t early;
    if (!(eps > 0.0 && eps < 1.0) || !(delta > 0.0 && delta < 1.0) || !(b > a)) return OO_EINVAL;
    gsra(arr_next, &c, eps, delta, a, b, scale, offset, mu, T, h, ups, &early);
    return c.overrun ? OO_ERANGE : OO_OK;
}

/* ------------------------------------------------------------------------ */
/* SOIEA (Alg. 4) and SIEA (Alg. 5) with IICP streams                        */
/* ------------------------------------------------------------------------ */
typedef struct {
    const oo_graph *g; const oo_table *t; uint32_t qid, seed; oo_scratch w;
    uint64_t sumE;
} iicp_ctx;

static uint32_t iicp_next(void *c, uint32_t stream, uint64_t index)
{
    iicp_ctx *x = c;
    uint64_t E;
    uint32_t y = iicp_sample(x->g, x->t, x->qid, x->seed, stream, index, &E, NULL, &x->w);
    x->sumE += E;
    return y;
}

/* mode 0 = SOIEA (X = Y, a = 1, b = n-|S|), 1 = SIEA (X = Z of Eq. z_s). */
int oo_estimate(int64_t n, int64_t m, const int64_t *row_ptr, const int32_t *col, const float *p,
                const int32_t *seeds, int64_t k, double eps, double delta, int mode,
                uint32_t qid, uint32_t seed, double *oi, double *is, double *beta0,
                int64_t *k_out, oo_rsa_result *r)
{
    oo_graph g = {n, m, row_ptr, col, p};
    oo_table t;
    memset(r, 0, sizeof(*r));
    if (!(eps > 0.0 && eps < 1.0) || !(delta > 0.0 && delta < 0.5) || (mode != 0 && mode != 1))
        return OO_EINVAL;
    int rc = oo_table_build(&g, seeds, k, &t);
    if (rc) return rc;
    *beta0 = t.beta0;
    *k_out = t.k;
    double kd = (double)t.k;
    if (t.beta0 == 0.0) {            /* R12 */
        *oi = 0.0; *is = kd;
        oo_table_free(&t);
        return OO_OK;
    }
    double nk = (double)(n - t.k);
    double a, b, scale, offset;
    if (mode == 0) { a = 1.0; b = nk; scale = 1.0; offset = 0.0; }
    else { a = kd + t.beta0; b = kd + t.beta0 * nk; scale = t.beta0; offset = kd; }
    iicp_ctx c = {&g, &t, qid, seed, {0, 0, 0, 0}, 0};
    if (scratch_init(&c.w, n)) { oo_table_free(&t); return OO_ENOMEM; }
    if (!(b > a)) {
        /* n-|S| = 1 (SOIEA) or beta_0 (n-|S|-1) = 0: Y is always 1 (Lemma 2) */
        r->mu = a;
        r->early = 1;
    } else {
        rc = oo_rsa(iicp_next, &c, eps, delta, a, b, scale, offset, r);
    }
    scratch_free(&c.w);
    if (rc == OO_OK) {
        if (mode == 0) { *oi = t.beta0 * r->mu; *is = *oi + kd; }   /* Alg. 4's output */
        else { *is = r->mu; *oi = *is - kd; }                        /* Alg. 5's output */
    }
    oo_table_free(&t);
    return rc;
}

/* SIEA_LT (R17): RSA (Alg. 3) on X = |S| + Y with Y from LT cascades,
 * [a, b] = [|S|, n].  IS = the RSA estimate, OI = IS - |S|. */
typedef struct {
    const oo_graph *g; const oo_table *t; const uint64_t *lo, *hi; uint32_t qid, seed; oo_scratch w;
} lt_ctx;

static uint32_t lt_next(void *c, uint32_t stream, uint64_t index)
{
    lt_ctx *x = c;
    return lt_sample(x->g, x->t, x->lo, x->hi, x->qid, x->seed, stream, index, NULL, &x->w);
}

int oo_estimate_lt(int64_t n, int64_t m, const int64_t *row_ptr, const int32_t *col, const float *p,
                   const int32_t *seeds, int64_t k, double eps, double delta, uint32_t qid, uint32_t seed,
                   double *oi, double *is, int64_t *k_out, oo_rsa_result *r)
{
    oo_graph g = {n, m, row_ptr, col, p};
    oo_table t;
    memset(r, 0, sizeof(*r));
    if (!(eps > 0.0 && eps < 1.0) || !(delta > 0.0 && delta < 0.5)) return OO_EINVAL;
    int rc = oo_table_build(&g, seeds, k, &t);
    if (rc) return rc;
    *k_out = t.k;
    double kd = (double)t.k;
    if (t.beta0 == 0.0 || t.k >= n) {   /* no edge leaves S: the cascade is S */
        *oi = 0.0; *is = kd;
        oo_table_free(&t);
        return OO_OK;
    }
    uint64_t *lo = malloc(sizeof(uint64_t) * (size_t)(m ? m : 1));
    uint64_t *hi = malloc(sizeof(uint64_t) * (size_t)(m ? m : 1));
    if (!lo || !hi) { free(lo); free(hi); oo_table_free(&t); return OO_ENOMEM; }
    rc = lt_intervals(&g, lo, hi);
    if (rc) { free(lo); free(hi); oo_table_free(&t); return rc; }
    lt_ctx c;
    c.g = &g; c.t = &t; c.lo = lo; c.hi = hi; c.qid = qid; c.seed = seed;
    if (scratch_init(&c.w, n)) { free(lo); free(hi); oo_table_free(&t); return OO_ENOMEM; }
    rc = oo_rsa(lt_next, &c, eps, delta, kd, (double)n, 1.0, kd, r);
    scratch_free(&c.w);
    free(lo); free(hi);
    if (rc == OO_OK) { *is = r->mu; *oi = *is - kd; }
    oo_table_free(&t);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Exact enumeration over all 2^m live-edge graphs (Sec. 2)                 */
/* ------------------------------------------------------------------------ */
/*
 * ext   : Ext(S) = sum_g |r_g(S) \ S| Pr[g]
 * dist  : n+1 entries, dist[y] = Pr[|r_g(S) \ S| = y]
 * grad  : m entries (or NULL), d Ext / d p_e.  Ext is multilinear in the
 *         edge probabilities, so the derivative is the sum over graphs of
 *         (+1 if e live, -1 if not) * |r_g(S)\S| * prod_{f != e} Pr[f's state].
 * Requires n <= 64 and m <= 30.
 */
int oo_exact(int64_t n, int64_t m, const int64_t *row_ptr, const int32_t *col, const float *p,
             const int32_t *seeds, int64_t k, double *ext, double *dist, double *grad)
{
    if (n > 64 || m > 30 || n <= 0) return OO_EINVAL;
    uint64_t Smask = 0;
    for (int64_t i = 0; i < k; ++i) {
        if (seeds[i] < 0 || seeds[i] >= n) return OO_ERANGE;
        Smask |= 1ull << seeds[i];
    }
    int ks = __builtin_popcountll(Smask);
    int32_t src[30], dst[30];
    double pe[30];
    for (int64_t u = 0; u < n; ++u)
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            src[e] = (int32_t)u; dst[e] = col[e]; pe[e] = (double)p[e];
        }
    double E = 0.0;
    for (int64_t y = 0; y <= n; ++y) dist[y] = 0.0;
    if (grad) for (int64_t e = 0; e < m; ++e) grad[e] = 0.0;
    double f[30], pre[31], suf[31];
    uint64_t total = 1ull << m;
    for (uint64_t mask = 0; mask < total; ++mask) {
        uint64_t adj[64];
        for (int64_t u = 0; u < n; ++u) adj[u] = 0;
        for (int64_t e = 0; e < m; ++e) {
            int live = (int)((mask >> e) & 1);
            f[e] = live ? pe[e] : 1.0 - pe[e];
            if (live) adj[src[e]] |= 1ull << dst[e];
        }
        uint64_t R = Smask, fr = Smask;
        while (fr) {
            uint64_t nx = 0, x = fr;
            while (x) {
                int u = __builtin_ctzll(x);
                x &= x - 1;
                nx |= adj[u];
            }
            nx &= ~R;
            R |= nx;
            fr = nx;
        }
        int y = __builtin_popcountll(R) - ks;
        pre[0] = 1.0;
        for (int64_t e = 0; e < m; ++e) pre[e + 1] = pre[e] * f[e];
        double pr = pre[m];
        dist[y] += pr;
        E += pr * (double)y;
        if (grad && y > 0) {
            suf[m] = 1.0;
            for (int64_t e = m - 1; e >= 0; --e) suf[e] = suf[e + 1] * f[e];
            for (int64_t e = 0; e < m; ++e) {
                double w = pre[e] * suf[e + 1] * (double)y;
                grad[e] += ((mask >> e) & 1) ? w : -w;
            }
        }
    }
    *ext = E;
    return OO_OK;
}

/* ------------------------------------------------------------------------ */
/* Score-function gradient of the fixed-count estimate (fp64)               */
/* ------------------------------------------------------------------------ */
/*
 * The paper gives no gradient.  This follows the likelihood-ratio identity
 * for the IICP importance distribution: with the Stage-1 node coins x_j of
 * all l entries and the coins of every out-edge (u, v), v not in S, of every
 * activated node u revealed, the leaf probability is
 *   P(leaf) = prod_j P_j^{x_j} (1-P_j)^{1-x_j} * prod_{revealed e} p_e^{x_e} (1-p_e)^{1-x_e},
 * IICP draws leaves with probability P(leaf)/beta_0 (Lemma 2's proof), so
 *   d Ext / d p_e = beta_0 * E[ Y * d log P(leaf) / d p_e ].
 * Per sample s the score of edge e is:
 *   Stage-2 edge (u activated, u, v not in S): x_e ? 1/p_e : -1/(1-p_e);
 *   S-edge (u in S) into table entry j: x_j = [j == i] or (j > i and coin j
 *     live), x_j = 0 for j < i;  x_j ? prod_{f != e}(1-p_f) / P_j : -1/(1-p_e);
 *   every other edge: 0.
 * The identity needs 0 < p_e < 1 for every edge with a nonzero score: at
 * p_e = 0 or 1 one coin outcome has probability zero, its branch never
 * appears in the samples, and the estimate is then not the derivative.
 * Outputs acc[e] = sum_s Y_s sc_s(e) and acc2[e] = sum_s (Y_s sc_s(e))^2; the
 * gradient of the estimate beta_0 * mean(Y) is beta_0 / N * acc.  Threads
 * split the samples; their accumulators are added in thread order.
 */
typedef struct {
    const oo_graph *g; const oo_table *t; uint32_t qid, seed;
    uint64_t first, count;
    double *acc, *acc2;
    uint64_t sumY;
    int rc;
} bwd_job;

static void *bwd_worker(void *arg)
{
    bwd_job *b = arg;
    const oo_graph *g = b->g;
    const oo_table *t = b->t;
    oo_scratch w;
    if (scratch_init(&w, g->n)) { b->rc = OO_ENOMEM; return NULL; }
    uint64_t sy = 0;
    for (uint64_t q = 0; q < b->count; ++q) {
        uint64_t s = b->first + q;
        int64_t i;
        uint32_t Y = iicp_sample(g, t, b->qid, b->seed, 0, s, NULL, &i, &w);
        double y = (double)Y;
        sy += Y;
        /* Stage-2 revealed edges: every out-edge of every activated node */
        for (uint32_t h = 0; h < Y; ++h) {
            int32_t u = w.queue[h];
            for (int64_t e = g->row_ptr[u]; e < g->row_ptr[u + 1]; ++e) {
                if (t->inS[g->col[e]]) continue;
                double pe = (double)g->p[e];
                double sc = edge_coin(b->qid, b->seed, 0, s, g, e) ? 1.0 / pe : -1.0 / (1.0 - pe);
                b->acc[e] += y * sc;
                if (b->acc2) b->acc2[e] += (y * sc) * (y * sc);
            }
        }
        /* Stage-1 node coins, mapped to the S-edges into each entry */
        for (int64_t j = 0; j < t->l; ++j) {
            int xj = (j == i) || (j > i && w.live[j]);
            for (int64_t a = t->se_off[j]; a < t->se_off[j + 1]; ++a) {
                int64_t e = t->se[a];
                double sc;
                if (xj) {
                    double prod = 1.0;
                    for (int64_t c = t->se_off[j]; c < t->se_off[j + 1]; ++c)
                        if (c != a) prod = prod * (1.0 - (double)g->p[t->se[c]]);
                    sc = prod / t->P[j];
                } else {
                    sc = -1.0 / (1.0 - (double)g->p[e]);
                }
                b->acc[e] += y * sc;
                if (b->acc2) b->acc2[e] += (y * sc) * (y * sc);
            }
        }
    }
    scratch_free(&w);
    b->sumY = sy;
    b->rc = OO_OK;
    return NULL;
}

int oo_backward(int64_t n, int64_t m, const int64_t *row_ptr, const int32_t *col, const float *p,
                const int32_t *seeds, int64_t k, uint32_t qid, uint32_t seed, uint64_t first,
                uint64_t count, double *acc, double *acc2, uint64_t *sumY, double *beta0,
                int nthreads)
{
    oo_graph g = {n, m, row_ptr, col, p};
    oo_table t;
    int rc = oo_table_build(&g, seeds, k, &t);
    if (rc) return rc;
    *beta0 = t.beta0;
    *sumY = 0;
    for (int64_t e = 0; e < m; ++e) { acc[e] = 0.0; if (acc2) acc2[e] = 0.0; }
    if (t.beta0 == 0.0 || count == 0) { oo_table_free(&t); return OO_OK; }
    if (nthreads < 1) nthreads = 1;
    if ((uint64_t)nthreads > count) nthreads = (int)count;
    bwd_job *jobs = calloc((size_t)nthreads, sizeof(bwd_job));
    pthread_t *th = calloc((size_t)nthreads, sizeof(pthread_t));
    uint64_t per = count / (uint64_t)nthreads, rem = count % (uint64_t)nthreads, off = 0;
    rc = OO_OK;
    for (int i = 0; i < nthreads; ++i) {
        uint64_t c = per + ((uint64_t)i < rem ? 1 : 0);
        double *a1 = i == 0 ? acc : calloc((size_t)m, sizeof(double));
        double *a2 = acc2 ? (i == 0 ? acc2 : calloc((size_t)m, sizeof(double))) : NULL;
        jobs[i] = (bwd_job){&g, &t, qid, seed, first + off, c, a1, a2, 0, 0};
        off += c;
        if (nthreads == 1) bwd_worker(&jobs[i]);
        else pthread_create(&th[i], NULL, bwd_worker, &jobs[i]);
    }
    for (int i = 0; i < nthreads; ++i) {
        if (nthreads > 1) pthread_join(th[i], NULL);
        if (jobs[i].rc) rc = jobs[i].rc;
        *sumY += jobs[i].sumY;
        if (i > 0) {
            for (int64_t e = 0; e < m; ++e) acc[e] += jobs[i].acc[e];
            free(jobs[i].acc);
            if (acc2) {
                for (int64_t e = 0; e < m; ++e) acc2[e] += jobs[i].acc2[e];
                free(jobs[i].acc2);
            }
        }
    }
    free(jobs); free(th);
    oo_table_free(&t);
    return rc;
}
