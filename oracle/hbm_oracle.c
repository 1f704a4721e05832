/*
 * hbm_oracle.c -- plain, slow CPU reference of the memory-efficient IMM hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this file's library.  It shares no
 * code, header, table or helper with the GPU library; the two agree only
 * because both follow the same written definitions:
 *
 *   graph       G = (V, E, w) and its transpose (the RR-set definition,
 *               Background section, "RR set" / "RRR set" definitions);
 *               in-edges of v listed by ascending source, edge id = position.
 *   IC / LT     the diffusion models of the Background section.  IC edge
 *               probability: the edge weight (EDGE) or 1/indeg(v) (WC).
 *               LT: a vertex keeps at most one in-edge, edge e with
 *               probability w_e (live-edge form of LT).
 *   RNG         Philox4x32-10 (Salmon et al., SC'11), key = 64-bit seed,
 *               counter = (j_lo, j_hi, c2, tag); tag 0 root, 1 IC edge group
 *               (c2 = e/4, word e%4), 2 LT step (c2 = current vertex).
 *   uniform     r = word >> 8 (24 bits); r/2^24 < p decided in float32.
 *   root        floor(x * n / 2^64), x = word0 | word1 << 32 (uniform root).
 *   greedy      max coverage, k picks, lowest id wins ties, selected vertices
 *               excluded (Seed Selection paragraph; Alg. 2 / Alg. 3 read as
 *               picking exactly k seeds).
 *   IMM         two-phase martingale schedule of Tang et al. (Eq. 1 read as
 *               lambda' with "+ l *" in place of the garbled product).
 *   coding      Huffman codebook from the warm-up block (Alg. 1, Huffmax
 *               encoding section), codeless vertices copied verbatim (the
 *               CP array), the warm-up top vertex moved to the front of
 *               each coded string and the other codes in canonical order
 *               (length, then id); hot-vertex bitmap rows (Bitmax encoding
 *               section, restricted to the top fraction of vertices), or a
 *               row for every vertex (Bitmax proper: an n-row bit matrix
 *               over the sets, columns padded to a multiple of 64).
 *   choice      Alg. 1's branch after characterizing the first block (Eq. 2):
 *               Bitmax when the skewness is negative and the density is
 *               above 1/32 (the density threshold of the RRR-set
 *               characterization section), else Huffmax.
 *   Alg. 3      Bitmax selection on the bit matrix: frequencies are row
 *               popcounts; after each pick u*, row u* is subtracted from
 *               every row (v AND (v XOR u*)) and the popcounts are taken
 *               again.
 *
 * Nothing here is blocked, fused or reordered beyond those definitions.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_IC 0
#define ORC_LT 1
#define ORC_PROB_EDGE 0
#define ORC_PROB_WC 1

#define ORC_ENC_NONE 0
#define ORC_ENC_HUFFMAN 1
#define ORC_ENC_HOT_BITMAP 2
#define ORC_ENC_HUFFMAN_HOT_BITMAP 3
#define ORC_ENC_BITMAX 4 /* every vertex in a bitmap row (the Bitmax encoding section) */
#define ORC_ENC_AUTO 5   /* Alg. 1: characterize the first block, then Bitmax or Huffmax */

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Random123): 10 rounds, key bumped between rounds.         */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; r++) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static void draw(uint64_t seed, uint64_t j, uint32_t c2, uint32_t tag, uint32_t out[4]) {
    uint32_t ctr[4] = {(uint32_t)j, (uint32_t)(j >> 32), c2, tag};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, out);
}

/* true iff the 24-bit uniform r/2^24 is below probability p (decided in float32) */
static int below(uint32_t word, float p) {
    float r = (float)(word >> 8);
    return r < p * 16777216.0f;
}

/* ------------------------------------------------------------------------ */
/* Graph: in-edge lists (transpose), probabilities                           */
/* ------------------------------------------------------------------------ */
typedef struct orc_graph {
    int32_t n;
    int64_t m;
    int model, prob;
    int64_t *in_ptr; /* n+1 */
    int32_t *in_src; /* m, ascending within each row */
    float *p_edge;   /* IC-EDGE: per in-edge probability */
    float *p_vert;   /* WC: 1/indeg(v) */
    float *cum;      /* LT: running sum of in-weights along each row */
    uint8_t *visited; /* the graph's own sampling scratch (one caller at a time) */
    int32_t *queue;
} orc_graph;

/* Sampling scratch of one thread: a visited flag per vertex (all clear between sets) and a
   BFS queue.  Threads that sample the same graph at once each bring their own. */
typedef struct orc_scratch {
    uint8_t *visited;
    int32_t *queue;
} orc_scratch;

orc_scratch *orc_scratch_new(int32_t n) {
    orc_scratch *sc = (orc_scratch *)calloc(1, sizeof(orc_scratch));
    sc->visited = (uint8_t *)calloc((size_t)n, 1);
    sc->queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    return sc;
}

void orc_scratch_free(orc_scratch *sc) {
    if (!sc) return;
    free(sc->visited); free(sc->queue);
    free(sc);
}

void orc_graph_free(orc_graph *g) {
    if (!g) return;
    free(g->in_ptr); free(g->in_src); free(g->p_edge); free(g->p_vert); free(g->cum);
    free(g->visited); free(g->queue);
    free(g);
}

orc_graph *orc_graph_new(int32_t n, int64_t m, const int64_t *row_ptr, const int32_t *dst, const float *w,
                         int model, int prob) {
    orc_graph *g = (orc_graph *)calloc(1, sizeof(orc_graph));
    g->n = n; g->m = m; g->model = model; g->prob = prob;
    g->in_ptr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    g->in_src = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
    float *w_in = (float *)malloc(sizeof(float) * (size_t)(m ? m : 1));
    /* in-degree, then prefix sums */
    for (int64_t e = 0; e < m; e++) g->in_ptr[dst[e] + 1]++;
    for (int32_t v = 0; v < n; v++) g->in_ptr[v + 1] += g->in_ptr[v];
    /* visiting sources in ascending order fills every in-row in ascending source order */
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (int32_t v = 0; v < n; v++) fill[v] = g->in_ptr[v];
    for (int32_t u = 0; u < n; u++) {
        for (int64_t f = row_ptr[u]; f < row_ptr[u + 1]; f++) {
            int32_t v = dst[f];
            int64_t e = fill[v]++;
            g->in_src[e] = u;
            w_in[e] = w ? w[f] : 0.0f;
        }
    }
    free(fill);
    /* rows must come out ascending; a forward row with unsorted dst does not change that,
       because sources are visited in ascending order */
    if (prob == ORC_PROB_WC) {
        g->p_vert = (float *)malloc(sizeof(float) * (size_t)n);
        for (int32_t v = 0; v < n; v++) {
            int64_t d = g->in_ptr[v + 1] - g->in_ptr[v];
            g->p_vert[v] = d > 0 ? 1.0f / (float)d : 0.0f;
        }
    }
    if (model == ORC_IC && prob == ORC_PROB_EDGE) {
        g->p_edge = w_in;
        w_in = NULL;
    }
    if (model == ORC_LT) {
        g->cum = (float *)malloc(sizeof(float) * (size_t)(m ? m : 1));
        for (int32_t v = 0; v < n; v++) {
            float acc = 0.0f;
            for (int64_t e = g->in_ptr[v]; e < g->in_ptr[v + 1]; e++) {
                float we = (prob == ORC_PROB_WC) ? g->p_vert[v] : w_in[e];
                acc = acc + we;
                g->cum[e] = acc;
            }
        }
    }
    free(w_in);
    g->visited = (uint8_t *)calloc((size_t)n, 1);
    g->queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    return g;
}

int64_t orc_graph_in_ptr(const orc_graph *g, int64_t **p) { *p = g->in_ptr; return g->n + 1; }
int64_t orc_graph_in_src(const orc_graph *g, int32_t **p) { *p = g->in_src; return g->m; }

/* ------------------------------------------------------------------------ */
/* One RR set                                                                */
/* ------------------------------------------------------------------------ */
int32_t orc_root(int32_t n, uint64_t seed, uint64_t j) {
    uint32_t y[4];
    draw(seed, j, 0u, 0u, y);
    uint64_t x = (uint64_t)y[0] | ((uint64_t)y[1] << 32);
    return (int32_t)(((unsigned __int128)x * (unsigned __int128)(uint64_t)n) >> 64);
}

/* IC: every vertex that reaches the root through live in-edges; plain BFS. */
static int64_t sample_ic(const orc_graph *g, orc_scratch *sc, uint64_t seed, uint64_t j, int32_t *out) {
    int32_t root = orc_root(g->n, seed, j);
    int64_t head = 0, tail = 0;
    sc->queue[tail++] = root;
    sc->visited[root] = 1;
    while (head < tail) {
        int32_t v = sc->queue[head++];
        uint64_t last_group = UINT64_MAX;
        uint32_t y[4] = {0, 0, 0, 0};
        for (int64_t e = g->in_ptr[v]; e < g->in_ptr[v + 1]; e++) {
            uint64_t group = (uint64_t)e >> 2;
            if (group != last_group) {
                draw(seed, j, (uint32_t)group, 1u, y);
                last_group = group;
            }
            float p = g->p_edge ? g->p_edge[e] : g->p_vert[v];
            if (below(y[e & 3], p)) {
                int32_t u = g->in_src[e];
                if (!sc->visited[u]) {
                    sc->visited[u] = 1;
                    sc->queue[tail++] = u;
                }
            }
        }
    }
    for (int64_t i = 0; i < tail; i++) {
        out[i] = sc->queue[i];
        sc->visited[sc->queue[i]] = 0;
    }
    return tail;
}

/* LT: reverse walk; at each step the current vertex keeps the first in-edge whose
   cumulative weight exceeds the draw, or none; the walk stops at none or at a repeat. */
static int64_t sample_lt(const orc_graph *g, orc_scratch *sc, uint64_t seed, uint64_t j, int32_t *out) {
    int32_t cur = orc_root(g->n, seed, j);
    int64_t len = 0;
    out[len++] = cur;
    sc->visited[cur] = 1;
    for (;;) {
        uint32_t y[4];
        draw(seed, j, (uint32_t)cur, 2u, y);
        int64_t pick = -1;
        for (int64_t e = g->in_ptr[cur]; e < g->in_ptr[cur + 1]; e++) {
            if (below(y[0], g->cum[e])) {
                pick = e;
                break;
            }
        }
        if (pick < 0) break;
        int32_t s = g->in_src[pick];
        if (sc->visited[s]) break;
        sc->visited[s] = 1;
        out[len++] = s;
        cur = s;
    }
    for (int64_t i = 0; i < len; i++) sc->visited[out[i]] = 0;
    return len;
}

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* RR set j, ascending; out must hold n entries.  Returns its size. */
static int64_t sample_with(const orc_graph *g, orc_scratch *sc, uint64_t seed, int64_t j, int32_t *out) {
    int64_t len = g->model == ORC_IC ? sample_ic(g, sc, seed, (uint64_t)j, out) : sample_lt(g, sc, seed, (uint64_t)j, out);
    qsort(out, (size_t)len, sizeof(int32_t), cmp_i32);
    return len;
}

int64_t orc_sample_one(orc_graph *g, uint64_t seed, int64_t j, int32_t *out) {
    orc_scratch own = {g->visited, g->queue};
    return sample_with(g, &own, seed, j, out);
}

/* ------------------------------------------------------------------------ */
/* Store of RR sets 0..nsets-1 (canonical: each set ascending)               */
/* ------------------------------------------------------------------------ */
typedef struct orc_store {
    int64_t nsets, cap_sets;
    int64_t *off; /* nsets+1 */
    int32_t *mem;
    int64_t cap_mem;
    uint64_t seed;
} orc_store;

orc_store *orc_store_new(void) {
    orc_store *s = (orc_store *)calloc(1, sizeof(orc_store));
    s->cap_sets = 1024;
    s->off = (int64_t *)calloc((size_t)s->cap_sets + 1, sizeof(int64_t));
    s->cap_mem = 1 << 16;
    s->mem = (int32_t *)malloc(sizeof(int32_t) * (size_t)s->cap_mem);
    return s;
}

void orc_store_free(orc_store *s) {
    if (!s) return;
    free(s->off); free(s->mem); free(s);
}

void orc_store_reset(orc_store *s) { s->nsets = 0; s->off[0] = 0; }

int64_t orc_store_nsets(const orc_store *s) { return s->nsets; }
int64_t orc_store_nmem(const orc_store *s) { return s->off[s->nsets]; }
const int64_t *orc_store_off(const orc_store *s) { return s->off; }
const int32_t *orc_store_mem(const orc_store *s) { return s->mem; }

/* Make the store hold sets 0..theta-1 under `seed` (appending). */
int orc_store_extend(orc_store *s, orc_graph *g, uint64_t seed, int64_t theta) {
    if (s->nsets > 0 && s->seed != seed) orc_store_reset(s);
    s->seed = seed;
    if (theta <= s->nsets) return 0;
    if (theta > s->cap_sets) {
        int64_t c = s->cap_sets;
        while (c < theta) c *= 2;
        s->off = (int64_t *)realloc(s->off, sizeof(int64_t) * (size_t)(c + 1));
        s->cap_sets = c;
    }
    int32_t *buf = (int32_t *)malloc(sizeof(int32_t) * (size_t)g->n);
    for (int64_t j = s->nsets; j < theta; j++) {
        int64_t len = orc_sample_one(g, seed, j, buf);
        int64_t base = s->off[j];
        if (base + len > s->cap_mem) {
            int64_t c = s->cap_mem;
            while (c < base + len) c *= 2;
            s->mem = (int32_t *)realloc(s->mem, sizeof(int32_t) * (size_t)c);
            s->cap_mem = c;
        }
        memcpy(s->mem + base, buf, sizeof(int32_t) * (size_t)len);
        s->off[j + 1] = base + len;
    }
    s->nsets = theta;
    free(buf);
    return 0;
}

/* Append RR sets j0..j1-1 as the store's next sets (a shard of the index range: set i
   of a store filled only this way from j0 is RR set j0 + i).  Results do not depend on
   how the index range is split, which lets the benchmark time shards on several threads,
   each with its own scratch `sc` (NULL: the graph's own, for one caller at a time). */
int orc_store_append_range(orc_store *s, orc_graph *g, orc_scratch *sc, uint64_t seed, int64_t j0, int64_t j1) {
    if (j1 <= j0) return 0;
    orc_scratch own = {g->visited, g->queue};
    if (!sc) sc = &own;
    int64_t need = s->nsets + (j1 - j0);
    if (need > s->cap_sets) {
        int64_t c = s->cap_sets;
        while (c < need) c *= 2;
        s->off = (int64_t *)realloc(s->off, sizeof(int64_t) * (size_t)(c + 1));
        s->cap_sets = c;
    }
    int32_t *buf = (int32_t *)malloc(sizeof(int32_t) * (size_t)g->n);
    for (int64_t j = j0; j < j1; j++) {
        int64_t len = sample_with(g, sc, seed, j, buf);
        int64_t i = s->nsets, base = s->off[i];
        if (base + len > s->cap_mem) {
            int64_t c = s->cap_mem;
            while (c < base + len) c *= 2;
            s->mem = (int32_t *)realloc(s->mem, sizeof(int32_t) * (size_t)c);
            s->cap_mem = c;
        }
        memcpy(s->mem + base, buf, sizeof(int32_t) * (size_t)len);
        s->off[i + 1] = base + len;
        s->nsets = i + 1;
    }
    s->seed = seed;
    free(buf);
    return 0;
}

/* Replace the store's contents with explicit sets (each must be ascending). */
int orc_store_set(orc_store *s, int64_t nsets, const int64_t *off, const int32_t *mem) {
    free(s->off);
    free(s->mem);
    s->cap_sets = nsets > 0 ? nsets : 1;
    s->off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(s->cap_sets + 1));
    memcpy(s->off, off, sizeof(int64_t) * (size_t)(nsets + 1));
    s->cap_mem = off[nsets] > 0 ? off[nsets] : 1;
    s->mem = (int32_t *)malloc(sizeof(int32_t) * (size_t)s->cap_mem);
    memcpy(s->mem, mem, sizeof(int32_t) * (size_t)off[nsets]);
    s->nsets = nsets;
    s->seed = 0;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Greedy max coverage over a set system                                     */
/* ------------------------------------------------------------------------ */
int orc_greedy_sets(int64_t nsets, const int64_t *off, const int32_t *mem, int32_t n, int32_t k, int32_t *seeds,
                    uint64_t *gains, uint64_t *coverage) {
    if (k < 1 || k > n) return 1;
    int64_t nm = off[nsets];
    uint64_t *cnt = (uint64_t *)calloc((size_t)n, sizeof(uint64_t));
    uint8_t *selected = (uint8_t *)calloc((size_t)n, 1);
    uint8_t *covered = (uint8_t *)calloc((size_t)(nsets ? nsets : 1), 1);
    /* inverted index: for every vertex, the sets containing it */
    int64_t *iptr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t *iset = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nm ? nm : 1));
    for (int64_t i = 0; i < nm; i++) iptr[mem[i] + 1]++;
    for (int32_t v = 0; v < n; v++) iptr[v + 1] += iptr[v];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (int32_t v = 0; v < n; v++) fill[v] = iptr[v];
    for (int64_t j = 0; j < nsets; j++)
        for (int64_t i = off[j]; i < off[j + 1]; i++) iset[fill[mem[i]]++] = j;
    free(fill);
    for (int64_t i = 0; i < nm; i++) cnt[mem[i]]++;
    uint64_t cov = 0;
    for (int32_t t = 0; t < k; t++) {
        int32_t best = -1;
        for (int32_t v = 0; v < n; v++) {
            if (selected[v]) continue;
            if (best < 0 || cnt[v] > cnt[best]) best = v;
        }
        uint64_t gain = cnt[best];
        seeds[t] = best;
        gains[t] = gain;
        cov += gain;
        selected[best] = 1;
        for (int64_t q = iptr[best]; q < iptr[best + 1]; q++) {
            int64_t j = iset[q];
            if (covered[j]) continue;
            covered[j] = 1;
            for (int64_t i = off[j]; i < off[j + 1]; i++) cnt[mem[i]]--;
        }
    }
    *coverage = cov;
    free(cnt); free(selected); free(covered); free(iptr); free(iset);
    return 0;
}

int orc_greedy(const orc_store *s, int32_t n, int32_t k, int32_t *seeds, uint64_t *gains, uint64_t *coverage) {
    return orc_greedy_sets(s->nsets, s->off, s->mem, n, k, seeds, gains, coverage);
}

/* vertex frequencies over sets [j0, j1) */
void orc_counts(const orc_store *s, int32_t n, int64_t j0, int64_t j1, uint64_t *cnt) {
    memset(cnt, 0, sizeof(uint64_t) * (size_t)n);
    for (int64_t i = s->off[j0]; i < s->off[j1]; i++) cnt[s->mem[i]]++;
}

/* Eq. 2: skewness (population moments) and density of the set sizes in [j0, j1) */
void orc_characterize(const orc_store *s, int32_t n, int64_t j0, int64_t j1, double *skew, double *density) {
    int64_t t = j1 - j0;
    double mean = 0.0;
    for (int64_t j = j0; j < j1; j++) mean += (double)(s->off[j + 1] - s->off[j]);
    mean /= (double)t;
    double m2 = 0.0, m3 = 0.0;
    for (int64_t j = j0; j < j1; j++) {
        double d = (double)(s->off[j + 1] - s->off[j]) - mean;
        m2 += d * d;
        m3 += d * d * d;
    }
    m2 /= (double)t;
    m3 /= (double)t;
    double sd = sqrt(m2);
    *skew = sd > 0.0 ? m3 / (sd * sd * sd) : 0.0;
    *density = (double)(s->off[j1] - s->off[j0]) / ((double)t * (double)n);
}

/* ------------------------------------------------------------------------ */
/* IMM (Tang, Shi, Xiao 2015): estimation rounds, lower bound, final theta   */
/* ------------------------------------------------------------------------ */
typedef struct orc_imm_stats {
    int32_t rounds;
    int64_t theta_round[64];
    uint64_t cov_round[64];
    double lb;
    int64_t theta_final;
    int64_t nsets_final;
    uint64_t coverage;
    double l_adj, eps_prime, lnC, lambda_prime, lambda_star;
} orc_imm_stats;

void orc_imm_params(int32_t n, int32_t k, double eps, double l, double *l_adj, double *eps_prime, double *lnC,
                    double *lambda_prime, double *lambda_star) {
    double dn = (double)n;
    double la = l * (1.0 + log(2.0) / log(dn));
    double ep = sqrt(2.0) * eps;
    double lc = 0.0;
    for (int32_t i = 1; i <= k; i++) lc += log((double)(n - k + i)) - log((double)i);
    double lp = (2.0 + 2.0 * ep / 3.0) * (lc + la * log(dn) + log(log2(dn))) * dn / (ep * ep);
    double e1 = 1.0 - 1.0 / exp(1.0);
    double alpha = sqrt(la * log(dn) + log(2.0));
    double beta = sqrt(e1 * (lc + la * log(dn) + log(2.0)));
    double ls = 2.0 * dn * (e1 * alpha + beta) * (e1 * alpha + beta) / (eps * eps);
    *l_adj = la; *eps_prime = ep; *lnC = lc; *lambda_prime = lp; *lambda_star = ls;
}

int orc_imm(orc_graph *g, orc_store *s, int32_t k, double eps, double l, uint64_t seed, int32_t *seeds,
            uint64_t *gains, orc_imm_stats *st) {
    int32_t n = g->n;
    double dn = (double)n;
    double la, ep, lc, lp, ls;
    orc_imm_params(n, k, eps, l, &la, &ep, &lc, &lp, &ls);
    memset(st, 0, sizeof(*st));
    st->l_adj = la; st->eps_prime = ep; st->lnC = lc; st->lambda_prime = lp; st->lambda_star = ls;
    orc_store_reset(s);
    double lb = 1.0;
    uint64_t cov = 0;
    for (int32_t i = 1; (double)i <= log2(dn) - 1.0; i++) {
        double x = dn / pow(2.0, (double)i);
        int64_t th = (int64_t)ceil(lp / x);
        orc_store_extend(s, g, seed, th);
        orc_greedy(s, n, k, seeds, gains, &cov);
        st->theta_round[st->rounds] = th;
        st->cov_round[st->rounds] = cov;
        st->rounds++;
        if (dn * (double)cov / (double)th >= (1.0 + ep) * x) {
            lb = dn * (double)cov / ((double)th * (1.0 + ep));
            break;
        }
    }
    int64_t theta = (int64_t)ceil(ls / lb);
    st->lb = lb;
    st->theta_final = theta;
    int64_t target = theta > s->nsets ? theta : s->nsets;
    orc_store_extend(s, g, seed, target);
    orc_greedy(s, n, k, seeds, gains, &cov);
    st->nsets_final = s->nsets;
    st->coverage = cov;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Huffman code lengths: two queues, leaves ordered by (weight, id), a leaf  */
/* wins a tie against an internal node; longest code 32 bits, otherwise      */
/* every weight w becomes ceil(w/2) and the tree is rebuilt.                 */
/* ------------------------------------------------------------------------ */
typedef struct { uint64_t w; int32_t id; } leaf_t;

static int cmp_leaf(const void *a, const void *b) {
    const leaf_t *x = (const leaf_t *)a, *y = (const leaf_t *)b;
    if (x->w != y->w) return x->w < y->w ? -1 : 1;
    return (x->id > y->id) - (x->id < y->id);
}

int orc_huffman_lengths(int32_t nsym, const uint64_t *weights, uint8_t *lens) {
    memset(lens, 0, (size_t)nsym);
    int64_t nl = 0;
    for (int32_t v = 0; v < nsym; v++) nl += weights[v] > 0;
    if (nl == 0) return 0;
    leaf_t *lv = (leaf_t *)malloc(sizeof(leaf_t) * (size_t)nl);
    uint64_t *wt = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)nsym);
    for (int32_t v = 0; v < nsym; v++) wt[v] = weights[v];
    if (nl == 1) {
        for (int32_t v = 0; v < nsym; v++)
            if (wt[v] > 0) lens[v] = 1;
        free(lv); free(wt);
        return 1;
    }
    int64_t nnode = 2 * nl - 1;
    uint64_t *nw = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)nnode);
    int64_t *parent = (int64_t *)malloc(sizeof(int64_t) * (size_t)nnode);
    int32_t *depth = (int32_t *)malloc(sizeof(int32_t) * (size_t)nnode);
    int maxlen;
    for (;;) {
        int64_t q = 0;
        for (int32_t v = 0; v < nsym; v++)
            if (wt[v] > 0) { lv[q].w = wt[v]; lv[q].id = v; q++; }
        qsort(lv, (size_t)nl, sizeof(leaf_t), cmp_leaf);
        for (int64_t i = 0; i < nl; i++) nw[i] = lv[i].w;
        int64_t i1 = 0, i2 = nl, next = nl; /* leaves in [i1,nl), internal nodes in [i2,next) */
        while (next < nnode) {
            int64_t pick[2];
            for (int c = 0; c < 2; c++) {
                if (i1 < nl && (i2 >= next || nw[i1] <= nw[i2])) pick[c] = i1++;
                else pick[c] = i2++;
            }
            nw[next] = nw[pick[0]] + nw[pick[1]];
            parent[pick[0]] = next;
            parent[pick[1]] = next;
            next++;
        }
        depth[nnode - 1] = 0;
        for (int64_t x = nnode - 2; x >= 0; x--) depth[x] = depth[parent[x]] + 1;
        maxlen = 0;
        for (int64_t i = 0; i < nl; i++)
            if (depth[i] > maxlen) maxlen = depth[i];
        if (maxlen <= 32) {
            for (int64_t i = 0; i < nl; i++) lens[lv[i].id] = (uint8_t)depth[i];
            break;
        }
        for (int32_t v = 0; v < nsym; v++)
            if (wt[v] > 0) wt[v] = (wt[v] + 1) / 2;
    }
    free(lv); free(wt); free(nw); free(parent); free(depth);
    return maxlen;
}

/* Canonical codes: symbols ordered by (length, id); each code is the previous one
   plus one, shifted left by the length increase; the first code is all zeros. */
typedef struct { uint8_t len; int32_t id; } lsym_t;
static int cmp_lsym(const void *a, const void *b) {
    const lsym_t *x = (const lsym_t *)a, *y = (const lsym_t *)b;
    if (x->len != y->len) return x->len < y->len ? -1 : 1;
    return (x->id > y->id) - (x->id < y->id);
}

void orc_canonical_codes(int32_t nsym, const uint8_t *lens, uint32_t *codes) {
    int64_t ns = 0;
    for (int32_t v = 0; v < nsym; v++) { codes[v] = 0; ns += lens[v] > 0; }
    if (ns == 0) return;
    lsym_t *s = (lsym_t *)malloc(sizeof(lsym_t) * (size_t)ns);
    int64_t q = 0;
    for (int32_t v = 0; v < nsym; v++)
        if (lens[v]) { s[q].len = lens[v]; s[q].id = v; q++; }
    qsort(s, (size_t)ns, sizeof(lsym_t), cmp_lsym);
    uint64_t code = 0;
    for (int64_t i = 0; i < ns; i++) {
        if (i > 0) code = (code + 1) << (s[i].len - s[i - 1].len);
        codes[s[i].id] = (uint32_t)code;
    }
    free(s);
}

/* ------------------------------------------------------------------------ */
/* Encoded store                                                             */
/* ------------------------------------------------------------------------ */
typedef struct orc_encoded {
    int enc;
    int implicit_roots;  /* the root of set j is not stored unless it is in a bitmap row */
    uint64_t seed;       /* the store's seed: root_j = orc_root(n, seed, j) */
    int32_t n;
    int64_t nsets, W;
    uint64_t *warm;      /* warm-up vertex frequencies, n */
    int32_t nhot;
    int32_t *hot;        /* hot vertices by rank */
    int64_t nwords;      /* ceil(nsets/64) */
    uint64_t *bitmap;    /* nwords * nhot, word-major: bitmap[w*nhot + r] */
    /* array containers (Roaring-style) for hot vertices of warm-up density below 1/16:
       per chunk c of 2^16 sets, array row a's sets are the sorted 16-bit offsets
       ar_low[ar_off[c*(nar+1) + a] .. ar_off[c*(nar+1) + a + 1]) */
    int32_t nar;
    int32_t *ar_hot;     /* array-row vertices, in hot order */
    int64_t nchunks;     /* ceil(nsets / 2^16) */
    int64_t *ar_off;     /* nchunks * (nar + 1), offsets into ar_low */
    uint16_t *ar_low;
    int64_t *cold_off;   /* raw cold members (NONE / HOT_BITMAP): nsets+1 */
    int32_t *cold_mem;
    uint8_t *lens;       /* Huffman lengths, n (0 = no code) */
    uint32_t *codes;     /* canonical codes, n */
    int32_t ustar_enc;   /* warm-up top vertex among coded symbols, -1 if none */
    int32_t wbits;       /* width of a verbatim id */
    int64_t *bitoff;     /* nsets+1 */
    uint32_t *payload;   /* ceil(bits/32)+1 words, MSB first */
    int64_t npayload;
    int64_t n_escapes;
    int64_t n_coded;
    int32_t maxlen;
} orc_encoded;

void orc_encoded_free(orc_encoded *e) {
    if (!e) return;
    free(e->ar_hot); free(e->ar_off); free(e->ar_low);
    free(e->warm); free(e->hot); free(e->bitmap); free(e->cold_off); free(e->cold_mem);
    free(e->lens); free(e->codes); free(e->bitoff); free(e->payload);
    free(e);
}

int64_t orc_warmup_count(double frac, int64_t theta) {
    int64_t w = (int64_t)ceil(frac * (double)theta);
    if (w < 1) w = 1;
    if (w > theta) w = theta;
    return w;
}

static void put_bits(uint32_t *buf, uint64_t pos, uint32_t value, int nbits) {
    for (int b = nbits - 1; b >= 0; b--) {
        if ((value >> b) & 1u) buf[pos >> 5] |= 1u << (31 - (pos & 31));
        pos++;
    }
}

static int floor_log2_u64(uint64_t x) {
    int l = -1;
    while (x) { l++; x >>= 1; }
    return l;
}

/* hot set: the ceil(hot_frac * n) vertices with the most warm-up occurrences (ties to the
 * lower id), counting only vertices in at least ceil(hot_min_density * W) warm-up sets
 * (and in at least one).  A bitmap row costs one bit per set, a stored id 32 bits per
 * occurrence, so a row pays for itself above density 1/32 (the density threshold of the
 * RRR-set characterization section), here applied vertex by vertex. */
/* Implicit roots: set j always holds its root (the uniform draw that starts it), which is a
 * function of (seed, j) alone, so with implicit_roots the root is dropped from the stored
 * plain ids or Huffman string (a root with a bitmap row keeps its bit) and regenerated when
 * the set is decoded.  Returns 2 if some set lacks its root (a store not sampled from the
 * graph). */
/* Row containers (Roaring-style, after Chambi et al.): with `containers`, a hot vertex whose
 * warm-up density is below 1/16 (in fewer than W/16 warm-up sets) keeps, per chunk of 2^16
 * sets, the sorted 16-bit offsets of its sets within the chunk (16 bits per occurrence, the
 * smaller form below that density) instead of a bitmap row (one bit per set); hot vertices
 * at or above 1/16 keep bitmap rows.  Either way the vertex is out of the cold part. */
int orc_encode(const orc_store *s, int32_t n, int enc, int64_t W, double hot_frac, double hot_min_density,
               int implicit_roots, int containers, orc_encoded **out) {
    int64_t T = s->nsets;
    if (implicit_roots) {
        for (int64_t j = 0; j < T; j++) {
            int32_t r = orc_root(n, s->seed, (uint64_t)j);
            int has = 0;
            for (int64_t i = s->off[j]; i < s->off[j + 1]; i++) has |= s->mem[i] == r;
            if (!has) return 2;
        }
    }
    orc_encoded *e = (orc_encoded *)calloc(1, sizeof(orc_encoded));
    e->enc = enc; e->n = n; e->nsets = T; e->W = W;
    e->implicit_roots = implicit_roots;
    e->seed = s->seed;
    e->warm = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    orc_counts(s, n, 0, W, e->warm);
    if (enc == ORC_ENC_AUTO) {
        /* Alg. 1: Characterize the first block; Bitmax needs S < 0 and D > 1/32 */
        double skew = 0.0, dens = 0.0;
        orc_characterize(s, n, 0, W, &skew, &dens);
        enc = (skew < 0.0 && dens > 1.0 / 32.0) ? ORC_ENC_BITMAX : ORC_ENC_HUFFMAN;
        e->enc = enc;
    }
    int use_hot = (enc == ORC_ENC_HOT_BITMAP || enc == ORC_ENC_HUFFMAN_HOT_BITMAP);
    int use_huff = (enc == ORC_ENC_HUFFMAN || enc == ORC_ENC_HUFFMAN_HOT_BITMAP);
    int32_t *rank = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *arank = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    for (int32_t v = 0; v < n; v++) rank[v] = arank[v] = -1;
#define ORC_COLD(v) (rank[(v)] < 0 && arank[(v)] < 0)
    if (enc == ORC_ENC_BITMAX) {
        /* the n x nsets bit matrix: row v holds bit j when v is in set j */
        e->nhot = n;
        e->hot = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        for (int32_t v = 0; v < n; v++) { e->hot[v] = v; rank[v] = v; }
        e->nwords = (T + 63) / 64;
        e->bitmap = (uint64_t *)calloc((size_t)(e->nwords * e->nhot + 1), sizeof(uint64_t));
        for (int64_t j = 0; j < T; j++)
            for (int64_t i = s->off[j]; i < s->off[j + 1]; i++)
                e->bitmap[(j / 64) * e->nhot + s->mem[i]] |= 1ull << (j % 64);
        free(rank);
        free(arank);
        *out = e;
        return 0;
    }
    if (use_hot) {
        int64_t want = (int64_t)ceil(hot_frac * (double)n);
        uint64_t min_cnt = (uint64_t)ceil(hot_min_density * (double)W);
        if (min_cnt < 1) min_cnt = 1;
        /* order eligible vertices by (count desc, id asc) */
        leaf_t *c = (leaf_t *)malloc(sizeof(leaf_t) * (size_t)n);
        int64_t q = 0;
        for (int32_t v = 0; v < n; v++)
            if (e->warm[v] >= min_cnt) { c[q].w = UINT64_MAX - e->warm[v]; c[q].id = v; q++; }
        qsort(c, (size_t)q, sizeof(leaf_t), cmp_leaf);
        int32_t keep = (int32_t)(q < want ? q : want);
        e->hot = (int32_t *)malloc(sizeof(int32_t) * (size_t)(keep ? keep : 1));
        e->ar_hot = (int32_t *)malloc(sizeof(int32_t) * (size_t)(keep ? keep : 1));
        e->nhot = 0;
        e->nar = 0;
        for (int32_t r = 0; r < keep; r++) {
            int32_t v = c[r].id;
            if (containers && (uint64_t)16 * e->warm[v] < (uint64_t)W) {
                arank[v] = e->nar;
                e->ar_hot[e->nar++] = v;
            } else {
                rank[v] = e->nhot;
                e->hot[e->nhot++] = v;
            }
        }
        free(c);
        e->nchunks = (T + 65535) / 65536;
        int64_t stride = (int64_t)e->nar + 1;
        e->ar_off = (int64_t *)calloc((size_t)(e->nchunks * stride + 1), sizeof(int64_t));
        /* counts per (chunk, row), then offsets in (chunk, row) order, then the offsets of
           the sets in ascending set order, which keeps each row's list ascending */
        int64_t *cnt = (int64_t *)calloc((size_t)(e->nchunks * stride + 1), sizeof(int64_t));
        for (int64_t j = 0; j < T; j++)
            for (int64_t i = s->off[j]; i < s->off[j + 1]; i++)
                if (arank[s->mem[i]] >= 0) cnt[(j / 65536) * stride + arank[s->mem[i]]]++;
        int64_t nlow = 0;
        for (int64_t ch = 0; ch < e->nchunks; ch++) {
            for (int32_t a = 0; a < e->nar; a++) {
                e->ar_off[ch * stride + a] = nlow;
                nlow += cnt[ch * stride + a];
            }
            e->ar_off[ch * stride + e->nar] = nlow;
        }
        e->ar_low = (uint16_t *)malloc(sizeof(uint16_t) * (size_t)(nlow ? nlow : 1));
        for (int64_t ch = 0; ch < e->nchunks; ch++)
            for (int32_t a = 0; a < e->nar; a++) cnt[ch * stride + a] = e->ar_off[ch * stride + a];
        for (int64_t j = 0; j < T; j++)
            for (int64_t i = s->off[j]; i < s->off[j + 1]; i++)
                if (arank[s->mem[i]] >= 0)
                    e->ar_low[cnt[(j / 65536) * stride + arank[s->mem[i]]]++] = (uint16_t)(j % 65536);
        free(cnt);
        e->nwords = (T + 63) / 64;
        e->bitmap = (uint64_t *)calloc((size_t)(e->nwords * e->nhot + 1), sizeof(uint64_t));
        for (int64_t j = 0; j < T; j++)
            for (int64_t i = s->off[j]; i < s->off[j + 1]; i++) {
                int32_t r = rank[s->mem[i]];
                if (r >= 0) e->bitmap[(j / 64) * e->nhot + r] |= 1ull << (j % 64);
            }
    }
    if (!use_huff) {
        e->cold_off = (int64_t *)calloc((size_t)T + 1, sizeof(int64_t));
        int64_t total = 0;
        for (int64_t j = 0; j < T; j++) {
            int32_t skip = implicit_roots ? orc_root(n, s->seed, (uint64_t)j) : -1;
            for (int64_t i = s->off[j]; i < s->off[j + 1]; i++) total += ORC_COLD(s->mem[i]) && s->mem[i] != skip;
            e->cold_off[j + 1] = total;
        }
        e->cold_mem = (int32_t *)malloc(sizeof(int32_t) * (size_t)(total ? total : 1));
        int64_t q = 0;
        for (int64_t j = 0; j < T; j++) {
            int32_t skip = implicit_roots ? orc_root(n, s->seed, (uint64_t)j) : -1;
            for (int64_t i = s->off[j]; i < s->off[j + 1]; i++)
                if (ORC_COLD(s->mem[i]) && s->mem[i] != skip) e->cold_mem[q++] = s->mem[i];
        }
    } else {
        /* codebook over the non-hot vertices seen in the warm-up block */
        uint64_t *wt = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
        for (int32_t v = 0; v < n; v++) wt[v] = ORC_COLD(v) ? e->warm[v] : 0;
        e->lens = (uint8_t *)malloc((size_t)n);
        e->codes = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
        e->maxlen = orc_huffman_lengths(n, wt, e->lens);
        orc_canonical_codes(n, e->lens, e->codes);
        e->ustar_enc = -1;
        for (int32_t v = 0; v < n; v++)
            if (wt[v] > 0 && (e->ustar_enc < 0 || wt[v] > wt[e->ustar_enc])) e->ustar_enc = v;
        free(wt);
        e->wbits = n > 1 ? floor_log2_u64((uint64_t)(n - 1)) + 1 : 1;
        /* bit lengths */
        e->bitoff = (int64_t *)calloc((size_t)T + 1, sizeof(int64_t));
        for (int64_t j = 0; j < T; j++) {
            uint64_t nesc = 0, bits = 0;
            int32_t skip = implicit_roots ? orc_root(n, s->seed, (uint64_t)j) : -1;
            for (int64_t i = s->off[j]; i < s->off[j + 1]; i++) {
                int32_t v = s->mem[i];
                if (!ORC_COLD(v) || v == skip) continue;
                if (e->lens[v]) bits += e->lens[v];
                else nesc++;
            }
            int L = floor_log2_u64(nesc + 1);
            bits += (uint64_t)(2 * L + 1) + nesc * (uint64_t)e->wbits;
            e->bitoff[j + 1] = e->bitoff[j] + (int64_t)bits;
        }
        int64_t total = e->bitoff[T];
        e->npayload = (total + 31) / 32 + 1;
        e->payload = (uint32_t *)calloc((size_t)e->npayload, sizeof(uint32_t));
        for (int64_t j = 0; j < T; j++) {
            uint64_t pos = (uint64_t)e->bitoff[j];
            uint64_t nesc = 0;
            int32_t skip = implicit_roots ? orc_root(n, s->seed, (uint64_t)j) : -1;
            for (int64_t i = s->off[j]; i < s->off[j + 1]; i++) {
                int32_t v = s->mem[i];
                if (ORC_COLD(v) && e->lens[v] == 0 && v != skip) nesc++;
            }
            /* Elias gamma of nesc+1 */
            int L = floor_log2_u64(nesc + 1);
            pos += (uint64_t)L; /* L zero bits */
            put_bits(e->payload, pos, (uint32_t)(nesc + 1), L + 1);
            pos += (uint64_t)(L + 1);
            /* verbatim ids of codeless members, ascending */
            for (int64_t i = s->off[j]; i < s->off[j + 1]; i++) {
                int32_t v = s->mem[i];
                if (ORC_COLD(v) && e->lens[v] == 0 && v != skip) {
                    put_bits(e->payload, pos, (uint32_t)v, e->wbits);
                    pos += (uint64_t)e->wbits;
                }
            }
            e->n_escapes += (int64_t)nesc;
            /* coded members: the warm-up top vertex first, then the rest in canonical code
               order, i.e. by (code length, id), which is ascending left-justified code value */
            int has_front = 0;
            for (int64_t i = s->off[j]; i < s->off[j + 1]; i++)
                if (s->mem[i] == e->ustar_enc && s->mem[i] != skip) has_front = 1;
            if (has_front) {
                put_bits(e->payload, pos, e->codes[e->ustar_enc], e->lens[e->ustar_enc]);
                pos += e->lens[e->ustar_enc];
                e->n_coded++;
            }
            for (int clen = 1; clen <= 32; clen++)
                for (int64_t i = s->off[j]; i < s->off[j + 1]; i++) {
                    int32_t v = s->mem[i];
                    if (!ORC_COLD(v) || e->lens[v] != clen || v == e->ustar_enc || v == skip) continue;
                    put_bits(e->payload, pos, e->codes[v], e->lens[v]);
                    pos += e->lens[v];
                    e->n_coded++;
                }
        }
    }
    free(rank);
    free(arank);
#undef ORC_COLD
    *out = e;
    return 0;
}

/* Alg. 3 on a Bitmax store: h[v] = POPCOUNT(row v); each round picks u* = the unselected
 * vertex with the largest h (lowest id on ties), then SUBTRACTs row u* from every row
 * (v AND (v XOR u*)) and recounts h.  Rows whose popcount reaches zero are flagged and
 * skipped afterwards (deleteVTXflag).  Exactly k picks.  `after` (may be NULL) receives
 * the matrix once the k-th row has been subtracted. */
int orc_bitmax_select(const orc_encoded *e, int32_t k, int32_t *seeds, uint64_t *gains, uint64_t *coverage,
                      uint64_t *after) {
    if (e->enc != ORC_ENC_BITMAX || k < 1 || k > e->n) return 1;
    int32_t n = e->n;
    int64_t nw = e->nwords;
    uint64_t *B = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(nw * n + 1));
    memcpy(B, e->bitmap, sizeof(uint64_t) * (size_t)(nw * n));
    uint64_t *h = (uint64_t *)calloc((size_t)n, sizeof(uint64_t));
    uint8_t *del = (uint8_t *)calloc((size_t)n, 1);
    uint8_t *sel = (uint8_t *)calloc((size_t)n, 1);
    uint64_t *urow = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(nw + 1));
    for (int32_t v = 0; v < n; v++)
        for (int64_t w = 0; w < nw; w++) h[v] += (uint64_t)__builtin_popcountll(B[w * n + v]);
    uint64_t cov = 0;
    for (int32_t t = 0; t < k; t++) {
        int32_t best = -1;
        for (int32_t v = 0; v < n; v++) {
            if (sel[v]) continue;
            if (best < 0 || h[v] > h[best]) best = v;
        }
        seeds[t] = best;
        gains[t] = h[best];
        cov += h[best];
        sel[best] = 1;
        for (int64_t w = 0; w < nw; w++) urow[w] = B[w * n + best];
        for (int32_t v = 0; v < n; v++) {
            if (del[v]) continue;
            uint64_t c = 0;
            for (int64_t w = 0; w < nw; w++) {
                uint64_t x = B[w * n + v];
                x = x & (x ^ urow[w]);  /* SUBTRACT */
                B[w * n + v] = x;
                c += (uint64_t)__builtin_popcountll(x);
            }
            h[v] = c;
            if (c == 0) del[v] = 1;
        }
    }
    *coverage = cov;
    if (after) memcpy(after, B, sizeof(uint64_t) * (size_t)(nw * n));
    free(B); free(h); free(del); free(sel); free(urow);
    return 0;
}

/* Accessors for the Python side */
void orc_encoded_info(const orc_encoded *e, int64_t *info) {
    info[0] = e->enc; info[1] = e->n; info[2] = e->nsets; info[3] = e->W; info[4] = e->nhot; info[5] = e->nwords;
    info[6] = e->cold_off ? e->cold_off[e->nsets] : 0;
    info[7] = e->ustar_enc; info[8] = e->wbits;
    info[9] = e->bitoff ? e->bitoff[e->nsets] : 0;
    info[10] = e->npayload; info[11] = e->n_escapes; info[12] = e->n_coded; info[13] = e->maxlen;
    info[14] = e->nar; info[15] = e->nchunks;
    info[16] = (e->nar > 0 && e->nchunks > 0) ? e->ar_off[e->nchunks * ((int64_t)e->nar + 1) - 1] : 0;
}
const int32_t *orc_encoded_ar_hot(const orc_encoded *e) { return e->ar_hot; }
const int64_t *orc_encoded_ar_off(const orc_encoded *e) { return e->ar_off; }
const uint16_t *orc_encoded_ar_low(const orc_encoded *e) { return e->ar_low; }
const uint64_t *orc_encoded_warm(const orc_encoded *e) { return e->warm; }
const int32_t *orc_encoded_hot(const orc_encoded *e) { return e->hot; }
const uint64_t *orc_encoded_bitmap(const orc_encoded *e) { return e->bitmap; }
const int64_t *orc_encoded_cold_off(const orc_encoded *e) { return e->cold_off; }
const int32_t *orc_encoded_cold_mem(const orc_encoded *e) { return e->cold_mem; }
const uint8_t *orc_encoded_lens(const orc_encoded *e) { return e->lens; }
const uint32_t *orc_encoded_codes(const orc_encoded *e) { return e->codes; }
const int64_t *orc_encoded_bitoff(const orc_encoded *e) { return e->bitoff; }
const uint32_t *orc_encoded_payload(const orc_encoded *e) { return e->payload; }

/* Decode set j back to ascending ids (plain bit-by-bit walk of the code tree). */
static uint32_t get_bit(const uint32_t *buf, uint64_t pos) { return (buf[pos >> 5] >> (31 - (pos & 31))) & 1u; }

int64_t orc_decode_set(const orc_encoded *e, int64_t j, int32_t *out) {
    int64_t len = 0;
    if (e->nhot > 0) {
        for (int32_t r = 0; r < e->nhot; r++)
            if ((e->bitmap[(j / 64) * e->nhot + r] >> (j % 64)) & 1ull) out[len++] = e->hot[r];
    }
    if (e->nar > 0) {  /* array rows: linear search of each row's offsets in j's chunk */
        int64_t ch = j / 65536;
        uint16_t low = (uint16_t)(j % 65536);
        const int64_t *o = e->ar_off + ch * ((int64_t)e->nar + 1);
        for (int32_t a = 0; a < e->nar; a++)
            for (int64_t i = o[a]; i < o[a + 1]; i++)
                if (e->ar_low[i] == low) { out[len++] = e->ar_hot[a]; break; }
    }
    if (e->cold_off) {
        for (int64_t i = e->cold_off[j]; i < e->cold_off[j + 1]; i++) out[len++] = e->cold_mem[i];
    } else if (e->bitoff) {
        uint64_t pos = (uint64_t)e->bitoff[j], end = (uint64_t)e->bitoff[j + 1];
        int L = 0;
        while (get_bit(e->payload, pos) == 0) { L++; pos++; }
        uint64_t g = 0;
        for (int b = 0; b <= L; b++) g = (g << 1) | get_bit(e->payload, pos++);
        uint64_t nesc = g - 1;
        for (uint64_t q = 0; q < nesc; q++) {
            uint32_t v = 0;
            for (int b = 0; b < e->wbits; b++) v = (v << 1) | get_bit(e->payload, pos++);
            out[len++] = (int32_t)v;
        }
        /* (length, code) -> symbol by linear search over the codebook: plain and slow */
        while (pos < end) {
            uint32_t code = 0;
            int clen = 0;
            int32_t sym = -1;
            while (sym < 0) {
                code = (code << 1) | get_bit(e->payload, pos++);
                clen++;
                if (clen > 32) return -1;
                for (int32_t v = 0; v < e->n; v++)
                    if (e->lens[v] == clen && e->codes[v] == code) { sym = v; break; }
            }
            out[len++] = sym;
        }
        if (pos != end) return -1;
    }
    if (e->implicit_roots) {  /* the root, unless its bitmap row already gave it */
        int32_t r = orc_root(e->n, e->seed, (uint64_t)j);
        int in_row = 0;
        for (int32_t q = 0; q < e->nhot; q++) in_row |= e->hot[q] == r;
        for (int32_t q = 0; q < e->nar; q++) in_row |= e->ar_hot[q] == r;
        if (!in_row) out[len++] = r;
    }
    qsort(out, (size_t)len, sizeof(int32_t), cmp_i32);
    return len;
}
