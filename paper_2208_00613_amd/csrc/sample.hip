// sample.hip -- RR-set sampling on the transposed graph (the sampling step of IMM:
// a randomized BFS in which only live in-edges enter the next frontier).
//
// IC (Background, IC model): in-edge e of v is live iff (word >> 8) < thr, with
// word = component e%4 of Philox(seed; j, e/4, tag 1).  The RR set is every
// vertex that reaches the root over live edges; because each coin is keyed by
// (j, e) alone, the set is independent of visit order, thread mapping or tier.
// LT (live-edge form of the LT model): vertex cur keeps in-edge e, the first
// whose running in-weight exceeds (word0 >> 8) / 2^24 of Philox(seed; j, cur,
// tag 2), or none; the reverse walk stops at none or at a repeated vertex.
//
// Tiers (each takes the sets the previous one gave up on).  IC: a wave per set with its
// visited set in an LDS hash and its queue in LDS, a frontier batch flattened into groups of
// four in-edges (one Philox call each) over the lanes, up to a group budget (k_ic_t1); a
// workgroup per set with an LDS hash and a 2048-member queue that keeps each member's
// in-edge range, threshold and first Philox group (k_big_lds<., 2048, .>; on large graphs a
// 1024-member one with four workgroups per CU in front, whose spilled levels it resumes); an extra-large
// pass of one 1024-thread workgroup per CU with room for 8192 members, their in-edge records
// in device memory beside it (k_big_lds<1024, 8192, 14>), which goes on from the BFS levels
// the 2048-member tier completed and spilled when the set outgrew it; a workgroup per set with a visited
// bitmap over V and a bounded device queue (k_big), which goes on in turn from the levels the
// extra-large pass spilled; and, for sets past that queue, slots
// with full n-entry queues.  LT: a lane per walk with its path in LDS, refilled from a list
// dealt to the lanes; a wave per walk with a 2048-step LDS path; then k_big and the slots.
//
// Every finished set is sorted ascending (its canonical form) and written to a
// scratch arena; pos[b] / size[b] record where.  Block offsets that found no
// arena space are marked POS_OVF and the lowest such offset is reported: the
// caller keeps the completed prefix of the block and resamples the rest.
#include "hbm_device.h"
#include "hbm_internal.h"

namespace hbm {

constexpr uint32_t EMPTY = 0xFFFFFFFFu;

struct SampleArgs {
    const int64_t *in_ptr;
    const int32_t *in_src;
    const uint4 *in_rec;    // per in-edge {source, its in-edge range, its WC threshold (IC) or thr[e] (LT)}
    const uint32_t *thr;
    const uint32_t *guide;  // LT cut-point index
    int32_t n;
    int wc;          // thresholds per vertex (IC-WC)
    uint64_t seed;
    int64_t j0;      // first set index of the block
    int64_t nb;      // sets in the block
    uint32_t *mem;   // scratch arena
    uint64_t cap;    // arena entries
    uint32_t *pos;
    uint32_t *size;
    unsigned long long *ctrl;
    uint32_t *defer;   // deferred block offsets (tier 1 -> tier 2)
    uint64_t gbudget;  // edge groups a tier-1 wave may expand per set (0 = no limit)
    unsigned long long *dctr;  // work counters (DC_*), or null
    uint32_t *defer2;  // deferred block offsets (tier 2 -> tier 3)
    uint32_t *defer3;  // sets that outgrew a big-set slot's queue (-> the huge pass)
    uint32_t slice;    // IC tier 1: arena entries each wave owns from the start (0 = none)
    uint32_t deal;     // IC tier 1: sets dealt to the waves in turn (1) or taken from CW_NEXT (0)
};

__device__ __forceinline__ uint32_t hash32(uint32_t v, int bits) { return (v * 0x9E3779B1u) >> (32 - bits); }

// Wave-wide bitonic sort of a[0..P) in LDS (P a power of two, pads hold EMPTY).
__device__ void wave_bitonic(uint32_t *a, int P, unsigned lane) {
    for (int k = 2; k <= P; k <<= 1) {
        for (int jj = k >> 1; jj > 0; jj >>= 1) {
            for (int i = lane; i < P; i += WAVE) {
                int ixj = i ^ jj;
                if (ixj > i) {
                    uint32_t x = a[i], y = a[ixj];
                    bool up = (i & k) == 0;
                    if ((x > y) == up) {
                        a[i] = y;
                        a[ixj] = x;
                    }
                }
            }
            wave_sync();
        }
    }
}

// Block-wide bitonic sort (blockDim threads, __syncthreads between stages).
__device__ void block_bitonic(uint32_t *a, int P) {
    for (int k = 2; k <= P; k <<= 1) {
        for (int jj = k >> 1; jj > 0; jj >>= 1) {
            for (int i = threadIdx.x; i < P; i += blockDim.x) {
                int ixj = i ^ jj;
                if (ixj > i) {
                    uint32_t x = a[i], y = a[ixj];
                    bool up = (i & k) == 0;
                    if ((x > y) == up) {
                        a[i] = y;
                        a[ixj] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
}

__device__ __forceinline__ int pow2_at_least(int s) {
    int P = 1;
    while (P < s) P <<= 1;
    return P;
}

// Per-wave arena cursor: chunks of the arena are claimed with one atomic each.
struct WaveArena {
    uint64_t cur = 0, end = 0;
};
constexpr uint64_t ARENA_CHUNK = 4096;
constexpr uint32_t T1_SLICE = 256;  // arena entries each IC tier-1 wave starts with

// Claim `s` entries for the calling wave (wave-uniform s).  Returns false when the arena is full.
__device__ __forceinline__ bool arena_claim(WaveArena &A, uint64_t s, const SampleArgs &a, uint64_t &at) {
    if (A.cur + s > A.end) {
        uint64_t want = s > ARENA_CHUNK ? s : ARENA_CHUNK;
        uint64_t base = 0;
        if (lane_id() == 0) base = atomicAdd(&a.ctrl[CW_CURSOR], (unsigned long long)want);
        base = __shfl(base, 0, WAVE);
        if (base + want > a.cap) return false;
        A.cur = base;
        A.end = base + want;
    }
    at = A.cur;
    A.cur += s;
    return true;
}

__device__ __forceinline__ void mark_ovf(const SampleArgs &a, uint32_t b) {
    a.pos[b] = POS_OVF;
    a.size[b] = 0;
    atomicMin(&a.ctrl[CW_FIRST_OVF], (unsigned long long)b);
}

// LT: the in-edge that vertex `cur` keeps for draw r -- the first e with thr[e] > r, or e1
// when there is none -- via the cut-point index; *probes counts threshold reads.
// LT: the in-edge that a vertex with in-edges [e0, e1) keeps for draw r -- the first e with
// thr[e] > r -- via the cut-point index, read as its in-edge record (source, the source's
// in-edge range, thr[e]) so the next step needs no range load; false when it keeps none.
// *probes counts the index and record reads.
__device__ __forceinline__ bool lt_step(const SampleArgs &a, uint32_t e0, uint32_t e1, uint32_t r, uint4 &rec,
                                        uint32_t &probes) {
    if (e1 == e0) return false;
    const uint32_t d = e1 - e0;
    const uint32_t lb = d > 1 ? min(32 - __clz(d - 1), 24) : 0;
    uint32_t e = a.guide[2 * (uint64_t)e0 + (r >> (24 - lb))];
    probes++;
    for (; e < e1; e++, probes++) {
        rec = a.in_rec[e];
        if (rec.w > r) return true;
    }
    return false;
}

// ---------------------------------------------------------------------------- IC tier 1
// The queue keeps each member's in-edge range and WC threshold beside it (from the in-edge
// record that found it), so expanding a level reads no device memory before its Philox calls.
template <int HB>
struct IcT1Lds {
    static constexpr int HC = 1 << HB;
    static constexpr int QC = HC / 2;
    static constexpr int LC = 256;  // live in-edges of a batch, inserted after its Philox loop
    uint32_t h[HC];
    uint32_t q[QC];
    uint32_t qe0[QC];
    uint32_t qe1[QC];
    uint32_t qt[QC];
    uint16_t qs[QC];
    uint32_t sP[WAVE];
    uint32_t live[LC];
    uint32_t cnt;
    uint32_t ovf;
    uint32_t nlive;
};

// A launch for one job deals its sets to the waves in turn (wave w takes w, w + W, ...) and
// gives each wave its own slice of the arena: same-address device atomics are serialized
// (about 12 ns each on MI355X), and thousands of waves taking sets or arena space from one
// counter queue up long enough to hold back the record loads of the sets in flight.  A
// grouped launch (several jobs) takes sets from each job's counter instead, which balances
// the jobs' waves better there (measured).
template <int HB, int WPB>
__device__ void ic_t1_body(const SampleArgs &a, uint32_t bid, uint32_t nblk) {
    using L = IcT1Lds<HB>;
    __shared__ L lds_all[WPB];
    const unsigned lane = lane_id();
    L &S = lds_all[threadIdx.x / WAVE];
    for (int i = lane; i < L::HC; i += WAVE) S.h[i] = EMPTY;
    wave_sync();
    const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
    const uint64_t gw = (uint64_t)bid * WPB + threadIdx.x / WAVE, nw = (uint64_t)nblk * WPB;
    // member u found over in-edge e: into the hash and, if new, the queue.  Once the queue is
    // full the set is redone by tier 2; inserting stops so the table never holds more than
    // QC + 64 keys (always has free slots).
    auto insert_edge = [&](uint32_t e) {
        if (S.cnt >= (uint32_t)L::QC) {
            S.ovf = 1;
            return;
        }
        const uint4 r = a.in_rec[e];
        const uint32_t u = r.x;
        uint32_t hs = hash32(u, HB);
        for (;;) {
            const uint32_t old = atomicCAS(&S.h[hs], EMPTY, u);
            if (old == EMPTY) {
                const uint32_t p = atomicAdd(&S.cnt, 1u);
                if (p < (uint32_t)L::QC) {
                    S.q[p] = u;
                    S.qe0[p] = r.y;
                    S.qe1[p] = r.z;
                    S.qt[p] = r.w;
                    S.qs[p] = (uint16_t)hs;
                } else {
                    S.ovf = 1;
                }
                return;
            }
            if (old == u) return;
            hs = (hs + 1) & (L::HC - 1);
        }
    };
    WaveArena A;
    A.cur = gw * a.slice;
    A.end = A.cur + a.slice;
    // work of completed sets (profiling): Philox calls, expanded vertices, in-edges, live edges, members
    uint64_t c_ph = 0, c_exp = 0, c_edges = 0, c_live = 0, c_mem = 0;
    {
        // the set after b (~0: the first): dealt, or from the counter in ranges of `step`
        const uint64_t step = a.nb >= 65536 ? 8 : 1;
        uint64_t je = 0;
        auto take = [&](uint64_t b) -> uint64_t {
            if (a.deal) return b == ~0ull ? gw : b + nw;
            if (b != ~0ull && b + 1 < je) return b + 1;
            uint64_t x = 0;
            if (lane == 0) x = atomicAdd(&a.ctrl[CW_NEXT], (unsigned long long)step);
            x = __shfl(x, 0, WAVE);
            je = x + step < (uint64_t)a.nb ? x + step : (uint64_t)a.nb;
            return x;
        };
        for (uint64_t b = take(~0ull); b < (uint64_t)a.nb; b = take(b)) {
            const uint64_t j = (uint64_t)a.j0 + b;
            const uint32_t jlo = (uint32_t)j, jhi = (uint32_t)(j >> 32);
            const uint32_t root = rr_root(a.seed, j, (uint32_t)a.n);
            if (lane == 0) {
                uint32_t hs = hash32(root, HB);
                S.h[hs] = root;
                S.q[0] = root;
                S.qe0[0] = (uint32_t)a.in_ptr[root];
                S.qe1[0] = (uint32_t)a.in_ptr[root + 1];
                S.qt[0] = a.wc ? a.thr[root] : 0u;
                S.qs[0] = (uint16_t)hs;
                S.cnt = 1;
                S.ovf = 0;
                S.nlive = 0;
            }
            wave_sync();
            uint32_t head = 0, qsize = 1;
            uint64_t work = 0, s_exp = 0, s_edges = 0;
            uint32_t s_live = 0;
            bool ovf = false;
            while (head < qsize) {
                const uint32_t nbat = qsize - head < (uint32_t)WAVE ? qsize - head : (uint32_t)WAVE;
                uint32_t e0 = 0, e1 = 0, ng = 0;
                if (lane < nbat) {
                    e0 = S.qe0[head + lane];
                    e1 = S.qe1[head + lane];
                    ng = e1 > e0 ? ((e1 - 1) >> 2) - (e0 >> 2) + 1 : 0;
                }
                const uint32_t P = wave_incl_scan(ng);
                const uint32_t G = __shfl(P, WAVE - 1, WAVE);
                work += G;
                if (a.gbudget && work > a.gbudget) {  // heavy set: tier 2 spreads it over a whole workgroup
                    ovf = true;
                    break;
                }
                if (a.dctr) {
                    s_exp += nbat;
                    s_edges += wave_sum(e1 - e0);
                }
                S.sP[lane] = P;
                wave_sync();
                const uint32_t hb = head;  // the batch's queue entries: hb + vertex index
                head += nbat;
                uint32_t i = 0;  // vertex of this lane's group: searched only when g leaves it
                for (uint32_t base = 0; base < G; base += WAVE) {
                    const uint32_t g = base + lane;
                    if (g < G) {
                        if (S.sP[i] <= g) i = upper_bound_dev<uint32_t, uint32_t>(S.sP, i + 1, (uint32_t)WAVE, g);
                        const uint32_t excl = i ? S.sP[i - 1] : 0u;
                        const uint32_t E0 = S.qe0[hb + i], E1 = S.qe1[hb + i];
                        const uint32_t grp = (E0 >> 2) + (g - excl);
                        const uint4 y = philox10(jlo, jhi, grp, 1u, k0, k1);
                        uint4 t4;
                        if (a.wc) {
                            const uint32_t T = S.qt[hb + i];
                            t4 = make_uint4(T, T, T, T);
                        } else {
                            t4 = *reinterpret_cast<const uint4 *>(a.thr + (size_t)grp * 4);
                        }
                        const uint32_t eb = grp * 4;
#pragma unroll
                        for (uint32_t qq = 0; qq < 4; qq++) {
                            const uint32_t e = eb + qq;
                            if (e >= E0 && e < E1 && (pick4(y, qq) >> 8) < pick4(t4, qq)) {
                                s_live++;
                                // listed: the batch's records then load together
                                const uint32_t p = atomicAdd(&S.nlive, 1u);
                                if (p < (uint32_t)L::LC) S.live[p] = e;
                                else insert_edge(e);  // the list is full: insert at once
                            }
                        }
                    }
                }
                wave_sync();
                const uint32_t nl = S.nlive < (uint32_t)L::LC ? S.nlive : (uint32_t)L::LC;
                for (uint32_t x = lane; x < nl; x += WAVE) insert_edge(S.live[x]);
                wave_sync();
                if (lane == 0) S.nlive = 0;
                qsize = S.cnt;
                if (S.ovf || qsize > (uint32_t)L::QC) {
                    ovf = true;
                    break;
                }
            }
            if (ovf) {
                for (int i = lane; i < L::HC; i += WAVE) S.h[i] = EMPTY;
                if (lane == 0) {
                    a.pos[b] = POS_DEFER;
                    a.size[b] = 0;
                    const uint64_t d = atomicAdd(&a.ctrl[CW_NDEFER], 1ull);
                    a.defer[d] = (uint32_t)b;
                }
                wave_sync();
                continue;
            }
            // canonical order, then release the hash slots
            const int s = (int)qsize;
            for (int i = lane; i < s; i += WAVE) S.h[S.qs[i]] = EMPTY;
            if (s > 1) {
                const int P2 = pow2_at_least(s);
                for (int i = s + lane; i < P2; i += WAVE) S.q[i] = EMPTY;
                wave_sync();
                wave_bitonic(S.q, P2, lane);
            }
            uint64_t at = 0;
            if (!arena_claim(A, (uint64_t)s, a, at)) {
                if (lane == 0) mark_ovf(a, (uint32_t)b);
                wave_sync();
                continue;
            }
            for (int i = lane; i < s; i += WAVE) a.mem[at + i] = S.q[i];
            if (lane == 0) {
                a.pos[b] = (uint32_t)at;
                a.size[b] = (uint32_t)s;
            }
            if (a.dctr) {
                c_ph += work;
                c_exp += s_exp;
                c_edges += s_edges;
                c_live += wave_sum(s_live);
                c_mem += (uint64_t)s;
            }
            wave_sync();
        }
    }
    if (a.dctr && lane == 0) {
        atomicAdd(&a.dctr[DC_PHILOX], (unsigned long long)c_ph);
        atomicAdd(&a.dctr[DC_EXPANDED], (unsigned long long)c_exp);
        atomicAdd(&a.dctr[DC_EDGES], (unsigned long long)c_edges);
        atomicAdd(&a.dctr[DC_LIVE], (unsigned long long)c_live);
        atomicAdd(&a.dctr[DC_MEMBERS], (unsigned long long)c_mem);
    }
}

template <int HB, int WPB>
__global__ __launch_bounds__(WPB *WAVE) void k_ic_t1(SampleArgs a) {
    ic_t1_body<HB, WPB>(a, blockIdx.x, gridDim.x);
}
template <int HB, int WPB>
__global__ __launch_bounds__(WPB *WAVE) void k_ic_t1_g(GroupArgs<SampleArgs> G) {
    const uint32_t i = group_of(G.boff, G.count, blockIdx.x);
    ic_t1_body<HB, WPB>(G.args[i], blockIdx.x - G.boff[i], G.boff[i + 1] - G.boff[i]);
}

// ---------------------------------------------------------------------------- IC tier 2
constexpr int T2_THREADS = 512;
constexpr int T2_WAVES = T2_THREADS / WAVE;
constexpr int T2_SORT_CAP = 4096;  // 24 KB of LDS per block: 4 blocks (32 waves) fit a CU

// LDS-tier capacities (members) and hash sizes (log2 slots): the regular tier, the extra-large pass
constexpr int T2L_CAP = 2048;
constexpr int T2L_CAP_REGULAR = T2L_CAP;
constexpr int T2L_HASH_BITS = 13;
constexpr int T2X_CAP = 8192;
constexpr int T2X_HASH_BITS = 14;
constexpr int T2S_CAP = 1024;  // the small tier in front (large graphs): 256 threads, four per CU
constexpr int T2S_HASH_BITS = 12;

struct T2Args {
    SampleArgs a;
    uint32_t *bitmap;  // slots * words
    uint32_t *queue;   // slots * qcap
    uint64_t words;    // ceil(n / 32)
    const uint32_t *list;
    uint32_t nlist;
    int model;         // HBM_IC or HBM_LT
    uint32_t qcap;     // queue entries per slot (n for the huge-set pass)
    int can_defer;     // a set outgrowing qcap goes to the huge list (else qcap == n)
    // IC: levels the extra-large pass spilled (or null): for list entry it < rs_cap, ids
    // rs_ids[it * T2X_CAP, + n) and rs_hdr[it] = (first member of the last completed level, n)
    const uint32_t *rs_ids;
    const uint2 *rs_hdr;
    uint32_t rs_cap;
};

// Block-wide inclusive scan of one value per thread (wave shuffles + one LDS pass).
__device__ __forceinline__ uint32_t block_incl_scan(uint32_t v, uint32_t *wsum) {
    const uint32_t inc = wave_incl_scan(v);
    const int wv = threadIdx.x / WAVE;
    if (lane_id() == WAVE - 1) wsum[wv] = inc;
    __syncthreads();
    uint32_t before = 0;
    for (int w = 0; w < wv; w++) before += wsum[w];
    return inc + before;
}

// Merge the ascending runs src[lo, mid) and src[mid, hi) into dst[lo, hi) with the whole
// block: each thread writes an equal share of the output, starting where a merge-path search
// on its first output index puts it (ids are distinct, so there are no ties).
__device__ void block_merge(const uint32_t *src, uint32_t *dst, uint32_t lo, uint32_t mid, uint32_t hi) {
    const uint32_t la = mid - lo, lb = hi - mid, tot = la + lb;
    const uint32_t per = (tot + blockDim.x - 1) / blockDim.x;
    const uint32_t d0 = min(tot, threadIdx.x * per), d1 = min(tot, d0 + per);
    if (d0 >= d1) return;
    const uint32_t *A = src + lo, *B = src + mid;
    // i = how many of the first d0 outputs come from A: the first i with A[i] > B[d0 - 1 - i]
    uint32_t ilo = d0 > lb ? d0 - lb : 0, ihi = min(d0, la);
    while (ilo < ihi) {
        const uint32_t i = (ilo + ihi) / 2;
        if (A[i] < B[d0 - 1 - i]) ilo = i + 1;
        else ihi = i;
    }
    uint32_t i = ilo, k = d0 - ilo;
    for (uint32_t d = d0; d < d1; d++) dst[lo + d] = (k >= lb || (i < la && A[i] < B[k])) ? A[i++] : B[k++];
}

// Sort the s members in `queue` (device memory, s > T2_SORT_CAP) into `out`: runs of
// T2_SORT_CAP sorted in LDS, then pairwise merges between `queue` and `out`, the first run
// placed so that the last merge lands in `out`.  `queue` keeps a permutation of the set.
__device__ void block_sort_long(uint32_t *queue, uint32_t *out, uint32_t s, uint32_t *sbuf) {
    const uint32_t runs = (s + T2_SORT_CAP - 1) / T2_SORT_CAP;
    int passes = 0;
    while ((1u << passes) < runs) passes++;
    uint32_t *src = (passes & 1) ? queue : out;
    uint32_t *dst = (passes & 1) ? out : queue;
    for (uint32_t r0 = 0; r0 < s; r0 += T2_SORT_CAP) {
        const uint32_t len = min((uint32_t)T2_SORT_CAP, s - r0);
        const int P2 = pow2_at_least((int)len);
        for (int i = threadIdx.x; i < P2; i += blockDim.x) sbuf[i] = i < (int)len ? queue[r0 + i] : EMPTY;
        __syncthreads();
        block_bitonic(sbuf, P2);
        for (int i = threadIdx.x; i < (int)len; i += blockDim.x) src[r0 + i] = sbuf[i];
        __syncthreads();
    }
    for (uint32_t w = T2_SORT_CAP; w < s; w *= 2) {
        for (uint32_t lo = 0; lo < s; lo += 2 * w) block_merge(src, dst, lo, min(lo + w, s), min(lo + 2 * w, s));
        __syncthreads();
        uint32_t *t = src;
        src = dst;
        dst = t;
    }
}

// One workgroup per big set: a visited bitmap over V and a queue in device memory.
// IC: each level's frontier is taken 512 vertices at a time; their edge groups are
// spread over all threads of the block.  LT: one thread walks with the exact bitmap.
__device__ void big_body(const T2Args &t, uint32_t bid) {
    const SampleArgs &a = t.a;
    __shared__ uint32_t sP[T2_THREADS];
    __shared__ uint32_t sE0[T2_THREADS];
    __shared__ uint32_t sE1[T2_THREADS];
    __shared__ uint32_t sT[T2_THREADS];
    __shared__ uint32_t wsum[T2_WAVES];
    __shared__ uint32_t sort_buf[T2_SORT_CAP];
    __shared__ uint32_t qn;
    __shared__ uint32_t item;
    __shared__ unsigned long long s_at;
    __shared__ int s_ok;
    __shared__ unsigned long long s_ctr[DC_COUNT];
    uint32_t *bm = t.bitmap + (uint64_t)bid * t.words;
    uint32_t *queue = t.queue + (uint64_t)bid * (uint64_t)t.qcap;
    const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
    if (threadIdx.x < DC_COUNT) s_ctr[threadIdx.x] = 0;
    for (;;) {
        if (threadIdx.x == 0) item = (uint32_t)atomicAdd(&a.ctrl[CW_NEXT2], 1ull);
        __syncthreads();
        const uint32_t it = item;
        __syncthreads();
        if (it >= t.nlist) break;
        const uint32_t b = t.list[it];
        const uint64_t j = (uint64_t)a.j0 + b;
        const uint32_t jlo = (uint32_t)j, jhi = (uint32_t)(j >> 32);
        const uint32_t root = rr_root(a.seed, j, (uint32_t)a.n);
        // IC: go on from the levels the extra-large pass completed, when they fit the queue
        uint32_t r_lo = 0;
        bool resumed = false;
        if (t.model == HBM_IC && t.rs_ids && it < t.rs_cap) {
            const uint2 hd = t.rs_hdr[it];
            if (hd.y <= t.qcap) {
                const uint32_t *src = t.rs_ids + (size_t)it * T2X_CAP;
                for (uint32_t x = threadIdx.x; x < hd.y; x += T2_THREADS) {
                    const uint32_t v = src[x];
                    queue[x] = v;
                    atomicOr(&bm[v >> 5], 1u << (v & 31));
                }
                if (threadIdx.x == 0) qn = hd.y;
                r_lo = hd.x;
                resumed = true;
            }
        }
        if (!resumed && threadIdx.x == 0) {
            bm[root >> 5] |= 1u << (root & 31);
            queue[0] = root;
            qn = 1;
        }
        __syncthreads();
        if (t.model == HBM_IC) {
            uint32_t head = r_lo;
            uint32_t tail = qn;
            while (head < tail && tail <= t.qcap) {
                for (uint32_t c0 = head; c0 < tail; c0 += T2_THREADS) {
                    const uint32_t cn = tail - c0 < (uint32_t)T2_THREADS ? tail - c0 : (uint32_t)T2_THREADS;
                    uint32_t e0 = 0, e1 = 0, ng = 0, tv = 0;
                    if (threadIdx.x < cn) {
                        const uint32_t v = queue[c0 + threadIdx.x];
                        e0 = (uint32_t)a.in_ptr[v];
                        e1 = (uint32_t)a.in_ptr[v + 1];
                        ng = e1 > e0 ? ((e1 - 1) >> 2) - (e0 >> 2) + 1 : 0;
                        if (a.wc) tv = a.thr[v];
                    }
                    const uint32_t P = block_incl_scan(ng, wsum);
                    sP[threadIdx.x] = P;
                    sE0[threadIdx.x] = e0;
                    sE1[threadIdx.x] = e1;
                    sT[threadIdx.x] = tv;
                    __syncthreads();
                    const uint32_t G = sP[T2_THREADS - 1];
                    if (a.dctr) {
                        if (threadIdx.x == 0) {
                            s_ctr[DC_PHILOX] += G;
                            s_ctr[DC_EXPANDED] += cn;
                        }
                        if (e1 > e0) atomicAdd(&s_ctr[DC_EDGES], (unsigned long long)(e1 - e0));
                    }
                    uint32_t i = 0;  // vertex of this thread's group: searched only when g leaves it
                    for (uint32_t g = threadIdx.x; g < G; g += T2_THREADS) {
                        if (sP[i] <= g) i = upper_bound_dev<uint32_t, uint32_t>(sP, i + 1, cn, g);
                        const uint32_t excl = i ? sP[i - 1] : 0u;
                        const uint32_t E0 = sE0[i], E1 = sE1[i];
                        const uint32_t grp = (E0 >> 2) + (g - excl);
                        const uint4 y = philox10(jlo, jhi, grp, 1u, k0, k1);
                        uint4 t4;
                        if (a.wc) {
                            const uint32_t T = sT[i];
                            t4 = make_uint4(T, T, T, T);
                        } else {
                            t4 = *reinterpret_cast<const uint4 *>(a.thr + (size_t)grp * 4);
                        }
                        const uint32_t eb = grp * 4;
#pragma unroll
                        for (uint32_t qq = 0; qq < 4; qq++) {
                            const uint32_t e = eb + qq;
                            if (e >= E0 && e < E1 && (pick4(y, qq) >> 8) < pick4(t4, qq)) {
                                const uint32_t u = (uint32_t)a.in_src[e];
                                if (a.dctr) atomicAdd(&s_ctr[DC_LIVE], 1ull);
                                const uint32_t bit = 1u << (u & 31);
                                const uint32_t old = atomicOr(&bm[u >> 5], bit);
                                if (!(old & bit)) {
                                    const uint32_t p = atomicAdd(&qn, 1u);
                                    if (p < t.qcap) queue[p] = u;  // else the set is redone with a full queue
                                }
                            }
                        }
                    }
                    __syncthreads();
                }
                head = tail;
                tail = qn;
                __syncthreads();
            }
        } else if (threadIdx.x == 0) {
            // LT walk with an exact visited bitmap
            uint32_t cur = root, len = 1;
            uint32_t e0 = (uint32_t)a.in_ptr[root], e1 = (uint32_t)a.in_ptr[root + 1];
            for (;;) {
                const uint4 y = philox10(jlo, jhi, cur, 2u, k0, k1);
                const uint32_t r = y.x >> 8;
                uint32_t probes = 0;
                uint4 rec;
                const bool kept = lt_step(a, e0, e1, r, rec, probes);
                if (a.dctr) {
                    s_ctr[DC_PHILOX] += 1;
                    s_ctr[DC_EXPANDED] += 1;
                    s_ctr[DC_PROBES] += probes;
                }
                if (!kept) break;
                const uint32_t s = rec.x;
                e0 = rec.y;
                e1 = rec.z;
                const uint32_t bit = 1u << (s & 31);
                if (bm[s >> 5] & bit) break;
                bm[s >> 5] |= bit;
                if (len >= t.qcap) {  // the walk outgrew the queue: redone with a full one
                    len++;
                    break;
                }
                queue[len++] = s;
                cur = s;
            }
            qn = len;
        }
        __syncthreads();
        if (qn > t.qcap) {
            // outgrew this slot's queue (only when can_defer): the visited bits of dropped members
            // are not in the queue, so clear the whole bitmap and hand the set to the huge pass
            for (uint64_t w = threadIdx.x; w < t.words; w += T2_THREADS) bm[w] = 0u;
            if (threadIdx.x == 0) {
                const uint64_t d = atomicAdd(&a.ctrl[CW_NHUGE], 1ull);
                a.defer3[d] = b;
            }
            __syncthreads();
            continue;
        }
        const uint32_t s = qn;
        if (threadIdx.x == 0) {
            s_ctr[DC_MEMBERS] += s;
            const unsigned long long at = atomicAdd(&a.ctrl[CW_CURSOR], (unsigned long long)s);
            s_at = at;
            s_ok = at + s <= a.cap;
        }
        __syncthreads();
        const uint64_t at = s_at;
        if (s_ok) {
            if ((int)s <= T2_SORT_CAP) {
                const int P2 = pow2_at_least((int)s);
                for (int i = threadIdx.x; i < P2; i += T2_THREADS) sort_buf[i] = i < (int)s ? queue[i] : EMPTY;
                __syncthreads();
                block_bitonic(sort_buf, P2);
                for (int i = threadIdx.x; i < (int)s; i += T2_THREADS) a.mem[at + i] = sort_buf[i];
            } else {
                block_sort_long(queue, a.mem + at, s, sort_buf);
            }
            if (threadIdx.x == 0) {
                a.pos[b] = (uint32_t)at;
                a.size[b] = s;
            }
        } else if (threadIdx.x == 0) {
            mark_ovf(a, b);
        }
        __syncthreads();
        // release the visited bits
        for (uint32_t i = threadIdx.x; i < s; i += T2_THREADS) bm[queue[i] >> 5] = 0u;
        __syncthreads();
    }
    if (a.dctr && threadIdx.x < DC_COUNT && s_ctr[threadIdx.x]) atomicAdd(&a.dctr[threadIdx.x], s_ctr[threadIdx.x]);
}

// IC sets with few members but heavy expansions (hubs of large in-degree): one workgroup of
// NT threads (256, 512 or 1024) per set with its visited set in an LDS hash and its queue in
// LDS, so a BFS level costs two dependent device loads (offsets, then sources) instead of four.
// A set that outgrows a tier's queue clears the hash, spills the levels it completed and
// moves on to the next capacity: on large graphs a 1024-member tier first (hash of 4096 slots,
// 38 KB, four 256-thread workgroups per CU); the regular tier of 2048 members (hash of 8192
// slots, 76-78 KB, two workgroups per CU); an extra-large pass of 8192 (hash of 16384 slots,
// 156 KB, one 1024-thread workgroup per CU); and only sets beyond that reach the
// device-bitmap tier (k_big).  The hash never holds more than CAP + NT keys.

struct T2LArgs {
    SampleArgs a;
    const uint32_t *list;
    uint32_t nlist;
    uint32_t *ovf_list;  // where sets that outgrow the LDS queue go
    int ovf_cw;          // control word counting them
    uint4 *xmeta;        // extra-large pass: CAP member records per workgroup of the launch
    // spilled levels (or null): a tier of LDS-resident records writes, for entry d < sp_cap of
    // its overflow list, the members of the BFS levels it had completed with their in-edge
    // records (CAP records from sp_rec + d * CAP) and sp_hdr[d] = (first member of the last
    // completed level, members); the next pass resumes entry d there
    uint4 *sp_rec;
    uint2 *sp_hdr;
    uint32_t sp_cap;
    // this pass's input spill (or null): list entry it < rin_cap resumes from the previous
    // pass's slot it (records from rin + it * rin_stride, header rin_hdr[it])
    const uint4 *rin;
    const uint2 *rin_hdr;
    uint32_t rin_cap;
    uint32_t rin_stride;
    // the extra-large pass's own overflow, spilled the same way for the device-bitmap tier
    // (ids only: T2X_CAP from xs_ids + d * T2X_CAP, header xs_hdr[d]; see T2Args::rs_ids)
    uint32_t *xs_ids;
    uint2 *xs_hdr;
    uint32_t xs_cap;
};

// META: the queue keeps each member's in-edge range and WC threshold beside it, taken from the
// in-edge record that found it, and the offset of its first Philox group among the set's
// groups, reserved with its queue slot by one 64-bit LDS atomic (members << 32 | groups), so a
// level reads no device memory before its Philox calls and needs no prefix sum (the regular
// capacity; the extra-large one has no LDS left for it, loads the ranges and scans per batch).
// Live in-edges of a level are listed in LDS and inserted after its Philox loop, so that their
// records load together.
template <int NT, int CAP, int HBITS>
__device__ void big_lds_body(const T2LArgs &t) {
    constexpr int T2L_HASH = 1 << HBITS;
    constexpr int T2L_HASH_BITS = HBITS;
    constexpr int T2L_CAP = CAP;
    constexpr bool META = CAP != T2X_CAP;  // the member records fit in LDS
    const SampleArgs &a = t.a;
    __shared__ uint32_t h[T2L_HASH];
    __shared__ uint32_t q[T2L_CAP];
    __shared__ uint32_t qe0[META ? T2L_CAP : 1];
    __shared__ uint32_t qe1[META ? T2L_CAP : 1];
    __shared__ uint32_t qt[META ? T2L_CAP : 1];
    __shared__ uint32_t qg[META ? T2L_CAP : 1];
    __shared__ unsigned long long qpack;  // META: members << 32 | their Philox groups
    __shared__ uint32_t sP[META ? 1 : NT];
    __shared__ uint32_t sE0[META ? 1 : NT];
    __shared__ uint32_t sE1[META ? 1 : NT];
    __shared__ uint32_t sT[META ? 1 : NT];
    __shared__ uint32_t wsum[NT / WAVE];
    constexpr uint32_t LIVE_CAP = META ? NT : 2 * NT;
    __shared__ uint32_t live[LIVE_CAP];
    __shared__ uint32_t nlive[2];  // by level parity: one is cleared while the other is read
    __shared__ uint32_t qn;        // members (the extra-large pass)
    __shared__ uint32_t item;
    __shared__ int ovf;
    __shared__ unsigned long long s_at;
    __shared__ int s_ok;
    __shared__ unsigned long long s_ctr[DC_COUNT];
    const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
    if (threadIdx.x < DC_COUNT) s_ctr[threadIdx.x] = 0;
    for (int i = threadIdx.x; i < T2L_HASH; i += NT) h[i] = EMPTY;
    // extra-large pass: the queue's in-edge records live in device memory (no LDS left for
    // them), this workgroup's CAP slots of the launch's buffer; a level's batch then reads each
    // member's range and threshold with one load that the workgroup itself wrote (L2), where it
    // read the member's in_ptr pair and threshold (two dependent loads from HBM)
    uint4 *const xm = META ? nullptr : t.xmeta + (size_t)blockIdx.x * (size_t)T2L_CAP;
    auto members = [&]() -> uint32_t {
        if constexpr (META) return (uint32_t)(qpack >> 32);
        else return qn;
    };
    // member u found over in-edge e: into the hash and, if new, the queue.  A full queue sends
    // the set on and stops inserting, so the hash never holds more than T2L_CAP + NT keys (one
    // insert per thread in flight).
    auto insert_edge = [&](uint32_t e) {
        if (members() >= (uint32_t)T2L_CAP) {
            ovf = 1;
            return;
        }
        const uint4 r = a.in_rec[e];
        const uint32_t u = r.x;
        uint32_t hs = hash32(u, T2L_HASH_BITS);
        for (;;) {
            const uint32_t old = atomicCAS(&h[hs], EMPTY, u);
            if (old == EMPTY) {
                uint32_t p;
                if constexpr (META) {
                    const uint32_t ng = r.z > r.y ? ((r.z - 1) >> 2) - (r.y >> 2) + 1 : 0;
                    const unsigned long long o = atomicAdd(&qpack, (1ull << 32) | ng);
                    p = (uint32_t)(o >> 32);
                    if (p < (uint32_t)T2L_CAP) {
                        qe0[p] = r.y;
                        qe1[p] = r.z;
                        qt[p] = r.w;
                        qg[p] = (uint32_t)o;
                    }
                } else {
                    p = atomicAdd(&qn, 1u);
                    if (p < (uint32_t)T2L_CAP) xm[p] = r;
                }
                if (p < (uint32_t)T2L_CAP) q[p] = u;
                else ovf = 1;
                return;
            }
            if (old == u) return;
            hs = (hs + 1) & (T2L_HASH - 1);
        }
    };
    // the live in-edges among the four slots of Philox group grp (words y) of a member with
    // in-edge range [E0, E1) and threshold T (WC)
    auto live_of = [&](uint32_t grp, const uint4 &y, uint32_t E0, uint32_t E1, uint32_t T, uint32_t &nl) {
        const uint4 t4 = a.wc ? make_uint4(T, T, T, T) : *reinterpret_cast<const uint4 *>(a.thr + (size_t)grp * 4);
        const uint32_t eb = grp * 4;
#pragma unroll
        for (uint32_t qq = 0; qq < 4; qq++) {
            const uint32_t e = eb + qq;
            if (e >= E0 && e < E1 && (pick4(y, qq) >> 8) < pick4(t4, qq)) {
                if (a.dctr) atomicAdd(&s_ctr[DC_LIVE], 1ull);
                const uint32_t p = atomicAdd(&nl, 1u);
                if (p < LIVE_CAP) live[p] = e;
                else insert_edge(e);  // the list is full: insert at once
            }
        }
    };
    // Groups [g, gend) of a level (or batch), one contiguous range per thread: the member of a
    // group is found once by binary search (mem_of), then by stepping forward (next_member), and
    // two groups' Philox calls are issued together so that each thread keeps two independent
    // chains of multiplies in flight.  mem_of(g) -> (member index); member(i, E0, E1, T, first
    // group) reads a member's range, threshold and first group; mend(i) is its groups' end.
    auto expand_range = [&](uint32_t jlo, uint32_t jhi, uint32_t g, uint32_t gend, uint32_t i, auto member,
                            auto mend, uint32_t &nl) {
        uint32_t E0, E1, T, gs;
        member(i, E0, E1, T, gs);
        uint32_t ie = mend(i);
        for (; g + 1 < gend; g += 2) {
            while (ie <= g) {
                ++i;
                member(i, E0, E1, T, gs);
                ie = mend(i);
            }
            const uint32_t ga = (E0 >> 2) + (g - gs);
            const uint32_t Ea0 = E0, Ea1 = E1, Ta = T;
            while (ie <= g + 1) {
                ++i;
                member(i, E0, E1, T, gs);
                ie = mend(i);
            }
            const uint32_t gb2 = (E0 >> 2) + (g + 1 - gs);
            const uint4 ya = philox10(jlo, jhi, ga, 1u, k0, k1);
            const uint4 yb = philox10(jlo, jhi, gb2, 1u, k0, k1);
            live_of(ga, ya, Ea0, Ea1, Ta, nl);
            live_of(gb2, yb, E0, E1, T, nl);
        }
        if (g < gend) {
            while (ie <= g) {
                ++i;
                member(i, E0, E1, T, gs);
                ie = mend(i);
            }
            const uint32_t ga = (E0 >> 2) + (g - gs);
            live_of(ga, philox10(jlo, jhi, ga, 1u, k0, k1), E0, E1, T, nl);
        }
    };
    __syncthreads();
    for (;;) {
        if (threadIdx.x == 0) item = (uint32_t)atomicAdd(&a.ctrl[CW_NEXT2], 1ull);
        __syncthreads();
        const uint32_t it = item;
        __syncthreads();
        if (it >= t.nlist) break;
        const uint32_t b = t.list[it];
        const uint64_t j = (uint64_t)a.j0 + b;
        const uint32_t jlo = (uint32_t)j, jhi = (uint32_t)(j >> 32);
        const uint32_t root = rr_root(a.seed, j, (uint32_t)a.n);
        // a set whose completed levels the previous pass spilled resumes there: members
        // [0, r_n) with their records, level [r_lo, r_n) to expand next
        uint32_t r_lo = 0, r_n = 1;
        bool resumed = false;
        if (t.rin && it < t.rin_cap) {
            const uint2 hd = t.rin_hdr[it];
            r_lo = hd.x;
            r_n = hd.y;
            resumed = true;
        }
        if (resumed) {
            const uint4 *src = t.rin + (size_t)it * t.rin_stride;
            for (uint32_t x = threadIdx.x; x < r_n; x += NT) {
                const uint4 r = src[x];
                q[x] = r.x;
                if constexpr (META) {
                    qe0[x] = r.y;
                    qe1[x] = r.z;
                    qt[x] = r.w;
                } else {
                    xm[x] = r;
                }
                uint32_t hs = hash32(r.x, T2L_HASH_BITS);
                while (atomicCAS(&h[hs], EMPTY, r.x) != EMPTY) hs = (hs + 1) & (T2L_HASH - 1);  // ids are distinct
            }
            if (threadIdx.x == 0) {
                if constexpr (!META) qn = r_n;
                nlive[0] = nlive[1] = 0;
                ovf = 0;
            }
            if constexpr (META) {
                // first Philox groups of the level to expand and of everything after it: only
                // members from r_lo on are expanded again
                __syncthreads();
                uint32_t carry = 0;
                for (uint32_t c0 = r_lo; c0 < r_n; c0 += NT) {
                    const uint32_t x = c0 + threadIdx.x;
                    uint32_t ng = 0;
                    if (x < r_n) {
                        const uint32_t e0 = qe0[x], e1 = qe1[x];
                        ng = e1 > e0 ? ((e1 - 1) >> 2) - (e0 >> 2) + 1 : 0u;
                    }
                    const uint32_t P = block_incl_scan(ng, wsum);
                    if (x < r_n) qg[x] = carry + P - ng;
                    for (int w = 0; w < NT / WAVE; w++) carry += wsum[w];
                    __syncthreads();  // wsum is the next chunk's
                }
                if (threadIdx.x == 0) qpack = ((unsigned long long)r_n << 32) | carry;
            }
        } else if (threadIdx.x == 0) {
            h[hash32(root, T2L_HASH_BITS)] = root;
            q[0] = root;
            if constexpr (META) {
                const uint32_t e0 = (uint32_t)a.in_ptr[root], e1 = (uint32_t)a.in_ptr[root + 1];
                qe0[0] = e0;
                qe1[0] = e1;
                qt[0] = a.wc ? a.thr[root] : 0u;
                qg[0] = 0;
                qpack = (1ull << 32) | (e1 > e0 ? ((e1 - 1) >> 2) - (e0 >> 2) + 1 : 0u);
            } else {
                qn = 1;
                xm[0] = make_uint4(root, (uint32_t)a.in_ptr[root], (uint32_t)a.in_ptr[root + 1],
                                   a.wc ? a.thr[root] : 0u);
            }
            nlive[0] = nlive[1] = 0;
            ovf = 0;
        }
        __syncthreads();
        uint32_t sp_lo = 0, sp_n = 0;  // at an overflow: the last completed level [sp_lo, sp_n)
        if constexpr (META) {
            // level [head, tail): its groups are [qg[head], the group total), every member's
            // group found by a search of qg only when a thread's group leaves its member
            uint32_t head = r_lo, lh = r_lo;
            for (uint32_t lev = 0;; lev ^= 1) {
                const unsigned long long pk = qpack;  // the previous level's inserts are done
                const uint32_t m = (uint32_t)(pk >> 32);
                const uint32_t tail = m < (uint32_t)T2L_CAP ? m : (uint32_t)T2L_CAP;
                if (ovf || head >= tail) {
                    // the level [lh, head) overflowed while it was expanded: members [0, head)
                    // are the levels up to it, all of them complete
                    sp_lo = lh;
                    sp_n = head;
                    break;
                }
                const uint32_t gb = qg[head], ge = (uint32_t)pk;
                if (a.dctr) {
                    if (threadIdx.x == 0) {
                        s_ctr[DC_PHILOX] += ge - gb;
                        s_ctr[DC_EXPANDED] += tail - head;
                    }
                    for (uint32_t x = head + threadIdx.x; x < tail; x += NT)
                        atomicAdd(&s_ctr[DC_EDGES], (unsigned long long)(qe1[x] - qe0[x]));
                }
                // thread t takes groups [gb + t per, + per)
                const uint32_t per = (ge - gb + NT - 1) / NT;
                const uint32_t g0 = gb + threadIdx.x * per;
                const uint32_t g1 = g0 + per < ge ? g0 + per : ge;
                if (g0 < g1) {
                    const uint32_t i0 = upper_bound_dev<uint32_t, uint32_t>(qg, head + 1, tail, g0) - 1;
                    expand_range(
                        jlo, jhi, g0, g1, i0,
                        [&](uint32_t i, uint32_t &E0, uint32_t &E1, uint32_t &T, uint32_t &gs) {
                            E0 = qe0[i];
                            E1 = qe1[i];
                            T = qt[i];
                            gs = qg[i];
                        },
                        [&](uint32_t i) { return i + 1 < tail ? qg[i + 1] : ge; }, nlive[lev]);
                }
                __syncthreads();
                const uint32_t nl = nlive[lev] < LIVE_CAP ? nlive[lev] : LIVE_CAP;
                for (uint32_t x = threadIdx.x; x < nl; x += NT) insert_edge(live[x]);
                if (threadIdx.x == 0) nlive[lev ^ 1] = 0;
                __syncthreads();
                lh = head;
                head = tail;
            }
        } else {
            uint32_t head = r_lo, tail = r_n, lh = r_lo;
            while (head < tail && !ovf) {
                for (uint32_t c0 = head; c0 < tail; c0 += NT) {
                    const uint32_t cn = tail - c0 < (uint32_t)NT ? tail - c0 : (uint32_t)NT;
                    uint32_t e0 = 0, e1 = 0, ng = 0, tv = 0;
                    if (threadIdx.x < cn) {
                        // the member's record, written by the insert that found it (or the root's)
                        const uint4 r = xm[c0 + threadIdx.x];
                        e0 = r.y;
                        e1 = r.z;
                        tv = r.w;
                        ng = e1 > e0 ? ((e1 - 1) >> 2) - (e0 >> 2) + 1 : 0;
                    }
                    const uint32_t P = block_incl_scan(ng, wsum);
                    sP[threadIdx.x] = P;
                    sE0[threadIdx.x] = e0;
                    sE1[threadIdx.x] = e1;
                    sT[threadIdx.x] = tv;
                    if (threadIdx.x == 0) nlive[0] = 0;
                    __syncthreads();
                    const uint32_t G = sP[NT - 1];
                    if (a.dctr) {
                        if (threadIdx.x == 0) {
                            s_ctr[DC_PHILOX] += G;
                            s_ctr[DC_EXPANDED] += cn;
                        }
                        if (e1 > e0) atomicAdd(&s_ctr[DC_EDGES], (unsigned long long)(e1 - e0));
                    }
                    // thread t takes groups [t per, + per)
                    const uint32_t per = (G + NT - 1) / NT;
                    const uint32_t g0 = threadIdx.x * per;
                    const uint32_t g1 = g0 + per < G ? g0 + per : G;
                    if (g0 < g1) {
                        const uint32_t i0 = upper_bound_dev<uint32_t, uint32_t>(sP, 0, cn, g0);
                        expand_range(
                            jlo, jhi, g0, g1, i0,
                            [&](uint32_t i, uint32_t &E0, uint32_t &E1, uint32_t &T, uint32_t &gs) {
                                E0 = sE0[i];
                                E1 = sE1[i];
                                T = sT[i];
                                gs = i ? sP[i - 1] : 0u;
                            },
                            [&](uint32_t i) { return sP[i]; }, nlive[0]);
                    }
                    __syncthreads();
                    const uint32_t nl = nlive[0] < LIVE_CAP ? nlive[0] : LIVE_CAP;
                    for (uint32_t x = threadIdx.x; x < nl; x += NT) insert_edge(live[x]);
                    __syncthreads();
                }
                lh = head;
                head = tail;
                tail = qn < (uint32_t)T2L_CAP ? qn : (uint32_t)T2L_CAP;
                __syncthreads();
            }
            sp_lo = lh;  // as in the regular tier: [0, head) are complete levels
            sp_n = head;
        }
        if (ovf) {
            for (int x = threadIdx.x; x < T2L_HASH; x += NT) h[x] = EMPTY;
            if (threadIdx.x == 0) {
                const uint64_t d = atomicAdd(&a.ctrl[t.ovf_cw], 1ull);
                t.ovf_list[d] = b;
                s_at = d;
            }
            __syncthreads();
            if constexpr (META) {
                // the completed levels, for the extra-large pass to resume from
                const uint64_t d = s_at;
                if (t.sp_rec && d < (uint64_t)t.sp_cap) {
                    uint4 *dst = t.sp_rec + (size_t)d * T2L_CAP;
                    for (uint32_t x = threadIdx.x; x < sp_n; x += NT) dst[x] = make_uint4(q[x], qe0[x], qe1[x], qt[x]);
                    if (threadIdx.x == 0) t.sp_hdr[d] = make_uint2(sp_lo, sp_n);
                }
                __syncthreads();  // q and the records are the next set's
            } else {
                const uint64_t d = s_at;
                if (t.xs_ids && d < (uint64_t)t.xs_cap) {
                    uint32_t *dst = t.xs_ids + (size_t)d * T2L_CAP;
                    for (uint32_t x = threadIdx.x; x < sp_n; x += NT) dst[x] = q[x];
                    if (threadIdx.x == 0) t.xs_hdr[d] = make_uint2(sp_lo, sp_n);
                }
                __syncthreads();
            }
            continue;
        }
        const uint32_t s = members();
        if (threadIdx.x == 0) {
            s_ctr[DC_MEMBERS] += s;
            const unsigned long long at = atomicAdd(&a.ctrl[CW_CURSOR], (unsigned long long)s);
            s_at = at;
            s_ok = at + s <= a.cap;
        }
        // canonical order: sort the members in LDS (pads hold EMPTY, above every id)
        const int P2 = pow2_at_least((int)s);
        for (int x = (int)s + threadIdx.x; x < P2; x += NT) q[x] = EMPTY;
        __syncthreads();
        if (s > 1) block_bitonic(q, P2);
        const uint64_t at = s_at;
        if (s_ok) {
            for (int x = threadIdx.x; x < (int)s; x += NT) a.mem[at + x] = q[x];
            if (threadIdx.x == 0) {
                a.pos[b] = (uint32_t)at;
                a.size[b] = s;
            }
        } else if (threadIdx.x == 0) {
            mark_ovf(a, b);
        }
        for (int x = threadIdx.x; x < T2L_HASH; x += NT) h[x] = EMPTY;
        __syncthreads();
    }
    if (a.dctr && threadIdx.x < DC_COUNT && s_ctr[threadIdx.x]) atomicAdd(&a.dctr[threadIdx.x], s_ctr[threadIdx.x]);
}

template <int NT, int CAP, int HBITS>
__global__ __launch_bounds__(NT) void k_big_lds(T2LArgs t) {
    big_lds_body<NT, CAP, HBITS>(t);
}
template <int NT, int CAP, int HBITS>
__global__ __launch_bounds__(NT) void k_big_lds_g(GroupArgs<T2LArgs> G) {
    big_lds_body<NT, CAP, HBITS>(G.args[group_of(G.boff, G.count, blockIdx.x)]);
}

__global__ __launch_bounds__(T2_THREADS) void k_big(T2Args t) { big_body(t, blockIdx.x); }
__global__ __launch_bounds__(T2_THREADS) void k_big_g(GroupArgs<T2Args> G) {
    const uint32_t i = group_of(G.boff, G.count, blockIdx.x);
    big_body(G.args[i], blockIdx.x - G.boff[i]);
}

// ---------------------------------------------------------------------------- LT tier 1
// LT_LW: path capacity per lane in LDS (walks longer than this go to tier 2).  Walks are dealt
// to the lanes of the launch in turn (lane l takes l, l + L, ...): same-address device atomics
// are serialized, and a counter refilled by every wave would hold back the walks' loads.
template <int LT_LW>
__device__ void lt_t1_body(const SampleArgs &a, uint32_t bid, uint32_t nblk) {
    __shared__ uint32_t path[LT_LW * WAVE];  // path[k * WAVE + lane]
    const unsigned lane = lane_id();
    const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
    WaveArena A;
    bool active = false, exhausted = false;
    uint32_t b = 0, cur = 0, len = 0, ce0 = 0, ce1 = 0;  // ce0, ce1: cur's in-edge range
    uint64_t j = 0;
    uint64_t next = (uint64_t)bid * WAVE + lane;  // this lane's next walk
    const uint64_t stride = (uint64_t)nblk * WAVE;
    uint64_t c_steps = 0, c_probes = 0, c_mem = 0;  // per lane (profiling)
    for (;;) {
        if (!active && !exhausted) {
            if (next < (uint64_t)a.nb) {
                b = (uint32_t)next;
                j = (uint64_t)a.j0 + next;
                next += stride;
                cur = rr_root(a.seed, j, (uint32_t)a.n);
                ce0 = (uint32_t)a.in_ptr[cur];
                ce1 = (uint32_t)a.in_ptr[cur + 1];
                path[lane] = cur;
                len = 1;
                active = true;
            } else {
                exhausted = true;
            }
        }
        if (!__ballot(active)) break;
        bool finished = false, deferred = false;
        if (active) {
            const uint4 y = philox10((uint32_t)j, (uint32_t)(j >> 32), cur, 2u, k0, k1);
            const uint32_t r = y.x >> 8;
            uint32_t probes = 0;
            uint4 rec;
            const bool kept = lt_step(a, ce0, ce1, r, rec, probes);
            c_steps++;
            c_probes += probes;
            if (!kept) {
                finished = true;
            } else {
                const uint32_t s = rec.x;
                bool seen = false;
                for (uint32_t k = 0; k < len; k++) seen |= path[k * WAVE + lane] == s;
                if (seen) {
                    finished = true;
                } else if (len == (uint32_t)LT_LW) {
                    deferred = true;
                } else {
                    path[len * WAVE + lane] = s;
                    len++;
                    cur = s;
                    ce0 = rec.y;
                    ce1 = rec.z;
                }
            }
        }
        // this step's deferred walks join the list with one atomic per wave
        const uint64_t dm = __ballot(deferred);
        if (dm) {
            uint64_t base = 0;
            if (lane == 0) base = atomicAdd(&a.ctrl[CW_NDEFER], (unsigned long long)__popcll(dm));
            base = __shfl(base, 0, WAVE);
            if (deferred) {
                a.defer[base + __popcll(dm & ((1ull << lane) - 1))] = b;
                active = false;
            }
        }
        const uint64_t fin = __ballot(finished);
        if (fin) {
            if (finished) {
                // insertion sort of this lane's column
                for (uint32_t x = 1; x < len; x++) {
                    const uint32_t v = path[x * WAVE + lane];
                    int y2 = (int)x - 1;
                    while (y2 >= 0 && path[y2 * WAVE + lane] > v) {
                        path[(y2 + 1) * WAVE + lane] = path[y2 * WAVE + lane];
                        y2--;
                    }
                    path[(y2 + 1) * WAVE + lane] = v;
                }
            }
            const uint32_t mine = finished ? len : 0u;
            const uint32_t incl = wave_incl_scan(mine);
            const uint32_t tot = __shfl(incl, WAVE - 1, WAVE);
            uint64_t at = 0;
            const bool ok = arena_claim(A, tot, a, at);
            if (finished) {
                if (ok) {
                    const uint64_t o = at + incl - mine;
                    for (uint32_t x = 0; x < len; x++) a.mem[o + x] = path[x * WAVE + lane];
                    a.pos[b] = (uint32_t)o;
                    a.size[b] = len;
                    c_mem += len;
                } else {
                    mark_ovf(a, b);
                }
                active = false;
            }
        }
    }
    if (a.dctr) {
        // steps of walks that were deferred are counted too: they are the work this kernel did
        const uint64_t st = wave_sum(c_steps), pr = wave_sum(c_probes), mm = wave_sum(c_mem);
        if (lane == 0) {
            atomicAdd(&a.dctr[DC_PHILOX], (unsigned long long)st);
            atomicAdd(&a.dctr[DC_EXPANDED], (unsigned long long)st);
            atomicAdd(&a.dctr[DC_PROBES], (unsigned long long)pr);
            atomicAdd(&a.dctr[DC_MEMBERS], (unsigned long long)mm);
        }
    }
}

template <int LT_LW>
__global__ __launch_bounds__(WAVE) void k_lt_t1(SampleArgs a) {
    lt_t1_body<LT_LW>(a, blockIdx.x, gridDim.x);
}
template <int LT_LW>
__global__ __launch_bounds__(WAVE) void k_lt_t1_g(GroupArgs<SampleArgs> G) {
    const uint32_t i = group_of(G.boff, G.count, blockIdx.x);
    lt_t1_body<LT_LW>(G.args[i], blockIdx.x - G.boff[i], G.boff[i + 1] - G.boff[i]);
}

// ---------------------------------------------------------------------------- LT tier 2
// One wave per long walk: lane 0 draws and follows the walk; the path lives in LDS and
// all 64 lanes scan it for the repeat check.  Walks longer than LT2_PC go to tier 3.
constexpr int LT2_PC = 2048;

struct Lt2Args {
    SampleArgs a;
    const uint32_t *list;
    uint32_t nlist;
};

// Long walks vary widely in length: each wave takes its next walk from a counter (dealing them
// in turn was measured slower here).
__device__ void lt_wave_body(const Lt2Args &t) {
    __shared__ uint32_t path[LT2_PC];
    const SampleArgs &a = t.a;
    const unsigned lane = lane_id();
    const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
    WaveArena A;
    uint64_t c_steps = 0, c_probes = 0, c_mem = 0;  // lane 0 (profiling)
    for (;;) {
        uint64_t it = 0;
        if (lane == 0) it = atomicAdd(&a.ctrl[CW_NEXT2], 1ull);
        it = __shfl(it, 0, WAVE);
        if (it >= t.nlist) break;
        const uint32_t b = t.list[it];
        const uint64_t j = (uint64_t)a.j0 + b;
        uint32_t cur = rr_root(a.seed, j, (uint32_t)a.n);
        uint32_t ce0 = 0, ce1 = 0;  // lane 0: cur's in-edge range
        if (lane == 0) {
            path[0] = cur;
            ce0 = (uint32_t)a.in_ptr[cur];
            ce1 = (uint32_t)a.in_ptr[cur + 1];
        }
        uint32_t len = 1;
        bool ok = true;
        for (;;) {
            uint32_t s = 0, stop = 0;
            if (lane == 0) {
                const uint4 y = philox10((uint32_t)j, (uint32_t)(j >> 32), cur, 2u, k0, k1);
                uint32_t probes = 0;
                uint4 rec;
                const bool kept = lt_step(a, ce0, ce1, y.x >> 8, rec, probes);
                c_steps++;
                c_probes += probes;
                if (!kept) {
                    stop = 1;
                } else {
                    s = rec.x;
                    ce0 = rec.y;  // used only if the walk goes on to s
                    ce1 = rec.z;
                }
            }
            stop = __shfl(stop, 0, WAVE);
            if (stop) break;
            s = __shfl(s, 0, WAVE);
            wave_sync();
            bool seen = false;
            for (uint32_t q = lane; q < len; q += WAVE) seen |= path[q] == s;
            if (__ballot(seen)) break;
            if (len == (uint32_t)LT2_PC) {
                ok = false;
                break;
            }
            if (lane == 0) path[len] = s;
            len++;
            cur = s;
        }
        wave_sync();
        if (!ok) {
            if (lane == 0) {
                a.pos[b] = POS_DEFER;
                a.size[b] = 0;
                const uint64_t d = atomicAdd(&a.ctrl[CW_NDEFER], 1ull);
                a.defer2[d] = b;
            }
            continue;
        }
        const int P2 = pow2_at_least((int)len);
        for (int q = (int)len + lane; q < P2; q += WAVE) path[q] = EMPTY;
        wave_sync();
        wave_bitonic(path, P2, lane);
        uint64_t at = 0;
        if (arena_claim(A, len, a, at)) {
            for (uint32_t q = lane; q < len; q += WAVE) a.mem[at + q] = path[q];
            if (lane == 0) {
                a.pos[b] = (uint32_t)at;
                a.size[b] = len;
                c_mem += len;
            }
        } else if (lane == 0) {
            mark_ovf(a, b);
        }
        wave_sync();
    }
    if (a.dctr && lane == 0) {
        atomicAdd(&a.dctr[DC_PHILOX], (unsigned long long)c_steps);
        atomicAdd(&a.dctr[DC_EXPANDED], (unsigned long long)c_steps);
        atomicAdd(&a.dctr[DC_PROBES], (unsigned long long)c_probes);
        atomicAdd(&a.dctr[DC_MEMBERS], (unsigned long long)c_mem);
    }
}

__global__ __launch_bounds__(WAVE) void k_lt_wave(Lt2Args t) { lt_wave_body(t); }
__global__ __launch_bounds__(WAVE) void k_lt_wave_g(GroupArgs<Lt2Args> G) {
    lt_wave_body(G.args[group_of(G.boff, G.count, blockIdx.x)]);
}

__global__ void k_iota_u32(uint32_t *p, uint64_t count) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < count; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = (uint32_t)i;
}

__global__ void k_fill_u32(uint32_t *p, uint64_t count, uint32_t v) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < count; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ---------------------------------------------------------------------------- host
// Big-set slots: a visited bitmap over V and a queue of qcap = min(n, t2_queue) entries each, as
// many slots as fit the context's byte cap (at most t2_per_cu per CU).  A set larger than qcap is
// redone in the huge pass, whose few slots hold a full n-entry queue.
static uint32_t t2_qcap(const Ctx &c) { return (uint32_t)std::min<int64_t>(c.g.n, c.t2_queue); }

static void ensure_t2(Ctx &c) {
    Scratch &sc = c.sc;
    if (sc.t2_slots) return;
    const uint64_t n = (uint64_t)c.g.n;
    const uint64_t words = (n + 31) / 32;
    const uint64_t qcap = t2_qcap(c);
    int slots = c.t2_per_cu * c.num_cus;
    const uint64_t per = words * 4 + qcap * 4;
    const uint64_t cap_bytes = (uint64_t)c.t2_cap;
    while (slots > 8 && per * slots > cap_bytes) slots /= 2;
    buf_alloc(c, sc.t2_bitmap, words * 4 * slots);
    buf_zero(c, sc.t2_bitmap, 0, words * 4 * slots);
    buf_alloc(c, sc.t2_queue, qcap * 4 * slots);
    sc.t2_slots = slots;
}

// Spill slots of one sampling launch, in a buffer of the driving context: job i gets cap[i]
// slots (at most its list's length, as a slot is indexed by the next pass's list entry), after
// the previous jobs' slots; each slot holds `slot` bytes of records (or ids), and the 8-byte
// headers follow all slots.  Entries past a job's slots start over from the root.
struct SpillPlan {
    std::vector<uint32_t> cap;
    std::vector<uint64_t> base;
    size_t slot = 0;
    uint64_t total = 0;
    char *p = nullptr;
    template <class T>
    T *rec(size_t i) const { return cap[i] ? reinterpret_cast<T *>(p + base[i] * slot) : nullptr; }
    uint2 *hdr(size_t i) const {
        return cap[i] ? reinterpret_cast<uint2 *>(p + total * slot + base[i] * sizeof(uint2)) : nullptr;
    }
};
static void spill_plan(Ctx &root, Buf &buf, size_t slot, const std::vector<uint32_t> &cap, SpillPlan &P) {
    P.cap = cap;
    P.slot = slot;
    P.base.assign(cap.size(), 0);
    uint64_t t = 0;
    for (size_t i = 0; i < cap.size(); i++) {
        P.base[i] = t;
        t += cap[i];
    }
    P.total = t;
    if (t) buf_grow(root, buf, (size_t)t * (slot + sizeof(uint2)), false);
    P.p = t ? buf.as<char>() : nullptr;
}
// Slots per job: a launch's budget (the driving context's SPILL_SLOTS for the 2048-member tier,
// twice that for the 1024-member one, whose overflow is the larger, and at most 256 for the
// extra-large pass: sets past 8192 members are rare) shared among its IC jobs in proportion to
// their lists (at least 16 each), and never more than a job's list
static std::vector<uint32_t> spill_caps(const std::vector<uint64_t> &listed, int64_t budget) {
    uint64_t sum = 0;
    for (uint64_t n : listed) sum += n;
    std::vector<uint32_t> cap(listed.size(), 0);
    for (size_t i = 0; i < listed.size(); i++) {
        if (!listed[i] || budget <= 0) continue;
        const uint64_t share = std::max<uint64_t>(16, (uint64_t)((double)budget * (double)listed[i] / (double)sum));
        cap[i] = (uint32_t)std::min<uint64_t>({listed[i], share, (uint64_t)budget});
    }
    return cap;
}
static void spill_out(const SpillPlan &P, size_t i, T2LArgs &t) {
    t.sp_rec = P.rec<uint4>(i);
    t.sp_hdr = P.hdr(i);
    t.sp_cap = P.cap[i];
}
static void spill_in(const SpillPlan &P, size_t i, T2LArgs &t, uint32_t stride) {
    t.rin = P.rec<uint4>(i);
    t.rin_hdr = P.hdr(i);
    t.rin_cap = P.cap[i];
    t.rin_stride = stride;
}

static void ensure_t2_huge(Ctx &c) {
    Scratch &sc = c.sc;
    if (sc.t2h_slots) return;
    const uint64_t n = (uint64_t)c.g.n;
    const uint64_t words = (n + 31) / 32;
    const uint64_t per = words * 4 + n * 4;
    const int slots = (int)std::max<uint64_t>(1, std::min<uint64_t>(16, (uint64_t)c.t2_cap / per));
    buf_alloc(c, sc.t2h_bitmap, words * 4 * slots);
    buf_zero(c, sc.t2h_bitmap, 0, words * 4 * slots);
    buf_alloc(c, sc.t2h_queue, n * 4 * slots);
    sc.t2h_slots = slots;
}

// Algorithmic traffic of the samplers from the work counters.
//  IC, per expanded vertex: its in_ptr pair (16 B) and threshold (4 B per vertex
//  under WC, 4 B per in-edge otherwise); 4 B per live in-edge (source id); 4 B per
//  member written.  Ops: Philox calls.
//  LT, per walk step: in_ptr pair (16 B), 4 B per binary-search probe, 4 B source
//  id; 4 B per member written.  Ops: Philox calls (one per step).
static void prof_sampler(Ctx &root, int slot, bool ic, const std::vector<Ctx *> &J) {
    if (slot < 0) return;
    unsigned long long k[DC_COUNT];
    prof_read_counters(root, k);
    bool wc = true;
    for (Ctx *c : J)
        if (c->g.model == HBM_IC) wc = c->g.prob == HBM_PROB_WC;
    double bytes;
    if (ic) {
        bytes = 16.0 * k[DC_EXPANDED] + 4.0 * (wc ? k[DC_EXPANDED] : k[DC_EDGES]) + 4.0 * k[DC_LIVE] +
                4.0 * k[DC_MEMBERS];
    } else {
        bytes = 20.0 * k[DC_EXPANDED] + 4.0 * k[DC_PROBES] + 4.0 * k[DC_MEMBERS];
    }
    prof_add(root, slot, bytes, (double)k[DC_PHILOX]);
}

// control words of job i in the root's arena
static unsigned long long *ctrl_of(Ctx &root, size_t i) {
    return root.ctrl_arena.as<unsigned long long>() + i * CW_COUNT;
}

static void ctrl_push(Ctx &root) {
    HBM_HIP(hipMemcpyAsync(root.ctrl_arena.p, root.ctrl_host.data(), root.ctrl_host.size() * 8,
                           hipMemcpyHostToDevice, root.stream));
}

static void ctrl_pull(Ctx &root) {
    HBM_HIP(hipMemcpyAsync(root.ctrl_host.data(), root.ctrl_arena.p, root.ctrl_host.size() * 8,
                           hipMemcpyDeviceToHost, root.stream));
    HBM_HIP(hipStreamSynchronize(root.stream));
}

void sample_blocks(Ctx &root, const std::vector<Ctx *> &J, const std::vector<int64_t> &j0,
                   const std::vector<int64_t> &nbv, const std::vector<uint64_t> &seed, std::vector<int64_t> &done) {
    const size_t N = J.size();
    done.assign(N, 0);
    buf_grow(root, root.ctrl_arena, N * CW_COUNT * 8, false);
    root.ctrl_host.assign(N * CW_COUNT, 0ull);
    std::vector<SampleArgs> A(N);
    for (size_t i = 0; i < N; i++) {
        Ctx &c = *J[i];
        Scratch &sc = c.sc;
        HBM_REQUIRE(nbv[i] <= sc.bcap, HBM_EDEVICE, "internal: block larger than scratch index");
        root.ctrl_host[i * CW_COUNT + CW_FIRST_OVF] = (unsigned long long)nbv[i];
        SampleArgs &a = A[i];
        a.in_ptr = c.g.in_ptr.as<int64_t>();
        a.in_src = c.g.in_src.as<int32_t>();
        a.in_rec = c.g.in_rec.as<uint4>();
        a.thr = c.g.thr.as<uint32_t>();
        a.guide = c.g.guide.as<uint32_t>();
        a.n = c.g.n;
        a.wc = c.g.model == HBM_IC && c.g.prob == HBM_PROB_WC;
        a.seed = seed[i];
        a.j0 = j0[i];
        a.nb = nbv[i];
        a.mem = sc.mem.as<uint32_t>();
        a.cap = sc.cap;
        a.pos = sc.pos.as<uint32_t>();
        a.size = sc.size.as<uint32_t>();
        a.ctrl = ctrl_of(root, i);
        a.defer = sc.defer.as<uint32_t>();
        a.defer2 = sc.defer.as<uint32_t>() + sc.bcap;
        a.defer3 = sc.defer.as<uint32_t>() + 2 * sc.bcap;
        a.gbudget = (uint64_t)root.ic_t1_budget;
        a.dctr = prof_counters(root);
        if (c.g.model == HBM_IC && !root.ic_tier1) {
            // every set goes to tier 2 (one workgroup per set)
            root.ctrl_host[i * CW_COUNT + CW_NDEFER] = (unsigned long long)nbv[i];
        }
    }
    const hipStream_t st = root.stream;
    const bool profiling = root.prof.on;
    // ---- tier 1
    std::vector<SampleArgs> ic, lt;
    std::vector<uint32_t> icb, ltb;
    constexpr int WPB = 4;
    const int lw = root.lt_lw;
    int n_t1 = 0;  // IC jobs whose sets go through tier 1
    for (size_t i = 0; i < N; i++) n_t1 += nbv[i] > 0 && J[i]->g.model == HBM_IC && root.ic_tier1;
    for (size_t i = 0; i < N; i++) {
        const int64_t nb = nbv[i];
        if (nb <= 0) continue;
        if (J[i]->g.model == HBM_IC) {
            if (!root.ic_tier1) {
                k_iota_u32<<<grid_for(nb, 256, 65536), 256, 0, st>>>(A[i].defer, (uint64_t)nb);
                continue;
            }
            const uint32_t nbk = (uint32_t)std::min<int64_t>((nb + WPB - 1) / WPB, (int64_t)root.num_cus * 8);
            // arena slices for the waves (a tier-1 set has at most 256 members), when they
            // take at most half the arena; the rest is claimed from CW_CURSOR beyond them
            const uint64_t waves = (uint64_t)nbk * WPB;
            A[i].deal = n_t1 == 1;
            const uint32_t slice = A[i].deal && waves * T1_SLICE * 2 <= J[i]->sc.cap ? T1_SLICE : 0u;
            A[i].slice = slice;
            root.ctrl_host[i * CW_COUNT + CW_CURSOR] = waves * slice;
            ic.push_back(A[i]);
            icb.push_back(nbk);
        } else {
            lt.push_back(A[i]);
            ltb.push_back(
                (uint32_t)std::min<int64_t>((nb + WAVE - 1) / WAVE, (int64_t)root.num_cus * std::max(1, 640 / lw)));
        }
    }
    ctrl_push(root);
    int s1 = ic.empty() ? -1 : prof_begin(root, "ic_sample_wave");
    glaunch(root, ic, icb, 0, [&](const SampleArgs &a, unsigned g) { k_ic_t1<9, WPB><<<g, WPB * WAVE, 0, st>>>(a); },
            [&](const SampleArgs *d, const uint32_t *b, uint32_t cnt, uint32_t g, int x) {
                k_ic_t1_g<9, WPB><<<g, WPB * WAVE, 0, st>>>(GroupArgs<SampleArgs>{d, b, cnt, x});
            });
    HBM_HIP(hipGetLastError());
    prof_end(root, s1);
    if (profiling && s1 >= 0) {
        HBM_HIP(hipStreamSynchronize(st));
        prof_sampler(root, s1, true, J);
    }
    int s1b = lt.empty() ? -1 : prof_begin(root, "lt_sample_lane");
    glaunch(root, lt, ltb, 0,
            [&](const SampleArgs &a, unsigned g) {
                if (lw == 32) k_lt_t1<32><<<g, WAVE, 0, st>>>(a);
                else if (lw == 64) k_lt_t1<64><<<g, WAVE, 0, st>>>(a);
                else if (lw == 128) k_lt_t1<128><<<g, WAVE, 0, st>>>(a);
                else k_lt_t1<256><<<g, WAVE, 0, st>>>(a);
            },
            [&](const SampleArgs *d, const uint32_t *b, uint32_t cnt, uint32_t g, int x) {
                if (lw == 32) k_lt_t1_g<32><<<g, WAVE, 0, st>>>(GroupArgs<SampleArgs>{d, b, cnt, x});
                else if (lw == 64) k_lt_t1_g<64><<<g, WAVE, 0, st>>>(GroupArgs<SampleArgs>{d, b, cnt, x});
                else if (lw == 128) k_lt_t1_g<128><<<g, WAVE, 0, st>>>(GroupArgs<SampleArgs>{d, b, cnt, x});
                else k_lt_t1_g<256><<<g, WAVE, 0, st>>>(GroupArgs<SampleArgs>{d, b, cnt, x});
            });
    HBM_HIP(hipGetLastError());
    prof_end(root, s1b);
    ctrl_pull(root);
    if (s1b >= 0) prof_sampler(root, s1b, false, J);
    // ---- tier 2: IC sets on a workgroup each (visited set in LDS); LT walks on a wave each
    // LDS-tier shape: by default 1024 threads, two per CU, on graphs below 2^22 vertices
    // (heavy sets there are few and deep) and 512 threads, three per CU, above (measured)
    int gmax = 0;
    for (size_t i = 0; i < N; i++) gmax = std::max(gmax, J[i]->g.n);
    const bool small_g = gmax < (1 << 22);
    const int lds_threads = root.lds_threads ? root.lds_threads : (small_g ? 1024 : 512);
    const int lds_per_cu = root.lds_per_cu ? root.lds_per_cu : (small_g ? 2 : 3);
    // IC on large graphs: a 1024-member tier first (four 256-thread workgroups per CU where the
    // 2048-member one fits two), whose overflow list `defer2` the 2048-member tier takes, with
    // the levels it spilled; that tier's overflow then goes to `defer3` for the extra-large pass
    const bool chain = root.lds_small == 1 || (root.lds_small == 2 && !small_g);
    SpillPlan sp0, sp1, sp2;  // 1024 -> 2048 members, 2048 -> extra-large, extra-large -> bitmap tier
    if (chain) {
        std::vector<uint64_t> listed(N, 0);
        for (size_t i = 0; i < N; i++)
            if (J[i]->g.model == HBM_IC) listed[i] = root.ctrl_host[i * CW_COUNT + CW_NDEFER];
        spill_plan(root, root.spill0, T2S_CAP * sizeof(uint4), spill_caps(listed, 2 * root.spill_slots), sp0);
        std::vector<T2LArgs> sm;
        std::vector<uint32_t> smb;
        for (size_t i = 0; i < N; i++) {
            Ctx &c = *J[i];
            const uint64_t nd = root.ctrl_host[i * CW_COUNT + CW_NDEFER];
            if (!nd || c.g.model != HBM_IC) continue;
            sm.push_back(T2LArgs{A[i], A[i].defer, (uint32_t)nd, A[i].defer2, CW_NDEFER2, nullptr});
            spill_out(sp0, i, sm.back());
            smb.push_back((uint32_t)std::min<uint64_t>(nd, (uint64_t)root.num_cus * 4));
        }
        if (!sm.empty()) {
            int s1 = prof_begin(root, "ic_sample_block_s");
            glaunch(root, sm, smb, 0,
                    [&](const T2LArgs &t, unsigned g) {
                        k_big_lds<256, T2S_CAP, T2S_HASH_BITS><<<g, 256, 0, st>>>(t);
                    },
                    [&](const T2LArgs *d, const uint32_t *b, uint32_t cnt, uint32_t g, int x) {
                        k_big_lds_g<256, T2S_CAP, T2S_HASH_BITS><<<g, 256, 0, st>>>(GroupArgs<T2LArgs>{d, b, cnt, x});
                    });
            HBM_HIP(hipGetLastError());
            prof_end(root, s1);
            ctrl_pull(root);
            if (s1 >= 0) prof_sampler(root, s1, true, J);
            for (size_t i = 0; i < N; i++)
                if (J[i]->g.model == HBM_IC) root.ctrl_host[i * CW_COUNT + CW_NEXT2] = 0;
            ctrl_push(root);
        }
    }
    std::vector<T2LArgs> lds;
    std::vector<uint32_t> ldsb;
    std::vector<Lt2Args> ltw;
    std::vector<uint32_t> ltwb;
    bool lt_deferred = false;
    {
        std::vector<uint64_t> listed(N, 0);
        for (size_t i = 0; i < N; i++)
            if (J[i]->g.model == HBM_IC) listed[i] = root.ctrl_host[i * CW_COUNT + (chain ? CW_NDEFER2 : CW_NDEFER)];
        spill_plan(root, root.spill, T2L_CAP_REGULAR * sizeof(uint4), spill_caps(listed, root.spill_slots), sp1);
    }
    for (size_t i = 0; i < N; i++) {
        Ctx &c = *J[i];
        const bool ic_chain = chain && c.g.model == HBM_IC;
        const uint64_t nd = root.ctrl_host[i * CW_COUNT + (ic_chain ? CW_NDEFER2 : CW_NDEFER)];
        if (!nd) continue;
        if (c.g.model == HBM_IC) {
            if (ic_chain) {
                lds.push_back(T2LArgs{A[i], A[i].defer2, (uint32_t)nd, A[i].defer3, CW_NDEFER3, nullptr});
                spill_in(sp0, i, lds.back(), T2S_CAP);
            } else {
                lds.push_back(T2LArgs{A[i], A[i].defer, (uint32_t)nd, A[i].defer2, CW_NDEFER2, nullptr});
            }
            spill_out(sp1, i, lds.back());
            ldsb.push_back((uint32_t)std::min<uint64_t>(nd, (uint64_t)root.num_cus * lds_per_cu));
        } else {
            root.ctrl_host[i * CW_COUNT + CW_NDEFER] = 0;  // reused as the tier-3 list length
            lt_deferred = true;
            Lt2Args t;
            t.a = A[i];
            t.list = A[i].defer;
            t.nlist = (uint32_t)nd;
            ltw.push_back(t);
            ltwb.push_back((uint32_t)std::min<uint64_t>(nd, (uint64_t)root.num_cus * 16));
        }
    }
    if (!lds.empty() || !ltw.empty()) {
        if (lt_deferred) ctrl_push(root);
        int s2 = lds.empty() ? -1 : prof_begin(root, "ic_sample_block");
        const bool wide = lds_threads == 1024;
        glaunch(root, lds, ldsb, 0,
                [&](const T2LArgs &t, unsigned g) {
                    if (wide) k_big_lds<1024, T2L_CAP, T2L_HASH_BITS><<<g, 1024, 0, st>>>(t);
                    else k_big_lds<512, T2L_CAP, T2L_HASH_BITS><<<g, 512, 0, st>>>(t);
                },
                [&](const T2LArgs *d, const uint32_t *b, uint32_t cnt, uint32_t g, int x) {
                    if (wide)
                        k_big_lds_g<1024, T2L_CAP, T2L_HASH_BITS><<<g, 1024, 0, st>>>(GroupArgs<T2LArgs>{d, b, cnt, x});
                    else k_big_lds_g<512, T2L_CAP, T2L_HASH_BITS><<<g, 512, 0, st>>>(GroupArgs<T2LArgs>{d, b, cnt, x});
                });
        HBM_HIP(hipGetLastError());
        prof_end(root, s2);
        if (profiling && s2 >= 0) {
            HBM_HIP(hipStreamSynchronize(st));
            prof_sampler(root, s2, true, J);
        }
        int s3 = ltw.empty() ? -1 : prof_begin(root, "lt_sample_wave");
        glaunch(root, ltw, ltwb, 0, [&](const Lt2Args &t, unsigned g) { k_lt_wave<<<g, WAVE, 0, st>>>(t); },
                [&](const Lt2Args *d, const uint32_t *b, uint32_t cnt, uint32_t g, int x) {
                    k_lt_wave_g<<<g, WAVE, 0, st>>>(GroupArgs<Lt2Args>{d, b, cnt, x});
                });
        HBM_HIP(hipGetLastError());
        prof_end(root, s3);
        ctrl_pull(root);
        if (s3 >= 0) prof_sampler(root, s3, false, J);
        // ---- extra-large LDS pass: IC sets past the LDS tier's 2048 members, one 1024-thread
        // workgroup per CU with room for 8192; the rest go on to tier 3 (list `defer`, whose
        // entries the LDS tier has consumed)
        std::vector<T2LArgs> xl;
        std::vector<uint32_t> xlb;
        {
            std::vector<uint64_t> listed(N, 0);
            for (size_t i = 0; i < N; i++)
                if (J[i]->g.model == HBM_IC)
                    listed[i] = root.ctrl_host[i * CW_COUNT + (chain ? CW_NDEFER3 : CW_NDEFER2)];
            spill_plan(root, root.spill2, T2X_CAP * sizeof(uint32_t),
                       spill_caps(listed, std::min<int64_t>(root.spill_slots, 256)), sp2);
        }
        for (size_t i = 0; i < N; i++) {
            Ctx &c = *J[i];
            if (c.g.model != HBM_IC) continue;
            // CW_NDEFER still counts the LDS tier's input: from here on it counts tier 3's
            root.ctrl_host[i * CW_COUNT + CW_NDEFER] = 0;
            const uint64_t nd2 = root.ctrl_host[i * CW_COUNT + (chain ? CW_NDEFER3 : CW_NDEFER2)];
            if (!nd2) continue;
            root.ctrl_host[i * CW_COUNT + CW_NEXT2] = 0;
            xl.push_back(T2LArgs{A[i], chain ? A[i].defer3 : A[i].defer2, (uint32_t)nd2, A[i].defer, CW_NDEFER, nullptr});
            spill_in(sp1, i, xl.back(), T2L_CAP_REGULAR);  // as the 2048-member tier wrote it
            xl.back().xs_ids = sp2.rec<uint32_t>(i);
            xl.back().xs_hdr = sp2.hdr(i);
            xl.back().xs_cap = sp2.cap[i];
            xlb.push_back((uint32_t)std::min<uint64_t>(nd2, (uint64_t)root.num_cus));
        }
        if (!xl.empty()) {
            // member records: T2X_CAP per workgroup of the launch (a grouped launch numbers its
            // workgroups across all jobs).  One such workgroup fits a CU, so more than two per CU
            // only queue: the jobs share 2 per CU (at least one each; each job's workgroups take
            // its sets from its own counter until none is left)
            uint64_t blocks = 0;
            for (uint32_t b : xlb) blocks += b;
            const uint64_t cap = std::max<uint64_t>((uint64_t)root.num_cus * 2, xlb.size());
            if (blocks > cap) {
                const uint64_t total = blocks;
                blocks = 0;
                for (uint32_t &b : xlb) {
                    b = (uint32_t)std::max<uint64_t>(1, (uint64_t)b * cap / total);
                    blocks += b;
                }
            }
            buf_grow(root, root.xmeta, (size_t)blocks * T2X_CAP * sizeof(uint4), false);
            for (T2LArgs &t : xl) t.xmeta = root.xmeta.as<uint4>();
            ctrl_push(root);
            int sx = prof_begin(root, "ic_sample_block_xl");
            glaunch(root, xl, xlb, 0,
                    [&](const T2LArgs &t, unsigned g) {
                        k_big_lds<1024, T2X_CAP, T2X_HASH_BITS><<<g, 1024, 0, st>>>(t);
                    },
                    [&](const T2LArgs *d, const uint32_t *b, uint32_t cnt, uint32_t g, int x) {
                        k_big_lds_g<1024, T2X_CAP, T2X_HASH_BITS><<<g, 1024, 0, st>>>(GroupArgs<T2LArgs>{d, b, cnt, x});
                    });
            HBM_HIP(hipGetLastError());
            prof_end(root, sx);
            ctrl_pull(root);
            if (sx >= 0) prof_sampler(root, sx, true, J);
        }
        // ---- tier 3: IC sets that outgrew the extra-large pass and LT walks longer than the LDS
        // path, a workgroup each with its visited bitmap and queue in device memory
        for (int model : {HBM_IC, HBM_LT}) {
            std::vector<T2Args> t3;
            std::vector<uint32_t> t3b;
            for (size_t i = 0; i < N; i++) {
                Ctx &c = *J[i];
                if (c.g.model != model) continue;
                const uint64_t nd3 = root.ctrl_host[i * CW_COUNT + CW_NDEFER];
                if (!nd3) continue;
                ensure_t2(c);
                root.ctrl_host[i * CW_COUNT + CW_NEXT2] = 0;
                T2Args t{};
                t.a = A[i];
                t.bitmap = c.sc.t2_bitmap.as<uint32_t>();
                t.queue = c.sc.t2_queue.as<uint32_t>();
                t.words = ((uint64_t)c.g.n + 31) / 32;
                t.list = model == HBM_IC ? A[i].defer : A[i].defer2;
                t.nlist = (uint32_t)nd3;
                t.model = model;
                t.qcap = t2_qcap(c);
                t.can_defer = 1;
                if (model == HBM_IC && !sp2.cap.empty()) {  // as the extra-large pass wrote them
                    t.rs_ids = sp2.rec<uint32_t>(i);
                    t.rs_hdr = sp2.hdr(i);
                    t.rs_cap = sp2.cap[i];
                }
                t3.push_back(t);
                t3b.push_back((uint32_t)std::min<uint64_t>(nd3, (uint64_t)c.sc.t2_slots));
            }
            if (t3.empty()) continue;
            ctrl_push(root);
            int s4 = prof_begin(root, model == HBM_IC ? "ic_sample_bitmap" : "lt_sample_block");
            glaunch(root, t3, t3b, 0, [&](const T2Args &t, unsigned g) { k_big<<<g, T2_THREADS, 0, st>>>(t); },
                    [&](const T2Args *d, const uint32_t *b, uint32_t cnt, uint32_t g, int x) {
                        k_big_g<<<g, T2_THREADS, 0, st>>>(GroupArgs<T2Args>{d, b, cnt, x});
                    });
            HBM_HIP(hipGetLastError());
            prof_end(root, s4);
            ctrl_pull(root);
            if (s4 >= 0) prof_sampler(root, s4, model == HBM_IC, J);
        }
    }
    // ---- huge pass: sets that outgrew a big-set slot's queue, redone with a full queue
    std::vector<T2Args> th;
    std::vector<uint32_t> thb;
    for (size_t i = 0; i < N; i++) {
        Ctx &c = *J[i];
        const uint64_t nh = root.ctrl_host[i * CW_COUNT + CW_NHUGE];
        if (!nh) continue;
        ensure_t2_huge(c);
        root.ctrl_host[i * CW_COUNT + CW_NEXT2] = 0;
        T2Args t{};
        t.a = A[i];
        t.bitmap = c.sc.t2h_bitmap.as<uint32_t>();
        t.queue = c.sc.t2h_queue.as<uint32_t>();
        t.words = ((uint64_t)c.g.n + 31) / 32;
        t.list = A[i].defer3;
        t.nlist = (uint32_t)nh;
        t.model = c.g.model;
        t.qcap = (uint32_t)c.g.n;
        t.can_defer = 0;
        th.push_back(t);
        thb.push_back((uint32_t)std::min<uint64_t>(nh, (uint64_t)c.sc.t2h_slots));
    }
    if (!th.empty()) {
        ctrl_push(root);
        int s5 = prof_begin(root, "sample_huge");
        glaunch(root, th, thb, 0, [&](const T2Args &t, unsigned g) { k_big<<<g, T2_THREADS, 0, st>>>(t); },
                [&](const T2Args *d, const uint32_t *b, uint32_t cnt, uint32_t g, int x) {
                    k_big_g<<<g, T2_THREADS, 0, st>>>(GroupArgs<T2Args>{d, b, cnt, x});
                });
        HBM_HIP(hipGetLastError());
        prof_end(root, s5);
        ctrl_pull(root);
        if (s5 >= 0) prof_sampler(root, s5, J[0]->g.model == HBM_IC, J);
    }
    for (size_t i = 0; i < N; i++)
        done[i] = (int64_t)std::min<unsigned long long>(root.ctrl_host[i * CW_COUNT + CW_FIRST_OVF],
                                                        (unsigned long long)nbv[i]);
}

int64_t sample_block(Ctx &c, int64_t j0, int64_t j1, uint64_t seed) {
    std::vector<Ctx *> J{&c};
    std::vector<int64_t> done;
    sample_blocks(c, J, {j0}, {j1 - j0}, {seed}, done);
    return done[0];
}

}  // namespace hbm
