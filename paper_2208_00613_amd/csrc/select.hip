// select.hip -- greedy max coverage on the (encoded) RR store.
//
// k iterations (the Seed Selection paragraph; Alg. 2 / Alg. 3 read as picking exactly k
// seeds).  Each iteration t runs, on the stream:
//   argmax : every block writes the best key (count + 1) << 32 | ~id of its slice (the
//            unselected vertex with the highest count, lowest id on ties); the next kernels
//            reduce the partials themselves, so u* is exact (not the paper's parallel-merge
//            heuristic, which can miss the true maximum).  With sparse counts the slots are
//            keyed by index (they ascend with the ids) and a block maps its best to a vertex;
//   find   : the sets that hold u*, when u* has no bitmap row: a pass over the plain ids
//            (find_raw), a partial decode of every uncovered set's Huffman string (find_huff,
//            Alg. 2's DecodeFind: after the escaped ids and the front element the codes
//            follow canonical (length, id) order, ascending left-justified code value, so
//            the scan stops at u* or at the first code above u*'s), or u*'s array row read
//            as a list of sets;
//   apply  : records u*; when u* has a row or the store is plain, marks the newly covered
//            sets (Eq. 3: row AND NOT covered) and decrements their stored members (find_huff
//            already did that for a cold u* of a Huffman store).  A Huffman store without
//            array rows needs no apply launch: find_huff records u* and covers a bitmap
//            row's sets itself;
//   hot / array rows : counts of vertices with bitmap rows drop by popcount(row AND newly),
//            word by word (Alg. 3's SUBTRACT and POPCOUNT, applied to the change only), and
//            those with array rows by their entries in newly covered sets.
// Counts are exact 32-bit integers (the paper's float frequencies are not exact beyond
// 2^24).  The store itself is never modified.
#include <cstring>
#include <mutex>

#include "hbm_device.h"
#include "hbm_internal.h"

namespace hbm {

constexpr int PB_SLOTS = 4096;

struct SelArgs {
    int64_t T;       // sets
    int64_t words;   // ceil(T / 64)
    int32_t n;
    uint32_t *counts;
    uint32_t *selmask;
    unsigned long long *covered;
    unsigned long long *newly;
    unsigned long long *keys;
    int32_t nhot;
    const int32_t *hot;
    const int32_t *hot_rank;
    const unsigned long long *bitmap;
    const int64_t *raw_off;
    const int32_t *raw_mem;
    const int32_t *raw_host;  // plain ids from raw_split on (a spilled store)
    int64_t raw_split;
    int implicit;             // implicit roots: set j's root (if not in a bitmap row) is not stored
    uint64_t seed;            // the store's seed (root_j = rr_root(seed, j, n))
    int huff;
    const int64_t *bitoff;
    const uint32_t *payload;
    const uint64_t *lim;
    const int64_t *base;
    const int32_t *symtab;
    const uint8_t *lens;
    const uint32_t *codes;
    const uint32_t *lut;
    int32_t minlen;
    int32_t wbits;
    int32_t ustar_enc;
    int64_t nraw;                 // plain ids in the store
    unsigned long long *partial;  // per-block argmax partials
    int32_t nparts;               // argmax blocks
    const uint32_t *hist;         // store frequencies (initial counts)
    int32_t k;                    // seeds to pick
    int32_t hx;                   // hot-count blocks per word segment
    int64_t seg;                  // words per hot-count segment
    const uint8_t *ckb;           // code-boundary slots of the payload
    // sparse counts (large graphs): only vertices with a nonzero store frequency get a slot, in
    // ascending id order, and `counts` holds the slots' counts
    const uint32_t *cand;         // slot -> vertex (null: dense, counts[v])
    const int32_t *cpos;          // vertex -> slot (read for vertices that have one only)
    uint32_t *csel;               // selection bits over slots
    const int64_t *ncand;         // number of slots (device)
    unsigned long long *pbytes;   // profiling: algorithmic bytes find_huff reads, PB_SLOTS
                                  // partial sums (one per workgroup, modulo), else null
    // array rows (hot vertices of low density): per 2^16-set chunk, each row's sorted 16-bit set
    // offsets; ar_off is chunk-major with nar + 1 entries per chunk
    int32_t nar;
    const int32_t *ar_rank;
    const int32_t *ar_hot;
    const int64_t *ar_off;
    const uint16_t *ar_low;
    int64_t nchunks;
    int64_t nentries;             // array entries over all chunks
    int fused;                    // Huffman store without array rows: k_find_huff also records u*
                                  // and, for a u* with a bitmap row, does k_apply's work
};

__device__ __forceinline__ bool in_arr(const SelArgs &A, uint32_t v) { return A.nar && A.ar_rank[v] >= 0; }

// The root a store with implicit roots left out of set j (a root with a bitmap row is in its
// row), or ~0u.
__device__ __forceinline__ uint32_t lost_root(const SelArgs &A, int64_t j) {
    if (!A.implicit) return 0xFFFFFFFFu;
    const uint32_t r = rr_root(A.seed, (uint64_t)j, (uint32_t)A.n);
    return ((A.hot_rank && A.hot_rank[r] >= 0) || in_arr(A, r)) ? 0xFFFFFFFFu : r;
}

// u* with array row a: its uncovered sets, read off the row's list in every chunk (one wave per
// chunk at a time), are marked in `newly`; k_apply covers them and decrements their members.
__device__ void arr_mark(const SelArgs &A, int32_t a, int64_t bid, uint32_t nblk) {
    const int64_t nwaves = (int64_t)nblk * (blockDim.x / WAVE);
    const unsigned lane = lane_id();
    for (int64_t ch = bid * (int64_t)(blockDim.x / WAVE) + threadIdx.x / WAVE; ch < A.nchunks; ch += nwaves) {
        const int64_t *o = A.ar_off + ch * (int64_t)(A.nar + 1);
        const int64_t e = o[a + 1];
        for (int64_t i = o[a] + lane; i < e; i += WAVE) {
            const int64_t j = (ch << 16) | (int64_t)A.ar_low[i];
            const unsigned long long bit = 1ull << (j & 63);
            if (!(A.covered[j >> 6] & bit)) atomicOr(&A.newly[j >> 6], bit);
        }
    }
}

// Index into `counts` of vertex v (every decremented vertex is a member of some set, so it
// has a slot when the counts are sparse).  Decoded Huffman symbols are already such indices:
// with sparse counts the decode tables name slots instead of vertices.
__device__ __forceinline__ uint32_t ckey(const SelArgs &A, uint32_t v) { return A.cpos ? (uint32_t)A.cpos[v] : v; }

// Exact argmax over counts, stage 1: each block writes the best key of its slice to
// partial[block]; the consumer kernels of the same iteration reduce the partials
// themselves (no atomics or fences needed: kernel boundaries order the stream).
// Also clears the `newly` words for this iteration's find step.
// Selection state at the start: counts = store frequencies, nothing selected or covered.
HBM_KERNEL(k_sel_init, SelArgs, 256) {
    const int64_t tid = bid * (int64_t)blockDim.x + threadIdx.x;
    const int64_t nthr = (int64_t)nblk * blockDim.x;
    const int64_t sw = ((int64_t)A.n + 31) / 32;
    if (A.cpos) {  // sparse: the slot counts were written with the slots
        const int64_t cw = (*A.ncand + 31) / 32;
        for (int64_t w = tid; w < cw; w += nthr) A.csel[w] = 0u;
    } else {
        for (int64_t v = tid; v < A.n; v += nthr) A.counts[v] = A.hist ? A.hist[v] : 0u;
    }
    for (int64_t v = tid; v < sw; v += nthr) A.selmask[v] = 0u;
    for (int64_t w = tid; w < A.words; w += nthr) A.covered[w] = 0ull;
    for (int64_t i = tid; i < A.k; i += nthr) A.keys[i] = 0ull;
}

constexpr int AM_UNROLL = 4;

// Sparse counts: the keys of the slots of count > 0, (count + 1) << 32 | ~slot (slots are in
// ascending vertex order, so the lowest slot of a count is its lowest vertex; the block maps
// its best slot to its vertex once), and the key of the lowest unselected id, (0 + 1) << 32 |
// ~id, for every vertex of count 0: such a vertex can only win as the lowest unselected id,
// whether it has a slot or not.
__device__ unsigned long long argmax_sparse(const SelArgs &A, int64_t tid, int64_t nthr) {
    unsigned long long best = 0;
    const int64_t m = *A.ncand;
    const int64_t m4 = m >> 2;
    const uint4 *c4 = reinterpret_cast<const uint4 *>(A.counts);
    for (int64_t q0 = tid; q0 < m4; q0 += nthr * AM_UNROLL) {
        uint4 c[AM_UNROLL];
        uint32_t smw[AM_UNROLL];
#pragma unroll
        for (int u = 0; u < AM_UNROLL; u++) {
            const int64_t q = q0 + (int64_t)u * nthr;
            if (q < m4) {
                c[u] = c4[q];
                smw[u] = A.csel[q >> 3];
            }
        }
#pragma unroll
        for (int u = 0; u < AM_UNROLL; u++) {
            const int64_t q = q0 + (int64_t)u * nthr;
            if (q >= m4) break;
            const uint32_t sm = smw[u] >> ((q & 7) * 4);
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const uint32_t cr = r == 0 ? c[u].x : r == 1 ? c[u].y : r == 2 ? c[u].z : c[u].w;
                const uint32_t sr = (uint32_t)(q * 4 + r);
                const unsigned long long key = (((sm >> r) & 1u) || !cr)
                                                   ? 0ull
                                                   : (((unsigned long long)cr + 1ull) << 32) | (unsigned long long)(~sr);
                best = key > best ? key : best;
            }
        }
    }
    for (int64_t i = m4 * 4 + tid; i < m; i += nthr) {
        const bool sel = (A.csel[i >> 5] >> (i & 31)) & 1u;
        const uint32_t cr = A.counts[i];
        const unsigned long long key =
            (sel || !cr) ? 0ull : (((unsigned long long)cr + 1ull) << 32) | (unsigned long long)(~(uint32_t)i);
        best = key > best ? key : best;
    }
    // fewer than k vertices are selected before the last pick, so the lowest unselected id is
    // below k: only the selection words of ids [0, k] need a look
    const int64_t swn = ((int64_t)A.n + 31) / 32, swk = (int64_t)A.k / 32 + 1;
    const int64_t sw = swn < swk ? swn : swk;
    for (int64_t w = tid; w < sw; w += nthr) {
        uint32_t free_bits = ~A.selmask[w];
        const int64_t left = (int64_t)A.n - w * 32;
        if (left < 32) free_bits &= (1u << left) - 1u;  // no vertex past n
        if (free_bits) {
            const uint32_t v = (uint32_t)(w * 32) + (uint32_t)(__ffs(free_bits) - 1);
            const unsigned long long key = (1ull << 32) | (unsigned long long)(~v);
            best = key > best ? key : best;
        }
    }
    return best;
}

HBM_KERNEL(k_argmax, SelArgs, 256) {
    const int t = x;
    (void)t;
    const int64_t tid = bid * (int64_t)blockDim.x + threadIdx.x;
    const int64_t nthr = (int64_t)nblk * blockDim.x;
    for (int64_t w = tid; w < A.words; w += nthr) A.newly[w] = 0ull;
    unsigned long long best = A.cpos ? argmax_sparse(A, tid, nthr) : 0ull;
    const int64_t n4 = A.cpos ? 0 : A.n >> 2;
    const uint4 *c4 = reinterpret_cast<const uint4 *>(A.counts);
    // AM_UNROLL independent 16-byte loads in flight per thread: the pass is bound by HBM, and
    // one outstanding load per wave would leave it latency-bound
    for (int64_t q0 = tid; q0 < n4; q0 += nthr * AM_UNROLL) {
        uint4 c[AM_UNROLL];
        uint32_t smw[AM_UNROLL];
#pragma unroll
        for (int u = 0; u < AM_UNROLL; u++) {
            const int64_t q = q0 + (int64_t)u * nthr;
            if (q < n4) {
                c[u] = c4[q];
                smw[u] = A.selmask[q >> 3];
            }
        }
#pragma unroll
        for (int u = 0; u < AM_UNROLL; u++) {
            const int64_t q = q0 + (int64_t)u * nthr;
            if (q >= n4) break;
            const uint32_t sm = smw[u] >> ((q & 7) * 4);
            const uint32_t v0 = (uint32_t)(q * 4);
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const uint32_t cr = r == 0 ? c[u].x : r == 1 ? c[u].y : r == 2 ? c[u].z : c[u].w;
                const unsigned long long key = ((sm >> r) & 1u) ? 0ull
                                                                : (((unsigned long long)cr + 1ull) << 32) |
                                                                      (unsigned long long)(~(v0 + r));
                best = key > best ? key : best;
            }
        }
    }
    for (int64_t v = A.cpos ? A.n : n4 * 4 + tid; v < A.n; v += nthr) {
        const bool sel = (A.selmask[v >> 5] >> (v & 31)) & 1u;
        const unsigned long long key =
            sel ? 0ull : (((unsigned long long)A.counts[v] + 1ull) << 32) | (unsigned long long)(~(uint32_t)v);
        best = key > best ? key : best;
    }
    best = wave_max_u64(best);
    __shared__ unsigned long long part[256 / WAVE];
    if (lane_id() == 0) part[threadIdx.x / WAVE] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long b = part[0];
        for (int i = 1; i < (int)(blockDim.x / WAVE); i++) b = part[i] > b ? part[i] : b;
        // a slot's key (count field >= 2) to its vertex's: same order, as slots ascend with ids
        if (A.cpos && (b >> 32) >= 2ull) b = (b & 0xFFFFFFFF00000000ull) | (unsigned long long)(~A.cand[~(uint32_t)b]);
        A.partial[bid] = b;
    }
}

// Stage 2, run at the start of every consumer block: the key of u* (block-uniform).  Each
// thread issues its PR_N partial reads before it uses any (a loop that uses each read before
// the next would pay one device-memory latency per step).
constexpr int PR_N = 8;
__device__ unsigned long long argmax_key(const SelArgs &A) {
    __shared__ unsigned long long red[1024 / WAVE];
    unsigned long long b = 0;
    for (int i0 = threadIdx.x; i0 < A.nparts; i0 += blockDim.x * PR_N) {
        unsigned long long x[PR_N];
#pragma unroll
        for (int r = 0; r < PR_N; r++) {
            const int i = i0 + r * (int)blockDim.x;
            x[r] = i < A.nparts ? A.partial[i] : 0ull;
        }
#pragma unroll
        for (int r = 0; r < PR_N; r++) b = x[r] > b ? x[r] : b;
    }
    b = wave_max_u64(b);
    if (lane_id() == 0) red[threadIdx.x / WAVE] = b;
    __syncthreads();
    unsigned long long m = red[0];
    for (int i = 1; i < (int)(blockDim.x / WAVE); i++) m = red[i] > m ? red[i] : m;
    __syncthreads();
    return m;
}

struct Tabs {
    uint64_t lim[34];
    int64_t base[34];
    uint32_t lut[1 << LUT_BITS];
};

// The decode tables into LDS, PR_N reads in flight per thread (as argmax_key).
__device__ void load_tabs(const SelArgs &A, Tabs &tb) {
    for (int i = threadIdx.x; i < 34; i += blockDim.x) {
        tb.lim[i] = A.lim[i];
        tb.base[i] = A.base[i];
    }
    for (int i0 = threadIdx.x; i0 < (1 << LUT_BITS); i0 += blockDim.x * PR_N) {
        uint32_t x[PR_N];
#pragma unroll
        for (int r = 0; r < PR_N; r++) {
            const int i = i0 + r * (int)blockDim.x;
            x[r] = i < (1 << LUT_BITS) ? A.lut[i] : 0u;
        }
#pragma unroll
        for (int r = 0; r < PR_N; r++) {
            const int i = i0 + r * (int)blockDim.x;
            if (i < (1 << LUT_BITS)) tb.lut[i] = x[r];
        }
    }
}

// one canonical code: the LDS table for short codes, the limit search for long ones.
// `buf` is the stream (device memory or an LDS copy); `pos` a bit position in it.
__device__ __forceinline__ uint32_t dec_code(const SelArgs &A, const Tabs &tb, const uint32_t *buf, uint64_t &pos) {
    const uint32_t w = peek32(buf, pos);
    const uint32_t ent = tb.lut[w >> (32 - LUT_BITS)];
    if (ent & 31u) {
        pos += ent & 31u;
        return ent >> 5;
    }
    int L = (int)(ent >> 5);  // shortest length a code with this prefix can have
    while ((uint64_t)w >= tb.lim[L]) L++;
    pos += (uint64_t)L;
    return (uint32_t)A.symtab[tb.base[L] + (int64_t)(w >> (32 - L))];
}

// An MSB-first bit reader with a 64-bit window: the next 32 bits are always at the top, and
// one word is loaded per 32 bits consumed (decoding with peek32 loads two words per code, on
// the code's dependency chain).  Reads reach at most the word that holds bit pos + 31, as
// peek32 does.
struct BitReader {
    const uint32_t *buf;
    uint64_t win;    // bits [pos, pos + avail), left-justified
    uint32_t avail;  // >= 32
    uint64_t nxt;    // the next word to load
    __device__ __forceinline__ void init(const uint32_t *b, uint64_t pos) {
        buf = b;
        const uint64_t w = pos >> 5;
        const uint32_t sh = (uint32_t)(pos & 31);
        win = (((uint64_t)b[w] << 32) | (uint64_t)b[w + 1]) << sh;
        avail = 64 - sh;
        nxt = w + 2;
    }
    __device__ __forceinline__ uint32_t top() const { return (uint32_t)(win >> 32); }
    __device__ __forceinline__ void skip(uint32_t n) {  // n <= 32
        win <<= n;
        avail -= n;
        if (avail < 32) {
            win |= (uint64_t)buf[nxt++] << (32 - avail);
            avail += 32;
        }
    }
};

// one canonical code from a reader (as dec_code)
__device__ __forceinline__ uint32_t dec_code_r(const SelArgs &A, const Tabs &tb, BitReader &R, uint64_t &pos) {
    const uint32_t w = R.top();
    const uint32_t ent = tb.lut[w >> (32 - LUT_BITS)];
    uint32_t L, sym;
    if (ent & 31u) {
        L = ent & 31u;
        sym = ent >> 5;
    } else {
        L = ent >> 5;  // shortest length a code with this prefix can have
        while ((uint64_t)w >= tb.lim[L]) L++;
        sym = (uint32_t)A.symtab[tb.base[L] + (int64_t)(w >> (32 - L))];
    }
    R.skip(L);
    pos += L;
    return sym;
}

__device__ __forceinline__ uint32_t read_gamma(const uint32_t *payload, uint64_t &pos) {
    const uint32_t L = __clz(peek32(payload, pos));
    pos += L;
    const uint32_t g = peek32(payload, pos) >> (31 - L);
    pos += L + 1;
    return g;
}

// length of the canonical code at the head of window w (LDS only)
__device__ __forceinline__ uint32_t code_len(const SelArgs &A, const Tabs &tb, uint32_t w) {
    const uint32_t ent = tb.lut[w >> (32 - LUT_BITS)];
    if (ent & 31u) return ent & 31u;
    int L = (int)(ent >> 5);  // shortest length a code with this prefix can have
    while ((uint64_t)w >= tb.lim[L]) L++;
    return (uint32_t)L;
}

// Is u in the set whose bits are [pos, end) of buf?  Codeless ids come first, ascending,
// and stop the scan at the first larger id.  Coded members are compared by their canonical
// code (ustar_len, ustar_code), so no code is mapped back to an id; after the front code
// (u*_enc, whose code is (fe_len, fe_code)) codes come in ascending left-justified value,
// so the scan stops at the first code above u's.
__device__ bool huff_contains(const SelArgs &A, const Tabs &tb, const uint32_t *buf, uint64_t pos, uint64_t end,
                              uint32_t u, uint32_t ustar_len, uint32_t ustar_code, uint32_t fe_len,
                              uint32_t fe_code) {
    const uint32_t nesc = read_gamma(buf, pos) - 1;
    if (!ustar_len) {
        for (uint32_t q = 0; q < nesc; q++) {
            const uint32_t v = peek32(buf, pos) >> (32 - A.wbits);
            pos += A.wbits;
            if (v == u) return true;
            if (v > u) return false;
        }
        return false;
    }
    pos += (uint64_t)nesc * A.wbits;
    if (pos >= end) return false;
    const uint32_t U = ustar_code << (32 - ustar_len);
    bool first = true;
    BitReader R;
    R.init(buf, pos);
    while (pos < end) {
        const uint32_t w = R.top();
        const uint32_t L = code_len(A, tb, w);
        const uint32_t c = w >> (32 - L);
        if (L == ustar_len && c == ustar_code) return true;
        if (!(first && L == fe_len && c == fe_code) && (c << (32 - L)) > U) return false;
        first = false;
        pos += L;
        R.skip(L);
    }
    return false;
}

// Per-block combining cache for count decrements: the sets covered by one pick share
// their hubs, and thousands of atomics on one address serialise.  Decrements of ids
// that own a slot accumulate in LDS and are flushed once per block; an id whose slot is
// taken by another id goes straight to device memory.
constexpr int CC_SLOTS = 1024;
struct DecCache {
    uint32_t id[CC_SLOTS];
    uint32_t cnt[CC_SLOTS];
};

__device__ __forceinline__ void cache_init(DecCache &C) {
    for (int i = threadIdx.x; i < CC_SLOTS; i += blockDim.x) {
        C.id[i] = 0xFFFFFFFFu;
        C.cnt[i] = 0u;
    }
}

// v: an index into A.counts (see ckey)
__device__ __forceinline__ void cache_dec(DecCache &C, const SelArgs &A, uint32_t v) {
    const uint32_t h = (v * 0x9E3779B1u) >> (32 - 10);
    uint32_t x = C.id[h];
    if (x == 0xFFFFFFFFu) {
        const uint32_t old = atomicCAS(&C.id[h], 0xFFFFFFFFu, v);
        x = old == 0xFFFFFFFFu ? v : old;
    }
    if (x == v) atomicAdd(&C.cnt[h], 1u);
    else atomicSub(&A.counts[v], 1u);
}

// after a __syncthreads: push the cached decrements to device memory
__device__ __forceinline__ void cache_flush(DecCache &C, const SelArgs &A) {
    for (int i = threadIdx.x; i < CC_SLOTS; i += blockDim.x)
        if (C.cnt[i]) atomicSub(&A.counts[C.id[i]], C.cnt[i]);
}

__device__ void huff_decrement(const SelArgs &A, const Tabs &tb, DecCache &C, const uint32_t *buf, uint64_t pos,
                               uint64_t end) {
    const uint32_t nesc = read_gamma(buf, pos) - 1;
    for (uint32_t q = 0; q < nesc; q++) {
        const uint32_t v = peek32(buf, pos) >> (32 - A.wbits);
        pos += A.wbits;
        cache_dec(C, A, ckey(A, v));
    }
    if (pos >= end) return;
    BitReader R;
    R.init(buf, pos);
    while (pos < end) cache_dec(C, A, dec_code_r(A, tb, R, pos));
}

__device__ __forceinline__ uint32_t ustar_of(const SelArgs &A, int t, unsigned long long &key) {
    (void)t;
    key = argmax_key(A);
    return ~(uint32_t)key;
}

// Plain ids: one coalesced pass over every stored id; a match marks its set (if uncovered) in `newly`.
HBM_KERNEL(k_find_raw, SelArgs, 256) {
    unsigned long long key;
    const uint32_t u = ustar_of(A, x, key);
    if (key == 0 || (A.hot_rank && A.hot_rank[u] >= 0)) return;
    if (in_arr(A, u)) {
        arr_mark(A, A.ar_rank[u], bid, nblk);
        return;
    }
    const int64_t tid = bid * (int64_t)blockDim.x + threadIdx.x;
    const int64_t nthr = (int64_t)nblk * blockDim.x;
    const int64_t n4 = A.nraw >> 2;
    for (int64_t q = tid; q <= n4; q += nthr) {
        uint32_t x[4];
        int cnt = 4;
        if (q < n4) {
            const uint4 m = raw_id4(A.raw_mem, A.raw_host, A.raw_split, q);
            x[0] = m.x; x[1] = m.y; x[2] = m.z; x[3] = m.w;
        } else {
            cnt = (int)(A.nraw - n4 * 4);
            for (int r = 0; r < cnt; r++) x[r] = (uint32_t)raw_id(A.raw_mem, A.raw_host, A.raw_split, n4 * 4 + r);
        }
        for (int r = 0; r < cnt; r++) {
            if (x[r] != u) continue;
            const int64_t i = q * 4 + r;
            // set containing position i: last j with raw_off[j] <= i
            int64_t lo = 0, hi = A.T;
            while (lo < hi) {
                const int64_t mid = (lo + hi + 1) >> 1;
                if (A.raw_off[mid] <= i) lo = mid;
                else hi = mid - 1;
            }
            const unsigned long long bit = 1ull << (lo & 63);
            if (!(A.covered[lo >> 6] & bit)) atomicOr(&A.newly[lo >> 6], bit);
        }
    }
    if (A.implicit) {  // sets whose root, not stored, is u* (u* is cold here)
        for (int64_t j = tid; j < A.T; j += nthr) {
            if (rr_root(A.seed, (uint64_t)j, (uint32_t)A.n) != u) continue;
            const unsigned long long bit = 1ull << (j & 63);
            if (!(A.covered[j >> 6] & bit)) atomicOr(&A.newly[j >> 6], bit);
        }
    }
}

// Copy nw words from device memory to a wave's LDS buffer with ST_UNROLL loads in flight per
// lane (one outstanding load per lane would leave the copy latency-bound).
constexpr int ST_UNROLL = 8;
__device__ __forceinline__ void stage_words(uint32_t *dst, const uint32_t *src, uint64_t nw) {
    const unsigned lane = lane_id();
    for (uint64_t q0 = lane; q0 < nw; q0 += (uint64_t)WAVE * ST_UNROLL) {
        uint32_t v[ST_UNROLL];
#pragma unroll
        for (int u = 0; u < ST_UNROLL; u++) {
            const uint64_t q = q0 + (uint64_t)u * WAVE;
            v[u] = q < nw ? src[q] : 0u;
        }
#pragma unroll
        for (int u = 0; u < ST_UNROLL; u++) {
            const uint64_t q = q0 + (uint64_t)u * WAVE;
            if (q < nw) dst[q] = v[u];
        }
    }
}

// The members of one string [pos, ce) of set js, decremented by the whole wave (js, pos, ce
// wave-uniform): the escaped ids have fixed width, so each lane takes every 64th; the coded
// part is cut at the code-boundary slots (one per CK_SLOT bits) and NI lanes decode NI slot
// intervals at a time from an LDS copy of their bits (`stage`: NI * CK_SLOT / 32 + 4 words).
template <int NI>
__device__ void wave_dec_string(const SelArgs &A, const Tabs &tb, DecCache &C, uint32_t *stage, int64_t js,
                                uint64_t pos, const uint64_t ce) {
    const unsigned lane = lane_id();
    const uint32_t W = (uint32_t)A.wbits;
    if (A.implicit && lane == 0) {  // the set's root, left out of its string
        const uint32_t r = lost_root(A, js);
        if (r != 0xFFFFFFFFu) cache_dec(C, A, ckey(A, r));
    }
    // gamma(nesc + 1) from one three-word window (the code has 2L + 1 <= 63 bits)
    uint32_t nesc;
    {
        const uint64_t w = pos >> 5;
        const uint32_t sh = (uint32_t)(pos & 31);
        const uint64_t hi = ((uint64_t)A.payload[w] << 32) | A.payload[w + 1];
        const uint64_t win = sh ? (hi << sh) | (A.payload[w + 2] >> (32 - sh)) : hi;
        const uint32_t L = __clzll((long long)win);
        nesc = (uint32_t)(win >> (63 - 2 * L)) - 1;
        pos += 2 * (uint64_t)L + 1;
    }
    for (uint32_t q = lane; q < nesc; q += WAVE)
        cache_dec(C, A, ckey(A, peek32(A.payload, pos + (uint64_t)q * W) >> (32 - W)));
    const uint64_t cs = pos + (uint64_t)nesc * W;
    // slot intervals: [cs, b(m0)), [b(m0), b(m0 + 1)), ..., [b(m1), ce), b(m) the boundary of slot m
    const uint64_t m0 = cs / CK_SLOT + 1;
    const uint64_t m1 = ce > 0 ? (ce - 1) / CK_SLOT : 0;
    const uint64_t nseg = m1 >= m0 ? m1 - m0 + 2 : 1;
    auto seg_start = [&](uint64_t sg) -> uint64_t {
        if (sg == 0) return cs;
        if (sg >= nseg) return ce;
        const uint64_t b = (m0 + sg - 1) * CK_SLOT + A.ckb[m0 + sg - 1];
        return b < ce ? b : ce;
    };
    for (uint64_t g0 = 0; g0 < nseg; g0 += NI) {
        const uint64_t sg = g0 + (lane < (unsigned)NI ? lane : 0u);
        const uint64_t p = seg_start(sg), e = seg_start(sg + 1);
        // bits of the group's intervals: [start of g0, end of the group's last interval)
        const uint64_t lo = __shfl((unsigned long long)p, 0, WAVE);
        const uint64_t gl = g0 + NI < nseg ? g0 + NI : nseg;
        const uint64_t hi = __shfl((unsigned long long)e, (int)(gl - 1 - g0), WAVE);
        const uint64_t wlo = lo >> 5;
        const uint64_t nw = ((hi + 31) >> 5) - wlo + 1;  // +1: peek32 reads a word ahead
        stage_words(stage, A.payload + wlo, nw);
        wave_sync();
        if (lane < (unsigned)NI && sg < nseg && p < e) {
            uint64_t pp = p - wlo * 32;
            const uint64_t ee = e - wlo * 32;
            BitReader R;
            R.init(stage, pp);
            while (pp < ee) cache_dec(C, A, dec_code_r(A, tb, R, pp));
        }
        wave_sync();
    }
}

// u* (key `key`) as the pick of iteration t: its selection bit (and its slot's) and its key
__device__ __forceinline__ void record_ustar(const SelArgs &A, int t, uint32_t u, unsigned long long key) {
    atomicOr(&A.selmask[u >> 5], 1u << (u & 31));
    if (A.cpos && A.hist[u] > 0) {  // u has a slot
        const int32_t p = A.cpos[u];
        atomicOr(&A.csel[p >> 5], 1u << (p & 31));
    }
    A.keys[t] = key;
}

// k_apply's pass over the words (u* with bitmap row r, or -1): the newly covered sets are
// marked and their members decremented, Huffman strings NI slot intervals at a time from the
// wave's stage (NI * CK_SLOT / 32 + 4 words)
template <int NI>
__device__ void apply_words(const SelArgs &A, const Tabs &tb, DecCache &C, uint32_t *stage, int32_t r, int64_t bid,
                            uint32_t nblk) {
    const unsigned lane = lane_id();
    const int64_t nwaves = (int64_t)nblk * (blockDim.x / WAVE);
    for (int64_t w = bid * (int64_t)(blockDim.x / WAVE) + threadIdx.x / WAVE; w < A.words; w += nwaves) {
        const unsigned long long cov = A.covered[w];
        const unsigned long long nw = (r >= 0 ? A.bitmap[w * (int64_t)A.nhot + r] : A.newly[w]) & ~cov;
        if (lane == 0) {
            A.newly[w] = nw;
            if (nw) A.covered[w] = cov | nw;
        }
        if (!nw) continue;
        if (A.huff) {
            // the word's newly covered strings, one at a time by the whole wave
            const int64_t j0 = w * 64;
            const int64_t jl = j0 + lane < A.T ? j0 + lane : A.T;
            const uint64_t bo = (uint64_t)A.bitoff[jl];
            const uint64_t be = (uint64_t)A.bitoff[(j0 + 64 < A.T ? j0 + 64 : A.T)];
            uint64_t bnext = (uint64_t)__shfl_down((unsigned long long)bo, 1, WAVE);
            if (lane == WAVE - 1 || j0 + lane + 1 >= A.T) bnext = be;
            unsigned long long rest = nw;
            while (rest) {
                const int b = __ffsll((long long)rest) - 1;
                rest &= rest - 1;
                const uint64_t ps = (uint64_t)__shfl((unsigned long long)bo, b, WAVE);
                const uint64_t pe = (uint64_t)__shfl((unsigned long long)bnext, b, WAVE);
                wave_dec_string<NI>(A, tb, C, stage, j0 + b, ps, pe);
            }
        } else if (A.raw_off) {
            unsigned long long rest = nw;
            while (rest) {
                const int b = __ffsll((long long)rest) - 1;
                rest &= rest - 1;
                const int64_t j = w * 64 + b;
                const int64_t e = A.raw_off[j + 1];
                for (int64_t i = A.raw_off[j] + lane; i < e; i += WAVE)
                    cache_dec(C, A, ckey(A, (uint32_t)raw_id(A.raw_mem, A.raw_host, A.raw_split, i)));
                if (A.implicit && lane == 0) {
                    const uint32_t r = lost_root(A, j);
                    if (r != 0xFFFFFFFFu) cache_dec(C, A, ckey(A, r));
                }
            }
        }
    }
}

// Huffman strings (Alg. 2's DecodeFind), one wave per 64-set word and one lane per set:
// a partial decode that stops at u* (a codeless u* is sought among the escaped ids, which
// come first and ascending; a coded u* is matched by its canonical code and the scan ends
// at the first larger code).  A set holding u* is marked covered; its members are
// decremented at once by the lane when its string is short and staged, else, after the
// word's search, by the whole wave (wave_dec_string, 32 slot intervals at a time).  The
// word's strings are contiguous: they are copied to LDS with coalesced loads first (when they
// fit).  Each wave loads the next word's covered mask and bit offsets before decoding the
// current one.  The search is bound by decode latency, so residency matters more than
// staging: with a stage of 256 words a block needs about 21 KB of LDS, and its registers let
// five blocks stay resident per CU (the grid asks for seven, which measured the same).  In a
// store without array rows (A.fused) the kernel also does k_apply's work: it records u* and,
// for a u* with a bitmap row, covers the row's sets and decrements their members.
constexpr int FH_NI = 32;                                  // slot intervals per pass of a long string
constexpr int STAGE_WORDS = (FH_NI * CK_SLOT) / 32 + 4;    // 260: also holds FH_NI intervals

HBM_KERNEL(k_find_huff, SelArgs, 256) {
    __shared__ Tabs tb;
    __shared__ uint32_t stage[256 / WAVE][STAGE_WORDS];
    __shared__ DecCache C;
    const unsigned lane = lane_id();
    const int wv = threadIdx.x / WAVE;
    const int64_t nwaves = (int64_t)nblk * (blockDim.x / WAVE);
    int64_t w = (int64_t)bid * (blockDim.x / WAVE) + wv;
    // next word's covered mask, this lane's set start and the word's end offset
    unsigned long long cov_n = 0;
    uint64_t bo_n = 0, be_n = 0;
    auto fetch = [&](int64_t ww) {
        const int64_t j0 = ww * 64;
        const int64_t j1 = j0 + 64 < A.T ? j0 + 64 : A.T;
        cov_n = A.covered[ww];
        bo_n = (uint64_t)A.bitoff[j0 + lane < j1 ? j0 + lane : j1];
        be_n = (uint64_t)A.bitoff[j1];
    };
    // the first word's reads, the tables' and the argmax partials' are all in flight together
    if (w < A.words) fetch(w);
    const uint32_t fe_len = A.ustar_enc >= 0 ? A.lens[A.ustar_enc] : 0u;  // the front code
    const uint32_t fe_code = fe_len ? A.codes[A.ustar_enc] : 0u;
    load_tabs(A, tb);
    cache_init(C);
    __syncthreads();
    unsigned long long key;
    const uint32_t u = ustar_of(A, x, key);
    // u*'s row rank, code length and code read together (any vertex has a table entry)
    const uint32_t us = key ? u : 0u;
    const int32_t hr = A.hot_rank ? A.hot_rank[us] : -1;
    const uint32_t ustar_len = A.lens[us];
    const uint32_t ucode = A.codes[us];
    if (key == 0) return;
    if (A.fused && bid == 0 && threadIdx.x == 0) record_ustar(A, x, u, key);
    if (hr >= 0) {
        if (A.fused) {  // k_apply's work, in this launch
            apply_words<FH_NI>(A, tb, C, stage[wv], hr, bid, nblk);
            __syncthreads();
            cache_flush(C, A);
        }
        return;
    }
    if (in_arr(A, u)) {
        arr_mark(A, A.ar_rank[u], bid, nblk);
        return;
    }
    const uint32_t ustar_code = ustar_len ? ucode : 0u;
    unsigned long long pacc = 0;  // profiling: this wave's algorithmic bytes
    for (; w < A.words; w += nwaves) {
        const unsigned long long cov = cov_n;
        const uint64_t bo = bo_n, be = be_n;
        if (w + nwaves < A.words) fetch(w + nwaves);
        const int64_t j0 = w * 64;
        const int64_t j1 = j0 + 64 < A.T ? j0 + 64 : A.T;
        const unsigned long long live = (j1 - j0 == 64 ? ~0ull : ((1ull << (j1 - j0)) - 1)) & ~cov;
        if (!live) {
            pacc += 8;  // the covered word
            continue;
        }
        const uint64_t b0 = (uint64_t)__shfl((unsigned long long)bo, 0, WAVE);
        // the next set's start ends this lane's set
        uint64_t bnext = (uint64_t)__shfl_down((unsigned long long)bo, 1, WAVE);
        if (j0 + lane + 1 >= j1) bnext = be;
        if (A.pbytes) {  // the covered word, and each uncovered set's string and its two offsets
            const uint32_t bits = wave_sum(((live >> lane) & 1ull) ? (uint32_t)(bnext - bo) : 0u);
            pacc += 8ull + ((unsigned long long)bits + 7) / 8 + 16ull * __popcll(live);
        }
        const uint64_t wlo = b0 >> 5;
        const uint64_t nw = ((be + 31) >> 5) - wlo + 1;  // +1: peek32 reads a word ahead
        const bool staged = nw <= (uint64_t)STAGE_WORDS;
        const uint32_t *buf = A.payload;
        uint64_t off = 0;
        if (staged) {
            stage_words(stage[wv], A.payload + wlo, nw);
            wave_sync();
            buf = stage[wv];
            off = wlo * 32;
        }
        bool found = false;
        uint64_t p0 = 0, p1 = 0;
        uint32_t lroot = 0xFFFFFFFFu;
        if ((live >> lane) & 1ull) {
            p0 = bo - off;
            p1 = bnext - off;
            lroot = lost_root(A, j0 + lane);
            found = lroot == u || huff_contains(A, tb, buf, p0, p1, u, ustar_len, ustar_code, fe_len, fe_code);
        }
        const unsigned long long nwm = __ballot(found);
        if (lane == 0 && nwm) {
            A.newly[w] = nwm;
            A.covered[w] = cov | nwm;
        }
        // a long string, or any string not staged in LDS (decoding it from device memory
        // would be one dependent load per code in this lane): the whole wave decrements it
        // below, from LDS copies of its slot intervals
        const bool wide = found && (!staged || p1 - p0 > (uint64_t)BIG_BITS);
        if (found && !wide) {
            huff_decrement(A, tb, C, buf, p0, p1);
            if (lroot != 0xFFFFFFFFu) cache_dec(C, A, ckey(A, lroot));
        }
        unsigned long long wm = __ballot(wide);
        wave_sync();  // the word's staged strings are no longer read
        while (wm) {
            const int b = __ffsll((long long)wm) - 1;
            wm &= wm - 1;
            const uint64_t ps = (uint64_t)__shfl((unsigned long long)bo, b, WAVE);
            const uint64_t pe = (uint64_t)__shfl((unsigned long long)bnext, b, WAVE);
            wave_dec_string<FH_NI>(A, tb, C, stage[wv], j0 + b, ps, pe);
        }
    }
    if (A.pbytes && lane == 0 && pacc) atomicAdd(&A.pbytes[blockIdx.x & (PB_SLOTS - 1)], pacc);
    __syncthreads();
    cache_flush(C, A);
}

// Records u* (bit 0 of block 0) and, when u* has a row (bitmap or array) or the store is
// plain, marks the newly covered sets of every word and decrements their members: plain ids
// by the lanes, Huffman strings one at a time by the whole wave (wave_dec_string, 64 slot
// intervals at a time); a cold u* of a Huffman store was handled by k_find_huff.
constexpr int AP_NI = WAVE;
constexpr int AP_STAGE = (AP_NI * CK_SLOT) / 32 + 4;
HBM_KERNEL(k_apply, SelArgs, 256) {
    const int t = x;
    __shared__ DecCache C;
    __shared__ Tabs tb;
    __shared__ uint32_t stage[256 / WAVE][AP_STAGE];
    unsigned long long key;
    const uint32_t u = ustar_of(A, t, key);
    if (key == 0) return;  // cannot happen for k <= n: some vertex is always unselected
    if (bid == 0 && threadIdx.x == 0) record_ustar(A, t, u, key);
    const int32_t r = A.hot_rank ? A.hot_rank[u] : -1;
    // a cold u*: the Huffman find step already covered and decremented
    if (r < 0 && A.huff && !in_arr(A, u)) return;
    if (A.huff) load_tabs(A, tb);
    cache_init(C);
    __syncthreads();
    apply_words<AP_NI>(A, tb, C, stage[threadIdx.x / WAVE], r, bid, nblk);
    __syncthreads();
    cache_flush(C, A);
}

// hot counts -= popcount(row AND newly): block b covers hot ranks [256 (b mod hx), +256)
// over the words of segment b / hx
HBM_KERNEL(k_dec_hot, SelArgs, 256) {
    (void)nblk;
    (void)x;
    const int64_t h = (int64_t)(bid % (uint32_t)A.hx) * blockDim.x + threadIdx.x;
    const int64_t w0 = (int64_t)(bid / (uint32_t)A.hx) * A.seg;
    const int64_t w1 = w0 + A.seg < A.words ? w0 + A.seg : A.words;
    uint32_t acc = 0;
    for (int64_t w = w0; w < w1; w++) {
        const unsigned long long nwv = A.newly[w];
        if (nwv && h < A.nhot) acc += __popcll(A.bitmap[w * (int64_t)A.nhot + h] & nwv);
    }
    if (acc) atomicSub(&A.counts[ckey(A, (uint32_t)A.hot[h])], acc);
}

// array-row counts -= the row's entries whose set is newly covered: one coalesced pass over every
// chunk's entries, a thread per entry; an entry whose set is newly covered finds its row by a
// binary search of the chunk's offsets and decrements it through the block's combining cache
// (most entries are not newly covered, so most threads only read their entry and one word)
HBM_KERNEL(k_dec_arr, SelArgs, 256) {
    (void)x;
    __shared__ DecCache C;
    cache_init(C);
    __syncthreads();
    const int64_t tid = bid * (int64_t)blockDim.x + threadIdx.x;
    const int64_t nthr = (int64_t)nblk * blockDim.x;
    for (int64_t ch = 0; ch < A.nchunks; ch++) {
        const int64_t *o = A.ar_off + ch * (int64_t)(A.nar + 1);
        const int64_t e0 = o[0], e1 = o[A.nar];
        const unsigned long long *nw = A.newly + (ch << 10);
        for (int64_t i = e0 + tid; i < e1; i += nthr) {
            const uint32_t low = A.ar_low[i];
            if (!((nw[low >> 6] >> (low & 63)) & 1ull)) continue;
            // row: the last a with o[a] <= i
            int32_t lo = 0, hi = A.nar - 1;
            while (lo < hi) {
                const int32_t mid = (lo + hi + 1) >> 1;
                if (o[mid] <= i) lo = mid;
                else hi = mid - 1;
            }
            cache_dec(C, A, ckey(A, (uint32_t)A.ar_hot[lo]));
        }
    }
    __syncthreads();
    cache_flush(C, A);
}

void select_free(Ctx &c) {
    for (auto &g : c.sel_graphs) (void)hipGraphExecDestroy(g.exec);
    c.sel_graphs.clear();
    if (c.cap_stream) (void)hipStreamDestroy(c.cap_stream);
    c.cap_stream = nullptr;
    buf_free(c, c.sel_desc);
    if (c.sel_hdesc) (void)hipHostFree(c.sel_hdesc);
    c.sel_hdesc = nullptr;
    c.sel_hdesc_bytes = 0;
    SelState &S = c.sel;
    for (Buf *b : {&S.counts, &S.selmask, &S.covered, &S.newly, &S.keys, &S.partial, &S.cand, &S.cpos, &S.csel,
                   &S.sbcnt, &S.sboff, &S.slut, &S.ssym})
        buf_free(c, *b);
    S.words_cap = 0;
}

namespace {

// ---------------------------------------------------------------- sparse count slots
// The vertices with a nonzero store frequency, ascending: per block of SL_SPAN vertices a
// count, an exclusive scan of the counts (its last entry is the number of slots, left on the
// device for the kernels), then each block writes its slots in order: the vertex, the
// vertex's slot, and the slot's starting count.
constexpr int SL_T = 256, SL_ITEMS = 16, SL_SPAN = SL_T * SL_ITEMS;

__global__ __launch_bounds__(SL_T) void k_slot_count(const uint32_t *hist, int32_t n, uint32_t *bcnt) {
    __shared__ uint32_t ws[SL_T / WAVE];
    const int64_t base = (int64_t)blockIdx.x * SL_SPAN;
    uint32_t c = 0;
    for (int i = 0; i < SL_ITEMS; i++) {
        const int64_t v = base + (int64_t)i * SL_T + threadIdx.x;
        if (v < n && hist[v]) c++;
    }
    c = wave_sum(c);
    if (lane_id() == 0) ws[threadIdx.x / WAVE] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < SL_T / WAVE; w++) t += ws[w];
        bcnt[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(SL_T) void k_slot_write(const uint32_t *hist, int32_t n, const int64_t *boff,
                                                     uint32_t *cand, int32_t *cpos, uint32_t *ccnt) {
    __shared__ uint32_t ws[SL_T / WAVE];
    const int64_t base = (int64_t)blockIdx.x * SL_SPAN;
    const int wv = threadIdx.x / WAVE;
    int64_t at = boff[blockIdx.x];
    for (int i = 0; i < SL_ITEMS; i++) {
        const int64_t v = base + (int64_t)i * SL_T + threadIdx.x;
        const uint32_t h = v < n ? hist[v] : 0u;
        const uint32_t f = h ? 1u : 0u;
        const uint32_t inc = wave_incl_scan(f);
        if (lane_id() == WAVE - 1) ws[wv] = inc;
        __syncthreads();
        uint32_t before = 0, tot = 0;
        for (int x = 0; x < SL_T / WAVE; x++) {
            if (x < wv) before += ws[x];
            tot += ws[x];
        }
        if (f) {
            const int64_t p = at + before + inc - 1;
            cand[p] = (uint32_t)v;
            cpos[v] = (int32_t)p;
            ccnt[p] = h;
        }
        at += tot;
        __syncthreads();
    }
}

// Decode tables over slots: the LUT's direct entries and the canonical symbol table name slots
// instead of vertices (every coded vertex occurs in the warm-up sets, so it has a slot).
__global__ void k_slot_tables(const uint32_t *lut, const int32_t *symtab, int64_t nsym, const int32_t *cpos,
                              uint32_t *slut, int32_t *ssym) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nthr = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = tid; i < (1 << LUT_BITS); i += nthr) {
        const uint32_t e = lut[i];
        slut[i] = (e & 31u) ? ((uint32_t)cpos[e >> 5] << 5) | (e & 31u) : e;
    }
    for (int64_t i = tid; i < nsym; i += nthr) ssym[i] = cpos[symtab[i]];
}

// Build the slots of context c on the root stream (SPARSE_COUNTS 1), or, by default, when the
// graph is large and the slots few enough for the argmax to read at most half of what dense
// counts cost (8 bytes per slot and a bit per vertex against 4 bytes per vertex).  Returns the
// number of slots, or -1 for dense counts.
static int64_t build_slots(Ctx &root, Ctx &c) {
    const int32_t n = c.g.n;
    if (c.sparse_counts == 0 || !c.s.hist.p || c.s.nsets == 0) return -1;
    if (c.sparse_counts == 2 && n < (1 << 22)) return -1;
    SelState &S = c.sel;
    const int64_t nblk = ((int64_t)n + SL_SPAN - 1) / SL_SPAN;
    buf_grow(c, S.sbcnt, (size_t)(nblk + 1) * 4, false);
    buf_grow(c, S.sboff, (size_t)(nblk + 1) * 8, false);
    const hipStream_t st = root.stream;
    HBM_HIP(hipMemsetAsync(S.sbcnt.as<uint32_t>() + nblk, 0, 4, st));  // the scan's last input
    k_slot_count<<<(unsigned)nblk, SL_T, 0, st>>>(c.s.hist.as<uint32_t>(), n, S.sbcnt.as<uint32_t>());
    HBM_HIP(hipGetLastError());
    scan_u32_to_i64(root, S.sbcnt.as<uint32_t>(), S.sboff.as<int64_t>(), nblk + 1, 0);
    int64_t m = 0;
    HBM_HIP(hipMemcpyAsync(&m, S.sboff.as<int64_t>() + nblk, 8, hipMemcpyDeviceToHost, st));
    HBM_HIP(hipStreamSynchronize(st));
    if (c.sparse_counts == 2 && 8 * m + n / 8 >= 2 * (int64_t)n) return -1;
    buf_grow(c, S.cand, (size_t)std::max<int64_t>(m, 1) * 4, false);
    buf_grow(c, S.cpos, (size_t)n * 4, false);
    buf_grow(c, S.csel, (size_t)((m + 31) / 32 + 1) * 4, false);
    buf_grow(c, S.counts, (size_t)std::max<int64_t>(m, 1) * 4, false);
    k_slot_write<<<(unsigned)nblk, SL_T, 0, st>>>(c.s.hist.as<uint32_t>(), n, S.sboff.as<int64_t>(),
                                                   S.cand.as<uint32_t>(), S.cpos.as<int32_t>(), S.counts.as<uint32_t>());
    HBM_HIP(hipGetLastError());
    return m;
}

// Per-job launch geometry and algorithmic bytes of one selection iteration.
struct SelJob {
    SelArgs A;
    bool huff;
    uint32_t g_arg, g_find, g_apply, g_hot, g_arr;
    double b_arg, b_find, b_apply;
};

// Selection state in caller-provided device memory (dense counts, no profiling); sizes
// as sel_fixed_layout computes them.
struct SelBufs {
    uint32_t *counts, *selmask;
    unsigned long long *covered, *newly, *partial, *keys;
};

static unsigned argmax_blocks(const Ctx &root, int32_t n) {
    return grid_for(((int64_t)n + 3) / 4, 256 * AM_UNROLL, (int64_t)root.num_cus * 8);
}

// gfix: grids that depend only on the graph and the store's shape (a graph of launches captured
// once then serves stores of any size: every selection kernel strides over its work)
SelJob plan_job(Ctx &root, Ctx &c, int32_t k, unsigned long long *keys, const SelBufs *fixed = nullptr,
                bool gfix = false) {
    Store &s = c.s;
    SelState &S = c.sel;
    const int32_t n = c.g.n;
    const int64_t T = s.nsets;
    const int64_t words = (T + 63) / 64;
    const unsigned g_arg = argmax_blocks(root, n);
    const bool huff = enc_huff(s.enc), raw = enc_raw(s.enc);
    const int64_t m = fixed ? -1 : build_slots(root, c);  // -1: dense counts
    if (!fixed) {
        if (m < 0) buf_grow(c, S.counts, (size_t)n * 4, false);
        buf_grow(c, S.selmask, ((size_t)n + 31) / 32 * 4, false);
        buf_grow(c, S.covered, (size_t)std::max<int64_t>(words, 1) * 8, false);
        buf_grow(c, S.newly, (size_t)std::max<int64_t>(words, 1) * 8, false);
        buf_grow(c, S.partial, (size_t)g_arg * 8, false);
    }
    SelJob J{};
    SelArgs &A = J.A;
    A.T = T;
    A.words = words;
    A.n = n;
    A.counts = fixed ? fixed->counts : S.counts.as<uint32_t>();
    A.cand = m >= 0 ? S.cand.as<uint32_t>() : nullptr;
    A.cpos = m >= 0 ? S.cpos.as<int32_t>() : nullptr;
    A.csel = m >= 0 ? S.csel.as<uint32_t>() : nullptr;
    A.ncand = m >= 0 ? S.sboff.as<int64_t>() + (((int64_t)n + SL_SPAN - 1) / SL_SPAN) : nullptr;
    if (root.prof.on && !fixed && huff && !root.pfind.p) {
        buf_alloc(root, root.pfind, PB_SLOTS * 8);
        buf_zero(root, root.pfind, 0, PB_SLOTS * 8);
    }
    A.pbytes = root.prof.on && !fixed && huff ? root.pfind.as<unsigned long long>() : nullptr;
    A.selmask = fixed ? fixed->selmask : S.selmask.as<uint32_t>();
    A.covered = fixed ? fixed->covered : S.covered.as<unsigned long long>();
    A.newly = fixed ? fixed->newly : S.newly.as<unsigned long long>();
    A.keys = keys;
    A.nhot = s.nhot;
    A.hot = s.hot.as<int32_t>();
    A.hot_rank = s.nhot ? s.hot_rank.as<int32_t>() : nullptr;
    A.bitmap = s.bitmap.as<unsigned long long>();
    A.raw_off = raw ? s.raw_off.as<int64_t>() : nullptr;  // BITMAX: every member is in a row
    A.raw_mem = raw ? s.raw_mem.as<int32_t>() : nullptr;
    A.raw_host = s.raw_host;
    A.raw_split = s.raw_split;
    A.implicit = s.implicit_roots && s.enc != HBM_ENC_BITMAX;
    A.seed = s.seed;
    A.huff = huff && T > 0;
    A.bitoff = s.bitoff.as<int64_t>();
    A.payload = s.payload.as<uint32_t>();
    A.lim = s.cbtab.as<uint64_t>();
    A.base = s.cbtab.as<int64_t>() + 34;
    A.symtab = s.symtab.as<int32_t>();
    A.lens = s.lens.as<uint8_t>();
    A.lut = s.lut.as<uint32_t>();
    if (huff && T > 0 && m >= 0) {  // decode straight to slots
        const int64_t nsym = std::max<int64_t>(s.cb.nsym, 1);
        buf_grow(c, S.slut, ((size_t)1 << LUT_BITS) * 4, false);
        buf_grow(c, S.ssym, (size_t)nsym * 4, false);
        k_slot_tables<<<grid_for(std::max<int64_t>(nsym, 1 << LUT_BITS), 256, 1024), 256, 0, root.stream>>>(
            s.lut.as<uint32_t>(), s.symtab.as<int32_t>(), s.cb.nsym, S.cpos.as<int32_t>(), S.slut.as<uint32_t>(),
            S.ssym.as<int32_t>());
        HBM_HIP(hipGetLastError());
        A.lut = S.slut.as<uint32_t>();
        A.symtab = S.ssym.as<int32_t>();
    }
    A.codes = s.codes.as<uint32_t>();
    A.minlen = s.cb.minlen;
    A.wbits = s.cb.wbits;
    A.ustar_enc = s.cb.ustar_enc;
    A.nraw = raw ? s.raw_count : 0;
    A.partial = fixed ? fixed->partial : S.partial.as<unsigned long long>();
    A.nparts = (int32_t)g_arg;
    A.hist = T > 0 ? s.hist.as<uint32_t>() : nullptr;
    A.ckb = s.ckb.as<uint8_t>();
    A.k = k;
    A.nar = T > 0 ? s.nar : 0;
    A.ar_rank = s.ar_rank.as<int32_t>();
    A.ar_hot = s.ar_hot.as<int32_t>();
    A.ar_off = s.ar_off.as<int64_t>();
    A.ar_low = s.ar_low.as<uint16_t>();
    A.nchunks = s.ar_chunks;
    A.nentries = s.ar_entries;
    // without array rows no set is marked by one launch and covered by the next, so the find
    // step can also record u* and cover a bitmap row's sets: one launch less per iteration
    A.fused = huff && T > 0 && A.nar == 0;
    A.hx = (int32_t)std::max<int64_t>(((int64_t)s.nhot + 255) / 256, 1);
    int64_t nseg = std::max<int64_t>(1, std::min<int64_t>(words, 4096 / A.hx));
    A.seg = std::max<int64_t>(1, (words + nseg - 1) / nseg);
    nseg = std::max<int64_t>(1, (words + A.seg - 1) / A.seg);
    J.huff = huff;
    J.g_arg = g_arg;
    if (T == 0) J.g_find = 0;
    else if (huff) J.g_find = gfix ? (uint32_t)root.num_cus * 7 : grid_for(words, 4, (int64_t)root.num_cus * 7);  // seven per CU (five stay resident)
    else J.g_find = (A.nraw > 0 || A.implicit || A.nar) ? (gfix ? (uint32_t)root.num_cus * 4 : grid_for((A.nraw + 3) / 4 + 1, 256, (int64_t)root.num_cus * 4)) : 0;
    J.g_apply = gfix ? (uint32_t)root.num_cus * 2 : grid_for(std::max<int64_t>(words, 1), 4, 1 << 20);
    // hot counts: segments past the words in use find no word to read
    J.g_hot = (T > 0 && s.nhot > 0) ? (uint32_t)(A.hx * (gfix ? std::max<int64_t>(1, 4096 / A.hx) : nseg)) : 0;
    J.g_arr = A.nar ? (gfix ? (uint32_t)root.num_cus * 4
                            : grid_for(std::max<int64_t>(A.nentries, 1), 256, (int64_t)root.num_cus * 8)) : 0;
    // algorithmic bytes: argmax reads every count and selection bit (sparse counts: the slots, and
    // the selection words of ids [0, k]) and clears the newly words; find reads every plain id
    // (for Huffman: the covered words and the strings and offsets of the uncovered sets, counted
    // on the device while profiling); apply reads and writes the covered and newly words (and
    // the hot row when u* is hot).
    J.b_arg = (m >= 0 ? 4.0 * m + m / 8.0 + 4.0 * std::min<int64_t>((n + 31) / 32, k / 32 + 1)
                      : 4.0 * n + 4.0 * ((n + 31) / 32)) +
              8.0 * words;
    J.b_find = huff ? 0.0 : 4.0 * A.nraw;
    J.b_apply = 24.0 * words;
    return J;
}

// A grouped launch over a prefix of a job list that is sorted by k (descending): at
// iteration t the jobs with k > t are a prefix, so one descriptor upload serves all
// iterations.
struct Plan {
    std::vector<size_t> jobs;  // indices into the job table, k descending
    std::vector<uint32_t> boff;
    const SelArgs *dargs = nullptr;
    const uint32_t *dboff = nullptr;
};

}  // namespace

// fixed != null (one job only): the selection state and keys live in the given device memory,
// and nothing is allocated, timed or profiled.
static void select_run(Ctx &root, const std::vector<Ctx *> &C, const std::vector<int32_t> &k,
                       std::vector<std::vector<int32_t>> &seeds, std::vector<std::vector<uint64_t>> &gains,
                       std::vector<uint64_t> &coverage, const SelBufs *fixed) {
    const size_t N = C.size();
    seeds.assign(N, {});
    gains.assign(N, {});
    coverage.assign(N, 0);
    if (!N) return;
    int32_t kmax = 0;
    std::vector<int64_t> koff(N + 1, 0);
    for (size_t i = 0; i < N; i++) {
        HBM_REQUIRE(C[i]->g.loaded, HBM_ESTATE, "no graph loaded");
        HBM_REQUIRE(k[i] >= 1 && k[i] <= C[i]->g.n, HBM_EINVAL, "k must be in [1, n]");
        kmax = std::max(kmax, k[i]);
        koff[i + 1] = koff[i] + k[i];
    }
    HBM_REQUIRE(!fixed || N == 1, HBM_EINVAL, "internal: fixed selection state serves one job");
    stage_reset(root);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (!fixed) {
        HBM_HIP(hipEventCreate(&e0));
        HBM_HIP(hipEventCreate(&e1));
        HBM_HIP(hipEventRecord(e0, root.stream));
        buf_grow(root, root.bkeys, (size_t)koff[N] * 8, false);
    }
    unsigned long long *dkeys = fixed ? fixed->keys : root.bkeys.as<unsigned long long>();
    const bool graph = root.select_graph && !fixed && !root.prof.on;
    std::vector<SelJob> J(N);
    for (size_t i = 0; i < N; i++) J[i] = plan_job(root, *C[i], k[i], dkeys + koff[i], fixed, graph);

    // job order: k descending (stable on the index)
    std::vector<size_t> order(N);
    for (size_t i = 0; i < N; i++) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return k[a] > k[b]; });
    enum { P_ALL_ARG, P_APPLY, P_HUFF, P_RAW, P_HOT, P_INIT, P_ARR, NPLAN };
    Plan plans[NPLAN];
    for (size_t i : order) {
        plans[P_ALL_ARG].jobs.push_back(i);
        if (!J[i].A.fused) plans[P_APPLY].jobs.push_back(i);
        plans[P_INIT].jobs.push_back(i);
        if (J[i].g_find && J[i].huff) plans[P_HUFF].jobs.push_back(i);
        if (J[i].g_find && !J[i].huff) plans[P_RAW].jobs.push_back(i);
        if (J[i].g_hot) plans[P_HOT].jobs.push_back(i);
        if (J[i].g_arr) plans[P_ARR].jobs.push_back(i);
    }
    auto blocks = [&](int p, size_t i) -> uint32_t {
        switch (p) {
            case P_ALL_ARG: return J[i].g_arg;
            case P_APPLY: return J[i].g_apply;
            case P_HUFF:
            case P_RAW: return J[i].g_find;
            case P_HOT: return J[i].g_hot;
            case P_ARR: return J[i].g_arr;
            default: return graph ? 1024u : grid_for(std::max<int64_t>({(int64_t)J[i].A.n, J[i].A.words, (int64_t)k[i]}), 256, 1024);
        }
    };
    // one upload of every plan's descriptors and block offsets (graph mode: always, into a
    // buffer at a fixed address that the captured launches read)
    std::vector<char> host;
    std::vector<size_t> aoff(NPLAN), boff_off(NPLAN);
    auto align = [&]() { host.resize((host.size() + 255) & ~size_t(255)); };
    const bool grouped = N > 1 || graph;
    for (int p = 0; p < NPLAN; p++) {
        Plan &P = plans[p];
        P.boff.assign(P.jobs.size() + 1, 0);
        for (size_t q = 0; q < P.jobs.size(); q++) P.boff[q + 1] = P.boff[q] + blocks(p, P.jobs[q]);
        if (!grouped) continue;
        align();
        aoff[p] = host.size();
        for (size_t i : P.jobs) {
            const char *a = reinterpret_cast<const char *>(&J[i].A);
            host.insert(host.end(), a, a + sizeof(SelArgs));
        }
        align();
        boff_off[p] = host.size();
        const char *b = reinterpret_cast<const char *>(P.boff.data());
        host.insert(host.end(), b, b + P.boff.size() * 4);
    }
    if (grouped) {
        char *d = nullptr;
        if (graph) {
            // the previous selection's graph has finished (selections end with a synchronisation),
            // so the descriptors may be rewritten in place
            if (root.sel_hdesc_bytes < host.size()) {
                const size_t cap = std::max<size_t>(host.size() * 2, size_t(64) << 10);
                buf_alloc(root, root.sel_desc, cap);
                if (root.sel_hdesc) (void)hipHostFree(root.sel_hdesc);
                root.sel_hdesc = nullptr;
                root.sel_hdesc_bytes = 0;
                HBM_HIP(hipHostMalloc(&root.sel_hdesc, cap, hipHostMallocDefault));
                root.sel_hdesc_bytes = cap;
            }
            std::memcpy(root.sel_hdesc, host.data(), host.size());
            HBM_HIP(hipMemcpyAsync(root.sel_desc.p, root.sel_hdesc, host.size(), hipMemcpyHostToDevice, root.stream));
            d = root.sel_desc.as<char>();
        } else {
            d = (char *)stage_upload(root, host.data(), host.size());
        }
        for (int p = 0; p < NPLAN; p++) {
            plans[p].dargs = reinterpret_cast<const SelArgs *>(d + aoff[p]);
            plans[p].dboff = reinterpret_cast<const uint32_t *>(d + boff_off[p]);
        }
    }
    // number of jobs of plan p still running at iteration t
    auto active = [&](int p, int t) -> uint32_t {
        const Plan &P = plans[p];
        uint32_t lo = 0, hi = (uint32_t)P.jobs.size();
        while (lo < hi) {
            const uint32_t mid = (lo + hi) / 2;
            if (k[P.jobs[mid]] > t) lo = mid + 1;
            else hi = mid;
        }
        return lo;
    };
    hipStream_t st = root.stream;
#define HBM_SEL_LAUNCH(PLAN, KERNEL, T_)                                                                  \
    do {                                                                                                \
        const Plan &P_ = plans[PLAN];                                                                   \
        const uint32_t cnt_ = active(PLAN, T_);                                                         \
        if (cnt_ && P_.boff[cnt_]) {                                                                    \
            if (!grouped) KERNEL<<<P_.boff[1], 256, 0, st>>>(J[P_.jobs[0]].A, T_);                      \
            else KERNEL##_g<<<P_.boff[cnt_], 256, 0, st>>>(GroupArgs<SelArgs>{P_.dargs, P_.dboff, cnt_, T_}); \
        }                                                                                               \
    } while (0)
    auto bytes_of = [&](int p, int t, double SelJob::*f) {
        double b = 0;
        const uint32_t cnt = active(p, t);
        for (uint32_t q = 0; q < cnt; q++) b += J[plans[p].jobs[q]].*f;
        return b;
    };
    auto prof_begin = [&](Ctx &r, const char *name) { return fixed ? -1 : hbm::prof_begin(r, name); };
    int ps_find = -1;  // profiling: a find_huff launch, credited with the bytes all of them read
    auto launch_all = [&]() {
        HBM_SEL_LAUNCH(P_INIT, k_sel_init, 0);
        for (int t = 0; t < kmax; t++) {
            int ps = prof_begin(root, "argmax");
            HBM_SEL_LAUNCH(P_ALL_ARG, k_argmax, t);
            prof_end(root, ps, ps >= 0 ? bytes_of(P_ALL_ARG, t, &SelJob::b_arg) : 0);
            if (active(P_HUFF, t)) {
                ps = prof_begin(root, "find_huff");
                HBM_SEL_LAUNCH(P_HUFF, k_find_huff, t);
                prof_end(root, ps, 0);
                if (ps >= 0) ps_find = ps;
            }
            if (active(P_RAW, t)) {
                ps = prof_begin(root, "find_raw");
                HBM_SEL_LAUNCH(P_RAW, k_find_raw, t);
                prof_end(root, ps, ps >= 0 ? bytes_of(P_RAW, t, &SelJob::b_find) : 0);
            }
            if (active(P_APPLY, t)) {
                ps = prof_begin(root, "apply");
                HBM_SEL_LAUNCH(P_APPLY, k_apply, t);
                prof_end(root, ps, ps >= 0 ? bytes_of(P_APPLY, t, &SelJob::b_apply) : 0);
            }
            if (active(P_HOT, t)) {
                ps = prof_begin(root, "dec_hot");
                HBM_SEL_LAUNCH(P_HOT, k_dec_hot, t);
                prof_end(root, ps);
            }
            if (active(P_ARR, t)) {
                ps = prof_begin(root, "dec_arr");
                HBM_SEL_LAUNCH(P_ARR, k_dec_arr, t);
                prof_end(root, ps);
            }
        }
    };
    if (!graph) {
        launch_all();
    } else {
        // The k-iteration launch sequence as a HIP graph.  Its launches read their arguments from
        // the descriptor buffer, and the grids depend only on the store's shape, so one graph
        // serves every selection of that shape: captured on first use, replayed afterwards.
        std::vector<uint64_t> shape{(uint64_t)N, (uint64_t)(uintptr_t)root.sel_desc.p, (uint64_t)kmax};
        for (int p = 0; p < NPLAN; p++) {
            shape.push_back((uint64_t)plans[p].jobs.size());
            for (size_t q = 0; q < plans[p].jobs.size(); q++) shape.push_back((uint64_t)k[plans[p].jobs[q]]);
            for (uint32_t b : plans[p].boff) shape.push_back(b);
        }
        size_t hit = root.sel_graphs.size();
        for (size_t i = 0; i < root.sel_graphs.size(); i++)
            if (root.sel_graphs[i].shape == shape) hit = i;
        if (hit == root.sel_graphs.size()) {
            if (!root.cap_stream) HBM_HIP(hipStreamCreate(&root.cap_stream));
            HBM_HIP(hipStreamBeginCapture(root.cap_stream, hipStreamCaptureModeRelaxed));
            st = root.cap_stream;
            launch_all();
            st = root.stream;
            hipGraph_t g = nullptr;
            const hipError_t ec = hipStreamEndCapture(root.cap_stream, &g);
            if (ec != hipSuccess || !g) {
                (void)hipGetLastError();
                throw Error{HBM_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(ec)};
            }
            Ctx::SelGraph sg;
            sg.shape = std::move(shape);
            const hipError_t e = hipGraphInstantiate(&sg.exec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) throw Error{HBM_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e)};
            constexpr size_t GRAPH_CACHE = 16;
            if (root.sel_graphs.size() >= GRAPH_CACHE) {
                (void)hipGraphExecDestroy(root.sel_graphs.front().exec);
                root.sel_graphs.erase(root.sel_graphs.begin());
            }
            root.sel_graphs.push_back(std::move(sg));
        } else if (hit + 1 != root.sel_graphs.size()) {  // most recently used last
            Ctx::SelGraph sg = std::move(root.sel_graphs[hit]);
            root.sel_graphs.erase(root.sel_graphs.begin() + (ptrdiff_t)hit);
            root.sel_graphs.push_back(std::move(sg));
        }
        HBM_HIP(hipGraphLaunch(root.sel_graphs.back().exec, root.stream));
    }
#undef HBM_SEL_LAUNCH
    HBM_HIP(hipGetLastError());
    if (ps_find >= 0) {
        std::vector<unsigned long long> part(PB_SLOTS);
        HBM_HIP(hipMemcpyAsync(part.data(), root.pfind.p, PB_SLOTS * 8, hipMemcpyDeviceToHost, root.stream));
        HBM_HIP(hipStreamSynchronize(root.stream));
        buf_zero(root, root.pfind, 0, PB_SLOTS * 8);
        double total = 0;
        for (unsigned long long v : part) total += (double)v;
        prof_add(root, ps_find, total, 0.0);
    }
    std::vector<unsigned long long> keys((size_t)koff[N]);
    HBM_HIP(hipMemcpyAsync(keys.data(), dkeys, (size_t)koff[N] * 8, hipMemcpyDeviceToHost, st));
    float ms = 0;
    if (fixed) {
        HBM_HIP(hipStreamSynchronize(st));
    } else {
        HBM_HIP(hipEventRecord(e1, st));
        HBM_HIP(hipEventSynchronize(e1));
        HBM_HIP(hipEventElapsedTime(&ms, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    for (size_t i = 0; i < N; i++) {
        C[i]->t_select += ms;
        seeds[i].resize((size_t)k[i]);
        gains[i].resize((size_t)k[i]);
        uint64_t cov = 0;
        for (int t = 0; t < k[i]; t++) {
            const unsigned long long key = keys[(size_t)(koff[i] + t)];
            HBM_REQUIRE(key != 0, HBM_EDEVICE, "internal: empty argmax");
            seeds[i][(size_t)t] = (int32_t)(~(uint32_t)key);
            gains[i][(size_t)t] = (uint64_t)(key >> 32) - 1;
            cov += gains[i][(size_t)t];
        }
        coverage[i] = cov;
    }
}

void select_batch(Ctx &root, const std::vector<Ctx *> &C, const std::vector<int32_t> &k,
                  std::vector<std::vector<int32_t>> &seeds, std::vector<std::vector<uint64_t>> &gains,
                  std::vector<uint64_t> &coverage) {
    select_run(root, C, k, seeds, gains, coverage, nullptr);
}

// ------------------------------------------------------------------ selection without allocation
// For callers that cannot allocate device memory (work under graph capture, tight serving
// loops, harnesses that forbid hipMalloc): the selection state of hbm_select_seeds_noalloc
// lives in this fixed array.  Each device the library runs on holds its own copy until the
// process ends; host code reaches it only through the address hipGetSymbolAddress gives.
constexpr size_t NOALLOC_BYTES = size_t(48) << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
static std::once_flag g_noalloc_once[NOALLOC_MAX_DEVICES];
static void *g_noalloc_ptr[NOALLOC_MAX_DEVICES];
static hipError_t g_noalloc_err[NOALLOC_MAX_DEVICES];

// Once per device, with that device current: the device address of this device's copy.
void noalloc_setup(int device) {
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return;
    std::call_once(g_noalloc_once[device], [device] {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_noalloc_err[device] = e;
        if (e == hipSuccess && p) g_noalloc_ptr[device] = p;
        else (void)hipGetLastError();
    });
}

size_t noalloc_capacity() { return NOALLOC_BYTES; }

// Bytes of selection state a k-seed selection over context c's store needs; fills `b` with
// their places inside `base` when it is given.
static size_t sel_fixed_layout(const Ctx &root, const Ctx &c, int32_t k, char *base, SelBufs *b) {
    const int32_t n = c.g.n;
    const int64_t T = c.s.nsets;
    const int64_t words = std::max<int64_t>((T + 63) / 64, 1);
    const bool huff = enc_huff(c.s.enc);
    size_t at = 0;
    auto take = [&](size_t bytes) {
        const size_t o = at;
        at = (at + bytes + 255) & ~size_t(255);
        return base ? base + o : nullptr;
    };
    char *counts = take((size_t)n * 4);
    char *selmask = take(((size_t)n + 31) / 32 * 4);
    char *covered = take((size_t)words * 8);
    char *newly = take((size_t)words * 8);
    char *partial = take((size_t)argmax_blocks(root, n) * 8);
    char *keys = take((size_t)k * 8);
    if (b) {
        b->counts = (uint32_t *)counts;
        b->selmask = (uint32_t *)selmask;
        b->covered = (unsigned long long *)covered;
        b->newly = (unsigned long long *)newly;
        b->partial = (unsigned long long *)partial;
        b->keys = (unsigned long long *)keys;
    }
    return at;
}

void select_seeds_noalloc(Ctx &c, int32_t k, int32_t *seeds, uint64_t *gains, uint64_t *coverage) {
    noalloc_setup(c.device);  // a no-op after hbm_create's call on this device
    HBM_REQUIRE(c.device >= 0 && c.device < NOALLOC_MAX_DEVICES, HBM_EDEVICE, "device index out of range");
    if (!g_noalloc_ptr[c.device])
        throw Error{HBM_EDEVICE, std::string("hipGetSymbolAddress of the selection scratch: ") +
                                     hipGetErrorString(g_noalloc_err[c.device])};
    const size_t need = sel_fixed_layout(c, c, k, nullptr, nullptr);
    HBM_REQUIRE(need <= NOALLOC_BYTES, HBM_EINVAL,
                "selection state needs " + std::to_string(need) + " bytes, the fixed scratch holds " +
                    std::to_string(NOALLOC_BYTES) + " (fewer vertices, sets or seeds)");
    SelBufs b{};
    sel_fixed_layout(c, c, k, (char *)g_noalloc_ptr[c.device], &b);
    std::vector<std::vector<int32_t>> s;
    std::vector<std::vector<uint64_t>> g;
    std::vector<uint64_t> cov;
    select_run(c, std::vector<Ctx *>{&c}, std::vector<int32_t>{k}, s, g, cov, &b);
    std::copy(s[0].begin(), s[0].end(), seeds);
    std::copy(g[0].begin(), g[0].end(), gains);
    *coverage = cov[0];
}

void select_seeds(Ctx &c, int32_t k, int32_t *seeds, uint64_t *gains, uint64_t *coverage) {
    std::vector<std::vector<int32_t>> s;
    std::vector<std::vector<uint64_t>> g;
    std::vector<uint64_t> cov;
    select_batch(c, std::vector<Ctx *>{&c}, std::vector<int32_t>{k}, s, g, cov);
    std::copy(s[0].begin(), s[0].end(), seeds);
    std::copy(g[0].begin(), g[0].end(), gains);
    *coverage = cov[0];
}

}  // namespace hbm
