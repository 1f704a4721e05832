// store.hip -- block-based sampling-and-encoding (Alg. 1) into the RR store.
//
// A request for sets [nsets, theta) runs in blocks sized to the scratch arena.
// With an encoding, the first request begins with a warm-up block over sets
// [0, W): their vertex frequencies give the hot set and the Huffman codebook
// (Alg. 1's first block; never rebuilt).  When the first block covers [0, W) it
// is encoded and stored whole once the model is built; otherwise the warm-up
// sets are pure functions of their index and are sampled again in the blocks
// that store them.  After each block the raw members are dropped; only the
// encoded form stays (the "Deallocate R_i" step).
//
// Store layouts (device memory):
//   hist      uint32[n]   frequency of every vertex over all sets (UpdateHistogram)
//   RAW       raw_off int64[nsets+1], raw_mem int32[]: ascending ids (all of a set,
//             or its part without rows under HOT_BITMAP); with a spill cap the ids past
//             a split point live in pinned host memory
//   HOT rows  bitmap uint64[ceil(nsets/64) * nhot], word-major: the bit of set j
//             for hot rank r is bit j%64 of word (j/64)*nhot + r (the Bitmax bit
//             matrix of its encoding section, restricted to hot vertices; BITMAX
//             itself is this matrix over all n vertices)
//   ARRAY rows (optional) per chunk of 2^16 sets, each sparse hot vertex's
//             ascending 16-bit set offsets: ar_off int64[chunks * (nar + 1)],
//             ar_low uint16[]
//   HUFFMAN   bitoff int64[nsets+1]; set j is bits [bitoff[j], bitoff[j+1]) of an
//             MSB-first stream: Elias-gamma(nesc+1), the nesc codeless ids as
//             fixed-width fields (the CP copies kept in-band), then the canonical
//             codes of the coded ids, the warm-up top vertex first (the u*
//             swap-to-front of the Huffmax encoding section), the rest in
//             canonical (length, id) order, i.e. ascending left-justified value;
//             ckb uint8 per 256 payload bits: the distance to the next code start
//   With implicit roots, a root that has no row is left out of its set's stored
//   part and regenerated from (seed, j).
#include <rocprim/device/device_segmented_radix_sort.hpp>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>

#include "hbm_device.h"
#include "hbm_internal.h"

namespace hbm {

struct BlockView {
    const uint32_t *mem;
    const uint32_t *pos;
    const uint32_t *size;
    int64_t nb;
};

// one wave per set: lanes stride over its members
struct HistArgs {
    BlockView bv;
    uint32_t *hist;
};
HBM_KERNEL(k_hist_add, HistArgs, 256) {
    const BlockView &bv = A.bv;
    uint32_t *__restrict__ hist = A.hist;
    const uint64_t wave = (bid * (uint64_t)blockDim.x + threadIdx.x) / WAVE;
    const uint64_t nw = (uint64_t)nblk * blockDim.x / WAVE;
    const unsigned lane = lane_id();
    for (uint64_t b = wave; b < (uint64_t)bv.nb; b += nw) {
        const uint32_t p = bv.pos[b], s = bv.size[b];
        for (uint32_t i = lane; i < s; i += WAVE) atomicAdd(&hist[bv.mem[p + i]], 1u);
    }
}

// per-set count of members kept as plain ids (all of them when hot_rank is null); one wave per set
struct SplitArgs {
    BlockView bv;
    const int32_t *hot_rank;      // null: no hot rows
    int64_t j0;
    const int64_t *off;           // raw offsets of the block's sets (null: bitmap only)
    int32_t *raw;
    int32_t *raw_host;            // ids from raw_split on (spilled store), else unused
    int64_t raw_split;
    unsigned long long *bitmap;
    int32_t nhot;
    uint32_t *cnt;                // per-set plain-id counts (cold_count output)
    int implicit;                 // implicit roots: a set's root is not written as a plain id
    uint64_t seed;
    uint32_t n;
    const int32_t *ar_rank;       // array-row members are neither cold nor bitmap bits (may be null)
};
HBM_KERNEL(k_cold_count, SplitArgs, 256) {
    const BlockView &bv = A.bv;
    const int32_t *__restrict__ hot_rank = A.hot_rank;
    uint32_t *__restrict__ out = A.cnt;
    const uint64_t wave = (bid * (uint64_t)blockDim.x + threadIdx.x) / WAVE;
    const uint64_t nw = (uint64_t)nblk * blockDim.x / WAVE;
    const unsigned lane = lane_id();
    for (uint64_t b = wave; b < (uint64_t)bv.nb; b += nw) {
        const uint32_t p = bv.pos[b], s = bv.size[b];
        uint32_t c = s;
        if (hot_rank || A.implicit || A.ar_rank) {
            const uint32_t root = dropped_root(A.implicit, A.seed, (uint64_t)A.j0 + b, A.n);
            c = 0;
            for (uint32_t i = lane; i < s; i += WAVE) {
                const uint32_t v = bv.mem[p + i];
                c += (!hot_rank || hot_rank[v] < 0) && (!A.ar_rank || A.ar_rank[v] < 0) && v != root;
            }
            c = wave_sum(c);
        }
        if (lane == 0) out[b] = c;
    }
    if (bid == 0 && threadIdx.x == 0) out[bv.nb] = 0u;  // the scan covers one extra element
}

// Copy plain ids to the raw store and set hot bits.  One wave per set.
HBM_KERNEL(k_split, SplitArgs, 256) {
    const BlockView &bv = A.bv;
    const int32_t *__restrict__ hot_rank = A.hot_rank;
    const int64_t j0 = A.j0;
    const int64_t *__restrict__ off = A.off;
    int32_t *__restrict__ raw = A.raw;
    unsigned long long *__restrict__ bitmap = A.bitmap;
    const int32_t nhot = A.nhot;
    const uint64_t wave = (bid * (uint64_t)blockDim.x + threadIdx.x) / WAVE;
    const uint64_t nw = (uint64_t)nblk * blockDim.x / WAVE;
    const unsigned lane = lane_id();
    for (uint64_t b = wave; b < (uint64_t)bv.nb; b += nw) {
        const uint32_t p = bv.pos[b], s = bv.size[b];
        const int64_t o = off ? off[b] : 0;
        const uint64_t j = (uint64_t)j0 + b;
        const uint32_t root = dropped_root(A.implicit, A.seed, j, A.n);
        uint32_t written = 0;
        for (uint32_t base = 0; base < s; base += WAVE) {
            const uint32_t i = base + lane;
            uint32_t v = 0;
            int32_t r = -1;
            if (i < s) {
                v = bv.mem[p + i];
                if (hot_rank) r = hot_rank[v];
            }
            const bool cold = i < s && r < 0 && v != root && !(A.ar_rank && A.ar_rank[v] >= 0);
            const uint64_t m = __ballot(cold);
            if (cold && raw) {
                const int64_t at = o + written + __popcll(m & ((1ull << lane) - 1));
                if (at < A.raw_split) raw[at] = (int32_t)v;
                else A.raw_host[at - A.raw_split] = (int32_t)v;
            }
            written += __popcll(m);
            if (i < s && r >= 0) atomicOr(&bitmap[(j >> 6) * (uint64_t)nhot + r], 1ull << (j & 63));
        }
    }
}

// ------------------------------------------------------------------ Huffman stream
struct HuffEnc {
    const unsigned long long *enc8;  // per vertex: code | length << 32 | (has a row) << 40
    const uint8_t *lens;
    const uint32_t *codes;
    const int32_t *hot_rank;  // may be null
    int32_t ustar;
    int32_t wbits;
    int implicit;             // implicit roots: a set's root is not coded
    uint64_t seed;
    int64_t j0;               // set index of the block's first set
    uint32_t n;
    const int32_t *ar_rank;   // array-row members are not coded (may be null)
};
struct HuffArgs {
    BlockView bv;
    HuffEnc h;
    uint64_t *bits;                    // per-set bit lengths (huff_bits output)
    uint32_t *meta;                    // per set: escapes | (u*_enc present) << 31
    const int64_t *bitoff;             // start bits of the block's sets
    uint32_t *payload;
    uint8_t *ckb;                      // code-boundary slots (see CK_SLOT)
    unsigned long long *nesc_total;
};

__device__ __forceinline__ int floor_log2_u32(uint32_t x) { return 31 - __clz(x); }

// One wave per set (sets range from a few members to millions): lanes stride over the
// members; the set's bit length is gamma(nesc + 1) + nesc * W + the code lengths.
// The escape count and whether u*_enc is present are kept in `meta` for the writer.
HBM_KERNEL(k_huff_bits, HuffArgs, 256) {
    const BlockView &bv = A.bv;
    const HuffEnc &h = A.h;
    const unsigned lane = lane_id();
    const uint64_t nw = (uint64_t)nblk * (blockDim.x / WAVE);
    for (uint64_t b = bid * (uint64_t)(blockDim.x / WAVE) + threadIdx.x / WAVE; b < (uint64_t)bv.nb; b += nw) {
        const uint32_t p = bv.pos[b], s = bv.size[b];
        const uint32_t root = dropped_root(h.implicit, h.seed, (uint64_t)h.j0 + b, h.n);
        uint64_t bits = 0;
        uint32_t nesc = 0, front = 0;
        for (uint32_t i = lane; i < s; i += WAVE) {
            const uint32_t v = bv.mem[p + i];
            const unsigned long long e = h.enc8[v];
            if ((e >> 40) || v == root) continue;  // in a row, or the dropped root
            const uint32_t L = (uint32_t)(e >> 32);
            if (L) bits += L;
            else nesc++;
            front |= (int32_t)v == h.ustar;
        }
        bits = wave_sum(bits);
        nesc = wave_sum(nesc);
        front = wave_sum(front);
        if (lane == 0) {
            A.bits[b] = bits + 2 * (uint64_t)floor_log2_u32(nesc + 1) + 1 + (uint64_t)nesc * h.wbits;
            A.meta[b] = nesc | (front ? 0x80000000u : 0u);
        }
    }
    if (bid == 0 && threadIdx.x == 0) A.bits[bv.nb] = 0ull;  // the scan covers one extra element
}

// Record the code at bits [p, p + len) in the boundary slots: a slot position inside it (or at
// its start) gets the distance to the first boundary at or after it.
__device__ __forceinline__ void mark_slot(uint8_t *ckb, uint64_t p, uint32_t len) {
    const uint64_t m = (p + CK_SLOT - 1) / CK_SLOT;
    const uint64_t at = m * CK_SLOT;
    if (at < p + len) ckb[m] = (uint8_t)(at == p ? 0 : p + len - at);
}

// OR `nbits` (<= 32) bits of `value` into the stream at bit `pos`, MSB first.
__device__ __forceinline__ void put_bits(uint32_t *buf, uint64_t pos, uint32_t value, uint32_t nbits) {
    if (!nbits) return;
    const uint64_t w = pos >> 5;
    const uint32_t off = (uint32_t)(pos & 31);
    const uint64_t v64 = (uint64_t)value << (64 - nbits - off);
    const uint32_t hi = (uint32_t)(v64 >> 32), lo = (uint32_t)v64;
    if (hi) atomicOr(&buf[w], hi);
    if (lo) atomicOr(&buf[w + 1], lo);
}

// One wave per set.  Layout of a set's string: gamma(nesc + 1), the escaped (codeless)
// ids ascending at W bits, the code of u*_enc if present, then the other codes in
// canonical order (by code length, then id: ascending left-justified code value).
// Members arrive ascending by id, so an escape's place is its rank among the escapes
// (a ballot) and a code's place is its length class's offset (from a per-set histogram
// of code lengths) plus its rank among the earlier members of the same length.
HBM_KERNEL(k_huff_write, HuffArgs, 256) {
    const BlockView &bv = A.bv;
    const HuffEnc &h = A.h;
    uint32_t *__restrict__ payload = A.payload;
    __shared__ uint32_t cls_n[256 / WAVE][33];  // members per code length
    __shared__ uint64_t cls_at[256 / WAVE][33]; // next bit of each length class
    const unsigned lane = lane_id();
    const int wv = threadIdx.x / WAVE;
    const unsigned long long below = lane ? (~0ull >> (WAVE - lane)) : 0ull;
    const uint64_t nw = (uint64_t)nblk * (blockDim.x / WAVE);
    uint64_t esc_local = 0;
    for (uint64_t b = bid * (uint64_t)(blockDim.x / WAVE) + wv; b < (uint64_t)bv.nb; b += nw) {
        const uint32_t p = bv.pos[b], s = bv.size[b];
        const uint32_t root = dropped_root(h.implicit, h.seed, (uint64_t)h.j0 + b, h.n);
        const uint32_t meta = A.meta[b];
        const uint32_t nesc = meta & 0x7FFFFFFFu;
        const bool has_front = meta >> 31;
        const uint64_t pos0 = (uint64_t)A.bitoff[b];
        const uint32_t L = (uint32_t)floor_log2_u32(nesc + 1);
        uint64_t esc_pos = pos0 + 2 * L + 1;
        uint64_t code_pos = esc_pos + (uint64_t)nesc * h.wbits;
        if (lane == 0) {
            put_bits(payload, pos0 + L, nesc + 1, L + 1);
            if (has_front) {
                put_bits(payload, code_pos, h.codes[h.ustar], h.lens[h.ustar]);
                mark_slot(A.ckb, code_pos, h.lens[h.ustar]);
            }
        }
        if (has_front) code_pos += h.lens[h.ustar];
        // code length of member i in the coded part (0: in a row, escaped or the front vertex)
        // and its code, from one read of the packed table
        auto code_of = [&](uint32_t i, uint32_t &v, bool &esc, uint32_t &code) -> uint32_t {
            v = bv.mem[p + i];
            esc = false;
            const unsigned long long e = h.enc8[v];
            code = (uint32_t)e;
            if ((e >> 40) || v == root) return 0u;
            const uint32_t len = (uint32_t)(e >> 32);
            esc = len == 0;
            return (int32_t)v == h.ustar ? 0u : len;
        };
        if (lane < 33) cls_n[wv][lane] = 0u;
        wave_sync();
        for (uint32_t c0 = 0; c0 < s; c0 += WAVE) {
            uint32_t v, code;
            bool esc;
            const uint32_t len = c0 + lane < s ? code_of(c0 + lane, v, esc, code) : 0u;
            if (len) atomicAdd(&cls_n[wv][len], 1u);
        }
        wave_sync();
        {  // class offsets: exclusive prefix of count * length over lengths 1..32
            const uint64_t mine = lane >= 1 && lane <= 32 ? (uint64_t)cls_n[wv][lane] * lane : 0ull;
            const uint64_t incl = wave_incl_scan(mine);
            if (lane >= 1 && lane <= 32) cls_at[wv][lane] = code_pos + incl - mine;
        }
        wave_sync();
        for (uint32_t c0 = 0; c0 < s; c0 += WAVE) {
            uint32_t v = 0, code = 0;
            bool esc = false;
            const uint32_t len = c0 + lane < s ? code_of(c0 + lane, v, esc, code) : 0u;
            const unsigned long long em = __ballot(esc);
            if (esc) put_bits(payload, esc_pos + (uint64_t)__popcll(em & below) * h.wbits, v, h.wbits);
            esc_pos += (uint64_t)__popcll(em) * h.wbits;
            // rank among this chunk's members of the same length, one length class at a time
            unsigned long long pending = __ballot(len != 0);
            uint32_t rank = 0, lead_n = 0, lead_len = 0;
            while (pending) {
                const int leader = __ffsll((long long)pending) - 1;
                const uint32_t ll = __shfl(len, leader, WAVE);
                const unsigned long long m = __ballot(len == ll) & pending;
                if (len == ll) rank = (uint32_t)__popcll(m & below);
                if ((int)lane == leader) {
                    lead_n = (uint32_t)__popcll(m);
                    lead_len = ll;
                }
                pending &= ~m;
            }
            if (len) {
                const uint64_t at = cls_at[wv][len] + (uint64_t)rank * len;
                put_bits(payload, at, code, len);
                mark_slot(A.ckb, at, len);
            }
            wave_sync();
            if (lead_n) cls_at[wv][lead_len] += (uint64_t)lead_n * lead_len;
            wave_sync();
        }
        esc_local += nesc;
    }
    if (lane == 0 && esc_local) atomicAdd(A.nesc_total, (unsigned long long)esc_local);
}

// gather one int64 per job (the last offset of its scan) into out[i]
struct TailArgs {
    const int64_t *src;
    int64_t *dst;
};
HBM_KERNEL(k_tail, TailArgs, 64) {
    (void)bid;
    (void)nblk;
    (void)x;
    if (threadIdx.x == 0) *A.dst = *A.src;
}

// ------------------------------------------------------------------ decode of whole sets (inspection)
struct DecodeView {
    int enc;
    int64_t nsets;
    int32_t nhot;
    const int32_t *hot;
    const unsigned long long *bitmap;
    const int64_t *raw_off;
    const int32_t *raw_mem;
    const int32_t *raw_host;
    int64_t raw_split;
    int implicit;            // implicit roots: the root is regenerated unless its row holds it
    uint64_t seed;
    uint32_t n;
    const int32_t *hot_rank;
    int32_t nar;             // array rows (chunk-major offsets, sorted 16-bit set offsets)
    const int32_t *ar_hot;
    const int32_t *ar_rank;
    const int64_t *ar_off;
    const uint16_t *ar_low;
    const int64_t *bitoff;
    const uint32_t *payload;
    const uint64_t *lim;    // [34]
    const int64_t *base;    // [34]
    const int32_t *symtab;
    int32_t minlen;
    int32_t wbits;
};

__device__ __forceinline__ uint32_t decode_code(const DecodeView &d, uint64_t &pos) {
    const uint32_t w = peek32(d.payload, pos);
    int L = d.minlen;
    while ((uint64_t)w >= d.lim[L]) L++;
    const uint32_t code = w >> (32 - L);
    pos += (uint64_t)L;
    return (uint32_t)d.symtab[d.base[L] + (int64_t)code];
}

// count (out != null: write) the members of set j; returns the count
__device__ uint32_t decode_set(const DecodeView &d, int64_t j, int32_t *out) {
    uint32_t c = 0;
    if (d.nhot) {
        const unsigned long long *row = d.bitmap + (uint64_t)(j >> 6) * d.nhot;
        for (int32_t r = 0; r < d.nhot; r++)
            if ((row[r] >> (j & 63)) & 1ull) {
                if (out) out[c] = d.hot[r];
                c++;
            }
    }
    if (d.nar) {  // binary search of each array row's list in j's chunk
        const int64_t *o = d.ar_off + (j >> 16) * (int64_t)(d.nar + 1);
        const uint16_t low = (uint16_t)(j & 0xffff);
        for (int32_t a = 0; a < d.nar; a++) {
            int64_t lo = o[a], hi = o[a + 1];
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (d.ar_low[mid] < low) lo = mid + 1;
                else hi = mid;
            }
            if (lo < o[a + 1] && d.ar_low[lo] == low) {
                if (out) out[c] = d.ar_hot[a];
                c++;
            }
        }
    }
    if (d.raw_off) {
        for (int64_t i = d.raw_off[j]; i < d.raw_off[j + 1]; i++) {
            if (out) out[c] = raw_id(d.raw_mem, d.raw_host, d.raw_split, i);
            c++;
        }
    } else if (d.bitoff) {
        uint64_t pos = (uint64_t)d.bitoff[j];
        const uint64_t end = (uint64_t)d.bitoff[j + 1];
        const uint32_t L = __clz(peek32(d.payload, pos));
        pos += L;
        const uint32_t g = peek32(d.payload, pos) >> (31 - L);
        pos += L + 1;
        for (uint32_t q = 1; q < g; q++) {
            const uint32_t v = peek32(d.payload, pos) >> (32 - d.wbits);
            pos += d.wbits;
            if (out) out[c] = (int32_t)v;
            c++;
        }
        while (pos < end) {
            const uint32_t v = decode_code(d, pos);
            if (out) out[c] = (int32_t)v;
            c++;
        }
    }
    if (d.implicit) {
        const uint32_t r = rr_root(d.seed, (uint64_t)j, d.n);
        if ((!d.nhot || d.hot_rank[r] < 0) && (!d.nar || d.ar_rank[r] < 0)) {
            if (out) out[c] = (int32_t)r;
            c++;
        }
    }
    if (out) {  // ascending
        for (uint32_t x = 1; x < c; x++) {
            const int32_t v = out[x];
            int y = (int)x - 1;
            while (y >= 0 && out[y] > v) {
                out[y + 1] = out[y];
                y--;
            }
            out[y + 1] = v;
        }
    }
    return c;
}

__global__ void k_decode_count(DecodeView d, int64_t j0, int64_t cnt, uint32_t *__restrict__ sizes) {
    for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < cnt; b += (int64_t)gridDim.x * blockDim.x)
        sizes[b] = decode_set(d, j0 + b, nullptr);
}

__global__ void k_decode_write(DecodeView d, int64_t j0, int64_t cnt, const int64_t *__restrict__ off,
                               int32_t *__restrict__ out) {
    for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < cnt; b += (int64_t)gridDim.x * blockDim.x)
        decode_set(d, j0 + b, out + off[b]);
}

// ------------------------------------------------------------------ host side
static DecodeView make_view(Ctx &c) {
    Store &s = c.s;
    DecodeView d{};
    d.enc = s.enc;
    d.nsets = s.nsets;
    d.nhot = s.nhot;
    d.hot = s.hot.as<int32_t>();
    d.bitmap = s.bitmap.as<unsigned long long>();
    const bool huff = enc_huff(s.enc), raw = enc_raw(s.enc);
    d.raw_off = raw ? s.raw_off.as<int64_t>() : nullptr;
    d.raw_mem = raw ? s.raw_mem.as<int32_t>() : nullptr;
    d.raw_host = s.raw_host;
    d.raw_split = s.raw_split;
    d.implicit = s.implicit_roots && s.enc != HBM_ENC_BITMAX;
    d.seed = s.seed;
    d.n = (uint32_t)c.g.n;
    d.hot_rank = s.nhot ? s.hot_rank.as<int32_t>() : nullptr;
    d.nar = s.nsets ? s.nar : 0;
    d.ar_hot = s.ar_hot.as<int32_t>();
    d.ar_rank = s.ar_rank.as<int32_t>();
    d.ar_off = s.ar_off.as<int64_t>();
    d.ar_low = s.ar_low.as<uint16_t>();
    d.bitoff = huff ? s.bitoff.as<int64_t>() : nullptr;
    d.payload = s.payload.as<uint32_t>();
    d.lim = s.cbtab.as<uint64_t>();
    d.base = s.cbtab.as<int64_t>() + 34;
    d.symtab = s.symtab.as<int32_t>();
    d.minlen = s.cb.minlen;
    d.wbits = s.cb.wbits;
    return d;
}

void store_reset(Ctx &c) {
    Store &s = c.s;
    s.enc = s.enc_req;  // AUTO decides again from the next warm-up block
    s.has_seed = false;
    s.nsets = 0;
    s.W = 0;
    s.wcur = 0;
    s.model_ready = false;
    s.members = 0;
    s.nhot = 0;
    s.nar = 0;
    s.ar_chunks = s.ar_entries = s.ar_last_start = 0;
    s.bm_words = 0;
    s.raw_count = 0;
    s.nbits = 0;
    s.escapes = 0;
    s.cb = Codebook{};
    s.skew = s.density = 0.0;
    s.warm_sizes.clear();
    if (s.hist.p) buf_zero(c, s.hist, 0, s.hist.bytes);
    if (s.bitmap.p) buf_zero(c, s.bitmap, 0, s.bitmap.bytes);
    if (s.payload.p) buf_zero(c, s.payload, 0, s.payload.bytes);
    if (s.raw_off.p) buf_zero(c, s.raw_off, 0, 8);
    if (s.bitoff.p) buf_zero(c, s.bitoff, 0, 8);
}

void store_free(Ctx &c) {
    Store &s = c.s;
    raw_host_free(c);
    for (Buf *b : {&s.hist, &s.warm, &s.hot, &s.hot_rank, &s.bitmap, &s.raw_off, &s.raw_mem, &s.lens, &s.codes,
                   &s.symtab, &s.cbtab, &s.lut, &s.bitoff, &s.payload, &s.ckb, &s.mtmp, &s.ar_hot, &s.ar_rank, &s.enc8,
                   &s.ar_off, &s.ar_low, &s.ar_tmp, &s.ar_keys, &s.ar_sort})
        buf_free(c, *b);
    Scratch &sc = c.sc;
    for (Buf *b : {&sc.mem, &sc.pos, &sc.size, &sc.ctrl, &sc.defer, &sc.t2_bitmap, &sc.t2_queue, &sc.t2h_bitmap,
                   &sc.t2h_queue, &sc.aux, &sc.cnt})
        buf_free(c, *b);
    sc.cap = 0;
    sc.bcap = 0;
    sc.t2_slots = 0;
    sc.t2h_slots = 0;
}

int64_t store_bytes(const Ctx &c) {
    const Store &s = c.s;
    int64_t b = 0;
    if (enc_huff(s.enc)) b += (s.nsets + 1) * 8 + (int64_t)((s.nbits + 7) / 8) + (int64_t)(s.nbits / CK_SLOT + 1);
    else if (enc_raw(s.enc)) b += (s.nsets + 1) * 8 + s.raw_count * 4;
    b += s.bm_words * (int64_t)s.nhot * 8;
    b += s.ar_chunks * (int64_t)(s.nar + 1) * 8 + s.ar_entries * 2;
    return b;
}

void ensure_scratch(Ctx &c, size_t entries, int64_t bcap) {
    Scratch &sc = c.sc;
    if (entries > sc.cap) {
        buf_alloc(c, sc.mem, entries * 4);
        sc.cap = entries;
    }
    if (bcap > sc.bcap) {
        buf_alloc(c, sc.pos, (size_t)bcap * 4);
        buf_alloc(c, sc.size, (size_t)(bcap + 1) * 4);
        buf_alloc(c, sc.defer, (size_t)bcap * 3 * 4);
        buf_alloc(c, sc.aux, (size_t)(bcap + 1) * 8);
        buf_alloc(c, sc.cnt, (size_t)(bcap + 1) * 4);
        sc.bcap = bcap;
    }
    if (!sc.ctrl.p) buf_alloc(c, sc.ctrl, CW_COUNT * 8);
}

// ---------------------------------------------------------------- host codebook (Huffman lengths, canonical codes)
// Code lengths: two queues; leaves ordered by (weight, id); on equal weight the
// leaf is taken before an internal node.  Longest code 32 bits: otherwise every
// weight w becomes ceil(w/2) and the lengths are recomputed.
static int huffman_lengths_host(const std::vector<std::pair<uint64_t, int32_t>> &syms, std::vector<uint8_t> &len_out) {
    const size_t L = syms.size();
    len_out.assign(L, 0);
    if (L == 0) return 0;
    if (L == 1) {
        len_out[0] = 1;
        return 1;
    }
    std::vector<uint64_t> w(L);
    for (size_t i = 0; i < L; i++) w[i] = syms[i].first;
    std::vector<size_t> order(L);
    std::vector<uint64_t> wt(2 * L - 1);
    std::vector<int64_t> up(2 * L - 1);
    std::vector<int32_t> depth(2 * L - 1);
    for (;;) {
        // (weight, id) order: syms come in ascending id order, so a stable sort by weight gives it;
        // warm-up counts are small integers, so a counting sort does it in linear time
        const uint64_t mx = *std::max_element(w.begin(), w.end());
        if (mx <= (uint64_t)std::max<size_t>(4 * L, size_t(1) << 16)) {
            std::vector<size_t> start((size_t)mx + 2, 0);
            for (size_t i = 0; i < L; i++) start[(size_t)w[i] + 1]++;
            for (size_t x = 1; x < start.size(); x++) start[x] += start[x - 1];
            for (size_t i = 0; i < L; i++) order[start[(size_t)w[i]]++] = i;
        } else {
            std::iota(order.begin(), order.end(), 0);
            std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return w[a] < w[b]; });
        }
        for (size_t i = 0; i < L; i++) wt[i] = w[order[i]];
        size_t leaf = 0, inner = L, made = L;
        auto take = [&]() -> size_t {
            if (leaf < L && (inner >= made || wt[leaf] <= wt[inner])) return leaf++;
            return inner++;
        };
        while (made < 2 * L - 1) {
            const size_t a = take();
            const size_t b = take();
            wt[made] = wt[a] + wt[b];
            up[a] = (int64_t)made;
            up[b] = (int64_t)made;
            made++;
        }
        depth[2 * L - 2] = 0;
        int maxd = 0;
        for (int64_t x = (int64_t)(2 * L) - 3; x >= 0; x--) depth[x] = depth[up[x]] + 1;
        for (size_t i = 0; i < L; i++) maxd = std::max(maxd, depth[i]);
        if (maxd <= 32) {
            for (size_t i = 0; i < L; i++) len_out[order[i]] = (uint8_t)depth[i];
            return maxd;
        }
        for (auto &x : w) x = (x + 1) / 2;
    }
}

// ---------------------------------------------------------------- warm-up symbols on the device
// The ids with a nonzero warm-up count, ascending, with their counts: every block of NZ_SPAN
// vertices counts its nonzero ones, the counts are scanned, and each block writes its ids in
// order from its offset.  Only this list (at most the warm-up's member count) goes to the
// host; the per-vertex tables are filled on the device from compact lists.
constexpr int NZ_T = 256, NZ_ITEMS = 16, NZ_SPAN = NZ_T * NZ_ITEMS;

__global__ __launch_bounds__(NZ_T) void k_nz_count(const uint32_t *warm, int32_t n, uint32_t *bcnt) {
    __shared__ uint32_t ws[NZ_T / WAVE];
    const int64_t base = (int64_t)blockIdx.x * NZ_SPAN;
    uint32_t c = 0;
    for (int i = 0; i < NZ_ITEMS; i++) {
        const int64_t v = base + (int64_t)i * NZ_T + threadIdx.x;
        if (v < n && warm[v]) c++;
    }
    c = wave_sum(c);
    if (lane_id() == 0) ws[threadIdx.x / WAVE] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < NZ_T / WAVE; w++) t += ws[w];
        bcnt[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(NZ_T) void k_nz_write(const uint32_t *warm, int32_t n, const int64_t *boff, uint32_t *ids,
                                                   uint32_t *cnt) {
    __shared__ uint32_t ws[NZ_T / WAVE];
    const int64_t base = (int64_t)blockIdx.x * NZ_SPAN;
    const int wv = threadIdx.x / WAVE;
    int64_t at = boff[blockIdx.x];
    for (int i = 0; i < NZ_ITEMS; i++) {
        const int64_t v = base + (int64_t)i * NZ_T + threadIdx.x;
        const uint32_t w = v < n ? warm[v] : 0u;
        const uint32_t f = w ? 1u : 0u;
        const uint32_t inc = wave_incl_scan(f);
        if (lane_id() == WAVE - 1) ws[wv] = inc;
        __syncthreads();
        uint32_t before = 0, tot = 0;
        for (int x = 0; x < NZ_T / WAVE; x++) {
            if (x < wv) before += ws[x];
            tot += ws[x];
        }
        if (f) {
            const int64_t p = at + before + inc - 1;
            ids[p] = (uint32_t)v;
            cnt[p] = w;
        }
        at += tot;
        __syncthreads();
    }
}

// p[i] = i for i < count (the all-vertex row list and rank of a BITMAX store)
__global__ void k_iota_i32(int32_t *p, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = (int32_t)i;
}

__global__ void k_fill_i32(int32_t *p, int64_t count, int32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// rank[ids[r]] = r (hot ranks)
__global__ void k_scatter_rank(const uint32_t *ids, int64_t k, int32_t *rank) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < k; r += (int64_t)gridDim.x * blockDim.x)
        rank[ids[r]] = (int32_t)r;
}

// lens[ids[i]] = len[i], codes[ids[i]] = code[i] (coded vertices)
// The encoders' packed table: code | length << 32 | (v has a bitmap or array row) << 40.
__global__ void k_pack_codes(const uint8_t *lens, const uint32_t *codes, const int32_t *hot_rank,
                             const int32_t *ar_rank, int64_t n, unsigned long long *enc8) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const bool row = (hot_rank && hot_rank[v] >= 0) || (ar_rank && ar_rank[v] >= 0);
        enc8[v] = (unsigned long long)codes[v] | ((unsigned long long)lens[v] << 32) | ((unsigned long long)row << 40);
    }
}

__global__ void k_scatter_codes(const uint32_t *ids, const uint8_t *len, const uint32_t *code, int64_t m,
                                uint8_t *lens, uint32_t *codes) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        lens[ids[i]] = len[i];
        codes[ids[i]] = code[i];
    }
}

// Vertices with a nonzero warm-up count, ascending, and their counts (device work; host copy
// of the compact list).
static void warm_symbols(Ctx &c, std::vector<uint32_t> &ids, std::vector<uint32_t> &cnt) {
    Store &s = c.s;
    const int32_t n = c.g.n;
    const hipStream_t st = c.stream;
    const int64_t nblk = ((int64_t)n + NZ_SPAN - 1) / NZ_SPAN;
    const size_t off_at = ((size_t)(nblk + 1) * 4 + 255) & ~size_t(255);
    buf_grow(c, s.mtmp, off_at + (size_t)(nblk + 1) * 8, false);
    uint32_t *bcnt = s.mtmp.as<uint32_t>();
    int64_t *boff = reinterpret_cast<int64_t *>(s.mtmp.as<char>() + off_at);
    buf_zero(c, s.mtmp, (size_t)nblk * 4, 4);  // the scan's last input (its output is the total)
    k_nz_count<<<(unsigned)nblk, NZ_T, 0, st>>>(s.warm.as<uint32_t>(), n, bcnt);
    HBM_HIP(hipGetLastError());
    scan_u32_to_i64(c, bcnt, boff, nblk + 1, 0);
    int64_t m = 0;
    HBM_HIP(hipMemcpyAsync(&m, boff + nblk, 8, hipMemcpyDeviceToHost, st));
    HBM_HIP(hipStreamSynchronize(st));
    ids.assign((size_t)m, 0);
    cnt.assign((size_t)m, 0);
    if (m == 0) return;
    const size_t ids_at = ((off_at + (size_t)(nblk + 1) * 8) + 255) & ~size_t(255);
    const size_t cnt_at = (ids_at + (size_t)m * 4 + 255) & ~size_t(255);
    buf_grow(c, s.mtmp, cnt_at + (size_t)m * 4, true);
    boff = reinterpret_cast<int64_t *>(s.mtmp.as<char>() + off_at);
    uint32_t *dids = reinterpret_cast<uint32_t *>(s.mtmp.as<char>() + ids_at);
    uint32_t *dcnt = reinterpret_cast<uint32_t *>(s.mtmp.as<char>() + cnt_at);
    k_nz_write<<<(unsigned)nblk, NZ_T, 0, st>>>(s.warm.as<uint32_t>(), n, boff, dids, dcnt);
    HBM_HIP(hipGetLastError());
    HBM_HIP(hipMemcpyAsync(ids.data(), dids, (size_t)m * 4, hipMemcpyDeviceToHost, st));
    HBM_HIP(hipMemcpyAsync(cnt.data(), dcnt, (size_t)m * 4, hipMemcpyDeviceToHost, st));
    HBM_HIP(hipStreamSynchronize(st));
}

static unsigned fill_grid(int64_t count) { return grid_for(count, 256, 8192); }

static void build_model(Ctx &c) {
    Store &s = c.s;
    const int32_t n = c.g.n;
    const hipStream_t st = c.stream;
    if (s.enc == HBM_ENC_AUTO)  // Alg. 1's branch on the warm-up block's Eq. 2 figures
        s.enc = (s.skew < 0.0 && s.density > 1.0 / 32.0) ? HBM_ENC_BITMAX : HBM_ENC_HUFFMAN;
    if (s.enc == HBM_ENC_BITMAX) {
        // the Bitmax encoding section's n-row bit matrix: vertex v owns row v
        s.nhot = n;
        buf_alloc(c, s.hot, (size_t)n * 4);
        buf_grow(c, s.hot_rank, (size_t)n * 4, false);
        k_iota_i32<<<fill_grid(n), 256, 0, st>>>(s.hot.as<int32_t>(), n);
        k_iota_i32<<<fill_grid(n), 256, 0, st>>>(s.hot_rank.as<int32_t>(), n);
        HBM_HIP(hipGetLastError());
        s.model_ready = true;
        return;
    }
    // the warm-up's symbols in ascending id order: every choice below is a total order
    // over (count, id), so it matches a scan over all n vertices
    std::vector<uint32_t> ids, wcnt;
    warm_symbols(c, ids, wcnt);
    const size_t m = ids.size();
    const bool hot = s.enc == HBM_ENC_HOT_BITMAP || s.enc == HBM_ENC_HUFFMAN_HOT_BITMAP;
    const bool huff = s.enc == HBM_ENC_HUFFMAN || s.enc == HBM_ENC_HUFFMAN_HOT_BITMAP;
    std::vector<char> is_hot(m, 0);
    s.nhot = 0;
    if (hot) {
        // eligible: in at least max(1, ceil(min_density * W)) warm-up sets (a bitmap row costs a
        // bit per set, a stored id 32 bits per occurrence: rows pay above density 1/32)
        const uint64_t min_cnt = std::max<uint64_t>(1, (uint64_t)std::ceil(s.hot_min_density * (double)s.W));
        std::vector<size_t> seen;  // indices into ids
        for (size_t i = 0; i < m; i++)
            if ((uint64_t)wcnt[i] >= min_cnt) seen.push_back(i);
        const int64_t want = (int64_t)std::ceil(s.hot_frac * (double)n);
        const size_t keep = (size_t)std::min<int64_t>(want, (int64_t)seen.size());
        std::partial_sort(seen.begin(), seen.begin() + keep, seen.end(), [&](size_t a, size_t b) {
            return wcnt[a] != wcnt[b] ? wcnt[a] > wcnt[b] : ids[a] < ids[b];
        });
        // with containers, a hot vertex below warm-up density 1/16 gets an array row (16 bits
        // per occurrence beats a bit per set there), the others bitmap rows; hot order is kept
        std::vector<uint32_t> hot_ids, ar_ids;
        for (size_t r = 0; r < keep; r++) {
            const bool arr = s.containers && (uint64_t)16 * wcnt[seen[r]] < (uint64_t)s.W;
            (arr ? ar_ids : hot_ids).push_back(ids[seen[r]]);
            is_hot[seen[r]] = 1;
        }
        s.nhot = (int32_t)hot_ids.size();
        s.nar = (int32_t)ar_ids.size();
        hot_ids.resize(std::max<size_t>(hot_ids.size(), 1), 0u);
        buf_alloc(c, s.hot, hot_ids.size() * 4);
        buf_grow(c, s.hot_rank, (size_t)n * 4, false);
        HBM_HIP(hipMemcpyAsync(s.hot.p, hot_ids.data(), hot_ids.size() * 4, hipMemcpyHostToDevice, st));
        k_fill_i32<<<fill_grid(n), 256, 0, st>>>(s.hot_rank.as<int32_t>(), n, -1);
        if (s.nhot) k_scatter_rank<<<fill_grid((int64_t)s.nhot), 256, 0, st>>>(s.hot.as<uint32_t>(), (int64_t)s.nhot,
                                                                            s.hot_rank.as<int32_t>());
        if (s.nar) {
            buf_alloc(c, s.ar_hot, ar_ids.size() * 4);
            buf_grow(c, s.ar_rank, (size_t)n * 4, false);
            HBM_HIP(hipMemcpyAsync(s.ar_hot.p, ar_ids.data(), ar_ids.size() * 4, hipMemcpyHostToDevice, st));
            k_fill_i32<<<fill_grid(n), 256, 0, st>>>(s.ar_rank.as<int32_t>(), n, -1);
            k_scatter_rank<<<fill_grid((int64_t)s.nar), 256, 0, st>>>(s.ar_hot.as<uint32_t>(), (int64_t)s.nar,
                                                                      s.ar_rank.as<int32_t>());
        }
        HBM_HIP(hipGetLastError());
        // the host vector is freed at return: the queued copy must have read it
        HBM_HIP(hipStreamSynchronize(st));
    }
    if (huff) {
        std::vector<std::pair<uint64_t, int32_t>> syms;
        for (size_t i = 0; i < m; i++)
            if (!is_hot[i]) syms.push_back({wcnt[i], (int32_t)ids[i]});
        std::vector<uint8_t> L;
        auto L_of = [&](size_t i) { return (int)L[i]; };
        Codebook &cb = s.cb;
        cb.maxlen = huffman_lengths_host(syms, L);
        cb.nsym = (int32_t)syms.size();
        cb.wbits = n > 1 ? 32 - __builtin_clz((uint32_t)(n - 1)) : 1;
        cb.ustar_enc = -1;
        uint64_t best = 0;
        for (auto &p : syms)
            if (p.first > best) { best = p.first; cb.ustar_enc = p.second; }
        // canonical assignment by (length, id)
        // (length, id) order: a stable bucket pass by length over the ascending ids
        std::vector<size_t> ord(syms.size());
        {
            size_t start[34] = {};
            for (size_t i = 0; i < syms.size(); i++) start[L[i] + 1]++;
            for (int x = 1; x < 34; x++) start[x] += start[x - 1];
            for (size_t i = 0; i < syms.size(); i++) ord[start[L[i]]++] = i;
        }
        std::vector<uint32_t> sym_code(syms.size(), 0), sym_id(std::max<size_t>(syms.size(), 1), 0);
        std::vector<int32_t> symtab(std::max<size_t>(syms.size(), 1), 0);
        uint64_t count[34] = {}, first[34] = {}, firstidx[34] = {};
        for (size_t i = 0; i < syms.size(); i++) count[L[i]]++;
        uint64_t code = 0;
        for (size_t q = 0; q < ord.size(); q++) {
            const size_t i = ord[q];
            if (q > 0) code = (code + 1) << (L[i] - L[ord[q - 1]]);
            sym_code[i] = (uint32_t)code;
            symtab[q] = syms[i].second;
        }
        for (size_t i = 0; i < syms.size(); i++) sym_id[i] = (uint32_t)syms[i].second;
        cb.minlen = 33;
        for (int l = 1; l <= 32; l++)
            if (count[l]) { cb.minlen = std::min(cb.minlen, l); }
        if (cb.minlen == 33) cb.minlen = 1;
        // first code and first symbol index of every length
        uint64_t fc = 0, fi = 0;
        for (int l = 1; l <= 33; l++) {
            first[l] = fc;
            firstidx[l] = fi;
            fc = (fc + (l <= 32 ? count[l] : 0)) << 1;
            fi += l <= 32 ? count[l] : 0;
        }
        uint64_t tab_lim[34] = {};
        int64_t tab_base[34] = {};
        for (int l = 1; l <= 32; l++) {
            cb.lim[l] = (first[l] + count[l]) << (32 - l);
            cb.base[l] = (int32_t)0;
            tab_lim[l] = cb.lim[l];
            tab_base[l] = (int64_t)firstidx[l] - (int64_t)first[l];
        }
        tab_lim[33] = ~0ull;  // sentinel: never decoded past the longest code
        // direct lookup for codes of at most LUT_BITS bits: every LUT_BITS-bit prefix that starts
        // with such a code maps to (symbol << 5) | length.  Any other prefix maps to Lmin << 5
        // (length field 0): the shortest length of a code starting with it, i.e. the first L
        // whose limit exceeds the prefix, so a decoder searches the limits from there.
        std::vector<uint32_t> lut((size_t)1 << LUT_BITS, 0u);
        for (size_t q = 0; q < ord.size(); q++) {
            const size_t i = ord[q];
            const int L = L_of(i);
            if (L > LUT_BITS) break;
            const uint32_t cd = sym_code[i];
            const uint32_t lo = cd << (LUT_BITS - L), hi = (cd + 1) << (LUT_BITS - L);
            for (uint32_t x = lo; x < hi; x++) lut[x] = ((uint32_t)syms[i].second << 5) | (uint32_t)L;
        }
        for (uint32_t t = 0; t < (1u << LUT_BITS); t++) {
            if (lut[t]) continue;
            int L = LUT_BITS + 1;
            while (L < 33 && tab_lim[L] <= ((uint64_t)t << (32 - LUT_BITS))) L++;
            lut[t] = (uint32_t)L << 5;
        }
        // per-vertex tables: zero, then the coded vertices scattered from compact lists
        const size_t ms = syms.size();
        buf_grow(c, s.lens, (size_t)n, false);
        buf_grow(c, s.codes, (size_t)n * 4, false);
        buf_zero(c, s.lens, 0, (size_t)n);
        buf_zero(c, s.codes, 0, (size_t)n * 4);
        const size_t len_at = (ms * 4 + 255) & ~size_t(255), code_at = (len_at + ms + 255) & ~size_t(255);
        buf_grow(c, s.mtmp, code_at + ms * 4 + 4, false);
        char *tb = s.mtmp.as<char>();
        if (ms) {
            HBM_HIP(hipMemcpyAsync(tb, sym_id.data(), ms * 4, hipMemcpyHostToDevice, st));
            HBM_HIP(hipMemcpyAsync(tb + len_at, L.data(), ms, hipMemcpyHostToDevice, st));
            HBM_HIP(hipMemcpyAsync(tb + code_at, sym_code.data(), ms * 4, hipMemcpyHostToDevice, st));
            k_scatter_codes<<<fill_grid((int64_t)ms), 256, 0, st>>>(
                reinterpret_cast<const uint32_t *>(tb), reinterpret_cast<const uint8_t *>(tb + len_at),
                reinterpret_cast<const uint32_t *>(tb + code_at), (int64_t)ms, s.lens.as<uint8_t>(), s.codes.as<uint32_t>());
            HBM_HIP(hipGetLastError());
        }
        buf_alloc(c, s.symtab, symtab.size() * 4);
        buf_alloc(c, s.cbtab, 68 * 8);
        buf_alloc(c, s.lut, lut.size() * 4);
        HBM_HIP(hipMemcpyAsync(s.lut.p, lut.data(), lut.size() * 4, hipMemcpyHostToDevice, st));
        HBM_HIP(hipMemcpyAsync(s.symtab.p, symtab.data(), symtab.size() * 4, hipMemcpyHostToDevice, st));
        HBM_HIP(hipMemcpyAsync(s.cbtab.p, tab_lim, 34 * 8, hipMemcpyHostToDevice, st));
        HBM_HIP(hipMemcpyAsync(s.cbtab.as<int64_t>() + 34, tab_base, 34 * 8, hipMemcpyHostToDevice, st));
        buf_grow(c, s.enc8, (size_t)n * 8, false);
        k_pack_codes<<<fill_grid(n), 256, 0, st>>>(s.lens.as<uint8_t>(), s.codes.as<uint32_t>(),
                                                   hot ? s.hot_rank.as<int32_t>() : nullptr,
                                                   s.nar ? s.ar_rank.as<int32_t>() : nullptr, n,
                                                   s.enc8.as<unsigned long long>());
        HBM_HIP(hipGetLastError());
        HBM_HIP(hipStreamSynchronize(st));
    }
    s.model_ready = true;
}

// Eq. 2 over the warm-up block sizes (diagnostic)
static void characterize(Store &s, int32_t n) {
    const auto &X = s.warm_sizes;
    if (X.empty()) return;
    double t = (double)X.size(), mean = 0.0;
    for (uint32_t x : X) mean += x;
    mean /= t;
    double m2 = 0.0, m3 = 0.0, sum = 0.0;
    for (uint32_t x : X) {
        const double d = x - mean;
        m2 += d * d;
        m3 += d * d * d;
        sum += x;
    }
    m2 /= t;
    m3 /= t;
    const double sd = std::sqrt(m2);
    s.skew = sd > 0 ? m3 / (sd * sd * sd) : 0.0;
    s.density = sum / (t * (double)n);
}

static void record_warm_sizes(Ctx &c, int64_t j0, int64_t done) {
    Store &s = c.s;
    if (j0 >= s.W) return;
    const int64_t cnt = std::min(done, s.W - j0);
    const size_t at = s.warm_sizes.size();
    s.warm_sizes.resize(at + (size_t)cnt);
    HBM_HIP(hipMemcpyAsync(s.warm_sizes.data() + at, c.sc.size.p, (size_t)cnt * 4, hipMemcpyDeviceToHost, c.stream));
    HBM_HIP(hipStreamSynchronize(c.stream));
}

template <class T>
static T read_dev(Ctx &c, const void *p) {
    T v;
    HBM_HIP(hipMemcpyAsync(&v, p, sizeof(T), hipMemcpyDeviceToHost, c.stream));
    HBM_HIP(hipStreamSynchronize(c.stream));
    return v;
}

static BlockView block_view(Ctx &c, int64_t done) {
    return BlockView{c.sc.mem.as<uint32_t>(), c.sc.pos.as<uint32_t>(), c.sc.size.as<uint32_t>(), done};
}

// Per job, the int64 at src[i] gathered into root.tails and copied to the host.
static void gather_tails(Ctx &root, const std::vector<const int64_t *> &src, std::vector<int64_t> &out) {
    const size_t N = src.size();
    out.assign(N, 0);
    if (!N) return;
    buf_grow(root, root.tails, N * 8, false);
    std::vector<TailArgs> ta(N);
    std::vector<uint32_t> nb(N, 1);
    for (size_t i = 0; i < N; i++) ta[i] = TailArgs{src[i], root.tails.as<int64_t>() + i};
    const hipStream_t st = root.stream;
    glaunch(root, ta, nb, 0, [&](const TailArgs &a, unsigned g) { k_tail<<<g, 64, 0, st>>>(a, 0); },
            [&](const TailArgs *d, const uint32_t *b, uint32_t cnt, uint32_t g, int x) {
                k_tail_g<<<g, 64, 0, st>>>(GroupArgs<TailArgs>{d, b, cnt, x});
            });
    HBM_HIP(hipGetLastError());
    HBM_HIP(hipMemcpyAsync(out.data(), root.tails.p, N * 8, hipMemcpyDeviceToHost, st));
    HBM_HIP(hipStreamSynchronize(st));
}

#define HBM_GLAUNCH(ROOT, ARGS, NB, X, KERNEL, THREADS, ATYPE)                                                 \
    glaunch(ROOT, ARGS, NB, X, [&](const ATYPE &a_, unsigned g_) { KERNEL<<<g_, THREADS, 0, (ROOT).stream>>>(a_, X); }, \
            [&](const ATYPE *d_, const uint32_t *b_, uint32_t c_, uint32_t g_, int x_) {                     \
                KERNEL##_g<<<g_, THREADS, 0, (ROOT).stream>>>(GroupArgs<ATYPE>{d_, b_, c_, x_});              \
            })

// Room for `total` plain ids: on the device, or with a spill cap the first raw_split ids on the
// device and the rest in pinned host memory (grown by copying once the stream is idle).
static void raw_grow(Ctx &c, int64_t total) {
    Store &s = c.s;
    if (s.spill_cap <= 0) {
        s.raw_split = INT64_MAX;
        buf_grow(c, s.raw_mem, (size_t)std::max<int64_t>(total, 1) * 4, true);
        return;
    }
    s.raw_split = (s.spill_cap / 16) * 4;
    buf_grow(c, s.raw_mem, (size_t)std::max<int64_t>(std::min(total, s.raw_split), 4) * 4, true);
    const int64_t nh = total - s.raw_split;
    if (nh <= 0 || (size_t)nh <= s.raw_host_cap) return;
    size_t cap = std::max<size_t>(s.raw_host_cap * 2, size_t(1) << 20);
    while (cap < (size_t)nh) cap *= 2;
    void *p = nullptr;
    HBM_HIP(hipHostMalloc(&p, cap * 4, hipHostMallocMapped | hipHostMallocCoherent));
    HBM_HIP(hipStreamSynchronize(c.stream));  // earlier blocks' ids are written
    if (s.raw_host_h) {
        const int64_t have = std::max<int64_t>(0, s.raw_count - s.raw_split);
        std::memcpy(p, s.raw_host_h, (size_t)have * 4);
        (void)hipHostFree(s.raw_host_h);
        s.raw_host = s.raw_host_h = nullptr;
        s.raw_host_cap = 0;
    }
    void *dp = nullptr;
    const hipError_t e = hipHostGetDevicePointer(&dp, p, 0);
    if (e != hipSuccess) {
        (void)hipHostFree(p);
        throw Error{HBM_EDEVICE, std::string("hipHostGetDevicePointer: ") + hipGetErrorString(e)};
    }
    s.raw_host_h = (int32_t *)p;
    s.raw_host = (int32_t *)dp;
    s.raw_host_cap = cap;
}

void raw_host_free(Ctx &c) {
    Store &s = c.s;
    if (!s.raw_host_h) return;
    (void)hipStreamSynchronize(c.stream);
    (void)hipHostFree(s.raw_host_h);
    s.raw_host = s.raw_host_h = nullptr;
    s.raw_host_cap = 0;
}

// ------------------------------------------------------------------ array containers
// A block's sets that fall in chunk ch (block-relative [b0, b1)) add, for every array row, the
// 16-bit offsets of the sets that hold the row's vertex.  Sets arrive in ascending order, so only
// the last chunk ever grows: it is rebuilt with each row's old entries followed by the new
// ones, then every row's list is sorted (the new entries are written in arbitrary order).
constexpr int AR_CHUNK_BITS = 16;
struct ArrArgs {
    BlockView bv;
    uint64_t b0, b1;             // block-relative sets, all in one chunk
    int64_t j0;                  // set index of the block's first set
    int64_t cbase;               // first set of the chunk
    const int32_t *ar_rank;
    uint32_t *cnt;               // count pass: new entries per row
    unsigned long long *cursor;  // write pass: next position per row
    uint16_t *low;
};

__global__ __launch_bounds__(256) void k_arr_count(ArrArgs A) {
    const uint64_t wave = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) / WAVE;
    const uint64_t nw = (uint64_t)gridDim.x * blockDim.x / WAVE;
    const unsigned lane = lane_id();
    for (uint64_t b = A.b0 + wave; b < A.b1; b += nw) {
        const uint32_t p = A.bv.pos[b], s = A.bv.size[b];
        for (uint32_t i = lane; i < s; i += WAVE) {
            const int32_t a = A.ar_rank[A.bv.mem[p + i]];
            if (a >= 0) atomicAdd(&A.cnt[a], 1u);
        }
    }
}

__global__ __launch_bounds__(256) void k_arr_write(ArrArgs A) {
    const uint64_t wave = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) / WAVE;
    const uint64_t nw = (uint64_t)gridDim.x * blockDim.x / WAVE;
    const unsigned lane = lane_id();
    for (uint64_t b = A.b0 + wave; b < A.b1; b += nw) {
        const uint32_t p = A.bv.pos[b], s = A.bv.size[b];
        const uint16_t low = (uint16_t)((uint64_t)A.j0 + b - (uint64_t)A.cbase);
        for (uint32_t i = lane; i < s; i += WAVE) {
            const int32_t a = A.ar_rank[A.bv.mem[p + i]];
            if (a >= 0) A.low[atomicAdd(&A.cursor[a], 1ull)] = low;
        }
    }
}

// per row: total = old + new entries (tot[nar] = 0 closes the scan)
__global__ void k_arr_tot(const int64_t *old_off, const uint32_t *cnt, uint32_t *tot, int32_t nar) {
    for (int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; a <= nar; a += (int64_t)gridDim.x * blockDim.x)
        tot[a] = a < nar ? cnt[a] + (old_off ? (uint32_t)(old_off[a + 1] - old_off[a]) : 0u) : 0u;
}

// per row: its old entries (in `keys`, chunk-relative) moved to their new place, the write cursor
// after them, and the chunk-relative segment start for the sort
__global__ void k_arr_move(const int64_t *old_off, const int64_t *new_off, int64_t start, const uint16_t *keys,
                           uint16_t *low, unsigned long long *cursor, uint32_t *rel, int32_t nar) {
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / WAVE;
    const int64_t nw = (int64_t)gridDim.x * blockDim.x / WAVE;
    const unsigned lane = lane_id();
    for (int64_t a = wave; a <= nar; a += nw) {
        if (lane == 0) rel[a] = (uint32_t)(new_off[a] - start);
        if (a == nar) continue;
        const int64_t oc = old_off ? old_off[a + 1] - old_off[a] : 0;
        for (int64_t i = lane; i < oc; i += WAVE) low[new_off[a] + i] = keys[old_off[a] - start + i];
        if (lane == 0) cursor[a] = (unsigned long long)(new_off[a] + oc);
    }
}

// One chunk's rebuild, planned before any store write: where its entries end and what it needs.
struct ArrPlan {
    int64_t ch, b0, b1, start, end;
    bool existed;
};

// Layout of ar_tmp: cnt u32[nar + 1] | tot u32[nar + 1] | rel u32[nar + 1] | new_off i64[nar + 1]
// | cursor u64[nar]
static size_t ar_tmp_at(int32_t nar, int part) {
    const size_t u = ((size_t)(nar + 1) * 4 + 255) & ~size_t(255), q = ((size_t)(nar + 1) * 8 + 255) & ~size_t(255);
    const size_t at[] = {0, u, 2 * u, 3 * u, 3 * u + q, 3 * u + 2 * q};
    return at[part];
}

// Counts and offsets of every chunk the block touches, then every allocation the rebuild needs
// (entries, chunk offsets, scratch, sort space): nothing of the store is written yet.
static void arr_plan(Ctx &c, int64_t j0, int64_t done, std::vector<ArrPlan> &plans) {
    Store &s = c.s;
    plans.clear();
    if (!s.nar || done <= 0) return;
    const int32_t nar = s.nar;
    const hipStream_t st = c.stream;
    buf_grow(c, s.ar_tmp, ar_tmp_at(nar, 5), false);
    uint32_t *cnt = (uint32_t *)(s.ar_tmp.as<char>() + ar_tmp_at(nar, 0));
    uint32_t *tot = (uint32_t *)(s.ar_tmp.as<char>() + ar_tmp_at(nar, 1));
    int64_t *noff = (int64_t *)(s.ar_tmp.as<char>() + ar_tmp_at(nar, 3));
    int64_t entries = s.ar_entries, chunks = s.ar_chunks, last_start = s.ar_last_start;
    const int64_t j1 = j0 + done;
    for (int64_t ch = j0 >> AR_CHUNK_BITS; ch <= (j1 - 1) >> AR_CHUNK_BITS; ch++) {
        ArrPlan p;
        p.ch = ch;
        p.b0 = std::max<int64_t>(j0, ch << AR_CHUNK_BITS) - j0;
        p.b1 = std::min<int64_t>(j1, (ch + 1) << AR_CHUNK_BITS) - j0;
        p.existed = ch < chunks;
        p.start = p.existed ? last_start : entries;
        buf_zero(c, s.ar_tmp, ar_tmp_at(nar, 0), (size_t)(nar + 1) * 4);
        ArrArgs A{};
        A.bv = block_view(c, done);
        A.b0 = (uint64_t)p.b0;
        A.b1 = (uint64_t)p.b1;
        A.ar_rank = s.ar_rank.as<int32_t>();
        A.cnt = cnt;
        k_arr_count<<<grid_for((p.b1 - p.b0) * WAVE, 256, 65536), 256, 0, st>>>(A);
        const int64_t *old_off = p.existed ? s.ar_off.as<int64_t>() + ch * (int64_t)(nar + 1) : nullptr;
        k_arr_tot<<<grid_for(nar + 1, 256, 1024), 256, 0, st>>>(old_off, cnt, tot, nar);
        HBM_HIP(hipGetLastError());
        scan_u32_to_i64(c, tot, noff, nar + 1, p.start);
        HBM_HIP(hipMemcpyAsync(&p.end, noff + nar, 8, hipMemcpyDeviceToHost, st));
        HBM_HIP(hipStreamSynchronize(st));
        plans.push_back(p);
        entries = p.end;
        last_start = p.start;
        chunks = ch + 1;
    }
    // every allocation of the rebuild
    int64_t span = 0;
    for (const ArrPlan &p : plans) span = std::max(span, p.end - p.start);
    buf_grow(c, s.ar_low, (size_t)std::max<int64_t>(entries, 1) * 2 + 64, true);
    buf_grow(c, s.ar_off, (size_t)chunks * (size_t)(nar + 1) * 8, true);
    buf_grow(c, s.ar_keys, (size_t)std::max<int64_t>(span, 1) * 2 + 64, false);
    size_t sort_bytes = 0;
    HBM_HIP(rocprim::segmented_radix_sort_keys(nullptr, sort_bytes, (const uint16_t *)nullptr, (uint16_t *)nullptr,
                                               (unsigned int)std::max<int64_t>(span, 1), (unsigned int)nar,
                                               (const uint32_t *)nullptr, (const uint32_t *)nullptr, 0, 16, st));
    buf_grow(c, s.ar_sort, std::max<size_t>(sort_bytes, 256), false);
}

// The rebuild of each planned chunk (no allocation): old entries moved behind their new offsets,
// new entries written, every row's list sorted, offsets stored.
static void arr_write(Ctx &c, int64_t j0, int64_t done, const std::vector<ArrPlan> &plans) {
    Store &s = c.s;
    const int32_t nar = s.nar;
    const hipStream_t st = c.stream;
    uint32_t *cnt = (uint32_t *)(s.ar_tmp.as<char>() + ar_tmp_at(nar, 0));
    uint32_t *tot = (uint32_t *)(s.ar_tmp.as<char>() + ar_tmp_at(nar, 1));
    uint32_t *rel = (uint32_t *)(s.ar_tmp.as<char>() + ar_tmp_at(nar, 2));
    int64_t *noff = (int64_t *)(s.ar_tmp.as<char>() + ar_tmp_at(nar, 3));
    unsigned long long *cursor = (unsigned long long *)(s.ar_tmp.as<char>() + ar_tmp_at(nar, 4));
    uint16_t *low = s.ar_low.as<uint16_t>();
    for (const ArrPlan &p : plans) {
        // offsets again (the plan's scratch was reused chunk by chunk)
        int64_t *old_off = p.existed ? s.ar_off.as<int64_t>() + p.ch * (int64_t)(nar + 1) : nullptr;
        buf_zero(c, s.ar_tmp, ar_tmp_at(nar, 0), (size_t)(nar + 1) * 4);
        ArrArgs A{};
        A.bv = block_view(c, done);
        A.b0 = (uint64_t)p.b0;
        A.b1 = (uint64_t)p.b1;
        A.j0 = j0;
        A.cbase = p.ch << AR_CHUNK_BITS;
        A.ar_rank = s.ar_rank.as<int32_t>();
        A.cnt = cnt;
        const unsigned g = grid_for((p.b1 - p.b0) * WAVE, 256, 65536);
        k_arr_count<<<g, 256, 0, st>>>(A);
        k_arr_tot<<<grid_for(nar + 1, 256, 1024), 256, 0, st>>>(old_off, cnt, tot, nar);
        HBM_HIP(hipGetLastError());
        scan_u32_to_i64(c, tot, noff, nar + 1, p.start);
        const int64_t old_end = p.existed ? s.ar_entries : p.start;
        if (old_end > p.start)
            HBM_HIP(hipMemcpyAsync(s.ar_keys.p, low + p.start, (size_t)(old_end - p.start) * 2,
                                   hipMemcpyDeviceToDevice, st));
        k_arr_move<<<grid_for((int64_t)(nar + 1) * WAVE, 256, 4096), 256, 0, st>>>(
            old_off, noff, p.start, s.ar_keys.as<uint16_t>(), low, cursor, rel, nar);
        A.cursor = cursor;
        A.low = low;
        k_arr_write<<<g, 256, 0, st>>>(A);
        HBM_HIP(hipGetLastError());
        const int64_t sz = p.end - p.start;
        if (sz > 0) {
            size_t sort_bytes = s.ar_sort.bytes;
            HBM_HIP(rocprim::segmented_radix_sort_keys(s.ar_sort.p, sort_bytes, low + p.start,
                                                       s.ar_keys.as<uint16_t>(), (unsigned int)sz, (unsigned int)nar,
                                                       rel, rel + 1, 0, 16, st));
            HBM_HIP(hipMemcpyAsync(low + p.start, s.ar_keys.p, (size_t)sz * 2, hipMemcpyDeviceToDevice, st));
        }
        HBM_HIP(hipMemcpyAsync(s.ar_off.as<int64_t>() + p.ch * (int64_t)(nar + 1), noff, (size_t)(nar + 1) * 8,
                               hipMemcpyDeviceToDevice, st));
        s.ar_entries = p.end;
        s.ar_last_start = p.start;
        s.ar_chunks = p.ch + 1;
    }
}

// Append sets [j0[i], j0[i] + done[i]) of every job from its scratch arena to its store
// (the job's encoding, then UpdateHistogram), one grouped launch per step.  Every allocation
// comes before the first write into the store and the histogram is updated last, so a failed
// allocation leaves each store as it was (nsets, histogram and encoded parts agree).
static void append_blocks(Ctx &root, const std::vector<Ctx *> &J, const std::vector<int64_t> &j0,
                          const std::vector<int64_t> &done) {
    const size_t N = J.size();
    // array rows: counts, offsets and every allocation before the first store write
    std::vector<std::vector<ArrPlan>> arr(N);
    for (size_t i = 0; i < N; i++) arr_plan(*J[i], j0[i], done[i], arr[i]);
    // plain-id jobs, Huffman jobs and all-vertex bitmap jobs
    std::vector<size_t> P, H, B;
    for (size_t i = 0; i < N; i++) {
        Store &s = J[i]->s;
        const int64_t new_sets = j0[i] + done[i];
        if (enc_rows(s.enc)) {
            const int64_t words = (new_sets + 63) / 64;
            buf_grow(*J[i], s.bitmap, (size_t)std::max<int64_t>(words * s.nhot, 1) * 8, true);
            s.bm_words = words;
        }
        if (enc_huff(s.enc)) H.push_back(i);
        else if (enc_raw(s.enc)) P.push_back(i);
        else B.push_back(i);
    }
    if (!B.empty()) {  // BITMAX: every member sets its bit in its own vertex's row
        std::vector<SplitArgs> sa;
        std::vector<uint32_t> sb;
        for (size_t i : B) {
            Store &s = J[i]->s;
            SplitArgs a{};
            a.bv = block_view(*J[i], done[i]);
            a.hot_rank = s.hot_rank.as<int32_t>();
            a.j0 = j0[i];
            a.bitmap = s.bitmap.as<unsigned long long>();
            a.nhot = s.nhot;
            sa.push_back(a);
            sb.push_back(grid_for(done[i] * WAVE, 256, 65536));
        }
        const int ps = prof_begin(root, "split");
        HBM_GLAUNCH(root, sa, sb, 0, k_split, 256, SplitArgs);
        prof_end(root, ps);
        HBM_HIP(hipGetLastError());
    }
    if (!P.empty()) {
        std::vector<SplitArgs> sa;
        std::vector<uint32_t> sb;
        for (size_t i : P) {
            Ctx &c = *J[i];
            Store &s = c.s;
            const bool hot = s.enc == HBM_ENC_HOT_BITMAP;
            buf_grow(c, s.raw_off, (size_t)(j0[i] + done[i] + 1) * 8, true);
            SplitArgs a{};
            a.bv = block_view(c, done[i]);
            a.hot_rank = hot ? s.hot_rank.as<int32_t>() : nullptr;
            a.j0 = j0[i];
            a.off = s.raw_off.as<int64_t>() + j0[i];
            a.bitmap = s.bitmap.as<unsigned long long>();
            a.nhot = s.nhot;
            a.cnt = c.sc.cnt.as<uint32_t>();
            a.implicit = s.implicit_roots;
            a.seed = s.seed;
            a.n = (uint32_t)c.g.n;
            a.ar_rank = s.nar ? s.ar_rank.as<int32_t>() : nullptr;
            sa.push_back(a);
            sb.push_back(grid_for(done[i] * WAVE, 256, 65536));
        }
        {
            const int ps = prof_begin(root, "cold_count");
            HBM_GLAUNCH(root, sa, sb, 0, k_cold_count, 256, SplitArgs);
            prof_end(root, ps);
        }
        HBM_HIP(hipGetLastError());
        std::vector<const int64_t *> tail;
        for (size_t q = 0; q < P.size(); q++) {
            Ctx &c = *J[P[q]];
            scan_u32_to_i64(root, sa[q].cnt, c.s.raw_off.as<int64_t>() + j0[P[q]], done[P[q]] + 1, c.s.raw_count);
            tail.push_back(c.s.raw_off.as<int64_t>() + j0[P[q]] + done[P[q]]);
        }
        std::vector<int64_t> total;
        gather_tails(root, tail, total);
        for (size_t q = 0; q < P.size(); q++) {
            Ctx &c = *J[P[q]];
            raw_grow(c, total[q]);
            sa[q].raw = c.s.raw_mem.as<int32_t>();
            sa[q].raw_host = c.s.raw_host;
            sa[q].raw_split = c.s.raw_split;
            sa[q].bitmap = c.s.bitmap.as<unsigned long long>();
            c.s.raw_count = total[q];
        }
        {
            const int ps = prof_begin(root, "split");
            HBM_GLAUNCH(root, sa, sb, 0, k_split, 256, SplitArgs);
            prof_end(root, ps);
        }
        HBM_HIP(hipGetLastError());
    }
    if (!H.empty()) {
        std::vector<HuffArgs> fa;
        std::vector<uint32_t> fb;
        for (size_t i : H) {
            Ctx &c = *J[i];
            Store &s = c.s;
            const bool hot = s.enc == HBM_ENC_HUFFMAN_HOT_BITMAP;
            buf_grow(c, s.bitoff, (size_t)(j0[i] + done[i] + 1) * 8, true);
            HuffArgs a{};
            a.bv = block_view(c, done[i]);
            a.h = HuffEnc{s.enc8.as<unsigned long long>(), s.lens.as<uint8_t>(), s.codes.as<uint32_t>(),
                          hot ? s.hot_rank.as<int32_t>() : nullptr,
                          s.cb.ustar_enc, s.cb.wbits, s.implicit_roots, s.seed, j0[i], (uint32_t)c.g.n,
                          s.nar ? s.ar_rank.as<int32_t>() : nullptr};
            a.bits = c.sc.aux.as<uint64_t>();
            a.meta = c.sc.cnt.as<uint32_t>();
            a.bitoff = s.bitoff.as<int64_t>() + j0[i];
            a.nesc_total = root.ctrl_arena.as<unsigned long long>() + i * CW_COUNT + CW_SUM;
            fa.push_back(a);
            fb.push_back(grid_for(done[i] * WAVE, 256, 65536));
        }
        {
            const int ps = prof_begin(root, "huff_bits");
            HBM_GLAUNCH(root, fa, fb, 0, k_huff_bits, 256, HuffArgs);
            prof_end(root, ps);
        }
        HBM_HIP(hipGetLastError());
        std::vector<const int64_t *> tail;
        for (size_t q = 0; q < H.size(); q++) {
            Ctx &c = *J[H[q]];
            scan_u64_to_i64(root, fa[q].bits, c.s.bitoff.as<int64_t>() + j0[H[q]], done[H[q]] + 1, (int64_t)c.s.nbits);
            tail.push_back(c.s.bitoff.as<int64_t>() + j0[H[q]] + done[H[q]]);
        }
        std::vector<int64_t> total;
        gather_tails(root, tail, total);
        std::vector<SplitArgs> sa;
        std::vector<uint32_t> sb;
        for (size_t q = 0; q < H.size(); q++) {
            Ctx &c = *J[H[q]];
            buf_grow(c, c.s.payload, (size_t)((total[q] + 31) / 32 + 2) * 4, true);
            buf_grow(c, c.s.ckb, (size_t)(total[q] / CK_SLOT + 2), true);
            fa[q].payload = c.s.payload.as<uint32_t>();
            fa[q].ckb = c.s.ckb.as<uint8_t>();
            c.s.nbits = (uint64_t)total[q];
            if (c.s.enc == HBM_ENC_HUFFMAN_HOT_BITMAP && c.s.nhot > 0) {  // hot bits (none: nothing to set)
                SplitArgs a{};
                a.bv = fa[q].bv;
                a.hot_rank = c.s.hot_rank.as<int32_t>();
                a.j0 = j0[H[q]];
                a.bitmap = c.s.bitmap.as<unsigned long long>();
                a.nhot = c.s.nhot;
                sa.push_back(a);
                sb.push_back(grid_for(done[H[q]] * WAVE, 256, 65536));
            }
        }
        // escape counters: zero this block's slots (the arena is the root's control block)
        HBM_HIP(hipMemsetAsync(root.ctrl_arena.p, 0, root.ctrl_arena.bytes, root.stream));
        {
            const int ps = prof_begin(root, "huff_write");
            HBM_GLAUNCH(root, fa, fb, 0, k_huff_write, 256, HuffArgs);
            prof_end(root, ps);
        }
        HBM_HIP(hipGetLastError());
        HBM_GLAUNCH(root, sa, sb, 0, k_split, 256, SplitArgs);
        HBM_HIP(hipGetLastError());
        std::vector<unsigned long long> esc(root.ctrl_arena.bytes / 8);
        HBM_HIP(hipMemcpyAsync(esc.data(), root.ctrl_arena.p, root.ctrl_arena.bytes, hipMemcpyDeviceToHost, root.stream));
        HBM_HIP(hipStreamSynchronize(root.stream));
        for (size_t i : H) J[i]->s.escapes += (int64_t)esc[i * CW_COUNT + CW_SUM];
    }
    for (size_t i = 0; i < N; i++)
        if (!arr[i].empty()) {
            const int ps = prof_begin(root, "arr_rows");
            arr_write(*J[i], j0[i], done[i], arr[i]);
            prof_end(root, ps);
        }
    std::vector<HistArgs> ha;
    std::vector<uint32_t> hb;
    for (size_t i = 0; i < N; i++) {
        ha.push_back(HistArgs{block_view(*J[i], done[i]), J[i]->s.hist.as<uint32_t>()});
        hb.push_back(grid_for(done[i] * WAVE, 256, 65536));
    }
    {
        const int ps = prof_begin(root, "hist_add");
        HBM_GLAUNCH(root, ha, hb, 0, k_hist_add, 256, HistArgs);
        prof_end(root, ps);
    }
    HBM_HIP(hipGetLastError());
    for (size_t i = 0; i < N; i++) J[i]->s.nsets = j0[i] + done[i];
}

// Bring a job's store in line with a request for sets [0, theta) under `seed`: a new seed
// or a smaller theta starts over; the warm-up size is fixed by the first request.
static void extend_prepare(Ctx &root, Ctx &c, int64_t theta, uint64_t seed) {
    HBM_REQUIRE(c.g.loaded, HBM_ESTATE, "no graph loaded");
    HBM_REQUIRE(theta >= 0 && theta < (int64_t(1) << 31), HBM_EINVAL, "theta must be in [0, 2^31)");
    Store &s = c.s;
    if ((s.has_seed && s.seed != seed) || theta < s.nsets) store_reset(c);
    s.has_seed = true;
    s.seed = seed;
    if (theta == s.nsets) return;
    if (!s.hist.p) {
        buf_alloc(c, s.hist, (size_t)c.g.n * 4);
        buf_zero(c, s.hist, 0, (size_t)c.g.n * 4);
    }
    if (s.W == 0) {
        const int64_t w = (int64_t)std::ceil(s.warmup_frac * (double)theta);
        s.W = std::max<int64_t>(1, std::min<int64_t>(w, theta));
    }
    if (s.enc != HBM_ENC_NONE && !s.model_ready && s.wcur == 0) {
        buf_grow(c, s.warm, (size_t)c.g.n * 4, false);
        buf_zero(c, s.warm, 0, (size_t)c.g.n * 4);
        s.warm_sizes.clear();
    }
    // arena sized to the request (about 64 ids per set), within [4M, 64M] entries
    const int64_t want_sets = std::min<int64_t>(theta - s.nsets, root.block_sets);
    const size_t entries =
        (size_t)std::min<int64_t>(std::max<int64_t>(want_sets * 64, int64_t(1) << 22), int64_t(64) << 20);
    ensure_scratch(c, std::max<size_t>(c.sc.cap, entries), std::max<int64_t>(c.sc.bcap, want_sets));
}

void extend_step(Ctx &root, const std::vector<Ctx *> &J, const std::vector<int64_t> &theta,
                 const std::vector<uint64_t> &seed, const std::vector<int64_t> &cap, std::vector<hbm_status> &st) {
    const size_t N = J.size();
    st.assign(N, HBM_OK);
    stage_reset(root);
    hipEvent_t e0, e1;
    HBM_HIP(hipEventCreate(&e0));
    HBM_HIP(hipEventCreate(&e1));
    HBM_HIP(hipEventRecord(e0, root.stream));
    try {
        std::vector<Ctx *> jobs;
        std::vector<size_t> idx;
        std::vector<int64_t> j0, nb, done;
        std::vector<uint64_t> sd;
        std::vector<char> warm, fuse;
        for (size_t i = 0; i < N; i++) {
            Ctx &c = *J[i];
            extend_prepare(root, c, theta[i], seed[i]);
            Store &s = c.s;
            if (s.nsets >= theta[i]) continue;
            const bool w = s.enc != HBM_ENC_NONE && !s.model_ready;
            const int64_t lim = (!cap.empty() && cap[i] >= 0) ? cap[i] : INT64_MAX;
            const int64_t from = w ? s.wcur : s.nsets;
            int64_t b = std::min<int64_t>({theta[i] - from, root.block_sets, c.sc.bcap, lim});
            // A fresh warm-up whose block may be stored whole and covers sets [0, W) counts
            // the frequencies of those W sets, builds the model and then encodes the whole
            // block with it: the warm-up sets are sampled once.  Otherwise a warm-up block
            // holds sets [wcur, W) only; it stores nothing, so the cap does not bound it.
            const bool f = w && s.wcur == 0 && b >= s.W;
            if (w && !f) b = std::min<int64_t>({s.W - s.wcur, root.block_sets, c.sc.bcap});
            if (b <= 0) continue;
            idx.push_back(i);
            jobs.push_back(&c);
            j0.push_back(from);
            nb.push_back(b);
            sd.push_back(seed[i]);
            warm.push_back(w);
            fuse.push_back(f);
        }
        if (!jobs.empty()) sample_blocks(root, jobs, j0, nb, sd, done);
        // warm-up blocks: frequencies of sets [0, W) only
        std::vector<HistArgs> ha;
        std::vector<uint32_t> hb;
        std::vector<Ctx *> ajobs;
        std::vector<int64_t> aj0, adone, wn(jobs.size(), 0);
        for (size_t q = 0; q < jobs.size(); q++) {
            Ctx &c = *jobs[q];
            if (done[q] == 0) {  // the first set did not fit the arena: retry with twice the room
                ensure_scratch(c, c.sc.cap * 2, c.sc.bcap);
                continue;
            }
            if (warm[q]) {
                wn[q] = std::min<int64_t>(done[q], c.s.W - c.s.wcur);  // the block's warm-up sets lead it
                ha.push_back(HistArgs{block_view(c, wn[q]), c.s.warm.as<uint32_t>()});
                hb.push_back(grid_for(wn[q] * WAVE, 256, 65536));
            } else {
                if (c.s.enc == HBM_ENC_NONE) record_warm_sizes(c, j0[q], done[q]);
                ajobs.push_back(&c);
                aj0.push_back(j0[q]);
                adone.push_back(done[q]);
            }
        }
        HBM_GLAUNCH(root, ha, hb, 0, k_hist_add, 256, HistArgs);
        HBM_HIP(hipGetLastError());
        for (size_t q = 0; q < jobs.size(); q++) {
            Ctx &c = *jobs[q];
            if (!warm[q] || !done[q]) continue;
            record_warm_sizes(c, j0[q], wn[q]);
            c.s.wcur += wn[q];
            if (c.s.wcur >= c.s.W) {
                characterize(c.s, c.g.n);
                try {
                    HBM_HIP(hipStreamSynchronize(c.stream));  // the warm-up block is done: time the model alone
                    const auto tm0 = std::chrono::steady_clock::now();
                    build_model(c);
                    c.t_encode += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tm0).count();
                } catch (...) {  // e.g. ENOMEM: the warm-up starts over at the next request
                    c.s.wcur = 0;
                    c.s.warm_sizes.clear();
                    c.s.enc = c.s.enc_req;
                    throw;
                }
                if (fuse[q]) {  // sets [0, done) are still in the arena
                    ajobs.push_back(&c);
                    aj0.push_back(j0[q]);
                    adone.push_back(done[q]);
                }
            }
        }
        if (!ajobs.empty()) append_blocks(root, ajobs, aj0, adone);
        for (size_t q = 0; q < ajobs.size(); q++) {
            Ctx &c = *ajobs[q];
            if (c.s.enc == HBM_ENC_NONE && aj0[q] < c.s.W && c.s.nsets >= c.s.W) characterize(c.s, c.g.n);
        }
        for (size_t q = 0; q < jobs.size(); q++) {
            Ctx &c = *jobs[q];
            if (c.budget > 0 && store_bytes(c) > c.budget) st[idx[q]] = HBM_EBUDGET;
        }
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    HBM_HIP(hipEventRecord(e1, root.stream));
    HBM_HIP(hipEventSynchronize(e1));
    float ms = 0;
    HBM_HIP(hipEventElapsedTime(&ms, e0, e1));
    for (Ctx *c : J) c->t_sample += ms;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
}

// Make every job's store hold sets 0..theta[i]-1 under seed[i], all jobs advancing together
// block by block.  A job over its budget stops the call with EBUDGET.
void extend_stores(Ctx &root, const std::vector<Ctx *> &J, const std::vector<int64_t> &theta,
                   const std::vector<uint64_t> &seed) {
    std::vector<hbm_status> st;
    for (;;) {
        bool more = false;
        for (size_t i = 0; i < J.size(); i++) more |= J[i]->s.nsets < theta[i] || (J[i]->s.has_seed && J[i]->s.seed != seed[i]);
        if (!more) {
            for (size_t i = 0; i < J.size(); i++) extend_prepare(root, *J[i], theta[i], seed[i]);
            return;
        }
        extend_step(root, J, theta, seed, {}, st);
        for (size_t i = 0; i < J.size(); i++)
            if (st[i] == HBM_EBUDGET)
                throw Error{HBM_EBUDGET, "store budget exceeded at " + std::to_string(J[i]->s.nsets) + " sets"};
    }
}

void store_extend(Ctx &c, int64_t theta, uint64_t seed) {
    extend_stores(c, std::vector<Ctx *>{&c}, std::vector<int64_t>{theta}, std::vector<uint64_t>{seed});
}

// sum of x[0, n) into *out (one atomic per workgroup; *out starts at zero)
__global__ __launch_bounds__(256) void k_sum_u32(const uint32_t *x, int64_t n, unsigned long long *out) {
    __shared__ unsigned long long ws[256 / WAVE];
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nthr = (int64_t)gridDim.x * blockDim.x;
    unsigned long long t = 0;
    const int64_t n4 = n >> 2;
    const uint4 *x4 = reinterpret_cast<const uint4 *>(x);
    for (int64_t q = tid; q < n4; q += nthr) {
        const uint4 v = x4[q];
        t += (unsigned long long)v.x + v.y + v.z + v.w;
    }
    for (int64_t i = n4 * 4 + tid; i < n; i += nthr) t += x[i];
    t = wave_sum(t);
    if (lane_id() == 0) ws[threadIdx.x / WAVE] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long b = 0;
        for (int w = 0; w < 256 / WAVE; w++) b += ws[w];
        if (b) atomicAdd(out, b);
    }
}

void store_stats(Ctx &c, hbm_store_stats *o) {
    Store &s = c.s;
    *o = hbm_store_stats{};
    o->nsets = s.nsets;
    o->warmup_sets = s.W;
    o->encoding = s.enc;
    o->nhot = s.nhot;
    o->alphabet = s.cb.nsym;
    o->max_code_len = s.cb.maxlen;
    o->ustar_enc = s.cb.ustar_enc;
    o->escape_bits = s.cb.wbits;
    o->escapes = s.escapes;
    o->payload_bits = s.nbits;
    const bool huff = enc_huff(s.enc), raw = enc_raw(s.enc);
    o->index_bytes = s.nsets && (huff || raw) ? (s.nsets + 1) * 8 + (huff ? (int64_t)(s.nbits / CK_SLOT + 1) : 0) : 0;
    o->bitmap_bytes = s.bm_words * (int64_t)s.nhot * 8;
    o->raw_bytes = raw ? s.raw_count * 4 : 0;
    o->codebook_bytes = huff ? (int64_t)c.g.n * (1 + 8) + (int64_t)s.cb.nsym * 4 + 68 * 8 : 0;
    if (s.nhot) o->codebook_bytes += (int64_t)s.nhot * 4;
    o->store_bytes = store_bytes(c);
    o->skewness = s.skew;
    o->density = s.density;
    o->narray = s.nar;
    o->array_entries = s.ar_entries;
    o->array_bytes = s.ar_chunks * (int64_t)(s.nar + 1) * 8 + s.ar_entries * 2;
    if (s.nar) o->codebook_bytes += (int64_t)s.nar * 4;
    // total members = sum of the histogram (reduced on the device; 8 bytes come back)
    if (s.hist.p && s.nsets) {
        buf_grow(c, s.mtmp, 8, true);
        buf_zero(c, s.mtmp, 0, 8);
        k_sum_u32<<<grid_for(((int64_t)c.g.n + 3) / 4, 256 * 8, (int64_t)c.num_cus), 256, 0, c.stream>>>(
            s.hist.as<uint32_t>(), c.g.n, s.mtmp.as<unsigned long long>());
        HBM_HIP(hipGetLastError());
        unsigned long long t = 0;
        HBM_HIP(hipMemcpyAsync(&t, s.mtmp.p, 8, hipMemcpyDeviceToHost, c.stream));
        HBM_HIP(hipStreamSynchronize(c.stream));
        o->members = (int64_t)t;
    }
}

void store_dump(Ctx &c, int64_t j0, int64_t j1, std::vector<int64_t> &off, std::vector<int32_t> &mem) {
    const int64_t cnt = j1 - j0;
    off.assign((size_t)cnt + 1, 0);
    mem.clear();
    if (cnt <= 0) return;
    DecodeView d = make_view(c);
    Buf sizes, offs, out;
    try {
        buf_alloc(c, sizes, (size_t)(cnt + 1) * 4);
        buf_alloc(c, offs, (size_t)(cnt + 1) * 8);
        k_decode_count<<<grid_for(cnt, 128, 65536), 128, 0, c.stream>>>(d, j0, cnt, sizes.as<uint32_t>());
        HBM_HIP(hipGetLastError());
        HBM_HIP(hipMemsetAsync(sizes.as<uint32_t>() + cnt, 0, 4, c.stream));
        scan_u32_to_i64(c, sizes.as<uint32_t>(), offs.as<int64_t>(), cnt + 1, 0);
        HBM_HIP(hipMemcpyAsync(off.data(), offs.p, (size_t)(cnt + 1) * 8, hipMemcpyDeviceToHost, c.stream));
        HBM_HIP(hipStreamSynchronize(c.stream));
        const int64_t total = off[(size_t)cnt];
        buf_alloc(c, out, (size_t)std::max<int64_t>(total, 1) * 4);
        k_decode_write<<<grid_for(cnt, 128, 65536), 128, 0, c.stream>>>(d, j0, cnt, offs.as<int64_t>(),
                                                                         out.as<int32_t>());
        HBM_HIP(hipGetLastError());
        mem.resize((size_t)total);
        HBM_HIP(hipMemcpyAsync(mem.data(), out.p, (size_t)total * 4, hipMemcpyDeviceToHost, c.stream));
        HBM_HIP(hipStreamSynchronize(c.stream));
    } catch (...) {
        buf_free(c, sizes);
        buf_free(c, offs);
        buf_free(c, out);
        throw;
    }
    buf_free(c, sizes);
    buf_free(c, offs);
    buf_free(c, out);
}

}  // namespace hbm
