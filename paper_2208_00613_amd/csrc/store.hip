// store.hip -- block-based sampling-and-encoding (Alg. 1) into the RR store.
//
// A request for sets [nsets, theta) runs in blocks sized to the scratch arena.
// With an encoding, the first request begins with a warm-up pass over sets
// [0, W): their vertex frequencies give the hot set and the Huffman codebook
// (Alg. 1's first block; never rebuilt).  Sets are pure functions of their
// index, so the warm-up sets are then simply sampled again and encoded like
// every other block.  After each block the raw members are dropped; only the
// encoded form stays (the "Deallocate R_i" step).
//
// Store layouts (device memory):
//   hist      uint32[n]   frequency of every vertex over all sets (UpdateHistogram)
//   RAW       raw_off int64[nsets+1], raw_mem int32[]: ascending ids (all of a set,
//             or its non-hot part under HOT_BITMAP)
//   HOT rows  bitmap uint64[ceil(nsets/64) * nhot], word-major: the bit of set j
//             for hot rank r is bit j%64 of word (j/64)*nhot + r (the Bitmax bit
//             matrix of its encoding section, restricted to hot vertices)
//   HUFFMAN   bitoff int64[nsets+1]; set j is bits [bitoff[j], bitoff[j+1]) of an
//             MSB-first stream: Elias-gamma(nesc+1), the nesc codeless ids as
//             fixed-width fields (the CP copies kept in-band), then the canonical
//             codes of the coded ids, the warm-up top vertex first (the u*
//             swap-to-front of the Huffmax encoding section), the rest ascending.
#include <algorithm>
#include <cmath>
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

__global__ void k_hist_add(BlockView bv, uint32_t *__restrict__ hist) {
    // one wave per set: lanes stride over its members
    const uint64_t wave = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) / WAVE;
    const uint64_t nw = (uint64_t)gridDim.x * blockDim.x / WAVE;
    const unsigned lane = lane_id();
    for (uint64_t b = wave; b < (uint64_t)bv.nb; b += nw) {
        const uint32_t p = bv.pos[b], s = bv.size[b];
        for (uint32_t i = lane; i < s; i += WAVE) atomicAdd(&hist[bv.mem[p + i]], 1u);
    }
}

// per-set count of members kept as plain ids (all of them when hot_rank is null); one wave per set
__global__ void k_cold_count(BlockView bv, const int32_t *__restrict__ hot_rank, uint32_t *__restrict__ out) {
    const uint64_t wave = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) / WAVE;
    const uint64_t nw = (uint64_t)gridDim.x * blockDim.x / WAVE;
    const unsigned lane = lane_id();
    for (uint64_t b = wave; b < (uint64_t)bv.nb; b += nw) {
        const uint32_t p = bv.pos[b], s = bv.size[b];
        uint32_t c = s;
        if (hot_rank) {
            c = 0;
            for (uint32_t i = lane; i < s; i += WAVE) c += hot_rank[bv.mem[p + i]] < 0;
            c = wave_sum(c);
        }
        if (lane == 0) out[b] = c;
    }
}

// Copy plain ids to the raw store and set hot bits.  One wave per set.
__global__ void k_split(BlockView bv, const int32_t *__restrict__ hot_rank, int64_t j0, const int64_t *__restrict__ off,
                        int32_t *__restrict__ raw, unsigned long long *__restrict__ bitmap, int32_t nhot) {
    const uint64_t wave = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) / WAVE;
    const uint64_t nw = (uint64_t)gridDim.x * blockDim.x / WAVE;
    const unsigned lane = lane_id();
    for (uint64_t b = wave; b < (uint64_t)bv.nb; b += nw) {
        const uint32_t p = bv.pos[b], s = bv.size[b];
        const int64_t o = off ? off[b] : 0;
        const uint64_t j = (uint64_t)j0 + b;
        uint32_t written = 0;
        for (uint32_t base = 0; base < s; base += WAVE) {
            const uint32_t i = base + lane;
            uint32_t v = 0;
            int32_t r = -1;
            if (i < s) {
                v = bv.mem[p + i];
                if (hot_rank) r = hot_rank[v];
            }
            const bool cold = i < s && r < 0;
            const uint64_t m = __ballot(cold);
            if (cold && raw) raw[o + written + __popcll(m & ((1ull << lane) - 1))] = (int32_t)v;
            written += __popcll(m);
            if (i < s && r >= 0) atomicOr(&bitmap[(j >> 6) * (uint64_t)nhot + r], 1ull << (j & 63));
        }
    }
}

// ------------------------------------------------------------------ Huffman stream
struct HuffEnc {
    const uint8_t *lens;
    const uint32_t *codes;
    const int32_t *hot_rank;  // may be null
    int32_t ustar;
    int32_t wbits;
};

__device__ __forceinline__ int floor_log2_u32(uint32_t x) { return 31 - __clz(x); }

__global__ void k_huff_bits(BlockView bv, HuffEnc h, uint64_t *__restrict__ bits_out) {
    for (uint64_t b = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; b < (uint64_t)bv.nb;
         b += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t p = bv.pos[b], s = bv.size[b];
        uint64_t bits = 0;
        uint32_t nesc = 0;
        for (uint32_t i = 0; i < s; i++) {
            const uint32_t v = bv.mem[p + i];
            if (h.hot_rank && h.hot_rank[v] >= 0) continue;
            const uint32_t L = h.lens[v];
            if (L) bits += L;
            else nesc++;
        }
        bits += 2 * (uint64_t)floor_log2_u32(nesc + 1) + 1 + (uint64_t)nesc * h.wbits;
        bits_out[b] = bits;
    }
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

__global__ void k_huff_write(BlockView bv, HuffEnc h, const int64_t *__restrict__ bitoff, uint32_t *__restrict__ payload,
                             unsigned long long *__restrict__ nesc_total) {
    uint64_t esc_local = 0;
    for (uint64_t b = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; b < (uint64_t)bv.nb;
         b += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t p = bv.pos[b], s = bv.size[b];
        uint64_t pos = (uint64_t)bitoff[b];
        uint32_t nesc = 0;
        bool has_front = false;
        for (uint32_t i = 0; i < s; i++) {
            const uint32_t v = bv.mem[p + i];
            if (h.hot_rank && h.hot_rank[v] >= 0) continue;
            if (!h.lens[v]) nesc++;
            if ((int32_t)v == h.ustar) has_front = true;
        }
        const uint32_t L = (uint32_t)floor_log2_u32(nesc + 1);
        pos += L;
        put_bits(payload, pos, nesc + 1, L + 1);
        pos += L + 1;
        for (uint32_t i = 0; i < s && nesc; i++) {
            const uint32_t v = bv.mem[p + i];
            if (h.hot_rank && h.hot_rank[v] >= 0) continue;
            if (!h.lens[v]) {
                put_bits(payload, pos, v, h.wbits);
                pos += h.wbits;
            }
        }
        if (has_front) {
            const uint32_t Lf = h.lens[h.ustar];
            put_bits(payload, pos, h.codes[h.ustar], Lf);
            pos += Lf;
        }
        for (uint32_t i = 0; i < s; i++) {
            const uint32_t v = bv.mem[p + i];
            if ((int32_t)v == h.ustar) continue;
            if (h.hot_rank && h.hot_rank[v] >= 0) continue;
            const uint32_t Lv = h.lens[v];
            if (Lv) {
                put_bits(payload, pos, h.codes[v], Lv);
                pos += Lv;
            }
        }
        esc_local += nesc;
    }
    if (esc_local) atomicAdd(nesc_total, (unsigned long long)esc_local);
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
    if (d.raw_off) {
        for (int64_t i = d.raw_off[j]; i < d.raw_off[j + 1]; i++) {
            if (out) out[c] = d.raw_mem[i];
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
    const bool huff = s.enc == HBM_ENC_HUFFMAN || s.enc == HBM_ENC_HUFFMAN_HOT_BITMAP;
    d.raw_off = huff ? nullptr : s.raw_off.as<int64_t>();
    d.raw_mem = huff ? nullptr : s.raw_mem.as<int32_t>();
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
    s.has_seed = false;
    s.nsets = 0;
    s.W = 0;
    s.model_ready = false;
    s.members = 0;
    s.nhot = 0;
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
    for (Buf *b : {&s.hist, &s.warm, &s.hot, &s.hot_rank, &s.bitmap, &s.raw_off, &s.raw_mem, &s.lens, &s.codes,
                   &s.symtab, &s.cbtab, &s.lut, &s.bitoff, &s.payload})
        buf_free(c, *b);
    Scratch &sc = c.sc;
    for (Buf *b : {&sc.mem, &sc.pos, &sc.size, &sc.ctrl, &sc.defer, &sc.t2_bitmap, &sc.t2_queue, &sc.aux, &sc.cnt})
        buf_free(c, *b);
    sc.cap = 0;
    sc.bcap = 0;
    sc.t2_slots = 0;
}

int64_t store_bytes(const Ctx &c) {
    const Store &s = c.s;
    int64_t b = 0;
    const bool huff = s.enc == HBM_ENC_HUFFMAN || s.enc == HBM_ENC_HUFFMAN_HOT_BITMAP;
    if (huff) b += (s.nsets + 1) * 8 + (int64_t)((s.nbits + 7) / 8);
    else b += (s.nsets + 1) * 8 + s.raw_count * 4;
    b += s.bm_words * (int64_t)s.nhot * 8;
    return b;
}

static void ensure_scratch(Ctx &c, size_t entries, int64_t bcap) {
    Scratch &sc = c.sc;
    if (entries > sc.cap) {
        buf_alloc(c, sc.mem, entries * 4);
        sc.cap = entries;
    }
    if (bcap > sc.bcap) {
        buf_alloc(c, sc.pos, (size_t)bcap * 4);
        buf_alloc(c, sc.size, (size_t)(bcap + 1) * 4);
        buf_alloc(c, sc.defer, (size_t)bcap * 2 * 4);
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
        std::iota(order.begin(), order.end(), 0);
        std::sort(order.begin(), order.end(), [&](size_t a, size_t b) {
            return w[a] != w[b] ? w[a] < w[b] : syms[a].second < syms[b].second;
        });
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

static void build_model(Ctx &c) {
    Store &s = c.s;
    const int32_t n = c.g.n;
    std::vector<uint32_t> warm(n);
    HBM_HIP(hipMemcpyAsync(warm.data(), s.warm.p, (size_t)n * 4, hipMemcpyDeviceToHost, c.stream));
    HBM_HIP(hipStreamSynchronize(c.stream));
    const bool hot = s.enc == HBM_ENC_HOT_BITMAP || s.enc == HBM_ENC_HUFFMAN_HOT_BITMAP;
    const bool huff = s.enc == HBM_ENC_HUFFMAN || s.enc == HBM_ENC_HUFFMAN_HOT_BITMAP;
    std::vector<int32_t> rank;
    s.nhot = 0;
    if (hot) {
        std::vector<int32_t> seen;
        for (int32_t v = 0; v < n; v++)
            if (warm[v]) seen.push_back(v);
        const int64_t want = (int64_t)std::ceil(s.hot_frac * (double)n);
        const size_t keep = (size_t)std::min<int64_t>(want, (int64_t)seen.size());
        std::partial_sort(seen.begin(), seen.begin() + keep, seen.end(), [&](int32_t a, int32_t b) {
            return warm[a] != warm[b] ? warm[a] > warm[b] : a < b;
        });
        seen.resize(keep);
        s.nhot = (int32_t)keep;
        rank.assign(n, -1);
        for (size_t r = 0; r < keep; r++) rank[seen[r]] = (int32_t)r;
        buf_alloc(c, s.hot, std::max<size_t>(keep, 1) * 4);
        buf_alloc(c, s.hot_rank, (size_t)n * 4);
        HBM_HIP(hipMemcpyAsync(s.hot.p, seen.data(), keep * 4, hipMemcpyHostToDevice, c.stream));
        HBM_HIP(hipMemcpyAsync(s.hot_rank.p, rank.data(), (size_t)n * 4, hipMemcpyHostToDevice, c.stream));
    }
    if (huff) {
        std::vector<std::pair<uint64_t, int32_t>> syms;
        for (int32_t v = 0; v < n; v++)
            if (warm[v] && (!hot || rank[v] < 0)) syms.push_back({warm[v], v});
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
        std::vector<size_t> ord(syms.size());
        std::iota(ord.begin(), ord.end(), 0);
        std::sort(ord.begin(), ord.end(), [&](size_t a, size_t b) {
            return L[a] != L[b] ? L[a] < L[b] : syms[a].second < syms[b].second;
        });
        std::vector<uint8_t> lens(n, 0);
        std::vector<uint32_t> codes(n, 0);
        std::vector<int32_t> symtab(std::max<size_t>(syms.size(), 1), 0);
        uint64_t count[34] = {}, first[34] = {}, firstidx[34] = {};
        for (size_t i = 0; i < syms.size(); i++) count[L[i]]++;
        uint64_t code = 0;
        for (size_t q = 0; q < ord.size(); q++) {
            const size_t i = ord[q];
            if (q > 0) code = (code + 1) << (L[i] - L[ord[q - 1]]);
            lens[syms[i].second] = L[i];
            codes[syms[i].second] = (uint32_t)code;
            symtab[q] = syms[i].second;
        }
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
        // with such a code maps to (symbol << 5) | length; longer codes keep 0 (search the limits)
        std::vector<uint32_t> lut((size_t)1 << LUT_BITS, 0u);
        for (size_t q = 0; q < ord.size(); q++) {
            const size_t i = ord[q];
            const int L = L_of(i);
            if (L > LUT_BITS) break;
            const uint32_t cd = codes[syms[i].second];
            const uint32_t lo = cd << (LUT_BITS - L), hi = (cd + 1) << (LUT_BITS - L);
            for (uint32_t x = lo; x < hi; x++) lut[x] = ((uint32_t)syms[i].second << 5) | (uint32_t)L;
        }
        buf_alloc(c, s.lens, (size_t)n);
        buf_alloc(c, s.codes, (size_t)n * 4);
        buf_alloc(c, s.symtab, symtab.size() * 4);
        buf_alloc(c, s.cbtab, 68 * 8);
        buf_alloc(c, s.lut, lut.size() * 4);
        HBM_HIP(hipMemcpyAsync(s.lut.p, lut.data(), lut.size() * 4, hipMemcpyHostToDevice, c.stream));
        HBM_HIP(hipMemcpyAsync(s.lens.p, lens.data(), (size_t)n, hipMemcpyHostToDevice, c.stream));
        HBM_HIP(hipMemcpyAsync(s.codes.p, codes.data(), (size_t)n * 4, hipMemcpyHostToDevice, c.stream));
        HBM_HIP(hipMemcpyAsync(s.symtab.p, symtab.data(), symtab.size() * 4, hipMemcpyHostToDevice, c.stream));
        HBM_HIP(hipMemcpyAsync(s.cbtab.p, tab_lim, 34 * 8, hipMemcpyHostToDevice, c.stream));
        HBM_HIP(hipMemcpyAsync(s.cbtab.as<int64_t>() + 34, tab_base, 34 * 8, hipMemcpyHostToDevice, c.stream));
        HBM_HIP(hipStreamSynchronize(c.stream));
    } else if (hot) {
        HBM_HIP(hipStreamSynchronize(c.stream));
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

// Append sets [j0, j0+done) from scratch to the store.
static void append_block(Ctx &c, int64_t j0, int64_t done) {
    Store &s = c.s;
    Scratch &sc = c.sc;
    const int32_t n = c.g.n;
    BlockView bv{sc.mem.as<uint32_t>(), sc.pos.as<uint32_t>(), sc.size.as<uint32_t>(), done};
    const unsigned gw = grid_for(done * WAVE, 256, 65536);
    const unsigned gt = grid_for(done, 256, 65536);
    {
        const int ps_ = prof_begin(c, "hist_add");
        k_hist_add<<<gw, 256, 0, c.stream>>>(bv, s.hist.as<uint32_t>());
        prof_end(c, ps_, 0);
    }
    HBM_HIP(hipGetLastError());
    const bool hot = s.enc == HBM_ENC_HOT_BITMAP || s.enc == HBM_ENC_HUFFMAN_HOT_BITMAP;
    const bool huff = s.enc == HBM_ENC_HUFFMAN || s.enc == HBM_ENC_HUFFMAN_HOT_BITMAP;
    const int64_t new_sets = j0 + done;
    if (hot) {
        const int64_t words = (new_sets + 63) / 64;
        buf_grow(c, s.bitmap, (size_t)std::max<int64_t>(words * s.nhot, 1) * 8, true);
        s.bm_words = words;
    }
    if (!huff) {
        // plain ids: sizes -> offsets -> copy
        uint32_t *cnt = sc.cnt.as<uint32_t>();
        {
            const int ps_ = prof_begin(c, "cold_count");
            k_cold_count<<<gw, 256, 0, c.stream>>>(bv, hot ? s.hot_rank.as<int32_t>() : nullptr, cnt);
            prof_end(c, ps_, 0);
        }
        HBM_HIP(hipGetLastError());
        buf_grow(c, s.raw_off, (size_t)(new_sets + 1) * 8, true);
        // scan of the block's counts, placed after the existing offsets
        HBM_HIP(hipMemsetAsync(cnt + done, 0, 4, c.stream));
        scan_u32_to_i64(c, cnt, s.raw_off.as<int64_t>() + j0, done + 1, s.raw_count);
        const int64_t total = read_dev<int64_t>(c, s.raw_off.as<int64_t>() + new_sets);
        buf_grow(c, s.raw_mem, (size_t)std::max<int64_t>(total, 1) * 4, true);
        {
            const int ps_ = prof_begin(c, "split");
            k_split<<<gw, 256, 0, c.stream>>>(bv, hot ? s.hot_rank.as<int32_t>() : nullptr, j0, s.raw_off.as<int64_t>() + j0,
                                          s.raw_mem.as<int32_t>(), s.bitmap.as<unsigned long long>(), s.nhot);
            prof_end(c, ps_, 0);
        }
        HBM_HIP(hipGetLastError());
        s.raw_count = total;
    } else {
        HuffEnc h{s.lens.as<uint8_t>(), s.codes.as<uint32_t>(), hot ? s.hot_rank.as<int32_t>() : nullptr,
                  s.cb.ustar_enc, s.cb.wbits};
        uint64_t *bits = sc.aux.as<uint64_t>();
        {
            const int ps_ = prof_begin(c, "huff_bits");
            k_huff_bits<<<gt, 256, 0, c.stream>>>(bv, h, bits);
            prof_end(c, ps_, 0);
        }
        HBM_HIP(hipGetLastError());
        HBM_HIP(hipMemsetAsync(bits + done, 0, 8, c.stream));
        buf_grow(c, s.bitoff, (size_t)(new_sets + 1) * 8, true);
        scan_u64_to_i64(c, bits, s.bitoff.as<int64_t>() + j0, done + 1, (int64_t)s.nbits);
        const int64_t total = read_dev<int64_t>(c, s.bitoff.as<int64_t>() + new_sets);
        buf_grow(c, s.payload, (size_t)((total + 31) / 32 + 2) * 4, true);
        HBM_HIP(hipMemsetAsync(sc.ctrl.as<unsigned long long>() + CW_SUM, 0, 8, c.stream));
        {
            const int ps_ = prof_begin(c, "huff_write");
            k_huff_write<<<gt, 256, 0, c.stream>>>(bv, h, s.bitoff.as<int64_t>() + j0, s.payload.as<uint32_t>(),
                                               sc.ctrl.as<unsigned long long>() + CW_SUM);
            prof_end(c, ps_, 0);
        }
        HBM_HIP(hipGetLastError());
        if (hot)
            k_split<<<gw, 256, 0, c.stream>>>(bv, s.hot_rank.as<int32_t>(), j0, nullptr, nullptr,
                                              s.bitmap.as<unsigned long long>(), s.nhot);
        s.escapes += (int64_t)read_dev<unsigned long long>(c, sc.ctrl.as<unsigned long long>() + CW_SUM);
        s.nbits = (uint64_t)total;
    }
    s.nsets = new_sets;
}

void store_extend(Ctx &c, int64_t theta, uint64_t seed) {
    HBM_REQUIRE(c.g.loaded, HBM_ESTATE, "no graph loaded");
    HBM_REQUIRE(theta >= 0 && theta < (int64_t(1) << 31), HBM_EINVAL, "theta must be in [0, 2^31)");
    Store &s = c.s;
    if ((s.has_seed && s.seed != seed) || theta < s.nsets) store_reset(c);
    if (theta == s.nsets) {
        s.has_seed = true;
        s.seed = seed;
        return;
    }
    const int32_t n = c.g.n;
    if (!s.hist.p) {
        buf_alloc(c, s.hist, (size_t)n * 4);
        buf_zero(c, s.hist, 0, (size_t)n * 4);
    }
    s.has_seed = true;
    s.seed = seed;
    if (s.W == 0) {
        int64_t w = (int64_t)std::ceil(s.warmup_frac * (double)theta);
        s.W = std::max<int64_t>(1, std::min<int64_t>(w, theta));
    }
    const int64_t nsets_before = s.nsets;
    const int64_t budget = c.budget;
    hipEvent_t e0, e1;
    HBM_HIP(hipEventCreate(&e0));
    HBM_HIP(hipEventCreate(&e1));
    HBM_HIP(hipEventRecord(e0, c.stream));
    ensure_scratch(c, std::max<size_t>(c.sc.cap, size_t(64) << 20), std::max<int64_t>(c.sc.bcap, c.block_sets));
    const bool encoded = s.enc != HBM_ENC_NONE;
    try {
        if (encoded && !s.model_ready) {
            buf_grow(c, s.warm, (size_t)n * 4, false);
            buf_zero(c, s.warm, 0, (size_t)n * 4);
            s.warm_sizes.clear();
            for (int64_t j = 0; j < s.W;) {
                const int64_t nb = std::min<int64_t>(s.W - j, c.block_sets);
                const int64_t done = sample_block(c, j, j + nb, seed);
                if (done == 0) {
                    ensure_scratch(c, c.sc.cap * 2, c.sc.bcap);
                    continue;
                }
                BlockView bv{c.sc.mem.as<uint32_t>(), c.sc.pos.as<uint32_t>(), c.sc.size.as<uint32_t>(), done};
                k_hist_add<<<grid_for(done * WAVE, 256, 65536), 256, 0, c.stream>>>(bv, s.warm.as<uint32_t>());
                HBM_HIP(hipGetLastError());
                record_warm_sizes(c, j, done);
                j += done;
            }
            characterize(s, n);
            build_model(c);
        }
        for (int64_t j = s.nsets; j < theta;) {
            const int64_t nb = std::min<int64_t>(theta - j, c.block_sets);
            const int64_t done = sample_block(c, j, j + nb, seed);
            if (done == 0) {
                ensure_scratch(c, c.sc.cap * 2, c.sc.bcap);
                continue;
            }
            if (!encoded) record_warm_sizes(c, j, done);
            append_block(c, j, done);
            j += done;
            if (budget > 0 && store_bytes(c) > budget)
                throw Error{HBM_EBUDGET, "store budget exceeded at " + std::to_string(j) + " sets"};
        }
        if (!encoded && nsets_before < s.W && s.nsets >= s.W) characterize(s, n);
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    HBM_HIP(hipEventRecord(e1, c.stream));
    HBM_HIP(hipEventSynchronize(e1));
    float ms = 0;
    HBM_HIP(hipEventElapsedTime(&ms, e0, e1));
    c.t_sample += ms;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
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
    const bool huff = s.enc == HBM_ENC_HUFFMAN || s.enc == HBM_ENC_HUFFMAN_HOT_BITMAP;
    o->index_bytes = s.nsets ? (s.nsets + 1) * 8 : 0;
    o->bitmap_bytes = s.bm_words * (int64_t)s.nhot * 8;
    o->raw_bytes = huff ? 0 : s.raw_count * 4;
    o->codebook_bytes = huff ? (int64_t)c.g.n + (int64_t)s.cb.nsym * 4 + 68 * 8 : 0;
    if (s.nhot) o->codebook_bytes += (int64_t)s.nhot * 4;
    o->store_bytes = store_bytes(c);
    o->skewness = s.skew;
    o->density = s.density;
    // total members = sum of the histogram
    if (s.hist.p && s.nsets) {
        std::vector<uint32_t> h(c.g.n);
        HBM_HIP(hipMemcpyAsync(h.data(), s.hist.p, (size_t)c.g.n * 4, hipMemcpyDeviceToHost, c.stream));
        HBM_HIP(hipStreamSynchronize(c.stream));
        int64_t t = 0;
        for (uint32_t x : h) t += x;
        o->members = t;
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
