// graph.hip -- ingest of G = (V, E, w): validation, transpose, live thresholds.
//
// The RR-set definition (Background section) reverses every edge, so sampling
// walks the in-edges of each vertex.  In-edges of v are ordered by ascending
// source; an edge's id is its position in that order (the Philox counter of an
// IC coin is derived from it).  A coin or LT draw is a 24-bit integer r, and
// "r / 2^24 < p" is decided exactly as "r < ceil(p * 2^24)" with p * 2^24
// formed in float32, so every threshold is stored as that integer.
#include <rocprim/device/device_radix_sort.hpp>

#include "hbm_device.h"
#include "hbm_internal.h"

namespace hbm {

enum : uint32_t {
    BAD_ROWPTR = 1u,
    BAD_DST = 2u,
    SELF_LOOP = 4u,
    BAD_W = 8u,
    IC_W_ABOVE_1 = 16u,
    DUPLICATE = 32u,
    LT_SUM = 64u
};

__global__ void k_check_rowptr(const int64_t *__restrict__ rp, int32_t n, int64_t m, uint32_t *flags) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i <= n; i += (int64_t)gridDim.x * blockDim.x) {
        bool bad = false;
        if (i == 0 && rp[0] != 0) bad = true;
        if (i == n && rp[n] != m) bad = true;
        if (i < n && rp[i] > rp[i + 1]) bad = true;
        if (rp[i] < 0 || rp[i] > m) bad = true;
        if (bad) atomicOr(flags, BAD_ROWPTR);
    }
}

// Source of every forward edge (binary search in row_ptr) and per-edge checks.
__global__ void k_expand(const int64_t *__restrict__ rp, const int32_t *__restrict__ dst, const float *__restrict__ w,
                         int32_t n, int64_t m, int ic_edge, uint32_t *__restrict__ src, uint32_t *__restrict__ key,
                         uint32_t *__restrict__ val, uint32_t *flags) {
    uint32_t f_local = 0;
    for (int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; f < m; f += (int64_t)gridDim.x * blockDim.x) {
        int64_t u = upper_bound_dev<int64_t, int64_t>(rp, 0, (int64_t)n + 1, f) - 1;
        int32_t v = dst[f];
        if (v < 0 || v >= n) f_local |= BAD_DST;
        if (v == u) f_local |= SELF_LOOP;
        if (w) {
            float x = w[f];
            if (!(x >= 0.0f)) f_local |= BAD_W;  // NaN or negative
            if (ic_edge && x > 1.0f) f_local |= IC_W_ABOVE_1;
        }
        src[f] = (uint32_t)u;
        key[f] = (uint32_t)(v < 0 || v >= n ? 0 : v);
        val[f] = (uint32_t)f;
    }
    if (f_local) atomicOr(flags, f_local);
}

// in_ptr[v] = first position of key v in the sorted keys
__global__ void k_inptr(const uint32_t *__restrict__ keys, int64_t m, int32_t n, int64_t *__restrict__ in_ptr) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v <= n; v += (int64_t)gridDim.x * blockDim.x) {
        int64_t lo = 0, hi = m;
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if ((int64_t)keys[mid] < v) lo = mid + 1;
            else hi = mid;
        }
        in_ptr[v] = lo;
    }
}

__global__ void k_gather(const uint32_t *__restrict__ vals, const uint32_t *__restrict__ keys,
                         const uint32_t *__restrict__ src, const float *__restrict__ w, int64_t m,
                         int32_t *__restrict__ in_src, float *__restrict__ w_in, uint32_t *flags) {
    uint32_t f_local = 0;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
        uint32_t f = vals[e];
        uint32_t s = src[f];
        in_src[e] = (int32_t)s;
        if (w_in) w_in[e] = w[f];
        // stable sort by target keeps sources ascending inside a row: equal neighbours are duplicates
        if (e > 0 && keys[e - 1] == keys[e] && src[vals[e - 1]] == s) f_local |= DUPLICATE;
    }
    if (f_local) atomicOr(flags, f_local);
}

__device__ __forceinline__ uint32_t thr_of(float p) {
    // p * 2^24 is exact in float32; an integer r < that value iff r < its ceiling
    float t = p * 16777216.0f;
    return (uint32_t)ceilf(t);
}

__global__ void k_thr_edge(const float *__restrict__ w_in, int64_t m, uint32_t *__restrict__ thr) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x)
        thr[e] = thr_of(w_in[e]);
}

__global__ void k_thr_wc(const int64_t *__restrict__ in_ptr, int32_t n, uint32_t *__restrict__ thr) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        int64_t d = in_ptr[v + 1] - in_ptr[v];
        thr[v] = d > 0 ? thr_of(__fdiv_rn(1.0f, (float)d)) : 0u;
    }
}

// LT: running float32 sum of in-weights along each row, added left to right
__global__ void k_thr_lt(const int64_t *__restrict__ in_ptr, const float *__restrict__ w_in, int32_t n, int wc,
                         uint32_t *__restrict__ thr, uint32_t *flags) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        int64_t e0 = in_ptr[v], e1 = in_ptr[v + 1];
        // 1 + 2^-20, plus what float32 left-to-right accumulation of d terms can add (d * 2^-23)
        const double limit = 1.0 + 9.5367431640625e-07 + (double)(e1 - e0) * 1.1920928955078125e-07;
        float p = wc && e1 > e0 ? __fdiv_rn(1.0f, (float)(e1 - e0)) : 0.0f;
        float acc = 0.0f;
        for (int64_t e = e0; e < e1; e++) {
            acc = __fadd_rn(acc, wc ? p : w_in[e]);
            thr[e] = thr_of(acc);
        }
        if (!wc && (double)acc > limit) atomicOr(flags, LT_SUM);  // WC sums are 1 up to float32 rounding
    }
}

// LT guide table (cut-point search): row v with d in-edges gets B = 2^ceil(log2 d) buckets
// stored at [2 * in_ptr[v], 2 * in_ptr[v] + B).  Bucket k holds the first in-edge whose
// threshold exceeds k * 2^24 / B, so the first edge with threshold > r is found by a
// forward scan from bucket r * B / 2^24 -- the same edge a binary search would find.
__global__ void k_guide_lt(const int64_t *__restrict__ in_ptr, const uint32_t *__restrict__ thr, int32_t n,
                           uint32_t *__restrict__ guide) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t e0 = (uint32_t)in_ptr[v], e1 = (uint32_t)in_ptr[v + 1];
        if (e1 == e0) continue;
        const uint32_t d = e1 - e0;
        const uint32_t lb = d > 1 ? min(32 - __clz(d - 1), 24) : 0;
        const uint32_t B = 1u << lb;
        uint32_t e = e0;
        uint32_t *G = guide + 2 * (uint64_t)e0;
        for (uint32_t k = 0; k < B; k++) {
            const uint32_t lo = k << (24 - lb);
            while (e < e1 && thr[e] <= lo) e++;
            G[k] = e;
        }
    }
}

static std::string flag_text(uint32_t f) {
    std::string s;
    if (f & BAD_ROWPTR) s += "row_ptr malformed; ";
    if (f & BAD_DST) s += "target id out of range; ";
    if (f & SELF_LOOP) s += "self-loop; ";
    if (f & BAD_W) s += "weight NaN or negative; ";
    if (f & IC_W_ABOVE_1) s += "IC edge probability above 1; ";
    if (f & DUPLICATE) s += "duplicate edge; ";
    if (f & LT_SUM) s += "LT in-weights sum above 1 + 2^-20 + indeg * 2^-23; ";
    return s;
}

static uint32_t read_flags(Ctx &c, Buf &flags) {
    uint32_t f = 0;
    HBM_HIP(hipMemcpyAsync(&f, flags.p, 4, hipMemcpyDeviceToHost, c.stream));
    HBM_HIP(hipStreamSynchronize(c.stream));
    return f;
}

// One 16-byte record per in-edge e of v, {u = in_src[e], u's in-edge range, w}: w is u's WC
// threshold for IC-WC (0 for per-edge probabilities), thr[e] for LT.  An IC sampler that finds
// e live learns everything it needs to expand u from this one load, so a BFS level costs one
// dependent device load; an LT walk reads the threshold it compares, the next vertex and that
// vertex's range in one load, so a step costs the cut-point index read and this one.
__global__ void k_in_rec(const int32_t *__restrict__ in_src, const int64_t *__restrict__ in_ptr,
                         const uint32_t *__restrict__ thr_v, const uint32_t *__restrict__ thr_e, int64_t m,
                         uint4 *__restrict__ rec) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t u = (uint32_t)in_src[e];
        const uint32_t w = thr_e ? thr_e[e] : thr_v ? thr_v[u] : 0u;
        rec[e] = make_uint4(u, (uint32_t)in_ptr[u], (uint32_t)in_ptr[u + 1], w);
    }
}

void graph_free(Ctx &c) {
    if (c.g.borrowed) {
        c.g = DGraph{};
        return;
    }
    buf_free(c, c.g.in_ptr);
    buf_free(c, c.g.in_src);
    buf_free(c, c.g.thr);
    buf_free(c, c.g.guide);
    buf_free(c, c.g.in_rec);
    c.g.loaded = false;
    c.g.n = 0;
    c.g.m = 0;
}

void graph_load(Ctx &c, int32_t n, int64_t m, const int64_t *row_ptr, const int32_t *dst, const float *w, int model,
                int prob) {
    HBM_REQUIRE(n > 0, HBM_EINVAL, "n must be positive");
    HBM_REQUIRE(m >= 0 && m < (int64_t(1) << 32), HBM_EINVAL, "m must be in [0, 2^32)");
    HBM_REQUIRE(model == HBM_IC || model == HBM_LT, HBM_EINVAL, "unknown diffusion model");
    HBM_REQUIRE(prob == HBM_PROB_EDGE || prob == HBM_PROB_WC, HBM_EINVAL, "unknown probability rule");
    HBM_REQUIRE(row_ptr != nullptr, HBM_EINVAL, "row_ptr is NULL");
    HBM_REQUIRE(m == 0 || dst != nullptr, HBM_EINVAL, "dst is NULL");
    HBM_REQUIRE(prob == HBM_PROB_WC || m == 0 || w != nullptr, HBM_EINVAL, "weights required unless prob is WC");
    if (prob == HBM_PROB_WC) w = nullptr;

    store_reset(c);
    graph_free(c);
    DGraph &g = c.g;

    Buf flags, src, keys, vals, keys2, vals2, w_in, tmp;
    auto cleanup = [&]() {
        buf_free(c, flags); buf_free(c, src); buf_free(c, keys); buf_free(c, vals);
        buf_free(c, keys2); buf_free(c, vals2); buf_free(c, w_in); buf_free(c, tmp);
    };
    try {
        buf_alloc(c, flags, 4);
        buf_zero(c, flags, 0, 4);
        k_check_rowptr<<<grid_for(n + 1, 256, 4096), 256, 0, c.stream>>>(row_ptr, n, m, flags.as<uint32_t>());
        HBM_HIP(hipGetLastError());
        uint32_t f = read_flags(c, flags);
        HBM_REQUIRE(f == 0, HBM_EINVAL, flag_text(f));

        const size_t mm = (size_t)(m ? m : 1);
        buf_alloc(c, src, mm * 4);
        buf_alloc(c, keys, mm * 4);
        buf_alloc(c, vals, mm * 4);
        buf_alloc(c, keys2, mm * 4);
        buf_alloc(c, vals2, mm * 4);
        if (m > 0) {
            k_expand<<<grid_for(m, 256, 65536), 256, 0, c.stream>>>(
                row_ptr, dst, w, n, m, model == HBM_IC && prob == HBM_PROB_EDGE, src.as<uint32_t>(),
                keys.as<uint32_t>(), vals.as<uint32_t>(), flags.as<uint32_t>());
            HBM_HIP(hipGetLastError());
        }
        f = read_flags(c, flags);
        HBM_REQUIRE(f == 0, HBM_EINVAL, flag_text(f));

        unsigned end_bit = 1;
        while (end_bit < 32 && (uint64_t(1) << end_bit) < (uint64_t)n) end_bit++;
        if (m > 0) {
            size_t tbytes = 0;
            HBM_HIP(rocprim::radix_sort_pairs(nullptr, tbytes, keys.as<uint32_t>(), keys2.as<uint32_t>(),
                                              vals.as<uint32_t>(), vals2.as<uint32_t>(), (size_t)m, 0u, end_bit,
                                              c.stream));
            buf_alloc(c, tmp, tbytes);
            HBM_HIP(rocprim::radix_sort_pairs(tmp.p, tbytes, keys.as<uint32_t>(), keys2.as<uint32_t>(),
                                              vals.as<uint32_t>(), vals2.as<uint32_t>(), (size_t)m, 0u, end_bit,
                                              c.stream));
            buf_free(c, tmp);
        }
        buf_free(c, keys);
        buf_free(c, vals);

        buf_alloc(c, g.in_ptr, ((size_t)n + 1) * 8);
        buf_alloc(c, g.in_src, mm * 4);
        k_inptr<<<grid_for(n + 1, 256, 65536), 256, 0, c.stream>>>(keys2.as<uint32_t>(), m, n, g.in_ptr.as<int64_t>());
        HBM_HIP(hipGetLastError());
        if (w) buf_alloc(c, w_in, mm * 4);
        if (m > 0) {
            k_gather<<<grid_for(m, 256, 65536), 256, 0, c.stream>>>(vals2.as<uint32_t>(), keys2.as<uint32_t>(),
                                                                   src.as<uint32_t>(), w, m, g.in_src.as<int32_t>(),
                                                                   w ? w_in.as<float>() : nullptr, flags.as<uint32_t>());
            HBM_HIP(hipGetLastError());
        }
        buf_free(c, src);
        buf_free(c, keys2);
        buf_free(c, vals2);

        if (model == HBM_IC && prob == HBM_PROB_WC) {
            buf_alloc(c, g.thr, (size_t)n * 4);
            k_thr_wc<<<grid_for(n, 256, 65536), 256, 0, c.stream>>>(g.in_ptr.as<int64_t>(), n, g.thr.as<uint32_t>());
        } else if (model == HBM_IC) {
            // padded to whole groups of four: the sampler loads thresholds four at a time
            buf_alloc(c, g.thr, ((mm + 3) / 4 + 1) * 16);
            if (m > 0)
                k_thr_edge<<<grid_for(m, 256, 65536), 256, 0, c.stream>>>(w_in.as<float>(), m, g.thr.as<uint32_t>());
        } else {
            buf_alloc(c, g.thr, mm * 4);
            k_thr_lt<<<grid_for(n, 64, 65536), 64, 0, c.stream>>>(g.in_ptr.as<int64_t>(),
                                                                   w ? w_in.as<float>() : nullptr, n,
                                                                   prob == HBM_PROB_WC, g.thr.as<uint32_t>(),
                                                                   flags.as<uint32_t>());
        }
        HBM_HIP(hipGetLastError());
        f = read_flags(c, flags);
        HBM_REQUIRE(f == 0, HBM_EINVAL, flag_text(f));
        buf_alloc(c, g.in_rec, mm * 16);
        if (m > 0)
            k_in_rec<<<grid_for(m, 256, 65536), 256, 0, c.stream>>>(
                g.in_src.as<int32_t>(), g.in_ptr.as<int64_t>(),
                model == HBM_IC && prob == HBM_PROB_WC ? g.thr.as<uint32_t>() : nullptr,
                model == HBM_LT ? g.thr.as<uint32_t>() : nullptr, m, g.in_rec.as<uint4>());
        HBM_HIP(hipGetLastError());
        if (model == HBM_LT) {
            buf_alloc(c, g.guide, mm * 8);
            k_guide_lt<<<grid_for(n, 64, 65536), 64, 0, c.stream>>>(g.in_ptr.as<int64_t>(), g.thr.as<uint32_t>(), n,
                                                                    g.guide.as<uint32_t>());
            HBM_HIP(hipGetLastError());
        }
        cleanup();
    } catch (...) {
        cleanup();
        graph_free(c);
        throw;
    }
    g.n = n;
    g.m = m;
    g.model = model;
    g.prob = prob;
    g.loaded = true;
}

}  // namespace hbm
