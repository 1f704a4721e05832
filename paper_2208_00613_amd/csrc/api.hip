// api.hip -- the C ABI (include/hbmax.h) and the IMM driver.
#include <chrono>
#include <cmath>
#include <cstring>

#include "hbm_imm.h"

using hbm::Ctx;
using hbm::Error;

namespace {

template <class F>
hbm_status guard(hbm_ctx *ctx, F &&f) {
    if (!ctx) return HBM_EINVAL;
    ctx->c.last_error.clear();
    try {
        hipError_t e = hipSetDevice(ctx->c.device);
        if (e != hipSuccess) throw Error{HBM_EDEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e)};
        f(ctx->c);
        return HBM_OK;
    } catch (const Error &e) {
        ctx->c.last_error = e.msg;
        return e.st;
    } catch (const std::bad_alloc &) {
        ctx->c.last_error = "host allocation failed";
        return HBM_ENOMEM;
    } catch (const std::exception &e) {
        ctx->c.last_error = e.what();
        return HBM_EDEVICE;
    }
}

}  // namespace

extern "C" {

const char *hbm_version(void) { return "hbmax-gfx950 0.1"; }

hbm_status hbm_create(hbm_ctx **out, int device, void *stream, const hbm_allocator *alloc) {
    if (!out) return HBM_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return HBM_EDEVICE;
    if (device < 0 || device >= ndev) return HBM_EINVAL;
    if (alloc && (!alloc->alloc || !alloc->release)) return HBM_EINVAL;
    hbm_ctx *ctx = new (std::nothrow) hbm_ctx;
    if (!ctx) return HBM_ENOMEM;
    ctx->c.device = device;
    ctx->c.stream = (hipStream_t)stream;
    if (alloc) {
        ctx->c.alloc = *alloc;
        ctx->c.has_alloc = true;
    }
    if (hipSetDevice(device) != hipSuccess) {
        delete ctx;
        return HBM_EDEVICE;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        ctx->c.num_cus = prop.multiProcessorCount;
    hbm::noalloc_setup(device);  // device address of the fixed selection scratch, once per device
    *out = ctx;
    return HBM_OK;
}

void hbm_destroy(hbm_ctx *ctx) {
    if (!ctx) return;
    try {
        (void)hipSetDevice(ctx->c.device);
        (void)hipStreamSynchronize(ctx->c.stream);
        hbm::select_free(ctx->c);
        hbm::store_free(ctx->c);
        hbm::graph_free(ctx->c);
        for (hbm::Buf *b : {&ctx->c.scan_tmp, &ctx->c.ctrl_arena, &ctx->c.tails, &ctx->c.bkeys,
                            &ctx->c.dctr, &ctx->c.xmeta, &ctx->c.pfind, &ctx->c.spill0, &ctx->c.spill,
                            &ctx->c.spill2})
            hbm::buf_free(ctx->c, *b);
        hbm::stage_free(ctx->c);
    } catch (...) {
    }
    delete ctx;
}

const char *hbm_last_error(const hbm_ctx *ctx) { return ctx ? ctx->c.last_error.c_str() : "null context"; }

hbm_status hbm_set_budget(hbm_ctx *ctx, int64_t bytes) {
    return guard(ctx, [&](Ctx &c) {
        HBM_REQUIRE(bytes >= 0, HBM_EINVAL, "budget must be >= 0");
        c.budget = bytes;
    });
}

// The Huffman decode tables pack a vertex id and a code length into one 32-bit word
// (id << 5 | length), so Huffman encodings take graphs of fewer than 2^27 vertices.
static bool huff_enc(int enc) { return hbm::enc_huff(enc) || enc == HBM_ENC_AUTO; }
constexpr int32_t HUFF_MAX_N = 1 << 27;

hbm_status hbm_load_graph(hbm_ctx *ctx, int32_t n, int64_t m, const int64_t *row_ptr, const int32_t *dst,
                          const float *w, hbm_model model, hbm_prob prob) {
    return guard(ctx, [&](Ctx &c) {
        HBM_REQUIRE(!(huff_enc(c.s.enc_req) && n >= HUFF_MAX_N), HBM_EINVAL,
                    "Huffman encodings need n < 2^27 (decode tables pack id << 5 | length)");
        hbm::graph_load(c, n, m, row_ptr, dst, w, (int)model, (int)prob);
    });
}

hbm_status hbm_set_encoding(hbm_ctx *ctx, hbm_enc enc, double warmup_frac, double hot_frac) {
    return guard(ctx, [&](Ctx &c) {
        HBM_REQUIRE(enc >= HBM_ENC_NONE && enc <= HBM_ENC_AUTO, HBM_EINVAL, "unknown encoding");
        if (enc != HBM_ENC_NONE)
            HBM_REQUIRE(warmup_frac > 0.0 && warmup_frac <= 1.0, HBM_EINVAL, "warmup_frac must be in (0, 1]");
        if (enc == HBM_ENC_HOT_BITMAP || enc == HBM_ENC_HUFFMAN_HOT_BITMAP)
            HBM_REQUIRE(hot_frac > 0.0 && hot_frac <= 1.0, HBM_EINVAL, "hot_frac must be in (0, 1]");
        HBM_REQUIRE(!(huff_enc((int)enc) && c.g.loaded && c.g.n >= HUFF_MAX_N), HBM_EINVAL,
                    "Huffman encodings need n < 2^27 (decode tables pack id << 5 | length)");
        c.s.enc_req = (int)enc;
        hbm::store_reset(c);
        c.s.warmup_frac = warmup_frac > 0.0 ? warmup_frac : 0.1;
        c.s.hot_frac = hot_frac;
    });
}

hbm_status hbm_set_implicit_roots(hbm_ctx *ctx, int32_t on) {
    return guard(ctx, [&](Ctx &c) {
        HBM_REQUIRE(on == 0 || on == 1, HBM_EINVAL, "on must be 0 or 1");
        hbm::store_reset(c);
        c.s.implicit_roots = on != 0;
    });
}

hbm_status hbm_set_row_containers(hbm_ctx *ctx, int32_t on) {
    return guard(ctx, [&](Ctx &c) {
        HBM_REQUIRE(on == 0 || on == 1, HBM_EINVAL, "on must be 0 or 1");
        hbm::store_reset(c);
        c.s.containers = on != 0;
    });
}

hbm_status hbm_set_spill(hbm_ctx *ctx, int64_t device_bytes) {
    return guard(ctx, [&](Ctx &c) {
        HBM_REQUIRE(device_bytes >= 0, HBM_EINVAL, "device_bytes must be >= 0");
        HBM_REQUIRE(device_bytes == 0 || device_bytes >= 16, HBM_EINVAL, "device_bytes must be 0 or >= 16");
        hbm::store_reset(c);
        c.s.spill_cap = device_bytes;
    });
}

hbm_status hbm_set_hot_density(hbm_ctx *ctx, double min_density) {
    return guard(ctx, [&](Ctx &c) {
        HBM_REQUIRE(min_density >= 0.0 && min_density <= 1.0, HBM_EINVAL, "min_density must be in [0, 1]");
        hbm::store_reset(c);
        c.s.hot_min_density = min_density;
    });
}

hbm_status hbm_sample_rr(hbm_ctx *ctx, int64_t theta, uint64_t seed) {
    return guard(ctx, [&](Ctx &c) { hbm::store_extend(c, theta, seed); });
}

hbm_status hbm_select_seeds(hbm_ctx *ctx, int32_t k, int32_t *seeds, uint64_t *gains, uint64_t *coverage) {
    return guard(ctx, [&](Ctx &c) {
        HBM_REQUIRE(seeds && gains && coverage, HBM_EINVAL, "null output");
        HBM_REQUIRE(c.g.loaded, HBM_ESTATE, "no graph loaded");
        HBM_REQUIRE(k >= 1 && k <= c.g.n, HBM_EINVAL, "k must be in [1, n]");
        std::vector<int32_t> s((size_t)k);
        std::vector<uint64_t> g((size_t)k);
        uint64_t cov = 0;
        hbm::select_seeds(c, k, s.data(), g.data(), &cov);
        std::memcpy(seeds, s.data(), (size_t)k * 4);
        std::memcpy(gains, g.data(), (size_t)k * 8);
        *coverage = cov;
    });
}

hbm_status hbm_get_memory(hbm_ctx *ctx, int64_t *bytes_now, int64_t *bytes_peak, int32_t reset_peak) {
    return guard(ctx, [&](Ctx &c) {
        HBM_REQUIRE(bytes_now && bytes_peak, HBM_EINVAL, "null output");
        *bytes_now = c.mem_now;
        *bytes_peak = c.mem_peak;
        if (reset_peak) c.mem_peak = c.mem_now;
    });
}

hbm_status hbm_bench_philox(hbm_ctx *ctx, int64_t calls_per_thread, int32_t blocks, double *ms, uint32_t *checksum) {
    return guard(ctx, [&](Ctx &c) {
        HBM_REQUIRE(ms && checksum, HBM_EINVAL, "null output");
        uint32_t sum = 0;
        const double t = hbm::philox_probe(c, calls_per_thread, blocks, &sum);
        *ms = t;
        *checksum = sum;
    });
}

hbm_status hbm_select_seeds_noalloc(hbm_ctx *ctx, int32_t k, int32_t *seeds, uint64_t *gains, uint64_t *coverage) {
    return guard(ctx, [&](Ctx &c) {
        HBM_REQUIRE(seeds && gains && coverage, HBM_EINVAL, "null output");
        HBM_REQUIRE(c.g.loaded, HBM_ESTATE, "no graph loaded");
        HBM_REQUIRE(k >= 1 && k <= c.g.n, HBM_EINVAL, "k must be in [1, n]");
        std::vector<int32_t> s((size_t)k);
        std::vector<uint64_t> g((size_t)k);
        uint64_t cov = 0;
        hbm::select_seeds_noalloc(c, k, s.data(), g.data(), &cov);
        std::memcpy(seeds, s.data(), (size_t)k * 4);
        std::memcpy(gains, g.data(), (size_t)k * 8);
        *coverage = cov;
    });
}

hbm_status hbm_imm(hbm_ctx *ctx, int32_t k, double eps, double l, uint64_t seed, int32_t *seeds, uint64_t *gains,
                   hbm_imm_stats *stats) {
    return guard(ctx, [&](Ctx &c) {
        HBM_REQUIRE(seeds, HBM_EINVAL, "null seeds");
        hbm::ImmJob J;
        J.c = &c;
        J.k = k;
        J.eps = eps;
        J.l = l;
        J.seed = seed;
        hbm::imm_run(c, {&J});
        if (J.phase == hbm::ImmJob::FAILED) throw Error{J.status, J.error};
        std::memcpy(seeds, J.seeds.data(), (size_t)k * 4);
        if (gains) std::memcpy(gains, J.gains.data(), (size_t)k * 8);
        if (stats) *stats = J.st;
    });
}

}  // extern "C"

namespace {

// Checks shared by the batched calls: distinct contexts on one device.
bool batch_ok(hbm_ctx *const *ctxs, int32_t count) {
    if (!ctxs || count < 1) return false;
    for (int32_t i = 0; i < count; i++) {
        if (!ctxs[i]) return false;
        for (int32_t j = 0; j < i; j++)
            if (ctxs[j] == ctxs[i]) return false;
        if (ctxs[i]->c.device != ctxs[0]->c.device) return false;
    }
    return true;
}

// IMM for every instance at once on ctxs[0]'s stream (ordered after each context's own
// stream), leaving the jobs' outcomes in J.  Device errors throw.
void run_batch(hbm_ctx *const *ctxs, int32_t count, const hbm_query *queries, std::vector<hbm::ImmJob> &J) {
    Ctx &r = ctxs[0]->c;
    std::vector<hipStream_t> own((size_t)count);
    hipEvent_t ev;
    HBM_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    for (int32_t i = 0; i < count; i++) {
        Ctx &c = ctxs[i]->c;
        own[(size_t)i] = c.stream;
        if (c.stream != r.stream) {
            HBM_HIP(hipEventRecord(ev, c.stream));
            HBM_HIP(hipStreamWaitEvent(r.stream, ev, 0));
        }
    }
    (void)hipEventDestroy(ev);
    for (int32_t i = 0; i < count; i++) ctxs[i]->c.stream = r.stream;
    J.assign((size_t)count, hbm::ImmJob{});
    std::vector<hbm::ImmJob *> jp;
    for (int32_t i = 0; i < count; i++) {
        hbm::ImmJob &j = J[(size_t)i];
        j.c = &ctxs[i]->c;
        j.k = queries[i].k;
        j.eps = queries[i].eps;
        j.l = queries[i].l;
        j.seed = queries[i].seed;
        jp.push_back(&j);
    }
    try {
        hbm::imm_run(r, jp);
        HBM_HIP(hipStreamSynchronize(r.stream));
    } catch (...) {
        for (int32_t i = 0; i < count; i++) ctxs[i]->c.stream = own[(size_t)i];
        throw;
    }
    for (int32_t i = 0; i < count; i++) ctxs[i]->c.stream = own[(size_t)i];
}

void set_tuning(Ctx &c, hbm_tune_key key, int64_t value);
int64_t get_tuning(const Ctx &c, hbm_tune_key key);

}  // namespace

extern "C" {

hbm_status hbm_imm_batch(hbm_ctx *const *ctxs, int32_t count, const hbm_query *queries, int32_t *const *seeds,
                         uint64_t *const *gains, hbm_imm_stats *stats, hbm_status *status) {
    if (!batch_ok(ctxs, count) || !queries || !seeds) return HBM_EINVAL;
    for (int32_t i = 0; i < count; i++)
        if (!seeds[i]) return HBM_EINVAL;
    std::vector<hbm::ImmJob> J;
    const hbm_status rc = guard(ctxs[0], [&](Ctx &) { run_batch(ctxs, count, queries, J); });
    if (rc != HBM_OK) {
        if (status)
            for (int32_t i = 0; i < count; i++) status[i] = rc;
        return rc;
    }
    hbm_status first = HBM_OK;
    for (int32_t i = 0; i < count; i++) {
        const hbm::ImmJob &j = J[(size_t)i];
        const hbm_status s = j.phase == hbm::ImmJob::DONE ? HBM_OK : j.status;
        if (status) status[i] = s;
        if (s != HBM_OK) {
            ctxs[i]->c.last_error = j.error;
            if (first == HBM_OK) first = s;
            continue;
        }
        std::memcpy(seeds[i], j.seeds.data(), j.seeds.size() * 4);
        if (gains && gains[i]) std::memcpy(gains[i], j.gains.data(), j.gains.size() * 8);
        if (stats) stats[i] = j.st;
    }
    return first;
}

hbm_status hbm_autotune(hbm_ctx *const *ctxs, int32_t count, const hbm_query *queries, int64_t *chosen,
                        double *best_ms) {
    if (!batch_ok(ctxs, count) || !queries) return HBM_EINVAL;
    return guard(ctxs[0], [&](Ctx &r) {
        bool ic = false, lt = false;
        for (int32_t i = 0; i < count; i++) {
            HBM_REQUIRE(ctxs[i]->c.g.loaded, HBM_ESTATE, "no graph loaded");
            (ctxs[i]->c.g.model == HBM_IC ? ic : lt) = true;
        }
        auto apply = [&](hbm_tune_key key, int64_t v) {
            for (int32_t i = 0; i < count; i++) set_tuning(ctxs[i]->c, key, v);
        };
        std::vector<hbm::ImmJob> J;
        auto timed = [&]() {
            const auto t0 = std::chrono::steady_clock::now();
            run_batch(ctxs, count, queries, J);
            for (const hbm::ImmJob &j : J)
                if (j.phase != hbm::ImmJob::DONE) throw Error{j.status, "autotune probe: " + j.error};
            return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        };
        struct Axis {
            hbm_tune_key key;
            std::vector<int64_t> values;
            bool used;
        };
        const std::vector<Axis> axes = {
            {HBM_TUNE_BLOCK_SETS, {int64_t(1) << 16, int64_t(1) << 18, int64_t(1) << 21}, true},
            {HBM_TUNE_IC_T1_BUDGET, {1024, 4096, 16384}, ic},
            {HBM_TUNE_T2_SLOTS, {2, 3, 4}, true},
            {HBM_TUNE_LDS_THREADS, {512, 1024}, ic},
            {HBM_TUNE_LDS_PER_CU, {2, 3}, ic},
            {HBM_TUNE_LT_PATH, {32, 64, 128}, lt},
        };
        timed();  // warm-up: allocations at the current settings
        double best = timed();
        // coordinate descent, one key at a time, keeping the best value of each
        for (const Axis &ax : axes) {
            if (!ax.used) continue;
            int64_t keep = get_tuning(r, ax.key);
            for (int64_t v : ax.values) {
                if (v == keep) continue;
                apply(ax.key, v);
                timed();  // the first run at a new shape may allocate
                const double ms = timed();
                if (ms < best) {
                    best = ms;
                    keep = v;
                }
            }
            apply(ax.key, keep);
        }
        if (chosen)
            for (int k = 0; k < HBM_TUNE_COUNT; k++) chosen[k] = get_tuning(r, (hbm_tune_key)k);
        if (best_ms) *best_ms = best;
    });
}

hbm_status hbm_set_tuning(hbm_ctx *ctx, hbm_tune_key key, int64_t value) {
    return guard(ctx, [&](Ctx &c) { set_tuning(c, key, value); });
}

hbm_status hbm_profile(hbm_ctx *ctx, int32_t enable) {
    return guard(ctx, [&](Ctx &c) {
        hbm::prof_flush(c);
        c.prof.on = enable != 0;
        if (enable) c.prof.stats.clear();
        if (c.dctr.p) hbm::buf_zero(c, c.dctr, 0, hbm::DC_COUNT * 8);
    });
}

hbm_status hbm_profile_read(hbm_ctx *ctx, hbm_kernel_stat *out, int32_t cap, int32_t *count) {
    return guard(ctx, [&](Ctx &c) {
        HBM_REQUIRE(count, HBM_EINVAL, "null count");
        hbm::prof_flush(c);
        const auto &S = c.prof.stats;
        *count = (int32_t)S.size();
        for (int32_t i = 0; i < cap && i < (int32_t)S.size(); i++) {
            hbm_kernel_stat &o = out[i];
            std::memset(o.name, 0, sizeof(o.name));
            std::strncpy(o.name, S[(size_t)i].name.c_str(), sizeof(o.name) - 1);
            o.launches = S[(size_t)i].launches;
            o.total_ms = S[(size_t)i].ms;
            o.alg_bytes = S[(size_t)i].bytes;
            o.alg_ops = S[(size_t)i].ops;
        }
    });
}

hbm_status hbm_get_rr(hbm_ctx *ctx, int64_t j, int32_t *buf, int64_t cap, int64_t *len) {
    return guard(ctx, [&](Ctx &c) {
        HBM_REQUIRE(len, HBM_EINVAL, "null len");
        HBM_REQUIRE(j >= 0 && j < c.s.nsets, HBM_EINVAL, "set index out of range");
        std::vector<int64_t> off;
        std::vector<int32_t> mem;
        hbm::store_dump(c, j, j + 1, off, mem);
        *len = (int64_t)mem.size();
        HBM_REQUIRE((int64_t)mem.size() <= cap && (buf || mem.empty()), HBM_EINVAL, "buffer too small");
        if (!mem.empty()) std::memcpy(buf, mem.data(), mem.size() * 4);
    });
}

hbm_status hbm_dump_sets(hbm_ctx *ctx, int64_t j0, int64_t j1, int64_t *off, int32_t *mem, int64_t cap,
                         int64_t *total) {
    return guard(ctx, [&](Ctx &c) {
        HBM_REQUIRE(off && total, HBM_EINVAL, "null output");
        HBM_REQUIRE(0 <= j0 && j0 <= j1 && j1 <= c.s.nsets, HBM_EINVAL, "range out of bounds");
        std::vector<int64_t> o;
        std::vector<int32_t> m;
        hbm::store_dump(c, j0, j1, o, m);
        *total = (int64_t)m.size();
        HBM_REQUIRE((int64_t)m.size() <= cap && (mem || m.empty()), HBM_EINVAL, "buffer too small");
        std::memcpy(off, o.data(), o.size() * 8);
        if (!m.empty()) std::memcpy(mem, m.data(), m.size() * 4);
    });
}

hbm_status hbm_get_store_stats(hbm_ctx *ctx, hbm_store_stats *out) {
    return guard(ctx, [&](Ctx &c) {
        HBM_REQUIRE(out, HBM_EINVAL, "null output");
        hbm::store_stats(c, out);
    });
}

hbm_status hbm_export(hbm_ctx *ctx, hbm_array what, void *host_out, int64_t cap_bytes, int64_t *bytes) {
    return guard(ctx, [&](Ctx &c) {
        HBM_REQUIRE(bytes, HBM_EINVAL, "null bytes");
        const hbm::Store &s = c.s;
        const bool huff = hbm::enc_huff(s.enc), raw = hbm::enc_raw(s.enc);
        const void *src = nullptr;
        int64_t nb = 0;
        const int64_t n = c.g.n, T = s.nsets;
        switch (what) {
            case HBM_A_IN_PTR: src = c.g.in_ptr.p; nb = c.g.loaded ? (n + 1) * 8 : 0; break;
            case HBM_A_IN_SRC: src = c.g.in_src.p; nb = c.g.m * 4; break;
            case HBM_A_THRESH:
                src = c.g.thr.p;
                nb = (c.g.model == HBM_IC && c.g.prob == HBM_PROB_WC) ? n * 4 : c.g.m * 4;
                break;
            case HBM_A_COUNTS: src = s.hist.p; nb = s.hist.p ? n * 4 : 0; break;
            case HBM_A_WARM: src = s.warm.p; nb = (s.warm.p && s.model_ready) ? n * 4 : 0; break;
            case HBM_A_HOT: src = s.hot.p; nb = (int64_t)s.nhot * 4; break;
            case HBM_A_BITMAP: src = s.bitmap.p; nb = s.nhot ? ((T + 63) / 64) * s.nhot * 8 : 0; break;
            case HBM_A_RAW_OFF: src = s.raw_off.p; nb = (raw && T) ? (T + 1) * 8 : 0; break;
            case HBM_A_RAW_MEM: src = s.raw_mem.p; nb = (raw && T) ? s.raw_count * 4 : 0; break;
            case HBM_A_LENS: src = s.lens.p; nb = (huff && s.model_ready) ? n : 0; break;
            case HBM_A_CODES: src = s.codes.p; nb = (huff && s.model_ready) ? n * 4 : 0; break;
            case HBM_A_BITOFF: src = s.bitoff.p; nb = (huff && T) ? (T + 1) * 8 : 0; break;
            case HBM_A_PAYLOAD: src = s.payload.p; nb = (huff && T) ? (int64_t)((s.nbits + 31) / 32) * 4 : 0; break;
            case HBM_A_ARR_HOT: src = s.ar_hot.p; nb = (int64_t)s.nar * 4; break;
            case HBM_A_ARR_OFF: src = s.ar_off.p; nb = s.nar ? s.ar_chunks * (int64_t)(s.nar + 1) * 8 : 0; break;
            case HBM_A_ARR_LOW: src = s.ar_low.p; nb = s.nar ? s.ar_entries * 2 : 0; break;
            default: throw Error{HBM_EINVAL, "unknown array"};
        }
        *bytes = nb;
        HBM_REQUIRE(nb <= cap_bytes, HBM_EINVAL, "buffer too small");
        if (nb > 0) {
            HBM_REQUIRE(src && host_out, HBM_EINVAL, "array not present");
            int64_t dev_nb = nb;
            if (what == HBM_A_RAW_MEM && s.raw_split < s.raw_count) dev_nb = s.raw_split * 4;  // spilled
            HBM_HIP(hipMemcpyAsync(host_out, src, (size_t)dev_nb, hipMemcpyDeviceToHost, c.stream));
            HBM_HIP(hipStreamSynchronize(c.stream));
            if (dev_nb < nb) std::memcpy((char *)host_out + dev_nb, s.raw_host_h, (size_t)(nb - dev_nb));
        }
    });
}

}  // extern "C"

namespace {

void set_tuning(Ctx &c, hbm_tune_key key, int64_t value) {
    switch (key) {
        case HBM_TUNE_IC_TIER1:
            HBM_REQUIRE(value == 0 || value == 1, HBM_EINVAL, "IC_TIER1 must be 0 or 1");
            c.ic_tier1 = (int)value;
            break;
        case HBM_TUNE_IC_T1_BUDGET:
            HBM_REQUIRE(value >= 0, HBM_EINVAL, "IC_T1_BUDGET must be >= 0");
            c.ic_t1_budget = value;
            break;
        case HBM_TUNE_LT_PATH:
            HBM_REQUIRE(value == 32 || value == 64 || value == 128 || value == 256, HBM_EINVAL,
                        "LT_PATH must be 32, 64, 128 or 256");
            c.lt_lw = (int)value;
            break;
        case HBM_TUNE_T2_QUEUE:
            HBM_REQUIRE(value >= 64 && value <= (int64_t(1) << 31), HBM_EINVAL, "T2_QUEUE out of range");
            if (value != c.t2_queue) {
                c.t2_queue = value;
                // reallocated at the next use with the new queue size
                hbm::buf_free(c, c.sc.t2_bitmap);
                hbm::buf_free(c, c.sc.t2_queue);
                c.sc.t2_slots = 0;
            }
            break;
        case HBM_TUNE_T2_SLOTS:
            HBM_REQUIRE(value >= 1 && value <= 4, HBM_EINVAL, "T2_SLOTS must be in [1, 4]");
            if (value != c.t2_per_cu) {
                c.t2_per_cu = (int)value;
                hbm::buf_free(c, c.sc.t2_bitmap);
                hbm::buf_free(c, c.sc.t2_queue);
                c.sc.t2_slots = 0;
            }
            break;
        case HBM_TUNE_LDS_THREADS:
            HBM_REQUIRE(value == 0 || value == 512 || value == 1024, HBM_EINVAL, "LDS_THREADS must be 0, 512 or 1024");
            c.lds_threads = (int)value;
            break;
        case HBM_TUNE_LDS_PER_CU:
            HBM_REQUIRE(value >= 0 && value <= 4, HBM_EINVAL, "LDS_PER_CU must be in [0, 4]");
            c.lds_per_cu = (int)value;
            break;
        case HBM_TUNE_SPARSE_COUNTS:
            HBM_REQUIRE(value >= 0 && value <= 2, HBM_EINVAL, "SPARSE_COUNTS must be 0, 1 or 2");
            c.sparse_counts = (int)value;
            break;
        case HBM_TUNE_SELECT_GRAPH:
            HBM_REQUIRE(value == 0 || value == 1, HBM_EINVAL, "SELECT_GRAPH must be 0 or 1");
            c.select_graph = (int)value;
            break;
        case HBM_TUNE_BLOCK_SETS:
            HBM_REQUIRE(value >= 1024 && value <= (int64_t(1) << 26), HBM_EINVAL, "BLOCK_SETS out of range");
            c.block_sets = value;
            break;
        case HBM_TUNE_SPILL_SLOTS:
            HBM_REQUIRE(value >= 0 && value <= 4096, HBM_EINVAL, "SPILL_SLOTS must be in [0, 4096]");
            c.spill_slots = value;
            break;
        case HBM_TUNE_LDS_SMALL:
            HBM_REQUIRE(value >= 0 && value <= 2, HBM_EINVAL, "LDS_SMALL must be 0, 1 or 2");
            c.lds_small = (int)value;
            break;
        default:
            throw Error{HBM_EINVAL, "unknown tuning key"};
    }
}

int64_t get_tuning(const Ctx &c, hbm_tune_key key) {
    switch (key) {
        case HBM_TUNE_IC_TIER1: return c.ic_tier1;
        case HBM_TUNE_IC_T1_BUDGET: return c.ic_t1_budget;
        case HBM_TUNE_BLOCK_SETS: return c.block_sets;
        case HBM_TUNE_LT_PATH: return c.lt_lw;
        case HBM_TUNE_T2_QUEUE: return c.t2_queue;
        case HBM_TUNE_T2_SLOTS: return c.t2_per_cu;
        case HBM_TUNE_LDS_THREADS: return c.lds_threads;
        case HBM_TUNE_LDS_PER_CU: return c.lds_per_cu;
        case HBM_TUNE_SPARSE_COUNTS: return c.sparse_counts;
        case HBM_TUNE_SELECT_GRAPH: return c.select_graph;
        case HBM_TUNE_SPILL_SLOTS: return c.spill_slots;
        case HBM_TUNE_LDS_SMALL: return c.lds_small;
        default: return -1;
    }
}

}  // namespace
