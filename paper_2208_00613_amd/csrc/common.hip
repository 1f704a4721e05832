// common.hip -- device memory through the context's allocator, and prefix sums.
#include <rocprim/device/device_scan.hpp>

#include <algorithm>
#include <cstring>

#include "hbm_device.h"
#include "hbm_internal.h"

namespace hbm {

static void *raw_alloc(Ctx &c, size_t bytes) {
    if (bytes == 0) bytes = 256;
    void *p = nullptr;
    if (c.has_alloc) {
        p = c.alloc.alloc(bytes, c.alloc.user);
        if (!p) throw Error{HBM_ENOMEM, "allocator callback returned NULL for " + std::to_string(bytes) + " bytes"};
    } else {
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            throw Error{HBM_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed"};
        }
    }
    c.mem_now += (int64_t)bytes;
    c.mem_peak = std::max(c.mem_peak, c.mem_now);
    return p;
}

static void raw_free(Ctx &c, void *p, size_t bytes) {
    if (!p) return;
    c.mem_now -= (int64_t)(bytes ? bytes : 256);
    if (c.has_alloc) {
        // the caller's allocator may recycle the block on another stream: finish our work first
        (void)hipStreamSynchronize(c.stream);
        c.alloc.release(p, c.alloc.user);
    } else {
        (void)hipStreamSynchronize(c.stream);
        (void)hipFree(p);
    }
}

void buf_free(Ctx &c, Buf &b) {
    raw_free(c, b.p, b.bytes);
    b.p = nullptr;
    b.bytes = 0;
}

void buf_alloc(Ctx &c, Buf &b, size_t bytes) {
    buf_free(c, b);
    b.p = raw_alloc(c, bytes);
    b.bytes = bytes;
}

void buf_grow(Ctx &c, Buf &b, size_t bytes, bool keep) {
    if (b.p && b.bytes >= bytes) return;
    size_t cap = b.bytes ? b.bytes : 256;
    while (cap < bytes) cap = cap < (size_t(1) << 30) ? cap * 2 : cap + (cap >> 1);
    void *np = raw_alloc(c, cap);
    if (keep && b.p && b.bytes) {
        hipError_t e = hipMemcpyAsync(np, b.p, b.bytes, hipMemcpyDeviceToDevice, c.stream);
        if (e != hipSuccess) {
            raw_free(c, np, cap);
            throw Error{HBM_EDEVICE, std::string("hipMemcpyAsync: ") + hipGetErrorString(e)};
        }
        // new tail must read as zero for buffers that are OR-ed into
        HBM_HIP(hipMemsetAsync((char *)np + b.bytes, 0, cap - b.bytes, c.stream));
    } else {
        HBM_HIP(hipMemsetAsync(np, 0, cap, c.stream));
    }
    raw_free(c, b.p, b.bytes);
    b.p = np;
    b.bytes = cap;
}

void buf_zero(Ctx &c, Buf &b, size_t off, size_t bytes) {
    if (bytes) HBM_HIP(hipMemsetAsync((char *)b.p + off, 0, bytes, c.stream));
}

// exclusive prefix sum with a 64-bit accumulator: out[i] = init + sum(in[0..i))

template <class In>
static void scan_impl(Ctx &c, const In *in, int64_t *out, int64_t count, int64_t init) {
    if (count <= 0) return;
    size_t bytes = 0;
    HBM_HIP(rocprim::exclusive_scan(nullptr, bytes, in, out, (int64_t)init, (size_t)count,
                                    rocprim::plus<int64_t>(), c.stream));
    buf_grow(c, c.scan_tmp, bytes, false);
    hipError_t e = rocprim::exclusive_scan(c.scan_tmp.p, bytes, in, out, (int64_t)init, (size_t)count,
                                           rocprim::plus<int64_t>(), c.stream);
    if (e != hipSuccess) throw Error{HBM_EDEVICE, std::string("exclusive_scan: ") + hipGetErrorString(e)};
}

void scan_u32_to_i64(Ctx &c, const uint32_t *in, int64_t *out, int64_t count, int64_t init) {
    scan_impl(c, in, out, count, init);
}
void scan_u64_to_i64(Ctx &c, const uint64_t *in, int64_t *out, int64_t count, int64_t init) {
    scan_impl(c, in, out, count, init);
}

// Descriptors are bump-allocated in a device buffer and copied from a pinned host mirror
// at the same offset, so no byte is rewritten while a queued copy or kernel may still use
// it; the space is recycled only once the stream has drained (stage_reset, or a refill).
void *stage_upload(Ctx &root, const void *host, size_t bytes) {
    const size_t need = (bytes + 255) & ~size_t(255);
    if (root.stage_pos + need > root.stage.bytes) {
        HBM_HIP(hipStreamSynchronize(root.stream));
        if (need > root.stage.bytes) {
            const size_t cap = std::max<size_t>(need, std::max<size_t>(root.stage.bytes * 2, size_t(4) << 20));
            buf_alloc(root, root.stage, cap);
            if (root.hstage) (void)hipHostFree(root.hstage);
            root.hstage = nullptr;
            HBM_HIP(hipHostMalloc(&root.hstage, cap, hipHostMallocDefault));
        }
        root.stage_pos = 0;
    }
    char *h = (char *)root.hstage + root.stage_pos;
    char *d = (char *)root.stage.p + root.stage_pos;
    std::memcpy(h, host, bytes);
    HBM_HIP(hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, root.stream));
    root.stage_pos += need;
    return d;
}

void stage_reset(Ctx &root) {
    if (root.stage_pos == 0) return;
    HBM_HIP(hipStreamSynchronize(root.stream));
    root.stage_pos = 0;
}

void stage_free(Ctx &root) {
    (void)hipStreamSynchronize(root.stream);
    buf_free(root, root.stage);
    if (root.hstage) (void)hipHostFree(root.hstage);
    root.hstage = nullptr;
    root.stage_pos = 0;
}

// ------------------------------------------------------------------ Philox throughput probe
// Each thread draws `calls` Philox4x32-10 outputs from counters of its own (two independent
// chains per iteration, so the products of one can issue under the other's xors), and the
// outputs are folded into one checksum word so no call can be dropped by the compiler.  Every
// counter word differs from lane to lane, as in the samplers (a counter word shared by the
// wave would let the compiler move part of the first round to the scalar unit).
__global__ __launch_bounds__(256) void k_philox_probe(int64_t calls, uint32_t k0, uint32_t k1, uint32_t *out) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t t1 = tid * 0x9E3779B9u, t2 = tid * 0x85EBCA6Bu, t3 = tid * 0xC2B2AE35u;
    uint32_t acc = 0;
    for (int64_t i = 0; i < calls; i += 2) {
        const uint32_t lo = (uint32_t)i, hi = (uint32_t)(i >> 32);
        // both multiplied words change with i, so no product of the first round is loop-invariant
        const uint4 a = philox10(lo ^ t1, tid, lo ^ t2, hi ^ t3, k0, k1);
        const uint4 b = philox10((lo + 1u) ^ t1, tid, (lo + 1u) ^ t2, hi ^ t3, k0, k1);
        acc += (a.x ^ a.y ^ a.z ^ a.w) + (b.x ^ b.y ^ b.z ^ b.w);
    }
    for (int o = WAVE / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane_id() == 0) atomicAdd(out, acc);
}

double philox_probe(Ctx &c, int64_t calls, int32_t blocks, uint32_t *checksum) {
    HBM_REQUIRE(calls >= 2 && calls % 2 == 0, HBM_EINVAL, "calls must be even and >= 2");
    HBM_REQUIRE(blocks >= 1, HBM_EINVAL, "blocks must be >= 1");
    buf_grow(c, c.tails, 256, false);
    uint32_t *out = c.tails.as<uint32_t>();
    buf_zero(c, c.tails, 0, 4);
    hipEvent_t e0, e1;
    HBM_HIP(hipEventCreate(&e0));
    HBM_HIP(hipEventCreate(&e1));
    HBM_HIP(hipEventRecord(e0, c.stream));
    k_philox_probe<<<(unsigned)blocks, 256, 0, c.stream>>>(calls, 0x2545F491u, 0x9E3779B9u, out);
    HBM_HIP(hipGetLastError());
    HBM_HIP(hipEventRecord(e1, c.stream));
    HBM_HIP(hipMemcpyAsync(checksum, out, 4, hipMemcpyDeviceToHost, c.stream));
    HBM_HIP(hipStreamSynchronize(c.stream));
    float ms = 0;
    HBM_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return (double)ms;
}

// ------------------------------------------------------------------ profiler
int prof_begin(Ctx &c, const char *name) {
    if (!c.prof.on) return -1;
    Prof &P = c.prof;
    int k = -1;
    for (size_t i = 0; i < P.stats.size(); i++)
        if (P.stats[i].name == name) k = (int)i;
    if (k < 0) {
        P.stats.push_back(KStat{name});
        k = (int)P.stats.size() - 1;
    }
    ProfPending e{k, nullptr, nullptr, 0, 0};
    for (hipEvent_t *ev : {&e.a, &e.b}) {
        if (!P.pool.empty()) {
            *ev = P.pool.back();
            P.pool.pop_back();
        } else {
            HBM_HIP(hipEventCreate(ev));
        }
    }
    HBM_HIP(hipEventRecord(e.a, c.stream));
    P.pending.push_back(e);
    return (int)P.pending.size() - 1;
}

void prof_end(Ctx &c, int slot, double bytes, double ops) {
    if (slot < 0) return;
    ProfPending &e = c.prof.pending[(size_t)slot];
    HBM_HIP(hipEventRecord(e.b, c.stream));
    e.bytes += bytes;
    e.ops += ops;
}

void prof_add(Ctx &c, int slot, double bytes, double ops) {
    if (slot < 0) return;
    c.prof.pending[(size_t)slot].bytes += bytes;
    c.prof.pending[(size_t)slot].ops += ops;
}

void prof_flush(Ctx &c) {
    Prof &P = c.prof;
    if (P.pending.empty()) return;
    HBM_HIP(hipEventSynchronize(P.pending.back().b));
    for (ProfPending &e : P.pending) {
        float ms = 0;
        HBM_HIP(hipEventElapsedTime(&ms, e.a, e.b));
        KStat &k = P.stats[(size_t)e.kernel];
        k.launches++;
        k.ms += ms;
        k.bytes += e.bytes;
        k.ops += e.ops;
        P.pool.push_back(e.a);
        P.pool.push_back(e.b);
    }
    P.pending.clear();
}

unsigned long long *prof_counters(Ctx &c) {
    if (!c.prof.on) return nullptr;
    if (!c.dctr.p) {
        buf_alloc(c, c.dctr, DC_COUNT * 8);
        buf_zero(c, c.dctr, 0, DC_COUNT * 8);
    }
    return c.dctr.as<unsigned long long>();
}

void prof_read_counters(Ctx &c, unsigned long long *host) {
    for (int i = 0; i < DC_COUNT; i++) host[i] = 0;
    if (!c.prof.on || !c.dctr.p) return;
    HBM_HIP(hipMemcpyAsync(host, c.dctr.p, DC_COUNT * 8, hipMemcpyDeviceToHost, c.stream));
    HBM_HIP(hipStreamSynchronize(c.stream));
    buf_zero(c, c.dctr, 0, DC_COUNT * 8);
}

}  // namespace hbm
