// hbm_internal.h -- shared internals of the gfx950 IMM library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/hbmax.h"

namespace hbm {

// ------------------------------------------------------------------ errors
struct Error {
    hbm_status st;
    std::string msg;
};

#define HBM_HIP(call)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            throw ::hbm::Error{HBM_EDEVICE, std::string(#call ": ") + hipGetErrorString(e_)}; \
    } while (0)

#define HBM_REQUIRE(cond, code, text)                           \
    do {                                                        \
        if (!(cond)) throw ::hbm::Error{code, std::string(text)}; \
    } while (0)

// ------------------------------------------------------------------ device memory
struct Ctx;

struct Buf {
    void *p = nullptr;
    size_t bytes = 0;
    template <class T>
    T *as() const { return reinterpret_cast<T *>(p); }
};

void buf_alloc(Ctx &c, Buf &b, size_t bytes);            // frees old contents
void buf_grow(Ctx &c, Buf &b, size_t bytes, bool keep);  // capacity >= bytes, optionally keeping contents
void buf_free(Ctx &c, Buf &b);
void buf_zero(Ctx &c, Buf &b, size_t off, size_t bytes);

// ------------------------------------------------------------------ graph
struct DGraph {
    int32_t n = 0;
    int64_t m = 0;
    int model = HBM_IC, prob = HBM_PROB_EDGE;
    Buf in_ptr;  // int64[n+1]
    Buf in_src;  // int32[m]
    Buf thr;     // uint32[m] (IC-EDGE, LT) or uint32[n] (IC-WC)
    Buf guide;   // uint32[2m] LT cut-point index (see graph.hip)
    Buf in_rec;  // uint32x4 per in-edge {source u, in_ptr[u], in_ptr[u+1], IC: WC threshold of u or 0; LT: thr[e]}
    bool loaded = false;
    bool borrowed = false;  // a copy of another context's graph: never freed here
};

// ------------------------------------------------------------------ store
constexpr int LUT_BITS = 11;
// Code-boundary slots of the Huffman payload: slot m holds the distance from bit m * CK_SLOT
// to the first code boundary at or after it (0..31) when that bit lies inside a code, so a
// long string can be decoded by many lanes at once, one slot interval each.
constexpr int CK_SLOT = 256;
constexpr int BIG_BITS = 2048;  // strings longer than this are decremented by a whole wave

struct Codebook {
    int32_t nsym = 0;       // coded vertices
    int32_t maxlen = 0;
    int32_t ustar_enc = -1;
    int32_t wbits = 1;      // verbatim id width
    uint64_t lim[34] = {};  // left-justified limit of codes of length <= L (index L), 33 bits
    int32_t base[34] = {};  // symbol index of a code c of length L: base[L] + c
    int32_t minlen = 0;
};

// What an encoding stores: Huffman strings; plain (cold) ids with per-set offsets; bitmap rows.
inline bool enc_huff(int e) { return e == HBM_ENC_HUFFMAN || e == HBM_ENC_HUFFMAN_HOT_BITMAP; }
inline bool enc_raw(int e) { return e == HBM_ENC_NONE || e == HBM_ENC_HOT_BITMAP; }
inline bool enc_rows(int e) { return e == HBM_ENC_HOT_BITMAP || e == HBM_ENC_HUFFMAN_HOT_BITMAP || e == HBM_ENC_BITMAX; }

struct Store {
    int enc_req = HBM_ENC_NONE;  // as requested (AUTO until the warm-up decides)
    int enc = HBM_ENC_NONE;      // in use
    double warmup_frac = 0.1, hot_frac = 0.01;
    double hot_min_density = 0.0;  // a hot vertex is in at least this fraction of warm-up sets
    bool implicit_roots = false;   // set j's root is regenerated from (seed, j), not stored
    bool containers = false;       // hot rows below warm-up density 1/16 as array containers
    bool has_seed = false;
    uint64_t seed = 0;
    int64_t nsets = 0;
    int64_t W = 0;          // warm-up sets (0 until the first request)
    int64_t wcur = 0;       // warm-up sets counted so far
    bool model_ready = false;
    int64_t members = 0;

    Buf hist;      // uint32[n] frequencies over all sets
    Buf warm;      // uint32[n] frequencies over the warm-up block
    // hot bitmap
    int32_t nhot = 0;
    Buf hot;       // int32[nhot]
    Buf hot_rank;  // int32[n], -1 if cold
    Buf bitmap;    // uint64[words * nhot]
    int64_t bm_words = 0;
    // raw (cold) ids
    Buf raw_off;   // int64[nsets+1]
    Buf raw_mem;   // int32[]: ids [0, raw_split) in device memory
    int64_t raw_count = 0;
    // spill of plain ids to pinned host memory: with spill_cap > 0 the device keeps the first
    // raw_split = floor(spill_cap / 16) * 4 ids and ids from raw_split on live in raw_host
    // (mapped, read by the kernels over the bus); spill_cap == 0 keeps every id on the device
    int64_t spill_cap = 0;
    int64_t raw_split = INT64_MAX;
    int32_t *raw_host = nullptr;    // device address of the host part
    int32_t *raw_host_h = nullptr;  // its host address
    size_t raw_host_cap = 0;        // ids
    // Huffman
    Codebook cb;
    Buf lens;      // uint8[n]
    Buf codes;     // uint32[n]
    Buf enc8;      // uint64[n]: code | length << 32 | (vertex has a row) << 40, the encoders' one read
    Buf symtab;    // int32[nsym] ids ordered by (length, id)
    Buf cbtab;     // uint64 lim[34], int64 base[34] decode tables
    Buf lut;       // uint32[2^LUT_BITS]: (symbol << 5) | length for codes of <= LUT_BITS bits, else 0
    Buf bitoff;    // int64[nsets+1]
    Buf payload;   // uint32[]
    Buf ckb;       // uint8 per CK_SLOT payload bits: code-boundary slots
    Buf mtmp;      // model building: warm-up symbol lists and their uploads
    // array containers (Roaring-style): array row a (a hot vertex of warm-up density below
    // 1/16) keeps, per chunk c of 2^16 sets, the ascending 16-bit offsets of its sets in
    // ar_low[ar_off[c (nar + 1) + a], ar_off[c (nar + 1) + a + 1]); chunks lie in order
    int32_t nar = 0;
    Buf ar_hot;    // int32[nar] array-row vertices, hot order
    Buf ar_rank;   // int32[n], -1 unless an array row
    Buf ar_off;    // int64[nchunks * (nar + 1)]
    Buf ar_low;    // uint16 entries
    int64_t ar_chunks = 0, ar_entries = 0;
    int64_t ar_last_start = 0;  // first entry of the last chunk
    Buf ar_tmp;    // rebuild scratch: per-row counts and offsets
    Buf ar_keys;   // rebuild scratch: the rebuilt chunk's entries, sorted copy
    Buf ar_sort;   // rebuild scratch: segmented-sort temporary storage
    uint64_t nbits = 0;
    int64_t escapes = 0;
    double skew = 0.0, density = 0.0;
    std::vector<uint32_t> warm_sizes;  // set sizes of the warm-up block (Eq. 2)
};

// ------------------------------------------------------------------ sampling scratch
struct Scratch {
    Buf mem;        // uint32 members of the current block
    size_t cap = 0; // entries
    Buf pos;        // uint32 per set: start in mem, or a status code
    Buf size;       // uint32 per set
    Buf ctrl;       // uint64 control words (cursor, counters, ...)
    Buf defer;      // uint32 deferred set offsets within the block
    int64_t bcap = 0;
    // big-set slots
    Buf t2_bitmap;  // uint32 words: slots * ceil(n/32)
    Buf t2_queue;   // uint32: slots * min(n, 2^20)
    int t2_slots = 0;
    Buf t2h_bitmap; // huge-set slots: bitmap + full n-entry queue each
    Buf t2h_queue;
    int t2h_slots = 0;
    Buf aux;        // uint64 per set (+1): bit lengths
    Buf cnt;        // uint32 per set (+1): plain-id counts
};

// control word indices
enum : int {
    CW_CURSOR = 0,     // next free scratch entry
    CW_NEXT = 1,       // next set (work distribution)
    CW_NDEFER = 2,     // deferred count
    CW_FIRST_OVF = 3,  // lowest block offset that ran out of scratch
    CW_NEXT2 = 4,      // tier-2 work counter
    CW_SUM = 5,        // generic accumulator
    CW_NHUGE = 6,      // sets that outgrew a big-set slot's queue
    CW_NDEFER2 = 7,    // IC sets that outgrew the LDS tier (-> device-bitmap tier)
    CW_NDEFER3 = 8,    // IC, three LDS capacities: sets that outgrew the middle one
    CW_COUNT = 9
};
constexpr uint32_t POS_DEFER = 0xFFFFFFFFu;
constexpr uint32_t POS_OVF = 0xFFFFFFFEu;

// ------------------------------------------------------------------ selection state
struct SelState {
    Buf counts;   // uint32[n]
    Buf selmask;  // uint32[ceil(n/32)]
    Buf covered;  // uint64[words]
    Buf newly;    // uint64[words]
    Buf keys;     // uint64[k]
    Buf partial;  // uint64 per argmax block + a ticket counter
    Buf cand;     // sparse counts: slot -> vertex
    Buf cpos;     // sparse counts: vertex -> slot
    Buf csel;     // sparse counts: selection bits over slots
    Buf sbcnt;    // sparse counts: per-block slot counts and their scan
    Buf sboff;
    Buf slut;     // sparse counts: decode LUT and symbol table over slots
    Buf ssym;
    int64_t words_cap = 0;
};

// ------------------------------------------------------------------ profiler
struct KStat {
    std::string name;
    int64_t launches = 0;
    double ms = 0, bytes = 0, ops = 0;
};
struct ProfPending {
    int kernel;
    hipEvent_t a, b;
    double bytes, ops;
};
struct Prof {
    bool on = false;
    std::vector<KStat> stats;
    std::vector<ProfPending> pending;
    std::vector<hipEvent_t> pool;
};

// device counters of the samplers (indices into Ctx::dctr)
enum : int { DC_PHILOX = 0, DC_EXPANDED = 1, DC_LIVE = 2, DC_EDGES = 3, DC_MEMBERS = 4, DC_PROBES = 5, DC_COUNT = 8 };

// ------------------------------------------------------------------ context
struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    hbm_allocator alloc{};
    bool has_alloc = false;
    std::string last_error;
    int64_t budget = 0;
    int num_cus = 256;
    // tuning (speed only)
    int ic_tier1 = 1;
    int64_t ic_t1_budget = 4096;
    int64_t block_sets = int64_t(1) << 21;
    int lt_lw = 32;
    int64_t t2_cap = int64_t(8) << 30;  // device bytes for big-set slots (bitmap + queue each)
    int64_t t2_queue = int64_t(1) << 20; // queue entries of a big-set slot
    int t2_per_cu = 4;                   // big-set slots (workgroups) per CU
    int lds_threads = 0;                 // threads of an LDS-tier workgroup (512 or 1024; 0 = by n)
    int lds_per_cu = 0;                  // LDS-tier workgroups launched per CU (0 = by n)
    int sparse_counts = 2;               // selection counts: 0 dense, 1 sparse slots, 2 by size
    int select_graph = 0;                // greedy launches replayed from a captured HIP graph
    int64_t spill_slots = 4096;          // LDS-tier spill slots per sampling block
    int lds_small = 2;                   // IC: a 1024-member LDS tier in front (0 no, 1 yes, 2 by n)
    hipStream_t cap_stream = nullptr;    // the stream the greedy is captured on
    // instantiated greedy graphs by launch shape (most recently used last), and the selection
    // descriptors they read: a device buffer at a fixed address with a pinned host mirror
    struct SelGraph {
        std::vector<uint64_t> shape;
        hipGraphExec_t exec = nullptr;
    };
    std::vector<SelGraph> sel_graphs;
    Buf sel_desc;
    void *sel_hdesc = nullptr;
    size_t sel_hdesc_bytes = 0;
    DGraph g;
    Store s;
    Scratch sc;
    SelState sel;
    Buf scan_tmp;  // rocPRIM temporary storage
    // batched jobs (this context drives them): control words, launch descriptors, readbacks
    Buf ctrl_arena;                        // uint64[jobs * CW_COUNT]
    std::vector<unsigned long long> ctrl_host;
    Buf stage;                             // grouped-launch descriptors (device)
    void *hstage = nullptr;                // pinned host mirror of `stage`
    size_t stage_pos = 0;                  // bump offset into both
    Buf tails;                             // uint64 per job: gathered totals
    Buf bkeys;                             // uint64 selection keys of every job
    Buf xmeta;                             // extra-large LDS pass: member records (uint4)
    // IC spill slots of one sampling launch, every job's after the previous job's: the levels a
    // set had completed when it outgrew an LDS tier (records, or ids for the device-bitmap
    // tier), for the next tier to resume; headers after the slots
    Buf spill0;                            // 1024-member tier -> 2048-member tier
    Buf spill;                             // 2048-member tier -> extra-large pass
    Buf spill2;                            // extra-large pass -> device-bitmap tier
    Buf pfind;                             // profiling: find_huff's algorithmic bytes (partial sums)
    Prof prof;
    Buf dctr;      // uint64[DC_COUNT] sampler counters (used while profiling)
    // timing of the last operations (ms)
    double t_sample = 0, t_encode = 0, t_select = 0;
    // device bytes this context holds now, and the most since creation or the last peak reset
    int64_t mem_now = 0, mem_peak = 0;
};

// ------------------------------------------------------------------ host entry points of each part
void graph_load(Ctx &c, int32_t n, int64_t m, const int64_t *row_ptr, const int32_t *dst, const float *w, int model,
                int prob);
void graph_free(Ctx &c);

void store_reset(Ctx &c);
void store_free(Ctx &c);
void store_extend(Ctx &c, int64_t theta, uint64_t seed);
void extend_stores(Ctx &root, const std::vector<Ctx *> &J, const std::vector<int64_t> &theta,
                   const std::vector<uint64_t> &seed);
// One block of progress for every job towards theta[i]: cap[i] >= 0 bounds the sets the
// job stores in this step (empty or negative: no bound).  While a job's codebook is not
// built, a block that may be stored and covers sets [0, W) builds it from those W sets
// and is stored whole; any other warm-up block counts frequencies only, up to set W.
// st[i] is EBUDGET when the job's store went over its context budget.
void extend_step(Ctx &root, const std::vector<Ctx *> &J, const std::vector<int64_t> &theta,
                 const std::vector<uint64_t> &seed, const std::vector<int64_t> &cap, std::vector<hbm_status> &st);
int64_t store_bytes(const Ctx &c);
void store_stats(Ctx &c, hbm_store_stats *out);
void store_dump(Ctx &c, int64_t j0, int64_t j1, std::vector<int64_t> &off, std::vector<int32_t> &mem);

// sample sets [j0, j1) into scratch; returns the number of sets completed (a prefix)
int64_t sample_block(Ctx &c, int64_t j0, int64_t j1, uint64_t seed);
// the same for several jobs at once (root drives the launches): job i samples
// [j0[i], j0[i] + nb[i]) with seed[i]; done[i] gets its completed prefix
void sample_blocks(Ctx &root, const std::vector<Ctx *> &J, const std::vector<int64_t> &j0,
                   const std::vector<int64_t> &nb, const std::vector<uint64_t> &seed, std::vector<int64_t> &done);
void ensure_scratch(Ctx &c, size_t entries, int64_t bcap);

// Philox throughput probe: `calls` Philox4x32-10 calls per thread over the whole chip
// (independent counters, results folded into a checksum); returns kernel milliseconds.
double philox_probe(Ctx &c, int64_t calls, int32_t blocks, uint32_t *checksum);

void select_seeds(Ctx &c, int32_t k, int32_t *seeds, uint64_t *gains, uint64_t *coverage);
// greedy selection for several jobs at once (root drives the launches)
void select_batch(Ctx &root, const std::vector<Ctx *> &C, const std::vector<int32_t> &k,
                  std::vector<std::vector<int32_t>> &seeds, std::vector<std::vector<uint64_t>> &gains,
                  std::vector<uint64_t> &coverage);
void select_free(Ctx &c);
void raw_host_free(Ctx &c);  // the pinned host part of a spilled plain-id store
// Selection with its state in a fixed per-device device array (no allocation); noalloc_setup
// takes that array's device address, once per device, with the device current.
void noalloc_setup(int device);
size_t noalloc_capacity();
void select_seeds_noalloc(Ctx &c, int32_t k, int32_t *seeds, uint64_t *gains, uint64_t *coverage);

// profiler: prof_begin records the start event of a launch (returns -1 when off),
// prof_end the stop event; prof_set fills in work that is known only later.
int prof_begin(Ctx &c, const char *name);
void prof_end(Ctx &c, int slot, double bytes = 0, double ops = 0);
void prof_add(Ctx &c, int slot, double bytes, double ops);
void prof_flush(Ctx &c);
unsigned long long *prof_counters(Ctx &c);  // device counters, or null when profiling is off
void prof_read_counters(Ctx &c, unsigned long long *host);  // and clear them

// Copy `bytes` of host data into fresh descriptor space on the device (ordered on the
// root's stream) and return its device address.  stage_reset recycles the space once the
// stream is idle; stage_free releases it.
void *stage_upload(Ctx &root, const void *host, size_t bytes);
void stage_reset(Ctx &root);
void stage_free(Ctx &root);

// Grouped launch: one job runs the plain kernel with arguments by value; several jobs run
// the grouped kernel over a descriptor array.  l1(args, blocks) / lg(GroupArgs, blocks).
template <class Args, class L1, class LG>
void glaunch(Ctx &root, const std::vector<Args> &args, const std::vector<uint32_t> &nblk, int x, L1 l1, LG lg) {
    if (args.empty()) return;
    if (args.size() == 1) {
        if (nblk[0]) l1(args[0], nblk[0]);
        return;
    }
    std::vector<uint32_t> boff(args.size() + 1, 0);
    for (size_t i = 0; i < args.size(); i++) boff[i + 1] = boff[i] + nblk[i];
    if (!boff.back()) return;
    Args *da = (Args *)stage_upload(root, args.data(), args.size() * sizeof(Args));
    uint32_t *db = (uint32_t *)stage_upload(root, boff.data(), boff.size() * 4);
    lg(da, db, (uint32_t)args.size(), boff.back(), x);
}

// launch helpers
inline unsigned grid_for(int64_t items, int per_block, int64_t cap = 1 << 20) {
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

// exclusive scan helpers (device), implemented with rocPRIM
void scan_u32_to_i64(Ctx &c, const uint32_t *in, int64_t *out, int64_t count, int64_t init);
void scan_u64_to_i64(Ctx &c, const uint64_t *in, int64_t *out, int64_t count, int64_t init);

}  // namespace hbm
