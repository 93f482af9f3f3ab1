// ara_api.hip -- host half of libara: the C ABI declared in include/ara.h.
//
// The host side validates inputs, owns device memory, builds the small
// per-call descriptors and launches the kernels of ara_kernels.hip; every
// step of the simulation itself runs on the GPU.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/ara.h"
#include "ara_internal.hpp"
#include "ara_surrogate.hpp"

static_assert(ara::kModeTable == ARA_MODE_TABLE, "the layer kernel's table variant must match ARA_MODE_TABLE");

using namespace ara;

namespace {

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

struct YetRec {
    bool live = false;
    DevBuf ev, offs;
    DevBuf sev, soff, scnt;   // mean mode: slice-major copy of the ids, its group offsets and sizes (built on first use)
    bool sliced = false;
    std::vector<int64_t> hoffs;   // host copy of the trial offsets (variable-length YETs)
    int64_t N = 0, total = 0;
    int32_t K = 0, C = 0;
};

struct EltRec {
    bool live = false;
    int32_t C = 0, n = 0;
    bool has_corr = false;
    DevBuf idx, ent, cw, mean, sol, tab;      // tab: built on the first table-mode run
    double ded = 0, lim = 0, share = 0;
};

// A layer whose tables were built once (ara_prepare_layer) and are reused.
struct PreparedRec {
    bool live = false;
    int mode = 0;
    int32_t C = 0;
    bool has_corr = false;
    DevBuf mem;
    ara::LayerDev dev;
};

// Pinned host + device slot pair used to pass per-call descriptors.
struct StageSlot {
    void* host = nullptr;
    void* dev = nullptr;
    hipEvent_t done = nullptr;
    bool pending = false;
};
constexpr size_t kStageBytes = 256 * 1024;
constexpr int kStageSlots = 8;

// Pinned host staging for bulk inputs (XELT loads): the call copies the
// caller's arrays here and returns without waiting for the device; a slot is
// reused once the copy out of it has completed.
struct BulkSlot {
    void* host = nullptr;
    size_t bytes = 0;
    hipEvent_t done = nullptr;
    bool pending = false;
};
constexpr int kBulkSlots = 4;

}  // namespace

struct ara_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    uint64_t budget = 0, used = 0;
    bool poisoned = false;
    std::string err;
    std::vector<YetRec> yets;
    std::vector<EltRec> elts;
    std::vector<PreparedRec> prepared;
    // grow-only workspaces
    DevBuf ws_tab;        // layer tables
    DevBuf ws_out;        // device staging for host outputs
    DevBuf ws_sel;        // risk-measure state
    DevBuf ws_in;         // device staging for host inputs
    DevBuf ws_mean;       // mean mode: per-slice partial sums
    double* sel_host = nullptr;
    StageSlot stage[kStageSlots];
    int next_stage = 0;
    BulkSlot bulk[kBulkSlots];
    int next_bulk = 0;
    hipEvent_t last = nullptr;
    hipStream_t last_stream = nullptr;
    bool have_last = false;
    // sampling surrogate
    bool sur_ready = false;
    bool sur_init = false;
    int64_t sur_step = 0;
    DevBuf sur_P, sur_m, sur_v, sur_grad, sur_frag, sur_mask, sur_bias, sur_loss;
    DevBuf sur_tuples, sur_gpart, sur_lpart, sur_calib;
    int32_t wpb[4] = {4, 1, 4, 1};  // trial tile (wavefronts per workgroup) per mode
    bool profiling = false;
    bool have_timing = false;
    hipEvent_t k_start = nullptr, k_stop = nullptr;
    // Freed device blocks kept for reuse: hipFree waits for the whole device,
    // so the context hands memory back to HIP only when its budget or the
    // pool cap needs it, or on ara_destroy.
    std::vector<DevBuf> pool;
    uint64_t pooled = 0;
    // device address of this GPU's copy of the allocation-free scratch array
    void* scratch_dev = nullptr;
    int32_t table_kind = ARA_TABLE_DIRECT;   // layer tables built from now on
};

// ---------------------------------------------------------------------------
// Scratch of the allocation-free risk measures (ara_risk_measures_noalloc):
// radix histograms, select state and per-block tail sums.  Each GPU the
// library runs on holds its own copy until the process ends.  Host code never
// passes the array's name to a kernel (on the host it is only a stand-in):
// ara_create looks up each device's address once, with that device current,
// and kernels receive that address.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = 64 * 1024;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxScratchDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_dev[kMaxScratchDevices];

namespace {

ara_status fail(ara_ctx* c, ara_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) {
        c->err = buf;
        if (st == ARA_E_DEVICE) c->poisoned = true;
    }
    return st;
}

#define HIPCHK(ctx, expr)                                                                     \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(ctx, ARA_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));    \
    } while (0)

// Pooled blocks are reused by later calls only.  Every call starts behind the
// previous call's last event (begin_call) or on the same stream, so a block a
// kernel may still read is never written before that kernel is done.
constexpr uint64_t kPoolCap = (uint64_t)8 << 30;

void pool_release(ara_ctx* c, size_t i)
{
    (void)hipFree(c->pool[i].p);
    c->pooled -= c->pool[i].bytes;
    c->pool.erase(c->pool.begin() + (std::ptrdiff_t)i);
}

void pool_release_largest(ara_ctx* c)
{
    size_t big = 0;
    for (size_t i = 1; i < c->pool.size(); ++i)
        if (c->pool[i].bytes > c->pool[big].bytes) big = i;
    pool_release(c, big);
}

ara_status dev_alloc(ara_ctx* c, DevBuf& b, size_t bytes)
{
    bytes = bytes == 0 ? 256 : (bytes + 255) & ~(size_t)255;
    // the smallest pooled block that fits without wasting more than a quarter of it
    size_t best = c->pool.size();
    for (size_t i = 0; i < c->pool.size(); ++i) {
        const size_t sz = c->pool[i].bytes;
        if (sz >= bytes && sz - bytes <= sz / 4 && (best == c->pool.size() || sz < c->pool[best].bytes)) best = i;
    }
    if (best < c->pool.size()) {
        b = c->pool[best];
        c->pool.erase(c->pool.begin() + (std::ptrdiff_t)best);
        c->pooled -= b.bytes;
        c->used += b.bytes;
        return ARA_OK;
    }
    while (c->budget && c->used + c->pooled + bytes > c->budget && !c->pool.empty()) pool_release_largest(c);
    if (c->budget && c->used + bytes > c->budget)
        return fail(c, ARA_E_BUDGET, "HBM budget exceeded: %llu in use + %llu requested > %llu",
                    (unsigned long long)c->used, (unsigned long long)bytes, (unsigned long long)c->budget);
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e == hipErrorOutOfMemory && !c->pool.empty()) {
        (void)hipGetLastError();
        while (!c->pool.empty()) pool_release(c, c->pool.size() - 1);
        e = hipMalloc(&b.p, bytes);
    }
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        b.p = nullptr;
        return fail(c, ARA_E_BUDGET, "device out of memory allocating %llu bytes", (unsigned long long)bytes);
    }
    if (e != hipSuccess) return fail(c, ARA_E_DEVICE, "hipMalloc: %s", hipGetErrorString(e));
    b.bytes = bytes;
    c->used += bytes;
    return ARA_OK;
}

// Return a block to the context's pool (no device synchronisation).
void dev_free(ara_ctx* c, DevBuf& b)
{
    if (b.p) {
        c->used -= b.bytes;
        c->pool.push_back(b);
        c->pooled += b.bytes;
        while (c->pooled > kPoolCap && c->pool.size() > 1) pool_release(c, 0);   // oldest first
    }
    b.p = nullptr;
    b.bytes = 0;
}

// Grow-only workspace; the old block goes back to the pool.
ara_status ws_reserve(ara_ctx* c, DevBuf& b, size_t bytes)
{
    if (b.bytes >= bytes) return ARA_OK;
    dev_free(c, b);
    return dev_alloc(c, b, bytes + bytes / 8);
}

bool is_device_ptr(const void* p)
{
    if (!p) return false;
    hipPointerAttribute_t a;
    hipError_t e = hipPointerGetAttributes(&a, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice;
}

ara_status begin_call(ara_ctx* c, hipStream_t s)
{
    if (c->poisoned) return fail(c, ARA_E_STATE, "context is unusable after a device error");
    HIPCHK(c, hipSetDevice(c->device));
    if (c->have_last && c->last_stream != s) HIPCHK(c, hipStreamWaitEvent(s, c->last, 0));
    return ARA_OK;
}

ara_status end_call(ara_ctx* c, hipStream_t s)
{
    HIPCHK(c, hipEventRecord(c->last, s));
    c->last_stream = s;
    c->have_last = true;
    return ARA_OK;
}

// Copy a small host descriptor to device memory through a pinned slot.
ara_status stage(ara_ctx* c, const void* src, size_t bytes, hipStream_t s, void** dev, StageSlot** slot_out)
{
    if (bytes > kStageBytes) return fail(c, ARA_E_INVAL, "descriptor too large (%zu bytes)", bytes);
    StageSlot& sl = c->stage[c->next_stage];
    c->next_stage = (c->next_stage + 1) % kStageSlots;
    if (sl.pending) HIPCHK(c, hipEventSynchronize(sl.done));
    std::memcpy(sl.host, src, bytes);
    HIPCHK(c, hipMemcpyAsync(sl.dev, sl.host, bytes, hipMemcpyHostToDevice, s));
    *dev = sl.dev;
    *slot_out = &sl;
    return ARA_OK;
}

ara_status release_stage(ara_ctx* c, StageSlot* sl, hipStream_t s)
{
    HIPCHK(c, hipEventRecord(sl->done, s));
    sl->pending = true;
    return ARA_OK;
}

hipStream_t pick_stream(ara_ctx*, void* s) { return (hipStream_t)s; }

bool is_finite(double x) { return std::isfinite(x); }

// The table mode's per-entry records of each XELT of a layer, built (FP64, on
// stream s) the first time a table-mode run uses the XELT and kept with it.
ara_status ensure_tabs(ara_ctx* c, int mode, const std::vector<const EltRec*>& es, hipStream_t s)
{
    if (mode != ARA_MODE_TABLE) return ARA_OK;
    for (const EltRec* ce : es) {
        EltRec& e = const_cast<EltRec&>(*ce);      // the context owns the record
        if (e.tab.p || e.n == 0) continue;
        ara_status st = dev_alloc(c, e.tab, (size_t)e.n * sizeof(TabRec));
        if (st) return st;
        HIPCHK(c, launch_elt_tab(e.n, (const EntryRec*)e.ent.p, (TabRec*)e.tab.p, s));
    }
    return ARA_OK;
}

// Validate a layer and resolve its XELT handles.
ara_status check_layer(ara_ctx* c, const YetRec& y, const ara_layer_desc* L, std::vector<const EltRec*>& out)
{
    if (!L) return fail(c, ARA_E_INVAL, "layer is NULL");
    if (L->n_elts < 1 || L->n_elts > kMaxEltsPerLayer)
        return fail(c, ARA_E_INVAL, "a layer holds 1..%d XELTs (got %d)", kMaxEltsPerLayer, L->n_elts);
    if (!L->elt_handles) return fail(c, ARA_E_INVAL, "elt_handles is NULL");
    const double t[4] = {L->occ_retention, L->occ_limit, L->agg_retention, L->agg_limit};
    for (double v : t)
        if (std::isnan(v) || v < 0) return fail(c, ARA_E_INVAL, "layer terms must be >= 0");
    if (!is_finite(L->occ_retention) || !is_finite(L->agg_retention))
        return fail(c, ARA_E_INVAL, "retentions must be finite");
    out.clear();
    for (int j = 0; j < L->n_elts; ++j) {
        const int32_t h = L->elt_handles[j];
        if (h < 0 || h >= (int32_t)c->elts.size() || !c->elts[h].live)
            return fail(c, ARA_E_STATE, "unknown XELT handle %d", h);
        const EltRec& e = c->elts[h];
        if (e.C != y.C)
            return fail(c, ARA_E_INVAL, "XELT %d has catalog %d, the YET %d", h, e.C, y.C);
        for (const EltRec* p : out)
            if (p == &e) return fail(c, ARA_E_INVAL, "XELT %d appears twice in a layer", h);
        out.push_back(&e);
    }
    return ARA_OK;
}

float to_f(double v) { return std::isinf(v) ? INFINITY : (float)v; }

struct LayerPlan {
    std::vector<EltDev> elts;
    LayerDev dev;
    size_t total = 0;
    bool has_corr = false;
};

void plan_layer(const ara_layer_desc* L, const std::vector<const EltRec*>& es, LayerPlan& p)
{
    p.elts.assign(es.size(), EltDev{});
    std::memset(&p.dev, 0, sizeof p.dev);
    p.total = 0;
    p.has_corr = false;
    for (size_t j = 0; j < es.size(); ++j) {
        const EltRec& e = *es[j];
        EltDev& d = p.elts[j];
        d.idx = (const int32_t*)e.idx.p;
        d.ent = (const EntryRec*)e.ent.p;
        d.cw = (const float2*)e.cw.p;
        d.mean = (const double*)e.mean.p;
        d.solve = (const SolveRec*)e.sol.p;
        d.tab = (const TabRec*)e.tab.p;
        d.ded = e.ded;
        d.lim = e.lim;
        d.share = e.share;
        d.n = e.n;
        p.total += (size_t)e.n;
        p.has_corr |= e.has_corr;
        p.dev.jt[j] = make_float4(to_f(e.ded), to_f(e.lim), (float)e.share, 0.0f);
    }
    p.dev.occR = to_f(L->occ_retention);
    p.dev.occL = to_f(L->occ_limit);
    p.dev.aggR = to_f(L->agg_retention);
    p.dev.aggL = to_f(L->agg_limit);
    p.dev.prog = L->program_id;
    p.dev.J = (int32_t)es.size();
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// log2 of the hashed layer table's slot count: at least twice the events the
// layer can hold (at most min(C, entries)), so probes stay short.
uint32_t hash_bits(int32_t C, const LayerPlan& p)
{
    const uint64_t keys = std::min<uint64_t>((uint64_t)C, (uint64_t)p.total);
    uint32_t b = 6;
    while ((1ull << b) < 2 * keys) ++b;
    return b;
}

// Workspace bytes for one layer's tables.
size_t table_bytes(int mode, int32_t C, const LayerPlan& p, int32_t kind)
{
    if (mode == ARA_MODE_MEAN) return align256((size_t)C * 4);
    size_t b = align256((size_t)C * 16) + 2 * align256((size_t)C * 4) + align256(scan_scratch_words(C) * 4) +
               align256(p.total * sizeof(EntryRec));
    if (kind == ARA_TABLE_HASHED) {
        const size_t slots = (size_t)1 << hash_bits(C, p);
        b += align256(slots * 32);
    }
    if (p.has_corr) b += align256(p.total * 8);
    if (mode != ARA_MODE_MEAN) b += align256(p.total * sizeof(TermThr));
    if (mode == ARA_MODE_PLAIN) b += align256(p.total * sizeof(SolveRec));
    if (mode == ARA_MODE_TABLE) b += align256(p.total * sizeof(TabRec));
    if (mode == ARA_MODE_SURROGATE) b += align256(p.total * sizeof(SurEntry));
    return b;
}

// Build one layer's tables inside ws at `base`; fills p.dev table pointers.
ara_status build_tables(ara_ctx* c, int mode, int32_t C, LayerPlan& p, char* base, const EltDev* elts_dev,
                        hipStream_t s, int32_t kind)
{
    const int32_t J = p.dev.J;
    if (mode == ARA_MODE_MEAN) {
        float* occ = (float*)base;
        HIPCHK(c, launch_mean_table(C, J, elts_dev, p.dev.occR, p.dev.occL, occ, s));
        p.dev.occ_tab = occ;
        return ARA_OK;
    }
    char* q = base;
    uint4* rows = (uint4*)q;
    q += align256((size_t)C * 16);
    uint32_t* cnt = (uint32_t*)q;
    q += align256((size_t)C * 4);
    uint32_t* off = (uint32_t*)q;
    q += align256((size_t)C * 4);
    uint32_t* scr = (uint32_t*)q;
    q += align256(scan_scratch_words(C) * 4);
    EntryRec* pent = (EntryRec*)q;
    q += align256(p.total * sizeof(EntryRec));
    float2* pcw = nullptr;
    if (p.has_corr) {
        pcw = (float2*)q;
        q += align256(p.total * 8);
    }
    SolveRec* psol = nullptr;
    if (mode == ARA_MODE_PLAIN) {
        psol = (SolveRec*)q;
        q += align256(p.total * sizeof(SolveRec));
    }
    TermThr* pthr = (TermThr*)q;           // every sampling mode
    q += align256(p.total * sizeof(TermThr));
    HIPCHK(c, launch_layer_count(C, J, elts_dev, rows, cnt, s));
    HIPCHK(c, launch_exclusive_scan(cnt, off, C, scr, s));
    TabRec* ptab = nullptr;
    if (mode == ARA_MODE_TABLE) {
        ptab = (TabRec*)q;
        q += align256(p.total * sizeof(TabRec));
    }
    HIPCHK(c, launch_layer_fill(C, J, elts_dev, off, rows, pent, pcw, psol, pthr, ptab, s));
    p.dev.rows = gptr(rows);
    p.dev.hbits = 0;
    p.dev.pent = gptr(pent);
    p.dev.pcw = gptr(pcw);
    p.dev.psol = gptr(psol);
    p.dev.pthr = gptr(pthr);
    p.dev.ptab = gptr(ptab);
    if (mode == ARA_MODE_SURROGATE) {
        SurEntry* psur = (SurEntry*)q;
        q += align256(p.total * sizeof(SurEntry));
        HIPCHK(c, launch_sur_entries(pent, (int64_t)p.total, psur, s));
        p.dev.psur = psur;
    }
    if (kind == ARA_TABLE_HASHED) {
        // the kernels read the compact table; the direct rows it was built from stay unread
        const uint32_t bits = hash_bits(C, p);
        const size_t slots = (size_t)1 << bits;
        uint4* hs = (uint4*)q;
        q += align256(slots * 32);
        HIPCHK(c, launch_layer_hash(C, rows, hs, bits, s));
        p.dev.rows = gptr(hs);
        p.dev.hbits = bits;
    }
    return ARA_OK;
}

// Mean mode reads a slice-major copy of the YET, built once per YET (left
// unbuilt, and the table read through L2, when its offsets would not fit 32
// bits).
ara_status ensure_sliced(ara_ctx* c, YetRec& y, const YetDev& yd, hipStream_t s)
{
    const int32_t ns = mean_slices(y.C);
    if (ns == 0 || y.sliced) return ARA_OK;
    y.sliced = true;
    const uint64_t ints = (uint64_t)y.total + (uint64_t)7 * ns * (uint64_t)y.N;     // ids with padding
    if (ints >= ((uint64_t)1 << 32) || y.N == 0) return ARA_OK;
    const size_t groups = (size_t)ns * (size_t)y.N;
    ara_status st;
    DevBuf scratch;
    if ((st = dev_alloc(c, y.scnt, groups * 4)) || (st = dev_alloc(c, y.soff, groups * 4)) ||
        (st = dev_alloc(c, scratch, scan_scratch_words((int64_t)groups) * 4)) ||
        (st = dev_alloc(c, y.sev, (size_t)ints * 2 + 16))) {
        dev_free(c, y.scnt);
        dev_free(c, y.soff);
        dev_free(c, scratch);
        y.sliced = false;
        return st;
    }
    HIPCHK(c, launch_yet_slice_count(yd, (uint32_t*)y.scnt.p, s));
    HIPCHK(c, launch_exclusive_scan((const uint32_t*)y.scnt.p, (uint32_t*)y.soff.p, (int64_t)groups,
                                    (uint32_t*)scratch.p, s));
    HIPCHK(c, launch_yet_slice_scatter(yd, (const uint32_t*)y.soff.p, (const uint32_t*)y.scnt.p, (uint16_t*)y.sev.p,
                                       s));
    dev_free(c, scratch);
    return ARA_OK;
}

// Layers of a batch are launched in groups whose tables together stay within
// kGroupTableBytes: a wavefront takes its trial through every layer of the
// group, and a group's solve records then stay in the caches (the 256 MB MALL,
// partly L2) while its launch runs.  One launch for 64 layers with 1 GB of
// records ran 25% slower than one launch per layer.  Results do not depend on
// the grouping (every layer of a trial is a fixed function of the trial).
constexpr uint64_t kGroupTableBytes = 24ull << 20;

ara_status launch_mode(ara_ctx* c, int mode, bool has_corr, YetRec& yr, const YetDev& yd, int64_t t0, int64_t t1,
                       const LayerDev* layers_dev, int32_t n_layers, int32_t maxJ, hipStream_t s, bool yelt = false,
                       const std::vector<uint64_t>* group_bytes = nullptr, const std::vector<bool>* group_corr = nullptr)
{
    if (mode == ARA_MODE_MEAN) {
        ara_status st = ws_reserve(c, c->ws_mean, mean_workspace_bytes(yd.C, t1 - t0));
        if (st) return st;
        if ((st = ensure_sliced(c, yr, yd, s))) return st;
    }
    if (c->profiling) HIPCHK(c, hipEventRecord(c->k_start, s));
    (void)maxJ;
    if (mode == ARA_MODE_SURROGATE)
        HIPCHK(c, launch_layers_surrogate(has_corr, yd, t0, t1, layers_dev, n_layers, (const MlpFrag*)c->sur_frag.p,
                                          (const uint32_t*)c->sur_mask.p, (const float*)c->sur_bias.p, c->wpb[mode],
                                          s));
    else if (mode == ARA_MODE_MEAN)
        HIPCHK(c, launch_mean(yd, t0, t1, layers_dev, n_layers, (const uint16_t*)yr.sev.p, (const uint32_t*)yr.soff.p,
                              (const uint32_t*)yr.scnt.p, c->ws_mean.p, yelt, s));
    else {
        for (int32_t g0 = 0; g0 < n_layers;) {
            int32_t g1 = n_layers;
            bool corr = has_corr;
            if (group_bytes) {
                uint64_t acc = (*group_bytes)[(size_t)g0];
                corr = (*group_corr)[(size_t)g0];
                for (g1 = g0 + 1; g1 < n_layers && acc + (*group_bytes)[(size_t)g1] <= kGroupTableBytes; ++g1) {
                    acc += (*group_bytes)[(size_t)g1];
                    corr = corr || (*group_corr)[(size_t)g1];
                }
            }
            HIPCHK(c, launch_layers(mode, corr, yd, t0, t1, layers_dev + g0, g1 - g0, c->wpb[mode], s));
            g0 = g1;
        }
    }
    if (c->profiling) {
        HIPCHK(c, hipEventRecord(c->k_stop, s));
        c->have_timing = true;
    }
    return ARA_OK;
}

ara_status run_impl(ara_ctx* c, int32_t yh, const ara_layer_desc* layers, int32_t n_layers, ara_mode mode,
                    uint32_t seed, int64_t t0, int64_t t1, float* const* ylt_outs, float* const* omax_outs,
                    float* const* yelt_outs, void* hip_stream, bool allow_host_out)
{
    if (!c) return ARA_E_STATE;
    if (mode != ARA_MODE_MEAN && mode != ARA_MODE_PLAIN && mode != ARA_MODE_SURROGATE && mode != ARA_MODE_TABLE)
        return fail(c, ARA_E_INVAL, "unknown mode %d", (int)mode);
    if (mode == ARA_MODE_SURROGATE && !c->sur_ready)
        return fail(c, ARA_E_STATE, "surrogate mode needs a trained or imported surrogate");
    if (yh < 0 || yh >= (int32_t)c->yets.size() || !c->yets[yh].live)
        return fail(c, ARA_E_STATE, "unknown YET handle %d", yh);
    if (n_layers < 1 || !layers || !ylt_outs) return fail(c, ARA_E_INVAL, "no layers or outputs");
    YetRec& y = c->yets[yh];
    if (t0 < 0 || t1 > y.N || t0 > t1) return fail(c, ARA_E_RANGE, "trial range [%lld, %lld) outside [0, %lld)",
                                                   (long long)t0, (long long)t1, (long long)y.N);
    hipStream_t s = pick_stream(c, hip_stream);
    ara_status st = begin_call(c, s);
    if (st) return st;

    std::vector<LayerPlan> plans((size_t)n_layers);
    std::vector<const EltRec*> es;
    std::vector<uint64_t> lbytes((size_t)n_layers);
    std::vector<bool> lcorr((size_t)n_layers);
    size_t tab_total = 0;
    bool has_corr = false;
    int32_t maxJ = 0;
    for (int32_t l = 0; l < n_layers; ++l) {
        if ((st = check_layer(c, y, &layers[l], es))) return st;
        if ((st = ensure_tabs(c, mode, es, s))) return st;
        plan_layer(&layers[l], es, plans[l]);
        lbytes[l] = table_bytes(mode, y.C, plans[l], c->table_kind);
        lcorr[l] = plans[l].has_corr;
        tab_total += lbytes[l];
        has_corr |= plans[l].has_corr;
        maxJ = std::max(maxJ, plans[l].dev.J);
    }
    const int64_t n = t1 - t0;
    // occurrences of trials [t0, t1): rows r0 .. r1 of the YET
    const int64_t r0 = y.hoffs.empty() ? t0 * (int64_t)y.K : y.hoffs[(size_t)t0];
    const int64_t r1 = y.hoffs.empty() ? t1 * (int64_t)y.K : y.hoffs[(size_t)t1];
    // host outputs go through a device staging buffer
    std::vector<bool> host_out((size_t)n_layers, false), host_om((size_t)n_layers, false),
        host_ye((size_t)n_layers, false);
    size_t out_bytes = 0;
    bool any_yelt = false;
    for (int32_t l = 0; l < n_layers; ++l) {
        if (!ylt_outs[l]) return fail(c, ARA_E_INVAL, "ylt output %d is NULL", l);
        host_out[l] = !is_device_ptr(ylt_outs[l]);
        if (omax_outs && omax_outs[l]) host_om[l] = !is_device_ptr(omax_outs[l]);
        if (yelt_outs && yelt_outs[l]) {
            host_ye[l] = !is_device_ptr(yelt_outs[l]);
            any_yelt = true;
        }
        if ((host_out[l] || host_om[l] || host_ye[l]) && !allow_host_out)
            return fail(c, ARA_E_INVAL, "batched runs need device output buffers");
        out_bytes += (host_out[l] ? align256((size_t)n * 4) : 0) + (host_om[l] ? align256((size_t)n * 4) : 0) +
                     (host_ye[l] ? align256((size_t)(r1 - r0) * 4) : 0);
    }
    if ((st = ws_reserve(c, c->ws_tab, tab_total))) return st;
    if (out_bytes && (st = ws_reserve(c, c->ws_out, out_bytes))) return st;

    // XELT descriptors of every layer, then tables, then the layer array
    std::vector<EltDev> all_elts;
    std::vector<size_t> first((size_t)n_layers);
    for (int32_t l = 0; l < n_layers; ++l) {
        first[l] = all_elts.size();
        all_elts.insert(all_elts.end(), plans[l].elts.begin(), plans[l].elts.end());
    }
    void* elts_dev = nullptr;
    StageSlot* sl1 = nullptr;
    if ((st = stage(c, all_elts.data(), all_elts.size() * sizeof(EltDev), s, &elts_dev, &sl1))) return st;
    char* tb = (char*)c->ws_tab.p;
    char* ob = (char*)c->ws_out.p;
    std::vector<LayerDev> devs((size_t)n_layers);
    for (int32_t l = 0; l < n_layers; ++l) {
        LayerPlan& p = plans[l];
        if ((st = build_tables(c, mode, y.C, p, tb, (const EltDev*)elts_dev + first[l], s, c->table_kind))) return st;
        tb += table_bytes(mode, y.C, p, c->table_kind);
        if (host_out[l]) {
            p.dev.ylt = (float*)ob;
            ob += align256((size_t)n * 4);
        } else {
            p.dev.ylt = ylt_outs[l];
        }
        if (yelt_outs && yelt_outs[l]) {
            if (host_ye[l]) {
                p.dev.yelt = (float*)ob;
                ob += align256((size_t)(r1 - r0) * 4);
            } else {
                p.dev.yelt = yelt_outs[l];
            }
            p.dev.yelt_base = r0;
        }
        if (omax_outs && omax_outs[l]) {
            if (host_om[l]) {
                p.dev.omax = (float*)ob;
                ob += align256((size_t)n * 4);
            } else {
                p.dev.omax = omax_outs[l];
            }
        }
        p.dev.seed = seed;
        devs[l] = p.dev;
    }
    void* layers_dev = nullptr;
    StageSlot* sl2 = nullptr;
    if ((st = stage(c, devs.data(), devs.size() * sizeof(LayerDev), s, &layers_dev, &sl2))) return st;
    YetDev yd{(const int32_t*)y.ev.p, (const int64_t*)y.offs.p, y.N, y.K, y.C};
    if ((st = launch_mode(c, mode, has_corr, y, yd, t0, t1, (const LayerDev*)layers_dev, n_layers, maxJ, s, any_yelt,
                          &lbytes, &lcorr)))
        return st;
    if ((st = release_stage(c, sl1, s))) return st;
    if ((st = release_stage(c, sl2, s))) return st;
    bool sync = false;
    for (int32_t l = 0; l < n_layers; ++l) {
        if (host_out[l]) {
            HIPCHK(c, hipMemcpyAsync(ylt_outs[l], devs[l].ylt, (size_t)n * 4, hipMemcpyDeviceToHost, s));
            sync = true;
        }
        if (omax_outs && omax_outs[l] && host_om[l]) {
            HIPCHK(c, hipMemcpyAsync(omax_outs[l], devs[l].omax, (size_t)n * 4, hipMemcpyDeviceToHost, s));
            sync = true;
        }
        if (yelt_outs && yelt_outs[l] && host_ye[l] && r1 > r0) {
            HIPCHK(c, hipMemcpyAsync(yelt_outs[l], devs[l].yelt, (size_t)(r1 - r0) * 4, hipMemcpyDeviceToHost, s));
            sync = true;
        }
    }
    if ((st = end_call(c, s))) return st;
    if (sync) HIPCHK(c, hipStreamSynchronize(s));
    return ARA_OK;
}


// ---- surrogate state ----
ara_status sur_alloc(ara_ctx* c)
{
    if (c->sur_init) return ARA_OK;
    ara_status st;
    const size_t pb = align256(kNumParams * 4);
    if ((st = dev_alloc(c, c->sur_P, pb)) || (st = dev_alloc(c, c->sur_m, pb)) || (st = dev_alloc(c, c->sur_v, pb)) ||
        (st = dev_alloc(c, c->sur_grad, pb)) || (st = dev_alloc(c, c->sur_frag, sizeof(MlpFrag))) ||
        (st = dev_alloc(c, c->sur_mask, kCells / 8)) || (st = dev_alloc(c, c->sur_bias, kCells * 4)) ||
        (st = dev_alloc(c, c->sur_loss, 256)))
        return st;
    HIPCHK(c, hipMemset(c->sur_m.p, 0, pb));
    HIPCHK(c, hipMemset(c->sur_v.p, 0, pb));
    HIPCHK(c, hipMemset(c->sur_mask.p, 0, kCells / 8));
    HIPCHK(c, hipMemset(c->sur_bias.p, 0, kCells * 4));
    c->sur_step = 0;
    c->sur_init = true;
    return ARA_OK;
}

uint64_t splitmix(uint64_t& x)
{
    uint64_t z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t gcd64(uint64_t a, uint64_t b)
{
    while (b) {
        const uint64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

ara_status sur_tuples_dev(ara_ctx* c, int64_t n, uint32_t seed)
{
    ara_status st;
    if ((st = ws_reserve(c, c->sur_tuples, (size_t)n * 20))) return st;
    HIPCHK(c, sur_launch_tuplegen(n, seed, (float*)c->sur_tuples.p, nullptr));
    return ARA_OK;
}

ara_status sur_step_ws(ara_ctx* c, int32_t batch)
{
    ara_status st;
    const int nw = batch / 64;
    if ((st = ws_reserve(c, c->sur_gpart, (size_t)nw * kNumParams * 4))) return st;
    if ((st = ws_reserve(c, c->sur_lpart, (size_t)nw * 4 + 256))) return st;
    return ARA_OK;
}
}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

ara_status ara_create(int device, uint64_t hbm_budget_bytes, ara_ctx** out)
{
    if (!out) return ARA_E_INVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
        (void)hipGetLastError();
        return ARA_E_DEVICE;
    }
    ara_ctx* c = new (std::nothrow) ara_ctx();
    if (!c) return ARA_E_NOMEM;
    c->device = device;
    c->budget = hbm_budget_bytes;
    c->stream = nullptr;     // loads run on the null stream and synchronise before returning
    if (hipSetDevice(device) != hipSuccess || hipEventCreateWithFlags(&c->last, hipEventDisableTiming) != hipSuccess) {
        delete c;
        return ARA_E_DEVICE;
    }
    for (auto& sl : c->stage) {
        if (hipHostMalloc(&sl.host, kStageBytes, hipHostMallocDefault) != hipSuccess ||
            hipMalloc(&sl.dev, kStageBytes) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) {
            ara_destroy(c);
            return ARA_E_DEVICE;
        }
    }
    for (auto& bs : c->bulk) {
        if (hipEventCreateWithFlags(&bs.done, hipEventDisableTiming) != hipSuccess) {
            ara_destroy(c);
            return ARA_E_DEVICE;
        }
    }
    if (hipHostMalloc((void**)&c->sel_host, 2 * kMaxRp * sizeof(double), hipHostMallocDefault) != hipSuccess ||
        hipEventCreate(&c->k_start) != hipSuccess || hipEventCreate(&c->k_stop) != hipSuccess) {
        ara_destroy(c);
        return ARA_E_DEVICE;
    }
    if (device < kMaxScratchDevices) {
        // once per device, with that device current (set above)
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_dev[device]) {
            void* p = nullptr;
            if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
                (void)hipGetLastError();
                ara_destroy(c);
                return ARA_E_DEVICE;
            }
            g_scratch_dev[device] = p;
        }
        c->scratch_dev = g_scratch_dev[device];
    }
    *out = c;
    return ARA_OK;
}

void ara_destroy(ara_ctx* c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    for (auto& y : c->yets) {
        dev_free(c, y.ev);
        dev_free(c, y.offs);
    }
    for (auto& e : c->elts) {
        dev_free(c, e.idx);
        dev_free(c, e.ent);
        dev_free(c, e.cw);
        dev_free(c, e.mean);
    }
    for (auto& pl : c->prepared) dev_free(c, pl.mem);
    for (auto& y : c->yets) {
        dev_free(c, y.sev);
        dev_free(c, y.soff);
        dev_free(c, y.scnt);
    }
    for (auto& e : c->elts) {
        dev_free(c, e.sol);
        dev_free(c, e.tab);
    }
    dev_free(c, c->ws_tab);
    dev_free(c, c->ws_out);
    dev_free(c, c->ws_sel);
    dev_free(c, c->ws_in);
    dev_free(c, c->ws_mean);
    for (DevBuf* b : {&c->sur_P, &c->sur_m, &c->sur_v, &c->sur_grad, &c->sur_frag, &c->sur_mask, &c->sur_bias, &c->sur_loss,
                      &c->sur_tuples, &c->sur_gpart, &c->sur_lpart, &c->sur_calib})
        dev_free(c, *b);
    while (!c->pool.empty()) pool_release(c, c->pool.size() - 1);
    for (auto& sl : c->stage) {
        if (sl.host) (void)hipHostFree(sl.host);
        if (sl.dev) (void)hipFree(sl.dev);
        if (sl.done) (void)hipEventDestroy(sl.done);
    }
    for (auto& bs : c->bulk) {
        if (bs.pending && bs.done) (void)hipEventSynchronize(bs.done);
        if (bs.host) (void)hipHostFree(bs.host);
        if (bs.done) (void)hipEventDestroy(bs.done);
    }
    if (c->sel_host) (void)hipHostFree(c->sel_host);
    if (c->k_start) (void)hipEventDestroy(c->k_start);
    if (c->k_stop) (void)hipEventDestroy(c->k_stop);
    if (c->last) (void)hipEventDestroy(c->last);
    delete c;
}

const char* ara_last_error(const ara_ctx* c) { return c ? c->err.c_str() : "null context"; }

uint64_t ara_bytes_in_use(const ara_ctx* c) { return c ? c->used + c->pooled : 0; }

ara_status ara_load_yet(ara_ctx* c, const int32_t* event_ids, const int64_t* trial_offsets, int64_t n_trials,
                        int32_t events_per_trial, int32_t catalog_size, int32_t* yet_handle)
{
    if (!c) return ARA_E_STATE;
    if (!yet_handle) return fail(c, ARA_E_INVAL, "yet_handle is NULL");
    if (n_trials < 0 || n_trials >= ((int64_t)1 << 32)) return fail(c, ARA_E_INVAL, "n_trials must be in [0, 2^32)");
    if (catalog_size <= 0) return fail(c, ARA_E_INVAL, "catalog_size must be positive");
    int64_t total;
    // the layer kernels index a trial's events with 24 bits
    const int64_t max_len = ((int64_t)1 << 24) - 1;
    if (trial_offsets) {
        if (trial_offsets[0] != 0) return fail(c, ARA_E_INVAL, "trial_offsets[0] must be 0");
        for (int64_t i = 0; i < n_trials; ++i) {
            if (trial_offsets[i + 1] < trial_offsets[i]) return fail(c, ARA_E_INVAL, "trial_offsets must not decrease");
            if (trial_offsets[i + 1] - trial_offsets[i] > max_len)
                return fail(c, ARA_E_INVAL, "trial %lld has more than 2^24 - 1 events", (long long)i);
        }
        total = trial_offsets[n_trials];
    } else {
        if (events_per_trial < 0 || events_per_trial > max_len)
            return fail(c, ARA_E_INVAL, "events_per_trial must be in [0, 2^24)");
        total = n_trials * (int64_t)events_per_trial;
    }
    if (total > 0 && !event_ids) return fail(c, ARA_E_INVAL, "event_ids is NULL");
    ara_status st = begin_call(c, c->stream);
    if (st) return st;
    YetRec y;
    y.N = n_trials;
    y.total = total;
    if (trial_offsets) y.hoffs.assign(trial_offsets, trial_offsets + n_trials + 1);
    y.K = trial_offsets ? 0 : events_per_trial;
    y.C = catalog_size;
    if ((st = dev_alloc(c, y.ev, (size_t)total * 4))) return st;
    if (trial_offsets) {
        if ((st = dev_alloc(c, y.offs, (size_t)(n_trials + 1) * 8))) {
            dev_free(c, y.ev);
            return st;
        }
        HIPCHK(c, hipMemcpy(y.offs.p, trial_offsets, (size_t)(n_trials + 1) * 8, hipMemcpyHostToDevice));
    }
    if (total > 0) {
        const hipMemcpyKind kind = is_device_ptr(event_ids) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
        HIPCHK(c, hipMemcpyAsync(y.ev.p, event_ids, (size_t)total * 4, kind, c->stream));
    }
    // every id must be a catalog event (checked on the device, where the ids live)
    if ((st = ws_reserve(c, c->ws_sel, 64 * 1024))) return st;
    unsigned int* bad = (unsigned int*)c->ws_sel.p;
    HIPCHK(c, hipMemsetAsync(bad, 0, sizeof(unsigned int), c->stream));
    HIPCHK(c, launch_validate_ids((const int32_t*)y.ev.p, total, catalog_size, bad, c->stream));
    unsigned int nbad = 0;
    HIPCHK(c, hipMemcpyAsync(&nbad, bad, sizeof nbad, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if ((st = end_call(c, c->stream))) return st;
    if (nbad) {
        dev_free(c, y.ev);
        dev_free(c, y.offs);
        return fail(c, ARA_E_RANGE, "%u event ids outside [0, %d)", nbad, catalog_size);
    }
    y.live = true;
    c->yets.push_back(y);
    *yet_handle = (int32_t)c->yets.size() - 1;
    return ARA_OK;
}

ara_status ara_free_yet(ara_ctx* c, int32_t h)
{
    if (!c) return ARA_E_STATE;
    if (h < 0 || h >= (int32_t)c->yets.size() || !c->yets[h].live) return fail(c, ARA_E_STATE, "unknown YET %d", h);
    dev_free(c, c->yets[h].ev);
    dev_free(c, c->yets[h].offs);
    dev_free(c, c->yets[h].sev);
    dev_free(c, c->yets[h].soff);
    dev_free(c, c->yets[h].scnt);
    c->yets[h].hoffs.clear();
    c->yets[h].hoffs.shrink_to_fit();
    c->yets[h].sliced = false;
    c->yets[h].live = false;
    return ARA_OK;
}

static ara_status validate_elt(ara_ctx* c, int32_t C, const ara_elt_desc& d, int j, std::vector<uint8_t>& seen)
{
    if (d.n_entries < 0) return fail(c, ARA_E_INVAL, "XELT %d: negative n_entries", j);
    if (d.n_entries > 0 && (!d.event_id || !d.mean || !d.sigma_i || !d.max_loss))
        return fail(c, ARA_E_INVAL, "XELT %d: NULL array", j);
    if (!(d.share >= 0.0 && d.share <= 1.0)) return fail(c, ARA_E_INVAL, "XELT %d: share outside [0,1]", j);
    if (!(d.deductible >= 0.0) || !is_finite(d.deductible)) return fail(c, ARA_E_INVAL, "XELT %d: bad deductible", j);
    if (!(d.limit > 0.0)) return fail(c, ARA_E_INVAL, "XELT %d: limit must be > 0", j);
    std::fill(seen.begin(), seen.end(), 0);
    for (int32_t r = 0; r < d.n_entries; ++r) {
        const int32_t e = d.event_id[r];
        if (e < 0 || e >= C) return fail(c, ARA_E_RANGE, "XELT %d entry %d: event %d outside [0,%d)", j, r, e, C);
        if (seen[e]) return fail(c, ARA_E_INVAL, "XELT %d: event %d appears twice", j, e);
        seen[e] = 1;
        const double mu = d.mean[r], si = d.sigma_i[r], sc = d.sigma_c ? d.sigma_c[r] : 0.0, mx = d.max_loss[r];
        if (!is_finite(mu) || !is_finite(si) || !is_finite(sc) || !is_finite(mx))
            return fail(c, ARA_E_INVAL, "XELT %d entry %d: non-finite value", j, r);
        if (!(mu > 0.0)) return fail(c, ARA_E_INVAL, "XELT %d entry %d: mean must be > 0", j, r);
        if (!(mx > mu)) return fail(c, ARA_E_INVAL, "XELT %d entry %d: max_loss must exceed the mean", j, r);
        if (si < 0.0 || sc < 0.0) return fail(c, ARA_E_INVAL, "XELT %d entry %d: negative sigma", j, r);
    }
    return ARA_OK;
}

ara_status ara_load_elts(ara_ctx* c, int32_t C, const ara_elt_desc* elts, int32_t n_elts, int32_t* handles)
{
    if (!c) return ARA_E_STATE;
    if (C <= 0 || n_elts < 0 || (n_elts > 0 && (!elts || !handles)))
        return fail(c, ARA_E_INVAL, "bad arguments to ara_load_elts");
    ara_status st;
    std::vector<uint8_t> seen((size_t)C);
    for (int j = 0; j < n_elts; ++j)
        if ((st = validate_elt(c, C, elts[j], j, seen))) return st;
    // one pinned block and one device block hold every XELT's raw inputs:
    // ids, mean, sigma_i, sigma_c, max (each array aligned to 256 bytes)
    std::vector<size_t> at((size_t)n_elts + 1, 0);
    for (int j = 0; j < n_elts; ++j) {
        const size_t n = (size_t)elts[j].n_entries;
        at[j + 1] = at[j] + align256(n * 4) + 4 * align256(n * 8);
    }
    const size_t in_bytes = at[(size_t)n_elts];
    BulkSlot& bs = c->bulk[c->next_bulk];
    c->next_bulk = (c->next_bulk + 1) % kBulkSlots;
    if (bs.pending) HIPCHK(c, hipEventSynchronize(bs.done));
    bs.pending = false;
    if (bs.bytes < in_bytes) {
        if (bs.host) HIPCHK(c, hipHostFree(bs.host));
        bs.host = nullptr;
        bs.bytes = 0;
        const size_t want = in_bytes + in_bytes / 4;
        if (hipHostMalloc(&bs.host, want, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            bs.host = nullptr;
            return fail(c, ARA_E_NOMEM, "pinned staging of %zu bytes", want);
        }
        bs.bytes = want;
    }
    for (int j = 0; j < n_elts; ++j) {
        const ara_elt_desc& d = elts[j];
        const size_t n = (size_t)d.n_entries;
        char* h = (char*)bs.host + at[j];
        std::memcpy(h, d.event_id, n * 4);
        h += align256(n * 4);
        std::memcpy(h, d.mean, n * 8);
        h += align256(n * 8);
        std::memcpy(h, d.sigma_i, n * 8);
        h += align256(n * 8);
        if (d.sigma_c) std::memcpy(h, d.sigma_c, n * 8);
        h += align256(n * 8);
        std::memcpy(h, d.max_loss, n * 8);
    }
    if ((st = begin_call(c, c->stream))) return st;
    if (in_bytes && (st = ws_reserve(c, c->ws_in, in_bytes))) return st;
    if (in_bytes) HIPCHK(c, hipMemcpyAsync(c->ws_in.p, bs.host, in_bytes, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipEventRecord(bs.done, c->stream));
    bs.pending = true;
    const size_t first = c->elts.size();
    for (int j = 0; j < n_elts; ++j) {
        const ara_elt_desc& d = elts[j];
        EltRec e;
        e.C = C;
        e.n = d.n_entries;
        e.ded = d.deductible;
        e.lim = d.limit;
        e.share = d.share;
        e.has_corr = false;
        if (d.sigma_c)
            for (int32_t r = 0; r < d.n_entries && !e.has_corr; ++r) e.has_corr = d.sigma_c[r] > 0.0;
        const size_t n = (size_t)d.n_entries;
        if ((st = dev_alloc(c, e.idx, (size_t)C * 4)) || (st = dev_alloc(c, e.ent, n * sizeof(EntryRec))) ||
            (st = dev_alloc(c, e.mean, n * 8)) || (e.has_corr && (st = dev_alloc(c, e.cw, n * 8))) ||
            (st = dev_alloc(c, e.sol, n * sizeof(SolveRec)))) {
            // a refused load changes nothing: the XELTs this call loaded go
            // too, and the next call is ordered behind the work queued for them
            dev_free(c, e.idx);
            dev_free(c, e.ent);
            dev_free(c, e.mean);
            dev_free(c, e.cw);
            dev_free(c, e.sol);
            for (size_t k = first; k < c->elts.size(); ++k) {
                EltRec& x = c->elts[k];
                dev_free(c, x.idx);
                dev_free(c, x.ent);
                dev_free(c, x.mean);
                dev_free(c, x.cw);
                dev_free(c, x.sol);
            }
            c->elts.resize(first);
            (void)end_call(c, c->stream);
            return st;
        }
        char* q = (char*)c->ws_in.p + at[j];
        const int32_t* ids = (const int32_t*)q;
        q += align256(n * 4);
        const double* mean = (const double*)q;
        q += align256(n * 8);
        const double* si = (const double*)q;
        q += align256(n * 8);
        const double* sc = (const double*)q;
        q += align256(n * 8);
        const double* mx = (const double*)q;
        HIPCHK(c, hipMemsetAsync(e.idx.p, 0xFF, (size_t)C * 4, c->stream));
        if (n) HIPCHK(c, hipMemcpyAsync(e.mean.p, mean, n * 8, hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(c, launch_elt_index(ids, d.n_entries, (int32_t*)e.idx.p, c->stream));
        HIPCHK(c, launch_elt_prepare(d.n_entries, (const double*)e.mean.p, si, d.sigma_c ? sc : nullptr, mx,
                                     (EntryRec*)e.ent.p, (float2*)e.cw.p, c->stream));
        HIPCHK(c, launch_elt_solve(d.n_entries, (const EntryRec*)e.ent.p, (SolveRec*)e.sol.p, c->stream));
        e.live = true;
        c->elts.push_back(e);
        handles[j] = (int32_t)c->elts.size() - 1;
    }
    // the device work is ordered behind this call's event; nothing waits here
    return end_call(c, c->stream);
}

ara_status ara_free_elts(ara_ctx* c, const int32_t* h, int32_t n)
{
    if (!c) return ARA_E_STATE;
    if (n < 0 || (n > 0 && !h)) return fail(c, ARA_E_INVAL, "bad arguments to ara_free_elts");
    for (int i = 0; i < n; ++i)
        if (h[i] < 0 || h[i] >= (int32_t)c->elts.size() || !c->elts[h[i]].live)
            return fail(c, ARA_E_STATE, "unknown XELT handle %d", h[i]);
    for (int i = 0; i < n; ++i) {
        EltRec& e = c->elts[h[i]];
        dev_free(c, e.idx);
        dev_free(c, e.ent);
        dev_free(c, e.sol);
        dev_free(c, e.tab);
        dev_free(c, e.cw);
        dev_free(c, e.mean);
        e.live = false;
    }
    return ARA_OK;
}

ara_status ara_run_layer(ara_ctx* c, int32_t yh, const ara_layer_desc* layer, ara_mode mode, uint32_t seed,
                         float* ylt_out, void* hip_stream)
{
    if (!c) return ARA_E_STATE;
    if (yh < 0 || yh >= (int32_t)c->yets.size() || !c->yets[yh].live) return fail(c, ARA_E_STATE, "unknown YET %d", yh);
    float* outs[1] = {ylt_out};
    return run_impl(c, yh, layer, 1, mode, seed, 0, c->yets[yh].N, outs, nullptr, nullptr, hip_stream, true);
}

ara_status ara_run_layer_ex(ara_ctx* c, int32_t yh, const ara_layer_desc* layer, ara_mode mode, uint32_t seed,
                            int64_t trial_begin, int64_t trial_end, float* ylt_out, float* max_occ_out,
                            void* hip_stream)
{
    float* outs[1] = {ylt_out};
    float* om[1] = {max_occ_out};
    return run_impl(c, yh, layer, 1, mode, seed, trial_begin, trial_end, outs, om, nullptr, hip_stream, true);
}

ara_status ara_run_layer_yelt(ara_ctx* c, int32_t yh, const ara_layer_desc* layer, ara_mode mode, uint32_t seed,
                              int64_t trial_begin, int64_t trial_end, float* ylt_out, float* max_occ_out,
                              float* yelt_out, void* hip_stream)
{
    if (!c) return ARA_E_STATE;
    if (!yelt_out) return fail(c, ARA_E_INVAL, "yelt_out is NULL");
    float* outs[1] = {ylt_out};
    float* om[1] = {max_occ_out};
    float* ye[1] = {yelt_out};
    return run_impl(c, yh, layer, 1, mode, seed, trial_begin, trial_end, outs, om, ye, hip_stream, true);
}

ara_status ara_yelt_increments(ara_ctx* c, int32_t yh, int64_t t0, int64_t t1, double agg_retention,
                               double agg_limit, const float* yelt, float* inc_out, void* hip_stream)
{
    if (!c) return ARA_E_STATE;
    if (yh < 0 || yh >= (int32_t)c->yets.size() || !c->yets[yh].live) return fail(c, ARA_E_STATE, "unknown YET %d", yh);
    YetRec& y = c->yets[yh];
    if (t0 < 0 || t1 > y.N || t0 > t1) return fail(c, ARA_E_RANGE, "trial range [%lld, %lld) outside [0, %lld)",
                                                   (long long)t0, (long long)t1, (long long)y.N);
    if (!yelt || !inc_out) return fail(c, ARA_E_INVAL, "yelt and inc_out must not be NULL");
    if (!(agg_retention >= 0.0) || !is_finite(agg_retention) || !(agg_limit >= 0.0))
        return fail(c, ARA_E_INVAL, "aggregate terms must be >= 0 (retention finite)");
    const bool din = is_device_ptr(yelt), dout = is_device_ptr(inc_out);
    if (din != dout) return fail(c, ARA_E_INVAL, "yelt and inc_out must both be device or both host memory");
    const int64_t r0 = y.hoffs.empty() ? t0 * (int64_t)y.K : y.hoffs[(size_t)t0];
    const int64_t r1 = y.hoffs.empty() ? t1 * (int64_t)y.K : y.hoffs[(size_t)t1];
    const size_t n = (size_t)(r1 - r0);
    hipStream_t s = pick_stream(c, hip_stream);
    ara_status st = begin_call(c, s);
    if (st) return st;
    const float* occ = yelt;
    float* inc = inc_out;
    if (!din) {
        if ((st = ws_reserve(c, c->ws_out, 2 * align256(n * 4)))) return st;
        float* in_dev = (float*)c->ws_out.p;
        inc = (float*)((char*)c->ws_out.p + align256(n * 4));
        if (n) HIPCHK(c, hipMemcpyAsync(in_dev, yelt, n * 4, hipMemcpyHostToDevice, s));
        occ = in_dev;
    }
    YetDev yd{(const int32_t*)y.ev.p, (const int64_t*)y.offs.p, y.N, y.K, y.C};
    HIPCHK(c, launch_yelt_increments(yd, t0, t1, r0, agg_retention, agg_limit, occ, inc, s));
    if (!din && n) HIPCHK(c, hipMemcpyAsync(inc_out, inc, n * 4, hipMemcpyDeviceToHost, s));
    if ((st = end_call(c, s))) return st;
    if (!din) HIPCHK(c, hipStreamSynchronize(s));
    return ARA_OK;
}

ara_status ara_elt_params(ara_ctx* c, int32_t h, double* alpha_out, double* beta_out)
{
    if (!c) return ARA_E_STATE;
    if (h < 0 || h >= (int32_t)c->elts.size() || !c->elts[h].live)
        return fail(c, ARA_E_STATE, "unknown XELT handle %d", h);
    if (!alpha_out || !beta_out) return fail(c, ARA_E_INVAL, "alpha_out and beta_out must not be NULL");
    const EltRec& e = c->elts[h];
    ara_status st = begin_call(c, c->stream);
    if (st) return st;
    std::vector<EntryRec> host((size_t)e.n);
    if (e.n) HIPCHK(c, hipMemcpyAsync(host.data(), e.ent.p, (size_t)e.n * sizeof(EntryRec), hipMemcpyDeviceToHost,
                                      c->stream));
    if ((st = end_call(c, c->stream))) return st;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int32_t r = 0; r < e.n; ++r) {
        alpha_out[r] = host[(size_t)r].a;     // 0 marks a degenerate entry (sigma = 0)
        beta_out[r] = host[(size_t)r].a == 0.0 ? 0.0 : host[(size_t)r].b;
    }
    return ARA_OK;
}

ara_status ara_run_layers(ara_ctx* c, int32_t yh, const ara_layer_desc* layers, int32_t n_layers, ara_mode mode,
                          uint32_t seed, float* const* ylt_outs, void* hip_stream)
{
    if (!c) return ARA_E_STATE;
    if (yh < 0 || yh >= (int32_t)c->yets.size() || !c->yets[yh].live) return fail(c, ARA_E_STATE, "unknown YET %d", yh);
    return run_impl(c, yh, layers, n_layers, mode, seed, 0, c->yets[yh].N, ylt_outs, nullptr, nullptr, hip_stream, false);
}


ara_status ara_prepare_layer(ara_ctx* c, const ara_layer_desc* layer, ara_mode mode, int32_t* handle)
{
    if (!c) return ARA_E_STATE;
    if (!handle || !layer) return fail(c, ARA_E_INVAL, "bad arguments to ara_prepare_layer");
    if (mode != ARA_MODE_MEAN && mode != ARA_MODE_PLAIN && mode != ARA_MODE_SURROGATE && mode != ARA_MODE_TABLE)
        return fail(c, ARA_E_INVAL, "unknown mode %d", (int)mode);
    if (layer->n_elts < 1 || !layer->elt_handles) return fail(c, ARA_E_INVAL, "empty layer");
    const int32_t h0 = layer->elt_handles[0];
    if (h0 < 0 || h0 >= (int32_t)c->elts.size() || !c->elts[h0].live) return fail(c, ARA_E_STATE, "unknown XELT %d", h0);
    YetRec pseudo;
    pseudo.C = c->elts[h0].C;
    std::vector<const EltRec*> es;
    ara_status st = check_layer(c, pseudo, layer, es);
    if (st) return st;
    if ((st = begin_call(c, nullptr))) return st;
    if ((st = ensure_tabs(c, mode, es, nullptr))) return st;
    PreparedRec pr;
    LayerPlan plan;
    plan_layer(layer, es, plan);
    const size_t bytes = table_bytes(mode, pseudo.C, plan, c->table_kind);
    if ((st = dev_alloc(c, pr.mem, bytes))) return st;
    void* elts_dev = nullptr;
    StageSlot* sl = nullptr;
    if ((st = stage(c, plan.elts.data(), plan.elts.size() * sizeof(EltDev), nullptr, &elts_dev, &sl))) {
        dev_free(c, pr.mem);
        return st;
    }
    if ((st = build_tables(c, mode, pseudo.C, plan, (char*)pr.mem.p, (const EltDev*)elts_dev, nullptr, c->table_kind)))
        return st;
    if ((st = release_stage(c, sl, nullptr))) return st;
    // no wait: runs that use the prepared layer are ordered behind this call
    pr.live = true;
    pr.mode = mode;
    pr.C = pseudo.C;
    pr.has_corr = plan.has_corr;
    pr.dev = plan.dev;
    c->prepared.push_back(pr);
    *handle = (int32_t)c->prepared.size() - 1;
    return end_call(c, nullptr);
}

ara_status ara_free_layer(ara_ctx* c, int32_t h)
{
    if (!c) return ARA_E_STATE;
    if (h < 0 || h >= (int32_t)c->prepared.size() || !c->prepared[h].live)
        return fail(c, ARA_E_STATE, "unknown prepared layer %d", h);
    dev_free(c, c->prepared[h].mem);
    c->prepared[h].live = false;
    return ARA_OK;
}

ara_status ara_run_prepared(ara_ctx* c, int32_t yh, const int32_t* handles, int32_t n, const uint32_t* seeds,
                            int64_t t0, int64_t t1, float* const* ylt_outs, float* const* max_occ_outs,
                            void* hip_stream)
{
    if (!c) return ARA_E_STATE;
    if (yh < 0 || yh >= (int32_t)c->yets.size() || !c->yets[yh].live) return fail(c, ARA_E_STATE, "unknown YET %d", yh);
    if (n < 1 || !handles || !seeds || !ylt_outs) return fail(c, ARA_E_INVAL, "bad arguments to ara_run_prepared");
    YetRec& y = c->yets[yh];
    if (t0 < 0 || t1 > y.N || t0 > t1) return fail(c, ARA_E_RANGE, "trial range outside the YET");
    std::vector<LayerDev> devs((size_t)n);
    std::vector<uint64_t> lbytes((size_t)n);
    std::vector<bool> lcorr((size_t)n);
    int mode = -1;
    bool has_corr = false;
    int32_t maxJ = 0;
    for (int32_t l = 0; l < n; ++l) {
        const int32_t h = handles[l];
        if (h < 0 || h >= (int32_t)c->prepared.size() || !c->prepared[h].live)
            return fail(c, ARA_E_STATE, "unknown prepared layer %d", h);
        const PreparedRec& pr = c->prepared[h];
        if (mode >= 0 && pr.mode != mode) return fail(c, ARA_E_INVAL, "prepared layers of different modes");
        mode = pr.mode;
        if (pr.C != y.C) return fail(c, ARA_E_INVAL, "prepared layer %d has catalog %d, the YET %d", h, pr.C, y.C);
        if (!ylt_outs[l] || !is_device_ptr(ylt_outs[l])) return fail(c, ARA_E_INVAL, "output %d must be device memory", l);
        devs[l] = pr.dev;
        devs[l].ylt = ylt_outs[l];
        devs[l].omax = max_occ_outs ? max_occ_outs[l] : nullptr;
        devs[l].seed = seeds[l];
        lbytes[l] = pr.mem.bytes;
        lcorr[l] = pr.has_corr;
        has_corr |= pr.has_corr;
        maxJ = std::max(maxJ, pr.dev.J);
    }
    if (mode == ARA_MODE_SURROGATE && !c->sur_ready)
        return fail(c, ARA_E_STATE, "surrogate mode needs a trained or imported surrogate");
    hipStream_t s = pick_stream(c, hip_stream);
    ara_status st = begin_call(c, s);
    if (st) return st;
    void* layers_dev = nullptr;
    StageSlot* sl = nullptr;
    if ((st = stage(c, devs.data(), devs.size() * sizeof(LayerDev), s, &layers_dev, &sl))) return st;
    YetDev yd{(const int32_t*)y.ev.p, (const int64_t*)y.offs.p, y.N, y.K, y.C};
    if ((st = launch_mode(c, mode, has_corr, y, yd, t0, t1, (const LayerDev*)layers_dev, n, maxJ, s, false, &lbytes,
                          &lcorr)))
        return st;
    if ((st = release_stage(c, sl, s))) return st;
    return end_call(c, s);
}

ara_status ara_set_trial_tile(ara_ctx* c, ara_mode mode, int32_t wpb)
{
    if (!c) return ARA_E_STATE;
    if (mode < ARA_MODE_MEAN || mode > ARA_MODE_TABLE) return fail(c, ARA_E_INVAL, "unknown mode");
    const bool ok = wpb == 1 || wpb == 2 || wpb == 4 || (wpb == 8 && mode != ARA_MODE_SURROGATE);
    if (!ok) return fail(c, ARA_E_INVAL, "trial tile %d not available for mode %d", wpb, (int)mode);
    c->wpb[mode] = wpb;
    return ARA_OK;
}

ara_status ara_set_table_kind(ara_ctx* c, int32_t kind)
{
    if (!c) return ARA_E_STATE;
    if (kind != ARA_TABLE_DIRECT && kind != ARA_TABLE_HASHED) return fail(c, ARA_E_INVAL, "unknown table kind %d", kind);
    c->table_kind = kind;
    return ARA_OK;
}

ara_status ara_autotune(ara_ctx* c, int32_t yh, const int32_t* handles, int32_t n, int64_t n_trials,
                        int32_t* best_out, float* ms_out)
{
    if (!c) return ARA_E_STATE;
    if (n < 1 || !handles) return fail(c, ARA_E_INVAL, "bad arguments to ara_autotune");
    if (yh < 0 || yh >= (int32_t)c->yets.size() || !c->yets[yh].live) return fail(c, ARA_E_STATE, "unknown YET %d", yh);
    if (handles[0] < 0 || handles[0] >= (int32_t)c->prepared.size() || !c->prepared[handles[0]].live)
        return fail(c, ARA_E_STATE, "unknown prepared layer %d", handles[0]);
    const int mode = c->prepared[handles[0]].mode;
    const int64_t nt = std::max<int64_t>(1, std::min<int64_t>(n_trials, c->yets[yh].N));
    // scratch outputs for the trial slice
    ara_status st;
    if ((st = ws_reserve(c, c->ws_out, (size_t)n * align256((size_t)nt * 4)))) return st;
    std::vector<float*> outs((size_t)n);
    for (int32_t l = 0; l < n; ++l) outs[l] = (float*)((char*)c->ws_out.p + (size_t)l * align256((size_t)nt * 4));
    std::vector<uint32_t> seeds((size_t)n, 1u);
    const int32_t cand[4] = {1, 2, 4, 8};
    const int32_t cur = c->wpb[mode];
    int32_t best = cur;
    float best_ms = 1e30f, cur_ms = 1e30f;
    const bool prof = c->profiling;
    c->profiling = true;
    for (int ci = 0; ci < 4; ++ci) {
        if (cand[ci] == 8 && mode == ARA_MODE_SURROGATE) continue;
        c->wpb[mode] = cand[ci];
        float ms = 0.0f;
        for (int rep = 0; rep < 2; ++rep) {      // first run warms up
            if ((st = ara_run_prepared(c, yh, handles, n, seeds.data(), 0, nt, outs.data(), nullptr, nullptr))) {
                c->profiling = prof;
                return st;
            }
            HIPCHK(c, hipEventSynchronize(c->k_stop));
            HIPCHK(c, hipEventElapsedTime(&ms, c->k_start, c->k_stop));
        }
        if (ms_out) ms_out[ci] = ms;
        if (cand[ci] == cur) cur_ms = ms;
        if (ms < best_ms) {
            best_ms = ms;
            best = cand[ci];
        }
    }
    c->profiling = prof;
    // a slice's timing is noisier than the full run: keep the current tile
    // unless another is clearly faster
    if (cur_ms <= 1.03f * best_ms) best = cur;
    c->wpb[mode] = best;
    if (best_out) *best_out = best;
    return ARA_OK;
}

ara_status ara_sum_ylts(ara_ctx* c, const float* const* ylts, int32_t n, int64_t n_trials, float* out,
                        void* hip_stream)
{
    if (!c) return ARA_E_STATE;
    if (n < 1 || !ylts || !out || n_trials < 0) return fail(c, ARA_E_INVAL, "bad arguments to ara_sum_ylts");
    if (n > (int32_t)(kStageBytes / sizeof(float*))) return fail(c, ARA_E_INVAL, "too many YLTs (%d)", n);
    if (!is_device_ptr(out)) return fail(c, ARA_E_INVAL, "out must be device memory");
    for (int32_t l = 0; l < n; ++l)
        if (!ylts[l] || !is_device_ptr(ylts[l])) return fail(c, ARA_E_INVAL, "YLT %d is not device memory", l);
    hipStream_t s = pick_stream(c, hip_stream);
    ara_status st = begin_call(c, s);
    if (st) return st;
    void* dev = nullptr;
    StageSlot* sl = nullptr;
    if ((st = stage(c, ylts, (size_t)n * sizeof(float*), s, &dev, &sl))) return st;
    HIPCHK(c, launch_sum_ylts((const float* const*)dev, n, n_trials, out, s));
    if ((st = release_stage(c, sl, s))) return st;
    return end_call(c, s);
}

ara_status ara_risk_measures(ara_ctx* c, const float* ylt, int64_t n, const double* rps, int32_t n_rp, double* pml,
                             double* tvar, void* hip_stream)
{
    if (!c) return ARA_E_STATE;
    if (!ylt || !rps || !pml || !tvar || n_rp < 1 || n_rp > kMaxRp || n < 1)
        return fail(c, ARA_E_INVAL, "bad arguments to ara_risk_measures");
    if (n > (int64_t)UINT32_MAX) return fail(c, ARA_E_RANGE, "n_trials above 2^32 - 1");
    uint32_t ks[kMaxRp];
    for (int r = 0; r < n_rp; ++r) {
        if (!(rps[r] > 0.0) || !is_finite(rps[r])) return fail(c, ARA_E_INVAL, "return period must be positive");
        const double k = std::floor((double)n / rps[r]);
        if (k < 1.0) return fail(c, ARA_E_RANGE, "floor(N/RP) < 1 for RP %g", rps[r]);
        if (k > 4294967295.0) return fail(c, ARA_E_RANGE, "k too large");
        ks[r] = (uint32_t)k;
    }
    hipStream_t s = pick_stream(c, hip_stream);
    ara_status st = begin_call(c, s);
    if (st) return st;
    const size_t sel_bytes = align256(kMaxRp * 256 * 4) + align256(2 * kMaxRp * 4) +
                             align256(kSelectBlocks * kMaxRp * 8) + align256(2 * kMaxRp * 8);
    const bool dev_in = is_device_ptr(ylt);
    const size_t in_bytes = dev_in ? 0 : align256((size_t)n * 4);
    if ((st = ws_reserve(c, c->ws_sel, sel_bytes + in_bytes))) return st;
    char* q = (char*)c->ws_sel.p;
    SelectWs ws;
    ws.hist = (uint32_t*)q;
    q += align256(kMaxRp * 256 * 4);
    ws.state = (uint32_t*)q;
    q += align256(2 * kMaxRp * 4);
    ws.partial = (double*)q;
    q += align256(kSelectBlocks * kMaxRp * 8);
    ws.out = (double*)q;
    q += align256(2 * kMaxRp * 8);
    const float* y = ylt;
    if (!dev_in) {
        HIPCHK(c, hipMemcpyAsync(q, ylt, (size_t)n * 4, hipMemcpyHostToDevice, s));
        y = (const float*)q;
    }
    HIPCHK(c, launch_risk_measures(y, n, ks, n_rp, ws, s));
    HIPCHK(c, hipMemcpyAsync(c->sel_host, ws.out, 2 * (size_t)n_rp * 8, hipMemcpyDeviceToHost, s));
    if ((st = end_call(c, s))) return st;
    HIPCHK(c, hipStreamSynchronize(s));
    for (int r = 0; r < n_rp; ++r) {
        pml[r] = c->sel_host[2 * r];
        tvar[r] = c->sel_host[2 * r + 1];
    }
    return ARA_OK;
}

ara_status ara_risk_measures_noalloc(ara_ctx* c, const float* ylt, int64_t n, const double* rps, int32_t n_rp,
                                     double* out, void* hip_stream)
{
    if (!c) return ARA_E_STATE;
    if (c->poisoned) return fail(c, ARA_E_STATE, "context is unusable after a device error");
    if (!ylt || !rps || !out || n < 1 || n_rp < 1)
        return fail(c, ARA_E_INVAL, "bad arguments to ara_risk_measures_noalloc");
    if (n_rp > kMaxRp)
        return fail(c, ARA_E_INVAL, "ara_risk_measures_noalloc: %d return periods, at most %d fit its scratch",
                    n_rp, kMaxRp);
    if (n > (int64_t)UINT32_MAX) return fail(c, ARA_E_RANGE, "n_trials above 2^32 - 1");
    if (!c->scratch_dev)
        return fail(c, ARA_E_STATE, "ara_risk_measures_noalloc: no scratch on device %d", c->device);
    uint32_t ks[kMaxRp];
    for (int r = 0; r < n_rp; ++r) {
        if (!(rps[r] > 0.0) || !is_finite(rps[r])) return fail(c, ARA_E_INVAL, "return period must be positive");
        const double k = std::floor((double)n / rps[r]);
        if (k < 1.0) return fail(c, ARA_E_RANGE, "floor(N/RP) < 1 for RP %g", rps[r]);
        ks[r] = (uint32_t)k;
    }
    if (!is_device_ptr(ylt) || !is_device_ptr(out))
        return fail(c, ARA_E_INVAL, "ara_risk_measures_noalloc takes device ylt and out");
    HIPCHK(c, hipSetDevice(c->device));
    char* q = (char*)c->scratch_dev;
    SelectWs ws;
    ws.hist = (uint32_t*)q;
    q += align256(kMaxRp * 256 * 4);
    ws.state = (uint32_t*)q;
    q += align256(2 * kMaxRp * 4);
    ws.partial = (double*)q;
    q += align256(kSelectBlocks * kMaxRp * 8);
    ws.out = out;
    // k_rm_init clears the histograms and the select state, so nothing a
    // previous call left in the scratch is read
    HIPCHK(c, launch_risk_measures(ylt, n, ks, n_rp, ws, (hipStream_t)hip_stream));
    return ARA_OK;
}
static_assert(((kMaxRp * 256 * 4 + 255) / 256 * 256) + ((2 * kMaxRp * 4 + 255) / 256 * 256) +
                      ((kSelectBlocks * kMaxRp * 8 + 255) / 256 * 256) <= kScratchBytes,
              "risk-measure scratch exceeds the static array");

ara_status ara_set_profiling(ara_ctx* c, int32_t enabled)
{
    if (!c) return ARA_E_STATE;
    c->profiling = enabled != 0;
    c->have_timing = false;
    return ARA_OK;
}

ara_status ara_last_kernel_ms(ara_ctx* c, double* ms)
{
    if (!c) return ARA_E_STATE;
    if (!ms) return fail(c, ARA_E_INVAL, "ms_out is NULL");
    if (!c->have_timing) return fail(c, ARA_E_STATE, "no timed launch (enable profiling first)");
    HIPCHK(c, hipEventSynchronize(c->k_stop));
    float f = 0.0f;
    HIPCHK(c, hipEventElapsedTime(&f, c->k_start, c->k_stop));
    *ms = (double)f;
    return ARA_OK;
}

ara_status ara_philox_uniforms(ara_ctx* c, const uint32_t* ctr, int64_t n, uint32_t key0, uint32_t key1, float* out,
                               void* hip_stream)
{
    if (!c) return ARA_E_STATE;
    if (n < 0 || (n > 0 && (!ctr || !out))) return fail(c, ARA_E_INVAL, "bad arguments to ara_philox_uniforms");
    if (n == 0) return ARA_OK;
    hipStream_t s = pick_stream(c, hip_stream);
    ara_status st = begin_call(c, s);
    if (st) return st;
    const bool din = is_device_ptr(ctr), dout = is_device_ptr(out);
    const size_t need = (din ? 0 : align256((size_t)n * 16)) + (dout ? 0 : align256((size_t)n * 4));
    if (need && (st = ws_reserve(c, c->ws_in, need))) return st;
    char* q = (char*)c->ws_in.p;
    const uint32_t* dc = ctr;
    float* dout_p = out;
    if (!din) {
        HIPCHK(c, hipMemcpyAsync(q, ctr, (size_t)n * 16, hipMemcpyHostToDevice, s));
        dc = (const uint32_t*)q;
        q += align256((size_t)n * 16);
    }
    if (!dout) dout_p = (float*)q;
    HIPCHK(c, launch_philox_uniforms(dc, n, key0, key1, dout_p, s));
    if (!dout) HIPCHK(c, hipMemcpyAsync(out, dout_p, (size_t)n * 4, hipMemcpyDeviceToHost, s));
    if ((st = end_call(c, s))) return st;
    if (!din || !dout) HIPCHK(c, hipStreamSynchronize(s));
    return ARA_OK;
}

ara_status ara_normal_quantile(ara_ctx* c, const double* p, int64_t n, double* x)
{
    if (!c) return ARA_E_STATE;
    if (n < 0 || (n > 0 && (!p || !x))) return fail(c, ARA_E_INVAL, "bad arguments to ara_normal_quantile");
    for (int64_t i = 0; i < n; ++i)
        if (!(p[i] > 0.0 && p[i] < 1.0)) return fail(c, ARA_E_INVAL, "p[%lld] must lie in (0,1)", (long long)i);
    if (n == 0) return ARA_OK;
    ara_status st = begin_call(c, nullptr);
    if (st) return st;
    const size_t nb = align256((size_t)n * 8);
    if ((st = ws_reserve(c, c->ws_in, 2 * nb))) return st;
    char* q = (char*)c->ws_in.p;
    HIPCHK(c, hipMemcpy(q, p, (size_t)n * 8, hipMemcpyHostToDevice));
    HIPCHK(c, launch_normal_quantile((const double*)q, n, (double*)(q + nb), nullptr));
    HIPCHK(c, hipMemcpy(x, q + nb, (size_t)n * 8, hipMemcpyDeviceToHost));
    return end_call(c, nullptr);
}

static ara_status beta_quantile_impl(ara_ctx* c, const double* a, const double* b, const double* u, int64_t n,
                                     double* x, void* hip_stream, int kind)   // 0 general, 1 layer, 2 table
{
    if (!c) return ARA_E_STATE;
    if (n < 0 || (n > 0 && (!a || !b || !u || !x))) return fail(c, ARA_E_INVAL, "bad arguments to ara_beta_quantile");
    if (n == 0) return ARA_OK;
    const bool da = is_device_ptr(a), db = is_device_ptr(b), du = is_device_ptr(u), dx = is_device_ptr(x);
    if (!da)
        for (int64_t i = 0; i < n; ++i)
            if (!(a[i] > 0.0) || !is_finite(a[i])) return fail(c, ARA_E_INVAL, "a[%lld] must be > 0", (long long)i);
    if (!db)
        for (int64_t i = 0; i < n; ++i)
            if (!(b[i] > 0.0) || !is_finite(b[i])) return fail(c, ARA_E_INVAL, "b[%lld] must be > 0", (long long)i);
    if (!du)
        for (int64_t i = 0; i < n; ++i)
            if (!(u[i] > 0.0 && u[i] < 1.0)) return fail(c, ARA_E_INVAL, "u[%lld] must lie in (0,1)", (long long)i);
    hipStream_t s = pick_stream(c, hip_stream);
    ara_status st = begin_call(c, s);
    if (st) return st;
    const size_t nb = align256((size_t)n * 8);
    const size_t need = (da ? 0 : nb) + (db ? 0 : nb) + (du ? 0 : nb) + (dx ? 0 : nb);
    if (need && (st = ws_reserve(c, c->ws_in, need))) return st;
    char* q = (char*)c->ws_in.p;
    const double* ptr[3] = {a, b, u};
    const bool dev[3] = {da, db, du};
    for (int i = 0; i < 3; ++i)
        if (!dev[i]) {
            HIPCHK(c, hipMemcpyAsync(q, ptr[i], (size_t)n * 8, hipMemcpyHostToDevice, s));
            ptr[i] = (const double*)q;
            q += nb;
        }
    double* xo = dx ? x : (double*)q;
    if (kind == 1) HIPCHK(c, launch_beta_quantile_layer(ptr[0], ptr[1], ptr[2], n, xo, s));
    else if (kind == 2) HIPCHK(c, launch_beta_quantile_table(ptr[0], ptr[1], ptr[2], n, xo, s));
    else HIPCHK(c, launch_beta_quantile(ptr[0], ptr[1], ptr[2], n, xo, s));
    if (!dx) HIPCHK(c, hipMemcpyAsync(x, xo, (size_t)n * 8, hipMemcpyDeviceToHost, s));
    if ((st = end_call(c, s))) return st;
    if (need) HIPCHK(c, hipStreamSynchronize(s));
    return ARA_OK;
}


ara_status ara_surrogate_train(ara_ctx* c, int64_t n, int32_t epochs, int32_t batch, double lr, uint32_t seed,
                               double* epoch_loss)
{
    if (!c) return ARA_E_STATE;
    if (n < batch || epochs < 0 || batch < 64 || batch % 64 || batch > 65536 || !(lr > 0.0) || n >= ((int64_t)1 << 31))
        return fail(c, ARA_E_INVAL, "bad training arguments");
    ara_status st = begin_call(c, nullptr);
    if (st) return st;
    if ((st = sur_alloc(c))) return st;
    if (c->sur_step == 0) HIPCHK(c, sur_launch_init((float*)c->sur_P.p, seed, nullptr));
    if ((st = sur_tuples_dev(c, n, seed))) return st;
    if ((st = sur_step_ws(c, batch))) return st;
    const int64_t steps_per_epoch = n / batch;
    const int64_t total = steps_per_epoch * (int64_t)epochs;
    const int64_t warm = std::max<int64_t>(1, total / 10);
    uint64_t rs = ((uint64_t)seed << 32) ^ 0xC0FFEEull;
    int64_t t = 0;
    for (int e = 0; e < epochs; ++e) {
        uint64_t pa;
        do {
            pa = splitmix(rs) % (uint64_t)n;
        } while (pa == 0 || gcd64(pa, (uint64_t)n) != 1);
        const uint64_t pc = splitmix(rs) % (uint64_t)n;
        HIPCHK(c, hipMemsetAsync(c->sur_loss.p, 0, 4, nullptr));
        for (int64_t k = 0; k < steps_per_epoch; ++k, ++t) {
            const double frac = (double)t / (double)std::max<int64_t>(1, total);
            double f = 0.5 * (1.0 + std::cos(3.14159265358979 * frac));
            if (t < warm) f *= (double)(t + 1) / (double)warm;
            ++c->sur_step;
            HIPCHK(c, sur_launch_train_step((const float*)c->sur_tuples.p, n, (int64_t)pa, (int64_t)pc, k * batch, batch,
                                            (float*)c->sur_P.p, (float*)c->sur_m.p, (float*)c->sur_v.p,
                                            (float*)c->sur_gpart.p, (float*)c->sur_lpart.p, (float*)c->sur_grad.p,
                                            (float*)c->sur_loss.p, (float)(lr * f), c->sur_step, true, nullptr));
        }
        if (epoch_loss) {
            float acc = 0.0f;
            HIPCHK(c, hipMemcpy(&acc, c->sur_loss.p, 4, hipMemcpyDeviceToHost));
            epoch_loss[e] = (double)acc / (double)(steps_per_epoch * batch);
        }
    }
    HIPCHK(c, sur_launch_build_frag((const float*)c->sur_P.p, (MlpFrag*)c->sur_frag.p, nullptr));
    // the region table described the old weights
    HIPCHK(c, hipMemset(c->sur_mask.p, 0, kCells / 8));
    HIPCHK(c, hipMemset(c->sur_bias.p, 0, kCells * 4));
    HIPCHK(c, hipDeviceSynchronize());
    c->sur_ready = true;
    return end_call(c, nullptr);
}

ara_status ara_surrogate_calibrate(ara_ctx* c, int64_t n_val, uint32_t seed, double tol, float* cell_max,
                                   float* cell_bias, int32_t* n_marked)
{
    if (!c) return ARA_E_STATE;
    if (!c->sur_init) return fail(c, ARA_E_STATE, "no surrogate to calibrate");
    if (n_val < 1 || !(tol > 0.0)) return fail(c, ARA_E_INVAL, "bad calibration arguments");
    ara_status st = begin_call(c, nullptr);
    if (st) return st;
    if ((st = sur_tuples_dev(c, n_val, seed))) return st;
    const size_t cb = (size_t)kCells * (4 + 8 + 4);
    if ((st = ws_reserve(c, c->sur_calib, cb))) return st;
    unsigned int* cnt = (unsigned int*)c->sur_calib.p;
    unsigned long long* sum = (unsigned long long*)((char*)c->sur_calib.p + kCells * 4);
    unsigned int* mx = (unsigned int*)((char*)c->sur_calib.p + kCells * 12);
    HIPCHK(c, sur_launch_build_frag((const float*)c->sur_P.p, (MlpFrag*)c->sur_frag.p, nullptr));
    std::vector<unsigned int> hc(kCells), hm(kCells);
    std::vector<long long> hs(kCells);
    std::vector<float> bias(kCells, 0.0f);
    // pass 1: each region's mean error; pass 2: the largest error left after
    // subtracting it (the bias the layer kernel applies)
    for (int pass = 0; pass < 2; ++pass) {
        HIPCHK(c, hipMemset(c->sur_calib.p, 0, cb));
        HIPCHK(c, sur_launch_calib((const float*)c->sur_tuples.p, n_val, (const MlpFrag*)c->sur_frag.p,
                                   pass ? (const float*)c->sur_bias.p : nullptr, cnt, sum, mx, nullptr));
        HIPCHK(c, hipMemcpy(hc.data(), cnt, kCells * 4, hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(hs.data(), sum, kCells * 8, hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(hm.data(), mx, kCells * 4, hipMemcpyDeviceToHost));
        if (pass == 0) {
            for (int i = 0; i < kCells; ++i) bias[i] = hc[i] ? (float)((double)hs[i] / kCalibScale / hc[i]) : 0.0f;
            HIPCHK(c, hipMemcpy(c->sur_bias.p, bias.data(), kCells * 4, hipMemcpyHostToDevice));
        }
    }
    std::vector<uint32_t> bits(kCells / 32, 0u);
    int marked = 0;
    for (int i = 0; i < kCells; ++i) {
        float m;
        std::memcpy(&m, &hm[i], 4);
        const bool bad = hc[i] < kCalibMinCount || kCalibMargin * (double)m > tol;
        if (bad) {
            bits[i >> 5] |= 1u << (i & 31);
            ++marked;
        }
        if (cell_max) cell_max[i] = hc[i] ? m : -1.0f;
        if (cell_bias) cell_bias[i] = bias[i];
    }
    HIPCHK(c, hipMemcpy(c->sur_mask.p, bits.data(), kCells / 8, hipMemcpyHostToDevice));
    if (n_marked) *n_marked = marked;
    c->sur_ready = true;
    return end_call(c, nullptr);
}

ara_status ara_surrogate_grad(ara_ctx* c, const float* tuples, int32_t n, float* grad_out, double* loss_out)
{
    if (!c) return ARA_E_STATE;
    if (!tuples || !grad_out || n < 64 || n % 64 || n > 65536) return fail(c, ARA_E_INVAL, "bad gradient arguments");
    ara_status st = begin_call(c, nullptr);
    if (st) return st;
    if ((st = sur_alloc(c))) return st;
    if (c->sur_step == 0 && !c->sur_ready) HIPCHK(c, sur_launch_init((float*)c->sur_P.p, 1u, nullptr));
    if ((st = ws_reserve(c, c->sur_tuples, (size_t)n * 20))) return st;
    if ((st = sur_step_ws(c, n))) return st;
    HIPCHK(c, hipMemcpy(c->sur_tuples.p, tuples, (size_t)n * 20, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemset(c->sur_loss.p, 0, 4));
    HIPCHK(c, sur_launch_train_step((const float*)c->sur_tuples.p, n, 1, 0, 0, n, (float*)c->sur_P.p,
                                    (float*)c->sur_m.p, (float*)c->sur_v.p, (float*)c->sur_gpart.p,
                                    (float*)c->sur_lpart.p, (float*)c->sur_grad.p, (float*)c->sur_loss.p, 0.0f, 1,
                                    false, nullptr));
    HIPCHK(c, hipMemcpy(grad_out, c->sur_grad.p, kNumParams * 4, hipMemcpyDeviceToHost));
    float acc = 0.0f;
    HIPCHK(c, hipMemcpy(&acc, c->sur_loss.p, 4, hipMemcpyDeviceToHost));
    if (loss_out) *loss_out = (double)acc / (double)n;
    return end_call(c, nullptr);
}

ara_status ara_surrogate_tuples(ara_ctx* c, int64_t n, uint32_t seed, float* out)
{
    if (!c) return ARA_E_STATE;
    if (n < 1 || !out) return fail(c, ARA_E_INVAL, "bad arguments to ara_surrogate_tuples");
    ara_status st = begin_call(c, nullptr);
    if (st) return st;
    if ((st = sur_tuples_dev(c, n, seed))) return st;
    HIPCHK(c, hipMemcpy(out, c->sur_tuples.p, (size_t)n * 20, hipMemcpyDeviceToHost));
    return end_call(c, nullptr);
}

ara_status ara_surrogate_export(ara_ctx* c, float* params, float* am, float* av, int64_t* step, uint8_t* mask,
                                float* cell_bias)
{
    if (!c) return ARA_E_STATE;
    if (!c->sur_init) return fail(c, ARA_E_STATE, "no surrogate to export");
    ara_status st = begin_call(c, nullptr);
    if (st) return st;
    HIPCHK(c, hipDeviceSynchronize());
    if (params) HIPCHK(c, hipMemcpy(params, c->sur_P.p, kNumParams * 4, hipMemcpyDeviceToHost));
    if (am) HIPCHK(c, hipMemcpy(am, c->sur_m.p, kNumParams * 4, hipMemcpyDeviceToHost));
    if (av) HIPCHK(c, hipMemcpy(av, c->sur_v.p, kNumParams * 4, hipMemcpyDeviceToHost));
    if (step) *step = c->sur_step;
    if (mask) {
        std::vector<uint32_t> bits(kCells / 32);
        HIPCHK(c, hipMemcpy(bits.data(), c->sur_mask.p, kCells / 8, hipMemcpyDeviceToHost));
        for (int i = 0; i < kCells; ++i) mask[i] = (uint8_t)((bits[i >> 5] >> (i & 31)) & 1u);
    }
    if (cell_bias) HIPCHK(c, hipMemcpy(cell_bias, c->sur_bias.p, kCells * 4, hipMemcpyDeviceToHost));
    return ARA_OK;
}

ara_status ara_surrogate_import(ara_ctx* c, const float* params, const float* am, const float* av, int64_t step,
                                const uint8_t* mask, const float* cell_bias)
{
    if (!c) return ARA_E_STATE;
    if (!params) return fail(c, ARA_E_INVAL, "params is NULL");
    for (int i = 0; i < kNumParams; ++i)
        if (!std::isfinite(params[i])) return fail(c, ARA_E_INVAL, "non-finite parameter %d", i);
    if (cell_bias)
        for (int i = 0; i < kCells; ++i)
            if (!std::isfinite(cell_bias[i]) || std::fabs(cell_bias[i]) > 1.0f)
                return fail(c, ARA_E_INVAL, "bad region bias %d", i);
    ara_status st = begin_call(c, nullptr);
    if (st) return st;
    if ((st = sur_alloc(c))) return st;
    HIPCHK(c, hipDeviceSynchronize());
    HIPCHK(c, hipMemcpy(c->sur_P.p, params, kNumParams * 4, hipMemcpyHostToDevice));
    if (am) HIPCHK(c, hipMemcpy(c->sur_m.p, am, kNumParams * 4, hipMemcpyHostToDevice));
    if (av) HIPCHK(c, hipMemcpy(c->sur_v.p, av, kNumParams * 4, hipMemcpyHostToDevice));
    c->sur_step = step > 0 ? step : 1;
    std::vector<uint32_t> bits(kCells / 32, 0u);
    if (mask)
        for (int i = 0; i < kCells; ++i)
            if (mask[i]) bits[i >> 5] |= 1u << (i & 31);
    HIPCHK(c, hipMemcpy(c->sur_mask.p, bits.data(), kCells / 8, hipMemcpyHostToDevice));
    if (cell_bias) HIPCHK(c, hipMemcpy(c->sur_bias.p, cell_bias, kCells * 4, hipMemcpyHostToDevice));
    else HIPCHK(c, hipMemset(c->sur_bias.p, 0, kCells * 4));
    HIPCHK(c, sur_launch_build_frag((const float*)c->sur_P.p, (MlpFrag*)c->sur_frag.p, nullptr));
    HIPCHK(c, hipDeviceSynchronize());
    c->sur_ready = true;
    return end_call(c, nullptr);
}

ara_status ara_surrogate_eval(ara_ctx* c, const double* a, const double* b, const double* u, int64_t n, double* x,
                              int32_t* used)
{
    if (!c) return ARA_E_STATE;
    if (!c->sur_ready) return fail(c, ARA_E_STATE, "no trained or imported surrogate");
    if (n < 1 || !a || !b || !u || !x) return fail(c, ARA_E_INVAL, "bad arguments to ara_surrogate_eval");
    for (int64_t i = 0; i < n; ++i)
        if (!(a[i] > 0.0) || !(b[i] > 0.0) || !(u[i] > 0.0 && u[i] < 1.0) || !std::isfinite(a[i]) || !std::isfinite(b[i]))
            return fail(c, ARA_E_INVAL, "bad (a, b, u) at %lld", (long long)i);
    ara_status st = begin_call(c, nullptr);
    if (st) return st;
    const size_t nb = align256((size_t)n * 8);
    if ((st = ws_reserve(c, c->ws_in, 4 * nb + align256((size_t)n * 4)))) return st;
    char* q = (char*)c->ws_in.p;
    HIPCHK(c, hipMemcpy(q, a, (size_t)n * 8, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(q + nb, b, (size_t)n * 8, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(q + 2 * nb, u, (size_t)n * 8, hipMemcpyHostToDevice));
    HIPCHK(c, sur_launch_eval((const double*)q, (const double*)(q + nb), (const double*)(q + 2 * nb), n,
                              (const MlpFrag*)c->sur_frag.p, (const uint32_t*)c->sur_mask.p,
                              (const float*)c->sur_bias.p, (double*)(q + 3 * nb),
                              (int32_t*)(q + 4 * nb), nullptr));
    HIPCHK(c, hipMemcpy(x, q + 3 * nb, (size_t)n * 8, hipMemcpyDeviceToHost));
    if (used) HIPCHK(c, hipMemcpy(used, q + 4 * nb, (size_t)n * 4, hipMemcpyDeviceToHost));
    return end_call(c, nullptr);
}

ara_status ara_beta_quantile(ara_ctx* c, const double* a, const double* b, const double* u, int64_t n, double* x,
                             void* hip_stream)
{
    return beta_quantile_impl(c, a, b, u, n, x, hip_stream, 0);
}

ara_status ara_beta_quantile_layer(ara_ctx* c, const double* a, const double* b, const double* u, int64_t n,
                                   double* x, void* hip_stream)
{
    return beta_quantile_impl(c, a, b, u, n, x, hip_stream, 1);
}

ara_status ara_beta_quantile_table(ara_ctx* c, const double* a, const double* b, const double* u, int64_t n,
                                   double* x, void* hip_stream)
{
    return beta_quantile_impl(c, a, b, u, n, x, hip_stream, 2);
}

}  // extern "C"
